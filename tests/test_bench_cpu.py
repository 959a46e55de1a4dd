"""Host-side checks of bench.py's bookkeeping (no GPU): the flop counts its
roofline uses, the multi-GPU refusal, and the traffic record lookup."""
import json
import os
import subprocess
import sys

import numpy as np


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import fefgen  # noqa: E402


def test_pair_flop_counts_config0():
    s = fefgen.make_system(0)
    # 28 water pairs, 2 ov_x ov_y P0 each
    assert bench.pair_flops(s) == 28 * 2 * 95 * 95 * 72
    # issued: whole 96-row tiles; FP64 K = 72; two terms: the three
    # products over K = 3 * 72 rounded to 224; three terms: the chains of
    # orders 0, 1, 2 over 72, 144, 216 rounded to 96, 160, 224
    assert bench.pair_issued_flops(s, "f64") == 28 * 2 * 96 * 96 * 72
    assert bench.pair_issued_flops(s, "fp16x2") == 28 * 2 * 96 * 96 * 224
    assert bench.pair_issued_flops(s, "bf16x3") == 28 * 2 * 96 * 96 * (96 + 160 + 224)
    assert bench.pair_issued_flops(s, "bf16x2") / bench.pair_flops(s) > 3.0


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_record_matches_sources():
    path = os.path.join(ROOT, "profiles", "pair_fp16x2_water4000-mixed_traffic.json")
    rec = json.load(open(path))
    got = bench.traffic_from_profiles("fp16x2", "water4000-mixed")
    if rec["sources_hash"] == bench.kernel_sources_hash():
        assert got == rec["bytes_per_launch"]
        # fetched bytes are calibrated against a plain copy of known size
        assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0
    else:
        assert got is None
    assert bench.traffic_from_profiles("fp16x2", "no-such-workload") is None


def test_scf_stage_model_config0():
    """Work model of the SCF stage rooflines on 8 water fragments (nbf 24,
    nocc 5, P 72): packed triangle 300 entries per slice."""
    s = fefgen.make_system(0)
    m = bench.scf_stage_model(s)
    tri = 24 * 25 // 2
    assert m["moments_bytes"] == 8 * (8 * 72 * tri + 8 * tri + 8 * 72)
    nn = 8 * 8 * 24 * 24
    assert m["field_bytes"] == 8 * 8 * 72 * tri + 8 * 8 * 72 + 8 * s.G.size + 2 * nn + (
        nn if s.htilde is not None else 0)
    assert m["eigh_flops"] == 8 * (9.0 * 24 ** 3 + 2.0 * 24 * 24 * 5)


def test_coupled_flops_counts_blocks_and_products():
    """Water pair (ox = oy = 5, vx = vy = 19, P0 = 72): five Kronecker-sum
    blocks and (iterations + 1) products of the four W blocks."""
    import types
    import bench
    sysm = types.SimpleNamespace(pair_x=np.array([0]), pair_y=np.array([1]),
                                 nocc=np.array([5, 5]), nbf=np.array([24, 24]),
                                 naux_class=np.array([72]))
    build = 2 * 72 * (95 * 95 + 361 ** 2 + 95 ** 2 + 95 ** 2 + 25 ** 2)
    apply = 2 * (361 ** 2 * 25 + 95 ** 2 * 95 * 2 + 25 ** 2 * 361)
    assert bench.coupled_flops(sysm, [8]) == build + 9 * apply


def test_cpu_baseline_reports_all_cores_and_one_thread():
    """The oracle sample on the default BLAS threads and again on one; both
    scaled to a full step of the workload (8 waters here, a short budget)."""
    s = fefgen.make_system(0)
    cb = bench.cpu_baseline(s, 10, 1.0)
    assert cb["kind"] == "oracle" and cb["unit"] == "pairs/s" and cb["cores"] >= 1
    assert cb["value"] > 0 and np.isfinite(cb["value"])
    assert "all 28 pairs" in cb["sample"]
    assert cb.get("value_1thread", 0) > 0 and "all 28 pairs" in cb["sample_1thread"]


def test_monomer_work_counts_the_symmetric_block():
    """Per water (ov = 95, P_0 = 72): the needed half of the symmetric
    block, 72 * 95 * 96 flops, plus 6 flops per (ia, jb); B_ov and W read
    once (2 * 72 * 95 doubles), 24 orbital energies and one result."""
    s = fefgen.make_system(0)
    flops, nbytes = bench.monomer_work(s)
    assert flops == s.nfrag * (72 * 95 * 96 + 6 * 95 * 95)
    assert nbytes == s.nfrag * 8 * (2 * 72 * 95 + 24 + 1)
