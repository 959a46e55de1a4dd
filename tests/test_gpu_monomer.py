"""GPU parity of the monomer energies E_M2 (fef_monomer_energies, Eq. EM2)
against the CPU oracle (oracle/monomer.py).

Same inputs on both sides: the generated orbitals for the small cases, and
at full size each side's own SCF (the oracle's stored by
tests/golden/make_golden_monomer.py).  Bar: on identical orbitals the
kernel and the oracle differ only in the rounding order of an FP64 GEMM of
depth P_0 and the energy sum, so 1e-12 relative (1e-15 Eh floor) per
fragment; after ten SCF steps on each side the orbitals themselves differ
by up to 1e-10, so 1e-9 Eh per fragment and the sum of those bars on the
total.
"""
import os
import sys

import numpy as np
import pytest

import fefgen
from oracle import fef as ofef
from oracle import monomer as om

pytestmark = pytest.mark.gpu

REL = 1e-12
ABS = 1e-15
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _ctx(sysm):
    import paper_1708_03377_amd as lib
    return lib.Context(sysm)


def _compare(E_gpu, E_ref, what, rel=REL, abs_=ABS):
    err = np.abs(E_gpu - E_ref)
    bound = rel * np.abs(E_ref) + abs_
    worst = int(np.argmax(err - bound)) if len(err) else 0
    _say(what, "fragments", len(err), "max abs err", float(err.max()) if len(err) else 0.0)
    assert np.all(err <= bound), (what, worst, E_gpu[worst], E_ref[worst])


def test_workload0_generated_orbitals(torch):
    s = fefgen.make_system(0)
    _say("case: 8 waters, generated orbitals")
    ctx = _ctx(s)
    E, tot = ctx.monomer_energies()
    torch.cuda.synchronize()
    ref, ref_tot = om.monomer_energies(s)
    _compare(E.cpu().numpy(), ref, "8 waters")
    assert float(tot.cpu()[0]) == pytest.approx(ref_tot, rel=1e-13)
    assert int(ctx.flags.cpu()[0]) == 0


def test_ragged_shapes_and_repeatability(torch):
    # ov = 95, 12, 9, 4, 0 (nvir = 0), 0 (nocc = 0), 128 (the largest), 2,
    # 51; P = 7 (a ragged k step)
    sizes = [(24, 5), (7, 3), (10, 1), (5, 4), (4, 4), (6, 0), (24, 8), (3, 1), (20, 3)]
    s = fefgen.make_random_system(31, sizes, naux=7)
    _say("case: ragged fragments", sizes)
    ctx = _ctx(s)
    E1, t1 = ctx.monomer_energies()
    E1, t1 = E1.cpu().numpy().copy(), float(t1.cpu()[0])
    ref, ref_tot = om.monomer_energies(s)
    _compare(E1, ref, "ragged")
    assert E1[4] == 0.0 and E1[5] == 0.0
    assert t1 == pytest.approx(ref_tot, rel=1e-13)
    # bitwise repeatable; the dense B_ov and W of a split mode are the FP64
    # ones, so the energies do not depend on the mode of the half transform
    E2, t2 = ctx.monomer_energies(prec=3)
    assert np.array_equal(E2.cpu().numpy(), E1) and float(t2.cpu()[0]) == t1


def test_largest_factor_rank(torch):
    """P_0 = 80, the largest factor rank (every register k step in use),
    with the largest ov and a water-sized fragment."""
    s = fefgen.make_random_system(35, [(24, 8), (24, 5), (11, 2)], naux=80)
    _say("case: P = 80, ov = 128, 95, 18")
    ctx = _ctx(s)
    E, _ = ctx.monomer_energies()
    ref, _ = om.monomer_energies(s)
    _compare(E.cpu().numpy(), ref, "P = 80")


def test_after_scf_against_the_oracles_scf(torch):
    s = fefgen.make_random_system(32, [(24, 5), (13, 4), (24, 5), (9, 2), (24, 5)], naux=16,
                                  spacing=3.0)
    niter = 4
    _say("case: 5 fragments after", niter, "SCF steps on each side")
    ctx = _ctx(s)
    ctx.scf(niter)
    E, _ = ctx.monomer_energies()
    C, e = s.C.copy(), s.eps.copy()
    for _ in range(niter):
        C, e, _, _, _ = ofef.scf_step(s, C, e)
    ref, _ = om.monomer_energies(s, C, e)
    _compare(E.cpu().numpy(), ref, "after SCF", rel=1e-10, abs_=1e-14)


def test_correlation_energy_of_workload0(torch):
    """E_corr = E_M2 + E_D2 (Eq. EFEF2) on the generated orbitals against the
    two oracle sums."""
    s = fefgen.make_system(0)
    _say("case: 8 waters, E_M2 + E_D2")
    ctx = _ctx(s)
    em2, ed2, tot = ctx.correlation_energy()
    ref_m, ref_m_tot = om.monomer_energies(s)
    _, ref_d = ofef.pair_energies(s)
    assert em2 == pytest.approx(ref_m_tot, rel=1e-13)
    assert ed2 == pytest.approx(ref_d, rel=1e-12)
    assert tot == pytest.approx(ref_m_tot + ref_d, rel=1e-13)


def test_rejections(torch):
    import paper_1708_03377_amd as lib
    from paper_1708_03377_amd import _fef as F
    two = fefgen.make_two_class_system(33, (8, 2, 6), [(6, 2), (7, 3)], naux0=5)
    _say("case: class-1 fragment, ov above 128")
    ctx = lib.Context(two)
    with pytest.raises(lib.FefError) as ei:
        ctx.monomer_energies()
    assert ei.value.status == F.FEF_E_SHAPE
    big = fefgen.make_random_system(34, [(24, 5), (30, 7)], naux=4)
    ctx = lib.Context(big)
    with pytest.raises(lib.FefError) as ei:
        ctx.monomer_energies()
    assert ei.value.status == F.FEF_E_UNSUPPORTED


@pytest.mark.parametrize("cfg", [1, 3])
def test_full_size_against_the_oracles_scf(torch, cfg):
    s = fefgen.make_system(cfg)
    path = os.path.join(GOLDEN, f"{s.spec.name}_monomer_oracle.npz")
    if not os.path.exists(path):
        pytest.fail(f"{path} is missing: run tests/golden/make_golden_monomer.py")
    gold = dict(np.load(path, allow_pickle=False))
    _say(f"case: {s.spec.name}, {s.spec.niter} SCF steps, every fragment")
    ctx = _ctx(s)
    ctx.scf(s.spec.niter)
    E, tot = ctx.monomer_energies(prec=3)
    torch.cuda.synchronize()
    assert int(ctx.flags.cpu()[0]) == 0
    err_e = float(np.max(np.abs(ctx.eps.cpu().numpy() - gold["eps"])))
    E = E.cpu().numpy()
    tot = float(tot.cpu()[0])
    _say(f"  eps vs oracle {err_e:.2e}; E_M2 total {tot:.12f} vs {float(gold['total']):.12f}")
    assert err_e <= 1e-10
    _compare(E, gold["E_M2"], s.spec.name, rel=0.0, abs_=1e-9)
    assert abs(tot - float(gold["total"])) <= 1e-9 * s.nfrag
