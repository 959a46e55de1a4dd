"""Benchmark: fragment-pair E2 evaluations per second on one MI355X.

One step = one whole FEF pass over a seeded synthetic liquid-like box, inputs
resident in HBM, replayed as one captured HIP graph: reset the orbitals to the
generated ones, run the effective-field SCF (niter simultaneous updates of
every fragment: density, Coulomb field, Fock diagonalisation), half-transform
every fragment, evaluate every pair energy and the deterministic total.

Every precision mode of the pair contraction is timed on the same box, each
with the tiling the native autotuner picks (untimed, before the mode's warmup).
The headline value is the fastest mode whose total energy stays within
1 micro-Hartree of the CPU oracle's own total for the workload (stored under
tests/golden/ by a script that runs only the oracle; without a stored value,
of the GPU FP64 path's total on the same step); the FP64 rate and each mode's
errors are reported beside it.

The roofline entry covers the pair contraction of the headline mode: the
algorithmic flops of one launch (2 ov_x ov_y P0 per pair, the products of the
exact method, not the three split products) divided by the launch's average
duration, timed with HIP events on the stream the library launches on.  The
flops the MFMA units actually issue (whole 96-row tiles, padded contraction
length, the three split products) are reported beside it (issued_frac).

Each mode also reports the half transform + pair energies unit on the final
orbitals on its own: 25 event-timed repetitions, the first 5 discarded,
median / min / max.

The coupled dimer doubles (W^[0] in H0, fef_coupled_pair_energies) are
timed on the same box and orbitals as a block of their own ("coupled"): one
warm call, then event-timed calls; their roofline counts the FP64 flops of
the operator blocks and of every product W p the solves took (the iteration
counts come back from the call).

Prints ONE JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 3]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X dense peaks for the arithmetic each pair mode's MFMA runs in
PEAK = {"f64": ("mfma", 78.6e12), "f32": ("mfma", 157.3e12),
        "bf16x2": ("mfma", 2.5e15), "fp16x2": ("mfma", 2.5e15), "bf16x3": ("mfma", 2.5e15)}
HBM_PEAK = 8.0e12
TOTAL_ERR_BAR = 1e-6  # Eh
METRIC = ("fragment-pair E2 evals/s at 1 GPU, mixed/surrogate vs FP64 at "
          "≤1 µEh total error")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=3, help="synthetic box id (0..4)")
    ap.add_argument("--modes", default=None,
                    help="pair modes to time (default: the workload's own set)")
    ap.add_argument("--surrogate-epochs", type=int, default=6)
    ap.add_argument("--surrogate-threshold", type=float, default=1e-8,
                    help="ensemble spread (Eh) above which a pair falls back to the exact kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-monomer", action="store_true",
                    help="skip the monomer-energy block")
    ap.add_argument("--no-coupled", action="store_true",
                    help="skip the coupled dimer-doubles block")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this size (counter calibration)")
    return ap.parse_args()


def pair_flops(sysm) -> float:
    """Algorithmic flops of one pair-energy launch: 2 ov_x ov_y P0 per pair."""
    ov = sysm.nocc.astype(np.int64) * (sysm.nbf - sysm.nocc).astype(np.int64)
    p0 = float(sysm.naux_class[0])
    return float(np.sum(2.0 * ov[sysm.pair_x] * ov[sysm.pair_y] * p0))


def pair_issued_flops(sysm, mode: str) -> float:
    """Flops the MFMA units issue for one launch: whole 96-row tiles on both
    sides and the padded contraction length (split modes: the products of
    order L over round_up((L + 1) pw, 32) contraction indices for L below the
    number of terms, pw = round_up(P0, 8))."""
    ov = sysm.nocc.astype(np.int64) * (sysm.nbf - sysm.nocc).astype(np.int64)
    ld = ((ov + 95) // 96) * 96
    p0 = int(sysm.naux_class[0])
    if mode in ("f64", "f32"):
        k = ((p0 + 3) // 4) * 4
    else:
        pw = ((p0 + 7) // 8) * 8
        if mode == "bf16x3":
            k = sum((((lv + 1) * pw + 31) // 32) * 32 for lv in range(3))
        else:
            k = ((3 * pw + 31) // 32) * 32
    return float(np.sum(2.0 * ld[sysm.pair_x] * ld[sysm.pair_y] * k))


def pair_operand_bytes(ctx, prec: int) -> int:
    """Bytes of the packed operand pool one launch reads at least once."""
    from paper_1708_03377_amd import _fef
    return _fef.fef_plan_query(ctx.plan, _fef.Q_OPS_BYTES, prec)


# Sources of the pair kernels, their work lists and their operand layout:
# the HBM traffic measured for a pair kernel stays valid while these are
# unchanged.
PAIR_KERNEL_SOURCES = ("fef_device.h", "fef_epilogue.h", "fef_internal.h", "fef_tiles.cpp",
                       "k_half.hip", "k_pair.hip", "k_split.hip")


def kernel_sources_hash() -> str:
    d = os.path.join(ROOT, "paper_1708_03377_amd", "csrc")
    h = hashlib.sha256()
    for f in PAIR_KERNEL_SOURCES:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(mode: str, workload: str):
    """HBM bytes per pair launch from the committed counter summary, or None
    when it is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"pair_{mode}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("sources_hash") != kernel_sources_hash():
        return None
    return rec.get("bytes_per_launch")


def oracle_total(name: str):
    """E_D2 of the CPU oracle's own SCF and pair energies for this workload,
    from the stored expected values (tests/golden/*_oracle.npz, written by a
    script that runs only the oracle), or None when none is stored."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}_oracle.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return float(z["total"])


def cpu_baseline(sysm, niter: int, budget_s: float):
    """The CPU oracle, untuned, on a bounded sample of the same workload:
    one SCF step over every fragment, then random pairs until the budget is
    spent; scaled to one full step (niter SCF steps + every pair)."""
    from oracle import fef as ofef
    threads = 1
    blas = "unknown"
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] or [1])
        blas = ", ".join(sorted({f"{i.get('internal_api')} {i.get('version')}" for i in info
                                 if i.get("user_api") == "blas"})) or blas
    except ImportError:
        pass
    cpu_model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                cpu_model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass

    def sample(budget):
        t0 = time.perf_counter()
        C, e, _, _, _ = ofef.scf_step(sysm, sysm.C.copy(), sysm.eps.copy())
        t_scf = time.perf_counter() - t0
        rng = np.random.default_rng(0)
        remaining = max(budget - t_scf, 2.0)
        n = min(sysm.npair, 1000)
        t_pairs, done = 0.0, 0
        while t_pairs < remaining and done < sysm.npair:
            idx = rng.choice(sysm.npair, size=n, replace=False)
            t0 = time.perf_counter()
            ofef.pair_energies(sysm, C, e, pairs=(sysm.pair_x[idx], sysm.pair_y[idx],
                                                  sysm.pair_s[idx]))
            t_pairs += time.perf_counter() - t0
            done += n
        step_s = niter * t_scf + sysm.npair * (t_pairs / done)
        text = (f"1 FP64 SCF step over all {sysm.nfrag} fragments ({t_scf:.2f} s) and "
                f"{done} random pairs ({t_pairs:.2f} s), scaled to {niter} SCF steps + "
                f"all {sysm.npair} pairs")
        return sysm.npair / step_s, text

    value, text = sample(budget_s)
    out = {"value": value, "unit": "pairs/s", "cores": int(threads),
           "kind": "oracle", "cpu_model": cpu_model, "blas": blas,
           "affinity_cpus": len(os.sched_getaffinity(0)), "sample": text}
    # the same sample on one BLAS thread (half the budget)
    try:
        import threadpoolctl
        with threadpoolctl.threadpool_limits(1):
            v1, t1 = sample(0.5 * budget_s)
        out["value_1thread"] = v1
        out["sample_1thread"] = t1
    except ImportError:
        pass
    return out


def coupled_flops(sysm, iters) -> float:
    """Algorithmic FP64 flops of the coupled solves: per pair the five
    Kronecker-sum blocks (v and the four W blocks, 2 P0 flops per element)
    and (iterations + 1) products W p (2 flops per block element per
    amplitude column)."""
    x, y = sysm.pair_x, sysm.pair_y
    ox, oy = sysm.nocc[x].astype(np.float64), sysm.nocc[y].astype(np.float64)
    vx, vy = sysm.nbf[x] - sysm.nocc[x], sysm.nbf[y] - sysm.nocc[y]
    vx, vy = vx.astype(np.float64), vy.astype(np.float64)
    P0 = float(sysm.naux_class[0])
    nV, nO, nPH, nHP = vx * vy, ox * oy, vx * oy, ox * vy
    build = 2 * P0 * (ox * vx * oy * vy + nV ** 2 + nPH ** 2 + nHP ** 2 + nO ** 2)
    apply = 2 * (nV ** 2 * nO + nPH ** 2 * nHP + nHP ** 2 * nPH + nO ** 2 * nV)
    return float(np.sum(build + (np.asarray(iters, dtype=np.float64) + 1) * apply))


def bench_coupled(ctx, sysm, torch, st, reps: int = 2):
    """The coupled pair solves (FP64 MFMA) on the current orbitals."""
    ev = lambda: torch.cuda.Event(enable_timing=True)
    _, _, it = ctx.coupled_pair_energies()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = ev(), ev()
        a.record(st)
        E, tot, it = ctx.coupled_pair_energies()
        b.record(st)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    iters = it.cpu().numpy()
    t = float(np.mean(ms))
    flops = coupled_flops(sysm, iters)
    # the one-body dressings of every fragment (uncoupled amplitudes, as the
    # pair energies take them; the coupled solve is timed above)
    ctx.dimer_dressing(maxit=0)
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record(st)
    ctx.dimer_dressing(maxit=0)
    b.record(st)
    torch.cuda.synchronize()
    dressing_ms = a.elapsed_time(b)
    ctx.flags.zero_()
    return {"ms": round(t, 3), "reps": reps, "pairs_per_s": sysm.npair / (t / 1e3),
            "E2_total": float(tot.item()), "flags": int(ctx.flags.item()),
            "iters_mean": float(iters.mean()) if len(iters) else 0.0,
            "iters_max": int(iters.max()) if len(iters) else 0,
            "dressing_ms": round(dressing_ms, 3),
            "roofline": {"kernel": "coupled pair solve (FP64 MFMA)", "bound": "mfma",
                         "achieved": flops / (t / 1e3) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                         "frac": flops / (t / 1e3) / 78.6e12, "algorithmic_flops": flops,
                         "note": "whole call (MO blocks, per-pair build and solve, total)"}}


def coupled_cpu_baseline(sysm, C, eps, npairs: int = 8):
    """The coupled oracle on a few pairs of the same box and orbitals."""
    from oracle import coupled as oc
    idx = np.random.default_rng(1).choice(sysm.npair, size=min(npairs, sysm.npair),
                                          replace=False)
    t0 = time.perf_counter()
    oc.coupled_pair_energies(sysm, C, eps, pairs=[int(k) for k in idx])
    dt = time.perf_counter() - t0
    return {"value": len(idx) / dt, "unit": "pairs/s", "kind": "oracle",
            "sample": f"{len(idx)} random pairs, CG to 1e-14 ({dt:.2f} s)"}


def monomer_work(sysm):
    """Algorithmic FP64 work of fef_monomer_energies: per fragment the
    symmetric block V = W^T B_ov = B_ov^T G_{0,0} B_ov over P_0, of which
    ov (ov + 1) / 2 elements are needed (2 P_0 flops each), and the
    exchange-weighted sum over every (ia, jb) (6 flops each); HBM bytes: B_ov
    and W read once (2 P_0 ov doubles), the fragment's orbital energies and
    one result."""
    ov = (sysm.nocc * (sysm.nbf - sysm.nocc)).astype(np.float64)
    P0 = float(sysm.naux_class[0])
    flops = float(np.sum(P0 * ov * (ov + 1) + 6 * ov ** 2))
    nbytes = float(np.sum(8 * (2 * P0 * ov + sysm.nbf + 1)))
    return flops, nbytes


def bench_monomer(ctx, sysm, torch, st, F, reps: int = 5):
    """The monomer energies E_M2 (FP64 MFMA) on the current orbitals: the
    half transform writes the dense B_ov and W once, then the monomer call
    alone is timed with events on its stream."""
    ev = lambda: torch.cuda.Event(enable_timing=True)
    E, tot = ctx.monomer_energies()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = ev(), ev()
        a.record(st)
        F.fef_monomer_energies(ctx.plan, ctx._mo_bov, ctx._mo_w, ctx.eps, ctx._mo_E,
                               ctx._mo_tot, ctx.flags, st)
        b.record(st)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    t = float(np.mean(ms))
    flops, nbytes = monomer_work(sysm)
    return {"ms": round(t, 4), "reps": reps, "fragments_per_s": sysm.nfrag / (t / 1e3),
            "E_M2_total": float(ctx._mo_tot.item()), "flags": int(ctx.flags.item()),
            "roofline": {"kernel": "monomer_energy_kernel (FP64 MFMA)", "bound": "mfma",
                         "achieved": flops / (t / 1e3) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                         "frac": flops / (t / 1e3) / 78.6e12, "algorithmic_flops": flops,
                         "algorithmic_bytes": nbytes,
                         "hbm_GBps": nbytes / (t / 1e3) / 1e9,
                         "note": "whole call (per-fragment kernel and the fixed-order total)"}}


def monomer_cpu_baseline(sysm, C, eps, nfrag: int = 200):
    """The monomer oracle on a sample of fragments of the same box."""
    from oracle import monomer as om
    idx = np.random.default_rng(2).choice(sysm.nfrag, size=min(nfrag, sysm.nfrag), replace=False)
    threads = 1
    try:
        import threadpoolctl
        threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
    except ImportError:
        pass
    t0 = time.perf_counter()
    om.monomer_energies(sysm, C, eps, frags=idx)
    dt = time.perf_counter() - t0
    return {"value": len(idx) / dt, "unit": "fragments/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(idx)} random fragments ({dt:.2f} s)"}


# pair modes timed per workload when --modes is not given
DEFAULT_MODES = {2: "f64,f32", 3: "f64,f32,bf16x2,fp16x2,bf16x3", 4: "f64,bf16x2,fp16x2,bf16x3"}


def bench_surrogate(args, sysm, ctx, lib, torch, st, niter, exact_mode):
    """The learned-surrogate pass of the 8000-water workload.  Untimed set-up:
    the ensemble is trained by the library's kernels on the exact FP64 pair
    energies of seeded 1000-water boxes at the same cutoff and density, and
    checked on a held-out box.  Timed step (eager, event-timed): orbital
    reset, niter SCF steps, fragment invariants, ensemble selection, half
    transform and the exact kernel of mode ``exact_mode`` on every pair the
    ensemble declines (all pairs below 6 A, every pair whose members disagree
    by more than the threshold)."""
    import fefgen
    from paper_1708_03377_amd import surrogate as sg
    ev = lambda: torch.cuda.Event(enable_timing=True)
    r6 = sg.R_EXACT_ANGSTROM * fefgen.BOHR_PER_ANGSTROM
    t0 = time.perf_counter()
    X, T = sg.training_set(sg.TRAIN_SEEDS)
    ens, hist = sg.train_ensemble(X, T, epochs=args.surrogate_epochs)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    ntrain = int(X.shape[0])
    del X, T
    # held-out box: error of the ensemble mean and spread of the members, in Eh
    hctx = lib.Context(fefgen.surrogate_training_box(sg.HELDOUT_SEED))
    Xh, Th, _ = sg.pair_dataset(hctx, r6, niter)
    Y = ens.forward(Xh).cpu().numpy().astype(np.float64)
    stt = ens.stats.cpu().numpy().astype(np.float64)
    R2 = Xh[:, 0].cpu().numpy().astype(np.float64) ** 2
    pred = (Y * stt[35] + stt[34]) / R2
    truth = Th.cpu().numpy().astype(np.float64) / R2
    spread = pred.max(0) - pred.min(0)
    held = {"pairs": int(len(truth)), "rmse_Eh": float(np.sqrt(np.mean((pred.mean(0) - truth) ** 2))),
            "median_spread_Eh": float(np.median(spread)),
            "frac_spread_below_threshold": float(np.mean(spread <= args.surrogate_threshold))}
    del hctx, Xh, Th
    prec = lib.PREC[exact_mode]
    thr = args.surrogate_threshold

    def step():
        ctx.reset_orbitals()
        ctx.scf(niter)
        U = ctx.invariants()
        return ctx.surrogate_energies(ens, U, r6, thr, prec)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ge = [(ev(), ev()) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ge:
        a.record(st)
        step()
        b.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sel = ctx._select[:ctx.npair].cpu().numpy()
    # the masked exact kernel alone, on the same selection
    pe = [(ev(), ev()) for _ in range(args.steps)]
    for a, b in pe:
        a.record(st)
        ctx.pair_energies_masked(prec, ctx._select)
        b.record(st)
    torch.cuda.synchronize()
    return {"ms_per_step": 1e3 * wall / args.steps,
            "gpu_ms_per_step": float(np.mean([a.elapsed_time(b) for a, b in ge])),
            "stage_ms": [float("nan")] * 3,
            "pair_ms": float(np.mean([a.elapsed_time(b) for a, b in pe])),
            "tiles": lib.fef_plan_get_tiles(ctx.plan, prec), "unit_ms": [float("nan")],
            "E_total": float(ctx.E2_total.cpu()[0]), "flags": int(ctx.flags.cpu()[0]),
            "E2": ctx.E2_pair[:ctx.npair].cpu().numpy().copy(),
            "surrogate": {"threshold_Eh": thr, "exact_below_A": sg.R_EXACT_ANGSTROM,
                          "predicted_fraction": float(np.mean(sel == 0)),
                          "exact_fraction": float(np.mean(sel != 0)),
                          "training_pairs": ntrain, "training_boxes": list(sg.TRAIN_SEEDS),
                          "epochs": args.surrogate_epochs, "train_s": round(train_s, 2),
                          "final_loss": hist[-1] if hist else None,
                          "heldout_box": sg.HELDOUT_SEED, "heldout": held,
                          "exact_kernel": exact_mode}}


HBM_PEAK = 8.0e12      # bytes/s
FP64_PEAK = 78.6e12    # FP64 vector FLOP/s


def scf_stage_model(sysm):
    """Algorithmic work of one packed SCF step (no re-reads counted):
    moments read the packed coefficients Bp [P][nbf (nbf + 1) / 2] and the
    weighted densities and write d [P]; the field and Coulomb build read Bp
    again, every d, G, F0 (and h~) and write F~ [nbf^2]; the eigensolver is
    counted as 9 n^3 FLOP per matrix (the conventional count of a dense
    symmetric eigendecomposition with eigenvectors) plus 2 n^2 nocc for the
    new density."""
    n = sysm.nbf.astype(np.int64)
    P = sysm.naux.astype(np.int64)
    tri = n * (n + 1) // 2
    bp = 8 * int(np.sum(P * tri))
    d = 8 * int(np.sum(P))
    nn = 8 * int(np.sum(n * n))
    g = 8 * int(sysm.G.size)
    ht = nn if sysm.htilde is not None else 0
    return {"moments_bytes": bp + 8 * int(np.sum(tri)) + d,
            "field_bytes": bp + d + g + nn + ht + nn,
            "eigh_flops": float(np.sum(9.0 * n ** 3 + 2.0 * n * n * sysm.nocc))}


def bench_scf_stages(ctx, lib, sysm, reps: int = 10):
    """Event-timed stages of eager packed SCF steps (the library records
    events at the stage boundaries): mean over `reps` steps after one
    untimed step, each stage against its roofline."""
    from paper_1708_03377_amd import _fef
    ctx.reset_orbitals()
    ctx.scf_step_packed()
    _fef.fef_plan_stage_timing(ctx.plan, True)
    rows = []
    try:
        for _ in range(reps):
            ctx.scf_step_packed()
            rows.append(_fef.fef_plan_stage_ms(ctx.plan))
    finally:
        _fef.fef_plan_stage_timing(ctx.plan, False)
    ms = np.mean(np.asarray(rows), axis=0)
    m = scf_stage_model(sysm)

    def hbm(nbytes, t):
        a = nbytes / (t / 1e3)
        return {"bound": "hbm", "achieved": a / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": a / HBM_PEAK, "bytes_per_launch": nbytes, "ms": round(float(t), 4)}
    fl = m["eigh_flops"] / (ms[3] / 1e3)
    return {"steps": reps,
            "density_ms": round(float(ms[0]), 4),
            "moments": hbm(m["moments_bytes"], ms[1]),
            "field_and_coulomb": hbm(m["field_bytes"], ms[2]),
            "eigensolver": {"bound": "fp64", "achieved": fl / 1e12, "peak": FP64_PEAK / 1e12,
                            "unit": "TFLOP/s", "frac": fl / FP64_PEAK,
                            "flops_per_launch": m["eigh_flops"], "ms": round(float(ms[3]), 4)},
            "step_ms": round(float(np.sum(ms)), 4)}


def copy_probe(mib: int):
    """A plain device-to-device copy of known size (counter calibration)."""
    import torch
    n = mib << 20
    a = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "launches": 3}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the FEF pair path "
              "runs on a single device here; multi-GPU sharding is not implemented",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return
    import torch

    import fefgen
    import paper_1708_03377_amd as lib

    sysm = fefgen.make_system(args.workload)
    spec = sysm.spec
    niter = spec.niter
    ctx = lib.Context(sysm, device="cuda:0")
    modes = [m for m in (args.modes or DEFAULT_MODES.get(args.workload, "f64")).split(",") if m]
    if "f64" not in modes:
        modes = ["f64"] + modes
    st = ctx.stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    results = {}
    for name in modes:
        prec = lib.PREC[name]
        print(f"[bench] mode {name}: autotune", file=sys.stderr, flush=True)
        ctx.reset_orbitals()
        ctx.scf(niter)
        xb, yc, tune_us = ctx.autotune(prec, reps=3)
        # stage breakdown of one eager step
        e = [ev() for _ in range(4)]
        ctx.reset_orbitals()
        e[0].record(st)
        ctx.scf(niter)
        e[1].record(st)
        ctx.half_transform(prec)
        e[2].record(st)
        ctx.pair_energies(prec)
        e[3].record(st)
        torch.cuda.synchronize()
        stage = [e[i].elapsed_time(e[i + 1]) for i in range(3)]
        # pair contraction launches, event-timed on the library's stream
        pe = [(ev(), ev()) for _ in range(args.steps)]
        for a, b in pe:
            a.record(st)
            ctx.pair_energies(prec)
            b.record(st)
        torch.cuda.synchronize()
        pair_ms = float(np.mean([a.elapsed_time(b) for a, b in pe]))
        # the half transform + pair energies unit on the current orbitals,
        # each repetition event-timed: median, min and max of 20 after 5
        hp = [(ev(), ev()) for _ in range(25)]
        for a, b in hp:
            a.record(st)
            ctx.half_transform(prec)
            ctx.pair_energies(prec)
            b.record(st)
        torch.cuda.synchronize()
        unit = [a.elapsed_time(b) for a, b in hp][5:]
        # the timed steps: graph replays of the whole pass
        g = ctx.graph(niter, prec, from_start=True)
        for _ in range(args.warmup):
            ctx.launch(g)
        torch.cuda.synchronize()
        ge = [(ev(), ev()) for _ in range(args.steps)]
        t0 = time.perf_counter()
        for a, b in ge:
            a.record(st)
            ctx.launch(g)
            b.record(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = float(np.mean([a.elapsed_time(b) for a, b in ge]))
        results[name] = {
            "ms_per_step": 1e3 * wall / args.steps, "gpu_ms_per_step": gpu_ms,
            "stage_ms": stage, "pair_ms": pair_ms, "tiles": (xb, yc), "unit_ms": unit,
            "E_total": float(ctx.E2_total.cpu()[0]), "flags": int(ctx.flags.cpu()[0]),
            "E2": ctx.E2_pair[:ctx.npair].cpu().numpy().copy()}
        del g
        print(f"[bench] mode {name}: {results[name]['ms_per_step']:.3f} ms/step", file=sys.stderr,
              flush=True)

    print("[bench] SCF stages", file=sys.stderr, flush=True)
    scf_stages = bench_scf_stages(ctx, lib, sysm)
    coupled = None
    if not args.no_coupled:
        print("[bench] coupled dimer doubles", file=sys.stderr, flush=True)
        coupled = bench_coupled(ctx, sysm, torch, st)
        coupled_C, coupled_eps = ctx.C.cpu().numpy(), ctx.eps.cpu().numpy()
    monomer = None
    if not args.no_monomer and int(np.max(sysm.cls)) == 0:
        print("[bench] monomer energies", file=sys.stderr, flush=True)
        from paper_1708_03377_amd import _fef
        # on the workload's final orbitals (the SCF stage timing above ran
        # further steps)
        ctx.reset_orbitals()
        ctx.scf(niter)
        monomer = bench_monomer(ctx, sysm, torch, st, _fef)
        gm = os.path.join(ROOT, "tests", "golden", f"{spec.name}_monomer_oracle.npz")
        if os.path.exists(gm):
            monomer["oracle_total"] = float(np.load(gm, allow_pickle=False)["total"])
            monomer["err_vs_oracle"] = monomer["E_M2_total"] - monomer["oracle_total"]
        monomer_C, monomer_eps = ctx.C.cpu().numpy(), ctx.eps.cpu().numpy()
    ref = results["f64"]
    ref_oracle = oracle_total(spec.name)
    ref_total = ref_oracle if ref_oracle is not None else ref["E_total"]
    if spec.cfg_id == 4:
        # the exact kernel of the surrogate pass: the fastest reduced-precision
        # mode whose own total meets the bar on this workload (else FP64)
        passing = [m for m in results if m != "f64" and results[m]["flags"] == 0
                   and abs(results[m]["E_total"] - ref_total) <= TOTAL_ERR_BAR]
        exact_mode = min(passing, key=lambda m: results[m]["ms_per_step"]) if passing else "f64"
        print(f"[bench] surrogate ({exact_mode} exact kernel): training, held-out check, "
              "timed passes", file=sys.stderr, flush=True)
        results["surrogate"] = bench_surrogate(args, sysm, ctx, lib, torch, st, niter,
                                               exact_mode)

    modes_out = {}
    for name, r in results.items():
        err_tot = abs(r["E_total"] - ref["E_total"])
        err_orc = abs(r["E_total"] - ref_oracle) if ref_oracle is not None else None
        err_pair = float(np.max(np.abs(r["E2"] - ref["E2"]))) if sysm.npair else 0.0
        sur = "surrogate" in r
        modes_out[name] = {
            "pairs_per_s": sysm.npair / (r["ms_per_step"] / 1e3),
            "ms_per_step": round(r["ms_per_step"], 4),
            "gpu_ms_per_step": round(r["gpu_ms_per_step"], 4),
            "scf_ms": None if sur else round(r["stage_ms"][0], 4),
            "half_ms": None if sur else round(r["stage_ms"][1], 4),
            "pair_ms": round(r["pair_ms"], 4),
            "pair_tflops": None if sur else pair_flops(sysm) / (r["pair_ms"] / 1e3) / 1e12,
            "half_plus_pair": None if sur else {
                "median_ms": round(float(np.median(r["unit_ms"])), 4),
                "min_ms": round(float(np.min(r["unit_ms"])), 4),
                "max_ms": round(float(np.max(r["unit_ms"])), 4),
                "reps": len(r["unit_ms"]), "warmup": 5,
                "pairs_per_s": sysm.npair / (float(np.median(r["unit_ms"])) / 1e3)},
            "tiles_xb_yc": list(r["tiles"]),
            "total_err_vs_f64": err_tot, "max_pair_err_vs_f64": err_pair,
            "total_err_vs_oracle": err_orc,
            "E2_total": r["E_total"], "flags": r["flags"]}
        if sur:
            modes_out[name]["surrogate"] = r["surrogate"]
    # the gate: total within 1 uEh of the oracle's own total when it is
    # stored for this workload, else of the GPU FP64 path's
    gate = "total_err_vs_oracle" if ref_oracle is not None else "total_err_vs_f64"
    ok = [m for m in modes_out if modes_out[m][gate] <= TOTAL_ERR_BAR
          and modes_out[m]["flags"] == 0]
    head = max(ok, key=lambda m: modes_out[m]["pairs_per_s"]) if ok else "f64"
    h = modes_out[head]
    # the dominant kernel: the exact pair kernel of the headline mode (the
    # surrogate pass runs its exact kernel on the pairs it declines)
    kmode = modes_out[head]["surrogate"]["exact_kernel"] if head == "surrogate" else head
    hk = modes_out[kmode]
    flops = pair_flops(sysm)
    bound, peak = PEAK[kmode]
    achieved = flops / (hk["pair_ms"] / 1e3)
    classes = []
    for c in range(sysm.nclass):
        f = int(np.nonzero(sysm.cls == c)[0][0])
        classes.append({"count": int(np.sum(sysm.cls == c)), "nbf": int(sysm.nbf[f]),
                        "nocc": int(sysm.nocc[f]), "P": int(sysm.naux_class[c])})
    line = {
        "metric": METRIC, "value": h["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": h["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": head,
        "data": "synthetic (seeded liquid-like water box, random-init fragment data)",
        "config": {"workload": spec.name, "nfrag": int(sysm.nfrag), "npair": int(sysm.npair),
                   "fragment_classes": classes, "cutoff_A": spec.cutoff, "niter": niter,
                   "step": ("eager: orbital reset + niter SCF steps + fragment invariants + "
                            "ensemble selection + half transform + exact pair energies of the "
                            "declined pairs + total" if head == "surrogate" else
                            "HIP-graph replay: orbital reset + niter SCF steps + half "
                            "transform + pair energies + total")},
        "roofline": {"kernel": f"pair contraction ({kmode})", "bound": bound,
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": traffic_from_profiles(kmode, spec.name),
                     "algorithmic_flops_per_launch": flops,
                     "issued_flops_per_launch": pair_issued_flops(sysm, kmode),
                     "issued_frac": pair_issued_flops(sysm, kmode) / (hk["pair_ms"] / 1e3) / peak,
                     "launch_ms": hk["pair_ms"],
                     "operand_bytes": pair_operand_bytes(ctx, lib.PREC[kmode])},
        "accuracy_gate": {"bar_Eh": TOTAL_ERR_BAR, "against": "oracle" if ref_oracle is not None
                          else "gpu_f64", "oracle_total": ref_oracle},
        "scf_roofline": scf_stages,
        # the SCF share of the timed captured pass: the pass less the half
        # transform + pair energies unit timed alone on the same orbitals
        "scf_in_pass_ms": round(h["gpu_ms_per_step"] - h["half_plus_pair"]["median_ms"], 4)
        if h.get("half_plus_pair") else None,
        "coupled": coupled,
        "monomer": monomer,
        "fp64_pairs_per_s": modes_out["f64"]["pairs_per_s"],
        "speedup_vs_fp64": h["pairs_per_s"] / modes_out["f64"]["pairs_per_s"],
        "modes": modes_out,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(sysm, niter, args.cpu_seconds)
        if coupled is not None:
            coupled["cpu_baseline"] = coupled_cpu_baseline(sysm, coupled_C, coupled_eps)
        if monomer is not None:
            monomer["cpu_baseline"] = monomer_cpu_baseline(sysm, monomer_C, monomer_eps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
