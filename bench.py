"""Benchmark: fragment-pair E2 evaluations per second on one MI355X.

One step = one whole FEF pass over a seeded synthetic box, inputs resident
in HBM: reset the orbitals to the generated ones, run the effective-field SCF
(niter simultaneous updates), half-transform every fragment, evaluate every
pair energy and the total.  Every precision mode of the pair contraction is
timed; the headline value is the fastest mode whose total energy stays within
1 micro-Hartree of the FP64 path's total on the same step.

Prints ONE JSON line (rank 0).  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 1]
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

PEAK = {"f64": ("mfma", 78.6e12), "f32": ("mfma", 157.3e12),
        "bf16x2": ("mfma", 2.5e15), "fp16x2": ("mfma", 2.5e15)}
TOTAL_ERR_BAR = 1e-6  # Eh


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=1, help="workload id (0..4)")
    ap.add_argument("--modes", default="f64,f32,bf16x2,fp16x2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def pair_flops(sysm) -> float:
    """Algorithmic flops of the pair contraction: 2 ov_x ov_y P0 per pair."""
    ov = (sysm.nocc.astype(np.int64) * (sysm.nbf - sysm.nocc).astype(np.int64))
    p0 = float(sysm.naux_class[0])
    return float(np.sum(2.0 * ov[sysm.pair_x] * ov[sysm.pair_y] * p0))


def kernel_sources_hash() -> str:
    d = os.path.join(ROOT, "paper_1708_03377_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".cpp", ".h")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(mode: str):
    """HBM bytes per launch of the pair kernel from committed PMC summaries,
    or None when they are missing or were taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"pair_{mode}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("sources_hash") != kernel_sources_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(sysm, niter: int, budget_s: float):
    """The CPU oracle, untuned, on a bounded sample of the same workload."""
    from oracle import fef as ofef
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] or [1])
    except Exception:
        threads = 1
    t0 = time.perf_counter()
    C, e, _, _, _ = ofef.scf_step(sysm, sysm.C.copy(), sysm.eps.copy())
    t_scf = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    remaining = max(budget_s - t_scf, 1.0)
    n = min(sysm.npair, 2000)
    t_pairs, done = 0.0, 0
    while t_pairs < remaining and done < sysm.npair:
        idx = rng.choice(sysm.npair, size=n, replace=False)
        t0 = time.perf_counter()
        ofef.pair_energies(sysm, C, e, pairs=(sysm.pair_x[idx], sysm.pair_y[idx],
                                              sysm.pair_s[idx]))
        t_pairs += time.perf_counter() - t0
        done += n
    step_s = niter * t_scf + sysm.npair * (t_pairs / done)
    return {"value": sysm.npair / step_s, "unit": "pairs/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"1 SCF step over all {sysm.nfrag} fragments ({t_scf:.2f} s) and "
                      f"{done} random pairs ({t_pairs:.2f} s), scaled to {niter} steps + "
                      f"{sysm.npair} pairs",
            "affinity_cpus": len(os.sched_getaffinity(0))}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the FEF pair path "
              "is not sharded across GPUs in this build", file=sys.stderr)
        sys.exit(2)
    import torch

    import fefgen
    import paper_1708_03377_amd as lib

    sysm = fefgen.make_system(args.workload)
    spec = sysm.spec
    niter = spec.niter
    ctx = lib.Context(sysm, device="cuda:0")
    modes = [m for m in args.modes.split(",") if m]
    if "f64" not in modes:
        modes = ["f64"] + modes
    st = ctx.stream()

    def step(prec, ev=None):
        ctx.reset_orbitals()
        if ev: ev[0].record(st)
        ctx.scf(niter)
        if ev: ev[1].record(st)
        ctx.half_transform(prec)
        if ev: ev[2].record(st)
        ctx.pair_energies(prec)
        if ev: ev[3].record(st)

    results = {}
    for name in modes:
        prec = lib.PREC[name]
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(prec, evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        scf = np.mean([e[0].elapsed_time(e[1]) for e in evs])
        half = np.mean([e[1].elapsed_time(e[2]) for e in evs])
        pair = np.mean([e[2].elapsed_time(e[3]) for e in evs])
        total = float(ctx.E2_total.cpu()[0])
        flags = int(ctx.flags.cpu()[0])
        results[name] = {"ms_per_step": 1e3 * wall / args.steps, "scf_ms": scf,
                         "half_ms": half, "pair_ms": pair, "E_D2": total, "flags": flags,
                         "E2": ctx.E2_pair[:ctx.npair].cpu().numpy().copy()}
    ref = results["f64"]
    modes_out = {}
    for name, r in results.items():
        err_tot = abs(r["E_D2"] - ref["E_D2"])
        err_pair = float(np.max(np.abs(r["E2"] - ref["E2"]))) if sysm.npair else 0.0
        modes_out[name] = {"pairs_per_s": sysm.npair / (r["ms_per_step"] / 1e3),
                           "ms_per_step": round(r["ms_per_step"], 4),
                           "scf_ms": round(r["scf_ms"], 4), "half_ms": round(r["half_ms"], 4),
                           "pair_ms": round(r["pair_ms"], 4),
                           "pair_kernel_pairs_per_s": sysm.npair / (r["pair_ms"] / 1e3),
                           "total_err_vs_f64": err_tot, "max_pair_err_vs_f64": err_pair,
                           "E_D2": r["E_D2"], "flags": r["flags"]}
    ok = [m for m in modes_out if modes_out[m]["total_err_vs_f64"] <= TOTAL_ERR_BAR]
    head = max(ok, key=lambda m: modes_out[m]["pairs_per_s"])
    h = modes_out[head]
    flops = pair_flops(sysm)
    bound, peak = PEAK[head]
    achieved = flops / (h["pair_ms"] / 1e3)
    line = {
        "metric": "fragment-pair E2 evals/s at 1 GPU, mixed/surrogate vs FP64 at <=1 uEh total error",
        "value": h["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": h["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head, "data": "synthetic",
        "config": {"workload": spec.name, "nfrag": sysm.nfrag, "npair": sysm.npair,
                   "niter": niter, "cutoff_A": spec.cutoff,
                   "step": "SCF(niter) + half transform + pair energies + total"},
        "roofline": {"kernel": f"pair contraction ({head})", "bound": bound,
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": traffic_from_profiles(head),
                     "algorithmic_flops_per_launch": flops},
        "fp64_pairs_per_s": modes_out["f64"]["pairs_per_s"],
        "speedup_vs_fp64": h["pairs_per_s"] / modes_out["f64"]["pairs_per_s"],
        "modes": modes_out,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sysm, niter, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
