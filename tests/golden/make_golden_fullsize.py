"""Writes the full-size expected values under tests/golden/ by calling only
the CPU oracle and the seeded input generator.

For each benchmark-sized workload the oracle runs its own effective-field
SCF from the generated orbitals (Sec. II.A, simultaneous updates, the
workload's number of iterations) and then evaluates the pair energies of
Eq. ED2 (first-order dimer doubles of Eq. dimDoubles) of every listed pair on
its own final orbitals.  Stored per workload (``<name>_oracle.npz``):

* ``E2``: every pair energy in pair-list order (omitted for the 8000-water
  box, whose 1.9 million values are summarised by ``E2_sample``);
* ``E2_sample_idx`` / ``E2_sample``: a seeded sample of pairs plus the
  closest and farthest pair;
* ``total``: E_D2, the correctly rounded sum of every pair energy;
* ``eps``: the final orbital-energy pool; ``dD``: max |Delta D| per iteration;
* ``D_idx`` / ``D``: final densities of a seeded sample of fragments
  (fragment 0 always included), flattened and concatenated;
* ``gap_ok``: every fragment's final HOMO-LUMO gap is positive.

The pair loop is split over worker processes; each pair is evaluated by the
oracle's own ``pair_energies`` and the total is order-independent
(``math.fsum``), so the split does not change any stored number.

Run:  python tests/golden/make_golden_fullsize.py [workload ids] [--procs N]
"""
import argparse
import math
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import fefgen  # noqa: E402
from oracle import fef  # noqa: E402

# workload id -> whether every pair energy is stored
STORE_ALL = {1: True, 2: True, 3: True, 4: False}
NSAMPLE_PAIRS = 4000
NSAMPLE_FRAGS = 64

_S = None
_C = None
_E = None


def _chunk(idx):
    E2, _ = fef.pair_energies(_S, _C, _E, pairs=(_S.pair_x[idx], _S.pair_y[idx],
                                                 _S.pair_s[idx]))
    return idx[0], E2


def golden_path(name: str) -> str:
    return os.path.join(HERE, f"{name}_oracle.npz")


def make(cfg: int, procs: int):
    global _S, _C, _E
    t0 = time.time()
    s = fefgen.make_system(cfg)
    niter = s.spec.niter
    print(f"[{s.spec.name}] {s.nfrag} fragments, {s.npair} pairs, {niter} iterations",
          flush=True)
    C, e = s.C.copy(), s.eps.copy()
    hist = []
    gap_ok = True
    for k in range(niter):
        C, e, Dl, dmax, ok = fef.scf_step(s, C, e)
        hist.append(dmax)
        gap_ok = ok
        print(f"  scf step {k + 1}: max|dD| {dmax:.3e} ({time.time() - t0:.0f} s)", flush=True)
    if niter == 0:
        Dl = fef.densities(s, C)
    _S, _C, _E = s, C, e
    bounds = np.linspace(0, s.npair, 8 * procs + 1).astype(np.int64)
    chunks = [np.arange(bounds[i], bounds[i + 1]) for i in range(len(bounds) - 1)
              if bounds[i + 1] > bounds[i]]
    E2 = np.zeros(s.npair)
    with mp.get_context("fork").Pool(procs) as pool:
        for first, part in pool.imap_unordered(_chunk, chunks):
            E2[first:first + len(part)] = part
    total = math.fsum(E2.tolist())
    print(f"  pairs done ({time.time() - t0:.0f} s): E_D2 = {total:.12f}", flush=True)
    rng = np.random.default_rng(np.random.SeedSequence([fefgen.ROOT_SEED, 5151, cfg]))
    sidx = np.unique(np.concatenate([rng.choice(s.npair, min(NSAMPLE_PAIRS, s.npair),
                                                replace=False),
                                     [int(np.argmax(s.pair_s)), int(np.argmin(s.pair_s))]]))
    didx = np.unique(np.concatenate([[0], rng.choice(s.nfrag, min(NSAMPLE_FRAGS, s.nfrag),
                                                     replace=False)]))
    out = dict(name=np.array(s.spec.name), nfrag=s.nfrag, npair=s.npair, niter=niter,
               total=total, eps=e, dD=np.array(hist), gap_ok=gap_ok,
               E2_sample_idx=sidx.astype(np.int64), E2_sample=E2[sidx],
               D_idx=didx.astype(np.int64),
               D=np.concatenate([Dl[int(f)].ravel() for f in didx]))
    if STORE_ALL[cfg]:
        out["E2"] = E2
    np.savez_compressed(golden_path(s.spec.name), **out)
    print(f"  wrote {golden_path(s.spec.name)} ({time.time() - t0:.0f} s)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="*", type=int, default=[1, 2, 3])
    ap.add_argument("--procs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    a = ap.parse_args()
    for w in a.workloads:
        make(w, a.procs)


if __name__ == "__main__":
    main()
