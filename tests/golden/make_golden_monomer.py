"""Writes the full-size expected monomer energies under tests/golden/ by
calling only the CPU oracle and the seeded input generator.

For each listed single-class (water) workload the oracle runs its own
effective-field SCF from the generated orbitals (Sec. II.A, simultaneous
updates, the workload's number of iterations) and then evaluates E_M2^x
(Eq. EM2 with the first-order doubles of Eq. monDoubles) of every fragment
on its own final orbitals.  Stored per workload
(``<name>_monomer_oracle.npz``):

* ``E_M2``: every fragment's energy in fragment order;
* ``total``: their correctly rounded sum;
* ``eps``: the final orbital-energy pool (the same SCF as the pair-energy
  expected values of make_golden_fullsize.py).

Run:  python tests/golden/make_golden_monomer.py [workload ids] [--procs N]
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
from oracle import fef, monomer  # noqa: E402

_S = None
_C = None
_E = None


def _chunk(idx):
    E, _ = monomer.monomer_energies(_S, _C, _E, frags=idx)
    return int(idx[0]), E


def golden_path(name: str) -> str:
    return os.path.join(HERE, f"{name}_monomer_oracle.npz")


def make(cfg: int, procs: int):
    global _S, _C, _E
    t0 = time.time()
    s = fefgen.make_system(cfg)
    print(f"[{s.spec.name}] {s.nfrag} fragments, {s.spec.niter} iterations", flush=True)
    C, e = s.C.copy(), s.eps.copy()
    for k in range(s.spec.niter):
        C, e, _, dmax, _ = fef.scf_step(s, C, e)
        print(f"  scf step {k + 1}: max|dD| {dmax:.3e} ({time.time() - t0:.0f} s)", flush=True)
    _S, _C, _E = s, C, e
    bounds = np.linspace(0, s.nfrag, 8 * procs + 1).astype(np.int64)
    chunks = [np.arange(bounds[i], bounds[i + 1]) for i in range(len(bounds) - 1)
              if bounds[i + 1] > bounds[i]]
    E = np.zeros(s.nfrag)
    with mp.get_context("fork").Pool(procs) as pool:
        for first, part in pool.imap_unordered(_chunk, chunks):
            E[first:first + len(part)] = part
    total = math.fsum(E.tolist())
    np.savez_compressed(golden_path(s.spec.name), name=np.array(s.spec.name), E_M2=E,
                        total=total, eps=e)
    print(f"  E_M2 = {total:.12f}; wrote {golden_path(s.spec.name)} "
          f"({time.time() - t0:.0f} s)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="*", type=int, default=[1, 3])
    ap.add_argument("--procs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    a = ap.parse_args()
    for w in a.workloads:
        make(w, a.procs)


if __name__ == "__main__":
    main()
