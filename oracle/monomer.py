"""Monomer part of the second-order FEF-CCPT energy, E_M2.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this
module.

Paper: arXiv:1708.03377, Sec. II.B.  The second-order correlation energy
splits into a sum over fragments and a sum over fragment pairs
(Eq. EFEF2).  The fragment part (Eq. EM2) contracts each fragment's
two-body de-excitation operator W^[-2]_x with its first-order doubles
T_2^x(1), which solve the fragment doubles equation written with the
effective fragment Hamiltonian (Eq. monDoubles).

Readings used here (the paper is silent or the workloads do not define
more):

* Integrals inside a fragment.  The workloads define the two-electron
  tensor between fragments only (oracle.fef, reading 1).  Inside a fragment
  of the solvent class (class 0) the same factored form is taken with that
  class's own coupling block at unit scale:
      (mu nu|lambda sigma)^{xx} = sum_PQ B^x_{P mu nu} G_{0,0}[P, Q] B^x_{Q lambda sigma}.
  G_{0,0} is symmetric positive definite, so this is a valid Coulomb-like
  tensor (every (ia|ia) >= 0).  The workloads give no G_{c,c} for another
  class, so E_M2 is defined for class-0 fragments only.
* Zeroth order.  As for the pair energies (oracle.fef, reading 4), the
  two-body part W^[0] of the fragment Hamiltonian is dropped from
  Eq. monDoubles; with the canonical FEF orbitals the remaining F^[0] is
  diagonal and the spin-orbital doubles are
      t^{ab}_{ij} = <ij||ab> / (eps_i + eps_j - eps_a - eps_b).
* Spin.  Closed-shell fragments whose electrons are antisymmetrised among
  themselves.  Summing the spin-orbital energy (1/4) sum |<ij||ab>|^2 / D
  over spins gives, in spatial orbitals,
      E_M2^x = sum_{ijab} (ia|jb) [2 (ia|jb) - (ib|ja)]
                          / (eps_i + eps_j - eps_a - eps_b),
  with i, j occupied and a, b virtual orbitals of fragment x.
"""
from __future__ import annotations

import math

import numpy as np


def intra_ao_integrals(B: np.ndarray, G00: np.ndarray) -> np.ndarray:
    """(mu nu|lambda sigma) = sum_PQ B[P, mu, nu] G00[P, Q] B[Q, lambda, sigma]."""
    return np.einsum("pmn,pq,qls->mnls", B, G00, B, optimize=True)


def mo_integrals(I_ao: np.ndarray, C: np.ndarray) -> np.ndarray:
    """(pq|rs) = sum C[mu, p] C[nu, q] C[lambda, r] C[sigma, s] (mu nu|lambda sigma)."""
    t = np.tensordot(C, I_ao, axes=([0], [0]))          # p nu lambda sigma
    t = np.tensordot(C, t, axes=([0], [1]))             # q p lambda sigma
    t = np.tensordot(C, t, axes=([0], [2]))             # r q p sigma
    t = np.tensordot(C, t, axes=([0], [3]))             # s r q p
    return t.transpose(3, 2, 1, 0)


def monomer_energy(B: np.ndarray, C: np.ndarray, eps: np.ndarray, nocc: int,
                   G00: np.ndarray) -> float:
    """E_M2 of one fragment (Eq. EM2 with the doubles of Eq. monDoubles,
    W^[0] dropped), in the closed-shell spatial-orbital form above."""
    o = int(nocc)
    I = mo_integrals(intra_ao_integrals(B, G00), C)
    K = I[:o, o:, :o, o:]                       # K[i, a, j, b] = (ia|jb)
    Kx = K.transpose(0, 3, 2, 1)                # Kx[i, a, j, b] = (ib|ja)
    e_o, e_v = eps[:o], eps[o:]
    D = (e_o[:, None, None, None] - e_v[None, :, None, None]
         + e_o[None, None, :, None] - e_v[None, None, None, :])
    return float(np.sum(K * (2.0 * K - Kx) / D))


def monomer_energies(sys, C_pool=None, eps_pool=None, frags=None):
    """E_M2^x for the listed fragments (all by default) and their sum.

    Every listed fragment must be of class 0 (the only class whose coupling
    with itself the workloads define).  Returns (per-fragment array, the
    correctly rounded sum of its entries).
    """
    idx = range(sys.nfrag) if frags is None else [int(f) for f in frags]
    G00 = sys.G_of(0)
    out = []
    for x in idx:
        if int(sys.cls[x]) != 0:
            raise ValueError("E_M2 is defined for class-0 fragments only")
        out.append(monomer_energy(sys.B_of(x), sys.C_of(x, C_pool), sys.eps_of(x, eps_pool),
                                  int(sys.nocc[x]), G00))
    E = np.array(out, dtype=np.float64)
    return E, math.fsum(E.tolist())
