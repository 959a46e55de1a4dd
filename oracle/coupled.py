"""Dimer doubles with the two-body part of the zeroth-order Hamiltonian.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this
module.

Paper: arXiv:1708.03377, Sec. II.B.  The particle-rank-conserving partition
(Eq. partitioning0) puts H0 = F^[0] + W^[0]; the first-order dimer amplitude
equation (Eq. dimDoubles) then reads

    <phi_2^xy| F^[0] T_2^xy + W^[0] T_2^xy + W^[+2] |phi_0^xy> = 0,

a linear system for the amplitudes t[i, a, j, b] of the excitations i -> a
on fragment x and j -> b on fragment y, whose pair energy is
E2_xy = 4 sum v t (the spin factor of the plain pair energy, reading 3 of
oracle.fef).  With W^[0] dropped (oracle.fef, reading 4) the system is
diagonal and t = -v / D.

Readings used here (the paper is silent or the workloads do not define
more):

* W^[0] between fragments only.  The workloads define the inter-fragment
  Coulomb tensor (oracle.fef, reading 1) and nothing inside a fragment, so
  the two-body operator that acts on the dimer doubles is the
  inter-fragment Coulomb operator sum (pq|rs)^{xy} {E^x_pq}{E^y_rs} in
  normal order (no exchange between fragments, A ~ 1, Eq. prodspace).  Its
  particle-rank-conserving part couples the dimer doubles through
      + (a a'|b b')  t[i, a', j, b']     particle ladder
      - (a a'|j' j)  t[i, a', j', b]     particle-hole, hole on y
      - (i' i|b b')  t[i', a, j, b']     hole-particle, hole on x
      + (i' i|j' j)  t[i', a, j', b]     hole ladder
  (the sign of each term is the product of the signs of the normal-ordered
  one-body operators on the two fragments: + for a particle line, - for a
  hole line).
* F^[0] is the diagonal of the canonical fragment Fock operators, so its
  action is D t with D = eps_a + eps_b - eps_i - eps_j (positive).
* The linear system (D + W) t = -v is symmetric: each term's matrix is
  symmetric under the exchange of its primed and unprimed indices, the
  integrals being real and symmetric in each fragment's index pair.
"""
from __future__ import annotations

import numpy as np

from . import fef as ofef


def mo_blocks(B: np.ndarray, C: np.ndarray, nocc: int):
    """The occupied-occupied, virtual-virtual and occupied-virtual blocks of
    B_P in the MO basis C^T B_P C: shapes (P, o, o), (P, v, v), (P, o, v)."""
    Bmo = np.einsum("mp,Pmn,nq->Ppq", C, B, C, optimize=True)
    o = nocc
    return Bmo[:, :o, :o], Bmo[:, o:, o:], Bmo[:, :o, o:]


def pair_blocks(Bx, Cx, ox, By, Cy, oy, T):
    """The four integral blocks of a pair and its (ia|jb), from the factored
    tensor (pq|rs) = sum_PQ Bx_P[p,q] T_PQ By_Q[r,s] (oracle.fef reading 1):
    oovv (i i'|b b'), vvoo (a a'|j j'), oooo (i i'|j j'), vvvv (a a'|b b'),
    ovov (i a|j b)."""
    xoo, xvv, xov = mo_blocks(Bx, Cx, ox)
    yoo, yvv, yov = mo_blocks(By, Cy, oy)
    TyBoo = np.einsum("PQ,Qrs->Prs", T, yoo)
    TyBvv = np.einsum("PQ,Qrs->Prs", T, yvv)
    TyBov = np.einsum("PQ,Qrs->Prs", T, yov)
    return {
        "oooo": np.einsum("Pij,Pkl->ijkl", xoo, TyBoo),   # (i i'|j j')
        "oovv": np.einsum("Pij,Pab->ijab", xoo, TyBvv),   # (i i'|b b')
        "vvoo": np.einsum("Pab,Pij->abij", xvv, TyBoo),   # (a a'|j j')
        "vvvv": np.einsum("Pab,Pcd->abcd", xvv, TyBvv),   # (a a'|b b')
        "ovov": np.einsum("Pia,Pjb->iajb", xov, TyBov),   # (i a|j b)
    }


def w0_apply(blk: dict, t: np.ndarray) -> np.ndarray:
    """(W t)[i,a,j,b] for the inter-fragment W^[0] of the module header."""
    pp = np.einsum("aAbB,iAjB->iajb", blk["vvvv"], t)
    ph = np.einsum("aAJj,iAJb->iajb", blk["vvoo"], t)
    hp = np.einsum("IibB,IajB->iajb", blk["oovv"], t)
    hh = np.einsum("IiJj,IaJb->iajb", blk["oooo"], t)
    return pp - ph - hp + hh


def denominators(ex: np.ndarray, ox: int, ey: np.ndarray, oy: int) -> np.ndarray:
    """D[i,a,j,b] = eps_a + eps_b - eps_i - eps_j (the F^[0] diagonal)."""
    dx = ex[ox:][None, :] - ex[:ox][:, None]   # [i, a]
    dy = ey[oy:][None, :] - ey[:oy][:, None]   # [j, b]
    return dx[:, :, None, None] + dy[None, None, :, :]


def solve_dense(blk: dict, D: np.ndarray, scale_w: float = 1.0) -> np.ndarray:
    """t of (D + scale_w W) t = -v by a dense LU solve (small pairs only)."""
    v = blk["ovov"]
    shape = v.shape
    n = v.size
    A = np.diag(D.reshape(n))
    if scale_w != 0.0:
        E = np.eye(n).reshape((n,) + shape)
        cols = np.stack([w0_apply(blk, E[k]).reshape(n) for k in range(n)], axis=1)
        A = A + scale_w * cols
    return np.linalg.solve(A, -v.reshape(n)).reshape(shape)


def solve_cg(blk: dict, D: np.ndarray, tol: float = 1e-14, maxit: int = 500) -> np.ndarray:
    """t of (D + W) t = -v by conjugate gradients preconditioned with D,
    stopped when ||r|| <= tol ||v||."""
    v = blk["ovov"]
    b = -v
    t = b / D
    r = b - (D * t + w0_apply(blk, t))
    z = r / D
    p = z.copy()
    rz = float(np.sum(r * z))
    nb = float(np.linalg.norm(b))
    for _ in range(maxit):
        if float(np.linalg.norm(r)) <= tol * nb:
            break
        Ap = D * p + w0_apply(blk, p)
        alpha = rz / float(np.sum(p * Ap))
        t = t + alpha * p
        r = r - alpha * Ap
        z = r / D
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return t


def coupled_pair_energy(sys, x: int, y: int, s: float, C_pool=None, eps_pool=None,
                        method: str = "cg") -> float:
    """E2_xy = 4 sum v t with t from (D + W) t = -v (module header)."""
    C_pool = sys.C if C_pool is None else C_pool
    eps_pool = sys.eps if eps_pool is None else eps_pool
    ox, oy = int(sys.nocc[x]), int(sys.nocc[y])
    T = ofef.coupling(sys, x, y, s)
    blk = pair_blocks(sys.B_of(x), sys.C_of(x, C_pool), ox, sys.B_of(y), sys.C_of(y, C_pool),
                      oy, T)
    D = denominators(sys.eps_of(x, eps_pool), ox, sys.eps_of(y, eps_pool), oy)
    t = solve_dense(blk, D) if method == "dense" else solve_cg(blk, D)
    return 4.0 * float(np.sum(blk["ovov"] * t))


def coupled_pair_energies(sys, C_pool=None, eps_pool=None, pairs=None, method: str = "cg"):
    """Coupled E2 of every pair (or the listed pair indices) and their sum."""
    idx = range(sys.npair) if pairs is None else pairs
    E = np.array([coupled_pair_energy(sys, int(sys.pair_x[k]), int(sys.pair_y[k]),
                                      float(sys.pair_s[k]), C_pool, eps_pool, method)
                  for k in idx])
    return E, float(np.sum(E))
