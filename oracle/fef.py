"""Plain FP64 definitions of the FEF pair energy and effective-field SCF.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path may import this module.

Paper: arXiv:1708.03377, Sec. II ("Theory").  Index domains follow
Sec. II.A: MO indices i (occupied), a (virtual), p on fragment x and j, b, q on
fragment y; AO indices mu, nu on x and lambda, sigma on y.  Fragment
quantities are real, so no complex conjugation appears.

Readings of the paper used here (where it is silent or its source is
garbled):

* Integral model.  The paper evaluates exact Gaussian integrals over
  monomer-centred bases (the "bubble" integrals, Eq. dp2e).  The synthetic
  workloads instead give a factored inter-fragment Coulomb tensor
  (mu nu|lambda sigma)^{xy} = sum_PQ B^x_{P mu nu} T^{xy}_{PQ} B^y_{Q lambda sigma}
  with T^{xy} = s_xy G_{c(x) c(y)}, s_xy = 1/R_xy (bohr^-1), G_{0,c} = G_{c,0}^T.
* Notation.  v^{pq}_{rs} = <pq|rs> = (pr|qs) with p, r on x and q, s on y
  (Eq. NHxy), so v^{ij}_{ab} = (ia|jb).
* Spin.  Restricted closed-shell fragments; the dimer doubles of Eq. 1dt2
  carry no antisymmetrisation (A ~ 1, Eq. prodspace), so each spatial
  (ia|jb) appears for 2 x 2 spin choices: E2_xy = 4 sum (ia|jb) t^{ab}_{ij}.
* Zeroth order.  H0's particle-rank-conserving two-body part W^[0]
  (Eq. partitioning0) is dropped from the dimer amplitude equation
  (Eq. dimDoubles); with canonical orbitals the remaining F^[0] is diagonal,
  so t^{ab}_{ij} = (ia|jb) / (eps_i + eps_j - eps_a - eps_b).
* Pair sum.  E_D2 (Eq. ED2) counts each unordered pair x < y once.
* Field.  omega_x = h~ + 2 v^{mu j}_{nu j} (Eq. wc) with the bubble integral
  of Eq. dp2e summed over every other fragment y inside the cutoff; the
  density D^y = C^y_occ C^y_occ^T carries no factor 2 (the 2 is in Eq. wc).
  h~ (nuclear attraction) is zero in every synthetic workload; an additive
  h~^x is accepted.
* SCF.  F~ = F0 + h~ + J (Eq. for the polarisation-screened Fock matrix),
  with F0^x = h + 2J - K of the isolated fragment frozen at its generated
  value; simultaneous (Jacobi-style) update of all fragments, no damping,
  Aufbau occupation, a fixed number of iterations; after the last iteration
  E2 uses the canonical eigenpairs of F~ (the paper's remark that the final
  FEF solution is canonical).  Zero iterations is the non-interacting
  (MCPT) reference.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np


# ---------------------------------------------------------------------------
# coupling
# ---------------------------------------------------------------------------
def coupling(sys, x: int, y: int, s: float) -> np.ndarray:
    """T^{xy} = s_xy G_{c(x) c(y)}, shape (P_{c(x)}, P_{c(y)}).

    The workloads give G_{c,0} for every class c; G_{0,c} is its transpose.
    A pair with neither fragment in class 0 has no defined coupling.
    """
    cx, cy = int(sys.cls[x]), int(sys.cls[y])
    if cy == 0:
        g = sys.G_of(cx)
    elif cx == 0:
        g = sys.G_of(cy).T
    else:
        raise ValueError("no coupling defined between two non-solvent classes")
    return s * g


# ---------------------------------------------------------------------------
# half transform and pair integrals (Sec. II.A MO coefficients; Eq. NHxy)
# ---------------------------------------------------------------------------
def half_transform(B: np.ndarray, C: np.ndarray, nocc: int) -> np.ndarray:
    """B_ov[P, i, a] = sum_{mu nu} C_{mu i} B[P, mu, nu] C_{nu a}.

    The x-side half of the four-index AO -> MO transform of the factored
    integrals; columns of C are MOs, occupied first.
    """
    Co = C[:, :nocc]
    Cv = C[:, nocc:]
    return np.einsum("mi,pmn,na->pia", Co, B, Cv, optimize=True)


def pair_integrals(Bov_x: np.ndarray, Bov_y: np.ndarray, T: np.ndarray) -> np.ndarray:
    """(ia|jb) = sum_{PQ} B^x_ov[P,i,a] T[P,Q] B^y_ov[Q,j,b] = v^{ij}_{ab}."""
    return np.einsum("pia,pq,qjb->iajb", Bov_x, T, Bov_y, optimize=True)


def orbital_gaps(eps: np.ndarray, nocc: int) -> np.ndarray:
    """Delta_ia = eps_i - eps_a (negative for a gapped fragment)."""
    return eps[:nocc, None] - eps[None, nocc:]


def pair_energies(sys, C_pool=None, eps_pool=None, pairs=None):
    """E2_xy for every listed pair and E_D2 = sum over the unordered pairs.

    Returns (E2[npair] float64, E_D2).  The per-fragment half transforms are
    computed once and reused; the pair integrals and the weighted sum follow
    the definitions above one pair at a time.  E_D2 is summed with
    ``math.fsum`` (correctly rounded), so it does not depend on pair order.
    """
    px = sys.pair_x if pairs is None else pairs[0]
    py = sys.pair_y if pairs is None else pairs[1]
    ps = sys.pair_s if pairs is None else pairs[2]
    need = np.unique(np.concatenate([px, py])) if len(px) else np.zeros(0, int)
    bov = {}
    gaps = {}
    for f in need:
        f = int(f)
        o = int(sys.nocc[f])
        bov[f] = half_transform(sys.B_of(f), sys.C_of(f, C_pool), o).reshape(
            sys.B_of(f).shape[0], -1)
        gaps[f] = orbital_gaps(sys.eps_of(f, eps_pool), o).ravel()
    E2 = np.zeros(len(px), dtype=np.float64)
    for k in range(len(px)):
        x, y = int(px[k]), int(py[k])
        T = coupling(sys, x, y, float(ps[k]))
        V = bov[x].T @ T @ bov[y]                       # (ia|jb), rows ia, cols jb
        D = gaps[x][:, None] + gaps[y][None, :]
        E2[k] = 4.0 * np.sum(V * V / D)
    return E2, math.fsum(E2.tolist())


def brute_force_pair_energy(Bx, By, Cx, Cy, ex, ey, ox, oy, T) -> float:
    """E2_xy by explicit loops: build every AO integral
    (mu nu|lambda sigma)^{xy} = sum_PQ B^x_{P mu nu} T_PQ B^y_{Q lambda sigma},
    transform all four indices one MO quadruple at a time, and sum
    4 (ia|jb)^2 / (e_i + e_j - e_a - e_b).  For tiny fragments only."""
    P, n, _ = Bx.shape
    Q, m, _ = By.shape
    ao = np.zeros((n, n, m, m))
    for mu in range(n):
        for nu in range(n):
            for la in range(m):
                for si in range(m):
                    acc = 0.0
                    for p in range(P):
                        for q in range(Q):
                            acc += Bx[p, mu, nu] * T[p, q] * By[q, la, si]
                    ao[mu, nu, la, si] = acc
    e = 0.0
    for i in range(ox):
        for a in range(ox, n):
            for j in range(oy):
                for b in range(oy, m):
                    v = 0.0
                    for mu in range(n):
                        for nu in range(n):
                            for la in range(m):
                                for si in range(m):
                                    v += (Cx[mu, i] * Cx[nu, a] * Cy[la, j] * Cy[si, b]
                                          * ao[mu, nu, la, si])
                    e += 4.0 * v * v / (ex[i] + ey[j] - ex[a] - ey[b])
    return e


# ---------------------------------------------------------------------------
# effective field (Eqs. wc and dp2e) and SCF step
# ---------------------------------------------------------------------------
def density(C: np.ndarray, nocc: int) -> np.ndarray:
    """D_{lambda sigma} = sum_j C_{lambda j} C_{sigma j} (no factor 2)."""
    Co = C[:, :nocc]
    return Co @ Co.T


def densities(sys, C_pool=None):
    return [density(sys.C_of(f, C_pool), int(sys.nocc[f])) for f in range(sys.nfrag)]


def neighbours(sys):
    """Every ordered neighbour (x, y, s_xy), both orientations of each pair."""
    out = [[] for _ in range(sys.nfrag)]
    for x, y, s in zip(sys.pair_x.tolist(), sys.pair_y.tolist(), sys.pair_s.tolist()):
        out[x].append((y, s))
        out[y].append((x, s))
    return out


def moments(B: np.ndarray, D: np.ndarray) -> np.ndarray:
    """d_Q = sum_{lambda sigma} B_{Q lambda sigma} D_{lambda sigma}."""
    return np.einsum("qls,ls->q", B, D)


def coulomb_field(sys, D_list, nbrs=None):
    """J^x_{mu nu} = 2 sum_{y != x, R < r_c} sum_j (mu nu|j j)^{xy}
    = 2 sum_y sum_{lambda sigma} (mu nu|lambda sigma)^{xy} D^y_{lambda sigma},
    written through the factored integrals as
    2 sum_P B^x_{P mu nu} sum_y (T^{xy} d^y)_P with d^y = B^y : D^y
    (Eqs. wc and dp2e).  Returns a list of J^x."""
    nbrs = neighbours(sys) if nbrs is None else nbrs
    d = [moments(sys.B_of(f), D_list[f]) for f in range(sys.nfrag)]
    J = []
    for x in range(sys.nfrag):
        phi = np.zeros(sys.B_of(x).shape[0])
        for y, s in nbrs[x]:
            phi += coupling(sys, x, y, s) @ d[y]
        J.append(2.0 * np.einsum("pmn,p->mn", sys.B_of(x), phi))
    return J


def coulomb_field_explicit(sys, D_list, nbrs=None):
    """J^x from explicitly built AO integrals (mu nu|lambda sigma)^{xy},
    contracted with D^y one neighbour at a time (small systems only)."""
    nbrs = neighbours(sys) if nbrs is None else nbrs
    J = []
    for x in range(sys.nfrag):
        Bx = sys.B_of(x)
        n = Bx.shape[1]
        acc = np.zeros((n, n))
        for y, s in nbrs[x]:
            T = coupling(sys, x, y, s)
            ao = np.einsum("pmn,pq,qls->mnls", Bx, T, sys.B_of(y))
            acc += 2.0 * np.einsum("mnls,ls->mn", ao, D_list[y])
        J.append(acc)
    return J


def scf_step(sys, C_pool, eps_pool, htilde=None):
    """One simultaneous FEF update of every fragment.

    F~^x = F0^x + h~^x + J^x[D^y from C_pool];  (eps, C) = eigh(F~^x) ascending;
    lowest nocc orbitals occupied.  Returns (C_pool', eps_pool', D_list',
    max |D' - D|, gap_ok).
    """
    D_old = densities(sys, C_pool)
    J = coulomb_field(sys, D_old)
    C_new = np.empty_like(C_pool)
    e_new = np.empty_like(eps_pool)
    D_new = []
    dmax = 0.0
    gap_ok = True
    oc = sys.off_C
    oe = sys.off_eps
    for x in range(sys.nfrag):
        n = int(sys.nbf[x]); o = int(sys.nocc[x])
        F = sys.F0_of(x) + J[x]
        if htilde is not None:
            F = F + htilde[oc[x]:oc[x + 1]].reshape(n, n)
        w, v = np.linalg.eigh(F)
        C_new[oc[x]:oc[x + 1]] = v.ravel()
        e_new[oe[x]:oe[x + 1]] = w
        Dx = density(v, o)
        D_new.append(Dx)
        dmax = max(dmax, float(np.max(np.abs(Dx - D_old[x]))) if n else 0.0)
        if 0 < o < n and not (w[o] > w[o - 1]):
            gap_ok = False
    return C_new, e_new, D_new, dmax, gap_ok


def run_scf(sys, niter: int, htilde=None):
    """``niter`` FEF iterations from the generated orbitals; returns
    (C_pool, eps_pool, [max|dD| per iteration])."""
    C = sys.C.copy()
    e = sys.eps.copy()
    hist = []
    for _ in range(niter):
        C, e, _, dmax, _ = scf_step(sys, C, e, htilde)
        hist.append(dmax)
    return C, e, hist


def fock_matrices(sys, C_pool, htilde=None):
    """F~^x for every fragment at the densities of C_pool."""
    J = coulomb_field(sys, densities(sys, C_pool))
    oc = sys.off_C
    out = []
    for x in range(sys.nfrag):
        n = int(sys.nbf[x])
        F = sys.F0_of(x) + J[x]
        if htilde is not None:
            F = F + htilde[oc[x]:oc[x + 1]].reshape(n, n)
        out.append(F)
    return out
