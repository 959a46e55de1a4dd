"""Cross-fragment dressing of the fragment one-body intermediates by the
dimer doubles.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this
module.

Paper: arXiv:1708.03377, Sec. III (equation-of-motion FEF-CCPT), Eqs. MPij
and MPab.  The one-body blocks of fragment x's inclusive similarity
transformed Hamiltonian gain, from every other fragment y, in spin orbitals
(repeated indices summed; j1, b1 on y; i, i1, a, a1 on x):
    H^i_{i1} += v^{i j1}_{i1 b1} t^{b1}_{j1} + v^{i j1}_{a1 b1} t^{a1 b1}_{i1 j1}
    H^a_{a1} += v^{a j1}_{a1 b1} t^{b1}_{j1} - v^{i1 j1}_{a1 b1} t^{a b1}_{i1 j1}

Readings used here:

* Singles.  The fragment singles t^b_j vanish at this order (the effective
  field is already inside each fragment's Fock operator, Sec. II.A), so only
  the dimer-doubles terms remain; H^i_a of Eq. MPia, which has no doubles
  term, gets no dressing.
* Spin.  Closed-shell fragments with no exchange between them (A ~ 1,
  Eq. prodspace): v^{ij}_{ab} = (ia|jb) couples a same-spin pair i, a on x
  and a same-spin pair j, b on y, and the dimer doubles have the same spin
  pattern.  The spin-orbital blocks are diagonal in spin and the same for
  both spins; summing the two spins of j1, b1 gives the spatial form
      Hoo^x[i, i1] =  2 sum_{a, j, b} V[i a, j b] t[i1 a, j b]
      Hvv^x[a, a1] = -2 sum_{i, j, b} V[i a1, j b] t[i a, j b]
  with V[ia, jb] = (ia|jb) and t the dimer doubles of the pair (t = -V / D
  with the diagonal F^[0], or the W^[0]-coupled amplitudes of
  oracle.coupled).  Fragment y of the pair gets the same blocks with the two
  fragments' roles swapped.
* The sum over y runs over the pair list (each unordered pair once, both of
  its fragments dressed).
"""
from __future__ import annotations

import numpy as np

from . import coupled as oc
from . import fef as ofef


def pair_dressing(V: np.ndarray, t: np.ndarray):
    """The four blocks one pair adds: (Hoo^x, Hvv^x, Hoo^y, Hvv^y) from the
    pair's (ia|jb) and amplitudes, both shaped [i, a, j, b]."""
    hoo_x = 2.0 * np.einsum("iajb,kajb->ik", V, t)
    hvv_x = -2.0 * np.einsum("iAjb,iajb->aA", V, t)
    hoo_y = 2.0 * np.einsum("iajb,iakb->jk", V, t)
    hvv_y = -2.0 * np.einsum("iajB,iajb->bB", V, t)
    return hoo_x, hvv_x, hoo_y, hvv_y


def pair_amplitudes(sys, x: int, y: int, s: float, C_pool=None, eps_pool=None,
                    coupled: bool = False):
    """(V, t) of one pair, shaped [i, a, j, b]: t = -V / D, or the solution
    of the W^[0]-coupled system."""
    C_pool = sys.C if C_pool is None else C_pool
    eps_pool = sys.eps if eps_pool is None else eps_pool
    ox, oy = int(sys.nocc[x]), int(sys.nocc[y])
    T = ofef.coupling(sys, x, y, s)
    blk = oc.pair_blocks(sys.B_of(x), sys.C_of(x, C_pool), ox, sys.B_of(y),
                         sys.C_of(y, C_pool), oy, T)
    D = oc.denominators(sys.eps_of(x, eps_pool), ox, sys.eps_of(y, eps_pool), oy)
    t = oc.solve_cg(blk, D) if coupled else -blk["ovov"] / D
    return blk["ovov"], t


def dressings(sys, C_pool=None, eps_pool=None, coupled: bool = False):
    """Per-fragment dressings summed over the pair list: (Hoo, Hvv, E2)
    with Hoo[f] [nocc][nocc], Hvv[f] [nvir][nvir] and the pair energies
    E2 = 4 sum V t."""
    Hoo = [np.zeros((int(o), int(o))) for o in sys.nocc]
    Hvv = [np.zeros((int(n - o), int(n - o))) for n, o in zip(sys.nbf, sys.nocc)]
    E2 = np.zeros(sys.npair)
    for k in range(sys.npair):
        x, y = int(sys.pair_x[k]), int(sys.pair_y[k])
        V, t = pair_amplitudes(sys, x, y, float(sys.pair_s[k]), C_pool, eps_pool, coupled)
        hox, hvx, hoy, hvy = pair_dressing(V, t)
        Hoo[x] += hox
        Hvv[x] += hvx
        Hoo[y] += hoy
        Hvv[y] += hvy
        E2[k] = 4.0 * float(np.sum(V * t))
    return Hoo, Hvv, E2
