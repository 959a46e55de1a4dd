"""Pins of the dressing oracle (oracle/dressing.py).

The spatial blocks are pinned against Eqs. MPij and MPab evaluated term by
term over spin orbitals (explicit spins, the spin-orbital integrals and
first-order amplitudes built by loops from the AO integrals), against the
trace identity tr Hoo = -tr Hvv = E2 / 2 per pair and fragment, and against
the exchange of the pair's two fragments."""
import itertools

import numpy as np
import pytest

import fefgen
from oracle import coupled as oc
from oracle import dressing as od
from oracle import fef as ofef


def tiny(seed=5, sizes=((4, 2), (5, 2)), naux=4):
    return fefgen.make_random_system(seed, list(sizes), naux=naux, spacing=2.0)


def test_spatial_blocks_match_spin_orbital_equations():
    sysm = tiny()
    x, y, s = 0, 1, float(1.0 / (np.linalg.norm(sysm.pos[0] - sysm.pos[1]) *
                                 fefgen.BOHR_PER_ANGSTROM))
    nx, ny = int(sysm.nbf[x]), int(sysm.nbf[y])
    ox, oy = int(sysm.nocc[x]), int(sysm.nocc[y])
    T = ofef.coupling(sysm, x, y, s)
    Bx, By, Cx, Cy = sysm.B_of(x), sysm.B_of(y), sysm.C_of(x), sysm.C_of(y)
    ex, ey = sysm.eps_of(x), sysm.eps_of(y)
    # MO integrals (pq|rs), p, q on x and r, s on y, by loops from the AO tensor
    ao = np.zeros((nx, nx, ny, ny))
    for m, n_, l, g in itertools.product(range(nx), range(nx), range(ny), range(ny)):
        ao[m, n_, l, g] = sum(Bx[P, m, n_] * T[P, Q] * By[Q, l, g]
                              for P in range(Bx.shape[0]) for Q in range(By.shape[0]))
    mo = np.zeros((nx, nx, ny, ny))
    for p, q, r, t in itertools.product(range(nx), range(nx), range(ny), range(ny)):
        mo[p, q, r, t] = sum(Cx[m, p] * Cx[n_, q] * Cy[l, r] * Cy[g, t] * ao[m, n_, l, g]
                             for m in range(nx) for n_ in range(nx)
                             for l in range(ny) for g in range(ny))

    # spin orbitals: (orbital, spin); <p q|r s> = (p r|q s) for spin(p) = spin(r),
    # spin(q) = spin(s) (p, r on x; q, s on y)
    def v(p, q, r, s_):
        (po, ps), (qo, qs), (ro, rs), (so, ss) = p, q, r, s_
        return mo[po, ro, qo, so] if (ps == rs and qs == ss) else 0.0

    occ_x = [(i, sp) for i in range(ox) for sp in (0, 1)]
    vir_x = [(a, sp) for a in range(ox, nx) for sp in (0, 1)]
    occ_y = [(j, sp) for j in range(oy) for sp in (0, 1)]
    vir_y = [(b, sp) for b in range(oy, ny) for sp in (0, 1)]

    def tamp(a, b, i, j):  # t^{ab}_{ij} = <ij|ab> / (e_i + e_j - e_a - e_b)
        return v(i, j, a, b) / (ex[i[0]] + ey[j[0]] - ex[a[0]] - ey[b[0]])

    Hoo_so = {(i, i1): sum(v(i, j1, a1, b1) * tamp(a1, b1, i1, j1)
                           for j1 in occ_y for a1 in vir_x for b1 in vir_y)
              for i in occ_x for i1 in occ_x}
    Hvv_so = {(a, a1): -sum(v(i1, j1, a1, b1) * tamp(a, b1, i1, j1)
                            for i1 in occ_x for j1 in occ_y for b1 in vir_y)
              for a in vir_x for a1 in vir_x}
    V, t = od.pair_amplitudes(sysm, x, y, s)
    hoo, hvv, _, _ = od.pair_dressing(V, t)
    scale = max(abs(x_) for x_ in Hoo_so.values())
    for (i, i1), val in Hoo_so.items():
        ref = hoo[i[0], i1[0]] if i[1] == i1[1] else 0.0
        assert val == pytest.approx(ref, abs=1e-12 * scale)
    scale = max(abs(x_) for x_ in Hvv_so.values())
    for (a, a1), val in Hvv_so.items():
        ref = hvv[a[0] - ox, a1[0] - ox] if a[1] == a1[1] else 0.0
        assert val == pytest.approx(ref, abs=1e-12 * scale)
    assert scale > 1e-8


@pytest.mark.parametrize("coupled", [False, True])
def test_trace_identity_per_pair(coupled):
    sysm = tiny(seed=9, sizes=((6, 2), (7, 3)), naux=5)
    V, t = od.pair_amplitudes(sysm, 0, 1, 0.3, coupled=coupled)
    hox, hvx, hoy, hvy = od.pair_dressing(V, t)
    e2 = 4.0 * np.sum(V * t)
    for tr, sign in ((np.trace(hox), 1), (np.trace(hoy), 1), (np.trace(hvx), -1),
                     (np.trace(hvy), -1)):
        assert tr == pytest.approx(sign * e2 / 2, rel=1e-12)
    # the uncoupled E2 is the plain pair energy
    if not coupled:
        T = ofef.coupling(sysm, 0, 1, 0.3)
        ref = ofef.brute_force_pair_energy(sysm.B_of(0), sysm.B_of(1), sysm.C_of(0),
                                           sysm.C_of(1), sysm.eps_of(0), sysm.eps_of(1),
                                           int(sysm.nocc[0]), int(sysm.nocc[1]), T)
        assert e2 == pytest.approx(ref, rel=1e-12)


def test_swapping_the_pair_swaps_the_blocks():
    sysm = tiny(seed=11, sizes=((5, 2), (4, 1)), naux=5)
    V, t = od.pair_amplitudes(sysm, 0, 1, 0.4, coupled=True)
    V2, t2 = od.pair_amplitudes(sysm, 1, 0, 0.4, coupled=True)
    a = od.pair_dressing(V, t)
    b = od.pair_dressing(V2, t2)
    for u, w in ((a[0], b[2]), (a[1], b[3]), (a[2], b[0]), (a[3], b[1])):
        np.testing.assert_allclose(u, w, rtol=0, atol=1e-12 * np.max(np.abs(u)))


def test_fragment_sums_of_workload0():
    """Every fragment's dressing is the sum over its pairs: its occupied trace
    is half the sum of its pairs' energies, and the virtual one minus that."""
    sysm = fefgen.make_system(0)
    Hoo, Hvv, E2 = od.dressings(sysm)
    E0, _ = ofef.pair_energies(sysm)
    np.testing.assert_allclose(E2, E0, rtol=1e-12)
    for f in range(sysm.nfrag):
        mine = (sysm.pair_x == f) | (sysm.pair_y == f)
        half = 0.5 * np.sum(E2[mine])
        assert np.trace(Hoo[f]) == pytest.approx(half, rel=1e-12)
        assert np.trace(Hvv[f]) == pytest.approx(-half, rel=1e-12)
    # not a scalar multiple of the identity: the blocks carry structure
    assert np.max(np.abs(Hoo[0] - np.diag(np.diag(Hoo[0])))) > 1e-6
