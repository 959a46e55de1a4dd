"""Pins of the coupled dimer-doubles oracle (oracle/coupled.py).

The operator W is pinned against an explicit second-quantised construction
in the occupation-number basis of two tiny fragments (independent of the
index bookkeeping of oracle/coupled.py: determinants, creation and
annihilation with their phases, the inter-fragment Coulomb operator built
from the AO integrals by brute force); the solver against a dense solve;
the limit without W against the plain pair energy; the linear system's
symmetry, its stationarity, and the x <-> y symmetry of the energy.
"""
import itertools

import numpy as np
import pytest

import fefgen
from oracle import coupled as oc
from oracle import fef as ofef


def tiny(seed=5, sizes=((3, 1), (4, 2)), naux=4):
    return fefgen.make_random_system(seed, list(sizes), naux=naux, spacing=2.0)


def pair_setup(sysm, x=0, y=1):
    s = float(1.0 / (np.linalg.norm(sysm.pos[x] - sysm.pos[y]) * fefgen.BOHR_PER_ANGSTROM))
    T = ofef.coupling(sysm, x, y, s)
    ox, oy = int(sysm.nocc[x]), int(sysm.nocc[y])
    blk = oc.pair_blocks(sysm.B_of(x), sysm.C_of(x), ox, sysm.B_of(y), sysm.C_of(y), oy, T)
    D = oc.denominators(sysm.eps_of(x), ox, sysm.eps_of(y), oy)
    return s, T, ox, oy, blk, D


# --- explicit Fock space ----------------------------------------------------
def _apply(op, state):
    """Apply a string of (create?, spin-orbital) from right to left to a
    state {occupation bitmask: coefficient}."""
    out = dict(state)
    for create, k in reversed(op):
        nxt = {}
        for det, c in out.items():
            occ = (det >> k) & 1
            if create == occ:
                continue
            sign = -1.0 if bin(det & ((1 << k) - 1)).count("1") % 2 else 1.0
            nd = det ^ (1 << k)
            nxt[nd] = nxt.get(nd, 0.0) + sign * c
        out = nxt
    return out


def _E(p, q, off):
    """Spin-summed E_pq = sum_s a+_{p s} a_{q s} on orbitals offset by off
    (spin-orbital 2 (off + p) + s)."""
    return [[(1, 2 * (off + p) + s), (0, 2 * (off + q) + s)] for s in (0, 1)]


def _apply_E(p, q, off, state):
    out = {}
    for op in _E(p, q, off):
        for d, c in _apply(op, state).items():
            out[d] = out.get(d, 0.0) + c
    return out


def _dot(a, b):
    return sum(c * b.get(d, 0.0) for d, c in a.items())


def test_w_matches_second_quantised_coulomb_operator():
    """<ia,jb| {E^x_pq} {E^y_rs} (pq|rs) |i'a',j'b'> over normalised singlet
    dimer doubles, built from determinants, equals oracle.coupled's W."""
    sysm = tiny()
    s, T, ox, oy, blk, D = pair_setup(sysm)
    nx, ny = int(sysm.nbf[0]), int(sysm.nbf[1])
    Cx, Cy = sysm.C_of(0), sysm.C_of(1)
    # MO-basis inter-fragment integrals by brute force from the AO tensor
    Bx, By = sysm.B_of(0), sysm.B_of(1)
    ao = np.zeros((nx, nx, ny, ny))
    for m, n_, l, sg in itertools.product(range(nx), range(nx), range(ny), range(ny)):
        ao[m, n_, l, sg] = sum(Bx[P, m, n_] * T[P, Q] * By[Q, l, sg]
                               for P in range(Bx.shape[0]) for Q in range(By.shape[0]))
    mo = np.einsum("mp,nq,lr,st,mnls->pqrt", Cx, Cx, Cy, Cy, ao)
    # closed-shell reference: fragment x orbitals 0..nx-1, y after them
    ref = 0
    for p in range(ox):
        ref |= 3 << (2 * p)
    for p in range(oy):
        ref |= 3 << (2 * (nx + p))
    zero = {ref: 1.0}

    def nE(p, q, off, state):
        # normal-ordered spin-summed one-body operator: E_pq - <0|E_pq|0>
        e = _apply_E(p, q, off, state)
        occ_ref = 2.0 if (p == q and ((off == 0 and p < ox) or (off == nx and p < oy))) else 0.0
        if occ_ref:
            for d, c in state.items():
                e[d] = e.get(d, 0.0) - occ_ref * c
        return e

    def dimer(i, a, j, b):
        st = _apply_E(nx + oy + b, nx + j, 0, _apply_E(ox + a, i, 0, zero))
        nrm = np.sqrt(_dot(st, st))
        return {d: c / nrm for d, c in st.items()}

    vx, vy = nx - ox, ny - oy
    idx = list(itertools.product(range(ox), range(vx), range(oy), range(vy)))
    states = {k: dimer(*k) for k in idx}
    W_ref = np.zeros((len(idx), len(idx)))
    for c2, k2 in enumerate(idx):
        st = states[k2]
        acc = {}
        for p, q in itertools.product(range(nx), range(nx)):
            sx = nE(p, q, 0, st)
            if not sx:
                continue
            for r, t in itertools.product(range(ny), range(ny)):
                if mo[p, q, r, t] == 0.0:
                    continue
                sy = nE(r, t, nx, sx)
                for d, c in sy.items():
                    acc[d] = acc.get(d, 0.0) + mo[p, q, r, t] * c
        for c1, k1 in enumerate(idx):
            W_ref[c1, c2] = _dot(states[k1], acc)
    n = len(idx)
    E = np.eye(n).reshape((n, ox, vx, oy, vy))
    W_oc = np.stack([oc.w0_apply(blk, E[k]).reshape(n) for k in range(n)], axis=1)
    np.testing.assert_allclose(W_oc, W_ref, rtol=0, atol=1e-13 * np.max(np.abs(W_ref)))
    assert np.max(np.abs(W_ref)) > 1e-6


def test_without_w_is_the_plain_pair_energy():
    sysm = tiny(seed=7, sizes=((5, 2), (6, 3)), naux=6)
    s, T, ox, oy, blk, D = pair_setup(sysm)
    t = oc.solve_dense(blk, D, scale_w=0.0)
    e0 = 4.0 * float(np.sum(blk["ovov"] * t))
    Bov_x = ofef.half_transform(sysm.B_of(0), sysm.C_of(0), ox)
    Bov_y = ofef.half_transform(sysm.B_of(1), sysm.C_of(1), oy)
    ref = ofef.brute_force_pair_energy(sysm.B_of(0), sysm.B_of(1), sysm.C_of(0), sysm.C_of(1),
                                       sysm.eps_of(0), sysm.eps_of(1), ox, oy, T)
    assert e0 == pytest.approx(ref, rel=1e-13, abs=1e-16)
    assert Bov_x.shape[0] == T.shape[0] and Bov_y.shape[0] == T.shape[1]


def test_cg_matches_dense_solve_and_system_is_symmetric():
    sysm = tiny(seed=9, sizes=((5, 2), (6, 3)), naux=6)
    s, T, ox, oy, blk, D = pair_setup(sysm)
    n = blk["ovov"].size
    E = np.eye(n).reshape((n,) + blk["ovov"].shape)
    W = np.stack([oc.w0_apply(blk, E[k]).reshape(n) for k in range(n)], axis=1)
    np.testing.assert_allclose(W, W.T, rtol=0, atol=1e-15 * np.max(np.abs(W)))
    td = oc.solve_dense(blk, D)
    tc = oc.solve_cg(blk, D)
    np.testing.assert_allclose(tc, td, rtol=0, atol=1e-12 * np.max(np.abs(td)))
    # W changes the energy (the system is really coupled)
    t0 = oc.solve_dense(blk, D, scale_w=0.0)
    assert abs(np.sum(blk["ovov"] * (td - t0))) > 1e-6 * abs(np.sum(blk["ovov"] * t0))


def test_energy_is_stationary_and_symmetric_in_the_pair():
    """J(t) = 4 (2 v.t + t.(D + W) t) is stationary at the solution, where it
    equals 4 v.t; swapping x and y leaves the energy unchanged."""
    sysm = tiny(seed=11, sizes=((5, 2), (4, 1)), naux=5)
    s, T, ox, oy, blk, D = pair_setup(sysm)
    v = blk["ovov"]
    t = oc.solve_dense(blk, D)

    def J(u):
        return 4.0 * (2.0 * np.sum(v * u) + np.sum(u * (D * u + oc.w0_apply(blk, u))))
    e = 4.0 * np.sum(v * t)
    assert J(t) == pytest.approx(e, rel=1e-12)
    rng = np.random.default_rng(3)
    d = rng.standard_normal(t.shape)
    for h in (1e-3, 1e-4):
        # J(t + h d) - J(t) = 4 h^2 d.(D + W) d exactly (no linear term)
        quad = 4.0 * h * h * np.sum(d * (D * d + oc.w0_apply(blk, d)))
        assert J(t + h * d) - J(t) == pytest.approx(quad, rel=1e-6)
    # the same pair with the fragments swapped
    s2 = s
    T2 = ofef.coupling(sysm, 1, 0, s2)
    blk2 = oc.pair_blocks(sysm.B_of(1), sysm.C_of(1), oy, sysm.B_of(0), sysm.C_of(0), ox, T2)
    D2 = oc.denominators(sysm.eps_of(1), oy, sysm.eps_of(0), ox)
    e2 = 4.0 * np.sum(blk2["ovov"] * oc.solve_dense(blk2, D2))
    assert e2 == pytest.approx(e, rel=1e-12)


def test_coupled_energies_of_workload0():
    """Workload 0 (8 waters): every pair converges, the coupled pair energy
    stays negative and within a few percent of the plain one (the
    inter-fragment ladders are small next to the orbital-energy gaps)."""
    sysm = fefgen.make_system(0)
    E, tot = oc.coupled_pair_energies(sysm)
    E0, tot0 = ofef.pair_energies(sysm)
    assert np.all(E < 0)
    rel = np.abs(E - E0) / np.abs(E0)
    assert np.all(rel < 0.2) and np.max(rel) > 1e-6
