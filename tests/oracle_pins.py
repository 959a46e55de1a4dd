"""Pins for the CPU oracle: checks against facts fixed by the paper and by
mathematics rather than by the oracle itself.

Each ``pin_*`` function raises AssertionError when the oracle (as currently
bound in ``oracle.fef``) disagrees with the fact it checks.  The same
functions run against deliberately broken copies of the oracle in
``test_oracle_pins.py`` to show that a plausible mistake fails at least one
of them.
"""
from __future__ import annotations

import numpy as np

import fefgen
from oracle import fef

REL = 1e-11


def _close(a, b, rel=REL, abs_=1e-14):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (a.shape, b.shape)
    tol = abs_ + rel * max(1.0, float(np.max(np.abs(b))) if b.size else 1.0)
    err = float(np.max(np.abs(a - b))) if a.size else 0.0
    assert err <= tol, f"max err {err:.3e} > tol {tol:.3e}"


def tiny_system(seed=1):
    return fefgen.make_random_system(seed, [(4, 2), (3, 1), (4, 1)], naux=3)


def tiny_two_class(seed=2, p1=3):
    # square solute coupling (P1 = P0) so that a transposed G keeps its shape
    return fefgen.make_two_class_system(seed, (4, 2, p1), [(3, 1), (4, 2)], naux0=3)


# ---------------------------------------------------------------------------
# pair energies
# ---------------------------------------------------------------------------
def pin_brute_force():
    """Factored, batched E2 equals the explicit four-index AO sum + loops."""
    for sysm in (tiny_system(1), tiny_two_class(2)):
        E2, tot = fef.pair_energies(sysm)
        for k in range(sysm.npair):
            x, y = int(sysm.pair_x[k]), int(sysm.pair_y[k])
            s = float(sysm.pair_s[k])
            cx, cy = int(sysm.cls[x]), int(sysm.cls[y])
            # T^{xy} = s G_{c(x)c(y)} with G_{0,c} = G_{c,0}^T, typed from the
            # workload definition
            if cy == 0:
                T = s * sysm.G_of(cx)
            else:
                T = s * sysm.G_of(cy).T
            ref = fef.brute_force_pair_energy(
                sysm.B_of(x), sysm.B_of(y), sysm.C_of(x), sysm.C_of(y),
                sysm.eps_of(x), sysm.eps_of(y), int(sysm.nocc[x]),
                int(sysm.nocc[y]), T)
            _close(E2[k], ref, rel=1e-12)
        _close(tot, sum(E2), rel=1e-13)


def pin_identity_coefficients():
    """C = I reduces the half transform to the occupied-virtual slice of B."""
    rng = np.random.default_rng(5)
    B = rng.standard_normal((3, 5, 5)); B = B + B.transpose(0, 2, 1)
    _close(fef.half_transform(B, np.eye(5), 2), B[:, :2, 2:], rel=0)


def pin_closed_form_one_by_one():
    """nocc = nvir = P = 1: E2 = 4 s^2 g^2 (b^x)^2 (b^y)^2 / (D^x + D^y) with
    b = C_{:,0}^T B C_{:,1} worked out for a 2x2 rotation by angle theta:
    b = (B11 - B00) sin t cos t + B01 cos 2t."""
    def frag(t, b00, b01, b11, e0, e1):
        C = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
        B = np.array([[[b00, b01], [b01, b11]]])
        b = (b11 - b00) * np.sin(t) * np.cos(t) + b01 * np.cos(2 * t)
        return B, C, np.array([e0, e1]), b
    Bx, Cx, ex, bx = frag(0.3, 0.2, -0.7, 0.5, -1.0, 0.5)
    By, Cy, ey, by = frag(-1.1, -0.4, 0.3, 0.9, -0.6, 1.7)
    g, s = 0.8, 0.25
    expect = 4 * s * s * g * g * bx * bx * by * by / ((-1.0 - 0.5) + (-0.6 - 1.7))
    sysm = fefgen.assemble([(Bx, Cx, ex, 1), (By, Cy, ey, 1)], [0, 0], [1],
                           [np.array([[g]])], np.zeros((2, 3)), None,
                           pairs=(np.array([0]), np.array([1]), np.array([1.0])))
    E2, _ = fef.pair_energies(sysm, pairs=(np.array([0]), np.array([1]),
                                           np.array([s])))
    _close(E2[0], expect, rel=1e-14)


def _degenerate(sysm):
    """Copy of sysm with one occupied and one virtual level per fragment."""
    eps = sysm.eps.copy()
    for f in range(sysm.nfrag):
        o = sysm.off_eps
        n = int(sysm.nbf[f]); no = int(sysm.nocc[f])
        e = np.empty(n); e[:no] = -0.8 - 0.1 * f; e[no:] = 0.9 + 0.05 * f
        eps[o[f]:o[f + 1]] = e
    return eps


def pin_gram_identity():
    """With degenerate levels the denominator is constant and
    E2 = 4 s^2 <B^x B^x^T, G B^y B^y^T G^T>_F / D (P x P Gram matrices)."""
    sysm = tiny_system(3)
    eps = _degenerate(sysm)
    E2, _ = fef.pair_energies(sysm, eps_pool=eps)
    G = sysm.G_of(0)
    for k in range(sysm.npair):
        x, y = int(sysm.pair_x[k]), int(sysm.pair_y[k]); s = float(sysm.pair_s[k])
        bx = np.einsum("mi,pmn,na->pia", sysm.C_of(x)[:, :sysm.nocc[x]],
                       sysm.B_of(x), sysm.C_of(x)[:, sysm.nocc[x]:]).reshape(3, -1)
        by = np.einsum("mi,pmn,na->pia", sysm.C_of(y)[:, :sysm.nocc[y]],
                       sysm.B_of(y), sysm.C_of(y)[:, sysm.nocc[y]:]).reshape(3, -1)
        ex = sysm.eps_of(x, eps); ey = sysm.eps_of(y, eps)
        D = (ex[0] - ex[-1]) + (ey[0] - ey[-1])
        gram = np.sum((bx @ bx.T) * (G @ by @ by.T @ G.T))
        _close(E2[k], 4 * s * s * gram / D, rel=1e-12)


def pin_distance_scaling():
    """At fixed orbitals every integral scales with s, so E2(c s) = c^2 E2(s)."""
    sysm = tiny_system(4)
    E2, _ = fef.pair_energies(sysm)
    E2c, _ = fef.pair_energies(sysm, pairs=(sysm.pair_x, sysm.pair_y,
                                            2.5 * sysm.pair_s))
    _close(E2c, 6.25 * E2, rel=1e-13)


def pin_pair_symmetry():
    """E2_xy = E2_yx (the pair energy does not depend on which fragment is
    called x), including the transposed coupling of a two-class pair."""
    for sysm in (tiny_system(5), tiny_two_class(6)):
        E2, _ = fef.pair_energies(sysm)
        E2r, _ = fef.pair_energies(sysm, pairs=(sysm.pair_y, sysm.pair_x,
                                                sysm.pair_s))
        _close(E2r, E2, rel=1e-13)


def pin_nonpositive():
    """Gapped canonical orbitals give E2 <= 0 for every pair."""
    sysm = fefgen.make_random_system(7, [(6, 2)] * 5, naux=4)
    E2, _ = fef.pair_energies(sysm)
    assert np.all(E2 <= 0.0) and np.any(E2 < 0.0)


def _rot(rng, n):
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q


def pin_rotation_sum_of_squares():
    """sum (ia|jb)^2 is unchanged by any rotation among the occupied and among
    the virtual orbitals of either fragment."""
    sysm = tiny_system(8)
    rng = np.random.default_rng(8)
    for k in range(sysm.npair):
        x, y = int(sysm.pair_x[k]), int(sysm.pair_y[k]); s = float(sysm.pair_s[k])
        T = fef.coupling(sysm, x, y, s)
        ox, oy = int(sysm.nocc[x]), int(sysm.nocc[y])
        Cx, Cy = sysm.C_of(x), sysm.C_of(y)
        V = fef.pair_integrals(fef.half_transform(sysm.B_of(x), Cx, ox),
                               fef.half_transform(sysm.B_of(y), Cy, oy), T)
        nx, ny = Cx.shape[0], Cy.shape[0]
        Ux = np.zeros((nx, nx)); Ux[:ox, :ox] = _rot(rng, ox); Ux[ox:, ox:] = _rot(rng, nx - ox)
        Uy = np.zeros((ny, ny)); Uy[:oy, :oy] = _rot(rng, oy); Uy[oy:, oy:] = _rot(rng, ny - oy)
        V2 = fef.pair_integrals(fef.half_transform(sysm.B_of(x), Cx @ Ux, ox),
                                fef.half_transform(sysm.B_of(y), Cy @ Uy, oy), T)
        _close(np.sum(V2 * V2), np.sum(V * V), rel=1e-13)


def pin_rotation_degenerate_blocks():
    """E2 is unchanged by rotations inside exactly degenerate levels."""
    sysm = fefgen.make_random_system(9, [(6, 3), (5, 2)], naux=4)
    eps = sysm.eps.copy()
    o = sysm.off_eps
    # fragment 0: occupied levels 0,1 degenerate; virtual 3,4,5 degenerate
    eps[o[0]:o[1]] = [-1.0, -1.0, -0.5, 0.4, 0.4, 0.4]
    eps[o[1]:o[2]] = [-0.9, -0.9, 0.7, 0.7, 1.3]
    E2, _ = fef.pair_energies(sysm, eps_pool=eps)
    rng = np.random.default_rng(9)
    C = sysm.C.copy()
    oc = sysm.off_C
    U0 = np.eye(6); U0[:2, :2] = _rot(rng, 2); U0[3:, 3:] = _rot(rng, 3)
    U1 = np.eye(5); U1[:2, :2] = _rot(rng, 2); U1[2:4, 2:4] = _rot(rng, 2)
    C[oc[0]:oc[1]] = (sysm.C_of(0) @ U0).ravel()
    C[oc[1]:oc[2]] = (sysm.C_of(1) @ U1).ravel()
    E2r, _ = fef.pair_energies(sysm, C_pool=C, eps_pool=eps)
    _close(E2r, E2, rel=1e-13)


# ---------------------------------------------------------------------------
# field and SCF
# ---------------------------------------------------------------------------
def pin_field_explicit():
    """Factored J equals J from explicitly built AO integrals; J is symmetric,
    linear in each D^y and vanishes with G = 0."""
    for sysm in (tiny_system(10), tiny_two_class(11)):
        D = fef.densities(sysm)
        J = fef.coulomb_field(sysm, D)
        Je = fef.coulomb_field_explicit(sysm, D)
        for a, b in zip(J, Je):
            _close(a, b, rel=1e-13)
            _close(a, a.T, rel=1e-14)
        D2 = [2.0 * d for d in D]
        for a, b in zip(fef.coulomb_field(sysm, D2), J):
            _close(a, 2.0 * b, rel=1e-14)
    sysm = tiny_system(12)
    sysm.G[:] = 0.0
    for a in fef.coulomb_field(sysm, fef.densities(sysm)):
        assert np.all(a == 0.0)


def pin_field_hand_two_fragments():
    """Two one-orbital-pair fragments with P = 1 written out by hand:
    J^x = 2 s g b^x (b^y : D^y), D^y = c_y c_y^T for the single occupied MO."""
    Bx = np.array([[[0.3, -0.2], [-0.2, 0.5]]]); By = np.array([[[0.1, 0.4], [0.4, -0.6]]])
    Cx = np.eye(2); t = 0.7
    Cy = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
    g, s = 0.6, 0.2
    sysm = fefgen.assemble([(Bx, Cx, np.array([-1., 1.]), 1),
                            (By, Cy, np.array([-1., 1.]), 1)], [0, 0], [1],
                           [np.array([[g]])], np.zeros((2, 3)), None,
                           pairs=(np.array([0]), np.array([1]), np.array([1.0 / s])))
    sysm.pair_s[:] = s
    cy = Cy[:, 0]
    dy = By[0, 0, 0] * cy[0] ** 2 + 2 * By[0, 0, 1] * cy[0] * cy[1] + By[0, 1, 1] * cy[1] ** 2
    J = fef.coulomb_field(sysm, fef.densities(sysm))
    _close(J[0], 2 * s * g * dy * Bx[0], rel=1e-14)


def pin_scf_properties():
    """After an SCF step: F~ C = C eps, C^T C = I, D^2 = D, tr D = nocc, eps
    ascending."""
    sysm = fefgen.make_random_system(13, [(6, 2), (5, 2), (6, 3), (4, 1)], naux=4)
    C, e, D, dmax, ok = fef.scf_step(sysm, sysm.C.copy(), sysm.eps.copy())
    F = fef.fock_matrices(sysm, sysm.C)
    for x in range(sysm.nfrag):
        Cx = sysm.C_of(x, C); ex = sysm.eps_of(x, e)
        _close(F[x] @ Cx, Cx * ex[None, :], rel=1e-12)
        _close(Cx.T @ Cx, np.eye(Cx.shape[0]), rel=1e-13)
        _close(D[x] @ D[x], D[x], rel=1e-13)
        _close(np.trace(D[x]), float(sysm.nocc[x]), rel=1e-13)
        assert np.all(np.diff(ex) >= 0)


def pin_scf_fixed_point():
    """With G = 0 there is no field and F~ = F0 = C0 diag(eps0) C0^T, so the
    generated orbitals are a fixed point: D and eps return unchanged."""
    sysm = fefgen.make_random_system(14, [(6, 2), (5, 3), (7, 2)], naux=3)
    sysm.G[:] = 0.0
    C, e, hist = fef.run_scf(sysm, 3)
    _close(e, sysm.eps, rel=1e-13)
    D0 = fef.densities(sysm); D1 = fef.densities(sysm, C)
    for a, b in zip(D1, D0):
        _close(a, b, rel=1e-12)


def pin_scf_input_rotation():
    """The step depends on the input orbitals only through D, so rotating the
    input C within occupied and within virtual orbitals changes neither the
    new D, eps nor the resulting E2."""
    sysm = fefgen.make_random_system(15, [(6, 2), (5, 2), (6, 3)], naux=4)
    rng = np.random.default_rng(15)
    C = sysm.C.copy()
    oc = sysm.off_C
    for x in range(sysm.nfrag):
        n = int(sysm.nbf[x]); o = int(sysm.nocc[x])
        U = np.zeros((n, n)); U[:o, :o] = _rot(rng, o); U[o:, o:] = _rot(rng, n - o)
        C[oc[x]:oc[x + 1]] = (sysm.C_of(x) @ U).ravel()
    Ca, ea, Da, _, _ = fef.scf_step(sysm, sysm.C.copy(), sysm.eps.copy())
    Cb, eb, Db, _, _ = fef.scf_step(sysm, C, sysm.eps.copy())
    _close(eb, ea, rel=1e-12)
    for a, b in zip(Db, Da):
        _close(a, b, rel=1e-11)
    _close(fef.pair_energies(sysm, Cb, eb)[0], fef.pair_energies(sysm, Ca, ea)[0],
           rel=1e-10)


PINS = [pin_brute_force, pin_identity_coefficients, pin_closed_form_one_by_one,
        pin_gram_identity, pin_distance_scaling, pin_pair_symmetry,
        pin_nonpositive, pin_rotation_sum_of_squares,
        pin_rotation_degenerate_blocks, pin_field_explicit,
        pin_field_hand_two_fragments, pin_scf_properties, pin_scf_fixed_point,
        pin_scf_input_rotation]
