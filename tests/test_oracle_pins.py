"""The oracle against its pins, and planted mistakes in the oracle (on the
CPU) against the same pins: every mutant must fail at least one pin."""
import numpy as np
import pytest

import fefgen
from oracle import fef

from . import oracle_pins as pins


@pytest.mark.parametrize("pin", pins.PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


# --- planted mistakes -------------------------------------------------------
_orig = {k: getattr(fef, k) for k in ("half_transform", "pair_integrals",
                                      "pair_energies", "coupling",
                                      "coulomb_field", "density", "scf_step",
                                      "orbital_gaps")}


def _m_transposed_C(B, C, nocc):
    return _orig["half_transform"](B, C.T.copy(), nocc)


def _m_gaps_sign(eps, nocc):
    return -_orig["orbital_gaps"](eps, nocc)


def _m_coupling_no_s(sysm, x, y, s):
    return _orig["coupling"](sysm, x, y, 1.0)


def _m_coupling_no_transpose(sysm, x, y, s):
    cx, cy = int(sysm.cls[x]), int(sysm.cls[y])
    g = sysm.G_of(cx) if cy == 0 else sysm.G_of(cy)
    return s * g


def _m_pair_energies_factor2(sysm, C_pool=None, eps_pool=None, pairs=None):
    E2, tot = _orig["pair_energies"](sysm, C_pool, eps_pool, pairs)
    return 0.5 * E2, 0.5 * tot


def _m_pair_energies_square_of_sum(sysm, C_pool=None, eps_pool=None, pairs=None):
    # weights applied before squaring: sum (V/D)^2 instead of V^2/D
    px = sysm.pair_x if pairs is None else pairs[0]
    py = sysm.pair_y if pairs is None else pairs[1]
    ps = sysm.pair_s if pairs is None else pairs[2]
    out = np.zeros(len(px))
    for k in range(len(px)):
        x, y = int(px[k]), int(py[k])
        ox, oy = int(sysm.nocc[x]), int(sysm.nocc[y])
        V = fef.pair_integrals(fef.half_transform(sysm.B_of(x), sysm.C_of(x, C_pool), ox),
                               fef.half_transform(sysm.B_of(y), sysm.C_of(y, C_pool), oy),
                               fef.coupling(sysm, x, y, float(ps[k])))
        dx = fef.orbital_gaps(sysm.eps_of(x, eps_pool), ox)
        dy = fef.orbital_gaps(sysm.eps_of(y, eps_pool), oy)
        D = dx[:, :, None, None] + dy[None, None, :, :]
        out[k] = -4.0 * np.sum((V / D) ** 2)
    return out, float(out.sum())


def _m_density_factor2(C, nocc):
    return 2.0 * _orig["density"](C, nocc)


def _m_field_self(sysm, D_list, nbrs=None):
    # uses the moment of x instead of y (index slip)
    nbrs = fef.neighbours(sysm) if nbrs is None else nbrs
    J = []
    for x in range(sysm.nfrag):
        phi = np.zeros(sysm.B_of(x).shape[0])
        dx = fef.moments(sysm.B_of(x), D_list[x])
        for y, s in nbrs[x]:
            T = fef.coupling(sysm, x, y, s)
            phi += T @ (dx if T.shape[1] == dx.shape[0] else fef.moments(sysm.B_of(y), D_list[y]))
        J.append(2.0 * np.einsum("pmn,p->mn", sysm.B_of(x), phi))
    return J


def _m_field_no_factor2(sysm, D_list, nbrs=None):
    return [0.5 * j for j in _orig["coulomb_field"](sysm, D_list, nbrs)]


def _m_scf_highest_occupied(sysm, C_pool, eps_pool, htilde=None):
    C, e, D, dmax, ok = _orig["scf_step"](sysm, C_pool, eps_pool, htilde)
    # occupy the highest orbitals: reverse the MO order of every fragment
    oc, oe = sysm.off_C, sysm.off_eps
    for x in range(sysm.nfrag):
        n = int(sysm.nbf[x])
        C[oc[x]:oc[x + 1]] = sysm.C_of(x, C)[:, ::-1].ravel()
        e[oe[x]:oe[x + 1]] = sysm.eps_of(x, e)[::-1]
    D = fef.densities(sysm, C)
    return C, e, D, dmax, ok


MUTANTS = {
    "transposed_C": ("half_transform", _m_transposed_C),
    "gap_sign": ("orbital_gaps", _m_gaps_sign),
    "coupling_without_distance": ("coupling", _m_coupling_no_s),
    "coupling_not_transposed": ("coupling", _m_coupling_no_transpose),
    "spin_factor_2": ("pair_energies", _m_pair_energies_factor2),
    "weight_before_square": ("pair_energies", _m_pair_energies_square_of_sum),
    "density_factor_2": ("density", _m_density_factor2),
    "field_self_moment": ("coulomb_field", _m_field_self),
    "field_missing_2": ("coulomb_field", _m_field_no_factor2),
    "aufbau_highest": ("scf_step", _m_scf_highest_occupied),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(fef, attr, fn)
    failed = []
    for pin in pins.PINS:
        try:
            pin()
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"


def test_pair_list_brute_force():
    """Generator pair lists match a brute-force minimum-image search; RSA
    centres respect the minimum distance; the cutoff is strict."""
    spec = fefgen.Spec(0, "t", 60, cutoff=9.0)
    sysm = fefgen.make_system(spec)
    L = sysm.box
    got = set(zip(sysm.pair_x.tolist(), sysm.pair_y.tolist()))
    exp = set()
    for i in range(sysm.nfrag):
        for j in range(i + 1, sysm.nfrag):
            d = sysm.pos[j] - sysm.pos[i]
            d = d - L * np.round(d / L)
            r = float(np.sqrt(d @ d))
            assert r >= 2.6
            if r < 9.0:
                exp.add((i, j))
    assert got == exp
    r_bohr = sysm.pair_r / 0.529177210903
    np.testing.assert_allclose(sysm.pair_s * r_bohr, 1.0, rtol=1e-15)


def test_config0_geometry():
    sysm = fefgen.make_system(0)
    assert sysm.npair == 28
    r = np.sort(np.round(sysm.pair_r / 0.529177210903, 3))
    assert list(np.unique(r)) == [5.858, 8.285, 10.147]


def test_conditioning_probe():
    """A 1e-13 relative perturbation of B moves the FP64 pair energies after
    the SCF by far less than the 1e-9 Eh parity tolerance."""
    spec = fefgen.Spec(1, "probe", 40, cutoff=9.0)
    sysm = fefgen.make_system(spec)
    C, e, _ = fef.run_scf(sysm, 4)
    E2, _ = fef.pair_energies(sysm, C, e)
    rng = np.random.default_rng(0)
    B0 = sysm.B.copy()
    sysm.B[:] = B0 * (1.0 + 1e-13 * rng.standard_normal(B0.shape))
    C2, e2, _ = fef.run_scf(sysm, 4)
    E2b, _ = fef.pair_energies(sysm, C2, e2)
    sysm.B[:] = B0
    assert np.max(np.abs(E2b - E2)) < 1e-11


def test_golden_config0_regression():
    """The oracle still reproduces the stored lattice-workload values."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "config0_e2.txt")
    rows = [l.split() for l in open(path) if not l.startswith("#")]
    sysm = fefgen.make_system(0)
    E0, _ = fef.pair_energies(sysm)
    C, e, _ = fef.run_scf(sysm, 3)
    E3, _ = fef.pair_energies(sysm, C, e)
    for k, r in enumerate(rows):
        assert (int(r[0]), int(r[1])) == (sysm.pair_x[k], sysm.pair_y[k])
        assert abs(float(r[2]) - E0[k]) <= 1e-13
        assert abs(float(r[3]) - E3[k]) <= 1e-12
