"""Pins of the monomer-energy oracle (oracle/monomer.py, Eq. EM2).

The closed-shell formula is pinned against two constructions that share
none of its index bookkeeping: the second-order Rayleigh-Schroedinger
energy summed over explicit doubly excited determinants in the
occupation-number basis (creation and annihilation operators with their
phases, the intra-fragment Coulomb operator built from the factored AO
tensor by Kronecker products), and the spin-orbital energy
(1/4) sum |<ij||ab>|^2 / D.  Further: the two-electron special case, the
sign of the energy, its quadratic scaling with the coupling, and the
class restriction.
"""
import itertools

import numpy as np
import pytest

import fefgen
from oracle import monomer as om


def fragment(seed, nbf, nocc, naux):
    s = fefgen.make_random_system(seed, [(nbf, nocc)], naux=naux)
    return s.B_of(0), s.C_of(0), s.eps_of(0), s.G_of(0)


def mo_tensor_kron(B, C, G):
    """(pq|rs) as a (pq, rs) matrix: the AO tensor as a sum over P, Q of
    outer products of the B slices, then (C x C)^T I (C x C)."""
    n = C.shape[0]
    I = np.zeros((n * n, n * n))
    for P in range(B.shape[0]):
        for Q in range(B.shape[0]):
            I += G[P, Q] * np.outer(B[P].ravel(), B[Q].ravel())
    K = np.kron(C, C)
    return (K.T @ I @ K).reshape(n, n, n, n)


def _apply(op, det):
    """Apply (create?, spin-orbital) operators right to left to one
    determinant (bitmask); returns (sign, det) or None."""
    sign = 1.0
    for create, k in reversed(op):
        occ = (det >> k) & 1
        if create == occ:
            return None
        if bin(det & ((1 << k) - 1)).count("1") % 2:
            sign = -sign
        det ^= 1 << k
    return sign, det


def determinant_second_order(B, C, eps, nocc, G):
    """sum over doubly excited D of |<D|W|0>|^2 / (E_0 - E_D), with
    W = 1/2 sum (pq|rs) a+_{p s1} a+_{r s2} a_{s s2} a_{q s1}."""
    n = C.shape[0]
    I = mo_tensor_kron(B, C, G)
    ref = (1 << (2 * nocc)) - 1
    amp = {}
    for p, q, r, s in itertools.product(range(n), repeat=4):
        v = I[p, q, r, s]
        if v == 0.0:
            continue
        for s1, s2 in itertools.product((0, 1), repeat=2):
            op = [(1, 2 * p + s1), (1, 2 * r + s2), (0, 2 * s + s2), (0, 2 * q + s1)]
            res = _apply(op, ref)
            if res is None:
                continue
            sg, d = res
            amp[d] = amp.get(d, 0.0) + 0.5 * v * sg
    e_so = np.repeat(eps, 2)

    def energy(det):
        return sum(e_so[k] for k in range(2 * n) if (det >> k) & 1)

    E0 = energy(ref)
    E2 = 0.0
    for d, c in amp.items():
        if bin(d & ~ref).count("1") == 2:            # doubles only
            E2 += c * c / (E0 - energy(d))
    return E2


def spin_orbital_energy(B, C, eps, nocc, G):
    n = C.shape[0]
    I = mo_tensor_kron(B, C, G)
    so = [(p, sp) for p in range(n) for sp in (0, 1)]

    def phys(P, Q, R, S):  # <PQ|RS> = (pr|qs) delta(spins)
        (p, sp), (q, sq), (r, sr), (s, ss) = so[P], so[Q], so[R], so[S]
        return I[p, r, q, s] if (sp == sr and sq == ss) else 0.0

    occ = range(2 * nocc)
    vir = range(2 * nocc, 2 * n)
    e = np.repeat(eps, 2)
    E = 0.0
    for i, j in itertools.product(occ, repeat=2):
        for a, b in itertools.product(vir, repeat=2):
            anti = phys(i, j, a, b) - phys(i, j, b, a)
            E += anti * anti / (e[i] + e[j] - e[a] - e[b])
    return 0.25 * E


@pytest.mark.parametrize("seed,nbf,nocc,naux", [(1, 4, 2, 3), (2, 5, 2, 4), (3, 5, 3, 2)])
def test_matches_second_order_over_determinants(seed, nbf, nocc, naux):
    B, C, eps, G = fragment(seed, nbf, nocc, naux)
    ref = determinant_second_order(B, C, eps, nocc, G)
    got = om.monomer_energy(B, C, eps, nocc, G)
    assert ref < 0.0
    assert got == pytest.approx(ref, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("seed,nbf,nocc,naux", [(4, 6, 2, 3), (5, 6, 4, 5)])
def test_matches_spin_orbital_energy(seed, nbf, nocc, naux):
    B, C, eps, G = fragment(seed, nbf, nocc, naux)
    ref = spin_orbital_energy(B, C, eps, nocc, G)
    assert om.monomer_energy(B, C, eps, nocc, G) == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_two_electron_case():
    """One doubly occupied orbital: no exchange survives the spin sum, so
    E = sum_ab (ia|ib)^2 / (2 eps_i - eps_a - eps_b)."""
    B, C, eps, G = fragment(6, 5, 1, 3)
    I = mo_tensor_kron(B, C, G)
    ref = sum(I[0, a, 0, b] ** 2 / (2 * eps[0] - eps[a] - eps[b])
              for a in range(1, 5) for b in range(1, 5))
    assert om.monomer_energy(B, C, eps, 1, G) == pytest.approx(ref, rel=1e-12)


def test_sign_and_quadratic_scaling_in_the_coupling():
    for seed in range(7, 12):
        B, C, eps, G = fragment(seed, 6, 2, 4)
        E = om.monomer_energy(B, C, eps, 2, G)
        assert E < 0.0
        assert om.monomer_energy(B, C, eps, 2, 3.0 * G) == pytest.approx(9.0 * E, rel=1e-12)


def test_energies_of_workload0_and_class_restriction():
    s = fefgen.make_system(0)
    E, tot = om.monomer_energies(s)
    assert E.shape == (s.nfrag,) and np.all(E < 0.0)
    assert tot == pytest.approx(float(np.sum(E)), rel=1e-14)
    one = om.monomer_energy(s.B_of(3), s.C_of(3), s.eps_of(3), int(s.nocc[3]), s.G_of(0))
    assert E[3] == one
    two = fefgen.make_two_class_system(2, (4, 2, 3), [(3, 1), (4, 2)], naux0=3)
    with pytest.raises(ValueError):
        om.monomer_energies(two)
    e12, _ = om.monomer_energies(two, frags=[1, 2])
    assert e12.shape == (2,)
