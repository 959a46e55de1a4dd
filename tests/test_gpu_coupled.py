"""GPU parity of the W^[0]-coupled dimer doubles (fef_coupled_pair_energies)
against the CPU oracle (oracle/coupled.py) on the same seeded inputs.

Bar: the solve runs to ||r|| <= 1e-14 ||v|| on both sides, so the pair
energies agree to rounding: 1e-11 relative (1e-13 Eh absolute floor) per
pair, and the totals likewise.  maxit = 0 must give the uncoupled pair
energy -4 sum v^2 / D exactly as the oracle's plain pair energy."""
import sys

import numpy as np
import pytest

import fefgen
from oracle import coupled as oc
from oracle import fef as ofef

pytestmark = pytest.mark.gpu

REL = 1e-11
ABS = 1e-13


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def ctx_for(sysm):
    import paper_1708_03377_amd as lib
    return lib.Context(sysm)


def ragged_system(seed=21):
    # odd ov, nocc = 1, nvir = 1, ov = 0 on either side, a 161-wide fragment
    sizes = [(24, 5), (7, 3), (10, 1), (5, 4), (4, 4), (6, 0), (30, 7), (3, 1)]
    return fefgen.make_random_system(seed, sizes, naux=6)


def two_class_system(seed=22):
    # a class-1 solute (nbf 40, nocc 10, P1 = 20) among P0 = 8 solvent
    # fragments: its pairs exceed the LDS of a workgroup (slot-resident path)
    return fefgen.make_two_class_system(seed, (40, 10, 20),
                                        [(24, 5), (9, 2), (24, 5), (13, 6)], naux0=8)


def _compare(E_gpu, E_ref, what):
    err = np.abs(E_gpu - E_ref)
    bound = REL * np.abs(E_ref) + ABS
    worst = int(np.argmax(err - bound)) if len(err) else 0
    _say(what, "pairs", len(err), "max abs err", float(err.max()) if len(err) else 0.0)
    assert np.all(err <= bound), (what, worst, E_gpu[worst], E_ref[worst])


def test_coupled_workload0_matches_oracle(torch):
    _say("coupled: workload 0 (8 waters)")
    sysm = fefgen.make_system(0)
    ctx = ctx_for(sysm)
    E, tot, it = ctx.coupled_pair_energies()
    torch.cuda.synchronize()
    E = E.cpu().numpy()
    E_ref, tot_ref = oc.coupled_pair_energies(sysm)
    _compare(E, E_ref, "workload0")
    assert abs(float(tot.item()) - tot_ref) <= REL * abs(tot_ref)
    it = it.cpu().numpy()
    assert np.all(it >= 1) and np.all(it <= 60)
    assert int(ctx.flags.item()) == 0
    # the coupling really changes the energies (not the plain ones)
    E0, _ = ofef.pair_energies(sysm)
    assert np.max(np.abs(E - E0) / np.abs(E0)) > 1e-6


def test_coupled_maxit0_is_the_plain_pair_energy(torch):
    _say("coupled: maxit 0 on workload 0")
    sysm = fefgen.make_system(0)
    ctx = ctx_for(sysm)
    E, tot, it = ctx.coupled_pair_energies(maxit=0)
    torch.cuda.synchronize()
    E0, tot0 = ofef.pair_energies(sysm)
    _compare(E.cpu().numpy(), E0, "maxit0")
    assert np.all(it.cpu().numpy() == 0)
    # every pair stopped at the limit without meeting the tolerance
    import paper_1708_03377_amd._fef as F
    assert int(ctx.flags.item()) & F.FEF_FLAG_NOCONV


@pytest.mark.parametrize("which", ["ragged", "two_class"])
def test_coupled_ragged_and_two_class_match_oracle(torch, which):
    sysm = ragged_system() if which == "ragged" else two_class_system()
    _say("coupled:", which, "npair", sysm.npair, "nbf", list(sysm.nbf), "nocc", list(sysm.nocc))
    ctx = ctx_for(sysm)
    E, tot, it = ctx.coupled_pair_energies()
    torch.cuda.synchronize()
    E = E.cpu().numpy()
    E_ref, tot_ref = oc.coupled_pair_energies(sysm)
    _compare(E, E_ref, which)
    assert abs(float(tot.item()) - tot_ref) <= REL * abs(tot_ref) + ABS
    assert int(ctx.flags.item()) == 0


def test_coupled_bitwise_repeatable(torch):
    _say("coupled: repeatability on the two-class system")
    sysm = two_class_system()
    ctx = ctx_for(sysm)
    E1, t1, i1 = [x.clone() for x in ctx.coupled_pair_energies()]
    E2, t2, i2 = ctx.coupled_pair_energies()
    torch.cuda.synchronize()
    assert torch.equal(E1, E2) and torch.equal(t1, t2) and torch.equal(i1, i2)


def test_coupled_thousand_waters_sampled_pairs(torch):
    """Workload 1 (1000 waters, ~1.2e5 pairs) in one call; 24 pairs spread
    over the list (nearest and farthest included) against the oracle."""
    _say("coupled: workload 1 (1000 waters), sampled pairs")
    sysm = fefgen.make_system(1)
    ctx = ctx_for(sysm)
    E, tot, it = ctx.coupled_pair_energies()
    torch.cuda.synchronize()
    E = E.cpu().numpy()
    assert int(ctx.flags.item()) == 0 and np.all(np.isfinite(E))
    R = 1.0 / np.asarray(sysm.pair_s)
    idx = sorted(set(np.linspace(0, sysm.npair - 1, 22).astype(int).tolist() +
                     [int(np.argmin(R)), int(np.argmax(R))]))
    E_ref, _ = oc.coupled_pair_energies(sysm, pairs=idx)
    _compare(E[idx], E_ref, "workload1 sample")
    # the total is the fixed-order sum of the pair energies
    assert float(tot.item()) == pytest.approx(float(np.sum(E)), rel=1e-12)


def test_coupled_nucleobase_box_sampled_pairs(torch):
    """Workload 2 (one nucleobase among 2000 waters, 2.4e5 pairs) in one call:
    the 231 nucleobase-water pairs take the slot-resident path (their p and
    W p exceed a workgroup's LDS).  The closest nucleobase-water pair and
    three water pairs against the oracle."""
    _say("coupled: workload 2 (nucleobase + 2000 waters), sampled pairs")
    sysm = fefgen.make_system(2)
    ctx = ctx_for(sysm)
    E, tot, it = ctx.coupled_pair_energies()
    torch.cuda.synchronize()
    E = E.cpu().numpy()
    assert int(ctx.flags.item()) == 0 and np.all(np.isfinite(E))
    nb = np.nonzero((sysm.cls[sysm.pair_x] != 0) | (sysm.cls[sysm.pair_y] != 0))[0]
    ww = np.nonzero((sysm.cls[sysm.pair_x] == 0) & (sysm.cls[sysm.pair_y] == 0))[0]
    R = 1.0 / np.asarray(sysm.pair_s)
    idx = [int(nb[np.argmin(R[nb])])] + [int(k) for k in ww[[0, len(ww) // 2, len(ww) - 1]]]
    E_ref, _ = oc.coupled_pair_energies(sysm, pairs=idx)
    _compare(E[idx], E_ref, "workload2 sample")
