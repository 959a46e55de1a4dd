"""GPU parity: every entry point of the HIP library against the CPU oracle on
the same seeded inputs (element by element), plus properties that hold at any
size.  FP64 bar: 1e-9 Eh per pair energy."""
import math
import sys

import numpy as np
import pytest

import fefgen
from oracle import fef as ofef

pytestmark = pytest.mark.gpu

PREC = {"f64": 0, "f32": 1, "bf16x2": 2, "fp16x2": 3, "bf16x3": 4}
TOL_PAIR_F64 = 1e-9


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def ctx_for(sysm, **kw):
    import paper_1708_03377_amd as lib
    return lib.Context(sysm, **kw)


def ragged_system(seed=21):
    # odd ov (not multiples of 16), nocc = 1, nvir = 1, ov = 0 on either side,
    # a two-tile fragment (ov = 161), P = 6 (padded to 8)
    sizes = [(24, 5), (7, 3), (10, 1), (5, 4), (4, 4), (6, 0), (30, 7), (3, 1)]
    return fefgen.make_random_system(seed, sizes, naux=6)


def odd_system(seed=23):
    # odd nbf with an odd number of factor slices (P = 5): slice groups of
    # the half transform start at odd offsets of the coefficient pool, so
    # both its 16-byte copy and its element-wise fallback run
    sizes = [(7, 3), (5, 2), (9, 4), (3, 1), (24, 5)]
    return fefgen.make_random_system(seed, sizes, naux=5)


def two_class_system(seed=22):
    # a 300-wide (4-tile) solute of class 1 with P1 = 20 among P0 = 8 solvent fragments
    return fefgen.make_two_class_system(seed, (40, 10, 20),
                                        [(24, 5), (9, 2), (24, 5), (13, 6)], naux0=8)


# ---------------------------------------------------------------------------
def test_half_transform_matches_oracle(torch):
    for sysm in (ragged_system(), two_class_system(), odd_system()):
        _say("half transform", sysm.nfrag)
        ctx = ctx_for(sysm)
        bov = torch.zeros(max(ctx.sizes["bov"], 1), dtype=torch.float64, device="cuda")
        w = torch.zeros(max(ctx.sizes["w"], 1), dtype=torch.float64, device="cuda")
        ctx.half_transform(PREC["f64"], bov, w)
        torch.cuda.synchronize()
        bov = bov.cpu().numpy(); w = w.cpu().numpy()
        ob = 0; ow = 0
        P0 = int(sysm.naux_class[0])
        for f in range(sysm.nfrag):
            o = int(sysm.nocc[f]); n = int(sysm.nbf[f]); P = int(sysm.naux[f])
            ov = o * (n - o)
            ref = ofef.half_transform(sysm.B_of(f), sysm.C_of(f), o).reshape(P, ov)
            got = bov[ob:ob + P * ov].reshape(P, ov)
            np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)
            refw = sysm.G_of(int(sysm.cls[f])).T @ ref
            gotw = w[ow:ow + P0 * ov].reshape(P0, ov)
            np.testing.assert_allclose(gotw, refw, rtol=0, atol=1e-13)
            ob += P * ov; ow += P0 * ov


@pytest.mark.parametrize("which", ["ragged", "two_class", "config0", "odd"])
def test_pair_energies_f64(torch, which):
    sysm = {"ragged": ragged_system, "two_class": two_class_system,
            "config0": lambda: fefgen.make_system(0), "odd": odd_system}[which]()
    _say("pair energies f64", which, sysm.npair)
    ref, ref_tot = ofef.pair_energies(sysm)
    ctx = ctx_for(sysm)
    E2, tot = ctx.energies(PREC["f64"])
    torch.cuda.synchronize()
    E2 = E2.cpu().numpy(); tot = float(tot.cpu()[0])
    assert np.max(np.abs(E2 - ref)) <= TOL_PAIR_F64
    assert abs(tot - ref_tot) <= TOL_PAIR_F64 * max(1, sysm.npair) ** 0.5
    assert int(ctx.flags.cpu()[0]) == 0


def test_zero_width_pairs_are_zero(torch):
    sysm = ragged_system()
    ctx = ctx_for(sysm)
    E2, _ = ctx.energies(PREC["f64"])
    E2 = E2.cpu().numpy()
    ov = sysm.nocc * (sysm.nbf - sysm.nocc)
    zero = (ov[sysm.pair_x] == 0) | (ov[sysm.pair_y] == 0)
    assert zero.any()
    assert np.all(E2[zero] == 0.0)
    assert np.all(E2[~zero] < 0.0)


def test_empty_pair_list(torch):
    sysm = fefgen.make_random_system(3, [(6, 2), (5, 2)], naux=4)
    sysm.pair_x = sysm.pair_x[:0]; sysm.pair_y = sysm.pair_y[:0]
    sysm.pair_s = sysm.pair_s[:0]; sysm.pair_r = sysm.pair_r[:0]
    ctx = ctx_for(sysm)
    ctx.E2_total.fill_(123.0)
    _, tot = ctx.energies(PREC["f64"])
    assert float(tot.cpu()[0]) == 0.0


def test_coulomb_field_matches_oracle(torch):
    for sysm in (ragged_system(), two_class_system(), fefgen.make_system(0)):
        _say("field", sysm.nfrag)
        ctx = ctx_for(sysm)
        Dl = ofef.densities(sysm)
        D = torch.from_numpy(np.concatenate([d.ravel() for d in Dl])).cuda()
        J = torch.zeros_like(D)
        ctx.coulomb_field(D, J)
        J = J.cpu().numpy()
        ref = ofef.coulomb_field(sysm, Dl)
        oc = sysm.off_C
        for f in range(sysm.nfrag):
            np.testing.assert_allclose(J[oc[f]:oc[f + 1]], ref[f].ravel(), rtol=0,
                                       atol=1e-12 * max(1.0, np.max(np.abs(ref[f]))))


@pytest.mark.parametrize("which,niter", [("config0", 3), ("ragged", 2), ("two_class", 2)])
def test_scf_then_pair_energies(torch, which, niter):
    sysm = {"ragged": ragged_system, "two_class": two_class_system,
            "config0": lambda: fefgen.make_system(0)}[which]()
    _say("scf", which, niter)
    ctx = ctx_for(sysm)
    C, e = sysm.C.copy(), sysm.eps.copy()
    for it in range(niter):
        dmax = float(ctx.scf_step().cpu()[0])
        C, e, Dl, odmax, ok = ofef.scf_step(sysm, C, e)
        assert abs(dmax - odmax) <= 1e-10
        np.testing.assert_allclose(ctx.eps.cpu().numpy(), e, rtol=0, atol=1e-10)
        D = ctx.D.cpu().numpy()
        oc = sysm.off_C
        for f in range(sysm.nfrag):
            np.testing.assert_allclose(D[oc[f]:oc[f + 1]], Dl[f].ravel(), rtol=0, atol=1e-10)
    ref, ref_tot = ofef.pair_energies(sysm, C, e)
    E2, tot = ctx.energies(PREC["f64"])
    E2 = E2.cpu().numpy()
    assert np.max(np.abs(E2 - ref)) <= TOL_PAIR_F64


def test_bitwise_repeatable_and_order_invariant(torch):
    sysm = fefgen.make_system(0)
    ctx = ctx_for(sysm)
    a = ctx.energies(PREC["f64"])[0].cpu().numpy().copy()
    b = ctx.energies(PREC["f64"])[0].cpu().numpy().copy()
    assert np.array_equal(a, b)
    perm = np.random.default_rng(0).permutation(sysm.npair)
    s2 = fefgen.make_system(0)
    s2.pair_x, s2.pair_y = s2.pair_y[perm].copy(), s2.pair_x[perm].copy()  # also swap x<->y
    s2.pair_s = s2.pair_s[perm].copy(); s2.pair_r = s2.pair_r[perm].copy()
    c = ctx_for(s2).energies(PREC["f64"])[0].cpu().numpy()
    np.testing.assert_allclose(c, a[perm], rtol=1e-13, atol=0)


def test_gap_and_nonfinite_flags(torch):
    sysm = fefgen.make_random_system(4, [(6, 2), (5, 2), (6, 3)], naux=4)
    o = sysm.off_eps
    sysm.eps[o[1]:o[2]] = [-0.5, 0.2, 0.1, 0.4, 0.9]  # LUMO below HOMO on fragment 1
    ctx = ctx_for(sysm)
    ctx.energies(PREC["f64"])
    assert int(ctx.flags.cpu()[0]) & 1
    sysm2 = fefgen.make_random_system(4, [(6, 2), (5, 2), (6, 3)], naux=4)
    sysm2.B[5] = np.nan
    ctx2 = ctx_for(sysm2)
    ctx2.energies(PREC["f64"])
    assert int(ctx2.flags.cpu()[0]) & 2


@pytest.mark.parametrize("prec,tol_pair", [("f32", 1e-5), ("bf16x2", 1e-5), ("fp16x2", 1e-6),
                                           ("bf16x3", 1e-6)])
def test_reduced_precision_config0(torch, prec, tol_pair):
    sysm = fefgen.make_system(0)
    ref, ref_tot = ofef.pair_energies(sysm)
    ctx = ctx_for(sysm)
    E2, tot = ctx.energies(PREC[prec])
    E2 = E2.cpu().numpy(); tot = float(tot.cpu()[0])
    err = np.max(np.abs(E2 - ref))
    _say(prec, "max pair err", err, "total err", tot - ref_tot)
    assert err <= tol_pair


@pytest.mark.parametrize("prec,tiles", [("f64", [(1, 1), (1, 7), (2, 1), (2, 5)]),
                                        ("f32", [(1, 3), (2, 2)]),
                                        ("bf16x2", [(2, 2), (2, 5), (4, 64)]),
                                        ("fp16x2", [(2, 1), (4, 3)]),
                                        ("bf16x3", [(2, 1), (2, 64), (4, 3)])])
def test_tilings_agree(torch, prec, tiles):
    """Every pair-kernel tiling gives the same pair energies (up to in-tile
    summation order), on ragged and two-class systems."""
    import paper_1708_03377_amd as lib
    for sysm in (ragged_system(), two_class_system()):
        ref, _ = ofef.pair_energies(sysm)
        ctx = ctx_for(sysm)
        base = ctx.energies(PREC[prec])[0].cpu().numpy().copy()
        tol = TOL_PAIR_F64 if prec == "f64" else 1e-5
        assert np.max(np.abs(base - ref)) <= tol
        for xb, yc in tiles:
            _say(prec, "tiles", xb, yc)
            lib.fef_plan_set_tiles(ctx.plan, PREC[prec], xb, yc)
            assert lib.fef_plan_get_tiles(ctx.plan, PREC[prec]) == (xb, yc)
            got = ctx.pair_energies(PREC[prec])[0].cpu().numpy()
            np.testing.assert_allclose(got, base, rtol=1e-12 if prec == "f64" else 1e-6, atol=0)


@pytest.mark.parametrize("prec", ["bf16x2", "fp16x2"])
def test_split_kernels_bitwise_on_water_width(torch, prec):
    """Water fragments (P = 72): the pipelined two-unit kernel (xb = 2) and
    the four-unit kernel (xb = 4) give bitwise the same pair energies (same
    products, same tile and half sums in the same order), and both match
    the oracle."""
    import paper_1708_03377_amd as lib
    sysm = fefgen.make_system(0)
    ref, _ = ofef.pair_energies(sysm)
    ctx = ctx_for(sysm)
    ctx.half_transform(PREC[prec])
    out = {}
    for xb, yc in ((2, 1), (2, 16), (4, 3), (4, 16)):
        lib.fef_plan_set_tiles(ctx.plan, PREC[prec], xb, yc)
        out[(xb, yc)] = ctx.pair_energies(PREC[prec])[0].cpu().numpy().copy()
    base = out[(4, 16)]
    assert np.max(np.abs(base - ref)) <= 1e-6
    for k, v in out.items():
        assert np.array_equal(v, base), k


def test_graph_replays_match_eager(torch):
    """A captured FEF pass replays bitwise like the eager calls, also with
    eager work and synchronisations between replays.  The packed coefficient
    pool is poisoned before each replay: the pass packs B itself (in its
    first SCF step) before anything reads the pool."""
    import paper_1708_03377_amd as lib
    for sysm, prec in ((fefgen.make_system(0), "f64"), (two_class_system(), "bf16x2"),
                       (two_class_system(), "bf16x3")):
        ctx = ctx_for(sysm)
        p = PREC[prec]
        ctx.reset_orbitals(); ctx.scf(3)
        E_eager = ctx.energies(p)[0].cpu().numpy().copy()
        C_eager = ctx.C.cpu().numpy().copy()
        g = ctx.graph(3, p)
        for rep in range(3):
            ctx.E2_pair.fill_(0.0); ctx.C.fill_(0.0)
            ctx.packed_coefficients().fill_(float("nan"))
            ctx.launch(g)
            torch.cuda.synchronize()
            assert np.array_equal(ctx.E2_pair[:ctx.npair].cpu().numpy(), E_eager), rep
            assert np.array_equal(ctx.C.cpu().numpy(), C_eager), rep
            ctx.pair_energies(p)  # eager work between replays
            torch.cuda.synchronize()


def test_autotune_keeps_results(torch):
    import paper_1708_03377_amd as lib
    sysm = fefgen.make_system(0)
    ref, _ = ofef.pair_energies(sysm)
    ctx = ctx_for(sysm)
    for prec in ("f64", "fp16x2"):
        xb, yc, us = ctx.autotune(PREC[prec], reps=2)
        assert lib.fef_plan_get_tiles(ctx.plan, PREC[prec]) == (xb, yc)
        assert us > 0
        E2 = ctx.pair_energies(PREC[prec])[0].cpu().numpy()
        assert np.max(np.abs(E2 - ref)) <= (TOL_PAIR_F64 if prec == "f64" else 1e-6)


def test_autotune_cache_file(torch, tmp_path):
    """fef_autotune_cached: a miss tunes and writes the entry, a hit applies
    the cached tiling without timing and gives bitwise the same energies;
    another system adds a second entry; lines that are not entries are
    skipped; an unwritable path reports FEF_E_IO with the tiling in place."""
    import json

    import paper_1708_03377_amd as lib
    from paper_1708_03377_amd import _fef as F
    _say("autotune cache: workload 0 and the ragged system, fp16x2")
    path = str(tmp_path / "tiles.json")
    p = PREC["fp16x2"]
    sysm = fefgen.make_system(0)
    ctx = ctx_for(sysm)
    xb, yc, us, hit = ctx.autotune_cached(p, path, reps=2)
    assert not hit and us > 0
    assert lib.fef_plan_get_tiles(ctx.plan, p) == (xb, yc)
    E_tuned = ctx.pair_energies(p)[0].cpu().numpy().copy()
    cache = json.load(open(path))
    assert len(cache) == 1
    key = next(iter(cache))
    assert key.split("/")[1] == "fp16x2" and cache[key]["xb"] == xb and cache[key]["yc"] == yc
    # a new context on the same work: served from the cache, same tiles and energies
    ctx2 = ctx_for(sysm)
    xb2, yc2, us2, hit2 = ctx2.autotune_cached(p, path, reps=2)
    assert hit2 and (xb2, yc2) == (xb, yc) and us2 == pytest.approx(us, rel=1e-3, abs=0.1)
    assert lib.fef_plan_get_tiles(ctx2.plan, p) == (xb, yc)
    assert np.array_equal(ctx2.pair_energies(p)[0].cpu().numpy(), E_tuned)
    # other work: a miss, and the file keeps both entries (plus a stray line)
    with open(path, "a") as f:
        f.write("not an entry\n")
    ctx3 = ctx_for(ragged_system())
    _, _, _, hit3 = ctx3.autotune_cached(p, path, reps=2)
    assert not hit3
    assert len(json.load(open(path))) == 2
    # an unwritable cache path
    bad = str(tmp_path / "no_such_dir" / "tiles.json")
    with pytest.raises(F.FefError) as ei:
        ctx3.autotune_cached(p, bad, reps=1)
    assert ei.value.status == F.FEF_E_IO


@pytest.mark.parametrize("which,niter", [("config0", 3), ("ragged", 2), ("two_class", 2)])
def test_packed_scf_matches_oracle(torch, which, niter):
    """SCF steps on the packed (upper-triangle) coefficients against the
    oracle: orbital energies and densities within 1e-10 at every step."""
    sysm = {"ragged": ragged_system, "two_class": two_class_system,
            "config0": lambda: fefgen.make_system(0)}[which]()
    ctx = ctx_for(sysm)
    Bp = ctx.packed_coefficients().cpu().numpy()
    # the packed pool is the upper triangle of every slice, fragments in order
    o = 0
    for f in range(sysm.nfrag):
        n = int(sysm.nbf[f]); iu = np.triu_indices(n)
        ref = np.stack([b[iu] for b in sysm.B_of(f)]).ravel()
        np.testing.assert_array_equal(Bp[o:o + ref.size], ref)
        o += ref.size
    C, e = sysm.C.copy(), sysm.eps.copy()
    for it in range(niter):
        dmax = float(ctx.scf_step_packed().cpu()[0])
        C, e, Dl, odmax, ok = ofef.scf_step(sysm, C, e)
        assert abs(dmax - odmax) <= 1e-10
        np.testing.assert_allclose(ctx.eps.cpu().numpy(), e, rtol=0, atol=1e-10)
        D = ctx.D.cpu().numpy()
        oc = sysm.off_C
        for f in range(sysm.nfrag):
            np.testing.assert_allclose(D[oc[f]:oc[f + 1]], Dl[f].ravel(), rtol=0, atol=1e-10)


@pytest.mark.parametrize("solute", [(49, 10, 8), (64, 12, 24), (65, 13, 24), (97, 20, 24),
                                    (150, 29, 24)])
def test_scf_large_fragment(torch, solute):
    """Fragments above 48 basis functions take the large-matrix eigensolver
    (Householder tridiagonalisation, multisection, inverse iteration,
    back-transformation); the sizes cover both register layouts (up to 96
    and up to 152 columns) with ragged padding.  Orbital energies and
    densities against the oracle over two SCF steps, for both the full and
    the packed coefficient paths, then the pair energies."""
    sysm = fefgen.make_two_class_system(31, solute, [(24, 5), (9, 2), (24, 5), (13, 6)], naux0=8)
    for packed in (False, True):
        ctx = ctx_for(sysm)
        C, e = sysm.C.copy(), sysm.eps.copy()
        for it in range(2):
            dmax = float((ctx.scf_step_packed() if packed else ctx.scf_step()).cpu()[0])
            C, e, Dl, odmax, ok = ofef.scf_step(sysm, C, e)
            assert abs(dmax - odmax) <= 1e-10
            np.testing.assert_allclose(ctx.eps.cpu().numpy(), e, rtol=0, atol=1e-10)
            D = ctx.D.cpu().numpy()
            oc = sysm.off_C
            for f in range(sysm.nfrag):
                np.testing.assert_allclose(D[oc[f]:oc[f + 1]], Dl[f].ravel(), rtol=0, atol=1e-10)
        ref, _ = ofef.pair_energies(sysm, C, e)
        E2, _ = ctx.energies(PREC["f64"])
        assert np.max(np.abs(E2.cpu().numpy() - ref)) <= TOL_PAIR_F64


@pytest.mark.parametrize("naux", [40, 76])
@pytest.mark.parametrize("prec,tol", [("f64", TOL_PAIR_F64), ("f32", 1e-5)])
def test_pair_energies_uncommon_rank(torch, naux, prec, tol):
    """Factor ranks other than 8 and 72 take the plain kernels' generic
    contraction length (20 k steps of 4): the rows past the padded rank are
    read as zeros, so the energies match the oracle."""
    sizes = [(24, 5), (13, 4), (24, 5), (9, 2), (30, 7), (24, 5), (7, 3)]
    sysm = fefgen.make_random_system(41 + naux, sizes, naux=naux)
    _say("pair energies", prec, "P0 =", naux, sysm.npair)
    ref, ref_tot = ofef.pair_energies(sysm)
    ctx = ctx_for(sysm)
    for _ in range(2):  # a second call finds the first call's data in LDS
        E2, tot = ctx.energies(PREC[prec])
        torch.cuda.synchronize()
        E2 = E2.cpu().numpy()
        assert np.all(np.isfinite(E2))
        assert np.max(np.abs(E2 - ref)) <= tol
        assert int(ctx.flags.cpu()[0]) == 0
