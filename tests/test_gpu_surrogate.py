"""GPU tests of the distant-pair surrogate and of the masked exact pair
energies, through the C ABI, against the CPU oracle (oracle/mlp.py,
oracle/fef.py) on the same seeded inputs."""
import math
import sys

import numpy as np
import pytest

import fefgen
from oracle import fef as ofef
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

PREC = {"f64": 0, "f32": 1, "bf16x2": 2, "fp16x2": 3}
BOHR = fefgen.BOHR_PER_ANGSTROM


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def lib():
    import paper_1708_03377_amd as m
    return m


def bf16_round(a):
    """Round to nearest even BF16 (kept in float64)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def moments(sysm, Dl):
    return [np.einsum("pmn,mn->p", sysm.B_of(f), Dl[f]) for f in range(sysm.nfrag)]


def small_box(seed, n_water=300, cutoff=10.0):
    return fefgen.surrogate_training_box(seed, n_water=n_water, cutoff=cutoff)


# ---------------------------------------------------------------------------
def test_coupling_modes(torch):
    sysm = fefgen.make_system(0)
    ctx = lib().Context(sysm)
    Q = ctx.coupling_modes().cpu().numpy().reshape(4, -1)
    w, q = np.linalg.eigh(sysm.G_of(0))
    top = q[:, ::-1][:, :4].T
    for k in range(4):
        assert abs(abs(Q[k] @ top[k]) - 1.0) <= 1e-10, k
    np.testing.assert_allclose(Q @ Q.T, np.eye(4), atol=1e-12)


@pytest.mark.parametrize("which", ["config0", "two_class"])
def test_invariants_match_oracle(torch, which):
    if which == "config0":
        sysm = fefgen.make_system(0)
    else:
        sysm = fefgen.make_two_class_system(22, (40, 10, 20), [(24, 5), (9, 2), (24, 5)], naux0=8)
    ctx = lib().Context(sysm)
    C, e = sysm.C.copy(), sysm.eps.copy()
    for _ in range(2):
        ctx.scf_step()
        C, e, Dl, _, _ = ofef.scf_step(sysm, C, e)
    U = ctx.invariants().cpu().numpy().reshape(sysm.nfrag, 8)
    d = moments(sysm, Dl)
    G = sysm.G_of(0)
    for f in range(sysm.nfrag):
        if sysm.cls[f] != 0:
            assert np.all(np.isnan(U[f]))
            continue
        ref = omlp.fragment_invariants(d[f], G)
        np.testing.assert_allclose(U[f], ref, rtol=1e-10, atol=1e-14)


def test_pair_features_and_targets(torch):
    sysm = fefgen.make_system(0)
    ctx = lib().Context(sysm)
    ctx.scf(2)
    E2, _ = ctx.energies(PREC["f64"])
    U = ctx.invariants()
    X, T = ctx.pair_features(U, with_targets=True)
    X = X.cpu().numpy(); T = T.cpu().numpy()
    Un = U.cpu().numpy().reshape(sysm.nfrag, 8)
    E2 = E2.cpu().numpy()
    for k in range(sysm.npair):
        x, y = int(sysm.pair_x[k]), int(sysm.pair_y[k])
        R = 1.0 / sysm.pair_s[k]
        ref = omlp.pair_features(R, Un[x], Un[y])
        np.testing.assert_allclose(X[k], ref.astype(np.float32), rtol=1e-6)
        assert T[k] == pytest.approx(E2[k] * R * R, rel=1e-6)
    # a subset through an index list
    idx = torch.tensor([5, 0, 27], dtype=torch.int32, device="cuda")
    Xs, _ = ctx.pair_features(U, idx)
    np.testing.assert_array_equal(Xs.cpu().numpy(), X[[5, 0, 27]])


def _ensemble_with_stats(torch, n=600, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 17)).astype(np.float32) * 3 + 1
    T = rng.standard_normal(n).astype(np.float32)
    ens = lib().Ensemble(nmember=5, seed=seed)
    Xd = torch.from_numpy(X).cuda(); Td = torch.from_numpy(T).cuda()
    ens.fit_stats(Xd, Td)
    return ens, X, T, Xd, Td


def _member_params(ens, m):
    P = ens.P.cpu().numpy().reshape(ens.nmember, -1)[m]
    return {k: bf16_round(v) for k, v in fefgen.mlp_unpack(P.astype(np.float64)).items()}


def test_column_stats(torch):
    ens, X, T, _, _ = _ensemble_with_stats(torch)
    st = ens.stats.cpu().numpy()
    np.testing.assert_allclose(st[:17], X.astype(np.float64).mean(0), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(st[17:34], 1.0 / X.astype(np.float64).std(0), rtol=1e-6)
    assert st[34] == pytest.approx(T.astype(np.float64).mean(), abs=1e-6)
    assert st[35] == pytest.approx(T.astype(np.float64).std(), rel=1e-6)


def test_mlp_forward_matches_oracle(torch):
    """MFMA inference against the oracle network at the BF16 weights: within
    1e-2 of the plain oracle forward (inputs and hidden activations are BF16
    on the MFMA path) and within 2e-3 of the oracle with those two roundings
    applied."""
    ens, X, T, Xd, Td = _ensemble_with_stats(torch)
    st = ens.stats.cpu().numpy().astype(np.float64)
    Y = ens.forward(Xd).cpu().numpy()
    Xs = ((X - st[:17].astype(np.float32)) * st[17:34].astype(np.float32)).astype(np.float64)
    for m in range(ens.nmember):
        p = _member_params(ens, m)
        ref, _ = omlp.forward(p, Xs)
        assert np.max(np.abs(Y[m] - ref)) <= 1e-2 * (1 + np.max(np.abs(ref)))
        xb = bf16_round(Xs)
        h0 = bf16_round(omlp.silu(xb @ p["W0"].T + p["b0"]))
        h1 = omlp.silu(h0 @ p["W1"].T + p["b1"])
        ref2 = (h1 @ p["W2"].T + p["b2"])[:, 0]
        err = np.max(np.abs(Y[m] - ref2))
        _say("member", m, "max |dY| vs oracle", np.max(np.abs(Y[m] - ref)), "vs rounded", err)
        assert err <= 2e-3 * (1 + np.max(np.abs(ref2)))


def test_mlp_gradients_match_oracle(torch):
    """Training gradients (FP32, BF16 weights) against the oracle's FP64
    backward at the same BF16 weights and standardised inputs: relative 1e-3
    on each parameter block's norm."""
    ens, X, T, Xd, Td = _ensemble_with_stats(torch, n=300)
    nb = 200
    rng = np.random.default_rng(4)
    idx = np.stack([rng.permutation(300)[:nb] for _ in range(ens.nmember)]).astype(np.int32)
    grad = torch.zeros_like(ens.P)
    P_before = ens.P.clone()
    ens.train_step(Xd, Td, torch.from_numpy(idx).cuda(), nb, 1e-3, grad=grad, update=False)
    assert torch.equal(P_before, ens.P)
    g = grad.cpu().numpy().reshape(ens.nmember, -1)
    st = ens.stats.cpu().numpy()
    for m in range(ens.nmember):
        p = _member_params(ens, m)
        Xs = ((X[idx[m]] - st[:17]) * st[17:34]).astype(np.float64)
        ts = ((T[idx[m]] - st[34]) / st[35]).astype(np.float64)
        ref = omlp.backward(p, Xs, ts)
        got = fefgen.mlp_unpack(g[m].astype(np.float64))
        for k in ref:
            a, b = got[k].ravel(), ref[k].ravel()
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            assert rel <= 1e-3, (m, k, rel)
        loss = float(ens.loss.cpu()[m])
        assert loss == pytest.approx(omlp.loss(p, Xs, ts), rel=1e-4)


def test_adam_step_matches_oracle(torch):
    ens, X, T, Xd, Td = _ensemble_with_stats(torch, n=256)
    nb = 128
    idx = np.tile(np.arange(nb, dtype=np.int32), (ens.nmember, 1))
    P0 = ens.P.cpu().numpy().astype(np.float64).reshape(ens.nmember, -1)
    grad = torch.zeros_like(ens.P)
    lr = 3e-3
    for t in (1, 2):
        Pb = ens.P.cpu().numpy().astype(np.float64).reshape(ens.nmember, -1)
        Mb = ens.M.cpu().numpy().astype(np.float64).reshape(ens.nmember, -1)
        Vb = ens.V.cpu().numpy().astype(np.float64).reshape(ens.nmember, -1)
        ens.train_step(Xd, Td, torch.from_numpy(idx).cuda(), nb, lr, grad=grad)
        g = grad.cpu().numpy().astype(np.float64).reshape(ens.nmember, -1)
        Pa = ens.P.cpu().numpy().astype(np.float64).reshape(ens.nmember, -1)
        n = fefgen.MLP_STRIDE
        p = {"w": Pb[:, :18945].copy()}
        mm = {"w": Mb[:, :18945].copy()}
        vv = {"w": Vb[:, :18945].copy()}
        omlp.adam_step(p, {"w": g[:, :18945]}, mm, vv, t, lr=lr)
        # the masters are FP32: |P| < 0.25 has an ulp of 1.5e-8
        np.testing.assert_allclose(Pa[:, :18945], p["w"], rtol=2e-6, atol=3e-8)
    W = ens.W.cpu().numpy().view(np.uint16).astype(np.uint32)
    np.testing.assert_array_equal((W << 16).view(np.float32),
                                  bf16_round(ens.P.cpu().numpy()).astype(np.float32))
    assert not np.allclose(P0, Pa)


def _dataset(torch, ctx, r_min_bohr):
    ctx.reset_orbitals(); ctx.scf(10)
    ctx.energies(PREC["f64"])
    U = ctx.invariants()
    far = np.nonzero(1.0 / ctx.system.pair_s >= r_min_bohr)[0].astype(np.int32)
    idx = torch.from_numpy(far).cuda()
    X, T = ctx.pair_features(U, idx, with_targets=True)
    return U, X.clone(), T.clone(), far


def test_training_learns_held_out(torch):
    """The GPU training kernels learn a target that is a smooth function of
    the 17 inputs: held-out error far below the target's variance, for every
    member, and the ensemble mean at least as good as the average member."""
    rng = np.random.default_rng(11)
    n = 24000
    X = rng.standard_normal((n, 17)).astype(np.float32) * 2 + 5
    z = (X - 5) / 2
    T = (np.sin(z[:, 0]) + 0.5 * z[:, 1] * z[:, 2] + 0.3 * z[:, 3] ** 2 - 0.2 * z[:, 4]
         ).astype(np.float32)
    tr, te = slice(0, 20000), slice(20000, n)
    Xd = torch.from_numpy(X[tr].copy()).cuda(); Td = torch.from_numpy(T[tr].copy()).cuda()
    ens = lib().Ensemble(nmember=5, seed=1)
    ens.fit_stats(Xd, Td)
    hist = ens.train(Xd, Td, epochs=25, nb=256, lr=2e-3, lr_final=2e-4)
    _say("train loss per epoch", [round(h, 4) for h in hist[::4]], hist[-1])
    assert hist[-1] < 0.2 * hist[0]
    Y = ens.forward(torch.from_numpy(X[te].copy()).cuda()).cpu().numpy()
    st = ens.stats.cpu().numpy()
    t = (T[te] - st[34]) / st[35]
    per = [float(np.mean((Y[m] - t) ** 2)) for m in range(ens.nmember)]
    mean_mse = float(np.mean((Y.mean(0) - t) ** 2))
    _say("held-out standardised MSE per member", per, "ensemble", mean_mse)
    assert max(per) < 0.1
    assert mean_mse <= np.mean(per) + 1e-6


@pytest.mark.parametrize("prec", ["f64", "bf16x2"])
def test_masked_pair_energies(torch, prec):
    for sysm in (fefgen.make_system(0),
                 fefgen.make_two_class_system(22, (40, 10, 20), [(24, 5), (9, 2), (24, 5)],
                                              naux0=8)):
        ctx = lib().Context(sysm)
        p = PREC[prec]
        full = ctx.energies(p)[0].cpu().numpy().copy()
        rng = np.random.default_rng(5)
        sel = (rng.random(sysm.npair) < 0.4).astype(np.int32)
        sel[0] = 1
        ctx.E2_pair.fill_(7.0)
        E2, tot = ctx.pair_energies_masked(p, torch.from_numpy(sel).cuda())
        E2 = E2.cpu().numpy()
        assert np.array_equal(E2[sel == 1], full[sel == 1])
        assert np.all(E2[sel == 0] == 7.0)
        assert float(tot.cpu()[0]) == pytest.approx(float(np.sum(E2)), rel=1e-13)
        # none selected: totals of the preset values only
        ctx.E2_pair.fill_(-1e-3)
        _, tot = ctx.pair_energies_masked(p, torch.zeros(sysm.npair, dtype=torch.int32,
                                                        device="cuda"))
        assert float(tot.cpu()[0]) == pytest.approx(-1e-3 * sysm.npair, rel=1e-12)


def test_surrogate_select_logic(torch):
    """Selection rules: threshold < 0 or r_exact beyond every pair sends all
    pairs to the exact kernel (bitwise the exact energies); an infinite
    threshold with r_exact = 0 predicts every class-0 pair with the ensemble
    mean; fragments outside class 0 always go exact."""
    train = lib().Context(small_box(103, n_water=200))
    _, X, T, _ = _dataset(torch, train, 6.0 * BOHR)
    ens = lib().Ensemble(nmember=5, seed=2)
    ens.fit_stats(X, T)
    ens.train(X, T, epochs=3, nb=256)
    sysm = small_box(104, n_water=200)
    ctx = lib().Context(sysm)
    ctx.scf(3)
    p = PREC["bf16x2"]
    exact = ctx.energies(p)[0].cpu().numpy().copy()
    U = ctx.invariants()
    E2, tot, sel = ctx.surrogate_energies(ens, U, 0.0, -1.0, p)
    assert np.all(sel.cpu().numpy() == 1)
    assert np.array_equal(E2.cpu().numpy(), exact)
    E2, tot, sel = ctx.surrogate_energies(ens, U, 1e9, 1.0, p)
    assert np.all(sel.cpu().numpy() == 1)
    E2, tot, sel = ctx.surrogate_energies(ens, U, 0.0, math.inf, p)
    assert np.all(sel.cpu().numpy() == 0)
    Xall, _ = ctx.pair_features(U)
    Y = ens.forward(Xall).cpu().numpy().astype(np.float64)
    st = ens.stats.cpu().numpy().astype(np.float64)
    R2 = (1.0 / sysm.pair_s) ** 2
    pred = (Y.mean(0) * st[35] + st[34]) / R2
    np.testing.assert_allclose(E2.cpu().numpy(), pred, rtol=1e-5, atol=1e-12)
    two = fefgen.make_two_class_system(22, (40, 10, 20), [(24, 5), (9, 2), (24, 5)], naux0=8)
    c2 = lib().Context(two)
    U2 = c2.invariants()
    _, _, sel2 = c2.surrogate_energies(ens, U2, 0.0, math.inf, p)
    sel2 = sel2.cpu().numpy()
    solute = (two.cls[two.pair_x] != 0) | (two.cls[two.pair_y] != 0)
    assert np.all(sel2[solute] == 1)


def test_surrogate_gain_report(torch):
    """What the trained ensemble gains over the exact path alone on a
    held-out box: the share of distant pairs it is allowed to predict at each
    disagreement threshold and the total-energy error it then makes (exact
    BF16x2 kernel for the rest and for R < 6 A).  The exact-only pass is the
    reference; fallback pairs must match it bitwise."""
    train = lib().Context(small_box(105))
    _, X, T, _ = _dataset(torch, train, 6.0 * BOHR)
    ens = lib().Ensemble(nmember=5, seed=3)
    ens.fit_stats(X, T)
    ens.train(X, T, epochs=20, nb=512, lr=2e-3)
    sysm = small_box(106)
    ctx = lib().Context(sysm)
    ctx.scf(10)
    p = PREC["bf16x2"]
    exact = ctx.energies(p)[0].cpu().numpy().copy()
    etot = float(np.sum(exact))
    U = ctx.invariants()
    prev = -1.0
    for thr in (1e-8, 1e-6, 1e-5, 1e-4, 1e-3):
        E2, tot, sel = ctx.surrogate_energies(ens, U, 6.0 * BOHR, thr, p)
        E2 = E2.cpu().numpy(); sel = sel.cpu().numpy()
        assert np.array_equal(E2[sel == 1], exact[sel == 1])
        frac = float(np.mean(sel == 0))
        err = float(tot.cpu()[0]) - etot
        _say(f"threshold {thr:g} Eh: predicted {frac:.4f} of pairs, total error {err:.3e} Eh")
        assert frac >= prev
        prev = frac
