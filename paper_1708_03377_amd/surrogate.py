"""Device state of the distant-pair surrogate ensemble.

``Ensemble`` owns the FP32 master parameters, the Adam moments, the BF16
copy the kernels evaluate and the feature / target statistics; training,
inference and selection all run in libfef (fef_mlp_train_step,
fef_mlp_forward, fef_surrogate_select).  Initial weights and mini-batch
orders are seeded draws from ``fefgen``.
"""
from __future__ import annotations

from typing import List

import numpy as np

from . import _fef as F


class Ensemble:
    def __init__(self, nmember: int = 5, seed: int = 0, device: str = "cuda:0"):
        import torch
        import fefgen
        self.torch = torch
        self.device = torch.device(device)
        self.nmember = int(nmember)
        self.seed = int(seed)
        p0 = fefgen.mlp_init(seed, nmember)
        self.P = torch.from_numpy(p0.ravel()).to(self.device)
        self.M = torch.zeros_like(self.P)
        self.V = torch.zeros_like(self.P)
        self.W = torch.zeros(self.P.numel(), dtype=torch.int16, device=self.device)
        self.stats = torch.zeros(F.MLP_NSTATS, dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(self.nmember, dtype=torch.float32, device=self.device)
        self.step = 0
        self._ws = None
        F.fef_mlp_pack(self.nmember, self.P, self.W, self.stream())

    def stream(self):
        return self.torch.cuda.current_stream(self.device)

    def fit_stats(self, X, T):
        """Feature means / inverse deviations and target mean / deviation."""
        n = int(X.shape[0])
        F.fef_column_stats(n, 17, 1, X, self.stats[0:17], self.stats[17:34], self.stream())
        F.fef_column_stats(n, 1, 0, T, self.stats[34:35], self.stats[35:36], self.stream())

    def _workspace(self, nb: int):
        need = F.fef_mlp_train_ws_bytes(self.nmember, nb)
        if self._ws is None or self._ws.numel() < need:
            self._ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        return self._ws

    def train_step(self, X, T, idx, nb: int, lr: float, grad=None, update: bool = True):
        ws = self._workspace(nb)
        if update:
            self.step += 1
        F.fef_mlp_train_step(self.nmember, X, T, idx, nb, self.stats, self.P, self.M, self.V,
                             self.W, self.step if update else 0, lr, self.loss, grad, ws,
                             self.stream())

    def train(self, X, T, epochs: int, nb: int = 1024, lr: float = 1e-3,
              lr_final: float = 1e-4) -> List[float]:
        """Adam over `epochs` passes of member-wise shuffled mini-batches
        (learning rate decays geometrically from lr to lr_final); returns the
        mean member loss after every epoch."""
        import fefgen
        n = int(X.shape[0])
        hist = []
        nsteps = max(n // nb, 1) * max(epochs, 1)
        decay = (lr_final / lr) ** (1.0 / max(nsteps - 1, 1))
        k = 0
        for ep in range(epochs):
            idx = self.torch.from_numpy(
                fefgen.epoch_batches(self.seed, ep, self.nmember, n, nb)).to(self.device)
            for s in range(idx.shape[0]):
                self.train_step(X, T, idx[s], nb, lr * decay ** k)
                k += 1
            hist.append(float(self.loss.mean().cpu()))
        return hist

    def forward(self, X):
        """Standardised predictions [nmember][n] for raw features X [n][17]."""
        n = int(X.shape[0])
        Y = self.torch.empty(self.nmember * max(n, 1), dtype=self.torch.float32,
                             device=self.device)
        F.fef_mlp_forward(self.nmember, n, X, self.stats, self.W, Y, self.stream())
        return Y[:self.nmember * n].view(self.nmember, n)


# ---------------------------------------------------------------------------
# Training recipe of the surrogate workload (8000 waters at 15 A): seeded
# 1000-water boxes of the same density and cutoff (workload 1's style), 10
# SCF steps each, the exact FP64 pair energies of every pair at R >= 6 A as
# labels.  Seeds >= 100 never coincide with a named workload.
TRAIN_SEEDS = (101, 102)
HELDOUT_SEED = 103
R_EXACT_ANGSTROM = 6.0


def pair_dataset(ctx, r_min_bohr: float, niter: int = 10):
    """Features X [n][17] and targets T [n] (device tensors) of the pairs of
    ``ctx``'s system at R >= r_min_bohr, after niter SCF steps from the
    generated orbitals, with the exact FP64 pair energies as targets; also
    returns the pair indices."""
    import torch
    ctx.reset_orbitals()
    ctx.scf(niter)
    ctx.energies(F.PREC["f64"])
    U = ctx.invariants()
    far = np.nonzero(1.0 / ctx.system.pair_s >= r_min_bohr)[0].astype(np.int32)
    idx = torch.from_numpy(far).to(ctx.device)
    X, T = ctx.pair_features(U, idx, with_targets=True)
    return X.clone(), T.clone(), far


def training_set(seeds=TRAIN_SEEDS, n_water: int = 1000, cutoff: float = 15.0,
                 niter: int = 10, device: str = "cuda:0"):
    """The concatenated pair dataset of the seeded training boxes."""
    import torch
    import fefgen
    from .runtime import Context
    r_min = R_EXACT_ANGSTROM * fefgen.BOHR_PER_ANGSTROM
    Xs, Ts = [], []
    for sd in seeds:
        ctx = Context(fefgen.surrogate_training_box(sd, n_water=n_water, cutoff=cutoff),
                      device=device)
        X, T, _ = pair_dataset(ctx, r_min, niter)
        Xs.append(X)
        Ts.append(T)
        del ctx
    return torch.cat(Xs), torch.cat(Ts)


def train_ensemble(X, T, nmember: int = 5, seed: int = 0, epochs: int = 6, nb: int = 1024,
                   lr: float = 2e-3, lr_final: float = 1e-4):
    """A fresh ensemble with statistics fitted on (X, T), trained by the
    library's kernels; returns (ensemble, loss per epoch)."""
    ens = Ensemble(nmember=nmember, seed=seed, device=str(X.device))
    ens.fit_stats(X, T)
    hist = ens.train(X, T, epochs=epochs, nb=nb, lr=lr, lr_final=lr_final)
    return ens, hist
