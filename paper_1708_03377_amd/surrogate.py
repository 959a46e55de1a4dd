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
