"""Device-side state for one fragment system: torch owns the HBM buffers,
libfef does every step of the computation.

``Context`` uploads the input pools once, allocates the operand pools and
workspaces the library asks for (fef_plan_query), and exposes the four entry
points plus an SCF driver loop.  Nothing here computes the method.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np

from . import _fef as F


class Context:
    def __init__(self, system, device: str = "cuda:0", htilde: Optional[np.ndarray] = None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        s = system
        self.system = s
        self.plan = F.fef_plan_create(s.nbf, s.nocc, s.cls, s.naux_class, s.pair_x, s.pair_y,
                                      s.pair_s)
        q = lambda what, prec=0: F.fef_plan_query(self.plan, what, prec)
        self.npair = q(F.Q_NPAIR)
        self.nitems = q(F.Q_NITEMS)
        up = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)
        self.B = up(s.B)
        self.G = up(s.G)
        self.F0 = up(s.F0)
        self.C0 = up(s.C)
        self.eps0 = up(s.eps)
        self.C = self.C0.clone()
        self.eps = self.eps0.clone()
        self.htilde = up(htilde) if htilde is not None else None
        self.D = torch.zeros(max(q(F.Q_C_ELEMS), 1), dtype=torch.float64, device=self.device)
        self.flags = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.dD_max = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.E2_pair = torch.zeros(max(self.npair, 1), dtype=torch.float64, device=self.device)
        self.E2_total = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.ops: Dict[int, "torch.Tensor"] = {}
        ws = max([q(F.Q_HALF_WS_BYTES, p) for p in F.PREC.values()] +
                 [q(F.Q_PAIR_WS_BYTES, p) for p in F.PREC.values()] +
                 [q(F.Q_FIELD_WS_BYTES), q(F.Q_SCF_WS_BYTES)])
        self.ws = torch.empty(ws, dtype=torch.uint8, device=self.device)
        self.sizes = {"bov": q(F.Q_BOV_ELEMS), "w": q(F.Q_W_ELEMS), "c": q(F.Q_C_ELEMS)}
        self._q = q

    # ---- buffers ---------------------------------------------------------
    def ops_for(self, prec: int):
        if prec not in self.ops:
            n = self._q(F.Q_OPS_BYTES, prec)
            self.ops[prec] = self.torch.zeros(n, dtype=self.torch.uint8, device=self.device)
        return self.ops[prec]

    def stream(self):
        return self.torch.cuda.current_stream(self.device)

    def reset_orbitals(self):
        self.C.copy_(self.C0)
        self.eps.copy_(self.eps0)
        self.flags.zero_()

    # ---- entry points ------------------------------------------------------
    def half_transform(self, prec: int, Bov=None, W=None):
        F.fef_half_transform(self.plan, self.B, self.C, self.G, Bov, W, self.ops_for(prec), prec,
                             self.ws, self.stream())

    def pair_energies(self, prec: int):
        F.fef_pair_energies(self.plan, self.ops_for(prec), self.eps, prec, self.E2_pair,
                            self.E2_total, self.flags, self.ws, self.stream())
        return self.E2_pair[:self.npair], self.E2_total

    def coulomb_field(self, D, J):
        F.fef_coulomb_field(self.plan, self.B, self.G, D, J, self.ws, self.stream())
        return J

    def scf_step(self, D_out=None):
        F.fef_scf_step(self.plan, self.B, self.G, self.F0, self.htilde, self.C, self.eps,
                       self.D if D_out is None else D_out, self.dD_max, self.flags, self.ws,
                       self.stream())
        return self.dD_max

    def scf(self, niter: int):
        for _ in range(niter):
            self.scf_step()

    def graph(self, niter: int, prec: int, from_start: bool = True):
        """A captured FEF pass: [reset to the generated orbitals], niter SCF
        steps, half transform and pair energies in mode ``prec``."""
        return F.fef_graph_create(self.plan, niter, prec, self.B, self.G, self.F0, self.htilde,
                                  self.C0 if from_start else None,
                                  self.eps0 if from_start else None, self.C, self.eps, self.D,
                                  self.dD_max, self.flags, self.ops_for(prec), self.E2_pair,
                                  self.E2_total, self.ws)

    def launch(self, graph):
        F.fef_graph_launch(graph, self.stream())

    def autotune(self, prec: int, reps: int = 3):
        """Picks the fastest pair-kernel tiling for the current operands
        (runs the half transform first)."""
        self.half_transform(prec)
        return F.fef_autotune(self.plan, self.ops_for(prec), self.eps, prec, self.ws, reps,
                              self.stream())

    def energies(self, prec: int):
        """Half transform + pair energies on the current orbitals."""
        self.half_transform(prec)
        return self.pair_energies(prec)
