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
                 [q(F.Q_MASKED_WS_BYTES, p) for p in F.PREC.values()] +
                 [q(F.Q_FIELD_WS_BYTES), q(F.Q_SCF_WS_BYTES), q(F.Q_SURR_WS_BYTES)])
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

    def packed_coefficients(self):
        """The upper-triangle copy of B (packed on first use)."""
        if getattr(self, "_Bp", None) is None:
            self._Bp = self.torch.empty(max(self._q(F.Q_BPACK_ELEMS), 1),
                                        dtype=self.torch.float64, device=self.device)
            F.fef_pack_coefficients(self.plan, self.B, self._Bp, self.stream())
        return self._Bp

    def scf_step_packed(self, D_out=None):
        F.fef_scf_step_packed(self.plan, self.packed_coefficients(), self.G, self.F0,
                              self.htilde, self.C, self.eps,
                              self.D if D_out is None else D_out, self.dD_max, self.flags,
                              self.ws, self.stream())
        return self.dD_max

    def scf(self, niter: int):
        """niter SCF steps on the packed coefficients (as the captured pass)."""
        for _ in range(niter):
            self.scf_step_packed()

    def graph(self, niter: int, prec: int, from_start: bool = True):
        """A captured FEF pass: [reset to the generated orbitals], niter SCF
        steps, half transform and pair energies in mode ``prec``."""
        return F.fef_graph_create(self.plan, niter, prec, self.B, self.G, self.F0, self.htilde,
                                  self.C0 if from_start else None,
                                  self.eps0 if from_start else None, self.C, self.eps, self.D,
                                  self.dD_max, self.flags, self.ops_for(prec), self.E2_pair,
                                  self.E2_total, self.ws, self.packed_coefficients())

    def launch(self, graph):
        F.fef_graph_launch(graph, self.stream())

    def autotune(self, prec: int, reps: int = 3):
        """Picks the fastest pair-kernel tiling for the current operands
        (runs the half transform first)."""
        self.half_transform(prec)
        return F.fef_autotune(self.plan, self.ops_for(prec), self.eps, prec, self.ws, reps,
                              self.stream())

    def autotune_cached(self, prec: int, cache_path: str, reps: int = 3):
        """autotune through a persisted cache file: (xb, yc, us, from_cache)
        (runs the half transform first)."""
        self.half_transform(prec)
        return F.fef_autotune_cached(self.plan, self.ops_for(prec), self.eps, prec, self.ws,
                                     cache_path, reps, self.stream())

    def energies(self, prec: int):
        """Half transform + pair energies on the current orbitals."""
        self.half_transform(prec)
        return self.pair_energies(prec)

    def coupled_pair_energies(self, tol: float = 1e-14, maxit: int = 500):
        """Pair energies with the W^[0]-coupled dimer doubles on the current
        orbitals; returns (E2_pair, E2_total, iterations per pair).  Its
        workspace is allocated on first use."""
        torch = self.torch
        if getattr(self, "_cp_ws", None) is None:
            self._cp_ws = torch.empty(max(self._q(F.Q_COUPLED_WS_BYTES), 1), dtype=torch.uint8,
                                      device=self.device)
            self._cp_E = torch.zeros(max(self.npair, 1), dtype=torch.float64, device=self.device)
            self._cp_tot = torch.zeros(1, dtype=torch.float64, device=self.device)
            self._cp_it = torch.zeros(max(self.npair, 1), dtype=torch.int32, device=self.device)
        F.fef_coupled_pair_energies(self.plan, self.B, self.C, self.eps, self.G, tol, maxit,
                                    self._cp_E, self._cp_tot, self._cp_it, self.flags,
                                    self._cp_ws, self.stream())
        return self._cp_E[:self.npair], self._cp_tot, self._cp_it[:self.npair]

    def dimer_dressing(self, tol: float = 1e-14, maxit: int = 0):
        """Cross-fragment one-body dressings from the dimer doubles (maxit = 0:
        the amplitudes -(ia|jb)/D of the pair energies; otherwise the
        W^[0]-coupled ones); returns (E2_pair, E2_total, Hoo, Hvv) with the
        per-fragment pools Hoo [nocc][nocc] and Hvv [nvir][nvir]."""
        torch = self.torch
        if getattr(self, "_dr_ws", None) is None:
            self._dr_ws = torch.empty(max(self._q(F.Q_DRESSING_WS_BYTES), 1), dtype=torch.uint8,
                                      device=self.device)
            self._dr_E = torch.zeros(max(self.npair, 1), dtype=torch.float64, device=self.device)
            self._dr_tot = torch.zeros(1, dtype=torch.float64, device=self.device)
            self._dr_oo = torch.zeros(max(self._q(F.Q_HOO_ELEMS), 1), dtype=torch.float64,
                                      device=self.device)
            self._dr_vv = torch.zeros(max(self._q(F.Q_HVV_ELEMS), 1), dtype=torch.float64,
                                      device=self.device)
        F.fef_dimer_dressing(self.plan, self.B, self.C, self.eps, self.G, tol, maxit, self._dr_E,
                             self._dr_tot, self._dr_oo, self._dr_vv, self.flags, self._dr_ws,
                             self.stream())
        return self._dr_E[:self.npair], self._dr_tot, self._dr_oo, self._dr_vv

    def monomer_energies(self, prec: int = 0):
        """E_M2 of every fragment on the current orbitals (Eq. EM2): the half
        transform in mode `prec` with its dense FP64 B_ov and W outputs, then
        the monomer kernel; returns (per-fragment energies, their sum).  The
        output buffers are allocated on first use."""
        torch = self.torch
        if getattr(self, "_mo_E", None) is None:
            self._mo_bov = torch.empty(max(self.sizes["bov"], 1), dtype=torch.float64,
                                       device=self.device)
            self._mo_w = torch.empty(max(self.sizes["w"], 1), dtype=torch.float64,
                                     device=self.device)
            self._mo_E = torch.zeros(max(self.system.nfrag, 1), dtype=torch.float64,
                                     device=self.device)
            self._mo_tot = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.half_transform(prec, self._mo_bov, self._mo_w)
        F.fef_monomer_energies(self.plan, self._mo_bov, self._mo_w, self.eps, self._mo_E,
                               self._mo_tot, self.flags, self.stream())
        return self._mo_E[:self.system.nfrag], self._mo_tot

    def correlation_energy(self, prec: int = 0):
        """Second-order correlation energy E_M2 + E_D2 (Eq. EFEF2) on the
        current orbitals: the monomer energies and the pair energies in mode
        `prec` (one half transform serves both); returns
        (E_M2, E_D2, E_M2 + E_D2) as floats."""
        _, em2 = self.monomer_energies(prec)
        _, ed2 = self.pair_energies(prec)
        em2, ed2 = float(em2.cpu()[0]), float(ed2.cpu()[0])
        return em2, ed2, em2 + ed2

    # ---- surrogate ---------------------------------------------------------
    def pair_energies_masked(self, prec: int, select):
        """Exact pair energies of the selected pairs; the others keep the
        values already in E2_pair."""
        F.fef_pair_energies_masked(self.plan, self.ops_for(prec), self.eps, prec, select,
                                   self.E2_pair, self.E2_total, self.flags, self.ws,
                                   self.stream())
        return self.E2_pair[:self.npair], self.E2_total

    def coupling_modes(self):
        if getattr(self, "_Q", None) is None:
            self._Q = self.torch.zeros(4 * int(self.system.naux_class[0]),
                                       dtype=self.torch.float64, device=self.device)
            F.fef_coupling_modes(self.plan, self.G, self._Q, self.ws, self.stream())
        return self._Q

    def invariants(self):
        """U [nfrag][8] from the current density D (after scf)."""
        U = self.torch.empty(max(self.system.nfrag, 1) * 8, dtype=self.torch.float64,
                             device=self.device)
        F.fef_fragment_invariants(self.plan, self.B, self.G, self.D, self.coupling_modes(), U,
                                  self.ws, self.stream())
        return U

    def pair_features(self, U, idx=None, with_targets=False):
        """Raw features X [n][17] (and targets E2 R^2) of the pairs idx
        (a device int32 tensor) or of every pair."""
        n = self.npair if idx is None else int(idx.numel())
        X = self.torch.empty(max(n, 1) * 17, dtype=self.torch.float32, device=self.device)
        T = self.torch.empty(max(n, 1), dtype=self.torch.float32, device=self.device) \
            if with_targets else None
        F.fef_pair_features(self.plan, U, self.E2_pair if with_targets else None, idx, n, X, T,
                            self.stream())
        return (X[:n * 17].view(n, 17), T[:n] if with_targets else None)

    def surrogate_energies(self, ens, U, r_exact_bohr: float, threshold: float,
                           prec: int = F.PREC["bf16x2"]):
        """Surrogate pass on the current orbitals: the ensemble predicts the
        pairs it agrees on, the exact kernel (mode ``prec``) evaluates the
        rest.  Returns (E2_pair, E2_total, select)."""
        if getattr(self, "_select", None) is None:
            self._select = self.torch.zeros(max(self.npair, 1), dtype=self.torch.int32,
                                            device=self.device)
        F.fef_surrogate_select(self.plan, U, ens.nmember, ens.stats, ens.W, r_exact_bohr,
                               threshold, self.E2_pair, self._select, self.stream())
        self.half_transform(prec)
        E2, tot = self.pair_energies_masked(prec, self._select)
        return E2, tot, self._select[:self.npair]
