"""ctypes binding of ``libfef.so`` (C ABI in include/fef.h).

Argument marshalling only: every function here has the C entry point's name,
turns tensors into device pointers and checks the returned status.  No
arithmetic of the method happens here.  A missing library is an error.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfef.so")

FEF_OK = 0
FEF_E_ARG = -1
FEF_E_SHAPE = -2
FEF_E_PREC = -3
FEF_E_WORKSPACE = -4
FEF_E_HIP = -5
FEF_E_UNSUPPORTED = -6
FEF_E_IO = -7
FEF_FLAG_GAP = 1
FEF_FLAG_NONFINITE = 2
FEF_FLAG_NOCONV = 4

PREC = {"f64": 0, "f32": 1, "bf16x2": 2, "fp16x2": 3, "bf16x3": 4}

Q_OPS_BYTES, Q_HALF_WS_BYTES, Q_PAIR_WS_BYTES, Q_FIELD_WS_BYTES, Q_SCF_WS_BYTES = range(5)
Q_BOV_ELEMS, Q_W_ELEMS, Q_NITEMS, Q_B_ELEMS, Q_C_ELEMS, Q_EPS_ELEMS, Q_G_ELEMS, Q_NPAIR = range(5, 13)
Q_NSLOT, Q_NENTRIES, Q_MASKED_WS_BYTES, Q_SURR_WS_BYTES, Q_BPACK_ELEMS = 13, 14, 15, 16, 17
Q_COUPLED_WS_BYTES = 18
Q_DRESSING_WS_BYTES, Q_HOO_ELEMS, Q_HVV_ELEMS = 19, 20, 21

MLP_NIN, MLP_NHID, MLP_NPARAM, MLP_STRIDE, MLP_NSTATS = 17, 128, 18945, 18952, 36

# every entry point declared in include/fef.h
ENTRY_POINTS = ("fef_plan_create", "fef_plan_destroy", "fef_plan_query",
                "fef_plan_set_tiles", "fef_plan_get_tiles",
                "fef_half_transform", "fef_pair_energies", "fef_coulomb_field",
                "fef_scf_step", "fef_graph_create", "fef_graph_launch", "fef_graph_destroy",
                "fef_autotune", "fef_pair_energies_masked", "fef_coupling_modes",
                "fef_fragment_invariants", "fef_pair_features", "fef_column_stats",
                "fef_mlp_pack", "fef_mlp_forward", "fef_mlp_train_step",
                "fef_mlp_train_ws_bytes", "fef_surrogate_select", "fef_pack_coefficients",
                "fef_scf_step_packed", "fef_pair_energies_noalloc", "fef_plan_stage_timing",
                "fef_plan_stage_ms", "fef_coupled_pair_energies", "fef_dimer_dressing",
                "fef_autotune_cached", "fef_monomer_energies", "fef_status_string")


class FefError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


class SystemDesc(ctypes.Structure):
    _fields_ = [("nfrag", ctypes.c_int32), ("nclass", ctypes.c_int32),
                ("nbf", ctypes.c_void_p), ("nocc", ctypes.c_void_p),
                ("cls", ctypes.c_void_p), ("naux", ctypes.c_void_p),
                ("npair", ctypes.c_int64),
                ("pair_x", ctypes.c_void_p), ("pair_y", ctypes.c_void_p),
                ("pair_s", ctypes.c_void_p)]


class PassArgs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("B", "G", "F0", "htilde", "C0", "eps0", "C", "eps", "D", "dD_max", "flags",
                 "ops", "E2_pair", "E2_total", "ws")] + [("ws_bytes", ctypes.c_size_t),
                                                         ("Bp", ctypes.c_void_p)]


_lib = None


def load_library(path: Optional[str] = None) -> ctypes.CDLL:
    """Loads libfef.so; raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with "
                           "`python -m paper_1708_03377_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(p)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.fef_plan_create.argtypes = [ctypes.POINTER(SystemDesc), ctypes.POINTER(vp)]
    lib.fef_plan_destroy.argtypes = [vp]
    lib.fef_plan_query.argtypes = [vp, i32, i32, ctypes.POINTER(i64)]
    lib.fef_plan_set_tiles.argtypes = [vp, i32, i32, i32]
    lib.fef_plan_get_tiles.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.fef_half_transform.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, vp, sz, vp]
    lib.fef_pair_energies.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, sz, vp]
    lib.fef_coulomb_field.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    lib.fef_scf_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.fef_graph_create.argtypes = [vp, ctypes.POINTER(PassArgs), i32, i32, ctypes.POINTER(vp)]
    lib.fef_graph_launch.argtypes = [vp, vp]
    lib.fef_graph_destroy.argtypes = [vp]
    lib.fef_autotune.argtypes = [vp, vp, vp, i32, vp, sz, i32, vp, ctypes.POINTER(i32),
                                 ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    lib.fef_autotune_cached.argtypes = [vp, vp, vp, i32, vp, sz, i32, vp, ctypes.c_char_p,
                                        ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]
    f32, f64 = ctypes.c_float, ctypes.c_double
    lib.fef_pair_energies_masked.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, sz, vp]
    lib.fef_coupling_modes.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.fef_fragment_invariants.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.fef_pair_features.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
    lib.fef_column_stats.argtypes = [i64, i32, i32, vp, vp, vp, vp]
    lib.fef_mlp_pack.argtypes = [i32, vp, vp, vp]
    lib.fef_mlp_forward.argtypes = [i32, i64, vp, vp, vp, vp, vp]
    lib.fef_mlp_train_step.argtypes = [i32, vp, vp, vp, i32, vp, vp, vp, vp, vp, i32, f32, vp,
                                       vp, vp, sz, vp]
    lib.fef_mlp_train_ws_bytes.argtypes = [i32, i32, ctypes.POINTER(i64)]
    lib.fef_surrogate_select.argtypes = [vp, vp, i32, vp, vp, f64, f64, vp, vp, vp]
    lib.fef_pack_coefficients.argtypes = [vp, vp, vp, vp]
    lib.fef_scf_step_packed.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.fef_pair_energies_noalloc.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
    lib.fef_coupled_pair_energies.argtypes = [vp, vp, vp, vp, vp, f64, i32, vp, vp, vp, vp, vp,
                                              sz, vp]
    lib.fef_dimer_dressing.argtypes = [vp, vp, vp, vp, vp, f64, i32, vp, vp, vp, vp, vp, vp, sz,
                                       vp]
    lib.fef_monomer_energies.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.fef_plan_stage_timing.argtypes = [vp, i32]
    lib.fef_plan_stage_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.fef_status_string.argtypes = [i32]
    lib.fef_status_string.restype = ctypes.c_char_p
    for name in ENTRY_POINTS:
        if name != "fef_status_string":
            getattr(lib, name).restype = i32
    if path is None:
        _lib = lib
    return lib


def fef_status_string(status: int) -> str:
    return load_library().fef_status_string(status).decode()


def _check(fn: str, status: int):
    if status != FEF_OK:
        raise FefError(fn, status, fef_status_string(status))


def _ptr(t) -> Optional[int]:
    """Device (or host) address of a tensor / array, None for None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _nbytes(t) -> int:
    if t is None:
        return 0
    if isinstance(t, np.ndarray):
        return t.nbytes
    return t.numel() * t.element_size()


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    return getattr(stream, "cuda_stream", stream)


class Plan:
    """Owns a fef_plan handle and the host arrays it was created from."""

    def __init__(self, handle: int, keep):
        self.handle = handle
        self._keep = keep

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                load_library().fef_plan_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def fef_plan_create(nbf, nocc, cls, naux, pair_x, pair_y, pair_s) -> Plan:
    lib = load_library()
    arrs = [np.ascontiguousarray(nbf, dtype=np.int32),
            np.ascontiguousarray(nocc, dtype=np.int32),
            np.ascontiguousarray(cls, dtype=np.int32),
            np.ascontiguousarray(naux, dtype=np.int32),
            np.ascontiguousarray(pair_x, dtype=np.int32),
            np.ascontiguousarray(pair_y, dtype=np.int32),
            np.ascontiguousarray(pair_s, dtype=np.float64)]
    d = SystemDesc(len(arrs[0]), len(arrs[3]), *(a.ctypes.data for a in arrs[:4]),
                   len(arrs[4]), *(a.ctypes.data for a in arrs[4:]))
    h = ctypes.c_void_p()
    _check("fef_plan_create", lib.fef_plan_create(ctypes.byref(d), ctypes.byref(h)))
    return Plan(h.value, arrs)


def fef_plan_query(plan: Plan, what: int, prec: int = 0) -> int:
    out = ctypes.c_int64()
    _check("fef_plan_query", load_library().fef_plan_query(plan.handle, what, prec,
                                                           ctypes.byref(out)))
    return out.value


def fef_plan_set_tiles(plan: Plan, prec: int, xb: int, yc: int):
    _check("fef_plan_set_tiles", load_library().fef_plan_set_tiles(plan.handle, prec, xb, yc))


def fef_plan_get_tiles(plan: Plan, prec: int):
    xb, yc = ctypes.c_int32(), ctypes.c_int32()
    _check("fef_plan_get_tiles", load_library().fef_plan_get_tiles(plan.handle, prec,
                                                                   ctypes.byref(xb),
                                                                   ctypes.byref(yc)))
    return xb.value, yc.value


def fef_half_transform(plan, B, C, G, Bov, W, ops, prec, ws, stream=None):
    _check("fef_half_transform", load_library().fef_half_transform(
        plan.handle, _ptr(B), _ptr(C), _ptr(G), _ptr(Bov), _ptr(W), _ptr(ops), prec,
        _ptr(ws), _nbytes(ws), _stream(stream)))


def fef_pair_energies(plan, ops, eps, prec, E2_pair, E2_total, flags, ws, stream=None):
    _check("fef_pair_energies", load_library().fef_pair_energies(
        plan.handle, _ptr(ops), _ptr(eps), prec, _ptr(E2_pair), _ptr(E2_total), _ptr(flags),
        _ptr(ws), _nbytes(ws), _stream(stream)))


def fef_plan_stage_timing(plan, enable: bool):
    _check("fef_plan_stage_timing", load_library().fef_plan_stage_timing(plan.handle, int(enable)))


def fef_plan_stage_ms(plan):
    """Stage durations (ms) of the last SCF step: density, moments, field +
    Coulomb build, eigensolver."""
    out = (ctypes.c_double * 4)()
    _check("fef_plan_stage_ms", load_library().fef_plan_stage_ms(plan.handle, out))
    return [float(v) for v in out]


def fef_pair_energies_noalloc(plan, ops, eps, prec, E2_pair, E2_total, flags, stream=None):
    _check("fef_pair_energies_noalloc", load_library().fef_pair_energies_noalloc(
        plan.handle, _ptr(ops), _ptr(eps), prec, _ptr(E2_pair), _ptr(E2_total), _ptr(flags),
        _stream(stream)))


def fef_coupled_pair_energies(plan, B, C, eps, G, tol, maxit, E2_pair, E2_total, iters, flags,
                              ws, stream=None):
    _check("fef_coupled_pair_energies", load_library().fef_coupled_pair_energies(
        plan.handle, _ptr(B), _ptr(C), _ptr(eps), _ptr(G), float(tol), int(maxit), _ptr(E2_pair),
        _ptr(E2_total), _ptr(iters), _ptr(flags), _ptr(ws), _nbytes(ws), _stream(stream)))


def fef_monomer_energies(plan, Bov, W, eps, E_M2, E_M2_total, flags, stream=None):
    _check("fef_monomer_energies", load_library().fef_monomer_energies(
        plan.handle, _ptr(Bov), _ptr(W), _ptr(eps), _ptr(E_M2), _ptr(E_M2_total), _ptr(flags),
        _stream(stream)))


def fef_dimer_dressing(plan, B, C, eps, G, tol, maxit, E2_pair, E2_total, Hoo, Hvv, flags, ws,
                       stream=None):
    _check("fef_dimer_dressing", load_library().fef_dimer_dressing(
        plan.handle, _ptr(B), _ptr(C), _ptr(eps), _ptr(G), float(tol), int(maxit), _ptr(E2_pair),
        _ptr(E2_total), _ptr(Hoo), _ptr(Hvv), _ptr(flags), _ptr(ws), _nbytes(ws),
        _stream(stream)))


def fef_coulomb_field(plan, B, G, D, J, ws, stream=None):
    _check("fef_coulomb_field", load_library().fef_coulomb_field(
        plan.handle, _ptr(B), _ptr(G), _ptr(D), _ptr(J), _ptr(ws), _nbytes(ws),
        _stream(stream)))


def fef_scf_step(plan, B, G, F0, htilde, C, eps, D, dD_max, flags, ws, stream=None):
    _check("fef_scf_step", load_library().fef_scf_step(
        plan.handle, _ptr(B), _ptr(G), _ptr(F0), _ptr(htilde), _ptr(C), _ptr(eps), _ptr(D),
        _ptr(dD_max), _ptr(flags), _ptr(ws), _nbytes(ws), _stream(stream)))


class Graph:
    """Owns a fef_graph handle (and references to the buffers it bakes in)."""

    def __init__(self, handle: int, keep):
        self.handle = handle
        self._keep = keep

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                load_library().fef_graph_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def fef_graph_create(plan, niter, prec, B, G, F0, htilde, C0, eps0, C, eps, D, dD_max, flags,
                     ops, E2_pair, E2_total, ws, Bp=None) -> Graph:
    bufs = (B, G, F0, htilde, C0, eps0, C, eps, D, dD_max, flags, ops, E2_pair, E2_total, ws, Bp)
    a = PassArgs(*[_ptr(t) for t in bufs[:-1]], _nbytes(ws), _ptr(Bp))
    h = ctypes.c_void_p()
    _check("fef_graph_create", load_library().fef_graph_create(plan.handle, ctypes.byref(a),
                                                               niter, prec, ctypes.byref(h)))
    return Graph(h.value, (plan, bufs))


def fef_graph_launch(graph: Graph, stream=None):
    _check("fef_graph_launch", load_library().fef_graph_launch(graph.handle, _stream(stream)))


def fef_autotune(plan, ops, eps, prec, ws, reps=3, stream=None):
    xb, yc, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check("fef_autotune", load_library().fef_autotune(
        plan.handle, _ptr(ops), _ptr(eps), prec, _ptr(ws), _nbytes(ws), reps, _stream(stream),
        ctypes.byref(xb), ctypes.byref(yc), ctypes.byref(us)))
    return xb.value, yc.value, us.value


def fef_autotune_cached(plan, ops, eps, prec, ws, cache_path, reps=3, stream=None):
    xb, yc, us, hit = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check("fef_autotune_cached", load_library().fef_autotune_cached(
        plan.handle, _ptr(ops), _ptr(eps), prec, _ptr(ws), _nbytes(ws), reps, _stream(stream),
        path, ctypes.byref(xb), ctypes.byref(yc), ctypes.byref(us), ctypes.byref(hit)))
    return xb.value, yc.value, us.value, bool(hit.value)


def fef_pair_energies_masked(plan, ops, eps, prec, select, E2_pair, E2_total, flags, ws,
                             stream=None):
    _check("fef_pair_energies_masked", load_library().fef_pair_energies_masked(
        plan.handle, _ptr(ops), _ptr(eps), prec, _ptr(select), _ptr(E2_pair), _ptr(E2_total),
        _ptr(flags), _ptr(ws), _nbytes(ws), _stream(stream)))


def fef_coupling_modes(plan, G, Q, ws, stream=None):
    _check("fef_coupling_modes", load_library().fef_coupling_modes(
        plan.handle, _ptr(G), _ptr(Q), _ptr(ws), _nbytes(ws), _stream(stream)))


def fef_fragment_invariants(plan, B, G, D, Q, U, ws, stream=None):
    _check("fef_fragment_invariants", load_library().fef_fragment_invariants(
        plan.handle, _ptr(B), _ptr(G), _ptr(D), _ptr(Q), _ptr(U), _ptr(ws), _nbytes(ws),
        _stream(stream)))


def fef_pair_features(plan, U, E2_pair, idx, n, X, T, stream=None):
    _check("fef_pair_features", load_library().fef_pair_features(
        plan.handle, _ptr(U), _ptr(E2_pair), _ptr(idx), n, _ptr(X), _ptr(T), _stream(stream)))


def fef_column_stats(n, ncol, inverse, A, mean, sdev, stream=None):
    _check("fef_column_stats", load_library().fef_column_stats(
        n, ncol, int(inverse), _ptr(A), _ptr(mean), _ptr(sdev), _stream(stream)))


def fef_mlp_pack(nmember, P, W, stream=None):
    _check("fef_mlp_pack", load_library().fef_mlp_pack(nmember, _ptr(P), _ptr(W),
                                                       _stream(stream)))


def fef_mlp_forward(nmember, n, X, stats, W, Y, stream=None):
    _check("fef_mlp_forward", load_library().fef_mlp_forward(
        nmember, n, _ptr(X), _ptr(stats), _ptr(W), _ptr(Y), _stream(stream)))


def fef_mlp_train_ws_bytes(nmember, nb) -> int:
    out = ctypes.c_int64()
    _check("fef_mlp_train_ws_bytes", load_library().fef_mlp_train_ws_bytes(
        nmember, nb, ctypes.byref(out)))
    return out.value


def fef_mlp_train_step(nmember, X, T, idx, nb, stats, P, M, V, W, step, lr, loss, grad, ws,
                       stream=None):
    _check("fef_mlp_train_step", load_library().fef_mlp_train_step(
        nmember, _ptr(X), _ptr(T), _ptr(idx), nb, _ptr(stats), _ptr(P), _ptr(M), _ptr(V),
        _ptr(W), step, lr, _ptr(loss), _ptr(grad), _ptr(ws), _nbytes(ws), _stream(stream)))


def fef_surrogate_select(plan, U, nmember, stats, W, r_exact, threshold, E2_pair, select,
                         stream=None):
    _check("fef_surrogate_select", load_library().fef_surrogate_select(
        plan.handle, _ptr(U), nmember, _ptr(stats), _ptr(W), float(r_exact), float(threshold),
        _ptr(E2_pair), _ptr(select), _stream(stream)))


def fef_pack_coefficients(plan, B, Bp, stream=None):
    _check("fef_pack_coefficients", load_library().fef_pack_coefficients(
        plan.handle, _ptr(B), _ptr(Bp), _stream(stream)))


def fef_scf_step_packed(plan, Bp, G, F0, htilde, C, eps, D, dD_max, flags, ws, stream=None):
    _check("fef_scf_step_packed", load_library().fef_scf_step_packed(
        plan.handle, _ptr(Bp), _ptr(G), _ptr(F0), _ptr(htilde), _ptr(C), _ptr(eps), _ptr(D),
        _ptr(dD_max), _ptr(flags), _ptr(ws), _nbytes(ws), _stream(stream)))
