"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/fef.h, and rejects bad arguments
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1708_03377_amd import _fef
    if not os.path.exists(_fef.LIB_PATH):
        pytest.fail("libfef.so is not built (run __graft_entry__.build())")
    return _fef, _fef.load_library()


def declared_entry_points():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?[\w\*]+\s+\*?(fef_\w+)\s*\(", txt, re.M))
    return names


def test_exports_every_declared_symbol():
    F, lib = _lib()
    names = declared_entry_points()
    assert {"fef_half_transform", "fef_pair_energies", "fef_coulomb_field",
            "fef_scf_step"} <= names
    for n in names:
        assert hasattr(lib, n), n
    assert names == set(F.ENTRY_POINTS)


def test_status_strings():
    F, lib = _lib()
    assert F.fef_status_string(0) == "ok"
    assert "workspace" in F.fef_status_string(F.FEF_E_WORKSPACE)
    assert F.fef_status_string(-99) == "unknown status"
    assert "file" in F.fef_status_string(F.FEF_E_IO)


def test_null_arguments_rejected():
    F, lib = _lib()
    h = ctypes.c_void_p()
    assert lib.fef_plan_create(None, ctypes.byref(h)) == F.FEF_E_ARG
    out = ctypes.c_int64()
    assert lib.fef_plan_query(None, 0, 0, ctypes.byref(out)) == F.FEF_E_ARG
    assert lib.fef_half_transform(None, None, None, None, None, None, None, 0, None, 0,
                                  None) == F.FEF_E_ARG
    assert lib.fef_pair_energies(None, None, None, 0, None, None, None, None, 0,
                                 None) == F.FEF_E_ARG
    assert lib.fef_coulomb_field(None, None, None, None, None, None, 0, None) == F.FEF_E_ARG
    assert lib.fef_scf_step(None, None, None, None, None, None, None, None, None, None, None,
                            0, None) == F.FEF_E_ARG
    assert lib.fef_coupled_pair_energies(None, None, None, None, None, 1e-14, 10, None, None,
                                         None, None, None, 0, None) == F.FEF_E_ARG
    assert lib.fef_dimer_dressing(None, None, None, None, None, 1e-14, 0, None, None, None, None,
                                  None, None, 0, None) == F.FEF_E_ARG
    assert lib.fef_monomer_energies(None, None, None, None, None, None, None,
                                    None) == F.FEF_E_ARG
    xb, yc, us, hit = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
    assert lib.fef_autotune_cached(None, None, None, 3, None, 0, 3, None, b"/tmp/x.json",
                                   ctypes.byref(xb), ctypes.byref(yc), ctypes.byref(us),
                                   ctypes.byref(hit)) == F.FEF_E_ARG


def test_coupled_flag_and_query_constants_match_header():
    import re
    F, lib = _lib()
    txt = open(os.path.join(ROOT, "include", "fef.h")).read()
    assert re.search(rf"#define FEF_FLAG_NOCONV {F.FEF_FLAG_NOCONV}\b", txt)
    assert re.search(rf"#define FEF_E_IO {F.FEF_E_IO}\b", txt)
    assert re.search(rf"FEF_Q_COUPLED_WS_BYTES = {F.Q_COUPLED_WS_BYTES}\b", txt)
    for name in ("DRESSING_WS_BYTES", "HOO_ELEMS", "HVV_ELEMS"):
        assert re.search(rf"FEF_Q_{name} = {getattr(F, 'Q_' + name)}\b", txt), name


def test_bad_shapes_rejected_before_device():
    import numpy as np
    F, lib = _lib()

    def desc(nbf, nocc, cls, naux):
        arrs = [np.array(a, dtype=np.int32) for a in (nbf, nocc, cls, naux)]
        d = F.SystemDesc(len(nbf), len(naux), *(a.ctypes.data for a in arrs), 0,
                         None, None, None)
        return d, arrs
    h = ctypes.c_void_p()
    for args in [([4], [5], [0], [3]),      # nocc > nbf
                 ([4], [-1], [0], [3]),     # negative nocc
                 ([4], [2], [1], [3]),      # class out of range
                 ([4], [2], [0], [0]),      # zero factor rank
                 ([0], [0], [0], [3])]:     # empty fragment
        d, keep = desc(*args)
        assert lib.fef_plan_create(ctypes.byref(d), ctypes.byref(h)) == F.FEF_E_SHAPE


def test_missing_library_fails_loudly(tmp_path):
    from paper_1708_03377_amd import _fef
    with pytest.raises(RuntimeError, match="missing"):
        _fef.load_library(str(tmp_path / "libfef.so"))


def test_surrogate_entry_points_reject_bad_arguments():
    F, lib = _lib()
    out = ctypes.c_int64()
    assert lib.fef_pair_energies_masked(None, None, None, 0, None, None, None, None, None, 0,
                                        None) == F.FEF_E_ARG
    assert lib.fef_coupling_modes(None, None, None, None, 0, None) == F.FEF_E_ARG
    assert lib.fef_fragment_invariants(None, None, None, None, None, None, None, 0,
                                       None) == F.FEF_E_ARG
    assert lib.fef_pair_features(None, None, None, None, 0, None, None, None) == F.FEF_E_ARG
    assert lib.fef_column_stats(10, 0, 0, None, None, None, None) == F.FEF_E_ARG
    assert lib.fef_mlp_pack(0, None, None, None) == F.FEF_E_ARG
    assert lib.fef_mlp_forward(0, 1, None, None, None, None, None) == F.FEF_E_ARG
    assert lib.fef_mlp_forward(65, 1, None, None, None, None, None) == F.FEF_E_ARG
    assert lib.fef_mlp_train_ws_bytes(0, 10, ctypes.byref(out)) == F.FEF_E_ARG
    assert lib.fef_mlp_train_ws_bytes(5, 64, ctypes.byref(out)) == F.FEF_OK
    # 2 blocks of 32 rows per member: partial gradients + partial losses
    assert out.value >= 5 * 2 * F.MLP_STRIDE * 4 + 5 * 2 * 4
    assert lib.fef_mlp_train_step(5, None, None, None, 8, None, None, None, None, None, 1,
                                  ctypes.c_float(1e-3), None, None, None, 0,
                                  None) == F.FEF_E_ARG
    assert lib.fef_surrogate_select(None, None, 5, None, None, 0.0, 0.0, None, None,
                                    None) == F.FEF_E_ARG
    assert lib.fef_pack_coefficients(None, None, None, None) == F.FEF_E_ARG
    assert lib.fef_scf_step_packed(None, None, None, None, None, None, None, None, None, None,
                                   None, 0, None) == F.FEF_E_ARG


def test_mlp_layout_constants_match_header():
    import fefgen
    F, _ = _lib()
    txt = open(os.path.join(ROOT, "include", "fef.h")).read()
    for name, val in (("FEF_MLP_NIN", F.MLP_NIN), ("FEF_MLP_NHID", F.MLP_NHID),
                      ("FEF_MLP_NPARAM", F.MLP_NPARAM), ("FEF_MLP_STRIDE", F.MLP_STRIDE),
                      ("FEF_MLP_NSTATS", F.MLP_NSTATS)):
        assert re.search(rf"#define {name} {val}\b", txt), name
    assert fefgen.MLP_STRIDE == F.MLP_STRIDE
    sizes = [17 * 128, 128, 128 * 128, 128, 128, 1]
    assert sum(sizes) == F.MLP_NPARAM
