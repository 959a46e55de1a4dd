"""MI355X (gfx950) FEF pair energies and effective-field SCF.

The computation lives in the HIP library ``libfef.so`` behind the C ABI of
include/fef.h; ``_fef`` binds it with ctypes and ``runtime.Context`` holds the
device buffers of one fragment system.
"""
from . import _fef  # noqa: F401
from ._fef import (PREC, FefError, fef_coulomb_field, fef_half_transform,  # noqa: F401
                   fef_pair_energies, fef_plan_create, fef_plan_get_tiles, fef_plan_query,
                   fef_plan_set_tiles, fef_scf_step, fef_graph_create, fef_graph_launch,
                   fef_autotune, fef_pair_energies_masked, fef_coupling_modes,
                   fef_fragment_invariants, fef_pair_features, fef_column_stats, fef_mlp_pack,
                   fef_mlp_forward, fef_mlp_train_step, fef_mlp_train_ws_bytes,
                   fef_surrogate_select, fef_pack_coefficients, fef_scf_step_packed,
                   fef_status_string, load_library)


def Context(*args, **kwargs):
    from .runtime import Context as _C
    return _C(*args, **kwargs)


def Ensemble(*args, **kwargs):
    from .surrogate import Ensemble as _E
    return _E(*args, **kwargs)
