"""The allocation-free pair-energy entry point against fef_pair_energies,
through the C ABI: two calls in a row on the same GPU (the library's fixed
scratch array keeps the first call's contents), the second on a smaller
system; every result bitwise equal to the workspace entry point's, which
runs the same kernels with the same tiling."""
import numpy as np
import pytest

import fefgen

pytestmark = pytest.mark.gpu

PREC = {"f64": 0, "f32": 1, "bf16x2": 2, "fp16x2": 3}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def run_both(torch, sysm, prec):
    import paper_1708_03377_amd as lib
    from paper_1708_03377_amd import _fef
    ctx = lib.Context(sysm)
    ctx.half_transform(prec)
    ref, ref_tot = ctx.pair_energies(prec)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy().copy()
    ref_tot = float(ref_tot.cpu()[0])
    flags_ref = int(ctx.flags.cpu()[0])
    E2 = torch.full((max(ctx.npair, 1),), float("nan"), dtype=torch.float64, device="cuda")
    tot = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    _fef.fef_pair_energies_noalloc(ctx.plan, ctx.ops_for(prec), ctx.eps, prec, E2, tot, flags,
                                   ctx.stream())
    torch.cuda.synchronize()
    got = E2[:ctx.npair].cpu().numpy()
    assert np.array_equal(got, ref)
    assert float(tot.cpu()[0]) == ref_tot
    assert int(flags.cpu()[0]) == flags_ref
    return ctx.npair


@pytest.mark.parametrize("prec", ["f64", "fp16x2"])
def test_noalloc_matches_workspace_entry_point(torch, prec):
    p = PREC[prec]
    big = fefgen.make_system(1, n_water=300, cutoff=10.0)
    small = fefgen.make_system(0)
    n1 = run_both(torch, big, p)
    n2 = run_both(torch, small, p)
    assert n2 < n1

