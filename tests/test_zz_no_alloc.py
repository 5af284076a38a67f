"""nb_forces_noalloc: the allocation-free variant of nb_forces, through the C ABI.

Its energy/virial partials live in a static device array of the library, so the call allocates nothing.
Two calls in a row -- the 96 000-atom production box, then a smaller 3 000-atom box on the same GPU (the
array keeps the first call's contents) -- must each reproduce nb_forces on the same list bit for bit, and
neither may change the context's or torch's device memory.
"""
import sys

import numpy as np
import pytest

import synth
from tests._nb import F

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu-case] %s" % request.node.nodeid, file=sys.stderr, flush=True)
    yield


def _system(mxn, torch, ctx, box, shape, rlist):
    dev = torch.device("cuda:0")
    s = dict(xyzq=torch.from_numpy(box.xyzq()).to(dev), type=torch.from_numpy(box.type).to(dev),
             eo=torch.from_numpy(box.excl_off).to(dev), ei=torch.from_numpy(box.excl_idx).to(dev), n=box.n)
    s["grid"] = mxn.nb_grid_sort(ctx, box.box, s["xyzq"], s["type"], shape)
    s["lst"] = mxn.nb_pairlist_build(ctx, s["grid"], rlist, -1.0, s["eo"], s["ei"])
    return s


def _run(mxn, torch, fn, ctx, s, params, flags):
    dev = torch.device("cuda:0")
    f = torch.full((s["n"], 3), 7.0, dtype=torch.float32, device=dev)
    e = torch.full((2,), 7.0, dtype=torch.float64, device=dev)
    v = torch.full((9,), 7.0, dtype=torch.float64, device=dev)
    fn(ctx, s["grid"], s["lst"], s["xyzq"], params, flags, f, e, v)
    mxn.nb_sync(ctx)
    return f.cpu().numpy(), e.cpu().numpy(), v.cpu().numpy()


def test_noalloc_matches_nb_forces_on_two_calls():
    import torch
    import paper_1306_1737_amd as mxn
    dev = torch.device("cuda:0")
    lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
    ctx = mxn.nb_create(0)
    big = small = None
    try:
        big = _system(mxn, torch, ctx, synth.water_box(32000, 9.86, seed=1306), (8, 8), 1.1)
        small = _system(mxn, torch, ctx, synth.water_box(1000, 3.104, seed=1306), (4, 4), 0.9)
        p_big = mxn.make_params(1.0, 3.12, F, lj)
        p_small = mxn.make_params(0.9, 3.47, F, lj)
        fl = mxn.NB_ENERGY | mxn.NB_VIRIAL
        ref_big = _run(mxn, torch, mxn.nb_forces, ctx, big, p_big, fl)
        ref_small = _run(mxn, torch, mxn.nb_forces, ctx, small, p_small, fl)
        ref_small_f = _run(mxn, torch, mxn.nb_forces, ctx, small, p_small, 0)
        torch.cuda.synchronize()
        held, torch_held = mxn.nb_memory_info(ctx), torch.cuda.memory_allocated(0)
        got_big = _run(mxn, torch, mxn.nb_forces_noalloc, ctx, big, p_big, fl)
        got_small = _run(mxn, torch, mxn.nb_forces_noalloc, ctx, small, p_small, fl)
        got_small_f = _run(mxn, torch, mxn.nb_forces_noalloc, ctx, small, p_small, 0)
        torch.cuda.synchronize()
        # the buffers the calls fill were allocated before the measurement; the calls themselves add nothing
        assert mxn.nb_memory_info(ctx) == held
        assert torch.cuda.memory_allocated(0) == torch_held   # the output tensors of _run are gone again
        for got, ref in ((got_big, ref_big), (got_small, ref_small)):
            np.testing.assert_array_equal(got[0].view(np.uint32), ref[0].view(np.uint32))
            np.testing.assert_array_equal(got[1], ref[1])
            np.testing.assert_array_equal(got[2], ref[2])
        np.testing.assert_array_equal(got_small_f[0].view(np.uint32), ref_small_f[0].view(np.uint32))
        # outputs not requested are left untouched
        assert np.all(got_small_f[1] == 7.0) and np.all(got_small_f[2] == 7.0)
        # the variant that needs a device table, and a list too large for the scratch, are refused
        with pytest.raises(mxn.NbError) as ei:
            _run(mxn, torch, mxn.nb_forces_noalloc, ctx, small,
                 mxn.make_params(0.9, 3.47, F, lj, True, mxn.NB_COULOMB_EWALD_TABLE), fl)
        assert ei.value.status == mxn.NB_ERR_UNSUPPORTED
        wide = _system(mxn, torch, ctx, synth.water_box(32000, 9.86, seed=1306), (4, 4), 2.4)
        with pytest.raises(mxn.NbError) as ei:
            _run(mxn, torch, mxn.nb_forces_noalloc, ctx, wide, p_big, fl)
        assert ei.value.status == mxn.NB_ERR_UNSUPPORTED
        mxn.nb_list_free(wide["lst"])
        mxn.nb_grid_free(wide["grid"])
    finally:
        for s in (big, small):
            if s is not None:
                mxn.nb_list_free(s["lst"])
                mxn.nb_grid_free(s["grid"])
        mxn.nb_destroy(ctx)
