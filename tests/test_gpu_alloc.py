"""Device memory through the caller's allocator (the nb_allocator argument of nb_create).

With PyTorch's caching allocator behind a context, every device buffer of the context and its handles --
grid, list, force rows and partials, batch tables, the learned-buffer model -- comes from torch's pool and
none from the library's own hipMalloc; freeing the handles returns it all.  Results do not depend on where
the memory came from.
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


def _cycle(mxn, torch, ctx, box, lj):
    dev = torch.device("cuda:0")
    xyzq = torch.from_numpy(box.xyzq()).to(dev)
    typ = torch.from_numpy(box.type).to(dev)
    eo = torch.from_numpy(box.excl_off).to(dev)
    ei = torch.from_numpy(box.excl_idx).to(dev)
    v = synth.velocities(box.mass, 300.0, seed=3)
    xs = [torch.from_numpy(box.xyzq(x)).to(dev) for x in synth.free_flight(box.xyz, v, 0.002, 10)]
    grid = mxn.nb_grid_sort(ctx, box.box, xyzq, typ, (8, 8))
    lst = mxn.nb_pairlist_build(ctx, grid, 1.1, -1.0, eo, ei)
    lst = mxn.nb_pairlist_build(ctx, grid, 1.1, -1.0, eo, ei, mxn.NB_LIST_ASYNC, lst)
    f = torch.zeros((box.n, 3), dtype=torch.float32, device=dev)
    e = torch.zeros(2, dtype=torch.float64, device=dev)
    vir = torch.zeros(9, dtype=torch.float64, device=dev)
    p = mxn.make_params(1.0, 3.12, F, lj)
    for k in range(10):
        mxn.nb_forces(ctx, grid, lst, xs[k], p, mxn.NB_ENERGY | mxn.NB_VIRIAL, f, e, vir)
    mxn.nb_sync(ctx)
    return grid, lst, f.cpu().numpy(), e.cpu().numpy(), vir.cpu().numpy()


def test_torch_allocator_backs_every_buffer():
    import torch
    import paper_1306_1737_amd as mxn
    box = synth.water_box(2000, synth.box_edge_for(2000), seed=21)
    dev = torch.device("cuda:0")
    lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    ctx = mxn.nb_create(0, allocator="torch")
    ref = mxn.nb_create(0, allocator=None)
    try:
        grid, lst, f, e, v = _cycle(mxn, torch, ctx, box, lj)
        # a batch of two replicas and a model on the same context
        batch = mxn.nb_batch_create(ctx, [grid], [lst], [torch.from_numpy(box.xyzq()).to(dev)],
                                    [torch.zeros((box.n, 3), dtype=torch.float32, device=dev)])
        model = mxn.nb_mlp_create(ctx, np.zeros(mxn.NB_MLP_PARAMS, np.float32), np.zeros(8), np.ones(8))
        via_alloc, via_hip = mxn.nb_memory_info(ctx)
        assert via_hip == 0
        assert via_alloc > 12 * box.n
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated(0) - base >= via_alloc
        # the same cycle on library-allocated memory gives bit-identical results
        grid2, lst2, f2, e2, v2 = _cycle(mxn, torch, ref, box, lj)
        assert mxn.nb_memory_info(ref)[0] == 0 and mxn.nb_memory_info(ref)[1] > 0
        np.testing.assert_array_equal(f.view(np.uint32), f2.view(np.uint32))
        np.testing.assert_array_equal(e, e2)
        np.testing.assert_array_equal(v, v2)
        mxn.nb_list_free(lst2)
        mxn.nb_grid_free(grid2)
        mxn.nb_mlp_free(model)
        mxn.nb_batch_free(batch)
        del batch   # the binding's handle keeps the replica tensors it was given alive
        mxn.nb_list_free(lst)
        mxn.nb_grid_free(grid)
        # the handles' memory is back; what is left is the context's own scratch (energy partials, flags),
        # returned by nb_destroy (checked against torch below)
        left = mxn.nb_memory_info(ctx)[0]
        assert left < via_alloc // 2
    finally:
        mxn.nb_destroy(ctx)
        mxn.nb_destroy(ref)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == base   # every block went back to torch


def test_allocator_out_of_memory_is_reported():
    import paper_1306_1737_amd as mxn
    import torch
    calls = []

    def _alloc(nbytes, stream, user):
        calls.append(nbytes)
        return None if nbytes > 1 << 20 else torch.cuda.caching_allocator_alloc(int(nbytes), device=0,
                                                                                 stream=int(stream or 0))

    def _free(ptr, stream, user):
        torch.cuda.caching_allocator_delete(ptr)

    al = mxn.nb_allocator(mxn._ALLOC_FN(_alloc), mxn._FREE_FN(_free), None)
    ctx = mxn.nb_create(0, allocator=al)
    try:
        box = synth.water_box(32000, 9.86, seed=1306)
        dev = torch.device("cuda:0")
        xyzq = torch.from_numpy(box.xyzq()).to(dev)
        typ = torch.from_numpy(box.type).to(dev)
        with pytest.raises(mxn.NbError) as ei:
            mxn.nb_grid_sort(ctx, box.box, xyzq, typ, (8, 8))
        assert ei.value.status == mxn.NB_ERR_OOM
        assert calls and max(calls) > 1 << 20
    finally:
        mxn.nb_destroy(ctx)
