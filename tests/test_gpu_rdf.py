"""Pair distance histogram (pair correlation function) over a box-only cluster-pair list on the GPU, against
the oracle's: bit-exact integer counts (the FP32 bin decisions are formed identically on both sides)."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4), (4, 8), (8, 4), (8, 8)]


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu-case] %s" % request.node.nodeid, file=sys.stderr, flush=True)
    yield


@pytest.fixture(scope="module")
def c1():
    return synth.water_box(1000, 3.104, seed=1306)


def _gpu_rdf(mxn, torch, ctx, box, x, shape, r_max, nbins, skip, margin=0.01, reps=1):
    dev = torch.device("cuda:0")
    xq = torch.from_numpy(box.xyzq(x)).to(dev)
    typ = torch.from_numpy(box.type).to(dev)
    eo = torch.from_numpy(box.excl_off).to(dev)
    ei = torch.from_numpy(box.excl_idx).to(dev)
    rl = r_max + margin
    g = mxn.nb_grid_sort(ctx, box.box, xq, typ, shape)
    lst = mxn.nb_pairlist_build(ctx, g, rl, rl, eo, ei)      # box-only list: no particle prune
    hist = torch.zeros(2 * 2 * nbins, dtype=torch.int64, device=dev)
    for _ in range(reps):
        mxn.nb_rdf(ctx, g, lst, xq, r_max, nbins, 2, hist, skip_excluded=skip)
    mxn.nb_sync(ctx)
    out = hist.cpu().numpy().astype(np.uint64).reshape(2, 2, nbins)
    mxn.nb_list_free(lst)
    mxn.nb_grid_free(g)
    return out


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("skip", [False, True])
def test_rdf_bitexact(c1, shape, skip):
    import torch
    import paper_1306_1737_amd as mxn
    ctx = mxn.nb_create(0)
    try:
        r_max, nbins = 1.0, 400
        got = _gpu_rdf(mxn, torch, ctx, c1, c1.xyz, shape, r_max, nbins, skip)
        g = oracle.grid_sort(c1.xyz, c1.box, *shape)
        ref = oracle.rdf(g, g["xs"], c1.type, c1.box, r_max, nbins, 2, c1.excl_off, c1.excl_idx, skip)
        np.testing.assert_array_equal(got, ref)
        assert int(ref.sum()) > 500_000       # ~ n (4 pi r^3 / 3) rho / 2 = 6.3e5 pairs within 1 nm
    finally:
        mxn.nb_destroy(ctx)


@pytest.mark.parametrize("shape", [(4, 4), (8, 8)])
def test_rdf_moved_positions_and_accumulation(c1, shape):
    """At later positions with the list built there (a list every evaluation); two calls add up."""
    import torch
    import paper_1306_1737_amd as mxn
    ctx = mxn.nb_create(0)
    try:
        x5 = synth.free_flight(c1.xyz, synth.velocities(c1.mass, 300.0, seed=23), 0.002, 6)[5].astype(np.float32)
        r_max, nbins = 0.9, 333
        got = _gpu_rdf(mxn, torch, ctx, c1, x5, shape, r_max, nbins, False, reps=2)
        g = oracle.grid_sort(x5, c1.box, *shape)
        ref = oracle.rdf(g, g["xs"], c1.type, c1.box, r_max, nbins, 2, c1.excl_off, c1.excl_idx)
        np.testing.assert_array_equal(got, 2 * ref)
    finally:
        mxn.nb_destroy(ctx)


def test_rdf_errors(c1):
    import torch
    import paper_1306_1737_amd as mxn
    from tests._nb import GpuSystem
    s = GpuSystem(c1, (8, 8), 1.0, rbb=1.0)
    try:
        hist = torch.zeros(4 * 400, dtype=torch.int64, device=s.dev)
        with pytest.raises(mxn.NbError):
            mxn.nb_rdf(s.ctx, s.grid, s.lst, s.xyzq, 1.2, 400, 2, hist)        # beyond the list radius
        big = torch.zeros(4 * 20000, dtype=torch.int64, device=s.dev)
        with pytest.raises(mxn.NbError):
            mxn.nb_rdf(s.ctx, s.grid, s.lst, s.xyzq, 1.0, 20000, 2, big)       # LDS histogram too large
        mxn.nb_rdf(s.ctx, s.grid, s.lst, s.xyzq, 1.0, 400, 2, hist)
        mxn.nb_sync(s.ctx)
        assert int(hist.sum().item()) > 0
    finally:
        s.close()
