"""Two-stage list on the GPU (Sec. 2.3: bounding-box search, then a particle-distance prune) through the C ABI,
against the CPU oracle: the pruned list bit-exact, forces on it within 1e-5 relative RMS of FP64."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._nb import F, GpuSystem, rel_rms

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4), (4, 8), (8, 4), (8, 8)]


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu-case] %s" % request.node.nodeid, file=sys.stderr, flush=True)
    yield


@pytest.fixture(scope="module")
def c1():
    return synth.water_box(1000, 3.104, seed=1306)


def _cmp(gpu, ref):
    assert len(gpu) == len(ref), (len(gpu), len(ref))
    for k in ("ci", "shift", "cj", "mask"):
        np.testing.assert_array_equal(gpu[k], ref[k], err_msg=k)


@pytest.mark.parametrize("shape", SHAPES)
def test_box_only_then_prune_equals_one_stage(c1, shape):
    """At the build positions, a box-only list (rbb = rlist) pruned at rlist is the one-stage list with rbb = 0."""
    rl = 1.0
    s = GpuSystem(c1, shape, rl, rbb=rl)   # box-only outer list
    try:
        mxn = s.mxn
        inner = mxn.nb_pairlist_prune(s.ctx, s.lst, s.xyzq, rl)
        one = mxn.nb_pairlist_build(s.ctx, s.grid, rl, 0.0, s.eo, s.ei)
        got = mxn.nb_list_export_canonical(inner)
        _cmp(got, mxn.nb_list_export_canonical(one))
        g = oracle.grid_sort(c1.xyz, c1.box, *shape)
        _cmp(got, oracle.pairlist(g, c1.box, np.float32(rl), np.float32(0.0), c1.excl_off, c1.excl_idx))
        assert len(mxn.nb_list_export_canonical(s.lst)) > len(got)
        mxn.nb_list_free(inner)
        mxn.nb_list_free(one)
    finally:
        s.close()


@pytest.mark.parametrize("shape", [(4, 4), (8, 4), (8, 8)])
@pytest.mark.parametrize("order", [0, 2], ids=["canonical", "distance"])   # NB_LIST_BY_DISTANCE = 2
def test_rolling_prune_after_motion(c1, shape, order):
    """A box-only outer list at 1.2 nm built once; pruned at 1.0 nm at later positions (free flight, steps 4
    and 9), reusing one inner handle: bit-exact against the oracle's prune, and forces on the pruned list at
    those positions match the FP64 oracle and the outer list's forces."""
    rl, rc, beta = 1.2, 1.0, 3.12
    s = GpuSystem(c1, shape, rl, rbb=rl, flags=order)
    try:
        mxn, torch = s.mxn, s.torch
        g = oracle.grid_sort(c1.xyz, c1.box, *shape)
        outer_ref = oracle.pairlist(g, c1.box, np.float32(rl), np.float32(rl), c1.excl_off, c1.excl_idx)
        _cmp(mxn.nb_list_export_canonical(s.lst), outer_ref)
        v = synth.velocities(c1.mass, 300.0, seed=17)
        traj = synth.free_flight(c1.xyz, v, 0.002, 10)
        inner = None
        for step in (4, 9):
            x = traj[step].astype(np.float32)
            xq = torch.from_numpy(c1.xyzq(x)).to(s.dev)
            inner = mxn.nb_pairlist_prune(s.ctx, s.lst, xq, rc, inner)
            ref = oracle.prune(g, oracle.gather(g, x, c1.box), c1.box, outer_ref, np.float32(rc))
            got = mxn.nb_list_export_canonical(inner)
            _cmp(got, ref)
            assert len(got) < len(outer_ref)
            fl = mxn.NB_ENERGY | mxn.NB_VIRIAL
            f_in, e_in, v_in = _forces(mxn, torch, s, inner, xq, rc, beta, fl)
            f_out, e_out, _ = _forces(mxn, torch, s, s.lst, xq, rc, beta, fl)
            fr, er, _ = oracle.forces(x, c1.q, c1.type, c1.box, c1.excl_off, c1.excl_idx, synth.lj_table_spce(),
                                      rc, beta, F, mode="brute")
            assert rel_rms(f_in, fr) <= 1e-5
            assert rel_rms(f_in, f_out) <= 1e-6
            np.testing.assert_allclose(e_in, er, rtol=1e-5)
            np.testing.assert_allclose(e_in, e_out, rtol=1e-6)
        mxn.nb_list_free(inner)
    finally:
        s.close()


def _forces(mxn, torch, s, lst, xq, rc, beta, flags):
    f = torch.zeros((s.box.n, 3), dtype=torch.float32, device=s.dev)
    e = torch.zeros(2, dtype=torch.float64, device=s.dev)
    v = torch.zeros(9, dtype=torch.float64, device=s.dev)
    mxn.nb_forces(s.ctx, s.grid, lst, xq, mxn.make_params(rc, beta, F, s.lj), flags, f, e, v)
    mxn.nb_sync(s.ctx)
    return f.cpu().numpy().astype(np.float64), e.cpu().numpy(), v.cpu().numpy()


def test_prune_errors_and_overflow(c1):
    shape, rl = (8, 8), 1.0
    s = GpuSystem(c1, shape, rl, rbb=rl)
    try:
        mxn = s.mxn
        with pytest.raises(mxn.NbError):
            mxn.nb_pairlist_prune(s.ctx, s.lst, s.xyzq, 0.0)
        with pytest.raises(mxn.NbError):
            mxn.nb_pairlist_prune(s.ctx, s.lst, s.xyzq, rl, s.lst)
        inner = mxn.nb_pairlist_prune(s.ctx, s.lst, s.xyzq, rl)
        mxn.nb_sync(s.ctx)
        # an asynchronous rebuild at a much larger radius overflows the outer list's regions ...
        s.lst = mxn.nb_pairlist_build(s.ctx, s.grid, 1.45, 1.45, s.eo, s.ei, mxn.NB_LIST_ASYNC, s.lst)
        with pytest.raises(mxn.NbError) as err:
            mxn.nb_sync(s.ctx)
        assert err.value.status == -5
        # ... and the prune of an overflowed list reports the overflow too
        inner = mxn.nb_pairlist_prune(s.ctx, s.lst, s.xyzq, rl, inner)
        with pytest.raises(mxn.NbError) as err:
            mxn.nb_sync(s.ctx)
        assert err.value.status == -5
        mxn.nb_list_free(inner)
    finally:
        s.close()


def test_production_box_rolling_prune():
    """The benchmark's rolling schedule on the 96k-atom production box: a box-only outer list at 1.3 nm,
    pruned at 1.05 nm at free-flight steps 20 and 39 (80 fs, where atoms of different waters have passed
    within 0.08 nm of each other).  Outer and inner lists bit-exact against the oracle on sampled
    i-clusters, and at step 39 the forces on the pruned list match the FP64 oracle everywhere."""
    box = synth.water_box(32000, 9.86, seed=1306)
    r_out, r_in, rc, beta = 1.3, 1.05, 1.0, 3.12
    s = GpuSystem(box, (8, 8), r_out, rbb=r_out)
    try:
        mxn, torch = s.mxn, s.torch
        g = oracle.grid_sort(box.xyz, box.box, 8, 8)
        nci = g["n_slots"] // 8
        outer = mxn.nb_list_export_canonical(s.lst)
        ranges = [(0, 40), (nci // 2, nci // 2 + 40), (nci - 40, nci)]
        sub = []
        for c0, c1_ in ranges:
            ref = oracle.pairlist(g, box.box, np.float32(r_out), np.float32(r_out), box.excl_off, box.excl_idx,
                                  c0, c1_)
            sel = outer[(outer["ci"] >= c0) & (outer["ci"] < c1_)]
            _cmp(sel, ref)
            sub.append(ref)
        traj = synth.free_flight(box.xyz, synth.velocities(box.mass, 300.0, seed=1306), 0.002, 40)
        inner = None
        for step in (20, 39):
            x = traj[step].astype(np.float32)
            xq = torch.from_numpy(box.xyzq(x)).to(s.dev)
            inner = mxn.nb_pairlist_prune(s.ctx, s.lst, xq, r_in, inner)
            got = mxn.nb_list_export_canonical(inner)
            xs_now = oracle.gather(g, x, box.box)
            for (c0, c1_), ref_out in zip(ranges, sub):
                ref = oracle.prune(g, xs_now, box.box, ref_out, np.float32(r_in))
                _cmp(got[(got["ci"] >= c0) & (got["ci"] < c1_)], ref)
        f, e, _ = _forces(mxn, torch, s, inner, xq, rc, beta, mxn.NB_ENERGY)
        assert np.isfinite(f).all()
        fr, er, _ = oracle.forces(x, box.q, box.type, box.box, box.excl_off, box.excl_idx, synth.lj_table_spce(),
                                  rc, beta, F, mode="binned")
        assert rel_rms(f, fr) <= 1e-5
        np.testing.assert_allclose(e, er, rtol=1e-5)
        mxn.nb_list_free(inner)
    finally:
        s.close()
