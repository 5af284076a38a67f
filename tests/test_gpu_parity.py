"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: grid sort, bounding boxes and the canonical cluster-pair list bit-exact;
forces within 1e-5 relative RMS of FP64; energies and virial (FP64
accumulation of FP32 pair terms) within 1e-5 relative.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._nb import F, GpuSystem, default_rbb, max_atom_err, rel_rms

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4), (4, 8), (8, 4), (8, 8)]


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu-case] %s" % request.node.nodeid, file=sys.stderr, flush=True)
    yield


@pytest.fixture(scope="module")
def c1():
    return synth.water_box(1000, 3.104, seed=1306)


@pytest.fixture(scope="module")
def ragged():
    # 97 waters: 291 atoms, no column holds a multiple of the cluster size
    return synth.water_box(97, 2.47, seed=97)


def _oracle_bb(g, m):
    xs, perm = g["xs"], g["perm"]
    nci = g["n_slots"] // m
    lo = np.full((nci, 3), np.inf, np.float32)
    hi = np.full((nci, 3), -np.inf, np.float32)
    for c in range(nci):
        real = [s for s in range(c * m, c * m + m) if perm[s] >= 0]
        if real:
            lo[c] = xs[real].min(0)
            hi[c] = xs[real].max(0)
    return lo, hi


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("which", ["c1", "ragged"])
def test_grid_sort_bitexact(shape, which, request):
    box = request.getfixturevalue(which)
    s = GpuSystem(box, shape, 1.0)
    try:
        ex = s.mxn.nb_grid_export(s.grid)
        g = oracle.grid_sort(box.xyz, box.box, *shape)
        info = ex["info"]
        assert (info["nx"], info["ny"], info["n_slots"]) == (g["nx"], g["ny"], g["n_slots"])
        np.testing.assert_array_equal(ex["col_start"], g["col_start"])
        np.testing.assert_array_equal(ex["perm"], g["perm"])
        np.testing.assert_array_equal(ex["img"], g["img"])
        real = g["perm"] >= 0
        # bit-exact wrapped coordinates
        np.testing.assert_array_equal(ex["xyzq"][real, :3].view(np.uint32), g["xs"][real].view(np.uint32))
        np.testing.assert_array_equal(ex["xyzq"][real, 3], box.q[g["perm"][real]])
        assert np.all(ex["xyzq"][~real, 3] == 0)
        lo, hi = _oracle_bb(g, shape[0])
        np.testing.assert_array_equal(ex["bb"][:, :3], lo)
        np.testing.assert_array_equal(ex["bb"][:, 4:7], hi)
    finally:
        s.close()


def _cmp_lists(gpu, ref):
    assert len(gpu) == len(ref), (len(gpu), len(ref))
    for k in ("ci", "shift", "cj", "mask"):
        np.testing.assert_array_equal(gpu[k], ref[k], err_msg=k)


@pytest.mark.parametrize("shape,rlist", [((4, 4), 0.9), ((4, 8), 0.9), ((8, 4), 0.9), ((8, 8), 0.9), ((4, 4), 1.1),
                                         ((8, 4), 1.1), ((8, 8), 1.1), ((4, 8), 1.2)])
def test_pairlist_bitexact(c1, shape, rlist):
    rbb = np.float32(default_rbb(c1, shape, rlist))
    s = GpuSystem(c1, shape, rlist, rbb=float(rbb))
    try:
        gpu = s.mxn.nb_list_export_canonical(s.lst)
        g = oracle.grid_sort(c1.xyz, c1.box, *shape)
        ref = oracle.pairlist(g, c1.box, np.float32(rlist), rbb, c1.excl_off, c1.excl_idx)
        _cmp_lists(gpu, ref)
    finally:
        s.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_async_rebuild_in_reserved_regions(c1, shape):
    """An asynchronous rebuild (one search pass into the regions a synchronous build reserved) after the
    particles moved equals the oracle's list for the new positions; a rebuild that outgrows the regions is
    reported, and a synchronous build then re-reserves."""
    rlist = 1.0
    rbb = np.float32(default_rbb(c1, shape, rlist))
    v = synth.velocities(c1.mass, 300.0, seed=11)
    x9 = synth.free_flight(c1.xyz, v, 0.002, 10)[9].astype(np.float32)
    s = GpuSystem(c1, shape, rlist, rbb=float(rbb))
    try:
        mxn, torch = s.mxn, s.torch
        xq9 = torch.from_numpy(c1.xyzq(x9)).to(s.dev)
        s.grid = mxn.nb_grid_sort(s.ctx, c1.box, xq9, s.type, shape, s.grid)
        s.lst = mxn.nb_pairlist_build(s.ctx, s.grid, rlist, float(rbb), s.eo, s.ei, mxn.NB_LIST_ASYNC, s.lst)
        mxn.nb_sync(s.ctx)
        g = oracle.grid_sort(x9, c1.box, *shape)
        _cmp_lists(mxn.nb_list_export_canonical(s.lst),
                   oracle.pairlist(g, c1.box, np.float32(rlist), rbb, c1.excl_off, c1.excl_idx))
        # a much larger radius cannot fit the regions reserved at rlist = 1.0
        big = 1.45
        rbb2 = np.float32(default_rbb(c1, shape, big))
        s.lst = mxn.nb_pairlist_build(s.ctx, s.grid, big, float(rbb2), s.eo, s.ei, mxn.NB_LIST_ASYNC, s.lst)
        with pytest.raises(mxn.NbError) as err:
            mxn.nb_sync(s.ctx)
        assert err.value.status == mxn.NB_ERR_OVERFLOW
        s.lst = mxn.nb_pairlist_build(s.ctx, s.grid, big, float(rbb2), s.eo, s.ei, 0, s.lst)
        mxn.nb_sync(s.ctx)
        _cmp_lists(mxn.nb_list_export_canonical(s.lst),
                   oracle.pairlist(g, c1.box, np.float32(big), rbb2, c1.excl_off, c1.excl_idx))
    finally:
        s.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_pairlist_same_for_every_search_split(c1, shape):
    """Wavefronts sharing one i-cluster's search (1, 2, 4, 8) change only the order of its entries."""
    rbb = np.float32(default_rbb(c1, shape, 1.0))
    g = oracle.grid_sort(c1.xyz, c1.box, *shape)
    ref = oracle.pairlist(g, c1.box, np.float32(1.0), rbb, c1.excl_off, c1.excl_idx)
    s = GpuSystem(c1, shape, 1.0, rbb=float(rbb))
    try:
        for parts in (1, 2, 4, 8, 0):
            s.mxn.nb_set_search_parts(s.ctx, parts)
            lst = s.mxn.nb_pairlist_build(s.ctx, s.grid, 1.0, float(rbb), s.eo, s.ei)
            try:
                _cmp_lists(s.mxn.nb_list_export_canonical(lst), ref)
            finally:
                s.mxn.nb_list_free(lst)
        with pytest.raises(s.mxn.NbError):
            s.mxn.nb_set_search_parts(s.ctx, 3)
    finally:
        s.close()


@pytest.mark.parametrize("rbb", [0.0, 1.0])
def test_pairlist_rbb_extremes(ragged, rbb):
    """rbb = 0: every pair checked at particle level; rbb = rlist: bounding boxes alone decide."""
    for shape in SHAPES:
        s = GpuSystem(ragged, shape, 1.0, rbb=rbb)
        try:
            gpu = s.mxn.nb_list_export_canonical(s.lst)
            g = oracle.grid_sort(ragged.xyz, ragged.box, *shape)
            _cmp_lists(gpu, oracle.pairlist(g, ragged.box, np.float32(1.0), np.float32(rbb), ragged.excl_off,
                                             ragged.excl_idx))
        finally:
            s.close()


def test_pairlist_deterministic(c1):
    """Two builds give the same list; the distance-ordered storage exports the same canonical list and the
    same forces."""
    s = GpuSystem(c1, (8, 8), 1.1)
    try:
        a = s.mxn.nb_list_export_canonical(s.lst)
        f0, e0, _ = s.forces(1.0, 3.12, s.mxn.NB_ENERGY)
        s.lst = s.mxn.nb_pairlist_build(s.ctx, s.grid, 1.1, -1.0, s.eo, s.ei, 0, s.lst)
        b = s.mxn.nb_list_export_canonical(s.lst)
        _cmp_lists(a, b)
        s.lst = s.mxn.nb_pairlist_build(s.ctx, s.grid, 1.1, -1.0, s.eo, s.ei, s.mxn.NB_LIST_BY_DISTANCE, s.lst)
        c = s.mxn.nb_list_export_canonical(s.lst)
        _cmp_lists(a, c)
        f1, e1, _ = s.forces(1.0, 3.12, s.mxn.NB_ENERGY)
        assert rel_rms(f1, f0) <= 1e-6
        np.testing.assert_allclose(e1, e0, rtol=1e-7)
    finally:
        s.close()


def _oracle_forces(box, rc, beta, xyz=None, mode="brute"):
    return oracle.forces(box.xyz if xyz is None else xyz, box.q, box.type, box.box, box.excl_off, box.excl_idx,
                         synth.lj_table_spce(), rc, beta, F, shift=True, mode=mode)


@pytest.mark.parametrize("variant", [0, 2], ids=["direct", "super"])
@pytest.mark.parametrize("shape", SHAPES)
def test_forces_energies_virial(c1, shape, variant):
    rc, rlist, beta = 0.9, 0.9, 3.47
    s = GpuSystem(c1, shape, rlist, variant=variant)
    try:
        f, e, v = s.forces(rc, beta, s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL)
        fr, er, vr = _oracle_forces(c1, rc, beta)
        assert rel_rms(f, fr) <= 1e-5
        np.testing.assert_allclose(e, er, rtol=1e-5)
        assert np.abs(v - vr).max() <= 1e-5 * np.abs(vr).max()
        # force-only kernel: same forces (atomics order aside)
        f2, _, _ = s.forces(rc, beta, 0)
        assert rel_rms(f2, f) <= 1e-6
        # FP32 accumulation variant: same physics, looser sums
        f3, e3, v3 = s.forces(rc, beta, s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL | s.mxn.NB_ACC_FP32)
        np.testing.assert_allclose(e3, er, rtol=1e-4)
    finally:
        s.close()


@pytest.mark.parametrize("variant", [0, 2], ids=["direct", "super"])
@pytest.mark.parametrize("shape", SHAPES)
def test_forces_buffered_after_motion(c1, shape, variant):
    """List built at rlist = rc + 0.1 from step-0 positions, forces at step 9 of ballistic motion (300 K, 2 fs)."""
    rc, rlist, beta = 0.9, 1.0, 3.47
    v = synth.velocities(c1.mass, 300.0, seed=5)
    x9 = synth.free_flight(c1.xyz, v, 0.002, 10)[9]
    s = GpuSystem(c1, shape, rlist, variant=variant)
    try:
        xq = s.torch.from_numpy(c1.xyzq(x9)).to(s.dev)
        f, e, _ = s.forces(rc, beta, s.mxn.NB_ENERGY, xyzq_now=xq)
        fr, er, _ = _oracle_forces(c1, rc, beta, xyz=x9)
        assert rel_rms(f, fr) <= 1e-5
        np.testing.assert_allclose(e, er, rtol=1e-5)
    finally:
        s.close()


def test_accumulate_flag(c1):
    s = GpuSystem(c1, (4, 4), 0.9)
    try:
        mxn, torch = s.mxn, s.torch
        f = torch.ones((c1.n, 3), dtype=torch.float32, device=s.dev)
        p = mxn.make_params(0.9, 3.47, F, s.lj)
        mxn.nb_forces(s.ctx, s.grid, s.lst, s.xyzq, p, mxn.NB_ACCUMULATE, f)
        mxn.nb_sync(s.ctx)
        f0, _, _ = s.forces(0.9, 3.47, 0)
        assert rel_rms(f.cpu().numpy() - 1.0, f0) < 1e-6
    finally:
        s.close()


@pytest.mark.parametrize("variant", [0, 2], ids=["direct", "super"])
@pytest.mark.parametrize("shape", [(4, 8), (8, 4), (8, 8)])
def test_forces_reproducible_across_rebuilds(c1, shape, variant):
    """The j-forces of a j-cluster are summed in fixed point, so the forces do not depend on the order in
    which the list build placed that j-cluster's rows (set by atomics): forces from two separate builds of
    the same list, and from two calls on one build, are bit-identical; the list itself is identical."""
    s = GpuSystem(c1, shape, 1.1, variant=variant)
    try:
        mxn = s.mxn
        fl = mxn.NB_ENERGY | mxn.NB_VIRIAL
        f1, e1, v1 = s.forces(1.0, 3.12, fl)
        f1b, e1b, _ = s.forces(1.0, 3.12, fl)
        ref = mxn.nb_list_export_canonical(s.lst)
        for flags in (0, mxn.NB_LIST_ASYNC):
            s.lst = mxn.nb_pairlist_build(s.ctx, s.grid, 1.1, -1.0, s.eo, s.ei, flags, s.lst)
            _cmp_lists(mxn.nb_list_export_canonical(s.lst), ref)
            f2, e2, v2 = s.forces(1.0, 3.12, fl)
            np.testing.assert_array_equal(f2.view(np.uint64), f1.view(np.uint64))
            np.testing.assert_array_equal(e2, e1)
            np.testing.assert_array_equal(v2, v1)
        np.testing.assert_array_equal(f1b.view(np.uint64), f1.view(np.uint64))
        np.testing.assert_array_equal(e1b, e1)
        fr, er, _ = _oracle_forces(c1, 1.0, 3.12)
        assert rel_rms(f1, fr) <= 1e-5
    finally:
        s.close()


@pytest.mark.parametrize("variant", [0, 2], ids=["direct", "super"])
def test_tiny_and_ragged(ragged, variant):
    """One water in a box; and a ragged 291-atom box, all shapes."""
    one = synth.water_box(1, 2.5, seed=1)
    for box, rc in ((one, 1.0), (ragged, 1.0)):
        fr, er, vr = _oracle_forces(box, rc, 3.12)
        for shape in SHAPES:
            s = GpuSystem(box, shape, rc, variant=variant)
            try:
                f, e, v = s.forces(rc, 3.12, s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL)
                assert rel_rms(f, fr) <= 1e-5
                np.testing.assert_allclose(e, er, rtol=1e-5, atol=1e-6)
            finally:
                s.close()


def test_production_box():
    """The 96k-atom, 8x8, rc 1.0 / rlist 1.1 workload the benchmark times: the whole cluster-pair list
    (about a million entries) bit-exact against the oracle's; forces on sampled atoms, and on all atoms
    with the worst per-particle error bounded too (a missing or extra close pair shows there even where the
    RMS over 96k atoms would hide it); total energy and virial against the cell-list oracle."""
    box = synth.water_box(32000, 9.86, seed=1306)
    rc, rlist, beta, shape = 1.0, 1.1, 3.12, (8, 8)
    rbb = np.float32(default_rbb(box, shape, rlist))
    s = GpuSystem(box, shape, rlist, rbb=float(rbb))
    try:
        gpu = s.mxn.nb_list_export_canonical(s.lst)
        g = oracle.grid_sort(box.xyz, box.box, *shape)
        ref = oracle.pairlist(g, box.box, np.float32(rlist), rbb, box.excl_off, box.excl_idx)
        assert len(ref) > 900000
        _cmp_lists(gpu, ref)
        f, e, v = s.forces(rc, beta, s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL)
        sub = np.random.default_rng(0).choice(box.n, 3000, replace=False).astype(np.int32)
        fs, _ = oracle.forces_subset(box.xyz, box.q, box.type, box.box, box.excl_off, box.excl_idx,
                                     synth.lj_table_spce(), rc, beta, F, sub)
        assert rel_rms(f[sub], fs) <= 1e-5
        fr, er, vr = _oracle_forces(box, rc, beta, mode="binned")
        assert rel_rms(f, fr) <= 1e-5
        worst = max_atom_err(f, fr)
        print("\n[production] force rel RMS %.3e, worst particle %.3e (of its force, floored at the RMS force)"
              % (rel_rms(f, fr), worst))
        assert worst <= 1e-4
        np.testing.assert_allclose(e, er, rtol=1e-5)
        assert np.abs(v - vr).max() <= 1e-5 * np.abs(vr).max()
    finally:
        s.close()


def test_error_paths(c1):
    import paper_1306_1737_amd as mxn
    import torch
    s = GpuSystem(c1, (4, 4), 0.9)
    try:
        with pytest.raises(mxn.NbError) as ei:
            mxn.nb_pairlist_build(s.ctx, s.grid, 1.6, -1.0, s.eo, s.ei)
        assert ei.value.status == mxn.NB_ERR_BOX
        p = mxn.make_params(0.9, 5.0, F, s.lj)
        f = torch.zeros((c1.n, 3), device=s.dev)
        with pytest.raises(mxn.NbError) as ei:
            mxn.nb_forces(s.ctx, s.grid, s.lst, s.xyzq, p, 0, f)
        assert ei.value.status == mxn.NB_ERR_UNSUPPORTED
        # asynchronous build that outgrows the capacity of a small list: overflow latched, then a synchronous rebuild
        small = mxn.nb_pairlist_build(s.ctx, s.grid, 0.3, -1.0, s.eo, s.ei)
        mxn.nb_pairlist_build(s.ctx, s.grid, 1.5, -1.0, s.eo, s.ei, mxn.NB_LIST_ASYNC, small)
        with pytest.raises(mxn.NbError) as ei:
            mxn.nb_sync(s.ctx)
        assert ei.value.status == mxn.NB_ERR_OVERFLOW
        mxn.nb_pairlist_build(s.ctx, s.grid, 1.5, -1.0, s.eo, s.ei, 0, small)
        assert mxn.nb_list_info(small)[0] > 0
        mxn.nb_list_free(small)
        # a non-finite coordinate is latched and reported
        bad = s.xyzq.clone()
        bad[5, 0] = float("nan")
        g2 = mxn.nb_grid_sort(s.ctx, c1.box, bad, s.type, (4, 4))
        with pytest.raises(mxn.NbError) as ei:
            mxn.nb_sync(s.ctx)
        assert ei.value.status == mxn.NB_ERR_NONFINITE
        mxn.nb_grid_free(g2)
        # LJ types outside [0, ntypes) are reported at nb_sync, not clamped silently
        big = s.type.clone()
        big[7] = 5
        g3 = mxn.nb_grid_sort(s.ctx, c1.box, s.xyzq, big, (4, 4))
        l3 = mxn.nb_pairlist_build(s.ctx, g3, 0.9, -1.0, s.eo, s.ei)
        mxn.nb_forces(s.ctx, g3, l3, s.xyzq, mxn.make_params(0.9, 3.47, F, s.lj), 0, f)
        with pytest.raises(mxn.NbError) as ei:
            mxn.nb_sync(s.ctx)
        assert ei.value.status == mxn.NB_ERR_ARG
        neg = s.type.clone()
        neg[3] = -1
        g4 = mxn.nb_grid_sort(s.ctx, c1.box, s.xyzq, neg, (4, 4))
        with pytest.raises(mxn.NbError) as ei:
            mxn.nb_sync(s.ctx)
        assert ei.value.status == mxn.NB_ERR_ARG
        mxn.nb_sync(s.ctx)
        mxn.nb_list_free(l3)
        mxn.nb_grid_free(g3)
        mxn.nb_grid_free(g4)
        # a list built before the grid's last sort is rejected
        s.grid = mxn.nb_grid_sort(s.ctx, c1.box, s.xyzq, s.type, (4, 4), s.grid)
        with pytest.raises(mxn.NbError) as ei:
            mxn.nb_forces(s.ctx, s.grid, s.lst, s.xyzq, mxn.make_params(0.9, 3.47, F, s.lj), 0, f)
        assert ei.value.status == mxn.NB_ERR_STATE
    finally:
        s.close()


def test_buffer_estimate_matches_oracle():
    import paper_1306_1737_amd as mxn
    from oracle import drift
    kw = dict(T=300.0, dt=0.002, masses=[synth.MASS_O, synth.MASS_H], charges=[synth.Q_O, synth.Q_H],
              c6c12=synth.lj_table_spce(), counts=[32000, 64000], volume=9.86 ** 3, rc=1.0, beta=3.12, f=F)
    for nst in (5, 10, 20, 40):
        ref = drift.min_buffer(0.005, nstlist=nst, **kw)
        rb, d, fb = mxn.nb_buffer_estimate(None, T=300.0, dt=0.002, nstlist=nst, mass=kw["masses"],
                                           charge=kw["charges"], c6c12=kw["c6c12"], count=kw["counts"],
                                           volume=kw["volume"], rc=1.0, beta=3.12, coulomb_f=F, shape=(8, 8),
                                           target=0.005)
        assert rb == pytest.approx(ref, abs=1e-9)
        assert d == pytest.approx(drift.drift_rate(rb, nstlist=nst, **kw), rel=1e-9)
        assert not fb


def test_timing_selects_timers(c1):
    """HIP-event timers: all, none, or a selection (the benchmark times one force kernel per step)."""
    s = GpuSystem(c1, (8, 8), 0.9)
    try:
        mxn = s.mxn
        mxn.nb_timing_read(s.ctx)
        mxn.nb_timing_enable(s.ctx, True, timers=[mxn.NB_TIMER_FORCE_KERNEL])
        s.forces(0.9, 3.47, 0)
        s.forces(0.9, 3.47, 0)
        t = mxn.nb_timing_read(s.ctx)
        assert t["force_kernel"][1] == 2 and t["force_kernel"][0] > 0
        assert t["force_call"][1] == 0 and t["grid_sort"][1] == 0
        mxn.nb_timing_enable(s.ctx, True)
        s.forces(0.9, 3.47, 0)
        t = mxn.nb_timing_read(s.ctx)
        assert t["force_kernel"][1] == 1 and t["force_call"][1] == 1
        mxn.nb_timing_enable(s.ctx, False)
        s.forces(0.9, 3.47, 0)
        assert mxn.nb_timing_read(s.ctx)["force_kernel"][1] == 0
        assert mxn.lib().nb_timing_enable(s.ctx, 5) != 0                           # neither 0, 1 nor a selection
        assert mxn.lib().nb_timing_enable(s.ctx, mxn.NB_TIMING_SELECT | 64) != 0   # no such timer
    finally:
        s.close()


@pytest.mark.parametrize("variant", [0, 2], ids=["direct", "super"])
def test_overlapping_particles_flagged(c1, variant):
    """Two oxygens of different waters 0.03 nm apart: their LJ force (~2e15 kJ/mol/nm) is beyond the fixed-point
    summation range, so exactly those two forces come back NaN and nb_sync reports NB_ERR_NONFINITE; the other
    forces stay finite, and the report clears the flag."""
    import paper_1306_1737_amd as mxn
    xyz = c1.xyz.copy()
    o1, o2 = 0, 3                                    # oxygens of waters 0 and 1
    shift = xyz[o1] + np.array([0.03, 0.0, 0.0]) - xyz[o2]
    xyz[o2:o2 + 3] += shift                          # move water 1 rigidly next to water 0's oxygen
    box = dataclasses.replace(c1, xyz=xyz.astype(np.float32))
    s = GpuSystem(box, (8, 8), 0.9, variant=variant)
    try:
        f = s.torch.zeros((box.n, 3), dtype=s.torch.float32, device=s.dev)
        p = mxn.make_params(0.9, 3.47, F, s.lj)
        mxn.nb_forces(s.ctx, s.grid, s.lst, s.xyzq, p, 0, f)
        with pytest.raises(mxn.NbError) as ei:
            mxn.nb_sync(s.ctx)
        assert ei.value.status == mxn.NB_ERR_NONFINITE
        fh = f.cpu().numpy()
        bad = np.flatnonzero(~np.isfinite(fh).all(axis=1))
        assert set(bad.tolist()) == {o1, o2}
        mxn.nb_sync(s.ctx)                           # the flag was cleared by the report
    finally:
        s.close()


@pytest.mark.parametrize("variant", [0, 2], ids=["direct", "super"])
def test_close_contact_within_range(c1, variant):
    """Two oxygens of different waters 0.075 nm apart, as free flight produces within 80 fs on the production
    box: their LJ force (1.3e10 kJ/mol/nm) is within the fixed-point summation range, so every force is finite,
    nb_sync reports nothing, and the forces match the FP64 oracle (the pair's own and all the others)."""
    xyz = c1.xyz.copy()
    o1, o2 = 0, 3                                    # oxygens of waters 0 and 1
    xyz[o2:o2 + 3] += xyz[o1] + np.array([0.075, 0.0, 0.0]) - xyz[o2]
    box = dataclasses.replace(c1, xyz=xyz.astype(np.float32))
    rc, beta = 0.9, 3.47
    s = GpuSystem(box, (8, 8), rc, variant=variant)
    try:
        f, e, _ = s.forces(rc, beta, s.mxn.NB_ENERGY)
        s.mxn.nb_sync(s.ctx)
        assert np.isfinite(f).all()
        fr, er, _ = _oracle_forces(box, rc, beta)
        assert np.linalg.norm(f[o1] - fr[o1]) <= 1e-5 * np.linalg.norm(fr[o1])
        assert np.linalg.norm(fr[o1]) > 2.0 ** 33
        rest = np.ones(box.n, dtype=bool)
        rest[[o1, o2]] = False
        assert rel_rms(f[rest], fr[rest]) <= 1e-5
        np.testing.assert_allclose(e, er, rtol=1e-5)
    finally:
        s.close()
