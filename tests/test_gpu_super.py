"""Super-cluster force kernel (NB_FORCE_SUPER; the grouped i-cluster layout of Sec. 2.3 and 3.2) through the
C ABI: forces within 1e-5 relative RMS of the FP64 oracle and within rounding of the direct kernel on the same
list, energies and virial likewise, bit-reproducible across calls and rebuilds, for super-clusters of 8 and 4
i-clusters, any number of entries per work item, both Coulomb variants beside analytic Ewald, pruned lists,
and shapes it does not take (which fall back to the direct kernel bit for bit)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._nb import F, GpuSystem, default_rbb, rel_rms

pytestmark = pytest.mark.gpu

DIRECT, SUPER = 0, 2


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu-case] %s" % request.node.nodeid, file=sys.stderr, flush=True)
    yield


@pytest.fixture(scope="module")
def c1():
    return synth.water_box(1000, 3.104, seed=1306)


@pytest.fixture(scope="module")
def w8k():
    return synth.water_box(8000, synth.box_edge_for(8000), seed=8)


def _oracle(box, rc, beta, xyz=None, mode="binned"):
    return oracle.forces(box.xyz if xyz is None else xyz, box.q, box.type, box.box, box.excl_off, box.excl_idx,
                         synth.lj_table_spce(), rc, beta, F, shift=True, mode=mode)


def _both(s, rc, beta, flags, xq=None):
    """Forces, energies and virial with the super-cluster and the direct kernel on one list."""
    mxn = s.mxn
    mxn.nb_set_force_variant(s.ctx, SUPER)
    sup = s.forces(rc, beta, flags, xyzq_now=xq)
    mxn.nb_set_force_variant(s.ctx, DIRECT)
    dr = s.forces(rc, beta, flags, xyzq_now=xq)
    mxn.nb_set_force_variant(s.ctx, SUPER)
    return sup, dr


def _close(sup, dr, ref=None):
    (f, e, v), (fd, ed, vd) = sup, dr
    assert rel_rms(f, fd) <= 2e-6
    np.testing.assert_allclose(e, ed, rtol=2e-6)
    assert np.abs(v - vd).max() <= 2e-6 * max(np.abs(vd).max(), 1e-30)
    if ref is not None:
        fr, er, vr = ref
        assert rel_rms(f, fr) <= 1e-5
        np.testing.assert_allclose(e, er, rtol=1e-5)
        assert np.abs(v - vr).max() <= 1e-5 * np.abs(vr).max()


@pytest.mark.parametrize("rlist", [1.0, 1.1, 1.6], ids=["rlist1.0", "rlist1.1", "rlist1.6-groups-of-4"])
def test_super_against_oracle_and_direct(w8k, rlist):
    """24k atoms, rc 1.0; at rlist 1.6 the i-cluster regions exceed 512 entries and the view groups 4."""
    rc, beta = 1.0, 3.12
    s = GpuSystem(w8k, (8, 8), rlist, rbb=default_rbb(w8k, (8, 8), rlist), variant=SUPER)
    try:
        fl = s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL
        sup, dr = _both(s, rc, beta, fl)
        _close(sup, dr, _oracle(w8k, rc, beta))
        f0, _, _ = s.forces(rc, beta, 0)                       # force-only kernel: same j/i sums
        np.testing.assert_array_equal(f0, sup[0])
        f32, e32, _ = s.forces(rc, beta, fl | s.mxn.NB_ACC_FP32)
        np.testing.assert_array_equal(f32, sup[0])
        np.testing.assert_allclose(e32, sup[1], rtol=1e-4)
    finally:
        s.close()


def test_super_after_motion_and_reproducible(w8k):
    """List at step 0, forces at step 9 of ballistic motion; repeated calls and separate (synchronous and
    asynchronous) builds of the same list give bit-identical forces, energies and virial."""
    rc, rlist, beta = 1.0, 1.1, 3.12
    x9 = synth.free_flight(w8k.xyz, synth.velocities(w8k.mass, 300.0, seed=9), 0.002, 10)[9]
    s = GpuSystem(w8k, (8, 8), rlist, variant=SUPER)
    try:
        mxn = s.mxn
        xq = s.torch.from_numpy(w8k.xyzq(x9)).to(s.dev)
        fl = mxn.NB_ENERGY | mxn.NB_VIRIAL
        sup, dr = _both(s, rc, beta, fl, xq=xq)
        _close(sup, dr, _oracle(w8k, rc, beta, xyz=x9))
        again = s.forces(rc, beta, fl, xyzq_now=xq)
        for k in range(3):
            np.testing.assert_array_equal(again[k], sup[k])
        for flags in (0, mxn.NB_LIST_ASYNC):
            s.lst = mxn.nb_pairlist_build(s.ctx, s.grid, rlist, -1.0, s.eo, s.ei, flags, s.lst)
            got = s.forces(rc, beta, fl, xyzq_now=xq)
            for k in range(3):
                np.testing.assert_array_equal(got[k], sup[k])
    finally:
        s.close()


@pytest.mark.parametrize("per_item", [1, 3, 16, 64])
def test_super_entries_per_item(c1, per_item):
    rc, beta = 0.9, 3.47
    s = GpuSystem(c1, (8, 8), 0.9, variant=SUPER)
    try:
        mxn = s.mxn
        mxn.nb_set_super_cluster(s.ctx, 0, per_item)
        fl = mxn.NB_ENERGY | mxn.NB_VIRIAL
        sup, dr = _both(s, rc, beta, fl)
        _close(sup, dr, _oracle(c1, rc, beta, mode="brute"))
        with pytest.raises(mxn.NbError):
            mxn.nb_set_super_cluster(s.ctx, 0, 65)
        with pytest.raises(mxn.NbError):
            mxn.nb_set_super_cluster(s.ctx, 2, 0)
    finally:
        s.close()


@pytest.mark.parametrize("coulomb,eps_rf", [(1, 78.0), (2, 0.0)], ids=["reaction-field", "ewald-table"])
def test_super_coulomb_variants(w8k, coulomb, eps_rf):
    rc, beta = 1.0, 3.12
    s = GpuSystem(w8k, (8, 8), 1.1, variant=SUPER)
    try:
        mxn, torch = s.mxn, s.torch
        out = []
        for variant in (SUPER, DIRECT):
            mxn.nb_set_force_variant(s.ctx, variant)
            f = torch.zeros((w8k.n, 3), dtype=torch.float32, device=s.dev)
            e = torch.zeros(2, dtype=torch.float64, device=s.dev)
            p = mxn.make_params(rc, beta, F, s.lj, True, coulomb, eps_rf)
            mxn.nb_forces(s.ctx, s.grid, s.lst, s.xyzq, p, mxn.NB_ENERGY, f, e)
            mxn.nb_sync(s.ctx)
            out.append((f.cpu().numpy().astype(np.float64), e.cpu().numpy()))
        assert rel_rms(out[0][0], out[1][0]) <= 2e-6
        np.testing.assert_allclose(out[0][1], out[1][1], rtol=2e-6)
        if coulomb == 1:
            fr, er, _ = oracle.forces_rf(w8k.xyz, w8k.q, w8k.type, w8k.box, w8k.excl_off, w8k.excl_idx,
                                         synth.lj_table_spce(), rc, eps_rf, F, shift=True, mode="binned")
        else:
            fr, er, _ = _oracle(w8k, rc, beta)
        assert rel_rms(out[0][0], fr) <= 1e-5
        np.testing.assert_allclose(out[0][1], er, rtol=1e-5)
    finally:
        s.close()


def test_super_on_pruned_list(c1):
    """A box-only outer list at 1.2 nm pruned at 1.0 nm after motion: the super-cluster view of the pruned
    list gives the direct kernel's forces; the view follows the second prune into the same handle."""
    rc, beta = 1.0, 3.12
    s = GpuSystem(c1, (8, 8), 1.2, rbb=1.2, variant=SUPER)
    try:
        mxn = s.mxn
        v = synth.velocities(c1.mass, 300.0, seed=4)
        traj = synth.free_flight(c1.xyz, v, 0.002, 10)
        inner = None
        for step in (4, 9):
            xq = s.torch.from_numpy(c1.xyzq(traj[step])).to(s.dev)
            inner = mxn.nb_pairlist_prune(s.ctx, s.lst, xq, 1.0, inner)
            outer_lst = s.lst
            s.lst = inner
            try:
                sup, dr = _both(s, rc, beta, mxn.NB_ENERGY | mxn.NB_VIRIAL, xq=xq)
            finally:
                s.lst = outer_lst
            _close(sup, dr, _oracle(c1, rc, beta, xyz=traj[step], mode="brute"))
        mxn.nb_list_free(inner)
    finally:
        s.close()


@pytest.mark.parametrize("shape", [(4, 4), (4, 8), (8, 4)])
def test_other_shapes_fall_back_to_direct(c1, shape):
    s = GpuSystem(c1, shape, 1.0, variant=SUPER)
    try:
        sup, dr = _both(s, 0.9, 3.47, s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL)
        for k in range(3):
            np.testing.assert_array_equal(sup[k], dr[k])
    finally:
        s.close()


def test_sparse_and_single_water():
    """Two waters far apart in a 6 nm box (only self cluster pairs and exclusions) and one water."""
    rng = np.random.default_rng(3)
    for nw, edge in ((2, 6.0), (1, 2.5), (40, 2.2)):
        box = synth.water_box(nw, edge, seed=int(rng.integers(1 << 30)))
        ref = _oracle(box, 1.0, 3.12, mode="brute")
        s = GpuSystem(box, (8, 8), 1.0, variant=SUPER)
        try:
            sup, dr = _both(s, 1.0, 3.12, s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL)
            assert rel_rms(sup[0], ref[0]) <= 1e-5
            np.testing.assert_allclose(sup[1], ref[1], rtol=1e-5, atol=1e-6)
            assert rel_rms(sup[0], dr[0]) <= 2e-6
        finally:
            s.close()


def test_production_box_super():
    """96k atoms, 8x8, rc 1.0 / rlist 1.1 (the benchmarked workload): the super-cluster kernel against the
    cell-list FP64 oracle on every atom and against the direct kernel."""
    box = synth.water_box(32000, 9.86, seed=1306)
    rc, rlist, beta = 1.0, 1.1, 3.12
    s = GpuSystem(box, (8, 8), rlist, rbb=default_rbb(box, (8, 8), rlist), variant=SUPER)
    try:
        sup, dr = _both(s, rc, beta, s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL)
        _close(sup, dr, _oracle(box, rc, beta))
    finally:
        s.close()
