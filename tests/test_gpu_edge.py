"""Degenerate inputs of the method through the C ABI, against the oracle: no particles (an error), a box
with no interacting pair (particles farther apart than r_list: the list holds only each cluster's entry
with itself), a single particle, two particles whose only interaction crosses a periodic boundary (with
and without an exclusion between them), and a batch in which one replica has no interacting pair beside
ordinary ones (Sec. 2.3 search, Sec. 2.4 exclusions, Sec. 3 kernel)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._nb import F, GpuSystem, rel_rms
from tests.test_gpu_parity import _cmp_lists

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4), (4, 8), (8, 4), (8, 8)]


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu-case] %s" % request.node.nodeid, file=sys.stderr, flush=True)
    yield


def _box(xyz, q, typ, L, excl=()):
    """A WaterBox holding arbitrary particles; excl: pairs (i, j) excluded from each other."""
    n = len(xyz)
    part = [[] for _ in range(n)]
    for i, j in excl:
        part[i].append(j)
        part[j].append(i)
    off = np.zeros(n + 1, np.int32)
    off[1:] = np.cumsum([len(p) for p in part])
    idx = np.array([j for p in part for j in sorted(p)], np.int32)
    return synth.WaterBox(xyz=np.asarray(xyz, np.float32), q=np.asarray(q, np.float32),
                          type=np.asarray(typ, np.int32), mass=np.full(n, 15.999), excl_off=off, excl_idx=idx,
                          box=np.array([L, L, L], np.float64), n_mol=0, seed=0, fallbacks=0)


def _lattice(k, spacing):
    g = (np.arange(k) + 0.5) * spacing
    return np.array([(x, y, z) for x in g for y in g for z in g])


def test_no_particles():
    import torch
    import paper_1306_1737_amd as mxn
    ctx = mxn.nb_create(0)
    try:
        dev = torch.device("cuda:0")
        with pytest.raises(mxn.NbError) as ei:
            mxn.nb_grid_sort(ctx, [3.0, 3.0, 3.0], torch.zeros((0, 4), dtype=torch.float32, device=dev),
                             torch.zeros(0, dtype=torch.int32, device=dev), (4, 4))
        assert ei.value.status == mxn.NB_ERR_ARG
    finally:
        mxn.nb_destroy(ctx)


@pytest.mark.parametrize("shape", SHAPES)
def test_no_interacting_pairs(shape):
    """27 charged LJ particles 3 nm apart, r_BB = 0: only each i-cluster's entry with itself qualifies (a
    particle is within r_list of itself), the list equals the oracle's, and forces and energies are exactly
    zero, with and without energies."""
    xyz = _lattice(3, 3.0)
    q = np.where(np.arange(27) % 2 == 0, 0.5, -0.5)
    b = _box(xyz, q, np.zeros(27), 9.0)
    s = GpuSystem(b, shape, 1.1, rbb=0.0)
    try:
        g = oracle.grid_sort(b.xyz, b.box, *shape)
        ref = oracle.pairlist(g, b.box, np.float32(1.1), np.float32(0.0), b.excl_off, b.excl_idx)
        assert np.all(ref["shift"] == 13)
        _cmp_lists(s.mxn.nb_list_export_canonical(s.lst), ref)
        for flags in (0, s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL):
            f, e, v = s.forces(1.0, 3.12, flags)
            assert np.all(f == 0.0)
            if flags:
                assert np.all(e == 0.0) and np.all(v == 0.0)
        fr, er, _ = oracle.forces(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, synth.lj_table_spce(), 1.0,
                                  3.12, F, mode="brute")
        assert np.all(fr == 0.0) and np.all(er == 0.0)
    finally:
        s.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_single_particle(shape):
    """One particle: a cluster of one real slot and dummies; its self entry holds no pair."""
    b = _box([[1.0, 2.0, 3.0]], [0.4], [0], 4.0)
    s = GpuSystem(b, shape, 1.1)
    try:
        f, e, v = s.forces(1.0, 3.12, s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL)
        assert np.all(f == 0.0) and np.all(e == 0.0) and np.all(v == 0.0)
    finally:
        s.close()


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("excluded", [False, True], ids=["pair", "excluded"])
def test_pair_across_the_boundary(shape, excluded):
    """Two particles 0.5 nm apart only through the periodic boundary (x = 0.2 and L - 0.3): the pair must
    come from an image shift; excluded, only its Ewald correction remains.  Forces, energies and virial
    against the brute-force oracle; Newton's third law exactly."""
    L = 5.0
    xyz = [[0.2, 2.5, 2.5], [L - 0.3, 2.5, 2.5]]
    b = _box(xyz, [0.6, -0.8], [0, 0], L, excl=[(0, 1)] if excluded else [])
    s = GpuSystem(b, shape, 1.1)
    try:
        f, e, v = s.forces(1.0, 3.12, s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL)
        fr, er, vr = oracle.forces(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, synth.lj_table_spce(), 1.0,
                                   3.12, F, mode="brute")
        assert np.abs(fr).max() > 1.0
        assert rel_rms(f, fr) <= 1e-5
        np.testing.assert_array_equal(f[0], -f[1])
        np.testing.assert_allclose(e, er, rtol=1e-5, atol=1e-9)
        assert np.abs(v - vr).max() <= 1e-5 * np.abs(vr).max()
        if excluded:
            assert er[0] == 0.0   # no LJ between excluded particles
    finally:
        s.close()


def test_batch_with_a_replica_without_pairs():
    """A batch whose second replica has no interacting pair: its forces and energies are zero, the other
    replicas equal their per-replica evaluation (to rounding: the batched kernel sums the i-forces of a
    work item in another order)."""
    import torch
    import paper_1306_1737_amd as mxn
    dev = torch.device("cuda:0")
    ctx = mxn.nb_create(0)
    try:
        lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
        p = mxn.make_params(1.0, 3.12, F, lj)
        boxes = [synth.water_box(600, synth.box_edge_for(600), seed=41),
                 _box(_lattice(3, 3.0), np.where(np.arange(27) % 2 == 0, 0.5, -0.5), np.zeros(27), 9.0),
                 synth.water_box(900, synth.box_edge_for(900), seed=42)]
        reps = []
        for k, b in enumerate(boxes):
            r = dict(box=b, xyzq=torch.from_numpy(b.xyzq()).to(dev), type=torch.from_numpy(b.type).to(dev),
                     eo=torch.from_numpy(b.excl_off).to(dev), ei=torch.from_numpy(b.excl_idx).to(dev),
                     f=torch.zeros((b.n, 3), dtype=torch.float32, device=dev))
            r["grid"] = mxn.nb_grid_sort(ctx, b.box, r["xyzq"], r["type"], (8, 8))
            r["lst"] = mxn.nb_pairlist_build(ctx, r["grid"], 1.1, 0.0 if k == 1 else -1.0, r["eo"], r["ei"])
            reps.append(r)
        ref_f, ref_e = [], []
        for r in reps:
            f = torch.zeros_like(r["f"])
            e = torch.zeros(2, dtype=torch.float64, device=dev)
            mxn.nb_forces(ctx, r["grid"], r["lst"], r["xyzq"], p, mxn.NB_ENERGY, f, e)
            mxn.nb_sync(ctx)
            ref_f.append(f.cpu().numpy())
            ref_e.append(e.cpu().numpy())
        batch = mxn.nb_batch_create(ctx, [r["grid"] for r in reps], [r["lst"] for r in reps],
                                    [r["xyzq"] for r in reps], [r["f"] for r in reps])
        energy = torch.zeros(2 * len(reps), dtype=torch.float64, device=dev)
        for r in reps:
            r["f"].fill_(float("nan"))
        mxn.nb_batch_forces(ctx, batch, p, mxn.NB_ENERGY, energy)
        mxn.nb_sync(ctx)
        en = energy.cpu().numpy().reshape(len(reps), 2)
        assert np.all(reps[1]["f"].cpu().numpy() == 0.0) and np.all(en[1] == 0.0)
        for k in (0, 2):
            assert rel_rms(reps[k]["f"].cpu().numpy().astype(np.float64), ref_f[k].astype(np.float64)) <= 1e-6
            np.testing.assert_allclose(en[k], ref_e[k], rtol=1e-9)
        mxn.nb_batch_free(batch)
        for r in reps:
            mxn.nb_list_free(r["lst"])
            mxn.nb_grid_free(r["grid"])
    finally:
        mxn.nb_destroy(ctx)
