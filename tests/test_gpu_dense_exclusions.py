"""Exclusion lists denser than the pair search stages per i-cluster (Sec. 2.4 exclusion masks).

The search holds up to 64 exclusion partners of an i-cluster in its lanes; an i-cluster with more reads its
partners from the CSR arrays for every accepted candidate instead.  Water gives an 8-particle cluster about 16
partners, so these boxes exclude every particle from its k nearest neighbours (periodic distance, made
symmetric): the excluded pairs are then the closest ones, all inside r_list, so the masks depend on them.
"dense" puts every i-cluster past the staging limit, "mixed" only those in the lower half of the box, so one
search takes both paths.  Lists bit-exact against the oracle; forces, energies and virial against the FP64
oracle, with the direct and the super-cluster force kernels, and through the batched rebuild.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._nb import F, GpuSystem, default_rbb, rel_rms

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4), (4, 8), (8, 4), (8, 8)]
STAGED = 64   # partners per i-cluster the search stages


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu-case] %s" % request.node.nodeid, file=sys.stderr, flush=True)
    yield


def _knn_exclusions(box, k, select):
    """Water exclusions plus, for every selected particle, its k nearest neighbours; symmetric CSR."""
    x = box.xyz.astype(np.float64)
    L = box.box
    part = [set(box.excl_idx[box.excl_off[i]:box.excl_off[i + 1]].tolist()) for i in range(box.n)]
    for i in np.nonzero(select)[0]:
        d = x - x[i]
        d -= L * np.round(d / L)
        r2 = (d * d).sum(1)
        r2[i] = np.inf
        for j in np.argpartition(r2, k)[:k]:
            part[i].add(int(j))
            part[int(j)].add(int(i))
    off = np.zeros(box.n + 1, np.int32)
    off[1:] = np.cumsum([len(p) for p in part])
    idx = np.array([j for p in part for j in sorted(p)], np.int32)
    return dataclasses.replace(box, excl_off=off, excl_idx=idx)


@pytest.fixture(scope="module")
def boxes():
    base = synth.water_box(1000, 3.104, seed=2406)
    dense = _knn_exclusions(base, 18, np.ones(base.n, bool))
    mixed = _knn_exclusions(base, 18, base.xyz[:, 2] < 0.5 * base.box[2])
    return {"dense": dense, "mixed": mixed}


def _partners_per_cluster(box, g, m):
    """Exclusion partners of each i-cluster's real particles (what the search would stage), and whether every
    slot of the cluster holds a particle."""
    perm = g["perm"]
    cnt = np.diff(box.excl_off)
    real = perm >= 0
    per_slot = np.where(real, cnt[np.where(real, perm, 0)], 0)
    return per_slot.reshape(-1, m).sum(1), real.reshape(-1, m).all(1)


@pytest.mark.parametrize("variant", [0, 2], ids=["direct", "super"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("which", ["dense", "mixed"])
def test_dense_exclusions(boxes, which, shape, variant):
    box = boxes[which]
    rc, rlist, beta = 0.9, 1.0, 3.47
    g = oracle.grid_sort(box.xyz, box.box, *shape)
    nx, full = _partners_per_cluster(box, g, shape[0])
    occupied = nx > 0
    if which == "dense":   # at least 18 partners per particle: every full cluster is past the limit
        assert np.all(nx[full] > STAGED), "every full i-cluster must exceed the staging limit"
    else:
        assert np.any(nx[occupied] > STAGED) and np.any(nx[occupied] <= STAGED), "both search paths"
    rbb = np.float32(default_rbb(box, shape, rlist))
    s = GpuSystem(box, shape, rlist, rbb=float(rbb), variant=variant)
    try:
        ref = oracle.pairlist(g, box.box, np.float32(rlist), rbb, box.excl_off, box.excl_idx)
        gpu = s.mxn.nb_list_export_canonical(s.lst)
        assert len(gpu) == len(ref), (len(gpu), len(ref))
        for k in ("ci", "shift", "cj", "mask"):
            np.testing.assert_array_equal(gpu[k], ref[k], err_msg=k)
        f, e, v = s.forces(rc, beta, s.mxn.NB_ENERGY | s.mxn.NB_VIRIAL)
        fr, er, vr = oracle.forces(box.xyz, box.q, box.type, box.box, box.excl_off, box.excl_idx,
                                   synth.lj_table_spce(), rc, beta, F, shift=True, mode="brute")
        assert rel_rms(f, fr) <= 1e-5
        np.testing.assert_allclose(e, er, rtol=1e-5)
        assert np.abs(v - vr).max() <= 1e-5 * np.abs(vr).max()
    finally:
        s.close()


@pytest.mark.parametrize("shape", [(4, 4), (8, 8)])
def test_dense_exclusions_batched_rebuild(boxes, shape):
    """The batched rebuild (one search launch over every replica, partner arrays read from the replicas'
    tables) on replicas with dense, mixed and water exclusions, after the particles moved: every list
    bit-exact against the oracle's for the moved positions, forces and energies against the FP64 oracle."""
    import torch
    import paper_1306_1737_amd as mxn
    dev = torch.device("cuda:0")
    rlist, rc, beta = 1.1, 1.0, 3.12
    systems = [boxes["dense"], synth.water_box(700, synth.box_edge_for(700), seed=2407), boxes["mixed"]]
    ctx = mxn.nb_create(0)
    try:
        lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
        p = mxn.make_params(rc, beta, F, lj)
        reps = []
        for b in systems:
            r = dict(box=b, xyzq=torch.from_numpy(b.xyzq()).to(dev), type=torch.from_numpy(b.type).to(dev),
                     eo=torch.from_numpy(b.excl_off).to(dev), ei=torch.from_numpy(b.excl_idx).to(dev),
                     f=torch.zeros((b.n, 3), dtype=torch.float32, device=dev))
            r["grid"] = mxn.nb_grid_sort(ctx, b.box, r["xyzq"], r["type"], shape)
            r["lst"] = mxn.nb_pairlist_build(ctx, r["grid"], rlist, -1.0, r["eo"], r["ei"])
            reps.append(r)
        batch = mxn.nb_batch_create(ctx, [r["grid"] for r in reps], [r["lst"] for r in reps],
                                    [r["xyzq"] for r in reps], [r["f"] for r in reps])
        mxn.nb_batch_bind_topology(batch, [r["type"] for r in reps], [r["eo"] for r in reps], [r["ei"] for r in reps])
        moved = []
        for k, r in enumerate(reps):
            b = r["box"]
            x9 = synth.free_flight(b.xyz, synth.velocities(b.mass, 300.0, seed=90 + k), 0.002, 10)[9].astype(np.float32)
            moved.append(x9)
            r["xyzq"].copy_(torch.from_numpy(b.xyzq(x9)).to(dev))   # in place: the batch keeps the pointer
        mxn.nb_batch_rebuild(ctx, batch)
        energy = torch.zeros(2 * len(reps), dtype=torch.float64, device=dev)
        mxn.nb_batch_forces(ctx, batch, p, mxn.NB_ENERGY, energy)
        mxn.nb_sync(ctx)
        en = energy.cpu().numpy().reshape(len(reps), 2)
        for k, r in enumerate(reps):
            b = r["box"]
            got = mxn.nb_list_export_canonical(r["lst"])
            og = oracle.grid_sort(moved[k], b.box, *shape)
            rbb = np.float32(default_rbb(b, shape, rlist))
            ref = oracle.pairlist(og, b.box, np.float32(rlist), rbb, b.excl_off, b.excl_idx)
            assert len(got) == len(ref), (k, len(got), len(ref))
            for key in ("ci", "shift", "cj", "mask"):
                np.testing.assert_array_equal(got[key], ref[key], err_msg="replica %d %s" % (k, key))
            fr, er, _ = oracle.forces(moved[k], b.q, b.type, b.box, b.excl_off, b.excl_idx, synth.lj_table_spce(),
                                      rc, beta, F)
            assert rel_rms(r["f"].cpu().numpy().astype(np.float64), fr) <= 1e-5
            np.testing.assert_allclose(en[k], er, rtol=1e-5)
        mxn.nb_batch_free(batch)
        for r in reps:
            mxn.nb_list_free(r["lst"])
            mxn.nb_grid_free(r["grid"])
    finally:
        mxn.nb_destroy(ctx)
