"""Batched replicas: one persistent launch over many uneven systems equals per-system evaluation; the
captured HIP graph replays correctly between eager work; the autotuner returns a valid, cached choice."""
import json
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._nb import F, rel_rms

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu-case] %s" % request.node.nodeid, file=sys.stderr, flush=True)
    yield


SIZES = [500, 1237, 733, 2100, 560, 1800]   # waters per replica (uneven)


def _replicas(torch, mxn, ctx, shape, rlist=1.1):
    dev = torch.device("cuda:0")
    reps = []
    for k, nw in enumerate(SIZES):
        b = synth.water_box(nw, synth.box_edge_for(nw), seed=300 + k)
        r = dict(box=b, xyzq=torch.from_numpy(b.xyzq()).to(dev), type=torch.from_numpy(b.type).to(dev),
                 eo=torch.from_numpy(b.excl_off).to(dev), ei=torch.from_numpy(b.excl_idx).to(dev),
                 f=torch.zeros((b.n, 3), dtype=torch.float32, device=dev))
        r["grid"] = mxn.nb_grid_sort(ctx, b.box, r["xyzq"], r["type"], shape)
        r["lst"] = mxn.nb_pairlist_build(ctx, r["grid"], rlist, -1.0, r["eo"], r["ei"])
        reps.append(r)
    return reps


@pytest.mark.parametrize("shape", [(4, 4), (4, 8), (8, 4), (8, 8)])
def test_batch_matches_per_replica_and_graph_replays(shape):
    import torch
    import paper_1306_1737_amd as mxn
    dev = torch.device("cuda:0")
    ctx = mxn.nb_create(0)
    try:
        lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
        p = mxn.make_params(1.0, 3.12, F, lj)
        reps = _replicas(torch, mxn, ctx, shape)
        n = len(reps)
        # per-replica reference through nb_forces
        ref_f, ref_e = [], []
        for r in reps:
            f = torch.zeros_like(r["f"]); e = torch.zeros(2, dtype=torch.float64, device=dev)
            mxn.nb_forces(ctx, r["grid"], r["lst"], r["xyzq"], p, mxn.NB_ENERGY, f, e)
            mxn.nb_sync(ctx)
            ref_f.append(f.cpu().numpy().astype(np.float64)); ref_e.append(e.cpu().numpy())
        batch = mxn.nb_batch_create(ctx, [r["grid"] for r in reps], [r["lst"] for r in reps],
                                    [r["xyzq"] for r in reps], [r["f"] for r in reps])
        energy = torch.zeros(2 * n, dtype=torch.float64, device=dev)

        def check():
            e = energy.cpu().numpy().reshape(n, 2)
            for k, r in enumerate(reps):
                assert rel_rms(r["f"].cpu().numpy().astype(np.float64), ref_f[k]) <= 1e-6
                np.testing.assert_allclose(e[k], ref_e[k], rtol=1e-9)

        for g in (1, 2, 4, 8):
            mxn.nb_batch_set_group(batch, g)
            mxn.nb_batch_forces(ctx, batch, p, mxn.NB_ENERGY, energy)
            mxn.nb_sync(ctx)
            check()
        mxn.nb_batch_capture(ctx, batch, p, mxn.NB_ENERGY, energy)
        for rep in range(4):
            for r in reps:
                r["f"].fill_(float("nan"))      # eager work between replays
            energy.zero_()
            torch.cuda.synchronize()
            mxn.nb_batch_replay(ctx, batch)
            mxn.nb_sync(ctx)
            check()
        mxn.nb_batch_free(batch)
        # one replica against the FP64 oracle
        b = reps[1]["box"]
        fr, er, _ = oracle.forces(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, synth.lj_table_spce(), 1.0, 3.12, F)
        assert rel_rms(ref_f[1], fr) <= 1e-5
        np.testing.assert_allclose(ref_e[1], er, rtol=1e-5)
        for r in reps:
            mxn.nb_list_free(r["lst"]); mxn.nb_grid_free(r["grid"])
    finally:
        mxn.nb_destroy(ctx)


@pytest.mark.parametrize("shape", [(4, 4), (4, 8), (8, 4), (8, 8)])
@pytest.mark.parametrize("coulomb,eps_rf,beta", [(1, 78.0, 0.0), (1, 0.0, 0.0), (2, 0.0, 3.12)],
                         ids=["rf78", "rf0", "table"])
def test_batch_coulomb_variants(shape, coulomb, eps_rf, beta):
    """Reaction field and the tabulated Ewald correction (Eq. 2's Coulomb variants) in the batched launch: each
    replica equals its own nb_forces with the same variant (to rounding: the batched kernel sums a work item's
    i-forces in another order), forces, energies and virial; one replica against the FP64 oracle; captured
    graphs of the tabulated variant (its table built before the capture), of a force call and of a whole
    cycle (batched rebuild + two force calls), replay with eager work between."""
    import torch
    import paper_1306_1737_amd as mxn
    dev = torch.device("cuda:0")
    ctx = mxn.nb_create(0)
    try:
        lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
        p = mxn.make_params(1.0, beta, F, lj, True, coulomb, eps_rf)
        reps = _replicas(torch, mxn, ctx, shape)
        n = len(reps)
        fl = mxn.NB_ENERGY | mxn.NB_VIRIAL
        ref_f, ref_e, ref_v = [], [], []
        for r in reps:
            f = torch.zeros_like(r["f"])
            e = torch.zeros(2, dtype=torch.float64, device=dev)
            v = torch.zeros(9, dtype=torch.float64, device=dev)
            mxn.nb_forces(ctx, r["grid"], r["lst"], r["xyzq"], p, fl, f, e, v)
            mxn.nb_sync(ctx)
            ref_f.append(f.cpu().numpy().astype(np.float64)); ref_e.append(e.cpu().numpy()); ref_v.append(v.cpu().numpy())
        batch = mxn.nb_batch_create(ctx, [r["grid"] for r in reps], [r["lst"] for r in reps],
                                    [r["xyzq"] for r in reps], [r["f"] for r in reps])
        energy = torch.zeros(2 * n, dtype=torch.float64, device=dev)
        virial = torch.zeros(9 * n, dtype=torch.float64, device=dev)

        def check():
            e = energy.cpu().numpy().reshape(n, 2)
            v = virial.cpu().numpy().reshape(n, 9)
            for k, r in enumerate(reps):
                assert rel_rms(r["f"].cpu().numpy().astype(np.float64), ref_f[k]) <= 1e-6
                np.testing.assert_allclose(e[k], ref_e[k], rtol=1e-9)
                assert np.abs(v[k] - ref_v[k]).max() <= 1e-6 * np.abs(ref_v[k]).max()

        mxn.nb_batch_forces(ctx, batch, p, fl, energy, virial)
        mxn.nb_sync(ctx)
        check()
        if coulomb == mxn.NB_COULOMB_EWALD_TABLE:
            mxn.nb_batch_capture(ctx, batch, p, fl, energy, virial)
            for _ in range(3):
                for r in reps:
                    r["f"].fill_(float("nan"))   # eager work between replays
                energy.zero_(); virial.zero_()
                torch.cuda.synchronize()
                mxn.nb_batch_replay(ctx, batch)
                mxn.nb_sync(ctx)
                check()
            # the whole cycle (batched rebuild + two force evaluations) as one graph, on a second batch (a
            # captured batch takes no new topology): replays equal an eager rebuild and force call
            cyc = mxn.nb_batch_create(ctx, [r["grid"] for r in reps], [r["lst"] for r in reps],
                                      [r["xyzq"] for r in reps], [r["f"] for r in reps])
            mxn.nb_batch_bind_topology(cyc, [r["type"] for r in reps], [r["eo"] for r in reps],
                                       [r["ei"] for r in reps])
            mxn.nb_batch_rebuild(ctx, cyc)
            mxn.nb_batch_forces(ctx, cyc, p, fl, energy, virial)
            mxn.nb_sync(ctx)
            eager_f = [r["f"].clone() for r in reps]
            eager_e, eager_v = energy.clone(), virial.clone()
            mxn.nb_batch_capture_cycle(ctx, cyc, 2, p, fl, energy, virial)
            for _ in range(2):
                for r in reps:
                    r["f"].fill_(float("nan"))
                energy.zero_(); virial.zero_()
                torch.cuda.synchronize()
                mxn.nb_batch_replay(ctx, cyc)
                mxn.nb_sync(ctx)
                for k, r in enumerate(reps):
                    assert torch.equal(r["f"], eager_f[k])
                assert torch.equal(energy, eager_e) and torch.equal(virial, eager_v)
            mxn.nb_batch_free(cyc)
        mxn.nb_batch_free(batch)
        b = reps[2]["box"]
        if coulomb == mxn.NB_COULOMB_RF:
            fr, er, _ = oracle.forces_rf(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, synth.lj_table_spce(), 1.0,
                                         eps_rf, F, shift=True, mode="brute")
        else:
            fr, er, _ = oracle.forces(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, synth.lj_table_spce(), 1.0,
                                      beta, F, shift=True, mode="brute")
        assert rel_rms(ref_f[2], fr) <= 1e-5
        np.testing.assert_allclose(ref_e[2], er, rtol=1e-5)
        for r in reps:
            mxn.nb_list_free(r["lst"]); mxn.nb_grid_free(r["grid"])
    finally:
        mxn.nb_destroy(ctx)


def test_batch_grid_size_does_not_change_results():
    """The main launch takes one item per wavefront over a grid sized from the lists' item estimates and a
    second launch strides over the rest: any main-grid size (a single workgroup per XCD, the default, far
    more than the items) gives bit-identical forces and energies, also from a captured graph."""
    import torch
    import paper_1306_1737_amd as mxn
    dev = torch.device("cuda:0")
    ctx = mxn.nb_create(0)
    try:
        lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
        p = mxn.make_params(1.0, 3.12, F, lj)
        reps = _replicas(torch, mxn, ctx, (8, 8))
        n = len(reps)
        batch = mxn.nb_batch_create(ctx, [r["grid"] for r in reps], [r["lst"] for r in reps],
                                    [r["xyzq"] for r in reps], [r["f"] for r in reps])
        energy = torch.zeros(2 * n, dtype=torch.float64, device=dev)

        def run(grid, group):
            mxn.nb_batch_set_group(batch, group)
            mxn.nb_batch_set_grid(batch, grid)
            for r in reps:
                r["f"].fill_(float("nan"))
            energy.zero_()
            mxn.nb_batch_forces(ctx, batch, p, mxn.NB_ENERGY, energy)
            mxn.nb_sync(ctx)
            return [r["f"].cpu().numpy().copy() for r in reps], energy.cpu().numpy().copy()

        ref_f, ref_e = run(0, 4)
        assert all(np.all(np.isfinite(f)) for f in ref_f)
        for grid, group in ((1, 4), (1, 1), (8 * 8, 8), (999, 2), (10 ** 7, 4)):
            f, e = run(grid, group)
            for k in range(n):
                np.testing.assert_array_equal(f[k], ref_f[k], err_msg="grid %d group %d replica %d" % (grid, group, k))
            np.testing.assert_array_equal(e, ref_e)
        for bad in (-1, (1 << 28) + 1):
            with pytest.raises(mxn.NbError):
                mxn.nb_batch_set_grid(batch, bad)
        # a graph captured with the smallest main grid: nearly every item from the strided launch
        mxn.nb_batch_set_group(batch, 4)
        mxn.nb_batch_set_grid(batch, 1)
        mxn.nb_batch_capture(ctx, batch, p, mxn.NB_ENERGY, energy)
        with pytest.raises(mxn.NbError):
            mxn.nb_batch_set_grid(batch, 0)
        for rep in range(3):
            for r in reps:
                r["f"].fill_(float("nan"))
            energy.zero_()
            torch.cuda.synchronize()
            mxn.nb_batch_replay(ctx, batch)
            mxn.nb_sync(ctx)
            for k, r in enumerate(reps):
                np.testing.assert_array_equal(r["f"].cpu().numpy(), ref_f[k])
            np.testing.assert_array_equal(energy.cpu().numpy(), ref_e)
        mxn.nb_batch_free(batch)
        for r in reps:
            mxn.nb_list_free(r["lst"]); mxn.nb_grid_free(r["grid"])
    finally:
        mxn.nb_destroy(ctx)


def test_autotuner_choice_is_valid_and_cached(tmp_path):
    import torch
    import paper_1306_1737_amd as mxn
    from paper_1306_1737_amd import autotune
    ctx = mxn.nb_create(0)
    try:
        boxes = [synth.water_box(nw, synth.box_edge_for(nw), seed=900 + k) for k, nw in enumerate(SIZES)]
        cache = tmp_path / "tune.json"
        held = mxn.nb_memory_info(ctx)
        res = autotune.tune_batch(ctx, boxes, rc=1.0, rlist=1.1, beta=3.12, reps=3, cache=str(cache))
        assert mxn.nb_memory_info(ctx) == held   # nb_autotune frees every grid, list, batch and buffer it made
        assert all(0 < row["ms"] < 1e3 for row in res["table"])
        assert tuple(res["shape"]) in autotune.SHAPES and res["group"] in autotune.GROUPS
        assert len(res["table"]) == len(autotune.SHAPES) * len(autotune.GROUPS)
        best = min(res["table"], key=lambda row: row["ms"])
        assert (tuple(best["shape"]), best["group"]) == (tuple(res["shape"]), res["group"])
        again = autotune.tune_batch(ctx, boxes, rc=1.0, rlist=1.1, beta=3.12, reps=3, cache=str(cache))
        assert again["cached"] and (tuple(again["shape"]), again["group"]) == (tuple(res["shape"]), res["group"])
        assert json.loads(cache.read_text())
    finally:
        mxn.nb_destroy(ctx)


@pytest.mark.parametrize("shape", [(4, 8), (8, 4), (8, 8)])
def test_batched_rebuild_and_cycle_graph(shape):
    """After the particles move, one batched rebuild (grid sort + list of every replica, one launch per stage)
    gives each replica the list its own build gives (bit-exact; two replicas also against the oracle); a graph
    of rebuild + three force evaluations replays correctly with eager work between the replays."""
    import torch
    import paper_1306_1737_amd as mxn
    dev = torch.device("cuda:0")
    ctx = mxn.nb_create(0)
    try:
        lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
        p = mxn.make_params(1.0, 3.12, F, lj)
        reps = _replicas(torch, mxn, ctx, shape)
        n = len(reps)
        batch = mxn.nb_batch_create(ctx, [r["grid"] for r in reps], [r["lst"] for r in reps],
                                    [r["xyzq"] for r in reps], [r["f"] for r in reps])
        mxn.nb_batch_bind_topology(batch, [r["type"] for r in reps], [r["eo"] for r in reps], [r["ei"] for r in reps])
        moved = []
        for k, r in enumerate(reps):
            b = r["box"]
            x9 = synth.free_flight(b.xyz, synth.velocities(b.mass, 300.0, seed=70 + k), 0.002, 10)[9].astype(np.float32)
            moved.append(x9)
            r["xyzq"].copy_(torch.from_numpy(b.xyzq(x9)).to(dev))   # in place: the batch keeps the pointer
        mxn.nb_batch_rebuild(ctx, batch)
        mxn.nb_sync(ctx)
        got = [mxn.nb_list_export_canonical(r["lst"]) for r in reps]
        # each replica's own synchronous build on the moved positions
        for k, r in enumerate(reps):
            g = mxn.nb_grid_sort(ctx, r["box"].box, r["xyzq"], r["type"], shape)
            lst = mxn.nb_pairlist_build(ctx, g, 1.1, -1.0, r["eo"], r["ei"])
            ref = mxn.nb_list_export_canonical(lst)
            assert len(ref) == len(got[k])
            for key in ("ci", "shift", "cj", "mask"):
                np.testing.assert_array_equal(got[k][key], ref[key], err_msg="replica %d %s" % (k, key))
            mxn.nb_list_free(lst)
            mxn.nb_grid_free(g)
        for k in (0, 2):
            b = reps[k]["box"]
            og = oracle.grid_sort(moved[k], b.box, *shape)
            rho = b.n / b.box.prod()
            rbb = np.float32(max(0.0, 1.1 - 0.5 * (max(shape) / rho) ** (1 / 3)))
            ref = oracle.pairlist(og, b.box, np.float32(1.1), rbb, b.excl_off, b.excl_idx)
            assert len(ref) == len(got[k])
            for key in ("ci", "shift", "cj", "mask"):
                np.testing.assert_array_equal(got[k][key], ref[key], err_msg="oracle replica %d %s" % (k, key))
        # forces after the batched rebuild, per replica, against the oracle
        energy = torch.zeros(2 * n, dtype=torch.float64, device=dev)
        mxn.nb_batch_forces(ctx, batch, p, mxn.NB_ENERGY, energy)
        mxn.nb_sync(ctx)
        ref_f = [r["f"].cpu().numpy().astype(np.float64) for r in reps]
        ref_e = energy.cpu().numpy().reshape(n, 2).copy()
        for k in (1, 3):
            b = reps[k]["box"]
            fr, er, _ = oracle.forces(moved[k], b.q, b.type, b.box, b.excl_off, b.excl_idx, synth.lj_table_spce(), 1.0,
                                      3.12, F)
            assert rel_rms(ref_f[k], fr) <= 1e-5
            np.testing.assert_allclose(ref_e[k], er, rtol=1e-5)
        # one graph: rebuild + 3 force evaluations
        mxn.nb_batch_capture_cycle(ctx, batch, 3, p, mxn.NB_ENERGY, energy)
        for rep in range(3):
            for r in reps:
                r["f"].fill_(float("nan"))
            energy.zero_()
            torch.cuda.synchronize()
            mxn.nb_batch_replay(ctx, batch)
            mxn.nb_sync(ctx)
            e = energy.cpu().numpy().reshape(n, 2)
            for k, r in enumerate(reps):
                assert rel_rms(r["f"].cpu().numpy().astype(np.float64), ref_f[k]) <= 1e-6
                np.testing.assert_allclose(e[k], ref_e[k], rtol=1e-9)
        mxn.nb_batch_free(batch)
        for r in reps:
            mxn.nb_list_free(r["lst"]); mxn.nb_grid_free(r["grid"])
    finally:
        mxn.nb_destroy(ctx)


def test_batched_256_replicas_against_oracle():
    """The batched configuration at its real size: 256 water boxes of 1 500-24 000 atoms (log-uniform, seeded),
    rc 1.0 / rlist 1.1 nm, 8x8, one batched launch for all replicas (and the captured cycle graph).  A sample of
    replicas (the smallest, the largest and six others) is checked against the FP64 oracle."""
    from concurrent.futures import ThreadPoolExecutor
    import torch
    import paper_1306_1737_amd as mxn
    sizes = synth.batched_sizes(256)

    def gen(k):
        return synth.water_box(int(sizes[k]), synth.box_edge_for(int(sizes[k])), seed=5000 + k)

    with ThreadPoolExecutor(16) as pool:
        boxes = list(pool.map(gen, range(len(sizes))))
    dev = torch.device("cuda:0")
    ctx = mxn.nb_create(0)
    reps = []
    try:
        lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
        p = mxn.make_params(1.0, 3.12, F, lj)
        for b in boxes:
            r = dict(box=b, xyzq=torch.from_numpy(b.xyzq()).to(dev), type=torch.from_numpy(b.type).to(dev),
                     eo=torch.from_numpy(b.excl_off).to(dev), ei=torch.from_numpy(b.excl_idx).to(dev),
                     f=torch.zeros((b.n, 3), dtype=torch.float32, device=dev))
            r["grid"] = mxn.nb_grid_sort(ctx, b.box, r["xyzq"], r["type"], (8, 8))
            r["lst"] = mxn.nb_pairlist_build(ctx, r["grid"], 1.1, -1.0, r["eo"], r["ei"])
            reps.append(r)
        n = len(reps)
        batch = mxn.nb_batch_create(ctx, [r["grid"] for r in reps], [r["lst"] for r in reps],
                                    [r["xyzq"] for r in reps], [r["f"] for r in reps])
        mxn.nb_batch_bind_topology(batch, [r["type"] for r in reps], [r["eo"] for r in reps],
                                   [r["ei"] for r in reps])
        energy = torch.zeros(2 * n, dtype=torch.float64, device=dev)
        mxn.nb_batch_forces(ctx, batch, p, mxn.NB_ENERGY, energy)
        mxn.nb_sync(ctx)
        f_batch = [r["f"].cpu().numpy().astype(np.float64) for r in reps]
        e_batch = energy.cpu().numpy().reshape(n, 2)
        # the whole cycle (batched rebuild + 10 force steps) as one graph: same results on the same positions
        mxn.nb_batch_capture_cycle(ctx, batch, 10, p, mxn.NB_ENERGY, energy)
        for _ in range(2):
            mxn.nb_batch_replay(ctx, batch)
            mxn.nb_sync(ctx)
            np.testing.assert_array_equal(energy.cpu().numpy().reshape(n, 2), e_batch)
        order = np.argsort(sizes)
        sample = sorted(set([int(order[0]), int(order[-1])] +
                            [int(k) for k in np.random.default_rng(7).choice(n, 6, replace=False)]))
        for k in sample:
            b = boxes[k]
            fr, er, _ = oracle.forces(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, synth.lj_table_spce(), 1.0,
                                      3.12, F, mode="binned")
            assert rel_rms(f_batch[k], fr) <= 1e-5, (k, b.n)
            np.testing.assert_allclose(e_batch[k], er, rtol=1e-5)
        mxn.nb_batch_free(batch)
    finally:
        for r in reps:
            mxn.nb_list_free(r["lst"])
            mxn.nb_grid_free(r["grid"])
        mxn.nb_destroy(ctx)
