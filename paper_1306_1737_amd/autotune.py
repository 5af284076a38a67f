"""Autotuner for batched replicas: cluster shape x work items per workgroup.

For a set of replica boxes it builds the grids and lists of every candidate
cluster shape (4x4, 4x8, 8x4, 8x8; the paper tunes M and N to the hardware,
Sec. 2.2 and 3.1), binds them to one batch and times the batched force
launch with 1, 2, 4 and 8 work items (wavefronts) per workgroup.  The fastest pair is
cached in a JSON file keyed by device, number of replicas, total size
(rounded to a power of two) and the cut-offs.  Timing uses wall-clock around
synchronised repetitions; every kernel runs in the library.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

import synth
import paper_1306_1737_amd as mxn

SHAPES = [(4, 4), (4, 8), (8, 4), (8, 8)]
GROUPS = [1, 2, 4, 8]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mxn_autotune.json")


def _key(boxes, rc, rlist):
    import torch
    dev = torch.cuda.get_device_name(0)
    total = sum(b.n for b in boxes)
    return "%s|rep=%d|atoms~2^%d|rc=%.3f|rlist=%.3f" % (dev, len(boxes), round(math.log2(max(total, 1))), rc, rlist)


def build_replicas(ctx, boxes, shape, rlist):
    import torch
    dev = torch.device("cuda:0")
    reps = []
    for b in boxes:
        r = dict(box=b, xyzq=torch.from_numpy(b.xyzq()).to(dev), type=torch.from_numpy(b.type).to(dev),
                 eo=torch.from_numpy(b.excl_off).to(dev), ei=torch.from_numpy(b.excl_idx).to(dev),
                 f=torch.zeros((b.n, 3), dtype=torch.float32, device=dev))
        r["grid"] = mxn.nb_grid_sort(ctx, b.box, r["xyzq"], r["type"], shape)
        r["lst"] = mxn.nb_pairlist_build(ctx, r["grid"], rlist, -1.0, r["eo"], r["ei"])
        reps.append(r)
    return reps


def free_replicas(reps):
    for r in reps:
        mxn.nb_list_free(r["lst"])
        mxn.nb_grid_free(r["grid"])


def time_batch(ctx, batch, params, energy, reps=5, warmup=2):
    for _ in range(warmup):
        mxn.nb_batch_forces(ctx, batch, params, mxn.NB_ENERGY, energy)
    mxn.nb_sync(ctx)
    t0 = time.perf_counter()
    for _ in range(reps):
        mxn.nb_batch_forces(ctx, batch, params, mxn.NB_ENERGY, energy)
    mxn.nb_sync(ctx)
    return (time.perf_counter() - t0) * 1e3 / reps


def tune_batch(ctx, boxes, rc, rlist, beta, reps=5, cache=DEFAULT_CACHE, shapes=SHAPES, groups=GROUPS):
    """Best (shape, group) for the batch, from the cache or by measurement."""
    import torch
    key = _key(boxes, rc, rlist)
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            db = json.load(fh)
    if key in db:
        hit = dict(db[key])
        hit["cached"] = True
        return hit
    dev = torch.device("cuda:0")
    lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
    params = mxn.make_params(rc, beta, synth.COULOMB_F, lj)
    energy = torch.zeros(2 * len(boxes), dtype=torch.float64, device=dev)
    table = []
    for shape in shapes:
        rs = build_replicas(ctx, boxes, shape, rlist)
        batch = mxn.nb_batch_create(ctx, [r["grid"] for r in rs], [r["lst"] for r in rs], [r["xyzq"] for r in rs],
                                    [r["f"] for r in rs])
        for g in groups:
            mxn.nb_batch_set_group(batch, g)
            table.append(dict(shape=list(shape), group=g, ms=time_batch(ctx, batch, params, energy, reps)))
        mxn.nb_batch_free(batch)
        free_replicas(rs)
    best = min(table, key=lambda row: row["ms"])
    res = dict(key=key, shape=best["shape"], group=best["group"], ms=best["ms"], table=table, cached=False)
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        db[key] = {k: v for k, v in res.items() if k != "cached"}
        with open(cache, "w") as fh:
            json.dump(db, fh, indent=1)
    return res
