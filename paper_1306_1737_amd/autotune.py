"""Autotuner for batched replicas: cluster shape x work items per workgroup.

The measurement is the library's nb_autotune: for a set of replica boxes it
builds the grids and lists of every candidate cluster shape (4x4, 4x8, 8x4,
8x8; the paper tunes M and N to the hardware, Sec. 2.2 and 3.1), binds them
to one batch and times the batched force launch with 1, 2, 4 and 8 work
items (wavefronts) per workgroup with HIP events.  This module keeps the
results in a JSON cache keyed by device, number of replicas, total size
(rounded to a power of two) and the cut-offs.
"""
from __future__ import annotations

import json
import math
import os

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
    up = [(torch.from_numpy(b.xyzq()).to(dev), torch.from_numpy(b.type).to(dev),
           torch.from_numpy(b.excl_off).to(dev), torch.from_numpy(b.excl_idx).to(dev)) for b in boxes]
    _, _, ms = mxn.nb_autotune(ctx, [b.box for b in boxes], *[[u[k] for u in up] for k in range(4)], rlist, params,
                               mxn.NB_ENERGY, shapes, groups, reps)
    table = [dict(shape=list(sh), group=g, ms=float(ms[i, j])) for i, sh in enumerate(shapes)
             for j, g in enumerate(groups)]
    best = min(table, key=lambda row: row["ms"])
    res = dict(key=key, shape=best["shape"], group=best["group"], ms=best["ms"], table=table, cached=False)
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        db[key] = {k: v for k, v in res.items() if k != "cached"}
        with open(cache, "w") as fh:
            json.dump(db, fh, indent=1)
    return res
