"""Energy and virial accumulation precision: the pair terms are computed in FP32 (the paper's kernels run in
single precision, Sec. 4), only the sums differ -- FP32 partial sums reduced in FP64 (default) against FP32
throughout (NB_ACC_FP32) -- compared with the FP64 cell-list oracle.

Both the 96k-atom box and the 3M-atom box (1e6 waters, 31.1 nm; generating it and the FP64 oracle take a
few minutes of host time) run.  Forces are also compared on the sub-box of waters whose oxygen lies in
[0, 6.22 nm)^3 (about 24k atoms), evaluated against the whole periodic system, and the worst per-particle
force error is reported next to the RMS.  The 3M report is also written to the JSON file that
MXN_PRECISION_REPORT names, if set.
"""
import json
import os
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from tests._nb import F, GpuSystem, default_rbb, max_atom_err, max_atom_err_over_rms, rel_rms

pytestmark = pytest.mark.gpu


def _log(msg):
    print("[precision] " + msg, file=sys.stderr, flush=True)


@pytest.fixture(autouse=True)
def _announce(request):
    _log("case %s" % request.node.nodeid)
    yield


def _grid_matches_oracle(mxn, s, box, shape):
    """The GPU grid sort of the box equals the oracle's bit for bit (permutation, images, column starts,
    sorted coordinates, i-cluster boxes): at 3M atoms the columns hold more particles than one pass of the
    column-sort workgroup, the multi-pass path."""
    ex = mxn.nb_grid_export(s.grid)
    g = oracle.grid_sort(box.xyz, box.box, *shape)
    assert ex["info"]["n_slots"] == g["n_slots"]
    np.testing.assert_array_equal(ex["col_start"], g["col_start"])
    np.testing.assert_array_equal(ex["perm"], g["perm"])
    np.testing.assert_array_equal(ex["img"], g["img"])
    real = g["perm"] >= 0
    np.testing.assert_array_equal(ex["xyzq"][real, :3].view(np.uint32), g["xs"][real].view(np.uint32))
    m = shape[0]
    xs = g["xs"][: g["n_slots"]].reshape(-1, m, 3)
    r = real[: g["n_slots"]].reshape(-1, m, 1)
    np.testing.assert_array_equal(ex["bb"][:, :3], np.where(r, xs, np.float32(np.inf)).min(1))
    np.testing.assert_array_equal(ex["bb"][:, 4:7], np.where(r, xs, np.float32(-np.inf)).max(1))
    return int(np.diff(g["col_start"]).max())


def _study(box, rc=1.0, rlist=1.1, beta=3.12, shape=(8, 8), sub_edge=6.22, check_grid=False):
    s = GpuSystem(box, shape, rlist, rbb=float(np.float32(default_rbb(box, shape, rlist))))
    try:
        mxn = s.mxn
        if check_grid:
            tallest = _grid_matches_oracle(mxn, s, box, shape)
            _log("grid sort bit-exact; tallest column %d slots" % tallest)
            assert tallest > 256
        t0 = time.perf_counter()
        f64, e64, v64 = s.forces(rc, beta, mxn.NB_ENERGY | mxn.NB_VIRIAL)
        f32, e32, v32 = s.forces(rc, beta, mxn.NB_ENERGY | mxn.NB_VIRIAL | mxn.NB_ACC_FP32)
        _log("gpu done in %.1f s; oracle (cell lists, FP64) on %d atoms" % (time.perf_counter() - t0, box.n))
    finally:
        s.close()
    t0 = time.perf_counter()
    fr, er, vr = oracle.forces(box.xyz, box.q, box.type, box.box, box.excl_off, box.excl_idx, synth.lj_table_spce(),
                               rc, beta, F, mode="binned")
    _log("oracle done in %.1f s" % (time.perf_counter() - t0))
    ox = box.xyz[0::3].astype(np.float64)
    wat = np.nonzero(np.all((ox >= 0.0) & (ox < sub_edge), axis=1))[0]
    sub = (3 * wat[:, None] + np.arange(3)).reshape(-1)
    vmax = np.abs(vr).max()
    rep = dict(n_atoms=int(box.n), box_nm=float(box.box[0]), shape="%dx%d" % shape, rc=rc, rlist=rlist, beta=beta,
               energy_ref=er.tolist(), energy_fp64_acc=e64.tolist(), energy_fp32_acc=e32.tolist(),
               energy_rel_err_fp64_acc=(np.abs(e64 - er) / np.abs(er)).tolist(),
               energy_rel_err_fp32_acc=(np.abs(e32 - er) / np.abs(er)).tolist(),
               virial_ref_trace=float(np.trace(vr)),
               virial_max_err_fp64_acc=float(np.abs(v64 - vr).max() / vmax),
               virial_max_err_fp32_acc=float(np.abs(v32 - vr).max() / vmax),
               force_rel_rms_all=rel_rms(f64, fr), force_rel_rms_fp32_vs_fp64_acc=rel_rms(f32, f64),
               sub_box_atoms=int(sub.size), force_rel_rms_sub_box=rel_rms(f64[sub], fr[sub]),
               force_max_atom_err_all=max_atom_err(f64, fr), force_max_atom_err_sub_box=max_atom_err(f64[sub], fr[sub]),
               force_max_atom_err_over_rms_all=max_atom_err_over_rms(f64, fr),
               force_max_atom_force_over_rms=float(np.sqrt((fr ** 2).sum(1)).max() / np.sqrt((fr ** 2).sum(1).mean())))
    return rep


def _check(rep):
    assert rep["force_rel_rms_all"] <= 1e-5
    assert rep["force_rel_rms_sub_box"] <= 1e-5
    # worst particle within ten times the RMS tolerance (of its own force, floored at the RMS force)
    assert rep["force_max_atom_err_all"] <= 1e-4
    assert rep["force_max_atom_err_sub_box"] <= 1e-4
    # the accumulation mode changes only the energy/virial sums, not the forces
    assert rep["force_rel_rms_fp32_vs_fp64_acc"] <= 1e-6
    assert max(rep["energy_rel_err_fp64_acc"]) <= 1e-5
    assert rep["virial_max_err_fp64_acc"] <= 1e-5
    assert max(rep["energy_rel_err_fp32_acc"]) <= 1e-3
    assert rep["virial_max_err_fp32_acc"] <= 1e-3


def test_accumulation_precision_96k():
    box = synth.water_box(32000, 9.86, seed=1306)
    rep = _study(box, sub_edge=4.0)
    _log(json.dumps(rep))
    _check(rep)


def test_accumulation_precision_3m():
    w = synth.PRECISION
    t0 = time.perf_counter()
    _log("generating %d waters in a %.2f nm box" % (w.n_mol, w.L))
    box = synth.water_box(w.n_mol, w.L, seed=1306)
    _log("generated in %.1f s" % (time.perf_counter() - t0))
    rep = _study(box, rc=w.rc, rlist=w.rlist, beta=w.beta, shape=(w.m, w.n), check_grid=True)
    rep["workload"] = w.name
    if os.environ.get("MXN_PRECISION_REPORT"):
        with open(os.environ["MXN_PRECISION_REPORT"], "w") as fh:
            json.dump(rep, fh, indent=1)
    _log(json.dumps(rep))
    _check(rep)
