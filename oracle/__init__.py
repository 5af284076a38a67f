"""CPU oracle for the cluster-pair non-bonded path -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check in __graft_entry__ and the CPU-baseline leg of
bench.py may import this package.  The GPU library never calls it and shares
no code with it; the only common module is `synth` (seeded input generation).

* `forces`, `forces_subset`: FP64 pair sums by definition (Eq. 1 LJ, Eq. 2
  Coulomb with the Ewald real-space correction g(r) = d/dr[erf(beta r)/r],
  exclusions with the correction still applied, Sec. 2.4 and 3.2).
* `forces_rf`: the same with the reaction-field correction g(r) = -2 k r.
* `grid_dims`, `grid_sort`, `pairlist`: FP32 canonical clustering and
  cluster-pair list (Sec. 2.3, cluster-pair search pseudocode; Sec. 2.4 masks).
* `gather`, `prune`: the second stage of a two-stage list (Sec. 2.3: box-only
  search, then a particle-distance prune), at positions of a later time.
* `rdf`: pair distance histogram (pair correlation function, Sec. 1 and 2.3).
* `recount`: exact missed-pair energy after displacements (Sec. 5, appendix).
* `drift` (module): the appendix's analytic drift bound (with its V'' term
  corrected) and its numerical quadrature.
* `mlp` (module): FP64 reference MLP for the learned buffer.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ENTRY_DTYPE = np.dtype([("ci", np.int32), ("shift", np.int32), ("cj", np.int32), ("pad", np.int32),
                        ("mask", np.uint64)])


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                        "-std=gnu99", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_h = None


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _lib():
    global _h
    if _h is None:
        if not os.path.exists(_LIB):
            build()
        _h = ctypes.CDLL(_LIB)
        _h.oracle_pairlist.restype = ctypes.c_long
        _h.oracle_recount.restype = ctypes.c_long
        _h.oracle_prune.restype = ctypes.c_long
    return _h


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _lj(c6c12):
    t = _c(c6c12, np.float64)
    nt = t.shape[0]
    return nt, t.reshape(-1)


def forces(xyz, q, typ, box, excl_off, excl_idx, c6c12, rc, beta, coulomb_f, shift=True, mode="binned"):
    """FP64 forces (n,3), energies (E_LJ, E_Coul), virial (3,3) = sum over pairs of r_ij (x) F_i."""
    xyz = _c(xyz, np.float32); q = _c(q, np.float32); typ = _c(typ, np.int32)
    box = _c(box, np.float64); eo = _c(excl_off, np.int32); ei = _c(excl_idx, np.int32)
    nt, tab = _lj(c6c12)
    n = xyz.shape[0]
    f = np.zeros((n, 3)); e = np.zeros(2); v = np.zeros(9)
    rcode = _lib().oracle_forces(ctypes.c_int(n), _p(xyz, ctypes.c_float), _p(q, ctypes.c_float),
                                 _p(typ, ctypes.c_int), _p(box, ctypes.c_double), _p(eo, ctypes.c_int),
                                 _p(ei, ctypes.c_int), ctypes.c_int(nt), _p(tab, ctypes.c_double),
                                 ctypes.c_double(rc), ctypes.c_double(beta), ctypes.c_double(coulomb_f),
                                 ctypes.c_int(int(shift)), ctypes.c_int(1 if mode == "binned" else 0),
                                 _p(f, ctypes.c_double), _p(e, ctypes.c_double), _p(v, ctypes.c_double))
    if rcode != 0:
        raise MemoryError("oracle_forces failed")
    return f, e, v.reshape(3, 3)


def forces_rf(xyz, q, typ, box, excl_off, excl_idx, c6c12, rc, eps_rf, coulomb_f, shift=True, mode="binned"):
    """FP64 reaction-field forces, energies and virial (Eq. 2 with g(r) = -2 k r); eps_rf = 0: conducting."""
    xyz = _c(xyz, np.float32); q = _c(q, np.float32); typ = _c(typ, np.int32)
    box = _c(box, np.float64); eo = _c(excl_off, np.int32); ei = _c(excl_idx, np.int32)
    nt, tab = _lj(c6c12)
    n = xyz.shape[0]
    f = np.zeros((n, 3)); e = np.zeros(2); v = np.zeros(9)
    rcode = _lib().oracle_forces_rf(ctypes.c_int(n), _p(xyz, ctypes.c_float), _p(q, ctypes.c_float),
                                    _p(typ, ctypes.c_int), _p(box, ctypes.c_double), _p(eo, ctypes.c_int),
                                    _p(ei, ctypes.c_int), ctypes.c_int(nt), _p(tab, ctypes.c_double),
                                    ctypes.c_double(rc), ctypes.c_double(eps_rf), ctypes.c_double(coulomb_f),
                                    ctypes.c_int(int(shift)), ctypes.c_int(1 if mode == "binned" else 0),
                                    _p(f, ctypes.c_double), _p(e, ctypes.c_double), _p(v, ctypes.c_double))
    if rcode != 0:
        raise MemoryError("oracle_forces_rf failed")
    return f, e, v.reshape(3, 3)


def forces_subset(xyz, q, typ, box, excl_off, excl_idx, c6c12, rc, beta, coulomb_f, sub, shift=True):
    """FP64 forces on atoms `sub` (brute force over all partners) and their half pair energies (k,2)."""
    xyz = _c(xyz, np.float32); q = _c(q, np.float32); typ = _c(typ, np.int32)
    box = _c(box, np.float64); eo = _c(excl_off, np.int32); ei = _c(excl_idx, np.int32)
    sub = _c(sub, np.int32)
    nt, tab = _lj(c6c12)
    f = np.zeros((sub.shape[0], 3)); ea = np.zeros((sub.shape[0], 2))
    _lib().oracle_forces_subset(ctypes.c_int(xyz.shape[0]), _p(xyz, ctypes.c_float), _p(q, ctypes.c_float),
                                _p(typ, ctypes.c_int), _p(box, ctypes.c_double), _p(eo, ctypes.c_int),
                                _p(ei, ctypes.c_int), ctypes.c_int(nt), _p(tab, ctypes.c_double),
                                ctypes.c_double(rc), ctypes.c_double(beta), ctypes.c_double(coulomb_f),
                                ctypes.c_int(int(shift)), ctypes.c_int(sub.shape[0]), _p(sub, ctypes.c_int),
                                _p(f, ctypes.c_double), _p(ea, ctypes.c_double))
    return f, ea


def grid_dims(n, box, cmax):
    box = _c(box, np.float64)
    nx = ctypes.c_int(); ny = ctypes.c_int(); ix = ctypes.c_float(); iy = ctypes.c_float()
    _lib().oracle_grid_dims(ctypes.c_int(n), _p(box, ctypes.c_double), ctypes.c_int(cmax), ctypes.byref(nx),
                            ctypes.byref(ny), ctypes.byref(ix), ctypes.byref(iy))
    return nx.value, ny.value, np.float32(ix.value), np.float32(iy.value)


def grid_sort(xyz, box, m, n_):
    """Canonical FP32 grid sort.  Returns a dict with per-atom slot/img/xw and per-slot perm/xs."""
    xyz = _c(xyz, np.float32); box = _c(box, np.float64)
    n = xyz.shape[0]
    cmax = max(m, n_)
    nx, ny, ix, iy = grid_dims(n, box, cmax)
    ncol = nx * ny
    slot_of = np.empty(n, np.int32); img = np.empty((n, 3), np.int32); xw = np.empty((n, 3), np.float32)
    cs = np.empty(ncol + 1, np.int32); cc = np.empty(ncol, np.int32)
    ns = _lib().oracle_grid_sort(ctypes.c_int(n), _p(xyz, ctypes.c_float), _p(box, ctypes.c_double),
                                 ctypes.c_int(cmax), ctypes.c_int(nx), ctypes.c_int(ny), ctypes.c_float(ix),
                                 ctypes.c_float(iy), _p(slot_of, ctypes.c_int), _p(img, ctypes.c_int),
                                 _p(xw, ctypes.c_float), _p(cs, ctypes.c_int), _p(cc, ctypes.c_int))
    perm = np.full(ns, -1, np.int32)
    perm[slot_of] = np.arange(n, dtype=np.int32)
    xs = np.zeros((ns, 3), np.float32)
    xs[slot_of] = xw
    return dict(nx=nx, ny=ny, inv_x=ix, inv_y=iy, n_slots=int(ns), slot_of=slot_of, img=img, xw=xw,
                col_start=cs, col_count=cc, perm=perm, xs=xs, m=m, n=n_)


def pairlist(grid, box, rlist, rbb, excl_off, excl_idx, ci_begin=0, ci_end=None):
    """Canonical FP32 cluster-pair list by brute force over (ci, shift, cj); structured array ENTRY_DTYPE."""
    m, n_ = grid["m"], grid["n"]
    ns = grid["n_slots"]
    if ci_end is None:
        ci_end = ns // m
    xs = _c(grid["xs"], np.float32); perm = _c(grid["perm"], np.int32); box = _c(box, np.float64)
    eo = _c(excl_off, np.int32); ei = _c(excl_idx, np.int32)
    cap = 1 << 16
    while True:
        out = np.zeros(cap, ENTRY_DTYPE)
        tot = _lib().oracle_pairlist(ctypes.c_int(ns), ctypes.c_int(m), ctypes.c_int(n_), _p(xs, ctypes.c_float),
                                     _p(perm, ctypes.c_int), _p(box, ctypes.c_double), ctypes.c_float(rlist),
                                     ctypes.c_float(rbb), _p(eo, ctypes.c_int), _p(ei, ctypes.c_int),
                                     ctypes.c_int(ci_begin), ctypes.c_int(ci_end),
                                     out.ctypes.data_as(ctypes.c_void_p), ctypes.c_long(cap))
        if tot <= cap:
            return out[:tot]
        cap = int(tot)


def gather(grid, xyz_now, box):
    """Slot positions (n_slots x 3, FP32) at new coordinates, each atom in its build-time image."""
    xyz = _c(xyz_now, np.float32); box = _c(box, np.float64)
    img = _c(grid["img"], np.int32); slot_of = _c(grid["slot_of"], np.int32)
    xs = np.zeros((grid["n_slots"], 3), np.float32)
    _lib().oracle_gather(ctypes.c_int(xyz.shape[0]), _p(xyz, ctypes.c_float), _p(img, ctypes.c_int),
                         _p(slot_of, ctypes.c_int), _p(box, ctypes.c_double), _p(xs, ctypes.c_float))
    return xs


def prune(grid, xs_now, box, entries, r):
    """Entries of a list with some real particle pair within r at slot positions xs_now (Sec. 2.3 prune)."""
    xs = _c(xs_now, np.float32); perm = _c(grid["perm"], np.int32); box = _c(box, np.float64)
    ent = np.ascontiguousarray(entries, dtype=ENTRY_DTYPE)
    out = np.zeros(max(len(ent), 1), ENTRY_DTYPE)
    k = _lib().oracle_prune(ctypes.c_int(grid["m"]), ctypes.c_int(grid["n"]), _p(xs, ctypes.c_float),
                            _p(perm, ctypes.c_int), _p(box, ctypes.c_double), ent.ctypes.data_as(ctypes.c_void_p),
                            ctypes.c_long(len(ent)), ctypes.c_float(r), out.ctypes.data_as(ctypes.c_void_p))
    return out[:k]


def rdf(grid, xs, typ, box, r_max, nbins, ntypes, excl_off, excl_idx, skip_excluded=False):
    """Pair distance histogram (ntypes, ntypes, nbins) uint64 over unordered real pairs below r_max, with the
    cluster kernels' FP32 distance and bin edges e_k = (float)((k r_max/nbins)^2) (see oracle.c)."""
    xs = _c(xs, np.float32); slot_of = _c(grid["slot_of"], np.int32); typ = _c(typ, np.int32)
    box = _c(box, np.float64); eo = _c(excl_off, np.int32); ei = _c(excl_idx, np.int32)
    hist = np.zeros(ntypes * ntypes * nbins, np.uint64)
    _lib().oracle_rdf(ctypes.c_int(slot_of.shape[0]), _p(xs, ctypes.c_float), _p(slot_of, ctypes.c_int),
                      _p(typ, ctypes.c_int), _p(box, ctypes.c_double), ctypes.c_float(r_max), ctypes.c_int(nbins),
                      ctypes.c_int(ntypes), _p(eo, ctypes.c_int), _p(ei, ctypes.c_int),
                      ctypes.c_int(int(skip_excluded)), hist.ctypes.data_as(ctypes.c_void_p))
    return hist.reshape(ntypes, ntypes, nbins)


def recount(xyz0, xyzt, q, typ, box, excl_off, excl_idx, c6c12, rc, beta, coulomb_f, m, n_, rl, c_bb, db, nb):
    """Missed-pair energy histogram over tau (see oracle.c section 4); E(k db) = hist[k:].sum()."""
    xyz0 = _c(xyz0, np.float32); xyzt = _c(xyzt, np.float32); q = _c(q, np.float32); typ = _c(typ, np.int32)
    box = _c(box, np.float64); eo = _c(excl_off, np.int32); ei = _c(excl_idx, np.int32)
    nt, tab = _lj(c6c12)
    hist = np.zeros(nb)
    _lib().oracle_recount(ctypes.c_int(xyz0.shape[0]), _p(xyz0, ctypes.c_float), _p(xyzt, ctypes.c_float),
                          _p(q, ctypes.c_float), _p(typ, ctypes.c_int), _p(box, ctypes.c_double),
                          _p(eo, ctypes.c_int), _p(ei, ctypes.c_int), ctypes.c_int(nt), _p(tab, ctypes.c_double),
                          ctypes.c_double(rc), ctypes.c_double(beta), ctypes.c_double(coulomb_f), ctypes.c_int(m),
                          ctypes.c_int(n_), ctypes.c_float(rl), ctypes.c_float(c_bb), ctypes.c_double(db),
                          ctypes.c_int(nb), _p(hist, ctypes.c_double))
    return hist
