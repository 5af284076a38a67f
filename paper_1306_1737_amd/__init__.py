"""Python binding of libmxn.so, the MI355X cluster-pair non-bonded library.

Thin ctypes marshalling over the C ABI in include/mxn.h: the functions keep
the C names and argument order; torch tensors supply device pointers and the
current HIP stream.  Every computation runs in the library's HIP kernels --
there is no CPU or PyTorch fallback: if libmxn.so is missing or fails to load,
importing the binding functions raises.

Method: Pall & Hess, "A flexible algorithm for calculating pair interactions
on SIMD architectures", CPC 2013 (grid sort, cluster-pair list, M x N kernel,
Verlet-buffer estimate).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmxn.so")

NB_OK, NB_ERR_ARG, NB_ERR_BOX, NB_ERR_OOM, NB_ERR_HIP, NB_ERR_OVERFLOW, NB_ERR_STATE, NB_ERR_NONFINITE, \
    NB_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7, -8
NB_LIST_ASYNC, NB_LIST_BY_DISTANCE = 1, 2
NB_ENERGY, NB_VIRIAL, NB_ACC_FP32, NB_ACCUMULATE = 1, 2, 4, 8
NB_BUFFER_ANALYTIC, NB_BUFFER_MLP, NB_BUFFER_AUTO = 0, 1, 2

# symbols declared in include/mxn.h (checked by the ABI test)
EXPORTS = [
    "nb_create", "nb_destroy", "nb_memory_info", "nb_set_stream", "nb_sync", "nb_last_error",
    "nb_grid_sort", "nb_grid_free", "nb_grid_info", "nb_grid_export",
    "nb_pairlist_build", "nb_pairlist_prune", "nb_rdf", "nb_list_free", "nb_list_info", "nb_list_export_canonical",
    "nb_forces", "nb_forces_noalloc", "nb_buffer_estimate", "nb_timing_enable", "nb_timing_read",
    "nb_list_stats", "nb_set_force_variant", "nb_set_super_cluster", "nb_set_search_parts", "nb_recount",
    "nb_mlp_create", "nb_mlp_free", "nb_mlp_get_params", "nb_mlp_train_step", "nb_mlp_grad", "nb_mlp_infer",
    "nb_buffer_set_mlp", "nb_mlp_set_domain",
    "nb_batch_create", "nb_batch_free", "nb_batch_set_group", "nb_batch_set_grid", "nb_batch_forces", "nb_batch_capture",
    "nb_batch_replay", "nb_batch_bind_topology", "nb_batch_rebuild", "nb_batch_capture_cycle", "nb_autotune",
]
NB_MLP_FEATURES, NB_MLP_PARAMS = 8, 4801
NB_FORCE_DIRECT, NB_FORCE_SUPER = 0, 2
NB_COULOMB_EWALD, NB_COULOMB_RF, NB_COULOMB_EWALD_TABLE = 0, 1, 2
NB_RDF_SKIP_EXCLUDED = 1
NB_TIMER_FORCE_KERNEL, NB_TIMER_FORCE_CALL, NB_TIMER_GRID_SORT, NB_TIMER_PAIRLIST, NB_TIMER_COUNT = 0, 1, 2, 3, 4
NB_TIMING_SELECT = 0x100


class NbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class nb_allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


class nb_shape(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("n", ctypes.c_int)]


class nb_params(ctypes.Structure):
    _fields_ = [("rc", ctypes.c_float), ("beta", ctypes.c_float), ("coulomb_f", ctypes.c_float),
                ("ntypes", ctypes.c_int), ("c6c12", ctypes.c_void_p), ("shift_energies", ctypes.c_int),
                ("coulomb", ctypes.c_int), ("eps_rf", ctypes.c_float)]


class nb_replicas(ctypes.Structure):
    _fields_ = [("n_rep", ctypes.c_int), ("box", ctypes.c_void_p), ("n", ctypes.c_void_p), ("xyzq", ctypes.c_void_p),
                ("type", ctypes.c_void_p), ("excl_off", ctypes.c_void_p), ("excl_idx", ctypes.c_void_p)]


class nb_grid_info_t(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int) for k in ("n", "n_slots", "m", "n_cl", "nx", "ny", "n_ci", "n_cj")]


class nb_entry(ctypes.Structure):
    _fields_ = [("ci", ctypes.c_int32), ("shift", ctypes.c_int32), ("cj", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("mask", ctypes.c_uint64)]


class nb_buffer_query(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("dt", ctypes.c_double), ("nstlist", ctypes.c_int), ("ntypes", ctypes.c_int),
                ("mass", ctypes.c_void_p), ("charge", ctypes.c_void_p), ("c6c12", ctypes.c_void_p),
                ("count", ctypes.c_void_p), ("volume", ctypes.c_double), ("rc", ctypes.c_double),
                ("beta", ctypes.c_double), ("coulomb_f", ctypes.c_double), ("shape", nb_shape),
                ("target", ctypes.c_double)]


_lib = None


def lib():
    """Load libmxn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmxn.so not built: run `python -m paper_1306_1737_amd.build`")
        # PyTorch supplies device memory and streams and ships its own HIP runtime: load it first so that
        # libmxn.so binds to the same runtime instance instead of a second copy from the system ROCm.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, ip, i, f, d, u = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_float, \
            ctypes.c_double, ctypes.c_uint
        pvp = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "nb_create": ([pvp, i, vp, ctypes.POINTER(nb_allocator)], i), "nb_destroy": ([vp], None),
            "nb_set_stream": ([vp, vp], i), "nb_memory_info": ([vp, ctypes.POINTER(ctypes.c_size_t),
                                                               ctypes.POINTER(ctypes.c_size_t)], i),
            "nb_sync": ([vp], i), "nb_last_error": ([], ctypes.c_char_p),
            "nb_grid_sort": ([vp, vp, i, vp, vp, nb_shape, pvp], i), "nb_grid_free": ([vp], None),
            "nb_grid_info": ([vp, ctypes.POINTER(nb_grid_info_t)], i),
            "nb_grid_export": ([vp, vp, vp, vp, vp, vp], i),
            "nb_pairlist_build": ([vp, vp, f, f, vp, vp, i, pvp], i), "nb_list_free": ([vp], None),
            "nb_pairlist_prune": ([vp, vp, vp, f, pvp], i),
            "nb_rdf": ([vp, vp, vp, vp, f, i, i, i, vp], i),
            "nb_list_info": ([vp, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)], i),
            "nb_list_export_canonical": ([vp, vp, ctypes.c_long, ctypes.POINTER(ctypes.c_long)], i),
            "nb_forces": ([vp, vp, vp, vp, ctypes.POINTER(nb_params), u, vp, vp, vp], i),
            "nb_forces_noalloc": ([vp, vp, vp, vp, ctypes.POINTER(nb_params), u, vp, vp, vp], i),
            "nb_buffer_estimate": ([vp, ctypes.POINTER(nb_buffer_query), i, ctypes.POINTER(d), ctypes.POINTER(d),
                                    ip], i),
            "nb_timing_enable": ([vp, i], i), "nb_timing_read": ([vp, vp, vp], i),
            "nb_list_stats": ([vp, vp, vp, vp, f, vp], i),
            "nb_set_force_variant": ([vp, i], i), "nb_set_super_cluster": ([vp, i, i], i),
            "nb_set_search_parts": ([vp, i], i),
            "nb_recount": ([vp, vp, vp, vp, ctypes.POINTER(nb_params), f, f, i, vp], i),
            "nb_mlp_create": ([vp, vp, vp, vp, pvp], i), "nb_mlp_free": ([vp], None),
            "nb_mlp_get_params": ([vp, vp], i), "nb_mlp_train_step": ([vp, vp, vp, vp, i, f, vp], i),
            "nb_mlp_grad": ([vp, vp, vp, vp, i, vp, vp], i), "nb_mlp_infer": ([vp, vp, vp, i, vp], i),
            "nb_buffer_set_mlp": ([vp, vp, d], i), "nb_mlp_set_domain": ([vp, ctypes.POINTER(nb_buffer_query)], i),
            "nb_batch_create": ([vp, i, vp, vp, vp, vp, pvp], i), "nb_batch_free": ([vp], None),
            "nb_batch_set_group": ([vp, i], i), "nb_batch_set_grid": ([vp, ctypes.c_long], i), "nb_batch_forces": ([vp, vp, ctypes.POINTER(nb_params), u, vp, vp], i),
            "nb_batch_capture": ([vp, vp, ctypes.POINTER(nb_params), u, vp, vp], i),
            "nb_batch_replay": ([vp, vp], i),
            "nb_batch_bind_topology": ([vp, vp, vp, vp], i), "nb_batch_rebuild": ([vp, vp], i),
            "nb_batch_capture_cycle": ([vp, vp, i, ctypes.POINTER(nb_params), u, vp, vp], i),
            "nb_autotune": ([vp, ctypes.POINTER(nb_replicas), f, ctypes.POINTER(nb_params), u, vp, i, vp, i, i,
                             ctypes.POINTER(nb_shape), ctypes.POINTER(ctypes.c_int), vp], i),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != NB_OK:
        raise NbError(rc, lib().nb_last_error().decode())
    return rc


def _ptr(t):
    """Device (or host) address of a torch tensor, numpy array or None."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(t.data_ptr())
    if hasattr(t, "ctypes"):
        return ctypes.c_void_p(t.ctypes.data)
    return ctypes.c_void_p(t)


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


_no_excl = {}   # device index -> a one-element int32 tensor standing in for an empty exclusion list


def _excl(t):
    """excl_idx as the library takes it: the C calls want a valid device pointer even when there are no
    exclusions (excl_off all zero), which an empty tensor does not have; a one-element tensor that is never
    read stands in for it."""
    if t is None or t.numel() > 0:
        return t
    import torch
    dev = t.device.index if t.device.index is not None else 0
    if dev not in _no_excl:
        _no_excl[dev] = torch.zeros(1, dtype=torch.int32, device=t.device)
    return _no_excl[dev]


def _need(t, dtype, numel, name):
    import torch
    if t.device.type != "cuda" or t.dtype != dtype or t.numel() < numel or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s CUDA tensor with >= %d elements" % (name, dtype, numel))


# ---------------------------------------------------------------- context

_allocators = {}   # context address -> the nb_allocator (and its callbacks) it was created with


def torch_allocator(device=0):
    """An nb_allocator backed by PyTorch's caching allocator: the library's grids, lists and scratch come from
    the same pool as the caller's tensors (allocation on the library's stream, stream-ordered reuse)."""
    import torch

    def _alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=device, stream=int(stream or 0))
        except RuntimeError:   # out of memory: the library reports NB_ERR_OOM
            return None

    def _free(ptr, stream, user):
        torch.cuda.caching_allocator_delete(ptr)

    return nb_allocator(_ALLOC_FN(_alloc), _FREE_FN(_free), None)


def nb_create(device=0, stream=None, allocator="torch"):
    """allocator: "torch" (PyTorch's caching allocator, the default), an nb_allocator, or None (hipMalloc)."""
    if isinstance(allocator, str):
        if allocator != "torch":
            raise ValueError("allocator must be 'torch', an nb_allocator or None")
        allocator = torch_allocator(device)
    h = ctypes.c_void_p()
    _check(lib().nb_create(ctypes.byref(h), int(device), _stream(stream),
                           ctypes.byref(allocator) if allocator is not None else None))
    if allocator is not None:
        _allocators[h.value] = allocator
    return h


def nb_destroy(ctx):
    lib().nb_destroy(ctx)
    _allocators.pop(ctx.value if isinstance(ctx, ctypes.c_void_p) else ctx, None)


def nb_memory_info(ctx):
    """(bytes held through the caller's allocator, bytes held through hipMalloc) by the context's handles."""
    a, h = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().nb_memory_info(ctx, ctypes.byref(a), ctypes.byref(h)))
    return a.value, h.value


def nb_set_stream(ctx, stream=None):
    _check(lib().nb_set_stream(ctx, _stream(stream)))


def nb_sync(ctx):
    return _check(lib().nb_sync(ctx))


def nb_last_error():
    return lib().nb_last_error().decode()


# ------------------------------------------------------------------ grid

def nb_grid_sort(ctx, box, xyzq, type_, shape, grid=None):
    """box: 3 floats (host); xyzq: (n,4) float32 cuda; type_: (n,) int32 cuda; shape: (m, n)."""
    import torch
    n = xyzq.shape[0]
    _need(xyzq, torch.float32, 4 * n, "xyzq")
    _need(type_, torch.int32, n, "type")
    b = (ctypes.c_double * 3)(*[float(v) for v in box])
    h = grid if grid is not None else ctypes.c_void_p()
    _check(lib().nb_grid_sort(ctx, b, int(n), _ptr(xyzq), _ptr(type_), nb_shape(*shape), ctypes.byref(h)))
    return h


def nb_grid_free(grid):
    lib().nb_grid_free(grid)


def nb_grid_info(grid):
    info = nb_grid_info_t()
    _check(lib().nb_grid_info(grid, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in nb_grid_info_t._fields_}


def nb_grid_export(grid):
    """Host copies (numpy) of perm, sorted xyzq, per-particle image, column starts, i-cluster boxes."""
    import numpy as np
    info = nb_grid_info(grid)
    ns, n, nci = info["n_slots"], info["n"], info["n_ci"]
    perm = np.empty(ns, np.int32)
    xyzq = np.empty((ns, 4), np.float32)
    img = np.empty((n, 3), np.int32)
    cs = np.empty(info["nx"] * info["ny"] + 1, np.int32)
    bb = np.empty((nci, 8), np.float32)
    _check(lib().nb_grid_export(grid, _ptr(perm), _ptr(xyzq), _ptr(img), _ptr(cs), _ptr(bb)))
    return dict(info=info, perm=perm, xyzq=xyzq, img=img, col_start=cs, bb=bb)


# ------------------------------------------------------------------ list

def nb_pairlist_build(ctx, grid, rlist, rbb, excl_off, excl_idx, flags=0, lst=None):
    import torch
    _need(excl_off, torch.int32, 1, "excl_off")
    h = lst if lst is not None else ctypes.c_void_p()
    _check(lib().nb_pairlist_build(ctx, grid, float(rlist), float(rbb), _ptr(excl_off), _ptr(_excl(excl_idx)), int(flags),
                                   ctypes.byref(h)))
    return h


def nb_pairlist_prune(ctx, outer, xyzq_now, r, inner=None):
    """Second stage of a two-stage list: the entries of `outer` with a particle pair within r at xyzq_now."""
    h = inner if inner is not None else ctypes.c_void_p()
    _check(lib().nb_pairlist_prune(ctx, outer, _ptr(xyzq_now), float(r), ctypes.byref(h)))
    return h


def nb_rdf(ctx, grid, lst, xyzq_now, r_max, nbins, ntypes, hist, skip_excluded=False):
    """Pair distance histogram added to hist (uint64 CUDA tensor of ntypes*ntypes*nbins; torch int64 is fine)."""
    _check(lib().nb_rdf(ctx, grid, lst, _ptr(xyzq_now), float(r_max), int(nbins), int(ntypes),
                        NB_RDF_SKIP_EXCLUDED if skip_excluded else 0, _ptr(hist)))


def nb_list_free(lst):
    lib().nb_list_free(lst)


def nb_list_info(lst):
    ne, ni = ctypes.c_long(), ctypes.c_long()
    _check(lib().nb_list_info(lst, ctypes.byref(ne), ctypes.byref(ni)))
    return ne.value, ni.value


ENTRY_DTYPE = [("ci", "<i4"), ("shift", "<i4"), ("cj", "<i4"), ("pad", "<i4"), ("mask", "<u8")]


def nb_list_export_canonical(lst):
    import numpy as np
    ne, _ = nb_list_info(lst)
    out = np.zeros(max(ne, 1), dtype=np.dtype(ENTRY_DTYPE))
    cnt = ctypes.c_long()
    _check(lib().nb_list_export_canonical(lst, _ptr(out), ctypes.c_long(ne), ctypes.byref(cnt)))
    return out[:cnt.value]


# ---------------------------------------------------------------- forces

def make_params(rc, beta, coulomb_f, c6c12, shift_energies=True, coulomb=0, eps_rf=0.0):
    """nb_params with c6c12 a (ntypes, ntypes, 2) float32 CUDA tensor (kept referenced by the struct's owner).
    coulomb: NB_COULOMB_EWALD (default), NB_COULOMB_RF (eps_rf: permittivity beyond rc, 0 = conducting) or
    NB_COULOMB_EWALD_TABLE."""
    nt = c6c12.shape[0]
    p = nb_params(float(rc), float(beta), float(coulomb_f), int(nt), c6c12.data_ptr(), int(bool(shift_energies)),
                  int(coulomb), float(eps_rf))
    p._keep = c6c12
    return p


def nb_set_force_variant(ctx, variant):
    _check(lib().nb_set_force_variant(ctx, int(variant)))


def nb_set_super_cluster(ctx, clusters=0, entries=0):
    _check(lib().nb_set_super_cluster(ctx, int(clusters), int(entries)))


def nb_set_search_parts(ctx, parts):
    """Wavefronts per i-cluster in the pair search: 1, 2, 4, 8, or 0 for automatic."""
    _check(lib().nb_set_search_parts(ctx, int(parts)))


def nb_forces(ctx, grid, lst, xyzq_now, params, flags, f, energy=None, virial=None):
    _check(lib().nb_forces(ctx, grid, lst, _ptr(xyzq_now), ctypes.byref(params), int(flags), _ptr(f), _ptr(energy),
                           _ptr(virial)))


def nb_forces_noalloc(ctx, grid, lst, xyzq_now, params, flags, f, energy=None, virial=None):
    """nb_forces without any device allocation (static library scratch; see include/mxn.h)."""
    _check(lib().nb_forces_noalloc(ctx, grid, lst, _ptr(xyzq_now), ctypes.byref(params), int(flags), _ptr(f),
                                   _ptr(energy), _ptr(virial)))


# --------------------------------------------------------------- recount

def nb_recount(ctx, grid, lst, xyzq_t, params, c_bb, db, nbins, hist):
    """Missed-pair energy histogram (hist: (nbins,) float64 CUDA tensor, overwritten)."""
    _check(lib().nb_recount(ctx, grid, lst, _ptr(xyzq_t), ctypes.byref(params), float(c_bb), float(db), int(nbins),
                            _ptr(hist)))


# ------------------------------------------------------- buffer estimate

def _query(T, dt, nstlist, mass, charge, c6c12, count, volume, rc, beta, coulomb_f, shape, target):
    """nb_buffer_query and the arrays it points to (kept alive by the caller)."""
    import numpy as np
    mass = np.ascontiguousarray(mass, np.float64); charge = np.ascontiguousarray(charge, np.float64)
    c6c12 = np.ascontiguousarray(c6c12, np.float64); count = np.ascontiguousarray(count, np.float64)
    q = nb_buffer_query(float(T), float(dt), int(nstlist), int(mass.shape[0]), mass.ctypes.data, charge.ctypes.data,
                        c6c12.ctypes.data, count.ctypes.data, float(volume), float(rc), float(beta),
                        float(coulomb_f), nb_shape(*shape), float(target))
    return q, (mass, charge, c6c12, count)


def nb_buffer_estimate(ctx, *, T, dt, nstlist, mass, charge, c6c12, count, volume, rc, beta, coulomb_f, shape,
                       target, mode=NB_BUFFER_ANALYTIC):
    q, keep = _query(T, dt, nstlist, mass, charge, c6c12, count, volume, rc, beta, coulomb_f, shape, target)
    rb, drift, fb = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    _check(lib().nb_buffer_estimate(ctx, ctypes.byref(q), int(mode), ctypes.byref(rb), ctypes.byref(drift),
                                    ctypes.byref(fb)))
    return rb.value, drift.value, bool(fb.value)


# ------------------------------------------------------- instrumentation

def nb_timing_enable(ctx, on=True, timers=None):
    """Every timer (on=True), none (on=False), or only the NB_TIMER_* indices in `timers`."""
    if not on:
        val = 0
    elif timers is None:
        val = 1
    else:
        val = NB_TIMING_SELECT | sum(1 << int(t) for t in timers)
    _check(lib().nb_timing_enable(ctx, val))


def nb_timing_read(ctx):
    """{timer: (total_ms, launches)} since the last read (synchronous)."""
    ms = (ctypes.c_double * NB_TIMER_COUNT)()
    cnt = (ctypes.c_long * NB_TIMER_COUNT)()
    _check(lib().nb_timing_read(ctx, ms, cnt))
    names = ("force_kernel", "force_call", "grid_sort", "pairlist")
    return {names[k]: (ms[k], cnt[k]) for k in range(NB_TIMER_COUNT)}


def nb_list_stats(ctx, grid, lst, xyzq_now, rc):
    """(listed pairs, real visited pairs, interacting pairs with r < rc, excluded pairs with r < rc)."""
    c = (ctypes.c_longlong * 4)()
    _check(lib().nb_list_stats(ctx, grid, lst, _ptr(xyzq_now), float(rc), c))
    return tuple(int(v) for v in c)


# ------------------------------------------------------------------- MLP

def nb_mlp_create(ctx, params, lo, hi):
    """params: host float32[4801]; lo, hi: feature ranges (8 each)."""
    import numpy as np
    p = np.ascontiguousarray(params, np.float32)
    if p.size != NB_MLP_PARAMS:
        raise ValueError("need %d parameters" % NB_MLP_PARAMS)
    lo = np.ascontiguousarray(lo, np.float64); hi = np.ascontiguousarray(hi, np.float64)
    h = ctypes.c_void_p()
    _check(lib().nb_mlp_create(ctx, _ptr(p), _ptr(lo), _ptr(hi), ctypes.byref(h)))
    return h


def nb_mlp_free(mlp):
    lib().nb_mlp_free(mlp)


def nb_mlp_get_params(mlp):
    import numpy as np
    p = np.empty(NB_MLP_PARAMS, np.float32)
    _check(lib().nb_mlp_get_params(mlp, _ptr(p)))
    return p


def nb_mlp_train_step(ctx, mlp, X, y, lr, loss=None):
    _check(lib().nb_mlp_train_step(ctx, mlp, _ptr(X), _ptr(y), int(X.shape[0]), float(lr), _ptr(loss)))


def nb_mlp_grad(ctx, mlp, X, y, grad, loss=None):
    _check(lib().nb_mlp_grad(ctx, mlp, _ptr(X), _ptr(y), int(X.shape[0]), _ptr(grad), _ptr(loss)))


def nb_mlp_infer(ctx, mlp, X, y):
    _check(lib().nb_mlp_infer(ctx, mlp, _ptr(X), int(X.shape[0]), _ptr(y)))


def nb_mlp_set_domain(mlp, *, dt, charge, c6c12, rc, beta, target, T=300.0, nstlist=10, mass=(1.0,),
                      count=None, volume=1.0, coulomb_f=138.935458, shape=(8, 8)):
    """Record the conditions the model's labels were generated for (target, dt, beta*rc, charges, LJ)."""
    nt = len(charge)
    mass = list(mass) * nt if len(mass) == 1 else mass
    count = [1.0] * nt if count is None else count
    q, keep = _query(T, dt, nstlist, mass, charge, c6c12, count, volume, rc, beta, coulomb_f, shape, target)
    _check(lib().nb_mlp_set_domain(mlp, ctypes.byref(q)))


def nb_buffer_set_mlp(ctx, mlp, margin):
    _check(lib().nb_buffer_set_mlp(ctx, mlp, float(margin)))


# ----------------------------------------------------------------- batch

def nb_batch_create(ctx, grids, lists, xyzq_now, forces):
    """grids, lists: handle lists; xyzq_now, forces: CUDA tensors per replica (bound to the batch)."""
    n = len(grids)
    ga = (ctypes.c_void_p * n)(*[g.value for g in grids])
    la = (ctypes.c_void_p * n)(*[lst.value for lst in lists])
    xa = (ctypes.c_void_p * n)(*[t.data_ptr() for t in xyzq_now])
    fa = (ctypes.c_void_p * n)(*[t.data_ptr() for t in forces])
    h = ctypes.c_void_p()
    _check(lib().nb_batch_create(ctx, n, ga, la, xa, fa, ctypes.byref(h)))
    h._keep = (list(xyzq_now), list(forces))
    return h


def nb_batch_free(batch):
    lib().nb_batch_free(batch)


def nb_batch_set_group(batch, items_per_group):
    _check(lib().nb_batch_set_group(batch, int(items_per_group)))


def nb_batch_set_grid(batch, waves):
    _check(lib().nb_batch_set_grid(batch, int(waves)))


def nb_batch_forces(ctx, batch, params, flags, energy=None, virial=None):
    _check(lib().nb_batch_forces(ctx, batch, ctypes.byref(params), int(flags), _ptr(energy), _ptr(virial)))


def nb_batch_capture(ctx, batch, params, flags, energy=None, virial=None):
    _check(lib().nb_batch_capture(ctx, batch, ctypes.byref(params), int(flags), _ptr(energy), _ptr(virial)))


def nb_batch_replay(ctx, batch):
    _check(lib().nb_batch_replay(ctx, batch))


def nb_batch_bind_topology(batch, types, excl_offs, excl_idxs):
    """types, excl_offs, excl_idxs: int32 CUDA tensors per replica (kept alive by the batch handle)."""
    n = len(types)
    ta = (ctypes.c_void_p * n)(*[t.data_ptr() for t in types])
    oa = (ctypes.c_void_p * n)(*[t.data_ptr() for t in excl_offs])
    excl_idxs = [_excl(t) for t in excl_idxs]
    ia = (ctypes.c_void_p * n)(*[t.data_ptr() for t in excl_idxs])
    _check(lib().nb_batch_bind_topology(batch, ta, oa, ia))
    batch._keep_topology = (list(types), list(excl_offs), excl_idxs)


def nb_batch_rebuild(ctx, batch):
    _check(lib().nb_batch_rebuild(ctx, batch))


def nb_batch_capture_cycle(ctx, batch, nsteps, params, flags, energy=None, virial=None):
    _check(lib().nb_batch_capture_cycle(ctx, batch, int(nsteps), ctypes.byref(params), int(flags), _ptr(energy),
                                        _ptr(virial)))


# -------------------------------------------------------------- autotuner

def nb_autotune(ctx, boxes, xyzq, types, excl_off, excl_idx, rlist, params, flags, shapes, groups, reps=5):
    """Fastest (shape, group) of the batched force launch over the replicas, measured by the library.

    boxes: (n_rep, 3) box edges; xyzq, types, excl_off, excl_idx: per-replica CUDA tensors.  Returns
    ((m, n), group, table) with table[shape, group] the mean milliseconds per batched launch."""
    import numpy as np
    nr = len(xyzq)
    box = np.ascontiguousarray(np.asarray(boxes, np.float64).reshape(nr, 3))
    n = np.ascontiguousarray([t.shape[0] for t in xyzq], np.int32)
    excl_idx = [_excl(t) for t in excl_idx]
    arrs = [(ctypes.c_void_p * nr)(*[t.data_ptr() for t in ts]) for ts in (xyzq, types, excl_off, excl_idx)]
    rep = nb_replicas(nr, box.ctypes.data, n.ctypes.data, *[ctypes.cast(a, ctypes.c_void_p) for a in arrs])
    shp = (nb_shape * len(shapes))(*[nb_shape(*sh) for sh in shapes])
    grp = (ctypes.c_int * len(groups))(*[int(g) for g in groups])
    best, bg = nb_shape(), ctypes.c_int()
    table = np.zeros(len(shapes) * len(groups), np.float32)
    _check(lib().nb_autotune(ctx, ctypes.byref(rep), float(rlist), ctypes.byref(params), int(flags), shp, len(shapes),
                             grp, len(groups), int(reps), ctypes.byref(best), ctypes.byref(bg), _ptr(table)))
    return (best.m, best.n), bg.value, table.reshape(len(shapes), len(groups))
