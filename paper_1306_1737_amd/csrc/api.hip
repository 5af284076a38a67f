// C ABI entry points: argument validation, handle and storage management,
// error reporting.  All numerical work is in the kernels of grid.hip,
// pairlist.hip and forces.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "internal.h"

namespace mxn {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int status, const std::string &msg) {
    g_last_error = msg;
    return status;
}

int ensure(const nb_ctx *c, DevBuf &b, size_t bytes) {
    if (bytes <= b.bytes && b.p) return NB_OK;
    if (!c) return fail(NB_ERR_STATE, "internal: device buffer without a context");
    release(b);
    const size_t want = bytes ? (bytes + 255) / 256 * 256 : 256;
    if (c->alloc.alloc) {
        void *p = c->alloc.alloc(want, (void *)c->stream, c->alloc.user);
        if (!p)
            return fail(NB_ERR_OOM, std::string("the caller's allocator returned no memory for ") + std::to_string(want) +
                                        " bytes");
        b.p = p;
        b.al = c->alloc;
        b.stream = (void *)c->stream;
        c->mem->via_allocator += want;
    } else {
        hipError_t e = hipMalloc(&b.p, want);
        if (e != hipSuccess) {
            b.p = nullptr;
            return fail(NB_ERR_OOM, std::string("hipMalloc of ") + std::to_string(want) + " bytes: " + hipGetErrorString(e));
        }
        b.al = nb_allocator{};
        b.stream = nullptr;
        c->mem->via_hip += want;
    }
    b.bytes = want;
    b.mem = c->mem;
    return NB_OK;
}

void release(DevBuf &b) {
    if (b.p) {
        if (b.al.free) {
            b.al.free(b.p, b.stream, b.al.user);
            if (b.mem) b.mem->via_allocator -= b.bytes;
        } else {
            (void)hipFree(b.p);   // teardown: nothing to report to
            if (b.mem) b.mem->via_hip -= b.bytes;
        }
    }
    b.p = nullptr;
    b.bytes = 0;
    b.mem.reset();
}

static hipEvent_t take_event(nb_ctx *c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ScopedTimer::ScopedTimer(nb_ctx *c, int w) : ctx(c), which(w) {
    if (which < 0 || !((ctx->timing >> which) & 1)) return;
    hipEvent_t start = take_event(ctx);
    stop = take_event(ctx);
    if (!start || !stop) {
        stop = nullptr;
        return;
    }
    (void)hipEventRecord(start, ctx->stream);   // a failed record shows as a missing sample
    ctx->timers[which].push_back({start, stop});
}

ScopedTimer::~ScopedTimer() {
    if (stop) (void)hipEventRecord(stop, ctx->stream);
}

double analytic_drift(const nb_buffer_query &q, double rb);
int analytic_buffer(const nb_buffer_query &q, double *rb_out, double *drift_out);
int validate_query(const nb_buffer_query *q);

}  // namespace mxn

using namespace mxn;

#define CHECK(rc_expr)            \
    do {                          \
        int rc_ = (rc_expr);      \
        if (rc_ != NB_OK) return rc_; \
    } while (0)

extern "C" {

const char *nb_last_error(void) { return g_last_error.c_str(); }

int nb_create(nb_ctx **ctx, int device, void *hip_stream, const nb_allocator *allocator) {
    if (!ctx) return fail(NB_ERR_ARG, "nb_create: ctx is null");
    if (allocator && (!allocator->alloc || !allocator->free))
        return fail(NB_ERR_ARG, "nb_create: an allocator needs both alloc and free");
    *ctx = nullptr;
    int ndev = 0;
    MXN_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(NB_ERR_ARG, "nb_create: no such device");
    MXN_HIP(hipSetDevice(device));
    nb_ctx *c = new (std::nothrow) nb_ctx();
    if (!c) return fail(NB_ERR_OOM, "nb_create: host allocation");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (allocator) c->alloc = *allocator;
    int rc = ensure(c, c->flags_buf, sizeof(int));
    if (rc != NB_OK) {
        delete c;
        return rc;
    }
    c->d_flags = (int *)c->flags_buf.p;
    {
        // the static scratch of nb_forces_noalloc: its address on this device, looked up once per device
        static std::mutex mu;
        static void *addr[64] = {};
        static int status[64] = {};
        std::lock_guard<std::mutex> lock(mu);
        if (device < 64) {
            if (!addr[device] && status[device] == 0) {
                status[device] = noalloc_scratch_address(&addr[device]) == NB_OK ? 1 : -1;
                if (status[device] < 0) c->noalloc_error = nb_last_error();
            }
            c->noalloc_scratch = addr[device];
            if (!c->noalloc_scratch && c->noalloc_error.empty())
                c->noalloc_error = "the static scratch address could not be looked up on this device";
        } else {
            c->noalloc_error = "devices beyond 63 have no static scratch";
        }
    }
    hipError_t e = hipMemsetAsync(c->d_flags, 0, sizeof(int), c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_pinned, 16 * sizeof(int));
    if (e != hipSuccess) {
        release(c->flags_buf);
        delete c;
        return fail(NB_ERR_HIP, std::string("nb_create: ") + hipGetErrorString(e));
    }
    *ctx = c;
    return NB_OK;
}

void nb_destroy(nb_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);   // teardown: errors cannot be reported from here
    (void)hipStreamSynchronize(c->stream);
    for (auto &v : c->timers)
        for (auto &pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    release(c->partials);
    release(c->blockpart);
    release(c->etab);
    release(c->rdf_edge);
    release(c->mlp_io);
    release(c->stats_buf);
    release(c->flags_buf);
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    delete c;
}

int nb_memory_info(const nb_ctx *c, size_t *via_allocator, size_t *via_hip) {
    if (!c) return fail(NB_ERR_ARG, "nb_memory_info: ctx is null");
    if (via_allocator) *via_allocator = c->mem->via_allocator.load();
    if (via_hip) *via_hip = c->mem->via_hip.load();
    return NB_OK;
}

int nb_set_stream(nb_ctx *c, void *hip_stream) {
    if (!c) return fail(NB_ERR_ARG, "nb_set_stream: ctx is null");
    c->stream = (hipStream_t)hip_stream;
    return NB_OK;
}

int nb_sync(nb_ctx *c) {
    if (!c) return fail(NB_ERR_ARG, "nb_sync: ctx is null");
    MXN_HIP(hipSetDevice(c->device));
    MXN_HIP(hipStreamSynchronize(c->stream));
    int flags = 0;
    MXN_HIP(hipMemcpy(&flags, c->d_flags, sizeof(int), hipMemcpyDeviceToHost));
    if (flags) MXN_HIP(hipMemset(c->d_flags, 0, sizeof(int)));
    if (flags & FLAG_NONFINITE) return fail(NB_ERR_NONFINITE, "non-finite or out-of-range coordinate or charge");
    if (flags & FLAG_OVERFLOW) return fail(NB_ERR_OVERFLOW, "pair-list capacity exceeded: rebuild the list");
    if (flags & FLAG_TYPE)
        return fail(NB_ERR_ARG, "an LJ type outside [0, ntypes): such particles were computed with a valid row "
                                "and their results are wrong");
    if (flags & FLAG_FORCE_RANGE)
        return fail(NB_ERR_NONFINITE, "a force term is non-finite or beyond the summation range (|F| >= 2^36 "
                                      "kJ/mol/nm, overlapping particles): those forces are NaN");
    return NB_OK;
}

// ------------------------------------------------------------------- grid

static void grid_release(nb_grid *g) {
    DevBuf *bufs[] = {&g->col_count, &g->col_start, &g->col_fill, &g->colbb, &g->col_hist, &g->atom_col, &g->atom_xw,
                      &g->atom_img, &g->bucket, &g->xs, &g->xs_now, &g->type_s, &g->perm, &g->img_s,
                      &g->slot_of, &g->bbi_lo, &g->bbi_hi, &g->bbj_lo, &g->bbj_hi, &g->nslots,
                      &g->shiftvec};
    for (DevBuf *b : bufs) release(*b);
}

int nb_grid_sort(nb_ctx *c, const double box[3], int n, const float *xyzq, const int *type, nb_shape shape,
                 nb_grid **grid) {
    if (!c || !box || !xyzq || !type || !grid) return fail(NB_ERR_ARG, "nb_grid_sort: null argument");
    if (n < 1) return fail(NB_ERR_ARG, "nb_grid_sort: n must be >= 1");
    const bool ok_shape = (shape.m == 4 && shape.n == 4) || (shape.m == 4 && shape.n == 8) ||
                          (shape.m == 8 && shape.n == 4) || (shape.m == 8 && shape.n == 8);
    if (!ok_shape) return fail(NB_ERR_ARG, "nb_grid_sort: supported shapes are 4x4, 4x8, 8x4, 8x8");
    for (int d = 0; d < 3; ++d)
        if (!(box[d] > 0.0) || !std::isfinite(box[d])) return fail(NB_ERR_ARG, "nb_grid_sort: bad box");
    MXN_HIP(hipSetDevice(c->device));
    nb_grid *g = *grid;
    if (g && g->ctx != c) return fail(NB_ERR_STATE, "nb_grid_sort: grid belongs to another context");
    bool fresh = false;
    if (!g) {
        g = new (std::nothrow) nb_grid();
        if (!g) return fail(NB_ERR_OOM, "nb_grid_sort: host allocation");
        g->ctx = c;
        fresh = true;
    }
    g->n = n;
    g->m = shape.m;
    g->nn = shape.n;
    g->cmin = shape.m < shape.n ? shape.m : shape.n;
    g->cmax = shape.m > shape.n ? shape.m : shape.n;
    for (int d = 0; d < 3; ++d) {
        g->box[d] = box[d];
        g->Lf[d] = (float)box[d];
        g->invL[d] = 1.0 / (double)g->Lf[d];
    }
    // column grid: spacing (max(M,N)/rho)^(1/3), rho = n / V
    const double rho = (double)n / (box[0] * box[1] * box[2]);
    const double s = std::cbrt((double)g->cmax / rho);
    g->spacing = s;
    g->nx = (int)std::floor(box[0] / s);
    g->ny = (int)std::floor(box[1] / s);
    if (g->nx < 1) g->nx = 1;
    if (g->ny < 1) g->ny = 1;
    g->inv_x = (float)((double)g->nx / box[0]);
    g->inv_y = (float)((double)g->ny / box[1]);
    g->ncol = g->nx * g->ny;
    long cap = (long)n + (long)g->ncol * (g->cmax - 1);
    cap = (cap + g->cmax - 1) / g->cmax * g->cmax;
    if (cap > (1L << 30)) return fail(NB_ERR_ARG, "nb_grid_sort: too many particles");
    g->slots_cap = (int)cap;
    const size_t nc = (size_t)g->ncol, ns = (size_t)cap, na = (size_t)n;
    int rc = NB_OK;
    rc = rc ? rc : ensure(g->ctx, g->col_count, nc * 4);
    rc = rc ? rc : ensure(g->ctx, g->col_start, (nc + 1) * 4);
    rc = rc ? rc : ensure(g->ctx, g->col_fill, nc * 4);
    rc = rc ? rc : ensure(g->ctx, g->col_hist, nc * (size_t)hist_blocks(n) * 4);
    rc = rc ? rc : ensure(g->ctx, g->colbb, nc * 16);
    rc = rc ? rc : ensure(g->ctx, g->atom_col, na * 4);
    rc = rc ? rc : ensure(g->ctx, g->atom_xw, na * 16);
    rc = rc ? rc : ensure(g->ctx, g->atom_img, na * 4);
    rc = rc ? rc : ensure(g->ctx, g->slot_of, na * 4);
    rc = rc ? rc : ensure(g->ctx, g->bucket, ns * 4);
    rc = rc ? rc : ensure(g->ctx, g->xs, ns * 16);
    rc = rc ? rc : ensure(g->ctx, g->xs_now, ns * 16);
    rc = rc ? rc : ensure(g->ctx, g->type_s, ns * 4);
    rc = rc ? rc : ensure(g->ctx, g->perm, ns * 4);
    rc = rc ? rc : ensure(g->ctx, g->img_s, ns * 4);
    rc = rc ? rc : ensure(g->ctx, g->bbi_lo, ns / g->m * 16);
    rc = rc ? rc : ensure(g->ctx, g->bbi_hi, ns / g->m * 16);
    if (g->nn != g->m) {
        rc = rc ? rc : ensure(g->ctx, g->bbj_lo, ns / g->nn * 16);
        rc = rc ? rc : ensure(g->ctx, g->bbj_hi, ns / g->nn * 16);
    }
    rc = rc ? rc : ensure(g->ctx, g->nslots, 16);
    rc = rc ? rc : ensure(g->ctx, g->shiftvec, 32 * 16);
    if (rc == NB_OK) {
        ScopedTimer tm(c, NB_TIMER_GRID_SORT);
        rc = launch_grid_sort(g, xyzq, type);
    }
    ++g->generation;
    if (rc != NB_OK) {
        if (fresh) {
            grid_release(g);
            delete g;
        }
        return rc;
    }
    *grid = g;
    return NB_OK;
}

void nb_grid_free(nb_grid *g) {
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    grid_release(g);
    delete g;
}

int nb_grid_info(nb_grid *g, nb_grid_info_t *info) {
    if (!g || !info) return fail(NB_ERR_ARG, "nb_grid_info: null argument");
    MXN_HIP(hipSetDevice(g->ctx->device));
    int ns = 0;
    MXN_HIP(hipMemcpyAsync(&ns, g->nslots.p, sizeof(int), hipMemcpyDeviceToHost, g->ctx->stream));
    MXN_HIP(hipStreamSynchronize(g->ctx->stream));
    info->n = g->n;
    info->n_slots = ns;
    info->m = g->m;
    info->n_cl = g->nn;
    info->nx = g->nx;
    info->ny = g->ny;
    info->n_ci = ns / g->m;
    info->n_cj = ns / g->nn;
    return NB_OK;
}

int nb_grid_export(nb_grid *g, int *perm, float *xyzq, int *img, int *col_start, float *bb) {
    nb_grid_info_t info;
    CHECK(nb_grid_info(g, &info));
    const int ns = info.n_slots;
    if (perm) MXN_HIP(hipMemcpy(perm, g->perm.p, (size_t)ns * 4, hipMemcpyDeviceToHost));
    if (xyzq) MXN_HIP(hipMemcpy(xyzq, g->xs.p, (size_t)ns * 16, hipMemcpyDeviceToHost));
    if (img) {
        int *packed = new (std::nothrow) int[g->n];
        if (!packed) return fail(NB_ERR_OOM, "nb_grid_export: host allocation");
        hipError_t e = hipMemcpy(packed, g->atom_img.p, (size_t)g->n * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            delete[] packed;
            return fail(NB_ERR_HIP, hipGetErrorString(e));
        }
        for (int i = 0; i < g->n; ++i) {
            img[3 * i] = (packed[i] & 1023) - 512;
            img[3 * i + 1] = ((packed[i] >> 10) & 1023) - 512;
            img[3 * i + 2] = ((packed[i] >> 20) & 1023) - 512;
        }
        delete[] packed;
    }
    if (col_start) MXN_HIP(hipMemcpy(col_start, g->col_start.p, (size_t)(g->ncol + 1) * 4, hipMemcpyDeviceToHost));
    if (bb) {
        const size_t nci = (size_t)info.n_ci;
        float *lo = new (std::nothrow) float[nci * 8];
        if (!lo) return fail(NB_ERR_OOM, "nb_grid_export: host allocation");
        hipError_t e = hipMemcpy(lo, g->bbi_lo.p, nci * 16, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(lo + nci * 4, g->bbi_hi.p, nci * 16, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            delete[] lo;
            return fail(NB_ERR_HIP, hipGetErrorString(e));
        }
        for (size_t k = 0; k < nci; ++k) {   // w = 0 (on the device lo.w holds the real-slot mask)
            for (int d = 0; d < 3; ++d) {
                bb[8 * k + d] = lo[4 * k + d];
                bb[8 * k + 4 + d] = lo[nci * 4 + 4 * k + d];
            }
            bb[8 * k + 3] = bb[8 * k + 7] = 0.0f;
        }
        delete[] lo;
    }
    return NB_OK;
}

// ------------------------------------------------------------------- list

static void list_release(nb_list *l) {
    DevBuf *bufs[] = {&l->entries,    &l->entries_canon, &l->keys,        &l->items,  &l->part_count,
                      &l->part_start, &l->part_istart,   &l->totals,      &l->jcount, &l->jstart,
                      &l->jrank,      &l->jrank_canon,   &l->fj,          &l->fi,
                      &l->sci_ent,    &l->sci_mask,      &l->sci_count,   &l->sci_base, &l->sci_istart,
                      &l->sci_items,  &l->sci_jcount,    &l->sci_jstart,  &l->sci_totals, &l->sci_fi};
    for (DevBuf *b : bufs) release(*b);
}

int nb_pairlist_build(nb_ctx *c, const nb_grid *g, float rlist, float rbb, const int *excl_off, const int *excl_idx,
                      int flags, nb_list **list) {
    if (!c || !g || !excl_off || !excl_idx || !list) return fail(NB_ERR_ARG, "nb_pairlist_build: null argument");
    if (g->ctx != c) return fail(NB_ERR_STATE, "nb_pairlist_build: grid belongs to another context");
    if (!(rlist > 0.0f) || !std::isfinite(rlist)) return fail(NB_ERR_ARG, "nb_pairlist_build: rlist must be > 0");
    if (flags & ~(NB_LIST_ASYNC | NB_LIST_BY_DISTANCE)) return fail(NB_ERR_ARG, "nb_pairlist_build: unknown flag");
    for (int d = 0; d < 3; ++d)
        if (!((double)g->Lf[d] > 2.0 * (double)rlist))
            return fail(NB_ERR_BOX, "nb_pairlist_build: every box edge must exceed 2*rlist");
    MXN_HIP(hipSetDevice(c->device));
    nb_list *l = *list;
    bool fresh = false;
    if (l && l->ctx != c) return fail(NB_ERR_STATE, "nb_pairlist_build: list belongs to another context");
    if (!l) {
        l = new (std::nothrow) nb_list();
        if (!l) return fail(NB_ERR_OOM, "nb_pairlist_build: host allocation");
        l->ctx = c;
        fresh = true;
    }
    l->grid = g;
    l->grid_generation = g->generation;
    l->rlist = rlist;
    l->rbb = rbb >= 0.0f ? rbb : (float)std::fmax(0.0, (double)rlist - 0.5 * g->spacing);
    const int nci_cap = g->slots_cap / g->m;
    int rc = NB_OK;
    const size_t nreg = (size_t)nci_cap * kMaxSearchParts + 1;
    rc = rc ? rc : ensure(l->ctx, l->part_count, nreg * 4);
    rc = rc ? rc : ensure(l->ctx, l->part_start, nreg * 4);
    rc = rc ? rc : ensure(l->ctx, l->part_istart, nreg * 4);
    rc = rc ? rc : ensure(l->ctx, l->totals, 16);
    // entry and item capacities are set by the reserving (synchronous) build
    if (rc == NB_OK) {
        ScopedTimer tm(c, NB_TIMER_PAIRLIST);
        rc = launch_pairlist(l, excl_off, excl_idx, !(flags & NB_LIST_ASYNC), (flags & NB_LIST_BY_DISTANCE) != 0);
    }
    if (rc != NB_OK) {
        if (fresh) {
            list_release(l);
            delete l;
        }
        return rc;
    }
    *list = l;
    return NB_OK;
}

int nb_pairlist_prune(nb_ctx *c, const nb_list *outer, const float *xyzq_now, float r, nb_list **inner) {
    if (!c || !outer || !xyzq_now || !inner) return fail(NB_ERR_ARG, "nb_pairlist_prune: null argument");
    if (outer->ctx != c) return fail(NB_ERR_STATE, "nb_pairlist_prune: list belongs to another context");
    if (*inner == outer) return fail(NB_ERR_ARG, "nb_pairlist_prune: the pruned list must be another handle");
    if (*inner && (*inner)->ctx != c) return fail(NB_ERR_STATE, "nb_pairlist_prune: list belongs to another context");
    if (!(r > 0.0f) || !std::isfinite(r)) return fail(NB_ERR_ARG, "nb_pairlist_prune: r must be > 0");
    const nb_grid *g = outer->grid;
    if (!g || outer->resv_parts == 0) return fail(NB_ERR_STATE, "nb_pairlist_prune: the outer list was never built");
    if (outer->grid_generation != g->generation)
        return fail(NB_ERR_STATE, "nb_pairlist_prune: the outer list was built before its grid's last sort");
    MXN_HIP(hipSetDevice(c->device));
    nb_list *l = *inner;
    bool fresh = false;
    if (!l) {
        l = new (std::nothrow) nb_list();
        if (!l) return fail(NB_ERR_OOM, "nb_pairlist_prune: host allocation");
        l->ctx = c;
        fresh = true;
    }
    int rc;
    {
        ScopedTimer tm(c, NB_TIMER_PAIRLIST);
        rc = launch_gather(c, g, xyzq_now);
        rc = rc ? rc : launch_prune(l, outer, r);
    }
    if (rc != NB_OK) {
        if (fresh) {
            list_release(l);
            delete l;
        }
        return rc;
    }
    *inner = l;
    return NB_OK;
}

void nb_list_free(nb_list *l) {
    if (!l) return;
    (void)hipSetDevice(l->ctx->device);
    (void)hipStreamSynchronize(l->ctx->stream);
    list_release(l);
    delete l;
}

int nb_list_info(nb_list *l, long *n_entries, long *n_items) {
    if (!l) return fail(NB_ERR_ARG, "nb_list_info: null list");
    MXN_HIP(hipSetDevice(l->ctx->device));
    int t[4];
    MXN_HIP(hipMemcpyAsync(t, l->totals.p, sizeof t, hipMemcpyDeviceToHost, l->ctx->stream));
    MXN_HIP(hipStreamSynchronize(l->ctx->stream));
    if (t[2] == 0 && t[1] > 0) return fail(NB_ERR_OVERFLOW, "nb_list_info: list overflowed its capacity");
    if (n_entries) *n_entries = t[0];
    if (n_items) *n_items = t[2];
    return NB_OK;
}

int nb_list_export_canonical(nb_list *l, nb_entry *out, long cap, long *count) {
    if (!l || (!out && cap > 0)) return fail(NB_ERR_ARG, "nb_list_export_canonical: null argument");
    long ne = 0;
    CHECK(nb_list_info(l, &ne, nullptr));
    if (count) *count = ne;
    const nb_grid *g = l->grid;
    const int M = g->m, N = g->nn, P = l->resv_parts;
    int ns = 0;
    MXN_HIP(hipMemcpy(&ns, g->nslots.p, sizeof(int), hipMemcpyDeviceToHost));
    const int nci = ns / M;
    const long nreg = (long)nci * P;
    std::vector<int> start, cnt;
    std::vector<nb_jentry> ent;
    try {
        start.resize(nreg + 1);
        cnt.resize(nreg > 0 ? nreg : 1);
        ent.resize(l->cap_entries > 0 ? l->cap_entries : 1);
    } catch (...) {
        return fail(NB_ERR_OOM, "nb_list_export_canonical: host allocation");
    }
    hipError_t e = hipSuccess;
    if (nreg > 0) e = hipMemcpy(start.data(), l->part_start.p, (size_t)(nreg + 1) * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && nreg > 0) e = hipMemcpy(cnt.data(), l->part_count.p, (size_t)nreg * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && l->cap_entries > 0)
        e = hipMemcpy(ent.data(), l->entries.p, (size_t)l->cap_entries * sizeof(nb_jentry), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(NB_ERR_HIP, hipGetErrorString(e));
    long k = 0;
    std::vector<nb_jentry> mine;
    for (int ci = 0; ci < nci; ++ci) {
        // the i-cluster's entries from all its regions, in canonical order (shift, then j-cluster)
        mine.clear();
        for (int p = 0; p < P; ++p) {
            const long r = (long)ci * P + p;
            const int n = std::min(cnt[r], start[r + 1] - start[r]);
            mine.insert(mine.end(), ent.begin() + start[r], ent.begin() + start[r] + n);
        }
        std::sort(mine.begin(), mine.end(), [](const nb_jentry &x, const nb_jentry &y) {
            return x.shift != y.shift ? x.shift < y.shift : x.cj < y.cj;
        });
        for (const nb_jentry &en : mine) {
            if (k < cap) {
                const uint64_t m = ((uint64_t)en.mhi << 32) | en.mlo;
                uint64_t canon = 0;   // kernel order bit b*M + a -> canonical bit a*N + b
                for (int b = 0; b < N; ++b)
                    for (int a = 0; a < M; ++a)
                        if ((m >> (b * M + a)) & 1ull) canon |= 1ull << (a * N + b);
                out[k].ci = ci;
                out[k].shift = en.shift;
                out[k].cj = en.cj;
                out[k].pad = 0;
                out[k].mask = canon;
            }
            ++k;
        }
    }
    return NB_OK;
}

// ----------------------------------------------------------------- forces

int nb_set_search_parts(nb_ctx *c, int parts) {
    if (!c) return fail(NB_ERR_ARG, "nb_set_search_parts: ctx is null");
    if (parts != 0 && parts != 1 && parts != 2 && parts != 4 && parts != 8)
        return fail(NB_ERR_ARG, "nb_set_search_parts: parts must be 0 (automatic), 1, 2, 4 or 8");
    c->search_parts = parts;
    return NB_OK;
}

int nb_set_force_variant(nb_ctx *c, int variant) {
    if (!c) return fail(NB_ERR_ARG, "nb_set_force_variant: ctx is null");
    if (variant != NB_FORCE_DIRECT && variant != NB_FORCE_SUPER)
        return fail(NB_ERR_ARG, "nb_set_force_variant: unknown variant");
    c->force_variant = variant;
    return NB_OK;
}

int nb_set_super_cluster(nb_ctx *c, int clusters, int entries) {
    if (!c) return fail(NB_ERR_ARG, "nb_set_super_cluster: ctx is null");
    if (clusters != 0 && clusters != 4 && clusters != 8)
        return fail(NB_ERR_ARG, "nb_set_super_cluster: clusters must be 0 (automatic), 4 or 8");
    if (entries < 0 || entries > 64) return fail(NB_ERR_ARG, "nb_set_super_cluster: entries must be 0..64");
    c->sci_clusters = clusters;
    c->sci_per_item = entries;
    return NB_OK;
}

static int forces_check(const char *who, nb_ctx *c, const nb_grid *g, const nb_list *l, const float *xyzq_now,
                        const nb_params *p, unsigned flags, float *f, double *energy, double *virial) {
    const std::string w(who);
    if (!c || !g || !l || !xyzq_now || !p || !f) return fail(NB_ERR_ARG, w + ": null argument");
    if (g->ctx != c || l->ctx != c || l->grid != g) return fail(NB_ERR_STATE, w + ": grid/list/context mismatch");
    if (l->grid_generation != g->generation)
        return fail(NB_ERR_STATE, w + ": the list was built before the grid's last sort: rebuild it");
    if (flags & ~(unsigned)(NB_ENERGY | NB_VIRIAL | NB_ACC_FP32 | NB_ACCUMULATE))
        return fail(NB_ERR_ARG, w + ": unknown flag");
    if ((flags & NB_ENERGY) && !energy) return fail(NB_ERR_ARG, w + ": energy output is null");
    if ((flags & NB_VIRIAL) && !virial) return fail(NB_ERR_ARG, w + ": virial output is null");
    if (!p->c6c12 || p->ntypes < 1 || p->ntypes > kMaxTypes) return fail(NB_ERR_ARG, w + ": ntypes must be 1..32");
    if (!(p->rc > 0.0f) || !(p->rc <= l->rlist)) return fail(NB_ERR_ARG, w + ": need 0 < rc <= rlist");
    if (!(p->beta >= 0.0f) || !std::isfinite(p->coulomb_f)) return fail(NB_ERR_ARG, w + ": bad beta/coulomb_f");
    if (p->coulomb < NB_COULOMB_EWALD || p->coulomb > NB_COULOMB_EWALD_TABLE)
        return fail(NB_ERR_ARG, w + ": unknown coulomb type");
    if (p->coulomb == NB_COULOMB_RF && !(p->eps_rf == 0.0f || (p->eps_rf >= 1.0f && std::isfinite(p->eps_rf))))
        return fail(NB_ERR_ARG, w + ": eps_rf must be >= 1, or 0 for a conducting boundary");
    if (p->coulomb != NB_COULOMB_RF && (double)p->beta * p->rc > 4.0)
        return fail(NB_ERR_UNSUPPORTED, w + ": beta*rc > 4 is outside the fitted Ewald range");
    if (p->coulomb == NB_COULOMB_EWALD_TABLE && p->rc > kMaxTableRc)
        return fail(NB_ERR_UNSUPPORTED, w + ": the Ewald table (LDS) covers rc <= 4 nm");
    return NB_OK;
}

int nb_forces(nb_ctx *c, const nb_grid *g, const nb_list *l, const float *xyzq_now, const nb_params *p,
              unsigned flags, float *f, double *energy, double *virial) {
    CHECK(forces_check("nb_forces", c, g, l, xyzq_now, p, flags, f, energy, virial));
    MXN_HIP(hipSetDevice(c->device));
    ScopedTimer tm(c, NB_TIMER_FORCE_CALL);
    return launch_forces(c, g, l, xyzq_now, p, flags, f, energy, virial);
}

int nb_forces_noalloc(nb_ctx *c, const nb_grid *g, const nb_list *l, const float *xyzq_now, const nb_params *p,
                      unsigned flags, float *f, double *energy, double *virial) {
    CHECK(forces_check("nb_forces_noalloc", c, g, l, xyzq_now, p, flags, f, energy, virial));
    if (!c->noalloc_scratch) return fail(NB_ERR_HIP, "nb_forces_noalloc: " + c->noalloc_error);
    if (l->cap_items < 1 || !l->fj.p || !l->fi.p)
        return fail(NB_ERR_STATE, "nb_forces_noalloc: the list has not had a synchronous build");
    MXN_HIP(hipSetDevice(c->device));
    return launch_forces(c, g, l, xyzq_now, p, flags, f, energy, virial, c->noalloc_scratch);
}

// ------------------------------------------------------------ pair histogram

int nb_rdf(nb_ctx *c, const nb_grid *g, const nb_list *l, const float *xyzq_now, float r_max, int nbins, int ntypes,
           int flags, unsigned long long *hist) {
    if (!c || !g || !l || !xyzq_now || !hist) return fail(NB_ERR_ARG, "nb_rdf: null argument");
    if (g->ctx != c || l->ctx != c || l->grid != g || l->grid_generation != g->generation)
        return fail(NB_ERR_STATE, "nb_rdf: grid/list/context mismatch or stale list");
    if (flags & ~NB_RDF_SKIP_EXCLUDED) return fail(NB_ERR_ARG, "nb_rdf: unknown flag");
    if (!(r_max > 0.0f) || !(r_max <= l->rlist)) return fail(NB_ERR_ARG, "nb_rdf: need 0 < r_max <= rlist");
    if (nbins < 1 || ntypes < 1 || ntypes > kMaxTypes) return fail(NB_ERR_ARG, "nb_rdf: bad nbins or ntypes");
    if (rdf_lds_bytes(nbins, ntypes) > 64 * 1024)
        return fail(NB_ERR_UNSUPPORTED, "nb_rdf: the histogram (ntypes^2 * nbins) and edges exceed 64 KB of LDS");
    MXN_HIP(hipSetDevice(c->device));
    int rc = launch_gather(c, g, xyzq_now, ntypes);
    return rc ? rc : launch_rdf(c, g, l, r_max, nbins, ntypes, (flags & NB_RDF_SKIP_EXCLUDED) ? 1 : 0, hist);
}

// -------------------------------------------------------- instrumentation

int nb_list_stats(nb_ctx *c, const nb_grid *g, const nb_list *l, const float *xyzq_now, float rc, long long *counts) {
    if (!c || !g || !l || !xyzq_now || !counts) return fail(NB_ERR_ARG, "nb_list_stats: null argument");
    if (g->ctx != c || l->ctx != c || l->grid != g || l->grid_generation != g->generation)
        return fail(NB_ERR_STATE, "nb_list_stats: grid/list/context mismatch");
    if (!(rc > 0.0f)) return fail(NB_ERR_ARG, "nb_list_stats: rc must be > 0");
    MXN_HIP(hipSetDevice(c->device));
    CHECK(ensure(c, c->stats_buf, 4 * sizeof(unsigned long long)));
    unsigned long long *d = (unsigned long long *)c->stats_buf.p;
    hipError_t e = hipMemsetAsync(d, 0, 4 * sizeof(unsigned long long), c->stream);
    int rc_ = e == hipSuccess ? launch_stats(c, g, l, xyzq_now, rc, d) : NB_ERR_HIP;
    unsigned long long h[4] = {0, 0, 0, 0};
    if (rc_ == NB_OK) e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (rc_ != NB_OK) return rc_;
    if (e != hipSuccess) return fail(NB_ERR_HIP, hipGetErrorString(e));
    long ne = 0;
    CHECK(nb_list_info(const_cast<nb_list *>(l), &ne, nullptr));
    counts[0] = (long long)ne * g->m * g->nn;
    counts[1] = (long long)h[0];
    counts[2] = (long long)h[1];
    counts[3] = (long long)h[2];
    return NB_OK;
}

int nb_timing_enable(nb_ctx *c, int on) {
    if (!c) return fail(NB_ERR_ARG, "nb_timing_enable: ctx is null");
    constexpr int all = (1 << NB_TIMER_COUNT) - 1;
    if (on == 0 || on == 1) c->timing = on ? all : 0;
    else if ((on & NB_TIMING_SELECT) && !(on & ~(NB_TIMING_SELECT | all))) c->timing = on & all;
    else return fail(NB_ERR_ARG, "nb_timing_enable: on must be 0, 1 or NB_TIMING_SELECT | timer bits");
    return NB_OK;
}

int nb_timing_read(nb_ctx *c, double *ms, long *launches) {
    if (!c || !ms || !launches) return fail(NB_ERR_ARG, "nb_timing_read: null argument");
    MXN_HIP(hipSetDevice(c->device));
    MXN_HIP(hipStreamSynchronize(c->stream));
    for (int t = 0; t < NB_TIMER_COUNT; ++t) {
        double sum = 0.0;
        for (auto &pr : c->timers[t]) {
            float el = 0.0f;
            if (hipEventElapsedTime(&el, pr.first, pr.second) == hipSuccess) sum += el;
            c->event_pool.push_back(pr.first);
            c->event_pool.push_back(pr.second);
        }
        ms[t] = sum;
        launches[t] = (long)c->timers[t].size();
        c->timers[t].clear();
    }
    return NB_OK;
}

// ----------------------------------------------------------------- batch

// (Re)build the replica table when a replica's storage moved or grew.
static int batch_refresh(nb_batch *b, const float *const *xyzq_now, float *const *f, bool force) {
    const size_t ds = rep_desc_size();
    bool changed = force;
    std::vector<long> caps(b->n_rep);
    for (int r = 0; r < b->n_rep; ++r) {
        const nb_list *l = b->lists[r];
        caps[r] = l->cap_items + 4;
        if (l->grid_generation != b->grids[r]->generation)
            return fail(NB_ERR_STATE, "nb_batch: a replica's list was built before its grid's last sort");
    }
    std::vector<char> host(ds * b->n_rep);
    std::vector<long> so(b->n_rep + 1), ao(b->n_rep + 1);
    long pb = 0;
    so[0] = ao[0] = 0;
    for (int r = 0; r < b->n_rep; ++r) {
        fill_rep_desc(host.data() + ds * r, b->grids[r], b->lists[r], xyzq_now ? xyzq_now[r] : nullptr,
                      f ? f[r] : nullptr, pb);
        pb += caps[r];
        so[r + 1] = so[r] + b->grids[r]->slots_cap;
        ao[r + 1] = ao[r] + b->grids[r]->n;
    }
    if (!force) {
        // keep the bound I/O pointers (the first two fields); compare the rest with the table in use
        const std::vector<char> &old = b->desc_host;
        for (int r = 0; r < b->n_rep; ++r) std::memcpy(host.data() + ds * r, old.data() + ds * r, 2 * sizeof(void *));
        changed = std::memcmp(old.data(), host.data(), ds * b->n_rep) != 0 || pb != b->pstride;
    }
    if (!changed) return NB_OK;
    if (b->graph_exec) return fail(NB_ERR_STATE, "nb_batch: replica storage changed since capture: capture again");
    CHECK(ensure(b->ctx, b->desc, ds * b->n_rep));
    CHECK(ensure(b->ctx, b->slot_off, sizeof(long) * (b->n_rep + 1)));
    CHECK(ensure(b->ctx, b->atom_off, sizeof(long) * (b->n_rep + 1)));
    CHECK(ensure(b->ctx, b->item_off, sizeof(long) * (b->n_rep + 1)));
    CHECK(ensure(b->ctx, b->partials, sizeof(double) * 11 * (size_t)pb));
    MXN_HIP(hipMemcpy(b->desc.p, host.data(), ds * b->n_rep, hipMemcpyHostToDevice));
    b->desc_host = host;
    MXN_HIP(hipMemcpy(b->slot_off.p, so.data(), sizeof(long) * (b->n_rep + 1), hipMemcpyHostToDevice));
    MXN_HIP(hipMemcpy(b->atom_off.p, ao.data(), sizeof(long) * (b->n_rep + 1), hipMemcpyHostToDevice));
    b->pstride = pb;
    b->total_slots = so[b->n_rep];
    b->total_atoms = ao[b->n_rep];
    return NB_OK;
}

int nb_batch_create(nb_ctx *c, int n_rep, nb_grid *const *grids, nb_list *const *lists, const float *const *xyzq_now,
                    float *const *f, nb_batch **out) {
    if (!c || n_rep < 1 || !grids || !lists || !xyzq_now || !f || !out)
        return fail(NB_ERR_ARG, "nb_batch_create: null argument or n_rep < 1");
    for (int r = 0; r < n_rep; ++r) {
        if (!grids[r] || !lists[r] || !xyzq_now[r] || !f[r]) return fail(NB_ERR_ARG, "nb_batch_create: null replica");
        if (grids[r]->ctx != c || lists[r]->ctx != c || lists[r]->grid != grids[r])
            return fail(NB_ERR_STATE, "nb_batch_create: grid/list/context mismatch");
        if (grids[r]->m != grids[0]->m || grids[r]->nn != grids[0]->nn)
            return fail(NB_ERR_ARG, "nb_batch_create: all replicas need the same cluster shape");
    }
    MXN_HIP(hipSetDevice(c->device));
    nb_batch *b = new (std::nothrow) nb_batch();
    if (!b) return fail(NB_ERR_OOM, "nb_batch_create: host allocation");
    b->ctx = c;
    b->n_rep = n_rep;
    b->m = grids[0]->m;
    b->nn = grids[0]->nn;
    b->grids.assign(grids, grids + n_rep);
    b->lists.assign(lists, lists + n_rep);
    b->xyzq.assign(xyzq_now, xyzq_now + n_rep);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || ncu < 1) ncu = 1;
    b->ncu = ncu;
    int rc = batch_refresh(b, xyzq_now, f, true);
    if (rc != NB_OK) {
        nb_batch_free(b);
        return rc;
    }
    *out = b;
    return NB_OK;
}

void nb_batch_free(nb_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    DevBuf *bufs[] = {&b->desc, &b->slot_off, &b->atom_off, &b->item_off, &b->partials,
                      &b->gjobs, &b->ljobs, &b->goff,     &b->loff,     &b->scans};
    for (DevBuf *d : bufs) release(*d);
    delete b;
}

int nb_batch_set_group(nb_batch *b, int waves) {
    if (!b || (waves != 1 && waves != 2 && waves != 4 && waves != 8))
        return fail(NB_ERR_ARG, "nb_batch_set_group: work items per workgroup must be 1, 2, 4 or 8");
    if (b->graph_exec) return fail(NB_ERR_STATE, "nb_batch_set_group: batch already captured");
    b->waves = waves;
    return NB_OK;
}

int nb_batch_set_grid(nb_batch *b, long waves) {
    if (!b || waves < 0 || waves > (1L << 28))
        return fail(NB_ERR_ARG, "nb_batch_set_grid: null batch or wavefront count outside [0, 2^28]");
    if (b->graph_exec) return fail(NB_ERR_STATE, "nb_batch_set_grid: batch already captured");
    b->grid_waves = waves;
    return NB_OK;
}

static int batch_check(nb_ctx *c, nb_batch *b, const nb_params *p, unsigned flags, double *energy, double *virial) {
    if (!c || !b || !p || !p->c6c12) return fail(NB_ERR_ARG, "nb_batch: null argument");
    if (b->ctx != c) return fail(NB_ERR_STATE, "nb_batch: batch belongs to another context");
    if (flags & ~(unsigned)(NB_ENERGY | NB_VIRIAL | NB_ACCUMULATE))
        return fail(NB_ERR_ARG, "nb_batch: supported flags are NB_ENERGY, NB_VIRIAL, NB_ACCUMULATE");
    if ((flags & NB_ENERGY) && !energy) return fail(NB_ERR_ARG, "nb_batch: energy output is null");
    if ((flags & NB_VIRIAL) && !virial) return fail(NB_ERR_ARG, "nb_batch: virial output is null");
    if (p->ntypes < 1 || p->ntypes > kMaxTypes || !(p->rc > 0.0f) || !(p->beta >= 0.0f))
        return fail(NB_ERR_ARG, "nb_batch: bad interaction parameters");
    for (int r = 0; r < b->n_rep; ++r)
        if (!(p->rc <= b->lists[r]->rlist)) return fail(NB_ERR_ARG, "nb_batch: rc exceeds a replica's rlist");
    if (p->coulomb < NB_COULOMB_EWALD || p->coulomb > NB_COULOMB_EWALD_TABLE)
        return fail(NB_ERR_ARG, "nb_batch: unknown coulomb type");
    if (p->coulomb == NB_COULOMB_RF && !(p->eps_rf == 0.0f || (p->eps_rf >= 1.0f && std::isfinite(p->eps_rf))))
        return fail(NB_ERR_ARG, "nb_batch: eps_rf must be >= 1, or 0 for a conducting boundary");
    if (p->coulomb != NB_COULOMB_RF && (double)p->beta * p->rc > 4.0)
        return fail(NB_ERR_UNSUPPORTED, "nb_batch: beta*rc > 4 is outside the fitted Ewald range");
    if (p->coulomb == NB_COULOMB_EWALD_TABLE && p->rc > kMaxTableRc)
        return fail(NB_ERR_UNSUPPORTED, "nb_batch: the Ewald table (LDS) covers rc <= 4 nm");
    return NB_OK;
}

int nb_batch_forces(nb_ctx *c, nb_batch *b, const nb_params *p, unsigned flags, double *energy, double *virial) {
    CHECK(batch_check(c, b, p, flags, energy, virial));
    MXN_HIP(hipSetDevice(c->device));
    CHECK(batch_refresh(b, nullptr, nullptr, false));
    return launch_batch(c, b, p, flags, energy, virial);
}

int nb_batch_capture(nb_ctx *c, nb_batch *b, const nb_params *p, unsigned flags, double *energy, double *virial) {
    CHECK(batch_check(c, b, p, flags, energy, virial));
    MXN_HIP(hipSetDevice(c->device));
    if (b->graph_exec) {
        (void)hipGraphExecDestroy(b->graph_exec);
        b->graph_exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    CHECK(batch_refresh(b, nullptr, nullptr, false));
    CHECK(prepare_coulomb(c, p));
    if (!b->capture_stream) MXN_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
    MXN_HIP(hipStreamSynchronize(c->stream));
    hipStream_t saved = c->stream;
    const int timing = c->timing;
    c->stream = b->capture_stream;
    c->timing = 0;
    hipError_t e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? launch_batch(c, b, p, flags, energy, virial) : NB_ERR_HIP;
    b->cycle = false;
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
    c->stream = saved;
    c->timing = timing;
    if (e != hipSuccess || e2 != hipSuccess || rc != NB_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc != NB_OK ? rc : fail(NB_ERR_HIP, std::string("nb_batch_capture: ") +
                                                       hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    e = hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        b->graph_exec = nullptr;
        return fail(NB_ERR_HIP, std::string("nb_batch_capture: instantiate: ") + hipGetErrorString(e));
    }
    return NB_OK;
}

static int rebuild_refresh(nb_batch *b);

int nb_batch_replay(nb_ctx *c, nb_batch *b) {
    if (!c || !b) return fail(NB_ERR_ARG, "nb_batch_replay: null argument");
    if (b->ctx != c) return fail(NB_ERR_STATE, "nb_batch_replay: batch belongs to another context");
    if (!b->graph_exec) return fail(NB_ERR_STATE, "nb_batch_replay: nothing captured");
    MXN_HIP(hipSetDevice(c->device));
    CHECK(batch_refresh(b, nullptr, nullptr, false));
    if (b->cycle) CHECK(rebuild_refresh(b));
    ScopedTimer tm(c, NB_TIMER_FORCE_CALL);
    MXN_HIP(hipGraphLaunch(b->graph_exec, c->stream));
    return NB_OK;
}

int nb_batch_bind_topology(nb_batch *b, const int *const *type, const int *const *excl_off,
                           const int *const *excl_idx) {
    if (!b || !type || !excl_off || !excl_idx) return fail(NB_ERR_ARG, "nb_batch_bind_topology: null argument");
    for (int r = 0; r < b->n_rep; ++r)
        if (!type[r] || !excl_off[r] || !excl_idx[r]) return fail(NB_ERR_ARG, "nb_batch_bind_topology: null replica");
    if (b->graph_exec) return fail(NB_ERR_STATE, "nb_batch_bind_topology: batch already captured");
    b->type.assign(type, type + b->n_rep);
    b->excl_off.assign(excl_off, excl_off + b->n_rep);
    b->excl_idx.assign(excl_idx, excl_idx + b->n_rep);
    // In one batched launch the replicas themselves fill the GPU: size every
    // list for one search wavefront per i-cluster, so that its work items
    // hold full runs of entries (several search parts would cut them short).
    nb_ctx *c = b->ctx;
    MXN_HIP(hipSetDevice(c->device));
    const int saved = c->search_parts;
    c->search_parts = 1;
    int rc = NB_OK;
    for (int r = 0; r < b->n_rep && rc == NB_OK; ++r) {
        nb_list *l = b->lists[r];
        if (l->resv_parts != 1 || l->resv_nci != b->grids[r]->slots_cap / b->grids[r]->m)
            rc = launch_pairlist(l, excl_off[r], excl_idx[r], true, false);
    }
    c->search_parts = saved;
    CHECK(rc);
    b->topology = true;
    return NB_OK;
}

// Job tables and per-stage workgroup offsets of the batched rebuild; uploaded
// (synchronously) only when a replica's storage changed.
static int rebuild_refresh(nb_batch *b) {
    if (!b->topology) return fail(NB_ERR_STATE, "nb_batch_rebuild: bind the replicas' topology first");
    const int n = b->n_rep;
    const size_t gs = grid_job_size(), ls = list_job_size();
    const int GS = grid_job_stages(), LS = list_job_stages();
    std::vector<char> gj(gs * n), lj(ls * n);
    std::vector<ScanJob> sj(2 * n);   // item offsets, then j-cluster view offsets
    std::vector<int> goff(GS * (n + 1)), loff(LS * (n + 1)), gtot(GS, 0), ltot(LS, 0), gb(GS), lb(LS);
    int max_ncol = 1;
    for (int r = 0; r < n; ++r) {
        nb_grid *g = b->grids[r];
        nb_list *l = b->lists[r];
        if (!grid_batchable(g)) return fail(NB_ERR_UNSUPPORTED, "nb_batch_rebuild: a replica's grid has too many columns");
        if (l->resv_parts == 0 || l->resv_nci != g->slots_cap / g->m || l->grid != g)
            return fail(NB_ERR_STATE, "nb_batch_rebuild: every replica's list needs a synchronous build on its grid");
        fill_grid_job(gj.data() + gs * r, g, b->xyzq[r], b->type[r]);
        fill_list_job(lj.data() + ls * r, l, b->excl_off[r], b->excl_idx[r], &sj[r], &sj[n + r]);
        grid_job_blocks(g, gb.data());
        list_job_blocks(l, lb.data());
        for (int k = 0; k < GS; ++k) {
            goff[k * (n + 1) + r] = gtot[k];
            gtot[k] += gb[k];
        }
        for (int k = 0; k < LS; ++k) {
            loff[k * (n + 1) + r] = ltot[k];
            ltot[k] += lb[k];
        }
        max_ncol = std::max(max_ncol, g->ncol);
    }
    for (int k = 0; k < GS; ++k) goff[k * (n + 1) + n] = gtot[k];
    for (int k = 0; k < LS; ++k) loff[k * (n + 1) + n] = ltot[k];
    if (gj == b->gjobs_host && lj == b->ljobs_host && gtot == b->gtotal && ltot == b->ltotal) return NB_OK;
    if (b->graph_exec) return fail(NB_ERR_STATE, "nb_batch: replica storage changed since capture: capture again");
    CHECK(ensure(b->ctx, b->gjobs, gj.size()));
    CHECK(ensure(b->ctx, b->ljobs, lj.size()));
    CHECK(ensure(b->ctx, b->goff, goff.size() * sizeof(int)));
    CHECK(ensure(b->ctx, b->loff, loff.size() * sizeof(int)));
    CHECK(ensure(b->ctx, b->scans, sj.size() * sizeof(ScanJob)));
    MXN_HIP(hipMemcpy(b->gjobs.p, gj.data(), gj.size(), hipMemcpyHostToDevice));
    MXN_HIP(hipMemcpy(b->ljobs.p, lj.data(), lj.size(), hipMemcpyHostToDevice));
    MXN_HIP(hipMemcpy(b->goff.p, goff.data(), goff.size() * sizeof(int), hipMemcpyHostToDevice));
    MXN_HIP(hipMemcpy(b->loff.p, loff.data(), loff.size() * sizeof(int), hipMemcpyHostToDevice));
    MXN_HIP(hipMemcpy(b->scans.p, sj.data(), sj.size() * sizeof(ScanJob), hipMemcpyHostToDevice));
    b->gjobs_host = gj;
    b->ljobs_host = lj;
    b->gtotal = gtot;
    b->ltotal = ltot;
    b->max_ncol = max_ncol;
    return NB_OK;
}

static int launch_rebuild(nb_ctx *c, nb_batch *b) {
    {
        ScopedTimer tm(c, NB_TIMER_GRID_SORT);
        CHECK(launch_grid_sort_batch(c->stream, b->gjobs.p, (const int *)b->goff.p, b->n_rep, b->gtotal.data(),
                                     b->max_ncol));
    }
    {
        ScopedTimer tm(c, NB_TIMER_PAIRLIST);
        CHECK(launch_pairlist_batch(c->stream, b->m, b->nn, b->ljobs.p, (const int *)b->loff.p, b->n_rep,
                                    b->ltotal.data(), (const ScanJob *)b->scans.p));
    }
    for (int r = 0; r < b->n_rep; ++r) {   // every replica's grid and list are now one generation newer
        ++b->grids[r]->generation;
        b->lists[r]->grid_generation = b->grids[r]->generation;
        b->lists[r]->sci_valid = false;
    }
    return NB_OK;
}

int nb_batch_rebuild(nb_ctx *c, nb_batch *b) {
    if (!c || !b) return fail(NB_ERR_ARG, "nb_batch_rebuild: null argument");
    if (b->ctx != c) return fail(NB_ERR_STATE, "nb_batch_rebuild: batch belongs to another context");
    MXN_HIP(hipSetDevice(c->device));
    CHECK(rebuild_refresh(b));
    return launch_rebuild(c, b);
}

// ------------------------------------------------------------- autotuner

// Times the batched force launch of the replicas for every (shape, work
// items per workgroup) candidate: each shape gets its own grids and lists
// (bound to one batch with the search unsplit, as in a batched cycle), each
// group two untimed launches and `reps` launches between HIP events on the
// context's stream.  Everything is freed again before returning.
int nb_autotune(nb_ctx *c, const nb_replicas *r, float rlist, const nb_params *p, unsigned flags,
                const nb_shape *shapes, int n_shapes, const int *groups, int n_groups, int reps, nb_shape *best,
                int *best_group, float *ms_table) {
    if (!c || !r || !p || !shapes || !groups || !best || !best_group) return fail(NB_ERR_ARG, "nb_autotune: null argument");
    if (r->n_rep < 1 || !r->box || !r->n || !r->xyzq || !r->type || !r->excl_off || !r->excl_idx)
        return fail(NB_ERR_ARG, "nb_autotune: incomplete replica description");
    if (n_shapes < 1 || n_groups < 1 || reps < 1) return fail(NB_ERR_ARG, "nb_autotune: need candidates and reps >= 1");
    if (flags & ~(unsigned)(NB_ENERGY | NB_VIRIAL)) return fail(NB_ERR_ARG, "nb_autotune: flags: NB_ENERGY, NB_VIRIAL");
    MXN_HIP(hipSetDevice(c->device));
    const int nr = r->n_rep;
    long atoms = 0;
    for (int k = 0; k < nr; ++k) {
        if (r->n[k] < 1 || !r->xyzq[k] || !r->type[k] || !r->excl_off[k] || !r->excl_idx[k])
            return fail(NB_ERR_ARG, "nb_autotune: bad replica " + std::to_string(k));
        atoms += r->n[k];
    }
    DevBuf fbuf, ebuf;
    int rc = ensure(c, fbuf, (size_t)atoms * 3 * sizeof(float));
    rc = rc ? rc : ensure(c, ebuf, (size_t)nr * 11 * sizeof(double));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (rc == NB_OK && (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess))
        rc = fail(NB_ERR_HIP, "nb_autotune: event creation");
    std::vector<float *> fptr(nr);
    for (long k = 0, off = 0; k < nr; off += 3L * r->n[k], ++k) fptr[k] = (float *)fbuf.p + off;
    double *energy = (double *)ebuf.p, *virial = energy + 2 * nr;
    float best_ms = INFINITY;
    for (int si = 0; si < n_shapes && rc == NB_OK; ++si) {
        std::vector<nb_grid *> gr(nr, nullptr);
        std::vector<nb_list *> li(nr, nullptr);
        nb_batch *b = nullptr;
        for (int k = 0; k < nr && rc == NB_OK; ++k) {
            rc = nb_grid_sort(c, r->box + 3 * k, r->n[k], r->xyzq[k], r->type[k], shapes[si], &gr[k]);
            rc = rc ? rc : nb_pairlist_build(c, gr[k], rlist, -1.0f, r->excl_off[k], r->excl_idx[k], 0, &li[k]);
        }
        rc = rc ? rc : nb_batch_create(c, nr, gr.data(), li.data(), r->xyzq, fptr.data(), &b);
        rc = rc ? rc : nb_batch_bind_topology(b, r->type, r->excl_off, r->excl_idx);
        for (int gi = 0; gi < n_groups && rc == NB_OK; ++gi) {
            rc = nb_batch_set_group(b, groups[gi]);
            for (int w = 0; w < 2 && rc == NB_OK; ++w) rc = nb_batch_forces(c, b, p, flags, energy, virial);
            if (rc == NB_OK && hipEventRecord(ev0, c->stream) != hipSuccess) rc = fail(NB_ERR_HIP, "nb_autotune: event");
            for (int w = 0; w < reps && rc == NB_OK; ++w) rc = nb_batch_forces(c, b, p, flags, energy, virial);
            if (rc == NB_OK && hipEventRecord(ev1, c->stream) != hipSuccess) rc = fail(NB_ERR_HIP, "nb_autotune: event");
            rc = rc ? rc : nb_sync(c);
            float ms = 0.0f;
            if (rc == NB_OK && hipEventElapsedTime(&ms, ev0, ev1) != hipSuccess) rc = fail(NB_ERR_HIP, "nb_autotune: timing");
            if (rc == NB_OK) {
                ms /= (float)reps;
                if (ms_table) ms_table[si * n_groups + gi] = ms;
                if (ms < best_ms) {
                    best_ms = ms;
                    *best = shapes[si];
                    *best_group = groups[gi];
                }
            }
        }
        if (b) nb_batch_free(b);
        for (int k = 0; k < nr; ++k) {
            if (li[k]) nb_list_free(li[k]);
            if (gr[k]) nb_grid_free(gr[k]);
        }
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    (void)hipStreamSynchronize(c->stream);
    release(fbuf);
    release(ebuf);
    return rc;
}

int nb_batch_capture_cycle(nb_ctx *c, nb_batch *b, int nsteps, const nb_params *p, unsigned flags, double *energy,
                           double *virial) {
    if (nsteps < 0) return fail(NB_ERR_ARG, "nb_batch_capture_cycle: nsteps must be >= 0");
    CHECK(batch_check(c, b, p, flags, energy, virial));
    MXN_HIP(hipSetDevice(c->device));
    if (b->graph_exec) {
        (void)hipGraphExecDestroy(b->graph_exec);
        b->graph_exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    CHECK(rebuild_refresh(b));
    CHECK(batch_refresh(b, nullptr, nullptr, false));
    CHECK(prepare_coulomb(c, p));
    if (!b->capture_stream) MXN_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
    MXN_HIP(hipStreamSynchronize(c->stream));
    hipStream_t saved = c->stream;
    const int timing = c->timing;
    c->stream = b->capture_stream;
    c->timing = 0;
    hipError_t e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? launch_rebuild(c, b) : NB_ERR_HIP;
    b->cycle = true;
    for (int r = 0; r < b->n_rep; ++r) b->lists[r]->sci_volatile = true;   // graph replays rebuild these lists
    for (int k = 0; k < nsteps && rc == NB_OK; ++k) rc = launch_batch(c, b, p, flags, energy, virial);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
    c->stream = saved;
    c->timing = timing;
    if (e != hipSuccess || e2 != hipSuccess || rc != NB_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc != NB_OK ? rc : fail(NB_ERR_HIP, std::string("nb_batch_capture_cycle: ") +
                                                       hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    e = hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        b->graph_exec = nullptr;
        return fail(NB_ERR_HIP, std::string("nb_batch_capture_cycle: instantiate: ") + hipGetErrorString(e));
    }
    return NB_OK;
}

// ---------------------------------------------------------------- recount

int nb_recount(nb_ctx *c, const nb_grid *g, const nb_list *l, const float *xyzq_t, const nb_params *p, float c_bb,
               float db, int nbins, double *hist) {
    if (!c || !g || !l || !xyzq_t || !p || !hist || !p->c6c12) return fail(NB_ERR_ARG, "nb_recount: null argument");
    if (g->ctx != c || l->ctx != c || l->grid != g || l->grid_generation != g->generation)
        return fail(NB_ERR_STATE, "nb_recount: grid/list/context mismatch");
    if (nbins < 1 || !(db > 0.0f) || !(c_bb >= 0.0f)) return fail(NB_ERR_ARG, "nb_recount: bad bins");
    if (p->ntypes < 1 || p->ntypes > kMaxTypes || !(p->rc > 0.0f) || !(p->rc <= l->rlist) || !(p->beta >= 0.0f))
        return fail(NB_ERR_ARG, "nb_recount: bad interaction parameters");
    if ((double)p->beta * p->rc > 4.0) return fail(NB_ERR_UNSUPPORTED, "nb_recount: beta*rc > 4");
    if (p->coulomb != NB_COULOMB_EWALD) return fail(NB_ERR_UNSUPPORTED, "nb_recount: Ewald (analytic) only");
    const float want = l->rlist - c_bb > 0.0f ? l->rlist - c_bb : 0.0f;
    if (l->rbb != want) return fail(NB_ERR_ARG, "nb_recount: the list must be built with rbb = rlist - c_bb");
    MXN_HIP(hipSetDevice(c->device));
    return launch_recount(c, g, l, xyzq_t, p, c_bb, db, nbins, hist);
}

// -------------------------------------------------------------------- MLP

int nb_mlp_create(nb_ctx *c, const float *params, const double lo[8], const double hi[8], nb_mlp **out) {
    if (!c || !params || !lo || !hi || !out) return fail(NB_ERR_ARG, "nb_mlp_create: null argument");
    for (int i = 0; i < 8; ++i)
        if (!(hi[i] > lo[i]) || !std::isfinite(lo[i]) || !std::isfinite(hi[i]))
            return fail(NB_ERR_ARG, "nb_mlp_create: every feature range needs hi > lo");
    MXN_HIP(hipSetDevice(c->device));
    nb_mlp *m = new (std::nothrow) nb_mlp();
    if (!m) return fail(NB_ERR_OOM, "nb_mlp_create: host allocation");
    m->ctx = c;
    float lof[8], hif[8];
    for (int i = 0; i < 8; ++i) {
        m->lo_h[i] = lo[i];
        m->hi_h[i] = hi[i];
        lof[i] = (float)lo[i];
        hif[i] = (float)hi[i];
    }
    int rc = ensure(m->ctx, m->params, kMlpParams * 4);
    rc = rc ? rc : ensure(m->ctx, m->m, kMlpParams * 4);
    rc = rc ? rc : ensure(m->ctx, m->v, kMlpParams * 4);
    rc = rc ? rc : ensure(m->ctx, m->step, 16);
    rc = rc ? rc : ensure(m->ctx, m->lo, 32);
    rc = rc ? rc : ensure(m->ctx, m->hi, 32);
    hipError_t e = hipSuccess;
    if (rc == NB_OK) {
        e = hipMemcpy(m->params.p, params, kMlpParams * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(m->m.p, 0, kMlpParams * 4);
        if (e == hipSuccess) e = hipMemset(m->v.p, 0, kMlpParams * 4);
        if (e == hipSuccess) e = hipMemset(m->step.p, 0, 16);
        if (e == hipSuccess) e = hipMemcpy(m->lo.p, lof, 32, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(m->hi.p, hif, 32, hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = fail(NB_ERR_HIP, std::string("nb_mlp_create: ") + hipGetErrorString(e));
    }
    if (rc != NB_OK) {
        DevBuf *bufs[] = {&m->params, &m->m, &m->v, &m->step, &m->lo, &m->hi};
        for (DevBuf *b : bufs) release(*b);
        delete m;
        return rc;
    }
    *out = m;
    return NB_OK;
}

void nb_mlp_free(nb_mlp *m) {
    if (!m) return;
    (void)hipSetDevice(m->ctx->device);
    (void)hipStreamSynchronize(m->ctx->stream);
    if (m->ctx->mlp == m) m->ctx->mlp = nullptr;
    DevBuf *bufs[] = {&m->params, &m->m, &m->v, &m->step, &m->lo, &m->hi};
    for (DevBuf *b : bufs) release(*b);
    delete m;
}

int nb_mlp_get_params(nb_mlp *m, float *params) {
    if (!m || !params) return fail(NB_ERR_ARG, "nb_mlp_get_params: null argument");
    MXN_HIP(hipSetDevice(m->ctx->device));
    MXN_HIP(hipStreamSynchronize(m->ctx->stream));
    MXN_HIP(hipMemcpy(params, m->params.p, kMlpParams * 4, hipMemcpyDeviceToHost));
    return NB_OK;
}

static int mlp_check(nb_ctx *c, const nb_mlp *m, const float *X, int batch) {
    if (!c || !m || !X) return fail(NB_ERR_ARG, "nb_mlp: null argument");
    if (m->ctx != c) return fail(NB_ERR_STATE, "nb_mlp: model belongs to another context");
    if (batch < 1) return fail(NB_ERR_ARG, "nb_mlp: batch must be >= 1");
    return NB_OK;
}

int nb_mlp_train_step(nb_ctx *c, nb_mlp *m, const float *X, const float *y, int batch, float lr, float *loss) {
    CHECK(mlp_check(c, m, X, batch));
    if (!y || !(lr > 0.0f)) return fail(NB_ERR_ARG, "nb_mlp_train_step: need targets and lr > 0");
    MXN_HIP(hipSetDevice(c->device));
    return launch_mlp_step(c, m, X, y, batch, lr, loss, nullptr);
}

int nb_mlp_grad(nb_ctx *c, nb_mlp *m, const float *X, const float *y, int batch, float *grad, float *loss) {
    CHECK(mlp_check(c, m, X, batch));
    if (!y || !grad) return fail(NB_ERR_ARG, "nb_mlp_grad: need targets and a gradient buffer");
    MXN_HIP(hipSetDevice(c->device));
    return launch_mlp_step(c, m, X, y, batch, 0.0f, loss, grad);
}

int nb_mlp_infer(nb_ctx *c, const nb_mlp *m, const float *X, int batch, float *y) {
    CHECK(mlp_check(c, m, X, batch));
    if (!y) return fail(NB_ERR_ARG, "nb_mlp_infer: output is null");
    MXN_HIP(hipSetDevice(c->device));
    return launch_mlp_infer(c, m, X, batch, y);
}

int nb_mlp_set_domain(nb_mlp *m, const nb_buffer_query *q) {
    if (!m) return fail(NB_ERR_ARG, "nb_mlp_set_domain: model is null");
    CHECK(validate_query(q));
    if (!(q->target > 0.0)) return fail(NB_ERR_ARG, "nb_mlp_set_domain: target must be > 0");
    m->dom_target = q->target;
    m->dom_dt = q->dt;
    m->dom_brc = q->beta * q->rc;
    m->dom_ntypes = q->ntypes;
    m->dom_charge.assign(q->charge, q->charge + q->ntypes);
    m->dom_c6c12.assign(q->c6c12, q->c6c12 + 2 * q->ntypes * q->ntypes);
    m->has_domain = true;
    return NB_OK;
}

// A query the model may answer: its labels were generated for the same time
// step, Ewald accuracy (beta * rc) and interaction parameters, and for a
// drift target no looser than the query's (a buffer meeting a stricter
// target also meets a looser one).
static bool mlp_domain_ok(const nb_mlp *m, const nb_buffer_query &q) {
    auto close = [](double a, double b, double rel) { return std::fabs(a - b) <= rel * std::fmax(std::fabs(a), std::fabs(b)); };
    if (!m->has_domain) return false;
    if (q.target < m->dom_target * (1.0 - 1e-12)) return false;
    if (!close(q.dt, m->dom_dt, 1e-9) || !close(q.beta * q.rc, m->dom_brc, 5e-3)) return false;
    if (q.ntypes != m->dom_ntypes) return false;
    for (int a = 0; a < q.ntypes; ++a)
        if (!close(q.charge[a], m->dom_charge[a], 1e-9)) return false;
    for (int k = 0; k < 2 * q.ntypes * q.ntypes; ++k)
        if (!close(q.c6c12[k], m->dom_c6c12[k], 1e-9)) return false;
    return true;
}

int nb_buffer_set_mlp(nb_ctx *c, const nb_mlp *m, double margin) {
    if (!c) return fail(NB_ERR_ARG, "nb_buffer_set_mlp: ctx is null");
    if (m && m->ctx != c) return fail(NB_ERR_STATE, "nb_buffer_set_mlp: model belongs to another context");
    if (!(margin >= 0.0)) return fail(NB_ERR_ARG, "nb_buffer_set_mlp: margin must be >= 0");
    c->mlp = m;
    c->mlp_margin = margin;
    return NB_OK;
}

// ------------------------------------------------------------ buffer size

// The predictor's inputs from a query: temperature, mass-weighted
// displacement width sqrt(kB T t^2 <1/m>) over t = (nstlist-1) dt, list
// lifetime in steps, mass density (g/cm^3), cut-off, cluster shape one-hot.
static bool buffer_features(const nb_buffer_query &q, float f[8]) {
    double n = 0.0, inv_m = 0.0, mass = 0.0;
    for (int a = 0; a < q.ntypes; ++a) {
        n += q.count[a];
        inv_m += q.count[a] / q.mass[a];
        mass += q.count[a] * q.mass[a];
    }
    if (!(n > 0.0)) return false;
    const double t = (q.nstlist - 1) * q.dt;
    f[0] = (float)q.T;
    f[1] = (float)std::sqrt(0.0083144626 * q.T * t * t * inv_m / n);
    f[2] = (float)q.nstlist;
    f[3] = (float)(mass / (q.volume * 602.214076));
    f[4] = (float)q.rc;
    const int s = q.shape.m == 4 && q.shape.n == 4 ? 0 : (q.shape.m == 4 && q.shape.n == 8 ? 1 : (q.shape.m == 8 && q.shape.n == 8 ? 2 : -1));
    if (s < 0) return false;
    f[5] = s == 0; f[6] = s == 1; f[7] = s == 2;
    return true;
}

int nb_buffer_estimate(nb_ctx *c, const nb_buffer_query *q, int mode, double *rb_out, double *drift_out,
                       int *used_fallback) {
    CHECK(validate_query(q));
    if (!rb_out) return fail(NB_ERR_ARG, "nb_buffer_estimate: rb_out is null");
    if (mode != NB_BUFFER_ANALYTIC && mode != NB_BUFFER_MLP && mode != NB_BUFFER_AUTO)
        return fail(NB_ERR_ARG, "nb_buffer_estimate: unknown mode");
    double rb_a = 0.0, d_a = 0.0;
    CHECK(analytic_buffer(*q, &rb_a, &d_a));
    int fb = mode != NB_BUFFER_ANALYTIC;
    double rb = rb_a;
    if (mode != NB_BUFFER_ANALYTIC) {
        if (!c) return fail(NB_ERR_ARG, "nb_buffer_estimate: the learned modes need a context");
        if (!c->mlp && mode == NB_BUFFER_MLP) return fail(NB_ERR_STATE, "nb_buffer_estimate: no model attached");
        float f[8];
        bool in_range = c->mlp && mlp_domain_ok(c->mlp, *q) && buffer_features(*q, f);
        if (in_range)
            for (int i = 0; i < 5; ++i)
                if (!(f[i] >= c->mlp->lo_h[i] && f[i] <= c->mlp->hi_h[i])) in_range = false;   // outside training data
        if (in_range) {
            MXN_HIP(hipSetDevice(c->device));
            CHECK(ensure(c, c->mlp_io, 64));
            float y = NAN;
            MXN_HIP(hipMemcpyAsync(c->mlp_io.p, f, sizeof f, hipMemcpyHostToDevice, c->stream));
            CHECK(launch_mlp_infer(c, c->mlp, (const float *)c->mlp_io.p, 1, (float *)c->mlp_io.p + 8));
            MXN_HIP(hipMemcpyAsync(&y, (float *)c->mlp_io.p + 8, sizeof y, hipMemcpyDeviceToHost, c->stream));
            MXN_HIP(hipStreamSynchronize(c->stream));
            if (std::isfinite(y) && y >= 0.0f) {
                rb = std::fmin((double)y + c->mlp_margin, rb_a);
                fb = 0;
            }
        }
    }
    *rb_out = rb;
    if (drift_out) *drift_out = rb == rb_a ? d_a : analytic_drift(*q, rb);
    if (used_fallback) *used_fallback = fb;
    return NB_OK;
}

}  // extern "C"
