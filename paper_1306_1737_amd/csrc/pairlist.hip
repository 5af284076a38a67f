// Cluster-pair search (Sec. 2.3 "Pair list construction", the cluster-pair
// search pseudocode, and Sec. 2.4 "Exclusion treatment"), run entirely on the
// GPU as the paper planned.  One wavefront per i-cluster: for each kept image
// shift it walks the candidate grid columns in increasing column order and
// tests that column's j-clusters 64 at a time (one per lane) against the
// bounding-box criterion, falling back to the particle-pair check outside the
// rBB shortcut.  A count pass, a deterministic scan and a fill pass give a
// list whose order depends only on the input.
//
// Compiled with -ffp-contract=off: the inclusion predicate and the
// exclusion-in-image test are defined by separately rounded FP32 operations.
#include "internal.h"

namespace mxn {
void launch_scan_mode(const int *in, int *out, int n, int mode, int p, int *total, hipStream_t s);
}

namespace {

struct SearchArgs {
    const int *nslots;
    const float4 *xs;
    const int *perm, *slot_of;
    const float4 *bbi_lo, *bbi_hi, *bbj_lo, *bbj_hi, *colbb;
    const int *col_start;
    const int *excl_off, *excl_idx;
    float Lx, Ly, Lz, inv_x, inv_y;
    int nx, ny;
    float rlist, rl2, rb2;
    int *ci_count;
    const int *ci_start, *ci_istart, *totals;
    nb_jentry *entries;
    int4 *items;
    long cap_entries, cap_items;
    int nci_cap;
};

__device__ inline float sq3(float x, float y, float z) { return (x * x + y * y) + z * z; }

__device__ inline float axis_gap(float jlo, float jhi, float ilo, float ihi) {
    float d1 = jlo - ihi, d2 = ilo - jhi;
    float m = d1 > d2 ? d1 : d2;
    return m > 0.0f ? m : 0.0f;
}

template <int M, int N, bool FILL>
__global__ __launch_bounds__(256) void k_search(SearchArgs a) {
    const int lane = threadIdx.x & 63;
    const int ci = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ci >= a.nci_cap) return;
    const int nci = *a.nslots / M;
    if (ci >= nci) {   // beyond the padded slot count of this sort: contributes nothing to the scans
        if (!FILL && lane == 0) a.ci_count[ci] = 0;
        return;
    }
    int wpos = 0, ipos = 0;
    if (FILL) {
        if ((long)a.totals[0] > a.cap_entries || (long)a.totals[1] > a.cap_items) return;   // overflow: latched later
        wpos = a.ci_start[ci];
        ipos = a.ci_istart[ci];
    }
    const float4 lo = a.bbi_lo[ci], hi = a.bbi_hi[ci];
    float ix[M], iy[M], iz[M];
    int iorig[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        float4 p = a.xs[ci * M + k];
        ix[k] = p.x; iy[k] = p.y; iz[k] = p.z;
        iorig[k] = a.perm[ci * M + k];
    }
    int cnt = 0;
    if (lo.x <= hi.x) {   // the cluster holds real particles
        for (int s = 13; s < 27; ++s) {
            const float sx = (float)(s / 9 - 1) * a.Lx, sy = (float)((s / 3) % 3 - 1) * a.Ly,
                        sz = (float)(s % 3 - 1) * a.Lz;
            const float slx = lo.x + sx, shx = hi.x + sx, sly = lo.y + sy, shy = hi.y + sy, slz = lo.z + sz,
                        shz = hi.z + sz;
            float six[M], siy[M], siz[M];
#pragma unroll
            for (int k = 0; k < M; ++k) { six[k] = ix[k] + sx; siy[k] = iy[k] + sy; siz[k] = iz[k] + sz; }
            // candidate columns: a superset, one column of margin against rounding
            int cx0 = (int)floorf((slx - a.rlist) * a.inv_x) - 1, cx1 = (int)floorf((shx + a.rlist) * a.inv_x) + 1;
            int cy0 = (int)floorf((sly - a.rlist) * a.inv_y) - 1, cy1 = (int)floorf((shy + a.rlist) * a.inv_y) + 1;
            cx0 = cx0 < 0 ? 0 : cx0; cy0 = cy0 < 0 ? 0 : cy0;
            cx1 = cx1 > a.nx - 1 ? a.nx - 1 : cx1; cy1 = cy1 > a.ny - 1 ? a.ny - 1 : cy1;
            for (int cx = cx0; cx <= cx1; ++cx)
                for (int cy = cy0; cy <= cy1; ++cy) {
                    const int c = cx * a.ny + cy;
                    const float4 cb = a.colbb[c];
                    const float gx = axis_gap(cb.x, cb.z, slx, shx), gy = axis_gap(cb.y, cb.w, sly, shy);
                    if (!(gx * gx + gy * gy < a.rl2)) continue;   // no cluster of this column can pass
                    const int cj0 = a.col_start[c] / N, cj1 = a.col_start[c + 1] / N;
                    for (int base = cj0; base < cj1; base += 64) {
                        const int cj = base + lane;
                        bool ok = cj < cj1;
                        if (ok && s == 13) ok = cj * N + N - 1 > ci * M;
                        float d2 = 0.0f;
                        if (ok) {
                            const float4 jl = a.bbj_lo[cj], jh = a.bbj_hi[cj];
                            d2 = sq3(axis_gap(jl.x, jh.x, slx, shx), axis_gap(jl.y, jh.y, sly, shy),
                                     axis_gap(jl.z, jh.z, slz, shz));
                            ok = d2 < a.rl2;
                        }
                        if (ok && !(d2 < a.rb2)) {
                            bool found = false;
                            for (int b = 0; b < N && !found; ++b) {
                                const int sb = cj * N + b;
                                if (a.perm[sb] < 0) continue;
                                const float4 pb = a.xs[sb];
#pragma unroll
                                for (int k = 0; k < M; ++k)
                                    if (iorig[k] >= 0 && sq3(six[k] - pb.x, siy[k] - pb.y, siz[k] - pb.z) < a.rl2)
                                        found = true;
                            }
                            ok = found;
                        }
                        const unsigned long long ballot = __ballot(ok);
                        if (FILL) {
                            if (ok) {
                                const int idx = wpos + __popcll(ballot & ((1ull << lane) - 1ull));
                                // mask in j-major order: bit b*M + a
                                unsigned long long mask = 0;
                                for (int b = 0; b < N; ++b) {
                                    const int sb = cj * N + b;
                                    if (a.perm[sb] < 0) continue;
#pragma unroll
                                    for (int k = 0; k < M; ++k)
                                        if (iorig[k] >= 0 && !(s == 13 && ci * M + k >= sb))
                                            mask |= 1ull << (b * M + k);
                                }
                                // force-field exclusions in this image (within rlist)
#pragma unroll
                                for (int k = 0; k < M; ++k) {
                                    if (iorig[k] < 0) continue;
                                    for (int e = a.excl_off[iorig[k]]; e < a.excl_off[iorig[k] + 1]; ++e) {
                                        const int ps = a.slot_of[a.excl_idx[e]];
                                        const int b = ps - cj * N;
                                        if (b < 0 || b >= N) continue;
                                        const unsigned long long bit = 1ull << (b * M + k);
                                        if (!(mask & bit)) continue;
                                        const float4 pb = a.xs[ps];
                                        if (sq3(six[k] - pb.x, siy[k] - pb.y, siz[k] - pb.z) < a.rl2) mask &= ~bit;
                                    }
                                }
                                nb_jentry en;
                                en.cj = cj;
                                en.shift = s;
                                en.mlo = (uint32_t)mask;
                                en.mhi = (uint32_t)(mask >> 32);
                                a.entries[idx] = en;
                            }
                            wpos += __popcll(ballot);
                        } else {
                            cnt += __popcll(ballot);
                        }
                    }
                }
        }
    }
    if (!FILL) {
        if (lane == 0) a.ci_count[ci] = cnt;
    } else {
        const int start = a.ci_start[ci], end = a.ci_start[ci + 1];
        const int nit = (end - start + mxn::kItemEntries - 1) / mxn::kItemEntries;
        for (int k = lane; k < nit; k += 64) {
            const int js = start + k * mxn::kItemEntries;
            const int je = js + mxn::kItemEntries < end ? js + mxn::kItemEntries : end;
            a.items[ipos + k] = make_int4(ci, js, je, 0);
        }
    }
}

// totals: [0] entries, [1] items (from the scans); writes [2] = usable item
// count (0 on overflow) and latches the overflow flag
__global__ void k_finalize(int *totals, long cap_entries, long cap_items, int *flags) {
    if (threadIdx.x != 0) return;
    bool over = (long)totals[0] > cap_entries || (long)totals[1] > cap_items;
    totals[2] = over ? 0 : totals[1];
    if (over) atomicOr(flags, mxn::FLAG_OVERFLOW);
}

template <int M, int N>
void run(nb_list *l, SearchArgs &a, bool fill, int nblocks, hipStream_t st) {
    if (fill)
        k_search<M, N, true><<<nblocks, 256, 0, st>>>(a);
    else
        k_search<M, N, false><<<nblocks, 256, 0, st>>>(a);
}

}  // namespace

namespace mxn {

int launch_pairlist(nb_list *l, const int *excl_off, const int *excl_idx, bool sync) {
    const nb_grid *g = l->grid;
    nb_ctx *ctx = l->ctx;
    hipStream_t st = ctx->stream;
    const int nci_cap = g->slots_cap / g->m;
    SearchArgs a{};
    a.nslots = (const int *)g->nslots.p;
    a.xs = (const float4 *)g->xs.p;
    a.perm = (const int *)g->perm.p;
    a.slot_of = (const int *)g->slot_of.p;
    a.bbi_lo = (const float4 *)g->bbi_lo.p;
    a.bbi_hi = (const float4 *)g->bbi_hi.p;
    a.bbj_lo = (const float4 *)(g->nn == g->m ? g->bbi_lo.p : g->bbj_lo.p);
    a.bbj_hi = (const float4 *)(g->nn == g->m ? g->bbi_hi.p : g->bbj_hi.p);
    a.colbb = (const float4 *)g->colbb.p;
    a.col_start = (const int *)g->col_start.p;
    a.excl_off = excl_off;
    a.excl_idx = excl_idx;
    a.Lx = g->Lf[0]; a.Ly = g->Lf[1]; a.Lz = g->Lf[2];
    a.inv_x = g->inv_x; a.inv_y = g->inv_y;
    a.nx = g->nx; a.ny = g->ny;
    a.rlist = l->rlist;
    volatile float rl2 = l->rlist * l->rlist, rb2 = l->rbb * l->rbb;
    a.rl2 = rl2; a.rb2 = rb2;
    a.ci_count = (int *)l->ci_count.p;
    a.ci_start = (const int *)l->ci_start.p;
    a.ci_istart = (const int *)l->ci_istart.p;
    a.totals = (const int *)l->totals.p;
    a.nci_cap = nci_cap;
    const int nblocks = (nci_cap + 3) / 4;
    // count pass
    if (g->m == 4 && g->nn == 4) run<4, 4>(l, a, false, nblocks, st);
    else if (g->m == 4 && g->nn == 8) run<4, 8>(l, a, false, nblocks, st);
    else run<8, 8>(l, a, false, nblocks, st);
    launch_scan_mode((const int *)l->ci_count.p, (int *)l->ci_start.p, nci_cap, 0, 1, (int *)l->totals.p, st);
    launch_scan_mode((const int *)l->ci_count.p, (int *)l->ci_istart.p, nci_cap, 2, kItemEntries,
                     (int *)l->totals.p + 1, st);
    if (sync) {
        MXN_HIP(hipMemcpyAsync(ctx->h_pinned, l->totals.p, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        MXN_HIP(hipStreamSynchronize(st));
        long ne = ctx->h_pinned[0], ni = ctx->h_pinned[1];
        if (ne > l->cap_entries || ni > l->cap_items) {
            long ce = ne + ne / 8 + 1024, cit = ni + ni / 8 + 256;
            int rc = ensure(l->entries, (size_t)ce * sizeof(nb_jentry));
            if (rc) return rc;
            rc = ensure(l->items, (size_t)cit * sizeof(int4));
            if (rc) return rc;
            l->cap_entries = ce;
            l->cap_items = cit;
        }
        l->last_entries = ne;
    }
    a.entries = (nb_jentry *)l->entries.p;
    a.items = (int4 *)l->items.p;
    a.cap_entries = l->cap_entries;
    a.cap_items = l->cap_items;
    if (g->m == 4 && g->nn == 4) run<4, 4>(l, a, true, nblocks, st);
    else if (g->m == 4 && g->nn == 8) run<4, 8>(l, a, true, nblocks, st);
    else run<8, 8>(l, a, true, nblocks, st);
    k_finalize<<<1, 64, 0, st>>>((int *)l->totals.p, l->cap_entries, l->cap_items, ctx->d_flags);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

}  // namespace mxn
