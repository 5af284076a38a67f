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
    nb_jentry *entries;   // canonical order (by shift, then j-cluster) within each i-cluster
    float *keys;          // bounding-box distance^2 of each entry
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

// first index k in [lo, hi) with key(k) >= v for a nondecreasing key (hi if none)
template <class F>
__device__ inline int lower_bound(int lo, int hi, F key, float v) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (key(mid) < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Lane layout of the particle-pair checks: lane = g*M*N + b*M + a handles the
// pair (i-slot a, j-slot b) of candidate group g, so P = 64/(M*N) candidates
// are checked per pass and one ballot yields their masks in j-major order.
template <int M, int N, bool FILL>
__global__ __launch_bounds__(256) void k_search(SearchArgs a) {
    constexpr int PAIRS = M * N;
    constexpr int P = 64 / PAIRS;
    constexpr unsigned long long GMASK = PAIRS == 64 ? ~0ull : ((1ull << PAIRS) - 1ull);
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
    const int pa = lane % M, pb = (lane / M) % N, grp = lane / PAIRS;
    const float4 pi = a.xs[ci * M + pa];
    const int iorig = a.perm[ci * M + pa];
    const float zmargin = 1e-3f;   // keeps the z window conservative against rounding
    int cnt = 0;
    if (lo.x <= hi.x) {   // the cluster holds real particles
        for (int s = 13; s < 27; ++s) {
            const float sx = (float)(s / 9 - 1) * a.Lx, sy = (float)((s / 3) % 3 - 1) * a.Ly,
                        sz = (float)(s % 3 - 1) * a.Lz;
            const float slx = lo.x + sx, shx = hi.x + sx, sly = lo.y + sy, shy = hi.y + sy, slz = lo.z + sz,
                        shz = hi.z + sz;
            const float pix = pi.x + sx, piy = pi.y + sy, piz = pi.z + sz;   // this lane's shifted i-particle
            // candidate columns: a superset, one column of margin against rounding
            int cx0 = (int)floorf((slx - a.rlist) * a.inv_x) - 1, cx1 = (int)floorf((shx + a.rlist) * a.inv_x) + 1;
            int cy0 = (int)floorf((sly - a.rlist) * a.inv_y) - 1, cy1 = (int)floorf((shy + a.rlist) * a.inv_y) + 1;
            cx0 = cx0 < 0 ? 0 : cx0; cy0 = cy0 < 0 ? 0 : cy0;
            cx1 = cx1 > a.nx - 1 ? a.nx - 1 : cx1; cy1 = cy1 > a.ny - 1 ? a.ny - 1 : cy1;
            if (cx0 > cx1 || cy0 > cy1) continue;
            const int ncy = cy1 - cy0 + 1, ncols = (cx1 - cx0 + 1) * ncy;
            for (int cb = 0; cb < ncols; cb += 64) {
                // one column per lane (ascending column id): its z window of j-clusters
                int k0 = 0, kc = 0;
                const int cidx = cb + lane;
                if (cidx < ncols) {
                    const int c = (cx0 + cidx / ncy) * a.ny + cy0 + cidx % ncy;
                    const float4 cbb = a.colbb[c];
                    const float gx = axis_gap(cbb.x, cbb.z, slx, shx), gy = axis_gap(cbb.y, cbb.w, sly, shy);
                    if (gx * gx + gy * gy < a.rl2) {
                        const int j0 = a.col_start[c] / N, j1 = a.col_start[c + 1] / N;
                        const float4 *blo = a.bbj_lo, *bhi = a.bbj_hi;
                        k0 = lower_bound(j0, j1, [&](int k) { return bhi[k].z; }, slz - a.rlist - zmargin);
                        const int k1 = lower_bound(k0, j1, [&](int k) { return blo[k].z; }, shz + a.rlist + zmargin);
                        kc = k1 - k0;
                    }
                }
                // flatten the windows of the 64 columns: exclusive offsets by a wave scan
                int incl = kc;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int v = __shfl_up(incl, o, 64);
                    if (lane >= o) incl += v;
                }
                const int total = __shfl(incl, 63, 64);
                const int excl = incl - kc;
                for (int t0 = 0; t0 < total; t0 += 64) {
                    const int t = t0 + lane;
                    bool ok = t < total;
                    // owner column: the last lane whose exclusive offset is <= t (fixed six-step search,
                    // executed by every lane so that all shuffles read active lanes)
                    const int tt = ok ? t : total - 1;
                    int own = 0;
#pragma unroll
                    for (int step = 32; step > 0; step >>= 1) {
                        const int cand = own + step;
                        const int ev = __shfl(excl, cand < 64 ? cand : 63, 64);
                        if (cand < 64 && ev <= tt) own = cand;
                    }
                    const int cj = __shfl(k0, own, 64) + (tt - __shfl(excl, own, 64));
                    if (ok && s == 13) ok = cj * N + N - 1 > ci * M;
                    float d2 = 0.0f;
                    if (ok) {
                        const float4 jl = a.bbj_lo[cj], jh = a.bbj_hi[cj];
                        d2 = sq3(axis_gap(jl.x, jh.x, slx, shx), axis_gap(jl.y, jh.y, sly, shy),
                                 axis_gap(jl.z, jh.z, slz, shz));
                        ok = d2 < a.rl2;
                    }
                    const bool chk = ok && !(d2 < a.rb2);
                    unsigned long long accepted = __ballot(ok && !chk);
                    unsigned long long need = __ballot(chk);
                    // particle-pair checks, P candidates per pass
                    while (need) {
                        int src = -1;
#pragma unroll
                        for (int g = 0; g < P; ++g) {
                            const int f = need ? __ffsll((long long)need) - 1 : -1;
                            if (f >= 0) need &= need - 1;
                            if (g == grp) src = f;
                        }
                        bool hit = false;
                        const int cjc = __shfl(cj, src < 0 ? 0 : src, 64);
                        if (src >= 0 && iorig >= 0) {
                            const int sb = cjc * N + pb;
                            if (a.perm[sb] >= 0) {
                                const float4 pbv = a.xs[sb];
                                hit = sq3(pix - pbv.x, piy - pbv.y, piz - pbv.z) < a.rl2;
                            }
                        }
                        const unsigned long long hb = __ballot(hit);
#pragma unroll
                        for (int g = 0; g < P; ++g) {
                            const int sg = __shfl(src, g * PAIRS, 64);
                            if (sg >= 0 && ((hb >> (g * PAIRS)) & GMASK)) accepted |= 1ull << sg;
                        }
                    }
                    if (FILL) {
                        // masks of the accepted candidates, in lane (= candidate) order
                        unsigned long long todo = accepted;
                        int base = wpos;
                        while (todo) {
                            int src = -1, rank = 0;
#pragma unroll
                            for (int g = 0; g < P; ++g) {
                                const int f = todo ? __ffsll((long long)todo) - 1 : -1;
                                if (f >= 0) todo &= todo - 1;
                                if (g == grp) src = f;
                            }
                            if (src >= 0) rank = __popcll(accepted & ((1ull << src) - 1ull));
                            const int cjc = __shfl(cj, src < 0 ? 0 : src, 64);
                            const float d2c = __shfl(d2, src < 0 ? 0 : src, 64);
                            bool bit = false;
                            if (src >= 0 && iorig >= 0) {
                                const int sb = cjc * N + pb;
                                const int jorig = a.perm[sb];
                                if (jorig >= 0 && !(s == 13 && ci * M + pa >= sb)) {
                                    bit = true;
                                    bool excluded = false;
                                    for (int e = a.excl_off[iorig]; e < a.excl_off[iorig + 1]; ++e)
                                        excluded |= a.excl_idx[e] == jorig;
                                    if (excluded) {
                                        const float4 pbv = a.xs[sb];
                                        if (sq3(pix - pbv.x, piy - pbv.y, piz - pbv.z) < a.rl2) bit = false;
                                    }
                                }
                            }
                            const unsigned long long mb = __ballot(bit);
                            if (src >= 0 && lane % PAIRS == 0) {
                                const unsigned long long mask = PAIRS == 64 ? mb : ((mb >> (grp * PAIRS)) & GMASK);
                                nb_jentry en;
                                en.cj = cjc;
                                en.shift = s;
                                en.mlo = (uint32_t)mask;
                                en.mhi = (uint32_t)(mask >> 32);
                                a.entries[base + rank] = en;
                                a.keys[base + rank] = d2c;
                            }
                        }
                        wpos += __popcll(accepted);
                    } else {
                        cnt += __popcll(accepted);
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

// Order the entries of each i-cluster by bounding-box distance (ties by
// canonical position), so that the far entries, whose pairs mostly lie beyond
// the cut-off, share force-kernel passes whose pair work can be skipped.
// One wavefront per i-cluster, rank sort with the keys staged in LDS.
__global__ __launch_bounds__(64) void k_sort_entries(const int *ci_start, const int *totals, long cap_entries,
                                                     long cap_items, const nb_jentry *in, const float *keys,
                                                     nb_jentry *out) {
    __shared__ float sk[1024];
    if ((long)totals[0] > cap_entries || (long)totals[1] > cap_items) return;
    const int ci = blockIdx.x, lane = threadIdx.x;
    const int b = ci_start[ci], n = ci_start[ci + 1] - b;
    const bool staged = n <= 1024;
    if (staged)
        for (int i = lane; i < n; i += 64) sk[i] = keys[b + i];
    __syncthreads();
    for (int i = lane; i < n; i += 64) {
        const float ki = staged ? sk[i] : keys[b + i];
        int r = 0;
        for (int j = 0; j < n; ++j) {
            const float kj = staged ? sk[j] : keys[b + j];
            r += (kj < ki) || (kj == ki && j < i);
        }
        out[b + r] = in[b + i];
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

int launch_pairlist(nb_list *l, const int *excl_off, const int *excl_idx, bool sync, bool by_distance) {
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
            rc = ensure(l->entries_canon, (size_t)ce * sizeof(nb_jentry));
            if (rc) return rc;
            rc = ensure(l->keys, (size_t)ce * sizeof(float));
            if (rc) return rc;
            rc = ensure(l->items, (size_t)cit * sizeof(int4));
            if (rc) return rc;
            l->cap_entries = ce;
            l->cap_items = cit;
        }
        l->last_entries = ne;
    }
    a.entries = (nb_jentry *)(by_distance ? l->entries_canon.p : l->entries.p);
    a.keys = (float *)l->keys.p;
    a.items = (int4 *)l->items.p;
    a.cap_entries = l->cap_entries;
    a.cap_items = l->cap_items;
    if (g->m == 4 && g->nn == 4) run<4, 4>(l, a, true, nblocks, st);
    else if (g->m == 4 && g->nn == 8) run<4, 8>(l, a, true, nblocks, st);
    else run<8, 8>(l, a, true, nblocks, st);
    if (by_distance)
        k_sort_entries<<<nci_cap, 64, 0, st>>>((const int *)l->ci_start.p, (const int *)l->totals.p, l->cap_entries,
                                           l->cap_items, (const nb_jentry *)l->entries_canon.p, (const float *)l->keys.p,
                                           (nb_jentry *)l->entries.p);
    k_finalize<<<1, 64, 0, st>>>((int *)l->totals.p, l->cap_entries, l->cap_items, ctx->d_flags);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

}  // namespace mxn
