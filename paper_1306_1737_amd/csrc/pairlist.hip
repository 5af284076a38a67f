// Cluster-pair search (Sec. 2.3 "Pair list construction", the cluster-pair
// search pseudocode, and Sec. 2.4 "Exclusion treatment"), run entirely on the
// GPU as the paper planned.  One wavefront per i-cluster: for each kept image
// shift it walks the candidate grid columns in increasing column order and
// tests that column's j-clusters 64 at a time (one per lane) against the
// bounding-box criterion; a lane whose candidate lies outside the rBB
// shortcut checks the candidate's particle pairs itself.  A count pass, a
// deterministic scan and a fill pass give a list whose order depends only on
// the input.
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
    int *part_count;                     // entries found by each (i-cluster, part)
    const int *part_start, *ci_start, *ci_istart, *totals;
    nb_jentry *entries;   // per i-cluster: part by part, each part in (shift, j-cluster) order
    float *keys;          // bounding-box distance^2 of each entry
    int4 *items;
    long cap_entries, cap_items;
    int nci_cap, parts;
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

// Candidates are handled one per lane: a lane owning a candidate j-cluster
// outside the rBB shortcut checks its M x N particle pairs itself (all loads
// independent, early exit on the first pair within rlist), and in the fill
// pass builds the interaction mask of an accepted candidate from the
// particles' realness, the self-pair triangle and the i-cluster's exclusions
// (their partners' slots and positions staged in LDS once per wavefront).
// a.parts wavefronts share an i-cluster: part p takes the p-th contiguous
// share of every image shift's candidate columns.
constexpr int kExclStage = 64;   // staged exclusion partners per wavefront

template <int M, int N, bool FILL>
__global__ __launch_bounds__(256) void k_search(SearchArgs a) {
    constexpr unsigned FULL = (1u << M) - 1u;
    __shared__ float4 xpos[4][kExclStage];
    __shared__ int xinfo[4][kExclStage];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gw = blockIdx.x * 4 + w;
    const int P = a.parts, ci = gw / P, part = gw % P;
    if (ci >= a.nci_cap) return;
    const int nci = *a.nslots / M;
    if (ci >= nci) {   // beyond the padded slot count of this sort: contributes nothing to the scans
        if (!FILL && lane == 0) a.part_count[gw] = 0;
        return;
    }
    int wpos = 0;
    if (FILL) {
        if ((long)a.totals[0] > a.cap_entries || (long)a.totals[1] > a.cap_items) return;   // overflow: latched later
        wpos = a.part_start[gw];
    }
    const float4 lo = a.bbi_lo[ci], hi = a.bbi_hi[ci];
    // the i-cluster (uniform across the wavefront)
    float ix[M], iy[M], iz[M];
    unsigned ireal = 0;
#pragma unroll
    for (int ia = 0; ia < M; ++ia) {
        const float4 p = a.xs[ci * M + ia];
        ix[ia] = p.x; iy[ia] = p.y; iz[ia] = p.z;
        ireal |= (a.perm[ci * M + ia] >= 0 ? 1u : 0u) << ia;
    }
    const float zmargin = 1e-3f;   // keeps the z window conservative against rounding
    const float pmargin = 1e-3f;   // keeps the particle-to-box prefilter conservative
    const float rp2 = (a.rlist + pmargin) * (a.rlist + pmargin);
    // exclusion partners of the i-particles: (slot * 8 + i-index, position), staged in LDS
    int nexcl = 0;
    bool staged = true;
    if (FILL) {
        int e0 = 0, e1 = 0;
        if (lane < M && ((ireal >> lane) & 1u)) {
            const int io = a.perm[ci * M + lane];
            e0 = a.excl_off[io];
            e1 = a.excl_off[io + 1];
        }
        int incl = e1 - e0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        nexcl = __shfl(incl, 63, 64);
        staged = nexcl <= kExclStage && (long)a.nci_cap * M < (1L << 28);   // slot * 8 + i-index fits an int
        if (staged && lane < M) {
            int q = incl - (e1 - e0);
            for (int e = e0; e < e1; ++e, ++q) {
                const int ps = a.slot_of[a.excl_idx[e]];
                xinfo[w][q] = ps * 8 + lane;
                xpos[w][q] = a.xs[ps];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    int cnt = 0;
    if (lo.x <= hi.x) {   // the cluster holds real particles
        for (int s = 13; s < 27; ++s) {
            const float sx = (float)(s / 9 - 1) * a.Lx, sy = (float)((s / 3) % 3 - 1) * a.Ly,
                        sz = (float)(s % 3 - 1) * a.Lz;
            const float slx = lo.x + sx, shx = hi.x + sx, sly = lo.y + sy, shy = hi.y + sy, slz = lo.z + sz,
                        shz = hi.z + sz;
            // candidate columns: a superset, one column of margin against rounding
            int cx0 = (int)floorf((slx - a.rlist) * a.inv_x) - 1, cx1 = (int)floorf((shx + a.rlist) * a.inv_x) + 1;
            int cy0 = (int)floorf((sly - a.rlist) * a.inv_y) - 1, cy1 = (int)floorf((shy + a.rlist) * a.inv_y) + 1;
            cx0 = cx0 < 0 ? 0 : cx0; cy0 = cy0 < 0 ? 0 : cy0;
            cx1 = cx1 > a.nx - 1 ? a.nx - 1 : cx1; cy1 = cy1 > a.ny - 1 ? a.ny - 1 : cy1;
            if (cx0 > cx1 || cy0 > cy1) continue;
            // wrapped particles lie in [0, L): no z window can be hit from beyond that range
            if (slz - a.rlist - zmargin > a.Lz + zmargin || shz + a.rlist + zmargin < -zmargin) continue;
            float px[M], py[M], pz[M];   // shifted i-particles
#pragma unroll
            for (int ia = 0; ia < M; ++ia) {
                px[ia] = ix[ia] + sx; py[ia] = iy[ia] + sy; pz[ia] = iz[ia] + sz;
            }
            const int ncy = cy1 - cy0 + 1, ncols = (cx1 - cx0 + 1) * ncy;
            const int c_lo = ncols * part / P, c_hi = ncols * (part + 1) / P;   // this part's columns
            for (int cb = c_lo; cb < c_hi; cb += 64) {
                // one column per lane (ascending column id): its z window of j-clusters
                int k0 = 0, kc = 0;
                const int cidx = cb + lane;
                if (cidx < c_hi) {
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
                    bool acc = ok;
                    if (ok && !(d2 < a.rb2)) {
                        // particle-pair check of this lane's candidate
                        bool hit = false;
                        for (int b = 0; b < N && !hit; ++b) {
                            const int sb = cj * N + b;
                            const float4 pj = a.xs[sb];
                            if (a.perm[sb] < 0) continue;
                            const float g = sq3(axis_gap(pj.x, pj.x, slx, shx), axis_gap(pj.y, pj.y, sly, shy),
                                                axis_gap(pj.z, pj.z, slz, shz));
                            if (!(g < rp2)) continue;   // too far from the whole i-cluster
#pragma unroll
                            for (int ia = 0; ia < M; ++ia)
                                hit |= ((ireal >> ia) & 1u) && sq3(px[ia] - pj.x, py[ia] - pj.y, pz[ia] - pj.z) < a.rl2;
                        }
                        acc = hit;
                    }
                    const unsigned long long accepted = __ballot(acc);
                    if (FILL) {
                        if (acc) {
                            // mask bit b*M + a: both particles real, slot(i) < slot(j) for the unshifted
                            // self/overlapping pair, not an exclusion in this image
                            unsigned long long mask = 0;
#pragma unroll
                            for (int b = 0; b < N; ++b) {
                                const int sb = cj * N + b;
                                unsigned keep = a.perm[sb] >= 0 ? ireal : 0u;
                                if (s == 13) {
                                    const int tr = sb - ci * M;
                                    keep &= tr >= M ? FULL : (tr <= 0 ? 0u : (1u << tr) - 1u);
                                }
                                mask |= (unsigned long long)keep << (b * M);
                            }
                            if (staged) {
                                for (int q = 0; q < nexcl; ++q) {
                                    const int v = xinfo[w][q], ia = v & 7, b = (v >> 3) - cj * N;
                                    if (b < 0 || b >= N) continue;
                                    const float4 pj = xpos[w][q];
                                    if (sq3(px[ia] - pj.x, py[ia] - pj.y, pz[ia] - pj.z) < a.rl2)
                                        mask &= ~(1ull << (b * M + ia));
                                }
                            } else {   // more partners than staged: read them from the CSR arrays
                                for (int ia = 0; ia < M; ++ia) {
                                    if (!((ireal >> ia) & 1u)) continue;
                                    const int io = a.perm[ci * M + ia];
                                    for (int e = a.excl_off[io]; e < a.excl_off[io + 1]; ++e) {
                                        const int ps = a.slot_of[a.excl_idx[e]];
                                        const int b = ps - cj * N;
                                        if (b < 0 || b >= N) continue;
                                        const float4 pj = a.xs[ps];
                                        if (sq3(px[ia] - pj.x, py[ia] - pj.y, pz[ia] - pj.z) < a.rl2)
                                            mask &= ~(1ull << (b * M + ia));
                                    }
                                }
                            }
                            const int rank = __popcll(accepted & ((1ull << lane) - 1ull));
                            nb_jentry en;
                            en.cj = cj;
                            en.shift = s;
                            en.mlo = (uint32_t)mask;
                            en.mhi = (uint32_t)(mask >> 32);
                            a.entries[wpos + rank] = en;
                            a.keys[wpos + rank] = d2;
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
        if (lane == 0) a.part_count[gw] = cnt;
    } else if (part == 0) {
        const int start = a.ci_start[ci], end = a.ci_start[ci + 1], ipos = a.ci_istart[ci];
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

// Per i-cluster entry counts and offsets from the per-part offsets.
__global__ void k_ci_offsets(const int *part_start, int nci_cap, int parts, int *ci_count, int *ci_start) {
    const int ci = blockIdx.x * blockDim.x + threadIdx.x;
    if (ci > nci_cap) return;
    const int s = part_start[(long)ci * parts];
    ci_start[ci] = s;
    if (ci < nci_cap) ci_count[ci] = part_start[(long)(ci + 1) * parts] - s;
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
    a.part_count = (int *)l->part_count.p;
    a.part_start = (const int *)l->part_start.p;
    a.ci_start = (const int *)l->ci_start.p;
    a.ci_istart = (const int *)l->ci_istart.p;
    a.totals = (const int *)l->totals.p;
    a.nci_cap = nci_cap;
    // parts per i-cluster: the largest power of two up to 8 that keeps about 6000
    // wavefronts or fewer (measured on MI355X: more parts only add per-part overhead
    // once the GPU holds that many latency-bound wavefronts)
    int parts = ctx->search_parts;
    if (parts == 0) {
        const long nci = std::max(1, g->n / g->m);
        parts = 1;
        while (parts < kMaxSearchParts && nci * parts * 2 <= 6000) parts *= 2;
    }
    a.parts = parts;
    const int nblocks = (int)(((long)nci_cap * parts + 3) / 4);
    // count pass
    if (g->m == 4 && g->nn == 4) run<4, 4>(l, a, false, nblocks, st);
    else if (g->m == 4 && g->nn == 8) run<4, 8>(l, a, false, nblocks, st);
    else run<8, 8>(l, a, false, nblocks, st);
    launch_scan_mode((const int *)l->part_count.p, (int *)l->part_start.p, nci_cap * parts, 0, 1,
                     (int *)l->totals.p, st);
    k_ci_offsets<<<(nci_cap + 256) / 256, 256, 0, st>>>((const int *)l->part_start.p, nci_cap, parts,
                                                      (int *)l->ci_count.p, (int *)l->ci_start.p);
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
