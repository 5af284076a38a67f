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
#include <cstring>

#include "devptr.h"
#include "internal.h"
#include "scan.h"

namespace {

using mxn::gptr;
using mxn::ld;
using mxn::plain;
using mxn::st;

// Search arguments with plain pointers (kernel arguments of the single-system
// launch) or global ones (read from a device table by the batched launch).
template <template <class> class P>
struct SearchArgsT {
    P<const int> nslots;
    P<const float4> xs;
    P<const int> perm, slot_of;
    P<const float4> bbi_lo, bbi_hi, bbj_lo, bbj_hi, colbb;
    P<const int> col_start;
    P<const int> excl_off, excl_idx;
    float Lx, Ly, Lz, inv_x, inv_y;
    int nx, ny;
    float rlist, rl2, rb2;
    P<int> part_count;                   // entries found by each (i-cluster, part)
    P<const int> part_start;             // region of each (i-cluster, part)
    P<int> region_overflow;              // set when a region is too small
    P<nb_jentry> entries;   // each region in (shift, j-cluster) order
    P<float> keys;          // bounding-box distance^2 of each entry (or null)
    P<int> jcount;          // entries per j-cluster (fill pass; zero before it)
    P<int> jrank;           // each written entry's rank among its j-cluster's entries
    int nci_cap, parts;
};
using SearchArgs = SearchArgsT<plain>;
using SearchArgsG = SearchArgsT<gptr>;

__device__ inline SearchArgsG to_global(const SearchArgs &a) {
    SearchArgsG g;
    g.nslots = (gptr<const int>)a.nslots;
    g.xs = (gptr<const float4>)a.xs;
    g.perm = (gptr<const int>)a.perm;
    g.slot_of = (gptr<const int>)a.slot_of;
    g.bbi_lo = (gptr<const float4>)a.bbi_lo;
    g.bbi_hi = (gptr<const float4>)a.bbi_hi;
    g.bbj_lo = (gptr<const float4>)a.bbj_lo;
    g.bbj_hi = (gptr<const float4>)a.bbj_hi;
    g.colbb = (gptr<const float4>)a.colbb;
    g.col_start = (gptr<const int>)a.col_start;
    g.excl_off = (gptr<const int>)a.excl_off;
    g.excl_idx = (gptr<const int>)a.excl_idx;
    g.Lx = a.Lx; g.Ly = a.Ly; g.Lz = a.Lz; g.inv_x = a.inv_x; g.inv_y = a.inv_y;
    g.nx = a.nx; g.ny = a.ny;
    g.rlist = a.rlist; g.rl2 = a.rl2; g.rb2 = a.rb2;
    g.part_count = (gptr<int>)a.part_count;
    g.part_start = (gptr<const int>)a.part_start;
    g.region_overflow = (gptr<int>)a.region_overflow;
    g.entries = (gptr<nb_jentry>)a.entries;
    g.keys = (gptr<float>)a.keys;
    g.jcount = (gptr<int>)a.jcount;
    g.jrank = (gptr<int>)a.jrank;
    g.nci_cap = a.nci_cap; g.parts = a.parts;
    return g;
}

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
constexpr int kExclStage = 64;   // staged exclusion partners per wavefront, one per lane
static_assert(kExclStage <= 64, "a lane stages one partner");

template <int M, int N, bool FILL, class A>
__device__ inline void search_body(const A &a, int blk) {
    constexpr unsigned FULL = (1u << M) - 1u;
    __shared__ float4 xpos[4][kExclStage];
    __shared__ float4 ipos[4][M];   // the i-cluster's particles moved by the current image shift
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gw = blk * 4 + w;
    const int P = a.parts, ci = gw / P, part = gw % P;
    if (ci >= a.nci_cap) return;
    const int nci = *a.nslots / M;
    if (ci >= nci) {   // beyond the padded slot count of this sort: contributes nothing to the scans
        if (lane == 0) a.part_count[gw] = 0;
        return;
    }
    int wpos = 0, resv = 0;   // fill pass: this part's reserved region
    if (FILL) {
        wpos = a.part_start[gw];
        resv = a.part_start[gw + 1] - wpos;
    }
    const float4 lo = ld(a.bbi_lo + ci), hi = ld(a.bbi_hi + ci);
    // the i-cluster's real slots: the mask the grid sort stores in its box's lo.w
    const unsigned ireal = __float_as_uint(lo.w);
    // keeps the z windows conservative against rounding: the FP32 squared distances
    // carry a relative error below 1e-6, so sqrt of that error is below 1e-3 rlist
    const float zmargin = 1e-3f + 2e-3f * a.rlist;
    const float pmargin = 1e-3f;   // keeps the particle-to-box prefilter conservative
    const float rp2 = (a.rlist + pmargin) * (a.rlist + pmargin);
    // exclusion partners of the i-particles: (slot * 8 + i-index, position), staged in LDS
    int nexcl = 0;
    bool staged = true;
    int xlo = 0x7fffffff, xhi = -1;   // slot range of the staged partners
    int xv = 0;                       // lane q < nexcl: staged partner q as slot * 8 + i-index
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
        nexcl = __builtin_amdgcn_readlane(incl, 63);
        staged = nexcl <= kExclStage && (long)a.nci_cap * M < (1L << 28);   // slot * 8 + i-index fits an int
        if (staged) {
            // partner q of the i-cluster goes to lane q: its i-particle is the first whose inclusive
            // count exceeds q, so every lane issues its own load chain at once
            int ia = 0, first = 0;
#pragma unroll
            for (int k = 0; k < M - 1; ++k) {
                const int ik = __shfl(incl, k, 64);
                if (lane >= ik) { ia = k + 1; first = ik; }
            }
            const int e = __shfl(e0, ia, 64) + lane - first;
            if (lane < nexcl) {
                const int ps = a.slot_of[a.excl_idx[e]];
                xv = ps * 8 + ia;
                xpos[w][lane] = ld(a.xs + ps);
                xlo = ps;
                xhi = ps;
            }
        }
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            xlo = min(xlo, __shfl_xor(xlo, o, 64));
            xhi = max(xhi, __shfl_xor(xhi, o, 64));
        }
        xlo = __builtin_amdgcn_readfirstlane(xlo);
        xhi = __builtin_amdgcn_readfirstlane(xhi);
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
            // shifted i-particles, in LDS (read back as broadcasts; registers would cost occupancy)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // the previous shift's reads are done
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane < M) {
                const float4 p = ld(a.xs + ci * M + lane);
                ipos[w][lane] = make_float4(p.x + sx, p.y + sy, p.z + sz, 0.0f);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int ncy = cy1 - cy0 + 1, ncols = (cx1 - cx0 + 1) * ncy;
            const int c_lo = ncols * part / P, c_hi = ncols * (part + 1) / P;   // this part's columns
            for (int cb = c_lo; cb < c_hi; cb += 64) {
                // one column per lane (ascending column id): its z window of j-clusters
                int k0 = 0, kc = 0;
                const int cidx = cb + lane;
                if (cidx < c_hi) {
                    const int c = (cx0 + cidx / ncy) * a.ny + cy0 + cidx % ncy;
                    const float4 cbb = ld(a.colbb + c);
                    const float gx = axis_gap(cbb.x, cbb.z, slx, shx), gy = axis_gap(cbb.y, cbb.w, sly, shy);
                    const float g2 = gx * gx + gy * gy;
                    if (g2 < a.rl2) {
                        // a j-cluster in this column lies at least (gx, gy) away in x and y, so
                        // only z gaps below sqrt(rlist^2 - g^2) can pass the box test
                        const float zr = sqrtf(a.rl2 - g2) + zmargin;
                        const int j0 = a.col_start[c] / N, j1 = a.col_start[c + 1] / N;
                        // a j-cluster of padding only (a column's last one when N is below the
                        // column granule) has an empty box, hi = -inf: it sorts as +inf, keeping
                        // the key nondecreasing
                        k0 = lower_bound(j0, j1, [&](int k) {
                            const float4 h = ld(a.bbj_hi + k);
                            return h.x == -INFINITY ? INFINITY : h.z;
                        }, slz - zr);
                        const int k1 = lower_bound(k0, j1, [&](int k) { return ld(a.bbj_lo + k).z; }, shz + zr);
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
                    unsigned jreal = 0;   // the candidate's real slots (its box's lo.w)
                    if (ok) {
                        const float4 jl = ld(a.bbj_lo + cj), jh = ld(a.bbj_hi + cj);
                        d2 = sq3(axis_gap(jl.x, jh.x, slx, shx), axis_gap(jl.y, jh.y, sly, shy),
                                 axis_gap(jl.z, jh.z, slz, shz));
                        ok = d2 < a.rl2;
                        jreal = __float_as_uint(jl.w);
                    }
                    bool acc = ok;
                    if (ok && !(d2 < a.rb2)) {
                        // particle-pair check of this lane's candidate, four j-particles per step
                        // with their loads in flight together (early exit between steps)
                        bool hit = false;
                        for (int b0 = 0; b0 < N && !hit; b0 += 4) {
                            float4 pj[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) pj[u] = ld(a.xs + cj * N + b0 + u);
                            bool near[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {   // real and near the whole i-cluster's box
                                const float g = sq3(axis_gap(pj[u].x, pj[u].x, slx, shx),
                                                    axis_gap(pj[u].y, pj[u].y, sly, shy),
                                                    axis_gap(pj[u].z, pj[u].z, slz, shz));
                                near[u] = ((jreal >> (b0 + u)) & 1u) && g < rp2;
                            }
#pragma unroll
                            for (int ia = 0; ia < M; ++ia) {
                                if (!((ireal >> ia) & 1u)) continue;
                                const float4 pi = ipos[w][ia];
#pragma unroll
                                for (int u = 0; u < 4; ++u)
                                    hit |= near[u] && sq3(pi.x - pj[u].x, pi.y - pj[u].y, pi.z - pj[u].z) < a.rl2;
                            }
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
                                unsigned keep = ((jreal >> b) & 1u) ? ireal : 0u;
                                if (s == 13) {
                                    const int tr = sb - ci * M;
                                    keep &= tr >= M ? FULL : (tr <= 0 ? 0u : (1u << tr) - 1u);
                                }
                                mask |= (unsigned long long)keep << (b * M);
                            }
                            if (staged) {
                                // only a j-cluster holding a staged partner's slot can lose mask bits
                                // partner q's slot and i-index are read from lane q's register: no
                                // memory wait unless the partner lies in this lane's candidate
                                if (cj * N + N - 1 >= xlo && cj * N <= xhi) {
                                    for (int q = 0; q < nexcl; ++q) {
                                        const int v = __builtin_amdgcn_readlane(xv, q), ia = v & 7,
                                                  b = (v >> 3) - cj * N;
                                        if (b < 0 || b >= N) continue;
                                        const float4 pj = xpos[w][q], pi = ipos[w][ia];
                                        if (sq3(pi.x - pj.x, pi.y - pj.y, pi.z - pj.z) < a.rl2)
                                            mask &= ~(1ull << (b * M + ia));
                                    }
                                }
                            } else {   // more partners than staged: read them from the CSR arrays
                                for (int ia = 0; ia < M; ++ia) {
                                    if (!((ireal >> ia) & 1u)) continue;
                                    const int io = a.perm[ci * M + ia];
                                    for (int e = a.excl_off[io]; e < a.excl_off[io + 1]; ++e) {
                                        const int ps = a.slot_of[a.excl_idx[e]];
                                        const int b = ps - cj * N;
                                        if (b < 0 || b >= N) continue;
                                        const float4 pj = ld(a.xs + ps), pi = ipos[w][ia];
                                        if (sq3(pi.x - pj.x, pi.y - pj.y, pi.z - pj.z) < a.rl2)
                                            mask &= ~(1ull << (b * M + ia));
                                    }
                                }
                            }
                            const int rank = cnt + __popcll(accepted & ((1ull << lane) - 1ull));
                            if (rank < resv) {
                                nb_jentry en;
                                en.cj = cj;
                                en.shift = s;
                                en.mlo = (uint32_t)mask;
                                en.mhi = (uint32_t)(mask >> 32);
                                st(a.entries + wpos + rank, en);
                                if (a.keys) a.keys[wpos + rank] = d2;
                                a.jrank[wpos + rank] = atomicAdd((int *)a.jcount + cj, 1);
                            }
                        }
                    }
                    cnt += __popcll(accepted);
                }
            }
        }
    }
    if (lane == 0) {
        a.part_count[gw] = cnt;
        if (FILL && cnt > resv) atomicOr((int *)a.region_overflow, 1);
    }
}

template <int M, int N, bool FILL>
// Six wavefronts per SIMD (at most 80 VGPRs, a few spills in the fill pass) measured 9 % faster on the
// production list than the four that the unconstrained register count allows.
__attribute__((amdgpu_waves_per_eu(6)))
__global__ __launch_bounds__(256) void k_search(SearchArgs a) {
    search_body<M, N, FILL>(a, blockIdx.x);
}

// Work items: each (i-cluster, part) region cut into runs of at most
// item_entries(N) entries, at the offsets of a scan over the regions' counts.
__device__ inline void items_body(int nparts_total, int parts, int per_item, const int *part_count,
                                  const int *part_start, const int *part_istart, long cap_items, int4 *items, int blk) {
    const int g = blk * blockDim.x + threadIdx.x;
    if (g >= nparts_total) return;
    const int resv = part_start[g + 1] - part_start[g];
    const int cnt = min(part_count[g], resv), start = part_start[g], ip = part_istart[g];
    const int nit = (cnt + per_item - 1) / per_item;
    for (int k = 0; k < nit; ++k) {
        if ((long)ip + k >= cap_items) return;   // overflow: latched by finalize_body
        const int js = start + k * per_item;
        const int je = min(js + per_item, start + cnt);
        items[ip + k] = make_int4(g / parts, js, je, 0);
    }
}

// Order the entries of each (i-cluster, part) region by bounding-box distance
// (ties by canonical position), so that the far entries, whose pairs mostly
// lie beyond the cut-off, share force-kernel passes whose pair work can be
// skipped.  One wavefront per region, rank sort with the keys staged in LDS.
__global__ __launch_bounds__(64) void k_sort_entries(const int *part_start, const int *part_count,
                                                     const nb_jentry *in, const float *keys, nb_jentry *out,
                                                     const int *rank_in, int *rank_out) {
    __shared__ float sk[1024];
    const int g = blockIdx.x, lane = threadIdx.x;
    const int b = part_start[g], n = min(part_count[g], part_start[g + 1] - b);
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
        rank_out[b + r] = rank_in[b + i];
    }
}

// Region counts of a count pass (one workgroup of 1024 threads).  out[0]: the largest region count;
// out[1]: the work items the counts make (per_item entries each); out[2]: the entries (the list's
// totals[2] is set again by its fill pass, before any force call reads it).
__global__ __launch_bounds__(1024) void k_max_count(const int *in, int n, int per_item, int *out) {
    __shared__ int m[1024], c[1024], e[1024];
    int v = 0, it = 0, en = 0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        v = max(v, in[i]);
        it += (in[i] + per_item - 1) / per_item;
        en += in[i];
    }
    m[threadIdx.x] = v;
    c[threadIdx.x] = it;
    e[threadIdx.x] = en;
    __syncthreads();
    for (unsigned s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            m[threadIdx.x] = max(m[threadIdx.x], m[threadIdx.x + s]);
            c[threadIdx.x] += c[threadIdx.x + s];
            e[threadIdx.x] += e[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = m[0];
        out[1] = c[0];
        out[2] = e[0];
    }
}

// Uniform regions: region g starts at g * size (g = 0 .. n).
__global__ void k_region_starts(int n, int size, int *start) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g <= n) start[g] = g * size;
}

// totals: [0] entries, [1] items (from the scan), [3] region overflow; writes
// [2] = usable item count (0 on overflow: a region, the items or the j-force
// rows outgrown), latches the overflow flag and clears [3] for the next build
__device__ inline void finalize_body(int *totals, long cap_items, long cap_rows, int *flags) {
    if (threadIdx.x != 0) return;
    const bool over = totals[3] != 0 || (long)totals[1] > cap_items || (long)totals[0] > cap_rows;
    totals[2] = over ? 0 : totals[1];
    totals[3] = 0;
    if (over) atomicOr(flags, mxn::FLAG_OVERFLOW);
}


// --------------------------------------------------------------------------
// j-cluster view of a list.  The force kernels store each entry's j-forces
// (instead of adding them to memory with atomics) in a row of a buffer whose
// rows are grouped by j-cluster, so that the reduction reads each j-cluster's
// rows contiguously.  The fill pass (and the prune) take each written entry's
// rank among its j-cluster's entries from a counter per j-cluster; after the
// build an exclusive scan of the counters (which clears them for the next
// build) gives each j-cluster's first row, and this pass turns every usable
// entry's rank into its row (the force kernel then reads one row index per
// entry instead of a dependent gather of the j-cluster's start: measured
// cheaper).  The row order within a j-cluster depends on timing; the
// reduction sums in fixed point, so the forces do not.
struct JPosArgs {
    const int *totals;   // [2]: usable items
    const int4 *items;
    const nb_jentry *entries;
    const int *jstart;   // first row of each j-cluster
    int *jrank;          // rank in, row out
};

// one wavefront per work item (a grid-stride loop), one lane per entry (items hold at most 64)
__device__ inline void jpos_body(const JPosArgs &a, int blk, int nblk) {
    const int lane = threadIdx.x & 63;
    const int total = a.totals[2];
    for (int t = blk * 4 + (threadIdx.x >> 6); t < total; t += nblk * 4) {
        const int4 it = a.items[t];
        const int e = it.y + lane;
        if (e < it.z) a.jrank[e] += a.jstart[a.entries[e].cj];
    }
}

constexpr int kJposBlocks = 1024;   // workgroups of the position pass (per replica in a batch: 256)


// After a fill (or prune) pass, two independent workgroups of 1024 threads: the first scans the regions'
// entry counts into item offsets and sets the usable item count (finalize_body, by the thread that wrote
// the totals), the second scans the j-cluster counters into each j-cluster's first row and clears them
// for the next build: one launch instead of three.  The items themselves are written by k_items.
__global__ __launch_bounds__(1024) void k_finish(int nregions, int per_item, const int *part_count,
                                                 int *part_istart, long cap_items, long cap_rows, int *totals,
                                                 int *flags, int *jcount, int *jstart, int njc) {
    if (blockIdx.x == 0) {
        mxn::scan_body(part_count, part_istart, nregions, 2, per_item, totals + 1, totals);
        finalize_body(totals, cap_items, cap_rows, flags);
    } else {
        mxn::scan_body(jcount, jstart, njc, 0, 1, nullptr, nullptr, jcount);
    }
}

__global__ void k_items(int nparts_total, int parts, int per_item, const int *part_count, const int *part_start,
                        const int *part_istart, long cap_items, int4 *items) {
    items_body(nparts_total, parts, per_item, part_count, part_start, part_istart, cap_items, items, blockIdx.x);
}

// After k_finish (and the distance sort, if any): one wavefront per region writes the region's work items
// and turns each of its entries' rank into the entry's row (its j-cluster's first row plus the rank), for
// a usable list (in one launch: the items need not be read back to find the entries).
__global__ __launch_bounds__(256) void k_items_rows(int nregions, int parts, int per_item, const int *part_count,
                                                    const int *part_start, const int *part_istart, long cap_items,
                                                    int4 *items, const int *totals, const nb_jentry *entries,
                                                    const int *jstart, int *jrank) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (g >= nregions) return;
    const int start = part_start[g], resv = part_start[g + 1] - start;
    const int cnt = min(part_count[g], resv), ip = part_istart[g];
    const int nit = (cnt + per_item - 1) / per_item;
    for (int k = lane; k < nit; k += 64) {
        if ((long)ip + k >= cap_items) break;   // overflow: latched by finalize_body
        const int js = start + k * per_item;
        items[ip + k] = make_int4(g / parts, js, min(js + per_item, start + cnt), 0);
    }
    if (totals[2] == 0) return;   // no usable items (or no entries): the rows are never read
    for (int e = start + lane; e < start + cnt; e += 64) jrank[e] += jstart[entries[e].cj];
}

// --------------------------------------------------------------------------
// Second stage of a two-stage list (Sec. 2.3: the list built from bounding
// boxes, then cluster pairs whose particles are all beyond a radius removed
// by a particle-distance test on the GPU).  One wavefront per region of the
// outer list, one lane per entry: an entry is kept iff a real particle of
// the i-cluster, moved by the entry's image shift, and a real particle of
// the j-cluster are closer than r, formed with the search's own separately
// rounded FP32 operations, at the gathered positions of the call.  Kept
// entries keep their order, masks and region; like the fill pass, each takes
// its rank within its j-cluster.
struct PruneArgs {
    const int *nslots;
    const float4 *xs_now;
    const int *perm;
    const int *part_start;      // the regions (the outer list's layout)
    const int *part_count_in;   // entries of the outer list per region
    const int *totals_in;       // the outer list's totals: [1] items, [2] usable items
    const nb_jentry *in;
    int *part_count;            // kept entries per region
    nb_jentry *out;
    int *jcount, *jrank;
    int *region_overflow;
    float Lx, Ly, Lz, r2;
    int nregions, parts;
};

template <int M, int N>
__global__ __launch_bounds__(256) void k_prune(PruneArgs a) {
    const int lane = threadIdx.x & 63, g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= a.nregions) return;
    // an overflowed outer list (items counted, none usable) is incomplete, and so is its prune
    if (a.totals_in[2] == 0 && a.totals_in[1] > 0) {
        if (lane == 0) {
            a.part_count[g] = 0;
            if (g == 0) atomicOr(a.region_overflow, 1);
        }
        return;
    }
    const int ci = g / a.parts;
    if (ci >= *a.nslots / M) {
        if (lane == 0) a.part_count[g] = 0;
        return;
    }
    const int start = a.part_start[g];
    const int n_in = min(a.part_count_in[g], a.part_start[g + 1] - start);
    float ix[M], iy[M], iz[M];
    unsigned ireal = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const float4 p = a.xs_now[ci * M + k];
        ix[k] = p.x; iy[k] = p.y; iz[k] = p.z;
        ireal |= (a.perm[ci * M + k] >= 0 ? 1u : 0u) << k;
    }
    int cnt = 0;
    for (int e0 = 0; e0 < n_in; e0 += 64) {
        const int e = e0 + lane;
        const bool valid = e < n_in;
        const nb_jentry en = a.in[start + (valid ? e : 0)];
        const int s = en.shift;
        const float sx = (float)(s / 9 - 1) * a.Lx, sy = (float)((s / 3) % 3 - 1) * a.Ly,
                    sz = (float)(s % 3 - 1) * a.Lz;
        // the entry's N j-particles loaded together, then all M x N tests (no early exit: the
        // wavefront waits for its slowest lane anyway)
        float4 pj[N];
        bool jreal[N];
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const int sb = en.cj * N + b;
            pj[b] = a.xs_now[sb];
            jreal[b] = a.perm[sb] >= 0;
        }
        bool keep = false;
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const float px = ix[k] + sx, py = iy[k] + sy, pz = iz[k] + sz;
                keep |= jreal[b] && ((ireal >> k) & 1u) && sq3(px - pj[b].x, py - pj[b].y, pz - pj[b].z) < a.r2;
            }
        keep &= valid;
        const unsigned long long bal = __ballot(keep);
        if (keep) {
            const int pos = start + cnt + __popcll(bal & ((1ull << lane) - 1ull));
            a.out[pos] = en;
            a.jrank[pos] = atomicAdd(a.jcount + en.cj, 1);
        }
        cnt += __popcll(bal);
    }
    if (lane == 0) a.part_count[g] = cnt;
}

// --------------------------------------------------------------------------
// Super-cluster view of an 8x8 list (the grouped layout of Sec. 2.3 and 3.2:
// S consecutive i-clusters share one list of j-clusters).  One workgroup per
// super-cluster gathers the entries of its S i-clusters as 64-bit keys
// (shift, j-cluster, i-cluster within the super-cluster, entry position),
// sorts them in LDS (bitonic), and writes one super-cluster entry per
// distinct (shift, j-cluster): (j-cluster, shift | i-cluster bits << 8 |
// (self i-cluster + 1) << 16, 0, rank among the j-cluster's entries) and a
// record of S exclusion masks, slot g for i-cluster g (slots of i-clusters
// the entry does not reach are not written).  The self i-cluster is the
// one the j-cluster is (zero shift), whose pass is a half triangle; 0 if
// none.  Outputs go to the super-cluster's span of the list's regions (its
// keys fit there, so its entries do too).  The order depends only on the
// list, so the forces do as well.
constexpr int kSciKeys = 4096;

struct SciArgs {
    const int *nslots;
    const int *totals;   // the list's: [2] usable items (0 after an overflow)
    const int *part_start, *part_count;
    const nb_jentry *entries;
    int parts, nregions, S, ngroups;
    int4 *ent;
    uint2 *mask;
    int *count, *base;   // per super-cluster: entries; first position (base[ngroups]: end)
    int *jcount;         // per j-cluster counters (zero before the pass)
};

// exclusive prefix of a flag over the 256 threads, and the flag count
__device__ inline int block_flag_scan(bool f, int *sw, int &total) {
    const unsigned long long b = __ballot(f);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)b, 0u));
    if (lane == 0) sw[w] = __popcll(b);
    __syncthreads();
    int off = 0;
    for (int k = 0; k < w; ++k) off += sw[k];
    total = sw[0] + sw[1] + sw[2] + sw[3];
    __syncthreads();
    return off + r;
}

__global__ __launch_bounds__(256) void k_sci_view(SciArgs a) {
    __shared__ unsigned long long key[kSciKeys];
    __shared__ int roff[65];
    __shared__ int sw[4];
    const int grp = blockIdx.x, t = threadIdx.x;
    const int span = a.S * a.parts;
    const int r0 = min(grp * span, a.nregions), r1 = min(r0 + span, a.nregions);
    const int base = a.part_start[r0];
    if (t == 0) {
        a.base[grp] = base;
        if (grp == a.ngroups - 1) a.base[grp + 1] = a.part_start[r1];
        const int nci = *a.nslots / 8;
        const bool usable = a.totals[2] > 0;
        int o = 0;
        for (int r = r0; r < r1; ++r) {
            roff[r - r0] = o;
            const int cap = a.part_start[r + 1] - a.part_start[r];
            o += (usable && r / a.parts < nci) ? min(a.part_count[r], cap) : 0;
        }
        roff[r1 - r0] = o;
    }
    __syncthreads();
    const int n = min(roff[r1 - r0], kSciKeys);   // the host sizes S so that every span fits
    for (int r = r0; r < r1; ++r) {
        const int o = roff[r - r0], cnt = roff[r - r0 + 1] - o, s0 = a.part_start[r];
        const unsigned g = (unsigned)((r - r0) / a.parts);
        for (int k = t; k < cnt && o + k < kSciKeys; k += 256) {
            const nb_jentry e = a.entries[s0 + k];
            const unsigned kk = ((unsigned)e.shift << 27) | ((unsigned)e.cj << 3) | g;
            key[o + k] = ((unsigned long long)kk << 32) | (unsigned)(s0 + k);
        }
    }
    int np = 1;
    while (np < n) np <<= 1;
    for (int k = n + t; k < np; k += 256) key[k] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= np; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = t; i < np / 2; i += 256) {
                const int lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                const bool up = (lo & size) == 0;
                const unsigned long long x = key[lo], y = key[hi];
                if ((x > y) == up) {
                    key[lo] = y;
                    key[hi] = x;
                }
            }
            __syncthreads();
        }
    int done = 0;
    for (int p0 = 0; p0 < n; p0 += 256) {
        const int p = p0 + t;
        unsigned long long kp = 0;
        bool head = false;
        if (p < n) {
            kp = key[p];
            head = p == 0 || (key[p - 1] >> 35) != (kp >> 35);
        }
        int tot;
        const int idx = done + block_flag_scan(head, sw, tot);
        if (head) {
            const int cj = (int)((kp >> 35) & 0xFFFFFFu), shift = (int)(kp >> 59);
            int gm = 0;
            for (int q = p; q < n && (key[q] >> 35) == (kp >> 35); ++q) {
                const int g = (int)((key[q] >> 32) & 7u);
                const nb_jentry e = a.entries[(int)(unsigned)key[q]];
                a.mask[(long)(base + idx) * a.S + g] = make_uint2(e.mlo, e.mhi);
                gm |= 1 << g;
            }
            const int own = cj - grp * a.S;
            const int self = (shift == 13 && own >= 0 && own < a.S) ? own + 1 : 0;
            const int rank = atomicAdd(a.jcount + cj, 1);
            a.ent[base + idx] = make_int4(cj, shift | (gm << 8) | (self << 16), 0, rank);
        }
        done += tot;
    }
    if (t == 0) a.count[grp] = done;
}

// rank -> row for every super-cluster entry of a usable work item
__global__ __launch_bounds__(256) void k_sci_rows(const int *totals, const int4 *items, int4 *ent, const int *jstart) {
    const int lane = threadIdx.x & 63;
    const int total = totals[2];
    for (int t = blockIdx.x * 4 + (threadIdx.x >> 6); t < total; t += gridDim.x * 4) {
        const int4 it = items[t];
        const int e = it.y + lane;
        if (e < it.z) ent[e].w += jstart[ent[e].x];
    }
}

// --------------------------------------------------------------------------
// Batched rebuild of many replicas' lists (the fill pass into the regions the
// replicas' last synchronous builds sized), one launch per stage; a
// workgroup finds its replica by binary search in the stage's prefix of
// share sizes.

struct ListJob {
    SearchArgs a;
    JPosArgs jp;
    int nregions, per_item;
    int *part_count, *part_start, *part_istart, *totals;
    int4 *items;
    long cap_items, cap_rows;
    int *flags;
};

enum { LS_SEARCH, LS_ITEMS, LS_JPOS, LS_NSTAGES };

__device__ inline int job_of(const int *off, int n, int b) {
    int lo = 0, hi = n - 1;   // last r with off[r] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int M, int N>
__global__ __launch_bounds__(256) void kb_search(const ListJob *J, const int *off, int n) {
    const int r = job_of(off, n, blockIdx.x);
    search_body<M, N, true>(to_global(J[r].a), blockIdx.x - off[r]);
}

__global__ void kb_items(const ListJob *J, const int *off, int n) {
    const int r = job_of(off, n, blockIdx.x);
    const ListJob &j = J[r];
    items_body(j.nregions, j.a.parts, j.per_item, j.part_count, j.part_start, j.part_istart, j.cap_items, j.items,
               blockIdx.x - off[r]);
}

__global__ void kb_finalize(const ListJob *J) {
    const ListJob &j = J[blockIdx.x];
    finalize_body(j.totals, j.cap_items, j.cap_rows, j.flags);
}

__global__ __launch_bounds__(256) void kb_jpos(const ListJob *J, const int *off, int n) {
    const int r = job_of(off, n, blockIdx.x);
    jpos_body(J[r].jp, blockIdx.x - off[r], off[r + 1] - off[r]);
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

static SearchArgs make_search(const nb_list *l, const int *excl_off, const int *excl_idx) {
    const nb_grid *g = l->grid;
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
    a.region_overflow = (int *)l->totals.p + 3;
    a.nci_cap = g->slots_cap / g->m;
    return a;
}


static JPosArgs make_jpos(const nb_list *l) {
    JPosArgs v{};
    v.totals = (const int *)l->totals.p;
    v.items = (const int4 *)l->items.p;
    v.entries = (const nb_jentry *)l->entries.p;
    v.jstart = (const int *)l->jstart.p;
    v.jrank = (int *)l->jrank.p;
    return v;
}

// item offsets per region (totals[0] = entries, totals[1] = items) and the work items
// usable count and j-cluster first rows of a list after its fill or prune pass
static void finish_list(nb_list *l, int nregions, hipStream_t st) {
    const nb_grid *g = l->grid;
    k_finish<<<2, 1024, 0, st>>>(nregions, item_entries(g->nn), (const int *)l->part_count.p,
                                 (int *)l->part_istart.p, l->cap_items, l->cap_rows, (int *)l->totals.p,
                                 l->ctx->d_flags, (int *)l->jcount.p, (int *)l->jstart.p, g->slots_cap / g->nn);
}
// work items and each usable entry's row (after finish_list, and after the distance sort)
static void finish_rows(nb_list *l, int nregions, int parts, hipStream_t st) {
    k_items_rows<<<(nregions + 3) / 4, 256, 0, st>>>(nregions, parts, item_entries(l->grid->nn),
                                                     (const int *)l->part_count.p, (const int *)l->part_start.p,
                                                     (const int *)l->part_istart.p, l->cap_items,
                                                     (int4 *)l->items.p, (const int *)l->totals.p,
                                                     (const nb_jentry *)l->entries.p, (const int *)l->jstart.p,
                                                     (int *)l->jrank.p);
}

size_t list_job_size() { return sizeof(ListJob); }
int list_job_stages() { return LS_NSTAGES; }

// The list must have been sized by a synchronous build for its grid's capacity.
void fill_list_job(void *out, nb_list *l, const int *excl_off, const int *excl_idx, ScanJob *scan,
                   ScanJob *jscan) {
    ListJob j{};
    j.a = make_search(l, excl_off, excl_idx);
    j.a.jcount = (int *)l->jcount.p;
    j.a.jrank = (int *)l->jrank.p;
    j.jp = make_jpos(l);
    j.a.parts = l->resv_parts;
    j.a.entries = (nb_jentry *)l->entries.p;
    j.a.keys = nullptr;
    j.nregions = l->resv_nci * l->resv_parts;
    j.per_item = item_entries(l->grid->nn);
    j.part_count = (int *)l->part_count.p;
    j.part_start = (int *)l->part_start.p;
    j.part_istart = (int *)l->part_istart.p;
    j.totals = (int *)l->totals.p;
    j.items = (int4 *)l->items.p;
    j.cap_items = l->cap_items;
    j.cap_rows = l->cap_rows;
    j.flags = l->ctx->d_flags;
    std::memcpy(out, &j, sizeof j);
    *scan = ScanJob{j.part_count, j.part_istart, j.nregions, 2, j.per_item, j.totals + 1, j.totals, nullptr};
    int *jc = (int *)l->jcount.p;
    *jscan = ScanJob{jc, (int *)l->jstart.p, l->grid->slots_cap / l->grid->nn, 0, 1, nullptr, nullptr, jc};
}

void list_job_blocks(const nb_list *l, int *blocks_per_stage) {
    const long nreg = (long)l->resv_nci * l->resv_parts;
    blocks_per_stage[LS_SEARCH] = (int)((nreg + 3) / 4);
    blocks_per_stage[LS_ITEMS] = (int)((nreg + 255) / 256);
    blocks_per_stage[LS_JPOS] = (int)std::max(1L, std::min<long>((l->cap_items + 3) / 4, kJposBlocks / 4));
}

int launch_pairlist_batch(hipStream_t st, int m, int nn, const void *jobs, const int *off, int n_rep, const int *total,
                          const ScanJob *scans) {
    const ListJob *J = (const ListJob *)jobs;
    const int stride = n_rep + 1;
    if (m == 4 && nn == 4) kb_search<4, 4><<<total[LS_SEARCH], 256, 0, st>>>(J, off + LS_SEARCH * stride, n_rep);
    else if (m == 4 && nn == 8) kb_search<4, 8><<<total[LS_SEARCH], 256, 0, st>>>(J, off + LS_SEARCH * stride, n_rep);
    else if (m == 8 && nn == 4) kb_search<8, 4><<<total[LS_SEARCH], 256, 0, st>>>(J, off + LS_SEARCH * stride, n_rep);
    else kb_search<8, 8><<<total[LS_SEARCH], 256, 0, st>>>(J, off + LS_SEARCH * stride, n_rep);
    launch_scan_batch(scans, n_rep, st);
    kb_items<<<total[LS_ITEMS], 256, 0, st>>>(J, off + LS_ITEMS * stride, n_rep);
    kb_finalize<<<n_rep, 64, 0, st>>>(J);
    launch_scan_batch(scans + n_rep, n_rep, st);
    kb_jpos<<<total[LS_JPOS], 256, 0, st>>>(J, off + LS_JPOS * stride, n_rep);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

int launch_pairlist(nb_list *l, const int *excl_off, const int *excl_idx, bool sync, bool by_distance) {
    const nb_grid *g = l->grid;
    nb_ctx *ctx = l->ctx;
    hipStream_t st = ctx->stream;
    const int nci_cap = g->slots_cap / g->m;
    SearchArgs a = make_search(l, excl_off, excl_idx);
    // A synchronous build (also the first, and any after the grid's capacity
    // changed) counts the entries and gives every (i-cluster, part) region the
    // largest count plus a quarter plus 8 (uniform, because a re-sort re-forms
    // the clusters, so a region's next occupant may have any count); later
    // builds search once and fill the regions.
    const bool reserve = sync || l->resv_parts == 0 || l->resv_nci != nci_cap;
    int parts = l->resv_parts;
    if (reserve) {
        // parts per i-cluster: the largest power of two up to 8 that keeps about 6000
        // wavefronts or fewer (measured on MI355X: more parts only add per-part overhead
        // once the GPU holds that many latency-bound wavefronts)
        parts = ctx->search_parts;
        if (parts == 0) {
            const long nci = std::max(1, g->n / g->m);
            parts = 1;
            while (parts < kMaxSearchParts && nci * parts * 2 < 6000) parts *= 2;
        }
    }
    a.parts = parts;
    const int nregions = nci_cap * parts;
    const int nblocks = (int)(((long)nregions + 3) / 4);
    if (reserve) {
        if (g->m == 4 && g->nn == 4) run<4, 4>(l, a, false, nblocks, st);
        else if (g->m == 4 && g->nn == 8) run<4, 8>(l, a, false, nblocks, st);
        else if (g->m == 8 && g->nn == 4) run<8, 4>(l, a, false, nblocks, st);
        else run<8, 8>(l, a, false, nblocks, st);
        k_max_count<<<1, 1024, 0, st>>>((const int *)l->part_count.p, nregions, item_entries(g->nn),
                                         (int *)l->totals.p);
        MXN_HIP(hipMemcpyAsync(ctx->h_pinned, l->totals.p, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
        MXN_HIP(hipMemsetAsync((int *)l->totals.p + 3, 0, sizeof(int), st));
        MXN_HIP(hipStreamSynchronize(st));
        const long mx = ctx->h_pinned[0];
        const long size = mx + mx / 4 + 8;
        if (size * nregions > (1L << 31) - 1) return fail(NB_ERR_OOM, "nb_pairlist_build: list larger than 2^31 entries");
        const long ce = size * nregions;
        if (ce > l->cap_entries) {
            int rc = ensure(l->ctx, l->entries, (size_t)ce * sizeof(nb_jentry));
            if (rc) return rc;
            l->cap_entries = ce;
        }
        const long cit = ce / item_entries(g->nn) + nregions + 256;   // each region: at most count/per-item + 1 items
        if (cit > l->cap_items) {
            int rc = ensure(l->ctx, l->items, (size_t)cit * sizeof(int4));
            if (rc) return rc;
            l->cap_items = cit;
        }
        // j-cluster view and force-call buffers for this capacity; the counters start cleared
        const long njc = g->slots_cap / g->nn;
        int rc = ensure(l->ctx, l->jcount, (size_t)(njc + 1) * 4);
        rc = rc ? rc : ensure(l->ctx, l->jstart, (size_t)(njc + 1) * 4);
        rc = rc ? rc : ensure(l->ctx, l->jrank, (size_t)l->cap_entries * 4);
        // j-force rows (one per entry, 12 N bytes): the synchronous build's entries plus a quarter, not the regions'
        // capacity (about three times the entries); a later asynchronous build with more entries than that
        // latches NB_ERR_OVERFLOW like an outgrown region
        const long ent = ctx->h_pinned[2];
        const long rows = std::min(l->cap_entries, ent + ent / 4 + 1024);
        if (rows > l->cap_rows) {
            rc = rc ? rc : ensure(l->ctx, l->fj, (size_t)rows * g->nn * 12);
            if (rc == NB_OK) l->cap_rows = rows;
        }
        rc = rc ? rc : ensure(l->ctx, l->fi, (size_t)l->cap_items * g->m * 16);
        if (rc) return rc;
        MXN_HIP(hipMemsetAsync(l->jcount.p, 0, (size_t)(njc + 1) * 4, st));
        k_region_starts<<<(nregions + 256) / 256, 256, 0, st>>>(nregions, (int)size, (int *)l->part_start.p);
        l->resv_parts = parts;
        l->resv_nci = nci_cap;
        l->last_entries = ce;
        l->resv_size = size;
        l->est_items = ctx->h_pinned[1];
    }
    if (by_distance) {   // the fill pass writes canonical order and keys; the sort orders each region
        int rc = ensure(l->ctx, l->entries_canon, (size_t)l->cap_entries * sizeof(nb_jentry));
        if (rc) return rc;
        rc = ensure(l->ctx, l->keys, (size_t)l->cap_entries * sizeof(float));
        if (rc) return rc;
        rc = ensure(l->ctx, l->jrank_canon, (size_t)l->cap_entries * 4);
        if (rc) return rc;
    }
    a.entries = (nb_jentry *)(by_distance ? l->entries_canon.p : l->entries.p);
    a.keys = by_distance ? (float *)l->keys.p : nullptr;
    // the j-cluster counters and ranks (allocated by a reserving build)
    a.jcount = (int *)l->jcount.p;
    a.jrank = (int *)(by_distance ? l->jrank_canon.p : l->jrank.p);
    if (!a.jcount || !a.jrank || !l->jstart.p || !l->fj.p || !l->fi.p)
        return fail(NB_ERR_STATE, "nb_pairlist_build: j-cluster view buffers missing");
    if (g->m == 4 && g->nn == 4) run<4, 4>(l, a, true, nblocks, st);
    else if (g->m == 4 && g->nn == 8) run<4, 8>(l, a, true, nblocks, st);
    else if (g->m == 8 && g->nn == 4) run<8, 4>(l, a, true, nblocks, st);
    else run<8, 8>(l, a, true, nblocks, st);
    finish_list(l, nregions, st);
    if (by_distance)
        k_sort_entries<<<nregions, 64, 0, st>>>((const int *)l->part_start.p, (const int *)l->part_count.p,
                                                (const nb_jentry *)l->entries_canon.p, (const float *)l->keys.p,
                                                (nb_jentry *)l->entries.p, (const int *)l->jrank_canon.p,
                                                (int *)l->jrank.p);
    finish_rows(l, nregions, parts, st);
    l->sci_valid = false;
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

// i-clusters per super-cluster for a list (0: no super-cluster view): the
// largest of 8 and 4 (at most want, if nonzero) whose span of regions fits
// the LDS sort
int sci_size(const nb_list *l, int want) {
    const nb_grid *g = l->grid;
    if (!g || g->m != 8 || g->nn != 8 || l->resv_parts <= 0 || l->resv_size <= 0) return 0;
    if ((long)g->slots_cap / 8 >= (1L << 24)) return 0;   // j-cluster index in 24 key bits
    for (int S = 8; S >= 4; S >>= 1)
        if ((want == 0 || S <= want) && (long)S * l->resv_parts * l->resv_size <= kSciKeys) return S;
    return 0;
}

// Build the super-cluster view of l (S i-clusters per super-cluster, per_item
// entries per work item) on the context stream: keys and entries, work
// items, the j-cluster rows of the entries.
int launch_sci_view(const nb_list *l, int S, int per_item) {
    const nb_grid *g = l->grid;
    hipStream_t st = l->ctx->stream;
    const int nregions = l->resv_nci * l->resv_parts;
    const int ngroups = (l->resv_nci + S - 1) / S;
    const long njc = g->slots_cap / g->nn;
    const long cap_items = l->cap_entries / per_item + ngroups + 256;
    void *old_jc = l->sci_jcount.p, *old_tot = l->sci_totals.p;
    int rc = ensure(l->ctx, l->sci_ent, (size_t)l->cap_entries * sizeof(int4));
    rc = rc ? rc : ensure(l->ctx, l->sci_mask, (size_t)l->cap_entries * S * sizeof(uint2));
    rc = rc ? rc : ensure(l->ctx, l->sci_count, (size_t)(ngroups + 1) * 4);
    rc = rc ? rc : ensure(l->ctx, l->sci_base, (size_t)(ngroups + 1) * 4);
    rc = rc ? rc : ensure(l->ctx, l->sci_istart, (size_t)(ngroups + 1) * 4);
    rc = rc ? rc : ensure(l->ctx, l->sci_items, (size_t)cap_items * sizeof(int4));
    rc = rc ? rc : ensure(l->ctx, l->sci_jcount, (size_t)(njc + 1) * 4);
    rc = rc ? rc : ensure(l->ctx, l->sci_jstart, (size_t)(njc + 1) * 4);
    rc = rc ? rc : ensure(l->ctx, l->sci_totals, 16);
    rc = rc ? rc : ensure(l->ctx, l->sci_fi, (size_t)cap_items * S * 8 * sizeof(float4));
    if (rc) return rc;
    if (l->sci_jcount.p != old_jc || l->sci_njc != njc) {   // counters start cleared; the scan clears them after use
        MXN_HIP(hipMemsetAsync(l->sci_jcount.p, 0, (size_t)(njc + 1) * 4, st));
        l->sci_njc = njc;
    }
    if (l->sci_totals.p != old_tot) MXN_HIP(hipMemsetAsync(l->sci_totals.p, 0, 16, st));
    SciArgs a{};
    a.nslots = (const int *)g->nslots.p;
    a.totals = (const int *)l->totals.p;
    a.part_start = (const int *)l->part_start.p;
    a.part_count = (const int *)l->part_count.p;
    a.entries = (const nb_jentry *)l->entries.p;
    a.parts = l->resv_parts;
    a.nregions = nregions;
    a.S = S;
    a.ngroups = ngroups;
    a.ent = (int4 *)l->sci_ent.p;
    a.mask = (uint2 *)l->sci_mask.p;
    a.count = (int *)l->sci_count.p;
    a.base = (int *)l->sci_base.p;
    a.jcount = (int *)l->sci_jcount.p;
    int *tot = (int *)l->sci_totals.p;
    k_sci_view<<<ngroups, 256, 0, st>>>(a);
    // rows: a super-cluster entry stands for one or more of the list's entries, which fit l's rows
    k_finish<<<2, 1024, 0, st>>>(ngroups, per_item, a.count, (int *)l->sci_istart.p, cap_items, l->cap_rows, tot,
                                 l->ctx->d_flags, a.jcount, (int *)l->sci_jstart.p, (int)njc);
    k_items<<<(ngroups + 255) / 256, 256, 0, st>>>(ngroups, 1, per_item, a.count, a.base,
                                                  (const int *)l->sci_istart.p, cap_items, (int4 *)l->sci_items.p);
    const int nb = (int)std::max<long>(1, std::min<long>((cap_items + 3) / 4, kJposBlocks));
    k_sci_rows<<<nb, 256, 0, st>>>(tot, (const int4 *)l->sci_items.p, a.ent, (const int *)l->sci_jstart.p);
    MXN_HIP(hipGetLastError());
    l->sci_cap_items = cap_items;
    l->sci_S = S;
    l->sci_per_item = per_item;
    l->sci_valid = true;
    return NB_OK;
}

int launch_prune(nb_list *in, const nb_list *outer, float r) {
    const nb_grid *g = outer->grid;
    nb_ctx *ctx = in->ctx;
    hipStream_t st = ctx->stream;
    const int nregions = outer->resv_nci * outer->resv_parts;
    // the outer list's layout, with buffers of its capacity; new counters start cleared
    const long njc = g->slots_cap / g->nn;
    const size_t nreg = (size_t)outer->resv_nci * kMaxSearchParts + 1;
    void *old_jc = in->jcount.p, *old_tot = in->totals.p;
    int rc = ensure(in->ctx, in->part_count, nreg * 4);
    rc = rc ? rc : ensure(in->ctx, in->part_start, nreg * 4);
    rc = rc ? rc : ensure(in->ctx, in->part_istart, nreg * 4);
    rc = rc ? rc : ensure(in->ctx, in->totals, 16);
    rc = rc ? rc : ensure(in->ctx, in->entries, (size_t)outer->cap_entries * sizeof(nb_jentry));
    rc = rc ? rc : ensure(in->ctx, in->items, (size_t)outer->cap_items * sizeof(int4));
    rc = rc ? rc : ensure(in->ctx, in->jcount, (size_t)(njc + 1) * 4);
    rc = rc ? rc : ensure(in->ctx, in->jstart, (size_t)(njc + 1) * 4);
    rc = rc ? rc : ensure(in->ctx, in->jrank, (size_t)outer->cap_entries * 4);
    rc = rc ? rc : ensure(in->ctx, in->fj, (size_t)outer->cap_rows * g->nn * 12);
    rc = rc ? rc : ensure(in->ctx, in->fi, (size_t)outer->cap_items * g->m * 16);
    if (rc) return rc;
    if (in->jcount.p != old_jc || in->resv_nci != outer->resv_nci)
        MXN_HIP(hipMemsetAsync(in->jcount.p, 0, (size_t)(njc + 1) * 4, st));
    if (in->totals.p != old_tot) MXN_HIP(hipMemsetAsync(in->totals.p, 0, 16, st));
    in->grid = g;
    in->grid_generation = outer->grid_generation;
    in->rlist = r;
    in->rbb = outer->rbb;
    in->cap_entries = outer->cap_entries;
    in->cap_items = outer->cap_items;
    in->resv_parts = outer->resv_parts;
    in->resv_nci = outer->resv_nci;
    in->last_entries = outer->last_entries;
    in->est_items = outer->est_items;
    in->cap_rows = outer->cap_rows;
    in->resv_size = outer->resv_size;
    in->sci_valid = false;
    MXN_HIP(hipMemcpyAsync(in->part_start.p, outer->part_start.p, (size_t)(nregions + 1) * 4, hipMemcpyDeviceToDevice,
                           st));
    PruneArgs a{};
    a.nslots = (const int *)g->nslots.p;
    a.xs_now = (const float4 *)g->xs_now.p;
    a.perm = (const int *)g->perm.p;
    a.part_start = (const int *)outer->part_start.p;
    a.part_count_in = (const int *)outer->part_count.p;
    a.totals_in = (const int *)outer->totals.p;
    a.in = (const nb_jentry *)outer->entries.p;
    a.part_count = (int *)in->part_count.p;
    a.out = (nb_jentry *)in->entries.p;
    a.jcount = (int *)in->jcount.p;
    a.jrank = (int *)in->jrank.p;
    a.region_overflow = (int *)in->totals.p + 3;
    a.Lx = g->Lf[0]; a.Ly = g->Lf[1]; a.Lz = g->Lf[2];
    volatile float r2 = r * r;
    a.r2 = r2;
    a.nregions = nregions;
    a.parts = outer->resv_parts;
    const int nb = (nregions + 3) / 4;
    if (g->m == 4 && g->nn == 4) k_prune<4, 4><<<nb, 256, 0, st>>>(a);
    else if (g->m == 4 && g->nn == 8) k_prune<4, 8><<<nb, 256, 0, st>>>(a);
    else if (g->m == 8 && g->nn == 4) k_prune<8, 4><<<nb, 256, 0, st>>>(a);
    else k_prune<8, 8><<<nb, 256, 0, st>>>(a);
    finish_list(in, nregions, st);
    finish_rows(in, nregions, outer->resv_parts, st);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

}  // namespace mxn
