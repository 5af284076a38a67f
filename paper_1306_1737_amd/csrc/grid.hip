// Grid sort and bounding boxes (Sec. 2.3 "Pair list construction": x/y column
// grid, pigeonhole sort into columns, z order inside a column, dummy padding,
// per-cluster bounding boxes).
//
// This file is compiled with -ffp-contract=off: the wrapped coordinates, the
// column index and the bounding boxes are defined by separately rounded FP32
// operations and must be bit-reproducible.
#include <cmath>
#include <cstring>

#include "internal.h"
#include "scan.h"

namespace {

using mxn::scan_body;

constexpr int kImgBias = 512;

__device__ inline unsigned sortable(float z) {
    unsigned u = __float_as_uint(z);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

struct WrapArgs {
    const float4 *xyzq;
    int n;
    float Lx, Ly, Lz;
    double ilx, ily, ilz;
    float inv_x, inv_y;
    int nx, ny;
    int *col_count, *atom_col, *atom_img;
    float4 *atom_xw;
    int *flags;
};

__device__ inline float wrap1(float x, float L, double il, int &k, bool &bad) {
    double kd = floor((double)x * il);
    if (!(kd > -kImgBias && kd < kImgBias)) {   // also catches NaN
        bad = true;
        kd = 0.0;
    }
    k = (int)kd;
    float kl = (float)k * L;
    float w = x - kl;
    return w + 0.0f;   // -0 -> +0
}

// Column counting without global atomics (many particles share few columns,
// and same-address atomics serialise): each workgroup histograms its block of
// kHistAtoms particles in LDS and writes the histogram as one column of the
// matrix hist[column][block]; a per-column prefix over blocks then gives every
// block its offset inside each column, and the block places its particles
// with LDS atomics.  The placement order inside a column is arbitrary (the
// column sort ranks by z and index).
constexpr int kHistThreads = 1024;
constexpr int kColsPerBlock = 4;   // columns per workgroup of the per-column prefix (one wavefront each)

__device__ inline int wrap_column(const WrapArgs &a, int i) {
    float4 p = a.xyzq[i];
    bool bad = !(isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w));
    int kx, ky, kz;
    float wx = wrap1(p.x, a.Lx, a.ilx, kx, bad);
    float wy = wrap1(p.y, a.Ly, a.ily, ky, bad);
    float wz = wrap1(p.z, a.Lz, a.ilz, kz, bad);
    if (bad) atomicOr(a.flags, mxn::FLAG_NONFINITE);
    int cx = (int)floorf(wx * a.inv_x);
    int cy = (int)floorf(wy * a.inv_y);
    cx = cx < 0 ? 0 : (cx > a.nx - 1 ? a.nx - 1 : cx);
    cy = cy < 0 ? 0 : (cy > a.ny - 1 ? a.ny - 1 : cy);
    int col = cx * a.ny + cy;
    a.atom_col[i] = col;
    a.atom_img[i] = (kx + kImgBias) | ((ky + kImgBias) << 10) | ((kz + kImgBias) << 20);
    a.atom_xw[i] = make_float4(wx, wy, wz, p.w);
    return col;
}

// Kernel bodies take their workgroup index `blk` explicitly: the
// single-system kernels pass blockIdx.x, the batched ones the index within
// their replica's share of the grid.
__device__ inline void wrap_hist_body(const WrapArgs &a, int ncol, int nhb, int *hist, int blk) {
    extern __shared__ int h[];
    for (int c = threadIdx.x; c < ncol; c += kHistThreads) h[c] = 0;
    __syncthreads();
    const int b0 = blk * mxn::kHistAtoms, b1 = min(a.n, b0 + mxn::kHistAtoms);
    for (int i = b0 + threadIdx.x; i < b1; i += kHistThreads) atomicAdd(&h[wrap_column(a, i)], 1);
    __syncthreads();
    for (int c = threadIdx.x; c < ncol; c += kHistThreads) hist[(long)c * nhb + blk] = h[c];
}

__global__ __launch_bounds__(kHistThreads) void k_wrap_hist(WrapArgs a, int ncol, int nhb, int *hist) {
    wrap_hist_body(a, ncol, nhb, hist, blockIdx.x);
}

// per column: counts over blocks -> exclusive offsets per block, total count
__device__ inline void col_prefix_body(int ncol, int nhb, int *hist, int *col_count, int blk) {
    // one wavefront per column (kColsPerBlock per workgroup of 256): a wavefront scan over the blocks
    const int lane = threadIdx.x & 63;
    const int c = blk * kColsPerBlock + (threadIdx.x >> 6);
    if (c >= ncol) return;
    int *row = hist + (long)c * nhb;
    int carry = 0;
    for (int b0 = 0; b0 < nhb; b0 += 64) {
        const int b = b0 + lane;
        const int v = b < nhb ? row[b] : 0;
        int incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (b < nhb) row[b] = carry + incl - v;
        carry += __shfl(incl, 63, 64);
    }
    if (lane == 0) col_count[c] = carry;
}

__global__ void k_col_prefix(int ncol, int nhb, int *hist, int *col_count) {
    col_prefix_body(ncol, nhb, hist, col_count, blockIdx.x);
}

__device__ inline void bucket_hist_body(int n, int ncol, int nhb, const int *atom_col, const int *col_start,
                                        const int *hist, int *bucket, int blk) {
    extern __shared__ int off[];
    for (int c = threadIdx.x; c < ncol; c += kHistThreads) off[c] = col_start[c] + hist[(long)c * nhb + blk];
    __syncthreads();
    const int b0 = blk * mxn::kHistAtoms, b1 = min(n, b0 + mxn::kHistAtoms);
    for (int i = b0 + threadIdx.x; i < b1; i += kHistThreads) bucket[atomicAdd(&off[atom_col[i]], 1)] = i;
}

__global__ __launch_bounds__(kHistThreads) void k_bucket_hist(int n, int ncol, int nhb, const int *atom_col,
                                                             const int *col_start, const int *hist, int *bucket) {
    bucket_hist_body(n, ncol, nhb, atom_col, col_start, hist, bucket, blockIdx.x);
}

// per particle: periodic wrap, image count, column, column histogram by
// global atomics (the path for grids with more columns than fit in LDS)
__global__ void k_wrap_count(WrapArgs a) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    atomicAdd(&a.col_count[wrap_column(a, i)], 1);
}

// scatter particle indices into their column's slot range (arbitrary order within a column)
__global__ void k_bucket(int n, const int *atom_col, const int *col_start, int *col_fill, int *bucket) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = atom_col[i];
    int pos = atomicAdd(&col_fill[c], 1);
    bucket[col_start[c] + pos] = i;
}

struct SortArgs {
    const int *col_count, *col_start, *bucket, *type, *atom_img;
    const float4 *atom_xw;
    float4 *xs, *xs_now, *colbb;
    int *type_s, *perm, *img_s, *slot_of;
    int *flags;
    int m, nn;                                   // i- and j-cluster sizes
    float4 *bbi_lo, *bbi_hi, *bbj_lo, *bbj_hi;   // cluster bounding boxes
};

// Bounding box of each cluster of `size` slots among clusters [c0, c1), one thread per cluster
// (dummies skipped: a cluster of dummies only keeps the empty box, lo = +inf, hi = -inf).  lo.w carries
// the bit pattern of the cluster's real-slot mask (bit k: slot k holds a particle), so the pair search
// reads which slots are real with the box instead of loading the permutation; hi.w is 0.
__device__ inline void cluster_boxes(const float4 *xs, const int *perm, int size, int c0, int c1, float4 *lo,
                                     float4 *hi, int t, int nt) {
    for (int cl = c0 + t; cl < c1; cl += nt) {
        float4 l = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
        float4 h = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
        unsigned real = 0;
        for (int s = cl * size; s < cl * size + size; ++s) {
            if (perm[s] < 0) continue;
            real |= 1u << (s - cl * size);
            const float4 p = xs[s];
            l.x = fminf(l.x, p.x); l.y = fminf(l.y, p.y); l.z = fminf(l.z, p.z);
            h.x = fmaxf(h.x, p.x); h.y = fmaxf(h.y, p.y); h.z = fmaxf(h.z, p.z);
        }
        l.w = __uint_as_float(real);
        lo[cl] = l;
        hi[cl] = h;
    }
}

// One workgroup per column: rank every particle by (z, original index) among
// the column's particles (keys streamed through LDS in tiles), write the
// sorted slot arrays, pad with dummies, reduce the column's x/y extent and
// form the bounding boxes of the column's clusters (column starts are
// multiples of both cluster sizes, so no cluster straddles two columns).
constexpr int kSortThreads = 256;
constexpr int kSortTile = 1024;

__device__ inline void col_sort_body(const SortArgs &a, int c) {
    __shared__ unsigned long long tile[kSortTile];
    __shared__ float red[4][kSortThreads];
    const int tid = threadIdx.x;
    const int start = a.col_start[c], nc = a.col_count[c], end = a.col_start[c + 1];
    float mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
    for (int mine = 0; mine < nc; mine += kSortThreads) {
        int j = mine + tid;
        unsigned long long key = ~0ull;
        int orig = -1, t = 0, img = 0;
        float4 p = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (j < nc) {   // everything the particle's slot needs, loaded before the ranking
            orig = a.bucket[start + j];
            p = a.atom_xw[orig];
            t = a.type[orig];
            img = a.atom_img[orig];
            key = ((unsigned long long)sortable(p.z) << 32) | (unsigned)orig;
        }
        int rank = 0;
        if (nc <= kSortThreads) {   // one pass holds the column: the tile is the threads' own keys
            tile[tid] = key;
            __syncthreads();
            if (j < nc)
                for (int k = 0; k < nc; ++k) rank += tile[k] < key;
        } else {
            for (int t0 = 0; t0 < nc; t0 += kSortTile) {
                __syncthreads();
                for (int k = tid; k < kSortTile && t0 + k < nc; k += kSortThreads) {
                    int o = a.bucket[start + t0 + k];
                    tile[k] = ((unsigned long long)sortable(a.atom_xw[o].z) << 32) | (unsigned)o;
                }
                __syncthreads();
                int lim = nc - t0 < kSortTile ? nc - t0 : kSortTile;
                if (j < nc)
                    for (int k = 0; k < lim; ++k) rank += tile[k] < key;
            }
        }
        if (j < nc) {
            int slot = start + rank;
            a.xs[slot] = p;
            a.xs_now[slot] = p;
            if (t < 0) atomicOr(a.flags, mxn::FLAG_TYPE);   // reported by nb_sync; -1 marks dummies
            a.type_s[slot] = max(t, 0);
            a.perm[slot] = orig;
            a.img_s[slot] = img;
            a.slot_of[orig] = slot;
            mnx = fminf(mnx, p.x); mny = fminf(mny, p.y);
            mxx = fmaxf(mxx, p.x); mxy = fmaxf(mxy, p.y);
        }
    }
    // dummies: no charge, type -1 (the kernels skip them), distinct far positions
    for (int slot = start + nc + tid; slot < end; slot += kSortThreads) {
        float4 d = make_float4(-1000.0f - 4.0f * (float)(slot & 1023), -1000.0f - 4.0f * (float)((slot >> 10) & 1023),
                               -1000.0f - 4.0f * (float)(slot >> 20), 0.0f);
        a.xs[slot] = d;
        a.xs_now[slot] = d;
        a.type_s[slot] = -1;
        a.perm[slot] = -1;
        a.img_s[slot] = kImgBias | (kImgBias << 10) | (kImgBias << 20);
    }
    red[0][tid] = mnx; red[1][tid] = mny; red[2][tid] = mxx; red[3][tid] = mxy;
    __syncthreads();
    for (int s = kSortThreads / 2; s > 0; s >>= 1) {
        if (tid < s) {
            red[0][tid] = fminf(red[0][tid], red[0][tid + s]);
            red[1][tid] = fminf(red[1][tid], red[1][tid + s]);
            red[2][tid] = fmaxf(red[2][tid], red[2][tid + s]);
            red[3][tid] = fmaxf(red[3][tid], red[3][tid + s]);
        }
        __syncthreads();
    }
    if (tid == 0) a.colbb[c] = make_float4(red[0][0], red[1][0], red[2][0], red[3][0]);
    // the slots written above are visible to the workgroup after the reduction's barriers
    cluster_boxes(a.xs, a.perm, a.m, start / a.m, end / a.m, a.bbi_lo, a.bbi_hi, tid, kSortThreads);
    if (a.nn != a.m) cluster_boxes(a.xs, a.perm, a.nn, start / a.nn, end / a.nn, a.bbj_lo, a.bbj_hi, tid, kSortThreads);
}

__global__ __launch_bounds__(kSortThreads) void k_col_sort(SortArgs a) { col_sort_body(a, blockIdx.x); }

__device__ inline void shiftvec_body(float4 *sv, float Lx, float Ly, float Lz) {
    int s = threadIdx.x;
    if (s < 27) sv[s] = make_float4((float)(s / 9 - 1) * Lx, (float)((s / 3) % 3 - 1) * Ly, (float)(s % 3 - 1) * Lz, 0.0f);
}

// Column starts (an exclusive scan of the column counts, each rounded up to a multiple of cmax; total
// into nslots) and the 27 image shift vectors, in one workgroup.
__global__ __launch_bounds__(1024) void k_col_scan(const int *col_count, int *col_start, int ncol, int cmax,
                                                   int *nslots, float4 *sv, float Lx, float Ly, float Lz) {
    shiftvec_body(sv, Lx, Ly, Lz);
    scan_body(col_count, col_start, ncol, 1, cmax, nslots, nullptr);
}


__global__ void k_fill_int(int *p, int n, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}


// --------------------------------------------------------------------------
// Batched grid sort: every stage is one launch over all replicas.  A stage's
// workgroups are the concatenation of the replicas' shares; a workgroup finds
// its replica by binary search in the stage's prefix of share sizes.

struct GridJob {
    WrapArgs w;
    SortArgs s;
    int ncol, nhb, cmax, m, nn, slots_cap;
    int *col_hist, *col_start, *nslots;
    float4 *shiftvec;
};

__device__ inline int job_of(const int *off, int n, int b) {
    int lo = 0, hi = n - 1;   // last r with off[r] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// stage offsets: off + stage * (n + 1)
enum { GS_HIST, GS_PREFIX, GS_SCAN, GS_COLSORT, GS_NSTAGES };

__global__ __launch_bounds__(kHistThreads) void kb_wrap_hist(const GridJob *J, const int *off, int n) {
    const int r = job_of(off, n, blockIdx.x);
    const GridJob &j = J[r];
    wrap_hist_body(j.w, j.ncol, j.nhb, j.col_hist, blockIdx.x - off[r]);
}

__global__ void kb_col_prefix(const GridJob *J, const int *off, int n) {
    const int r = job_of(off, n, blockIdx.x);
    const GridJob &j = J[r];
    col_prefix_body(j.ncol, j.nhb, j.col_hist, j.w.col_count, blockIdx.x - off[r]);
}

__global__ __launch_bounds__(1024) void kb_col_scan(const GridJob *J) {
    const GridJob &j = J[blockIdx.x];
    shiftvec_body(j.shiftvec, j.w.Lx, j.w.Ly, j.w.Lz);
    scan_body(j.w.col_count, j.col_start, j.ncol, 1, j.cmax, j.nslots, nullptr);
}

__global__ __launch_bounds__(kHistThreads) void kb_bucket_hist(const GridJob *J, const int *off, int n) {
    const int r = job_of(off, n, blockIdx.x);
    const GridJob &j = J[r];
    bucket_hist_body(j.w.n, j.ncol, j.nhb, j.w.atom_col, j.col_start, j.col_hist, const_cast<int *>(j.s.bucket),
                     blockIdx.x - off[r]);
}

__global__ __launch_bounds__(kSortThreads) void kb_col_sort(const GridJob *J, const int *off, int n) {
    const int r = job_of(off, n, blockIdx.x);
    col_sort_body(J[r].s, blockIdx.x - off[r]);
}

__global__ __launch_bounds__(1024) void kb_scan(const mxn::ScanJob *J) {
    const mxn::ScanJob &j = J[blockIdx.x];
    scan_body(j.in, j.out, j.n, j.mode, j.p, j.total, j.raw_total, j.clear);
}

inline int blocks(long n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

namespace mxn {


static WrapArgs make_wrap(const nb_grid *g, const float *xyzq) {
    return WrapArgs{(const float4 *)xyzq, g->n, g->Lf[0], g->Lf[1], g->Lf[2], g->invL[0], g->invL[1], g->invL[2],
                    g->inv_x, g->inv_y, g->nx, g->ny, (int *)g->col_count.p, (int *)g->atom_col.p,
                    (int *)g->atom_img.p, (float4 *)g->atom_xw.p, g->ctx->d_flags};
}

static SortArgs make_sort(const nb_grid *g, const int *type) {
    return SortArgs{(const int *)g->col_count.p, (const int *)g->col_start.p, (const int *)g->bucket.p, type,
                    (const int *)g->atom_img.p, (const float4 *)g->atom_xw.p, (float4 *)g->xs.p, (float4 *)g->xs_now.p,
                    (float4 *)g->colbb.p, (int *)g->type_s.p, (int *)g->perm.p, (int *)g->img_s.p,
                    (int *)g->slot_of.p, g->ctx->d_flags, g->m, g->nn, (float4 *)g->bbi_lo.p, (float4 *)g->bbi_hi.p,
                    (float4 *)g->bbj_lo.p, (float4 *)g->bbj_hi.p};
}

size_t grid_job_size() { return sizeof(GridJob); }
int grid_job_stages() { return GS_NSTAGES; }

bool grid_batchable(const nb_grid *g) { return g->ncol <= kMaxHistColumns; }

void fill_grid_job(void *out, const nb_grid *g, const float *xyzq, const int *type) {
    GridJob j{};
    j.w = make_wrap(g, xyzq);
    j.s = make_sort(g, type);
    j.ncol = g->ncol;
    j.nhb = hist_blocks(g->n);
    j.cmax = g->cmax;
    j.m = g->m;
    j.nn = g->nn;
    j.slots_cap = g->slots_cap;
    j.col_hist = (int *)g->col_hist.p;
    j.col_start = (int *)g->col_start.p;
    j.nslots = (int *)g->nslots.p;
    j.shiftvec = (float4 *)g->shiftvec.p;
    std::memcpy(out, &j, sizeof j);
}

// workgroups of one replica in each batched stage (the histogram stages share GS_HIST)
void grid_job_blocks(const nb_grid *g, int *blocks_per_stage) {
    blocks_per_stage[GS_HIST] = hist_blocks(g->n);
    blocks_per_stage[GS_PREFIX] = blocks(g->ncol, kColsPerBlock);
    blocks_per_stage[GS_SCAN] = 1;
    blocks_per_stage[GS_COLSORT] = g->ncol;
}

// off: DEVICE int[GS_NSTAGES * (n_rep + 1)], each stage's exclusive prefix of the
// replicas' workgroups; total: HOST int[GS_NSTAGES] workgroups per stage
int launch_grid_sort_batch(hipStream_t st, const void *jobs, const int *off, int n_rep, const int *total,
                           int max_ncol) {
    const GridJob *J = (const GridJob *)jobs;
    const int *o = off;
    const int stride = n_rep + 1;
    const size_t hb = (size_t)max_ncol * sizeof(int);
    kb_wrap_hist<<<total[GS_HIST], kHistThreads, hb, st>>>(J, o + GS_HIST * stride, n_rep);
    kb_col_prefix<<<total[GS_PREFIX], 256, 0, st>>>(J, o + GS_PREFIX * stride, n_rep);
    kb_col_scan<<<n_rep, 1024, 0, st>>>(J);
    kb_bucket_hist<<<total[GS_HIST], kHistThreads, hb, st>>>(J, o + GS_HIST * stride, n_rep);
    kb_col_sort<<<total[GS_COLSORT], kSortThreads, 0, st>>>(J, o + GS_COLSORT * stride, n_rep);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

// one exclusive scan per job, one workgroup each
void launch_scan_batch(const ScanJob *jobs, int n_jobs, hipStream_t st) { kb_scan<<<n_jobs, 1024, 0, st>>>(jobs); }

int launch_grid_sort(nb_grid *g, const float *xyzq, const int *type) {
    hipStream_t st = g->ctx->stream;
    const int n = g->n, ncol = g->ncol;
    const WrapArgs w = make_wrap(g, xyzq);
    const bool lds_hist = ncol <= kMaxHistColumns;
    const int nhb = hist_blocks(n);
    const size_t hb = (size_t)ncol * sizeof(int);
    if (lds_hist) {
        k_wrap_hist<<<nhb, kHistThreads, hb, st>>>(w, ncol, nhb, (int *)g->col_hist.p);
        k_col_prefix<<<blocks(ncol, kColsPerBlock), 256, 0, st>>>(ncol, nhb, (int *)g->col_hist.p,
                                                                   (int *)g->col_count.p);
    } else {
        k_fill_int<<<blocks(ncol, 256), 256, 0, st>>>((int *)g->col_count.p, ncol, 0);
        k_wrap_count<<<blocks(n, 256), 256, 0, st>>>(w);
    }
    k_col_scan<<<1, 1024, 0, st>>>((const int *)g->col_count.p, (int *)g->col_start.p, ncol, g->cmax,
                                   (int *)g->nslots.p, (float4 *)g->shiftvec.p, g->Lf[0], g->Lf[1], g->Lf[2]);
    if (lds_hist) {
        k_bucket_hist<<<nhb, kHistThreads, hb, st>>>(n, ncol, nhb, (const int *)g->atom_col.p,
                                                     (const int *)g->col_start.p, (const int *)g->col_hist.p,
                                                     (int *)g->bucket.p);
    } else {
        k_fill_int<<<blocks(ncol, 256), 256, 0, st>>>((int *)g->col_fill.p, ncol, 0);
        k_bucket<<<blocks(n, 256), 256, 0, st>>>(n, (const int *)g->atom_col.p, (const int *)g->col_start.p,
                                                 (int *)g->col_fill.p, (int *)g->bucket.p);
    }
    const SortArgs s = make_sort(g, type);
    k_col_sort<<<ncol, kSortThreads, 0, st>>>(s);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

}  // namespace mxn
