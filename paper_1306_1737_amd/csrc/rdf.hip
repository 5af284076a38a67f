// Pair distance histogram over a cluster-pair list: the pair correlation
// function, which Sec. 1 names as a limited-range pair evaluation like the
// forces.  Sec. 2.3: when the list is built for every evaluation the particle
// prune is skipped (a list built from bounding boxes, rbb = rlist), and for
// interactions this cheap the kernel needs no cut-off conditional.
//
// Work items as in the force kernel: a wavefront takes entries of one
// i-cluster, a lane one j-particle of one entry, and loops over the M
// i-particles (scalar registers).  Every lane forms its squared distance and
// bin without branching; only the count itself is predicated (real, active
// pair below r_max).  Counts go to a per-workgroup LDS histogram, flushed
// once with 64-bit atomics; integer sums, so the result is exact.
//
// The bin is decided in FP32 from r2 alone: e_k = (float)((k dr)^2) in FP64,
// bin k the largest with e_k <= r2 (a sqrt guess corrected by one step each
// way).  r2 is formed as the search forms its particle test (j moved back by
// the entry's image shift, separately rounded operations; this file is
// compiled with -ffp-contract=off).
#include <cmath>
#include <vector>

#include "internal.h"

namespace {

struct RdfArgs {
    const float4 *xs_now;   // slot positions at the evaluated time (gathered)
    const int *type_s;      // -1 for dummy slots
    const int4 *items;
    const nb_jentry *entries;
    const int *totals;      // [2]: usable work items
    const float4 *shiftvec;
    const float *edge;      // nbins + 1 squared bin edges
    unsigned long long *hist;
    int nbins, nt, skip_excl;
    float inv_dr;
};

template <int M, int N>
__global__ __launch_bounds__(256) void k_rdf(RdfArgs a) {
    constexpr int B = 64 / N;
    constexpr unsigned FULL = (1u << M) - 1u;
    extern __shared__ float4 smem[];
    float4 *svec = smem;                                         // 27 image shift vectors
    float *edge = reinterpret_cast<float *>(smem + 32);          // nbins + 1
    unsigned *h = reinterpret_cast<unsigned *>(edge + a.nbins + 1);
    const int nh = a.nt * a.nt * a.nbins;
    for (int t = threadIdx.x; t < 27; t += blockDim.x) svec[t] = a.shiftvec[t];
    for (int t = threadIdx.x; t <= a.nbins; t += blockDim.x) edge[t] = a.edge[t];
    for (int t = threadIdx.x; t < nh; t += blockDim.x) h[t] = 0u;
    __syncthreads();
    const float r2max = edge[a.nbins];
    const long total = a.totals[2];
    const int lane = threadIdx.x & 63, jb = lane % N, eo = lane / N;
    for (long item = (long)blockIdx.x * 4 + (threadIdx.x >> 6); item < total; item += (long)gridDim.x * 4) {
        const int4 it = a.items[item];
        const int ci = __builtin_amdgcn_readfirstlane(it.x);
        const int js = __builtin_amdgcn_readfirstlane(it.y);
        const int je = __builtin_amdgcn_readfirstlane(it.z);
        float xi[M], yi[M], zi[M];
        int ti[M];
        unsigned ireal = 0;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const float4 p = a.xs_now[ci * M + k];
            xi[k] = p.x; yi[k] = p.y; zi[k] = p.z;
            const int t = a.type_s[ci * M + k];
            ireal |= (t >= 0 ? 1u : 0u) << k;
            ti[k] = t < 0 ? 0 : (t >= a.nt ? a.nt - 1 : t);
        }
        for (int e0 = js; e0 < je; e0 += B) {
            const int e = e0 + eo;
            const bool valid = e < je;
            const nb_jentry en = a.entries[valid ? e : e0];
            const int jslot = en.cj * N + jb;
            const float4 pj = a.xs_now[jslot];
            const int tjr = a.type_s[jslot];
            const int tj = tjr < 0 ? 0 : (tjr >= a.nt ? a.nt - 1 : tjr);
            const float4 sv = svec[en.shift];
            const float xj = pj.x - sv.x, yj = pj.y - sv.y, zj = pj.z - sv.z;
            const unsigned long long m64 = ((unsigned long long)en.mhi << 32) | en.mlo;
            const unsigned mb = (unsigned)(m64 >> (jb * M)) & FULL;
            unsigned act = ireal;
            if (en.shift == 13) {   // self or overlapping cluster pair: only slot(i) < slot(j)
                const int t = jslot - ci * M;
                act &= t >= M ? FULL : (t <= 0 ? 0u : (1u << t) - 1u);
            }
            if (a.skip_excl) act &= mb;
            if (!valid || tjr < 0) act = 0u;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const float dx = xi[k] - xj, dy = yi[k] - yj, dz = zi[k] - zj;
                const float r2 = (dx * dx + dy * dy) + dz * dz;
                int bin = (int)(sqrtf(r2) * a.inv_dr);
                bin = bin < 0 ? 0 : (bin > a.nbins - 1 ? a.nbins - 1 : bin);
                bin -= edge[bin] > r2 ? 1 : 0;
                bin += (bin + 1 < a.nbins && !(edge[bin + 1] > r2)) ? 1 : 0;
                const int lo = ti[k] < tj ? ti[k] : tj, hi = ti[k] < tj ? tj : ti[k];
                if (((act >> k) & 1u) && r2 < r2max) atomicAdd(h + (lo * a.nt + hi) * a.nbins + bin, 1u);
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nh; t += blockDim.x)
        if (h[t]) atomicAdd(a.hist + t, (unsigned long long)h[t]);
}

}  // namespace

namespace mxn {

size_t rdf_lds_bytes(int nbins, int nt) { return 32 * 16 + (size_t)(nbins + 1) * 4 + (size_t)nt * nt * nbins * 4; }

int launch_rdf(nb_ctx *ctx, const nb_grid *g, const nb_list *l, float r_max, int nbins, int nt, int skip_excl,
               unsigned long long *hist) {
    hipStream_t st = ctx->stream;
    // squared bin edges e_k = (float)((k dr)^2), dr = r_max / nbins, in FP64 (rebuilt when they change)
    if (!ctx->rdf_edge.p || ctx->rdf_rmax != r_max || ctx->rdf_nbins != nbins) {
        std::vector<float> e((size_t)nbins + 1);
        const double dr = (double)r_max / nbins;
        for (int k = 0; k <= nbins; ++k) e[(size_t)k] = (float)((k * dr) * (k * dr));
        int rc = ensure(ctx, ctx->rdf_edge, e.size() * sizeof(float));
        if (rc) return rc;
        MXN_HIP(hipMemcpyAsync(ctx->rdf_edge.p, e.data(), e.size() * sizeof(float), hipMemcpyHostToDevice, st));
        MXN_HIP(hipStreamSynchronize(st));   // e is released on return
        ctx->rdf_rmax = r_max;
        ctx->rdf_nbins = nbins;
    }
    RdfArgs a{};
    a.xs_now = (const float4 *)g->xs_now.p;
    a.type_s = (const int *)g->type_s.p;
    a.items = (const int4 *)l->items.p;
    a.entries = (const nb_jentry *)l->entries.p;
    a.totals = (const int *)l->totals.p;
    a.shiftvec = (const float4 *)g->shiftvec.p;
    a.edge = (const float *)ctx->rdf_edge.p;
    a.hist = hist;
    a.nbins = nbins;
    a.nt = nt;
    a.skip_excl = skip_excl;
    a.inv_dr = (float)((double)nbins / (double)r_max);
    // persistent workgroups: enough to fill the GPU, each flushes its histogram once
    const long need = (l->cap_items + 3) / 4;
    const int nb = (int)std::max(1L, std::min(need, 2048L));
    const size_t lds = rdf_lds_bytes(nbins, nt);
    if (g->m == 4 && g->nn == 4) k_rdf<4, 4><<<nb, 256, lds, st>>>(a);
    else if (g->m == 4 && g->nn == 8) k_rdf<4, 8><<<nb, 256, lds, st>>>(a);
    else if (g->m == 8 && g->nn == 4) k_rdf<8, 4><<<nb, 256, lds, st>>>(a);
    else k_rdf<8, 8><<<nb, 256, lds, st>>>(a);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

}  // namespace mxn
