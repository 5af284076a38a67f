// Exact missed-pair recount for the Verlet-buffer study (Sec. 5 "Effective
// pair list buffering" and the appendix's drift model).
//
// The list is built once at a large radius rl from the undisplaced positions
// with the bounding-box shortcut radius rl - c.  For any smaller list radius
// r'_l = rc + r_b the same cluster pair is listed iff its threshold
//     tau = min(d_bb + c, d_min)
// is below r'_l, where d_bb is its bounding-box distance and d_min the
// smallest distance of its real particle pairs (both at sort time).  A
// non-excluded pair of that cluster pair is missed at buffer r_b iff
// tau >= rc + r_b and its displaced distance is below rc; it then adds its
// shifted pair potential V(r_t) - V(rc) (LJ + Ewald real-space Coulomb) to the
// missed energy.  The kernel bins every such contribution by
// k = floor((tau - rc)/db), so that E(k db) = sum over bins k' >= k.
#include "ewald_fit.h"
#include "internal.h"

namespace {

struct RecountArgs {
    const int *perm, *type_s;
    const float4 *xs, *xs_now;
    const float4 *bbi_lo, *bbi_hi, *bbj_lo, *bbj_hi;
    const int4 *items;
    const nb_jentry *entries;
    const int *totals;
    const float4 *shiftvec;
    const float *c6c12;
    int nt;
    float rc, rc2, beta, c_exp, coulomb_f, shiftC, rc6inv, c_bb, db;
    int nbins;
    double *hist;
};

__device__ inline float sq3(float x, float y, float z) { return (x * x + y * y) + z * z; }

__device__ inline float axis_gap(float jlo, float jhi, float ilo, float ihi) {
    float d1 = jlo - ihi, d2 = ilo - jhi;
    float m = d1 > d2 ? d1 : d2;
    return m > 0.0f ? m : 0.0f;
}

template <int M, int N>
__global__ __launch_bounds__(256) void k_recount(RecountArgs a) {
    __shared__ float4 svec[32];
    extern __shared__ float4 ljt[];
    for (int t = threadIdx.x; t < 27; t += blockDim.x) svec[t] = a.shiftvec[t];
    for (int t = threadIdx.x; t < a.nt * a.nt; t += blockDim.x) {
        const float c6 = a.c6c12[2 * t], c12 = a.c6c12[2 * t + 1];
        ljt[t] = make_float4(c6, c12, c12 * a.rc6inv * a.rc6inv - c6 * a.rc6inv, 0.0f);
    }
    __syncthreads();
    constexpr int B = 64 / N;
    constexpr unsigned FULL = (1u << M) - 1u;
    const int lane = threadIdx.x & 63;
    const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= a.totals[2]) return;
    const int4 it = a.items[item];
    const int ci = __builtin_amdgcn_readfirstlane(it.x);
    const int js = __builtin_amdgcn_readfirstlane(it.y);
    const int je = __builtin_amdgcn_readfirstlane(it.z);
    float x0[M], y0[M], z0[M], xt[M], yt[M], zt[M], qi[M];
    int ti[M];
    bool ireal[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const float4 p0 = a.xs[ci * M + k], pt = a.xs_now[ci * M + k];
        x0[k] = p0.x; y0[k] = p0.y; z0[k] = p0.z;
        xt[k] = pt.x; yt[k] = pt.y; zt[k] = pt.z;
        qi[k] = pt.w * a.coulomb_f;
        const int t = a.type_s[ci * M + k];
        ti[k] = (t < 0 ? 0 : (t >= a.nt ? a.nt - 1 : t)) * a.nt;
        ireal[k] = a.perm[ci * M + k] >= 0;
    }
    const float4 ilo = a.bbi_lo[ci], ihi = a.bbi_hi[ci];
    const int jb = lane % N, eo = lane / N;
    for (int e0 = js; e0 < je; e0 += B) {
        const int e = e0 + eo;
        const bool valid = e < je;
        const nb_jentry en = a.entries[valid ? e : e0];
        const int jslot = en.cj * N + jb;
        const float4 pj0 = a.xs[jslot], pjt = a.xs_now[jslot];
        const float4 sv = svec[en.shift];
        const bool jreal = a.perm[jslot] >= 0;
        // cluster-pair threshold from the sort-time geometry
        const float4 jl = a.bbj_lo[en.cj], jh = a.bbj_hi[en.cj];
        const float d2bb = sq3(axis_gap(jl.x, jh.x, ilo.x + sv.x, ihi.x + sv.x),
                               axis_gap(jl.y, jh.y, ilo.y + sv.y, ihi.y + sv.y),
                               axis_gap(jl.z, jh.z, ilo.z + sv.z, ihi.z + sv.z));
        float m2 = INFINITY;
#pragma unroll
        for (int k = 0; k < M; ++k)
            if (ireal[k] && jreal) m2 = fminf(m2, sq3(x0[k] + sv.x - pj0.x, y0[k] + sv.y - pj0.y, z0[k] + sv.z - pj0.z));
#pragma unroll
        for (int o = 1; o < N; o <<= 1) m2 = fminf(m2, __shfl_xor(m2, o, 64));   // over the entry's N lanes
        const float tau = fminf(sqrtf(d2bb) + a.c_bb, sqrtf(m2));
        int kb = (int)floorf((tau - a.rc) / a.db);
        if (!valid || kb < 0) continue;   // listed even without a buffer: never missed
        if (kb >= a.nbins) kb = a.nbins - 1;
        const unsigned long long m64 = ((unsigned long long)en.mhi << 32) | en.mlo;
        const unsigned mb = (unsigned)(m64 >> (jb * M)) & FULL;
        unsigned act = FULL;
        if (en.shift == 13) {
            const int t = jslot - ci * M;
            act = t >= M ? FULL : (t <= 0 ? 0u : (1u << t) - 1u);
        }
        const unsigned use = act & mb;   // real, non-excluded pairs of the half list
        const int tj = min(max(a.type_s[jslot], 0), a.nt - 1);
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            if (!((use >> k) & 1u)) continue;
            const float dx = xt[k] + sv.x - pjt.x, dy = yt[k] + sv.y - pjt.y, dz = zt[k] + sv.z - pjt.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 < a.rc2)) continue;
            const float rinv = __builtin_amdgcn_rsqf(r2);
            const float rinv2 = rinv * rinv;
            const float u = r2 * rinv * a.beta;
            const float ex = __builtin_amdgcn_exp2f(a.c_exp * r2);
            const float P = fmaf(fmaf(fmaf(MXN_EWALD_P3, u, MXN_EWALD_P2), u, MXN_EWALD_P1), u, MXN_EWALD_P0);
            const float Q = fmaf(fmaf(fmaf(fmaf(MXN_EWALD_Q4, u, MXN_EWALD_Q3), u, MXN_EWALD_Q2), u, MXN_EWALD_Q1), u,
                                 1.0f);
            const float erfcv = ex * P * __builtin_amdgcn_rcpf(Q);
            const float4 lj = ljt[ti[k] + tj];
            const float rinv6 = rinv2 * rinv2 * rinv2;
            acc += lj.y * rinv6 * rinv6 - lj.x * rinv6 - lj.z + qi[k] * pjt.w * (erfcv * rinv - a.shiftC);
        }
        if (acc != 0.0f) unsafeAtomicAdd(a.hist + kb, (double)acc);
    }
}

__global__ void k_zero_d(double *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace

namespace mxn {


int launch_recount(nb_ctx *ctx, const nb_grid *g, const nb_list *l, const float *xyzq_t, const nb_params *p, float c_bb,
                   float db, int nbins, double *hist) {
    hipStream_t st = ctx->stream;
    k_zero_d<<<(nbins + 255) / 256, 256, 0, st>>>(hist, nbins);
    int rc = launch_gather(ctx, g, xyzq_t, p->ntypes);
    if (rc) return rc;
    RecountArgs a{};
    a.perm = (const int *)g->perm.p;
    a.type_s = (const int *)g->type_s.p;
    a.xs = (const float4 *)g->xs.p;
    a.xs_now = (const float4 *)g->xs_now.p;
    a.bbi_lo = (const float4 *)g->bbi_lo.p;
    a.bbi_hi = (const float4 *)g->bbi_hi.p;
    a.bbj_lo = (const float4 *)(g->nn == g->m ? g->bbi_lo.p : g->bbj_lo.p);
    a.bbj_hi = (const float4 *)(g->nn == g->m ? g->bbi_hi.p : g->bbj_hi.p);
    a.items = (const int4 *)l->items.p;
    a.entries = (const nb_jentry *)l->entries.p;
    a.totals = (const int *)l->totals.p;
    a.shiftvec = (const float4 *)g->shiftvec.p;
    a.c6c12 = p->c6c12;
    a.nt = p->ntypes;
    a.rc = p->rc;
    a.rc2 = p->rc * p->rc;
    a.beta = p->beta;
    a.c_exp = (float)(-(double)p->beta * (double)p->beta * 1.4426950408889634);
    a.coulomb_f = p->coulomb_f;
    a.shiftC = (float)(std::erfc((double)p->beta * p->rc) / (double)p->rc);
    a.rc6inv = (float)(1.0 / std::pow((double)p->rc, 6));
    a.c_bb = c_bb;
    a.db = db;
    a.nbins = nbins;
    a.hist = hist;
    const int nb = (int)((l->cap_items + 3) / 4) + 1;
    const size_t lds = (size_t)p->ntypes * p->ntypes * sizeof(float4);
    if (g->m == 4 && g->nn == 4) k_recount<4, 4><<<nb, 256, lds, st>>>(a);
    else if (g->m == 4 && g->nn == 8) k_recount<4, 8><<<nb, 256, lds, st>>>(a);
    else if (g->m == 8 && g->nn == 4) k_recount<8, 4><<<nb, 256, lds, st>>>(a);
    else k_recount<8, 8><<<nb, 256, lds, st>>>(a);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

}  // namespace mxn
