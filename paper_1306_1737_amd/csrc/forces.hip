// M x N cluster-pair force kernels (Sec. 3 "Pair interaction kernels"; Eq. 1
// Lennard-Jones, Eq. 2 Coulomb with the Ewald real-space correction; Sec. 2.4
// exclusions) plus the per-step coordinate gather and force scatter.
//
// Wavefront mapping on gfx950 (wave64): a wavefront owns one work item, i.e.
// up to 32 consecutive j-entries of one i-cluster.  Its M i-particles are
// wave-uniform (scalar registers); each of the 64 lanes owns one j-particle of
// one entry (64/N entries per pass) and loops over the M i-particles, so each
// lane evaluates M pair interactions per pass with no cross-lane traffic:
// j-forces stay in the lane and are added to memory once per entry with
// one store per entry into the entry's row of a buffer whose rows are grouped
// by j-cluster (the N lanes of an entry write one 12N-byte row); i-forces stay
// in registers for the whole item, are reduced across the wavefront once at
// its end and stored per item.  A second kernel sums each cluster's stored j-
// and i-forces in fixed point (exact, so order-independent) and writes them in
// input order, so no force goes through an atomic and the forces of a given
// list and positions are reproducible bit for bit.  The image shift is
// applied to the j-particle, so entries of different shifts can share a pass.
//
// Pair math (FP32): r^-1 from the hardware reciprocal square root;
// exp(-beta^2 r^2) from the hardware exp2; erfc(beta r) = exp(-beta^2 r^2) *
// P(u)/Q(u) with a project-fitted rational approximation of erfcx on [0, 4]
// (see fit_ewald.py).  Energies and the virial are accumulated per lane in
// FP64 (or FP32 for the precision study) and reduced deterministically.
#include <type_traits>

#include "devptr.h"
#include "ewald_fit.h"
#include "internal.h"

namespace {

constexpr int kNAcc = 11;   // per work item: E_LJ, E_Coulomb, virial[9]

// Per-system arrays a work item touches (one system, or one replica of a batch),
// as global pointers (see devptr.h).
using mxn::gptr;
using mxn::ld;

struct SysView {
    gptr<const float4> xs_now;
    gptr<const int> type_s;
    gptr<float> fj;        // j-force (x, y, z) per (row, j-particle)
    gptr<float4> fi;       // i-force per (item, i-particle)
    gptr<const int> jpos;  // row of each entry position
    gptr<const int4> items;
    gptr<const nb_jentry> entries;
    gptr<double> partials;
    long pstride, pbase;   // partial of item i, value k: partials[k * pstride + pbase + i]
};

__device__ inline SysView make_view(const float4 *xs_now, const int *type_s, float *fj, float4 *fi, const int *jpos,
                                    const int4 *items, const nb_jentry *entries, double *partials, long pstride,
                                    long pbase) {
    return SysView{(gptr<const float4>)xs_now, (gptr<const int>)type_s, (gptr<float>)fj,
                   (gptr<float4>)fi,           (gptr<const int>)jpos,   (gptr<const int4>)items,
                   (gptr<const nb_jentry>)entries, (gptr<double>)partials, pstride, pbase};
}

struct ForceArgs {
    const int *nslots, *perm, *img_s, *slot_of, *type_s;
    const float4 *xyzq_now;
    float4 *xs_now;
    float *fj;         // j-force (x, y, z) per (row, j-particle)
    float4 *fi;        // i-force per (item, i-particle)
    const int *jstart, *jpos, *part_istart;   // first row of each j-cluster, row of each entry; first item of each region
    double *blockpart;   // energy reduction: per-share sums [kNAcc][kReduceParts]
    double *energy, *virial;
    int ener, vir;
    int parts;         // regions per i-cluster
    int sci;           // i-clusters per work-item group of the fold's i-forces (super-cluster kernel), else 1
    int n;
    const int4 *items;
    const nb_jentry *entries;
    const int *totals;
    const float4 *shiftvec;
    const float *c6c12;
    int nt, shift_en;
    float rc2, beta, c_exp, c2bpi, coulomb_f, shiftC, rc6inv;
    float ep[4], eq[5];   // erfc(beta r) exp(beta^2 r^2) = P(r) / Q(r): the fit's coefficients times beta^k
    // Coulomb variant: 0 Ewald (rational erfc), 1 reaction field, 2 Ewald from a table
    int elec;
    float krf, k2rf, crf;      // reaction field: k, 2k, c
    const float2 *etab;        // Ewald table: (G, H) at r = i / tab_scale, i < ntab
    int ntab;
    float tab_scale;
    float Lx, Ly, Lz;
    double *partials;
    float *f_out;
    int accumulate;
    int *flags;
    long pstride;     // partials layout: [kNAcc][pstride]
};

// A particle's position at the evaluated time moved by the periodic image its
// slot was sorted with (packed image offsets, 10 bits per axis, biased by 512):
// x - (float)k * L with the product and the difference rounded separately,
// the definition the list's particle tests are checked against (a contracted
// multiply-add differs once k * L is inexact, for inputs many boxes away).
__device__ inline float4 apply_image(float4 p, int im, float Lx, float Ly, float Lz) {
    p.x = __fsub_rn(p.x, __fmul_rn((float)((im & 1023) - 512), Lx));
    p.y = __fsub_rn(p.y, __fmul_rn((float)(((im >> 10) & 1023) - 512), Ly));
    p.z = __fsub_rn(p.z, __fmul_rn((float)(((im >> 20) & 1023) - 512), Lz));
    return p;
}

__global__ void k_gather(ForceArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= *a.nslots) return;
    const int o = a.perm[s];
    if (o >= 0) {
        const float4 p = a.xyzq_now[o];
        if (!(isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w))) atomicOr(a.flags, mxn::FLAG_NONFINITE);
        if (a.nt > 0 && a.type_s[s] >= a.nt) atomicOr(a.flags, mxn::FLAG_TYPE);
        a.xs_now[s] = apply_image(p, a.img_s[s], a.Lx, a.Ly, a.Lz);
    }
}

template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the 64 lanes with DPP row shifts (prefix sums inside each row of
// 16 lanes) and row broadcasts; the total ends up in lane 63.
__device__ inline float wave_sum_dpp(float v) {
    int x = __float_as_int(v);
    x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true)));
    x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true)));
    x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true)));
    x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true)));
    x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false)));
    x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false)));
    return __int_as_float(x);
}

// Per-type-pair table in LDS: row 1 + ti*nt + tj = (6 C6, 12 C12, 12 x LJ
// shift at rc, Coulomb shift at rc), and the all-zero row 0 that a pair with a
// clear mask bit (excluded) reads instead, so the pair math needs no per-term
// selects for it.  The kernels address rows by byte offset (row x 16).  The LJ energy is accumulated as 12 V_LJ and
// scaled once per work item (kLJScale).
constexpr double kLJScale = 1.0 / 12.0;

__device__ inline void fill_ljt(const ForceArgs &a, float4 *ljt) {
    for (int t = threadIdx.x; t <= a.nt * a.nt; t += blockDim.x) {
        if (t == 0) {
            ljt[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            continue;
        }
        const float c6 = a.c6c12[2 * (t - 1)], c12 = a.c6c12[2 * (t - 1) + 1];
        const float sh = a.shift_en ? c12 * a.rc6inv * a.rc6inv - c6 * a.rc6inv : 0.0f;
        ljt[t] = make_float4(6.0f * c6, 12.0f * c12, 12.0f * sh, a.shiftC);
    }
}

// Byte offset of the LJ row of i-type ti (clamped to the table) and j-row offset of j-type tj.
__device__ inline int lj_ioff(const ForceArgs &a, int ti) {
    return (1 + (ti < 0 ? 0 : (ti >= a.nt ? a.nt - 1 : ti)) * a.nt) * 16;
}
__device__ inline int lj_joff(const ForceArgs &a, int tj) {
    return min(max(tj, 0), a.nt - 1) * 16;
}

// The rational erfc fit in powers of r (ForceArgs::ep, eq).  p2 and q3 are
// held in vector registers for the whole work item: the Horner steps that
// start from them would otherwise read two scalar operands, which one VALU
// instruction cannot, and the compiler copies them again for every pair.
struct EwPoly {
    float p0, p1, p2, p3, q1, q2, q3, q4;
};
__device__ inline float in_vreg(float x) {
    float y;
    asm("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
    return y;
}
__device__ inline EwPoly ew_poly(const ForceArgs &a) {
    return {a.ep[0], a.ep[1], in_vreg(a.ep[2]), a.ep[3], a.eq[1], a.eq[2], in_vreg(a.eq[3]), a.eq[4]};
}

// Force factor F/r of one pair within the cut-off, and its energy terms
// added to el (12 x Lennard-Jones) and ec (Coulomb).  Coulomb variants
// (ELEC): 0 Ewald with erfc from a rational approximation; 1 reaction field,
// F/r = qq (e/r^3 - 2k), V = qq (e/r + k r^2 - c); 2 Ewald with
// F/r = qq (e/r^3 - G(r)) and V = qq (e/r - H(r) - e shift), where
// G = (erf(beta r)/r - 2 beta/sqrt(pi) exp(-beta^2 r^2)) / r^2 and
// H = erf(beta r)/r are smooth (finite at r = 0) and interpolated linearly
// from the LDS table; e = bit = 1 for an interacting pair, 0 for an
// excluded one (which keeps its Ewald correction and reads the all-zero
// LJ row).  ljoff: byte offset of the type pair's row of the LDS table.  Both terms are
// gathered as F/r = (qq T + B / r^6) / r^2 with T = r F_Coulomb / qq (1/r
// for plain Coulomb) and B = 12 C12 / r^6 - 6 C6; 12 V_LJ = (B - 6 C6) / r^6.
template <bool ENER, int ELEC>
__device__ inline float pair_term(const ForceArgs &a, const EwPoly &ew, const float4 *ljt, const float2 *tab, float r2,
                                  float qq, bool bit, int ljoff, float &el, float &ec) {
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rinv2 = rinv * rinv;
    float T, vc;
    if (ELEC == 0) {
        const float r = r2 * rinv;
        const float ex = __builtin_amdgcn_exp2f(a.c_exp * r2);
        // erfc(beta r) = exp(-beta^2 r^2) P(r) / Q(r)
        const float P = fmaf(fmaf(fmaf(ew.p3, r, ew.p2), r, ew.p1), r, ew.p0);
        const float Q = fmaf(fmaf(fmaf(fmaf(ew.q4, r, ew.q3), r, ew.q2), r, ew.q1), r, 1.0f);
        // erfc for an interacting pair, erfc - 1 = -erf(beta r) for an excluded one
        const float em = fmaf(ex * P, __builtin_amdgcn_rcpf(Q), bit ? 0.0f : -1.0f);
        vc = em * rinv;
        T = fmaf(a.c2bpi, ex, vc);
    } else if (ELEC == 1) {
        const float einv = bit ? rinv : 0.0f;
        vc = einv + fmaf(a.krf, r2, -a.crf);
        T = fmaf(-a.k2rf, r2, einv);
    } else {
        const float t = r2 * rinv * a.tab_scale;
        const int i0 = (int)t;
        const float eps = t - (float)i0;
        const float2 g0 = tab[i0], g1 = tab[i0 + 1];
        const float einv = bit ? rinv : 0.0f;
        vc = einv - fmaf(eps, g1.y - g0.y, g0.y);
        T = fmaf(-fmaf(eps, g1.x - g0.x, g0.x), r2, einv);
    }
    const float4 lj = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(ljt) + (bit ? ljoff : 0));
    const float rinv6 = rinv2 * rinv2 * rinv2;
    const float B = fmaf(lj.y, rinv6, -lj.x);
    const float fsc = rinv2 * fmaf(qq, T, B * rinv6);
    if (ENER) {
        el = fmaf(rinv6, B - lj.x, el) - lj.z;
        ec += qq * (ELEC == 1 ? vc : vc - lj.w);   // the reaction field's c is in vc
    }
    return fsc;
}

// One pass of the direct kernel's inner loop: this lane's j-particle against
// the M i-particles.  lv: this lane holds a real j-particle of a valid entry;
// tri: i-slots below it take part (slot(i) < slot(j) for the self cluster
// pair, else M).  With LM (the single-system kernel) which lanes take part is
// decided in scalar registers, without branches: live (the lanes with lv),
// cleared for a dummy i-particle, and the compare k < tri straight into a
// lane mask; the exclusion bits become a lane mask the same way, read with
// inverse_ballot.  Without LM (the batched kernel) the tests are per-lane
// bit tests of an activity mask; each form measured faster in its kernel
// (single 96k box 95.5 against 100.9 us, batch of 256 replicas 3.57 against
// 3.75 ms).  Measured slower and not used: a copy of the pass without
// exclusion handling for passes that have none; a branch-free body whose
// eight i-particle chains the compiler can interleave (132 registers).
template <int M, bool ENER, int ELEC, bool LM>
__device__ inline void pair_pass(const ForceArgs &a, const EwPoly &ew, const float4 *ljt, const float2 *tab, const float (&xi)[M],
                                 const float (&yi)[M], const float (&zi)[M], const float (&qi)[M], const int (&ti)[M],
                                 float xj, float yj, float zj, float qj, int tj, unsigned mb, unsigned ireal, bool lv,
                                 unsigned long long live, int tri, float (&fix)[M],
                                 float (&fiy)[M], float (&fiz)[M], float &fjx, float &fjy, float &fjz, float &el,
                                 float &ec) {
    const unsigned act = lv ? ireal & ((1u << tri) - 1u) : 0u;   // the per-lane form
    const float rc2l = lv ? a.rc2 : -1.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const float dx = xi[k] - xj, dy = yi[k] - yj, dz = zi[k] - zj;
        const float r2 = dx * dx + dy * dy + dz * dz;
        bool in, bit;
        if (LM) {
            const unsigned long long am =
                (((ireal >> k) & 1u) ? live : 0ull) & __builtin_amdgcn_ballot_w64(k < tri);
            const unsigned long long bm = __builtin_amdgcn_ballot_w64((mb >> k) & 1u);
            in = (r2 < a.rc2) & __builtin_amdgcn_inverse_ballot_w64(am);
            bit = __builtin_amdgcn_inverse_ballot_w64(bm);
        } else {
            in = r2 < rc2l && ((act >> k) & 1u);
            bit = (mb >> k) & 1u;
        }
        if (in) {
            const float fsc = pair_term<ENER, ELEC>(a, ew, ljt, tab, r2, qi[k] * qj, bit, ti[k] + tj, el, ec);
            fix[k] = fmaf(fsc, dx, fix[k]);
            fiy[k] = fmaf(fsc, dy, fiy[k]);
            fiz[k] = fmaf(fsc, dz, fiz[k]);
            fjx = fmaf(-fsc, dx, fjx);
            fjy = fmaf(-fsc, dy, fjy);
            fjz = fmaf(-fsc, dz, fjz);
        }
    }
}

// Work items are split between the eight XCDs by the device-side item count:
// workgroups go to the XCDs round-robin by index, so XCD x = blockIdx % 8
// takes the x-th contiguous eighth of the items (neighbouring i-clusters share
// j-clusters, which then stay in one L2) and every XCD gets an equal share
// however far the launched grid (sized from the list capacity) exceeds it.
// Items of this workgroup's wavefronts: first_item() + wave; -1 past the end.
__device__ inline long xcd_block_first(long total, int waves_per_block) {
    const long per = (total + 7) / 8;
    const long k = (long)(blockIdx.x / 8) * waves_per_block;
    return k < per ? k : -1;
}
__device__ inline long xcd_item(long total, int waves_per_block, int wave) {
    const long per = (total + 7) / 8;
    const long k = (long)(blockIdx.x / 8) * waves_per_block + wave;
    if (k >= per) return -1;
    const long it = (long)(blockIdx.x % 8) * per + k;
    return it < total ? it : -1;
}

// sum over the 8 lanes of each aligned octet (DPP: quad swaps, then the half-row mirror)
__device__ inline float octet_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, false));   // [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xf, 0xf, false));   // [2,3,0,1]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xf, 0xf, false));  // half mirror
    return v;
}

// Totals of eight per-lane partials v[0..7] over the wavefront, transposed:
// afterwards every lane of octet o (lanes 8o..8o+7) holds the total of
// v[o].  Each exchange halves the values a lane carries: the lane halves
// (v_permlane32_swap) and then the row pairs (v_permlane16_swap) trade the
// partials they do not keep, a DPP rotate by 8 does the same inside a row,
// and the octet is summed with DPP: 18 instructions against 48 for eight
// separate wavefront sums.
__device__ inline float wave_sum8_t(const float (&v)[8], int lane) {
    float g[4], h[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) {   // lanes 0-31 keep v[k], lanes 32-63 keep v[k + 4]
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]), __float_as_uint(v[k + 4]), false, false);
        g[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {   // even rows keep g[k], odd rows g[k + 2]
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(g[k]), __float_as_uint(g[k + 2]), false, false);
        h[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool odd8 = (lane >> 3) & 1;   // lanes with bit 3 set keep h[1]
    const float keep = odd8 ? h[1] : h[0], send = odd8 ? h[0] : h[1];
    return octet_sum(keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), 0x128, 0xf, 0xf, false)));
}

// One work item of the direct kernel: up to 32 j-entries of one i-cluster on
// one wavefront (lane = entry slot x j-particle), i-forces in registers.
// (Issuing a pass's j-force atomics after the next pass's loads, so that the
// in-order wait for those loads does not include them, measured slower on
// gfx950: it costs registers and occupancy for no gain.)
template <int M, int N, bool ENER, bool VIR, bool ACC64, int ELEC, bool LM = true>
__device__ inline void force_item(const ForceArgs &a, const SysView &v, const float4 *ljt, const float2 *tab,
                                  const float4 *svec, int item, int lane) {
    using acc_t = typename std::conditional<ACC64, double, float>::type;
    constexpr int B = 64 / N;                      // entries per pass
    constexpr unsigned FULL = (1u << M) - 1u;
    const int4 it = ld(v.items + item);
    const int ci = __builtin_amdgcn_readfirstlane(it.x);
    const int js = __builtin_amdgcn_readfirstlane(it.y);
    const int je = __builtin_amdgcn_readfirstlane(it.z);

    float xi[M], yi[M], zi[M], qi[M];
    int ti[M];
    unsigned ireal = 0;   // i-slots holding particles (dummies have type -1)
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const float4 p = ld(v.xs_now + ci * M + k);
        xi[k] = p.x; yi[k] = p.y; zi[k] = p.z;
        qi[k] = p.w * a.coulomb_f;
        const int t = v.type_s[ci * M + k];
        ireal |= (t >= 0 ? 1u : 0u) << k;
        ti[k] = lj_ioff(a, t);   // types beyond ntypes are clamped
    }
    ireal = __builtin_amdgcn_readfirstlane(ireal);
    const EwPoly ew = ew_poly(a);
    float fix[M], fiy[M], fiz[M];
#pragma unroll
    for (int k = 0; k < M; ++k) fix[k] = fiy[k] = fiz[k] = 0.0f;
    acc_t elj = 0, ec = 0;
    acc_t vir[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) vir[k] = 0;

    const int jb = lane % N, eo = lane / N;
    for (int e0 = js; e0 < je; e0 += B) {
        const int e = e0 + eo;
        const bool valid = e < je;
        const nb_jentry en = ld(v.entries + (valid ? e : e0));
        const int row = v.jpos[valid ? e : e0];
        const int jslot = en.cj * N + jb;
        const float4 pj = ld(v.xs_now + jslot);
        const int tjr = v.type_s[jslot];
        const int tj = lj_joff(a, tjr);
        const float4 sv = svec[en.shift];
        const float xj = pj.x - sv.x, yj = pj.y - sv.y, zj = pj.z - sv.z;
        const float qj = pj.w;
        const unsigned long long m64 = ((unsigned long long)en.mhi << 32) | en.mlo;
        const unsigned mb = (unsigned)(m64 >> (jb * M)) & FULL;
        const bool lv = valid && tjr >= 0;   // pairs of real particles only: dummies never interact
        // self or overlapping cluster pair (zero shift): only slot(i) < slot(j), i.e. i-slot k < tri
        const int tri = en.shift == 13 ? min(max(jslot - ci * M, 0), M) : M;
        const unsigned long long live = __builtin_amdgcn_ballot_w64(lv);
        float fjx = 0.0f, fjy = 0.0f, fjz = 0.0f, el = 0.0f, ecl = 0.0f;
        pair_pass<M, ENER, ELEC, LM>(a, ew, ljt, tab, xi, yi, zi, qi, ti, xj, yj, zj, qj, tj, mb, ireal, lv, live, tri,
                                     fix, fiy, fiz, fjx, fjy, fjz, el, ecl);
        if (ENER) {
            elj += (acc_t)el;
            ec += (acc_t)ecl;
        }
        if (valid) {
            const gptr<float> o = v.fj + ((long)row * N + jb) * 3;
            o[0] = fjx;
            o[1] = fjy;
            o[2] = fjz;
        }
        if (VIR) {
            vir[0] += (acc_t)(xj * fjx); vir[1] += (acc_t)(xj * fjy); vir[2] += (acc_t)(xj * fjz);
            vir[3] += (acc_t)(yj * fjx); vir[4] += (acc_t)(yj * fjy); vir[5] += (acc_t)(yj * fjz);
            vir[6] += (acc_t)(zj * fjx); vir[7] += (acc_t)(zj * fjy); vir[8] += (acc_t)(zj * fjz);
        }
    }
    // i-forces: one reduction across the wavefront per work item
    acc_t viri[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) viri[k] = 0;
    // transposed sums (octet o stores i-particle o) in the single-system kernel; the batched kernel keeps
    // eight wavefront sums (the transposed form takes it to 75 registers and measured 2 % slower there)
    if constexpr (M == 8 && !VIR && LM) {
        const float fx = wave_sum8_t(fix, lane), fy = wave_sum8_t(fiy, lane), fz = wave_sum8_t(fiz, lane);
        if ((lane & 7) == 0) mxn::st(v.fi + (long)item * M + (lane >> 3), make_float4(fx, fy, fz, 0.0f));
    } else {
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const float fx = wave_sum_dpp(fix[k]), fy = wave_sum_dpp(fiy[k]), fz = wave_sum_dpp(fiz[k]);
        if (lane == 63) {
            mxn::st(v.fi + (long)item * M + k, make_float4(fx, fy, fz, 0.0f));
            if (VIR) {
                viri[0] += (acc_t)xi[k] * (acc_t)fx; viri[1] += (acc_t)xi[k] * (acc_t)fy; viri[2] += (acc_t)xi[k] * (acc_t)fz;
                viri[3] += (acc_t)yi[k] * (acc_t)fx; viri[4] += (acc_t)yi[k] * (acc_t)fy; viri[5] += (acc_t)yi[k] * (acc_t)fz;
                viri[6] += (acc_t)zi[k] * (acc_t)fx; viri[7] += (acc_t)zi[k] * (acc_t)fy; viri[8] += (acc_t)zi[k] * (acc_t)fz;
            }
        }
    }
    }
    if (ENER || VIR) {
        acc_t out[kNAcc];
        out[0] = ENER ? wave_sum(elj) * (acc_t)kLJScale : (acc_t)0;
        out[1] = ENER ? wave_sum(ec) : (acc_t)0;
#pragma unroll
        for (int k = 0; k < 9; ++k) out[2 + k] = VIR ? wave_sum(vir[k]) + viri[k] : (acc_t)0;
        if (lane == 63)   // the lane that holds the i-force terms (virial slots are read only with the virial)
            for (int k = 0; k < (VIR ? kNAcc : 2); ++k)
                v.partials[(size_t)k * v.pstride + v.pbase + item] = (double)out[k];
    }
}

template <int M, int N, bool ENER, bool VIR, bool ACC64, int ELEC>
__global__ __launch_bounds__(256) void k_forces(ForceArgs a) {
    const long total = a.totals[2];
    if (xcd_block_first(total, 4) < 0) return;   // whole workgroup past the end
    // tables at fixed LDS addresses: the LJ row of a pair is one add from its type offsets
    __shared__ float4 ljt[1 + mxn::kMaxTypes * mxn::kMaxTypes];   // LJ rows by type pair (fill_ljt)
    __shared__ float4 svec[32];                                   // 27 image shift vectors
    extern __shared__ float4 smem[];
    float2 *tab = reinterpret_cast<float2 *>(smem);   // Ewald table (ELEC == 2)
    for (int t = threadIdx.x; t < 27; t += blockDim.x) svec[t] = a.shiftvec[t];
    fill_ljt(a, ljt);
    if (ELEC == 2)
        for (int t = threadIdx.x; t < a.ntab; t += blockDim.x) tab[t] = a.etab[t];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const long item = xcd_item(total, 4, threadIdx.x >> 6);
    if (item < 0) return;
    const SysView v = make_view(a.xs_now, a.type_s, a.fj, a.fi, a.jpos, a.items, a.entries, a.partials, a.pstride, 0);
    force_item<M, N, ENER, VIR, ACC64, ELEC>(a, v, ljt, tab, svec, (int)item, lane);
}

// ---------------------------------------------------------------------------
// Super-cluster kernel (8x8 clusters).  The GPU layout of Sec. 2.3 and 3.2:
// S consecutive i-clusters form a super-cluster whose list holds each
// j-cluster (with its image shift) once, with a bit per i-cluster that has
// the pair and that pair's exclusion mask.  A wavefront owns a run of such
// super-cluster entries; lane = 8 b + a holds i-particle a of every
// i-cluster of the super-cluster (registers) and j-particle b of the
// current entry, so one pass evaluates the 64 pairs of one cluster pair and
// the list's j-major mask bit b*8 + a is the lane's own bit: the mask and
// the half-list triangle act as lane masks straight from scalar registers.
// The i-clusters an entry does not reach are skipped without cost (uniform
// branch).  Per entry the j-forces, summed over the S cluster pairs in
// registers, are reduced over the 8 a-lanes with DPP and stored once into
// the entry's row, so a j-cluster has one row per super-cluster that
// reaches it instead of one per i-cluster; i-forces are reduced across the
// wavefront once per work item and stored per (item, i-particle).  Dummy
// slots are moved far apart (i to +1e20, j to -1e20 in x), so that their
// squared distance overflows to infinity and fails the cut-off test.
constexpr float kFarX = 1.0e20f;

constexpr unsigned long long upper_triangle_lanes() {   // lanes 8b + a with a < b
    unsigned long long m = 0;
    for (int l = 0; l < 64; ++l)
        if ((l & 7) < (l >> 3)) m |= 1ull << l;
    return m;
}

// sum over the lanes with equal (lane & 7)
__device__ inline float stride8_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));  // row_ror 8
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// The cluster pairs of one super-cluster entry: for each i-cluster g that the
// entry reaches (bit g of gm), one pass of the 64 pairs with the pair's
// exclusion mask (slot g of the entry's mask record).  selfg: the i-cluster
// that is the entry's j-cluster itself (zero shift; -1 if none), whose pass
// takes the half-list triangle a < b only.
template <int S, bool ENER, int ELEC>
__device__ inline void sci_entry(const ForceArgs &a, const EwPoly &ew, const float4 *ljt, const float2 *tab, const uint2 *mrec, int gm,
                                 int selfg, const float4 *ip, const int *it, float xj, float yj, float zj, float qj,
                                 int tj, float (&fix)[S], float (&fiy)[S], float (&fiz)[S], float &fjx, float &fjy,
                                 float &fjz, float &el, float &ec) {
    constexpr unsigned long long kUpper = upper_triangle_lanes();
    uint2 mw[S];   // the whole record at once (one scalar load; unreached slots are not used)
#pragma unroll
    for (int g = 0; g < S; ++g) mw[g] = mrec[g];
#pragma unroll
    for (int g = 0; g < S; ++g) {
        if ((gm >> g) & 1) {
            const unsigned long long m64 = ((unsigned long long)mw[g].y << 32) | mw[g].x;
            const float4 pi = ip[g * 8];   // (x, y, z, f q) of i-particle a of i-cluster g
            const float dx = pi.x - xj, dy = pi.y - yj, dz = pi.z - zj;
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (__builtin_amdgcn_inverse_ballot_w64(g == selfg ? kUpper : ~0ull) && r2 < a.rc2) {
                const bool bit = __builtin_amdgcn_inverse_ballot_w64(m64);
                const float fsc = pair_term<ENER, ELEC>(a, ew, ljt, tab, r2, pi.w * qj, bit, it[g * 8] + tj, el, ec);
                fix[g] = fmaf(fsc, dx, fix[g]);
                fiy[g] = fmaf(fsc, dy, fiy[g]);
                fiz[g] = fmaf(fsc, dz, fiz[g]);
                fjx = fmaf(-fsc, dx, fjx);
                fjy = fmaf(-fsc, dy, fjy);
                fjz = fmaf(-fsc, dz, fjz);
            }
        }
    }
}

template <int S, bool ENER, bool VIR, bool ACC64, int ELEC>
__global__ __launch_bounds__(256) void k_forces_sci(ForceArgs a, const int4 *__restrict__ sent,
                                                    const uint2 *__restrict__ smask,
                                                    const int4 *__restrict__ sitems) {
    using acc_t = typename std::conditional<ACC64, double, float>::type;
    const long total = a.totals[2];
    if (xcd_block_first(total, 4) < 0) return;
    extern __shared__ float4 smem[];
    float4 *svec = smem;
    float4 *ljt = smem + 32;
    float2 *tab = reinterpret_cast<float2 *>(smem + 32 + a.nt * a.nt + 1);
    // per wavefront: its super-cluster's i-particles, (x, y, z, f q) and the type row
    const int ioff = 32 + a.nt * a.nt + 1 + (ELEC == 2 ? (a.ntab + 1) / 2 : 0);
    float4 *ipw = smem + ioff + (threadIdx.x >> 6) * S * 8;
    int *itw = reinterpret_cast<int *>(smem + ioff + 4 * S * 8) + (threadIdx.x >> 6) * S * 8;
    for (int t = threadIdx.x; t < 27; t += blockDim.x) svec[t] = a.shiftvec[t];
    fill_ljt(a, ljt);
    if (ELEC == 2)
        for (int t = threadIdx.x; t < a.ntab; t += blockDim.x) tab[t] = a.etab[t];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const long item = xcd_item(total, 4, threadIdx.x >> 6);
    if (item < 0) return;
    const int4 it = sitems[item];
    const int grp = __builtin_amdgcn_readfirstlane(it.x);
    const int js = __builtin_amdgcn_readfirstlane(it.y);
    const int je = __builtin_amdgcn_readfirstlane(it.z);
    const int ia = lane & 7, jb = lane >> 3;
    const int ci0 = grp * S;
    const int nci = *a.nslots / 8;
    const gptr<const float4> xs = (gptr<const float4>)a.xs_now;
    const gptr<const int> types = (gptr<const int>)a.type_s;
    if (jb < S) {   // lane (a, b) stages i-particle a of i-cluster b
        const bool in = ci0 + jb < nci;
        const int slot = in ? (ci0 + jb) * 8 + ia : ia;
        const float4 p = ld(xs + slot);
        const int t = in ? types[slot] : -1;
        ipw[lane] = make_float4(t >= 0 ? p.x : kFarX, p.y, p.z, p.w * a.coulomb_f);
        itw[lane] = lj_ioff(a, t);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // the wavefront's staging is visible to all its lanes
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float4 *ip = ipw + ia;
    const EwPoly ew = ew_poly(a);
    const int *itp = itw + ia;
    float fix[S], fiy[S], fiz[S];
#pragma unroll
    for (int g = 0; g < S; ++g) fix[g] = fiy[g] = fiz[g] = 0.0f;
    acc_t elj = 0, ec = 0;
    acc_t vir[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) vir[k] = 0;

    for (int e = js; e < je; ++e) {
        const int4 en = sent[e];   // uniform: scalar load
        const int cj = en.x, shift = en.y & 31, gm = (en.y >> 8) & 255, selfg = ((en.y >> 16) & 15) - 1, row = en.w;
        const uint2 *mrec = smask + (long)e * S;   // exclusion mask of i-cluster g in slot g
        const int jslot = cj * 8 + jb;
        const float4 pj = ld(xs + jslot);
        const int tjr = types[jslot];
        const int tj = lj_joff(a, tjr);
        const float4 sv = svec[shift];
        const float xj = tjr >= 0 ? pj.x - sv.x : -kFarX, yj = pj.y - sv.y, zj = pj.z - sv.z;
        const float qj = pj.w;
        float fjx = 0.0f, fjy = 0.0f, fjz = 0.0f, el = 0.0f, ecl = 0.0f;
        sci_entry<S, ENER, ELEC>(a, ew, ljt, tab, mrec, gm, selfg, ip, itp, xj, yj, zj, qj, tj, fix, fiy, fiz, fjx, fjy,
                                 fjz, el, ecl);
        if (ENER) {
            elj += (acc_t)el;
            ec += (acc_t)ecl;
        }
        if (VIR) {   // this lane's share of the j-force (the octet sum is linear)
            vir[0] += (acc_t)(xj * fjx); vir[1] += (acc_t)(xj * fjy); vir[2] += (acc_t)(xj * fjz);
            vir[3] += (acc_t)(yj * fjx); vir[4] += (acc_t)(yj * fjy); vir[5] += (acc_t)(yj * fjz);
            vir[6] += (acc_t)(zj * fjx); vir[7] += (acc_t)(zj * fjy); vir[8] += (acc_t)(zj * fjz);
        }
        fjx = octet_sum(fjx);
        fjy = octet_sum(fjy);
        fjz = octet_sum(fjz);
        if (ia < 3) {   // lanes a = 0, 1, 2 of octet b store its x, y, z: one 96-byte row
            const float c = ia == 0 ? fjx : (ia == 1 ? fjy : fjz);
            ((gptr<float>)a.fj)[((long)row * 8 + jb) * 3 + ia] = c;
        }
    }
    acc_t viri[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) viri[k] = 0;
    const gptr<float4> fo = (gptr<float4>)a.fi;
#pragma unroll
    for (int g = 0; g < S; ++g) {
        const float fx = stride8_sum(fix[g]), fy = stride8_sum(fiy[g]), fz = stride8_sum(fiz[g]);
        if (jb == 0) {
            mxn::st(fo + ((long)item * S + g) * 8 + ia, make_float4(fx, fy, fz, 0.0f));
            const float4 pi = ip[g * 8];
            if (VIR && pi.x != kFarX) {
                viri[0] += (acc_t)pi.x * (acc_t)fx; viri[1] += (acc_t)pi.x * (acc_t)fy; viri[2] += (acc_t)pi.x * (acc_t)fz;
                viri[3] += (acc_t)pi.y * (acc_t)fx; viri[4] += (acc_t)pi.y * (acc_t)fy; viri[5] += (acc_t)pi.y * (acc_t)fz;
                viri[6] += (acc_t)pi.z * (acc_t)fx; viri[7] += (acc_t)pi.z * (acc_t)fy; viri[8] += (acc_t)pi.z * (acc_t)fz;
            }
        }
    }
    if (ENER || VIR) {
        acc_t out[kNAcc];
        out[0] = ENER ? wave_sum(elj) * (acc_t)kLJScale : (acc_t)0;
        out[1] = ENER ? wave_sum(ec) : (acc_t)0;
#pragma unroll
        for (int k = 0; k < 9; ++k) out[2 + k] = VIR ? wave_sum(vir[k] + viri[k]) : (acc_t)0;
        if (lane == 0)
            for (int k = 0; k < kNAcc; ++k) a.partials[(size_t)k * a.pstride + item] = (double)out[k];
    }
}

// Forces of one j-cluster's N slots: the j-forces in the j-cluster's rows
// plus the i-forces stored by the work items of the i-cluster(s) holding
// these slots; written to the caller's array in input order (or added to it).
// One wavefront per j-cluster, lane = (group g, j-particle b): the 64/N
// groups take every (64/N)-th row and item (four rows in flight per lane;
// each step reads 64/N consecutive rows), and a butterfly sums the groups.
// The sums are taken in fixed point: each term rounded to a multiple of
// 2^-16 (the FP32 rounding step of a term of magnitude 128; a few hundred
// such roundings per force stay near 1e-4 in force units, against forces of
// order 1e3) and held as an integer-valued double, so every addition is
// exact while the running sums stay below 2^53 units (1.4e11 in force units;
// guaranteed for terms below 2^26 with at most 2^11 of them per force, i.e.
// rows of a j-cluster plus items of an i-cluster: a few hundred), and the
// sums do not depend on the order of the rows.  A non-finite term, or one of
// 2^52 units (6.9e10) or more (overlapping particles), makes the force NaN
// and latches FLAG_FORCE_RANGE for nb_sync.  After an overflowed build (no usable
// items) every force is zero.
struct FoldView {
    gptr<const int> nslots, perm, totals, jstart, part_istart;
    gptr<const float> fj;
    gptr<const float4> fi;
    float *f_out;
    int parts, accumulate;
    int sci;   // i-clusters per item group: the i-forces of cluster c are slot c % sci of group c / sci's items
    int *flags;
};

constexpr double kFixScale = 65536.0;          // 2^16
constexpr double kFixInv = 1.0 / 65536.0;
constexpr double kFixMax = 4503599627370496.0;   // 2^52 units: terms below 2^36

// x in 2^-16 units, rounded (exact: FP32 to FP64, times a power of two, to
// the nearest integer); bad set for NaN, infinities and values beyond the range
__device__ inline double to_fix(float x, bool &bad) {
    const double y = rint((double)x * kFixScale);
    bad |= !(fabs(y) < kFixMax);
    return y;
}

template <int M, int N>
__device__ inline void fold_body(const FoldView &v, int cj, int lane) {
    constexpr int G = 64 / N;
    cj = __builtin_amdgcn_readfirstlane(cj);   // wave-uniform: scalar loads of the row bounds
    if (cj >= *v.nslots / N) return;
    const int b = lane % N, g = lane / N, s = cj * N + b;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    bool bad = false;
    const int at = v.perm[s];   // loaded early: the output index, needed at the end
    if (v.totals[2] > 0) {
        // the i-forces of the first work item of this lane's i-cluster, loaded before the rows so that the
        // two chains of loads overlap
        const int ci = s / M, o = s % M;
        const int gi = ci / v.sci, sub = ci % v.sci;
        const int t0 = v.part_istart[gi * v.parts] + g, t1 = v.part_istart[(gi + 1) * v.parts];
        const float4 fi0 = t0 < t1 ? ld(v.fi + ((long)t0 * v.sci + sub) * M + o) : make_float4(0.f, 0.f, 0.f, 0.f);
        const int k1 = v.jstart[cj + 1];
        for (int k0 = v.jstart[cj] + g; k0 < k1; k0 += 4 * G) {
            // all four loads issued before any is used: past the last row a
            // lane re-reads row k0 (valid) and drops the value
            float f[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const gptr<const float> p = v.fj + ((long)(k0 + u * G < k1 ? k0 + u * G : k0) * N + b) * 3;
                f[u][0] = p[0];
                f[u][1] = p[1];
                f[u][2] = p[2];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {   // branch-free: the loads above stay in flight together
                const bool ok = k0 + u * G < k1;
                bool b3 = false;
                const double qx = to_fix(f[u][0], b3), qy = to_fix(f[u][1], b3), qz = to_fix(f[u][2], b3);
                sx += ok ? qx : 0.0;
                sy += ok ? qy : 0.0;
                sz += ok ? qz : 0.0;
                bad |= ok && b3;
            }
        }
        sx += to_fix(fi0.x, bad);
        sy += to_fix(fi0.y, bad);
        sz += to_fix(fi0.z, bad);
        for (int t = t0 + G; t < t1; t += G) {
            const float4 f = ld(v.fi + ((long)t * v.sci + sub) * M + o);
            sx += to_fix(f.x, bad);
            sy += to_fix(f.y, bad);
            sz += to_fix(f.z, bad);
        }
    }
#pragma unroll
    for (int o = N; o < 64; o <<= 1) {
        sx += __shfl_xor(sx, o, 64);
        sy += __shfl_xor(sy, o, 64);
        sz += __shfl_xor(sz, o, 64);
    }
    const unsigned long long badm = __ballot(bad);
    if (g == 0) {
        if (at >= 0) {
            bool nonfinite = false;
#pragma unroll
            for (int q = 0; q < G; ++q) nonfinite |= (badm >> (q * N + b)) & 1ull;
            float fx = (float)(sx * kFixInv), fy = (float)(sy * kFixInv), fz = (float)(sz * kFixInv);
            if (nonfinite) {
                fx = fy = fz = __builtin_nanf("");
                atomicOr(v.flags, mxn::FLAG_FORCE_RANGE);
            }
            float *out = v.f_out + 3 * (long)at;
            if (v.accumulate) {
                fx += out[0]; fy += out[1]; fz += out[2];
            }
            out[0] = fx;
            out[1] = fy;
            out[2] = fz;
        }
    }
}

// Energy and virial from the per-item partials, deterministic and in two
// stages: the first kReduceParts fold workgroups each sum a contiguous share
// of the items (fixed thread assignment and tree) into one value per
// quantity, then one wavefront sums those values in a fixed order.  (A single
// launch with a last-workgroup ticket needs a device-scope release per
// workgroup, which writes back the L2 of every XCD: measured far slower.)
// FP64, or FP32 throughout for the precision study.
constexpr int kReduceParts = 256;
static_assert(kReduceParts % 64 == 0, "the second stage gives each lane the same number of shares");

template <bool ACC64>
__device__ inline void fold_energy(const ForceArgs &a) {
    using acc_t = typename std::conditional<ACC64, double, float>::type;
    __shared__ acc_t red[256];
    const int t = threadIdx.x, w = blockIdx.x;
    const int R = min((int)gridDim.x, kReduceParts);
    if (w >= R) return;
    const long nit = a.totals[2];
    const long per = (nit + R - 1) / R, i0 = w * per, i1 = min(nit, i0 + per);
    for (int k = 0; k < kNAcc; ++k) {
        if ((k < 2 && !a.ener) || (k >= 2 && !a.vir)) continue;
        acc_t s = 0;
        for (long i = i0 + t; i < i1; i += 256) s += (acc_t)a.partials[(size_t)k * a.pstride + i];
        red[t] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (t < h) red[t] += red[t + h];
            __syncthreads();
        }
        if (t == 0) a.blockpart[(size_t)k * kReduceParts + w] = (double)red[0];
    }
}

// The second stage: one wavefront, every share's value loaded at once (one
// memory latency instead of one per quantity), four per lane summed in order
// and then across the lanes by a fixed butterfly.
template <bool ACC64>
__global__ __launch_bounds__(64) void k_reduce_parts(const double *blockpart, int R, double *energy, double *virial,
                                                     int ener, int vir) {
    using acc_t = typename std::conditional<ACC64, double, float>::type;
    constexpr int P = kReduceParts / 64;
    const int t = threadIdx.x;
    double v[kNAcc][P];
#pragma unroll
    for (int k = 0; k < kNAcc; ++k) {
        const bool on = k < 2 ? ener : vir;
#pragma unroll
        for (int u = 0; u < P; ++u)
            v[k][u] = on && t + 64 * u < R ? blockpart[(size_t)k * kReduceParts + t + 64 * u] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kNAcc; ++k) {
        if ((k < 2 && !ener) || (k >= 2 && !vir)) continue;
        acc_t s = 0;
#pragma unroll
        for (int u = 0; u < P; ++u) s += (acc_t)v[k][u];
        s = wave_sum(s);
        if (t == 0) {
            if (k < 2) energy[k] = (double)s;
            else virial[k - 2] = (double)s;
        }
    }
}

template <int M, int N, int ACC>   // ACC: 0 no energy/virial, 1 FP32, 2 FP64 sums
__global__ __launch_bounds__(256) void k_fold(ForceArgs a) {
    const FoldView v{(gptr<const int>)a.nslots, (gptr<const int>)a.perm,   (gptr<const int>)a.totals,
                     (gptr<const int>)a.jstart, (gptr<const int>)a.part_istart,
                     (gptr<const float>)a.fj,   (gptr<const float4>)a.fi,  a.f_out,
                     a.parts,                   a.accumulate,              a.sci > 1 ? a.sci : 1,
                     a.flags};
    fold_body<M, N>(v, blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
    if (ACC == 1) fold_energy<false>(a);
    if (ACC == 2) fold_energy<true>(a);
}

// Pair statistics of a list at the current positions (the paper's effective
// pair ratio, Sec. 5): c[0] real listed pairs (active mask/triangle), c[1]
// interacting pairs within rc, c[2] excluded pairs within rc.
template <int M, int N>
__global__ __launch_bounds__(256) void k_stats(ForceArgs a, unsigned long long *c) {
    constexpr int B = 64 / N;
    constexpr unsigned FULL = (1u << M) - 1u;
    const int lane = threadIdx.x & 63;
    const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= a.totals[2]) return;
    const int4 it = a.items[item];
    const int ci = it.x;
    unsigned long long real = 0, inr = 0, exc = 0;
    const int jb = lane % N, eo = lane / N;
    for (int e0 = it.y; e0 < it.z; e0 += B) {
        const int e = e0 + eo;
        if (e >= it.z) continue;
        const nb_jentry en = a.entries[e];
        const int jslot = en.cj * N + jb;
        const float4 pj = a.xs_now[jslot];
        const float4 sv = a.shiftvec[en.shift];
        const unsigned long long m64 = ((unsigned long long)en.mhi << 32) | en.mlo;
        const unsigned mb = (unsigned)(m64 >> (jb * M)) & FULL;
        unsigned act = FULL;
        if (en.shift == 13) {
            const int t = jslot - ci * M;
            act = t >= M ? FULL : (t <= 0 ? 0u : (1u << t) - 1u);
        }
        for (int k = 0; k < M; ++k) {
            if (!((act >> k) & 1u) || a.perm[ci * M + k] < 0 || a.perm[jslot] < 0) continue;
            ++real;
            const float4 pi = a.xs_now[ci * M + k];
            const float dx = pi.x - (pj.x - sv.x), dy = pi.y - (pj.y - sv.y), dz = pi.z - (pj.z - sv.z);
            if (dx * dx + dy * dy + dz * dz < a.rc2) {
                if ((mb >> k) & 1u) ++inr;
                else ++exc;
            }
        }
    }
    real = wave_sum(real); inr = wave_sum(inr); exc = wave_sum(exc);
    if (lane == 0) {
        atomicAdd(c, real);
        atomicAdd(c + 1, inr);
        atomicAdd(c + 2, exc);
    }
}

template <int M, int N>
void launch_fold(const ForceArgs &a, int acc, int nb, hipStream_t st) {
    const int R = std::min(nb, kReduceParts);
    if (acc == 0) {
        k_fold<M, N, 0><<<nb, 256, 0, st>>>(a);
    } else if (acc == 1) {
        k_fold<M, N, 1><<<nb, 256, 0, st>>>(a);
        k_reduce_parts<false><<<1, 64, 0, st>>>(a.blockpart, R, a.energy, a.virial, a.ener, a.vir);
    } else {
        k_fold<M, N, 2><<<nb, 256, 0, st>>>(a);
        k_reduce_parts<true><<<1, 64, 0, st>>>(a.blockpart, R, a.energy, a.virial, a.ener, a.vir);
    }
}

template <int M, int N, bool E, bool V, bool D>
void launch_k(const ForceArgs &a, int nb, size_t lds, int variant, hipStream_t st) {
    (void)variant;   // direct (also for lists the super-cluster kernel does not take)
    (void)lds;       // its LJ and shift tables are static LDS; only the Ewald table is dynamic
    if (a.elec == NB_COULOMB_RF)
        k_forces<M, N, E, V, D, 1><<<nb, 256, 0, st>>>(a);
    else if (a.elec == NB_COULOMB_EWALD_TABLE)
        k_forces<M, N, E, V, D, 2><<<nb, 256, (size_t)a.ntab * sizeof(float2), st>>>(a);
    else
        k_forces<M, N, E, V, D, 0><<<nb, 256, 0, st>>>(a);
}

template <int S, bool E, bool V, bool D>
void launch_sci_k(const ForceArgs &a, const int4 *sent, const uint2 *smask, const int4 *sitems, int nb, size_t lds,
                  hipStream_t st) {
    lds += 4 * S * 8 * (sizeof(float4) + sizeof(int));   // staged i-particles of the four wavefronts
    if (a.elec == NB_COULOMB_RF)
        k_forces_sci<S, E, V, D, 1><<<nb, 256, lds, st>>>(a, sent, smask, sitems);
    else if (a.elec == NB_COULOMB_EWALD_TABLE)
        k_forces_sci<S, E, V, D, 2><<<nb, 256, lds + (size_t)(a.ntab + 1) / 2 * sizeof(float4), st>>>(a, sent, smask,
                                                                                                    sitems);
    else
        k_forces_sci<S, E, V, D, 0><<<nb, 256, lds, st>>>(a, sent, smask, sitems);
}

template <int S>
void launch_sci(const ForceArgs &a, const nb_list *l, unsigned flags, int nb, size_t lds, hipStream_t st) {
    const bool E = flags & NB_ENERGY, V = flags & NB_VIRIAL, D = !(flags & NB_ACC_FP32);
    const int4 *se = (const int4 *)l->sci_ent.p, *si = (const int4 *)l->sci_items.p;
    const uint2 *sm = (const uint2 *)l->sci_mask.p;
    if (E && V && D) launch_sci_k<S, true, true, true>(a, se, sm, si, nb, lds, st);
    else if (E && V) launch_sci_k<S, true, true, false>(a, se, sm, si, nb, lds, st);
    else if (E && D) launch_sci_k<S, true, false, true>(a, se, sm, si, nb, lds, st);
    else if (E) launch_sci_k<S, true, false, false>(a, se, sm, si, nb, lds, st);
    else if (V && D) launch_sci_k<S, false, true, true>(a, se, sm, si, nb, lds, st);
    else if (V) launch_sci_k<S, false, true, false>(a, se, sm, si, nb, lds, st);
    else launch_sci_k<S, false, false, true>(a, se, sm, si, nb, lds, st);
}

template <int M, int N>
void launch_shape(const ForceArgs &a, unsigned flags, int nb, size_t lds, int var, hipStream_t st) {
    const bool E = flags & NB_ENERGY, V = flags & NB_VIRIAL, D = !(flags & NB_ACC_FP32);
    if (E && V && D) launch_k<M, N, true, true, true>(a, nb, lds, var, st);
    else if (E && V) launch_k<M, N, true, true, false>(a, nb, lds, var, st);
    else if (E && D) launch_k<M, N, true, false, true>(a, nb, lds, var, st);
    else if (E) launch_k<M, N, true, false, false>(a, nb, lds, var, st);
    else if (V && D) launch_k<M, N, false, true, true>(a, nb, lds, var, st);
    else if (V) launch_k<M, N, false, true, false>(a, nb, lds, var, st);
    else launch_k<M, N, false, false, true>(a, nb, lds, var, st);
}


// ---------------------------------------------------------------------------
// Batched replicas: many independent systems of one cluster shape in one
// launch per stage.  Work items of all replicas form one index space (a
// device-side prefix of the replicas' item counts), split between the XCDs
// like a single system's.  Each replica keeps its own grid and list; the
// kernels see them through a device table.

struct RepDesc {
    const float4 *xyzq_now;
    float *f_out;
    float4 *xs_now;
    const int *type_s, *perm, *img_s, *slot_of, *nslots;
    float *fj;
    float4 *fi;
    const int *jstart, *jpos, *part_istart;
    int parts, n;
    const int4 *items;
    const nb_jentry *entries;
    const int *totals;
    const float4 *shiftvec;
    float Lx, Ly, Lz;
    long pbase;   // first partial slot of this replica
};

struct BatchArgs {
    const RepDesc *rep;
    int n_rep;
    const long *slot_off, *atom_off;   // host-known prefixes (slots_cap, n)
    long *item_off;                    // device prefix of the replicas' item counts
    int waves;                         // wavefronts (work items) per workgroup
    double *partials;
    long pstride;
    double *energy, *virial;
    int accumulate;
    int *flags;
    int nt;                            // LJ types: particles of a type >= nt are reported
};

__device__ inline int find_rep(const long *off, int n, long x) {
    int lo = 0, hi = n - 1;   // last r with off[r] <= x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Exclusive prefix of the replicas' item counts (one workgroup of 1024
// threads: contiguous runs per thread, then a scan of the run sums).
__global__ __launch_bounds__(1024) void k_batch_prefix(BatchArgs b) {
    __shared__ long run[1024];
    const int t = threadIdx.x, per = (b.n_rep + 1023) / 1024;
    const int r0 = t * per, r1 = min(r0 + per, b.n_rep);
    long s = 0;
    for (int r = r0; r < r1; ++r) s += b.rep[r].totals[2];
    run[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scan
        const long v = t >= o ? run[t - o] : 0;
        __syncthreads();
        run[t] += v;
        __syncthreads();
    }
    long acc = run[t] - s;
    for (int r = r0; r < r1; ++r) {
        b.item_off[r] = acc;
        acc += b.rep[r].totals[2];
    }
    if (t == 1023) b.item_off[b.n_rep] = run[1023];
}

// The replica of each thread's element x in [first, first + blockDim): the binary search runs once per
// workgroup, for first (x < the total, off[n] > first), then each thread steps forward from it (a
// workgroup spans one replica or a few).  Every thread of the workgroup must call it.
__device__ inline int block_rep(const long *off, int n, long first, long x) {
    __shared__ int rep0;
    if (threadIdx.x == 0) rep0 = find_rep(off, n, first);
    __syncthreads();
    int r = rep0;
    while (r + 1 < n && off[r + 1] <= x) ++r;
    return r;
}

__global__ void k_batch_gather(BatchArgs b) {
    const long total = b.slot_off[b.n_rep], g0 = (long)blockIdx.x * blockDim.x, g = g0 + threadIdx.x;
    if (g0 >= total) return;   // whole workgroup past the end
    const int r = block_rep(b.slot_off, b.n_rep, g0, min(g, total - 1));
    if (g >= total) return;
    const RepDesc &d = b.rep[r];
    const int s = (int)(g - b.slot_off[r]);
    if (s >= *d.nslots) return;
    const int o = d.perm[s];
    if (o >= 0) {
        const float4 p = d.xyzq_now[o];
        if (!(isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w))) atomicOr(b.flags, mxn::FLAG_NONFINITE);
        if (d.type_s[s] >= b.nt) atomicOr(b.flags, mxn::FLAG_TYPE);
        d.xs_now[s] = apply_image(p, d.img_s[s], d.Lx, d.Ly, d.Lz);
    }
}

// Work item idx of the concatenated items of all replicas, which belongs to replica r.
template <int M, int N, bool ENER, bool VIR, int ELEC>
__device__ inline void batch_item(const ForceArgs &a, const BatchArgs &b, const float4 *ljt, const float2 *tab, long idx,
                                  int r, int lane) {
    const RepDesc &d = b.rep[r];
    const SysView v =
        make_view(d.xs_now, d.type_s, d.fj, d.fi, d.jpos, d.items, d.entries, b.partials, b.pstride, d.pbase);
    force_item<M, N, ENER, VIR, true, ELEC, false>(a, v, ljt, tab, d.shiftvec, (int)(idx - b.item_off[r]), lane);
}

// One launch over the concatenated work items of all replicas, one wavefront per item, split between the
// XCDs like the single-system kernel: wavefront k of XCD x takes item x * per + k.  The grid is sized from
// the replicas' item counts at their last synchronous list builds, so it may hold fewer than per
// wavefronts per XCD; k_batch_tail takes the items beyond.
template <int M, int N, bool ENER, bool VIR, int ELEC>
__global__ __launch_bounds__(512) void k_batch_forces(ForceArgs a, BatchArgs b) {
    const long total = b.item_off[b.n_rep];
    const long first = xcd_block_first(total, b.waves);
    if (first < 0) return;   // whole workgroup past the end
    extern __shared__ float4 ljt[];
    __shared__ int rep0;
    // the replica of the workgroup's first item, by binary search in the item prefix (one thread, while
    // the others fill the LJ table); each wavefront then steps forward from it, usually not at all
    if (threadIdx.x == 0) {
        const long per = (total + 7) / 8;
        rep0 = find_rep(b.item_off, b.n_rep, min((long)(blockIdx.x % 8) * per + first, total - 1));
    }
    fill_ljt(a, ljt);
    float2 *tab = reinterpret_cast<float2 *>(ljt + a.nt * a.nt + 1);   // Ewald table after the LJ rows
    if (ELEC == 2)
        for (int t = threadIdx.x; t < a.ntab; t += blockDim.x) tab[t] = a.etab[t];
    __syncthreads();
    const long idx = xcd_item(total, b.waves, threadIdx.x >> 6);
    if (idx < 0) return;
    const long x = __builtin_amdgcn_readfirstlane(idx);
    int r = rep0;
    while (r + 1 < b.n_rep && b.item_off[r + 1] <= x) ++r;
    batch_item<M, N, ENER, VIR, ELEC>(a, b, ljt, tab, x, r, threadIdx.x & 63);
}

// Items k >= covered of each XCD's share (covered: the main launch's wavefronts per XCD), strided over
// this launch's wavefronts; nothing to do, and an immediate exit, while the estimate holds.  A separate
// kernel because the loop costs registers (and occupancy) that the one-item kernel does not need.
template <int M, int N, bool ENER, bool VIR, int ELEC>
__global__ __launch_bounds__(512) void k_batch_tail(ForceArgs a, BatchArgs b, long covered) {
    const long total = b.item_off[b.n_rep];
    const long per = (total + 7) / 8;
    const long k0 = covered + (long)(blockIdx.x / 8) * b.waves;
    if (k0 >= per) return;   // uniform over the workgroup
    extern __shared__ float4 ljt[];
    fill_ljt(a, ljt);
    float2 *tab = reinterpret_cast<float2 *>(ljt + a.nt * a.nt + 1);
    if (ELEC == 2)
        for (int t = threadIdx.x; t < a.ntab; t += blockDim.x) tab[t] = a.etab[t];
    __syncthreads();
    const long x0 = (long)(blockIdx.x % 8) * per, x1 = min(x0 + per, total);
    const long stride = (long)(gridDim.x / 8) * b.waves;
    for (long idx = x0 + k0 + (threadIdx.x >> 6); idx < x1; idx += stride)
        batch_item<M, N, ENER, VIR, ELEC>(a, b, ljt, tab, idx,
                                          __builtin_amdgcn_readfirstlane(find_rep(b.item_off, b.n_rep, idx)),
                                          threadIdx.x & 63);
}

// one wavefront per j-cluster of every replica (the replicas' slot capacities
// are multiples of N, so wavefront w covers global slots w*N .. w*N + N - 1)
template <int M, int N>
__global__ __launch_bounds__(256) void k_batch_fold(BatchArgs b) {
    const long total = b.slot_off[b.n_rep], first = (long)blockIdx.x * 4 * N;
    const long g0 = ((long)blockIdx.x * 4 + (threadIdx.x >> 6)) * N;
    if (first >= total) return;   // whole workgroup past the end
    const int r = __builtin_amdgcn_readfirstlane(block_rep(b.slot_off, b.n_rep, first, min(g0, total - 1)));
    if (g0 >= total) return;
    const RepDesc &d = b.rep[r];
    const FoldView v{(gptr<const int>)d.nslots, (gptr<const int>)d.perm,   (gptr<const int>)d.totals,
                     (gptr<const int>)d.jstart, (gptr<const int>)d.part_istart,
                     (gptr<const float>)d.fj,   (gptr<const float4>)d.fi,  d.f_out,
                     d.parts,                   b.accumulate,              1,
                     b.flags};
    fold_body<M, N>(v, (int)((g0 - b.slot_off[r]) / N), threadIdx.x & 63);
}

// one workgroup per replica: its energies (and virial) from the per-item partials, in a fixed order
__global__ __launch_bounds__(256) void k_batch_reduce(BatchArgs b, int ener, int vir) {
    __shared__ double red[256];
    const int r = blockIdx.x, t = threadIdx.x;
    const RepDesc &d = b.rep[r];
    const int n = d.totals[2];
    for (int k = 0; k < kNAcc; ++k) {
        if ((k < 2 && !ener) || (k >= 2 && !vir)) continue;
        double s = 0.0;
        for (int i = t; i < n; i += 256) s += b.partials[(size_t)k * b.pstride + d.pbase + i];
        red[t] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (t < w) red[t] += red[t + w];
            __syncthreads();
        }
        if (t == 0) {
            if (k < 2) b.energy[2 * r + k] = red[0];
            else b.virial[9 * r + k - 2] = red[0];
        }
        __syncthreads();
    }
}

template <int M, int N, bool E, bool V, int ELEC>
int launch_batch_forces_k(const ForceArgs &a, const BatchArgs &b, long est_items, size_t lds, hipStream_t st) {
    // enough workgroups for every XCD to hold an eighth of the estimated items; the tail launch
    // (32 workgroups per XCD) takes whatever lies beyond
    const long per = (est_items + 7) / 8;
    const long nb = 8 * std::max(1L, (per + b.waves - 1) / b.waves);
    k_batch_forces<M, N, E, V, ELEC><<<(unsigned)nb, 64 * b.waves, lds, st>>>(a, b);
    k_batch_tail<M, N, E, V, ELEC><<<8 * 32, 64 * b.waves, lds, st>>>(a, b, (nb / 8) * b.waves);
    return NB_OK;
}

template <int M, int N, int ELEC>
int launch_batch_elec(const ForceArgs &a, const BatchArgs &b, unsigned flags, long est_items, size_t lds,
                      hipStream_t st) {
    const bool E = flags & NB_ENERGY, V = flags & NB_VIRIAL;
    if (E && V) return launch_batch_forces_k<M, N, true, true, ELEC>(a, b, est_items, lds, st);
    if (E) return launch_batch_forces_k<M, N, true, false, ELEC>(a, b, est_items, lds, st);
    if (V) return launch_batch_forces_k<M, N, false, true, ELEC>(a, b, est_items, lds, st);
    return launch_batch_forces_k<M, N, false, false, ELEC>(a, b, est_items, lds, st);
}

template <int M, int N>
int launch_batch_shape(const ForceArgs &a, const BatchArgs &b, unsigned flags, long est_items, size_t lds,
                       hipStream_t st) {
    if (a.elec == NB_COULOMB_RF) return launch_batch_elec<M, N, 1>(a, b, flags, est_items, lds, st);
    if (a.elec == NB_COULOMB_EWALD_TABLE)
        return launch_batch_elec<M, N, 2>(a, b, flags, est_items, lds + (size_t)a.ntab * sizeof(float2), st);
    return launch_batch_elec<M, N, 0>(a, b, flags, est_items, lds, st);
}
}  // namespace

namespace mxn {

int launch_gather(nb_ctx *ctx, const nb_grid *g, const float *xyzq_now, int nt) {
    ForceArgs a{};
    a.type_s = (const int *)g->type_s.p;
    a.nt = nt;
    a.nslots = (const int *)g->nslots.p;
    a.perm = (const int *)g->perm.p;
    a.img_s = (const int *)g->img_s.p;
    a.xyzq_now = (const float4 *)xyzq_now;
    a.xs_now = (float4 *)g->xs_now.p;
    a.Lx = g->Lf[0]; a.Ly = g->Lf[1]; a.Lz = g->Lf[2];
    a.flags = ctx->d_flags;
    k_gather<<<(g->slots_cap + 255) / 256, 256, 0, ctx->stream>>>(a);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

int launch_stats(nb_ctx *ctx, const nb_grid *g, const nb_list *l, const float *xyzq_now, float rc,
                 unsigned long long *d_counts) {
    hipStream_t st = ctx->stream;
    ForceArgs a{};
    a.nslots = (const int *)g->nslots.p;
    a.perm = (const int *)g->perm.p;
    a.img_s = (const int *)g->img_s.p;
    a.slot_of = (const int *)g->slot_of.p;
    a.type_s = (const int *)g->type_s.p;
    a.xyzq_now = (const float4 *)xyzq_now;
    a.xs_now = (float4 *)g->xs_now.p;
    a.n = g->n;
    a.items = (const int4 *)l->items.p;
    a.entries = (const nb_jentry *)l->entries.p;
    a.totals = (const int *)l->totals.p;
    a.shiftvec = (const float4 *)g->shiftvec.p;
    a.rc2 = rc * rc;
    a.Lx = g->Lf[0]; a.Ly = g->Lf[1]; a.Lz = g->Lf[2];
    a.flags = ctx->d_flags;
    k_gather<<<(g->slots_cap + 255) / 256, 256, 0, st>>>(a);
    const int nb = (int)((l->cap_items + 3) / 4) + 1;
    if (g->m == 4 && g->nn == 4) k_stats<4, 4><<<nb, 256, 0, st>>>(a, d_counts);
    else if (g->m == 4 && g->nn == 8) k_stats<4, 8><<<nb, 256, 0, st>>>(a, d_counts);
    else if (g->m == 8 && g->nn == 4) k_stats<8, 4><<<nb, 256, 0, st>>>(a, d_counts);
    else k_stats<8, 8><<<nb, 256, 0, st>>>(a, d_counts);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

// The Ewald table of the tabulated variant: (G, H) at r = i h, h = 1 pm, i < ntab, with
// G = (erf(beta r)/r - 2 beta/sqrt(pi) exp(-beta^2 r^2)) / r^2 and H = erf(beta r)/r, in FP64
// rounded once; at r = 0 their limits 4 beta^3 / (3 sqrt(pi)) and 2 beta / sqrt(pi).  One
// entry beyond rc guards the upper neighbour of the last interval.  Rebuilt (synchronously)
// only when beta or rc change.
constexpr double kTabScale = 1000.0;

static int ensure_ewald_table(nb_ctx *ctx, float beta, float rc, int *ntab) {
    const int n = (int)((double)rc * kTabScale) + 3;
    *ntab = n;
    if (ctx->etab.p && ctx->etab_beta == beta && ctx->etab_rc == rc) return NB_OK;
    std::vector<float2> h((size_t)n);
    const double b = beta, c = 2.0 * b / std::sqrt(M_PI);
    for (int i = 0; i < n; ++i) {
        const double r = i / kTabScale;
        double G, H;
        if (i == 0) {
            G = 4.0 * b * b * b / (3.0 * std::sqrt(M_PI));
            H = c;
        } else {
            H = std::erf(b * r) / r;
            G = (H - c * std::exp(-b * b * r * r)) / (r * r);
        }
        h[(size_t)i] = make_float2((float)G, (float)H);
    }
    int rc_ = ensure(ctx, ctx->etab, (size_t)n * sizeof(float2));
    if (rc_) return rc_;
    MXN_HIP(hipMemcpyAsync(ctx->etab.p, h.data(), (size_t)n * sizeof(float2), hipMemcpyHostToDevice, ctx->stream));
    MXN_HIP(hipStreamSynchronize(ctx->stream));   // h is released on return
    ctx->etab_beta = beta;
    ctx->etab_rc = rc;
    return NB_OK;
}


// The Coulomb variant's constants (Eq. 2 for Ewald; the reaction field's k and c; the Ewald table, built
// on first use and kept in the context).
static int set_coulomb(nb_ctx *ctx, ForceArgs &a, const nb_params *p) {
    a.elec = p->coulomb;
    if (p->coulomb == NB_COULOMB_RF) {   // k = (eps_rf - 1) / ((2 eps_rf + 1) rc^3), 0 = conducting; c = 1/rc + k rc^2
        const double rc = p->rc, eps = p->eps_rf;
        const double k = eps == 0.0 ? 1.0 / (2.0 * rc * rc * rc) : (eps - 1.0) / ((2.0 * eps + 1.0) * rc * rc * rc);
        a.krf = (float)k;
        a.k2rf = (float)(2.0 * k);
        a.crf = (float)(1.0 / rc + k * rc * rc);
    } else if (p->coulomb == NB_COULOMB_EWALD_TABLE) {
        int rc = ensure_ewald_table(ctx, p->beta, p->rc, &a.ntab);
        if (rc) return rc;
        a.etab = (const float2 *)ctx->etab.p;
        a.tab_scale = (float)kTabScale;
    }
    return NB_OK;
}

// The rational erfc fit in powers of r instead of u = beta r (coefficient k times beta^k), so the kernels
// evaluate it without forming u.
void set_ewald_poly(ForceArgs &a, float beta) {
    const double P[4] = {MXN_EWALD_P0, MXN_EWALD_P1, MXN_EWALD_P2, MXN_EWALD_P3};
    const double Q[5] = {MXN_EWALD_Q0, MXN_EWALD_Q1, MXN_EWALD_Q2, MXN_EWALD_Q3, MXN_EWALD_Q4};
    double bk = 1.0;
    for (int k = 0; k < 5; ++k, bk *= (double)beta) {
        if (k < 4) a.ep[k] = (float)(P[k] * bk);
        a.eq[k] = (float)(Q[k] * bk);
    }
}

// Device memory that exists from load time on, for nb_forces_noalloc: the per-work-item energy/virial
// partials and, after them, the per-share sums of their reduction.  One copy per GPU, held until the
// process ends; every call on a GPU shares it (calls that overlap in time on one GPU race).
static __device__ __align__(256) unsigned char scratch[NB_NOALLOC_SCRATCH_BYTES];

// The array's device address on the current device (host code uses this, never the array's name).
int noalloc_scratch_address(void **ptr) {
    *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(NB_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    return NB_OK;
}

int launch_forces(nb_ctx *ctx, const nb_grid *g, const nb_list *l, const float *xyzq_now, const nb_params *p,
                  unsigned flags, float *f, double *energy, double *virial, void *noalloc) {
    hipStream_t st = ctx->stream;
    const bool need_acc = flags & (NB_ENERGY | NB_VIRIAL);
    // super-cluster view: (re)built by the first call after a list build (not for the allocation-free call)
    const int S = !noalloc && ctx->force_variant == NB_FORCE_SUPER ? sci_size(l, ctx->sci_clusters) : 0;
    if (S) {
        const int per = ctx->sci_per_item > 0 ? ctx->sci_per_item : kSciPerItem;
        if (!l->sci_valid || l->sci_volatile || l->sci_S != S || l->sci_per_item != per) {
            int rc = launch_sci_view(l, S, per);
            if (rc) return rc;
        }
    }
    const long cap_items = S ? l->sci_cap_items : l->cap_items;
    const long pstride = cap_items + 4;
    const size_t part_bytes = (size_t)pstride * kNAcc * sizeof(double);
    const size_t block_off = (part_bytes + 255) / 256 * 256;
    if (noalloc) {
        if (block_off + (size_t)kReduceParts * kNAcc * sizeof(double) > (size_t)NB_NOALLOC_SCRATCH_BYTES)
            return fail(NB_ERR_UNSUPPORTED, "nb_forces_noalloc: the list's " + std::to_string(cap_items) +
                                                " work items need more energy partials than the static scratch holds");
        if (p->coulomb == NB_COULOMB_EWALD_TABLE)
            return fail(NB_ERR_UNSUPPORTED, "nb_forces_noalloc: the Ewald table variant needs a device table");
    } else if (need_acc) {
        int rc = ensure(ctx, ctx->partials, part_bytes);
        if (rc) return rc;
    }
    ForceArgs a{};
    a.nslots = (const int *)g->nslots.p;
    a.perm = (const int *)g->perm.p;
    a.img_s = (const int *)g->img_s.p;
    a.slot_of = (const int *)g->slot_of.p;
    a.type_s = (const int *)g->type_s.p;
    a.xyzq_now = (const float4 *)xyzq_now;
    a.xs_now = (float4 *)g->xs_now.p;
    a.fj = (float *)l->fj.p;
    a.fi = (float4 *)l->fi.p;
    a.jstart = (const int *)l->jstart.p;
    a.jpos = (const int *)l->jrank.p;   // rows, after the build's position pass
    a.part_istart = (const int *)l->part_istart.p;
    a.parts = l->resv_parts;
    a.n = g->n;
    a.items = (const int4 *)l->items.p;
    a.entries = (const nb_jentry *)l->entries.p;
    a.totals = (const int *)l->totals.p;
    a.shiftvec = (const float4 *)g->shiftvec.p;
    a.c6c12 = p->c6c12;
    a.nt = p->ntypes;
    a.shift_en = p->shift_energies;
    a.rc2 = p->rc * p->rc;
    a.beta = p->beta;
    a.c_exp = (float)(-(double)p->beta * (double)p->beta * 1.4426950408889634);
    a.c2bpi = (float)(2.0 * (double)p->beta / 1.7724538509055160);
    set_ewald_poly(a, p->beta);
    a.coulomb_f = p->coulomb_f;
    a.shiftC = p->shift_energies ? (float)(std::erfc((double)p->beta * p->rc) / (double)p->rc) : 0.0f;
    a.rc6inv = (float)(1.0 / std::pow((double)p->rc, 6));
    {
        const int rc_ = set_coulomb(ctx, a, p);
        if (rc_) return rc_;
    }
    a.Lx = g->Lf[0]; a.Ly = g->Lf[1]; a.Lz = g->Lf[2];
    a.sci = 1;
    if (S) {   // the fold reads the view's rows, i-forces and items
        a.fi = (float4 *)l->sci_fi.p;
        a.jstart = (const int *)l->sci_jstart.p;
        a.part_istart = (const int *)l->sci_istart.p;
        a.parts = 1;
        a.totals = (const int *)l->sci_totals.p;
        a.sci = S;
    }
    a.partials = noalloc ? (double *)noalloc : (double *)ctx->partials.p;
    a.pstride = pstride;
    a.f_out = f;
    a.accumulate = (flags & NB_ACCUMULATE) ? 1 : 0;
    a.flags = ctx->d_flags;
    // fold launch: one wavefront per j-cluster; with energies it also reduces the partials
    const int nfold = (g->slots_cap / g->nn + 3) / 4;
    if (need_acc) {
        if (noalloc) {
            a.blockpart = (double *)((char *)noalloc + block_off);
        } else {
            int rc = ensure(ctx, ctx->blockpart, (size_t)kReduceParts * kNAcc * sizeof(double));
            if (rc) return rc;
            a.blockpart = (double *)ctx->blockpart.p;
        }
        a.energy = energy;
        a.virial = virial;
        a.ener = (flags & NB_ENERGY) ? 1 : 0;
        a.vir = (flags & NB_VIRIAL) ? 1 : 0;
    }
    k_gather<<<(g->slots_cap + 255) / 256, 256, 0, st>>>(a);
    const long nwaves = cap_items;
    int nb = (int)((nwaves + 3) / 4);
    nb = (nb + 7) / 8 * 8;
    if (nb == 0) nb = 8;
    const size_t lds = (32 + (size_t)p->ntypes * p->ntypes + 1) * sizeof(float4);
    {
        ScopedTimer tm(ctx, noalloc ? -1 : NB_TIMER_FORCE_KERNEL);
        const int var = noalloc ? NB_FORCE_DIRECT : ctx->force_variant;
        if (S == 8) launch_sci<8>(a, l, flags, nb, lds, st);
        else if (S == 4) launch_sci<4>(a, l, flags, nb, lds, st);
        else if (g->m == 4 && g->nn == 4) launch_shape<4, 4>(a, flags, nb, lds, var, st);
        else if (g->m == 4 && g->nn == 8) launch_shape<4, 8>(a, flags, nb, lds, var, st);
        else if (g->m == 8 && g->nn == 4) launch_shape<8, 4>(a, flags, nb, lds, var, st);
        else launch_shape<8, 8>(a, flags, nb, lds, var, st);
    }
    const int acc = !need_acc ? 0 : ((flags & NB_ACC_FP32) ? 1 : 2);
    if (g->m == 4 && g->nn == 4) launch_fold<4, 4>(a, acc, nfold, st);
    else if (g->m == 4 && g->nn == 8) launch_fold<4, 8>(a, acc, nfold, st);
    else if (g->m == 8 && g->nn == 4) launch_fold<8, 4>(a, acc, nfold, st);
    else launch_fold<8, 8>(a, acc, nfold, st);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}


// The Coulomb variant's device tables, built before a graph capture (which may not allocate or copy from
// the host); the captured launches then find them ready.
int prepare_coulomb(nb_ctx *ctx, const nb_params *p) {
    if (p->coulomb != NB_COULOMB_EWALD_TABLE) return NB_OK;
    int ntab = 0;
    return ensure_ewald_table(ctx, p->beta, p->rc, &ntab);
}

int launch_batch(nb_ctx *ctx, nb_batch *bt, const nb_params *p, unsigned flags, double *energy, double *virial) {
    hipStream_t st = ctx->stream;
    ForceArgs a{};
    a.c6c12 = p->c6c12;
    a.nt = p->ntypes;
    a.shift_en = p->shift_energies;
    a.rc2 = p->rc * p->rc;
    a.beta = p->beta;
    a.c_exp = (float)(-(double)p->beta * (double)p->beta * 1.4426950408889634);
    a.c2bpi = (float)(2.0 * (double)p->beta / 1.7724538509055160);
    set_ewald_poly(a, p->beta);
    a.coulomb_f = p->coulomb_f;
    a.shiftC = p->shift_energies ? (float)(std::erfc((double)p->beta * p->rc) / (double)p->rc) : 0.0f;
    a.rc6inv = (float)(1.0 / std::pow((double)p->rc, 6));
    {
        const int rc_ = set_coulomb(ctx, a, p);
        if (rc_) return rc_;
    }
    BatchArgs b{};
    b.rep = (const RepDesc *)bt->desc.p;
    b.n_rep = bt->n_rep;
    b.slot_off = (const long *)bt->slot_off.p;
    b.atom_off = (const long *)bt->atom_off.p;
    b.item_off = (long *)bt->item_off.p;
    b.waves = bt->waves;
    b.partials = (double *)bt->partials.p;
    b.pstride = bt->pstride;
    b.energy = energy;
    b.virial = virial;
    b.accumulate = (flags & NB_ACCUMULATE) ? 1 : 0;
    b.flags = ctx->d_flags;
    b.nt = p->ntypes;
    k_batch_prefix<<<1, 1024, 0, st>>>(b);
    k_batch_gather<<<(int)((bt->total_slots + 255) / 256), 256, 0, st>>>(b);
    const size_t lds = ((size_t)p->ntypes * p->ntypes + 1) * sizeof(float4);
    // main-launch wavefronts: a quarter more than the replicas' items at their last synchronous builds
    // (or the count set by nb_batch_set_grid)
    long est = 0;
    for (const nb_list *l : bt->lists) {
        if (l->est_items <= 0) { est = bt->pstride; break; }
        est += l->est_items + l->est_items / 4;
    }
    est = std::min(bt->pstride, est + 256);
    if (bt->grid_waves > 0) est = bt->grid_waves;
    {
        ScopedTimer tm(ctx, NB_TIMER_FORCE_KERNEL);
        if (bt->m == 4 && bt->nn == 4) launch_batch_shape<4, 4>(a, b, flags, est, lds, st);
        else if (bt->m == 4 && bt->nn == 8) launch_batch_shape<4, 8>(a, b, flags, est, lds, st);
        else if (bt->m == 8 && bt->nn == 4) launch_batch_shape<8, 4>(a, b, flags, est, lds, st);
        else launch_batch_shape<8, 8>(a, b, flags, est, lds, st);
    }
    const int nfold = (int)((bt->total_slots / bt->nn + 3) / 4);
    if (bt->m == 4 && bt->nn == 4) k_batch_fold<4, 4><<<nfold, 256, 0, st>>>(b);
    else if (bt->m == 4 && bt->nn == 8) k_batch_fold<4, 8><<<nfold, 256, 0, st>>>(b);
    else if (bt->m == 8 && bt->nn == 4) k_batch_fold<8, 4><<<nfold, 256, 0, st>>>(b);
    else k_batch_fold<8, 8><<<nfold, 256, 0, st>>>(b);
    if (flags & (NB_ENERGY | NB_VIRIAL))
        k_batch_reduce<<<bt->n_rep, 256, 0, st>>>(b, (flags & NB_ENERGY) != 0, (flags & NB_VIRIAL) != 0);
    MXN_HIP(hipGetLastError());
    return NB_OK;
}

size_t rep_desc_size() { return sizeof(RepDesc); }

void fill_rep_desc(void *out, const nb_grid *g, const nb_list *l, const float *xyzq_now, float *f, long pbase) {
    RepDesc d{};
    d.xyzq_now = (const float4 *)xyzq_now;
    d.f_out = f;
    d.xs_now = (float4 *)g->xs_now.p;
    d.type_s = (const int *)g->type_s.p;
    d.perm = (const int *)g->perm.p;
    d.img_s = (const int *)g->img_s.p;
    d.slot_of = (const int *)g->slot_of.p;
    d.nslots = (const int *)g->nslots.p;
    d.fj = (float *)l->fj.p;
    d.fi = (float4 *)l->fi.p;
    d.jstart = (const int *)l->jstart.p;
    d.jpos = (const int *)l->jrank.p;
    d.part_istart = (const int *)l->part_istart.p;
    d.parts = l->resv_parts;
    d.n = g->n;
    d.items = (const int4 *)l->items.p;
    d.entries = (const nb_jentry *)l->entries.p;
    d.totals = (const int *)l->totals.p;
    d.shiftvec = (const float4 *)g->shiftvec.p;
    d.Lx = g->Lf[0]; d.Ly = g->Lf[1]; d.Lz = g->Lf[2];
    d.pbase = pbase;
    *(RepDesc *)out = d;
}

}  // namespace mxn
