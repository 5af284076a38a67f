/*
 * CPU ORACLE - test infrastructure only.
 *
 * Plain, slow, obviously-correct reference for the cluster-pair non-bonded
 * path of Pall & Hess, "A flexible algorithm for calculating pair interactions
 * on SIMD architectures" (CPC 2013).  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library; the GPU library
 * never links, calls or shares code with it.
 *
 * Contents
 *   1. FP64 forces / energies / virial by the plain definition (Sec. 3.2,
 *      Eq. 1 LJ and Eq. 2 Coulomb with the Ewald real-space correction g(r)),
 *      by brute force over all atom pairs, by a cell-list double loop, and for
 *      a subset of atoms.
 *   2. FP32 canonical grid sort (Sec. 2.3: x/y column grid with spacing
 *      (max(M,N)/rho)^(1/3), z-sort in each column, dummy padding).
 *   3. FP32 canonical cluster-pair list (Sec. 2.3, cluster-pair search
 *      pseudocode: bounding-box distance < rlist and (< rBB or some atom pair
 *      < rlist); half list by Newton's third law; periodic shifts stored per
 *      pair; exclusion bitmasks, Sec. 2.4), by brute force over every
 *      (i-cluster, shift, j-cluster) triple.
 *   4. Exact missed-pair recount for the Verlet-buffer study (Sec. 5 and the
 *      appendix): for every non-excluded atom pair the cluster-level list
 *      threshold and the displaced-pair potential.
 *
 * Conventions that the paper leaves open are fixed the same way as in the
 * GPU library's documentation; each is named where it is used.
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math (FP32 list code
 * must not be contracted into FMA: the list is defined by separately rounded
 * products and sums).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* 1. FP64 pair interactions by definition                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
    double rc, beta, f;      /* cut-off (nm), Ewald splitting (1/nm), 1/(4 pi eps0) */
    int ntypes;
    const double *c6c12;     /* [ti][tj][2] = C6, C12 */
    int shift;               /* 1: potentials shifted to zero at rc */
    int rf;                  /* 1: reaction field instead of Ewald (Eq. 2 with g(r) = -2 k r) */
    double k_rf, c_rf;       /* reaction-field constant k and energy shift c */
} oracle_params;

static int is_excluded(const int *off, const int *idx, int a, int b) {
    for (int k = off[a]; k < off[a + 1]; ++k)
        if (idx[k] == b) return 1;
    for (int k = off[b]; k < off[b + 1]; ++k)
        if (idx[k] == a) return 1;
    return 0;
}

/*
 * Interaction of atom i with atom j (i != j) at minimum-image separation
 * d = x_i - x_j.  Adds the force on i to fi, returns the pair energy split
 * into LJ and Coulomb, and the pair virial d (x) F_i.
 *
 * Non-excluded pair within rc (Eq. 1 with e_ij = 1, Eq. 2 with e_ij = 1):
 *   F_i = [12 C12/r^13 - 6 C6/r^7 + f qi qj (1/r^2 + g(r))] d/r,
 *   g(r) = d/dr[erf(beta r)/r]   (so 1/r^2 + g(r) = erfc(beta r)/r^2 + 2 beta/sqrt(pi) exp(-beta^2 r^2)/r)
 *   V    = C12/r^12 - C6/r^6 + f qi qj erfc(beta r)/r   (minus its value at rc when shifted)
 * Force-field-excluded pair within rc (Eq. 2 with e_ij = 0; the Ewald
 * correction is still applied, Sec. 2.4):
 *   F_i = f qi qj g(r) d/r,  V = -f qi qj erf(beta r)/r.
 * Reaction field instead (Sec. 3.2, g(r) = -2 k r): F_i = [LJ + f qi qj (e/r^2
 * - 2 k r)] d/r, V_C = f qi qj (e/r + k r^2 - c), with e = 1 for a
 * non-excluded pair and 0 for an excluded one.
 */
static void pair_term(const oracle_params *p, double qi, double qj, int ti, int tj, int excluded,
                      const double d[3], double fi[3], double *elj, double *ec, double vir[9]) {
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(r2 < p->rc * p->rc)) return;
    double r = sqrt(r2);
    double qq = p->f * qi * qj;
    double fr;                                    /* |F| along d/r, positive = repulsive */
    if (p->rf) {
        /* Reaction field (Eq. 2 with g(r) = -2 k r): |F| = qq (e/r^2 - 2 k r); the potential is
         * qq (e/r + k r^2 - c) with c = 1/rc + k rc^2, so a non-excluded pair's is zero at rc */
        double gk = -2.0 * p->k_rf * r;
        if (excluded) {
            fr = qq * gk;
            *ec += qq * (p->k_rf * r2 - p->c_rf);
        } else {
            double c6 = p->c6c12[2 * (ti * p->ntypes + tj)];
            double c12 = p->c6c12[2 * (ti * p->ntypes + tj) + 1];
            double r6 = r2 * r2 * r2;
            fr = 12.0 * c12 / (r6 * r6 * r) - 6.0 * c6 / (r6 * r) + qq * (1.0 / r2 + gk);
            double vlj = c12 / (r6 * r6) - c6 / r6;
            if (p->shift) {
                double rc6 = pow(p->rc, 6);
                vlj -= c12 / (rc6 * rc6) - c6 / rc6;
            }
            *elj += vlj;
            *ec += qq * (1.0 / r + p->k_rf * r2 - p->c_rf);
        }
    } else {
        double br = p->beta * r;
        double gauss = 2.0 * p->beta / sqrt(M_PI) * exp(-br * br);
        double g = gauss / r - erf(br) / r2;          /* d/dr [erf(beta r)/r] */
        if (excluded) {
            fr = qq * g;
            *ec += -qq * erf(br) / r;
        } else {
            double c6 = p->c6c12[2 * (ti * p->ntypes + tj)];
            double c12 = p->c6c12[2 * (ti * p->ntypes + tj) + 1];
            double r6 = r2 * r2 * r2;
            fr = 12.0 * c12 / (r6 * r6 * r) - 6.0 * c6 / (r6 * r) + qq * (1.0 / r2 + g);
            double vlj = c12 / (r6 * r6) - c6 / r6;
            double vc = qq * erfc(br) / r;
            if (p->shift) {
                double rc6 = pow(p->rc, 6);
                vlj -= c12 / (rc6 * rc6) - c6 / rc6;
                vc -= qq * erfc(p->beta * p->rc) / p->rc;
            }
            *elj += vlj;
            *ec += vc;
        }
    }
    for (int a = 0; a < 3; ++a) {
        double fa = fr * d[a] / r;
        fi[a] += fa;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) vir[3 * a + b] += d[a] * fr * d[b] / r;
}

static void min_image(const double L[3], const float *xi, const float *xj, double d[3]) {
    for (int a = 0; a < 3; ++a) {
        double v = (double)xi[a] - (double)xj[a];
        v -= L[a] * floor(v / L[a] + 0.5);
        d[a] = v;
    }
}

/* sum over j of the interaction of atom i; per-atom energies are half the pair sum */
static void atom_sum(const oracle_params *p, int n, const float *xyz, const float *q, const int *type,
                     const double L[3], const int *eo, const int *ei, int i, const int *cand, int ncand,
                     double fi[3], double *elj, double *ec, double vir[9]) {
    for (int k = 0; k < (cand ? ncand : n); ++k) {
        int j = cand ? cand[k] : k;
        if (j == i) continue;
        double d[3];
        min_image(L, xyz + 3 * i, xyz + 3 * j, d);
        pair_term(p, q[i], q[j], type[i], type[j], is_excluded(eo, ei, i, j), d, fi, elj, ec, vir);
    }
}

/*
 * Forces (n x 3), energies e[0] = LJ, e[1] = Coulomb, virial[9] = sum over
 * unordered pairs of r_ij (x) F_i, all FP64.  mode 0: brute force over all
 * pairs; mode 1: cell list with cells >= rc (falls back to brute force when
 * fewer than 3 cells fit along a dimension).  Each atom's force is summed
 * independently over all of its partners, so Newton's third law is not built
 * in and the zero-net-force test is a real check.
 */
static int forces_impl(const oracle_params *pp, int n, const float *xyz, const float *q, const int *type,
                       const double L[3], const int *excl_off, const int *excl_idx, int mode, double *f, double *e,
                       double *virial) {
    const oracle_params p = *pp;
    const double rc = p.rc;
    double *ea = (double *)calloc((size_t)n * 2, sizeof(double));
    double *va = (double *)calloc((size_t)n * 9, sizeof(double));
    if (!ea || !va) { free(ea); free(va); return -1; }
    int nc[3] = {1, 1, 1};
    int use_cells = (mode == 1);
    for (int a = 0; a < 3; ++a) {
        nc[a] = (int)floor(L[a] / rc);
        if (nc[a] < 3) use_cells = 0;
    }
    int *head = NULL, *next = NULL;
    if (use_cells) {
        size_t ncell = (size_t)nc[0] * nc[1] * nc[2];
        head = (int *)malloc(ncell * sizeof(int));
        next = (int *)malloc((size_t)n * sizeof(int));
        for (size_t c = 0; c < ncell; ++c) head[c] = -1;
        for (int i = n - 1; i >= 0; --i) {
            int c[3];
            for (int a = 0; a < 3; ++a) {
                double u = xyz[3 * i + a] - L[a] * floor(xyz[3 * i + a] / L[a]);
                c[a] = (int)(u / (L[a] / nc[a]));
                if (c[a] >= nc[a]) c[a] = nc[a] - 1;
            }
            int cell = (c[0] * nc[1] + c[1]) * nc[2] + c[2];
            next[i] = head[cell];
            head[cell] = i;
        }
    }
#pragma omp parallel
    {
        int *cand = NULL;
        int cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int i = 0; i < n; ++i) {
            double fi[3] = {0, 0, 0}, elj = 0, ec = 0, vir[9] = {0};
            if (!use_cells) {
                atom_sum(&p, n, xyz, q, type, L, excl_off, excl_idx, i, NULL, 0, fi, &elj, &ec, vir);
            } else {
                int c[3], m = 0;
                for (int a = 0; a < 3; ++a) {
                    double u = xyz[3 * i + a] - L[a] * floor(xyz[3 * i + a] / L[a]);
                    c[a] = (int)(u / (L[a] / nc[a]));
                    if (c[a] >= nc[a]) c[a] = nc[a] - 1;
                }
                for (int dx = -1; dx <= 1; ++dx)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dz = -1; dz <= 1; ++dz) {
                            int cx = (c[0] + dx + nc[0]) % nc[0], cy = (c[1] + dy + nc[1]) % nc[1],
                                cz = (c[2] + dz + nc[2]) % nc[2];
                            for (int j = head[(cx * nc[1] + cy) * nc[2] + cz]; j >= 0; j = next[j]) {
                                if (m == cap) {
                                    cap = cap ? 2 * cap : 4096;
                                    cand = (int *)realloc(cand, (size_t)cap * sizeof(int));
                                }
                                cand[m++] = j;
                            }
                        }
                atom_sum(&p, n, xyz, q, type, L, excl_off, excl_idx, i, cand, m, fi, &elj, &ec, vir);
            }
            for (int a = 0; a < 3; ++a) f[3 * i + a] = fi[a];
            ea[2 * i] = 0.5 * elj;
            ea[2 * i + 1] = 0.5 * ec;
            for (int a = 0; a < 9; ++a) va[9 * (size_t)i + a] = 0.5 * vir[a];
        }
        free(cand);
    }
    e[0] = e[1] = 0.0;
    for (int a = 0; a < 9; ++a) virial[a] = 0.0;
    for (int i = 0; i < n; ++i) {
        e[0] += ea[2 * i];
        e[1] += ea[2 * i + 1];
        for (int a = 0; a < 9; ++a) virial[a] += va[9 * (size_t)i + a];
    }
    free(ea); free(va); free(head); free(next);
    return 0;
}

int oracle_forces(int n, const float *xyz, const float *q, const int *type, const double L[3],
                  const int *excl_off, const int *excl_idx, int ntypes, const double *c6c12,
                  double rc, double beta, double coulomb_f, int shift, int mode,
                  double *f, double *e, double *virial) {
    oracle_params p = {rc, beta, coulomb_f, ntypes, c6c12, shift, 0, 0.0, 0.0};
    return forces_impl(&p, n, xyz, q, type, L, excl_off, excl_idx, mode, f, e, virial);
}

/* Reaction-field constants (the paper gives g(r) = -2 k r with k a constant; the usual choice for a
 * dielectric continuum eps_rf beyond rc): k = (eps_rf - 1) / ((2 eps_rf + 1) rc^3), eps_rf = 0 meaning a
 * conducting boundary (k = 1 / (2 rc^3)); c = 1/rc + k rc^2. */
static void rf_constants(double rc, double eps_rf, double *k, double *c) {
    *k = eps_rf == 0.0 ? 1.0 / (2.0 * rc * rc * rc) : (eps_rf - 1.0) / ((2.0 * eps_rf + 1.0) * rc * rc * rc);
    *c = 1.0 / rc + *k * rc * rc;
}

int oracle_forces_rf(int n, const float *xyz, const float *q, const int *type, const double L[3],
                     const int *excl_off, const int *excl_idx, int ntypes, const double *c6c12, double rc,
                     double eps_rf, double coulomb_f, int shift, int mode, double *f, double *e, double *virial) {
    oracle_params p = {rc, 0.0, coulomb_f, ntypes, c6c12, shift, 1, 0.0, 0.0};
    rf_constants(rc, eps_rf, &p.k_rf, &p.c_rf);
    return forces_impl(&p, n, xyz, q, type, L, excl_off, excl_idx, mode, f, e, virial);
}

/* forces on the listed atoms only (brute force over all partners); per-atom half energies */
int oracle_forces_subset(int n, const float *xyz, const float *q, const int *type, const double L[3],
                         const int *excl_off, const int *excl_idx, int ntypes, const double *c6c12,
                         double rc, double beta, double coulomb_f, int shift, int nsub, const int *sub,
                         double *f, double *e_atom) {
    oracle_params p = {rc, beta, coulomb_f, ntypes, c6c12, shift, 0, 0.0, 0.0};
#pragma omp parallel for schedule(dynamic, 16)
    for (int s = 0; s < nsub; ++s) {
        int i = sub[s];
        double fi[3] = {0, 0, 0}, elj = 0, ec = 0, vir[9] = {0};
        atom_sum(&p, n, xyz, q, type, L, excl_off, excl_idx, i, NULL, 0, fi, &elj, &ec, vir);
        for (int a = 0; a < 3; ++a) f[3 * s + a] = fi[a];
        e_atom[2 * s] = 0.5 * elj;
        e_atom[2 * s + 1] = 0.5 * ec;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* 2. FP32 canonical grid sort                                               */
/* ------------------------------------------------------------------------- */

/*
 * Column grid (Sec. 2.3): spacing s = (max(M,N)/rho)^(1/3) with rho = n/V,
 * n_x = max(1, floor(L_x/s)), likewise y.  The per-atom column index uses
 * inv_x = (float)(n_x/L_x) (host FP64 then rounded to FP32).
 */
void oracle_grid_dims(int n, const double box[3], int cmax, int *nx, int *ny, float *inv_x, float *inv_y) {
    double rho = (double)n / (box[0] * box[1] * box[2]);
    double s = cbrt((double)cmax / rho);
    int gx = (int)floor(box[0] / s), gy = (int)floor(box[1] / s);
    if (gx < 1) gx = 1;
    if (gy < 1) gy = 1;
    *nx = gx;
    *ny = gy;
    *inv_x = (float)((double)gx / box[0]);
    *inv_y = (float)((double)gy / box[1]);
}

typedef struct { float z; int orig; } zkey;

static int zkey_cmp(const void *a, const void *b) {
    const zkey *x = (const zkey *)a, *y = (const zkey *)b;
    if (x->z < y->z) return -1;
    if (x->z > y->z) return 1;
    return (x->orig > y->orig) - (x->orig < y->orig);
}

/*
 * Wrap, column assignment and z-sort.
 *   Wrap: L = (float)box, k = floor((double)x * (1.0/(double)L)) per dimension,
 *         x_w = x - (float)k * L in FP32 (separately rounded), -0 -> +0.
 *   Column: c_x = clamp(floor(x_w * inv_x), 0, n_x - 1), id = c_x * n_y + c_y.
 *   Order inside a column: ascending (z_w, original index); each column is
 *   padded with dummies to a multiple of cmax = max(M,N) slots.
 * Outputs (caller-allocated): slot_of[n], img[3n], xw[3n] (per original atom),
 * col_start[ncol+1] (slot offsets), col_count[ncol]; returns n_slots.
 */
int oracle_grid_sort(int n, const float *xyz, const double box[3], int cmax, int nx, int ny, float inv_x,
                     float inv_y, int *slot_of, int *img, float *xw, int *col_start, int *col_count) {
    float Lf[3] = {(float)box[0], (float)box[1], (float)box[2]};
    int ncol = nx * ny;
    int *col = (int *)malloc((size_t)n * sizeof(int));
    for (int c = 0; c < ncol; ++c) col_count[c] = 0;
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            double invL = 1.0 / (double)Lf[a];
            int k = (int)floor((double)xyz[3 * i + a] * invL);
            volatile float kl = (float)k * Lf[a];
            float w = xyz[3 * i + a] - kl;
            w = w + 0.0f;
            img[3 * i + a] = k;
            xw[3 * i + a] = w;
        }
        int cx = (int)floorf(xw[3 * i] * inv_x), cy = (int)floorf(xw[3 * i + 1] * inv_y);
        if (cx < 0) cx = 0;
        if (cx > nx - 1) cx = nx - 1;
        if (cy < 0) cy = 0;
        if (cy > ny - 1) cy = ny - 1;
        col[i] = cx * ny + cy;
        col_count[col[i]]++;
    }
    col_start[0] = 0;
    for (int c = 0; c < ncol; ++c) col_start[c + 1] = col_start[c] + (col_count[c] + cmax - 1) / cmax * cmax;
    for (int c = 0; c < ncol; ++c) {
        zkey *keys = (zkey *)malloc((size_t)(col_count[c] > 0 ? col_count[c] : 1) * sizeof(zkey));
        int m = 0;
        for (int i = 0; i < n; ++i)
            if (col[i] == c) { keys[m].z = xw[3 * i + 2]; keys[m].orig = i; ++m; }
        qsort(keys, (size_t)m, sizeof(zkey), zkey_cmp);
        for (int r = 0; r < m; ++r) slot_of[keys[r].orig] = col_start[c] + r;
        free(keys);
    }
    free(col);
    return col_start[ncol];
}

/* ------------------------------------------------------------------------- */
/* 3. FP32 canonical cluster-pair list                                       */
/* ------------------------------------------------------------------------- */

/*
 * Shift index s = 9 (sx+1) + 3 (sy+1) + (sz+1), sx,sy,sz in {-1,0,1}: the
 * i-cluster is moved by (sx Lx, sy Ly, sz Lz).  Half list: keep s > 13
 * (lexicographically positive shift), and for s == 13 keep (ci, cj) iff the
 * last slot of cj is after the first slot of ci, processing only atom pairs
 * with slot(i) < slot(j).
 *
 * Predicate per (ci, s, cj), all FP32 with separately rounded operations:
 *   lo' = lo_i + s L, hi' = hi_i + s L      (BB of real atoms, shifted)
 *   d_k = max(0, lo_j,k - hi'_k, lo'_k - hi_j,k)
 *   d2  = (d_x d_x + d_y d_y) + d_z d_z
 *   keep iff d2 < rlist^2 and (d2 < rbb^2 or some real pair has r2 < rlist^2)
 *   r2  = (dx dx + dy dy) + dz dz with dx = (x_a + s L_x) - x_b
 * Mask bit a*N + b (a = i-slot in ci, b = j-slot in cj) is 1 iff both atoms
 * are real, not (s == 13 and slot_a >= slot_b), and not (a force-field
 * excluded pair with r2 < rlist^2 in this shift).
 */
typedef struct { int ci, shift, cj, pad; uint64_t mask; } oracle_entry;

static void bb_of(const float *xs, const int *perm, int first, int size, float lo[3], float hi[3]) {
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int s = first; s < first + size; ++s) {
        if (perm[s] < 0) continue;
        for (int a = 0; a < 3; ++a) {
            float v = xs[3 * s + a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    }
}

static float sq_sum3(float a, float b, float c) {
    volatile float aa = a * a, bb = b * b, cc = c * c;
    volatile float ab = aa + bb;
    return ab + cc;
}

/* Entries of one i-cluster in canonical order (shift, cj), appended to *buf. */
typedef struct {
    oracle_entry *e;
    long n, cap;
} entry_buf;

static void buf_push(entry_buf *b, int ci, int s, int cj, uint64_t mask) {
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->e = (oracle_entry *)realloc(b->e, (size_t)b->cap * sizeof(oracle_entry));
    }
    oracle_entry *o = b->e + b->n++;
    o->ci = ci;
    o->shift = s;
    o->cj = cj;
    o->pad = 0;
    o->mask = mask;
}

static void list_one_ci(int ci, int M, int N, int ncj, const float *xs, const int *perm, const float Lf[3],
                        const float *blo, const float *bhi, float rl2, float rb2, const int *excl_off,
                        const int *excl_idx, entry_buf *out) {
    float ilo[3], ihi[3];
    bb_of(xs, perm, ci * M, M, ilo, ihi);
    for (int s = 13; s < 27; ++s) {
        int sh[3] = {s / 9 - 1, (s / 3) % 3 - 1, s % 3 - 1};
        float sv[3];
        for (int a = 0; a < 3; ++a) sv[a] = (float)sh[a] * Lf[a];
        float slo[3], shi[3];
        for (int a = 0; a < 3; ++a) { volatile float l = ilo[a] + sv[a], h = ihi[a] + sv[a]; slo[a] = l; shi[a] = h; }
        for (int cj = 0; cj < ncj; ++cj) {
            if (s == 13 && !(cj * N + N - 1 > ci * M)) continue;
            float d[3];
            for (int a = 0; a < 3; ++a) {
                volatile float d1 = blo[3 * cj + a] - shi[a], d2 = slo[a] - bhi[3 * cj + a];
                float m = d1 > d2 ? d1 : d2;
                d[a] = m > 0.0f ? m : 0.0f;
            }
            float bd2 = sq_sum3(d[0], d[1], d[2]);
            if (!(bd2 < rl2)) continue;
            int keep = bd2 < rb2;
            uint64_t mask = 0;
            for (int a = 0; a < M; ++a) {
                int sa = ci * M + a, oa = perm[sa];
                if (oa < 0) continue;
                float xa[3];
                for (int k = 0; k < 3; ++k) { volatile float t = xs[3 * sa + k] + sv[k]; xa[k] = t; }
                for (int b = 0; b < N; ++b) {
                    int sb = cj * N + b, ob = perm[sb];
                    if (ob < 0) continue;
                    volatile float dx = xa[0] - xs[3 * sb], dy = xa[1] - xs[3 * sb + 1], dz = xa[2] - xs[3 * sb + 2];
                    float r2 = sq_sum3(dx, dy, dz);
                    if (r2 < rl2) keep = 1;
                    int bit = 1;
                    if (s == 13 && sa >= sb) bit = 0;
                    if (bit && r2 < rl2 && is_excluded(excl_off, excl_idx, oa, ob)) bit = 0;
                    if (bit) mask |= (uint64_t)1 << (a * N + b);
                }
            }
            if (keep) buf_push(out, ci, s, cj, mask);
        }
    }
}

/*
 * xs: sorted FP32 positions per slot (3 per slot; dummy slots ignored);
 * perm: slot -> original atom or -1.  Brute force over all triples for
 * ci in [ci_begin, ci_end).  Writes up to cap entries in canonical order
 * (ci, shift, cj) and returns the total count (which may exceed cap).
 * The i-clusters are split into fixed blocks listed in parallel (OpenMP)
 * and concatenated in block order, so the output does not depend on the
 * thread count.
 */
long oracle_pairlist(int n_slots, int M, int N, const float *xs, const int *perm, const double box[3],
                     float rlist, float rbb, const int *excl_off, const int *excl_idx, int ci_begin,
                     int ci_end, oracle_entry *out, long cap) {
    float Lf[3] = {(float)box[0], (float)box[1], (float)box[2]};
    int nci = n_slots / M, ncj = n_slots / N;
    float *blo = (float *)malloc((size_t)ncj * 3 * sizeof(float)), *bhi = (float *)malloc((size_t)ncj * 3 * sizeof(float));
    for (int cj = 0; cj < ncj; ++cj) bb_of(xs, perm, cj * N, N, blo + 3 * cj, bhi + 3 * cj);
    volatile float rl2v = rlist * rlist, rb2v = rbb * rbb;
    float rl2 = rl2v, rb2 = rb2v;
    if (ci_end > nci) ci_end = nci;
    if (ci_begin < 0) ci_begin = 0;
    const int blk = 16;
    int nblk = ci_end > ci_begin ? (ci_end - ci_begin + blk - 1) / blk : 0;
    entry_buf *bufs = (entry_buf *)calloc((size_t)(nblk > 0 ? nblk : 1), sizeof(entry_buf));
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nblk; ++b) {
        int c1 = ci_begin + (b + 1) * blk;
        if (c1 > ci_end) c1 = ci_end;
        for (int ci = ci_begin + b * blk; ci < c1; ++ci)
            list_one_ci(ci, M, N, ncj, xs, perm, Lf, blo, bhi, rl2, rb2, excl_off, excl_idx, bufs + b);
    }
    long total = 0;
    for (int b = 0; b < nblk; ++b) {
        for (long k = 0; k < bufs[b].n; ++k, ++total)
            if (total < cap) out[total] = bufs[b].e[k];
        free(bufs[b].e);
    }
    free(bufs);
    free(blo); free(bhi);
    return total;
}

/* ------------------------------------------------------------------------- */
/* 3b. Two-stage list: prune of a cluster-pair list at given positions       */
/* ------------------------------------------------------------------------- */

/*
 * Sec. 2.3: the list can be built from bounding boxes alone (rbb >= rlist in
 * oracle_pairlist), and the cluster pairs whose particles are all beyond a
 * radius are then removed with a particle-distance test.  Positions at a
 * later time keep the atoms' build-time images (the pair list's shifts are
 * fixed for its lifetime): slot position = x - (float)k * L in FP32, k the
 * image of oracle_grid_sort.
 */
void oracle_gather(int n, const float *xyz, const int *img, const int *slot_of, const double box[3], float *xs_now) {
    float Lf[3] = {(float)box[0], (float)box[1], (float)box[2]};
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            volatile float kl = (float)img[3 * i + a] * Lf[a];
            volatile float x = xyz[3 * i + a] - kl;
            xs_now[3 * slot_of[i] + a] = x;
        }
}

/*
 * Keep an entry (ci, s, cj) iff some real particle a of ci and real b of cj
 * have r2 < r^2, with r2 formed exactly as in the search's particle test
 * (i moved by the shift, separately rounded FP32 operations); exclusions
 * and the half-list triangle do not enter, as in that test.  Entries keep
 * their order and masks.  Returns the number kept.
 */
long oracle_prune(int M, int N, const float *xs, const int *perm, const double box[3], const oracle_entry *in,
                  long n_in, float r, oracle_entry *out) {
    float Lf[3] = {(float)box[0], (float)box[1], (float)box[2]};
    volatile float r2v = r * r;
    float r2 = r2v;
    long kept = 0;
    for (long e = 0; e < n_in; ++e) {
        int ci = in[e].ci, cj = in[e].cj, s = in[e].shift;
        int sh[3] = {s / 9 - 1, (s / 3) % 3 - 1, s % 3 - 1};
        float sv[3];
        for (int a = 0; a < 3; ++a) sv[a] = (float)sh[a] * Lf[a];
        int keep = 0;
        for (int a = 0; a < M && !keep; ++a) {
            int sa = ci * M + a;
            if (perm[sa] < 0) continue;
            float xa[3];
            for (int k = 0; k < 3; ++k) { volatile float t = xs[3 * sa + k] + sv[k]; xa[k] = t; }
            for (int b = 0; b < N && !keep; ++b) {
                int sb = cj * N + b;
                if (perm[sb] < 0) continue;
                volatile float dx = xa[0] - xs[3 * sb], dy = xa[1] - xs[3 * sb + 1], dz = xa[2] - xs[3 * sb + 2];
                if (sq_sum3(dx, dy, dz) < r2) keep = 1;
            }
        }
        if (keep) out[kept++] = in[e];
    }
    return kept;
}

/* ------------------------------------------------------------------------- */
/* 3c. Pair distance histogram (pair correlation function)                   */
/* ------------------------------------------------------------------------- */

/*
 * Sec. 1 and 2.3: pair correlation functions are pair evaluations of limited
 * range too, with a list built every evaluation and no particle pruning.
 * For every unordered pair of real atoms (a, b) -- optionally skipping
 * force-field exclusions -- with separation below r_max, count it in bin k of
 * its type pair (lo, hi) = (min, max of the types, each clamped to
 * [0, ntypes)): hist[(lo * ntypes + hi) * nbins + k] += 1.
 * The distance is the FP32 one of the cluster-pair kernels: positions are the
 * wrapped slot positions xs; the pair is oriented and shifted as the half
 * list holds it (the image s with x_a + s L nearest x_b, found in FP64; index
 * s > 13 keeps (i, j) = (a, b), s < 13 swaps them and negates s, s == 13 puts
 * the lower slot first); then d = x_i - (x_j - s L), r2 = (dx dx + dy dy) +
 * dz dz, separately rounded.  Bin k is the largest with e_k <= r2 and r2 <
 * e_nbins, where e_k = (float)((k dr)^2) in FP64, dr = r_max / nbins.
 */
void oracle_rdf(int n, const float *xs, const int *slot_of, const int *type, const double box[3], float r_max,
                int nbins, int ntypes, const int *excl_off, const int *excl_idx, int skip_excl,
                unsigned long long *hist) {
    float Lf[3] = {(float)box[0], (float)box[1], (float)box[2]};
    double dr = (double)r_max / nbins;
    float *edge = (float *)malloc((size_t)(nbins + 1) * sizeof(float));
    for (int k = 0; k <= nbins; ++k) edge[k] = (float)((k * dr) * (k * dr));
    for (int a = 0; a < n; ++a) {
        for (int b = a + 1; b < n; ++b) {
            if (skip_excl && is_excluded(excl_off, excl_idx, a, b)) continue;
            int sa = slot_of[a], sb = slot_of[b];
            const float *xa = xs + 3 * sa, *xb = xs + 3 * sb;
            int sh[3];
            for (int k = 0; k < 3; ++k) {   /* the image of a nearest b: x_a + s L ~ x_b */
                double d = ((double)xb[k] - (double)xa[k]) / (double)Lf[k];
                sh[k] = d > 0.5 ? 1 : (d < -0.5 ? -1 : 0);
            }
            int idx = 9 * (sh[0] + 1) + 3 * (sh[1] + 1) + (sh[2] + 1);
            const float *xi = xa, *xj = xb;
            int ti = type[a], tj = type[b];
            if (idx < 13 || (idx == 13 && sb < sa)) {
                xi = xb; xj = xa; ti = type[b]; tj = type[a];
                for (int k = 0; k < 3; ++k) sh[k] = -sh[k];
            }
            float d[3];
            for (int k = 0; k < 3; ++k) {
                volatile float sv = (float)sh[k] * Lf[k];
                volatile float xjs = xj[k] - sv;
                volatile float dk = xi[k] - xjs;
                d[k] = dk;
            }
            float r2 = sq_sum3(d[0], d[1], d[2]);
            if (!(r2 < edge[nbins])) continue;
            int k = nbins - 1;
            while (edge[k] > r2) --k;
            ti = ti < 0 ? 0 : (ti >= ntypes ? ntypes - 1 : ti);
            tj = tj < 0 ? 0 : (tj >= ntypes ? ntypes - 1 : tj);
            int lo = ti < tj ? ti : tj, hi = ti < tj ? tj : ti;
            hist[(size_t)(lo * ntypes + hi) * nbins + k] += 1;
        }
    }
    free(edge);
}

/* ------------------------------------------------------------------------- */
/* 4. Exact missed-pair recount (Verlet-buffer study, Sec. 5 and appendix)   */
/* ------------------------------------------------------------------------- */

/*
 * For every non-excluded atom pair (a < b) of a cluster-pair list built at
 * radius rl with BB shortcut rbb = rl - c (c >= 0 fixed), the pair is in the
 * list at any smaller radius r'_l = rc + r_b iff its cluster pair passes
 * there.  With the BB test monotone in the radius, the cluster pair's
 * inclusion threshold is tau = min(d_bb + c, d_atom_min) where d_bb is the
 * bounding-box distance and d_atom_min the smallest real-pair distance of the
 * cluster pair in that shift (both from the undisplaced positions): the pair
 * is listed at radius r'_l iff tau < r'_l.
 *
 * Missed energy for buffer r_b: sum over non-excluded pairs not listed at
 * rc + r_b whose displaced distance r_t < rc of the shifted pair potential
 * V(r_t) - V(rc) (LJ + Ewald real-space Coulomb).  Accumulated into buckets
 * over r_b = k * db (k = 0..nb-1): pair contributes to every bucket k with
 * rc + k db <= tau, i.e. E(r_b) = sum over pairs with tau >= rc + r_b.
 * This routine returns per-pair (tau, V_shift(r_t)) contributions binned by
 * tau into hist[nb] (FP64) such that E(k db) = sum_{k' >= k} hist[k'].
 *
 * Domain: the pairs of cluster pairs listed at rl itself (tau < rl); the
 * largest buffer considered is rl - rc.
 * Brute force over all pairs and all 27 images for tiny boxes: it uses the
 * canonical grid sort of section 2 to form the clusters.
 */
long oracle_recount(int n, const float *xyz0, const float *xyzt, const float *q, const int *type,
                    const double box[3], const int *excl_off, const int *excl_idx, int ntypes,
                    const double *c6c12, double rc, double beta, double coulomb_f, int M, int N,
                    float rl, float c_bb, double db, int nb, double *hist) {
    int cmax = M > N ? M : N;
    int nx, ny;
    float ix, iy;
    oracle_grid_dims(n, box, cmax, &nx, &ny, &ix, &iy);
    int ncol = nx * ny;
    int *slot_of = (int *)malloc((size_t)n * sizeof(int));
    int *img = (int *)malloc((size_t)n * 3 * sizeof(int));
    float *xw = (float *)malloc((size_t)n * 3 * sizeof(float));
    int *cs = (int *)malloc((size_t)(ncol + 1) * sizeof(int));
    int *cc = (int *)malloc((size_t)ncol * sizeof(int));
    int n_slots = oracle_grid_sort(n, xyz0, box, cmax, nx, ny, ix, iy, slot_of, img, xw, cs, cc);
    int *perm = (int *)malloc((size_t)n_slots * sizeof(int));
    float *xs = (float *)calloc((size_t)n_slots * 3, sizeof(float));
    for (int s = 0; s < n_slots; ++s) perm[s] = -1;
    for (int i = 0; i < n; ++i) {
        perm[slot_of[i]] = i;
        for (int a = 0; a < 3; ++a) xs[3 * slot_of[i] + a] = xw[3 * i + a];
    }
    float Lf[3] = {(float)box[0], (float)box[1], (float)box[2]};
    int nci = n_slots / M, ncj = n_slots / N;
    float *blo = (float *)malloc((size_t)ncj * 3 * sizeof(float)), *bhi = (float *)malloc((size_t)ncj * 3 * sizeof(float));
    for (int cj = 0; cj < ncj; ++cj) bb_of(xs, perm, cj * N, N, blo + 3 * cj, bhi + 3 * cj);
    oracle_params p = {rc, beta, coulomb_f, ntypes, c6c12, 1, 0, 0.0, 0.0};
    /* i-clusters in fixed blocks, each with its own histogram, summed in block
     * order afterwards: the result does not depend on the thread count */
    const int blk = 16;
    int nblk = (nci + blk - 1) / blk;
    double *bh = (double *)calloc((size_t)(nblk > 0 ? nblk : 1) * nb, sizeof(double));
    long counted = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : counted)
    for (int bk = 0; bk < nblk; ++bk) {
      double *h = bh + (size_t)bk * nb;
      int c1 = (bk + 1) * blk < nci ? (bk + 1) * blk : nci;
      for (int ci = bk * blk; ci < c1; ++ci) {
        float ilo[3], ihi[3];
        bb_of(xs, perm, ci * M, M, ilo, ihi);
        for (int s = 13; s < 27; ++s) {
            int sh[3] = {s / 9 - 1, (s / 3) % 3 - 1, s % 3 - 1};
            float sv[3];
            for (int a = 0; a < 3; ++a) sv[a] = (float)sh[a] * Lf[a];
            for (int cj = 0; cj < ncj; ++cj) {
                if (s == 13 && !(cj * N + N - 1 > ci * M)) continue;
                float d[3];
                for (int a = 0; a < 3; ++a) {
                    volatile float l = ilo[a] + sv[a], hh = ihi[a] + sv[a];
                    volatile float d1 = blo[3 * cj + a] - hh, d2 = l - bhi[3 * cj + a];
                    float m = d1 > d2 ? d1 : d2;
                    d[a] = m > 0.0f ? m : 0.0f;
                }
                double dbb = sqrt((double)sq_sum3(d[0], d[1], d[2]));
                if (dbb >= rl) continue;           /* beyond the largest list considered */
                double dmin = INFINITY;
                for (int a = 0; a < M; ++a) {
                    int sa = ci * M + a;
                    if (perm[sa] < 0) continue;
                    for (int b = 0; b < N; ++b) {
                        int sb = cj * N + b;
                        if (perm[sb] < 0) continue;
                        double r = sqrt((double)sq_sum3(xs[3 * sa] + sv[0] - xs[3 * sb], xs[3 * sa + 1] + sv[1] - xs[3 * sb + 1],
                                                         xs[3 * sa + 2] + sv[2] - xs[3 * sb + 2]));
                        if (r < dmin) dmin = r;
                    }
                }
                double tau = dbb + (double)c_bb;
                if (dmin < tau) tau = dmin;
                if (tau >= rl) continue;           /* not listed even at the largest radius */
                for (int a = 0; a < M; ++a) {
                    int sa = ci * M + a, oa = perm[sa];
                    if (oa < 0) continue;
                    for (int b = 0; b < N; ++b) {
                        int sb = cj * N + b, ob = perm[sb];
                        if (ob < 0) continue;
                        if (s == 13 && sa >= sb) continue;
                        if (is_excluded(excl_off, excl_idx, oa, ob)) continue;
                        /* displaced separation in the same image */
                        double dd[3];
                        for (int k = 0; k < 3; ++k) {
                            double x0a = (double)xyz0[3 * oa + k] - (double)img[3 * oa + k] * Lf[k] + sh[k] * (double)Lf[k];
                            double x0b = (double)xyz0[3 * ob + k] - (double)img[3 * ob + k] * Lf[k];
                            double ua = (double)xyzt[3 * oa + k] - (double)xyz0[3 * oa + k];
                            double ub = (double)xyzt[3 * ob + k] - (double)xyz0[3 * ob + k];
                            dd[k] = (x0a + ua) - (x0b + ub);
                        }
                        double fi[3] = {0, 0, 0}, elj = 0, ec = 0, vir[9] = {0};
                        pair_term(&p, q[oa], q[ob], type[oa], type[ob], 0, dd, fi, &elj, &ec, vir);
                        if (elj == 0.0 && ec == 0.0) continue;
                        int kb = (int)floor((tau - rc) / db);
                        if (kb < 0) continue;          /* listed even at zero buffer */
                        if (kb >= nb) kb = nb - 1;
                        h[kb] += elj + ec;
                        ++counted;
                    }
                }
            }
        }
      }
    }
    for (int k = 0; k < nb; ++k) hist[k] = 0.0;
    for (int bk = 0; bk < nblk; ++bk)
        for (int k = 0; k < nb; ++k) hist[k] += bh[(size_t)bk * nb + k];
    free(bh); free(blo); free(bhi);
    free(slot_of); free(img); free(xw); free(cs); free(cc); free(perm); free(xs);
    return counted;
}
