/*
 * Seeded synthetic water boxes: random sequential addition (RSA) of rigid
 * 3-site water molecules (O at the centre, two H at 0.1 nm, H-O-H 109.47 deg)
 * with uniformly random orientation, in a cubic or orthorhombic periodic box.
 *
 * This is an input generator only. It holds none of the pair-interaction,
 * clustering or pair-list arithmetic; both the CPU oracle and the GPU library
 * consume what it writes.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), the
 * published 64-bit finaliser with the golden-ratio increment.  Orientation:
 * Shoemake's uniform random unit quaternion (Graphics Gems III, 1992).
 *
 * Placement rule: a trial molecule (uniform O position, uniform orientation)
 * is accepted when its O is at least `d_oo` from every other O and every
 * intermolecular atom pair is at least `d_any` apart (minimum image).  After
 * `max_tries` rejections for one molecule the O position is taken from the
 * next free site of a jittered simple-cubic lattice and only the orientation
 * is redrawn; such fallbacks are counted and returned.
 */
#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s; } sm64;

static uint64_t sm64_next(sm64 *r) {
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform in [0, 1) with 53 random bits */
static double sm64_u01(sm64 *r) { return (double)(sm64_next(r) >> 11) * (1.0 / 9007199254740992.0); }

static void random_rotation(sm64 *r, double R[9]) {
    const double two_pi = 6.283185307179586476925286766559;
    double u1 = sm64_u01(r), u2 = sm64_u01(r), u3 = sm64_u01(r);
    double a = sqrt(1.0 - u1), b = sqrt(u1);
    double w = a * sin(two_pi * u2), x = a * cos(two_pi * u2);
    double y = b * sin(two_pi * u3), z = b * cos(two_pi * u3);
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w);     R[2] = 2 * (x * z + y * w);
    R[3] = 2 * (x * y + z * w);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
    R[6] = 2 * (x * z - y * w);     R[7] = 2 * (y * z + x * w);     R[8] = 1 - 2 * (x * x + y * y);
}

typedef struct {
    double L[3];
    int nc[3];
    double cw[3];
    int *head;  /* per cell: first molecule or -1 */
    int *next;  /* per molecule: next molecule in the same cell */
    double *pos; /* 9 doubles per molecule: O, H1, H2 */
} cellgrid;

static int cell_of(const cellgrid *g, const double o[3]) {
    int c[3];
    for (int d = 0; d < 3; ++d) {
        double u = o[d] - g->L[d] * floor(o[d] / g->L[d]);
        int k = (int)(u / g->cw[d]);
        if (k < 0) k = 0;
        if (k >= g->nc[d]) k = g->nc[d] - 1;
        c[d] = k;
    }
    return (c[0] * g->nc[1] + c[1]) * g->nc[2] + c[2];
}

static double mi_d2(const cellgrid *g, const double *a, const double *b) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        double v = a[d] - b[d];
        v -= g->L[d] * floor(v / g->L[d] + 0.5);
        s += v * v;
    }
    return s;
}

static int trial_ok(const cellgrid *g, const double m[9], double d_oo2, double d_any2) {
    int c0 = cell_of(g, m);
    int cz = c0 % g->nc[2], cy = (c0 / g->nc[2]) % g->nc[1], cx = c0 / (g->nc[2] * g->nc[1]);
    int rng[3] = {g->nc[0] < 3 ? 0 : 1, g->nc[1] < 3 ? 0 : 1, g->nc[2] < 3 ? 0 : 1};
    /* small grids: scan every cell once */
    int lo[3], hi[3];
    int cc[3] = {cx, cy, cz};
    for (int d = 0; d < 3; ++d) {
        if (rng[d]) { lo[d] = cc[d] - 1; hi[d] = cc[d] + 1; }
        else { lo[d] = 0; hi[d] = g->nc[d] - 1; }
    }
    for (int ix = lo[0]; ix <= hi[0]; ++ix)
        for (int iy = lo[1]; iy <= hi[1]; ++iy)
            for (int iz = lo[2]; iz <= hi[2]; ++iz) {
                int jx = (ix + g->nc[0]) % g->nc[0], jy = (iy + g->nc[1]) % g->nc[1], jz = (iz + g->nc[2]) % g->nc[2];
                int cell = (jx * g->nc[1] + jy) * g->nc[2] + jz;
                for (int k = g->head[cell]; k >= 0; k = g->next[k]) {
                    const double *o = g->pos + 9 * (size_t)k;
                    if (mi_d2(g, m, o) < d_oo2) return 0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            if (mi_d2(g, m + 3 * a, o + 3 * b) < d_any2) return 0;
                }
            }
    return 1;
}

/*
 * Place n_mol molecules in box L (nm).  Writes 3*n_mol atoms (O, H, H order)
 * into xyz[3 * 3 * n_mol] (double).  Returns the number of lattice fallbacks,
 * or -1 on allocation failure, or -2 if a fallback site could not be used.
 */
int synth_water_rsa(int n_mol, const double L[3], uint64_t seed, double d_oo, double d_any,
                    int max_tries, double *xyz) {
    const double r_oh = 0.1;
    const double half = 0.5 * 109.47 * 3.14159265358979323846 / 180.0;
    const double hloc[2][3] = {{r_oh * sin(half), 0.0, r_oh * cos(half)},
                               {-r_oh * sin(half), 0.0, r_oh * cos(half)}};
    cellgrid g;
    double cmin = d_oo > d_any + 2 * r_oh ? d_oo : d_any + 2 * r_oh;
    size_t ncell = 1;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = L[d];
        g.nc[d] = (int)floor(L[d] / cmin);
        if (g.nc[d] < 1) g.nc[d] = 1;
        g.cw[d] = L[d] / g.nc[d];
        ncell *= (size_t)g.nc[d];
    }
    g.head = (int *)malloc(ncell * sizeof(int));
    g.next = (int *)malloc((size_t)n_mol * sizeof(int));
    g.pos = xyz;
    if (!g.head || !g.next) { free(g.head); free(g.next); return -1; }
    for (size_t c = 0; c < ncell; ++c) g.head[c] = -1;

    sm64 rng = {seed * 0x2545F4914F6CDD1DULL + 1306ULL};
    int fallbacks = 0;
    /* lattice for fallbacks: smallest simple-cubic lattice with >= n_mol sites */
    int nl = (int)ceil(cbrt((double)n_mol));
    int next_site = 0;
    for (int i = 0; i < n_mol; ++i) {
        double m[9], R[9], o[3];
        int placed = 0;
        for (int t = 0; t < max_tries && !placed; ++t) {
            for (int d = 0; d < 3; ++d) o[d] = sm64_u01(&rng) * L[d];
            random_rotation(&rng, R);
            for (int d = 0; d < 3; ++d) m[d] = o[d];
            for (int h = 0; h < 2; ++h)
                for (int d = 0; d < 3; ++d)
                    m[3 + 3 * h + d] = o[d] + R[3 * d + 0] * hloc[h][0] + R[3 * d + 1] * hloc[h][1] + R[3 * d + 2] * hloc[h][2];
            placed = trial_ok(&g, m, d_oo * d_oo, d_any * d_any);
        }
        while (!placed) {
            if (next_site >= nl * nl * nl) { free(g.head); free(g.next); return -2; }
            int s = next_site++;
            int sx = s / (nl * nl), sy = (s / nl) % nl, sz = s % nl;
            int sc[3] = {sx, sy, sz};
            for (int t = 0; t < 64 && !placed; ++t) {
                for (int d = 0; d < 3; ++d) o[d] = (sc[d] + 0.5 + 0.1 * (sm64_u01(&rng) - 0.5)) * (L[d] / nl);
                random_rotation(&rng, R);
                for (int d = 0; d < 3; ++d) m[d] = o[d];
                for (int h = 0; h < 2; ++h)
                    for (int d = 0; d < 3; ++d)
                        m[3 + 3 * h + d] = o[d] + R[3 * d + 0] * hloc[h][0] + R[3 * d + 1] * hloc[h][1] + R[3 * d + 2] * hloc[h][2];
                placed = trial_ok(&g, m, d_oo * d_oo, d_any * d_any);
            }
            if (placed) ++fallbacks;
        }
        memcpy(xyz + 9 * (size_t)i, m, sizeof m);
        int c = cell_of(&g, m);
        g.next[i] = g.head[c];
        g.head[c] = i;
        if (n_mol >= 200000 && (i + 1) % 100000 == 0) {   /* large boxes take minutes: report progress */
            fprintf(stderr, "[synth] %d of %d molecules placed\n", i + 1, n_mol);
            fflush(stderr);
        }
    }
    free(g.head);
    free(g.next);
    return fallbacks;
}
