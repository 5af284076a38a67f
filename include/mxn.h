/*
 * mxn.h - C ABI of the MI355X (gfx950) cluster-pair non-bonded library.
 *
 * Method: Pall & Hess, "A flexible algorithm for calculating pair
 * interactions on SIMD architectures", Comput. Phys. Commun. 184 (2013).
 * Particles are grid-sorted into spatial clusters of fixed size, a
 * cluster-pair list is built at a buffered cut-off rlist from bounding-box
 * distances, and an M x N cluster-pair kernel evaluates Lennard-Jones plus
 * Ewald real-space Coulomb interactions with per-pair exclusion masks.
 *
 * Conventions for every entry point
 *   - Units: nm, ps, kJ/mol, e, u.  Positions/charges FP32, energies and
 *     virial FP64.
 *   - "device" pointers are HIP device memory owned by the caller (for
 *     example torch tensors on cuda:N); "host" pointers are ordinary host
 *     memory.  Nothing the caller passes is retained after a call returns,
 *     except that nb_grid / nb_list handles remember the box and shapes.
 *   - Handles (nb_ctx, nb_grid, nb_list, nb_batch, nb_mlp) are owned by the
 *     library and released with their *_free / nb_destroy call.
 *   - Work is enqueued on the context's HIP stream and is asynchronous unless
 *     stated otherwise.  Errors found on the host are returned immediately as
 *     a negative nb_status; errors found by kernels (non-finite coordinates,
 *     list capacity overflow, LJ types out of range) are latched on the device and returned by the
 *     next nb_sync on that context.  nb_last_error() describes the most recent
 *     non-OK status of the calling thread.  No C++ exception crosses the ABI.
 *   - Periodic orthorhombic boxes only, every edge longer than 2 * rlist.
 */
#ifndef MXN_H
#define MXN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NB_OK = 0,
    NB_ERR_ARG = -1,         /* invalid argument (null pointer, bad size or shape, out-of-range parameter) */
    NB_ERR_BOX = -2,         /* a box edge is not longer than 2 * rlist */
    NB_ERR_OOM = -3,         /* device allocation failed */
    NB_ERR_HIP = -4,         /* HIP runtime error */
    NB_ERR_OVERFLOW = -5,    /* pair-list capacity exceeded during an asynchronous build: rebuild */
    NB_ERR_STATE = -6,       /* handle used with an incompatible grid, list or context */
    NB_ERR_NONFINITE = -7,   /* non-finite or out-of-range coordinate seen by a kernel */
    NB_ERR_UNSUPPORTED = -8  /* valid request the library does not implement (for example beta*rc > 4) */
} nb_status;

typedef struct nb_ctx nb_ctx;
typedef struct nb_grid nb_grid;
typedef struct nb_list nb_list;
typedef struct nb_mlp nb_mlp;
typedef struct nb_batch nb_batch;

/* Cluster shape M x N: i-clusters of M particles against j-clusters of N
 * particles (Sec. 2.2 "The M x N algorithm").  Supported: 4x4, 4x8, 8x4 (the
 * paper's GPU shape: i-clusters are pairs of 4-clusters), 8x8. */
typedef struct { int m, n; } nb_shape;

/* Interaction parameters (Sec. 3.2 "Pair interaction functions", Eq. 1 and 2).
 *   rc        cut-off (nm); pairs with r >= rc contribute nothing
 *   beta      Ewald splitting parameter (1/nm); beta * rc must be <= 4
 *   coulomb_f 1/(4 pi eps0) in the caller's units (138.935458 kJ mol^-1 nm e^-2)
 *   ntypes    number of LJ types (1..32)
 *   c6c12     DEVICE, ntypes*ntypes*2 floats: [ti][tj] = (C6, C12), symmetric
 *   shift_energies  1: LJ and Coulomb potentials shifted to zero at rc
 *   coulomb   the long-range correction g(r) of Eq. 2:
 *             NB_COULOMB_EWALD (0): Ewald real space, g = d/dr[erf(beta r)/r],
 *               evaluated analytically (a rational approximation of erfc);
 *             NB_COULOMB_RF (1): reaction field, g = -2 k r with
 *               k = (eps_rf - 1) / ((2 eps_rf + 1) rc^3) (eps_rf = 0: conducting,
 *               k = 1/(2 rc^3)); potential e/r + k r^2 - c, c = 1/rc + k rc^2,
 *               also for excluded pairs (e = 0); shift_energies affects LJ only;
 *             NB_COULOMB_EWALD_TABLE (2): Ewald as 0, with the smooth parts of
 *               force and potential interpolated linearly from a table in LDS
 *               (spacing 1 pm, 8 KB per nm of rc: rc <= 4 nm, NB_ERR_UNSUPPORTED
 *               beyond).
 *             RF and the table are supported by the force kernels of single
 *             systems and by batches; nb_recount takes Ewald only.
 *   eps_rf    reaction field: relative permittivity beyond rc (>= 1, or 0) */
enum { NB_COULOMB_EWALD = 0, NB_COULOMB_RF = 1, NB_COULOMB_EWALD_TABLE = 2 };
typedef struct {
    float rc, beta, coulomb_f;
    int ntypes;
    const float *c6c12;
    int shift_energies;
    int coulomb;
    float eps_rf;
} nb_params;

/* ---------------------------------------------------------------- context */

/* Device memory for the library's handles, supplied by the caller (for
 * example PyTorch's caching allocator, so that one pool backs the caller's
 * tensors and the library's grids, lists and scratch).
 *   alloc(bytes, stream, user)  returns device memory on the context's device
 *                               usable in stream order on `stream` (the
 *                               context's stream at the time), or NULL when
 *                               out of memory (the call then fails with
 *                               NB_ERR_OOM)
 *   free(ptr, stream, user)     takes back a block, with the stream it was
 *                               allocated on; work the library enqueued on
 *                               that stream may still use it (stream order)
 * Blocks are requested when a handle grows (the first grid sort, list build
 * or force call of a size, nb_batch_create, nb_mlp_create, ...) and returned
 * when it is freed or grows again; never inside a captured graph.  After
 * nb_set_stream, synchronise the old stream before freeing handles whose
 * blocks came from it. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, void *stream, void *user);
    void *user;
} nb_allocator;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *ctx receives the handle.
 *   allocator  HOST, copied: device memory of every handle of this context
 *              (and of the context itself) comes from it; NULL: hipMalloc.
 * Handles must be freed before their context (nb_destroy). */
int nb_create(nb_ctx **ctx, int device, void *hip_stream, const nb_allocator *allocator);
void nb_destroy(nb_ctx *ctx);
/* Live device bytes held by this context and its handles: through the
 * caller's allocator and through hipMalloc (zero when an allocator was
 * given).  HOST outputs; either may be NULL. */
int nb_memory_info(const nb_ctx *ctx, size_t *via_allocator, size_t *via_hip);
/* Change the stream subsequent calls enqueue on. */
int nb_set_stream(nb_ctx *ctx, void *hip_stream);
/* Wait for the stream; return the first latched kernel error (and clear it). */
int nb_sync(nb_ctx *ctx);
/* Text for the calling thread's most recent non-OK status ("" if none). */
const char *nb_last_error(void);

/* -------------------------------------------------------------- grid sort */

/*
 * Cluster the particles (Sec. 2.3 "Pair list construction", gridding):
 * a 2-D x/y column grid of spacing (max(M,N)/rho)^(1/3), rho = n/V; particles
 * go into columns by counting sort, are ordered by z inside each column and
 * consecutive groups of min(M,N) form clusters; each column is padded with
 * dummy particles (no charge, no LJ, far away) to a multiple of max(M,N).
 * Per-cluster bounding boxes over real particles follow (for M != N both the
 * M- and N-particle boxes, the latter the union of two adjacent M-boxes).
 *
 *   box     HOST double[3] box edges (nm); kernels use (float)box
 *   n       number of particles (>= 1)
 *   xyzq    DEVICE float[4n]: x, y, z, q in original order (x may lie outside
 *           the box; each particle is wrapped and its image count recorded)
 *   type    DEVICE int[n]: LJ type in [0, ntypes).  A negative type latches
 *           NB_ERR_ARG for nb_sync; so does a type >= ntypes, found by the
 *           first nb_forces, nb_batch_forces, nb_recount or nb_rdf call that
 *           is given ntypes (the results of that call are then wrong)
 *   shape   cluster shape
 *   grid    in/out: *grid == NULL creates a grid, otherwise it is reused
 *           (storage grows as needed).
 * Canonical FP32 rules (wrap, column index, z order with ties by original
 * index) are stated in the library documentation and are bit-reproducible.
 */
int nb_grid_sort(nb_ctx *ctx, const double box[3], int n, const float *xyzq, const int *type, nb_shape shape,
                 nb_grid **grid);
void nb_grid_free(nb_grid *grid);

typedef struct {
    int n, n_slots, m, n_cl;      /* particles, padded slots, M, N */
    int nx, ny;                   /* column grid */
    int n_ci, n_cj;               /* i- and j-cluster counts (n_slots/M, n_slots/N) */
} nb_grid_info_t;

/* Synchronous.  Fills *info. */
int nb_grid_info(nb_grid *grid, nb_grid_info_t *info);

/* Synchronous copy of the sorted layout to HOST arrays (any may be NULL):
 *   perm[n_slots]      original index per slot, -1 for dummies
 *   xyzq[4*n_slots]    wrapped sorted positions and charges at sort time
 *   img[3*n]           per original particle image count k: wrapped = x - k*L
 *   col_start[nx*ny+1] first slot of each column
 *   bb[8*n_ci]         per i-cluster (lo.x, lo.y, lo.z, 0, hi.x, hi.y, hi.z, 0) */
int nb_grid_export(nb_grid *grid, int *perm, float *xyzq, int *img, int *col_start, float *bb);

/* ------------------------------------------------------------- pair list */

enum {
    NB_LIST_ASYNC = 1,          /* do not synchronise: search once into the regions reserved by the
                                   handle's last synchronous build; latch NB_ERR_OVERFLOW (reported
                                   by nb_sync) if an i-cluster outgrows its region */
    NB_LIST_BY_DISTANCE = 2     /* store each i-cluster's entries by bounding-box distance instead of
                                   in canonical order (groups the entries beyond the cut-off) */
};

/*
 * Cluster-pair search (Sec. 2.3, cluster-pair search pseudocode; Sec. 2.4
 * "Exclusion treatment"): for every i-cluster and periodic image shift, every
 * j-cluster whose bounding-box distance d satisfies d < rlist and (d < rbb or
 * some real particle pair is closer than rlist).  Half list (Newton's third
 * law): only image shifts that are zero or lexicographically positive, and for
 * the zero shift only pairs with slot(i) < slot(j).  Per entry an M*N-bit mask
 * clears dummy pairs, the lower triangle of self pairs and force-field
 * exclusions in the image where they lie within rlist (the Ewald correction is
 * still applied to those).
 *
 *   rlist     list radius (nm), > 0; every box edge must exceed 2*rlist
 *   rbb       bounding-box shortcut radius (nm); < 0 selects
 *             max(0, rlist - s/2) with s the column spacing
 *   excl_off  DEVICE int[n+1], excl_idx DEVICE int[excl_off[n]]: force-field
 *             exclusions as CSR in original indices; must be symmetric.  Both
 *             non-NULL (NB_ERR_ARG otherwise); with no exclusions excl_off is
 *             all zero and excl_idx any valid device address (never read)
 *   flags     0, NB_LIST_ASYNC, NB_LIST_BY_DISTANCE
 *   list      in/out: NULL creates, otherwise reused
 * Storage: each (i-cluster, search part) owns an equal region of the entry
 * array.  A synchronous build (no NB_LIST_ASYNC; also the first build of a
 * handle and any build after the grid's capacity changed) counts the
 * entries, sizes every region to the largest count plus a quarter plus 8
 * (synchronising once), then fills the regions.  An asynchronous build
 * searches once and fills the regions, with no host synchronisation (it can
 * be captured in a graph); a region that would overflow, or more entries
 * than the j-force rows of the last synchronous build hold (its entry count
 * plus a quarter), latches NB_ERR_OVERFLOW, and the next synchronous build
 * re-sizes.
 * Order is deterministic: regions by i-cluster, each region by image shift
 * and j-cluster (canonical), or with NB_LIST_BY_DISTANCE by bounding-box
 * distance (ties in canonical order).
 */
int nb_pairlist_build(nb_ctx *ctx, const nb_grid *grid, float rlist, float rbb, const int *excl_off,
                      const int *excl_idx, int flags, nb_list **list);
void nb_list_free(nb_list *list);

/*
 * Second stage of a two-stage list (Sec. 2.3: a list built from bounding
 * boxes, then cluster pairs whose particles are all beyond a radius removed
 * with a particle-distance test, done on the GPU).  `*inner` receives the
 * entries of `outer` that hold a pair of real particles closer than r at the
 * positions xyzq_now, the i-particle moved by the entry's image shift; the
 * test is the search's own FP32 particle test (exclusions and the half-list
 * triangle do not enter it), so a list built with rbb = rlist and pruned at
 * rlist at its build positions equals the one-stage list built with rbb = 0.
 * Kept entries keep their order, masks and regions; `*inner` is a complete
 * list for nb_forces on outer's grid (same lifetime rules as outer).  With r
 * at least rc plus the distance any pair can close in until the next prune,
 * forces on the pruned list equal those on the outer one; a rolling prune
 * every few steps lets the outer list (and its search) live longer.
 *
 *   outer     a list built on the current sort of its grid; not modified
 *   xyzq_now  DEVICE float4[n], caller's order, the same array nb_forces takes
 *   r         prune radius (nm), > 0
 *   inner     in/out: NULL creates, otherwise reused; must not be outer
 * Asynchronous (no host synchronisation, capturable in a graph).  An outer
 * list that overflowed gives an inner list that reports NB_ERR_OVERFLOW at
 * nb_sync.  Non-finite positions are reported as by nb_forces.
 */
int nb_pairlist_prune(nb_ctx *ctx, const nb_list *outer, const float *xyzq_now, float r, nb_list **inner);

/*
 * Pair distance histogram: the pair correlation function, a limited-range
 * pair evaluation named in Sec. 1.  Sec. 2.3: with a list built for every
 * evaluation, build it from bounding boxes alone (rbb = rlist, no particle
 * prune); the kernel then has no cut-off conditional.  Every unordered pair
 * of real particles of the list closer than r_max (optionally skipping
 * force-field exclusions) is counted in bin k of its type pair:
 *   hist[(lo * ntypes + hi) * nbins + k] += 1,  lo <= hi the two types
 * (a type outside [0, ntypes) latches NB_ERR_ARG, as for nb_forces); the
 * (hi, lo) half stays untouched.  The bin is
 * decided in FP32: k is the largest with e_k <= r2, e_k = (float)((k dr)^2)
 * computed in FP64 with dr = r_max / nbins, and r2 the squared FP32
 * distance of the pair in its listed image.  Counts are exact (integer).
 *   list      built on grid; must hold every pair below r_max at xyzq_now
 *             (at its build positions any list with rlist >= r_max does)
 *   xyzq_now  DEVICE float4[n], caller's order
 *   r_max     histogram range (nm), 0 < r_max <= the list's rlist
 *   nbins     bins; the histogram and the edges must fit 64 KB of LDS:
 *             4 (ntypes^2 nbins + nbins + 1) + 512 bytes
 *   flags     0 or NB_RDF_SKIP_EXCLUDED
 *   hist      DEVICE uint64[ntypes * ntypes * nbins], added to (not cleared)
 * Asynchronous; the first call with new r_max or nbins uploads the bin edges
 * (one synchronisation).
 */
enum { NB_RDF_SKIP_EXCLUDED = 1 };
int nb_rdf(nb_ctx *ctx, const nb_grid *grid, const nb_list *list, const float *xyzq_now, float r_max, int nbins,
           int ntypes, int flags, unsigned long long *hist);

/* Synchronous.  Number of cluster-pair entries and force work items. */
int nb_list_info(nb_list *list, long *n_entries, long *n_items);

/* One cluster pair in canonical form: i-cluster, image shift index
 * s = 9(sx+1) + 3(sy+1) + (sz+1) (the i-cluster is moved by s.L), j-cluster,
 * and mask bit a*N + b for i-slot a, j-slot b. */
typedef struct { int32_t ci, shift, cj, pad; uint64_t mask; } nb_entry;

/* Synchronous.  Copies min(cap, n_entries) entries in canonical order to
 * HOST `out`, *count receives n_entries. */
int nb_list_export_canonical(nb_list *list, nb_entry *out, long cap, long *count);

/* ----------------------------------------------------------------- forces */

enum {
    NB_ENERGY = 1,       /* also compute LJ and Coulomb energies */
    NB_VIRIAL = 2,       /* also compute the virial sum over pairs of r_ij (x) F_i */
    NB_ACC_FP32 = 4,     /* accumulate energies/virial in FP32 end to end (precision study);
                            default is FP64 accumulation of FP32 pair terms */
    NB_ACCUMULATE = 8    /* add forces to f instead of overwriting */
};

/*
 * Pair interactions over the list (Sec. 3 "Pair interaction kernels";
 * Eq. 1 LJ, Eq. 2 Coulomb with the Ewald real-space correction
 * g(r) = d/dr[erf(beta r)/r], Sec. 2.4 exclusions).  For each listed pair with
 * r < rc: mask bit 1 -> LJ + erfc-screened Coulomb; mask bit 0 (force-field
 * exclusion) -> the Ewald correction -erf(beta r)/r only.
 *
 *   xyzq_now DEVICE float[4n]: current positions and charges, ORIGINAL order,
 *            not re-wrapped since nb_grid_sort (the grid's image counts apply)
 *   f        DEVICE float[3n] forces in original order (overwritten unless
 *            NB_ACCUMULATE)
 *   energy   DEVICE double[2] (E_LJ, E_Coulomb), written when NB_ENERGY
 *   virial   DEVICE double[9] row-major sum of r_ij (x) F_i, when NB_VIRIAL
 *
 * Forces are summed per particle in fixed point (each partial force rounded
 * to a multiple of 2^-16 kJ mol^-1 nm^-1).  Every addition is exact while a
 * particle's running sum stays below 2^53 units (1.4e11 kJ mol^-1 nm^-1),
 * which holds whenever its partial forces are below 2^26 (6.7e7) and number
 * at most 2^11; then the forces do not depend on the order of the partial
 * sums, and for a given list and positions they are reproducible bit for
 * bit.  Partial forces up to 2^36 are accepted (close contacts), and a sum
 * of such terms beyond 2^53 units may round.  A partial force of 2^36
 * kJ mol^-1 nm^-1 or more (overlapping particles) or a non-finite one makes
 * that particle's force NaN and latches NB_ERR_NONFINITE for nb_sync.
 */
int nb_forces(nb_ctx *ctx, const nb_grid *grid, const nb_list *list, const float *xyzq_now, const nb_params *p,
              unsigned flags, float *f, double *energy, double *virial);

/*
 * nb_forces for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, checks and results as nb_forces with the direct force
 * kernel (bit for bit: forces, energies and virial), but the energy/virial
 * partials of the work items and their block sums live in a static device
 * array of the library (NB_NOALLOC_SCRATCH_BYTES on every GPU the library
 * runs on, held until the process ends) instead of context memory, so the
 * call allocates, frees and uploads nothing and records no timers.
 * Requirements and limits:
 *   - the list has had a synchronous build (which sizes its storage);
 *   - the energy partials fit: (work-item capacity + 4) * 88 bytes, rounded up
 *     to 256, plus 22528 bytes, at most NB_NOALLOC_SCRATCH_BYTES (about
 *     190 000 work items, e.g. the 96 000-atom 8x8 list); NB_ERR_UNSUPPORTED
 *     otherwise, as for NB_COULOMB_EWALD_TABLE (it needs a device table);
 *   - the context's force-kernel variant is ignored (direct kernel).
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap in time on one GPU (other streams, contexts
 * or threads) race and must be serialised by the caller.
 */
enum { NB_NOALLOC_SCRATCH_BYTES = 16 << 20 };
int nb_forces_noalloc(nb_ctx *ctx, const nb_grid *grid, const nb_list *list, const float *xyzq_now,
                      const nb_params *p, unsigned flags, float *f, double *energy, double *virial);

/* Force-kernel variant used by nb_forces on this context.
 *   NB_FORCE_DIRECT (default): every listed pair is visited in lock-step with
 *     a per-lane cut-off branch (the cut-off conditional of the paper's GPU
 *     kernel); passes whose pairs are all beyond rc skip the interaction.
 *   NB_FORCE_SUPER: the super-cluster layout of the paper's GPU kernel
 *     (Sec. 2.3 and 3.2): 8 (or 4) consecutive i-clusters share one list
 *     of j-clusters, each with a bit per i-cluster it reaches, so each
 *     j-cluster's data is loaded and its j-force reduced and stored once per
 *     super-cluster.  The view is built from the list by the first force
 *     call after each build (or every call, for lists rebuilt inside a
 *     captured batch graph).  Applies to 8x8 lists whose reserved entries
 *     per i-cluster (all its search parts) are at most 512 (8 i-clusters
 *     per super-cluster) or 1024 (4); other lists use the direct kernel.
 * Results agree to rounding; the choice is a tuning knob.  Each variant's
 * forces are reproducible bit for bit for a given list and positions. */
enum { NB_FORCE_DIRECT = 0, NB_FORCE_SUPER = 2 };
int nb_set_force_variant(nb_ctx *ctx, int variant);

/* Super-cluster layout: i-clusters per super-cluster (4 or 8, or 0 for the
 * largest that fits) and super-cluster entries per force work item (one
 * wavefront each; 1..64, or 0 for the default 16).  Takes effect at the
 * next force call (which rebuilds the view). */
int nb_set_super_cluster(nb_ctx *ctx, int clusters, int entries);

/* Wavefronts that share the pair search of one i-cluster (each takes a
 * contiguous share of the candidate grid columns of every image shift): 1, 2,
 * 4 or 8, or 0 (default) to choose from the number of i-clusters so that small
 * systems still fill the GPU.  Takes effect at a list's next synchronous
 * build.  The list's content does not depend on it; the order of entries
 * within an i-cluster does (part by part). */
int nb_set_search_parts(nb_ctx *ctx, int parts);

/* ------------------------------------------------------- batched replicas */

/*
 * Many independent systems of one cluster shape (for example replicas of
 * uneven size, each too small to fill the GPU: the paper notes GPU kernels
 * need tens of thousands of particles to approach peak, Sec. 4.2) evaluated
 * in one launch.  Each replica keeps its own grid and list; the work items
 * of all replicas are concatenated on the device (a prefix of the replicas'
 * item counts, so list sizes never travel to the host) and split into eight
 * contiguous shares, one per XCD, one wavefront per item.  nb_batch_forces enqueues: batched coordinate gather,
 * force kernel, batched force scatter and per-replica energy
 * reduction -- no host synchronisation, no allocation, no memset, so the
 * sequence can be captured in a HIP graph (nb_batch_capture) and replayed.
 *   grids, lists        HOST arrays of n_rep handles (same shape); a replica's
 *                       list must be rebuilt after its grid is re-sorted
 *   xyzq_now, f         HOST arrays of n_rep DEVICE pointers bound to the
 *                       batch: positions (original order) and forces
 *   energy              DEVICE double[2*n_rep] (E_LJ, E_Coul per replica)
 *   virial              DEVICE double[9*n_rep]
 * If a replica's storage moved (a synchronous list build grew it), the next
 * nb_batch_forces refreshes the batch's tables (synchronously); a captured
 * graph must then be captured again (nb_batch_replay returns NB_ERR_STATE).
 * The graph keeps the params' c6c12 pointer and the output pointers passed
 * to nb_batch_capture.  Supported flags: NB_ENERGY, NB_VIRIAL, NB_ACCUMULATE.
 * Every Coulomb variant of nb_params (Eq. 2: analytic Ewald, reaction field,
 * tabulated Ewald); the tabulated variant's table is built in the context on
 * first use, and before a capture begins, so captured launches only read it.
 */
int nb_batch_create(nb_ctx *ctx, int n_rep, nb_grid *const *grids, nb_list *const *lists,
                    const float *const *xyzq_now, float *const *f, nb_batch **batch);
void nb_batch_free(nb_batch *batch);
/* Work items (wavefronts) per workgroup of the batched force kernel: 1, 2, 4 or 8 (default 4). */
int nb_batch_set_group(nb_batch *batch, int items_per_group);
/*
 * Wavefronts of the batched force kernel's main launch, which takes one work
 * item per wavefront.  0 (default): a quarter more than the replicas' work
 * items at their lists' last synchronous builds (plus 256), at most the
 * lists' capacity.  A second launch strides over the items beyond the main
 * launch's share (lists grown by later asynchronous or batched rebuilds), so
 * any value gives the same forces, bit for bit; a value above the total
 * only launches workgroups that exit at once.  Fails with NB_ERR_ARG for a
 * count outside [0, 2^28] and NB_ERR_STATE once the batch is captured.
 */
int nb_batch_set_grid(nb_batch *batch, long waves);
int nb_batch_forces(nb_ctx *ctx, nb_batch *batch, const nb_params *p, unsigned flags, double *energy, double *virial);
int nb_batch_capture(nb_ctx *ctx, nb_batch *batch, const nb_params *p, unsigned flags, double *energy,
                     double *virial);
int nb_batch_replay(nb_ctx *ctx, nb_batch *batch);

/*
 * Batched list rebuild: the grid sort (Sec. 2.3) and the pair search of
 * every replica, each stage one launch over all replicas, from the bound
 * positions.  Every replica's list must have had a synchronous build on its
 * grid (which sizes its regions); the rebuild then fills those regions like
 * an NB_LIST_ASYNC build, at the list's own rlist and rbb, latching
 * NB_ERR_OVERFLOW if a region overflows.  No host synchronisation.
 *   type, excl_off, excl_idx   HOST arrays of n_rep DEVICE pointers (each as
 *                              for nb_grid_sort / nb_pairlist_build)
 * nb_batch_bind_topology re-sizes (synchronously) any replica list whose
 * search is split over several wavefronts per i-cluster to one wavefront per
 * i-cluster: in a batched launch the replicas fill the GPU, and unsplit
 * regions give the force kernel full work items.
 * nb_batch_capture_cycle captures one rebuild followed by nsteps batched force
 * evaluations as a single graph, replayed with nb_batch_replay.
 */
int nb_batch_bind_topology(nb_batch *batch, const int *const *type, const int *const *excl_off,
                           const int *const *excl_idx);
int nb_batch_rebuild(nb_ctx *ctx, nb_batch *batch);
int nb_batch_capture_cycle(nb_ctx *ctx, nb_batch *batch, int nsteps, const nb_params *p, unsigned flags,
                           double *energy, double *virial);

/*
 * Autotuner for batched replicas.  The paper chooses the cluster shape M x N
 * to fit the SIMD width and the cost of the hardware (Sec. 2.2, Sec. 3.1); here
 * the fastest (shape, work items per workgroup) pair for a given set of
 * replicas is measured.  For each candidate shape every replica is grid-sorted
 * and its list built at rlist (rbb default), the lists are bound to one batch
 * (search unsplit, as nb_batch_bind_topology) and, for each candidate group,
 * the batched force launch (nb_batch_forces with `flags`) is run twice
 * untimed and `reps` times between HIP events on the context's stream.
 * Synchronous; every grid, list, batch and buffer it made is freed again.
 *   r          replicas: box edges (HOST double[3 n_rep]), particle counts
 *              (HOST int[n_rep]) and, per replica, DEVICE pointers to
 *              positions/charges, types and the exclusion CSR (HOST arrays of
 *              n_rep pointers, as for nb_grid_sort and nb_pairlist_build)
 *   rlist      list radius; every replica box edge must exceed 2 rlist
 *   p, flags   interaction parameters and NB_ENERGY / NB_VIRIAL, as timed
 *   shapes, n_shapes, groups, n_groups   candidates (groups: 1, 2, 4 or 8)
 *   reps       timed launches per candidate (>= 1)
 *   best, best_group  HOST outputs: the fastest candidate
 *   ms_table   HOST float[n_shapes * n_groups] (may be NULL): mean ms per
 *              launch, row = shape, column = group
 */
typedef struct {
    int n_rep;
    const double *box;
    const int *n;
    const float *const *xyzq;
    const int *const *type;
    const int *const *excl_off;
    const int *const *excl_idx;
} nb_replicas;
int nb_autotune(nb_ctx *ctx, const nb_replicas *r, float rlist, const nb_params *p, unsigned flags,
                const nb_shape *shapes, int n_shapes, const int *groups, int n_groups, int reps, nb_shape *best,
                int *best_group, float *ms_table);

/* ---------------------------------------------------------- exact recount */

/*
 * Missed-pair energy of a finite Verlet buffer, counted exactly (Sec. 5
 * "Effective pair list buffering"; the appendix bounds the same quantity).
 * The list must have been built on `grid` from the undisplaced positions at
 * a large radius rl with rbb = rl - c_bb.  A cluster pair is then listed at
 * any radius r <= rl iff tau = min(d_bb + c_bb, d_min) < r (bounding-box and
 * smallest particle distance at sort time).  For every real, non-excluded
 * pair of the half list whose displaced distance r_t is below p->rc, the
 * shifted potential V(r_t) - V(rc) (always shifted here) is added to
 * hist[min(floor((tau - rc)/db), nbins - 1)] when tau >= rc.  The missed
 * energy at buffer r_b = k*db is then sum(hist[k:]).
 *   xyzq_t  DEVICE float[4n] displaced positions, original order, in the same
 *           periodic images as the sorted positions (not re-wrapped)
 *   hist    DEVICE double[nbins], overwritten
 */
int nb_recount(nb_ctx *ctx, const nb_grid *grid, const nb_list *list, const float *xyzq_t, const nb_params *p,
               float c_bb, float db, int nbins, double *hist);

/* -------------------------------------------------------- buffer estimate */

/*
 * Verlet-buffer query (Sec. 5 "Effective pair list buffering" and appendix).
 * Per-type arrays are HOST pointers of length ntypes.
 */
typedef struct {
    double T;              /* temperature (K) */
    double dt;             /* time step (ps) */
    int nstlist;           /* list lifetime in steps */
    int ntypes;
    const double *mass;    /* u */
    const double *charge;  /* e */
    const double *c6c12;   /* ntypes*ntypes*2 */
    const double *count;   /* particles per type */
    double volume;         /* nm^3 */
    double rc, beta, coulomb_f;
    nb_shape shape;        /* cluster shape the list will use (learned mode) */
    double target;         /* allowed drift, kJ/mol/ps per particle */
} nb_buffer_query;

enum { NB_BUFFER_ANALYTIC = 0, NB_BUFFER_MLP = 1, NB_BUFFER_AUTO = 2 };

/*
 * Smallest buffer r_b (on a 0.0005 nm grid) whose estimated drift is within
 * q->target.  ANALYTIC: the appendix bound (free-particle Gaussian
 * displacements over t = (nstlist-1)*dt, second-order expansion of the
 * potential at rc, second-order term with 2 sigma^2 as the integral gives),
 * summed as 1/2 sum_a N_a sum_b |dV_ab| and divided by N*nstlist*dt; host
 * FP64.  MLP / AUTO: the learned predictor attached with nb_buffer_set_mlp
 * (its inference kernel on the context's stream, synchronous), giving
 * min(prediction + margin, analytic buffer); outside the model's feature
 * ranges, outside its training domain (nb_mlp_set_domain: a query with a
 * stricter target, another time step, another beta * rc or other charges or
 * LJ parameters than the model's labels were generated for, or a model with
 * no recorded domain), for a non-finite prediction, or (AUTO) without a
 * model, the analytic buffer is returned and *used_fallback = 1.  MLP
 * without a model: NB_ERR_STATE.
 *   ctx        may be NULL for ANALYTIC
 *   rb_out     nm;  drift_out  analytic drift estimate at *rb_out
 */
int nb_buffer_estimate(nb_ctx *ctx, const nb_buffer_query *q, int mode, double *rb_out, double *drift_out,
                       int *used_fallback);

/* ------------------------------------------------ learned buffer predictor */

/*
 * A small multilayer perceptron that predicts the minimal Verlet buffer from
 * 8 features: temperature (K), mass-weighted displacement width
 * sqrt(kB T t^2 <1/m>) (nm, t = (nstlist-1) dt), list lifetime (steps), mass
 * density (g/cm^3), cut-off (nm), and the cluster shape one-hot
 * (4x4, 4x8, 8x8; other shapes take the analytic bound).  It is trained on
 * labels from nb_recount (the paper's
 * drift criterion evaluated exactly, Sec. 5).  Architecture 8-64-64-1, tanh
 * hidden layers, softplus output, MSE loss, Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8); features are normalised to [-1, 1] with the ranges lo/hi given
 * at creation.  Parameters: NB_MLP_PARAMS floats, order W1 (64x8 row-major),
 * b1, W2 (64x64 row-major), b2, w3, b3.  Kernels run on the context's stream.
 *   X  DEVICE float[batch*8] raw features, row-major;  y  DEVICE float[batch]
 */
enum { NB_MLP_FEATURES = 8, NB_MLP_PARAMS = 4801 };
int nb_mlp_create(nb_ctx *ctx, const float *params_host, const double lo[8], const double hi[8], nb_mlp **mlp);
void nb_mlp_free(nb_mlp *mlp);
/* Synchronous copy of the current parameters to HOST params[NB_MLP_PARAMS]. */
int nb_mlp_get_params(nb_mlp *mlp, float *params);
/* One Adam step on a minibatch (one workgroup); loss: DEVICE float or NULL. */
int nb_mlp_train_step(nb_ctx *ctx, nb_mlp *mlp, const float *X, const float *y, int batch, float lr, float *loss);
/* Gradient of the batch loss (DEVICE float[NB_MLP_PARAMS]) without updating the model. */
int nb_mlp_grad(nb_ctx *ctx, nb_mlp *mlp, const float *X, const float *y, int batch, float *grad, float *loss);
int nb_mlp_infer(nb_ctx *ctx, const nb_mlp *mlp, const float *X, int batch, float *y);
/* Record the conditions the model's labels were generated for: q->target,
 * q->dt, q->beta * q->rc (relative tolerance 5e-3), and the per-type charges
 * and C6/C12 table (relative 1e-9); the other fields of q are ignored.  The
 * learned modes of nb_buffer_estimate answer only queries inside this domain
 * (Sec. 5: the buffer is chosen for a given drift target and potential). */
int nb_mlp_set_domain(nb_mlp *mlp, const nb_buffer_query *q);
/* Attach (mlp != NULL) or detach the predictor used by nb_buffer_estimate;
 * margin (nm) is added to its prediction. */
int nb_buffer_set_mlp(nb_ctx *ctx, const nb_mlp *mlp, double margin);

/* ------------------------------------------------------------ instrumentation */

/* Pair statistics of a list at the given positions (Sec. 5: the effective
 * pair ratio counts only pairs within the cut-off).  Synchronous.  HOST
 * counts[4]: [0] listed pairs (entries * M * N), [1] real pairs the kernel
 * visits (dummies and the lower triangle of self pairs excluded), [2]
 * interacting pairs with r < rc, [3] force-field-excluded pairs with r < rc.
 * xyzq_now as in nb_forces. */
int nb_list_stats(nb_ctx *ctx, const nb_grid *grid, const nb_list *list, const float *xyzq_now, float rc,
                  long long *counts);

/* Kernel timing with HIP events recorded on the context's stream around the
 * force kernel, the whole nb_forces call, nb_grid_sort and nb_pairlist_build.
 * Off by default.  on: 0 off, 1 every timer, or NB_TIMING_SELECT with the
 * bits 1 << NB_TIMER_* of the timers wanted (each recorded event costs a few
 * microseconds of stream time, so a caller timing a long sequence can time
 * a sample of its launches).  nb_timing_read synchronises, returns the
 * summed elapsed milliseconds and the number of timed launches per timer
 * since the last read (HOST arrays of NB_TIMER_COUNT), and resets. */
enum { NB_TIMER_FORCE_KERNEL = 0, NB_TIMER_FORCE_CALL = 1, NB_TIMER_GRID_SORT = 2, NB_TIMER_PAIRLIST = 3,
       NB_TIMER_COUNT = 4 };
enum { NB_TIMING_SELECT = 0x100 };
int nb_timing_enable(nb_ctx *ctx, int on);
int nb_timing_read(nb_ctx *ctx, double *ms, long *launches);

#ifdef __cplusplus
}
#endif
#endif
