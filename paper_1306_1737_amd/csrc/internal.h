// Internal declarations of the MI355X cluster-pair library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mxn.h"

namespace mxn {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);

#define MXN_HIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return ::mxn::fail(e_ == hipErrorOutOfMemory ? NB_ERR_OOM : NB_ERR_HIP,                \
                               std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)

// bits latched by kernels in ctx->d_flags
enum : int { FLAG_NONFINITE = 1, FLAG_OVERFLOW = 2, FLAG_FORCE_RANGE = 4, FLAG_TYPE = 8 };

// work items of the force kernel hold at most this many j-entries of one i-cluster
// Entries per force work item: four wavefront passes of 64/N entries each.
constexpr int item_entries(int n) { return 256 / n; }
constexpr int kHistAtoms = 4096;         // particles per workgroup in the column histogram
constexpr int kMaxHistColumns = 16384;   // larger grids count columns with global atomics
inline int hist_blocks(int n) { return n < 1 ? 1 : (n + kHistAtoms - 1) / kHistAtoms; }
constexpr int kMaxSearchParts = 8;   // wavefronts that may share the pair search of one i-cluster
constexpr int kMaxTypes = 32;

// Live device bytes of one context's handles, by source (nb_memory_info).
struct MemCount {
    std::atomic<size_t> via_allocator{0}, via_hip{0};
};

// A device buffer owned by a handle.  It remembers the allocator (and the
// stream) it came from, so that it is returned to the same one.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    nb_allocator al{};          // al.alloc == nullptr: hipMalloc / hipFree
    void *stream = nullptr;     // stream given to al.alloc, passed back to al.free
    std::shared_ptr<MemCount> mem;
};
// grow-only device allocation through the context's allocator (hipMalloc without one)
int ensure(const ::nb_ctx *c, DevBuf &b, size_t bytes);
void release(DevBuf &b);

}  // namespace mxn

// Cluster-pair list entry as the kernels use it (16 bytes): j-cluster, image
// shift index, and the M*N mask in j-major bit order (bit b*M + a).
struct nb_jentry {
    int cj;
    int shift;
    uint32_t mlo, mhi;
};

struct nb_mlp;

struct nb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    nb_allocator alloc{};       // caller's device allocator (alloc == nullptr: hipMalloc)
    std::shared_ptr<mxn::MemCount> mem = std::make_shared<mxn::MemCount>();
    mxn::DevBuf flags_buf;      // holds d_flags
    mxn::DevBuf stats_buf;      // nb_list_stats counters
    int *d_flags = nullptr;     // latched kernel errors
    void *noalloc_scratch = nullptr;   // device address of nb_forces_noalloc's static scratch (set at creation)
    std::string noalloc_error;         // why it is null
    int *h_pinned = nullptr;    // pinned host scratch (16 ints)
    mxn::DevBuf partials;       // per-work-item energy/virial partials
    mxn::DevBuf blockpart;      // sums of the partials over contiguous shares of the work items
    mxn::DevBuf etab;           // Ewald table of the tabulated Coulomb variant
    mxn::DevBuf rdf_edge;       // squared bin edges of the pair distance histogram
    float rdf_rmax = -1.0f;
    int rdf_nbins = 0;
    float etab_beta = -1.0f, etab_rc = -1.0f;
    int timing = 0;   // bit k: timer k records events
    int force_variant = NB_FORCE_DIRECT;
    int sci_clusters = 0;   // i-clusters per super-cluster (0: the largest that fits)
    int sci_per_item = 0;   // super-cluster entries per work item (0: default)
    int search_parts = 0;   // 0: chosen from the number of i-clusters
    const nb_mlp *mlp = nullptr;   // attached buffer predictor (nb_buffer_set_mlp)
    double mlp_margin = 0.0;
    mxn::DevBuf mlp_io;            // one feature row and one output for nb_buffer_estimate
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timers[NB_TIMER_COUNT];
    std::vector<hipEvent_t> event_pool;
};

struct nb_grid {
    nb_ctx *ctx = nullptr;
    int n = 0, m = 0, nn = 0, cmin = 0, cmax = 0;
    int nx = 0, ny = 0, ncol = 0;
    int slots_cap = 0;          // n + ncol*(cmax-1): upper bound of the padded slot count
    double box[3] = {0, 0, 0};
    float Lf[3] = {0, 0, 0};
    double invL[3] = {0, 0, 0};
    float inv_x = 0, inv_y = 0;
    double spacing = 0;
    // device storage
    mxn::DevBuf col_count, col_start, col_fill, colbb, col_hist;
    mxn::DevBuf atom_col, atom_xw, atom_img, bucket;
    mxn::DevBuf xs, xs_now, type_s, perm, img_s, slot_of;
    mxn::DevBuf bbi_lo, bbi_hi, bbj_lo, bbj_hi;
    mxn::DevBuf nslots;        // int on device
    mxn::DevBuf shiftvec;      // 27 float4 image shift vectors
    long generation = 0;       // incremented by every sort; lists remember the one they were built on
};

struct nb_list {
    const nb_grid *grid = nullptr;
    nb_ctx *ctx = nullptr;
    float rlist = 0, rbb = 0;
    long cap_entries = 0;
    long cap_items = 0;
    // Entries live in equal regions, one per (i-cluster, search part):
    // part_start holds the region starts (sized by a synchronous build),
    // part_count the entries found by the latest build.
    mxn::DevBuf entries, items;        // entries: canonical order, or by bounding-box distance
    mxn::DevBuf entries_canon, keys;   // fill-pass output before a distance sort, and its sort keys
    mxn::DevBuf part_count, part_start, part_istart;
    mxn::DevBuf totals;        // int[4]: entries, items, usable items (0 after an overflow), region overflow
    // j-cluster view, rebuilt with the list: entries per j-cluster (counters,
    // zero between builds), their exclusive scan (first row of each j-cluster),
    // and for each entry position its rank among the j-cluster's entries,
    // turned into its row jstart[cj] + rank by the build's last pass
    // (jrank_canon: the fill pass's ranks before a distance sort)
    mxn::DevBuf jcount, jstart, jrank, jrank_canon;
    // force-call buffers: j-force (x, y, z) per (row, j-particle), rows grouped
    // by j-cluster, and float4 i-force per (work item, i-particle); summed per
    // cluster after the force kernel
    mxn::DevBuf fj, fi;
    int resv_parts = 0;        // search parts of the reserved layout (0: none yet)
    int resv_nci = 0;          // i-cluster capacity of the reserved layout
    long resv_size = 0;        // entries per region of the reserved layout
    long est_items = 0;        // work items of the last synchronous build (sizes the force-kernel grid)
    long cap_rows = 0;         // j-force rows fj holds: the last synchronous build's entries plus a quarter
    long last_entries = 0;     // host copy after a synchronous build
    long grid_generation = -1;
    // Super-cluster view (8x8 lists; the grouped force kernel): a cache built
    // from the list by the first force call after each build.  Entries and
    // masks use the list's capacity; rows reuse fj; items, their i-forces and
    // the j-cluster counters, starts and totals are its own.
    mutable mxn::DevBuf sci_ent, sci_mask, sci_count, sci_base, sci_istart, sci_items, sci_jcount, sci_jstart,
        sci_totals, sci_fi;
    mutable long sci_cap_items = 0, sci_njc = 0;
    mutable int sci_S = 0, sci_per_item = 0;
    mutable bool sci_valid = false;   // built from the list's latest build
    bool sci_volatile = false;        // rebuilt inside a captured graph: the view is rebuilt by every call
};

struct nb_batch {
    nb_ctx *ctx = nullptr;
    int n_rep = 0, m = 0, nn = 0, waves = 4, ncu = 1;
    long grid_waves = 0;   // main force-launch wavefronts (0: from the lists' item estimates)
    long total_slots = 0, total_atoms = 0, pstride = 0;
    std::vector<nb_grid *> grids;
    std::vector<nb_list *> lists;
    std::vector<long> generations;
    mxn::DevBuf desc, slot_off, atom_off, item_off, partials;
    std::vector<char> desc_host;   // the replica table as last copied to the device
    // batched rebuild (grid sort + list fill of every replica)
    std::vector<const float *> xyzq;
    std::vector<const int *> type, excl_off, excl_idx;
    bool topology = false;
    bool cycle = false;   // the captured graph holds the rebuild too
    mxn::DevBuf gjobs, ljobs, goff, loff, scans;
    std::vector<char> gjobs_host, ljobs_host;   // job tables as last copied to the device
    std::vector<int> gtotal, ltotal;
    int max_ncol = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t capture_stream = nullptr;
};

struct nb_mlp {
    nb_ctx *ctx = nullptr;
    mxn::DevBuf params, m, v, step, lo, hi;
    double lo_h[8] = {0}, hi_h[8] = {0};
    // the conditions the model's labels were generated for (nb_mlp_set_domain):
    // drift target, time step, beta * rc and the interaction parameters per type
    bool has_domain = false;
    double dom_target = 0, dom_dt = 0, dom_brc = 0;
    int dom_ntypes = 0;
    std::vector<double> dom_charge, dom_c6c12;
};

namespace mxn {

constexpr int kMlpParams = 4801;
int launch_batch(nb_ctx *ctx, nb_batch *b, const nb_params *p, unsigned flags, double *energy, double *virial);
int prepare_coulomb(nb_ctx *ctx, const nb_params *p);
// largest rc of the tabulated Ewald variant: its table (8 KB per nm) and the LJ rows (up to 16.4 KB) stay
// within a workgroup's 64 KB of LDS
constexpr float kMaxTableRc = 4.0f;
size_t rep_desc_size();
// batched list rebuild (grid sort and pair search of many replicas, one launch per stage)
struct ScanJob {
    const int *in;
    int *out;
    int n, mode, p;
    int *total, *raw_total;
    int *clear;   // the input, zeroed once read (or null)
};
void launch_scan_batch(const ScanJob *jobs, int n_jobs, hipStream_t st);
size_t grid_job_size();
int grid_job_stages();
bool grid_batchable(const nb_grid *g);
void fill_grid_job(void *out, const nb_grid *g, const float *xyzq, const int *type);
void grid_job_blocks(const nb_grid *g, int *blocks_per_stage);
int launch_grid_sort_batch(hipStream_t st, const void *jobs, const int *off, int n_rep, const int *total, int max_ncol);
size_t list_job_size();
int list_job_stages();
void fill_list_job(void *out, nb_list *l, const int *excl_off, const int *excl_idx, ScanJob *scan,
                   ScanJob *jscan);
void list_job_blocks(const nb_list *l, int *blocks_per_stage);
int launch_pairlist_batch(hipStream_t st, int m, int nn, const void *jobs, const int *off, int n_rep, const int *total,
                          const ScanJob *scans);
void fill_rep_desc(void *out, const nb_grid *g, const nb_list *l, const float *xyzq_now, float *f, long pbase);
int launch_mlp_step(nb_ctx *ctx, nb_mlp *mlp, const float *X, const float *y, int batch, float lr, float *loss,
                    float *grad_out);
int launch_mlp_infer(nb_ctx *ctx, const nb_mlp *mlp, const float *X, int batch, float *y);

// kernel launchers (grid.hip, pairlist.hip, forces.hip)
int launch_grid_sort(nb_grid *g, const float *xyzq, const int *type);
int launch_pairlist(nb_list *l, const int *excl_off, const int *excl_idx, bool sync, bool by_distance);
// noalloc: the device address of the static scratch (nb_forces_noalloc), or null
int launch_forces(nb_ctx *ctx, const nb_grid *g, const nb_list *l, const float *xyzq_now, const nb_params *p,
                  unsigned flags, float *f, double *energy, double *virial, void *noalloc = nullptr);
// device address of nb_forces_noalloc's static scratch on the current device
int noalloc_scratch_address(void **ptr);
// event-pair timing on the context stream (no-ops unless enabled)
struct ScopedTimer {
    nb_ctx *ctx;
    int which;
    hipEvent_t stop = nullptr;
    ScopedTimer(nb_ctx *c, int w);
    ~ScopedTimer();
};
int launch_recount(nb_ctx *ctx, const nb_grid *g, const nb_list *l, const float *xyzq_t, const nb_params *p, float c_bb,
                   float db, int nbins, double *hist);
int launch_stats(nb_ctx *ctx, const nb_grid *g, const nb_list *l, const float *xyzq_now, float rc,
                 unsigned long long *d_counts);
// second stage of a two-stage list: `in` gets outer's entries with a pair within r
// at the grid's gathered positions (xs_now)
int launch_prune(nb_list *in, const nb_list *outer, float r);
// coordinate gather into the grid's slot order; with nt > 0 it also latches
// FLAG_TYPE for a particle whose LJ type is not below nt
int launch_gather(nb_ctx *ctx, const nb_grid *g, const float *xyzq_now, int nt = 0);
// super-cluster view of an 8x8 list: i-clusters per super-cluster (0: none) and the build
constexpr int kSciPerItem = 16;
int sci_size(const nb_list *l, int want);
int launch_sci_view(const nb_list *l, int S, int per_item);
// pair distance histogram at the grid's gathered positions (xs_now)
size_t rdf_lds_bytes(int nbins, int nt);
int launch_rdf(nb_ctx *ctx, const nb_grid *g, const nb_list *l, float r_max, int nbins, int nt, int skip_excl,
               unsigned long long *hist);

}  // namespace mxn
