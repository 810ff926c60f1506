// Internal declarations shared by the device sources of libsphmap.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sphmap.h"

namespace sphmap {

// ------------------------------------------------------------ error model
struct Error {
  int code;
  std::string msg;
};

#define SPH_HIP(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      throw ::sphmap::Error{SPHMAP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)};      \
  } while (0)

#define SPH_REQUIRE(cond, code, what)                                                              \
  do {                                                                                             \
    if (!(cond)) throw ::sphmap::Error{code, std::string(what)};                                   \
  } while (0)

#define SPH_LAUNCH_CHECK() SPH_HIP(hipGetLastError())

// --------------------------------------------------------- device buffers
struct Buffer {
  void *p = nullptr;
  size_t bytes = 0;
};

// Device blocks given back by freed pair lists, kept by size for the next
// allocations of the same context (a caching allocator: repeated steps make
// no hipMalloc or hipFree).  take() hands out the smallest kept block of at
// least `bytes` and under twice that; put() keeps a block while the kept
// total stays within `cap` and returns it to the device otherwise.  Only
// blocks that no queued work still uses may be put back.
struct BlockPool {
  std::multimap<size_t, void *> blocks;
  size_t held = 0;
  size_t cap = 0;
  void *take(size_t bytes, size_t &got);
  void put(void *p, size_t bytes);
  void trim();  // frees the largest blocks until the kept total is within cap
  void release();
  ~BlockPool() { release(); }
};

// A cap on the device bytes a context's scratch may hold (its workspace).
// limit = 0: no cap.  `required` records the most a refused call asked for.
struct Budget {
  size_t limit = 0;
  size_t held = 0;
  size_t required = 0;
};

// Grow-only device allocations keyed by purpose, owned by a context or a
// handle.  get() never shrinks; contents are not preserved on growth.  With
// a pool, first allocations come from it and release() gives the blocks
// back to it.  With a budget, growth that would take the budget's holdings
// past its limit fails with SPHMAP_ENOMEM before anything is allocated.
struct Arena {
  std::map<std::string, Buffer> bufs;
  BlockPool *pool = nullptr;
  Budget *budget = nullptr;
  // fixed-region mode: buffers are carved in turn (256-byte aligned) from
  // [region, region + region_cap); nothing is allocated or freed, and a
  // request past the end fails with SPHMAP_EINVAL
  char *region = nullptr;
  size_t region_cap = 0, region_used = 0;
  // while set, every request goes to that arena instead
  Arena *redirect = nullptr;
  void *get(const std::string &name, size_t bytes);
  template <typename T>
  T *get(const std::string &name, size_t count) {
    return (T *)get(name, count * sizeof(T) + 16);
  }
  void release();
  ~Arena() { release(); }
};

// ----------------------------------------------------------------- timing
struct TimerRecord {
  hipEvent_t start, stop;
};

struct PairsDev;

// a launch shape chosen by the autotuner
struct TuneChoice {
  int blocks_per_cu;
  int per_fetch;
  double ms;
};

struct Ctx {
  int device = 0;
  PairsDev *scratch_pairs = nullptr;  // pair list of calls that do not keep one
  Budget ws;                          // workspace cap over arena and scratch pair lists
  Arena arena;
  std::string last_error;
  bool timing = false;
  bool counting = false;
  std::map<std::string, std::vector<TimerRecord>> timers;
  int64_t counters[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t *d_counters = nullptr;  // device copy of the work counters
  int *d_status = nullptr;        // device status word (non-finite results)
  void *pinned = nullptr;         // pinned host staging for small tables
  size_t pinned_bytes = 0;
  std::vector<PairsDev *> scratch_batch;  // pair lists of batched calls that do not keep them
  BlockPool pool;                         // blocks of freed retained pair lists
  int n_cu = 0, exact_per_cu = 0;  // compute units; resident Exact workgroups per CU
  bool autotune = false;
  std::map<int, TuneChoice> tuned;  // by floor(log2(pairs)) of the Exact launch
  // A second stream (default priority) for work that can overlap the
  // caller's, forked from and joined back to it by the two events.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t side_stream() {
    if (!side) {
      SPH_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
      SPH_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
      SPH_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
    }
    return side;
  }
  // Pinned host staging of at least `bytes`.  Its previous contents must no
  // longer be needed by queued copies (every forward call synchronises its
  // stream once, for the pair count, before it stages a table).
  void *pinned_get(size_t bytes) {
    if (pinned_bytes < bytes) {
      if (pinned) {
        SPH_HIP(hipDeviceSynchronize());
        SPH_HIP(hipHostFree(pinned));
        pinned = nullptr;
        pinned_bytes = 0;
      }
      SPH_HIP(hipHostMalloc(&pinned, bytes + 4096, hipHostMallocDefault));
      pinned_bytes = bytes + 4096;
    }
    return pinned;
  }
};

// RAII scope that records events around one launch when timing is on.
struct KernelTimer {
  Ctx *ctx;
  const char *name;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  KernelTimer(Ctx *c, const char *n, hipStream_t st) : ctx(c), name(n), s(st) {
    if (ctx->timing) {
      SPH_HIP(hipEventCreate(&a));
      SPH_HIP(hipEventCreate(&b));
      SPH_HIP(hipEventRecord(a, s));
    }
  }
  void done() {
    if (a) {
      SPH_HIP(hipEventRecord(b, s));
      ctx->timers[name].push_back({a, b});
      a = b = nullptr;
    }
  }
  ~KernelTimer() {
    if (a) {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  }
};

// ------------------------------------------------------------ tessellation
struct TessDev {
  int64_t n_cells = 0, n_faces = 0, n_vertices = 0, n_fv = 0;
  int device = 0;
  double box_lo[3] = {0, 0, 0};  // bounding cube of the vertices
  double box_size = 1.0;
  Arena mem;
  // as given
  double *gen = nullptr;          // [C][3]
  double *vert = nullptr;         // [V][3]
  int64_t *cell_face_off = nullptr;
  int64_t *face_vtx_off = nullptr;
  int32_t *face_vtx = nullptr;
  // prepared on the device
  int32_t *face_cell = nullptr;   // [F]
  double4 *fplane = nullptr;      // outward unit normal, plane offset about g (<= 0: skip face)
  double4 *fsphere = nullptr;     // centroid about g, radius
  double *fvpos = nullptr;        // [FV][3] oriented vertex positions about g
  float4 *fvpos32 = nullptr;      // [FV] binary32 copies (w unused)
  float4 *fplane32 = nullptr;     // binary32 copies of fplane
  // per face-vertex slot k, the edge from slot k to the next slot of its face
  // (binary32): start vertex about g and length; unit direction; in-plane
  // normal n x e (pointing into the polygon)
  float4 *edgeA = nullptr;        // [FV] A.xyz, |B - A|
  float4 *edgeE = nullptr;        // [FV] e.xyz, 0
  float4 *edgeM = nullptr;        // [FV] m.xyz, 0
  double *volume = nullptr;       // [C]
  float *radius = nullptr;        // [C]
  float4 *gen32 = nullptr;        // [C] fl(g), R_c in w
  int32_t *cell_order = nullptr;  // [C] cells in Morton order of the generators
  int32_t *face_nbr = nullptr;    // [F] neighbour each face faces (grids built here, or declared)
  // [F] the other cell of a face shared with it (verified), -1 otherwise;
  // nullptr when no face is shared (every face is evaluated from its own side)
  int32_t *face_twin = nullptr;
  int32_t *twin_face = nullptr;   // [F] the matching face of the twin cell
  // [F] the face's role in the mixed path: its slot among the cell's shared
  // faces that it evaluates (>= 0), -1 evaluated for this cell only, or
  // -2 - s when the twin evaluates it in its slot s
  int32_t *face_code = nullptr;
  int32_t *cell_slots = nullptr;  // [C] shared faces the cell evaluates
};

// ---------------------------------------------------------------- pairs
struct PairsDev {
  int64_t n_pairs = 0, n_cells = 0, n_particles = 0;
  int device = 0;
  Arena mem;
  int64_t *cell_off = nullptr;  // [C+1]
  int32_t *pair_p = nullptr;    // [P]
  int32_t *pair_c = nullptr;    // [P]
  double *w = nullptr;          // [P]
  int64_t *part_off = nullptr;  // [N+1]
  int32_t *pm_cell = nullptr;   // [P] particle-major cell index
  double *pm_w = nullptr;       // [P] particle-major weights
  double *coverage = nullptr;   // [N]
  // capacity mode (graph-captured batches): cap > 0 sizes the lists for cap
  // pairs and keeps the count on the device
  int64_t cap = 0;
  int64_t *d_np = nullptr;      // the pair count (0 when it passed cap)
  int32_t *d_over = nullptr;    // 1 when the count passed cap (list emptied)
  int32_t *d_flag = nullptr;    // or-ed with every overflow of the plan
};

// ---------------------------------------------------------- primitives
// exclusive scan of n int64 values in place-safe (in may equal out);
// returns nothing; the total is written to out[n] if write_total.
void scan_exclusive_i64(Arena &ar, const int64_t *in, int64_t *out, int64_t n, bool write_total, hipStream_t s);
// stable LSD radix sort of (key, value) pairs on the low `bits` bits.
void radix_sort_u64(Arena &ar, uint64_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s);
// Stable sort by key bits [lo, hi) only (the order of keys equal there is kept).
void radix_sort_u64_range(Arena &ar, uint64_t *keys, int32_t *vals, int64_t n, int lo, int hi, hipStream_t s);
void radix_sort_u32(Arena &ar, uint32_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s);
// Stable sort of n (key, a, b) triples by the low `bits` bits of key, from the
// input arrays into the output arrays (which must not overlap them).  dn: a
// device count of at most n items to sort instead (the launches cover n).
void sort_by_key_kv(Arena &ar, int64_t n, int bits, const uint32_t *kin, const int32_t *ain, const double *bin,
                    uint32_t *kout, int32_t *aout, double *bout, hipStream_t s, const int64_t *dn = nullptr);
// 63-bit Morton keys (21 bits per axis) of points in [lo, lo+size)^3,
// interleaved x (bit 0), y (bit 1), z (bit 2) at each level.
void morton_keys(const double *xyz, int stride, int64_t n, double lo0, double lo1, double lo2, double size,
                 uint64_t *keys, int32_t *idx, hipStream_t s);
void fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);
void iota_i32(int32_t *p, int64_t n, hipStream_t s);

// ------------------------------------------------------------ launchers
void tess_prepare(Ctx &ctx, TessDev &t, hipStream_t s);
// face twins from each face's declared neighbour (d_nbr [F] device; nullptr
// clears them); returns the number of shared faces
int64_t tess_set_twins(Ctx &ctx, TessDev &t, const int32_t *d_nbr, hipStream_t s);

struct PartDev {
  int64_t n;
  const double *xyz;  // [n][3]
  const double *h;
  const double *m;
  float4 *x32;        // fl(x), fl(y), fl(z), fl(h)
};
void particles_prepare(Ctx &ctx, PartDev &p, hipStream_t s);

// candidate pairs into P (allocates P's cell_off/pair_p/pair_c)
void find_pairs(Ctx &ctx, const TessDev &t, const PartDev &p, PairsDev &P, hipStream_t s);
// weights
void exact_integral(Ctx &ctx, const TessDev &t, const PartDev &p, PairsDev &P, int precision, hipStream_t s);
// several independent instances in one persistent launch
struct ExactJob {
  const TessDev *t;
  const PartDev *p;
  PairsDev *P;
};
// the instance table of a batch whose pair counts stay on the device: the
// pointer table (uploaded once), chunk offsets, and each instance's count
struct ExactTable {
  void *insts = nullptr;
  int64_t *chunk0 = nullptr;
  const int64_t **np = nullptr;
  int32_t *flag = nullptr;  // set when a step's gift slots pass their capacity
  void *gifts = nullptr;    // the plan of the shared faces' gifts (exact.hip)
};
void exact_integral_batch(Ctx &ctx, const std::vector<ExactJob> &jobs, int precision, hipStream_t s,
                          const ExactTable *tab = nullptr);
// gift buffers from `mem` (held with the plan); headroom as for the pair lists
void exact_table_upload(Ctx &ctx, const std::vector<ExactJob> &jobs, ExactTable &tab, Arena &mem, double headroom,
                        hipStream_t s);
void exact_table_free(ExactTable &tab);
size_t exact_inst_bytes();

// A batch of forward mappings captured as one HIP graph (batch.hip).
constexpr int kBatchBranches = 4;
struct BatchPlan {
  int n_inst = 0;
  bool normalize = false;
  std::vector<const TessDev *> t;
  std::vector<PartDev> pd;
  std::vector<std::unique_ptr<PairsDev>> P;
  std::vector<double *> mass, dens, cov;
  std::vector<Arena> scratch;  // one per branch stream
  std::vector<int64_t> n_max;  // largest instance of each branch
  hipStream_t origin = nullptr;  // the stream the step was captured on
  std::vector<hipStream_t> branch;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  Arena mem;
  int64_t *d_np = nullptr;
  int32_t *d_over = nullptr, *d_flag = nullptr;
  ExactTable tab;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchPlan() = default;
  BatchPlan(const BatchPlan &) = delete;
  BatchPlan &operator=(const BatchPlan &) = delete;
  ~BatchPlan();
};
void batch_plan_build(Ctx &ctx, BatchPlan &B, double headroom, hipStream_t s);
void batch_plan_run(Ctx &ctx, BatchPlan &B, hipStream_t s);
void batch_plan_check(Ctx &ctx, BatchPlan &B, hipStream_t s, int64_t *h_pairs, int32_t *overflow);
// upper bound of the context scratch the Exact integral of n_pairs pairs takes
size_t exact_workspace_bytes(Ctx &ctx, int64_t n_pairs);
// transpose + coverage
void particle_major(Ctx &ctx, PairsDev &P, hipStream_t s);
// M_c and rho_c (scale: optional per-particle mass factor 1/c_i)
void cell_reduce(Ctx &ctx, const TessDev &t, const PartDev &p, const PairsDev &P, bool normalize, double *mass,
                 double *rho, hipStream_t s);
void reverse_map(Ctx &ctx, const PairsDev &P, const double *cell_values, int ncomp, double *out, hipStream_t s);

struct PseudoArgs {
  int64_t n;
  const double *xyz, *h, *m;
  int n_src;
  const double *src;  // host [n_src][3]
  sphmap_pseudo_opts opts;
  int64_t capacity;
  double *o_xyz, *o_h, *o_m, *o_s;
  int32_t *o_kind;
  int64_t *o_first, *o_count;
  int32_t *o_branch;
  uint64_t *o_label = nullptr;            // node label of each entry's unit
  int64_t *o_owner = nullptr;             // [n] entry that holds each particle
  int64_t n_open = 0;                     // labels of nodes to open (device)
  const uint64_t *open_labels = nullptr;
  int64_t n_out;
  sphmap_pseudo_stats stats;
};
void pseudo_build(Ctx &ctx, PseudoArgs &a, hipStream_t s);
// node smoothing lengths of the np pseudo-particles plist (entries) over the
// nu units upos; n_mid > 0: trial neighbours from the k_mid neighbour-find
void node_hsolve(Ctx &ctx, int64_t np, const int32_t *plist, int64_t nu, const double4 *upos, const double *o_xyz,
                 const double *o_s, double hfact, double eps, int64_t bypass, double *o_h, int32_t *o_branch,
                 unsigned long long *bcount, int64_t n_mid, const double4 *mid_com, const int32_t *mid_u0,
                 const int32_t *mid_u1, const double *rcut, hipStream_t s);
// pseudo-particles from the k-d tree (recursive coordinate bisection)
struct KdArgs {
  PseudoArgs base;  // opts.leaf_max unused; max_depth up to 62
  double r_leaf;
  int32_t leaf_split, up_levels;
  int64_t nf_threshold;
  int32_t *o_level = nullptr;
  int32_t k_mid = -1;
};
void kd_pseudo_build(Ctx &ctx, KdArgs &a, hipStream_t s);
// labels of under-resolved pseudo-particles (eq. resol_param), entry order
int64_t select_underresolved(Ctx &ctx, int64_t n, const int32_t *kind, const uint64_t *label, const double *s_node,
                             const double *fneu, double s_root, double K, uint64_t *out, hipStream_t s);

// Voronoi grid of n generators in the box after n_lloyd Lloyd iterations
void voronoi_build(Ctx &ctx, TessDev &t, int64_t n, const double *d_gen, const double lo[3], const double hi[3],
                   int n_lloyd, double *d_gen_out, hipStream_t s);
// per-particle values from the mixed set (Sec. 3.3)
void interpolate_particles(Ctx &ctx, int64_t n, const double *xyz, const int64_t *owner, int64_t ne,
                           const double *exyz, const double *eh, const int32_t *ekind, const double *val, int ncomp,
                           double *out, hipStream_t s);
// the same with its scratch in the device's fixed region (no allocation)
void interpolate_particles_noalloc(Ctx &ctx, int64_t n, const double *xyz, const int64_t *owner, int64_t ne,
                                   const double *exyz, const double *eh, const int32_t *ekind, const double *val,
                                   int ncomp, double *out, hipStream_t s);
// this device's address of the fixed scratch (looked up on first use with
// the device current); its size; the bytes an interpolation needs
void *noalloc_scratch_init(int device);
size_t noalloc_scratch_bytes();
size_t interp_scratch_bound(int64_t n, int64_t ne);

inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace sphmap
