// A batch of independent forward mappings captured as one HIP graph, for
// repeated steps over fixed buffers (the timestep loop of the method calls
// the mapping on every step, Sec. 2.3; here many instances at once).
//
// Plan: the pair counts are found once with a host read (the ordinary
// path), each instance's lists are given that count plus headroom as their
// capacity, and one uncaptured pass in capacity mode grows every buffer to
// its final size.  The step is then captured:
//   fork    instances are dealt to four branch streams in turn; each branch
//           stages, Morton-sorts and walks its instances one after another
//           into its own scratch (the pair count stays on the device);
//   join    one persistent Exact launch over all instances, its instance
//           table completed on the device from the device counts;
//   fork    each branch transposes its instances' lists (sort by particle
//           with the device count) and forms coverage and cell masses;
//   join.
// The graph has no host reads, allocations or memory sets; independent
// branches run side by side.  A list whose count passes its capacity is
// emptied and flagged, so a replay never writes out of bounds; the caller
// reads the flag with the per-instance counts after the step and makes a
// new plan if it is set.  Every kernel is the ordinary path's, so results
// equal the uncaptured call's bit for bit.
#include <algorithm>
#include <memory>

#include "common.hpp"

namespace sphmap {

namespace {

// the plan's streams keep the default priority
hipStream_t new_stream() {
  hipStream_t st = nullptr;
  SPH_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  return st;
}

hipEvent_t new_event() {
  hipEvent_t ev = nullptr;
  SPH_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  return ev;
}

// every branch stream waits for `from`
void fork(BatchPlan &B, hipStream_t from) {
  SPH_HIP(hipEventRecord(B.ev_fork, from));
  for (hipStream_t b : B.branch) SPH_HIP(hipStreamWaitEvent(b, B.ev_fork, 0));
}

// `to` waits for every branch stream
void join(BatchPlan &B, hipStream_t to) {
  for (size_t b = 0; b < B.branch.size(); ++b) {
    SPH_HIP(hipEventRecord(B.ev_join[b], B.branch[b]));
    SPH_HIP(hipStreamWaitEvent(to, B.ev_join[b], 0));
  }
}

struct Redirect {  // scratch requests of the enclosed work go to one branch's arena
  Ctx &c;
  Redirect(Ctx &cc, Arena *a) : c(cc) { c.arena.redirect = a; }
  ~Redirect() { c.arena.redirect = nullptr; }
};

// One step of the plan on stream s (ordinary launches; captured or not).
void enqueue_step(Ctx &ctx, BatchPlan &B, hipStream_t s) {
  const int nb = (int)B.branch.size();
  fork(B, s);
  for (int k = 0; k < B.n_inst; ++k) {
    const int b = k % nb;
    Redirect r(ctx, &B.scratch[b]);
    B.pd[k].x32 = ctx.arena.get<float4>("x32", B.n_max[b]);
    particles_prepare(ctx, B.pd[k], B.branch[b]);
    find_pairs(ctx, *B.t[k], B.pd[k], *B.P[k], B.branch[b]);
  }
  join(B, s);
  std::vector<ExactJob> jobs(B.n_inst);
  for (int k = 0; k < B.n_inst; ++k) jobs[k] = ExactJob{B.t[k], &B.pd[k], B.P[k].get()};
  exact_integral_batch(ctx, jobs, SPHMAP_PREC_MIXED, s, &B.tab);
  fork(B, s);
  for (int k = 0; k < B.n_inst; ++k) {
    const int b = k % nb;
    Redirect r(ctx, &B.scratch[b]);
    particle_major(ctx, *B.P[k], B.branch[b]);
    cell_reduce(ctx, *B.t[k], B.pd[k], *B.P[k], B.normalize, B.mass[k], B.dens[k], B.branch[b]);
    if (B.cov[k])
      SPH_HIP(hipMemcpyAsync(B.cov[k], B.P[k]->coverage, B.pd[k].n * sizeof(double), hipMemcpyDeviceToDevice,
                             B.branch[b]));
  }
  join(B, s);
}

}  // namespace

BatchPlan::~BatchPlan() {
  exact_table_free(tab);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  for (hipStream_t b : branch) (void)hipStreamDestroy(b);
  if (origin) (void)hipStreamDestroy(origin);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  for (hipEvent_t e : ev_join) (void)hipEventDestroy(e);
}

void batch_plan_build(Ctx &ctx, BatchPlan &B, double headroom, hipStream_t s) {
  SPH_REQUIRE(headroom >= 0.0 && headroom <= 16.0, SPHMAP_EINVAL, "headroom must be in [0, 16]");
  const int nb = std::min(kBatchBranches, B.n_inst);
  for (int b = 0; b < nb; ++b) {
    B.branch.push_back(new_stream());
    B.ev_join.push_back(new_event());
  }
  B.ev_fork = new_event();
  B.scratch.resize(nb);
  B.n_max.assign(nb, 1);
  for (int k = 0; k < B.n_inst; ++k) B.n_max[k % nb] = std::max(B.n_max[k % nb], B.pd[k].n);
  // per-instance device counts, overflow bits, the plan's flag, the table
  B.d_np = B.mem.get<int64_t>("np", B.n_inst);
  B.d_over = B.mem.get<int32_t>("over", B.n_inst);
  B.d_flag = B.mem.get<int32_t>("flag", 1);
  B.tab.insts = B.mem.get("insts", B.n_inst * exact_inst_bytes() + 64);
  B.tab.chunk0 = B.mem.get<int64_t>("chunk0", B.n_inst + 1);
  B.tab.np = (const int64_t **)B.mem.get<int64_t *>("np_ptrs", B.n_inst);
  SPH_HIP(hipMemsetAsync(B.d_flag, 0, sizeof(int32_t), s));
  // planning pass: the counts with a host read (the ordinary pair search)
  for (int k = 0; k < B.n_inst; ++k) {
    PairsDev &P = *B.P[k];
    P.device = ctx.device;
    P.cap = 0;
    B.pd[k].x32 = ctx.arena.get<float4>("x32", B.pd[k].n);
    particles_prepare(ctx, B.pd[k], s);
    find_pairs(ctx, *B.t[k], B.pd[k], P, s);
    const int64_t cap = P.n_pairs + std::max<int64_t>((int64_t)((double)P.n_pairs * headroom), 4096);
    SPH_REQUIRE(cap < ((int64_t)1 << 31), SPHMAP_EINVAL, "pair capacity of an instance passes 2^31");
    P.cap = cap;
    P.d_np = B.d_np + k;
    P.d_over = B.d_over + k;
    P.d_flag = B.d_flag;
  }
  // warm pass in capacity mode: every buffer reaches its final size
  const bool timing = ctx.timing, counting = ctx.counting;
  ctx.timing = ctx.counting = false;
  struct Restore {
    Ctx &c;
    bool t, n;
    ~Restore() {
      c.timing = t;
      c.counting = n;
    }
  } restore{ctx, timing, counting};
  {
    // the pointer table of the Exact launch needs the lists' final buffers:
    // size them first (the warm pass then finds them in place)
    for (int k = 0; k < B.n_inst; ++k) {
      PairsDev &P = *B.P[k];
      P.pair_p = P.mem.get<int32_t>("pair_p", P.cap);
      P.pair_c = P.mem.get<int32_t>("pair_c", P.cap);
      P.w = P.mem.get<double>("w", P.cap);
    }
    std::vector<ExactJob> jobs(B.n_inst);
    for (int k = 0; k < B.n_inst; ++k) jobs[k] = ExactJob{B.t[k], &B.pd[k], B.P[k].get()};
    B.tab.flag = B.d_flag;
    exact_table_upload(ctx, jobs, B.tab, B.mem, headroom, s);
  }
  enqueue_step(ctx, B, s);
  SPH_HIP(hipStreamSynchronize(s));
  // capture on the plan's own stream (the caller's may be the legacy
  // default stream, which cannot be captured); the graph is later launched
  // on the caller's stream
  B.origin = new_stream();
  SPH_HIP(hipStreamBeginCapture(B.origin, hipStreamCaptureModeThreadLocal));
  try {
    enqueue_step(ctx, B, B.origin);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(B.origin, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  SPH_HIP(hipStreamEndCapture(B.origin, &B.graph));
  SPH_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
}

void batch_plan_run(Ctx &ctx, BatchPlan &B, hipStream_t s) {
  (void)ctx;
  SPH_HIP(hipGraphLaunch(B.exec, s));
}

void batch_plan_check(Ctx &ctx, BatchPlan &B, hipStream_t s, int64_t *h_pairs, int32_t *overflow) {
  (void)ctx;
  std::vector<int64_t> np(B.n_inst);
  int32_t flag = 0;
  SPH_HIP(hipMemcpyAsync(np.data(), B.d_np, B.n_inst * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipMemcpyAsync(&flag, B.d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  SPH_HIP(hipMemsetAsync(B.d_flag, 0, sizeof(int32_t), s));  // outside the graph
  if (h_pairs)
    for (int k = 0; k < B.n_inst; ++k) h_pairs[k] = np[k];
  *overflow = flag;
}

}  // namespace sphmap
