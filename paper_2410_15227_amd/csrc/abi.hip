// C-ABI entry points of libsphmap (declared in include/sphmap.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "common.hpp"

struct sphmap_ctx {
  sphmap::Ctx c;
};
struct sphmap_tess {
  sphmap::TessDev t;
};
struct sphmap_pairs {
  sphmap::PairsDev p;
};
struct sphmap_batch {
  sphmap::BatchPlan b;
};

namespace {

template <typename F>
int guarded(sphmap_ctx *ctx, F &&fn) {
  try {
    if (ctx) {
      ctx->c.last_error.clear();
      SPH_HIP(hipSetDevice(ctx->c.device));
    }
    fn();
    return SPHMAP_OK;
  } catch (const sphmap::Error &e) {
    if (ctx) ctx->c.last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    if (ctx) ctx->c.last_error = "host allocation failed";
    return SPHMAP_ENOMEM;
  } catch (...) {
    if (ctx) ctx->c.last_error = "unexpected exception";
    return SPHMAP_EHIP;
  }
}

inline hipStream_t as_stream(void *s) { return (hipStream_t)s; }

// A retained pair list allocates from the context's block pool and gives
// its blocks back to it when freed, so repeated steps allocate nothing.
sphmap_pairs *new_pairs(sphmap::Ctx &C) {
  sphmap_pairs *q = new sphmap_pairs;
  q->p.mem.pool = &C.pool;
  return q;
}

// The context's pair list for calls that keep none (counted in its workspace).
sphmap::PairsDev *scratch_pairs(sphmap::Ctx &C) {
  if (!C.scratch_pairs) {
    C.scratch_pairs = new sphmap::PairsDev;
    C.scratch_pairs->mem.budget = &C.ws;
  }
  return C.scratch_pairs;
}

// Upper bounds of the device bytes of one forward + inverse mapping (see
// sphmap_estimate_footprint).
sphmap_footprint footprint(sphmap::Ctx &C, int64_t n_particles, int64_t n_pairs, int64_t n_cells, int64_t n_faces,
                           int64_t n_face_vertices, int64_t n_vertices) {
  const int64_t N = n_particles, Cn = n_cells, P = n_pairs > 0 ? n_pairs : 200 * n_particles;
  // arena buffers grow to 9/8 of the request; the device allocator hands
  // out whole 2 MiB granules, once per named buffer
  auto grown = [](double b, int n_buffers) { return (size_t)(b * 1.125 + 2097152.0 * n_buffers); };
  // per particle: staged float4, Morton key + index, sorted copy, radix
  // temporaries, search boxes; per pair: the transpose's sorted keys, one
  // set of (key, cell, weight) temporaries (two above 2^20 particles, when
  // the sort takes three passes) and its digit histograms; per cell: pair
  // counts, the bounded candidate buffer of the pair search (512 entries),
  // the overflow list
  const double per_pair = 4.0 + (N > ((int64_t)1 << 20) ? 32.0 : 16.0) + 8.0;
  const double ws = 16.0 * N + 12.0 * N + 16.0 * N + 12.0 * N + 3.0 * N + per_pair * P +
                    (8.0 + 2048.0 + 4.0) * Cn + (double)sphmap::exact_workspace_bytes(C, P);
  // retained list: cell offsets, pair indices, weights, particle-major
  // copy, particle offsets and coverage
  const double pr = 8.0 * Cn + (4.0 + 4.0 + 8.0 + 4.0 + 8.0) * P + 16.0 * N;
  // grid: generators, offsets, orders and volumes per cell; planes, spheres
  // and cell per face; oriented vertices and edge frames per face vertex
  const double tb = 96.0 * Cn + 96.0 * n_faces + 96.0 * n_face_vertices + 24.0 * n_vertices;
  sphmap_footprint f;
  f.workspace = grown(ws, 56);
  f.pairs = grown(pr, 8);
  f.tessellation = grown(tb, 24);
  return f;
}

// Workspace a mapping call of N particles on t needs: the scratch, plus
// the pair list when the call keeps none.  P: the pair count if known.
size_t workspace_need(sphmap::Ctx &C, int64_t N, int64_t P, const sphmap::TessDev &t, bool scratch_list) {
  const sphmap_footprint f = footprint(C, N, P, t.n_cells, t.n_faces, t.n_fv, t.n_vertices);
  return f.workspace + (scratch_list ? f.pairs : 0);
}

// An ENOMEM from a capped workspace, restated with what the call needs.
[[noreturn]] void workspace_refused(sphmap::Ctx &C, const sphmap::Error &e, size_t need) {
  C.ws.required = std::max(C.ws.required, need);
  throw sphmap::Error{SPHMAP_ENOMEM, e.msg + "; the call needs a workspace of up to " +
                                         std::to_string(C.ws.required) + " bytes (sphmap_workspace_info)"};
}

}  // namespace

extern "C" {

int sphmap_version(void) { return 100; }

int sphmap_create(int32_t device, size_t workspace_bytes, sphmap_ctx **out) {
  if (!out) return SPHMAP_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SPHMAP_EINVAL;
  std::unique_ptr<sphmap_ctx> ctx(new sphmap_ctx);
  ctx->c.device = device;
  ctx->c.ws.limit = workspace_bytes;
  ctx->c.arena.budget = &ctx->c.ws;
  int rc = guarded(ctx.get(), [&] {
    size_t free_b = 0, total_b = 0;
    SPH_HIP(hipMemGetInfo(&free_b, &total_b));
    ctx->c.pool.cap = total_b / 8;
    // this device's address of the fixed scratch of the no-allocation entry point
    (void)sphmap::noalloc_scratch_init(device);
    ctx->c.d_counters = ctx->c.arena.get<int64_t>("counters", 8);
    ctx->c.d_status = ctx->c.arena.get<int>("status", 4);
    SPH_HIP(hipMemset(ctx->c.d_counters, 0, 8 * sizeof(int64_t)));
    SPH_HIP(hipMemset(ctx->c.d_status, 0, 4 * sizeof(int)));
  });
  if (rc != SPHMAP_OK) return rc;
  *out = ctx.release();
  return SPHMAP_OK;
}

int sphmap_destroy(sphmap_ctx *ctx) {
  if (!ctx) return SPHMAP_EINVAL;
  (void)hipSetDevice(ctx->c.device);
  (void)hipDeviceSynchronize();
  for (auto &kv : ctx->c.timers)
    for (auto &r : kv.second) {
      (void)hipEventDestroy(r.start);
      (void)hipEventDestroy(r.stop);
    }
  delete ctx->c.scratch_pairs;
  ctx->c.scratch_pairs = nullptr;
  for (auto *P : ctx->c.scratch_batch) delete P;
  ctx->c.scratch_batch.clear();
  ctx->c.pool.release();
  if (ctx->c.pinned) (void)hipHostFree(ctx->c.pinned);
  ctx->c.pinned = nullptr;
  if (ctx->c.side) {
    (void)hipEventDestroy(ctx->c.ev_fork);
    (void)hipEventDestroy(ctx->c.ev_join);
    (void)hipStreamDestroy(ctx->c.side);
  }
  delete ctx;
  return SPHMAP_OK;
}

const char *sphmap_last_error(const sphmap_ctx *ctx) { return ctx ? ctx->c.last_error.c_str() : "null context"; }

int sphmap_tess_upload(sphmap_ctx *ctx, int64_t n_cells, int64_t n_faces, int64_t n_vertices,
                       const double *h_generators, const double *h_vertices, const int64_t *h_cell_face_off,
                       const int64_t *h_face_vtx_off, const int32_t *h_face_vtx, void *stream, sphmap_tess **out) {
  if (!ctx || !out) return SPHMAP_EINVAL;
  *out = nullptr;
  std::unique_ptr<sphmap_tess> T(new sphmap_tess);
  int rc = guarded(ctx, [&] {
    SPH_REQUIRE(n_cells >= 1 && n_cells < ((int64_t)1 << 31), SPHMAP_EINVAL, "n_cells out of range");
    SPH_REQUIRE(n_faces >= 0 && n_faces < ((int64_t)1 << 31), SPHMAP_EINVAL, "n_faces out of range");
    SPH_REQUIRE(n_vertices >= 0 && n_vertices < ((int64_t)1 << 31), SPHMAP_EINVAL, "n_vertices out of range");
    SPH_REQUIRE(h_generators && h_vertices && h_cell_face_off && h_face_vtx_off && h_face_vtx, SPHMAP_EINVAL,
                "null tessellation array");
    SPH_REQUIRE(h_cell_face_off[0] == 0 && h_cell_face_off[n_cells] == n_faces, SPHMAP_EINVAL,
                "cell_face_off must start at 0 and end at n_faces");
    for (int64_t c = 0; c < n_cells; ++c)
      SPH_REQUIRE(h_cell_face_off[c + 1] >= h_cell_face_off[c], SPHMAP_EINVAL, "cell_face_off not non-decreasing");
    SPH_REQUIRE(h_face_vtx_off[0] == 0, SPHMAP_EINVAL, "face_vtx_off must start at 0");
    for (int64_t f = 0; f < n_faces; ++f) {
      SPH_REQUIRE(h_face_vtx_off[f + 1] >= h_face_vtx_off[f], SPHMAP_EINVAL, "face_vtx_off not non-decreasing");
      SPH_REQUIRE(h_face_vtx_off[f + 1] - h_face_vtx_off[f] <= 128, SPHMAP_EINVAL, "a face has more than 128 vertices");
    }
    const int64_t FV = h_face_vtx_off[n_faces];
    for (int64_t k = 0; k < FV; ++k)
      SPH_REQUIRE(h_face_vtx[k] >= 0 && h_face_vtx[k] < n_vertices, SPHMAP_EINVAL, "face vertex index out of range");
    double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int64_t v = 0; v < n_vertices; ++v)
      for (int j = 0; j < 3; ++j) {
        double x = h_vertices[3 * v + j];
        SPH_REQUIRE(std::isfinite(x), SPHMAP_EINVAL, "non-finite vertex");
        lo[j] = std::min(lo[j], x);
        hi[j] = std::max(hi[j], x);
      }
    for (int64_t c = 0; c < 3 * n_cells; ++c)
      SPH_REQUIRE(std::isfinite(h_generators[c]), SPHMAP_EINVAL, "non-finite generator");
    sphmap::TessDev &t = T->t;
    t.n_cells = n_cells;
    t.n_faces = n_faces;
    t.n_vertices = n_vertices;
    t.n_fv = FV;
    t.device = ctx->c.device;
    double size = 0;
    for (int j = 0; j < 3; ++j) {
      t.box_lo[j] = n_vertices ? lo[j] : 0.0;
      size = std::max(size, n_vertices ? hi[j] - lo[j] : 1.0);
    }
    t.box_size = size > 0 ? size * (1.0 + 1e-12) : 1.0;
    hipStream_t s = as_stream(stream);
    t.gen = t.mem.get<double>("gen", 3 * n_cells);
    t.vert = t.mem.get<double>("vert", 3 * std::max<int64_t>(n_vertices, 1));
    t.cell_face_off = t.mem.get<int64_t>("cfo", n_cells + 1);
    t.face_vtx_off = t.mem.get<int64_t>("fvo", n_faces + 1);
    t.face_vtx = t.mem.get<int32_t>("fv", std::max<int64_t>(FV, 1));
    SPH_HIP(hipMemcpyAsync(t.gen, h_generators, 3 * n_cells * sizeof(double), hipMemcpyHostToDevice, s));
    if (n_vertices)
      SPH_HIP(hipMemcpyAsync(t.vert, h_vertices, 3 * n_vertices * sizeof(double), hipMemcpyHostToDevice, s));
    SPH_HIP(hipMemcpyAsync(t.cell_face_off, h_cell_face_off, (n_cells + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                           s));
    SPH_HIP(hipMemcpyAsync(t.face_vtx_off, h_face_vtx_off, (n_faces + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (FV) SPH_HIP(hipMemcpyAsync(t.face_vtx, h_face_vtx, FV * sizeof(int32_t), hipMemcpyHostToDevice, s));
    sphmap::tess_prepare(ctx->c, t, s);
  });
  if (rc != SPHMAP_OK) return rc;
  *out = T.release();
  return SPHMAP_OK;
}

int sphmap_tess_set_face_neighbours(sphmap_ctx *ctx, sphmap_tess *tess, const int32_t *h_face_nbr, void *stream,
                                    int64_t *n_shared) {
  if (!ctx || !tess) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    sphmap::TessDev &t = tess->t;
    hipStream_t s = as_stream(stream);
    int64_t n = 0;
    if (!h_face_nbr) {
      t.face_nbr = nullptr;
      n = sphmap::tess_set_twins(ctx->c, t, nullptr, s);
    } else {
      for (int64_t f = 0; f < t.n_faces; ++f)
        SPH_REQUIRE(h_face_nbr[f] < t.n_cells, SPHMAP_EINVAL, "face neighbour out of range");
      t.face_nbr = t.mem.get<int32_t>("fnbr", std::max<int64_t>(t.n_faces, 1));
      if (t.n_faces)
        SPH_HIP(hipMemcpyAsync(t.face_nbr, h_face_nbr, t.n_faces * sizeof(int32_t), hipMemcpyHostToDevice, s));
      n = sphmap::tess_set_twins(ctx->c, t, t.face_nbr, s);
    }
    if (n_shared) *n_shared = n;
  });
}

int sphmap_tess_build_voronoi(sphmap_ctx *ctx, int64_t n, const double *d_generators, const double *h_box_lo,
                              const double *h_box_hi, int32_t n_lloyd, double *d_generators_out, void *stream,
                              sphmap_tess **out) {
  if (!ctx || !out) return SPHMAP_EINVAL;
  *out = nullptr;
  std::unique_ptr<sphmap_tess> T(new sphmap_tess);
  int rc = guarded(ctx, [&] {
    SPH_REQUIRE(n >= 1 && n < ((int64_t)1 << 31), SPHMAP_EINVAL, "n out of range [1, 2^31)");
    SPH_REQUIRE(d_generators && h_box_lo && h_box_hi, SPHMAP_EINVAL, "null array");
    SPH_REQUIRE(n_lloyd >= 0, SPHMAP_EINVAL, "n_lloyd must be >= 0");
    for (int a = 0; a < 3; ++a)
      SPH_REQUIRE(std::isfinite(h_box_lo[a]) && std::isfinite(h_box_hi[a]) && h_box_hi[a] > h_box_lo[a],
                  SPHMAP_EINVAL, "empty or non-finite box");
    sphmap::voronoi_build(ctx->c, T->t, n, d_generators, h_box_lo, h_box_hi, n_lloyd, d_generators_out,
                          as_stream(stream));
  });
  if (rc != SPHMAP_OK) return rc;
  *out = T.release();
  return SPHMAP_OK;
}

int sphmap_tess_counts(const sphmap_tess *tess, int64_t *n_cells, int64_t *n_faces, int64_t *n_face_vertices,
                       int64_t *n_vertices) {
  if (!tess) return SPHMAP_EINVAL;
  if (n_cells) *n_cells = tess->t.n_cells;
  if (n_faces) *n_faces = tess->t.n_faces;
  if (n_face_vertices) *n_face_vertices = tess->t.n_fv;
  if (n_vertices) *n_vertices = tess->t.n_vertices;
  return SPHMAP_OK;
}

int sphmap_tess_export(sphmap_ctx *ctx, const sphmap_tess *tess, double *d_generators, double *d_vertices,
                       int64_t *d_cell_face_off, int64_t *d_face_vtx_off, int32_t *d_face_vtx, int32_t *d_face_nbr,
                       void *stream) {
  if (!ctx || !tess) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    const auto &t = tess->t;
    SPH_REQUIRE(!d_face_nbr || t.face_nbr, SPHMAP_EINVAL, "the grid records no face neighbours");
    hipStream_t s = as_stream(stream);
    auto cp = [&](void *dst, const void *src, size_t bytes) {
      if (dst && bytes) SPH_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
    };
    cp(d_generators, t.gen, 3 * t.n_cells * sizeof(double));
    cp(d_vertices, t.vert, 3 * t.n_vertices * sizeof(double));
    cp(d_cell_face_off, t.cell_face_off, (t.n_cells + 1) * sizeof(int64_t));
    cp(d_face_vtx_off, t.face_vtx_off, (t.n_faces + 1) * sizeof(int64_t));
    cp(d_face_vtx, t.face_vtx, t.n_fv * sizeof(int32_t));
    cp(d_face_nbr, t.face_nbr, t.n_faces * sizeof(int32_t));
  });
}

int sphmap_tess_free(sphmap_ctx *ctx, sphmap_tess *tess) {
  if (!ctx || !tess) return SPHMAP_EINVAL;
  (void)hipSetDevice(ctx->c.device);
  (void)hipDeviceSynchronize();
  delete tess;
  return SPHMAP_OK;
}

int sphmap_tess_cell_info(sphmap_ctx *ctx, const sphmap_tess *tess, double *d_volume, float *d_radius,
                          void *stream) {
  if (!ctx || !tess) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    hipStream_t s = as_stream(stream);
    const auto &t = tess->t;
    if (d_volume)
      SPH_HIP(hipMemcpyAsync(d_volume, t.volume, t.n_cells * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (d_radius)
      SPH_HIP(hipMemcpyAsync(d_radius, t.radius, t.n_cells * sizeof(float), hipMemcpyDeviceToDevice, s));
  });
}

int map_particles_to_cells(sphmap_ctx *ctx, const sphmap_tess *tess, int64_t n, const double *d_xyz,
                           const double *d_h, const double *d_m, int32_t precision, int32_t normalize,
                           double *d_cell_mass, double *d_cell_density, double *d_coverage, void *stream,
                           sphmap_pairs **pairs_out) {
  if (!ctx) return SPHMAP_EINVAL;
  if (pairs_out) *pairs_out = nullptr;
  std::unique_ptr<sphmap_pairs> owned;
  int rc = guarded(ctx, [&] {
    SPH_REQUIRE(tess, SPHMAP_EINVAL, "null tessellation");
    SPH_REQUIRE(n >= 1 && n < ((int64_t)1 << 31), SPHMAP_EINVAL, "n out of range [1, 2^31)");
    SPH_REQUIRE(d_xyz && d_h && d_m && d_cell_mass, SPHMAP_EINVAL, "null required pointer");
    SPH_REQUIRE(precision == SPHMAP_PREC_FP64 || precision == SPHMAP_PREC_MIXED, SPHMAP_EINVAL, "bad precision");
    SPH_REQUIRE(normalize == 0 || normalize == 1, SPHMAP_EINVAL, "normalize must be 0 or 1");
    SPH_REQUIRE(tess->t.device == ctx->c.device, SPHMAP_EINVAL, "tessellation belongs to another device");
    hipStream_t s = as_stream(stream);
    sphmap::Ctx &C = ctx->c;
    sphmap::PairsDev *P;
    if (pairs_out) {
      owned.reset(new_pairs(C));
      P = &owned->p;
    } else {
      P = scratch_pairs(C);
    }
    P->device = C.device;
    P->n_pairs = 0;
    try {
      sphmap::PartDev pd{n, d_xyz, d_h, d_m, C.arena.get<float4>("x32", n)};
      sphmap::particles_prepare(C, pd, s);
      sphmap::find_pairs(C, tess->t, pd, *P, s);
      sphmap::exact_integral(C, tess->t, pd, *P, precision, s);
      if (normalize == 0) {
        // the cell sums need only the weights: they run on the side stream
        // while the particle-major copy runs on the caller's
        hipStream_t s2 = C.side_stream();
        SPH_HIP(hipEventRecord(C.ev_fork, s));
        SPH_HIP(hipStreamWaitEvent(s2, C.ev_fork, 0));
        sphmap::cell_reduce(C, tess->t, pd, *P, false, d_cell_mass, d_cell_density, s2);
        SPH_HIP(hipEventRecord(C.ev_join, s2));
        try {
          sphmap::particle_major(C, *P, s);
        } catch (...) {  // joined on the error path too
          (void)hipStreamWaitEvent(s, C.ev_join, 0);
          throw;
        }
        SPH_HIP(hipStreamWaitEvent(s, C.ev_join, 0));
      } else {  // normalised sums divide by the coverage the copy computes
        sphmap::particle_major(C, *P, s);
        sphmap::cell_reduce(C, tess->t, pd, *P, true, d_cell_mass, d_cell_density, s);
      }
    } catch (const sphmap::Error &e) {
      if (e.code != SPHMAP_ENOMEM || !C.ws.limit) throw;
      workspace_refused(C, e, workspace_need(C, n, P->n_pairs, tess->t, !pairs_out));
    }
    if (d_coverage)
      SPH_HIP(hipMemcpyAsync(d_coverage, P->coverage, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (C.counting) {
      SPH_HIP(hipMemcpyAsync(C.counters, C.d_counters, 8 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
      SPH_HIP(hipStreamSynchronize(s));
      C.counters[0] = P->n_pairs;
    }
  });
  if (rc == SPHMAP_OK && pairs_out) *pairs_out = owned.release();
  return rc;
}

int map_particles_to_cells_batch(sphmap_ctx *ctx, int32_t n_inst, const sphmap_tess *const *tess, const int64_t *n,
                                 const double *const *d_xyz, const double *const *d_h, const double *const *d_m,
                                 int32_t precision, int32_t normalize, double *const *d_cell_mass,
                                 double *const *d_cell_density, double *const *d_coverage, void *stream,
                                 sphmap_pairs **pairs_out) {
  if (!ctx) return SPHMAP_EINVAL;
  std::vector<std::unique_ptr<sphmap_pairs>> owned;
  int rc = guarded(ctx, [&] {
    SPH_REQUIRE(n_inst >= 1, SPHMAP_EINVAL, "n_inst < 1");
    SPH_REQUIRE(tess && n && d_xyz && d_h && d_m && d_cell_mass, SPHMAP_EINVAL, "null required array");
    SPH_REQUIRE(precision == SPHMAP_PREC_FP64 || precision == SPHMAP_PREC_MIXED, SPHMAP_EINVAL, "bad precision");
    SPH_REQUIRE(normalize == 0 || normalize == 1, SPHMAP_EINVAL, "normalize must be 0 or 1");
    int64_t n_max = 0;
    for (int k = 0; k < n_inst; ++k) {
      SPH_REQUIRE(tess[k], SPHMAP_EINVAL, "null tessellation of instance " + std::to_string(k));
      SPH_REQUIRE(n[k] >= 1 && n[k] < ((int64_t)1 << 31), SPHMAP_EINVAL,
                  "n out of range [1, 2^31) for instance " + std::to_string(k));
      SPH_REQUIRE(d_xyz[k] && d_h[k] && d_m[k] && d_cell_mass[k], SPHMAP_EINVAL,
                  "null required pointer of instance " + std::to_string(k));
      SPH_REQUIRE(tess[k]->t.device == ctx->c.device, SPHMAP_EINVAL, "tessellation belongs to another device");
      n_max = std::max(n_max, n[k]);
    }
    hipStream_t s = as_stream(stream);
    sphmap::Ctx &C = ctx->c;
    std::vector<sphmap::PairsDev *> P(n_inst);
    if (pairs_out) {
      for (int k = 0; k < n_inst; ++k) {
        owned.emplace_back(new_pairs(C));
        P[k] = &owned.back()->p;
      }
    } else {
      while ((int)C.scratch_batch.size() < n_inst) {
        C.scratch_batch.push_back(new sphmap::PairsDev);
        C.scratch_batch.back()->mem.budget = &C.ws;
      }
      for (int k = 0; k < n_inst; ++k) P[k] = C.scratch_batch[k];
    }
    float4 *x32 = C.arena.get<float4>("x32", n_max);
    std::vector<sphmap::PartDev> pd(n_inst);
    std::vector<sphmap::ExactJob> jobs(n_inst);
    int64_t total = 0;
    for (int k = 0; k < n_inst; ++k) {
      P[k]->device = C.device;
      pd[k] = sphmap::PartDev{n[k], d_xyz[k], d_h[k], d_m[k], x32};
      sphmap::particles_prepare(C, pd[k], s);
      sphmap::find_pairs(C, tess[k]->t, pd[k], *P[k], s);
      jobs[k] = sphmap::ExactJob{&tess[k]->t, &pd[k], P[k]};
      total += P[k]->n_pairs;
    }
    sphmap::exact_integral_batch(C, jobs, precision, s);
    for (int k = 0; k < n_inst; ++k) {
      sphmap::particle_major(C, *P[k], s);
      sphmap::cell_reduce(C, tess[k]->t, pd[k], *P[k], normalize != 0, d_cell_mass[k],
                          d_cell_density ? d_cell_density[k] : nullptr, s);
      if (d_coverage && d_coverage[k])
        SPH_HIP(hipMemcpyAsync(d_coverage[k], P[k]->coverage, n[k] * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    if (C.counting) {
      SPH_HIP(hipMemcpyAsync(C.counters, C.d_counters, 8 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
      SPH_HIP(hipStreamSynchronize(s));
      C.counters[0] = total;
    }
  });
  if (rc == SPHMAP_OK && pairs_out)
    for (int k = 0; k < n_inst; ++k) pairs_out[k] = owned[k].release();
  return rc;
}

int sphmap_batch_create(sphmap_ctx *ctx, int32_t n_inst, const sphmap_tess *const *tess, const int64_t *n,
                        const double *const *d_xyz, const double *const *d_h, const double *const *d_m,
                        int32_t normalize, double *const *d_cell_mass, double *const *d_cell_density,
                        double *const *d_coverage, double headroom, void *stream, sphmap_batch **out) {
  if (!ctx || !out) return SPHMAP_EINVAL;
  *out = nullptr;
  std::unique_ptr<sphmap_batch> B(new sphmap_batch);
  int rc = guarded(ctx, [&] {
    SPH_REQUIRE(n_inst >= 1, SPHMAP_EINVAL, "n_inst < 1");
    SPH_REQUIRE(tess && n && d_xyz && d_h && d_m && d_cell_mass, SPHMAP_EINVAL, "null required array");
    SPH_REQUIRE(normalize == 0 || normalize == 1, SPHMAP_EINVAL, "normalize must be 0 or 1");
    sphmap::BatchPlan &P = B->b;
    P.n_inst = n_inst;
    P.normalize = normalize != 0;
    for (int k = 0; k < n_inst; ++k) {
      SPH_REQUIRE(tess[k], SPHMAP_EINVAL, "null tessellation of instance " + std::to_string(k));
      SPH_REQUIRE(n[k] >= 1 && n[k] < ((int64_t)1 << 31), SPHMAP_EINVAL,
                  "n out of range [1, 2^31) for instance " + std::to_string(k));
      SPH_REQUIRE(d_xyz[k] && d_h[k] && d_m[k] && d_cell_mass[k], SPHMAP_EINVAL,
                  "null required pointer of instance " + std::to_string(k));
      SPH_REQUIRE(tess[k]->t.device == ctx->c.device, SPHMAP_EINVAL, "tessellation belongs to another device");
      P.t.push_back(&tess[k]->t);
      P.pd.push_back(sphmap::PartDev{n[k], d_xyz[k], d_h[k], d_m[k], nullptr});
      P.P.emplace_back(new sphmap::PairsDev);
      P.mass.push_back(d_cell_mass[k]);
      P.dens.push_back(d_cell_density ? d_cell_density[k] : nullptr);
      P.cov.push_back(d_coverage ? d_coverage[k] : nullptr);
    }
    sphmap::batch_plan_build(ctx->c, P, headroom, as_stream(stream));
  });
  if (rc != SPHMAP_OK) {
    (void)hipDeviceSynchronize();
    return rc;
  }
  *out = B.release();
  return SPHMAP_OK;
}

int sphmap_batch_run(sphmap_ctx *ctx, sphmap_batch *batch, void *stream) {
  if (!ctx || !batch) return SPHMAP_EINVAL;
  return guarded(ctx, [&] { sphmap::batch_plan_run(ctx->c, batch->b, as_stream(stream)); });
}

int sphmap_batch_check(sphmap_ctx *ctx, sphmap_batch *batch, void *stream, int64_t *h_pairs, int32_t *overflow) {
  if (!ctx || !batch || !overflow) return SPHMAP_EINVAL;
  return guarded(ctx, [&] { sphmap::batch_plan_check(ctx->c, batch->b, as_stream(stream), h_pairs, overflow); });
}

int sphmap_batch_free(sphmap_ctx *ctx, sphmap_batch *batch) {
  if (!ctx || !batch) return SPHMAP_EINVAL;
  (void)hipSetDevice(ctx->c.device);
  (void)hipDeviceSynchronize();
  delete batch;
  return SPHMAP_OK;
}

int sphmap_pairs_info(const sphmap_pairs *pairs, int64_t *n_pairs, int64_t *n_cells, int64_t *n_particles) {
  if (!pairs) return SPHMAP_EINVAL;
  if (n_pairs) *n_pairs = pairs->p.n_pairs;
  if (n_cells) *n_cells = pairs->p.n_cells;
  if (n_particles) *n_particles = pairs->p.n_particles;
  return SPHMAP_OK;
}

int sphmap_pairs_export(sphmap_ctx *ctx, const sphmap_pairs *pairs, int64_t *d_cell_off, int32_t *d_particle,
                        double *d_w, void *stream) {
  if (!ctx || !pairs) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    hipStream_t s = as_stream(stream);
    const auto &P = pairs->p;
    if (d_cell_off)
      SPH_HIP(hipMemcpyAsync(d_cell_off, P.cell_off, (P.n_cells + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    if (d_particle && P.n_pairs)
      SPH_HIP(hipMemcpyAsync(d_particle, P.pair_p, P.n_pairs * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (d_w && P.n_pairs)
      SPH_HIP(hipMemcpyAsync(d_w, P.w, P.n_pairs * sizeof(double), hipMemcpyDeviceToDevice, s));
  });
}

int sphmap_pairs_free(sphmap_ctx *ctx, sphmap_pairs *pairs) {
  if (!ctx || !pairs) return SPHMAP_EINVAL;
  (void)hipSetDevice(ctx->c.device);
  (void)hipDeviceSynchronize();
  delete pairs;  // its blocks go to the context's pool
  return SPHMAP_OK;
}

int sphmap_set_pool_limit(sphmap_ctx *ctx, uint64_t bytes) {
  if (!ctx) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    sphmap::BlockPool &pool = ctx->c.pool;
    pool.cap = (size_t)bytes;
    if (pool.held > pool.cap) {
      SPH_HIP(hipDeviceSynchronize());
      pool.trim();
    }
  });
}

int map_cells_to_particles(sphmap_ctx *ctx, const sphmap_tess *tess, int64_t n, const double *d_xyz,
                           const double *d_h, int32_t precision, const sphmap_pairs *pairs,
                           const double *d_cell_values, int32_t n_components, double *d_particle_values,
                           void *stream) {
  if (!ctx) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    SPH_REQUIRE(d_cell_values && d_particle_values, SPHMAP_EINVAL, "null value array");
    SPH_REQUIRE(n_components >= 1, SPHMAP_EINVAL, "n_components must be >= 1");
    sphmap::Ctx &C = ctx->c;
    hipStream_t s = as_stream(stream);
    if (pairs) {
      SPH_REQUIRE(pairs->p.device == C.device, SPHMAP_EINVAL, "pair list belongs to another device");
      SPH_REQUIRE(n == 0 || n == pairs->p.n_particles, SPHMAP_EINVAL, "n differs from the pair list's particles");
      sphmap::reverse_map(C, pairs->p, d_cell_values, n_components, d_particle_values, s);
      return;
    }
    // no retained list: the weights are recomputed from the particles and
    // the grid (the forward mapping's pair search, Exact integral and
    // particle-major copy, without the cell sums)
    SPH_REQUIRE(tess, SPHMAP_EINVAL, "null tessellation (needed when no pair list is given)");
    SPH_REQUIRE(n >= 1 && n < ((int64_t)1 << 31), SPHMAP_EINVAL, "n out of range [1, 2^31)");
    SPH_REQUIRE(d_xyz && d_h, SPHMAP_EINVAL, "null particle array (needed when no pair list is given)");
    SPH_REQUIRE(precision == SPHMAP_PREC_FP64 || precision == SPHMAP_PREC_MIXED, SPHMAP_EINVAL, "bad precision");
    SPH_REQUIRE(tess->t.device == C.device, SPHMAP_EINVAL, "tessellation belongs to another device");
    sphmap::PairsDev *P = scratch_pairs(C);
    P->device = C.device;
    P->n_pairs = 0;
    try {
      sphmap::PartDev pd{n, d_xyz, d_h, nullptr, C.arena.get<float4>("x32", n)};
      sphmap::particles_prepare(C, pd, s);
      sphmap::find_pairs(C, tess->t, pd, *P, s);
      sphmap::exact_integral(C, tess->t, pd, *P, precision, s);
      sphmap::particle_major(C, *P, s);
      sphmap::reverse_map(C, *P, d_cell_values, n_components, d_particle_values, s);
    } catch (const sphmap::Error &e) {
      if (e.code != SPHMAP_ENOMEM || !C.ws.limit) throw;
      workspace_refused(C, e, workspace_need(C, n, P->n_pairs, tess->t, true));
    }
  });
}

int sphmap_set_workspace_limit(sphmap_ctx *ctx, size_t bytes) {
  if (!ctx) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    sphmap::Ctx &C = ctx->c;
    C.ws.limit = bytes;
    C.ws.required = 0;
    if (bytes && C.ws.held > bytes) {
      // drop the scratch so that later calls grow within the new limit
      SPH_HIP(hipDeviceSynchronize());
      if (C.scratch_pairs) C.scratch_pairs->mem.release();
      for (auto *P : C.scratch_batch) P->mem.release();
      int64_t *ctr = C.d_counters;
      int *st = C.d_status;
      int64_t hc[8];
      int hs[4];
      SPH_HIP(hipMemcpy(hc, ctr, sizeof hc, hipMemcpyDeviceToHost));
      SPH_HIP(hipMemcpy(hs, st, sizeof hs, hipMemcpyDeviceToHost));
      C.arena.release();
      C.d_counters = C.arena.get<int64_t>("counters", 8);
      C.d_status = C.arena.get<int>("status", 4);
      SPH_HIP(hipMemcpy(C.d_counters, hc, sizeof hc, hipMemcpyHostToDevice));
      SPH_HIP(hipMemcpy(C.d_status, hs, sizeof hs, hipMemcpyHostToDevice));
    }
  });
}

int sphmap_workspace_info(sphmap_ctx *ctx, size_t *held, size_t *limit, size_t *required) {
  if (!ctx) return SPHMAP_EINVAL;
  if (held) *held = ctx->c.ws.held;
  if (limit) *limit = ctx->c.ws.limit;
  if (required) *required = ctx->c.ws.required;
  return SPHMAP_OK;
}

int build_pseudo_particles_open(sphmap_ctx *ctx, int64_t n, const double *d_xyz, const double *d_h,
                                const double *d_m, int32_t n_src, const double *h_sources,
                                const sphmap_pseudo_opts *opts, int64_t n_open, const uint64_t *d_open_labels,
                                int64_t capacity, double *d_out_xyz, double *d_out_h, double *d_out_m,
                                double *d_out_s, int32_t *d_out_kind, int64_t *d_out_first, int64_t *d_out_count,
                                int32_t *d_out_branch, uint64_t *d_out_label, int64_t *d_out_owner,
                                int64_t *n_out, sphmap_pseudo_stats *stats, void *stream) {
  if (!ctx) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    SPH_REQUIRE(n >= 1 && n < ((int64_t)1 << 31), SPHMAP_EINVAL, "n out of range [1, 2^31)");
    SPH_REQUIRE(d_xyz && d_h && d_m, SPHMAP_EINVAL, "null particle array");
    SPH_REQUIRE(n_src >= 1 && h_sources, SPHMAP_EINVAL, "at least one source is required");
    SPH_REQUIRE(opts, SPHMAP_EINVAL, "null options");
    SPH_REQUIRE(opts->leaf_max >= 1, SPHMAP_EINVAL, "leaf_max must be >= 1");
    SPH_REQUIRE(opts->max_depth >= 1 && opts->max_depth <= 21, SPHMAP_EINVAL, "max_depth must be in [1, 21]");
    SPH_REQUIRE(opts->theta >= 0 && opts->h_fact > 0 && opts->eps_h > 0, SPHMAP_EINVAL, "bad option value");
    SPH_REQUIRE(d_out_xyz && d_out_h && d_out_m && n_out, SPHMAP_EINVAL, "null required output");
    SPH_REQUIRE(n_open >= 0 && (n_open == 0 || d_open_labels), SPHMAP_EINVAL, "null open-label list");
    sphmap::PseudoArgs a;
    a.n = n;
    a.xyz = d_xyz;
    a.h = d_h;
    a.m = d_m;
    a.n_src = n_src;
    a.src = h_sources;
    a.opts = *opts;
    a.capacity = capacity;
    a.o_xyz = d_out_xyz;
    a.o_h = d_out_h;
    a.o_m = d_out_m;
    a.o_s = d_out_s;
    a.o_kind = d_out_kind;
    a.o_first = d_out_first;
    a.o_count = d_out_count;
    a.o_branch = d_out_branch;
    a.o_label = d_out_label;
    a.o_owner = d_out_owner;
    a.n_open = n_open;
    a.open_labels = d_open_labels;
    a.n_out = 0;
    std::memset(&a.stats, 0, sizeof a.stats);
    sphmap::pseudo_build(ctx->c, a, as_stream(stream));
    *n_out = a.n_out;
    if (stats) *stats = a.stats;
  });
}

int build_pseudo_particles(sphmap_ctx *ctx, int64_t n, const double *d_xyz, const double *d_h, const double *d_m,
                           int32_t n_src, const double *h_sources, const sphmap_pseudo_opts *opts, int64_t capacity,
                           double *d_out_xyz, double *d_out_h, double *d_out_m, double *d_out_s, int32_t *d_out_kind,
                           int64_t *d_out_first, int64_t *d_out_count, int32_t *d_out_branch, int64_t *n_out,
                           sphmap_pseudo_stats *stats, void *stream) {
  return build_pseudo_particles_open(ctx, n, d_xyz, d_h, d_m, n_src, h_sources, opts, 0, nullptr, capacity,
                                     d_out_xyz, d_out_h, d_out_m, d_out_s, d_out_kind, d_out_first, d_out_count,
                                     d_out_branch, nullptr, nullptr, n_out, stats, stream);
}

int build_pseudo_particles_kd(sphmap_ctx *ctx, int64_t n, const double *d_xyz, const double *d_h, const double *d_m,
                              int32_t n_src, const double *h_sources, const sphmap_pseudo_opts *opts,
                              const sphmap_kd_opts *kd, int64_t n_open, const uint64_t *d_open_labels,
                              int64_t capacity, double *d_out_xyz, double *d_out_h, double *d_out_m, double *d_out_s,
                              int32_t *d_out_kind, int64_t *d_out_first, int64_t *d_out_count, int32_t *d_out_branch,
                              uint64_t *d_out_label, int32_t *d_out_level, int64_t *d_out_owner, int64_t *n_out,
                              sphmap_pseudo_stats *stats, int32_t *k_mid, void *stream) {
  if (!ctx) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    SPH_REQUIRE(n >= 1 && n < ((int64_t)1 << 30), SPHMAP_EINVAL, "n out of range [1, 2^30)");
    SPH_REQUIRE(d_xyz && d_h && d_m, SPHMAP_EINVAL, "null particle array");
    SPH_REQUIRE(n_src >= 1 && h_sources, SPHMAP_EINVAL, "at least one source is required");
    SPH_REQUIRE(opts && kd, SPHMAP_EINVAL, "null options");
    SPH_REQUIRE(opts->theta >= 0 && opts->h_fact > 0 && opts->eps_h > 0 && opts->r_part >= 0, SPHMAP_EINVAL,
                "bad option value");
    SPH_REQUIRE(d_out_xyz && d_out_h && d_out_m && n_out, SPHMAP_EINVAL, "null required output");
    SPH_REQUIRE(n_open >= 0 && (n_open == 0 || d_open_labels), SPHMAP_EINVAL, "null open-label list");
    sphmap::KdArgs k;
    sphmap::PseudoArgs &a = k.base;
    a.n = n;
    a.xyz = d_xyz;
    a.h = d_h;
    a.m = d_m;
    a.n_src = n_src;
    a.src = h_sources;
    a.opts = *opts;
    a.capacity = capacity;
    a.o_xyz = d_out_xyz;
    a.o_h = d_out_h;
    a.o_m = d_out_m;
    a.o_s = d_out_s;
    a.o_kind = d_out_kind;
    a.o_first = d_out_first;
    a.o_count = d_out_count;
    a.o_branch = d_out_branch;
    a.o_label = d_out_label;
    a.o_owner = d_out_owner;
    a.n_open = n_open;
    a.open_labels = d_open_labels;
    a.n_out = 0;
    std::memset(&a.stats, 0, sizeof a.stats);
    k.r_leaf = kd->r_leaf;
    k.leaf_split = kd->leaf_split;
    k.up_levels = kd->up_levels;
    k.nf_threshold = kd->nf_threshold;
    k.o_level = d_out_level;
    sphmap::kd_pseudo_build(ctx->c, k, as_stream(stream));
    *n_out = a.n_out;
    if (stats) *stats = a.stats;
    if (k_mid) *k_mid = k.k_mid;
  });
}

int select_underresolved(sphmap_ctx *ctx, int64_t n, const int32_t *d_kind, const uint64_t *d_label,
                         const double *d_s, const double *d_fneu, double s_root, double K, uint64_t *d_out_labels,
                         int64_t *n_found, void *stream) {
  if (!ctx) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    SPH_REQUIRE(n >= 0 && n_found, SPHMAP_EINVAL, "bad count or null output count");
    SPH_REQUIRE(n == 0 || (d_kind && d_label && d_s && d_fneu && d_out_labels), SPHMAP_EINVAL, "null array");
    SPH_REQUIRE(s_root > 0.0 && K > 1.0, SPHMAP_EINVAL, "need s_root > 0 and K > 1");
    *n_found = sphmap::select_underresolved(ctx->c, n, d_kind, d_label, d_s, d_fneu, s_root, K, d_out_labels,
                                            as_stream(stream));
  });
}

int interpolate_to_particles(sphmap_ctx *ctx, int64_t n, const double *d_xyz, const int64_t *d_owner,
                             int64_t n_entries, const double *d_entry_xyz, const double *d_entry_h,
                             const int32_t *d_entry_kind, const double *d_values, int32_t ncomp, double *d_out,
                             void *stream) {
  if (!ctx) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    SPH_REQUIRE(n >= 0 && n < ((int64_t)1 << 31), SPHMAP_EINVAL, "n out of range [0, 2^31)");
    SPH_REQUIRE(n_entries >= 1 && n_entries < ((int64_t)1 << 31), SPHMAP_EINVAL,
                "n_entries out of range [1, 2^31)");
    SPH_REQUIRE(ncomp >= 1, SPHMAP_EINVAL, "ncomp must be at least 1");
    SPH_REQUIRE(n == 0 || (d_xyz && d_owner && d_out), SPHMAP_EINVAL, "null particle array");
    SPH_REQUIRE(d_entry_xyz && d_entry_h && d_entry_kind && d_values, SPHMAP_EINVAL, "null entry array");
    sphmap::interpolate_particles(ctx->c, n, d_xyz, d_owner, n_entries, d_entry_xyz, d_entry_h, d_entry_kind,
                                  d_values, ncomp, d_out, as_stream(stream));
  });
}

int interpolate_to_particles_noalloc(sphmap_ctx *ctx, int64_t n, const double *d_xyz, const int64_t *d_owner,
                                     int64_t n_entries, const double *d_entry_xyz, const double *d_entry_h,
                                     const int32_t *d_entry_kind, const double *d_values, int32_t ncomp,
                                     double *d_out, void *stream) {
  if (!ctx) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    SPH_REQUIRE(n >= 0 && n < ((int64_t)1 << 31), SPHMAP_EINVAL, "n out of range [0, 2^31)");
    SPH_REQUIRE(n_entries >= 1 && n_entries < ((int64_t)1 << 31), SPHMAP_EINVAL,
                "n_entries out of range [1, 2^31)");
    SPH_REQUIRE(ncomp >= 1, SPHMAP_EINVAL, "ncomp must be at least 1");
    SPH_REQUIRE(n == 0 || (d_xyz && d_owner && d_out), SPHMAP_EINVAL, "null particle array");
    SPH_REQUIRE(d_entry_xyz && d_entry_h && d_entry_kind && d_values, SPHMAP_EINVAL, "null entry array");
    sphmap::interpolate_particles_noalloc(ctx->c, n, d_xyz, d_owner, n_entries, d_entry_xyz, d_entry_h,
                                          d_entry_kind, d_values, ncomp, d_out, as_stream(stream));
  });
}

int sphmap_sync_status(sphmap_ctx *ctx, void *stream, int32_t clear, int32_t *status) {
  if (!ctx || !status) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    int v = 0;
    hipStream_t s = as_stream(stream);
    SPH_HIP(hipMemcpyAsync(&v, ctx->c.d_status, sizeof(int), hipMemcpyDeviceToHost, s));
    if (clear) SPH_HIP(hipMemsetAsync(ctx->c.d_status, 0, sizeof(int), s));
    SPH_HIP(hipStreamSynchronize(s));
    *status = v;
  });
}

int sphmap_estimate_footprint(sphmap_ctx *ctx, int64_t n_particles, int64_t n_pairs, int64_t n_cells,
                              int64_t n_faces, int64_t n_face_vertices, int64_t n_vertices, sphmap_footprint *out) {
  if (!ctx || !out) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    SPH_REQUIRE(n_particles >= 0 && n_pairs >= 0 && n_cells >= 0 && n_faces >= 0 && n_face_vertices >= 0 &&
                    n_vertices >= 0,
                SPHMAP_EINVAL, "negative size");
    *out = footprint(ctx->c, n_particles, n_pairs, n_cells, n_faces, n_face_vertices, n_vertices);
  });
}

int sphmap_set_timing(sphmap_ctx *ctx, int32_t enabled) {
  if (!ctx) return SPHMAP_EINVAL;
  ctx->c.timing = enabled != 0;
  return SPHMAP_OK;
}

int sphmap_kernel_time(sphmap_ctx *ctx, const char *name, double *total_ms, int64_t *launches) {
  if (!ctx || !name) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    double tot = 0;
    int64_t cnt = 0;
    auto it = ctx->c.timers.find(name);
    if (it != ctx->c.timers.end())
      for (auto &r : it->second) {
        SPH_HIP(hipEventSynchronize(r.stop));
        float ms = 0;
        SPH_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
        tot += ms;
        ++cnt;
      }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
  });
}

int sphmap_reset_timing(sphmap_ctx *ctx) {
  if (!ctx) return SPHMAP_EINVAL;
  return guarded(ctx, [&] {
    for (auto &kv : ctx->c.timers)
      for (auto &r : kv.second) {
        SPH_HIP(hipEventSynchronize(r.stop));
        SPH_HIP(hipEventDestroy(r.start));
        SPH_HIP(hipEventDestroy(r.stop));
      }
    ctx->c.timers.clear();
  });
}

int sphmap_set_counting(sphmap_ctx *ctx, int32_t enabled) {
  if (!ctx) return SPHMAP_EINVAL;
  ctx->c.counting = enabled != 0;
  return SPHMAP_OK;
}

int sphmap_set_autotune(sphmap_ctx *ctx, int32_t enabled) {
  if (!ctx) return SPHMAP_EINVAL;
  ctx->c.autotune = enabled != 0;
  return SPHMAP_OK;
}

int sphmap_tuned_shape(sphmap_ctx *ctx, int64_t n_pairs, int32_t *blocks_per_cu, int32_t *chunks_per_fetch,
                       double *ms) {
  if (!ctx || n_pairs < 1 || !blocks_per_cu || !chunks_per_fetch) return SPHMAP_EINVAL;
  const int bucket = 63 - __builtin_clzll((unsigned long long)n_pairs);
  auto it = ctx->c.tuned.find(bucket);
  *blocks_per_cu = it == ctx->c.tuned.end() ? 0 : it->second.blocks_per_cu;
  *chunks_per_fetch = it == ctx->c.tuned.end() ? 0 : it->second.per_fetch;
  if (ms) *ms = it == ctx->c.tuned.end() ? 0.0 : it->second.ms;
  return SPHMAP_OK;
}

int sphmap_work_counters(sphmap_ctx *ctx, int64_t *out8) {
  if (!ctx || !out8) return SPHMAP_EINVAL;
  for (int k = 0; k < 8; ++k) out8[k] = ctx->c.counters[k];
  return SPHMAP_OK;
}

}  // extern "C"
