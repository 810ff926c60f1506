// Accumulations over the pair list.
//
//  cell_reduce     M_c = sum_i m_i w_ic (forward mapping, Sec. 2.3) over the
//                  cell's pairs, rho_c = M_c / V_c.  One wave per cell; lanes
//                  take the cell's pairs in stride and a fixed butterfly
//                  combines them, so the result does not depend on the launch
//                  (products are rounded before they are added, so the order
//                  stated in include/sphmap.h reproduces the sums exactly).
//  particle_major  the pair list re-ordered by particle (stable radix sort of
//                  the particle index, so each particle's cells stay in
//                  ascending cell order) with c_i = sum_c w_ic.
//  reverse_map     q_i = sum_c w_ic q_c / c_i (inverse mapping, Sec. 2.3).
#include "common.hpp"

namespace sphmap {
namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Several particles per wavefront in the coverage sum: every lane issues
// the loads of all of its group's runs before it adds any, so a wavefront
// keeps many loads in flight instead of waiting out one short run at a time.
constexpr int kGroup = 4;  // particles per wavefront
constexpr int kTurns = 4;  // 64-entry turns of each run per round of loads

__device__ inline int64_t uniform_i64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__global__ void __launch_bounds__(256) k_cell_mass(int64_t C, const int64_t *off, const int32_t *pair_p,
                                                  const double *w, const double *m, const double *cov,
                                                  const double *vol, double *mass, double *rho, int *status) {
#pragma clang fp contract(off)  // each product rounded, then added: the order include/sphmap.h states
  const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (c >= C) return;
  const int64_t s = off[c], e = off[c + 1];
  double acc = 0.0;
  // four turns of the lane's loop at a time: their index and weight loads,
  // then their mass gathers, are in flight together; the additions keep the
  // lane's order
  for (int64_t k0 = s + lane; k0 < e; k0 += 256) {
    int32_t i[4];
    double wk[4], mi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t k = k0 + 64 * j;
      i[j] = k < e ? pair_p[k] : 0;
      wk[j] = k < e ? w[k] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      mi[j] = m[i[j]];
      if (cov) mi[j] = cov[i[j]] > 0.0 ? mi[j] / cov[i[j]] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (k0 + 64 * j < e) acc += mi[j] * wk[j];
  }
  acc = wave_sum(acc);
  if (lane == 0) {
    mass[c] = acc;
    if (rho) rho[c] = acc / vol[c];
    if (!isfinite(acc)) atomicOr(status, SPHMAP_STATUS_NONFINITE_MASS);
  }
}

// Particle offsets from the sorted particle keys: position k starts every
// particle in (key[k-1], key[k]] (particles without pairs start where the
// next one does); the end, NP, starts every particle after the last key.
// (dNP: a pair count known only on the device, at most NP.)
__global__ void k_part_offsets(int64_t NP, int64_t N, const uint32_t *key, int64_t *part_off,
                               const int64_t *dNP = nullptr) {
  // four positions per thread, their keys loaded together
  const int64_t k0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (dNP) NP = *dNP;
  if (k0 > NP) return;
  int64_t kv[5];
  kv[0] = k0 == 0 ? -1 : (int64_t)key[k0 - 1];
#pragma unroll
  for (int q = 0; q < 4; ++q) kv[q + 1] = k0 + q < NP ? (int64_t)key[k0 + q] : N;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t k = k0 + q;
    if (k > NP) break;
    for (int64_t j = kv[q] + 1; j <= kv[q + 1]; ++j) part_off[j] = k;
  }
}

// c_i = sum_c w_ic over each particle's run of the particle-major list
// (ascending cell order), kGroup particles per wavefront.
__global__ void __launch_bounds__(256) k_coverage(int64_t N, const int64_t *poff, const double *pm_w, double *cov) {
  const int64_t i0 = uniform_i64((((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * kGroup);
  const int lane = threadIdx.x & 63;
  if (i0 >= N) return;
  int64_t s[kGroup], e[kGroup], len = 0;
#pragma unroll
  for (int g = 0; g < kGroup; ++g) {
    const int64_t a = min(i0 + g, N), b = min(i0 + g + 1, N);
    s[g] = uniform_i64(poff[a]);
    e[g] = a < N ? uniform_i64(poff[b]) : s[g];
    len = max(len, e[g] - s[g]);
  }
  double acc[kGroup];
#pragma unroll
  for (int g = 0; g < kGroup; ++g) acc[g] = 0.0;
  for (int64_t t0 = lane; t0 < len; t0 += 64 * kTurns) {
    double v[kGroup][kTurns];
#pragma unroll
    for (int g = 0; g < kGroup; ++g)
#pragma unroll
      for (int u = 0; u < kTurns; ++u) {
        const int64_t j = s[g] + t0 + 64 * u;
        v[g][u] = j < e[g] ? pm_w[j] : 0.0;
      }
#pragma unroll
    for (int g = 0; g < kGroup; ++g)
#pragma unroll
      for (int u = 0; u < kTurns; ++u)
        if (s[g] + t0 + 64 * u < e[g]) acc[g] += v[g][u];
  }
#pragma unroll
  for (int g = 0; g < kGroup; ++g) acc[g] = wave_sum(acc[g]);
  if (lane < kGroup) {
    double a = acc[0];
#pragma unroll
    for (int g = 1; g < kGroup; ++g) a = lane == g ? acc[g] : a;
    if (i0 + lane < N) cov[i0 + lane] = a;
  }
}

template <int kComp>
__global__ void __launch_bounds__(256) k_reverse(int64_t N, int ncomp, const int64_t *poff, const int32_t *pm_cell,
                                                const double *pm_w, const double *cov, const double *q,
                                                double *out, int *status) {
#pragma clang fp contract(off)  // each product rounded, then added: the order include/sphmap.h states
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int lane = threadIdx.x & 15;  // 16 lanes per particle
  if (i >= N) return;
  const int nc = kComp > 0 ? kComp : ncomp;
  const int64_t s = poff[i], e = poff[i + 1];
  double acc[kComp > 0 ? kComp : 1];
  for (int j = 0; j < (kComp > 0 ? kComp : 1); ++j) acc[j] = 0.0;
  if (kComp > 0) {
    // unrolled so that several turns' loads are in flight; each lane still
    // adds its terms in index order
#pragma unroll 4
    for (int64_t j = s + lane; j < e; j += 16) {
      const double wj = pm_w[j];
      const int64_t c = pm_cell[j];
#pragma unroll
      for (int r = 0; r < kComp; ++r) acc[r] += wj * q[c * kComp + r];
    }
#pragma unroll
    for (int r = 0; r < kComp; ++r) {
      double v = acc[r];
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
      acc[r] = v;
    }
    if (lane == 0) {
      const double ci = cov[i];
      int bad = ci > 0.0 ? 0 : SPHMAP_STATUS_ZERO_COVERAGE;
      for (int r = 0; r < kComp; ++r) {
        const double v = ci > 0.0 ? acc[r] / ci : 0.0;
        out[i * kComp + r] = v;
        if (!isfinite(v)) bad |= SPHMAP_STATUS_NONFINITE_VALUE;
      }
      if (bad) atomicOr(status, bad);
    }
  } else {
    const double ci = cov[i];
    int bad = ci > 0.0 ? 0 : SPHMAP_STATUS_ZERO_COVERAGE;
    for (int r = 0; r < nc; ++r) {
      double v = 0.0;
      for (int64_t j = s + lane; j < e; j += 16) v += pm_w[j] * q[(int64_t)pm_cell[j] * nc + r];
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
      v = ci > 0.0 ? v / ci : 0.0;
      if (lane == 0) out[i * nc + r] = v;
      if (!isfinite(v)) bad |= SPHMAP_STATUS_NONFINITE_VALUE;
    }
    if (lane == 0 && bad) atomicOr(status, bad);
  }
}

}  // namespace

void cell_reduce(Ctx &ctx, const TessDev &t, const PartDev &p, const PairsDev &P, bool normalize, double *mass,
                 double *rho, hipStream_t s) {
  const int64_t C = t.n_cells;
  if (C == 0) return;
  KernelTimer kt(&ctx, "cell_reduce", s);
  k_cell_mass<<<(unsigned)div_up(C * 64, 256), 256, 0, s>>>(C, P.cell_off, P.pair_p, P.w, p.m,
                                                            normalize ? P.coverage : nullptr, t.volume, mass, rho,
                                                            ctx.d_status);
  SPH_LAUNCH_CHECK();
  kt.done();
}

void particle_major(Ctx &ctx, PairsDev &P, hipStream_t s) {
  Arena &ar = ctx.arena;
  const int64_t N = P.n_particles, NP = P.n_pairs;
  P.part_off = P.mem.get<int64_t>("part_off", N + 1);
  P.pm_cell = P.mem.get<int32_t>("pm_cell", NP);
  P.pm_w = P.mem.get<double>("pm_w", NP);
  P.coverage = P.mem.get<double>("coverage", N);
  KernelTimer kt(&ctx, "transpose", s);
  if (NP > 0) {
    // stable sort of the (particle, cell, w) triples by particle: each
    // particle's pairs keep ascending cell order, and cell and weight move
    // with the key, so nothing is gathered afterwards
    uint32_t *keys = ar.get<uint32_t>("pm_keys", NP);
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) < N) ++bits;
    // (capacity mode: NP is the capacity and P.d_np the count on the device)
    sort_by_key_kv(ar, NP, bits, (const uint32_t *)P.pair_p, P.pair_c, P.w, keys, P.pm_cell, P.pm_w, s,
                   P.cap > 0 ? P.d_np : nullptr);
    k_part_offsets<<<(unsigned)div_up(div_up(NP + 1, 4), 256), 256, 0, s>>>(NP, N, keys, P.part_off,
                                                                 P.cap > 0 ? P.d_np : nullptr);
    SPH_LAUNCH_CHECK();
    k_coverage<<<(unsigned)div_up(div_up(N, kGroup) * 64, 256), 256, 0, s>>>(N, P.part_off, P.pm_w, P.coverage);
    SPH_LAUNCH_CHECK();
  } else {
    fill_i64(P.part_off, 0, N + 1, s);
    SPH_HIP(hipMemsetAsync(P.coverage, 0, N * sizeof(double), s));
  }
  kt.done();
}

void reverse_map(Ctx &ctx, const PairsDev &P, const double *q, int ncomp, double *out, hipStream_t s) {
  const int64_t N = P.n_particles;
  if (N == 0) return;
  KernelTimer kt(&ctx, "reverse", s);
  const unsigned grid = (unsigned)div_up(N * 16, 256);
  if (ncomp == 1)
    k_reverse<1><<<grid, 256, 0, s>>>(N, 1, P.part_off, P.pm_cell, P.pm_w, P.coverage, q, out, ctx.d_status);
  else if (ncomp == 2)
    k_reverse<2><<<grid, 256, 0, s>>>(N, 2, P.part_off, P.pm_cell, P.pm_w, P.coverage, q, out, ctx.d_status);
  else if (ncomp == 4)
    k_reverse<4><<<grid, 256, 0, s>>>(N, 4, P.part_off, P.pm_cell, P.pm_w, P.coverage, q, out, ctx.d_status);
  else
    k_reverse<0><<<grid, 256, 0, s>>>(N, ncomp, P.part_off, P.pm_cell, P.pm_w, P.coverage, q, out,
                                      ctx.d_status);
  SPH_LAUNCH_CHECK();
  kt.done();
}

}  // namespace sphmap
