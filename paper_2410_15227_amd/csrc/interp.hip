// Per-particle values from the mixed set of real particles and pseudo-
// particles (Sec. 3.3: rather than giving every member of a pseudo-particle
// its node's value, each SPH particle is interpolated from the entries whose
// smoothing spheres reach it).
//
//   q_i = sum_j V_j W(r_ij, h_j) q_j / sum_j V_j W(r_ij, h_j)
//       = sum_j w(r_ij / h_j) q_j / sum_j w(r_ij / h_j)
//
// the Shepard-normalised SPH interpolant over the entries j with
// r_ij = |x_i - x_j| < 2 h_j, each entry standing for the volume
// V_j = (h_j / h_fact)^3 of the h-density relation (eq. h_node), so that
// only the dimensionless M4 kernel w remains.  A particle that is an entry
// itself keeps that entry's value; a particle no sphere reaches keeps its
// owner's value.
//
// Gather, not scatter: the entries are Morton-sorted under the ball
// hierarchy of the pair search, and one thread walks it per particle, so
// every sum is formed by one thread in an order fixed by the hierarchy (no
// atomics; results repeat bit for bit).  Particles are taken grouped by the
// entry that holds them; the entries are in depth-first (Morton) order, so
// the particles of one wavefront lie in one or a few neighbouring tree nodes
// and their walks visit the same boxes.  Candidates pass a binary32 sphere
// test with the hierarchy's slack before the binary64 distance decides.
#include <mutex>

#include "ballsearch.hpp"

namespace sphmap {
namespace {

constexpr int kCompPass = 4;  // components accumulated per walk

__device__ inline double m4w(double q) {
#pragma clang fp contract(off)
  if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
  if (q < 2.0) return 0.25 * (2.0 - q) * (2.0 - q) * (2.0 - q);
  return 0.0;
}

__global__ void k_interp_check(int64_t n, const double *xyz, const int64_t *owner, int64_t ne, const double *exyz,
                               int *bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double *p = xyz + 3 * i;
    const bool in = p[0] >= 0.0 && p[0] < 1.0 && p[1] >= 0.0 && p[1] < 1.0 && p[2] >= 0.0 && p[2] < 1.0;
    if (!in) atomicOr(bad, 1);
    if (!(owner[i] >= 0 && owner[i] < ne)) atomicOr(bad, 2);
  }
  if (i < ne) {
    const double *p = exyz + 3 * i;
    const bool in = p[0] >= 0.0 && p[0] < 1.0 && p[1] >= 0.0 && p[1] < 1.0 && p[2] >= 0.0 && p[2] < 1.0;
    if (!in) atomicOr(bad, 4);
  }
}

__global__ void k_entry_prep(int64_t ne, const int32_t *sidx, const double *exyz, const double *eh, float4 *sx,
                             double4 *sd) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ne) return;
  const int64_t j = sidx[k];
  const double x = exyz[3 * j], y = exyz[3 * j + 1], z = exyz[3 * j + 2], h = eh[j];
  sx[k] = make_float4((float)x, (float)y, (float)z, (float)h);
  sd[k] = make_double4(x, y, z, h);
}

__global__ void k_owner_keys(int64_t n, const int64_t *owner, uint32_t *key, int32_t *idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = (uint32_t)owner[i];
  idx[i] = (int32_t)i;
}

// One thread per particle, components [c0, c0 + kCompPass) of ncomp.
__global__ void __launch_bounds__(256) k_interp(Hier H, const double4 *sd, int64_t n, const int32_t *qidx,
                                                const double *xyz, const int64_t *owner, const int32_t *ekind,
                                                const double *val, int ncomp, int c0, double *out,
                                                int *status) {
#pragma clang fp contract(off)
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t i = qidx[t];
  const int64_t o = owner[i];
  const int nc = min(kCompPass, ncomp - c0);
  double *oi = out + (int64_t)ncomp * i + c0;
  const double *vo = val + (int64_t)ncomp * o + c0;
  if (ekind[o] == 0) {
    int bad = 0;
    for (int k = 0; k < nc; ++k) {
      oi[k] = vo[k];
      if (!isfinite(vo[k])) bad = SPHMAP_STATUS_NONFINITE_VALUE;
    }
    if (bad) atomicOr(status, bad);
    return;
  }
  const double px = xyz[3 * i], py = xyz[3 * i + 1], pz = xyz[3 * i + 2];
  const float4 g = make_float4((float)px, (float)py, (float)pz, 0.0f);
  const float r2box = H.margin_abs * H.margin_abs;
  double den = 0.0;
  double num[kCompPass] = {0.0, 0.0, 0.0, 0.0};
  uint32_t st[kFan * kMaxLevels];  // node << 4 | level (a level-1 node index is below 2^27)
  int sp = 0;
  const int top = H.levels;
  for (int64_t j = H.n[top] - 1; j >= 0; --j)
    if (box_hit(H.lo[top][j], H.hi[top][j], g, r2box)) st[sp++] = ((uint32_t)j << 4) | (uint32_t)top;
  while (sp > 0) {
    --sp;
    const int l = (int)(st[sp] & 15u);
    const int64_t j = (int64_t)(st[sp] >> 4);
    if (l == 1) {
      const int64_t e = min(H.n[0], (j + 1) * kFan);
      for (int64_t k = j * kFan; k < e; ++k) {
        const float4 b = H.sx[k];
        float dx = b.x - g.x, dy = b.y - g.y, dz = b.z - g.z;
        float rr = 2.0f * b.w * 1.00001f + H.margin_abs;
        if (dx * dx + dy * dy + dz * dz > rr * rr) continue;
        const double4 d = sd[k];
        const double ex = px - d.x, ey = py - d.y, ez = pz - d.z;
        const double r = sqrt(ex * ex + ey * ey + ez * ez);
        if (!(r < 2.0 * d.w)) continue;
        const double W = m4w(r / d.w);
        den += W;
        const double *vj = val + (int64_t)ncomp * H.sidx[k] + c0;
        for (int c = 0; c < nc; ++c) num[c] += W * vj[c];
      }
    } else {
      const int lc = l - 1;
      const int64_t e = min(H.n[lc], (j + 1) * kFan);
      for (int64_t k = e - 1; k >= j * kFan; --k)
        if (box_hit(H.lo[lc][k], H.hi[lc][k], g, r2box)) st[sp++] = ((uint32_t)k << 4) | (uint32_t)lc;
    }
  }
  int bad = 0;
  for (int c = 0; c < nc; ++c) {
    const double v = den > 0.0 ? num[c] / den : vo[c];
    oi[c] = v;
    if (!isfinite(v)) bad = SPHMAP_STATUS_NONFINITE_VALUE;
  }
  if (bad) atomicOr(status, bad);
}

}  // namespace

// ------------------------------------------------- fixed device scratch
// Device memory for callers that cannot allocate (the no-allocation
// interpolation entry point): each device holds one copy for the life of
// the process.  Host code must not pass `scratch` itself to a kernel -- on
// the host that name is a stand-in, not a device address -- but the address
// hipGetSymbolAddress returns on each device, looked up once per device.
constexpr size_t kNoAllocScratch = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Look up this device's copy of the scratch (called with `device` current,
// by context creation).  Later lookups return the recorded address.
void *noalloc_scratch_init(int device) {
  SPH_REQUIRE(device >= 0 && device < kMaxDevices, SPHMAP_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    SPH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    SPH_REQUIRE(p != nullptr, SPHMAP_EHIP, "no device address for the fixed scratch");
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

size_t noalloc_scratch_bytes() { return kNoAllocScratch; }

// Upper bound of the scratch interpolate_particles carves for n particles
// and ne entries: Morton keys, index, sorted float4 and double4 copies and
// radix temporaries per entry; owner keys, index and radix temporaries per
// particle; the search boxes; digit histograms and scan sums; and 256 bytes
// of alignment and padding for each of up to 64 named buffers.
size_t interp_scratch_bound(int64_t n, int64_t ne) {
  const double per_entry = 8 + 4 + 8 + 4 + 16 + 32 + 2.2 * 16;
  const double per_part = 4 + 4 + 4 + 4;
  const double hist = 4.0 * (16.0 * (double)(div_up(std::max(n, ne), 2048) + 1) * 8.0 + 64.0);
  return (size_t)(per_entry * (double)ne + per_part * (double)n + hist + 64.0 * 512.0 + 65536.0);
}

void interpolate_particles(Ctx &ctx, int64_t n, const double *xyz, const int64_t *owner, int64_t ne,
                           const double *exyz, const double *eh, const int32_t *ekind, const double *val, int ncomp,
                           double *out, hipStream_t s) {
  if (n <= 0) return;
  SPH_REQUIRE(ne > 0 && ne < ((int64_t)1 << 31), SPHMAP_EINVAL, "entry count out of range");
  SPH_REQUIRE(n < ((int64_t)1 << 31), SPHMAP_EINVAL, "particle count out of range");
  SPH_REQUIRE(ncomp >= 1, SPHMAP_EINVAL, "ncomp must be at least 1");
  Arena &ar = ctx.arena;
  int *bad = ar.get<int>("ip_bad", 1);
  SPH_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  k_interp_check<<<(unsigned)div_up(std::max(n, ne), 256), 256, 0, s>>>(n, xyz, owner, ne, exyz, bad);
  SPH_LAUNCH_CHECK();
  int bad_h = 0;
  SPH_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  SPH_REQUIRE(!(bad_h & 2), SPHMAP_EINVAL, "owner index outside [0, n_entries)");
  SPH_REQUIRE(!(bad_h & 5), SPHMAP_EINVAL, "particle or entry outside [0,1)^3");

  // entries in Morton order under the ball hierarchy
  uint64_t *keys = ar.get<uint64_t>("ip_keys", ne);
  int32_t *sidx = ar.get<int32_t>("ip_sidx", ne);
  morton_keys(exyz, 3, ne, 0.0, 0.0, 0.0, 1.0, keys, sidx, s);
  radix_sort_u64_range(ar, keys, sidx, ne, 33, 63, s);  // top 10 bits per axis
  float4 *sx = ar.get<float4>("ip_sx", ne);
  double4 *sd = ar.get<double4>("ip_sd", ne);
  k_entry_prep<<<(unsigned)div_up(ne, 256), 256, 0, s>>>(ne, sidx, exyz, eh, sx, sd);
  SPH_LAUNCH_CHECK();
  Hier H;
  H.sx = sx;
  H.sidx = sidx;
  build_hier(ar, sx, ne, 1e-6f, "ip", H, s);

  // particles grouped by the entry that holds them
  uint32_t *okey = ar.get<uint32_t>("ip_okey", n);
  int32_t *qidx = ar.get<int32_t>("ip_qidx", n);
  k_owner_keys<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, owner, okey, qidx);
  SPH_LAUNCH_CHECK();
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < ne) ++bits;
  radix_sort_u32(ar, okey, qidx, n, bits, s);

  KernelTimer kt(&ctx, "interp", s);
  for (int c0 = 0; c0 < ncomp; c0 += kCompPass) {
    k_interp<<<(unsigned)div_up(n, 256), 256, 0, s>>>(H, sd, n, qidx, xyz, owner, ekind, val, ncomp, c0, out,
                                                       ctx.d_status);
    SPH_LAUNCH_CHECK();
  }
  kt.done();
}

// The same with every buffer carved from this device's fixed scratch: no
// device memory is allocated or freed.  Calls on one device share the
// scratch, so calls that overlap in time on one device race.
void interpolate_particles_noalloc(Ctx &ctx, int64_t n, const double *xyz, const int64_t *owner, int64_t ne,
                                   const double *exyz, const double *eh, const int32_t *ekind, const double *val,
                                   int ncomp, double *out, hipStream_t s) {
  SPH_REQUIRE(ne > 0 && ne < ((int64_t)1 << 31) && n >= 0 && n < ((int64_t)1 << 31), SPHMAP_EINVAL,
              "particle or entry count out of range");
  const size_t need = interp_scratch_bound(n, ne);
  SPH_REQUIRE(need <= kNoAllocScratch, SPHMAP_EINVAL,
              "n = " + std::to_string(n) + " particles and " + std::to_string(ne) + " entries need up to " +
                  std::to_string(need) + " bytes, more than the " + std::to_string(kNoAllocScratch) +
                  "-byte fixed scratch");
  void *base = g_scratch_ptr[ctx.device];
  SPH_REQUIRE(base != nullptr, SPHMAP_EHIP, "the fixed scratch of this device was not looked up");
  Arena region;
  region.region = (char *)base;
  region.region_cap = kNoAllocScratch;
  struct Swap {  // every request of the call goes to the region; timing off (no events)
    Ctx &c;
    bool timing;
    Swap(Ctx &cc, Arena *r) : c(cc), timing(cc.timing) {
      c.arena.redirect = r;
      c.timing = false;
    }
    ~Swap() {
      c.arena.redirect = nullptr;
      c.timing = timing;
    }
  } swap(ctx, &region);
  interpolate_particles(ctx, n, xyz, owner, ne, exyz, eh, ekind, val, ncomp, out, s);
}

}  // namespace sphmap
