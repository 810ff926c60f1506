// The Voronoi grid on the device (Sec. 2.3: the grid code builds the Voronoi
// grid of the generation sites and regularises it with Lloyd iterations
// before the forward mapping).
//
// Cell of generator g: the box cut by the bisector half-space of every
// generator that can reach it.  One wavefront builds one cell.  The convex
// cell is held as the triangulation dual to its faces: each vertex of the
// cell is a triangle (a, b, c) of the three planes that meet there, in an
// orientation shared by all triangles, and a table T[a][b] names the
// triangle holding the directed edge a -> b.  A cut by plane p removes the
// vertices beyond it; every edge a -> b of a removed triangle whose twin
// b -> a belongs to a kept triangle is a cell edge crossing p, and becomes
// the new vertex (a, b, p) at the crossing point.  The 64 lanes classify,
// create and compact vertices in parallel; cuts are applied one after the
// other.
//
// Neighbours come from a uniform grid (about two generators per grid cell)
// searched in rings of growing Chebyshev radius, nearest ring cells first.
// A generator at distance D can cut only when D/2 does not exceed the
// largest vertex distance R of the current cell, so the search stops once
// the next ring is further than 2R (the security radius).
//
// Outputs, per mode: volume and centroid (Lloyd iterations); face, face
// vertex and vertex counts; the faces themselves (each face's vertex cycle
// walked through T) with the neighbour each one faces.
#include "common.hpp"

namespace sphmap {
namespace {

constexpr int kVP = 64;     // planes per cell: 6 box planes + neighbours
constexpr int kVT = 128;    // vertices per cell
constexpr int kVWaves = 4;  // cells per workgroup
constexpr int kCand = 256;  // sites listed at a time per wave

// error bits
constexpr int kErrCoincident = 1;
constexpr int kErrPlanes = 2;
constexpr int kErrVertices = 4;
constexpr int kErrCycle = 8;
constexpr int kErrOutside = 16;

struct VorLds {
  double pn[kVP][4];     // plane: unit normal, offset from the generator
  int32_t pid[kVP];      // neighbouring generator, or -1..-6 for box planes
  uint8_t tri[kVT][4];   // the three planes of each vertex
  double vx[kVT], vy[kVT], vz[kVT];  // vertex positions about the generator
  uint8_t T[kVP][kVP];   // vertex holding directed edge a -> b
  uint8_t first[kVP];    // a vertex on each plane (valid when it holds it)
  uint8_t outf[kVT];
  uint8_t remap[kVP];
  int32_t list[kCand];   // sorted-array positions of a group's sites
};

struct VorGrid {
  double lo[3], hi[3], cs[3];
  int G[3];
  const int32_t *start, *end;  // per grid cell, into sorted
  const int32_t *sorted;       // generator indices by grid cell
  const double *gen;
};

__device__ inline void vsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int vscan_excl(int v, int lane) {
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x - v;
}

__device__ inline int vsum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double vsumd(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double vmaxd(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ inline double readlane_d(double v, int j) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, j);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), j);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ inline uint64_t ballot64(bool p) { return (uint64_t)__ballot(p); }

// Rebuild the edge table and plane anchors from the current vertices, and
// return the largest squared vertex distance.
__device__ inline double vrebuild(VorLds &L, int nT, int lane) {
  double r2 = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = lane + 64 * h;
    if (t < nT) {
      const int a = L.tri[t][0], b = L.tri[t][1], c = L.tri[t][2];
      L.T[a][b] = (uint8_t)t;
      L.T[b][c] = (uint8_t)t;
      L.T[c][a] = (uint8_t)t;
      L.first[a] = (uint8_t)t;
      L.first[b] = (uint8_t)t;
      L.first[c] = (uint8_t)t;
      r2 = fmax(r2, L.vx[t] * L.vx[t] + L.vy[t] * L.vy[t] + L.vz[t] * L.vz[t]);
    }
  }
  vsync();
  return vmaxd(r2);
}

// Drop the planes no vertex lies on any more and renumber the rest; returns
// the new plane count.
__device__ int vcompact(VorLds &L, int nP, int nT, int lane) {
  bool used = false;
  if (lane < nP) {
    const int t0 = L.first[lane] & (kVT - 1);
    used = t0 < nT && (L.tri[t0][0] == lane || L.tri[t0][1] == lane || L.tri[t0][2] == lane);
  }
  const uint64_t um = ballot64(used);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int to = __popcll(um & below);
  double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
  int32_t id = 0;
  if (used) {
    q0 = L.pn[lane][0];
    q1 = L.pn[lane][1];
    q2 = L.pn[lane][2];
    q3 = L.pn[lane][3];
    id = L.pid[lane];
    L.remap[lane] = (uint8_t)to;
  }
  uint32_t tr[2] = {0, 0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = lane + 64 * h;
    if (t < nT) tr[h] = *(const uint32_t *)L.tri[t];
  }
  vsync();
  if (used) {
    L.pn[to][0] = q0;
    L.pn[to][1] = q1;
    L.pn[to][2] = q2;
    L.pn[to][3] = q3;
    L.pid[to] = id;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = lane + 64 * h;
    if (t < nT) {
      L.tri[t][0] = L.remap[tr[h] & 0xff];
      L.tri[t][1] = L.remap[(tr[h] >> 8) & 0xff];
      L.tri[t][2] = L.remap[(tr[h] >> 16) & 0xff];
    }
  }
  vsync();
  (void)vrebuild(L, nT, lane);
  return __popcll(um);
}

// Cut by n.x <= d (about the generator).  Returns false on an overflow
// (bit in *err); r2 is refreshed after a cut.
__device__ bool vclip(VorLds &L, int &nP, int &nT, double nx, double ny, double nz, double d, int32_t id, double eps,
                      double &r2, int lane, int *err) {
  double s[2] = {0.0, 0.0};
  bool o[2] = {false, false};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = lane + 64 * h;
    if (t < nT) {
      s[h] = nx * L.vx[t] + ny * L.vy[t] + nz * L.vz[t] - d;
      o[h] = s[h] > eps;
    }
  }
  const uint64_t m0 = ballot64(o[0]), m1 = ballot64(o[1]);
  if (!(m0 | m1)) return true;
  if (nP >= kVP) nP = vcompact(L, nP, nT, lane);
  if (nP >= kVP) {
    if (lane == 0) atomicOr(err, kErrPlanes);
    return false;
  }
  const int p = nP;
  if (lane == 0) {
    L.pn[p][0] = nx;
    L.pn[p][1] = ny;
    L.pn[p][2] = nz;
    L.pn[p][3] = d;
    L.pid[p] = id;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = lane + 64 * h;
    if (t < nT) L.outf[t] = o[h] ? 1 : 0;
  }
  vsync();
  // the vertices each removed vertex hands to the cut: one per edge whose
  // twin is kept, at the point where that cell edge crosses the plane
  uint8_t na[6], nb[6];
  double nxs[6], nys[6], nzs[6];
  bool nv[6];
  int cnt = 0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = lane + 64 * h;
    const bool rm = o[h];
    int a = 0, b = 0, c = 0;
    double px = 0.0, py = 0.0, pz = 0.0;
    if (rm) {
      a = L.tri[t][0];
      b = L.tri[t][1];
      c = L.tri[t][2];
      px = L.vx[t];
      py = L.vy[t];
      pz = L.vz[t];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int u = r == 0 ? a : (r == 1 ? b : c);
      const int v = r == 0 ? b : (r == 1 ? c : a);
      const int k = 3 * h + r;
      nv[k] = false;
      na[k] = (uint8_t)u;
      nb[k] = (uint8_t)v;
      nxs[k] = nys[k] = nzs[k] = 0.0;
      if (rm) {
        const int t2 = L.T[v][u] & (kVT - 1);
        if (!L.outf[t2]) {
          const double qx = L.vx[t2], qy = L.vy[t2], qz = L.vz[t2];
          const double s2 = nx * qx + ny * qy + nz * qz - d;
          double w = s[h] / (s[h] - s2);
          w = fmin(fmax(w, 0.0), 1.0);
          nxs[k] = px + w * (qx - px);
          nys[k] = py + w * (qy - py);
          nzs[k] = pz + w * (qz - pz);
          nv[k] = true;
          ++cnt;
        }
      }
    }
  }
  const int base_new = vscan_excl(cnt, lane);
  const int total_new = vsum(cnt);
  const int removed = __popcll(m0) + __popcll(m1);
  const int K = nT - removed;
  if (K + total_new > kVT) {
    if (lane == 0) atomicOr(err, kErrVertices);
    return false;
  }
  // kept vertices keep their order; new ones follow
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint64_t v0 = nT >= 64 ? ~0ull : ((1ull << nT) - 1ull);
  const uint64_t v1 = nT - 64 >= 64 ? ~0ull : (nT > 64 ? ((1ull << (nT - 64)) - 1ull) : 0ull);
  const uint64_t k0 = v0 & ~m0, k1 = v1 & ~m1;
  int dst[2];
  dst[0] = __popcll(k0 & below);
  dst[1] = __popcll(k0) + __popcll(k1 & below);
  uint32_t keep_tri[2];
  double kx[2], ky[2], kz[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = lane + 64 * h;
    keep_tri[h] = 0;
    kx[h] = ky[h] = kz[h] = 0.0;
    if (t < nT && !o[h]) {
      keep_tri[h] = *(const uint32_t *)L.tri[t];
      kx[h] = L.vx[t];
      ky[h] = L.vy[t];
      kz[h] = L.vz[t];
    }
  }
  vsync();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = lane + 64 * h;
    if (t < nT && !o[h]) {
      *(uint32_t *)L.tri[dst[h]] = keep_tri[h];
      L.vx[dst[h]] = kx[h];
      L.vy[dst[h]] = ky[h];
      L.vz[dst[h]] = kz[h];
    }
  }
  int at = K + base_new;
#pragma unroll
  for (int k = 0; k < 6; ++k)
    if (nv[k]) {
      L.tri[at][0] = na[k];
      L.tri[at][1] = nb[k];
      L.tri[at][2] = (uint8_t)p;
      L.tri[at][3] = 0;
      L.vx[at] = nxs[k];
      L.vy[at] = nys[k];
      L.vz[at] = nzs[k];
      ++at;
    }
  nT = K + total_new;
  nP = p + 1;
  vsync();
  r2 = vrebuild(L, nT, lane);
  return true;
}

// Cut by the candidates of one batch (lane: a position in the sorted site
// array, or -1), nearest first.  Returns false on an error (bit in *err).
__device__ bool vbatch(VorLds &L, const VorGrid &Gd, int64_t c, double gx, double gy, double gz, int k, int &nP,
                       int &nT, double &r2, double eps, int lane, int *err) {
  int32_t j = -1;
  double ex = 0.0, ey = 0.0, ez = 0.0, dist = 0.0;
  if (k >= 0) {
    j = Gd.sorted[k];
    ex = Gd.gen[3 * (int64_t)j] - gx;
    ey = Gd.gen[3 * (int64_t)j + 1] - gy;
    ez = Gd.gen[3 * (int64_t)j + 2] - gz;
    dist = sqrt(ex * ex + ey * ey + ez * ez);
  }
  const bool cand = j >= 0 && j != (int32_t)c && 0.5 * dist <= sqrt(r2) + eps;
  const int ncand = __popcll(ballot64(cand));
  if (ncand == 0) return true;
  // sort (distance, lane) across the wave
  uint64_t key = cand ? (((uint64_t)__float_as_uint((float)dist) << 32) | (uint64_t)lane) : ~0ull;
#pragma unroll
  for (int kk = 2; kk <= 64; kk <<= 1)
#pragma unroll
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      const uint64_t other = (uint64_t)__shfl_xor((long long)key, jj, 64);
      const bool up = (lane & kk) == 0, lower = (lane & jj) == 0;
      key = (lower == up) ? (key < other ? key : other) : (key > other ? key : other);
    }
  for (int i = 0; i < ncand; ++i) {
    const int l = __builtin_amdgcn_readlane((int)(uint32_t)key, i) & 63;
    const double dd = readlane_d(dist, l);
    if (0.5 * dd > sqrt(r2) + eps) break;
    if (!(dd > 0.0)) {
      if (lane == 0) atomicOr(err, kErrCoincident);
      return false;
    }
    const int32_t jj = __builtin_amdgcn_readlane(j, l);
    const double nx = readlane_d(ex, l) / dd, ny = readlane_d(ey, l) / dd, nz = readlane_d(ez, l) / dd;
    if (!vclip(L, nP, nT, nx, ny, nz, 0.5 * dd, jj, eps, r2, lane, err)) return false;
  }
  return true;
}

// Sort one 64-bit key per lane across the wave, ascending.
__device__ inline uint64_t vsort64(uint64_t key, int lane) {
#pragma unroll
  for (int kk = 2; kk <= 64; kk <<= 1)
#pragma unroll
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      const uint64_t other = (uint64_t)__shfl_xor((long long)key, jj, 64);
      const bool up = (lane & kk) == 0, lower = (lane & jj) == 0;
      key = (lower == up) ? (key < other ? key : other) : (key > other ? key : other);
    }
  return key;
}

// Keep the 64 smallest of two ascending 64-lane lists, ascending.
__device__ inline uint64_t vmerge64(uint64_t best, uint64_t chunk, int lane) {
  const uint64_t rev = (uint64_t)__shfl((long long)chunk, 63 - lane, 64);
  uint64_t key = best < rev ? best : rev;  // bitonic: the 64 smallest of both
#pragma unroll
  for (int jj = 32; jj > 0; jj >>= 1) {
    const uint64_t other = (uint64_t)__shfl_xor((long long)key, jj, 64);
    const bool lower = (lane & jj) == 0;
    key = lower ? (key < other ? key : other) : (key > other ? key : other);
  }
  return key;
}

// A group of grid cells (lane l: sites [s0, s0 + cnt) of the sorted array,
// at offset off of the group's tot sites) is listed kCand sites at a time.
__device__ inline void vwindow(VorLds &L, int s0, int cnt, int off, int w0, int lane) {
  (void)lane;
  const int e0 = max(0, w0 - off), e1 = min(cnt, w0 + kCand - off);
  for (int e = e0; e < e1; ++e) L.list[off + e - w0] = s0 + e;
  vsync();
}

// Cut by every site of a group.  With `nearest`, the 64 sites nearest to
// the generator cut first, so that the cell is close to its final shape
// before the rest are tested (far sites cutting a large cell first would
// leave many short-lived faces).
__device__ bool vgroup(VorLds &L, const VorGrid &Gd, int64_t c, double gx, double gy, double gz, int s0, int cnt,
                       bool nearest, int &nP, int &nT, double &r2, double eps, int lane, int *err) {
  const int off = vscan_excl(cnt, lane);
  const int tot = vsum(cnt);
  if (nearest) {
    uint64_t best = ~0ull;
    for (int w0 = 0; w0 < tot; w0 += kCand) {
      vwindow(L, s0, cnt, off, w0, lane);
      const int wn = min(kCand, tot - w0);
      for (int b = 0; b < wn; b += 64) {
        uint64_t key = ~0ull;
        if (b + lane < wn) {
          const int32_t j = Gd.sorted[L.list[b + lane]];
          const double ex = Gd.gen[3 * (int64_t)j] - gx, ey = Gd.gen[3 * (int64_t)j + 1] - gy,
                       ez = Gd.gen[3 * (int64_t)j + 2] - gz;
          if (j != (int32_t)c)
            key = ((uint64_t)__float_as_uint((float)sqrt(ex * ex + ey * ey + ez * ez)) << 32) | (uint32_t)j;
        }
        best = vmerge64(best, vsort64(key, lane), lane);
      }
      vsync();
    }
    int32_t j = -1;
    double ex = 0.0, ey = 0.0, ez = 0.0, dist = 0.0;
    if (best != ~0ull) {
      j = (int32_t)(best & 0xffffffffull);
      ex = Gd.gen[3 * (int64_t)j] - gx;
      ey = Gd.gen[3 * (int64_t)j + 1] - gy;
      ez = Gd.gen[3 * (int64_t)j + 2] - gz;
      dist = sqrt(ex * ex + ey * ey + ez * ez);
    }
    const int nb = __popcll(ballot64(j >= 0));
    for (int l = 0; l < nb; ++l) {
      const double dd = readlane_d(dist, l);
      if (0.5 * dd > sqrt(r2) + eps) break;
      if (!(dd > 0.0)) {
        if (lane == 0) atomicOr(err, kErrCoincident);
        return false;
      }
      const int32_t jj = __builtin_amdgcn_readlane(j, l);
      if (!vclip(L, nP, nT, readlane_d(ex, l) / dd, readlane_d(ey, l) / dd, readlane_d(ez, l) / dd, 0.5 * dd, jj,
                 eps, r2, lane, err))
        return false;
    }
  }
  for (int w0 = 0; w0 < tot; w0 += kCand) {
    vwindow(L, s0, cnt, off, w0, lane);
    const int wn = min(kCand, tot - w0);
    for (int b = 0; b < wn; b += 64)
      if (!vbatch(L, Gd, c, gx, gy, gz, b + lane < wn ? L.list[b + lane] : -1, nP, nT, r2, eps, lane, err))
        return false;
    vsync();
  }
  return true;
}

__device__ inline int gcell(double x, double lo, double cs, int G) {
  int i = (int)floor((x - lo) / cs);
  return min(max(i, 0), G - 1);
}

template <int kMode>  // 0: volume and centroid; 1: counts; 2: faces
__global__ void __launch_bounds__(64 * kVWaves) k_voronoi(VorGrid Gd, int64_t n, double eps, double *centroid,
                                                          double *volume, int64_t *cnt, const int64_t *off,
                                                          double *vert, int64_t *cell_face_off, int64_t *face_vtx_off,
                                                          int32_t *face_vtx, int32_t *face_nbr, int *err) {
  __shared__ VorLds S[kVWaves];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * kVWaves + w;
  if (c >= n) return;
  VorLds &L = S[w];
  const double gx = Gd.gen[3 * c], gy = Gd.gen[3 * c + 1], gz = Gd.gen[3 * c + 2];
  // the box: planes x-, x+, y-, y+, z-, z+ and its eight corners
  if (lane < 6) {
    const int ax = lane >> 1;
    const bool up = lane & 1;
    const double g = ax == 0 ? gx : (ax == 1 ? gy : gz);
    L.pn[lane][0] = ax == 0 ? (up ? 1.0 : -1.0) : 0.0;
    L.pn[lane][1] = ax == 1 ? (up ? 1.0 : -1.0) : 0.0;
    L.pn[lane][2] = ax == 2 ? (up ? 1.0 : -1.0) : 0.0;
    L.pn[lane][3] = up ? Gd.hi[ax] - g : g - Gd.lo[ax];
    L.pid[lane] = -1 - lane;
  }
  if (lane < 8) {
    const int sx = lane & 1, sy = (lane >> 1) & 1, sz = (lane >> 2) & 1;
    const int px = sx ? 1 : 0, py = sy ? 3 : 2, pz = sz ? 5 : 4;
    // corner (+,+,+) is (x+, y+, z+); a reflection swaps the orientation
    const bool pos3 = (sx ? 1 : -1) * (sy ? 1 : -1) * (sz ? 1 : -1) > 0;
    L.tri[lane][0] = (uint8_t)px;
    L.tri[lane][1] = (uint8_t)(pos3 ? py : pz);
    L.tri[lane][2] = (uint8_t)(pos3 ? pz : py);
    L.tri[lane][3] = 0;
    L.vx[lane] = (sx ? Gd.hi[0] : Gd.lo[0]) - gx;
    L.vy[lane] = (sy ? Gd.hi[1] : Gd.lo[1]) - gy;
    L.vz[lane] = (sz ? Gd.hi[2] : Gd.lo[2]) - gz;
  }
  int nP = 6, nT = 8;
  vsync();
  double r2 = vrebuild(L, nT, lane);
  bool ok = true;
  const int hx = gcell(gx, Gd.lo[0], Gd.cs[0], Gd.G[0]);
  const int hy = gcell(gy, Gd.lo[1], Gd.cs[1], Gd.G[1]);
  const int hz = gcell(gz, Gd.lo[2], Gd.cs[2], Gd.G[2]);
  const double csmin = fmin(Gd.cs[0], fmin(Gd.cs[1], Gd.cs[2]));
  const int gmax = max(Gd.G[0], max(Gd.G[1], Gd.G[2]));
  // Candidates are gathered 64 grid cells at a time (one per lane) into an
  // LDS list of sorted-array positions; rings 0 and 1 form the first group,
  // so the nearest sites cut first.
  for (int level = 0; ok; ++level) {
    const int r = level == 0 ? 1 : level + 1;
    if (level >= 1 && r > gmax - 1) break;
    if (level >= 1 && (r - 1) * csmin > 2.0 * sqrt(r2) + eps) break;
    const int side = 2 * r + 1, ncube = side * side * side;
    for (int q0 = 0; ok && q0 < ncube; q0 += 64) {
      const int q = q0 + lane;
      int cnt = 0, s0 = 0;
      if (q < ncube) {
        const int cx = q % side - r, cy = (q / side) % side - r, cz = q / (side * side) - r;
        const bool shell = level == 0 || max(abs(cx), max(abs(cy), abs(cz))) == r;
        const int ix = hx + cx, iy = hy + cy, iz = hz + cz;
        if (shell && ix >= 0 && iy >= 0 && iz >= 0 && ix < Gd.G[0] && iy < Gd.G[1] && iz < Gd.G[2]) {
          // nearest point of the grid cell: nothing there can cut beyond 2R
          const double bx = fmax(fmax(Gd.lo[0] + ix * Gd.cs[0] - gx, gx - (Gd.lo[0] + (ix + 1) * Gd.cs[0])), 0.0);
          const double by = fmax(fmax(Gd.lo[1] + iy * Gd.cs[1] - gy, gy - (Gd.lo[1] + (iy + 1) * Gd.cs[1])), 0.0);
          const double bz = fmax(fmax(Gd.lo[2] + iz * Gd.cs[2] - gz, gz - (Gd.lo[2] + (iz + 1) * Gd.cs[2])), 0.0);
          if (sqrt(bx * bx + by * by + bz * bz) <= 2.0 * sqrt(r2) + eps) {
            const int64_t cell = ((int64_t)iz * Gd.G[1] + iy) * Gd.G[0] + ix;
            s0 = Gd.start[cell];
            cnt = Gd.end[cell] - s0;
          }
        }
      }
      if (!ballot64(cnt > 0)) continue;
      ok = vgroup(L, Gd, c, gx, gy, gz, s0, cnt, level == 0, nP, nT, r2, eps, lane, err);
    }
  }
  if (!ok) return;

  if (kMode == 0) {
    // volume and centroid: over every directed cell edge on face x, the
    // tetrahedron (g, foot of g on x, edge start, edge end)
    double V = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = lane + 64 * h;
      if (t < nT) {
        const int a = L.tri[t][0], b = L.tri[t][1], cc = L.tri[t][2];
        const double px = L.vx[t], py = L.vy[t], pz = L.vz[t];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const int x = r == 0 ? a : (r == 1 ? b : cc);
          const int z = r == 0 ? cc : (r == 1 ? a : b);
          const int t2 = L.T[x][z] & (kVT - 1);
          const double qd = L.pn[x][3];
          const double fx = qd * L.pn[x][0], fy = qd * L.pn[x][1], fz = qd * L.pn[x][2];
          const double ux = L.vx[t2], uy = L.vy[t2], uz = L.vz[t2];
          const double cx = py * uz - pz * uy, cy = pz * ux - px * uz, cz = px * uy - py * ux;
          const double vol = (fx * cx + fy * cy + fz * cz) / 6.0;
          V += vol;
          Sx += vol * (fx + px + ux) / 4.0;
          Sy += vol * (fy + py + uy) / 4.0;
          Sz += vol * (fz + pz + uz) / 4.0;
        }
      }
    }
    V = vsumd(V);
    Sx = vsumd(Sx);
    Sy = vsumd(Sy);
    Sz = vsumd(Sz);
    if (lane == 0) {
      centroid[3 * c] = gx + Sx / V;
      centroid[3 * c + 1] = gy + Sy / V;
      centroid[3 * c + 2] = gz + Sz / V;
      if (volume) volume[c] = V;
    }
    return;
  }

  // faces: one lane per plane; a plane is a face when a current vertex lies on it
  bool present = false;
  int len = 0;
  if (lane < nP) {
    const int t0 = L.first[lane] & (kVT - 1);
    if (t0 < nT && (L.tri[t0][0] == lane || L.tri[t0][1] == lane || L.tri[t0][2] == lane)) {
      present = true;
      int t = t0;
      do {
        const int a = L.tri[t][0], b = L.tri[t][1], cc = L.tri[t][2];
        const int nxt = a == lane ? cc : (b == lane ? a : b);  // the vertex after `lane` in (a, b, c)
        t = L.T[lane][nxt] & (kVT - 1);
        ++len;
      } while (t != t0 && len <= kVT);
    }
  }
  if (ballot64(len > kVT)) {
    if (lane == 0) atomicOr(err, kErrCycle);
    return;
  }
  const int nf = __popcll(ballot64(present));
  const int fv = vsum(len);
  if (kMode == 1) {
    if (lane == 0) {
      cnt[3 * c] = nf;
      cnt[3 * c + 1] = fv;
      cnt[3 * c + 2] = nT;
    }
    return;
  }
  const int64_t f0 = off[3 * c], p0 = off[3 * c + 1], v0 = off[3 * c + 2];
  const int fi = vscan_excl(present ? 1 : 0, lane);
  const int pi = vscan_excl(len, lane);
  if (lane == 0) cell_face_off[c] = f0;
  if (present) {
    face_vtx_off[f0 + fi] = p0 + pi;
    face_nbr[f0 + fi] = L.pid[lane];
    const int t0 = L.first[lane] & (kVT - 1);
    int t = t0, k = 0;
    do {
      face_vtx[p0 + pi + k] = (int32_t)(v0 + t);
      const int a = L.tri[t][0], b = L.tri[t][1], cc = L.tri[t][2];
      const int nxt = a == lane ? cc : (b == lane ? a : b);
      t = L.T[lane][nxt] & (kVT - 1);
      ++k;
    } while (t != t0 && k < len);
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = lane + 64 * h;
    if (t < nT) {
      vert[3 * (v0 + t)] = gx + L.vx[t];
      vert[3 * (v0 + t) + 1] = gy + L.vy[t];
      vert[3 * (v0 + t) + 2] = gz + L.vz[t];
    }
  }
}

__global__ void k_vor_keys(int64_t n, const double *g, VorGrid Gd, uint32_t *key, int32_t *idx, int *err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = g[3 * i], y = g[3 * i + 1], z = g[3 * i + 2];
  const bool in = x >= Gd.lo[0] && x <= Gd.hi[0] && y >= Gd.lo[1] && y <= Gd.hi[1] && z >= Gd.lo[2] && z <= Gd.hi[2];
  if (!in) atomicOr(err, kErrOutside);
  const int ix = gcell(x, Gd.lo[0], Gd.cs[0], Gd.G[0]);
  const int iy = gcell(y, Gd.lo[1], Gd.cs[1], Gd.G[1]);
  const int iz = gcell(z, Gd.lo[2], Gd.cs[2], Gd.G[2]);
  key[i] = (uint32_t)(((int64_t)iz * Gd.G[1] + iy) * Gd.G[0] + ix);
  idx[i] = (int32_t)i;
}

__global__ void k_vor_bounds(int64_t n, const uint32_t *key, int32_t *start, int32_t *end) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t c = key[k];
  if (k == 0 || key[k - 1] != c) start[c] = (int32_t)k;
  if (k == n - 1 || key[k + 1] != c) end[c] = (int32_t)(k + 1);
}

__global__ void k_vor_zero(int64_t m, int32_t *a, int32_t *b) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) {
    a[k] = 0;
    b[k] = 0;
  }
}

__global__ void k_vor_offsets(int64_t n, const int64_t *cnt, const int64_t *scan_f, const int64_t *scan_p,
                              const int64_t *scan_v, int64_t *off) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  off[3 * c] = scan_f[c];
  off[3 * c + 1] = scan_p[c];
  off[3 * c + 2] = scan_v[c];
}

__global__ void k_vor_set(int64_t *a, int64_t va, int64_t *b, int64_t vb) {
  if (threadIdx.x == 0) {
    *a = va;
    *b = vb;
  }
}

__global__ void k_vor_split(int64_t n, const int64_t *cnt, int64_t *f, int64_t *p, int64_t *v) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  f[c] = cnt[3 * c];
  p[c] = cnt[3 * c + 1];
  v[c] = cnt[3 * c + 2];
}

void vor_check(Ctx &ctx, int *err, hipStream_t s) {
  int e = 0;
  SPH_HIP(hipMemcpyAsync(&e, err, sizeof(int), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  SPH_REQUIRE(!(e & kErrOutside), SPHMAP_EINVAL, "a generator lies outside the box");
  SPH_REQUIRE(!(e & kErrCoincident), SPHMAP_EINVAL, "two generators coincide");
  SPH_REQUIRE(!(e & kErrPlanes), SPHMAP_EGEOM, "a Voronoi cell has more than 58 neighbours");
  SPH_REQUIRE(!(e & kErrVertices), SPHMAP_EGEOM, "a Voronoi cell has more than 128 vertices");
  SPH_REQUIRE(!(e & kErrCycle), SPHMAP_EGEOM, "a Voronoi face did not close");
}

// the neighbour grid of the current generators
VorGrid vor_grid(Ctx &ctx, const double *g, int64_t n, const double lo[3], const double hi[3], int *err,
                 hipStream_t s) {
  Arena &ar = ctx.arena;
  VorGrid Gd;
  double vol = 1.0;
  for (int a = 0; a < 3; ++a) {
    Gd.lo[a] = lo[a];
    Gd.hi[a] = hi[a];
    vol *= hi[a] - lo[a];
  }
  const double cs = cbrt(vol * 2.0 / (double)n);
  int64_t cells = 1;
  for (int a = 0; a < 3; ++a) {
    Gd.G[a] = (int)std::min<double>(1024.0, std::max(1.0, ceil((hi[a] - lo[a]) / cs)));
    Gd.cs[a] = (hi[a] - lo[a]) / Gd.G[a];
    cells *= Gd.G[a];
  }
  uint32_t *key = ar.get<uint32_t>("vo_key", n);
  int32_t *idx = ar.get<int32_t>("vo_idx", n);
  k_vor_keys<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, g, Gd, key, idx, err);
  SPH_LAUNCH_CHECK();
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) < cells) ++bits;
  radix_sort_u32(ar, key, idx, n, bits, s);
  int32_t *st = ar.get<int32_t>("vo_start", cells);
  int32_t *en = ar.get<int32_t>("vo_end", cells);
  k_vor_zero<<<(unsigned)div_up(cells, 256), 256, 0, s>>>(cells, st, en);
  SPH_LAUNCH_CHECK();
  k_vor_bounds<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, key, st, en);
  SPH_LAUNCH_CHECK();
  Gd.start = st;
  Gd.end = en;
  Gd.sorted = idx;
  Gd.gen = g;
  return Gd;
}

}  // namespace

void voronoi_build(Ctx &ctx, TessDev &t, int64_t n, const double *d_gen, const double lo[3], const double hi[3],
                   int n_lloyd, double *d_gen_out, hipStream_t s) {
  Arena &ar = ctx.arena;
  int *err = ar.get<int>("vo_err", 1);
  SPH_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
  double L = 0.0;
  for (int a = 0; a < 3; ++a) L = std::max(L, hi[a] - lo[a]);
  const double eps = 1e-13 * L;
  double *ga = ar.get<double>("vo_ga", 3 * n);
  double *gb = ar.get<double>("vo_gb", 3 * n);
  SPH_HIP(hipMemcpyAsync(ga, d_gen, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  const unsigned blocks = (unsigned)div_up(n, kVWaves);
  for (int it = 0; it < n_lloyd; ++it) {
    VorGrid Gd = vor_grid(ctx, ga, n, lo, hi, err, s);
    KernelTimer kt(&ctx, "voronoi_lloyd", s);
    k_voronoi<0><<<blocks, 64 * kVWaves, 0, s>>>(Gd, n, eps, gb, nullptr, nullptr, nullptr, nullptr, nullptr,
                                                  nullptr, nullptr, nullptr, err);
    SPH_LAUNCH_CHECK();
    kt.done();
    vor_check(ctx, err, s);
    std::swap(ga, gb);
  }
  VorGrid Gd = vor_grid(ctx, ga, n, lo, hi, err, s);
  int64_t *cnt = ar.get<int64_t>("vo_cnt", 3 * n);
  {
    KernelTimer kt(&ctx, "voronoi_count", s);
    k_voronoi<1><<<blocks, 64 * kVWaves, 0, s>>>(Gd, n, eps, nullptr, nullptr, cnt, nullptr, nullptr, nullptr,
                                                  nullptr, nullptr, nullptr, err);
    SPH_LAUNCH_CHECK();
    kt.done();
  }
  vor_check(ctx, err, s);
  int64_t *cf = ar.get<int64_t>("vo_cf", n + 1), *cp = ar.get<int64_t>("vo_cp", n + 1),
          *cv = ar.get<int64_t>("vo_cv", n + 1);
  int64_t *sf = ar.get<int64_t>("vo_sf", n + 1), *sp = ar.get<int64_t>("vo_sp", n + 1),
          *sv = ar.get<int64_t>("vo_sv", n + 1);
  k_vor_split<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, cnt, cf, cp, cv);
  SPH_LAUNCH_CHECK();
  scan_exclusive_i64(ar, cf, sf, n, true, s);
  scan_exclusive_i64(ar, cp, sp, n, true, s);
  scan_exclusive_i64(ar, cv, sv, n, true, s);
  int64_t tot[3];
  SPH_HIP(hipMemcpyAsync(&tot[0], sf + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipMemcpyAsync(&tot[1], sp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipMemcpyAsync(&tot[2], sv + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  const int64_t F = tot[0], FV = tot[1], V = tot[2];
  SPH_REQUIRE(F < ((int64_t)1 << 31) && FV < ((int64_t)1 << 31) && V < ((int64_t)1 << 31), SPHMAP_EINVAL,
              "grid too large");
  int64_t *off = ar.get<int64_t>("vo_off", 3 * n);
  k_vor_offsets<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, cnt, sf, sp, sv, off);
  SPH_LAUNCH_CHECK();
  t.n_cells = n;
  t.n_faces = F;
  t.n_vertices = V;
  t.n_fv = FV;
  t.device = ctx.device;
  double size = 0.0;
  for (int a = 0; a < 3; ++a) {
    t.box_lo[a] = lo[a];
    size = std::max(size, hi[a] - lo[a]);
  }
  t.box_size = size * (1.0 + 1e-12);
  t.gen = t.mem.get<double>("gen", 3 * n);
  t.vert = t.mem.get<double>("vert", 3 * std::max<int64_t>(V, 1));
  t.cell_face_off = t.mem.get<int64_t>("cfo", n + 1);
  t.face_vtx_off = t.mem.get<int64_t>("fvo", F + 1);
  t.face_vtx = t.mem.get<int32_t>("fv", std::max<int64_t>(FV, 1));
  t.face_nbr = t.mem.get<int32_t>("fnbr", std::max<int64_t>(F, 1));
  {
    KernelTimer kt(&ctx, "voronoi_faces", s);
    k_voronoi<2><<<blocks, 64 * kVWaves, 0, s>>>(Gd, n, eps, nullptr, nullptr, nullptr, off, t.vert, t.cell_face_off,
                                                  t.face_vtx_off, t.face_vtx, t.face_nbr, err);
    SPH_LAUNCH_CHECK();
    kt.done();
  }
  k_vor_set<<<1, 64, 0, s>>>(t.cell_face_off + n, F, t.face_vtx_off + F, FV);
  SPH_LAUNCH_CHECK();
  SPH_HIP(hipMemcpyAsync(t.gen, ga, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (d_gen_out) SPH_HIP(hipMemcpyAsync(d_gen_out, ga, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  vor_check(ctx, err, s);
  tess_prepare(ctx, t, s);
}

}  // namespace sphmap
