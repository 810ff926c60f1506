// Tree-node pseudo-particles (Sec. 2.4).
//
// The gravity tree here is an octree of the unit cube built from 63-bit
// Morton keys: a node at level l is a run of particles sharing the top 3l key
// bits, a node with more than leaf_max particles (and below max_depth) splits
// into the runs of its next 3-bit digit (child order = octant order x = 1,
// y = 2, z = 4).  Node position is the centre of mass and node size the
// distance from it to the furthest member (Sec. 2.2.1).  So that a host
// reference reproduces the accepted set bit for bit, node sums are formed in a
// fixed order without contraction: a leaf adds its members in ascending
// particle index, an internal node adds its children's sums in octant order.
//
// Walk (Sec. 2.2.2, Sec. 2.4.1): a node is emitted when it is accepted and no
// ancestor is; a leaf that is not accepted and has no accepted ancestor is
// opened and its particles are emitted as themselves (they keep their h).
// Acceptance: for every source, r - s > r_part and not (theta^2 r^2 < s^2)
// (eq. opening_angle).  Each emitted node or opened leaf is one "unit"; the
// units tile the particle order, so depth-first emission order is the order
// of their first particle.
//
// Node smoothing lengths (Sec. 2.4.2, eqs. h_node, n_node, hnode_func,
// hnode_func_deriv, hnode_newton_raphson, hnode_estval): n(h) sums
// W(|r_a - r_b|, h) over all units b (opened leaves stand in for their
// particles; self term included).  Newton from h0 = h_fact 2 s to
// |h_new - h| / h0 < eps_h; Newton fails after 30 steps, when an iterate
// leaves [1e-2 h0, 1e2 h0] or when |f'| < 1e-12; then bisection on
// [1e-2 h0, 1e2 h0] when f changes sign there, else h0.  Newton's sums over
// units run in unit order, one wavefront per pseudo-particle; the nodes it
// leaves go to a second kernel, 16 wavefronts per node, whose bracket and
// bisection steps decide from fixed-order tree sums (falling back to the
// unit-order sums within their rounding margin), so every decision is that
// of the unit-order sums.
#include "common.hpp"

namespace sphmap {
namespace {

constexpr int kMaxLevels = 22;

struct NodeArrays {
  int32_t *first, *count, *parent, *child_first, *nchild, *level;
};

__global__ void k_check_unit_cube(int64_t n, const double *xyz, int *bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) {
    double x = xyz[3 * i + k];
    if (!(x >= 0.0 && x < 1.0)) {
      atomicAdd(bad, 1);
      return;
    }
  }
}

__global__ void k_root(NodeArrays N, int64_t n) {
  N.first[0] = 0;
  N.count[0] = (int32_t)n;
  N.parent[0] = -1;
  N.level[0] = 0;
  N.child_first[0] = -1;
  N.nchild[0] = 0;
}

__device__ inline int digit_of(uint64_t key, int level) {
  // digit selecting the child at `level` (1 = first split below the root)
  return (int)((key >> (3 * (21 - level))) & 7ull);
}

// For each node of the level [b, e): the non-empty child runs.
__global__ void k_split(NodeArrays N, int64_t b, int64_t e, int level, const uint64_t *keys, int leaf_max,
                        int max_depth, int32_t *tfirst, int32_t *tcount, int64_t *nch) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= e - b) return;
  const int64_t node = b + j;
  const int32_t f = N.first[node], c = N.count[node];
  int k = 0;
  if (c > leaf_max && level < max_depth) {
    int32_t lo = f;
    const int32_t end = f + c;
    for (int d = 0; d < 8; ++d) {
      // first position in [lo, end) whose digit exceeds d
      int32_t a = lo, z = end;
      while (a < z) {
        int32_t mid = a + (z - a) / 2;
        if (digit_of(keys[mid], level + 1) <= d) a = mid + 1;
        else z = mid;
      }
      if (a > lo) {
        tfirst[8 * j + k] = lo;
        tcount[8 * j + k] = a - lo;
        ++k;
      }
      lo = a;
    }
  }
  nch[j] = k;
}

__global__ void k_children(NodeArrays N, int64_t b, int64_t e, int level, int64_t next_off, const int32_t *tfirst,
                           const int32_t *tcount, const int64_t *nch, const int64_t *choff) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= e - b) return;
  const int64_t node = b + j;
  const int k = (int)nch[j];
  N.nchild[node] = k;
  N.child_first[node] = k ? (int32_t)(next_off + choff[j]) : -1;
  for (int q = 0; q < k; ++q) {
    const int64_t cid = next_off + choff[j] + q;
    N.first[cid] = tfirst[8 * j + q];
    N.count[cid] = tcount[8 * j + q];
    N.parent[cid] = (int32_t)node;
    N.level[cid] = level + 1;
    N.child_first[cid] = -1;
    N.nchild[cid] = 0;
  }
}

// Leaves: sums over members in ascending particle index.  A leaf whose
// members already lie in ascending index (every leaf at the depth limit:
// its members share the whole key, and the key sort is stable) is summed in
// one pass and marked in asc; any other (at most leaf_max members) takes
// them in order by selection.
__global__ void k_leaf_moments(NodeArrays N, int64_t nn, const int32_t *sidx, const double *xyz, const double *m,
                               double *M, double4 *S, int8_t *asc) {
#pragma clang fp contract(off)
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nn || N.nchild[node] != 0) return;
  const int32_t f = N.first[node], c = N.count[node];
  bool up = true;
  for (int32_t u = f + 1; u < f + c && up; ++u) up = sidx[u] > sidx[u - 1];
  asc[node] = up ? 1 : 0;
  double sm = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
  int32_t prev = -1;
  for (int32_t t = 0; t < c; ++t) {
    int32_t best = INT32_MAX;
    if (up) {
      best = sidx[f + t];
    } else {
      for (int32_t u = f; u < f + c; ++u) {
        int32_t j = sidx[u];
        if (j > prev && j < best) best = j;
      }
    }
    prev = best;
    const double mj = m[best];
    sm += mj;
    sx += mj * xyz[3 * (int64_t)best];
    sy += mj * xyz[3 * (int64_t)best + 1];
    sz += mj * xyz[3 * (int64_t)best + 2];
  }
  M[node] = sm;
  S[node] = make_double4(sx, sy, sz, 0.0);
}

// Internal nodes of one level: children's sums in octant order.
__global__ void k_internal_moments(NodeArrays N, int64_t b, int64_t e, double *M, double4 *S) {
#pragma clang fp contract(off)
  int64_t node = b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= e) return;
  const int k = N.nchild[node];
  if (k == 0) return;
  const int32_t c0 = N.child_first[node];
  double sm = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
  for (int q = 0; q < k; ++q) {
    sm += M[c0 + q];
    double4 s = S[c0 + q];
    sx += s.x;
    sy += s.y;
    sz += s.z;
  }
  M[node] = sm;
  S[node] = make_double4(sx, sy, sz, 0.0);
}

__global__ void k_com(int64_t nn, const double *M, const double4 *S, double4 *com) {
#pragma clang fp contract(off)
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nn) return;
  const double mm = M[node];
  const double4 s = S[node];
  com[node] = make_double4(s.x / mm, s.y / mm, s.z / mm, 0.0);
}

constexpr int kBigNode = 4096;  // members above which a node's size takes a whole workgroup

// One wave per node of at most kBigNode members: max squared member
// distance from the centre of mass and the lowest member particle index.
// positions in the sorted order of sidx, so that the node-size kernels read
// each node's particles contiguously instead of gathering them
__global__ void k_sorted_xyz(int64_t n, const int32_t *sidx, const double *xyz, double4 *sx) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t j = sidx[t];
  sx[t] = make_double4(xyz[3 * j], xyz[3 * j + 1], xyz[3 * j + 2], 0.0);
}

__global__ void __launch_bounds__(256) k_node_size(NodeArrays N, int64_t nn, const int32_t *sidx, const double4 *sx,
                                                  const double4 *com, double *s2, int32_t *minidx) {
#pragma clang fp contract(off)
  const int64_t node = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (node >= nn) return;
  const int32_t f = N.first[node], c = N.count[node];
  if (c > kBigNode) {  // k_node_size_big combines its chunks into these
    if (lane == 0) {
      s2[node] = 0.0;
      minidx[node] = INT32_MAX;
    }
    return;
  }
  const double4 g = com[node];
  double mx = 0.0;
  int32_t mi = INT32_MAX;
  for (int32_t t = f + lane; t < f + c; t += 64) {
    const int32_t j = sidx[t];
    const double4 p = sx[t];
    const double dx = p.x - g.x, dy = p.y - g.y, dz = p.z - g.z;
    const double s = (dx * dx + dy * dy) + dz * dz;
    mx = fmax(mx, s);
    mi = min(mi, j);
  }
  for (int o = 32; o > 0; o >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, o, 64));
    mi = min(mi, __shfl_xor(mi, o, 64));
  }
  if (lane == 0) {
    s2[node] = mx;
    minidx[node] = mi;
  }
}

// Chunks of kBigNode members: none for a node handled by k_node_size.
__global__ void k_flag_big(NodeArrays N, int64_t nn, int64_t *flag) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node < nn) {
    const int32_t c = N.count[node];
    flag[node] = c > kBigNode ? (c + kBigNode - 1) / kBigNode : 0;
  }
}

// The node of every chunk (off: each node's first chunk).
__global__ void k_list_big(NodeArrays N, int64_t nn, const int64_t *off, int32_t *list) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node < nn && N.count[node] > kBigNode)
    for (int64_t q = off[node]; q < off[node + 1]; ++q) list[q] = (int32_t)node;
}

// The same for the nodes above kBigNode members, one workgroup per chunk of
// kBigNode members (grid-stride over the device-side chunk list); the
// chunks combine by atomic maximum (non-negative binary64 values order as
// their bit patterns) and minimum, which do not depend on the order in
// which they finish.
__global__ void __launch_bounds__(1024) k_node_size_big(NodeArrays N, const int32_t *list, const int64_t *off,
                                                       const int64_t *n_list, const int32_t *sidx, const double4 *sx,
                                                       const double4 *com, double *s2, int32_t *minidx) {
#pragma clang fp contract(off)
  __shared__ double smx[16];
  __shared__ int32_t smi[16];
  const int64_t nb = *n_list;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const int32_t node = list[b];
    const int32_t k = (int32_t)(b - off[node]);  // the chunk within the node
    const int32_t f0 = N.first[node], c = N.count[node];
    const int32_t f = f0 + k * kBigNode, fe = min(f0 + c, f + kBigNode);
    const double4 g = com[node];
    double mx = 0.0;
    int32_t mi = INT32_MAX;
    for (int32_t t = f + (int32_t)threadIdx.x; t < fe; t += (int32_t)blockDim.x) {
      const int32_t j = sidx[t];
      const double4 p = sx[t];
      const double dx = p.x - g.x, dy = p.y - g.y, dz = p.z - g.z;
      const double s = (dx * dx + dy * dy) + dz * dz;
      mx = fmax(mx, s);
      mi = min(mi, j);
    }
    for (int o = 32; o > 0; o >>= 1) {
      mx = fmax(mx, __shfl_xor(mx, o, 64));
      mi = min(mi, __shfl_xor(mi, o, 64));
    }
    if (lane == 0) {
      smx[wid] = mx;
      smi[wid] = mi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
        mx = fmax(mx, smx[w]);
        mi = min(mi, smi[w]);
      }
      atomicMax((unsigned long long *)&s2[node], (unsigned long long)__double_as_longlong(mx));
      atomicMin(&minidx[node], mi);
    }
    __syncthreads();
  }
}

// Node label: a 1 followed by the octant digits from the root down (3 bits
// per level), read off the Morton key of the node's first member.
__global__ void k_label(NodeArrays N, int64_t nn, const uint64_t *keys, uint64_t *label) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nn) return;
  const int l = N.level[node];
  const uint64_t key = keys[N.first[node]];
  label[node] = (1ull << (3 * l)) | (l == 0 ? 0ull : key >> (3 * (21 - l)));
}

// Nodes whose labels are in the sorted list are opened (Sec. 2.4.1: the
// nodes that failed the resolution check).
__global__ void k_force_open(int64_t nn, const uint64_t *label, int64_t n_open, const uint64_t *open, int8_t *acc) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nn || !acc[node]) return;
  const uint64_t l = label[node];
  int64_t lo = 0, hi = n_open;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (open[mid] < l) lo = mid + 1;
    else hi = mid;
  }
  if (lo < n_open && open[lo] == l) acc[node] = 0;
}

__global__ void k_accept(int64_t nn, const double4 *com, const double *s2, int n_src, const double *src, double r_part,
                         double theta, int8_t *acc) {
#pragma clang fp contract(off)
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nn) return;
  const double4 g = com[node];
  const double ss = s2[node];
  const double s = sqrt(ss);
  int8_t ok = 1;
  for (int k = 0; k < n_src && ok; ++k) {
    const double dx = g.x - src[3 * k], dy = g.y - src[3 * k + 1], dz = g.z - src[3 * k + 2];
    const double r2 = (dx * dx + dy * dy) + dz * dz;
    const double r = sqrt(r2);
    if (!(r - s > r_part)) ok = 0;
    else if ((theta * theta) * r2 < ss) ok = 0;
  }
  acc[node] = ok;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Emitted units: accepted without an accepted ancestor, or an opened leaf.
__global__ void k_units(NodeArrays N, int64_t nn, const int8_t *acc, int32_t *unit_at) {
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nn) return;
  for (int32_t p = N.parent[node]; p >= 0; p = N.parent[p])
    if (acc[p]) return;
  if (acc[node] || N.nchild[node] == 0) unit_at[N.first[node]] = (int32_t)node;
}

__global__ void k_flag(int64_t n, const int32_t *unit_at, int64_t *flag) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) flag[t] = unit_at[t] >= 0 ? 1 : 0;
}

__global__ void k_unit_list(int64_t n, const int32_t *unit_at, const int64_t *uoff, int32_t *units) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && unit_at[t] >= 0) units[uoff[t]] = unit_at[t];
}

__global__ void k_unit_counts(int64_t nu, const int32_t *units, NodeArrays N, const int8_t *acc, int64_t *ecnt,
                              int64_t *pcnt) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nu) return;
  const int32_t node = units[u];
  const bool a = acc[node] != 0;
  ecnt[u] = a ? 1 : N.count[node];
  pcnt[u] = (a && N.count[node] > 1) ? 1 : 0;
}

__global__ void k_entries(int64_t nu, const int32_t *units, NodeArrays N, const int8_t *acc, const int64_t *eoff,
                          const int64_t *poff, const int32_t *sidx, const double *xyz, const double *hh,
                          const double *m, const double *M, const double4 *com, const double *s2,
                          const int32_t *minidx, double *o_xyz, double *o_h, double *o_m, double *o_s,
                          int32_t *o_kind, int64_t *o_first, int64_t *o_count, int32_t *o_branch, double4 *upos,
                          int32_t *plist, const uint64_t *label, uint64_t *o_label, const int8_t *asc) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nu) return;
  const int32_t node = units[u];
  const int32_t f = N.first[node], c = N.count[node];
  const double4 g = com[node];
  upos[u] = g;
  int64_t e = eoff[u];
  auto emit_real = [&](int32_t j) {
    o_xyz[3 * e] = xyz[3 * (int64_t)j];
    o_xyz[3 * e + 1] = xyz[3 * (int64_t)j + 1];
    o_xyz[3 * e + 2] = xyz[3 * (int64_t)j + 2];
    o_h[e] = hh[j];
    o_m[e] = m[j];
    if (o_s) o_s[e] = 0.0;
    if (o_kind) o_kind[e] = 0;
    if (o_first) o_first[e] = j;
    if (o_count) o_count[e] = 1;
    if (o_branch) o_branch[e] = -1;
    if (o_label) o_label[e] = label[node];
    ++e;
  };
  if (acc[node]) {
    if (c == 1) {
      emit_real(sidx[f]);
    } else {
      o_xyz[3 * e] = g.x;
      o_xyz[3 * e + 1] = g.y;
      o_xyz[3 * e + 2] = g.z;
      o_h[e] = 0.0;
      o_m[e] = M[node];
      if (o_s) o_s[e] = sqrt(s2[node]);
      if (o_kind) o_kind[e] = 1;
      if (o_first) o_first[e] = minidx[node];
      if (o_count) o_count[e] = c;
      if (o_branch) o_branch[e] = 0;
      if (o_label) o_label[e] = label[node];
      plist[poff[u]] = (int32_t)e;
    }
  } else {
    // opened leaf: its particles in ascending index
    int32_t prev = -1;
    for (int32_t t = 0; t < c; ++t) {
      int32_t best = INT32_MAX;
      if (asc[node]) {
        best = sidx[f + t];
      } else {
        for (int32_t q = f; q < f + c; ++q) {
          int32_t j = sidx[q];
          if (j > prev && j < best) best = j;
        }
      }
      prev = best;
      emit_real(best);
    }
  }
}

// Entry that holds each particle: the sorted position's unit is the last unit
// starting at or before it; an opened leaf's particles are its entries in
// ascending index, so a particle's entry is offset by its rank among them.
__global__ void k_owner(int64_t n, const int64_t *flag, const int64_t *uoff, const int32_t *units, NodeArrays N,
                        const int8_t *acc, const int64_t *eoff, const int32_t *sidx, const int8_t *asc,
                        int64_t *owner) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int64_t u = uoff[q] + flag[q] - 1;
  const int32_t node = units[u];
  const int32_t j = sidx[q];
  int64_t e = eoff[u];
  if (!acc[node]) {
    const int32_t f = N.first[node], c = N.count[node];
    if (asc[node]) e += q - f;  // members in ascending index: the rank is the position
    else
      for (int32_t t = f; t < f + c; ++t) e += sidx[t] < j;
  }
  owner[j] = e;
}

constexpr double kInvPi = 0.31830988618379067154;

__device__ inline double m4w(double q) {
#pragma clang fp contract(off)
  if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
  if (q < 2.0) return 0.25 * (2.0 - q) * (2.0 - q) * (2.0 - q);
  return 0.0;
}
__device__ inline double m4dw(double q) {
#pragma clang fp contract(off)
  if (q < 1.0) return -3.0 * q + 2.25 * q * q;
  if (q < 2.0) return -0.75 * (2.0 - q) * (2.0 - q);
  return 0.0;
}

__device__ inline double readlane_d(double v, int j) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, j);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), j);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// What the node h-solve sums over: the units (their positions and the
// boxes of their tiles of 64 and of their blocks of 64 tiles) and, with
// n_mid > 0, the trial-neighbour ranges.
struct HUnits {
  int64_t nu;
  const double4 *upos;
  const double4 *tlo, *thi;  // tile t: units [64 t, 64 t + 64)
  const double4 *blo, *bhi;  // block b: tiles [64 b, 64 b + 64)
  int64_t n_mid;
  const double4 *mid_com;
  const int32_t *mid_u0, *mid_u1;
  const double *rcut;
};

// The sums of one h-solve step at node position (ax, ay, az) and length he,
// over every unit within 2 he, by one wavefront.
//
// Unit order (fast == false): the 64 lanes evaluate 64 consecutive units at
// a time, the tile's non-zero terms go to LDS (hb, 64 entries) in lane order
// and lanes 0 and 1 add them one after the other (lane 0 the w terms, lane 1
// the dt terms), so sw and sd, returned to every lane, are the sums of a
// plain sequential loop over the units.
//
// Tree order (fast == true): sw only, and only this wave's share, the tiles
// t with t % step == first: each tile's terms are added by a butterfly and
// the tiles in order; every lane holds the share, and nhit counts its
// non-zero terms.
//
// A block or tile whose bounding box lies beyond 2 he holds only zero terms
// and is skipped.  A block's box holds its tiles' boxes and the distance test
// is monotone in the box bounds, so no tile that passes the test is skipped
// with its block.  Blocks and tiles are visited in ascending order.  With
// n_mid > 0 the sums run over trial neighbours only: the units of the ranges
// [mid_u0, mid_u1) of the nodes whose centres of mass lie within rcut[e] of
// the target; the ranges follow unit order, so unit-order terms are still
// added in unit order.
// kBatch: LDS reads in flight in the unit-order adds.
template <int kBatch>
__device__ __forceinline__ void hsums(const HUnits &U, int32_t e, double ax, double ay, double az, double he,
                                      bool fast, int first, int step, double2 *hb, double &sw, double &sd,
                                      int64_t &nhit) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const double ih = 1.0 / he;
  double acc = 0.0;  // unit order: lane 0's sw, lane 1's sd
  sw = sd = 0.0;
  nhit = 0;
  // the terms of one tile's units (one per lane, `live` lanes hold one)
  auto tile_terms = [&](const double4 &p, bool live) __attribute__((always_inline)) {
    double w = 0.0, dt = 0.0;
    bool hit = false;
    if (live) {
      const double dx = ax - p.x, dy = ay - p.y, dz = az - p.z;
      const double qq = sqrt((dx * dx + dy * dy) + dz * dz) * ih;
      if (qq < 2.0) {
        hit = true;
        w = m4w(qq);
        if (!fast) dt = -(3.0 * w + qq * m4dw(qq));
      }
    }
    const uint64_t mask = __ballot(hit);
    if (fast) {
      nhit += __popcll(mask);
      if (mask) {
        double v = hit ? w : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        sw += readlane_d(v, 0);
      }
      return;
    }
    if (mask) {
      if (hit) hb[__popcll(mask & below)] = make_double2(w, dt);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane < 2) {  // lane 0 adds the w terms, lane 1 the dt terms
        const double *src = reinterpret_cast<const double *>(hb) + lane;
        const int cnt = __popcll(mask);
        int k = 0;
        for (; k + kBatch <= cnt; k += kBatch) {  // kBatch reads in flight, added in order
          double v[kBatch];
#pragma unroll
          for (int u = 0; u < kBatch; ++u) v[u] = src[2 * (k + u)];
#pragma unroll
          for (int u = 0; u < kBatch; ++u) acc += v[u];
        }
        for (; k < cnt; ++k) acc += src[2 * k];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  };
  auto beyond = [&](const double4 &lo, const double4 &hi) __attribute__((always_inline)) {
    const double bx = fmax(fmax(lo.x - ax, ax - hi.x), 0.0);
    const double by = fmax(fmax(lo.y - ay, ay - hi.y), 0.0);
    const double bz = fmax(fmax(lo.z - az, az - hi.z), 0.0);
    return !(((bx * bx + by * by) + bz * bz) * ih * ih < 4.0 * (1.0 + 1e-9));
  };
  // units [u0, u1), tiles t with t % step == first
  auto tile_sums = [&](int64_t u0, int64_t u1) __attribute__((always_inline)) {
    const int64_t t0 = u0 >> 6, t1 = (u1 + 63) >> 6;
    const int64_t b0 = t0 >> 6, b1 = (t1 + 63) >> 6;
    for (int64_t bb = b0; bb < b1; bb += 64) {
      const int64_t bi = bb + lane;
      bool bnear = false;
      if (bi < b1) bnear = !beyond(U.blo[bi], U.bhi[bi]);
      uint64_t bm = __ballot(bnear);
      while (bm) {
        const int64_t tb = 64 * (bb + __builtin_ctzll(bm));
        bm &= bm - 1;
        const int64_t ti = tb + lane;
        bool near = false;
        if (ti >= t0 && ti < t1 && ti % step == first) near = !beyond(U.tlo[ti], U.thi[ti]);
        uint64_t nm = __ballot(near);
        while (nm) {
          // up to four near tiles at once: their loads are in flight together,
          // and their terms are added tile after tile
          int64_t ua0, ub0, ua1, ub1, ua2, ub2, ua3, ub3;
          double4 p0, p1, p2, p3;
          auto take = [&](int64_t &ua, int64_t &ub, double4 &pv) __attribute__((always_inline)) {
            ua = ub = 0;
            if (nm) {
              const int64_t t = tb + __builtin_ctzll(nm);
              nm &= nm - 1;
              ua = max(u0, 64 * t);
              ub = min(u1, 64 * t + 64);
            }
            if (ua + lane < ub) pv = U.upos[ua + lane];
          };
          take(ua0, ub0, p0);
          take(ua1, ub1, p1);
          take(ua2, ub2, p2);
          take(ua3, ub3, p3);
          if (ub0 > ua0) tile_terms(p0, ua0 + lane < ub0);
          if (ub1 > ua1) tile_terms(p1, ua1 + lane < ub1);
          if (ub2 > ua2) tile_terms(p2, ua2 + lane < ub2);
          if (ub3 > ua3) tile_terms(p3, ua3 + lane < ub3);
        }
      }
    }
  };
  if (U.n_mid == 0) {
    tile_sums(0, U.nu);
  } else {
    const double rc = U.rcut[e];
    for (int64_t m0 = 0; m0 < U.n_mid; m0 += 64) {
      const int64_t mi = m0 + lane;
      bool flag = false;
      if (mi < U.n_mid) {
        const double4 c = U.mid_com[mi];
        const double dx = ax - c.x, dy = ay - c.y, dz = az - c.z;
        flag = sqrt((dx * dx + dy * dy) + dz * dz) < rc;
      }
      uint64_t fm = __ballot(flag);
      while (fm) {
        const int j = __builtin_ctzll(fm);
        fm &= fm - 1;
        tile_sums(U.mid_u0[m0 + j], U.mid_u1[m0 + j]);
      }
    }
  }
  if (!fast) {
    sw = readlane_d(acc, 0);
    sd = readlane_d(acc, 1);
  }
}

// f(he) = hfact n(he)^(-1/3) - he from sw, the sum of the M4 terms at he
__device__ __forceinline__ double h_residual(double sw, double he, double hfact) {
#pragma clang fp contract(off)
  const double ih = 1.0 / he;
  const double n = sw * ih * ih * ih * kInvPi;
  return hfact * pow(n, -1.0 / 3.0) - he;
}

constexpr int kHWaves = 4;    // pseudo-particles per workgroup in the Newton kernel
constexpr int kBWaves = 16;   // wavefronts per pseudo-particle in the bracket kernel

// Node h-solve, first part: up to 30 Newton steps from h0 = 2 hfact s, one
// wavefront per pseudo-particle, with unit-order sums.  A converged node
// writes its h (branch 0); a node whose step fails (a vanishing derivative,
// a step out of [h0/100, 100 h0], or 30 steps) is appended to `fails` for
// the bracket kernel, in whatever order the atomics give (each node's result
// depends on that node alone).  Above `bypass` pseudo-particles every node
// takes h0 (branch 3).
__global__ void __launch_bounds__(64 * kHWaves) k_hsolve_newton(int64_t np, const int32_t *plist, HUnits U,
                                                               const double *o_xyz, const double *o_s, double hfact,
                                                               double eps, int64_t bypass, double *o_h,
                                                               int32_t *o_branch, unsigned long long *bcount,
                                                               int32_t *fails, int32_t *n_fails) {
#pragma clang fp contract(off)
  __shared__ double2 hbuf[kHWaves][64];
  const int64_t pid = (int64_t)blockIdx.x * kHWaves + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (pid >= np) return;  // the whole wavefront
  const int32_t e = plist[pid];
  const double ax = o_xyz[3 * (int64_t)e], ay = o_xyz[3 * (int64_t)e + 1], az = o_xyz[3 * (int64_t)e + 2];
  const double h0 = hfact * 2.0 * o_s[e];
  const double lo = 1e-2 * h0, hi = 1e2 * h0;
  double hres = h0;
  int branch = 3;
  if (np <= bypass) {
    branch = -1;  // failed unless a step converges
    double h = h0;
    for (int it = 0; it < 30; ++it) {
      double sw, sd;
      int64_t nhit;
      hsums<16>(U, e, ax, ay, az, h, false, 0, 1, hbuf[threadIdx.x >> 6], sw, sd, nhit);
      const double ih = 1.0 / h;
      const double n = sw * ih * ih * ih * kInvPi;
      const double dn = sd * ih * ih * ih * ih * kInvPi;
      const double f = hfact * pow(n, -1.0 / 3.0) - h;
      const double fp = -(1.0 / 3.0) * hfact * dn * pow(n, -4.0 / 3.0) - 1.0;
      if (!(fabs(fp) >= 1e-12)) break;
      const double hn = h - f / fp;
      if (!(hn >= lo && hn <= hi)) break;
      if (fabs(hn - h) / h0 < eps) {
        hres = hn;
        branch = 0;
        break;
      }
      h = hn;
    }
  }
  if (lane == 0) {
    if (branch < 0) {
      fails[atomicAdd(n_fails, 1)] = e;
    } else {
      o_h[e] = hres;
      if (o_branch) o_branch[e] = branch;
      atomicAdd(&bcount[branch], 1ull);
    }
  }
}

// Node h-solve, second part: the bracket [h0/100, 100 h0] and bisection to
// a width below eps h0, one workgroup of kBWaves wavefronts per node that
// Newton did not solve.  These steps use only the sign of f (and f == 0), so
// they first take sw in tree order, each wave summing its share and the
// shares added in wave order.  The terms are non-negative, so that sum is
// within 2 nhit 2^-53 sw of the unit-order one, which moves f by less than
// nhit 2^-53 he; only when |f| is within that margin are the sums taken again
// in unit order (by the first wave).  Every decision, and so every result,
// is that of the unit-order sums.
__global__ void __launch_bounds__(64 * kBWaves) k_hsolve_bracket(const int32_t *fails, const int32_t *n_fails,
                                                                HUnits U, const double *o_xyz, const double *o_s,
                                                                double hfact, double eps, double *o_h,
                                                                int32_t *o_branch, unsigned long long *bcount) {
#pragma clang fp contract(off)
  __shared__ double2 hb[64];
  __shared__ double part_sw[kBWaves];
  __shared__ long long part_hit[kBWaves];
  __shared__ double uo_sw;
  if ((int)blockIdx.x >= *n_fails) return;  // the whole workgroup
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int32_t e = fails[blockIdx.x];
  const double ax = o_xyz[3 * (int64_t)e], ay = o_xyz[3 * (int64_t)e + 1], az = o_xyz[3 * (int64_t)e + 2];
  const double h0 = hfact * 2.0 * o_s[e];
  double lo = 1e-2 * h0, hi = 1e2 * h0;
  double flo = 0.0, hres = h0;
  int phase = 1;  // 1 eval lo, 2 eval hi, 3 bisect, 9 done
  int branch = 1;
  while (phase != 9) {
    double he = lo;
    if (phase == 2) he = hi;
    else if (phase == 3) he = 0.5 * (lo + hi);
    double sw, sd;
    int64_t nhit;
    hsums<8>(U, e, ax, ay, az, he, true, wid, kBWaves, hb, sw, sd, nhit);
    if ((threadIdx.x & 63) == 0) {
      part_sw[wid] = sw;
      part_hit[wid] = nhit;
    }
    __syncthreads();
    sw = 0.0;
    nhit = 0;
    for (int k = 0; k < kBWaves; ++k) {  // in wave order
      sw += part_sw[k];
      nhit += part_hit[k];
    }
    double f = h_residual(sw, he, hfact);
    if (!(fabs(f) > he * (1e-12 + 4.0 * (double)nhit * 0x1p-53))) {  // the same in every wave
      if (wid == 0) {
        hsums<8>(U, e, ax, ay, az, he, false, 0, 1, hb, sw, sd, nhit);
        if ((threadIdx.x & 63) == 0) uo_sw = sw;
      }
      __syncthreads();
      f = h_residual(uo_sw, he, hfact);
    }
    __syncthreads();  // every wave has read the shared sums before they are written again
    if (phase == 1) {
      flo = f;
      if (f == 0.0) {
        hres = lo;
        phase = 9;
      } else {
        phase = 2;
      }
    } else if (phase == 2) {
      if (f == 0.0) {
        hres = hi;
        phase = 9;
      } else if ((flo < 0.0) == (f < 0.0)) {
        hres = h0;
        branch = 2;
        phase = 9;
      } else if (!(hi - lo >= eps * h0)) {
        hres = 0.5 * (lo + hi);
        phase = 9;
      } else {
        phase = 3;
      }
    } else {  // bisection step at mid = he
      if (f == 0.0) {
        hres = he;
        phase = 9;
      } else {
        if ((f < 0.0) == (flo < 0.0)) {
          lo = he;
          flo = f;
        } else {
          hi = he;
        }
        if (!(hi - lo >= eps * h0)) {
          hres = 0.5 * (lo + hi);
          phase = 9;
        }
      }
    }
  }
  if (threadIdx.x == 0) {
    o_h[e] = hres;
    if (o_branch) o_branch[e] = branch;
    atomicAdd(&bcount[branch], 1ull);
  }
}

struct Grow {
  Arena &ar;
  int64_t cap = 0;
  NodeArrays N{};
  explicit Grow(Arena &a) : ar(a) {}
  void ensure(int64_t need, int64_t used, hipStream_t s) {
    if (need <= cap) return;
    int64_t nc = std::max<int64_t>(need, cap * 2);
    NodeArrays M;
    const char *names[6] = {"ps_first", "ps_count", "ps_parent", "ps_cfirst", "ps_nchild", "ps_level"};
    int32_t **dst[6] = {&M.first, &M.count, &M.parent, &M.child_first, &M.nchild, &M.level};
    int32_t *src[6] = {N.first, N.count, N.parent, N.child_first, N.nchild, N.level};
    for (int k = 0; k < 6; ++k) {
      std::string nm = std::string(names[k]) + (cap ? "_b" : "_a") + std::to_string(nc);
      *dst[k] = ar.get<int32_t>(nm, nc);
      if (used > 0) SPH_HIP(hipMemcpyAsync(*dst[k], src[k], used * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    N = M;
    cap = nc;
  }
};

}  // namespace

namespace {
__global__ void k_unit_tiles(int64_t nu, const double4 *upos, double4 *tlo, double4 *thi) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t * 64 >= nu) return;
  double4 lo = make_double4(INFINITY, INFINITY, INFINITY, 0.0), hi = make_double4(-INFINITY, -INFINITY, -INFINITY, 0.0);
  for (int64_t u = 64 * t; u < min(nu, 64 * t + 64); ++u) {
    const double4 p = upos[u];
    lo.x = fmin(lo.x, p.x);
    lo.y = fmin(lo.y, p.y);
    lo.z = fmin(lo.z, p.z);
    hi.x = fmax(hi.x, p.x);
    hi.y = fmax(hi.y, p.y);
    hi.z = fmax(hi.z, p.z);
  }
  tlo[t] = lo;
  thi[t] = hi;
}

// the boxes of blocks of 64 tiles, from the tiles' boxes
__global__ void k_unit_blocks(int64_t nt, const double4 *tlo, const double4 *thi, double4 *blo, double4 *bhi) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b * 64 >= nt) return;
  double4 lo = tlo[64 * b], hi = thi[64 * b];
  for (int64_t t = 64 * b + 1; t < min(nt, 64 * b + 64); ++t) {
    const double4 l = tlo[t], u = thi[t];
    lo.x = fmin(lo.x, l.x);
    lo.y = fmin(lo.y, l.y);
    lo.z = fmin(lo.z, l.z);
    hi.x = fmax(hi.x, u.x);
    hi.y = fmax(hi.y, u.y);
    hi.z = fmax(hi.z, u.z);
  }
  blo[b] = lo;
  bhi[b] = hi;
}
}  // namespace

void node_hsolve(Ctx &ctx, int64_t np, const int32_t *plist, int64_t nu, const double4 *upos, const double *o_xyz,
                 const double *o_s, double hfact, double eps, int64_t bypass, double *o_h, int32_t *o_branch,
                 unsigned long long *bcount, int64_t n_mid, const double4 *mid_com, const int32_t *mid_u0,
                 const int32_t *mid_u1, const double *rcut, hipStream_t s) {
  if (np <= 0) return;
  const int64_t nt = div_up(nu, 64);
  double4 *tlo = ctx.arena.get<double4>("hs_tlo", std::max<int64_t>(nt, 1));
  double4 *thi = ctx.arena.get<double4>("hs_thi", std::max<int64_t>(nt, 1));
  const int64_t nb = div_up(nt, 64);
  double4 *blo = ctx.arena.get<double4>("hs_blo", std::max<int64_t>(nb, 1));
  double4 *bhi = ctx.arena.get<double4>("hs_bhi", std::max<int64_t>(nb, 1));
  if (nt > 0) {
    k_unit_tiles<<<(unsigned)div_up(nt, 256), 256, 0, s>>>(nu, upos, tlo, thi);
    SPH_LAUNCH_CHECK();
    k_unit_blocks<<<(unsigned)div_up(nb, 256), 256, 0, s>>>(nt, tlo, thi, blo, bhi);
    SPH_LAUNCH_CHECK();
  }
  int32_t *fails = ctx.arena.get<int32_t>("hs_fails", np);
  int32_t *n_fails = ctx.arena.get<int32_t>("hs_nfails", 1);
  k_fill_i32<<<1, 64, 0, s>>>(n_fails, 0, 1);
  SPH_LAUNCH_CHECK();
  const HUnits U{nu, upos, tlo, thi, blo, bhi, n_mid, mid_com, mid_u0, mid_u1, rcut};
  KernelTimer kt(&ctx, "node_hsolve", s);
  KernelTimer kt1(&ctx, "node_hsolve_newton", s);
  k_hsolve_newton<<<(unsigned)div_up(np, kHWaves), 64 * kHWaves, 0, s>>>(np, plist, U, o_xyz, o_s, hfact, eps, bypass,
                                                                        o_h, o_branch, bcount, fails, n_fails);
  SPH_LAUNCH_CHECK();
  kt1.done();
  // one workgroup per node that Newton did not solve (the rest exit at
  // once); above the bypass every node took h0 and none is left
  if (np <= bypass) {
    KernelTimer kt2(&ctx, "node_hsolve_bracket", s);
    k_hsolve_bracket<<<(unsigned)np, 64 * kBWaves, 0, s>>>(fails, n_fails, U, o_xyz, o_s, hfact, eps, o_h, o_branch,
                                                           bcount);
    SPH_LAUNCH_CHECK();
    kt2.done();
  }
  kt.done();
}

void pseudo_build(Ctx &ctx, PseudoArgs &a, hipStream_t s) {
  Arena &ar = ctx.arena;
  const int64_t n = a.n;
  const auto &o = a.opts;
  int *bad = ar.get<int>("ps_bad", 1);
  SPH_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  k_check_unit_cube<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, a.xyz, bad);
  SPH_LAUNCH_CHECK();
  int bad_h = 0;
  SPH_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  SPH_REQUIRE(bad_h == 0, SPHMAP_EINVAL, std::to_string(bad_h) + " particle(s) outside [0,1)^3");

  // Morton order in the unit cube
  uint64_t *keys = ar.get<uint64_t>("ps_keys", n);
  int32_t *sidx = ar.get<int32_t>("ps_sidx", n);
  morton_keys(a.xyz, 3, n, 0.0, 0.0, 0.0, 1.0, keys, sidx, s);
  radix_sort_u64(ar, keys, sidx, n, 63, s);

  // level-synchronous octree build
  Grow G(ar);
  G.ensure(std::max<int64_t>(2 * n / std::max(o.leaf_max, 1) + 64, 1024), 0, s);
  k_root<<<1, 1, 0, s>>>(G.N, n);
  SPH_LAUNCH_CHECK();
  std::vector<int64_t> loff = {0, 1};  // level offsets
  for (int level = 0; level < kMaxLevels; ++level) {
    const int64_t b = loff[level], e = loff[level + 1], cnt = e - b;
    if (cnt == 0) break;
    int32_t *tfirst = ar.get<int32_t>("ps_tfirst", 8 * cnt);
    int32_t *tcount = ar.get<int32_t>("ps_tcount", 8 * cnt);
    int64_t *nch = ar.get<int64_t>("ps_nch", cnt + 1);
    int64_t *choff = ar.get<int64_t>("ps_choff", cnt + 1);
    k_split<<<(unsigned)div_up(cnt, 256), 256, 0, s>>>(G.N, b, e, level, keys, o.leaf_max, o.max_depth, tfirst,
                                                        tcount, nch);
    SPH_LAUNCH_CHECK();
    scan_exclusive_i64(ar, nch, choff, cnt, true, s);
    int64_t tot = 0;
    SPH_HIP(hipMemcpyAsync(&tot, choff + cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    G.ensure(e + tot, e, s);
    k_children<<<(unsigned)div_up(cnt, 256), 256, 0, s>>>(G.N, b, e, level, e, tfirst, tcount, nch, choff);
    SPH_LAUNCH_CHECK();
    loff.push_back(e + tot);
    if (tot == 0) break;
  }
  const int64_t nn = loff.back();
  const NodeArrays &N = G.N;

  // moments
  double *M = ar.get<double>("ps_M", nn);
  double4 *S = ar.get<double4>("ps_S", nn);
  double4 *com = ar.get<double4>("ps_com", nn);
  double *s2 = ar.get<double>("ps_s2", nn);
  int32_t *minidx = ar.get<int32_t>("ps_minidx", nn);
  int8_t *acc = ar.get<int8_t>("ps_acc", nn);
  int8_t *asc = ar.get<int8_t>("ps_asc", nn);
  k_leaf_moments<<<(unsigned)div_up(nn, 256), 256, 0, s>>>(N, nn, sidx, a.xyz, a.m, M, S, asc);
  SPH_LAUNCH_CHECK();
  for (int level = (int)loff.size() - 2; level >= 0; --level) {
    const int64_t b = loff[level], e = loff[level + 1];
    if (e > b) {
      k_internal_moments<<<(unsigned)div_up(e - b, 256), 256, 0, s>>>(N, b, e, M, S);
      SPH_LAUNCH_CHECK();
    }
  }
  k_com<<<(unsigned)div_up(nn, 256), 256, 0, s>>>(nn, M, S, com);
  SPH_LAUNCH_CHECK();
  double4 *sx = ar.get<double4>("ps_sx", n);
  k_sorted_xyz<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, sidx, a.xyz, sx);
  SPH_LAUNCH_CHECK();
  k_node_size<<<(unsigned)div_up(nn * 64, 256), 256, 0, s>>>(N, nn, sidx, sx, com, s2, minidx);
  SPH_LAUNCH_CHECK();
  {
    int64_t *bflag = ar.get<int64_t>("ps_bflag", nn + 1);
    int64_t *boff = ar.get<int64_t>("ps_boff", nn + 1);
    // the nodes of a level are disjoint, so its big nodes hold at most
    // n / kBigNode + (their number, itself at most n / kBigNode) chunks
    const int64_t bound = std::max<int64_t>(1, (int64_t)(loff.size() - 1) * (2 * (n / kBigNode) + 1));
    int32_t *blist = ar.get<int32_t>("ps_blist", bound);
    k_flag_big<<<(unsigned)div_up(nn, 256), 256, 0, s>>>(N, nn, bflag);
    SPH_LAUNCH_CHECK();
    scan_exclusive_i64(ar, bflag, boff, nn, true, s);
    k_list_big<<<(unsigned)div_up(nn, 256), 256, 0, s>>>(N, nn, boff, blist);
    SPH_LAUNCH_CHECK();
    k_node_size_big<<<(unsigned)std::min<int64_t>(bound, 2048), 1024, 0, s>>>(N, blist, boff, boff + nn, sidx, sx,
                                                                              com, s2, minidx);
    SPH_LAUNCH_CHECK();
  }
  double *src = ar.get<double>("ps_src", 3 * a.n_src);
  SPH_HIP(hipMemcpyAsync(src, a.src, 3 * a.n_src * sizeof(double), hipMemcpyHostToDevice, s));
  k_accept<<<(unsigned)div_up(nn, 256), 256, 0, s>>>(nn, com, s2, a.n_src, src, o.r_part, o.theta, acc);
  SPH_LAUNCH_CHECK();
  uint64_t *label = ar.get<uint64_t>("ps_label", nn);
  k_label<<<(unsigned)div_up(nn, 256), 256, 0, s>>>(N, nn, keys, label);
  SPH_LAUNCH_CHECK();
  if (a.n_open > 0) {
    uint64_t *op = ar.get<uint64_t>("ps_open", a.n_open);
    int32_t *dummy = ar.get<int32_t>("ps_open_idx", a.n_open);
    SPH_HIP(hipMemcpyAsync(op, a.open_labels, a.n_open * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    iota_i32(dummy, a.n_open, s);
    radix_sort_u64(ar, op, dummy, a.n_open, 64, s);
    k_force_open<<<(unsigned)div_up(nn, 256), 256, 0, s>>>(nn, label, a.n_open, op, acc);
    SPH_LAUNCH_CHECK();
  }

  // units in depth-first order
  int32_t *unit_at = ar.get<int32_t>("ps_unit_at", n);
  k_fill_i32<<<(unsigned)div_up(n, 256), 256, 0, s>>>(unit_at, -1, n);
  SPH_LAUNCH_CHECK();
  k_units<<<(unsigned)div_up(nn, 256), 256, 0, s>>>(N, nn, acc, unit_at);
  SPH_LAUNCH_CHECK();
  int64_t *flag = ar.get<int64_t>("ps_flag", n + 1);
  int64_t *uoff = ar.get<int64_t>("ps_uoff", n + 1);
  k_flag<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, unit_at, flag);
  SPH_LAUNCH_CHECK();
  scan_exclusive_i64(ar, flag, uoff, n, true, s);
  int64_t nu = 0;
  SPH_HIP(hipMemcpyAsync(&nu, uoff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  int32_t *units = ar.get<int32_t>("ps_units", nu);
  k_unit_list<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, unit_at, uoff, units);
  SPH_LAUNCH_CHECK();
  int64_t *ecnt = ar.get<int64_t>("ps_ecnt", nu + 1);
  int64_t *eoff = ar.get<int64_t>("ps_eoff", nu + 1);
  int64_t *pcnt = ar.get<int64_t>("ps_pcnt", nu + 1);
  int64_t *poff = ar.get<int64_t>("ps_poff", nu + 1);
  k_unit_counts<<<(unsigned)div_up(nu, 256), 256, 0, s>>>(nu, units, N, acc, ecnt, pcnt);
  SPH_LAUNCH_CHECK();
  scan_exclusive_i64(ar, ecnt, eoff, nu, true, s);
  scan_exclusive_i64(ar, pcnt, poff, nu, true, s);
  int64_t tot[2] = {0, 0};
  SPH_HIP(hipMemcpyAsync(&tot[0], eoff + nu, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipMemcpyAsync(&tot[1], poff + nu, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  const int64_t n_out = tot[0], np = tot[1];
  SPH_REQUIRE(n_out <= a.capacity, SPHMAP_ERANGE,
              "pseudo-particle output needs " + std::to_string(n_out) + " entries, capacity " +
                  std::to_string(a.capacity));
  double4 *upos = ar.get<double4>("ps_upos", nu);
  int32_t *plist = ar.get<int32_t>("ps_plist", np + 1);
  // the solve reads the node sizes back: keep them in scratch when the
  // caller does not ask for them
  double *o_s = a.o_s ? a.o_s : ar.get<double>("ps_os", n_out);
  k_entries<<<(unsigned)div_up(nu, 256), 256, 0, s>>>(nu, units, N, acc, eoff, poff, sidx, a.xyz, a.h, a.m, M, com,
                                                      s2, minidx, a.o_xyz, a.o_h, a.o_m, o_s, a.o_kind, a.o_first,
                                                      a.o_count, a.o_branch, upos, plist, label, a.o_label, asc);
  SPH_LAUNCH_CHECK();
  if (a.o_owner && n > 0) {
    k_owner<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, flag, uoff, units, N, acc, eoff, sidx, asc, a.o_owner);
    SPH_LAUNCH_CHECK();
  }

  // node smoothing lengths
  unsigned long long *bcount = ar.get<unsigned long long>("ps_bcount", 4);
  SPH_HIP(hipMemsetAsync(bcount, 0, 4 * sizeof(unsigned long long), s));
  node_hsolve(ctx, np, plist, nu, upos, a.o_xyz, o_s, o.h_fact, o.eps_h, o.bypass_threshold, a.o_h, a.o_branch,
              bcount, 0, nullptr, nullptr, nullptr, nullptr, s);
  unsigned long long bc[4] = {0, 0, 0, 0};
  SPH_HIP(hipMemcpyAsync(bc, bcount, sizeof bc, hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  a.n_out = n_out;
  a.stats.n_nodes = nn;
  a.stats.n_units = nu;
  a.stats.n_pseudo = np;
  a.stats.n_real = n_out - np;
  {
    double r2 = 0.0;
    SPH_HIP(hipMemcpyAsync(&r2, s2, sizeof(double), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    a.stats.s_root = sqrt(r2);
  }
  for (int k = 0; k < 4; ++k) a.stats.branch_count[k] = (int64_t)bc[k];
}

__global__ void k_underresolved_flag(int64_t n, const int32_t *kind, const double *s_node, const double *fneu,
                                     double s_root, double K, int64_t *flag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  // eq. resol_param: f_neu,limit = (1/K) (K - 1 / (s_node / s_root))
  flag[e] = (kind[e] == 1 && fneu[e] < (K - 1.0 / (s_node[e] / s_root)) / K) ? 1 : 0;
}

__global__ void k_underresolved_list(int64_t n, const int64_t *flag, const int64_t *off, const uint64_t *label,
                                     uint64_t *out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && flag[e]) out[off[e]] = label[e];
}

int64_t select_underresolved(Ctx &ctx, int64_t n, const int32_t *kind, const uint64_t *label, const double *s_node,
                             const double *fneu, double s_root, double K, uint64_t *out, hipStream_t s) {
  if (n <= 0) return 0;
  int64_t *flag = ctx.arena.get<int64_t>("ur_flag", n + 1);
  int64_t *off = ctx.arena.get<int64_t>("ur_off", n + 1);
  k_underresolved_flag<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, kind, s_node, fneu, s_root, K, flag);
  SPH_LAUNCH_CHECK();
  scan_exclusive_i64(ctx.arena, flag, off, n, true, s);
  k_underresolved_list<<<(unsigned)div_up(n, 256), 256, 0, s>>>(n, flag, off, label, out);
  SPH_LAUNCH_CHECK();
  int64_t cnt = 0;
  SPH_HIP(hipMemcpyAsync(&cnt, off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  return cnt;
}

}  // namespace sphmap
