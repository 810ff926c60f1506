// Pseudo-particles from the paper's own tree (Sec. 2.2.1, 2.4): a binary k-d
// tree built top down by recursive coordinate bisection.
//
// Build, one level at a time: each node of the level sums its particles'
// m and m x as fixed-point integers of 2^-K (atomics: the sums are exact,
// so the centre of mass, and with it the split plane, does not depend on
// the order of the additions); a node with at least leaf_split particles
// (below max_depth) splits its domain through the centre of mass along the
// domain's longest axis.  One scan over the particle order per level gives
// every splitting node a stable partition (left: coordinate below the
// split), so each node is a contiguous run of the particle order and its
// members stay in ascending index.  Labels: root 1, children 2n and 2n + 1.
//
// Walk (Sec. 2.4.1): per source, a node reaches r_part when r - s <= r_part,
// reaches r_leaf when r - s <= r_leaf, and fails the opening angle when
// theta^2 r^2 < s^2 (eq. opening_angle); it is accepted when none holds for
// any source and it is not named for opening.  Emitted units are the
// accepted nodes without an accepted ancestor and the leaves that are not
// accepted; such a leaf gives its particles (own h) when it reaches r_part,
// is named or holds one particle, else it is a leaf pseudo-particle.
//
// Node smoothing lengths: the h-solve of the octree builder, over all
// units, or, with more than nf_threshold units, over the trial neighbours
// of the neighbour-find of Sec. 2.4.3 (k_mid one level above the highest
// unit; r_cut from the k_mid ancestor's size, or eq.
// compact_support_radius with the ancestor up_levels above the target).
#include <cmath>
#include <cstring>

#include "common.hpp"

namespace sphmap {
namespace {

struct KdNodes {
  uint64_t *label;
  int32_t *level, *parent, *first, *count, *left, *nleft;
  double4 *lo, *hi;        // domain
  long long *q;            // [4 node]: m, m x, m y, m z in units of 2^-K
  double4 *com;            // centre of mass; w = mass
  unsigned long long *s2;  // squared size (non-negative doubles order as their bits)
  int32_t *axis;           // split axis, -1 for a leaf
  double *split;
};

__global__ void k_kd_check(int64_t n, const double *xyz, const double *m, int *bad, unsigned long long *mmax) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) {
    const double x = xyz[3 * i + k];
    if (!(x >= 0.0 && x < 1.0)) atomicOr(bad, 1);
  }
  const double mi = m[i];
  if (!(mi > 0.0 && mi < INFINITY)) atomicOr(bad, 2);
  else atomicMax(mmax, (unsigned long long)__double_as_longlong(mi));
}

// pxm[i] holds the position and mass of particle perm[i], so that the
// per-level kernels read their particles contiguously instead of gathering
__global__ void k_kd_init(int64_t n, const double *xyz, const double *m, int32_t *perm, int32_t *nop,
                          double4 *pxm, KdNodes N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    perm[i] = (int32_t)i;
    nop[i] = 0;
    pxm[i] = make_double4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], m[i]);
  }
  if (i == 0) {
    N.label[0] = 1;
    N.level[0] = 0;
    N.parent[0] = -1;
    N.first[0] = 0;
    N.count[0] = (int32_t)n;
    N.left[0] = -1;
    N.lo[0] = make_double4(0.0, 0.0, 0.0, 0.0);
    N.hi[0] = make_double4(1.0, 1.0, 1.0, 0.0);
  }
}

__global__ void k_kd_zero(int64_t b, int64_t e, KdNodes N) {
  const int64_t k = b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= e) return;
  N.q[4 * k] = N.q[4 * k + 1] = N.q[4 * k + 2] = N.q[4 * k + 3] = 0;
  N.s2[k] = 0ull;
}

// Levels with at most kLdsNodes nodes (the top of the tree, where every
// particle of the level adds to a handful of nodes) accumulate per
// workgroup in LDS first; integer sums and maxima do not depend on how the
// additions are grouped.
constexpr int kLdsNodes = 1024;

// Runs of equal keys among a wave's lanes (the particles of a node are
// contiguous, so a wave holds few runs): each lane's position in its run and
// the run's inclusive sums or maxima by a segmented scan over the lanes.
// Returns true in the last lane of each run, which then holds the run's
// total; the other lanes hold partial results.  Integer sums and maxima do
// not depend on how they are grouped.
struct WaveRuns {
  int lane;
  int seg;  // lanes [seg, lane] hold the same key
  __device__ explicit WaveRuns(int64_t key) {
    lane = threadIdx.x & 63;
    const int64_t prev = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || prev != key;
    const uint64_t heads = __ballot(head);
    const uint64_t upto = heads & (lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull));
    seg = 63 - __builtin_clzll(upto);  // lane 0 is always a head
    next_differs = __shfl_down(key, 1, 64) != key || lane == 63;
  }
  bool next_differs;
  __device__ bool last() const { return next_differs; }
  __device__ void add(unsigned long long &v) const {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long u = __shfl_up(v, o, 64);
      if (lane - o >= seg) v += u;
    }
  }
  __device__ void max(unsigned long long &v) const {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long u = __shfl_up(v, o, 64);
      if (lane - o >= seg && u > v) v = u;
    }
  }
};

__global__ void __launch_bounds__(256) k_kd_sums(int64_t n, const double4 *pxm, const int32_t *nop, int64_t b,
                                                 int64_t e, int K, KdNodes N) {
#pragma clang fp contract(off)
  __shared__ unsigned long long acc[4 * kLdsNodes];
  const bool lds = e - b <= kLdsNodes;
  if (lds) {
    for (int t = threadIdx.x; t < 4 * (e - b); t += blockDim.x) acc[t] = 0ull;
    __syncthreads();
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t node = -1;
  if (i < n) {
    node = nop[i];
    if (node < b || node >= e) node = -1;
  }
  unsigned long long v[4] = {0ull, 0ull, 0ull, 0ull};
  if (node >= 0) {
    const double4 pj = pxm[i];
    const double mj = pj.w;
    v[0] = (unsigned long long)__double2ll_rn(ldexp(mj, K));
    v[1] = (unsigned long long)__double2ll_rn(ldexp(mj * pj.x, K));
    v[2] = (unsigned long long)__double2ll_rn(ldexp(mj * pj.y, K));
    v[3] = (unsigned long long)__double2ll_rn(ldexp(mj * pj.z, K));
  }
  // one addition per run of the wave's lanes that share a node
  const WaveRuns runs(node);
  for (int k = 0; k < 4; ++k) runs.add(v[k]);
  if (node >= 0 && runs.last()) {
    if (lds) {
      for (int k = 0; k < 4; ++k) atomicAdd(&acc[4 * (node - b) + k], v[k]);
    } else {
      unsigned long long *q = (unsigned long long *)N.q + 4 * node;
      for (int k = 0; k < 4; ++k) atomicAdd(q + k, v[k]);
    }
  }
  if (lds) {
    __syncthreads();
    for (int t = threadIdx.x; t < 4 * (e - b); t += blockDim.x)
      if (acc[t]) atomicAdd((unsigned long long *)N.q + 4 * b + t, acc[t]);
  }
}

__global__ void k_kd_com(int64_t b, int64_t e, int K, int leaf_split, int max_depth, KdNodes N) {
  const int64_t k = b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= e) return;
  const double qm = (double)N.q[4 * k];
  double4 c;
  c.x = (double)N.q[4 * k + 1] / qm;
  c.y = (double)N.q[4 * k + 2] / qm;
  c.z = (double)N.q[4 * k + 3] / qm;
  c.w = ldexp(qm, -K);
  N.com[k] = c;
  int axis = -1;
  if (N.count[k] >= leaf_split && N.level[k] < max_depth) {
    const double4 lo = N.lo[k], hi = N.hi[k];
    const double ex = hi.x - lo.x, ey = hi.y - lo.y, ez = hi.z - lo.z;
    axis = 0;
    double best = ex;
    if (ey > best) {
      axis = 1;
      best = ey;
    }
    if (ez > best) axis = 2;
  }
  N.axis[k] = axis;
  N.split[k] = axis == 0 ? c.x : (axis == 1 ? c.y : c.z);
  N.left[k] = -1;
}

__global__ void __launch_bounds__(256) k_kd_size_flags(int64_t n, const double4 *pxm, const int32_t *nop,
                                                       int64_t b, int64_t e, KdNodes N, int64_t *flag) {
#pragma clang fp contract(off)
  __shared__ unsigned long long mx[kLdsNodes];
  const bool lds = e - b <= kLdsNodes;
  if (lds) {
    for (int t = threadIdx.x; t < e - b; t += blockDim.x) mx[t] = 0ull;
    __syncthreads();
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t node = -1;
  unsigned long long bits = 0ull;
  if (i < n) {
    node = nop[i];
    int64_t f = 0;
    if (node >= b && node < e) {
      const double4 pj = pxm[i];
      const double4 c = N.com[node];
      const double dx = pj.x - c.x, dy = pj.y - c.y, dz = pj.z - c.z;
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      bits = (unsigned long long)__double_as_longlong(d2);
      const int a = N.axis[node];
      if (a >= 0) f = (a == 0 ? pj.x : (a == 1 ? pj.y : pj.z)) < N.split[node] ? 1 : 0;
    } else {
      node = -1;
    }
    flag[i] = f;
  }
  // one maximum per run of the wave's lanes that share a node
  const WaveRuns runs(node);
  runs.max(bits);
  if (node >= 0 && runs.last()) {
    if (lds) atomicMax(&mx[node - b], bits);
    else atomicMax(&N.s2[node], bits);
  }
  if (lds) {
    __syncthreads();
    for (int t = threadIdx.x; t < e - b; t += blockDim.x)
      if (mx[t]) atomicMax(&N.s2[b + t], mx[t]);
  }
}

// children per splitting node: 2 when both sides are non-empty
__global__ void k_kd_nch(int64_t b, int64_t e, const int64_t *scan, KdNodes N, int64_t *nch) {
  const int64_t k = b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= e) return;
  int64_t c = 0;
  if (N.axis[k] >= 0) {
    const int64_t f = N.first[k], cnt = N.count[k];
    const int64_t nl = scan[f + cnt] - scan[f];
    N.nleft[k] = (int32_t)nl;
    if (nl > 0 && nl < cnt) c = 2;
    else N.axis[k] = -1;
  }
  nch[k - b] = c;
}

__global__ void k_kd_children(int64_t b, int64_t e, int64_t base, const int64_t *choff, KdNodes N) {
  const int64_t k = b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= e || N.axis[k] < 0) return;
  const int64_t l = base + choff[k - b];
  const int a = N.axis[k];
  const double sp = N.split[k];
  N.left[k] = (int32_t)l;
  for (int side = 0; side < 2; ++side) {
    const int64_t c = l + side;
    N.label[c] = 2 * N.label[k] + side;
    N.level[c] = N.level[k] + 1;
    N.parent[c] = (int32_t)k;
    N.first[c] = side ? N.first[k] + N.nleft[k] : N.first[k];
    N.count[c] = side ? N.count[k] - N.nleft[k] : N.nleft[k];
    N.left[c] = -1;
    double4 lo = N.lo[k], hi = N.hi[k];
    if (side == 0) {
      if (a == 0) hi.x = sp;
      else if (a == 1) hi.y = sp;
      else hi.z = sp;
    } else {
      if (a == 0) lo.x = sp;
      else if (a == 1) lo.y = sp;
      else lo.z = sp;
    }
    N.lo[c] = lo;
    N.hi[c] = hi;
  }
}

__global__ void k_kd_permute(int64_t n, const int32_t *perm, const int32_t *nop, const double4 *pxm, int32_t *perm2,
                             int32_t *nop2, double4 *pxm2, int64_t b, int64_t e, const int64_t *scan,
                             const int64_t *flag, KdNodes N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t node = nop[i];
  if (node < b || node >= e || N.axis[node] < 0) {
    perm2[i] = perm[i];
    nop2[i] = (int32_t)node;
    pxm2[i] = pxm[i];
    return;
  }
  const int64_t f = N.first[node];
  const int64_t lrank = scan[i] - scan[f];
  int64_t to;
  int32_t child;
  if (flag[i]) {
    to = f + lrank;
    child = N.left[node];
  } else {
    to = f + N.nleft[node] + ((i - f) - lrank);
    child = N.left[node] + 1;
  }
  perm2[to] = perm[i];
  nop2[to] = child;
  pxm2[to] = pxm[i];
}

__device__ inline bool kd_in(uint64_t label, int64_t n_open, const uint64_t *open) {
  int64_t lo = 0, hi = n_open;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (open[mid] < label) lo = mid + 1;
    else hi = mid;
  }
  return lo < n_open && open[lo] == label;
}

// bit 0: accepted; bit 1: a leaf here gives its particles
__global__ void k_kd_accept(int64_t nn, KdNodes N, int n_src, const double *src, double r_part, double r_leaf,
                            double theta, int64_t n_open, const uint64_t *open, int8_t *acc) {
#pragma clang fp contract(off)
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const double4 c = N.com[k];
  const double s2 = __longlong_as_double((long long)N.s2[k]);
  const double s = sqrt(s2);
  bool part = false, leafz = false, angle = false;
  for (int q = 0; q < n_src; ++q) {
    const double dx = c.x - src[3 * q], dy = c.y - src[3 * q + 1], dz = c.z - src[3 * q + 2];
    const double r = sqrt((dx * dx + dy * dy) + dz * dz);
    if (r - s <= r_part) part = true;
    if (r - s <= r_leaf) leafz = true;
    if (theta * theta * r * r < s2) angle = true;
  }
  const bool forced = n_open > 0 && kd_in(N.label[k], n_open, open);
  const bool accepted = !(part || leafz || angle || forced);
  acc[k] = (int8_t)((accepted ? 1 : 0) | ((part || forced || N.count[k] == 1) ? 2 : 0));
}

__global__ void k_kd_fill(int32_t *p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_kd_units(int64_t nn, KdNodes N, const int8_t *acc, int32_t *unit_at) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  for (int32_t p = N.parent[k]; p >= 0; p = N.parent[p])
    if (acc[p] & 1) return;
  if ((acc[k] & 1) || N.left[k] < 0) unit_at[N.first[k]] = (int32_t)k;
}

__global__ void k_kd_uflag(int64_t n, const int32_t *unit_at, int64_t *flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) flag[t] = unit_at[t] >= 0 ? 1 : 0;
}

__global__ void k_kd_ulist(int64_t n, const int32_t *unit_at, const int64_t *uoff, int32_t *units) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && unit_at[t] >= 0) units[uoff[t]] = unit_at[t];
}

// does unit node k give its particles?
__device__ inline bool kd_gives_particles(int8_t a, int32_t count) { return count == 1 || (!(a & 1) && (a & 2)); }

__global__ void k_kd_ucounts(int64_t nu, const int32_t *units, KdNodes N, const int8_t *acc, int64_t *ecnt,
                             int64_t *pcnt, int *kmin) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nu) return;
  const int32_t k = units[u];
  const bool parts = kd_gives_particles(acc[k], N.count[k]);
  ecnt[u] = parts ? N.count[k] : 1;
  pcnt[u] = parts ? 0 : 1;
  atomicMin(kmin, N.level[k]);
}

__global__ void k_kd_entries(int64_t nu, const int32_t *units, KdNodes N, const int8_t *acc, const int64_t *eoff,
                             const int64_t *poff, const int32_t *perm, const double *xyz, const double *hh,
                             const double *m, double *o_xyz, double *o_h, double *o_m, double *o_s, int32_t *o_kind,
                             int64_t *o_first, int64_t *o_count, int32_t *o_branch, uint64_t *o_label,
                             int32_t *o_level, int32_t *e_node, double4 *upos, int32_t *plist) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nu) return;
  const int32_t k = units[u];
  const double4 c = N.com[k];
  upos[u] = c;
  int64_t e = eoff[u];
  const int32_t f = N.first[k], cnt = N.count[k];
  if (kd_gives_particles(acc[k], cnt)) {
    for (int32_t t = 0; t < cnt; ++t, ++e) {  // members in ascending index
      const int64_t j = perm[f + t];
      o_xyz[3 * e] = xyz[3 * j];
      o_xyz[3 * e + 1] = xyz[3 * j + 1];
      o_xyz[3 * e + 2] = xyz[3 * j + 2];
      o_h[e] = hh[j];
      o_m[e] = m[j];
      o_s[e] = 0.0;
      if (o_kind) o_kind[e] = 0;
      if (o_first) o_first[e] = j;
      if (o_count) o_count[e] = 1;
      if (o_branch) o_branch[e] = -1;
      if (o_label) o_label[e] = N.label[k];
      if (o_level) o_level[e] = N.level[k];
      e_node[e] = k;
    }
    return;
  }
  o_xyz[3 * e] = c.x;
  o_xyz[3 * e + 1] = c.y;
  o_xyz[3 * e + 2] = c.z;
  o_h[e] = 0.0;
  o_m[e] = c.w;
  o_s[e] = sqrt(__longlong_as_double((long long)N.s2[k]));
  if (o_kind) o_kind[e] = 1;
  if (o_first) o_first[e] = perm[f];
  if (o_count) o_count[e] = cnt;
  if (o_branch) o_branch[e] = 0;
  if (o_label) o_label[e] = N.label[k];
  if (o_level) o_level[e] = N.level[k];
  e_node[e] = k;
  plist[poff[u]] = (int32_t)e;
}

__global__ void k_kd_owner(int64_t n, const int64_t *flag, const int64_t *uoff, const int32_t *units, KdNodes N,
                           const int8_t *acc, const int64_t *eoff, const int32_t *perm, int64_t *owner) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int64_t u = uoff[q] + flag[q] - 1;
  const int32_t k = units[u];
  int64_t e = eoff[u];
  if (kd_gives_particles(acc[k], N.count[k])) e += q - N.first[k];
  owner[perm[q]] = e;
}

__device__ inline int32_t kd_ancestor(const KdNodes &N, int32_t k, int level) {
  while (k >= 0 && N.level[k] > level) k = N.parent[k];
  return k;
}

// unit range of every k_mid node (units of one subtree are contiguous)
__global__ void k_kd_midrange(int64_t nu, const int32_t *units, KdNodes N, int k_mid, int64_t mid_base,
                              int32_t *u0, int32_t *u1) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nu) return;
  const int32_t a = kd_ancestor(N, units[u], k_mid);
  const int64_t mi = a - mid_base;
  if (u == 0 || kd_ancestor(N, units[u - 1], k_mid) != a) u0[mi] = (int32_t)u;
  if (u == nu - 1 || kd_ancestor(N, units[u + 1], k_mid) != a) u1[mi] = (int32_t)(u + 1);
}

__global__ void k_kd_rcut(int64_t np, const int32_t *plist, const int32_t *e_node, const double *o_s, KdNodes N,
                          int k_mid, int up, double hfact, double *rcut) {
#pragma clang fp contract(off)
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int32_t e = plist[p];
  const int32_t k = e_node[e];
  const int32_t mid = kd_ancestor(N, k, k_mid);
  double rc = sqrt(3.0) * sqrt(__longlong_as_double((long long)N.s2[mid]));
  if (rc < 4.0 * hfact * o_s[e]) {
    const int lv = N.level[k] - up;
    const int32_t above = kd_ancestor(N, k, lv > 0 ? lv : 0);
    rc = 4.0 * hfact * sqrt(__longlong_as_double((long long)N.s2[above]));
  }
  rcut[e] = rc;
}

__global__ void k_kd_midcom(int64_t n_mid, int64_t base, KdNodes N, double4 *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_mid) out[i] = N.com[base + i];
}

__global__ void k_kd_zero_i32(int64_t n, int32_t *a, int32_t *b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    a[i] = 0;
    b[i] = 0;
  }
}

inline unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, div_up(n, 256)); }

}  // namespace

void kd_pseudo_build(Ctx &ctx, KdArgs &ka, hipStream_t s) {
  PseudoArgs &a = ka.base;
  Arena &ar = ctx.arena;
  const int64_t n = a.n;
  const auto &o = a.opts;
  SPH_REQUIRE(ka.leaf_split >= 2, SPHMAP_EINVAL, "leaf_split must be >= 2");
  SPH_REQUIRE(o.max_depth >= 0 && o.max_depth <= 62, SPHMAP_EINVAL, "max_depth must be in [0, 62]");
  SPH_REQUIRE(ka.r_leaf >= 0.0 && ka.up_levels >= 0, SPHMAP_EINVAL, "bad r_leaf or up_levels");
  int *bad = ar.get<int>("kd_bad", 1);
  unsigned long long *dmax = ar.get<unsigned long long>("kd_mmax", 1);
  SPH_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  SPH_HIP(hipMemsetAsync(dmax, 0, sizeof(unsigned long long), s));
  k_kd_check<<<grid_of(n), 256, 0, s>>>(n, a.xyz, a.m, bad, dmax);
  SPH_LAUNCH_CHECK();
  int bad_h = 0;
  unsigned long long mm = 0;
  SPH_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipMemcpyAsync(&mm, dmax, sizeof mm, hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  SPH_REQUIRE(!(bad_h & 1), SPHMAP_EINVAL, "particle(s) outside [0,1)^3");
  SPH_REQUIRE(!(bad_h & 2), SPHMAP_EINVAL, "masses must be positive and finite");
  double mmax_d;
  std::memcpy(&mmax_d, &mm, sizeof mmax_d);
  int ex = 0;
  std::frexp((double)n * mmax_d, &ex);
  const int K = 62 - ex;

  // nodes: at most 2n - 1
  const int64_t cap = 2 * n + 1;
  KdNodes N;
  N.label = ar.get<uint64_t>("kd_label", cap);
  N.level = ar.get<int32_t>("kd_level", cap);
  N.parent = ar.get<int32_t>("kd_parent", cap);
  N.first = ar.get<int32_t>("kd_first", cap);
  N.count = ar.get<int32_t>("kd_count", cap);
  N.left = ar.get<int32_t>("kd_left", cap);
  N.nleft = ar.get<int32_t>("kd_nleft", cap);
  N.lo = ar.get<double4>("kd_lo", cap);
  N.hi = ar.get<double4>("kd_hi", cap);
  N.q = ar.get<long long>("kd_q", 4 * cap);
  N.com = ar.get<double4>("kd_com", cap);
  N.s2 = ar.get<unsigned long long>("kd_s2", cap);
  N.axis = ar.get<int32_t>("kd_axis", cap);
  N.split = ar.get<double>("kd_split", cap);
  int32_t *perm = ar.get<int32_t>("kd_perm", n), *perm2 = ar.get<int32_t>("kd_perm2", n);
  int32_t *nop = ar.get<int32_t>("kd_nop", n), *nop2 = ar.get<int32_t>("kd_nop2", n);
  double4 *pxm = ar.get<double4>("kd_pxm", n), *pxm2 = ar.get<double4>("kd_pxm2", n);
  int64_t *flag = ar.get<int64_t>("kd_flag", n + 1), *scan = ar.get<int64_t>("kd_scan", n + 1);
  k_kd_init<<<grid_of(n), 256, 0, s>>>(n, a.xyz, a.m, perm, nop, pxm, N);
  SPH_LAUNCH_CHECK();
  std::vector<int64_t> loff = {0, 1};
  {
    KernelTimer kt(&ctx, "kd_build", s);
    for (;;) {
      const int64_t b = loff[loff.size() - 2], e = loff.back();
      const int64_t cnt = e - b;
      k_kd_zero<<<grid_of(cnt), 256, 0, s>>>(b, e, N);
      SPH_LAUNCH_CHECK();
      k_kd_sums<<<grid_of(n), 256, 0, s>>>(n, pxm, nop, b, e, K, N);
      SPH_LAUNCH_CHECK();
      k_kd_com<<<grid_of(cnt), 256, 0, s>>>(b, e, K, ka.leaf_split, o.max_depth, N);
      SPH_LAUNCH_CHECK();
      k_kd_size_flags<<<grid_of(n), 256, 0, s>>>(n, pxm, nop, b, e, N, flag);
      SPH_LAUNCH_CHECK();
      scan_exclusive_i64(ar, flag, scan, n, true, s);
      int64_t *nch = ar.get<int64_t>("kd_nch", cnt + 1), *choff = ar.get<int64_t>("kd_choff", cnt + 1);
      k_kd_nch<<<grid_of(cnt), 256, 0, s>>>(b, e, scan, N, nch);
      SPH_LAUNCH_CHECK();
      scan_exclusive_i64(ar, nch, choff, cnt, true, s);
      int64_t tot = 0;
      SPH_HIP(hipMemcpyAsync(&tot, choff + cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      SPH_HIP(hipStreamSynchronize(s));
      if (tot == 0) break;
      SPH_REQUIRE(e + tot <= cap, SPHMAP_EINVAL, "k-d tree larger than 2n nodes");
      k_kd_children<<<grid_of(cnt), 256, 0, s>>>(b, e, e, choff, N);
      SPH_LAUNCH_CHECK();
      k_kd_permute<<<grid_of(n), 256, 0, s>>>(n, perm, nop, pxm, perm2, nop2, pxm2, b, e, scan, flag, N);
      SPH_LAUNCH_CHECK();
      std::swap(perm, perm2);
      std::swap(nop, nop2);
      std::swap(pxm, pxm2);
      loff.push_back(e + tot);
    }
    kt.done();
  }
  const int64_t nn = loff.back();

  // walk
  double *src = ar.get<double>("kd_src", 3 * a.n_src);
  SPH_HIP(hipMemcpyAsync(src, a.src, 3 * a.n_src * sizeof(double), hipMemcpyHostToDevice, s));
  uint64_t *op = nullptr;
  if (a.n_open > 0) {
    op = ar.get<uint64_t>("kd_open", a.n_open);
    int32_t *dummy = ar.get<int32_t>("kd_open_idx", a.n_open);
    SPH_HIP(hipMemcpyAsync(op, a.open_labels, a.n_open * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    iota_i32(dummy, a.n_open, s);
    radix_sort_u64(ar, op, dummy, a.n_open, 64, s);
  }
  int8_t *acc = ar.get<int8_t>("kd_acc", nn);
  k_kd_accept<<<grid_of(nn), 256, 0, s>>>(nn, N, a.n_src, src, o.r_part, ka.r_leaf, o.theta, a.n_open, op, acc);
  SPH_LAUNCH_CHECK();
  int32_t *unit_at = ar.get<int32_t>("kd_unit_at", n);
  k_kd_fill<<<grid_of(n), 256, 0, s>>>(unit_at, -1, n);
  SPH_LAUNCH_CHECK();
  k_kd_units<<<grid_of(nn), 256, 0, s>>>(nn, N, acc, unit_at);
  SPH_LAUNCH_CHECK();
  int64_t *uflag = ar.get<int64_t>("kd_uflag", n + 1), *uoff = ar.get<int64_t>("kd_uoff", n + 1);
  k_kd_uflag<<<grid_of(n), 256, 0, s>>>(n, unit_at, uflag);
  SPH_LAUNCH_CHECK();
  scan_exclusive_i64(ar, uflag, uoff, n, true, s);
  int64_t nu = 0;
  SPH_HIP(hipMemcpyAsync(&nu, uoff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  int32_t *units = ar.get<int32_t>("kd_units", nu);
  k_kd_ulist<<<grid_of(n), 256, 0, s>>>(n, unit_at, uoff, units);
  SPH_LAUNCH_CHECK();
  int64_t *ecnt = ar.get<int64_t>("kd_ecnt", nu + 1), *eoff = ar.get<int64_t>("kd_eoff", nu + 1);
  int64_t *pcnt = ar.get<int64_t>("kd_pcnt", nu + 1), *poff = ar.get<int64_t>("kd_poff", nu + 1);
  int *kmin = ar.get<int>("kd_kmin", 1);
  k_kd_fill<<<1, 64, 0, s>>>(kmin, 1 << 30, 1);
  SPH_LAUNCH_CHECK();
  k_kd_ucounts<<<grid_of(nu), 256, 0, s>>>(nu, units, N, acc, ecnt, pcnt, kmin);
  SPH_LAUNCH_CHECK();
  scan_exclusive_i64(ar, ecnt, eoff, nu, true, s);
  scan_exclusive_i64(ar, pcnt, poff, nu, true, s);
  int64_t tot[2] = {0, 0};
  int kmin_h = 0;
  SPH_HIP(hipMemcpyAsync(&tot[0], eoff + nu, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipMemcpyAsync(&tot[1], poff + nu, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipMemcpyAsync(&kmin_h, kmin, sizeof(int), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  const int64_t n_out = tot[0], np = tot[1];
  SPH_REQUIRE(n_out <= a.capacity, SPHMAP_ERANGE,
              "pseudo-particle output needs " + std::to_string(n_out) + " entries, capacity " +
                  std::to_string(a.capacity));
  double4 *upos = ar.get<double4>("kd_upos", nu);
  int32_t *plist = ar.get<int32_t>("kd_plist", np + 1);
  int32_t *e_node = ar.get<int32_t>("kd_enode", n_out);
  double *o_s = a.o_s ? a.o_s : ar.get<double>("kd_os", n_out);
  k_kd_entries<<<grid_of(nu), 256, 0, s>>>(nu, units, N, acc, eoff, poff, perm, a.xyz, a.h, a.m, a.o_xyz, a.o_h,
                                           a.o_m, o_s, a.o_kind, a.o_first, a.o_count, a.o_branch, a.o_label,
                                           ka.o_level, e_node, upos, plist);
  SPH_LAUNCH_CHECK();
  if (a.o_owner) {
    k_kd_owner<<<grid_of(n), 256, 0, s>>>(n, uflag, uoff, units, N, acc, eoff, perm, a.o_owner);
    SPH_LAUNCH_CHECK();
  }

  // node smoothing lengths
  unsigned long long *bcount = ar.get<unsigned long long>("kd_bcount", 4);
  SPH_HIP(hipMemsetAsync(bcount, 0, 4 * sizeof(unsigned long long), s));
  ka.k_mid = -1;
  int64_t n_mid = 0;
  double4 *mid_com = nullptr;
  int32_t *mu0 = nullptr, *mu1 = nullptr;
  double *rcut = nullptr;
  if (np > 0 && nu > ka.nf_threshold) {
    const int k_mid = kmin_h > 0 ? kmin_h - 1 : 0;
    ka.k_mid = k_mid;
    const int64_t mb = loff[k_mid], me = loff[k_mid + 1];
    n_mid = me - mb;
    mid_com = ar.get<double4>("kd_midcom", n_mid);
    mu0 = ar.get<int32_t>("kd_mu0", n_mid);
    mu1 = ar.get<int32_t>("kd_mu1", n_mid);
    rcut = ar.get<double>("kd_rcut", n_out);
    k_kd_midcom<<<grid_of(n_mid), 256, 0, s>>>(n_mid, mb, N, mid_com);
    SPH_LAUNCH_CHECK();
    k_kd_zero_i32<<<grid_of(n_mid), 256, 0, s>>>(n_mid, mu0, mu1);
    SPH_LAUNCH_CHECK();
    k_kd_midrange<<<grid_of(nu), 256, 0, s>>>(nu, units, N, k_mid, mb, mu0, mu1);
    SPH_LAUNCH_CHECK();
    k_kd_rcut<<<grid_of(np), 256, 0, s>>>(np, plist, e_node, o_s, N, k_mid, ka.up_levels, o.h_fact, rcut);
    SPH_LAUNCH_CHECK();
  }
  node_hsolve(ctx, np, plist, nu, upos, a.o_xyz, o_s, o.h_fact, o.eps_h, o.bypass_threshold, a.o_h, a.o_branch,
              bcount, n_mid, mid_com, mu0, mu1, rcut, s);
  unsigned long long bc[4] = {0, 0, 0, 0};
  unsigned long long r2 = 0;
  SPH_HIP(hipMemcpyAsync(bc, bcount, sizeof bc, hipMemcpyDeviceToHost, s));
  SPH_HIP(hipMemcpyAsync(&r2, N.s2, sizeof r2, hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  a.n_out = n_out;
  a.stats.n_nodes = nn;
  a.stats.n_units = nu;
  a.stats.n_pseudo = np;
  a.stats.n_real = n_out - np;
  double r2d;
  std::memcpy(&r2d, &r2, sizeof r2d);
  a.stats.s_root = sqrt(r2d);
  for (int k = 0; k < 4; ++k) a.stats.branch_count[k] = (int64_t)bc[k];
}

}  // namespace sphmap
