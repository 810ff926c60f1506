// Candidate particle-cell pairs.
//
// A pair (c, i) is a candidate when the canonical binary32 test holds:
//   dx = fl(x_i) - fl(g_x) (same for y, z), d2 = (dx*dx + dy*dy) + dz*dz,
//   s = R_c + 2 fl(h_i), candidate iff d2 < s*s
// with R_c the canonical bounding radius of cell c.  The number of candidate
// pairs is the method's unit of work (the paper's runtime grows with the
// number of particle-cell pairs, Sec. 1).
//
// Search structure: particles sorted by Morton key, grouped 16 at a time into
// a 16-ary hierarchy of boxes that bound the particles' 2h balls (inflated so
// that the box test can never reject a pair the canonical test accepts).
// Smoothing lengths span a factor ~20 in log-normal clouds, so a single
// uniform hash grid would be either overfull in dense regions or hold each
// large-h particle in many buckets; the Morton hierarchy is a uniform grid
// at every level and adapts to both.  One thread per cell walks it, cells in
// Morton order of their sites so that a wave's walks stay coherent.  The walk
// counts every cell's candidates and keeps the first kCap of them in a
// bounded per-cell buffer; after the scan that sizes the CSR, each list that
// fitted is sorted by particle index in LDS and written out, and the few
// longer ones are walked a second time straight into the CSR and sorted.
#include "ballsearch.hpp"

namespace sphmap {
namespace {

__global__ void k_gather_sorted(int64_t n, const int32_t *sidx, const float4 *x32, float4 *sx) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) sx[k] = x32[sidx[k]];
}

// level-1 boxes over groups of kFan sorted particles, each ball inflated by
// 1e-5 relative plus an absolute slack
__global__ void k_leaf_boxes(int64_t n, const float4 *sx, int64_t nb, float4 *lo, float4 *hi, float slack) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  float l0 = INFINITY, l1 = INFINITY, l2 = INFINITY, h0 = -INFINITY, h1 = -INFINITY, h2 = -INFINITY;
  for (int64_t k = b * kFan; k < min(n, (b + 1) * kFan); ++k) {
    float4 p = sx[k];
    float r = 2.0f * p.w * 1.00001f + slack;
    l0 = fminf(l0, p.x - r);
    l1 = fminf(l1, p.y - r);
    l2 = fminf(l2, p.z - r);
    h0 = fmaxf(h0, p.x + r);
    h1 = fmaxf(h1, p.y + r);
    h2 = fmaxf(h2, p.z + r);
  }
  lo[b] = make_float4(l0 - slack, l1 - slack, l2 - slack, 0.0f);
  hi[b] = make_float4(h0 + slack, h1 + slack, h2 + slack, 0.0f);
}

__global__ void k_up_boxes(int64_t nc, const float4 *clo, const float4 *chi, int64_t nb, float4 *lo, float4 *hi) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  float4 l = make_float4(INFINITY, INFINITY, INFINITY, 0.0f), h = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
  for (int64_t k = b * kFan; k < min(nc, (b + 1) * kFan); ++k) {
    float4 a = clo[k], c = chi[k];
    l.x = fminf(l.x, a.x);
    l.y = fminf(l.y, a.y);
    l.z = fminf(l.z, a.z);
    h.x = fmaxf(h.x, c.x);
    h.y = fmaxf(h.y, c.y);
    h.z = fmaxf(h.z, c.z);
  }
  lo[b] = l;
  hi[b] = h;
}

// The canonical binary32 test, evaluated without contraction.
__device__ inline bool canon_pair(const float4 &p, const float4 &g) {
#pragma clang fp contract(off)
  float dx = p.x - g.x, dy = p.y - g.y, dz = p.z - g.z;
  float d2 = (dx * dx + dy * dy) + dz * dz;
  float s = g.w + 2.0f * p.w;
  return d2 < s * s;
}

// Walk modes: kFill writes the list straight into the CSR (offsets known);
// otherwise the first kCap candidates go to the cell's slot of a bounded
// buffer and all are counted.
constexpr int kCap = 512;

// One wavefront per cell.  A step takes up to four hierarchy nodes of one
// level from the top of the wave's LDS stack, and its 64 lanes test their
// 16 children each: boxes that the cell's ball reaches go on the stack,
// balls that pass the canonical test are appended to the cell's list (in
// the order of a ballot; the lists are sorted afterwards).  Taking only
// nodes of the top's level keeps the stack ordered by level with at most
// 64 nodes pending per level, so 64 kMaxLevels entries always suffice.
constexpr int kWalkStack = 64 * kMaxLevels;

// One wavefront per listed cell; the grid's wavefronts step through the
// list (C entries, or *dC when given: a count known only on the device).
// The fill skips a cell whose list would end past `cap` pairs.
template <bool kFill>
__global__ void __launch_bounds__(256) k_pairs(Hier H, int64_t C, const int32_t *cells, const float4 *gen32,
                                              int64_t *counts, const int64_t *off, int32_t *pair_p,
                                              int32_t *pair_c, int32_t *buf, const int32_t *dC = nullptr,
                                              int64_t cap = INT64_MAX) {
  __shared__ uint32_t stk[4][kWalkStack];  // node << 4 | level
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t nt = dC ? (int64_t)*dC : C;
  for (int64_t t = (int64_t)blockIdx.x * 4 + w; t < nt; t += (int64_t)gridDim.x * 4) {
  const int32_t c = cells[t];
  if (kFill && off[c + 1] > cap) continue;  // past the capacity: flagged by the caller
  const float4 g = gen32[c];
  const float rr = g.w * 1.00001f + H.margin_abs;
  const float r2 = rr * rr;
  const int64_t base = kFill ? off[c] : 0;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));  // lanes below this one
  uint32_t *S = stk[w];
  int64_t cnt = 0;
  int sp = 0;
  {
    const int top = H.levels;  // at most kFan nodes
    const bool hit = lane < H.n[top] && box_hit(H.lo[top][lane], H.hi[top][lane], g, r2);
    const uint64_t m = __ballot(hit);
    if (hit) S[__popcll(m & lt)] = ((uint32_t)lane << 4) | (uint32_t)top;
    sp = __popcll(m);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  while (sp > 0) {
    // up to four entries from the top, all of the top entry's level
    const int lvl = (int)(S[sp - 1] & 15u);
    const uint32_t peek = lane < 4 && lane < sp ? S[sp - 1 - lane] : 0u;
    const uint64_t same = __ballot(lane < 4 && lane < sp && (int)(peek & 15u) == lvl);
    const int take = __builtin_ctzll(~same);  // entries from the top of that level
    const int q = lane >> 4, ch = lane & 15;
    const bool act = q < take;
    const uint32_t e = act ? S[sp - 1 - q] : 0u;
    sp -= take;
    const int64_t k = (int64_t)(e >> 4) * kFan + ch;
    bool ball = false, box = false;
    if (act) {
      if (lvl == 1) {
        ball = k < H.n[0] && canon_pair(H.sx[k], g);
      } else {
        const int lc = lvl - 1;
        box = k < H.n[lc] && box_hit(H.lo[lc][k], H.hi[lc][k], g, r2);
      }
    }
    const uint64_t mb = __ballot(ball);
    if (ball) {
      const int64_t pos = cnt + __popcll(mb & lt);
      const int32_t pid = H.sidx[k];
      if (kFill) {
        pair_p[base + pos] = pid;
        pair_c[base + pos] = c;
      } else if (pos < kCap) {
        buf[(int64_t)c * kCap + pos] = pid;
      }
    }
    cnt += __popcll(mb);
    const uint64_t mx = __ballot(box);
    if (box) S[sp + __popcll(mx & lt)] = ((uint32_t)k << 4) | (uint32_t)(lvl - 1);
    sp += __popcll(mx);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if (!kFill && lane == 0) counts[c] = cnt;
  }  // listed cells of this wavefront
}

// Sort each cell's particle list ascending: lists of up to kSortCap entries
// by a bitonic sort in LDS; longer lists (large cells of a mixed set of
// pseudo-particles) as kSortCap-entry runs sorted the same way, then merged
// pairwise by the whole workgroup (merge path: each thread finds where its
// share of the output starts by a binary search and merges it alone),
// ping-ponging with a scratch copy of the list.  Particle indices within a
// list are distinct, so the result does not depend on the method.
constexpr int kSortCap = 4096;

__device__ void sort_run_lds(int32_t *buf, const int32_t *src, int32_t *dst, int n) {
  int m = 2;
  while (m < n) m <<= 1;
  for (int k = threadIdx.x; k < m; k += blockDim.x) buf[k] = k < n ? src[k] : INT32_MAX;
  __syncthreads();
  for (int size = 2; size <= m; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int k = threadIdx.x; k < m; k += blockDim.x) {
        int q = k ^ stride;
        if (q > k) {
          bool up = (k & size) == 0;
          int32_t a = buf[k], b = buf[q];
          if ((a > b) == up) {
            buf[k] = b;
            buf[q] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int k = threadIdx.x; k < n; k += blockDim.x) dst[k] = buf[k];
  __syncthreads();
}

// merge sorted A[0, na) and B[0, nb) into out[0, na + nb), all threads
__device__ void merge_block(const int32_t *A, int na, const int32_t *B, int nb, int32_t *out) {
  const int total = na + nb;
  const int per = (total + blockDim.x - 1) / blockDim.x;
  const int d0 = min((int)threadIdx.x * per, total), d1 = min(d0 + per, total);
  if (d0 >= d1) return;
  // merge path: i elements of A and d0 - i of B come before output d0
  int lo = max(0, d0 - nb), hi = min(d0, na);
  while (lo < hi) {
    const int i = (lo + hi) >> 1;
    if (A[i] < B[d0 - 1 - i]) lo = i + 1;
    else hi = i;
  }
  int i = lo, j = d0 - lo;
  for (int d = d0; d < d1; ++d) {
    if (j >= nb || (i < na && A[i] < B[j])) out[d] = A[i++];
    else out[d] = B[j++];
  }
}

// Bitonic sort of 64 R keys held by one wavefront, key r * 64 + lane in
// v[r]: distances of 64 and more pair registers of the same lane, shorter
// ones pair lanes (an exchange across lanes); no LDS and no barriers.
template <int R>
__device__ inline void wave_bitonic(int32_t (&v)[R], int lane) {
  constexpr int m = 64 * R;
#pragma unroll
  for (int size = 2; size <= m; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= 64) {
        const int rs = stride >> 6;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if ((r & rs) == 0) {
            const bool up = ((r * 64) & size) == 0;
            const int32_t a = v[r], b = v[r | rs];
            v[r] = up ? min(a, b) : max(a, b);
            v[r | rs] = up ? max(a, b) : min(a, b);
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int32_t o = __shfl_xor(v[r], stride, 64);
          const bool up = ((r * 64 + lane) & size) == 0;
          const bool lower = (lane & stride) == 0;
          v[r] = (lower == up) ? min(v[r], o) : max(v[r], o);
        }
      }
    }
  }
}

template <int R>
__device__ inline void wave_sort_copy(const int32_t *src, int32_t *dst, int n, int lane) {
  int32_t v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = r * 64 + lane < n ? src[r * 64 + lane] : INT32_MAX;
  wave_bitonic<R>(v, lane);
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r * 64 + lane < n) dst[r * 64 + lane] = v[r];
}

// Lists that fitted the bounded buffer: each sorted by one wavefront in
// registers and written to the CSR with its cell; the others are listed for
// a second walk.
static_assert(kCap <= 512, "a wavefront sorts at most 8 keys per lane");
__global__ void __launch_bounds__(256) k_compact_sort(int64_t C, const int64_t *off, const int32_t *buf,
                                                      int32_t *pair_p, int32_t *pair_c, int32_t *over,
                                                      int32_t *n_over, int64_t cap = INT64_MAX) {
  const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;  // one cell per wavefront
  const int lane = threadIdx.x & 63;
  if (c >= C) return;
  const int64_t s = off[c];
  if (off[c + 1] > cap) return;  // past the capacity: flagged by the caller
  const int n = (int)(off[c + 1] - s);
  if (n > kCap) {
    if (lane == 0) over[atomicAdd(n_over, 1)] = (int32_t)c;
    return;
  }
  for (int k = lane; k < n; k += 64) pair_c[s + k] = (int32_t)c;
  const int32_t *src = buf + c * kCap;
  if (n <= 64)
    wave_sort_copy<1>(src, pair_p + s, n, lane);
  else if (n <= 128)
    wave_sort_copy<2>(src, pair_p + s, n, lane);
  else if (n <= 256)
    wave_sort_copy<4>(src, pair_p + s, n, lane);
  else
    wave_sort_copy<8>(src, pair_p + s, n, lane);
}

// One workgroup per listed cell (blockIdx.x), or, with a device count dC,
// the grid's workgroups step through the *dC listed cells.
__device__ void sort_segment(const int64_t *off, int32_t *pair_p, int32_t *tmp, int64_t c, int32_t *buf);

__global__ void __launch_bounds__(256) k_sort_segments(int64_t C, const int64_t *off, int32_t *pair_p, int32_t *tmp,
                                                       const int32_t *cells, const int32_t *dC = nullptr,
                                                       int64_t cap = INT64_MAX) {
  __shared__ int32_t buf[kSortCap];
  if (!dC) {
    const int64_t c = cells ? cells[blockIdx.x] : blockIdx.x;
    if (off[c + 1] <= cap) sort_segment(off, pair_p, tmp, c, buf);
    return;
  }
  const int64_t nt = *dC;
  for (int64_t b = blockIdx.x; b < nt; b += gridDim.x) {  // uniform over the workgroup
    const int64_t c = cells[b];
    if (off[c + 1] <= cap) sort_segment(off, pair_p, tmp, c, buf);
    __syncthreads();
  }
}

__device__ void sort_segment(const int64_t *off, int32_t *pair_p, int32_t *tmp, int64_t c, int32_t *buf) {
  const int64_t s = off[c], e = off[c + 1];
  const int n = (int)(e - s);
  if (n <= 1) return;
  int32_t *a = pair_p + s;
  if (n <= kSortCap) {
    sort_run_lds(buf, a, a, n);
    return;
  }
  for (int r0 = 0; r0 < n; r0 += kSortCap) sort_run_lds(buf, a + r0, a + r0, min(kSortCap, n - r0));
  int32_t *src = a, *dst = tmp + s;
  for (int w = kSortCap; w < n; w <<= 1) {
    for (int lo = 0; lo < n; lo += 2 * w) {
      const int mid = min(lo + w, n), hi = min(lo + 2 * w, n);
      merge_block(src + lo, mid - lo, src + mid, hi - mid, dst + lo);
    }
    __syncthreads();
    int32_t *t = src;
    src = dst;
    dst = t;
  }
  if (src != a)
    for (int k = threadIdx.x; k < n; k += blockDim.x) a[k] = src[k];
}

}  // namespace

void build_hier(Arena &ar, const float4 *sx, int64_t n, float slack, const std::string &tag, Hier &H, hipStream_t s) {
  H.n[0] = n;
  H.lo[0] = H.hi[0] = nullptr;
  H.margin_abs = 2.0f * slack;
  int l = 0;
  int64_t cnt = n;
  do {
    ++l;
    SPH_REQUIRE(l <= kMaxLevels, SPHMAP_EINVAL, "too many balls for the search hierarchy");
    int64_t nb = div_up(cnt, kFan);
    H.n[l] = nb;
    H.lo[l] = ar.get<float4>(tag + "_lo" + std::to_string(l), nb);
    H.hi[l] = ar.get<float4>(tag + "_hi" + std::to_string(l), nb);
    if (l == 1)
      k_leaf_boxes<<<(unsigned)div_up(nb, 256), 256, 0, s>>>(n, sx, nb, H.lo[1], H.hi[1], slack);
    else
      k_up_boxes<<<(unsigned)div_up(nb, 256), 256, 0, s>>>(cnt, H.lo[l - 1], H.hi[l - 1], nb, H.lo[l], H.hi[l]);
    SPH_LAUNCH_CHECK();
    cnt = nb;
  } while (cnt > kFan);
  H.levels = l;
}

namespace {

// Capacity mode: the pair count (the scanned total) stays on the device.
// np = total when it fits the capacity, else 0 with the list's overflow bit
// and the plan's flag set; the long-list count starts at 0.
__global__ void k_cap_count(const int64_t *total, int64_t cap, int64_t *np, int32_t *over_bit, int32_t *n_over,
                            int32_t *flag) {
  if (threadIdx.x != 0) return;
  const int64_t tot = *total;
  const bool over = tot > cap;
  *np = over ? 0 : tot;
  *over_bit = over ? 1 : 0;
  *n_over = 0;
  if (over) atomicOr(flag, 1);
}

// An overflowed list is emptied: every cell offset becomes 0.
__global__ void k_zero_if_over(int64_t *off, int64_t n, const int32_t *over_bit) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && *over_bit) off[i] = 0;
}

}  // namespace

// find_pairs with the lists sized for P.cap pairs and no host read of the
// count: cells whose lists would end past the capacity are skipped, and an
// overflowed list is emptied and flagged (P.d_over, *P.d_flag); later steps
// read the count P.d_np.  Nothing is allocated here once the buffers have
// their size, and no buffer is cleared by a memory set, so the work can be
// captured in a graph.
static void find_pairs_capped(Ctx &ctx, const TessDev &t, PairsDev &P, const Hier &H, const int32_t *buf,
                              hipStream_t s) {
  Arena &ar = ctx.arena;
  const int64_t C = t.n_cells;
  P.n_pairs = P.cap;
  P.pair_p = P.mem.get<int32_t>("pair_p", P.cap);
  P.pair_c = P.mem.get<int32_t>("pair_c", P.cap);
  int32_t *over = ar.get<int32_t>("pp_over", std::max<int64_t>(C, 1));
  int32_t *n_over = ar.get<int32_t>("pp_nover", 1);
  k_cap_count<<<1, 64, 0, s>>>(P.cell_off + C, P.cap, P.d_np, P.d_over, n_over, P.d_flag);
  SPH_LAUNCH_CHECK();
  if (C == 0) return;
  k_compact_sort<<<(unsigned)div_up(C, 4), 256, 0, s>>>(C, P.cell_off, buf, P.pair_p, P.pair_c, over, n_over, P.cap);
  SPH_LAUNCH_CHECK();
  // longer lists: the grid steps through however many the device listed
  k_pairs<true><<<(unsigned)std::min<int64_t>(div_up(C, 4), 2048), 256, 0, s>>>(
      H, C, over, t.gen32, nullptr, P.cell_off, P.pair_p, P.pair_c, nullptr, n_over, P.cap);
  SPH_LAUNCH_CHECK();
  int32_t *tmp = ar.get<int32_t>("pp_sort_tmp", P.cap);
  k_sort_segments<<<(unsigned)std::min<int64_t>(C, 1024), 256, 0, s>>>(C, P.cell_off, P.pair_p, tmp, over, n_over,
                                                                        P.cap);
  SPH_LAUNCH_CHECK();
  k_zero_if_over<<<(unsigned)div_up(C + 1, 256), 256, 0, s>>>(P.cell_off, C + 1, P.d_over);
  SPH_LAUNCH_CHECK();
}

void find_pairs(Ctx &ctx, const TessDev &t, const PartDev &p, PairsDev &P, hipStream_t s) {
  Arena &ar = ctx.arena;
  const int64_t N = p.n, C = t.n_cells;
  // Morton order of the particles in the tessellation's bounding cube
  uint64_t *keys = ar.get<uint64_t>("pp_keys", N);
  int32_t *sidx = ar.get<int32_t>("pp_sidx", N);
  morton_keys(p.xyz, 3, N, t.box_lo[0], t.box_lo[1], t.box_lo[2], t.box_size, keys, sidx, s);
  // the top 10 bits per axis order the balls (1024^3 boxes; equal keys keep
  // index order): the hierarchy bounds the balls themselves, so any order
  // gives the same pairs, and half the passes of the full 63-bit key
  radix_sort_u64_range(ar, keys, sidx, N, 33, 63, s);
  float4 *sx = ar.get<float4>("pp_sx", N);
  k_gather_sorted<<<(unsigned)div_up(N, 256), 256, 0, s>>>(N, sidx, p.x32, sx);
  SPH_LAUNCH_CHECK();
  Hier H;
  H.sx = sx;
  H.sidx = sidx;
  const float slack = (float)(1e-6 * t.box_size);
  build_hier(ar, sx, N, slack, "pp", H, s);

  P.n_cells = C;
  P.n_particles = N;
  int64_t *counts = ar.get<int64_t>("pp_counts", C + 1);
  int32_t *buf = ar.get<int32_t>("pp_buf", C * (int64_t)kCap);
  P.cell_off = P.mem.get<int64_t>("cell_off", C + 1);
  // one walk: up to kCap candidates per cell into the bounded buffer, all counted
  {
    KernelTimer kt(&ctx, "pair_count", s);
    k_pairs<false><<<(unsigned)div_up(C, 4), 256, 0, s>>>(H, C, t.cell_order, t.gen32, counts, nullptr, nullptr,
                                                             nullptr, buf);
    SPH_LAUNCH_CHECK();
    kt.done();
  }
  scan_exclusive_i64(ar, counts, P.cell_off, C, true, s);
  if (P.cap > 0) {
    find_pairs_capped(ctx, t, P, H, buf, s);
    return;
  }
  int64_t total = 0;
  SPH_HIP(hipMemcpyAsync(&total, P.cell_off + C, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  SPH_REQUIRE(total < ((int64_t)1 << 31), SPHMAP_EINVAL, "more than 2^31 candidate pairs");
  P.n_pairs = total;
  P.pair_p = P.mem.get<int32_t>("pair_p", total);
  P.pair_c = P.mem.get<int32_t>("pair_c", total);
  if (C == 0) return;
  int32_t *over = ar.get<int32_t>("pp_over", C);
  int32_t *n_over = ar.get<int32_t>("pp_nover", 1);
  SPH_HIP(hipMemsetAsync(n_over, 0, sizeof(int32_t), s));
  {
    KernelTimer kt(&ctx, "pair_fill", s);
    k_compact_sort<<<(unsigned)div_up(C, 4), 256, 0, s>>>(C, P.cell_off, buf, P.pair_p, P.pair_c, over, n_over);
    SPH_LAUNCH_CHECK();
    kt.done();
  }
  int32_t no = 0;
  SPH_HIP(hipMemcpyAsync(&no, n_over, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  if (no > 0) {
    // longer lists: walked again straight into the CSR, then sorted
    KernelTimer kt(&ctx, "pair_fill_long", s);
    k_pairs<true><<<(unsigned)div_up(no, 4), 256, 0, s>>>(H, no, over, t.gen32, nullptr, P.cell_off, P.pair_p,
                                                             P.pair_c, nullptr);
    SPH_LAUNCH_CHECK();
    int32_t *tmp = ar.get<int32_t>("pp_sort_tmp", std::max<int64_t>(total, 1));
    k_sort_segments<<<(unsigned)no, 256, 0, s>>>(C, P.cell_off, P.pair_p, tmp, over);
    SPH_LAUNCH_CHECK();
    kt.done();
  }
}

}  // namespace sphmap
