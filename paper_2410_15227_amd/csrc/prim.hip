// Device primitives: exclusive scan, stable LSD radix sort, Morton keys.
#include <algorithm>

#include "common.hpp"

namespace sphmap {

void *BlockPool::take(size_t bytes, size_t &got) {
  auto it = blocks.lower_bound(bytes);
  if (it == blocks.end() || it->first / 2 >= bytes) return nullptr;
  void *p = it->second;
  got = it->first;
  held -= got;
  blocks.erase(it);
  return p;
}

void BlockPool::put(void *p, size_t bytes) {
  if (held + bytes > cap) {
    (void)hipFree(p);
    return;
  }
  blocks.emplace(bytes, p);
  held += bytes;
}

void BlockPool::trim() {
  while (held > cap && !blocks.empty()) {
    auto it = std::prev(blocks.end());
    (void)hipFree(it->second);
    held -= it->first;
    blocks.erase(it);
  }
}

void BlockPool::release() {
  for (auto &kv : blocks) (void)hipFree(kv.second);
  blocks.clear();
  held = 0;
}

void *Arena::get(const std::string &name, size_t bytes) {
  if (redirect) return redirect->get(name, bytes);
  Buffer &b = bufs[name];
  if (region) {
    if (b.bytes >= bytes) return b.p;
    const size_t off = (region_used + 255) & ~(size_t)255;
    if (off > region_cap || bytes > region_cap - off)
      throw Error{SPHMAP_EINVAL, "the fixed scratch region of " + std::to_string(region_cap) + " bytes is too small (" +
                                     name + " needs " + std::to_string(bytes) + " more)"};
    b.p = region + off;
    b.bytes = bytes;
    region_used = off + bytes;
    return b.p;
  }
  if (b.bytes < bytes) {
    size_t want = bytes + bytes / 8 + 256;
    if (budget && budget->limit && budget->held - b.bytes + want > budget->limit) {
      budget->required = std::max(budget->required, budget->held - b.bytes + want);
      throw Error{SPHMAP_ENOMEM, "workspace limit of " + std::to_string(budget->limit) + " bytes exceeded by " + name +
                                     " (" + std::to_string(want) + " bytes)"};
    }
    // a block in use may still be read by queued work: hipFree waits for it
    if (b.p) SPH_HIP(hipFree(b.p));
    if (budget) budget->held -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
    if (pool) {
      size_t got = 0;
      if (void *q = pool->take(want, got)) {
        b.p = q;
        b.bytes = got;
        return b.p;
      }
    }
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess && pool && !pool->blocks.empty()) {
      // the kept blocks first go back to the device
      (void)hipGetLastError();
      pool->release();
      e = hipMalloc(&b.p, want);
    }
    if (e != hipSuccess) {
      b.p = nullptr;
      b.bytes = 0;
      (void)hipGetLastError();
      throw Error{SPHMAP_ENOMEM, "device allocation of " + std::to_string(want) + " bytes for " + name + " failed"};
    }
    b.bytes = want;
    if (budget) budget->held += want;
  }
  return b.p;
}

void Arena::release() {
  if (region) {  // carved from a region this arena does not own
    bufs.clear();
    region_used = 0;
    return;
  }
  // pooled blocks are handed out again at once: queued work must be done
  if (pool && !bufs.empty()) (void)hipDeviceSynchronize();
  for (auto &kv : bufs) {
    if (!kv.second.p) continue;
    if (budget) budget->held -= kv.second.bytes;
    if (pool)
      pool->put(kv.second.p, kv.second.bytes);
    else
      (void)hipFree(kv.second.p);
  }
  bufs.clear();
}

namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;

// Block-wide exclusive scan of one value per thread (256 threads, 4 waves).
template <typename T>
__device__ T block_exclusive_scan(T v, T *total) {
  __shared__ T wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wid) off += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const int64_t *in, int64_t n, int64_t *bsum) {
  const int64_t base = (int64_t)blockIdx.x * kTile;
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) s += in[i];
  }
  int64_t tot;
  block_exclusive_scan<int64_t>(s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(const int64_t *in, int64_t *out, int64_t n,
                                                       const int64_t *boff, bool write_total) {
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  int64_t v[kItems];
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + j;
    v[j] = i < n ? in[i] : 0;
    s += v[j];
  }
  int64_t tot;
  int64_t ex = block_exclusive_scan<int64_t>(s, &tot);
  int64_t off = (boff ? boff[blockIdx.x] : 0) + ex;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + j;
    if (i < n) out[i] = off;
    off += v[j];
  }
  if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) out[n] = off;
}

}  // namespace

void scan_exclusive_i64(Arena &ar, const int64_t *in, int64_t *out, int64_t n, bool write_total, hipStream_t s) {
  if (n <= 0) {
    if (write_total) SPH_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
    return;
  }
  int64_t nb = div_up(n, kTile);
  if (nb == 1) {
    k_scan_apply<<<1, kBlock, 0, s>>>(in, out, n, nullptr, write_total);
    SPH_LAUNCH_CHECK();
    return;
  }
  // per-level scratch, named by size so recursion levels do not collide
  std::string tag = "scan_bsum_" + std::to_string(nb);
  int64_t *bsum = ar.get<int64_t>(tag, nb + 1);
  int64_t *boff = ar.get<int64_t>(tag + "_off", nb + 1);
  k_scan_reduce<<<(unsigned)nb, kBlock, 0, s>>>(in, n, bsum);
  SPH_LAUNCH_CHECK();
  scan_exclusive_i64(ar, bsum, boff, nb, false, s);
  k_scan_apply<<<(unsigned)nb, kBlock, 0, s>>>(in, out, n, boff, write_total);
  SPH_LAUNCH_CHECK();
}

// ------------------------------------------------------------ radix sort
namespace {

constexpr int kRadixBits = 4;
constexpr int kBins = 1 << kRadixBits;

template <typename K>
__global__ void __launch_bounds__(kBlock) k_radix_hist(const K *keys, int64_t n, int shift, int64_t *hist,
                                                       int64_t nblocks) {
  __shared__ int cnt[kBins];
  if (threadIdx.x < kBins) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(int)((keys[i] >> shift) & (kBins - 1))], 1);
  }
  __syncthreads();
  if (threadIdx.x < kBins) hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

template <typename K>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const K *kin, const int32_t *vin, K *kout, int32_t *vout,
                                                          int64_t n, int shift, const int64_t *off,
                                                          int64_t nblocks) {
  __shared__ int T[kBins * kBlock];
  const int t = threadIdx.x;
#pragma unroll
  for (int d = 0; d < kBins; ++d) T[d * kBlock + t] = 0;
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)t * kItems;
  K k[kItems];
  int32_t v[kItems];
  int dg[kItems];
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + j;
    if (i < n) {
      k[j] = kin[i];
      v[j] = vin ? vin[i] : (int32_t)i;
      dg[j] = (int)((k[j] >> shift) & (kBins - 1));
      T[dg[j] * kBlock + t] += 1;
    } else {
      dg[j] = -1;
    }
  }
  __syncthreads();
  // exclusive scan of T in digit-major order: thread t owns entries
  // [t*16, t*16+16)
  int loc[kBins];
  int s = 0;
#pragma unroll
  for (int q = 0; q < kBins; ++q) {
    loc[q] = T[t * kBins + q];
    s += loc[q];
  }
  int tot;
  int ex = block_exclusive_scan<int>(s, &tot);
#pragma unroll
  for (int q = 0; q < kBins; ++q) {
    int c = loc[q];
    T[t * kBins + q] = ex;
    ex += c;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    if (dg[j] < 0) continue;
    int d = dg[j];
    int before = 0;
#pragma unroll
    for (int q = 0; q < j; ++q) before += (dg[q] == d);
    int64_t pos = off[(int64_t)d * nblocks + blockIdx.x] + (T[d * kBlock + t] - T[d * kBlock]) + before;
    kout[pos] = k[j];
    vout[pos] = v[j];
  }
}

template <typename K>
__global__ void k_copy_pairs(const K *ks, const int32_t *vs, K *kd, int32_t *vd, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    kd[i] = ks[i];
    vd[i] = vs[i];
  }
}

template <typename K>
void radix_sort_impl(Arena &ar, K *keys, int32_t *vals, int64_t n, int bits, hipStream_t s, const char *tag,
                     int lo = 0) {
  if (n <= 1) return;
  int64_t nb = div_up(n, kTile);
  std::string t(tag);
  K *k2 = ar.get<K>(t + "_k2", n);
  int32_t *v2 = ar.get<int32_t>(t + "_v2", n);
  int64_t *hist = ar.get<int64_t>(t + "_hist", (int64_t)kBins * nb + 1);
  int64_t *off = ar.get<int64_t>(t + "_off", (int64_t)kBins * nb + 1);
  K *ka = keys, *kb = k2;
  int32_t *va = vals, *vb = v2;
  int passes = 0;
  for (int shift = lo; shift < bits; shift += kRadixBits, ++passes) {
    k_radix_hist<K><<<(unsigned)nb, kBlock, 0, s>>>(ka, n, shift, hist, nb);
    SPH_LAUNCH_CHECK();
    scan_exclusive_i64(ar, hist, off, (int64_t)kBins * nb, false, s);
    k_radix_scatter<K><<<(unsigned)nb, kBlock, 0, s>>>(ka, va, kb, vb, n, shift, off, nb);
    SPH_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (passes & 1) {
    k_copy_pairs<K><<<(unsigned)div_up(n, 256), 256, 0, s>>>(ka, va, keys, vals, n);
    SPH_LAUNCH_CHECK();
  }
}

}  // namespace

// ------------------------------------------- stable sort by key, two payloads
// LSD passes of up to 10 key bits.  A tile of 2048 items is split into four
// 512-item runs, one per wavefront, taken 64 at a time in input order; a lane
// finds the lanes that share its digit from one ballot per digit bit, so its
// rank is the running count of the digit in its wave plus the matching lanes
// below it.  The tile is then laid out digit by digit in LDS and written out
// with consecutive threads on consecutive positions of each digit's run.
namespace {

// IT items per thread: 8 (2,048 per tile), or 16 (4,096) for a long sort
// by 9-bit digits -- a digit's runs then average 8 items, as 8-bit digits'
// do in the smaller tile, so the scatter's stores touch half as many lines,
// and the tile's LDS (78 KB) still lets two workgroups share a CU.  Short
// sorts keep the smaller tiles for more workgroups in flight; 10-bit digits
// keep them for their LDS.
constexpr int kSortThreads = 256;
constexpr int64_t kLongSort = (int64_t)1 << 23;  // items from which 4,096-item tiles are used

// Workgroups are dealt to the 8 XCDs in turn; give each XCD a contiguous run
// of tiles, so that neighbouring tiles -- which fill the same output lines
// of each digit -- share one L2.
__device__ inline int64_t xcd_tile(int64_t ntiles) {
  const int64_t b = blockIdx.x, x = b & 7, k = b >> 3;
  const int64_t q = ntiles >> 3, r = ntiles & 7;  // XCD x takes q + (x < r) tiles
  return x * q + (x < r ? x : r) + k;
}

// The item count is n, or *dn when dn is given (a count known only on the
// device, at most n: the launch covers n items' tiles and the tiles past *dn
// count nothing and write nothing).
template <int NB, int IT>
__global__ void __launch_bounds__(kSortThreads) k_kv_hist(const uint32_t *key, int64_t n, const int64_t *dn,
                                                         int shift, int rb, int64_t ntiles, int64_t *hist) {
  constexpr int kTileN = kSortThreads * IT;  // items per tile
  __shared__ unsigned h[NB];
  if (dn) n = *dn;
  const int nd = 1 << rb;
  for (int d = threadIdx.x; d < nd; d += kSortThreads) h[d] = 0;
  __syncthreads();
  // XCD-aware like the scatter: neighbouring tiles write neighbouring counts
  const int64_t tile = xcd_tile(ntiles);
  const int64_t base = tile * kTileN;
  const unsigned mask = (unsigned)nd - 1u;
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const int64_t i = base + (int64_t)j * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < nd; d += kSortThreads) hist[(int64_t)d * ntiles + tile] = h[d];
}

template <int NB, int IT>
__global__ void __launch_bounds__(kSortThreads) k_kv_scatter(const uint32_t *kin, const int32_t *ain,
                                                            const double *bin, int64_t n, const int64_t *dn,
                                                            int shift, int rb, int64_t ntiles, const int64_t *off,
                                                            uint32_t *kout, int32_t *aout, double *bout) {
  constexpr int kTileN = kSortThreads * IT;  // items per tile
  constexpr int kPer = NB / kSortThreads > 0 ? NB / kSortThreads : 1;  // digits per thread
  __shared__ unsigned cnt[4][NB];  // per wave: running count, then the wave's offset
  __shared__ unsigned tex[NB];     // the tile's exclusive offset per digit
  __shared__ int64_t goff[NB];     // output position of the digit's run minus tex
  __shared__ uint32_t sk[kTileN];
  __shared__ int32_t sa[kTileN];
  __shared__ double sbv[kTileN];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int nd = 1 << rb;
  const unsigned mask = (unsigned)nd - 1u;
  for (int d = t; d < nd; d += kSortThreads) cnt[0][d] = cnt[1][d] = cnt[2][d] = cnt[3][d] = 0u;
  __syncthreads();
  const int64_t tile = xcd_tile(ntiles);
  const int64_t tile0 = tile * kTileN;
  if (dn) n = *dn;
  if (tile0 >= n) return;  // a tile past the count (uniform over the workgroup)
  const int64_t wbase = tile0 + (int64_t)w * (kTileN / 4);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes below this one
  uint32_t kk[IT];
  int32_t aa[IT];
  double bb[IT];
  unsigned rk[IT];  // rank within the wave's run | digit << 16; ~0 for no item
  // all of the wave's loads first, so that they are in flight together
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const int64_t i = std::min(wbase + (int64_t)j * 64 + lane, n - 1);  // past n: read, not used
    kk[j] = kin[i];
    aa[j] = ain[i];
    bb[j] = bin[i];
  }
  // rank round by round; a wave's LDS operations complete in order, so the
  // counter a lane reads is the one the previous round's first lane wrote
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const bool valid = wbase + (int64_t)j * 64 + lane < n;
    const unsigned d = (kk[j] >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < rb; ++b) {
      const bool set = (d >> b) & 1u;
      const uint64_t bal = __ballot(set);
      peers &= set ? bal : ~bal;
    }
    const unsigned r = (unsigned)__popcll(peers & lt);
    const unsigned c = valid ? cnt[w][d] : 0u;
    if (valid && r == 0u) cnt[w][d] = c + (unsigned)__popcll(peers);  // the digit's first lane
    rk[j] = valid ? ((c + r) | (d << 16)) : ~0u;
  }
  __syncthreads();
  // per digit: each wave's offset inside the digit's run, the run's length,
  // and an exclusive scan of the lengths over the digits
  unsigned loc[kPer];
  unsigned sum = 0u;
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int d = t * kPer + m;
    loc[m] = 0u;
    if (d < nd) {
      const unsigned c0 = cnt[0][d], c1 = cnt[1][d], c2 = cnt[2][d], c3 = cnt[3][d];
      cnt[0][d] = 0u;
      cnt[1][d] = c0;
      cnt[2][d] = c0 + c1;
      cnt[3][d] = c0 + c1 + c2;
      loc[m] = c0 + c1 + c2 + c3;
      sum += loc[m];
    }
  }
  unsigned tot;
  unsigned ex = block_exclusive_scan<unsigned>(sum, &tot);
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int d = t * kPer + m;
    if (d < nd) {
      tex[d] = ex;
      goff[d] = off[(int64_t)d * ntiles + tile] - (int64_t)ex;
      ex += loc[m];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    if (rk[j] != ~0u) {
      const unsigned d = rk[j] >> 16;
      const unsigned p = tex[d] + cnt[w][d] + (rk[j] & 0xffffu);
      sk[p] = kk[j];
      sa[p] = aa[j];
      sbv[p] = bb[j];
    }
  }
  __syncthreads();
  const int nt = (int)std::min<int64_t>(kTileN, n - tile0);
  for (int p = t; p < nt; p += kSortThreads) {
    const uint32_t k = sk[p];
    const int64_t g = goff[(k >> shift) & mask] + p;
    if (g >= 0 && g < n) {  // always true for a consistent histogram; keeps the store in bounds
      kout[g] = k;
      aout[g] = sa[p];
      bout[g] = sbv[p];
    }
  }
}

template <int NB, int IT>
void kv_pass(Arena &ar, int64_t n, const int64_t *dn, int shift, int rb, const uint32_t *kin, const int32_t *ain,
             const double *bin, uint32_t *kout, int32_t *aout, double *bout, hipStream_t s) {
  constexpr int kTileN = kSortThreads * IT;
  const int64_t ntiles = div_up(n, kTileN);
  const int64_t m = ((int64_t)1 << rb) * ntiles;
  int64_t *hist = ar.get<int64_t>("kv_hist", m + 1);
  int64_t *off = ar.get<int64_t>("kv_off", m + 1);
  k_kv_hist<NB, IT><<<(unsigned)ntiles, kSortThreads, 0, s>>>(kin, n, dn, shift, rb, ntiles, hist);
  SPH_LAUNCH_CHECK();
  scan_exclusive_i64(ar, hist, off, m, false, s);
  k_kv_scatter<NB, IT><<<(unsigned)ntiles, kSortThreads, 0, s>>>(kin, ain, bin, n, dn, shift, rb, ntiles, off, kout,
                                                              aout, bout);
  SPH_LAUNCH_CHECK();
}

}  // namespace

void sort_by_key_kv(Arena &ar, int64_t n, int bits, const uint32_t *kin, const int32_t *ain, const double *bin,
                    uint32_t *kout, int32_t *aout, double *bout, hipStream_t s, const int64_t *dn) {
  if (n <= 0) return;
  SPH_REQUIRE(n < ((int64_t)1 << 31), SPHMAP_EINVAL, "sort length out of range");
  SPH_REQUIRE(bits >= 1 && bits <= 32, SPHMAP_EINVAL, "sort key bits out of range");
  const int passes = (bits + 9) / 10;
  const int rb0 = (bits + passes - 1) / passes;
  uint32_t *kt[2] = {ar.get<uint32_t>("kv_k0", n), passes > 2 ? ar.get<uint32_t>("kv_k1", n) : nullptr};
  int32_t *at[2] = {ar.get<int32_t>("kv_a0", n), passes > 2 ? ar.get<int32_t>("kv_a1", n) : nullptr};
  double *bt[2] = {ar.get<double>("kv_b0", n), passes > 2 ? ar.get<double>("kv_b1", n) : nullptr};
  const uint32_t *ks = kin;
  const int32_t *as = ain;
  const double *bs = bin;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * rb0, rb = std::min(rb0, bits - shift);
    const bool last = p == passes - 1;
    uint32_t *kd = last ? kout : kt[p & 1];
    int32_t *ad = last ? aout : at[p & 1];
    double *bd = last ? bout : bt[p & 1];
    if (rb <= 8)
      kv_pass<256, 8>(ar, n, dn, shift, rb, ks, as, bs, kd, ad, bd, s);
    else if (rb == 9 && n >= kLongSort)
      kv_pass<512, 16>(ar, n, dn, shift, rb, ks, as, bs, kd, ad, bd, s);
    else if (rb == 9)
      kv_pass<512, 8>(ar, n, dn, shift, rb, ks, as, bs, kd, ad, bd, s);
    else
      kv_pass<1024, 8>(ar, n, dn, shift, rb, ks, as, bs, kd, ad, bd, s);
    ks = kd;
    as = ad;
    bs = bd;
  }
}

void radix_sort_u64(Arena &ar, uint64_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s) {
  radix_sort_impl<uint64_t>(ar, keys, vals, n, bits, s, "rs64");
}

void radix_sort_u64_range(Arena &ar, uint64_t *keys, int32_t *vals, int64_t n, int lo, int hi, hipStream_t s) {
  radix_sort_impl<uint64_t>(ar, keys, vals, n, hi, s, "rs64", lo);
}
void radix_sort_u32(Arena &ar, uint32_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s) {
  radix_sort_impl<uint32_t>(ar, keys, vals, n, bits, s, "rs32");
}

// ------------------------------------------------------------ Morton keys
namespace {

__device__ inline uint64_t spread21(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__device__ inline uint64_t quant21(double x, double lo, double size) {
  double q = (x - lo) / size * 2097152.0;
  if (!(q > 0.0)) return 0;
  if (q >= 2097151.0) return 2097151;
  return (uint64_t)q;
}

__global__ void k_morton(const double *xyz, int stride, int64_t n, double lo0, double lo1, double lo2, double size,
                         uint64_t *keys, int32_t *idx) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *p = xyz + (int64_t)stride * i;
  uint64_t qx = quant21(p[0], lo0, size), qy = quant21(p[1], lo1, size), qz = quant21(p[2], lo2, size);
  keys[i] = spread21(qx) | (spread21(qy) << 1) | (spread21(qz) << 2);
  if (idx) idx[i] = (int32_t)i;
}

__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_iota_i32(int32_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

}  // namespace

void morton_keys(const double *xyz, int stride, int64_t n, double lo0, double lo1, double lo2, double size,
                 uint64_t *keys, int32_t *idx, hipStream_t s) {
  if (n <= 0) return;
  k_morton<<<(unsigned)div_up(n, 256), 256, 0, s>>>(xyz, stride, n, lo0, lo1, lo2, size, keys, idx);
  SPH_LAUNCH_CHECK();
}
void fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill_i64<<<(unsigned)div_up(n, 256), 256, 0, s>>>(p, v, n);
  SPH_LAUNCH_CHECK();
}
void iota_i32(int32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_iota_i32<<<(unsigned)div_up(n, 256), 256, 0, s>>>(p, n);
  SPH_LAUNCH_CHECK();
}

}  // namespace sphmap
