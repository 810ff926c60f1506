// Device primitives: exclusive scan, stable LSD radix sort, Morton keys.
#include "common.hpp"

namespace sphmap {

void *Arena::get(const std::string &name, size_t bytes) {
  Buffer &b = bufs[name];
  if (b.bytes < bytes) {
    if (b.p) SPH_HIP(hipFree(b.p));
    b.p = nullptr;
    size_t want = bytes + bytes / 8 + 256;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
      b.p = nullptr;
      b.bytes = 0;
      (void)hipGetLastError();
      throw Error{SPHMAP_ENOMEM, "device allocation of " + std::to_string(want) + " bytes for " + name + " failed"};
    }
    b.bytes = want;
  }
  return b.p;
}

void Arena::release() {
  for (auto &kv : bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
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
void radix_sort_impl(Arena &ar, K *keys, int32_t *vals, int64_t n, int bits, hipStream_t s, const char *tag) {
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
  for (int shift = 0; shift < bits; shift += kRadixBits, ++passes) {
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

void radix_sort_u64(Arena &ar, uint64_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s) {
  radix_sort_impl<uint64_t>(ar, keys, vals, n, bits, s, "rs64");
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
