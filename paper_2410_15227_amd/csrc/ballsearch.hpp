// A 16-ary hierarchy of boxes over Morton-sorted balls, the search structure
// of the candidate-pair search and of the gather from the mixed set.  Level 1
// boxes bound groups of 16 consecutive balls (radius 2h, inflated by 1e-5
// relative plus an absolute slack so that binary32 box tests never reject a
// pair the exact test accepts); each higher level bounds 16 boxes of the
// level below.  The Morton hierarchy is a uniform grid at every level, so it
// adapts both to clustering and to the wide range of smoothing lengths.
#pragma once
#include "common.hpp"

namespace sphmap {

constexpr int kFan = 16;        // children per hierarchy node
constexpr int kMaxLevels = 10;  // 16^10 > 2^31 balls

struct Hier {
  int levels;                 // number of box levels (level 1 = groups of balls)
  int64_t n[kMaxLevels + 1];  // nodes per level (n[0] = balls)
  float4 *lo[kMaxLevels + 1];
  float4 *hi[kMaxLevels + 1];
  const float4 *sx;           // sorted balls: fl(x), fl(y), fl(z), fl(h)
  const int32_t *sidx;        // sorted -> original index
  float margin_abs;           // absolute slack of the box test
};

// squared distance from point g to the box, compared with r2
__device__ inline bool box_hit(const float4 &lo, const float4 &hi, const float4 &g, float r2) {
  float dx = fmaxf(fmaxf(lo.x - g.x, g.x - hi.x), 0.0f);
  float dy = fmaxf(fmaxf(lo.y - g.y, g.y - hi.y), 0.0f);
  float dz = fmaxf(fmaxf(lo.z - g.z, g.z - hi.z), 0.0f);
  return dx * dx + dy * dy + dz * dz <= r2;
}

// Box levels over the n sorted balls sx (arena buffers named after tag);
// fills every field of H but sx and sidx.
void build_hier(Arena &ar, const float4 *sx, int64_t n, float slack, const std::string &tag, Hier &H, hipStream_t s);

}  // namespace sphmap
