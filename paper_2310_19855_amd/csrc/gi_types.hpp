// Data layouts shared by the host builder and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gi {

// One BVH node = one 128-byte cache line: the boxes of its 4 children as structure-of-arrays
// plus 4 child references.  A reference with kLeafBit set is a leaf: triangles
// [first, first + count) of the leaf-ordered triangle array.
struct alignas(128) Node4 {
  float lox[4], hix[4], loy[4], hiy[4], loz[4], hiz[4];
  uint32_t child[4];
  uint32_t pad[4];
};
static_assert(sizeof(Node4) == 128, "node must be one cache line");

constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kLeafCountShift = 24;
constexpr uint32_t kLeafCountMask = 0x7Fu;        // count - 1 in 7 bits (<= 128 triangles)
constexpr uint32_t kLeafFirstMask = 0x00FFFFFFu;  // first triangle < 2^24
constexpr uint32_t kNodeEmpty = 0xFFFFFFFFu;

constexpr uint32_t kBucketSlots = 32;   // world-cache slots per bucket (one 128-byte line of fingerprints)
constexpr uint32_t kStatStripesHost = 64;   // copies of the stats counters (and hit-list stripes)
constexpr int kMaxDyn = 64;
constexpr int kLdsStackEntries = 16;           // traversal-stack entries per lane kept in LDS
constexpr int kNumCells = 64;

// Light grid geometry (Section 2.3.2) from the box of the frame's hit points, kept as
// order-preserving codes of floats (so that integer minima and maxima order them): cubic cells
// of side h = longest extent / G, at most G per axis; an empty box gives one cell of side 1.
struct LightGridGeom {
  float lo[3];
  float h;
  uint32_t dim[3];
};

__host__ __device__ inline uint32_t lg_encode(float f) {
  uint32_t b;
  __builtin_memcpy(&b, &f, 4);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__host__ __device__ inline float lg_decode(uint32_t u) {
  const uint32_t b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
  float f;
  __builtin_memcpy(&f, &b, 4);
  return f;
}

__host__ __device__ inline LightGridGeom light_grid_geom(const uint32_t* box, uint32_t G) {
  LightGridGeom g;
  float lo[3], hi[3];
  bool empty = false;
  for (int k = 0; k < 3; ++k) {
    lo[k] = lg_decode(box[k]);
    hi[k] = lg_decode(box[3 + k]);
    if (!(lo[k] <= hi[k])) empty = true;
  }
  if (empty)
    for (int k = 0; k < 3; ++k) lo[k] = hi[k] = 0.0f;
  float emax = 0.0f;
  for (int k = 0; k < 3; ++k) {
    const float e = hi[k] - lo[k];
    emax = emax > e ? emax : e;
  }
  const float h = emax / (float)G;
  g.h = h > 0.0f ? h : 1.0f;
  for (int k = 0; k < 3; ++k) {
    const float q = -floorf(-((hi[k] - lo[k]) / g.h));
    const uint32_t d = q < 1.0f ? 1u : (uint32_t)q;
    g.dim[k] = d > G ? G : d;
    g.lo[k] = lo[k];
  }
  return g;
}

}  // namespace gi
