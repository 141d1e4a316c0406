// Data layouts shared by the host builder and the gfx950 kernels.
#pragma once
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

}  // namespace gi
