// Device-side building blocks of the GI pass for gfx950: counter-based random numbers, the
// two world-cache hashes, trig-free direction sampling, watertight ray/triangle tests and a
// 4-wide BVH walk with an LDS stack.
//
// Numerics: every float result that decides an integer (hit triangle, hit distance, cell key,
// hemisphere cell, fixed-point sample) follows one written float32 operation order with no
// contraction (built with -ffp-contract=off, correctly rounded division and square root,
// denormals kept).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gi.h"
#include "gi_types.hpp"

namespace gi {

constexpr uint32_t kMiss = 0xFFFFFFFFu;
constexpr uint32_t kSentinel = 0xFFFFFFFFu;
constexpr uint32_t kBucket = kBucketSlots;

// ---- hashes (Section 2.2.1 names two fast hash functions from Jarzynski and Olano 2020) ----
__device__ __host__ inline uint32_t hash_pcg(uint32_t v) {
  const uint32_t s = v * 747796405u + 2891336453u;
  const uint32_t w = ((s >> ((s >> 28u) + 4u)) ^ s) * 277803737u;
  return (w >> 22u) ^ w;
}

// XXH32 of the four little-endian bytes of v, seed 0
__device__ __host__ inline uint32_t hash_xxh32(uint32_t v) {
  uint32_t h = 374761393u + 4u + v * 3266489917u;
  h = ((h << 17) | (h >> 15)) * 668265263u;
  h = (h ^ (h >> 15)) * 2246822519u;
  h = (h ^ (h >> 13)) * 3266489917u;
  return h ^ (h >> 16);
}

__device__ inline uint32_t rand_u32(uint32_t seed, uint32_t frame, uint32_t id, uint32_t dim) {
  return hash_pcg(dim + hash_pcg(id + hash_pcg(frame + hash_pcg(seed))));
}

__device__ inline float rand_unit(uint32_t h) { return (float)(h >> 8) * 5.9604644775390625e-08f; }
__host__ inline float rand_unit_host(uint32_t h) { return (float)(h >> 8) * 5.9604644775390625e-08f; }

// ---- cos/sin(2 pi u): exact octant reduction, Taylor polynomials (1/n!) on [0, pi/4] ----
__device__ inline void cos_sin_2pi(float u, float& co, float& si) {
  const float v = u * 8.0f;
  const int k = (int)v;
  const float fr = v - (float)k;
  const float g = (k & 1) ? (1.0f - fr) : fr;
  const float x = g * 0.785398163397448310f;
  const float x2 = x * x;
  const float s = x * (1.0f + x2 * (-0.166666666666666667f + x2 * (0.00833333333333333333f +
                  x2 * (-0.000198412698412698413f + x2 * 2.75573192239858907e-06f))));
  const float c = 1.0f + x2 * (-0.5f + x2 * (0.0416666666666666667f + x2 * (-0.00138888888888888889f +
                  x2 * (2.48015873015873016e-05f + x2 * -2.75573192239858907e-07f))));
  // rotate (c, s) into octant k: the even octants use phi = fr*pi/4, the odd ones the
  // complement (1 - fr)*pi/4 of the next quarter turn
  const int q = k & 7;
  const float a = (q == 0 || q == 3 || q == 4 || q == 7) ? c : s;   // |cos| source
  const float b = (q == 0 || q == 3 || q == 4 || q == 7) ? s : c;   // |sin| source
  co = (q >= 2 && q <= 5) ? -a : a;
  si = (q >= 4) ? -b : b;
}

// ---- orthonormal basis around a unit normal (Duff et al. 2017) ----
struct Basis { float tx, ty, tz, bx, by, bz; };

__device__ inline Basis make_basis(float nx, float ny, float nz) {
  const float sg = nz >= 0.0f ? 1.0f : -1.0f;
  const float a = -1.0f / (sg + nz);
  const float b = (nx * ny) * a;
  Basis r;
  r.tx = 1.0f + ((sg * nx) * nx) * a;
  r.ty = sg * b;
  r.tz = -(sg * nx);
  r.bx = b;
  r.by = sg + (ny * ny) * a;
  r.bz = -ny;
  return r;
}

// cosine-distributed direction about n (unit) and the 8x8 hemi-octahedral atlas cell of its
// local coordinates (Section 2.1: octahedral mapping of the oriented hemisphere)
__device__ inline void cosine_direction(float nx, float ny, float nz, float u0, float u1,
                                        float& dx, float& dy, float& dz, uint32_t& cell) {
  float c, s;
  cos_sin_2pi(u1, c, s);
  const float r = sqrtf(u0);
  const float lx = r * c, ly = r * s;
  const float lz = sqrtf(fmaxf(0.0f, 1.0f - u0));
  const Basis B = make_basis(nx, ny, nz);
  dx = (lx * B.tx + ly * B.bx) + lz * nx;
  dy = (lx * B.ty + ly * B.by) + lz * ny;
  dz = (lx * B.tz + ly * B.bz) + lz * nz;
  const float sum = (fabsf(lx) + fabsf(ly)) + lz;
  const float a = lx / sum, b = ly / sum;
  int ix = (int)floorf(4.0f * ((a + b) + 1.0f));
  int iy = (int)floorf(4.0f * ((a - b) + 1.0f));
  ix = ix < 0 ? 0 : (ix > 7 ? 7 : ix);
  iy = iy < 0 ? 0 : (iy > 7 ? 7 : iy);
  cell = (uint32_t)(8 * iy + ix);
}

// normalised centre of hemi-octahedral cell `cell` in the frame about n
__device__ inline void cell_centre_direction(uint32_t cell, float nx, float ny, float nz, float& dx, float& dy,
                                             float& dz) {
  const float u = (float)(2 * (cell & 7u) + 1) / 8.0f - 1.0f;
  const float v = (float)(2 * (cell >> 3) + 1) / 8.0f - 1.0f;
  const float a = (u + v) * 0.5f, b = (u - v) * 0.5f;
  const float z = (1.0f - fabsf(a)) - fabsf(b);
  const float len = sqrtf((a * a + b * b) + z * z);
  const float lx = a / len, ly = b / len, lz = z / len;
  const Basis B = make_basis(nx, ny, nz);
  dx = (lx * B.tx + ly * B.bx) + lz * nx;
  dy = (lx * B.ty + ly * B.by) + lz * ny;
  dz = (lx * B.tz + ly * B.bz) + lz * nz;
}

// the atlas cell of a local direction (lx, ly, lz >= 0), not necessarily unit
__device__ inline uint32_t local_cell(float lx, float ly, float lz) {
  const float sum = (fabsf(lx) + fabsf(ly)) + lz;
  const float a = lx / sum, b = ly / sum;
  int ix = (int)floorf(4.0f * ((a + b) + 1.0f));
  int iy = (int)floorf(4.0f * ((a - b) + 1.0f));
  ix = ix < 0 ? 0 : (ix > 7 ? 7 : ix);
  iy = iy < 0 ? 0 : (iy > 7 ? 7 : iy);
  return (uint32_t)(8 * iy + ix);
}

// ray guiding: the direction of the point (u0, u1) of atlas cell k's square in the
// hemi-octahedral domain, about n
__device__ inline void guided_direction(float nx, float ny, float nz, uint32_t k, float u0, float u1, float& dx,
                                        float& dy, float& dz) {
  const float uu = ((float)(k & 7u) + u0) * 0.25f - 1.0f;
  const float vv = ((float)(k >> 3) + u1) * 0.25f - 1.0f;
  const float a = (uu + vv) * 0.5f, b = (uu - vv) * 0.5f;
  const float z = (1.0f - fabsf(a)) - fabsf(b);
  const float len = sqrtf((a * a + b * b) + z * z);
  const float lx = a / len, ly = b / len, lz = z / len;
  const Basis B = make_basis(nx, ny, nz);
  dx = (lx * B.tx + ly * B.bx) + lz * nx;
  dy = (lx * B.ty + ly * B.by) + lz * ny;
  dz = (lx * B.tz + ly * B.bz) + lz * nz;
}

__device__ inline float origin_offset(float scale, float px, float py, float pz) {
  const float m = fmaxf(fmaxf(fabsf(px), fabsf(py)), fabsf(pz));
  return scale * (1.0f + m);
}

// ---- world-cache descriptor (Section 2.2.1, 2.2.2) ----
// Level of detail: the cell size is the base size times 2^lod, the smallest power of two
// (lod <= 7) with 2^lod >= lod_scale * d * S, d the distance from the camera; 0 when lod_scale
// is 0.  Doubling in a loop keeps the decision exact.
__device__ inline uint32_t cell_lod(float S, float lod_scale, float cx, float cy, float cz, float yx, float yy,
                                    float yz) {
  if (!(lod_scale > 0.0f)) return 0u;
  const float dx = yx - cx, dy = yy - cy, dz = yz - cz;
  const float d = sqrtf((dx * dx + dy * dy) + dz * dz);
  const float x = (lod_scale * d) * S;
  uint32_t lod = 0;
  float p = 1.0f;
  while (p < x && lod < 7u) {
    p = p * 2.0f;
    ++lod;
  }
  return lod;
}

// Two-level cache (Section 2.2.3): with `tiled` the descriptor names a tile of 8x8x8 cells
// (quantised position >> 3, a floor division) and `tcell` is the hit's 2D cell inside it:
// 8 (v & 7) + (u & 7), u and v the quantised coordinates along the two axes other than the
// main axis of the normal class, u the lower-numbered one.
__device__ inline uint64_t descriptor(float S0, uint32_t leak_on, float lod_scale, float cx, float cy, float cz,
                                      float yx, float yy, float yz, float nx, float ny, float nz, float t,
                                      bool with_leak, uint32_t tiled, uint32_t& tcell) {
  const uint32_t lod = cell_lod(S0, lod_scale, cx, cy, cz, yx, yy, yz);
  const float S = S0 * (1.0f / (float)(1u << lod));
  int32_t qx = (int32_t)floorf(yx * S);
  int32_t qy = (int32_t)floorf(yy * S);
  int32_t qz = (int32_t)floorf(yz * S);
  const float ax = fabsf(nx), ay = fabsf(ny), az = fabsf(nz);
  uint32_t axis = 0;
  float best = ax;
  float comp = nx;
  if (ay > best) { axis = 1; best = ay; comp = ny; }
  if (az > best) { axis = 2; comp = nz; }
  tcell = 0u;
  if (tiled) {
    const int32_t u = axis == 0u ? qy : qx, v = axis == 2u ? qy : qz;
    tcell = 8u * (uint32_t)(v & 7) + (uint32_t)(u & 7);
    qx >>= 3;
    qy >>= 3;
    qz >>= 3;
  }
  const uint64_t cls = 2u * axis + (comp < 0.0f ? 1u : 0u);
  const uint64_t leak = (with_leak && leak_on && t * S < 1.0f) ? 1u : 0u;
  return ((uint64_t)((uint32_t)qx & 0x3FFFFu)) | ((uint64_t)((uint32_t)qy & 0x3FFFFu) << 18) |
         ((uint64_t)((uint32_t)qz & 0x3FFFFu) << 36) | (cls << 54) | (leak << 57) | ((uint64_t)lod << 58);
}

__device__ inline uint32_t bucket_of(uint64_t key, uint32_t bucket_mask) {
  return hash_pcg((uint32_t)key + hash_pcg((uint32_t)(key >> 32))) & bucket_mask;
}

__device__ inline uint32_t fingerprint_of(uint64_t key) {
  const uint32_t h = hash_xxh32((uint32_t)key + hash_xxh32((uint32_t)(key >> 32)));
  return h == 0u ? 1u : h;
}

// ---- rays ----
struct RayQ {
  float ox, oy, oz;
  float dx, dy, dz;
  float ix, iy, iz;       // conservative inverse direction
  int kx, ky, kz;
  float sx, sy, sz;       // watertight shear
};

__device__ inline float sel3(float a, float b, float c, int k) { return k == 0 ? a : (k == 1 ? b : c); }

__device__ inline float safe_inv(float d) {
  float dd = d;
  if (fabsf(dd) < 1e-30f) dd = dd < 0.0f ? -1e-30f : 1e-30f;
  return 1.0f / dd;
}

__device__ inline RayQ make_ray(float ox, float oy, float oz, float dx, float dy, float dz) {
  RayQ r;
  r.ox = ox; r.oy = oy; r.oz = oz;
  r.dx = dx; r.dy = dy; r.dz = dz;
  r.ix = safe_inv(dx); r.iy = safe_inv(dy); r.iz = safe_inv(dz);
  int kz = 0;
  if (fabsf(dy) > fabsf(dx)) kz = 1;
  if (fabsf(dz) > fabsf(sel3(dx, dy, dz, kz))) kz = 2;
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  if (sel3(dx, dy, dz, kz) < 0.0f) { const int t = kx; kx = ky; ky = t; }
  r.kx = kx; r.ky = ky; r.kz = kz;
  const float dkz = sel3(dx, dy, dz, kz);
  r.sx = sel3(dx, dy, dz, kx) / dkz;
  r.sy = sel3(dx, dy, dz, ky) / dkz;
  r.sz = 1.0f / dkz;
  return r;
}

// watertight two-sided triangle test (Woop, Benthin and Wald 2013); hit if 0 < t < tmax
__device__ inline bool hit_triangle(const RayQ& r, float4 v0, float4 v1, float4 v2, float tmax, float& t_out) {
  const float Ax_ = v0.x - r.ox, Ay_ = v0.y - r.oy, Az_ = v0.z - r.oz;
  const float Bx_ = v1.x - r.ox, By_ = v1.y - r.oy, Bz_ = v1.z - r.oz;
  const float Cx_ = v2.x - r.ox, Cy_ = v2.y - r.oy, Cz_ = v2.z - r.oz;
  const float Akz = sel3(Ax_, Ay_, Az_, r.kz), Bkz = sel3(Bx_, By_, Bz_, r.kz), Ckz = sel3(Cx_, Cy_, Cz_, r.kz);
  const float ax = sel3(Ax_, Ay_, Az_, r.kx) - r.sx * Akz;
  const float ay = sel3(Ax_, Ay_, Az_, r.ky) - r.sy * Akz;
  const float bx = sel3(Bx_, By_, Bz_, r.kx) - r.sx * Bkz;
  const float by = sel3(Bx_, By_, Bz_, r.ky) - r.sy * Bkz;
  const float cx = sel3(Cx_, Cy_, Cz_, r.kx) - r.sx * Ckz;
  const float cy = sel3(Cx_, Cy_, Cz_, r.ky) - r.sy * Ckz;
  float U = cx * by - cy * bx;
  float V = ax * cy - ay * cx;
  float W = bx * ay - by * ax;
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    U = (float)((double)cx * (double)by - (double)cy * (double)bx);
    V = (float)((double)ax * (double)cy - (double)ay * (double)cx);
    W = (float)((double)bx * (double)ay - (double)by * (double)ax);
  }
  if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
  const float det = U + V + W;
  if (det == 0.0f) return false;
  const float T = U * (r.sz * Akz) + V * (r.sz * Bkz) + W * (r.sz * Ckz);
  const float t = T / det;
  if (!(t > 0.0f) || !(t < tmax)) return false;
  t_out = t;
  return true;
}

// conservative entry distance of the 4 children of a node; returns a 4-bit mask of children
// whose box the ray enters at or before tcull
__device__ inline uint32_t enter_children(const RayQ& r, const Node4& n, float tcull, float tn_out[4]) {
  uint32_t mask = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float t0x = (n.lox[c] - r.ox) * r.ix, t1x = (n.hix[c] - r.ox) * r.ix;
    float t0y = (n.loy[c] - r.oy) * r.iy, t1y = (n.hiy[c] - r.oy) * r.iy;
    float t0z = (n.loz[c] - r.oz) * r.iz, t1z = (n.hiz[c] - r.oz) * r.iz;
    const float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
    const float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z)) * 1.0000153f;
    tn_out[c] = tn;
    if (n.child[c] != kNodeEmpty && tn <= tf && tn <= tcull) mask |= 1u << c;
  }
  return mask;
}

struct SceneView {
  const Node4* nodes;
  const float4* tris;       // [3 * leaf-ordered triangles]; v0.w = triangle index bits
  const float4* dyn;        // [3 * n_dyn]
  uint32_t n_dyn;
  uint32_t has_bvh;
  uint32_t* spill;          // traversal-stack spill array [rows][spill_stride]
  uint32_t spill_stride;    // lane ids per row
};

// Traversal stack of one lane.  The top K entries live in LDS (column `lane` of a [K][BLOCK]
// array, K a power of two); when a push finds them all live, the oldest one moves to a
// per-lane global array laid out [depth][lane] (coalesced across a wave), and a pop below what
// LDS holds reads it back.  Live entries [lo, sp) are in LDS, [0, lo) in the spill array.
// Beside each LDS entry sits the upper half of its entry distance's float bits (a value at or
// below the distance); spilled entries carry 0.
template <int K, int BLOCK>
struct TStack {
  // the LDS part is a ring indexed with & (K - 1)
  static_assert(K > 0 && (K & (K - 1)) == 0, "the LDS stack holds a power-of-two number of entries");
  uint32_t* lds;      // &lds_array[lane]
  uint16_t* tlds;     // &lds_distance_array[lane]
  uint32_t* spill;    // &spill_array[lane id]; entry i at spill[i * stride]
  uint32_t stride;
  int sp, lo;
  __device__ TStack(uint32_t* l, uint16_t* tl, uint32_t* s, uint32_t st)
      : lds(l), tlds(tl), spill(s), stride(st), sp(0), lo(0) {}
  __device__ void reset() { sp = 0; lo = 0; }
  __device__ void push(uint32_t v, float t = 0.0f) {
    if (sp - lo == K) {
      spill[(size_t)lo * stride] = lds[(lo & (K - 1)) * BLOCK];
      ++lo;
    }
    lds[(sp & (K - 1)) * BLOCK] = v;
    tlds[(sp & (K - 1)) * BLOCK] = (uint16_t)(__float_as_uint(t) >> 16);
    ++sp;
  }
  __device__ uint32_t pop() {
    --sp;
    if (sp >= lo) return lds[(sp & (K - 1)) * BLOCK];
    lo = sp;
    return spill[(size_t)sp * stride];
  }
  // pop with the entry's distance bound (0 for an entry read back from the spill array)
  __device__ uint32_t pop(float& t) {
    --sp;
    if (sp >= lo) {
      t = __uint_as_float((uint32_t)tlds[(sp & (K - 1)) * BLOCK] << 16);
      return lds[(sp & (K - 1)) * BLOCK];
    }
    lo = sp;
    t = 0.0f;
    return spill[(size_t)sp * stride];
  }
  __device__ bool empty() const { return sp == 0; }
};

// ---- closest-hit BVH walks ----
// Both visit every node whose box the ray enters at or before the best hit found so far (with
// the conservative margins), so both return the same (t, triangle) minimum.

// nearest-first order of the entered children; pushes the farther ones with their entry
// distance and returns the nearest (kNodeEmpty when none is entered)
template <int K, int BLOCK>
__device__ inline uint32_t visit_node(const Node4& n, const RayQ& r, float tcull, TStack<K, BLOCK>& stk) {
  float tn[4];
  const uint32_t m = enter_children(r, n, tcull, tn);
  // 5-exchange sorting network held in registers (children not entered sort last, t = +inf)
  float t0 = (m & 1u) ? tn[0] : __builtin_inff(), t1 = (m & 2u) ? tn[1] : __builtin_inff();
  float t2 = (m & 4u) ? tn[2] : __builtin_inff(), t3 = (m & 8u) ? tn[3] : __builtin_inff();
  uint32_t c0 = n.child[0], c1 = n.child[1], c2 = n.child[2], c3 = n.child[3];
  auto cswap = [](float& ta, uint32_t& ca, float& tb, uint32_t& cb) {
    const bool sw = tb < ta;
    const float tt = sw ? tb : ta;
    tb = sw ? ta : tb;
    ta = tt;
    const uint32_t cc = sw ? cb : ca;
    cb = sw ? ca : cb;
    ca = cc;
  };
  cswap(t0, c0, t1, c1);
  cswap(t2, c2, t3, c3);
  cswap(t0, c0, t2, c2);
  cswap(t1, c1, t3, c3);
  cswap(t1, c1, t2, c2);
  const int cnt = __builtin_popcount(m);
  if (cnt > 3) stk.push(c3, t3);
  if (cnt > 2) stk.push(c2, t2);
  if (cnt > 1) stk.push(c1, t1);
  return cnt > 0 ? c0 : kNodeEmpty;
}

// next stack entry whose box may still hold a better hit: an entry whose box starts beyond
// tcull is dropped without reading its node (its distance bound is at or below its entry
// distance); kNodeEmpty once the stack is empty
template <int K, int BLOCK>
__device__ inline uint32_t next_entry(TStack<K, BLOCK>& stk, float tcull) {
  while (!stk.empty()) {
    float te;
    const uint32_t nx = stk.pop(te);
    if (te <= tcull) return nx;
  }
  return kNodeEmpty;
}

template <bool COUNT>
__device__ inline void test_leaf(const SceneView& sv, const RayQ& r, float tmax, uint32_t leaf, uint32_t& best,
                                 float& best_t, uint32_t* n_tris) {
  const uint32_t first = leaf & kLeafFirstMask;
  const uint32_t count = ((leaf >> kLeafCountShift) & kLeafCountMask) + 1u;
  if (COUNT) *n_tris += count;
  for (uint32_t i = 0; i < count; ++i) {
    const float4 a = sv.tris[3 * (first + i)], b = sv.tris[3 * (first + i) + 1], c = sv.tris[3 * (first + i) + 2];
    float t;
    if (hit_triangle(r, a, b, c, tmax, t)) {
      const uint32_t id = __float_as_uint(a.w);
      if (t < best_t || (t == best_t && id < best)) { best_t = t; best = id; }
    }
  }
}

// one node or one leaf per step
template <int K, int BLOCK, bool COUNT>
__device__ inline void walk_closest(const SceneView& sv, const RayQ& r, float tmax, TStack<K, BLOCK>& stk,
                                    uint32_t& best, float& best_t, uint32_t* n_nodes, uint32_t* n_tris) {
  stk.reset();
  uint32_t cur = 0;   // root is always an inner node
  while (cur != kNodeEmpty) {
    if (!(cur & kLeafBit)) {
      if (COUNT) ++*n_nodes;
      cur = visit_node(sv.nodes[cur], r, best_t * 1.0001221f, stk);
      if (cur != kNodeEmpty) continue;
    } else {
      test_leaf<COUNT>(sv, r, tmax, cur, best, best_t, n_tris);
    }
    cur = next_entry(stk, best_t * 1.0001221f);
  }
}

// Closest hit: lexicographic minimum of (t, triangle index) over every triangle; the BVH walk
// only prunes boxes that cannot hold a better hit.
template <int K, int BLOCK, bool COUNT = false>
__device__ inline void closest_hit(const SceneView& sv, const RayQ& r, float tmax, TStack<K, BLOCK>& stk,
                                   uint32_t& tri_out, float& t_out, uint32_t* n_nodes = nullptr,
                                   uint32_t* n_tris = nullptr) {
  float best_t = tmax;
  uint32_t best = kMiss;
  for (uint32_t k = 0; k < sv.n_dyn; ++k) {
    const float4 a = sv.dyn[3 * k], b = sv.dyn[3 * k + 1], c = sv.dyn[3 * k + 2];
    float t;
    if (hit_triangle(r, a, b, c, tmax, t)) {
      const uint32_t id = __float_as_uint(a.w);
      if (t < best_t || (t == best_t && id < best)) { best_t = t; best = id; }
    }
  }
  if (sv.has_bvh) walk_closest<K, BLOCK, COUNT>(sv, r, tmax, stk, best, best_t, n_nodes, n_tris);
  tri_out = best;
  t_out = best == kMiss ? 0.0f : best_t;
}

// Any hit in (0, tmax)
template <int K, int BLOCK, bool COUNT = false>
__device__ inline bool any_hit(const SceneView& sv, const RayQ& r, float tmax, TStack<K, BLOCK>& stk,
                               uint32_t* n_nodes = nullptr, uint32_t* n_tris = nullptr) {
  for (uint32_t k = 0; k < sv.n_dyn; ++k) {
    float t;
    if (hit_triangle(r, sv.dyn[3 * k], sv.dyn[3 * k + 1], sv.dyn[3 * k + 2], tmax, t)) return true;
  }
  if (!sv.has_bvh) return false;
  const float tcull = tmax * 1.0001221f;
  stk.reset();
  uint32_t cur = 0;
  while (true) {
    if (!(cur & kLeafBit)) {
      const Node4 n = sv.nodes[cur];
      if (COUNT) ++*n_nodes;
      float tn[4];
      uint32_t m = enter_children(r, n, tcull, tn);
      if (m) {
        // nearest entered child first (occluders near the ray's origin end the walk early),
        // the others pushed farthest first; 5-exchange sorting network in registers
        float t0 = (m & 1u) ? tn[0] : __builtin_inff(), t1 = (m & 2u) ? tn[1] : __builtin_inff();
        float t2 = (m & 4u) ? tn[2] : __builtin_inff(), t3 = (m & 8u) ? tn[3] : __builtin_inff();
        uint32_t c0 = n.child[0], c1 = n.child[1], c2 = n.child[2], c3 = n.child[3];
        auto cswap = [](float& ta, uint32_t& ca, float& tb, uint32_t& cb) {
          const bool sw = tb < ta;
          const float tt = sw ? tb : ta;
          tb = sw ? ta : tb;
          ta = tt;
          const uint32_t cc = sw ? cb : ca;
          cb = sw ? ca : cb;
          ca = cc;
        };
        cswap(t0, c0, t1, c1);
        cswap(t2, c2, t3, c3);
        cswap(t0, c0, t2, c2);
        cswap(t1, c1, t3, c3);
        cswap(t1, c1, t2, c2);
        const int cnt = __builtin_popcount(m);
        if (cnt > 3) stk.push(c3);
        if (cnt > 2) stk.push(c2);
        if (cnt > 1) stk.push(c1);
        cur = c0;
        continue;
      }
    } else {
      const uint32_t first = cur & kLeafFirstMask;
      const uint32_t count = ((cur >> kLeafCountShift) & kLeafCountMask) + 1u;
      if (COUNT) *n_tris += count;
      for (uint32_t i = 0; i < count; ++i) {
        float t;
        if (hit_triangle(r, sv.tris[3 * (first + i)], sv.tris[3 * (first + i) + 1], sv.tris[3 * (first + i) + 2], tmax, t))
          return true;
      }
    }
    if (stk.empty()) break;
    cur = stk.pop();
  }
  return false;
}

// ---- wave helpers ----
__device__ inline uint32_t wave_popc(bool pred) { return (uint32_t)__popcll(__ballot(pred)); }

// Counters are striped over kStatStripes copies (chosen by block) so that concurrent waves do
// not serialise on one address; the host sums the stripes.
constexpr uint32_t kStatStripes = 64;

__device__ inline void stat_add(unsigned long long* stats, int idx, bool pred) {
  const uint64_t m = __ballot(pred);
  if (m != 0 && (threadIdx.x & 63u) == (uint32_t)__ffsll((long long)__ballot(1)) - 1u)
    atomicAdd(&stats[(blockIdx.x % kStatStripes) * GI_STAT_COUNT + idx], (unsigned long long)__popcll(m));
}

// lanes below this one in the wave
__device__ inline uint64_t lanes_below() { return (1ull << (threadIdx.x & 63u)) - 1ull; }

}  // namespace gi
