// gfx950 kernels of the per-frame GI pass (plain world cache) and their launchers.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "gi_device.hpp"
#include "gi_host.hpp"

namespace gi {

constexpr int kTraceBlock = 64;   // one wave per block: the LDS part of the stack is [K][64]
constexpr int kLdsStack = kLdsStackEntries;   // traversal-stack entries per lane in LDS (the rest spill)

// orders the LDS accesses of one wave (a block barrier is not needed when no other wave of the
// block reads them)
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct ShadeTables {
  const float4* tnrm;    // unit normal, w = material index bits
  const float4* mats;    // [2m] albedo, [2m+1] emission
  const uint32_t* etri;
  const uint32_t* ethr;
  const float4* evert;   // [3 * n_emit] emitter vertices in emitter order (first w: area)
  uint32_t n_emit;
  float area_total;
  // light grid (config light_grid; null list = area-proportional sampling)
  const uint32_t* lg_box;
  const uint32_t* lg_list;
  const uint32_t* lg_count;
  uint32_t lg_dim, lg_k, ris_m;
};

// ------------------------------------------------------------------------------------------
// G-buffer: one primary ray through each pixel centre (test input)
// ------------------------------------------------------------------------------------------
template <int STACK>
__global__ __launch_bounds__(kTraceBlock) void k_gbuffer(SceneView sv, ShadeTables st, gi_frame f, uint32_t W,
                                                         uint32_t H, float4* pos, float4* nrm, float4* alb,
                                                         uint32_t* prim) {
  __shared__ uint32_t stk[STACK * kTraceBlock];
  __shared__ uint16_t stkt[STACK * kTraceBlock];
  TStack<STACK, kTraceBlock> ts(stk + threadIdx.x, stkt + threadIdx.x, sv.spill + (blockIdx.x * kTraceBlock + threadIdx.x), sv.spill_stride);
  const uint32_t i = blockIdx.x * kTraceBlock + threadIdx.x;
  if (i >= W * H) return;
  const uint32_t x = i % W, y = i / W;
  const float aspect = (float)W / (float)H;
  const float sx = (2.0f * ((float)x + 0.5f)) / (float)W - 1.0f;
  const float sy = 1.0f - (2.0f * ((float)y + 0.5f)) / (float)H;
  const float a = (sx * f.tan_half) * aspect;
  const float b = sy * f.tan_half;
  float dx = (f.fwd[0] + a * f.right[0]) + b * f.up[0];
  float dy = (f.fwd[1] + a * f.right[1]) + b * f.up[1];
  float dz = (f.fwd[2] + a * f.right[2]) + b * f.up[2];
  const float len = sqrtf((dx * dx + dy * dy) + dz * dz);
  dx = dx / len; dy = dy / len; dz = dz / len;
  const RayQ r = make_ray(f.pos[0], f.pos[1], f.pos[2], dx, dy, dz);
  uint32_t tri;
  float t;
  closest_hit<STACK, kTraceBlock>(sv, r, 3.0e38f, ts, tri, t);
  prim[i] = tri;
  if (tri == kMiss) {
    pos[i] = nrm[i] = alb[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const float4 n = st.tnrm[tri];
  const float dn = (n.x * dx + n.y * dy) + n.z * dz;
  const float sg = dn > 0.0f ? -1.0f : 1.0f;
  pos[i] = make_float4(f.pos[0] + t * dx, f.pos[1] + t * dy, f.pos[2] + t * dz, t);
  nrm[i] = make_float4(sg * n.x, sg * n.y, sg * n.z, 0.0f);
  const float4 al = st.mats[2 * __float_as_uint(n.w)];
  alb[i] = make_float4(al.x, al.y, al.z, 0.0f);
}

// ------------------------------------------------------------------------------------------
// Probe reprojection (Section 2.1.1, Algorithm 1): one wave per tile, lane = pixel
// 8 (y % 8) + (x % 8).  A pixel that is not sky projects its world position with the previous
// frame's camera; if the previous probe of that tile lies within the cell size (Algorithm 6)
// of the pixel's tangent plane with a normal cosine above 0.95, the pixel bids
// (half(distance) << 16) | lane; the smallest bid wins and the tile's probe moves there.
// ------------------------------------------------------------------------------------------
struct PrevCamera {
  float pos[3], fwd[3], right[3], up[3];
  float tan_half;
};

// the previous frame's pixel (qx, qy) whose centre region holds the projection of X
__device__ inline bool project_prev(const PrevCamera& pc, uint32_t W, uint32_t H, float Xx, float Xy, float Xz,
                                    uint32_t& qx, uint32_t& qy) {
  const float v0 = Xx - pc.pos[0], v1 = Xy - pc.pos[1], v2 = Xz - pc.pos[2];
  const float z = (v0 * pc.fwd[0] + v1 * pc.fwd[1]) + v2 * pc.fwd[2];
  if (!(z > 0.0f)) return false;
  const float a = ((v0 * pc.right[0] + v1 * pc.right[1]) + v2 * pc.right[2]) / z;
  const float b = ((v0 * pc.up[0] + v1 * pc.up[1]) + v2 * pc.up[2]) / z;
  const float aspect = (float)W / (float)H;
  const float sx = a / (pc.tan_half * aspect), sy = b / pc.tan_half;
  const float fx = ((sx + 1.0f) * (float)W) * 0.5f, fy = ((1.0f - sy) * (float)H) * 0.5f;
  if (!(fx >= 0.0f && fx < (float)W && fy >= 0.0f && fy < (float)H)) return false;
  qx = (uint32_t)fx;
  qy = (uint32_t)fy;
  return true;
}

__global__ __launch_bounds__(64) void k_reproject(const float4* gpos, const float4* gnrm, const uint32_t* gprim,
                                                  uint32_t W, uint32_t H, uint32_t TW, const uint32_t* prev_mask,
                                                  const float4* prev_pos, const float4* prev_nrm, PrevCamera pc,
                                                  float cx, float cy, float cz, float kappa, uint32_t* win,
                                                  uint32_t* hist) {
  __shared__ uint32_t best;
  const uint32_t t = blockIdx.x, lane = threadIdx.x;
  const uint32_t tx = t % TW, ty = t / TW;
  const uint32_t init = (0x7BFFu << 16) | 0xFFFFu;   // half(65504) above an impossible lane
  if (lane == 0) best = init;
  __syncthreads();
  const uint32_t x = 8u * tx + (lane & 7u), y = 8u * ty + (lane >> 3);
  uint32_t myq = kSentinel;
  if (x < W && y < H) {
    const uint32_t pix = y * W + x;
    if (gprim[pix] != kMiss) {
      const float4 X = gpos[pix], n = gnrm[pix];
      uint32_t qx, qy;
      if (project_prev(pc, W, H, X.x, X.y, X.z, qx, qy)) {
        const uint32_t q = (qy >> 3) * TW + (qx >> 3);
        if (prev_mask[q] != kSentinel) {
          const float4 wq = prev_pos[q], nq = prev_nrm[q];
          const float dx = X.x - cx, dy = X.y - cy, dz = X.z - cz;
          const float cs = kappa * sqrtf((dx * dx + dy * dy) + dz * dz);
          const float pd = fabsf(((wq.x - X.x) * n.x + (wq.y - X.y) * n.y) + (wq.z - X.z) * n.z);
          const float nc = (nq.x * n.x + nq.y * n.y) + nq.z * n.z;
          if (pd < cs && nc > 0.95f) {
            const float ex = wq.x - X.x, ey = wq.y - X.y, ez = wq.z - X.z;
            const float dist = sqrtf((ex * ex + ey * ey) + ez * ez);
            const uint32_t score = ((uint32_t)__half_as_ushort(__float2half_rn(dist)) << 16) | lane;
            atomicMin(&best, score);
            myq = q;
          }
        }
      }
    }
  }
  __syncthreads();
  const uint32_t b = best;
  if ((b & 0xFFFFu) != 0xFFFFu) {
    if (lane == (b & 0xFFFFu)) {
      win[t] = (y << 16) | x;
      hist[t] = myq;
    }
  } else if (lane == 0) {
    win[t] = kSentinel;
    hist[t] = kSentinel;
  }
}

// ------------------------------------------------------------------------------------------
// Temporal upscaling and adaptive sampling (Section 2.1.1 spawn tiles, Section 2.1.2,
// Algorithm 2).  A spawn tile is u x u probe tiles; the frame's jitter (sjx, sjy) in
// [0, 8u)^2 picks one pixel per spawn tile, and the probe tile holding it is spawned if the
// pixel is not sky.  Placement: a reprojected probe keeps its pixel, else a spawned tile
// takes the jittered pixel.  Only spawned tiles trace; a spawned tile whose probe also
// reprojected is an override tile, and a tile with neither ("empty") whose own pixel of the
// jitter (modulo 8 inside the tile) is not sky picks one override tile at random (counter
// hash, dimension 7) and, if it is the lowest-numbered tile to pick it, takes its rays and
// places a probe at that pixel.  Four small launches: classify, ordered override list (one
// block), pick (atomic minimum per override tile), apply.
// ------------------------------------------------------------------------------------------
struct UpscaleArgs {
  uint32_t W, H, TW, P, u, sjx, sjy, seed, frame;
};

__device__ inline uint32_t own_jitter_pixel(const UpscaleArgs& ua, const uint32_t* gprim, uint32_t t) {
  const uint32_t tx = t % ua.TW, ty = t / ua.TW;
  const uint32_t px = 8u * tx + ua.sjx % 8u, py = 8u * ty + ua.sjy % 8u;
  if (px < ua.W && py < ua.H && gprim[py * ua.W + px] != kMiss) return (py << 16) | px;
  return kSentinel;
}

__global__ __launch_bounds__(256) void k_upscale_classify(const uint32_t* gprim, UpscaleArgs ua, const uint32_t* win,
                                                          uint32_t* place, uint32_t* traced, uint32_t* cls,
                                                          uint32_t* assigned) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= ua.P) return;
  const uint32_t tx = t % ua.TW, ty = t / ua.TW;
  const uint32_t spx = 8u * ua.u * (tx / ua.u) + ua.sjx, spy = 8u * ua.u * (ty / ua.u) + ua.sjy;
  const bool spawned = spx / 8u == tx && spy / 8u == ty && spx < ua.W && spy < ua.H && gprim[spy * ua.W + spx] != kMiss;
  const uint32_t w = win ? win[t] : kSentinel;
  const bool reproj = w != kSentinel;
  place[t] = reproj ? w : (spawned ? ((spy << 16) | spx) : kSentinel);
  traced[t] = spawned ? 1u : 0u;
  uint32_t k = 0u;
  if (spawned && reproj) k = 1u;
  else if (!spawned && !reproj && own_jitter_pixel(ua, gprim, t) != kSentinel) k = 2u;
  cls[t] = k;
  assigned[t] = kSentinel;
}

// one block of 1024: override tiles (class 1) compacted in tile order, 1024 tiles per pass
__global__ __launch_bounds__(1024) void k_upscale_list(const uint32_t* cls, uint32_t P, uint32_t* over,
                                                       uint32_t* count) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t base;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  if (tid == 0) base = 0u;
  __syncthreads();
  for (uint32_t start = 0; start < P; start += 1024u) {
    const uint32_t t = start + tid;
    const bool on = t < P && cls[t] == 1u;
    const uint64_t b = __ballot(on);
    if (lane == 0) wsum[w] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t off = base;
    for (uint32_t i = 0; i < w; ++i) off += wsum[i];
    if (on) over[off + (uint32_t)__popcll(b & ((1ull << lane) - 1ull))] = t;
    __syncthreads();
    if (tid == 0) {
      uint32_t s = base;
      for (uint32_t i = 0; i < 16u; ++i) s += wsum[i];
      base = s;
    }
    __syncthreads();
  }
  if (tid == 0) count[0] = base;
}

__global__ __launch_bounds__(256) void k_upscale_pick(const uint32_t* cls, UpscaleArgs ua, const uint32_t* over,
                                                      const uint32_t* count, uint32_t* assigned) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= ua.P || cls[t] != 2u) return;
  const uint32_t n = count[0];
  if (n == 0u) return;
  const uint32_t o = over[rand_u32(ua.seed, ua.frame, t, 7u) % n];
  atomicMin(&assigned[o], t);
}

__global__ __launch_bounds__(256) void k_upscale_apply(const uint32_t* gprim, UpscaleArgs ua, const uint32_t* over,
                                                       const uint32_t* count, const uint32_t* assigned,
                                                       uint32_t* place, uint32_t* traced) {
  const uint32_t k = blockIdx.x * 256u + threadIdx.x;
  if (k >= count[0]) return;
  const uint32_t o = over[k], e = assigned[o];
  if (e == kSentinel) return;
  traced[o] = 0u;
  traced[e] = 1u;
  place[e] = own_jitter_pixel(ua, gprim, e);
}

// ------------------------------------------------------------------------------------------
// Spawn (Section 2.1.1), probe mask and its MIP chain (Section 2.1.5).  A MIP entry is the
// first valid probe of its 2x2 children in raster order (out-of-bounds children skipped).
// One block spawns a 16x16 patch of tiles and builds MIP levels 1..4 of that patch in LDS
// (a level-k entry of the patch depends on that patch only); levels 5+ are built from level
// 4 by one block.
// ------------------------------------------------------------------------------------------
struct MipInfo {
  uint32_t n;
  uint32_t w[16], h[16], off[16];
};

__global__ __launch_bounds__(256) void k_spawn_mips(const float4* gpos, const float4* gnrm, const uint32_t* gprim,
                                                    uint32_t W, uint32_t H, uint32_t TW, uint32_t TH, uint32_t jx,
                                                    uint32_t jy, MipInfo mi, const uint32_t* win,
                                                    const uint32_t* place, uint32_t* mask,
                                                    float4* ppos, float4* pnrm, unsigned long long* stats,
                                                    uint32_t* hit_count) {
  __shared__ uint32_t lv[2][256];
  const uint32_t t = threadIdx.x;
  if (blockIdx.x == 0 && blockIdx.y == 0 && t < kStatStripes) {
    // per-frame counters restart; so do the hit-list stripes of this frame's trace
    stats[t * GI_STAT_COUNT + GI_STAT_LIVE] = 0;
    stats[t * GI_STAT_COUNT + GI_STAT_RELAXED] = 0;
    stats[t * GI_STAT_COUNT + GI_STAT_NOPROBE] = 0;
    hit_count[t] = 0;
  }
  const uint32_t tx = blockIdx.x * 16u + (t & 15u), ty = blockIdx.y * 16u + (t >> 4);
  uint32_t m = kSentinel;
  if (tx < TW && ty < TH) {
    uint32_t px = 8u * tx + jx, py = 8u * ty + jy;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
    const uint32_t p = ty * TW + tx;
    // temporal reuse: a reprojected previous probe keeps its pixel instead of the Halton one
    // temporal upscaling: the placement is final (kept, spawned or adaptive-sampling probes)
    const uint32_t w = place ? place[p] : (win ? win[p] : kSentinel);
    if (place && w == kSentinel) {
      // no probe in this tile
    } else if (w != kSentinel) {
      px = w & 0xFFFFu;
      py = w >> 16;
      m = w;
      a = gpos[py * W + px];
      b = gnrm[py * W + px];
    } else if (px < W && py < H) {
      const uint32_t pix = py * W + px;
      if (gprim[pix] != kMiss) {
        m = (py << 16) | px;
        a = gpos[pix];
        b = gnrm[pix];
      }
    }
    mask[p] = m;
    ppos[p] = a;
    pnrm[p] = b;
  }
  // tiles outside the grid hold the sentinel, which the child scan skips like an absent child
  lv[0][t] = m;
  __syncthreads();
  uint32_t side = 16u, cur = 0u;
  for (uint32_t k = 1; k < mi.n && k <= 4u; ++k) {
    const uint32_t ns = side >> 1;
    if (t < ns * ns) {
      const uint32_t x = t % ns, y = t / ns;
      uint32_t v = kSentinel;
#pragma unroll
      for (uint32_t c = 0; c < 4; ++c) {
        const uint32_t cx = 2u * x + (c & 1u), cy = 2u * y + (c >> 1);
        if (v == kSentinel) v = lv[cur][cy * side + cx];
      }
      lv[cur ^ 1u][t] = v;
      const uint32_t gx = blockIdx.x * ns + x, gy = blockIdx.y * ns + y;
      if (gx < mi.w[k] && gy < mi.h[k]) mask[mi.off[k] + gy * mi.w[k] + gx] = v;
    }
    __syncthreads();
    cur ^= 1u;
    side = ns;
  }
}

// MIP levels 5.. from level 4 (one block; levels in sequence)
__global__ __launch_bounds__(1024) void k_mask_mips_top(MipInfo mi, uint32_t* mask) {
  for (uint32_t k = 5; k < mi.n; ++k) {
    const uint32_t sw = mi.w[k - 1], sh = mi.h[k - 1], dw = mi.w[k], dh = mi.h[k];
    const uint32_t* src = mask + mi.off[k - 1];
    for (uint32_t i = threadIdx.x; i < dw * dh; i += blockDim.x) {
      const uint32_t x = i % dw, y = i / dw;
      uint32_t v = kSentinel;
#pragma unroll
      for (uint32_t c = 0; c < 4; ++c) {
        const uint32_t cx = 2u * x + (c & 1u), cy = 2u * y + (c >> 1);
        if (v == kSentinel && cx < sw && cy < sh) v = src[cy * sw + cx];
      }
      mask[mi.off[k] + i] = v;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------
// Ray guiding (Section 2.1.2): parallax-corrected reconstruction of each new probe's
// hemisphere from the previous frame's probes, one wave per probe.  Candidates are the
// previous probes of the 3x3 tiles around the previous-frame tile that holds the probe's
// projection, if they pass the reprojection's tests (plane distance below the probe's cell
// size, normal cosine above 0.95).  Lane c of a candidate takes its cell c's hit point
// (position + travelled distance along the cell's centre direction) and sends the cell's
// radiance and the point's distance to the new probe's cell of that point.  Lanes sending
// to one cell are folded by the first of them in ascending lane order, candidates in row
// then column order, so every float sum has one fixed order.  Then per cell the weight
// floor(2^20 lum / max lum) (lum = channel mean) and the inclusive sums that the trace
// inverts; an empty cell holds distance -1.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_reconstruct(const uint32_t* mask, const float4* ppos, const float4* pnrm,
                                                    uint32_t W, uint32_t H, uint32_t TW, uint32_t TH, PrevCamera pc,
                                                    float cx, float cy, float cz, float kappa,
                                                    const uint32_t* prev_mask, const float4* prev_pos,
                                                    const float4* prev_nrm, const float4* prev_atlas, float4* recon,
                                                    uint32_t* cdf) {
  __shared__ float sum[64][4];
  __shared__ uint32_t cnt[64];
  __shared__ float rv[64][4];
  const uint32_t p = blockIdx.x, lane = threadIdx.x;
  sum[lane][0] = sum[lane][1] = sum[lane][2] = sum[lane][3] = 0.0f;
  cnt[lane] = 0u;
  __syncthreads();
  const float4 pp = ppos[p], pn = pnrm[p];
  uint32_t qx = 0, qy = 0;
  if (mask[p] != kSentinel && project_prev(pc, W, H, pp.x, pp.y, pp.z, qx, qy)) {
    const float ex = pp.x - cx, ey = pp.y - cy, ez = pp.z - cz;
    const float cs = kappa * sqrtf((ex * ex + ey * ey) + ez * ez);
    const Basis B = make_basis(pn.x, pn.y, pn.z);
    for (int dy = -1; dy <= 1; ++dy) {
      for (int dx = -1; dx <= 1; ++dx) {
        // tile, validity and the tests are the same for every lane: the wave takes one branch
        const int32_t tx = (int32_t)(qx >> 3) + dx, ty = (int32_t)(qy >> 3) + dy;
        if (tx < 0 || ty < 0 || tx >= (int32_t)TW || ty >= (int32_t)TH) continue;
        const uint32_t q = (uint32_t)ty * TW + (uint32_t)tx;
        if (prev_mask[q] == kSentinel) continue;
        const float4 wq = prev_pos[q], nq = prev_nrm[q];
        const float pd = fabsf(((wq.x - pp.x) * pn.x + (wq.y - pp.y) * pn.y) + (wq.z - pp.z) * pn.z);
        const float nc = (nq.x * pn.x + nq.y * pn.y) + nq.z * pn.z;
        if (!(pd < cs && nc > 0.95f)) continue;
        const float4 qa = prev_atlas[(size_t)q * 64 + lane];
        float d0, d1, d2;
        cell_centre_direction(lane, nq.x, nq.y, nq.z, d0, d1, d2);
        const float v0 = (wq.x + qa.w * d0) - pp.x;
        const float v1 = (wq.y + qa.w * d1) - pp.y;
        const float v2 = (wq.z + qa.w * d2) - pp.z;
        const float lz = (v0 * pn.x + v1 * pn.y) + v2 * pn.z;
        const bool on = lz > 0.0f;
        uint32_t k = 0u;
        if (on) {
          const float lx = (v0 * B.tx + v1 * B.ty) + v2 * B.tz;
          const float ly = (v0 * B.bx + v1 * B.by) + v2 * B.bz;
          k = local_cell(lx, ly, lz);
        }
        rv[lane][0] = qa.x;
        rv[lane][1] = qa.y;
        rv[lane][2] = qa.z;
        rv[lane][3] = sqrtf((v0 * v0 + v1 * v1) + v2 * v2);
        uint64_t same = __ballot(on);
#pragma unroll
        for (int b = 0; b < 6; ++b) {
          const uint64_t mb = __ballot(on && ((k >> b) & 1u));
          same &= ((k >> b) & 1u) ? mb : ~mb;
        }
        __syncthreads();
        if (on && (uint32_t)__ffsll((long long)same) - 1u == lane) {
          float x0 = sum[k][0], x1 = sum[k][1], x2 = sum[k][2], x3 = sum[k][3];
          uint32_t m = cnt[k];
          for (uint64_t s = same; s; s &= s - 1u) {
            const int i = __ffsll((long long)s) - 1;
            x0 = x0 + rv[i][0]; x1 = x1 + rv[i][1]; x2 = x2 + rv[i][2]; x3 = x3 + rv[i][3];
            ++m;
          }
          sum[k][0] = x0; sum[k][1] = x1; sum[k][2] = x2; sum[k][3] = x3;
          cnt[k] = m;
        }
        __syncthreads();
      }
    }
  }
  const uint32_t n = cnt[lane];
  float4 r = make_float4(0.0f, 0.0f, 0.0f, -1.0f);
  float lum = 0.0f;
  if (n) {
    const float fn = (float)n;
    r = make_float4(sum[lane][0] / fn, sum[lane][1] / fn, sum[lane][2] / fn, sum[lane][3] / fn);
    const float third = 1.0f / 3.0f;
    lum = (r.x * third + r.y * third) + r.z * third;
  }
  float maxl = lum;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) maxl = fmaxf(maxl, __shfl_xor(maxl, o, 64));
  uint32_t w = (n && maxl > 0.0f) ? (uint32_t)((lum / maxl) * 1048576.0f) : 0u;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t up = __shfl_up(w, o, 64);
    if (lane >= (uint32_t)o) w += up;
  }
  recon[(size_t)p * 64 + lane] = r;
  cdf[(size_t)p * 64 + lane] = w;
}

// ------------------------------------------------------------------------------------------
// Probe rays (Section 2.1.3): cosine-distributed direction, closest hit, ray record
// ------------------------------------------------------------------------------------------
struct ProbeRayArgs {
  const uint32_t* mask;
  const uint32_t* traced;   // temporal upscaling: probes that trace this frame (else every probe)
  const uint32_t* cdf;      // ray guiding: per probe the 64 inclusive weight sums (else none)
  const float4* ppos;
  const float4* pnrm;
  uint32_t P, R, seed, frame;
  float eps_scale, t_sky;
};

__device__ inline void probe_ray(const ProbeRayArgs& a, uint32_t gid, uint32_t p, float& ox, float& oy, float& oz,
                                 float& dx, float& dy, float& dz, uint32_t& cell) {
  const float4 pp = a.ppos[p], pn = a.pnrm[p];
  const float u0 = rand_unit(rand_u32(a.seed, a.frame, gid, 0u));
  const float u1 = rand_unit(rand_u32(a.seed, a.frame, gid, 1u));
  const uint32_t* cdf = a.cdf ? a.cdf + (size_t)p * 64 : nullptr;
  const uint32_t total = cdf ? cdf[63] : 0u;
  if (total) {
    // ray guiding: the first cell whose inclusive weight sum exceeds floor(r * total / 2^32),
    // then a uniform point of that cell
    const uint32_t target = (uint32_t)(((uint64_t)rand_u32(a.seed, a.frame, gid, 8u) * total) >> 32);
    uint32_t lo = 0u, hi = 63u;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (cdf[mid] > target) hi = mid;
      else lo = mid + 1u;
    }
    cell = lo;
    guided_direction(pn.x, pn.y, pn.z, cell, u0, u1, dx, dy, dz);
  } else {
    cosine_direction(pn.x, pn.y, pn.z, u0, u1, dx, dy, dz, cell);
  }
  const float eps = origin_offset(a.eps_scale, pp.x, pp.y, pp.z);
  ox = pp.x + pn.x * eps;
  oy = pp.y + pn.y * eps;
  oz = pp.z + pn.z * eps;
}

// Hits are regrouped for the shading pass: each wave ballots its hit lanes and appends their
// ray ids to the list stripe of its block range with one atomic per wave, so the shading
// waves run dense.  The list order is not deterministic; nothing downstream depends on it
// (cell sums are integer and the cell map is order-free).
struct HitList {
  uint32_t* ids;          // [kStatStripes * stripe_cap]
  uint32_t* count;        // [kStatStripes]
  uint32_t stripe_cap;    // ray slots per stripe (= blocks per stripe * 64)
  uint32_t blocks_per_stripe;
};

template <int STACK>
__global__ __launch_bounds__(kTraceBlock) void k_trace_probes(SceneView sv, ShadeTables st, ProbeRayArgs a,
                                                              uint4* rec, uint2* rkey, HitList hl,
                                                              unsigned long long* stats) {
  __shared__ uint32_t stk[STACK * kTraceBlock];
  __shared__ uint16_t stkt[STACK * kTraceBlock];
  TStack<STACK, kTraceBlock> ts(stk + threadIdx.x, stkt + threadIdx.x, sv.spill + (blockIdx.x * kTraceBlock + threadIdx.x), sv.spill_stride);
  const uint32_t gid = blockIdx.x * kTraceBlock + threadIdx.x;
  if (gid >= a.P * a.R) return;
  const uint32_t p = gid / a.R;
  const bool valid = a.traced ? a.traced[p] != 0u : a.mask[p] != kSentinel;
  stat_add(stats, GI_STAT_RAYS, valid);
  if (!valid) {
    rec[gid] = make_uint4(0xFFFFFFFFu, 0u, kMiss, 0u);
    rkey[gid] = make_uint2(0u, 0u);
    return;
  }
  float ox, oy, oz, dx, dy, dz;
  uint32_t cell;
  probe_ray(a, gid, p, ox, oy, oz, dx, dy, dz, cell);
  const RayQ r = make_ray(ox, oy, oz, dx, dy, dz);
  uint32_t tri;
  float t;
  closest_hit<STACK, kTraceBlock>(sv, r, 3.0e38f, ts, tri, t);
  uint32_t flags = cell | GI_RAY_TRACED;
  const bool hit = tri != kMiss;
  if (!hit) {
    rec[gid] = make_uint4(0xFFFFFFFFu, __float_as_uint(a.t_sky), kMiss, flags);
    rkey[gid] = make_uint2(0u, 0u);
  } else {
    const float4 n = st.tnrm[tri];
    const float dn = (n.x * dx + n.y * dy) + n.z * dz;
    flags |= GI_RAY_HIT;
    if (dn < 0.0f) {
      flags |= GI_RAY_FRONT;
      const float4 e = st.mats[2 * __float_as_uint(n.w) + 1];
      if (e.x > 0.0f || e.y > 0.0f || e.z > 0.0f) flags |= GI_RAY_EMIT;
    }
    rec[gid] = make_uint4(0xFFFFFFFFu, __float_as_uint(t), tri, flags);
  }
  const uint64_t m = __ballot(hit);
  if (m) {
    const uint32_t stripe = blockIdx.x / hl.blocks_per_stripe;
    const uint32_t leader = (uint32_t)__ffsll((long long)__ballot(1)) - 1u;
    uint32_t base = 0;
    if ((threadIdx.x & 63u) == leader) base = atomicAdd(&hl.count[stripe], (uint32_t)__popcll(m));
    base = __shfl(base, (int)leader, 64);
    if (hit) hl.ids[stripe * hl.stripe_cap + base + (uint32_t)__popcll(m & lanes_below())] = gid;
  }
}

// ------------------------------------------------------------------------------------------
// Hit shading (Sections 2.2.1-2.2.4, 2.3.1): descriptor -> find-or-insert -> one light
// sample with a shadow ray (+ cached bounce) -> fixed-point accumulation
// ------------------------------------------------------------------------------------------
struct CacheArgs {
  uint32_t* fp;
  uint64_t* key;
  uint4* acc;
  const float4* L;
  uint32_t* accessed;
  uint32_t bucket_mask;
  float cell_scale;
  uint32_t leak_bit;
  uint32_t frac_bits;
  float r_max;
  uint32_t bounces;
  float sky[3];
  float lod_scale;     // levels of detail of the descriptor (0 = one level)
  float cam[3];        // camera of the frame's spawn
  uint32_t tiled;      // two-level cache: slots are tiles of 64 cells, L is the prefiltered radiance
  uint32_t n_slots;    // table slots (tiles)
};

// World-cache entry of a hit: its slot, or with tiles cell * n_slots + slot.  Cell-major: the
// 64 cells of one tile lie in 64 different cache lines (each shared with the same cell of
// neighbouring slots), so the atomics of a tile that collects thousands of hits per frame
// spread over 64 lines instead of queueing at the 8 lines of a tile-major block.
__device__ inline int32_t cache_entry(const CacheArgs& c, int32_t slot, uint32_t tcell) {
  return slot < 0 ? slot : (c.tiled ? (int32_t)tcell * (int32_t)c.n_slots + slot : slot);
}

__device__ inline int32_t table_lookup(const CacheArgs& c, uint64_t key) {
  const uint32_t b = bucket_of(key, c.bucket_mask), f = fingerprint_of(key);
  const uint4* line = reinterpret_cast<const uint4*>(c.fp + b * kBucket);
  // the whole 128-B line first (independent loads), then the first slot holding f
  uint4 v[kBucket / 4];
#pragma unroll
  for (int q = 0; q < (int)kBucket / 4; ++q) v[q] = line[q];
  int32_t r = -1;
#pragma unroll
  for (int q = (int)kBucket / 4 - 1; q >= 0; --q) {
    if (v[q].w == f) r = 4 * q + 3;
    if (v[q].z == f) r = 4 * q + 2;
    if (v[q].y == f) r = 4 * q + 1;
    if (v[q].x == f) r = 4 * q;
  }
  return r < 0 ? -1 : (int32_t)(b * kBucket) + r;
}

// find-or-insert: the fingerprint is searched in the whole bucket first; otherwise the first
// empty slot is claimed with compare-and-swap.  Each round reads the bucket's fingerprints
// with coherent loads issued together; a CAS that finds our own fingerprint means another
// lane inserted the same cell, one that finds another fingerprint starts a new round (at most
// one per slot, so at most kBucket + 1 rounds).
__device__ inline int32_t table_insert(const CacheArgs& c, uint64_t key, bool& inserted) {
  inserted = false;
  const int32_t found = table_lookup(c, key);
  if (found >= 0) return found;
  const uint32_t b = bucket_of(key, c.bucket_mask), f = fingerprint_of(key);
  uint32_t* line = c.fp + b * kBucket;
  for (uint32_t round = 0; round <= kBucket; ++round) {
    uint32_t cur[kBucket];
#pragma unroll
    for (uint32_t s = 0; s < kBucket; ++s) cur[s] = __hip_atomic_load(line + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int32_t own = -1, empty = -1;
#pragma unroll
    for (int s = (int)kBucket - 1; s >= 0; --s) {
      if (cur[s] == f) own = s;
      if (cur[s] == 0u) empty = s;
    }
    if (own >= 0) return (int32_t)(b * kBucket) + own;
    if (empty < 0) return -1;
    const uint32_t prev = atomicCAS(line + empty, 0u, f);
    if (prev == 0u) {
      c.key[b * kBucket + (uint32_t)empty] = key;
      inserted = true;
      return (int32_t)(b * kBucket) + empty;
    }
    if (prev == f) return (int32_t)(b * kBucket) + empty;
  }
  return -1;
}

// One light sample (the single-candidate form of the light sampling of Section 2.3.1): an
// emitter triangle picked in proportion to its area, a uniform point on it, and the shadow
// ray towards it.  g = cos_y cos_l A_E / d^2 is the estimator's geometry factor.
struct LightSample {
  bool cast;
  RayQ ray;
  float tmax;
  float g;
  uint32_t mat;
};

// the part of the light sample that does not depend on the hit: the emitter (its index, the
// point on it and its normal), so that its loads can be issued before the hit's own
struct LightPick {
  uint32_t e;
  float xlx, xly, xlz;
  float4 ne;
};

__device__ inline LightPick pick_light(const ShadeTables& st, uint32_t seed, uint32_t frame, uint32_t gid) {
  LightPick lp;
  lp.e = 0u;
  lp.xlx = lp.xly = lp.xlz = 0.0f;
  lp.ne = make_float4(0.f, 0.f, 0.f, 0.f);
  if (st.n_emit == 0) return lp;
  const uint32_t rsel = rand_u32(seed, frame, gid, 2u);
  uint32_t lo = 0, hi = st.n_emit - 1u;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (rsel < st.ethr[mid]) hi = mid;
    else lo = mid + 1u;
  }
  lp.e = st.etri[lo];
  const float u3 = rand_unit(rand_u32(seed, frame, gid, 3u));
  const float u4 = rand_unit(rand_u32(seed, frame, gid, 4u));
  const float su = sqrtf(u3);
  const float b0 = 1.0f - su, b1 = su * (1.0f - u4), b2 = su * u4;
  const float4 A = st.evert[3 * lo], B = st.evert[3 * lo + 1], C = st.evert[3 * lo + 2];
  lp.xlx = (b0 * A.x + b1 * B.x) + b2 * C.x;
  lp.xly = (b0 * A.y + b1 * B.y) + b2 * C.y;
  lp.xlz = (b0 * A.z + b1 * B.z) + b2 * C.z;
  lp.ne = st.tnrm[lp.e];
  return lp;
}

__device__ inline LightSample sample_light(const ShadeTables& st, const LightPick& lp, float px, float py, float pz,
                                           float nx, float ny, float nz) {
  LightSample ls;
  ls.cast = false;
  ls.tmax = 0.0f;
  ls.g = 0.0f;
  ls.mat = 0;
  if (st.n_emit == 0) return ls;
  const float wx = lp.xlx - px, wy = lp.xly - py, wz = lp.xlz - pz;
  const float d2 = (wx * wx + wy * wy) + wz * wz;
  if (!(d2 > 0.0f)) return ls;
  const float dist = sqrtf(d2);
  const float omx = wx / dist, omy = wy / dist, omz = wz / dist;
  const float4 ne = lp.ne;
  const float cos_y = (nx * omx + ny * omy) + nz * omz;
  const float cos_l = -((ne.x * omx + ne.y * omy) + ne.z * omz);
  if (!(cos_y > 0.0f && cos_l > 0.0f)) return ls;
  ls.cast = true;
  ls.ray = make_ray(px, py, pz, omx, omy, omz);
  ls.tmax = dist * 0.9999f;
  ls.g = ((cos_y * cos_l) * st.area_total) / d2;
  ls.mat = __float_as_uint(ne.w);
  return ls;
}

// Section 2.3: resampled importance sampling over the light-grid cell of the hit point y.
// Candidates j: a light picked uniformly from the cell's list (hash dimension 16 + 4j), a
// uniform point on it (17 + 4j, 18 + 4j); weight = target / source pdf = lum * cos_y * cos_l
// / d^2 * count * area; weighted reservoir sampling keeps candidate j when u (19 + 4j) * sum
// < weight.  With world-space reservoir reuse (Section 2.3.1), the previous frame's reservoir
// of the hit's quantised position (a normal cosine above 0.9) enters with weight
// target(y_prev) * W_prev * min(M_prev, restir_cap * ris_m) by one more step (dimension 48), and the
// hit's final reservoir is offered to this frame's table (the lowest ray id per cell stays).
// The kept light's g is cos_y cos_l / d^2 * sum / (M * target).
__device__ inline float lum709(float4 le) { return (0.2126f * le.x + 0.7152f * le.y) + 0.0722f * le.z; }

struct RestirArgs {
  uint32_t on;                  // reservoirs are kept
  uint32_t cap;                 // largest count a reused reservoir enters with
  uint32_t has_prev;            // the read table holds the previous frame's
  CacheArgs prev, next;         // fp / key / bucket_mask of the read and written tables
  const float4* pyw;            // read table: light point, weight
  const float4* pn;             // read table: normal, w = light bits
  const uint32_t* pm;           // read table: count
  uint32_t* claim;              // written table: lowest ray id per slot
  float4* r_yw;                 // per ray: final reservoir
  float4* r_n;
  uint32_t* r_m;
  int32_t* r_slot;
  float cell_scale, lod_scale, cam[3];
};

__device__ inline void light_target(const ShadeTables& st, uint32_t k, float xx, float xy, float xz, float px,
                                    float py, float pz, float nx, float ny, float nz, float& ph, float& gg,
                                    float& dist, float& mx, float& my, float& mz) {
  const uint32_t e = st.etri[k];
  const float wx = xx - px, wy = xy - py, wz = xz - pz;
  const float d2 = (wx * wx + wy * wy) + wz * wz;
  ph = 0.0f;
  gg = 0.0f;
  dist = 0.0f;
  mx = my = mz = 0.0f;
  if (!(d2 > 0.0f)) return;
  dist = sqrtf(d2);
  mx = wx / dist;
  my = wy / dist;
  mz = wz / dist;
  const float4 ne = st.tnrm[e];
  const float cos_y = (nx * mx + ny * my) + nz * mz;
  const float cos_l = -((ne.x * mx + ne.y * my) + ne.z * mz);
  if (cos_y > 0.0f && cos_l > 0.0f) {
    gg = (cos_y * cos_l) / d2;
    ph = lum709(st.mats[2 * __float_as_uint(ne.w) + 1]) * gg;
  }
}

__device__ inline LightSample sample_light_ris(const ShadeTables& st, const RestirArgs& ra, uint32_t seed,
                                               uint32_t frame, uint32_t gid, float yx, float yy, float yz, float px,
                                               float py, float pz, float nx, float ny, float nz) {
  LightSample ls;
  ls.cast = false;
  ls.tmax = 0.0f;
  ls.g = 0.0f;
  ls.mat = 0;
  const LightGridGeom g = light_grid_geom(st.lg_box, st.lg_dim);
  const float yv[3] = {yx, yy, yz};
  uint32_t ci[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float f = floorf((yv[k] - g.lo[k]) / g.h);
    ci[k] = f < 0.0f ? 0u : (f > (float)(g.dim[k] - 1u) ? g.dim[k] - 1u : (uint32_t)f);
  }
  const uint32_t cell = (ci[2] * g.dim[1] + ci[1]) * g.dim[0] + ci[0];
  const uint32_t m = st.lg_count[cell];
  const uint32_t* list = st.lg_list + (size_t)cell * st.lg_k;
  float wsum = 0.0f, ph_sel = 0.0f, g_sel = 0.0f, dist_sel = 0.0f;
  float ox = 0.f, oy = 0.f, oz = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
  uint32_t k_sel = 0xFFFFFFFFu, M = 0u;
  if (m > 0u) {
    M = st.ris_m;
    for (uint32_t j = 0; j < st.ris_m; ++j) {
      const uint32_t rp = rand_u32(seed, frame, gid, 16u + 4u * j);
      const uint32_t k = list[(uint32_t)(((uint64_t)rp * m) >> 32)];
      const float u3 = rand_unit(rand_u32(seed, frame, gid, 17u + 4u * j));
      const float u4 = rand_unit(rand_u32(seed, frame, gid, 18u + 4u * j));
      const float us = rand_unit(rand_u32(seed, frame, gid, 19u + 4u * j));
      const float su = sqrtf(u3);
      const float b0 = 1.0f - su, b1 = su * (1.0f - u4), b2 = su * u4;
      const float4 A = st.evert[3 * k], B = st.evert[3 * k + 1], C = st.evert[3 * k + 2];
      const float xx = (b0 * A.x + b1 * B.x) + b2 * C.x;
      const float xy = (b0 * A.y + b1 * B.y) + b2 * C.y;
      const float xz = (b0 * A.z + b1 * B.z) + b2 * C.z;
      float ph, gg, dist, mx, my, mz;
      light_target(st, k, xx, xy, xz, px, py, pz, nx, ny, nz, ph, gg, dist, mx, my, mz);
      const float wj = (ph * (float)m) * A.w;
      wsum = wsum + wj;
      if (wj > 0.0f && us * wsum < wj) {
        k_sel = k;
        ph_sel = ph;
        g_sel = gg;
        dist_sel = dist;
        ox = mx; oy = my; oz = mz;
        sx = xx; sy = xy; sz = xz;
      }
    }
  }
  uint64_t pkey = 0;
  if (ra.on) {
    uint32_t tc;
    pkey = descriptor(ra.cell_scale, 0u, ra.lod_scale, ra.cam[0], ra.cam[1], ra.cam[2], yx, yy, yz, 1.0f, 0.0f,
                      0.0f, 0.0f, false, 0u, tc);
  }
  if (ra.on && ra.has_prev) {
    const int32_t s = table_lookup(ra.prev, pkey);
    if (s >= 0) {
      const float4 np = ra.pn[s];
      const float cn = (nx * np.x + ny * np.y) + nz * np.z;
      if (cn > 0.9f) {
        const uint32_t kp = __float_as_uint(np.w);
        const float4 xp = ra.pyw[s];
        const uint32_t Mp = ra.pm[s] < ra.cap ? ra.pm[s] : ra.cap;
        float ph, gg, dist, mx, my, mz;
        light_target(st, kp, xp.x, xp.y, xp.z, px, py, pz, nx, ny, nz, ph, gg, dist, mx, my, mz);
        const float wp = (ph * xp.w) * (float)Mp;
        wsum = wsum + wp;
        const float us = rand_unit(rand_u32(seed, frame, gid, 48u));
        if (wp > 0.0f && us * wsum < wp) {
          k_sel = kp;
          ph_sel = ph;
          g_sel = gg;
          dist_sel = dist;
          ox = mx; oy = my; oz = mz;
          sx = xp.x; sy = xp.y; sz = xp.z;
        }
        M = M + Mp;
      }
    }
  }
  if (k_sel == 0xFFFFFFFFu) {
    if (ra.on) {
      ra.r_m[gid] = 0u;
      ra.r_slot[gid] = -1;
    }
    return ls;
  }
  const float W = wsum / ((float)M * ph_sel);
  if (ra.on) {
    bool ins;
    const int32_t slot = table_insert(ra.next, pkey, ins);
    ra.r_yw[gid] = make_float4(sx, sy, sz, W);
    ra.r_n[gid] = make_float4(nx, ny, nz, __uint_as_float(k_sel));
    ra.r_m[gid] = M;
    ra.r_slot[gid] = slot;
    if (slot >= 0) atomicMin(ra.claim + slot, gid);
  }
  ls.cast = true;
  ls.ray = make_ray(px, py, pz, ox, oy, oz);
  ls.tmax = dist_sel * 0.9999f;
  ls.g = g_sel * W;
  ls.mat = __float_as_uint(st.tnrm[st.etri[k_sel]].w);
  return ls;
}

// ------------------------------------------------------------------------------------------
// Light grid (Section 2.3.2).  The box of this frame's probe-ray hit points: per block the
// minimum and maximum codes (lg_encode) of the hit coordinates, y = o + t d exactly as the
// shading computes it, then one block reduces the partial boxes (integer minima and maxima:
// the box does not depend on the order).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lg_box_partial(ProbeRayArgs a, const uint4* rec, uint32_t* part) {
  __shared__ uint32_t red[6][4];
  const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
  uint32_t v[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
  if (gid < a.P * a.R) {
    const uint4 r = rec[gid];
    if (r.w & GI_RAY_HIT) {
      float ox, oy, oz, dx, dy, dz;
      uint32_t cell;
      probe_ray(a, gid, gid / a.R, ox, oy, oz, dx, dy, dz, cell);
      const float t = __uint_as_float(r.y);
      const uint32_t cx = lg_encode(ox + t * dx), cy = lg_encode(oy + t * dy), cz = lg_encode(oz + t * dz);
      v[0] = cx; v[1] = cy; v[2] = cz; v[3] = cx; v[4] = cy; v[5] = cz;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint32_t lo = __shfl_xor(v[k], o, 64), hi = __shfl_xor(v[3 + k], o, 64);
      v[k] = lo < v[k] ? lo : v[k];
      v[3 + k] = hi > v[3 + k] ? hi : v[3 + k];
    }
  }
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0u)
    for (int k = 0; k < 6; ++k) red[k][w] = v[k];
  __syncthreads();
  if (threadIdx.x < 6u) {
    const uint32_t k = threadIdx.x;
    uint32_t x = red[k][0];
    for (int i = 1; i < 4; ++i) x = k < 3u ? (red[k][i] < x ? red[k][i] : x) : (red[k][i] > x ? red[k][i] : x);
    part[(size_t)blockIdx.x * 6 + k] = x;
  }
}

__global__ __launch_bounds__(1024) void k_lg_box_final(const uint32_t* part, uint32_t nparts, uint32_t* box) {
  __shared__ uint32_t red[6][16];
  uint32_t v[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
  for (uint32_t b = threadIdx.x; b < nparts; b += 1024u)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const uint32_t x = part[(size_t)b * 6 + k];
      v[k] = k < 3 ? (x < v[k] ? x : v[k]) : (x > v[k] ? x : v[k]);
    }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint32_t lo = __shfl_xor(v[k], o, 64), hi = __shfl_xor(v[3 + k], o, 64);
      v[k] = lo < v[k] ? lo : v[k];
      v[3 + k] = hi > v[3 + k] ? hi : v[3 + k];
    }
  }
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0u)
    for (int k = 0; k < 6; ++k) red[k][w] = v[k];
  __syncthreads();
  if (threadIdx.x < 6u) {
    const uint32_t k = threadIdx.x;
    uint32_t x = red[k][0];
    for (int i = 1; i < 16; ++i) x = k < 3u ? (red[k][i] < x ? red[k][i] : x) : (red[k][i] > x ? red[k][i] : x);
    box[k] = x;
  }
}

// Light lists, one wave per grid cell: each light's importance (mean over the cell's 8
// corners of luminance * area * cos / max(d^2, area); culled when the cell's bounding sphere
// lies behind the light's plane or beyond its range sqrt(luminance * area / threshold) plus
// the radius) into LDS, then lgrid_k rounds of the largest importance > 0 (ties: lower index).
constexpr uint32_t kLgMaxLights = 2048;

__global__ __launch_bounds__(64) void k_light_grid(ShadeTables st, uint32_t n_emit, float threshold, uint32_t* list,
                                                   uint32_t* count) {
  __shared__ float imp[kLgMaxLights];
  const LightGridGeom g = light_grid_geom(st.lg_box, st.lg_dim);
  const uint32_t ncell = g.dim[0] * g.dim[1] * g.dim[2];
  const uint32_t ci = blockIdx.x, lane = threadIdx.x;
  if (ci >= ncell) return;
  const uint32_t cxyz[3] = {ci % g.dim[0], (ci / g.dim[0]) % g.dim[1], ci / (g.dim[0] * g.dim[1])};
  float cc[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) cc[j] = g.lo[j] + ((float)cxyz[j] + 0.5f) * g.h;
  const float R = g.h * 0.8660254037844386f;
  for (uint32_t k = lane; k < n_emit; k += 64u) {
    const float4 A = st.evert[3 * k], B = st.evert[3 * k + 1], C = st.evert[3 * k + 2];
    const float cen[3] = {(float)((((double)A.x + (double)B.x) + (double)C.x) / 3.0),
                          (float)((((double)A.y + (double)B.y) + (double)C.y) / 3.0),
                          (float)((((double)A.z + (double)B.z) + (double)C.z) / 3.0)};
    const float4 n = st.tnrm[st.etri[k]];
    const float phi = lum709(st.mats[2 * __float_as_uint(n.w) + 1]) * A.w;
    float v = -1.0f;
    const float sd = ((cc[0] - cen[0]) * n.x + (cc[1] - cen[1]) * n.y) + (cc[2] - cen[2]) * n.z;
    const float ex = cc[0] - cen[0], ey = cc[1] - cen[1], ez = cc[2] - cen[2];
    const float dist = sqrtf((ex * ex + ey * ey) + ez * ez);
    const float range = sqrtf(phi / threshold);
    if (!(sd < -R) && !(dist > range + R)) {
      float s = 0.0f;
      for (uint32_t q = 0; q < 8u; ++q) {
        float vv3[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) vv3[j] = (g.lo[j] + (float)(cxyz[j] + ((q >> j) & 1u)) * g.h) - cen[j];
        const float vv = (vv3[0] * vv3[0] + vv3[1] * vv3[1]) + vv3[2] * vv3[2];
        const float len = sqrtf(vv);
        const float cs = len > 0.0f ? ((vv3[0] * n.x + vv3[1] * n.y) + vv3[2] * n.z) / len : 0.0f;
        if (cs > 0.0f) s = s + (phi * cs) / (vv > A.w ? vv : A.w);
      }
      v = s * 0.125f;
    }
    imp[k] = v;
  }
  __syncthreads();
  const uint32_t K = st.lg_k < n_emit ? st.lg_k : n_emit;
  uint32_t cnt = 0;
  for (uint32_t r = 0; r < K; ++r) {
    float bv = -1.0f;
    uint32_t bi = 0xFFFFFFFFu;
    for (uint32_t k = lane; k < n_emit; k += 64u) {
      const float x = imp[k];
      if (x > 0.0f && (bi == 0xFFFFFFFFu || x > bv)) {
        bv = x;
        bi = k;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const float ov = __shfl_xor(bv, o, 64);
      const uint32_t oi = __shfl_xor(bi, o, 64);
      const bool better = oi != 0xFFFFFFFFu && (bi == 0xFFFFFFFFu || ov > bv || (ov == bv && oi < bi));
      if (better) {
        bv = ov;
        bi = oi;
      }
    }
    if (bi == 0xFFFFFFFFu) break;
    if (lane == 0u) {
      list[(size_t)ci * st.lg_k + cnt] = bi;
      imp[bi] = -1.0f;
    }
    ++cnt;
    __syncthreads();
  }
  if (lane == 0u) count[ci] = cnt;
}

// World-space reservoirs (Section 2.3.1): the table written this frame starts empty; after
// the shading, each slot takes the reservoir of the lowest ray id that offered to it.
__global__ __launch_bounds__(256) void k_restir_clear(uint32_t* fp, uint64_t* key, uint32_t* claim, uint32_t n) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  fp[i] = 0u;
  key[i] = 0u;
  claim[i] = 0xFFFFFFFFu;
}

__global__ __launch_bounds__(256) void k_restir_store(const uint4* rec, uint32_t n, RestirArgs ra, float4* yw,
                                                      float4* nrm, uint32_t* cnt) {
  const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
  if (gid >= n || !(rec[gid].w & GI_RAY_HIT)) return;
  if (ra.r_m[gid] == 0u) return;
  const int32_t s = ra.r_slot[gid];
  if (s < 0 || ra.claim[s] != gid) return;
  yw[s] = ra.r_yw[gid];
  nrm[s] = ra.r_n[gid];
  cnt[s] = ra.r_m[gid];
}

template <int STACK>
__global__ __launch_bounds__(kTraceBlock) void k_shade_hits(SceneView sv, ShadeTables st, ProbeRayArgs a,
                                                            CacheArgs c, uint4* rec, uint2* rkey, HitList hl,
                                                            LearnedShadeOut lo, RestirArgs ra,
                                                            unsigned long long* stats) {
  // the traversal stacks; after the walks their LDS holds the wave's entry grouping
  __shared__ __align__(8) uint32_t stk[STACK * kTraceBlock];
  __shared__ uint16_t stkt[STACK * kTraceBlock];
  static_assert(STACK * kTraceBlock >= 576, "the entry grouping needs 576 words of the stack's LDS");
  // block b shades items [w * 64, w * 64 + 64) of list stripe b / blocks_per_stripe
  const uint32_t stripe = blockIdx.x / hl.blocks_per_stripe;
  const uint32_t item = (blockIdx.x % hl.blocks_per_stripe) * kTraceBlock + threadIdx.x;
  if (stripe >= kStatStripes || item >= hl.count[stripe]) return;
  const uint32_t gid = hl.ids[stripe * hl.stripe_cap + item];
  TStack<STACK, kTraceBlock> ts(stk + threadIdx.x, stkt + threadIdx.x, sv.spill + gid, sv.spill_stride);
  const uint4 rr = rec[gid];
  // the emitter of the light sample depends on the ray's random numbers only: its loads go
  // first, beside the hit's
  const LightPick lpick = st.lg_list ? LightPick{} : pick_light(st, a.seed, a.frame, gid);
  stat_add(stats, GI_STAT_HITS, true);
  const uint32_t p = gid / a.R;
  float ox, oy, oz, dx, dy, dz;
  uint32_t cell;
  probe_ray(a, gid, p, ox, oy, oz, dx, dy, dz, cell);
  const float t = __uint_as_float(rr.y);
  const uint32_t tri = rr.z;
  const float4 n = st.tnrm[tri];
  const float dn = (n.x * dx + n.y * dy) + n.z * dz;
  const float sg = dn > 0.0f ? -1.0f : 1.0f;
  const float yx = ox + t * dx, yy = oy + t * dy, yz = oz + t * dz;
  const float nx = sg * n.x, ny = sg * n.y, nz = sg * n.z;
  uint32_t tcell;
  const uint64_t key = descriptor(c.cell_scale, c.leak_bit, c.lod_scale, c.cam[0], c.cam[1], c.cam[2], yx, yy, yz, nx,
                                  ny, nz, t, true, c.tiled, tcell);
  rkey[gid] = make_uint2((uint32_t)key, (uint32_t)(key >> 32));
  if (lo.hitpos) {
    lo.hitpos[gid] = make_float4(yx, yy, yz, t);
    lo.hitnrm[gid] = make_float4(nx, ny, nz, 0.0f);
  }
  bool inserted;
  const int32_t tslot = table_insert(c, key, inserted);
  stat_add(stats, GI_STAT_INSERTS, inserted);
  stat_add(stats, GI_STAT_OVERFLOW, tslot < 0);
  // set once: with tiles thousands of hits share one flag, and a store from each would queue
  // at its L2 line (the flag is read here and written after the light sample, so that the
  // read's latency passes meanwhile)
  const uint32_t was_accessed = tslot >= 0 ? c.accessed[tslot] : 1u;
  const int32_t slot = cache_entry(c, tslot, tcell);

  // one light sample: area-proportional emitter, uniform point, one shadow ray
  const float eps = origin_offset(a.eps_scale, yx, yy, yz);
  const float px = yx + nx * eps, py = yy + ny * eps, pz = yz + nz * eps;
  float E0 = 0.f, E1 = 0.f, E2 = 0.f;
  const LightSample ls = st.lg_list ? sample_light_ris(st, ra, a.seed, a.frame, gid, yx, yy, yz, px, py, pz, nx, ny, nz)
                                    : sample_light(st, lpick, px, py, pz, nx, ny, nz);
  const bool cast = ls.cast;
  bool occl = false;
  if (cast) {
    occl = any_hit<STACK, kTraceBlock>(sv, ls.ray, ls.tmax, ts);
    if (!occl) {
      const float4 le = st.mats[2 * ls.mat + 1];
      E0 = le.x * ls.g;
      E1 = le.y * ls.g;
      E2 = le.z * ls.g;
    }
  }
  stat_add(stats, GI_STAT_SHADOW, cast);
  stat_add(stats, GI_STAT_OCCLUDED, occl);
  if (was_accessed == 0u) c.accessed[tslot] = 1u;
  // cached bounce (temporal radiance feedback, Section 2.2.4)
  float Lb0 = 0.f, Lb1 = 0.f, Lb2 = 0.f;
  if (c.bounces >= 2) {
    stat_add(stats, GI_STAT_BOUNCE, true);
    const float u5 = rand_unit(rand_u32(a.seed, a.frame, gid, 5u));
    const float u6 = rand_unit(rand_u32(a.seed, a.frame, gid, 6u));
    float bx, by, bz;
    uint32_t bcell;
    cosine_direction(nx, ny, nz, u5, u6, bx, by, bz, bcell);
    const RayQ br = make_ray(px, py, pz, bx, by, bz);
    uint32_t btri;
    float bt;
    closest_hit<STACK, kTraceBlock>(sv, br, 3.0e38f, ts, btri, bt);
    if (btri == kMiss) {
      Lb0 = c.sky[0]; Lb1 = c.sky[1]; Lb2 = c.sky[2];
    } else {
      const float4 bn = st.tnrm[btri];
      const float bdn = (bn.x * bx + bn.y * by) + bn.z * bz;
      const float bs = bdn > 0.0f ? -1.0f : 1.0f;
      uint32_t btcell;
      const uint64_t bkey = descriptor(c.cell_scale, c.leak_bit, c.lod_scale, c.cam[0], c.cam[1], c.cam[2],
                                       px + bt * bx, py + bt * by, pz + bt * bz,
                                       bs * bn.x, bs * bn.y, bs * bn.z, bt, true, c.tiled, btcell);
      const int32_t bslot = table_lookup(c, bkey);
      if (bslot >= 0) {
        if (c.accessed[bslot] == 0u) c.accessed[bslot] = 1u;
        const float4 lv = c.L[cache_entry(c, bslot, btcell)];
        Lb0 = lv.x; Lb1 = lv.y; Lb2 = lv.z;
      }
    }
  }
  rec[gid].x = (uint32_t)slot;
  if (slot < 0) return;
  const float4 alb = st.mats[2 * __float_as_uint(n.w)];
  const float s0 = alb.x * (E0 * 0.31830988618379067f + Lb0);
  const float s1 = alb.y * (E1 * 0.31830988618379067f + Lb1);
  const float s2 = alb.z * (E2 * 0.31830988618379067f + Lb2);
  const bool finite = isfinite(s0) && isfinite(s1) && isfinite(s2);
  stat_add(stats, GI_STAT_NONFINITE, !finite);
  if (lo.trec && finite) {
    // learned mode: the sample (before quantisation) is the ray's training record; the flag
    // puts the ray in the frame's training list, which is compacted in ray order
    lo.trec[gid] = make_float4(s0, s1, s2, 1.0f);
    lo.tflag[gid] = 1u;
  }
  if (!finite) return;
  const float scale = (float)(1u << c.frac_bits);
  const uint32_t q0 = (uint32_t)rintf(fminf(fmaxf(s0, 0.0f), c.r_max) * scale);
  const uint32_t q1 = (uint32_t)rintf(fminf(fmaxf(s1, 0.0f), c.r_max) * scale);
  const uint32_t q2 = (uint32_t)rintf(fminf(fmaxf(s2, 0.0f), c.r_max) * scale);
  // the lanes of this wave that add to one entry are summed first, by the first of them, which
  // issues the entry's atomics once (integer sums: the grouping does not change the result,
  // nor the number of carries, as every partial sum stays below 2^32).  The lanes of an entry
  // are found through a wave-private hash of the entries in the stacks' LDS (insert by
  // compare-and-swap with linear probing, then an OR of the lane's bit; 128 places for at most
  // 64 entries, so every insert ends)
  const uint32_t ent = (uint32_t)slot;
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t active = __ballot(true);
  const uint32_t nact = (uint32_t)__popcll(active), rank = (uint32_t)__popcll(active & lanes_below());
  uint32_t* keys = stk;                                                          // entry + 1, 0 = free
  unsigned long long* lanes = reinterpret_cast<unsigned long long*>(stk + 128);   // lane mask per place
  uint32_t* qv = stk + 384;                                                      // [64][3] samples
  wave_sync();
  for (uint32_t k = rank; k < 128u; k += nact) {
    keys[k] = 0u;
    lanes[k] = 0ull;
  }
  qv[3 * lane] = q0;
  qv[3 * lane + 1] = q1;
  qv[3 * lane + 2] = q2;
  wave_sync();
  uint32_t h = (ent * 0x9E3779B1u) >> 25;
  while (true) {
    const uint32_t old = atomicCAS(&keys[h], 0u, ent + 1u);
    if (old == 0u || old == ent + 1u) break;
    h = (h + 1u) & 127u;
  }
  atomicOr(&lanes[h], 1ull << lane);
  wave_sync();
  const uint64_t same = lanes[h];
  uint32_t g0 = 0u, g1 = 0u, g2 = 0u;
  for (uint64_t m = (uint32_t)__ffsll((long long)same) - 1u == lane ? same : 0ull; m; m &= m - 1u) {
    const int i = __ffsll((long long)m) - 1;
    g0 += qv[3 * i];
    g1 += qv[3 * i + 1];
    g2 += qv[3 * i + 2];
  }
  if ((uint32_t)__ffsll((long long)same) - 1u == (threadIdx.x & 63u)) {
    uint32_t* accp = reinterpret_cast<uint32_t*>(c.acc + slot);
    const uint32_t o0 = atomicAdd(accp + 0, g0);
    const uint32_t o1 = atomicAdd(accp + 1, g1);
    const uint32_t o2 = atomicAdd(accp + 2, g2);
    atomicAdd(accp + 3, (uint32_t)__popcll(same));
    const uint32_t wraps = (o0 + g0 < o0) + (o1 + g1 < o1) + (o2 + g2 < o2);
    if (wraps) atomicAdd(&stats[GI_STAT_WRAPS], (unsigned long long)wraps);
  }
}

// ------------------------------------------------------------------------------------------
// Cache update (Section 2.2.1 decay, Section 2.2.3 moving average): one thread per slot
// ------------------------------------------------------------------------------------------
// thread t of the grid updates slots t and t + T (T = threads of the grid): all fingerprints,
// then the live slots' state, are loaded before any is used (2 slots per thread measured a
// little faster than 1, 4 or 8)
constexpr uint32_t kUpdateSlots = 2;

__global__ __launch_bounds__(256) void k_cache_update(uint32_t N, uint32_t* fp, uint64_t* key, uint4* acc, float4* L,
                                                      uint2* meta, uint32_t* accessed, uint32_t n_cap,
                                                      uint32_t max_life, uint32_t frac_bits,
                                                      unsigned long long* stats) {
  __shared__ uint32_t bcount[2];   // the block's live and evicted slots: one atomic each per block
  if (threadIdx.x < 2u) bcount[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t T = gridDim.x * blockDim.x;
  const uint32_t s0 = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t f[kUpdateSlots];
#pragma unroll
  for (uint32_t k = 0; k < kUpdateSlots; ++k) {
    const uint32_t s = s0 + k * T;
    f[k] = s < N ? fp[s] : 0u;
  }
  uint4 a[kUpdateSlots];
  float4 l[kUpdateSlots];
  uint2 m[kUpdateSlots];
  uint32_t acc_bit[kUpdateSlots];
#pragma unroll
  for (uint32_t k = 0; k < kUpdateSlots; ++k)
    if (f[k] != 0u) {
      const uint32_t s = s0 + k * T;
      a[k] = acc[s];
      l[k] = L[s];
      m[k] = meta[s];
      acc_bit[k] = accessed[s];
    }
  uint32_t nlive = 0, nevict = 0;
#pragma unroll
  for (uint32_t k = 0; k < kUpdateSlots; ++k) {
    if (f[k] == 0u) continue;
    const uint32_t s = s0 + k * T;
    if (a[k].w > 0u) {
      const uint32_t h = m[k].x < n_cap ? m[k].x : n_cap;
      const float w = (float)a[k].w / (float)((double)h + (double)a[k].w);
      const double den = (double)a[k].w * (double)(1u << frac_bits);
      const float m0 = (float)((double)a[k].x / den);
      const float m1 = (float)((double)a[k].y / den);
      const float m2 = (float)((double)a[k].z / den);
      l[k].x = l[k].x + w * (m0 - l[k].x);
      l[k].y = l[k].y + w * (m1 - l[k].y);
      l[k].z = l[k].z + w * (m2 - l[k].z);
      const uint64_t nh = (uint64_t)m[k].x + a[k].w;
      m[k].x = nh < n_cap ? (uint32_t)nh : n_cap;
    }
    m[k].y = acc_bit[k] ? max_life : m[k].y - 1u;
    if (m[k].y == 0u) {
      fp[s] = 0u;
      key[s] = 0u;
      m[k].x = 0u;
      l[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      ++nevict;
    } else {
      ++nlive;
    }
    L[s] = l[k];
    meta[s] = m[k];
    if (a[k].w | a[k].x | a[k].y | a[k].z) acc[s] = make_uint4(0u, 0u, 0u, 0u);
    if (acc_bit[k]) accessed[s] = 0u;
  }
  // the block's counts: a wave sum, then one LDS atomic per wave and one global one per block
  for (int o = 32; o >= 1; o >>= 1) {
    nlive += (uint32_t)__shfl_xor((int)nlive, o, 64);
    nevict += (uint32_t)__shfl_xor((int)nevict, o, 64);
  }
  if ((threadIdx.x & 63u) == 0u) {
    if (nlive) atomicAdd(&bcount[0], nlive);
    if (nevict) atomicAdd(&bcount[1], nevict);
  }
  __syncthreads();
  if (threadIdx.x == 0u) {
    unsigned long long* st = stats + (blockIdx.x % kStatStripes) * GI_STAT_COUNT;
    if (bcount[0]) atomicAdd(&st[GI_STAT_LIVE], (unsigned long long)bcount[0]);
    if (bcount[1]) atomicAdd(&st[GI_STAT_EVICT], (unsigned long long)bcount[1]);
  }
}

// ------------------------------------------------------------------------------------------
// Probe gather + radiance backup (Section 2.1.4) + SH projection (Section 2.4.2):
// one wave per probe, lane = atlas cell
// ------------------------------------------------------------------------------------------

// the configuration caps the rays per probe at 256; up to 64 rays the kernel is built with a
// 64-entry ray stage, which cuts its LDS from 7.25 to 3.25 KiB and lets more waves share a CU
constexpr int kGatherMaxR = 256;
constexpr uint32_t kGatherWaves = 4;

// one butterfly step of a transpose-reduce over the first 2H entries of v: lanes whose bit
// log2(2H) is set keep the upper half, the others the lower half, each adding its partner's copy
template <int H>
__device__ inline float lane_xor(float x) {
  const uint32_t u = __float_as_uint(x);
  if (H == 4) return __uint_as_float(__builtin_amdgcn_update_dpp(0u, u, 0x128, 0xF, 0xF, false));   // row_ror:8 = xor 8
  if (H == 2) return __uint_as_float(__builtin_amdgcn_ds_swizzle(u, 0x101F));                       // xor 4
  return __uint_as_float(__builtin_amdgcn_update_dpp(0u, u, 0x4E, 0xF, 0xF, false));                 // quad_perm 2301 = xor 2
}

// balanced pairwise sum over the 64 lanes (lanes 2i and 2i + 1 first, then pairs of those
// sums, and so on up to the two halves): the radiance backup's sum in a fixed order.
// Each step adds the partner's value (lane ^ 1, 2, 4, 8, 16, 32); float addition commutes, so
// both partners hold the same sum and every lane ends with the total.
__device__ inline float wave_pair_sum(float x) {
  x = x + __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(x), 0xB1, 0xF, 0xF, false));   // xor 1
  x = x + __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(x), 0x4E, 0xF, 0xF, false));   // xor 2
  x = x + __uint_as_float(__builtin_amdgcn_ds_swizzle(__float_as_uint(x), 0x101F));                       // xor 4
  x = x + __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(x), 0x128, 0xF, 0xF, false));  // xor 8
  const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  x = __uint_as_float(r16[0]) + __uint_as_float(r16[1]);                                                 // xor 16
  const auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(r32[0]) + __uint_as_float(r32[1]);                                              // xor 32
}

template <int H>
__device__ inline void transpose_reduce_step(float (&v)[32], uint32_t lane, uint32_t& coef) {
  const bool up = (lane & (uint32_t)(2 * H)) != 0u;
  if (H >= 8) {
    // lane halves (H = 16) or rows of 16 (H = 8) exchange whole registers: the swap hands each
    // lane its own and its partner's copy of the half it keeps
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const auto r = H == 16 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[H + i]), false, false)
                             : __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[H + i]), false, false);
      v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const float keep = up ? v[H + i] : v[i];
      const float send = up ? v[i] : v[H + i];
      v[i] = keep + lane_xor<H>(send);
    }
  }
  coef += up ? (uint32_t)H : 0u;
}

// SH projection of one probe's atlas (Section 2.4.2), one wave per probe, lane = cell:
// exact integrals of the 9 real basis functions over the cell from its direction moments
// rotated into the probe frame (columns t, b, n); c0..c2 = the cell's radiance
struct CellMoments {
  float v[10];   // solid angle, first moments (3), second moments xx yy zz xy xz yz
};

__device__ inline CellMoments load_moments(const float* moments, uint32_t lane) {
  CellMoments m;
  const float* mo = moments + lane * 10;
#pragma unroll
  for (int i = 0; i < 10; ++i) m.v[i] = mo[i];
  return m;
}

__device__ inline void probe_sh(uint32_t p, uint32_t lane, float4 nn, const CellMoments& cm, float c0, float c1,
                                float c2, float* sh) {
  const Basis B = make_basis(nn.x, nn.y, nn.z);
  const float R00 = B.tx, R10 = B.ty, R20 = B.tz;
  const float R01 = B.bx, R11 = B.by, R21 = B.bz;
  const float R02 = nn.x, R12 = nn.y, R22 = nn.z;
  const float* mo = cm.v;
  const float om = mo[0];
  const float mlx = mo[1], mly = mo[2], mlz = mo[3];
  const float Mxx = mo[4], Myy = mo[5], Mzz = mo[6], Mxy = mo[7], Mxz = mo[8], Myz = mo[9];
  // the projection is compared within a tolerance (no integer decision depends on its bits),
  // so its dot products are fused multiply-adds
  auto dot3 = [](float a0, float b0, float a1, float b1, float a2, float b2) {
    return fmaf(a0, b0, fmaf(a1, b1, a2 * b2));
  };
  const float mwx = dot3(R00, mlx, R01, mly, R02, mlz);
  const float mwy = dot3(R10, mlx, R11, mly, R12, mlz);
  const float mwz = dot3(R20, mlx, R21, mly, R22, mlz);
  // T = R M (rows i), W = T R^T
  const float T00 = dot3(R00, Mxx, R01, Mxy, R02, Mxz), T01 = dot3(R00, Mxy, R01, Myy, R02, Myz),
              T02 = dot3(R00, Mxz, R01, Myz, R02, Mzz);
  const float T10 = dot3(R10, Mxx, R11, Mxy, R12, Mxz), T11 = dot3(R10, Mxy, R11, Myy, R12, Myz),
              T12 = dot3(R10, Mxz, R11, Myz, R12, Mzz);
  const float T20 = dot3(R20, Mxx, R21, Mxy, R22, Mxz), T21 = dot3(R20, Mxy, R21, Myy, R22, Myz),
              T22 = dot3(R20, Mxz, R21, Myz, R22, Mzz);
  const float Wxx = dot3(T00, R00, T01, R01, T02, R02);
  const float Wyy = dot3(T10, R10, T11, R11, T12, R12);
  const float Wzz = dot3(T20, R20, T21, R21, T22, R22);
  const float Wxy = dot3(T00, R10, T01, R11, T02, R12);
  const float Wxz = dot3(T00, R20, T01, R21, T02, R22);
  const float Wyz = dot3(T10, R20, T11, R21, T12, R22);
  const float k0 = 0.28209479177387814f, k1 = 0.48860251190291992f, k2 = 1.09254843059207907f,
              k20 = 0.31539156525252005f, k22 = 0.54627421529603959f;
  const float I[9] = {k0 * om, k1 * mwy, k1 * mwz, k1 * mwx, k2 * Wxy, k2 * Wyz, k20 * (3.0f * Wzz - om),
                      k2 * Wxz, k22 * (Wxx - Wyy)};
  // the 27 wave sums of c_ch I_l as one transpose-reduce: at each butterfly step a lane keeps
  // half of its partial sums (the half its lane bit selects) and adds the partner's copy of that
  // half; after the steps over lane bits 5..1 lane L holds coefficient
  // k = 16 b5 + 8 b4 + 4 b3 + 2 b2 + b1 summed over 32 lanes, and the step over bit 0 completes it
  float v[32];
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    v[3 * l] = c0 * I[l];
    v[3 * l + 1] = c1 * I[l];
    v[3 * l + 2] = c2 * I[l];
  }
#pragma unroll
  for (int k = 27; k < 32; ++k) v[k] = 0.0f;
  uint32_t coef = 0;
  transpose_reduce_step<16>(v, lane, coef);
  transpose_reduce_step<8>(v, lane, coef);
  transpose_reduce_step<4>(v, lane, coef);
  transpose_reduce_step<2>(v, lane, coef);
  transpose_reduce_step<1>(v, lane, coef);
  const float out = v[0] + __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(v[0]), 0xB1, 0xF, 0xF, false));
  if ((lane & 1u) == 0u && coef < 28u) sh[(size_t)p * 28 + coef] = coef < 27u ? out : 0.0f;}

// kGatherWaves independent waves per block, wave w of block b gathering probe b * kGatherWaves + w
// with its own LDS: the waves share no data, so they order their LDS accesses with wave-level
// barriers and a block holds several probes (a single-wave block per probe is launched at a
// third of the rate)
template <int MAXR>
__global__ __launch_bounds__(64 * kGatherWaves) void k_gather_sh(const uint32_t* mask, const float4* pnrm,
                                                                 const uint4* rec, const float4* L,
                                                                 const float4* tnrm, const float4* mats,
                                                                 const float* moments, uint32_t P, uint32_t R,
                                                                 float s0, float s1, float s2, LearnedGatherIn lg,
                                                                 uint32_t do_sh, const uint32_t* hist,
                                                                 const uint32_t* traced, const float4* recon,
                                                                 const float4* prev_atlas, const float* prev_sh,
                                                                 float4* atlas, float* sh) {
  __shared__ float rv_s[kGatherWaves][MAXR][4];
  __shared__ uint32_t rc_s[kGatherWaves][MAXR];
  __shared__ float cs_s[kGatherWaves][64][4];
  __shared__ uint32_t cn_s[kGatherWaves][64];
  __shared__ unsigned long long cm_s[kGatherWaves][64];
  const uint32_t wv = threadIdx.x >> 6;
  float (*rv)[4] = rv_s[wv];
  uint32_t* rc = rc_s[wv];
  float (*cs)[4] = cs_s[wv];
  uint32_t* cn = cn_s[wv];
  unsigned long long* cm = cm_s[wv];
  const uint32_t p = blockIdx.x * kGatherWaves + wv;
  const uint32_t lane = threadIdx.x & 63u;
  if (p >= P) return;
  // the ray records are read once the probe is known to be traced (a third of the probes of
  // an outdoor view are sky, whose records hold nothing); the cell moments of the SH projection
  // are loaded where they are used (held from the start they cost a wave of occupancy)
  const float4 pn = pnrm[p];
  if (mask[p] == kSentinel) {
    atlas[(size_t)p * 64 + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (do_sh && lane < 28) sh[(size_t)p * 28 + lane] = 0.0f;
    return;
  }
  if (traced && traced[p] == 0u) {
    // a kept probe that traces nothing this frame (temporal upscaling) keeps the radiance of
    // the probe it was reprojected from; with ray guiding, the reconstruction, its empty
    // cells filled with the mean of the others (summed in ascending cell order)
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    if (recon) {
      const float4 r = recon[(size_t)p * 64 + lane];
      const bool has = r.w >= 0.0f;
      const uint64_t pop = __ballot(has);
      const float m0 = wave_pair_sum(has ? r.x : 0.0f), m1 = wave_pair_sum(has ? r.y : 0.0f);
      const float m2 = wave_pair_sum(has ? r.z : 0.0f), m3 = wave_pair_sum(has ? r.w : 0.0f);
      if (has) {
        q = r;
      } else if (pop) {
        const float inv = 1.0f / (float)__popcll(pop);
        q = make_float4(m0 * inv, m1 * inv, m2 * inv, m3 * inv);
      }
    } else {
      const uint32_t hp = hist ? hist[p] : kSentinel;
      if (hp != kSentinel) {
        atlas[(size_t)p * 64 + lane] = prev_atlas[(size_t)hp * 64 + lane];
        // SH reprojection (Section 2.4.2): the copied atlas keeps its SH as well, as the
        // world-space radiance it was, without a new projection
        if (do_sh && lane < 28) sh[(size_t)p * 28 + lane] = prev_sh[(size_t)hp * 28 + lane];
        return;
      }
    }
    atlas[(size_t)p * 64 + lane] = q;
    if (do_sh) probe_sh(p, lane, pnrm[p], load_moments(moments, lane), q.x, q.y, q.z, sh);
    return;
  }
  uint4 rr0 = make_uint4(0u, 0u, 0u, 0u);
  if (lane < R) rr0 = rec[(size_t)p * R + lane];
  // a ray's value: the sky on a miss, else the hit's front-face emission plus the cached
  // radiance of its cell (or the surrogate's); .w = the travelled distance
  auto ray_value = [&](const uint4 r, uint32_t j) -> float4 {
    if (!(r.w & GI_RAY_HIT)) return make_float4(s0, s1, s2, __uint_as_float(r.y));
    float le0 = 0.f, le1 = 0.f, le2 = 0.f;
    if (r.w & GI_RAY_EMIT) {
      const float4 e = mats[2 * __float_as_uint(tnrm[r.z].w) + 1];
      le0 = e.x; le1 = e.y; le2 = e.z;
    }
    float l0 = 0.f, l1 = 0.f, l2 = 0.f;
    const bool confident = (int32_t)r.x >= 0 && lg.meta && lg.meta[r.x].x >= 64u;
    if (lg.lmlp && (lg.flags[4] == 0.0f || !confident)) {
      // learned mode: the surrogate's radiance at this hit, unless the judge fell back to the
      // plain cache and this hit's cell is confident
      const float4 lv = lg.lmlp[(size_t)p * R + j];
      l0 = lv.x; l1 = lv.y; l2 = lv.z;
    } else if ((int32_t)r.x >= 0) {
      const float4 lv = L[r.x];
      l0 = lv.x; l1 = lv.y; l2 = lv.z;
    }
    return make_float4(le0 + l0, le1 + l1, le2 + l2, __uint_as_float(r.y));
  };
  // per-cell sums in ray order (the same float32 order as a sequential loop over the rays from
  // zero); lane k then holds cell k's sums a0..a3 and ray count
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  uint32_t cnt = 0;
  if (MAXR <= 64) {
    // lane j holds ray j.  The rays of each cell are marked in a per-cell lane mask (an LDS OR,
    // whose result does not depend on order); the cell's first ray folds the others into its
    // value, reading up to three of them at a time and adding them in ascending order
    const bool on = lane < R;
    const uint32_t c = rr0.w & 63u;
    const float4 v = on ? ray_value(rr0, lane) : make_float4(0.f, 0.f, 0.f, 0.f);
    rv[lane][0] = v.x; rv[lane][1] = v.y; rv[lane][2] = v.z; rv[lane][3] = v.w;
    cm[lane] = 0ull;
    wave_sync();
    if (on) atomicOr(&cm[c], 1ull << lane);
    wave_sync();
    const uint64_t mine = cm[lane];
    const uint64_t same = on ? cm[c] : 0ull;
    cnt = (uint32_t)__popcll(mine);
    if (on && (uint32_t)__ffsll((long long)same) - 1u == lane) {
      float x0 = 0.0f + v.x, x1 = 0.0f + v.y, x2 = 0.0f + v.z, x3 = 0.0f + v.w;
      uint64_t m = same & (same - 1u);
      while (m) {
        const uint32_t i1 = (uint32_t)__ffsll((long long)m) - 1u;
        m &= m - 1u;
        const bool h2 = m != 0u;
        const uint32_t i2 = h2 ? (uint32_t)__ffsll((long long)m) - 1u : i1;
        m &= m - 1u;
        const bool h3 = m != 0u;
        const uint32_t i3 = h3 ? (uint32_t)__ffsll((long long)m) - 1u : i1;
        m &= m - 1u;
        const float y10 = rv[i1][0], y11 = rv[i1][1], y12 = rv[i1][2], y13 = rv[i1][3];
        const float y20 = rv[i2][0], y21 = rv[i2][1], y22 = rv[i2][2], y23 = rv[i2][3];
        const float y30 = rv[i3][0], y31 = rv[i3][1], y32 = rv[i3][2], y33 = rv[i3][3];
        x0 = x0 + y10; x1 = x1 + y11; x2 = x2 + y12; x3 = x3 + y13;
        if (h2) { x0 = x0 + y20; x1 = x1 + y21; x2 = x2 + y22; x3 = x3 + y23; }
        if (h3) { x0 = x0 + y30; x1 = x1 + y31; x2 = x2 + y32; x3 = x3 + y33; }
      }
      cs[c][0] = x0; cs[c][1] = x1; cs[c][2] = x2; cs[c][3] = x3;
    }
    wave_sync();
    if (cnt) {
      a0 = cs[lane][0]; a1 = cs[lane][1]; a2 = cs[lane][2]; a3 = cs[lane][3];
    }
  } else {
    for (uint32_t j = lane; j < R; j += 64) {
      const uint4 r = j == lane ? rr0 : rec[(size_t)p * R + j];
      const float4 v = ray_value(r, j);
      rv[j][0] = v.x; rv[j][1] = v.y; rv[j][2] = v.z; rv[j][3] = v.w;
      rc[j] = r.w & 63u;
    }
    cs[lane][0] = cs[lane][1] = cs[lane][2] = cs[lane][3] = 0.0f;
    cn[lane] = 0u;
    wave_sync();
    // in each chunk of 64 rays, the lanes whose rays share a cell are found with one ballot per
    // bit of the cell id, and the first of them folds their rays, in ascending order, into the
    // cell's running sums
    for (uint32_t base = 0; base < R; base += 64u) {
      const uint32_t j = base + lane;
      const bool on = j < R;
      const uint32_t c = on ? rc[j] : 0u;
      uint64_t same = __ballot(on);
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        const uint64_t mb = __ballot(on && ((c >> b) & 1u));
        same &= ((c >> b) & 1u) ? mb : ~mb;
      }
      if (on && (uint32_t)__ffsll((long long)same) - 1u == lane) {
        float x0 = cs[c][0], x1 = cs[c][1], x2 = cs[c][2], x3 = cs[c][3];
        uint32_t k = cn[c];
        uint64_t m = same;
        while (m) {
          const uint32_t i = base + (uint32_t)__ffsll((long long)m) - 1u;
          m &= m - 1u;
          x0 = x0 + rv[i][0]; x1 = x1 + rv[i][1]; x2 = x2 + rv[i][2]; x3 = x3 + rv[i][3];
          ++k;
        }
        cs[c][0] = x0; cs[c][1] = x1; cs[c][2] = x2; cs[c][3] = x3;
        cn[c] = k;
      }
      wave_sync();
    }
    a0 = cs[lane][0]; a1 = cs[lane][1]; a2 = cs[lane][2]; a3 = cs[lane][3];
    cnt = cn[lane];
  }
  float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
  if (cnt) {
    // every mean is its sum times the rounded reciprocal of its count
    const float inv = 1.0f / (float)cnt;
    c0 = a0 * inv; c1 = a1 * inv; c2 = a2 * inv; c3 = a3 * inv;
  }
  const uint64_t populated = __ballot(cnt != 0u);
  if (populated != ~0ull && populated != 0ull) {
    // radiance backup: the mean of the populated cells (a balanced pairwise sum over the 64
    // cells, empty ones counting as zero: the probe filter's decisions depend on these bits)
    const float inv = 1.0f / (float)__popcll(populated);
    const float b0 = wave_pair_sum(c0) * inv, b1 = wave_pair_sum(c1) * inv;
    const float b2 = wave_pair_sum(c2) * inv, b3 = wave_pair_sum(c3) * inv;
    if (!cnt) {
      c0 = b0; c1 = b1; c2 = b2; c3 = b3;
    }
  }
  if (recon || hist) {
    // Algorithm 3: biased shadow-preserving hysteresis against the history: the reprojected
    // probe's atlas, or with ray guiding the reconstruction (its empty cells keep the new value)
    const uint32_t hp = recon ? 0u : hist[p];
    const float4 q = recon ? recon[(size_t)p * 64 + lane]
                           : (hp != kSentinel ? prev_atlas[(size_t)hp * 64 + lane] : make_float4(0.f, 0.f, 0.f, -1.f));
    if (recon ? q.w >= 0.0f : hp != kSentinel) {
      const float third = 1.0f / 3.0f;
      const float l1 = (c0 * third + c1 * third) + c2 * third;
      const float l2 = (q.x * third + q.y * third) + q.z * third;
      float a = fmaxf((l1 - l2) - fminf(l1, l2), 0.0f) / fmaxf(fmaxf(l1, l2), 1e-4f);
      a = a < 0.0f ? 0.0f : (a > 0.95f ? 0.95f : a);
      a = a * a;
      c0 = c0 + a * (q.x - c0);
      c1 = c1 + a * (q.y - c1);
      c2 = c2 + a * (q.z - c2);
      c3 = c3 + a * (q.w - c3);
    }
  }
  atlas[(size_t)p * 64 + lane] = make_float4(c0, c1, c2, c3);
  if (do_sh) probe_sh(p, lane, pn, load_moments(moments, lane), c0, c1, c2, sh);
}

// Algorithm 4: first valid probe of the probe-mask MIP chain at a tile offset from a pixel's tile
__device__ inline uint32_t find_closest_probe(const uint32_t* mask, const MipInfo& mi, int32_t px, int32_t py,
                                              int32_t ox, int32_t oy) {
  int32_t x = px >> 3, y = py >> 3;
  for (uint32_t m = 0; m < mi.n; ++m) {
    const int32_t qx = x + ox, qy = y + oy;
    if (qx < 0 || qy < 0 || qx >= (int32_t)mi.w[m] || qy >= (int32_t)mi.h[m]) break;
    const uint32_t v = mask[mi.off[m] + (uint32_t)qy * mi.w[m] + (uint32_t)qx];
    if (v != kSentinel) return v;
    x >>= 1;
    y >>= 1;
  }
  return kSentinel;
}

// ------------------------------------------------------------------------------------------
// Probe-space filter (Section 2.1.6, Algorithm 5): separable 7x7 sparse blur of the atlas, one
// pass along x, then one along y (which also projects the result to SH).  One wave per probe,
// lane = cell.  For each tap at -1, +1, -2, +2, -3, +3 tiles, Algorithm 4 finds the probe in
// that direction (the same for every lane); its cell of the same index contributes unless the
// plane distance exceeds the probe's cell size (Algorithm 6), the cell direction points below
// the neighbour's surface, or the neighbour's hit point (at the smaller travelled distance) is
// seen more than pi/50 away from the cell direction.  Depth weight cs / (cs + |d_q - d_p|);
// the travelled distance is re-averaged after each contribution.  The cell direction is the
// normalised centre of the hemi-octahedral cell in the probe frame.
// ------------------------------------------------------------------------------------------

template <bool VERTICAL>
__global__ __launch_bounds__(64) void k_filter_probes(const uint32_t* mask, MipInfo mi, uint32_t TW, const float4* ppos,
                                                      const float4* pnrm, const float4* in, float4* out, float cx,
                                                      float cy, float cz, float kappa, const float* moments,
                                                      float* sh) {
  __shared__ uint32_t tap_q[6];        // neighbour probe of each tap (sentinel: none, or off the plane)
  __shared__ float4 tap_w[6], tap_n[6];
  const uint32_t p = blockIdx.x, lane = threadIdx.x;
  const float4 self = in[(size_t)p * 64 + lane];
  const uint32_t m = mask[p];
  if (m == kSentinel) {
    out[(size_t)p * 64 + lane] = self;
    if (VERTICAL && lane < 28) sh[(size_t)p * 28 + lane] = 0.0f;
    return;
  }
  const int32_t px = (int32_t)(m & 0xFFFFu), py = (int32_t)(m >> 16);
  const float4 wp = ppos[p], np = pnrm[p];
  const float ex = wp.x - cx, ey = wp.y - cy, ez = wp.z - cz;
  const float cs = kappa * sqrtf((ex * ex + ey * ey) + ez * ez);
  // the six searches and the plane test are the same for every cell: lanes 0..5 take one tap
  // each and publish the neighbour
  if (lane < 6) {
    const int32_t step = (((lane & 1) << 1) - 1) * ((lane >> 1) + 1);
    const uint32_t qm = find_closest_probe(mask, mi, px, py, VERTICAL ? 0 : step, VERTICAL ? step : 0);
    uint32_t q = kSentinel;
    if (qm != kSentinel) {
      const uint32_t qi = ((qm >> 16) >> 3) * TW + ((qm & 0xFFFFu) >> 3);
      const float4 wq = ppos[qi];
      const float pd = fabsf(((wq.x - wp.x) * np.x + (wq.y - wp.y) * np.y) + (wq.z - wp.z) * np.z);
      tap_w[lane] = wq;
      tap_n[lane] = pnrm[qi];
      if (!(pd > cs)) q = qi;
    }
    tap_q[lane] = q;
  }
  __syncthreads();
  float4 rqs[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const uint32_t q = tap_q[i];
    rqs[i] = q != kSentinel ? in[(size_t)q * 64 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  float dx, dy, dz;
  cell_centre_direction(lane, np.x, np.y, np.z, dx, dy, dz);
  float r0 = self.x, r1 = self.y, r2 = self.z, r3 = self.w;
  float hit = r3, wsum = 1.0f;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    if (tap_q[i] == kSentinel) continue;
    const float4 wq = tap_w[i], nq = tap_n[i];
    const float nc = (dx * nq.x + dy * nq.y) + dz * nq.z;
    if (nc < 0.0f) continue;
    const float4 rq = rqs[i];
    const float hd = fminf(rq.w, hit);
    const float e0 = (wq.x + dx * hd) - wp.x, e1 = (wq.y + dy * hd) - wp.y, e2 = (wq.z + dz * hd) - wp.z;
    const float el = sqrtf((e0 * e0 + e1 * e1) + e2 * e2);
    if (!(el > 0.0f)) continue;
    const float ang = (dx * (e0 / el) + dy * (e1 / el)) + dz * (e2 / el);
    if (ang < 0.9980267284282716f) continue;
    const float w = cs / (cs + fabsf(wq.w - wp.w));
    r0 = r0 + w * rq.x;
    r1 = r1 + w * rq.y;
    r2 = r2 + w * rq.z;
    r3 = r3 + w * hd;
    wsum = wsum + w;
    hit = r3 / wsum;
  }
  const float o0 = r0 / wsum, o1 = r1 / wsum, o2 = r2 / wsum, o3 = r3 / wsum;
  out[(size_t)p * 64 + lane] = make_float4(o0, o1, o2, o3);
  if (VERTICAL) probe_sh(p, lane, np, load_moments(moments, lane), o0, o1, o2, sh);
}

// ------------------------------------------------------------------------------------------
// Per-pixel interpolation (Section 2.4.1, Algorithms 4 and 6)
// ------------------------------------------------------------------------------------------

// One wave per 8x8 lattice cell of the jittered probe grid (WAVES cells per block, in a row):
// all pixels of a cell share the same four neighbour probes (Algorithm 4 depends only on the
// cell and the offset), so lanes 0..3 find them once and stage their position, normal and
// A_l-weighted SH coefficients in LDS.  The pixel's G-buffer loads are issued first, so their
// latency overlaps the search.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_interpolate(const float4* gpos, const float4* gnrm,
                                                            const uint32_t* gprim, uint32_t W, uint32_t H,
                                                            uint32_t TW, const uint32_t* mask, MipInfo mi,
                                                            const float4* ppos, const float4* pnrm, const float* sh,
                                                            float cx, float cy, float cz, float kappa, int32_t jx,
                                                            int32_t jy, int32_t bx0, int32_t bx1, int32_t by0,
                                                            float4* out, unsigned long long* stats) {
  __shared__ uint32_t nq_s[WAVES][4];
  __shared__ float4 np_s[WAVES][4], nn_s[WAVES][4];
  __shared__ float ash_s[WAVES][4][28];
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  uint32_t* nq = nq_s[wv];
  float4* np4 = np_s[wv];
  float4* nn4 = nn_s[wv];
  float(*ash)[28] = ash_s[wv];
  const int32_t bx = (int32_t)(blockIdx.x * WAVES + wv) + bx0, by = (int32_t)blockIdx.y + by0;
  const int32_t x = 8 * bx + jx + (int32_t)(lane & 7u), y = 8 * by + jy + (int32_t)(lane >> 3);
  const bool on = bx <= bx1 && x >= 0 && y >= 0 && x < (int32_t)W && y < (int32_t)H;
  const uint32_t i = on ? (uint32_t)y * W + (uint32_t)x : 0u;
  uint32_t prim = kMiss;
  float4 pp = make_float4(0.f, 0.f, 0.f, 0.f), pn = pp;
  if (on) {
    prim = gprim[i];
    pp = gpos[i];
    pn = gnrm[i];
  }
  if (lane < 4) {
    const int32_t ox = lane & 1, oy = lane >> 1;
    const uint32_t m = bx <= bx1 ? find_closest_probe(mask, mi, 8 * bx, 8 * by, ox, oy) : kSentinel;
    uint32_t q = kSentinel;
    if (m != kSentinel) {
      q = ((m >> 16) >> 3) * TW + ((m & 0xFFFFu) >> 3);
      np4[lane] = ppos[q];
      nn4[lane] = pnrm[q];
    }
    nq[lane] = q;
  }
  __syncthreads();
  for (uint32_t e = lane; e < 4u * 27u; e += 64u) {
    const uint32_t k = e / 27u, j = e - 27u * k;
    const uint32_t q = nq[k];
    const float A = j < 3u ? 3.14159265358979324f : (j < 12u ? 2.09439510239319549f : 0.78539816339744831f);
    ash[k][j] = q != kSentinel ? A * sh[(size_t)q * 28 + j] : 0.0f;
  }
  __syncthreads();
  bool relaxed = false, none = false;
  if (on) {
    if (prim == kMiss) {
      out[i] = make_float4(0.f, 0.f, 0.f, GI_INTERP_SKY);
    } else {
      const float dx = pp.x - cx, dy = pp.y - cy, dz = pp.z - cz;
      const float cell_size = kappa * sqrtf((dx * dx + dy * dy) + dz * dz);
      const float fx = (float)(lane & 7u) * 0.125f, fy = (float)(lane >> 3) * 0.125f;
      const float k0 = 0.28209479177387814f, k1 = 0.48860251190291992f, k2 = 1.09254843059207907f,
                  k20 = 0.31539156525252005f, k22 = 0.54627421529603959f;
      const float Y[9] = {k0, k1 * pn.y, k1 * pn.z, k1 * pn.x, k2 * (pn.x * pn.y), k2 * (pn.y * pn.z),
                          k20 * (3.0f * (pn.z * pn.z) - 1.0f), k2 * (pn.x * pn.z), k22 * (pn.x * pn.x - pn.y * pn.y)};
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, ws = 0.f;
      float r0 = 0.f, r1 = 0.f, r2 = 0.f;   // equal-weight sum for the relaxed fallback
      int nf = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (nq[k] == kSentinel) continue;
        const int32_t ox = k & 1, oy = k >> 1;
        const float4 qp = np4[k], qn = nn4[k];
        const float wb = (ox ? fx : 1.0f - fx) * (oy ? fy : 1.0f - fy);
        const float pd = fabsf(((qp.x - pp.x) * pn.x + (qp.y - pp.y) * pn.y) + (qp.z - pp.z) * pn.z);
        const float nd = (pn.x * qn.x + pn.y * qn.y) + pn.z * qn.z;
        const float w = (pd <= cell_size) ? wb * fmaxf(0.0f, nd) : 0.0f;
        // irradiance from the probe's SH at this pixel's normal: sum over l of (A_l c_l) Y_l(n)
        // (values compared within a tolerance: fused multiply-adds; the weights, which decide
        // the pixel's flag, stay as written)
        float E0 = 0.f, E1 = 0.f, E2 = 0.f;
#pragma unroll
        for (int l = 0; l < 9; ++l) {
          E0 = fmaf(ash[k][3 * l], Y[l], E0);
          E1 = fmaf(ash[k][3 * l + 1], Y[l], E1);
          E2 = fmaf(ash[k][3 * l + 2], Y[l], E2);
        }
        r0 = r0 + E0; r1 = r1 + E1; r2 = r2 + E2;
        a0 = fmaf(w, E0, a0); a1 = fmaf(w, E1, a1); a2 = fmaf(w, E2, a2);
        ws = ws + w;
        ++nf;
      }
      if (ws > 0.0f) {
        out[i] = make_float4(a0 / ws, a1 / ws, a2 / ws, GI_INTERP_OK);
      } else if (nf > 0) {
        const float fn = (float)nf;
        out[i] = make_float4(r0 / fn, r1 / fn, r2 / fn, GI_INTERP_RELAXED);
        relaxed = true;
      } else {
        out[i] = make_float4(0.f, 0.f, 0.f, GI_INTERP_NO_PROBE);
        none = true;
      }
    }
  }
  stat_add(stats, GI_STAT_RELAXED, relaxed);
  stat_add(stats, GI_STAT_NOPROBE, none);
}

// ------------------------------------------------------------------------------------------
// Lookup-only query for caller points
// ------------------------------------------------------------------------------------------
// ------------------------------------------------------------------------------------------
// Two-level cache update (Section 2.2.3): a workgroup of 512 updates 8 consecutive slots.
// Entries are cell-major (see cache_entry): one cache line holds one cell of 8 consecutive
// slots, so thread (wave w, lane l) takes cell 8 w + l / 8 of slot l % 8 and every load or
// store of a wave covers 8 whole lines.  Phase 1: each cell's moving average as in
// k_cache_update, the tile's life and eviction, level 0 into LDS.  Phase 2: MIP levels 4x4,
// 2x2, 1x1 of the 8 tiles as sample-weighted means of their 2x2 children (children in raster
// order).  Phase 3: each cell's radiance for readers from the finest of its level and its
// parents that holds at least tile_min samples, else the coarsest level if it holds any, else
// zero.  Every thread reaches every barrier; empty and evicted tiles skip the work.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_cache_update_tiles(uint32_t* fp, uint64_t* key, uint4* acc, float4* L,
                                                            uint32_t* cn, float4* Lq, uint2* meta, uint32_t* accessed,
                                                            uint32_t n_cap, uint32_t max_life, uint32_t frac_bits,
                                                            uint32_t tile_min, unsigned long long* stats) {
  __shared__ float lv[8][85][3];   // per tile: level 0 at 0..63, 1 at 64..79, 2 at 80..83, 3 at 84
  __shared__ uint32_t nv[8][85];
  __shared__ uint32_t keep_s[8], live_s[8], life_s[8];
  const uint32_t t = threadIdx.x, w = t >> 6, l = t & 63u;
  const uint32_t j = l & 7u, cell = 8u * w + (l >> 3);
  const uint32_t N = gridDim.x * 8u;
  const uint32_t s = blockIdx.x * 8u + j;
  const size_t e = (size_t)cell * N + s;
  // the tile's state, read once before the thread of cell 0 rewrites it
  if (t < 8u) {
    const uint32_t st = blockIdx.x * 8u + t;
    keep_s[t] = 0u;
    live_s[t] = fp[st] != 0u;
    life_s[t] = live_s[t] ? (accessed[st] ? max_life : meta[st].y - 1u) : 0u;
  }
  __syncthreads();
  if (live_s[j]) {
    const uint4 a = acc[e];
    float4 lc = L[e];
    uint32_t nh = cn[e];
    if (a.w > 0u) {
      const uint32_t h = nh < n_cap ? nh : n_cap;
      const float wt = (float)a.w / (float)((double)h + (double)a.w);
      const double den = (double)a.w * (double)(1u << frac_bits);
      const float m0 = (float)((double)a.x / den);
      const float m1 = (float)((double)a.y / den);
      const float m2 = (float)((double)a.z / den);
      lc.x = lc.x + wt * (m0 - lc.x);
      lc.y = lc.y + wt * (m1 - lc.y);
      lc.z = lc.z + wt * (m2 - lc.z);
      const uint64_t u = (uint64_t)nh + a.w;
      nh = u < n_cap ? (uint32_t)u : n_cap;
    }
    acc[e] = make_uint4(0u, 0u, 0u, 0u);
    const uint32_t life = life_s[j];
    unsigned long long* st = stats + (s % kStatStripes) * GI_STAT_COUNT;
    if (life == 0u) {
      L[e] = make_float4(0.f, 0.f, 0.f, 0.f);
      cn[e] = 0u;
      Lq[e] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (cell == 0u) {
        fp[s] = 0u;
        key[s] = 0u;
        meta[s] = make_uint2(0u, 0u);
        accessed[s] = 0u;
        atomicAdd(&st[GI_STAT_EVICT], 1ull);
      }
    } else {
      L[e] = lc;
      cn[e] = nh;
      if (cell == 0u) {
        meta[s] = make_uint2(0u, life);
        accessed[s] = 0u;
        keep_s[j] = 1u;
        atomicAdd(&st[GI_STAT_LIVE], 1ull);
      }
      lv[j][cell][0] = lc.x;
      lv[j][cell][1] = lc.y;
      lv[j][cell][2] = lc.z;
      nv[j][cell] = nh;
    }
  }
  __syncthreads();
  // level k + 1 (side 8 >> (k+1), 8 tiles x side^2 entries) from level k (side 8 >> k)
  const uint32_t base[4] = {0u, 64u, 80u, 84u};
#pragma unroll
  for (uint32_t k = 0; k < 3; ++k) {
    const uint32_t side = 8u >> (k + 1u), per = side * side;
    if (t < 8u * per) {
      const uint32_t tj = t / per, i = t % per;
      if (keep_s[tj]) {
        const uint32_t x = i % side, y = i / side;
        float w0 = 0.f, w1 = 0.f, w2 = 0.f;
        uint32_t ns = 0u;
#pragma unroll
        for (uint32_t c = 0; c < 4; ++c) {
          const uint32_t ch = base[k] + (2u * y + (c >> 1)) * (2u * side) + (2u * x + (c & 1u));
          const float fn = (float)nv[tj][ch];
          w0 = w0 + fn * lv[tj][ch][0];
          w1 = w1 + fn * lv[tj][ch][1];
          w2 = w2 + fn * lv[tj][ch][2];
          ns += nv[tj][ch];
        }
        const uint32_t o = base[k + 1u] + i;
        nv[tj][o] = ns;
        lv[tj][o][0] = ns ? w0 / (float)ns : 0.0f;
        lv[tj][o][1] = ns ? w1 / (float)ns : 0.0f;
        lv[tj][o][2] = ns ? w2 / (float)ns : 0.0f;
      }
    }
    __syncthreads();
  }
  if (!keep_s[j]) return;
  const uint32_t x = cell & 7u, y = cell >> 3;
  int32_t pick = -1;
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    const uint32_t o = base[k] + (y >> k) * (8u >> k) + (x >> k);
    if (pick < 0 && nv[j][o] >= tile_min) pick = (int32_t)o;
  }
  if (pick < 0 && nv[j][84] > 0u) pick = 84;
  Lq[e] = pick < 0 ? make_float4(0.f, 0.f, 0.f, 0.f)
                   : make_float4(lv[j][pick][0], lv[j][pick][1], lv[j][pick][2], 0.f);
}

__global__ void k_query(const float4* pos, const float4* nrm, uint32_t n, CacheArgs c, float4* out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 p = pos[i], q = nrm[i];
  const bool wl = p.w >= 0.0f;
  uint32_t tcell;
  const uint64_t key = descriptor(c.cell_scale, c.leak_bit, c.lod_scale, c.cam[0], c.cam[1], c.cam[2], p.x, p.y, p.z,
                                  q.x, q.y, q.z, wl ? p.w : 0.0f, wl, c.tiled, tcell);
  const int32_t s = cache_entry(c, table_lookup(c, key), tcell);
  if (s < 0) {
    out[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    const float4 l = c.L[s];
    out[i] = make_float4(l.x, l.y, l.z, 1.0f);
  }
}

// traversal only
template <int STACK>
__global__ __launch_bounds__(kTraceBlock) void k_trace_rays(SceneView sv, const float4* o, const float4* d, uint32_t n,
                                                            uint32_t any, uint32_t* tri, float* t) {
  __shared__ uint32_t stk[STACK * kTraceBlock];
  __shared__ uint16_t stkt[STACK * kTraceBlock];
  TStack<STACK, kTraceBlock> ts(stk + threadIdx.x, stkt + threadIdx.x, sv.spill + (blockIdx.x * kTraceBlock + threadIdx.x), sv.spill_stride);
  const uint32_t i = blockIdx.x * kTraceBlock + threadIdx.x;
  if (i >= n) return;
  const float4 a = o[i], b = d[i];
  const RayQ r = make_ray(a.x, a.y, a.z, b.x, b.y, b.z);
  if (any) {
    tri[i] = any_hit<STACK, kTraceBlock>(sv, r, a.w, ts) ? 1u : 0u;
    t[i] = 0.0f;
  } else {
    uint32_t h;
    float tt;
    closest_hit<STACK, kTraceBlock>(sv, r, a.w, ts, h, tt);
    tri[i] = h;
    t[i] = tt;
  }
}

// instrumented copy of the probe-ray and shadow-ray walks: nodes visited and triangles
// tested (the algorithmic traffic of the traversal), no other side effect
template <int STACK>
__global__ __launch_bounds__(kTraceBlock) void k_count_traversal(SceneView sv, ShadeTables st, ProbeRayArgs a,
                                                                 CacheArgs c, const uint4* rec, RestirArgs ra,
                                                                 unsigned long long* out) {
  __shared__ uint32_t stk[STACK * kTraceBlock];
  __shared__ uint16_t stkt[STACK * kTraceBlock];
  TStack<STACK, kTraceBlock> ts(stk + threadIdx.x, stkt + threadIdx.x, sv.spill + (blockIdx.x * kTraceBlock + threadIdx.x), sv.spill_stride);
  const uint32_t gid = blockIdx.x * kTraceBlock + threadIdx.x;
  uint32_t pn = 0, pt = 0, sn = 0, st_ = 0;
  bool probe = false, shadow = false;
  if (gid < a.P * a.R) {
    const uint32_t p = gid / a.R;
    if (a.traced ? a.traced[p] != 0u : a.mask[p] != kSentinel) {
      probe = true;
      float ox, oy, oz, dx, dy, dz;
      uint32_t cell;
      probe_ray(a, gid, p, ox, oy, oz, dx, dy, dz, cell);
      const RayQ r = make_ray(ox, oy, oz, dx, dy, dz);
      uint32_t tri;
      float t;
      closest_hit<STACK, kTraceBlock, true>(sv, r, 3.0e38f, ts, tri, t, &pn, &pt);
      const uint4 rr = rec[gid];
      if (rr.w & GI_RAY_HIT) {
        const float4 n = st.tnrm[tri];
        const float dn = (n.x * dx + n.y * dy) + n.z * dz;
        const float sg = dn > 0.0f ? -1.0f : 1.0f;
        const float yx = ox + t * dx, yy = oy + t * dy, yz = oz + t * dz;
        const float nx = sg * n.x, ny = sg * n.y, nz = sg * n.z;
        const float eps = origin_offset(a.eps_scale, yx, yy, yz);
        const float px = yx + nx * eps, py = yy + ny * eps, pz = yz + nz * eps;
        const LightSample ls = st.lg_list
                                   ? sample_light_ris(st, ra, a.seed, a.frame, gid, yx, yy, yz, px, py, pz, nx, ny, nz)
                                   : sample_light(st, pick_light(st, a.seed, a.frame, gid), px, py, pz, nx, ny, nz);
        if (ls.cast) {
          shadow = true;
          (void)any_hit<STACK, kTraceBlock, true>(sv, ls.ray, ls.tmax, ts, &sn, &st_);
        }
      }
    }
  }
  if (probe) {
    atomicAdd(&out[0], 1ull);
    atomicAdd(&out[1], (unsigned long long)pn);
    atomicAdd(&out[2], (unsigned long long)pt);
  }
  if (shadow) {
    atomicAdd(&out[3], 1ull);
    atomicAdd(&out[4], (unsigned long long)sn);
    atomicAdd(&out[5], (unsigned long long)st_);
  }
}

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_zero_u64(unsigned long long* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
static SceneView scene_view(const gi_context* c) {
  SceneView v;
  v.nodes = c->d_nodes;
  v.tris = c->d_tris;
  v.dyn = c->d_dyn;
  v.n_dyn = c->n_dyn;
  v.has_bvh = c->nt > 0 ? 1u : 0u;
  v.spill = c->d_spill;
  v.spill_stride = c->spill_stride;
  return v;
}

static ShadeTables shade_tables(const gi_context* c) {
  ShadeTables t;
  t.tnrm = c->d_tnrm;
  t.mats = c->d_mats;
  t.etri = c->d_etri;
  t.ethr = c->d_ethr;
  t.evert = c->d_evert;
  t.n_emit = c->n_emit;
  t.area_total = c->area_total;
  t.lg_box = c->cfg.light_grid ? c->d_lg_box : nullptr;
  t.lg_list = c->cfg.light_grid ? c->d_lg_list : nullptr;
  t.lg_count = c->cfg.light_grid ? c->d_lg_count : nullptr;
  t.lg_dim = c->cfg.lgrid_dim;
  t.lg_k = c->cfg.lgrid_k;
  t.ris_m = c->cfg.ris_candidates;
  return t;
}

static ProbeRayArgs probe_args(const gi_context* c) {
  ProbeRayArgs a;
  a.mask = c->d_mask;
  a.traced = c->cfg.upscale > 1 ? c->d_traced : nullptr;
  a.cdf = c->guided ? c->d_cdf : nullptr;
  a.ppos = c->d_ppos;
  a.pnrm = c->d_pnrm;
  a.P = c->P;
  a.R = c->R;
  a.seed = c->cfg.seed;
  a.frame = c->fa.index;
  a.eps_scale = c->cfg.eps_scale;
  a.t_sky = c->cfg.t_sky;
  return a;
}

static HitList hit_list(const gi_context* c) {
  HitList h;
  h.ids = c->d_hit_ids;
  h.count = c->d_hit_count;
  h.stripe_cap = c->hit_stripe_cap;
  h.blocks_per_stripe = c->hit_blocks_per_stripe;
  return h;
}

static CacheArgs cache_args(const gi_context* c) {
  CacheArgs a;
  a.fp = c->tab.fp;
  a.key = c->tab.key;
  a.acc = c->tab.acc;
  a.L = c->cfg.cache_tiles ? c->tab.Lq : c->tab.L;
  a.accessed = c->tab.accessed;
  a.tiled = c->cfg.cache_tiles;
  a.n_slots = c->N;
  a.bucket_mask = c->N / kBucket - 1u;
  a.cell_scale = c->cfg.cell_scale;
  a.leak_bit = c->cfg.leak_bit;
  a.frac_bits = c->cfg.frac_bits;
  a.r_max = c->cfg.r_max;
  a.bounces = c->cfg.bounces;
  a.sky[0] = c->cfg.sky[0];
  a.sky[1] = c->cfg.sky[1];
  a.sky[2] = c->cfg.sky[2];
  a.lod_scale = c->cfg.lod_scale;
  for (int k = 0; k < 3; ++k) a.cam[k] = c->fa.cam[k];
  return a;
}

static RestirArgs restir_args(const gi_context* c) {
  RestirArgs r;
  r.on = c->cfg.restir;
  r.cap = c->cfg.restir_cap * c->cfg.ris_candidates;
  r.has_prev = c->cfg.restir && c->rs_has_prev;
  const uint32_t cur = c->rs_cur, nxt = c->rs_cur ^ 1u;
  r.prev = cache_args(c);
  r.next = r.prev;
  if (c->cfg.restir) {
    const uint32_t mask = ((1u << c->cfg.restir_log2) / kBucket) - 1u;
    r.prev.fp = c->d_rs_fp[cur];
    r.prev.key = c->d_rs_key[cur];
    r.prev.bucket_mask = mask;
    r.next.fp = c->d_rs_fp[nxt];
    r.next.key = c->d_rs_key[nxt];
    r.next.bucket_mask = mask;
    r.pyw = c->d_rs_yw[cur];
    r.pn = c->d_rs_n[cur];
    r.pm = c->d_rs_m[cur];
  } else {
    r.pyw = nullptr;
    r.pn = nullptr;
    r.pm = nullptr;
  }
  r.claim = c->d_rs_claim;
  r.r_yw = c->d_r_rs_yw;
  r.r_n = c->d_r_rs_n;
  r.r_m = c->d_r_rs_m;
  r.r_slot = c->d_r_rs_slot;
  r.cell_scale = c->cfg.cell_scale;
  r.lod_scale = c->cfg.lod_scale;
  for (int k = 0; k < 3; ++k) r.cam[k] = c->fa.cam[k];
  return r;
}

// the per-kernel timers only measure: their events skip the system-scope fence (the cache
// writeback and invalidation it costs would slow the next kernel and lengthen short ones)
static hipError_t timer_event(hipEvent_t* e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

void timer_begin(gi_context* c, const char* name, hipStream_t s, hipEvent_t* a) {
  *a = nullptr;
  if (!c->prof || (c->prof == 2u && std::strcmp(name, "trace_probes") != 0)) return;
  if (c->event_pool.empty()) {
    hipEvent_t e;
    if (timer_event(&e) != hipSuccess) return;
    c->event_pool.push_back(e);
  }
  *a = c->event_pool.back();
  c->event_pool.pop_back();
  (void)hipEventRecord(*a, s);
}

void timer_end(gi_context* c, const char* name, hipStream_t s, hipEvent_t a) {
  if (!c->prof || !a) return;
  hipEvent_t b;
  if (c->event_pool.empty()) {
    if (timer_event(&b) != hipSuccess) return;
  } else {
    b = c->event_pool.back();
    c->event_pool.pop_back();
  }
  (void)hipEventRecord(b, s);
  c->timers.push_back(KernelTimer{name, a, b});
}

#define GI_TIMED(ctx, name, stream, launch_stmt) \
  do {                                            \
    hipEvent_t ev_;                               \
    timer_begin(ctx, name, stream, &ev_);         \
    launch_stmt;                                  \
    timer_end(ctx, name, stream, ev_);            \
  } while (0)

static inline uint32_t blocks(uint64_t n, uint32_t b) { return (uint32_t)((n + b - 1) / b); }

hipError_t launch_gbuffer(gi_context* c, const gi_frame* f, float4* pos, float4* nrm, float4* alb, uint32_t* prim,
                          hipStream_t s) {
  const uint32_t n = c->W * c->H;
    GI_TIMED(c, "gbuffer", s, (k_gbuffer<kLdsStack><<<blocks(n, kTraceBlock), kTraceBlock, 0, s>>>(scene_view(c), shade_tables(c), *f, c->W, c->H, pos, nrm, alb, prim)));
  return hipGetLastError();
}

static MipInfo mip_info(const gi_context* c) {
  MipInfo mi;
  mi.n = c->nmip < 16 ? c->nmip : 16;
  for (uint32_t k = 0; k < 16; ++k) {
    mi.w[k] = k < mi.n ? c->mip_w[k] : 0u;
    mi.h[k] = k < mi.n ? c->mip_h[k] : 0u;
    mi.off[k] = k < mi.n ? c->mip_off[k] : 0u;
  }
  return mi;
}

hipError_t launch_spawn(gi_context* c, const float4* pos, const float4* nrm, const uint32_t* prim, hipStream_t s) {
  const MipInfo mi = mip_info(c);
  const dim3 grid((c->TW + 15u) / 16u, (c->TH + 15u) / 16u);
  c->reprojected = c->cfg.temporal && c->has_prev;
  if (c->reprojected) {
    const gi_frame& pf = c->prev_frame;
    PrevCamera pc;
    for (int k = 0; k < 3; ++k) {
      pc.pos[k] = pf.pos[k];
      pc.fwd[k] = pf.fwd[k];
      pc.right[k] = pf.right[k];
      pc.up[k] = pf.up[k];
    }
    pc.tan_half = pf.tan_half;
    GI_TIMED(c, "reproject", s, (k_reproject<<<c->P, 64, 0, s>>>(pos, nrm, prim, c->W, c->H, c->TW, c->d_prev_mask, c->d_prev_pos, c->d_prev_nrm, pc, c->fa.cam[0], c->fa.cam[1], c->fa.cam[2], c->fa.kappa, c->d_win, c->d_hist)));
  }
  const uint32_t* place = nullptr;
  if (c->cfg.upscale > 1) {
    UpscaleArgs ua;
    ua.W = c->W;
    ua.H = c->H;
    ua.TW = c->TW;
    ua.P = c->P;
    ua.u = c->cfg.upscale;
    ua.sjx = c->fa.sjx;
    ua.sjy = c->fa.sjy;
    ua.seed = c->cfg.seed;
    ua.frame = c->fa.index;
    const uint32_t nb = (c->P + 255u) / 256u;
    const uint32_t* win = c->reprojected ? c->d_win : nullptr;
    GI_TIMED(c, "upscale_classify", s, (k_upscale_classify<<<nb, 256, 0, s>>>(prim, ua, win, c->d_place, c->d_traced, c->d_cls, c->d_assigned)));
    GI_TIMED(c, "upscale_list", s, (k_upscale_list<<<1, 1024, 0, s>>>(c->d_cls, c->P, c->d_over, c->d_over_count)));
    GI_TIMED(c, "upscale_pick", s, (k_upscale_pick<<<nb, 256, 0, s>>>(c->d_cls, ua, c->d_over, c->d_over_count, c->d_assigned)));
    GI_TIMED(c, "upscale_apply", s, (k_upscale_apply<<<nb, 256, 0, s>>>(prim, ua, c->d_over, c->d_over_count, c->d_assigned, c->d_place, c->d_traced)));
    place = c->d_place;
  }
  GI_TIMED(c, "spawn", s, (k_spawn_mips<<<grid, 256, 0, s>>>(pos, nrm, prim, c->W, c->H, c->TW, c->TH, c->fa.jx, c->fa.jy, mi, c->reprojected ? c->d_win : nullptr, place, c->d_mask, c->d_ppos, c->d_pnrm, c->d_stats, c->d_hit_count)));
  if (mi.n > 5) GI_TIMED(c, "mask_mip", s, (k_mask_mips_top<<<1, 1024, 0, s>>>(mi, c->d_mask)));
  c->guided = c->reprojected && c->cfg.ray_guiding;
  if (c->guided) {
    const gi_frame& pf = c->prev_frame;
    PrevCamera pc;
    for (int k = 0; k < 3; ++k) {
      pc.pos[k] = pf.pos[k];
      pc.fwd[k] = pf.fwd[k];
      pc.right[k] = pf.right[k];
      pc.up[k] = pf.up[k];
    }
    pc.tan_half = pf.tan_half;
    GI_TIMED(c, "reconstruct", s, (k_reconstruct<<<c->P, 64, 0, s>>>(c->d_mask, c->d_ppos, c->d_pnrm, c->W, c->H, c->TW, c->TH, pc, c->fa.cam[0], c->fa.cam[1], c->fa.cam[2], c->fa.kappa, c->d_prev_mask, c->d_prev_pos, c->d_prev_nrm, c->d_prev_atlas, c->d_recon, c->d_cdf)));
  }
  return hipGetLastError();
}

hipError_t launch_trace(gi_context* c, hipStream_t s) {
  const uint64_t n = (uint64_t)c->P * c->R;
  const SceneView sv = scene_view(c);
  const ShadeTables st = shade_tables(c);
  const ProbeRayArgs a = probe_args(c);
  const CacheArgs ca = cache_args(c);
  const LearnedShadeOut lso = learned_shade_out(c);
  if (lso.tflag) k_zero_u32<<<blocks(lso.tflag_words, 256), 256, 0, s>>>(reinterpret_cast<uint32_t*>(lso.tflag), lso.tflag_words);
  GI_TIMED(c, "trace_probes", s, (k_trace_probes<kLdsStack><<<blocks(n, kTraceBlock), kTraceBlock, 0, s>>>(sv, st, a, c->d_rec, c->d_rkey, hit_list(c), c->d_stats)));
  const RestirArgs ra = restir_args(c);
  if (ra.on) {
    const uint32_t NR = 1u << c->cfg.restir_log2;
    GI_TIMED(c, "restir_clear", s, (k_restir_clear<<<blocks(NR, 256), 256, 0, s>>>(ra.next.fp, ra.next.key, ra.claim, NR)));
  }
  if (c->cfg.light_grid) {
    // the light grid over this frame's hit points, before the shading that samples it
    const uint32_t nb = blocks(n, 256);
    GI_TIMED(c, "lg_box", s, (k_lg_box_partial<<<nb, 256, 0, s>>>(a, c->d_rec, c->d_lg_part)));
    GI_TIMED(c, "lg_box_final", s, (k_lg_box_final<<<1, 1024, 0, s>>>(c->d_lg_part, nb, c->d_lg_box)));
    const uint32_t G = c->cfg.lgrid_dim;
    GI_TIMED(c, "light_grid", s, (k_light_grid<<<G * G * G, 64, 0, s>>>(st, c->n_emit, c->cfg.lgrid_threshold, c->d_lg_list, c->d_lg_count)));
  }
  GI_TIMED(c, "shade_hits", s, (k_shade_hits<kLdsStack><<<blocks(n, kTraceBlock), kTraceBlock, 0, s>>>(sv, st, a, ca, c->d_rec, c->d_rkey, hit_list(c), learned_shade_out(c), ra, c->d_stats)));
  if (ra.on) {
    // this frame's reservoirs into the written table (the lowest ray id per slot), which the
    // next frame reads
    GI_TIMED(c, "restir_store", s, (k_restir_store<<<blocks(n, 256), 256, 0, s>>>(c->d_rec, (uint32_t)n, ra, c->d_rs_yw[c->rs_cur ^ 1u], c->d_rs_n[c->rs_cur ^ 1u], c->d_rs_m[c->rs_cur ^ 1u])));
    c->rs_cur ^= 1u;
    c->rs_has_prev = true;
  }
  return hipGetLastError();
}

hipError_t launch_update(gi_context* c, hipStream_t s) {
  if (c->cfg.cache_tiles) {
    GI_TIMED(c, "cache_update_tiles", s, (k_cache_update_tiles<<<c->N / 8u, 512, 0, s>>>(c->tab.fp, c->tab.key, c->tab.acc, c->tab.L, c->tab.cn, c->tab.Lq, c->tab.meta, c->tab.accessed, c->cfg.n_cap, c->cfg.max_life, c->cfg.frac_bits, c->cfg.tile_min_samples, c->d_stats)));
  } else {
    GI_TIMED(c, "cache_update", s, (k_cache_update<<<blocks(c->N, 256 * kUpdateSlots), 256, 0, s>>>(c->N, c->tab.fp, c->tab.key, c->tab.acc, c->tab.L, c->tab.meta, c->tab.accessed, c->cfg.n_cap, c->cfg.max_life, c->cfg.frac_bits, c->d_stats)));
  }
  if (c->learned && c->cfg.cache_mode != GI_CACHE_PLAIN) {
    // the surrogate's radiance at every hit, then the judge against confident plain cells
    const hipError_t e = learned_infer_rays(c, s);
    if (e != hipSuccess) return e;
  }
  const uint32_t filt = c->cfg.probe_filter;
#define GI_GATHER_ARGS c->d_mask, c->d_pnrm, c->d_rec, c->cfg.cache_tiles ? c->tab.Lq : c->tab.L, c->d_tnrm, c->d_mats, c->d_moments, c->P, c->R, c->cfg.sky[0], c->cfg.sky[1], c->cfg.sky[2], learned_gather_in(c), filt ? 0u : 1u, c->reprojected ? c->d_hist : nullptr, c->cfg.upscale > 1 ? c->d_traced : nullptr, c->guided ? c->d_recon : nullptr, c->d_prev_atlas, c->d_prev_sh, c->d_atlas, c->d_sh
  const uint32_t gb = blocks(c->P, kGatherWaves);
  if (c->R <= 64u)
    GI_TIMED(c, "gather_sh", s, (k_gather_sh<64><<<gb, 64 * kGatherWaves, 0, s>>>(GI_GATHER_ARGS)));
  else
    GI_TIMED(c, "gather_sh", s, (k_gather_sh<kGatherMaxR><<<gb, 64 * kGatherWaves, 0, s>>>(GI_GATHER_ARGS)));
#undef GI_GATHER_ARGS
  if (filt) {
    // Algorithm 5: x pass into the scratch atlas, y pass back (and the SH of the result)
    const MipInfo mi = mip_info(c);
    GI_TIMED(c, "filter_x", s, (k_filter_probes<false><<<c->P, 64, 0, s>>>(c->d_mask, mi, c->TW, c->d_ppos, c->d_pnrm, c->d_atlas, c->d_atlas_tmp, c->fa.cam[0], c->fa.cam[1], c->fa.cam[2], c->fa.kappa, c->d_moments, c->d_sh)));
    GI_TIMED(c, "filter_y", s, (k_filter_probes<true><<<c->P, 64, 0, s>>>(c->d_mask, mi, c->TW, c->d_ppos, c->d_pnrm, c->d_atlas_tmp, c->d_atlas, c->fa.cam[0], c->fa.cam[1], c->fa.cam[2], c->fa.kappa, c->d_moments, c->d_sh)));
  }
  return hipGetLastError();
}

hipError_t launch_interpolate(gi_context* c, const float4* pos, const float4* nrm, const uint32_t* prim, float4* out,
                              hipStream_t s) {
  const MipInfo mi = mip_info(c);
  // lattice cells (base = floor((pixel - jitter) / 8)) that hold at least one pixel
  const int32_t jx = (int32_t)c->fa.jx, jy = (int32_t)c->fa.jy;
  const int32_t bx0 = (0 - jx) >> 3, by0 = (0 - jy) >> 3;
  const int32_t bx1 = ((int32_t)c->W - 1 - jx) >> 3, by1 = ((int32_t)c->H - 1 - jy) >> 3;
  constexpr int kWaves = 4;
  const dim3 grid((uint32_t)(bx1 - bx0 + kWaves) / kWaves, (uint32_t)(by1 - by0 + 1));
  GI_TIMED(c, "interpolate", s, (k_interpolate<kWaves><<<grid, 64 * kWaves, 0, s>>>(pos, nrm, prim, c->W, c->H, c->TW, c->d_mask, mi, c->d_ppos, c->d_pnrm, c->d_sh, c->fa.cam[0], c->fa.cam[1], c->fa.cam[2], c->fa.kappa, jx, jy, bx0, bx1, by0, out, c->d_stats)));
  return hipGetLastError();
}

hipError_t launch_query(gi_context* c, const float4* pos, const float4* nrm, uint32_t n, float4* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  GI_TIMED(c, "cache_query", s, (k_query<<<blocks(n, 256), 256, 0, s>>>(pos, nrm, n, cache_args(c), out)));
  return hipGetLastError();
}

hipError_t launch_trace_rays(gi_context* c, const float4* o, const float4* d, uint32_t n, uint32_t any, uint32_t* tri,
                             float* t, hipStream_t s) {
  if (n == 0) return hipSuccess;
  // the spill array has one column per lane id: launch in chunks of at most its width
  const uint32_t cap = c->spill_stride;
  for (uint32_t off = 0; off < n; off += cap) {
    const uint32_t m = n - off < cap ? n - off : cap;
    GI_TIMED(c, "trace_rays", s, (k_trace_rays<kLdsStack><<<blocks(m, kTraceBlock), kTraceBlock, 0, s>>>(scene_view(c), o + off, d + off, m, any, tri + off, t + off)));
  }
  return hipGetLastError();
}

// Traversal-stack spill rows of gi_trace_rays_noalloc: one fixed array per GPU (the loaded
// code object holds it until the process ends), so that the call allocates nothing.  Host
// code never uses the symbol itself: its device address is looked up once per device, with
// that device current, and kept in scratch_ptr.
static __device__ __align__(256) uint32_t scratch[kNoAllocScratchWords];

static std::mutex scratch_mu;
static uint32_t* scratch_ptr[kMaxDevices] = {};

hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  scratch_ptr[device] = static_cast<uint32_t*>(p);
  return hipSuccess;
}

uint32_t noalloc_chunk_rays(uint32_t spill_rows) {
  if (spill_rows == 0) return 0xFFFFFFFFu;
  const size_t per = kNoAllocScratchWords / spill_rows;   // lane ids one row can hold
  return (uint32_t)(per / kTraceBlock * kTraceBlock);
}

hipError_t launch_trace_rays_noalloc(gi_context* c, const float4* o, const float4* d, uint32_t n, uint32_t any,
                                     uint32_t* tri, float* t, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint32_t* sp = nullptr;
  {
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (c->device >= 0 && c->device < kMaxDevices) sp = scratch_ptr[c->device];
  }
  if (!sp) return hipErrorNotInitialized;
  const uint32_t cap = noalloc_chunk_rays(c->spill_rows);
  if (cap == 0) return hipErrorInvalidValue;
  SceneView v = scene_view(c);
  v.spill = sp;                  // rows of cap lane ids each, in the static array
  v.spill_stride = c->spill_rows ? cap : 0u;
  for (uint32_t off = 0; off < n; off += cap) {
    const uint32_t m = n - off < cap ? n - off : cap;
    // no per-kernel timer here: its events may be created on first use
    k_trace_rays<kLdsStack><<<blocks(m, kTraceBlock), kTraceBlock, 0, s>>>(v, o + off, d + off, m, any, tri + off, t + off);
    if (cap == 0xFFFFFFFFu) break;
  }
  return hipGetLastError();
}

hipError_t launch_count_traversal(gi_context* c, unsigned long long* out, hipStream_t s) {
  const uint64_t n = (uint64_t)c->P * c->R;
  k_zero_u64<<<1, 64, 0, s>>>(out, 8);
  RestirArgs off = restir_args(c);
  off.on = 0u;   // counting rays must not write reservoirs
  off.has_prev = 0u;
  k_count_traversal<kLdsStack><<<blocks(n, kTraceBlock), kTraceBlock, 0, s>>>(scene_view(c), shade_tables(c), probe_args(c), cache_args(c), c->d_rec, off, out);
  return hipGetLastError();
}

hipError_t launch_zero_stats(gi_context* c, hipStream_t s) {
  k_zero_u64<<<blocks((uint64_t)GI_STAT_COUNT * kStatStripes, 256), 256, 0, s>>>(c->d_stats, GI_STAT_COUNT * kStatStripes);
  return hipGetLastError();
}

}  // namespace gi
