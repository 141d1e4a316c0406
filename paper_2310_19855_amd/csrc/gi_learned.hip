// Learned surrogate of the world cache for gfx950 (not part of the GI-1.0 paper): a
// multiresolution hash encoding (16 levels x 2^19 entries x 2 FP16 features) feeding a
// 64-64 ReLU MLP, trained online on the radiance samples the pass produces each frame.
//
// Kernels: the frame's training rays compacted in ray order and picked stratified; per
// optimiser step, training forward + backward fused per block of 8 waves and 32 samples
// (encoding gathers, BF16 MFMA layers with FP32 accumulation, relative-L2 loss with static
// loss scaling, backward through the MLP on MFMA, weight gradients as per-block MFMA partials,
// the encoding gradient as (entry, contribution) pairs), a fixed-order reduction of the weight
// gradients, a stable radix sort of the pairs and per-entry sums in a fixed order with a lazy
// Adam step of the touched grid entries, Adam on the MLP, a skip of the whole step on
// non-finite gradients; BF16 or FP8 (OCP e4m3) inference at every probe-ray hit, and the judge
// that falls back to confident plain cells when the surrogate is off.  Every sum has a fixed
// order, so training is reproducible run to run.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gi_device.hpp"
#include "gi_host.hpp"

namespace gi {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kLd64 = 72;   // padded LDS row of a 64-wide bf16 tile (breaks bank conflicts)
constexpr int kLd32 = 40;   // padded LDS row of a 32-wide bf16 tile
constexpr int kMlpParams = 64 * 64 + 64 * 64 + 16 * 64;
constexpr int kOffW1 = 0, kOffW2 = 4096, kOffW3 = 8192;
static_assert(kMlpParams % 256 == 0, "the weight-gradient reduction takes 256 parameters per block");
constexpr uint32_t kRedGroups = 16;   // runs of training blocks summed separately, then in order
constexpr uint32_t kPrimeY = 2654435761u, kPrimeZ = 805459861u;
constexpr int kMaxLevels = 16;

struct LearnedParams {
  uint32_t L, T;
  float res[kMaxLevels];
  uint32_t dense_mask;
  float lo[3], ext[3];
};

struct LearnedState {
  LearnedParams lp;
  uint32_t grid_n = 0;           // L * T * 2
  // FP32 master values and Adam moments of the grid, interleaved per table entry (its two
  // features) in one 32-byte line: p0 p1 m0 m1 v0 v1 0 0 (entry e at gstate[8e])
  float* gstate = nullptr;
  __half* grid_h = nullptr;      // FP16 working copy [L][T][2]
  float* grid_g = nullptr;       // gradient of a gradient-only step (scaled by the loss scale)
  float* mlp = nullptr;          // FP32 master: W1 [64][64], W2 [64][64], W3 [16][64]
  float* mlp_g = nullptr;
  float* mlp_m = nullptr;
  float* mlp_v = nullptr;
  float* mlp_part = nullptr;     // [train_blocks][kMlpParams] per-block weight-gradient partials
  float* mlp_part2 = nullptr;    // [kRedGroups][kMlpParams] sums of consecutive runs of blocks
  __bf16* wb = nullptr;          // W1 [64][64] | W1t [64][64] | W2 | W2t | W3 [16][64] | W3t [64][32]
  uint8_t* w8 = nullptr;         // e4m3 W1 | W2 | W3 (row-major [out][in])
  float* scales = nullptr;       // [0..2] weight scales, [3..5] activation amax (X, H1, H2), [6..8] act scales
  float4* hitpos = nullptr;      // [P*R] hit point (learned mode), w = hit distance
  float4* hitnrm = nullptr;      // [P*R] face-forwarded normal
  float4* trec = nullptr;        // [P*R] training target of the ray's hit (rgb, w = 1)
  uint8_t* tflag = nullptr;      // [tflag_blocks * kTile] 1 where trec holds this frame's sample
  uint32_t tflag_blocks = 0;
  uint32_t* clist = nullptr;     // [P*R] the frame's training rays in ray order
  uint32_t* ccount = nullptr;    // [tflag_blocks + 1] per-block counts -> offsets, [last] = total
  float4* batch_raw = nullptr;   // [rows][3]: pos, nrm (w = ray id bits), target as selected
  float4* batch = nullptr;       // the same rows grouped by spatial (Morton) bucket, stable
  // radix sort buffers: batch keys and row indices (rows), gradient pairs (B * L * 8)
  uint32_t* bkeys[2] = {nullptr, nullptr};
  uint32_t* bvals[2] = {nullptr, nullptr};
  uint32_t* pkeys[2] = {nullptr, nullptr};
  float2* pvals[2] = {nullptr, nullptr};
  uint32_t* rs_hist = nullptr;   // [256][blocks] digit counts -> offsets
  float2* tail_sum = nullptr;    // per reduction tile: partial sum of its last entry and
  uint32_t* tail_in = nullptr;   // whether that entry began inside the tile
  size_t n_pairs = 0;
  uint32_t key_bits = 0;         // bits of a gradient pair key (level * T + entry)
  float* lpart = nullptr;        // [train_blocks] loss partials
  float2* judge_part = nullptr;  // per-wave (error, norm) partials of the judge
  uint32_t B = 0;
  uint32_t sub = 1;              // sub-batches held by the frame's batch (rows = sub * B)
  float4* lmlp = nullptr;        // [P*R] surrogate radiance at each hit
  float* acc = nullptr;          // [0] loss sum, [1] non-finite flag, [2] judge |diff|, [3] judge |plain|,
                                 // [4] fallback flag, [5] last loss, [6] last judged error, [7] batch n
  uint32_t train_blocks = 0;
  bool grad_dirty = false;       // grid_g holds a gradient-only step's result
  int step = 0, skipped = 0;
  float host_stats[8] = {0};
};

// ---- small helpers --------------------------------------------------------------------------

__device__ inline f32x4_t mma_bf16(const __bf16* A, int lda, const __bf16* Bt, int ldb, f32x4_t acc) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, kb = (lane >> 4) * 8;
  const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(A + r * lda + kb);
  const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(Bt + r * ldb + kb);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

// the B fragment of mma_bf16 for this lane, loaded ahead of its product
__device__ inline bf16x8_t frag_bf16(const __bf16* Bt, int ldb) {
  const int lane = threadIdx.x & 63;
  return *reinterpret_cast<const bf16x8_t*>(Bt + (lane & 15) * ldb + (lane >> 4) * 8);
}

__device__ inline f32x4_t mma_bf16f(const __bf16* A, int lda, const bf16x8_t& b, f32x4_t acc) {
  const int lane = threadIdx.x & 63;
  const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(A + (lane & 15) * lda + (lane >> 4) * 8);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

__device__ inline f32x4_t mma_fp8(const uint8_t* A, int lda, const uint8_t* Bt, int ldb, f32x4_t acc) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, kb = (lane >> 4) * 8;
  const long a = *reinterpret_cast<const long*>(A + r * lda + kb);
  const long b = *reinterpret_cast<const long*>(Bt + r * ldb + kb);
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, acc, 0, 0, 0);
}

__device__ inline __bf16 to_bf16(float x) { return static_cast<__bf16>(x); }
__device__ inline float from_bf16(__bf16 x) { return static_cast<float>(x); }

// OCP e4m3 code of x (1 sign, 4 exponent bits with bias 7, 3 mantissa bits): round to nearest
// even, saturating to +-448, NaN -> 0x7F.  The hardware conversion v_cvt_pk_fp8_f32 after a
// clamp to +-448 gives this code for every non-NaN float (checked over all of them).
__device__ inline uint32_t e4m3_code(float x) {
  if (x != x) return 0x7Fu;
  const float c = fminf(fmaxf(x, -448.0f), 448.0f);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(c, c, 0, false) & 0xFFu;
}

__global__ void k_e4m3_encode(const float* in, uint8_t* out, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (uint8_t)e4m3_code(in[i]);
}

// encoding input of a point: x = clamp((y - lo) / (hi - lo), 0, 1)
__device__ inline void norm_pos(const LearnedParams& lp, float y0, float y1, float y2, float& x0, float& x1, float& x2) {
  x0 = fminf(fmaxf((y0 - lp.lo[0]) / lp.ext[0], 0.0f), 1.0f);
  x1 = fminf(fmaxf((y1 - lp.lo[1]) / lp.ext[1], 0.0f), 1.0f);
  x2 = fminf(fmaxf((y2 - lp.lo[2]) / lp.ext[2], 0.0f), 1.0f);
}

// the 8 corners of level l: table index and trilinear weight
struct Corners {
  uint32_t idx[8];
  float w[8];
};

__device__ inline void level_corners(const LearnedParams& lp, int l, float x0, float x1, float x2, Corners& cn) {
  const float N = lp.res[l];
  const float p0 = x0 * N, p1 = x1 * N, p2 = x2 * N;
  const float Nm1 = N - 1.0f;
  const float v0f = fminf(floorf(p0), Nm1), v1f = fminf(floorf(p1), Nm1), v2f = fminf(floorf(p2), Nm1);
  const float f0 = p0 - v0f, f1 = p1 - v1f, f2 = p2 - v2f;
  const uint32_t v0 = (uint32_t)v0f, v1 = (uint32_t)v1f, v2 = (uint32_t)v2f;
  const bool dense = (lp.dense_mask >> l) & 1u;
  const uint32_t n1 = (uint32_t)N + 1u;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const uint32_t cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
    const uint32_t a = v0 + cx, b = v1 + cy, d = v2 + cz;
    cn.idx[c] = dense ? (a + b * n1 + d * n1 * n1) : ((a ^ (b * kPrimeY) ^ (d * kPrimeZ)) & (lp.T - 1u));
    cn.w[c] = (cx ? f0 : 1.0f - f0) * (cy ? f1 : 1.0f - f1) * (cz ? f2 : 1.0f - f2);
  }
}

// ---- initialisation: counter-based seeded values, (2u - 1) * scale in float32 -----------

__device__ inline float init_value(uint32_t seed, uint32_t stream, uint32_t i, float scale) {
  const float u = rand_unit(rand_u32(seed, stream, i, 0u));
  return (u * 2.0f - 1.0f) * scale;
}

__global__ void k_learned_init(float* gstate, __half* grid_h, uint32_t L, uint32_t T, float* mlp, uint32_t seed) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t n = (uint64_t)L * T * 2u;
  if (i < n) {
    const uint32_t l = (uint32_t)(i / ((uint64_t)T * 2u));
    const uint32_t k = (uint32_t)(i % ((uint64_t)T * 2u));
    const float v = init_value(seed, 100u + l, k, 1e-4f);
    gstate[8u * (i >> 1) + (i & 1u)] = v;   // moments are zeroed by the caller
    grid_h[i] = __float2half(v);
  }
  if (i < (uint64_t)kMlpParams) {
    const float s = 0.30618621784789726f;   // sqrt(6 / 64)
    float v = 0.0f;
    if (i < 4096) v = init_value(seed, 1u, (uint32_t)i, s);
    else if (i < 8192) v = init_value(seed, 2u, (uint32_t)(i - 4096), s);
    else if (i < 8192 + 3 * 64) v = init_value(seed, 3u, (uint32_t)(i - 8192), s);
    mlp[i] = v;
  }
}

// bf16 and e4m3 working copies of the MLP weights and their per-tensor scales (one block of
// 1024 threads)
// BF16 copies of weight i (of the three tensors laid out W1, W2, W3): row-major and transposed
// (W3t is [64][32], its columns 16..31 zero)
__device__ inline void mlp_bf16_copy(int i, float w, __bf16* wb) {
  const __bf16 b = to_bf16(w);
  if (i < 4096) {
    wb[i] = b;
    wb[4096 + (i & 63) * 64 + (i >> 6)] = b;
  } else if (i < 8192) {
    const int j = i - 4096;
    wb[8192 + j] = b;
    wb[12288 + (j & 63) * 64 + (j >> 6)] = b;
  } else {
    const int j = i - 8192, r = j >> 6, c = j & 63;
    wb[16384 + j] = b;
    wb[16384 + 1024 + c * 32 + r] = b;
    wb[16384 + 1024 + c * 32 + 16 + r] = to_bf16(0.0f);
  }
}

// per-tensor e4m3 scales (max |w| / 448) and e4m3 copies of the weights; one block of 1024
__device__ void mlp_e4m3_copies(const float* mlp, uint8_t* w8, float* scales) {
  __shared__ float red[3][32];
  const int t = threadIdx.x;
  float am[3] = {0.f, 0.f, 0.f};
  for (int i = t; i < kMlpParams; i += 1024) {
    const int tensor = i < 4096 ? 0 : (i < 8192 ? 1 : 2);
    am[tensor] = fmaxf(am[tensor], fabsf(mlp[i]));
  }
  for (int k = 0; k < 3; ++k) {
    float v = am[k];
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((t & 63) == 0) red[k][t >> 6] = v;
  }
  __syncthreads();
  if (t < 3) {
    float v = 0.f;
    for (int w = 0; w < 16; ++w) v = fmaxf(v, red[t][w]);
    scales[t] = v > 0.0f ? v / 448.0f : 1.0f;
  }
  __syncthreads();
  const float s0 = scales[0], s1 = scales[1], s2 = scales[2];
  for (int i = t; i < kMlpParams; i += 1024) {
    const float sc = i < 4096 ? s0 : (i < 8192 ? s1 : s2);
    w8[i] = (uint8_t)e4m3_code(mlp[i] / sc);
  }
}

__device__ void mlp_copies(const float* mlp, __bf16* wb, uint8_t* w8, float* scales) {
  for (int i = threadIdx.x; i < kMlpParams; i += 1024) mlp_bf16_copy(i, mlp[i], wb);
  mlp_e4m3_copies(mlp, w8, scales);
}

__global__ __launch_bounds__(1024) void k_mlp_copies(const float* mlp, __bf16* wb, uint8_t* w8, float* scales) {
  mlp_copies(mlp, wb, w8, scales);
}

// ---- the frame's training rays, compacted in ray order ---------------------------------
// A ray is a training sample when its probe ray hit, its hit found or created a world-cache
// cell and its sample is finite (flag set by the shading pass).  Blocks of kTile flags:
// count, one-block exclusive scan of the counts, then each block writes its rays' ids at
// their ranks.  The list is a function of the flags alone.
constexpr uint32_t kTile = 4096;      // items per block of 256 threads (16 each)

// orders the LDS accesses of one wave's lanes (no cost beyond keeping the compiler's order)
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// exclusive prefix over the NT threads of a block, in thread order; every thread of the block
// must call it (it holds two barriers); lds holds NT / 64 words
template <uint32_t NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* lds, uint32_t& total) {
  const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = (uint32_t)__shfl_up((int)x, d, 64);
    if (lane >= (uint32_t)d) x += o;
  }
  if (lane == 63u) lds[w] = x;
  __syncthreads();
  uint32_t base = 0;
  total = 0;
#pragma unroll
  for (uint32_t k = 0; k < NT / 64u; ++k) {
    if (k < w) base += lds[k];
    total += lds[k];
  }
  __syncthreads();
  return base + x - v;
}

__device__ inline uint32_t block_excl_scan256(uint32_t v, uint32_t* lds, uint32_t& total) {
  return block_excl_scan<256>(v, lds, total);
}

__global__ __launch_bounds__(256) void k_tflag_count(const uint8_t* flag, uint32_t* cnt) {
  __shared__ uint32_t lds[4];
  const uint4 f = reinterpret_cast<const uint4*>(flag + (size_t)blockIdx.x * kTile)[threadIdx.x];
  // every byte is 0 or 1: the popcount of a word is its number of set flags
  const uint32_t c = __popc(f.x) + __popc(f.y) + __popc(f.z) + __popc(f.w);
  uint32_t total;
  block_excl_scan256(c, lds, total);
  if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

// exclusive scan of n counts in place; cnt[n] = total (one block of 1024 threads)
__global__ __launch_bounds__(1024) void k_scan_counts(uint32_t* cnt, uint32_t n) {
  __shared__ uint32_t part[1024];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (n + 1023u) / 1024u;
  const uint32_t b0 = t * per, b1 = min(b0 + per, n);
  uint32_t sum = 0u;
  for (uint32_t i = b0; i < b1; ++i) sum += cnt[i];
  part[t] = sum;
  __syncthreads();
  for (uint32_t d = 1; d < 1024u; d <<= 1) {
    const uint32_t o = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += o;
    __syncthreads();
  }
  uint32_t run = part[t] - sum;
  for (uint32_t i = b0; i < b1; ++i) {
    const uint32_t v = cnt[i];
    cnt[i] = run;
    run += v;
  }
  if (t == 1023u) cnt[n] = part[1023];
}

__global__ __launch_bounds__(256) void k_tflag_compact(const uint8_t* flag, const uint32_t* off, uint32_t* list) {
  __shared__ uint32_t lds[4];
  const uint32_t base_id = blockIdx.x * kTile + 16u * threadIdx.x;
  const uint4 f = reinterpret_cast<const uint4*>(flag + (size_t)blockIdx.x * kTile)[threadIdx.x];
  const uint32_t c = __popc(f.x) + __popc(f.y) + __popc(f.z) + __popc(f.w);
  uint32_t total;
  uint32_t at = off[blockIdx.x] + block_excl_scan256(c, lds, total);
  const uint32_t w[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if ((w[q] >> (8 * b)) & 1u) list[at++] = base_id + 4u * q + b;
}

// ---- training batch selection: k-th of `rows` samples = list entry floor((k + u) n / rows) --

__global__ void k_select_batch(const uint32_t* list, const uint32_t* count, const float4* trec, const float4* hitpos,
                               const float4* hitnrm, float u, uint32_t rows, float4* batch, float* acc) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = *count;
  if (k == 0) acc[7] = (float)n;
  if (k >= rows) return;
  if (n == 0) {
    batch[3 * k] = batch[3 * k + 1] = batch[3 * k + 2] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  uint32_t r = (uint32_t)(((double)k + (double)u) * (double)n / (double)rows);
  if (r >= n) r = n - 1u;
  const uint32_t gid = list[r];
  const float4 nv = hitnrm[gid];
  batch[3 * k] = hitpos[gid];
  batch[3 * k + 1] = make_float4(nv.x, nv.y, nv.z, __uint_as_float(gid));
  batch[3 * k + 2] = trec[gid];
}

// ---- stable LSD radix sort of (u32 key, payload) pairs, 8-bit digits ---------------------
// Per pass: per-block digit counts (blocks of kRsTile items), a scan of each digit's block
// counts (one block per digit), and a scatter in which every item goes to its digit's offset
// plus the number of items of its block with the same digit and a lower index (wave ballots
// within a round, each wave's counts over its rounds, then the waves in order), so equal keys
// keep their input order.
constexpr uint32_t kRsThreads = 512, kRsRounds = 4, kRsTile = kRsThreads * kRsRounds;

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint32_t* key, uint32_t n, uint32_t shift, uint32_t nb,
                                                        uint32_t* hist) {
  __shared__ uint32_t h[256];
  if (threadIdx.x < 256u) h[threadIdx.x] = 0u;
  __syncthreads();
  // thread t counts keys 4t..4t+3 of the tile (one 16-byte load when all are in range)
  const uint32_t i0 = blockIdx.x * kRsTile + kRsRounds * threadIdx.x;
  if (i0 + kRsRounds <= n) {
    const uint4 k4 = *reinterpret_cast<const uint4*>(key + i0);
    atomicAdd(&h[(k4.x >> shift) & 255u], 1u);
    atomicAdd(&h[(k4.y >> shift) & 255u], 1u);
    atomicAdd(&h[(k4.z >> shift) & 255u], 1u);
    atomicAdd(&h[(k4.w >> shift) & 255u], 1u);
  } else {
    for (uint32_t i = i0; i < n; ++i) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 256u) hist[threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// block d: exclusive prefix of digit d's block counts (in place) and the digit's total
__global__ __launch_bounds__(256) void k_rs_digit_scan(uint32_t* hist, uint32_t nb, uint32_t* dtot) {
  __shared__ uint32_t lds[4];
  uint32_t* h = hist + (size_t)blockIdx.x * nb;
  uint32_t carry = 0u;
  for (uint32_t c = 0; c < nb; c += 256u) {
    const uint32_t i = c + threadIdx.x;
    const uint32_t v = i < nb ? h[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan256(v, lds, total);
    if (i < nb) h[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// The tile is first ordered by digit in LDS, then written out so that consecutive threads
// write consecutive addresses of each digit's run.  Wave w owns the tile's items
// w*256 .. w*256+255 (four rounds of 64): an item's rank among its wave's items of the same
// digit is its rank in its round's ballot plus the wave's count of that digit in earlier
// rounds (a per-wave LDS row, touched by that wave alone); the waves' rows, scanned in wave
// order, and the digits' tile offsets place it.  Equal digits keep their input order.
template <typename V>
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint32_t* kin, const V* vin, uint32_t* kout, V* vout,
                                                           uint32_t n, uint32_t shift, uint32_t nb, const uint32_t* off,
                                                           const uint32_t* dtot) {
  constexpr uint32_t W = kRsThreads / 64u, PW = kRsTile / W;
  static_assert(PW == 64u * kRsRounds && kRsThreads >= 256u, "a wave holds kRsRounds rounds of 64 items");
  __shared__ uint32_t sk[kRsTile];
  __shared__ V sv[kRsTile];
  __shared__ uint32_t wc[W][256];      // per wave: digit counts, then their prefix over earlier waves
  __shared__ uint32_t lbase[256];      // local position of each digit's first item
  __shared__ uint32_t gbase[256];      // global position of each digit's first item of this tile
  __shared__ uint32_t lc[W], ld[W];
  const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
  const uint32_t b0 = blockIdx.x * kRsTile;
  const uint32_t m = n - b0 < kRsTile ? n - b0 : kRsTile;     // items of this tile
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t key[kRsRounds], rk[kRsRounds];
  V val[kRsRounds];
#pragma unroll
  for (uint32_t j = 0; j < kRsRounds; ++j) {
    const uint32_t i = w * PW + 64u * j + lane;
    key[j] = i < m ? kin[b0 + i] : 0u;
    if (i < m) val[j] = vin[b0 + i];
  }
#pragma unroll
  for (uint32_t k = 0; k < 256u; k += 64u) wc[w][k + lane] = 0u;
#pragma unroll
  for (uint32_t j = 0; j < kRsRounds; ++j) {
    const bool on = w * PW + 64u * j + lane < m;
    const uint32_t d = (key[j] >> shift) & 255u;
    uint64_t same = __ballot(on);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t mb = __ballot((d >> b) & 1u);
      same &= ((d >> b) & 1u) ? mb : ~mb;
    }
    const uint32_t r = (uint32_t)__popcll(same & below);
    wave_sync();                        // the row as left by the previous round
    const uint32_t base = on ? wc[w][d] : 0u;
    rk[j] = base + r;
    wave_sync();                        // every lane has read before the row changes
    if (on && r == 0u) wc[w][d] = base + (uint32_t)__popcll(same);
  }
  __syncthreads();
  // digit t: prefix of the waves' counts in wave order, then exclusive scans over the digits
  // of the tile counts (local starts) and of the digit totals (global starts), together
  uint32_t c = 0u;
  if (t < 256u) {
#pragma unroll
    for (uint32_t q = 0; q < W; ++q) {
      const uint32_t x = wc[q][t];
      wc[q][t] = c;
      c += x;
    }
  }
  uint32_t x1 = c, x2 = t < 256u ? dtot[t] : 0u;
#pragma unroll
  for (int dd = 1; dd < 64; dd <<= 1) {
    const uint32_t o1 = (uint32_t)__shfl_up((int)x1, dd, 64), o2 = (uint32_t)__shfl_up((int)x2, dd, 64);
    if (lane >= (uint32_t)dd) {
      x1 += o1;
      x2 += o2;
    }
  }
  if (lane == 63u) {
    lc[w] = x1;
    ld[w] = x2;
  }
  __syncthreads();
  if (t < 256u) {
    uint32_t e1 = x1 - c, e2 = x2 - dtot[t];
    for (uint32_t q = 0; q < w; ++q) {
      e1 += lc[q];
      e2 += ld[q];
    }
    lbase[t] = e1;
    gbase[t] = e2 + off[t * nb + blockIdx.x];
  }
  __syncthreads();
#pragma unroll
  for (uint32_t j = 0; j < kRsRounds; ++j) {
    if (w * PW + 64u * j + lane < m) {
      const uint32_t d = (key[j] >> shift) & 255u;
      const uint32_t at = lbase[d] + wc[w][d] + rk[j];
      sk[at] = key[j];
      sv[at] = val[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (uint32_t j = 0; j < kRsRounds; ++j) {
    const uint32_t i = j * kRsThreads + t;
    if (i < m) {
      const uint32_t k = sk[i];
      const uint32_t d = (k >> shift) & 255u;
      const uint32_t g = gbase[d] + (i - lbase[d]);
      kout[g] = k;
      vout[g] = sv[i];
    }
  }
}

// sorts (keys[0], vals[0]) by the low `bits` bits of the keys, stable; returns the index of
// the buffer pair holding the result.  first_hist: the tile counts of the lowest digit are
// already in hist (written with the keys)
template <typename V>
static hipError_t radix_sort(uint32_t* keys[2], V* vals[2], uint32_t n, uint32_t bits, uint32_t* hist,
                             hipStream_t st, int& which, bool first_hist = false) {
  which = 0;
  if (n == 0) return hipSuccess;
  const uint32_t nb = (n + kRsTile - 1u) / kRsTile;
  uint32_t* dtot = hist + 256u * nb;
  for (uint32_t shift = 0; shift < bits; shift += 8u) {
    if (shift > 0u || !first_hist) k_rs_hist<<<nb, kRsThreads, 0, st>>>(keys[which], n, shift, nb, hist);
    k_rs_digit_scan<<<256, 256, 0, st>>>(hist, nb, dtot);
    k_rs_scatter<V><<<nb, kRsThreads, 0, st>>>(keys[which], vals[which], keys[which ^ 1], vals[which ^ 1], n, shift, nb,
                                               hist, dtot);
    which ^= 1;
  }
  return hipGetLastError();
}

// ---- spatial grouping of the frame's batch: rows stably sorted by a 15-bit Morton code of
// the normalised position (32 cells per axis), so that the 32 samples of a training group
// are neighbours and share coarse grid entries ------------------------------------------------
__device__ inline uint32_t spread5(uint32_t v) {
  v &= 0x1Fu;
  v = (v | (v << 8)) & 0x0000F00Fu;
  v = (v | (v << 4)) & 0x000C30C3u;
  v = (v | (v << 2)) & 0x00249249u;
  return v;
}

__device__ inline uint32_t sort_bucket(const LearnedParams& lp, const float4& p) {
  float x0, x1, x2;
  norm_pos(lp, p.x, p.y, p.z, x0, x1, x2);
  const uint32_t q0 = min((uint32_t)(x0 * 32.0f), 31u);
  const uint32_t q1 = min((uint32_t)(x1 * 32.0f), 31u);
  const uint32_t q2 = min((uint32_t)(x2 * 32.0f), 31u);
  return spread5(q0) | (spread5(q1) << 1) | (spread5(q2) << 2);
}

__global__ void k_batch_keys(LearnedParams lp, const float4* in, uint32_t rows, uint32_t* key, uint32_t* idx) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  key[i] = sort_bucket(lp, in[3 * (size_t)i]);
  idx[i] = i;
}

__global__ void k_batch_gather(const float4* in, const uint32_t* idx, uint32_t rows, float4* out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const size_t r = idx[i];
  out[3 * (size_t)i] = in[3 * r];
  out[3 * (size_t)i + 1] = in[3 * r + 1];
  out[3 * (size_t)i + 2] = in[3 * r + 2];
}

__global__ void k_zero_f32(float* p, uint64_t n);
static inline uint32_t nblk(uint64_t n, uint32_t b) { return (uint32_t)((n + b - 1) / b); }

static hipError_t sort_batch(gi_context* c, hipStream_t st, uint32_t rows) {
  LearnedState* s = c->learned;
  hipEvent_t ev;
  timer_begin(c, "learned_sort", st, &ev);
  k_batch_keys<<<nblk(rows, 256), 256, 0, st>>>(s->lp, s->batch_raw, rows, s->bkeys[0], s->bvals[0]);
  int which = 0;
  hipError_t e = radix_sort<uint32_t>(s->bkeys, s->bvals, rows, 15u, s->rs_hist, st, which);
  k_batch_gather<<<nblk(rows, 256), 256, 0, st>>>(s->batch_raw, s->bvals[which], rows, s->batch);
  timer_end(c, "learned_sort", st, ev);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// ---- fused training forward + backward, one block of 8 waves per 32-sample group -------

struct TrainSmem {
  __bf16 X[32 * kLd64], Xt[64 * kLd32];
  __bf16 H1[32 * kLd64], H1t[64 * kLd32];
  __bf16 H2[32 * kLd64], H2t[64 * kLd32];
  __bf16 dY[32 * kLd32], dYt[16 * kLd32];
  __bf16 dZ2[32 * kLd64], dZ2t[64 * kLd32];
  __bf16 dZ1[32 * kLd64], dZ1t[64 * kLd32];
  float dX[32 * 33];
  float4 tgt[32];
  float4 pos[32];        // sample positions, for the gradient pairs at the end of the group
};

// store a 16x16 accumulator tile (rows r0.., cols c0..) as bf16 into M[row][ld] and Mt[col][ldt]
__device__ inline void store_tile(const f32x4_t& v, __bf16* M, int ld, __bf16* Mt, int ldt, int r0, int c0) {
  const int lane = threadIdx.x & 63;
  const int col = c0 + (lane & 15), rb = r0 + 4 * (lane >> 4);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const __bf16 b = to_bf16(v[i]);
    M[(rb + i) * ld + col] = b;
    Mt[col * ldt + rb + i] = b;
  }
}

__device__ inline void atomic_max_abs(float* p, float v) {
  atomicMax(reinterpret_cast<unsigned int*>(p), __float_as_uint(fabsf(v)));
}

// sample i of the step is row off + stride * i of the batch array.  The encoding gradient is
// written as (level * T + entry, corner weight * dX) pairs, to be sorted and summed per entry:
// no float atomics, so the step is deterministic.  Group g (samples 32 g .. 32 g + 31) fills
// pairs [256 L g, 256 L (g + 1)) in (level, sample, corner) order, so the pairs of one level,
// which hold every copy of its keys, come in sample order across the groups.  When 256 L is a
// whole number of sort tiles (L a multiple of 8) the block also counts the low key digits of
// its tiles for the sort's first pass.
constexpr uint32_t kTrainWaves = 8;   // waves of a training block: one 16x16 tile of each layer's output each
static_assert(64 * kTrainWaves == 32 * kMaxLevels, "one thread of a training block per (sample, level) of its group");

// 4 waves per SIMD (two blocks per CU, as the LDS tiles allow) caps the registers at 128
__global__ __launch_bounds__(64 * kTrainWaves) __attribute__((amdgpu_waves_per_eu(4)))
void k_train(LearnedParams lp, const float4* batch, uint32_t B, uint32_t off, uint32_t stride, const __half* grid_h,
             const __bf16* wb, float loss_scale, float* part, float* lpart, float* acc, float* amax, uint32_t log2T,
             uint32_t* pkey, float2* pval, uint32_t nb, uint32_t* hist) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TrainSmem& S = *reinterpret_cast<TrainSmem*>(smem_raw);
  __shared__ float red[kTrainWaves][4];
  __shared__ uint32_t hs[2][256];       // low-digit counts of the group's sort tiles
  static_assert(kRsTile == 2048u && kMaxLevels <= 16, "a group's pairs are at most two sort tiles");
  const bool tiles = (lp.L & 7u) == 0u;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const __bf16* W1 = wb;
  const __bf16* W1t = wb + 4096;
  const __bf16* W2 = wb + 8192;
  const __bf16* W2t = wb + 12288;
  const __bf16* W3 = wb + 16384;
  const __bf16* W3t = wb + 16384 + 1024;
  const f32x4_t z4 = {0.f, 0.f, 0.f, 0.f};
  // wave w: forward and backward tile (sample rows 16*fm, unit columns 16*fn); of the weight
  // gradients, dW1 and dW2 tiles (row tile gm, column tiles 2*gh, 2*gh+1) and, for w < 4,
  // column tile w of dW3
  const int fm = w >> 2, fn = w & 3, gm = w & 3, gh = w >> 2;
  f32x4_t g1[2], g2[2], g3 = z4;
#pragma unroll
  for (int a = 0; a < 2; ++a) g1[a] = g2[a] = z4;
  const uint32_t groups = B / 32u;
  const float inv3b = 1.0f / (3.0f * (float)B);
  float loss = 0.0f;
  bool bad = false;
  float ax = 0.f, ah1 = 0.f, ah2 = 0.f;
  // input fill: thread = (sample s, level lg: its encoding, two of the 32 other columns)
  const int s = t & 31, lg = t >> 5;
  for (uint32_t g = blockIdx.x; g < groups; g += gridDim.x) {
    const uint32_t si = 32 * g + s;          // sample of the step
    const uint32_t row = off + stride * si;
    const float4 pos = batch[3 * row];
    const float4 nrm = batch[3 * row + 1];
    if (t < 32) {
      S.tgt[s] = batch[3 * row + 2];
      S.pos[s] = pos;
    }
    if (t < 256) {
      hs[0][t] = 0u;
      hs[1][t] = 0u;
    }
    // each phase's weight fragments are requested one phase ahead, so that their latency
    // passes during the phase before
    const bf16x8_t f1a = frag_bf16(W1 + 16 * fn * 64, 64), f1b = frag_bf16(W1 + 16 * fn * 64 + 32, 64);
    {
      // the sample's encoding at level l: trilinear blend of the FP16 corner features
      const int l = lg;
      float f0 = 0.f, f1 = 0.f;
      if (l < (int)lp.L) {
        float x0, x1, x2;
        norm_pos(lp, pos.x, pos.y, pos.z, x0, x1, x2);
        Corners cn;
        level_corners(lp, l, x0, x1, x2, cn);
        const __half2* tab = reinterpret_cast<const __half2*>(grid_h) + (size_t)l * lp.T;
        float2 v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = __half22float2(tab[cn.idx[c]]);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          f0 = f0 + cn.w[c] * v[c].x;
          f1 = f1 + cn.w[c] * v[c].y;
        }
      }
      const __bf16 b0 = to_bf16(f0), b1 = to_bf16(f1);
      S.X[s * kLd64 + 2 * l] = b0;
      S.X[s * kLd64 + 2 * l + 1] = b1;
      S.Xt[(2 * l) * kLd32 + s] = b0;
      S.Xt[(2 * l + 1) * kLd32 + s] = b1;
      ax = fmaxf(ax, fmaxf(fabsf(f0), fabsf(f1)));
    }
    // normal features, constant input, zero padding: columns 32..63, two per thread
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int c = 32 + 2 * lg + k;
      float v = 0.0f;
      if (c == 32) v = (nrm.x + 1.0f) * 0.5f;
      else if (c == 33) v = (nrm.y + 1.0f) * 0.5f;
      else if (c == 34) v = (nrm.z + 1.0f) * 0.5f;
      else if (c == 35) v = 1.0f;
      S.X[s * kLd64 + c] = to_bf16(v);
      S.Xt[c * kLd32 + s] = to_bf16(v);
      ax = fmaxf(ax, fabsf(v));
    }
    const bf16x8_t f2a = frag_bf16(W2 + 16 * fn * 64, 64), f2b = frag_bf16(W2 + 16 * fn * 64 + 32, 64);
    __syncthreads();
    // -- layer 1: Z1 = X W1^T, tile (fm, fn)
    {
      f32x4_t a = z4;
      a = mma_bf16f(S.X + 16 * fm * kLd64, kLd64, f1a, a);
      a = mma_bf16f(S.X + 16 * fm * kLd64 + 32, kLd64, f1b, a);
#pragma unroll
      for (int i = 0; i < 4; ++i) { a[i] = fmaxf(a[i], 0.0f); ah1 = fmaxf(ah1, a[i]); }
      store_tile(a, S.H1, kLd64, S.H1t, kLd32, 16 * fm, 16 * fn);
    }
    const bf16x8_t f3a = frag_bf16(W3, 64), f3b = frag_bf16(W3 + 32, 64);
    const bf16x8_t f3t = frag_bf16(W3t + 16 * fn * 32, 32);
    __syncthreads();
    // -- layer 2
    {
      f32x4_t a = z4;
      a = mma_bf16f(S.H1 + 16 * fm * kLd64, kLd64, f2a, a);
      a = mma_bf16f(S.H1 + 16 * fm * kLd64 + 32, kLd64, f2b, a);
#pragma unroll
      for (int i = 0; i < 4; ++i) { a[i] = fmaxf(a[i], 0.0f); ah2 = fmaxf(ah2, a[i]); }
      store_tile(a, S.H2, kLd64, S.H2t, kLd32, 16 * fm, 16 * fn);
    }
    __syncthreads();
    // -- layer 3 and the loss gradient (scaled by the loss scale): waves 0 and 1, one row tile each
    if (w < 2) {
      const int mt = w;
      f32x4_t a = z4;
      a = mma_bf16f(S.H2 + 16 * mt * kLd64, kLd64, f3a, a);
      a = mma_bf16f(S.H2 + 16 * mt * kLd64 + 32, kLd64, f3b, a);
      const int col = lane & 15;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * mt + 4 * (lane >> 4) + i;
        float d = 0.0f;
        if (col < 3) {
          const float4 t4 = S.tgt[r];
          const float tv = col == 0 ? t4.x : (col == 1 ? t4.y : t4.z);
          const float y = a[i];
          const float den = y * y + 0.01f;
          const float diff = y - tv;
          loss += diff * diff / den;
          d = loss_scale * (2.0f * diff / den) * inv3b;
          if (!isfinite(d)) bad = true;
        }
        const __bf16 b = to_bf16(d);
        S.dY[r * kLd32 + col] = b;
        S.dY[r * kLd32 + 16 + col] = to_bf16(0.0f);
        S.dYt[col * kLd32 + r] = b;
      }
    }
    const bf16x8_t f2ta = frag_bf16(W2t + 16 * fn * 64, 64), f2tb = frag_bf16(W2t + 16 * fn * 64 + 32, 64);
    __syncthreads();
    // -- dW3 += dY^T H2 (column tile w, waves 0..3)
    if (w < 4) g3 = mma_bf16(S.dYt, kLd32, S.H2t + 16 * w * kLd32, kLd32, g3);
    // -- dH2 = dY W3 (K = 16 padded to 32), dZ2 = dH2 * [H2 > 0]; tile (fm, fn)
    {
      f32x4_t a = z4;
      a = mma_bf16f(S.dY + 16 * fm * kLd32, kLd32, f3t, a);
      const int col = 16 * fn + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * fm + 4 * (lane >> 4) + i;
        if (!(from_bf16(S.H2[r * kLd64 + col]) > 0.0f)) a[i] = 0.0f;
      }
      store_tile(a, S.dZ2, kLd64, S.dZ2t, kLd32, 16 * fm, 16 * fn);
    }
    const bf16x8_t f1ta = frag_bf16(W1t + 16 * (w & 1) * 64, 64), f1tb = frag_bf16(W1t + 16 * (w & 1) * 64 + 32, 64);
    __syncthreads();
    // -- dW2 += dZ2^T H1 (row tile gm, column tiles 2gh, 2gh+1)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      g2[j] = mma_bf16(S.dZ2t + 16 * gm * kLd32, kLd32, S.H1t + 16 * (2 * gh + j) * kLd32, kLd32, g2[j]);
    // -- dH1 = dZ2 W2, dZ1 = dH1 * [H1 > 0]; tile (fm, fn)
    {
      f32x4_t a = z4;
      a = mma_bf16f(S.dZ2 + 16 * fm * kLd64, kLd64, f2ta, a);
      a = mma_bf16f(S.dZ2 + 16 * fm * kLd64 + 32, kLd64, f2tb, a);
      const int col = 16 * fn + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * fm + 4 * (lane >> 4) + i;
        if (!(from_bf16(S.H1[r * kLd64 + col]) > 0.0f)) a[i] = 0.0f;
      }
      store_tile(a, S.dZ1, kLd64, S.dZ1t, kLd32, 16 * fm, 16 * fn);
    }
    __syncthreads();
    // -- dW1 += dZ1^T X (row tile gm, column tiles 2gh, 2gh+1)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      g1[j] = mma_bf16(S.dZ1t + 16 * gm * kLd32, kLd32, S.Xt + 16 * (2 * gh + j) * kLd32, kLd32, g1[j]);
    // -- dX[:, 0:32] = dZ1 W1 (encoding columns only), kept in float32: waves 0..3, a tile each
    if (w < 4) {
      const int mt = w >> 1, nt = w & 1;
      f32x4_t a = z4;
      a = mma_bf16f(S.dZ1 + 16 * mt * kLd64, kLd64, f1ta, a);
      a = mma_bf16f(S.dZ1 + 16 * mt * kLd64 + 32, kLd64, f1tb, a);
      const int col = 16 * nt + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * mt + 4 * (lane >> 4) + i;
        S.dX[r * 33 + col] = a[i];
        if (!isfinite(a[i])) bad = true;
      }
    }
    __syncthreads();
    // -- the encoding gradient: thread (s, l) writes its 8 corner pairs, contiguous
    if (lg < (int)lp.L) {
      const int l = lg;
      const float4 ps = S.pos[s];
      float x0, x1, x2;
      norm_pos(lp, ps.x, ps.y, ps.z, x0, x1, x2);
      Corners cn;
      level_corners(lp, l, x0, x1, x2, cn);
      const float d0 = S.dX[s * 33 + 2 * l], d1 = S.dX[s * 33 + 2 * l + 1];
      uint32_t k[8];
      float v[16];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        k[c] = ((uint32_t)l << log2T) | cn.idx[c];
        v[2 * c] = cn.w[c] * d0;
        v[2 * c + 1] = cn.w[c] * d1;
        if (tiles) atomicAdd(&hs[l >> 3][k[c] & 255u], 1u);
      }
      const size_t q = ((size_t)g * lp.L + (size_t)l) * 32u + (size_t)s;
      uint4* kq = reinterpret_cast<uint4*>(pkey + q * 8u);
      kq[0] = make_uint4(k[0], k[1], k[2], k[3]);
      kq[1] = make_uint4(k[4], k[5], k[6], k[7]);
      float4* vq = reinterpret_cast<float4*>(pval + q * 8u);
#pragma unroll
      for (int j = 0; j < 4; ++j) vq[j] = make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
    }
    __syncthreads();
    if (tiles && t < 256) {
      const uint32_t t0 = g * (lp.L >> 3);
      for (uint32_t j = 0; j < (lp.L >> 3); ++j) hist[(size_t)t * nb + t0 + j] = hs[j][t];
    }
    __syncthreads();
  }
  // per-block weight-gradient partials (C layout: row 4*(lane/16)+i, column lane%16 of a tile)
  float* pw = part + (size_t)blockIdx.x * kMlpParams;
  const int col = lane & 15, rb = 4 * (lane >> 4);
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      pw[kOffW1 + (16 * gm + rb + i) * 64 + 16 * (2 * gh + j) + col] = g1[j][i];
      pw[kOffW2 + (16 * gm + rb + i) * 64 + 16 * (2 * gh + j) + col] = g2[j][i];
    }
  if (w < 4)
#pragma unroll
    for (int i = 0; i < 4; ++i) pw[kOffW3 + (rb + i) * 64 + 16 * w + col] = g3[i];
  // loss, non-finite flag and activation ranges: per wave, then the block's waves in order
  for (int o = 32; o >= 1; o >>= 1) {
    loss += __shfl_xor(loss, o, 64);
    ax = fmaxf(ax, __shfl_xor(ax, o, 64));
    ah1 = fmaxf(ah1, __shfl_xor(ah1, o, 64));
    ah2 = fmaxf(ah2, __shfl_xor(ah2, o, 64));
  }
  if (__ballot(bad) != 0 && lane == 0) acc[1] = 1.0f;
  if (lane == 0) {
    red[w][0] = loss;
    red[w][1] = ax;
    red[w][2] = ah1;
    red[w][3] = ah2;
  }
  __syncthreads();
  if (t == 0) {
    float l = red[0][0], bx = red[0][1], b1 = red[0][2], b2 = red[0][3];
#pragma unroll
    for (uint32_t q = 1; q < kTrainWaves; ++q) {
      l += red[q][0];
      bx = fmaxf(bx, red[q][1]);
      b1 = fmaxf(b1, red[q][2]);
      b2 = fmaxf(b2, red[q][3]);
    }
    lpart[blockIdx.x] = l * inv3b;
    atomic_max_abs(&amax[0], bx);
    atomic_max_abs(&amax[1], b1);
    atomic_max_abs(&amax[2], b2);
  }
}

// deterministic sum of the per-block partials (fixed order) -> gradient; flags non-finite.
// Stage 1: block (x, y) sums the partials of run y (kRedGroups consecutive runs of training
// blocks) for 256 parameters, four slices of the run (one float4 column per thread) added in
// a fixed order; stage 2 (reduce_mlp_finish) adds the runs in order.
__global__ __launch_bounds__(256) void k_reduce_mlp(const float* part, uint32_t parts, float* part2) {
  __shared__ float4 red[4][64];
  const uint32_t l = threadIdx.x & 63u, slice = threadIdx.x >> 6;
  const uint32_t c4 = blockIdx.x * 64u + l;                    // float4 column
  const uint32_t per = (parts + kRedGroups - 1u) / kRedGroups;
  const uint32_t w0 = blockIdx.y * per, w1 = w0 + per < parts ? w0 + per : parts;
  const float4* p4 = reinterpret_cast<const float4*>(part);
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  if (c4 < kMlpParams / 4)
    for (uint32_t w = w0 + slice; w < w1; w += 4u) {
      const float4 v = p4[(size_t)w * (kMlpParams / 4) + c4];
      s.x += v.x;
      s.y += v.y;
      s.z += v.z;
      s.w += v.w;
    }
  red[slice][l] = s;
  __syncthreads();
  if (slice == 0u && c4 < kMlpParams / 4) {
    float4 t = red[0][l];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      const float4 v = red[k][l];
      t.x += v.x;
      t.y += v.y;
      t.z += v.z;
      t.w += v.w;
    }
    reinterpret_cast<float4*>(part2 + (size_t)blockIdx.y * kMlpParams)[c4] = t;
  }
}

// stage 2, run by the blocks of the first pass over the sorted grid pairs (which comes after
// stage 1 and before any reader of the gradient or of the flags)
struct MlpFinish {
  const float* part2;
  const float* lpart;
  uint32_t parts;
  float* g;
};

__device__ inline void reduce_mlp_finish(const MlpFinish& mf, float* acc) {
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    // the step's loss: lane j sums partials j, j + 64, ... in order, then a fixed butterfly
    float l = 0.0f;
    for (uint32_t w = threadIdx.x; w < mf.parts; w += 64u) l += mf.lpart[w];
    for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
    if (threadIdx.x == 0) acc[0] = l;
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < (uint32_t)kMlpParams; i += gridDim.x * blockDim.x) {
    float t = mf.part2[i];
    for (uint32_t k = 1; k < kRedGroups; ++k) t += mf.part2[(size_t)k * kMlpParams + i];
    mf.g[i] = t;
    if (!isfinite(t)) acc[1] = 1.0f;
  }
}

// Adam on the unscaled gradient; the whole step is skipped when any gradient is non-finite
struct AdamArgs {
  float lr, eps, b1, b2, c1, c2, inv_scale;
};

// Grid entries take the step only where this step's gradient is non-zero (lazy Adam: an
// entry no sample touched keeps its value and moments).  The gradient buffer is left zeroed
// for the next step, also when the step is skipped.
__device__ inline void adam_lazy(float graw, float& p, float& m, float& v, const AdamArgs& a) {
  if (graw == 0.0f) return;
  const float gi = graw * a.inv_scale;
  m = a.b1 * m + (1.0f - a.b1) * gi;
  v = a.b2 * v + (1.0f - a.b2) * gi * gi;
  const float mh = m / a.c1, vh = v / a.c2;
  p = p - a.lr * mh / (sqrtf(vh) + a.eps);
}

// ---- per-entry sums of the sorted gradient pairs, then the grid step --------------------
// Tiles of kGredTile sorted pairs, thread t of a tile holding pairs kGredItems t ..
// kGredItems (t + 1) - 1 (one pair per thread: 256-pair tiles, whose many blocks overlap one
// another's loads).  Each thread sums its pairs in order, restarting where the key changes; a segmented scan over the
// threads (fixed association) extends every pair's sum back to the tile start or to its
// entry's first pair.  MODE 0 records each tile's last partial sum and whether its entry began
// inside the tile.  In MODE 1 and 2 a tile's carry-in (the sums, in earlier tiles, of the entry
// open at its start) is the run of those tail sums from the tile where that entry began,
// added oldest first; MODE 1 adds the carry to entries that began in an earlier tile and, at each
// entry's last pair, takes the lazy Adam step of its two parameters (none when the step's
// gradients are non-finite); MODE 2 writes the dense gradient instead (a gradient-only step).
// Every order is fixed, so the sums, and the step, are deterministic.
constexpr uint32_t kGredItems = 1, kGredTile = 256 * kGredItems;
static_assert(kGredItems <= 32, "a thread's key changes fit one word");

template <int MODE>
__global__ __launch_bounds__(256) void k_gred(const uint32_t* key, const float2* val, uint32_t n, float2* tail_sum,
                                              uint32_t* tail_in, float* gstate, __half* ph, float* gdense, AdamArgs a,
                                              float* acc, MlpFinish mf) {
  __shared__ float2 cs[2][256];
  __shared__ uint32_t cf[2][256];
  __shared__ float2 cin_s;
  const uint32_t t = threadIdx.x;
  if (MODE != 0 && t < 64u) {
    // wave 0: the carry-in.  Walk back over the earlier tiles' flags, 64 at a time, to the
    // nearest tile whose last entry began inside it (tile 0's always did), then add the tail
    // sums from that tile up to this one's predecessor in tile order.
    const uint32_t b = blockIdx.x;
    uint32_t first = 0u, top = b;
    while (top > 0u) {
      const bool f = t < top && tail_in[top - 1u - t] != 0u;
      const uint64_t m = __ballot(f);
      if (m) {
        first = top - (uint32_t)__ffsll((long long)m);
        break;
      }
      top = top > 64u ? top - 64u : 0u;
    }
    float2 cs0 = make_float2(0.0f, 0.0f);
    for (uint32_t c0 = first; c0 < b; c0 += 64u) {
      const float2 v = c0 + t < b ? tail_sum[c0 + t] : make_float2(0.0f, 0.0f);
      const uint32_t cnt = b - c0 < 64u ? b - c0 : 64u;
      for (uint32_t q = 0; q < cnt; ++q) {
        const float ox = __shfl(v.x, (int)q, 64), oy = __shfl(v.y, (int)q, 64);
        cs0.x = cs0.x + ox;
        cs0.y = cs0.y + oy;
      }
    }
    if (t == 0u) cin_s = cs0;
  }
  const uint32_t i0 = blockIdx.x * kGredTile + kGredItems * t;
  uint32_t k[kGredItems];
  float2 w[kGredItems];
#pragma unroll
  for (uint32_t j = 0; j < kGredItems; ++j) {
    const bool on = i0 + j < n;
    k[j] = on ? key[i0 + j] : 0xFFFFFFFFu;          // keys are < 2^28: never equal to padding
    w[j] = on ? val[i0 + j] : make_float2(0.0f, 0.0f);
  }
  const uint32_t kprev = i0 > 0 && i0 - 1 < n ? key[i0 - 1] : 0xFFFFFFFFu;
  const uint32_t knext = i0 + kGredItems < n ? key[i0 + kGredItems] : 0xFFFFFFFFu;
  // an entry's last pair is known from the keys alone: its Adam state is loaded now, so that
  // the loads overlap the scan below
  bool last[kGredItems];
  float4 pm[kGredItems], vz[kGredItems];
  float4* gs = reinterpret_cast<float4*>(gstate);
#pragma unroll
  for (uint32_t j = 0; j < kGredItems; ++j) {
    const uint32_t kn = j + 1 < kGredItems ? k[j + 1] : knext;
    last[j] = i0 + j < n && kn != k[j];
    if (MODE == 1 && last[j]) {
      pm[j] = gs[2u * (size_t)k[j]];
      vz[j] = gs[2u * (size_t)k[j] + 1u];
    }
  }
  // bit j: the pair's key differs from the one before it (a key change at or before pair j
  // inside this thread's chunk once OR-ed forward)
  uint32_t heads = 0;
  float2 loc[kGredItems];
  float sx = 0.0f, sy = 0.0f;
  uint32_t kp = kprev;
#pragma unroll
  for (uint32_t j = 0; j < kGredItems; ++j) {
    if (k[j] != kp) {
      sx = 0.0f;
      sy = 0.0f;
      heads |= ((0xFFFFFFFFu >> (32u - kGredItems)) << j) & (0xFFFFFFFFu >> (32u - kGredItems));
    }
    sx = sx + w[j].x;
    sy = sy + w[j].y;
    loc[j] = make_float2(sx, sy);
    kp = k[j];
  }
  int cur = 0;
  cs[0][t] = make_float2(sx, sy);
  cf[0][t] = heads ? 1u : 0u;
  __syncthreads();
  for (uint32_t d = 1; d < 256u; d <<= 1) {
    float2 s2 = cs[cur][t];
    uint32_t f = cf[cur][t];
    if (t >= d && !f) {
      const float2 o = cs[cur][t - d];
      s2 = make_float2(o.x + s2.x, o.y + s2.y);
      f = cf[cur][t - d];
    }
    cs[cur ^ 1][t] = s2;
    cf[cur ^ 1][t] = f;
    cur ^= 1;
    __syncthreads();
  }
  const float2 carry = t > 0 ? cs[cur][t - 1] : make_float2(0.0f, 0.0f);
  const bool carry_in_tile = t > 0 && cf[cur][t - 1] != 0u;
  if (MODE == 0) {
    reduce_mlp_finish(mf, acc);
    if (t == 255u) {
      const uint32_t j = kGredItems - 1;
      const bool own = (heads >> j) & 1u;
      tail_sum[blockIdx.x] = own ? loc[j] : make_float2(carry.x + loc[j].x, carry.y + loc[j].y);
      tail_in[blockIdx.x] = (own || carry_in_tile) ? 1u : 0u;
    }
    return;
  }
  const float2 cin = cin_s;
  const bool skip = MODE == 1 && acc[1] != 0.0f;
  float gx[kGredItems], gy[kGredItems];
#pragma unroll
  for (uint32_t j = 0; j < kGredItems; ++j) {
    const bool own = (heads >> j) & 1u;
    float2 sum = own ? loc[j] : make_float2(carry.x + loc[j].x, carry.y + loc[j].y);
    if (!(own || carry_in_tile)) sum = make_float2(sum.x + cin.x, sum.y + cin.y);
    gx[j] = sum.x;
    gy[j] = sum.y;
  }
  if (MODE == 2) {
#pragma unroll
    for (uint32_t j = 0; j < kGredItems; ++j)
      if (last[j]) *reinterpret_cast<float2*>(gdense + 2u * (size_t)k[j]) = make_float2(gx[j], gy[j]);
    return;
  }
  if (skip) return;
#pragma unroll
  for (uint32_t j = 0; j < kGredItems; ++j)
    if (last[j]) {
      adam_lazy(gx[j], pm[j].x, pm[j].z, vz[j].x, a);
      adam_lazy(gy[j], pm[j].y, pm[j].w, vz[j].y, a);
      gs[2u * (size_t)k[j]] = pm[j];
      gs[2u * (size_t)k[j] + 1u] = vz[j];
      *reinterpret_cast<__half2*>(ph + 2u * (size_t)k[j]) = __halves2half2(__float2half(pm[j].x), __float2half(pm[j].y));
    }
}

// end of an applied step (one block of 1024 threads): Adam on the MLP weights, their bf16 and
// e4m3 working copies, the e4m3 activation scales of the step's batch, the step's statistics
// Adam on the MLP weights (dense), one parameter per thread
// the MLP's Adam step (skipped when the step's loss was not finite) and the weights' BF16
// copies; the e4m3 copies, which need every weight's new value for their scales, follow in
// k_mlp_step
__global__ __launch_bounds__(256) void k_mlp_adam(float* p, const float* g, float* m, float* v, AdamArgs a,
                                                  const float* acc, __bf16* wb) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kMlpParams) return;
  float w = p[i];
  if (acc[1] == 0.0f) {
    const float gi = g[i] * a.inv_scale;
    const float mi = a.b1 * m[i] + (1.0f - a.b1) * gi;
    const float vi = a.b2 * v[i] + (1.0f - a.b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w = w - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
    p[i] = w;
  }
  mlp_bf16_copy(i, w, wb);
}

// fp8: the e4m3 copies and scales are formed only for FP8 inference (no other reader)
__global__ __launch_bounds__(1024) void k_mlp_step(float* p, float* acc, uint8_t* w8, float* scales,
                                                   unsigned long long* stats, bool fp8) {
  const bool skip = acc[1] != 0.0f;
  if (fp8) mlp_e4m3_copies(p, w8, scales);
  __syncthreads();                      // every thread has read the flag
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) {
      const float am = scales[3 + k];
      scales[6 + k] = am > 0.0f ? am / 448.0f : 1.0f;
      scales[3 + k] = 0.0f;             // the next step's activation ranges start from zero
    }
    acc[5] = acc[0];
    if (skip) stats[GI_STAT_MLP_SKIPPED] += 1ull;
    acc[1] = 0.0f;                      // and its non-finite flag
  }
}

__global__ void k_learned_copy_half(const float* gstate, __half* h, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) h[i] = __float2half(gstate[8u * (i >> 1) + (i & 1u)]);
}

__global__ void k_zero_f32(float* p, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// ---- inference: one wave evaluates 64 points (4 row tiles) ------------------------------

// one activation tile per wave, BF16 or e4m3 rows: each layer's outputs stay in the MFMA
// accumulators until every product has read the tile, then overwrite it in place (one tile
// instead of a ping-pong pair per precision: 9 KiB per wave, so 17 waves share a CU's LDS)
union InferSmem {
  __bf16 A[64 * kLd64];
  uint8_t A8[64 * 80];
  float y[64 * 4];
};

// 4 waves per SIMD is what the activation tile's LDS allows; asked for, the compiler keeps the
// layer accumulators in VGPRs instead of adding AGPRs on top of the gather phase's registers
template <bool FP8, bool HITLIST>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_infer(LearnedParams lp, const __half* grid_h, const __bf16* wb,
                                              const uint8_t* w8, const float* scales, const float4* pos,
                                              const float4* nrm, uint32_t n, const uint32_t* list_ids,
                                              const uint32_t* list_count, uint32_t stripe_cap,
                                              uint32_t blocks_per_stripe, float4* out) {
  __shared__ __align__(16) InferSmem S;
  const int lane = threadIdx.x;
  uint32_t item, oidx;
  bool valid;
  if (HITLIST) {
    const uint32_t stripe = blockIdx.x / blocks_per_stripe;
    item = (blockIdx.x % blocks_per_stripe) * 64u + lane;
    valid = stripe < kStatStripes && item < list_count[stripe];
    oidx = valid ? list_ids[stripe * stripe_cap + item] : 0u;
  } else {
    item = blockIdx.x * 64u + lane;
    valid = item < n;
    oidx = item;
  }
  if (__ballot(valid) == 0) return;
  float4 p4 = make_float4(0.f, 0.f, 0.f, 0.f), n4 = p4;
  if (valid) {
    p4 = pos[oidx];
    n4 = nrm[oidx];
  }
  float x0, x1, x2;
  norm_pos(lp, p4.x, p4.y, p4.z, x0, x1, x2);
  // the input row of this lane (64 features: 2 per level, the normal mapped to [0, 1], a 1,
  // zeros) goes straight into the tile, as BF16 or as e4m3 codes of feature x (1 / s_x) (the
  // activation scales' reciprocals are taken once: this quantisation is the kernel's own
  // approximation, held to a tolerance against the float64 forward pass)
  const float sx = FP8 ? scales[6] : 1.0f;
  const float rsx = FP8 ? 1.0f / sx : 1.0f;
  auto put = [&](int c, float v) {
    if (FP8) S.A8[lane * 80 + c] = (uint8_t)e4m3_code(v * rsx);
    else S.A[lane * kLd64 + c] = to_bf16(v);
  };
  // levels in groups of 4: the group's 32 corner loads are issued together (levels past L
  // load level L - 1's entries and are dropped), then summed per level in corner order
#pragma unroll
  for (int gl = 0; gl < kMaxLevels; gl += 4) {
    if (gl >= (int)lp.L) break;
    Corners cn[4];
    __half2 hv[4][8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int l = min(gl + q, (int)lp.L - 1);
      level_corners(lp, l, x0, x1, x2, cn[q]);
      const __half2* tab = reinterpret_cast<const __half2*>(grid_h) + (size_t)l * lp.T;
#pragma unroll
      for (int c = 0; c < 8; ++c) hv[q][c] = tab[cn[q].idx[c]];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float f0 = 0.f, f1 = 0.f;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const float2 v = __half22float2(hv[q][c]);
        f0 = f0 + cn[q].w[c] * v.x;
        f1 = f1 + cn[q].w[c] * v.y;
      }
      if (gl + q < (int)lp.L) {
        put(2 * (gl + q), f0);
        put(2 * (gl + q) + 1, f1);
      }
    }
  }
  for (int c = 2 * (int)lp.L; c < 32; ++c) put(c, 0.0f);
  put(32, (n4.x + 1.0f) * 0.5f);
  put(33, (n4.y + 1.0f) * 0.5f);
  put(34, (n4.z + 1.0f) * 0.5f);
  put(35, 1.0f);
#pragma unroll
  for (int c = 36; c < 64; ++c) put(c, 0.0f);
  __syncthreads();
  const f32x4_t z4 = {0.f, 0.f, 0.f, 0.f};
  // one hidden layer: the 16 output tiles of tile x W^T, then (after every product has read
  // the tile) relu, rescaled and rounded to the tile's format, in place
  auto hidden = [&](const void* W, float dq, float rsn) {
    f32x4_t acc[16];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f32x4_t a = z4;
        if (FP8) {
          const uint8_t* W8 = static_cast<const uint8_t*>(W);
          a = mma_fp8(S.A8 + 16 * mt * 80, 80, W8 + 16 * nt * 64, 64, a);
          a = mma_fp8(S.A8 + 16 * mt * 80 + 32, 80, W8 + 16 * nt * 64 + 32, 64, a);
        } else {
          const __bf16* Wb = static_cast<const __bf16*>(W);
          a = mma_bf16(S.A + 16 * mt * kLd64, kLd64, Wb + 16 * nt * 64, 64, a);
          a = mma_bf16(S.A + 16 * mt * kLd64 + 32, kLd64, Wb + 16 * nt * 64 + 32, 64, a);
        }
        acc[4 * mt + nt] = a;
      }
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int col = 16 * nt + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * mt + 4 * (lane >> 4) + i;
          if (FP8) S.A8[row * 80 + col] = (uint8_t)e4m3_code(fmaxf(acc[4 * mt + nt][i] * dq, 0.0f) * rsn);
          else S.A[row * kLd64 + col] = to_bf16(fmaxf(acc[4 * mt + nt][i], 0.0f));
        }
      }
    __syncthreads();
  };
  // per-tensor scaled e4m3 operands for FP8 (float32 accumulation, dequantised by s_x * s_w)
  const float s1 = FP8 ? scales[7] : 1.0f, s2 = FP8 ? scales[8] : 1.0f;
  const float d1 = FP8 ? sx * scales[0] : 1.0f, d2 = FP8 ? s1 * scales[1] : 1.0f, d3 = FP8 ? s2 * scales[2] : 1.0f;
  if (FP8) {
    hidden(w8, d1, 1.0f / s1);
    hidden(w8 + 4096, d2, 1.0f / s2);
  } else {
    hidden(wb, 1.0f, 1.0f);
    hidden(wb + 8192, 1.0f, 1.0f);
  }
  // output layer (3 of 16 columns used) into registers, then through the tile to the rows' lanes
  f32x4_t o[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4_t a = z4;
    if (FP8) {
      a = mma_fp8(S.A8 + 16 * mt * 80, 80, w8 + 8192, 64, a);
      a = mma_fp8(S.A8 + 16 * mt * 80 + 32, 80, w8 + 8192 + 32, 64, a);
    } else {
      a = mma_bf16(S.A + 16 * mt * kLd64, kLd64, wb + 16384, 64, a);
      a = mma_bf16(S.A + 16 * mt * kLd64 + 32, kLd64, wb + 16384 + 32, 64, a);
    }
    o[mt] = a;
  }
  __syncthreads();
  {
    const int col = lane & 15;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (col < 3) S.y[(16 * mt + 4 * (lane >> 4) + i) * 4 + col] = o[mt][i] * d3;
  }
  __syncthreads();
  const float y0 = S.y[lane * 4], y1 = S.y[lane * 4 + 1], y2 = S.y[lane * 4 + 2];
  if (valid) out[oidx] = make_float4(fmaxf(y0, 0.0f), fmaxf(y1, 0.0f), fmaxf(y2, 0.0f), 1.0f);
}

// judge: relative error of the surrogate against confident plain cells (hits whose cell has
// at least 64 history samples); one partial (error, norm) per wave, summed by k_judge_decide
__global__ void k_judge(const uint32_t* ids, const uint32_t* count, uint32_t stripe_cap, uint32_t blocks_per_stripe,
                        const uint4* rec, const uint2* meta, const float4* L, const float4* lmlp, float2* part) {
  const uint32_t stripe = blockIdx.x / blocks_per_stripe;
  const uint32_t item = (blockIdx.x % blocks_per_stripe) * blockDim.x + threadIdx.x;
  float dn = 0.f, dd = 0.f;
  if (stripe < kStatStripes && item < count[stripe]) {
    const uint32_t gid = ids[stripe * stripe_cap + item];
    const int32_t slot = (int32_t)rec[gid].x;
    if (slot >= 0 && meta[slot].x >= 64u) {
      const float4 a = lmlp[gid], b = L[slot];
      dn = fabsf(a.x - b.x) + fabsf(a.y - b.y) + fabsf(a.z - b.z);
      dd = fabsf(b.x) + fabsf(b.y) + fabsf(b.z);
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    dn += __shfl_xor(dn, o, 64);
    dd += __shfl_xor(dd, o, 64);
  }
  if (threadIdx.x == 0) part[blockIdx.x] = make_float2(dn, dd);
}

__global__ __launch_bounds__(1024) void k_judge_decide(const float2* part, uint32_t n, float* acc, float threshold,
                                                       unsigned long long* stats) {
  __shared__ float sn[1024], sd[1024];
  const uint32_t t = threadIdx.x;
  float a = 0.f, b = 0.f;
  for (uint32_t i = t; i < n; i += 1024u) {
    const float2 v = part[i];
    a += v.x;
    b += v.y;
  }
  sn[t] = a;
  sd[t] = b;
  __syncthreads();
  for (uint32_t h = 512; h >= 1; h >>= 1) {
    if (t < h) {
      sn[t] += sn[t + h];
      sd[t] += sd[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    const float err = sd[0] > 0.0f ? sn[0] / sd[0] : 0.0f;
    acc[6] = err;
    const bool fb = sd[0] > 0.0f && err > threshold;
    acc[4] = fb ? 1.0f : 0.0f;
    if (fb) stats[GI_STAT_MLP_FALLBACK] += 1ull;
  }
}

// closes a gradient-only step (the applied step's k_mlp_step does the same): the loss is
// published, and the flag and activation ranges are cleared for the next step
__global__ void k_train_end(float* acc, float* amax, unsigned long long* stats) {
  if (threadIdx.x == 0) {
    acc[5] = acc[0];
    if (acc[1] != 0.0f) stats[GI_STAT_MLP_SKIPPED] += 1ull;
    acc[1] = 0.0f;
    amax[0] = amax[1] = amax[2] = 0.0f;
  }
}

// ---- host side -----------------------------------------------------------------------------


template <typename T>
static hipError_t lalloc(T** p, size_t n) {
  *p = nullptr;
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (n ? n : 1));
}

hipError_t learned_create(gi_context* c) {
  LearnedState* s = new LearnedState();
  c->learned = s;
  const gi_config& g = c->cfg;
  LearnedParams& lp = s->lp;
  lp.L = g.mlp_levels ? g.mlp_levels : 16u;
  if (lp.L > (uint32_t)kMaxLevels) lp.L = kMaxLevels;
  const uint32_t tl = g.mlp_table_log2 ? g.mlp_table_log2 : 19u;
  lp.T = 1u << (tl > 24 ? 24 : tl);
  const double nmin = 16.0, nmax = 4096.0;
  const double lb = lp.L > 1 ? (std::log(nmax) - std::log(nmin)) / (double)(lp.L - 1) : 0.0;
  lp.dense_mask = 0;
  for (uint32_t l = 0; l < (uint32_t)kMaxLevels; ++l) {
    const double N = l < lp.L ? std::floor(nmin * std::exp((double)l * lb) + 1e-6) : 1.0;
    lp.res[l] = (float)N;
    if (l < lp.L && (N + 1.0) * (N + 1.0) * (N + 1.0) <= (double)lp.T) lp.dense_mask |= 1u << l;
  }
  for (int a = 0; a < 3; ++a) {
    lp.lo[a] = 0.0f;
    lp.ext[a] = 1.0f;
  }
  s->grid_n = lp.L * lp.T * 2u;
  s->B = 1u << (g.mlp_batch_log2 ? (g.mlp_batch_log2 > 20 ? 20 : g.mlp_batch_log2) : 16u);
  if (s->B < 32) s->B = 32;
  s->train_blocks = 512;
  const size_t PR = (size_t)c->P * c->R;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  A(lalloc(&s->gstate, 4 * (size_t)s->grid_n));
  A(lalloc(&s->grid_h, s->grid_n));
  A(lalloc(&s->grid_g, s->grid_n));
  A(lalloc(&s->mlp, kMlpParams));
  A(lalloc(&s->mlp_g, kMlpParams));
  A(lalloc(&s->mlp_m, kMlpParams));
  A(lalloc(&s->mlp_v, kMlpParams));
  A(lalloc(&s->mlp_part, (size_t)s->train_blocks * kMlpParams));
  A(lalloc(&s->mlp_part2, (size_t)kRedGroups * kMlpParams));
  A(lalloc(&s->wb, 16384 + 1024 + 2048));
  A(lalloc(&s->w8, kMlpParams));
  A(lalloc(&s->scales, 16));
  A(lalloc(&s->hitpos, PR));
  A(lalloc(&s->hitnrm, PR));
  A(lalloc(&s->trec, PR));
  s->tflag_blocks = (uint32_t)((PR + kTile - 1) / kTile);
  A(lalloc(&s->tflag, (size_t)s->tflag_blocks * kTile));
  A(lalloc(&s->clist, PR));
  A(lalloc(&s->ccount, (size_t)s->tflag_blocks + 1));
  // the frame's batch holds one sub-batch per optimiser step (at most 2^20 rows)
  const uint32_t steps = g.mlp_steps ? g.mlp_steps : 1u;
  s->sub = std::max<uint32_t>(1u, std::min<uint32_t>(steps, (1u << 20) / s->B));
  const size_t rows = (size_t)s->B * s->sub;
  A(lalloc(&s->batch, 3 * rows));
  A(lalloc(&s->batch_raw, 3 * rows));
  // gradient pairs of a step: every sample, level and corner; keys of level * T + entry
  s->n_pairs = (size_t)s->B * lp.L * 8u;
  uint32_t lbits = 0;
  while ((1u << lbits) < lp.L) ++lbits;
  uint32_t tbits = 0;
  while ((1u << tbits) < lp.T) ++tbits;
  s->key_bits = lbits + tbits;
  for (int k = 0; k < 2; ++k) {
    A(lalloc(&s->bkeys[k], rows));
    A(lalloc(&s->bvals[k], rows));
    A(lalloc(&s->pkeys[k], s->n_pairs));
    A(lalloc(&s->pvals[k], s->n_pairs));
  }
  const size_t nb_max = (std::max(rows, s->n_pairs) + kRsTile - 1) / kRsTile;
  A(lalloc(&s->rs_hist, 256 * nb_max + 256));
  const size_t ntiles = (s->n_pairs + kGredTile - 1) / kGredTile;
  A(lalloc(&s->tail_sum, ntiles));
  A(lalloc(&s->tail_in, ntiles));
  A(lalloc(&s->lpart, s->train_blocks));
  A(lalloc(&s->judge_part, (size_t)c->hit_blocks_per_stripe * kStatStripes));
  A(lalloc(&s->lmlp, PR));
  A(lalloc(&s->acc, 16));
  if (e != hipSuccess) return e;
  A(hipFuncSetAttribute(reinterpret_cast<const void*>(k_train), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)sizeof(TrainSmem)));
  A(hipMemset(s->grid_g, 0, 4 * (size_t)s->grid_n));
  A(hipMemset(s->gstate, 0, 16 * (size_t)s->grid_n));
  A(hipMemset(s->mlp_m, 0, 4 * kMlpParams));
  A(hipMemset(s->mlp_v, 0, 4 * kMlpParams));
  A(hipMemset(s->mlp_g, 0, 4 * kMlpParams));
  A(hipMemset(s->scales, 0, 64));
  A(hipMemset(s->acc, 0, 64));
  A(hipMemset(s->tflag, 0, (size_t)s->tflag_blocks * kTile));
  A(hipMemset(s->lmlp, 0, 16 * PR));
  if (e != hipSuccess) return e;
  const uint64_t n = std::max<uint64_t>(s->grid_n, kMlpParams);
  k_learned_init<<<nblk(n, 256), 256>>>(s->gstate, s->grid_h, lp.L, lp.T, s->mlp, g.seed);
  k_mlp_copies<<<1, 1024>>>(s->mlp, s->wb, s->w8, s->scales);
  {
    // unit activation scales until the first training step measures them
    const float one[3] = {1.0f, 1.0f, 1.0f};
    A(hipMemcpy(s->scales + 6, one, 12, hipMemcpyHostToDevice));
  }
  A(hipGetLastError());
  A(hipDeviceSynchronize());
  return e;
}

void learned_destroy(gi_context* c) {
  LearnedState* s = c->learned;
  if (!s) return;
  void* ptrs[] = {s->gstate, s->grid_h, s->grid_g, s->mlp, s->mlp_g, s->mlp_m, s->mlp_v,
                  s->mlp_part, s->mlp_part2, s->wb, s->w8, s->scales, s->hitpos, s->hitnrm, s->trec, s->tflag, s->clist,
                  s->ccount, s->batch, s->batch_raw, s->bkeys[0], s->bkeys[1], s->bvals[0], s->bvals[1],
                  s->pkeys[0], s->pkeys[1], s->pvals[0], s->pvals[1], s->rs_hist, s->tail_sum, s->tail_in,
                  s->lpart, s->judge_part, s->lmlp, s->acc};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete s;
  c->learned = nullptr;
}

void learned_set_domain(gi_context* c) {
  LearnedState* s = c->learned;
  if (!s) return;
  for (int a = 0; a < 3; ++a) {
    float lo = c->cfg.scene_min[a], hi = c->cfg.scene_max[a];
    if (!(hi > lo)) {
      lo = c->scene_lo[a];
      hi = c->scene_hi[a];
    }
    s->lp.lo[a] = lo;
    s->lp.ext[a] = (hi > lo) ? hi - lo : 1.0f;
  }
}

// one optimiser step on the batch currently in s->batch
static hipError_t train_step(gi_context* c, hipStream_t st, bool apply, uint32_t off, uint32_t stride) {
  LearnedState* s = c->learned;
  const float S = c->cfg.mlp_loss_scale > 0.0f ? c->cfg.mlp_loss_scale : 1.0f;
  // a gradient-only step leaves its dense gradient in grid_g; clear it before the next
  if (s->grad_dirty) k_zero_f32<<<nblk(s->grid_n, 256), 256, 0, st>>>(s->grid_g, s->grid_n);
  s->grad_dirty = false;
  const uint32_t groups = s->B / 32u;
  const uint32_t tblocks = std::min<uint32_t>(s->train_blocks, std::max<uint32_t>(groups, 1u));
  uint32_t log2T = 0;
  while ((1u << log2T) < s->lp.T) ++log2T;
  hipEvent_t ev;
  timer_begin(c, "learned_train", st, &ev);
  // every launched block writes its whole partial, so the partials need no clearing; the
  // gradient pairs fill [0, n_pairs) (L * B * 8)
  const uint32_t n = (uint32_t)s->n_pairs;
  const uint32_t nbt = nblk(n, kRsTile);
  const bool tiles = (s->lp.L & 7u) == 0u;
  k_train<<<tblocks, 64 * kTrainWaves, sizeof(TrainSmem), st>>>(s->lp, s->batch, s->B, off, stride, s->grid_h, s->wb, S,
                                                              s->mlp_part, s->lpart, s->acc, s->scales + 3, log2T,
                                                              s->pkeys[0], s->pvals[0], nbt, s->rs_hist);
  timer_end(c, "learned_train", st, ev);
  k_reduce_mlp<<<dim3(kMlpParams / 256, kRedGroups), 256, 0, st>>>(s->mlp_part, tblocks, s->mlp_part2);
  // the encoding gradient: pairs sorted by entry, summed per entry in a fixed order
  timer_begin(c, "learned_grad_sort", st, &ev);
  int which = 0;
  hipError_t e = radix_sort<float2>(s->pkeys, s->pvals, n, s->key_bits, s->rs_hist, st, which, tiles);
  timer_end(c, "learned_grad_sort", st, ev);
  if (e != hipSuccess) return e;
  const uint32_t nt = nblk(n, kGredTile);
  AdamArgs ag{};
  if (apply) {
    s->step += 1;
    ag.b1 = 0.9f;
    ag.b2 = 0.99f;
    ag.c1 = (float)(1.0 - std::pow(0.9, (double)s->step));
    ag.c2 = (float)(1.0 - std::pow(0.99, (double)s->step));
    ag.inv_scale = 1.0f / S;
    ag.lr = c->cfg.mlp_lr_grid;
    ag.eps = 1e-15f;
  }
  const MlpFinish mf{s->mlp_part2, s->lpart, tblocks, s->mlp_g};
  timer_begin(c, "learned_grad_apply", st, &ev);
  k_gred<0><<<nt, 256, 0, st>>>(s->pkeys[which], s->pvals[which], n, s->tail_sum, s->tail_in, s->gstate, s->grid_h,
                                s->grid_g, ag, s->acc, mf);
  if (apply)
    k_gred<1><<<nt, 256, 0, st>>>(s->pkeys[which], s->pvals[which], n, s->tail_sum, s->tail_in, s->gstate, s->grid_h,
                                  s->grid_g, ag, s->acc, mf);
  else
    k_gred<2><<<nt, 256, 0, st>>>(s->pkeys[which], s->pvals[which], n, s->tail_sum, s->tail_in, s->gstate, s->grid_h,
                                  s->grid_g, ag, s->acc, mf);
  timer_end(c, "learned_grad_apply", st, ev);
  if (apply) {
    AdamArgs am = ag;
    am.lr = c->cfg.mlp_lr_mlp;
    am.eps = 1e-8f;
    timer_begin(c, "learned_adam", st, &ev);
    k_mlp_adam<<<nblk(kMlpParams, 256), 256, 0, st>>>(s->mlp, s->mlp_g, s->mlp_m, s->mlp_v, am, s->acc, s->wb);
    k_mlp_step<<<1, 1024, 0, st>>>(s->mlp, s->acc, s->w8, s->scales, c->d_stats,
                                   c->cfg.cache_mode == GI_CACHE_MLP_FP8);
    timer_end(c, "learned_adam", st, ev);
  } else {
    s->grad_dirty = true;
    k_train_end<<<1, 64, 0, st>>>(s->acc, s->scales + 3, c->d_stats);
  }
  return hipGetLastError();
}

hipError_t learned_train(gi_context* c, hipStream_t st) {
  LearnedState* s = c->learned;
  learned_set_domain(c);
  // the frame's training rays in ray order, then sub * B stratified picks over them, grouped
  // by Morton bucket once; step k trains on rows k, k + sub, k + 2 sub, ... (each step spans
  // the whole scene and its rows stay in spatial order)
  const uint32_t steps = c->cfg.mlp_steps ? c->cfg.mlp_steps : 1u;
  const uint32_t rows = s->B * s->sub;
  const float u = rand_unit_host(hash_pcg(hash_pcg(hash_pcg(hash_pcg(c->cfg.seed) + c->fa.index) + 0x7FFFFFFFu) + 9u));
  hipEvent_t ev;
  timer_begin(c, "learned_select", st, &ev);
  k_tflag_count<<<s->tflag_blocks, 256, 0, st>>>(s->tflag, s->ccount);
  k_scan_counts<<<1, 1024, 0, st>>>(s->ccount, s->tflag_blocks);
  k_tflag_compact<<<s->tflag_blocks, 256, 0, st>>>(s->tflag, s->ccount, s->clist);
  k_select_batch<<<nblk(rows, 256), 256, 0, st>>>(s->clist, s->ccount + s->tflag_blocks, s->trec, s->hitpos,
                                                  s->hitnrm, u, rows, s->batch_raw, s->acc);
  timer_end(c, "learned_select", st, ev);
  hipError_t e = sort_batch(c, st, rows);
  for (uint32_t k = 0; k < steps && e == hipSuccess; ++k) e = train_step(c, st, true, k % s->sub, s->sub);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t learned_step_on(gi_context* c, const float4* pos, const float4* nrm, const float4* tgt, uint32_t n,
                           bool apply, hipStream_t st) {
  LearnedState* s = c->learned;
  learned_set_domain(c);
  if (n != s->B) return hipErrorInvalidValue;
  // batch rows: pos, nrm, target
  hipError_t e = hipMemcpy2DAsync(s->batch_raw, 48, pos, 16, 16, n, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpy2DAsync(s->batch_raw + 1, 48, nrm, 16, 16, n, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpy2DAsync(s->batch_raw + 2, 48, tgt, 16, 16, n, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = sort_batch(c, st, n);
  if (e != hipSuccess) return e;
  return train_step(c, st, apply, 0u, 1u);
}

hipError_t learned_infer_rays(gi_context* c, hipStream_t st) {
  LearnedState* s = c->learned;
  const uint64_t n = (uint64_t)c->P * c->R;
  const uint32_t nb = nblk(n, 64);
  hipEvent_t ev;
  timer_begin(c, "learned_infer", st, &ev);
  if (c->cfg.cache_mode == GI_CACHE_MLP_FP8)
    k_infer<true, true><<<nb, 64, 0, st>>>(s->lp, s->grid_h, s->wb, s->w8, s->scales, s->hitpos, s->hitnrm, 0,
                                           c->d_hit_ids, c->d_hit_count, c->hit_stripe_cap,
                                           c->hit_blocks_per_stripe, s->lmlp);
  else
    k_infer<false, true><<<nb, 64, 0, st>>>(s->lp, s->grid_h, s->wb, s->w8, s->scales, s->hitpos, s->hitnrm, 0,
                                            c->d_hit_ids, c->d_hit_count, c->hit_stripe_cap,
                                            c->hit_blocks_per_stripe, s->lmlp);
  timer_end(c, "learned_infer", st, ev);
  const uint32_t jb = c->hit_blocks_per_stripe * kStatStripes;
  k_judge<<<jb, 64, 0, st>>>(c->d_hit_ids, c->d_hit_count, c->hit_stripe_cap, c->hit_blocks_per_stripe, c->d_rec,
                             c->tab.meta, c->tab.L, s->lmlp, s->judge_part);
  k_judge_decide<<<1, 1024, 0, st>>>(s->judge_part, jb, s->acc, c->cfg.mlp_judge, c->d_stats);
  return hipGetLastError();
}

hipError_t e4m3_encode_array(const float* in, uint8_t* out, uint32_t n, hipStream_t st) {
  if (n) k_e4m3_encode<<<nblk(n, 256), 256, 0, st>>>(in, out, n);
  return hipGetLastError();
}

hipError_t learned_query(gi_context* c, const float4* pos, const float4* nrm, uint32_t n, float4* out, hipStream_t st) {
  LearnedState* s = c->learned;
  if (n == 0) return hipSuccess;
  learned_set_domain(c);
  if (c->cfg.cache_mode == GI_CACHE_MLP_FP8)
    k_infer<true, false><<<nblk(n, 64), 64, 0, st>>>(s->lp, s->grid_h, s->wb, s->w8, s->scales, pos, nrm, n, nullptr,
                                                     nullptr, 0, 1, out);
  else
    k_infer<false, false><<<nblk(n, 64), 64, 0, st>>>(s->lp, s->grid_h, s->wb, s->w8, s->scales, pos, nrm, n, nullptr,
                                                      nullptr, 0, 1, out);
  return hipGetLastError();
}

// blob: header (16 x u32) | grid master | MLP master | grid grad | MLP grad | grid m | grid v |
//       MLP m | MLP v      (grads are scaled by the loss scale)
size_t learned_blob_size(gi_context* c) {
  LearnedState* s = c->learned;
  return 64 + 4 * ((size_t)s->grid_n * 4 + (size_t)kMlpParams * 4);
}

hipError_t learned_save(gi_context* c, void* blob) {
  LearnedState* s = c->learned;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  uint32_t hdr[16] = {0x47494D31u, s->lp.L, s->lp.T, (uint32_t)kMlpParams, (uint32_t)s->step, s->B, 0};
  char* p = static_cast<char*>(blob);
  std::memcpy(p, hdr, 64);
  p += 64;
  const size_t G = 4 * (size_t)s->grid_n, M = 4 * (size_t)kMlpParams;
  // the interleaved grid state goes out as three arrays (values, first and second moments)
  std::vector<float> gs(4 * (size_t)s->grid_n);
  e = hipMemcpy(gs.data(), s->gstate, 16 * (size_t)s->grid_n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  std::vector<float> gp(s->grid_n), gm(s->grid_n), gv(s->grid_n);
  for (size_t i = 0; i < s->grid_n; ++i) {
    const size_t b = 8 * (i >> 1) + (i & 1);
    gp[i] = gs[b];
    gm[i] = gs[b + 2];
    gv[i] = gs[b + 4];
  }
  const void* src[8] = {gp.data(), s->mlp, s->grid_g, s->mlp_g, gm.data(), gv.data(), s->mlp_m, s->mlp_v};
  const bool dev[8] = {false, true, true, true, false, false, true, true};
  const size_t sz[8] = {G, M, G, M, G, G, M, M};
  for (int k = 0; k < 8 && e == hipSuccess; ++k) {
    if (dev[k]) e = hipMemcpy(p, src[k], sz[k], hipMemcpyDeviceToHost);
    else std::memcpy(p, src[k], sz[k]);
    p += sz[k];
  }
  return e;
}

hipError_t learned_load(gi_context* c, const void* blob) {
  LearnedState* s = c->learned;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  uint32_t hdr[16];
  const char* p = static_cast<const char*>(blob);
  std::memcpy(hdr, p, 64);
  if (hdr[0] != 0x47494D31u || hdr[1] != s->lp.L || hdr[2] != s->lp.T) return hipErrorInvalidValue;
  s->step = (int)hdr[4];
  p += 64;
  const size_t G = 4 * (size_t)s->grid_n, M = 4 * (size_t)kMlpParams;
  std::vector<float> gp(s->grid_n), gm(s->grid_n), gv(s->grid_n);
  void* dst[8] = {gp.data(), s->mlp, s->grid_g, s->mlp_g, gm.data(), gv.data(), s->mlp_m, s->mlp_v};
  const bool dev[8] = {false, true, true, true, false, false, true, true};
  const size_t sz[8] = {G, M, G, M, G, G, M, M};
  for (int k = 0; k < 8 && e == hipSuccess; ++k) {
    if (dev[k]) e = hipMemcpy(dst[k], p, sz[k], hipMemcpyHostToDevice);
    else std::memcpy(dst[k], p, sz[k]);
    p += sz[k];
  }
  if (e != hipSuccess) return e;
  std::vector<float> gs(4 * (size_t)s->grid_n, 0.0f);
  for (size_t i = 0; i < s->grid_n; ++i) {
    const size_t b = 8 * (i >> 1) + (i & 1);
    gs[b] = gp[i];
    gs[b + 2] = gm[i];
    gs[b + 4] = gv[i];
  }
  e = hipMemcpy(s->gstate, gs.data(), 16 * (size_t)s->grid_n, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  s->grad_dirty = true;   // the restored gradient is the saved state's, not a clean buffer
  // rebuild the working copies
  k_learned_copy_half<<<nblk(s->grid_n, 256), 256>>>(s->gstate, s->grid_h, s->grid_n);
  k_mlp_copies<<<1, 1024>>>(s->mlp, s->wb, s->w8, s->scales);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return e;
}

hipError_t learned_batch_export(gi_context* c, float* h_raw, float* h_grouped, uint32_t cap_rows, uint32_t& rows,
                                uint32_t& n_train) {
  LearnedState* s = c->learned;
  rows = s->B * s->sub;
  hipError_t e = hipMemcpy(&n_train, s->ccount + s->tflag_blocks, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess || cap_rows < rows) return e;
  if (h_raw) e = hipMemcpy(h_raw, s->batch_raw, 48 * (size_t)rows, hipMemcpyDeviceToHost);
  if (e == hipSuccess && h_grouped) e = hipMemcpy(h_grouped, s->batch, 48 * (size_t)rows, hipMemcpyDeviceToHost);
  return e;
}

void learned_stats(gi_context* c, float* out8) {
  LearnedState* s = c->learned;
  float acc[16];
  if (hipMemcpy(acc, s->acc, 64, hipMemcpyDeviceToHost) != hipSuccess) {
    for (int i = 0; i < 8; ++i) out8[i] = 0.0f;
    return;
  }
  out8[0] = acc[5];
  out8[1] = acc[6];
  out8[2] = acc[4];
  out8[3] = (float)s->step;
  out8[4] = 0.0f;
  out8[5] = acc[7];
  out8[6] = 0.0f;
  out8[7] = 0.0f;
}

// learned-mode outputs of the shading pass
LearnedShadeOut learned_shade_out(gi_context* c) {
  LearnedShadeOut o{};
  LearnedState* s = c->learned;
  if (!s) return o;
  o.hitpos = s->hitpos;
  o.hitnrm = s->hitnrm;
  o.trec = s->trec;
  o.tflag = s->tflag;
  o.tflag_words = s->tflag_blocks * (kTile / 4u);
  return o;
}

LearnedGatherIn learned_gather_in(gi_context* c) {
  LearnedGatherIn g{};
  LearnedState* s = c->learned;
  if (!s) return g;
  g.lmlp = s->lmlp;
  g.flags = s->acc;
  g.meta = c->tab.meta;
  return g;
}

}  // namespace gi
