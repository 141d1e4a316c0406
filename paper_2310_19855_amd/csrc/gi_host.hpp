// Host-side context of the GI library and the launch interface of its kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/gi.h"
#include "gi_types.hpp"

namespace gi {

void build_bvh4(const float* tv, uint32_t n, std::vector<Node4>& nodes, std::vector<uint32_t>& order,
                uint32_t& depth);
void cell_moment_table(double out[64][10]);

// device arrays of the world cache (Section 2.2.1): structure of arrays over N slots
struct Table {
  uint32_t* fp = nullptr;        // fingerprint, 0 = empty
  uint64_t* key = nullptr;       // descriptor of the cell (written by the inserting ray)
  uint4* acc = nullptr;          // fixed-point r, g, b sums and sample count of this frame
  float4* L = nullptr;           // cached outgoing radiance (rgb)
  uint2* meta = nullptr;         // (history samples, life)
  uint32_t* accessed = nullptr;  // touched this frame
  // two-level cache (config cache_tiles): slots are tiles; acc and L are per cell [64][N]
  // (cell-major: entry = cell * N + slot)
  uint32_t* cn = nullptr;        // [64][N] history samples of each cell
  float4* Lq = nullptr;          // [64][N] prefiltered radiance the readers see
};

struct LearnedState;  // learned surrogate (gi_learned.hip)

struct FrameArgs {
  uint32_t index;
  float cam[3];
  float kappa;      // Algorithm 6 distance scale
  uint32_t jx, jy;   // lattice offset of the interpolation (the jitter modulo 8)
  uint32_t sjx, sjy; // the jitter inside a spawn tile of 8 * upscale pixels
};

struct KernelTimer {
  const char* name;
  hipEvent_t a, b;
};

}  // namespace gi

struct gi_context {
  gi_config cfg{};
  int device = 0;
  std::string err;
  // sizes
  uint32_t W = 0, H = 0, TW = 0, TH = 0, P = 0, R = 0, N = 0;
  uint32_t nmip = 0, mask_total = 0;
  uint32_t mip_w[32]{}, mip_h[32]{}, mip_off[32]{};
  // scene
  bool has_scene = false;
  uint32_t nt = 0, n_mats = 0, n_nodes = 0, bvh_depth = 0, stack_depth = 0;
  gi::Node4* d_nodes = nullptr;
  uint32_t* d_spill = nullptr;  // traversal-stack spill rows [spill_rows][spill_stride]
  uint32_t spill_rows = 0, spill_stride = 0;
  float4* d_tris = nullptr;     // leaf-ordered triangles, 3 float4 each (v0.w = index)
  float4* d_tnrm = nullptr;     // [nt + kMaxDyn] unit normal, w = material index
  float4* d_mats = nullptr;     // [2 * n_mats]: albedo, emission
  float4* d_dyn = nullptr;      // [3 * kMaxDyn]
  uint32_t n_dyn = 0;
  uint32_t* d_etri = nullptr;   // emitter triangles
  uint32_t* d_ethr = nullptr;   // their cumulative-area thresholds (scaled to 2^32)
  float4* d_evert = nullptr;    // their vertices, 3 float4 each
  uint32_t n_emit = 0, emit_cap = 0;
  float area_total = 0.0f;
  std::vector<float> h_static_tv;       // static triangles [nt][9] (emitter rebuilds)
  std::vector<uint32_t> h_static_mat;
  std::vector<float> h_mats;
  std::vector<uint32_t> h_static_emit;  // static emitter triangle indices
  std::vector<double> h_static_emit_area;
  float scene_lo[3]{}, scene_hi[3]{};
  // frame state
  uint32_t stage = 0;  // 0 none, 1 spawned, 2 traced, 3 updated
  gi::FrameArgs fa{};
  uint32_t* d_mask = nullptr;   // all MIP levels
  float4* d_ppos = nullptr;
  float4* d_pnrm = nullptr;
  uint4* d_rec = nullptr;       // [P*R] slot, t bits, tri, flags
  uint2* d_rkey = nullptr;      // [P*R] descriptor of the hit (export / learned training)
  float4* d_atlas = nullptr;    // [P*64]
  float4* d_atlas_tmp = nullptr;  // [P*64] between the two filter passes (probe_filter only)
  // temporal reuse (config temporal): the previous frame's final probes and their camera
  uint32_t* d_prev_mask = nullptr;   // [P] level 0
  float4* d_prev_pos = nullptr;      // [P]
  float4* d_prev_nrm = nullptr;      // [P]
  float4* d_prev_atlas = nullptr;    // [P*64]
  float* d_prev_sh = nullptr;        // [P*28] with upscale > 1: SH kept by probes that trace nothing
  uint32_t* d_win = nullptr;         // [P] pixel the previous probe moved to, or sentinel
  uint32_t* d_hist = nullptr;        // [P] previous tile of that probe, or sentinel
  // temporal upscaling (config upscale > 1, Algorithm 2): placement, traced flags, override list
  uint32_t* d_place = nullptr;       // [P] final probe pixel of each tile, or sentinel
  uint32_t* d_traced = nullptr;      // [P] 1 where the tile's probe traces rays this frame
  uint32_t* d_cls = nullptr;         // [P] 1 override tile, 2 empty tile that may take rays
  uint32_t* d_assigned = nullptr;    // [P] per override tile: the lowest empty tile that picked it
  uint32_t* d_over = nullptr;        // [P] override tiles in tile order
  uint32_t* d_over_count = nullptr;  // [1]
  // ray guiding (config ray_guiding): reconstruction and sampling weights of this frame's probes
  float4* d_recon = nullptr;         // [P*64] rgb, distance (-1: empty cell)
  uint32_t* d_cdf = nullptr;         // [P*64] inclusive weight sums
  bool guided = false;               // this frame's spawn built them
  // light grid (config light_grid): box of the frame's hits (order-preserving float codes),
  // per cell the light list and its length
  uint32_t* d_lg_box = nullptr;      // [6] min x, y, z, max x, y, z
  uint32_t* d_lg_part = nullptr;     // [blocks of 256 rays][6] partial boxes
  uint32_t* d_lg_list = nullptr;     // [dim^3][lgrid_k]
  uint32_t* d_lg_count = nullptr;    // [dim^3]
  // world-space reservoirs (config restir): two position-keyed tables, read / written in turn
  uint32_t* d_rs_fp[2] = {nullptr, nullptr};
  uint64_t* d_rs_key[2] = {nullptr, nullptr};
  float4* d_rs_yw[2] = {nullptr, nullptr};   // light point, contribution weight
  float4* d_rs_n[2] = {nullptr, nullptr};    // normal of the storing vertex, w = light bits
  uint32_t* d_rs_m[2] = {nullptr, nullptr};  // count
  uint32_t* d_rs_claim = nullptr;            // lowest ray id offering to each slot
  float4* d_r_rs_yw = nullptr;               // [P*R] each hit's final reservoir
  float4* d_r_rs_n = nullptr;
  uint32_t* d_r_rs_m = nullptr;              // 0: none
  int32_t* d_r_rs_slot = nullptr;
  uint32_t rs_cur = 0;                       // table read this frame
  bool rs_has_prev = false;
  bool has_prev = false;             // a previous frame's probes are stored
  bool reprojected = false;          // this frame's spawn reprojected them
  gi_frame prev_frame{};
  float* d_sh = nullptr;        // [P*28]
  gi::Table tab;
  unsigned long long* d_stats = nullptr;  // [kStatStripes][GI_STAT_COUNT]
  uint32_t* d_hit_ids = nullptr;          // compacted hit list, kStatStripes stripes
  uint32_t* d_hit_count = nullptr;        // [kStatStripes]
  uint32_t hit_blocks_per_stripe = 0, hit_stripe_cap = 0;
  float* d_moments = nullptr;   // [64*10]
  // learned
  gi::LearnedState* learned = nullptr;
  // pinned staging ring for per-frame host-to-device uploads (slot reuse waits on its event)
  static constexpr int kStageSlots = 8;
  char* stage_base = nullptr;
  size_t stage_slot_bytes = 0;
  hipEvent_t stage_ev[kStageSlots]{};
  bool stage_used[kStageSlots]{};
  int stage_next = 0;
  std::vector<uint32_t> h_etri, h_ethr;   // current emitter table (host mirror)
  std::vector<float> h_evert;
  // profiling
  uint32_t prof = 0;   // kernel timers: 0 off, 1 every kernel, 2 the probe-ray traversal only
  std::vector<gi::KernelTimer> timers;
  std::vector<hipEvent_t> event_pool;
  std::vector<std::string> prof_names;
  std::vector<uint32_t> prof_counts;
  std::vector<double> prof_ms;
};

namespace gi {

// launch helpers (gi_kernels.hip)
void timer_begin(gi_context* c, const char* name, hipStream_t s, hipEvent_t* a);
void timer_end(gi_context* c, const char* name, hipStream_t s, hipEvent_t a);

hipError_t launch_gbuffer(gi_context* c, const gi_frame* f, float4* pos, float4* nrm, float4* alb,
                          uint32_t* prim, hipStream_t s);
hipError_t launch_spawn(gi_context* c, const float4* pos, const float4* nrm, const uint32_t* prim, hipStream_t s);
hipError_t launch_trace(gi_context* c, hipStream_t s);
hipError_t launch_update(gi_context* c, hipStream_t s);
hipError_t launch_interpolate(gi_context* c, const float4* pos, const float4* nrm, const uint32_t* prim,
                              float4* out, hipStream_t s);
hipError_t launch_query(gi_context* c, const float4* pos, const float4* nrm, uint32_t n, float4* out,
                        hipStream_t s);
hipError_t launch_trace_rays(gi_context* c, const float4* o, const float4* d, uint32_t n, uint32_t any,
                             uint32_t* tri, float* t, hipStream_t s);
hipError_t launch_zero_stats(gi_context* c, hipStream_t s);
hipError_t launch_count_traversal(gi_context* c, unsigned long long* out, hipStream_t s);
// gi_trace_rays_noalloc: a static device array of kNoAllocScratchWords u32 (16 MiB) per GPU
// holds the traversal-stack spill rows; scratch_init looks up its address on the current
// device (once per device, at gi_create); rays are traced in chunks of
// noalloc_chunk_rays(spill_rows) lane ids (0: the BVH is too deep for the array)
constexpr size_t kNoAllocScratchWords = (size_t)4 << 20;
constexpr int kMaxDevices = 64;
hipError_t scratch_init(int device);
uint32_t noalloc_chunk_rays(uint32_t spill_rows);
hipError_t launch_trace_rays_noalloc(gi_context* c, const float4* o, const float4* d, uint32_t n, uint32_t any,
                                     uint32_t* tri, float* t, hipStream_t s);

// learned surrogate (gi_learned.hip)
struct LearnedShadeOut {       // written by the shading pass in learned mode (else all null)
  float4* hitpos = nullptr;    // [P*R] hit point
  float4* hitnrm = nullptr;    // [P*R] face-forwarded normal
  float4* trec = nullptr;      // [P*R] training target of the ray's hit (rgb, w = 1)
  uint8_t* tflag = nullptr;    // [P*R, padded] 1 where trec holds this frame's sample
  uint32_t tflag_words = 0;    // u32 words of tflag cleared per frame
};
struct LearnedGatherIn {       // read by the probe gather in learned mode (else all null)
  const float4* lmlp = nullptr;   // [P*R] surrogate radiance at each hit
  const float* flags = nullptr;   // [4] = fallback flag
  const uint2* meta = nullptr;    // world-cache (history samples, life)
};
LearnedShadeOut learned_shade_out(gi_context* c);
LearnedGatherIn learned_gather_in(gi_context* c);
void learned_set_domain(gi_context* c);
hipError_t learned_step_on(gi_context* c, const float4* pos, const float4* nrm, const float4* tgt, uint32_t n,
                           bool apply, hipStream_t st);
hipError_t learned_create(gi_context* c);
void learned_destroy(gi_context* c);
hipError_t learned_train(gi_context* c, hipStream_t s);
hipError_t learned_infer_rays(gi_context* c, hipStream_t s);
hipError_t learned_query(gi_context* c, const float4* pos, const float4* nrm, uint32_t n, float4* out,
                         hipStream_t s);
size_t learned_blob_size(gi_context* c);
hipError_t learned_save(gi_context* c, void* blob);
hipError_t learned_load(gi_context* c, const void* blob);
void learned_stats(gi_context* c, float* out8);
// the frame's training batch as selected and as grouped (rows x 3 float4 each), the number of
// rows and of the frame's training rays; copies only when cap_rows >= rows
hipError_t learned_batch_export(gi_context* c, float* h_raw, float* h_grouped, uint32_t cap_rows, uint32_t& rows,
                                uint32_t& n_train);
hipError_t e4m3_encode_array(const float* in, uint8_t* out, uint32_t n, hipStream_t st);

}  // namespace gi
