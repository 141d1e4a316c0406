// C ABI of the GI library: argument checks, buffer ownership, frame-order state and the
// host-side parts of the method (Halton jitter, Algorithm 6 distance scale, emitter table).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>

#include "gi_host.hpp"

using gi::Node4;

namespace {

#define GI_TRY_HIP(ctx, expr)                                                         \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
      return e_ == hipErrorOutOfMemory ? GI_ERR_OOM : GI_ERR_HIP;                     \
    }                                                                                 \
  } while (0)

gi_status fail(gi_context* c, gi_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * count);
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// floor(n * radical_inverse_base(index)) in exact integer arithmetic (Section 2.1.1 jitter)
uint32_t halton_cell(uint32_t index, uint32_t base, uint32_t n) {
  uint64_t num = 0, den = 1;
  for (uint32_t i = index; i > 0; i /= base) {
    num = num * base + (i % base);
    den *= base;
  }
  return (uint32_t)(((uint64_t)n * num) / den);
}

double tri_area(const float* v) {
  const double ax = (double)v[3] - v[0], ay = (double)v[4] - v[1], az = (double)v[5] - v[2];
  const double bx = (double)v[6] - v[0], by = (double)v[7] - v[1], bz = (double)v[8] - v[2];
  const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
  return 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
}

// unit winding normal in float32 (the order of operations is part of the numerics contract)
void unit_normal(const float* v, float* n) {
  const float e1x = v[3] - v[0], e1y = v[4] - v[1], e1z = v[5] - v[2];
  const float e2x = v[6] - v[0], e2y = v[7] - v[1], e2z = v[8] - v[2];
  const float cx = e1y * e2z - e1z * e2y;
  const float cy = e1z * e2x - e1x * e2z;
  const float cz = e1x * e2y - e1y * e2x;
  const float len = std::sqrt(cx * cx + cy * cy + cz * cz);
  if (len > 0.0f) {
    n[0] = cx / len;
    n[1] = cy / len;
    n[2] = cz / len;
  } else {
    n[0] = n[1] = n[2] = 0.0f;
  }
}

bool emits(const std::vector<float>& mats, uint32_t m) {
  return mats[6 * m + 3] > 0.0f || mats[6 * m + 4] > 0.0f || mats[6 * m + 5] > 0.0f;
}

// One staging slot of pinned host memory holding `bytes`; waits until the slot's previous
// copies have completed.  Returns nullptr on failure.
char* stage_acquire(gi_context* c, size_t bytes, int* slot_out) {
  if (bytes > c->stage_slot_bytes) {
    for (int i = 0; i < gi_context::kStageSlots; ++i)
      if (c->stage_used[i]) (void)hipEventSynchronize(c->stage_ev[i]);
    if (c->stage_base) (void)hipHostFree(c->stage_base);
    c->stage_base = nullptr;
    size_t sb = 1 << 16;
    while (sb < bytes) sb <<= 1;
    if (hipHostMalloc(reinterpret_cast<void**>(&c->stage_base), sb * gi_context::kStageSlots) != hipSuccess) {
      c->stage_slot_bytes = 0;
      return nullptr;
    }
    c->stage_slot_bytes = sb;
    for (int i = 0; i < gi_context::kStageSlots; ++i) {
      if (!c->stage_ev[i] && hipEventCreateWithFlags(&c->stage_ev[i], hipEventDisableTiming) != hipSuccess) return nullptr;
      c->stage_used[i] = false;
    }
  }
  const int k = c->stage_next;
  c->stage_next = (k + 1) % gi_context::kStageSlots;
  if (c->stage_used[k]) (void)hipEventSynchronize(c->stage_ev[k]);
  *slot_out = k;
  return c->stage_base + (size_t)k * c->stage_slot_bytes;
}

void stage_release(gi_context* c, int slot, hipStream_t s) {
  (void)hipEventRecord(c->stage_ev[slot], s);
  c->stage_used[slot] = true;
}

// Area-proportional emitter table over static then dynamic emitters: global triangle index,
// cumulative-area thresholds scaled to 2^32 (last = 2^32 - 1) and vertices.  Only the entries
// that changed since the last upload are copied, through the pinned staging ring.
gi_status upload_emitters(gi_context* c, const float* dyn_tv, const uint32_t* dyn_mat, uint32_t nd,
                          hipStream_t s) {
  std::vector<uint32_t> etri;
  std::vector<double> area;
  std::vector<float> verts;
  for (size_t k = 0; k < c->h_static_emit.size(); ++k) {
    const uint32_t t = c->h_static_emit[k];
    etri.push_back(t);
    area.push_back(c->h_static_emit_area[k]);
    const float* v = &c->h_static_tv[9 * (size_t)t];
    // w of the first vertex: the triangle's area, rounded once from float64
    for (int i = 0; i < 3; ++i)
      verts.insert(verts.end(), {v[3 * i], v[3 * i + 1], v[3 * i + 2], i == 0 ? (float)area.back() : 0.0f});
  }
  for (uint32_t k = 0; k < nd; ++k) {
    if (!emits(c->h_mats, dyn_mat[k])) continue;
    etri.push_back(c->nt + k);
    area.push_back(tri_area(dyn_tv + 9 * (size_t)k));
    const float* v = dyn_tv + 9 * (size_t)k;
    for (int i = 0; i < 3; ++i)
      verts.insert(verts.end(), {v[3 * i], v[3 * i + 1], v[3 * i + 2], i == 0 ? (float)area.back() : 0.0f});
  }
  const uint32_t n = (uint32_t)etri.size();
  std::vector<uint32_t> thr(n);
  double acc = 0.0;
  for (uint32_t i = 0; i < n; ++i) acc += area[i];
  double run = 0.0;
  for (uint32_t i = 0; i < n; ++i) {
    run += area[i];
    const double t = std::floor(run / acc * 4294967296.0);
    thr[i] = (i + 1 == n || t >= 4294967295.0) ? 4294967295u : (uint32_t)t;
  }
  if (n > c->emit_cap) {
    // the kernels of earlier frames may still read the old table
    GI_TRY_HIP(c, hipDeviceSynchronize());
    dfree(c->d_etri);
    dfree(c->d_ethr);
    dfree(c->d_evert);
    GI_TRY_HIP(c, dalloc(&c->d_etri, n));
    GI_TRY_HIP(c, dalloc(&c->d_ethr, n));
    GI_TRY_HIP(c, dalloc(&c->d_evert, 3 * (size_t)n));
    c->emit_cap = n;
    c->h_etri.clear();
    c->h_ethr.clear();
    c->h_evert.clear();
  }
  // first entry that differs from what the device holds
  uint32_t first = 0;
  if (c->h_etri.size() == n) {
    while (first < n && c->h_etri[first] == etri[first] && c->h_ethr[first] == thr[first] &&
           std::memcmp(&c->h_evert[12 * (size_t)first], &verts[12 * (size_t)first], 48) == 0)
      ++first;
  }
  if (first < n) {
    const size_t m = n - first;
    const size_t bytes = m * (4 + 4 + 48);
    int slot;
    char* st = stage_acquire(c, bytes, &slot);
    if (!st) return fail(c, GI_ERR_OOM, "pinned staging allocation failed");
    std::memcpy(st, &etri[first], 4 * m);
    std::memcpy(st + 4 * m, &thr[first], 4 * m);
    std::memcpy(st + 8 * m, &verts[12 * (size_t)first], 48 * m);
    GI_TRY_HIP(c, hipMemcpyAsync(c->d_etri + first, st, 4 * m, hipMemcpyHostToDevice, s));
    GI_TRY_HIP(c, hipMemcpyAsync(c->d_ethr + first, st + 4 * m, 4 * m, hipMemcpyHostToDevice, s));
    GI_TRY_HIP(c, hipMemcpyAsync(c->d_evert + 3 * (size_t)first, st + 8 * m, 48 * m, hipMemcpyHostToDevice, s));
    stage_release(c, slot, s);
  }
  c->h_etri = std::move(etri);
  c->h_ethr = std::move(thr);
  c->h_evert = std::move(verts);
  c->n_emit = n;
  c->area_total = (float)acc;
  return GI_OK;
}

void free_frame_buffers(gi_context* c) {
  dfree(c->d_mask);
  dfree(c->d_ppos);
  dfree(c->d_pnrm);
  dfree(c->d_rec);
  dfree(c->d_rkey);
  dfree(c->d_atlas);
  dfree(c->d_atlas_tmp);
  dfree(c->d_prev_mask);
  dfree(c->d_prev_pos);
  dfree(c->d_prev_nrm);
  dfree(c->d_prev_atlas);
  dfree(c->d_prev_sh);
  dfree(c->d_win);
  dfree(c->d_hist);
  dfree(c->d_place);
  dfree(c->d_traced);
  dfree(c->d_cls);
  dfree(c->d_assigned);
  dfree(c->d_over);
  dfree(c->d_over_count);
  dfree(c->d_recon);
  dfree(c->d_cdf);
  dfree(c->d_lg_box);
  dfree(c->d_lg_part);
  dfree(c->d_lg_list);
  dfree(c->d_lg_count);
  for (int t = 0; t < 2; ++t) {
    dfree(c->d_rs_fp[t]);
    dfree(c->d_rs_key[t]);
    dfree(c->d_rs_yw[t]);
    dfree(c->d_rs_n[t]);
    dfree(c->d_rs_m[t]);
  }
  dfree(c->d_rs_claim);
  dfree(c->d_r_rs_yw);
  dfree(c->d_r_rs_n);
  dfree(c->d_r_rs_m);
  dfree(c->d_r_rs_slot);
  dfree(c->d_sh);
  dfree(c->tab.fp);
  dfree(c->tab.key);
  dfree(c->tab.acc);
  dfree(c->tab.L);
  dfree(c->tab.meta);
  dfree(c->tab.accessed);
  dfree(c->tab.cn);
  dfree(c->tab.Lq);
  dfree(c->d_stats);
  dfree(c->d_hit_ids);
  dfree(c->d_hit_count);
  dfree(c->d_moments);
}

void free_scene(gi_context* c) {
  dfree(c->d_nodes);
  dfree(c->d_spill);
  c->spill_rows = 0;
  dfree(c->d_tris);
  dfree(c->d_tnrm);
  dfree(c->d_mats);
  dfree(c->d_dyn);
  dfree(c->d_etri);
  dfree(c->d_ethr);
  dfree(c->d_evert);
  c->emit_cap = 0;
  c->n_emit = 0;
  c->has_scene = false;
}

gi_status check_config(const gi_config* g, std::string& why) {
  if (g->width < 8 || g->height < 8 || g->width > 8192 || g->height > 8192) { why = "width/height out of [8, 8192]"; return GI_ERR_INVALID_ARG; }
  if (g->rays_per_probe < 1 || g->rays_per_probe > 256) { why = "rays_per_probe out of [1, 256]"; return GI_ERR_INVALID_ARG; }
  if (g->table_log2 < 6 || g->table_log2 > 28) { why = "table_log2 out of [6, 28]"; return GI_ERR_INVALID_ARG; }
  if (g->bounces < 1 || g->bounces > 2) { why = "bounces must be 1 or 2"; return GI_ERR_INVALID_ARG; }
  if (g->frac_bits < 1 || g->frac_bits > 16) { why = "frac_bits out of [1, 16]"; return GI_ERR_INVALID_ARG; }
  if (g->max_life < 1) { why = "max_life must be >= 1"; return GI_ERR_INVALID_ARG; }
  if (!(g->cell_scale > 0.0f) || !(g->r_max > 0.0f) || !(g->eps_scale >= 0.0f)) { why = "cell_scale, r_max must be > 0"; return GI_ERR_INVALID_ARG; }
  // a wave adds up to 64 quantised samples of one cell before its atomic: that group sum must
  // fit a u32, or it would wrap without the carry being seen
  if (!(g->r_max < 1e30f) || (double)g->r_max * std::ldexp(1.0, (int)g->frac_bits) * 64.0 >= 4294967296.0 - 64.0) {
    why = "r_max * 2^frac_bits * 64 must stay below 2^32";
    return GI_ERR_INVALID_ARG;
  }
  if (g->cache_mode > GI_CACHE_MLP_FP8) { why = "unknown cache_mode"; return GI_ERR_INVALID_ARG; }
  if (g->probe_filter > 1) { why = "probe_filter must be 0 or 1"; return GI_ERR_INVALID_ARG; }
  if (!(g->lod_scale >= 0.0f) || !(g->lod_scale < 1e30f)) { why = "lod_scale must be finite and >= 0"; return GI_ERR_INVALID_ARG; }
  if (g->temporal > 1) { why = "temporal must be 0 or 1"; return GI_ERR_INVALID_ARG; }
  if (g->upscale > 4) { why = "upscale must be 0..4"; return GI_ERR_INVALID_ARG; }
  if (g->upscale > 1 && !g->temporal) { why = "upscale > 1 needs temporal = 1"; return GI_ERR_INVALID_ARG; }
  if (g->ray_guiding > 1) { why = "ray_guiding must be 0 or 1"; return GI_ERR_INVALID_ARG; }
  if (g->ray_guiding && !g->temporal) { why = "ray_guiding needs temporal = 1"; return GI_ERR_INVALID_ARG; }
  if (g->cache_tiles > 1) { why = "cache_tiles must be 0 or 1"; return GI_ERR_INVALID_ARG; }
  if (g->cache_tiles && g->cache_mode != GI_CACHE_PLAIN) { why = "cache_tiles needs the plain cache"; return GI_ERR_INVALID_ARG; }
  if (g->cache_tiles && g->table_log2 > 22) { why = "cache_tiles: table_log2 (tiles) out of [6, 22]"; return GI_ERR_INVALID_ARG; }
  if (g->light_grid > 1) { why = "light_grid must be 0 or 1"; return GI_ERR_INVALID_ARG; }
  if (g->light_grid && (g->lgrid_dim < 1 || g->lgrid_dim > 32 || g->lgrid_k < 1 || g->lgrid_k > 256 ||
                        g->ris_candidates < 1 || g->ris_candidates > 8 || !(g->lgrid_threshold > 0.0f))) {
    why = "light grid: lgrid_dim in [1, 32], lgrid_k in [1, 256], ris_candidates in [1, 8], lgrid_threshold > 0";
    return GI_ERR_INVALID_ARG;
  }
  if (g->restir > 1 || (g->restir && !g->light_grid)) { why = "restir must be 0 or 1 and needs light_grid"; return GI_ERR_INVALID_ARG; }
  if (g->restir && (g->restir_log2 < 6 || g->restir_log2 > 24)) { why = "restir_log2 out of [6, 24]"; return GI_ERR_INVALID_ARG; }
  if (g->restir && (g->restir_cap < 1 || g->restir_cap > 64)) { why = "restir_cap out of [1, 64]"; return GI_ERR_INVALID_ARG; }
  return GI_OK;
}

}  // namespace

extern "C" {

const char* gi_version(void) { return "gi-mi355x 0.1 (gfx950)"; }

const char* gi_last_error(const gi_context* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gi_status gi_create(const gi_config* cfg, gi_context** out) {
  if (!cfg || !out) return GI_ERR_INVALID_ARG;
  *out = nullptr;
  std::string why;
  if (check_config(cfg, why) != GI_OK) return GI_ERR_INVALID_ARG;
  gi_context* c = nullptr;
  try {
    c = new gi_context();
  } catch (...) {
    return GI_ERR_OOM;
  }
  c->cfg = *cfg;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    delete c;
    return GI_ERR_HIP;
  }
  c->device = dev;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete c;
    return GI_ERR_HIP;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    delete c;
    return GI_ERR_UNSUPPORTED;
  }
  // the device address of gi_trace_rays_noalloc's static scratch array on this device
  if (gi::scratch_init(dev) != hipSuccess) {
    delete c;
    return GI_ERR_HIP;
  }
  c->W = cfg->width;
  c->H = cfg->height;
  c->TW = (c->W + 7) / 8;
  c->TH = (c->H + 7) / 8;
  c->P = c->TW * c->TH;
  c->R = cfg->rays_per_probe;
  c->N = 1u << cfg->table_log2;
  uint32_t w = c->TW, h = c->TH, off = 0, k = 0;
  for (;;) {
    c->mip_w[k] = w;
    c->mip_h[k] = h;
    c->mip_off[k] = off;
    off += w * h;
    ++k;
    if (w == 1 && h == 1) break;
    w = (w + 1) / 2;
    h = (h + 1) / 2;
  }
  c->nmip = k;
  c->mask_total = off;
  const size_t PR = (size_t)c->P * c->R;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  A(dalloc(&c->d_mask, c->mask_total));
  A(dalloc(&c->d_ppos, c->P));
  A(dalloc(&c->d_pnrm, c->P));
  A(dalloc(&c->d_rec, PR));
  A(dalloc(&c->d_rkey, PR));
  A(dalloc(&c->d_atlas, (size_t)c->P * 64));
  if (cfg->probe_filter) A(dalloc(&c->d_atlas_tmp, (size_t)c->P * 64));
  if (cfg->temporal) {
    A(dalloc(&c->d_prev_mask, (size_t)c->P));
    A(dalloc(&c->d_prev_pos, (size_t)c->P));
    A(dalloc(&c->d_prev_nrm, (size_t)c->P));
    A(dalloc(&c->d_prev_atlas, (size_t)c->P * 64));
    A(dalloc(&c->d_win, (size_t)c->P));
    A(dalloc(&c->d_hist, (size_t)c->P));
  }
  if (cfg->upscale > 1) {
    A(dalloc(&c->d_prev_sh, (size_t)c->P * 28));
    A(dalloc(&c->d_place, (size_t)c->P));
    A(dalloc(&c->d_traced, (size_t)c->P));
    A(dalloc(&c->d_cls, (size_t)c->P));
    A(dalloc(&c->d_assigned, (size_t)c->P));
    A(dalloc(&c->d_over, (size_t)c->P));
    A(dalloc(&c->d_over_count, 1));
  }
  if (cfg->ray_guiding) {
    A(dalloc(&c->d_recon, (size_t)c->P * 64));
    A(dalloc(&c->d_cdf, (size_t)c->P * 64));
  }
  if (cfg->light_grid) {
    const size_t cells = (size_t)cfg->lgrid_dim * cfg->lgrid_dim * cfg->lgrid_dim;
    A(dalloc(&c->d_lg_box, 6));
    A(dalloc(&c->d_lg_part, 6 * ((PR + 255) / 256)));
    A(dalloc(&c->d_lg_list, cells * cfg->lgrid_k));
    A(dalloc(&c->d_lg_count, cells));
  }
  if (cfg->restir) {
    const size_t NR = (size_t)1 << cfg->restir_log2;
    for (int t = 0; t < 2; ++t) {
      A(dalloc(&c->d_rs_fp[t], NR));
      A(dalloc(&c->d_rs_key[t], NR));
      A(dalloc(&c->d_rs_yw[t], NR));
      A(dalloc(&c->d_rs_n[t], NR));
      A(dalloc(&c->d_rs_m[t], NR));
    }
    A(dalloc(&c->d_rs_claim, NR));
    A(dalloc(&c->d_r_rs_yw, PR));
    A(dalloc(&c->d_r_rs_n, PR));
    A(dalloc(&c->d_r_rs_m, PR));
    A(dalloc(&c->d_r_rs_slot, PR));
  }
  A(dalloc(&c->d_sh, (size_t)c->P * 28));
  A(dalloc(&c->tab.fp, c->N));
  A(dalloc(&c->tab.key, c->N));
  const size_t NC = (size_t)c->N * (cfg->cache_tiles ? 64u : 1u);   // cells
  A(dalloc(&c->tab.acc, NC));
  A(dalloc(&c->tab.L, NC));
  if (cfg->cache_tiles) {
    A(dalloc(&c->tab.cn, NC));
    A(dalloc(&c->tab.Lq, NC));
  }
  A(dalloc(&c->tab.meta, c->N));
  A(dalloc(&c->tab.accessed, c->N));
  A(dalloc(&c->d_stats, (size_t)GI_STAT_COUNT * gi::kStatStripesHost));
  {
    const uint32_t nblk = (uint32_t)((PR + 63) / 64);
    c->hit_blocks_per_stripe = (nblk + gi::kStatStripesHost - 1) / gi::kStatStripesHost;
    c->hit_stripe_cap = c->hit_blocks_per_stripe * 64;
    A(dalloc(&c->d_hit_ids, (size_t)c->hit_stripe_cap * gi::kStatStripesHost));
    A(dalloc(&c->d_hit_count, gi::kStatStripesHost));
  }
  A(dalloc(&c->d_moments, 640));
  if (e == hipSuccess) {
    A(hipMemset(c->tab.fp, 0, 4 * (size_t)c->N));
    A(hipMemset(c->tab.key, 0, 8 * (size_t)c->N));
    A(hipMemset(c->tab.acc, 0, 16 * NC));
    A(hipMemset(c->tab.L, 0, 16 * NC));
    if (cfg->cache_tiles) {
      A(hipMemset(c->tab.cn, 0, 4 * NC));
      A(hipMemset(c->tab.Lq, 0, 16 * NC));
    }
    A(hipMemset(c->tab.meta, 0, 8 * (size_t)c->N));
    A(hipMemset(c->tab.accessed, 0, 4 * (size_t)c->N));
    A(hipMemset(c->d_stats, 0, 8 * (size_t)GI_STAT_COUNT * gi::kStatStripesHost));
    A(hipMemset(c->d_hit_count, 0, 4 * gi::kStatStripesHost));
    A(hipMemset(c->d_rec, 0, 16 * PR));
    A(hipMemset(c->d_rkey, 0, 8 * PR));
    A(hipMemset(c->d_atlas, 0, 16 * (size_t)c->P * 64));
    A(hipMemset(c->d_sh, 0, 4 * (size_t)c->P * 28));
  }
  if (e == hipSuccess) {
    double mom[64][10];
    gi::cell_moment_table(mom);
    float fm[640];
    for (int i = 0; i < 64; ++i)
      for (int j = 0; j < 10; ++j) fm[10 * i + j] = (float)mom[i][j];
    A(hipMemcpy(c->d_moments, fm, sizeof(fm), hipMemcpyHostToDevice));
  }
  if (e == hipSuccess && cfg->cache_mode != GI_CACHE_PLAIN) A(gi::learned_create(c));
  if (e != hipSuccess) {
    free_frame_buffers(c);
    gi::learned_destroy(c);
    delete c;
    return e == hipErrorOutOfMemory ? GI_ERR_OOM : GI_ERR_HIP;
  }
  *out = c;
  return GI_OK;
}

void gi_destroy(gi_context* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  free_frame_buffers(c);
  free_scene(c);
  gi::learned_destroy(c);
  for (auto& t : c->timers) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto& ev : c->event_pool) (void)hipEventDestroy(ev);
  for (int i = 0; i < gi_context::kStageSlots; ++i)
    if (c->stage_ev[i]) (void)hipEventDestroy(c->stage_ev[i]);
  if (c->stage_base) (void)hipHostFree(c->stage_base);
  delete c;
}

gi_status gi_build_bvh(gi_context* c, const float* h_verts, uint32_t n_verts, const uint32_t* h_idx, uint32_t n_tris,
                       const uint32_t* h_tri_mat, const float* h_mats, uint32_t n_mats) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (!h_verts || !h_idx || !h_tri_mat || !h_mats || n_mats == 0) return fail(c, GI_ERR_INVALID_ARG, "null scene array");
  if (n_tris >= (1u << 24)) return fail(c, GI_ERR_INVALID_ARG, "at most 2^24 - 1 triangles");
  try {
    for (uint32_t i = 0; i < 3 * n_tris; ++i)
      if (h_idx[i] >= n_verts) return fail(c, GI_ERR_INVALID_ARG, "vertex index out of range");
    for (uint32_t i = 0; i < n_tris; ++i)
      if (h_tri_mat[i] >= n_mats) return fail(c, GI_ERR_INVALID_ARG, "material index out of range");
    free_scene(c);
    c->nt = n_tris;
    c->n_mats = n_mats;
    c->h_static_tv.assign(9 * (size_t)n_tris, 0.0f);
    c->h_static_mat.assign(h_tri_mat, h_tri_mat + n_tris);
    c->h_mats.assign(h_mats, h_mats + 6 * (size_t)n_mats);
    float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
    for (uint32_t i = 0; i < n_tris; ++i)
      for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) {
          const float v = h_verts[3 * (size_t)h_idx[3 * (size_t)i + k] + a];
          c->h_static_tv[9 * (size_t)i + 3 * k + a] = v;
          lo[a] = std::min(lo[a], v);
          hi[a] = std::max(hi[a], v);
        }
    for (int a = 0; a < 3; ++a) {
      c->scene_lo[a] = lo[a];
      c->scene_hi[a] = hi[a];
    }
    std::vector<Node4> nodes;
    std::vector<uint32_t> order;
    uint32_t depth = 0;
    gi::build_bvh4(c->h_static_tv.data(), n_tris, nodes, order, depth);
    c->n_nodes = (uint32_t)nodes.size();
    c->bvh_depth = depth;
    const uint32_t need = 3 * depth + 1;
    // an ordered 4-wide walk holds at most 3 entries per level: the top 16 stay in LDS, the
    // rest go to one spill row each, per lane id
    if (need > 256) return fail(c, GI_ERR_UNSUPPORTED, "BVH deeper than 85 levels");
    c->stack_depth = need;
    const uint32_t lds = (uint32_t)gi::kLdsStackEntries;
    c->spill_rows = need > lds ? need - lds : 0;
    c->spill_stride = std::max(c->P * c->R, c->W * c->H);
    if (c->spill_rows) GI_TRY_HIP(c, dalloc(&c->d_spill, (size_t)c->spill_rows * c->spill_stride));
    // leaf slots in order; a triangle split in space by the builder fills several
    std::vector<float4> tris(3 * std::max<size_t>(order.size(), 1));
    for (size_t i = 0; i < order.size(); ++i) {
      const uint32_t t = order[i];
      const float* v = &c->h_static_tv[9 * (size_t)t];
      uint32_t bits = t;
      float w;
      std::memcpy(&w, &bits, 4);
      tris[3 * (size_t)i] = make_float4(v[0], v[1], v[2], w);
      tris[3 * (size_t)i + 1] = make_float4(v[3], v[4], v[5], 0.0f);
      tris[3 * (size_t)i + 2] = make_float4(v[6], v[7], v[8], 0.0f);
    }
    std::vector<float4> tn((size_t)n_tris + gi::kMaxDyn);
    for (uint32_t i = 0; i < n_tris; ++i) {
      float n[3];
      unit_normal(&c->h_static_tv[9 * (size_t)i], n);
      uint32_t mb = h_tri_mat[i];
      float w;
      std::memcpy(&w, &mb, 4);
      tn[i] = make_float4(n[0], n[1], n[2], w);
    }
    std::vector<float4> mats(2 * (size_t)n_mats);
    for (uint32_t m = 0; m < n_mats; ++m) {
      mats[2 * m] = make_float4(h_mats[6 * m], h_mats[6 * m + 1], h_mats[6 * m + 2], 0.0f);
      mats[2 * m + 1] = make_float4(h_mats[6 * m + 3], h_mats[6 * m + 4], h_mats[6 * m + 5], 0.0f);
    }
    GI_TRY_HIP(c, dalloc(&c->d_nodes, nodes.size()));
    GI_TRY_HIP(c, dalloc(&c->d_tris, tris.size()));
    GI_TRY_HIP(c, dalloc(&c->d_tnrm, tn.size()));
    GI_TRY_HIP(c, dalloc(&c->d_mats, mats.size()));
    GI_TRY_HIP(c, dalloc(&c->d_dyn, 3 * (size_t)gi::kMaxDyn));
    GI_TRY_HIP(c, hipMemcpy(c->d_nodes, nodes.data(), sizeof(Node4) * nodes.size(), hipMemcpyHostToDevice));
    GI_TRY_HIP(c, hipMemcpy(c->d_tris, tris.data(), sizeof(float4) * tris.size(), hipMemcpyHostToDevice));
    GI_TRY_HIP(c, hipMemcpy(c->d_tnrm, tn.data(), sizeof(float4) * tn.size(), hipMemcpyHostToDevice));
    GI_TRY_HIP(c, hipMemcpy(c->d_mats, mats.data(), sizeof(float4) * mats.size(), hipMemcpyHostToDevice));
    c->n_dyn = 0;
    c->h_static_emit.clear();
    c->h_static_emit_area.clear();
    for (uint32_t i = 0; i < n_tris; ++i)
      if (emits(c->h_mats, h_tri_mat[i])) {
        c->h_static_emit.push_back(i);
        c->h_static_emit_area.push_back(tri_area(&c->h_static_tv[9 * (size_t)i]));
      }
    const gi_status st = upload_emitters(c, nullptr, nullptr, 0, nullptr);
    if (st != GI_OK) return st;
    GI_TRY_HIP(c, hipDeviceSynchronize());
    c->has_scene = true;
    c->stage = 0;
    if (c->learned) {
      for (int a = 0; a < 3; ++a) {
        if (c->cfg.scene_min[a] == 0.0f && c->cfg.scene_max[a] == 0.0f) {
          c->cfg.scene_min[a] = lo[a];
          c->cfg.scene_max[a] = hi[a];
        }
      }
    }
    return GI_OK;
  } catch (const std::bad_alloc&) {
    return fail(c, GI_ERR_OOM, "host allocation failed");
  } catch (const std::exception& ex) {
    return fail(c, GI_ERR_INTERNAL, ex.what());
  }
}

gi_status gi_bvh_build_host(const float* h_tv, uint32_t n_tris, void* h_nodes, uint32_t cap_nodes, uint32_t* h_slots,
                            uint32_t cap_slots, uint32_t* n_nodes, uint32_t* n_slots, uint32_t* depth) {
  if ((!h_tv && n_tris) || !n_nodes || !n_slots || !depth) return GI_ERR_INVALID_ARG;
  try {
    std::vector<Node4> nodes;
    std::vector<uint32_t> order;
    uint32_t d = 0;
    gi::build_bvh4(h_tv, n_tris, nodes, order, d);
    *n_nodes = (uint32_t)nodes.size();
    *n_slots = (uint32_t)order.size();
    *depth = d;
    if (h_nodes) {
      if (cap_nodes < nodes.size()) return GI_ERR_INVALID_ARG;
      std::memcpy(h_nodes, nodes.data(), sizeof(Node4) * nodes.size());
    }
    if (h_slots) {
      if (cap_slots < order.size()) return GI_ERR_INVALID_ARG;
      std::memcpy(h_slots, order.data(), sizeof(uint32_t) * order.size());
    }
    return GI_OK;
  } catch (const std::bad_alloc&) {
    return GI_ERR_OOM;
  } catch (...) {
    return GI_ERR_INTERNAL;
  }
}

gi_status gi_set_dynamic_triangles(gi_context* c, const float* h_tv, const uint32_t* h_mat, uint32_t n, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (!c->has_scene) return fail(c, GI_ERR_STATE, "gi_build_bvh first");
  if (n > (uint32_t)gi::kMaxDyn || (n && (!h_tv || !h_mat))) return fail(c, GI_ERR_INVALID_ARG, "at most 64 dynamic triangles");
  try {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (uint32_t k = 0; k < n; ++k)
      if (h_mat[k] >= c->n_mats) return fail(c, GI_ERR_INVALID_ARG, "material index out of range");
    std::vector<float4> tv(3 * (size_t)std::max(n, 1u));
    std::vector<float4> tn(std::max(n, 1u));
    for (uint32_t k = 0; k < n; ++k) {
      const float* v = h_tv + 9 * (size_t)k;
      uint32_t id = c->nt + k;
      float w;
      std::memcpy(&w, &id, 4);
      tv[3 * k] = make_float4(v[0], v[1], v[2], w);
      tv[3 * k + 1] = make_float4(v[3], v[4], v[5], 0.0f);
      tv[3 * k + 2] = make_float4(v[6], v[7], v[8], 0.0f);
      float nn[3];
      unit_normal(v, nn);
      uint32_t mb = h_mat[k];
      std::memcpy(&w, &mb, 4);
      tn[k] = make_float4(nn[0], nn[1], nn[2], w);
    }
    if (n) {
      int slot;
      char* st = stage_acquire(c, sizeof(float4) * 4 * n, &slot);
      if (!st) return fail(c, GI_ERR_OOM, "pinned staging allocation failed");
      std::memcpy(st, tv.data(), sizeof(float4) * 3 * n);
      std::memcpy(st + sizeof(float4) * 3 * n, tn.data(), sizeof(float4) * n);
      GI_TRY_HIP(c, hipMemcpyAsync(c->d_dyn, st, sizeof(float4) * 3 * n, hipMemcpyHostToDevice, s));
      GI_TRY_HIP(c, hipMemcpyAsync(c->d_tnrm + c->nt, st + sizeof(float4) * 3 * n, sizeof(float4) * n,
                                   hipMemcpyHostToDevice, s));
      stage_release(c, slot, s);
    }
    const gi_status st = upload_emitters(c, h_tv, h_mat, n, s);
    if (st != GI_OK) return st;
    c->n_dyn = n;
    return GI_OK;
  } catch (const std::exception& ex) {
    return fail(c, GI_ERR_INTERNAL, ex.what());
  }
}

gi_status gi_render_gbuffer(gi_context* c, const gi_frame* f, float* pos, float* nrm, float* alb, uint32_t* prim,
                            void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (!f || !pos || !nrm || !alb || !prim) return fail(c, GI_ERR_INVALID_ARG, "null argument");
  if (!aligned16(pos) || !aligned16(nrm) || !aligned16(alb)) return fail(c, GI_ERR_INVALID_ARG, "G-buffer not 16-byte aligned");
  if (!c->has_scene) return fail(c, GI_ERR_STATE, "gi_build_bvh first");
  GI_TRY_HIP(c, gi::launch_gbuffer(c, f, reinterpret_cast<float4*>(pos), reinterpret_cast<float4*>(nrm),
                                   reinterpret_cast<float4*>(alb), prim, reinterpret_cast<hipStream_t>(stream)));
  return GI_OK;
}

gi_status gi_spawn_probes(gi_context* c, const gi_frame* f, const float* pos, const float* nrm, const uint32_t* prim,
                          void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (!f || !pos || !nrm || !prim) return fail(c, GI_ERR_INVALID_ARG, "null argument");
  if (!aligned16(pos) || !aligned16(nrm)) return fail(c, GI_ERR_INVALID_ARG, "G-buffer not 16-byte aligned");
  if (!c->has_scene) return fail(c, GI_ERR_STATE, "gi_build_bvh first");
  c->fa.index = f->index;
  const uint32_t u = c->cfg.upscale > 1 ? c->cfg.upscale : 1u;
  c->fa.sjx = halton_cell(f->index + 1u, 2u, 8u * u);
  c->fa.sjy = halton_cell(f->index + 1u, 3u, 8u * u);
  c->fa.jx = c->fa.sjx % 8u;
  c->fa.jy = c->fa.sjy % 8u;
  for (int k = 0; k < 3; ++k) c->fa.cam[k] = f->pos[k];
  {
    // Algorithm 6: distance scale on the host in float64, rounded once
    const double a = 1.0 / (double)c->H, b = (double)c->H / ((double)c->W * (double)c->W);
    c->fa.kappa = (float)std::tan((double)f->fov_y * 8.0 * std::max(a, b));
  }
  GI_TRY_HIP(c, gi::launch_spawn(c, reinterpret_cast<const float4*>(pos), reinterpret_cast<const float4*>(nrm), prim,
                                 reinterpret_cast<hipStream_t>(stream)));
  c->stage = 1;
  return GI_OK;
}

gi_status gi_trace_probes(gi_context* c, const gi_frame* f, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (c->cfg.light_grid && c->n_emit > 2048) return fail(c, GI_ERR_UNSUPPORTED, "light grid: more than 2048 emitter triangles");
  if (!f) return fail(c, GI_ERR_INVALID_ARG, "null frame");
  if (c->stage != 1 || f->index != c->fa.index) return fail(c, GI_ERR_STATE, "gi_spawn_probes of this frame first");
  GI_TRY_HIP(c, gi::launch_trace(c, reinterpret_cast<hipStream_t>(stream)));
  c->stage = 2;
  return GI_OK;
}

gi_status gi_learned_train(gi_context* c, const gi_frame* f, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (!f) return fail(c, GI_ERR_INVALID_ARG, "null frame");
  if (c->cfg.cache_mode == GI_CACHE_PLAIN || !c->learned) return fail(c, GI_ERR_STATE, "learned cache disabled");
  if (c->stage != 2) return fail(c, GI_ERR_STATE, "gi_trace_probes of this frame first");
  GI_TRY_HIP(c, gi::learned_train(c, reinterpret_cast<hipStream_t>(stream)));
  return GI_OK;
}

gi_status gi_cache_update(gi_context* c, const gi_frame* f, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (!f) return fail(c, GI_ERR_INVALID_ARG, "null frame");
  if (c->stage != 2) return fail(c, GI_ERR_STATE, "gi_trace_probes of this frame first");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  GI_TRY_HIP(c, gi::launch_update(c, s));
  if (c->cfg.temporal) {
    // this frame's final probes become the history of the next one
    GI_TRY_HIP(c, hipMemcpyAsync(c->d_prev_mask, c->d_mask, 4 * (size_t)c->P, hipMemcpyDeviceToDevice, s));
    GI_TRY_HIP(c, hipMemcpyAsync(c->d_prev_pos, c->d_ppos, 16 * (size_t)c->P, hipMemcpyDeviceToDevice, s));
    GI_TRY_HIP(c, hipMemcpyAsync(c->d_prev_nrm, c->d_pnrm, 16 * (size_t)c->P, hipMemcpyDeviceToDevice, s));
    GI_TRY_HIP(c, hipMemcpyAsync(c->d_prev_atlas, c->d_atlas, 16 * 64 * (size_t)c->P, hipMemcpyDeviceToDevice, s));
    if (c->d_prev_sh)
      GI_TRY_HIP(c, hipMemcpyAsync(c->d_prev_sh, c->d_sh, 4 * 28 * (size_t)c->P, hipMemcpyDeviceToDevice, s));
    c->prev_frame = *f;
    c->has_prev = true;
  }
  c->stage = 3;
  return GI_OK;
}

gi_status gi_interpolate_probes(gi_context* c, const gi_frame* f, const float* pos, const float* nrm,
                                const uint32_t* prim, float* out, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (!f || !pos || !nrm || !prim || !out) return fail(c, GI_ERR_INVALID_ARG, "null argument");
  if (!aligned16(pos) || !aligned16(nrm) || !aligned16(out)) return fail(c, GI_ERR_INVALID_ARG, "not 16-byte aligned");
  if (c->stage != 3) return fail(c, GI_ERR_STATE, "gi_cache_update of this frame first");
  GI_TRY_HIP(c, gi::launch_interpolate(c, reinterpret_cast<const float4*>(pos), reinterpret_cast<const float4*>(nrm),
                                       prim, reinterpret_cast<float4*>(out), reinterpret_cast<hipStream_t>(stream)));
  return GI_OK;
}

gi_status gi_cache_query(gi_context* c, const float* pos, const float* nrm, uint32_t n, float* out, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (n && (!pos || !nrm || !out)) return fail(c, GI_ERR_INVALID_ARG, "null argument");
  if (n && (!aligned16(pos) || !aligned16(nrm) || !aligned16(out))) return fail(c, GI_ERR_INVALID_ARG, "not 16-byte aligned");
  GI_TRY_HIP(c, gi::launch_query(c, reinterpret_cast<const float4*>(pos), reinterpret_cast<const float4*>(nrm), n,
                                 reinterpret_cast<float4*>(out), reinterpret_cast<hipStream_t>(stream)));
  return GI_OK;
}

gi_status gi_e4m3_encode(gi_context* c, const float* in, uint8_t* out, uint32_t n, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (n && (!in || !out)) return fail(c, GI_ERR_INVALID_ARG, "null argument");
  GI_TRY_HIP(c, gi::e4m3_encode_array(in, out, n, reinterpret_cast<hipStream_t>(stream)));
  return GI_OK;
}

gi_status gi_trace_rays(gi_context* c, const float* o, const float* d, uint32_t n, uint32_t any_hit, uint32_t* tri,
                        float* t, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (n && (!o || !d || !tri || !t)) return fail(c, GI_ERR_INVALID_ARG, "null argument");
  if (n && (!aligned16(o) || !aligned16(d))) return fail(c, GI_ERR_INVALID_ARG, "not 16-byte aligned");
  if (!c->has_scene) return fail(c, GI_ERR_STATE, "gi_build_bvh first");
  GI_TRY_HIP(c, gi::launch_trace_rays(c, reinterpret_cast<const float4*>(o), reinterpret_cast<const float4*>(d), n,
                                      any_hit, tri, t, reinterpret_cast<hipStream_t>(stream)));
  return GI_OK;
}

gi_status gi_trace_rays_noalloc(gi_context* c, const float* o, const float* d, uint32_t n, uint32_t any_hit,
                                uint32_t* tri, float* t, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (n && (!o || !d || !tri || !t)) return fail(c, GI_ERR_INVALID_ARG, "null argument");
  if (n && (!aligned16(o) || !aligned16(d))) return fail(c, GI_ERR_INVALID_ARG, "not 16-byte aligned");
  if (!c->has_scene) return fail(c, GI_ERR_STATE, "gi_build_bvh first");
  if (gi::noalloc_chunk_rays(c->spill_rows) == 0)
    return fail(c, GI_ERR_UNSUPPORTED, "BVH too deep: its traversal-stack spill rows do not fit the 16 MiB static scratch");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != c->device)
    return fail(c, GI_ERR_INVALID_ARG, "the context's device is not the current device");
  GI_TRY_HIP(c, gi::launch_trace_rays_noalloc(c, reinterpret_cast<const float4*>(o), reinterpret_cast<const float4*>(d),
                                              n, any_hit, tri, t, reinterpret_cast<hipStream_t>(stream)));
  return GI_OK;
}

gi_status gi_measure_traversal(gi_context* c, uint64_t* out8, void* stream) {
  if (!c || !out8) return GI_ERR_INVALID_ARG;
  if (c->stage < 2) return fail(c, GI_ERR_STATE, "gi_trace_probes first");
  unsigned long long* d = nullptr;
  GI_TRY_HIP(c, dalloc(&d, 8));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = gi::launch_count_traversal(c, d, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(out8, d, 64, hipMemcpyDeviceToHost);
  dfree(d);
  GI_TRY_HIP(c, e);
  return GI_OK;
}

gi_status gi_learned_step(gi_context* c, const float* pos, const float* nrm, const float* tgt, uint32_t n,
                          uint32_t apply, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (c->cfg.cache_mode == GI_CACHE_PLAIN || !c->learned) return fail(c, GI_ERR_STATE, "learned cache disabled");
  if (!pos || !nrm || !tgt) return fail(c, GI_ERR_INVALID_ARG, "null argument");
  if (!aligned16(pos) || !aligned16(nrm) || !aligned16(tgt)) return fail(c, GI_ERR_INVALID_ARG, "not 16-byte aligned");
  if (!c->has_scene) return fail(c, GI_ERR_STATE, "gi_build_bvh first (it fixes the encoding domain)");
  const hipError_t e = gi::learned_step_on(c, reinterpret_cast<const float4*>(pos), reinterpret_cast<const float4*>(nrm),
                                           reinterpret_cast<const float4*>(tgt), n, apply != 0,
                                           reinterpret_cast<hipStream_t>(stream));
  if (e == hipErrorInvalidValue) return fail(c, GI_ERR_INVALID_ARG, "n must equal 2^mlp_batch_log2");
  GI_TRY_HIP(c, e);
  return GI_OK;
}

gi_status gi_learned_query(gi_context* c, const float* pos, const float* nrm, uint32_t n, float* out, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  if (c->cfg.cache_mode == GI_CACHE_PLAIN || !c->learned) return fail(c, GI_ERR_STATE, "learned cache disabled");
  if (n && (!pos || !nrm || !out)) return fail(c, GI_ERR_INVALID_ARG, "null argument");
  if (n && (!aligned16(pos) || !aligned16(nrm) || !aligned16(out))) return fail(c, GI_ERR_INVALID_ARG, "not 16-byte aligned");
  GI_TRY_HIP(c, gi::learned_query(c, reinterpret_cast<const float4*>(pos), reinterpret_cast<const float4*>(nrm), n,
                                  reinterpret_cast<float4*>(out), reinterpret_cast<hipStream_t>(stream)));
  return GI_OK;
}

// ---- exports ------------------------------------------------------------------------------

gi_status gi_restir_export(gi_context* c, uint64_t* h_id, uint64_t* h_key, float* h_yw, float* h_n, uint32_t* h_k,
                           uint32_t* h_m, uint32_t cap, uint32_t* n_out) {
  if (!c || !n_out) return GI_ERR_INVALID_ARG;
  if (!c->cfg.restir) return fail(c, GI_ERR_UNSUPPORTED, "gi_restir_export needs restir = 1");
  try {
    GI_TRY_HIP(c, hipDeviceSynchronize());
    const size_t N = (size_t)1 << c->cfg.restir_log2;
    const uint32_t t = c->rs_cur;   // the table the last trace wrote
    std::vector<uint32_t> fp(N), m(N);
    std::vector<uint64_t> key(N);
    std::vector<float4> yw(N), nr(N);
    GI_TRY_HIP(c, hipMemcpy(fp.data(), c->d_rs_fp[t], 4 * N, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(key.data(), c->d_rs_key[t], 8 * N, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(yw.data(), c->d_rs_yw[t], 16 * N, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(nr.data(), c->d_rs_n[t], 16 * N, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(m.data(), c->d_rs_m[t], 4 * N, hipMemcpyDeviceToHost));
    uint32_t n = 0;
    // live slots in ascending key order (slot positions are not part of the result)
    std::vector<uint32_t> live;
    for (size_t s = 0; s < N; ++s)
      if (fp[s] && c->rs_has_prev) live.push_back((uint32_t)s);
    std::sort(live.begin(), live.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b] || (key[a] == key[b] && a < b); });
    for (const uint32_t s : live) {
      if (n < cap) {
        if (h_id) h_id[n] = ((uint64_t)(s / gi::kBucketSlots) << 32) | fp[s];
        if (h_key) h_key[n] = key[s];
        if (h_yw) {
          h_yw[4 * (size_t)n] = yw[s].x;
          h_yw[4 * (size_t)n + 1] = yw[s].y;
          h_yw[4 * (size_t)n + 2] = yw[s].z;
          h_yw[4 * (size_t)n + 3] = yw[s].w;
        }
        if (h_n) {
          h_n[3 * (size_t)n] = nr[s].x;
          h_n[3 * (size_t)n + 1] = nr[s].y;
          h_n[3 * (size_t)n + 2] = nr[s].z;
        }
        if (h_k) {
          uint32_t kb;
          std::memcpy(&kb, &nr[s].w, 4);
          h_k[n] = kb;
        }
        if (h_m) h_m[n] = m[s];
      }
      ++n;
    }
    *n_out = n;
    return GI_OK;
  } catch (const std::exception& ex) {
    return fail(c, GI_ERR_INTERNAL, ex.what());
  }
}

gi_status gi_light_grid_export(gi_context* c, float* h_geom, uint32_t* h_dims, uint32_t* h_list, uint32_t* h_count,
                               uint32_t cap_cells) {
  if (!c || !h_geom || !h_dims) return GI_ERR_INVALID_ARG;
  if (!c->cfg.light_grid) return fail(c, GI_ERR_UNSUPPORTED, "gi_light_grid_export needs light_grid = 1");
  try {
    GI_TRY_HIP(c, hipDeviceSynchronize());
    uint32_t box[6];
    GI_TRY_HIP(c, hipMemcpy(box, c->d_lg_box, sizeof(box), hipMemcpyDeviceToHost));
    gi::LightGridGeom g = gi::light_grid_geom(box, c->cfg.lgrid_dim);
    for (int k = 0; k < 3; ++k) {
      h_geom[k] = g.lo[k];
      h_dims[k] = g.dim[k];
    }
    h_geom[3] = g.h;
    const size_t n = std::min<size_t>((size_t)g.dim[0] * g.dim[1] * g.dim[2], cap_cells);
    if (h_list) GI_TRY_HIP(c, hipMemcpy(h_list, c->d_lg_list, 4 * n * c->cfg.lgrid_k, hipMemcpyDeviceToHost));
    if (h_count) GI_TRY_HIP(c, hipMemcpy(h_count, c->d_lg_count, 4 * n, hipMemcpyDeviceToHost));
    return GI_OK;
  } catch (const std::exception& ex) {
    return fail(c, GI_ERR_INTERNAL, ex.what());
  }
}

gi_status gi_tiles_export(gi_context* c, uint64_t* h_id, uint64_t* h_key, uint32_t* h_life, uint32_t* h_acc,
                          float* h_L, uint32_t* h_nhist, float* h_Lq, uint32_t cap, uint32_t* n_out) {
  if (!c || !n_out) return GI_ERR_INVALID_ARG;
  if (!c->cfg.cache_tiles) return fail(c, GI_ERR_UNSUPPORTED, "gi_tiles_export needs cache_tiles = 1");
  try {
    GI_TRY_HIP(c, hipDeviceSynchronize());
    const size_t N = c->N, NC = N * 64;
    std::vector<uint32_t> fp(N), cn(NC);
    std::vector<uint64_t> key(N);
    std::vector<uint2> meta(N);
    std::vector<uint4> acc(NC);
    std::vector<float4> L(NC), Lq(NC);
    GI_TRY_HIP(c, hipMemcpy(fp.data(), c->tab.fp, 4 * N, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(key.data(), c->tab.key, 8 * N, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(meta.data(), c->tab.meta, 8 * N, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(acc.data(), c->tab.acc, 16 * NC, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(L.data(), c->tab.L, 16 * NC, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(cn.data(), c->tab.cn, 4 * NC, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(Lq.data(), c->tab.Lq, 16 * NC, hipMemcpyDeviceToHost));
    // live cells in ascending key order (slot positions are not part of the result)
    std::vector<uint32_t> live;
    for (size_t s = 0; s < N; ++s)
      if (fp[s]) live.push_back((uint32_t)s);
    std::sort(live.begin(), live.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b] || (key[a] == key[b] && a < b); });
    uint32_t n = 0;
    for (const uint32_t s : live) {
      if (n < cap) {
        if (h_id) h_id[n] = ((uint64_t)(s / gi::kBucketSlots) << 32) | fp[s];
        if (h_key) h_key[n] = key[s];
        if (h_life) h_life[n] = meta[s].y;
        for (size_t i = 0; i < 64; ++i) {
          const size_t e = i * N + s, o = (size_t)n * 64 + i;   // cell-major on the device
          if (h_acc) {
            h_acc[4 * o] = acc[e].x;
            h_acc[4 * o + 1] = acc[e].y;
            h_acc[4 * o + 2] = acc[e].z;
            h_acc[4 * o + 3] = acc[e].w;
          }
          if (h_L) {
            h_L[3 * o] = L[e].x;
            h_L[3 * o + 1] = L[e].y;
            h_L[3 * o + 2] = L[e].z;
          }
          if (h_nhist) h_nhist[o] = cn[e];
          if (h_Lq) {
            h_Lq[3 * o] = Lq[e].x;
            h_Lq[3 * o + 1] = Lq[e].y;
            h_Lq[3 * o + 2] = Lq[e].z;
          }
        }
      }
      ++n;
    }
    *n_out = n;
    return GI_OK;
  } catch (const std::exception& ex) {
    return fail(c, GI_ERR_INTERNAL, ex.what());
  }
}

gi_status gi_cache_export(gi_context* c, uint64_t* h_id, uint64_t* h_key, uint32_t* h_acc, float* h_L,
                          uint32_t* h_nhist, uint32_t* h_life, uint32_t cap, uint32_t* n_out) {
  if (!c || !n_out) return GI_ERR_INVALID_ARG;
  if (c->cfg.cache_tiles) return fail(c, GI_ERR_UNSUPPORTED, "two-level cache: use gi_tiles_export");
  try {
    GI_TRY_HIP(c, hipDeviceSynchronize());
    const size_t N = c->N;
    std::vector<uint32_t> fp(N);
    std::vector<uint64_t> key(N);
    std::vector<uint4> acc(N);
    std::vector<float4> L(N);
    std::vector<uint2> meta(N);
    GI_TRY_HIP(c, hipMemcpy(fp.data(), c->tab.fp, 4 * N, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(key.data(), c->tab.key, 8 * N, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(acc.data(), c->tab.acc, 16 * N, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(L.data(), c->tab.L, 16 * N, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(meta.data(), c->tab.meta, 8 * N, hipMemcpyDeviceToHost));
    // live cells in ascending key order (slot positions are not part of the result)
    std::vector<uint32_t> live;
    for (size_t s = 0; s < N; ++s)
      if (fp[s]) live.push_back((uint32_t)s);
    std::sort(live.begin(), live.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b] || (key[a] == key[b] && a < b); });
    uint32_t n = 0;
    for (const uint32_t s : live) {
      if (n < cap) {
        if (h_id) h_id[n] = ((uint64_t)(s / gi::kBucketSlots) << 32) | fp[s];
        if (h_key) h_key[n] = key[s];
        if (h_acc) {
          h_acc[4 * (size_t)n] = acc[s].x;
          h_acc[4 * (size_t)n + 1] = acc[s].y;
          h_acc[4 * (size_t)n + 2] = acc[s].z;
          h_acc[4 * (size_t)n + 3] = acc[s].w;
        }
        if (h_L) {
          h_L[3 * (size_t)n] = L[s].x;
          h_L[3 * (size_t)n + 1] = L[s].y;
          h_L[3 * (size_t)n + 2] = L[s].z;
        }
        if (h_nhist) h_nhist[n] = meta[s].x;
        if (h_life) h_life[n] = meta[s].y;
      }
      ++n;
    }
    *n_out = n;
    return GI_OK;
  } catch (const std::exception& ex) {
    return fail(c, GI_ERR_INTERNAL, ex.what());
  }
}

gi_status gi_cache_save(gi_context* c, void* blob, size_t cap, size_t* size_out) {
  if (!c || !size_out) return GI_ERR_INVALID_ARG;
  if (c->cfg.cache_tiles) return fail(c, GI_ERR_UNSUPPORTED, "two-level cache: use gi_tiles_export");
  const size_t N = c->N;
  const size_t bytes = 16 + N * (4 + 8 + 16 + 16 + 8 + 4);
  *size_out = bytes;
  if (!blob) return GI_OK;
  if (cap < bytes) return fail(c, GI_ERR_INVALID_ARG, "blob too small");
  GI_TRY_HIP(c, hipDeviceSynchronize());
  char* p = static_cast<char*>(blob);
  const uint32_t hdr[4] = {0x47494331u, c->cfg.table_log2, 0u, 0u};
  std::memcpy(p, hdr, 16);
  p += 16;
  GI_TRY_HIP(c, hipMemcpy(p, c->tab.fp, 4 * N, hipMemcpyDeviceToHost)); p += 4 * N;
  GI_TRY_HIP(c, hipMemcpy(p, c->tab.key, 8 * N, hipMemcpyDeviceToHost)); p += 8 * N;
  GI_TRY_HIP(c, hipMemcpy(p, c->tab.acc, 16 * N, hipMemcpyDeviceToHost)); p += 16 * N;
  GI_TRY_HIP(c, hipMemcpy(p, c->tab.L, 16 * N, hipMemcpyDeviceToHost)); p += 16 * N;
  GI_TRY_HIP(c, hipMemcpy(p, c->tab.meta, 8 * N, hipMemcpyDeviceToHost)); p += 8 * N;
  GI_TRY_HIP(c, hipMemcpy(p, c->tab.accessed, 4 * N, hipMemcpyDeviceToHost));
  return GI_OK;
}

gi_status gi_cache_load(gi_context* c, const void* blob, size_t size) {
  if (!c || !blob) return GI_ERR_INVALID_ARG;
  if (c->cfg.cache_tiles) return fail(c, GI_ERR_UNSUPPORTED, "two-level cache: use gi_tiles_export");
  const size_t N = c->N;
  const size_t bytes = 16 + N * (4 + 8 + 16 + 16 + 8 + 4);
  if (size != bytes) return fail(c, GI_ERR_INVALID_ARG, "blob size does not match this config");
  const char* p = static_cast<const char*>(blob);
  uint32_t hdr[4];
  std::memcpy(hdr, p, 16);
  if (hdr[0] != 0x47494331u || hdr[1] != c->cfg.table_log2) return fail(c, GI_ERR_INVALID_ARG, "not a cache blob of this config");
  p += 16;
  GI_TRY_HIP(c, hipDeviceSynchronize());
  GI_TRY_HIP(c, hipMemcpy(c->tab.fp, p, 4 * N, hipMemcpyHostToDevice)); p += 4 * N;
  GI_TRY_HIP(c, hipMemcpy(c->tab.key, p, 8 * N, hipMemcpyHostToDevice)); p += 8 * N;
  GI_TRY_HIP(c, hipMemcpy(c->tab.acc, p, 16 * N, hipMemcpyHostToDevice)); p += 16 * N;
  GI_TRY_HIP(c, hipMemcpy(c->tab.L, p, 16 * N, hipMemcpyHostToDevice)); p += 16 * N;
  GI_TRY_HIP(c, hipMemcpy(c->tab.meta, p, 8 * N, hipMemcpyHostToDevice)); p += 8 * N;
  GI_TRY_HIP(c, hipMemcpy(c->tab.accessed, p, 4 * N, hipMemcpyHostToDevice));
  return GI_OK;
}

gi_status gi_rays_export(gi_context* c, int32_t* h_slot, float* h_t, uint32_t* h_tri, uint32_t* h_flags, uint64_t* h_key) {
  if (!c) return GI_ERR_INVALID_ARG;
  try {
    GI_TRY_HIP(c, hipDeviceSynchronize());
    const size_t PR = (size_t)c->P * c->R;
    std::vector<uint4> rec(PR);
    std::vector<uint2> key(PR);
    GI_TRY_HIP(c, hipMemcpy(rec.data(), c->d_rec, 16 * PR, hipMemcpyDeviceToHost));
    GI_TRY_HIP(c, hipMemcpy(key.data(), c->d_rkey, 8 * PR, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < PR; ++i) {
      if (h_slot) h_slot[i] = (int32_t)rec[i].x;
      if (h_t) std::memcpy(&h_t[i], &rec[i].y, 4);
      if (h_tri) h_tri[i] = rec[i].z;
      if (h_flags) h_flags[i] = rec[i].w;
      if (h_key) h_key[i] = (uint64_t)key[i].x | ((uint64_t)key[i].y << 32);
    }
    return GI_OK;
  } catch (const std::exception& ex) {
    return fail(c, GI_ERR_INTERNAL, ex.what());
  }
}

gi_status gi_probes_export(gi_context* c, uint32_t* h_mask, float* h_pos, float* h_nrm, float* h_atlas, float* h_sh) {
  if (!c) return GI_ERR_INVALID_ARG;
  try {
    GI_TRY_HIP(c, hipDeviceSynchronize());
    if (h_mask) GI_TRY_HIP(c, hipMemcpy(h_mask, c->d_mask, 4 * (size_t)c->mask_total, hipMemcpyDeviceToHost));
    if (h_pos) GI_TRY_HIP(c, hipMemcpy(h_pos, c->d_ppos, 16 * (size_t)c->P, hipMemcpyDeviceToHost));
    if (h_nrm) GI_TRY_HIP(c, hipMemcpy(h_nrm, c->d_pnrm, 16 * (size_t)c->P, hipMemcpyDeviceToHost));
    if (h_atlas) GI_TRY_HIP(c, hipMemcpy(h_atlas, c->d_atlas, 16 * 64 * (size_t)c->P, hipMemcpyDeviceToHost));
    if (h_sh) {
      std::vector<float> sh((size_t)c->P * 28);
      GI_TRY_HIP(c, hipMemcpy(sh.data(), c->d_sh, 4 * sh.size(), hipMemcpyDeviceToHost));
      for (size_t p = 0; p < c->P; ++p)
        for (int k = 0; k < 27; ++k) h_sh[27 * p + k] = sh[28 * p + k];
    }
    return GI_OK;
  } catch (const std::exception& ex) {
    return fail(c, GI_ERR_INTERNAL, ex.what());
  }
}

gi_status gi_get_dims(gi_context* c, uint32_t* out) {
  if (!c || !out) return GI_ERR_INVALID_ARG;
  const uint32_t v[16] = {c->P, c->R, c->N, c->TW, c->TH, c->nmip, c->mask_total, c->fa.jx, c->fa.jy,
                          c->n_nodes, c->bvh_depth, c->stack_depth, c->n_emit, c->nt, c->n_dyn, 0};
  std::memcpy(out, v, sizeof(v));
  return GI_OK;
}

gi_status gi_get_stats(gi_context* c, uint64_t* out) {
  if (!c || !out) return GI_ERR_INVALID_ARG;
  GI_TRY_HIP(c, hipDeviceSynchronize());
  std::vector<uint64_t> st((size_t)GI_STAT_COUNT * gi::kStatStripesHost);
  GI_TRY_HIP(c, hipMemcpy(st.data(), c->d_stats, 8 * st.size(), hipMemcpyDeviceToHost));
  for (int k = 0; k < GI_STAT_COUNT; ++k) {
    uint64_t v = 0;
    for (uint32_t s = 0; s < gi::kStatStripesHost; ++s) v += st[(size_t)s * GI_STAT_COUNT + k];
    out[k] = v;
  }
  return GI_OK;
}

gi_status gi_reset_stats(gi_context* c, void* stream) {
  if (!c) return GI_ERR_INVALID_ARG;
  GI_TRY_HIP(c, gi::launch_zero_stats(c, reinterpret_cast<hipStream_t>(stream)));
  return GI_OK;
}

gi_status gi_profile_enable(gi_context* c, uint32_t on) {
  if (!c || on > 2u) return GI_ERR_INVALID_ARG;
  c->prof = on;
  return GI_OK;
}

gi_status gi_profile_read(gi_context* c, char* names, size_t names_cap, uint32_t* counts, double* ms, uint32_t cap,
                          uint32_t* n_out) {
  if (!c || !n_out) return GI_ERR_INVALID_ARG;
  GI_TRY_HIP(c, hipDeviceSynchronize());
  for (auto& t : c->timers) {
    float e = 0.0f;
    GI_TRY_HIP(c, hipEventElapsedTime(&e, t.a, t.b));
    size_t k = 0;
    while (k < c->prof_names.size() && c->prof_names[k] != t.name) ++k;
    if (k == c->prof_names.size()) {
      c->prof_names.emplace_back(t.name);
      c->prof_counts.push_back(0);
      c->prof_ms.push_back(0.0);
    }
    c->prof_counts[k] += 1;
    c->prof_ms[k] += e;
    c->event_pool.push_back(t.a);
    c->event_pool.push_back(t.b);
  }
  c->timers.clear();
  const uint32_t n = (uint32_t)c->prof_names.size();
  *n_out = n;
  size_t pos = 0;
  for (uint32_t k = 0; k < n && k < cap; ++k) {
    if (counts) counts[k] = c->prof_counts[k];
    if (ms) ms[k] = c->prof_ms[k];
    if (names) {
      const std::string& s = c->prof_names[k];
      if (pos + s.size() + 1 <= names_cap) {
        std::memcpy(names + pos, s.c_str(), s.size() + 1);
        pos += s.size() + 1;
      }
    }
  }
  c->prof_names.clear();
  c->prof_counts.clear();
  c->prof_ms.clear();
  return GI_OK;
}

gi_status gi_learned_save(gi_context* c, void* blob, size_t cap, size_t* size_out) {
  if (!c || !size_out) return GI_ERR_INVALID_ARG;
  if (!c->learned) return fail(c, GI_ERR_STATE, "learned cache disabled");
  const size_t n = gi::learned_blob_size(c);
  *size_out = n;
  if (!blob) return GI_OK;
  if (cap < n) return fail(c, GI_ERR_INVALID_ARG, "blob too small");
  GI_TRY_HIP(c, gi::learned_save(c, blob));
  return GI_OK;
}

gi_status gi_learned_load(gi_context* c, const void* blob, size_t size) {
  if (!c || !blob) return GI_ERR_INVALID_ARG;
  if (!c->learned) return fail(c, GI_ERR_STATE, "learned cache disabled");
  if (size != gi::learned_blob_size(c)) return fail(c, GI_ERR_INVALID_ARG, "blob size does not match this config");
  GI_TRY_HIP(c, gi::learned_load(c, blob));
  return GI_OK;
}

gi_status gi_learned_batch_export(gi_context* c, float* h_raw, float* h_grouped, uint32_t cap_rows, uint32_t* rows_out,
                                  uint32_t* n_train_out) {
  if (!c || !rows_out || !n_train_out) return GI_ERR_INVALID_ARG;
  if (!c->learned) return fail(c, GI_ERR_STATE, "learned cache disabled");
  GI_TRY_HIP(c, hipDeviceSynchronize());
  uint32_t rows = 0, n = 0;
  GI_TRY_HIP(c, gi::learned_batch_export(c, h_raw, h_grouped, cap_rows, rows, n));
  *rows_out = rows;
  *n_train_out = n;
  if ((h_raw || h_grouped) && cap_rows < rows) return fail(c, GI_ERR_INVALID_ARG, "cap_rows below the batch rows");
  return GI_OK;
}

gi_status gi_cache_import(gi_context* c, const void* h_blob, size_t size) { return gi_cache_load(c, h_blob, size); }

gi_status gi_learned_export(gi_context* c, void* h_blob, size_t cap, size_t* size_out) {
  return gi_learned_save(c, h_blob, cap, size_out);
}

gi_status gi_learned_import(gi_context* c, const void* h_blob, size_t size) { return gi_learned_load(c, h_blob, size); }

gi_status gi_learned_stats(gi_context* c, float* out8) {
  if (!c || !out8) return GI_ERR_INVALID_ARG;
  if (!c->learned) return fail(c, GI_ERR_STATE, "learned cache disabled");
  GI_TRY_HIP(c, hipDeviceSynchronize());
  gi::learned_stats(c, out8);
  return GI_OK;
}

}  // extern "C"
