// Screen-space denoiser (Section 2.4.3) for gfx950: temporal accumulation of the interpolated
// irradiance over the reprojected history, then a spatial filter whose radius shrinks as the
// history grows (wider where the history is short: the dilated blur mask), edge-aware by depth
// and normal.  A separate object from the GI context: it needs only the G-buffer, the
// irradiance and the camera.
//
// Per pixel (one thread each):
//   temporal  the world position projected with the previous camera lands on a previous pixel;
//             the history is valid if that pixel held one, was not sky, lies within the
//             pixel's cell size (Algorithm 6) of its tangent plane and its normal's cosine
//             exceeds 0.9.  Valid: n = min(n_prev + 1, hist_max), value = hist + (E - hist) / n;
//             else n = 1, value = E.  A pixel without a probe (flag 2) keeps its history as it
//             is, or stays empty (n = 0).
//   radius    floor(radius_max / n) (radius_max at n = 0), 0 on sky.
//   spatial   R = the largest radius of the 3x3 neighbourhood; the mean over the (2R+1)^2 window
//             of the neighbours holding a value, weights cs / (cs + |depth difference|) times
//             max(0, normal cosine)^8, summed in row order.
// The accumulated values (before the spatial filter) and this G-buffer become the history.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>

#include "gi.h"

namespace {

constexpr uint32_t kMiss = 0xFFFFFFFFu;

struct DnCamera {
  float pos[3], fwd[3], right[3], up[3];
  float tan_half;
};

struct DnArgs {
  const float4* pos;
  const float4* nrm;
  const uint32_t* prim;
  const float4* in;
  const float4* hist;    // previous accumulated values (rgb, n)
  const float4* ppos;    // previous G-buffer
  const float4* pnrm;
  const uint32_t* pprim;
  float4* acc;
  uint32_t* rad;
  uint32_t W, H, hist_max, radius_max, has_prev;
  float kappa;
  float cam[3];
  DnCamera prev;
};

__device__ inline bool project_prev_cam(const DnCamera& pc, uint32_t W, uint32_t H, float Xx, float Xy, float Xz,
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

__global__ __launch_bounds__(256) void k_dn_temporal(DnArgs d) {
  const uint32_t p = blockIdx.x * 256u + threadIdx.x;
  if (p >= d.W * d.H) return;
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
  uint32_t r = 0u;
  if (d.prim[p] != kMiss) {
    const float4 X = d.pos[p], n = d.nrm[p], E = d.in[p];
    bool hv = false;
    float4 Hh = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t qx, qy;
    if (d.has_prev && project_prev_cam(d.prev, d.W, d.H, X.x, X.y, X.z, qx, qy)) {
      const uint32_t q = qy * d.W + qx;
      Hh = d.hist[q];
      if (d.pprim[q] != kMiss && Hh.w > 0.0f) {
        const float4 Xq = d.ppos[q], nq = d.pnrm[q];
        const float ex = X.x - d.cam[0], ey = X.y - d.cam[1], ez = X.z - d.cam[2];
        const float cs = d.kappa * sqrtf((ex * ex + ey * ey) + ez * ez);
        const float pd = fabsf(((Xq.x - X.x) * n.x + (Xq.y - X.y) * n.y) + (Xq.z - X.z) * n.z);
        const float nc = (nq.x * n.x + nq.y * n.y) + nq.z * n.z;
        hv = pd < cs && nc > 0.9f;
      }
    }
    if (E.w == 2.0f) {
      if (hv) a = Hh;
    } else if (hv) {
      const float np = Hh.w + 1.0f;
      const float nn = np < (float)d.hist_max ? np : (float)d.hist_max;
      a = make_float4(Hh.x + (E.x - Hh.x) / nn, Hh.y + (E.y - Hh.y) / nn, Hh.z + (E.z - Hh.z) / nn, nn);
    } else {
      a = make_float4(E.x, E.y, E.z, 1.0f);
    }
    const uint32_t nh = (uint32_t)a.w;
    r = nh == 0u ? d.radius_max : d.radius_max / nh;
  }
  d.acc[p] = a;
  d.rad[p] = r;
}

__global__ __launch_bounds__(256) void k_dn_spatial(DnArgs d, float4* out) {
  const uint32_t p = blockIdx.x * 256u + threadIdx.x;
  if (p >= d.W * d.H) return;
  const float4 E = d.in[p];
  if (d.prim[p] == kMiss) {
    out[p] = make_float4(0.f, 0.f, 0.f, E.w);
    return;
  }
  const int32_t x = (int32_t)(p % d.W), y = (int32_t)(p / d.W);
  const int32_t W = (int32_t)d.W, H = (int32_t)d.H;
  uint32_t R = 0u;
  for (int32_t dy = -1; dy <= 1; ++dy)
    for (int32_t dx = -1; dx <= 1; ++dx) {
      const int32_t yy = y + dy, xx = x + dx;
      if (yy < 0 || xx < 0 || yy >= H || xx >= W) continue;
      const uint32_t r = d.rad[yy * W + xx];
      R = r > R ? r : R;
    }
  const float4 a = d.acc[p];
  if (R == 0u) {
    out[p] = make_float4(a.x, a.y, a.z, E.w);
    return;
  }
  const float4 X = d.pos[p], n = d.nrm[p];
  const float ex = X.x - d.cam[0], ey = X.y - d.cam[1], ez = X.z - d.cam[2];
  const float cs = d.kappa * sqrtf((ex * ex + ey * ey) + ez * ez);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, ws = 0.f;
  const int32_t r = (int32_t)R;
  for (int32_t dy = -r; dy <= r; ++dy)
    for (int32_t dx = -r; dx <= r; ++dx) {
      const int32_t yy = y + dy, xx = x + dx;
      if (yy < 0 || xx < 0 || yy >= H || xx >= W) continue;
      const uint32_t q = (uint32_t)(yy * W + xx);
      const float4 aq = d.acc[q];
      if (d.prim[q] == kMiss || aq.w == 0.0f) continue;
      const float4 nq = d.nrm[q];
      float nd = (n.x * nq.x + n.y * nq.y) + n.z * nq.z;
      nd = nd > 0.0f ? nd : 0.0f;
      const float n2 = nd * nd, n4 = n2 * n2, n8 = n4 * n4;
      const float w = (cs / (cs + fabsf(d.pos[q].w - X.w))) * n8;
      s0 = s0 + w * aq.x;
      s1 = s1 + w * aq.y;
      s2 = s2 + w * aq.z;
      ws = ws + w;
    }
  out[p] = ws > 0.0f ? make_float4(s0 / ws, s1 / ws, s2 / ws, E.w) : make_float4(a.x, a.y, a.z, E.w);
}

// this frame becomes the history: accumulated values, G-buffer
__global__ __launch_bounds__(256) void k_dn_keep(const float4* acc, const float4* pos, const float4* nrm,
                                                 const uint32_t* prim, float4* hist, float4* ppos, float4* pnrm,
                                                 uint32_t* pprim, uint32_t n) {
  const uint32_t p = blockIdx.x * 256u + threadIdx.x;
  if (p >= n) return;
  hist[p] = acc[p];
  ppos[p] = pos[p];
  pnrm[p] = nrm[p];
  pprim[p] = prim[p];
}

}  // namespace

struct gi_denoiser {
  uint32_t W = 0, H = 0, hist_max = 16, radius_max = 4;
  float4 *hist = nullptr, *acc = nullptr, *ppos = nullptr, *pnrm = nullptr;
  uint32_t *pprim = nullptr, *rad = nullptr;
  bool has_prev = false;
  gi_frame prev{};
};

namespace {

void dn_free(gi_denoiser* d) {
  for (void* p : {(void*)d->hist, (void*)d->acc, (void*)d->ppos, (void*)d->pnrm, (void*)d->pprim, (void*)d->rad})
    if (p) (void)hipFree(p);
  delete d;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

extern "C" {

gi_status gi_denoiser_create(uint32_t width, uint32_t height, uint32_t hist_max, uint32_t radius_max,
                             gi_denoiser** out) {
  if (!out) return GI_ERR_INVALID_ARG;
  *out = nullptr;
  if (width < 8 || height < 8 || width > 8192 || height > 8192 || hist_max < 1 || hist_max > 1024 ||
      radius_max > 16)
    return GI_ERR_INVALID_ARG;
  gi_denoiser* d = new (std::nothrow) gi_denoiser();
  if (!d) return GI_ERR_OOM;
  d->W = width;
  d->H = height;
  d->hist_max = hist_max;
  d->radius_max = radius_max;
  const size_t n = (size_t)width * height;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  A(hipMalloc(&d->hist, 16 * n));
  A(hipMalloc(&d->acc, 16 * n));
  A(hipMalloc(&d->ppos, 16 * n));
  A(hipMalloc(&d->pnrm, 16 * n));
  A(hipMalloc(&d->pprim, 4 * n));
  A(hipMalloc(&d->rad, 4 * n));
  if (e != hipSuccess) {
    dn_free(d);
    return e == hipErrorOutOfMemory ? GI_ERR_OOM : GI_ERR_HIP;
  }
  *out = d;
  return GI_OK;
}

void gi_denoiser_destroy(gi_denoiser* d) {
  if (d) dn_free(d);
}

gi_status gi_denoiser_reset(gi_denoiser* d) {
  if (!d) return GI_ERR_INVALID_ARG;
  d->has_prev = false;
  return GI_OK;
}

gi_status gi_denoise(gi_denoiser* d, const gi_frame* f, const float* pos, const float* nrm, const uint32_t* prim,
                     const float* irradiance, float* out, void* stream) {
  if (!d || !f || !pos || !nrm || !prim || !irradiance || !out) return GI_ERR_INVALID_ARG;
  if (!aligned16(pos) || !aligned16(nrm) || !aligned16(irradiance) || !aligned16(out)) return GI_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  DnArgs a;
  a.pos = reinterpret_cast<const float4*>(pos);
  a.nrm = reinterpret_cast<const float4*>(nrm);
  a.prim = prim;
  a.in = reinterpret_cast<const float4*>(irradiance);
  a.hist = d->hist;
  a.ppos = d->ppos;
  a.pnrm = d->pnrm;
  a.pprim = d->pprim;
  a.acc = d->acc;
  a.rad = d->rad;
  a.W = d->W;
  a.H = d->H;
  a.hist_max = d->hist_max;
  a.radius_max = d->radius_max;
  a.has_prev = d->has_prev ? 1u : 0u;
  {
    // Algorithm 6's distance scale on the host in float64, rounded once
    const double x = 1.0 / (double)d->H, y = (double)d->H / ((double)d->W * (double)d->W);
    a.kappa = (float)std::tan((double)f->fov_y * 8.0 * (x > y ? x : y));
  }
  for (int k = 0; k < 3; ++k) {
    a.cam[k] = f->pos[k];
    a.prev.pos[k] = d->prev.pos[k];
    a.prev.fwd[k] = d->prev.fwd[k];
    a.prev.right[k] = d->prev.right[k];
    a.prev.up[k] = d->prev.up[k];
  }
  a.prev.tan_half = d->prev.tan_half;
  const uint32_t n = d->W * d->H, blocks = (n + 255u) / 256u;
  k_dn_temporal<<<blocks, 256, 0, s>>>(a);
  k_dn_spatial<<<blocks, 256, 0, s>>>(a, reinterpret_cast<float4*>(out));
  k_dn_keep<<<blocks, 256, 0, s>>>(d->acc, a.pos, a.nrm, prim, d->hist, d->ppos, d->pnrm, d->pprim, n);
  if (hipGetLastError() != hipSuccess) return GI_ERR_HIP;
  d->prev = *f;
  d->has_prev = true;
  return GI_OK;
}

gi_status gi_denoiser_export(gi_denoiser* d, float* h_hist, uint32_t* h_radius) {
  if (!d) return GI_ERR_INVALID_ARG;
  if (hipDeviceSynchronize() != hipSuccess) return GI_ERR_HIP;
  const size_t n = (size_t)d->W * d->H;
  if (h_hist && hipMemcpy(h_hist, d->hist, 16 * n, hipMemcpyDeviceToHost) != hipSuccess) return GI_ERR_HIP;
  if (h_radius && hipMemcpy(h_radius, d->rad, 4 * n, hipMemcpyDeviceToHost) != hipSuccess) return GI_ERR_HIP;
  return GI_OK;
}

}  // extern "C"
