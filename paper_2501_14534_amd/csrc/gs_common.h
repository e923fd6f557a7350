// Device-side definitions shared by the libgs kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs_api.h"

namespace gs {

// Compositing constants of the rasterizer the paper builds on: alpha cap,
// skip threshold and the transmittance floor that stops a pixel.
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kLog2e = 1.44269504088896341f;

constexpr int kWave = 64;

// Per-view constants, passed by value in kernel arguments (graph-capture safe).
struct ViewArgs {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float campos[3];     // -R^T t
  float limx, limy;    // lateral ratio guard of the Jacobian
  int32_t W, H, TX, TY;
  int32_t tile_off;    // first global tile of the view
  int32_t pix_off;     // first pixel of the view in the concatenated planes
  float lowpass;       // s of Sigma' + sI for this view
};

struct ViewTable {
  ViewArgs v[GS_MAX_VIEWS];
  int32_t nviews;
  int32_t total_tiles;
};

__device__ __forceinline__ int view_of_tile(const ViewTable& vt, int gtile) {
  int v = 0;
#pragma unroll 1
  for (int i = 1; i < vt.nviews; ++i) v = (gtile >= vt.v[i].tile_off) ? i : v;
  return v;
}

// Tile rectangle of a record in single precision: x in
// [floor((u - r)/TW), floor((u + r)/TW)] clipped to [0, TX-1], likewise y.
// u - r and u + r are single IEEE operations; TW, TH are powers of two so the
// scaling by 1/TW is exact.  Returns false when the rectangle is empty.
__device__ __forceinline__ bool tile_rect(float u, float v, float r, float inv_tw, float inv_th, int TX, int TY,
                                          int* x0, int* y0, int* x1, int* y1) {
#pragma clang fp contract(off)
  float fx0 = floorf((u - r) * inv_tw);
  float fx1 = floorf((u + r) * inv_tw);
  float fy0 = floorf((v - r) * inv_th);
  float fy1 = floorf((v + r) * inv_th);
  fx0 = fmaxf(fx0, 0.0f);
  fy0 = fmaxf(fy0, 0.0f);
  fx1 = fminf(fx1, (float)(TX - 1));
  fy1 = fminf(fy1, (float)(TY - 1));
  if (!(fx1 >= fx0) || !(fy1 >= fy0)) return false;
  *x0 = (int)fx0;
  *x1 = (int)fx1;
  *y0 = (int)fy0;
  *y1 = (int)fy1;
  return true;
}

// exp(-q/2) = exp2(k q) with k = -log2(e)/2.  The walks stage each record
// with its conic scaled for that: (a, b, c) = (k A, 2 k B, k C), so the
// exponent is dx (a dx + b dy) + c dy dy.
constexpr float kQScale = -0.5f * kLog2e;
__device__ __forceinline__ float4 staged_a(float4 ra) {  // (u, v, a, b)
  return make_float4(ra.x, ra.y, kQScale * ra.z, (2.0f * kQScale) * ra.w);
}
__device__ __forceinline__ float4 staged_b(float4 rb) {  // (c, o', radius, depth)
  return make_float4(kQScale * rb.x, rb.y, rb.z, rb.w);
}

// One (pixel, splat) evaluation shared bit-for-bit by the forward and the
// backward walks (both stage the same scaled conic): square test, Gaussian
// falloff G and alpha = min(0.99, o' G).  Every operation is explicit (fused
// multiply-adds written out, no other contraction), so both kernels take
// identical skip/stop decisions.  Computed without branching; returns the
// square test's outcome.
struct Eval {
  float dx, dy, G, raw, alpha;
};

__device__ __forceinline__ bool eval_splat_all(float px, float py, float u, float v, float a, float b, float c,
                                               float o, float rad, Eval* e) {
#pragma clang fp contract(off)
  const float dx = px - u;
  const float dy = py - v;
  const float t = __builtin_fmaf(b, dy, a * dx);
  const float ex = __builtin_fmaf(dx, t, (c * dy) * dy);
  const float G = __builtin_amdgcn_exp2f(ex);
  const float raw = o * G;
  e->dx = dx;
  e->dy = dy;
  e->G = G;
  e->raw = raw;
  e->alpha = fminf(kAlphaMax, raw);
  return fabsf(dx) <= rad && fabsf(dy) <= rad;
}

// Sum over the 64 lanes of a wave, result valid in lane 63.  Row-local
// shifted adds (row_shr 1, 2, 4, 8) give each row's total in its lane 15;
// row_bcast:15 and row_bcast:31 then fold rows 0..3 into lane 63.
__device__ __forceinline__ float wave_sum_lane63(float v) {
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x111, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x112, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x114, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x118, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xa, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xc, 0xf, false));
  return v;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// The wave's earlier LDS writes are visible to all its lanes' later LDS
// accesses (and its earlier reads are done before later writes).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Real SH basis constants (closed forms: 1/2 sqrt(15/pi) etc.), single precision.
constexpr float kC1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
constexpr float kC2a = 1.09254843059207907f;  // 1/2 sqrt(15/pi)
constexpr float kC2b = 0.31539156525252005f;  // 1/4 sqrt(5/pi)
constexpr float kC2c = 0.54627421529603959f;  // 1/4 sqrt(15/pi)
constexpr float kC3a = 0.59004358992664352f;  // 1/4 sqrt(35/(2 pi))
constexpr float kC3b = 2.89061144264055405f;  // 1/2 sqrt(105/pi)
constexpr float kC3c = 0.45704579946446572f;  // 1/4 sqrt(21/(2 pi))
constexpr float kC3d = 0.37317633259011540f;  // 1/4 sqrt(7/pi)
constexpr float kC3e = 1.44530572132027737f;  // 1/4 sqrt(105/pi)

// Basis functions k = 1..15 (band 0 is the diffuse colour) at unit (x, y, z).
// Coefficients of SH degree 3 and the band of coefficient k (band l holds k in [l^2, (l+1)^2)).
constexpr int kShCoeffs = 16;
__host__ __device__ constexpr int sh_band(int k) { return k < 1 ? 0 : k < 4 ? 1 : k < 9 ? 2 : 3; }

__device__ __forceinline__ void sh_basis15(float x, float y, float z, float Y[15]) {
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = -kC1 * y;
  Y[1] = kC1 * z;
  Y[2] = -kC1 * x;
  Y[3] = kC2a * x * y;
  Y[4] = -kC2a * y * z;
  Y[5] = kC2b * (2.0f * zz - xx - yy);
  Y[6] = -kC2a * x * z;
  Y[7] = kC2c * (xx - yy);
  Y[8] = -kC3a * y * (3.0f * xx - yy);
  Y[9] = kC3b * x * y * z;
  Y[10] = -kC3c * y * (4.0f * zz - xx - yy);
  Y[11] = kC3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[12] = -kC3c * x * (4.0f * zz - xx - yy);
  Y[13] = kC3e * z * (xx - yy);
  Y[14] = -kC3a * x * (xx - 3.0f * yy);
}

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + __expf(-x)); }

__device__ __forceinline__ bool finitef(float x) { return __builtin_isfinite(x); }

}  // namespace gs
