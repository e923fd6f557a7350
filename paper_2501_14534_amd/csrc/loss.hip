// Photometric loss of Eq. 7 (the L1 and D-SSIM terms) and its gradient with
// respect to the rendered image, over all views of a call.
//
//   L_v = (1 - lambda) mean|x - y| + lambda (1 - mean S),   L = mean_v L_v
//
// S is the SSIM map of each colour plane from Gaussian-weighted local moments
// (11 x 11 window = outer product of two 11-tap Gaussians of standard deviation
// 1.5, as Sec. 3.2.5 describes; zero padding; C1 = 0.01^2, C2 = 0.03^2).
//
// Two passes over 32 x 32 output tiles, one workgroup per (view, plane, tile),
// each staging the tile plus a 5-pixel halo in LDS (42 x 42: 1.7 reads per
// pixel) and filtering it with two 1-D passes, 4 output pixels per thread:
//   ssim_fwd: the five moments mu_x, mu_y, E[xx], E[yy], E[xy]; S and its
//             partial derivatives dS/dmu_x, dS/dE[xx], dS/dE[xy] (written to
//             the workspace); per-workgroup sums of S and |x - y|;
//   ssim_bwd: the window's correlation of the three partial-derivative maps
//             (the window is symmetric, so this is the adjoint of the forward
//             filtering), combined per pixel as
//             dS/dx = w*A + 2 x (w*B) + y (w*C), then the L1 term.
// One workgroup per view adds its workgroups' sums in a fixed order (double)
// into the view's loss; a last kernel takes their mean.  No atomics:
// reproducible.
#include "gs_common.h"
#include "kernels.h"

namespace gs {

constexpr int kLT = kLossTile;       // output tile edge (32)
constexpr int kLR = 5;               // window radius
constexpr int kLS = kLT + 2 * kLR;   // staged edge (42)
constexpr int kLQ = kLT * kLT / 256; // output pixels per thread (4)
constexpr float kSsimC1 = 0.0001f;   // (0.01)^2
constexpr float kSsimC2 = 0.0009f;   // (0.03)^2

// Staged value at (row, col) of the tile's window: zero outside the image.
__device__ __forceinline__ float staged(const float* plane, int W, int H, int x0, int y0, int i) {
  const int r = i / kLS, c = i - r * kLS;
  const int x = x0 - kLR + c, y = y0 - kLR + r;
  return (x >= 0 && x < W && y >= 0 && y < H) ? plane[(int64_t)y * W + x] : 0.0f;
}

// Thread t owns column t % 32 of the tile, rows t / 32 + 8 k (k < 4).
__device__ __forceinline__ int out_col(int t) { return t & (kLT - 1); }
__device__ __forceinline__ int out_row(int t, int k) { return (t / kLT) + k * (256 / kLT); }

__global__ __launch_bounds__(256) void ssim_fwd_kernel(const float* __restrict__ image,
                                                       const float* __restrict__ target, LossViews lv,
                                                       float* __restrict__ dmap, float* __restrict__ bsum) {
  __shared__ float s_x[kLS * kLS], s_y[kLS * kLS];
  __shared__ float s_h[5][kLS * kLT];
  __shared__ float s_red[2][4];
  const LossTile tl = loss_tile(lv, blockIdx.x);
  const LossView& q = lv.v[tl.view];
  const int W = q.W, H = q.H, t = threadIdx.x;
  const int64_t plane_px = (int64_t)W * H;
  const int64_t poff = 3 * q.pix_off + tl.plane * plane_px;  // this plane in the view-concatenated layout
  const float* xp = image + poff;
  const float* yp = target + poff;
  const int x0 = tl.tx * kLT, y0 = tl.ty * kLT;
  for (int i = t; i < kLS * kLS; i += 256) {
    s_x[i] = staged(xp, W, H, x0, y0, i);
    s_y[i] = staged(yp, W, H, x0, y0, i);
  }
  __syncthreads();
  // horizontal pass: rows of the staged window, the tile's columns
  for (int i = t; i < kLS * kLT; i += 256) {
    const int r = i / kLT, c = i - r * kLT;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
      const float g = lv.g[k], x = s_x[r * kLS + c + k], y = s_y[r * kLS + c + k];
      a0 += g * x;
      a1 += g * y;
      a2 += g * (x * x);
      a3 += g * (y * y);
      a4 += g * (x * y);
    }
    s_h[0][i] = a0;
    s_h[1][i] = a1;
    s_h[2][i] = a2;
    s_h[3][i] = a3;
    s_h[4][i] = a4;
  }
  __syncthreads();
  // vertical pass: kLQ output pixels per thread
  const int ox = out_col(t);
  float s_val = 0.f, l1 = 0.f;
#pragma unroll
  for (int j = 0; j < kLQ; ++j) {
    const int oy = out_row(t, j);
    float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
      const float g = lv.g[k];
      const int i = (oy + k) * kLT + ox;
      mx += g * s_h[0][i];
      my += g * s_h[1][i];
      exx += g * s_h[2][i];
      eyy += g * s_h[3][i];
      exy += g * s_h[4][i];
    }
    const int px = x0 + ox, py = y0 + oy;
    if (px < W && py < H) {
      const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
      const float n1 = 2.f * mx * my + kSsimC1, n2 = 2.f * sxy + kSsimC2;
      const float d1 = mx * mx + my * my + kSsimC1, d2 = sxx + syy + kSsimC2;
      const float id = 1.0f / (d1 * d2);
      const float S = n1 * n2 * id;
      const float dmx = 2.f * my * (n2 - n1) * id - 2.f * mx * S * (1.0f / d1 - 1.0f / d2);
      const float dexx = -S / d2;
      const float dexy = 2.f * n1 * id;
      const int64_t pix = (int64_t)py * W + px;
      const int64_t o = 3 * (poff + pix);  // [pixel][3] partial-derivative triples
      dmap[o + 0] = dmx;
      dmap[o + 1] = dexx;
      dmap[o + 2] = dexy;
      s_val += S;
      l1 += fabsf(s_x[(oy + kLR) * kLS + ox + kLR] - s_y[(oy + kLR) * kLS + ox + kLR]);
    }
  }
  // fixed-order block sums
  s_val = wave_sum_lane63(s_val);
  l1 = wave_sum_lane63(l1);
  const int lane = t & (kWave - 1), wave = t / kWave;
  if (lane == kWave - 1) {
    s_red[0][wave] = s_val;
    s_red[1][wave] = l1;
  }
  __syncthreads();
  if (t == 0) {
    bsum[2 * blockIdx.x + 0] = (s_red[0][0] + s_red[0][1]) + (s_red[0][2] + s_red[0][3]);
    bsum[2 * blockIdx.x + 1] = (s_red[1][0] + s_red[1][1]) + (s_red[1][2] + s_red[1][3]);
  }
}

__global__ __launch_bounds__(256) void ssim_bwd_kernel(const float* __restrict__ image,
                                                       const float* __restrict__ target, LossViews lv,
                                                       const float* __restrict__ dmap, float lambda,
                                                       float* __restrict__ dL) {
  __shared__ float s_d[3][kLS * kLS];
  __shared__ float s_h[3][kLS * kLT];
  const LossTile tl = loss_tile(lv, blockIdx.x);
  const LossView& q = lv.v[tl.view];
  const int W = q.W, H = q.H, t = threadIdx.x;
  const int64_t plane_px = (int64_t)W * H;
  const int64_t poff = 3 * q.pix_off + tl.plane * plane_px;
  const int x0 = tl.tx * kLT, y0 = tl.ty * kLT;
  for (int i = t; i < kLS * kLS; i += 256) {
    const int r = i / kLS, c = i - r * kLS;
    const int x = x0 - kLR + c, y = y0 - kLR + r;
    float a = 0.f, b = 0.f, d = 0.f;
    if (x >= 0 && x < W && y >= 0 && y < H) {
      const int64_t o = 3 * (poff + (int64_t)y * W + x);
      a = dmap[o + 0];
      b = dmap[o + 1];
      d = dmap[o + 2];
    }
    s_d[0][i] = a;
    s_d[1][i] = b;
    s_d[2][i] = d;
  }
  __syncthreads();
  for (int i = t; i < kLS * kLT; i += 256) {
    const int r = i / kLT, c = i - r * kLT;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
      const float g = lv.g[k];
      a0 += g * s_d[0][r * kLS + c + k];
      a1 += g * s_d[1][r * kLS + c + k];
      a2 += g * s_d[2][r * kLS + c + k];
    }
    s_h[0][i] = a0;
    s_h[1][i] = a1;
    s_h[2][i] = a2;
  }
  __syncthreads();
  const int ox = out_col(t);
  const float scale = 1.0f / ((float)lv.nviews * 3.0f * (float)plane_px);
#pragma unroll
  for (int j = 0; j < kLQ; ++j) {
    const int oy = out_row(t, j);
    const int px = x0 + ox, py = y0 + oy;
    if (px >= W || py >= H) continue;
    float wa = 0.f, wb = 0.f, wc = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
      const float g = lv.g[k];
      const int i = (oy + k) * kLT + ox;
      wa += g * s_h[0][i];
      wb += g * s_h[1][i];
      wc += g * s_h[2][i];
    }
    const int64_t gi = poff + (int64_t)py * W + px;
    const float x = image[gi], y = target[gi];
    const float dsdx = wa + 2.f * x * wb + y * wc;
    const float sg = x > y ? 1.f : (x < y ? -1.f : 0.f);
    dL[gi] = ((1.0f - lambda) * sg - lambda * dsdx) * scale;
  }
}

// Per-view loss from its workgroups' sums: one workgroup per view, each thread
// a fixed stride of the sums in double, then a fixed tree.
__global__ __launch_bounds__(256) void loss_reduce_kernel(const float* __restrict__ bsum, LossViews lv,
                                                          float lambda, double* __restrict__ per_view,
                                                          float* __restrict__ loss) {
  __shared__ double s_s[256], s_l[256];
  const int v = blockIdx.x, t = threadIdx.x;
  const LossView& q = lv.v[v];
  const int nb = 3 * q.TX * q.TY;
  double s = 0.0, l1 = 0.0;
  for (int b = t; b < nb; b += 256) {
    s += (double)bsum[2 * (q.block_off + b) + 0];
    l1 += (double)bsum[2 * (q.block_off + b) + 1];
  }
  s_s[t] = s;
  s_l[t] = l1;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      s_s[t] += s_s[t + o];
      s_l[t] += s_l[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double n = 3.0 * (double)q.W * (double)q.H;
    const double lval = (1.0 - (double)lambda) * (s_l[0] / n) + (double)lambda * (1.0 - s_s[0] / n);
    per_view[v] = lval;
    loss[v] = (float)lval;
  }
}

// loss[V] = mean of the per-view losses, in view order.
__global__ void loss_mean_kernel(const double* __restrict__ per_view, int V, float* __restrict__ loss) {
  if (threadIdx.x != 0) return;
  double m = 0.0;
  for (int v = 0; v < V; ++v) m += per_view[v];
  loss[V] = (float)(m / V);
}

hipError_t launch_loss(const LossViews& lv, const float* image, const float* target, float lambda, float* loss,
                       float* dL, float* dmap, float* bsum, double* per_view, hipStream_t s) {
  const int nb = lv.total_blocks;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(ssim_fwd_kernel, dim3((unsigned)nb), dim3(256), 0, s, image, target, lv, dmap, bsum);
  if (dL) hipLaunchKernelGGL(ssim_bwd_kernel, dim3((unsigned)nb), dim3(256), 0, s, image, target, lv, dmap, lambda, dL);
  if (loss) {
    hipLaunchKernelGGL(loss_reduce_kernel, dim3((unsigned)lv.nviews), dim3(256), 0, s, bsum, lv, lambda, per_view, loss);
    hipLaunchKernelGGL(loss_mean_kernel, dim3(1), dim3(64), 0, s, per_view, lv.nviews, loss);
  }
  return hipGetLastError();
}

}  // namespace gs

namespace gs {

// Mask terms of Eq. 7: lambda_m mean sigmoid(m) + lambda_sh mean sum_l w_l
// sigmoid(m^l), w_l = (2l + 1) / sum (2l' + 1) over bands 1..deg (each band
// weighted by its coefficient count, Sec. 3.2.3).  One thread per Gaussian:
// gradients accumulated (+=) into the mask-logit gradients; per-workgroup sums
// in a fixed order; a one-workgroup kernel adds them in double.
__global__ __launch_bounds__(256) void mask_loss_kernel(const float* __restrict__ m, const float* __restrict__ msh,
                                                        int64_t n, int deg, float lam_m, float lam_sh,
                                                        float* __restrict__ gm, float* __restrict__ gsh,
                                                        float* __restrict__ bsum) {
  __shared__ float s_red[2][4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float a = 0.f, b = 0.f;
  if (i < n) {
    const float inv_n = 1.0f / (float)n;
    if (m) {
      const float s = 1.0f / (1.0f + __expf(-m[i]));
      a = s;
      if (gm) gm[i] += lam_m * s * (1.0f - s) * inv_n;
    }
    if (msh && deg > 0) {
      const float wsum = (float)(deg * (deg + 2));  // sum_{l=1..deg} (2l + 1)
      for (int l = 1; l <= deg; ++l) {
        const float w = (float)(2 * l + 1) / wsum;
        const float s = 1.0f / (1.0f + __expf(-msh[(int64_t)(l - 1) * n + i]));
        b += w * s;
        if (gsh) gsh[(int64_t)(l - 1) * n + i] += lam_sh * w * s * (1.0f - s) * inv_n;
      }
    }
  }
  a = wave_sum_lane63(a);
  b = wave_sum_lane63(b);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == kWave - 1) {
    s_red[0][wave] = a;
    s_red[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bsum[2 * blockIdx.x + 0] = ((s_red[0][0] + s_red[0][1]) + s_red[0][2]) + s_red[0][3];
    bsum[2 * blockIdx.x + 1] = ((s_red[1][0] + s_red[1][1]) + s_red[1][2]) + s_red[1][3];
  }
}

__global__ __launch_bounds__(256) void mask_loss_reduce_kernel(const float* __restrict__ bsum, int nb, int64_t n,
                                                               float lam_m, float lam_sh, float* __restrict__ loss) {
  __shared__ double s_a[256], s_b[256];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int k = t; k < nb; k += 256) {
    a += (double)bsum[2 * k + 0];
    b += (double)bsum[2 * k + 1];
  }
  s_a[t] = a;
  s_b[t] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      s_a[t] += s_a[t + o];
      s_b[t] += s_b[t + o];
    }
    __syncthreads();
  }
  if (t == 0) loss[0] = (float)((double)lam_m * s_a[0] / (double)n + (double)lam_sh * s_b[0] / (double)n);
}

hipError_t launch_mask_loss(const float* m, const float* msh, int64_t n, int deg, float lam_m, float lam_sh,
                            float* gm, float* gsh, float* loss, float* bsum, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(mask_loss_kernel, dim3((unsigned)nb), dim3(256), 0, s, m, msh, n, deg, lam_m, lam_sh, gm, gsh,
                     bsum);
  if (loss) hipLaunchKernelGGL(mask_loss_reduce_kernel, dim3(1), dim3(256), 0, s, bsum, nb, n, lam_m, lam_sh, loss);
  return hipGetLastError();
}

// One thread per element: dL = scale_v (image - target), v the element's view.
__global__ __launch_bounds__(256) void l2_grad_kernel(const float* __restrict__ image,
                                                      const float* __restrict__ target, float* __restrict__ dL,
                                                      L2Args a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.end[a.nviews - 1]) return;
  int v = 0;
  while (e >= a.end[v]) ++v;
  dL[e] = a.scale[v] * (image[e] - target[e]);
}

hipError_t launch_l2_grad(const float* image, const float* target, float* dL, const L2Args& a, hipStream_t s) {
  const int64_t total = a.nviews > 0 ? a.end[a.nviews - 1] : 0;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(l2_grad_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, image, target, dL, a);
  return hipGetLastError();
}

}  // namespace gs
