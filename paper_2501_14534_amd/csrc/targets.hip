// Target images for progressive training (Sec. 3.2.4): Gaussian blur with a
// shrinking kernel and area resampling to the current training resolution
// (Eq. 6).  Both act on every view of a call ([3][H][W] planes, views
// concatenated) and run when the schedule changes, not every step.
//
// Blur: one workgroup per (view, plane, 16 x 16 output tile) stages the tile
// and a halo of r = (k - 1) / 2 pixels in LDS, reflected about the edge pixels
// (index -1 reads 1), then filters rows and columns with the k normalised
// taps (two 1-D passes, k <= 31).
//
// Resize: one thread per output value averages the input over the value's
// box [x' W / W', (x' + 1) W / W') x [y' H / H', (y' + 1) H / H').  Overlaps
// are integers in units of 1 / W' (1 / H'), so the weights are exact; the sum
// runs over rows of the box in float and is divided by W H once.
#include "gs_common.h"
#include "kernels.h"

namespace gs {

constexpr int kBT = kBlurTile;                   // output tile edge
constexpr int kBS = kBT + 2 * kMaxBlurRadius;    // largest staged edge

__device__ __forceinline__ int mirror_index(int i, int n) {
  if (n == 1) return 0;
  const int p = 2 * (n - 1);
  i %= p;
  if (i < 0) i += p;
  return i < n ? i : p - i;
}

__global__ __launch_bounds__(256) void blur_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                   BlurArgs b) {
  __shared__ float s_in[kBS * kBS];
  __shared__ float s_h[kBS * kBT];
  const LossTile tl = loss_tile(b.views, blockIdx.x);
  const LossView& q = b.views.v[tl.view];
  const int W = q.W, H = q.H, r = b.r, S = kBT + 2 * r, t = threadIdx.x;
  const int64_t poff = 3 * q.pix_off + tl.plane * (int64_t)W * H;
  const float* src = in + poff;
  const int x0 = tl.tx * kBT, y0 = tl.ty * kBT;
  for (int i = t; i < S * S; i += 256) {
    const int row = i / S, col = i - row * S;
    const int y = mirror_index(y0 - r + row, H), x = mirror_index(x0 - r + col, W);
    s_in[i] = src[(int64_t)y * W + x];
  }
  __syncthreads();
  for (int i = t; i < S * kBT; i += 256) {  // rows of the staged window, the tile's 16 columns
    const int row = i / kBT, col = i - row * kBT;
    float acc = 0.f;
    for (int k = 0; k <= 2 * r; ++k) acc += b.g[k] * s_in[row * S + col + k];
    s_h[i] = acc;
  }
  __syncthreads();
  const int oy = t / kBT, ox = t - oy * kBT;
  const int px = x0 + ox, py = y0 + oy;
  if (px < W && py < H) {
    float acc = 0.f;
    for (int k = 0; k <= 2 * r; ++k) acc += b.g[k] * s_h[(oy + k) * kBT + ox];
    out[poff + (int64_t)py * W + px] = acc;
  }
}

__global__ __launch_bounds__(256) void resize_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                     ResizeArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.total_out) return;
  int v = 0;
  while (v + 1 < a.nviews && e >= 3 * a.v[v + 1].out_off) ++v;
  const ResizeView& q = a.v[v];
  const int64_t plane_out = (int64_t)q.Wo * q.Ho;
  const int64_t le = e - 3 * q.out_off;
  const int c = (int)(le / plane_out);
  const int64_t p = le - c * plane_out;
  const int yo = (int)(p / q.Wo), xo = (int)(p - (int64_t)yo * q.Wo);
  const int W = q.W, H = q.H, Wo = q.Wo, Ho = q.Ho;
  // input pixels whose box overlaps output pixel (xo, yo)
  const int xa = (int)(((int64_t)xo * W) / Wo), xb = (int)(((int64_t)(xo + 1) * W + Wo - 1) / Wo);
  const int ya = (int)(((int64_t)yo * H) / Ho), yb = (int)(((int64_t)(yo + 1) * H + Ho - 1) / Ho);
  const float* src = in + 3 * q.in_off + c * (int64_t)W * H;
  float acc = 0.f;
  for (int y = ya; y < yb; ++y) {
    const int64_t ny = min((int64_t)(y + 1) * Ho, (int64_t)(yo + 1) * H) - max((int64_t)y * Ho, (int64_t)yo * H);
    float row = 0.f;
    for (int x = xa; x < xb; ++x) {
      const int64_t nx = min((int64_t)(x + 1) * Wo, (int64_t)(xo + 1) * W) - max((int64_t)x * Wo, (int64_t)xo * W);
      row += (float)nx * src[(int64_t)y * W + x];
    }
    acc += (float)ny * row;
  }
  out[e] = acc * a.v[v].inv_area;
}

hipError_t launch_blur(const float* in, float* out, const BlurArgs& b, hipStream_t s) {
  if (b.views.total_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(blur_kernel, dim3((unsigned)b.views.total_blocks), dim3(256), 0, s, in, out, b);
  return hipGetLastError();
}

hipError_t launch_resize(const float* in, float* out, const ResizeArgs& a, hipStream_t s) {
  if (a.total_out == 0) return hipSuccess;
  hipLaunchKernelGGL(resize_kernel, dim3((unsigned)((a.total_out + 255) / 256)), dim3(256), 0, s, in, out, a);
  return hipGetLastError();
}

}  // namespace gs
