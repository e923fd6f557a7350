// Backward of the projection: per-pair splat gradients (u, v, A, B, C, o',
// r, g, b) -> raw Gaussian parameters, accumulated over the V views of the
// call and added (+=) to the caller's gradient arrays.  Straight-through
// estimator for the hard masks (Eq. 3, Eq. 5): d(mask)/d(logit) = sigmoid'.
//
// Two kernels (no atomics):
//   colour:   one thread per Gaussian, the views in order: first its record's
//             pair gradients summed in emission order (double, rounded once to
//             float; a wave's records in one view own one contiguous run of
//             pairs, staged through LDS), then the SH chain in single
//             precision (diffuse colour, band-mask logits, bands 1..3 when that
//             gradient is asked for, and the view-direction term of the mean);
//             the record sums and the colour term go to per-record planes;
//   geometry: one thread per Gaussian, reading those planes: the EWA chain
//             in double precision (the 2x2 inverse amplifies rounding by the
//             condition number of Sigma'):
//     dL/dSigma'  = -Q G_Q Q              (G_Q = [[gA, gB/2], [gB/2, gC]], Q = conic)
//     dL/dSigma   = T^T dL/dSigma' T,     dL/dT = 2 dL/dSigma' T Sigma,  T = J W
//     dL/dJ -> camera-space mean (J's entries, the clamp of the lateral ratios),
//     plus the screen mean (u, v); dL/dmu = W^T dL/dt + colour term;
//     dL/dM = 2 dL/dSigma M with M = Rq diag(s) -> scales, rotation, through
//     the quaternion normalisation; opacity and volume mask.
// Each view's contribution is rounded to float and added to the running
// totals in view order with non-contracted adds: the association a sequence
// of per-view calls produces, so a batched call equals the per-view calls.
#include "gs_common.h"
#include "kernels.h"

namespace gs {

// Gradient of the 15 SH basis polynomials (k = 1..15) w.r.t. (x, y, z),
// contracted with per-function weights w[k-1]: returns sum_k w_k grad Y_k.
__device__ __forceinline__ void sh_grad15(float x, float y, float z, const float w[15], float* gx, float* gy,
                                          float* gz) {
  const float xx = x * x, yy = y * y, zz = z * z;
  float ax = 0.f, ay = 0.f, az = 0.f;
  // band 1
  ay += -kC1 * w[0];
  az += kC1 * w[1];
  ax += -kC1 * w[2];
  // band 2
  ax += kC2a * y * w[3];
  ay += kC2a * x * w[3];
  ay += -kC2a * z * w[4];
  az += -kC2a * y * w[4];
  ax += -2.f * kC2b * x * w[5];
  ay += -2.f * kC2b * y * w[5];
  az += 4.f * kC2b * z * w[5];
  ax += -kC2a * z * w[6];
  az += -kC2a * x * w[6];
  ax += 2.f * kC2c * x * w[7];
  ay += -2.f * kC2c * y * w[7];
  // band 3
  ax += -6.f * kC3a * x * y * w[8];
  ay += -kC3a * (3.f * xx - 3.f * yy) * w[8];
  ax += kC3b * y * z * w[9];
  ay += kC3b * x * z * w[9];
  az += kC3b * x * y * w[9];
  ax += 2.f * kC3c * x * y * w[10];
  ay += -kC3c * (4.f * zz - xx - 3.f * yy) * w[10];
  az += -8.f * kC3c * y * z * w[10];
  ax += -6.f * kC3d * x * z * w[11];
  ay += -6.f * kC3d * y * z * w[11];
  az += kC3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[11];
  ax += -kC3c * (4.f * zz - 3.f * xx - yy) * w[12];
  ay += 2.f * kC3c * x * y * w[12];
  az += -8.f * kC3c * x * z * w[12];
  ax += 2.f * kC3e * x * z * w[13];
  ay += -2.f * kC3e * y * z * w[13];
  az += kC3e * (xx - yy) * w[13];
  ax += -kC3a * (3.f * xx - 3.f * yy) * w[14];
  ay += 6.f * kC3a * x * y * w[14];
  *gx = ax;
  *gy = ay;
  *gz = az;
}

// t + x without fusing into a preceding multiply (same rounding as two calls).
__device__ __forceinline__ float acc_add(float t, float x) {
#pragma clang fp contract(off)
  return t + x;
}
__device__ __forceinline__ float acc_mul_add(float t, float a, float b) {
#pragma clang fp contract(off)
  const float p = a * b;
  return t + p;
}

// Sums of the 9 pair gradients of each lane's record (cnt pairs from pair
// index off; cnt = 0 gives zeros), accumulated in double and rounded once to
// float.  Called by all 64 lanes of a wave together, for records of
// consecutive Gaussians in one view: their pairs form one contiguous run of
// the [K][9] array (emission order is record order).  A pair the backward walk
// did not reach has no row this step (its live byte is 0) and counts as zero.
//  - Light records (at most kHeavyPairs pairs): the wave copies the run into
//    LDS window by window with 16-byte loads of consecutive addresses, with the
//    pairs' live bytes, and each lane adds its own pairs from LDS in emission
//    order.  (Loading its pairs directly would touch a separate cache line per
//    lane and load.)  Windows holding no light record's pairs are skipped.
//  - Heavy records (the nearest Gaussians cover thousands of tiles, which one
//    lane would add up alone) are summed beforehand by heavy_sums_kernel, the
//    whole wave on one record, and are left at zero here.
// Both orders depend only on the record's own pairs, not on where its run
// starts, so a record's sums are the same in a batched and a per-view call.
constexpr int kSumWindow = 256;  // pairs per window (9 x 256 floats = 576 float4, 9 per lane)
constexpr uint32_t kHeavyPairs = 256;

__device__ __forceinline__ void record_sums(const float* __restrict__ grad_pair, const uint8_t* __restrict__ live,
                                            uint32_t cnt, uint32_t off, float4* win4, uint32_t* livew, int lane,
                                            float out[GS_GRAD_FLOATS]) {
  double gsum[GS_GRAD_FLOATS] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const uint32_t lcnt = cnt > kHeavyPairs ? 0u : cnt;
  // offsets grow with the lane (consecutive records), so the light records'
  // pairs lie between the first light lane's start and the last one's end
  const uint64_t act = __ballot(lcnt != 0u);
  const uint32_t lo = act ? (uint32_t)__builtin_amdgcn_readlane((int)off, __builtin_ctzll(act)) : 0u;
  const uint32_t hi = act ? (uint32_t)__builtin_amdgcn_readlane((int)(off + lcnt), 63 - __builtin_clzll(act)) : 0u;
  float* win = (float*)win4;
  uint32_t w0 = lo & ~3u;  // windows start on 16 bytes
  while (w0 < hi) {
    const uint32_t w1 = min(w0 + (uint32_t)kSumWindow, hi);
    if (__ballot(lcnt != 0u && off < w1 && off + lcnt > w0) == 0) {  // only heavy records' pairs here
      w0 += kSumWindow;
      continue;
    }
    const int nfl = (int)(w1 - w0) * GS_GRAD_FLOATS, nf4 = nfl / 4;
    const float* src = grad_pair + (size_t)w0 * GS_GRAD_FLOATS;
    // loads straight into LDS, no registers in between: lane l of load j
    // fills float4 64 j + l (lanes past the window are masked off), then
    // lanes 0 .. nfl % 4 - 1 the floats after the last whole float4
    constexpr int kPerLane = kSumWindow * GS_GRAD_FLOATS / 4 / kWave;
#pragma unroll
    for (int j = 0; j < kPerLane; ++j)
      if (lane + j * kWave < nf4)
        __builtin_amdgcn_global_load_lds((const void*)((const float4*)src + lane + j * kWave),
                                         (__attribute__((address_space(3))) void*)(win4 + j * kWave), 16, 0, 0);
    if (lane < nfl % 4)
      __builtin_amdgcn_global_load_lds((const void*)(src + nf4 * 4 + lane),
                                       (__attribute__((address_space(3))) void*)(win + nf4 * 4), 4, 0, 0);
    // the pairs' live bytes, a word per lane (w0 is a multiple of 4; the array
    // is padded past the last pair)
    if (lane < (int)(w1 - w0 + 3) / 4)
      __builtin_amdgcn_global_load_lds((const void*)(live + w0 + 4 * lane),
                                       (__attribute__((address_space(3))) void*)livew, 4, 0, 0);
    __builtin_amdgcn_s_waitcnt(0);  // the LDS writes of the loads above have landed
    wave_lds_sync();
    const uint32_t k1 = min(off + lcnt, w1);
    const uint8_t* lv = (const uint8_t*)livew;
    for (uint32_t k = max(off, w0); k < k1; ++k)
      if (lv[k - w0])  // rows of pairs the walk did not reach are not written: they count as zero
#pragma unroll
        for (int c = 0; c < GS_GRAD_FLOATS; ++c) gsum[c] += (double)win[(k - w0) * GS_GRAD_FLOATS + c];
    wave_lds_sync();  // every lane has read the window before the next one overwrites it
    w0 += kSumWindow;
  }
#pragma unroll
  for (int c = 0; c < GS_GRAD_FLOATS; ++c) out[c] = (float)gsum[c];
}

__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// Sums of the pair gradients of the heavy records (more than kHeavyPairs
// pairs), written to the record planes (all nine) for the colour kernel to
// read.  One thread per record finds them; each wave then takes its heavy
// records one at a time: lane j adds pairs j, j + 64, ... of the record in
// double, a butterfly in a fixed pattern adds the lanes, and the sum is
// rounded once to float.
__global__ __launch_bounds__(256) void heavy_sums_kernel(ProjectBwdArgs b, int64_t nrec) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t cnt = r < nrec && *b.status == 0 ? b.tiles_touched[r] : 0u;
  uint64_t hv = __ballot(cnt > kHeavyPairs);
  while (hv) {
    const int L = __builtin_ctzll(hv);
    hv &= hv - 1;
    const int64_t hr = (int64_t)__builtin_amdgcn_readlane((int)(r - (int64_t)blockIdx.x * blockDim.x), L) +
                       (int64_t)blockIdx.x * blockDim.x;
    const uint32_t hcnt = (uint32_t)__builtin_amdgcn_readlane((int)cnt, L);
    const uint32_t hoff = b.offsets[hr];
    double part[GS_GRAD_FLOATS] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t j = (uint32_t)lane; j < hcnt; j += kWave) {
      const size_t k = (size_t)hoff + j;
      if (b.pair_live[k]) {
        const float* row = b.grad_pair + k * GS_GRAD_FLOATS;
#pragma unroll
        for (int c = 0; c < GS_GRAD_FLOATS; ++c) part[c] += (double)row[c];
      }
    }
#pragma unroll
    for (int c = 0; c < GS_GRAD_FLOATS; ++c) {
      const double t = wave_sum_f64(part[c]);
      if (lane == L) b.rec[c * b.rec_stride + hr] = (float)t;
    }
  }
}

// A parameter gradient: written (assign) or added.
__device__ __forceinline__ void grad_out(float* g, bool assign, float t) { *g = assign ? t : *g + t; }

// Colour-kernel outputs of Gaussian i.
template <int DEG, bool REST>
__device__ __forceinline__ void colour_grads_out(const ProjectBwdArgs& b, int64_t n, int64_t i, const float tdc[3],
                                                 const float tbm[3], const float (*trest)[3]) {
  const bool as = b.assign != 0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (b.g_sh_dc) grad_out(&b.g_sh_dc[k * n + i], as, tdc[k]);
  if (DEG > 0 && b.g_sh_mask_logits && b.p.sh_mask_logits) {
#pragma unroll
    for (int l = 1; l <= DEG; ++l) grad_out(&b.g_sh_mask_logits[(l - 1) * n + i], as, tbm[l - 1]);
  }
  if (REST) {
    constexpr int NR = (DEG + 1) * (DEG + 1) - 1;
#pragma unroll
    for (int k = 1; k <= NR; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) grad_out(&b.g_sh_rest[((k - 1) * 3 + c) * n + i], as, trest[k - 1][c]);
  }
}

// Views (bit v) in which record (v, i) touches a tile.
__device__ __forceinline__ uint32_t visible_views(const ProjectBwdArgs& b, int V, int64_t n, int64_t i) {
  uint32_t vis = 0;
  for (int v = 0; v < V; ++v) vis |= (b.tiles_touched[(size_t)v * n + i] != 0u ? 1u : 0u) << v;
  return vis;
}

// Band masks of Gaussian i (Eq. 5): sigmoid(m_l) > eps <=> m_l > logit(eps).
__device__ __forceinline__ void band_masks(const ProjectArgs& a, int64_t n, int64_t i, float bm[3], bool on[4]) {
  on[0] = on[1] = on[2] = on[3] = true;
  bm[0] = bm[1] = bm[2] = 0.f;
  if (a.sh_mask_logits) {
#pragma unroll
    for (int l = 1; l <= 3; ++l) {
      bm[l - 1] = a.sh_mask_logits[(l - 1) * n + i];
      on[l] = bm[l - 1] > a.sh_mask_thr;
    }
  }
}

// Unit view direction from the camera centre to the mean, and 1 / distance.
__device__ __forceinline__ void view_dir(const ViewArgs& c, const float mu[3], float* dx, float* dy, float* dz,
                                        float* il) {
  const float d0 = mu[0] - c.campos[0], d1 = mu[1] - c.campos[1], d2 = mu[2] - c.campos[2];
  *il = 1.0f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
  *dx = d0 * *il, *dy = d1 * *il, *dz = d2 * *il;
}

// Per Gaussian over the views: the record sums of each visible view
// (record_sums), then the colour chain: the gradient of the clamped colour,
// the diffuse colour and band-mask gradients, with REST the SH bands 1..DEG
// (sum over the views of Y_k(d_v) times that gradient; bands whose hard mask
// is off get nothing), and the colour term of the mean gradient (through the
// view direction).  Every lane of a wave writes its record's planes in each
// view the wave visits (zeros where the Gaussian is not visible), so the
// record planes are written in whole cache lines.
template <int DEG, bool REST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void project_bwd_color_kernel(
    ProjectBwdArgs b, ViewTable vt) {
  __shared__ float4 s_win[256 / kWave][kSumWindow * GS_GRAD_FLOATS / 4];
  __shared__ uint32_t s_live[256 / kWave][kSumWindow / 4];
  const ProjectArgs& a = b.p;
  const int64_t n = a.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const bool valid = i < n;
  const int V = vt.nviews;
  constexpr int NRT = REST ? (DEG + 1) * (DEG + 1) - 1 : 1;
  const float zero3[3] = {0.f, 0.f, 0.f};
  float trest[NRT][3];
#pragma unroll
  for (int k = 0; k < NRT; ++k) trest[k][0] = trest[k][1] = trest[k][2] = 0.f;
  // binning overflowed (no lists, no gradients), or the whole wave culled or
  // off-screen everywhere: zeros when the gradients are written, else nothing
  const uint32_t vis = valid && *b.status == 0 ? visible_views(b, V, n, i) : 0u;
  if (__ballot(vis != 0u) == 0) {
    if (b.assign && valid) colour_grads_out<DEG, REST>(b, n, i, zero3, zero3, trest);
    return;
  }

  constexpr int NR = DEG > 0 ? (DEG + 1) * (DEG + 1) - 1 : 1;
  float mu[3] = {0.f, 0.f, 0.f}, dc[3] = {0.f, 0.f, 0.f};
  float rest[NR][3];
  float bm[3] = {0.f, 0.f, 0.f};
  bool band_on[4] = {true, true, true, true};
#pragma unroll
  for (int k = 0; k < NR; ++k) rest[k][0] = rest[k][1] = rest[k][2] = 0.f;
  if (vis) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      mu[k] = a.means[k * n + i];
      dc[k] = a.sh_dc[k * n + i];
    }
    band_masks(a, n, i, bm, band_on);
    if (DEG > 0) {
      // every band's coefficients are read: the band-mask gradient needs them
      // even when the band is off (straight-through estimator)
#pragma unroll
      for (int k = 1; k <= NR; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) rest[k - 1][c] = a.sh_rest[((k - 1) * 3 + c) * n + i];
    }
  }
  float tdc[3] = {0.f, 0.f, 0.f}, tbm[3] = {0.f, 0.f, 0.f};

  // v is the same in every lane: camera constants are scalar loads, and a
  // wave's records in view v are consecutive
  // (the next view's pair counts and offsets load while this view is processed)
  uint32_t cnt_next = (vis & 1u) ? b.tiles_touched[i] : 0u, off_next = (vis & 1u) ? b.offsets[i] : 0u;
  for (int v = 0; v < V; ++v) {
    const bool on = (vis >> v) & 1u;
    const int64_t r = (int64_t)v * n + i;
    const uint32_t cnt = cnt_next, off = off_next;
    if (v + 1 < V) {
      const bool on1 = (vis >> (v + 1)) & 1u;
      cnt_next = on1 ? b.tiles_touched[r + n] : 0u;
      off_next = on1 ? b.offsets[r + n] : 0u;
    }
    if (__ballot(on) == 0) continue;
    float g9[GS_GRAD_FLOATS];
    record_sums(b.grad_pair, b.pair_live, cnt, off, s_win[wave], s_live[wave], lane, g9);
    if (cnt > kHeavyPairs) {  // summed by heavy_sums_kernel
#pragma unroll
      for (int c = 0; c < GS_GRAD_FLOATS; ++c) g9[c] = b.rec[c * b.rec_stride + r];
    }
    if (b.g_mean2d && on) {
      b.g_mean2d[(v * 2 + 0) * n + i] += g9[0];
      b.g_mean2d[(v * 2 + 1) * n + i] += g9[1];
    }
    float gmu_col[3] = {0.f, 0.f, 0.f};
    const float grgb[3] = {g9[6], g9[7], g9[8]};
    if (on && (grgb[0] != 0.f || grgb[1] != 0.f || grgb[2] != 0.f)) {
      const ViewArgs& c = vt.v[v];
      float pre[3] = {dc[0], dc[1], dc[2]};
      float Y[15];
      float dx = 0.f, dy = 0.f, dz = 0.f, il = 1.f;
      if (DEG > 0) {
        view_dir(c, mu, &dx, &dy, &dz, &il);
        sh_basis15(dx, dy, dz, Y);
        // flat loops with constant trip counts keep rest/Y in registers
#pragma unroll
        for (int k = 1; k < kShCoeffs; ++k) {
          const int l = sh_band(k);
          if (l > DEG || !band_on[l]) continue;
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) pre[ch] += Y[k - 1] * rest[k - 1][ch];
        }
      }
      float gpre[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        gpre[ch] = pre[ch] < 0.f ? 0.f : grgb[ch];
        tdc[ch] = acc_add(tdc[ch], gpre[ch]);
      }
      if (DEG > 0) {
        float wY[15];
#pragma unroll
        for (int k = 0; k < 15; ++k) wY[k] = 0.f;
        float band[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 1; k < kShCoeffs; ++k) {
          const int l = sh_band(k);
          if (l > DEG) continue;
          const float cg = rest[k - 1][0] * gpre[0] + rest[k - 1][1] * gpre[1] + rest[k - 1][2] * gpre[2];
          band[l - 1] += Y[k - 1] * cg;
          if (band_on[l]) wY[k - 1] = cg;
        }
#pragma unroll
        for (int l = 1; l <= DEG; ++l) {
          const float sb = sigmoidf(bm[l - 1]);
          tbm[l - 1] = acc_mul_add(tbm[l - 1], band[l - 1], sb * (1.f - sb));
        }
        float gdx, gdy, gdz;
        sh_grad15(dx, dy, dz, wY, &gdx, &gdy, &gdz);
        const float dot = dx * gdx + dy * gdy + dz * gdz;
        gmu_col[0] = (gdx - dx * dot) * il;
        gmu_col[1] = (gdy - dy * dot) * il;
        gmu_col[2] = (gdz - dz * dot) * il;
        if (REST && (gpre[0] != 0.f || gpre[1] != 0.f || gpre[2] != 0.f)) {  // else it adds exact zeros
#pragma unroll
          for (int k = 1; k < kShCoeffs; ++k) {
            const int l = sh_band(k);
            if (l > DEG || !band_on[l]) continue;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
              trest[k - 1][ch] = acc_mul_add(trest[k - 1][ch], Y[k - 1], gpre[ch]);
          }
        }
      }
    }
    if (valid) {
      float* rp = b.rec + r;
#pragma unroll
      for (int k = 0; k < 6; ++k) rp[k * b.rec_stride] = on ? g9[k] : 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) rp[(6 + k) * b.rec_stride] = gmu_col[k];
    }
  }

  if (!valid || (!vis && !b.assign)) return;
  colour_grads_out<DEG, REST>(b, n, i, tdc, tbm, trest);
}

// Geometry-kernel outputs of Gaussian i (null arrays: zeros).
__device__ __forceinline__ void geom_grads_out(const ProjectBwdArgs& b, int64_t n, int64_t i, const float* tmu,
                                               const float* tls, const float* tq, float top, float tmask) {
  const bool as = b.assign != 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (b.g_means) grad_out(&b.g_means[k * n + i], as, tmu ? tmu[k] : 0.f);
    if (b.g_log_scales) grad_out(&b.g_log_scales[k * n + i], as, tls ? tls[k] : 0.f);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (b.g_quats) grad_out(&b.g_quats[k * n + i], as, tq ? tq[k] : 0.f);
  if (b.g_opacity_logits) grad_out(&b.g_opacity_logits[i], as, top);
  if (b.g_mask_logits && b.p.mask_logits) grad_out(&b.g_mask_logits[i], as, tmask);
}

__global__ __launch_bounds__(256) void project_bwd_geom_kernel(ProjectBwdArgs b, ViewTable vt) {
  const ProjectArgs& a = b.p;
  const int64_t n = a.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t vis = *b.status == 0 ? visible_views(b, vt.nviews, n, i) : 0u;
  if (!vis) {  // no gradient (culled, off-screen, or the binning overflowed)
    if (b.assign) geom_grads_out(b, n, i, nullptr, nullptr, nullptr, 0.f, 0.f);
    return;
  }

  float mu[3], ls[3], q[4];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    mu[k] = a.means[k * n + i];
    ls[k] = a.log_scales[k * n + i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = a.quats[k * n + i];
  const float ol = a.opacity_logits[i];

  const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
  const double iq = 1.0 / sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const double w = q0 * iq, x = q1 * iq, y = q2 * iq, z = q3 * iq;
  const double Rq[3][3] = {{1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                           {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                           {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
  double s[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) s[k] = exp((double)ls[k]);
  double Sig[6];  // xx, xy, xz, yy, yz, zz
  {
    double M[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) M[r][k] = Rq[r][k] * s[k];
    Sig[0] = M[0][0] * M[0][0] + M[0][1] * M[0][1] + M[0][2] * M[0][2];
    Sig[1] = M[0][0] * M[1][0] + M[0][1] * M[1][1] + M[0][2] * M[1][2];
    Sig[2] = M[0][0] * M[2][0] + M[0][1] * M[2][1] + M[0][2] * M[2][2];
    Sig[3] = M[1][0] * M[1][0] + M[1][1] * M[1][1] + M[1][2] * M[1][2];
    Sig[4] = M[1][0] * M[2][0] + M[1][1] * M[2][1] + M[1][2] * M[2][2];
    Sig[5] = M[2][0] * M[2][0] + M[2][1] * M[2][1] + M[2][2] * M[2][2];
  }
  const double op = 1.0 / (1.0 + exp(-(double)ol));
  double sm = 0.0;
  if (a.mask_logits) sm = 1.0 / (1.0 + exp(-(double)a.mask_logits[i]));

  float tmu[3] = {0.f, 0.f, 0.f}, tls[3] = {0.f, 0.f, 0.f}, tq[4] = {0.f, 0.f, 0.f, 0.f};
  float top = 0.f, tmask = 0.f;
  // the views in order, v wave-uniform as in the colour kernel
  const int V = vt.nviews;
  for (int v = 0; v < V; ++v) {
    if (!((vis >> v) & 1u)) continue;
    const float* rp = b.rec + (size_t)v * n + i;
    const int64_t rs = b.rec_stride;
    const double gu = rp[0], gv = rp[rs], gA = rp[2 * rs], gB = rp[3 * rs], gC = rp[4 * rs], go = rp[5 * rs];
    const float cmu[3] = {rp[6 * rs], rp[7 * rs], rp[8 * rs]};  // colour term of the mean gradient
    if (gu == 0.0 && gv == 0.0 && gA == 0.0 && gB == 0.0 && gC == 0.0 && go == 0.0 && cmu[0] == 0.f &&
        cmu[1] == 0.f && cmu[2] == 0.f)
      continue;
    const ViewArgs& c = vt.v[v];
    const double fx = c.fx, fy = c.fy;
    const double t0 = (double)c.R[0] * mu[0] + (double)c.R[1] * mu[1] + (double)c.R[2] * mu[2] + (double)c.t[0];
    const double t1 = (double)c.R[3] * mu[0] + (double)c.R[4] * mu[1] + (double)c.R[5] * mu[2] + (double)c.t[1];
    const double t2 = (double)c.R[6] * mu[0] + (double)c.R[7] * mu[1] + (double)c.R[8] * mu[2] + (double)c.t[2];
    const double iz = 1.0 / t2;
    const double ux = t0 * iz, uy = t1 * iz;
    const double lx = c.limx, ly = c.limy;
    const bool inx = ux >= -lx && ux <= lx;
    const bool iny = uy >= -ly && uy <= ly;
    const double rx = fmin(fmax(ux, -lx), lx);
    const double ry = fmin(fmax(uy, -ly), ly);
    const double j00 = fx * iz, j02 = -fx * rx * iz, j11 = fy * iz, j12 = -fy * ry * iz;
    double Tm[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Tm[0][k] = j00 * (double)c.R[k] + j02 * (double)c.R[6 + k];
      Tm[1][k] = j11 * (double)c.R[3 + k] + j12 * (double)c.R[6 + k];
    }
    double TS[2][3];  // T Sigma
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      TS[rr][0] = Tm[rr][0] * Sig[0] + Tm[rr][1] * Sig[1] + Tm[rr][2] * Sig[2];
      TS[rr][1] = Tm[rr][0] * Sig[1] + Tm[rr][1] * Sig[3] + Tm[rr][2] * Sig[4];
      TS[rr][2] = Tm[rr][0] * Sig[2] + Tm[rr][1] * Sig[4] + Tm[rr][2] * Sig[5];
    }
    const double ca = TS[0][0] * Tm[0][0] + TS[0][1] * Tm[0][1] + TS[0][2] * Tm[0][2] + (double)c.lowpass;
    const double cb = TS[0][0] * Tm[1][0] + TS[0][1] * Tm[1][1] + TS[0][2] * Tm[1][2];
    const double cc = TS[1][0] * Tm[1][0] + TS[1][1] * Tm[1][1] + TS[1][2] * Tm[1][2] + (double)c.lowpass;
    const double idet = 1.0 / (ca * cc - cb * cb);
    const double QA = cc * idet, QB = -cb * idet, QC = ca * idet;
    // dL/dSigma' = -Q G_Q Q
    const double P00 = QA * gA + QB * 0.5 * gB, P01 = QA * 0.5 * gB + QB * gC;
    const double P10 = QB * gA + QC * 0.5 * gB, P11 = QB * 0.5 * gB + QC * gC;
    const double G00 = -(P00 * QA + P01 * QB);
    const double G01 = -(P00 * QB + P01 * QC);
    const double G11 = -(P10 * QB + P11 * QC);
    // dL/dT = 2 G T Sigma; T = J W with J00, J02, J11, J12 varying
    double gT[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gT[0][k] = 2.0 * (G00 * TS[0][k] + G01 * TS[1][k]);
      gT[1][k] = 2.0 * (G01 * TS[0][k] + G11 * TS[1][k]);
    }
    const double gj00 = gT[0][0] * c.R[0] + gT[0][1] * c.R[1] + gT[0][2] * c.R[2];
    const double gj02 = gT[0][0] * c.R[6] + gT[0][1] * c.R[7] + gT[0][2] * c.R[8];
    const double gj11 = gT[1][0] * c.R[3] + gT[1][1] * c.R[4] + gT[1][2] * c.R[5];
    const double gj12 = gT[1][0] * c.R[6] + gT[1][1] * c.R[7] + gT[1][2] * c.R[8];
    const double iz2 = iz * iz;
    double gt0 = gu * fx * iz, gt1 = gv * fy * iz;
    double gt2 = -gu * fx * t0 * iz2 - gv * fy * t1 * iz2;
    gt2 += -gj00 * fx * iz2 - gj11 * fy * iz2;
    // J02 = -fx rx / z, rx = clamp(x / z): d/dx = -fx/z^2 (unclamped); d/dz = fx rx/z^2 (+ fx x/z^3 unclamped)
    gt2 += gj02 * fx * rx * iz2 + gj12 * fy * ry * iz2;
    if (inx) {
      gt0 += -gj02 * fx * iz2;
      gt2 += gj02 * fx * t0 * iz2 * iz;
    }
    if (iny) {
      gt1 += -gj12 * fy * iz2;
      gt2 += gj12 * fy * t1 * iz2 * iz;
    }
    // dL/dSigma = T^T G T (symmetric), then dL/dM = (G + G^T) M = 2 G M
    double gS[3][3];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        gS[rr][k] = Tm[0][rr] * (G00 * Tm[0][k] + G01 * Tm[1][k]) + Tm[1][rr] * (G01 * Tm[0][k] + G11 * Tm[1][k]);
    double gsc[3], gR[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double acc[3];
#pragma unroll
      for (int rr = 0; rr < 3; ++rr)
        acc[rr] = (gS[rr][0] + gS[0][rr]) * Rq[0][k] * s[k] + (gS[rr][1] + gS[1][rr]) * Rq[1][k] * s[k] +
                  (gS[rr][2] + gS[2][rr]) * Rq[2][k] * s[k];
      gsc[k] = acc[0] * Rq[0][k] + acc[1] * Rq[1][k] + acc[2] * Rq[2][k];
      gR[0][k] = acc[0] * s[k];
      gR[1][k] = acc[1] * s[k];
      gR[2][k] = acc[2] * s[k];
    }
    const double gw = 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
    const double gx = 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.0 * x * gR[1][1] - w * gR[1][2] +
                             z * gR[2][0] + w * gR[2][1] - 2.0 * x * gR[2][2]);
    const double gy = 2.0 * (-2.0 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] -
                             w * gR[2][0] + z * gR[2][1] - 2.0 * y * gR[2][2]);
    const double gz = 2.0 * (-2.0 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2.0 * z * gR[1][1] +
                             y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
    const double qd = w * gw + x * gx + y * gy + z * gz;
    // this view's contribution, rounded to float, added in view order
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double gmu = (double)c.R[k] * gt0 + (double)c.R[3 + k] * gt1 + (double)c.R[6 + k] * gt2;
      tmu[k] = acc_add(tmu[k], (float)(gmu + (double)cmu[k]));
      tls[k] = acc_add(tls[k], (float)(gsc[k] * s[k]));
    }
    tq[0] = acc_add(tq[0], (float)((gw - w * qd) * iq));
    tq[1] = acc_add(tq[1], (float)((gx - x * qd) * iq));
    tq[2] = acc_add(tq[2], (float)((gy - y * qd) * iq));
    tq[3] = acc_add(tq[3], (float)((gz - z * qd) * iq));
    top = acc_add(top, (float)(go * op * (1.0 - op)));
    if (a.mask_logits)  // o' = M o, s' = M s (M = 1 here): dL/dM = o dL/do' + sum_k s_k dL/ds'_k
      tmask = acc_add(tmask, (float)((go * op + gsc[0] * s[0] + gsc[1] * s[1] + gsc[2] * s[2]) * sm * (1.0 - sm)));
  }

  geom_grads_out(b, n, i, tmu, tls, tq, top, tmask);
}

hipError_t launch_project_bwd(const ProjectBwdArgs& a, const ViewTable& vt, int deg, hipStream_t s) {
  if (a.p.n == 0) return hipSuccess;
  const dim3 block(256), grid((unsigned)((a.p.n + 255) / 256));
  const int64_t nrec = (int64_t)vt.nviews * a.p.n;
  hipLaunchKernelGGL(heavy_sums_kernel, dim3((unsigned)((nrec + 255) / 256)), block, 0, s, a, nrec);
  const bool rest = a.g_sh_rest != nullptr && deg > 0;
  switch (deg) {
    case 0: hipLaunchKernelGGL((project_bwd_color_kernel<0, false>), grid, block, 0, s, a, vt); break;
    case 1:
      if (rest) hipLaunchKernelGGL((project_bwd_color_kernel<1, true>), grid, block, 0, s, a, vt);
      else hipLaunchKernelGGL((project_bwd_color_kernel<1, false>), grid, block, 0, s, a, vt);
      break;
    case 2:
      if (rest) hipLaunchKernelGGL((project_bwd_color_kernel<2, true>), grid, block, 0, s, a, vt);
      else hipLaunchKernelGGL((project_bwd_color_kernel<2, false>), grid, block, 0, s, a, vt);
      break;
    default:
      if (rest) hipLaunchKernelGGL((project_bwd_color_kernel<3, true>), grid, block, 0, s, a, vt);
      else hipLaunchKernelGGL((project_bwd_color_kernel<3, false>), grid, block, 0, s, a, vt);
      break;
  }
  hipLaunchKernelGGL(project_bwd_geom_kernel, grid, block, 0, s, a, vt);
  return hipGetLastError();
}

}  // namespace gs
