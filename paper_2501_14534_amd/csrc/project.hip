// Projection of 3D Gaussians into V views (forward).
//
// One thread per Gaussian reads its raw parameters once (coalesced SoA loads,
// band-0 colour separate from bands 1..3 as in Sec. 3.2.5) and writes one
// 48-byte splat record per view.  Bound by HBM traffic: ~252 bytes read per
// Gaussian at degree 3 with masks, 48 + 4 bytes written per (view, Gaussian).
#include "gs_common.h"
#include "kernels.h"

namespace gs {

template <int DEG>
__global__ __launch_bounds__(256) void project_kernel(ProjectArgs a, ViewTable vt) {
  const int64_t n = a.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int V = vt.nviews;
  float4* out = a.splats;

  // Hard masks (Eq. 3, Eq. 5): sigmoid(m) > eps  <=>  m > logit(eps); the
  // threshold logit is precomputed on the host (rounded down to float so the
  // comparison is exact for every float m).
  bool ok = true;
  if (a.mask_logits) {
    const float m = a.mask_logits[i];
    ok = finitef(m) && m > a.mask_thr;
  }
  float mu[3], ls[3], q[4], ol = 0.f, dc[3];
  if (ok) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      mu[k] = a.means[k * n + i];
      ls[k] = a.log_scales[k * n + i];
      dc[k] = a.sh_dc[k * n + i];
      ok = ok && finitef(mu[k]) && finitef(ls[k]) && finitef(dc[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      q[k] = a.quats[k * n + i];
      ok = ok && finitef(q[k]);
    }
    ol = a.opacity_logits[i];
    ok = ok && finitef(ol);
  }
  // SH bands 1..DEG, only the bands whose hard mask is on are read.
  float rest[DEG > 0 ? (DEG + 1) * (DEG + 1) - 1 : 1][3];
  bool band_on[4] = {true, true, true, true};
  if (ok && DEG > 0) {
    if (a.sh_mask_logits) {
#pragma unroll
      for (int l = 1; l <= 3; ++l) {
        const float m = a.sh_mask_logits[(l - 1) * n + i];
        ok = ok && finitef(m);
        band_on[l] = m > a.sh_mask_thr;
      }
    }
    // flat loops with constant trip counts, so the coefficients stay in registers
#pragma unroll
    for (int k = 1; k < kShCoeffs; ++k) {
      const int l = sh_band(k);
      if (l > DEG) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float x = 0.f;
        if (band_on[l]) {
          x = a.sh_rest[((k - 1) * 3 + c) * n + i];
          ok = ok && finitef(x);
        }
        rest[k - 1][c] = x;
      }
    }
  }

  // 3D covariance Sigma = Rq diag(s^2) Rq^T (upper triangle), opacity.
  float S00 = 0.f, S01 = 0.f, S02 = 0.f, S11 = 0.f, S12 = 0.f, S22 = 0.f, op = 0.f;
  if (ok) {
    const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    ok = qn > 0.f && finitef(qn);
    if (ok) {
      const float iq = 1.0f / qn;
      const float w = q[0] * iq, x = q[1] * iq, y = q[2] * iq, z = q[3] * iq;
      const float R00 = 1.f - 2.f * (y * y + z * z), R01 = 2.f * (x * y - w * z), R02 = 2.f * (x * z + w * y);
      const float R10 = 2.f * (x * y + w * z), R11 = 1.f - 2.f * (x * x + z * z), R12 = 2.f * (y * z - w * x);
      const float R20 = 2.f * (x * z - w * y), R21 = 2.f * (y * z + w * x), R22 = 1.f - 2.f * (x * x + y * y);
      const float s0 = __expf(2.f * ls[0]), s1 = __expf(2.f * ls[1]), s2 = __expf(2.f * ls[2]);  // squared scales
      S00 = R00 * R00 * s0 + R01 * R01 * s1 + R02 * R02 * s2;
      S01 = R00 * R10 * s0 + R01 * R11 * s1 + R02 * R12 * s2;
      S02 = R00 * R20 * s0 + R01 * R21 * s1 + R02 * R22 * s2;
      S11 = R10 * R10 * s0 + R11 * R11 * s1 + R12 * R12 * s2;
      S12 = R10 * R20 * s0 + R11 * R21 * s1 + R12 * R22 * s2;
      S22 = R20 * R20 * s0 + R21 * R21 * s1 + R22 * R22 * s2;
      op = sigmoidf(ol);
    }
  }

  for (int v = 0; v < V; ++v) {
    const ViewArgs& c = vt.v[v];
    const int64_t rec = (int64_t)v * n + i;
    float4 o0 = make_float4(0.f, 0.f, 0.f, 0.f), o1 = o0, o2 = o0;
    uint32_t touched = 0;
    bool vis = ok;
    float t0 = 0.f, t1 = 0.f, t2 = 0.f;
    if (vis) {
      t0 = c.R[0] * mu[0] + c.R[1] * mu[1] + c.R[2] * mu[2] + c.t[0];
      t1 = c.R[3] * mu[0] + c.R[4] * mu[1] + c.R[5] * mu[2] + c.t[1];
      t2 = c.R[6] * mu[0] + c.R[7] * mu[1] + c.R[8] * mu[2] + c.t[2];
      vis = t2 > a.near_plane;
    }
    if (vis) {
      // EWA: J = [[fx/z, 0, -fx rx/z], [0, fy/z, -fy ry/z]], rx = clamp(x/z) (Eq. 1).
      const float iz = 1.0f / t2;
      const float rx = fminf(fmaxf(t0 * iz, -c.limx), c.limx);
      const float ry = fminf(fmaxf(t1 * iz, -c.limy), c.limy);
      const float j00 = c.fx * iz, j02 = -c.fx * rx * iz, j11 = c.fy * iz, j12 = -c.fy * ry * iz;
      // T = J W (2x3)
      const float a0 = j00 * c.R[0] + j02 * c.R[6], a1 = j00 * c.R[1] + j02 * c.R[7], a2 = j00 * c.R[2] + j02 * c.R[8];
      const float b0 = j11 * c.R[3] + j12 * c.R[6], b1 = j11 * c.R[4] + j12 * c.R[7], b2 = j11 * c.R[5] + j12 * c.R[8];
      // Sigma T^T columns
      const float sa0 = S00 * a0 + S01 * a1 + S02 * a2, sa1 = S01 * a0 + S11 * a1 + S12 * a2,
                  sa2 = S02 * a0 + S12 * a1 + S22 * a2;
      const float sb0 = S00 * b0 + S01 * b1 + S02 * b2, sb1 = S01 * b0 + S11 * b1 + S12 * b2,
                  sb2 = S02 * b0 + S12 * b1 + S22 * b2;
      // Sigma' + sI (Sec. 3.2.4)
      const float ca = a0 * sa0 + a1 * sa1 + a2 * sa2 + c.lowpass;
      const float cb = a0 * sb0 + a1 * sb1 + a2 * sb2;
      const float cc = b0 * sb0 + b1 * sb1 + b2 * sb2 + c.lowpass;
      const float det = ca * cc - cb * cb;
      vis = det > 0.f;
      if (vis) {
        const float idet = 1.0f / det;
        const float mid = 0.5f * (ca + cc);
        const float lam = mid + sqrtf(fmaxf(0.f, mid * mid - det));
        const float rad = ceilf(3.0f * sqrtf(lam));
        const float u = c.fx * t0 * iz + c.cx;
        const float vv = c.fy * t1 * iz + c.cy;
        // colour: diffuse + masked SH bands at the unit view direction, clamped at 0
        float rgb[3] = {dc[0], dc[1], dc[2]};
        if (DEG > 0) {
          float d0 = mu[0] - c.campos[0], d1 = mu[1] - c.campos[1], d2 = mu[2] - c.campos[2];
          const float il = 1.0f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
          d0 *= il, d1 *= il, d2 *= il;
          float Y[15];
          sh_basis15(d0, d1, d2, Y);
#pragma unroll
          for (int k = 1; k < kShCoeffs; ++k) {
            const int l = sh_band(k);
            if (l > DEG || !band_on[l]) continue;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) rgb[ch] += Y[k - 1] * rest[k - 1][ch];
          }
        }
        o0 = make_float4(u, vv, cc * idet, -cb * idet);
        o1 = make_float4(ca * idet, op, rad, t2);
        o2 = make_float4(fmaxf(rgb[0], 0.f), fmaxf(rgb[1], 0.f), fmaxf(rgb[2], 0.f), 1.0f);
        int x0, y0, x1, y1;
        if (tile_rect(u, vv, rad, a.inv_tw, a.inv_th, c.TX, c.TY, &x0, &y0, &x1, &y1))
          touched = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
      }
    }
    out[rec * 3 + 0] = o0;
    out[rec * 3 + 1] = o1;
    out[rec * 3 + 2] = o2;
    a.tiles_touched[rec] = touched;
  }
}

hipError_t launch_project(const ProjectArgs& a, const ViewTable& vt, int deg, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const dim3 block(256), grid((unsigned)((a.n + 255) / 256));
  switch (deg) {
    case 0: hipLaunchKernelGGL(project_kernel<0>, grid, block, 0, s, a, vt); break;
    case 1: hipLaunchKernelGGL(project_kernel<1>, grid, block, 0, s, a, vt); break;
    case 2: hipLaunchKernelGGL(project_kernel<2>, grid, block, 0, s, a, vt); break;
    default: hipLaunchKernelGGL(project_kernel<3>, grid, block, 0, s, a, vt); break;
  }
  return hipGetLastError();
}

}  // namespace gs
