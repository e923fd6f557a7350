// Significance score of Eq. 4, after the ray hits are counted by the
// counting variant of the forward walk (render.hip):
//
//   GS_j = hits_j * o'_j * min(vol_j / v_q, 1)
//
// o'_j = sigmoid(opacity logit) times the hard volume mask (Eq. 3); vol_j =
// the product of the three scales; v_q the volume at ascending rank ceil(q n)
// over all n Gaussians (Sec. 3.2.2 normalises by the volume of the largest
// Gaussians).  Volumes are handled as log-volumes lv = sum of the log-scales
// (monotone, no overflow), so gamma = exp(min(lv - lv_q, 0)).
//
// v_q is found by an exact radix select on the order-preserving 32-bit image
// of lv, 8 bits per pass: each pass histograms the digit of the keys that
// still match the prefix chosen so far (LDS histograms, then one global add
// per non-empty bin), and one small workgroup picks the digit holding the
// wanted rank.  Four passes, no host round trip, integer counts only: the
// selected key is exact and the result reproducible.
#include "gs_common.h"
#include "kernels.h"

namespace gs {

// Order-preserving map of a float to uint32 (negative values reversed); NaN
// goes last.
__device__ __forceinline__ uint32_t order_key(float x) {
  if (x != x) return 0xffffffffu;
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// The same sum in both kernels, so that the selected Gaussian gets gamma = 1.
__device__ __forceinline__ float log_volume(const float* ls, int64_t n, int64_t i) {
  return (ls[i] + ls[n + i]) + ls[2 * n + i];
}

__global__ __launch_bounds__(256) void select_init_kernel(SelectState* st, uint32_t rank) {
  st->hist[threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    st->prefix = 0u;
    st->rank = rank;
  }
}

__global__ __launch_bounds__(256) void select_hist_kernel(const float* __restrict__ ls, int64_t n, int shift,
                                                          SelectState* st) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  // keys whose bits above this digit equal the prefix chosen so far
  const uint32_t prefix = st->prefix;
  const uint32_t high = shift == 24 ? 0u : (0xffffffffu << (shift + 8));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = order_key(log_volume(ls, n, i));
    if (((k ^ prefix) & high) == 0u) atomicAdd(&h[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  const uint32_t c = h[threadIdx.x];
  if (c != 0u) atomicAdd(&st->hist[threadIdx.x], c);
}

// One wave: the digit d where the running count passes the remaining rank.
__global__ __launch_bounds__(64) void select_pick_kernel(int shift, SelectState* st) {
  const int lane = threadIdx.x;
  uint32_t c[4], s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c[k] = st->hist[lane * 4 + k];
    s += c[k];
  }
  // inclusive scan of the lanes' sums (ascending digit order)
  uint32_t inc = s;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(inc, o);
    if (lane >= o) inc += v;
  }
  const uint32_t rank = st->rank;
  uint32_t before = inc - s;
  int found = -1;
  uint32_t below = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (found < 0 && rank >= before && rank < before + c[k]) {
      found = lane * 4 + k;
      below = before;
    }
    before += c[k];
  }
  __syncthreads();  // every lane has read the histogram
#pragma unroll
  for (int k = 0; k < 4; ++k) st->hist[lane * 4 + k] = 0u;  // ready for the next pass
  if (found >= 0) {  // exactly one lane
    st->prefix |= (uint32_t)found << shift;
    st->rank = rank - below;
  }
}

__global__ __launch_bounds__(256) void significance_kernel(const float* __restrict__ ls,
                                                           const float* __restrict__ opacity_logits,
                                                           const float* __restrict__ mask_logits, float mask_thr,
                                                           const uint32_t* __restrict__ hits, int64_t n,
                                                           const SelectState* st, float* __restrict__ score) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t h = hits[i];
  float s = 0.0f;
  if (h != 0u) {
    const float lvq = key_value(st->prefix);
    const float g = __expf(fminf(log_volume(ls, n, i) - lvq, 0.0f));
    float op = sigmoidf(opacity_logits[i]);
    if (mask_logits && !(mask_logits[i] > mask_thr)) op = 0.0f;
    s = (float)h * op * g;
  }
  score[i] = s;
}

hipError_t launch_significance(const float* log_scales, const float* opacity_logits, const float* mask_logits,
                               float mask_thr, const uint32_t* hits, int64_t n, uint32_t rank, SelectState* st,
                               float* score, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, s, st, rank);
  const int64_t want = (n + 255) / 256;
  const unsigned nb = (unsigned)(want < 2048 ? want : 2048);
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(select_hist_kernel, dim3(nb), dim3(256), 0, s, log_scales, n, shift, st);
    hipLaunchKernelGGL(select_pick_kernel, dim3(1), dim3(64), 0, s, shift, st);
  }
  hipLaunchKernelGGL(significance_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, log_scales,
                     opacity_logits, mask_logits, mask_thr, hits, n, st, score);
  return hipGetLastError();
}

}  // namespace gs
