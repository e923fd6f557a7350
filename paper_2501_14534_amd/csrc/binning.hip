// Tile binning and (tile, depth) ordering of projected records.
//
//   1. count_reduce + scan_top: device-wide exclusive scan of tiles_touched
//      (1024 records per block); the top level also writes K and the
//      capacity status.
//   2. emit_keys: each block rescans its 1024 counts, then its threads fill
//      the block's contiguous output range slot by slot (binary search of the
//      owning record in LDS), so writes are coalesced and big Gaussians do not
//      serialise a lane.  Keys come out in record order.
//   3. LSD radix sort, 8-bit digits, over the significant key bits only
//      (32 depth bits + ceil(log2 #tiles) tile bits).  Each pass: per-block
//      digit histogram, per-digit scan across blocks, stable scatter ranked
//      with 64-lane ballots.  Stability keeps record order among equal keys.
//   4. tile_ranges: [start, end) of every tile from run boundaries.
// Every kernel reads K from device memory, so nothing waits for the host.
#include "gs_common.h"
#include "kernels.h"

namespace gs {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;  // records per scan block
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per sort block
constexpr int kRadix = 256;

__device__ __forceinline__ uint32_t effective_count(const uint32_t* count, const int32_t* status) {
  return *status != 0 ? 0u : *count;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_exclusive_scan_256(uint32_t x, uint32_t* total, uint32_t* s_wave) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    const uint32_t c = s_wave[w];
    off += (w < wave) ? c : 0u;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return incl - x + off;
}

__global__ __launch_bounds__(kScanThreads) void count_reduce(const uint32_t* __restrict__ tt, int64_t len,
                                                             uint32_t* __restrict__ block_sums) {
  __shared__ uint32_t s_wave[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < len) s += tt[base + k];
  uint32_t tot;
  block_exclusive_scan_256(s, &tot, s_wave);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of nb block sums; total K in 64 bits.
__global__ __launch_bounds__(1024) void scan_top(const uint32_t* __restrict__ sums, int64_t nb,
                                                 uint32_t* __restrict__ offsets, uint64_t capacity,
                                                 uint32_t* count, int32_t* status) {
  __shared__ uint32_t s_wave[16];
  __shared__ unsigned long long s_carry;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const uint32_t x = i < nb ? sums[i] : 0u;
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    unsigned long long off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      const unsigned long long c = s_wave[w];
      off += (w < wave) ? c : 0ull;
      tot += c;
    }
    const unsigned long long carry = s_carry;
    if (i < nb) offsets[i] = (uint32_t)(carry + off + incl - x);
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && count) {
    const unsigned long long K = s_carry;
    *count = K > 0xffffffffull ? 0xffffffffu : (uint32_t)K;
    *status = K > (unsigned long long)capacity ? 1 : 0;
  }
}

// Emission: pair e of record r (e in [offsets[r], offsets[r] + tiles_touched[r]),
// the record's tiles in row-major order) gets key (tile << 32 | depth bits),
// value e, and owner[e] = r.
__global__ __launch_bounds__(kScanThreads) void emit_keys(const float4* __restrict__ splats,
                                                          const uint32_t* __restrict__ tt, int64_t nrec, int64_t n,
                                                          const uint32_t* __restrict__ block_offsets,
                                                          const int32_t* __restrict__ status, ViewTable vt,
                                                          float inv_tw, float inv_th, uint64_t* __restrict__ keys,
                                                          uint32_t* __restrict__ vals, uint32_t* __restrict__ owner,
                                                          uint32_t* __restrict__ offsets) {
  __shared__ uint32_t s_wave[kScanThreads / kWave];
  __shared__ uint32_t s_pref[kScanTile];
  __shared__ uint32_t s_base[kScanTile];
  __shared__ uint32_t s_w[kScanTile];
  __shared__ uint32_t s_tx[kScanTile];
  __shared__ uint32_t s_depth[kScanTile];
  if (*status != 0) return;
  const int64_t blk = (int64_t)blockIdx.x * kScanTile;
  const int li0 = threadIdx.x * kScanItems;
  uint32_t c[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t r = blk + li0 + k;
    c[k] = r < nrec ? tt[r] : 0u;
    s += c[k];
  }
  uint32_t total;
  uint32_t ex = block_exclusive_scan_256(s, &total, s_wave);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int li = li0 + k;
    s_pref[li] = ex;
    if (c[k]) {
      const int64_t r = blk + li;
      const int v = (int)(r / n);
      const ViewArgs& va = vt.v[v];
      const float4 p0 = splats[r * 3 + 0];
      const float4 p1 = splats[r * 3 + 1];
      int x0, y0, x1, y1;
      tile_rect(p0.x, p0.y, p1.z, inv_tw, inv_th, va.TX, va.TY, &x0, &y0, &x1, &y1);
      s_base[li] = (uint32_t)(va.tile_off + y0 * va.TX + x0);
      s_w[li] = (uint32_t)(x1 - x0 + 1);
      s_tx[li] = (uint32_t)va.TX;
      s_depth[li] = __float_as_uint(p1.w);
    }
    ex += c[k];
  }
  __syncthreads();
  const uint32_t out0 = block_offsets[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t r = blk + li0 + k;
    if (r < nrec) offsets[r] = out0 + s_pref[li0 + k];
  }
  for (uint32_t slot = threadIdx.x; slot < total; slot += kScanThreads) {
    // last record whose exclusive prefix is <= slot
    int lo = 0, hi = kScanTile;  // invariant: s_pref[lo] <= slot < s_pref[hi] (virtual s_pref[kScanTile] = total)
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_pref[mid] <= slot) lo = mid; else hi = mid;
    }
    const uint32_t j = slot - s_pref[lo];
    const uint32_t w = s_w[lo];
    const uint32_t ty = j / w, tx = j - ty * w;
    const uint32_t gt = s_base[lo] + ty * s_tx[lo] + tx;
    const uint32_t e = out0 + slot;
    keys[e] = ((uint64_t)gt << 32) | s_depth[lo];
    vals[e] = e;
    owner[e] = (uint32_t)(blk + lo);
  }
}

__global__ __launch_bounds__(kSortThreads) void radix_hist(const uint64_t* __restrict__ keys,
                                                           const uint32_t* __restrict__ count,
                                                           const int32_t* __restrict__ status, int shift, int64_t nblk,
                                                           uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kRadix];
  const uint32_t K = effective_count(count, status);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base < K) {
#pragma unroll 4
    for (int k = 0; k < kSortItems; ++k) {
      const int64_t i = base + k * kSortThreads + threadIdx.x;
      if (i < K) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (kRadix - 1)], 1u);
    }
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// One block per digit: exclusive scan of that digit's counts over the sort
// blocks (in place) and the digit's total.
__global__ __launch_bounds__(256) void radix_digit_scan(uint32_t* __restrict__ hist, int64_t nblk,
                                                        uint32_t* __restrict__ digit_total) {
  __shared__ uint32_t s_wave[4];
  __shared__ uint32_t s_carry;
  uint32_t* row = hist + (int64_t)blockIdx.x * nblk;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nblk; base += 256) {
    const int64_t i = base + threadIdx.x;
    const uint32_t x = i < nblk ? row[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan_256(x, &tot, s_wave);
    const uint32_t carry = s_carry;
    if (i < nblk) row[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) digit_total[blockIdx.x] = s_carry;
}

// Lanes of the wave holding the same 8-bit digit (among valid lanes).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter(const uint64_t* __restrict__ kin,
                                                              const uint32_t* __restrict__ vin,
                                                              uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                              const uint32_t* __restrict__ count,
                                                              const int32_t* __restrict__ status, int shift,
                                                              int64_t nblk, const uint32_t* __restrict__ hist,
                                                              const uint32_t* __restrict__ digit_total) {
  constexpr int kWaves = kSortThreads / kWave;
  __shared__ uint32_t s_run[kRadix];
  __shared__ uint32_t s_cnt[kWaves][kRadix];
  __shared__ uint32_t s_pre[kWaves][kRadix];
  __shared__ uint32_t s_wave[kWaves];
  const uint32_t K = effective_count(count, status);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= K) return;  // uniform across the block
  const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
  // digit bases: exclusive scan of the digit totals
  uint32_t tot;
  const uint32_t dbase = block_exclusive_scan_256(digit_total[t], &tot, s_wave);
  s_run[t] = dbase + hist[(int64_t)t * nblk + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s_cnt[w][t] = 0;
  uint64_t key[kSortItems];
  uint32_t val[kSortItems];
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t i = base + k * kSortThreads + t;
    if (i < K) {
      key[k] = kin[i];
      val[k] = vin[i];
    }
  }
  __syncthreads();
  const uint64_t lt_mask = (1ull << lane) - 1ull;
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t i = base + k * kSortThreads + t;
    const bool valid = i < K;
    const uint32_t d = valid ? (uint32_t)(key[k] >> shift) & (kRadix - 1) : 0u;
    const uint64_t peers = match_digit(d, valid);
    const uint32_t rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) s_cnt[wave][d] = __popcll(peers);
    __syncthreads();
    {
      uint32_t r = s_run[t];
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        s_pre[w][t] = r;
        r += s_cnt[w][t];
        s_cnt[w][t] = 0;
      }
      s_run[t] = r;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = s_pre[wave][d] + rank;
      kout[pos] = key[k];
      vout[pos] = val[k];
    }
  }
}

// Per sorted pair: record id from its emission position, and the tile's run boundaries.
__global__ void tile_ranges(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ pair_index,
                            const uint32_t* __restrict__ owner, const uint32_t* __restrict__ count,
                            const int32_t* __restrict__ status, uint32_t* __restrict__ ids,
                            uint32_t* __restrict__ ranges) {
  const uint32_t K = effective_count(count, status);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  ids[i] = owner[pair_index[i]];
  const uint32_t t = (uint32_t)(keys[i] >> 32);
  if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ranges[2 * (int64_t)t] = (uint32_t)i;
  if (i == (int64_t)K - 1 || (uint32_t)(keys[i + 1] >> 32) != t) ranges[2 * (int64_t)t + 1] = (uint32_t)(i + 1);
}

__global__ void fill_u32(uint32_t* p, int64_t count, uint32_t value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct SortWs {
  uint32_t* block_sums;
  uint32_t* block_offsets;
  uint64_t* keys_alt;
  uint32_t* vals_alt;
  uint32_t* owner;
  uint32_t* hist;
  uint32_t* digit_total;
  size_t bytes;
};

static SortWs carve(const SortPlan& p, uint64_t capacity, void* ws) {
  SortWs w{};
  char* b = (char*)ws;
  size_t o = 0;
  w.block_sums = (uint32_t*)(b + o), o += align256(sizeof(uint32_t) * (size_t)p.scan_blocks);
  w.block_offsets = (uint32_t*)(b + o), o += align256(sizeof(uint32_t) * (size_t)p.scan_blocks);
  w.keys_alt = (uint64_t*)(b + o), o += align256(sizeof(uint64_t) * (size_t)capacity);
  w.vals_alt = (uint32_t*)(b + o), o += align256(sizeof(uint32_t) * (size_t)capacity);
  w.owner = (uint32_t*)(b + o), o += align256(sizeof(uint32_t) * (size_t)capacity);
  w.hist = (uint32_t*)(b + o), o += align256(sizeof(uint32_t) * kRadix * (size_t)p.sort_blocks);
  w.digit_total = (uint32_t*)(b + o), o += align256(sizeof(uint32_t) * kRadix);
  w.bytes = o;
  return w;
}

size_t bin_sort_ws_bytes(const SortPlan& p) {
  return carve(p, (uint64_t)p.sort_blocks * kSortTile, nullptr).bytes;
}

hipError_t launch_bin_sort(const SortPlan& plan, const float4* splats, const uint32_t* tiles_touched, int64_t n,
                           const ViewTable& vt, float inv_tw, float inv_th, const BinOut& out, uint64_t capacity,
                           void* ws, hipStream_t s) {
  const SortWs w = carve(plan, (uint64_t)plan.sort_blocks * kSortTile, ws);
  hipError_t e;
  if ((e = launch_fill_u32(out.ranges, 2 * (int64_t)vt.total_tiles, 0u, s)) != hipSuccess) return e;
  const int64_t nb = plan.scan_blocks;
  if (nb > 0) {
    hipLaunchKernelGGL(count_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, tiles_touched, plan.nrec,
                       w.block_sums);
  }
  hipLaunchKernelGGL(scan_top, dim3(1), dim3(1024), 0, s, w.block_sums, nb, w.block_offsets, capacity, out.count,
                     out.status);
  // ping-pong so that the last pass lands in (keys, pair_index)
  uint64_t* kbuf[2] = {out.keys, w.keys_alt};
  uint32_t* vbuf[2] = {out.pair_index, w.vals_alt};
  int cur = (plan.passes % 2 == 0) ? 0 : 1;
  uint32_t* count = out.count;
  int32_t* status = out.status;
  if (nb > 0) {
    hipLaunchKernelGGL(emit_keys, dim3((unsigned)nb), dim3(kScanThreads), 0, s, splats, tiles_touched, plan.nrec, n,
                       w.block_offsets, status, vt, inv_tw, inv_th, kbuf[cur], vbuf[cur], w.owner, out.offsets);
  }
  const int64_t sb = plan.sort_blocks;
  for (int p = 0; p < plan.passes && sb > 0; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(radix_hist, dim3((unsigned)sb), dim3(kSortThreads), 0, s, kbuf[cur], count, status, shift, sb,
                       w.hist);
    hipLaunchKernelGGL(radix_digit_scan, dim3(kRadix), dim3(256), 0, s, w.hist, sb, w.digit_total);
    hipLaunchKernelGGL(radix_scatter, dim3((unsigned)sb), dim3(kSortThreads), 0, s, kbuf[cur], vbuf[cur],
                       kbuf[cur ^ 1], vbuf[cur ^ 1], count, status, shift, sb, w.hist, w.digit_total);
    cur ^= 1;
  }
  const int64_t cap_blocks = ((int64_t)capacity + 255) / 256;
  if (cap_blocks > 0)
    hipLaunchKernelGGL(tile_ranges, dim3((unsigned)cap_blocks), dim3(256), 0, s, out.keys, out.pair_index, w.owner,
                       count, status, out.ids, out.ranges);
  return hipGetLastError();
}

}  // namespace gs
