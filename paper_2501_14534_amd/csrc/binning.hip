// Tile binning and (tile, depth) ordering of projected records, depth first.
//
//   1. count_reduce + scan_top: device-wide exclusive scans of tiles_touched
//      (the canonical emission offsets, K and the capacity status) and of
//      the visibility flags (tiles_touched > 0), 1024 records per block.
//   2. compact_visible: writes each record's canonical offset and packs each
//      visible record as (depth bits, compact index) plus a 16-byte emission
//      descriptor (first tile, rect width and height, canonical offset, id).
//   3. LSD radix sort of the visible records by their 32 depth bits (four
//      8-bit passes; stable, so equal depths keep record order).
//   4. gather_reduce gathers the descriptors into depth order once (the only
//      random access of the emission) and sums the pairs per block;
//      emit_prefix: each depth-sorted record's first output position;
//      emit_pairs: the records, now in depth order, emit one (tile, canonical
//      pair index, record id) per touched tile into a contiguous
//      depth-ordered range; each workgroup fills a fixed chunk of output
//      positions slot by slot (binary search of the owning record in LDS), so
//      writes are coalesced and neither a big Gaussian nor a block of them
//      serialises the work.
//   5. LSD radix sort of the pairs by tile id only (ceil(log2 #tiles) bits,
//      two passes up to 65536 tiles), carrying pair index and record id.
//      Stability keeps depth order, and record order among equal depths,
//      inside every tile: the order of a sort by (tile << 32 | depth bits)
//      then record id.
//   6. tile_ranges: [start, end) of every tile and, if asked for, the 64-bit keys.
//   7. tile_order_*: the heaviest-first tile schedule.
// The sort passes move 8 bytes per element: 4 passes over the visible
// records plus 2 over the pairs, instead of 6 passes of 12 bytes over the
// pairs.  Each pass: per-block digit histogram, per-digit scan across blocks,
// stable scatter ranked with 64-lane ballots.  Every kernel reads its
// element count from device memory, so nothing waits for the host.
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

// Data block of workgroup p among the first `nact` workgroups: workgroups are
// dealt round-robin to the 8 XCDs, so p % 8 is p's XCD; the remap gives each
// XCD a contiguous stretch of data blocks.  Neighbouring blocks share the
// cache lines at the ends of their output runs (the scatter) and the lines
// of their histogram column (32 blocks per line), which are then completed in
// one L2 and written back whole.
__device__ __forceinline__ int64_t xcd_block(int64_t p, int64_t nact) {
  constexpr int kXcds = 8;
  const int64_t q = nact / kXcds;
  return p < q * kXcds ? (p % kXcds) * q + p / kXcds : p;
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

// Per block of 1024 records: sum of tiles_touched and number of visible records.
__global__ __launch_bounds__(kScanThreads) void count_reduce(const uint32_t* __restrict__ tt, int64_t len,
                                                             uint32_t* __restrict__ block_sums,
                                                             uint32_t* __restrict__ vis_sums) {
  __shared__ uint32_t s_wave[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t s = 0, v = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < len) {
      const uint32_t c = tt[base + k];
      s += c;
      v += c != 0u;
    }
  uint32_t tot;
  block_exclusive_scan_256(s, &tot, s_wave);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
  block_exclusive_scan_256(v, &tot, s_wave);
  if (threadIdx.x == 0) vis_sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of nb block sums and their total (64-bit
// accumulation, saturated to 32 bits).  With a status word: status = 1 when
// the total exceeds capacity.
__global__ __launch_bounds__(1024) void scan_top(const uint32_t* __restrict__ sums, int64_t nb,
                                                 uint32_t* __restrict__ offsets, uint64_t capacity,
                                                 uint32_t* total_out, int32_t* status) {
  constexpr int kItems = 8;  // consecutive sums per thread: 8192 per step, one step up to 8M records
  __shared__ uint32_t s_wave[16];
  __shared__ unsigned long long s_carry;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += kItems * 1024) {
    const int64_t i0 = base + (int64_t)kItems * threadIdx.x;
    uint32_t x[kItems], sum = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      x[j] = i0 + j < nb ? sums[i0 + j] : 0u;
      sum += x[j];
    }
    uint32_t incl = sum;
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
    unsigned long long ex = carry + off + incl - sum;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      if (i0 + j < nb) offsets[i0 + j] = (uint32_t)ex;
      ex += x[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const unsigned long long K = s_carry;
    *total_out = K > 0xffffffffull ? 0xffffffffu : (uint32_t)K;
    if (status) *status = K > (unsigned long long)capacity ? 1 : 0;
  }
}

// Exclusive scans of two values per thread over a 256-thread block (one pass
// of barriers for both).
__device__ __forceinline__ void block_exclusive_scan2_256(uint32_t x, uint32_t y, uint32_t* ex, uint32_t* ey,
                                                          uint32_t* tx, uint32_t* ty, uint2* s_wave) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t ix = x, iy = y;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t a = __shfl_up(ix, o, kWave), b = __shfl_up(iy, o, kWave);
    if (lane >= o) ix += a, iy += b;
  }
  if (lane == kWave - 1) s_wave[wave] = make_uint2(ix, iy);
  __syncthreads();
  uint32_t ox = 0, oy = 0, sx = 0, sy = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    const uint2 c = s_wave[w];
    ox += (w < wave) ? c.x : 0u;
    oy += (w < wave) ? c.y : 0u;
    sx += c.x;
    sy += c.y;
  }
  __syncthreads();
  *ex = ix - x + ox;
  *ey = iy - y + oy;
  *tx = sx;
  *ty = sy;
}

// Canonical emission offsets of every record (pairs of record r occupy
// [offsets[r], offsets[r] + tiles_touched[r]), records in index order), and
// the visible records packed in record order as (depth bits, compact index)
// with their emission descriptors; drec[r] = depth bits for the keys.  The
// block's 1024 records are taken in four slices of 256 consecutive records,
// one per thread, so loads and stores are coalesced.
__global__ __launch_bounds__(kScanThreads) void compact_visible(const float4* __restrict__ splats,
                                                                const uint32_t* __restrict__ tt, int64_t nrec,
                                                                int64_t n, ViewTable vt, float inv_tw, float inv_th,
                                                                const uint32_t* __restrict__ block_offsets,
                                                                const uint32_t* __restrict__ vis_offsets,
                                                                const int32_t* __restrict__ status,
                                                                uint32_t* __restrict__ offsets,
                                                                uint32_t* __restrict__ dkey,
                                                                uint32_t* __restrict__ dval, uint4* __restrict__ desc,
                                                                uint32_t* __restrict__ drec) {
  __shared__ uint2 s_wave[kScanThreads / kWave];
  if (*status != 0) return;  // overflow: no lists this step
  const int64_t blk = (int64_t)blockIdx.x * kScanTile;
  uint32_t ex_base = block_offsets[blockIdx.x], vx_base = vis_offsets[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t r = blk + k * kScanThreads + threadIdx.x;
    const uint32_t c = r < nrec ? tt[r] : 0u;
    uint32_t ex, vx, ts, tv;
    block_exclusive_scan2_256(c, c != 0u ? 1u : 0u, &ex, &vx, &ts, &tv, s_wave);
    ex += ex_base;
    vx += vx_base;
    ex_base += ts;
    vx_base += tv;
    if (r < nrec) offsets[r] = ex;
    if (c) {
      const float4 p0 = splats[r * 3 + 0];
      const float4 p1 = splats[r * 3 + 1];
      int v = 0;
      while (v + 1 < vt.nviews && r >= (int64_t)(v + 1) * n) ++v;
      const ViewArgs& va = vt.v[v];
      int x0, y0, x1, y1;
      tile_rect(p0.x, p0.y, p1.z, inv_tw, inv_th, va.TX, va.TY, &x0, &y0, &x1, &y1);
      const uint32_t dbits = __float_as_uint(p1.w);  // depth > near plane > 0: bits order as values
      dkey[vx] = dbits;
      dval[vx] = vx;
      desc[vx] = make_uint4((uint32_t)(va.tile_off + y0 * va.TX + x0),
                            (uint32_t)(x1 - x0 + 1) | ((uint32_t)(y1 - y0 + 1) << 16), ex, (uint32_t)r);
      if (drec) drec[r] = dbits;
    }
  }
}

// Per block of 1024 depth-sorted records: their descriptors gathered into
// depth order (sdesc, read sequentially by emit_pairs) and their number of
// pairs.
__global__ __launch_bounds__(kScanThreads) void gather_reduce(const uint4* __restrict__ desc,
                                                              const uint32_t* __restrict__ dval,
                                                              const uint32_t* __restrict__ nvis,
                                                              const int32_t* __restrict__ status,
                                                              uint4* __restrict__ sdesc,
                                                              uint32_t* __restrict__ block_sums) {
  __shared__ uint32_t s_wave[kScanThreads / kWave];
  const uint32_t N = effective_count(nvis, status);
  const int64_t blk = (int64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t m = blk + k * kScanThreads + threadIdx.x;
    if (m < N) {
      const uint4 d = desc[dval[m]];
      sdesc[m] = d;
      s += (d.y & 0xffffu) * (d.y >> 16);
    }
  }
  uint32_t tot;
  block_exclusive_scan_256(s, &tot, s_wave);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Output positions per emission workgroup.
constexpr int kEmitChunk = 1536;  // 5 staged words per record: 30 KB of LDS, 5 workgroups per CU

// Emission offsets in depth order: epref[m] = the first output position of
// depth-sorted record m (its block's offset plus the exclusive prefix of the
// pair counts within the block of 1024), and for every chunk of kEmitChunk
// output positions the record holding its first position (chunk_first).
__global__ __launch_bounds__(kScanThreads) void emit_prefix(const uint4* __restrict__ sdesc,
                                                            const uint32_t* __restrict__ nvis,
                                                            const uint32_t* __restrict__ eblock_offsets,
                                                            const int32_t* __restrict__ status,
                                                            uint32_t* __restrict__ epref,
                                                            uint32_t* __restrict__ chunk_first) {
  __shared__ uint32_t s_wave[kScanThreads / kWave];
  const uint32_t N = effective_count(nvis, status);
  const int64_t blk = (int64_t)blockIdx.x * kScanTile;
  if (blk >= N) return;  // uniform
  // thread t takes 4 consecutive records, so the block scan runs in record order
  const int64_t m0 = blk + (int64_t)threadIdx.x * kScanItems;
  uint32_t c[kScanItems], sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    c[k] = 0u;
    if (m0 + k < N) {
      const uint32_t wh = sdesc[m0 + k].y;
      c[k] = (wh & 0xffffu) * (wh >> 16);
    }
    sum += c[k];
  }
  uint32_t total;
  uint32_t ex = block_exclusive_scan_256(sum, &total, s_wave) + eblock_offsets[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (m0 + k < N) {
      epref[m0 + k] = ex;
      // chunks whose first position lies in [ex, ex + c)
      for (uint32_t q = (ex + kEmitChunk - 1) / kEmitChunk; q * (uint64_t)kEmitChunk < (uint64_t)ex + c[k]; ++q)
        chunk_first[q] = (uint32_t)(m0 + k);
    }
    ex += c[k];
  }
}

// Emission in depth order: sorted record m emits, at output positions
// [epref[m], epref[m] + w h), its tiles in row-major order of its tile
// rectangle: tile id, the pair's canonical index offsets[r] + j, and r.
// Workgroup c owns output positions [c C, (c + 1) C), C = kEmitChunk: it
// stages the descriptors of the records from the one holding its first
// position to the one holding the next chunk's (at most C + 1: every record
// has a pair) and fills its slots in order (binary search of the owning
// record in LDS).  Work per workgroup is bounded by C slots however many
// pairs one record has (the nearest Gaussians cover thousands of tiles), and
// consecutive threads write consecutive positions.
__global__ __launch_bounds__(kScanThreads) void emit_pairs(const uint4* __restrict__ sdesc,
                                                           const uint32_t* __restrict__ epref,
                                                           const uint32_t* __restrict__ chunk_first,
                                                           const uint32_t* __restrict__ nvis,
                                                           const uint32_t* __restrict__ count,
                                                           const int32_t* __restrict__ status, ViewTable vt,
                                                           uint32_t* __restrict__ tkey, uint32_t* __restrict__ tval,
                                                           uint32_t* __restrict__ trec) {
  constexpr int kR = kEmitChunk + 1;
  __shared__ uint32_t s_pref[kR];
  __shared__ uint32_t s_base[kR];
  __shared__ uint32_t s_wtx[kR];  // rect width | the view's tile columns << 16
  __shared__ uint32_t s_rec[kR];
  __shared__ uint32_t s_off[kR];
  const uint32_t N = effective_count(nvis, status);
  const uint32_t K = effective_count(count, status);
  const uint32_t slot0 = blockIdx.x * (uint32_t)kEmitChunk;
  if (N == 0 || slot0 >= K) return;  // uniform
  const uint32_t slot1 = min(slot0 + (uint32_t)kEmitChunk, K);
  const uint32_t m0 = chunk_first[blockIdx.x];
  const uint32_t m_end = slot1 < K ? chunk_first[blockIdx.x + 1] + 1u : N;
  const int nr = (int)(m_end - m0);  // records that may own slots of the chunk (<= kR)
  for (int i = threadIdx.x; i < nr; i += kScanThreads) {
    const uint4 d = sdesc[m0 + i];
    int v = 0;  // view of the record's first tile
    while (v + 1 < vt.nviews && d.x >= (uint32_t)vt.v[v + 1].tile_off) ++v;
    s_pref[i] = epref[m0 + i];
    s_base[i] = d.x;
    s_wtx[i] = (d.y & 0xffffu) | ((uint32_t)vt.v[v].TX << 16);
    s_off[i] = d.z;
    s_rec[i] = d.w;
  }
  __syncthreads();
  for (uint32_t slot = slot0 + threadIdx.x; slot < slot1; slot += kScanThreads) {
    // last staged record whose first position is <= slot
    int lo = 0, hi = nr;  // invariant: s_pref[lo] <= slot, and slot < s_pref[hi] when hi < nr
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_pref[mid] <= slot) lo = mid; else hi = mid;
    }
    const uint32_t j = slot - s_pref[lo];
    const uint32_t wtx = s_wtx[lo], w = wtx & 0xffffu;
    const uint32_t ty = j / w, tx = j - ty * w;
    tkey[slot] = s_base[lo] + ty * (wtx >> 16) + tx;
    tval[slot] = s_off[lo] + j;  // canonical pair index
    trec[slot] = s_rec[lo];
  }
}

template <typename KT>
__global__ __launch_bounds__(kSortThreads) void radix_hist(const KT* __restrict__ keys,
                                                           const uint32_t* __restrict__ count,
                                                           const int32_t* __restrict__ status, int shift, int64_t nblk,
                                                           uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kRadix];
  const uint32_t K = effective_count(count, status);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t blk = xcd_block((int64_t)blockIdx.x, ((int64_t)K + kSortTile - 1) / kSortTile);
  const int64_t base = blk * kSortTile;
  if (base < K) {
#pragma unroll 4
    for (int k = 0; k < kSortItems; ++k) {
      const int64_t i = base + k * kSortThreads + threadIdx.x;
      if (i < K) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (kRadix - 1)], 1u);
    }
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blk] = h[threadIdx.x];
}

// One block per digit: exclusive scan of that digit's counts over the first
// nact sort blocks, the ones holding keys (in place), and the digit's total.
// Each thread takes 4 consecutive columns per step of 1024.
__global__ __launch_bounds__(256) void radix_digit_scan(uint32_t* __restrict__ hist, int64_t nblk,
                                                        const uint32_t* __restrict__ count,
                                                        const int32_t* __restrict__ status,
                                                        uint32_t* __restrict__ digit_total) {
  __shared__ uint32_t s_wave[4];
  __shared__ uint32_t s_carry;
  const int64_t nact = ((int64_t)effective_count(count, status) + kSortTile - 1) / kSortTile;
  uint32_t* row = hist + (int64_t)blockIdx.x * nblk;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nact; base += 4 * 256) {
    const int64_t i0 = base + 4 * (int64_t)threadIdx.x;
    uint32_t x[4], sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x[j] = i0 + j < nact ? row[i0 + j] : 0u;
      sum += x[j];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan_256(sum, &tot, s_wave) + s_carry;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (i0 + j < nact) row[i0 + j] = ex;
      ex += x[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) s_carry += tot;
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

// One stable scatter pass for 32-bit keys; NV value arrays travel with the
// keys (NV = 1 or 2; the second may be null when NV = 1).  Each wave owns a
// contiguous quarter (1024 elements) of the block's 4096 and ranks its items
// in element order against wave-private running digit counts in LDS (match
// by ballots; only the leader of a digit group updates the count), so the
// ranking needs no block barrier.  Then one barrier, per-digit prefixes over
// the four waves, the elements placed in LDS in (digit, index) order, and
// written out run by run, so consecutive threads write consecutive addresses.
template <int NV>
__global__ __launch_bounds__(kSortThreads) void radix_scatter(const uint32_t* __restrict__ kin,
                                                              const uint32_t* __restrict__ vin,
                                                              const uint32_t* __restrict__ vin2,
                                                              uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                              uint32_t* __restrict__ vout2,
                                                              const uint32_t* __restrict__ count,
                                                              const int32_t* __restrict__ status, int shift,
                                                              int64_t nblk, const uint32_t* __restrict__ hist,
                                                              const uint32_t* __restrict__ digit_total) {
  constexpr int kWaves = kSortThreads / kWave;
  constexpr int kPerWave = kSortTile / kWaves;
  __shared__ uint32_t s_gbase[kRadix];  // global position of this block's first element of each digit
  __shared__ uint32_t s_lbase[kRadix];  // its position within the block's digit-ordered elements
  __shared__ uint32_t s_cnt[kWaves][kRadix];  // running counts per wave, then the waves' prefixes
  __shared__ uint32_t s_wave[kWaves];
  __shared__ uint32_t s_k[kSortTile];
  __shared__ uint32_t s_v[kSortTile];
  __shared__ uint32_t s_v2[NV == 2 ? kSortTile : 1];
  const uint32_t K = effective_count(count, status);
  const int64_t nact = ((int64_t)K + kSortTile - 1) / kSortTile;
  if ((int64_t)blockIdx.x >= nact) return;  // uniform across the block
  const int64_t blk = xcd_block((int64_t)blockIdx.x, nact);
  const int64_t base = blk * kSortTile;
  const int nvalid = (int)min((int64_t)kSortTile, (int64_t)K - base);
  const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s_cnt[w][t] = 0;
  __syncthreads();
  uint32_t key[kSortItems], val[kSortItems], val2[NV == 2 ? kSortItems : 1], rk[kSortItems];
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  uint32_t* cnt = s_cnt[wave];
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int li = wave * kPerWave + k * kWave + lane;
    const bool valid = li < nvalid;
    key[k] = valid ? kin[base + li] : 0u;
    val[k] = valid ? vin[base + li] : 0u;
    if (NV == 2) val2[k] = valid ? vin2[base + li] : 0u;
  }
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int li = wave * kPerWave + k * kWave + lane;
    const bool valid = li < nvalid;
    const uint32_t d = (key[k] >> shift) & (kRadix - 1);
    const uint64_t peers = match_digit(d, valid);
    const uint32_t r = __popcll(peers & lt_mask);
    const uint32_t c = valid ? cnt[d] : 0u;  // elements of digit d earlier in this wave
    rk[k] = c + r;
    if (valid && r == 0) cnt[d] = c + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();  // the wave's LDS updates stay in item order
  }
  __syncthreads();
  {
    // digit t: the waves' prefixes and the block's count
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = s_cnt[w][t];
      s_cnt[w][t] = run;
      run += c;
    }
    uint32_t tot;
    const uint32_t lb = block_exclusive_scan_256(run, &tot, s_wave);
    const uint32_t dbase = block_exclusive_scan_256(digit_total[t], &tot, s_wave);
    s_lbase[t] = lb;
    s_gbase[t] = dbase + hist[(int64_t)t * nblk + blk];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int li = wave * kPerWave + k * kWave + lane;
    if (li < nvalid) {
      const uint32_t d = (key[k] >> shift) & (kRadix - 1);
      const uint32_t pos = s_lbase[d] + cnt[d] + rk[k];
      s_k[pos] = key[k];
      s_v[pos] = val[k];
      if (NV == 2) s_v2[pos] = val2[k];
    }
  }
  __syncthreads();
  for (int i = t; i < nvalid; i += kSortThreads) {
    const uint32_t kk = s_k[i];
    const uint32_t d = (kk >> shift) & (kRadix - 1);
    const uint32_t pos = s_gbase[d] + ((uint32_t)i - s_lbase[d]);
    kout[pos] = kk;
    vout[pos] = s_v[i];
    if (NV == 2) vout2[pos] = s_v2[i];
  }
}

// Per sorted pair: [start, end) of its tile's run and, if asked for, the
// 64-bit key.  Each thread takes 4 consecutive pairs (one 16-byte load; the
// key arrays are 256-byte aligned) and compares them with their neighbours.
__global__ void tile_ranges(const uint32_t* __restrict__ tkey, const uint32_t* __restrict__ ids,
                            const uint32_t* __restrict__ drec, const uint32_t* __restrict__ count,
                            const int32_t* __restrict__ status, uint64_t* __restrict__ keys,
                            uint32_t* __restrict__ ranges) {
  const uint32_t K = effective_count(count, status);
  const int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (i0 >= K) return;
  uint32_t t[6];  // pairs i0 - 1 .. i0 + 4 (outside [0, K): no tile)
  if (i0 + 4 <= (int64_t)K) {
    const uint4 q = *(const uint4*)(tkey + i0);
    t[1] = q.x, t[2] = q.y, t[3] = q.z, t[4] = q.w;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) t[1 + j] = i0 + j < (int64_t)K ? tkey[i0 + j] : 0xffffffffu;
  }
  t[0] = i0 > 0 ? tkey[i0 - 1] : 0xffffffffu;
  t[5] = i0 + 4 < (int64_t)K ? tkey[i0 + 4] : 0xffffffffu;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t i = i0 + j;
    if (i >= (int64_t)K) break;
    const uint32_t c = t[1 + j];
    if (keys) keys[i] = ((uint64_t)c << 32) | drec[ids[i]];
    if (t[j] != c) ranges[2 * (int64_t)c] = (uint32_t)i;
    if (t[2 + j] != c) ranges[2 * (int64_t)c + 1] = (uint32_t)(i + 1);
  }
}

// Heaviest-first tile schedule: tiles grouped by the bit length of their list
// length (33 groups), groups in decreasing order.  hist[0..63] counts the
// groups, hist[64..127] becomes each group's running write position.
__device__ __forceinline__ int length_group(uint32_t len) { return len ? 32 - __clz(len) : 0; }

__device__ __forceinline__ uint32_t tile_len(const uint32_t* ranges, const int32_t* status, int64_t t) {
  return *status == 0 ? ranges[2 * t + 1] - ranges[2 * t] : 0u;
}

__global__ __launch_bounds__(256) void tile_order_count(const uint32_t* __restrict__ ranges,
                                                        const int32_t* __restrict__ status, int64_t tiles,
                                                        uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[64];
  if (threadIdx.x < 64) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tiles) atomicAdd(&h[length_group(tile_len(ranges, status, t))], 1u);
  __syncthreads();
  if (threadIdx.x < 64 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void tile_order_scan(uint32_t* __restrict__ hist) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (int g = 63; g >= 0; --g) {
    hist[64 + g] = run;
    run += hist[g];
  }
}

__global__ __launch_bounds__(256) void tile_order_scatter(const uint32_t* __restrict__ ranges,
                                                          const int32_t* __restrict__ status, int64_t tiles,
                                                          uint32_t* __restrict__ hist, uint32_t* __restrict__ order) {
  // ranks within the block per group (LDS), one global reservation per group and block
  __shared__ uint32_t h[64], base[64];
  if (threadIdx.x < 64) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int g = 0;
  uint32_t rank = 0;
  if (t < tiles) {
    g = length_group(tile_len(ranges, status, t));
    rank = atomicAdd(&h[g], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 64 && h[threadIdx.x]) base[threadIdx.x] = atomicAdd(&hist[64 + threadIdx.x], h[threadIdx.x]);
  __syncthreads();
  if (t < tiles) order[base[g] + rank] = (uint32_t)t;
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
  uint32_t* block_sums;     // [scan blocks] pairs per block of records
  uint32_t* vis_sums;       // [scan blocks] visible records per block
  uint32_t* block_offsets;  // canonical emission offset of each block
  uint32_t* vis_offsets;    // compaction offset of each block
  uint32_t* eblock_sums;    // pairs per block of depth-sorted records
  uint32_t* eblock_offsets;
  uint32_t* nvis;           // [1] number of visible records
  uint32_t* dkey;           // [nrec] depth bits of the visible records
  uint32_t* dval;           // [nrec] their compact indices
  uint32_t* dkey_alt;
  uint32_t* dval_alt;
  uint4* desc;              // [nrec] emission descriptors of the visible records (compact index)
  uint4* sdesc;             // [nrec] the same in depth order
  uint32_t* drec;           // [nrec] depth bits by record (for the keys)
  uint32_t* tkey;           // [capacity] tile id of each pair
  uint32_t* tkey_alt;
  uint32_t* tval_alt;       // [capacity] canonical pair index (second buffer)
  uint32_t* trec_alt;       // [capacity] record id (second buffer)
  uint32_t* hist;           // [256][sort blocks]
  uint32_t* digit_total;    // [256]
  uint32_t* tile_hist;      // [128] tile schedule counters
  uint32_t* chunk_first;    // [capacity / kEmitChunk + 1] first record of each emission chunk
  size_t bytes;
};

static SortWs carve(const SortPlan& p, uint64_t capacity, void* ws) {
  SortWs w{};
  char* b = (char*)ws;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    uint32_t* q = (uint32_t*)(b + o);
    o += align256(bytes);
    return q;
  };
  const size_t nb = (size_t)p.scan_blocks, nrec = (size_t)p.nrec;
  w.block_sums = take(4 * nb);
  w.vis_sums = take(4 * nb);
  w.block_offsets = take(4 * nb);
  w.vis_offsets = take(4 * nb);
  w.eblock_sums = take(4 * nb);
  w.eblock_offsets = take(4 * nb);
  w.nvis = take(8);  // [0] visible records, [1] their pairs (unused)
  w.dkey = take(4 * nrec);
  w.dval = take(4 * nrec);
  w.dkey_alt = take(4 * nrec);
  w.dval_alt = take(4 * nrec);
  w.desc = (uint4*)take(16 * nrec);
  w.sdesc = (uint4*)take(16 * nrec);
  w.drec = take(4 * nrec);
  w.tkey = take(4 * (size_t)capacity);
  w.tkey_alt = take(4 * (size_t)capacity);
  w.tval_alt = take(4 * (size_t)capacity);
  w.trec_alt = take(4 * (size_t)capacity);
  w.hist = take(4 * (size_t)kRadix * (size_t)(p.sort_blocks > p.rec_sort_blocks ? p.sort_blocks : p.rec_sort_blocks));
  w.digit_total = take(4 * (size_t)kRadix);
  w.tile_hist = take(4 * 128);
  w.chunk_first = take(4 * ((size_t)capacity / kEmitChunk + 2));
  w.bytes = o;
  return w;
}

size_t bin_sort_ws_bytes(const SortPlan& p) { return carve(p, p.capacity, nullptr).bytes; }

// One stable LSD pass per 8 key bits; the result lands back in (k0, v0, u0)
// when the number of passes is even and in (k1, v1, u1) when it is odd.
template <typename KT, int NV>
static void radix_sort(KT* k0, uint32_t* v0, uint32_t* u0, KT* k1, uint32_t* v1, uint32_t* u1, int passes,
                       const uint32_t* count, const int32_t* status, int64_t nblk, const SortWs& w, hipStream_t s) {
  KT* kb[2] = {k0, k1};
  uint32_t* vb[2] = {v0, v1};
  uint32_t* ub[2] = {u0, u1};
  int cur = 0;
  for (int p = 0; p < passes && nblk > 0; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL((radix_hist<KT>), dim3((unsigned)nblk), dim3(kSortThreads), 0, s, kb[cur], count, status,
                       shift, nblk, w.hist);
    hipLaunchKernelGGL(radix_digit_scan, dim3(kRadix), dim3(256), 0, s, w.hist, nblk, count, status, w.digit_total);
    hipLaunchKernelGGL((radix_scatter<NV>), dim3((unsigned)nblk), dim3(kSortThreads), 0, s, kb[cur], vb[cur],
                       ub[cur], kb[cur ^ 1], vb[cur ^ 1], ub[cur ^ 1], count, status, shift, nblk, w.hist,
                       w.digit_total);
    cur ^= 1;
  }
}

hipError_t launch_bin_sort(const SortPlan& plan, const float4* splats, const uint32_t* tiles_touched, int64_t n,
                           const ViewTable& vt, float inv_tw, float inv_th, const BinOut& out, uint64_t capacity,
                           void* ws, hipStream_t s) {
  const SortWs w = carve(plan, capacity, ws);
  hipError_t e;
  if ((e = launch_fill_u32(out.ranges, 2 * (int64_t)vt.total_tiles, 0u, s)) != hipSuccess) return e;
  const int64_t nb = plan.scan_blocks;
  uint32_t* count = out.count;
  int32_t* status = out.status;
  if (nb > 0)
    hipLaunchKernelGGL(count_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, tiles_touched, plan.nrec,
                       w.block_sums, w.vis_sums);
  // K and the capacity status, then the number of visible records
  hipLaunchKernelGGL(scan_top, dim3(1), dim3(1024), 0, s, w.block_sums, nb, w.block_offsets, capacity, count, status);
  hipLaunchKernelGGL(scan_top, dim3(1), dim3(1024), 0, s, w.vis_sums, nb, w.vis_offsets, (uint64_t)0, w.nvis,
                     (int32_t*)nullptr);
  if (nb > 0) {
    hipLaunchKernelGGL(compact_visible, dim3((unsigned)nb), dim3(kScanThreads), 0, s, splats, tiles_touched,
                       plan.nrec, n, vt, inv_tw, inv_th, w.block_offsets, w.vis_offsets, status, out.offsets, w.dkey,
                       w.dval, w.desc, out.keys ? w.drec : (uint32_t*)nullptr);
    // depth order of the visible records (four passes: the result is back in dkey/dval)
    radix_sort<uint32_t, 1>(w.dkey, w.dval, nullptr, w.dkey_alt, w.dval_alt, nullptr, 4, w.nvis, status,
                            plan.rec_sort_blocks, w, s);
    hipLaunchKernelGGL(gather_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, w.desc, w.dval, w.nvis, status,
                       w.sdesc, w.eblock_sums);
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(1024), 0, s, w.eblock_sums, nb, w.eblock_offsets, (uint64_t)0,
                       w.nvis + 1, (int32_t*)nullptr);  // total unused (equals K)
    // per-record emission offsets (in dkey_alt, free after the depth sort), then
    // emit so that the tile sort ends in (tkey, pair_index, ids)
    uint32_t* epref = w.dkey_alt;
    hipLaunchKernelGGL(emit_prefix, dim3((unsigned)nb), dim3(kScanThreads), 0, s, w.sdesc, w.nvis, w.eblock_offsets,
                       status, epref, w.chunk_first);
    const bool even = plan.tile_passes % 2 == 0;
    const int64_t emit_blocks = ((int64_t)capacity + kEmitChunk - 1) / kEmitChunk;
    if (emit_blocks > 0)
      hipLaunchKernelGGL(emit_pairs, dim3((unsigned)emit_blocks), dim3(kScanThreads), 0, s, w.sdesc, epref,
                         w.chunk_first, w.nvis, count, status, vt, even ? w.tkey : w.tkey_alt,
                         even ? out.pair_index : w.tval_alt, even ? out.ids : w.trec_alt);
    if (even)
      radix_sort<uint32_t, 2>(w.tkey, out.pair_index, out.ids, w.tkey_alt, w.tval_alt, w.trec_alt, plan.tile_passes,
                              count, status, plan.sort_blocks, w, s);
    else
      radix_sort<uint32_t, 2>(w.tkey_alt, w.tval_alt, w.trec_alt, w.tkey, out.pair_index, out.ids, plan.tile_passes,
                              count, status, plan.sort_blocks, w, s);
  }
  const int64_t cap_blocks = ((int64_t)capacity + 1023) / 1024;
  if (cap_blocks > 0 && nb > 0)
    hipLaunchKernelGGL(tile_ranges, dim3((unsigned)cap_blocks), dim3(256), 0, s, w.tkey, out.ids, w.drec, count,
                       status, out.keys, out.ranges);
  if (out.order && vt.total_tiles > 0) {
    const int64_t T = vt.total_tiles;
    const unsigned tb = (unsigned)((T + 255) / 256);
    if ((e = launch_fill_u32(w.tile_hist, 128, 0u, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(tile_order_count, dim3(tb), dim3(256), 0, s, out.ranges, status, T, w.tile_hist);
    hipLaunchKernelGGL(tile_order_scan, dim3(1), dim3(64), 0, s, w.tile_hist);
    hipLaunchKernelGGL(tile_order_scatter, dim3(tb), dim3(256), 0, s, out.ranges, status, T, w.tile_hist, out.order);
  }
  return hipGetLastError();
}

}  // namespace gs
