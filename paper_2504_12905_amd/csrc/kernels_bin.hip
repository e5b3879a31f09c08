// Tile binning and depth sort (Sec. 3: Gaussians are sorted by depth before
// blending; Supp. A: 16x16 tiles).
//
// Gaussians of one view are processed in chunks of kChunk by one workgroup,
// which keeps a histogram / cursor over all tiles of the view in LDS, so the
// only atomics are LDS atomics inside a workgroup (a single hot tile can hold
// thousands of entries; global atomics on it serialise across the chip).
// 1. hist: per (view, chunk) count of the chunk's Gaussians per tile.
// 2. column scan: per (view, tile), the chunks' counts become running offsets
//    and the tile total is formed.
// 3. scan: exclusive prefix sum over the V*T totals -> tile_start (int64),
//    total -> n_instances.
// 4. depth ranks: one workgroup per view sorts (depth bits, Gaussian id)
//    pairs by a stable LSD radix sort (ties keep ascending id), giving each
//    Gaussian its depth rank in the view and the rank -> id table.
//    Depths are > znear > 0 for every Gaussian that is emitted, so their IEEE
//    bits order like the values (culled ones sort anywhere; they are never
//    emitted).
// 5. emit: each (view, Gaussian) writes its depth rank (32 bits) into its
//    tiles' segments at (tile start + chunk offset + LDS cursor).
// 6. sort: one workgroup per tile sorts its segment of ranks by a stable LSD
//    radix sort (8- or 9-bit digits, as few passes as the ranks allow) and
//    writes ids = rank -> id of the view. A block of up to 2048 keys sits in
//    LDS: each wave counts the digits of its quarter, the counts become
//    (digit, wave) offsets, and every wave scatters its quarter in order, 64
//    keys at a time, ranking equal digits within the 64 by ballots (one per
//    digit bit). Longer segments take the digit totals of the whole segment
//    per pass, then sort 2048-key blocks this way and write each block out
//    as runs of consecutive addresses. Ranks are unique within a view, so the
//    order is the depth order with ties by id, and every pass is linear in
//    the segment.
#include "common.hpp"
#include "launch.hpp"

namespace lmrs {

namespace {

constexpr int kChunk = 8192;  // Gaussians per binning workgroup

constexpr int kBinThreads = 1024;

__global__ __launch_bounds__(kBinThreads) void hist_kernel(const int4* __restrict__ rect, int n, int TX, int T,
                                                            int n_chunks, int32_t* __restrict__ chunk_hist) {
  extern __shared__ int32_t s_hist[];
  const int chunk = blockIdx.x, v = blockIdx.y;
  for (int t = threadIdx.x; t < T; t += kBinThreads) s_hist[t] = 0;
  __syncthreads();
  const int g0 = chunk * kChunk;
  const int g1 = min(n, g0 + kChunk);
  for (int g = g0 + (int)threadIdx.x; g < g1; g += kBinThreads) {
    const int4 rc = rect[(size_t)v * n + g];
    for (int ty = rc.y; ty < rc.w; ++ty)
      for (int tx = rc.x; tx < rc.z; ++tx) atomicAdd(&s_hist[ty * TX + tx], 1);
  }
  __syncthreads();
  int32_t* dst = chunk_hist + ((size_t)v * n_chunks + chunk) * T;
  for (int t = threadIdx.x; t < T; t += kBinThreads) dst[t] = s_hist[t];
}

// Per (view, tile): chunk counts -> running offsets; tile total -> counts.
__global__ __launch_bounds__(256) void colscan_kernel(int32_t* __restrict__ chunk_hist, int V, int T,
                                                      int n_chunks, int32_t* __restrict__ counts) {
  const int64_t vt = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (vt >= (int64_t)V * T) return;
  const int v = (int)(vt / T), t = (int)(vt % T);
  int32_t run = 0;
  for (int c = 0; c < n_chunks; ++c) {
    int32_t* h = chunk_hist + ((size_t)v * n_chunks + c) * T + t;
    const int32_t x = *h;
    *h = run;
    run += x;
  }
  counts[vt] = run;
}

// Single workgroup of 1024 threads scans `m` counts.
__global__ __launch_bounds__(1024) void scan_kernel(int32_t* __restrict__ counts, int64_t m,
                                                    int64_t* __restrict__ tile_start,
                                                    int64_t* __restrict__ total) {
  __shared__ int64_t s_part[1024];
  const int tid = threadIdx.x;
  const int64_t per = (m + 1023) / 1024;
  const int64_t a = tid * per, b = min(m, a + per);
  int64_t acc = 0;
  for (int64_t i = a; i < b; ++i) acc += counts[i];
  s_part[tid] = acc;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive Hillis-Steele scan of the partials
    int64_t y = tid >= d ? s_part[tid - d] : 0;
    __syncthreads();
    s_part[tid] += y;
    __syncthreads();
  }
  int64_t run = s_part[tid] - acc;
  for (int64_t i = a; i < b; ++i) {
    tile_start[i] = run;
    run += counts[i];
    counts[i] = 0;
  }
  if (tid == 1023) {
    tile_start[m] = s_part[1023];
    *total = s_part[1023];
  }
}

__global__ __launch_bounds__(kBinThreads) void emit_kernel(const int4* __restrict__ rect,
                                                            const int32_t* __restrict__ rank, int n, int TX, int T,
                                                            int n_chunks, const int32_t* __restrict__ chunk_hist,
                                                            const int64_t* __restrict__ tile_start,
                                                            uint32_t* __restrict__ keys) {
  extern __shared__ int32_t s_cur[];
  const int chunk = blockIdx.x, v = blockIdx.y;
  const int32_t* off = chunk_hist + ((size_t)v * n_chunks + chunk) * T;
  for (int t = threadIdx.x; t < T; t += kBinThreads) s_cur[t] = off[t];
  __syncthreads();
  const int64_t* ts = tile_start + (size_t)v * T;
  const int g0 = chunk * kChunk;
  const int g1 = min(n, g0 + kChunk);
  for (int g = g0 + (int)threadIdx.x; g < g1; g += kBinThreads) {
    const size_t vg = (size_t)v * n + g;
    const int4 rc = rect[vg];
    if (rc.x >= rc.z) continue;
    const uint32_t key = (uint32_t)rank[vg];
    for (int ty = rc.y; ty < rc.w; ++ty)
      for (int tx = rc.x; tx < rc.z; ++tx) {
        const int t = ty * TX + tx;
        const int slot = atomicAdd(&s_cur[t], 1);
        keys[ts[t] + slot] = key;
      }
  }
}

// ------------------------------------------------------------ radix sort
// Stable LSD radix sorts of 32-bit keys, digits of up to 9 bits. A "part" is a
// contiguous range of the input owned by one wave: the wave counts the
// digits of its part, the counts of all parts become (digit, part) offsets,
// and the wave scatters its part in order, 64 keys at a time, ranking equal
// digits within the 64 by 8 ballots. Keys are loaded kRadixUnroll steps
// ahead so that the loads of a wave overlap.
constexpr int kRadixBins = 256;
constexpr int kRadixUnroll = 8;

__device__ __forceinline__ int digit_of(uint32_t key, int shift, int bins) {
  return (int)((key >> shift) & (uint32_t)(bins - 1));
}

// Adds the digit counts of src[b0, b1) to cnt[] (LDS). One wave.
__device__ __forceinline__ void part_count(const uint32_t* src, int64_t b0, int64_t b1, int shift, int bins,
                                           int* cnt) {
  const int lane = lane_id();
  for (int64_t i0 = b0; i0 < b1; i0 += kWave * kRadixUnroll) {
    uint32_t key[kRadixUnroll];
#pragma unroll
    for (int u = 0; u < kRadixUnroll; ++u) {
      const int64_t i = i0 + u * kWave + lane;
      key[u] = i < b1 ? src[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kRadixUnroll; ++u)
      if (i0 + u * kWave + lane < b1) atomicAdd(&cnt[digit_of(key[u], shift, bins)], 1);
  }
}

// Scatters src[b0, b1) (and vsrc, if given) to dst at the running cursors
// cur[digit] (LDS, advanced here). One wave; the order within a digit is
// the input order.
__device__ __forceinline__ void part_scatter(const uint32_t* src, uint32_t* dst, const uint32_t* vsrc,
                                             uint32_t* vdst, int64_t b0, int64_t b1, int shift, int bins,
                                             int* cur) {
  const int lane = lane_id();
  const uint64_t below_mask = (1ull << lane) - 1ull;
  for (int64_t i0 = b0; i0 < b1; i0 += kWave * kRadixUnroll) {
    uint32_t key[kRadixUnroll], val[kRadixUnroll];
#pragma unroll
    for (int u = 0; u < kRadixUnroll; ++u) {
      const int64_t i = i0 + u * kWave + lane;
      key[u] = i < b1 ? src[i] : 0u;
      val[u] = vsrc && i < b1 ? vsrc[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kRadixUnroll; ++u) {
      if (i0 + u * kWave >= b1) break;  // wave-uniform
      const bool valid = i0 + u * kWave + lane < b1;
      const int dg = digit_of(key[u], shift, bins);
      uint64_t peers = __ballot(valid);  // lanes of this step with the same digit
      for (int bit = 1, q = 0; bit < bins; bit <<= 1, ++q) {
        const uint64_t set = __ballot((dg >> q) & 1);
        peers &= ((dg >> q) & 1) ? set : ~set;
      }
      const int before = __popcll(peers & below_mask);
      const int base = cur[dg];
      if (valid) {
        dst[base + before] = key[u];
        if (vdst) vdst[base + before] = val[u];
        if (before == 0) cur[dg] = base + __popcll(peers);  // one lane per digit moves the cursor
      }
    }
  }
}

// Exclusive scan of x over the first kRadixBins threads of the workgroup
// (one digit each); the other threads pass 0 and get 0. wsum: LDS, 4 ints.
__device__ __forceinline__ int bins_exclusive_scan(int x, int* wsum) {
  const int tid = threadIdx.x, lane = lane_id();
  int y = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int z = __shfl_up(y, d, kWave);
    if (lane >= d) y += z;
  }
  if (tid < kRadixBins && lane == kWave - 1) wsum[tid / kWave] = y;
  __syncthreads();
  int run = y - x;
  if (tid < kRadixBins)
    for (int v = 0; v < tid / kWave; ++v) run += wsum[v];
  __syncthreads();
  return tid < kRadixBins ? run : 0;
}

// ---- per-view depth sort: every wave of the grid owns kViewPart keys of a view
constexpr int kViewPart = 4096;
constexpr int kViewThreads = 256;
constexpr int kViewWaves = kViewThreads / kWave;

__device__ __forceinline__ int view_parts(int n) { return (n + kViewPart - 1) / kViewPart; }

__global__ __launch_bounds__(kViewThreads) void view_init_kernel(const float* __restrict__ rec, int n, int V,
                                                                  uint32_t* __restrict__ key,
                                                                  uint32_t* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * kViewThreads + threadIdx.x;
  if (i >= (int64_t)V * n) return;
  key[i] = __float_as_uint(rec[i * LMRS_REC + 9]);
  val[i] = (uint32_t)(i % n);
}

// counts[v][digit][part]
__global__ __launch_bounds__(kViewThreads) void view_count_kernel(const uint32_t* __restrict__ key, int n, int V,
                                                                   int shift, int32_t* __restrict__ counts) {
  __shared__ int cnt[kViewWaves][kRadixBins];
  const int w = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < kViewWaves * kRadixBins; i += kViewThreads) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const int np = view_parts(n);
  const int64_t part = (int64_t)blockIdx.x * kViewWaves + w;  // over V * np
  if (part < (int64_t)V * np) {
    const int v = (int)(part / np), p = (int)(part % np);
    const int64_t b0 = (int64_t)v * n + (int64_t)p * kViewPart, b1 = (int64_t)v * n + min(n, (p + 1) * kViewPart);
    part_count(key, b0, b1, shift, kRadixBins, cnt[w]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kViewWaves * kRadixBins; i += kViewThreads) {
    const int ww = i / kRadixBins, d = i % kRadixBins;
    const int64_t pt = (int64_t)blockIdx.x * kViewWaves + ww;
    if (pt < (int64_t)V * np) {
      const int v = (int)(pt / np), p = (int)(pt % np);
      counts[((int64_t)v * kRadixBins + d) * np + p] = cnt[ww][d];
    }
  }
}

// One workgroup per view: counts -> exclusive offsets in (digit, part) order,
// relative to the view's first key.
__global__ __launch_bounds__(1024) void view_offsets_kernel(int32_t* __restrict__ counts, int n) {
  __shared__ int64_t part_sum[1024];
  const int np = view_parts(n);
  const int64_t m = (int64_t)kRadixBins * np;
  int32_t* c = counts + (int64_t)blockIdx.x * m;
  const int tid = threadIdx.x;
  const int64_t per = (m + 1023) / 1024, a = tid * per, b = min(m, a + per);
  int64_t acc = 0;
  for (int64_t i = a; i < b; ++i) acc += c[i];
  part_sum[tid] = acc;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t y = tid >= d ? part_sum[tid - d] : 0;
    __syncthreads();
    part_sum[tid] += y;
    __syncthreads();
  }
  int64_t run = part_sum[tid] - acc;
  for (int64_t i = a; i < b; ++i) {
    const int32_t x = c[i];
    c[i] = (int32_t)run;
    run += x;
  }
}

__global__ __launch_bounds__(kViewThreads) void view_scatter_kernel(const uint32_t* __restrict__ ksrc,
                                                                     uint32_t* __restrict__ kdst,
                                                                     const uint32_t* __restrict__ vsrc,
                                                                     uint32_t* __restrict__ vdst, int n, int V,
                                                                     int shift,
                                                                     const int32_t* __restrict__ counts) {
  __shared__ int cur[kViewWaves][kRadixBins];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int np = view_parts(n);
  const int64_t part = (int64_t)blockIdx.x * kViewWaves + w;
  if (part >= (int64_t)V * np) return;  // whole wave
  const int v = (int)(part / np), p = (int)(part % np);
  const int64_t vb = (int64_t)v * n;
  for (int d = lane; d < kRadixBins; d += kWave) cur[w][d] = counts[((int64_t)v * kRadixBins + d) * np + p];
  const int64_t b0 = vb + (int64_t)p * kViewPart, b1 = vb + min(n, (p + 1) * kViewPart);
  part_scatter(ksrc, kdst + vb, vsrc, vdst + vb, b0, b1, shift, kRadixBins, cur[w]);
}

__global__ __launch_bounds__(kViewThreads) void view_rank_kernel(const uint32_t* __restrict__ sorted_val, int n,
                                                                  int V, int32_t* __restrict__ rank,
                                                                  int32_t* __restrict__ order) {
  const int64_t i = (int64_t)blockIdx.x * kViewThreads + threadIdx.x;
  if (i >= (int64_t)V * n) return;
  const int64_t vb = i / n * n;
  const uint32_t g = sorted_val[i];
  order[i] = (int32_t)g;
  rank[vb + g] = (int32_t)(i - vb);
}

// ---- per-tile sort of depth ranks: one workgroup per tile, wave w owns the
// part [len w / 4, len (w + 1) / 4) of the segment. Segments of up to
// kTileSortLds keys are sorted in LDS (one coalesced load and store), longer
// ones pass through the keys / tmp buffers in global memory.
constexpr int kTileSortThreads = 256;
constexpr int kTileSortWaves = kTileSortThreads / kWave;
constexpr int kTileSortLds = 2048;

// The tile sort uses digits of 9 bits when that saves a pass (ranks of 17
// or 18 bits: two passes instead of three), else of 8 bits (fewer, longer
// runs of equal digits in the block write-out). Counters for up to 512
// digits, two per thread of the workgroup.
constexpr int kTileBins = 512;
static_assert(kTileBins == 2 * kTileSortThreads, "two digits per thread");

// Exclusive scan over the kTileBins digit totals, thread t owning digits 2t
// and 2t + 1 (totals x0, x1); returns the start of digit 2t. wsum: LDS, 4 ints.
__device__ __forceinline__ int pair_exclusive_scan(int x0, int x1, int* wsum) {
  const int tid = threadIdx.x, lane = lane_id();
  const int x = x0 + x1;
  int y = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int z = __shfl_up(y, d, kWave);
    if (lane >= d) y += z;
  }
  if (lane == kWave - 1) wsum[tid / kWave] = y;
  __syncthreads();
  int run = y - x;
  for (int v = 0; v < tid / kWave; ++v) run += wsum[v];
  __syncthreads();
  return run;
}

// One stable counting pass of a block that is in LDS: src -> dst (both LDS,
// blen <= kTileSortLds) by digit; leaves the block's digit totals in tot[]
// and their exclusive prefix in start[]. Every thread of the workgroup calls it.
__device__ void lds_block_pass(const uint32_t* src, uint32_t* dst, int blen, int shift, int bins,
                               int (*cnt)[kTileBins], int* wsum, int* tot, int* start) {
  const int tid = threadIdx.x, w = tid / kWave;
  const int64_t b0 = (int64_t)blen * w / kTileSortWaves, b1 = (int64_t)blen * (w + 1) / kTileSortWaves;
  for (int i = tid; i < kTileSortWaves * kTileBins; i += kTileSortThreads) (&cnt[0][0])[i] = 0;
  __syncthreads();
  part_count(src, b0, b1, shift, bins, cnt[w]);
  __syncthreads();
  int c0[kTileSortWaves], c1[kTileSortWaves], t0 = 0, t1 = 0;
#pragma unroll
  for (int v = 0; v < kTileSortWaves; ++v) {
    c0[v] = cnt[v][2 * tid];
    c1[v] = cnt[v][2 * tid + 1];
    t0 += c0[v];
    t1 += c1[v];
  }
  int run0 = pair_exclusive_scan(t0, t1, wsum), run1 = run0 + t0;
  tot[2 * tid] = t0;
  tot[2 * tid + 1] = t1;
  start[2 * tid] = run0;
  start[2 * tid + 1] = run1;
#pragma unroll
  for (int v = 0; v < kTileSortWaves; ++v) {
    cnt[v][2 * tid] = run0;
    cnt[v][2 * tid + 1] = run1;
    run0 += c0[v];
    run1 += c1[v];
  }
  __syncthreads();
  part_scatter(src, dst, nullptr, nullptr, b0, b1, shift, bins, cnt[w]);
  __syncthreads();
}

__global__ __launch_bounds__(kTileSortThreads) void tile_sort_kernel(const int64_t* __restrict__ tile_start,
                                                                     uint32_t* __restrict__ keys,
                                                                     uint32_t* __restrict__ tmp,
                                                                     const int32_t* __restrict__ order, int n, int T,
                                                                     int rank_bits, int digit_bits,
                                                                     int32_t* __restrict__ ids) {
  __shared__ int cnt[kTileSortWaves][kTileBins];
  __shared__ int wsum[kTileSortThreads / kWave];
  __shared__ int tot[kTileBins], start[kTileBins], goff[kTileBins];
  __shared__ uint32_t buf[2][kTileSortLds];
  const int64_t a = tile_start[blockIdx.x];
  const int64_t len = tile_start[blockIdx.x + 1] - a;
  if (len == 0) return;
  const int tid = threadIdx.x, w = tid / kWave;
  const int32_t* ord = order + (size_t)(blockIdx.x / T) * n;
  if (len <= kTileSortLds) {  // the whole segment in LDS
    for (int i = tid; i < len; i += kTileSortThreads) buf[0][i] = keys[a + i];
    __syncthreads();
    int q = 0;
    for (int shift = 0; shift < rank_bits; shift += digit_bits, q ^= 1)
      lds_block_pass(buf[q], buf[q ^ 1], (int)len, shift, 1 << min(digit_bits, rank_bits - shift), cnt, wsum, tot,
                     start);
    for (int i = tid; i < len; i += kTileSortThreads) ids[a + i] = ord[buf[q][i]];
    return;
  }
  // Longer segments: per pass, the digit totals of the whole segment give
  // each digit its output range; then blocks of kTileSortLds keys are
  // sorted by the digit in LDS, in order, and written out as runs of equal
  // digits (consecutive addresses) at the digits' running offsets.
  uint32_t* src = keys + a;
  uint32_t* dst = tmp + a;
  const int64_t b0 = len * w / kTileSortWaves, b1 = len * (w + 1) / kTileSortWaves;
  for (int shift = 0; shift < rank_bits; shift += digit_bits) {
    const int bins = 1 << min(digit_bits, rank_bits - shift);
    for (int i = tid; i < kTileSortWaves * kTileBins; i += kTileSortThreads) (&cnt[0][0])[i] = 0;
    __syncthreads();
    part_count(src, b0, b1, shift, bins, cnt[w]);
    __syncthreads();
    int t0 = 0, t1 = 0;
#pragma unroll
    for (int v = 0; v < kTileSortWaves; ++v) {
      t0 += cnt[v][2 * tid];
      t1 += cnt[v][2 * tid + 1];
    }
    const int run0 = pair_exclusive_scan(t0, t1, wsum);
    goff[2 * tid] = run0;
    goff[2 * tid + 1] = run0 + t0;
    __syncthreads();
    for (int64_t base = 0; base < len; base += kTileSortLds) {
      const int blen = (int)min<int64_t>(kTileSortLds, len - base);
      for (int i = tid; i < blen; i += kTileSortThreads) buf[0][i] = src[base + i];
      __syncthreads();
      lds_block_pass(buf[0], buf[1], blen, shift, bins, cnt, wsum, tot, start);
      for (int i = tid; i < blen; i += kTileSortThreads) {
        const uint32_t key = buf[1][i];
        const int d = digit_of(key, shift, bins);
        dst[goff[d] + (i - start[d])] = key;
      }
      __syncthreads();
      goff[2 * tid] += tot[2 * tid];
      goff[2 * tid + 1] += tot[2 * tid + 1];
      __syncthreads();
    }
    uint32_t* tt = src;
    src = dst;
    dst = tt;
  }
  for (int64_t i = tid; i < len; i += kTileSortThreads) ids[a + i] = ord[src[i]];
}

}  // namespace

int bin_chunks(int n) { return (n + kChunk - 1) / kChunk; }

void launch_bin_count(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s) {
  const int nc = bin_chunks(d.n);
  const size_t lds = (size_t)d.T * sizeof(int32_t);
  hist_kernel<<<dim3(nc, d.V), kBinThreads, lds, s>>>(reinterpret_cast<const int4*>(f->rect), d.n, d.TX, d.T,
                                                      nc, b.chunk_hist);
  const int64_t m = (int64_t)d.V * d.T;
  colscan_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(b.chunk_hist, d.V, d.T, nc, b.counts);
  scan_kernel<<<1, 1024, 0, s>>>(b.counts, m, f->tile_start, f->n_instances);
}

void launch_view_sort(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s) {
  // depth ranks per view: four 8-bit passes over the FP32 depth bits
  const int64_t vn = (int64_t)d.V * d.n;
  const int np = (d.n + kViewPart - 1) / kViewPart;
  const unsigned vblocks = (unsigned)((vn + kViewThreads - 1) / kViewThreads);
  const unsigned pblocks = (unsigned)(((int64_t)d.V * np + kViewWaves - 1) / kViewWaves);
  view_init_kernel<<<vblocks, kViewThreads, 0, s>>>(f->rec, d.n, d.V, b.vkey[0], b.vval[0]);
  for (int pass = 0; pass < 4; ++pass) {
    const int q = pass & 1;
    view_count_kernel<<<pblocks, kViewThreads, 0, s>>>(b.vkey[q], d.n, d.V, 8 * pass, b.vcount);
    view_offsets_kernel<<<d.V, 1024, 0, s>>>(b.vcount, d.n);
    view_scatter_kernel<<<pblocks, kViewThreads, 0, s>>>(b.vkey[q], b.vkey[q ^ 1], b.vval[q], b.vval[q ^ 1], d.n,
                                                          d.V, 8 * pass, b.vcount);
  }
  view_rank_kernel<<<vblocks, kViewThreads, 0, s>>>(b.vval[0], d.n, d.V, b.rank, b.order);
}

void launch_bin_emit_sort(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s) {
  const int nc = bin_chunks(d.n);
  const size_t lds = (size_t)d.T * sizeof(int32_t);
  emit_kernel<<<dim3(nc, d.V), kBinThreads, lds, s>>>(reinterpret_cast<const int4*>(f->rect), b.rank, d.n, d.TX,
                                                      d.T, nc, b.chunk_hist, f->tile_start, b.keys);
  const int rank_bits = d.n > 1 ? 32 - __builtin_clz((unsigned)(d.n - 1)) : 0;
  const int digit_bits = (rank_bits + 8) / 9 < (rank_bits + 7) / 8 ? 9 : 8;
  tile_sort_kernel<<<(unsigned)((int64_t)d.V * d.T), kTileSortThreads, 0, s>>>(
      f->tile_start, b.keys, b.tmp, b.order, d.n, d.T, rank_bits, digit_bits, f->ids);
}

int view_sort_count_ints(int n, int V) { return V * ((n + kViewPart - 1) / kViewPart) * kRadixBins; }

}  // namespace lmrs
