// Tile binning and depth sort (Sec. 3: Gaussians are sorted by depth before
// blending; Supp. A: 16x16 tiles).
//
// 1. total: the number of tile-list entries (sum of the rect areas), copied
//    to the host first so that its wait overlaps the steps below.
// 2. depth ranks: per view, a stable LSD radix sort of (32-bit depth key,
//    Gaussian id) over all waves of the grid (ties keep ascending id; the key
//    is monotone in the FP64 depth, see depth_sort_key), then runs of equal
//    keys re-ordered by the FP64 depth (its bits, then id), give each
//    Gaussian its rank in FP64 depth order and the rank -> id table. Depths
//    are > znear > 0 for every Gaussian that is emitted (culled ones sort
//    anywhere; they are never emitted).
// 3. hist: the Gaussians of a view in rank order, cut into chunks of kChunk
//    ranks; one workgroup per (view, chunk) counts its Gaussians per tile in
//    LDS (the only atomics are LDS atomics: a hot tile can hold thousands of
//    entries, and global atomics on it would serialise across the chip).
// 4. column scan per (view, tile) over the chunks -> running offsets; scan
//    over the V*T totals -> tile_start (int64), in 256-tile workgroups.
// 5. emit: each chunk writes its Gaussians' ranks into their tiles'
//    segments at (tile start + chunk offset + LDS cursor). A tile's list is
//    thereby ordered by chunk, i.e. by rank up to the order inside each
//    chunk's run, and a run holds at most kChunk entries.
// 6. sort: one workgroup per tile takes windows of up to kTileSortLds
//    entries that end at a run boundary (the runs are read off the ranks),
//    sorts each in LDS by the ranks relative to the window's first chunk (a
//    bitmap of the ranks when they span up to 64 chunks, else a stable LSD
//    radix sort with digits of up to 9 bits), and writes ids = rank -> id.
//    Every entry is read and written once; ranks are unique within a view,
//    so the order is the depth order with ties by id.
#include "common.hpp"
#include "launch.hpp"

namespace lmrs {

namespace {

constexpr int kChunkBits = 11;
constexpr int kChunk = 1 << kChunkBits;  // ranks per binning workgroup (and entries per run, at most)
static_assert(kChunk <= 2048, "a run must fit one sort window");

constexpr int kBinThreads = 1024;

__device__ __forceinline__ int rect_area(const int4& rc) {
  return rc.x < rc.z && rc.y < rc.w ? (rc.z - rc.x) * (rc.w - rc.y) : 0;
}

// Sum of the rect areas of all (view, Gaussian) pairs: partial sums per block.
constexpr int kAreaBlocks = kBinAreaParts;
__global__ __launch_bounds__(256) void area_kernel(const int4* __restrict__ rect, int64_t m,
                                                   int64_t* __restrict__ part) {
  __shared__ double s_red[256];
  int64_t acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
    acc += rect_area(rect[i]);
  // exact: the sums stay far below 2^53
  const double tot = block_sum((double)acc, s_red);
  if (threadIdx.x == 0) part[blockIdx.x] = (int64_t)tot;
}

__global__ __launch_bounds__(256) void area_total_kernel(const int64_t* __restrict__ part, int np,
                                                         int64_t* __restrict__ total) {
  __shared__ double s_red[256];
  int64_t acc = 0;
  for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
  const double tot = block_sum((double)acc, s_red);
  if (threadIdx.x == 0) *total = (int64_t)tot;
}

// Calls body(t, r) for every tile t of the rect of each rank r in [r0, r1)
// of view v (the Gaussians in depth order), with the work spread over the
// wave: rect areas are very uneven (at 1.5M Gaussians, mean 54 tiles, the
// largest 4,108), and a lane looping over its own rect left the wave at 23 %
// lane efficiency. A rect of up to kLaneArea tiles is walked by its own lane;
// larger ones are taken by the whole wave one at a time, kWave / width rows
// per step (a row at a time, 64 tiles per step, for rects wider than 64).
// Every thread of the workgroup calls it.
constexpr int kLaneArea = 16;

template <class Body>
__device__ __forceinline__ void for_rect_tiles(const int4* __restrict__ rect, const int32_t* __restrict__ order,
                                               int n, int v, int r0, int r1, int TX, Body body) {
  const int lane = lane_id();
  for (int base = r0; base < r1; base += kBinThreads) {
    const int r = base + (int)threadIdx.x;
    int4 rc = make_int4(0, 0, 0, 0);
    if (r < r1) rc = rect[(size_t)v * n + order[(size_t)v * n + r]];
    const int w = max(rc.z - rc.x, 0), h = max(rc.w - rc.y, 0);
    const bool big = w * h > kLaneArea;
    if (!big)
      for (int ty = rc.y; ty < rc.w; ++ty)
        for (int tx = rc.x; tx < rc.z; ++tx) body(ty * TX + tx, r);
    for (uint64_t bm = __ballot(big); bm; bm &= bm - 1) {
      const int src = __ffsll((unsigned long long)bm) - 1;
      const int x0 = readlane(rc.x, src), y0 = readlane(rc.y, src);
      const int bw = readlane(w, src), y1 = readlane(rc.w, src), rb = readlane(r, src);
      if (bw <= kWave) {
        const int rows = kWave / bw, row = lane / bw, col = lane - row * bw;
        if (row < rows)
          for (int ty = y0 + row; ty < y1; ty += rows) body(ty * TX + x0 + col, rb);
      } else {
        for (int ty = y0; ty < y1; ++ty)
          for (int tx = x0 + lane; tx < x0 + bw; tx += kWave) body(ty * TX + tx, rb);
      }
    }
  }
}

__global__ __launch_bounds__(kBinThreads) void hist_kernel(const int4* __restrict__ rect,
                                                            const int32_t* __restrict__ order, int n, int TX,
                                                            int T, int n_chunks, int32_t* __restrict__ chunk_hist) {
  extern __shared__ int32_t s_hist[];
  const int chunk = blockIdx.x, v = blockIdx.y;
  for (int t = threadIdx.x; t < T; t += kBinThreads) s_hist[t] = 0;
  __syncthreads();
  const int r0 = chunk * kChunk;
  const int r1 = min(n, r0 + kChunk);
  for_rect_tiles(rect, order, n, v, r0, r1, TX, [&](int t, int) { atomicAdd(&s_hist[t], 1); });
  __syncthreads();
  int32_t* dst = chunk_hist + ((size_t)v * n_chunks + chunk) * T;
  for (int t = threadIdx.x; t < T; t += kBinThreads) dst[t] = s_hist[t];
}

// Per (view, tile): chunk counts -> running offsets; tile total -> counts;
// each workgroup's sum of its 256 tile totals -> col_part. The counts are
// read kColUnroll chunks ahead of the running sum.
constexpr int kColUnroll = 8;
__global__ __launch_bounds__(256) void colscan_kernel(int32_t* __restrict__ chunk_hist, int V, int T,
                                                      int n_chunks, int32_t* __restrict__ counts,
                                                      int64_t* __restrict__ col_part) {
  __shared__ double s_red[256];
  const int64_t vt = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int32_t run = 0;
  if (vt < (int64_t)V * T) {
    const int v = (int)(vt / T), t = (int)(vt % T);
    int32_t* h = chunk_hist + (size_t)v * n_chunks * T + t;
    for (int c0 = 0; c0 < n_chunks; c0 += kColUnroll) {
      int32_t x[kColUnroll];
#pragma unroll
      for (int u = 0; u < kColUnroll; ++u) x[u] = c0 + u < n_chunks ? h[(size_t)(c0 + u) * T] : 0;
#pragma unroll
      for (int u = 0; u < kColUnroll; ++u)
        if (c0 + u < n_chunks) {
          h[(size_t)(c0 + u) * T] = run;
          run += x[u];
        }
    }
    counts[vt] = run;
  }
  const double sum = block_sum((double)run, s_red);  // exact: far below 2^53
  if (threadIdx.x == 0) col_part[blockIdx.x] = (int64_t)sum;
}

// tile_start = exclusive prefix sum of the m tile totals, in the workgroups
// of colscan_kernel: each adds the col_part of the workgroups before it to a
// scan of its own 256 totals; the counts are reset to zero for the cursors of
// the next binning. The last entry also gives tile_start[m].
// When the total (the rect-area sum written before) exceeds `capacity`,
// every list is left empty instead (tile_start all 0): the entries would not
// fit the caller's buffers, and the kernels after this one then see no list.
__global__ __launch_bounds__(256) void tile_start_kernel(int32_t* __restrict__ counts, int64_t m,
                                                         const int64_t* __restrict__ col_part,
                                                         int64_t* __restrict__ tile_start,
                                                         int64_t* __restrict__ total, int64_t capacity) {
  __shared__ double s_red[256];
  __shared__ int64_t s_wave[256 / kWave];
  const int tid = threadIdx.x, lane = lane_id();
  const bool over = *total > capacity;  // the same value in every workgroup (written by area_total_kernel)
  int64_t before = 0;
  for (int b = tid; b < (int)blockIdx.x; b += 256) before += col_part[b];
  const int64_t off = (int64_t)block_sum((double)before, s_red);
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  const int64_t x = i < m ? counts[i] : 0;
  int64_t y = x;  // inclusive scan over the workgroup
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t z = __shfl_up(y, d, kWave);
    if (lane >= d) y += z;
  }
  if (lane == kWave - 1) s_wave[tid / kWave] = y;
  __syncthreads();
  for (int w = 0; w < tid / kWave; ++w) y += s_wave[w];
  if (i < m) {
    tile_start[i] = over ? 0 : off + y - x;
    counts[i] = 0;
  }
  if (i == m - 1) tile_start[m] = over ? 0 : off + y;
}

__global__ __launch_bounds__(kBinThreads) void emit_kernel(const int4* __restrict__ rect,
                                                            const int32_t* __restrict__ order, int n, int TX, int T,
                                                            int n_chunks, const int32_t* __restrict__ chunk_hist,
                                                            const int64_t* __restrict__ tile_start,
                                                            const int64_t* __restrict__ total, int64_t capacity,
                                                            uint32_t* __restrict__ keys) {
  extern __shared__ int32_t s_cur[];
  if (*total > capacity) return;  // lists left empty (tile_start_kernel)
  const int chunk = blockIdx.x, v = blockIdx.y;
  const int32_t* off = chunk_hist + ((size_t)v * n_chunks + chunk) * T;
  for (int t = threadIdx.x; t < T; t += kBinThreads) s_cur[t] = off[t];
  __syncthreads();
  const int64_t* ts = tile_start + (size_t)v * T;
  const int r0 = chunk * kChunk;
  const int r1 = min(n, r0 + kChunk);
  for_rect_tiles(rect, order, n, v, r0, r1, TX, [&](int t, int r) {
    const int slot = atomicAdd(&s_cur[t], 1);
    keys[ts[t] + slot] = (uint32_t)r;
  });
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
  key[i] = depth_sort_key(depth_bits(rec[i * LMRS_REC + 9], rec[i * LMRS_REC + 11]));
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

// ---- ties of the depth key. The radix passes order a view's Gaussians by
// (32-bit depth key, id); a run of equal keys (depths within 2^-27 relative)
// is then re-ordered by (FP64 depth bits, id), which gives the order of the
// FP64 depths with ties by id. One wave per 64 ranks. A run of up to
// kTieShort members (nearly all runs) is sorted by the lane at its head in
// registers; the wave holding the first rank of a longer run sorts it: each
// member's place is the count of members before it, written to tmp and
// copied back, and runs already in order are left alone after one pass over
// them (equal FP64 depths keep the id order of the radix passes). Key 0
// (depth <= 0, culled, never listed) is not looked at.
constexpr int kTieShort = 8;

__device__ __forceinline__ uint64_t depth_of(const float* __restrict__ rec, int64_t vn, uint32_t g) {
  const float* r = rec + (vn + g) * LMRS_REC;
  return depth_bits(r[9], r[11]);
}

__global__ __launch_bounds__(256) void view_ties_kernel(const uint32_t* __restrict__ key, uint32_t* __restrict__ val,
                                                        uint32_t* __restrict__ tmp, const float* __restrict__ rec,
                                                        int n, int V) {
  const int lane = lane_id();
  const int per_view = (n + kWave - 1) / kWave;
  const int64_t wave = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
  if (wave >= (int64_t)V * per_view) return;  // whole wave
  const int v = (int)(wave / per_view);
  const int i0 = (int)(wave % per_view) * kWave;
  const int64_t vn = (int64_t)v * n;
  const uint32_t* kv = key + vn;
  uint32_t* ids = val + vn;
  uint32_t* tv = tmp + vn;
  const int i = i0 + lane;
  const uint32_t k = i < n ? kv[i] : 0u;
  const bool prev_differs = i == 0 || (i < n && kv[i - 1] != k);
  const bool next_same = i + 1 < n && kv[i + 1] == k;
  const bool positive = k != 0u;  // z > 0
  const bool head = i < n && prev_differs && next_same && positive;
  // Short runs (up to kTieShort members, nearly all of them) are put in
  // order by the lane at their head, with an insertion sort in registers;
  // longer ones by the whole wave below.
  bool long_run = false;
  if (head) {
    uint32_t g[kTieShort];
    uint64_t z[kTieShort];
    int len = 0;
#pragma unroll
    for (int q = 0; q < kTieShort; ++q) {
      if (q == len && i + q < n && (q < 2 || kv[i + q] == k)) {
        g[q] = ids[i + q];
        z[q] = depth_of(rec, vn, g[q]);
        ++len;
      }
    }
    long_run = len == kTieShort && i + kTieShort < n && kv[i + kTieShort] == k;
    if (!long_run) {
      // odd-even transposition sort of (depth bits, id) with fixed indices;
      // slots past the run hold the largest key and stay last
      uint32_t g0[kTieShort];
#pragma unroll
      for (int q = 0; q < kTieShort; ++q) {
        if (q >= len) {
          g[q] = 0xffffffffu;
          z[q] = ~0ull;
        }
        g0[q] = g[q];
      }
#pragma unroll
      for (int r = 0; r < kTieShort; ++r) {
#pragma unroll
        for (int q = r & 1; q + 1 < kTieShort; q += 2) {
          const bool swap = z[q] > z[q + 1] || (z[q] == z[q + 1] && g[q] > g[q + 1]);
          const uint64_t za = swap ? z[q + 1] : z[q], zb = swap ? z[q] : z[q + 1];
          const uint32_t ga = swap ? g[q + 1] : g[q], gb = swap ? g[q] : g[q + 1];
          z[q] = za;
          z[q + 1] = zb;
          g[q] = ga;
          g[q + 1] = gb;
        }
      }
#pragma unroll
      for (int q = 0; q < kTieShort; ++q)
        if (q < len && g[q] != g0[q]) ids[i + q] = g[q];
    }
  }
  for (uint64_t heads = __ballot(head && long_run); heads; heads &= heads - 1) {
    const int src = __ffsll((unsigned long long)heads) - 1;
    const int a = i0 + src;
    const uint32_t K = (uint32_t)readlane((int)k, src);
    // end of the run, and whether it is already in (sub, id) order
    int e = n;
    bool sorted = true;
    for (int base = a; base < n; base += kWave) {
      const int j = base + lane;
      const bool in = j < n && kv[j] == K;
      uint32_t g = 0u;
      uint64_t sb = 0u;
      if (in) {
        g = ids[j];
        sb = depth_of(rec, vn, g);
      }
      // order against the next member, held by lane + 1 (or the next step's lane 0)
      const uint32_t g1 = (uint32_t)__shfl_down((int)g, 1);
      const uint64_t s1 = ((uint64_t)(uint32_t)__shfl_down((int)(uint32_t)(sb >> 32), 1) << 32) |
                          (uint32_t)__shfl_down((int)(uint32_t)sb, 1);
      bool ok = true;
      if (in && lane < kWave - 1 && j + 1 < n && kv[j + 1] == K) ok = sb < s1 || (sb == s1 && g < g1);
      if (in && lane == kWave - 1 && j + 1 < n && kv[j + 1] == K) {
        const uint32_t gn = ids[j + 1];
        const uint64_t sn = depth_of(rec, vn, gn);
        ok = sb < sn || (sb == sn && g < gn);
      }
      sorted = sorted && (__ballot(!ok) == 0);
      const uint64_t out = __ballot(!in);
      if (out) {
        e = base + __ffsll((unsigned long long)out) - 1;
        break;
      }
    }
    if (sorted) continue;
    for (int jb = a; jb < e; jb += kWave) {
      const int j = jb + lane;
      uint32_t gj = 0xffffffffu;
      uint64_t sj = ~0ull;
      if (j < e) {
        gj = ids[j];
        sj = depth_of(rec, vn, gj);
      }
      int place = 0;
      for (int mb = a; mb < e; mb += kWave) {
        const int m = mb + lane;
        uint32_t gm = 0xffffffffu;
        uint64_t sm = ~0ull;
        if (m < e) {
          gm = ids[m];
          sm = depth_of(rec, vn, gm);
        }
        const int cnt = min(kWave, e - mb);
        for (int q = 0; q < cnt; ++q) {
          const uint64_t s2 = ((uint64_t)(uint32_t)readlane((int)(uint32_t)(sm >> 32), q) << 32) |
                              (uint32_t)readlane((int)(uint32_t)sm, q);
          const uint32_t g2 = (uint32_t)readlane((int)gm, q);
          place += (s2 < sj || (s2 == sj && g2 < gj)) ? 1 : 0;
        }
      }
      if (j < e) tv[a + place] = gj;
    }
    __threadfence();  // the run's places are written; read them back
    for (int jb = a; jb < e; jb += kWave) {
      const int j = jb + lane;
      if (j < e) ids[j] = tv[j];
    }
    __threadfence();
  }
}

// ---- per-tile sort of depth ranks: one workgroup per tile, windows of up to
// kTileSortLds entries in LDS, wave w owning the part [len w / 4,
// len (w + 1) / 4) of a window.
constexpr int kTileSortThreads = 256;
constexpr int kTileSortWaves = kTileSortThreads / kWave;
constexpr int kTileSortLds = 2048;
static_assert(kChunk <= kTileSortLds, "a run must fit one sort window");

// Digits of up to 9 bits; counters for up to 512 digits, two per thread.
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
// blen <= kTileSortLds) by digit. Every thread of the workgroup calls it.
__device__ void lds_block_pass(const uint32_t* src, uint32_t* dst, int blen, int shift, int bins,
                               int (*cnt)[kTileBins], int* wsum) {
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

// A tile's list arrives as runs of ranks, one per chunk in chunk order (rank
// >> kChunkBits non-decreasing along the list), each run unordered and at
// most kChunk long. A window starts at a run and ends before the run that
// the entry after it belongs to, so it holds whole runs only, at least one.
// Its ranks relative to the first run's chunk are unique and below
// (runs spanned) * kChunk: up to kBitmapWords * 32 they are sorted by
// setting one bit each in an LDS bitmap and reading the set bits back in
// order (each thread a range of words, at the running count of the ranges
// before it) into LDS, from where the ids are written out coalesced; wider
// windows (short lists spanning many chunks) take the
// radix passes.
constexpr int kBitmapWords = kTileSortLds + kTileSortWaves * kTileBins;

__global__ __launch_bounds__(kTileSortThreads) void tile_sort_kernel(const int64_t* __restrict__ tile_start,
                                                                     const uint32_t* __restrict__ keys,
                                                                     const int32_t* __restrict__ order, int n, int T,
                                                                     int32_t* __restrict__ ids) {
  // s_work: the radix passes' second buffer and digit counters, or the bitmap
  __shared__ uint32_t s_keys[kTileSortLds];
  __shared__ uint32_t s_work[kBitmapWords];
  __shared__ int wsum[kTileSortThreads / kWave];
  int(*cnt)[kTileBins] = reinterpret_cast<int(*)[kTileBins]>(s_work + kTileSortLds);
  const int64_t a = tile_start[blockIdx.x];
  const int64_t len = tile_start[blockIdx.x + 1] - a;
  const int tid = threadIdx.x;
  const int32_t* ord = order + (size_t)(blockIdx.x / T) * n;
  for (int64_t pos = 0; pos < len;) {
    const int wlen = (int)min<int64_t>(kTileSortLds, len - pos);
    for (int i = tid; i < wlen; i += kTileSortThreads) s_keys[i] = keys[a + pos + i];
    // the run of the entry after the window (none: past every run)
    const uint32_t next_run = pos + wlen < len ? keys[a + pos + wlen] >> kChunkBits : 0xffffffffu;
    __syncthreads();
    // m: the entries of runs before next_run's, a prefix of the window
    // (never empty for lists written by emit_kernel)
    int m = 0;
    for (int i0 = 0; i0 < wlen; i0 += kTileSortThreads) {
      const int i = i0 + tid;
      m += __syncthreads_count(i < wlen && (s_keys[i] >> kChunkBits) < next_run);
    }
    m = m > 0 ? m : wlen;
    // ranks relative to the first run's chunk; the largest lies in the last run
    const uint32_t base = (s_keys[0] >> kChunkBits) << kChunkBits;
    const uint32_t top = ((s_keys[m - 1] >> kChunkBits) << kChunkBits) + (kChunk - 1) - base;
    int32_t* out = ids + a + pos;
    if (top < (uint32_t)kBitmapWords * 32u) {
      const int nwords = (int)(top >> 5) + 1;
      for (int i = tid; i < nwords; i += kTileSortThreads) s_work[i] = 0u;
      __syncthreads();
      for (int i = tid; i < m; i += kTileSortThreads) {
        const uint32_t r = s_keys[i] - base;
        atomicOr(&s_work[r >> 5], 1u << (r & 31));
      }
      __syncthreads();
      const int wpt = (nwords + kTileSortThreads - 1) / kTileSortThreads;
      const int w0 = min(nwords, tid * wpt), w1 = min(nwords, w0 + wpt);
      int own = 0;
      for (int w = w0; w < w1; ++w) own += __popc(s_work[w]);
      int p = pair_exclusive_scan(own, 0, wsum);  // (its barriers also retire the reads of s_keys)
      for (int w = w0; w < w1; ++w)
        for (uint32_t bits = s_work[w]; bits; bits &= bits - 1u)
          s_keys[p++] = base + ((uint32_t)w << 5) + (uint32_t)(__ffs(bits) - 1);
      __syncthreads();
      for (int i = tid; i < m; i += kTileSortThreads) out[i] = ord[s_keys[i]];
    } else {
      const int nbits = 32 - __clz(top);
      const int passes = (nbits + 8) / 9;
      const int digit_bits = (nbits + passes - 1) / passes;
      __syncthreads();
      for (int i = tid; i < m; i += kTileSortThreads) s_keys[i] -= base;
      __syncthreads();
      uint32_t *src = s_keys, *dst = s_work;
      for (int shift = 0; shift < nbits; shift += digit_bits) {
        lds_block_pass(src, dst, m, shift, 1 << min(digit_bits, nbits - shift), cnt, wsum);
        uint32_t* t = src;
        src = dst;
        dst = t;
      }
      for (int i = tid; i < m; i += kTileSortThreads) out[i] = ord[src[i] + base];
    }
    pos += m;
    __syncthreads();
  }
}

}  // namespace

int bin_chunks(int n) { return (n + kChunk - 1) / kChunk; }

void launch_bin_total(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s) {
  const int64_t m = (int64_t)d.V * d.n;
  const int blocks = (int)std::min<int64_t>(kAreaBlocks, std::max<int64_t>(1, (m + 255) / 256));
  area_kernel<<<blocks, 256, 0, s>>>(reinterpret_cast<const int4*>(f->rect), m, b.area_part);
  area_total_kernel<<<1, 256, 0, s>>>(b.area_part, blocks, f->n_instances);
}

void launch_bin_count(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s) {
  const int nc = bin_chunks(d.n);
  const size_t lds = (size_t)d.T * sizeof(int32_t);
  hist_kernel<<<dim3(nc, d.V), kBinThreads, lds, s>>>(reinterpret_cast<const int4*>(f->rect), b.order, d.n, d.TX,
                                                      d.T, nc, b.chunk_hist);
  const int64_t m = (int64_t)d.V * d.T;
  const unsigned cblocks = (unsigned)((m + 255) / 256);
  colscan_kernel<<<cblocks, 256, 0, s>>>(b.chunk_hist, d.V, d.T, nc, b.counts, b.col_part);
  tile_start_kernel<<<cblocks, 256, 0, s>>>(b.counts, m, b.col_part, f->tile_start, f->n_instances, f->capacity);
}

void launch_view_sort(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s) {
  // depth ranks per view: four 8-bit passes over the 32-bit depth keys
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
  // after four passes the sorted ids are in vval[0]; with the ties of the FP32
  // key ordered by the FP64 depth that is the rank -> id table
  const unsigned tblocks = (unsigned)(((int64_t)d.V * ((d.n + kWave - 1) / kWave) + 3) / 4);
  view_ties_kernel<<<tblocks, 256, 0, s>>>(b.vkey[0], b.vval[0], b.vkey[1], f->rec, d.n, d.V);
}

void launch_bin_emit_sort(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s) {
  const int nc = bin_chunks(d.n);
  const size_t lds = (size_t)d.T * sizeof(int32_t);
  emit_kernel<<<dim3(nc, d.V), kBinThreads, lds, s>>>(reinterpret_cast<const int4*>(f->rect), b.order, d.n, d.TX,
                                                      d.T, nc, b.chunk_hist, f->tile_start, f->n_instances,
                                                      f->capacity, b.keys);
  tile_sort_kernel<<<(unsigned)((int64_t)d.V * d.T), kTileSortThreads, 0, s>>>(f->tile_start, b.keys, b.order,
                                                                              d.n, d.T, f->ids);
}

int view_sort_count_ints(int n, int V) { return V * ((n + kViewPart - 1) / kViewPart) * kRadixBins; }

}  // namespace lmrs
