// Per-tile splat kernels: forward render (Sec. 3 eq. 3; Supp. A Alg. 2),
// J p (forward mode, Alg. 3), J^T u (reverse accumulation, Supp. A "J^T v
// kernel"), their fused composition J^T W J p (the operator product of the
// PCG loop in Alg. 1), and the weighted Gram blocks behind diag(J^T W J).
//
// Work layout. The paper launches one thread per sampled pixel; with ~10 %
// of a 16x16 tile sampled that leaves most of a wave64 idle and forces
// cross-lane reductions of every Gaussian's gradient. Here the lanes own list
// entries instead: a chunk of 64 entries of the tile's depth-sorted list is
// loaded, one record per lane, and a wave walks its share of the tile's
// sampled pixels one after another (a tile's pixels are dealt to 1, 2 or 4
// waves of a workgroup, see deriv_tile; the derivative kernels hand tiles to
// a persistent grid, longest walk first, see "tile schedule" below). For
// each pixel the transmittance in front of every entry is a prefix product
// of (1 - alpha) across the lanes (a DPP scan), carried from chunk to chunk;
// J p needs one prefix sum more for its derivative. J^T u walks the chunks
// back to front with the lane order reversed inside a chunk, so the colour
// blended behind an entry and the transmittance product behind it are prefix
// scans as well. Each lane accumulates its entry's screen-space gradient
// over the wave's pixels; per chunk the waves' partials meet in LDS and are
// flushed transposed, an atomic instruction covering whole 64-byte gradient
// rows of 4 entries. A pixel's loop stops at its last blended entry (`last`
// from the render), so work follows the actual blend depth per pixel.
// Per-pixel state lives in lane registers (pixel 64 s + l in slot s of lane
// l) and is read and written with readlane / writelane. The residual scores
// (every pixel of a tile) take a lane per pixel instead (score_kernel).
//
// Discrete decisions (list, opacity skip, cap, stop position) come from the
// render and are recomputed bit-identically by pair_alpha().
#include <algorithm>
#include <atomic>

#include "common.hpp"
#include "launch.hpp"

namespace lmrs {

namespace {

constexpr int kMaxK = 256;

struct TileCtx {
  int v, t;
  int64_t tile_lin, start, len;
  float ox, oy;
};

__device__ __forceinline__ TileCtx tile_ctx(const int64_t* tile_start, int T, int TX, int64_t tile_lin) {
  TileCtx c;
  c.tile_lin = tile_lin;
  c.v = (int)(c.tile_lin / T);
  c.t = (int)(c.tile_lin % T);
  c.start = tile_start[c.tile_lin];
  c.len = tile_start[c.tile_lin + 1] - c.start;
  c.ox = (float)((c.t % TX) * kTile);
  c.oy = (float)((c.t / TX) * kTile);
  return c;
}

__device__ __forceinline__ void pixel_center(const uint8_t* pix, int k, const TileCtx& c, int j, float* xc,
                                             float* yc) {
  const int p = pix ? (int)pix[c.tile_lin * k + j] : j;
  *xc = c.ox + (float)(p & 15) + 0.5f;
  *yc = c.oy + (float)(p >> 4) + 0.5f;
}

// u, v, conic factor f11 f12 f22, opacity, rgb (see proj_geom)
struct RecF {
  float u, v, f11, f12, f22, o, r, g, b;
};

__device__ __forceinline__ RecF load_rec(const float* rec, size_t vg) {
  const float4* p = reinterpret_cast<const float4*>(rec + vg * LMRS_REC);
  const float4 a = p[0], b = p[1], c = p[2];
  return RecF{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x};
}

// The footprint part of a record (u, v, f11, f12, f22, opacity): two loads.
__device__ __forceinline__ RecF load_geo(const float* rec, size_t vg) {
  const float* p = rec + vg * LMRS_REC;
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float2 b = *reinterpret_cast<const float2*>(p + 4);
  return RecF{a.x, a.y, a.z, a.w, b.x, b.y, 0.f, 0.f, 0.f};
}

// List id at entry c0 + lane of the tile, -1 past the end of the list.
__device__ __forceinline__ int fwd_chunk_id(const int32_t* ids, const TileCtx& c, int c0) {
  const int e = c0 + lane_id();
  return e < c.len ? ids[c.start + e] : -1;
}

// List id at entry c0 + 63 - lane of the tile (the reverse walk's lane
// order), -1 past the end of the list.
__device__ __forceinline__ int rev_chunk_id(const int32_t* ids, const TileCtx& c, int c0) {
  const int e = c0 + kWave - 1 - lane_id();
  return e < c.len ? ids[c.start + e] : -1;
}

// Makes the wave wait here until the loads into these registers (prefetched
// for the next chunk) have landed. The reverse walk places it before the
// chunk's gradient atomics: one counter orders all vector memory operations
// of a wave, so a wait for those loads at the top of the next chunk would
// also wait for the atomics issued in between.
__device__ __forceinline__ void landed(const RecF& r) {
  asm volatile("" ::"v"(r.u), "v"(r.v), "v"(r.f11), "v"(r.f12), "v"(r.f22), "v"(r.o), "v"(r.r), "v"(r.g),
               "v"(r.b));
}
__device__ __forceinline__ void landed(int x) { asm volatile("" ::"v"(x)); }

// Pixel 64 s + l of a tile lives in slot s of lane l.
template <int NS>
struct PixelRegs {
  float xc[NS], yc[NS], w[NS];
  int last[NS];
};

// w[s]: the sample weight, or with per-channel weights wc ([S][3], the SSIM
// residual's operator weights) their channel mean (the weight of the diagonal
// pass).
template <int NS>
__device__ __forceinline__ int load_pixel_regs(const uint8_t* pix, const float* wts, const float* wc,
                                               const int32_t* lastv, int k, const TileCtx& c, PixelRegs<NS>& pr) {
  int lmax = -1;
  const int lane = lane_id();
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int j = s * kWave + lane;
    pr.xc[s] = pr.yc[s] = 0.f;
    pr.w[s] = 0.f;
    pr.last[s] = -1;
    if (j < k) {
      const int64_t i = c.tile_lin * k + j;
      pixel_center(pix, k, c, j, &pr.xc[s], &pr.yc[s]);
      pr.w[s] = wc ? ((wc[3 * i] + wc[3 * i + 1]) + wc[3 * i + 2]) * (1.f / 3.f) : wts ? wts[i] : 1.f;
      if (lastv) pr.last[s] = lastv[i];
      lmax = max(lmax, pr.last[s]);
    }
  }
  return uniform(wave_max_i(lmax));
}

// ------------------------------------------------------------ tile schedule
// A tile's cost in the derivative walks is its walk length: the number of
// (sampled pixel, 64-entry chunk) steps, i.e. the sum over its pixels of the
// chunks up to the pixel's last blended entry. Within one view batch it
// ranges from 0 (empty tiles, often most of an object-centred image) to
// hundreds, and one wave per tile in grid order leaves some SIMDs with twice
// the mean work while others idle. The derivative kernels therefore run a
// persistent grid whose waves take tiles from a shared ticket counter in
// order of decreasing walk length (list scheduling: longest first, then
// whoever is free takes the next), which keeps every SIMD busy to the end.
// Cutting long tiles into parts over their pixels was tried and is slower:
// every part walks the list chunks again and flushes its own atomics.
//
// sched = [order (tiles) | walk length (tiles) | ticket, finished, busy, 0].
constexpr int kSchedBins = 1024;
constexpr int kSchedThreads = 1024;
constexpr int kSchedUnroll = 8;

struct SchedRef {
  const int32_t* order;
  int32_t* ctr;
  int tiles;
};

__device__ __forceinline__ SchedRef sched_ref(int32_t* sched, int tiles) {
  return SchedRef{sched, sched + 2 * (int64_t)tiles, tiles};
}

// Tiles handed out by one persistent launch: every tile, or (for the walks
// that do nothing on a tile without blended entries) only the busy ones,
// which the schedule puts first.
__device__ __forceinline__ int sched_count(const SchedRef& sr, bool busy_only) {
  return busy_only ? min(max(sr.ctr[2], 0), sr.tiles) : sr.tiles;
}

// Next tile of this wave, -1 when the launch has run out of tickets, -2 for
// an entry that is not a tile of this frame (skipped).
__device__ __forceinline__ int sched_next(const SchedRef& sr, int count) {
  int t = 0;
  if (lane_id() == 0) t = atomicAdd(sr.ctr, 1);
  t = readlane(t, 0);
  if (t < 0 || t >= count) return -1;
  const int tile = sr.order[t];
  return (unsigned)tile < (unsigned)sr.tiles ? tile : -2;
}

// Called once by every wave of the launch: the last wave to finish returns
// the counters to zero for the next launch on the frame.
__device__ __forceinline__ void sched_finish(const SchedRef& sr) {
  if (lane_id() == 0) {
    if (atomicAdd(sr.ctr + 1, 1) == (int)gridDim.x - 1) {
      atomicExch(sr.ctr, 0);
      atomicExch(sr.ctr + 1, 0);
    }
  }
}

// The same for a workgroup whose waves share one tile: one thread takes the
// ticket (the caller broadcasts it) and signs the workgroup off.
__device__ __forceinline__ int sched_take(const SchedRef& sr, int count) {
  const int t = atomicAdd(sr.ctr, 1);
  if (t < 0 || t >= count) return -1;
  const int tile = sr.order[t];
  return (unsigned)tile < (unsigned)sr.tiles ? tile : -2;
}
__device__ __forceinline__ void sched_sign_off(const SchedRef& sr) {
  if (atomicAdd(sr.ctr + 1, 1) == (int)gridDim.x - 1) {
    atomicExch(sr.ctr, 0);
    atomicExch(sr.ctr + 1, 0);
  }
}

// Bin of a walk length, 0 = longest: exact below 512, then 16 per bin.
__device__ __forceinline__ int sched_bin(int len) {
  const int key = len < 512 ? len : min(kSchedBins - 1, 512 + ((len - 512) >> 4));
  return kSchedBins - 1 - key;
}

// One workgroup: counting sort of the tiles by walk-length bin (descending),
// then the counters for the launches that follow.
__global__ __launch_bounds__(kSchedThreads) void sched_kernel(int32_t* __restrict__ sched, int tiles) {
  __shared__ int hist[kSchedBins];
  __shared__ int wsum[kSchedThreads / kWave];
  const int tid = threadIdx.x;
  const int32_t* len = sched + tiles;
  hist[tid] = 0;
  __syncthreads();
  for (int base = 0; base < tiles; base += kSchedThreads * kSchedUnroll) {
    int b[kSchedUnroll];
#pragma unroll
    for (int u = 0; u < kSchedUnroll; ++u) {
      const int i = base + u * kSchedThreads + tid;
      b[u] = i < tiles ? sched_bin(max(len[i], 0)) : -1;
    }
    // empty tiles (often most of them) all fall in the last bin: counted
    // per wave by ballot rather than by one LDS atomic each on one address
#pragma unroll
    for (int u = 0; u < kSchedUnroll; ++u) {
      const uint64_t empty = __ballot(b[u] == kSchedBins - 1);
      if (b[u] >= 0 && b[u] != kSchedBins - 1) atomicAdd(&hist[b[u]], 1);
      if (lane_id() == 0 && empty) atomicAdd(&hist[kSchedBins - 1], __popcll(empty));
    }
  }
  __syncthreads();
  const int own = hist[tid];
  int x = own;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int y = __shfl_up(x, d, kWave);
    if ((tid & (kWave - 1)) >= d) x += y;
  }
  if ((tid & (kWave - 1)) == kWave - 1) wsum[tid / kWave] = x;
  __syncthreads();
  for (int w = 0; w < tid / kWave; ++w) x += wsum[w];
  hist[tid] = x - own;  // first position of this bin
  __syncthreads();
  for (int base = 0; base < tiles; base += kSchedThreads * kSchedUnroll) {
    int b[kSchedUnroll];
#pragma unroll
    for (int u = 0; u < kSchedUnroll; ++u) {
      const int i = base + u * kSchedThreads + tid;
      b[u] = i < tiles ? sched_bin(max(len[i], 0)) : -1;
    }
#pragma unroll
    for (int u = 0; u < kSchedUnroll; ++u) {
      const int i = base + u * kSchedThreads + tid;
      const uint64_t empty = __ballot(b[u] == kSchedBins - 1);
      if (b[u] >= 0 && b[u] != kSchedBins - 1) sched[atomicAdd(&hist[b[u]], 1)] = i;
      int first = 0;
      if (lane_id() == 0 && empty) first = atomicAdd(&hist[kSchedBins - 1], __popcll(empty));
      first = readlane(first, 0);
      if (b[u] == kSchedBins - 1) sched[first + __popcll(empty & ((1ull << lane_id()) - 1ull))] = i;
    }
  }
  if (tid == kSchedBins - 1) {  // the last bin holds the tiles with walk length 0
    int32_t* ctr = sched + 2 * (int64_t)tiles;
    atomicExch(ctr, 0);
    atomicExch(ctr + 1, 0);
    atomicExch(ctr + 2, tiles - own);
    atomicExch(ctr + 3, 0);
  }
}

// ------------------------------------------------------------------ render
// Colour (with background), final transmittance and last blended position of
// every sampled pixel, and the tile's walk length for the schedule.
// score_kernel below: for every pixel only its residual magnitude
// |C_R - I_R| + |C_G - I_G| + |C_B - I_B| against the target image of its
// camera, for the residual-weighted sampler.
struct ScoreOut {
  const float* targets;     // [cameras][H][W][3]
  const int32_t* view_ids;  // [V] or NULL
  int W, H;
  float* score;             // [V][T][256], or the image [V][H][W][3]
};

// What score_kernel writes per pixel.
enum ScoreMode { kScoreResidual = 0, kScoreCount = 1, kScoreImage = 2 };

// W waves share a tile; wave wv renders the sample slots j with j % W == wv.
// With one slot of pixels and MP > 1 (at most MP pixels per wave), each lane
// keeps its entry's colour contribution to each of the wave's pixels in
// registers and the wave sums them once at the end, instead of three wave
// sums per step.
template <int NS, int W, int MP>
__global__ __launch_bounds__(kWave* W) void render_kernel(const float* __restrict__ rec,
                                                       const int64_t* __restrict__ tile_start,
                                                       const int32_t* __restrict__ ids,
                                                       const uint8_t* __restrict__ pix, int n, int T,
                                                       int TX, int k, lmrs_render_opts o,
                                                       float* __restrict__ color, float* __restrict__ trans,
                                                       int32_t* __restrict__ last,
                                                       int32_t* __restrict__ walk_len,
                                                       int64_t* __restrict__ pair_count) {
  const int lane = lane_id();
  const int wv = uniform((int)(threadIdx.x / kWave));
  const bool mine = (lane & (W - 1)) == wv;
  const TileCtx c = tile_ctx(tile_start, T, TX, blockIdx.x);
  PixelRegs<NS> pr;
  load_pixel_regs<NS>(pix, nullptr, nullptr, nullptr, k, c, pr);
  float sT[NS], sC0[NS], sC1[NS], sC2[NS];
  int sLast[NS], sDone[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    sT[s] = 1.f;
    sC0[s] = sC1[s] = sC2[s] = 0.f;
    sLast[s] = -1;
    sDone[s] = 0;
  }
  constexpr bool ACC = NS == 1 && MP > 1;
  float A0[ACC ? MP : 1], A1[ACC ? MP : 1], A2[ACC ? MP : 1];
#pragma unroll
  for (int m = 0; m < (ACC ? MP : 1); ++m) A0[m] = A1[m] = A2[m] = 0.f;
  int remaining = k / W + (wv < k % W ? 1 : 0);  // this wave's pixels
  int npairs = 0;  // blending (pixel, entry) pairs of this wave's pixels
  for (int c0 = 0; c0 < c.len && remaining > 0; c0 += kWave) {
    const bool valid = c0 + lane < c.len;
    RecF r{};
    if (valid) r = load_rec(rec, (size_t)c.v * n + ids[c.start + c0 + lane]);
    // pixel l of slot s (accumulator m in the accumulator path) against the chunk
    auto step = [&](int s, int l, int m) {
      const Alpha al = pair_alpha(r.u, r.v, r.f11, r.f12, r.f22, r.o, readlane(pr.xc[s], l), readlane(pr.yc[s], l), o);
      const bool inc = valid && al.inc;
      const float a = inc ? al.a : 0.f;
      const float om = inc ? 1.f - a : 1.f;
      const float Tc = readlane(sT[s], l);
      const float Taft = Tc * scan_mul(om);  // T behind this entry
      // first entry whose blending would take T below t_min
      const uint64_t stop = __ballot(inc && Taft < o.t_min);
      const int f = stop ? __ffsll((unsigned long long)stop) - 1 : kWave;
      const bool ok = inc && lane < f;
      const float Tex = Taft * __builtin_amdgcn_rcpf(om);  // T in front of it
      const float wgt = ok ? a * Tex : 0.f;
      if (ACC) {
        A0[m] += wgt * r.r;
        A1[m] += wgt * r.g;
        A2[m] += wgt * r.b;
      } else {
        const float cr = wave_total(wgt * r.r), cg = wave_total(wgt * r.g), cb = wave_total(wgt * r.b);
        sC0[s] = writelane(sC0[s], readlane(sC0[s], l) + cr, l);
        sC1[s] = writelane(sC1[s], readlane(sC1[s], l) + cg, l);
        sC2[s] = writelane(sC2[s], readlane(sC2[s], l) + cb, l);
      }
      const uint64_t okm = __ballot(ok);
      npairs += __popcll(okm);
      const float Tnext = f < kWave ? readlane(Tex, f) : readlane(Taft, kWave - 1);
      sT[s] = writelane(sT[s], Tnext, l);
      if (okm) sLast[s] = writelane(sLast[s], c0 + 63 - __clzll((long long)okm), l);
      if (f < kWave) {
        sDone[s] = writelane(sDone[s], 1, l);
        --remaining;
      }
    };
    if (ACC) {
#pragma unroll
      for (int m = 0; m < (ACC ? MP : 1); ++m) {
        const int l = wv + m * W;
        if (l < k && !readlane(sDone[0], l)) step(0, l, m);
      }
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int cnt = min(kWave, k - s * kWave);
        for (int l = wv; l < cnt; l += W)
          if (!readlane(sDone[s], l)) step(s, l, 0);
      }
    }
  }
  if (ACC) {
#pragma unroll
    for (int m = 0; m < (ACC ? MP : 1); ++m) {
      const int l = wv + m * W;
      if (l >= k) break;
      sC0[0] = writelane(sC0[0], wave_total(A0[m]), l);
      sC1[0] = writelane(sC1[0], wave_total(A1[m]), l);
      sC2[0] = writelane(sC2[0], wave_total(A2[m]), l);
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int j = s * kWave + lane;
    if (j < k && mine) {
      const int64_t i = c.tile_lin * k + j;
      color[3 * i] = sC0[s] + sT[s] * o.bg[0];
      color[3 * i + 1] = sC1[s] + sT[s] * o.bg[1];
      color[3 * i + 2] = sC2[s] + sT[s] * o.bg[2];
      trans[i] = sT[s];
      last[i] = sLast[s];
    }
  }
  int steps = 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) steps += mine && sLast[s] >= 0 ? sLast[s] / kWave + 1 : 0;
  __shared__ float part[W];
  __shared__ int part_pairs[W];
  const float total = wave_total((float)steps);  // a sort key: exact up to 2^24 steps
  if (lane == 0) {
    part[wv] = total;
    part_pairs[wv] = npairs;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float sum = 0.f;
    int64_t pairs = 0;
    for (int w = 0; w < W; ++w) {
      sum += part[w];
      pairs += part_pairs[w];
    }
    walk_len[c.tile_lin] = (int32_t)sum;
    if (pair_count) pair_count[c.tile_lin] = pairs;
  }
}

// Blend-table offsets: the per-tile pair counts the render wrote into
// start[0, m) become exclusive offsets; start[m] = total, start[m + 1] = 0
// (the table is stale until the reverse walk rebuilds it). One workgroup;
// each thread scans a contiguous block of tiles.
constexpr int kBlendScanThreads = 1024;
constexpr int kBlendScanPer = 8;  // consecutive counts per thread and round
// One workgroup: exclusive scan of the tiles' pair counts in place, in
// rounds of kBlendScanThreads * kBlendScanPer counts (each thread reads its
// counts as one coalesced block), with a running carry between rounds;
// start[m] = total pairs, start[m + 1] = 0 (the table is not built yet).
__global__ __launch_bounds__(kBlendScanThreads) void blend_scan_kernel(int64_t* __restrict__ start, int64_t m) {
  __shared__ int64_t s_wave[kBlendScanThreads / kWave];
  __shared__ int64_t s_carry;
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < m; base += (int64_t)kBlendScanThreads * kBlendScanPer) {
    const int64_t a = base + (int64_t)tid * kBlendScanPer;
    int64_t x[kBlendScanPer];
    int64_t acc = 0;
#pragma unroll
    for (int q = 0; q < kBlendScanPer; ++q) {
      x[q] = a + q < m ? start[a + q] : 0;
      acc += x[q];
    }
    int64_t y = acc;  // inclusive scan over the wave
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int64_t z = __shfl_up(y, d, kWave);
      if (lane >= d) y += z;
    }
    if (lane == kWave - 1) s_wave[wv] = y;
    __syncthreads();
    int64_t before = s_carry;
    for (int w = 0; w < wv; ++w) before += s_wave[w];
    int64_t run = before + (y - acc);
#pragma unroll
    for (int q = 0; q < kBlendScanPer; ++q) {
      if (a + q < m) start[a + q] = run;
      run += x[q];
    }
    __syncthreads();  // s_wave and s_carry have been read
    if (tid == kBlendScanThreads - 1) s_carry = before + y;
    __syncthreads();
  }
  if (tid == 0) {
    start[m] = s_carry;
    start[m + 1] = 0;
  }
}

// Residual scores of every pixel (lmrs_residual_scores). With all 256 pixels
// of a tile to render, a lane per pixel needs about half the instructions
// per (pixel, entry) pair of the entry-per-lane walk, which pays prefix
// scans and three wave sums per pixel step: thread j blends pixel j, the
// list's records pass through LDS 256 at a time (one loaded per thread, the
// next chunk's while this one is blended) and every lane reads the same
// record at once (an LDS broadcast). A pixel stops where the walk above
// stops it (the first entry that would take T below t_min), here with the
// transmittance multiplied entry by entry; a wave leaves a chunk when all
// its pixels have stopped, the workgroup its list when all 256 have.
// kScoreCount writes instead the number of Gaussians blended into each pixel
// (the G_p of the contribution-weighted sampler, Supp. E eq. 17), kScoreImage
// the rendered colour (background added) into a [V][H][W][3] image.
constexpr int kScoreThreads = 256;

template <int MODE>
__global__ __launch_bounds__(kScoreThreads) void score_kernel(const float* __restrict__ rec,
                                                              const int64_t* __restrict__ tile_start,
                                                              const int32_t* __restrict__ ids, int n, int T,
                                                              int TX, lmrs_render_opts o, ScoreOut so) {
  __shared__ float4 s_rec[kScoreThreads * 3];
  const int tid = threadIdx.x;
  const TileCtx c = tile_ctx(tile_start, T, TX, blockIdx.x);
  const float xc = c.ox + (float)(tid & 15) + 0.5f, yc = c.oy + (float)(tid >> 4) + 0.5f;
  const float4* rec4 = reinterpret_cast<const float4*>(rec);
  const size_t vb = (size_t)c.v * n;
  float Tr = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  int blended = 0;
  bool done = false;
  float4 q0{}, q1{}, q2{};
  if (tid < c.len) {
    const size_t g = (vb + (size_t)ids[c.start + tid]) * 3;
    q0 = rec4[g];
    q1 = rec4[g + 1];
    q2 = rec4[g + 2];
  }
  for (int64_t c0 = 0; c0 < c.len; c0 += kScoreThreads) {
    __syncthreads();  // the previous chunk has been read
    s_rec[3 * tid] = q0;
    s_rec[3 * tid + 1] = q1;
    s_rec[3 * tid + 2] = q2;
    __syncthreads();
    if (c0 + kScoreThreads + tid < c.len) {
      const size_t g = (vb + (size_t)ids[c.start + c0 + kScoreThreads + tid]) * 3;
      q0 = rec4[g];
      q1 = rec4[g + 1];
      q2 = rec4[g + 2];
    }
    const int cnt = (int)min<int64_t>(kScoreThreads, c.len - c0);
    if (!done) {
      for (int e = 0; e < cnt; ++e) {
        const float4 a = s_rec[3 * e], b = s_rec[3 * e + 1];
        const float cb = s_rec[3 * e + 2].x;
        const Alpha al = pair_alpha(a.x, a.y, a.z, a.w, b.x, b.y, xc, yc, o);
        if (al.inc) {
          const float Tn = Tr * (1.f - al.a);
          if (Tn < o.t_min) {
            done = true;
            break;
          }
          const float wgt = al.a * Tr;
          C0 += wgt * b.z;
          C1 += wgt * b.w;
          C2 += wgt * cb;
          Tr = Tn;
          ++blended;
        }
      }
    }
    if (__syncthreads_and(done)) break;
  }
  if (MODE == kScoreCount) {
    so.score[c.tile_lin * 256 + tid] = (float)blended;
    return;
  }
  const int x = (c.t % TX) * kTile + (tid & 15), y = (c.t / TX) * kTile + (tid >> 4);
  const float r0 = C0 + Tr * o.bg[0], r1 = C1 + Tr * o.bg[1], r2 = C2 + Tr * o.bg[2];
  if (MODE == kScoreImage) {
    float* px = so.score + (((int64_t)c.v * so.H + y) * so.W + x) * 3;
    px[0] = r0;
    px[1] = r1;
    px[2] = r2;
    return;
  }
  const int cam = so.view_ids ? so.view_ids[c.v] : c.v;
  const float* tg = so.targets + (((int64_t)cam * so.H + y) * so.W + x) * 3;
  so.score[c.tile_lin * 256 + tid] = (fabsf(r0 - tg[0]) + fabsf(r1 - tg[1])) + fabsf(r2 - tg[2]);
}

// ----------------------------------------------------- J p, J^T u, fused GN
// LDS of one reverse-walk chunk of a W-wave workgroup: the waves' partial
// gradients (rows of 65 floats per (wave, component)) and the chunk's ids.
template <int W>
constexpr int kRedBuf = W * 9 * (kWave + 1) + kWave;

// One forward step: pixel (xc, yc) (transmittance Tc and its tangent dTc in
// front of the chunk, last blended entry lj) against the chunk's entries, one
// per lane. cr/cg/cb: this lane's entry's term of the colour tangent; tp / tq:
// the chunk's transmittance product and the sum of its tangent ratios.
struct FwdStep {
  float cr, cg, cb, Tc, dTc, tp, tq;
};

__device__ __forceinline__ FwdStep fwd_step(const RecF& r, const RecF& dr, int e, bool valid, int lj, float xc,
                                            float yc, float Tc, float dTc, const lmrs_render_opts& o) {
  // written with selects only (no per-lane branches), so that the steps of
  // several pixels can share one basic block
  const Alpha al = pair_alpha(r.u, r.v, r.f11, r.f12, r.f22, r.o, xc, yc, o);
  const bool inc = valid && e <= lj && al.inc;
  const float a = inc ? al.a : 0.f;
  const float ds = -al.q1 * (dr.f11 * al.dx + dr.f12 * al.dy + r.f11 * dr.u + r.f12 * dr.v) -
                   al.q2 * (dr.f22 * al.dy + r.f22 * dr.v);
  const float da = inc && !al.capped ? al.es * (dr.o + r.o * ds) : 0.f;
  const float om = inc ? 1.f - a : 1.f;
  const float rom = __builtin_amdgcn_rcpf(om);
  const float q = inc ? -da * rom : 0.f;
  const float Pinc = scan_mul(om);  // product of (1 - alpha) up to and including this entry
  const float Qinc = scan_add(q);
  const float pin = Pinc * rom;  // product of (1 - alpha) in front, within the chunk
  const float Tn = Tc * pin;
  const float dTn = pin * (dTc + Tc * (Qinc - q));
  const float aT = a * Tn, gT = da * Tn + a * dTn;
  FwdStep st;
  st.cr = inc ? dr.r * aT + r.r * gT : 0.f;
  st.cg = inc ? dr.g * aT + r.g * gT : 0.f;
  st.cb = inc ? dr.b * aT + r.b * gT : 0.f;
  st.Tc = Tc;
  st.dTc = dTc;
  st.tp = readlane(Pinc, kWave - 1);
  st.tq = readlane(Qinc, kWave - 1);
  return st;
}

// MODE 1: jp = J p.  MODE 2: grad2d += J^T u.  MODE 3: grad2d += J^T W J p.
//
// W waves share a tile. With one slot of pixels (NS == 1) and at most MP
// pixels per wave (MP > 1), the tile's pixels are dealt by depth: ranked by
// last blended entry (deepest first, ties by slot), the first ranks go to
// wave 0, the next to wave 1, and so on, so that the pixels of a wave walk
// about as far as each other and a wave stops at its own deepest pixel.
// Wave wv's pixel m is slot px[m] with last entry pl[m] (-1 for m past its
// pixels). Otherwise slot j goes to wave j % W. Each wave keeps the state of
// its pixels in its own registers from the forward walk to the reverse walk.
template <int MODE, int NS, int W, int MP>
__device__ __forceinline__ void deriv_tile(
    const float* __restrict__ rec, const float* __restrict__ tan, const int64_t* __restrict__ tile_start,
    const int32_t* __restrict__ ids, const uint8_t* __restrict__ pix, const float* __restrict__ wts,
    const float* __restrict__ wc, const float* __restrict__ trans, const int32_t* __restrict__ lastv, int n,
    int T, int TX, int k, const lmrs_render_opts& o, const float* __restrict__ u_in, float* __restrict__ jp_out,
    float* __restrict__ grad2d, bool fixed, int64_t tile_lin, int wv, float* red) {
  constexpr bool FWD = MODE != 2;
  constexpr bool REV = MODE != 1;
  constexpr bool DEALT = W > 1 && NS == 1 && MP > 1;
  const int lane = lane_id();
  const TileCtx c = tile_ctx(tile_start, T, TX, tile_lin);
  PixelRegs<NS> pr;
  const int lmax = load_pixel_regs<NS>(pix, wts, nullptr, lastv, k, c, pr);
  int px[DEALT ? MP : 1], pl[DEALT ? MP : 1];
  bool own[NS];
  int lmax_own;
  if (DEALT) {
    // rank of this lane's pixel; wave w takes ranks [first_w, first_w + count_w)
    const int my_last = pr.last[0];
    int rank = 0;
    for (int q = 0; q < k; ++q) {
      const int lq = readlane(pr.last[0], q);
      rank += lq > my_last || (lq == my_last && q < lane) ? 1 : 0;
    }
    const int base = k / W, extra = k % W;
    const int first = wv * base + min(wv, extra), cnt = base + (wv < extra ? 1 : 0);
    own[0] = lane < k && rank >= first && rank < first + cnt;
#pragma unroll
    for (int m = 0; m < MP; ++m) {
      const uint64_t b = __ballot(lane < k && rank == first + m && m < cnt);
      px[m] = b ? __ffsll((unsigned long long)b) - 1 : 0;
      pl[m] = b ? readlane(pr.last[0], px[m]) : -1;
    }
    lmax_own = pl[0];
  } else {
    int lm_own = -1;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      own[s] = s * kWave + lane < k && (lane & (W - 1)) == wv;
      if (own[s]) lm_own = max(lm_own, pr.last[s]);
    }
    lmax_own = uniform(wave_max_i(lm_own));
    px[0] = pl[0] = 0;
  }
  // forward: a = T in front of the chunk, b = its tangent, u0..u2 = d colour
  // reverse: a = T behind the chunk range already walked, b = u . (colour behind + T_final bg), u = weights
  float sa[NS], sb[NS], su0[NS], su1[NS], su2[NS];

  if (FWD) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      sa[s] = 1.f;
      sb[s] = su0[s] = su1[s] = su2[s] = 0.f;
    }
    // With dealt pixels each lane keeps its entry's colour-tangent
    // contribution to each of the wave's pixels in registers (A[m] for the
    // wave's pixel m) and the wave sums them once after the walk, instead
    // of three wave sums per step.
    float A0[DEALT ? MP : 1], A1[DEALT ? MP : 1], A2[DEALT ? MP : 1];
#pragma unroll
    for (int m = 0; m < (DEALT ? MP : 1); ++m) A0[m] = A1[m] = A2[m] = 0.f;
    // the next chunk's records and tangents and the list ids of the one
    // after load while a chunk is walked
    RecF rn{}, drn{};
    {
      const int id0 = fwd_chunk_id(ids, c, 0);
      if (lmax_own >= 0 && id0 >= 0) {
        rn = load_rec(rec, (size_t)c.v * n + id0);
        drn = load_rec(tan, (size_t)c.v * n + id0);
      }
    }
    int idn = lmax_own >= kWave ? fwd_chunk_id(ids, c, kWave) : -1;
    for (int c0 = 0; c0 <= lmax_own; c0 += kWave) {
      const int e = c0 + lane;
      const bool valid = e < c.len;
      const RecF r = rn, dr = drn;
      rn = RecF{};
      drn = RecF{};
      if (idn >= 0) {
        rn = load_rec(rec, (size_t)c.v * n + idn);
        drn = load_rec(tan, (size_t)c.v * n + idn);
      }
      idn = c0 + 2 * kWave <= lmax_own ? fwd_chunk_id(ids, c, c0 + 2 * kWave) : -1;
      if (DEALT) {
#pragma unroll
        for (int m = 0; m < MP; ++m) {
          // no branches: for a pixel past its last entry (or a slot without
          // a pixel, last -1) the step adds nothing and leaves T and its
          // tangent as they are, and the steps of the wave's pixels form
          // one block that the compiler can interleave
          const int l = px[m];
          const FwdStep st = fwd_step(r, dr, e, valid, pl[m], readlane(pr.xc[0], l), readlane(pr.yc[0], l),
                                      readlane(sa[0], l), readlane(sb[0], l), o);
          A0[m] += st.cr;
          A1[m] += st.cg;
          A2[m] += st.cb;
          sa[0] = writelane(sa[0], st.Tc * st.tp, l);
          sb[0] = writelane(sb[0], st.tp * (st.dTc + st.Tc * st.tq), l);
        }
      } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int cnt = min(kWave, k - s * kWave);
          for (int l = wv; l < cnt; l += W) {
            const int lj = readlane(pr.last[s], l);
            if (c0 > lj) continue;
            const FwdStep st = fwd_step(r, dr, e, valid, lj, readlane(pr.xc[s], l), readlane(pr.yc[s], l),
                                        readlane(sa[s], l), readlane(sb[s], l), o);
            su0[s] = writelane(su0[s], readlane(su0[s], l) + wave_total(st.cr), l);
            su1[s] = writelane(su1[s], readlane(su1[s], l) + wave_total(st.cg), l);
            su2[s] = writelane(su2[s], readlane(su2[s], l) + wave_total(st.cb), l);
            sa[s] = writelane(sa[s], st.Tc * st.tp, l);
            sb[s] = writelane(sb[s], st.tp * (st.dTc + st.Tc * st.tq), l);
          }
        }
      }
    }
    if (DEALT) {
#pragma unroll
      for (int m = 0; m < MP; ++m) {
        if (pl[m] < 0) break;  // no blended entry (or no pixel): the tangent stays 0
        su0[0] = writelane(su0[0], wave_total(A0[m]), px[m]);
        su1[0] = writelane(su1[0], wave_total(A1[m]), px[m]);
        su2[0] = writelane(su2[0], wave_total(A2[m]), px[m]);
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int j = s * kWave + lane;
      const float d0 = su0[s] + o.bg[0] * sb[s], d1 = su1[s] + o.bg[1] * sb[s], d2 = su2[s] + o.bg[2] * sb[s];
      if (MODE == 1) {
        if (own[s]) {
          const int64_t i = c.tile_lin * k + j;
          jp_out[3 * i] = d0;
          jp_out[3 * i + 1] = d1;
          jp_out[3 * i + 2] = d2;
        }
      } else if (wc) {  // per-channel operator weights
        float w0 = 0.f, w1 = 0.f, w2 = 0.f;
        if (j < k) {
          const int64_t i = c.tile_lin * k + j;
          w0 = wc[3 * i];
          w1 = wc[3 * i + 1];
          w2 = wc[3 * i + 2];
        }
        su0[s] = w0 * d0;
        su1[s] = w1 * d1;
        su2[s] = w2 * d2;
      } else {
        su0[s] = pr.w[s] * d0;
        su1[s] = pr.w[s] * d1;
        su2[s] = pr.w[s] * d2;
      }
    }
  }

  if (REV) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int j = s * kWave + lane;
      if (j < k) {
        const int64_t i = c.tile_lin * k + j;
        if (!FWD) {
          su0[s] = u_in[3 * i];
          su1[s] = u_in[3 * i + 1];
          su2[s] = u_in[3 * i + 2];
        }
        sa[s] = trans[i];
      } else {
        if (!FWD) su0[s] = su1[s] = su2[s] = 0.f;
        sa[s] = 0.f;
      }
      sb[s] = sa[s] * (su0[s] * o.bg[0] + su1[s] * o.bg[1] + su2[s] * o.bg[2]);
    }
    if (lmax < 0) return;  // the same for every wave of the workgroup
    int chunk = 0;
    // reversed: lane 0 holds the chunk's deepest entry. The next chunk's
    // records and the list ids of the one after load while a chunk is walked.
    const int ctop = (lmax / kWave) * kWave;
    int idc = rev_chunk_id(ids, c, ctop);
    RecF rn{};
    if (idc >= 0) rn = load_rec(rec, (size_t)c.v * n + idc);
    int idn = ctop >= kWave ? rev_chunk_id(ids, c, ctop - kWave) : -1;
    landed(rn);  // so that no path reaches the loop head with a load pending
    landed(idn);
    for (int c0 = ctop; c0 >= 0; c0 -= kWave) {
      const int e = c0 + (kWave - 1 - lane);
      const bool valid = e < c.len;
      const RecF r = rn;
      const int id = max(idc, 0);
      rn = RecF{};
      if (idn >= 0) rn = load_rec(rec, (size_t)c.v * n + idn);
      idc = idn;
      idn = c0 >= 2 * kWave ? rev_chunk_id(ids, c, c0 - 2 * kWave) : -1;
      float g[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      // one pixel (slot s, lane l, last entry lj) against the chunk
      auto rev_step = [&](int s, int l, int lj) {
        const Alpha al =
            pair_alpha(r.u, r.v, r.f11, r.f12, r.f22, r.o, readlane(pr.xc[s], l), readlane(pr.yc[s], l), o);
        const bool inc = valid && e <= lj && al.inc;
        const float a = inc ? al.a : 0.f;
        // product of (1 - alpha) over this entry and the ones behind it in the chunk
        const float rP = __builtin_amdgcn_rcpf(scan_mul(inc ? 1.f - a : 1.f));
        const float Tafter = readlane(sa[s], l);
        const float Tn = Tafter * rP;
        const float u0 = readlane(su0[s], l), u1 = readlane(su1[s], l), u2 = readlane(su2[s], l);
        const float urgb = u0 * r.r + u1 * r.g + u2 * r.b;
        const float term = inc ? urgb * a * Tn : 0.f;
        const float Sinc = scan_add(term);
        const float S = readlane(sb[s], l);
        if (inc) {
          const float aT = a * Tn;
          g[6] += u0 * aT;
          g[7] += u1 * aT;
          g[8] += u2 * aT;
          if (!al.capped) {
            const float behind = S + (Sinc - term);
            const float ga = Tn * urgb - behind * __builtin_amdgcn_rcpf(1.f - a);
            const float gs = ga * a;
            g[5] += ga * al.es;
            g[0] -= gs * (al.q1 * r.f11);
            g[1] -= gs * (al.q1 * r.f12 + al.q2 * r.f22);
            g[2] -= gs * (al.q1 * al.dx);
            g[3] -= gs * (al.q1 * al.dy);
            g[4] -= gs * (al.q2 * al.dy);
          }
        }
        sa[s] = writelane(sa[s], Tafter * readlane(rP, kWave - 1), l);
        sb[s] = writelane(sb[s], S + readlane(Sinc, kWave - 1), l);
      };
      if (DEALT) {
#pragma unroll
        for (int m = 0; m < MP; ++m)
          if (c0 <= pl[m]) rev_step(0, px[m], pl[m]);
      } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int cnt = min(kWave, k - s * kWave);
          for (int l = wv; l < cnt; l += W) {
            const int lj = readlane(pr.last[s], l);
            if (c0 <= lj) rev_step(s, l, lj);
          }
        }
      }
      // the waves' partial gradients of each entry meet in LDS (double
      // buffered by chunk, so one barrier per chunk); wave wv adds up and
      // flushes components wv, wv + W, ...
      float* buf = red + (chunk & 1) * kRedBuf<W>;
#pragma unroll
      for (int q = 0; q < 9; ++q) buf[(wv * 9 + q) * (kWave + 1) + lane] = g[q];
      if (wv == 0) reinterpret_cast<int*>(buf + W * 9 * (kWave + 1))[lane] = valid ? id : -1;
      landed(rn);
      landed(idn);
      __syncthreads();
      // flush transposed: an atomic instruction covers 4 entries with 16 lanes
      // each (their 9 components), i.e. 4 gradient rows of 64 bytes
      const int* ent_id = reinterpret_cast<const int*>(buf + W * 9 * (kWave + 1));
      const int q = lane & (kGradRow - 1);
      for (int t = wv; t < kWave / 4; t += W) {
        const int ent = 4 * t + (lane >> 4);
        const int ide = ent_id[ent];
        float sum = 0.f;
        if (q < 9) {
#pragma unroll
          for (int w = 0; w < W; ++w) sum += buf[(w * 9 + q) * (kWave + 1) + ent];
        }
        if (ide >= 0 && q < 9 && sum != 0.f) grad_add(grad2d, fixed, (size_t)c.v * n + ide, q, sum);
      }
      ++chunk;
    }
  }
}

// Persistent grid over the tile schedule; J p visits every tile (it writes
// every sample), the reverse walks only tiles with blended entries. A
// workgroup of W waves takes one tile at a time and deals its sampled pixels
// to the waves (deriv_tile): more waves per SIMD without cutting the work
// into more, smaller items. W and MP are chosen from the samples per tile
// (launch_deriv).
template <int MODE, int NS, int W, int MP>
__global__ __launch_bounds__(kWave* W) void deriv_kernel(
    const float* __restrict__ rec, const float* __restrict__ tan, const int64_t* __restrict__ tile_start,
    const int32_t* __restrict__ ids, const uint8_t* __restrict__ pix, const float* __restrict__ wts,
    const float* __restrict__ wc, const float* __restrict__ trans, const int32_t* __restrict__ lastv, int n,
    int T, int TX, int k, lmrs_render_opts o, const float* __restrict__ u_in, float* __restrict__ jp_out,
    float* __restrict__ grad2d, bool fixed, int32_t* __restrict__ sched, int tiles,
    const int64_t* __restrict__ built) {
  __shared__ int next_tile[2];
  __shared__ float red[MODE == 1 ? 1 : 2 * kRedBuf<W>];
  if (built && *built == 1) return;  // the blend table holds this render: blend_gn_kernel ran instead
  const int wv = uniform((int)(threadIdx.x / kWave));
  const SchedRef sr = sched_ref(sched, tiles);
  const int count = sched_count(sr, MODE != 1);
  for (int it = 0;; ++it) {
    // double buffered: a slot is rewritten two tickets later, after every
    // wave has passed the barrier of the ticket in between
    if (threadIdx.x == 0) next_tile[it & 1] = sched_take(sr, count);
    __syncthreads();
    const int tile = next_tile[it & 1];
    if (tile == -1) break;
    if (tile >= 0)
      deriv_tile<MODE, NS, W, MP>(rec, tan, tile_start, ids, pix, wts, wc, trans, lastv, n, T, TX, k, o, u_in,
                                  jp_out, grad2d, fixed, tile, wv, red);
  }
  if (threadIdx.x == 0) sched_sign_off(sr);
}

// --------------------------------------------------------------- Gram
// Per (view, Gaussian) weighted Gram of d C_c / d rec over the tile's pixels
// and channels: geometry block, geometry x colour, colour, opacity. Walks
// like the reverse pass of deriv_kernel, with one "colour behind" per channel.
// With VJP it also forms J^T u (u = u_in, e.g. the weighted residuals) on the
// same walk: the colour behind an entry seen through u is sum_c u_c times the
// per-channel colour behind, so the right-hand side b = J^T W r of an LM step
// costs no walk of its own.
//
// With a blend table to fill (BlendOut::on) the walk also writes one record
// per blending (pixel, entry) pair: K = d C / d alpha per channel (the
// quantity ga below; 0 when alpha is capped) and alpha T, with the Gaussian
// id and the sample slot, twice. A tile's pairs start at blend_start[tile],
// the chunks back to front; inside a chunk's block the first copy is grouped
// by entry (an entry's pixels in slot order; each entry's pairs form runs of
// at most kBlendRun, whose starts go to blend_run), the second, at offset
// blend_capacity, by pixel (a pixel's entries in lane order). A first pass
// over the chunk's pixels counts each entry's pairs so that every lane knows
// where its entry-grouped pairs go; the pixel-grouped ones follow from a
// ballot per pixel.
constexpr int kBlendRun = 32;

struct BlendOut {
  float4* k;
  uint32_t* m;
  int32_t* run;
  int32_t* runs;
  const int64_t* start;
  bool on;
  int64_t pix_major;  // offset of the pixel-major copy in k and m (the capacity)
};

__device__ __forceinline__ int wave_excl_scan_i(int x) {
  int y = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int z = __shfl_up(y, d, kWave);
    if (lane_id() >= d) y += z;
  }
  return y - x;
}

template <int NS, bool VJP, bool GRAM>
__device__ __forceinline__ void gram_tile(const float* __restrict__ rec, const int64_t* __restrict__ tile_start,
                                          const int32_t* __restrict__ ids, const uint8_t* __restrict__ pix,
                                          const float* __restrict__ wts, const float* __restrict__ wc,
                                          const float* __restrict__ trans,
                                          const int32_t* __restrict__ lastv, int n, int T, int TX, int k,
                                          const lmrs_render_opts& o, float* __restrict__ gram,
                                          const float* __restrict__ u_in, float* __restrict__ grad2d,
                                          bool fixed, const BlendOut& bo, int64_t tile_lin, float* tr,
                                          int* tr_id) {
  const int lane = lane_id();
  const TileCtx c = tile_ctx(tile_start, T, TX, tile_lin);
  PixelRegs<NS> pr;
  const int lmax = load_pixel_regs<NS>(pix, wts, wc, lastv, k, c, pr);
  float sT[NS], sS0[NS], sS1[NS], sS2[NS], sU0[NS], sU1[NS], sU2[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int j = s * kWave + lane;
    sT[s] = j < k ? trans[c.tile_lin * k + j] : 0.f;
    sS0[s] = sT[s] * o.bg[0];
    sS1[s] = sT[s] * o.bg[1];
    sS2[s] = sT[s] * o.bg[2];
    sU0[s] = sU1[s] = sU2[s] = 0.f;
    if (VJP && j < k) {
      const int64_t i = c.tile_lin * k + j;
      sU0[s] = u_in[3 * i];
      sU1[s] = u_in[3 * i + 1];
      sU2[s] = u_in[3 * i + 2];
    }
  }
  if (lmax < 0) return;
  const int64_t blend_base = bo.on ? bo.start[c.tile_lin] : 0;
  // the render counted the tile's pairs with the same opacity tests; writes
  // stay inside the tile's range regardless
  const int64_t blend_end = bo.on ? bo.start[c.tile_lin + 1] : 0;
  int64_t blend_cursor = 0;  // pairs of the tile written so far
  int run_cursor = 0;        // runs of the tile written so far
  for (int c0 = (lmax / kWave) * kWave; c0 >= 0; c0 -= kWave) {
    const int e = c0 + (kWave - 1 - lane);
    const bool valid = e < c.len;
    RecF r{};
    int id = 0;
    if (valid) {
      id = ids[c.start + e];
      r = load_rec(rec, (size_t)c.v * n + id);
    }
    int64_t my_pair = 0, chunk_block = 0;
    if (bo.on) {
      // the pixels that blend this lane's entry, counted first
      int cnt = 0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int ccount = min(kWave, k - s * kWave);
        for (int l = 0; l < ccount; ++l) {
          const int lj = readlane(pr.last[s], l);
          if (c0 > lj) continue;
          const Alpha al =
              pair_alpha(r.u, r.v, r.f11, r.f12, r.f22, r.o, readlane(pr.xc[s], l), readlane(pr.yc[s], l), o);
          cnt += (valid && e <= lj && al.inc) ? 1 : 0;
        }
      }
      const int pieces = (cnt + kBlendRun - 1) / kBlendRun;
      const int off = wave_excl_scan_i(cnt), roff = wave_excl_scan_i(pieces);
      const int tot = readlane(off + cnt, kWave - 1), rtot = readlane(roff + pieces, kWave - 1);
      for (int j = 0; j < pieces; ++j) {
        const int64_t at = blend_base + run_cursor + roff + j;
        if (at < blend_end) bo.run[at] = (int32_t)(blend_cursor + off + j * kBlendRun);
      }
      my_pair = blend_base + blend_cursor + off;
      chunk_block = blend_base + blend_cursor;
      blend_cursor += tot;
      run_cursor += rtot;
    }
    int64_t pix_cursor = 0;  // pixel-major copy: pairs of the chunk written so far
    float G[GRAM ? kGram : 1], g[9];
    for (int q = 0; q < (GRAM ? kGram : 1); ++q) G[q] = 0.f;
    for (int q = 0; q < 9; ++q) g[q] = 0.f;
    const float rgb[3] = {r.r, r.g, r.b};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int cnt = min(kWave, k - s * kWave);
      for (int l = 0; l < cnt; ++l) {
        const int lj = readlane(pr.last[s], l);
        if (c0 > lj) continue;
        const Alpha al =
            pair_alpha(r.u, r.v, r.f11, r.f12, r.f22, r.o, readlane(pr.xc[s], l), readlane(pr.yc[s], l), o);
        const bool inc = valid && e <= lj && al.inc;
        int64_t my_pix_pair = 0;
        if (bo.on) {  // pixel-major copy: this pixel's pairs in lane order
          const uint64_t incm = __ballot(inc);
          my_pix_pair = chunk_block + pix_cursor + __popcll(incm & ((1ull << lane) - 1ull));
          pix_cursor += __popcll(incm);
        }
        const float a = inc ? al.a : 0.f;
        const float rP = __builtin_amdgcn_rcpf(scan_mul(inc ? 1.f - a : 1.f));
        const float Tafter = readlane(sT[s], l);
        const float Tn = Tafter * rP;
        const float S[3] = {readlane(sS0[s], l), readlane(sS1[s], l), readlane(sS2[s], l)};
        float behind[3], tot[3];
        for (int ch = 0; ch < 3; ++ch) {
          const float term = inc ? rgb[ch] * a * Tn : 0.f;
          const float Sinc = scan_add(term);
          behind[ch] = S[ch] + (Sinc - term);
          tot[ch] = readlane(Sinc, kWave - 1);
        }
        if (inc) {
          const float wj = readlane(pr.w[s], l);
          const float aT = a * Tn;
          if (GRAM) G[GRAM ? 30 : 0] += wj * aT * aT;
          float u[3] = {0.f, 0.f, 0.f};
          if (VJP) {
            u[0] = readlane(sU0[s], l);
            u[1] = readlane(sU1[s], l);
            u[2] = readlane(sU2[s], l);
            g[6] += u[0] * aT;
            g[7] += u[1] * aT;
            g[8] += u[2] * aT;
          }
          float ga[3] = {0.f, 0.f, 0.f};
          if (!al.capped) {
            float sga2 = 0.f;
            const float iom = __builtin_amdgcn_rcpf(1.f - a);
            for (int ch = 0; ch < 3; ++ch) {
              ga[ch] = Tn * rgb[ch] - behind[ch] * iom;
              sga2 += ga[ch] * ga[ch];
            }
            const float h[5] = {-(al.q1 * r.f11), -(al.q1 * r.f12 + al.q2 * r.f22), -(al.q1 * al.dx),
                                -(al.q1 * al.dy), -(al.q2 * al.dy)};
            if (GRAM) {
              const float fg = wj * a * a * sga2;
              for (int p = 0; p < 5; ++p) {
                for (int q = p; q < 5; ++q) G[GRAM ? sym5(p, q) : 0] += fg * h[p] * h[q];
                for (int ch = 0; ch < 3; ++ch) G[GRAM ? 15 + 3 * p + ch : 0] += wj * ga[ch] * a * h[p] * aT;
              }
              G[GRAM ? 31 : 0] += wj * sga2 * al.es * al.es;
            }
            if (VJP) {
              const float gu = u[0] * ga[0] + u[1] * ga[1] + u[2] * ga[2];
              g[5] += gu * al.es;
              for (int p = 0; p < 5; ++p) g[p] += gu * a * h[p];
            }
          }
          if (bo.on && my_pair < blend_end) {
            const float4 kv = make_float4(ga[0], ga[1], ga[2], aT);
            const uint32_t mv = ((uint32_t)id << 8) | (uint32_t)(s * kWave + l);
            bo.k[my_pair] = kv;
            bo.m[my_pair] = mv;
            if (my_pix_pair < blend_end) {
              bo.k[bo.pix_major + my_pix_pair] = kv;
              bo.m[bo.pix_major + my_pix_pair] = mv;
            }
          }
          ++my_pair;
        }
        sT[s] = writelane(sT[s], Tafter * readlane(rP, kWave - 1), l);
        sS0[s] = writelane(sS0[s], S[0] + tot[0], l);
        sS1[s] = writelane(sS1[s], S[1] + tot[1], l);
        sS2[s] = writelane(sS2[s], S[2] + tot[2], l);
      }
    }
    tr_id[lane] = valid ? id : -1;
    if (GRAM) {
      // Gram flush, transposed through LDS: the atomic instruction t covers
      // entries 2t and 2t + 1 with lanes holding their 32 components, so that
      // each instruction updates two Gaussians' 128-byte Gram rows instead of
      // one word in each of 64 rows.
#pragma unroll
      for (int q = 0; q < (GRAM ? kGram : 1); ++q) tr[q * (kWave + 1) + lane] = G[q];
      const int q = lane & (kGram - 1), half = lane >> 5;
      for (int t = 0; t < kWave / 2; ++t) {
        const int e2 = 2 * t + half;
        const int ide = tr_id[e2];
        const float val = tr[q * (kWave + 1) + e2];
        if (ide >= 0 && val != 0.f) {
          const size_t row = (size_t)c.v * n + ide;
          if (fixed)
            fix_add<kFixGramLo, kFixGramPoison>(reinterpret_cast<unsigned long long*>(gram) + row * kFixGramRow, q,
                                                val);
          else atomicAdd(&gram[row * kGram + q], val);
        }
      }
    }
    if (VJP) {  // J^T u, transposed the same way: 4 gradient rows per instruction
#pragma unroll
      for (int q = 0; q < 9; ++q) tr[q * (kWave + 1) + lane] = g[q];
      const int q = lane & (kGradRow - 1);
      for (int t = 0; t < kWave / 4; ++t) {
        const int e2 = 4 * t + (lane >> 4);
        const int ide = tr_id[e2];
        const float val = q < 9 ? tr[q * (kWave + 1) + e2] : 0.f;
        if (ide >= 0 && val != 0.f) grad_add(grad2d, fixed, (size_t)c.v * n + ide, q, val);
      }
    }
  }
  if (bo.on && lane == 0) bo.runs[c.tile_lin] = run_cursor;
}

template <int NS, bool VJP, bool GRAM>
__global__ __launch_bounds__(kWave) void gram_kernel(const float* __restrict__ rec,
                                                     const int64_t* __restrict__ tile_start,
                                                     const int32_t* __restrict__ ids,
                                                     const uint8_t* __restrict__ pix,
                                                     const float* __restrict__ wts,
                                                     const float* __restrict__ wc,
                                                     const float* __restrict__ trans,
                                                     const int32_t* __restrict__ lastv, int n, int T,
                                                     int TX, int k, lmrs_render_opts o,
                                                     float* __restrict__ gram, const float* __restrict__ u_in,
                                                     float* __restrict__ grad2d, bool fixed,
                                                     int32_t* __restrict__ sched, int tiles, BlendOut bo,
                                                     int64_t blend_capacity) {
  __shared__ float tr[kGram * (kWave + 1)];  // flush transposes (padded rows: no bank conflicts)
  __shared__ int tr_id[kWave];
  const SchedRef sr = sched_ref(sched, tiles);
  const int count = sched_count(sr, true);
  // the table is written only when the render's pair count fits
  bo.on = bo.on && bo.start[tiles] <= blend_capacity;
  for (;;) {
    const int tile = sched_next(sr, count);
    if (tile == -1) break;
    if (tile >= 0)
      gram_tile<NS, VJP, GRAM>(rec, tile_start, ids, pix, wts, wc, trans, lastv, n, T, TX, k, o, gram, u_in,
                               grad2d, fixed, bo, tile, tr, tr_id);
  }
  sched_finish(sr);
}

// After the walk that fills the blend table: built iff the pairs fitted.
__global__ void blend_built_kernel(int64_t* __restrict__ start, int64_t m, int64_t capacity) {
  if (threadIdx.x == 0 && blockIdx.x == 0) start[m + 1] = start[m] <= capacity ? 1 : 0;
}

// ------------------------------------------------- GN product from the table
// J^T W J p (eq. 14) over the blend table instead of the tile lists. Per
// tile (one workgroup of kBlendGnThreads, one workgroup per busy tile in the
// schedule's order, longest first), lanes take consecutive pairs of the
// tile's table (the pixel-grouped copy, then the Gaussian-grouped one), so
// every load of the table is coalesced:
//  1. J p, over the pixel-grouped copy of the table: each pair's
//     d C = a T d rgb + K d a (d a from its Gaussian's screen record and
//     tangent record, gathered; the pixel centre from LDS), summed over the
//     lanes holding the same pixel by a segmented DPP scan; one LDS atomic
//     per pixel segment (per-pair LDS float atomics took 0.19 ms for this
//     phase on the 100k workload against 0.07 with plain stores);
//  2. u = w J p in place;
//  3. J^T u: each pair's record gradient, (u . K) d a / d rec and a T u on
//     the colour, then a segmented sum over the lanes holding the same
//     Gaussian (the table keeps a Gaussian's pairs together): DPP shifts
//     inside rows of 16 lanes and row broadcasts across them, each step
//     masked by the distance to the segment head. The last lane of each
//     segment hands its sums to a transposed flush through LDS (one atomic
//     instruction per 4 Gaussians' 64-byte rows).
// The opacity, exponent and their record derivatives are recomputed from the
// screen record and the pixel centre (pair_alpha, the render's own
// arithmetic), so a pair costs 20 bytes of table.
constexpr int kBlendGnThreads = 512;
constexpr int kBlendGnWaves = kBlendGnThreads / kWave;

// Inclusive sums over each segment of consecutive lanes (dist = lane minus
// the segment's first lane): per step, x += x[source] * keep, keep = 1 when
// the source lane lies in the same segment, as one v_fmac_f32_dpp (DPP on
// the first operand; a lane without a source in its row, or outside the row
// mask, keeps its value). Steps: row shifts by 1, 2, 4, 8, then the row-15
// and row-31 broadcasts. The components of a step are independent, which
// covers the two wait states a DPP read needs after a VALU write of the same
// register; the s_nop at either end covers the code around.
__device__ __forceinline__ void seg_scan3(float (&g)[3], int dist) {
  const int lane = lane_id();
  const float k1 = dist >= 1 ? 1.f : 0.f, k2 = dist >= 2 ? 1.f : 0.f, k4 = dist >= 4 ? 1.f : 0.f,
              k8 = dist >= 8 ? 1.f : 0.f;
  const float k15 = dist > (lane & 15) ? 1.f : 0.f, k31 = dist > (lane & 31) ? 1.f : 0.f;
  asm volatile("s_nop 1\n\t"
               "v_fmac_f32_dpp %0, %0, %3 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %3 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %3 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2])
               : "v"(k1));
  asm volatile("v_fmac_f32_dpp %0, %0, %3 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %3 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %3 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2])
               : "v"(k2));
  asm volatile("v_fmac_f32_dpp %0, %0, %3 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %3 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %3 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2])
               : "v"(k4));
  asm volatile("v_fmac_f32_dpp %0, %0, %3 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %3 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %3 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2])
               : "v"(k8));
  asm volatile("v_fmac_f32_dpp %0, %0, %3 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %3 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %3 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2])
               : "v"(k15));
  asm volatile("v_fmac_f32_dpp %0, %0, %3 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %3 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %3 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "s_nop 1"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2])
               : "v"(k31));
}

__device__ __forceinline__ void seg_scan9(float (&g)[9], int dist) {
  const int lane = lane_id();
  const float k1 = dist >= 1 ? 1.f : 0.f, k2 = dist >= 2 ? 1.f : 0.f, k4 = dist >= 4 ? 1.f : 0.f,
              k8 = dist >= 8 ? 1.f : 0.f;
  const float k15 = dist > (lane & 15) ? 1.f : 0.f, k31 = dist > (lane & 31) ? 1.f : 0.f;
  asm volatile("s_nop 1\n\t"
               "v_fmac_f32_dpp %0, %0, %9 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %9 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %9 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %3, %3, %9 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %4, %4, %9 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %5, %5, %9 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %6, %6, %9 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %7, %7, %9 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %8, %8, %9 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]), "+v"(g[3]), "+v"(g[4]), "+v"(g[5]), "+v"(g[6]), "+v"(g[7]), "+v"(g[8])
               : "v"(k1));
  asm volatile("v_fmac_f32_dpp %0, %0, %9 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %9 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %9 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %3, %3, %9 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %4, %4, %9 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %5, %5, %9 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %6, %6, %9 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %7, %7, %9 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %8, %8, %9 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]), "+v"(g[3]), "+v"(g[4]), "+v"(g[5]), "+v"(g[6]), "+v"(g[7]), "+v"(g[8])
               : "v"(k2));
  asm volatile("v_fmac_f32_dpp %0, %0, %9 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %9 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %9 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %3, %3, %9 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %4, %4, %9 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %5, %5, %9 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %6, %6, %9 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %7, %7, %9 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %8, %8, %9 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]), "+v"(g[3]), "+v"(g[4]), "+v"(g[5]), "+v"(g[6]), "+v"(g[7]), "+v"(g[8])
               : "v"(k4));
  asm volatile("v_fmac_f32_dpp %0, %0, %9 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %9 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %9 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %3, %3, %9 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %4, %4, %9 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %5, %5, %9 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %6, %6, %9 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %7, %7, %9 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %8, %8, %9 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]), "+v"(g[3]), "+v"(g[4]), "+v"(g[5]), "+v"(g[6]), "+v"(g[7]), "+v"(g[8])
               : "v"(k8));
  asm volatile("v_fmac_f32_dpp %0, %0, %9 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %9 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %9 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %3, %3, %9 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %4, %4, %9 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %5, %5, %9 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %6, %6, %9 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %7, %7, %9 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %8, %8, %9 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]), "+v"(g[3]), "+v"(g[4]), "+v"(g[5]), "+v"(g[6]), "+v"(g[7]), "+v"(g[8])
               : "v"(k15));
  asm volatile("v_fmac_f32_dpp %0, %0, %9 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %1, %1, %9 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %2, %2, %9 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %3, %3, %9 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %4, %4, %9 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %5, %5, %9 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %6, %6, %9 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %7, %7, %9 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "v_fmac_f32_dpp %8, %8, %9 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
               "s_nop 1"
               : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]), "+v"(g[3]), "+v"(g[4]), "+v"(g[5]), "+v"(g[6]), "+v"(g[7]), "+v"(g[8])
               : "v"(k31));
}

template <bool DET>
__global__ __launch_bounds__(kBlendGnThreads) void blend_gn_kernel(
    const float* __restrict__ rec, const float* __restrict__ tan, const float4* __restrict__ bk,
    const uint32_t* __restrict__ bm, const int64_t* __restrict__ bstart, const uint8_t* __restrict__ pix,
    const float* __restrict__ wts, const float* __restrict__ wc, int n, int T, int TX, int k, lmrs_render_opts o,
    float* __restrict__ grad2d,
    int32_t* __restrict__ sched, int tiles, int64_t pix_major) {
  __shared__ float4 s_u[kMaxK];    // J p, then u, of each sample slot (4th word unused)
  __shared__ float2 s_xy[kMaxK];  // pixel centre of each sample slot
  __shared__ float s_tr[kBlendGnWaves][9 * (kWave + 1)];
  __shared__ int s_id[kBlendGnWaves][kWave];
  // deterministic mode: J p of each sample slot in fixed point (3 hi words,
  // 3 lo words, poison word, padding)
  __shared__ unsigned long long s_fix[DET ? kMaxK * 8 : 1];
  if (bstart[tiles + 1] != 1) return;  // no table for this render: the list walk runs instead
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
  const uint64_t below = (1ull << lane) - 1ull;
  // one workgroup per busy tile, the longest first (the dispatcher hands out
  // workgroups in index order as CUs free up: no shared ticket counter)
  const SchedRef sr = sched_ref(sched, tiles);
  if ((int)blockIdx.x >= sched_count(sr, true)) return;
  {
    const int tile = sr.order[blockIdx.x];
    if ((unsigned)tile >= (unsigned)tiles) return;
    const int v = tile / T, t = tile % T;
    const float ox = (float)((t % TX) * kTile), oy = (float)((t / TX) * kTile);
    const int64_t ps = bstart[tile], pe = bstart[tile + 1];
    const size_t vb = (size_t)v * n;
    for (int j = tid; j < k; j += kBlendGnThreads) {
      const int p = pix ? (int)pix[(int64_t)tile * k + j] : j;
      s_xy[j] = make_float2(ox + (float)(p & 15) + 0.5f, oy + (float)(p >> 4) + 0.5f);
      s_u[j] = float4{};
      if constexpr (DET) {
#pragma unroll
        for (int w = 0; w < 8; ++w) s_fix[8 * j + w] = 0ull;
      }
    }
    __syncthreads();
    // 1. J p at the tile's sampled pixels, over the pixel-grouped copy of
    // the table (64 consecutive pairs per wave step; the table entry two steps
    // ahead and the records one step ahead in flight): each pair's
    // d C = a T d rgb + K d a, summed over the lanes of the same pixel, the
    // last lane of each pixel adding the sums into its LDS slot
    {
      const float4* __restrict__ pk = bk + pix_major;
      const uint32_t* __restrict__ pm = bm + pix_major;
      const RecF zero{};
      auto valid_g = [&](uint32_t m) { return m != 0xffffffffu && (int)(m >> 8) < n; };
      int64_t i = ps + (int64_t)wv * kWave + lane;
      uint32_t m1 = 0xffffffffu, m2 = 0xffffffffu;
      float4 k1{}, k2{};
      RecF r1 = zero, d1 = zero;
      if (i < pe) { m1 = pm[i]; k1 = pk[i]; }
      if (i + kBlendGnThreads < pe) { m2 = pm[i + kBlendGnThreads]; k2 = pk[i + kBlendGnThreads]; }
      if (valid_g(m1)) { r1 = load_geo(rec, vb + (m1 >> 8)); d1 = load_rec(tan, vb + (m1 >> 8)); }
      for (int64_t base = ps + (int64_t)wv * kWave; base < pe; base += kBlendGnThreads, i += kBlendGnThreads) {
        const uint32_t m0 = m1;
        const float4 kk = k1;
        const RecF r = r1, dr = d1;
        m1 = m2; k1 = k2;
        m2 = 0xffffffffu;
        if (i + 2 * kBlendGnThreads < pe) { m2 = pm[i + 2 * kBlendGnThreads]; k2 = pk[i + 2 * kBlendGnThreads]; }
        if (valid_g(m1)) { r1 = load_geo(rec, vb + (m1 >> 8)); d1 = load_rec(tan, vb + (m1 >> 8)); }
        int j = (int)(m0 & 255u);
        if (!valid_g(m0) || j >= k) j = -1;  // not a pair of this frame
        float dc[3] = {0.f, 0.f, 0.f};
        if (j >= 0) {
          const float2 xy = s_xy[j];
          const Alpha al = pair_alpha(r.u, r.v, r.f11, r.f12, r.f22, r.o, xy.x, xy.y, o);
          const float ds = -al.q1 * (dr.f11 * al.dx + dr.f12 * al.dy + r.f11 * dr.u + r.f12 * dr.v) -
                           al.q2 * (dr.f22 * al.dy + r.f22 * dr.v);
          const float da = al.es * (dr.o + r.o * ds);  // multiplies K, which is 0 when alpha is capped
          dc[0] = dr.r * kk.w + kk.x * da;
          dc[1] = dr.g * kk.w + kk.y * da;
          dc[2] = dr.b * kk.w + kk.z * da;
        }
        const int prev = __builtin_amdgcn_update_dpp(-2, j, dpp::kWaveShr1, 0xf, 0xf, false);
        const uint64_t heads = __ballot(lane == 0 || j != prev);
        const int dist = lane - (63 - __clzll((long long)(heads & (below | (1ull << lane)))));
        seg_scan3(dc, dist);
        const bool is_end = lane == kWave - 1 || ((heads >> (lane + 1)) & 1ull);
        if (is_end && j >= 0) {
          if constexpr (DET) {
            fix_add<3, 6>(s_fix + 8 * j, 0, dc[0]);
            fix_add<3, 6>(s_fix + 8 * j, 1, dc[1]);
            fix_add<3, 6>(s_fix + 8 * j, 2, dc[2]);
          } else {
            atomicAdd(&s_u[j].x, dc[0]);
            atomicAdd(&s_u[j].y, dc[1]);
            atomicAdd(&s_u[j].z, dc[2]);
          }
        }
      }
    }
    __syncthreads();
    // 2. u = w J p (per channel with operator weights wc)
    for (int j = tid; j < k; j += kBlendGnThreads) {
      const int64_t i = (int64_t)tile * k + j;
      float4 x = s_u[j];
      if constexpr (DET) {
        const unsigned long long* fx = s_fix + 8 * j;
        x = fx[6] ? make_float4(NAN, NAN, NAN, 0.f)
                  : make_float4(fix_value(fx[0], fx[3]), fix_value(fx[1], fx[4]), fix_value(fx[2], fx[5]), 0.f);
      }
      if (wc) {
        s_u[j] = make_float4(x.x * wc[3 * i], x.y * wc[3 * i + 1], x.z * wc[3 * i + 2], 0.f);
      } else {
        const float w = wts ? wts[i] : 1.f;
        s_u[j] = make_float4(x.x * w, x.y * w, x.z * w, 0.f);
      }
    }
    __syncthreads();
    // 3. J^T u over 64 consecutive pairs per wave step, pipelined like 1.
    const RecF zero_r{};
    int64_t base = ps + (int64_t)wv * kWave;
    uint32_t n1 = 0xffffffffu, n2 = 0xffffffffu;
    float4 c1{}, c2{};
    RecF q1r = zero_r;
    auto ok_g = [&](uint32_t m) { return m != 0xffffffffu && (int)(m >> 8) < n; };
    if (base + lane < pe) { n1 = bm[base + lane]; c1 = bk[base + lane]; }
    if (base + kBlendGnThreads + lane < pe) { n2 = bm[base + kBlendGnThreads + lane]; c2 = bk[base + kBlendGnThreads + lane]; }
    if (ok_g(n1)) q1r = load_geo(rec, vb + (n1 >> 8));
    for (; base < pe; base += kBlendGnThreads) {
      const uint32_t m = n1;
      const float4 kk = c1;
      const RecF r = q1r;
      n1 = n2; c1 = c2;
      n2 = 0xffffffffu;
      if (base + 2 * kBlendGnThreads + lane < pe) {
        n2 = bm[base + 2 * kBlendGnThreads + lane];
        c2 = bk[base + 2 * kBlendGnThreads + lane];
      }
      if (ok_g(n1)) q1r = load_geo(rec, vb + (n1 >> 8));
      float g[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      int gid = -1;
      {
        const int j = (int)(m & 255u);
        if (ok_g(m) && j < k) {
          gid = (int)(m >> 8);
          const float2 xy = s_xy[j];
          const Alpha al = pair_alpha(r.u, r.v, r.f11, r.f12, r.f22, r.o, xy.x, xy.y, o);
          const float4 uu = s_u[j];
          const float u0 = uu.x, u1 = uu.y, u2 = uu.z;
          g[6] = u0 * kk.w;
          g[7] = u1 * kk.w;
          g[8] = u2 * kk.w;
          const float ga = kk.x * u0 + kk.y * u1 + kk.z * u2;
          const float gs = ga * al.a;
          g[5] = ga * al.es;
          g[0] = -(gs * (al.q1 * r.f11));
          g[1] = -(gs * (al.q1 * r.f12 + al.q2 * r.f22));
          g[2] = -(gs * (al.q1 * al.dx));
          g[3] = -(gs * (al.q1 * al.dy));
          g[4] = -(gs * (al.q2 * al.dy));
        }
      }
      // segments: lanes holding the same Gaussian (consecutive in the table)
      const int prev = __builtin_amdgcn_update_dpp(-2, gid, dpp::kWaveShr1, 0xf, 0xf, false);
      const uint64_t heads = __ballot(lane == 0 || gid != prev);
      const int dist = lane - (63 - __clzll((long long)(heads & (below | (1ull << lane)))));
      seg_scan9(g, dist);
      // the last lane of each segment hands its Gaussian's sums to a
      // transposed flush: an atomic instruction covers 7 Gaussians' rows, 9
      // lanes each (4 rows of 16 lanes, 7 of them idle, was 1.7 % slower)
      const uint64_t ends = (heads >> 1) | (1ull << 63);
      const bool is_end = (ends >> lane) & 1ull;
      const int slot = __popcll(ends & below);
      const int nseg = __popcll(ends);
      float* tr = s_tr[wv];
      if (is_end) {
#pragma unroll
        for (int q = 0; q < 9; ++q) tr[q * (kWave + 1) + slot] = g[q];
        s_id[wv][slot] = gid;
      }
      const int sub = lane / 9, q = lane - 9 * sub;  // 7 entries per step, 9 lanes each
      for (int e = 0; 7 * e < nseg; ++e) {
        const int ent = 7 * e + sub;
        if (sub < 7 && ent < nseg) {
          const int ide = s_id[wv][ent];
          const float val = tr[q * (kWave + 1) + ent];
          if (ide >= 0 && val != 0.f) grad_add(grad2d, DET, vb + ide, q, val);
        }
      }
    }
  }
}

// Waves of a persistent splat launch: one per kTilesPerWave tiles of the
// batch, between kMinWavesPerCU and kMaxWavesPerCU per CU. With few busy
// tiles of uneven walks (an object in the middle of the views), few waves per
// SIMD let the ticket order balance the work; with many tiles, more waves
// hide more latency. Measured on the 100k- and 1.5M-Gaussian workloads:
// 8 per CU is best for 20,000 tiles of which a third are busy, 32 per CU for
// 65,728 busy tiles. The busy count is only known on the device, so the tile
// count of the batch stands in for it.
constexpr int kMinWavesPerCU = 8;
constexpr int kMaxWavesPerCU = 32;
constexpr int kTilesPerWave = 10;

unsigned persistent_grid(int64_t tiles) {
  static std::atomic<int> cus[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int c = cus[dev].load(std::memory_order_relaxed);
  if (c <= 0) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cus[dev].store(c, std::memory_order_relaxed);
  }
  const int64_t want = std::min<int64_t>((int64_t)c * kMaxWavesPerCU,
                                         std::max<int64_t>((int64_t)c * kMinWavesPerCU,
                                                           (tiles + kTilesPerWave - 1) / kTilesPerWave));
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, want));
}

// Workgroups of W waves for a persistent derivative launch: one wave per
// kTilesPerWave / W tiles, between kMinWavesPerCU and kMaxWavesPerCU waves
// per CU (see persistent_grid; the LDS of the reduction buffers allows 32
// waves per CU).
unsigned persistent_groups(int64_t tiles, int w) {
  const int64_t waves = (int64_t)persistent_grid(tiles * w);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, waves / w));
}

// Walk counts of the sampled render (measurement): one wave per tile, lanes
// own 64-entry chunks of its list up to the deepest last blended entry. An
// entry at or before a pixel's last blended one is blended by that pixel iff
// it passes the opacity test (the transmittance stop only ends a walk after
// its last blended entry), so the counts need no transmittance.
// counts: [0] sum of L*_t (max over the tile's pixels of last + 1), [1] sum
// of C_t (entries blended by at least one of the tile's pixels), [2] blending
// (pixel, entry) pairs, [3] (pixel, entry) pairs up to each pixel's last.
__global__ __launch_bounds__(kWave) void walk_count_kernel(const float* __restrict__ rec,
                                                            const int64_t* __restrict__ tile_start,
                                                            const int32_t* __restrict__ ids,
                                                            const uint8_t* __restrict__ pix,
                                                            const int32_t* __restrict__ lastv, int n, int T, int TX,
                                                            int k, lmrs_render_opts o,
                                                            unsigned long long* __restrict__ counts) {
  const int lane = lane_id();
  const TileCtx c = tile_ctx(tile_start, T, TX, blockIdx.x);
  int lmax = -1;
  for (int j = lane; j < k; j += kWave) lmax = max(lmax, lastv[c.tile_lin * k + j]);
  lmax = uniform(wave_max_i(lmax));
  unsigned long long contrib = 0, act = 0, walked = 0;
  for (int c0 = 0; c0 <= lmax; c0 += kWave) {
    const int e = c0 + lane;
    const bool valid = e <= lmax && e < c.len;
    RecF r{};
    if (valid) r = load_rec(rec, (size_t)c.v * n + ids[c.start + e]);
    bool any = false;
    for (int j = 0; j < k; ++j) {
      const int lj = lastv[c.tile_lin * k + j];
      if (lj < c0) continue;
      float xc, yc;
      pixel_center(pix, k, c, j, &xc, &yc);
      const Alpha al = pair_alpha(r.u, r.v, r.f11, r.f12, r.f22, r.o, xc, yc, o);
      if (valid && e <= lj) {
        ++walked;
        if (al.inc) {
          ++act;
          any = true;
        }
      }
    }
    contrib += __popcll(__ballot(any));
  }
  // per-lane counts to lane 0 through LDS (exact in 64-bit)
  __shared__ unsigned long long s_act[kWave], s_walk[kWave];
  s_act[lane] = act;
  s_walk[lane] = walked;
  __syncthreads();
  if (lane == 0) {
    unsigned long long ta = 0, tw = 0;
    for (int l = 0; l < kWave; ++l) {
      ta += s_act[l];
      tw += s_walk[l];
    }
    atomicAdd(&counts[0], (unsigned long long)(lmax + 1));
    atomicAdd(&counts[1], contrib);
    atomicAdd(&counts[2], ta);
    atomicAdd(&counts[3], tw);
  }
}

__global__ void zero_u64_kernel(unsigned long long* __restrict__ x, int m) {
  if ((int)threadIdx.x < m) x[threadIdx.x] = 0ull;
}

}  // namespace

void launch_walk_counts(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, int64_t* counts,
                        hipStream_t s) {
  auto* cnt = reinterpret_cast<unsigned long long*>(counts);
  zero_u64_kernel<<<1, kWave, 0, s>>>(cnt, 4);
  const unsigned tiles = (unsigned)((int64_t)d.V * d.T);
  walk_count_kernel<<<tiles, kWave, 0, s>>>(f->rec, f->tile_start, f->ids, f->pix, f->last, d.n, d.T, d.TX, d.k, o,
                                            cnt);
}

template <int W>
void launch_render_w(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, hipStream_t s) {
  const unsigned tiles = (unsigned)((int64_t)d.V * d.T);
  int32_t* walk_len = f->sched + tiles;
  // pixels per wave with per-lane colour accumulators: up to 8 or 16
  const int per_wave = (d.k + W - 1) / W;
  auto go = [&](auto kern) {
    kern<<<tiles, kWave * W, 0, s>>>(f->rec, f->tile_start, f->ids, f->pix, d.n, d.T, d.TX, d.k, o, f->color,
                                     f->trans, f->last, walk_len, f->blend_k ? f->blend_start : nullptr);
  };
  if (d.k > kWave) go(render_kernel<4, W, 1>);
  else if (per_wave <= 8) go(render_kernel<1, W, 8>);
  else if (per_wave <= 16) go(render_kernel<1, W, 16>);
  else go(render_kernel<1, W, 1>);
}

void launch_render(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, hipStream_t s) {
  // 4 waves per tile share its pixels from 24 samples per tile up (as in the derivative walks)
  if (d.k >= 24) launch_render_w<4>(f, d, o, s);
  else launch_render_w<1>(f, d, o, s);
  const unsigned tiles = (unsigned)((int64_t)d.V * d.T);
  sched_kernel<<<1, kSchedThreads, 0, s>>>(f->sched, (int)tiles);
  if (f->blend_k) blend_scan_kernel<<<1, kBlendScanThreads, 0, s>>>(f->blend_start, (int64_t)tiles);
}

void launch_render_scores(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                          const float* targets, float* scores, hipStream_t s) {
  const unsigned tiles = (unsigned)((int64_t)d.V * d.T);
  const ScoreOut so{targets, f->view_ids, d.W, d.H, scores};
  score_kernel<kScoreResidual><<<tiles, kScoreThreads, 0, s>>>(f->rec, f->tile_start, f->ids, d.n, d.T, d.TX, o,
                                                                so);
}

void launch_render_image(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, float* image,
                         hipStream_t s) {
  const unsigned tiles = (unsigned)((int64_t)d.V * d.T);
  const ScoreOut so{nullptr, f->view_ids, d.W, d.H, image};
  score_kernel<kScoreImage><<<tiles, kScoreThreads, 0, s>>>(f->rec, f->tile_start, f->ids, d.n, d.T, d.TX, o, so);
}

void launch_render_counts(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, float* counts,
                          hipStream_t s) {
  const unsigned tiles = (unsigned)((int64_t)d.V * d.T);
  const ScoreOut so{nullptr, f->view_ids, d.W, d.H, counts};
  score_kernel<kScoreCount><<<tiles, kScoreThreads, 0, s>>>(f->rec, f->tile_start, f->ids, d.n, d.T, d.TX, o, so);
}

template <int MODE, int W>
void launch_deriv_mode(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, const float* tan,
                       const float* u, float* jp, float* grad2d, hipStream_t s, const int64_t* built) {
  static_assert(kWave % W == 0, "pixel slots are dealt to the waves by lane");
  const int tiles = d.V * d.T;
  const unsigned grid = persistent_groups(tiles, W);
  const unsigned block = kWave * W;
  const bool small = d.k <= kWave;
  // pixels per wave when they are dealt by depth (several waves, one slot,
  // at most 8 per wave), else 1 (dealt by slot)
  const int mp = W > 1 && small && d.k <= 8 * W ? (d.k + W - 1) / W : 1;
  auto go = [&](auto kern) {
    kern<<<grid, block, 0, s>>>(f->rec, tan, f->tile_start, f->ids, f->pix, f->w, MODE == 3 ? f->wc : nullptr,
                                f->trans, f->last, d.n, d.T, d.TX, d.k, o, u, jp, grad2d, d.det, f->sched, tiles,
                                built);
  };
  if (!small) {
    go(deriv_kernel<MODE, 4, W, 1>);
  } else if (mp <= 1) {
    go(deriv_kernel<MODE, 1, W, 1>);
  } else if constexpr (W > 1) {
    if (mp <= 6) go(deriv_kernel<MODE, 1, W, 6>);
    else if (mp == 7) go(deriv_kernel<MODE, 1, W, 7>);
    else go(deriv_kernel<MODE, 1, W, 8>);
  }
}

template <int W>
void launch_deriv_w(int mode, const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                    const float* tan, const float* u, float* jp, float* grad2d, hipStream_t s,
                    const int64_t* built) {
  if (mode == 1) launch_deriv_mode<1, W>(f, d, o, tan, u, jp, grad2d, s, nullptr);
  else if (mode == 2) launch_deriv_mode<2, W>(f, d, o, tan, u, jp, grad2d, s, nullptr);
  else launch_deriv_mode<3, W>(f, d, o, tan, u, jp, grad2d, s, built);
}

void launch_deriv(int mode, const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                  const float* tan, const float* u, float* jp, float* grad2d, hipStream_t s) {
  // the fused walk (mode 3) steps aside when the blend table is built
  const int64_t* built = mode == 3 && f->blend_k ? f->blend_start + (int64_t)d.V * d.T + 1 : nullptr;
  // Measured: 4 waves per tile at 26 samples per tile (100k workload) took the
  // fused splat from 0.59 to 0.535 ms with pixels dealt by slot. At 13 samples
  // (1.5M workload) 2 or 4 slot-dealt waves were slower than one (9.24 and
  // 9.47 against 9.13 ms); 2 waves with pixels dealt by depth are faster
  // (4.07 -> 3.90 ms).
  if (d.k >= 24) launch_deriv_w<4>(mode, f, d, o, tan, u, jp, grad2d, s, built);
  else if (d.k >= 12) launch_deriv_w<2>(mode, f, d, o, tan, u, jp, grad2d, s, built);
  else launch_deriv_w<1>(mode, f, d, o, tan, u, jp, grad2d, s, built);
}

void launch_gram(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, float* gram,
                 const float* u, float* grad2d, hipStream_t s, bool gram_sums) {
  const int tiles = d.V * d.T;
  const unsigned grid = persistent_grid(tiles);
  BlendOut bo{reinterpret_cast<float4*>(f->blend_k), f->blend_m, f->blend_run, f->blend_runs, f->blend_start,
              f->blend_k != nullptr, f->blend_capacity};
#define LMRS_GRAM_ARGS                                                                                      \
  f->rec, f->tile_start, f->ids, f->pix, f->w, f->wc, f->trans, f->last, d.n, d.T, d.TX, d.k, o, gram, u, grad2d, \
      d.det, f->sched, tiles, bo, f->blend_capacity
  const bool wide = d.k > kWave;
  if (!gram_sums) {
    if (!wide) gram_kernel<1, false, false><<<grid, kWave, 0, s>>>(LMRS_GRAM_ARGS);
    else gram_kernel<4, false, false><<<grid, kWave, 0, s>>>(LMRS_GRAM_ARGS);
  } else if (u) {
    if (!wide) gram_kernel<1, true, true><<<grid, kWave, 0, s>>>(LMRS_GRAM_ARGS);
    else gram_kernel<4, true, true><<<grid, kWave, 0, s>>>(LMRS_GRAM_ARGS);
  } else {
    if (!wide) gram_kernel<1, false, true><<<grid, kWave, 0, s>>>(LMRS_GRAM_ARGS);
    else gram_kernel<4, false, true><<<grid, kWave, 0, s>>>(LMRS_GRAM_ARGS);
  }
#undef LMRS_GRAM_ARGS
  if (f->blend_k) blend_built_kernel<<<1, 64, 0, s>>>(f->blend_start, (int64_t)tiles, f->blend_capacity);
}

void launch_blend_gn(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, const float* tan,
                     float* grad2d, hipStream_t s) {
  if (!f->blend_k) return;
  const int tiles = d.V * d.T;
  auto go = [&](auto kern) {
    kern<<<(unsigned)tiles, kBlendGnThreads, 0, s>>>(f->rec, tan, reinterpret_cast<const float4*>(f->blend_k),
                                                     f->blend_m, f->blend_start, f->pix, f->w, f->wc, d.n, d.T, d.TX,
                                                     d.k, o, grad2d, f->sched, tiles, f->blend_capacity);
  };
  if (d.det) go(blend_gn_kernel<true>);
  else go(blend_gn_kernel<false>);
}

}  // namespace lmrs
