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
// 4. emit: each (view, Gaussian) writes the 64-bit key (depth bits << 32 | id)
//    into its tiles' segments at (tile start + chunk offset + LDS cursor).
//    Depths are > znear > 0, so their IEEE bits order like the values; the id
//    breaks ties.
// 5. sort: one workgroup per tile sorts its segment. Segments of up to 4096
//    keys are sorted in LDS by a bitonic network; longer ones sort 4096-key
//    runs in LDS and then merge runs pairwise by merge path (keys are unique
//    within a tile). The merged output is cut into windows of 2048 keys; the
//    split of every window boundary between the two runs is found first, one
//    binary search per thread in parallel; then each window's two input
//    slices are loaded into LDS with coalesced reads, each thread locates its
//    8 outputs on the merge path inside LDS and merges them, and the window
//    is written back coalesced. Tiles near the image centre of large scenes
//    hold hundreds of thousands of keys, so this merge (not the LDS sort)
//    sets the time of the whole launch.
#include "common.hpp"
#include "launch.hpp"

namespace lmrs {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortChunk = 4096;
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
                                                            const float* __restrict__ rec, int n, int TX, int T,
                                                            int n_chunks, const int32_t* __restrict__ chunk_hist,
                                                            const int64_t* __restrict__ tile_start,
                                                            uint64_t* __restrict__ keys) {
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
    const uint32_t dbits = __float_as_uint(rec[vg * LMRS_REC + 9]);
    const uint64_t key = ((uint64_t)dbits << 32) | (uint32_t)g;
    for (int ty = rc.y; ty < rc.w; ++ty)
      for (int tx = rc.x; tx < rc.z; ++tx) {
        const int t = ty * TX + tx;
        const int slot = atomicAdd(&s_cur[t], 1);
        keys[ts[t] + slot] = key;
      }
  }
}

// Bitonic sort of s[0..m) in LDS, m a power of two.
__device__ void lds_bitonic(uint64_t* s, int m) {
  for (int size = 2; size <= m; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (m >> 1); i += kSortThreads) {
        const int lo = 2 * stride * (i / stride) + (i % stride);
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t x = s[lo], y = s[hi];
        if ((x > y) == up) {
          s[lo] = y;
          s[hi] = x;
        }
      }
      __syncthreads();
    }
}

// Sort keys[a, a+len) of one chunk through LDS; result to dst (may equal src).
__device__ void sort_chunk(const uint64_t* src, uint64_t* dst, int len, uint64_t* s) {
  int m = 1;
  while (m < len) m <<= 1;
  for (int i = threadIdx.x; i < m; i += kSortThreads) s[i] = i < len ? src[i] : ~0ull;
  __syncthreads();
  lds_bitonic(s, m);
  for (int i = threadIdx.x; i < len; i += kSortThreads) dst[i] = s[i];
  __syncthreads();
}

constexpr int kMergeWindow = 2048;                 // merged keys per LDS window
constexpr int kMergePer = kMergeWindow / kSortThreads;  // outputs per thread per window

// Number of A keys among the first d keys of the merge of sorted A[0, na) and B[0, nb).
__device__ __forceinline__ int64_t merge_split(const uint64_t* A, int64_t na, const uint64_t* B, int64_t nb,
                                               int64_t d) {
  int64_t lo = max<int64_t>(0, d - nb), hi = min(d, na);
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (A[mid] < B[d - 1 - mid]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Merge sorted runs A[0, na) and B[0, nb) into out[0, na + nb) through LDS
// windows. s: 2 * kMergeWindow keys of LDS (window data, then the splits).
__device__ void merge_runs(const uint64_t* A, int64_t na, const uint64_t* B, int64_t nb, uint64_t* out,
                           uint64_t* s) {
  const int64_t total = na + nb;
  const int64_t nw = (total + kMergeWindow - 1) / kMergeWindow;
  int64_t* split = reinterpret_cast<int64_t*>(s + kMergeWindow);
  constexpr int64_t kBatch = kMergeWindow - 1;  // windows whose boundaries fit the split array
  for (int64_t w0 = 0; w0 < nw; w0 += kBatch) {
    const int64_t wn = min(kBatch, nw - w0);
    for (int64_t q = threadIdx.x; q <= wn; q += kSortThreads)
      split[q] = merge_split(A, na, B, nb, min((w0 + q) * kMergeWindow, total));
    __syncthreads();
    for (int64_t q = 0; q < wn; ++q) {
      const int64_t d0 = (w0 + q) * kMergeWindow, d1 = min(d0 + kMergeWindow, total);
      const int64_t a0 = split[q], a1 = split[q + 1];
      const int la = (int)(a1 - a0), lb = (int)((d1 - d0) - la);
      const int64_t b0 = d0 - a0;
      for (int i = threadIdx.x; i < la; i += kSortThreads) s[i] = A[a0 + i];
      for (int i = threadIdx.x; i < lb; i += kSortThreads) s[la + i] = B[b0 + i];
      __syncthreads();
      const int o0 = threadIdx.x * kMergePer, n_out = (int)(d1 - d0);
      if (o0 < n_out) {
        const uint64_t* sa = s;
        const uint64_t* sb = s + la;
        int lo = max(0, o0 - lb), hi = min(o0, la);
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (sa[mid] < sb[o0 - 1 - mid]) lo = mid + 1; else hi = mid;
        }
        int i = lo, j = o0 - lo;
        const int o1 = min(o0 + kMergePer, n_out);
        for (int o = o0; o < o1; ++o) {
          const bool take_a = j >= lb || (i < la && sa[i] < sb[j]);
          out[d0 + o] = take_a ? sa[i++] : sb[j++];
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kSortThreads) void sort_kernel(const int64_t* __restrict__ tile_start,
                                                            uint64_t* __restrict__ keys,
                                                            uint64_t* __restrict__ tmp,
                                                            int32_t* __restrict__ ids) {
  __shared__ uint64_t s[kSortChunk];
  const int64_t a = tile_start[blockIdx.x];
  const int64_t len = tile_start[blockIdx.x + 1] - a;
  if (len == 0) return;
  uint64_t* src = keys + a;
  uint64_t* dst = tmp + a;
  if (len <= kSortChunk) {
    sort_chunk(src, src, (int)len, s);
  } else {
    for (int64_t c = 0; c < len; c += kSortChunk)
      sort_chunk(src + c, src + c, (int)min<int64_t>(kSortChunk, len - c), s);
    for (int64_t run = kSortChunk; run < len; run <<= 1) {
      for (int64_t base = 0; base < len; base += 2 * run) {
        const int64_t na = min(run, len - base);
        const int64_t nb = max<int64_t>(0, min(run, len - base - run));
        merge_runs(src + base, na, src + base + na, nb, dst + base, s);
      }
      uint64_t* t = src;
      src = dst;
      dst = t;
    }
  }
  for (int64_t i = threadIdx.x; i < len; i += kSortThreads) ids[a + i] = (int32_t)(src[i] & 0xffffffffu);
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

void launch_bin_emit_sort(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s) {
  const int nc = bin_chunks(d.n);
  const size_t lds = (size_t)d.T * sizeof(int32_t);
  emit_kernel<<<dim3(nc, d.V), kBinThreads, lds, s>>>(reinterpret_cast<const int4*>(f->rect), f->rec, d.n, d.TX,
                                                      d.T, nc, b.chunk_hist, f->tile_start, b.keys);
  sort_kernel<<<(unsigned)((int64_t)d.V * d.T), kSortThreads, 0, s>>>(f->tile_start, b.keys, b.tmp,
                                                                     f->ids);
}

}  // namespace lmrs
