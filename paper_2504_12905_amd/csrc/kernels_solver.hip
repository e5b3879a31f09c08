// Solver-side kernels: stratified residual sampling (Sec. 4.4), residuals
// (eq. 7), the vector recurrences of the matrix-free PCG loop (Alg. 1) and the
// learning-rate rule with the parameter update (Sec. 4.5).
//
// Reductions are two-stage and deterministic: kRedBlocks partial sums in FP64,
// then one workgroup sums them. PCG scalars stay in device memory, so a PCG
// iteration is a fixed sequence of launches with no host round trip.
#include "common.hpp"
#include "launch.hpp"

namespace lmrs {

namespace {

// One wave per (view, tile), four pixels per lane (pixel p = 64 j + lane in
// register j): pixel p draws its key from counter (p, tile, camera id,
// iteration); the k pixels with the smallest 40-bit (key, p) are taken,
// listed in ascending pixel order, each with weight 256/k. The k-th smallest
// key is found by a bitwise radix select over ballots (each step counts the
// candidates whose next bit is 0), so a tile needs no LDS and no barrier.
constexpr int kSampleWaves = 4;  // tiles per workgroup
__global__ __launch_bounds__(kWave* kSampleWaves) void sample_kernel(const int32_t* __restrict__ view_ids, int T,
                                                                     int k, int64_t tiles, uint32_t seed_lo,
                                                                     uint32_t seed_hi, uint32_t iter,
                                                                     uint8_t* __restrict__ pix,
                                                                     float* __restrict__ w) {
  const int lane = lane_id();
  const int64_t tile_lin = (int64_t)blockIdx.x * kSampleWaves + threadIdx.x / kWave;
  if (tile_lin >= tiles) return;  // the whole wave
  const int v = (int)(tile_lin / T), t = (int)(tile_lin % T);
  const uint32_t cam = (uint32_t)(view_ids ? view_ids[v] : v);
  uint64_t c[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t p = (uint32_t)(j * kWave + lane);
    const uint4 r = philox4x32_10(make_uint4(p, (uint32_t)t, cam, iter), seed_lo, seed_hi);
    c[j] = ((uint64_t)r.x << 8) | (uint64_t)p;
  }
  // radix select, high bit first: `above` marks the decided bits, prefix
  // their values in the k-th smallest key, cand counts the keys that match
  // them and need how many of those are still to be taken. It stops when
  // every candidate is taken (after about 8 of the 40 bits for distinct keys).
  uint64_t prefix = 0, above = 0;
  int need = k, cand = 256;
  for (int b = 39; b >= 0 && cand > need; --b) {
    const uint64_t bit = 1ull << b;
    int zeros = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) zeros += __popcll(__ballot((c[j] & above) == prefix && (c[j] & bit) == 0));
    above |= bit;
    if (zeros >= need) {
      cand = zeros;
    } else {
      need -= zeros;
      cand -= zeros;
      prefix |= bit;
    }
  }
  // selected: the candidates and every key below them, written in
  // ascending pixel order
  const uint64_t below = (1ull << lane) - 1ull;
  int base = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool sel = (c[j] & above) <= prefix;
    const uint64_t m = __ballot(sel);
    if (sel) {
      const int64_t at = tile_lin * k + base + __popcll(m & below);
      pix[at] = (uint8_t)(j * kWave + lane);
      w[at] = 256.f / (float)k;
    }
    base += __popcll(m);
  }
}

// Residual-weighted sampling (Supp. E, q_residual) inside each tile: pixel p
// has probability q(p) = e_p / Z with e_p = exp(s_p - max s), Z = sum e_p and
// s_p the pixel's residual magnitude. One workgroup of 256 lanes per (view,
// tile); lane p computes e_p, one lane forms the running sums Q_p = e_0 + ...
// + e_p in pixel order (so Q is non-decreasing), and lane j < k takes draw j:
// the 24-bit uniform u_j from the first Philox word of counter
// (256 + j, tile, camera id, iteration), then the smallest p with
// Q_p > u_j Z, weight 1 / (k q(p)) = Z / (k e_p). Draws are with
// replacement and listed in draw order.
__global__ __launch_bounds__(256) void sample_residual_kernel(const float* __restrict__ scores,
                                                              const int32_t* __restrict__ view_ids, int T,
                                                              int k, uint32_t seed_lo, uint32_t seed_hi,
                                                              uint32_t iter, uint8_t* __restrict__ pix,
                                                              float* __restrict__ w) {
  __shared__ float s_e[256];
  __shared__ float s_q[256];
  __shared__ float s_m[4];
  const int p = threadIdx.x;
  const int64_t tile_lin = blockIdx.x;
  const int v = (int)(tile_lin / T), t = (int)(tile_lin % T);
  const float sp = scores[tile_lin * 256 + p];
  const float wm = wave_max_f(sp);
  if (lane_id() == 0) s_m[p / kWave] = wm;
  __syncthreads();
  const float m = fmaxf(fmaxf(s_m[0], s_m[1]), fmaxf(s_m[2], s_m[3]));
  const float e = expf(sp - m);
  s_e[p] = e;
  __syncthreads();
  if (p == 0) {
    float acc = 0.f;
    for (int q = 0; q < 256; ++q) {
      acc += s_e[q];
      s_q[q] = acc;
    }
  }
  __syncthreads();
  if (p >= k) return;
  const uint32_t cam = (uint32_t)(view_ids ? view_ids[v] : v);
  const uint4 r = philox4x32_10(make_uint4(256u + (uint32_t)p, (uint32_t)t, cam, iter), seed_lo, seed_hi);
  const float Z = s_q[255];
  const float target = (float)(r.x >> 8) * 0x1p-24f * Z;
  int lo = 0, hi = 255;  // smallest index with s_q > target; index 255 if none
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (s_q[mid] > target) hi = mid; else lo = mid + 1;
  }
  pix[tile_lin * k + p] = (uint8_t)lo;
  w[tile_lin * k + p] = Z / ((float)k * s_e[lo]);
}

// Contribution-weighted sampling (Supp. E, q_Gaussian) inside each tile:
// pixel p has probability q(p) = G_p / Z, Z = sum G, G_p the number of
// Gaussians blended into the pixel; a tile with Z = 0 is sampled uniformly
// (G_p taken as 1). Draw j takes the 24-bit word d_j of counter
// (256 + j, tile, camera id, iteration) (as the residual sampler) and the
// smallest p with Q_p 2^24 > d_j Z, Q_p = G_0 + ... + G_p, all in 64-bit
// integers, so the draw is exact; weight Z / (k G_p).
__global__ __launch_bounds__(256) void sample_gaussian_kernel(const float* __restrict__ counts,
                                                              const int32_t* __restrict__ view_ids, int T,
                                                              int k, uint32_t seed_lo, uint32_t seed_hi,
                                                              uint32_t iter, uint8_t* __restrict__ pix,
                                                              float* __restrict__ w) {
  __shared__ int64_t s_q[256];
  __shared__ int s_g[256];
  const int p = threadIdx.x;
  const int64_t tile_lin = blockIdx.x;
  const int v = (int)(tile_lin / T), t = (int)(tile_lin % T);
  s_g[p] = (int)counts[tile_lin * 256 + p];
  __syncthreads();
  if (p == 0) {
    int64_t acc = 0;
    for (int q = 0; q < 256; ++q) acc += s_g[q];
    const bool empty = acc == 0;
    acc = 0;
    for (int q = 0; q < 256; ++q) {
      if (empty) s_g[q] = 1;
      acc += s_g[q];
      s_q[q] = acc;
    }
  }
  __syncthreads();
  if (p >= k) return;
  const uint32_t cam = (uint32_t)(view_ids ? view_ids[v] : v);
  const uint4 r = philox4x32_10(make_uint4(256u + (uint32_t)p, (uint32_t)t, cam, iter), seed_lo, seed_hi);
  const int64_t Z = s_q[255];
  const int64_t target = (int64_t)(r.x >> 8) * Z;
  int lo = 0, hi = 255;  // smallest index with s_q * 2^24 > target (index 255 always qualifies)
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((s_q[mid] << 24) > target) hi = mid; else lo = mid + 1;
  }
  pix[tile_lin * k + p] = (uint8_t)lo;
  w[tile_lin * k + p] = (float)Z / ((float)k * (float)s_g[lo]);
}

// wr = w * (C - I) at every sampled pixel; partial sums of w |C - I|^2.
__global__ __launch_bounds__(256) void residual_kernel(const float* __restrict__ color,
                                                       const float* __restrict__ targets,
                                                       const uint8_t* __restrict__ pix,
                                                       const float* __restrict__ wts,
                                                       const int32_t* __restrict__ view_ids, int T,
                                                       int TX, int W, int H, int k, int64_t S,
                                                       float* __restrict__ wr, double* __restrict__ partials) {
  __shared__ double s_red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < S; i += (int64_t)gridDim.x * 256) {
    const int64_t tile_lin = i / k;
    const int j = (int)(i % k);
    const int v = (int)(tile_lin / T), t = (int)(tile_lin % T);
    const int p = pix ? (int)pix[i] : j;
    const int x = (t % TX) * kTile + (p & 15), y = (t / TX) * kTile + (p >> 4);
    const int cam = view_ids ? view_ids[v] : v;
    const float* tg = targets + (((int64_t)cam * H + y) * W + x) * 3;
    const float wi = wts ? wts[i] : 1.f;
    for (int c = 0; c < 3; ++c) {
      const float r = color[3 * i + c] - tg[c];
      wr[3 * i + c] = wi * r;
      acc += (double)wi * r * r;
    }
  }
  s_red[threadIdx.x] = acc;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) s_red[threadIdx.x] += s_red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = s_red[0];
}


__global__ __launch_bounds__(256) void dot_partial_kernel(const float* __restrict__ a,
                                                          const float* __restrict__ b, int64_t n,
                                                          double* __restrict__ partials) {
  __shared__ double s_red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    acc += (double)a[i] * (double)b[i];
  const double r = block_sum(acc, s_red);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// out[o] = sum of partials[o * stride + 0 .. count), for `outs` outputs.
__global__ __launch_bounds__(256) void finalize_kernel(const double* __restrict__ partials, int count,
                                                       int outs, int stride, double* __restrict__ out) {
  __shared__ double s_red[256];
  for (int o = 0; o < outs; ++o) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) acc += partials[o * stride + i];
    const double r = block_sum(acc, s_red);
    if (threadIdx.x == 0) out[o] = r;
  }
}

// Report slot writer: report[slot] = (float)value[0].
__global__ void report_kernel(const double* __restrict__ value, float* __restrict__ report, int slot) {
  if (threadIdx.x == 0 && blockIdx.x == 0) report[slot] = (float)value[0];
}

// report[INST] = the step's tile-list entries; when they exceeded the
// caller's capacity (the lists were left empty) the capacity bit joins the
// failure bits.
__global__ void report_count_kernel(const int64_t* __restrict__ count, int64_t capacity,
                                    float* __restrict__ report, const int64_t* __restrict__ pairs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  report[LMRS_REP_INST] = (float)count[0];
  if (pairs) report[LMRS_REP_PAIRS] = (float)pairs[0];
  if (count[0] > capacity) report[LMRS_REP_STATUS] = (float)((int)report[LMRS_REP_STATUS] | LMRS_FAIL_CAPACITY);
}

// PCG scalar slots.
enum : int {
  kRZ = 0,      // r_i^T z_i
  kRZ0 = 1,     // r_0^T z_0
  kPU = 2,      // p_i^T u
  kRZNew = 3,   // r_{i+1}^T z_{i+1}
  kRR = 4,      // r^T r
  kAlpha = 5,
  kBeta = 6,
  kStop = 7,
  kDone = 8,
  kRR0 = 9,
  kFail = 11,   // LMRS_FAIL_* bits (slot 10 holds b^T x for the report)
  kScalars = 16
};

// VEC floats as one unit: float4 (16-byte accesses) or a single float.
template <int VEC>
struct Vec;
template <>
struct Vec<1> {
  using T = float;
  __device__ static float load(const float* a, int64_t i) { return a[i]; }
  __device__ static void store(float* a, int64_t i, float v) { a[i] = v; }
  __device__ static float& at(float& v, int) { return v; }
  __device__ static float at(const float& v, int) { return v; }
};
template <>
struct Vec<4> {
  using T = float4;
  __device__ static float4 load(const float* a, int64_t i) { return reinterpret_cast<const float4*>(a)[i]; }
  __device__ static void store(float* a, int64_t i, float4 v) { reinterpret_cast<float4*>(a)[i] = v; }
  __device__ static float& at(float4& v, int c) { return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w; }
  __device__ static float at(const float4& v, int c) { return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w; }
};

// Sum of partials[0, count) in a fixed order (the same in every block).
__device__ __forceinline__ double reduce_partials(const double* __restrict__ partials, int count,
                                                  double* s_red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) acc += partials[i];
  return block_sum(acc, s_red);
}

// x = 0, r = b, M^-1 = 1 / (diag + lambda d), z = p = M^-1 r, and the
// partials of r^T z and r^T r; VEC consecutive elements per thread and step.
template <int VEC>
__global__ __launch_bounds__(256) void pcg_init_kernel(const float* __restrict__ b,
                                                       const float* __restrict__ diag, float lambda,
                                                       const float* __restrict__ dvec, int64_t P,
                                                       float* __restrict__ x, float* __restrict__ r,
                                                       float* __restrict__ z, float* __restrict__ p,
                                                       float* __restrict__ minv, double* __restrict__ partials) {
  __shared__ double s_red[256];
  double rz = 0.0, rr = 0.0;
  using V = Vec<VEC>;
  const int64_t units = P / VEC;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < units; i += (int64_t)gridDim.x * 256) {
    const typename V::T dv = V::load(diag, i), bv = V::load(b, i);
    typename V::T ev;
    if (dvec) ev = V::load(dvec, i);
    typename V::T mv, zv, xv;
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      const float m = 1.f / (V::at(dv, c) + lambda * (dvec ? V::at(ev, c) : 1.f));
      const float bi = V::at(bv, c), zi = m * bi;
      V::at(mv, c) = m;
      V::at(zv, c) = zi;
      V::at(xv, c) = 0.f;
      rz += (double)bi * zi;
      rr += (double)bi * bi;
    }
    V::store(minv, i, mv);
    V::store(x, i, xv);
    V::store(r, i, bv);
    V::store(z, i, zv);
    V::store(p, i, zv);
  }
  if (blockIdx.x == 0) {  // the last P % VEC elements
    for (int64_t i = units * VEC + threadIdx.x; i < P; i += 256) {
      const float m = 1.f / (diag[i] + lambda * (dvec ? dvec[i] : 1.f));
      const float bi = b[i], zi = m * bi;
      minv[i] = m;
      x[i] = 0.f;
      r[i] = bi;
      z[i] = zi;
      p[i] = zi;
      rz += (double)bi * zi;
      rr += (double)bi * bi;
    }
  }
  const double a = block_sum(rz, s_red);
  const double c = block_sum(rr, s_red);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = a;
    partials[kRedBlocks + blockIdx.x] = c;
  }
}

// Scalars after pcg_init_kernel: r0^T z0 and r0^T r0 from its partials.
__global__ __launch_bounds__(256) void pcg_init_scalars_kernel(const double* __restrict__ partials,
                                                               double* __restrict__ sc) {
  __shared__ double s_red[256];
  const double rz = reduce_partials(partials, kRedBlocks, s_red);
  const double rr = reduce_partials(partials + kRedBlocks, kRedBlocks, s_red);
  if (threadIdx.x == 0) {
    for (int i = 0; i < kScalars; ++i) sc[i] = 0.0;
    sc[kRZ] = sc[kRZ0] = rz;
    sc[kRR] = sc[kRR0] = rr;
    if (!isfinite(rz) || !isfinite(rr)) {  // NaN / Inf in b or the preconditioner
      sc[kFail] = LMRS_FAIL_NONFINITE;
      sc[kStop] = 1.0;
    }
  }
}

// Iteration i reads the scalar bank cur and pcg_dir_kernel writes the bank
// of iteration i + 1, so no kernel reads a slot that it writes.
// alpha = r^T z / p^T u (0 once stopped); x += alpha p; r -= alpha u; z = M^-1 r.
// p^T u comes from the partials that the GN product's chain kernel leaves
// (pu_count of them, reduced in every block).
template <int VEC>
__global__ __launch_bounds__(256) void pcg_update_kernel(int64_t P, double* __restrict__ cur,
                                                         const double* __restrict__ pu_partials, int pu_count,
                                                         float* __restrict__ x, float* __restrict__ r,
                                                         float* __restrict__ z, const float* __restrict__ p,
                                                         const float* __restrict__ u,
                                                         const float* __restrict__ minv,
                                                         double* __restrict__ partials) {
  __shared__ double s_red[256];
  const double pu = reduce_partials(pu_partials, pu_count, s_red);
  const double rz = cur[kRZ];
  const bool go = cur[kStop] == 0.0 && pu > 0.0 && rz > 1e-30 * cur[kRZ0];
  if (blockIdx.x == 0 && threadIdx.x == 0) cur[kPU] = pu;
  const float alpha = go ? (float)(rz / pu) : 0.f;
  double rz1 = 0.0, rr = 0.0;
  // VEC consecutive elements per thread and step (16-byte loads when 4)
  using V = Vec<VEC>;
  const int64_t units = P / VEC;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < units; i += (int64_t)gridDim.x * 256) {
    typename V::T rv = V::load(r, i);
    const typename V::T mv = V::load(minv, i);
    if (go) {
      typename V::T xv = V::load(x, i);
      const typename V::T pv = V::load(p, i), uv = V::load(u, i);
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        V::at(xv, c) += alpha * V::at(pv, c);
        V::at(rv, c) -= alpha * V::at(uv, c);
      }
      V::store(x, i, xv);
      V::store(r, i, rv);
    }
    typename V::T zv;
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      const float ri = V::at(rv, c), zi = V::at(mv, c) * ri;
      V::at(zv, c) = zi;
      rz1 += (double)ri * zi;
      rr += (double)ri * ri;
    }
    V::store(z, i, zv);
  }
  if (blockIdx.x == 0) {  // the last P % VEC elements
    for (int64_t i = units * VEC + threadIdx.x; i < P; i += 256) {
      float ri = r[i];
      if (go) {
        x[i] += alpha * p[i];
        ri -= alpha * u[i];
        r[i] = ri;
      }
      const float zi = minv[i] * ri;
      z[i] = zi;
      rz1 += (double)ri * zi;
      rr += (double)ri * ri;
    }
  }
  const double a = block_sum(rz1, s_red);
  const double c = block_sum(rr, s_red);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = a;
    partials[kRedBlocks + blockIdx.x] = c;
  }
}

// r_{i+1}^T z_{i+1} and r^T r from pcg_update_kernel's partials; beta, the
// stop flag and the next scalar bank; p = z + beta p.
template <int VEC>
__global__ __launch_bounds__(256) void pcg_dir_kernel(int64_t P, const double* __restrict__ cur,
                                                      double* __restrict__ next,
                                                      const double* __restrict__ partials,
                                                      const float* __restrict__ z, float* __restrict__ p) {
  __shared__ double s_red[256];
  const double rz_new = reduce_partials(partials, kRedBlocks, s_red);
  const double rr = reduce_partials(partials + kRedBlocks, kRedBlocks, s_red);
  const double rz = cur[kRZ], pu = cur[kPU];
  const bool live = cur[kStop] == 0.0 && rz > 1e-30 * cur[kRZ0];  // not stopped, not converged
  bool go = live && pu > 0.0;
  // failures: p^T A p <= 0 (or not a number) before convergence, which an SPD
  // operator cannot give (breakdown); a residual that is not finite
  double fail = cur[kFail];
  if (live && !(pu > 0.0 && isfinite(pu))) fail = (double)((int)fail | LMRS_FAIL_BREAKDOWN);
  if (go && !(isfinite(rz_new) && isfinite(rr))) {
    fail = (double)((int)fail | LMRS_FAIL_NONFINITE);
    go = false;
  }
  const double beta = go ? rz_new / rz : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int i = 0; i < kScalars; ++i) next[i] = cur[i];
    next[kRZNew] = rz_new;
    next[kRR] = rr;
    next[kBeta] = beta;
    next[kFail] = fail;
    if (go) {
      next[kRZ] = rz_new;
      next[kDone] = cur[kDone] + 1.0;
    } else {
      next[kStop] = 1.0;
    }
  }
  if (!go) return;
  const float b = (float)beta;
  using V = Vec<VEC>;
  const int64_t units = P / VEC;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < units; i += (int64_t)gridDim.x * 256) {
    const typename V::T zv = V::load(z, i);
    typename V::T pv = V::load(p, i);
#pragma unroll
    for (int c = 0; c < VEC; ++c) V::at(pv, c) = V::at(zv, c) + b * V::at(pv, c);
    V::store(p, i, pv);
  }
  if (blockIdx.x == 0)
    for (int64_t i = units * VEC + threadIdx.x; i < P; i += 256) p[i] = z[i] + b * p[i];
}

__global__ void pcg_report_kernel(const double* __restrict__ sc, const double* __restrict__ bx,
                                  float* __restrict__ report) {
  if (threadIdx.x != 0) return;
  report[LMRS_REP_CG_DONE] = (float)sc[kDone];
  report[LMRS_REP_R0] = (float)sqrt(sc[kRR0]);
  report[LMRS_REP_RN] = (float)sqrt(sc[kRR]);
  report[LMRS_REP_BX] = (float)bx[0];
  report[LMRS_REP_STATUS] = (float)sc[kFail];
}

// Partials per block of max |x| over the DC colour coefficients [dc0, dc0 + ndc)
// and of the count of entries of x (all P) that are not finite.
__global__ __launch_bounds__(256) void absmax_partial_kernel(const float* __restrict__ x, int64_t P, int64_t dc0,
                                                             int64_t ndc, double* __restrict__ partials) {
  __shared__ double s_red[256];
  double m = 0.0, bad = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < P; i += (int64_t)gridDim.x * 256) {
    const float v = x[i];
    if (!isfinite(v)) bad += 1.0;
    else if (i >= dc0 && i < dc0 + ndc) m = fmax(m, (double)fabsf(v));
  }
  s_red[threadIdx.x] = m;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) s_red[threadIdx.x] = fmax(s_red[threadIdx.x], s_red[threadIdx.x + d]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = s_red[0];
  const double nb = block_sum(bad, s_red);
  if (threadIdx.x == 0) partials[kRedBlocks + blockIdx.x] = nb;
}

// eta from the partials, and the step's failure bits: the PCG's, plus
// LMRS_FAIL_NONFINITE when x has an entry that is not finite. out[0] = eta,
// out[1] = failure bits (the update is skipped when they are non-zero).
__global__ __launch_bounds__(256) void lr_kernel(const double* __restrict__ partials, int count,
                                                  lmrs_lm_params prm, const double* __restrict__ pcg_fail,
                                                  double* __restrict__ out, float* __restrict__ report) {
  __shared__ double s_red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) m = fmax(m, partials[i]);
  s_red[threadIdx.x] = m;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) s_red[threadIdx.x] = fmax(s_red[threadIdx.x], s_red[threadIdx.x + d]);
    __syncthreads();
  }
  m = s_red[0];
  __syncthreads();
  double bad = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) bad += partials[kRedBlocks + i];
  bad = block_sum(bad, s_red);
  if (threadIdx.x != 0) return;
  int fail = pcg_fail ? (int)pcg_fail[0] : 0;
  if (bad > 0.0) fail |= LMRS_FAIL_NONFINITE;
  double eta;
  if (prm.iter < prm.warm_iters) eta = prm.eta_warm;
  else eta = m > 0.0 ? fmin((double)prm.eta_cap, 1.0 / m) : (double)prm.eta_cap;
  out[0] = eta;
  out[1] = (double)fail;
  if (report) {
    report[LMRS_REP_ETA] = (float)eta;
    report[LMRS_REP_XDC_MAX] = (float)m;
    report[LMRS_REP_STATUS] = (float)fail;
  }
}

__global__ __launch_bounds__(256) void lm_apply_kernel(float* __restrict__ beta, const float* __restrict__ x,
                                                       int64_t P, const double* __restrict__ eta) {
  if (eta[1] != 0.0) return;  // a numeric failure: the parameters stay as they are
  const float e = (float)eta[0];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < P; i += (int64_t)gridDim.x * 256)
    beta[i] -= e * x[i];
}

// SSIM residual with the diagonal approximation (Supp. B; Sec. 6 names the
// approximation, the paper gives no formula). One workgroup per (view, tile):
// the tile's pixels and a 5-pixel ring around it, of the rendered image and
// of the target, are staged in LDS (zero outside the image), and each
// (sample, channel) item sums its 11 x 11 Gaussian window (sigma 1.5, weights
// summing to 1) in FP64: the local means, variances and covariance of the
// SSIM of Wang et al., C1 = 0.01^2, C2 = 0.03^2. With the centre pixel's
// window weight g0, the derivative of SSIM with respect to the rendered
// colour of the centre pixel alone (the diagonal approximation) follows from
// d mu_x = g0, d sigma_x^2 = 2 g0 (x_p - mu_x), d sigma_xy = g0 (y_p - mu_y).
// Writes, with r = x_p - y_p, rho = 1 - SSIM, delta = -d SSIM / d x_p:
//   u = w (r + s delta rho), wc = w (1 + s delta^2),
// and the tile's share of the objective, sum w (r^2 + s rho^2).
constexpr int kSsimHalf = 5;                      // 11 x 11 window
constexpr int kSsimSpan = kTile + 2 * kSsimHalf;  // staged rows and columns
constexpr int kSsimPlane = kSsimSpan * kSsimSpan;

__global__ __launch_bounds__(256) void ssim_kernel(const float* __restrict__ image, const float* __restrict__ targets,
                                                   const int32_t* __restrict__ view_ids,
                                                   const uint8_t* __restrict__ pix, const float* __restrict__ wts,
                                                   int T, int TX, int W, int H, int k, double s_w,
                                                   float* __restrict__ u, float* __restrict__ wc,
                                                   double* __restrict__ tile_loss) {
  __shared__ float sx[3 * kSsimPlane];
  __shared__ float sy[3 * kSsimPlane];
  __shared__ double s_red[256];
  const int tid = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int v = (int)(tile / T), t = (int)(tile % T);
  const int cam = view_ids ? view_ids[v] : v;
  const int x0 = (t % TX) * kTile - kSsimHalf, y0 = (t / TX) * kTile - kSsimHalf;
  for (int e = tid; e < kSsimPlane; e += 256) {
    const int gx = x0 + e % kSsimSpan, gy = y0 + e / kSsimSpan;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    const int64_t pi = in ? (((int64_t)v * H + gy) * W + gx) * 3 : 0;
    const int64_t ti = in ? (((int64_t)cam * H + gy) * W + gx) * 3 : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sx[c * kSsimPlane + e] = in ? image[pi + c] : 0.f;
      sy[c * kSsimPlane + e] = in ? targets[ti + c] : 0.f;
    }
  }
  // the window's 1-D weights exp(-d^2 / (2 sigma^2)), normalised
  double g[2 * kSsimHalf + 1];
  double gs = 0.0;
#pragma unroll
  for (int a = 0; a <= 2 * kSsimHalf; ++a) {
    const double d = (double)(a - kSsimHalf);
    g[a] = exp(-d * d / (2.0 * 1.5 * 1.5));
    gs += g[a];
  }
#pragma unroll
  for (int a = 0; a <= 2 * kSsimHalf; ++a) g[a] /= gs;
  const double g0 = g[kSsimHalf] * g[kSsimHalf];
  constexpr double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
  __syncthreads();
  double loss = 0.0;
  for (int q = tid; q < 3 * k; q += 256) {
    const int j = q / 3, c = q % 3;
    const int64_t i = tile * k + j;
    const int p = pix ? (int)pix[i] : j;
    const int off = c * kSsimPlane + (p >> 4) * kSsimSpan + (p & 15);  // the window's first row and column
    double mx = 0.0, my = 0.0, mxx = 0.0, myy = 0.0, mxy = 0.0;
#pragma unroll
    for (int a = 0; a <= 2 * kSsimHalf; ++a) {
      double rx = 0.0, ry = 0.0, rxx = 0.0, ryy = 0.0, rxy = 0.0;
#pragma unroll
      for (int b = 0; b <= 2 * kSsimHalf; ++b) {
        const double xv = sx[off + a * kSsimSpan + b], yv = sy[off + a * kSsimSpan + b];
        rx += g[b] * xv;
        ry += g[b] * yv;
        rxx += g[b] * (xv * xv);
        ryy += g[b] * (yv * yv);
        rxy += g[b] * (xv * yv);
      }
      mx += g[a] * rx;
      my += g[a] * ry;
      mxx += g[a] * rxx;
      myy += g[a] * ryy;
      mxy += g[a] * rxy;
    }
    const double vx = mxx - mx * mx, vy = myy - my * my, cxy = mxy - mx * my;
    const double a1 = 2.0 * mx * my + C1, a2 = 2.0 * cxy + C2;
    const double b1 = mx * mx + my * my + C1, b2 = vx + vy + C2;
    const double ssim = (a1 * a2) / (b1 * b2);
    const int centre = off + kSsimHalf * kSsimSpan + kSsimHalf;
    const double xp = sx[centre], yp = sy[centre];
    const double dssim = 2.0 * g0 * ((my * a2 + a1 * (yp - my)) / (b1 * b2) - ssim * (mx / b1 + (xp - mx) / b2));
    const double delta = -dssim, rho = 1.0 - ssim, r = xp - yp;
    const double w = wts ? (double)wts[i] : 1.0;
    u[3 * i + c] = (float)(w * (r + s_w * delta * rho));
    wc[3 * i + c] = (float)(w * (1.0 + s_w * delta * delta));
    loss += w * (r * r + s_w * rho * rho);
  }
  const double tot = block_sum(loss, s_red);
  if (tid == 0 && tile_loss) tile_loss[tile] = tot;
}

}  // namespace

void launch_sample_uniform(const lmrs_frame* f, const FrameDims& d, uint64_t seed, int iter, hipStream_t s) {
  const int64_t tiles = (int64_t)d.V * d.T;
  sample_kernel<<<(unsigned)((tiles + kSampleWaves - 1) / kSampleWaves), kWave * kSampleWaves, 0, s>>>(
      f->view_ids, d.T, d.k, tiles, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), (uint32_t)iter,
      f->pix, f->w);
}

void launch_sample_residual(const lmrs_frame* f, const FrameDims& d, const float* scores, uint64_t seed,
                            int iter, hipStream_t s) {
  sample_residual_kernel<<<(unsigned)((int64_t)d.V * d.T), 256, 0, s>>>(
      scores, f->view_ids, d.T, d.k, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), (uint32_t)iter,
      f->pix, f->w);
}

void launch_sample_gaussian(const lmrs_frame* f, const FrameDims& d, const float* counts, uint64_t seed,
                            int iter, hipStream_t s) {
  sample_gaussian_kernel<<<(unsigned)((int64_t)d.V * d.T), 256, 0, s>>>(
      counts, f->view_ids, d.T, d.k, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), (uint32_t)iter,
      f->pix, f->w);
}

void launch_residual(const lmrs_frame* f, const FrameDims& d, const float* targets, float* wr,
                     double* partials, float* report, hipStream_t s) {
  residual_kernel<<<kRedBlocks, 256, 0, s>>>(f->color, targets, f->pix, f->w, f->view_ids, d.T, d.TX,
                                             d.W, d.H, d.k, d.S, wr, partials);
  finalize_kernel<<<1, 256, 0, s>>>(partials, kRedBlocks, 1, kRedBlocks, partials + 2 * kRedBlocks);
  if (report) report_kernel<<<1, 64, 0, s>>>(partials + 2 * kRedBlocks, report, LMRS_REP_LOSS);
}

void launch_ssim(const lmrs_frame* f, const FrameDims& d, const float* targets, float s_w, float* u,
                 double* tile_loss, double* loss_out, float* report, hipStream_t s) {
  const int64_t tiles = (int64_t)d.V * d.T;
  ssim_kernel<<<(unsigned)tiles, 256, 0, s>>>(f->image, targets, f->view_ids, f->pix, f->w, d.T, d.TX, d.W, d.H,
                                              d.k, (double)s_w, u, f->wc, tile_loss);
  if (loss_out && tile_loss) {
    finalize_kernel<<<1, 256, 0, s>>>(tile_loss, (int)tiles, 1, (int)tiles, loss_out);
    if (report) report_kernel<<<1, 64, 0, s>>>(loss_out, report, LMRS_REP_LOSS);
  }
}

void launch_report_count(const int64_t* count, int64_t capacity, float* report, hipStream_t s,
                         const int64_t* pairs) {
  report_count_kernel<<<1, 64, 0, s>>>(count, capacity, report, pairs);
}

void launch_dot(const float* a, const float* b, int64_t n, double* partials, double* out, hipStream_t s) {
  dot_partial_kernel<<<kRedBlocks, 256, 0, s>>>(a, b, n, partials);
  finalize_kernel<<<1, 256, 0, s>>>(partials, kRedBlocks, 1, kRedBlocks, out);
}

static bool aligned16(const void* a) { return (reinterpret_cast<uintptr_t>(a) & 15) == 0; }

void launch_pcg_init(const float* b, const float* diag, float lambda, const float* dvec, int64_t P,
                     PcgState st, hipStream_t s) {
  if (aligned16(b) && aligned16(diag) && (!dvec || aligned16(dvec)) && aligned16(st.x) && aligned16(st.r) &&
      aligned16(st.z) && aligned16(st.p) && aligned16(st.minv))
    pcg_init_kernel<4><<<kRedBlocks, 256, 0, s>>>(b, diag, lambda, dvec, P, st.x, st.r, st.z, st.p, st.minv,
                                                  st.partials);
  else
    pcg_init_kernel<1><<<kRedBlocks, 256, 0, s>>>(b, diag, lambda, dvec, P, st.x, st.r, st.z, st.p, st.minv,
                                                  st.partials);
  pcg_init_scalars_kernel<<<1, 256, 0, s>>>(st.partials, st.bank(0));
}

void launch_pcg_iteration(int it, int64_t P, int pu_count, PcgState st, hipStream_t s) {
  double* cur = st.bank(it);
  const bool vec = aligned16(st.x) && aligned16(st.r) && aligned16(st.z) && aligned16(st.p) && aligned16(st.u) &&
                   aligned16(st.minv);
  if (vec) {
    pcg_update_kernel<4><<<kRedBlocks, 256, 0, s>>>(P, cur, st.partials, pu_count, st.x, st.r, st.z, st.p, st.u,
                                                    st.minv, st.partials + 2 * kRedBlocks);
    pcg_dir_kernel<4><<<kRedBlocks, 256, 0, s>>>(P, cur, st.bank(it + 1), st.partials + 2 * kRedBlocks, st.z,
                                                 st.p);
  } else {
    pcg_update_kernel<1><<<kRedBlocks, 256, 0, s>>>(P, cur, st.partials, pu_count, st.x, st.r, st.z, st.p, st.u,
                                                    st.minv, st.partials + 2 * kRedBlocks);
    pcg_dir_kernel<1><<<kRedBlocks, 256, 0, s>>>(P, cur, st.bank(it + 1), st.partials + 2 * kRedBlocks, st.z,
                                                 st.p);
  }
}

void launch_pcg_report(const float* b, int iters, int64_t P, PcgState st, float* report, hipStream_t s) {
  double* fin = st.bank(iters);
  launch_dot(b, st.x, P, st.partials, fin + 10, s);
  pcg_report_kernel<<<1, 64, 0, s>>>(fin, fin + 10, report);
}

const double* pcg_fail_slot(int iters, PcgState st) { return st.bank(iters) + kFail; }

void launch_lm_update(float* beta, const float* x, int n, int64_t P, const lmrs_lm_params& prm,
                      const double* pcg_fail, double* partials, float* report, hipStream_t s) {
  absmax_partial_kernel<<<kRedBlocks, 256, 0, s>>>(x, P, (int64_t)11 * n, (int64_t)3 * n, partials);
  lr_kernel<<<1, 256, 0, s>>>(partials, kRedBlocks, prm, pcg_fail, partials + 2 * kRedBlocks, report);
  lm_apply_kernel<<<kRedBlocks, 256, 0, s>>>(beta, x, P, partials + 2 * kRedBlocks);
}

}  // namespace lmrs
