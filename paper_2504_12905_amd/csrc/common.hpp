// Device-side building blocks shared by the lmrs kernels (gfx950, wave64).
//
// * dualf: (value, derivative) pairs for forward-mode differentiation, the
//   dual numbers of the paper's J p kernel (Supp. A, Alg. 3);
// * the real spherical-harmonic colour basis of degree <= 3;
// * projection of one Gaussian into one view (Sec. 3, eq. 1-3, EWA splatting):
//   templated on the scalar so the same code gives the record (float) and its
//   tangent (dualf), plus the hand-written adjoint used by J^T u;
// * the per-pixel opacity test shared by every splat kernel;
// * wave64 scans and reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lmrs.h"

namespace lmrs {

constexpr int kTile = 16;
constexpr int kWave = 64;
constexpr int kGram = 32;            // Gram entries kept per (view, Gaussian)
constexpr int kGradRow = 16;         // floats per (view, Gaussian) row of screen gradients (9 used)

// ---------------------------------------------------------------- fixed point
// Deterministic accumulation (lmrs_frame.deterministic). A float term v goes
// into an accumulator as two 64-bit integers: hi = floor(v 2^20) and lo = the
// rest in units of 2^-60 (0 <= lo < 2^40), each added by an integer atomic.
// Integer sums do not depend on the order of the adds, so the accumulated
// value hi 2^-20 + lo 2^-60 has the same bits on every run. v 2^20 is exact
// (a power-of-two scaling of a float, in FP64), so is its fractional part;
// the split is exact for |v| >= 2^-37 and rounds only below 2^-60. Range:
// |v| < 2^30 per term (a term beyond that, or not finite, sets the row's
// poison word and the reader takes the row as NaN), |sum| < 2^42, at most
// 2^23 terms per accumulator. A row holds the hi words of its components,
// then (from word LO) their lo words, and a poison word P; the hi and the lo
// words of a screen-gradient row each fill part of one 128-byte line, so an
// atomic instruction over a row's components touches one line, as the float
// rows do.
constexpr int kFixGradRow = 32, kFixGradLo = 16, kFixGradPoison = 25;  // 256 B per row
constexpr int kFixGramRow = 80, kFixGramLo = 32, kFixGramPoison = 64;  // 640 B per row
constexpr int kFixGradFloats = 2 * kFixGradRow;  // the same rows counted in 32-bit words
constexpr int kFixGramFloats = 2 * kFixGramRow;

__device__ __forceinline__ void fix_split(float v, long long& hi, long long& lo) {
  const double s = (double)v * 0x1p20;
  const double h = floor(s);
  hi = (long long)h;
  lo = (long long)rint((s - h) * 0x1p40);
}

// Component q of a fixed-point row += v (hi word row[q], lo word row[LO + q],
// poison word row[P]).
template <int LO, int P>
__device__ __forceinline__ void fix_add(unsigned long long* row, int q, float v) {
  if (!(fabsf(v) < 0x1p30f)) {  // NaN fails the test too
    atomicOr(row + P, 1ull);
    return;
  }
  long long hi, lo;
  fix_split(v, hi, lo);
  if (hi) atomicAdd(row + q, (unsigned long long)hi);
  if (lo) atomicAdd(row + LO + q, (unsigned long long)lo);
}

__device__ __forceinline__ float fix_value(unsigned long long hi, unsigned long long lo) {
  return (float)((double)(long long)hi * 0x1p-20 + (double)(long long)lo * 0x1p-60);
}

// Screen-gradient row `row` (= view * n + Gaussian), component q < 9: a float
// atomic into the kGradRow-float rows, or fixed point into kFixGradRow-word rows.
__device__ __forceinline__ void grad_add(float* grad2d, bool fixed, size_t row, int q, float v) {
  if (fixed) fix_add<kFixGradLo, kFixGradPoison>(reinterpret_cast<unsigned long long*>(grad2d) + row * kFixGradRow, q, v);
  else atomicAdd(&grad2d[row * kGradRow + q], v);
}

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC 2011): 10 rounds of two 32x32->64
// multiplies with key bumps by the Weyl constants. Host and device.
__host__ __device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

// ------------------------------------------------------------------ duals
struct dualf {
  float v, d;
  __device__ __forceinline__ dualf() : v(0.f), d(0.f) {}
  __device__ __forceinline__ dualf(float a) : v(a), d(0.f) {}  // NOLINT
  __device__ __forceinline__ dualf(float a, float b) : v(a), d(b) {}
};
__device__ __forceinline__ dualf operator+(dualf a, dualf b) { return dualf(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ dualf operator-(dualf a, dualf b) { return dualf(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ dualf operator-(dualf a) { return dualf(-a.v, -a.d); }
__device__ __forceinline__ dualf operator*(dualf a, dualf b) {
  return dualf(a.v * b.v, a.v * b.d + a.d * b.v);
}
__device__ __forceinline__ dualf operator/(dualf a, dualf b) {
  const float r = 1.f / b.v;
  const float q = a.v * r;
  return dualf(q, (a.d - q * b.d) * r);
}
__device__ __forceinline__ float tval(float x) { return x; }
__device__ __forceinline__ double tval(double x) { return x; }
__device__ __forceinline__ float tval(dualf x) { return x.v; }
__device__ __forceinline__ float texp(float x) { return expf(x); }
__device__ __forceinline__ double texp(double x) { return exp(x); }
__device__ __forceinline__ double trsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ dualf texp(dualf x) {
  const float e = expf(x.v);
  return dualf(e, e * x.d);
}
__device__ __forceinline__ float trsqrt(float x) { return 1.f / sqrtf(x); }
__device__ __forceinline__ dualf trsqrt(dualf x) {
  const float r = 1.f / sqrtf(x.v);
  return dualf(r, -0.5f * r * r * r * x.d);
}

// --------------------------------------------------------------- SH basis
template <int DEG>
struct ShDims {
  static constexpr int K = (DEG + 1) * (DEG + 1);  // coefficients per channel
  static constexpr int PG = 11 + 3 * K;            // parameters per Gaussian
};

// Real spherical harmonics, index l*l + l + m: Y_{l,0} = Y_l^0,
// Y_{l,m} = sqrt(2) Re Y_l^m, Y_{l,-m} = sqrt(2) Im Y_l^m (m > 0), with the
// Condon-Shortley phase in Y_l^m, written as polynomials of a unit direction.
template <int DEG, class T>
__device__ __forceinline__ void sh_eval(T x, T y, T z, T* Y) {
  Y[0] = T(0.28209479177387814f);
  if constexpr (DEG >= 1) {
    Y[1] = T(-0.48860251190291987f) * y;
    Y[2] = T(0.48860251190291987f) * z;
    Y[3] = T(-0.48860251190291987f) * x;
  }
  if constexpr (DEG >= 2) {
    const T xx = x * x, yy = y * y, zz = z * z;
    Y[4] = T(1.0925484305920792f) * x * y;
    Y[5] = T(-1.0925484305920792f) * y * z;
    Y[6] = T(0.31539156525252005f) * (T(2.f) * zz - xx - yy);
    Y[7] = T(-1.0925484305920792f) * x * z;
    Y[8] = T(0.5462742152960396f) * (xx - yy);
    if constexpr (DEG >= 3) {
      Y[9] = T(-0.5900435899266435f) * y * (T(3.f) * xx - yy);
      Y[10] = T(2.890611442640554f) * x * y * z;
      Y[11] = T(-0.4570457994644658f) * y * (T(4.f) * zz - xx - yy);
      Y[12] = T(0.3731763325901154f) * z * (T(2.f) * zz - T(3.f) * xx - T(3.f) * yy);
      Y[13] = T(-0.4570457994644658f) * x * (T(4.f) * zz - xx - yy);
      Y[14] = T(1.445305721320277f) * z * (xx - yy);
      Y[15] = T(-0.5900435899266435f) * x * (xx - T(3.f) * yy);
    }
  }
}

// --------------------------------------------------------------- cameras
struct CamView {
  lmrs_camera c;
  float pos[3];  // camera centre -R^T t
};

__device__ __forceinline__ CamView load_cam(const lmrs_camera* cams, const int32_t* view_ids, int v) {
  CamView cv;
  cv.c = cams[view_ids ? view_ids[v] : v];
  for (int i = 0; i < 3; ++i)
    cv.pos[i] = -(cv.c.R[i] * cv.c.t[0] + cv.c.R[3 + i] * cv.c.t[1] + cv.c.R[6 + i] * cv.c.t[2]);
  return cv;
}

// Camera-space mean and projected centre in FP64: these decide the near-plane
// cull, the tile rectangle and the depth order, so they are taken to FP64
// accuracy (two FP64 evaluations of them agree unless a value lies within
// ~1e-12 of its threshold).
__device__ __forceinline__ void decision_point(const lmrs_camera& c, double mx, double my, double mz,
                                               double* tc, double* u, double* v) {
  for (int i = 0; i < 3; ++i) {
    double acc = (double)c.t[i];
    acc = fma((double)c.R[3 * i + 0], mx, acc);
    acc = fma((double)c.R[3 * i + 1], my, acc);
    acc = fma((double)c.R[3 * i + 2], mz, acc);
    tc[i] = acc;
  }
  *u = fma((double)c.fx, tc[0] / tc[2], (double)c.cx);
  *v = fma((double)c.fy, tc[1] / tc[2], (double)c.cy);
}

// The camera depth z of a (view, Gaussian) travels in the screen record as
// the two 32-bit halves of its FP64 bits (record slots 9 = low, 11 = high);
// for z > 0 those bits order like z itself.
__device__ __forceinline__ void depth_words(double z, float* lo, float* hi) {
  const uint64_t b = (uint64_t)__double_as_longlong(z);
  *lo = __uint_as_float((uint32_t)b);
  *hi = __uint_as_float((uint32_t)(b >> 32));
}
__device__ __forceinline__ uint64_t depth_bits(float lo, float hi) {
  return ((uint64_t)__float_as_uint(hi) << 32) | __float_as_uint(lo);
}

// 32-bit sort key of a depth, monotone in z: 0 for z <= 0 (never listed); for
// z > 0, 5 bits of binary exponent e - kDepthEmin and the top 27 bits of the
// mantissa, saturating at 1 below 2^kDepthEmin and at 2^32 - 1 from
// 2^(kDepthEmin + 32) on. Depths with equal keys (within 2^-27 relative of
// each other) are put in FP64 order by a tie pass over the sorted keys.
constexpr int kDepthEmin = -16;
__device__ __forceinline__ uint32_t depth_sort_key(uint64_t b) {
  if ((int64_t)b <= 0) return 0u;
  const int e = (int)((b >> 52) & 0x7ff) - 1023 - kDepthEmin;
  if (e < 0) return 1u;
  if (e >= 32) return 0xffffffffu;
  return max(((uint32_t)e << 27) | (uint32_t)((b >> 25) & 0x7ffffffu), 1u);
}

// Load the PG parameters of Gaussian g (component-major beta).
template <int PG, class T>
__device__ __forceinline__ void load_params(const float* beta, int n, int g, T* prm) {
#pragma unroll
  for (int j = 0; j < PG; ++j) prm[j] = T(beta[(size_t)j * n + g]);
}

// ----------------------------------------------------------- projection
// Geometry of the screen record, (u, v, f11, f12, f22), from mean, log-scale
// and quaternion (prm[0..10)). Sigma = R S S^T R^T (eq. 2); Sigma_2D =
// J W Sigma W^T J^T + lowpass I = [[a, b], [b, c]] with J the pinhole
// Jacobian at the camera-space mean, computed as K K^T with K = J W R S (rows
// k1, k2). The record holds the Cholesky factor F = [[f11, f12], [0, f22]] of
// the conic Q = Sigma_2D^-1 = F^T F instead of Q itself, so that the exponent
// of eq. 3, -1/2 d^T Q d, is evaluated as -1/2 (|f11 dx + f12 dy|^2 + |f22 dy|^2)
// (a sum of squares: no cancellation between terms of size |Q| |d|^2 along
// the long axis of a large, thin footprint):
//   f22 = 1 / sqrt(c),  f11 = c r,  f12 = -b r,  r = 1 / sqrt(c det),
// with det = a c - b^2 formed without cancellation by the Cauchy-Binet
// identity det = |k1 x k2|^2 + lowpass (|k1|^2 + |k2|^2) + lowpass^2.
// The covariance factor M = R diag(s) of Sigma = M M^T (eq. 2), from the
// quaternion (normalised here) and the log-scales; it does not depend on the
// view.
template <class T>
__device__ __forceinline__ void cov_factor(const T* prm, T* M) {
  const T inv = trsqrt(prm[6] * prm[6] + prm[7] * prm[7] + prm[8] * prm[8] + prm[9] * prm[9]);
  const T w = prm[6] * inv, x = prm[7] * inv, y = prm[8] * inv, z = prm[9] * inv;
  const T R[9] = {T(1.f) - T(2.f) * (y * y + z * z), T(2.f) * (x * y - w * z), T(2.f) * (x * z + w * y),
                  T(2.f) * (x * y + w * z), T(1.f) - T(2.f) * (x * x + z * z), T(2.f) * (y * z - w * x),
                  T(2.f) * (x * z - w * y), T(2.f) * (y * z + w * x), T(1.f) - T(2.f) * (x * x + y * y)};
  const T s[3] = {texp(prm[3]), texp(prm[4]), texp(prm[5])};
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[3 * l + j] = R[3 * l + j] * s[j];
}

// proj_geom with the covariance factor M given (cov_factor).
template <class T>
__device__ __forceinline__ void proj_geom_m(const T* prm, const T* M, const CamView& cv, float lowpass, T* rec,
                                            double* a_out, double* b_out, double* c_out) {
  const lmrs_camera& c = cv.c;
  const T mx = prm[0], my = prm[1], mz = prm[2];
  const T tx = T(c.R[0]) * mx + T(c.R[1]) * my + T(c.R[2]) * mz + T(c.t[0]);
  const T ty = T(c.R[3]) * mx + T(c.R[4]) * my + T(c.R[5]) * mz + T(c.t[1]);
  const T tz = T(c.R[6]) * mx + T(c.R[7]) * my + T(c.R[8]) * mz + T(c.t[2]);
  const T iz = T(1.f) / tz;
  const T J00 = T(c.fx) * iz, J02 = -(T(c.fx) * tx * iz * iz);
  const T J11 = T(c.fy) * iz, J12 = -(T(c.fy) * ty * iz * iz);
  T Tm[6];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    Tm[j] = J00 * T(c.R[j]) + J02 * T(c.R[6 + j]);
    Tm[3 + j] = J11 * T(c.R[3 + j]) + J12 * T(c.R[6 + j]);
  }
  T K[6];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      K[3 * i + j] = Tm[3 * i + 0] * M[j] + Tm[3 * i + 1] * M[3 + j] + Tm[3 * i + 2] * M[6 + j];
  const T n1 = K[0] * K[0] + K[1] * K[1] + K[2] * K[2];
  const T n2 = K[3] * K[3] + K[4] * K[4] + K[5] * K[5];
  const T b = K[0] * K[3] + K[1] * K[4] + K[2] * K[5];
  const T w0 = K[1] * K[5] - K[2] * K[4], w1 = K[2] * K[3] - K[0] * K[5], w2 = K[0] * K[4] - K[1] * K[3];
  const T det = (w0 * w0 + w1 * w1 + w2 * w2) + T(lowpass) * (n1 + n2) + T(lowpass) * T(lowpass);
  const T cc = n2 + T(lowpass);
  const T r = trsqrt(cc * det);
  rec[0] = T(c.fx) * tx * iz + T(c.cx);
  rec[1] = T(c.fy) * ty * iz + T(c.cy);
  rec[2] = cc * r;
  rec[3] = -(b * r);
  rec[4] = trsqrt(cc);
  if (a_out) { *a_out = tval(n1 + T(lowpass)); *b_out = tval(b); *c_out = tval(cc); }
}

template <class T>
__device__ __forceinline__ void proj_geom(const T* prm, const CamView& cv, float lowpass, T* rec,
                                          double* a_out, double* b_out, double* c_out) {
  T M[9];
  cov_factor(prm, M);
  proj_geom_m(prm, M, cv, lowpass, rec, a_out, b_out, c_out);
}

// Unit direction from the camera centre to the mean.
template <class T>
__device__ __forceinline__ void view_dir(const T* prm, const CamView& cv, T* d) {
  T dx = prm[0] - T(cv.pos[0]), dy = prm[1] - T(cv.pos[1]), dz = prm[2] - T(cv.pos[2]);
  const T dinv = trsqrt(dx * dx + dy * dy + dz * dz);
  d[0] = dx * dinv; d[1] = dy * dinv; d[2] = dz * dinv;
}

// View-dependent colour 0.5 + sum_k Y_k(dir) f_k (prm[11 + 3k + c] = f_kc).
template <int DEG, class T>
__device__ __forceinline__ void proj_color(const T* prm, const CamView& cv, T* rgb) {
  constexpr int K = ShDims<DEG>::K;
  T d[3];
  view_dir(prm, cv, d);
  T Y[K];
  sh_eval<DEG>(d[0], d[1], d[2], Y);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    T acc = T(0.5f);
#pragma unroll
    for (int k = 0; k < K; ++k) acc = acc + Y[k] * prm[11 + 3 * k + ch];
    rgb[ch] = acc;
  }
}

// Screen record (u, v, f11, f12, f22, opacity, r, g, b) of one Gaussian in one view.
template <int DEG, class T>
__device__ __forceinline__ void proj_core(const T* prm, const CamView& cv, float lowpass, T* rec, double* a_out,
                                          double* b_out, double* c_out) {
  proj_geom(prm, cv, lowpass, rec, a_out, b_out, c_out);
  rec[5] = T(1.f) / (T(1.f) + texp(-prm[10]));
  proj_color<DEG>(prm, cv, rec + 6);
}

// d rgb / d mean (3x3, [channel][axis]) through the view direction, by one
// dual pass of the SH basis per axis.
template <int DEG>
__device__ __forceinline__ void color_mean_jacobian(const float* prm, const CamView& cv, float* drgb) {
  constexpr int K = ShDims<DEG>::K;
  float dx = prm[0] - cv.pos[0], dy = prm[1] - cv.pos[1], dz = prm[2] - cv.pos[2];
  const float dinv = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
  dx *= dinv; dy *= dinv; dz *= dinv;
  const float dd[3] = {dx, dy, dz};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    // tangent of the unit direction along mean axis ax: (e_ax - d d_ax) / |dir|
    dualf Yd[K];
    sh_eval<DEG>(dualf(dx, ((ax == 0) - dx * dd[ax]) * dinv), dualf(dy, ((ax == 1) - dy * dd[ax]) * dinv),
                 dualf(dz, ((ax == 2) - dz * dd[ax]) * dinv), Yd);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float acc = 0.f;
#pragma unroll
      for (int k = 1; k < K; ++k) acc += Yd[k].d * prm[11 + 3 * k + ch];
      drgb[3 * ch + ax] = acc;
    }
  }
}

// Adjoint of proj_core, split so that what does not depend on the view is
// done once per Gaussian: GeoFactors holds the rotation, scales and
// M = R diag(s) of the 3-D covariance factor; proj_vjp_view adds one view's
// mean and SH-coefficient gradients to gp and its gradients of R, s and the
// opacity to an accumulator (linear in them), and proj_vjp_finish takes the
// accumulated ones back to the quaternion, log-scales and opacity logit.
struct GeoFactors {
  float w, x, y, z, inv;  // normalised quaternion and 1 / |q|
  float R[9], s[3], M[9];
};

struct GeoGrad {
  float gR[9], gs[3], go;
};

__device__ __forceinline__ GeoFactors geo_factors(const float* prm) {
  GeoFactors f;
  f.inv = 1.f / sqrtf(prm[6] * prm[6] + prm[7] * prm[7] + prm[8] * prm[8] + prm[9] * prm[9]);
  const float w = prm[6] * f.inv, x = prm[7] * f.inv, y = prm[8] * f.inv, z = prm[9] * f.inv;
  f.w = w;
  f.x = x;
  f.y = y;
  f.z = z;
  const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                      2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                      2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
#pragma unroll
  for (int q = 0; q < 9; ++q) f.R[q] = R[q];
  f.s[0] = expf(prm[3]);
  f.s[1] = expf(prm[4]);
  f.s[2] = expf(prm[5]);
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int j = 0; j < 3; ++j) f.M[3 * l + j] = f.R[3 * l + j] * f.s[j];
  return f;
}

__device__ __forceinline__ void geo_grad_zero(GeoGrad& a) {
#pragma unroll
  for (int q = 0; q < 9; ++q) a.gR[q] = 0.f;
  a.gs[0] = a.gs[1] = a.gs[2] = 0.f;
  a.go = 0.f;
}

// One view's share of gp[j] += sum_q grec[q] d rec_q / d prm_j.
template <int DEG>
__device__ __forceinline__ void proj_vjp_view(const float* prm, const GeoFactors& gf, const CamView& cv,
                                              float lowpass, const float* gr, float* gp, GeoGrad& acc) {
  constexpr int K2 = ShDims<DEG>::K;
  const lmrs_camera& c = cv.c;
  const float mx = prm[0], my = prm[1], mz = prm[2];
  const float tx = c.R[0] * mx + c.R[1] * my + c.R[2] * mz + c.t[0];
  const float ty = c.R[3] * mx + c.R[4] * my + c.R[5] * mz + c.t[1];
  const float tz = c.R[6] * mx + c.R[7] * my + c.R[8] * mz + c.t[2];
  const float iz = 1.f / tz, iz2 = iz * iz, iz3 = iz2 * iz;
  const float* M = gf.M;
  const float J00 = c.fx * iz, J02 = -c.fx * tx * iz2, J11 = c.fy * iz, J12 = -c.fy * ty * iz2;
  float Tm[6];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    Tm[j] = J00 * c.R[j] + J02 * c.R[6 + j];
    Tm[3 + j] = J11 * c.R[3 + j] + J12 * c.R[6 + j];
  }
  float K[6];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      K[3 * i + j] = Tm[3 * i] * M[j] + Tm[3 * i + 1] * M[3 + j] + Tm[3 * i + 2] * M[6 + j];
  const float n1 = K[0] * K[0] + K[1] * K[1] + K[2] * K[2];
  const float n2 = K[3] * K[3] + K[4] * K[4] + K[5] * K[5];
  const float b = K[0] * K[3] + K[1] * K[4] + K[2] * K[5];
  const float cw[3] = {K[1] * K[5] - K[2] * K[4], K[2] * K[3] - K[0] * K[5], K[0] * K[4] - K[1] * K[3]};
  const float det = (cw[0] * cw[0] + cw[1] * cw[1] + cw[2] * cw[2]) + lowpass * (n1 + n2) + lowpass * lowpass;
  const float cc = n2 + lowpass;
  const float r = 1.f / sqrtf(cc * det), ic = 1.f / cc;
  const float gu = gr[0], gv = gr[1], g11 = gr[2], g12 = gr[3], g22 = gr[4];
  // F: f11 = c r, f12 = -b r, f22 = c^-1/2 with r = (c det)^-1/2
  const float g_r = g11 * cc - g12 * b;
  const float gc = g11 * r - 0.5f * g_r * r * ic - 0.5f * g22 * ic * sqrtf(ic);
  const float gb = -g12 * r;
  const float gdet = -0.5f * g_r * r / det;
  // det = |k1 x k2|^2 + lowpass (|k1|^2 + |k2|^2) + lowpass^2; b = k1.k2; c = |k2|^2 + lowpass
  float gK[6];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
    const float k2xw = K[3 + j1] * cw[j2] - K[3 + j2] * cw[j1];  // (k2 x w)_j, w = k1 x k2
    const float wxk1 = cw[j1] * K[j2] - cw[j2] * K[j1];          // (w x k1)_j
    gK[j] = gb * K[3 + j] + gdet * 2.f * (k2xw + lowpass * K[j]);
    gK[3 + j] = gb * K[j] + 2.f * gc * K[3 + j] + gdet * 2.f * (wxk1 + lowpass * K[3 + j]);
  }
  // K = Tm M
  float gTm[6];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int l = 0; l < 3; ++l)
      gTm[3 * i + l] = gK[3 * i] * M[3 * l] + gK[3 * i + 1] * M[3 * l + 1] + gK[3 * i + 2] * M[3 * l + 2];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float gM = Tm[l] * gK[j] + Tm[3 + l] * gK[3 + j];
      acc.gR[3 * l + j] += gM * gf.s[j];
      acc.gs[j] += gM * gf.R[3 * l + j];
    }
  // Tm = J W
  float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    gJ00 += gTm[j] * c.R[j];
    gJ02 += gTm[j] * c.R[6 + j];
    gJ11 += gTm[3 + j] * c.R[3 + j];
    gJ12 += gTm[3 + j] * c.R[6 + j];
  }
  const float gtx = -gJ02 * c.fx * iz2 + gu * c.fx * iz;
  const float gty = -gJ12 * c.fy * iz2 + gv * c.fy * iz;
  const float gtz = -gJ00 * c.fx * iz2 + 2.f * gJ02 * c.fx * tx * iz3 - gJ11 * c.fy * iz2 +
                    2.f * gJ12 * c.fy * ty * iz3 - gu * c.fx * tx * iz2 - gv * c.fy * ty * iz2;
  float gm[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) gm[i] = c.R[i] * gtx + c.R[3 + i] * gty + c.R[6 + i] * gtz;
  acc.go += gr[5];
  // colour: d/d f_kc = Y_k(dir); d/d mean through the direction
  float d[3];
  view_dir(prm, cv, d);
  float Y[K2];
  sh_eval<DEG>(d[0], d[1], d[2], Y);
#pragma unroll
  for (int k = 0; k < K2; ++k)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) gp[11 + 3 * k + ch] += gr[6 + ch] * Y[k];
  if constexpr (DEG > 0) {
    float J[9];
    color_mean_jacobian<DEG>(prm, cv, J);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) gm[ax] += gr[6] * J[ax] + gr[7] * J[3 + ax] + gr[8] * J[6 + ax];
  }
  gp[0] += gm[0];
  gp[1] += gm[1];
  gp[2] += gm[2];
}

// The accumulated gradients of R, s and the opacity back to the quaternion
// (through its normalisation), the log-scales and the opacity logit.
__device__ __forceinline__ void proj_vjp_finish(const float* prm, const GeoFactors& gf, const GeoGrad& a,
                                                float* gp) {
#pragma unroll
  for (int j = 0; j < 3; ++j) gp[3 + j] += a.gs[j] * gf.s[j];
  const float w = gf.w, x = gf.x, y = gf.y, z = gf.z;
  const float* gR = a.gR;
  const float gw = 2.f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
  const float gx = 2.f * (y * gR[1] + z * gR[2] + y * gR[3] - 2.f * x * gR[4] - w * gR[5] + z * gR[6] +
                          w * gR[7] - 2.f * x * gR[8]);
  const float gy = 2.f * (-2.f * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
                          z * gR[7] - 2.f * y * gR[8]);
  const float gz = 2.f * (-2.f * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.f * z * gR[4] +
                          y * gR[5] + x * gR[6] + y * gR[7]);
  const float dq = w * gw + x * gx + y * gy + z * gz;
  gp[6] += (gw - w * dq) * gf.inv;
  gp[7] += (gx - x * dq) * gf.inv;
  gp[8] += (gy - y * dq) * gf.inv;
  gp[9] += (gz - z * dq) * gf.inv;
  const float op = 1.f / (1.f + expf(-prm[10]));
  gp[10] += a.go * op * (1.f - op);
}

// --------------------------------------------------- per-pixel opacity test
// Exponent and opacity of one (pixel, Gaussian) pair, evaluated identically in
// every splat kernel so that skip decisions agree between render, J p, J^T u
// and the diagonal. Returns the alpha before capping in *raw.
// The exponent is -1/2 (q1^2 + q2^2) with q1 = f11 dx + f12 dy, q2 = f22 dy
// (the conic's Cholesky factor, see proj_geom); q1, q2 are kept for the
// derivatives: ds/du = -q1 f11, ds/dv = -(q1 f12 + q2 f22),
// ds/df11 = -q1 dx, ds/df12 = -q1 dy, ds/df22 = -q2 dy.
struct Alpha {
  float dx, dy, q1, q2, es, a;
  bool inc, capped;
};

__device__ __forceinline__ Alpha pair_alpha(float u, float v, float f11, float f12, float f22, float o,
                                            float xc, float yc, const lmrs_render_opts& op) {
#pragma clang fp contract(off)
  Alpha r;
  r.dx = u - xc;
  r.dy = v - yc;
  r.q1 = f11 * r.dx + f12 * r.dy;
  r.q2 = f22 * r.dy;
  const float s = -0.5f * (r.q1 * r.q1 + r.q2 * r.q2);
  r.es = __expf(s);
  const float raw = o * r.es;
  r.capped = raw > op.alpha_max;
  r.a = r.capped ? op.alpha_max : raw;
  r.inc = (s <= 0.f) && (r.a >= op.alpha_min);
  if (!r.inc) r.a = 0.f;
  return r;
}

// ---------------------------------------------------- wave64 collectives
// Scans across the 64 lanes of a wave from DPP: row shifts by 1, 2, 4, 8
// within each row of 16 lanes (these fold into v_add_f32_dpp), then the
// row-15 and row-31 broadcasts carry the row totals to the later rows. They
// must be called with all 64 lanes active.
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

namespace dpp {
constexpr int kRowShr = 0x110;     // row_shr:n = kRowShr + n
constexpr int kRowBcast15 = 0x142; // lane 15 of each row to the next row
constexpr int kRowBcast31 = 0x143; // lane 31 to rows 2 and 3
constexpr int kWaveShr1 = 0x138;   // lane l - 1 to lane l across the whole wave
}  // namespace dpp

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_mov(float old, float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, ROW_MASK,
                                                    0xf, false));
}
__device__ __forceinline__ float readlane(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ int readlane(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }
// reg with lane `lane` replaced by the wave-uniform `value`
__device__ __forceinline__ float writelane(float reg, float value, int lane) {
  return lane_id() == lane ? value : reg;
}
__device__ __forceinline__ int writelane(int reg, int value, int lane) { return lane_id() == lane ? value : reg; }
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uniform(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Inclusive prefix sum over lanes 0..lane.
__device__ __forceinline__ float scan_add(float x) {
  x += dpp_mov<dpp::kRowShr + 1>(0.f, x);
  x += dpp_mov<dpp::kRowShr + 2>(0.f, x);
  x += dpp_mov<dpp::kRowShr + 4>(0.f, x);
  x += dpp_mov<dpp::kRowShr + 8>(0.f, x);
  x += dpp_mov<dpp::kRowBcast15, 0xa>(0.f, x);
  x += dpp_mov<dpp::kRowBcast31, 0xc>(0.f, x);
  return x;
}

// Inclusive product scan over the same DPP steps. Each step is one
// v_mul_f32_dpp with bound_ctrl off, so a lane without a source (and a row
// outside the mask) keeps its value, i.e. multiplies by 1; the compiler folds
// no multiply into DPP, hence the assembly. Every DPP read of a VGPR written
// by the VALU instruction before it needs two wait states (s_nop 1), also the
// first one and whatever reads the result after the block.
__device__ __forceinline__ float scan_mul(float x) {
  asm("s_nop 1\n\t"
      "v_mul_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "s_nop 1\n\t"
      "v_mul_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
      "s_nop 1\n\t"
      "v_mul_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
      "s_nop 1\n\t"
      "v_mul_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
      "s_nop 1\n\t"
      "v_mul_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
      "s_nop 1\n\t"
      "v_mul_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
      "s_nop 1"
      : "+v"(x));
  return x;
}

// Sum over all 64 lanes (wave-uniform).
__device__ __forceinline__ float wave_total(float x) { return readlane(scan_add(x), kWave - 1); }

__device__ __forceinline__ int wave_max_i(int x) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x = max(x, __shfl_xor(x, d, kWave));
  return x;
}
__device__ __forceinline__ float wave_max_f(float x) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x = fmaxf(x, __shfl_xor(x, d, kWave));
  return x;
}

// Sum of x over a workgroup of 256 threads in a fixed order (deterministic);
// s_red: 256 doubles of LDS. Every thread of the workgroup must call it.
__device__ __forceinline__ double block_sum(double x, double* s_red) {
  s_red[threadIdx.x] = x;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) s_red[threadIdx.x] += s_red[threadIdx.x + d];
    __syncthreads();
  }
  const double r = s_red[0];
  __syncthreads();
  return r;
}

// Upper-triangle index of (i, j), i <= j < 5, in a 5x5 symmetric block.
__host__ __device__ constexpr int sym5(int i, int j) { return i * 5 - i * (i - 1) / 2 + (j - i); }

}  // namespace lmrs
