// Per-(view, Gaussian) kernels: projection (Sec. 3, eq. 1-3), its forward
// tangent (dual numbers, Supp. A Alg. 3), and the reverse chain from screen
// records back to parameters for J^T u and for diag(J^T W J).
//
// Launch shape: one lane per Gaussian, 256 lanes per workgroup; beta is read
// component-major so consecutive lanes read consecutive words. Records are
// [V][n][12] floats (three float4) so the splat kernels gather one record
// with three 16-byte loads.
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"

namespace lmrs {

namespace {

constexpr int kBlock = 256;

template <int DEG>
__global__ __launch_bounds__(kBlock) void project_kernel(const float* __restrict__ beta, int n,
                                                         const lmrs_camera* __restrict__ cams,
                                                         const int32_t* __restrict__ view_ids, int TX,
                                                         int TY, lmrs_render_opts o,
                                                         float* __restrict__ rec, int4* __restrict__ rect) {
  constexpr int PG = ShDims<DEG>::PG;
  const int g = blockIdx.x * kBlock + threadIdx.x;
  const int v = blockIdx.y;
  if (g >= n) return;
  const CamView cv = load_cam(cams, view_ids, v);
  const size_t vg = (size_t)v * n + g;
  float4* out = reinterpret_cast<float4*>(rec + vg * LMRS_REC);
  // the list decisions (near-plane cull, footprint radius, tile rectangle,
  // depth order) from FP64 values
  double tc[3], u, vv;
  decision_point(cv.c, (double)beta[g], (double)beta[(size_t)n + g], (double)beta[(size_t)2 * n + g], tc, &u,
                 &vv);
  float zlo, zhi;
  depth_words(tc[2], &zlo, &zhi);
  int4 rc = make_int4(0, 0, 0, 0);
  float r[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float radius = 0.f;
  if (tc[2] > (double)o.znear && isfinite(u) && isfinite(vv)) {
    float prm[PG];
    load_params<PG>(beta, n, g, prm);
    proj_core<DEG>(prm, cv, o.lowpass, r, nullptr, nullptr, nullptr);
    // the record's geometry (centre, conic factor) rounded from FP64, and the
    // 2-D covariance whose largest eigenvalue sets the radius
    double pd[10], gd[5], a, b, c;
#pragma unroll
    for (int j = 0; j < 10; ++j) pd[j] = (double)prm[j];
    proj_geom(pd, cv, o.lowpass, gd, &a, &b, &c);
    r[0] = (float)u;
    r[1] = (float)vv;
    r[2] = (float)gd[2];
    r[3] = (float)gd[3];
    r[4] = (float)gd[4];
    const double lam = 0.5 * (a + c) + sqrt(0.25 * (a - c) * (a - c) + b * b);
    const double rad = ceil((double)o.cutoff * sqrt(lam));
    if (rad < 1.0e6) {
      auto tile_of = [](double q) { return (int)fmin(fmax(floor(q / 16.0), -1.0e6), 1.0e6); };
      int x0 = max(tile_of(u - rad), 0), x1 = min(tile_of(u + rad), TX - 1);
      int y0 = max(tile_of(vv - rad), 0), y1 = min(tile_of(vv + rad), TY - 1);
      if (x0 <= x1 && y0 <= y1) {
        rc = make_int4(x0, y0, x1 + 1, y1 + 1);
        radius = (float)rad;
      }
    }
  }
  out[0] = make_float4(r[0], r[1], r[2], r[3]);
  out[1] = make_float4(r[4], r[5], r[6], r[7]);
  out[2] = make_float4(r[8], zlo, radius, zhi);
  rect[vg] = rc;
}

// Tangent of the screen record along direction p (forward mode). One thread
// per Gaussian loads its parameters and direction once and forms the tangent
// in every view of the batch.
template <int DEG>
__global__ __launch_bounds__(kBlock) void tangent_kernel(const float* __restrict__ beta,
                                                         const float* __restrict__ p, int n, int V,
                                                         const lmrs_camera* __restrict__ cams,
                                                         const int32_t* __restrict__ view_ids,
                                                         const int4* __restrict__ rect, float lowpass,
                                                         float* __restrict__ tan) {
  constexpr int PG = ShDims<DEG>::PG;
  const int g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= n) return;
  dualf prm[PG];
#pragma unroll
  for (int j = 0; j < PG; ++j) prm[j] = dualf(beta[(size_t)j * n + g], p[(size_t)j * n + g]);
  // the view-independent parts: covariance factor and opacity
  dualf M[9];
  cov_factor(prm, M);
  const dualf op = dualf(1.f) / (dualf(1.f) + texp(-prm[10]));
  // the next view's rectangle is loaded while this view's tangent is formed
  int4 rc_next = V > 0 ? rect[g] : make_int4(0, 0, 0, 0);
  for (int v = 0; v < V; ++v) {
    const size_t vg = (size_t)v * n + g;
    float4* out = reinterpret_cast<float4*>(tan + vg * LMRS_REC);
    const int4 rc = rc_next;
    if (v + 1 < V) rc_next = rect[vg + n];
    if (rc.x >= rc.z) {
      out[0] = out[1] = out[2] = make_float4(0.f, 0.f, 0.f, 0.f);
      continue;
    }
    const CamView cv = load_cam(cams, view_ids, v);
    dualf r[9];
    proj_geom_m(prm, M, cv, lowpass, r, nullptr, nullptr, nullptr);
    r[5] = op;
    proj_color<DEG>(prm, cv, r + 6);
    out[0] = make_float4(r[0].d, r[1].d, r[2].d, r[3].d);
    out[1] = make_float4(r[4].d, r[5].d, r[6].d, r[7].d);
    out[2] = make_float4(r[8].d, 0.f, 0.f, 0.f);
  }
}

// A fixed-point row of NC components (hi words from word 0, lo words from
// word LO, poison word P; see fix_add) read into floats; false when the row
// is all zero (nothing accumulated), NaN components when it is poisoned.
// With clear the row is zeroed after the read. Rows are 16-byte aligned and
// their words past the components up to an even count are zero.
template <int NC, int LO, int P>
__device__ __forceinline__ bool fix_row(unsigned long long* row, float* out, bool clear) {
  constexpr int kPairs = (NC + 1) / 2;
  const ulonglong2* hp = reinterpret_cast<const ulonglong2*>(row);
  const ulonglong2* lp = reinterpret_cast<const ulonglong2*>(row + LO);
  unsigned long long hi[2 * kPairs], lo[2 * kPairs];
#pragma unroll
  for (int i = 0; i < kPairs; ++i) {
    const ulonglong2 h = hp[i], l = lp[i];
    hi[2 * i] = h.x;
    hi[2 * i + 1] = h.y;
    lo[2 * i] = l.x;
    lo[2 * i + 1] = l.y;
  }
  const unsigned long long poison = row[P];
  unsigned long long any = poison;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    any |= hi[q] | lo[q];
    out[q] = poison ? NAN : fix_value(hi[q], lo[q]);
  }
  if (!any) return false;
  if (clear) {
    ulonglong2* hw = reinterpret_cast<ulonglong2*>(row);
    ulonglong2* lw = reinterpret_cast<ulonglong2*>(row + LO);
#pragma unroll
    for (int i = 0; i < kPairs; ++i) hw[i] = lw[i] = make_ulonglong2(0ull, 0ull);
    row[P] = 0ull;
  }
  return true;
}

// out[beta_g] = sum_v (d rec_vg / d beta_g)^T grad2d[v][g][0..9)  (+ lambda d p).
// With pu_part, each workgroup also leaves its partial sum of p . out in
// pu_part[blockIdx.x] (FP64; the PCG update reduces them), which saves the
// operator product's separate pass over p and u. With zero_rows it clears
// the non-zero rows it has read, so that grad2d is all zero again for the
// next accumulation (instead of a fill of the whole buffer). With fixed the
// rows are the fixed-point rows of deterministic accumulation.
template <int DEG>
__global__ __launch_bounds__(kBlock) void chain_vjp_kernel(
    const float* __restrict__ beta, int n, int V, const lmrs_camera* __restrict__ cams,
    const int32_t* __restrict__ view_ids, float lowpass, float* __restrict__ grad2d, bool fixed,
    const float* __restrict__ p, float lambda, const float* __restrict__ dvec, float* __restrict__ out,
    double* __restrict__ pu_part, bool zero_rows) {
  constexpr int PG = ShDims<DEG>::PG;
  double pu = 0.0;
  for (int g = blockIdx.x * kBlock + threadIdx.x; g < n; g += gridDim.x * kBlock) {
    float prm[PG], gp[PG];
    load_params<PG>(beta, n, g, prm);
#pragma unroll
    for (int j = 0; j < PG; ++j) gp[j] = 0.f;
    const GeoFactors gf = geo_factors(prm);
    GeoGrad acc;
    geo_grad_zero(acc);
    if (fixed) {
      unsigned long long* rows = reinterpret_cast<unsigned long long*>(grad2d);
      for (int v = 0; v < V; ++v) {
        float gr[9];
        if (!fix_row<9, kFixGradLo, kFixGradPoison>(rows + ((size_t)v * n + g) * kFixGradRow, gr, zero_rows))
          continue;
        const CamView cv = load_cam(cams, view_ids, v);
        proj_vjp_view<DEG>(prm, gf, cv, lowpass, gr, gp, acc);
      }
    }
    const int Vf = fixed ? 0 : V;  // views of float rows
    // the next view's row is loaded while this view's row is taken back
    float4 a_next{}, b_next{};
    float c_next = 0.f;
    if (Vf > 0) {
      const float* row0 = grad2d + (size_t)g * kGradRow;
      a_next = reinterpret_cast<const float4*>(row0)[0];
      b_next = reinterpret_cast<const float4*>(row0)[1];
      c_next = row0[8];
    }
    for (int v = 0; v < Vf; ++v) {
      float gr[9];
      bool any = false;
      float* row = grad2d + ((size_t)v * n + g) * kGradRow;
      const float4 a = a_next, b = b_next;
      gr[0] = a.x; gr[1] = a.y; gr[2] = a.z; gr[3] = a.w;
      gr[4] = b.x; gr[5] = b.y; gr[6] = b.z; gr[7] = b.w;
      gr[8] = c_next;
      if (v + 1 < Vf) {
        const float* nrow = row + (size_t)n * kGradRow;
        a_next = reinterpret_cast<const float4*>(nrow)[0];
        b_next = reinterpret_cast<const float4*>(nrow)[1];
        c_next = nrow[8];
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) any |= gr[q] != 0.f;
      if (!any) continue;
      if (zero_rows) {
        reinterpret_cast<float4*>(row)[0] = reinterpret_cast<float4*>(row)[1] = make_float4(0.f, 0.f, 0.f, 0.f);
        row[8] = 0.f;
      }
      const CamView cv = load_cam(cams, view_ids, v);
      proj_vjp_view<DEG>(prm, gf, cv, lowpass, gr, gp, acc);
    }
    proj_vjp_finish(prm, gf, acc, gp);
#pragma unroll
    for (int j = 0; j < PG; ++j) {
      const size_t idx = (size_t)j * n + g;
      float val = gp[j];
      if (p) {
        const float pj = p[idx];
        val += lambda * (dvec ? dvec[idx] : 1.f) * pj;
        pu += (double)pj * (double)val;
      }
      out[idx] = val;
    }
  }
  if (pu_part) {
    __shared__ double s_red[kBlock];
    const double r = block_sum(pu, s_red);
    if (threadIdx.x == 0) pu_part[blockIdx.x] = r;
  }
}

// diag(J^T W J) from the per-(view, Gaussian) Gram blocks of the screen-record
// derivatives: D_j = col_j^T G col_j, col_j = d rec / d beta_j. Gram layout per
// (view, Gaussian): [0,15) geometry (u v A B C) upper triangle, [15,30)
// geometry x colour channel (3 k + c), 30 colour (same for all channels),
// 31 opacity. Geometric columns (mean, log-scale, quaternion) come from one
// dual pass each of the geometric projection; the mean's colour rows from
// the SH basis derivative; opacity and SH columns have closed forms.
template <int DEG>
__global__ __launch_bounds__(kBlock) void chain_diag_kernel(
    const float* __restrict__ beta, int n, int V, const lmrs_camera* __restrict__ cams,
    const int32_t* __restrict__ view_ids, float lowpass, const float* __restrict__ gram, bool fixed,
    float* __restrict__ out) {
  constexpr int K2 = ShDims<DEG>::K;
  constexpr int PG = ShDims<DEG>::PG;
  const int g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= n) return;
  float prm[PG], D[PG];
  load_params<PG>(beta, n, g, prm);
#pragma unroll
  for (int j = 0; j < PG; ++j) D[j] = 0.f;
  const float op = 1.f / (1.f + expf(-prm[10]));
  const float dop = op * (1.f - op);
  for (int v = 0; v < V; ++v) {
    float G[kGram];
    bool any = false;
    if (fixed) {
      // const_cast: fix_row clears nothing here
      any = fix_row<kGram, kFixGramLo, kFixGramPoison>(
          const_cast<unsigned long long*>(reinterpret_cast<const unsigned long long*>(gram)) +
              ((size_t)v * n + g) * kFixGramRow,
          G, false);
    } else {
      const float4* row = reinterpret_cast<const float4*>(gram + ((size_t)v * n + g) * kGram);
#pragma unroll
      for (int e4 = 0; e4 < kGram / 4; ++e4) {
        const float4 x = row[e4];
        G[4 * e4] = x.x;
        G[4 * e4 + 1] = x.y;
        G[4 * e4 + 2] = x.z;
        G[4 * e4 + 3] = x.w;
      }
#pragma unroll
      for (int e = 0; e < kGram; ++e) any |= G[e] != 0.f;
    }
    if (!any) continue;
    const CamView cv = load_cam(cams, view_ids, v);
    float Jc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if constexpr (DEG > 0) color_mean_jacobian<DEG>(prm, cv, Jc);
#pragma unroll
    for (int j = 0; j < 10; ++j) {
      dualf dp[10];
#pragma unroll
      for (int i = 0; i < 10; ++i) dp[i] = dualf(prm[i], i == j ? 1.f : 0.f);
      dualf r[5];
      proj_geom(dp, cv, lowpass, r, nullptr, nullptr, nullptr);
      float col[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) col[q] = r[q].d;
      float crgb[3] = {0.f, 0.f, 0.f};
      if (j < 3) {
        crgb[0] = Jc[j];
        crgb[1] = Jc[3 + j];
        crgb[2] = Jc[6 + j];
      }
      float acc = 0.f;
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        acc += G[sym5(a, a)] * col[a] * col[a];
#pragma unroll
        for (int b = a + 1; b < 5; ++b) acc += 2.f * G[sym5(a, b)] * col[a] * col[b];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc += 2.f * G[15 + 3 * a + c] * col[a] * crgb[c];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) acc += G[30] * crgb[c] * crgb[c];
      D[j] += acc;
    }
    D[10] += dop * dop * G[31];
    float d[3];
    view_dir(prm, cv, d);
    float Y[K2];
    sh_eval<DEG>(d[0], d[1], d[2], Y);
#pragma unroll
    for (int k = 0; k < K2; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) D[11 + 3 * k + c] += Y[k] * Y[k] * G[30];
  }
#pragma unroll
  for (int j = 0; j < PG; ++j) out[(size_t)j * n + g] = D[j];
}

__global__ void fill_kernel(float* __restrict__ x, int64_t count, float value) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) x[i] = value;
}

}  // namespace

void launch_project(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, hipStream_t s) {
  dim3 grid((d.n + kBlock - 1) / kBlock, d.V);
  auto* rect = reinterpret_cast<int4*>(f->rect);
  switch (d.deg) {
    case 0: project_kernel<0><<<grid, kBlock, 0, s>>>(f->beta, d.n, f->cams, f->view_ids, d.TX, d.TY, o, f->rec, rect); break;
    case 1: project_kernel<1><<<grid, kBlock, 0, s>>>(f->beta, d.n, f->cams, f->view_ids, d.TX, d.TY, o, f->rec, rect); break;
    case 2: project_kernel<2><<<grid, kBlock, 0, s>>>(f->beta, d.n, f->cams, f->view_ids, d.TX, d.TY, o, f->rec, rect); break;
    default: project_kernel<3><<<grid, kBlock, 0, s>>>(f->beta, d.n, f->cams, f->view_ids, d.TX, d.TY, o, f->rec, rect); break;
  }
}

void launch_tangent(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, const float* p,
                    float* tan, hipStream_t s) {
  const unsigned grid = (d.n + kBlock - 1) / kBlock;
  auto* rect = reinterpret_cast<const int4*>(f->rect);
  switch (d.deg) {
    case 0: tangent_kernel<0><<<grid, kBlock, 0, s>>>(f->beta, p, d.n, d.V, f->cams, f->view_ids, rect, o.lowpass, tan); break;
    case 1: tangent_kernel<1><<<grid, kBlock, 0, s>>>(f->beta, p, d.n, d.V, f->cams, f->view_ids, rect, o.lowpass, tan); break;
    case 2: tangent_kernel<2><<<grid, kBlock, 0, s>>>(f->beta, p, d.n, d.V, f->cams, f->view_ids, rect, o.lowpass, tan); break;
    default: tangent_kernel<3><<<grid, kBlock, 0, s>>>(f->beta, p, d.n, d.V, f->cams, f->view_ids, rect, o.lowpass, tan); break;
  }
}

int chain_vjp_blocks(int n, bool partials) {
  const int blocks = (n + kBlock - 1) / kBlock;
  return partials ? std::min(blocks, kRedBlocks) : blocks;
}

void launch_chain_vjp(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                      float* grad2d, const float* p, float lambda, const float* dvec, float* out,
                      hipStream_t s, double* pu_part, bool zero_rows) {
  const unsigned grid = (unsigned)chain_vjp_blocks(d.n, pu_part != nullptr);
  switch (d.deg) {
    case 0: chain_vjp_kernel<0><<<grid, kBlock, 0, s>>>(f->beta, d.n, d.V, f->cams, f->view_ids, o.lowpass, grad2d, d.det, p, lambda, dvec, out, pu_part, zero_rows); break;
    case 1: chain_vjp_kernel<1><<<grid, kBlock, 0, s>>>(f->beta, d.n, d.V, f->cams, f->view_ids, o.lowpass, grad2d, d.det, p, lambda, dvec, out, pu_part, zero_rows); break;
    case 2: chain_vjp_kernel<2><<<grid, kBlock, 0, s>>>(f->beta, d.n, d.V, f->cams, f->view_ids, o.lowpass, grad2d, d.det, p, lambda, dvec, out, pu_part, zero_rows); break;
    default: chain_vjp_kernel<3><<<grid, kBlock, 0, s>>>(f->beta, d.n, d.V, f->cams, f->view_ids, o.lowpass, grad2d, d.det, p, lambda, dvec, out, pu_part, zero_rows); break;
  }
}

void launch_chain_diag(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                       const float* gram, float* out, hipStream_t s) {
  const unsigned grid = (d.n + kBlock - 1) / kBlock;
  switch (d.deg) {
    case 0: chain_diag_kernel<0><<<grid, kBlock, 0, s>>>(f->beta, d.n, d.V, f->cams, f->view_ids, o.lowpass, gram, d.det, out); break;
    case 1: chain_diag_kernel<1><<<grid, kBlock, 0, s>>>(f->beta, d.n, d.V, f->cams, f->view_ids, o.lowpass, gram, d.det, out); break;
    case 2: chain_diag_kernel<2><<<grid, kBlock, 0, s>>>(f->beta, d.n, d.V, f->cams, f->view_ids, o.lowpass, gram, d.det, out); break;
    default: chain_diag_kernel<3><<<grid, kBlock, 0, s>>>(f->beta, d.n, d.V, f->cams, f->view_ids, o.lowpass, gram, d.det, out); break;
  }
}

void launch_fill(float* x, int64_t count, float value, hipStream_t s) {
  if (count <= 0) return;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  fill_kernel<<<(unsigned)blocks, 256, 0, s>>>(x, count, value);
}

}  // namespace lmrs
