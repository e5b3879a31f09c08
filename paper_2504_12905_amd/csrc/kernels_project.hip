// Per-(view, Gaussian) kernels: projection (Sec. 3, eq. 1-3), its forward
// tangent (dual numbers, Supp. A Alg. 3), and the reverse chain from screen
// records back to parameters for J^T u and for diag(J^T W J).
//
// Launch shape: one lane per Gaussian, 256 lanes per workgroup; beta is read
// component-major so consecutive lanes read consecutive words. Records are
// [V][n][12] floats (three float4) so the splat kernels gather one record
// with three 16-byte loads.
#include "common.hpp"
#include "launch.hpp"

namespace lmrs {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void project_kernel(const float* __restrict__ beta, int n, int deg,
                                                         const lmrs_camera* __restrict__ cams,
                                                         const int32_t* __restrict__ view_ids, int TX,
                                                         int TY, lmrs_render_opts o,
                                                         float* __restrict__ rec, int4* __restrict__ rect) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  const int v = blockIdx.y;
  if (g >= n) return;
  const CamView cv = load_cam(cams, view_ids, v);
  const size_t vg = (size_t)v * n + g;
  float4* out = reinterpret_cast<float4*>(rec + vg * LMRS_REC);
  float tc[3], u, vv;
  decision_point(cv.c, beta[g], beta[(size_t)n + g], beta[(size_t)2 * n + g], tc, &u, &vv);
  int4 rc = make_int4(0, 0, 0, 0);
  float r[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float radius = 0.f;
  if (tc[2] > o.znear && isfinite(u) && isfinite(vv)) {
    float prm[kMaxPg];
    const int pg = 11 + 3 * (deg + 1) * (deg + 1);
    load_params(beta, n, g, pg, prm);
    float a, b, c;
    proj_core(prm, deg, cv, o.lowpass, r, &a, &b, &c);
    r[0] = u;
    r[1] = vv;
    const float lam = 0.5f * (a + c) + sqrtf(0.25f * (a - c) * (a - c) + b * b);
    const float rad = ceilf(o.cutoff * sqrtf(lam));
    if (rad < 1.0e6f) {
      auto tile_of = [](float q) {
        const float f = floorf(q / 16.f);
        return (int)fminf(fmaxf(f, -1.0e6f), 1.0e6f);
      };
      int x0 = max(tile_of(u - rad), 0), x1 = min(tile_of(u + rad), TX - 1);
      int y0 = max(tile_of(vv - rad), 0), y1 = min(tile_of(vv + rad), TY - 1);
      if (x0 <= x1 && y0 <= y1) {
        rc = make_int4(x0, y0, x1 + 1, y1 + 1);
        radius = rad;
      }
    }
  }
  out[0] = make_float4(r[0], r[1], r[2], r[3]);
  out[1] = make_float4(r[4], r[5], r[6], r[7]);
  out[2] = make_float4(r[8], tc[2], radius, 0.f);
  rect[vg] = rc;
}

// Tangent of the screen record along direction p (forward mode).
__global__ __launch_bounds__(kBlock) void tangent_kernel(const float* __restrict__ beta,
                                                         const float* __restrict__ p, int n, int deg,
                                                         const lmrs_camera* __restrict__ cams,
                                                         const int32_t* __restrict__ view_ids,
                                                         const int4* __restrict__ rect, float lowpass,
                                                         float* __restrict__ tan) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  const int v = blockIdx.y;
  if (g >= n) return;
  const size_t vg = (size_t)v * n + g;
  float4* out = reinterpret_cast<float4*>(tan + vg * LMRS_REC);
  const int4 rc = rect[vg];
  if (rc.x >= rc.z) {
    out[0] = out[1] = out[2] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const CamView cv = load_cam(cams, view_ids, v);
  const int pg = 11 + 3 * (deg + 1) * (deg + 1);
  dualf prm[kMaxPg];
  for (int j = 0; j < pg; ++j) prm[j] = dualf(beta[(size_t)j * n + g], p[(size_t)j * n + g]);
  dualf r[9];
  proj_core(prm, deg, cv, lowpass, r, nullptr, nullptr, nullptr);
  out[0] = make_float4(r[0].d, r[1].d, r[2].d, r[3].d);
  out[1] = make_float4(r[4].d, r[5].d, r[6].d, r[7].d);
  out[2] = make_float4(r[8].d, 0.f, 0.f, 0.f);
}

// out[beta_g] = sum_v (d rec_vg / d beta_g)^T grad2d[v][:][g]  (+ lambda d p)
__global__ __launch_bounds__(kBlock) void chain_vjp_kernel(
    const float* __restrict__ beta, int n, int deg, int V, const lmrs_camera* __restrict__ cams,
    const int32_t* __restrict__ view_ids, float lowpass, const float* __restrict__ grad2d,
    const float* __restrict__ p, float lambda, const float* __restrict__ dvec, float* __restrict__ out) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= n) return;
  const int pg = 11 + 3 * (deg + 1) * (deg + 1);
  float prm[kMaxPg], gp[kMaxPg];
  load_params(beta, n, g, pg, prm);
  for (int j = 0; j < pg; ++j) gp[j] = 0.f;
  for (int v = 0; v < V; ++v) {
    float gr[9];
    bool any = false;
    for (int q = 0; q < 9; ++q) {
      gr[q] = grad2d[((size_t)v * 9 + q) * n + g];
      any |= gr[q] != 0.f;
    }
    if (!any) continue;
    const CamView cv = load_cam(cams, view_ids, v);
    proj_vjp(prm, deg, cv, lowpass, gr, gp);
  }
  for (int j = 0; j < pg; ++j) {
    const size_t idx = (size_t)j * n + g;
    float val = gp[j];
    if (p) val += lambda * (dvec ? dvec[idx] : 1.f) * p[idx];
    out[idx] = val;
  }
}

// diag(J^T W J) from the per-(view, Gaussian) Gram blocks of the screen-record
// derivatives: D_j = col_j^T G col_j, col_j = d rec / d beta_j. Gram layout per
// (view, Gaussian): [0,15) geometry (u v A B C) upper triangle, [15,30)
// geometry x colour channel (3 k + c), 30 colour (same for all channels),
// 31 opacity.
__global__ __launch_bounds__(kBlock) void chain_diag_kernel(
    const float* __restrict__ beta, int n, int deg, int V, const lmrs_camera* __restrict__ cams,
    const int32_t* __restrict__ view_ids, float lowpass, const float* __restrict__ gram,
    float* __restrict__ out) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= n) return;
  const int K2 = (deg + 1) * (deg + 1);
  const int pg = 11 + 3 * K2;
  float prm[kMaxPg], D[kMaxPg];
  load_params(beta, n, g, pg, prm);
  for (int j = 0; j < pg; ++j) D[j] = 0.f;
  const float op = 1.f / (1.f + expf(-prm[10]));
  const float dop = op * (1.f - op);
  for (int v = 0; v < V; ++v) {
    float G[kGram];
    bool any = false;
    for (int e = 0; e < kGram; ++e) {
      G[e] = gram[((size_t)v * kGram + e) * n + g];
      any |= G[e] != 0.f;
    }
    if (!any) continue;
    const CamView cv = load_cam(cams, view_ids, v);
    // geometric parameters: mean (3), log-scale (3), quaternion (4)
    for (int j = 0; j < 10; ++j) {
      dualf dp[kMaxPg];
      for (int i = 0; i < pg; ++i) dp[i] = dualf(prm[i], i == j ? 1.f : 0.f);
      dualf r[9];
      proj_core(dp, deg, cv, lowpass, r, nullptr, nullptr, nullptr);
      float col[9];
      for (int q = 0; q < 9; ++q) col[q] = r[q].d;
      float acc = 0.f;
      for (int a = 0; a < 5; ++a) {
        acc += G[sym5(a, a)] * col[a] * col[a];
        for (int b = a + 1; b < 5; ++b) acc += 2.f * G[sym5(a, b)] * col[a] * col[b];
        for (int c = 0; c < 3; ++c) acc += 2.f * G[15 + 3 * a + c] * col[a] * col[6 + c];
      }
      for (int c = 0; c < 3; ++c) acc += G[30] * col[6 + c] * col[6 + c];
      D[j] += acc;
    }
    D[10] += dop * dop * G[31];
    // colour coefficients: d rgb_c / d f_kc = Y_k(dir)
    float dx = prm[0] - cv.pos[0], dy = prm[1] - cv.pos[1], dz = prm[2] - cv.pos[2];
    const float dinv = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
    float Y[16];
    sh_eval(deg, dx * dinv, dy * dinv, dz * dinv, Y);
    for (int k = 0; k < K2; ++k)
      for (int c = 0; c < 3; ++c) D[11 + 3 * k + c] += Y[k] * Y[k] * G[30];
  }
  for (int j = 0; j < pg; ++j) out[(size_t)j * n + g] = D[j];
}

__global__ void fill_kernel(float* __restrict__ x, int64_t count, float value) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) x[i] = value;
}

}  // namespace

void launch_project(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, hipStream_t s) {
  dim3 grid((d.n + kBlock - 1) / kBlock, d.V);
  project_kernel<<<grid, kBlock, 0, s>>>(f->beta, d.n, d.deg, f->cams, f->view_ids, d.TX, d.TY, o,
                                         f->rec, reinterpret_cast<int4*>(f->rect));
}

void launch_tangent(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, const float* p,
                    float* tan, hipStream_t s) {
  dim3 grid((d.n + kBlock - 1) / kBlock, d.V);
  tangent_kernel<<<grid, kBlock, 0, s>>>(f->beta, p, d.n, d.deg, f->cams, f->view_ids,
                                         reinterpret_cast<const int4*>(f->rect), o.lowpass, tan);
}

void launch_chain_vjp(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                      const float* grad2d, const float* p, float lambda, const float* dvec, float* out,
                      hipStream_t s) {
  chain_vjp_kernel<<<(d.n + kBlock - 1) / kBlock, kBlock, 0, s>>>(
      f->beta, d.n, d.deg, d.V, f->cams, f->view_ids, o.lowpass, grad2d, p, lambda, dvec, out);
}

void launch_chain_diag(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                       const float* gram, float* out, hipStream_t s) {
  chain_diag_kernel<<<(d.n + kBlock - 1) / kBlock, kBlock, 0, s>>>(f->beta, d.n, d.deg, d.V, f->cams,
                                                                    f->view_ids, o.lowpass, gram, out);
}

void launch_fill(float* x, int64_t count, float value, hipStream_t s) {
  if (count <= 0) return;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  fill_kernel<<<(unsigned)blocks, 256, 0, s>>>(x, count, value);
}

}  // namespace lmrs
