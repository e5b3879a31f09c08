// Per-tile splat kernels: forward render (Sec. 3 eq. 3; Supp. A Alg. 2),
// J p (forward mode, Alg. 3), J^T u (reverse accumulation, Supp. A "J^T v
// kernel"), their fused composition J^T W J p (the operator product of the
// PCG loop in Alg. 1), and the weighted Gram blocks behind diag(J^T W J).
//
// Work layout (one 64-lane wave per (view, tile)). The paper launches one
// thread per sampled pixel; with ~10 % of a 16x16 tile sampled that leaves
// most of a wave64 idle and forces cross-lane reductions of every Gaussian's
// gradient. Here the lanes own list entries instead: a chunk of 64 entries
// of the tile's depth-sorted list is loaded, one record per lane, and the
// wave walks the tile's sampled pixels one after another. For each pixel
// the transmittance in front of every entry is an exclusive prefix product
// of (1 - alpha) across the lanes, carried from chunk to chunk; J p needs one
// more prefix sum for its derivative; J^T u walks the chunks back to front
// and needs a suffix sum for the colour blended behind each entry. Each lane
// then holds its Gaussian's screen-space gradient summed over all pixels of
// the tile and issues one atomic add per component: no per-Gaussian
// cross-lane reduction. A pixel's loop stops at its last blended entry
// (`last` from the render), so work follows the actual blend depth per pixel.
//
// Discrete decisions (list, opacity skip, cap, stop position) come from the
// render and are recomputed bit-identically by pair_alpha().
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

__device__ __forceinline__ TileCtx tile_ctx(const int64_t* tile_start, int T, int TX) {
  TileCtx c;
  c.tile_lin = blockIdx.x;
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

struct RecF {
  float u, v, A, B, C, o, r, g, b;
};

__device__ __forceinline__ RecF load_rec(const float* rec, size_t vg) {
  const float4* p = reinterpret_cast<const float4*>(rec + vg * LMRS_REC);
  const float4 a = p[0], b = p[1], c = p[2];
  return RecF{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x};
}

// ------------------------------------------------------------------ render
__global__ __launch_bounds__(kWave) void render_kernel(const float* __restrict__ rec,
                                                       const int64_t* __restrict__ tile_start,
                                                       const int32_t* __restrict__ ids,
                                                       const uint8_t* __restrict__ pix, int n, int T,
                                                       int TX, int k, lmrs_render_opts o,
                                                       float* __restrict__ color, float* __restrict__ trans,
                                                       int32_t* __restrict__ last) {
  __shared__ float s_xc[kMaxK], s_yc[kMaxK], s_T[kMaxK], s_C[3 * kMaxK];
  __shared__ int s_last[kMaxK], s_done[kMaxK];
  const int lane = lane_id();
  const TileCtx c = tile_ctx(tile_start, T, TX);
  for (int j = lane; j < k; j += kWave) {
    pixel_center(pix, k, c, j, &s_xc[j], &s_yc[j]);
    s_T[j] = 1.f;
    s_C[3 * j] = s_C[3 * j + 1] = s_C[3 * j + 2] = 0.f;
    s_last[j] = -1;
    s_done[j] = 0;
  }
  __syncthreads();
  int remaining = k;
  for (int64_t c0 = 0; c0 < c.len && remaining > 0; c0 += kWave) {
    const bool valid = c0 + lane < c.len;
    RecF r{};
    if (valid) r = load_rec(rec, (size_t)c.v * n + ids[c.start + c0 + lane]);
    for (int j = 0; j < k; ++j) {
      if (s_done[j]) continue;
      const Alpha al = pair_alpha(r.u, r.v, r.A, r.B, r.C, r.o, s_xc[j], s_yc[j], o);
      const bool inc = valid && al.inc;
      const float a = inc ? al.a : 0.f;
      const float ip = incl_prod(1.f - a, lane);
      float ep = __shfl_up(ip, 1, kWave);
      if (lane == 0) ep = 1.f;
      const float Tc = s_T[j];
      const uint64_t stop = __ballot(inc && Tc * ip < o.t_min);
      const int f = stop ? __ffsll((unsigned long long)stop) - 1 : kWave;
      const bool ok = inc && lane < f;
      const float wgt = ok ? a * Tc * ep : 0.f;
      const float cr = wave_sum(wgt * r.r), cg = wave_sum(wgt * r.g), cb = wave_sum(wgt * r.b);
      const uint64_t okm = __ballot(ok);
      const float Tnext = f < kWave ? Tc * bcast(ep, f) : Tc * bcast(ip, kWave - 1);
      if (lane == 0) {
        s_C[3 * j] += cr;
        s_C[3 * j + 1] += cg;
        s_C[3 * j + 2] += cb;
        if (okm) s_last[j] = (int)c0 + 63 - __clzll((long long)okm);
        s_T[j] = Tnext;
        if (f < kWave) s_done[j] = 1;
      }
      if (f < kWave) --remaining;
    }
  }
  __syncthreads();
  for (int j = lane; j < k; j += kWave) {
    const int64_t i = c.tile_lin * k + j;
    const float Tf = s_T[j];
    color[3 * i] = s_C[3 * j] + Tf * o.bg[0];
    color[3 * i + 1] = s_C[3 * j + 1] + Tf * o.bg[1];
    color[3 * i + 2] = s_C[3 * j + 2] + Tf * o.bg[2];
    trans[i] = Tf;
    last[i] = s_last[j];
  }
}

// ----------------------------------------------------- J p, J^T u, fused GN
// MODE 1: jp = J p.  MODE 2: grad2d += J^T u.  MODE 3: grad2d += J^T W J p.
template <int MODE>
__global__ __launch_bounds__(kWave) void deriv_kernel(
    const float* __restrict__ rec, const float* __restrict__ tan, const int64_t* __restrict__ tile_start,
    const int32_t* __restrict__ ids, const uint8_t* __restrict__ pix, const float* __restrict__ wts,
    const float* __restrict__ trans, const int32_t* __restrict__ lastv, int n, int T, int TX, int k,
    lmrs_render_opts o, const float* __restrict__ u_in, float* __restrict__ jp_out,
    float* __restrict__ grad2d) {
  constexpr bool FWD = MODE != 2;
  constexpr bool REV = MODE != 1;
  __shared__ float s_xc[kMaxK], s_yc[kMaxK], s_a[kMaxK], s_b[kMaxK], s_u[3 * kMaxK];
  __shared__ int s_last[kMaxK];
  const int lane = lane_id();
  const TileCtx c = tile_ctx(tile_start, T, TX);
  int lmax = -1;
  for (int j = lane; j < k; j += kWave) {
    const int64_t i = c.tile_lin * k + j;
    pixel_center(pix, k, c, j, &s_xc[j], &s_yc[j]);
    s_last[j] = lastv[i];
    lmax = max(lmax, s_last[j]);
  }
  lmax = wave_max_i(lmax);
  __syncthreads();

  if (FWD) {
    // s_a = T carried in front of the chunk, s_b = its derivative, s_u = d colour
    for (int j = lane; j < k; j += kWave) {
      s_a[j] = 1.f;
      s_b[j] = 0.f;
      s_u[3 * j] = s_u[3 * j + 1] = s_u[3 * j + 2] = 0.f;
    }
    __syncthreads();
    for (int64_t c0 = 0; c0 <= lmax; c0 += kWave) {
      const int64_t e = c0 + lane;
      const bool valid = e < c.len;
      RecF r{}, dr{};
      if (valid) {
        const size_t vg = (size_t)c.v * n + ids[c.start + e];
        r = load_rec(rec, vg);
        dr = load_rec(tan, vg);
      }
      for (int j = 0; j < k; ++j) {
        const int lj = s_last[j];
        if (c0 > lj) continue;
        const Alpha al = pair_alpha(r.u, r.v, r.A, r.B, r.C, r.o, s_xc[j], s_yc[j], o);
        const bool inc = valid && e <= lj && al.inc;
        float a = 0.f, da = 0.f;
        if (inc) {
          a = al.a;
          if (!al.capped) {
            const float ds = -(r.A * al.dx * dr.u + r.C * al.dy * dr.v) -
                             0.5f * (dr.A * al.dx * al.dx + dr.C * al.dy * al.dy) - dr.B * al.dx * al.dy -
                             r.B * (dr.u * al.dy + al.dx * dr.v);
            da = al.es * (dr.o + r.o * ds);
          }
        }
        const float om = 1.f - a;
        const float ip = incl_prod(om, lane);
        float ep = __shfl_up(ip, 1, kWave);
        const float q = inc ? -da / om : 0.f;
        const float iq = incl_sum(q, lane);
        float eq = __shfl_up(iq, 1, kWave);
        if (lane == 0) {
          ep = 1.f;
          eq = 0.f;
        }
        const float Tc = s_a[j], dTc = s_b[j];
        const float Tn = Tc * ep;
        const float dTn = ep * (dTc + Tc * eq);
        float cr = 0.f, cg = 0.f, cb = 0.f;
        if (inc) {
          const float aT = a * Tn, gT = da * Tn + a * dTn;
          cr = dr.r * aT + r.r * gT;
          cg = dr.g * aT + r.g * gT;
          cb = dr.b * aT + r.b * gT;
        }
        cr = wave_sum(cr);
        cg = wave_sum(cg);
        cb = wave_sum(cb);
        const float tp = bcast(ip, kWave - 1), tq = bcast(iq, kWave - 1);
        if (lane == 0) {
          s_u[3 * j] += cr;
          s_u[3 * j + 1] += cg;
          s_u[3 * j + 2] += cb;
          s_b[j] = tp * (dTc + Tc * tq);
          s_a[j] = Tc * tp;
        }
      }
    }
    __syncthreads();
    for (int j = lane; j < k; j += kWave) {
      const int64_t i = c.tile_lin * k + j;
      float d0 = s_u[3 * j] + o.bg[0] * s_b[j];
      float d1 = s_u[3 * j + 1] + o.bg[1] * s_b[j];
      float d2 = s_u[3 * j + 2] + o.bg[2] * s_b[j];
      if (MODE == 1) {
        jp_out[3 * i] = d0;
        jp_out[3 * i + 1] = d1;
        jp_out[3 * i + 2] = d2;
      } else {
        const float wj = wts ? wts[i] : 1.f;
        s_u[3 * j] = wj * d0;
        s_u[3 * j + 1] = wj * d1;
        s_u[3 * j + 2] = wj * d2;
      }
    }
    __syncthreads();
  }

  if (REV) {
    // s_a = T behind the chunk range already walked, s_b = u . (colour behind + T_final bg)
    for (int j = lane; j < k; j += kWave) {
      const int64_t i = c.tile_lin * k + j;
      if (!FWD) {
        s_u[3 * j] = u_in[3 * i];
        s_u[3 * j + 1] = u_in[3 * i + 1];
        s_u[3 * j + 2] = u_in[3 * i + 2];
      }
      const float Tf = trans[i];
      s_a[j] = Tf;
      s_b[j] = Tf * (s_u[3 * j] * o.bg[0] + s_u[3 * j + 1] * o.bg[1] + s_u[3 * j + 2] * o.bg[2]);
    }
    __syncthreads();
    if (lmax < 0) return;
    for (int64_t c0 = (lmax / kWave) * kWave; c0 >= 0; c0 -= kWave) {
      const int64_t e = c0 + lane;
      const bool valid = e < c.len;
      RecF r{};
      int id = 0;
      if (valid) {
        id = ids[c.start + e];
        r = load_rec(rec, (size_t)c.v * n + id);
      }
      float g[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      for (int j = 0; j < k; ++j) {
        const int lj = s_last[j];
        if (c0 > lj) continue;
        const Alpha al = pair_alpha(r.u, r.v, r.A, r.B, r.C, r.o, s_xc[j], s_yc[j], o);
        const bool inc = valid && e <= lj && al.inc;
        const float a = inc ? al.a : 0.f;
        const float om = 1.f - a;
        const float ip = incl_prod(om, lane);
        float ep = __shfl_up(ip, 1, kWave);
        if (lane == 0) ep = 1.f;
        const float Tin = s_a[j] / bcast(ip, kWave - 1);
        const float Tn = Tin * ep;
        const float u0 = s_u[3 * j], u1 = s_u[3 * j + 1], u2 = s_u[3 * j + 2];
        const float urgb = u0 * r.r + u1 * r.g + u2 * r.b;
        const float term = inc ? urgb * a * Tn : 0.f;
        const float sinc = suffix_sum(term, lane);
        if (inc) {
          const float aT = a * Tn;
          g[6] += u0 * aT;
          g[7] += u1 * aT;
          g[8] += u2 * aT;
          if (!al.capped) {
            const float behind = s_b[j] + (sinc - term);
            const float ga = Tn * urgb - behind / om;
            const float gs = ga * a;
            g[5] += ga * al.es;
            g[0] -= gs * (r.A * al.dx + r.B * al.dy);
            g[1] -= gs * (r.B * al.dx + r.C * al.dy);
            g[2] -= 0.5f * gs * al.dx * al.dx;
            g[3] -= gs * al.dx * al.dy;
            g[4] -= 0.5f * gs * al.dy * al.dy;
          }
        }
        const float tot = bcast(sinc, 0);
        if (lane == 0) {
          s_a[j] = Tin;
          s_b[j] += tot;
        }
      }
      if (valid) {
        bool any = false;
        for (int q = 0; q < 9; ++q) any |= g[q] != 0.f;
        if (any)
          for (int q = 0; q < 9; ++q) atomicAdd(&grad2d[((size_t)c.v * 9 + q) * n + id], g[q]);
      }
    }
  }
}

// --------------------------------------------------------------- Gram
// Per (view, Gaussian) weighted Gram of d C_c / d rec over the tile's pixels
// and channels: geometry block, geometry x colour, colour, opacity.
__global__ __launch_bounds__(kWave) void gram_kernel(const float* __restrict__ rec,
                                                     const int64_t* __restrict__ tile_start,
                                                     const int32_t* __restrict__ ids,
                                                     const uint8_t* __restrict__ pix,
                                                     const float* __restrict__ wts,
                                                     const float* __restrict__ trans,
                                                     const int32_t* __restrict__ lastv, int n, int T,
                                                     int TX, int k, lmrs_render_opts o,
                                                     float* __restrict__ gram) {
  __shared__ float s_xc[kMaxK], s_yc[kMaxK], s_T[kMaxK], s_S[3 * kMaxK], s_w[kMaxK];
  __shared__ int s_last[kMaxK];
  const int lane = lane_id();
  const TileCtx c = tile_ctx(tile_start, T, TX);
  int lmax = -1;
  for (int j = lane; j < k; j += kWave) {
    const int64_t i = c.tile_lin * k + j;
    pixel_center(pix, k, c, j, &s_xc[j], &s_yc[j]);
    s_last[j] = lastv[i];
    lmax = max(lmax, s_last[j]);
    const float Tf = trans[i];
    s_T[j] = Tf;
    for (int ch = 0; ch < 3; ++ch) s_S[3 * j + ch] = Tf * o.bg[ch];
    s_w[j] = wts ? wts[i] : 1.f;
  }
  lmax = wave_max_i(lmax);
  __syncthreads();
  if (lmax < 0) return;
  for (int64_t c0 = (lmax / kWave) * kWave; c0 >= 0; c0 -= kWave) {
    const int64_t e = c0 + lane;
    const bool valid = e < c.len;
    RecF r{};
    int id = 0;
    if (valid) {
      id = ids[c.start + e];
      r = load_rec(rec, (size_t)c.v * n + id);
    }
    float G[kGram];
    for (int q = 0; q < kGram; ++q) G[q] = 0.f;
    const float rgb[3] = {r.r, r.g, r.b};
    for (int j = 0; j < k; ++j) {
      const int lj = s_last[j];
      if (c0 > lj) continue;
      const Alpha al = pair_alpha(r.u, r.v, r.A, r.B, r.C, r.o, s_xc[j], s_yc[j], o);
      const bool inc = valid && e <= lj && al.inc;
      const float a = inc ? al.a : 0.f;
      const float om = 1.f - a;
      const float ip = incl_prod(om, lane);
      float ep = __shfl_up(ip, 1, kWave);
      if (lane == 0) ep = 1.f;
      const float Tin = s_T[j] / bcast(ip, kWave - 1);
      const float Tn = Tin * ep;
      float behind[3], tot[3];
      for (int ch = 0; ch < 3; ++ch) {
        const float term = inc ? rgb[ch] * a * Tn : 0.f;
        const float sinc = suffix_sum(term, lane);
        behind[ch] = s_S[3 * j + ch] + (sinc - term);
        tot[ch] = bcast(sinc, 0);
      }
      if (inc) {
        const float wj = s_w[j];
        const float aT = a * Tn;
        G[30] += wj * aT * aT;
        if (!al.capped) {
          float ga[3], sga2 = 0.f;
          for (int ch = 0; ch < 3; ++ch) {
            ga[ch] = Tn * rgb[ch] - behind[ch] / om;
            sga2 += ga[ch] * ga[ch];
          }
          const float h[5] = {-(r.A * al.dx + r.B * al.dy), -(r.B * al.dx + r.C * al.dy),
                              -0.5f * al.dx * al.dx, -al.dx * al.dy, -0.5f * al.dy * al.dy};
          const float fg = wj * a * a * sga2;
          for (int p = 0; p < 5; ++p) {
            for (int q = p; q < 5; ++q) G[sym5(p, q)] += fg * h[p] * h[q];
            for (int ch = 0; ch < 3; ++ch) G[15 + 3 * p + ch] += wj * ga[ch] * a * h[p] * aT;
          }
          G[31] += wj * sga2 * al.es * al.es;
        }
      }
      if (lane == 0) {
        s_T[j] = Tin;
        for (int ch = 0; ch < 3; ++ch) s_S[3 * j + ch] += tot[ch];
      }
    }
    if (valid) {
      bool any = false;
      for (int q = 0; q < kGram; ++q) any |= G[q] != 0.f;
      if (any)
        for (int q = 0; q < kGram; ++q) atomicAdd(&gram[((size_t)c.v * kGram + q) * n + id], G[q]);
    }
  }
}

}  // namespace

void launch_render(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, hipStream_t s) {
  const int64_t tiles = (int64_t)d.V * d.T;
  render_kernel<<<(unsigned)tiles, kWave, 0, s>>>(f->rec, f->tile_start, f->ids, f->pix, d.n, d.T, d.TX,
                                                  d.k, o, f->color, f->trans, f->last);
}

void launch_deriv(int mode, const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                  const float* tan, const float* u, float* jp, float* grad2d, hipStream_t s) {
  const unsigned tiles = (unsigned)((int64_t)d.V * d.T);
#define LMRS_DERIV_ARGS                                                                              \
  f->rec, tan, f->tile_start, f->ids, f->pix, f->w, f->trans, f->last, d.n, d.T, d.TX, d.k, o, u, jp, \
      grad2d
  if (mode == 1) deriv_kernel<1><<<tiles, kWave, 0, s>>>(LMRS_DERIV_ARGS);
  else if (mode == 2) deriv_kernel<2><<<tiles, kWave, 0, s>>>(LMRS_DERIV_ARGS);
  else deriv_kernel<3><<<tiles, kWave, 0, s>>>(LMRS_DERIV_ARGS);
#undef LMRS_DERIV_ARGS
}

void launch_gram(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, float* gram,
                 hipStream_t s) {
  const unsigned tiles = (unsigned)((int64_t)d.V * d.T);
  gram_kernel<<<tiles, kWave, 0, s>>>(f->rec, f->tile_start, f->ids, f->pix, f->w, f->trans, f->last,
                                      d.n, d.T, d.TX, d.k, o, gram);
}

}  // namespace lmrs
