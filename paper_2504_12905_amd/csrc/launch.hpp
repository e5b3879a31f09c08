// Host-side launchers of the lmrs kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lmrs.h"

namespace lmrs {

// Geometry shared by the splat kernels of one frame.
struct FrameDims {
  int n, deg, pg, V, W, H, TX, TY, T, k;
  int64_t S;  // sampled pixels V*T*k
  bool det;   // deterministic accumulation: grad2d and gram hold fixed-point rows
};

FrameDims dims_of(const lmrs_frame* f);

// sets the calling thread's lmrs_last_error() message and returns s
lmrs_status report_error(lmrs_status s, const char* msg);

// projection side (kernels_project.hip)
void launch_project(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, hipStream_t s);
void launch_tangent(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, const float* p,
                    float* tan, hipStream_t s);
// pu_part (optional): one FP64 partial of p . out per workgroup, chain_vjp_blocks(n, true) of them
// zero_rows: clear the non-zero grad2d rows after reading them (grad2d is
// then all zero for the next accumulation).
void launch_chain_vjp(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                      float* grad2d, const float* p, float lambda, const float* dvec, float* out,
                      hipStream_t s, double* pu_part = nullptr, bool zero_rows = false);
int chain_vjp_blocks(int n, bool partials);
void launch_chain_diag(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                       const float* gram, float* out, hipStream_t s);
void launch_fill(float* x, int64_t count, float value, hipStream_t s);

// binning (kernels_bin.hip)
struct BinScratch {
  int32_t* counts;      // [V*T]
  int32_t* chunk_hist;  // [V][bin_chunks(n)][T]
  uint32_t* keys;       // [capacity] depth ranks per tile segment
  uint32_t* vkey[2];    // [V][n] depth bits, sort ping-pong
  uint32_t* vval[2];    // [V][n] Gaussian ids, sort ping-pong
  int32_t* order;       // [V][n] Gaussian id of each depth rank (= vval[0] after the sort)
  int32_t* vcount;      // [view_sort_count_ints(n, V)] digit counts / offsets of the view sort
  int64_t* area_part;   // [kBinAreaParts] partial sums of the entry count
  int64_t* col_part;    // [ceil(V*T / 256)] per-workgroup sums of the tile totals
};
constexpr int kBinAreaParts = 1024;
int view_sort_count_ints(int n, int V);
constexpr int kMaxTilesPerView = 16384;  // LDS histogram of one view's tiles (64 KB)
int bin_chunks(int n);
void launch_bin_total(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s);
void launch_bin_count(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s);
// per-view depth ranks (independent of the tile counts)
void launch_view_sort(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s);
// emission of the ranks and per-tile sort (after launch_view_sort)
void launch_bin_emit_sort(const lmrs_frame* f, const FrameDims& d, BinScratch b, hipStream_t s);

// splatting (kernels_splat.hip)
void launch_render(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, hipStream_t s);
// every pixel of the batch views: scores[V][T][256] = sum_c |C_c - I_c| against targets
void launch_render_scores(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                          const float* targets, float* scores, hipStream_t s);
// every pixel of the batch views: counts[V][T][256] = Gaussians blended into the pixel
void launch_render_counts(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, float* counts,
                          hipStream_t s);
// every pixel of the batch views: image[V][H][W][3] = rendered colour with background
void launch_render_image(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, float* image,
                         hipStream_t s);
// counts[4] (int64, device): traversed entries, contributing entries, blending
// pairs, pairs up to each pixel's last blended entry (see walk_count_kernel)
void launch_walk_counts(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, int64_t* counts,
                        hipStream_t s);
// mode: 1 = J p only (writes jp), 2 = J^T u only (reads u), 3 = fused GN (J^T W J p)
void launch_deriv(int mode, const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o,
                  const float* tan, const float* u, float* jp, float* grad2d, hipStream_t s);
// gram[V][n][32] (one 128-byte row per (view, Gaussian)); with u non-NULL also grad2d += J^T u (u: [S][3])
void launch_gram(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, float* gram,
                 const float* u, float* grad2d, hipStream_t s, bool gram_sums = true);
// J^T W J p from the blend table into grad2d (exits at once unless the table
// is built; the fused walk of launch_deriv(3) then runs instead)
void launch_blend_gn(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, const float* tan,
                     float* grad2d, hipStream_t s);

// solver side (kernels_solver.hip)
constexpr int kRedBlocks = 512;  // partial sums per reduction
void launch_sample_uniform(const lmrs_frame* f, const FrameDims& d, uint64_t seed, int iter,
                           hipStream_t s);
void launch_sample_residual(const lmrs_frame* f, const FrameDims& d, const float* scores, uint64_t seed,
                            int iter, hipStream_t s);
// counts: [V][T][256] Gaussians blended into each pixel (integers held in floats)
void launch_sample_gaussian(const lmrs_frame* f, const FrameDims& d, const float* counts, uint64_t seed,
                            int iter, hipStream_t s);
void launch_residual(const lmrs_frame* f, const FrameDims& d, const float* targets, float* wr,
                     double* partials, float* report, hipStream_t s);
// SSIM residual at the samples from f->image and the targets: u[S][3], f->wc;
// tile_loss[V*T] (may be NULL) the tiles' shares of the objective, summed
// into *loss_out (and report[LOSS]) when loss_out is not NULL
void launch_ssim(const lmrs_frame* f, const FrameDims& d, const float* targets, float s_w, float* u,
                 double* tile_loss, double* loss_out, float* report, hipStream_t s);
void launch_dot(const float* a, const float* b, int64_t n, double* partials, double* out, hipStream_t s);
// report[INST] = *count; ORs LMRS_FAIL_CAPACITY into report[STATUS] when *count > capacity
// and report[PAIRS] = *pairs when pairs is not NULL
void launch_report_count(const int64_t* count, int64_t capacity, float* report, hipStream_t s,
                         const int64_t* pairs = nullptr);
// PCG state in device memory
struct PcgState {
  float *x, *r, *z, *p, *u, *minv;
  double* sc;        // two banks of 16 scalars: iteration i reads bank i % 2 (see kernels_solver.hip)
  double* partials;  // [4 * kRedBlocks]
  __host__ __device__ double* bank(int it) const { return sc + 16 * (it & 1); }
};
void launch_pcg_init(const float* b, const float* diag, float lambda, const float* dvec, int64_t P,
                     PcgState st, hipStream_t s);
// one PCG iteration after the product u = A p, whose chain kernel left pu_count
// partials of p^T u in st.partials: alpha, x, r, z, beta, p
void launch_pcg_iteration(int it, int64_t P, int pu_count, PcgState st, hipStream_t s);
void launch_pcg_report(const float* b, int iters, int64_t P, PcgState st, float* report, hipStream_t s);
// the failure bits the PCG left after `iters` iterations (device)
const double* pcg_fail_slot(int iters, PcgState st);
// learning rate and update; partials: at least 2 * kRedBlocks + 2 doubles.
// Skips the update when pcg_fail (device, may be NULL) or a non-finite entry
// of x flags a numeric failure.
void launch_lm_update(float* beta, const float* x, int n, int64_t P, const lmrs_lm_params& prm,
                      const double* pcg_fail, double* partials, float* report, hipStream_t s);

}  // namespace lmrs
