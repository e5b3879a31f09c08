/*
 * lmrs.h -- C ABI of the MI355X (gfx950) library for the Gauss-Newton hot path
 * of matrix-free Levenberg-Marquardt with residual sampling for 3D Gaussian
 * Splatting (Pehlivan et al., "Matrix-free Second-order Optimization of
 * Gaussian Splats with Residual Sampling", arXiv 2504.12905).
 *
 * The operator at the centre is the sampled, damped Gauss-Newton matrix
 *     A = J^T W J + lambda diag(d)                      (Sec. 4.1 eq. 8, Sec. 4.4 eq. 14)
 * where J is the Jacobian of the residuals r = I_hat - I (eq. 7) of the
 * alpha-blended render (Sec. 3 eq. 3) with respect to all Gaussian parameters,
 * evaluated at the sampled pixels, and W = diag(w) repeats each sampled
 * pixel's importance weight over its 3 colour channels (eq. 12-14).
 *
 * Conventions shared by every call
 * --------------------------------
 * Memory.  Every pointer marked "device" is HBM owned by the caller; the
 *   library never allocates, frees or retains device memory, and keeps no
 *   device state between calls. Host structs are read during the call only.
 *   For its wait on the tile-instance count, lmrs_bin_tiles / lmrs_lm_step
 *   create once per host thread one HIP event and one pinned host word, kept
 *   for the life of the thread.
 * Streams. `stream` is a hipStream_t passed as void* (NULL = default stream).
 *   Work is enqueued and the call returns, except lmrs_bin_tiles and
 *   lmrs_lm_step, which wait for the tile-instance count (see there). Calls
 *   on one frame must be ordered on one stream: they share the frame's
 *   buffers, including the work counters in lmrs_frame.sched.
 * Errors.  Arguments are checked on the host before anything is enqueued; a
 *   failed check returns a negative status and enqueues nothing.
 *   lmrs_last_error() gives a message for the calling thread. A fault inside
 *   a kernel surfaces as LMRS_EHIP from a later call or stream sync.
 * Outputs are overwritten, never accumulated.
 *
 * Parameter vector beta (float32, P = n (11 + 3K), K = (sh_degree+1)^2),
 * component-major segments (all Gaussians' first component, then the next):
 *     [0n,3n) mean xyz | [3n,6n) log-scale xyz | [6n,10n) quaternion wxyz
 *     (normalised inside) | [10n,11n) opacity logit | [11n + (3k+c) n] SH
 *     coefficient k of colour channel c.
 * These are the per-Gaussian opacity, colour, mean, scale and rotation of
 * Sec. 4.1; colour is 0.5 + sum_k Y_k(dir) f_k with the real SH basis of
 * degree <= 3 (degree 0 is the paper's Lambertian setting, Sec. 3).
 *
 * Cameras: lmrs_camera rows, world-to-camera R (row-major) and t, pinhole
 * fx fy cx cy; x right, y down, z forward; pixel (i, j) has centre
 * (i + 0.5, j + 0.5). Images are split in 16x16 tiles (Supp. A); width and
 * height must be multiples of 16, with at most 16384 tiles per view. T = (width/16)(height/16) tiles per view,
 * tile id = ty * (width/16) + tx, pixel-in-tile index = 16 * (y%16) + (x%16).
 *
 * Sampled pixels (Sec. 4.4, stratified per tile): k per tile, sample index
 * i = (v * T + t) * k + j for view v, tile t, slot j; S = V T k.
 */
#ifndef LMRS_H
#define LMRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lmrs_status;
#define LMRS_OK 0
#define LMRS_EINVAL (-1)       /* bad argument (message in lmrs_last_error) */
#define LMRS_ECAPACITY (-2)    /* tile-instance buffer too small; count written */
#define LMRS_EWORKSPACE (-3)   /* workspace smaller than lmrs_workspace_bytes */
#define LMRS_EHIP (-4)         /* HIP runtime error */
#define LMRS_ENUMERIC (-5)     /* numeric failure recorded on the device (see
                                  LMRS_REP_STATUS and lmrs_report_status)    */
#define LMRS_EUNSUPPORTED (-6) /* well-formed request this library does not
                                  handle (SH degree above 3, more than 16384
                                  tiles per view)                            */

/* Floats per screen record: u v f11 f12 f22 opacity r g b | key radius sub
 * (Sec. 3 eq. 3). (f11, f12, f22) is the upper-triangular Cholesky factor F of
 * the conic Q = Sigma_2D^-1 = F^T F, so that the Gaussian's exponent at pixel
 * offset (dx, dy) from (u, v) is -1/2 ((f11 dx + f12 dy)^2 + (f22 dy)^2).
 * The list decisions are taken in FP64: the camera depth z of the mean, the
 * projected centre and the footprint radius ceil(cutoff sqrt(lambda_max)) of
 * the 2-D covariance. key is the FP32 number nearest z; sub (the bits of a
 * uint32) is the number of FP64 values between key and z plus 2^30, so that
 * (key, sub) orders like z. */
#define LMRS_REC 12

typedef struct lmrs_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
} lmrs_camera;

/* Rasteriser constants. The paper follows 3DGS for these (Supp. A) and states
 * none; the defaults used throughout are alpha_min 1/255, alpha_max 0.99,
 * t_min 1e-4, lowpass 0.3 px^2, znear 0.2, cutoff 3 sigmas, black background. */
typedef struct lmrs_render_opts {
  float alpha_min;  /* a Gaussian with alpha below this is skipped            */
  float alpha_max;  /* alpha is capped here; a capped alpha has no derivative  */
  float t_min;      /* blending stops before the Gaussian taking T below this  */
  float lowpass;    /* added to the 2-D covariance diagonal (px^2)             */
  float znear;      /* Gaussians with camera depth <= znear are culled          */
  float cutoff;     /* footprint radius = ceil(cutoff * sqrt(lambda_max))       */
  float bg[3];      /* background colour added with the final transmittance    */
} lmrs_render_opts;

/* One view batch at one parameter vector. All pointers are device memory
 * owned by the caller; which call reads or writes each field is listed. */
typedef struct lmrs_frame {
  int32_t n;              /* Gaussians                                          */
  int32_t sh_degree;      /* 0..3                                               */
  int32_t n_views;        /* V, views in this batch                            */
  int32_t width, height;  /* pixels per view, multiples of 16                   */
  int32_t k;              /* samples per tile, 1..256                           */
  const float* beta;      /* [P] parameters                     (read by all)   */
  const lmrs_camera* cams;/* [>= max view id + 1] cameras       (project, lm)   */
  const int32_t* view_ids;/* [V] camera index of batch view v, or NULL = v      */
  float* rec;             /* [V][n][LMRS_REC] screen records    (project: out)  */
  int32_t* rect;          /* [V][n][4] tile rect x0 y0 x1 y1, end exclusive;
                             empty (x0 == x1) when culled        (project: out)  */
  int64_t* tile_start;    /* [V*T + 1] list offsets into ids    (bin: out)      */
  int32_t* ids;           /* [capacity] Gaussian ids per tile    (bin: out)      */
  int64_t capacity;       /* entries available in ids                            */
  int64_t* n_instances;   /* [1] total list entries             (bin: out)      */
  uint8_t* pix;           /* [V][T][k] pixel-in-tile indices, or NULL = all 256
                             pixels in order (k must be 256)    (lm: out)       */
  float* w;               /* [V][T][k] weights, or NULL = 1      (lm: out)       */
  float* color;           /* [S][3] rendered colour             (render: out)   */
  float* trans;           /* [S] final transmittance            (render: out)   */
  int32_t* last;          /* [S] list position of the last blended Gaussian,
                             -1 if none                          (render: out)   */
  int32_t* sched;         /* [LMRS_SCHED_INTS(V*T)] tile schedule of the splat
                             walks (render: out; jvp, vjp, gn, lm: read, counters
                             updated). Layout: [0, V*T) tile ids by decreasing
                             walk length; [V*T, 2 V*T) walk length of each tile
                             (sum over its samples of the 64-entry list chunks
                             up to their last blended Gaussian); then 4 counters
                             (next ticket, finished waves, tiles with a
                             non-empty walk, 0). The splat kernels hand tiles to
                             their waves in this order and leave the counters as
                             they found them.                                  */
  /* Blend table: the linearization of the sampled render at the current
   * parameters, one record per blending (sampled pixel, list entry) pair
   * (optional: blend_k NULL = not kept, and every GN product walks the tile
   * lists). For pair (pixel i, Gaussian g) with opacity a and transmittance
   * T in front of g, K = d C_i / d a = T rgb_g - (colour behind g, background
   * included) / (1 - a) per channel (0 when a is capped), so that
   * d C_i = a T d rgb_g + K d a. The record derivatives of a are recomputed
   * from g's screen record and the pixel. The Gauss-Newton products of eq. 14
   * are then sums over these pairs instead of walks over the lists.
   * lmrs_render counts the pairs of each tile into blend_start and marks the
   * table stale; the right-hand-side / diagonal pass (lmrs_gn_diag,
   * lmrs_linearize, lmrs_pcg, lmrs_lm_*) writes it when the count fits
   * blend_capacity and marks it built; lmrs_gn_product and the PCG's products
   * use it when built and walk the lists otherwise. Gaussian ids < 2^24. */
  float* blend_k;         /* [2][blend_capacity][4]: K_R, K_G, K_B, a T; copy 0
                             grouped by Gaussian, copy 1 by pixel (within each
                             tile and 64-entry list chunk)                    */
  uint32_t* blend_m;      /* [2][blend_capacity]: Gaussian id << 8 | sample
                             slot, for the pairs of blend_k                   */
  int32_t* blend_run;     /* [blend_capacity]: starts (relative to the tile's
                             first pair) of runs of at most 32 pairs of one
                             Gaussian; the runs of a tile are in order and
                             cover its pairs                                  */
  int32_t* blend_runs;    /* [V*T] runs per tile                               */
  int64_t* blend_start;   /* [V*T + 2] pair offset of each tile; [V*T] = total
                             pairs of the batch; [V*T + 1] = 1 when the table
                             is built for the current render, else 0          */
  int64_t blend_capacity; /* pairs available in blend_k, blend_m, blend_run   */
  /* SSIM residual (Supp. B, Sec. 6; see lmrs_ssim_residual). NULL when not
   * used. With wc set, the operator of lmrs_gn_product, lmrs_pcg and the LM
   * calls is J^T diag(wc) J + lambda D, and the diagonal of lmrs_gn_diag and
   * of the Jacobi preconditioner is that of J^T diag(wbar) J, wbar the mean
   * of a sample's three channel weights. */
  float* wc;              /* [S][3] per-channel operator weights, or NULL = w
                             on every channel         (ssim, lm with SSIM: out) */
  float* image;           /* [V][height][width][3] full render of the batch
                             views                    (ssim, lm with SSIM: out) */
  /* Deterministic accumulation: 0 = the sums over tiles (screen gradients of
   * J^T u and b, Gram blocks of the diagonal) and the per-pixel sums of J p
   * over the blend table are float atomics, whose order, and so the last
   * bits of every result, changes from run to run; 1 = they are fixed-point
   * integer sums (each float term split into two 64-bit integers in units of
   * 2^-20 and 2^-60), so every call gives the same bits for the same inputs
   * on the same GPU, whatever the order of the adds. Every other stage is
   * deterministic either way. Mode 1 needs a larger workspace
   * (lmrs_workspace_bytes reads this field) and holds per term: magnitudes
   * below 2^30 (a term beyond that, or not finite, makes its whole row NaN),
   * sums below 2^42, resolution 2^-60. */
  int32_t deterministic;
} lmrs_frame;

/* Length in int32 of lmrs_frame.sched for a batch of `tiles` = V*T tiles. */
#define LMRS_SCHED_INTS(tiles) (2 * (int64_t)(tiles) + 4)

/* Operation codes for lmrs_workspace_bytes. */
#define LMRS_OP_BIN 1
#define LMRS_OP_JVP 2
#define LMRS_OP_VJP 3
#define LMRS_OP_GN 4
#define LMRS_OP_DIAG 5
#define LMRS_OP_PCG 6
#define LMRS_OP_LM 7
#define LMRS_OP_SOLVE 8

/* Learning-rate and solver settings of one LM step (Alg. 1; Sec. 4.5; Supp. D). */
typedef struct lmrs_lm_params {
  int32_t iter;         /* LM iteration index (schedule, sampler counter)      */
  int32_t cg_iters;     /* GN products in the PCG loop                          */
  float lambda;         /* fixed damping (Sec. 4.1)                             */
  float eta_cap;        /* learning-rate cap (0.2)                              */
  float eta_warm;       /* fixed learning rate of the first iterations (0.05)  */
  int32_t warm_iters;   /* number of such iterations (10)                       */
  uint64_t seed;        /* residual-sampler seed                                */
  int32_t sampler;      /* LMRS_SAMPLER_UNIFORM, _RESIDUAL or _GAUSSIAN         */
  int32_t cg_iters_late;/* GN products from iteration late_iter on (Sec. 5: CG
                           steps rise to 8 after the 50th iteration); 0 keeps
                           cg_iters throughout                                  */
  int32_t late_iter;    /* first iteration of cg_iters_late (50)                */
  float ssim_weight;    /* s > 0 adds the SSIM residual with weight s beside the
                           colour residual (Supp. B: 0.2; see
                           lmrs_ssim_residual) and needs f->wc and f->image;
                           0 = colour residual only (f->wc ignored)             */
} lmrs_lm_params;

/* Pixel samplers (lmrs_sample, lmrs_lm_params.sampler). */
#define LMRS_SAMPLER_UNIFORM 0   /* Sec. 4.4: k distinct pixels per tile        */
#define LMRS_SAMPLER_RESIDUAL 1  /* Supp. E q_residual: k draws per tile with
                                    replacement from the softmax of |r|         */
#define LMRS_SAMPLER_GAUSSIAN 2  /* Supp. E q_Gaussian: k draws per tile with
                                    replacement in proportion to the number of
                                    Gaussians blended into each pixel           */

/* Slots of the device report written by lmrs_pcg / lmrs_lm_step. */
#define LMRS_REPORT_FLOATS 12
#define LMRS_REP_LOSS 0        /* sampled weighted loss sum_i w_i |r_i|^2 (with
                                  SSIM: sum_i w_i (|r_i|^2 + s |rho_i|^2))     */
#define LMRS_REP_ETA 1         /* learning rate applied                           */
#define LMRS_REP_XDC_MAX 2     /* max |x| over the DC colour coefficients         */
#define LMRS_REP_CG_DONE 3     /* PCG iterations that updated x                  */
#define LMRS_REP_R0 4          /* ||r_0|| = ||b||                                 */
#define LMRS_REP_RN 5          /* ||r|| after the last iteration                  */
#define LMRS_REP_BX 6          /* b^T x (> 0 for a descent step)                  */
#define LMRS_REP_INST 7        /* tile-list entries of this step                  */
#define LMRS_REP_STATUS 8      /* LMRS_FAIL_* bits of this step, 0 when none      */
#define LMRS_REP_PAIRS 9       /* blending (pixel, Gaussian) pairs of this step
                                  (the blend table needs that many entries)      */

/* Numeric failures, detected on the device (calls enqueue and return, so they
 * cannot be returned as a status). PCG stops at the first one; lmrs_lm_step /
 * lmrs_lm_solve then leave beta unchanged. */
#define LMRS_FAIL_NONFINITE 1  /* NaN or Inf in b, the preconditioner, the PCG
                                  residual or the solution x                   */
#define LMRS_FAIL_BREAKDOWN 2  /* p^T A p <= 0 (or NaN) before convergence: not
                                  possible for the SPD operator of Alg. 1, so
                                  NaN/Inf in p or A p, or a corrupt input      */
#define LMRS_FAIL_CAPACITY 4   /* (lmrs_lm_iterate) the tile lists needed more
                                  entries than capacity: they were left empty
                                  and the step changed nothing; report[INST]
                                  holds the count needed                       */

const char* lmrs_status_str(lmrs_status s);
const char* lmrs_last_error(void);

/* The status a host copy of a report (LMRS_REPORT_FLOATS floats) carries in
 * LMRS_REP_STATUS: LMRS_ECAPACITY for LMRS_FAIL_CAPACITY, LMRS_ENUMERIC for
 * the numeric bits, LMRS_OK for none (message in lmrs_last_error). report:
 * host memory; NULL gives LMRS_EINVAL. */
lmrs_status lmrs_report_status(const float* report);

/* Scratch bytes that call `op` needs for frame `f` (uses n, sh_degree,
 * n_views, width, height, k and capacity). Pass a buffer of at least this
 * size as (ws, ws_bytes); its contents need not be initialised. */
size_t lmrs_workspace_bytes(int32_t op, const lmrs_frame* f);

/* a1. Projection (Sec. 3 eq. 1-3, EWA splatting): for every batch view v and
 * Gaussian g, rec[v][g] = (u, v, conic factor f11 f12 f22, opacity sigmoid(logit),
 * rgb = 0.5 + sum_k Y_k(dir) f_k, low word of the FP64 camera depth's bits,
 * radius, high word) and rect[v][g]. The near-plane cull, the footprint
 * radius ceil(cutoff sqrt(lambda_max)) and the tile rectangle are decided in
 * FP64. Reads beta, cams, view_ids; writes rec, rect. */
lmrs_status lmrs_project(const lmrs_frame* f, const lmrs_render_opts* o, void* stream);

/* a2. Tile binning and depth sort (Sec. 3: projected Gaussians are sorted by
 * depth; Supp. A: 16x16 tiles). For each view and tile, ids of the Gaussians
 * whose rect holds the tile, ascending FP64 camera depth, ties by ascending id.
 * Reads rect and rec; writes n_instances, tile_start and ids. Waits for the
 * instance count; if it exceeds capacity returns LMRS_ECAPACITY with
 * *n_instances (device) holding the count needed and ids untouched. */
lmrs_status lmrs_bin_tiles(const lmrs_frame* f, void* ws, size_t ws_bytes, void* stream);

/* a3. Forward render of the sampled pixels (Sec. 3 eq. 3; Supp. A Alg. 2):
 * front-to-back blending of each pixel's tile list. Writes color (with
 * background), trans (final T), last, and sched (the tile order the
 * derivative kernels follow, from the walk lengths that last fixes). */
lmrs_status lmrs_render(const lmrs_frame* f, const lmrs_render_opts* o, void* stream);

/* J p at every sampled pixel (Sec. 4.2; Supp. A "Jv kernel", Alg. 3):
 * forward-mode derivative of the rendered colour along p, with the discrete
 * decisions of lmrs_render (lists, skips, last) held fixed.
 * p: device [P]; jp: device [S][3]. Needs rec, rect, lists and render outputs. */
lmrs_status lmrs_jvp(const lmrs_frame* f, const lmrs_render_opts* o, const float* p, float* jp,
                     void* ws, size_t ws_bytes, void* stream);

/* J^T u (Supp. A "J^T v kernel"): u device [S][3] (no weights applied),
 * out device [P]. Same state as lmrs_jvp. */
lmrs_status lmrs_vjp(const lmrs_frame* f, const lmrs_render_opts* o, const float* u, float* out,
                     void* ws, size_t ws_bytes, void* stream);

/* a6. Gauss-Newton product out = J^T W J p + lambda d.p, the operator product
 * inside the PCG loop of Alg. 1 (eq. 8 with the sampled Hessian of eq. 14),
 * W from f->w. d: device [P] or NULL
 * (all ones, the paper's lambda I). p, out: device [P], must not alias. */
lmrs_status lmrs_gn_product(const lmrs_frame* f, const lmrs_render_opts* o, const float* p,
                            float lambda, const float* d, float* out, void* ws, size_t ws_bytes,
                            void* stream);

/* lmrs_gn_product for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same launches and result, with its scratch (tangent records and screen
 * gradients, lmrs_workspace_bytes(LMRS_OP_GN, f) bytes) taken from a static
 * device array of 64 MiB per GPU instead of a workspace argument (frames up to
 * about 599k views x Gaussians, 220k with deterministic accumulation). The array is loaded with the library and held
 * until the process ends; the call allocates nothing. A frame that needs more
 * returns LMRS_EWORKSPACE. Every call on one GPU uses that GPU's array, so
 * calls that overlap on one GPU (other streams or threads) race: serialize
 * them. The first call on a device looks up the array's address there. */
lmrs_status lmrs_gn_product_noalloc(const lmrs_frame* f, const lmrs_render_opts* o, const float* p,
                                    float lambda, const float* d, float* out, void* stream);

/* Measurement variant of lmrs_gn_product: the same launches (tangent
 * projection, zero fill, the splat from the blend table, the fused list walk
 * (one of the two exits at once), reverse chain) with HIP events recorded on
 * `stream` between them; waits for the last event and writes the elapsed
 * milliseconds of each launch to ms[5] (host): ms[0] tangent, ms[1] fill,
 * ms[2] blend-table splat, ms[3] fused walk, ms[4] chain. For profiling and
 * benchmarks; the result in out is identical to lmrs_gn_product's. */
lmrs_status lmrs_gn_product_timed(const lmrs_frame* f, const lmrs_render_opts* o, const float* p,
                                  float lambda, const float* d, float* out, void* ws, size_t ws_bytes,
                                  void* stream, float* ms);

/* Measurement helper: what the sampled render's walk touches, for the
 * algorithmic bytes and flops of the splat kernels. Needs the state of
 * lmrs_jvp (lists, samples, render outputs). counts: device int64[4],
 * overwritten:
 *   [0] sum over tiles of L*_t = max over the tile's sampled pixels of last + 1
 *       (the list prefix a walk traverses);
 *   [1] sum over tiles of C_t = list entries blended by at least one of the
 *       tile's sampled pixels (the entries that receive gradient);
 *   [2] blending (pixel, entry) pairs (Sec. 3 eq. 3 terms with alpha >= alpha_min);
 *   [3] (pixel, entry) pairs up to and including each pixel's last blended entry. */
lmrs_status lmrs_walk_counts(const lmrs_frame* f, const lmrs_render_opts* o, int64_t* counts, void* stream);

/* Builds the blend table of f (see lmrs_frame) for the current render: one
 * reverse walk over the lists (the walk of the diagonal pass without its
 * sums). Needs the state of lmrs_jvp and the blend buffers; when the pair
 * count (blend_start[V*T], written by lmrs_render) exceeds blend_capacity the
 * table stays unbuilt and the GN products walk the lists. No workspace. */
lmrs_status lmrs_linearize(const lmrs_frame* f, const lmrs_render_opts* o, void* stream);

/* a5. diag(J^T W J) (Alg. 1 preconditioner; Supp. A "Diag(J^T J) kernel"),
 * exact: per (view, Gaussian) the weighted Gram matrix of the screen-record
 * derivatives, then contracted with the record Jacobian. out: device [P]. */
lmrs_status lmrs_gn_diag(const lmrs_frame* f, const lmrs_render_opts* o, float* out, void* ws,
                         size_t ws_bytes, void* stream);

/* a5 + a7. Matrix-free PCG of Alg. 1 from x0 = 0: Jacobi preconditioner
 * 1 / (diag(J^T W J) + lambda d), exactly `iters` GN products; x stops
 * changing if p^T A p <= 0 or r^T z collapses. b, x: device [P].
 * report: device [LMRS_REPORT_FLOATS] or NULL (slots CG_DONE, R0, RN, BX,
 * STATUS). A numeric failure stops the iteration and sets LMRS_REP_STATUS. */
lmrs_status lmrs_pcg(const lmrs_frame* f, const lmrs_render_opts* o, const float* b, float lambda,
                     const float* d, int32_t iters, float* x, float* report, void* ws,
                     size_t ws_bytes, void* stream);

/* Residual magnitudes for the residual-weighted sampler (Supp. E, eq. 16):
 * renders every pixel of the batch views (as lmrs_render with k = 256) and
 * writes scores[(v * T + t) * 256 + p] = |C_R - I_R| + |C_G - I_G| + |C_B - I_B|,
 * C with background, I from targets (device [*][height][width][3], indexed
 * by camera id f->view_ids[v]). Needs rec, rect and the tile lists; f->k,
 * f->pix and the render outputs are not used. scores: device [V][T][256]. */
lmrs_status lmrs_residual_scores(const lmrs_frame* f, const lmrs_render_opts* o, const float* targets,
                                 float* scores, void* stream);

/* Contributor counts for the contribution-weighted sampler (Supp. E, eq. 17):
 * renders every pixel of the batch views (as lmrs_render with k = 256) and
 * writes counts[(v * T + t) * 256 + p] = G_p, the number of Gaussians blended
 * into the pixel (skipped transparent ones and those behind the transmittance
 * stop not counted), as floats. Needs rec, rect and the tile lists.
 * counts: device [V][T][256]. */
lmrs_status lmrs_contributor_counts(const lmrs_frame* f, const lmrs_render_opts* o, float* counts, void* stream);

/* SSIM residual with the diagonal approximation (Supp. B "Results with SSIM
 * loss"; Sec. 6 Limitations). The paper adds SSIM to the colour loss with
 * weights 0.2 and 1.0 and keeps only the dependence of each pixel's SSIM on
 * that pixel's own rendered colour; it gives no formula. Here: per colour
 * channel c, SSIM_c(p) of Wang et al. over an 11 x 11 Gaussian window
 * (sigma 1.5, weights summing to 1, zero outside the image), C1 = 0.01^2,
 * C2 = 0.03^2, enters the least-squares objective as a second residual
 * rho = 1 - SSIM_c(p) per sampled pixel and channel with weight s:
 *   E = sum_i w_i sum_c (r_ic^2 + s rho_ic^2),  r = C - I.
 * With delta = -d SSIM_c(p) / d C_c(p) (the centre pixel only), the
 * Gauss-Newton system has b = J^T u and operator J^T diag(wc) J + lambda D,
 *   u_ic = w_i (r_ic + s delta_ic rho_ic),  wc_ic = w_i (1 + s delta_ic^2).
 * This call renders every pixel of the batch views into f->image (as
 * lmrs_render with k = 256, background added), then at every sample writes
 * u (device [S][3]) and f->wc. r, SSIM and delta come from f->image and the
 * targets (device [*][height][width][3], indexed by camera id); the window
 * sums are taken in FP64. tile_loss: device double [V*T] (the tile's share
 * of E) or NULL. Needs rec, rect, the tile lists and f->pix / f->w (or k =
 * 256 with pix NULL); s >= 0. lmrs_lm_step with prm->ssim_weight = s calls
 * it in place of the colour residual. */
lmrs_status lmrs_ssim_residual(const lmrs_frame* f, const lmrs_render_opts* o, const float* targets, float s,
                               float* u, double* tile_loss, void* stream);

/* a4. Stratified pixel sampling (Sec. 4.4), writes f->pix and f->w
 * ([V][T][k], device; both must be non-NULL).
 * LMRS_SAMPLER_UNIFORM: k distinct pixels per tile, the k smallest
 *   (Philox4x32-10 word of counter (p, tile, camera id, iter), p) with
 *   key = seed, in ascending pixel order; weight 256/k.
 * LMRS_SAMPLER_RESIDUAL (Supp. E q_residual): inside each tile
 *   q(p) = exp(s_p) / sum exp(s), s = scores (lmrs_residual_scores); draw j
 *   takes u_j = (top 24 bits of the first Philox word of counter
 *   (256 + j, tile, camera id, iter)) * 2^-24 and the smallest p whose
 *   running sum of q in pixel order exceeds u_j; k draws with replacement
 *   in draw order, weight 1 / (k q(p)).
 * LMRS_SAMPLER_GAUSSIAN (Supp. E q_Gaussian, eq. 17): scores holds the
 *   counts G_p of lmrs_contributor_counts; inside each tile q(p) = G_p / Z,
 *   Z = sum G (a tile with Z = 0 is sampled uniformly, G_p taken as 1); draw j
 *   takes the 24-bit word d_j of the same counter as the residual sampler and
 *   the smallest p with (G_0 + ... + G_p) 2^24 > d_j Z, in integers; weight
 *   Z / (k G_p).
 * scores is ignored by the uniform sampler and may be NULL there. Unknown
 * sampler: LMRS_EINVAL. */
lmrs_status lmrs_sample(const lmrs_frame* f, int32_t sampler, uint64_t seed, int32_t iter, const float* scores,
                        void* stream);

/* View batches by camera clustering (Sec. 4.3), host code (no device work).
 * lmrs_view_clusters splits n_cams cameras (host lmrs_camera array) into
 * `batch` clusters by K-means on the 6-D features (camera centre moved to the
 * centres' mean and scaled by their largest distance from it; viewing
 * direction = third row of R): D^2 seeding from Philox4x32-10 words of
 * counters (s, 0, batch, 0x4b4d0001) with key = seed, then Lloyd rounds until
 * no assignment changes (at most 100; an empty cluster takes the camera
 * farthest from its own centre). labels: host int32[n_cams], cluster of each
 * camera. Needs 0 < batch <= n_cams, else LMRS_EINVAL. */
lmrs_status lmrs_view_clusters(const lmrs_camera* cams, int32_t n_cams, int32_t batch, uint64_t seed,
                               int32_t* labels);

/* One camera from each cluster for LM iteration `iter`: cluster j (members in
 * ascending camera index, m of them) gives member floor(d m / 2^24), d the top
 * 24 bits of the first Philox4x32-10 word of counter (j, iter, batch,
 * 0x4b4d0002), key = seed. labels: host int32[n_cams] from
 * lmrs_view_clusters; view_ids: host int32[batch] (out). */
lmrs_status lmrs_view_batch(const int32_t* labels, int32_t n_cams, int32_t batch, uint64_t seed, int32_t iter,
                            int32_t* view_ids);

/* a1-a8. One LM iteration of Alg. 1 on the batch views f->view_ids:
 * project, bin, sample k pixels per tile (prm->sampler, as lmrs_sample;
 * the weighted samplers first render every pixel for their scores or
 * counts; with the
 * uniform sampler and f->pix NULL, k = 256 takes every pixel with weight 1),
 * render, residuals r = C - I against targets
 * (device [*][height][width][3], indexed by camera id), b = J^T W r (with
 * prm->ssim_weight > 0: the SSIM residual of lmrs_ssim_residual added, b =
 * J^T u and the operator weighted by f->wc),
 * Jacobi-PCG, learning rate (Sec. 4.5: eta_warm for iter < warm_iters, else
 * min(eta_cap, 1 / max |x_dc|)) and the descent update beta <- beta - eta x.
 * f->beta must equal beta; f->pix and f->w receive the samples. Waits for the
 * instance count like lmrs_bin_tiles (LMRS_ECAPACITY leaves beta unchanged).
 * report: device [LMRS_REPORT_FLOATS] or NULL. */
lmrs_status lmrs_lm_step(lmrs_frame* f, float* beta, const float* targets, const float* d,
                         const lmrs_lm_params* prm, const lmrs_render_opts* o, float* report,
                         void* ws, size_t ws_bytes, void* stream);

/* lmrs_bin_tiles without the host's wait: enqueues every launch and returns.
 * If the count exceeds f->capacity, every list comes out empty (tile_start
 * all 0, ids untouched) and *n_instances (device) holds the count needed; the
 * caller finds out by reading it. f->ids must be non-NULL. Graph-capturable. */
lmrs_status lmrs_bin_tiles_async(const lmrs_frame* f, void* ws, size_t ws_bytes, void* stream);

/* One LM iteration as lmrs_lm_step (same arguments and workspace,
 * LMRS_OP_LM), with the binning of lmrs_bin_tiles_async: it never waits on
 * the host, so a whole iteration can be captured into a HIP graph. A count
 * above f->capacity leaves beta unchanged and sets LMRS_FAIL_CAPACITY in
 * report[LMRS_REP_STATUS], with the count in report[LMRS_REP_INST]. */
lmrs_status lmrs_lm_iterate(lmrs_frame* f, float* beta, const float* targets, const float* d,
                            const lmrs_lm_params* prm, const lmrs_render_opts* o, float* report,
                            void* ws, size_t ws_bytes, void* stream);

/* a4-a8. The part of lmrs_lm_step after lmrs_project and lmrs_bin_tiles:
 * sampling, render, residuals, b = J^T W r, preconditioner, PCG, learning
 * rate and update (Alg. 1), with the same arguments and results. It never
 * waits on the host, so a caller can capture it into a HIP graph and replay
 * it on later LM iterations whose kernel arguments are unchanged: the same
 * buffers, and an iteration index that changes neither the learning-rate
 * branch (iter < warm_iters) nor the samples (k = 256 with f->pix NULL).
 * The tile lists of f must be current (lmrs_bin_tiles on the current beta).
 * Workspace: lmrs_workspace_bytes(LMRS_OP_SOLVE, f). */
lmrs_status lmrs_lm_solve(lmrs_frame* f, float* beta, const float* targets, const float* d,
                          const lmrs_lm_params* prm, const lmrs_render_opts* o, float* report,
                          void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LMRS_H */
