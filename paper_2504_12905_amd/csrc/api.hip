// C ABI of liblmrs (see include/lmrs.h for the contract of every call).
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "common.hpp"
#include "launch.hpp"

namespace lmrs {

namespace {

thread_local char g_err[512] = "";

lmrs_status fail(lmrs_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

lmrs_status hip_check(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LMRS_EHIP, "%s: %s", what, hipGetErrorString(e));
  return LMRS_OK;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int kRedDoubles = 4 * kRedBlocks + 64;

// Bump allocator over the caller's workspace; the same sequence of take()
// calls sizes the workspace (base == nullptr) and carves it.
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += align_up(count * sizeof(T));
    return p;
  }
};

struct Scratch {
  float* tan = nullptr;
  float* grad2d = nullptr;
  float* gram = nullptr;
  float* diag = nullptr;
  float *r = nullptr, *z = nullptr, *p = nullptr, *u = nullptr, *minv = nullptr;
  float* b = nullptr;
  float* x = nullptr;
  float* wr = nullptr;
  float* scores = nullptr;
  double* tile_loss = nullptr;
  double* sc = nullptr;
  double* red = nullptr;
  BinScratch bin{};
};

// 32-bit words of the screen-gradient and Gram accumulators (float rows, or
// the fixed-point rows of deterministic accumulation).
int64_t grad_floats(const FrameDims& d) { return (int64_t)d.V * d.n * (d.det ? kFixGradFloats : kGradRow); }
int64_t gram_floats(const FrameDims& d) { return (int64_t)d.V * d.n * (d.det ? kFixGramFloats : kGram); }

// Workspace layout of each operation.
Scratch carve(int op, const FrameDims& d, int64_t capacity, Carver& c) {
  Scratch s;
  const int64_t P = (int64_t)d.n * d.pg;
  const int64_t VN = (int64_t)d.V * d.n;
  const bool lm = op == LMRS_OP_LM || op == LMRS_OP_SOLVE;
  const bool need_bin = op == LMRS_OP_BIN || op == LMRS_OP_LM;
  const bool need_tan = op == LMRS_OP_JVP || op == LMRS_OP_GN || op == LMRS_OP_PCG || lm;
  const bool need_grad = op == LMRS_OP_VJP || op == LMRS_OP_GN || op == LMRS_OP_PCG || lm;
  const bool need_gram = op == LMRS_OP_DIAG || op == LMRS_OP_PCG || lm;
  const bool need_pcg = op == LMRS_OP_PCG || lm;
  if (need_bin) {
    s.bin.counts = c.take<int32_t>((size_t)d.V * d.T);
    s.bin.chunk_hist = c.take<int32_t>((size_t)d.V * bin_chunks(d.n) * d.T);
    s.bin.keys = c.take<uint32_t>((size_t)capacity);
    for (int q = 0; q < 2; ++q) {
      s.bin.vkey[q] = c.take<uint32_t>((size_t)VN);
      s.bin.vval[q] = c.take<uint32_t>((size_t)VN);
    }
    s.bin.order = reinterpret_cast<int32_t*>(s.bin.vval[0]);
    s.bin.vcount = c.take<int32_t>((size_t)view_sort_count_ints(d.n, d.V));
    s.bin.area_part = c.take<int64_t>(kBinAreaParts);
    s.bin.col_part = c.take<int64_t>(((size_t)d.V * d.T + 255) / 256);
  }
  if (need_tan) s.tan = c.take<float>((size_t)VN * LMRS_REC);
  if (need_grad) s.grad2d = c.take<float>((size_t)grad_floats(d));
  if (need_gram) s.gram = c.take<float>((size_t)gram_floats(d));
  if (need_pcg) {
    s.diag = c.take<float>(P);
    s.r = c.take<float>(P);
    s.z = c.take<float>(P);
    s.p = c.take<float>(P);
    s.u = c.take<float>(P);
    s.minv = c.take<float>(P);
    s.sc = c.take<double>(32);
  }
  if (lm) {
    s.b = c.take<float>(P);
    s.x = c.take<float>(P);
    s.wr = c.take<float>((size_t)d.S * 3);
    s.scores = c.take<float>((size_t)d.V * d.T * 256);
    s.tile_loss = c.take<double>((size_t)d.V * d.T);
  }
  s.red = c.take<double>(kRedDoubles);
  return s;
}

lmrs_status check_frame(const lmrs_frame* f, bool need_samples_k = true) {
  if (!f) return fail(LMRS_EINVAL, "frame is NULL");
  if (f->n <= 0) return fail(LMRS_EINVAL, "n = %d must be positive", f->n);
  if (f->sh_degree < 0) return fail(LMRS_EINVAL, "sh_degree = %d is negative", f->sh_degree);
  if (f->sh_degree > 3) return fail(LMRS_EUNSUPPORTED, "sh_degree = %d: degrees 0..3 are built", f->sh_degree);
  if (f->n_views <= 0) return fail(LMRS_EINVAL, "n_views = %d must be positive", f->n_views);
  if (f->width <= 0 || f->height <= 0 || f->width % kTile || f->height % kTile)
    return fail(LMRS_EINVAL, "image %dx%d must be positive multiples of 16", f->width, f->height);
  if ((int64_t)(f->width / kTile) * (f->height / kTile) > kMaxTilesPerView)
    return fail(LMRS_EUNSUPPORTED, "%d x %d image has more than %d tiles", f->width, f->height, kMaxTilesPerView);
  const int64_t tiles = (int64_t)f->n_views * (f->width / kTile) * (f->height / kTile);
  if (tiles > 0x7fffffffLL) return fail(LMRS_EINVAL, "too many tiles");
  if (need_samples_k) {
    if (f->k < 1 || f->k > 256) return fail(LMRS_EINVAL, "k = %d not in 1..256", f->k);
    if (!f->pix && f->k != 256) return fail(LMRS_EINVAL, "pix is NULL but k = %d != 256", f->k);
  }
  if (!f->beta) return fail(LMRS_EINVAL, "beta is NULL");
  if (f->deterministic != 0 && f->deterministic != 1)
    return fail(LMRS_EINVAL, "deterministic = %d must be 0 or 1", f->deterministic);
  if (f->blend_k) {
    if (!f->blend_m || !f->blend_run || !f->blend_runs || !f->blend_start)
      return fail(LMRS_EINVAL, "blend_k is set: blend_m, blend_run, blend_runs and blend_start are needed");
    if (f->blend_capacity < 0) return fail(LMRS_EINVAL, "blend_capacity is negative");
    if (f->n >= (1 << 24)) return fail(LMRS_EUNSUPPORTED, "the blend table holds Gaussian ids below 2^24 (n = %d)", f->n);
  }
  return LMRS_OK;
}

lmrs_status need(const void* p, const char* name) {
  return p ? LMRS_OK : fail(LMRS_EINVAL, "%s is NULL", name);
}

lmrs_status check_ws(int op, const lmrs_frame* f, void* ws, size_t ws_bytes) {
  const size_t req = lmrs_workspace_bytes(op, f);
  if (ws_bytes < req || (!ws && req > 0))
    return fail(LMRS_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, req);
  if (reinterpret_cast<uintptr_t>(ws) % kAlign)
    return fail(LMRS_EWORKSPACE, "workspace must be 256-byte aligned");
  return LMRS_OK;
}

lmrs_status check_render_state(const lmrs_frame* f) {
  lmrs_status st;
  if ((st = need(f->rec, "rec")) || (st = need(f->rect, "rect")) || (st = need(f->tile_start, "tile_start")) ||
      (st = need(f->ids, "ids")) || (st = need(f->cams, "cams")))
    return st;
  return LMRS_OK;
}

lmrs_status check_deriv_state(const lmrs_frame* f) {
  lmrs_status st = check_render_state(f);
  if (st) return st;
  if ((st = need(f->trans, "trans")) || (st = need(f->last, "last")) || (st = need(f->sched, "sched"))) return st;
  return LMRS_OK;
}

#define LMRS_TRY(x)              \
  do {                           \
    const lmrs_status _s = (x);  \
    if (_s != LMRS_OK) return _s; \
  } while (0)

// J^T W J p + lambda d p into out (tangent, fused splat, chain).
// pu_part (optional): partials of p . out for the PCG update.
// grad_zero: s.grad2d is known to be all zero (a previous chain cleared it),
// so it needs no fill; the chain leaves it all zero again.
void gn_sequence(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, const float* p,
                 float lambda, const float* dvec, float* out, const Scratch& s, hipStream_t st,
                 double* pu_part = nullptr, bool grad_zero = false) {
  launch_tangent(f, d, o, p, s.tan, st);
  if (!grad_zero) launch_fill(s.grad2d, grad_floats(d), 0.f, st);
  // from the blend table when it is built for this render, else the fused walk
  launch_blend_gn(f, d, o, s.tan, s.grad2d, st);
  launch_deriv(3, f, d, o, s.tan, nullptr, nullptr, s.grad2d, st);
  launch_chain_vjp(f, d, o, s.grad2d, p, lambda, dvec, out, st, pu_part, true);
}

void vjp_sequence(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, const float* u,
                  float* out, const Scratch& s, hipStream_t st) {
  launch_fill(s.grad2d, grad_floats(d), 0.f, st);
  launch_deriv(2, f, d, o, nullptr, u, nullptr, s.grad2d, st);
  launch_chain_vjp(f, d, o, s.grad2d, nullptr, 0.f, nullptr, out, st);
}

void diag_sequence(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, float* out,
                   const Scratch& s, hipStream_t st) {
  launch_fill(s.gram, gram_floats(d), 0.f, st);
  launch_gram(f, d, o, s.gram, nullptr, nullptr, st);
  launch_chain_diag(f, d, o, s.gram, out, st);
}

// b = J^T u and diag(J^T W J) from one reverse walk (the Gram pass with J^T u).
void vjp_diag_sequence(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, const float* u,
                       float* b, float* diag, const Scratch& s, hipStream_t st) {
  launch_fill(s.gram, gram_floats(d), 0.f, st);
  launch_fill(s.grad2d, grad_floats(d), 0.f, st);
  launch_gram(f, d, o, s.gram, u, s.grad2d, st);
  launch_chain_vjp(f, d, o, s.grad2d, nullptr, 0.f, nullptr, b, st, nullptr, true);  // leaves grad2d zero
  launch_chain_diag(f, d, o, s.gram, diag, st);
}

// PCG of Alg. 1; diag(J^T W J) is formed here unless have_diag (then s.diag
// holds it). grad_zero: s.grad2d is all zero on entry (vjp_diag_sequence ran).
void pcg_sequence(const lmrs_frame* f, const FrameDims& d, const lmrs_render_opts& o, const float* b,
                  float lambda, const float* dvec, int iters, float* x, float* report, const Scratch& s,
                  hipStream_t st, bool have_diag = false, bool grad_zero = false) {
  const int64_t P = (int64_t)d.n * d.pg;
  if (!have_diag) diag_sequence(f, d, o, s.diag, s, st);
  PcgState ps{x, s.r, s.z, s.p, s.u, s.minv, s.sc, s.red};
  launch_pcg_init(b, s.diag, lambda, dvec, P, ps, st);
  for (int it = 0; it < iters; ++it) {
    gn_sequence(f, d, o, s.p, lambda, dvec, s.u, s, st, ps.partials, grad_zero || it > 0);
    launch_pcg_iteration(it, P, chain_vjp_blocks(d.n, true), ps, st);
  }
  if (report) launch_pcg_report(b, iters, P, ps, report, st);
}

// Count, then the per-view depth sort (it does not need the count, so it
// runs on the device while the host waits for the total), then emit and sort.
lmrs_status bin_sequence(const lmrs_frame* f, const FrameDims& d, const Scratch& s, hipStream_t st,
                         int64_t* total_out = nullptr) {
  // per host thread: an event after the count's copy and a pinned host word
  // for the count (kept for the life of the thread)
  static thread_local hipEvent_t counted = nullptr;
  static thread_local int64_t* count_host = nullptr;
  if (!counted && hipEventCreateWithFlags(&counted, hipEventDisableTiming) != hipSuccess) {
    counted = nullptr;
    return hip_check("bin count event");
  }
  if (!count_host && hipHostMalloc(reinterpret_cast<void**>(&count_host), sizeof(int64_t)) != hipSuccess) {
    count_host = nullptr;
    return hip_check("bin count buffer");
  }
  launch_bin_total(f, d, s.bin, st);
  if (hipMemcpyAsync(count_host, f->n_instances, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipEventRecord(counted, st) != hipSuccess)
    return hip_check("bin count");
  // while the host waits for the count: depth ranks, per-chunk tile counts, tile_start
  launch_view_sort(f, d, s.bin, st);
  launch_bin_count(f, d, s.bin, st);
  if (hipEventSynchronize(counted) != hipSuccess) return hip_check("bin count");
  LMRS_TRY(hip_check("bin count"));
  const int64_t total = *count_host;
  if (total > f->capacity)
    return fail(LMRS_ECAPACITY, "%lld tile-list entries needed, capacity %lld", (long long)total,
                (long long)f->capacity);
  if (total_out) *total_out = total;
  launch_bin_emit_sort(f, d, s.bin, st);
  return hip_check("bin sort");
}

// The same launches without the host's wait for the count: when the count
// exceeds f->capacity the lists come out empty (on the device) and
// *n_instances holds the count needed.
void bin_sequence_async(const lmrs_frame* f, const FrameDims& d, const Scratch& s, hipStream_t st) {
  launch_bin_total(f, d, s.bin, st);
  launch_view_sort(f, d, s.bin, st);
  launch_bin_count(f, d, s.bin, st);
  launch_bin_emit_sort(f, d, s.bin, st);
}

lmrs_status check_lm_args(const lmrs_frame* f, const float* beta, const float* targets,
                          const lmrs_lm_params* prm, const lmrs_render_opts* o) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(need(prm, "params"));
  LMRS_TRY(need(beta, "beta"));
  LMRS_TRY(need(targets, "targets"));
  if (f->beta != beta) return fail(LMRS_EINVAL, "frame->beta must equal beta");
  LMRS_TRY(check_render_state(f));
  LMRS_TRY(need(f->n_instances, "n_instances"));
  LMRS_TRY(need(f->color, "color"));
  LMRS_TRY(need(f->trans, "trans"));
  LMRS_TRY(need(f->last, "last"));
  LMRS_TRY(need(f->sched, "sched"));
  if (f->k < 256 && (!f->pix || !f->w)) return fail(LMRS_EINVAL, "k < 256 needs pix and w buffers");
  if (prm->sampler != LMRS_SAMPLER_UNIFORM && prm->sampler != LMRS_SAMPLER_RESIDUAL &&
      prm->sampler != LMRS_SAMPLER_GAUSSIAN)
    return fail(LMRS_EINVAL, "unknown sampler %d", prm->sampler);
  if (prm->sampler != LMRS_SAMPLER_UNIFORM && (!f->pix || !f->w))
    return fail(LMRS_EINVAL, "the weighted samplers need pix and w buffers");
  if (prm->cg_iters < 0 || prm->cg_iters_late < 0) return fail(LMRS_EINVAL, "cg_iters must be >= 0");
  if (!(prm->lambda >= 0.f)) return fail(LMRS_EINVAL, "lambda must be >= 0");
  if (!(prm->ssim_weight >= 0.f) || prm->ssim_weight > 1e30f)
    return fail(LMRS_EINVAL, "ssim_weight must be finite and >= 0");
  if (prm->ssim_weight > 0.f && (!f->wc || !f->image))
    return fail(LMRS_EINVAL, "ssim_weight > 0 needs the frame's wc and image buffers");
  return LMRS_OK;
}

// Alg. 1 after binning: samples, render, residuals, b, preconditioner, PCG,
// learning rate and update. Enqueue only (no host synchronisation).
void solve_sequence(const lmrs_frame* f_in, const FrameDims& d, float* beta, const float* targets,
                    const float* dvec, const lmrs_lm_params& prm, const lmrs_render_opts& o, float* report,
                    const Scratch& s, hipStream_t st) {
  const int64_t P = (int64_t)d.n * d.pg;
  // the operator takes per-channel weights only from this step's SSIM residual
  const bool ssim = prm.ssim_weight > 0.f;
  lmrs_frame fc = *f_in;
  if (!ssim) fc.wc = nullptr;
  const lmrs_frame* f = &fc;
  if (prm.sampler == LMRS_SAMPLER_RESIDUAL) {
    launch_render_scores(f, d, o, targets, s.scores, st);
    launch_sample_residual(f, d, s.scores, prm.seed, prm.iter, st);
  } else if (prm.sampler == LMRS_SAMPLER_GAUSSIAN) {
    launch_render_counts(f, d, o, s.scores, st);
    launch_sample_gaussian(f, d, s.scores, prm.seed, prm.iter, st);
  } else if (f->pix) {
    launch_sample_uniform(f, d, prm.seed, prm.iter, st);
  }
  launch_render(f, d, o, st);
  if (ssim) {
    launch_render_image(f, d, o, f->image, st);
    launch_ssim(f, d, targets, prm.ssim_weight, s.wr, s.tile_loss, s.red + 2 * kRedBlocks, report, st);
  } else {
    launch_residual(f, d, targets, s.wr, s.red, report, st);
  }
  vjp_diag_sequence(f, d, o, s.wr, s.b, s.diag, s, st);
  // CG schedule (Sec. 5): cg_iters_late GN products from iteration late_iter on
  const bool late = prm.cg_iters_late > 0 && prm.late_iter > 0 && prm.iter >= prm.late_iter;
  const int cg = late ? prm.cg_iters_late : prm.cg_iters;
  pcg_sequence(f, d, o, s.b, prm.lambda, dvec, cg, s.x, report, s, st, true, true);
  const PcgState ps{s.x, s.r, s.z, s.p, s.u, s.minv, s.sc, s.red};
  launch_lm_update(beta, s.x, d.n, P, prm, pcg_fail_slot(cg, ps), s.red, report, st);
  if (report)
    launch_report_count(f->n_instances, f->capacity, report, st,
                        f->blend_k ? f->blend_start + (int64_t)d.V * d.T : nullptr);
}

}  // namespace

lmrs_status report_error(lmrs_status s, const char* msg) { return fail(s, "%s", msg); }

FrameDims dims_of(const lmrs_frame* f) {
  FrameDims d;
  d.n = f->n;
  d.deg = f->sh_degree;
  d.pg = 11 + 3 * (f->sh_degree + 1) * (f->sh_degree + 1);
  d.V = f->n_views;
  d.W = f->width;
  d.H = f->height;
  d.TX = f->width / kTile;
  d.TY = f->height / kTile;
  d.T = d.TX * d.TY;
  d.k = f->k;
  d.S = (int64_t)d.V * d.T * d.k;
  d.det = f->deterministic != 0;
  return d;
}

// ------------------------------------------------------------ no-alloc GN
// Scratch memory of lmrs_gn_product_noalloc: one array per GPU, loaded with
// the code object and held until the process ends, shared by every call on
// that GPU. Host code never passes the array's name to a kernel (on the host
// it is only a stand-in for the symbol): it takes the array's device address
// from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kNoAllocDevices = 64;

}  // namespace lmrs

static __device__ __align__(256) unsigned char scratch[lmrs::kNoAllocBytes];

namespace lmrs {
namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocDevices] = {};

// Device address of the current device's scratch array.
lmrs_status noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return hip_check("hipGetDevice");
  if (dev < 0 || dev >= kNoAllocDevices) return fail(LMRS_EUNSUPPORTED, "device %d: scratch kept for %d devices", dev,
                                                      kNoAllocDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail(LMRS_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LMRS_OK;
}

}  // namespace
}  // namespace lmrs

using namespace lmrs;

extern "C" {

const char* lmrs_status_str(lmrs_status s) {
  switch (s) {
    case LMRS_OK: return "ok";
    case LMRS_EINVAL: return "invalid argument";
    case LMRS_ECAPACITY: return "tile-list capacity exceeded";
    case LMRS_EWORKSPACE: return "workspace too small";
    case LMRS_EHIP: return "HIP runtime error";
    case LMRS_ENUMERIC: return "numeric failure on the device";
    case LMRS_EUNSUPPORTED: return "not supported by this library";
    default: return "unknown status";
  }
}

const char* lmrs_last_error(void) { return g_err; }

lmrs_status lmrs_report_status(const float* report) {
  if (!report) return fail(LMRS_EINVAL, "report is NULL");
  const float st = report[LMRS_REP_STATUS];
  if (st == 0.f) return LMRS_OK;
  const int bits = (int)st;
  if (bits & LMRS_FAIL_CAPACITY)
    return fail(LMRS_ECAPACITY, "tile lists needed %.0f entries, more than the capacity", (double)report[LMRS_REP_INST]);
  return fail(LMRS_ENUMERIC, "numeric failure on the device:%s%s (status %g)",
              (bits & LMRS_FAIL_NONFINITE) ? " non-finite values" : "",
              (bits & LMRS_FAIL_BREAKDOWN) ? " PCG breakdown (p^T A p <= 0)" : "", (double)st);
}

size_t lmrs_workspace_bytes(int32_t op, const lmrs_frame* f) {
  if (!f || f->n <= 0 || f->n_views <= 0 || f->width <= 0 || f->height <= 0) return 0;
  FrameDims d = dims_of(f);
  if (d.k < 1) d.k = 1;
  d.S = (int64_t)d.V * d.T * d.k;
  Carver c(nullptr);
  carve(op, d, f->capacity > 0 ? f->capacity : 0, c);
  return c.used;
}

lmrs_status lmrs_project(const lmrs_frame* f, const lmrs_render_opts* o, void* stream) {
  LMRS_TRY(check_frame(f, false));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(need(f->cams, "cams"));
  LMRS_TRY(need(f->rec, "rec"));
  LMRS_TRY(need(f->rect, "rect"));
  launch_project(f, dims_of(f), *o, (hipStream_t)stream);
  return hip_check("lmrs_project");
}

lmrs_status lmrs_bin_tiles(const lmrs_frame* f, void* ws, size_t ws_bytes, void* stream) {
  LMRS_TRY(check_frame(f, false));
  LMRS_TRY(need(f->rec, "rec"));
  LMRS_TRY(need(f->rect, "rect"));
  LMRS_TRY(need(f->tile_start, "tile_start"));
  LMRS_TRY(need(f->n_instances, "n_instances"));
  if (f->capacity > 0) LMRS_TRY(need(f->ids, "ids"));
  LMRS_TRY(check_ws(LMRS_OP_BIN, f, ws, ws_bytes));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_BIN, d, f->capacity, c);
  return bin_sequence(f, d, s, (hipStream_t)stream);
}

lmrs_status lmrs_render(const lmrs_frame* f, const lmrs_render_opts* o, void* stream) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_render_state(f));
  LMRS_TRY(need(f->color, "color"));
  LMRS_TRY(need(f->trans, "trans"));
  LMRS_TRY(need(f->last, "last"));
  LMRS_TRY(need(f->sched, "sched"));
  launch_render(f, dims_of(f), *o, (hipStream_t)stream);
  return hip_check("lmrs_render");
}

lmrs_status lmrs_jvp(const lmrs_frame* f, const lmrs_render_opts* o, const float* p, float* jp, void* ws,
                     size_t ws_bytes, void* stream) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_deriv_state(f));
  LMRS_TRY(need(p, "p"));
  LMRS_TRY(need(jp, "jp"));
  LMRS_TRY(check_ws(LMRS_OP_JVP, f, ws, ws_bytes));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_JVP, d, f->capacity, c);
  hipStream_t st = (hipStream_t)stream;
  launch_tangent(f, d, *o, p, s.tan, st);
  launch_deriv(1, f, d, *o, s.tan, nullptr, jp, nullptr, st);
  return hip_check("lmrs_jvp");
}

lmrs_status lmrs_vjp(const lmrs_frame* f, const lmrs_render_opts* o, const float* u, float* out, void* ws,
                     size_t ws_bytes, void* stream) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_deriv_state(f));
  LMRS_TRY(need(u, "u"));
  LMRS_TRY(need(out, "out"));
  LMRS_TRY(check_ws(LMRS_OP_VJP, f, ws, ws_bytes));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_VJP, d, f->capacity, c);
  vjp_sequence(f, d, *o, u, out, s, (hipStream_t)stream);
  return hip_check("lmrs_vjp");
}

lmrs_status lmrs_gn_product(const lmrs_frame* f, const lmrs_render_opts* o, const float* p, float lambda,
                            const float* dvec, float* out, void* ws, size_t ws_bytes, void* stream) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_deriv_state(f));
  LMRS_TRY(need(p, "p"));
  LMRS_TRY(need(out, "out"));
  if (p == out) return fail(LMRS_EINVAL, "p and out must not alias");
  LMRS_TRY(check_ws(LMRS_OP_GN, f, ws, ws_bytes));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_GN, d, f->capacity, c);
  gn_sequence(f, d, *o, p, lambda, dvec, out, s, (hipStream_t)stream);
  return hip_check("lmrs_gn_product");
}

lmrs_status lmrs_gn_product_timed(const lmrs_frame* f, const lmrs_render_opts* o, const float* p,
                                  float lambda, const float* dvec, float* out, void* ws, size_t ws_bytes,
                                  void* stream, float* ms) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_deriv_state(f));
  LMRS_TRY(need(p, "p"));
  LMRS_TRY(need(out, "out"));
  LMRS_TRY(need(ms, "ms"));
  if (p == out) return fail(LMRS_EINVAL, "p and out must not alias");
  LMRS_TRY(check_ws(LMRS_OP_GN, f, ws, ws_bytes));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_GN, d, f->capacity, c);
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev[6];
  for (int i = 0; i < 6; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) return hip_check("hipEventCreate");
  (void)hipEventRecord(ev[0], st);
  launch_tangent(f, d, *o, p, s.tan, st);
  (void)hipEventRecord(ev[1], st);
  launch_fill(s.grad2d, grad_floats(d), 0.f, st);
  (void)hipEventRecord(ev[2], st);
  launch_blend_gn(f, d, *o, s.tan, s.grad2d, st);
  (void)hipEventRecord(ev[3], st);
  launch_deriv(3, f, d, *o, s.tan, nullptr, nullptr, s.grad2d, st);
  (void)hipEventRecord(ev[4], st);
  launch_chain_vjp(f, d, *o, s.grad2d, p, lambda, dvec, out, st);
  (void)hipEventRecord(ev[5], st);
  lmrs_status status = LMRS_OK;
  if (hipEventSynchronize(ev[5]) != hipSuccess) status = hip_check("hipEventSynchronize");
  for (int i = 0; i < 5 && status == LMRS_OK; ++i)
    if (hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]) != hipSuccess) status = hip_check("hipEventElapsedTime");
  for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
  if (status != LMRS_OK) return status;
  return hip_check("lmrs_gn_product_timed");
}

lmrs_status lmrs_walk_counts(const lmrs_frame* f, const lmrs_render_opts* o, int64_t* counts, void* stream) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_deriv_state(f));
  LMRS_TRY(need(counts, "counts"));
  launch_walk_counts(f, dims_of(f), *o, counts, (hipStream_t)stream);
  return hip_check("lmrs_walk_counts");
}

lmrs_status lmrs_linearize(const lmrs_frame* f, const lmrs_render_opts* o, void* stream) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_deriv_state(f));
  if (!f->blend_k) return fail(LMRS_EINVAL, "lmrs_linearize: the frame has no blend table (blend_k is NULL)");
  launch_gram(f, dims_of(f), *o, nullptr, nullptr, nullptr, (hipStream_t)stream, false);
  return hip_check("lmrs_linearize");
}

lmrs_status lmrs_gn_diag(const lmrs_frame* f, const lmrs_render_opts* o, float* out, void* ws,
                         size_t ws_bytes, void* stream) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_deriv_state(f));
  LMRS_TRY(need(out, "out"));
  LMRS_TRY(check_ws(LMRS_OP_DIAG, f, ws, ws_bytes));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_DIAG, d, f->capacity, c);
  diag_sequence(f, d, *o, out, s, (hipStream_t)stream);
  return hip_check("lmrs_gn_diag");
}

lmrs_status lmrs_pcg(const lmrs_frame* f, const lmrs_render_opts* o, const float* b, float lambda,
                     const float* dvec, int32_t iters, float* x, float* report, void* ws, size_t ws_bytes,
                     void* stream) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_deriv_state(f));
  LMRS_TRY(need(b, "b"));
  LMRS_TRY(need(x, "x"));
  if (iters < 0) return fail(LMRS_EINVAL, "iters = %d must be >= 0", iters);
  if (!(lambda >= 0.f)) return fail(LMRS_EINVAL, "lambda must be >= 0");
  LMRS_TRY(check_ws(LMRS_OP_PCG, f, ws, ws_bytes));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_PCG, d, f->capacity, c);
  pcg_sequence(f, d, *o, b, lambda, dvec, iters, x, report, s, (hipStream_t)stream);
  return hip_check("lmrs_pcg");
}

lmrs_status lmrs_residual_scores(const lmrs_frame* f, const lmrs_render_opts* o, const float* targets,
                                 float* scores, void* stream) {
  LMRS_TRY(check_frame(f, false));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_render_state(f));
  LMRS_TRY(need(targets, "targets"));
  LMRS_TRY(need(scores, "scores"));
  launch_render_scores(f, dims_of(f), *o, targets, scores, (hipStream_t)stream);
  return hip_check("lmrs_residual_scores");
}

lmrs_status lmrs_contributor_counts(const lmrs_frame* f, const lmrs_render_opts* o, float* counts, void* stream) {
  LMRS_TRY(check_frame(f, false));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_render_state(f));
  LMRS_TRY(need(counts, "counts"));
  launch_render_counts(f, dims_of(f), *o, counts, (hipStream_t)stream);
  return hip_check("lmrs_contributor_counts");
}

lmrs_status lmrs_ssim_residual(const lmrs_frame* f, const lmrs_render_opts* o, const float* targets, float s,
                               float* u, double* tile_loss, void* stream) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_render_state(f));
  LMRS_TRY(need(targets, "targets"));
  LMRS_TRY(need(u, "u"));
  LMRS_TRY(need(f->wc, "wc"));
  LMRS_TRY(need(f->image, "image"));
  if (!(s >= 0.f) || s > 1e30f) return fail(LMRS_EINVAL, "s must be finite and >= 0");
  const FrameDims d = dims_of(f);
  launch_render_image(f, d, *o, f->image, (hipStream_t)stream);
  launch_ssim(f, d, targets, s, u, tile_loss, nullptr, nullptr, (hipStream_t)stream);
  return hip_check("lmrs_ssim_residual");
}

lmrs_status lmrs_sample(const lmrs_frame* f, int32_t sampler, uint64_t seed, int32_t iter, const float* scores,
                        void* stream) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(f->pix, "pix"));
  LMRS_TRY(need(f->w, "w"));
  const FrameDims d = dims_of(f);
  if (sampler == LMRS_SAMPLER_UNIFORM) {
    launch_sample_uniform(f, d, seed, iter, (hipStream_t)stream);
  } else if (sampler == LMRS_SAMPLER_RESIDUAL) {
    LMRS_TRY(need(scores, "scores"));
    launch_sample_residual(f, d, scores, seed, iter, (hipStream_t)stream);
  } else if (sampler == LMRS_SAMPLER_GAUSSIAN) {
    LMRS_TRY(need(scores, "scores (contributor counts)"));
    launch_sample_gaussian(f, d, scores, seed, iter, (hipStream_t)stream);
  } else {
    return fail(LMRS_EINVAL, "unknown sampler %d", sampler);
  }
  return hip_check("lmrs_sample");
}

lmrs_status lmrs_lm_step(lmrs_frame* f, float* beta, const float* targets, const float* dvec,
                         const lmrs_lm_params* prm, const lmrs_render_opts* o, float* report, void* ws,
                         size_t ws_bytes, void* stream) {
  LMRS_TRY(check_lm_args(f, beta, targets, prm, o));
  LMRS_TRY(check_ws(LMRS_OP_LM, f, ws, ws_bytes));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_LM, d, f->capacity, c);
  hipStream_t st = (hipStream_t)stream;
  launch_project(f, d, *o, st);
  LMRS_TRY(bin_sequence(f, d, s, st));
  solve_sequence(f, d, beta, targets, dvec, *prm, *o, report, s, st);
  return hip_check("lmrs_lm_step");
}

lmrs_status lmrs_bin_tiles_async(const lmrs_frame* f, void* ws, size_t ws_bytes, void* stream) {
  LMRS_TRY(check_frame(f, false));
  LMRS_TRY(need(f->rec, "rec"));
  LMRS_TRY(need(f->rect, "rect"));
  LMRS_TRY(need(f->tile_start, "tile_start"));
  LMRS_TRY(need(f->n_instances, "n_instances"));
  LMRS_TRY(need(f->ids, "ids"));
  LMRS_TRY(check_ws(LMRS_OP_BIN, f, ws, ws_bytes));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_BIN, d, f->capacity, c);
  bin_sequence_async(f, d, s, (hipStream_t)stream);
  return hip_check("lmrs_bin_tiles_async");
}

lmrs_status lmrs_lm_iterate(lmrs_frame* f, float* beta, const float* targets, const float* dvec,
                            const lmrs_lm_params* prm, const lmrs_render_opts* o, float* report, void* ws,
                            size_t ws_bytes, void* stream) {
  LMRS_TRY(check_lm_args(f, beta, targets, prm, o));
  LMRS_TRY(check_ws(LMRS_OP_LM, f, ws, ws_bytes));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_LM, d, f->capacity, c);
  hipStream_t st = (hipStream_t)stream;
  launch_project(f, d, *o, st);
  bin_sequence_async(f, d, s, st);
  solve_sequence(f, d, beta, targets, dvec, *prm, *o, report, s, st);
  return hip_check("lmrs_lm_iterate");
}

lmrs_status lmrs_lm_solve(lmrs_frame* f, float* beta, const float* targets, const float* dvec,
                          const lmrs_lm_params* prm, const lmrs_render_opts* o, float* report, void* ws,
                          size_t ws_bytes, void* stream) {
  LMRS_TRY(check_lm_args(f, beta, targets, prm, o));
  LMRS_TRY(check_ws(LMRS_OP_SOLVE, f, ws, ws_bytes));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_SOLVE, d, f->capacity, c);
  solve_sequence(f, d, beta, targets, dvec, *prm, *o, report, s, (hipStream_t)stream);
  return hip_check("lmrs_lm_solve");
}


lmrs_status lmrs_gn_product_noalloc(const lmrs_frame* f, const lmrs_render_opts* o, const float* p, float lambda,
                                    const float* dvec, float* out, void* stream) {
  LMRS_TRY(check_frame(f));
  LMRS_TRY(need(o, "opts"));
  LMRS_TRY(check_deriv_state(f));
  LMRS_TRY(need(p, "p"));
  LMRS_TRY(need(out, "out"));
  if (p == out) return fail(LMRS_EINVAL, "p and out must not alias");
  const size_t need_bytes = lmrs_workspace_bytes(LMRS_OP_GN, f);
  if (need_bytes > kNoAllocBytes)
    return fail(LMRS_EWORKSPACE,
                "lmrs_gn_product_noalloc: this frame needs %zu bytes of scratch, the static array holds %zu "
                "(views x Gaussians up to about %zu); use lmrs_gn_product with a workspace",
                need_bytes, kNoAllocBytes,
                kNoAllocBytes / ((LMRS_REC + (f->deterministic ? kFixGradFloats : kGradRow)) * sizeof(float)));
  void* ws = nullptr;
  LMRS_TRY(noalloc_scratch(&ws));
  const FrameDims d = dims_of(f);
  Carver c(ws);
  const Scratch s = carve(LMRS_OP_GN, d, f->capacity, c);
  // the tangent records are written in full; the screen-gradient rows hold
  // the previous call's values and are cleared by a fill kernel first
  gn_sequence(f, d, *o, p, lambda, dvec, out, s, (hipStream_t)stream);
  return hip_check("lmrs_gn_product_noalloc");
}

}  // extern "C"
