// FP64 CPU oracle for the LM-RS Gauss-Newton hot path (test infrastructure only).
//
// Plain, slow, obviously-correct reference for what the HIP library computes.
// Only the test-suite, the smoke check and the CPU-baseline leg of the
// benchmark load it; the product path never does. It shares no source with the
// HIP library.
//
// What it follows (arXiv 2504.12905):
//   * Gaussian primitive and covariance Sigma = R S S^T R^T        (Sec. 3, eq. 1-2)
//   * projection, depth sort, alpha blending                       (Sec. 3, eq. 3; Alg. 2)
//   * residual r = I_hat - I, normal equation (J^T J + lam I)      (Sec. 4.1, eq. 6-8)
//   * J p by forward-mode dual numbers                             (Sec. 4.2; Supp. A, Alg. 3)
//   * J^T u by reverse accumulation                                (Supp. A, "J^T v kernel")
//   * sampled operator J^T W J with weights 1/(N q)                (Sec. 4.4, eq. 12-14)
//   * Jacobi preconditioner diag(J^T W J)                          (Sec. 4.2; Supp. A)
// Rasteriser constants (alpha floor/cap, transmittance stop, low-pass, near
// plane, 3-sigma extent) are the options block; the paper defers them to 3DGS.
//
// Every floating-point computation is FP64, the discrete decisions that build
// the tile lists included: a Gaussian is listed when its camera depth exceeds
// the near plane and its footprint square of half-width ceil(3 sqrt(lambda_max))
// around the projected centre overlaps the tile; lists are ordered by camera
// depth, ties by Gaussian index. The distance of each such decision to its
// threshold (extent to the next integer, square edge to a tile edge, depth to
// the near plane) is reported as a margin.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- dual numbers
// (real, prime) pairs with the product, quotient and chain rules: the
// DualFloat of Supp. A, Alg. 3, in FP64.
struct Dual {
  double re, du;
  Dual() : re(0.0), du(0.0) {}
  Dual(double r) : re(r), du(0.0) {}  // NOLINT: constants promote implicitly
  Dual(double r, double d) : re(r), du(d) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.re + b.re, a.du + b.du); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.re - b.re, a.du - b.du); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.re * b.re, a.re * b.du + a.du * b.re); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.re / b.re, (a.du * b.re - a.re * b.du) / (b.re * b.re));
}
inline Dual operator-(Dual a) { return Dual(-a.re, -a.du); }
inline Dual exp(Dual a) {
  double e = std::exp(a.re);
  return Dual(e, e * a.du);
}
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.re);
  return Dual(s, a.du / (2.0 * s));
}
inline double exp(double a) { return std::exp(a); }
inline double sqrt(double a) { return std::sqrt(a); }
inline double re(double x) { return x; }
inline double re(const Dual& x) { return x.re; }
inline double du(double) { return 0.0; }
inline double du(const Dual& x) { return x.du; }

// ------------------------------------------------------------------ inputs
struct Opts {
  double alpha_min, alpha_max, t_min, lowpass, znear, cutoff, bg[3];
};

struct Cam {
  double R[9], t[3], fx, fy, cx, cy, campos[3];
};

constexpr int kTile = 16;
constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------- real spherical harmonics
// Real basis built from the complex harmonics Y_l^m (Condon-Shortley phase
// included): Y_{l,0} = Y_l^0, Y_{l,m} = sqrt(2) Re Y_l^m and
// Y_{l,-m} = sqrt(2) Im Y_l^m for m > 0, index l*l + l + m. Evaluated from the
// associated-Legendre recurrence on a unit direction (x, y, z):
//   Y_l^m = K_l^m Q_l^m(z) (x + i y)^m,   Q_l^m = P_l^m / sin^m(theta),
//   K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
template <class S>
void sh_basis(int deg, S x, S y, S z, S* Y) {
  auto fact = [](int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
  };
  // (x + i y)^m for m = 0..deg
  S pr[4], pi[4];
  pr[0] = S(1.0);
  pi[0] = S(0.0);
  for (int m = 1; m <= deg; ++m) {
    pr[m] = pr[m - 1] * x - pi[m - 1] * y;
    pi[m] = pr[m - 1] * y + pi[m - 1] * x;
  }
  for (int m = 0; m <= deg; ++m) {
    // Q_m^m = (-1)^m (2m-1)!!, Q_{m+1}^m = (2m+1) z Q_m^m, then the 3-term recurrence.
    double dfact = 1.0;
    for (int i = 1; i <= 2 * m - 1; i += 2) dfact *= i;
    S q_prev2(0.0), q_prev1(0.0);
    for (int l = m; l <= deg; ++l) {
      S q;
      if (l == m) {
        q = S(((m & 1) ? -1.0 : 1.0) * dfact);
      } else if (l == m + 1) {
        q = S(double(2 * m + 1)) * z * q_prev1;
      } else {
        q = (S(double(2 * l - 1)) * z * q_prev1 - S(double(l + m - 1)) * q_prev2) / S(double(l - m));
      }
      double K = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) * fact(l - m) / fact(l + m));
      if (m == 0) {
        Y[l * l + l] = S(K) * q;
      } else {
        Y[l * l + l + m] = S(std::sqrt(2.0) * K) * q * pr[m];
        Y[l * l + l - m] = S(std::sqrt(2.0) * K) * q * pi[m];
      }
      q_prev2 = q_prev1;
      q_prev1 = q;
    }
  }
}

// ------------------------------------------------------- projection (eq. 1-3)
// Screen record of one Gaussian in one view: 2-D mean (u, v), conic (inverse
// 2-D covariance, A B / B C), activated opacity and view-dependent RGB.
template <class S>
struct Rec {
  S u, v, A, B, C, o, rgb[3];
};
constexpr int kRec = 9;

template <class S>
void rec_to_array(const Rec<S>& r, S* a) {
  a[0] = r.u; a[1] = r.v; a[2] = r.A; a[3] = r.B; a[4] = r.C; a[5] = r.o;
  a[6] = r.rgb[0]; a[7] = r.rgb[1]; a[8] = r.rgb[2];
}

// prm: the P_g parameters of one Gaussian, in the order
//   mean(3) log_scale(3) quat wxyz(4) opacity_logit(1) sh[k][c] (3K).
// Returns false when the mean is not in front of the near plane.
template <class S>
bool project_cont(const S* prm, int deg, const Cam& cam, const Opts& op, Rec<S>& out,
                  double* lam_max) {
  const S mx = prm[0], my = prm[1], mz = prm[2];
  // camera-space mean t = R_w mu + t_w
  S tc[3];
  for (int i = 0; i < 3; ++i)
    tc[i] = S(cam.R[3 * i + 0]) * mx + S(cam.R[3 * i + 1]) * my + S(cam.R[3 * i + 2]) * mz +
            S(cam.t[i]);
  if (re(tc[2]) <= op.znear) return false;
  // rotation from the normalised quaternion (w, x, y, z)
  S qn = sqrt(prm[6] * prm[6] + prm[7] * prm[7] + prm[8] * prm[8] + prm[9] * prm[9]);
  S w = prm[6] / qn, x = prm[7] / qn, y = prm[8] / qn, z = prm[9] / qn;
  S Rq[9] = {S(1.0) - S(2.0) * (y * y + z * z), S(2.0) * (x * y - w * z), S(2.0) * (x * z + w * y),
             S(2.0) * (x * y + w * z), S(1.0) - S(2.0) * (x * x + z * z), S(2.0) * (y * z - w * x),
             S(2.0) * (x * z - w * y), S(2.0) * (y * z + w * x), S(1.0) - S(2.0) * (x * x + y * y)};
  // Sigma = R S S^T R^T with S = diag(exp(log_scale))   (eq. 2)
  S sc[3] = {exp(prm[3]), exp(prm[4]), exp(prm[5])};
  S Sig[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S acc(0.0);
      for (int k = 0; k < 3; ++k) acc = acc + Rq[3 * i + k] * sc[k] * sc[k] * Rq[3 * j + k];
      Sig[3 * i + j] = acc;
    }
  // EWA: Sigma_2D = J W Sigma W^T J^T + lowpass * I, J the pinhole Jacobian at t
  S inv_z = S(1.0) / tc[2];
  S J[6] = {S(cam.fx) * inv_z, S(0.0), -S(cam.fx) * tc[0] * inv_z * inv_z,
            S(0.0), S(cam.fy) * inv_z, -S(cam.fy) * tc[1] * inv_z * inv_z};
  S T[6];  // J W (2x3)
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      S acc(0.0);
      for (int k = 0; k < 3; ++k) acc = acc + J[3 * i + k] * S(cam.R[3 * k + j]);
      T[3 * i + j] = acc;
    }
  S S2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      S acc(0.0);
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc = acc + T[3 * i + k] * Sig[3 * k + l] * T[3 * j + l];
      S2[2 * i + j] = acc;
    }
  S a = S2[0] + S(op.lowpass), b = S2[1], c = S2[3] + S(op.lowpass);
  S det = a * c - b * b;
  out.A = c / det;
  out.B = -b / det;
  out.C = a / det;
  out.u = S(cam.fx) * tc[0] * inv_z + S(cam.cx);
  out.v = S(cam.fy) * tc[1] * inv_z + S(cam.cy);
  out.o = S(1.0) / (S(1.0) + exp(-prm[10]));
  // view-dependent colour 0.5 + sum_k Y_k(dir) f_k, dir from camera centre to mean
  S dx = mx - S(cam.campos[0]), dy = my - S(cam.campos[1]), dz = mz - S(cam.campos[2]);
  S dn = sqrt(dx * dx + dy * dy + dz * dz);
  dx = dx / dn; dy = dy / dn; dz = dz / dn;
  const int K = (deg + 1) * (deg + 1);
  S Y[16];
  sh_basis(deg, dx, dy, dz, Y);
  for (int ch = 0; ch < 3; ++ch) {
    S acc(0.5);
    for (int k = 0; k < K; ++k) acc = acc + Y[k] * prm[11 + 3 * k + ch];
    out.rgb[ch] = acc;
  }
  if (lam_max) {
    double ar = re(a), br = re(b), cr = re(c);
    *lam_max = 0.5 * (ar + cr) + std::sqrt(0.25 * (ar - cr) * (ar - cr) + br * br);
  }
  return true;
}

// --------------------------------------------------------- per-pixel render
// Front-to-back alpha blending of eq. 3 / Alg. 2 over a depth-sorted list.
// A Gaussian is skipped when its exponent is positive or its alpha is below
// alpha_min; alpha is capped at alpha_max (capped alphas carry no derivative);
// the walk stops before the Gaussian that would take T below t_min.
template <class S>
struct PixelOut {
  S C[3];
  S T;
  int last;        // position in the tile list of the last blended Gaussian, -1 if none
  int n_contrib;   // number of blended Gaussians
  uint64_t trace;  // hash of the discrete decisions taken along the walk
  double margin;   // smallest relative distance of a decision to its threshold
};

template <class S>
void render_pixel(const Rec<S>* const* recs, const int* list, int len, double xc, double yc,
                  const Opts& op, PixelOut<S>& po) {
  S T(1.0);
  S C[3] = {S(0.0), S(0.0), S(0.0)};
  int last = -1, nc = 0;
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
  // Decision margins: |s| for the s > 0 test, |alpha - threshold| / threshold
  // for the alpha floor and cap, |T (1 - alpha) - t_min| / t_min for the stop.
  double margin = 1e30;
  for (int i = 0; i < len; ++i) {
    const Rec<S>& r = *recs[i];
    S dx = r.u - S(xc), dy = r.v - S(yc);
    S s = S(-0.5) * (r.A * dx * dx + r.C * dy * dy) - r.B * dx * dy;
    margin = std::min(margin, std::fabs(re(s)));
    if (re(s) > 0.0) continue;
    S a = r.o * exp(s);
    margin = std::min(margin, std::fabs(re(a) - op.alpha_min) / op.alpha_min);
    margin = std::min(margin, std::fabs(re(a) - op.alpha_max) / op.alpha_max);
    bool capped = false;
    if (re(a) > op.alpha_max) {
      a = S(op.alpha_max);
      capped = true;
    }
    if (re(a) < op.alpha_min) continue;
    S Tn = T * (S(1.0) - a);
    margin = std::min(margin, std::fabs(re(Tn) - op.t_min) / op.t_min);
    if (re(Tn) < op.t_min) {
      mix(0xffffffffull);
      break;
    }
    for (int c = 0; c < 3; ++c) C[c] = C[c] + r.rgb[c] * a * T;
    T = Tn;
    last = i;
    ++nc;
    mix((uint64_t)list[i] * 2 + (capped ? 1 : 0));
  }
  for (int c = 0; c < 3; ++c) po.C[c] = C[c] + T * S(op.bg[c]);
  po.T = T;
  po.last = last;
  po.n_contrib = nc;
  po.trace = h;
  po.margin = margin;
}

// ------------------------------------------------------------------ problem
struct Problem {
  int n = 0, deg = 0, K = 1, Pg = 14, V = 0, W = 0, H = 0, TX = 0, TY = 0, T = 0;
  std::vector<double> beta;      // [P] parameters
  std::vector<Cam> cams;         // [V]
  Opts op{};
  // projection, per (view, Gaussian)
  std::vector<Rec<double>> rec;  // [V*n]
  std::vector<uint8_t> visible;  // [V*n]
  std::vector<double> depth;     // [V*n] camera-space z of the mean (the sort key)
  std::vector<int> rect;         // [V*n*4] x0, y0, x1, y1 (tile coords, end exclusive)
  std::vector<int> radius;       // [V*n]
  std::vector<double> margin_rad;  // [V*n] distance of cutoff*sqrt(lam_max) to an integer
  std::vector<double> margin_list; // [V*n] smallest distance of a list decision to its threshold
  std::vector<int> radius_all;   // [V*n] footprint radius before the image-bounds cull (0 if not projected)
  std::vector<double> ext_all;   // [V*n] cutoff * sqrt(lambda_max) (0 if not projected)
  // tile lists
  std::vector<int64_t> tile_start;  // [V*T+1]
  std::vector<int> ids;
  // samples (k per tile); empty pix => all 256 pixels in order
  int k = 256;
  std::vector<uint8_t> pix;      // [V*T*k]
  std::vector<double> w;         // [V*T*k]
  std::vector<uint8_t> tile_mask;  // [V*T]; empty => all tiles
  // forward-mode Jacobian of the screen record w.r.t. the P_g parameters,
  // cached per (view, Gaussian) on demand: [9][P_g]
  std::vector<int> pj_slot;        // [V*n] -> slot or -1
  std::vector<double> pj;          // [slots * 9 * P_g]

  int64_t S() const { return (int64_t)V * T * k; }
  bool tile_on(int v, int t) const { return tile_mask.empty() || tile_mask[(size_t)v * T + t]; }
  void params_of(int g, double* out) const {
    for (int j = 0; j < Pg; ++j) out[j] = beta[(size_t)j * n + g];
  }
  void pixel_of(int v, int t, int j, int* px, int* py) const {
    int p = pix.empty() ? j : pix[((size_t)v * T + t) * k + j];
    *px = (t % TX) * kTile + (p % kTile);
    *py = (t / TX) * kTile + (p / kTile);
  }
  double weight_of(int64_t i) const { return w.empty() ? 1.0 : w[(size_t)i]; }
  // per-channel weights of the GN operator (empty: weight_of for every channel)
  std::vector<double> wc;        // [V*T*k*3]
  double op_weight_of(int64_t i, int c) const { return wc.empty() ? weight_of(i) : wc[(size_t)i * 3 + c]; }
};

// Tile index floor(q / 16), clamped before the int conversion (a centre far
// outside the image gives an index far outside too).
int tile_index(double q) { return (int)std::min(std::max(std::floor(q / kTile), -1.0e6), 1.0e6); }

// Distance of q to the nearest multiple of 16 (a tile edge, in pixels).
double edge_margin(double q) {
  const double f = q / kTile;
  return std::fabs(f - std::round(f)) * kTile;
}

// Per (view, Gaussian): camera depth t_z = (R mu + t)_z, the screen record and,
// when t_z is beyond the near plane and the projected centre is finite, the
// footprint radius r = ceil(cutoff sqrt(lambda_max)) and the tile rectangle
// {tile x : 16 x <= u + r and 16 x + 16 > u - r} (same for y), clipped to the
// image; an empty rectangle means the Gaussian is listed nowhere.
void project_all(Problem& pb) {
  const size_t VN = (size_t)pb.V * pb.n;
  pb.rec.assign(VN, Rec<double>{});
  pb.visible.assign(VN, 0);
  pb.depth.assign(VN, 0.0);
  pb.rect.assign(VN * 4, 0);
  pb.radius.assign(VN, 0);
  pb.margin_rad.assign(VN, 1.0);
  pb.margin_list.assign(VN, 1e30);
  pb.radius_all.assign(VN, 0);
  pb.ext_all.assign(VN, 0.0);
#pragma omp parallel for schedule(static)
  for (long long vg = 0; vg < (long long)VN; ++vg) {
    const int v = (int)(vg / pb.n), g = (int)(vg % pb.n);
    double prm[11 + 48];
    pb.params_of(g, prm);
    const Cam& c = pb.cams[v];
    double tc[3];
    for (int i = 0; i < 3; ++i)
      tc[i] = c.R[3 * i + 0] * prm[0] + c.R[3 * i + 1] * prm[1] + c.R[3 * i + 2] * prm[2] + c.t[i];
    pb.depth[vg] = tc[2];
    pb.margin_list[vg] = std::fabs(tc[2] - pb.op.znear);
    Rec<double> r;
    double lam = 0.0;
    if (!project_cont(prm, pb.deg, c, pb.op, r, &lam)) continue;  // t_z <= znear
    if (!std::isfinite(r.u) || !std::isfinite(r.v)) continue;
    pb.rec[vg] = r;
    const double ext = pb.op.cutoff * std::sqrt(lam);
    const double rad_d = std::ceil(ext);
    pb.margin_rad[vg] = std::min(ext - std::floor(ext), std::ceil(ext) - ext);
    pb.ext_all[vg] = ext;
    if (!(rad_d < 1e6)) continue;
    const int rad = (int)rad_d;
    pb.radius_all[vg] = rad;
    const double lo_x = r.u - rad, hi_x = r.u + rad, lo_y = r.v - rad, hi_y = r.v + rad;
    pb.margin_list[vg] = std::min({pb.margin_list[vg], pb.margin_rad[vg], edge_margin(lo_x), edge_margin(hi_x),
                                   edge_margin(lo_y), edge_margin(hi_y)});
    int x0 = tile_index(lo_x), x1 = tile_index(hi_x);
    int y0 = tile_index(lo_y), y1 = tile_index(hi_y);
    x0 = std::max(x0, 0); y0 = std::max(y0, 0);
    x1 = std::min(x1, pb.TX - 1); y1 = std::min(y1, pb.TY - 1);
    if (x0 > x1 || y0 > y1) continue;
    pb.visible[vg] = 1;
    pb.radius[vg] = rad;
    int* rc = &pb.rect[vg * 4];
    rc[0] = x0; rc[1] = y0; rc[2] = x1 + 1; rc[3] = y1 + 1;
  }
}

// Tile lists: every visible Gaussian whose tile rectangle holds the tile,
// ascending camera depth, ties by ascending Gaussian index. With `only`
// (uint8 [V*T]), the lists of the other tiles are left empty (a cheaper setup
// for checks restricted to a few tiles; the listed tiles are unchanged).
void bin_all(Problem& pb, const uint8_t* only = nullptr) {
  std::vector<std::vector<std::pair<double, int>>> lists((size_t)pb.V * pb.T);
  for (int v = 0; v < pb.V; ++v)
    for (int g = 0; g < pb.n; ++g) {
      const size_t vg = (size_t)v * pb.n + g;
      if (!pb.visible[vg]) continue;
      const int* rc = &pb.rect[vg * 4];
      for (int ty = rc[1]; ty < rc[3]; ++ty)
        for (int tx = rc[0]; tx < rc[2]; ++tx) {
          const size_t t = (size_t)v * pb.T + ty * pb.TX + tx;
          if (!only || only[t]) lists[t].push_back({pb.depth[vg], g});
        }
    }
  pb.tile_start.assign((size_t)pb.V * pb.T + 1, 0);
  for (size_t i = 0; i < lists.size(); ++i) pb.tile_start[i + 1] = pb.tile_start[i] + lists[i].size();
  pb.ids.assign(pb.tile_start.back(), 0);
#pragma omp parallel for schedule(dynamic, 16)
  for (long long i = 0; i < (long long)lists.size(); ++i) {
    auto& L = lists[i];
    std::sort(L.begin(), L.end());
    for (size_t j = 0; j < L.size(); ++j) pb.ids[pb.tile_start[i] + j] = L[j].second;
  }
}

void setup(Problem& pb, int n, int deg, const double* beta, int V, const float* cams, int W, int H,
           const double* opts, const uint8_t* only = nullptr) {
  pb.n = n; pb.deg = deg; pb.K = (deg + 1) * (deg + 1); pb.Pg = 11 + 3 * pb.K;
  pb.V = V; pb.W = W; pb.H = H; pb.TX = W / kTile; pb.TY = H / kTile; pb.T = pb.TX * pb.TY;
  pb.beta.assign(beta, beta + (size_t)n * pb.Pg);
  pb.op = Opts{opts[0], opts[1], opts[2], opts[3], opts[4], opts[5], {opts[6], opts[7], opts[8]}};
  pb.cams.resize(V);
  for (int v = 0; v < V; ++v) {
    const float* c = cams + 16 * v;
    Cam& k = pb.cams[v];
    for (int i = 0; i < 9; ++i) k.R[i] = c[i];
    for (int i = 0; i < 3; ++i) k.t[i] = c[9 + i];
    k.fx = c[12]; k.fy = c[13]; k.cx = c[14]; k.cy = c[15];
    for (int i = 0; i < 3; ++i)  // camera centre -R^T t
      k.campos[i] = -(k.R[0 + i] * k.t[0] + k.R[3 + i] * k.t[1] + k.R[6 + i] * k.t[2]);
  }
  project_all(pb);
  bin_all(pb, only);
  pb.pj_slot.assign((size_t)V * n, -1);
  pb.pj.clear();
}

// Forward-mode Jacobian d rec / d prm of one (view, Gaussian): P_g dual passes.
void proj_jacobian(const Problem& pb, int v, int g, double* J /*9 x Pg*/) {
  double prm[11 + 48];
  pb.params_of(g, prm);
  Dual d[11 + 48];
  for (int j = 0; j < pb.Pg; ++j) {
    for (int i = 0; i < pb.Pg; ++i) d[i] = Dual(prm[i], i == j ? 1.0 : 0.0);
    Rec<Dual> r;
    project_cont(d, pb.deg, pb.cams[v], pb.op, r, nullptr);
    Dual a[kRec];
    rec_to_array(r, a);
    for (int q = 0; q < kRec; ++q) J[q * pb.Pg + j] = a[q].du;
  }
}

// Make sure the Jacobians of every (view, Gaussian) listed in an active tile exist.
void ensure_jacobians(Problem& pb) {
  std::vector<int> need;
  std::vector<uint8_t> mark((size_t)pb.V * pb.n, 0);
  for (int v = 0; v < pb.V; ++v)
    for (int t = 0; t < pb.T; ++t) {
      if (!pb.tile_on(v, t)) continue;
      const size_t ti = (size_t)v * pb.T + t;
      for (int64_t e = pb.tile_start[ti]; e < pb.tile_start[ti + 1]; ++e) {
        const size_t vg = (size_t)v * pb.n + pb.ids[e];
        if (!mark[vg] && pb.pj_slot[vg] < 0) { mark[vg] = 1; need.push_back((int)vg); }
      }
    }
  const size_t base = pb.pj.size() / ((size_t)kRec * pb.Pg);
  pb.pj.resize((base + need.size()) * kRec * pb.Pg);
  for (size_t i = 0; i < need.size(); ++i) pb.pj_slot[need[i]] = (int)(base + i);
#pragma omp parallel for schedule(dynamic, 64)
  for (long long i = 0; i < (long long)need.size(); ++i) {
    const int vg = need[i];
    proj_jacobian(pb, vg / pb.n, vg % pb.n, &pb.pj[(base + i) * kRec * pb.Pg]);
  }
}

// Gather the per-list-entry record pointers of one tile.
template <class S>
void tile_recs(const Problem& pb, const std::vector<Rec<S>>& recs, int v, int t,
               std::vector<const Rec<S>*>& ptrs, const int** list, int* len) {
  const size_t ti = (size_t)v * pb.T + t;
  const int64_t a = pb.tile_start[ti], b = pb.tile_start[ti + 1];
  ptrs.resize(b - a);
  for (int64_t e = a; e < b; ++e) ptrs[e - a] = &recs[(size_t)v * pb.n + pb.ids[e]];
  *list = pb.ids.data() + a;
  *len = (int)(b - a);
}

template <class S>
void walk_all(const Problem& pb, const std::vector<Rec<S>>& recs, double* C, double* Cdu, double* T,
              int* last, int* ncontrib, uint64_t* trace, double* margin = nullptr) {
#pragma omp parallel
  {
    std::vector<const Rec<S>*> ptrs;
#pragma omp for schedule(dynamic, 4)
    for (long long vt = 0; vt < (long long)pb.V * pb.T; ++vt) {
      const int v = (int)(vt / pb.T), t = (int)(vt % pb.T);
      if (!pb.tile_on(v, t)) continue;
      const int* list;
      int len;
      tile_recs(pb, recs, v, t, ptrs, &list, &len);
      for (int j = 0; j < pb.k; ++j) {
        int px, py;
        pb.pixel_of(v, t, j, &px, &py);
        PixelOut<S> po;
        render_pixel(ptrs.data(), list, len, px + 0.5, py + 0.5, pb.op, po);
        const int64_t i = vt * pb.k + j;
        for (int c = 0; c < 3; ++c) {
          if (C) C[3 * i + c] = re(po.C[c]);
          if (Cdu) Cdu[3 * i + c] = du(po.C[c]);
        }
        if (T) T[i] = re(po.T);
        if (last) last[i] = po.last;
        if (ncontrib) ncontrib[i] = po.n_contrib;
        if (trace) trace[i] = po.trace;
        if (margin) margin[i] = po.margin;
      }
    }
  }
}

// Records carrying the tangent d rec = (d rec / d beta) p, by dual-number projection.
void dual_records(const Problem& pb, const double* p, std::vector<Rec<Dual>>& drec) {
  drec.assign((size_t)pb.V * pb.n, Rec<Dual>{});
#pragma omp parallel for schedule(static)
  for (long long vg = 0; vg < (long long)pb.V * pb.n; ++vg) {
    if (!pb.visible[vg]) continue;
    const int v = (int)(vg / pb.n), g = (int)(vg % pb.n);
    double prm[11 + 48];
    pb.params_of(g, prm);
    Dual d[11 + 48];
    for (int j = 0; j < pb.Pg; ++j) d[j] = Dual(prm[j], p[(size_t)j * pb.n + g]);
    project_cont(d, pb.deg, pb.cams[v], pb.op, drec[vg], nullptr);
  }
}

// Reverse accumulation through one pixel's blend: for weight vector u (3),
// add d(u . C)/d rec_n into grad[list entry] (9 per entry), back to front.
// Also, if gch is non-null, store per-channel derivatives d C_c / d rec_n for
// each blended entry (used by the diagonal).
struct Blended {
  int pos;         // list position
  double a, T, es, dx, dy;
  bool capped;
};

void blend_trace(const Problem& pb, const Rec<double>* const* recs, int len, double xc, double yc,
                 std::vector<Blended>& out, double* Tfinal) {
  out.clear();
  double T = 1.0;
  for (int i = 0; i < len; ++i) {
    const Rec<double>& r = *recs[i];
    double dx = r.u - xc, dy = r.v - yc;
    double s = -0.5 * (r.A * dx * dx + r.C * dy * dy) - r.B * dx * dy;
    if (s > 0.0) continue;
    double es = std::exp(s);
    double a = r.o * es;
    bool capped = false;
    if (a > pb.op.alpha_max) { a = pb.op.alpha_max; capped = true; }
    if (a < pb.op.alpha_min) continue;
    double Tn = T * (1.0 - a);
    if (Tn < pb.op.t_min) break;
    out.push_back({i, a, T, es, dx, dy, capped});
    T = Tn;
  }
  *Tfinal = T;
}

// d(u . C)/d rec for each blended entry, with C = sum_n rgb_n a_n T_n + T_final bg.
//   d/d rgb_n   = u a_n T_n
//   d/d a_n     = T_n (u . rgb_n) - (u . (sum_{m>n} rgb_m a_m T_m + T_final bg)) / (1 - a_n)
//   a_n = o_n exp(s_n) unless capped; s_n = -1/2 (A dx^2 + C dy^2) - B dx dy, dx = u_n - x.
void pixel_adjoint(const Problem& pb, const Rec<double>* const* recs, const std::vector<Blended>& bl,
                   double Tfinal, const double* u, double* grad /*[len][9]*/) {
  double behind = Tfinal * (u[0] * pb.op.bg[0] + u[1] * pb.op.bg[1] + u[2] * pb.op.bg[2]);
  for (int q = (int)bl.size() - 1; q >= 0; --q) {
    const Blended& b = bl[q];
    const Rec<double>& r = *recs[b.pos];
    const double urgb = u[0] * r.rgb[0] + u[1] * r.rgb[1] + u[2] * r.rgb[2];
    const double ga = b.T * urgb - behind / (1.0 - b.a);
    behind += urgb * b.a * b.T;
    double* g = grad + (size_t)b.pos * kRec;
    for (int c = 0; c < 3; ++c) g[6 + c] += u[c] * b.a * b.T;
    if (b.capped) continue;
    const double gs = ga * b.a;  // d/d s
    g[5] += ga * b.es;           // d/d o
    g[0] += gs * (-(r.A * b.dx + r.B * b.dy));
    g[1] += gs * (-(r.B * b.dx + r.C * b.dy));
    g[2] += gs * (-0.5 * b.dx * b.dx);
    g[3] += gs * (-b.dx * b.dy);
    g[4] += gs * (-0.5 * b.dy * b.dy);
  }
}

// grad_rec[v][g][9] = sum over active pixels of d(u_i . C_i)/d rec_{v,g}
void screen_adjoint(const Problem& pb, const double* u, std::vector<double>& grad_rec) {
  const size_t VN = (size_t)pb.V * pb.n;
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  std::vector<std::vector<double>> part(nth);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    std::vector<double>& acc = part[tid];
    acc.assign(VN * kRec, 0.0);
    std::vector<const Rec<double>*> ptrs;
    std::vector<Blended> bl;
    std::vector<double> g;
#pragma omp for schedule(dynamic, 4)
    for (long long vt = 0; vt < (long long)pb.V * pb.T; ++vt) {
      const int v = (int)(vt / pb.T), t = (int)(vt % pb.T);
      if (!pb.tile_on(v, t)) continue;
      const int* list;
      int len;
      tile_recs(pb, pb.rec, v, t, ptrs, &list, &len);
      g.assign((size_t)len * kRec, 0.0);
      for (int j = 0; j < pb.k; ++j) {
        const int64_t i = vt * pb.k + j;
        const double* ui = u + 3 * i;
        if (ui[0] == 0.0 && ui[1] == 0.0 && ui[2] == 0.0) continue;
        int px, py;
        pb.pixel_of(v, t, j, &px, &py);
        double Tf;
        blend_trace(pb, ptrs.data(), len, px + 0.5, py + 0.5, bl, &Tf);
        pixel_adjoint(pb, ptrs.data(), bl, Tf, ui, g.data());
      }
      for (int e = 0; e < len; ++e) {
        double* dst = &acc[((size_t)v * pb.n + list[e]) * kRec];
        for (int q = 0; q < kRec; ++q) dst[q] += g[(size_t)e * kRec + q];
      }
    }
  }
  grad_rec.assign(VN * kRec, 0.0);
  for (int th = 0; th < nth; ++th)
    if (!part[th].empty())
      for (size_t i = 0; i < VN * kRec; ++i) grad_rec[i] += part[th][i];
}

// Magnitude of the terms J^T u is summed from, as the method forms it: the
// adjoint of pixel_adjoint with every quantity replaced by the sum of the
// magnitudes of the terms it is made of (u . rgb by sum_c |u_c||rgb_c|, the
// colour behind by the sum of its terms, d/d a_n by
// T_n |u.rgb| + |behind| / (1 - a_n), d/d s by that times a_n and the conic
// and offset factors by their magnitudes), summed over pixels per (view,
// Gaussian) and record component; then per parameter the sum over views and
// record components of |d rec / d beta| times that. It bounds |J^T u| and
// |J|^T |u| entry by entry and scales the rounding error of an evaluation in
// this order, cancellation inside d/d a_n included (a test scale, not part of
// the method).
void pixel_adjoint_abs(const Problem& pb, const Rec<double>* const* recs, const std::vector<Blended>& bl,
                       double Tfinal, const double* u, double* grad /*[len][9]*/) {
  const double au[3] = {std::fabs(u[0]), std::fabs(u[1]), std::fabs(u[2])};
  double behind = Tfinal * (au[0] * std::fabs(pb.op.bg[0]) + au[1] * std::fabs(pb.op.bg[1]) +
                            au[2] * std::fabs(pb.op.bg[2]));
  for (int q = (int)bl.size() - 1; q >= 0; --q) {
    const Blended& b = bl[q];
    const Rec<double>& r = *recs[b.pos];
    const double urgb = au[0] * std::fabs(r.rgb[0]) + au[1] * std::fabs(r.rgb[1]) + au[2] * std::fabs(r.rgb[2]);
    const double ga = b.T * urgb + behind / (1.0 - b.a);
    behind += urgb * b.a * b.T;
    double* g = grad + (size_t)b.pos * kRec;
    for (int c = 0; c < 3; ++c) g[6 + c] += au[c] * b.a * b.T;
    if (b.capped) continue;
    const double gs = ga * b.a;
    g[5] += ga * b.es;
    g[0] += gs * (std::fabs(r.A * b.dx) + std::fabs(r.B * b.dy));
    g[1] += gs * (std::fabs(r.B * b.dx) + std::fabs(r.C * b.dy));
    g[2] += gs * (0.5 * b.dx * b.dx);
    g[3] += gs * std::fabs(b.dx * b.dy);
    g[4] += gs * (0.5 * b.dy * b.dy);
  }
}

void screen_adjoint_abs(const Problem& pb, const double* u, std::vector<double>& grad_rec) {
  const size_t VN = (size_t)pb.V * pb.n;
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  std::vector<std::vector<double>> part(nth);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    std::vector<double>& acc = part[tid];
    acc.assign(VN * kRec, 0.0);
    std::vector<const Rec<double>*> ptrs;
    std::vector<Blended> bl;
    std::vector<double> g;
#pragma omp for schedule(dynamic, 4)
    for (long long vt = 0; vt < (long long)pb.V * pb.T; ++vt) {
      const int v = (int)(vt / pb.T), t = (int)(vt % pb.T);
      if (!pb.tile_on(v, t)) continue;
      const int* list;
      int len;
      tile_recs(pb, pb.rec, v, t, ptrs, &list, &len);
      for (int j = 0; j < pb.k; ++j) {
        const int64_t i = vt * pb.k + j;
        const double* ui = u + 3 * i;
        int px, py;
        pb.pixel_of(v, t, j, &px, &py);
        double Tf;
        blend_trace(pb, ptrs.data(), len, px + 0.5, py + 0.5, bl, &Tf);
        if (ui[0] == 0.0 && ui[1] == 0.0 && ui[2] == 0.0) continue;
        g.assign((size_t)len * kRec, 0.0);
        pixel_adjoint_abs(pb, ptrs.data(), bl, Tf, ui, g.data());
        for (const Blended& b : bl) {
          double* dst = &acc[((size_t)v * pb.n + list[b.pos]) * kRec];
          const double* src = &g[(size_t)b.pos * kRec];
          for (int q = 0; q < kRec; ++q) dst[q] += src[q];
        }
      }
    }
  }
  grad_rec.assign(VN * kRec, 0.0);
  for (int th = 0; th < nth; ++th)
    if (!part[th].empty())
      for (size_t i = 0; i < VN * kRec; ++i) grad_rec[i] += part[th][i];
}

// out[beta_g] = sum_v (d rec_{v,g} / d beta_g)^T grad_rec[v][g]
void chain_to_params(Problem& pb, const std::vector<double>& grad_rec, double* out, bool abs_terms = false) {
  ensure_jacobians(pb);
  const size_t P = (size_t)pb.n * pb.Pg;
  std::fill(out, out + P, 0.0);
#pragma omp parallel for schedule(static)
  for (long long g = 0; g < pb.n; ++g) {
    for (int v = 0; v < pb.V; ++v) {
      const size_t vg = (size_t)v * pb.n + g;
      const double* gr = &grad_rec[vg * kRec];
      bool any = false;
      for (int q = 0; q < kRec; ++q) any |= gr[q] != 0.0;
      if (!any) continue;
      const int slot = pb.pj_slot[vg];
      if (slot < 0) continue;  // not listed in any active tile => zero gradient
      const double* J = &pb.pj[(size_t)slot * kRec * pb.Pg];
      for (int j = 0; j < pb.Pg; ++j) {
        double acc = 0.0;
        for (int q = 0; q < kRec; ++q) acc += abs_terms ? gr[q] * std::fabs(J[q * pb.Pg + j]) : gr[q] * J[q * pb.Pg + j];
        out[(size_t)j * pb.n + g] += acc;
      }
    }
  }
}

}  // namespace

// =========================================================== C interface
extern "C" {

// only: NULL, or uint8 [V*T] tiles whose lists are built (the others empty)
void* or_create(int n, int deg, const double* beta, int V, const float* cams, int W, int H,
                const double* opts, const uint8_t* only) {
  if (n < 0 || deg < 0 || deg > 3 || V <= 0 || W % kTile || H % kTile) return nullptr;
  Problem* pb = new Problem();
  setup(*pb, n, deg, beta, V, cams, W, H, opts, only);
  return pb;
}

void or_destroy(void* h) { delete static_cast<Problem*>(h); }

int64_t or_num_instances(void* h) { return (int64_t) static_cast<Problem*>(h)->ids.size(); }

// margin: per (view, Gaussian) the smallest distance of a list decision to
// its threshold (radius extent to an integer, rectangle edge to a tile edge,
// depth to the near plane); margin_rad: the radius part alone.
void or_get_projection(void* h, double* rec, double* depth, int* rect, int* radius, double* margin,
                       uint8_t* visible, double* margin_rad) {
  Problem& pb = *static_cast<Problem*>(h);
  const size_t VN = (size_t)pb.V * pb.n;
  for (size_t i = 0; i < VN; ++i) {
    if (rec) rec_to_array(pb.rec[i], rec + i * kRec);
    if (depth) depth[i] = pb.depth[i];
    if (radius) radius[i] = pb.radius[i];
    if (margin) margin[i] = pb.margin_list[i];
    if (margin_rad) margin_rad[i] = pb.margin_rad[i];
    if (visible) visible[i] = pb.visible[i];
    if (rect) std::memcpy(rect + 4 * i, &pb.rect[4 * i], 4 * sizeof(int));
  }
}

// Tiles whose list membership a less exact evaluation of the radius may
// decide differently: for every Gaussian whose extent cutoff * sqrt(lambda_max)
// lies within tau of an integer, the tiles held by its rectangle with exactly
// one of the radius r and the neighbouring radius such an evaluation may give
// instead: r - 1 when the extent lies just above the integer, r + 1 when just
// below.
void or_undecided_tiles(void* h, double tau, uint8_t* flags) {
  Problem& pb = *static_cast<Problem*>(h);
  std::fill(flags, flags + (size_t)pb.V * pb.T, (uint8_t)0);
  const size_t VN = (size_t)pb.V * pb.n;
  for (size_t vg = 0; vg < VN; ++vg) {
    if (!(pb.margin_rad[vg] < tau) || pb.radius_all[vg] <= 0) continue;
    const int v = (int)(vg / pb.n);
    const double u = pb.rec[vg].u, vv = pb.rec[vg].v;
    const double ext = pb.ext_all[vg];
    const int alt = ext - std::floor(ext) < 0.5 ? -1 : 1;
    auto tile_of = tile_index;
    int box[2][4];
    for (int k = 0; k < 2; ++k) {
      const double rf = pb.radius_all[vg] + (k == 0 ? 0 : alt);
      box[k][0] = std::max(tile_of(u - rf), 0);
      box[k][1] = std::max(tile_of(vv - rf), 0);
      box[k][2] = std::min(tile_of(u + rf), pb.TX - 1);
      box[k][3] = std::min(tile_of(vv + rf), pb.TY - 1);
    }
    const int big = alt > 0 ? 1 : 0;  // the larger of the two rectangles
    const int* o = box[big];
    const int* in = box[1 - big];
    for (int ty = o[1]; ty <= o[3]; ++ty)
      for (int tx = o[0]; tx <= o[2]; ++tx) {
        const bool inner = tx >= in[0] && tx <= in[2] && ty >= in[1] && ty <= in[3];
        if (!inner) flags[(size_t)v * pb.T + ty * pb.TX + tx] = 1;
      }
  }
}

void or_get_lists(void* h, int64_t* tile_start, int* ids) {
  Problem& pb = *static_cast<Problem*>(h);
  std::memcpy(tile_start, pb.tile_start.data(), pb.tile_start.size() * sizeof(int64_t));
  std::memcpy(ids, pb.ids.data(), pb.ids.size() * sizeof(int));
}

// k samples per tile; pix [V*T*k] pixel-in-tile indices, w [V*T*k] weights.
// pix == NULL selects all 256 pixels in row-major tile order with weight 1.
void or_set_samples(void* h, int k, const uint8_t* pix, const float* w) {
  Problem& pb = *static_cast<Problem*>(h);
  pb.k = k;
  const size_t cnt = (size_t)pb.V * pb.T * k;
  if (pix) pb.pix.assign(pix, pix + cnt); else pb.pix.clear();
  if (w) { pb.w.resize(cnt); for (size_t i = 0; i < cnt; ++i) pb.w[i] = w[i]; } else pb.w.clear();
  pb.wc.clear();
}

// Per-channel weights [S*3] of the GN operator (NULL: the sample weights).
void or_set_channel_weights(void* h, const double* wc) {
  Problem& pb = *static_cast<Problem*>(h);
  if (wc) pb.wc.assign(wc, wc + (size_t)pb.S() * 3); else pb.wc.clear();
}

void or_set_tile_mask(void* h, const uint8_t* mask) {
  Problem& pb = *static_cast<Problem*>(h);
  if (mask) pb.tile_mask.assign(mask, mask + (size_t)pb.V * pb.T); else pb.tile_mask.clear();
}

void or_render(void* h, double* C, double* T, int* last, int* ncontrib, uint64_t* trace, double* margin) {
  Problem& pb = *static_cast<Problem*>(h);
  walk_all<double>(pb, pb.rec, C, nullptr, T, last, ncontrib, trace, margin);
}

// J p at every sampled pixel (3 channels), by dual numbers.
void or_jvp(void* h, const double* p, double* jp) {
  Problem& pb = *static_cast<Problem*>(h);
  std::vector<Rec<Dual>> drec;
  dual_records(pb, p, drec);
  walk_all<Dual>(pb, drec, nullptr, jp, nullptr, nullptr, nullptr, nullptr);
}

// J^T u over the sampled pixels (u is [S][3]); out is [P].
void or_vjp(void* h, const double* u, double* out) {
  Problem& pb = *static_cast<Problem*>(h);
  std::vector<double> grad_rec;
  screen_adjoint(pb, u, grad_rec);
  chain_to_params(pb, grad_rec, out);
}

// Term magnitudes of J^T u (see screen_adjoint_abs); out is [P].
void or_vjp_abs(void* h, const double* u, double* out) {
  Problem& pb = *static_cast<Problem*>(h);
  std::vector<double> grad_rec;
  screen_adjoint_abs(pb, u, grad_rec);
  chain_to_params(pb, grad_rec, out, true);
}

// Screen-space adjoint only: grad_rec [V][n][9].
void or_vjp_screen(void* h, const double* u, double* grad_rec_out) {
  Problem& pb = *static_cast<Problem*>(h);
  std::vector<double> grad_rec;
  screen_adjoint(pb, u, grad_rec);
  std::memcpy(grad_rec_out, grad_rec.data(), grad_rec.size() * sizeof(double));
}

// Gauss-Newton product out = J^T W J p + lam d.p   (eq. 8, eq. 14)
void or_gn(void* h, const double* p, double lam, const double* d, double* out) {
  Problem& pb = *static_cast<Problem*>(h);
  const int64_t S = pb.S();
  std::vector<double> jp((size_t)S * 3, 0.0);
  or_jvp(h, p, jp.data());
  for (int64_t i = 0; i < S; ++i)
    for (int c = 0; c < 3; ++c) jp[3 * i + c] *= pb.op_weight_of(i, c);
  or_vjp(h, jp.data(), out);
  const size_t P = (size_t)pb.n * pb.Pg;
  for (size_t j = 0; j < P; ++j) out[j] += lam * (d ? d[j] : 1.0) * p[j];
}

// diag(J^T W J)_j = sum_i w_i sum_c J_{(i,c), j}^2 from the exact local blocks.
void or_diag(void* h, double* D) {
  Problem& pb = *static_cast<Problem*>(h);
  ensure_jacobians(pb);
  const size_t P = (size_t)pb.n * pb.Pg;
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  std::vector<std::vector<double>> part(nth);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    std::vector<double>& acc = part[tid];
    acc.assign(P, 0.0);
    std::vector<const Rec<double>*> ptrs;
    std::vector<Blended> bl;
    std::vector<double> g;
#pragma omp for schedule(dynamic, 4)
    for (long long vt = 0; vt < (long long)pb.V * pb.T; ++vt) {
      const int v = (int)(vt / pb.T), t = (int)(vt % pb.T);
      if (!pb.tile_on(v, t)) continue;
      const int* list;
      int len;
      tile_recs(pb, pb.rec, v, t, ptrs, &list, &len);
      for (int j = 0; j < pb.k; ++j) {
        const int64_t i = vt * pb.k + j;
        const double wi = pb.weight_of(i);
        int px, py;
        pb.pixel_of(v, t, j, &px, &py);
        double Tf;
        blend_trace(pb, ptrs.data(), len, px + 0.5, py + 0.5, bl, &Tf);
        for (int c = 0; c < 3; ++c) {
          // d C_c / d rec for every list entry, via the adjoint with u = e_c
          double u[3] = {0.0, 0.0, 0.0};
          u[c] = 1.0;
          g.assign((size_t)len * kRec, 0.0);
          pixel_adjoint(pb, ptrs.data(), bl, Tf, u, g.data());
          for (const Blended& b : bl) {
            const int gi = list[b.pos];
            const double* a = &g[(size_t)b.pos * kRec];
            const int slot = pb.pj_slot[(size_t)v * pb.n + gi];
            const double* J = &pb.pj[(size_t)slot * kRec * pb.Pg];
            for (int q = 0; q < pb.Pg; ++q) {
              double Jij = 0.0;
              for (int r = 0; r < kRec; ++r) Jij += a[r] * J[r * pb.Pg + q];
              acc[(size_t)q * pb.n + gi] += wi * Jij * Jij;
            }
          }
        }
      }
    }
  }
  std::fill(D, D + P, 0.0);
  for (int th = 0; th < nth; ++th)
    if (!part[th].empty())
      for (size_t j = 0; j < P; ++j) D[j] += part[th][j];
}

// d rec_{v,g} / d beta_g as a 9 x P_g row-major block.
void or_proj_jacobian(void* h, int v, int g, double* J) {
  proj_jacobian(*static_cast<Problem*>(h), v, g, J);
}

// Real SH basis (for pinning against a library routine).
void or_sh_basis(int deg, double x, double y, double z, double* Y) { sh_basis<double>(deg, x, y, z, Y); }

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads of the following parallel regions (the calling thread's setting).
void or_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

}  // extern "C"
