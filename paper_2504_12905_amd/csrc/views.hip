// View batches by camera clustering (Sec. 4.3): host code of the library.
//
// Every camera i gets the feature f_i = (x, y, z, dx, dy, dz): its centre
// -R^T t, moved to the mean of all centres and divided by the largest distance
// from that mean (so the positions lie in the unit ball, on the scale of the
// unit viewing directions), and its viewing direction, the camera's forward
// (+z) axis in world coordinates (the third row of the world-to-camera R).
// K-means (Lloyd's algorithm in FP64) splits the features into B clusters,
// B the batch size, and one camera is drawn from each cluster.
//
// K-means details (the paper names the method only):
// * seeding by D^2 sampling (k-means++): centre 0 is camera floor(u_0 N), centre
//   s > 0 the first camera whose running sum of D^2 (squared distance to the
//   nearest centre so far) exceeds u_s times the total; when every D^2 is 0 the
//   first camera not yet a centre;
// * then assignment to the nearest centre (ties: lower cluster index) and
//   centres to the means of their members, until no assignment changes (at
//   most 100 rounds); a cluster left empty takes the camera farthest from its
//   own centre (ties: lower camera index) and the round repeats;
// * u_s = (24-bit word of Philox4x32-10 counter (s, 0, B, 0x4b4d0001), key
//   seed) * 2^-24; the seeding depends on (cameras, B, seed) only, so the
//   clusters are the same at every LM iteration;
// * at LM iteration `iter` cluster j (members in ascending camera index, m of
//   them) gives member floor(d m / 2^24), d the 24-bit word of counter
//   (j, iter, B, 0x4b4d0002).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "launch.hpp"

namespace lmrs {
namespace {

constexpr uint32_t kSeedTag = 0x4b4d0001u;
constexpr uint32_t kPickTag = 0x4b4d0002u;
constexpr int kMaxRounds = 100;

uint32_t word24(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed) {
  const uint4 r = philox4x32_10(make_uint4(c0, c1, c2, c3), (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  return r.x >> 8;
}

double dist2(const double* a, const double* b) {
  double s = 0.0;
  for (int q = 0; q < 6; ++q) s += (a[q] - b[q]) * (a[q] - b[q]);
  return s;
}

void features(const lmrs_camera* cams, int n, std::vector<double>& f) {
  f.assign((size_t)n * 6, 0.0);
  double mean[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < n; ++i) {
    const lmrs_camera& c = cams[i];
    for (int a = 0; a < 3; ++a) {
      const double pos = -((double)c.R[a] * c.t[0] + (double)c.R[3 + a] * c.t[1] + (double)c.R[6 + a] * c.t[2]);
      f[(size_t)i * 6 + a] = pos;
      mean[a] += pos;
    }
    for (int a = 0; a < 3; ++a) f[(size_t)i * 6 + 3 + a] = (double)c.R[6 + a];
  }
  for (int a = 0; a < 3; ++a) mean[a] /= n;
  double rmax = 0.0;
  for (int i = 0; i < n; ++i) {
    double r2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      f[(size_t)i * 6 + a] -= mean[a];
      r2 += f[(size_t)i * 6 + a] * f[(size_t)i * 6 + a];
    }
    rmax = std::max(rmax, std::sqrt(r2));
  }
  if (rmax > 0.0)
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) f[(size_t)i * 6 + a] /= rmax;
}

// labels[i] in [0, B) after Lloyd's algorithm from D^2 seeding.
void kmeans(const std::vector<double>& f, int n, int B, uint64_t seed, std::vector<int>& labels) {
  std::vector<double> cen((size_t)B * 6);
  std::vector<char> is_centre(n, 0);
  std::vector<double> d2(n, 0.0);
  {
    const int first = (int)(((uint64_t)word24(0, 0, (uint32_t)B, kSeedTag, seed) * (uint64_t)n) >> 24);
    std::copy(&f[(size_t)first * 6], &f[(size_t)first * 6 + 6], &cen[0]);
    is_centre[first] = 1;
    for (int i = 0; i < n; ++i) d2[i] = dist2(&f[(size_t)i * 6], &cen[0]);
  }
  for (int s = 1; s < B; ++s) {
    double total = 0.0;
    for (int i = 0; i < n; ++i) total += d2[i];
    int pick = -1;
    if (total > 0.0) {
      const double target = (double)word24((uint32_t)s, 0, (uint32_t)B, kSeedTag, seed) * 0x1p-24 * total;
      double run = 0.0;
      for (int i = 0; i < n && pick < 0; ++i) {
        run += d2[i];
        if (run > target) pick = i;
      }
      if (pick < 0) pick = n - 1;
    } else {
      for (int i = 0; i < n && pick < 0; ++i)
        if (!is_centre[i]) pick = i;
    }
    std::copy(&f[(size_t)pick * 6], &f[(size_t)pick * 6 + 6], &cen[(size_t)s * 6]);
    is_centre[pick] = 1;
    for (int i = 0; i < n; ++i) d2[i] = std::min(d2[i], dist2(&f[(size_t)i * 6], &cen[(size_t)s * 6]));
  }
  labels.assign(n, -1);
  std::vector<int> count(B);
  for (int round = 0; round < kMaxRounds; ++round) {
    bool changed = false;
    for (int i = 0; i < n; ++i) {
      int best = 0;
      double bd = dist2(&f[(size_t)i * 6], &cen[0]);
      for (int c = 1; c < B; ++c) {
        const double d = dist2(&f[(size_t)i * 6], &cen[(size_t)c * 6]);
        if (d < bd) { bd = d; best = c; }
      }
      if (labels[i] != best) { labels[i] = best; changed = true; }
    }
    // an empty cluster takes the camera farthest from its own centre
    std::fill(count.begin(), count.end(), 0);
    for (int i = 0; i < n; ++i) ++count[labels[i]];
    bool reseeded = false;
    for (int c = 0; c < B; ++c) {
      if (count[c] > 0) continue;
      int far = -1;
      double fd = -1.0;
      for (int i = 0; i < n; ++i) {
        if (count[labels[i]] < 2) continue;
        const double d = dist2(&f[(size_t)i * 6], &cen[(size_t)labels[i] * 6]);
        if (d > fd) { fd = d; far = i; }
      }
      if (far < 0) break;  // cannot happen for B <= n
      --count[labels[far]];
      labels[far] = c;
      count[c] = 1;
      reseeded = true;
    }
    // centres = means of the members
    std::fill(cen.begin(), cen.end(), 0.0);
    for (int i = 0; i < n; ++i)
      for (int q = 0; q < 6; ++q) cen[(size_t)labels[i] * 6 + q] += f[(size_t)i * 6 + q];
    for (int c = 0; c < B; ++c)
      for (int q = 0; q < 6; ++q) cen[(size_t)c * 6 + q] /= count[c];
    if (!changed && !reseeded) break;
  }
}

}  // namespace
}  // namespace lmrs

extern "C" {

lmrs_status lmrs_view_clusters(const lmrs_camera* cams, int32_t n_cams, int32_t batch, uint64_t seed,
                               int32_t* labels) {
  if (!cams || !labels) return lmrs::report_error(LMRS_EINVAL, "cams and labels must not be NULL");
  if (n_cams <= 0 || batch <= 0 || batch > n_cams)
    return lmrs::report_error(LMRS_EINVAL, "need 0 < batch <= n_cams");
  std::vector<double> f;
  lmrs::features(cams, n_cams, f);
  std::vector<int> lab;
  lmrs::kmeans(f, n_cams, batch, seed, lab);
  for (int i = 0; i < n_cams; ++i) labels[i] = lab[i];
  return LMRS_OK;
}

lmrs_status lmrs_view_batch(const int32_t* labels, int32_t n_cams, int32_t batch, uint64_t seed, int32_t iter,
                            int32_t* view_ids) {
  if (!labels || !view_ids) return lmrs::report_error(LMRS_EINVAL, "labels and view_ids must not be NULL");
  if (n_cams <= 0 || batch <= 0 || batch > n_cams)
    return lmrs::report_error(LMRS_EINVAL, "need 0 < batch <= n_cams");
  std::vector<std::vector<int>> members(batch);
  for (int i = 0; i < n_cams; ++i) {
    if (labels[i] < 0 || labels[i] >= batch) return lmrs::report_error(LMRS_EINVAL, "label out of range");
    members[labels[i]].push_back(i);
  }
  for (int j = 0; j < batch; ++j) {
    const auto& m = members[j];
    if (m.empty()) return lmrs::report_error(LMRS_EINVAL, "a cluster has no camera");
    const uint64_t d = lmrs::word24((uint32_t)j, (uint32_t)iter, (uint32_t)batch, lmrs::kPickTag, seed);
    view_ids[j] = m[(size_t)((d * (uint64_t)m.size()) >> 24)];
  }
  return LMRS_OK;
}

}  // extern "C"
