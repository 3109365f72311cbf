// Physics-based interface functions (paper, section 3.1, eqs. (new_basis1)
// to (new_basis6)), built on the host at set-up.  Plain C++ (no HIP), so
// that the host tests can compile it on its own.
#pragma once

#include <algorithm>
#include <vector>

namespace mrcm {
namespace phys {

// The channels and barriers of an interface are the maximal runs of faces whose conductance t_j (harmonic mean of K across the
// face) is at least STRUCT_RATIO times the median of t over the interface
// (channels), or at most the median over STRUCT_RATIO (barriers); at most
// PHYS_NH channels and PHYS_NL barriers are kept, the widest first (the
// left one on ties).  A space with no structure of its kind is the linear
// one; functions without support are left out.  The pressure functions go
// to slots 0.. of the interface's rows, the flux functions to slots
// PHYS_P.., the rest stay zero (inactive dofs).
constexpr int PHYS_NH = 2, PHYS_NL = 1, PHYS_P = 4, PHYS_U = 4;
constexpr double STRUCT_RATIO = 10.0;

struct Run {
  int j0, j1;
};

inline std::vector<Run> face_runs(const std::vector<char>& mask) {
  std::vector<Run> runs;
  const int m = (int)mask.size();
  for (int j = 0; j < m;) {
    if (!mask[j]) { ++j; continue; }
    int k = j;
    while (k + 1 < m && mask[k + 1]) ++k;
    runs.push_back({j, k});
    j = k + 1;
  }
  return runs;
}

inline std::vector<Run> widest(std::vector<Run> runs, int n) {
  std::stable_sort(runs.begin(), runs.end(),
                   [](const Run& x, const Run& y) { return x.j1 - x.j0 > y.j1 - y.j0; });
  if ((int)runs.size() > n) runs.resize(n);
  std::sort(runs.begin(), runs.end(), [](const Run& x, const Run& y) { return x.j0 < y.j0; });
  return runs;
}

// channels and barriers of one interface from its faces' conductances
inline void classify_faces(const std::vector<double>& t, std::vector<Run>& channels, std::vector<Run>& barriers) {
  const int m = (int)t.size();
  std::vector<double> srt(t);
  std::sort(srt.begin(), srt.end());
  const double med = (m % 2) ? srt[m / 2] : 0.5 * (srt[m / 2 - 1] + srt[m / 2]);
  std::vector<char> hi(m), lo(m);
  for (int j = 0; j < m; ++j) {
    hi[j] = t[j] >= STRUCT_RATIO * med;
    lo[j] = t[j] <= med / STRUCT_RATIO;
  }
  channels = widest(face_runs(hi), PHYS_NH);
  barriers = widest(face_runs(lo), PHYS_NL);
}

// the functions of one interface into out[(PHYS_P + PHYS_U) * M]; returns
// the numbers of pressure and flux functions
inline void physics_space(const std::vector<double>& t, double* out, int M, int& n_p, int& n_u) {
  std::vector<Run> ch, bar;
  classify_faces(t, ch, bar);
  auto x = [M](int j) { return (j + 0.5) / M; };
  n_p = 0;
  if (ch.empty()) {   // linear
    for (int j = 0; j < M; ++j) {
      out[0 * M + j] = 1.0 - x(j);
      out[1 * M + j] = x(j);
    }
    n_p = 2;
  } else {
    const int n = (int)ch.size();
    std::vector<double> a(n), b(n);
    for (int k = 0; k < n; ++k) {
      a[k] = (double)ch[k].j0 / M;
      b[k] = (double)(ch[k].j1 + 1) / M;
    }
    if (a[0] > 0.0) {   // falls from the interface start to the first channel
      for (int j = 0; j < M; ++j) out[n_p * M + j] = x(j) < a[0] ? (a[0] - x(j)) / a[0] : 0.0;
      ++n_p;
    }
    for (int k = 0; k < n; ++k) {   // 1 on channel k, ramps to the neighbouring structures
      const double l = k == 0 ? 0.0 : b[k - 1], h = k == n - 1 ? 1.0 : a[k + 1];
      for (int j = 0; j < M; ++j) {
        const double xj = x(j);
        double v = 0.0;
        if (xj > l && xj < a[k]) v = (xj - l) / (a[k] - l);
        else if (xj >= a[k] && xj <= b[k]) v = 1.0;
        else if (xj > b[k] && xj < h) v = (h - xj) / (h - b[k]);
        out[n_p * M + j] = v;
      }
      ++n_p;
    }
    if (b[n - 1] < 1.0) {   // rises from the last channel to the interface end
      for (int j = 0; j < M; ++j)
        out[n_p * M + j] = x(j) > b[n - 1] ? (x(j) - b[n - 1]) / (1.0 - b[n - 1]) : 0.0;
      ++n_p;
    }
  }
  double* u = out + PHYS_P * M;
  n_u = 0;
  if (bar.empty()) {
    for (int j = 0; j < M; ++j) {
      u[0 * M + j] = 1.0 - x(j);
      u[1 * M + j] = x(j);
    }
    n_u = 2;
  } else {   // indicators of the segments before, on and after each barrier
    std::vector<double> edges{0.0};
    for (const Run& r : bar) {
      edges.push_back((double)r.j0 / M);
      edges.push_back((double)(r.j1 + 1) / M);
    }
    edges.push_back(1.0);
    for (size_t q = 0; q + 1 < edges.size(); ++q) {
      if (!(edges[q + 1] > edges[q])) continue;
      for (int j = 0; j < M; ++j) u[n_u * M + j] = (x(j) > edges[q] && x(j) < edges[q + 1]) ? 1.0 : 0.0;
      ++n_u;
    }
  }
}

}  // namespace phys
}  // namespace mrcm
