// Lattice tables and equilibrium weights of the DdQ(2d^2+1) model, c = 1.
//
// Velocity order (Sec. 2.3, eqs. d1q3, d2q9, d3q19, ddqq): rest; +e_1..+e_d;
// -e_1..-e_d; then for each pair i < j in lexicographic order four diagonals
// whose (c_i, c_j) are (1,1), (-1,1), (-1,-1), (1,-1).
//
// Weights: the closed form eq. (omega_k-2) with one fourth-order moment m4 for
// every pair (Remark 5), m4 from eq. (meq-4rd).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace lbm {

constexpr int kMaxDim = 4;
constexpr int kMaxQ = 33;

constexpr int q_of(int d) { return 2 * d * d + 1; }

// Component a of velocity k of the D-dimensional set.
constexpr int vel_comp(int D, int k, int a) {
  if (k == 0) return 0;
  if (k <= D) return (a == k - 1) ? 1 : 0;
  if (k <= 2 * D) return (a == k - D - 1) ? -1 : 0;
  const int idx = k - 2 * D - 1;
  const int pair = idx / 4, m = idx % 4;
  int cnt = 0;
  for (int i = 0; i < D; ++i) {
    for (int j = i + 1; j < D; ++j) {
      if (cnt == pair) {
        // (c_i, c_j) = (1,1), (-1,1), (-1,-1), (1,-1)
        const int ci = (m == 0 || m == 3) ? 1 : -1;
        const int cj = (m <= 1) ? 1 : -1;
        if (a == i) return ci;
        if (a == j) return cj;
        return 0;
      }
      ++cnt;
    }
  }
  return 0;
}

// Index of the opposite velocity (c_kbar = -c_k).
constexpr int opp_index(int D, int k) {
  const int Q = q_of(D);
  for (int m = 0; m < Q; ++m) {
    bool same = true;
    for (int a = 0; a < D; ++a)
      if (vel_comp(D, m, a) != -vel_comp(D, k, a)) same = false;
    if (same) return m;
  }
  return -1;
}

// Fourth-order moment, eq. (meq-4rd), sigma = u; defined for d >= 2.
__host__ __device__ inline double m4_interpolated(int d, const double* u, double g) {
  double s2 = 0.0;
  for (int i = 0; i < d; ++i) s2 += u[i] * u[i];
  double lo = (-6.0 + 2.0 * d + 4.0 * s2) / (3.0 * d * (d - 1));
  for (int i = 0; i < d; ++i)
    for (int j = i + 1; j < d; ++j) {
      const double a = (std::fabs(u[i] + u[j]) - 2.0 * u[i] * u[j]) / 3.0;
      const double b = (std::fabs(u[i] - u[j]) + 2.0 * u[i] * u[j]) / 3.0;
      lo = std::fmax(lo, std::fmax(a, b));
    }
  double hi = 1e300;
  for (int i = 0; i < d; ++i)
    hi = std::fmin(hi, (1.0 + 2.0 * u[i] * u[i] - std::fabs((4 - d) * u[i])) / (3.0 * (d - 1)));
  return g * lo + (1.0 - g) * hi;
}

// EDF weights, closed form eq. (omega_k-2) with c = 1 and equal m4.
__host__ __device__ inline void omega_closed_form(int d, const double* u, double m4,
                                                     double* w) {
  double s2 = 0.0;
  for (int i = 0; i < d; ++i) s2 += u[i] * u[i];
  const int npairs = d * (d - 1) / 2;
  w[0] = (3.0 - d - 2.0 * s2 + 3.0 * npairs * m4) / 3.0;
  for (int i = 0; i < d; ++i) {
    const double common = 1.0 + 2.0 * u[i] * u[i] - 3.0 * (d - 1) * m4;
    w[1 + i] = ((4 - d) * u[i] + common) / 6.0;
    w[1 + d + i] = (-(4 - d) * u[i] + common) / 6.0;
  }
  const int q = q_of(d);
  for (int k = 2 * d + 1; k < q; ++k) {
    int i = -1, j = -1;
    for (int a = 0; a < d; ++a)
      if (vel_comp(d, k, a) != 0) {
        if (i < 0) i = a; else j = a;
      }
    const int si = vel_comp(d, k, i), sj = vel_comp(d, k, j);
    w[k] = (3.0 * m4 + 2.0 * si * sj * u[i] * u[j] + si * u[i] + sj * u[j]) / 12.0;
  }
}

}  // namespace lbm
