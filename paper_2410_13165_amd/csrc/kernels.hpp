// Device code of the stream-collide, wall, initialisation and reduction
// kernels (templates), shared by kernels.hip (bulk passes and launchers) and
// walls_d*.hip (the wall-row and x_1-face kernels).  A kernel template is compiled
// only in the translation unit that launches it.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "engine.hpp"
#include "fuse.hpp"
#include "meta.hpp"

namespace lbm {

// ----------------------------------------------------------------- helpers --

template <int D>
struct RowInfo {
  int i[D];
  int dm[D];     // node offset of the upwind neighbour for c_a = +1 (wrapped)
  int dp[D];     // node offset of the upwind neighbour for c_a = -1 (wrapped)
  bool lo[D];    // node lies on the lower Dirichlet wall of axis a
  bool hi[D];    // node lies on the upper Dirichlet wall of axis a
  bool rowwall;  // some axis a >= 1 puts the whole row on a wall
  int rowbase;
};

template <int D>
__device__ __forceinline__ void row_setup(const KParams& p, int row, RowInfo<D>& r) {
  int rr = row;
  r.rowwall = false;
#pragma unroll
  for (int a = 1; a < D; ++a) {
    const int n = p.n[a];
    const int ia = rr % n;
    rr /= n;
    const int st = p.stride[a];
    r.i[a] = ia;
    r.dm[a] = (ia == 0) ? (n - 1) * st : -st;
    r.dp[a] = (ia == n - 1) ? -(n - 1) * st : st;
    const bool wall = p.bc[a] != 0;
    r.lo[a] = wall && ia == 0;
    r.hi[a] = wall && ia == n - 1;
    r.rowwall = r.rowwall || r.lo[a] || r.hi[a];
  }
  r.rowbase = row * p.n[0];
}

// row_setup for d = 3 from the row's coordinates (i_2, i_3), without the
// divisions that recover them from the row index
__device__ __forceinline__ void row_setup_yz(const KParams& p, int iy, int iz, RowInfo<3>& r) {
  const int ia[3] = {0, iy, iz};
  r.rowwall = false;
#pragma unroll
  for (int a = 1; a < 3; ++a) {
    const int n = p.n[a];
    const int st = p.stride[a];
    r.i[a] = ia[a];
    r.dm[a] = (ia[a] == 0) ? (n - 1) * st : -st;
    r.dp[a] = (ia[a] == n - 1) ? -(n - 1) * st : st;
    const bool wall = p.bc[a] != 0;
    r.lo[a] = wall && ia[a] == 0;
    r.hi[a] = wall && ia[a] == n - 1;
    r.rowwall = r.rowwall || r.lo[a] || r.hi[a];
  }
  r.rowbase = (iz * p.n[1] + iy) * p.n[0];
}

template <int D>
__device__ __forceinline__ void col_setup(const KParams& p, int x, RowInfo<D>& r) {
  const int n0 = p.n[0];
  r.i[0] = x;
  r.dm[0] = (x == 0) ? n0 - 1 : -1;
  r.dp[0] = (x == n0 - 1) ? -(n0 - 1) : 1;
  const bool wall = p.bc[0] != 0;
  r.lo[0] = wall && x == 0;
  r.hi[0] = wall && x == n0 - 1;
}

template <int D, int k>
__device__ __forceinline__ int pull_offset(const RowInfo<D>& r) {
  constexpr Vec4i c = vel_vec(D, k);
  int off = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (c.v[a] == 1) off += r.dm[a];
    if (c.v[a] == -1) off += r.dp[a];
  }
  return off;
}

template <int D, int k>
__device__ __forceinline__ bool outside(const RowInfo<D>& r) {
  constexpr Vec4i c = vel_vec(D, k);
  bool o = false;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (c.v[a] == 1) o = o || r.lo[a];
    if (c.v[a] == -1) o = o || r.hi[a];
  }
  return o;
}

// Lowest axis through whose wall population k enters the node from outside
// (0 when it enters through none).
template <int D, int k>
__device__ __forceinline__ int wall_axis(const RowInfo<D>& r) {
  constexpr Vec4i c = vel_vec(D, k);
  int ax = -1;
#pragma unroll
  for (int a = D - 1; a >= 0; --a) {
    if ((c.v[a] == 1 && r.lo[a]) || (c.v[a] == -1 && r.hi[a])) ax = a;
  }
  return ax < 0 ? 0 : ax;
}

template <int D>
__device__ __forceinline__ bool on_wall(const RowInfo<D>& r) {
  return r.rowwall || r.lo[0] || r.hi[0];
}

// Error-free sum a + b = s + e (Knuth's TwoSum), used for the compensated
// float32 moment sums.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

// -------------------------------------------------- analytic field values ---

// phi*(x, t) for the RMSE reference and the analytic initial state.
template <int D>
__device__ double field_value(const FieldDev& F, const KParams& p, const double (&x)[D],
                              double t) {
  double v = 0.0;
  if (F.kind == kFieldTanh) {
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double y = x[a] - p.u[a] * t - F.center[a];
      r2 += y * y;
    }
    v = 0.5 - 0.5 * tanh((F.Rr - sqrt(r2)) / (2.0 * F.W));
  } else {
    for (int j = 0; j < F.nmodes; ++j) {
      double ph = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) ph += F.kvec[j][a] * (x[a] - p.u[a] * t);
      v += (F.kind == kFieldCos) ? F.amp[j] * cos(ph + F.phase[j]) : F.amp[j] * exp(ph);
    }
  }
  return v + p.R * t;
}

// phi*(x, 0) and its gradient.
template <int D>
__device__ void field_initial(const FieldDev& F, const KParams& p, const double (&x)[D],
                              double& phi, double (&grad)[D]) {
#pragma unroll
  for (int a = 0; a < D; ++a) grad[a] = 0.0;
  phi = 0.0;
  if (F.kind == kFieldTanh) {
    double y[D];
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      y[a] = x[a] - F.center[a];
      r2 += y[a] * y[a];
    }
    const double r = sqrt(r2);
    const double z = (F.Rr - r) / (2.0 * F.W);
    phi = 0.5 - 0.5 * tanh(z);
    const double ch = cosh(z);
    const double dphi_dr = 0.5 / (ch * ch) / (2.0 * F.W);
    if (r > 0.0) {
#pragma unroll
      for (int a = 0; a < D; ++a) grad[a] = dphi_dr * y[a] / r;
    }
    return;
  }
  for (int j = 0; j < F.nmodes; ++j) {
    double ph = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) ph += F.kvec[j][a] * x[a];
    if (F.kind == kFieldCos) {
      double s, c;
      sincos(ph + F.phase[j], &s, &c);
      phi += F.amp[j] * c;
#pragma unroll
      for (int a = 0; a < D; ++a) grad[a] -= F.amp[j] * F.kvec[j][a] * s;
    } else {
      const double e = F.amp[j] * exp(ph);
      phi += e;
#pragma unroll
      for (int a = 0; a < D; ++a) grad[a] += F.kvec[j][a] * e;
    }
  }
}

// --------------------------------------------------------- wall schemes -----
//
// The exact solution is phi*(x,t) = F(x - u t) + R t, so on one Fourier or
// exponential mode every time derivative multiplies by w = -kappa.u and every
// derivative along c_k by pc = kappa.c_k; derivatives of cos cycle through
// cos, -sin, -cos, sin.
//
// Full-way, eq. (bun-1) at (x_b = node, t_{n+1}): with a = dt d_t and
// b = dt c_k.grad the printed polynomial is 1 - (a+b)/2 + (a+b)^3/24 applied to
// f^eq (its R terms cancel against the R t part), i.e. per mode
//   omega_k [F - (dt/2) v.grad F + (dt^3/24) (v.grad)^3 F] + omega_k R t,
// v = c_k - u; order 3 drops the cubic term, order 1 keeps F only.
//
// Half-way, eq. (bun2) at (x_b = x_f - c_k dx/2, t_n): the sum of
//   (omega_k + omega_kbar) [1 + (dt/2) d_t - (dt^2/8)(c.grad)^2
//                           - (dt^3/16)(c.grad)^2 d_t - (dt^3/24) d_t^3]
//   (omega_k - omega_kbar) [-(dt^2/4) c.grad d_t - (dt^3/8) c.grad d_t^2]
// applied to phi*, plus (dt/2)(R_k + R_kbar), truncated at order P; the new
// population is that minus the post-collision f*_kbar at x_f.

// The wall kernels of d = 2 and 3 are compiled per variant of the wall
// formula, V = full-way (bit 0) | cosine field (bit 1; otherwise exponential):
// a kernel then holds the registers of one variant, not of all four (which
// left one wavefront per SIMD).  V = -1 takes both from the lattice at run
// time (d = 1 and 4, to bound the build).
template <int V>
__device__ __forceinline__ bool wall_full(const KParams& p) {
  if constexpr (V < 0) return p.scheme == kFullWay;
  else return (V & 1) != 0;
}
template <int V>
__device__ __forceinline__ bool wall_cos(const KParams& p) {
  if constexpr (V < 0) return p.field.kind == kFieldCos;
  else return (V & 2) != 0;
}
inline int wall_variant(const KParams& p) {
  return (p.scheme == kFullWay ? 1 : 0) | (p.field.kind == kFieldCos ? 2 : 0);
}

// Analytic wall values at one node (coordinates x) for the step
// t_n -> t_{n+1}, for every population k with sel(k) true, into val[k]:
// full-way: eq. (bun-1) at (x, t_{n+1}), the whole pre-collision f_k;
// half-way: the right side of eq. (bun2) at (x - c_k dx/2, t_n), to which the
// caller adds -f*_kbar(x, t_n).  One sincos (or exp) per mode serves every
// population: the half-way shift -(dx/2) kappa . c_k is applied by rotating
// with the per-axis factors of FieldDev::rot.
//
// Every derivative of a mode along c_k multiplies it by kappa . c_k.  With
// tangential wall data (TAN, p.wall_data == 1) that factor is assembled from what
// the data on the wall of axis j = axis(k) provide, as Remark 1 does with the
// equation: c_k . grad F = alpha . grad_tan F + beta d_t F with
// alpha = c_k - (c_kj / u_j) u (tangential, alpha_j = 0) and beta = -c_kj / u_j,
// i.e. the factor alpha . kappa + beta (-kappa . u).
//
// wall_mode gives mode j's factor at the wall point (cos and sin of its phase,
// or its exponential in C), wall_term the mode's contribution to population k,
// wall_close the terms outside the mode sum.

// t: t_{n+1} full-way, t_n half-way
template <int D, int V>
__device__ __forceinline__ void wall_mode(const KParams& p, const double (&x)[kMaxDim], double t,
                                          int j, double& C, double& S) {
  const FieldDev& F = p.field;
  double ph = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) ph += F.kvec[j][a] * (x[a] - p.u[a] * t);
  if (wall_cos<V>(p)) {
    sincos(ph + F.phase[j], &S, &C);
  } else {
    C = exp(ph);
    S = 0.0;
  }
}

template <int D, bool TAN, int V, int k, class Axis>
__device__ __forceinline__ double wall_term(const KParams& p, int j, double C, double S,
                                            Axis axis) {
  const FieldDev& F = p.field;
  const double dt = p.dt;
  const double o2 = p.P >= 2 ? 1.0 : 0.0;
  const double o3 = p.P >= 3 ? 1.0 : 0.0;
  const double o4 = p.P >= 4 ? 1.0 : 0.0;
  const double dt2 = dt * dt, dt3 = dt2 * dt;
  const bool is_cos = wall_cos<V>(p);
  constexpr Vec4i c = vel_vec(D, k);
  const double amp = F.amp[j];
  const double w = -F.ku[j];
  double pc = 0.0;
  if constexpr (!TAN) {
#pragma unroll
    for (int a = 0; a < D; ++a) pc += c.v[a] * F.kvec[j][a];
  } else {
    const int ja = axis(k);
    double r = 0.0;  // c_kj / u_j
#pragma unroll
    for (int a = 0; a < D; ++a)
      if (a == ja) r = c.v[a] * p.inv_u[a];
#pragma unroll
    for (int a = 0; a < D; ++a)
      if (a != ja) pc += (c.v[a] - r * p.u[a]) * F.kvec[j][a];
    pc -= r * w;
  }
  if (wall_full<V>(p)) {
    const double pv = pc + w;  // kappa . (c_k - u)
    const double pv3 = pv * pv * pv;
    if (is_cos) return amp * (C + (o3 * 0.5 * dt * pv + o4 * dt3 / 24.0 * pv3) * S);
    return amp * C * (1.0 - o3 * 0.5 * dt * pv + o4 * dt3 / 24.0 * pv3);
  }
  constexpr int kb = opp_index(D, k);
  const double wp = p.omega[k] + p.omega[kb];
  const double wm = p.omega[k] - p.omega[kb];
  const double T0 = wp;
  const double T1 = o2 * wp * 0.5 * dt * w;
  const double T2 = -o3 * (wp * dt2 / 8.0 * pc * pc + wm * dt2 / 4.0 * pc * w);
  const double T3 = -o4 * (wp * (dt3 / 16.0 * pc * pc * w + dt3 / 24.0 * w * w * w) +
                           wm * dt3 / 8.0 * pc * w * w);
  if (is_cos) {
    double Ck = C, Sk = S;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (c.v[a] == 0) continue;
      const double cr = F.rot[j][a][0];
      const double sr = c.v[a] * F.rot[j][a][1];
      const double nc = Ck * cr + Sk * sr;
      Sk = Sk * cr - Ck * sr;
      Ck = nc;
    }
    return amp * ((T0 - T2) * Ck + (T3 - T1) * Sk);
  }
  double Ek = C;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (c.v[a] == 1) Ek *= F.rot[j][a][0];
    if (c.v[a] == -1) Ek *= F.rot[j][a][1];
  }
  return amp * (T0 + T1 + T2 + T3) * Ek;
}

template <int D, int V, int k>
__device__ __forceinline__ double wall_close(const KParams& p, double v, double t_n) {
  if (wall_full<V>(p)) return p.omega[k] * (v + p.R * (t_n + p.dt));
  constexpr int kb = opp_index(D, k);
  const double o2 = p.P >= 2 ? 1.0 : 0.0;
  const double wp = p.omega[k] + p.omega[kb];
  return v + wp * p.R * t_n + o2 * wp * p.R * p.dt;
}

// Only the populations K0 <= k < K1 are evaluated; each val[k] is the same sum
// over the modes in the same order whatever the range.  M0: the caller gives
// mode 0's factor (C0, S0) from wall_mode.
template <int D, bool TAN, int V, int K0 = 0, int K1 = q_of(D), bool M0 = false, class Sel,
          class Axis>
__device__ __forceinline__ void wall_analytic(const KParams& p, const double (&x)[kMaxDim],
                                              double t_n, Sel sel, Axis axis,
                                              double (&val)[q_of(D)], double C0 = 0.0,
                                              double S0 = 0.0) {
  const double t = wall_full<V>(p) ? t_n + p.dt : t_n;
#pragma unroll
  for (int k = K0; k < K1; ++k) val[k] = 0.0;
#pragma unroll 1
  for (int j = 0; j < p.field.nmodes; ++j) {
    double C = C0, S = S0;
    if (!M0 || j > 0) wall_mode<D, V>(p, x, t, j, C, S);
    static_for<K0, K1>([&](auto K) {
      constexpr int k = decltype(K)::value;
      if (!sel(k)) return;
      val[k] += wall_term<D, TAN, V, k>(p, j, C, S, axis);
    });
  }
  static_for<K0, K1>([&](auto K) {
    constexpr int k = decltype(K)::value;
    if (!sel(k)) return;
    val[k] = wall_close<D, V, k>(p, val[k], t_n);
  });
}

// Modes whose factors the half-way wall path of d = 3 keeps in registers
constexpr int kWallModeCache = 4;

// The population in slot s (0 <= s < 2D - 1) of those entering through the
// lower (cx = +1) or upper (cx = -1) x_1 face: xface_slot's inverse.
constexpr int face_pop(int D, int cx, int s) {
  int n = 0;
  for (int k = 0; k < q_of(D); ++k) {
    if (vel_comp(D, k, 0) != cx) continue;
    if (n == s) return k;
    ++n;
  }
  return -1;
}

// Slot of population k among those entering through the lower (c_k1 = +1) or
// upper (c_k1 = -1) x_1 face; there are 2D - 1 of each.
constexpr int xface_slot(int D, int k) {
  const int cx = vel_comp(D, k, 0);
  int slot = 0;
  for (int m = 0; m < k; ++m)
    if (vel_comp(D, m, 0) == cx) ++slot;
  return slot;
}

// Wall values of every wall node of a row (any Dirichlet axis; used for the
// rows that lie on a wall of an axis >= 2 and by the x_1 faces through
// k_xface).  fstar_local(kb) returns the absolute post-collision f*_kb at the
// node.
template <int D, bool TAN, int V, class A, class FStarLocal>
__device__ __forceinline__ void wall_values(A (&f)[q_of(D)], const KParams& p, const RowInfo<D>& r,
                                            double t_n, double ref, FStarLocal fstar_local) {
  double x[kMaxDim] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < D; ++a) x[a] = p.origin[a] + (r.i[a] + p.shift[a]) * p.dx;
  bool out[q_of(D)];
  static_for<0, q_of(D)>([&](auto K) {
    constexpr int k = decltype(K)::value;
    out[k] = outside<D, k>(r);
  });
  int ax[q_of(D)];
  static_for<0, q_of(D)>([&](auto K) {
    constexpr int k = decltype(K)::value;
    ax[k] = TAN ? wall_axis<D, k>(r) : 0;
  });
  const bool half = !wall_full<V>(p);
  // Half-way walls of d = 3 and all walls of d = 4 take one population at a
  // time, skipping those that enter from inside: their sums and coefficients
  // held at once took 256 VGPRs (d = 4 with spills), one wavefront per SIMD.
  // Half-way walls of d = 3 with up to kWallModeCache modes first take every
  // mode's factor once per node; otherwise the first mode's factor is taken
  // once per node and the others' again for each population.
  if constexpr (D == 3 && V >= 0 && (V & 1) == 0) {
    if (p.field.nmodes <= kWallModeCache) {
      double mc[kWallModeCache], ms[kWallModeCache];
#pragma unroll
      for (int j = 0; j < kWallModeCache; ++j)
        if (j < p.field.nmodes) wall_mode<D, V>(p, x, t_n, j, mc[j], ms[j]);
      static_for<0, q_of(D)>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if (!out[k]) return;
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < kWallModeCache; ++j)
          if (j < p.field.nmodes)
            v += wall_term<D, TAN, V, k>(p, j, mc[j], ms[j], [&](int kk) { return ax[kk]; });
        v = wall_close<D, V, k>(p, v, t_n) - fstar_local(opp_index(D, k));
        f[k] = static_cast<A>(v - p.omega[k] * ref);
      });
      return;
    }
  }
  constexpr int G = (D == 4 || (D == 3 && V >= 0 && (V & 1) == 0)) ? 1 : q_of(D);
  double c0 = 0.0, s0 = 0.0;
  if constexpr (G < q_of(D)) {
    if (p.field.nmodes > 0) wall_mode<D, V>(p, x, half ? t_n : t_n + p.dt, 0, c0, s0);
  }
  static_for<0, (q_of(D) + G - 1) / G>([&](auto Gi) {
    constexpr int k0 = decltype(Gi)::value * G;
    constexpr int k1 = k0 + G < q_of(D) ? k0 + G : q_of(D);
    if constexpr (G < q_of(D)) {
      bool any = false;
      static_for<k0, k1>([&](auto K) { any = any || out[decltype(K)::value]; });
      if (!any) return;
    }
    double val[q_of(D)];
    wall_analytic<D, TAN, V, k0, k1, (G < q_of(D))>(p, x, t_n, [&](int k) { return out[k]; },
                                                    [&](int k) { return ax[k]; }, val, c0, s0);
    static_for<k0, k1>([&](auto K) {
      constexpr int k = decltype(K)::value;
      if (!out[k]) return;
      double v = val[k];
      if (half) v -= fstar_local(opp_index(D, k));
      f[k] = static_cast<A>(v - p.omega[k] * ref);
    });
  });
}

// Analytic wall data of the x_1 faces for the step t_n -> t_{n+1}: one
// thread per (face, row).  A population with c_k1 = +1 (-1) is unknown on the
// lower (upper) x_1 face only, so its value for row `row` is kept in its own
// population plane of the source buffer, at element p.xoff + row past the
// nodes; the bulk kernel then reads it with the same base address as its
// pulls.  Values are stored in the storage type T:
//   full-way  f_k - omega_k ref,
//   half-way  B_k - (omega_k + omega_kbar) ref  (the bulk kernel subtracts the
//             stored post-collision kbar value of the node),
// with ref = phi_ref + R t_{n+1} in float32 mode and 0 otherwise.  The split
// mode keeps float64 values in p.xdata[(side * (2D-1) + slot) * rows + row].
template <int D, class T, bool TAN, int V>
__global__ void __launch_bounds__(256)
    k_xface(T* __restrict__ buf, const KParams p, const double t_n, const int mode) {
  constexpr int S = 2 * D - 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * p.rows) return;
  const int side = idx >= p.rows ? 1 : 0;
  const int row = idx - side * p.rows;
  double x[kMaxDim] = {0.0, 0.0, 0.0, 0.0};
  x[0] = p.origin[0] + ((side ? p.n[0] - 1 : 0) + p.shift[0]) * p.dx;
  int rr = row;
#pragma unroll
  for (int a = 1; a < D; ++a) {
    const int ia = rr % p.n[a];
    rr /= p.n[a];
    x[a] = p.origin[a] + (ia + p.shift[a]) * p.dx;
  }
  const double ref = (mode == kFP32) ? p.phi_ref + p.R * (t_n + p.dt) : 0.0;
  const bool half = !wall_full<V>(p);
  const long long ps = p.pstride;
  const int want = side ? -1 : 1;
  double val[q_of(D)];
  wall_analytic<D, TAN, V>(p, x, t_n, [&](int k) { return p.cv[k][0] == want; },
                           [](int) { return 0; }, val);
  static_for<0, q_of(D)>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr int cx = vel_comp(D, k, 0);
    if constexpr (cx == 0) {
      return;
    } else {
      if (cx != want) return;
      if (split_layout(mode)) {
        p.xdata[((long long)side * S + xface_slot(D, k)) * p.rows + row] = val[k];
      } else {
        constexpr int kb = opp_index(D, k);
        const double wref = (half ? p.omega[k] + p.omega[kb] : p.omega[k]) * ref;
        buf[k * ps + p.xoff + row] = static_cast<T>(val[k] - wref);
      }
    }
  });
}

// ------------------------------------------------------------ step kernels --

// Collision of the pulled pre-collision populations (collide_vals, in place)
// and store of the post-collision ones (collide_store; non-temporal stores:
// nothing rereads them this step).
// float64: f*_k = (1-s) f_k + s omega_k phi + dt omega_k R.
// float32 stores deviations from the uniform exact state omega_k (phi_ref + R t),
// which is a fixed point of stream + collide, so the deviations follow the same
// update without the source term; phi is summed with TwoSum compensation.
template <int D, class T>
__device__ __forceinline__ void collide_vals(T (&f)[q_of(D)], const KParams& p) {
  constexpr int Q = q_of(D);
  if constexpr (std::is_same<T, float>::value) {
    float sum = f[0], comp = 0.0f;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      float e;
      two_sum(sum, f[k], sum, e);
      comp += e;
    }
    const float phi = sum + comp;
    const float oms = 1.0f - p.s_f;
#pragma unroll
    for (int k = 0; k < Q; ++k) f[k] = fmaf(p.s_f * p.omega_f[k], phi, oms * f[k]);
  } else {
    double phi = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) phi += f[k];
    const double oms = 1.0 - p.s;
    // omega_k (s phi + dt R) + (1 - s) f_k: one uniform constant per
    // population (omega_k) instead of two (s omega_k, dt R omega_k)
    const double a = fma(p.s, phi, p.dt * p.R);
#pragma unroll
    for (int k = 0; k < Q; ++k) f[k] = fma(p.omega[k], a, oms * f[k]);
  }
}

template <int D, class T>
__device__ __forceinline__ void collide_store(T (&f)[q_of(D)], T* __restrict__ dst, long long ps,
                                              int node, const KParams& p) {
  collide_vals<D, T>(f, p);
#pragma unroll
  for (int k = 0; k < q_of(D); ++k) __builtin_nontemporal_store(f[k], dst + k * ps + node);
}

// Bulk rows: post-collision populations stored (float64, or float32
// deviations from omega_k (phi_ref + R t_{n+1})).  Rows on a wall of an axis
// >= 2 are left to k_wall.  On the x_1 faces the unknown populations are read
// from k_xface's data instead of the upwind node (an index select on the same
// base address, so the common path keeps its registers); the half-way scheme
// then subtracts the node's own post-collision kbar value.
template <int D, class T>
__device__ __forceinline__ void step_row(const T* __restrict__ src, T* __restrict__ dst,
                                         const KParams& p, int row) {
  constexpr int Q = q_of(D);
  RowInfo<D> r;
  row_setup<D>(p, row, r);
  if (r.rowwall) return;
  const long long ps = p.pstride;
  const bool half = p.scheme == kHalfWay;
  for (int x = threadIdx.x; x < p.n[0]; x += blockDim.x) {
    col_setup<D>(p, x, r);
    const int node = r.rowbase + x;
    const bool xwall = r.lo[0] || r.hi[0];
    T f[Q];
    static_for<0, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr int cx = vel_comp(D, k, 0);
      int idx = node + pull_offset<D, k>(r);
      if constexpr (cx != 0) {
        if ((cx == 1) ? r.lo[0] : r.hi[0]) idx = p.xoff + row;
      }
      f[k] = src[k * ps + idx];
    });
    if (xwall && half) {
      static_for<0, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        constexpr int cx = vel_comp(D, k, 0);
        if constexpr (cx != 0) {
          if ((cx == 1) ? r.lo[0] : r.hi[0]) f[k] -= src[opp_index(D, k) * ps + node];
        }
      });
    }
    collide_store<D, T>(f, dst, ps, node, p);
  }
}

template <int D, class T>
__global__ void __launch_bounds__(256)
    k_step(const T* __restrict__ src, T* __restrict__ dst, const KParams p) {
  const int row = blockIdx.x * blockDim.y + threadIdx.y;
  if (row >= p.rows) return;
  step_row<D, T>(src, dst, p, row);
}

// ------------------------------------------------------ two fused steps --
//
// Two time steps t_n -> t_{n+2} in one pass (float32 or float64 storage,
// d = 3), so each
// stored population is read and written about once per two steps instead of
// once per step.  A block owns an x_1-x_2 tile of TX x TY output nodes and
// a chunk of x_3 planes (fuse_tile), and marches along x_3: for step-1 plane z it updates
// the tile plus a one-node halo (from A, the state at t_n) into LDS, then
// updates output plane z - 1 of step 2 by pulling from the LDS planes z - 2,
// z - 1 and z, and stores it to B.  Each plane's step-1 values stay in LDS only
// as long as step 2 needs them: populations with c_3 = 0 for two planes, c_3 =
// +1 for three, c_3 = -1 for one (two with half-way walls, whose x_1 faces need
// the node's own step-1 value of the opposite population).
//
// Rows on a Dirichlet wall of x_2 or x_3 are not updated here.  Their step-1
// values come from k_wall(A -> C) launched before, and k_wall(C -> B) updates
// them for step 2 afterwards; for that second launch this kernel also stores
// its step-1 values of the rows next to those walls in C.  The x_1-face wall
// data of step 1 are in A's row slots and those of step 2 in B's (k_xface on
// both before the launch).  Every node goes through exactly the arithmetic of
// k_step, so the result is bitwise that of two single steps.
template <class T, bool HALF>
__global__ void __launch_bounds__((FuseFwdShape<T, HALF>::NT))
    k_fused2(const T* __restrict__ A, T* __restrict__ B, T* __restrict__ C, const KParams p,
             const int zc) {
  using S = FuseFwdShape<T, HALF>;
  constexpr int D = 3, Q = q_of(3), TX = S::TX, TY = S::TY, NT = S::NT;
  constexpr int RX = TX + 2, RY = TY + 2, R = RX * RY;
  extern __shared__ __align__(16) unsigned char fuse_lds[];
  T* lds = reinterpret_cast<T*>(fuse_lds);
  T* side = lds + S::SLOTS * R;  // half-way only: side[((parity * 2) + face) * RY + ry]
  const long long ps = p.pstride;
  const int n0 = p.n[0], n1 = p.n[1], n2 = p.n[2];
  int tx_, ty_, tz_;
  fuse_tile(p, TX, TY, tx_, ty_, tz_);
  const int x0 = tx_ * TX, y0 = ty_ * TY, zc0 = tz_ * zc;
  const int zend = min(zc0 + zc, n2);
  const int iters = zend - zc0 + 2;
  for (int it = 0; it < iters; ++it) {
    const int zp = zc0 - 1 + it;  // step-1 plane of this iteration
    // ---- step 1 on the tile and its halo of plane zp
    for (int t = threadIdx.x; t < R; t += NT) {
      const int r = fuse_region<TX, TY>(t);
      const int rx = r % RX, ry = r / RX;
      int gx = x0 - 1 + rx, gy = y0 - 1 + ry, gz = zp;
      if (gx < 0 || gx >= n0) {
        if (p.bc[0] != 0) continue;
        gx = fuse_wrap(gx, n0);
      }
      if (gy < 0 || gy >= n1) {
        if (p.bc[1] != 0) continue;
        gy = fuse_wrap(gy, n1);
      }
      if (gz < 0 || gz >= n2) {
        if (p.bc[2] != 0) continue;
        gz = fuse_wrap(gz, n2);
      }
      const int row = gz * n1 + gy;
      RowInfo<D> ri;
      row_setup_yz(p, gy, gz, ri);
      col_setup<D>(p, gx, ri);
      const int node = ri.rowbase + gx;
      T f[Q];
      if (ri.rowwall) {
        static_for<0, Q>([&](auto K) {
          constexpr int k = decltype(K)::value;
          f[k] = C[k * ps + node];
        });
      } else {
        static_for<0, Q>([&](auto K) {
          constexpr int k = decltype(K)::value;
          constexpr int cx = vel_comp(D, k, 0);
          int idx = node + pull_offset<D, k>(ri);
          if constexpr (cx != 0) {
            if ((cx == 1) ? ri.lo[0] : ri.hi[0]) idx = p.xoff + row;
          }
          f[k] = A[k * ps + idx];
        });
        if (HALF && (ri.lo[0] || ri.hi[0])) {
          // the node's own f*_kbar of the face's 2D - 1 unknowns, every load
          // issued before any is used (one branch per population had the
          // compiler wait for each load in turn)
          const bool lo = ri.lo[0];
          T sb[2 * D - 1];
          static_for<0, 2 * D - 1>([&](auto Sx) {
            constexpr int sl = decltype(Sx)::value;
            constexpr int kl = face_pop(D, 1, sl), kh = face_pop(D, -1, sl);
            sb[sl] = A[(lo ? opp_index(D, kl) : opp_index(D, kh)) * ps + node];
          });
          asm volatile("" ::: "memory");
          static_for<0, 2 * D - 1>([&](auto Sx) {
            constexpr int sl = decltype(Sx)::value;
            constexpr int kl = face_pop(D, 1, sl), kh = face_pop(D, -1, sl);
            if (lo) f[kl] -= sb[sl];
            else f[kh] -= sb[sl];
          });
        }
        collide_vals<D, T>(f, p);
        // rows next to a wall of x_2 / x_3, owned by this block: kept for the
        // step-2 wall kernel
        const bool own = rx >= 1 && rx <= TX && ry >= 1 && ry <= TY && x0 - 1 + rx < n0 &&
                         y0 - 1 + ry < n1 && zp >= zc0 && zp < zend;
        const bool near = (p.bc[1] != 0 && (ri.i[1] == 1 || ri.i[1] == n1 - 2)) ||
                          (p.bc[2] != 0 && (ri.i[2] == 1 || ri.i[2] == n2 - 2));
        if (own && near) {
#pragma unroll
          for (int k = 0; k < Q; ++k) __builtin_nontemporal_store(f[k], C + k * ps + node);
        }
      }
      static_for<0, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        lds[fuse_slot<false, k>(it) * R + r] = f[k];
      });
      if (HALF && (ri.lo[0] || ri.hi[0])) {
        // f*_kbar with c_3(kbar) = -1 opposite the face's unknowns, for step 2
        // of this plane (read one iteration later)
        static_for<0, Q>([&](auto K) {
          constexpr int k = decltype(K)::value;
          constexpr int cx = vel_comp(D, k, 0);
          if constexpr (cx != 0 && vel_comp(D, k, 2) == 1) {
            const int face = cx == 1 ? 0 : 1;
            if ((cx == 1) ? ri.lo[0] : ri.hi[0])
              side[((it & 1) * 2 + face) * RY + ry] = f[opp_index(D, k)];
          }
        });
      }
    }
    __syncthreads();
    // ---- step 2 on output plane zp - 1
    if (it >= 2) {
      const int gz = zp - 1;
      for (int o = threadIdx.x; o < TX * TY; o += NT) {
        const int ox = o % TX, oy = o / TX;
        const int gx = x0 + ox, gy = y0 + oy;
        if (gx >= n0 || gy >= n1) continue;
        const int row = gz * n1 + gy;
        RowInfo<D> ri;
        row_setup_yz(p, gy, gz, ri);
        if (ri.rowwall) continue;
        col_setup<D>(p, gx, ri);
        const int node = ri.rowbase + gx;
        // every pull from LDS, then the x_1-face unknowns from B's row slots
        // in a branch of their own (a per-lane choice between the two would
        // become one generic-pointer load, which waits on all memory traffic)
        T f[Q];
        static_for<0, Q>([&](auto K) {
          constexpr int k = decltype(K)::value;
          constexpr Vec4i c = vel_vec(D, k);
          constexpr int src_it = c.v[2] == 0 ? 1 : (c.v[2] == 1 ? 2 : 0);
          const int rr = (oy + 1 - c.v[1]) * RX + (ox + 1 - c.v[0]);
          f[k] = lds[fuse_slot<false, k>(it - src_it) * R + rr];
        });
        if (ri.lo[0] || ri.hi[0]) {
          // the face's 2D - 1 unknowns from B's row slots (half-way: minus the
          // node's own step-1 f*_kbar, from LDS), every load issued before
          // any is used
          const bool lo = ri.lo[0];
          const int own = (oy + 1) * RX + (ox + 1);
          // LDS element of the own f*_kbar of face population k on face fc
          auto own_at = [&](auto K, int fc) {
            constexpr int k = decltype(K)::value;
            if constexpr (vel_comp(D, k, 2) == 1)
              return S::SLOTS * R + (((it - 1) & 1) * 2 + fc) * RY + oy + 1;
            else
              return fuse_slot<false, opp_index(D, k)>(it - 1) * R + own;
          };
          T fx[2 * D - 1], sb[2 * D - 1];
          static_for<0, 2 * D - 1>([&](auto Sx) {
            constexpr int sl = decltype(Sx)::value;
            constexpr int kl = face_pop(D, 1, sl), kh = face_pop(D, -1, sl);
            fx[sl] = B[(lo ? kl : kh) * ps + p.xoff + row];
            if constexpr (HALF)
              sb[sl] = lds[lo ? own_at(std::integral_constant<int, kl>{}, 0)
                              : own_at(std::integral_constant<int, kh>{}, 1)];
          });
          asm volatile("" ::: "memory");
          static_for<0, 2 * D - 1>([&](auto Sx) {
            constexpr int sl = decltype(Sx)::value;
            constexpr int kl = face_pop(D, 1, sl), kh = face_pop(D, -1, sl);
            T v = fx[sl];
            if constexpr (HALF) v -= sb[sl];
            if (lo) f[kl] = v;
            else f[kh] = v;
          });
        }
        collide_store<D, T>(f, B, ps, node, p);
      }
    }
    __syncthreads();
  }
}

// The two-step pass for d = 2: a block owns TX nodes of x_1 and a chunk of
// x_2 rows and marches along x_2 (rows play the part of the planes of
// k_fused2, with no halo across x_2 besides the marching itself).  Rows on a
// Dirichlet wall of x_2 go through C as in k_fused2.
// One tile (x_1 nodes x0 .. x0 + TX - 1, output rows yc0 .. yend - 1) of the
// d = 2 two-step pass; lds holds the block's SLOTS x (TX + 2) row-slots.
template <class T, bool HALF>
__device__ __forceinline__ void fused2_d2_tile(const T* __restrict__ A, T* __restrict__ B,
                                               T* __restrict__ C, const KParams& p, T* lds,
                                               const int x0, const int yc0, const int yend) {
  using S = FuseShape2<T, HALF>;
  constexpr int D = 2, Q = q_of(2), TX = S::TX, NT = S::NT;
  constexpr int R = TX + 2;
  static_assert(TX == NT, "one output node per thread");
  const long long ps = p.pstride;
  const int n0 = p.n[0], n1 = p.n[1];
  const int iters = yend - yc0 + 2;
  const int r = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
    const int yp = yc0 - 1 + it;  // step-1 row of this iteration
    // ---- step 1 on the tile and its halo of row yp
    for (int rr = r; rr < R; rr += NT) {
      int gx = x0 - 1 + rr, gy = yp;
      bool skip = false;
      if (gx < 0 || gx >= n0) {
        if (p.bc[0] != 0) skip = true;
        else gx = fuse_wrap(gx, n0);
      }
      if (gy < 0 || gy >= n1) {
        if (p.bc[1] != 0) skip = true;
        else gy = fuse_wrap(gy, n1);
      }
      if (!skip) {
        const int row = gy;
        RowInfo<D> ri;
        row_setup<D>(p, row, ri);
        col_setup<D>(p, gx, ri);
        const int node = ri.rowbase + gx;
        T f[Q];
        if (ri.rowwall) {
          static_for<0, Q>([&](auto K) {
            constexpr int k = decltype(K)::value;
            f[k] = C[k * ps + node];
          });
        } else {
          static_for<0, Q>([&](auto K) {
            constexpr int k = decltype(K)::value;
            constexpr int cx = vel_comp(D, k, 0);
            int idx = node + pull_offset<D, k>(ri);
            if constexpr (cx != 0) {
              if ((cx == 1) ? ri.lo[0] : ri.hi[0]) idx = p.xoff + row;
            }
            f[k] = A[k * ps + idx];
          });
          if (HALF && (ri.lo[0] || ri.hi[0])) {
            static_for<0, Q>([&](auto K) {
              constexpr int k = decltype(K)::value;
              constexpr int cx = vel_comp(D, k, 0);
              if constexpr (cx != 0) {
                if ((cx == 1) ? ri.lo[0] : ri.hi[0]) f[k] -= A[opp_index(D, k) * ps + node];
              }
            });
          }
          collide_vals<D, T>(f, p);
          // rows next to a wall of x_2, owned by this block: kept for the
          // step-2 wall kernel
          const bool own = rr >= 1 && rr <= TX && x0 - 1 + rr < n0 && yp >= yc0 && yp < yend;
          const bool near = p.bc[1] != 0 && (ri.i[1] == 1 || ri.i[1] == n1 - 2);
          if (own && near) {
#pragma unroll
            for (int k = 0; k < Q; ++k) __builtin_nontemporal_store(f[k], C + k * ps + node);
          }
        }
        static_for<0, Q>([&](auto K) {
          constexpr int k = decltype(K)::value;
          lds[fuse_slot2<HALF, k>(it) * R + rr] = f[k];
        });
      }
    }
    __syncthreads();
    // ---- step 2 on output row yp - 1
    if (it >= 2 && r < TX) {
      const int gy = yp - 1;
      const int gx = x0 + r;
      if (gx < n0) {
        const int row = gy;
        RowInfo<D> ri;
        row_setup<D>(p, row, ri);
        if (!ri.rowwall) {
          col_setup<D>(p, gx, ri);
          const int node = ri.rowbase + gx;
          // pulls from LDS, x_1-face unknowns from B's row slots (as k_fused2)
          T f[Q];
          static_for<0, Q>([&](auto K) {
            constexpr int k = decltype(K)::value;
            constexpr Vec4i c = vel_vec(D, k);
            constexpr int src_it = c.v[1] == 0 ? 1 : (c.v[1] == 1 ? 2 : 0);
            f[k] = lds[fuse_slot2<HALF, k>(it - src_it) * R + (r + 1 - c.v[0])];
          });
          if (ri.lo[0] || ri.hi[0]) {
            static_for<0, Q>([&](auto K) {
              constexpr int k = decltype(K)::value;
              constexpr int cx = vel_comp(D, k, 0);
              if constexpr (cx != 0) {
                if ((cx == 1) ? ri.lo[0] : ri.hi[0]) f[k] = B[k * ps + p.xoff + row];
              }
            });
          }
          if (HALF && (ri.lo[0] || ri.hi[0])) {
            static_for<0, Q>([&](auto K) {
              constexpr int k = decltype(K)::value;
              constexpr int cx = vel_comp(D, k, 0);
              if constexpr (cx != 0) {
                constexpr int kb = opp_index(D, k);
                if ((cx == 1) ? ri.lo[0] : ri.hi[0])
                  f[k] -= lds[fuse_slot2<HALF, kb>(it - 1) * R + (r + 1)];
              }
            });
          }
          collide_store<D, T>(f, B, ps, node, p);
        }
      }
    }
    __syncthreads();
  }
}

template <class T, bool HALF>
__global__ void __launch_bounds__(256)
    k_fused2_d2(const T* __restrict__ A, T* __restrict__ B, T* __restrict__ C, const KParams p,
                const int yc) {
  extern __shared__ __align__(16) unsigned char fuse_lds[];
  int tx_, ty_;
  fuse_tile2(p, FuseShape2<T, HALF>::TX, tx_, ty_);
  const int yc0 = ty_ * yc;
  fused2_d2_tile<T, HALF>(A, B, C, p, reinterpret_cast<T*>(fuse_lds),
                          tx_ * FuseShape2<T, HALF>::TX, yc0, min(yc0 + yc, p.n[1]));
}

// Two steps of many periodic d = 2 lattices in one launch: block b takes tile
// tiles[b] (instance, x_1 start, row range) with the instance's parameter
// block and buffers (cur selects the source).
template <class T>
__global__ void __launch_bounds__(256)
    k_fused2_d2_batch(const KParams* __restrict__ kps, T* const* __restrict__ bufs,
                      const BatchTile2* __restrict__ tiles, const int cur) {
  extern __shared__ __align__(16) unsigned char fuse_lds[];
  const BatchTile2 t = tiles[blockIdx.x];
  fused2_d2_tile<T, false>(bufs[2 * t.inst + cur], bufs[2 * t.inst + 1 - cur], nullptr,
                           kps[t.inst], reinterpret_cast<T*>(fuse_lds), t.x0, t.y0, t.y1);
}

// Every pair of steps of a call for a batch of d = 2 lattices in one launch,
// one block per instance: block b takes instance order[b] and advances it
// through all npairs pairs, tile after tile of the instance's table
// (tiles[first[i] .. first[i + 1])), with the block barrier that ends each
// tile body as the only synchronisation (the instance's state never leaves
// its block, so no block waits for another).  Bitwise the result of the
// per-pair launches: the same tile body on the same tiles.
template <class T>
__global__ void __launch_bounds__(256)
    k_fused2_d2_resident(const KParams* __restrict__ kps, T* const* __restrict__ bufs,
                         const BatchTile2* __restrict__ tiles, const int* __restrict__ first,
                         const int* __restrict__ order, const int npairs, const int cur) {
  extern __shared__ __align__(16) unsigned char fuse_lds[];
  const int inst = order[blockIdx.x];
  const KParams& p = kps[inst];
  const int t0 = first[inst], t1 = first[inst + 1];
  for (int pair = 0; pair < npairs; ++pair) {
    const int c = (cur + pair) & 1;
    const T* A = bufs[2 * inst + c];
    T* B = bufs[2 * inst + 1 - c];
    for (int t = t0; t < t1; ++t) {
      const BatchTile2 tl = tiles[t];
      fused2_d2_tile<T, false>(A, B, nullptr, p, reinterpret_cast<T*>(fuse_lds), tl.x0, tl.y0,
                               tl.y1);
    }
    // this pair's output (B) is read by the next pair: the block's global
    // stores must be visible to all of its threads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
}

// Many lattices in one launch (periodic instances): block b updates rows
// tiles[b].row0 .. + blockDim.y - 1 of instance tiles[b].inst, whose parameter
// block is kps[inst] and whose two state buffers are bufs[2 inst], bufs[2 inst + 1]
// (cur selects the source).
template <int D, class T>
__global__ void __launch_bounds__(256)
    k_step_batch(const KParams* __restrict__ kps, T* const* __restrict__ bufs,
                 const BatchTile* __restrict__ tiles, const int cur) {
  const BatchTile t = tiles[blockIdx.x];
  const KParams& p = kps[t.inst];
  const int row = t.row0 + threadIdx.y;
  if (row >= p.rows) return;
  step_row<D, T>(bufs[2 * t.inst + cur], bufs[2 * t.inst + 1 - cur], p, row);
}

// Split representation: phi (float64) and g_k = f_k - omega_k phi (float32),
// pre-collision.  f*_k(y) = omega_k (phi(y) + dt R) + (1 - s) g_k(y), so the
// pull needs phi and g_k at the upwind node only; arithmetic is float64.
// Every kernel of the mode evaluates f* from t = split_src(phi) with
// split_fstar_t (two-step passes equal single steps bit for bit); the passes
// that keep phi of a plane in LDS keep t, formed once per node.
__device__ __forceinline__ double split_src(double phi, const KParams& p) { return phi + p.dtR; }

__device__ __forceinline__ double split_fstar_t(double omega, double t, float g,
                                                const KParams& p) {
  return fma(omega, t, (1.0 - p.s) * static_cast<double>(g));
}

__device__ __forceinline__ double split_fstar_val(double omega, double phi, float g,
                                                  const KParams& p) {
  return split_fstar_t(omega, split_src(phi, p), g, p);
}

// phi of a split-layout mode: float64, or (hi/lo mode) the unevaluated sum
// hi + lo of two float32 with |lo| <= ulp(hi) / 2
typedef float hilo_vec __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double phi_get(const double* __restrict__ ph, long long i) {
  return ph[i];
}
__device__ __forceinline__ double phi_get(const float2* __restrict__ ph, long long i) {
  const float2 v = ph[i];
  return static_cast<double>(v.x) + static_cast<double>(v.y);
}
__device__ __forceinline__ float2 hilo_of(double v) {
  const float h = static_cast<float>(v);
  return make_float2(h, static_cast<float>(v - static_cast<double>(h)));
}
__device__ __forceinline__ void phi_put(double* __restrict__ ph, long long i, double v) {
  __builtin_nontemporal_store(v, ph + i);
}
__device__ __forceinline__ void hilo_put(float2* __restrict__ ph, long long i, float2 v) {
  const hilo_vec w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<hilo_vec*>(ph) + i);
}
__device__ __forceinline__ void phi_put(float2* __restrict__ ph, long long i, double v) {
  hilo_put(ph, i, hilo_of(v));
}

template <int D, class PT>
__device__ __forceinline__ void split_pull(double (&f)[q_of(D)], const float* __restrict__ gsrc,
                                           const PT* __restrict__ phisrc, long long ps,
                                           int node, const RowInfo<D>& r, const KParams& p) {
  static_for<0, q_of(D)>([&](auto K) {
    constexpr int k = decltype(K)::value;
    const int idx = node + pull_offset<D, k>(r);
    f[k] = split_fstar_val(p.omega[k], phi_get(phisrc, idx), gsrc[k * ps + idx], p);
  });
}

template <int D, class PT>
__device__ __forceinline__ double split_fstar(const float* __restrict__ gsrc,
                                              const PT* __restrict__ phisrc, long long ps,
                                              int node, int kb, const KParams& p) {
  return split_fstar_val(p.omega[kb], phi_get(phisrc, node), gsrc[kb * ps + node], p);
}

template <int D, class PT>
__device__ __forceinline__ void split_store(const double (&f)[q_of(D)], float* __restrict__ gdst,
                                            PT* __restrict__ phidst, long long ps, int node,
                                            const KParams& p) {
  constexpr int Q = q_of(D);
  double phi = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) phi += f[k];
  phi_put(phidst, node, phi);
#pragma unroll
  for (int k = 0; k < Q; ++k)
    __builtin_nontemporal_store(static_cast<float>(f[k] - p.omega[k] * phi), gdst + k * ps + node);
}

// ---- hi/lo mode: the step in float32 arithmetic.  With b_k = f_k - omega_k
// (phi(x) + dt R) at the node x being updated (sum_k omega_k = 1):
//   bulk population, pulled from y = x - c_k:
//     b_k = omega_k (phi(y) - phi(x)) + (1 - s) g_k(y);
//   population set by a wall scheme to the value v (float64):
//     b_k = v - omega_k (phi(x) + dt R);
//   beta = sum_k b_k, phi_new = phi(x) + dt R + beta, g_new_k = b_k - omega_k beta.
// Every quantity is kept free of rounding until g_new_k and phi_new are
// rounded once: phi(y) - phi(x) as the pair (hi' - hi, lo' - lo) (exact for
// neighbouring values, Sterbenz), omega_k as the float32 pair omega_f +
// omega_lo, the product omega_f (hi' - hi) with its exact error (fma), beta
// as a TwoSum over those products plus the small terms, dt R as an exact
// float32 pair.  Rounded to float32 on the way, the first-order differences
// and the weights repeat nearly the same error every step, which then adds
// up like a bias (measured: 4e-8 drift from float64 after 2000 steps at 512^3,
// where the split mode drifts 1e-9).  The helpers disable floating-point
// contraction, which would break the error-free sums.  Every kernel of the
// mode uses them in the same order (two-step passes equal single steps bit
// for bit); rows on walls of x_2.. go through the float64 split formulas
// (split_pull / split_store on the pair), in single steps and pairs alike.
struct HiloTerm {
  float p;  // omega_f (hi' - hi), rounded
  float q;  // (1 - s) g_k(y)
  float r;  // the error of p plus the small terms
};

__device__ __forceinline__ HiloTerm hilo_term(int k, float2 py, float2 own, float g,
                                              const KParams& p) {
#pragma clang fp contract(off)
  const float dh = py.x - own.x, dl = py.y - own.y;
  const float pp = p.omega_f[k] * dh;
  const float ep = fmaf(p.omega_f[k], dh, -pp);
  return {pp, p.oms_f * g, fmaf(p.omega_lo[k], dh, fmaf(p.omega_f[k], dl, ep))};
}

// a b_k given in float64 (wall-set populations)
__device__ __forceinline__ HiloTerm hilo_term_of(double b) {
  const float h = static_cast<float>(b);
  return {h, 0.0f, static_cast<float>(b - static_cast<double>(h))};
}

__device__ __forceinline__ void two_sum_f(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  const float bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

struct HiloAcc {
  float s = 0.0f, c = 0.0f, q = 0.0f, r = 0.0f;
};

__device__ __forceinline__ void hilo_add(HiloAcc& acc, const HiloTerm& t) {
#pragma clang fp contract(off)
  float e;
  two_sum_f(acc.s, t.p, acc.s, e);
  acc.c += e;
  acc.q += t.q;
  acc.r += t.r;
}

// beta as a normalised pair
__device__ __forceinline__ float2 hilo_beta(const HiloAcc& acc) {
#pragma clang fp contract(off)
  const float t = (acc.c + acc.r) + acc.q;
  const float h = acc.s + t;
  return make_float2(h, t - (h - acc.s));
}

// g_new_k = b_k - omega_k beta, rounded once
__device__ __forceinline__ float hilo_gnew(int k, const HiloTerm& t, float2 beta,
                                           const KParams& p) {
#pragma clang fp contract(off)
  const float m = p.omega_f[k] * beta.x;
  const float em = fmaf(p.omega_f[k], beta.x, -m);
  float d, ed;
  two_sum_f(t.p, -m, d, ed);
  const float small =
      fmaf(-p.omega_f[k], beta.y, fmaf(-p.omega_lo[k], beta.x, (ed - em) + t.r));
  return d + (t.q + small);
}

// (hi + lo) + (dtR_hi + dtR_lo) + beta as a normalised pair
__device__ __forceinline__ float2 hilo_advance(float2 v, float2 beta, const KParams& p) {
#pragma clang fp contract(off)
  float s1, e1, s2, e2;
  two_sum_f(v.x, p.dtR_hi, s1, e1);
  two_sum_f(s1, beta.x, s2, e2);
  const float lo = (((v.y + p.dtR_lo) + beta.y) + e1) + e2;
  const float h = s2 + lo;
  return make_float2(h, lo - (h - s2));
}

// the step of one node from its terms: term(K) gives HiloTerm of population
// K; it is evaluated twice (beta first, then g_new), and a compiler memory
// barrier between the passes makes the second pass reload its LDS inputs
// instead of holding three values per population in registers
template <int D, class Term>
__device__ __forceinline__ void hilo_node(Term&& term, float2 own, float2& phi_new,
                                          float (&g)[q_of(D)], const KParams& p) {
  HiloAcc acc;
  static_for<0, q_of(D)>([&](auto K) { hilo_add(acc, term(K)); });
  const float2 beta = hilo_beta(acc);
  phi_new = hilo_advance(own, beta, p);
  asm volatile("" ::: "memory");
  static_for<0, q_of(D)>([&](auto K) {
    constexpr int k = decltype(K)::value;
    g[k] = hilo_gnew(k, term(K), beta, p);
  });
}

template <int D>
__global__ void __launch_bounds__(256)
    k_step_split(const float* __restrict__ gsrc, float* __restrict__ gdst,
                 const double* __restrict__ phisrc, double* __restrict__ phidst, const KParams p) {
  constexpr int Q = q_of(D);
  constexpr int S = 2 * D - 1;
  const int row = blockIdx.x * blockDim.y + threadIdx.y;
  if (row >= p.rows) return;
  RowInfo<D> r;
  row_setup<D>(p, row, r);
  if (r.rowwall) return;
  const long long ps = p.pstride;
  const bool half = p.scheme == kHalfWay;
  for (int x = threadIdx.x; x < p.n[0]; x += blockDim.x) {
    col_setup<D>(p, x, r);
    const int node = r.rowbase + x;
    double f[Q];
    split_pull<D>(f, gsrc, phisrc, ps, node, r, p);
    if (r.lo[0] || r.hi[0]) {
      const double* W = p.xdata + (r.hi[0] ? S * p.rows : 0) + row;
      static_for<0, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        constexpr int cx = vel_comp(D, k, 0);
        if constexpr (cx != 0) {
          if ((cx == 1) ? r.lo[0] : r.hi[0]) {
            double v = W[(long long)xface_slot(D, k) * p.rows];
            if (half) v -= split_fstar<D>(gsrc, phisrc, ps, node, opp_index(D, k), p);
            f[k] = v;
          }
        }
      });
    }
    split_store<D>(f, gdst, phidst, ps, node, p);
  }
}

// One step of the hi/lo mode (the b_k form above).
template <int D>
__global__ void __launch_bounds__(256)
    k_step_hilo(const float* __restrict__ gsrc, float* __restrict__ gdst,
                const float2* __restrict__ phisrc, float2* __restrict__ phidst, const KParams p) {
  constexpr int Q = q_of(D);
  constexpr int S = 2 * D - 1;
  const int row = blockIdx.x * blockDim.y + threadIdx.y;
  if (row >= p.rows) return;
  RowInfo<D> r;
  row_setup<D>(p, row, r);
  if (r.rowwall) return;
  const long long ps = p.pstride;
  const bool half = p.scheme == kHalfWay;
  for (int x = threadIdx.x; x < p.n[0]; x += blockDim.x) {
    col_setup<D>(p, x, r);
    const int node = r.rowbase + x;
    const float2 own = phisrc[node];
    float2 py[Q];
    float gy[Q];
    static_for<0, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      const int idx = node + pull_offset<D, k>(r);
      py[k] = phisrc[idx];
      gy[k] = gsrc[k * ps + idx];
    });
    const double phx = static_cast<double>(own.x) + static_cast<double>(own.y);
    const double* W = p.xdata + (r.hi[0] ? S * p.rows : 0) + row;
    auto term = [&](auto K) -> HiloTerm {
      constexpr int k = decltype(K)::value;
      constexpr int cx = vel_comp(D, k, 0);
      if constexpr (cx != 0) {
        if ((cx == 1) ? r.lo[0] : r.hi[0]) {
          double v = W[(long long)xface_slot(D, k) * p.rows];
          if (half) {
            constexpr int kb = opp_index(D, k);
            v -= split_fstar_val(p.omega[kb], phx, gsrc[kb * ps + node], p);
          }
          return hilo_term_of(v - p.omega[k] * (phx + p.dtR));
        }
      }
      return hilo_term(k, py[k], own, gy[k], p);
    };
    float2 phi_new;
    float g[Q];
    hilo_node<D>(term, own, phi_new, g, p);
    hilo_put(phidst, node, phi_new);
#pragma unroll
    for (int k = 0; k < Q; ++k) __builtin_nontemporal_store(g[k], gdst + k * ps + node);
  }
}

// Two fused steps of the split representation (d = 3), organised as k_fused2:
// the LDS keeps the step-1 g_k (float32, the same plane slots) and
// t = split_src(phi) (float64, a ring of three planes).  The x_1-face data of
// step 2 come from a second x-face array (xd2); rows on and next to the walls
// of x_2 / x_3 go through the scratch state (gC, phiC) as in k_fused2.
//
// Step 1 pulls phi from the 19 upwind nodes of every node of its region.  A
// third ring of three planes holds t of the source phi over the region and a
// halo of one more node, (TX + 4)(TY + 4) values per plane, loaded once per
// plane.  Gathered from global memory instead, every source plane is read 19
// times per node over three iterations, more than the L2 of an XCD holds
// (measured: 1.67x the algorithmic reads of the pass, 1.17x with the ring).
//
// With half-way x_1 walls an x_1-face node of output plane z - 1 also needs its
// own step-1 g of every kbar opposite an unknown; of these only kbar =
// (-+1, 0, -1) has c_3 = -1, whose single slot the next plane overwrites, so a
// side buffer keeps that one value per face node (two faces x (TY + 2) rows x
// two plane parities), as in the forward pass, and the tile is the full-way one.
template <bool HALF>
struct FuseSplitShape {
  static constexpr int TX = 64, TY = 10, NT = 1024, SLOTS = 38;
  static constexpr int SIDE = HALF ? 4 * (TY + 2) : 0;
};

// bytes of LDS of a split pass: g slots, the step-1 phi ring, the source phi
// ring, the half-way side buffer
template <bool HALF>
constexpr size_t fuse_split_lds() {
  using S = FuseSplitShape<HALF>;
  return sizeof(float) * S::SLOTS * (S::TX + 2) * (S::TY + 2) +
         sizeof(double) * 3 * (S::TX + 2) * (S::TY + 2) +
         sizeof(double) * 3 * (S::TX + 4) * (S::TY + 4) + sizeof(float) * S::SIDE;
}

// HILO: the hi/lo mode, whose rings hold the (hi, lo) pairs of phi instead of t.
template <bool HALF, bool HILO>
__global__ void __launch_bounds__((FuseSplitShape<HALF>::NT))
    k_fused2_split(const float* __restrict__ gA, float* __restrict__ gB, float* __restrict__ gC,
                   const std::conditional_t<HILO, float2, double>* __restrict__ phiA,
                   std::conditional_t<HILO, float2, double>* __restrict__ phiB,
                   std::conditional_t<HILO, float2, double>* __restrict__ phiC, const KParams p,
                   const double* __restrict__ xd2, const int zc) {
  using S = FuseSplitShape<HALF>;
  using PT = std::conditional_t<HILO, float2, double>;
  static_assert(sizeof(PT) == sizeof(double), "both rings hold 8 bytes per node");
  constexpr int D = 3, Q = q_of(3), TX = S::TX, TY = S::TY, NT = S::NT;
  constexpr int RX = TX + 2, RY = TY + 2, R = RX * RY;
  constexpr int PX = TX + 4, PY = TY + 4, P2 = PX * PY;
  constexpr int SX = 2 * D - 1;
  extern __shared__ __align__(16) unsigned char fuse_lds[];
  float* lg = reinterpret_cast<float*>(fuse_lds);
  PT* lphi = reinterpret_cast<PT*>(fuse_lds + sizeof(float) * S::SLOTS * R);
  PT* lsrc = lphi + 3 * R;
  // half-way only: side[((parity * 2) + face) * RY + ry]
  float* side = reinterpret_cast<float*>(lsrc + 3 * P2);
  const long long ps = p.pstride;
  const int n0 = p.n[0], n1 = p.n[1], n2 = p.n[2];
  int tx_, ty_, tz_;
  fuse_tile(p, TX, TY, tx_, ty_, tz_);
  const int x0 = tx_ * TX, y0 = ty_ * TY, zc0 = tz_ * zc;
  const int zend = min(zc0 + zc, n2);
  const int iters = zend - zc0 + 2;
  // ring value of a node's phi: t = split_src(phi), or the hi/lo pair itself
  auto ring_val = [&](PT v) -> PT {
    if constexpr (HILO) return v;
    else return split_src(v, p);
  };
  // The source phi of plane z (zc0 - 2 <= z <= zend + 1) goes to ring slot
  // (z - zc0 + 2) mod 3 at (x_1, x_2) = (x0 - 2 + sx, y0 - 2 + sy): the TX
  // interior columns of every row first (aligned wavefront loads), then the
  // four halo columns.  Every thread loads and writes one position in every
  // iteration, with no branch, so that the compiler's wait for the load is the
  // one before the ring write and never a wait at the loop head, which would
  // also wait for the previous iteration's stores.  So threads past the P2
  // positions repeat those of threads tid - P2 (the same value to the same
  // LDS word), and positions outside a Dirichlet axis hold the value of the
  // nearest node inside: they are read only by pulls whose result the x_1-face
  // data replace (rows on the walls of x_2 / x_3 pull nothing), and planes
  // outside a Dirichlet x_3 axis or past the chunk are never read.
  static_assert(P2 <= NT && NT - P2 <= P2, "one or two threads per source-ring position");
  auto ring_xy = [&](int t, int& sx, int& sy) {
    if (t < TX * PY) {
      sy = t / TX;
      sx = 2 + t % TX;
    } else {
      const int h = t - TX * PY;
      sy = h >> 2;
      sx = (h & 3) < 2 ? (h & 3) : TX + (h & 3);
    }
  };
  int sx, sy;
  ring_xy(static_cast<int>(threadIdx.x) < P2 ? static_cast<int>(threadIdx.x)
                                              : static_cast<int>(threadIdx.x) - P2,
          sx, sy);
  auto ring_axis = [&](int i, int n, int a) {
    if (i >= 0 && i < n) return i;
    return p.bc[a] != 0 ? min(max(i, 0), n - 1) : fuse_wrap(i, n);
  };
  const int sgx = ring_axis(x0 - 2 + sx, n0, 0), sgy = ring_axis(y0 - 2 + sy, n1, 1);
  const int s_off = sy * PX + sx;
  auto stage_load = [&](int z) -> PT {
    const int gz = ring_axis(z, n2, 2);
    return phiA[(static_cast<long long>(gz) * n1 + sgy) * n0 + sgx];
  };
  auto stage_put = [&](int z, PT v) { lsrc[((z - zc0 + 2) % 3) * P2 + s_off] = ring_val(v); };
  // the hi/lo pass's staging after step 2, positions recomputed per call
  auto stage_late = [&](int z) {
    const int gz = ring_axis(z, n2, 2);
    const int t = threadIdx.x;
    if (t >= P2) return;
    int tx, ty;
    ring_xy(t, tx, ty);
    const int gx = ring_axis(x0 - 2 + tx, n0, 0), gy = ring_axis(y0 - 2 + ty, n1, 1);
    lsrc[((z - zc0 + 2) % 3) * P2 + ty * PX + tx] =
        ring_val(phiA[(static_cast<long long>(gz) * n1 + gy) * n0 + gx]);
  };
  {
    const PT v0 = stage_load(zc0 - 2), v1 = stage_load(zc0 - 1), v2 = stage_load(zc0);
    stage_put(zc0 - 2, v0);
    stage_put(zc0 - 1, v1);
    stage_put(zc0, v2);
  }
  __syncthreads();
  for (int it = 0; it < iters; ++it) {
    const int zp = zc0 - 1 + it;
    // The source plane zp + 2 of the next iteration replaces plane zp - 1 (ring
    // slot it mod 3) after the barrier that ends step 1, the last reader of
    // that plane.  The split pass loads it here, so that the load is in flight
    // with step 1's gathers.  Loaded after step 2 instead, the wait for it
    // before the ring write also waits for all of step 2's stores, since the
    // vector-memory counter covers stores on this chip: 6.60 against 6.07 ms
    // per 512^3 launch.  (In the last iteration the plane is loaded and written
    // but not read.)  The hi/lo pass stages after step 2 (below): its step 1
    // spills registers, and the value and ring position held through the loop
    // made it spill more (16.9 and 18.7 ms against 15.7 ms, loaded before and
    // after step 1).
    PT nxt{};
    if constexpr (!HILO) nxt = stage_load(zp + 2);
    // fuse_region order: a wavefront's gathers start on the tile's aligned
    // x_1 origin (measured 7% faster than plain region order at 512^3)
    for (int t = threadIdx.x; t < R; t += NT) {
      const int r = fuse_region<TX, TY>(t);
      const int rx = r % RX, ry = r / RX;
      int gx = x0 - 1 + rx, gy = y0 - 1 + ry, gz = zp;
      if (gx < 0 || gx >= n0) {
        if (p.bc[0] != 0) continue;
        gx = fuse_wrap(gx, n0);
      }
      if (gy < 0 || gy >= n1) {
        if (p.bc[1] != 0) continue;
        gy = fuse_wrap(gy, n1);
      }
      if (gz < 0 || gz >= n2) {
        if (p.bc[2] != 0) continue;
        gz = fuse_wrap(gz, n2);
      }
      const int row = gz * n1 + gy;
      RowInfo<D> ri;
      row_setup_yz(p, gy, gz, ri);
      col_setup<D>(p, gx, ri);
      const int node = ri.rowbase + gx;
      float g[Q];
      PT phi;
      if (ri.rowwall) {
        phi = phiC[node];
        static_for<0, Q>([&](auto K) {
          constexpr int k = decltype(K)::value;
          g[k] = gC[k * ps + node];
        });
      } else {
        // the pull with phi from the source ring: plane zp - c_3 is in slot
        // (it + 1 - c_3) mod 3
        const int sown = (ry + 1) * PX + rx + 1;
        const PT* s0 = lsrc + ((it + 1) % 3) * P2 + sown;
        if constexpr (HILO) {
          const float2 own = *s0;
          const double phx = static_cast<double>(own.x) + static_cast<double>(own.y);
          float gy[Q];
          static_for<0, Q>([&](auto K) {
            constexpr int k = decltype(K)::value;
            gy[k] = gA[k * ps + node + pull_offset<D, k>(ri)];
          });
          const double* W = p.xdata + (ri.hi[0] ? SX * p.rows : 0) + row;
          auto term = [&](auto K) -> HiloTerm {
            constexpr int k = decltype(K)::value;
            constexpr int cx = vel_comp(D, k, 0);
            if constexpr (cx != 0) {
              if ((cx == 1) ? ri.lo[0] : ri.hi[0]) {
                double v = W[(long long)xface_slot(D, k) * p.rows];
                if (HALF) {
                  constexpr int kb = opp_index(D, k);
                  v -= split_fstar_val(p.omega[kb], phx, gA[kb * ps + node], p);
                }
                return hilo_term_of(v - p.omega[k] * (phx + p.dtR));
              }
            }
            constexpr Vec4i c = vel_vec(D, k);
            const PT* sp = c.v[2] == 0 ? s0 : lsrc + ((it + 1 - c.v[2]) % 3) * P2 + sown;
            return hilo_term(k, sp[-c.v[1] * PX - c.v[0]], own, gy[k], p);
          };
          hilo_node<D>(term, own, phi, g, p);
        } else {
          // all 19 gathers issued before any is used: at its register limit
          // the half-way pass otherwise took them one to four at a time, each
          // followed by a wait for all outstanding loads (10.6 ms per 512^3
          // launch against 5.8 ms full-way)
          float gy[Q];
          static_for<0, Q>([&](auto K) {
            constexpr int k = decltype(K)::value;
            gy[k] = gA[k * ps + node + pull_offset<D, k>(ri)];
          });
          asm volatile("" ::: "memory");
          double f[Q];
          static_for<0, Q>([&](auto K) {
            constexpr int k = decltype(K)::value;
            constexpr Vec4i c = vel_vec(D, k);
            const PT* sp = c.v[2] == 0 ? s0 : lsrc + ((it + 1 - c.v[2]) % 3) * P2 + sown;
            const double ph = sp[-c.v[1] * PX - c.v[0]];
            f[k] = split_fstar_t(p.omega[k], ph, gy[k], p);
          });
          if (ri.lo[0] || ri.hi[0]) {
            const double* W = p.xdata + (ri.hi[0] ? SX * p.rows : 0) + row;
            static_for<0, Q>([&](auto K) {
              constexpr int k = decltype(K)::value;
              constexpr int cx = vel_comp(D, k, 0);
              if constexpr (cx != 0) {
                if ((cx == 1) ? ri.lo[0] : ri.hi[0]) {
                  double v = W[(long long)xface_slot(D, k) * p.rows];
                  if (HALF) {
                    constexpr int kb = opp_index(D, k);
                    v -= split_fstar_t(p.omega[kb], *s0, gA[kb * ps + node], p);
                  }
                  f[k] = v;
                }
              }
            });
          }
          // split_store's arithmetic, into registers
          phi = 0.0;
#pragma unroll
          for (int k = 0; k < Q; ++k) phi += f[k];
#pragma unroll
          for (int k = 0; k < Q; ++k) g[k] = static_cast<float>(f[k] - p.omega[k] * phi);
        }
        const bool own = rx >= 1 && rx <= TX && ry >= 1 && ry <= TY && x0 - 1 + rx < n0 &&
                         y0 - 1 + ry < n1 && zp >= zc0 && zp < zend;
        const bool near = (p.bc[1] != 0 && (ri.i[1] == 1 || ri.i[1] == n1 - 2)) ||
                          (p.bc[2] != 0 && (ri.i[2] == 1 || ri.i[2] == n2 - 2));
        if (own && near) {
          if constexpr (HILO) hilo_put(phiC, node, phi);
          else __builtin_nontemporal_store(phi, phiC + node);
#pragma unroll
          for (int k = 0; k < Q; ++k) __builtin_nontemporal_store(g[k], gC + k * ps + node);
        }
      }
      static_for<0, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        lg[fuse_slot<false, k>(it) * R + r] = g[k];
      });
      lphi[(it % 3) * R + r] = ring_val(phi);
      if constexpr (HALF) {
        if (!ri.rowwall && (ri.lo[0] || ri.hi[0])) {
          // g of kbar = (-+1, 0, -1) opposite the face's unknown (+-1, 0, +1),
          // for step 2 of this plane (read one iteration later)
          static_for<0, Q>([&](auto K) {
            constexpr int k = decltype(K)::value;
            constexpr int cx = vel_comp(D, k, 0);
            if constexpr (cx != 0 && vel_comp(D, k, 2) == 1) {
              if ((cx == 1) ? ri.lo[0] : ri.hi[0])
                side[((it & 1) * 2 + (cx == 1 ? 0 : 1)) * RY + ry] = g[opp_index(D, k)];
            }
          });
        }
      }
    }
    __syncthreads();
    if constexpr (!HILO) stage_put(zp + 2, nxt);
    if (it >= 2) {
      const int gz = zp - 1;
      for (int o = threadIdx.x; o < TX * TY; o += NT) {
        const int ox = o % TX, oy = o / TX;
        const int gx = x0 + ox, gy = y0 + oy;
        if (gx >= n0 || gy >= n1) continue;
        const int row = gz * n1 + gy;
        RowInfo<D> ri;
        row_setup_yz(p, gy, gz, ri);
        if (ri.rowwall) continue;
        col_setup<D>(p, gx, ri);
        const int node = ri.rowbase + gx;
        const int own = (oy + 1) * RX + (ox + 1);
        // the node's own step-1 g of kbar (half-way faces): the side buffer for
        // c_3(kbar) = -1, whose slot the current plane has overwritten
        auto own_g = [&](auto KB, int cx) -> float {
          constexpr int kb = decltype(KB)::value;
          if constexpr (vel_comp(D, kb, 2) == -1)
            return side[(((it - 1) & 1) * 2 + (cx == 1 ? 0 : 1)) * RY + oy + 1];
          else
            return lg[fuse_slot<false, kb>(it - 1) * R + own];
        };
        if constexpr (HILO) {
          const float2 me = lphi[((it - 1) % 3) * R + own];
          const double phx = static_cast<double>(me.x) + static_cast<double>(me.y);
          const double* W = xd2 + (ri.hi[0] ? SX * p.rows : 0) + row;
          auto term = [&](auto K) -> HiloTerm {
            constexpr int k = decltype(K)::value;
            constexpr int cx = vel_comp(D, k, 0);
            if constexpr (cx != 0) {
              if ((cx == 1) ? ri.lo[0] : ri.hi[0]) {
                double v = W[(long long)xface_slot(D, k) * p.rows];
                if constexpr (HALF) {
                  constexpr int kb = opp_index(D, k);
                  const float gb = own_g(std::integral_constant<int, kb>{}, cx);
                  v -= split_fstar_val(p.omega[kb], phx, gb, p);
                }
                return hilo_term_of(v - p.omega[k] * (phx + p.dtR));
              }
            }
            constexpr Vec4i c = vel_vec(D, k);
            constexpr int src_it = c.v[2] == 0 ? 1 : (c.v[2] == 1 ? 2 : 0);
            const int rr = (oy + 1 - c.v[1]) * RX + (ox + 1 - c.v[0]);
            return hilo_term(k, lphi[((it - src_it) % 3) * R + rr], me,
                             lg[fuse_slot<false, k>(it - src_it) * R + rr], p);
          };
          float2 phi_new;
          float g[Q];
          hilo_node<D>(term, me, phi_new, g, p);
          hilo_put(phiB, node, phi_new);
#pragma unroll
          for (int k = 0; k < Q; ++k) __builtin_nontemporal_store(g[k], gB + k * ps + node);
        } else {
          double f[Q];
          static_for<0, Q>([&](auto K) {
            constexpr int k = decltype(K)::value;
            constexpr Vec4i c = vel_vec(D, k);
            constexpr int src_it = c.v[2] == 0 ? 1 : (c.v[2] == 1 ? 2 : 0);
            const int rr = (oy + 1 - c.v[1]) * RX + (ox + 1 - c.v[0]);
            const double ph = lphi[((it - src_it) % 3) * R + rr];
            const float gk = lg[fuse_slot<false, k>(it - src_it) * R + rr];
            f[k] = split_fstar_t(p.omega[k], ph, gk, p);
          });
          if (ri.lo[0] || ri.hi[0]) {
            const double* W = xd2 + (ri.hi[0] ? SX * p.rows : 0) + row;
            static_for<0, Q>([&](auto K) {
              constexpr int k = decltype(K)::value;
              constexpr int cx = vel_comp(D, k, 0);
              if constexpr (cx != 0) {
                if ((cx == 1) ? ri.lo[0] : ri.hi[0]) {
                  double v = W[(long long)xface_slot(D, k) * p.rows];
                  if constexpr (HALF) {
                    constexpr int kb = opp_index(D, k);
                    const double ph = lphi[((it - 1) % 3) * R + own];
                    const float gb = own_g(std::integral_constant<int, kb>{}, cx);
                    v -= split_fstar_t(p.omega[kb], ph, gb, p);
                  }
                  f[k] = v;
                }
              }
            });
          }
          split_store<D>(f, gB, phiB, ps, node, p);
        }
      }
    }
    if constexpr (HILO) {
      if (it + 1 < iters) stage_late(zp + 2);
    }
    __syncthreads();
  }
}

// Rows on a wall of an axis >= 2.  Face (a, side), a >= 2, lists the rows
// with i_a at that side whose indices on the Dirichlet axes 2 <= b < a are
// interior, so every wall row is visited once; threads run along x_1 as in the
// bulk kernels, so loads and stores stay coalesced.
template <int D>
__device__ __forceinline__ int wall_row(const KParams& p, int idx) {
  int f = 0;
  while (f < p.nwfaces - 1 && idx >= p.wface_count[f]) {
    idx -= p.wface_count[f];
    ++f;
  }
  const int a0 = p.wface_axis[f];
  int l = idx, row = 0, rstride = 1;
#pragma unroll
  for (int b = 1; b < D; ++b) {
    int ib;
    if (b == a0) {
      ib = p.wface_side[f] ? p.n[b] - 1 : 0;
    } else {
      const bool inner = (b < a0) && p.bc[b] != 0;
      const int nb = inner ? p.n[b] - 2 : p.n[b];
      ib = l % nb + (inner ? 1 : 0);
      l /= nb;
    }
    row += ib * rstride;
    rstride *= p.n[b];
  }
  return row;
}

template <int D, class T, bool TAN, int V>
__global__ void __launch_bounds__(256)
    k_wall(const T* __restrict__ src, T* __restrict__ dst, const KParams p, const double t_n) {
  constexpr int Q = q_of(D);
  constexpr bool kF32 = std::is_same<T, float>::value;
  const int widx = blockIdx.x * blockDim.y + threadIdx.y;
  if (widx >= p.wall_rows) return;
  const int row = wall_row<D>(p, widx);
  RowInfo<D> r;
  row_setup<D>(p, row, r);
  const long long ps = p.pstride;
  // reference of the float32 deviations at t_{n+1}
  const double ref = kF32 ? p.phi_ref + p.R * (t_n + p.dt) : 0.0;
  auto update = [&](int x) {
    col_setup<D>(p, x, r);
    const int node = r.rowbase + x;
    T f[Q];
    auto fstar = [&](int kb) {
      return static_cast<double>(src[kb * ps + node]) + p.omega[kb] * ref;
    };
    if constexpr (D == 4 && kF32) {
      // the wall values first, then the pulls of the populations that enter
      // from inside: the 33 pulled values are not held across the wall formula
      // (212 to 151 VGPRs, three wavefronts per SIMD; float64 stays at two
      // either way and runs faster with the pulls first)
      wall_values<D, TAN, V, T>(f, p, r, t_n, ref, fstar);
      static_for<0, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if (!outside<D, k>(r)) f[k] = src[k * ps + node + pull_offset<D, k>(r)];
      });
    } else {
      static_for<0, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        f[k] = src[k * ps + node + pull_offset<D, k>(r)];
      });
      wall_values<D, TAN, V, T>(f, p, r, t_n, ref, fstar);
    }
    collide_store<D, T>(f, dst, ps, node, p);
  };
  if constexpr (D >= 3) {
    // one node per thread, the grid's y over x_1 chunks: in a loop over the
    // row the compiler kept the wall formula's per-population constants live
    // across it (d = 4: 256 VGPRs and one wavefront per SIMD; d = 3: 204
    // against 119 for the full-way cosine variant)
    const int x = blockIdx.y * blockDim.x + threadIdx.x;
    if (x < p.n[0]) update(x);
  } else {
    for (int x = threadIdx.x; x < p.n[0]; x += blockDim.x) update(x);
  }
}

template <int D, bool TAN, int V, class PT>
__global__ void __launch_bounds__(256)
    k_wall_split(const float* __restrict__ gsrc, float* __restrict__ gdst,
                 const PT* __restrict__ phisrc, PT* __restrict__ phidst, const KParams p,
                 const double t_n) {
  constexpr int Q = q_of(D);
  const int widx = blockIdx.x * blockDim.y + threadIdx.y;
  if (widx >= p.wall_rows) return;
  const int row = wall_row<D>(p, widx);
  RowInfo<D> r;
  row_setup<D>(p, row, r);
  const long long ps = p.pstride;
  auto update = [&](int x) {
    col_setup<D>(p, x, r);
    const int node = r.rowbase + x;
    double f[Q];
    split_pull<D>(f, gsrc, phisrc, ps, node, r, p);
    wall_values<D, TAN, V, double>(f, p, r, t_n, 0.0, [&](int kb) {
      return split_fstar<D>(gsrc, phisrc, ps, node, kb, p);
    });
    split_store<D>(f, gdst, phidst, ps, node, p);
  };
  if constexpr (D >= 3) {
    const int x = blockIdx.y * blockDim.x + threadIdx.x;  // as in k_wall
    if (x < p.n[0]) update(x);
  } else {
    for (int x = threadIdx.x; x < p.n[0]; x += blockDim.x) update(x);
  }
}

// ------------------------------------------------------------ node helpers --

template <int D>
__device__ __forceinline__ void node_index(const KParams& p, int node, int (&i)[D]) {
  int rr = node;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    i[a] = rr % p.n[a];
    rr /= p.n[a];
  }
}

template <int D>
__device__ __forceinline__ void node_coords(const KParams& p, const int (&i)[D], double (&x)[D]) {
#pragma unroll
  for (int a = 0; a < D; ++a) x[a] = p.origin[a] + (i[a] + p.shift[a]) * p.dx;
}

// ------------------------------------------------------------------ init ----

template <int D>
__device__ double fd4_derivative(const double* phi, const KParams& p, const int (&i)[D], int node,
                                 int a) {
  const int n = p.n[a];
  const int st = p.stride[a];
  auto at = [&](int s) {
    int j = i[a] + s;
    j = (j % n + n) % n;
    return phi[node + (j - i[a]) * st];
  };
  return (-at(2) + 8.0 * at(1) - 8.0 * at(-1) + at(-2)) / (12.0 * p.dx);
}

template <int D, class T>
__global__ void __launch_bounds__(256)
    k_init(T* __restrict__ dst, double* __restrict__ phidst, const double* __restrict__ phi0,
           const double* __restrict__ grad0, const KParams p, int mode) {
  constexpr int Q = q_of(D);
  const long long ps = p.pstride;
  for (int node = blockIdx.x * blockDim.x + threadIdx.x; node < p.nodes;
       node += gridDim.x * blockDim.x) {
    int i[D];
    node_index<D>(p, node, i);
    double phi, grad[D];
    if (phi0 == nullptr) {
      double x[D];
      node_coords<D>(p, i, x);
      field_initial<D>(p.field, p, x, phi, grad);
    } else {
      phi = phi0[node];
#pragma unroll
      for (int a = 0; a < D; ++a)
        grad[a] = (p.K == 3) ? (grad0 ? grad0[(long long)a * p.nodes + node]
                                      : fd4_derivative<D>(phi0, p, i, node, a))
                             : 0.0;
    }
    // f_k = omega_k [phi0 + tau dt (u - c_k) . grad phi0]  (eq. ini-simp at tau = 1/2)
    double f[Q];
    static_for<0, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr Vec4i c = vel_vec(D, k);
      double dir = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) dir += (p.u[a] - c.v[a]) * grad[a];
      f[k] = p.omega[k] * (p.K == 3 ? phi + p.tau * p.dt * dir : phi);
    });
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) sum += f[k];
    if (split_layout(mode)) {
      if (mode == kHiLo)
        reinterpret_cast<float2*>(phidst)[node] = hilo_of(sum);
      else
        phidst[node] = sum;
#pragma unroll
      for (int k = 0; k < Q; ++k)
        reinterpret_cast<float*>(dst)[k * ps + node] = static_cast<float>(f[k] - p.omega[k] * sum);
    } else {
      // post-collision state at t_0; float32 stores the deviation from
      // omega_k (phi_ref + R t_1)
      const double ref = (mode == kFP32) ? p.phi_ref + p.R * p.dt : 0.0;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const double fs = (1.0 - p.s) * f[k] + p.s * p.omega[k] * sum + p.dt * p.omega[k] * p.R;
        dst[k * ps + node] = static_cast<T>(fs - p.omega[k] * ref);
      }
    }
  }
}

// --------------------------------------------------------------- moments ----

__device__ __forceinline__ void block_reduce(double (&v)[kNumAcc], double* sh) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int m = 0; m < kNumAcc; ++m) sh[m * kRedThreads + tid] = v[m];
  __syncthreads();
  for (int half = kRedThreads / 2; half > 0; half >>= 1) {
    if (tid < half) {
#pragma unroll
      for (int m = 0; m < kNumAcc; ++m) {
        const double a = sh[m * kRedThreads + tid], b = sh[m * kRedThreads + tid + half];
        sh[m * kRedThreads + tid] = (m == 4) ? fmax(a, b) : a + b;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < kNumAcc; ++m) v[m] = sh[m * kRedThreads];
}

// accumulators: 0 sum phi, 1 sum phi^2, 2 sum (phi - phi*)^2,
// 3 sum_k f_k^2 / (2 omega_k), 4 max |phi|, 5 non-finite count
// `what` selects the work (kMom* bits of engine.hpp): without kMomRmse the
// per-node analytic field is not evaluated, without kMomEntropy the
// pre-collision populations are not rebuilt, and without any scalar bit no
// partial sums are written.
template <int D, class T>
__global__ void __launch_bounds__(kRedThreads)
    k_moments(const T* __restrict__ f, const double* __restrict__ phis, const KParams p,
              const int mode, const double t_n, double* __restrict__ phi_out,
              double* __restrict__ partial, const unsigned what) {
  constexpr int Q = q_of(D);
  __shared__ double sh[kNumAcc * kRedThreads];
  double acc[kNumAcc] = {0, 0, 0, 0, 0, 0};
  const long long ps = p.pstride;
  const bool want_err = (what & kMomRmse) && p.field.kind != kFieldNone;
  const bool want_ent = (what & kMomEntropy) != 0;
  const bool want_red = (what & (kMomSums | kMomRmse | kMomEntropy)) != 0;
  const double ref = (mode == kFP32) ? p.phi_ref + p.R * (t_n + p.dt) : 0.0;
  for (int node = blockIdx.x * blockDim.x + threadIdx.x; node < p.nodes;
       node += gridDim.x * blockDim.x) {
    double fk[Q];
    double phi;
    if (split_layout(mode)) {
      phi = mode == kHiLo ? phi_get(reinterpret_cast<const float2*>(phis), node) : phis[node];
      const float* g = reinterpret_cast<const float*>(f);
#pragma unroll
      for (int k = 0; k < Q; ++k) fk[k] = static_cast<double>(g[k * ps + node]) + p.omega[k] * phi;
    } else {
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        fk[k] = static_cast<double>(f[k * ps + node]) + p.omega[k] * ref;
        sum += fk[k];
      }
      phi = sum - p.dt * p.R;
      if (want_ent) {
        // pre-collision populations from the post-collision ones (s != 1)
        const double inv = 1.0 / (1.0 - p.s);
#pragma unroll
        for (int k = 0; k < Q; ++k)
          fk[k] = (fk[k] - p.dt * p.omega[k] * p.R - p.s * p.omega[k] * phi) * inv;
      }
    }
    if (phi_out) phi_out[node] = phi;
    if (!want_red) continue;
    if (want_ent) {
      double ent = 0.0;
#pragma unroll
      for (int k = 0; k < Q; ++k) ent += fk[k] * fk[k] / (2.0 * p.omega[k]);
      acc[3] += ent;
    }
    acc[0] += phi;
    acc[1] += phi * phi;
    if (want_err) {
      int i[D];
      double x[D];
      node_index<D>(p, node, i);
      node_coords<D>(p, i, x);
      const double e = phi - field_value<D>(p.field, p, x, t_n);
      acc[2] += e * e;
    }
    acc[4] = fmax(acc[4], fabs(phi));
    acc[5] += isfinite(phi) ? 0.0 : 1.0;
  }
  if (!want_red) return;  // uniform over the grid
  block_reduce(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < kNumAcc; ++m) partial[blockIdx.x * kNumAcc + m] = acc[m];
  }
}

template <int D>
__global__ void __launch_bounds__(kRedThreads)
    k_sum_phi0(const double* __restrict__ arr, const KParams p, double* __restrict__ partial) {
  __shared__ double sh[kNumAcc * kRedThreads];
  double acc[kNumAcc] = {0, 0, 0, 0, 0, 0};
  for (int node = blockIdx.x * blockDim.x + threadIdx.x; node < p.nodes;
       node += gridDim.x * blockDim.x) {
    double v;
    if (arr) {
      v = arr[node];
    } else {
      int i[D];
      double x[D], g[D];
      node_index<D>(p, node, i);
      node_coords<D>(p, i, x);
      field_initial<D>(p.field, p, x, v, g);
    }
    acc[0] += v;
  }
  block_reduce(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < kNumAcc; ++m) partial[blockIdx.x * kNumAcc + m] = acc[m];
  }
}

}  // namespace lbm
