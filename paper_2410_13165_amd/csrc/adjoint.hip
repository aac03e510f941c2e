// Adjoint (transposed) kernels of the lattice Boltzmann step, for gradients of
// a final-time misfit L(phi^N).
//
// The stored forward state is g^n = C f^n + b (post-collision; C = (1-s) I +
// s omega 1^T, b = dt omega R) or, in the split mode, the pre-collision f^n.
// One forward step is f^{n+1} = P_in S g^n + (wall values), S the pull
// streaming; on half-way walls the wall value also holds -g^n_kbar(x_f).
// With lambda^n = dL/df^n and nu^n = dL/dg^n:
//   nu^n     = S^T P_in^T lambda^{n+1}  (minus lambda^{n+1}_k(x_f) in the kbar
//                                        component at half-way wall nodes)
//   lambda^n = C^T nu^n,   (C^T v)_k = (1-s) v_k + s sum_j omega_j v_j.
// S^T is a pull from x + c_k; populations that leave the domain contribute 0.
// The seed is lambda^N = dL/dphi^N for every k (phi = sum_k f_k).
// dL/ds = sum_{n<N} <nu^n, (omega 1^T - I) f^n>, with f^n recovered from the
// stored g^n.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace lbm {

namespace {

// node offset of x + c_k (wrapped) and whether x + c_k leaves the domain
template <int D, int k>
__device__ __forceinline__ int push_offset(const RowInfo<D>& r) {
  constexpr Vec4i c = vel_vec(D, k);
  int off = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (c.v[a] == 1) off += r.dp[a];
    if (c.v[a] == -1) off += r.dm[a];
  }
  return off;
}

template <int D, int k>
__device__ __forceinline__ bool leaves(const RowInfo<D>& r) {
  constexpr Vec4i c = vel_vec(D, k);
  bool o = false;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (c.v[a] == 1) o = o || r.hi[a];
    if (c.v[a] == -1) o = o || r.lo[a];
  }
  return o;
}

// Block sum of v; thread 0 stores it to *out, or adds it when accumulate.
__device__ __forceinline__ void block_sum(double v, double* sh, double* out,
                                          bool accumulate = false) {
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int nt = blockDim.x * blockDim.y;
  sh[tid] = v;
  __syncthreads();
  for (int half = 128; half > 0; half >>= 1) {
    if (tid < half && tid + half < nt) sh[tid] += sh[tid + half];
    __syncthreads();
  }
  if (tid == 0) *out = accumulate ? *out + sh[0] : sh[0];
}

// acc + <mu, (omega 1^T - I) f^n> at one node, f^n recovered from the stored
// forward state g (post-collision, or the split g_k = f_k - omega_k phi).
template <int D, class T>
__device__ __forceinline__ double zdot(double acc, const T (&mu)[q_of(D)], const T* __restrict__ g,
                                       int node, long long ps, int mode, const KParams& p) {
  constexpr int Q = q_of(D);
  double z[Q];
  if (mode == kSplit) {
#pragma unroll
    for (int k = 0; k < Q; ++k) z[k] = -static_cast<double>(g[k * ps + node]);
  } else {
    // omega_k phi + dt omega_k R - g_k with phi = sum_j g_j - dt R, which is
    // omega_k sum_j g_j - g_k; the same form holds for the float32
    // deviations from the uniform state
    double gk[Q];
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      gk[k] = static_cast<double>(g[k * ps + node]);
      sum += gk[k];
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) z[k] = p.omega[k] * sum - gk[k];
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) acc += static_cast<double>(mu[k]) * z[k];
  return acc;
}

}  // namespace

// One adjoint step lambda^{n+1} -> lambda^n over every row.  `g` is the
// forward state at step n (post-collision g^n, or the split (phi, g) pair);
// when it is given, the block's share of <nu^n, (omega 1^T - I) f^n> is added
// to partial[block] (for dL/ds, without the 1/(1-s) factor of the
// post-collision modes, which the host applies); every block adds its own
// steps in order, so the final sum is deterministic.
template <int D, class T>
__global__ void __launch_bounds__(256)
    k_adjoint(const T* __restrict__ lsrc, T* __restrict__ ldst, const T* __restrict__ g,
              const double* __restrict__ gphi, const KParams p, const int mode,
              double* __restrict__ partial) {
  constexpr int Q = q_of(D);
  __shared__ double sh[256];
  const int row = blockIdx.x * blockDim.y + threadIdx.y;
  double acc = 0.0;
  if (row < p.rows) {
    RowInfo<D> r;
    row_setup<D>(p, row, r);
    const long long ps = p.pstride;
    const bool half = p.scheme == kHalfWay;
    for (int x = threadIdx.x; x < p.n[0]; x += blockDim.x) {
      col_setup<D>(p, x, r);
      const int node = r.rowbase + x;
      T mu[Q];
      static_for<0, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        mu[k] = lsrc[k * ps + node + push_offset<D, k>(r)];
      });
      // populations that leave the domain: zero, or on half-way walls the
      // reflected coupling -lambda_kbar(x) of the wall formula
      static_for<0, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if (leaves<D, k>(r)) {
          constexpr int kb = opp_index(D, k);
          mu[k] = half ? -lsrc[kb * ps + node] : T(0);
        }
      });
      double m = 0.0;
#pragma unroll
      for (int k = 0; k < Q; ++k) m += p.omega[k] * static_cast<double>(mu[k]);
      const T ms = static_cast<T>(p.s * m);
      const T oms = static_cast<T>(1.0 - p.s);
#pragma unroll
      for (int k = 0; k < Q; ++k) __builtin_nontemporal_store(oms * mu[k] + ms, ldst + k * ps + node);
      if (g) acc = zdot<D, T>(acc, mu, g, node, ps, mode, p);
    }
  }
  if (g) block_sum(acc, sh, partial + blockIdx.x, true);
}

// Two adjoint steps lambda^{n+1} -> lambda^{n-1} in one pass (d = 3), laid
// out as the forward two-step pass (fuse.hpp) but pulling from x + c_k, so
// the LDS planes of the c_3 = -1 values are the long-lived ones.  g1 and g2
// are the forward states at steps n and n - 1 (both null when no dL/ds is
// wanted); each block adds its share of both steps' contractions to
// partial[block] (its own nodes only: the halo belongs to other blocks).
template <class T, bool HALF>
__global__ void __launch_bounds__((FuseShape<T, HALF>::NT))
    k_adjoint2(const T* __restrict__ lsrc, T* __restrict__ ldst, const T* __restrict__ g1,
               const T* __restrict__ g2, const KParams p, const int mode,
               double* __restrict__ partial, const int zc) {
  using S = FuseShape<T, HALF>;
  constexpr int D = 3, Q = q_of(3), TX = S::TX, TY = S::TY, NT = S::NT;
  constexpr int RX = TX + 2, RY = TY + 2, R = RX * RY;
  extern __shared__ __align__(16) unsigned char fuse_lds[];
  T* lds = reinterpret_cast<T*>(fuse_lds);
  const long long ps = p.pstride;
  const int n0 = p.n[0], n1 = p.n[1], n2 = p.n[2];
  int tx_, ty_, tz_;
  fuse_tile(p, TX, TY, tx_, ty_, tz_);
  const int x0 = tx_ * TX, y0 = ty_ * TY, zc0 = tz_ * zc;
  const int zend = min(zc0 + zc, n2);
  const int iters = zend - zc0 + 2;
  const T oms = static_cast<T>(1.0 - p.s);
  double acc = 0.0;
  for (int it = 0; it < iters; ++it) {
    const int zp = zc0 - 1 + it;
    // ---- lambda^n on the tile and its halo of plane zp
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
      RowInfo<D> nb;
      row_setup_yz(p, gy, gz, nb);
      col_setup<D>(p, gx, nb);
      const int node = nb.rowbase + gx;
      T mu[Q];
      static_for<0, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        mu[k] = lsrc[k * ps + node + push_offset<D, k>(nb)];
      });
      static_for<0, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if (leaves<D, k>(nb)) {
          constexpr int kb = opp_index(D, k);
          mu[k] = HALF ? -lsrc[kb * ps + node] : T(0);
        }
      });
      double m = 0.0;
#pragma unroll
      for (int k = 0; k < Q; ++k) m += p.omega[k] * static_cast<double>(mu[k]);
      const T ms = static_cast<T>(p.s * m);
      const bool own = rx >= 1 && rx <= TX && ry >= 1 && ry <= TY && x0 - 1 + rx < n0 &&
                       y0 - 1 + ry < n1 && zp >= zc0 && zp < zend;
      if (g1 && own) acc = zdot<D, T>(acc, mu, g1, node, ps, mode, p);
      static_for<0, Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        lds[adj_slot<HALF, k>(it) * R + r] = oms * mu[k] + ms;
      });
    }
    __syncthreads();
    // ---- lambda^{n-1} on output plane zp - 1
    if (it >= 2) {
      const int gz = zp - 1;
      for (int o = threadIdx.x; o < TX * TY; o += NT) {
        const int ox = o % TX, oy = o / TX;
        const int gx = x0 + ox, gy = y0 + oy;
        if (gx >= n0 || gy >= n1) continue;
        RowInfo<D> nb;
        row_setup_yz(p, gy, gz, nb);
        col_setup<D>(p, gx, nb);
        const int node = nb.rowbase + gx;
        const int own = (oy + 1) * RX + (ox + 1);
        T mu[Q];
        static_for<0, Q>([&](auto K) {
          constexpr int k = decltype(K)::value;
          constexpr Vec4i c = vel_vec(D, k);
          constexpr int src_it = c.v[2] == 1 ? 0 : (c.v[2] == 0 ? 1 : 2);
          if (leaves<D, k>(nb)) {
            if constexpr (HALF) {
              constexpr int kb = opp_index(D, k);
              mu[k] = -lds[adj_slot<HALF, kb>(it - 1) * R + own];
            } else {
              mu[k] = T(0);
            }
          } else {
            const int rr = (oy + 1 + c.v[1]) * RX + (ox + 1 + c.v[0]);
            mu[k] = lds[adj_slot<HALF, k>(it - src_it) * R + rr];
          }
        });
        double m = 0.0;
#pragma unroll
        for (int k = 0; k < Q; ++k) m += p.omega[k] * static_cast<double>(mu[k]);
        const T ms = static_cast<T>(p.s * m);
        // the contraction's loads before the stores: the wait for them would
        // otherwise also wait for the stores, since the vector-memory counter
        // covers both on this chip
        if (g2) acc = zdot<D, T>(acc, mu, g2, node, ps, mode, p);
#pragma unroll
        for (int k = 0; k < Q; ++k)
          __builtin_nontemporal_store(oms * mu[k] + ms, ldst + k * ps + node);
      }
    }
    __syncthreads();
  }
  if (g1 || g2) {
    // deterministic block sum over 1024 slots (zeros past NT), reusing the LDS
    double* sh = reinterpret_cast<double*>(fuse_lds);
    sh[threadIdx.x] = acc;
    if (threadIdx.x + NT < 1024) sh[threadIdx.x + NT] = 0.0;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
      if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] += sh[0];
  }
}

// Seed lambda^N_k(x) = dL/dphi^N(x) for every k.
template <class T>
__global__ void __launch_bounds__(256)
    k_adjoint_seed(const double* __restrict__ dldphi, T* __restrict__ lam, const KParams p) {
  for (int node = blockIdx.x * blockDim.x + threadIdx.x; node < p.nodes;
       node += gridDim.x * blockDim.x) {
    const T v = static_cast<T>(dldphi[node]);
    for (int k = 0; k < p.q; ++k) lam[k * p.pstride + node] = v;
  }
}

// Transpose of the initialisation f_k = omega_k [phi0 + tau dt (u - c_k) . grad phi0]:
//   dL/dphi0 (direct part)  = sum_k omega_k lambda_k
//   dL/d(grad phi0)_a       = tau dt sum_k omega_k (u_a - c_ka) lambda_k
// and the tau-derivative of the initial state, (f^0_k - omega_k phi0) / tau,
// contracted with lambda^0 (per-block partial sums).  g0 is the stored initial
// state (post-collision, or split).
template <int D, class T>
__global__ void __launch_bounds__(256)
    k_adjoint_init(const T* __restrict__ lam, const T* __restrict__ g0,
                   const double* __restrict__ g0phi, const KParams p, const int mode,
                   double* __restrict__ dphi, double* __restrict__ dgrad,
                   double* __restrict__ partial) {
  constexpr int Q = q_of(D);
  __shared__ double sh[256];
  double acc = 0.0;
  const long long ps = p.pstride;
  for (int node = blockIdx.x * blockDim.x + threadIdx.x; node < p.nodes;
       node += gridDim.x * blockDim.x) {
    double l[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) l[k] = static_cast<double>(lam[k * ps + node]);
    double s0 = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) s0 += p.omega[k] * l[k];
    dphi[node] = s0;
    if (dgrad) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double h = 0.0;
        static_for<0, Q>([&](auto K) {
          constexpr int k = decltype(K)::value;
          constexpr Vec4i c = vel_vec(D, k);
          h += p.omega[k] * (p.u[a] - c.v[a]) * l[k];
        });
        dgrad[(long long)a * p.nodes + node] = p.tau * p.dt * h;
      }
    }
    // f^0_k - omega_k phi0
    double z[Q];
    if (mode == kSplit) {
#pragma unroll
      for (int k = 0; k < Q; ++k) z[k] = static_cast<double>(g0[k * ps + node]);
    } else {
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < Q; ++k) sum += static_cast<double>(g0[k * ps + node]);
      // post-collision g = C f + b:  f_k - omega_k phi = (g_k - b_k - omega_k phi)/(1-s),
      // phi = sum g - dt R; in deviation form (g_k - omega_k sum_j g_j)/(1-s)
#pragma unroll
      for (int k = 0; k < Q; ++k)
        z[k] = (static_cast<double>(g0[k * ps + node]) - p.omega[k] * sum) / (1.0 - p.s);
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) acc += l[k] * z[k];
  }
  (void)g0phi;
  block_sum(acc / p.tau, sh, partial + blockIdx.x);
}

// dphi -= sum_a D_a(dgrad_a), D_a the fourth-order central difference on the
// periodic grid (its transpose is -D_a).
template <int D>
__global__ void __launch_bounds__(256)
    k_adjoint_fd(const double* __restrict__ dgrad, double* __restrict__ dphi, const KParams p) {
  for (int node = blockIdx.x * blockDim.x + threadIdx.x; node < p.nodes;
       node += gridDim.x * blockDim.x) {
    int i[D];
    int rr = node;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      i[a] = rr % p.n[a];
      rr /= p.n[a];
    }
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int n = p.n[a];
      const int st = p.stride[a];
      const double* h = dgrad + (long long)a * p.nodes;
      auto at = [&](int s) {
        int j = i[a] + s;
        j = (j % n + n) % n;
        return h[node + (j - i[a]) * st];
      };
      acc += (-at(2) + 8.0 * at(1) - 8.0 * at(-1) + at(-2)) / (12.0 * p.dx);
    }
    dphi[node] -= acc;
  }
}

__global__ void __launch_bounds__(256)
    k_sum_partials(const double* __restrict__ partial, long long n, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (long long b = threadIdx.x; b < n; b += blockDim.x) acc += partial[b];
  block_sum(acc, sh, out);
}

// ------------------------------------------------- wall-data sensitivities --
//
// The populations that enter through a Dirichlet wall at step n+1 are the
// wall values W_k(x): full-way, eq. (bun1) at (x, t_{n+1}); half-way, the data
// part B_k(x_b, t_n) of eq. (bun2) (its -f*_kbar term is part of the linear
// step above).  For the analytic field F = sum_j a_j cos(kappa_j . y + theta_j)
// (or a_j exp(kappa_j . y)) every W_k is linear in each amplitude a_j and
// depends on the phase theta_j through cos / sin, so with
// lambda^{n+1}_k(x) = dL/df^{n+1}_k(x),
//   dL/da_j     += sum over unknown (x, k) of lambda^{n+1}_k(x) dW_k(x)/da_j,
//   dL/dtheta_j += ... dW_k(x)/dtheta_j.
// The per-mode factors are those of wall_analytic (kernels.hpp): full-way
//   W_k = omega_k [sum_j a_j (C_j + q_kj S_j) + R t],
//   q_kj = (dt/2) pv + (dt^3/24) pv^3 (order-dependent),  pv = kappa_j . (c_k - u),
// with C_j, S_j = cos, sin of kappa_j . (x - u t) + theta_j; half-way
//   B_k = sum_j a_j [(T0 - T2) C_kj + (T3 - T1) S_kj] + R terms,
// with C_kj, S_kj at the half-cell-shifted wall point.

// Contributions of one boundary node x (coordinates xc, lk[k] = lambda_k(x)
// for the unknown k, 0 otherwise) to acc[j] (d/da_j) and acc[kMaxModes + j]
// (d/dtheta_j).
template <int D>
__device__ void wall_param_grad(const KParams& p, const double (&xc)[kMaxDim], double t_n,
                                const bool (&out)[q_of(D)], const int (&ax)[q_of(D)],
                                const double (&lk)[q_of(D)], double (&acc)[2 * kMaxModes]) {
  constexpr int Q = q_of(D);
  const FieldDev& F = p.field;
  const double dt = p.dt, dt2 = dt * dt, dt3 = dt2 * dt;
  const bool full = p.scheme == kFullWay;
  const bool is_cos = F.kind == kFieldCos;
  const bool tan = p.wall_data != 0;
  const double o2 = p.P >= 2 ? 1.0 : 0.0;
  const double o3 = p.P >= 3 ? 1.0 : 0.0;
  const double o4 = p.P >= 4 ? 1.0 : 0.0;
  const double t = full ? t_n + dt : t_n;
  for (int j = 0; j < F.nmodes; ++j) {
    double ph = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) ph += F.kvec[j][a] * (xc[a] - p.u[a] * t);
    double C = 0.0, S = 0.0, E = 0.0;
    if (is_cos)
      sincos(ph + F.phase[j], &S, &C);
    else
      E = exp(ph);
    const double amp = F.amp[j];
    const double w = -F.ku[j];
    double ga = 0.0, gt = 0.0;
    static_for<0, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr Vec4i c = vel_vec(D, k);
      if (!out[k]) return;
      // kappa_j . c_k, or with tangential wall data its Remark-1 form
      double pc = 0.0;
      if (!tan) {
#pragma unroll
        for (int a = 0; a < D; ++a) pc += c.v[a] * F.kvec[j][a];
      } else {
        double r = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a)
          if (a == ax[k]) r = c.v[a] * p.inv_u[a];
#pragma unroll
        for (int a = 0; a < D; ++a)
          if (a != ax[k]) pc += (c.v[a] - r * p.u[a]) * F.kvec[j][a];
        pc -= r * w;
      }
      const double l = lk[k];
      if (full) {
        const double pv = pc + w;
        const double pv3 = pv * pv * pv;
        if (is_cos) {
          const double q = o3 * 0.5 * dt * pv + o4 * dt3 / 24.0 * pv3;
          ga += l * p.omega[k] * (C + q * S);
          gt += l * p.omega[k] * amp * (q * C - S);
        } else {
          ga += l * p.omega[k] * E * (1.0 - o3 * 0.5 * dt * pv + o4 * dt3 / 24.0 * pv3);
        }
      } else {
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
          ga += l * ((T0 - T2) * Ck + (T3 - T1) * Sk);
          gt += l * amp * ((T3 - T1) * Ck - (T0 - T2) * Sk);
        } else {
          double Ek = E;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            if (c.v[a] == 1) Ek *= F.rot[j][a][0];
            if (c.v[a] == -1) Ek *= F.rot[j][a][1];
          }
          ga += l * (T0 + T1 + T2 + T3) * Ek;
        }
      }
    });
    acc[j] += ga;
    acc[kMaxModes + j] += gt;
  }
}

// One adjoint step's wall-data contractions over every boundary node: the
// nodes of the rows on a wall of an axis >= 2 (wall_row), then the two x_1-face
// nodes of every other row.  A fixed grid of kWallGradBlocks blocks walks them;
// block b adds its sums to partial[b * 2 kMaxModes + m], so the steps'
// contributions are summed in a fixed order.
constexpr int kWallGradBlocks = 256;

template <int D, class T>
__global__ void __launch_bounds__(256)
    k_wall_grad(const T* __restrict__ lam, const KParams p, const double t_n,
                double* __restrict__ partial) {
  constexpr int Q = q_of(D);
  __shared__ double sh[256];
  double acc[2 * kMaxModes];
#pragma unroll
  for (int m = 0; m < 2 * kMaxModes; ++m) acc[m] = 0.0;
  const long long ps = p.pstride;
  const long long nA = static_cast<long long>(p.wall_rows) * p.n[0];
  const long long nB = p.bc[0] != 0 ? 2LL * p.rows : 0;
  for (long long it = blockIdx.x * 256LL + threadIdx.x; it < nA + nB; it += 256LL * gridDim.x) {
    int row, x;
    if (it < nA) {
      row = wall_row<D>(p, static_cast<int>(it / p.n[0]));
      x = static_cast<int>(it % p.n[0]);
    } else {
      const long long b = it - nA;
      row = static_cast<int>(b >> 1);
      x = (b & 1) ? p.n[0] - 1 : 0;
    }
    RowInfo<D> r;
    row_setup<D>(p, row, r);
    if (it >= nA && r.rowwall) continue;  // visited among the wall rows
    col_setup<D>(p, x, r);
    bool out[Q];
    int ax[Q];
    bool any = false;
    static_for<0, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      out[k] = outside<D, k>(r);
      ax[k] = wall_axis<D, k>(r);
      any = any || out[k];
    });
    if (!any) continue;
    const int node = r.rowbase + x;
    double lk[Q];
    static_for<0, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      lk[k] = out[k] ? static_cast<double>(lam[k * ps + node]) : 0.0;
    });
    double xc[kMaxDim] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < D; ++a) xc[a] = p.origin[a] + (r.i[a] + p.shift[a]) * p.dx;
    wall_param_grad<D>(p, xc, t_n, out, ax, lk, acc);
  }
  const int M = p.field.nmodes;
  for (int m = 0; m < M; ++m) {
    block_sum(acc[m], sh, partial + blockIdx.x * 2 * kMaxModes + m, true);
    block_sum(acc[kMaxModes + m], sh, partial + blockIdx.x * 2 * kMaxModes + kMaxModes + m, true);
  }
}

// out[m] = sum over the blocks b of partial[b * ncols + m], in block order
__global__ void __launch_bounds__(64)
    k_sum_columns(const double* __restrict__ partial, int nblocks, int ncols,
                  double* __restrict__ out) {
  const int m = threadIdx.x;
  if (m >= ncols) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[b * ncols + m];
  out[m] = s;
}

// --------------------------------------------------------------- launchers --

template <int D>
static hipError_t adjoint_d(const KParams& p, int mode, const void* lsrc, void* ldst,
                            const void* g, const double* gphi, double* partial,
                            hipStream_t stream) {
  const LaunchShape s = step_shape(p);
  const dim3 block(s.tx, s.ty), grid(s.blocks);
  if (mode == kFP64)
    hipLaunchKernelGGL((k_adjoint<D, double>), grid, block, 0, stream,
                       static_cast<const double*>(lsrc), static_cast<double*>(ldst),
                       static_cast<const double*>(g), gphi, p, mode, partial);
  else
    hipLaunchKernelGGL((k_adjoint<D, float>), grid, block, 0, stream,
                       static_cast<const float*>(lsrc), static_cast<float*>(ldst),
                       static_cast<const float*>(g), gphi, p, mode, partial);
  return hipGetLastError();
}

template <class T>
static long long pair_blocks_t(const KParams& p) {
  using S = FuseShape<T, false>;
  using H = FuseShape<T, true>;
  const bool half = p.scheme == kHalfWay;
  const int tx = half ? H::TX : S::TX, ty = half ? H::TY : S::TY;
  const int tiles_xy = ((p.n[0] + tx - 1) / tx) * ((p.n[1] + ty - 1) / ty);
  const int zc = fuse_zchunk(tiles_xy, p.n[2]);
  return static_cast<long long>(tiles_xy) * ((p.n[2] + zc - 1) / zc);
}

long long adjoint_pair_blocks(const KParams& p, int mode) {
  if (p.d != 3) return 0;
  return mode == kFP64 ? pair_blocks_t<double>(p) : pair_blocks_t<float>(p);
}

template <class T, bool HALF>
static hipError_t adjoint_pair_t(const KParams& p, int mode, const void* lsrc, void* ldst,
                                 const void* g1, const void* g2, double* partial,
                                 hipStream_t stream) {
  using S = FuseShape<T, HALF>;
  constexpr int R = (S::TX + 2) * (S::TY + 2);
  constexpr size_t lds = sizeof(T) * S::SLOTS * R;
  static_assert(lds <= 160 * 1024 && lds >= 1024 * sizeof(double), "LDS of the adjoint pass");
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adjoint2<T, HALF>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int tiles_xy = ((p.n[0] + S::TX - 1) / S::TX) * ((p.n[1] + S::TY - 1) / S::TY);
  const int zc = fuse_zchunk(tiles_xy, p.n[2]);
  const dim3 grid(static_cast<unsigned>(tiles_xy * ((p.n[2] + zc - 1) / zc)));
  hipLaunchKernelGGL((k_adjoint2<T, HALF>), grid, dim3(S::NT), lds, stream,
                     static_cast<const T*>(lsrc), static_cast<T*>(ldst),
                     static_cast<const T*>(g1), static_cast<const T*>(g2), p, mode, partial, zc);
  return hipGetLastError();
}

hipError_t launch_adjoint_pair(const KParams& p, int mode, const void* lsrc, void* ldst,
                               const void* g1, const void* g2, double* partial,
                               hipStream_t stream) {
  if (p.d != 3) return hipErrorInvalidValue;
  const bool half = p.scheme == kHalfWay;
  if (mode == kFP64)
    return half ? adjoint_pair_t<double, true>(p, mode, lsrc, ldst, g1, g2, partial, stream)
                : adjoint_pair_t<double, false>(p, mode, lsrc, ldst, g1, g2, partial, stream);
  return half ? adjoint_pair_t<float, true>(p, mode, lsrc, ldst, g1, g2, partial, stream)
              : adjoint_pair_t<float, false>(p, mode, lsrc, ldst, g1, g2, partial, stream);
}

hipError_t launch_adjoint_step(const KParams& p, int mode, const void* lsrc, void* ldst,
                               const void* g, const double* gphi, double* partial,
                               hipStream_t stream) {
  switch (p.d) {
    case 1: return adjoint_d<1>(p, mode, lsrc, ldst, g, gphi, partial, stream);
    case 2: return adjoint_d<2>(p, mode, lsrc, ldst, g, gphi, partial, stream);
    case 3: return adjoint_d<3>(p, mode, lsrc, ldst, g, gphi, partial, stream);
    case 4: return adjoint_d<4>(p, mode, lsrc, ldst, g, gphi, partial, stream);
    default: return hipErrorInvalidValue;
  }
}

static unsigned node_grid(long long nodes) {
  long long b = (nodes + 255) / 256;
  if (b > 65536) b = 65536;
  return static_cast<unsigned>(b < 1 ? 1 : b);
}

hipError_t launch_adjoint_seed(const KParams& p, int mode, const double* dldphi, void* lam,
                               hipStream_t stream) {
  if (mode == kFP64)
    hipLaunchKernelGGL((k_adjoint_seed<double>), dim3(node_grid(p.nodes)), dim3(256), 0, stream,
                       dldphi, static_cast<double*>(lam), p);
  else
    hipLaunchKernelGGL((k_adjoint_seed<float>), dim3(node_grid(p.nodes)), dim3(256), 0, stream,
                       dldphi, static_cast<float*>(lam), p);
  return hipGetLastError();
}

template <int D>
static hipError_t adjoint_init_d(const KParams& p, int mode, const void* lam, const void* g0,
                                 const double* g0phi, double* dphi, double* dgrad,
                                 bool fd, double* partial, hipStream_t stream) {
  const dim3 grid(node_grid(p.nodes)), block(256);
  if (mode == kFP64)
    hipLaunchKernelGGL((k_adjoint_init<D, double>), grid, block, 0, stream,
                       static_cast<const double*>(lam), static_cast<const double*>(g0), g0phi,
                       p, mode, dphi, dgrad, partial);
  else
    hipLaunchKernelGGL((k_adjoint_init<D, float>), grid, block, 0, stream,
                       static_cast<const float*>(lam), static_cast<const float*>(g0), g0phi, p,
                       mode, dphi, dgrad, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !fd) return e;
  hipLaunchKernelGGL((k_adjoint_fd<D>), grid, block, 0, stream, dgrad, dphi, p);
  return hipGetLastError();
}

hipError_t launch_adjoint_init(const KParams& p, int mode, const void* lam, const void* g0,
                               const double* g0phi, double* dphi, double* dgrad, bool fd,
                               double* partial, unsigned* nblocks, hipStream_t stream) {
  *nblocks = node_grid(p.nodes);
  switch (p.d) {
    case 1: return adjoint_init_d<1>(p, mode, lam, g0, g0phi, dphi, dgrad, fd, partial, stream);
    case 2: return adjoint_init_d<2>(p, mode, lam, g0, g0phi, dphi, dgrad, fd, partial, stream);
    case 3: return adjoint_init_d<3>(p, mode, lam, g0, g0phi, dphi, dgrad, fd, partial, stream);
    case 4: return adjoint_init_d<4>(p, mode, lam, g0, g0phi, dphi, dgrad, fd, partial, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sum_partials(const double* partial, long long n, double* out,
                               hipStream_t stream) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, stream, partial, n, out);
  return hipGetLastError();
}

template <int D>
static hipError_t wall_grad_d(const KParams& p, int mode, const void* lam, double t_n,
                              double* partial, hipStream_t stream) {
  const dim3 grid(kWallGradBlocks), block(256);
  if (mode == kFP64)
    hipLaunchKernelGGL((k_wall_grad<D, double>), grid, block, 0, stream,
                       static_cast<const double*>(lam), p, t_n, partial);
  else
    hipLaunchKernelGGL((k_wall_grad<D, float>), grid, block, 0, stream,
                       static_cast<const float*>(lam), p, t_n, partial);
  return hipGetLastError();
}

long long wall_grad_partials() { return static_cast<long long>(kWallGradBlocks) * 2 * kMaxModes; }

hipError_t launch_wall_grad(const KParams& p, int mode, const void* lam, long long n,
                            double* partial, hipStream_t stream) {
  const double t_n = static_cast<double>(n) * p.dt;
  switch (p.d) {
    case 1: return wall_grad_d<1>(p, mode, lam, t_n, partial, stream);
    case 2: return wall_grad_d<2>(p, mode, lam, t_n, partial, stream);
    case 3: return wall_grad_d<3>(p, mode, lam, t_n, partial, stream);
    case 4: return wall_grad_d<4>(p, mode, lam, t_n, partial, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sum_wall_grad(const double* partial, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(64), 0, stream, partial, kWallGradBlocks,
                     2 * kMaxModes, out);
  return hipGetLastError();
}

}  // namespace lbm
