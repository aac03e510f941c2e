// Batched von Neumann analysis of the periodic scheme (Sec. 4.2, eq. (G)):
// the spectral radius of the amplification matrix over a grid of wave
// numbers, for many parameter points (sigma = u, s) at once, and the
// smallest equilibrium weight (the entropy criterion of Sec. 4.1, Prop. 1).
//
// In population space the Fourier symbol of one step is
//     G(xi) = T(xi) [(1 - s) I + s omega 1^T],   T(xi) = diag(exp(-i c_k . xi)),
// which is similar to the moment-space matrix of eq. (G) (M is invertible;
// s = 2 gives eq. (G) itself).  G is a diagonal matrix plus a rank-one term,
// so its spectrum has a closed structure.  Let the velocities be grouped by
// equal tau_k = exp(-i c_k . xi) (groups g with tau_g, W_g = sum of their
// omega_k, n_g members).  Then
//   * every vector supported on one group with zero sum is an eigenvector
//     with eigenvalue (1 - s) tau_g (n_g - 1 of them per group), and
//   * the other eigenvalues are the roots of the secular equation
//         1 = s sum_g W_g tau_g / (lambda - (1 - s) tau_g)
//     (the matrix determinant lemma), i.e. of a polynomial of degree equal
//     to the number of groups with W_g != 0.
// On the grid xi = 2 pi j / m the phase c_k . xi is 2 pi (c_k . j) / m, so the
// grouping is exact integer arithmetic on (c_k . j) mod m.
//
// The roots come from the Aberth-Ehrlich simultaneous iteration (Aberth,
// Math. Comp. 27 (1973); Ehrlich, Comm. ACM 10 (1967)).  With a = 1 - s,
// v_g = s W_g tau_g and poles a tau_g, the polynomial is
//     p(lambda) = prod_g (lambda - a tau_g) - sum_g v_g prod_{g' != g} (lambda - a tau_g'),
// and its Newton ratio p / p' is evaluated in secular form with the pole h
// nearest to lambda factored out, which stays accurate when a root sits next
// to a pole (a weight near 0):
//     p / prod_{g != h} = e f_h - v_h,   e = lambda - a tau_h,
//     f_h = 1 - sum_{g != h} v_g / (lambda - a tau_g).
// All but one root sit near the poles a tau_g (exactly so for s -> 1, where
// they collapse to 0); the remaining one carries the conserved mode (1 at
// xi = 0) and starts from sum_g v_g + a mean(tau).  One thread
// takes one wave number; a block reduces the maximum over the grid of one
// parameter point.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "engine.hpp"
#include "lattice.hpp"
#include "meta.hpp"

namespace lbm {
namespace {

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx cscale(cplx a, double r) { return {a.re * r, a.im * r}; }
__device__ __forceinline__ cplx cinv(cplx a) {
  const double n = a.re * a.re + a.im * a.im;
  return {a.re / n, -a.im / n};
}
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) { return cmul(a, cinv(b)); }
__device__ __forceinline__ double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ bool cfinite(cplx a) { return isfinite(a.re) && isfinite(a.im); }

constexpr int kStabThreads = 256;
constexpr int kAberthSweeps = 200;
constexpr double kAberthTol = 1e-14;
constexpr double kAberthFloor = 1e-12;

// rho(G(xi)) at xi = 2 pi j / m; *converged is false when the iteration did
// not settle within kAberthSweeps sweeps.
template <int D>
__device__ double rho_at(const double (&w)[q_of(D)], double s, const int (&j)[kMaxDim], int m,
                         bool* converged) {
  constexpr int Q = q_of(D);
  int key[Q];
  double W[Q];
  int cnt[Q];
  int n = 0;
  static_for<0, Q>([&](auto K) {
    constexpr int k = decltype(K)::value;
    int ph = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) ph += vel_comp(D, k, a) * j[a];
    ph %= m;
    if (ph < 0) ph += m;
    int g = 0;
    while (g < n && key[g] != ph) ++g;
    if (g == n) {
      key[n] = ph;
      W[n] = 0.0;
      cnt[n] = 0;
      ++n;
    }
    W[g] += w[k];
    cnt[g] += 1;
  });
  const double a = 1.0 - s;
  double rho = 0.0;
  cplx pole[Q], v[Q], lam[Q];
  int ng = 0;
  for (int g = 0; g < n; ++g) {
    // (1 - s) tau_g from the zero-sum vectors of a group, and from a group
    // whose weights cancel (its pole is then a root)
    if (cnt[g] > 1 || W[g] == 0.0) rho = fmax(rho, fabs(a));
    if (W[g] == 0.0) continue;
    double sn, cs;
    sincospi(2.0 * key[g] / m, &sn, &cs);
    const cplx tau{cs, -sn};
    pole[ng] = cscale(tau, a);
    v[ng] = cscale(tau, s * W[g]);
    ++ng;
  }
  *converged = true;
  if (ng == 0) return rho;
  if (a == 0.0) {
    // all poles at 0: p(lambda) = lambda^(ng-1) (lambda - sum_g v_g)
    cplx sum{0.0, 0.0};
    for (int g = 0; g < ng; ++g) sum = cadd(sum, v[g]);
    return fmax(rho, sqrt(cabs2(sum)));
  }
  // Start: ng - 1 roots just beside the poles (scaled by 1.01, turned by
  // pi / (4 ng)); the one of the largest |v_g| is replaced by the estimate of
  // the root that carries the conserved mode, sum_g v_g + a mean(tau).
  {
    double sn, cs;
    sincospi(0.25 / ng, &sn, &cs);
    const cplx turn{1.01 * cs, 1.01 * sn};
    cplx vsum{0.0, 0.0}, psum{0.0, 0.0};
    int big = 0;
    double vbig = -1.0;
    for (int g = 0; g < ng; ++g) {
      lam[g] = cmul(pole[g], turn);
      vsum = cadd(vsum, v[g]);
      psum = cadd(psum, pole[g]);
      const double vg = cabs2(v[g]);
      if (vg > vbig) {
        vbig = vg;
        big = g;
      }
    }
    lam[big] = cadd(cadd(vsum, cscale(psum, 1.0 / ng)), cplx{0.0, 1e-3});
  }
  bool done = false;
  double prev = INFINITY;
  for (int it = 0; it < kAberthSweeps && !done; ++it) {
    double worst = 0.0;
    for (int i = 0; i < ng; ++i) {
      const cplx z = lam[i];
      // nearest pole h, kept out of the sums so that nothing blows up near it
      int h = 0;
      double dh = cabs2(csub(z, pole[0]));
      for (int g = 1; g < ng; ++g) {
        const double dg = cabs2(csub(z, pole[g]));
        if (dg < dh) {
          dh = dg;
          h = g;
        }
      }
      cplx f{1.0, 0.0}, fp{0.0, 0.0}, S{0.0, 0.0};
      for (int g = 0; g < ng; ++g) {
        if (g == h) continue;
        const cplx inv = cinv(csub(z, pole[g]));
        const cplx vi = cmul(v[g], inv);
        f = csub(f, vi);
        fp = cadd(fp, cmul(vi, inv));
        S = cadd(S, inv);
      }
      // p / p' with p = prod_{g != h} (z - pole_g) [(z - pole_h) f_h - v_h]
      const cplx e = csub(z, pole[h]);
      const cplx num = csub(cmul(e, f), v[h]);
      const cplx den = csub(cadd(f, cmul(e, cadd(cmul(S, f), fp))), cmul(v[h], S));
      const cplx N = cdiv(num, den);
      cplx ab{0.0, 0.0};
      for (int l = 0; l < ng; ++l)
        if (l != i) ab = cadd(ab, cinv(csub(z, lam[l])));
      cplx corr = cdiv(N, csub(cplx{1.0, 0.0}, cmul(N, ab)));
      if (!cfinite(corr)) corr = cplx{1e-8, 1e-8};  // landed on a pole or a root
      lam[i] = csub(z, corr);
      const double rel = sqrt(cabs2(corr)) / fmax(1.0, sqrt(cabs2(lam[i])));
      worst = fmax(worst, rel);
    }
    // settled: corrections below the tolerance, or at the rounding floor
    // (small and no longer shrinking the way a converging iteration does)
    done = worst < kAberthTol || (worst < kAberthFloor && worst > 0.5 * prev);
    prev = worst;
  }
  *converged = done;
  for (int g = 0; g < ng; ++g) {
    if (!cfinite(lam[g])) {
      *converged = false;
      return INFINITY;
    }
    rho = fmax(rho, sqrt(cabs2(lam[g])));
  }
  return rho;
}

template <int D>
__global__ void __launch_bounds__(kStabThreads)
    k_stability(const double* __restrict__ sigma, const double* __restrict__ s_arr, double gm4,
                int m, long long nxi, double* __restrict__ rho_out,
                double* __restrict__ min_omega_out, int32_t* __restrict__ unconv_out) {
  constexpr int Q = q_of(D);
  const long long pt = blockIdx.x;
  double u[kMaxDim] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < D; ++a) u[a] = sigma[pt * D + a];
  const double s = s_arr[pt];
  const double m4 = (D >= 2) ? m4_interpolated(D, u, gm4) : 0.0;
  double w[Q];
  omega_closed_form(D, u, m4, w);
  double best = 0.0;
  int bad = 0;
  for (long long e = threadIdx.x; e < nxi; e += blockDim.x) {
    int j[kMaxDim] = {0, 0, 0, 0};
    long long r = e;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      j[a] = static_cast<int>(r % m);
      r /= m;
    }
    bool ok = true;
    best = fmax(best, rho_at<D>(w, s, j, m, &ok));
    bad += ok ? 0 : 1;
  }
  __shared__ double sb[kStabThreads];
  __shared__ int si[kStabThreads];
  sb[threadIdx.x] = best;
  si[threadIdx.x] = bad;
  __syncthreads();
  for (int h = kStabThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + h]);
      si[threadIdx.x] += si[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    rho_out[pt] = sb[0];
    if (unconv_out) unconv_out[pt] = si[0];
    if (min_omega_out) {
      double mw = w[0];
#pragma unroll
      for (int k = 1; k < Q; ++k) mw = fmin(mw, w[k]);
      min_omega_out[pt] = mw;
    }
  }
}

}  // namespace

hipError_t launch_stability(int d, long long count, const double* sigma, const double* s,
                            double g, int m, long long nxi, double* rho, double* min_omega,
                            int32_t* unconverged, hipStream_t stream) {
  const dim3 grid(static_cast<unsigned>(count)), block(kStabThreads);
  switch (d) {
    case 1:
      hipLaunchKernelGGL(k_stability<1>, grid, block, 0, stream, sigma, s, g, m, nxi, rho,
                         min_omega, unconverged);
      break;
    case 2:
      hipLaunchKernelGGL(k_stability<2>, grid, block, 0, stream, sigma, s, g, m, nxi, rho,
                         min_omega, unconverged);
      break;
    case 3:
      hipLaunchKernelGGL(k_stability<3>, grid, block, 0, stream, sigma, s, g, m, nxi, rho,
                         min_omega, unconverged);
      break;
    case 4:
      hipLaunchKernelGGL(k_stability<4>, grid, block, 0, stream, sigma, s, g, m, nxi, rho,
                         min_omega, unconverged);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lbm
