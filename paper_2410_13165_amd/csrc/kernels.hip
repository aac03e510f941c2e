// gfx950 kernels of the fourth-order BGK lattice Boltzmann model.
//
// k_xface      analytic wall data (eq. bun1 or bun2) of the two x_1 faces for
//              the coming step, one value per row and unknown population.
// k_step       fused pull-streaming + BGK collision (eq. BGK-LB-Evolution) over
//              the DdQ(2d^2+1) lattice for every row that is not on a wall of
//              an axis >= 2; its x_1-face nodes take their unknown populations
//              from k_xface's data.
// k_wall       the same update for the rows on a wall of an axis >= 2, with the
//              full-way (eq. bun1) or half-way (eq. bun2) formulas replacing
//              the populations whose upwind node lies outside the domain.
//              The three kernels run in this order on one stream; k_step and
//              k_wall write disjoint rows.
// k_step_split, k_wall_split
//              the same step on the (phi float64, g = f - omega phi float32)
//              representation.
// k_fused2, k_fused2_split, k_fused2_d2
//              two time steps per pass (d = 3 any storage, d = 2 float32 and
//              float64), the intermediate state in LDS; bitwise two k_step.
// k_step_batch, k_fused2_d2_batch, k_fused2_d2_resident
//              many periodic lattices in one launch per step, per pair of
//              steps, or (resident) per call with one block per instance.
// k_init       initial state of order K = 1 or 3 (eq. ini-simp).
// k_moments    phi, RMSE (eq. rmse), total microscopic entropy (eq. skfk) and
//              safety statistics as deterministic float64 reductions, the
//              work selected by the caller's mask.
// k_count_nonfinite
//              the periodic non-finite check of lbm_step.
//
// Memory layout: structure of arrays, population k of node `node` at
// base[k * pstride + node], nodes ordered with x_1 fastest.  A block covers
// ty rows of tx threads along x_1; a thread handles the nodes x, x + tx, ...
// of its row.  The update reads every stored population once and writes every
// population once per step, so the kernel is bound by HBM bandwidth; there is
// no contraction to put on the matrix cores.
//
// The kernel templates are in kernels.hpp; this file launches the bulk,
// initialisation and reduction kernels, walls.hpp and walls_d*.hip the wall
// kernels.
#include <algorithm>

#include "kernels.hpp"

namespace lbm {

__global__ void __launch_bounds__(kRedThreads)
    k_reduce_final(const double* __restrict__ partial, int nblocks, double* __restrict__ out) {
  __shared__ double sh[kNumAcc * kRedThreads];
  double acc[kNumAcc] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int m = 0; m < kNumAcc; ++m) {
      const double v = partial[b * kNumAcc + m];
      acc[m] = (m == 4) ? fmax(acc[m], v) : acc[m] + v;
    }
  }
  block_reduce(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < kNumAcc; ++m) out[m] = acc[m];
  }
}

// ------------------------------------------------------------- launchers ----

LaunchShape step_shape(const KParams& p) {
  int tx = 64;
  while (tx < p.n[0] && tx < 256) tx *= 2;
  const int ty = 256 / tx;
  LaunchShape s;
  s.tx = tx;
  s.ty = ty;
  s.blocks = static_cast<unsigned>((p.rows + ty - 1) / ty);
  return s;
}

static unsigned grid_for(long long nodes, int threads) {
  long long b = (nodes + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

// Launches of the wall kernels (defined in walls.hpp, instantiated in
// walls_d*.hip, translation units of their own).
template <int D, class T, bool TAN>
void launch_xface(unsigned blocks, hipStream_t stream, T* buf, const KParams& p, double t,
                  int mode);
template <int D, class T, bool TAN>
void launch_wall(dim3 g, dim3 b, hipStream_t stream, const T* src, T* dst, const KParams& p,
                 double t);
template <int D, bool TAN, class PT>
void launch_wall_split(dim3 g, dim3 b, hipStream_t stream, const float* gs, float* gd,
                       const PT* ps, PT* pd, const KParams& p, double t);

template <int D, bool TAN>
static hipError_t step_dt(const KParams& p, int mode, const void* src, void* dst,
                          const double* phi_src, double* phi_dst, long long n,
                          hipStream_t stream, hipEvent_t* ev) {
  const LaunchShape s = step_shape(p);
  const dim3 block(s.tx, s.ty), grid(s.blocks);
  const dim3 wgrid(static_cast<unsigned>((p.wall_rows + s.ty - 1) / s.ty));
  const double t_n = static_cast<double>(n) * p.dt;
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], stream);
  };
  if (p.bc[0] != 0) {
    const unsigned xb = static_cast<unsigned>((2 * p.rows + 255) / 256);
    if (mode == kFP64)
      launch_xface<D, double, TAN>(xb, stream, static_cast<double*>(const_cast<void*>(src)), p,
                                   t_n, mode);
    else
      launch_xface<D, float, TAN>(xb, stream, static_cast<float*>(const_cast<void*>(src)), p,
                                  t_n, mode);
  }
  mark(0);
  if (mode == kFP64) {
    auto* a = static_cast<const double*>(src);
    auto* b = static_cast<double*>(dst);
    hipLaunchKernelGGL((k_step<D, double>), grid, block, 0, stream, a, b, p);
    mark(1);
    if (p.wall_rows > 0)
      launch_wall<D, double, TAN>(wgrid, block, stream, a, b, p, t_n);
  } else if (mode == kFP32) {
    auto* a = static_cast<const float*>(src);
    auto* b = static_cast<float*>(dst);
    hipLaunchKernelGGL((k_step<D, float>), grid, block, 0, stream, a, b, p);
    mark(1);
    if (p.wall_rows > 0)
      launch_wall<D, float, TAN>(wgrid, block, stream, a, b, p, t_n);
  } else if (mode == kSplit) {
    auto* a = static_cast<const float*>(src);
    auto* b = static_cast<float*>(dst);
    hipLaunchKernelGGL((k_step_split<D>), grid, block, 0, stream, a, b, phi_src, phi_dst, p);
    mark(1);
    if (p.wall_rows > 0)
      launch_wall_split<D, TAN, double>(wgrid, block, stream, a, b, phi_src, phi_dst, p, t_n);
  } else {
    auto* a = static_cast<const float*>(src);
    auto* b = static_cast<float*>(dst);
    auto* pa = reinterpret_cast<const float2*>(phi_src);
    auto* pb = reinterpret_cast<float2*>(phi_dst);
    hipLaunchKernelGGL((k_step_hilo<D>), grid, block, 0, stream, a, b, pa, pb, p);
    mark(1);
    if (p.wall_rows > 0)
      launch_wall_split<D, TAN, float2>(wgrid, block, stream, a, b, pa, pb, p, t_n);
  }
  mark(2);
  return hipGetLastError();
}

template <int D>
static hipError_t step_d(const KParams& p, int mode, const void* src, void* dst,
                         const double* phi_src, double* phi_dst, long long n,
                         hipStream_t stream, hipEvent_t* ev) {
  if (p.wall_data)
    return step_dt<D, true>(p, mode, src, dst, phi_src, phi_dst, n, stream, ev);
  return step_dt<D, false>(p, mode, src, dst, phi_src, phi_dst, n, stream, ev);
}

template <class T, bool TAN, bool HALF>
static hipError_t fused_pair_t(const KParams& p, const T* A, T* B, T* C, long long n,
                               hipStream_t stream, hipEvent_t* ev) {
  using S = FuseFwdShape<T, HALF>;
  constexpr int R = (S::TX + 2) * (S::TY + 2);
  constexpr size_t lds = sizeof(T) * (S::SLOTS * R + S::SIDE);
  static_assert(lds <= 160 * 1024, "fused tile exceeds the LDS of a CU");
  constexpr int mode = std::is_same<T, float>::value ? kFP32 : kFP64;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused2<T, HALF>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const LaunchShape s = step_shape(p);
  const dim3 block(s.tx, s.ty);
  const dim3 wgrid(static_cast<unsigned>((p.wall_rows + s.ty - 1) / s.ty));
  const double t0 = static_cast<double>(n) * p.dt, t1 = static_cast<double>(n + 1) * p.dt;
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], stream);
  };
  if (p.bc[0] != 0) {
    const unsigned xb = static_cast<unsigned>((2 * p.rows + 255) / 256);
    launch_xface<3, T, TAN>(xb, stream, const_cast<T*>(A), p, t0, mode);
    launch_xface<3, T, TAN>(xb, stream, B, p, t1, mode);
  }
  if (p.wall_rows > 0)
    launch_wall<3, T, TAN>(wgrid, block, stream, A, C, p, t0);
  const int tiles_xy = ((p.n[0] + S::TX - 1) / S::TX) * ((p.n[1] + S::TY - 1) / S::TY);
  const int zc = fuse_zchunk(tiles_xy, p.n[2]);
  const dim3 grid(static_cast<unsigned>(tiles_xy * ((p.n[2] + zc - 1) / zc)));
  mark(0);
  hipLaunchKernelGGL((k_fused2<T, HALF>), grid, dim3(S::NT), lds, stream, A, B, C, p, zc);
  mark(1);
  if (p.wall_rows > 0)
    launch_wall<3, T, TAN>(wgrid, block, stream, C, B, p, t1);
  mark(2);
  return hipGetLastError();
}

template <bool TAN, bool HALF, bool HILO>
static hipError_t fused_pair_split(const KParams& p, const FusedBufs& fb, long long n,
                                   hipStream_t stream, hipEvent_t* ev) {
  using S = FuseSplitShape<HALF>;
  using PT = std::conditional_t<HILO, float2, double>;
  constexpr int R = (S::TX + 2) * (S::TY + 2);
  constexpr size_t lds = fuse_split_lds<HALF>();
  static_assert(lds <= 160 * 1024, "fused tile exceeds the LDS of a CU");
  static_assert((sizeof(float) * S::SLOTS * R) % 8 == 0, "phi planes must be 8-byte aligned");
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused2_split<HALF, HILO>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  auto* gA = static_cast<const float*>(fb.A);
  auto* gB = static_cast<float*>(fb.B);
  auto* gC = static_cast<float*>(fb.C);
  auto* pA = reinterpret_cast<const PT*>(fb.phiA);
  auto* pB = reinterpret_cast<PT*>(fb.phiB);
  auto* pC = reinterpret_cast<PT*>(fb.phiC);
  const LaunchShape s = step_shape(p);
  const dim3 block(s.tx, s.ty);
  const dim3 wgrid(static_cast<unsigned>((p.wall_rows + s.ty - 1) / s.ty));
  const double t0 = static_cast<double>(n) * p.dt, t1 = static_cast<double>(n + 1) * p.dt;
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], stream);
  };
  if (p.bc[0] != 0) {
    // the x_1-face data of the split mode live in p.xdata; the second step's
    // go to the second array
    KParams p2 = p;
    p2.xdata = fb.xdata2;
    const unsigned xb = static_cast<unsigned>((2 * p.rows + 255) / 256);
    launch_xface<3, float, TAN>(xb, stream, const_cast<float*>(gA), p, t0,
                                static_cast<int>(kSplit));
    launch_xface<3, float, TAN>(xb, stream, gB, p2, t1, static_cast<int>(kSplit));
  }
  if (p.wall_rows > 0)
    launch_wall_split<3, TAN, PT>(wgrid, block, stream, gA, gC, pA, pC, p, t0);
  const int tiles_xy = ((p.n[0] + S::TX - 1) / S::TX) * ((p.n[1] + S::TY - 1) / S::TY);
  const int zc = fuse_zchunk(tiles_xy, p.n[2]);
  const dim3 grid(static_cast<unsigned>(tiles_xy * ((p.n[2] + zc - 1) / zc)));
  mark(0);
  hipLaunchKernelGGL((k_fused2_split<HALF, HILO>), grid, dim3(S::NT), lds, stream, gA, gB, gC,
                     pA, pB, pC, p, static_cast<const double*>(fb.xdata2), zc);
  mark(1);
  if (p.wall_rows > 0)
    launch_wall_split<3, TAN, PT>(wgrid, block, stream, gC, gB, pC, pB, p, t1);
  mark(2);
  return hipGetLastError();
}

template <class T>
static hipError_t fused_pair_m(const KParams& p, const FusedBufs& fb, long long n,
                               hipStream_t stream, hipEvent_t* ev) {
  auto* a = static_cast<const T*>(fb.A);
  auto* b = static_cast<T*>(fb.B);
  auto* c = static_cast<T*>(fb.C);
  const bool half = p.scheme == kHalfWay;
  if (p.wall_data) {
    return half ? fused_pair_t<T, true, true>(p, a, b, c, n, stream, ev)
                : fused_pair_t<T, true, false>(p, a, b, c, n, stream, ev);
  }
  return half ? fused_pair_t<T, false, true>(p, a, b, c, n, stream, ev)
              : fused_pair_t<T, false, false>(p, a, b, c, n, stream, ev);
}

template <class T, bool TAN, bool HALF>
static hipError_t fused_pair2_t(const KParams& p, const T* A, T* B, T* C, long long n,
                                hipStream_t stream, hipEvent_t* ev) {
  using S = FuseShape2<T, HALF>;
  constexpr size_t lds = sizeof(T) * S::SLOTS * (S::TX + 2);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused2_d2<T, HALF>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  constexpr int mode = std::is_same<T, float>::value ? kFP32 : kFP64;
  const LaunchShape s = step_shape(p);
  const dim3 block(s.tx, s.ty);
  const dim3 wgrid(static_cast<unsigned>((p.wall_rows + s.ty - 1) / s.ty));
  const double t0 = static_cast<double>(n) * p.dt, t1 = static_cast<double>(n + 1) * p.dt;
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], stream);
  };
  if (p.bc[0] != 0) {
    const unsigned xb = static_cast<unsigned>((2 * p.rows + 255) / 256);
    launch_xface<2, T, TAN>(xb, stream, const_cast<T*>(A), p, t0, mode);
    launch_xface<2, T, TAN>(xb, stream, B, p, t1, mode);
  }
  if (p.wall_rows > 0)
    launch_wall<2, T, TAN>(wgrid, block, stream, A, C, p, t0);
  const int tiles_x = (p.n[0] + S::TX - 1) / S::TX;
  const int yc = fuse_ychunk(tiles_x, p.n[1]);
  const dim3 grid(static_cast<unsigned>(tiles_x * ((p.n[1] + yc - 1) / yc)));
  mark(0);
  hipLaunchKernelGGL((k_fused2_d2<T, HALF>), grid, dim3(S::NT), lds, stream, A, B, C, p, yc);
  mark(1);
  if (p.wall_rows > 0)
    launch_wall<2, T, TAN>(wgrid, block, stream, C, B, p, t1);
  mark(2);
  return hipGetLastError();
}

template <class T>
static hipError_t fused_pair2_m(const KParams& p, const FusedBufs& fb, long long n,
                                hipStream_t stream, hipEvent_t* ev) {
  auto* a = static_cast<const T*>(fb.A);
  auto* b = static_cast<T*>(fb.B);
  auto* c = static_cast<T*>(fb.C);
  const bool half = p.scheme == kHalfWay;
  if (p.wall_data) {
    return half ? fused_pair2_t<T, true, true>(p, a, b, c, n, stream, ev)
                : fused_pair2_t<T, true, false>(p, a, b, c, n, stream, ev);
  }
  return half ? fused_pair2_t<T, false, true>(p, a, b, c, n, stream, ev)
              : fused_pair2_t<T, false, false>(p, a, b, c, n, stream, ev);
}

hipError_t launch_fused_pair(const KParams& p, int mode, const FusedBufs& fb, long long n,
                             hipStream_t stream, hipEvent_t* ev) {
  if (p.d == 2) {
    if (mode == kFP32) return fused_pair2_m<float>(p, fb, n, stream, ev);
    if (mode == kFP64) return fused_pair2_m<double>(p, fb, n, stream, ev);
    return hipErrorInvalidValue;
  }
  if (p.d != 3) return hipErrorInvalidValue;
  if (mode == kFP32) return fused_pair_m<float>(p, fb, n, stream, ev);
  if (mode == kFP64) return fused_pair_m<double>(p, fb, n, stream, ev);
  if (split_layout(mode)) {
    if (p.bc[0] != 0 && !fb.xdata2) return hipErrorInvalidValue;
    const bool half = p.scheme == kHalfWay;
    if (mode == kHiLo) {
      if (p.wall_data)
        return half ? fused_pair_split<true, true, true>(p, fb, n, stream, ev)
                    : fused_pair_split<true, false, true>(p, fb, n, stream, ev);
      return half ? fused_pair_split<false, true, true>(p, fb, n, stream, ev)
                  : fused_pair_split<false, false, true>(p, fb, n, stream, ev);
    }
    if (p.wall_data)
      return half ? fused_pair_split<true, true, false>(p, fb, n, stream, ev)
                  : fused_pair_split<true, false, false>(p, fb, n, stream, ev);
    return half ? fused_pair_split<false, true, false>(p, fb, n, stream, ev)
                : fused_pair_split<false, false, false>(p, fb, n, stream, ev);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step(const KParams& p, int mode, const void* src, void* dst,
                       const double* phi_src, double* phi_dst, long long n,
                       hipStream_t stream, hipEvent_t* ev) {
  switch (p.d) {
    case 1: return step_d<1>(p, mode, src, dst, phi_src, phi_dst, n, stream, ev);
    case 2: return step_d<2>(p, mode, src, dst, phi_src, phi_dst, n, stream, ev);
    case 3: return step_d<3>(p, mode, src, dst, phi_src, phi_dst, n, stream, ev);
    case 4: return step_d<4>(p, mode, src, dst, phi_src, phi_dst, n, stream, ev);
    default: return hipErrorInvalidValue;
  }
}


template <int D>
static hipError_t init_d(const KParams& p, int mode, void* dst, double* phi_dst,
                         const double* phi0, const double* grad0, hipStream_t stream) {
  const dim3 block(256), grid(grid_for(p.nodes, 256));
  if (mode == kFP64)
    hipLaunchKernelGGL((k_init<D, double>), grid, block, 0, stream, static_cast<double*>(dst),
                       phi_dst, phi0, grad0, p, mode);
  else
    hipLaunchKernelGGL((k_init<D, float>), grid, block, 0, stream, static_cast<float*>(dst),
                       phi_dst, phi0, grad0, p, mode);
  return hipGetLastError();
}

hipError_t launch_init(const KParams& p, int mode, void* dst, double* phi_dst,
                       const double* phi0, const double* grad0, hipStream_t stream) {
  switch (p.d) {
    case 1: return init_d<1>(p, mode, dst, phi_dst, phi0, grad0, stream);
    case 2: return init_d<2>(p, mode, dst, phi_dst, phi0, grad0, stream);
    case 3: return init_d<3>(p, mode, dst, phi_dst, phi0, grad0, stream);
    case 4: return init_d<4>(p, mode, dst, phi_dst, phi0, grad0, stream);
    default: return hipErrorInvalidValue;
  }
}

template <int D>
static hipError_t moments_d(const KParams& p, int mode, const void* f, const double* phi,
                            long long n, double* phi_out, double* partial, double* out,
                            unsigned what, hipStream_t stream) {
  const double t_n = static_cast<double>(n) * p.dt;
  const dim3 block(kRedThreads), grid(kRedBlocks);
  if (mode == kFP64)
    hipLaunchKernelGGL((k_moments<D, double>), grid, block, 0, stream,
                       static_cast<const double*>(f), phi, p, mode, t_n, phi_out, partial, what);
  else
    hipLaunchKernelGGL((k_moments<D, float>), grid, block, 0, stream,
                       static_cast<const float*>(f), phi, p, mode, t_n, phi_out, partial, what);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!(what & (kMomSums | kMomRmse | kMomEntropy))) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, stream, partial, kRedBlocks,
                     out);
  return hipGetLastError();
}

hipError_t launch_moments(const KParams& p, int mode, const void* f, const double* phi,
                          long long n, double* phi_out, double* partial, double* out,
                          unsigned what, hipStream_t stream) {
  switch (p.d) {
    case 1: return moments_d<1>(p, mode, f, phi, n, phi_out, partial, out, what, stream);
    case 2: return moments_d<2>(p, mode, f, phi, n, phi_out, partial, out, what, stream);
    case 3: return moments_d<3>(p, mode, f, phi, n, phi_out, partial, out, what, stream);
    case 4: return moments_d<4>(p, mode, f, phi, n, phi_out, partial, out, what, stream);
    default: return hipErrorInvalidValue;
  }
}

template <class T>
__global__ void __launch_bounds__(256)
    k_count_nonfinite(const T* __restrict__ v, long long n, unsigned* __restrict__ count) {
  unsigned bad = 0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x)
    bad += isfinite(v[i]) ? 0u : 1u;
  if (bad) atomicAdd(count, bad);
}

__global__ void k_zero_count(unsigned* count) { *count = 0u; }

hipError_t launch_count_nonfinite(const void* vals, bool dbl, long long n, unsigned* count,
                                  hipStream_t stream) {
  const dim3 grid(grid_for(n, 256)), block(256);
  if (dbl)
    hipLaunchKernelGGL((k_count_nonfinite<double>), grid, block, 0, stream,
                       static_cast<const double*>(vals), n, count);
  else
    hipLaunchKernelGGL((k_count_nonfinite<float>), grid, block, 0, stream,
                       static_cast<const float*>(vals), n, count);
  return hipGetLastError();
}

hipError_t launch_zero_count(unsigned* count, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, stream, count);
  return hipGetLastError();
}

template <int D>
static hipError_t sum_phi0_d(const KParams& p, const double* arr, double* partial, double* out,
                             hipStream_t stream) {
  hipLaunchKernelGGL((k_sum_phi0<D>), dim3(kRedBlocks), dim3(kRedThreads), 0, stream, arr, p,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, stream, partial, kRedBlocks,
                     out);
  return hipGetLastError();
}

hipError_t launch_sum_phi0(const KParams& p, const double* arr, double* partial, double* out,
                           hipStream_t stream) {
  switch (p.d) {
    case 1: return sum_phi0_d<1>(p, arr, partial, out, stream);
    case 2: return sum_phi0_d<2>(p, arr, partial, out, stream);
    case 3: return sum_phi0_d<3>(p, arr, partial, out, stream);
    case 4: return sum_phi0_d<4>(p, arr, partial, out, stream);
    default: return hipErrorInvalidValue;
  }
}

template <int D>
static hipError_t batch_d(const KParams* kps, void* const* bufs, const BatchTile* tiles,
                          int ntiles, int tx, int ty, int mode, int cur, int nsteps,
                          hipStream_t stream) {
  const dim3 block(tx, ty);
  for (int s = 0; s < nsteps; ++s) {
    const int c = (cur + s) & 1;
    if (mode == kFP64)
      hipLaunchKernelGGL((k_step_batch<D, double>), dim3(ntiles), block, 0, stream, kps,
                         reinterpret_cast<double* const*>(bufs), tiles, c);
    else
      hipLaunchKernelGGL((k_step_batch<D, float>), dim3(ntiles), block, 0, stream, kps,
                         reinterpret_cast<float* const*>(bufs), tiles, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <class T>
static hipError_t batch_pair_t(const KParams* kps, void* const* bufs, const BatchTile2* tiles,
                               int ntiles, int cur, int npairs, hipStream_t stream) {
  using S = FuseShape2<T, false>;
  constexpr size_t lds = sizeof(T) * S::SLOTS * (S::TX + 2);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused2_d2_batch<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  for (int i = 0; i < npairs; ++i) {
    // a two-step pass reads buffer c and writes buffer 1 - c, as one step does
    const int c = (cur + i) & 1;
    hipLaunchKernelGGL((k_fused2_d2_batch<T>), dim3(ntiles), dim3(S::NT), lds, stream, kps,
                       reinterpret_cast<T* const*>(bufs), tiles, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_batch_pair(const KParams* kps, void* const* bufs, const BatchTile2* tiles,
                             int ntiles, int mode, int cur, int npairs, hipStream_t stream) {
  if (mode == kFP64) return batch_pair_t<double>(kps, bufs, tiles, ntiles, cur, npairs, stream);
  if (mode == kFP32) return batch_pair_t<float>(kps, bufs, tiles, ntiles, cur, npairs, stream);
  return hipErrorInvalidValue;
}

template <class T>
static hipError_t batch_resident_t(const KParams* kps, void* const* bufs, const BatchTile2* tiles,
                                   const int* first, const int* order, int count, int cur,
                                   int npairs, hipStream_t stream) {
  using S = FuseShape2<T, false>;
  constexpr size_t lds = sizeof(T) * S::SLOTS * (S::TX + 2);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused2_d2_resident<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_fused2_d2_resident<T>), dim3(static_cast<unsigned>(count)), dim3(S::NT),
                     lds, stream, kps, reinterpret_cast<T* const*>(bufs), tiles, first, order,
                     npairs, cur);
  return hipGetLastError();
}

hipError_t launch_batch_resident(const KParams* kps, void* const* bufs, const BatchTile2* tiles,
                                 const int* first, const int* order, int count, int mode, int cur,
                                 int npairs, hipStream_t stream) {
  if (npairs <= 0 || count <= 0) return hipSuccess;
  if (mode == kFP64)
    return batch_resident_t<double>(kps, bufs, tiles, first, order, count, cur, npairs, stream);
  if (mode == kFP32)
    return batch_resident_t<float>(kps, bufs, tiles, first, order, count, cur, npairs, stream);
  return hipErrorInvalidValue;
}

int batch_pair_tile_width(int mode) {
  return mode == kFP64 ? FuseShape2<double, false>::TX : FuseShape2<float, false>::TX;
}

hipError_t launch_batch(int d, const KParams* kps, void* const* bufs, const BatchTile* tiles,
                        int ntiles, int tx, int ty, int mode, int cur, int nsteps,
                        hipStream_t stream) {
  switch (d) {
    case 1: return batch_d<1>(kps, bufs, tiles, ntiles, tx, ty, mode, cur, nsteps, stream);
    case 2: return batch_d<2>(kps, bufs, tiles, ntiles, tx, ty, mode, cur, nsteps, stream);
    case 3: return batch_d<3>(kps, bufs, tiles, ntiles, tx, ty, mode, cur, nsteps, stream);
    case 4: return batch_d<4>(kps, bufs, tiles, ntiles, tx, ty, mode, cur, nsteps, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbm
