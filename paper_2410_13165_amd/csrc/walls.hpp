// Launches of the wall-row (k_wall, k_wall_split) and x_1-face (k_xface)
// kernels, compiled per wall-formula variant for d = 2 and 3 (k_wall_split
// for both split-layout modes).  The explicit
// instantiations are spread over walls_d*.hip, translation units of their own
// that compile in parallel with each other and with the bulk kernels.
#pragma once

#include "kernels.hpp"

namespace lbm {

// Per-variant launches of the wall kernels (d = 2 and 3; d = 1 and 4 take the
// run-time variant).
template <int D, class T, bool TAN>
void launch_xface(unsigned blocks, hipStream_t stream, T* buf, const KParams& p, double t,
                  int mode) {
  const dim3 g(blocks), b(256);
  if constexpr (D == 1 || D == 4) {
    hipLaunchKernelGGL((k_xface<D, T, TAN, -1>), g, b, 0, stream, buf, p, t, mode);
  } else {
    switch (wall_variant(p)) {
      case 0: hipLaunchKernelGGL((k_xface<D, T, TAN, 0>), g, b, 0, stream, buf, p, t, mode); break;
      case 1: hipLaunchKernelGGL((k_xface<D, T, TAN, 1>), g, b, 0, stream, buf, p, t, mode); break;
      case 2: hipLaunchKernelGGL((k_xface<D, T, TAN, 2>), g, b, 0, stream, buf, p, t, mode); break;
      default: hipLaunchKernelGGL((k_xface<D, T, TAN, 3>), g, b, 0, stream, buf, p, t, mode);
    }
  }
}

// The wall kernels of d >= 3 take one node per thread: the grid's y covers the
// x_1 chunks of blockDim.x nodes.
inline dim3 wall_grid(int D, dim3 g, dim3 b, const KParams& p) {
  if (D >= 3) g.y = static_cast<unsigned>((p.n[0] + b.x - 1) / b.x);
  return g;
}

template <int D, class T, bool TAN>
void launch_wall(dim3 g, dim3 b, hipStream_t stream, const T* src, T* dst, const KParams& p,
                 double t) {
  g = wall_grid(D, g, b, p);
  if constexpr (D == 1 || D == 4) {
    hipLaunchKernelGGL((k_wall<D, T, TAN, -1>), g, b, 0, stream, src, dst, p, t);
  } else {
    switch (wall_variant(p)) {
      case 0: hipLaunchKernelGGL((k_wall<D, T, TAN, 0>), g, b, 0, stream, src, dst, p, t); break;
      case 1: hipLaunchKernelGGL((k_wall<D, T, TAN, 1>), g, b, 0, stream, src, dst, p, t); break;
      case 2: hipLaunchKernelGGL((k_wall<D, T, TAN, 2>), g, b, 0, stream, src, dst, p, t); break;
      default: hipLaunchKernelGGL((k_wall<D, T, TAN, 3>), g, b, 0, stream, src, dst, p, t);
    }
  }
}

// PT: the phi of the split layout, double (split mode) or float2 (hi/lo mode)
template <int D, bool TAN, class PT>
void launch_wall_split(dim3 g, dim3 b, hipStream_t stream, const float* gs, float* gd,
                       const PT* ps, PT* pd, const KParams& p, double t) {
  g = wall_grid(D, g, b, p);
  if constexpr (D == 1 || D == 4) {
    hipLaunchKernelGGL((k_wall_split<D, TAN, -1, PT>), g, b, 0, stream, gs, gd, ps, pd, p, t);
  } else {
    switch (wall_variant(p)) {
      case 0:
        hipLaunchKernelGGL((k_wall_split<D, TAN, 0, PT>), g, b, 0, stream, gs, gd, ps, pd, p, t);
        break;
      case 1:
        hipLaunchKernelGGL((k_wall_split<D, TAN, 1, PT>), g, b, 0, stream, gs, gd, ps, pd, p, t);
        break;
      case 2:
        hipLaunchKernelGGL((k_wall_split<D, TAN, 2, PT>), g, b, 0, stream, gs, gd, ps, pd, p, t);
        break;
      default:
        hipLaunchKernelGGL((k_wall_split<D, TAN, 3, PT>), g, b, 0, stream, gs, gd, ps, pd, p, t);
    }
  }
}

#define LBM_WALL_INST(D, TAN)                                                        \
  template void launch_xface<D, float, TAN>(unsigned, hipStream_t, float*, const KParams&,  \
                                            double, int);                              \
  template void launch_xface<D, double, TAN>(unsigned, hipStream_t, double*,             \
                                             const KParams&, double, int);             \
  template void launch_wall<D, float, TAN>(dim3, dim3, hipStream_t, const float*, float*,  \
                                           const KParams&, double);                    \
  template void launch_wall<D, double, TAN>(dim3, dim3, hipStream_t, const double*,       \
                                            double*, const KParams&, double);          \
  template void launch_wall_split<D, TAN, double>(dim3, dim3, hipStream_t, const float*,  \
                                                  float*, const double*, double*,          \
                                                  const KParams&, double);                 \
  template void launch_wall_split<D, TAN, float2>(dim3, dim3, hipStream_t, const float*,  \
                                                  float*, const float2*, float2*,          \
                                                  const KParams&, double);

}  // namespace lbm
