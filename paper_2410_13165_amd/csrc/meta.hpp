// Compile-time helpers shared by the kernel sources: an unrolled loop over a
// constant range and the velocity vectors of the DdQ(2d^2+1) lattice as
// constants (Sec. 2.3 order, lattice.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "lattice.hpp"

namespace lbm {

// f(integral_constant<I>) ... f(integral_constant<N-1>), fully unrolled.
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

struct Vec4i {
  int v[4];
};

// c_k of the D-dimensional lattice, components past D zero.
constexpr Vec4i vel_vec(int D, int k) {
  Vec4i r{{0, 0, 0, 0}};
  for (int a = 0; a < D; ++a) r.v[a] = vel_comp(D, k, a);
  return r;
}

}  // namespace lbm
