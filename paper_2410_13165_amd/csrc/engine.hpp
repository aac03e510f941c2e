// Device-side parameter block and kernel launchers shared by the C ABI layer
// (capi.hip) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "lattice.hpp"

namespace lbm {

constexpr int kMaxModes = 16;
constexpr int kNumAcc = 6;        // accumulators of the moment reduction
constexpr int kRedBlocks = 1024;  // fixed grid of the deterministic reductions
constexpr int kRedThreads = 256;

enum Scheme : int { kNoWall = 0, kFullWay = 1, kHalfWay = 2 };
// work selected by the `what` mask of lbm_moments (the LBM_MOM_* bits)
enum MomentBits : unsigned { kMomPhi = 1, kMomSums = 2, kMomRmse = 4, kMomEntropy = 8 };
// Storage modes (the values of lbm_precision).  kSplit and kHiLo share the
// layout: float32 g_k = f_k - omega_k phi plus 8 bytes of phi per node
// (float64, or an unevaluated float32 pair hi + lo).
enum Mode : int { kFP64 = 0, kFP32 = 1, kSplit = 2, kHiLo = 3 };
constexpr bool split_layout(int mode) { return mode == kSplit || mode == kHiLo; }
enum FieldKind : int { kFieldNone = 0, kFieldCos = 1, kFieldExp = 2, kFieldTanh = 3 };

// Analytic solution phi*(x, t) = F(x - u t) + R t (see include/lbm.h).
struct FieldDev {
  int kind;
  int nmodes;
  double amp[kMaxModes];
  double phase[kMaxModes];
  double ku[kMaxModes];                 // kappa_j . u
  double kvec[kMaxModes][kMaxDim];
  // half-cell shifts of the half-way wall points, h = dx / 2, per axis a:
  // cos sums (cos(h kappa_ja), sin(h kappa_ja)); exp sums
  // (exp(-h kappa_ja), exp(h kappa_ja))
  double rot[kMaxModes][kMaxDim][2];
  double Rr, W;
  double center[kMaxDim];
};

// Everything a kernel needs about one lattice, passed by value.
struct KParams {
  int d, q;
  int n[kMaxDim];          // nodes per axis, n[0] fastest in memory
  int stride[kMaxDim];     // node strides
  int nodes;
  int rows;                // nodes / n[0]
  long long pstride;       // elements between two population planes
  int bc[kMaxDim];         // 0 periodic, 1 full-way, 2 half-way
  int scheme;              // Scheme of the Dirichlet axes
  int P;                   // wall scheme order
  int K;                   // initialisation order
  double omega[kMaxQ];
  float omega_f[kMaxQ];
  float omega_lo[kMaxQ];    // omega - omega_f, rounded (hi/lo mode)
  signed char cv[kMaxQ][kMaxDim];  // velocities (Sec. 2.3 order)
  int kbar[kMaxQ];                 // c_kbar = -c_k
  double s, tau, dt, dx, R;
  double dtR;              // dt R, the source term of one step (split modes)
  float dtR_hi, dtR_lo;    // dt R as a float32 pair (hi/lo mode)
  float oms_f;             // 1 - s in float32 (hi/lo mode)
  float s_f;
  double origin[kMaxDim];
  double shift[kMaxDim];   // 1/2 on half-way axes, else 0
  double u[kMaxDim];
  double inv_u[kMaxDim];   // 1 / u_j on Dirichlet axes (tangential wall data)
  int wall_data;           // 0: jets of the exact solution; 1: Remark-1 construction
  double phi_ref;          // FP32 mode: mean of phi0
  // rows on a wall of an axis >= 2, listed face by face (see k_wall)
  int nwfaces;
  int wface_axis[2 * kMaxDim];
  int wface_side[2 * kMaxDim];
  int wface_count[2 * kMaxDim];
  int wall_rows;
  // analytic wall data of the x_1 faces: element xoff + row of each
  // population plane (float64 / float32 modes); split mode:
  // xdata[(side * (2d - 1) + slot) * rows + row]
  int xoff;
  double* xdata;
  FieldDev field;
};

// One block of a batched launch: rows row0 .. row0 + blockDim.y - 1 of an
// instance.
struct BatchTile {
  int inst;
  int row0;
};

// Tile of a batched two-step pass (d = 2): instance, first x_1 node, output
// rows y0 .. y1 - 1.
struct BatchTile2 {
  int inst;
  int x0, y0, y1;
};

struct LaunchShape {
  int tx, ty;
  unsigned blocks;
};

LaunchShape step_shape(const KParams& p);

// One time step t_n -> t_{n+1}.  Non-split modes read/write post-collision
// populations; split mode reads/writes (phi, g) pre-collision.
// ev (nullable): three events recorded before the bulk kernel, between the
// bulk and the wall kernel, and after the wall kernel.
hipError_t launch_step(const KParams& p, int mode, const void* src, void* dst,
                       const double* phi_src, double* phi_dst, long long n,
                       hipStream_t stream, hipEvent_t* ev = nullptr);

// Buffers of a two-step pass: A holds the state at t_n, B receives t_{n+2},
// C is a scratch state of the same layout for the rows on and next to the
// walls of x_2 / x_3.  Split mode adds the phi planes and a second x_1-face
// array (the step-2 data; p.xdata holds step 1's).
struct FusedBufs {
  const void* A;
  void* B;
  void* C;
  const double* phiA;
  double* phiB;
  double* phiC;
  double* xdata2;
};

// Two steps t_n -> t_{n+2} of a lattice with d = 3 (any mode) in one pass of
// the bulk kernel (k_fused2, k_fused2_split).  Bitwise equal to two
// launch_step calls.  ev (nullable): three events around the fused kernel and
// after the step-2 wall kernel.
hipError_t launch_fused_pair(const KParams& p, int mode, const FusedBufs& fb, long long n,
                             hipStream_t stream, hipEvent_t* ev = nullptr);

// Initial state from the analytic field (phi0 == nullptr) or from device
// arrays (grad0 == nullptr: fourth-order central differences).
hipError_t launch_init(const KParams& p, int mode, void* dst, double* phi_dst,
                       const double* phi0, const double* grad0, hipStream_t stream);

// Moments of the state at step n selected by `what` (MomentBits); with any
// scalar bit, writes kRedBlocks x kNumAcc partials, then the final kNumAcc
// values into out.
hipError_t launch_moments(const KParams& p, int mode, const void* f, const double* phi,
                          long long n, double* phi_out, double* partial, double* out,
                          unsigned what, hipStream_t stream);

// Count the non-finite values among n float64 (dbl) or float32 values at
// `vals` into *count (added); zero_count sets *count = 0 with a kernel (no
// memset node in a captured graph).
hipError_t launch_count_nonfinite(const void* vals, bool dbl, long long n, unsigned* count,
                                  hipStream_t stream);
hipError_t launch_zero_count(unsigned* count, hipStream_t stream);

// Sum over the nodes of phi0 (analytic when arr == nullptr), into out[0].
hipError_t launch_sum_phi0(const KParams& p, const double* arr, double* partial,
                           double* out, hipStream_t stream);

// nsteps steps of every instance of a batch (periodic lattices of one d and
// precision), one launch per step over the tile table.
hipError_t launch_batch(int d, const KParams* kps, void* const* bufs, const BatchTile* tiles,
                        int ntiles, int tx, int ty, int mode, int cur, int nsteps,
                        hipStream_t stream);

// npairs two-step passes of every instance of a d = 2 batch (float32 or
// float64), one launch per pair over the BatchTile2 table.
hipError_t launch_batch_pair(const KParams* kps, void* const* bufs, const BatchTile2* tiles,
                             int ntiles, int mode, int cur, int npairs, hipStream_t stream);
// x_1 width of the tiles of launch_batch_pair
int batch_pair_tile_width(int mode);

// npairs two-step passes of every instance of a d = 2 batch in one launch:
// block b advances instance order[b] (largest first) through all the pairs,
// over its tiles tiles[first[i] .. first[i + 1]) of launch_batch_pair's table;
// the instances never share a block, so no block waits for another.
hipError_t launch_batch_resident(const KParams* kps, void* const* bufs, const BatchTile2* tiles,
                                 const int* first, const int* order, int count, int mode, int cur,
                                 int npairs, hipStream_t stream);

// Adjoint step lambda^{n+1} -> lambda^n (adjoint.hip).  g: forward state at
// step n (nullable); when given, per-block partial sums of
// <nu^n, (omega 1^T - I) f^n> (without the 1/(1-s) factor of the
// post-collision modes) go to partial[0 .. step_shape(p).blocks).
hipError_t launch_adjoint_step(const KParams& p, int mode, const void* lsrc, void* ldst,
                               const void* g, const double* gphi, double* partial,
                               hipStream_t stream);
// Two adjoint steps lambda^{n+1} -> lambda^{n-1} in one pass (d = 3; the
// layout of the forward two-step pass).  g1, g2: forward states at steps n and
// n - 1 (both nullable); their contractions are added to
// partial[0 .. adjoint_pair_blocks(p, mode)).
hipError_t launch_adjoint_pair(const KParams& p, int mode, const void* lsrc, void* ldst,
                               const void* g1, const void* g2, double* partial,
                               hipStream_t stream);
long long adjoint_pair_blocks(const KParams& p, int mode);
hipError_t launch_adjoint_seed(const KParams& p, int mode, const double* dldphi, void* lam,
                               hipStream_t stream);
// Transpose of the initialisation; partial[0 .. *nblocks) receives the
// contraction of lambda^0 with d f^0 / d tau.
hipError_t launch_adjoint_init(const KParams& p, int mode, const void* lam, const void* g0,
                               const double* g0phi, double* dphi, double* dgrad, bool fd,
                               double* partial, unsigned* nblocks, hipStream_t stream);
hipError_t launch_sum_partials(const double* partial, long long n, double* out,
                               hipStream_t stream);
// Wall-data sensitivities of the adjoint step that consumes lambda^{n+1}
// (lam): adds its contractions with dW/da_j and dW/dtheta_j of the analytic
// field to partial[0 .. wall_grad_partials()); launch_sum_wall_grad reduces
// them to out[0 .. 2 kMaxModes) (d/da_j at j, d/dtheta_j at kMaxModes + j).
long long wall_grad_partials();
hipError_t launch_wall_grad(const KParams& p, int mode, const void* lam, long long n,
                            double* partial, hipStream_t stream);
hipError_t launch_sum_wall_grad(const double* partial, double* out, hipStream_t stream);

// Spectral radius of the amplification matrix over the wave-number grid
// xi = 2 pi j / m, j in [0, m)^d (nxi = m^d points), for count parameter
// points (sigma[pt*d .. pt*d+d), s[pt]); one block per point
// (stability.hip).  min_omega and unconverged are nullable.
hipError_t launch_stability(int d, long long count, const double* sigma, const double* s,
                            double g, int m, long long nxi, double* rho, double* min_omega,
                            int32_t* unconverged, hipStream_t stream);

}  // namespace lbm
