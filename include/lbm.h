/*
 * lbm.h -- C ABI of the MI355X (gfx950) implementation of the unified
 * fourth-order BGK lattice Boltzmann model for the d-dimensional linear
 * hyperbolic equation  d_t phi + u . grad phi = R  (Chen, Chai & Shi,
 * arXiv:2410.13165).
 *
 * What one handle computes (paper references are to that article):
 *   - the DdQ(2d^2+1) lattice of Sec. 2.3 (eqs. d1q3, d2q9, d3q19, ddqq), d = 1..4,
 *     in lattice units c = 1, so dt = dx (acoustic scaling, Sec. 2.2 and Sec. 5);
 *   - equilibria f^eq_k = omega_k phi and sources R_k = omega_k R with
 *     omega = M^{-1} eps, eps from eq. (meq) and the fourth-order moment m4 from
 *     eq. (meq-4rd) (Remark 5), g = 1/2 unless overridden;
 *   - the BGK update eq. (BGK-LB-Evolution) with s = 1/tau (the paper's method is
 *     s = 2, eq. BGK-LB-Evolution-seq2), fused with pull streaming;
 *   - initialisation eq. (ini) / (ini-simp) of order K = 1 or 3;
 *   - Dirichlet walls by the full-way schemes eq. (bun1) (orders 1, 3, 4) or the
 *     half-way schemes eq. (bun2) (orders 1..4), the latter applied as
 *     f_k(x_f, t+dt) = -f*_kbar(x_f, t) + [right side of bun2 at (x_b, t)],
 *     with f* the post-collision value of eq. (collision) (Appendix A);
 *   - diagnostics: phi, the RMSE of eq. (rmse) against an analytic solution, and
 *     the total microscopic entropy sum_x sum_k f_k^2/(2 omega_k) (eqs. entropy,
 *     skfk; conserved for s = 2, R = 0 on periodic lattices, Remark 6).
 *
 * Conventions for every call:
 *   - Return value: LBM_OK (0) or a negative lbm_status.  Nothing throws across
 *     the ABI.  The message of the last failure of a handle is returned by
 *     lbm_last_error(handle); failures of lbm_create are reported by
 *     lbm_last_error(NULL) (per thread).
 *   - Node layout in device memory: x_1 fastest, then x_2, ..., x_d (C order of
 *     an array shaped [N_d]...[N_1]).  dims[0] = N_1.
 *   - Device buffers are owned by the handle and obtained through the allocator
 *     callbacks of lbm_params (or hipMalloc when they are NULL).  Pointers passed
 *     by the caller are borrowed for the duration of the call only.
 *   - All device work is enqueued on lbm_params.stream (a hipStream_t borrowed
 *     from the caller, never destroyed; NULL = the null stream).  Only
 *     lbm_create with an analytic field, lbm_set_initial in LBM_FP32 mode and
 *     lbm_moments with scalars_host != NULL synchronise that stream.
 *   - A handle must not be used from two threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_MAX_DIM 4
#define LBM_MAX_Q 33
#define LBM_MAX_MODES 16
#define LBM_NSCALARS 8

typedef struct lbm_handle lbm_handle;

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,        /* an argument is out of range or inconsistent     */
  LBM_ENOMEM = -2,        /* a device allocation failed                      */
  LBM_EDEVICE = -3,       /* a HIP runtime call or kernel launch failed      */
  LBM_EUNSUPPORTED = -4,  /* valid request this build does not provide       */
  LBM_ENONFINITE = -5     /* non-finite values detected (lbm_params.check_every) */
} lbm_status;

/* Boundary kind of one face (lbm_params.bc[axis][side]).  The two faces of an
   axis are both periodic or both Dirichlet (LBM_EINVAL otherwise), and every
   Dirichlet face of a lattice uses the same scheme: a lattice that mixes
   full-way and half-way faces, on one axis or on two, is LBM_EUNSUPPORTED
   (Sec. 3.2 defines the two schemes; a population entering through faces of
   both kinds at an edge would need a rule the paper does not give). */
typedef enum {
  LBM_BC_PERIODIC = 0,    /* periodic wrap, nodes at origin + i dx                       */
  LBM_BC_FULLWAY = 1,     /* wall on the nodes i = 0 and i = N-1 (Fig. 1, full-way case)  */
  LBM_BC_HALFWAY = 2      /* walls half a cell outside, nodes at origin + (i + 1/2) dx   */
} lbm_bc;

/* How populations are stored and updated. */
typedef enum {
  LBM_FP64 = 0,           /* post-collision populations in float64, float64 arithmetic   */
  LBM_FP32 = 1,           /* post-collision populations in float32 as deviations from the
                             uniform exact state omega_k (phi_mean + R t), float32
                             arithmetic with compensated sums                            */
  LBM_FP32_SPLIT = 2,     /* phi in float64 plus g_k = f_k - omega_k phi in float32,
                             float64 arithmetic                                          */
  LBM_FP32_HILO = 3       /* g_k as in LBM_FP32_SPLIT, phi as an unevaluated pair
                             hi + lo of float32 (the same 8 bytes per node), float32
                             arithmetic with error-free transformations: each
                             population enters as its offset b_k = f_k - omega_k
                             (phi(x) + dt R) from the node's own phi, kept as exact
                             float32 pieces (phi(x - c_k) - phi(x) as the pair
                             (hi' - hi, lo' - lo), omega_k and dt R as float32
                             pairs, products split by fma, sums by TwoSum); the new
                             phi and g_k are rounded once (values a wall scheme
                             sets, and rows on the walls of x_2 .. x_d, use
                             float64).  No tapes or batches.                     */
} lbm_precision;

/* Analytic solution family phi*(x, t) = F(x - u t) + R t used for the analytic
   initial state, the Dirichlet data (with all its time and space derivatives,
   which the wall schemes need) and the RMSE reference. */
typedef enum {
  LBM_FIELD_NONE = 0,
  LBM_FIELD_COS_SUM = 1,     /* F(y) = sum_j a_j cos(kappa_j . y + theta_j)            */
  LBM_FIELD_EXP_SUM = 2,     /* F(y) = sum_j a_j exp(kappa_j . y)                      */
  LBM_FIELD_TANH_BUBBLE = 3  /* F(y) = 1/2 - 1/2 tanh((Rr - |y - center|)/(2W)),
                                Example 2; periodic lattices only                        */
} lbm_field_kind;

/* Which derivatives of the Dirichlet data the wall schemes may use. */
typedef enum {
  LBM_WALL_JETS = 0,        /* every time/space derivative of the exact solution    */
  LBM_WALL_TANGENTIAL = 1   /* only h = phi* on the wall: its time and tangential
                               derivatives; the normal derivatives follow from the
                               equation (Remark 1, with the division by u_j that the
                               printed form omits).  Needs u_j != 0 on every
                               Dirichlet axis j.  A population entering through
                               several walls (edges, corners) uses the data of the
                               lowest such axis.                                     */
} lbm_wall_data;

typedef struct {
  int32_t kind;                 /* lbm_field_kind                                   */
  int32_t n_modes;              /* 1..LBM_MAX_MODES for the sums, ignored otherwise  */
  const double* amps;           /* host, n_modes values a_j (copied)                 */
  const double* kvecs;          /* host, n_modes x d row-major kappa_j (copied)      */
  const double* phases;         /* host, n_modes values theta_j, or NULL for zeros   */
  double Rr, W;                 /* tanh bubble radius and interface width            */
  double center[LBM_MAX_DIM];   /* tanh bubble centre at t = 0                       */
} lbm_field;

typedef struct {
  uint32_t struct_size;         /* sizeof(lbm_params), set by lbm_params_default     */
  double dx;                    /* lattice spacing; dt = dx                           */
  double origin[LBM_MAX_DIM];   /* a_l: lower end of the domain along each axis      */
  double u[LBM_MAX_DIM];        /* transport velocity (sigma = u since c = 1)        */
  double R;                     /* constant source term                               */
  double g;                     /* interpolation weight of eq. (meq-4rd), default 1/2 */
  double m4;                    /* explicit fourth-order moment when use_m4 != 0      */
  int32_t use_m4;
  int32_t bc[LBM_MAX_DIM][2];   /* lbm_bc of the lower [a][0] and upper [a][1] face
                                   of axis a (see lbm_bc for the combinations)        */
  int32_t bc_order;             /* P: full-way {1,3,4}, half-way {1,2,3,4}; default 4 */
  int32_t init_order;           /* K in {1,3}; default 3                              */
  int32_t precision;            /* lbm_precision; default LBM_FP64                    */
  const lbm_field* field;       /* NULL: the caller must call lbm_set_initial, and
                                   every axis must be periodic                        */
  void* (*alloc)(size_t bytes, void* ctx);   /* device allocator, NULL = hipMalloc  */
  void (*free_fn)(void* ptr, void* ctx);     /* matching free, NULL = hipFree       */
  void* alloc_ctx;
  void* stream;                 /* hipStream_t used for all work, borrowed            */
  int32_t wall_data;            /* lbm_wall_data; default LBM_WALL_JETS               */
  int32_t steps_per_pass;       /* 2 (default): lattices with d = 3 (every storage
                                   mode) or d = 2 (LBM_FP32, LBM_FP64) advance two
                                   time steps per pass of the bulk kernel (bitwise the
                                   same result, about half the HBM traffic); 1: one
                                   step per pass.  Other lattices always use 1.        */
  int32_t check_every;          /* M > 0: every M steps lbm_step counts the non-finite
                                   values of one population plane (split mode: phi),
                                   which any non-finite population of a node reaches
                                   through the collision; a call that found some
                                   returns LBM_ENONFINITE.  Calls that ran a check
                                   synchronise the stream.  0 (default): no checks.   */
} lbm_params;

typedef struct {
  int32_t d, q;
  int32_t precision;
  int32_t entropy_stable;       /* 1 when every omega_k > 0 (Sec. 4.1)               */
  int64_t dims[LBM_MAX_DIM];
  int64_t nodes;                /* prod(dims)                                         */
  int64_t step;                 /* n: the state holds time t_n = n dt                 */
  double omega[LBM_MAX_Q];      /* EDF weights in the velocity order of Sec. 2.3      */
  double m4, min_omega;
  double s, dt;
  double phi_ref;               /* LBM_FP32: phi_mean of the deviation reference      */
  int32_t bytes_per_lu;         /* algorithmic HBM bytes per lattice update of a step */
  int32_t steps_per_pass;       /* time steps per bulk-kernel pass lbm_step uses      */
  int64_t pstride;              /* elements between population planes in the state
                                   blob of lbm_get_state (nodes first, then padding) */
} lbm_info_t;

/* Fill p with defaults: dx = 1, origin 0, u 0, R 0, g = 1/2, all axes periodic,
   P = 4, K = 3, LBM_FP64, no field, hipMalloc/hipFree, null stream,
   LBM_WALL_JETS, steps_per_pass = 2, check_every = 0. */
void lbm_params_default(lbm_params* p);

/* Create a lattice with d in 1..4 axes of dims[0..d-1] nodes and relaxation time
   tau = 1/s > 0 (the paper's method: tau = 1/2).  Computes eps, m4 and omega
   (Sec. 2.3, eqs. meq, meq-4rd, omega_k-2), allocates two state buffers and,
   when p->field is given, writes the initial state of order p->init_order
   (eq. ini-simp) from the analytic field.  Parameters outside the entropy-stability
   region are accepted; lbm_info reports min_omega and entropy_stable.
   Errors: LBM_EINVAL (d, dims, tau, dx, orders, bc codes, a periodic face opposite
   a Dirichlet face, a Dirichlet axis without a field, fewer than 2 nodes on a
   Dirichlet axis, more than 2^31-1 nodes), LBM_EUNSUPPORTED (full-way and
   half-way faces in one lattice, a tanh field with walls),
   LBM_ENOMEM, LBM_EDEVICE.  On failure *out is NULL. */
int lbm_create(int d, const int64_t* dims, double tau, const lbm_params* p,
               lbm_handle** out);

/* Initial state at t = 0 from a device float64 field phi0 (layout above) and,
   for K = 3, its gradient grad_phi0 (device float64, d planes of N nodes, plane j
   holding d phi0 / d x_{j+1}).  grad_phi0 = NULL uses fourth-order central
   differences, which needs every axis periodic (LBM_EINVAL otherwise).  Resets
   the step counter to 0. */
int lbm_set_initial(lbm_handle* h, const double* phi0_dev, const double* grad_phi0_dev);

/* Advance n >= 0 time steps of the fused pull-stream + collide kernel with
   the wall schemes applied inline.  With steps_per_pass = 2 (see lbm_params)
   the steps go in pairs through one bulk pass that keeps the intermediate
   state in LDS, plus one single step when n is odd; while a tape is recording
   (lbm_tape_begin) pairs are used only with an even checkpoint interval, never
   across a checkpoint.  The first paired call allocates, through the
   allocator, a scratch state (lbm_state_bytes) when the lattice has Dirichlet
   walls on x_2 or x_3, and in split mode with x_1 walls the x_1-face data of a
   second step (LBM_ENOMEM if that fails).  Asynchronous on the stream. */
int lbm_step(lbm_handle* h, int64_t n);

/* lbm_step for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, hosts that forbid hipMalloc): the same
   kernels and bitwise the same result as lbm_step, but the scratch of the
   two-step passes (the scratch state of lattices with walls on x_2 or x_3,
   the second x_1-face array in split mode) lives in a fixed device array of
   the library, 128 MiB per GPU, held from the first lbm_create on that GPU
   until the process ends.  This call allocates nothing and calls no
   allocator.  Every lbm_step_static on one GPU uses that same array and
   leaves its contents behind (nothing in it has to start at zero): calls
   whose work overlaps on one GPU (lattices stepped concurrently on
   different streams) race, and must be serialised by the caller.
   Errors: as lbm_step, plus LBM_EINVAL when the lattice needs more scratch
   than the array holds (the message gives both sizes) or a tape is
   recording (its checkpoints are allocated), LBM_EDEVICE when the array's
   address could not be obtained. */
int lbm_step_static(lbm_handle* h, int64_t n);

/* Bits of the `what` mask of lbm_moments. */
typedef enum {
  LBM_MOM_PHI = 1,        /* the phi field into phi_out_dev                           */
  LBM_MOM_SUMS = 2,       /* scalars [0], [1], [4], [5]                                */
  LBM_MOM_RMSE = 4,       /* scalars [2], [6]: evaluates the analytic field per node  */
  LBM_MOM_ENTROPY = 8,    /* scalar [3]                                               */
  LBM_MOM_ALL = 15
} lbm_moment_bits;

/* Moments of the current state t_n, only those selected by `what` (one read
   of the stored state; the per-node analytic field is evaluated only for
   LBM_MOM_RMSE).
   phi_out_dev (LBM_MOM_PHI): device float64 buffer of N nodes that receives
     phi(x, t_n) = sum_k f_k (pre-collision, eq. 0-1-meq).
   scalars_host (any scalar bit): host buffer of LBM_NSCALARS doubles that
   receives, NaN where not selected:
     [0] sum_x phi, [1] sum_x phi^2, [2] sum_x (phi - phi*)^2 (NaN without a field),
     [3] sum_x sum_k f_k^2 / (2 omega_k) over the pre-collision populations
         (NaN when s = 1, where they cannot be recovered from the stored state),
     [4] max_x |phi|, [5] number of non-finite phi values,
     [6] RMSE of eq. (rmse) = sqrt([2] / N), [7] t_n (always).
   The reductions are float64 and deterministic; this call synchronises the
   stream when a scalar bit is set.  Errors: LBM_EINVAL for unknown bits, a
   selected output whose pointer is NULL, or no initial state. */
int lbm_moments(lbm_handle* h, uint32_t what, double* phi_out_dev, double* scalars_host);

int lbm_info(const lbm_handle* h, lbm_info_t* out);

/* Size in bytes of the state blob used by lbm_get_state / lbm_set_state. */
int64_t lbm_state_bytes(const lbm_handle* h);
/* Device-to-device copy of the current state (for checkpoints). */
int lbm_get_state(const lbm_handle* h, void* dst_dev);
/* Replace the state by a blob from lbm_get_state of a handle with the same
   parameters, taken at step `step`. */
int lbm_set_state(lbm_handle* h, const void* src_dev, int64_t step);

/* Kernel timing with HIP events recorded on the lattice's stream, for
   benchmarks.  After lbm_profile_begin, each of the next max_launches bulk
   passes (one step, or two with steps_per_pass = 2) records events before the
   bulk kernel, after it, and after the wall kernel of its last step.
   lbm_profile_end synchronises the stream and returns the summed durations in
   milliseconds of the bulk passes (bulk_ms) and of the wall kernels after them
   (wall_ms, 0 without Dirichlet axes >= 2), the number of time steps those
   passes covered (steps) and the number of passes (launches), and releases the
   events.  All outputs are nullable.  Errors: LBM_EINVAL (max_launches < 1 or
   > 2^20, profiling already active / not active), LBM_EDEVICE. */
int lbm_profile_begin(lbm_handle* h, int64_t max_launches);
int lbm_profile_end(lbm_handle* h, double* bulk_ms, double* wall_ms, int64_t* steps,
                    int64_t* launches);

/* Gradients of a final-time misfit L(phi^N) by the adjoint (transposed)
   stream-collide (see adjoint.hip): the step is linear in the populations,
   f^{n+1} = P_in S (C f^n + b) + wall values, so dL/df^n = C^T S^T P_in^T dL/df^{n+1}
   plus, on half-way walls, the local reflected coupling; populations that
   leave the domain carry no adjoint (their replacements come from the wall
   data).
   lbm_tape_begin(h, every) checkpoints the current state (at step n0) and then
   every `every` steps taken by lbm_step (device copies through the allocator).
   lbm_tape_gradient(h, dl_dphi, ...) takes dL/dphi^N (device float64, one value
   per node, N = current step) and returns, all nullable:
     dl_dphi0  (device float64, N nodes)  dL/dphi0, through the transpose of the
               initialisation; with finite-difference gradients (lbm_set_initial
               without grad) their transpose is folded in;
     dl_dgrad0 (device float64, d planes) dL/d(grad phi0) for initial states built
               from an explicit or analytic gradient (tau dt sum_k omega_k (u - c_k) lambda_k);
     dl_dtau   (host) dL/dtau, the sum over the steps of
               <dL/dg^n, (omega 1^T - I) f^n> d s/d tau plus the initialisation's
               tau dependence.  It replays each segment from its checkpoint
               (segment buffers of `every` states), so memory is
               (n_ckpt + every) states; without it no replay is needed.
     dl_dwall  (host, 2 x n_modes) the gradient with respect to the Dirichlet
               data: the populations entering through the walls (eq. bun1
               full-way, the data part of eq. bun2 half-way) are linear in
               the amplitudes a_j of the analytic field and depend on its
               phases theta_j, so dl_dwall[j] = dL/da_j and
               dl_dwall[n_modes + j] = dL/dtheta_j (0 for exponential fields)
               for the field as it enters the wall data of the steps taken
               since lbm_tape_begin (the initial state held fixed).  Needs
               Dirichlet walls and a cos or exp field; the adjoint then runs
               one step per pass.
   The phi0 outputs need a tape that starts at step 0 right after lbm_create
   with a field or lbm_set_initial.  The handle's state is left unchanged.
   Errors: LBM_EINVAL (no tape, a tape that does not cover the current step,
   NULL dl_dphi, phi0 outputs without an initial tape, dl_dwall without
   Dirichlet walls or without a cos/exp field), LBM_EUNSUPPORTED (dL/dtau at
   s = 1 with post-collision storage; lbm_tape_begin on an LBM_FP32_HILO
   lattice), LBM_ENOMEM, LBM_EDEVICE.  lbm_tape_end
   frees the checkpoints; lbm_set_state and lbm_set_initial drop the tape. */
int lbm_tape_begin(lbm_handle* h, int64_t every);
int lbm_tape_gradient(lbm_handle* h, const double* dl_dphi_dev, double* dl_dphi0_dev,
                      double* dl_dgrad0_dev, double* dl_dtau_host, double* dl_dwall_host);
int lbm_tape_end(lbm_handle* h);

/* Host-only helper (no device work): the EDF weights of a DdQ(2d^2+1) lattice.
   omega_out receives 2d^2+1 values in the velocity order of Sec. 2.3, from the
   closed form eq. (omega_k-2) with one m4 for every pair (Remark 5); m4 is the
   interpolation eq. (meq-4rd) with weight g (NaN = 1/2) unless use_m4 != 0.
   m4_out and min_omega_out are nullable.  Entropy stability (Sec. 4.1) holds
   iff *min_omega_out > 0.  Returns LBM_EINVAL for d outside 1..4 or null
   u / omega_out. */
int lbm_equilibrium_weights(int d, const double* u, double g, int use_m4, double m4,
                            double* omega_out, double* m4_out, double* min_omega_out);

/* Stability maps (Sec. 4): for each of `count` parameter points, the
   spectral radius of the amplification matrix of eq. (G) over the wave-number
   grid xi = 2 pi j / m, j in {0..m-1}^d, and the smallest equilibrium weight.
   The matrix is taken for a general relaxation rate s, G(xi) =
   T(xi) [(1 - s) I + s omega 1^T] with T(xi) = diag(exp(-i c_k . xi)) (the
   streaming symbol with the imaginary unit the printed form omits); s = 2 is
   eq. (G).  Point pt has sigma = sigma_dev[pt*d .. pt*d+d) (c = 1, so
   sigma = u) and s = s_dev[pt]; omega comes from eq. (omega_k-2) with m4 from
   eq. (meq-4rd) at weight g (NaN = 1/2).  Outputs, all device arrays of
   `count` entries: rho_dev[pt] = max over the grid of rho(G(xi));
   min_omega_dev[pt] = min_k omega_k (nullable; entropy stability, Prop. 1,
   holds iff it is > 0); unconverged_dev[pt] = the number of grid points whose
   eigenvalue iteration did not settle (nullable; 0 in every tested case).
   The paper's L^2 stability at s = 2 is rho = 1; rho > 1 means growth.
   All pointers are device memory borrowed for the call; the work is queued on
   `stream` (a hipStream_t, NULL = default stream) and the call returns without
   synchronising.  Errors (reported by lbm_last_error(NULL)): LBM_EINVAL for d
   outside 1..4, count < 0 or > 2^31 - 1, m outside 1..2^20, m^d > 2^31,
   non-finite g, or null sigma_dev / s_dev / rho_dev with count > 0;
   LBM_EDEVICE for a failed launch. */
int lbm_stability_map(int d, int64_t count, const double* sigma_dev, const double* s_dev,
                      double g, int32_t m, double* rho_dev, double* min_omega_dev,
                      int32_t* unconverged_dev, void* stream);

/* Batches: many independent periodic lattices of one dimension d and one
   precision (LBM_FP64 or LBM_FP32), each with its own dims, tau, u, R and m4,
   advanced together.  Instance i takes dims[i*d .. i*d+d-1], tau[i] and
   params[i] (periodic axes; one stream for all; the allocator of each
   instance serves its buffers, that of instance 0 the batch tables).
   lbm_batch_step advances every instance by n steps.  d = 2 batches (every
   instance with steps_per_pass = 2) go two steps per pass over a table of
   (instance, x_1 tile, chunk of rows) tiles, in one of two launch forms:
     LBM_BATCH_PER_PAIR   one launch per pair of steps over every tile of every
                          instance (default);
     LBM_BATCH_RESIDENT   one launch for all the pairs of the call, one block
                          per instance: the block advances its instance pair
                          after pair over the instance's tiles, so the
                          per-instance barrier between pairs is the block's
                          own barrier and no block waits for another.
   Odd remainders, and batches without pairs, take one launch per step over a
   table of (instance, row) tiles.  Both forms give bitwise the same states.
   lbm_batch_set_launch(b, form, ychunk) selects the form and the rows per tile
   (8..64, 0 = 64 halved down to 8 while there are fewer than four tiles per
   CU); LBM_EUNSUPPORTED for batches without pairs.
   lbm_batch_tune times every launch the batch can use over trial_steps steps
   (the single-step block shapes 64x4, 128x2, 256x1; with pairs both forms at
   8, 16, 32 and 64 rows per tile), restores the states, keeps the fastest and
   reports config_out[0..4] = {form (-1 without pairs), rows per tile, tx, ty,
   1 if the result came from the cache} and the time per step of the pass form
   that runs.  Results are cached by device (architecture name, CU count), d,
   precision and instance sizes, for the process and, when the environment
   variable LBM_TUNE_CACHE names a file, across processes.
   lbm_batch_instance(b, i) returns the handle of instance i for lbm_moments,
   lbm_info and lbm_get_state; lbm_step, lbm_set_state and tapes on it are
   rejected.  lbm_batch_set_initial takes the instances' phi0 concatenated in
   instance order (and their gradients, d planes per instance, or NULL for
   finite differences).  lbm_batch_moments fills count x LBM_NSCALARS scalars
   (see lbm_moments).  Errors as for the single-lattice calls, plus
   LBM_EUNSUPPORTED for walls or the split mode; messages through
   lbm_batch_last_error (NULL batch: failures of lbm_batch_create). */
typedef enum { LBM_BATCH_PER_PAIR = 0, LBM_BATCH_RESIDENT = 1 } lbm_batch_launch;
typedef struct lbm_batch lbm_batch;
int lbm_batch_create(int count, int d, const int64_t* dims, const double* tau,
                     const lbm_params* params, lbm_batch** out);
int lbm_batch_set_initial(lbm_batch* b, const double* phi0_dev, const double* grad_dev);
int lbm_batch_step(lbm_batch* b, int64_t n);
int lbm_batch_set_launch(lbm_batch* b, int form, int ychunk);
int lbm_batch_tune(lbm_batch* b, int trial_steps, int32_t* config_out, double* ms_per_step_out);
lbm_handle* lbm_batch_instance(const lbm_batch* b, int i);
int lbm_batch_moments(lbm_batch* b, double* scalars_host);
const char* lbm_batch_last_error(const lbm_batch* b);
int lbm_batch_destroy(lbm_batch* b);

/* Streaming probe of the device memory (no lattice): the bandwidth a plain
   float4 grid-stride stream reaches, the denominator of the fraction of what
   the memory system delivers (beside the nominal peak).  kind 0: copy src to
   dst (bytes read + bytes written count); 1: read src (dst receives one float
   per block, so it holds at least 4 * blocks bytes); 2: write dst with
   non-temporal stores.  bytes: the array size, a multiple of 16; blocks of 256
   threads, 1..2^20; iters timed launches after one warm-up, on `stream`
   (hipStream_t, NULL = default), synchronising it.  *gbs_out = bytes moved per
   launch x iters / elapsed.  Errors: LBM_EINVAL for arguments out of range,
   LBM_EDEVICE for a failed launch; lbm_probe_last_error() gives the message. */
int lbm_bandwidth_probe(int kind, void* dst_dev, const void* src_dev, int64_t bytes, int blocks,
                        int iters, void* stream, double* gbs_out);
const char* lbm_probe_last_error(void);

const char* lbm_last_error(const lbm_handle* h);

/* Release all device memory of h (through free_fn).  NULL is accepted. */
int lbm_destroy(lbm_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
