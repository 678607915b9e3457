/* blr.h -- C ABI of the MI355X (gfx950) collision hot path for the adaptive
 * dynamical low-rank (DLR) Boltzmann method.
 *
 * Reference: J. Hu and Y. Wang, "An adaptive dynamical low rank method for the
 * nonlinear Boltzmann equation".  Every entry point below names the passage of
 * the paper that defines the operation.
 *
 * Conventions shared by all calls
 *   - Every call returns blr_status; no C++ exception crosses this boundary.
 *     On failure blr_last_error(ctx) returns a message valid until the next
 *     call on the same context.
 *   - Arrays passed in are DEVICE pointers (memory of the context's device)
 *     unless stated otherwise, and are owned by the caller.  The library owns
 *     only its context (tables, workspace, events).
 *   - Work is issued on the context's HIP stream.  blr_collision_pairs is
 *     asynchronous; blr_dlr_step and blr_steady_solve wait once per step
 *     (the rank decision needs the singular values on the host), and the
 *     write of the new state after that wait stays queued on the stream:
 *     readers on another stream order themselves after it.
 *   - One context per host thread.
 *
 * Velocity grid (Sec. 2.1: the collision solver is a discrete velocity method
 * on a uniform grid of [-L, L]^d): nodes v_q = -L + q * 2L/n, q in
 * {0..n-1}^d, stored in C order (last axis fastest), n^d values per function.
 */
#ifndef BLR_H_
#define BLR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct blr_ctx_t* blr_ctx;

typedef enum {
  BLR_OK = 0,
  BLR_ERR_ARG = 1,            /* invalid argument (shape, range, null pointer)   */
  BLR_ERR_NOMEM = 2,          /* device allocation failed                        */
  BLR_ERR_HIP = 3,            /* a HIP runtime call failed                       */
  BLR_ERR_UNSUPPORTED = 4,    /* valid but not built (grid size, dimension)      */
  BLR_ERR_NUMERIC = 5,        /* NaN/Inf or a failed factorisation               */
  BLR_ERR_NOT_CONVERGED = 6   /* steady solve reached max_steps                  */
} blr_status;

typedef enum { BLR_FP32 = 0, BLR_FP64 = 1 } blr_precision;

/* blr_vgrid.flags */
#define BLR_NO_CONSERVE      0x1u  /* skip the FP64 moment-conservation projection   */
#define BLR_PLAIN_SCHEDULE   0x2u  /* one pair at a time, no shift reuse (baseline)   */
#define BLR_GENERIC_FFT      0x4u  /* force the multi-pass FFT path (no fused kernels) */
/* The Carleman form of the fast spectral method instead of the (rho, sigma)
 * form: for 2D Maxwell molecules (gamma = 0) and 3D hard spheres (gamma = 1),
 * the two kernels for which the paper names this algorithm (Sec. 2.1; Sec. 5
 * runs it for every 2D example), the Carleman representation of the
 * operator has a constant kernel 2^(d-1) C and the collision weight splits
 * over directions e on a half sphere into products of two closed-form
 * filters of the modes; Q+ is then a sum over directions of pointwise
 * products of filtered inverse transforms, and the loss is f times the
 * inverse transform of beta(l, l) g^.  m_sigma: 2D, an even number M of
 * equispaced directions on [0, pi); 3D, 38 (one direction per antipodal pair
 * of the Lebedev rule, 19).  m_rho is not used.  BLR_ERR_ARG unless
 * gamma = d - 2. */
#define BLR_CARLEMAN         0x8u
/* De-aliased convolution: the Galerkin sum over l + m = k exactly instead of
 * l + m = k mod n (the circular convolution an n-point transform computes),
 * for every collision form (isotropic, anisotropic, Carleman).  Two inputs
 * without Nyquist modes have products with modes |k_i| <= n - 2.  3D n in
 * {8, 16} and 2D n = 16: the pipeline runs on the grid of 2n points per axis
 * (the band-limited interpolants of the inputs; no sum of two input modes
 * wraps there).  The other grids: the mean of 2^d runs of the pipeline on the
 * interpolants sampled at v + s dv / 2 for every subset s of the axes, each
 * output spectrum with its shift's phase removed; a wrap k + jn (|j_i| <= 1)
 * enters with sign (-1)^(j.s), so only j = 0 survives the mean (2^d times the
 * work of the circular operator, no grid of 2n points).  Either way the
 * output modes k of the n-point mode set are kept and every mode with a
 * component -n/2 is dropped (the rule the inputs follow), so the output is
 * real.  The projection (unless BLR_NO_CONSERVE) acts on that output.  The
 * two evaluations agree to rounding. */
#define BLR_DEALIAS          0x10u

/* Velocity discretisation and collision kernel.
 *   d       velocity dimension, 2 or 3
 *   n       points per axis: 3D n in {8, 16, 24, 32}; 2D n in {16, 32}
 *   L       half width of the velocity box
 *   R       truncation radius of |v - v*|; R <= 0 selects 4L/(3 + sqrt 2)
 *   C,gamma B(|v - v*|) = C |v - v*|^gamma (isotropic: Maxwell gamma = 0,
 *           hard spheres gamma = 1)
 *   m_rho   Gauss-Legendre nodes on [0, R] (1..64)
 *   m_sigma sphere nodes: 2D an even count of equispaced angles (2..64);
 *           3D must be 38 (Lebedev rule exact to degree 9); 0 = default 8 / 38
 *   aniso_n, aniso
 *           anisotropic kernel B(|q|, cos chi) = C |q|^gamma sum_{i < aniso_n}
 *           aniso[i] Y_i(cos chi), cos chi = sigma . q^ the cosine of the
 *           deflection angle, Y_i the Legendre polynomial P_i (3D) or the
 *           Chebyshev polynomial T_i (2D), 1 <= aniso_n <= 5; aniso_n = 0 is
 *           the isotropic kernel (aniso ignored).  The angular integral is then
 *           no longer a closed-form radial factor: every antipodal sphere pair's
 *           product is transformed and weighted on its own (Funk-Hecke factors
 *           |S^{d-1}| (-1)^(i/2) Z_i(theta |k|) Y_i(sigma . k^), Z_i the
 *           spherical Bessel j_i in 3D and J_i in 2D), which costs m_sigma / 2
 *           times the pair transforms of the isotropic case.  Q_s is symmetric
 *           under sigma -> -sigma, so only the even i enter it (odd aniso[i]
 *           are accepted and do not change the result).  The loss carries
 *           aniso[0].  Not with BLR_CARLEMAN.
 */
typedef struct {
  int32_t d, n;
  double L, R;
  double C, gamma;
  int32_t m_rho, m_sigma;
  uint32_t flags;
  int32_t aniso_n;
  double aniso[5];
} blr_vgrid;

blr_status blr_create(int device, void* hip_stream, blr_ctx* out);
blr_status blr_destroy(blr_ctx ctx);
const char* blr_last_error(blr_ctx ctx);

/* Bytes of device workspace that blr_collision_pairs (and the steps built on
 * it) will hold for rank up to r_max at this grid and precision. */
blr_status blr_workspace_bytes(blr_ctx ctx, const blr_vgrid* vg, int32_t r_max,
                               blr_precision prec, size_t* out);

/* Symmetrised pair collisions Q_s(V_i, V_j) = (Q(V_i,V_j) + Q(V_j,V_i)) / 2.
 *
 * Defines: the bilinear collision operator of eq. (collision_operator) with
 * the post-collision velocities of eq. (collision velocity); the low-rank
 * method needs Q only on pairs of velocity basis functions because Q is
 * bilinear and local in x (remark after eq. K-step detailed).  The operator
 * is the Fourier-Galerkin one on the grid: Nyquist modes of the inputs are
 * dropped, convolutions are circular, the radial integral uses m_rho Gauss-
 * Legendre nodes and the angular one the sigma rule (the loss term uses the
 * same sigma rule, so mass is conserved exactly); unless BLR_NO_CONSERVE,
 * each Q_s is then corrected in FP64 by the least-squares projection that
 * zeroes its d+2 discrete moments (mass, momentum, energy).
 *
 *   V      r rows of n^d values (row i = V_i), float (BLR_FP32) or double
 *   r      number of basis functions, 1 <= r <= 64
 *   pairs  HOST int32 [npairs][2], 0 <= i, j < r (order within a pair is
 *          free); read during the call to plan the launch, not retained
 *   Q_out  npairs rows of n^d values, same type as V; row p = Q_s(pairs[p])
 * FP32: FFTs, products and sums in float; the projection in double.
 * FP64: everything in double.  Async on the context stream. */
blr_status blr_collision_pairs(blr_ctx ctx, const blr_vgrid* vg, blr_precision prec,
                               const void* V, int32_t r, const int32_t* pairs,
                               int32_t npairs, void* Q_out);
/* npairs may be 0 (no work).  1 <= npairs <= 4096. */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as blr_collision_pairs, same arguments and results, with every
 * workspace buffer and the quadrature tables in a fixed device array that the
 * library holds on each device it runs on (BLR_NOALLOC_SCRATCH_BYTES, from
 * its first use there until the process ends) instead of in the context's
 * workspace.  The call allocates no device or pinned host memory; it copies
 * its tables and index arrays from pageable host memory on the context
 * stream (such copies may wait for earlier work on that stream).
 *   BLR_ERR_ARG when the call's workspace (shifted fields, products, spectra,
 *   tables) would exceed BLR_NOALLOC_SCRATCH_BYTES; nothing is issued then.
 *   BLR_DEALIAS (a second grid and its tables) is BLR_ERR_UNSUPPORTED here.
 * All calls on one device share that array: calls that overlap on a device
 * (other contexts or streams included) race; serialise them.  Nothing left
 * in the array by an earlier call is relied on. */
#define BLR_NOALLOC_SCRATCH_BYTES (64u << 20)
blr_status blr_collision_pairs_noalloc(blr_ctx ctx, const blr_vgrid* vg, blr_precision prec,
                                       const void* V, int32_t r, const int32_t* pairs,
                                       int32_t npairs, void* Q_out);

/* ------------------------------------------------------------------ DLR -- */

/* One-dimensional physical space along the first velocity axis (the normal
 * shock geometry of Sec. 4 and 5.2, the Fourier flow of Sec. 5.3).  Cells
 * x_p = x_lo + (p + 1/2) dx, dx = (x_hi - x_lo)/nx.  Boundary values
 * (Sec. 2.3, eq. boundary general): at x_lo the boundary function is used
 * where v_1 > 0, at x_hi where v_1 < 0 (device arrays f_left, f_right, n^d
 * doubles each); the outflow halves come from the adjacent interior cell.
 *   wall_left / wall_right = 0: inflow boundary, the boundary function is
 *     the array itself (the prescribed inflow Maxwellian);
 *   = 1: Maxwell diffusive wall at rest in x (any wall velocity tangential):
 *     the array is the wall Maxwellian's shape exp(-|v - u_w|^2 / 2 T_w), any
 *     positive multiple, and must be positive somewhere on the incoming
 *     half; the boundary function is rho_w times it, with rho_w set by zero
 *     net mass flux through the wall, from the distribution leaving the
 *     domain (the adjacent cell) at each use: the ghost values of every
 *     substep, the boundary rows of the basis augmentation, the full-tensor
 *     step.  Other values: BLR_ERR_ARG. */
typedef struct {
  int32_t nx;
  double x_lo, x_hi;
  const double* f_left;
  const double* f_right;
  blr_vgrid v;
  int32_t wall_left, wall_right;
  /* Two-dimensional physical space (Sec. 2.2, the upwind scheme applied along
   * each axis of a rectangular grid; Sec. 2.3 on every face) when ny >= 2:
   * [x_lo, x_hi] x [y_lo, y_hi] with nx x ny cells, cell p = ix ny + iy (the
   * row of F), velocity axis 0 along x and 1 along y.  f_bottom / f_top are
   * the boundary functions of the faces y = y_lo / y_hi (v_2 > 0 / v_2 < 0
   * incoming), wall_bottom / wall_top as wall_left / wall_right.  face_rows
   * bit k (k = 0 x_lo, 1 x_hi, 2 y_lo, 3 y_hi) set: that face's array holds
   * one row of n^d values per face cell (ny rows on an x face, nx on a y
   * face, in order of the other coordinate), for boundary functions that vary
   * along the face; clear: one row for the whole face.  A diffusive wall's
   * rho_w is then set per face cell.  ny = 0 or 1: one-dimensional space
   * (these fields are ignored).  In two dimensions blr_full_step,
   * blr_dlr_step and blr_steady_solve run on the rectangle (the state's X
   * has rows of nx ny values; the rank is capped at nx ny); BLR_STEP_ADD
   * takes one boundary row per face cell and needs 2 (nx + ny) (plus the
   * obstacle's faces, below) <= 64, else BLR_ERR_UNSUPPORTED; steps there
   * run eagerly (no recorded graph). */
  int32_t ny;
  double y_lo, y_hi;
  const double* f_bottom;
  const double* f_top;
  int32_t wall_bottom, wall_top;
  int32_t face_rows;
  /* Obstacle (two-dimensional space only; Sec. 2.3 on the faces of solid
   * cells inside the rectangle).  solid: host array of nx ny bytes (cell
   * ix ny + iy), nonzero = solid, or NULL for none; read at every call.
   * f_obstacle: device, n^d doubles, the shape of the obstacle walls'
   * Maxwellian (any positive multiple, positive somewhere on every incoming
   * half); needed when solid marks a cell.  Solid cells hold no gas: steps
   * set their rows to zero.  Every face between a gas cell and a solid
   * neighbour is a Maxwell diffusive wall whose outward normal points from
   * the gas cell to the solid one: on the incoming half its ghost is rho_w
   * times f_obstacle with rho_w from zero net mass flux through that face,
   * on the outgoing half the gas cell itself.  These faces are numbered after
   * the 2 (nx + ny) face cells of the rectangle, gas cell by gas cell (cell
   * index ascending), within a cell in the order -x, +x, -y, +y of the solid
   * neighbour; a solid cell on the rectangle's edge gives a zero boundary
   * row.  BLR_STEP_ADD takes one boundary row per face: 2 (nx + ny) + the
   * obstacle's faces <= 64. */
  const uint8_t* solid;
  const double* f_obstacle;
} blr_problem;

/* Low-rank state f = sum_ij X_i S_ij V_j (eq. lowrank decomposition) with
 * <X_i,X_j>_x = dx sum X_i X_j = delta_ij and <V_i,V_j>_v = dv^d sum V_i V_j
 * = delta_ij (eq. orthogonality).  Device FP64, caller-owned, sized for r_cap:
 *   X  r_cap rows of nx   (row i = X_i)
 *   S  r_cap x r_cap row-major, leading r x r block used
 *   V  r_cap rows of n^d  (row j = V_j)
 * r is updated by the adaptive steps; 1 <= r <= r_cap <= 64.  Rows r ..
 * r_cap - 1 of X and V are scratch: a step may write them.  step counts
 * the steps taken; seed is reserved (the step draws no random numbers: the
 * random block X_h of the basis augmentation, Sec. 3.1, multiplies a zero
 * block of S, so the step never reads it and uses zero rows). */
typedef struct {
  int32_t r, r_cap;
  double* X;
  double* S;
  double* V;
  int64_t step;
  uint64_t seed;
} blr_state;

/* blr_step_params.flags */
#define BLR_STEP_ADD            0x1u  /* add the boundary basis first (Sec. 3.1) */
#define BLR_STEP_DROP           0x2u  /* drop small singular values of S (Sec. 3.2) */
#define BLR_STEP_FP64_COLLISION 0x4u  /* pair collisions in FP64 (default FP32) */
/* Orthogonalise the added boundary functions against V by Householder QR of
 * [V; V_b] (default: two projection passes with a Cholesky normalisation,
 * which fall back to Householder QR by themselves when a new function lies
 * almost inside span V).  Both give the same step up to rounding. */
#define BLR_STEP_HOUSEHOLDER_ADD 0x8u
/* K- and L-step QR factorisations by Householder QR (default for r <= 16:
 * shifted Cholesky QR in three passes, which falls back to Householder QR
 * by itself when the matrix is numerically rank deficient).  Both give the
 * same step up to rounding. */
#define BLR_STEP_HOUSEHOLDER_QR  0x10u
/* Issue every kernel of the step one by one (default: the device work of a
 * step attempt is recorded as a HIP graph the second time the same
 * configuration -- shapes, arrays, parameters -- is seen, and replayed from
 * then on; kernel timing turns graphs off).  Results are identical. */
#define BLR_STEP_EAGER           0x20u
/* FP32 pair collisions with an FP64 defect correction (1D space only, r_cap
 * <= 32, not with BLR_STEP_FP64_COLLISION).  A refresh step evaluates its
 * pairs in FP64 and in FP32, steps with the FP64 ones, and keeps on the
 * context their difference D_mn = Q_s^64(V_m, V_n) - Q_s^32(V_m, V_n) with the
 * basis V.  Every other step adds to its FP32 pairs the kept defect carried
 * to its own basis W through the bilinearity of Q_s:
 *   Q_ab = Q_s^32(W_a, W_b) + sum_mn R_am R_bn D_mn,   R_am = <W_a, V_m>,
 * and steps with Q_ab in FP64.  Most of the FP32 error of Q_s stays the same
 * while the basis changes little; near a steady state (Sec. 5.1) that part
 * piles up in slowly relaxing modes and shifts the steady state, and the
 * correction removes it.  What is left is the part of the FP32 rounding that
 * changes from step to step.  A refresh step costs one FP64 and one FP32
 * evaluation of the pairs.  A step with this flag refreshes by itself when
 * the context keeps no defect for this velocity grid; blr_steady_solve
 * refreshes on its first step and every blr_solve_params.defect_every
 * steps. */
#define BLR_STEP_FP64_DEFECT     0x40u
/* With BLR_STEP_FP64_DEFECT: make this step a refresh step. */
#define BLR_STEP_DEFECT_REFRESH  0x80u

typedef struct {
  double dt;
  double c_drop;     /* drop_tol = c_drop * err (Sec. 5.1 uses 0.2)            */
  double add_tol;    /* boundary singular values kept if > add_tol (1e-10)    */
  int32_t r_min, r_max;
  uint32_t flags;
} blr_step_params;

/* err: residual estimate of the step; err_ada: the same after the drop
 * (exact, Sec. 5.1); drop_tol = c_drop * err; ranks before the step, added
 * boundary functions, after the drop.  ms_collision: GPU time of the pair
 * collisions (0 when the step ran as a recorded graph); ms_step: GPU time
 * from the start of the step to the rank decision (the final write of the
 * state is not included). */
typedef struct {
  double err, err_ada, drop_tol;
  int32_t r_in, r_added, r_out;
  float ms_collision, ms_step;
} blr_step_info;

/* SVD of a small square FP64 matrix on the device: A = U diag(sig) W^T
 * (trans != 0: of A^T).  The rank truncation of Sec. 3.2 factors the step's
 * new S (r x r) with it, and the augmentation of Sec. 3.1 the R factor of the
 * boundary rows.  A, U, W: device, r x r row-major; sig: device, r values,
 * descending; all caller-owned, A not modified, outputs must not overlap A.
 * One-sided Jacobi on one wavefront (columns of A rotated until every pair is
 * orthogonal to rounding, at most 40 sweeps).  complete != 0: the columns of U
 * whose sigma underflows (<= 1e-14 sigma_1) are completed to an orthonormal
 * U; complete == 0: they are left as computed (zero where sigma is 0).
 * 1 <= r <= 64, else BLR_ERR_ARG.  Asynchronous on the context's stream. */
blr_status blr_svd_small(blr_ctx ctx, const double* A, int32_t r, int32_t trans, int32_t complete,
                         double* U, double* sig, double* W);

/* Truncated SVD of a full f0 (Sec. 2.4, first paragraph: the initial factors
 * are the truncated SVD of f at t = 0).  f0: device FP64, caller-owned, one
 * row of n^d values per cell (nx rows; nx ny on a rectangle, cell ix ny + iy),
 * not modified.  Writes the rank-r factors of sqrt(wx dv^d) f0 = U Sigma W^T
 * (wx = dx, or dx dy on a rectangle) into *state: X_i = U_i / sqrt(wx),
 * V_i = W_i / sqrt(dv^d), S = diag(sigma_1 >= .. >= sigma_r); state->r = r.
 * The SVD is one-sided Jacobi on the device (FP64; no Gram matrix), so every
 * singular value keeps high relative accuracy.  1 <= r <= min(r_cap, cells,
 * n^d), else BLR_ERR_ARG; at most 8192 cells (BLR_ERR_UNSUPPORTED); f0 of
 * rank below r or not finite: BLR_ERR_NUMERIC.  Uses workspace of cells x
 * (n^d + cells) doubles and waits for the result (one host wait per sweep of
 * the Jacobi rotations). */
blr_status blr_state_from_full(blr_ctx ctx, const blr_problem* pb, const double* f0,
                               int32_t r, blr_state* state);

/* One time step: [add boundary basis] -> K-step -> S-step -> L-step with
 * forward Euler and QR (Sec. 2.4, first-order upwind transport of eq.
 * scheme:fullupwind, ghost values of eq. boundary general) -> residual err
 * from the pieces (eqs. err low rank1, err low rank2) -> [drop with
 * drop_tol = c_drop * err] -> err_ada.  On error the state (r, S and the first
 * r rows of X and V) is left unchanged. */
blr_status blr_dlr_step(blr_ctx ctx, const blr_problem* pb, blr_state* state,
                        const blr_step_params* sp, blr_step_info* info);

typedef struct {
  blr_step_params step;
  double res_tol;     /* stop when err_ada <= res_tol (Sec. 5.1)  */
  int64_t max_steps;
  int32_t defect_every; /* with BLR_STEP_FP64_DEFECT: steps between refreshes
                           (<= 0: 4) */
  int32_t reserved;     /* 0 */
} blr_solve_params;

typedef struct {
  int64_t steps;
  double err_ada;
  int32_t r, converged;
  double ms_wall;
  int64_t pair_evals;   /* Q_s(V_i, V_j) evaluations over the steps taken: each
                           step evaluates r(r+1)/2 pairs at its rank after the
                           basis augmentation (a step attempt that is redone
                           counts once) */
} blr_solve_info;

/* Repeated blr_dlr_step until err_ada <= res_tol (Sec. 5.1) or max_steps
 * (then BLR_ERR_NOT_CONVERGED with the state of the last step). */
blr_status blr_steady_solve(blr_ctx ctx, const blr_problem* pb, blr_state* state,
                            const blr_solve_params* p, blr_solve_info* info);

/* --------------------------------------------------------- full tensor -- */

/* One forward-Euler step of the full-tensor discretisation that the low-rank
 * method is projected from (first-order upwind transport, eq. scheme:fullupwind
 * of Sec. 2.2; walls of Sec. 2.3; the reference method of Sec. 5):
 *   f_p <- f_p - dt (v1+ (f_p - f_{p-1}) + v1- (f_{p+1} - f_p)) / dx + dt Q_s(f_p, f_p)
 * for every cell p, with the ghost f_{-1} = f_left where v1 > 0 and
 * f_{nx} = f_right where v1 < 0.  Q_s is the pair operator of
 * blr_collision_pairs (conservation projection unless pb->v.flags has
 * BLR_NO_CONSERVE) in `prec`: FP32 runs the collisions on a float copy of the
 * cells, FP64 in double; transport and the update are FP64.
 *   F         device FP64, nx rows of n^d values (row p = cell p), caller-owned,
 *             updated in place
 *   err_full  host; ||f^{n+1} - f^n||_{L2(x,v)} (eq. err full grid), the
 *             midpoint inner product dx dv^d sum
 * Waits for the step (one host wait).  dt >= 0.  On error F is unchanged
 * unless the error is reported by the device after the update was issued. */
blr_status blr_full_step(blr_ctx ctx, const blr_problem* pb, blr_precision prec, double* F,
                         double dt, double* err_full);

/* ------------------------------------------------------------ serving -- */

/* A server runs many steady solves (blr_steady_solve, Sec. 5.1: the method's
 * target is the steady state of each problem) on one device at once.  It owns
 * `slots` contexts, each with its own HIP stream (default priority) and host
 * thread, so the steps of different solves overlap on the device.  Requests
 * are admitted first in, first out, as soon as a slot is free and the device
 * memory held by the live solves plus the new one's estimate fits in
 * hbm_budget (continuous batching: a request that arrives while others run
 * starts when one of them ends, not when all have).  An idle slot's
 * workspace is released when the budget needs the room.  Each solve runs the
 * same kernels in the same order as blr_steady_solve on a fresh context, so
 * its result does not depend on what else is running.  Slots record their
 * steps as HIP graphs: while a server runs, other threads of the process
 * synchronize their own streams, not the whole device (HIP refuses
 * hipDeviceSynchronize while any stream is being recorded). */
typedef struct blr_server_t* blr_server;

typedef struct {
  int32_t slots;        /* solves on the device at once, 1..16 */
  int64_t hbm_budget;   /* bytes of device workspace the slots may hold;
                           <= 0: no limit */
  int32_t batch_collisions; /* nonzero: the FP32 pair collisions of every live
                           solve on the fused grids (3D velocity, n = 16, 24
                           or 32, 38 directions, one-dimensional space) run
                           together: each step hands its collisions in, and
                           once every such live solve has, they run as one
                           launch sequence over all their bases and pairs,
                           recorded as a HIP graph per composition.  The steps
                           themselves then run unrecorded.  A pair's result is
                           the same in any batch, alone included; it can
                           differ from an unbatched solve's in the last bits
                           (the pair transforms group the radial nodes two by
                           two).  0: each solve runs on its own. */
} blr_server_params;

typedef struct {
  blr_problem problem;      /* copied at submit; f_left, f_right stay
                               caller-owned and unchanged until completion */
  blr_state* state;         /* caller-owned (struct and arrays); updated in
                               place; neither read nor written by the caller
                               until this request's completion is returned */
  blr_solve_params solve;
  int64_t tag;              /* caller's identifier, returned in the completion */
} blr_request;

typedef struct {
  int64_t tag;
  int32_t status;           /* blr_status of the solve: BLR_OK (converged),
                               BLR_ERR_NOT_CONVERGED (max_steps reached), or
                               the error that stopped it (state as after the
                               last successful step) */
  int32_t slot;             /* slot that ran it */
  blr_solve_info info;
  double t_submit, t_admit, t_done;  /* seconds since blr_server_create */
  int64_t bytes;            /* device workspace its slot held at the end */
  char message[128];        /* error text when status is not OK/NOT_CONVERGED */
} blr_completion;

/* Start a server on `device`.  Creates the slot threads and streams. */
blr_status blr_server_create(int device, const blr_server_params* params, blr_server* out);

/* Queue one request (returns at once).  BLR_ERR_ARG for a malformed request
 * (null state, r or r_cap out of range, bad grid); BLR_ERR_NOMEM when its
 * estimate alone exceeds hbm_budget.  Other errors arrive in the completion. */
blr_status blr_server_submit(blr_server sv, const blr_request* req);

/* Completions in the order they finished: waits until at least one is
 * available, or timeout_s seconds (< 0: no limit) have passed, or no request
 * is queued or running; then copies up to max_out of them into out (host)
 * and sets *n_out. */
blr_status blr_server_wait(blr_server sv, int32_t max_out, double timeout_s,
                           blr_completion* out, int32_t* n_out);

/* Requests queued (not yet admitted) and running. */
blr_status blr_server_load(blr_server sv, int64_t* queued, int64_t* running);

/* Seconds since blr_server_create on the server's clock (the clock of the
 * completion times). */
blr_status blr_server_clock(blr_server sv, double* t);

/* With batch_collisions: the batches run so far and the step collisions
 * (one per solve and step attempt) they held; both 0 otherwise. */
blr_status blr_server_batch_stats(blr_server sv, int64_t* rounds, int64_t* jobs);

/* Message of the last failed blr_server_submit (valid until the next one). */
const char* blr_server_last_error(blr_server sv);

/* Stop: queued requests are dropped (their states untouched, no completion),
 * running solves end at their next step boundary, threads are joined and the
 * slot contexts freed. */
blr_status blr_server_destroy(blr_server sv);

/* ----------------------------------------------------------- timing -- */

/* Per-kernel timing for measurement.  mode 1: from now on every kernel launch
 * of the library is bracketed by HIP events on the context stream; mode 0:
 * stop recording; mode 2: discard what was accumulated.  Not part of the
 * method; adds two event records per launch while on. */
blr_status blr_timing(blr_ctx ctx, int32_t mode);

/* Accumulated time of the idx-th distinct kernel name seen since the last
 * reset (synchronises on the recorded events).  name: caller buffer of
 * name_len bytes (NUL-terminated, truncated); ms: total milliseconds;
 * launches: number of launches; bytes: total algorithmic bytes of those
 * launches (the compulsory reads and writes of each kernel's inputs and
 * outputs, counted once).  BLR_ERR_ARG when idx is past the end. */
blr_status blr_timing_read(blr_ctx ctx, int32_t idx, char* name, int32_t name_len,
                           double* ms, int64_t* launches, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* BLR_H_ */
