/*
 * kpcg -- tensor-structured preconditioned CG for the finite-difference
 * Poisson equation  -Laplace(u) = eta  on a rectangle or a cuboid, on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Chumchal, Marton, Plesinger, Simunkova, "Tensor-structured PCG for
 * finite difference solver of domain patterns in ferroelectric material",
 * arXiv 2501.03377.  The discrete operator is the Kronecker sum of the 1D
 * operators of eq. (3.1) (eqs. 3.2-3.3); the solver is Algorithm 1 (PCG); the
 * preconditioner is the Moore-Penrose pseudoinverse of the operator, built
 * from the 1D eigendecompositions (Algs. 4-5) and applied as three mode
 * products forward, a Hadamard scaling, and three mode products back
 * (Algs. 6-7).
 *
 * Conventions shared by every entry point
 *   Layout.    A grid function is an array of nx*ny*nz doubles with x
 *              fastest, then y, then z: element (i, j, k) at i + nx*(j + ny*k).
 *              This is the paper's vec() order (Sec. 2.1).  A batch of B
 *              right-hand sides is B such arrays back to back.  nz = 1
 *              selects the 2D problem (matrices instead of tensors).
 *   Memory.    Pointers documented as "device" are HIP device allocations
 *              owned by the caller (for example torch.empty(..., device='cuda')),
 *              16-byte aligned.  The library never frees caller memory.
 *   Streams.   Work is enqueued on the plan's HIP stream.  kp_solve blocks
 *              until the solve has finished (kp_solve_async returns at once
 *              with a ticket); kp_apply_* only enqueue.
 *   Errors.    Every call returns a kp_status; negative values are errors and
 *              leave outputs undefined; no call throws across the ABI.
 *   Threads.   One plan must be used by one host thread at a time; distinct
 *              plans are independent.
 *   Units.     Unit grid spacing (eq. 3.1 has unit entries): scale eta by h^2.
 *   Boundary data.  Homogeneous; non-homogeneous Dirichlet/Neumann values
 *              are folded into eta by the caller as in Sec. 3.4.2.
 */
#ifndef KPCG_H
#define KPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary condition per axis, eq. (3.1): corners (alpha, beta, gamma) are
 * P (2,2,-1), D (2,2,0), N (1,1,0), DN (2,1,0), ND (1,2,0). */
enum kp_bc { KP_BC_P = 0, KP_BC_D = 1, KP_BC_N = 2, KP_BC_DN = 3, KP_BC_ND = 4 };

/* Arithmetic of the preconditioner's mode products.  Vectors, residuals,
 * inner products and the solution are FP64 in every mode.  F32 uses FP32
 * matrix cores; BF16 uses BF16 matrix cores with FP32 accumulation and a
 * per-right-hand-side power-of-two input scale; BF16X6 reaches FP32 accuracy
 * on the BF16 matrix cores: both operands are split into three BF16 terms
 * (x = x1 + x2 + x3, each the round-to-nearest remainder of the previous)
 * and the six products xi*bj with i + j <= 4 (1-based) are accumulated in
 * FP32, the dropped terms being below 2^-24 relative; intermediates are FP32
 * and the input scale is as for BF16.  I8X7 reaches FP64 accuracy on the
 * int8 matrix cores: every row of the data (along the contracted axis) and
 * every column of V_l is scaled by a power of two and cut into seven signed
 * 7-bit integer digits; the 28 digit products i + j <= 6 (0-based) are summed
 * exactly in int32 and recombined in FP64, the dropped terms and digits
 * being about 2^-49 relative; intermediates are FP64 and nothing is scaled
 * per right-hand side.  I8X6 does the same with six balanced base-256
 * digits in [-128, 127] (the image of every value truncated to 47 bits and
 * split with carries, so the dropped parts have either sign) and the 21
 * products i + j <= 5, a quarter fewer matrix-core operations than I8X7 at
 * about the same accuracy (each dropped product is at most 2^-48 relative
 * and they take either sign).  I8X7 and I8X6 plans need every axis a multiple
 * of 16 and at most 512 (kp_plan_create returns KP_EINVAL otherwise).  The
 * Hadamard factor of eq. (4.6) is always applied in at least FP32. */
enum kp_prec {
  KP_PREC_F64 = 0, KP_PREC_F32 = 1, KP_PREC_BF16 = 2, KP_PREC_BF16X6 = 3, KP_PREC_I8X7 = 4,
  KP_PREC_I8X6 = 5
};

enum kp_status {
  KP_OK = 0,
  KP_NOT_CONVERGED = 1,   /* warning: max_iter reached; u holds the last iterate */
  KP_EINVAL = -1,         /* invalid argument */
  KP_ENOMEM = -2,         /* device allocation failed or workspace too small */
  KP_EHIP = -3,           /* a HIP runtime call failed */
  KP_ENONFINITE = -4,     /* eta or an iterate contains NaN/Inf */
  KP_EBREAKDOWN = -5,     /* <W,P> <= 0 or rho <= 0 before convergence */
  KP_EBUSY = -6           /* the plan has a solve in flight (kp_solve_async
                             not yet waited for) */
};

/* Solve flags (bitwise or). */
enum kp_flags {
  KP_FLAG_NO_PRECOND = 1,   /* M = I: plain CG (Experiment 5.5's baseline) */
  KP_FLAG_FLEX_BETA = 2,    /* beta_s = <R_s - R_{s-1}, Z_s>/rho_{s-1} instead of
                               Algorithm 1's rho_s/rho_{s-1}; for inexact
                               (low-precision) preconditioners */
  KP_FLAG_RESIDUAL_ONLY = 4,/* stop on the relative residual alone (see kp_solve) */
  KP_FLAG_NO_GRAPH = 8,     /* launch every kernel directly (no HIP graph replay) */
  KP_FLAG_DIAGNOSTICS = 16, /* record the convergence descriptors of every iterate
                               (kp_plan_diagnostics); costs one stencil pass over
                               U and eta per iteration, results are unchanged */
  KP_FLAG_ANORM_STOP = 32,  /* stop on an estimate of the L-norm error instead of
                               the residual tests (see kp_solve) */
  KP_FLAG_WARM_START = 64   /* Algorithm 1 from the U_0 held in u on entry
                               instead of U_0 = 0 (see kp_solve) */
};

typedef struct kp_plan kp_plan;   /* opaque */
typedef struct kp_ticket kp_ticket; /* opaque: a solve in flight (kp_solve_async) */

/* Per right-hand-side outcome of kp_solve. */
typedef struct {
  int32_t status;         /* kp_status of this right-hand side */
  int32_t iterations;     /* s at exit (Algorithm 1's iteration counter) */
  int32_t pinv_applications; /* preconditioner applications, including Z_0 */
  int32_t reserved;
  double rel_res;         /* ||R_s|| / ||eta_c||, recursive residual */
  double true_rel_res;    /* ||eta_c - L u|| / ||eta_c|| recomputed at exit */
  double err_est;         /* relative error estimate at exit: ||Z_s|| / ||U_s||
                             (Z_s approximates the error), or the bound
                             ||R_s|| / (lambda_min ||U_s||) or the low-mode
                             bound when that stopped the solve (see kp_solve;
                             both are bounds for the recursive residual R_s) */
  double removed_mean;    /* mean of eta projected out (singular operators) */
} kp_result;

/* Closed-form orthonormal eigenbasis of the 1D operator L_n of eq. (3.1) for
 * one boundary condition (Lemmas 3.1-3.4, normalised as eq. 4.5 requires).
 * Host memory only; needs no GPU.
 *   n      >= 3
 *   bc     kp_bc
 *   Q      host, n*n doubles, row-major: Q[j*n + c] = entry j of eigenvector c
 *   lambda host, n doubles, ascending eigenvalues
 * Returns KP_OK or KP_EINVAL. */
int kp_basis_1d(int n, int bc, double* Q, double* lambda);

/* Creates a plan: the preconditioner's initialisation (Algs. 4-5) for one
 * grid, boundary-condition triple and precision.  Computes the closed-form
 * bases on the host, uploads V_l, V_l^T and the eigenvalues to the current
 * HIP device once, and records the stream.
 *   out        receives the plan
 *   nx, ny     >= 3;  nz >= 3, or nz == 1 for a 2D problem (bc[2] ignored)
 *   bc         host, 3 kp_bc values for the x, y and z axes
 *   prec       kp_prec
 *   max_batch  largest batch a solve may use (>= 1)
 *   hip_stream hipStream_t to enqueue on (NULL = default stream)
 * Limits: nx*ny*nz < 2^31; ceil(nx/64)*ceil(ny/4) <= 8192; max_batch <= 65535.
 * Returns KP_OK, KP_EINVAL, KP_ENOMEM or KP_EHIP. */
int kp_plan_create(kp_plan** out, int nx, int ny, int nz, const int bc[3], int prec,
                   int max_batch, void* hip_stream);

/* Releases the plan's resident operands and any workspace it allocated. */
void kp_plan_destroy(kp_plan* plan);

/* Device bytes a solve of `batch` right-hand sides needs beyond the caller's
 * eta and u (vectors R, P, W, Z, two preconditioner scratch grids, partial
 * sums and scalar state).  0 for invalid arguments. */
size_t kp_plan_workspace_bytes(const kp_plan* plan, int batch);

/* Device bytes held by the plan itself (eigenvectors and eigenvalues). */
size_t kp_plan_resident_bytes(const kp_plan* plan);

/* Hands the plan a caller-owned device workspace of `bytes` (>=
 * kp_plan_workspace_bytes(plan, max_batch)), replacing any it allocated.
 * Without this call the plan allocates its workspace on first use.
 * Returns KP_OK, KP_EINVAL or KP_ENOMEM (too small). */
int kp_plan_set_workspace(kp_plan* plan, void* dev_ptr, size_t bytes);

/* Changes the stream later calls enqueue on. */
int kp_plan_set_stream(kp_plan* plan, void* hip_stream);

/* W = -Delta_FD(P), eq. (3.2), for `batch` grid functions (the sparse
 * application of Sec. 4.2).  P, W: device, batch*N doubles, must not overlap.
 * Enqueue only. */
int kp_apply_laplacian(kp_plan* plan, const double* P, double* W, int batch);

/* Z = M_p-inv(R), Algs. 6-7, in the plan's precision, for `batch` grid
 * functions.  R, Z: device, batch*N doubles, must not overlap.  No centering
 * is applied.  Uses the plan's workspace.  Enqueue only. */
int kp_apply_pinv(kp_plan* plan, const double* R, double* Z, int batch);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation as kp_apply_pinv with the same kernels and results, but the
 * intermediate grids of the mode products live in a static device array of
 * KP_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on
 * until the process ends; the call allocates nothing (the plan's workspace
 * is not used or created).  Its address is looked up on the first call on a
 * device.  Limit: 2 * ceil256(batch * N * e) <= KP_NOALLOC_SCRATCH_BYTES,
 * e = 8 bytes for F64, I8X7 and I8X6 plans, 4 for F32 and BF16X6, 2 for BF16
 * (e.g. 2^22 FP64 unknowns: 256 x 128 x 128, or 128^3 x 2); beyond it the
 * call returns KP_ENOMEM before any work (kp_last_error says how much was
 * needed).  The plan's device must be current (KP_EINVAL otherwise).  Every
 * call on a device shares that device's array: calls that overlap on one
 * device (other host threads, other streams, plans or processes' streams
 * still running) race and give wrong results; calls ordered on one stream
 * are safe.  Enqueue only.  Returns KP_OK, KP_EINVAL, KP_EBUSY, KP_ENOMEM or
 * KP_EHIP. */
#define KP_NOALLOC_SCRATCH_BYTES (64u << 20)
int kp_apply_pinv_noalloc(kp_plan* plan, const double* R, double* Z, int batch);

/* Solves -Delta_FD(u) = eta for `batch` right-hand sides with Algorithm 1
 * from U_0 = 0 (or from the U_0 in u with KP_FLAG_WARM_START) and the
 * pseudoinverse preconditioner (or M = I with KP_FLAG_NO_PRECOND).
 *   eta       device, batch*N doubles, read only
 *   u         device, batch*N doubles, output; must not overlap eta; with
 *             KP_FLAG_WARM_START it holds U_0 on entry (Algorithm 1's
 *             input, Sec. 4.1)
 *   tol       > 0, relative tolerance
 *   max_iter  >= 1, largest iteration count s
 *   flags     kp_flags
 *   results   host, batch entries (may be NULL)
 *   res_hist  host, batch*(max_iter+1) doubles (may be NULL): ||R_s||/||eta_c||
 *             for s = 0..iterations; entries past `iterations` are 0
 * Singular operators (every axis P or N, Sec. 3.4.1): eta is centred
 * (eq. 3.6; the removed mean is reported), Z_s is centred every iteration
 * (Remark 4.1), and u is returned with zero mean: the minimum-norm solution.
 * Warm start: R_0 = eta_c - L U_0 (one stencil pass); res_hist[0] is
 * ||R_0||/||eta_c|| and the start itself may already stop the solve (s = 0)
 * by the residual test with the lambda_min bound below (or the residual alone
 * with KP_FLAG_RESIDUAL_ONLY); a singular set returns the minimum-norm
 * (zero-mean) solution whatever the mean of U_0; a right-hand side with
 * eta_c = 0 returns u = 0.  With KP_FLAG_ANORM_STOP the estimate below is
 * then relative to the error of U_0 rather than to ||u||_L.  Not with the
 * one-kernel 2D path (the general path runs instead); the serving layer does
 * not take the flag.
 * Stopping: the paper fixes the iteration count (Remark 4.2); here iteration
 * s stops when ||R_s||/||eta_c|| <= tol and, unless KP_FLAG_RESIDUAL_ONLY is
 * set, also the relative error of U_s is bounded by tol, by the first of:
 *   - the bound ||U_s - u|| <= ||R_s|| / lambda_min (lambda_min the smallest
 *     nonzero eigenvalue of the Kronecker sum, from the closed-form spectra),
 *     which costs nothing;
 *   - the sharper bound ||U_s - u||^2 <= sum_box rhat^2 / lambda^2 +
 *     (||R_s||^2 - sum_box rhat^2) / theta^2, where rhat are the exact
 *     coefficients of R_s on the box of the min(n_a, 32) lowest eigenmodes
 *     per axis and theta the smallest eigenvalue outside the box (three
 *     small FP64 GEMMs, about one read of R_s; tried in the iterations where
 *     the solve is expected to stop, i.e. the last of each chunk below);
 *   - the estimate ||Z_s||/||U_s|| <= tol after the next preconditioner
 *     application (Z_s = M(R_s) estimates the error of U_s).
 * With KP_FLAG_ANORM_STOP the rule is instead the A-norm error estimate that
 * Remark 4.2 recommends (Hestenes-Stiefel, as analysed by Strakos and Tichy):
 * with t_j = alpha_j rho_{j-1}, iteration s >= d stops when
 * sqrt((t_{s-d+1} + ... + t_s) / (t_1 + ... + t_s)) <= tol, d = 4, an
 * estimate of ||U_{s-d} - u||_L / ||u||_L (U_s is returned, whose L-norm
 * error is no larger).  It suits slowly converging preconditioners (Jacobi,
 * M = I); with the pseudoinverse it costs d extra iterations.
 * Execution: the solve runs on a stream private to the plan, ordered after
 * earlier work on the plan's stream.  The first chunk of iterations (as many
 * as the previous solve on this plan needed) is captured once as a HIP graph
 * and replayed; the cache is keyed by batch, iteration count, flags, tol,
 * max_iter and u, and invalidated by kp_plan_set_workspace, the tuning calls
 * and kp_plan_set_profiling.  Results are identical with KP_FLAG_NO_GRAPH.
 * 2D plans of at most 64 x 64 with the FP64 pseudoinverse run the whole
 * solve as one kernel, one workgroup per right-hand side (not with
 * KP_FLAG_DIAGNOSTICS, KP_FLAG_NO_PRECOND, KP_FLAG_FLEX_BETA or
 * KP_FLAG_ANORM_STOP, nor with another preconditioner); the same recurrences
 * and stopping rules except the low-mode certificate, with reductions summed
 * in another fixed order, so results agree with the general path to rounding.
 * Returns the most severe per-RHS status (errors first, then
 * KP_NOT_CONVERGED); KP_EINVAL before any work for bad arguments.  Blocks
 * until the results are on the host. */
int kp_solve(kp_plan* plan, const double* eta, double* u, int batch, double tol, int max_iter,
             int flags, kp_result* results, double* res_hist);

/* R_s is Algorithm 1's recursive residual; U_s - u = -L^+ R_s holds for
 * the true residual eta_c - L U_s, which equals R_s up to the rounding the
 * recurrence accumulates (the exit step recomputes the true residual and
 * reports it as true_rel_res, so a caller sees any gap).  The inner
 * products <R, Z> and <W, P> of alpha and beta are FP64 in every precision:
 * with the FP64 and int8 split products <R, Z> comes by Parseval from the
 * FP64 eigenbasis coefficients the application produces anyway, with FP32
 * and BF16 products from an FP64 pass over R and Z.
 *
 * Asynchronous solve.  kp_solve_async validates and enqueues the start of
 * the same solve as kp_solve (same arguments and flags) and returns at once
 * with a ticket; the results and res_hist arrays it was given are written
 * when the solve finishes.  The solve runs on the plan's private stream
 * after earlier work on the plan's stream.  Its first chunk of iterations
 * and the exit step are enqueued at the start; a solve that needs more
 * iterations than the previous solve on the plan is continued by kp_poll or
 * kp_wait (one iteration per call to kp_poll that finds the device idle), so
 * the host must poll or wait for it to progress.  Until kp_wait has returned,
 * the plan belongs to the ticket: every other call on the plan returns
 * KP_EBUSY (kp_plan_destroy finishes the solve first and releases the
 * ticket, which must then not be used), and eta, u, results and res_hist
 * must stay valid.  u is complete when kp_poll has returned 1.
 *   ticket  receives the ticket (NULL on error)
 * Returns KP_OK (enqueued), KP_EBUSY, or the errors kp_solve returns before
 * any work. */
int kp_solve_async(kp_plan* plan, const double* eta, double* u, int batch, double tol,
                   int max_iter, int flags, kp_result* results, double* res_hist,
                   kp_ticket** ticket);
/* Non-blocking: 1 when the solve has finished (results written), 0 while it
 * runs; KP_EINVAL for a NULL ticket. */
int kp_poll(kp_ticket* ticket);
/* Blocks until the solve has finished, releases the ticket (it must not be
 * used again) and returns the solve's status, as kp_solve would have. */
int kp_wait(kp_ticket* ticket);

/* Preconditioner of kp_solve and kp_apply_preconditioner (Sec. 4.3).
 *   KP_PRECOND_PINV    the Moore-Penrose pseudoinverse (Sec. 4.3.3), default
 *   KP_PRECOND_JACOBI  Jacobi(p, omega) (Sec. 4.3.1, Algs. 2-3): `steps` = p
 *                      steps of the weighted Jacobi iteration on L x = R from
 *                      x_0 = 0, splitting D_omega = omega D (eqs. 4.1-4.4);
 *                      p >= 1, omega >= 1 (the paper's experiment uses
 *                      p = 3, omega = 1.3); solves with it stop on the
 *                      relative residual alone (M(R) is no error estimate)
 *   KP_PRECOND_LOWRANK the low-Kronecker-rank approximation of the
 *                      pseudoinverse (Sec. 4.3.2), 2D plans only: `steps` =
 *                      the Kronecker rank r, 1 <= r <= min(KP_LOWRANK_MAX, nx,
 *                      ny).  The best rank-r approximation G_r of the
 *                      Hadamard pseudoinverse (eq. 4.7) is computed on the
 *                      host at this call (kp_lowrank_table) and kept on the
 *                      device (nx*ny doubles); the operator
 *                      sum_rho M_{q,rho} (x) M_{n,rho} is applied in its
 *                      factored form, the pseudoinverse's mode products with
 *                      G_r in place of Ghat.  It may be indefinite for
 *                      1 < r < min(nx, ny), as the paper notes; solves stop
 *                      on the relative residual alone
 * (KP_FLAG_NO_PRECOND still selects M = I per solve.)  Jacobi needs one more
 * FP64 grid of workspace per right-hand side (kp_plan_workspace_bytes
 * follows the current choice); a library-owned workspace is reallocated, a
 * caller-provided one that is too small gives KP_ENOMEM and leaves the
 * choice unchanged.  Returns KP_OK, KP_EINVAL or KP_ENOMEM. */
enum kp_precond { KP_PRECOND_PINV = 0, KP_PRECOND_JACOBI = 1, KP_PRECOND_LOWRANK = 2 };
#define KP_LOWRANK_MAX 16
int kp_plan_set_preconditioner(kp_plan* plan, int kind, int steps, double omega);

/* The low-rank preconditioner's factor (Sec. 4.3.2), host only, no GPU: the
 * best rank-r approximation G_r (Eckart-Young-Mirsky) of the n x q Hadamard
 * pseudoinverse g_ij = 1/(lambda_i(L_n) + lambda_j(L_q)) (0 where the sum is
 * below 1e-13 in modulus; eigenvalues in kp_basis_1d's order for bc_n and
 * bc_q), written to table[j*n + i] (n*q doubles, caller-owned).  Computed by
 * block subspace iteration with r + 6 columns and a Rayleigh-Ritz step, in
 * O(n q (r + 6)) work per iteration.  Returns KP_OK, or KP_EINVAL for bad
 * sizes, boundary conditions, r outside 1..min(KP_LOWRANK_MAX, n, q) or a
 * NULL table. */
int kp_lowrank_table(int n, int bc_n, int q, int bc_q, int rank, double* table);

/* Z = M(R) with the plan's preconditioner (pinv or Jacobi); device
 * pointers, batch grids each, not overlapping; enqueued on the plan's
 * stream.  Returns KP_OK, KP_EINVAL, KP_ENOMEM or KP_EHIP. */
int kp_apply_preconditioner(kp_plan* plan, const double* R, double* Z, int batch);

/* Right-hand side of a problem with non-homogeneous boundary data
 * (Sec. 3.4.2): rhs = eta plus, for every non-periodic axis end, its
 * prescribed value added to each cell next to that face -- at a Dirichlet
 * end the potential of the boundary node (L u = h + i_1 u_B), at a Neumann
 * end the outward normal derivative e of the potential, defined by the ghost
 * node u_0 = u_1 + e (L u = h + i_1 e); cells on edges and corners receive
 * every face they touch.  Solving kp_solve with rhs then gives the potential
 * of the non-homogeneous problem.
 *   eta, rhs  device, batch grids (rhs may equal eta: in place; otherwise
 *             they must not overlap)
 *   faces     host, [batch][dim][2] doubles: value at the beginning and at
 *             the end of each axis (x, y, z); entries of periodic axes must
 *             be 0; NULL means homogeneous data (rhs = eta)
 * Enqueued on the plan's stream (the face data is copied first and the call
 * waits for that copy).  Returns KP_OK, KP_EINVAL (bad pointer, size,
 * alignment, overlap, non-finite or periodic face data), KP_ENOMEM, KP_EHIP. */
int kp_assemble_rhs(kp_plan* plan, const double* eta, double* rhs, int batch,
                    const double* faces);

/* Electric field eps = -grad u (Sec. 1) by second-order central differences
 * at the grid points, eps_a = -(u_{+1} - u_{-1}) / 2 along axis a (unit
 * spacing); a neighbour outside the grid is the periodic wrap, the
 * prescribed potential at a Dirichlet end, or the boundary cell plus the
 * prescribed outward derivative at a Neumann end (faces as for
 * kp_assemble_rhs; NULL: homogeneous).
 *   u    device, batch grids
 *   eps  device, batch * dim grids, [rhs][component x, y(, z)][grid]; must
 *        not overlap u
 * Enqueued on the plan's stream.  Returns KP_OK, KP_EINVAL, KP_ENOMEM or
 * KP_EHIP. */
int kp_field(kp_plan* plan, const double* u, double* eps, int batch, const double* faces);

/* Autotuner for the preconditioner's mode products.  Every product of
 * Algs. 6-7 is one GEMM; several tile shapes are compiled (waves per block,
 * rows and columns per wave).  For each product of this plan the call times
 * every tile shape on `batch` right-hand sides (`reps` launches each, HIP
 * events on the plan's stream, on scratch data in the workspace) and keeps
 * the fastest.  chosen: host, 2*dim ints (may be NULL), receives the choice in
 * product order x, y, z forward then x, y, z backward (2D: x, y, x, y).
 * Results do not depend on the choice beyond floating-point summation order
 * within a tile, which is fixed per shape.  Returns KP_OK, KP_EINVAL,
 * KP_ENOMEM or KP_EHIP. */
int kp_plan_autotune(kp_plan* plan, int batch, int reps, int* chosen);
/* Copies the current tile choices (2*dim ints) to cfg; returns 2*dim or
 * KP_EINVAL.  kp_plan_set_tuning installs saved choices (n must be 2*dim;
 * KP_EINVAL for unknown ids and for an operator-resident id on an axis
 * longer than 128), e.g. from a cache of earlier autotune runs. */
int kp_plan_get_tuning(const kp_plan* plan, int* cfg, int n);
int kp_plan_set_tuning(kp_plan* plan, const int* cfg, int n);
/* Shape of tile configuration `id` for precision `prec` (kp_prec): column
 * fragments per wave (wn), row fragments per wave (wm) and column wave groups
 * (wc) of 16 x 16; a block has 4*wc waves and covers 64*wm rows and
 * 16*wn*wc columns of the GEMM.  Host only, no GPU needed.  Returns KP_OK, or
 * KP_EINVAL if the id is unknown or not compiled for that precision.  A
 * product whose contracted length is not a multiple of 4 (8 in BF16) runs
 * one fixed shape (wn 4, wm 2, wc 2) whatever the choice.  Ids 20 and 21
 * keep the whole operator in LDS and sweep row tiles with persistent blocks;
 * they serve contractions of length at most 128 only (kp_plan_set_tuning
 * refuses them for a longer axis, the autotuner skips them there).  I8X7
 * and I8X6 products run their own kernels (one 16-column fragment per step;
 * contractions of length at most 128 with the whole operator in LDS); their
 * plans accept and report id 13 only. */
int kp_tile_shape(int id, int prec, int* wn, int* wm, int* wc);

/* Per-kernel timing (the library's tracing facility).  When enabled, every
 * kernel launch of the plan is bracketed by HIP events on the plan's stream
 * and its duration is added to one of KP_KERNEL_CLASSES classes, named by
 * kp_kernel_class_name (stencil, vector updates, reductions, the six mode
 * products of Algs. 6-7, ...).  Timing adds two event records per launch;
 * while it is on, kp_solve launches every kernel directly (no graph replay). */
#define KP_KERNEL_CLASSES 18
int kp_plan_set_profiling(kp_plan* plan, int enable);
/* Synchronises the plan's stream, then returns the accumulated milliseconds
 * and launch count of one class.  KP_EINVAL for a bad class. */
int kp_plan_profile(kp_plan* plan, int cls, double* total_ms, int64_t* launches);
/* Clears the accumulated timings. */
int kp_plan_profile_reset(kp_plan* plan);
/* Convergence descriptors of the plan's last kp_solve, which must have been
 * made with KP_FLAG_DIAGNOSTICS (Experiment 5.4 and Remark 4.2).  For every
 * right-hand side b and iterate s = 0 .. hs-1 (hs = that solve's max_iter + 1)
 * out[(b*hs + s)*KP_DIAG_COLUMNS + c] receives, for U_s of Algorithm 1
 * (before the exit centring of a singular problem), with eta_c the centred
 * right-hand side (eq. 3.6):
 *   0  true relative residual ||eta_c - L U_s|| / ||eta_c||
 *   1  recursive relative residual ||R_s|| / ||eta_c|| (as res_hist)
 *   2  kappa_s = U_s^T L U_s - 2 U_s^T eta_c; ||U_s - u||_L^2 = kappa_s + ||u||_L^2
 *   3  the paper's L-norm-of-error proxy sqrt(kappa_s - min_j kappa_j), the
 *      minimum over the recorded iterates of b
 *   4  null-space component |sum U_s| / sqrt(N) (singular operators; else 0)
 *   5  alpha_s rho_{s-1} (0 at s = 0): by the Hestenes-Stiefel identity the
 *      decrease of ||U - u||_L^2 from iterate s-1 to s
 *   6  Hestenes-Stiefel estimate of ||U_s - u||_L: the square root of column
 *      5 summed over the next `delay` recorded iterates (a lower bound that
 *      tightens as the error falls; fewer terms near the last iterate)
 * Rows after a right-hand side's last iterate are NaN.  Host only, no GPU
 * work.  Returns KP_OK, or KP_EINVAL if out is NULL, delay < 1, or (batch,
 * hs) is not the shape of a last solve made with the flag.  The serving
 * layer does not take the flag. */
#define KP_DIAG_COLUMNS 7
int kp_plan_diagnostics(const kp_plan* plan, double* out, int batch, int hs, int delay);

/* Average duration of one kernel of class `cls` (milliseconds), measured
 * as `reps` back-to-back launches between two HIP events on the plan's
 * stream after one warm-up launch: the duration a kernel profiler reports
 * per dispatch, without the launch gaps and event records that per-launch
 * tracing adds.  Classes: the six (2D: four) mode products of Algs. 6-7 with
 * the plan's current tile choices, and the stencil, update_ur, dot_rz and
 * update_p kernels of Alg. 1.  The launch is the one an iteration on `batch`
 * right-hand sides makes (flags: 0 or KP_FLAG_FLEX_BETA, which adds the
 * flexible beta's extra operand), on workspace data: a fixed pseudo-random
 * pattern, each product reading what the previous products of one
 * application produce from it, every right-hand side running.  It overwrites
 * the workspace (never the caller's buffers) and synchronises the plan's
 * stream.  The one-kernel solve of small 2D plans (class "small_solve")
 * is timed on the arguments of the plan's last kp_solve that took that path
 * (its eta, u, tol, max_iter, flags; batch at most its batch): each launch
 * rewrites the same u and the workspace state.  Returns KP_OK, KP_EINVAL
 * (bad class for the plan, no such solve yet, batch, reps outside 1..100000
 * or other flags), KP_ENOMEM or KP_EHIP. */
int kp_plan_time_kernel(kp_plan* plan, int cls, int batch, int flags, int reps, double* avg_ms);
/* Name of a kernel class, "unknown" when out of range. */
const char* kp_kernel_class_name(int cls);

/* Number of captured iteration graphs the plan holds, or -1 if graph capture
 * turned out to be unavailable (solves then launch kernels directly). */
int kp_plan_graph_count(const kp_plan* plan);

/* ------------------------------------------------------------ serving ----
 * A request server on one GPU for streams of independent solves of mixed
 * grids, boundary conditions and tolerances (the serving layer is this
 * library's, not the paper's; every request is one Algorithm 1 solve).  It
 * keeps a cache of plans (the packed eigenbases and
 * eigenvalues of Algs. 4-5, per grid, boundary triple and precision) under an
 * HBM budget, admits a request only when its plan and workspace fit (evicting
 * idle plans least recently used first), and runs `workers` host threads,
 * each with its own HIP stream.  Continuous batching: a free worker takes the
 * oldest queued request and opens a batch of `max_batch` slots on that
 * request's plan; every queued request of the same plan, tolerance,
 * iteration limit and flags takes a free slot, also while the batch runs:
 * it starts at the next step (its R_0, Z_0 are formed in the step in which
 * the other slots make an iteration) and leaves the batch, its answer copied
 * out and its completion posted, at the end of the step in which its own
 * solve ended.  A step is one iteration while a request of the batch's kind
 * waits for a slot, otherwise it runs until the first slot is expected to
 * end (by the iteration count of the plan's previous solve), at most four
 * iterations: fewer host round trips per solve.  The batch closes when no
 * slot is busy.  Each
 * slot runs Algorithm 1 with kp_solve's arithmetic and stopping rules (the
 * low-mode certificate is tried in every iteration), so a request's result
 * is bitwise the same alone and in any mix.
 *
 * Timestamps are seconds on the server's monotonic clock (kp_server_now). */
typedef struct kp_server kp_server;   /* opaque */

enum kp_mem { KP_MEM_DEVICE = 0, KP_MEM_HOST = 1 };

typedef struct {
  int64_t id;             /* caller's tag, returned in the completion */
  int nx, ny, nz;         /* grid; nz = 1 for 2D */
  int bc[3];              /* kp_bc per axis */
  int prec;               /* kp_prec of the preconditioner */
  double tol;             /* stopping tolerance, as kp_solve */
  int max_iter;           /* as kp_solve */
  int flags;              /* as kp_solve (KP_FLAG_NO_GRAPH ignored) */
  int mem;                /* kp_mem: where eta and u live */
  const double* eta;      /* nx*ny*nz doubles; must stay valid and unchanged
                             until the request's completion is returned */
  double* u;              /* nx*ny*nz doubles written before completion, or
                             NULL to discard the solution */
} kp_request;

typedef struct {
  int64_t id;
  int32_t status;         /* kp_status of this right-hand side */
  int32_t iterations;
  int32_t batch;          /* busy slots of its batch when it completed */
  int32_t worker;
  double rel_res, true_rel_res, err_est;
  double t_submit, t_start, t_end;   /* server clock, seconds */
} kp_completion;

typedef struct {
  int64_t submitted, completed,
      batches,            /* continuous batches opened */
      plans_created, plans_evicted, rejected;
  int32_t plans_cached, queued;
  size_t hbm_used, hbm_high_water, hbm_budget;
} kp_server_stats;

/* Starts a server on the current HIP device.  hbm_budget: bytes the server
 * may hold in plans, workspaces and batch staging buffers (0 = no limit);
 * workers >= 1 host threads; max_batch >= 1 right-hand sides per batch.
 * Returns KP_OK, KP_EINVAL, KP_ENOMEM or KP_EHIP. */
int kp_server_create(kp_server** out, size_t hbm_budget, int workers, int max_batch);
/* Queues a request (the descriptor is copied; eta and u are used later, see
 * kp_request).  Never blocks on the GPU.  Returns KP_OK or KP_EINVAL (bad
 * grid, boundary code, precision, tolerance or null eta; flags other than
 * KP_FLAG_NO_PRECOND, KP_FLAG_FLEX_BETA, KP_FLAG_RESIDUAL_ONLY and
 * KP_FLAG_NO_GRAPH (ignored); for KP_PREC_I8X7 and KP_PREC_I8X6 also an
 * axis that is not a multiple of 16 or exceeds 512). */
int kp_server_submit(kp_server* srv, const kp_request* req);
/* Moves up to `max` completions to `out` (host array), waiting up to
 * timeout_s seconds for the first one; returns how many (0 on timeout), or
 * KP_EINVAL.  A request the budget can never hold completes with status
 * KP_ENOMEM. */
int kp_server_poll(kp_server* srv, kp_completion* out, int max, double timeout_s);
/* Seconds on the server's clock. */
double kp_server_now(const kp_server* srv);
/* Counters and HBM use (out: host).  Returns KP_OK or KP_EINVAL. */
int kp_server_stats_get(kp_server* srv, kp_server_stats* out);
/* Description of the most recent failed batch (the HIP call and error, or
 * the failing step), "" if none.  Owned by the server, valid until the next
 * call of this function on it. */
const char* kp_server_last_error(kp_server* srv);
/* Finishes every queued request, stops the workers and frees every plan and
 * buffer; completions not polled are dropped. */
void kp_server_destroy(kp_server* srv);

/* Text of the HIP call and error behind the last KP_EHIP (or allocation
 * failure) returned to the calling host thread; "" if none.  The string is
 * owned by the library and valid until the thread's next call. */
const char* kp_last_error(void);

/* Human-readable name of a status code. */
const char* kp_strerror(int status);

/* Library version string. */
const char* kp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KPCG_H */
