// Host-side interfaces between the kpcg translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kp_common.h"
#include "kp_slots.h"  // continuous batches (declared for the request server)

struct kp_plan;

namespace kp {

// Closed-form orthonormal eigenbasis (host), see kp_basis.cpp.
int basis_1d(int n, int bc, double* Q, double* lam);

// Device operands of the pseudoinverse preconditioner for one plan.
struct PinvOps {
  int dim;              // 2 or 3
  int prec;             // Prec
  int n[3];             // nx, ny, nz (nz = 1 in 2D)
  int64_t N;            // nx * ny * nz
  const void* Bf[3];    // V_l packed for the forward product (mp_pack)
  const void* Bb[3];    // V_l^T packed for the backward product
  const double* lam[3]; // eigenvalues (FP64)
  int cfg[6];           // tile configuration of each mode product, in order
  const double* gtab = nullptr;   // 2D low-rank preconditioner: G_r in place of Ghat
  double* rpart = nullptr;        // the G product also leaves <R, Z>, ||Z||^2 (spectral)
  double* hpart = nullptr;        // int8 splits: the first product also leaves the sum and
                                  // the sum of squares of its FP64 input (S_SUM, S_SQ)
};
// Blocks per right-hand side of the product that carries Ghat (the number of
// its spectral partial sums).
int pinv_ghat_blocks(const PinvOps& op);
// Blocks per right-hand side of the first product of an int8 split (the
// number of its input sums); 0 for the other precisions.
int pinv_first_blocks(const PinvOps& op);

// G_r, the best rank-r approximation of the 2D Hadamard pseudoinverse with
// g_ij = 1/(ln_i + lq_j) (kp_lowrank.cpp, host), to tab[j*n + i]; 0 or -1.
int lowrank_table(const double* ln, int n, const double* lq, int q, int r, double* tab);

// Mode-product kernel configuration and packed operator layout (kp_modeprod.hip).
int mp_num_configs();
void mp_config(int id, int* wn, int* wm, int* wc);
int mp_default_config(int K, int prec);
bool mp_config_allowed(int id, int prec);
// operator-resident configurations (mp_res) and whether `id` serves K x K
bool mp_config_resident(int id);
bool mp_config_fits(int id, int K);
void pinv_product(const PinvOps& op, int q, const void* in, void* out, int batch, hipStream_t s);
size_t mp_packed_bytes(int K, int prec);
void mp_pack(const double* B, int K, int prec, void* dst);

void pinv_apply(const PinvOps& op, const double* R, double* Z, void* T0, void* T1, int batch,
                const RhsState* st, hipStream_t s);
// Product q alone, with the buffers and arguments pinv_apply gives it.
void pinv_step(const PinvOps& op, int q, const double* R, double* Z, void* T0, void* T1,
               int batch, const RhsState* st, hipStream_t s);

// Grid geometry and boundary conditions of one plan.
struct Geom {
  int nx, ny, nz, dim;
  int bc[3];
  int64_t N;
  int singular;
  double lam_min;   // smallest nonzero eigenvalue of the Kronecker sum
};

// Vector-kernel launchers (kp_vector.hip).  `part` holds NSLOTS x G block
// partials per right-hand side; G is vec_blocks(N, batch).
int vec_blocks(int64_t N, int batch);
// Boundary data (Sec. 3.4.2) and the field eps = -grad u; faces is a device
// array [rhs][axis][end] (null: homogeneous for the field).
void launch_face_updates(const Geom& g, double* h, const double* faces, int batch, hipStream_t s);
void launch_field(const Geom& g, const double* u, double* eps, const double* faces, int batch,
                  hipStream_t s);
// Jacobi(p, omega) preconditioner (Sec. 4.3.1, Algs. 2-3); J is FP64 scratch.
void launch_jacobi(const Geom& g, const double* R, double* Z, double* J, int p, double omega,
                   const RhsState* st, int batch, int G, hipStream_t s);
bool zgrid_fits(const Geom& g);
// Small 2D problems (kp_small.hip): the whole solve in one kernel, one
// workgroup per right-hand side, FP64 pseudoinverse.  Vx, Vy are the full
// eigenbases [n][n] (column = mode), Vxt, Vyt their transposes, lx, ly the
// eigenvalues.
struct SmallOps {
  const double* Vx;
  const double* Vy;
  const double* Vxt;
  const double* Vyt;
  const double* lx;
  const double* ly;
};
bool small_solve_fits(const Geom& g);
void launch_small_solve(const Geom& g, const SmallOps& o, const double* eta, double* U,
                        RhsState* st, RhsState* mirror, double* hist, int hist_stride, int batch,
                        double tol, int max_iter, int flags, hipStream_t s);
// Convergence descriptors of the current iterate U_s into row s of a
// [batch][stride][DIAG_RAW] table (Experiment 5.4), for every right-hand
// side whose iterate s is not yet recorded.
constexpr int DIAG_RAW = 4;
// Low-mode error certificate.  The error U_s - u = -L^+ R_s has squared norm
// sum_m rhat_m^2 / lambda_m^2 over the eigenmodes m of the Kronecker sum;
// the coefficients of the box of the m_a <= CERT_M lowest modes per axis are
// computed exactly (three small FP64 GEMMs on the matrix cores) and every
// other mode is bounded by 1/theta^2, theta the smallest eigenvalue outside
// the box.
constexpr int CERT_M = 32;
struct CertOps {
  const double* V[3];   // per axis [n_a][CERT_M]: its m_a lowest eigenvectors, zero-padded
  const double* w;      // [CERT_M][CERT_M][CERT_M] (z, y, x): 1/lambda^2 in the box, else 0
  double theta2inv;     // 1/theta^2, or 0 when the box holds every mode
};
// C1 and C2 hold the coefficients after the x and y products, `part`
// CERT_PARTS doubles per right-hand side for the per-tile sums of the box.
constexpr int CERT_PARTS = 2 * 2 * CERT_M;   // two sums per tile, at most 2 * CERT_M tiles
void launch_cert(const Geom& g, const CertOps& c, const double* R, double* C1, double* C2,
                 double* part, RhsState* st, int batch, double tol, hipStream_t s);
void launch_diag(const Geom& g, const double* eta, const double* U, double* part, RhsState* st,
                 double* diag, int stride, int batch, hipStream_t s);
// Timing support: fills n doubles with a fixed pseudo-random pattern in
// [-1, 1), marks batch states as running with finite scalars, and launches
// the one kernel of a vector class (stencil, update_ur, dot_rz, update_p)
// as an iteration does; false for other classes.
void launch_fill(double* x, int64_t n, uint64_t seed, hipStream_t s);
void launch_timing_states(RhsState* st, int batch, hipStream_t s);
bool launch_vector_class(int cls, const Geom& g, double* P, double* W, double* R, double* U,
                         double* Z, double* part, const RhsState* st, int batch, int G,
                         int flags, hipStream_t s);
// R_0 = eta_c with its sums; R_0 is stored only when R is not null (a
// nonsingular set uses eta itself), U_0 = 0 only when U is not null (the
// first U/R update takes it as 0 without reading it, the exit step writes it
// for a right-hand side that made no iteration).
// slots: a continuous batch (only JOINING right-hand sides start).
// state_only: only the states are reset; the sums of eta come from the first
// preconditioner product instead (launch_fin_h after it).
void launch_init(const Geom& g, const double* eta, double* R, double* U, double* part,
                 RhsState* st, double* hist, int hist_stride, int batch, int G, hipStream_t s,
                 int slots = 0, bool state_only = false);
// ||eta_c||^2 and its consequences (zero or non-finite right-hand sides) from
// G block sums in the S_SUM and S_SQ slots.
void launch_fin_h(const Geom& g, double* part, RhsState* st, double* hist, int hist_stride,
                  int batch, int G, hipStream_t s);
// Warm start: R_0 = eta_c - L U_0 with its sums and the stopping rule at
// s = 0 (after launch_init without R, which gives ||eta_c||).
void launch_warm(const Geom& g, const double* eta, const double* U, double* R, double* part,
                 RhsState* st, double* hist, int hist_stride, int batch, double tol, int flags,
                 hipStream_t s);
// Gdot > 0: the preconditioner already left Gdot partial sums of <R, Z> etc.
// p_written: P already holds the new P (P_0 = Z_0 written by the application).
void launch_after_pinv(const Geom& g, const double* R, const double* Z, const double* W,
                       double* P, double* part, RhsState* st, int batch, int G, int first,
                       double tol, int flags, hipStream_t s, int Gdot = 0,
                       bool p_written = false);
// A right-hand side's first iteration takes U_0 = 0 without reading it
// (unless it was a warm start); r0: if not null, R_{s-1} is read from it
// (R_0 = eta of a nonsingular set, in a solve's first iteration).  Right-hand
// sides without a preconditioned residual yet are skipped.  first: the
// solve's first iteration from U_0 = 0, whose update also takes the exit
// step's sums of U_1 (the exit step then skips its pass for a right-hand side
// that stopped there).
void launch_iter_head(const Geom& g, double* P, double* W, double* R, double* U, double* part,
                      RhsState* st, double* hist, int hist_stride, int batch, int G, double tol,
                      int flags, hipStream_t s, const double* r0, bool first);
// gate: a continuous batch, where only right-hand sides whose solve ended
// run their exit step, once; the mirror is written for all.
void launch_finish(const Geom& g, const double* eta, double* U, double* part, RhsState* st,
                   RhsState* mirror, int batch, int G, hipStream_t s, int gate = 0);
// Slot marks of a continuous batch: slot < 0 empties every slot, else the
// slot's done code becomes `code` (JOINING or CAPPED).
void launch_slot_set(RhsState* st, int batch, int slot, int code, hipStream_t s);
void launch_laplacian(const Geom& g, const double* P, double* W, int batch, int G, hipStream_t s);
void launch_copy(const Geom& g, const double* src, double* dst, const RhsState* st, int batch,
                 int G, hipStream_t s);

// Solve flags (mirrors include/kpcg.h), plus internal ones above the public
// range.
enum {
  F_NO_PRECOND = 1,
  F_FLEX_BETA = 2,
  F_RESIDUAL_ONLY = 4,
  F_ANORM_STOP = 32,
  F_CERT = 1 << 16,   // the low-mode error certificate runs after the residual test
};

}  // namespace kp

namespace kp {

// Kernel classes for the optional per-launch timing (HIP events).
enum KernelClass {
  KC_STENCIL = 0,   // W = -Delta(P) with <W,P>
  KC_UPDATE_UR,     // U += alpha P, R -= alpha W, ||R||^2
  KC_DOT_RZ,        // <R,Z>, sum Z, ||Z||^2
  KC_UPDATE_P,      // P = Z - mean + beta P
  KC_FINALIZE,      // one-block scalar recurrences
  KC_INIT,          // centering of eta, R_0
  KC_FINISH,        // true residual, centering of U
  KC_MP_Z_FWD,      // mode products of the preconditioner; the Hadamard
  KC_MP_Y_FWD,      // factor rides on the last forward one (z in 3D, y in 2D)
  KC_MP_X_FWD,
  KC_MP_X_BWD,
  KC_MP_Y_BWD,
  KC_MP_Z_BWD,
  KC_COPY,          // Z = R when M = I
  KC_JACOBI,        // Jacobi(p, omega) preconditioner steps
  KC_DIAG,          // convergence descriptors of the iterate (diagnostic solves)
  KC_CERT,          // low-mode error certificate
  KC_SMALL,         // whole solve of a small 2D problem in one kernel
  KC_COUNT
};

// Records begin/end events around a launch when a tracer is active on this
// host thread; no-ops otherwise.
void trace_begin(int cls, hipStream_t s);
void trace_end(int cls, hipStream_t s);

}  // namespace kp
