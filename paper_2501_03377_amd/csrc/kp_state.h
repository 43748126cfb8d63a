// Per right-hand-side state of a solve, shared by the device kernels, the
// solver driver and the request server (plain C++: no device code here).
#pragma once

#include <stdint.h>

namespace kp {

// Termination codes kept per right-hand side on the device.  The slots of a
// continuous batch (the request server) are also IDLE (empty), JOINING (a
// request waits for its start at the next iteration boundary) or CAPPED
// (stopped at its iteration limit).
enum Done {
  RUNNING = 0, CONVERGED = 1, BREAKDOWN = 2, NONFINITE = 3, ZERO_RHS = 4,
  IDLE = 5, JOINING = 6, CAPPED = 7
};
// A right-hand side whose solve has ended (its exit step is due or done).
constexpr bool terminal(int done) {
  return done != RUNNING && done != IDLE && done != JOINING;
}

// Per right-hand-side scalar state of Algorithm 1, resident on the device so
// that no iteration needs a host round trip.
// Delay of the Hestenes-Stiefel error estimate that KP_FLAG_ANORM_STOP uses.
constexpr int HS_DELAY = 4;

struct RhsState {
  double h2;          // ||eta_c||^2
  double mean;        // mean removed from eta (singular operators, eq. 3.6)
  double rho;         // rho_{s-1} = <R_{s-1}, Z_{s-1}>
  double alpha;       // alpha_s
  double beta;        // beta_s
  double rr;          // ||R_s||^2
  double rsum;        // sum of the entries of R_s
  double uu;          // ||U_s||^2
  double pw;          // <W_s, P_{s-1}>
  double wsum;        // sum of the entries of W_s
  double rz;          // <R_s, Z_s> after centering of Z_s
  double zz;          // ||Z_s||^2 after centering
  double zmean;       // mean of Z_s (centering, Remark 4.1)
  double rel_res;     // ||R_s|| / ||eta_c||
  double err_est;     // ||Z_s|| / ||U_s||
  double true_rel_res;// ||eta_c - L U|| / ||eta_c|| at exit
  double umean;       // mean of U removed at exit (singular operators)
  double scale;       // power-of-two scale applied to the preconditioner input
  double inv_scale;   // its inverse, applied to the preconditioner output
  double hs_sum;      // sum of alpha_j rho_{j-1}, j = 1..s (Hestenes-Stiefel terms)
  double hs_ring[4];  // the last HS_DELAY of those terms, term j at j % HS_DELAY
  int iter;           // s
  int done;           // Done code
  int pinv_count;     // preconditioner applications so far
  int diag_iter;      // last iterate whose descriptors were recorded (-1: none)
  int need_cert;      // residual small enough, error bound still to be certified
  int warm;           // U_0 came from the caller (warm start): kept at exit
  int exit_gen;       // gated exit step (continuous batches): 0 due, 1 running, 2 done
  int true_pre;       // the S_TSQ, S_TSUM sums hold the exit step's for the current U
  double u0mean;      // mean of U_0 (singular operators: the iterates keep it)
};

}  // namespace kp
