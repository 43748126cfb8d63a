// FP64 vector kernels of Algorithm 1 (Sec. 4.1): the sparse minus Laplacian
// of eq. (3.2), the saxpy-type updates and inner products of Sec. 4.2, the
// centering of eq. (3.6) / Remark 4.1, and the per-RHS scalar recurrences.
//
// Every streaming kernel runs on a (G, batch) grid of 256-thread blocks with a
// grid-stride loop over one right-hand side; block partial sums go to `part`
// and a one-block-per-RHS "finalize" kernel reduces them in a fixed order, so
// results are bitwise reproducible run to run (no floating-point atomics).
#include <math.h>

#include "kp_common.h"
#include "kp_internal.h"

namespace kp {

constexpr int VT = 256;

__device__ __forceinline__ double* slot_ptr(double* part, int rhs, int slot, int G) {
  return part + ((int64_t)rhs * NSLOTS + slot) * G;
}

// One axis of the 3/5/7-point stencil: 2c - lo - hi with the ghost rule of the
// boundary condition (the rows of eq. 3.1): periodic wraps around, a Dirichlet
// end has ghost 0, a Neumann end has ghost equal to the boundary cell (which
// turns its diagonal entry 2 into 1).
__device__ __forceinline__ double axis_term(const double* __restrict__ p, uint32_t idx, int pos,
                                            int n, uint32_t stride, int bc, double c) {
  double lo, hi;
  if (pos > 0) lo = p[idx - stride];
  else if (bc == BC_P) lo = p[idx + (uint32_t)(n - 1) * stride];
  else lo = (bc == BC_N || bc == BC_ND) ? c : 0.0;
  if (pos < n - 1) hi = p[idx + stride];
  else if (bc == BC_P) hi = p[idx - (uint32_t)(n - 1) * stride];
  else hi = (bc == BC_N || bc == BC_DN) ? c : 0.0;
  return (2.0 * c - lo) - hi;
}

__device__ __forceinline__ double minus_laplacian_at(const Geom& g, const double* __restrict__ p,
                                                     uint32_t idx) {
  const uint32_t nx = g.nx, ny = g.ny;
  const uint32_t i = idx % nx, t = idx / nx;
  const uint32_t j = t % ny, k = t / ny;
  const double c = p[idx];
  double v = axis_term(p, idx, i, g.nx, 1u, g.bc[0], c);
  v += axis_term(p, idx, j, g.ny, nx, g.bc[1], c);
  if (g.dim == 3) v += axis_term(p, idx, k, g.nz, nx * ny, g.bc[2], c);
  return v;
}

template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], const int (&slots)[NV],
                                               double* part, int rhs, int G) {
  __shared__ double lds[4 * NV];
  block_sum<NV>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) slot_ptr(part, rhs, slots[q], G)[blockIdx.x] = v[q];
  }
}

template <int NV>
__device__ __forceinline__ void read_partials(const double* part, int rhs, const int (&slots)[NV],
                                              int G, double (&v)[NV]) {
  __shared__ double lds[4 * NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double t = 0.0;
    const double* src = part + ((int64_t)rhs * NSLOTS + slots[q]) * G;
    for (int b = threadIdx.x; b < G; b += VT) t += src[b];
    v[q] = t;
  }
  block_sum<NV>(v, lds);
}

__device__ __forceinline__ void set_scale(RhsState& s, double sq, double N) {
  // power-of-two scale bringing the RMS of the preconditioner input to [1, 2)
  double rms = sqrt(sq / N);
  int e = (rms > 0.0 && isfinite(rms)) ? ilogb(rms) : 0;
  if (e > 900) e = 900;
  if (e < -900) e = -900;
  s.scale = ldexp(1.0, -e);
  s.inv_scale = ldexp(1.0, e);
}

// ----------------------------------------------------------------- init ----
__global__ __launch_bounds__(VT) void k_eta_sum(Geom g, const double* __restrict__ eta,
                                                double* part, int G) {
  const int rhs = blockIdx.y;
  const double* e = eta + (int64_t)rhs * g.N;
  double v[1] = {0.0};
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT) v[0] += e[i];
  const int sl[1] = {S_SUM};
  write_partials<1>(v, sl, part, rhs, G);
}

__global__ __launch_bounds__(VT) void k_fin_mean(Geom g, const double* part, RhsState* st, int G) {
  const int rhs = blockIdx.x;
  double v[1];
  const int sl[1] = {S_SUM};
  read_partials<1>(part, rhs, sl, G, v);
  if (threadIdx.x == 0) {
    RhsState s = {};
    s.mean = g.singular ? v[0] / (double)g.N : 0.0;
    s.scale = s.inv_scale = 1.0;
    st[rhs] = s;
  }
}

__global__ __launch_bounds__(VT) void k_eta_center(Geom g, const double* __restrict__ eta,
                                                   double* __restrict__ R, double* __restrict__ U,
                                                   double* part, const RhsState* st, int G) {
  const int rhs = blockIdx.y;
  const int64_t off = (int64_t)rhs * g.N;
  const double m = st[rhs].mean;
  double v[2] = {0.0, 0.0};
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT) {
    const double r = eta[off + i] - m;      // eq. (3.6); m = 0 if nonsingular
    R[off + i] = r;
    U[off + i] = 0.0;                       // U_0 = 0
    v[0] += r;
    v[1] += r * r;
  }
  const int sl[2] = {S_SUM, S_SQ};
  write_partials<2>(v, sl, part, rhs, G);
}

__global__ __launch_bounds__(VT) void k_fin_h(Geom g, const double* part, RhsState* st,
                                              double* hist, int hist_stride, int G) {
  const int rhs = blockIdx.x;
  double v[2];
  const int sl[2] = {S_SUM, S_SQ};
  read_partials<2>(part, rhs, sl, G, v);
  if (threadIdx.x == 0) {
    RhsState& s = st[rhs];
    s.rsum = v[0];
    s.h2 = v[1];
    s.rr = v[1];
    if (!isfinite(v[1])) {
      s.done = NONFINITE;
    } else if (v[1] == 0.0) {
      s.done = ZERO_RHS;
      s.rel_res = 0.0;
    } else {
      s.rel_res = 1.0;
    }
    if (hist) hist[(int64_t)rhs * hist_stride] = s.rel_res;
    set_scale(s, v[1], (double)g.N);
  }
}

// -------------------------------------------------- after preconditioner ----
// <R, Z>, sum Z, ||Z||^2 and optionally <W, Z> (flexible beta).
__global__ __launch_bounds__(VT) void k_dot_rz(Geom g, const double* __restrict__ R,
                                               const double* __restrict__ Z,
                                               const double* __restrict__ W, double* part,
                                               const RhsState* st, int G) {
  const int rhs = blockIdx.y;
  if (st[rhs].done) return;
  const int64_t off = (int64_t)rhs * g.N;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT) {
    const double z = Z[off + i];
    v[0] += R[off + i] * z;
    v[1] += z;
    v[2] += z * z;
    if (W) v[3] += W[off + i] * z;
  }
  const int sl[4] = {S_DOT, S_SUM, S_SQ, S_AUX2};
  write_partials<4>(v, sl, part, rhs, G);
}

__global__ __launch_bounds__(VT) void k_fin_rho(Geom g, const double* part, RhsState* st, int G,
                                                int first, double tol, int flags) {
  const int rhs = blockIdx.x;
  if (st[rhs].done) return;
  double v[4];
  const int sl[4] = {S_DOT, S_SUM, S_SQ, S_AUX2};
  read_partials<4>(part, rhs, sl, G, v);
  if (threadIdx.x != 0) return;
  RhsState& s = st[rhs];
  const double N = (double)g.N;
  const double zmean = g.singular ? v[1] / N : 0.0;        // Remark 4.1
  const double rz = v[0] - zmean * s.rsum;                 // <R, Z - mean>
  double zz = v[2] - N * zmean * zmean;
  if (zz < 0.0) zz = 0.0;
  s.zmean = zmean;
  s.rz = rz;
  s.zz = zz;
  s.pinv_count += 1;
  if (!isfinite(rz) || !isfinite(zz)) { s.done = NONFINITE; return; }
  if (first) {                                             // rho_0, P_0 = Z_0
    if (!(rz > 0.0)) { s.done = BREAKDOWN; return; }
    s.rho = rz;
    s.beta = 0.0;
    return;
  }
  s.err_est = s.uu > 0.0 ? sqrt(zz / s.uu) : INFINITY;
  if (!(flags & F_RESIDUAL_ONLY) && s.rel_res <= tol && s.err_est <= tol) {
    s.done = CONVERGED;
    return;
  }
  if (!(rz > 0.0)) { s.done = (s.rel_res <= tol) ? CONVERGED : BREAKDOWN; return; }
  if (flags & F_FLEX_BETA) {
    // <R_s - R_{s-1}, Z_s> / rho_{s-1} with R_s - R_{s-1} = -alpha_s W_s
    s.beta = -s.alpha * (v[3] - zmean * s.wsum) / s.rho;
  } else {
    s.beta = rz / s.rho;                                   // beta_s = rho_s / rho_{s-1}
  }
  s.rho = rz;
}

__global__ __launch_bounds__(VT) void k_update_p(Geom g, const double* __restrict__ Z,
                                                 double* __restrict__ P, const RhsState* st,
                                                 int G, int first) {
  const int rhs = blockIdx.y;
  if (st[rhs].done) return;
  const int64_t off = (int64_t)rhs * g.N;
  const double zm = st[rhs].zmean, b = st[rhs].beta;
  if (first) {
    for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT)
      P[off + i] = Z[off + i] - zm;
  } else {
    for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT)
      P[off + i] = (Z[off + i] - zm) + b * P[off + i];   // P_s = Z_s + beta_s P_{s-1}
  }
}

// ------------------------------------------------------- iteration head ----
// W = -Delta(P), with <W, P> and sum W.
__global__ __launch_bounds__(VT) void k_stencil_dot(Geom g, const double* __restrict__ P,
                                                    double* __restrict__ W, double* part,
                                                    const RhsState* st, int G) {
  const int rhs = blockIdx.y;
  if (st && st[rhs].done) return;
  const int64_t off = (int64_t)rhs * g.N;
  const double* p = P + off;
  double v[2] = {0.0, 0.0};
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT) {
    const double w = minus_laplacian_at(g, p, i);
    W[off + i] = w;
    v[0] += w * p[i];
    v[1] += w;
  }
  if (part) {
    const int sl[2] = {S_DOT, S_SUM};
    write_partials<2>(v, sl, part, rhs, G);
  }
}

__global__ __launch_bounds__(VT) void k_fin_alpha(Geom g, const double* part, RhsState* st, int G) {
  const int rhs = blockIdx.x;
  if (st[rhs].done) return;
  double v[2];
  const int sl[2] = {S_DOT, S_SUM};
  read_partials<2>(part, rhs, sl, G, v);
  if (threadIdx.x != 0) return;
  RhsState& s = st[rhs];
  s.pw = v[0];
  s.wsum = v[1];
  if (!isfinite(v[0])) { s.done = NONFINITE; return; }
  if (!(v[0] > 0.0)) { s.done = BREAKDOWN; return; }
  s.alpha = s.rho / v[0];                                  // alpha_s
}

__global__ __launch_bounds__(VT) void k_update_ur(Geom g, const double* __restrict__ P,
                                                  const double* __restrict__ W,
                                                  double* __restrict__ R, double* __restrict__ U,
                                                  double* part, const RhsState* st, int G) {
  const int rhs = blockIdx.y;
  if (st[rhs].done) return;
  const int64_t off = (int64_t)rhs * g.N;
  const double a = st[rhs].alpha;
  double v[3] = {0.0, 0.0, 0.0};
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT) {
    const double u = U[off + i] + a * P[off + i];        // U_s = U_{s-1} + alpha_s P_{s-1}
    const double r = R[off + i] - a * W[off + i];        // R_s = R_{s-1} - alpha_s W_s
    U[off + i] = u;
    R[off + i] = r;
    v[0] += r;
    v[1] += r * r;
    v[2] += u * u;
  }
  const int sl[3] = {S_SUM, S_SQ, S_AUX};
  write_partials<3>(v, sl, part, rhs, G);
}

__global__ __launch_bounds__(VT) void k_fin_res(Geom g, const double* part, RhsState* st,
                                                double* hist, int hist_stride, int G, double tol,
                                                int flags) {
  const int rhs = blockIdx.x;
  if (st[rhs].done) return;
  double v[3];
  const int sl[3] = {S_SUM, S_SQ, S_AUX};
  read_partials<3>(part, rhs, sl, G, v);
  if (threadIdx.x != 0) return;
  RhsState& s = st[rhs];
  s.rsum = v[0];
  s.rr = v[1];
  s.uu = v[2];
  s.iter += 1;
  s.rel_res = sqrt(v[1] / s.h2);
  if (hist) hist[(int64_t)rhs * hist_stride + s.iter] = s.rel_res;
  if (!isfinite(s.rel_res)) { s.done = NONFINITE; return; }
  if ((flags & F_RESIDUAL_ONLY) && s.rel_res <= tol) { s.done = CONVERGED; return; }
  set_scale(s, v[1], (double)g.N);
}

// --------------------------------------------------------------- finish ----
// True residual ||(eta - mean) - L U||^2 and sum U (no early exit).
__global__ __launch_bounds__(VT) void k_true_res(Geom g, const double* __restrict__ eta,
                                                 const double* __restrict__ U, double* part,
                                                 const RhsState* st, int G) {
  const int rhs = blockIdx.y;
  const int64_t off = (int64_t)rhs * g.N;
  const double m = st[rhs].mean;
  double v[2] = {0.0, 0.0};
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT) {
    const double r = (eta[off + i] - m) - minus_laplacian_at(g, U + off, i);
    v[0] += r * r;
    v[1] += U[off + i];
  }
  const int sl[2] = {S_SQ, S_SUM};
  write_partials<2>(v, sl, part, rhs, G);
}

__global__ __launch_bounds__(VT) void k_fin_true(Geom g, const double* part, RhsState* st, int G) {
  const int rhs = blockIdx.x;
  double v[2];
  const int sl[2] = {S_SQ, S_SUM};
  read_partials<2>(part, rhs, sl, G, v);
  if (threadIdx.x != 0) return;
  RhsState& s = st[rhs];
  s.true_rel_res = s.h2 > 0.0 ? sqrt(v[0] / s.h2) : 0.0;
  s.umean = g.singular ? v[1] / (double)g.N : 0.0;
}

__global__ __launch_bounds__(VT) void k_center_u(Geom g, double* __restrict__ U, const RhsState* st,
                                                 int G) {
  const int rhs = blockIdx.y;
  const int64_t off = (int64_t)rhs * g.N;
  const double m = st[rhs].umean;
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT) U[off + i] -= m;
}

// ------------------------------------------------------------------ host ----
int vec_blocks(int64_t N, int batch) {
  // Depends on N only, so that a right-hand side reduces in the same order
  // alone and inside any batch (batch invariance of every result).
  (void)batch;
  int64_t g = (N + VT * 4 - 1) / (VT * 4);
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (int)g;
}

void launch_init(const Geom& g, const double* eta, double* R, double* U, double* part,
                 RhsState* st, double* hist, int hist_stride, int batch, int G, hipStream_t s) {
  dim3 grid(G, batch);
  trace_begin(KC_INIT, s);
  hipLaunchKernelGGL(k_eta_sum, grid, dim3(VT), 0, s, g, eta, part, G);
  trace_end(KC_INIT, s);
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_mean, dim3(batch), dim3(VT), 0, s, g, part, st, G);
  trace_end(KC_FINALIZE, s);
  trace_begin(KC_INIT, s);
  hipLaunchKernelGGL(k_eta_center, grid, dim3(VT), 0, s, g, eta, R, U, part, st, G);
  trace_end(KC_INIT, s);
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_h, dim3(batch), dim3(VT), 0, s, g, part, st, hist, hist_stride, G);
  trace_end(KC_FINALIZE, s);
}

void launch_after_pinv(const Geom& g, const double* R, const double* Z, const double* W,
                       double* P, double* part, RhsState* st, int batch, int G, int first,
                       double tol, int flags, hipStream_t s) {
  dim3 grid(G, batch);
  trace_begin(KC_DOT_RZ, s);
  hipLaunchKernelGGL(k_dot_rz, grid, dim3(VT), 0, s, g, R, Z, (flags & F_FLEX_BETA) ? W : nullptr,
                     part, st, G);
  trace_end(KC_DOT_RZ, s);
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_rho, dim3(batch), dim3(VT), 0, s, g, part, st, G, first, tol, flags);
  trace_end(KC_FINALIZE, s);
  trace_begin(KC_UPDATE_P, s);
  hipLaunchKernelGGL(k_update_p, grid, dim3(VT), 0, s, g, Z, P, st, G, first);
  trace_end(KC_UPDATE_P, s);
}

void launch_iter_head(const Geom& g, double* P, double* W, double* R, double* U, double* part,
                      RhsState* st, double* hist, int hist_stride, int batch, int G, double tol,
                      int flags, hipStream_t s) {
  dim3 grid(G, batch);
  trace_begin(KC_STENCIL, s);
  hipLaunchKernelGGL(k_stencil_dot, grid, dim3(VT), 0, s, g, P, W, part, st, G);
  trace_end(KC_STENCIL, s);
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_alpha, dim3(batch), dim3(VT), 0, s, g, part, st, G);
  trace_end(KC_FINALIZE, s);
  trace_begin(KC_UPDATE_UR, s);
  hipLaunchKernelGGL(k_update_ur, grid, dim3(VT), 0, s, g, P, W, R, U, part, st, G);
  trace_end(KC_UPDATE_UR, s);
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_res, dim3(batch), dim3(VT), 0, s, g, part, st, hist, hist_stride, G,
                     tol, flags);
  trace_end(KC_FINALIZE, s);
}

void launch_finish(const Geom& g, const double* eta, double* U, double* part, RhsState* st,
                   int batch, int G, hipStream_t s) {
  dim3 grid(G, batch);
  trace_begin(KC_FINISH, s);
  hipLaunchKernelGGL(k_true_res, grid, dim3(VT), 0, s, g, eta, U, part, st, G);
  hipLaunchKernelGGL(k_fin_true, dim3(batch), dim3(VT), 0, s, g, part, st, G);
  if (g.singular) hipLaunchKernelGGL(k_center_u, grid, dim3(VT), 0, s, g, U, st, G);
  trace_end(KC_FINISH, s);
}

void launch_laplacian(const Geom& g, const double* P, double* W, int batch, int G, hipStream_t s) {
  trace_begin(KC_STENCIL, s);
  hipLaunchKernelGGL(k_stencil_dot, dim3(G, batch), dim3(VT), 0, s, g, P, W, (double*)nullptr,
                     (const RhsState*)nullptr, G);
  trace_end(KC_STENCIL, s);
}

}  // namespace kp
