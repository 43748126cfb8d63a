// FP64 vector kernels of Algorithm 1 (Sec. 4.1): the sparse minus Laplacian
// of eq. (3.2), the saxpy-type updates and inner products of Sec. 4.2, the
// centering of eq. (3.6) / Remark 4.1, and the per-RHS scalar recurrences.
//
// Every streaming kernel runs on a (G, batch) grid of 256-thread blocks with a
// grid-stride loop over one right-hand side; block partial sums go to `part`
// and a one-block-per-RHS "finalize" kernel reduces them in a fixed order, so
// results are bitwise reproducible run to run (no floating-point atomics).
#include <math.h>

#include <algorithm>

#include "kp_common.h"
#include "kp_internal.h"

namespace kp {

typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int VT = 256;

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

template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], const int (&slots)[NV],
                                               double* part, int rhs, int bid) {
  __shared__ double lds[4 * NV];
  block_sum<NV>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) slot_ptr(part, rhs, slots[q])[bid] = v[q];
  }
}

// Reduces the G <= GMAX block partials of each slot in a fixed order: thread t
// adds partials t, t + VT, t + 2 VT, ... in rounds of four loads issued
// together, then the block reduction of block_sum.
template <int NV>
__device__ __forceinline__ void read_partials(const double* part, int rhs, const int (&slots)[NV],
                                              int G, double (&v)[NV]) {
  __shared__ double lds[4 * NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double* src = part + ((int64_t)rhs * NSLOTS + slots[q]) * GMAX;
    double t = 0.0;
    for (int b0 = 0; b0 < G; b0 += 4 * VT) {
      double x[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int b = b0 + threadIdx.x + w * VT;
        x[w] = b < G ? src[b] : 0.0;
      }
      t += ((x[0] + x[1]) + x[2]) + x[3];
    }
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
// slots: a continuous batch, where only JOINING right-hand sides start (the
// others are left as they are); otherwise every right-hand side starts.
// With N even and the arrays 16-byte aligned (every right-hand side's slice
// then is as well), a lane reads pairs, ET pairs in flight (all issued before any is used, with
// clamped indices), block b sweeping chunks of ET * VT pairs from ET * VT * b
// with stride ET * VT * G.  The split depends on N only.
constexpr int ET = 4;

__global__ __launch_bounds__(VT) void k_eta_sum(Geom g, const double* __restrict__ eta,
                                                double* part, int G, const RhsState* st,
                                                int slots) {
  const int rhs = blockIdx.y;
  if (slots && st[rhs].done != JOINING) return;
  const double* e = eta + (int64_t)rhs * g.N;
  double v[1] = {0.0};
  if ((g.N & 1) == 0 && ((uintptr_t)e & 15) == 0) {
    const d2* e2 = reinterpret_cast<const d2*>(e);
    const uint32_t n2 = (uint32_t)(g.N >> 1);
    for (uint32_t i0 = blockIdx.x * ET * VT + threadIdx.x; i0 < n2; i0 += G * ET * VT) {
      d2 x[ET];
#pragma unroll
      for (int u = 0; u < ET; ++u) x[u] = e2[min(i0 + u * VT, n2 - 1)];
#pragma unroll
      for (int u = 0; u < ET; ++u)
        if (i0 + u * VT < n2) v[0] += x[u].x + x[u].y;
    }
  } else {
#pragma unroll 4
    for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT) v[0] += e[i];
  }
  const int sl[1] = {S_SUM};
  write_partials<1>(v, sl, part, rhs, blockIdx.x);
}

__global__ __launch_bounds__(VT) void k_fin_mean(Geom g, const double* part, RhsState* st, int G,
                                                 int slots) {
  const int rhs = blockIdx.x;
  if (slots && st[rhs].done != JOINING) return;
  double v[1] = {0.0};
  const int sl[1] = {S_SUM};
  if (g.singular) read_partials<1>(part, rhs, sl, G, v);   // no mean to remove otherwise
  if (threadIdx.x == 0) {
    RhsState s = {};
    s.mean = g.singular ? v[0] / (double)g.N : 0.0;
    s.scale = s.inv_scale = 1.0;
    s.diag_iter = -1;
    st[rhs] = s;
  }
}

// A right-hand side that started in this launch sequence (state reset, no
// preconditioner application yet).
__device__ __forceinline__ bool fresh(const RhsState& s) {
  return s.done == RUNNING && s.pinv_count == 0 && s.iter == 0;
}

__global__ __launch_bounds__(VT) void k_eta_center(Geom g, const double* __restrict__ eta,
                                                   double* __restrict__ R, double* __restrict__ U,
                                                   double* part, const RhsState* st, int G,
                                                   int slots) {
  const int rhs = blockIdx.y;
  if (slots && !fresh(st[rhs])) return;
  const int64_t off = (int64_t)rhs * g.N;
  const double m = st[rhs].mean;
  double v[2] = {0.0, 0.0};
  if ((g.N & 1) == 0 && (((uintptr_t)(eta + off) | (uintptr_t)(R ? R + off : nullptr) |
                          (uintptr_t)(U ? U + off : nullptr)) & 15) == 0) {
    const d2* e2 = reinterpret_cast<const d2*>(eta + off);
    d2* R2 = R ? reinterpret_cast<d2*>(R + off) : nullptr;
    d2* U2 = U ? reinterpret_cast<d2*>(U + off) : nullptr;
    const uint32_t n2 = (uint32_t)(g.N >> 1);
    for (uint32_t i0 = blockIdx.x * ET * VT + threadIdx.x; i0 < n2; i0 += G * ET * VT) {
      d2 x[ET];
#pragma unroll
      for (int u = 0; u < ET; ++u) x[u] = e2[min(i0 + u * VT, n2 - 1)];
#pragma unroll
      for (int u = 0; u < ET; ++u) {
        const uint32_t i = i0 + u * VT;
        if (i >= n2) continue;
        const d2 r = {x[u].x - m, x[u].y - m};   // eq. (3.6); m = 0 if nonsingular
        if (R2) R2[i] = r;                     // (a nonsingular set reads eta as R_0)
        if (U2) U2[i] = (d2){0.0, 0.0};        // U_0 = 0 (stored only when read before
                                               // the first iteration writes U)
        v[0] += r.x + r.y;
        v[1] += r.x * r.x + r.y * r.y;
      }
    }
  } else {
#pragma unroll 4
    for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT) {
      const double r = eta[off + i] - m;
      if (R) R[off + i] = r;
      if (U) U[off + i] = 0.0;
      v[0] += r;
      v[1] += r * r;
    }
  }
  const int sl[2] = {S_SUM, S_SQ};
  write_partials<2>(v, sl, part, rhs, blockIdx.x);
}

__global__ __launch_bounds__(VT) void k_fin_h(Geom g, const double* part, RhsState* st,
                                              double* hist, int hist_stride, int G, int slots) {
  const int rhs = blockIdx.x;
  if (slots && !fresh(st[rhs])) return;
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
#pragma unroll 4
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT) {
    const double z = Z[off + i];
    v[0] += R[off + i] * z;
    v[1] += z;
    v[2] += z * z;
    if (W) v[3] += W[off + i] * z;
  }
  const int sl[4] = {S_DOT, S_SUM, S_SQ, S_AUX2};
  write_partials<4>(v, sl, part, rhs, blockIdx.x);
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
  // the first application of this right-hand side's solve (in a continuous
  // batch it may come while other right-hand sides iterate)
  first = first || s.pinv_count == 0;
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
  if (!(flags & (F_RESIDUAL_ONLY | F_ANORM_STOP)) && s.rel_res <= tol && s.err_est <= tol) {
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
  if (first || st[rhs].iter == 0) {   // P_0 = Z_0 (a right-hand side that just started)
  #pragma unroll 4
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT)
      P[off + i] = Z[off + i] - zm;
  } else {
  #pragma unroll 4
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT)
      P[off + i] = (Z[off + i] - zm) + b * P[off + i];   // P_s = Z_s + beta_s P_{s-1}
  }
}

// ------------------------------------------------------ marching stencil ----
// Kernels that apply the 7-point (5-point in 2D) minus Laplacian of eq. (3.2).
// A 256-thread block owns a 64 x 16 tile of (x, y) cells and marches over PB
// consecutive z-planes.  Each wave covers the 64 columns of 4 consecutive
// rows: lane l holds the cells of column i0 + l in those rows for the planes
// k-1, k and k+1 in registers, so a plane's centre values are loaded once
// from memory.  The x-neighbours come from the adjacent lanes (DPP moves);
// the two tile-edge columns of the 4 rows are fetched by one load in which
// 8 lanes take part and broadcast with readlane; the y-neighbours of the
// inner rows are the lane's own registers and only the rows above and below
// the strip are loaded.  The centre loads of plane k+2, the halo loads of
// plane k+2 (k+1 in the U/R update) and the other streams of plane k+1 are
// issued before plane k is computed.  Blocks are mapped to work
// XCD-aware: the hardware deals blocks to the 8 XCDs round robin, and block
// b is given work item (b % 8) * share + b / 8, so that each XCD sweeps a
// contiguous range of plane groups and finds the neighbours in its own L2.
// Boundary neighbours are loaded from a valid address and replaced at compute
// time by the ghost rule of eq. (3.1); periodic neighbours are loaded wrapped.
constexpr int STX = 64, RY = 4, STY = RY * (VT / 64);
constexpr int NXCD = 8;

enum ZMode { ZM_PW = 0, ZM_UR, ZM_TRUE, ZM_LAP, ZM_JAC, ZM_DIAG, ZM_RES, ZM_UR1 };

struct ZGrid {
  int ntx, ntiles;    // tiles along x, tiles per plane
  int pb, ngroups;    // planes per block, plane groups
  int nwork, share;   // work items (tiles x groups) and items per XCD
  int nblocks;        // blocks per right-hand side
};

__device__ __forceinline__ double ghost_lo(int bc, double c) {
  return (bc == BC_N || bc == BC_ND) ? c : 0.0;   // Neumann end: ghost = cell
}
__device__ __forceinline__ double ghost_hi(int bc, double c) {
  return (bc == BC_N || bc == BC_DN) ? c : 0.0;
}

// diagonal entry of L_n at position pos (eq. 3.1): the corners alpha, beta
// at the ends, 2 inside and on periodic axes
__device__ __forceinline__ double diag_1d(int pos, int n, int bc) {
  if (pos == 0) return (bc == BC_N || bc == BC_ND) ? 1.0 : 2.0;
  if (pos == n - 1) return (bc == BC_N || bc == BC_DN) ? 1.0 : 2.0;
  return 2.0;
}

// Whole-wave DPP moves of a double: lane i receives lane i - 1 (shr) or
// lane i + 1 (shl); the lane without a source receives 0.  VALU moves, where
// a shuffle would take the LDS crossbar.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double wave_shr1(double v) { return dpp_d<0x138>(v); }   // wave_shr:1
__device__ __forceinline__ double wave_shl1(double v) { return dpp_d<0x130>(v); }   // wave_shl:1

__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// plane index of a z-neighbour: wrapped when periodic, else clamped (the
// value loaded at a wall is replaced by the ghost rule)
__device__ __forceinline__ int zload(int k, int nz, int bcz) {
  if (k < 0) return bcz == BC_P ? nz - 1 : 0;
  if (k >= nz) return bcz == BC_P ? 0 : nz - 1;
  return k;
}

// ZM_PW:   partials <L P, P>, sum L P; W = L P stored when W != nullptr
// ZM_UR:   U += alpha P, R -= alpha L P; partials sum R, ||R||^2, ||U||^2;
//          in a right-hand side's first iteration the previous U is 0 and is
//          not read (unless a warm start supplied it);
//          with eta the previous R is read from eta (R_0 of a nonsingular set)
// ZM_UR1:  ZM_UR for the first iteration from U_0 = 0, which also takes the
//          exit step's sums of U_1 = alpha P: the true residual
//          R_0 - L U_1 (R_0 = eta - mean) from alpha times each loaded P value,
//          i.e. from the very values U receives, in ZM_TRUE's order of
//          operations and summation (S_TSQ, S_TSUM); a right-hand side not at
//          its first iteration, or warm started, is updated as by ZM_UR
// ZM_TRUE: P is U; partials ||(eta - mean) - L U||^2, sum U; a right-hand
//          side that made no iteration has U = 0, which is written to U here
//          (it was never stored) and used in place of what P holds; one whose
//          sums the first U/R update took (true_pre) is skipped
// ZM_LAP:  W = L P only
// ZM_JAC:  one Jacobi(omega) step on L x = R (Sec. 4.3.1): P is x_{j-1}, W
//          receives x_j = x_{j-1} + (R - L x_{j-1}) / (omega d), d the
//          diagonal of L (eq. 4.4: sum of the 1D diagonals, corners of
//          eq. 3.1 at the ends)
// ZM_DIAG: P is the iterate U_s, h = eta - mean; partials ||h - L U||^2,
//          sum U, <U, L U>, <U, h> (the descriptors of Experiment 5.4); runs
//          only for a right-hand side whose iterate s is not yet recorded
// ZM_RES:  P is a caller's start U_0 (warm start), R receives
//          R_0 = (eta - mean) - L U_0; partials sum R, ||R||^2, ||U_0||^2,
//          sum U_0
template <int MODE>
__global__ __launch_bounds__(VT) void k_zm(Geom g, ZGrid zg, const double* __restrict__ P,
                                           double* __restrict__ W, double* __restrict__ R,
                                           double* __restrict__ U, const double* __restrict__ eta,
                                           double* part, const RhsState* st, double omega,
                                           int gate) {
  const int rhs = blockIdx.y;
  if (MODE == ZM_DIAG) {
    if (st[rhs].iter <= st[rhs].diag_iter) return;
  } else if (MODE == ZM_TRUE) {
    // exit step; with `gate`, only right-hand sides whose solve ended and
    // whose exit step has not run
    if (gate && !(terminal(st[rhs].done) && st[rhs].exit_gen == 0)) return;
    if (st[rhs].true_pre) return;
  } else if (MODE != ZM_LAP && st && (st[rhs].done || (MODE != ZM_JAC && MODE != ZM_RES &&
                                                       st[rhs].pinv_count == 0))) {
    // (an iteration needs the right-hand side's first preconditioned
    // residual: a continuous batch starts requests between iterations)
    return;
  }
  const int b = blockIdx.x;
  const int w = (b % NXCD) * zg.share + b / NXCD;   // XCD-aware work item
  const bool wok = w < zg.nwork;
  const int tile = wok ? w % zg.ntiles : 0, grp = wok ? w / zg.ntiles : 0;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int bcx = g.bc[0], bcy = g.bc[1], bcz = g.bc[2];
  const int lane = threadIdx.x & 63;
  const int i0 = (tile % zg.ntx) * STX;
  const int i = i0 + lane;
  const int y0 = (tile / zg.ntx) * STY + (threadIdx.x >> 6) * RY;   // first row of the wave
  const bool run = wok && y0 < ny;                                   // wave-uniform
  const bool col_ok = i < nx;
  const int ic = col_ok ? i : nx - 1;
  // tile-edge columns: left neighbour of lane 0, right neighbour of lane e
  const int ie = min(i0 + STX - 1, nx - 1), e = ie - i0;
  const int xl = i0 > 0 ? i0 - 1 : (bcx == BC_P ? nx - 1 : 0);
  const int xr = ie < nx - 1 ? ie + 1 : (bcx == BC_P ? 0 : ie);
  const bool lwall = i0 == 0 && bcx != BC_P, rwall = ie == nx - 1 && bcx != BC_P;
  // rows of the strip and the halo rows above and below it
  const int re = min(y0 + RY - 1, ny - 1) - y0;          // last valid row offset
  const int yl = y0 > 0 ? y0 - 1 : (bcy == BC_P ? ny - 1 : 0);
  const int yh = y0 + re < ny - 1 ? y0 + re + 1 : (bcy == BC_P ? 0 : y0 + re);
  const bool bwall = y0 == 0 && bcy != BC_P, twall = y0 + re == ny - 1 && bcy != BC_P;
  const bool three = g.dim == 3;
  const uint32_t plane = (uint32_t)nx * ny;
  const int64_t off = (int64_t)rhs * g.N;
  // U_0 = 0 is never stored: a right-hand side that made no iteration takes
  // its stencil loads from eta (discarded) and writes U = 0 instead, so that
  // no cell is both read through P and written through U
  const bool uz = MODE == ZM_TRUE && st[rhs].iter == 0 && !st[rhs].warm;
  const double* p = (uz ? eta : P) + off;
  constexpr bool UR = MODE == ZM_UR || MODE == ZM_UR1;
  const double alpha = UR ? st[rhs].alpha : 0.0;
  // U/R update of a right-hand side's first iteration: U_0 = 0 is not read
  // (unless a warm start supplied it)
  const bool ufirst = UR && st[rhs].iter == 0 && !st[rhs].warm;
  const bool tfirst = MODE == ZM_UR1 && ufirst;   // block-uniform
  const double mean =
      (MODE == ZM_TRUE || MODE == ZM_DIAG || MODE == ZM_RES) ? st[rhs].mean : 0.0;
  const int kb = grp * zg.pb, ke = run ? min(kb + zg.pb, nz) : kb;
  // edge-load lanes: lane r < RY fetches the left edge of row r, lane 32 + r
  // the right edge
  const int er = (lane & 31) < RY ? (lane & 31) : 0;
  const bool eload = (lane & 31) < RY;
  const uint32_t erow = (uint32_t)min(y0 + er, ny - 1) * nx + (lane < 32 ? xl : xr);

  auto centre = [&](int kk, double (&v)[RY]) {
    const uint32_t base = (uint32_t)zload(kk, nz, bcz) * plane + ic;
#pragma unroll
    for (int r = 0; r < RY; ++r) v[r] = p[base + (uint32_t)min(y0 + r, ny - 1) * nx];
  };
  auto halo = [&](int kk, double& lo, double& hi, double& ed) {
    const uint32_t base = (uint32_t)kk * plane;
    lo = p[base + (uint32_t)yl * nx + ic];
    hi = p[base + (uint32_t)yh * nx + ic];
    ed = eload ? p[base + erow] : 0.0;
  };

  // the other streams of a mode (R and U, or eta, or R) at the cells of plane kk
  constexpr bool XS = UR || MODE == ZM_TRUE || MODE == ZM_JAC || MODE == ZM_DIAG ||
                      MODE == ZM_RES;
  auto extra = [&](int kk, double (&a)[RY], double (&b)[RY]) {
    const uint32_t base = (uint32_t)kk * plane;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int64_t idx = off + base + (uint32_t)min(y0 + r, ny - 1) * nx + ic;
      if (UR) {
        a[r] = eta ? eta[idx] : R[idx];   // R_0 = eta (nonsingular) is never stored
        b[r] = ufirst ? 0.0 : U[idx];
      } else if (MODE == ZM_JAC) {
        a[r] = R[idx];
      } else {
        a[r] = eta[idx];
      }
    }
  };

  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0;
  double pv[RY], cv[RY], nv[RY], nn[RY], ea[RY], eb[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) pv[r] = cv[r] = nv[r] = nn[r] = ea[r] = eb[r] = 0.0;
  // halo lookahead in planes: two, except for the U/R update, whose extra
  // streams leave no registers for it at four waves per SIMD
  constexpr int HA = UR ? 1 : 2;
  double hlo = 0.0, hhi = 0.0, hed = 0.0;      // halo of plane k
  double h1lo = 0.0, h1hi = 0.0, h1ed = 0.0;   // halo of plane k + 1 (HA == 2)
  if (kb < ke) {
    if (three) {
      centre(kb - 1, pv);
      centre(kb + 1, nv);
    }
    centre(kb, cv);
    halo(kb, hlo, hhi, hed);
    if (HA == 2 && kb + 1 < ke) halo(kb + 1, h1lo, h1hi, h1ed);
    if (XS) extra(kb, ea, eb);
  }
  for (int k = kb; k < ke; ++k) {
    // issue the loads of later steps: centres and halos two planes ahead,
    // the other streams one plane ahead
    double nlo = 0.0, nhi = 0.0, ned = 0.0;
    double na[RY], nb[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) na[r] = nb[r] = 0.0;
    if (k + 1 < ke) {
      if (three) centre(k + 2, nn);
      if (XS) extra(k + 1, na, nb);
    }
    if (k + HA < ke) halo(k + HA, nlo, nhi, ned);
    const uint32_t pbase = (uint32_t)k * plane;
    // x-neighbours from the adjacent lanes, tile edges from the edge lanes
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const double cc = cv[r];
      const double el = readlane_d(hed, r), eh = readlane_d(hed, 32 + r);
      double vxl = wave_shr1(cc), vxh = wave_shl1(cc);
      if (lane == 0) vxl = lwall ? ghost_lo(bcx, cc) : el;
      if (lane == e) vxh = rwall ? ghost_hi(bcx, cc) : eh;
      double vyl = r > 0 ? cv[r > 0 ? r - 1 : 0] : (bwall ? ghost_lo(bcy, cc) : hlo);
      double vyh = cv[r < RY - 1 ? r + 1 : r];
      if (r >= re) vyh = twall ? ghost_hi(bcy, cc) : hhi;
      double wv = (2.0 * cc - vxl) - vxh;
      wv += (2.0 * cc - vyl) - vyh;
      double vzl = 0.0, vzh = 0.0;
      if (three) {
        vzl = k > 0 || bcz == BC_P ? pv[r] : ghost_lo(bcz, cc);
        vzh = k < nz - 1 || bcz == BC_P ? nv[r] : ghost_hi(bcz, cc);
        wv += (2.0 * cc - vzl) - vzh;
      }
      // L U_1 from the values U_1 = alpha P takes at the cell and its
      // neighbours (ghosts follow: alpha times a ghost is the ghost of U_1);
      // each product is rounded before it is subtracted, as U_1 is stored
      // rounded (no fused multiply-add in this block)
      double wt = 0.0;
      if (MODE == ZM_UR1 && tfirst) {
#pragma clang fp contract(off)
        const double uc = alpha * cc;
        wt = (2.0 * uc - alpha * vxl) - alpha * vxh;
        wt += (2.0 * uc - alpha * vyl) - alpha * vyh;
        if (three) wt += (2.0 * uc - alpha * vzl) - alpha * vzh;
      }
      if (col_ok && r <= re) {
        const int64_t idx = off + pbase + (uint32_t)(y0 + r) * nx + i;
        if (MODE == ZM_PW) {
          a0 += wv * cc;
          a1 += wv;
          if (W) W[idx] = wv;
        } else if (UR) {
          const double u = eb[r] + alpha * cc;    // U_s = U_{s-1} + alpha_s P_{s-1}
          const double rr = ea[r] - alpha * wv;   // R_s = R_{s-1} - alpha_s W_s
          U[idx] = u;
          R[idx] = rr;
          a0 += rr;
          a1 += rr * rr;
          a2 += u * u;
          if (MODE == ZM_UR1 && tfirst) {
            const double rt = ea[r] - wt;         // R_0 - L U_1, as ZM_TRUE forms it
            a3 += rt * rt;
            a4 += u;                              // U_1 = 0 + alpha P, as stored
          }
        } else if (MODE == ZM_TRUE) {
          const double rr = (ea[r] - mean) - (uz ? 0.0 : wv);
          a0 += rr * rr;
          a1 += uz ? 0.0 : cc;
          if (uz) U[idx] = 0.0;
        } else if (MODE == ZM_DIAG) {
          const double h = ea[r] - mean;
          const double rr = h - wv;
          a0 += rr * rr;
          a1 += cc;
          a2 += cc * wv;
          a3 += cc * h;
        } else if (MODE == ZM_RES) {
          const double rr = (ea[r] - mean) - wv;
          R[idx] = rr;
          a0 += rr;
          a1 += rr * rr;
          a2 += cc * cc;
          a3 += cc;
        } else if (MODE == ZM_JAC) {
          const double d = diag_1d(i, nx, bcx) + diag_1d(y0 + r, ny, bcy) +
                           (three ? diag_1d(k, nz, bcz) : 0.0);
          W[idx] = cc + (ea[r] - wv) / (omega * d);
        } else {
          W[idx] = wv;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      pv[r] = cv[r];
      cv[r] = nv[r];
      nv[r] = nn[r];
      ea[r] = na[r];
      eb[r] = nb[r];
    }
    if (HA == 2) {
      hlo = h1lo;
      hhi = h1hi;
      hed = h1ed;
      h1lo = nlo;
      h1hi = nhi;
      h1ed = ned;
    } else {
      hlo = nlo;
      hhi = nhi;
      hed = ned;
    }
  }
  if (MODE == ZM_LAP || MODE == ZM_JAC) return;
  if (MODE == ZM_UR) {
    double v[3] = {a0, a1, a2};
    const int sl[3] = {S_SUM, S_SQ, S_AUX};
    write_partials<3>(v, sl, part, rhs, b);
  } else if (MODE == ZM_UR1) {
    double v[5] = {a0, a1, a2, a3, a4};
    const int sl[5] = {S_SUM, S_SQ, S_AUX, S_TSQ, S_TSUM};
    write_partials<5>(v, sl, part, rhs, b);
  } else if (MODE == ZM_PW) {
    double v[2] = {a0, a1};
    const int sl[2] = {S_DOT, S_SUM};
    write_partials<2>(v, sl, part, rhs, b);
  } else if (MODE == ZM_DIAG) {
    double v[4] = {a0, a1, a2, a3};
    const int sl[4] = {S_SQ, S_SUM, S_DOT, S_AUX};
    write_partials<4>(v, sl, part, rhs, b);
  } else if (MODE == ZM_RES) {
    double v[4] = {a0, a1, a2, a3};
    const int sl[4] = {S_SUM, S_SQ, S_AUX, S_AUX2};
    write_partials<4>(v, sl, part, rhs, b);
  } else {
    double v[2] = {a0, a1};
    const int sl[2] = {S_SQ, S_SUM};
    write_partials<2>(v, sl, part, rhs, b);
  }
}

ZGrid zgrid_for(const Geom& g) {
  ZGrid z;
  z.ntx = (g.nx + STX - 1) / STX;
  z.ntiles = z.ntx * ((g.ny + STY - 1) / STY);
  // planes per block: up to 16, fewer while a right-hand side would have
  // under `least` blocks, more while it would exceed the GMAX partial slots
  // (a function of the grid only, so batched and single solves sum alike).
  // From 4 M unknowns on, 512 blocks fill the chip: longer marches re-read
  // fewer halo planes (the U/R update on 256 x 256 x 128: 58.0 -> 53.7 us);
  // smaller grids keep 1024.
  const int64_t least = g.N >= ((int64_t)1 << 22) ? 512 : 1024;
  z.pb = 16;
  auto blocks = [&](int pb) { return (int64_t)z.ntiles * ((g.nz + pb - 1) / pb); };
  while (z.pb > 1 && blocks(z.pb) < least) z.pb >>= 1;
  while (blocks(z.pb) > GMAX - NXCD && z.pb < g.nz) z.pb <<= 1;
  z.ngroups = (g.nz + z.pb - 1) / z.pb;
  z.nwork = z.ntiles * z.ngroups;
  z.share = (z.nwork + NXCD - 1) / NXCD;
  z.nblocks = z.share * NXCD;
  return z;
}

// The partial sums of one right-hand side fit in GMAX slots.
bool zgrid_fits(const Geom& g) { return zgrid_for(g).nblocks <= GMAX; }

__global__ __launch_bounds__(VT) void k_fin_alpha(Geom g, const double* part, RhsState* st, int G) {
  const int rhs = blockIdx.x;
  if (st[rhs].done || st[rhs].pinv_count == 0) return;   // as the stencil pass
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
  // alpha_s rho_{s-1}: the decrease of ||U - u||_L^2 in this iteration
  // (Hestenes-Stiefel), for the A-norm stopping rule
  const double t = s.alpha * s.rho;
  s.hs_sum += t;
  s.hs_ring[(s.iter + 1) % HS_DELAY] = t;
}

// fused: the update was ZM_UR1, whose exit-step sums hold for a right-hand
// side at its first iteration from U_0 = 0 (any later update voids them).
__global__ __launch_bounds__(VT) void k_fin_res(Geom g, const double* part, RhsState* st,
                                                double* hist, int hist_stride, int G, double tol,
                                                int flags, int fused) {
  const int rhs = blockIdx.x;
  if (st[rhs].done || st[rhs].pinv_count == 0) return;   // as the U/R update
  double v[3];
  const int sl[3] = {S_SUM, S_SQ, S_AUX};
  read_partials<3>(part, rhs, sl, G, v);
  if (threadIdx.x != 0) return;
  RhsState& s = st[rhs];
  s.rsum = v[0];
  s.rr = v[1];
  // ||U_s||^2 of the zero-mean iterate: the updates have zero mean on a
  // singular set, so U_s keeps the mean of a warm start U_0 (removed at exit)
  s.uu = s.warm ? fmax(v[2] - (double)g.N * s.u0mean * s.u0mean, 0.0) : v[2];
  s.true_pre = (fused && s.iter == 0 && !s.warm) ? 1 : 0;
  s.iter += 1;
  s.need_cert = 0;   // a certificate applies to this iterate only
  s.rel_res = sqrt(v[1] / s.h2);
  if (hist) hist[(int64_t)rhs * hist_stride + s.iter] = s.rel_res;
  if (!isfinite(s.rel_res)) { s.done = NONFINITE; return; }
  if (flags & F_ANORM_STOP) {
    // relative L-norm error of U_{s-d}, estimated by the last d terms over
    // all of them (their sum estimates ||u||_L^2 from U_0 = 0)
    if (s.iter >= HS_DELAY && s.hs_sum > 0.0) {
      const double w = (s.hs_ring[0] + s.hs_ring[1]) + (s.hs_ring[2] + s.hs_ring[3]);
      if (sqrt(w / s.hs_sum) <= tol) { s.done = CONVERGED; return; }
    }
  } else if ((flags & F_RESIDUAL_ONLY) && s.rel_res <= tol) {
    s.done = CONVERGED;
    return;
  } else if (!(flags & F_RESIDUAL_ONLY) && s.rel_res <= tol && s.uu > 0.0) {
    // the error U_s - u = -L^+ R_s has norm at most ||R_s|| / lambda_min:
    // when this bound already meets tol, the error estimate ||Z_s|| / ||U_s||
    // and the preconditioner application it needs are skipped; otherwise
    // the sharper low-mode bound is tried next
    const double bound = sqrt(v[1] / s.uu) / g.lam_min;
    if (bound <= tol) {
      s.err_est = bound;
      s.done = CONVERGED;
      return;
    }
    s.need_cert = (flags & F_CERT) ? 1 : 0;
  }
  set_scale(s, v[1], (double)g.N);
}

// Warm start: the residual of the caller's U_0 (ZM_RES partials) becomes
// R_0's sums; the start itself may already meet the stopping rule (s = 0).
__global__ __launch_bounds__(VT) void k_fin_warm(Geom g, const double* part, RhsState* st,
                                                 double* hist, int hist_stride, int G, double tol,
                                                 int flags) {
  const int rhs = blockIdx.x;
  if (st[rhs].done) return;
  double v[4];
  const int sl[4] = {S_SUM, S_SQ, S_AUX, S_AUX2};
  read_partials<4>(part, rhs, sl, G, v);
  if (threadIdx.x != 0) return;
  RhsState& s = st[rhs];
  s.warm = 1;
  s.u0mean = g.singular ? v[3] / (double)g.N : 0.0;
  s.rsum = v[0];
  s.rr = v[1];
  s.uu = fmax(v[2] - (double)g.N * s.u0mean * s.u0mean, 0.0);
  s.rel_res = sqrt(v[1] / s.h2);
  if (hist) hist[(int64_t)rhs * hist_stride] = s.rel_res;
  if (!isfinite(s.rel_res) || !isfinite(v[2])) { s.done = NONFINITE; return; }
  if (!(flags & F_ANORM_STOP) && s.rel_res <= tol) {
    if (flags & F_RESIDUAL_ONLY) { s.done = CONVERGED; return; }
    // the error of U_0 is L^+ R_0, at most ||R_0|| / lambda_min
    const double bound = s.uu > 0.0 ? sqrt(v[1] / s.uu) / g.lam_min : INFINITY;
    if (bound <= tol) {
      s.err_est = bound;
      s.done = CONVERGED;
      return;
    }
  }
  set_scale(s, v[1], (double)g.N);
}

// --------------------------------------------------------------- finish ----
// gate: a continuous batch, where only right-hand sides whose solve ended
// and whose exit step is due are processed (exit_gen 0 -> 1); the host
// mirror is written for every right-hand side either way.
__global__ __launch_bounds__(VT) void k_fin_true(Geom g, const double* part, RhsState* st, int G,
                                                 RhsState* mirror, int gate) {
  const int rhs = blockIdx.x;
  const bool run = !gate || (terminal(st[rhs].done) && st[rhs].exit_gen == 0);
  double v[2] = {0.0, 0.0};
  // the sums of the first U/R update when they hold for U, else ZM_TRUE's
  const bool pre = st[rhs].true_pre;
  const int sl[2] = {pre ? S_TSQ : S_SQ, pre ? S_TSUM : S_SUM};
  if (run) read_partials<2>(part, rhs, sl, G, v);
  if (threadIdx.x != 0) return;
  RhsState& s = st[rhs];
  if (run) {
    s.true_rel_res = s.h2 > 0.0 ? sqrt(v[0] / s.h2) : 0.0;
    s.umean = g.singular ? v[1] / (double)g.N : 0.0;
    if (gate) s.exit_gen = g.singular ? 1 : 2;   // centring of U still due, or done
  }
  if (mirror) mirror[rhs] = s;   // host-mapped copy read after the stream sync
}

// gated exit of a singular set: the centring of U has run (exit_gen 1 -> 2)
__global__ void k_exit_done(RhsState* st, RhsState* mirror, int batch) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= batch || st[rhs].exit_gen != 1) return;
  st[rhs].exit_gen = 2;
  if (mirror) mirror[rhs] = st[rhs];
}

// Empties every slot of a continuous batch, or marks one slot (JOINING: a
// request starts at the next step; CAPPED: stop at the iteration limit).
__global__ void k_slot_set(RhsState* st, int batch, int slot, int code) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= batch) return;
  if (slot < 0) {
    RhsState s = {};
    s.done = IDLE;
    s.exit_gen = 2;
    st[rhs] = s;
  } else if (rhs == slot) {
    st[rhs].done = code;
    if (code == CAPPED) st[rhs].exit_gen = 0;
  }
}

// Z = R for M = I (a kernel rather than a device copy, so that it can sit in
// a captured graph).
__global__ __launch_bounds__(VT) void k_copy(Geom g, const double* __restrict__ src,
                                             double* __restrict__ dst, const RhsState* st, int G) {
  const int rhs = blockIdx.y;
  if (st && st[rhs].done) return;
  const int64_t off = (int64_t)rhs * g.N;
#pragma unroll 4
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT)
    dst[off + i] = src[off + i];
}

__global__ __launch_bounds__(VT) void k_center_u(Geom g, double* __restrict__ U, const RhsState* st,
                                                 int G, int gate) {
  const int rhs = blockIdx.y;
  if (gate && st[rhs].exit_gen != 1) return;
  const int64_t off = (int64_t)rhs * g.N;
  const double m = st[rhs].umean;
#pragma unroll 4
  for (uint32_t i = blockIdx.x * VT + threadIdx.x; i < (uint32_t)g.N; i += G * VT) U[off + i] -= m;
}

// ------------------------------------------------------------------ host ----
int vec_blocks(int64_t N, int batch) {
  // Depends on N only, so that a right-hand side reduces in the same order
  // alone and inside any batch (batch invariance of every result).  At most
  // 4 * VT partials, which the finalize kernels read in one round of loads.
  (void)batch;
  int64_t g = (N + VT * 16 - 1) / (VT * 16);
  if (g > 4 * VT) g = 4 * VT;
  if (g < 1) g = 1;
  return (int)g;
}

void launch_fin_h(const Geom& g, double* part, RhsState* st, double* hist, int hist_stride,
                  int batch, int G, hipStream_t s) {
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_h, dim3(batch), dim3(VT), 0, s, g, (const double*)part, st, hist,
                     hist_stride, G, 0);
  trace_end(KC_FINALIZE, s);
}

void launch_init(const Geom& g, const double* eta, double* R, double* U, double* part,
                 RhsState* st, double* hist, int hist_stride, int batch, int G, hipStream_t s,
                 int slots, bool state_only) {
  dim3 grid(G, batch);
  if (g.singular) {   // the mean of eta (eq. 3.6); a nonsingular set keeps eta as it is
    trace_begin(KC_INIT, s);
    hipLaunchKernelGGL(k_eta_sum, grid, dim3(VT), 0, s, g, eta, part, G, (const RhsState*)st,
                       slots);
    trace_end(KC_INIT, s);
  }
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_mean, dim3(batch), dim3(VT), 0, s, g, part, st, G, slots);
  trace_end(KC_FINALIZE, s);
  if (state_only) return;
  trace_begin(KC_INIT, s);
  hipLaunchKernelGGL(k_eta_center, grid, dim3(VT), 0, s, g, eta, R, U, part, (const RhsState*)st,
                     G, slots);
  trace_end(KC_INIT, s);
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_h, dim3(batch), dim3(VT), 0, s, g, part, st, hist, hist_stride, G,
                     slots);
  trace_end(KC_FINALIZE, s);
}

void launch_warm(const Geom& g, const double* eta, const double* U, double* R, double* part,
                 RhsState* st, double* hist, int hist_stride, int batch, double tol, int flags,
                 hipStream_t s) {
  const ZGrid z = zgrid_for(g);
  trace_begin(KC_INIT, s);
  hipLaunchKernelGGL(k_zm<ZM_RES>, dim3(z.nblocks, batch), dim3(VT), 0, s, g, z, U,
                     (double*)nullptr, R, (double*)nullptr, eta, part, (const RhsState*)st, 0.0,
                     0);
  trace_end(KC_INIT, s);
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_warm, dim3(batch), dim3(VT), 0, s, g, part, st, hist, hist_stride,
                     z.nblocks, tol, flags);
  trace_end(KC_FINALIZE, s);
}

void launch_after_pinv(const Geom& g, const double* R, const double* Z, const double* W,
                       double* P, double* part, RhsState* st, int batch, int G, int first,
                       double tol, int flags, hipStream_t s, int Gdot, bool p_written) {
  dim3 grid(G, batch);
  if (Gdot == 0) {
    trace_begin(KC_DOT_RZ, s);
    hipLaunchKernelGGL(k_dot_rz, grid, dim3(VT), 0, s, g, R, Z,
                       (flags & F_FLEX_BETA) ? W : nullptr, part, st, G);
    trace_end(KC_DOT_RZ, s);
  }
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_rho, dim3(batch), dim3(VT), 0, s, g, part, st, Gdot ? Gdot : G, first,
                     tol, flags);
  trace_end(KC_FINALIZE, s);
  if (p_written) return;
  trace_begin(KC_UPDATE_P, s);
  hipLaunchKernelGGL(k_update_p, grid, dim3(VT), 0, s, g, Z, P, st, G, first);
  trace_end(KC_UPDATE_P, s);
}

void launch_iter_head(const Geom& g, double* P, double* W, double* R, double* U, double* part,
                      RhsState* st, double* hist, int hist_stride, int batch, int G, double tol,
                      int flags, hipStream_t s, const double* r0, bool first) {
  const ZGrid z = zgrid_for(g);
  const int Gz = z.nblocks;
  dim3 zgrid(z.nblocks, batch);
  // W is only needed by the flexible beta (<W, Z>)
  trace_begin(KC_STENCIL, s);
  hipLaunchKernelGGL(k_zm<ZM_PW>, zgrid, dim3(VT), 0, s, g, z, (const double*)P,
                     (flags & F_FLEX_BETA) ? W : (double*)nullptr, (double*)nullptr,
                     (double*)nullptr, (const double*)nullptr, part, (const RhsState*)st, 0.0, 0);
  trace_end(KC_STENCIL, s);
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_alpha, dim3(batch), dim3(VT), 0, s, g, part, st, Gz);
  trace_end(KC_FINALIZE, s);
  // a solve's first iteration from U_0 = 0 also takes the exit step's sums
  trace_begin(KC_UPDATE_UR, s);
  if (first)
    hipLaunchKernelGGL(k_zm<ZM_UR1>, zgrid, dim3(VT), 0, s, g, z, (const double*)P,
                       (double*)nullptr, R, U, r0, part, (const RhsState*)st, 0.0, 0);
  else
    hipLaunchKernelGGL(k_zm<ZM_UR>, zgrid, dim3(VT), 0, s, g, z, (const double*)P,
                       (double*)nullptr, R, U, r0, part, (const RhsState*)st, 0.0, 0);
  trace_end(KC_UPDATE_UR, s);
  trace_begin(KC_FINALIZE, s);
  hipLaunchKernelGGL(k_fin_res, dim3(batch), dim3(VT), 0, s, g, part, st, hist, hist_stride, Gz,
                     tol, flags, first ? 1 : 0);
  trace_end(KC_FINALIZE, s);
  (void)G;
}

void launch_finish(const Geom& g, const double* eta, double* U, double* part, RhsState* st,
                   RhsState* mirror, int batch, int G, hipStream_t s, int gate) {
  const ZGrid z = zgrid_for(g);
  const int Gz = z.nblocks;
  trace_begin(KC_FINISH, s);
  hipLaunchKernelGGL(k_zm<ZM_TRUE>, dim3(z.nblocks, batch), dim3(VT), 0, s, g, z,
                     (const double*)U, (double*)nullptr, (double*)nullptr, U, eta, part,
                     (const RhsState*)st, 0.0, gate);
  hipLaunchKernelGGL(k_fin_true, dim3(batch), dim3(VT), 0, s, g, part, st, Gz, mirror, gate);
  if (g.singular) {
    hipLaunchKernelGGL(k_center_u, dim3(G, batch), dim3(VT), 0, s, g, U, (const RhsState*)st, G,
                       gate);
    if (gate)
      hipLaunchKernelGGL(k_exit_done, dim3((batch + 63) / 64), dim3(64), 0, s, st, mirror, batch);
  }
  trace_end(KC_FINISH, s);
}

void launch_slot_set(RhsState* st, int batch, int slot, int code, hipStream_t s) {
  hipLaunchKernelGGL(k_slot_set, dim3((batch + 63) / 64), dim3(64), 0, s, st, batch, slot, code);
}

void launch_copy(const Geom& g, const double* src, double* dst, const RhsState* st, int batch,
                 int G, hipStream_t s) {
  trace_begin(KC_COPY, s);
  hipLaunchKernelGGL(k_copy, dim3(G, batch), dim3(VT), 0, s, g, src, dst, st, G);
  trace_end(KC_COPY, s);
}

void launch_laplacian(const Geom& g, const double* P, double* W, int batch, int G, hipStream_t s) {
  const ZGrid z = zgrid_for(g);
  (void)G;
  trace_begin(KC_STENCIL, s);
  hipLaunchKernelGGL(k_zm<ZM_LAP>, dim3(z.nblocks, batch), dim3(VT), 0, s, g, z, P, W,
                     (double*)nullptr, (double*)nullptr, (const double*)nullptr, (double*)nullptr,
                     (const RhsState*)nullptr, 0.0, 0);
  trace_end(KC_STENCIL, s);
}



// First Jacobi step from x_0 = 0: x_1 = R / (omega d).
__global__ __launch_bounds__(VT) void k_jac_first(Geom g, const double* __restrict__ R,
                                                  double* __restrict__ X, double omega,
                                                  const RhsState* st, int G) {
  const int rhs = blockIdx.y;
  if (st && st[rhs].done) return;
  const int64_t off = (int64_t)rhs * g.N;
  const int nx = g.nx, ny = g.ny;
  for (uint32_t idx = blockIdx.x * VT + threadIdx.x; idx < (uint32_t)g.N; idx += G * VT) {
    const int i = idx % nx, j = (idx / nx) % ny, k = idx / ((uint32_t)nx * ny);
    const double d = diag_1d(i, nx, g.bc[0]) + diag_1d(j, ny, g.bc[1]) +
                     (g.dim == 3 ? diag_1d(k, g.nz, g.bc[2]) : 0.0);
    X[off + idx] = R[off + idx] / (omega * d);
  }
}

// Jacobi(p, omega) preconditioner (Algs. 2-3): p steps from x_0 = 0,
// alternating between Z and J so that x_p lands in Z.
void launch_jacobi(const Geom& g, const double* R, double* Z, double* J, int p, double omega,
                   const RhsState* st, int batch, int G, hipStream_t s) {
  double* buf[2] = {Z, J};
  const ZGrid z = zgrid_for(g);
  trace_begin(KC_JACOBI, s);
  hipLaunchKernelGGL(k_jac_first, dim3(G, batch), dim3(VT), 0, s, g, R, buf[(p - 1) % 2], omega,
                     st, G);
  for (int j = 2; j <= p; ++j)
    hipLaunchKernelGGL(k_zm<ZM_JAC>, dim3(z.nblocks, batch), dim3(VT), 0, s, g, z,
                       (const double*)buf[(p - j + 1) % 2], buf[(p - j) % 2], (double*)R,
                       (double*)nullptr, (const double*)nullptr, (double*)nullptr, st, omega, 0);
  trace_end(KC_JACOBI, s);
}

// ------------------------------------------------ boundary data and field ----
// Non-homogeneous boundary data (Sec. 3.4.2): a prescribed value on one face
// is added to every cell next to that face.  One launch per face, in stream
// order, so cells on an edge or corner sum their faces deterministically.
// faces: [rhs][axis][end] doubles.
__global__ __launch_bounds__(VT) void k_face_add(Geom g, double* __restrict__ h,
                                                 const double* __restrict__ faces, int axis,
                                                 int end) {
  const int rhs = blockIdx.y;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int na = axis == 0 ? nx : (axis == 1 ? ny : nz);
  const int fixed = end ? na - 1 : 0;
  const uint32_t cells = (uint32_t)(g.N / na);
  const double v = faces[((int64_t)rhs * g.dim + axis) * 2 + end];
  double* hr = h + (int64_t)rhs * g.N;
  for (uint32_t c = blockIdx.x * VT + threadIdx.x; c < cells; c += gridDim.x * VT) {
    int i, j, k;
    if (axis == 0) { i = fixed; j = c % ny; k = c / ny; }
    else if (axis == 1) { i = c % nx; j = fixed; k = c / nx; }
    else { i = c % nx; j = c / nx; k = fixed; }
    hr[i + (int64_t)nx * (j + (int64_t)ny * k)] += v;
  }
}

// eps = -grad u (Sec. 1) by central differences at the grid points; the
// neighbour outside the grid follows the ghost rule of the axis end:
// periodic wrap, the prescribed potential at a Dirichlet end, the boundary
// cell plus the prescribed outward derivative at a Neumann end (faces may be
// null: homogeneous data).  eps: [rhs][component][grid].
__global__ __launch_bounds__(VT) void k_field(Geom g, const double* __restrict__ u,
                                              double* __restrict__ eps,
                                              const double* __restrict__ faces) {
  const int rhs = blockIdx.y;
  const int nx = g.nx, ny = g.ny;
  const double* ur = u + (int64_t)rhs * g.N;
  for (uint32_t idx = blockIdx.x * VT + threadIdx.x; idx < (uint32_t)g.N;
       idx += gridDim.x * VT) {
    const int i = idx % nx, j = (idx / nx) % ny, k = idx / ((uint32_t)nx * ny);
    const double c = ur[idx];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a >= g.dim) break;
      const int pos = a == 0 ? i : (a == 1 ? j : k);
      const int n = a == 0 ? nx : (a == 1 ? ny : g.nz);
      const uint32_t stride = a == 0 ? 1u : (a == 1 ? (uint32_t)nx : (uint32_t)nx * ny);
      const int bc = g.bc[a];
      const double f0 = faces ? faces[((int64_t)rhs * g.dim + a) * 2 + 0] : 0.0;
      const double f1 = faces ? faces[((int64_t)rhs * g.dim + a) * 2 + 1] : 0.0;
      double lo, hi;
      if (pos > 0) lo = ur[idx - stride];
      else if (bc == BC_P) lo = ur[idx + (uint32_t)(n - 1) * stride];
      else if (bc == BC_D || bc == BC_DN) lo = f0;     // Dirichlet node at the beginning
      else lo = c + f0;                                // Neumann ghost at the beginning
      if (pos < n - 1) hi = ur[idx + stride];
      else if (bc == BC_P) hi = ur[idx - (uint32_t)(n - 1) * stride];
      else if (bc == BC_D || bc == BC_ND) hi = f1;     // Dirichlet node at the end
      else hi = c + f1;                                // Neumann ghost at the end
      eps[((int64_t)rhs * g.dim + a) * g.N + idx] = -(hi - lo) * 0.5;
    }
  }
}

void launch_face_updates(const Geom& g, double* h, const double* faces, int batch,
                         hipStream_t s) {
  for (int a = 0; a < g.dim; ++a) {
    if (g.bc[a] == BC_P) continue;
    const int na = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
    const int64_t cells = g.N / na;
    const int G = (int)std::min<int64_t>((cells + VT - 1) / VT, 1024);
    for (int end = 0; end < 2; ++end)
      hipLaunchKernelGGL(k_face_add, dim3(G, batch), dim3(VT), 0, s, g, h, faces, a, end);
  }
}

void launch_field(const Geom& g, const double* u, double* eps, const double* faces, int batch,
                  hipStream_t s) {
  const int G = (int)std::min<int64_t>((g.N + VT - 1) / VT, 4096);
  hipLaunchKernelGGL(k_field, dim3(G, batch), dim3(VT), 0, s, g, u, eps, faces);
}

// ---------------------------------------------------------- diagnostics ----
// Descriptors of iterate U_s (Experiment 5.4) into row s of the table:
// true relative residual, kappa_s = <U, L U> - 2 <U, h>, null-space
// component |sum U| / sqrt(N) (singular operators; 0 otherwise) and the
// Hestenes-Stiefel term alpha_s rho_{s-1} (0 at s = 0).
__global__ __launch_bounds__(VT) void k_fin_diag(Geom g, const double* part, RhsState* st,
                                                 double* diag, int stride, int G) {
  const int rhs = blockIdx.x;
  if (st[rhs].iter <= st[rhs].diag_iter) return;
  double v[4];
  const int sl[4] = {S_SQ, S_SUM, S_DOT, S_AUX};
  read_partials<4>(part, rhs, sl, G, v);
  if (threadIdx.x != 0) return;
  RhsState& s = st[rhs];
  double* row = diag + ((int64_t)rhs * stride + s.iter) * DIAG_RAW;
  row[0] = s.h2 > 0.0 ? sqrt(v[0] / s.h2) : 0.0;
  row[1] = v[2] - 2.0 * v[3];
  row[2] = g.singular ? fabs(v[1]) / sqrt((double)g.N) : 0.0;
  row[3] = s.iter > 0 ? s.alpha * s.rho : 0.0;
  s.diag_iter = s.iter;
}

void launch_diag(const Geom& g, const double* eta, const double* U, double* part, RhsState* st,
                 double* diag, int stride, int batch, hipStream_t s) {
  const ZGrid z = zgrid_for(g);
  trace_begin(KC_DIAG, s);
  hipLaunchKernelGGL(k_zm<ZM_DIAG>, dim3(z.nblocks, batch), dim3(VT), 0, s, g, z, U,
                     (double*)nullptr, (double*)nullptr, (double*)nullptr, eta, part,
                     (const RhsState*)st, 0.0, 0);
  hipLaunchKernelGGL(k_fin_diag, dim3(batch), dim3(VT), 0, s, g, part, st, diag, stride,
                     z.nblocks);
  trace_end(KC_DIAG, s);
}

// ---------------------------------------------------------- certificate ----
// D(r, c) = sum_k A(r, k) B(k, c) per plane p and right-hand side, with
// arbitrary strides, in FP64 on the matrix cores.  A block owns one 16 x 32
// tile of D (two 16 x 16 fragments); its four waves take interleaved blocks
// of 16 k each and their partial tiles are added in a fixed order in LDS.
// Operand layout of v_mfma_f64_16x16x4f64: lane l supplies A(l % 16, k) and
// B(k, l % 16) for the k of its group l / 16; result element v of lane l is
// D(4 v + l / 16, l % 16).  Within a block of 16 k, group g takes
// k = 4 g + step.
// With w set, the tile is not stored: its sums sum d^2 w[i] and sum d^2
// (i the element's index in D) go to part[rhs][tile][2] instead.
// VA: A is contiguous in k (a_k = 1, K a multiple of 16, 16-byte aligned
// rows), so a lane's four consecutive k come as two 16-byte loads.
struct SmallGemm {
  const double* A; int64_t a_r, a_k, a_p, a_rhs;
  const double* B; int64_t b_k, b_c, b_p, b_rhs;
  double* D; int64_t d_r, d_c, d_p, d_rhs;
  int rows, cols, K, planes;
  const double* w; double* part;
};

template <bool VA>
__global__ __launch_bounds__(VT) void k_cert_gemm(SmallGemm q, const RhsState* st) {
  const int rhs = blockIdx.y;
  if (!st[rhs].need_cert) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rtn = (q.rows + 15) / 16, ctn = (q.cols + 31) / 32;
  const int tile = blockIdx.x;                       // < rtn * ctn * planes
  const int p = tile / (rtn * ctn), rem = tile % (rtn * ctn);
  const int rt = rem % rtn, ct = rem / rtn;
  const int l16 = lane & 15, grp = lane >> 4;
  const int r = rt * 16 + l16;
  const bool rok = r < q.rows;
  const double* A = q.A + rhs * q.a_rhs + p * q.a_p + (int64_t)(rok ? r : 0) * q.a_r;
  const double* B = q.B + rhs * q.b_rhs + p * q.b_p;
  const int c0 = ct * 32 + l16, c1 = c0 + 16;
  const bool c0ok = c0 < q.cols, c1ok = c1 < q.cols;
  const double* B0 = B + (int64_t)(c0ok ? c0 : 0) * q.b_c;
  const double* B1 = B + (int64_t)(c1ok ? c1 : 0) * q.b_c;
  d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  const int nkb = (q.K + 15) / 16;
  for (int kb = wave; kb < nkb; kb += VT / 64) {
    // every load of the k-block first, then its eight MFMAs
    double a[4], b0[4], b1[4];
    if constexpr (VA) {
      const d2 lo = *reinterpret_cast<const d2*>(A + kb * 16 + 4 * grp);
      const d2 hi = *reinterpret_cast<const d2*>(A + kb * 16 + 4 * grp + 2);
      a[0] = rok ? lo.x : 0.0;
      a[1] = rok ? lo.y : 0.0;
      a[2] = rok ? hi.x : 0.0;
      a[3] = rok ? hi.y : 0.0;
    }
#pragma unroll
    for (int st4 = 0; st4 < 4; ++st4) {
      const int k = kb * 16 + 4 * grp + st4;
      const bool kok = k < q.K;
      const int kc = kok ? k : 0;
      if constexpr (!VA) a[st4] = A[(int64_t)kc * q.a_k];
      b0[st4] = B0[(int64_t)kc * q.b_k];
      b1[st4] = B1[(int64_t)kc * q.b_k];
      if constexpr (!VA) a[st4] = (rok && kok) ? a[st4] : 0.0;
      b0[st4] = (c0ok && kok) ? b0[st4] : 0.0;
      b1[st4] = (c1ok && kok) ? b1[st4] : 0.0;
    }
#pragma unroll
    for (int st4 = 0; st4 < 4; ++st4) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st4], b0[st4], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st4], b1[st4], acc1, 0, 0, 0);
    }
  }
  // waves 1..3 hand their tiles to wave 0, which adds them in order
  __shared__ double red[3][8][64];
  if (wave > 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      red[wave - 1][v][lane] = acc0[v];
      red[wave - 1][4 + v][lane] = acc1[v];
    }
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      acc0[v] += red[w][v][lane];
      acc1[v] += red[w][4 + v][lane];
    }
  if (q.w) {
    double t[2] = {0.0, 0.0};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rt * 16 + 4 * v + grp;
      if (row >= q.rows) continue;
      if (c0ok) {
        const double x2 = acc0[v] * acc0[v];
        t[0] += x2 * q.w[(int64_t)row * q.d_r + (int64_t)c0 * q.d_c];
        t[1] += x2;
      }
      if (c1ok) {
        const double x2 = acc1[v] * acc1[v];
        t[0] += x2 * q.w[(int64_t)row * q.d_r + (int64_t)c1 * q.d_c];
        t[1] += x2;
      }
    }
    t[0] = wave_sum(t[0]);
    t[1] = wave_sum(t[1]);
    if (lane == 0) {
      const int ntiles = rtn * ctn * q.planes;
      q.part[((int64_t)rhs * ntiles + tile) * 2] = t[0];
      q.part[((int64_t)rhs * ntiles + tile) * 2 + 1] = t[1];
    }
    return;
  }
  double* D = q.D + rhs * q.d_rhs + p * q.d_p;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = rt * 16 + 4 * v + grp;
    if (row >= q.rows) continue;
    if (c0ok) D[(int64_t)row * q.d_r + (int64_t)c0 * q.d_c] = acc0[v];
    if (c1ok) D[(int64_t)row * q.d_r + (int64_t)c1 * q.d_c] = acc1[v];
  }
}

// The bound from the per-tile sums of the box coefficients:
// ||L^+ R||^2 <= sum_box rhat^2 / lambda^2 + (||R||^2 - sum_box rhat^2) / theta^2,
// relative to ||U_s||.
__global__ __launch_bounds__(64) void k_cert_fin(const double* part, int ntiles,
                                                 double theta2inv, RhsState* st, double tol) {
  const int rhs = blockIdx.x;
  if (!st[rhs].need_cert) return;
  const double* pp = part + (int64_t)rhs * ntiles * 2;
  double low = 0.0, box = 0.0;
  for (int t = threadIdx.x; t < ntiles; t += 64) {
    low += pp[2 * t];
    box += pp[2 * t + 1];
  }
  low = wave_sum(low);
  box = wave_sum(box);
  if (threadIdx.x != 0) return;
  RhsState& s = st[rhs];
  s.need_cert = 0;
  const double rest = s.rr - box;
  const double bound = sqrt((low + (rest > 0.0 ? rest : 0.0) * theta2inv) / s.uu);
  if (bound <= tol) {
    s.err_est = bound;
    s.done = CONVERGED;
  }
}

void launch_cert(const Geom& g, const CertOps& c, const double* R, double* C1, double* C2,
                 double* part, RhsState* st, int batch, double tol, hipStream_t s) {
  const int M = CERT_M;
  const int64_t rows1 = g.N / g.nx;                 // (z, y) rows of R
  auto run = [&](const SmallGemm& q) {
    const int tiles = ((q.rows + 15) / 16) * ((q.cols + 31) / 32) * q.planes;
    const bool va = q.a_k == 1 && q.K % 16 == 0 && q.a_r % 2 == 0 && q.a_p % 2 == 0 &&
                    q.a_rhs % 2 == 0 && ((uintptr_t)q.A & 15) == 0;
    if (va)
      hipLaunchKernelGGL(k_cert_gemm<true>, dim3(tiles, batch), dim3(VT), 0, s, q,
                         (const RhsState*)st);
    else
      hipLaunchKernelGGL(k_cert_gemm<false>, dim3(tiles, batch), dim3(VT), 0, s, q,
                         (const RhsState*)st);
  };
  trace_begin(KC_CERT, s);
  const int nzp = g.dim == 3 ? g.nz : 1;
  // x: C1[(z, y)][i] = sum_x R[(z, y)][x] Vx[x][i]
  run({R, g.nx, 1, 0, g.N,
       c.V[0], M, 1, 0, 0,
       C1, M, 1, 0, rows1 * M,
       (int)rows1, M, g.nx, 1, nullptr, nullptr});
  // y, per z-plane: C2[z][j][i] = sum_y Vy[y][j] C1[(z, y)][i]; in 2D this is
  // the box, reduced at once into per-tile sums
  const bool last_y = g.dim == 2;
  const SmallGemm qy{c.V[1], 1, M, 0, 0,
                     C1, M, 1, (int64_t)g.ny * M, rows1 * M,
                     C2, M, 1, (int64_t)M * M, (int64_t)nzp * M * M,
                     M, M, g.ny, nzp, last_y ? c.w : nullptr, last_y ? part : nullptr};
  run(qy);
  int ntiles = ((M + 15) / 16) * ((M + 31) / 32) * nzp;
  if (g.dim == 3) {
    // z: box[k][(j, i)] = sum_z Vz[z][k] C2[z][(j, i)], reduced into per-tile sums
    const SmallGemm qz{c.V[2], 1, M, 0, 0,
                       C2, (int64_t)M * M, 1, 0, (int64_t)nzp * M * M,
                       nullptr, (int64_t)M * M, 1, 0, 0,
                       M, M * M, g.nz, 1, c.w, part};
    run(qz);
    ntiles = ((M + 15) / 16) * ((M * M + 31) / 32);
  }
  hipLaunchKernelGGL(k_cert_fin, dim3(batch), dim3(64), 0, s, (const double*)part, ntiles,
                     c.theta2inv, st, tol);
  trace_end(KC_CERT, s);
}

// ------------------------------------------------------------- timing ----
// splitmix64's output function of the index (Steele, Lea, Flood 2014) as a
// fixed pattern of doubles in [-1, 1).
__global__ __launch_bounds__(VT) void k_fill(double* __restrict__ x, int64_t n, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
    uint64_t z = (uint64_t)i + seed * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
  }
}

__global__ void k_timing_states(RhsState* st, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  RhsState s = {};
  s.h2 = 1.0;
  s.rho = 1.0;
  s.alpha = 0.5;
  s.beta = 0.5;
  s.scale = 1.0;
  s.inv_scale = 1.0;
  s.done = RUNNING;
  s.iter = 1;          // an iteration past the first (reads U)
  s.pinv_count = 1;
  st[b] = s;
}

void launch_fill(double* x, int64_t n, uint64_t seed, hipStream_t s) {
  const int64_t want = (n + VT - 1) / VT;
  const int blocks = (int)(want < 4096 ? (want < 1 ? 1 : want) : 4096);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(VT), 0, s, x, n, seed);
}

void launch_timing_states(RhsState* st, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_timing_states, dim3((batch + 63) / 64), dim3(64), 0, s, st, batch);
}

bool launch_vector_class(int cls, const Geom& g, double* P, double* W, double* R, double* U,
                         double* Z, double* part, const RhsState* st, int batch, int G,
                         int flags, hipStream_t s) {
  const ZGrid z = zgrid_for(g);
  const dim3 zgrid(z.nblocks, batch), grid(G, batch);
  const bool flex = (flags & F_FLEX_BETA) != 0;
  switch (cls) {
    case KC_STENCIL:
      hipLaunchKernelGGL(k_zm<ZM_PW>, zgrid, dim3(VT), 0, s, g, z, (const double*)P,
                         flex ? W : (double*)nullptr, (double*)nullptr, (double*)nullptr,
                         (const double*)nullptr, part, st, 0.0, 0);
      return true;
    case KC_UPDATE_UR:
      hipLaunchKernelGGL(k_zm<ZM_UR>, zgrid, dim3(VT), 0, s, g, z, (const double*)P,
                         (double*)nullptr, R, U, (const double*)nullptr, part, st, 0.0, 0);
      return true;
    case KC_DOT_RZ:
      hipLaunchKernelGGL(k_dot_rz, grid, dim3(VT), 0, s, g, (const double*)R, (const double*)Z,
                         flex ? (const double*)W : nullptr, part, st, G);
      return true;
    case KC_UPDATE_P:
      hipLaunchKernelGGL(k_update_p, grid, dim3(VT), 0, s, g, (const double*)Z, P, st, G, 0);
      return true;
    default:
      return false;
  }
}

}  // namespace kp
