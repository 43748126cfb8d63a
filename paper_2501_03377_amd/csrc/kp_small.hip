// Whole solves of small 2D problems in one kernel: Algorithm 1 with the FP64
// pseudoinverse preconditioner (Alg. 6), one 1024-thread workgroup per
// right-hand side, every vector resident in LDS.
//
// For n x q grids up to 64 x 64 a solve is a few dozen tiny steps, so the
// multi-kernel path spends its time launching kernels.  Here R, P and two
// transform buffers (4 x 33 KiB, rows padded to 65 doubles) stay in LDS, U
// stays in registers, the four mode products of an application run on the
// FP64 matrix cores with the eigenbases (and their transposes) read through
// the cache, Ghat is applied in the epilogue of the second product, and the
// scalar recurrences, the stopping tests and the exit step (true residual,
// centring) run in the same kernel.
// The recurrences and stopping tests are those of the multi-kernel path,
// except that the low-mode certificate is not tried (the bound
// ||R|| / lambda_min or the estimate after the next application decide);
// the inner products, <R, Z> and the mean of Z included, are summed in space
// in a fixed order of their own, so results agree with that path to
// rounding.
#include <math.h>

#include "kp_common.h"
#include "kp_internal.h"

namespace kp {
namespace {

constexpr int ST = 1024;                 // threads per workgroup
constexpr int SW = ST / 64;              // waves
constexpr int SMAX = 64;                 // largest axis
constexpr int LP = SMAX + 1;             // LDS row pitch in doubles (odd, see wg_gemm)
constexpr int SL = SMAX * LP;            // doubles per grid buffer in LDS
constexpr int SE = SMAX / SW;            // grid rows per thread

// Lane moves of a double by DPP (two 32-bit halves) and reads of one lane.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double lane_d(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 16 lanes of each DPP row (pairs, quads, then two rotations);
// the first lane of a row holds the total in a fixed association.
__device__ __forceinline__ double row_sum(double v) {
  v += dpp<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp<0x124>(v);   // row_ror:4
  v += dpp<0x128>(v);   // row_ror:8
  return v;
}

// Fixed-order reduction of NV values over the workgroup: rows of each wave,
// the four row totals in order, then the SW wave totals by one more row sum.
// Every thread returns the same totals.  All lanes must be active.
template <int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double (*red)[4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double t = row_sum(v[q]);
    v[q] = (lane_d(t, 0) + lane_d(t, 16)) + (lane_d(t, 32) + lane_d(t, 48));
  }
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[wave][q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = lane_d(row_sum(red[lane % SW][q]), 0);
  __syncthreads();
}

__device__ __forceinline__ double ghat_s(double s) { return fabs(s) < 1e-13 ? 0.0 : 1.0 / s; }

// D[r][c] (pitch LP in LDS) = sum_k A(r, k) B(k, c) for r < rows <= 64,
// c < cols <= 64, on the FP64 matrix cores; with gc, gr each result is then
// multiplied by ghat(gc[c] + gr[r]).  Wave w owns the 16 x 16 tile
// (w % 4, w / 4); v_mfma_f64_16x16x4f64 takes A(l % 16, k) and B(k, l % 16)
// from lane l for k = k0 + l / 16 and returns D(4 v + l / 16, l % 16) in
// element v.  The sixteen lanes of a k group read sixteen consecutive r (A)
// or c (B): every operand layout below makes that index the unit-stride one
// in global memory, and LDS rows have an odd pitch so that a column read hits
// distinct banks.  The operands of KB steps are loaded together (indices
// clamped into range, out-of-range values replaced by zeros afterwards) so
// that their latencies overlap.
__device__ __forceinline__ void wg_gemm(const double* A, int a_r, int a_k, const double* B,
                                        int b_k, int b_c, double* D, int rows, int cols, int K,
                                        const double* gc, const double* gr) {
  constexpr int KB = 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rt = wave % 4, ct = wave / 4;
  if (rt * 16 < rows && ct * 16 < cols) {
    const int l16 = lane & 15, grp = lane >> 4;
    const int r = rt * 16 + l16, c = ct * 16 + l16;
    const bool rok = r < rows, cok = c < cols;
    const double* Ar = A + (rok ? r : 0) * a_r;
    const double* Bc = B + (cok ? c : 0) * b_c;
    double lc = 0.0, lr[4] = {0.0, 0.0, 0.0, 0.0};
    if (gc) {
      lc = gc[cok ? c : 0];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rt * 16 + 4 * v + grp;
        lr[v] = gr[row < rows ? row : 0];
      }
    }
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4 * KB) {
      double a[KB], b[KB];
#pragma unroll
      for (int j = 0; j < KB; ++j) {
        const int k = k0 + 4 * j + grp;
        const int kc = k < K ? k : 0;
        a[j] = Ar[kc * a_k];
        b[j] = Bc[kc * b_k];
      }
#pragma unroll
      for (int j = 0; j < KB; ++j) {
        const bool kok = k0 + 4 * j + grp < K;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((rok && kok) ? a[j] : 0.0,
                                                   (cok && kok) ? b[j] : 0.0, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rt * 16 + 4 * v + grp;
      if (row < rows && cok) D[row * LP + c] = gc ? acc[v] * ghat_s(lc + lr[v]) : acc[v];
    }
  }
  __syncthreads();
}

// One axis of the minus Laplacian at LDS index i (ghost rule of eq. 3.1 at
// the ends).
__device__ __forceinline__ double axis(const double* p, int i, int pos, int n, int stride, int bc,
                                       double c) {
  double lo, hi;
  if (pos > 0) lo = p[i - stride];
  else if (bc == BC_P) lo = p[i + (n - 1) * stride];
  else lo = (bc == BC_N || bc == BC_ND) ? c : 0.0;
  if (pos < n - 1) hi = p[i + stride];
  else if (bc == BC_P) hi = p[i - (n - 1) * stride];
  else hi = (bc == BC_N || bc == BC_DN) ? c : 0.0;
  return (2.0 * c - lo) - hi;
}

__device__ __forceinline__ double lap(const Geom& g, const double* p, int x, int y) {
  const int i = y * LP + x;
  const double c = p[i];
  return axis(p, i, x, g.nx, 1, g.bc[0], c) + axis(p, i, y, g.ny, LP, g.bc[1], c);
}

// Z (in zb) = M(R) for R in rb (Alg. 6), grids [y][x] with pitch LP:
// F1 = R Vx, F2 = Ghat o (Vy^T F1), G1 = F2 Vx^T, Z = Vy G1; tb is scratch.
// V[p][m] holds basis vector m at point p, Vt its transpose.
__device__ __forceinline__ void pinv(const Geom& g, const SmallOps& o, const double* rb, double* tb,
                                     double* zb) {
  const int nx = g.nx, ny = g.ny;
  wg_gemm(rb, LP, 1, o.Vx, nx, 1, tb, ny, nx, nx, nullptr, nullptr);    // F1[y][i]
  wg_gemm(o.Vy, 1, ny, tb, LP, 1, zb, ny, nx, ny, o.lx, o.ly);          // F2[j][i]
  wg_gemm(zb, LP, 1, o.Vxt, nx, 1, tb, ny, nx, nx, nullptr, nullptr);   // G1[j][x]
  wg_gemm(o.Vyt, 1, ny, tb, LP, 1, zb, ny, nx, ny, nullptr, nullptr);   // Z[y][x]
}

// Thread (lane x, wave y0) owns the points (x, y0 + SW q), q < SE.
__global__ __launch_bounds__(ST) void k_small_solve(Geom g, SmallOps o, const double* eta,
                                                    double* Uout, RhsState* st, RhsState* mirror,
                                                    double* hist, int hist_stride, double tol,
                                                    int max_iter, int flags) {
  __shared__ double R[SL], P[SL], TA[SL], TB[SL];
  __shared__ double red[SW][4];
  const int rhs = blockIdx.x;
  const int nx = g.nx, ny = g.ny;
  const int x = threadIdx.x & 63, y0 = threadIdx.x >> 6;
  const int64_t off = (int64_t)rhs * g.N;
  const double Nd = (double)g.N;
  // point q of this thread: in the grid, its LDS index, its index in the
  // right-hand side's grid (clamped into it)
  auto in = [&](int q) { return x < nx && y0 + SW * q < ny; };
  auto li = [&](int q) { return (y0 + SW * q) * LP + x; };
  auto gi = [&](int q) { return in(q) ? (y0 + SW * q) * nx + x : 0; };
  double u[SE];
#pragma unroll
  for (int q = 0; q < SE; ++q) u[q] = 0.0;

  // the recurrences' scalars (only scalars, so that they stay in registers)
  struct {
    double h2, mean, rho, alpha, beta, rr, rsum, uu, pw, rz, zz, zmean, rel_res, err_est;
    int iter, done, pinv_count;
  } s = {};

  // eta_c (eq. 3.6) into R; R_0 = eta_c since U_0 = 0
  {
    double e[SE];
#pragma unroll
    for (int q = 0; q < SE; ++q) e[q] = eta[off + gi(q)];
    if (g.singular) {
      double v[1] = {0.0};
#pragma unroll
      for (int q = 0; q < SE; ++q)
        if (in(q)) v[0] += e[q];
      wg_sum<1>(v, red);
      s.mean = v[0] / Nd;
    }
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int q = 0; q < SE; ++q)
      if (in(q)) {
        const double t = e[q] - s.mean;
        R[li(q)] = t;
        v[0] += t;
        v[1] += t * t;
      }
    wg_sum<2>(v, red);
    s.rsum = v[0];
    s.h2 = v[1];
    s.rr = v[1];
  }
  if (!isfinite(s.h2)) s.done = NONFINITE;
  else if (s.h2 == 0.0) s.done = ZERO_RHS;
  s.rel_res = s.done == ZERO_RHS ? 0.0 : 1.0;
  if (hist && threadIdx.x == 0) hist[(int64_t)rhs * hist_stride] = s.rel_res;

  // Z = M(R), rho, P = Z + beta P (centred, Remark 4.1), with the stopping
  // tests that follow an application
  auto precondition = [&](bool first) {
    pinv(g, o, R, TA, TB);
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < SE; ++q)
      if (in(q)) {
        const double z = TB[li(q)];
        v[0] += R[li(q)] * z;
        v[1] += z;
        v[2] += z * z;
      }
    wg_sum<3>(v, red);
    const double zmean = g.singular ? v[1] / Nd : 0.0;
    const double rz = v[0] - zmean * s.rsum;
    double zz = v[2] - Nd * zmean * zmean;
    if (zz < 0.0) zz = 0.0;
    s.zmean = zmean;
    s.rz = rz;
    s.zz = zz;
    s.pinv_count += 1;
    if (!isfinite(rz) || !isfinite(zz)) { s.done = NONFINITE; return; }
    if (first) {
      if (!(rz > 0.0)) { s.done = BREAKDOWN; return; }
      s.rho = rz;
      s.beta = 0.0;
    } else {
      s.err_est = s.uu > 0.0 ? sqrt(zz / s.uu) : INFINITY;
      if (!(flags & F_RESIDUAL_ONLY) && s.rel_res <= tol && s.err_est <= tol) {
        s.done = CONVERGED;
        return;
      }
      if (!(rz > 0.0)) { s.done = (s.rel_res <= tol) ? CONVERGED : BREAKDOWN; return; }
      s.beta = rz / s.rho;                                   // beta_s = rho_s / rho_{s-1}
      s.rho = rz;
    }
#pragma unroll
    for (int q = 0; q < SE; ++q)
      if (in(q)) P[li(q)] = (TB[li(q)] - zmean) + (first ? 0.0 : s.beta * P[li(q)]);
    __syncthreads();
  };
  if (s.done == RUNNING) precondition(true);

  while (s.done == RUNNING && s.iter < max_iter) {
    // W_s = -Delta(P_{s-1}), alpha_s = rho_{s-1} / <W_s, P_{s-1}>
    double w[SE];
    {
      double v[1] = {0.0};
#pragma unroll
      for (int q = 0; q < SE; ++q) {
        w[q] = 0.0;
        if (in(q)) {
          w[q] = lap(g, P, x, y0 + SW * q);
          v[0] += w[q] * P[li(q)];
        }
      }
      wg_sum<1>(v, red);
      s.pw = v[0];
      if (!isfinite(v[0])) { s.done = NONFINITE; break; }
      if (!(v[0] > 0.0)) { s.done = BREAKDOWN; break; }
      s.alpha = s.rho / v[0];
    }
    // U_s = U_{s-1} + alpha P, R_s = R_{s-1} - alpha W
    {
      double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < SE; ++q)
        if (in(q)) {
          u[q] += s.alpha * P[li(q)];
          const double r = R[li(q)] - s.alpha * w[q];
          R[li(q)] = r;
          v[0] += r;
          v[1] += r * r;
          v[2] += u[q] * u[q];
        }
      wg_sum<3>(v, red);
      s.rsum = v[0];
      s.rr = v[1];
      s.uu = v[2];
      s.iter += 1;
      s.rel_res = sqrt(v[1] / s.h2);
      if (hist && threadIdx.x == 0) hist[(int64_t)rhs * hist_stride + s.iter] = s.rel_res;
      if (!isfinite(s.rel_res)) { s.done = NONFINITE; break; }
      if (s.rel_res <= tol) {
        if (flags & F_RESIDUAL_ONLY) { s.done = CONVERGED; break; }
        // ||U_s - u|| = ||L^+ R_s|| <= ||R_s|| / lambda_min
        const double bound = v[2] > 0.0 ? sqrt(v[1] / v[2]) / g.lam_min : INFINITY;
        if (bound <= tol) {
          s.err_est = bound;
          s.done = CONVERGED;
          break;
        }
      }
    }
    precondition(false);
  }

  // exit step: true residual ||eta_c - L U|| / ||eta_c||, centring of U
  double true_rel, umean;
  {
    double e[SE];
#pragma unroll
    for (int q = 0; q < SE; ++q) e[q] = eta[off + gi(q)];
#pragma unroll
    for (int q = 0; q < SE; ++q)
      if (in(q)) TA[li(q)] = u[q];
    __syncthreads();
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int q = 0; q < SE; ++q)
      if (in(q)) {
        const double r = (e[q] - s.mean) - lap(g, TA, x, y0 + SW * q);
        v[0] += r * r;
        v[1] += u[q];
      }
    wg_sum<2>(v, red);
    true_rel = s.h2 > 0.0 ? sqrt(v[0] / s.h2) : 0.0;
    umean = g.singular ? v[1] / Nd : 0.0;
#pragma unroll
    for (int q = 0; q < SE; ++q)
      if (in(q)) Uout[off + gi(q)] = u[q] - umean;
  }
  if (threadIdx.x == 0) {
    RhsState out = {};
    out.h2 = s.h2;
    out.mean = s.mean;
    out.rho = s.rho;
    out.alpha = s.alpha;
    out.beta = s.beta;
    out.rr = s.rr;
    out.rsum = s.rsum;
    out.uu = s.uu;
    out.pw = s.pw;
    out.rz = s.rz;
    out.zz = s.zz;
    out.zmean = s.zmean;
    out.rel_res = s.rel_res;
    out.err_est = s.err_est;
    out.true_rel_res = true_rel;
    out.umean = umean;
    out.scale = out.inv_scale = 1.0;
    out.iter = s.iter;
    out.done = s.done;
    out.pinv_count = s.pinv_count;
    out.diag_iter = -1;
    st[rhs] = out;
    if (mirror) mirror[rhs] = out;
  }
}

}  // namespace

bool small_solve_fits(const Geom& g) { return g.dim == 2 && g.nx <= SMAX && g.ny <= SMAX; }

void launch_small_solve(const Geom& g, const SmallOps& o, const double* eta, double* U,
                        RhsState* st, RhsState* mirror, double* hist, int hist_stride, int batch,
                        double tol, int max_iter, int flags, hipStream_t s) {
  trace_begin(KC_SMALL, s);
  hipLaunchKernelGGL(k_small_solve, dim3(batch), dim3(ST), 0, s, g, o, eta, U, st, mirror, hist,
                     hist_stride, tol, max_iter, flags);
  trace_end(KC_SMALL, s);
}

}  // namespace kp
