// Mode products of the pseudoinverse preconditioner (Algs. 6 and 7, Sec. 4.3.3)
// on the gfx950 matrix cores.
//
// The preconditioner is Z = (V_x, V_y, V_z | G .* (V_x^T, V_y^T, V_z^T | R)).
// With the grid stored [z][y][x] (x contiguous) each l-mode product is a GEMM:
//   * y- and z-modes ("left" products): Y[b][m][n] = sum_k A[m][k] X[b][k][n],
//     where k runs over the contracted axis (stride ldk) and n over the
//     contiguous rest; A = V^T (forward) or V (backward);
//   * x-mode ("right" product): Y[r][n] = sum_k X[r][k] B[k][n], with r the
//     (y, z) fibre index and B = V_x (forward) or V_x^T (backward); the
//     forward x product also applies the Hadamard factor G of eq. (4.6).
//
// Precisions: FP64 MFMA (v_mfma_f64_16x16x4), FP32 MFMA (v_mfma_f32_16x16x4)
// and BF16 MFMA with FP32 accumulation (v_mfma_f32_16x16x32_bf16).  Operands:
// lane l supplies row (A) or column (B) l%16 of the 16x16 fragment.  Output
// item v of lane l is column l%16 and row 4*(l/16)+v for the FP32 and BF16
// instructions but row 4*v+l/16 for the FP64 one (measured on gfx950).  The
// contracted index is split across lanes the same way for both operands, so
// any assignment of k to (lane, slot) gives the same sum.
#include "kp_common.h"
#include "kp_internal.h"

namespace kp {

template <int PREC> struct PT;
template <> struct PT<PREC_F64> {
  using tc = double; using acc = d4; using frag = double; using af = double;
  static constexpr int VEC = 1;
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct PT<PREC_F32> {
  using tc = float; using acc = f4; using frag = float; using af = float;
  static constexpr int VEC = 1;
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct PT<PREC_BF16> {
  using tc = __bf16; using acc = f4; using frag = bf8; using af = float;
  static constexpr int VEC = 8;
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <class T, class S> __device__ __forceinline__ T cvt(S x);
template <> __device__ __forceinline__ double cvt<double, double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt<float, double>(double x) { return (float)x; }
template <> __device__ __forceinline__ __bf16 cvt<__bf16, double>(double x) { return (__bf16)(float)x; }
template <> __device__ __forceinline__ float cvt<float, float>(float x) { return x; }
template <> __device__ __forceinline__ __bf16 cvt<__bf16, float>(float x) { return (__bf16)x; }
template <> __device__ __forceinline__ __bf16 cvt<__bf16, __bf16>(__bf16 x) { return x; }
template <> __device__ __forceinline__ double cvt<double, float>(float x) { return (double)x; }
template <> __device__ __forceinline__ float cvt<float, __bf16>(__bf16 x) { return (float)x; }

// Tile: 64 x 64 outputs per 256-thread block, 2 x 2 waves of 32 x 32, each a
// 2 x 2 grid of 16 x 16 MFMA fragments; the contracted axis advances by BK.
constexpr int BM = 64, BN = 64, BK = 32, NT = 256;
constexpr int PAD = 4;

// Hadamard pseudoinverse entry of eq. (4.6)/(4.7): 1/sum, or 0 when the
// eigenvalue sum has modulus below 1e-13.
__device__ __forceinline__ double ghat(double s) { return fabs(s) < 1e-13 ? 0.0 : 1.0 / s; }

// ---------------------------------------------------------------------------
// Left product: Y[b][m][n] = sum_k A[m][k] X[b][k][n], m, k in [0, K).
//   A  : K x K operator (row pitch lda), zero-padded to a multiple of BK
//   X  : input, element (b, k, n) at b*bstride + k*ldk + n   (type Ti)
//   Y  : output, same indexing                               (type To)
//   nbatch_rhs: number of b-slices per right-hand side (for the done flag)
//   in_scale / out_scale: multiply input / output by the per-RHS power-of-two
//   scale or its inverse (low-precision range guard).
// For VEC = 1 the kernel reads At (= A^T, row-major) so that its LDS tile is
// [k][m]; for VEC = 8 it reads A itself and keeps [m][k].
// ---------------------------------------------------------------------------
template <int PREC, class Ti, class To>
__global__ __launch_bounds__(NT) void mode_left_kernel(
    const typename PT<PREC>::tc* __restrict__ Aop, int lda, const Ti* __restrict__ X,
    To* __restrict__ Y, int K, int ninner, int64_t ldk, int64_t bstride, int nbatch_rhs,
    const RhsState* __restrict__ st, int in_scale, int out_scale) {
  using P = PT<PREC>;
  using tc = typename P::tc;
  constexpr int VEC = P::VEC;
  const int b = blockIdx.z;
  const int rhs = b / nbatch_rhs;
  if (st && st[rhs].done) return;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const double sin_ = (st && in_scale) ? st[rhs].scale : 1.0;
  const Ti* Xb = X + (int64_t)b * bstride;

  // VEC==1: As[k][m], Xs[k][n];  VEC==8: As[m][k], Xs[n][k]
  __shared__ __attribute__((aligned(16))) tc As[VEC == 1 ? BK * (BM + PAD) : BM * (BK + 8)];
  __shared__ __attribute__((aligned(16))) tc Xs[VEC == 1 ? BK * (BN + PAD) : BN * (BK + 8)];

  typename P::acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;

  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    // operator tile (padded, always in bounds)
#pragma unroll
    for (int q = 0; q < (BM * BK) / NT; ++q) {
      const int e = tid + q * NT;
      if constexpr (VEC == 1) {
        const int kr = e / BM, mc = e % BM;
        As[kr * (BM + PAD) + mc] = Aop[(int64_t)(k0 + kr) * lda + (m0 + mc)];
      } else {
        const int mr = e / BK, kc = e % BK;
        As[mr * (BK + 8) + kc] = Aop[(int64_t)(m0 + mr) * lda + (k0 + kc)];
      }
    }
    // data tile with bounds checks (zero fill)
#pragma unroll
    for (int q = 0; q < (BK * BN) / NT; ++q) {
      const int e = tid + q * NT;
      const int kr = e / BN, nc = e % BN;
      const int k = k0 + kr, n = n0 + nc;
      tc v = (tc)0.0f;
      if (k < K && n < ninner) {
        if (in_scale) v = cvt<tc>(to_double(Xb[(int64_t)k * ldk + n]) * sin_);
        else v = cvt<tc>(Xb[(int64_t)k * ldk + n]);
      }
      if constexpr (VEC == 1) Xs[kr * (BN + PAD) + nc] = v;
      else Xs[nc * (BK + 8) + kr] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4 * VEC) {
      typename P::frag af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int mrow = wm * 32 + i * 16 + (lane & 15);
        const int ncol = wn * 32 + i * 16 + (lane & 15);
        if constexpr (VEC == 1) {
          af[i] = As[(kk + (lane >> 4)) * (BM + PAD) + mrow];
          bfr[i] = Xs[(kk + (lane >> 4)) * (BN + PAD) + ncol];
        } else {
          af[i] = *reinterpret_cast<const bf8*>(&As[mrow * (BK + 8) + kk + (lane >> 4) * 8]);
          bfr[i] = *reinterpret_cast<const bf8*>(&Xs[ncol * (BK + 8) + kk + (lane >> 4) * 8]);
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = P::mma(af[i], bfr[j], acc[i][j]);
    }
  }

  const double sout = (st && out_scale) ? st[rhs].inv_scale : 1.0;
  To* Yb = Y + (int64_t)b * bstride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * 32 + i * 16 + P::row(lane, v);
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m < K && n < ninner) {
          if (out_scale) Yb[(int64_t)m * ldk + n] = cvt<To>((double)acc[i][j][v] * sout);
          else Yb[(int64_t)m * ldk + n] = cvt<To>(acc[i][j][v]);
        }
      }
}

// ---------------------------------------------------------------------------
// Right product along x: Y[r][n] = sum_k X[r][k] B[k][n], r in [0, rows).
//   X, Y: rows of length nx (contiguous), right-hand side b at b*N.
//   VEC == 1 reads B (row-major, tile [k][n]); VEC == 8 reads Bt = B^T
//   (tile [n][k]).  Both are zero-padded to multiples of the tile.
//   With lam != nullptr the outputs are multiplied by ghat(lx[n] + ly[j] +
//   lz[k]) where r = k*ny + j (the Hadamard step of Algs. 6-7).
// ---------------------------------------------------------------------------
template <int PREC, class Ti, class To>
__global__ __launch_bounds__(NT) void mode_right_kernel(
    const typename PT<PREC>::tc* __restrict__ Bop, int ldb, const Ti* __restrict__ X,
    To* __restrict__ Y, int nx, int rows, int64_t N, const RhsState* __restrict__ st,
    const double* __restrict__ lx, const double* __restrict__ ly, const double* __restrict__ lz,
    int ny) {
  using P = PT<PREC>;
  using tc = typename P::tc;
  constexpr int VEC = P::VEC;
  const int rhs = blockIdx.z;
  if (st && st[rhs].done) return;
  const int r0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const Ti* Xb = X + (int64_t)rhs * N;

  __shared__ __attribute__((aligned(16))) tc Xs[BM * (BK + (VEC == 1 ? 1 : 8))];   // [r][k]
  __shared__ __attribute__((aligned(16))) tc Bs[VEC == 1 ? BK * (BN + PAD) : BN * (BK + 8)];
  constexpr int XP = BK + (VEC == 1 ? 1 : 8);

  typename P::acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;

  for (int k0 = 0; k0 < nx; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (BM * BK) / NT; ++q) {
      const int e = tid + q * NT;
      const int rr = e / BK, kc = e % BK;
      const int r = r0 + rr, k = k0 + kc;
      tc v = (tc)0.0f;
      if (r < rows && k < nx) v = cvt<tc>(Xb[(int64_t)r * nx + k]);
      Xs[rr * XP + kc] = v;
    }
#pragma unroll
    for (int q = 0; q < (BK * BN) / NT; ++q) {
      const int e = tid + q * NT;
      if constexpr (VEC == 1) {
        const int kr = e / BN, nc = e % BN;
        Bs[kr * (BN + PAD) + nc] = Bop[(int64_t)(k0 + kr) * ldb + (n0 + nc)];
      } else {
        const int nr = e / BK, kc = e % BK;
        Bs[nr * (BK + 8) + kc] = Bop[(int64_t)(n0 + nr) * ldb + (k0 + kc)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4 * VEC) {
      typename P::frag af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int rrow = wm * 32 + i * 16 + (lane & 15);
        const int ncol = wn * 32 + i * 16 + (lane & 15);
        if constexpr (VEC == 1) {
          af[i] = Xs[rrow * XP + kk + (lane >> 4)];
          bfr[i] = Bs[(kk + (lane >> 4)) * (BN + PAD) + ncol];
        } else {
          af[i] = *reinterpret_cast<const bf8*>(&Xs[rrow * XP + kk + (lane >> 4) * 8]);
          bfr[i] = *reinterpret_cast<const bf8*>(&Bs[ncol * (BK + 8) + kk + (lane >> 4) * 8]);
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = P::mma(af[i], bfr[j], acc[i][j]);
    }
  }

  To* Yb = Y + (int64_t)rhs * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + wm * 32 + i * 16 + P::row(lane, v);
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (r < rows && n < nx) {
          double val = (double)acc[i][j][v];
          if (lx) {
            const int jy = r % ny, kz = r / ny;
            val *= ghat(lx[n] + ly[jy] + (lz ? lz[kz] : 0.0));
          }
          Yb[(int64_t)r * nx + n] = cvt<To>(val);
        }
      }
}

// ------------------------------------------------------------------ host ----
template <int PREC, class Ti, class To>
static void launch_left(int cls, const void* A, int lda, const void* X, void* Y, int K,
                        int ninner, int64_t ldk, int64_t bstride, int nb_total, int nbatch_rhs,
                        const RhsState* st, int in_scale, int out_scale, hipStream_t s) {
  dim3 grid((ninner + BN - 1) / BN, (K + BM - 1) / BM, nb_total);
  trace_begin(cls, s);
  hipLaunchKernelGGL((mode_left_kernel<PREC, Ti, To>), grid, dim3(NT), 0, s,
                     (const typename PT<PREC>::tc*)A, lda, (const Ti*)X, (To*)Y, K, ninner, ldk,
                     bstride, nbatch_rhs, st, in_scale, out_scale);
  trace_end(cls, s);
}

template <int PREC, class Ti, class To>
static void launch_right(int cls, const void* B, int ldb, const void* X, void* Y, int nx,
                         int rows, int64_t N, int batch, const RhsState* st, const double* lx,
                         const double* ly, const double* lz, int ny, hipStream_t s) {
  dim3 grid((nx + BN - 1) / BN, (rows + BM - 1) / BM, batch);
  trace_begin(cls, s);
  hipLaunchKernelGGL((mode_right_kernel<PREC, Ti, To>), grid, dim3(NT), 0, s,
                     (const typename PT<PREC>::tc*)B, ldb, (const Ti*)X, (To*)Y, nx, rows, N, st,
                     lx, ly, lz, ny);
  trace_end(cls, s);
}

int pad_to_tile(int n) { return ((n + 63) / 64) * 64; }

// Applies Z = M(R) for `batch` right-hand sides.  R and Z are FP64 grids;
// T0 and T1 are scratch grids in the preconditioner's storage type.
template <int PREC>
static void pinv_apply_t(const PinvOps& op, const double* R, double* Z, void* T0, void* T1,
                         int batch, const RhsState* st, hipStream_t s) {
  using tc = typename PT<PREC>::tc;
  const int nx = op.n[0], ny = op.n[1], nz = op.n[2];
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t plane = (int64_t)nx * ny;
  const bool three_d = op.dim == 3;
  const int scl = (PREC == PREC_F64) ? 0 : 1;
  // A-side operand selection: VEC 1 reads A^T, VEC 8 reads A.
  constexpr bool V1 = PT<PREC>::VEC == 1;
  auto fwdA = [&](int ax) { return V1 ? op.Q[ax] : op.Qt[ax]; };   // A = V^T
  auto bwdA = [&](int ax) { return V1 ? op.Qt[ax] : op.Q[ax]; };   // A = V
  // x-mode B operand: VEC 1 reads B, VEC 8 reads B^T.
  const void* Bf = V1 ? op.Q[0] : op.Qt[0];    // forward  B = V_x
  const void* Bb = V1 ? op.Qt[0] : op.Q[0];    // backward B = V_x^T
  const int ldp[3] = {op.np[0], op.np[1], op.np[2]};

  if (three_d) {
    // forward z: T0 = R x_3 V_z^T  (reads FP64, scales into the compute range)
    launch_left<PREC, double, tc>(KC_MP_Z_FWD, fwdA(2), ldp[2], R, T0, nz, (int)plane, plane, N, batch, 1, st,
                                  scl, 0, s);
    // forward y: T1 = T0 x_2 V_y^T, one slice per z-plane
    launch_left<PREC, tc, tc>(KC_MP_Y_FWD, fwdA(1), ldp[1], T0, T1, ny, nx, nx, plane, batch * nz, nz, st, 0, 0,
                              s);
  } else {
    launch_left<PREC, double, tc>(KC_MP_Y_FWD, fwdA(1), ldp[1], R, T1, ny, nx, nx, plane, batch, 1, st, scl, 0,
                                  s);
  }
  // forward x with the Hadamard factor: T0 = G .* (T1 x_1 V_x^T)
  launch_right<PREC, tc, tc>(KC_MP_X_FWD, Bf, ldp[0], T1, T0, nx, ny * nz, N, batch, st, op.lam[0], op.lam[1],
                             three_d ? op.lam[2] : nullptr, ny, s);
  // backward x: T1 = T0 x_1 V_x
  launch_right<PREC, tc, tc>(KC_MP_X_BWD, Bb, ldp[0], T0, T1, nx, ny * nz, N, batch, st, nullptr, nullptr,
                             nullptr, ny, s);
  if (three_d) {
    launch_left<PREC, tc, tc>(KC_MP_Y_BWD, bwdA(1), ldp[1], T1, T0, ny, nx, nx, plane, batch * nz, nz, st, 0, 0,
                              s);
    launch_left<PREC, tc, double>(KC_MP_Z_BWD, bwdA(2), ldp[2], T0, Z, nz, (int)plane, plane, N, batch, 1, st, 0,
                                  scl, s);
  } else {
    launch_left<PREC, tc, double>(KC_MP_Y_BWD, bwdA(1), ldp[1], T1, Z, ny, nx, nx, plane, batch, 1, st, 0, scl,
                                  s);
  }
}

void pinv_apply(const PinvOps& op, const double* R, double* Z, void* T0, void* T1, int batch,
                const RhsState* st, hipStream_t s) {
  switch (op.prec) {
    case PREC_F64: pinv_apply_t<PREC_F64>(op, R, Z, T0, T1, batch, st, s); break;
    case PREC_F32: pinv_apply_t<PREC_F32>(op, R, Z, T0, T1, batch, st, s); break;
    default: pinv_apply_t<PREC_BF16>(op, R, Z, T0, T1, batch, st, s); break;
  }
}

}  // namespace kp
