// Mode products of the pseudoinverse preconditioner (Algs. 6 and 7, Sec. 4.3.3)
// on the gfx950 matrix cores.
//
// Z = (V_x, V_y, V_z | G .* (V_x^T, V_y^T, V_z^T | R)).  Every l-mode product
// is applied as one GEMM that contracts the *contiguous* axis of its input:
//     C[r][n] = sum_k X[r][k] B[k][n],    X viewed as [A0][A1][K] -> rows r,
// and writes C transposed, Y[n][r], i.e. the layout [K'][A0][A1]: the
// transformed axis moves to the front.  Three such products return the
// original layout, so the sequence (3D; grids stored [z][y][x], x fastest)
//   [z][y][x] -x->  [x'][z][y] -y-> [y'][x'][z] -z,G-> [z'][y'][x']
//             -x->  [x][z'][y'] -y-> [y][x][z']  -z->  [z][y][x]
// contracts x, y, z forward, applies the Hadamard factor G of eq. (4.6) in the
// third product's epilogue, and contracts x, y, z backward (2D: x, y+G, x, y).
// The mode products commute (Sec. 2.2), so this order is the paper's operator.
//
// Operands.  B (V_l forward, V_l^T backward) is packed at plan time in
// fragment order and streamed through a double-buffered LDS chunk shared by
// the block's four waves; each wave loads its own rows of X straight into
// registers (CH consecutive k per lane, 16-byte loads).  MFMA: FP64
// v_mfma_f64_16x16x4, FP32 v_mfma_f32_16x16x4, BF16 v_mfma_f32_16x16x32_bf16
// with FP32 accumulation.  Lane l supplies row (X) / column (B) l%16 and the k
// values CH*(l/16) .. +CH-1 of each k-block; output item v of lane l is column
// l%16 and row 4*(l/16)+v (FP32, BF16) or 4*v+l/16 (FP64, measured on gfx950).
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <type_traits>

#include "kp_common.h"
#include "kp_internal.h"

namespace kp {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));   // one 16-byte unit
typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

template <int PREC> struct MT;
template <> struct MT<PREC_F64> {
  using tc = double; using acc = d4;
  static constexpr int CH = 4, NV = 2;       // k per lane per k-block, 16-byte units
  static constexpr int STEPS = 4;            // MFMAs per k-block and fragment pair
  struct chunk { double v[4]; };
  static __device__ __forceinline__ acc mma(const chunk& a, const chunk& b, acc c, int s) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[s], b.v[s], c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct MT<PREC_F32> {
  using tc = float; using acc = f4;
  static constexpr int CH = 4, NV = 1, STEPS = 4;
  struct chunk { float v[4]; };
  static __device__ __forceinline__ acc mma(const chunk& a, const chunk& b, acc c, int s) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[s], b.v[s], c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct MT<PREC_BF16> {
  using tc = __bf16; using acc = f4;
  static constexpr int CH = 8, NV = 1, STEPS = 1;
  struct chunk { bf8 v; };
  static __device__ __forceinline__ acc mma(const chunk& a, const chunk& b, acc c, int) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// FP32-accurate products on the BF16 matrix cores: a chunk holds the three
// BF16 terms of 8 values (x = x1 + x2 + x3); step s accumulates the product
// of data term split_a(s) and operator term split_b(s), the six pairs with
// i + j <= 2 (0-based), largest first.
constexpr int split_a(int s) { return (s == 2 || s == 4) ? 1 : (s == 5 ? 2 : 0); }
constexpr int split_b(int s) { return (s == 1 || s == 4) ? 1 : (s == 3 ? 2 : 0); }
template <> struct MT<PREC_BF16X6> {
  using tc = float; using acc = f4;
  static constexpr int CH = 8, NV = 3, STEPS = 6;
  struct chunk { bf8 p[3]; };
  static __device__ __forceinline__ acc mma(const chunk& a, const chunk& b, acc c, int s) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[split_a(s)], b.p[split_b(s)], c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// The int8 split products (mp_oz below) keep FP64 between products.
template <> struct MT<PREC_I8X7> {
  using tc = double;
};
template <> struct MT<PREC_I8X6> {
  using tc = double;
};

// Block = WR x WC waves (WR = 4 row groups, WC column groups); each wave owns
// WM row fragments x WN column fragments of 16 x 16.
constexpr int WR = 4;

// Hadamard pseudoinverse entry of eqs. (4.6)-(4.7): 1/sum, or 0 below 1e-13.
__device__ __forceinline__ double ghat(double s) { return fabs(s) < 1e-13 ? 0.0 : 1.0 / s; }

template <int PREC>
__device__ __forceinline__ typename MT<PREC>::tc to_tc(double x) {
  if constexpr (PREC == PREC_BF16) return (__bf16)(float)x;
  else return (typename MT<PREC>::tc)x;
}

// ---- one lane's CH consecutive k values of one row --------------------------
// Loaded raw (source type) into a register ring and converted only when the
// MFMA needs them, so that no arithmetic waits on a load in flight.  Lanes
// past the end of the row (k0 >= K, and rows past the end, which arrive with
// k0 = K) read the row's last CH values instead: the packed operator is zero
// for k >= K, so they add nothing (both are finite data of the same grid).
// VEC: the row length is a multiple of CH (16-byte loads); else CH scalar
// loads.
template <int PREC, class Ti> struct XRaw { Ti v[MT<PREC>::CH]; };

template <int PREC, class Ti, bool VEC>
__device__ __forceinline__ XRaw<PREC, Ti> load_raw(const Ti* __restrict__ row, int k0, int K) {
  constexpr int CH = MT<PREC>::CH;
  XRaw<PREC, Ti> x;
  if constexpr (VEC) {
    const Ti* src = row + (k0 < K ? k0 : K - CH);
    static_assert((CH * sizeof(Ti)) % 16 == 0, "whole 16-byte units");
#pragma unroll
    for (int q = 0; q < (int)(CH * sizeof(Ti)) / 16; ++q) {
      const u4 u = *reinterpret_cast<const u4*>(reinterpret_cast<const char*>(src) + 16 * q);
      __builtin_memcpy(reinterpret_cast<char*>(x.v) + 16 * q, &u, 16);
    }
  } else {
#pragma unroll
    for (int s = 0; s < CH; ++s) x.v[s] = row[k0 + s < K ? k0 + s : K - 1];
  }
  return x;
}

template <int PREC, class Ti>
__device__ __forceinline__ typename MT<PREC>::chunk cvt_raw(const XRaw<PREC, Ti>& x, double scale,
                                                           bool scaled) {
  using M = MT<PREC>;
  typename M::chunk c;
  if constexpr (PREC == PREC_BF16X6) {
    // three round-to-nearest BF16 terms; each remainder is exact in FP32
#pragma unroll
    for (int s = 0; s < M::CH; ++s) {
      float f;
      if constexpr (sizeof(Ti) == 8) f = (float)(scaled ? x.v[s] * scale : x.v[s]);
      else f = x.v[s];
      const __bf16 t1 = (__bf16)f;
      const float r1 = f - (float)t1;
      const __bf16 t2 = (__bf16)r1;
      const float r2 = r1 - (float)t2;
      c.p[0][s] = t1;
      c.p[1][s] = t2;
      c.p[2][s] = (__bf16)r2;
    }
  } else if constexpr (std::is_same<Ti, typename M::tc>::value) {
    __builtin_memcpy(&c, &x, sizeof(c));
  } else {
#pragma unroll
    for (int s = 0; s < M::CH; ++s) {
      const double d = to_double(x.v[s]);
      c.v[s] = to_tc<PREC>(scaled ? d * scale : d);
    }
  }
  return c;
}

template <int PREC>
__device__ __forceinline__ typename MT<PREC>::chunk load_b(const u4* __restrict__ l, int g,
                                                          int c, int CB) {
  using M = MT<PREC>;
  typename M::chunk b;
  static_assert(sizeof(b) == 16 * M::NV, "a chunk is NV 16-byte units");
#pragma unroll
  for (int h = 0; h < M::NV; ++h) {
    const u4 u = l[(g * M::NV + h) * CB + c];
    __builtin_memcpy(reinterpret_cast<char*>(&b) + 16 * h, &u, 16);
  }
  return b;
}

// ---------------------------------------------------------------------------
// One mode product for `batch` right-hand sides.
//   Bpk   packed operator: 16-byte unit (kb, g, h, n) at ((kb*4+g)*NV+h)*npk+n
//   X     input  [rhs][rows][K]  (type Ti)
//   Y     output [rhs][K][rows]  (type To): Y[n*rows + r] = sum_k X[r][k] B[k][n]
//   G epilogue (lc != nullptr): times ghat(la[r % a1] + lb[r / a1] + lc[n])
//   table epilogue (gt != nullptr): times gt[n * rows + r], a precomputed
//   factor in the output's layout (the low-rank preconditioner's G_r)
//   spectral inner products (rpart != nullptr, with the G epilogue): the
//   inputs are the coefficients rhat of R in the eigenbasis and the outputs
//   those of Z = M(R), so by Parseval <R, Z> = sum rhat zhat and ||Z||^2 =
//   sum zhat^2; the block's sums (times the square of the input scale's
//   inverse when rscl) go to the partial slots of the CG step, block
//   blockIdx.x.  Z has no component on the null space (Ghat is 0 there), so
//   its sum is taken as 0.
//   in_scale / out_scale: per-RHS power-of-two scale on the input / its
//   inverse on the output (low-precision range guard)
// Grid: x = row blocks * column chunks, y = right-hand side.
// ---------------------------------------------------------------------------
constexpr int group_size(int wn, int most) {
  int j = wn < most ? wn : most;
  while (wn % j != 0) --j;
  return j;
}
static_assert(group_size(6, 4) == 3 && group_size(12, 8) == 6 && group_size(16, 8) == 8, "");

template <int PREC, class Ti, class To, int WN, int WM, int WC, bool VEC>
__global__ __launch_bounds__(64 * WR * WC, WC == 1 ? 2 : 1) void mp_kernel(
    const u4* __restrict__ Bpk, int npk, int ncc, const Ti* __restrict__ X, To* __restrict__ Y,
    int K, int rows, int64_t N, const RhsState* __restrict__ st, int in_scale, int out_scale,
    const double* __restrict__ la, const double* __restrict__ lb, const double* __restrict__ lc,
    int a1, const double* __restrict__ gt, double* __restrict__ rpart, int rscl) {
  using M = MT<PREC>;
  constexpr int NT = 64 * WR * WC;
  constexpr int CW = 16 * WN;                 // columns per wave
  constexpr int CB = WC * CW;                 // columns per block
  constexpr int BR = WR * 16 * WM;            // rows per block
  constexpr int CH = M::CH, NV = M::NV, KB = 4 * CH;
  constexpr int UNITS = 4 * NV * CB;          // 16-byte units per operator k-block
  // k-blocks per LDS stage (one barrier per stage), at most 32 KiB per stage
  // (two stages resident), 64 KiB for the eight-wave tiles, which run one
  // block per CU anyway.  The data rows are prefetched one stage ahead in a
  // register ring of KS k-blocks indexed by the unrolled step, so no register
  // ever moves inside the ring; larger stages prefetch further ahead.
  constexpr int KSP = PREC == PREC_F64 ? 2 : 4;
  constexpr int SBYTES = (WC == 2 && WM < 4) ? 65536 : 32768;
  constexpr int KSL = SBYTES / (16 * UNITS) > 0 ? SBYTES / (16 * UNITS) : 1;
  constexpr int KS = KSP < KSL ? KSP : KSL;
  constexpr int SUNITS = KS * UNITS;          // units per stage
  constexpr int UPT = (SUNITS + NT - 1) / NT; // units per thread per stage
  // operator fragments read per group: the largest divisor of WN whose
  // fragments take at most 32 VGPRs
  constexpr int JG = group_size(WN, (PREC == PREC_F64 || PREC == PREC_BF16X6) ? 4 : 8);
  // data ring depth: KS k-blocks, halved while the raw data would take more
  // than 64 VGPRs (the FP64 sources of the first product are twice as wide)
  constexpr int RAWV = CH * (int)sizeof(Ti) / 4;
  constexpr int XD = (KS * WM * RAWV <= 64 || KS == 1) ? KS
                     : ((KS / 2) * WM * RAWV <= 64 || KS == 2) ? KS / 2 : KS / 4;
  static_assert(KS % XD == 0, "ring depth divides the stage");

  const int rhs = blockIdx.y;
  if (st && st[rhs].done) return;
  const int cc = blockIdx.x % ncc, rb = blockIdx.x / ncc;
  const int c0 = cc * CB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WR, wc = wave / WR;
  const int g = lane >> 4, l16 = lane & 15;
  const int rw = rb * BR + wr * WM * 16;      // this wave's first row
  const int cw = wc * CW;                     // this wave's first column in the block
  const Ti* Xb = X + (int64_t)rhs * N;
  const bool scaled = (st != nullptr) && in_scale;
  const double scale = scaled ? st[rhs].scale : 1.0;
  const int nkb = (K + KB - 1) / KB;

  __shared__ u4 lds[2][SUNITS];

  const Ti* xrow[WM];
  bool rok[WM];
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    const int r = rw + 16 * i + l16;
    rok[i] = r < rows;
    xrow[i] = Xb + (int64_t)(rok[i] ? r : 0) * K;
  }

  typename M::acc acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;

  // Plain unrolled loops, no closures over these arrays: a captured array
  // gets an address and lands in scratch memory.
  u4 breg[UPT];
  XRaw<PREC, Ti> xq[XD][WM];
  constexpr bool FULL = (SUNITS % NT) == 0;
  const u4* bsrc = Bpk + c0;
  const int cmax = npk - c0;                  // packed columns left for this block
  const int nst = (nkb + KS - 1) / KS;

  // Loads stage `sg` of the operator into breg.  Every load is issued
  // unconditionally, with clamped indices, so that the compiler counts the
  // same loads in flight on every path and waits only for the ones it needs:
  // k-blocks past the end (last stage) and columns past the end (ragged last
  // column chunk) only feed accumulators that are never stored, and threads
  // past the stage size repeat the last unit (the same value to the same
  // LDS address).
#define KP_LOAD_STAGE(sg)                                                                  \
  _Pragma("unroll") for (int q = 0; q < UPT; ++q) {                                       \
    const int su = FULL ? tid + q * NT : min(tid + q * NT, SUNITS - 1);                    \
    const int kk = su / UNITS, u = su % UNITS, gh = u / CB;                                \
    const int c = min(u % CB, cmax - 1);                                                   \
    const int kbg = min((sg) * KS + kk, nkb - 1);                                          \
    breg[q] = bsrc[((int64_t)kbg * 4 * NV + gh) * npk + c];                                \
  }
#define KP_STORE_STAGE(bf)                                                                 \
  _Pragma("unroll") for (int q = 0; q < UPT; ++q) {                                       \
    const int su = FULL ? tid + q * NT : min(tid + q * NT, SUNITS - 1);                    \
    lds[bf][su] = breg[q];                                                                 \
  }

  KP_LOAD_STAGE(0)
#pragma unroll
  for (int d = 0; d < XD; ++d) {
    const int k0 = d * KB + CH * g;
#pragma unroll
    for (int i = 0; i < WM; ++i)
      xq[d][i] = load_raw<PREC, Ti, VEC>(xrow[i], (rok[i] && d < nkb) ? k0 : K, K);
  }
  KP_STORE_STAGE(0)
  __syncthreads();

  for (int sg = 0; sg < nst; ++sg) {
    const int buf = sg & 1;
    KP_LOAD_STAGE(sg + 1)   // past the last stage: a harmless reload
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const int kb = sg * KS + kk;
      const int slot = kk % XD;
      if (KS == 1 || kb < nkb) {
        typename M::chunk xa[WM];
#pragma unroll
        for (int i = 0; i < WM; ++i) xa[i] = cvt_raw<PREC, Ti>(xq[slot][i], scale, scaled);
#pragma unroll
        for (int j0 = 0; j0 < WN; j0 += JG) {
          typename M::chunk b[JG];
#pragma unroll
          for (int jj = 0; jj < JG; ++jj)
            b[jj] = load_b<PREC>(lds[buf] + kk * UNITS, g, cw + 16 * (j0 + jj) + l16, CB);
          // consecutive MFMAs update different accumulators
#pragma unroll
          for (int s = 0; s < M::STEPS; ++s)
#pragma unroll
            for (int jj = 0; jj < JG; ++jj)
#pragma unroll
              for (int i = 0; i < WM; ++i)
                acc[i][j0 + jj] = M::mma(xa[i], b[jj], acc[i][j0 + jj], s);
        }
      }
      // this ring slot now takes k-block kb + XD
      const int kn = kb + XD;
      const int k0 = kn * KB + CH * g;
#pragma unroll
      for (int i = 0; i < WM; ++i)
        xq[slot][i] = load_raw<PREC, Ti, VEC>(xrow[i], (rok[i] && kn < nkb) ? k0 : K, K);
    }
    KP_STORE_STAGE(buf ^ 1)   // the buffer not read in this stage
    __syncthreads();
  }
#undef KP_LOAD_STAGE
#undef KP_STORE_STAGE

  // ---- epilogue: optional G factor and output scale, transposed store ------
  const double oscale = (st && out_scale) ? st[rhs].inv_scale : 1.0;
  To* Yb = Y + (int64_t)rhs * N;
  double fs[2] = {0.0, 0.0};   // spectral <R, Z> and ||Z||^2
  double rowsum[WM][4];
  if (lc) {
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rw + 16 * i + M::row(lane, v);
        const int rc = r < rows ? r : 0;
        rowsum[i][v] = la[rc % a1] + (lb ? lb[rc / a1] : 0.0);
      }
  }
  // Outputs of at most 4 bytes: the block's tile is staged in LDS (free after
  // the k-loop) as [column][row], then written column by column, 16 bytes a
  // thread, so that each column gets one contiguous run of BR rows instead
  // of 16-row pieces from every wave.
  constexpr int SE = 16 / (int)sizeof(To);          // elements per 16-byte chunk
  constexpr int BRP = BR + SE;                      // padded column length
  constexpr bool STG = sizeof(To) <= 4 && (size_t)CB * BRP * sizeof(To) <= sizeof(lds);
  const bool stage = STG && rows % SE == 0;
  To* stg = reinterpret_cast<To*>(&lds[0][0]);
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int n = c0 + cw + 16 * j + l16;
    if (n >= K) continue;
    const double lcn = lc ? lc[n] : 0.0;
    To* dst = Yb + (int64_t)n * rows;
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      To out[4];
      int rr[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        rr[v] = rw + 16 * i + M::row(lane, v);
        double val = (double)acc[i][j][v];
        if (lc) {
          const double sum = rowsum[i][v] + lcn;
          if constexpr (PREC == PREC_F64) {
            val *= ghat(sum);
          } else {
            // FP32 reciprocal: the low-precision preconditioner is accurate
            // to its own rounding anyway
            val = fabs(sum) < 1e-13 ? 0.0 : (double)((float)val * __frcp_rn((float)sum));
          }
        }
        const double rhat = (double)acc[i][j][v];
        if (gt) val *= gt[(int64_t)n * rows + (rr[v] < rows ? rr[v] : 0)];
        if (out_scale) val *= oscale;
        if constexpr (sizeof(To) == 2) out[v] = (__bf16)(float)val;
        else out[v] = (To)val;
        if (rpart && rr[v] < rows) {
          const double zhat = (double)out[v];
          fs[0] += rhat * zhat;
          fs[1] += zhat * zhat;
        }
      }
      if constexpr (STG) {
        if (stage) {
          // the four rows of this lane are consecutive
          To* q = stg + (cw + 16 * j + l16) * BRP + wr * WM * 16 + 16 * i + M::row(lane, 0);
          if constexpr (sizeof(To) == 4) {
            const f4 a = {out[0], out[1], out[2], out[3]};
            *reinterpret_cast<f4*>(q) = a;
          } else {
            const bf4 a = {out[0], out[1], out[2], out[3]};
            *reinterpret_cast<bf4*>(q) = a;
          }
          continue;
        }
      }
      bool done_store = false;
      if constexpr (PREC != PREC_F64) {
        // the four rows of this lane are consecutive
        if ((rows & 3) == 0 && rr[3] < rows) {
          if constexpr (sizeof(To) == 8) {
            const d2 a = {out[0], out[1]}, b2 = {out[2], out[3]};
            *reinterpret_cast<d2*>(dst + rr[0]) = a;
            *reinterpret_cast<d2*>(dst + rr[0] + 2) = b2;
          } else if constexpr (sizeof(To) == 4) {
            const f4 a = {out[0], out[1], out[2], out[3]};
            *reinterpret_cast<f4*>(dst + rr[0]) = a;
          } else {
            const bf4 a = {out[0], out[1], out[2], out[3]};
            *reinterpret_cast<bf4*>(dst + rr[0]) = a;
          }
          done_store = true;
        }
      }
      if (!done_store) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (rr[v] < rows) dst[rr[v]] = out[v];
      }
    }
  }
  if constexpr (STG) {
    if (stage) {
      __syncthreads();
      constexpr int CPC = BR / SE;                  // chunks per column
      const int nvalid = min(CB, K - c0);
      const int r0 = rb * BR;
      for (int c = tid; c < CB * CPC; c += NT) {
        const int col = c / CPC, part = c - col * CPC;
        const int row = r0 + part * SE;
        if (col >= nvalid || row >= rows) continue;   // (rows is a multiple of SE)
        *reinterpret_cast<u4*>(Yb + (int64_t)(c0 + col) * rows + row) =
            *reinterpret_cast<const u4*>(stg + col * BRP + part * SE);
      }
    }
  }
  if (rpart) {
    // fixed-order block reduction: lanes, then waves in order
    __shared__ double fred[NT / 64][2];
    fs[0] = wave_sum(fs[0]);
    fs[1] = wave_sum(fs[1]);
    if (lane == 0) {
      fred[wave][0] = fs[0];
      fred[wave][1] = fs[1];
    }
    __syncthreads();
    if (tid == 0) {
      double t0 = 0.0, t1 = 0.0;
      for (int w = 0; w < NT / 64; ++w) {
        t0 += fred[w][0];
        t1 += fred[w][1];
      }
      const double m = (rscl && st) ? st[rhs].inv_scale * st[rhs].inv_scale : 1.0;
      slot_ptr(rpart, rhs, S_DOT)[blockIdx.x] = t0 * m;
      slot_ptr(rpart, rhs, S_SUM)[blockIdx.x] = 0.0;
      slot_ptr(rpart, rhs, S_SQ)[blockIdx.x] = t1 * m;
      slot_ptr(rpart, rhs, S_AUX2)[blockIdx.x] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Operator-resident variant for short contractions (K <= 128).  The whole
// packed operator of one product (at most 128 KiB) is loaded into LDS once
// per block; the block then sweeps row tiles of 64 rows x 128 columns
// (WR x WC waves, each 16 rows x 16*WN columns) with no further barrier on
// the operator.  A tile's rows are converted to the compute type, then the
// next tile's rows are requested, so their loads overlap this tile's
// products and stores.  Every output is summed over k in the same order as
// in mp_kernel (bitwise the same product).  Spectral partials go to one slot
// per row tile (their number depends on the grid only).  BF16 outputs (the
// HBM-bound products) are staged in LDS as [column][64 rows] and written a
// column's 128 contiguous bytes at a time, 16 bytes a thread, instead of 8
// bytes a lane scattered over 16 columns.
template <int PREC, class Ti, class To, int WN, int WC>
__global__ __launch_bounds__(64 * WR * WC, 1) void mp_res(
    const u4* __restrict__ Bpk, int npk, const Ti* __restrict__ X, To* __restrict__ Y, int K,
    int rows, int64_t N, const RhsState* __restrict__ st, int in_scale, int out_scale,
    const double* __restrict__ la, const double* __restrict__ lb, const double* __restrict__ lc,
    int a1, const double* __restrict__ gt, double* __restrict__ rpart, int rscl) {
  using M = MT<PREC>;
  constexpr int NT = 64 * WR * WC;
  constexpr int CW = 16 * WN;                 // columns per wave
  constexpr int CB = WC * CW;                 // columns per block
  static_assert(CB == 128, "one block covers the operator's 128 columns");
  constexpr int BR = WR * 16;                 // rows per tile
  constexpr int CH = M::CH, NV = M::NV, KB = 4 * CH;
  constexpr int UNITS = 4 * NV * CB;          // 16-byte units per operator k-block
  constexpr int KBMAX = 128 / KB;             // k-blocks of a 128 x 128 operator
  constexpr int JG = group_size(WN, (PREC == PREC_F64 || PREC == PREC_BF16X6) ? 4 : 8);

  const int rhs = blockIdx.y;
  if (st && st[rhs].done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WR, wc = wave / WR;
  const int g = lane >> 4, l16 = lane & 15;
  const int cw = wc * CW;
  const Ti* Xb = X + (int64_t)rhs * N;
  To* Yb = Y + (int64_t)rhs * N;
  const bool scaled = (st != nullptr) && in_scale;
  const double scale = scaled ? st[rhs].scale : 1.0;
  const double oscale = (st && out_scale) ? st[rhs].inv_scale : 1.0;
  const int nkb = (K + KB - 1) / KB;
  const int nrb = (rows + BR - 1) / BR;

  __shared__ u4 lds[KBMAX * UNITS];
  constexpr bool STG = sizeof(To) == 2;
  constexpr int SE = 8, BRP = BR + SE;          // elements per 16-byte chunk; padded column
  __shared__ __attribute__((aligned(16))) To stg[STG ? CB * BRP : 1];
  const bool stage = STG && rows % SE == 0;
  for (int su = tid; su < nkb * UNITS; su += NT) {
    const int kk = su / UNITS, u = su % UNITS, gh = u / CB;
    const int c = min(u % CB, npk - 1);
    lds[su] = Bpk[((int64_t)kk * 4 * NV + gh) * npk + c];
  }

  // this lane's row data of tile rb (rows past the end, and k-blocks past the
  // operator, read valid data that only feeds unused sums)
  XRaw<PREC, Ti> xq[KBMAX];
  int rb = blockIdx.x;
  {
    const int r = rb * BR + wr * 16 + l16;
    const bool ok = r < rows;
    const Ti* xr = Xb + (int64_t)(ok ? r : 0) * K;
#pragma unroll
    for (int d = 0; d < KBMAX; ++d)
      xq[d] = load_raw<PREC, Ti, true>(xr, (ok && d < nkb) ? d * KB + CH * g : K, K);
  }
  __syncthreads();

  for (; rb < nrb; rb += gridDim.x) {
    typename M::chunk xa[KBMAX];
#pragma unroll
    for (int d = 0; d < KBMAX; ++d) xa[d] = cvt_raw<PREC, Ti>(xq[d], scale, scaled);
    {
      // the next tile's rows, while this one is computed
      const int rn = rb + gridDim.x;
      const int r = rn * BR + wr * 16 + l16;
      const bool ok = rn < nrb && r < rows;
      const Ti* xr = Xb + (int64_t)(ok ? r : 0) * K;
#pragma unroll
      for (int d = 0; d < KBMAX; ++d)
        xq[d] = load_raw<PREC, Ti, true>(xr, (ok && d < nkb) ? d * KB + CH * g : K, K);
    }
    typename M::acc acc[WN];
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[j][v] = 0;
#pragma unroll
    for (int kk = 0; kk < KBMAX; ++kk) {
      if (kk < nkb) {
#pragma unroll
        for (int j0 = 0; j0 < WN; j0 += JG) {
          typename M::chunk b[JG];
#pragma unroll
          for (int jj = 0; jj < JG; ++jj)
            b[jj] = load_b<PREC>(lds + kk * UNITS, g, cw + 16 * (j0 + jj) + l16, CB);
#pragma unroll
          for (int s = 0; s < M::STEPS; ++s)
#pragma unroll
            for (int jj = 0; jj < JG; ++jj)
              acc[j0 + jj] = M::mma(xa[kk], b[jj], acc[j0 + jj], s);
        }
      }
    }

    // epilogue: optional G factor and output scale, transposed store
    const int rw = rb * BR + wr * 16;
    double rowsum[4];
    if (lc) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rw + M::row(lane, v);
        const int rc = r < rows ? r : 0;
        rowsum[v] = la[rc % a1] + (lb ? lb[rc / a1] : 0.0);
      }
    }
    double ts[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int n = cw + 16 * j + l16;
      if (n >= K) continue;
      const double lcn = lc ? lc[n] : 0.0;
      To* dst = Yb + (int64_t)n * rows;
      To out[4];
      int rr[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        rr[v] = rw + M::row(lane, v);
        double val = (double)acc[j][v];
        if (lc) {
          const double sum = rowsum[v] + lcn;
          if constexpr (PREC == PREC_F64) {
            val *= ghat(sum);
          } else {
            val = fabs(sum) < 1e-13 ? 0.0 : (double)((float)val * __frcp_rn((float)sum));
          }
        }
        const double rhat = (double)acc[j][v];
        if (gt) val *= gt[(int64_t)n * rows + (rr[v] < rows ? rr[v] : 0)];
        if (out_scale) val *= oscale;
        if constexpr (sizeof(To) == 2) out[v] = (__bf16)(float)val;
        else out[v] = (To)val;
        if (rpart && rr[v] < rows) {
          const double zhat = (double)out[v];
          ts[0] += rhat * zhat;
          ts[1] += zhat * zhat;
        }
      }
      if constexpr (STG) {
        if (stage) {
          // the four rows of this lane are consecutive
          To* q = stg + (cw + 16 * j + l16) * BRP + wr * 16 + M::row(lane, 0);
          *reinterpret_cast<bf4*>(q) = (bf4){out[0], out[1], out[2], out[3]};
          continue;
        }
      }
      bool done_store = false;
      if constexpr (PREC != PREC_F64) {
        if ((rows & 3) == 0 && rr[3] < rows) {
          if constexpr (sizeof(To) == 8) {
            const d2 a = {out[0], out[1]}, b2 = {out[2], out[3]};
            *reinterpret_cast<d2*>(dst + rr[0]) = a;
            *reinterpret_cast<d2*>(dst + rr[0] + 2) = b2;
          } else if constexpr (sizeof(To) == 4) {
            const f4 a = {out[0], out[1], out[2], out[3]};
            *reinterpret_cast<f4*>(dst + rr[0]) = a;
          } else {
            const bf4 a = {out[0], out[1], out[2], out[3]};
            *reinterpret_cast<bf4*>(dst + rr[0]) = a;
          }
          done_store = true;
        }
      }
      if (!done_store) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (rr[v] < rows) dst[rr[v]] = out[v];
      }
    }
    if constexpr (STG) {
      if (stage) {
        __syncthreads();
        constexpr int CPC = BR / SE;            // 16-byte chunks per column
        const int nvalid = min(CB, K);
        for (int c = tid; c < CB * CPC; c += NT) {
          const int col = c / CPC, part = c - col * CPC;
          const int row = rw - wr * 16 + part * SE;   // the tile's first row + 8 part
          if (col >= nvalid || row >= rows) continue;  // (rows is a multiple of SE)
          *reinterpret_cast<u4*>(Yb + (int64_t)col * rows + row) =
              *reinterpret_cast<const u4*>(stg + col * BRP + part * SE);
        }
        __syncthreads();                        // the next tile stages over it
      }
    }
    if (rpart) {
      // this tile's sums, in a fixed order: lanes, then waves in order
      __shared__ double fred[NT / 64][2];
      ts[0] = wave_sum(ts[0]);
      ts[1] = wave_sum(ts[1]);
      if (lane == 0) {
        fred[wave][0] = ts[0];
        fred[wave][1] = ts[1];
      }
      __syncthreads();
      if (tid == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
          t0 += fred[w][0];
          t1 += fred[w][1];
        }
        const double m = (rscl && st) ? st[rhs].inv_scale * st[rhs].inv_scale : 1.0;
        slot_ptr(rpart, rhs, S_DOT)[rb] = t0 * m;
        slot_ptr(rpart, rhs, S_SUM)[rb] = 0.0;
        slot_ptr(rpart, rhs, S_SQ)[rb] = t1 * m;
        slot_ptr(rpart, rhs, S_AUX2)[rb] = 0.0;
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// FP64-accurate products on the int8 matrix cores (PREC_I8X7, PREC_I8X6),
// after the splitting idea of Ozaki et al.: every value is a short sum of
// small integers times powers of two, the integer products are exact on the
// matrix cores, and only their recombination rounds.  S digits per value:
//   S = 7 (I8X7).  Each row r of X (its K values along the contracted axis)
//   gets the power of two 2^e_r with |x| < 2^e_r and is cut into 7 digits,
//       x = 2^e_r sum_i a_i 128^-(i+1),  a_i integers in [-127, 127]
//   (truncation at every step, so all digits carry the sign of x and a
//   small value has small digits; the remainder after the seventh is below
//   2^(e_r - 49)).  Digits of one sign matter here: with two's complement
//   digits a small negative value has large low digits, and the dropped
//   products below would then carry the full 2^-49 scale for every such
//   value.
//   S = 6 (I8X6).  2^e_r with |x| < 2^e_r * 126/128, the image
//   F = trunc(x 2^(47 - e_r)) (|F| < 126 * 2^40) and its balanced base-256
//   digits, low to high with carries,
//       F = sum_i d_i 256^(5-i),  d_i in [-128, 127], |d_0| <= 126,
//   so x = 2^(e_r - 47) sum_i d_i 256^(5-i) up to the truncation (below
//   2^(e_r - 47)).  A small value still has small digits (its high digits
//   are zero), and the digits below a cut take either sign, so the dropped
//   products cancel rather than add.
//   Operator: column n of B likewise with 2^f_n, packed at plan time.
//   Product: the digit products with i + j < S are summed exactly in int32
//   by v_mfma_i32_16x16x64_i8, one accumulator per diagonal d = i + j
//   (|sum| <= 7 * 128^2 * K < 2^31 for K <= 512), and recombined in FP64,
//       y = 2^(e_r + f_n - 14) sum_d base^-d acc_d,  base 128 or 256
//   (for S = 6 the two 2^-47 and the 256^10 of the top diagonal give the
//   same 2^-14).  The error per output is a few units of 2^-49 (S = 7) or
//   2^-48 (S = 6) K max|x_r| max|b_n| at worst, far below what FP64
//   preconditioning needs (one CG iteration).
// The data is read from HBM once and digitised in registers (16 consecutive
// k per lane and k-block of 64); the operator digits stream through LDS one
// column fragment (16 columns) at a time.  Two kernels:
//   mp_oz (K <= 256): blocks of 4 waves x 16 rows, two blocks per CU, the
//     operator fragment double-buffered through registers.
//   mp_ozh (K > 256): the k-blocks split over two waves per row group (their
//     int32 sums added exactly through LDS), blocks of 2 row groups (32 rows,
//     4 waves) so that two blocks share a CU and one block's data loads,
//     operator refill and epilogue overlap the other's matrix-core work; the
//     operator fragment single-buffered and refilled straight from memory
//     into LDS (no registers) while the finishing wave runs the epilogue.
// Both need K % 16 == 0 and rows % 16 == 0 (every extent of an int8 split
// plan is a multiple of 16).  A row with a non-finite value yields NaN
// outputs.
// ---------------------------------------------------------------------------
constexpr int OZ_SMAX = 7;            // most digits per value
constexpr int OZ_KMAX = 512;          // longest axis the int8 splits serve (plan check)
constexpr int OZ_BAD = 0x40000000;    // exponent marker of a non-finite row

static int oz_split(int K) { return K > 256 ? 2 : 1; }
static int oz_kb_per_wave(int K) {
  const int nkb = (K + 63) / 64, ks = oz_split(K);
  return (nkb + ks - 1) / ks;
}
// bytes of the operator digits: column fragments x padded k-blocks x S digits
// x 64 lanes x 16 bytes; the column exponents (int32) follow
static size_t oz_digit_bytes(int K, int S) {
  return (size_t)((K + 15) / 16) * oz_split(K) * oz_kb_per_wave(K) * S * 64 * 16;
}

// The lane's 16 consecutive values of each of its KBW k-blocks (from kb0)
// of one row, read once, with their largest magnitude and whether any is not
// finite.  k-blocks past K (padding of the split) read as zeros.  Every load
// is issued unconditionally (a padding k-block reads the row's first values,
// then zeroed) and before any is used, so that all are in flight at once.
template <int KBW>
__device__ __forceinline__ void oz_load(const double* xr, int kb0, int K, int g,
                                        d2 (&raw)[KBW][8], double& mx, int& bad) {
#pragma unroll
  for (int kb = 0; kb < KBW; ++kb) {
    // a block past K reads the row's first 16 values (K >= 16), zeroed below
    const int k0 = (kb0 + kb) * 64 + 16 * g;
    const double* src = xr + (k0 < K ? k0 : 0);
#pragma unroll
    for (int q = 0; q < 8; ++q) raw[kb][q] = *reinterpret_cast<const d2*>(src + 2 * q);
  }
  mx = 0.0;
  bad = 0;
#pragma unroll
  for (int kb = 0; kb < KBW; ++kb) {
    const bool in = (kb0 + kb) * 64 + 16 * g < K;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (!in) raw[kb][q] = (d2){0.0, 0.0};
      const double a = fabs(raw[kb][q].x), b = fabs(raw[kb][q].y);
      bad |= !(a <= DBL_MAX) | !(b <= DBL_MAX);
      mx = fmax(mx, fmax(a, b));
    }
  }
}

// oz_load in two halves, for a kernel that loads the next rows early: the
// loads (issued together) and, once they are used, the masking of k past K
// with the row's largest magnitude and finiteness.
template <int KBW>
__device__ __forceinline__ void oz_issue(const double* xr, int K, int g, d2 (&raw)[KBW][8]) {
#pragma unroll
  for (int kb = 0; kb < KBW; ++kb) {
    const int k0 = kb * 64 + 16 * g;
    const double* src = xr + (k0 < K ? k0 : 0);
#pragma unroll
    for (int q = 0; q < 8; ++q) raw[kb][q] = *reinterpret_cast<const d2*>(src + 2 * q);
  }
}
template <int KBW>
__device__ __forceinline__ void oz_scan(int K, int g, d2 (&raw)[KBW][8], double& mx, int& bad) {
  mx = 0.0;
  bad = 0;
#pragma unroll
  for (int kb = 0; kb < KBW; ++kb) {
    const bool in = kb * 64 + 16 * g < K;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (!in) raw[kb][q] = (d2){0.0, 0.0};
      const double a = fabs(raw[kb][q].x), b = fabs(raw[kb][q].y);
      bad |= !(a <= DBL_MAX) | !(b <= DBL_MAX);
      mx = fmax(mx, fmax(a, b));
    }
  }
}

// The row's exponent e from its largest magnitude: |x| < 2^e (S = 7), and
// |x| < 2^e * 126/128 for the balanced split (S = 6), whose top digit must
// stay below 127 after the carries.
template <int S>
__device__ __forceinline__ int oz_exponent(double mx) {
  int e = 0;
  if (mx > 0.0) {
    const double m = frexp(mx, &e);
    if (S == 6 && m >= 0.984375) ++e;
  }
  return max(e, -1021);                         // images of subnormal rows fit too
}

// The right shift of the 53-bit significand that gives a value's image,
// plus the biased exponent field: 49 - e bits (S = 7) or 47 - e (S = 6)
// below the binary point.
template <int S>
__device__ __forceinline__ int oz_cshift(int e) { return e + (S == 7 ? 1026 : 1028); }

// Digits from the bit pattern: the image F = floor(|x| 2^(49 - e)) < 2^49 is
// the 53-bit significand shifted right by e + 1026 - max(ef, 1) >= 4 (ef the
// biased exponent field; cshift = e + 1026, or past 63 for a non-finite row,
// which shifts everything out); its 7-bit fields from the top are the digit
// magnitudes, which take the sign of x (negated two values at a time on
// 16-bit halves).  These are the digits of truncating |x| 2^-e one base-128
// place at a time.  xa[kb][s] holds digit s of the lane's 16 values of
// k-block kb, four to a dword.
template <int KBW>
__device__ __forceinline__ void oz_digits7(const d2 (&raw)[KBW][8], int cshift,
                                           v4i (&xa)[KBW][OZ_SMAX]) {
#pragma unroll
  for (int kb = 0; kb < KBW; ++kb)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      unsigned u[7][4], sg[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const d2 pr = raw[kb][2 * w + (c >> 1)];
        const uint64_t bits = (uint64_t)__double_as_longlong((c & 1) ? pr.y : pr.x);
        const unsigned hi = (unsigned)(bits >> 32);
        const unsigned ef = (hi >> 20) & 0x7ffu;
        const unsigned sh = (unsigned)min(cshift - (int)max(ef, 1u), 63);
        const uint64_t sig = ((uint64_t)((hi & 0xfffffu) | (min(ef, 1u) << 20)) << 32) |
                             (bits & 0xffffffffull);
        const uint64_t F = sig >> sh;
        const unsigned fh = (unsigned)(F >> 32), fl = (unsigned)F;
        sg[c] = (unsigned)((int)hi >> 31);      // 0 or all ones
        u[0][c] = fh >> 10;
        u[1][c] = (fh >> 3) & 127u;
        u[2][c] = ((fh << 4) | (fl >> 28)) & 127u;
        u[3][c] = (fl >> 21) & 127u;
        u[4][c] = (fl >> 14) & 127u;
        u[5][c] = (fl >> 7) & 127u;
        u[6][c] = fl & 127u;
      }
      const unsigned m01 = (sg[0] & 0xffffu) | (sg[1] & 0xffff0000u);
      const unsigned m23 = (sg[2] & 0xffffu) | (sg[3] & 0xffff0000u);
#pragma unroll
      for (int s = 0; s < 7; ++s) {
        // (d ^ m) - m on each 16-bit half negates where m is all ones; the
        // low bytes of the four signed digits then make one dword
        const u16x2 p01 = __builtin_bit_cast(u16x2, (u[s][0] | (u[s][1] << 16)) ^ m01) -
                          __builtin_bit_cast(u16x2, m01);
        const u16x2 p23 = __builtin_bit_cast(u16x2, (u[s][2] | (u[s][3] << 16)) ^ m23) -
                          __builtin_bit_cast(u16x2, m23);
        xa[kb][s][w] = (int)__builtin_amdgcn_perm(__builtin_bit_cast(unsigned, p23),
                                                  __builtin_bit_cast(unsigned, p01), 0x06040200u);
      }
    }
}

// Balanced digits (S = 6) from the same kind of image, F = floor(|x|
// 2^(47 - e)) (the significand shifted right by cshift - max(ef, 1) >= 6),
// signed.  Adding 128 to each of its five low bytes in one 64-bit add,
// G = F + 0x8080808080, turns every low digit d into the byte d + 128 (the
// digits in [-128, 127] of an integer are unique, and d + 128 is its byte of
// G), so XOR 0x80 gives the two's complement digit, four at a time; the top
// digit is G >> 40 (arithmetic), at most 126 in magnitude.  A 4 x 4 byte
// transpose (v_perm_b32) then gathers digit s of the lane's four values.
template <int KBW>
__device__ __forceinline__ void oz_digits6(const d2 (&raw)[KBW][8], int cshift,
                                           v4i (&xa)[KBW][OZ_SMAX]) {
#pragma unroll
  for (int kb = 0; kb < KBW; ++kb)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      unsigned lo[4], hi[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const d2 pr = raw[kb][2 * w + (c >> 1)];
        const uint64_t bits = (uint64_t)__double_as_longlong((c & 1) ? pr.y : pr.x);
        const unsigned h = (unsigned)(bits >> 32);
        const unsigned ef = (h >> 20) & 0x7ffu;
        const unsigned sh = (unsigned)min(cshift - (int)max(ef, 1u), 63);
        const uint64_t sig = ((uint64_t)((h & 0xfffffu) | (min(ef, 1u) << 20)) << 32) |
                             (bits & 0xffffffffull);
        const uint64_t F = sig >> sh;
        const uint64_t m = (uint64_t)(int64_t)((int)h >> 31);   // 0 or all ones
        const uint64_t G = ((F ^ m) - m) + 0x8080808080ull;
        lo[c] = (unsigned)G ^ 0x80808080u;      // digits 5, 4, 3, 2 (bytes 0..3)
        hi[c] = (unsigned)(G >> 32);            // byte 0: digit 1 + 128, byte 1: digit 0
      }
      // byte k of value c -> byte c of dword k (two rounds of byte pairs)
      const unsigned l01a = __builtin_amdgcn_perm(lo[1], lo[0], 0x05010400u);
      const unsigned l01b = __builtin_amdgcn_perm(lo[1], lo[0], 0x07030602u);
      const unsigned l23a = __builtin_amdgcn_perm(lo[3], lo[2], 0x05010400u);
      const unsigned l23b = __builtin_amdgcn_perm(lo[3], lo[2], 0x07030602u);
      xa[kb][5][w] = (int)__builtin_amdgcn_perm(l23a, l01a, 0x05040100u);
      xa[kb][4][w] = (int)__builtin_amdgcn_perm(l23a, l01a, 0x07060302u);
      xa[kb][3][w] = (int)__builtin_amdgcn_perm(l23b, l01b, 0x05040100u);
      xa[kb][2][w] = (int)__builtin_amdgcn_perm(l23b, l01b, 0x07060302u);
      const unsigned h01 = __builtin_amdgcn_perm(hi[1], hi[0], 0x05010400u);
      const unsigned h23 = __builtin_amdgcn_perm(hi[3], hi[2], 0x05010400u);
      xa[kb][1][w] = (int)(__builtin_amdgcn_perm(h23, h01, 0x05040100u) ^ 0x80808080u);
      xa[kb][0][w] = (int)__builtin_amdgcn_perm(h23, h01, 0x07060302u);
    }
}

template <int KBW, int S>
__device__ __forceinline__ void oz_digits(const d2 (&raw)[KBW][8], int cshift,
                                          v4i (&xa)[KBW][OZ_SMAX]) {
  if constexpr (S == 7) oz_digits7<KBW>(raw, cshift, xa);
  else oz_digits6<KBW>(raw, cshift, xa);
}

// The digit products of k-block kb into the diagonal sums acc[d], d = i + s,
// for i + s < S; consecutive products update different diagonals.
template <int S>
__device__ __forceinline__ void oz_products(const v4i (&a)[OZ_SMAX], const v4i (&b)[OZ_SMAX],
                                            v4i (&acc)[OZ_SMAX]) {
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int s = 0; s + i < S; ++s)
      acc[i + s] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[s], acc[i + s], 0, 0, 0);
}

// 16 bytes a lane from global memory into LDS at the wave-uniform address
// lds_addr + 16 lane (global_load_lds_dwordx4), no registers written.  The
// caller waits for it (vmcnt) before any wave reads that LDS.
// m0 is named as clobbered; no other code in these kernels keeps a value in it.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void oz_dma16(const u4* src, unsigned lds_addr) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
               :: "v"(src), "s"(lds_addr) : "memory", "m0");
}
#pragma clang diagnostic pop

// The S operator digit fragments of one k-block from LDS (16 bytes a lane).
template <int S>
__device__ __forceinline__ void oz_ldsb(const u4* lds, int at, v4i (&b)[OZ_SMAX]) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const u4 u = lds[at + s * 64];
    b[s] = (v4i){(int)u.x, (int)u.y, (int)u.z, (int)u.w};
  }
}

// The products of KBW consecutive k-blocks whose operator digits sit in LDS
// at at[(kb S + s) 64] (at: the first k-block, offset by the lane): each
// k-block's digits are read while the k-block before it is multiplied (two
// register sets, alternating), the reads spread over the first products.
template <int KBW, int S>
__device__ __forceinline__ void oz_kloop(const u4* at, const v4i (&xa)[KBW][OZ_SMAX],
                                         v4i (&acc)[OZ_SMAX]) {
  v4i b[2][OZ_SMAX];
  oz_ldsb<S>(at, 0, b[0]);
#pragma unroll
  for (int kb = 0; kb < KBW; ++kb) {
    if (kb + 1 < KBW) oz_ldsb<S>(at, (kb + 1) * S * 64, b[(kb + 1) & 1]);
    oz_products<S>(xa[kb], b[kb & 1], acc);
  }
  __builtin_amdgcn_sched_group_barrier(0x100, S, 0);     // DS reads
#pragma unroll
  for (int kb = 0; kb + 1 < KBW; ++kb) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // matrix-core ops
    }
    __builtin_amdgcn_sched_group_barrier(0x008, S * (S + 1) / 2 - 2 * S, 0);
  }
  __builtin_amdgcn_sched_group_barrier(0x008, S * (S + 1) / 2, 0);
}

// Ghat for the int8 split epilogues: the hardware reciprocal estimate and two
// Newton steps r <- r + r (1 - s r), each squaring the relative error, reach
// FP64 accuracy (within an ulp of 1/s) without the IEEE division sequence.
__device__ __forceinline__ double ghat_fast(double s) {
  double r = __builtin_amdgcn_rcp(s);
  double e = fma(-s, r, 1.0);
  r = fma(r, e, r);
  e = fma(-s, r, 1.0);
  r = fma(r, e, r);
  return fabs(s) < 1e-13 ? 0.0 : r;
}

// One output from its exact diagonal sums a[d]: sum_d base^-d a[d] (Horner,
// low diagonals first; base 128 for S = 7, 256 for S = 6), scaled by
// 2^(e + f - 14); NaN for a non-finite row.
template <int S>
__device__ __forceinline__ double oz_value(const int (&a)[OZ_SMAX], int e, int f) {
  constexpr double inv = S == 7 ? 1.0 / 128.0 : 1.0 / 256.0;
  double val = (double)a[S - 1];
#pragma unroll
  for (int d = S - 2; d >= 0; --d) val = (double)a[d] + val * inv;
  return e == OZ_BAD ? NAN : ldexp(val, e + f - 14);
}

// This lane's sums of its input values (rows past the end count nothing;
// k past the operator was loaded as 0), reduced over the wave; lane 0 leaves
// them in red[wave].  The block adds red over its waves in order.
template <int KBW>
__device__ __forceinline__ void oz_input_sums(const d2 (&raw)[KBW][8], bool row_ok, int lane,
                                              int wave, double (*red)[2]) {
  double s1 = 0.0, s2 = 0.0;
  if (row_ok) {
#pragma unroll
    for (int kb = 0; kb < KBW; ++kb)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        s1 += raw[kb][q].x + raw[kb][q].y;
        s2 += raw[kb][q].x * raw[kb][q].x + raw[kb][q].y * raw[kb][q].y;
      }
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    red[wave][0] = s1;
    red[wave][1] = s2;
  }
}

// The block's input sums (after a barrier that follows oz_input_sums) to the
// sum and sum-of-squares slots, in wave order.
template <int NW>
__device__ __forceinline__ void oz_input_store(const double (*red)[2], double* part, int rhs) {
  double t0 = 0.0, t1 = 0.0;
  for (int w = 0; w < NW; ++w) {
    t0 += red[w][0];
    t1 += red[w][1];
  }
  slot_ptr(part, rhs, S_SUM)[blockIdx.x] = t0;
  slot_ptr(part, rhs, S_SQ)[blockIdx.x] = t1;
}

// rpart: with the Ghat epilogue (lc), the spectral <R, Z> and ||Z||^2; in a
// plain product (no lc, no gt), the sum and the sum of squares of X's
// entries, one partial per block (a nonsingular right-hand side's ||eta||^2
// when the product is the solve's first and X is eta).
template <int KBW, int KS, int S>
__global__ __launch_bounds__(256 * KS, 2 / KS) void mp_oz(
    const u4* __restrict__ Bpk, const int* __restrict__ fexp, const double* __restrict__ X,
    double* __restrict__ Y, int K, int rows, int64_t N, const RhsState* __restrict__ st,
    const double* __restrict__ la, const double* __restrict__ lb, const double* __restrict__ lc,
    int a1, const double* __restrict__ gt, double* __restrict__ rpart) {
  constexpr int NT = 256 * KS;
  constexpr int SU = KS * KBW * S * 64;      // 16-byte units per column fragment
  constexpr int UPT = (SU + NT - 1) / NT;
  __shared__ u4 lds[2][SU];
  __shared__ double hmax[KS][4][16];
  __shared__ v4i xch[KS == 2 ? 4 : 1][S][64];
  __shared__ double fred[NT / 64][2];
  __shared__ int sfx[OZ_KMAX];                  // the column exponents and eigenvalues
  __shared__ double slc[OZ_KMAX];               // of the epilogue, read once

  const int rhs = blockIdx.y;
  if (st && st[rhs].done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int wr = wave & 3, h = wave >> 2;       // row group, k half
  const int r0 = blockIdx.x * 64 + wr * 16;
  const int r = r0 + l16;
  const double* xr = X + (int64_t)rhs * N + (int64_t)(r < rows ? r : 0) * K;
  const int kb0 = h * KBW;

  // the lane's values, read once; the row's maximum and finiteness
  d2 raw[KBW][8];
  double mx;
  int bad;
  oz_load<KBW>(xr, kb0, K, g, raw, mx, bad);
  const bool insum = rpart && !lc && !gt;
  if (insum) oz_input_sums<KBW>(raw, r < rows, lane, wave, fred);
  mx = fmax(mx, __shfl_xor(mx, 16, 64));
  mx = fmax(mx, __shfl_xor(mx, 32, 64));
  bad |= __shfl_xor(bad, 16, 64);
  bad |= __shfl_xor(bad, 32, 64);
  if constexpr (KS == 2) {
    if (g == 0) hmax[h][wr][l16] = bad ? INFINITY : mx;
    __syncthreads();
    const double o = hmax[h ^ 1][wr][l16];
    bad |= !(o <= DBL_MAX);
    mx = fmax(mx, o);
  }
  const int e = oz_exponent<S>(mx);
  v4i xa[KBW][OZ_SMAX];
  oz_digits<KBW, S>(raw, bad ? 4096 : oz_cshift<S>(e), xa);
  // exponents of this lane's output rows 4g + v (held by lane 4g + v)
  const int eo = bad ? OZ_BAD : e;
  int erow[4];
  double rowsum[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    erow[v] = __shfl(eo, 4 * g + v, 64);
    const int rr = r0 + 4 * g + v, rc = rr < rows ? rr : 0;
    rowsum[v] = lc ? la[rc % a1] + (lb ? lb[rc / a1] : 0.0) : 0.0;
  }

  const int nfr = (K + 15) / 16;
  u4 breg[UPT];
#pragma unroll
  for (int q = 0; q < UPT; ++q) breg[q] = Bpk[min(tid + q * NT, SU - 1)];
#pragma unroll
  for (int q = 0; q < UPT; ++q) lds[0][min(tid + q * NT, SU - 1)] = breg[q];
  for (int i = tid; i < K; i += NT) {
    sfx[i] = fexp[i];
    if (lc) slc[i] = lc[i];
  }
  __syncthreads();
  if (insum && tid == 0) oz_input_store<NT / 64>(fred, rpart, rhs);

  double* Yb = Y + (int64_t)rhs * N;
  double fs[2] = {0.0, 0.0};                   // spectral <R, Z> and ||Z||^2
  for (int j = 0; j < nfr; ++j) {
    const int buf = j & 1;
    const int64_t nxt = (int64_t)min(j + 1, nfr - 1) * SU;   // past the last: a reload
#pragma unroll
    for (int q = 0; q < UPT; ++q) breg[q] = Bpk[nxt + min(tid + q * NT, SU - 1)];
    v4i acc[OZ_SMAX];
#pragma unroll
    for (int d = 0; d < S; ++d) acc[d] = (v4i){0, 0, 0, 0};
    oz_kloop<KBW, S>(lds[buf] + kb0 * S * 64 + lane, xa, acc);
    if constexpr (KS == 2) {
      if (h == 1) {
#pragma unroll
        for (int d = 0; d < S; ++d) xch[wr][d][lane] = acc[d];
      }
      __syncthreads();
      if (h == 0) {
#pragma unroll
        for (int d = 0; d < S; ++d) acc[d] += xch[wr][d][lane];
      }
    }
    const int n = 16 * j + l16;
    if (h == 0 && n < K) {
      const int f = sfx[n];
      const double lcn = lc ? slc[n] : 0.0;
      double out[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = r0 + 4 * g + v;
        int a[OZ_SMAX];
#pragma unroll
        for (int d = 0; d < S; ++d) a[d] = acc[d][v];
        double val = oz_value<S>(a, erow[v], f);
        const double rhat = val;
        if (lc) val *= ghat_fast(rowsum[v] + lcn);
        if (gt) val *= gt[(int64_t)n * rows + (rr < rows ? rr : 0)];
        if (rpart && rr < rows) {
          fs[0] += rhat * val;
          fs[1] += val * val;
        }
        out[v] = val;
      }
      double* dst = Yb + (int64_t)n * rows + r0 + 4 * g;
      if ((rows & 1) == 0 && r0 + 4 * g + 3 < rows) {
        *reinterpret_cast<d2*>(dst) = (d2){out[0], out[1]};
        *reinterpret_cast<d2*>(dst + 2) = (d2){out[2], out[3]};
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (r0 + 4 * g + v < rows) dst[v] = out[v];
      }
    }
#pragma unroll
    for (int q = 0; q < UPT; ++q) lds[buf ^ 1][min(tid + q * NT, SU - 1)] = breg[q];
    __syncthreads();
  }
  if (lc && rpart) {
    // fixed-order block reduction: lanes, then waves in order
    fs[0] = wave_sum(fs[0]);
    fs[1] = wave_sum(fs[1]);
    if (lane == 0) {
      fred[wave][0] = fs[0];
      fred[wave][1] = fs[1];
    }
    __syncthreads();
    if (tid == 0) {
      double t0 = 0.0, t1 = 0.0;
      for (int w = 0; w < NT / 64; ++w) {
        t0 += fred[w][0];
        t1 += fred[w][1];
      }
      slot_ptr(rpart, rhs, S_DOT)[blockIdx.x] = t0;
      slot_ptr(rpart, rhs, S_SUM)[blockIdx.x] = 0.0;
      slot_ptr(rpart, rhs, S_SQ)[blockIdx.x] = t1;
      slot_ptr(rpart, rhs, S_AUX2)[blockIdx.x] = 0.0;
    }
  }
}

// K > 256: 32 rows per block (row group wr = wave & 1, k half h = wave >> 1).
// EPI: 0 plain (rpart, when given, takes the sum and the sum of squares of
// X's entries, as in mp_oz), 1 the Hadamard factor Ghat from the eigenvalue
// sums (la, lb over the rows, lc over the columns; rpart, when given, takes
// the spectral <R, Z> and ||Z||^2), 2 the Hadamard factor from the table
// gt [K][rows].
// The k half (j & 1) finishes fragment j, the other hands it its sums.
template <int KBW, int EPI, int S>
__global__ __launch_bounds__(256, 2) void mp_ozh(
    const u4* __restrict__ Bpk, const int* __restrict__ fexp, const double* __restrict__ X,
    double* __restrict__ Y, int K, int rows, int64_t N, const RhsState* __restrict__ st,
    const double* __restrict__ la, const double* __restrict__ lb, const double* __restrict__ lc,
    int a1, const double* __restrict__ gt, double* __restrict__ rpart) {
  constexpr int NT = 256;
  constexpr int SU = 2 * KBW * S * 64;       // 16-byte units per column fragment
  constexpr int UPT = (SU + NT - 1) / NT;
  __shared__ u4 lds[SU];
  __shared__ double hmax[2][2][16];
  __shared__ v4i xch[2][S][64];
  __shared__ double fred[NT / 64][2];
  __shared__ int sfx[OZ_KMAX];                  // the column exponents and eigenvalues
  __shared__ double slc[EPI == 1 ? OZ_KMAX : 1];  // of the epilogue, read once

  const int rhs = blockIdx.y;
  if (st && st[rhs].done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int wr = wave & 1, h = wave >> 1;
  const int r0 = blockIdx.x * 32 + wr * 16;
  const int r = r0 + l16;
  const double* xr = X + (int64_t)rhs * N + (int64_t)(r < rows ? r : 0) * K;
  const int kb0 = h * KBW;
  const int nfr = K / 16;

  // operator digits of fragment j into LDS without registers: each wave moves
  // 64 consecutive 16-byte units (the builtin writes lane l's 16 bytes at the
  // wave-uniform LDS address + 16 l), so a wave's chunk lies wholly inside or
  // wholly past the fragment
  // (issued from asm, which the compiler does not track: every wait for these
  // loads is explicit below, so that none also waits for the output stores)
  auto stage = [&](int j) {
    const u4* src = Bpk + (int64_t)j * SU;
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      const int u0 = (tid & ~63) + q * NT;
      if (u0 < SU)
        oz_dma16(src + u0 + lane, __builtin_amdgcn_readfirstlane(
            (unsigned)(uintptr_t)(__attribute__((address_space(3))) u4*)&lds[u0]));
    }
  };
  stage(0);                                     // in flight while the data loads

  d2 raw[KBW][8];
  double mx;
  int bad;
  oz_load<KBW>(xr, kb0, K, g, raw, mx, bad);
  const bool insum = EPI == 0 && rpart;
  if (insum) oz_input_sums<KBW>(raw, r < rows, lane, wave, fred);
  mx = fmax(mx, __shfl_xor(mx, 16, 64));
  mx = fmax(mx, __shfl_xor(mx, 32, 64));
  bad |= __shfl_xor(bad, 16, 64);
  bad |= __shfl_xor(bad, 32, 64);
  if (g == 0) hmax[h][wr][l16] = bad ? INFINITY : mx;
  __syncthreads();
  if (insum && tid == 0) oz_input_store<NT / 64>(fred, rpart, rhs);
  {
    const double o = hmax[h ^ 1][wr][l16];
    bad |= !(o <= DBL_MAX);
    mx = fmax(mx, o);
  }
  const int e = oz_exponent<S>(mx);
  v4i xa[KBW][OZ_SMAX];
  oz_digits<KBW, S>(raw, bad ? 4096 : oz_cshift<S>(e), xa);
  const int eo = bad ? OZ_BAD : e;
  int erow[4];
  double rowsum[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    erow[v] = __shfl(eo, 4 * g + v, 64);
    const int rr = r0 + 4 * g + v, rc = rr < rows ? rr : 0;
    rowsum[v] = EPI == 1 ? la[rc % a1] + (lb ? lb[rc / a1] : 0.0) : 0.0;
  }
  for (int i = tid; i < K; i += NT) {
    sfx[i] = fexp[i];
    if constexpr (EPI == 1) slc[i] = lc[i];
  }
  __builtin_amdgcn_s_waitcnt(0);                // the first fragment has landed
  __syncthreads();

  double* Yb = Y + (int64_t)rhs * N;
  const bool rows_ok = r0 < rows;               // the row group lies inside (rows % 16 == 0)
  double fs0 = 0.0, fs1 = 0.0;                  // spectral <R, Z> and ||Z||^2
  // Ghat of this lane's four outputs in the next fragment the wave finishes:
  // a wave computes them while the other k half finishes the fragment
  // between (fragment 0: here)
  double gn[4] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (EPI == 1) {
    if (h == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) gn[v] = ghat_fast(rowsum[v] + slc[l16]);
    }
  }
  for (int j = 0; j < nfr; ++j) {
    const int n = 16 * j + l16;
    v4i acc[OZ_SMAX];
#pragma unroll
    for (int d = 0; d < S; ++d) acc[d] = (v4i){0, 0, 0, 0};
    oz_kloop<KBW, S>(lds + kb0 * S * 64 + lane, xa, acc);
    const int fh = j & 1;
    if (h != fh) {
#pragma unroll
      for (int d = 0; d < S; ++d) xch[wr][d][lane] = acc[d];
    }
    __syncthreads();                            // the fragment's digits are consumed
    if (j + 1 < nfr) stage(j + 1);
    if constexpr (EPI == 1) {
      if (h != fh && j + 1 < nfr) {
        const double lcn = slc[16 * (j + 1) + l16];
#pragma unroll
        for (int v = 0; v < 4; ++v) gn[v] = ghat_fast(rowsum[v] + lcn);
      }
    }
    if (h == fh) {
      const int f = sfx[n];
      double gv[4] = {0.0, 0.0, 0.0, 0.0};
      if constexpr (EPI == 2) {
        const d2* src =
            reinterpret_cast<const d2*>(gt + (int64_t)n * rows + (rows_ok ? r0 + 4 * g : 0));
        const d2 t0 = src[0], t1 = src[1];
        gv[0] = t0.x; gv[1] = t0.y; gv[2] = t1.x; gv[3] = t1.y;
      }
#pragma unroll
      for (int d = 0; d < S; ++d) acc[d] += xch[wr][d][lane];
      double out[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int a[OZ_SMAX];
#pragma unroll
        for (int d = 0; d < S; ++d) a[d] = acc[d][v];
        double val = oz_value<S>(a, erow[v], f);
        const double rhat = val;
        if constexpr (EPI == 1) {
          val *= gn[v];
          fs0 += rows_ok ? rhat * val : 0.0;
          fs1 += rows_ok ? val * val : 0.0;
        }
        if constexpr (EPI == 2) val *= gv[v];
        out[v] = val;
      }
      if (rows_ok) {
        double* dst = Yb + (int64_t)n * rows + r0 + 4 * g;
        *reinterpret_cast<d2*>(dst) = (d2){out[0], out[1]};
        *reinterpret_cast<d2*>(dst + 2) = (d2){out[2], out[3]};
      }
    }
    // the next fragment has landed.  Vector memory operations complete in
    // issue order, and a finishing wave's two output stores (one 16-byte
    // store each) come after its loads of the next fragment, so that wave
    // waits until at most those two are outstanding: the stores need not
    // reach memory before the barrier.
    // (__syncthreads() would wait for the stores as well: its fence orders
    // the loads into LDS by waiting for every vector memory operation.)
    if (__builtin_amdgcn_readfirstlane(h == fh && rows_ok))
      asm volatile("s_waitcnt vmcnt(2) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else
      asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  }
  if (EPI == 1 && rpart) {
    // fixed-order block reduction: lanes, then waves in order
    fs0 = wave_sum(fs0);
    fs1 = wave_sum(fs1);
    if (lane == 0) {
      fred[wave][0] = fs0;
      fred[wave][1] = fs1;
    }
    __syncthreads();
    if (tid == 0) {
      double t0 = 0.0, t1 = 0.0;
      for (int w = 0; w < NT / 64; ++w) {
        t0 += fred[w][0];
        t1 += fred[w][1];
      }
      slot_ptr(rpart, rhs, S_DOT)[blockIdx.x] = t0;
      slot_ptr(rpart, rhs, S_SUM)[blockIdx.x] = 0.0;
      slot_ptr(rpart, rhs, S_SQ)[blockIdx.x] = t1;
      slot_ptr(rpart, rhs, S_AUX2)[blockIdx.x] = 0.0;
    }
  }
}

// K <= 128: the operator's digits, every column fragment, stay in LDS (at
// most 112 KiB) and the block sweeps 128-row tiles, eight waves of 16 rows
// with all of K each, so that no wave waits for another inside the sweep;
// the next tile's rows are loaded while the current tile is multiplied.
// Products, recombination and epilogues are those of mp_oz (bitwise the same
// outputs).  EPI as in mp_ozh.  rpart: one partial per wave and row tile
// (slot 8 t + wave), the spectral sums (EPI 1) or the sum and sum of squares
// of X's entries (EPI 0).
template <int KBW, int EPI, int S>
__global__ __launch_bounds__(512, 1) void mp_ozr(
    const u4* __restrict__ Bpk, const int* __restrict__ fexp, const double* __restrict__ X,
    double* __restrict__ Y, int K, int rows, int64_t N, const RhsState* __restrict__ st,
    const double* __restrict__ la, const double* __restrict__ lb, const double* __restrict__ lc,
    int a1, const double* __restrict__ gt, double* __restrict__ rpart) {
  constexpr int NT = 512, NW = NT / 64, BR = 16 * NW;
  constexpr int FU = KBW * S * 64;              // 16-byte units per column fragment
  constexpr int KM = 64 * KBW;                  // longest K of this instance
  __shared__ u4 lds[(KM / 16) * FU];
  __shared__ int sfx[KM];
  __shared__ double slc[EPI == 1 ? KM : 1];

  const int rhs = blockIdx.y;
  if (st && st[rhs].done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int nfr = K / 16;                       // K is a multiple of 16 here
  const int nrb = (rows + BR - 1) / BR;
  const double* Xb = X + (int64_t)rhs * N;
  double* Yb = Y + (int64_t)rhs * N;
  for (int u = tid; u < nfr * FU; u += NT) lds[u] = Bpk[u];
  for (int i = tid; i < K; i += NT) {
    sfx[i] = fexp[i];
    if constexpr (EPI == 1) slc[i] = lc[i];
  }
  // this lane's row of tile t (rows past the end read row 0, unused)
  auto row_src = [&](int t) {
    const int r = t * BR + wave * 16 + l16;
    return Xb + (int64_t)((t < nrb && r < rows) ? r : 0) * K;
  };
  d2 raw[KBW][8];
  oz_issue<KBW>(row_src(blockIdx.x), K, g, raw);
  __syncthreads();

  for (int t = blockIdx.x; t < nrb; t += gridDim.x) {
    const int r0 = t * BR + wave * 16;
    const bool row_ok = r0 + l16 < rows;
    double mx;
    int bad;
    oz_scan<KBW>(K, g, raw, mx, bad);
    double s0 = 0.0, s1 = 0.0;                  // input sums (EPI 0) or spectral (EPI 1)
    if (EPI == 0 && rpart && row_ok) {
#pragma unroll
      for (int kb = 0; kb < KBW; ++kb)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          s0 += raw[kb][q].x + raw[kb][q].y;
          s1 += raw[kb][q].x * raw[kb][q].x + raw[kb][q].y * raw[kb][q].y;
        }
    }
    mx = fmax(mx, __shfl_xor(mx, 16, 64));
    mx = fmax(mx, __shfl_xor(mx, 32, 64));
    bad |= __shfl_xor(bad, 16, 64);
    bad |= __shfl_xor(bad, 32, 64);
    const int e = oz_exponent<S>(mx);
    v4i xa[KBW][OZ_SMAX];
    oz_digits<KBW, S>(raw, bad ? 4096 : oz_cshift<S>(e), xa);
    const int eo = bad ? OZ_BAD : e;
    int erow[4];
    double rowsum[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      erow[v] = __shfl(eo, 4 * g + v, 64);
      const int rr = r0 + 4 * g + v, rc = rr < rows ? rr : 0;
      rowsum[v] = EPI == 1 ? la[rc % a1] + (lb ? lb[rc / a1] : 0.0) : 0.0;
    }
    // the next tile's rows, while this one is multiplied
    oz_issue<KBW>(row_src(t + gridDim.x), K, g, raw);

    for (int j = 0; j < nfr; ++j) {
      v4i acc[OZ_SMAX];
#pragma unroll
      for (int d = 0; d < S; ++d) acc[d] = (v4i){0, 0, 0, 0};
      oz_kloop<KBW, S>(lds + j * KBW * S * 64 + lane, xa, acc);
      const int n = 16 * j + l16;
      const int f = sfx[n];
      const double lcn = EPI == 1 ? slc[n] : 0.0;
      double out[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = r0 + 4 * g + v;
        int a[OZ_SMAX];
#pragma unroll
        for (int d = 0; d < S; ++d) a[d] = acc[d][v];
        double val = oz_value<S>(a, erow[v], f);
        const double rhat = val;
        if constexpr (EPI == 1) {
          val *= ghat_fast(rowsum[v] + lcn);
          if (rr < rows) {
            s0 += rhat * val;
            s1 += val * val;
          }
        }
        if constexpr (EPI == 2) val *= gt[(int64_t)n * rows + (rr < rows ? rr : 0)];
        out[v] = val;
      }
      double* dst = Yb + (int64_t)n * rows + r0 + 4 * g;
      if ((rows & 1) == 0 && r0 + 4 * g + 3 < rows) {
        *reinterpret_cast<d2*>(dst) = (d2){out[0], out[1]};
        *reinterpret_cast<d2*>(dst + 2) = (d2){out[2], out[3]};
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (r0 + 4 * g + v < rows) dst[v] = out[v];
      }
    }
    if (EPI != 2 && rpart) {
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      if (lane == 0) {
        const int slot = t * NW + wave;
        if (EPI == 1) {
          slot_ptr(rpart, rhs, S_DOT)[slot] = s0;
          slot_ptr(rpart, rhs, S_SUM)[slot] = 0.0;
          slot_ptr(rpart, rhs, S_SQ)[slot] = s1;
          slot_ptr(rpart, rhs, S_AUX2)[slot] = 0.0;
        } else {
          slot_ptr(rpart, rhs, S_SUM)[slot] = s0;
          slot_ptr(rpart, rhs, S_SQ)[slot] = s1;
        }
      }
    }
  }
}

// Packs B (K x K, row-major, FP64) as the S digits read by mp_oz and mp_ozh:
// for column fragment j, k-block kb (padded to the split), digit s and lane
// 16 g + c, 16 bytes hold digit s of B[64 kb + 16 g + b][16 j + c],
// b = 0..15; then the K column exponents f_n.  S = 7: the truncated base-128
// digits of B 2^-f_n (max_k |B[k][n]| < 2^f_n).  S = 6: the balanced
// base-256 digits of the integer image trunc(B 2^(47 - f_n)) (max_k |B[k][n]|
// < 2^f_n * 126/128), low to high; the digits in [-128, 127] of an integer
// are unique, so they are those the device takes from its data.
static void oz_pack(const double* B, int K, int S, void* dst) {
  const int nkb = oz_split(K) * oz_kb_per_wave(K);
  const size_t db = oz_digit_bytes(K, S);
  int8_t* o = (int8_t*)dst;
  for (size_t i = 0; i < db; ++i) o[i] = 0;
  int* fx = (int*)(o + db);
  for (int n = 0; n < K; ++n) {
    double mx = 0.0;
    for (int k = 0; k < K; ++k) mx = std::max(mx, std::fabs(B[(size_t)k * K + n]));
    int f = 0;
    if (mx > 0.0) {
      const double m = std::frexp(mx, &f);
      if (S == 6 && m >= 0.984375) ++f;
    }
    fx[n] = f;
    const int j = n / 16, c = n % 16;
    for (int k = 0; k < K; ++k) {
      const int kb = k / 64, g = (k % 64) / 16, b = k % 16;
      int dg[OZ_SMAX] = {0, 0, 0, 0, 0, 0, 0};
      if (S == 7) {
        double t = std::ldexp(B[(size_t)k * K + n], -f);
        for (int q = 0; q < 7; ++q) {
          t *= 128.0;
          const double d = std::trunc(t);
          t -= d;
          dg[q] = (int)d;
        }
      } else {
        int64_t F = (int64_t)std::trunc(std::ldexp(B[(size_t)k * K + n], 47 - f));
        for (int q = 5; q >= 1; --q) {
          const int64_t d = ((F + 128) & 255) - 128;
          dg[q] = (int)d;
          F = (F - d) / 256;                    // exact
        }
        dg[0] = (int)F;                         // |F| <= 126
      }
      for (int q = 0; q < S; ++q) {
        const size_t unit = (((size_t)j * nkb + kb) * S + q) * 64 + 16 * g + c;
        o[unit * 16 + b] = (int8_t)dg[q];
      }
    }
  }
}

// Rows per block of the int8 split product for a K x K operator.
static int oz_block_rows(int K) { return oz_split(K) == 2 ? 32 : 64; }

// Whether the operator-resident kernel (mp_ozr) serves the product: K <= 128,
// and its partial sums (eight per 128-row tile) fit the slots.
static bool oz_resident(int K, int64_t rows) { return K <= 128 && (rows + 127) / 128 * 8 <= GMAX; }

// Partial sums per right-hand side that an int8 product leaves.
static int oz_partials(int K, int64_t rows) {
  const int64_t t = oz_resident(K, rows) ? (rows + 127) / 128 * 8
                                         : (rows + oz_block_rows(K) - 1) / oz_block_rows(K);
  return t > (1 << 30) ? (1 << 30) : (int)t;
}

template <int S>
static void launch_oz_t(const PinvOps& op, int ax, bool fwd, const void* X, void* Y, int batch,
                      const RhsState* st, const double* la, const double* lb, const double* lc,
                      int a1, const double* gt, double* rpart, hipStream_t s) {
  const int K = op.n[ax];
  const int rows = (int)(op.N / K);
  const char* Bp = (const char*)(fwd ? op.Bf[ax] : op.Bb[ax]);
  const int* fx = (const int*)(Bp + oz_digit_bytes(K, S));
  const int br = oz_block_rows(K);
  dim3 grid((rows + br - 1) / br, batch);
  const int kbw = oz_kb_per_wave(K), ks = oz_split(K);
  if (oz_resident(K, rows)) {
    // one or two blocks per CU (by LDS), each sweeping 128-row tiles
    const int nrb = (rows + 127) / 128;
    const size_t lds_b = (size_t)(kbw * 4) * kbw * S * 64 * 16 + (size_t)64 * kbw * 12;
    const int per_cu = lds_b * 2 <= 160 * 1024 ? 2 : 1;
    const int nblk = std::max(1, std::min(nrb, (256 * per_cu + batch - 1) / batch));
    dim3 rg(nblk, batch);
    const int epi = lc ? 1 : (gt ? 2 : 0);
#define KP_OZR(W, E)                                                                         \
  hipLaunchKernelGGL((mp_ozr<W, E, S>), rg, dim3(512), 0, s, (const u4*)Bp, fx,               \
                     (const double*)X, (double*)Y, K, rows, (int64_t)op.N, st, la, lb, lc, a1, \
                     gt, rpart)
    if (kbw == 1) {
      if (epi == 1) KP_OZR(1, 1);
      else if (epi == 2) KP_OZR(1, 2);
      else KP_OZR(1, 0);
    } else {
      if (epi == 1) KP_OZR(2, 1);
      else if (epi == 2) KP_OZR(2, 2);
      else KP_OZR(2, 0);
    }
#undef KP_OZR
    return;
  }
#define KP_OZ(W, S_)                                                                         \
  hipLaunchKernelGGL((mp_oz<W, S_, S>), grid, dim3(256 * S_), 0, s, (const u4*)Bp, fx,          \
                     (const double*)X, (double*)Y, K, rows, (int64_t)op.N, st, la, lb, lc, a1, \
                     gt, rpart)
#define KP_OZH(W, E)                                                                         \
  hipLaunchKernelGGL((mp_ozh<W, E, S>), grid, dim3(256), 0, s, (const u4*)Bp, fx,               \
                     (const double*)X, (double*)Y, K, rows, (int64_t)op.N, st, la, lb, lc, a1, \
                     gt, rpart)
  if (ks == 1) {
    switch (kbw) {
      case 1: KP_OZ(1, 1); break;
      case 2: KP_OZ(2, 1); break;
      case 3: KP_OZ(3, 1); break;
      default: KP_OZ(4, 1); break;
    }
  } else {
    const int epi = lc ? 1 : (gt ? 2 : 0);
    if (kbw == 3) {
      if (epi == 1) KP_OZH(3, 1);
      else if (epi == 2) KP_OZH(3, 2);
      else KP_OZH(3, 0);
    } else {
      if (epi == 1) KP_OZH(4, 1);
      else if (epi == 2) KP_OZH(4, 2);
      else KP_OZH(4, 0);
    }
  }
#undef KP_OZ
#undef KP_OZH
}

static void launch_oz(const PinvOps& op, int ax, bool fwd, const void* X, void* Y, int batch,
                      const RhsState* st, const double* la, const double* lb, const double* lc,
                      int a1, const double* gt, double* rpart, hipStream_t s) {
  if (prec_digits(op.prec) == 6)
    launch_oz_t<6>(op, ax, fwd, X, Y, batch, st, la, lb, lc, a1, gt, rpart, s);
  else
    launch_oz_t<7>(op, ax, fwd, X, Y, batch, st, la, lb, lc, a1, gt, rpart, s);
}


// ------------------------------------------------------------------ host ----
// Tile configurations (column fragments per wave, row fragments per wave,
// column wave groups).  Block = 4 x wc waves, rows per block 64*wm, columns
// per block 16*wn*wc.  The operator packing does not depend on the choice, so
// any configuration may serve any product; the autotuner times them.
struct MpCfg { int wn, wm, wc; };
static const MpCfg kCfgs[] = {
    {1, 4, 1}, {2, 4, 1}, {3, 4, 1}, {4, 4, 1}, {6, 2, 1}, {8, 2, 1}, {12, 1, 1}, {16, 1, 1},
    {2, 4, 2}, {3, 4, 2}, {4, 2, 2}, {4, 4, 2}, {6, 2, 2}, {8, 1, 2}, {8, 2, 2}, {16, 1, 2},
    // tall tiles (FP32 and BF16 accumulators only): fewer re-reads of the operator
    {16, 2, 1}, {8, 4, 2},
    // short tiles of 128 columns: more blocks for short contractions
    {8, 1, 1}, {4, 1, 2},
    // operator-resident tiles (mp_res) of the same shapes, for K <= 128
    {8, 1, 1}, {4, 1, 2},
};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);
constexpr int kResFirst = 20;   // ids from here on are operator-resident
constexpr int kOzCfg = 13;      // the id an int8 split plan reports (mp_oz has one shape)

int mp_num_configs() { return kNumCfgs; }

bool mp_config_resident(int id) { return id >= kResFirst && id < kNumCfgs; }

// Whether configuration `id` can serve a K x K operator: the operator-resident
// tiles hold at most 128 x 128.
bool mp_config_fits(int id, int K) { return !mp_config_resident(id) || K <= 128; }

// Whether configuration `id` is compiled for `prec` (tiles whose registers
// would spill are left out: in FP64 those 16 fragments wide or with 4 row
// fragments of 4 or more columns, in BF16 the 16 x 2 tile).
bool mp_config_allowed(int id, int prec) {
  if (id < 0 || id >= kNumCfgs) return false;
  if (prec_int8(prec)) return id == kOzCfg;     // one kernel serves every product
  if (prec == PREC_F64) return !(id == 3 || id == 7 || id == 11 || (id >= 15 && id <= 17));
  if (prec == PREC_BF16) return id != 16;
  if (prec == PREC_BF16X6) return !(id == 3 || id == 7 || id == 11 || (id >= 15 && id <= 17));
  return true;
}

void mp_config(int id, int* wn, int* wm, int* wc) {
  *wn = kCfgs[id].wn; *wm = kCfgs[id].wm; *wc = kCfgs[id].wc;
}

// Default configuration for a K x K operator: the two-column-group tile whose
// block width covers K most tightly (eight waves per block), else the widest
// single-group tile.
int mp_default_config(int K, int prec) {
  if (prec_int8(prec)) return kOzCfg;
  const int frags = (K + 15) / 16;
  int best = -1, best_cb = 1 << 30;
  for (int id = 0; id < kNumCfgs; ++id) {
    const MpCfg& c = kCfgs[id];
    if (c.wc != 2 || c.wm == 4 || !mp_config_allowed(id, prec)) continue;
    const int cb = c.wn * c.wc;
    if (cb >= frags && cb < best_cb) { best = id; best_cb = cb; }
  }
  if (best >= 0) return best;
  return prec == PREC_F64 ? 13 : 15;   // widest: 256 (FP64) or 512 columns per block
}

static bool bf16_mfma(int prec) { return prec == PREC_BF16 || prec == PREC_BF16X6; }
static int chunk_k(int prec) { return bf16_mfma(prec) ? 32 : 16; }
static int elem_size(int prec) { return prec == PREC_F64 ? 8 : (prec == PREC_F32 ? 4 : 2); }
static int split_terms(int prec) { return prec == PREC_BF16X6 ? 3 : 1; }

static void packed_geometry(int K, int prec, int* npk, int* nkb) {
  *npk = ((K + 15) / 16) * 16;
  *nkb = (K + chunk_k(prec) - 1) / chunk_k(prec);
}

size_t mp_packed_bytes(int K, int prec) {
  if (prec_int8(prec)) return oz_digit_bytes(K, prec_digits(prec)) + (size_t)K * sizeof(int);
  int npk, nkb;
  packed_geometry(K, prec, &npk, &nkb);
  return (size_t)nkb * chunk_k(prec) * npk * elem_size(prec) * split_terms(prec);
}

static uint16_t bf16_rne(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}

static double bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return (double)f;
}

// Packs B (K x K, row-major, FP64) into the fragment order read by mp_kernel,
// converted to the compute type (round to nearest even).  Zero padding.
// BF16X6 packs the three BF16 terms of every entry (b = b1 + b2 + b3, each
// the round-to-nearest remainder of the previous, from the FP64 value) as
// three consecutive 16-byte units.
void mp_pack(const double* B, int K, int prec, void* dst) {
  if (prec_int8(prec)) {
    oz_pack(B, K, prec_digits(prec), dst);
    return;
  }
  int npk, nkb;
  packed_geometry(K, prec, &npk, &nkb);
  const int KBk = chunk_k(prec), es = elem_size(prec), T = split_terms(prec);
  const int CH = bf16_mfma(prec) ? 8 : 4;
  const int NV = (CH * es) / 16 * T, per = 16 / es;
  const size_t total = (size_t)nkb * KBk * npk * T;
  for (size_t e = 0; e < total * es; ++e) ((unsigned char*)dst)[e] = 0;
  for (int k = 0; k < K; ++k)
    for (int n = 0; n < K; ++n) {
      const int kb = k / KBk, rem = k % KBk, g = rem / CH, s = rem % CH;
      const int h = (s * es) / 16, w = s % per;
      const double v = B[(size_t)k * K + n];
      if (T == 3) {
        double r = v;
        for (int t = 0; t < 3; ++t) {
          const uint16_t b = bf16_rne((float)r);
          const size_t idx = ((((size_t)kb * 4 + g) * NV + t) * npk + n) * per + w;
          ((uint16_t*)dst)[idx] = b;
          r -= bf16_value(b);
        }
        continue;
      }
      const size_t idx = ((((size_t)kb * 4 + g) * NV + h) * npk + n) * per + w;
      if (es == 8) {
        ((double*)dst)[idx] = v;
      } else if (es == 4) {
        ((float*)dst)[idx] = (float)v;
      } else {
        ((uint16_t*)dst)[idx] = bf16_rne((float)v);
      }
    }
}

template <int PREC, class Ti, class To, int WN, int WM, int WC, bool VEC>
static void launch_cfg(const PinvOps& op, int ax, bool fwd, const void* X, void* Y, int rows,
                       int batch, const RhsState* st, int in_scale, int out_scale,
                       const double* la, const double* lb, const double* lc, int a1,
                       const double* gt, double* rpart, int rscl, hipStream_t s) {
  const int K = op.n[ax];
  const int cb = 16 * WN * WC, ncc = (K + cb - 1) / cb;
  constexpr int BR = WR * 16 * WM;
  const int nrb = (rows + BR - 1) / BR;
  int npk, nkb;
  packed_geometry(K, PREC, &npk, &nkb);
  dim3 grid(nrb * ncc, batch);
  hipLaunchKernelGGL((mp_kernel<PREC, Ti, To, WN, WM, WC, VEC>), grid, dim3(64 * WR * WC), 0, s,
                     (const u4*)(fwd ? op.Bf[ax] : op.Bb[ax]), npk, ncc, (const Ti*)X, (To*)Y, K,
                     rows, (int64_t)op.N, st, in_scale, out_scale, la, lb, lc, a1, gt, rpart,
                     rscl);
}

// Persistent blocks of the operator-resident tile: as many per right-hand
// side as fill the chip once (the operator's LDS share sets the blocks per
// CU), never more than the row tiles.
template <int PREC>
constexpr int res_lds_bytes() {
  return (128 / (4 * MT<PREC>::CH)) * 4 * MT<PREC>::NV * 128 * 16;
}

template <int PREC, class Ti, class To, int WN, int WC>
static void launch_res(const PinvOps& op, int ax, bool fwd, const void* X, void* Y, int rows,
                       int batch, const RhsState* st, int in_scale, int out_scale,
                       const double* la, const double* lb, const double* lc, int a1,
                       const double* gt, double* rpart, int rscl, hipStream_t s) {
  const int K = op.n[ax];
  constexpr int BR = WR * 16;
  const int nrb = (rows + BR - 1) / BR;
  int npk, nkb;
  packed_geometry(K, PREC, &npk, &nkb);
  // LDS per block: the operator, and for BF16 outputs the staged tile
  constexpr int lds_b = res_lds_bytes<PREC>() + (sizeof(To) == 2 ? 128 * (WR * 16 + 8) * 2 : 0);
  constexpr int per_cu = (160 * 1024) / lds_b < 1 ? 1
                         : ((160 * 1024) / lds_b > 4 ? 4 : (160 * 1024) / lds_b);
  const int want = (256 * per_cu + batch - 1) / batch;
  const int nblk = std::max(1, std::min(nrb, want));
  dim3 grid(nblk, batch);
  hipLaunchKernelGGL((mp_res<PREC, Ti, To, WN, WC>), grid, dim3(64 * WR * WC), 0, s,
                     (const u4*)(fwd ? op.Bf[ax] : op.Bb[ax]), npk, (const Ti*)X, (To*)Y, K, rows,
                     (int64_t)op.N, st, in_scale, out_scale, la, lb, lc, a1, gt, rpart, rscl);
}

template <int PREC, class Ti, class To>
static void launch_mp(int cls, int cfg, const PinvOps& op, int ax, bool fwd, const void* X,
                      void* Y, int batch, const RhsState* st, int in_scale, int out_scale,
                      const double* la, const double* lb, const double* lc, int a1,
                      const double* gt, hipStream_t s, double* rpart = nullptr,
                      int rscl = 0) {
  trace_begin(cls, s);
  if constexpr (prec_int8(PREC)) {
    (void)cfg;
    launch_oz(op, ax, fwd, X, Y, batch, st, la, lb, lc, a1, gt, rpart, s);
    trace_end(cls, s);
    return;
  } else {
  const int K = op.n[ax];
  const int rows = (int)(op.N / K);
  const int CH = MT<PREC>::CH;
  if (K % CH != 0) {
    // rows too ragged for 16-byte loads: one scalar-load tile serves every
    // configuration (such grids are small)
    launch_cfg<PREC, Ti, To, 4, 2, 2, false>(op, ax, fwd, X, Y, rows, batch, st, in_scale,
                                             out_scale, la, lb, lc, a1, gt, rpart, rscl, s);
    trace_end(cls, s);
    return;
  }
#define KP_CASE(ID, W, M_, C)                                                                 \
  case ID:                                                                                    \
    launch_cfg<PREC, Ti, To, W, M_, C, true>(op, ax, fwd, X, Y, rows, batch, st, in_scale,    \
                                             out_scale, la, lb, lc, a1, gt, rpart, rscl, s);  \
    break;
  if (mp_config_resident(cfg) && K <= 128) {
    if (cfg == kResFirst)
      launch_res<PREC, Ti, To, 8, 1>(op, ax, fwd, X, Y, rows, batch, st, in_scale, out_scale, la,
                                     lb, lc, a1, gt, rpart, rscl, s);
    else
      launch_res<PREC, Ti, To, 4, 2>(op, ax, fwd, X, Y, rows, batch, st, in_scale, out_scale, la,
                                     lb, lc, a1, gt, rpart, rscl, s);
    trace_end(cls, s);
    return;
  }
#define KP_COMMON_CASES                                                                      \
  KP_CASE(0, 1, 4, 1) KP_CASE(1, 2, 4, 1) KP_CASE(2, 3, 4, 1) KP_CASE(4, 6, 2, 1)             \
  KP_CASE(5, 8, 2, 1) KP_CASE(6, 12, 1, 1) KP_CASE(8, 2, 4, 2) KP_CASE(9, 3, 4, 2)            \
  KP_CASE(10, 4, 2, 2) KP_CASE(12, 6, 2, 2) KP_CASE(14, 8, 2, 2)                            \
  KP_CASE(18, 8, 1, 1) KP_CASE(19, 4, 1, 2)
  // tiles whose registers would spill are left out: FP64 accumulators and
  // operands are twice as wide, and the FP64-sourced BF16 product holds
  // 16 VGPRs of raw data per row fragment and k-block
  if constexpr (PREC == PREC_F64) {
    switch (cfg) {
      KP_COMMON_CASES
      default: KP_CASE(13, 8, 1, 2)
    }
  } else if constexpr (PREC == PREC_F32) {
    switch (cfg) {
      KP_COMMON_CASES
      KP_CASE(3, 4, 4, 1)
      KP_CASE(7, 16, 1, 1)
      KP_CASE(11, 4, 4, 2)
      KP_CASE(15, 16, 1, 2)
      KP_CASE(16, 16, 2, 1)
      KP_CASE(17, 8, 4, 2)
      default: KP_CASE(13, 8, 1, 2)
    }
  } else if constexpr (PREC == PREC_BF16) {
    switch (cfg) {
      KP_COMMON_CASES
      KP_CASE(3, 4, 4, 1)
      KP_CASE(7, 16, 1, 1)
      KP_CASE(11, 4, 4, 2)
      KP_CASE(15, 16, 1, 2)
      KP_CASE(17, 8, 4, 2)
      default: KP_CASE(13, 8, 1, 2)
    }
  } else {
    switch (cfg) {
      KP_COMMON_CASES
      default: KP_CASE(13, 8, 1, 2)
    }
  }
#undef KP_COMMON_CASES
#undef KP_CASE
  trace_end(cls, s);
  }
}

// Product q of one application Z = M(R) (Algs. 6-7) for `batch` right-hand
// sides with the solver's buffers: R -> T0 -> T1 -> T0 ... -> Z (R and Z FP64
// in the natural layout, T0 and T1 in the compute type).  The first product
// scales its input per right-hand side and the last unscales its output (not
// in FP64); the last forward one carries the Hadamard factor, Ghat from the
// eigenvalues or, for the low-rank preconditioner, the table op.gtab.
template <int PREC>
static void pinv_step_t(const PinvOps& op, int q, const double* R, double* Z, void* T0,
                        void* T1, int batch, const RhsState* st, hipStream_t s) {
  using tc = typename MT<PREC>::tc;
  const int scl = (PREC == PREC_F64 || prec_int8(PREC)) ? 0 : 1;
  const int dim = op.dim, ax = q % dim, last = 2 * dim - 1;
  const bool fwd = q < dim;
  void* T[2] = {T0, T1};
  const void* in = q == 0 ? (const void*)R : (const void*)T[(q - 1) % 2];
  void* out = q == last ? (void*)Z : T[q % 2];
  const int cls = fwd ? (ax == 0 ? KC_MP_X_FWD : (ax == 1 ? KC_MP_Y_FWD : KC_MP_Z_FWD))
                      : (ax == 0 ? KC_MP_X_BWD : (ax == 1 ? KC_MP_Y_BWD : KC_MP_Z_BWD));
  if (q == 0) {
    launch_mp<PREC, double, tc>(cls, op.cfg[q], op, ax, fwd, in, out, batch, st, scl, 0, nullptr,
                                nullptr, nullptr, 1, nullptr, s,
                                prec_int8(PREC) ? op.hpart : nullptr);
  } else if (q == last) {
    launch_mp<PREC, tc, double>(cls, op.cfg[q], op, ax, fwd, in, out, batch, st, 0, scl, nullptr,
                                nullptr, nullptr, 1, nullptr, s);
  } else if (q == dim - 1 && op.gtab) {
    launch_mp<PREC, tc, tc>(cls, op.cfg[q], op, ax, fwd, in, out, batch, st, 0, 0, nullptr,
                            nullptr, nullptr, 1, op.gtab, s);
  } else if (q == dim - 1) {
    launch_mp<PREC, tc, tc>(cls, op.cfg[q], op, ax, fwd, in, out, batch, st, 0, 0, op.lam[0],
                            dim == 3 ? op.lam[1] : nullptr, op.lam[dim - 1], op.n[0], nullptr, s,
                            op.rpart, scl);
  } else {
    launch_mp<PREC, tc, tc>(cls, op.cfg[q], op, ax, fwd, in, out, batch, st, 0, 0, nullptr,
                            nullptr, nullptr, 1, nullptr, s);
  }
}

template <int PREC>
static void pinv_apply_t(const PinvOps& op, const double* R, double* Z, void* T0, void* T1,
                         int batch, const RhsState* st, hipStream_t s) {
  for (int q = 0; q < 2 * op.dim; ++q) pinv_step_t<PREC>(op, q, R, Z, T0, T1, batch, st, s);
}

// Launches product q of the preconditioner alone (autotuning): q < dim are the
// forward products (the first reads FP64, the last carries G), q >= dim the
// backward ones (the last writes FP64).
template <int PREC>
static void product_t(const PinvOps& op, int q, const void* in, void* out, int batch,
                      hipStream_t s) {
  using tc = typename MT<PREC>::tc;
  const int dim = op.dim, ax = q % dim;
  const bool fwd = q < dim;
  const bool gq = q == dim - 1;
  const double* la = gq ? op.lam[0] : nullptr;
  const double* lb = (gq && dim == 3) ? op.lam[1] : nullptr;
  const double* lc = gq ? op.lam[dim - 1] : nullptr;
  const int cls = fwd ? (ax == 0 ? KC_MP_X_FWD : (ax == 1 ? KC_MP_Y_FWD : KC_MP_Z_FWD))
                      : (ax == 0 ? KC_MP_X_BWD : (ax == 1 ? KC_MP_Y_BWD : KC_MP_Z_BWD));
  if (q == 0)
    launch_mp<PREC, double, tc>(cls, op.cfg[q], op, ax, fwd, in, out, batch, nullptr, 0, 0, la,
                                lb, lc, op.n[0], nullptr, s);
  else if (q == 2 * dim - 1)
    launch_mp<PREC, tc, double>(cls, op.cfg[q], op, ax, fwd, in, out, batch, nullptr, 0, 0, la,
                                lb, lc, op.n[0], nullptr, s);
  else
    launch_mp<PREC, tc, tc>(cls, op.cfg[q], op, ax, fwd, in, out, batch, nullptr, 0, 0, la, lb,
                            lc, op.n[0], nullptr, s);
}

int pinv_first_blocks(const PinvOps& op) {
  if (!prec_int8(op.prec)) return 0;
  const int K = op.n[0];
  return oz_partials(K, op.N / K);
}

int pinv_ghat_blocks(const PinvOps& op) {
  const int q = op.dim - 1, ax = q;
  const int K = op.n[ax];
  const int64_t rows = op.N / K;
  if (prec_int8(op.prec))     // eight per 128 rows (K <= 128), else one per block of 64 or 32 rows
    return oz_partials(K, rows);
  const int CH = op.prec == PREC_F64 || op.prec == PREC_F32 ? 4 : 8;
  int wn = 4, wm = 2, wc = 2;   // the scalar-load tile of ragged contractions
  // the operator-resident tiles write one partial per 64-row tile
  if (K % CH == 0 && mp_config_resident(op.cfg[q]) && K <= 128) {
    const int64_t t = (rows + WR * 16 - 1) / (WR * 16);
    return t > (1 << 30) ? (1 << 30) : (int)t;
  }
  // a configuration not compiled for the precision launches tile 13, as the
  // dispatch in launch_mp does
  if (K % CH == 0)
    mp_config((mp_config_allowed(op.cfg[q], op.prec) && !mp_config_resident(op.cfg[q]))
                  ? op.cfg[q] : 13, &wn, &wm, &wc);
  const int64_t nrb = (rows + WR * 16 * wm - 1) / (WR * 16 * wm);
  const int64_t ncc = (K + 16 * wn * wc - 1) / (16 * wn * wc);
  const int64_t b = nrb * ncc;
  return b > (1 << 30) ? (1 << 30) : (int)b;
}

void pinv_product(const PinvOps& op, int q, const void* in, void* out, int batch,
                  hipStream_t s) {
  switch (op.prec) {
    case PREC_F64: product_t<PREC_F64>(op, q, in, out, batch, s); break;
    case PREC_F32: product_t<PREC_F32>(op, q, in, out, batch, s); break;
    case PREC_BF16X6: product_t<PREC_BF16X6>(op, q, in, out, batch, s); break;
    case PREC_I8X7: product_t<PREC_I8X7>(op, q, in, out, batch, s); break;
    case PREC_I8X6: product_t<PREC_I8X6>(op, q, in, out, batch, s); break;
    default: product_t<PREC_BF16>(op, q, in, out, batch, s); break;
  }
}

void pinv_step(const PinvOps& op, int q, const double* R, double* Z, void* T0, void* T1,
               int batch, const RhsState* st, hipStream_t s) {
  switch (op.prec) {
    case PREC_F64: pinv_step_t<PREC_F64>(op, q, R, Z, T0, T1, batch, st, s); break;
    case PREC_F32: pinv_step_t<PREC_F32>(op, q, R, Z, T0, T1, batch, st, s); break;
    case PREC_BF16X6: pinv_step_t<PREC_BF16X6>(op, q, R, Z, T0, T1, batch, st, s); break;
    case PREC_I8X7: pinv_step_t<PREC_I8X7>(op, q, R, Z, T0, T1, batch, st, s); break;
    case PREC_I8X6: pinv_step_t<PREC_I8X6>(op, q, R, Z, T0, T1, batch, st, s); break;
    default: pinv_step_t<PREC_BF16>(op, q, R, Z, T0, T1, batch, st, s); break;
  }
}

void pinv_apply(const PinvOps& op, const double* R, double* Z, void* T0, void* T1, int batch,
                const RhsState* st, hipStream_t s) {
  switch (op.prec) {
    case PREC_F64: pinv_apply_t<PREC_F64>(op, R, Z, T0, T1, batch, st, s); break;
    case PREC_F32: pinv_apply_t<PREC_F32>(op, R, Z, T0, T1, batch, st, s); break;
    case PREC_BF16X6: pinv_apply_t<PREC_BF16X6>(op, R, Z, T0, T1, batch, st, s); break;
    case PREC_I8X7: pinv_apply_t<PREC_I8X7>(op, R, Z, T0, T1, batch, st, s); break;
    case PREC_I8X6: pinv_apply_t<PREC_I8X6>(op, R, Z, T0, T1, batch, st, s); break;
    default: pinv_apply_t<PREC_BF16>(op, R, Z, T0, T1, batch, st, s); break;
  }
}

}  // namespace kp
