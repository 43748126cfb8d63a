// Shared device-side definitions of the kpcg library (gfx950 / CDNA4).
//
// Grid layout of every vector: [rhs][z][y][x] with x contiguous, which is the
// paper's vec() ordering (Sec. 2.1): the first index i varies fastest, then j,
// then k.  A batch of right-hand sides is stacked RHS-major.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include "kp_state.h"

namespace kp {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

// Boundary conditions of eq. (3.1).
enum Bc { BC_P = 0, BC_D = 1, BC_N = 2, BC_DN = 3, BC_ND = 4 };
enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2, PREC_BF16X6 = 3, PREC_I8X7 = 4, PREC_I8X6 = 5 };

// The FP64-accurate splits on the int8 matrix cores, and their digit counts.
__host__ __device__ constexpr bool prec_int8(int p) { return p == PREC_I8X7 || p == PREC_I8X6; }
__host__ __device__ constexpr int prec_digits(int p) { return p == PREC_I8X6 ? 6 : 7; }

// Reduction slots written by the vector and mode-product kernels, one block
// partial per slot; reduced in a fixed order for bitwise reproducibility.
enum Slot {
  S_SUM = 0,   // sum of entries (eta, R or Z)
  S_SQ,        // sum of squares
  S_DOT,       // inner product
  S_AUX,       // second sum of squares (||U||^2)
  S_AUX2,      // <R_old, Z> for the flexible beta
  S_TSQ,       // ||eta_c - L U_1||^2 from the first U/R update (exit step's sums)
  S_TSUM,      // sum of U_1, from the same pass
  NSLOTS
};

constexpr int GMAX = 8192;     // most block partials per slot

__device__ __forceinline__ double* slot_ptr(double* part, int rhs, int slot) {
  return part + ((int64_t)rhs * NSLOTS + slot) * GMAX;
}

__device__ __forceinline__ double wave_sum(double v) {
  // 64-lane butterfly; every lane ends with the same total, in a fixed order
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block reduction of NV values for a 256-thread block.  Fixed order:
// butterfly within the wave, then wave 0..3 in sequence.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /*[4*NV]*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) lds[wave * NV + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += lds[w * NV + q];
    v[q] = t;
  }
  __syncthreads();
}

// bf16 <-> float with round-to-nearest-even
__device__ __forceinline__ __bf16 f2bf(float x) { return (__bf16)x; }
__device__ __forceinline__ float bf2f(__bf16 x) { return (float)x; }

template <class T> __device__ __forceinline__ T from_double(double x);
template <> __device__ __forceinline__ double from_double<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_double<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ __bf16 from_double<__bf16>(double x) { return (__bf16)(float)x; }

template <class T> __device__ __forceinline__ T from_float(float x);
template <> __device__ __forceinline__ double from_float<double>(float x) { return (double)x; }
template <> __device__ __forceinline__ float from_float<float>(float x) { return x; }
template <> __device__ __forceinline__ __bf16 from_float<__bf16>(float x) { return (__bf16)x; }

template <class T> __device__ __forceinline__ double to_double(T x) { return (double)x; }
template <> __device__ __forceinline__ double to_double<__bf16>(__bf16 x) { return (double)(float)x; }

}  // namespace kp
