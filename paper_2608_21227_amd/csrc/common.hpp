// Shared device helpers for the svdv kernels (gfx950 / CDNA4, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace svdv {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Strided matrix view: element (r, c) lives at p[r * rs + c * cs].
// QR sweeps use the column-major matrix as is (rs = 1, cs = ld); LQ sweeps use
// its transpose (rs = ld, cs = 1), so one kernel body serves both sides.
template <typename T>
struct View {
  T* p;
  int64_t rs, cs;
  __device__ __forceinline__ T& at(int64_t r, int64_t c) const { return p[r * rs + c * cs]; }
};

// Rows of one TSQR chunk inside the panel.  Level 1 chunks are contiguous row
// ranges; chunks of level >= 2 stack the top `per_unit` rows of the chunks
// below them:  row(c, q) = base + c * chunk_stride + (q / per_unit) * unit_stride + q % per_unit.
struct RowMap {
  int64_t base;
  int64_t chunk_stride;
  int64_t unit_stride;
  int32_t per_unit;   // 0 = contiguous chunk
  __device__ __forceinline__ int64_t row(int64_t c, int64_t q) const {
    if (per_unit == 0) return base + c * chunk_stride + q;
    return base + c * chunk_stride + (q / per_unit) * unit_stride + (q % per_unit);
  }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// MFMA 16x16x4: D[16x16] += A[16x4] * B[4x16].
// Operand layout (lane l): A holds A[l % 16][l / 16], B holds B[l / 16][l % 16].
// Result layout is per-type (see acc_row()).
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T> struct Acc;
template <> struct Acc<float> { typedef f32x4 type; };
template <> struct Acc<double> { typedef f64x4 type; };

}  // namespace svdv
