// Shared device helpers for the svdv kernels (gfx950 / CDNA4, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace svdv {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
// Scale exponent recorded for an input that holds a NaN or an infinity: no
// finite maximum has a binary exponent anywhere near it.  Every output stage
// that reads the exponent then writes NaN (the input has no singular values).
constexpr int kExpNonFinite = -(1 << 30);

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

// Quotient a / b by a reciprocal and Newton-Raphson (Markstein's scheme): the
// hardware reciprocal r ~ 1/b (about 24 correct bits) is refined once,
// r += r (1 - b r), then q = a r gets one residual correction q += r (a - b q).
// Valid for normal b whose reciprocal is normal; the result is within one unit
// in the last place of the rounded quotient.
__device__ __forceinline__ double nr_div(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}

// Wave-wide sums with DPP lane moves (quad permutes, row shifts and the row
// broadcasts of wave64), the total collected in lane 63 and returned to every
// lane through a scalar register, so all lanes see bitwise the same value.
// Must be called with the whole wave active.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = dpp_i<CTRL>(__double2loint(v));
  const int hi = dpp_i<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
// Sums over the first 16 or 32 lanes only (the other lanes must hold 0): the
// same DPP tree as wave_sum stopped after the stages that reach lane 15 (one
// row) or lane 31 (two rows), so the value equals wave_sum's bitwise.
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_d<0xb1>(v);
  v += dpp_d<0x4e>(v);
  v += dpp_d<0x114>(v);
  v += dpp_d<0x118>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 15);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 15);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row_sum32(double v) {
  v += dpp_d<0xb1>(v);
  v += dpp_d<0x4e>(v);
  v += dpp_d<0x114>(v);
  v += dpp_d<0x118>(v);
  v += dpp_d<0x142>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 31);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 31);
  return __hiloint2double(hi, lo);
}

// Value of lane l (wave-uniform l) of v, as a wave-uniform result.
__device__ __forceinline__ double lane_value(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// LDS pointer types: indexing through them keeps address arithmetic in 32 bits.
typedef __attribute__((address_space(3))) double lds_f64;
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) f64x2 lds_f64x2;

__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<0xb1>(v);   // quad_perm 1,0,3,2
  v += dpp_f<0x4e>(v);   // quad_perm 2,3,0,1
  v += dpp_f<0x114>(v);  // row_shr:4
  v += dpp_f<0x118>(v);  // row_shr:8
  v += dpp_f<0x142>(v);  // row_bcast:15
  v += dpp_f<0x143>(v);  // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xb1>(v);
  v += dpp_d<0x4e>(v);
  v += dpp_d<0x114>(v);
  v += dpp_d<0x118>(v);
  v += dpp_d<0x142>(v);
  v += dpp_d<0x143>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
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

// Reduced-precision MFMA 16x16x16 with float32 accumulation: lane l supplies
// A[l % 16][4 (l / 16) + i] and B[4 (l / 16) + i][l % 16], i = 0..3, rounded to
// BF16 (PREC 2, round to nearest even) or FP16 (PREC 3); the result layout is
// that of the float32 16x16x4 instruction.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ short f32_to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
template <int PREC>
__device__ __forceinline__ f32x4 mfma16x16(const float (&a)[4], const float (&b)[4], f32x4 c) {
  if constexpr (PREC == 2) {
    const bf16x4 av = {f32_to_bf16(a[0]), f32_to_bf16(a[1]), f32_to_bf16(a[2]), f32_to_bf16(a[3])};
    const bf16x4 bv = {f32_to_bf16(b[0]), f32_to_bf16(b[1]), f32_to_bf16(b[2]), f32_to_bf16(b[3])};
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c, 0, 0, 0);
  } else {
    const f16x4 av = {(_Float16)a[0], (_Float16)a[1], (_Float16)a[2], (_Float16)a[3]};
    const f16x4 bv = {(_Float16)b[0], (_Float16)b[1], (_Float16)b[2], (_Float16)b[3]};
    return __builtin_amdgcn_mfma_f32_16x16x16f16(av, bv, c, 0, 0, 0);
  }
}

// Row of the 16x16 MFMA result held in register i of lane-group g (g = lane / 16):
// float: 4g + i, double: 4i + g (measured on gfx950).
template <typename T> __device__ __forceinline__ int acc_row(int g, int i);
template <> __device__ __forceinline__ int acc_row<float>(int g, int i) { return 4 * g + i; }
template <> __device__ __forceinline__ int acc_row<double>(int g, int i) { return 4 * i + g; }

template <typename T> struct Acc;
template <> struct Acc<float> { typedef f32x4 type; };
template <> struct Acc<double> { typedef f64x4 type; };

}  // namespace svdv
