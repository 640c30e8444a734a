// Device helpers shared by the stage kernels: element types, conversions,
// MFMA wrappers and their accumulator layouts.
#pragma once

#include "ssm_internal.h"

namespace ssmc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Fourth word of a raw buffer resource on gfx9-family GPUs (32-bit data
// format, no swizzle), as used for untyped buffer loads and stores.
constexpr int kBufferWord3 = 0x00020000;

// FP32 -> BF16, round to nearest even (NaN stays NaN): the conversion
// instruction of gfx950 (v_cvt_pk_bf16_f32), branch-free.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}

template <int CT>
struct CTraits;
template <>
struct CTraits<DT_BF16> {
  using X = float;      // state / accumulator element
  using Op = uint16_t;  // MFMA operand element (bf16 bits)
  using Acc = f32x4;
  static constexpr int KI = 32;  // K of one 16x16 MFMA
  static constexpr int KPL = 8;  // K elements per lane
  static constexpr int PAD = 8;  // LDS row padding (elements)
  // accumulator register v of lane group g holds row 4g + v of the 16x16 block
  static __device__ __forceinline__ int acc_row(int g, int v) { return 4 * g + v; }
};
template <>
struct CTraits<DT_F32> {
  using X = float;
  using Op = float;
  using Acc = f32x4;
  static constexpr int KI = 4;
  static constexpr int KPL = 1;
  static constexpr int PAD = 4;  // keeps LDS rows 16-byte aligned
  static __device__ __forceinline__ int acc_row(int g, int v) { return 4 * g + v; }
};
template <>
struct CTraits<DT_F64> {
  using X = double;
  using Op = double;
  using Acc = f64x4;
  static constexpr int KI = 4;
  static constexpr int KPL = 1;
  static constexpr int PAD = 2;  // keeps LDS rows 16-byte aligned
  // the FP64 16x16x4 MFMA interleaves rows: register v of lane group g is row g + 4v
  static __device__ __forceinline__ int acc_row(int g, int v) { return g + 4 * v; }
};

template <typename Op, typename X>
__device__ __forceinline__ Op to_op(X v);
template <>
__device__ __forceinline__ uint16_t to_op<uint16_t, float>(float v) {
  return f32_to_bf16_bits(v);
}
template <>
__device__ __forceinline__ float to_op<float, float>(float v) {
  return v;
}
template <>
__device__ __forceinline__ double to_op<double, double>(double v) {
  return v;
}

template <typename X>
__device__ __forceinline__ X load_src(const void* src, int dtype, int64_t i) {
  if (dtype == DT_F64) return (X)((const double*)src)[i];
  if (dtype == DT_F32) return (X)((const float*)src)[i];
  return (X)bf16_bits_to_f32(((const uint16_t*)src)[i]);
}

// Elements i .. i+3 of an FP32 or BF16 input as FP32; one 16- or 8-byte load
// when vec (the caller has checked that element i is 16- or 8-byte aligned).
__device__ __forceinline__ f32x4 load_src4(const void* src, int dtype, int64_t i, bool vec) {
  if (dtype == DT_F32) {
    const float* s = (const float*)src + i;
    if (vec) return *reinterpret_cast<const f32x4*>(s);
    return f32x4{s[0], s[1], s[2], s[3]};
  }
  const uint16_t* s = (const uint16_t*)src + i;
  if (vec) {
    const uint2 w = *reinterpret_cast<const uint2*>(s);
    return f32x4{__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xffff0000u),
                 __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xffff0000u)};
  }
  return f32x4{bf16_bits_to_f32(s[0]), bf16_bits_to_f32(s[1]), bf16_bits_to_f32(s[2]),
               bf16_bits_to_f32(s[3])};
}
// Whether element i of src may be loaded four at a time by load_src4.
__device__ __forceinline__ bool src4_aligned(const void* src, int dtype, int64_t i) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(src) + (uintptr_t)i * (dtype == DT_F32 ? 4u : 2u);
  return (a & (dtype == DT_F32 ? 15u : 7u)) == 0;
}

// One 16x16 MFMA step for each compute type.
template <int CT>
struct Mfma;
template <>
struct Mfma<DT_BF16> {
  static __device__ __forceinline__ f32x4 run(const uint16_t* a, const uint16_t* b, f32x4 c) {
    bf16x8 av = *reinterpret_cast<const bf16x8*>(a);
    bf16x8 bv = *reinterpret_cast<const bf16x8*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
};
template <>
struct Mfma<DT_F32> {
  static __device__ __forceinline__ f32x4 run(const float* a, const float* b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(*a, *b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<DT_F64> {
  static __device__ __forceinline__ f64x4 run(const double* a, const double* b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(*a, *b, c, 0, 0, 0);
  }
};

}  // namespace ssmc
