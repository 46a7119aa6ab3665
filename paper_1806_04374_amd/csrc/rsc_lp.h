// 16-bit MFMA operands (BF16 / FP16) shared by the precision-form kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "rsc.h"
#include "rsc_device.h"

namespace rsc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// unit: unit roundoff of the format (round to nearest); mfma: v_mfma_f32_32x32x16 of
// the format (lane l supplies A[l%32][8(l/32)+i] and B[8(l/32)+i][l%32], i = 0..7).
template <int PREC>
struct Lp;

template <>
struct Lp<RSC_BF16> {
  using V8 = bf16x8;
  using V2 = bf16x2;
  static constexpr float unit = 0x1p-8f;
  __device__ static f32x16 mfma(V8 a, V8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Lp<RSC_FP16> {
  using V8 = f16x8;
  using V2 = f16x2;
  static constexpr float unit = 0x1p-11f;
  __device__ static f32x16 mfma(V8 a, V8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// Two floats rounded to the 16-bit format (round to nearest even), packed into
// one 32-bit register (x in the low half).
template <class P>
__device__ __forceinline__ unsigned pack2(float x, float y) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{x, y}, typename P::V2));
}

// Eight floats rounded to the 16-bit format (round to nearest even), packed.
template <class P>
__device__ __forceinline__ typename P::V8 pack8(const float (&v)[8]) {
  typename P::V8 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const typename P::V2 h = __builtin_convertvector(f32x2{v[2 * i], v[2 * i + 1]}, typename P::V2);
    r[2 * i] = h[0];
    r[2 * i + 1] = h[1];
  }
  return r;
}

// x = hi + lo with hi the 16-bit rounding of x and lo the 16-bit rounding of the
// (exact, in FP32) remainder x - hi: eight values of one lane, packed.
template <class P>
__device__ __forceinline__ void split8(const float (&x)[8], typename P::V8& hi, typename P::V8& lo) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const typename P::V2 h = __builtin_convertvector(f32x2{x[2 * i], x[2 * i + 1]}, typename P::V2);
    const f32x2 back = __builtin_convertvector(h, f32x2);
    const typename P::V2 l = __builtin_convertvector(f32x2{x[2 * i] - back[0], x[2 * i + 1] - back[1]},
                                                     typename P::V2);
    hi[2 * i] = h[0];
    hi[2 * i + 1] = h[1];
    lo[2 * i] = l[0];
    lo[2 * i + 1] = l[1];
  }
}

// x = hi + mid + lo, each part the 16-bit rounding of what the previous ones leave
// (exact remainders in FP32): eight values of one lane, packed.
template <class P>
__device__ __forceinline__ void split8x3(const float (&x)[8], typename P::V8& hi, typename P::V8& mid,
                                         typename P::V8& lo) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const f32x2 v{x[2 * i], x[2 * i + 1]};
    const typename P::V2 h = __builtin_convertvector(v, typename P::V2);
    const f32x2 r1 = v - __builtin_convertvector(h, f32x2);
    const typename P::V2 m = __builtin_convertvector(r1, typename P::V2);
    const f32x2 r2 = r1 - __builtin_convertvector(m, f32x2);
    const typename P::V2 l = __builtin_convertvector(r2, typename P::V2);
    hi[2 * i] = h[0];
    hi[2 * i + 1] = h[1];
    mid[2 * i] = m[0];
    mid[2 * i + 1] = m[1];
    lo[2 * i] = l[0];
    lo[2 * i + 1] = l[1];
  }
}

}  // namespace rsc
