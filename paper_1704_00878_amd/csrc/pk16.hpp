// Packed 16-bit helpers shared by the packed kernels (two pairs per lane:
// one in the low and one in the high half of every register).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

typedef short pk16 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ pk16 as_pk(uint32_t x) { return __builtin_bit_cast(pk16, x); }
__device__ __forceinline__ uint32_t as_u(pk16 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ pk16 pmax(pk16 a, pk16 b) { return __builtin_elementwise_max(a, b); }

// Biased 16-bit values: every H, E*, F* and H - go - ge is held plus
// kBias16, which keeps each operand of the three-way maxima a non-negative
// 16-bit pattern below 0x7c00 (a finite non-negative half), whose order as a
// half is its order as an integer.  The host bound H < 15000 gives values in
// [kBias16 - 512, kBias16 + 15000); a padding entry of kPadProf16 makes H - go
// - ge + pad below kBias16, so it never wins against the floor, and at least
// 0.
constexpr int kBias16 = 15616;
constexpr int kPadProf16 = -15360;

// max(a, b, c) per half with one v_pk_maximum3_f16 (operands as above)
__device__ __forceinline__ pk16 max3h(pk16 a, pk16 b, pk16 c) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 r = __builtin_elementwise_maximum(
        __builtin_elementwise_maximum(__builtin_bit_cast(h2, a), __builtin_bit_cast(h2, b)), __builtin_bit_cast(h2, c));
    return __builtin_bit_cast(pk16, r);
}

// bitwise select m ? x : y (written out: with a mask known to be whole
// halves, the compiler would select per half with compares instead)
__device__ __forceinline__ uint32_t bfi(uint32_t m, uint32_t x, uint32_t y) {
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(m), "v"(x), "v"(y));
    return r;
}

// the same with a wave-uniform mask in an SGPR
__device__ __forceinline__ uint32_t bfi_s(uint32_t m, uint32_t x, uint32_t y) {
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "s"(m), "v"(x), "v"(y));
    return r;
}

}  // namespace hk
