// fp8.h -- OCP E4M3 encoding with E8M0 block scales, shared by the
// quantization kernels and the sketch kernel's quantizing epilogue.
//
// Per block of 64 values: s = the smallest integer with max|x| <= 448 * 2^s
// (so nothing saturates), clamped to [-127, 127]; code = RNE(x * 2^-s) in
// E4M3 (4 exponent bits, bias 7, 3 fraction bits; largest finite value 448,
// subnormals down to 2^-9).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace osk {

__device__ __forceinline__ int e8m0_exponent(float amax) {
    if (!(amax > 0.f)) return -127;
    int E;
    const float f = frexpf(amax, &E);          // amax = f * 2^E, f in [0.5, 1)
    // 448 = 0.875 * 2^9: amax <= 448 * 2^s  <=>  s >= E - 9 + log2(f / 0.875)
    int s = (f <= 0.875f) ? E - 9 : E - 8;
    return max(-127, min(127, s));
}

// E4M3 code (sign in bit 7) of v, |v| <= 448, round to nearest even.
__device__ __forceinline__ uint32_t e4m3_rne(float v) {
    const uint32_t bits = __float_as_uint(v);
    const uint32_t sign = (bits >> 24) & 0x80u;
    const float a = fabsf(v);
    uint32_t code;
    if (a < 0.015625f) {                        // below 2^-6: subnormal, step 2^-9
        code = (uint32_t)rintf(a * 512.f);      // 0 .. 8 (8 = the smallest normal)
    } else {
        uint32_t u = __float_as_uint(a);        // keep 3 fraction bits, RNE on the 20 dropped
        u += 0x7FFFFu + ((u >> 20) & 1u);
        code = (u >> 20) - (120u << 3);         // exponent bias 127 -> 7
    }
    return sign | code;
}

__device__ __forceinline__ float e4m3_value(uint32_t code) {
    const uint32_t e = (code >> 3) & 0xFu, m = code & 7u;
    const float mag = e ? ldexpf(1.f + (float)m * 0.125f, (int)e - 7) : (float)m * 0.001953125f;
    return (code & 0x80u) ? -mag : mag;
}

}  // namespace osk
