// quant.hip -- low-precision copies of a line-major FP32 sketch for the
// block product.
//
// BF16: every value is rounded to nearest even (v_cvt_pk_bf16_f32).  BF16
// keeps FP32's exponent range, so no scaling is needed.  The split form also
// stores the residual lo = bf16(x - hi), so that hi*hi' + hi*lo' + lo*hi'
// recovers the product to about 2^-16 relative (the lo*lo' term is below
// FP32 rounding of the sum and is dropped).
//
// Layout: block j of the FP32 sketch (columns j*bp .. j*bp + bp - 1) becomes
// columns j*bpq .. j*bpq + bpq - 1 of the BF16 copy, bpq = b rounded up to 64
// (the BF16 K step); columns at or past b are zero.  The low parts follow the
// high parts: column nst*bpq + j*bpq + c.
#include "internal.h"

namespace osk {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// One thread writes 8 consecutive BF16 values (16 bytes) of one row of the
// high part and, when split, the same 8 of the low part.
__global__ __launch_bounds__(256) void quant_bf16_kernel(const float* __restrict__ S, int64_t lines,
                                                         int64_t lds, int32_t b, int32_t bp,
                                                         int32_t bpq, int32_t nst, int split,
                                                         __bf16* __restrict__ Q, int64_t ldq) {
    const int64_t zq = (int64_t)nst * bpq;
    const int64_t per_row = zq / 8;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= per_row * lines) return;
    const int64_t row = t / per_row;
    const int64_t oc = (t - row * per_row) * 8;          // first output column
    const int32_t j = (int32_t)(oc / bpq);
    const int32_t c0 = (int32_t)(oc - (int64_t)j * bpq);
    const float* src = S + row * lds + (int64_t)j * bp;
    float x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = (c0 + u < b) ? src[c0 + u] : 0.f;
    bf16x8 hi, lo;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        hi[u] = (__bf16)x[u];
        lo[u] = (__bf16)(x[u] - (float)hi[u]);
    }
    __bf16* dst = Q + row * ldq + oc;
    *reinterpret_cast<bf16x8*>(dst) = hi;
    if (split) *reinterpret_cast<bf16x8*>(dst + zq) = lo;
}

}  // namespace

int32_t block_stride_bf16(int32_t b) { return (int32_t)round_up(b, 64); }

hipError_t launch_quant_bf16(const float* S, int64_t lines, int64_t lds, int32_t b, int32_t nst,
                             int split, void* Q, int64_t ldq, hipStream_t s) {
    const int32_t bp = (int32_t)round_up(b, kBlockAlign);
    const int32_t bpq = block_stride_bf16(b);
    const int64_t items = lines * ((int64_t)nst * bpq / 8);
    const int64_t grid = (items + 255) / 256;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(quant_bf16_kernel, dim3((unsigned)grid), dim3(256), 0, s, S, lines, lds, b,
                       bp, bpq, nst, split, static_cast<__bf16*>(Q), ldq);
    return hipGetLastError();
}

}  // namespace osk
