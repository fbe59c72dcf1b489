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
#include "fp8.h"

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


// ---------------------------------------------------------------------------
// FP8 (OCP E4M3: 4 exponent bits, bias 7, 3 fraction bits; largest finite
// value 448, subnormals down to 2^-9) with one power-of-two scale per 64
// consecutive values of a row (an E8M0 byte, value 2^(e - 127)), consumed by
// the gfx950 scaled MFMA: one 32x32x64 MFMA covers one scale block, both of
// its 32-value halves taking the same scale.
//
// Per block of 64 values: s = the smallest integer with max|x| <= 448 * 2^s
// (so nothing saturates), clamped to [-127, 127]; code = RNE(x * 2^-s) in
// E4M3.  The split form also quantizes the residual r = x - code * 2^s
// (exact in FP32) with its own scale.
//
// Row layout of the copy (bytes): the codes of the nst blocks (block stride
// bq = b rounded up to 128), the codes of the residual (split), then one
// scale byte per 64 codes in the same order.
// ---------------------------------------------------------------------------
namespace {

// One thread per (row, block of 64 values).
__global__ __launch_bounds__(256) void quant_fp8_kernel(const float* __restrict__ S, int64_t lines,
                                                        int64_t lds, int32_t b, int32_t bp,
                                                        int32_t bq, int32_t nst, int split,
                                                        uint8_t* __restrict__ Q, int64_t ldq) {
    const int64_t zq = (int64_t)nst * bq;               // codes of the high part
    const int64_t width = zq * (split ? 2 : 1);
    const int64_t kb_per_row = zq / kFp8Block;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= kb_per_row * lines) return;
    const int64_t row = t / kb_per_row;
    const int64_t kb = t - row * kb_per_row;
    const int64_t oc = kb * kFp8Block;
    const int32_t j = (int32_t)(oc / bq);
    const int32_t c0 = (int32_t)(oc - (int64_t)j * bq);
    const float* src = S + row * lds + (int64_t)j * bp;
    float x[kFp8Block];
    float amax = 0.f;
#pragma unroll
    for (int u = 0; u < kFp8Block; ++u) {
        x[u] = (c0 + u < b) ? src[c0 + u] : 0.f;
        amax = fmaxf(amax, fabsf(x[u]));
    }
    uint8_t* qrow = Q + row * ldq;
    uint8_t* srow = qrow + width;                       // scale bytes after all codes
    int s = e8m0_exponent(amax);
    uint32_t w[kFp8Block / 4];
    float r[kFp8Block];
    float ramax = 0.f;
#pragma unroll
    for (int u = 0; u < kFp8Block; ++u) {
        const uint32_t c = e4m3_rne(ldexpf(x[u], -s));
        w[u / 4] = (u % 4 == 0 ? 0u : w[u / 4]) | (c << (8 * (u % 4)));
        r[u] = x[u] - ldexpf(e4m3_value(c), s);
        ramax = fmaxf(ramax, fabsf(r[u]));
    }
    uint4* dst = reinterpret_cast<uint4*>(qrow + oc);
#pragma unroll
    for (int v = 0; v < kFp8Block / 16; ++v)
        dst[v] = make_uint4(w[4 * v], w[4 * v + 1], w[4 * v + 2], w[4 * v + 3]);
    srow[kb] = (uint8_t)(s + 127);
    if (split) {
        const int s2 = e8m0_exponent(ramax);
#pragma unroll
        for (int u = 0; u < kFp8Block; ++u) {
            const uint32_t c = e4m3_rne(ldexpf(r[u], -s2));
            w[u / 4] = (u % 4 == 0 ? 0u : w[u / 4]) | (c << (8 * (u % 4)));
        }
        uint4* dlo = reinterpret_cast<uint4*>(qrow + zq + oc);
#pragma unroll
        for (int v = 0; v < kFp8Block / 16; ++v)
            dlo[v] = make_uint4(w[4 * v], w[4 * v + 1], w[4 * v + 2], w[4 * v + 3]);
        srow[kb_per_row + kb] = (uint8_t)(s2 + 127);
    }
}

}  // namespace

int32_t block_stride_fp8(int32_t b) { return (int32_t)round_up(b, 128); }

int64_t fp8_row_bytes(int32_t b, int32_t nst, int split) {
    const int64_t width = (int64_t)nst * block_stride_fp8(b) * (split ? 2 : 1);
    return width + width / kFp8Block;
}

hipError_t launch_quant_fp8(const float* S, int64_t lines, int64_t lds, int32_t b, int32_t nst,
                            int split, void* Q, int64_t ldq, hipStream_t s) {
    const int32_t bp = (int32_t)round_up(b, kBlockAlign);
    const int32_t bq = block_stride_fp8(b);
    const int64_t items = lines * ((int64_t)nst * bq / kFp8Block);
    const int64_t grid = (items + 255) / 256;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(quant_fp8_kernel, dim3((unsigned)grid), dim3(256), 0, s, S, lines, lds, b,
                       bp, bq, nst, split, static_cast<uint8_t*>(Q), ldq);
    return hipGetLastError();
}

}  // namespace osk
