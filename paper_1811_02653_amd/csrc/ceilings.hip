// ceilings.hip -- measured ceilings of the units the sketched product's
// kernels are bound by, on the GPU the benchmark runs on: HBM streaming
// (copy and read-only), the FP32 / BF16 / FP8 MFMA pipes, and 16-byte LDS
// gathers at random and at conflict-free addresses (the sketch kernel's
// inner access).  Each kernel does only that one thing, with enough
// independent work per wave to keep its unit busy; the benchmark times them
// and reports every kernel's rate as a fraction of both the published peak
// and these measured ceilings.  Not part of the sketched product.
//
// Built into libosk_ceilings.so (separate from liboversketch.so); the C
// entry points take plain device pointers and a HIP stream.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// dst[i] = src[i] for i < n4 (16-byte elements), grid-stride.
__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src,
                                                   float4* __restrict__ dst, int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        dst[i] = src[i];
}

// Reads src[0, n4) once (16-byte elements, four loads in flight per lane)
// and writes one float per thread (so the reads are not removed).
__global__ __launch_bounds__(256) void read_kernel(const float4* __restrict__ src, int64_t n4,
                                                   float* __restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float s = 0.f;
    int64_t i = t;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride],
                     d = src[i + 3 * stride];
        s += a.x + b.y + c.z + d.w;
    }
    for (; i < n4; i += stride) s += src[i].x;
    sink[t] = s;
}

// kChains independent 32x32 accumulators per wave, iters MFMAs on each.
constexpr int kChains = 4;

template <int kKind>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void mfma_kernel(int iters, float* __restrict__ out) {
    v16f acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.f;
    const int lane = threadIdx.x & 63;
    const float fa = 1.0f + lane * 1e-3f;
    bf16x8 ba, bb;
    i32x8 ia, ib;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        ba[k] = (__bf16)(fa + k);
        bb[k] = (__bf16)(1.0f - k * 1e-2f);
        ia[k] = 0x38383838 + lane;     // E4M3 codes near 1.0
        ib[k] = 0x30303030;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (kKind == 0)
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa, 0.5f, acc[c], 0, 0, 0);
            else if constexpr (kKind == 1)
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ba, bb, acc[c], 0, 0, 0);
            else
                acc[c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(ia, ib, acc[c], 0, 0, 0,
                                                                         127, 0, 127);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) s += acc[c][r];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 16-byte LDS gathers from a 128 KiB buffer, 8 reads in flight per lane,
// then a running sum (as the sketch's summing loop: read, then add).
// random = 1: lane addresses from a per-lane xorshift stream (bank conflicts
// as random bucket lists have them); random = 0: lane-consecutive slots.
constexpr int kSlots = 8192;          // 16-byte slots: 128 KiB

__global__ __launch_bounds__(512) void lds_gather_kernel(int iters, int random,
                                                         float* __restrict__ out) {
    __shared__ float4 buf[kSlots];
    for (int i = threadIdx.x; i < kSlots; i += blockDim.x)
        buf[i] = make_float4(i * 1e-3f, 1.f, 2.f, 3.f);
    __syncthreads();
    uint32_t x = 0x9E3779B9u * (threadIdx.x + 1) + blockIdx.x;
    const int lane = threadIdx.x & 63;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int it = 0; it < iters; ++it) {
        int slot[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (random) {
                x ^= x << 13;
                x ^= x >> 17;
                x ^= x << 5;
                slot[u] = (int)(x & (kSlots - 1));
            } else {
                slot[u] = ((it * 8 + u) * 64 + lane) & (kSlots - 1);
            }
        }
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = buf[slot[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            acc.x += v[u].x;
            acc.y += v[u].y;
            acc.z += v[u].z;
            acc.w += v[u].w;
        }
    }
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

}  // namespace

extern "C" {

// dst = src, n4 16-byte elements (both 16-byte aligned); 0 on success, else
// the hipError_t of the launch.
int osk_ceiling_copy(const void* src, void* dst, int64_t n4, int grid, void* stream) {
    if (!src || !dst || n4 < 1 || grid < 1) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n4);
    return (int)hipGetLastError();
}

// Reads src (n4 16-byte elements); sink holds grid * 256 floats.
int osk_ceiling_read(const void* src, int64_t n4, float* sink, int grid, void* stream) {
    if (!src || !sink || n4 < 1 || grid < 1) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(read_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                       static_cast<const float4*>(src), n4, sink);
    return (int)hipGetLastError();
}

// kind 0 = FP32 32x32x2, 1 = BF16 32x32x16, 2 = FP8 (E4M3, scaled) 32x32x64;
// grid workgroups of 512 threads, each wave iters * 4 MFMAs; out holds
// grid * 512 floats.  Flops per launch: grid * 8 * iters * 4 * (32*32*2*k).
int osk_ceiling_mfma(int kind, int iters, int grid, float* out, void* stream) {
    if (!out || iters < 1 || grid < 1) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    if (kind == 0)
        hipLaunchKernelGGL(mfma_kernel<0>, dim3((unsigned)grid), dim3(512), 0, s, iters, out);
    else if (kind == 1)
        hipLaunchKernelGGL(mfma_kernel<1>, dim3((unsigned)grid), dim3(512), 0, s, iters, out);
    else if (kind == 2)
        hipLaunchKernelGGL(mfma_kernel<2>, dim3((unsigned)grid), dim3(512), 0, s, iters, out);
    else
        return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

// grid workgroups of 512 threads (one per CU: 128 KiB of LDS each), each
// lane iters * 8 16-byte LDS reads; out holds grid * 512 floats.
int osk_ceiling_lds_gather(int iters, int random, int grid, float* out, void* stream) {
    if (!out || iters < 1 || grid < 1) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(lds_gather_kernel, dim3((unsigned)grid), dim3(512), 0,
                       (hipStream_t)stream, iters, random, out);
    return (int)hipGetLastError();
}

}  // extern "C"
