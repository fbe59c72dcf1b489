// hash.hip -- the random choices of the count sketch on the GPU.
//
// Algorithm "Calculating Count-sketch of a matrix A" (Section 4.1) flips
// each index with probability 1/2 and sends it to a uniform bucket of [0, b);
// Eq. (sketch_matrix) uses N+e independent such sketches.  The paper names no
// generator; this library evaluates SplitMix64 (Steele, Lea & Flood, OOPSLA
// 2014) as a counter-based function of (seed, block, index), so every entry
// is computed independently and in parallel:
//   state = seed + (ctr + 1) * golden_gamma,  ctr = (block << 40) | index
//   word  = SplitMix64 output mix of state
//   bucket = high 32 bits of word scaled to [0, b) by multiply-shift
//   sign   = -1 when the low bit of word is set
#include "internal.h"

namespace osk {
namespace {

constexpr uint64_t kGoldenGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t splitmix64_output(uint64_t state) {
    uint64_t w = state;
    w = (w ^ (w >> 30)) * 0xBF58476D1CE4E5B9ull;
    w = (w ^ (w >> 27)) * 0x94D049BB133111EBull;
    return w ^ (w >> 31);
}

__device__ __forceinline__ uint64_t sketch_word(uint64_t seed, uint64_t blk, uint64_t k) {
    const uint64_t ctr = (blk << 40) | k;
    return splitmix64_output(seed + (ctr + 1ull) * kGoldenGamma);
}

__device__ __forceinline__ uint32_t word_bucket(uint64_t w, uint32_t b) {
    return (uint32_t)(((w >> 32) * (uint64_t)b) >> 32);
}

__device__ __forceinline__ uint32_t clamp_bucket(int32_t h, int32_t b) {
    return (uint32_t)(h < 0 ? 0 : (h >= b ? b - 1 : h));
}

// One packed entry per (block, index): bucket in bits 0..30, bit 31 = negative.
__global__ __launch_bounds__(256) void table_hash_kernel(uint64_t seed, int64_t n, int64_t nt,
                                                         uint32_t b, uint32_t* __restrict__ table) {
    const int64_t blk = blockIdx.y;
    uint32_t* row = table + blk * nt;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nt;
         k += (int64_t)gridDim.x * blockDim.x) {
        uint32_t v = 0;
        if (k < n) {
            const uint64_t w = sketch_word(seed, (uint64_t)blk, (uint64_t)k);
            v = word_bucket(w, b) | ((uint32_t)(w & 1ull) << 31);
        }
        row[k] = v;
    }
}

__global__ __launch_bounds__(256) void table_explicit_kernel(const int32_t* __restrict__ h,
                                                             const int8_t* __restrict__ sigma,
                                                             int64_t n, int64_t nt, int32_t b,
                                                             uint32_t* __restrict__ table) {
    const int64_t blk = blockIdx.y;
    uint32_t* row = table + blk * nt;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nt;
         k += (int64_t)gridDim.x * blockDim.x) {
        uint32_t v = 0;
        if (k < n) {
            v = clamp_bucket(h[blk * n + k], b) | (sigma[blk * n + k] < 0 ? 0x80000000u : 0u);
        }
        row[k] = v;
    }
}

__global__ __launch_bounds__(256) void hash_fill_kernel(uint64_t seed, const int32_t* __restrict__ h_in,
                                                        const int8_t* __restrict__ sigma_in, int64_t n,
                                                        int32_t b, int32_t* __restrict__ h_out,
                                                        int8_t* __restrict__ sigma_out) {
    const int64_t blk = blockIdx.y;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t at = blk * n + k;
        if (h_in) {
            h_out[at] = (int32_t)clamp_bucket(h_in[at], b);
            sigma_out[at] = sigma_in[at] < 0 ? (int8_t)-1 : (int8_t)1;
        } else {
            const uint64_t w = sketch_word(seed, (uint64_t)blk, (uint64_t)k);
            h_out[at] = (int32_t)word_bucket(w, (uint32_t)b);
            sigma_out[at] = (w & 1ull) ? (int8_t)-1 : (int8_t)1;
        }
    }
}

// Hash step of many prepared sketches: task t fills 256 indices of one
// block of the descriptor whose hash_task0 range holds t.
__global__ __launch_bounds__(256) void table_batch_kernel(const PrepDesc* __restrict__ descs,
                                                          int32_t count, int64_t tasks) {
    for (int64_t t = blockIdx.x; t < tasks; t += gridDim.x) {
        const int32_t p = find_task(descs, count, t, [](const PrepDesc& d) {
            return d.hash_task0;
        });
        const PrepDesc& d = descs[p];
        const int64_t local = t - d.hash_task0;
        const int64_t blk = local / d.hash_chunks;
        const int64_t k = (local % d.hash_chunks) * 256 + threadIdx.x;
        if (k >= d.nt) continue;
        uint32_t v = 0;
        if (k < d.n) {
            if (d.h) {
                v = clamp_bucket(d.h[blk * d.n + k], d.b) |
                    (d.sigma[blk * d.n + k] < 0 ? 0x80000000u : 0u);
            } else {
                const uint64_t w = sketch_word(d.seed, (uint64_t)blk, (uint64_t)k);
                v = word_bucket(w, (uint32_t)d.b) | ((uint32_t)(w & 1ull) << 31);
            }
        }
        d.table[blk * d.nt + k] = v;
    }
}

dim3 grid_for(int64_t len, int32_t nblk) {
    int64_t gx = (len + 255) / 256;
    if (gx > 4096) gx = 4096;
    if (gx < 1) gx = 1;
    return dim3((unsigned)gx, (unsigned)nblk, 1);
}

}  // namespace

hipError_t launch_table_hash(uint64_t seed, int32_t nblk, int64_t n, int64_t nt, int32_t b,
                             uint32_t* table, hipStream_t s) {
    hipLaunchKernelGGL(table_hash_kernel, grid_for(nt, nblk), dim3(256), 0, s, seed, n, nt,
                       (uint32_t)b, table);
    return hipGetLastError();
}

hipError_t launch_table_explicit(const int32_t* h, const int8_t* sigma, int32_t nblk, int64_t n,
                                 int64_t nt, int32_t b, uint32_t* table, hipStream_t s) {
    hipLaunchKernelGGL(table_explicit_kernel, grid_for(nt, nblk), dim3(256), 0, s, h, sigma, n,
                       nt, b, table);
    return hipGetLastError();
}

hipError_t launch_table_batch(const PrepDesc* descs, int32_t count, int64_t tasks,
                              hipStream_t s) {
    if (count < 1 || tasks < 1) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)(tasks < (int64_t(1) << 20) ? tasks : (int64_t(1) << 20));
    hipLaunchKernelGGL(table_batch_kernel, dim3(grid), dim3(256), 0, s, descs, count, tasks);
    return hipGetLastError();
}

hipError_t launch_hash_fill(uint64_t seed, const int32_t* h_in, const int8_t* sigma_in,
                            int32_t nblk, int64_t n, int32_t b, int32_t* h_out,
                            int8_t* sigma_out, hipStream_t s) {
    hipLaunchKernelGGL(hash_fill_kernel, grid_for(n, nblk), dim3(256), 0, s, seed, h_in,
                       sigma_in, n, b, h_out, sigma_out);
    return hipGetLastError();
}

}  // namespace osk
