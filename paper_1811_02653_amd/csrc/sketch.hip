// sketch.hip -- count-sketch kernels for gfx950.
//
// Both kernels apply the blocks of S (Eq. (sketch_matrix)) to one operand:
// every input element x at sketched index k is added, with sign
// sigma_i(k), into bucket h_i(k) of every stored block i (Algorithm
// "Calculating Count-sketch of a matrix A", applied per block as in
// Algorithm "Over sketching A in parallel").  The paper notes that the
// count sketch streams over its input (the "memory constrained distributed
// sketching" remark of Section 4.1); both kernels stream the operand once
// from HBM in order and keep the buckets of the lines they own in LDS.
//
// sketch_cols: X is rows x n row-major and the sketched index runs along a
//   row (contiguous).  Lanes walk k (coalesced float4 reads), each wave owns
//   RW whole rows, and the buckets of those rows for G blocks live in LDS.
//   The scatter is a ds_add_f32 per (element, block) at a data-dependent
//   bucket; a wave owns its rows, so the order of additions into a bucket is
//   fixed and results are bitwise reproducible.
// sketch_rows: X is n x cols row-major and the sketched index runs down the
//   columns (strided).  Lanes walk the columns of a strip of WC columns, so
//   the bucket of a row is the same for all lanes reading it (no bank
//   conflicts); LDS holds bucket rows x WC columns for G blocks.  Workgroups
//   sharing a strip are placed on one XCD so the strip is read from HBM once
//   and re-read from that XCD's L2.
#include "internal.h"

#include <mutex>

namespace osk {
namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kColsMaxSlots = 10;   // blocks per workgroup, sketch_cols
constexpr int kRowsMaxSlots = 4;    // blocks per workgroup, sketch_rows

__device__ __forceinline__ float flip_sign(float v, uint32_t signbit) {
    return __uint_as_float(__float_as_uint(v) ^ signbit);
}

__device__ __forceinline__ void lds_add(float* p, float v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Spread consecutive task ids over the 8 XCDs in contiguous runs: task T is
// run by the workgroup with linear id L where T = (L % 8) * (tasks / 8) + L / 8,
// so neighbouring tasks (same strip / same rows) share an XCD and its L2.
__device__ __forceinline__ int64_t xcd_task(int64_t L, int64_t tasks) {
    if (tasks % 8 != 0) return L;
    return (L % 8) * (tasks / 8) + L / 8;
}

// ---------------------------------------------------------------------------
// sketch_cols
// ---------------------------------------------------------------------------
template <int RW>
struct ColsChunk {
    float4 x[RW];
    uint4 e[kColsMaxSlots];
};

template <int RW>
__device__ __forceinline__ void cols_load(ColsChunk<RW>& c, const float* const* xrow, bool live,
                                          int64_t k, int64_t n, const uint32_t* const* trow,
                                          int gn) {
    if (!live || k >= n) return;
#pragma unroll
    for (int rr = 0; rr < RW; ++rr) {
        if (k + 3 < n) {
            c.x[rr] = *reinterpret_cast<const float4*>(xrow[rr] + k);
        } else {
            const float* p = xrow[rr] + k;
            c.x[rr] = make_float4(p[0], (k + 1 < n) ? p[1] : 0.f, (k + 2 < n) ? p[2] : 0.f, 0.f);
        }
    }
#pragma unroll
    for (int g = 0; g < kColsMaxSlots; ++g)
        if (g < gn) c.e[g] = *reinterpret_cast<const uint4*>(trow[g] + k);
}

template <int RW>
__device__ __forceinline__ void cols_scatter(const ColsChunk<RW>& c, bool live, int64_t k, int64_t n,
                                             char* wave_acc, uint32_t slot_bytes, int gn) {
    constexpr int kShift = 2 + (RW == 4 ? 2 : (RW == 2 ? 1 : 0));
    if (!live || k >= n) return;
#pragma unroll
    for (int g = 0; g < kColsMaxSlots; ++g) {
        if (g < gn) {
            const uint32_t base = g * slot_bytes;
            const uint32_t ev[4] = {c.e[g].x, c.e[g].y, c.e[g].z, c.e[g].w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // bucket h in bits 0..30: byte offset h*RW*4 (the shift drops the sign bit)
                float* p = reinterpret_cast<float*>(wave_acc + ((ev[q] << kShift) + base));
                const uint32_t sg = ev[q] & 0x80000000u;
#pragma unroll
                for (int rr = 0; rr < RW; ++rr) {
                    const float xv = (q == 0) ? c.x[rr].x : (q == 1) ? c.x[rr].y : (q == 2) ? c.x[rr].z : c.x[rr].w;
                    lds_add(p + rr, flip_sign(xv, sg));
                }
            }
        }
    }
}

// LDS layout per wave: acc[(g*bp + h)*RW + rr], g < G, h < bp, rr < RW.
template <int RW>
__global__ __launch_bounds__(kThreads) void sketch_cols_kernel(
    const float* __restrict__ X, int64_t rows, int64_t n, int64_t ldx,
    const uint32_t* __restrict__ table, int64_t nt, BlockList bl, int32_t nst, int32_t bp,
    int32_t G, int64_t nslices, float* __restrict__ out, int64_t ldo) {
    extern __shared__ __align__(16) float acc[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t rowgroups = (rows + kWaves * RW - 1) / (kWaves * RW);
    const int64_t task = xcd_task(blockIdx.x, rowgroups * nslices);
    const int64_t rg = task / nslices;
    const int slice = (int)(task % nslices);
    const int g0 = slice * G;
    const int gn = min(G, nst - g0);
    const int64_t wave_floats = (int64_t)G * bp * RW;

    for (int64_t i = threadIdx.x * 4; i < kWaves * wave_floats; i += kThreads * 4)
        *reinterpret_cast<float4*>(acc + i) = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();

    const int64_t r0 = rg * (kWaves * RW) + (int64_t)wave * RW;
    const bool live = r0 < rows;   // wave-uniform
    const float* xrow[RW];
#pragma unroll
    for (int rr = 0; rr < RW; ++rr) xrow[rr] = X + min(r0 + rr, rows - 1) * ldx;
    const uint32_t* trow[kColsMaxSlots];
#pragma unroll
    for (int g = 0; g < kColsMaxSlots; ++g)
        trow[g] = table + (int64_t)bl.idx[g0 + (g < gn ? g : 0)] * nt;
    char* wave_acc = reinterpret_cast<char*>(acc + wave * wave_floats);
    const uint32_t slot_bytes = (uint32_t)bp * RW * 4u;

    // Rows past the end (r0 + rr >= rows) alias the last row: their buckets
    // are accumulated but never written out.
    ColsChunk<RW> a, b;
    int64_t k0 = 0;
    cols_load<RW>(a, xrow, live, k0 + lane * 4, n, trow, gn);
    while (live) {
        if (k0 + 256 < n) cols_load<RW>(b, xrow, live, k0 + 256 + lane * 4, n, trow, gn);
        cols_scatter<RW>(a, live, k0 + lane * 4, n, wave_acc, slot_bytes, gn);
        k0 += 256;
        if (k0 >= n) break;
        if (k0 + 256 < n) cols_load<RW>(a, xrow, live, k0 + 256 + lane * 4, n, trow, gn);
        cols_scatter<RW>(b, live, k0 + lane * 4, n, wave_acc, slot_bytes, gn);
        k0 += 256;
        if (k0 >= n) break;
    }
    __syncthreads();

    if (!live) return;
    const float* wa = acc + wave * wave_floats;
    const int64_t width = (int64_t)gn * bp;
    for (int64_t j = lane * 4; j < width; j += 256) {
        float v[4 * RW];
#pragma unroll
        for (int t = 0; t < RW; ++t) {
            const float4 f = *reinterpret_cast<const float4*>(wa + j * RW + 4 * t);
            v[4 * t + 0] = f.x; v[4 * t + 1] = f.y; v[4 * t + 2] = f.z; v[4 * t + 3] = f.w;
        }
#pragma unroll
        for (int rr = 0; rr < RW; ++rr) {
            if (r0 + rr < rows) {
                float* o = out + (r0 + rr) * ldo + (int64_t)g0 * bp + j;
                *reinterpret_cast<float4*>(o) =
                    make_float4(v[0 * RW + rr], v[1 * RW + rr], v[2 * RW + rr], v[3 * RW + rr]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// sketch_rows
// ---------------------------------------------------------------------------
// LDS layout: acc[(g*bp + h)*WC + col].  A wave instruction covers RPI =
// 64/WC rows x WC columns.
template <int WC>
__global__ __launch_bounds__(kThreads) void sketch_rows_kernel(
    const float* __restrict__ X, int64_t n, int64_t cols, int64_t ldx,
    const uint32_t* __restrict__ table, int64_t nt, BlockList bl, int32_t nst, int32_t bp,
    int32_t G, int64_t nslices, float* __restrict__ outT, int64_t ldo) {
    constexpr int RPI = 64 / WC;
    constexpr int kShift = 2 + (WC == 64 ? 6 : WC == 32 ? 5 : WC == 16 ? 4 : WC == 8 ? 3 : WC == 4 ? 2 : WC == 2 ? 1 : 0);
    constexpr int U = 4;   // rows per lane in flight
    extern __shared__ __align__(16) float acc[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane % WC;
    const int sub = lane / WC;
    const int64_t strips = (cols + WC - 1) / WC;
    const int64_t task = xcd_task(blockIdx.x, strips * nslices);
    const int64_t strip = task / nslices;
    const int slice = (int)(task % nslices);
    const int g0 = slice * G;
    const int gn = min(G, nst - g0);
    const int64_t j0 = strip * WC;
    const int64_t acc_floats = (int64_t)G * bp * WC;

    for (int64_t i = threadIdx.x * 4; i < acc_floats; i += kThreads * 4)
        *reinterpret_cast<float4*>(acc + i) = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();

    const bool cv = j0 + col < cols;
    const float* xcol = X + (cv ? j0 + col : 0);
    const uint32_t* trow[kRowsMaxSlots];
    uint32_t lbase[kRowsMaxSlots];
#pragma unroll
    for (int g = 0; g < kRowsMaxSlots; ++g) {
        trow[g] = table + (int64_t)bl.idx[g0 + (g < gn ? g : 0)] * nt;
        lbase[g] = (uint32_t)(g * bp * WC + col) * 4u;
    }
    char* accb = reinterpret_cast<char*>(acc);

    const int64_t step = (int64_t)kWaves * RPI;          // rows per WG instruction
    const int64_t kfirst = (int64_t)wave * RPI + sub;
    for (int64_t kb = kfirst; kb < n; kb += step * U) {
        float xv[U];
        uint32_t ev[U][kRowsMaxSlots];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = kb + u * step;
            const bool ok = k < n;
            xv[u] = (ok && cv) ? xcol[k * ldx] : 0.f;
#pragma unroll
            for (int g = 0; g < kRowsMaxSlots; ++g)
                ev[u][g] = (ok && g < gn) ? trow[g][k] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (kb + u * step < n) {
#pragma unroll
                for (int g = 0; g < kRowsMaxSlots; ++g) {
                    if (g < gn) {
                        const uint32_t e = ev[u][g];
                        float* p = reinterpret_cast<float*>(accb + ((e << kShift) + lbase[g]));
                        lds_add(p, flip_sign(xv[u], e & 0x80000000u));
                    }
                }
            }
        }
    }
    __syncthreads();

    // outT[j0 + jj][g0*bp + c] = acc[c*WC + jj]
    constexpr int CG = kThreads / WC;                    // column groups of 4 buckets
    const int jj = threadIdx.x % WC;
    const int cgi = threadIdx.x / WC;
    const int64_t width = (int64_t)gn * bp;
    if (j0 + jj < cols) {
        float* orow = outT + (j0 + jj) * ldo + (int64_t)g0 * bp;
        for (int64_t c = 4 * (int64_t)cgi; c < width; c += 4 * CG) {
            const float4 v = make_float4(acc[(c + 0) * WC + jj], acc[(c + 1) * WC + jj],
                                         acc[(c + 2) * WC + jj], acc[(c + 3) * WC + jj]);
            *reinterpret_cast<float4*>(orow + c) = v;
        }
    }
}

// Dynamic LDS above 64 KiB: raise the per-kernel limit once per instantiation.
template <typename F>
void allow_full_lds(F* kernel) {
    static std::once_flag once;
    std::call_once(once, [kernel] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    });
}

}  // namespace

ColsPlan plan_sketch_cols(int64_t rows, int32_t nst, int32_t bp, int rw, int g) {
    ColsPlan p{};
    const int64_t row_bytes = (int64_t)bp * 4;
    if (rows < 1 || nst < 1 || bp < kBlockAlign || bp % kBlockAlign) return p;
    // Rows per wave: more rows share each table read; prefer 4, then 2,
    // while two blocks of every row still fit in LDS.
    if (rw == 0) {
        rw = 1;
        if ((int64_t)kWaves * 4 * 2 * row_bytes <= kLdsBytes) rw = 4;
        else if ((int64_t)kWaves * 2 * 2 * row_bytes <= kLdsBytes) rw = 2;
    }
    if (rw != 1 && rw != 2 && rw != 4) return p;
    int64_t gmax = kLdsBytes / ((int64_t)kWaves * rw * row_bytes);
    if (gmax < 1) return p;
    if (gmax > kColsMaxSlots) gmax = kColsMaxSlots;
    if (g > 0 && g < gmax) gmax = g;
    // same number of slices, fewest blocks per slice
    p.nslices = (nst + gmax - 1) / gmax;
    p.g = (int)((nst + p.nslices - 1) / p.nslices);
    p.rw = rw;
    p.lds = (size_t)kWaves * rw * p.g * row_bytes;
    p.tasks = (rows + kWaves * rw - 1) / (kWaves * rw) * p.nslices;
    p.valid = p.tasks <= 0x7fffffff;
    return p;
}

RowsPlan plan_sketch_rows(int64_t cols, int32_t nst, int32_t bp, int wc, int g) {
    RowsPlan p{};
    const int64_t bucket_bytes = (int64_t)bp * 4;
    if (cols < 1 || nst < 1 || bp < kBlockAlign || bp % kBlockAlign) return p;
    if (wc == 0) {
        wc = 64;
        while (wc > 1 && (int64_t)wc * bucket_bytes > kLdsBytes) wc >>= 1;
    }
    if (wc < 1 || wc > 64 || (wc & (wc - 1)) || (int64_t)wc * bucket_bytes > kLdsBytes) return p;
    int64_t gmax = kLdsBytes / ((int64_t)wc * bucket_bytes);
    if (gmax > kRowsMaxSlots) gmax = kRowsMaxSlots;
    if (g > 0 && g < gmax) gmax = g;
    p.nslices = (nst + gmax - 1) / gmax;
    p.g = (int)((nst + p.nslices - 1) / p.nslices);
    p.wc = wc;
    p.lds = (size_t)wc * p.g * bucket_bytes;
    p.tasks = (cols + wc - 1) / wc * p.nslices;
    p.valid = p.tasks <= 0x7fffffff;
    return p;
}

hipError_t launch_sketch_cols(const float* X, int64_t rows, int64_t n, int64_t ldx,
                              const uint32_t* table, int64_t nt, const BlockList& bl,
                              int32_t nst, int32_t bp, float* out, int64_t ldo,
                              const ColsPlan& p, hipStream_t s) {
    if (!p.valid) return hipErrorInvalidValue;
    switch (p.rw) {
#define OSK_COLS(R)                                                                                  \
    case R:                                                                                          \
        allow_full_lds(sketch_cols_kernel<R>);                                                       \
        hipLaunchKernelGGL(sketch_cols_kernel<R>, dim3((unsigned)p.tasks), dim3(kThreads), p.lds, s, \
                           X, rows, n, ldx, table, nt, bl, nst, bp, p.g, p.nslices, out, ldo);       \
        return hipGetLastError();
        OSK_COLS(1)
        OSK_COLS(2)
        OSK_COLS(4)
#undef OSK_COLS
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sketch_rows(const float* X, int64_t n, int64_t cols, int64_t ldx,
                              const uint32_t* table, int64_t nt, const BlockList& bl,
                              int32_t nst, int32_t bp, float* outT, int64_t ldo,
                              const RowsPlan& p, hipStream_t s) {
    if (!p.valid) return hipErrorInvalidValue;
    switch (p.wc) {
#define OSK_ROWS(W)                                                                                  \
    case W:                                                                                          \
        allow_full_lds(sketch_rows_kernel<W>);                                                       \
        hipLaunchKernelGGL(sketch_rows_kernel<W>, dim3((unsigned)p.tasks), dim3(kThreads), p.lds, s, \
                           X, n, cols, ldx, table, nt, bl, nst, bp, p.g, p.nslices, outT, ldo);      \
        return hipGetLastError();
        OSK_ROWS(64)
        OSK_ROWS(32)
        OSK_ROWS(16)
        OSK_ROWS(8)
        OSK_ROWS(4)
        OSK_ROWS(2)
        OSK_ROWS(1)
#undef OSK_ROWS
    }
    return hipErrorInvalidValue;
}

}  // namespace osk
