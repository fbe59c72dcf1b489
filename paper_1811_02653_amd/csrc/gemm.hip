// gemm.hip -- grouped FP32 MFMA product over the kept sketch blocks.
//
// Computes C = scale * sum_{j kept} At_j^T * Bt_j, where At_j (bp x m) and
// Bt_j (bp x l) are the j-th row blocks of the bucket-major sketches
// (A S)^T and S^T B.
// This is the computation phase and the reduction phase of Algorithm
// "OverSketch" fused into one K loop: the paper's b x b worker products
// A_tilde(i,k) B_tilde(k,j) for the blocks that returned (Fig. (bMM)) are
// summed in registers instead of through storage, and blocks that
// straggled are skipped by walking only the kept-block list.
//
// Design (gfx950, FP32 MFMA v_mfma_f32_32x32x2_f32):
//   - 256 x 256 output tile per workgroup of 4 waves; each wave owns a
//     128 x 128 sub-tile = 4 x 4 MFMA blocks of 32 x 32 (256 accumulators
//     per lane, kept in AGPRs).
//   - K steps of 32: both operands are K-major (a K row holds 256 contiguous
//     m or l values, read as 1 KiB per wave instruction), staged through LDS
//     with a row stride of 260 floats so the two lane halves of an operand
//     read (k and k + 8) fall in disjoint banks; the next step's tile is
//     prefetched into registers during the MFMAs.
//   - Within a 16-deep half step, lane half h of every MFMA reads k = 8h + kk
//     (kk = 0..7); A and B use the same k order, so the dot products are
//     unchanged (only their summation order differs).
//   - Workgroup -> tile mapping keeps neighbouring tiles on one XCD (shared
//     L2) and rasterises in groups of 4 tile rows.
#include "internal.h"

namespace osk {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int BM = 256;
constexpr int BN = 256;
constexpr int BK = 32;
constexpr int LDT = 260;        // LDS row stride (floats) of a K row of a tile
constexpr int kThreads = 256;
constexpr int kGroupM = 4;

__device__ __forceinline__ int64_t xcd_task(int64_t L, int64_t tasks) {
    if (tasks % 8 != 0) return L;
    return (L % 8) * (tasks / 8) + L / 8;
}

// Global -> register tile loads: wave w covers K rows 8w .. 8w+7 of the step;
// lane L the 4 values at column 4L of the 256-wide tile.  Columns at or past
// `ncols` load zero (a float4 that starts below ncols stays inside the row,
// whose leading dimension is a multiple of 4 and >= ncols).
__device__ __forceinline__ void load_tile(float4 (&r)[8], const float* __restrict__ base,
                                          int64_t ld, int64_t col0, int64_t ncols, int64_t krow,
                                          int tid) {
    const int w = tid >> 6;
    const int64_t col = col0 + 4 * (tid & 63);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (col < ncols)
            r[i] = *reinterpret_cast<const float4*>(base + (krow + 8 * w + i) * ld + col);
        else
            r[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

__device__ __forceinline__ void store_tile(float* __restrict__ s, const float4 (&r)[8], int tid) {
    const int w = tid >> 6;
    const int c = 4 * (tid & 63);
#pragma unroll
    for (int i = 0; i < 8; ++i) *reinterpret_cast<float4*>(s + (8 * w + i) * LDT + c) = r[i];
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_kept_kernel(const float* __restrict__ At, int64_t ldat, const float* __restrict__ Bt,
                      int64_t ldbt, int64_t m, int64_t l, int32_t bp, BlockList kept,
                      int32_t nkept, float scale, float* __restrict__ C, int64_t ldc,
                      int32_t tilesM, int32_t tilesN) {
    __shared__ __align__(16) float As[BK * LDT];
    __shared__ __align__(16) float Bs[BK * LDT];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1;
    const int wn = wave & 1;

    const int64_t ntiles = (int64_t)tilesM * tilesN;
    const int64_t T = xcd_task(blockIdx.x, ntiles);
    const int64_t group = T / ((int64_t)kGroupM * tilesN);
    const int64_t first_m = group * kGroupM;
    const int64_t gsz = min((int64_t)kGroupM, (int64_t)tilesM - first_m);
    const int64_t in_group = T - group * kGroupM * tilesN;
    const int64_t tm = first_m + in_group % gsz;
    const int64_t tn = in_group / gsz;
    const int64_t row0 = tm * BM;
    const int64_t col0 = tn * BN;

    v16f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int tpb = bp / BK;                       // K steps per block
    const int total = nkept * tpb;
    int kb = 0, kt = 0;
    int64_t krow = (int64_t)kept.idx[0] * bp;

    float4 ra[8], rb[8];
    load_tile(ra, At, ldat, row0, m, krow, tid);
    load_tile(rb, Bt, ldbt, col0, l, krow, tid);

    // operand element (k, lane's m or n) lives at [k * LDT + col]
    const int acol = wm * 128 + (lane & 31);
    const int bcol = wn * 128 + (lane & 31);
    const int krow_lane = 8 * (lane >> 5);

    for (int t = 0; t < total; ++t) {
        __syncthreads();
        store_tile(As, ra, tid);
        store_tile(Bs, rb, tid);
        __syncthreads();
        if (++kt == tpb) {
            kt = 0;
            ++kb;
            krow = (kb < nkept) ? (int64_t)kept.idx[kb] * bp : 0;
        } else {
            krow += BK;
        }
        if (t + 1 < total) {
            load_tile(ra, At, ldat, row0, m, krow, tid);
            load_tile(rb, Bt, ldbt, col0, l, krow, tid);
        }
#pragma unroll
        for (int half = 0; half < 2; ++half) {
#pragma unroll
            for (int quad = 0; quad < 2; ++quad) {
                float a[4][4], b[4][4];
                const int k0 = half * 16 + krow_lane + 4 * quad;
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        a[i][kk] = As[(k0 + kk) * LDT + acol + 32 * i];
                        b[i][kk] = Bs[(k0 + kk) * LDT + bcol + 32 * i];
                    }
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][kk], b[j][kk],
                                                                             acc[i][j], 0, 0, 0);
            }
        }
    }

    // 32x32 accumulator layout: register r of lane L holds row
    // 8*(r/4) + 4*(L/32) + r%4 and column L%32 of the block.
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t col = col0 + wn * 128 + j * 32 + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + wm * 128 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row < m && col < l) C[row * ldc + col] = acc[i][j][r] * scale;
            }
        }
    }
}

}  // namespace

bool plan_gemm_ok(int64_t m, int64_t l, int32_t bp) {
    if (m < 1 || l < 1 || bp < BK || bp % BK) return false;
    const int64_t tilesM = (m + BM - 1) / BM;
    const int64_t tilesN = (l + BN - 1) / BN;
    return tilesM * tilesN <= 0x7fffffff;
}

hipError_t launch_gemm_kept(const float* At, int64_t ldat, const float* Bt, int64_t ldbt,
                            int64_t m, int64_t l, int32_t bp, const BlockList& kept,
                            int32_t nkept, float scale, float* C, int64_t ldc, hipStream_t s) {
    if (!plan_gemm_ok(m, l, bp) || nkept < 1) return hipErrorInvalidValue;
    const int64_t tilesM = (m + BM - 1) / BM;
    const int64_t tilesN = (l + BN - 1) / BN;
    hipLaunchKernelGGL(gemm_kept_kernel, dim3((unsigned)(tilesM * tilesN)), dim3(kThreads), 0, s,
                       At, ldat, Bt, ldbt, m, l, bp, kept, nkept, scale, C, ldc, (int32_t)tilesM,
                       (int32_t)tilesN);
    return hipGetLastError();
}

}  // namespace osk
