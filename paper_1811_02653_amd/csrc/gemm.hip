// gemm.hip -- grouped FP32 MFMA product over the kept sketch blocks.
//
// Computes C = scale * sum_{j kept} At_j * Bt_j^T, where At_j (m x bp) and
// Bt_j (l x bp) are the j-th column blocks of the sketches of A and B^T.
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
//   - K steps of 32: both operands are K-contiguous, staged through LDS with
//     a padded row stride of 36 floats (conflict-free 128-bit reads); the
//     next step's tile is prefetched into registers during the MFMAs.
//   - Within a 16-deep half step, lane half h of every MFMA reads k = 8h + kk
//     (kk = 0..7), so each lane fetches its 8 operand values of a half step
//     with two 128-bit LDS reads; A and B use the same k order, so the dot
//     products are unchanged (only their summation order differs).
//   - Workgroup -> tile mapping keeps neighbouring tiles on one XCD (shared
//     L2) and rasterises in groups of 4 tile rows.
#include "internal.h"

namespace osk {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int BM = 256;
constexpr int BN = 256;
constexpr int BK = 32;
constexpr int LDK = BK + 4;     // padded LDS row stride (floats)
constexpr int kThreads = 256;
constexpr int kGroupM = 4;

__device__ __forceinline__ int64_t xcd_task(int64_t L, int64_t tasks) {
    if (tasks % 8 != 0) return L;
    return (L % 8) * (tasks / 8) + L / 8;
}

// Global -> register tile loads: thread t covers rows t/8 + 32*i (i < 8) and
// the 4 floats starting at column 4*(t%8) of the 32-wide K step.
__device__ __forceinline__ void load_tile(float4 (&r)[8], const float* __restrict__ base,
                                          int64_t ld, int64_t row0, int64_t nrows, int64_t kcol,
                                          int tid) {
    const int lr = tid >> 3;
    const int lq = tid & 7;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t row = row0 + lr + 32 * i;
        if (row < nrows)
            r[i] = *reinterpret_cast<const float4*>(base + row * ld + kcol + 4 * lq);
        else
            r[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

__device__ __forceinline__ void store_tile(float* __restrict__ s, const float4 (&r)[8], int tid) {
    const int lr = tid >> 3;
    const int lq = tid & 7;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        *reinterpret_cast<float4*>(s + (lr + 32 * i) * LDK + 4 * lq) = r[i];
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_kept_kernel(const float* __restrict__ At, int64_t ldat, const float* __restrict__ Bt,
                      int64_t ldbt, int64_t m, int64_t l, int32_t bp, BlockList kept,
                      int32_t nkept, float scale, float* __restrict__ C, int64_t ldc,
                      int32_t tilesM, int32_t tilesN) {
    __shared__ __align__(16) float As[BM * LDK];
    __shared__ __align__(16) float Bs[BN * LDK];

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
    int64_t kcol = (int64_t)kept.idx[0] * bp;

    float4 ra[8], rb[8];
    load_tile(ra, At, ldat, row0, m, kcol, tid);
    load_tile(rb, Bt, ldbt, col0, l, kcol, tid);

    const int arow = wm * 128 + (lane & 31);
    const int brow = wn * 128 + (lane & 31);
    const int koff = (lane >> 5) * 8;

    for (int t = 0; t < total; ++t) {
        __syncthreads();
        store_tile(As, ra, tid);
        store_tile(Bs, rb, tid);
        __syncthreads();
        if (++kt == tpb) {
            kt = 0;
            ++kb;
            kcol = (kb < nkept) ? (int64_t)kept.idx[kb] * bp : 0;
        } else {
            kcol += BK;
        }
        if (t + 1 < total) {
            load_tile(ra, At, ldat, row0, m, kcol, tid);
            load_tile(rb, Bt, ldbt, col0, l, kcol, tid);
        }
#pragma unroll
        for (int half = 0; half < 2; ++half) {
#pragma unroll
            for (int quad = 0; quad < 2; ++quad) {
                float4 a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    a[i] = *reinterpret_cast<const float4*>(As + (arow + 32 * i) * LDK + half * 16 + koff + 4 * quad);
                    b[i] = *reinterpret_cast<const float4*>(Bs + (brow + 32 * i) * LDK + half * 16 + koff + 4 * quad);
                }
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float av = kk == 0 ? a[i].x : kk == 1 ? a[i].y : kk == 2 ? a[i].z : a[i].w;
                            const float bv = kk == 0 ? b[j].x : kk == 1 ? b[j].y : kk == 2 ? b[j].z : b[j].w;
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[i][j], 0, 0, 0);
                        }
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
