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

// Fragments of one "quad" (4 consecutive k of each lane half) of a 16-deep
// half step: a[i][kk] = A-tile element (k0 + kk, acol + 32 i), likewise b.
__device__ __forceinline__ void read_frag(float (&a)[4][4], float (&b)[4][4],
                                          const float* __restrict__ As,
                                          const float* __restrict__ Bs, int k0, int acol, int bcol) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            a[i][kk] = As[(k0 + kk) * LDT + acol + 32 * i];
            b[i][kk] = Bs[(k0 + kk) * LDT + bcol + 32 * i];
        }
}

__device__ __forceinline__ void mfma_quad(v16f (&acc)[4][4], const float (&a)[4][4],
                                          const float (&b)[4][4]) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][kk], b[j][kk], acc[i][j], 0, 0, 0);
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_kept_kernel(const float* __restrict__ At, int64_t ldat, const float* __restrict__ Bt,
                      int64_t ldbt, int64_t m, int64_t l, int32_t bp, BlockList kept,
                      int32_t nkept, float scale, float* __restrict__ C, int64_t ldc,
                      int32_t tilesM, int32_t tilesN) {
    // two buffers per operand: step t reads buffer t % 2 while the tile of
    // step t + 1 is stored into the other one
    __shared__ __align__(16) float As[2][BK * LDT];
    __shared__ __align__(16) float Bs[2][BK * LDT];

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
    // K row of step `step` (kept blocks in order, BK rows per step)
    auto step_row = [&](int step) -> int64_t {
        return (int64_t)kept.idx[step / tpb] * bp + (int64_t)(step % tpb) * BK;
    };

    // operand element (k, lane's m or n) lives at [k * LDT + col]
    const int acol = wm * 128 + (lane & 31);
    const int bcol = wn * 128 + (lane & 31);
    const int krow_lane = 8 * (lane >> 5);
    // first k of quad q (0..3): half q / 2, lane half's 8 rows, 4 per quad
    auto quad_k = [&](int q) { return (q >> 1) * 16 + krow_lane + 4 * (q & 1); };

    float4 ra[8], rb[8];
    load_tile(ra, At, ldat, row0, m, step_row(0), tid);
    load_tile(rb, Bt, ldbt, col0, l, step_row(0), tid);
    store_tile(As[0], ra, tid);
    store_tile(Bs[0], rb, tid);
    if (total > 1) {
        load_tile(ra, At, ldat, row0, m, step_row(1), tid);
        load_tile(rb, Bt, ldbt, col0, l, step_row(1), tid);
    }
    __syncthreads();

    float fa[4][4], fb[4][4], ga[4][4], gb[4][4];
    read_frag(fa, fb, As[0], Bs[0], quad_k(0), acol, bcol);
    for (int t = 0; t < total; ++t) {
        const int cur = t & 1;
        const float* as = As[cur];
        const float* bs = Bs[cur];
        read_frag(ga, gb, as, bs, quad_k(1), acol, bcol);
        mfma_quad(acc, fa, fb);
        read_frag(fa, fb, as, bs, quad_k(2), acol, bcol);
        mfma_quad(acc, ga, gb);
        // the next step's tile goes into the other buffer (last read before
        // the previous step's barrier); the loads for the step after are
        // issued a whole step ahead of their use
        if (t + 1 < total) {
            store_tile(As[cur ^ 1], ra, tid);
            store_tile(Bs[cur ^ 1], rb, tid);
            if (t + 2 < total) {
                load_tile(ra, At, ldat, row0, m, step_row(t + 2), tid);
                load_tile(rb, Bt, ldbt, col0, l, step_row(t + 2), tid);
            }
        }
        read_frag(ga, gb, as, bs, quad_k(3), acol, bcol);
        mfma_quad(acc, fa, fb);
        mfma_quad(acc, ga, gb);
        __syncthreads();
        if (t + 1 < total) read_frag(fa, fb, As[cur ^ 1], Bs[cur ^ 1], quad_k(0), acol, bcol);
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
