// internal.h -- shared declarations of the HIP translation units of
// liboversketch.so (not installed; the public interface is oversketch.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/oversketch.h"

namespace osk {

// gfx950 allows 160 KiB of LDS per workgroup.
constexpr int kLdsBytes = 163840;
// Every sketched block is padded to a multiple of this many columns, which
// is also the K depth of one GEMM main-loop step.
constexpr int kBlockAlign = 32;

// Stored-block -> sketch-block index map, passed by value as a kernel
// argument (OS_MAX_BLOCKS entries).
struct BlockList {
    int32_t idx[OS_MAX_BLOCKS];
};

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Launchers (return the hipError_t of the launch).
hipError_t launch_table_hash(uint64_t seed, int32_t nblk, int64_t n, int64_t nt, int32_t b,
                             uint32_t* table, hipStream_t s);
hipError_t launch_table_explicit(const int32_t* h, const int8_t* sigma, int32_t nblk, int64_t n,
                                 int64_t nt, int32_t b, uint32_t* table, hipStream_t s);
hipError_t launch_hash_fill(uint64_t seed, const int32_t* h_in, const int8_t* sigma_in,
                            int32_t nblk, int64_t n, int32_t b, int32_t* h_out,
                            int8_t* sigma_out, hipStream_t s);

// Prepared lists (see sketch.hip): for every block, window of
// kSketchWindow sketched indices and group of 64 buckets, the entries of
// each bucket (window offset and sign), lane-interleaved and padded.
constexpr int kSketchWindow = 8192;

// Longest sketched dimension (list entries hold k as 32 bits).
constexpr int64_t kMaxSketchedLen = OS_MAX_N;

// Bytes of the list structures for nblk blocks of padded width bp.
size_t list_bytes(int32_t nblk, int64_t n, int32_t bp);
// One prepared sketch of a batch prepared in one launch per step
// (device-resident).  The hash step writes table (nblk x nt packed entries:
// bucket | sign << 31, from SplitMix64 of seed, or from the explicit tables
// h / sigma when h is set); the list step builds the lists (hdr, ell) from
// it.  Tasks: hash task t of the batch is chunk (t - hash_task0) % hash_chunks
// of 256 indices of block (t - hash_task0) / hash_chunks; list task t is
// window (t - ell_task0) % nwin of block (t - ell_task0) / nwin.  The task0
// fields ascend with the descriptor index.
struct PrepDesc {
    uint64_t seed;
    const int32_t* h;
    const int8_t* sigma;
    uint32_t* table;
    uint32_t* hdr;
    uint16_t* ell;
    const int32_t* inv;     // bucket -> list position per block (nblk x bp), or nullptr
    int64_t n;
    int64_t nt;
    int64_t RC;
    int64_t hash_task0;
    int64_t ell_task0;
    int32_t b;
    int32_t bp;
    int32_t qn;
    int32_t nwin;
    int32_t nblk;
    int32_t hash_chunks;
};
// Index of the descriptor whose task range holds t (task0 ascending, the
// first one 0): the last p with task0(descs[p]) <= t.
template <typename F>
__device__ __forceinline__ int32_t find_task(const PrepDesc* descs, int32_t count, int64_t t,
                                             F task0) {
    int32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) / 2;
        if (task0(descs[mid]) <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}
// Sets the list fields (hdr, ell, qn, nwin, RC) of d (n, bp, nblk set) for
// its lists region.
void prep_desc_lists(PrepDesc& d, void* lists);
// The hash step / the list step of every descriptor (tasks = the total
// task count of that step; max_bp = the largest bp).
hipError_t launch_table_batch(const PrepDesc* descs, int32_t count, int64_t tasks,
                              hipStream_t s);
hipError_t launch_lists_batch(const PrepDesc* descs, int32_t count, int64_t tasks,
                              int32_t max_bp, hipStream_t s);
// Lists for every block i < nblk of a packed table; with inv (DEVICE
// [nblk][bp], bucket -> list position), bucket c's entries go to position
// inv[i * bp + c] (its column in the sketch), else to position c.
hipError_t launch_build_lists(const uint32_t* table, int64_t n, int64_t nt, int32_t nblk,
                              int32_t bp, void* lists, hipStream_t s,
                              const int32_t* inv = nullptr);
// inv for every block: buckets of similar list lengths grouped into the
// same 64-bucket groups (the identity when b <= 64).
hipError_t launch_group_buckets(const uint32_t* table, int64_t n, int64_t nt, int32_t nblk,
                                int32_t b, int32_t bp, int32_t* inv, hipStream_t s);
// inv = the identity (natural bucket order).
hipError_t launch_identity_inv(int32_t nblk, int32_t bp, int32_t* inv, hipStream_t s);
// order[i * bp + p] = the bucket at position p of block i (p for p >= b).
hipError_t launch_bucket_order(const int32_t* inv, int32_t nblk, int32_t b, int32_t bp,
                               int32_t* order, hipStream_t s);
// Shapes a sketch launch supports (lines = the dimension that is not sketched).
bool plan_sketch_ok(int64_t lines, int32_t nst, int32_t bp, int64_t n);
// out (cols x nst*bp, ld ldo) = (S^T X)^T for X n x cols row-major (ld ldx);
// stored block j is sketch block bl.idx[j]; lists built for nblk blocks.
hipError_t launch_sketch_rows(const float* X, int64_t n, int64_t cols, int64_t ldx,
                              const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                              const void* lists, float* out, int64_t ldo, hipStream_t s);
// True when launch_sketch_rows reads X's columns with 16-byte loads and the
// next window spread over the slots (X 16-byte aligned, ldx and cols
// multiples of 4): then reading them in place is faster than transposing X
// first and sketching the rows of X^T (the sums are the same, bit for bit).
bool sketch_rows_in_place_ok(const float* X, int64_t cols, int64_t ldx);
// launch_sketch_rows writing the BF16 copy, as launch_sketch_cols_q.
hipError_t launch_sketch_rows_q(const float* X, int64_t n, int64_t cols, int64_t ldx,
                                const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                                const void* lists, void* out, int64_t ldo, int split,
                                hipStream_t s);
// out (rows x nst*bp, ld ldo) = X S for X rows x n row-major (ld ldx);
// with wd (DEVICE [n]) it is X diag(sqrt(wd)) S.
hipError_t launch_sketch_cols(const float* X, int64_t rows, int64_t n, int64_t ldx,
                              const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                              const void* lists, float* out, int64_t ldo, hipStream_t s,
                              const float* wd = nullptr);

// Longest row pitch (bytes) of a sketch read by the block product: byte
// offsets within a 256-row tile, K offset included, stay below 2^32.
constexpr int64_t kMaxSketchLdBytes = (int64_t(1) << 24) - 256;
// Y (cols x rows, ld ldy: a multiple of 4, Y 16-byte aligned) = X^T for X
// rows x cols row-major (ld ldx); transpose_bytes = the size of Y with ldy =
// rows rounded up to 4.
size_t transpose_bytes(int64_t rows, int64_t cols);
hipError_t launch_transpose(const float* X, int64_t rows, int64_t cols, int64_t ldx, float* Y,
                            int64_t ldy, hipStream_t s);
// Y (cols x rows, BF16, ld ldy % 4 == 0, Y 8-byte aligned) = X^T, X BF16
// rows x cols (values copied exactly).
hipError_t launch_transpose_bf16_raw(const void* X, int64_t rows, int64_t cols, int64_t ldx,
                                     void* Y, int64_t ldy, hipStream_t s);
// launch_sketch_cols for a BF16 X (each value converted exactly to FP32 as
// its window is staged; the sums are those of the FP32 path on those values).
hipError_t launch_sketch_cols_bf16(const void* X, int64_t rows, int64_t n, int64_t ldx,
                                   const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                                   const void* lists, float* out, int64_t ldo, hipStream_t s);
// launch_sketch_cols (X FP32, or BF16 when x_bf16) writing the BF16 copy
// that launch_quant_bf16 would make of the FP32 sketch, bit for bit: each
// sum rounded to nearest even, block j at columns j*bpq .. (bpq = b rounded
// up to 64, zero past b), with split the residuals nst*bpq columns on; Q
// BF16 with ld ldo (in values).
hipError_t launch_sketch_cols_q(const void* X, bool x_bf16, int64_t rows, int64_t n, int64_t ldx,
                                const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                                const void* lists, void* out, int64_t ldo, int split,
                                hipStream_t s);
// The same for the FP8 copy launch_quant_fp8 would make without the split
// form (codes and E8M0 scales, ldo in bytes), bit for bit.  Only when
// sketch_fp8_fusable(b, nst):
// the FP8 block stride (b rounded up to 128) equals the sketch's 64-bucket
// groups (b rounded up to 64), so every code of the copy belongs to a group,
// and the sketch needs at most 20 slots per pass.
bool sketch_fp8_fusable(int32_t b, int32_t nst);
hipError_t launch_sketch_cols_fp8(const void* X, bool x_bf16, int64_t rows, int64_t n,
                                  int64_t ldx, const BlockList& bl, int32_t nst, int32_t nblk,
                                  int32_t bp, const void* lists, void* out, int64_t ldo,
                                  hipStream_t s);

// Shapes the block product supports for operands of elem bytes per value
// (4: FP32, 2: BF16, 1: FP8); bp must be a multiple of 128 / elem.
bool plan_gemm_ok(int64_t m, int64_t l, int32_t bp, int64_t ldat, int64_t ldbt, int elem);

// C = scale * sum over the kept stored blocks (kept.idx[0 .. nkept)) of
// At_j * Bt_j^T, with At (m x nst*bp) and Bt (l x nst*bp) line-major
// sketches (column block j = columns j*bp .. j*bp + bp - 1).
hipError_t launch_gemm_kept(const float* At, int64_t ldat, const float* Bt, int64_t ldbt,
                            int64_t m, int64_t l, int32_t bp, const BlockList& kept,
                            int32_t nkept, float scale, float* C, int64_t ldc, hipStream_t s);
// Partial-product bytes the split launches may use for an m x l product of
// at most max_steps K steps (128 bytes of every tile row each: 32 FP32, 64
// BF16 or 128 FP8 values); 0 when it never splits (enough tiles to fill the
// device).
size_t gemm_split_bytes(int64_t m, int64_t l, int64_t max_steps);
// launch_gemm_kept, with the K loop split over several workgroups per tile
// when the product has few tiles (partials in part, then summed in split
// order: deterministic, but summed in a different order than unsplit); the
// plain launch when it would not split or part_bytes is too small.
hipError_t launch_gemm_kept_split(const float* At, int64_t ldat, const float* Bt, int64_t ldbt,
                                  int64_t m, int64_t l, int32_t bp, const BlockList& kept,
                                  int32_t nkept, float scale, float* C, int64_t ldc, float* part,
                                  size_t part_bytes, hipStream_t s);
// The same with BF16 sketches (block stride bp, a multiple of 64; leading
// dimensions in BF16 values).  split != 0 adds the terms A_j * lo(B_j)^T and
// lo(A_j) * B_j^T, the low parts lo_off columns after the high parts.
hipError_t launch_gemm_kept_bf16(const void* At, int64_t ldat, const void* Bt, int64_t ldbt,
                                 int64_t m, int64_t l, int32_t bp, const BlockList& kept,
                                 int32_t nkept, int split, int64_t lo_off, float scale, float* C,
                                 int64_t ldc, hipStream_t s);
// The same with FP8 copies (launch_quant_fp8 layout: ld in bytes, the scale
// bytes of a row `scales` bytes after its start; block stride bp a multiple
// of 128).
hipError_t launch_gemm_kept_fp8(const void* At, int64_t ldat, const void* Bt, int64_t ldbt,
                                int64_t scales, int64_t m, int64_t l, int32_t bp,
                                const BlockList& kept, int32_t nkept, int split, int64_t lo_off,
                                float scale, float* C, int64_t ldc, hipStream_t s);
// launch_gemm_kept_bf16 / launch_gemm_kept_fp8 with the split K loop of
// launch_gemm_kept_split (partials in part, summed in split order).
hipError_t launch_gemm_kept_bf16_split(const void* At, int64_t ldat, const void* Bt, int64_t ldbt,
                                       int64_t m, int64_t l, int32_t bp, const BlockList& kept,
                                       int32_t nkept, int split, int64_t lo_off, float scale,
                                       float* C, int64_t ldc, float* part, size_t part_bytes,
                                       hipStream_t s);
hipError_t launch_gemm_kept_fp8_split(const void* At, int64_t ldat, const void* Bt, int64_t ldbt,
                                      int64_t scales, int64_t m, int64_t l, int32_t bp,
                                      const BlockList& kept, int32_t nkept, int split,
                                      int64_t lo_off, float scale, float* C, int64_t ldc,
                                      float* part, size_t part_bytes, hipStream_t s);
// FP32 block product with a keep mask per C block: cmask DEVICE [ceil(m/cblk)]
// [ceil(l/cblk)][nst]; block (I, J) of C (cblk x cblk) = (1/K_IJ) * sum of its
// kept blocks' products (zero when it keeps none).
hipError_t launch_gemm_cmask(const float* At, int64_t ldat, const float* Bt, int64_t ldbt,
                             int64_t m, int64_t l, int32_t bp, int32_t nst, const uint8_t* cmask,
                             int64_t cblk, float* C, int64_t ldc, hipStream_t s);

// One problem of a batched symmetric block product (device-resident): the
// sketch S stores only the kept blocks, so its first ksteps * 32 columns
// are summed over (ksteps = K * bp / 32 rounded up to even; the columns past
// K * bp are zero).
struct BatchProblem {
    const float* S;      // line-major sketch, m x (ksteps*32), ld (floats, multiple of 4)
    float* H;            // output m x m, ld ldh
    int64_t ld;
    int64_t ldh;
    int64_t m;
    int32_t ksteps;
    float scale;         // 1 / K
};
// H_k = scale_k * S_k S_k^T for every problem in one persistent launch:
// tiles DEVICE int4 {problem, tile row, tile col >= tile row, 0} for tile
// side `tile` (256 or 128), grouped by workgroup: workgroup g computes tiles
// starts[g] .. starts[g+1] - 1 (starts DEVICE [grid + 1]).  full != 0 also
// writes the mirror of each off-diagonal tile.  tile = OS_GRAM_MIXED: the
// list holds jobs of two int4 each, {problem, kind, tile row, tile col} and
// {second tile row, second tile col, has second, 0}: kind 0 one 256 tile,
// kind 1 one or two 128 tiles of the problem; starts count jobs.
hipError_t launch_gemm_batch_sym(const BatchProblem* probs, const int4* tiles,
                                 const int32_t* starts, int tile, int full, int32_t grid,
                                 hipStream_t s);
// Workgroups of the batched kernel for `tile` (256, 128 or OS_GRAM_MIXED)
// that fit on one CU at once (0 on error).
int batch_sym_blocks_per_cu(int tile);

// BF16 copy of a line-major FP32 sketch (lines x nst*bp, ld lds): block
// stride block_stride_bf16(b) = b rounded up to 64, the residual part (when
// split) after the nst blocks of the high part; Q 16-byte aligned, ldq a
// multiple of 8 and >= nst * bpq * (split ? 2 : 1).
int32_t block_stride_bf16(int32_t b);
hipError_t launch_quant_bf16(const float* S, int64_t lines, int64_t lds, int32_t b, int32_t nst,
                             int split, void* Q, int64_t ldq, hipStream_t s);
// FP8 (E4M3) copy with one E8M0 scale per kFp8Block values: block stride
// block_stride_fp8(b) = b rounded up to 128; row = codes (high part, then
// residual when split), then the scale bytes in the same order:
// fp8_row_bytes(b, nst, split) bytes; ldq (bytes) a multiple of 16.
constexpr int kFp8Block = 64;
int32_t block_stride_fp8(int32_t b);
int64_t fp8_row_bytes(int32_t b, int32_t nst, int split);
hipError_t launch_quant_fp8(const float* S, int64_t lines, int64_t lds, int32_t b, int32_t nst,
                            int split, void* Q, int64_t ldq, hipStream_t s);

}  // namespace osk
