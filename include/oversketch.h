/*
 * oversketch.h -- C ABI of liboversketch.so, an MI355X (gfx950) library for
 * OverSketch's approximate matrix product  C ~= A * S * S^T * B
 * (Gupta, Wang, Courtade, Ramchandran, "OverSketch: Approximate Matrix
 * Multiplication for the Cloud").
 *
 * The method (Section 4.1):
 *   - A is m x n, B is n x l.
 *   - S = N^{-1/2} (S_1, ..., S_{N+e}) (Eq. (sketch_matrix)) is a row of N+e
 *     independent count-sketch blocks S_i, each n x b: every index k in
 *     [0, n) is sent to one bucket h_i(k) in [0, b) with a sign
 *     sigma_i(k) = +-1 (Algorithm "Calculating Count-sketch of a matrix A").
 *   - A_tilde = A S and B_tilde = S^T B are formed block by block (Algorithm
 *     "Over sketching A in parallel"), and the product is assembled from any
 *     N of the N+e blocks (Algorithm "OverSketch", termination step).  On one
 *     GPU a host keep-mask stands in for the blocks that straggled.
 *
 * Readings of the paper used by this library:
 *   - Normalisation: the result is (1/K) * sum over kept blocks i of
 *     (A S_i)(S_i^T B), K = number of kept blocks.  This equals the paper's
 *     N^{-1/2} * N^{-1/2} whenever K = N and stays unbiased when K != N.
 *   - Random source: bucket and sign of (block i, index k) come from
 *     SplitMix64 (Steele, Lea & Flood 2014) evaluated at state
 *     seed + (ctr + 1) * 0x9E3779B97F4A7C15 with ctr = (i << 40) | k:
 *     h = ((word >> 32) * b) >> 32, sigma = (word & 1) ? -1 : +1.
 *     Explicit buckets and signs may be supplied instead (os_sketch.h/sigma).
 *   - Indices are 0-based.
 *
 * Conventions for every entry point:
 *   - Matrices are FP32 and row-major with a leading dimension ("ld", in
 *     elements) >= their column count.  Inputs (A, B, the X of the sketch
 *     calls) and the product C need 4-byte alignment; a sketch (the output of
 *     os_sketch_cols / os_sketch_rows, the inputs of os_gemm_kept) is read 16
 *     bytes at a time and needs a 16-byte aligned base and an ld that is a
 *     multiple of 4.  Violations return OS_EALIGN.
 *   - Size limits: the sketched dimension n <= OS_MAX_N; the other dimension
 *     of each operand (m, l) <= OS_MAX_ROWS.
 *   - Device pointers are HIP device memory owned by the caller; the library
 *     never allocates device memory and never retains a pointer past return.
 *     Host pointers (keep masks) are read before the call returns.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     on it and the call returns; outputs are valid once the stream has
 *     completed.  Every argument check happens before anything is enqueued:
 *     on any error nothing is launched and no output is touched.
 *   - No C++ exception crosses this interface.  No entry point keeps mutable
 *     global state; the only per-thread state is os_last_hip_error.
 *
 * Sketch layout ("line-major"): the sketch of a matrix with L lines (rows of
 * A, columns of B) over nst stored blocks is a row-major L x (nst * bp)
 * matrix, bp = os_block_stride(b) = b rounded up to a multiple of 32: column
 * j*bp + c of row r holds bucket c of stored block j for line r -- i.e. the
 * sketch of A is A S and the sketch of B is (S^T B)^T, each without the
 * N^{-1/2} factor.  Columns j*bp + b .. (j+1)*bp - 1 are written as zero.
 * With kept_only = 0 every one of the N+e blocks is stored (block i at
 * position i); with kept_only = 1 only the kept blocks are stored, in
 * ascending block order (the "straggler-resilient sketching" remark of
 * Section 4.1: blocks dropped at sketch time count as stragglers).
 *
 * Prepared sketch: an opaque device buffer holding, for all N+e blocks, the
 * bucket/sign of every index and, per block, window of 8192 indices and group
 * of 64 buckets, the indices of each bucket (ascending), lane-interleaved and
 * padded to the group's longest bucket.  It depends only on (seed or explicit
 * tables, b, N, e, n), not on a keep mask, and can be reused by every sketch
 * call with the same values.  Its size is bounded for ANY tables (a bucket
 * holding a whole window included): about (N+e) * n * 128 bytes plus
 * (N+e) * ceil(n / 8192) * (ceil(bp / 64) * 1028) bytes.
 */
#ifndef OVERSKETCH_H
#define OVERSKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int os_status;

#define OS_OK          0   /* success */
#define OS_EINVAL     -1   /* a size, count or parameter outside its range */
#define OS_ENULL      -2   /* a required pointer is NULL */
#define OS_EALIGN     -3   /* a pointer or leading dimension misaligned (see conventions) */
#define OS_EWORKSPACE -4   /* workspace / prepared buffer missing or smaller than required */
#define OS_EHIP       -5   /* the HIP runtime reported an error (os_last_hip_error) */
#define OS_ENOKEEP    -6   /* the keep mask keeps no block */

#define OS_MAX_BLOCKS 256                   /* upper limit on N + e */

/* Element types of an operand read by os_sketch_rows_ex. */
#define OS_DTYPE_F32  0
#define OS_DTYPE_BF16 1

/* Operand precision of the block product (FP32 accumulation in all).  The
 * paper's products are FP64; these trade the rounding of the sketched
 * operands, which is small next to the sketch's own error, for MFMA rate. */
#define OS_PREC_FP32   0   /* FP32 operands, v_mfma_f32_32x32x2_f32 */
#define OS_PREC_BF16   1   /* BF16 operands (round to nearest even), v_mfma_f32_32x32x16_bf16 */
#define OS_PREC_BF16X3 2   /* split BF16: x = hi + lo, product hi*hi' + hi*lo' + lo*hi' */
#define OS_PREC_FP8    3   /* FP8 E4M3 with an E8M0 (power-of-two) scale per 64 values,
                              v_mfma_scale_f32_32x32x64_f8f6f4 */
#define OS_PREC_FP8X3  4   /* split FP8: the residual quantized with its own scales */
#define OS_MAX_B      8192                  /* upper limit on the block width b */
#define OS_MAX_N      (2147483647LL - 64LL) /* upper limit on the sketched dimension n */
#define OS_MAX_ROWS   16777216LL            /* upper limit on m and l */

/* Sketch description.  b in [1, OS_MAX_B], N >= 1, e >= 0, N + e <=
 * OS_MAX_BLOCKS.  When h is non-NULL, sigma must be non-NULL too and both
 * are DEVICE arrays [N+e][n] (row i = block i) holding explicit buckets in
 * [0, b) and signs in {-1, +1}; the seed is then ignored.  Explicit buckets
 * outside [0, b) are clamped into it and any negative sign counts as -1, so a
 * bad table gives a wrong result, never an out-of-bounds access. */
typedef struct os_sketch {
    uint64_t seed;
    int32_t b;
    int32_t N;
    int32_t e;
    const int32_t* h;
    const int8_t* sigma;
} os_sketch;

/* Human-readable name of a status code (static string, never NULL). */
const char* os_status_string(os_status status);

/* hipError_t of the most recent OS_EHIP returned on the calling thread
 * (0 if none). */
int os_last_hip_error(void);

/* Rows taken by one stored block in a sketch: b rounded up to a multiple of
 * 32 (0 if b < 1). */
int32_t os_block_stride(int32_t b);

/* Step "hash": the random choices of Algorithm "Calculating Count-sketch of
 * a matrix A" for all N+e blocks, materialised on the device:
 * h_out[i*n + k] = bucket h_i(k) in [0, b), sigma_out[i*n + k] = sigma_i(k).
 * h_out: DEVICE int32 [(N+e) * n] (4-byte aligned); sigma_out: DEVICE int8
 * [(N+e) * n].  With explicit tables the clamped values are copied. */
os_status os_hash_fill(const os_sketch* sk, int64_t n, int32_t* h_out, int8_t* sigma_out,
                       void* stream);

/* Bytes of the prepared sketch for an n-long sketched dimension (0 on
 * invalid arguments). */
size_t os_sketch_prepare_bytes(const os_sketch* sk, int64_t n);

/* Step "hash" as the sketch kernels consume it: fills the prepared sketch
 * (buckets and signs of all N+e blocks, then every block's indices grouped
 * by bucket range, ascending).  prep: DEVICE, 256-byte aligned, >=
 * os_sketch_prepare_bytes(sk, n) bytes (else OS_EWORKSPACE). */
os_status os_sketch_prepare(const os_sketch* sk, int64_t n, void* prep, size_t prep_bytes,
                            void* stream);

/* Flags of os_sketch_prepare_ex. */
#define OS_PREPARE_GROUPED 1   /* bucket order chosen for the sketch kernel */

/* os_sketch_prepare with flags.  OS_PREPARE_GROUPED: within every block the
 * buckets are laid out in an order of the library's choosing, not 0..b-1:
 * buckets whose index lists have similar lengths share the sketch kernel's
 * groups of 64, so the kernel walks less padding (the lanes of a group step
 * through their lists together).  A sketch taken with such a prepared
 * sketch holds bucket order[i*bp + p] of block i at column j*bp + p (see
 * os_sketch_bucket_order); A's and B's sketches use the same order, so the
 * product (1/K) sum_i (A S_i)(S_i^T B) is the same up to FP32 summation
 * order (Eq. (sketch_matrix): any ordering of the columns of S_i).  The
 * ordering itself costs a sort per block in the prepare step; the
 * whole-path calls (os_matmul*, os_gram_*) use the natural order.  Other
 * flags: OS_EINVAL. */
os_status os_sketch_prepare_ex(const os_sketch* sk, int64_t n, int flags, void* prep,
                               size_t prep_bytes, void* stream);

/* The bucket at every column of a prepared sketch's blocks:
 * order[i*bp + p] = the bucket held at column p of block i (p < b), and p
 * for the empty columns b <= p < bp.  order: DEVICE int32 [(N+e) * bp].
 * The identity for a prepared sketch made without OS_PREPARE_GROUPED. */
os_status os_sketch_bucket_order(const os_sketch* sk, int64_t n, const void* prep,
                                 size_t prep_bytes, int32_t* order, void* stream);

/* Diagnostic (synchronous: waits for `stream`): the list entries the sketch
 * kernel walks per group of 4 lines over all N+e blocks (walked, padding
 * included) and the real ones (real = (N+e) * n), from a prepared sketch.
 * walked / real is the kernel's padding factor. */
os_status os_sketch_list_entries(const os_sketch* sk, int64_t n, const void* prep,
                                 size_t prep_bytes, int64_t* walked, int64_t* real,
                                 void* stream);

/* Step "sketch A's columns" (Algorithm "Over sketching A in parallel" with
 * Algorithm "Calculating Count-sketch" per block) for a row-major X
 * (rows x n, ld ldx), line-major output:
 *   out[r][j*bp + c] = sum_{k : h_{s_j}(k) = c} sigma_{s_j}(k) * X[r][k]
 * for every stored block j (sketch block s_j), i.e. out = X S_{s_j} side by
 * side over j.  Each bucket is summed in FP32 in ascending k.  (With a
 * prepared sketch made with OS_PREPARE_GROUPED, column j*bp + p holds
 * bucket order[s_j*bp + p] in place of bucket p; see
 * os_sketch_bucket_order.)
 * prep: a prepared sketch for the same sk and n.  keep_host: HOST uint8
 * [N+e] (nonzero = kept) or NULL (= blocks [0, N)); it selects the stored
 * blocks when kept_only != 0.  out: DEVICE rows x (nst*bp), ld ldo >=
 * nst*bp.  A column-major matrix is sketched along its rows by passing its
 * transpose (which is row-major). */
os_status os_sketch_cols(const os_sketch* sk, const void* prep, size_t prep_bytes,
                         const float* X, int64_t rows, int64_t n, int64_t ldx,
                         const uint8_t* keep_host, int kept_only, float* out, int64_t ldo,
                         void* stream);

/* Device workspace bytes os_sketch_rows uses, when given one, for an n x
 * cols operand (0 on invalid sizes): room for the operand transposed. */
size_t os_sketch_rows_workspace_bytes(int64_t n, int64_t cols);

/* Step "sketch B's rows" (S^T B: the same sketch applied from the left,
 * Section 4) for a row-major X (n x cols, ld ldx), line-major output:
 *   out[q][j*bp + c] = sum_{k : h_{s_j}(k) = c} sigma_{s_j}(k) * X[k][q],
 * i.e. out = (S_{s_j}^T X)^T side by side over j.  Other arguments as in
 * os_sketch_cols; out: DEVICE cols x (nst*bp), ld ldo >= nst*bp.
 * workspace: optional DEVICE buffer (256-byte aligned, >=
 * os_sketch_rows_workspace_bytes, else OS_EWORKSPACE).  With it, X is first
 * transposed into the workspace and its rows sketched as by os_sketch_cols
 * (the faster path: every line is then read as whole cache lines); with
 * workspace = NULL the columns of X are sketched in place.  Both paths give
 * the same sums in the same order. */
os_status os_sketch_rows(const os_sketch* sk, const void* prep, size_t prep_bytes,
                         const float* X, int64_t n, int64_t cols, int64_t ldx,
                         const uint8_t* keep_host, int kept_only, float* out, int64_t ldo,
                         void* workspace, size_t ws_bytes, void* stream);

/* os_sketch_rows for an X of element type x_dtype: OS_DTYPE_F32 is
 * os_sketch_rows; OS_DTYPE_BF16 reads a BF16 X (2-byte aligned, ld ldx in
 * values), transposes it (as BF16) into the workspace (required: >=
 * os_sketch_rows_workspace_bytes(n, cols)) and sketches it as os_sketch_rows
 * does, each value converted exactly to FP32 as it is read, FP32 sums.  Used for the sketched
 * weight gradient of a linear layer, X^T S S^T dY with the sketch over the
 * tokens (the rows of X and dY). */
os_status os_sketch_rows_ex(const os_sketch* sk, const void* prep, size_t prep_bytes,
                            const void* X, int x_dtype, int64_t n, int64_t cols, int64_t ldx,
                            const uint8_t* keep_host, int kept_only, float* out, int64_t ldo,
                            void* workspace, size_t ws_bytes, void* stream);

/* Step "grouped product over the kept blocks" (Algorithm "OverSketch":
 * computation phase plus reduction phase, Fig. (bMM)):
 *   C = (1/K) * sum_{j : keep[j]} At_j * Bt_j^T,
 * At: DEVICE m x (nst*bp) line-major sketch of A (ld ldat >= nst*bp), Bt:
 * DEVICE l x (nst*bp) line-major sketch of B (ld ldbt >= nst*bp), At_j /
 * Bt_j = their columns j*bp .. j*bp + bp - 1; keep_host: HOST uint8 [nst]
 * over the STORED blocks, or NULL (= all stored blocks); K = number kept.
 * C: DEVICE m x l (ld ldc >= l), overwritten.  FP32 inputs, FP32 MFMA
 * accumulation. */
os_status os_gemm_kept(const float* At, int64_t ldat, const float* Bt, int64_t ldbt,
                       int64_t m, int64_t l, int32_t b, int32_t nst,
                       const uint8_t* keep_host, float* C, int64_t ldc, void* stream);

/* Step "grouped product" with a keep mask per block of C: the paper's
 * stragglers differ per C block (Algorithm "OverSketch": each b x b block of
 * C is assembled from the first workers that return for it).  C is divided
 * into b x b blocks (the last ones partial); block (I, J) keeps the stored
 * blocks j with cmask[(I * ceil(l/b) + J) * nst + j] != 0 and is
 *   C_IJ = (1/K_IJ) * sum_{kept j} At_j[I rows] * Bt_j[J rows]^T,
 * K_IJ = its kept count; a block that keeps none is written as zero.
 * cmask: DEVICE uint8 [ceil(m/b)][ceil(l/b)][nst] (read by the kernel).
 * Other arguments as in os_gemm_kept. */
os_status os_gemm_kept_cmask(const float* At, int64_t ldat, const float* Bt, int64_t ldbt,
                             int64_t m, int64_t l, int32_t b, int32_t nst,
                             const uint8_t* cmask, float* C, int64_t ldc, void* stream);

/* Columns taken by one stored block in a sketch of the given precision:
 * b rounded up to 32 (FP32), 64 (BF16 forms) or 128 (FP8 forms); 0 on
 * invalid arguments. */
int32_t os_block_stride_prec(int32_t b, int precision);

/* Length of one row of a quantized sketch over nst blocks: BF16 values for
 * the BF16 forms, bytes for the FP8 forms (codes, then one scale byte per
 * 64 codes); 0 for OS_PREC_FP32 or invalid arguments. */
int64_t os_quantized_row(int32_t b, int32_t nst, int precision);

/* Low-precision copy of a line-major FP32 sketch S (lines x nst*bp, ld lds,
 * bp = os_block_stride(b)) for os_gemm_kept_prec.  bq =
 * os_block_stride_prec(b, precision); block j of S becomes codes j*bq ..
 * j*bq + bq - 1 of a row (zero past b), the split forms' residual part
 * follows at nst*bq.
 *   OS_PREC_BF16:   hi = round-to-nearest-even BF16 of S;
 *   OS_PREC_BF16X3: [hi | lo], lo = bf16(S - hi);
 *   OS_PREC_FP8:    per 64 consecutive values of a row: s = the smallest
 *                   integer with max|x| <= 448 * 2^s (clamped to
 *                   [-127, 127]), code = E4M3 round-to-nearest-even of
 *                   x * 2^-s; the row's scale bytes (s + 127, one per 64
 *                   codes, in code order) follow its codes;
 *   OS_PREC_FP8X3:  the same for S and for the residual S - dequant(code).
 * Q: DEVICE, lines x os_quantized_row(b, nst, precision) (BF16 values or
 * bytes), ld ldq in the same unit, rows 16-byte aligned (Q 16-byte aligned,
 * ldq a multiple of 16 bytes). */
os_status os_sketch_quantize(const float* S, int64_t lines, int64_t lds, int32_t b, int32_t nst,
                             int precision, void* Q, int64_t ldq, void* stream);

/* Step "grouped product over the kept blocks" with operands of the given
 * precision: OS_PREC_FP32 is os_gemm_kept; the other forms take the copies
 * os_sketch_quantize makes (At: m rows, Bt: l rows, each
 * os_quantized_row(b, nst, precision) long, leading dimensions in the same
 * unit, rows 16-byte aligned) and compute
 *   C = (1/K) * sum_{kept j} hi(A_j) hi(B_j)^T [+ hi(A_j) lo(B_j)^T + lo(A_j) hi(B_j)^T]
 * (FP8: each 64-value block times its scale) with FP32 MFMA accumulation. */
os_status os_gemm_kept_prec(const void* At, int64_t ldat, const void* Bt, int64_t ldbt,
                            int64_t m, int64_t l, int32_t b, int32_t nst,
                            const uint8_t* keep_host, int precision, float* C, int64_t ldc,
                            void* stream);

/* Workspace bytes os_matmul needs: the prepared sketch and both sketches,
 * sized for all N+e blocks so one workspace serves any mask, plus, for a
 * row-major B (b_col_major = 0), room for B transposed (l x n; used only when
 * B cannot be read in place, see os_matmul), plus, for a product of at most
 * 128 tiles of 256 x 256, the partial products of the block product's split
 * K loop (S m x l FP32 matrices, S <= 256 / tiles, at most 64 MiB).  0 on
 * invalid arguments. */
size_t os_matmul_workspace_bytes(const os_sketch* sk, int64_t m, int64_t n, int64_t l,
                                 int b_col_major);

/* The whole path: C ~= (1/K) * sum_{kept i} (A S_i)(S_i^T B)
 * (Algorithm "OverSketch" on one GPU).  A: DEVICE m x n row-major (lda).
 * B: DEVICE n x l; b_col_major = 0 -> row-major with ld ldb >= l;
 * b_col_major = 1 -> column-major, element (k, q) at B[q*ldb + k], ldb >= n.
 * keep_host: HOST uint8 [N+e] or NULL (= blocks [0, N) kept).  kept_only != 0
 * skips the dropped blocks already in the sketch step.  C: DEVICE m x l
 * (ldc).  workspace: DEVICE, 256-byte aligned, >= os_matmul_workspace_bytes
 * for the same b_col_major.  Enqueues: prepare, sketch of A, (transpose of
 * a row-major B,) sketch of B, block product.  A row-major B that is 16-byte
 * aligned with ldb and l multiples of 4 has its columns sketched in place
 * (no transpose; the same sums).  A product of at most 128 tiles splits
 * its block product's K loop over several workgroups per tile (partials in
 * the workspace, summed in a fixed order: repeatable bit for bit, summed in
 * another order than os_gemm_kept). */
os_status os_matmul(const os_sketch* sk, const float* A, int64_t lda, const float* B,
                    int64_t ldb, int b_col_major, int64_t m, int64_t n, int64_t l,
                    const uint8_t* keep_host, int kept_only, float* C, int64_t ldc,
                    void* workspace, size_t ws_bytes, void* stream);

/* The whole path with a keep mask per block of C (see os_gemm_kept_cmask):
 * all N+e blocks are sketched; cmask: DEVICE uint8 [ceil(m/b)][ceil(l/b)][N+e].
 * Other arguments and the workspace as in os_matmul. */
os_status os_matmul_cmask(const os_sketch* sk, const float* A, int64_t lda, const float* B,
                          int64_t ldb, int b_col_major, int64_t m, int64_t n, int64_t l,
                          const uint8_t* cmask, float* C, int64_t ldc, void* workspace,
                          size_t ws_bytes, void* stream);

/* Workspace bytes os_matmul_prec needs: those of os_matmul plus, for the
 * BF16 and FP8 forms, the quantized copies of both sketches.  0 on invalid
 * arguments. */
size_t os_matmul_prec_workspace_bytes(const os_sketch* sk, int64_t m, int64_t n, int64_t l,
                                      int b_col_major, int precision);

/* The whole path with the block product in the given precision (os_matmul
 * is precision OS_PREC_FP32): prepare, sketch of A, (transpose of a
 * row-major B,) sketch of B, quantization of both sketches as
 * os_sketch_quantize does it, block product.  The BF16 forms always, and
 * plain FP8 when b rounded up to 64 is a multiple of 128 and each wave of
 * the sketch holds at most 20 groups of 64 buckets per pass, quantize in
 * the sketch itself (same values, no FP32 sketch written).  Arguments as in os_matmul;
 * workspace >= os_matmul_prec_workspace_bytes for the same b_col_major and
 * precision. */
os_status os_matmul_prec(const os_sketch* sk, const float* A, int64_t lda, const float* B,
                         int64_t ldb, int b_col_major, int64_t m, int64_t n, int64_t l,
                         const uint8_t* keep_host, int kept_only, int precision, float* C,
                         int64_t ldc, void* workspace, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * os_matmul_prec without a workspace argument.  The workspace lives in a
 * fixed device array inside the library, os_noalloc_scratch_bytes() bytes
 * (256 MiB) on every GPU the library runs on, held from module load until
 * the process ends.  Arguments, layouts and results are those of
 * os_matmul_prec (the same kernels, so C is bit for bit the same).  A
 * problem whose os_matmul_prec_workspace_bytes exceeds the array returns
 * OS_EWORKSPACE before anything is enqueued.  No call allocates or frees
 * device memory.  All calls on one GPU share the array and the results of
 * the previous call stay in it: calls that overlap in time on one GPU (two
 * streams, two host threads) race and must be serialized by the caller. */
size_t os_noalloc_scratch_bytes(void);
os_status os_matmul_noalloc(const os_sketch* sk, const float* A, int64_t lda, const float* B,
                            int64_t ldb, int b_col_major, int64_t m, int64_t n, int64_t l,
                            const uint8_t* keep_host, int kept_only, int precision, float* C,
                            int64_t ldc, void* stream);

/* Workspace bytes os_matmul_ex needs for the given operand layouts and
 * precision (0 on invalid arguments). */
size_t os_matmul_ex_workspace_bytes(const os_sketch* sk, int64_t m, int64_t n, int64_t l,
                                    int a_col_major, int b_col_major, int precision);

/* The whole path with more operand layouts and types: A m x n, row-major
 * (a_col_major = 0, element (r, k) at A[r*lda + k]) or column-major
 * (a_col_major = 1, at A[k*lda + r], lda >= m); B n x l as in os_matmul.
 * a_dtype / b_dtype: OS_DTYPE_F32 or OS_DTYPE_BF16 (2-byte aligned, ld in
 * values), in either layout.  A column-major A and a row-major B are first
 * transposed into the workspace in their own type (an FP32 one that is
 * 16-byte aligned with its ld and line count multiples of 4 is read in place
 * instead, unless the FP8 copy is written by the sketch); BF16 values are converted
 * exactly to FP32 as the sketch reads them, so the result equals that of the
 * FP32 path on the converted values, bit for bit.  With A = X^T for a
 * row-major X (n x m: A is
 * X read as column-major) and B = dY this is the sketched weight gradient of
 * a linear layer, X^T S S^T dY, sketched over the n tokens (the product of
 * Section 4 with the tokens as the inner dimension).  Other arguments as in
 * os_matmul_prec; workspace >= os_matmul_ex_workspace_bytes. */
os_status os_matmul_ex(const os_sketch* sk, const void* A, int a_dtype, int a_col_major,
                       int64_t lda, const void* B, int b_dtype, int b_col_major, int64_t ldb,
                       int64_t m, int64_t n, int64_t l, const uint8_t* keep_host, int kept_only,
                       int precision, float* C, int64_t ldc, void* workspace, size_t ws_bytes,
                       void* stream);

/* ------------------------------------------------------------------------
 * Batched sketched Gram matrices: the Hessian sketch of the interior-point
 * application (Section 5.2, Eq. (int_point) and the Hessian after it).  The
 * Newton step of the log-barrier LP needs A^T diag(1/(b_i - a_i x)^2) A,
 * whose square root is diag(1/|b_i - a_i x|) A; it is approximated by the
 * Gram matrix of the sketched square root, (S^T grad2f^{1/2})^T
 * (S^T grad2f^{1/2}).  In this library's row-major convention a problem is A
 * (m x n: the LP's constraint matrix transposed, its n constraints along the
 * sketched side) and D = diag(d), d_i = 1/(b_i - a_i x)^2, and
 *   H = (1/K) * sum_{kept i} (A D^{1/2} S_i)(A D^{1/2} S_i)^T,
 * the OverSketch product of A D^{1/2} with its own transpose.  A batch of
 * such problems of different sizes runs as: per problem, prepare and sketch
 * (D^{1/2} applied to A's entries as they are read, only the kept blocks
 * stored), then ONE persistent launch computing the upper-triangle tiles of
 * every H (and their mirrors), the tiles spread over the workgroups by a
 * static largest-first schedule computed on the host.
 *
 * Lifetime: a plan is a HOST object.  It copies the problem descriptions
 * (sizes, sketch parameters, keep masks) and keeps the DEVICE pointers A, d,
 * H of every problem: they must stay valid while the plan (or a graph made
 * from it) is used.  The plan's workspace (os_gram_workspace_bytes) holds
 * the schedule, the prepared sketches and the sketches; os_gram_configure
 * writes the schedule into it, and os_gram_run / os_gram_graph_create
 * require the workspace last configured.
 * ------------------------------------------------------------------------ */

/* One problem of a batch.  sk: its sketch (buckets over n; explicit tables,
 * if given, are DEVICE [N+e][n]).  A: DEVICE m x n row-major, ld lda, 4-byte
 * aligned.  d: DEVICE FP32 [n] with d[k] >= 0 (the diagonal of D), or NULL
 * for D = I.  keep: HOST uint8 [N+e] or NULL (= blocks [0, N)), copied by
 * os_gram_plan_create.  H: DEVICE m x m row-major, ld ldh >= m, overwritten
 * (with full = 0 only its tiles on or above the diagonal are written). */
typedef struct os_gram_problem {
    os_sketch sk;
    const float* A;
    int64_t lda;
    const float* d;
    int64_t m;
    int64_t n;
    const uint8_t* keep;
    float* H;
    int64_t ldh;
} os_gram_problem;

typedef struct os_gram_plan os_gram_plan;

/* Validates every problem (count in [1, OS_GRAM_MAX_PROBLEMS]) and makes a
 * plan (*plan_out, released by os_gram_plan_destroy).  full != 0: H is
 * written whole (the lower triangle mirrored from the upper); full = 0: only
 * the tiles on or above the diagonal are written.  On error *plan_out is
 * NULL.  Allocates host memory only. */
#define OS_GRAM_MAX_PROBLEMS 65536
os_status os_gram_plan_create(const os_gram_problem* probs, int32_t count, int full,
                              os_gram_plan** plan_out);

/* Releases a plan (NULL is ignored).  Graphs made from it stay valid. */
void os_gram_plan_destroy(os_gram_plan* plan);

/* DEVICE workspace bytes the plan needs (256-byte aligned base); one size
 * serves every tile configuration.  0 for a NULL plan. */
size_t os_gram_workspace_bytes(const os_gram_plan* plan);

/* Tile form of the batched product (os_gram_configure's `tile`):
 *   256 -- 256 x 256 tiles, eight waves each (the diagonal tiles computed
 *          whole);
 *   128 -- 128 x 128 tiles, four waves each, two workgroups per CU;
 *   OS_GRAM_MIXED -- eight-wave workgroups computing 256 x 256 tiles inside
 *          each upper triangle and pairs of 128 x 128 tiles along its
 *          diagonal and in a last tile column of at most 128 columns (less
 *          work outside the triangle than 256, fewer LDS reads per MFMA than
 *          128 inside it).
 * With full = 0 the entries written are those of the tiles on or above the
 * diagonal at tile side 256, 128 and 128 respectively. */
#define OS_GRAM_MIXED 1

/* Chooses the tile form of the batched product (256, 128 or OS_GRAM_MIXED;
 * 0 = OS_GRAM_MIXED) and its number of persistent workgroups (grid; 0 = as
 * many as fit on the device at once), computes the static schedule and
 * copies it and the per-problem descriptors into the workspace.
 * Synchronizes `stream` before returning.  OS_EINVAL for another tile or a
 * grid above 65536. */
os_status os_gram_configure(os_gram_plan* plan, int32_t tile, int32_t grid, void* workspace,
                            size_t ws_bytes, void* stream);

/* The tile side and grid the plan is configured with (0, 0 before
 * os_gram_configure); either pointer may be NULL. */
void os_gram_config(const os_gram_plan* plan, int32_t* tile, int32_t* grid);

/* Stages of a batch run (os_gram_run, os_gram_graph_create), OR-ed. */
#define OS_GRAM_PREPARE 1   /* hash and bucket lists of every problem */
#define OS_GRAM_SKETCH  2   /* the weighted sketch of every A (kept blocks) */
#define OS_GRAM_PRODUCT 4   /* the one batched product writing every H */
#define OS_GRAM_ALL     7

/* Enqueues the given stages (a nonzero subset of OS_GRAM_ALL) of the batch
 * on `stream`, in the order prepare, sketch, product.  A stage left out
 * uses what an earlier run left in the workspace (prepared sketches are
 * reusable while the plan's sketch parameters stand; the sketches while A
 * and d are unchanged).  Only kernels are enqueued (no copies, no memsets),
 * so the call can be captured into a graph.  Requires the workspace of the
 * last os_gram_configure (else OS_EINVAL). */
os_status os_gram_run(const os_gram_plan* plan, int stages, void* workspace, size_t ws_bytes,
                      void* stream);

/* One configuration the autotuner timed: tile form, grid, and the average
 * time of the product stage in milliseconds. */
typedef struct os_gram_candidate {
    int32_t tile;
    int32_t grid;
    float ms;
} os_gram_candidate;

/* Autotuner: runs the prepare and sketch stages once, then for each
 * candidate -- tile form OS_GRAM_MIXED, 256 and 128, each with one and with
 * two times the resident grid (workgroups that fit on the device at once)
 * -- configures the plan, runs the product stage once to warm up and times
 * `reps` (>= 1) further product runs with HIP events on `stream`; leaves
 * the plan configured with the fastest.  The H outputs are overwritten.
 * cands (HOST, may be NULL when cap = 0) receives up to cap candidates in
 * the order timed and *count (may be NULL) how many were timed; *best_ms
 * (may be NULL) the fastest average product time.  OS_EINVAL for reps < 1,
 * cap < 0, or cap > 0 with cands NULL. */
os_status os_gram_autotune_ex(os_gram_plan* plan, int32_t reps, void* workspace,
                              size_t ws_bytes, void* stream, os_gram_candidate* cands,
                              int32_t cap, int32_t* count, float* best_ms);

/* os_gram_autotune_ex without the candidate list. */
os_status os_gram_autotune(os_gram_plan* plan, int32_t reps, void* workspace, size_t ws_bytes,
                           void* stream, float* best_ms);

/* Captures one os_gram_run of the given stages on `stream` (a created
 * stream, not NULL) into a HIP graph and instantiates it: *graph_out is an
 * executable graph for os_graph_launch.  The graph uses the plan's current
 * configuration and workspace. */
os_status os_gram_graph_create(const os_gram_plan* plan, int stages, void* workspace,
                               size_t ws_bytes, void* stream, void** graph_out);

/* Launches an executable graph from os_gram_graph_create on `stream`. */
os_status os_graph_launch(void* graph, void* stream);

/* Releases an executable graph (NULL is ignored). */
void os_graph_destroy(void* graph);

#ifdef __cplusplus
}
#endif

#endif /* OVERSKETCH_H */
