// api.hip -- the extern "C" entry points declared in include/oversketch.h:
// argument validation, keep-mask handling (Algorithm "OverSketch":
// termination keeps any N of the N+e blocks; K kept blocks are weighted
// 1/K), workspace carving and the launch sequence.  Every check happens
// before the first launch of a call.
#include <algorithm>
#include <vector>

#include "api_common.h"

namespace {

using namespace osk::api;

bool valid_prec(int p) { return p >= OS_PREC_FP32 && p <= OS_PREC_FP8X3; }
bool is_fp8(int p) { return p == OS_PREC_FP8 || p == OS_PREC_FP8X3; }
bool is_split(int p) { return p == OS_PREC_BF16X3 || p == OS_PREC_FP8X3; }

// Block stride of a quantized copy (values).
int32_t quant_stride(int32_t b, int prec) {
    return is_fp8(prec) ? osk::block_stride_fp8(b) : osk::block_stride_bf16(b);
}

// Values (BF16) or bytes (FP8: codes then scale bytes) of one row of a
// quantized sketch over nst blocks; 0 for FP32 (no copy).
int64_t quant_width(int32_t b, int32_t nst, int prec) {
    if (prec == OS_PREC_FP32) return 0;
    if (is_fp8(prec)) return osk::fp8_row_bytes(b, nst, is_split(prec));
    return (int64_t)nst * osk::block_stride_bf16(b) * (is_split(prec) ? 2 : 1);
}

// Bytes of one row of a quantized copy with leading dimension ld (values).
int64_t quant_row_bytes(int64_t ld, int prec) { return ld * (is_fp8(prec) ? 1 : 2); }

// Codes of one row (the FP8 scale bytes start there).
int64_t quant_codes(int32_t b, int32_t nst, int prec) {
    return (int64_t)nst * quant_stride(b, prec) * (is_split(prec) ? 2 : 1);
}

// Partial products of the block product's split K loop (products with few
// tiles), sized for all N+e blocks: K steps of 128 bytes of a row (32 FP32,
// 64 BF16 or 128 FP8 values of each block's stride), three terms per block
// in the split forms.
size_t split_part_bytes(const os_sketch* sk, int64_t m, int64_t l, int prec) {
    int64_t steps;
    if (prec == OS_PREC_FP32)
        steps = (int64_t)os_block_stride(sk->b) / 32;
    else if (is_fp8(prec))
        steps = (int64_t)osk::block_stride_fp8(sk->b) / 128;
    else
        steps = (int64_t)osk::block_stride_bf16(sk->b) / 64;
    steps *= (int64_t)nblocks(sk) * (is_split(prec) ? 3 : 1);
    return align256(osk::gemm_split_bytes(m, l, steps));
}

}  // namespace

extern "C" {

const char* os_status_string(os_status status) {
    switch (status) {
        case OS_OK: return "OS_OK";
        case OS_EINVAL: return "OS_EINVAL: argument out of range";
        case OS_ENULL: return "OS_ENULL: required pointer is NULL";
        case OS_EALIGN: return "OS_EALIGN: pointer not aligned or leading dimension not a multiple of 4";
        case OS_EWORKSPACE: return "OS_EWORKSPACE: workspace or prepared buffer too small";
        case OS_EHIP: return "OS_EHIP: HIP runtime error";
        case OS_ENOKEEP: return "OS_ENOKEEP: keep mask keeps no block";
        default: return "unknown os_status";
    }
}

int os_last_hip_error(void) { return t_last_hip_error; }

int32_t os_block_stride(int32_t b) {
    if (b < 1) return 0;
    return (int32_t)osk::round_up(b, osk::kBlockAlign);
}

os_status os_hash_fill(const os_sketch* sk, int64_t n, int32_t* h_out, int8_t* sigma_out,
                       void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if (!h_out || !sigma_out) return OS_ENULL;
    if (!aligned(h_out, 4)) return OS_EALIGN;
    return hip_status(osk::launch_hash_fill(sk->seed, sk->h, sk->sigma, nblocks(sk), n, sk->b,
                                            h_out, sigma_out, (hipStream_t)stream));
}

size_t os_sketch_prepare_bytes(const os_sketch* sk, int64_t n) {
    if (check_sketch(sk) != OS_OK || check_len(n) != OS_OK) return 0;
    return prepare_bytes(sk, n);
}

os_status os_sketch_prepare(const os_sketch* sk, int64_t n, void* prep, size_t prep_bytes,
                            void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if ((st = check_prep(sk, n, prep, prep_bytes)) != OS_OK) return st;
    return prepare(sk, n, prep, (hipStream_t)stream);
}

os_status os_sketch_prepare_ex(const os_sketch* sk, int64_t n, int flags, void* prep,
                               size_t prep_bytes, void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if (flags & ~OS_PREPARE_GROUPED) return OS_EINVAL;
    if ((st = check_prep(sk, n, prep, prep_bytes)) != OS_OK) return st;
    return prepare(sk, n, prep, (hipStream_t)stream, (flags & OS_PREPARE_GROUPED) != 0);
}

os_status os_sketch_bucket_order(const os_sketch* sk, int64_t n, const void* prep,
                                 size_t prep_bytes, int32_t* order, void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if ((st = check_prep(sk, n, prep, prep_bytes)) != OS_OK) return st;
    if (!order) return OS_ENULL;
    if (!aligned(order, 4)) return OS_EALIGN;
    return hip_status(osk::launch_bucket_order(prep_inv(prep, sk, n), nblocks(sk), sk->b,
                                               os_block_stride(sk->b), order,
                                               (hipStream_t)stream));
}

os_status os_sketch_list_entries(const os_sketch* sk, int64_t n, const void* prep,
                                 size_t prep_bytes, int64_t* walked, int64_t* real, void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if ((st = check_prep(sk, n, prep, prep_bytes)) != OS_OK) return st;
    if (!walked || !real) return OS_ENULL;
    const int32_t bp = os_block_stride(sk->b);
    const int32_t qn = (bp + 63) / 64;
    const int64_t nwin = (n + osk::kSketchWindow - 1) / osk::kSketchWindow;
    const size_t count = (size_t)nblocks(sk) * (size_t)nwin * (size_t)qn;
    hipStream_t s = (hipStream_t)stream;
    // the list headers come first in the lists area (see sketch.hip)
    const void* lists = prep_lists(prep, sk, n);
    try {
        std::vector<uint32_t> hdr(count);
        hipError_t e = hipMemcpyAsync(hdr.data(), lists, count * 4u, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_status(e);
        int64_t chunks = 0;
        for (size_t q = 0; q < count; ++q) chunks += hdr[q] >> 16;
        *walked = chunks * 8 * 64;
        *real = (int64_t)nblocks(sk) * n;
        return OS_OK;
    } catch (...) {
        return hip_status(hipErrorOutOfMemory);
    }
}

os_status os_sketch_cols(const os_sketch* sk, const void* prep, size_t prep_bytes, const float* X,
                         int64_t rows, int64_t n, int64_t ldx, const uint8_t* keep_host,
                         int kept_only, float* out, int64_t ldo, void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if ((st = check_extent(rows)) != OS_OK) return st;
    if ((st = check_prep(sk, n, prep, prep_bytes)) != OS_OK) return st;
    if ((st = check_matrix(X, rows, n, ldx, false)) != OS_OK) return st;
    Blocks bs;
    if ((st = block_sets(sk, keep_host, kept_only, bs)) != OS_OK) return st;
    const int32_t bp = os_block_stride(sk->b);
    if ((st = check_matrix(out, rows, (int64_t)bs.nst * bp, ldo, true)) != OS_OK) return st;
    if (!osk::plan_sketch_ok(rows, bs.nst, bp, n)) return OS_EINVAL;
    return hip_status(osk::launch_sketch_cols(X, rows, n, ldx, bs.stored, bs.nst, nblocks(sk), bp,
                                              prep_lists(prep, sk, n), out, ldo,
                                              (hipStream_t)stream));
}

size_t os_sketch_rows_workspace_bytes(int64_t n, int64_t cols) {
    if (check_len(n) != OS_OK || check_extent(cols) != OS_OK) return 0;
    return osk::transpose_bytes(n, cols);
}

os_status os_sketch_rows(const os_sketch* sk, const void* prep, size_t prep_bytes, const float* X,
                         int64_t n, int64_t cols, int64_t ldx, const uint8_t* keep_host,
                         int kept_only, float* out, int64_t ldo, void* workspace, size_t ws_bytes,
                         void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if ((st = check_extent(cols)) != OS_OK) return st;
    if ((st = check_prep(sk, n, prep, prep_bytes)) != OS_OK) return st;
    if ((st = check_matrix(X, n, cols, ldx, false)) != OS_OK) return st;
    Blocks bs;
    if ((st = block_sets(sk, keep_host, kept_only, bs)) != OS_OK) return st;
    const int32_t bp = os_block_stride(sk->b);
    if ((st = check_matrix(out, cols, (int64_t)bs.nst * bp, ldo, true)) != OS_OK) return st;
    if (!osk::plan_sketch_ok(cols, bs.nst, bp, n)) return OS_EINVAL;
    if (workspace) {
        if (!aligned(workspace, 256) || ws_bytes < osk::transpose_bytes(n, cols))
            return OS_EWORKSPACE;
        hipStream_t s = (hipStream_t)stream;
        float* Xt = static_cast<float*>(workspace);
        const int64_t ldt = osk::round_up(n, 4);
        if ((st = hip_status(osk::launch_transpose(X, n, cols, ldx, Xt, ldt, s))) != OS_OK) return st;
        return hip_status(osk::launch_sketch_cols(Xt, cols, n, ldt, bs.stored, bs.nst, nblocks(sk),
                                                  bp, prep_lists(prep, sk, n), out, ldo, s));
    }
    return hip_status(osk::launch_sketch_rows(X, n, cols, ldx, bs.stored, bs.nst, nblocks(sk), bp,
                                              prep_lists(prep, sk, n), out, ldo,
                                              (hipStream_t)stream));
}

os_status os_sketch_rows_ex(const os_sketch* sk, const void* prep, size_t prep_bytes,
                            const void* X, int x_dtype, int64_t n, int64_t cols, int64_t ldx,
                            const uint8_t* keep_host, int kept_only, float* out, int64_t ldo,
                            void* workspace, size_t ws_bytes, void* stream) {
    if (x_dtype == OS_DTYPE_F32)
        return os_sketch_rows(sk, prep, prep_bytes, static_cast<const float*>(X), n, cols, ldx,
                              keep_host, kept_only, out, ldo, workspace, ws_bytes, stream);
    if (x_dtype != OS_DTYPE_BF16) return OS_EINVAL;
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if ((st = check_extent(cols)) != OS_OK) return st;
    if ((st = check_prep(sk, n, prep, prep_bytes)) != OS_OK) return st;
    if (!X) return OS_ENULL;
    if (ldx < cols) return OS_EINVAL;
    if (!aligned(X, 2)) return OS_EALIGN;
    Blocks bs;
    if ((st = block_sets(sk, keep_host, kept_only, bs)) != OS_OK) return st;
    const int32_t bp = os_block_stride(sk->b);
    if ((st = check_matrix(out, cols, (int64_t)bs.nst * bp, ldo, true)) != OS_OK) return st;
    if (!osk::plan_sketch_ok(cols, bs.nst, bp, n)) return OS_EINVAL;
    if (!workspace || !aligned(workspace, 256) || ws_bytes < osk::transpose_bytes(n, cols))
        return OS_EWORKSPACE;
    // transposed as BF16 (half the bytes of an FP32 copy); the sketch converts
    // each value exactly to FP32 as it stages it
    hipStream_t s = (hipStream_t)stream;
    const int64_t ldt = osk::round_up(n, 4);
    if ((st = hip_status(osk::launch_transpose_bf16_raw(X, n, cols, ldx, workspace, ldt, s))) !=
        OS_OK)
        return st;
    return hip_status(osk::launch_sketch_cols_bf16(workspace, cols, n, ldt, bs.stored, bs.nst,
                                                   nblocks(sk), bp, prep_lists(prep, sk, n), out,
                                                   ldo, s));
}

os_status os_gemm_kept(const float* At, int64_t ldat, const float* Bt, int64_t ldbt, int64_t m,
                       int64_t l, int32_t b, int32_t nst, const uint8_t* keep_host, float* C,
                       int64_t ldc, void* stream) {
    if (b < 1 || b > OS_MAX_B || nst < 1 || nst > OS_MAX_BLOCKS) return OS_EINVAL;
    os_status st;
    if ((st = check_extent(m)) != OS_OK || (st = check_extent(l)) != OS_OK) return st;
    const int32_t bp = os_block_stride(b);
    if ((st = check_matrix(At, m, (int64_t)nst * bp, ldat, true)) != OS_OK) return st;
    if ((st = check_matrix(Bt, l, (int64_t)nst * bp, ldbt, true)) != OS_OK) return st;
    if ((st = check_matrix(C, m, l, ldc, false)) != OS_OK) return st;
    BlockList kept;
    int32_t K = 0;
    for (int32_t j = 0; j < nst; ++j)
        if (!keep_host || keep_host[j]) kept.idx[K++] = j;
    for (int32_t j = K; j < OS_MAX_BLOCKS; ++j) kept.idx[j] = 0;
    if (K == 0) return OS_ENOKEEP;
    if (!osk::plan_gemm_ok(m, l, bp, ldat, ldbt, 4)) return OS_EINVAL;
    return hip_status(osk::launch_gemm_kept(At, ldat, Bt, ldbt, m, l, bp, kept, K, 1.0f / (float)K, C,
                                            ldc, (hipStream_t)stream));
}

os_status os_gemm_kept_cmask(const float* At, int64_t ldat, const float* Bt, int64_t ldbt,
                             int64_t m, int64_t l, int32_t b, int32_t nst,
                             const uint8_t* cmask, float* C, int64_t ldc, void* stream) {
    if (b < 1 || b > OS_MAX_B || nst < 1 || nst > OS_MAX_BLOCKS) return OS_EINVAL;
    os_status st;
    if ((st = check_extent(m)) != OS_OK || (st = check_extent(l)) != OS_OK) return st;
    const int32_t bp = os_block_stride(b);
    if ((st = check_matrix(At, m, (int64_t)nst * bp, ldat, true)) != OS_OK) return st;
    if ((st = check_matrix(Bt, l, (int64_t)nst * bp, ldbt, true)) != OS_OK) return st;
    if ((st = check_matrix(C, m, l, ldc, false)) != OS_OK) return st;
    if (!cmask) return OS_ENULL;
    if (!osk::plan_gemm_ok(m, l, bp, ldat, ldbt, 4)) return OS_EINVAL;
    return hip_status(osk::launch_gemm_cmask(At, ldat, Bt, ldbt, m, l, bp, nst, cmask, b, C, ldc,
                                             (hipStream_t)stream));
}

int32_t os_block_stride_prec(int32_t b, int precision) {
    if (b < 1 || !valid_prec(precision)) return 0;
    return precision == OS_PREC_FP32 ? os_block_stride(b) : quant_stride(b, precision);
}

int64_t os_quantized_row(int32_t b, int32_t nst, int precision) {
    if (b < 1 || b > OS_MAX_B || nst < 1 || nst > OS_MAX_BLOCKS || !valid_prec(precision)) return 0;
    return quant_width(b, nst, precision);
}

os_status os_sketch_quantize(const float* S, int64_t lines, int64_t lds, int32_t b, int32_t nst,
                             int precision, void* Q, int64_t ldq, void* stream) {
    if (b < 1 || b > OS_MAX_B || nst < 1 || nst > OS_MAX_BLOCKS) return OS_EINVAL;
    if (!valid_prec(precision) || precision == OS_PREC_FP32) return OS_EINVAL;
    os_status st;
    if ((st = check_extent(lines)) != OS_OK) return st;
    const int32_t bp = os_block_stride(b);
    if ((st = check_matrix(S, lines, (int64_t)nst * bp, lds, false)) != OS_OK) return st;
    const int64_t w = quant_width(b, nst, precision);
    if (!Q) return OS_ENULL;
    if (ldq < w) return OS_EINVAL;
    if (!aligned(Q, 16) || (quant_row_bytes(ldq, precision) & 15)) return OS_EALIGN;
    if (is_fp8(precision))
        return hip_status(osk::launch_quant_fp8(S, lines, lds, b, nst, is_split(precision), Q, ldq,
                                                (hipStream_t)stream));
    return hip_status(osk::launch_quant_bf16(S, lines, lds, b, nst, is_split(precision), Q, ldq,
                                             (hipStream_t)stream));
}

os_status os_gemm_kept_prec(const void* At, int64_t ldat, const void* Bt, int64_t ldbt, int64_t m,
                            int64_t l, int32_t b, int32_t nst, const uint8_t* keep_host,
                            int precision, float* C, int64_t ldc, void* stream) {
    if (!valid_prec(precision)) return OS_EINVAL;
    if (precision == OS_PREC_FP32)
        return os_gemm_kept(static_cast<const float*>(At), ldat, static_cast<const float*>(Bt),
                            ldbt, m, l, b, nst, keep_host, C, ldc, stream);
    if (b < 1 || b > OS_MAX_B || nst < 1 || nst > OS_MAX_BLOCKS) return OS_EINVAL;
    os_status st;
    if ((st = check_extent(m)) != OS_OK || (st = check_extent(l)) != OS_OK) return st;
    const int64_t w = quant_width(b, nst, precision);
    if (!At || !Bt) return OS_ENULL;
    if (ldat < w || ldbt < w) return OS_EINVAL;
    if (!aligned(At, 16) || !aligned(Bt, 16) || (quant_row_bytes(ldat, precision) & 15) ||
        (quant_row_bytes(ldbt, precision) & 15))
        return OS_EALIGN;
    if ((st = check_matrix(C, m, l, ldc, false)) != OS_OK) return st;
    BlockList kept;
    int32_t K = 0;
    for (int32_t j = 0; j < nst; ++j)
        if (!keep_host || keep_host[j]) kept.idx[K++] = j;
    for (int32_t j = K; j < OS_MAX_BLOCKS; ++j) kept.idx[j] = 0;
    if (K == 0) return OS_ENOKEEP;
    const int32_t bpq = quant_stride(b, precision);
    if (!osk::plan_gemm_ok(m, l, bpq, ldat, ldbt, is_fp8(precision) ? 1 : 2)) return OS_EINVAL;
    if (is_fp8(precision))
        return hip_status(osk::launch_gemm_kept_fp8(At, ldat, Bt, ldbt,
                                                    quant_codes(b, nst, precision), m, l, bpq,
                                                    kept, K, is_split(precision),
                                                    (int64_t)nst * bpq, 1.0f / (float)K, C, ldc,
                                                    (hipStream_t)stream));
    return hip_status(osk::launch_gemm_kept_bf16(At, ldat, Bt, ldbt, m, l, bpq, kept, K,
                                                 is_split(precision), (int64_t)nst * bpq,
                                                 1.0f / (float)K, C, ldc, (hipStream_t)stream));
}

size_t os_matmul_ex_workspace_bytes(const os_sketch* sk, int64_t m, int64_t n, int64_t l,
                                    int a_col_major, int b_col_major, int precision) {
    if (check_sketch(sk) != OS_OK || check_len(n) != OS_OK || check_extent(m) != OS_OK ||
        check_extent(l) != OS_OK || !valid_prec(precision))
        return 0;
    // Sized for all N+e blocks whatever the mask, so one workspace serves
    // every call; an operand whose lines are not rows in memory (a
    // column-major A, a row-major B) is transposed first, one after the
    // other, into one buffer; a low-precision product adds the quantized
    // copies of both sketches.
    const int64_t zp = (int64_t)nblocks(sk) * os_block_stride(sk->b);
    const int64_t qrow = quant_row_bytes(osk::round_up(quant_width(sk->b, nblocks(sk), precision),
                                                       16), precision);
    const size_t tx = std::max(a_col_major ? osk::transpose_bytes(n, m) : 0,
                               b_col_major ? 0 : osk::transpose_bytes(n, l));
    return align256(prepare_bytes(sk, n)) + align256((size_t)m * zp * 4u) +
           align256((size_t)l * zp * 4u) + tx + align256((size_t)m * qrow) +
           align256((size_t)l * qrow) + split_part_bytes(sk, m, l, precision);
}

size_t os_matmul_prec_workspace_bytes(const os_sketch* sk, int64_t m, int64_t n, int64_t l,
                                      int b_col_major, int precision) {
    return os_matmul_ex_workspace_bytes(sk, m, n, l, 0, b_col_major, precision);
}

size_t os_matmul_workspace_bytes(const os_sketch* sk, int64_t m, int64_t n, int64_t l,
                                 int b_col_major) {
    return os_matmul_prec_workspace_bytes(sk, m, n, l, b_col_major, OS_PREC_FP32);
}

os_status os_matmul_ex(const os_sketch* sk, const void* A, int a_dtype, int a_col_major,
                       int64_t lda, const void* B, int b_dtype, int b_col_major, int64_t ldb,
                       int64_t m, int64_t n, int64_t l, const uint8_t* keep_host, int kept_only,
                       int precision, float* C, int64_t ldc, void* workspace, size_t ws_bytes,
                       void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if (!valid_prec(precision)) return OS_EINVAL;
    if ((a_dtype != OS_DTYPE_F32 && a_dtype != OS_DTYPE_BF16) ||
        (b_dtype != OS_DTYPE_F32 && b_dtype != OS_DTYPE_BF16))
        return OS_EINVAL;
    if ((st = check_len(n)) != OS_OK) return st;
    if ((st = check_extent(m)) != OS_OK || (st = check_extent(l)) != OS_OK) return st;
    auto check_op = [](const void* p, int dtype, int64_t rows, int64_t cols, int64_t ld) {
        if (dtype == OS_DTYPE_F32) return check_matrix(p, rows, cols, ld, false);
        if (!p) return OS_ENULL;
        if (rows < 1 || cols < 1 || ld < cols) return OS_EINVAL;
        return aligned(p, 2) ? OS_OK : OS_EALIGN;
    };
    if (a_col_major) {
        if ((st = check_op(A, a_dtype, n, m, lda)) != OS_OK) return st;
    } else {
        if ((st = check_op(A, a_dtype, m, n, lda)) != OS_OK) return st;
    }
    if (b_col_major) {
        if ((st = check_op(B, b_dtype, l, n, ldb)) != OS_OK) return st;
    } else {
        if ((st = check_op(B, b_dtype, n, l, ldb)) != OS_OK) return st;
    }
    if ((st = check_matrix(C, m, l, ldc, false)) != OS_OK) return st;
    Blocks bs;
    if ((st = block_sets(sk, keep_host, kept_only, bs)) != OS_OK) return st;
    const size_t need =
        os_matmul_ex_workspace_bytes(sk, m, n, l, a_col_major, b_col_major, precision);
    if (!workspace || !aligned(workspace, 256) || ws_bytes < need) return OS_EWORKSPACE;
    const int32_t bp = os_block_stride(sk->b);
    const int32_t bpq = quant_stride(sk->b, precision);
    // quantized copies: rows padded to 16 bytes
    const int64_t wq = osk::round_up(quant_width(sk->b, bs.nst, precision), 16);
    const bool gemm_ok = precision == OS_PREC_FP32
                             ? osk::plan_gemm_ok(m, l, bp, (int64_t)bs.nst * bp,
                                                 (int64_t)bs.nst * bp, 4)
                             : osk::plan_gemm_ok(m, l, bpq, wq, wq, is_fp8(precision) ? 1 : 2);
    if (!osk::plan_sketch_ok(m, bs.nst, bp, n) || !osk::plan_sketch_ok(l, bs.nst, bp, n) ||
        !gemm_ok)
        return OS_EINVAL;

    // both sketches use the stored width as leading dimension (a multiple of 32)
    const int64_t zs = (int64_t)bs.nst * bp;
    const int64_t zp = (int64_t)nblocks(sk) * bp;
    const int64_t wqp = quant_row_bytes(
        osk::round_up(quant_width(sk->b, nblocks(sk), precision), 16), precision);
    const size_t tx = std::max(a_col_major ? osk::transpose_bytes(n, m) : 0,
                               b_col_major ? 0 : osk::transpose_bytes(n, l));
    char* ws = static_cast<char*>(workspace);
    void* prep = ws;
    char* at_p = ws + align256(prepare_bytes(sk, n));
    char* bt_p = at_p + align256((size_t)m * zp * 4u);
    char* tx_p = bt_p + align256((size_t)l * zp * 4u);
    char* aq_p = tx_p + tx;
    char* bq_p = aq_p + align256((size_t)m * wqp);
    char* part_p = bq_p + align256((size_t)l * wqp);
    const size_t part_bytes = split_part_bytes(sk, m, l, precision);
    float* At = reinterpret_cast<float*>(at_p);
    float* Bt = reinterpret_cast<float*>(bt_p);
    hipStream_t s = (hipStream_t)stream;
    const void* lists = prep_lists(prep, sk, n);

    // An operand's lines (rows of A, columns of B) are sketched as rows in
    // memory: a column-major A and a row-major B are transposed first (in
    // their own type), so that every sketch reads whole lines (16-byte
    // requests along a column would each bring in a separate cache line) --
    // except an FP32 row-major B whose columns the sketch can read with
    // 16-byte loads and its window spread over the slots
    // (sketch_rows_in_place_ok), which is faster read in place than
    // transposed (no fused FP8 copy in that form; the sums are the same).
    // BF16 values are converted exactly to FP32 as the sketch stages them.
    // With a BF16 block product the sketch writes its BF16 copy directly
    // (rounded in the sketch's epilogue, bit for bit what the quantization
    // of the FP32 sketch gives); with an FP8 one its FP8 copy when every
    // code belongs to a sketch group (b rounded up to 64 is a multiple of
    // 128) and the sketch takes at most 20 slots (FP8 without the split
    // form); otherwise the FP32 sketch, quantized after.
    const bool bf16_product = precision != OS_PREC_FP32 && !is_fp8(precision);
    // (the split FP8 form stays staged: its second group maximum made the
    // fused sketch slower than the separate quantization)
    const bool fp8_fused =
        is_fp8(precision) && !is_split(precision) && osk::sketch_fp8_fusable(sk->b, bs.nst);
    auto sketch_lines = [&](const void* X, int dtype, bool transpose, int64_t lines,
                            int64_t ldx, float* out, void* qout) -> os_status {
        const void* Xl = X;
        int64_t ldl = ldx;
        if (transpose && dtype == OS_DTYPE_F32 && !fp8_fused &&
            osk::sketch_rows_in_place_ok(static_cast<const float*>(X), lines, ldx)) {
            const float* Xf = static_cast<const float*>(X);
            if (bf16_product)
                return hip_status(osk::launch_sketch_rows_q(Xf, n, lines, ldx, bs.stored, bs.nst,
                                                            nblocks(sk), bp, lists, qout, wq,
                                                            is_split(precision), s));
            return hip_status(osk::launch_sketch_rows(Xf, n, lines, ldx, bs.stored, bs.nst,
                                                      nblocks(sk), bp, lists, out, zs, s));
        }
        if (transpose) {
            ldl = osk::round_up(n, 4);
            const hipError_t e =
                dtype == OS_DTYPE_BF16
                    ? osk::launch_transpose_bf16_raw(X, n, lines, ldx, tx_p, ldl, s)
                    : osk::launch_transpose(static_cast<const float*>(X), n, lines, ldx,
                                            reinterpret_cast<float*>(tx_p), ldl, s);
            if (e != hipSuccess) return hip_status(e);
            Xl = tx_p;
        }
        if (bf16_product)
            return hip_status(osk::launch_sketch_cols_q(Xl, dtype == OS_DTYPE_BF16, lines, n, ldl,
                                                        bs.stored, bs.nst, nblocks(sk), bp, lists,
                                                        qout, wq, is_split(precision), s));
        if (fp8_fused)
            return hip_status(osk::launch_sketch_cols_fp8(Xl, dtype == OS_DTYPE_BF16, lines, n,
                                                          ldl, bs.stored, bs.nst, nblocks(sk), bp,
                                                          lists, qout, wq, s));
        return hip_status(
            dtype == OS_DTYPE_BF16
                ? osk::launch_sketch_cols_bf16(Xl, lines, n, ldl, bs.stored, bs.nst, nblocks(sk),
                                               bp, lists, out, zs, s)
                : osk::launch_sketch_cols(static_cast<const float*>(Xl), lines, n, ldl,
                                          bs.stored, bs.nst, nblocks(sk), bp, lists, out, zs, s));
    };
    if ((st = prepare(sk, n, prep, s)) != OS_OK) return st;
    if ((st = sketch_lines(A, a_dtype, a_col_major != 0, m, lda, At, aq_p)) != OS_OK) return st;
    if ((st = sketch_lines(B, b_dtype, b_col_major == 0, l, ldb, Bt, bq_p)) != OS_OK) return st;
    if (precision == OS_PREC_FP32)
        return hip_status(osk::launch_gemm_kept_split(
            At, zs, Bt, zs, m, l, bp, bs.kept_pos, bs.K, 1.0f / (float)bs.K, C, ldc,
            reinterpret_cast<float*>(part_p), part_bytes, s));
    const int split = is_split(precision);
    if (is_fp8(precision)) {
        if (!fp8_fused) {
            if ((st = hip_status(osk::launch_quant_fp8(At, m, zs, sk->b, bs.nst, split, aq_p, wq,
                                                       s))) != OS_OK)
                return st;
            if ((st = hip_status(osk::launch_quant_fp8(Bt, l, zs, sk->b, bs.nst, split, bq_p, wq,
                                                       s))) != OS_OK)
                return st;
        }
        return hip_status(osk::launch_gemm_kept_fp8_split(
            aq_p, wq, bq_p, wq, quant_codes(sk->b, bs.nst, precision), m, l, bpq, bs.kept_pos,
            bs.K, split, (int64_t)bs.nst * bpq, 1.0f / (float)bs.K, C, ldc,
            reinterpret_cast<float*>(part_p), part_bytes, s));
    }
    return hip_status(osk::launch_gemm_kept_bf16_split(
        aq_p, wq, bq_p, wq, m, l, bpq, bs.kept_pos, bs.K, split, (int64_t)bs.nst * bpq,
        1.0f / (float)bs.K, C, ldc, reinterpret_cast<float*>(part_p), part_bytes, s));
}

os_status os_matmul_prec(const os_sketch* sk, const float* A, int64_t lda, const float* B,
                         int64_t ldb, int b_col_major, int64_t m, int64_t n, int64_t l,
                         const uint8_t* keep_host, int kept_only, int precision, float* C,
                         int64_t ldc, void* workspace, size_t ws_bytes, void* stream) {
    return os_matmul_ex(sk, A, OS_DTYPE_F32, 0, lda, B, OS_DTYPE_F32, b_col_major, ldb, m, n, l,
                        keep_host, kept_only, precision, C, ldc, workspace, ws_bytes, stream);
}

os_status os_matmul_cmask(const os_sketch* sk, const float* A, int64_t lda, const float* B,
                          int64_t ldb, int b_col_major, int64_t m, int64_t n, int64_t l,
                          const uint8_t* cmask, float* C, int64_t ldc, void* workspace,
                          size_t ws_bytes, void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if ((st = check_extent(m)) != OS_OK || (st = check_extent(l)) != OS_OK) return st;
    if ((st = check_matrix(A, m, n, lda, false)) != OS_OK) return st;
    if (b_col_major) {
        if ((st = check_matrix(B, l, n, ldb, false)) != OS_OK) return st;
    } else {
        if ((st = check_matrix(B, n, l, ldb, false)) != OS_OK) return st;
    }
    if ((st = check_matrix(C, m, l, ldc, false)) != OS_OK) return st;
    if (!cmask) return OS_ENULL;
    // every block is sketched: the blocks each C block keeps differ
    uint8_t all[OS_MAX_BLOCKS];
    for (int32_t i = 0; i < nblocks(sk); ++i) all[i] = 1;
    Blocks bs;
    if ((st = block_sets(sk, all, 0, bs)) != OS_OK) return st;
    const size_t need = os_matmul_workspace_bytes(sk, m, n, l, b_col_major);
    if (!workspace || !aligned(workspace, 256) || ws_bytes < need) return OS_EWORKSPACE;
    const int32_t bp = os_block_stride(sk->b);
    const int64_t zs = (int64_t)bs.nst * bp;
    if (!osk::plan_sketch_ok(m, bs.nst, bp, n) || !osk::plan_sketch_ok(l, bs.nst, bp, n) ||
        !osk::plan_gemm_ok(m, l, bp, zs, zs, 4))
        return OS_EINVAL;
    char* ws = static_cast<char*>(workspace);
    void* prep = ws;
    float* At = reinterpret_cast<float*>(ws + align256(prepare_bytes(sk, n)));
    float* Bt = reinterpret_cast<float*>(reinterpret_cast<char*>(At) + align256((size_t)m * zs * 4u));
    float* Bx = reinterpret_cast<float*>(reinterpret_cast<char*>(Bt) + align256((size_t)l * zs * 4u));
    hipStream_t s = (hipStream_t)stream;
    const void* lists = prep_lists(prep, sk, n);
    if ((st = prepare(sk, n, prep, s)) != OS_OK) return st;
    if ((st = hip_status(osk::launch_sketch_cols(A, m, n, lda, bs.stored, bs.nst, nblocks(sk), bp,
                                                 lists, At, zs, s))) != OS_OK)
        return st;
    if (!b_col_major && osk::sketch_rows_in_place_ok(B, l, ldb)) {
        // B's columns read in place (faster than transposed, same sums)
        if ((st = hip_status(osk::launch_sketch_rows(B, n, l, ldb, bs.stored, bs.nst, nblocks(sk),
                                                     bp, lists, Bt, zs, s))) != OS_OK)
            return st;
    } else {
        const float* Bl = B;
        int64_t ldl = ldb;
        if (!b_col_major) {
            ldl = osk::round_up(n, 4);
            if ((st = hip_status(osk::launch_transpose(B, n, l, ldb, Bx, ldl, s))) != OS_OK)
                return st;
            Bl = Bx;
        }
        if ((st = hip_status(osk::launch_sketch_cols(Bl, l, n, ldl, bs.stored, bs.nst,
                                                     nblocks(sk), bp, lists, Bt, zs, s))) != OS_OK)
            return st;
    }
    return hip_status(osk::launch_gemm_cmask(At, zs, Bt, zs, m, l, bp, bs.nst, cmask, sk->b, C,
                                             ldc, s));
}

os_status os_matmul(const os_sketch* sk, const float* A, int64_t lda, const float* B, int64_t ldb,
                    int b_col_major, int64_t m, int64_t n, int64_t l, const uint8_t* keep_host,
                    int kept_only, float* C, int64_t ldc, void* workspace, size_t ws_bytes,
                    void* stream) {
    return os_matmul_prec(sk, A, lda, B, ldb, b_col_major, m, n, l, keep_host, kept_only,
                          OS_PREC_FP32, C, ldc, workspace, ws_bytes, stream);
}

}  // extern "C"
