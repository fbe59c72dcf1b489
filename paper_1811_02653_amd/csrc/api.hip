// api.hip -- the extern "C" entry points declared in include/oversketch.h:
// argument validation, keep-mask handling (Algorithm "OverSketch":
// termination keeps any N of the N+e blocks; K kept blocks are weighted
// 1/K), workspace carving and the launch sequence.
#include "internal.h"

#include <mutex>

namespace {

using osk::BlockList;

thread_local int t_last_hip_error = 0;

os_status hip_status(hipError_t e) {
    if (e == hipSuccess) return OS_OK;
    t_last_hip_error = (int)e;
    return OS_EHIP;
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

os_status check_sketch(const os_sketch* sk) {
    if (!sk) return OS_ENULL;
    if (sk->b < 1 || sk->b > OS_MAX_B || sk->N < 1 || sk->e < 0 ||
        (int64_t)sk->N + sk->e > OS_MAX_BLOCKS)
        return OS_EINVAL;
    if ((sk->h == nullptr) != (sk->sigma == nullptr)) return OS_ENULL;
    return OS_OK;
}

os_status check_len(int64_t n) { return (n >= 1 && n < (int64_t(1) << 40)) ? OS_OK : OS_EINVAL; }

// The dimension that is not sketched (rows of A, columns of B, m and l).
os_status check_extent(int64_t x) { return (x >= 1 && x <= OS_MAX_ROWS) ? OS_OK : OS_EINVAL; }

// vec4: rows are read or written 16 bytes at a time (base 16-byte aligned,
// ld a multiple of 4); otherwise only 4-byte alignment is needed.
os_status check_matrix(const float* p, int64_t rows, int64_t cols, int64_t ld, bool vec4 = true) {
    if (!p) return OS_ENULL;
    if (rows < 1 || cols < 1 || rows >= (int64_t(1) << 40) || ld < cols) return OS_EINVAL;
    if (vec4 ? (!aligned(p, 16) || (ld & 3)) : !aligned(p, 4)) return OS_EALIGN;
    return OS_OK;
}

int32_t nblocks(const os_sketch* sk) { return sk->N + sk->e; }

// Kept flags over the N+e blocks (NULL mask = the first N).
void kept_flags(const os_sketch* sk, const uint8_t* keep_host, bool* kept) {
    for (int32_t i = 0; i < nblocks(sk); ++i) kept[i] = keep_host ? keep_host[i] != 0 : i < sk->N;
}

// Stored blocks of a sketch: all N+e, or only the kept ones (ascending).
os_status stored_list(const os_sketch* sk, const uint8_t* keep_host, int kept_only, BlockList& bl,
                      int32_t& nst) {
    bool kept[OS_MAX_BLOCKS];
    kept_flags(sk, keep_host, kept);
    nst = 0;
    for (int32_t i = 0; i < nblocks(sk); ++i)
        if (!kept_only || kept[i]) bl.idx[nst++] = i;
    for (int32_t i = nst; i < OS_MAX_BLOCKS; ++i) bl.idx[i] = 0;
    return nst > 0 ? OS_OK : OS_ENOKEEP;
}

int64_t table_stride(int64_t n) { return osk::round_up(n, 4); }

os_status fill_table(const os_sketch* sk, int64_t n, uint32_t* table, hipStream_t s) {
    const int64_t nt = table_stride(n);
    hipError_t e = sk->h ? osk::launch_table_explicit(sk->h, sk->sigma, nblocks(sk), n, nt, sk->b,
                                                      table, s)
                         : osk::launch_table_hash(sk->seed, nblocks(sk), n, nt, sk->b, table, s);
    return hip_status(e);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

extern "C" {

const char* os_status_string(os_status status) {
    switch (status) {
        case OS_OK: return "OS_OK";
        case OS_EINVAL: return "OS_EINVAL: argument out of range";
        case OS_ENULL: return "OS_ENULL: required pointer is NULL";
        case OS_EALIGN: return "OS_EALIGN: pointer not 16-byte aligned or leading dimension not a multiple of 4";
        case OS_EWORKSPACE: return "OS_EWORKSPACE: workspace missing, misaligned or too small";
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

size_t os_table_bytes(const os_sketch* sk, int64_t n) {
    if (check_sketch(sk) != OS_OK || check_len(n) != OS_OK) return 0;
    return (size_t)nblocks(sk) * (size_t)table_stride(n) * 4u;
}

os_status os_hash_fill(const os_sketch* sk, int64_t n, int32_t* h_out, int8_t* sigma_out,
                       void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if (!h_out || !sigma_out) return OS_ENULL;
    return hip_status(osk::launch_hash_fill(sk->seed, sk->h, sk->sigma, nblocks(sk), n, sk->b,
                                            h_out, sigma_out, (hipStream_t)stream));
}

os_status os_sketch_table(const os_sketch* sk, int64_t n, uint32_t* table, void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if (!table) return OS_ENULL;
    if (!aligned(table, 16)) return OS_EALIGN;
    return fill_table(sk, n, table, (hipStream_t)stream);
}

os_status os_sketch_cols(const os_sketch* sk, const uint32_t* table, const float* X, int64_t rows,
                         int64_t n, int64_t ldx, const uint8_t* keep_host, int kept_only,
                         float* out, int64_t ldo, void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if (!table) return OS_ENULL;
    if (!aligned(table, 16)) return OS_EALIGN;
    if ((st = check_extent(rows)) != OS_OK) return st;
    if ((st = check_matrix(X, rows, n, ldx)) != OS_OK) return st;
    BlockList bl;
    int32_t nst = 0;
    if ((st = stored_list(sk, keep_host, kept_only, bl, nst)) != OS_OK) return st;
    const int32_t bp = os_block_stride(sk->b);
    if ((st = check_matrix(out, rows, (int64_t)nst * bp, ldo)) != OS_OK) return st;
    const osk::ColsPlan plan = osk::plan_sketch_cols(rows, nst, bp);
    if (!plan.valid) return OS_EINVAL;
    return hip_status(osk::launch_sketch_cols(X, rows, n, ldx, table, table_stride(n), bl, nst, bp,
                                              out, ldo, plan, (hipStream_t)stream));
}

os_status os_sketch_rows(const os_sketch* sk, const uint32_t* table, const float* X, int64_t n,
                         int64_t cols, int64_t ldx, const uint8_t* keep_host, int kept_only,
                         float* outT, int64_t ldo, void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if (!table) return OS_ENULL;
    if (!aligned(table, 16)) return OS_EALIGN;
    if ((st = check_extent(cols)) != OS_OK) return st;
    if ((st = check_matrix(X, n, cols, ldx, false)) != OS_OK) return st;
    BlockList bl;
    int32_t nst = 0;
    if ((st = stored_list(sk, keep_host, kept_only, bl, nst)) != OS_OK) return st;
    const int32_t bp = os_block_stride(sk->b);
    if ((st = check_matrix(outT, cols, (int64_t)nst * bp, ldo)) != OS_OK) return st;
    const osk::RowsPlan plan = osk::plan_sketch_rows(cols, nst, bp);
    if (!plan.valid) return OS_EINVAL;
    return hip_status(osk::launch_sketch_rows(X, n, cols, ldx, table, table_stride(n), bl, nst, bp,
                                              outT, ldo, plan, (hipStream_t)stream));
}

os_status os_gemm_kept(const float* At, int64_t ldat, const float* Bt, int64_t ldbt, int64_t m,
                       int64_t l, int32_t b, int32_t nst, const uint8_t* keep_host, float* C,
                       int64_t ldc, void* stream) {
    if (b < 1 || b > OS_MAX_B || nst < 1 || nst > OS_MAX_BLOCKS) return OS_EINVAL;
    const int32_t bp = os_block_stride(b);
    os_status st;
    if ((st = check_extent(m)) != OS_OK || (st = check_extent(l)) != OS_OK) return st;
    if ((st = check_matrix(At, m, (int64_t)nst * bp, ldat)) != OS_OK) return st;
    if ((st = check_matrix(Bt, l, (int64_t)nst * bp, ldbt)) != OS_OK) return st;
    if (!C) return OS_ENULL;
    if (m < 1 || l < 1 || ldc < l) return OS_EINVAL;
    if (!aligned(C, 4)) return OS_EALIGN;
    BlockList kept;
    int32_t K = 0;
    for (int32_t j = 0; j < nst; ++j)
        if (!keep_host || keep_host[j]) kept.idx[K++] = j;
    for (int32_t j = K; j < OS_MAX_BLOCKS; ++j) kept.idx[j] = 0;
    if (K == 0) return OS_ENOKEEP;
    if (!osk::plan_gemm_ok(m, l, bp)) return OS_EINVAL;
    return hip_status(osk::launch_gemm_kept(At, ldat, Bt, ldbt, m, l, bp, kept, K, 1.0f / (float)K, C,
                                            ldc, (hipStream_t)stream));
}

size_t os_matmul_workspace_bytes(const os_sketch* sk, int64_t m, int64_t n, int64_t l,
                                 int kept_only) {
    if (check_sketch(sk) != OS_OK || check_len(n) != OS_OK || check_extent(m) != OS_OK ||
        check_extent(l) != OS_OK)
        return 0;
    // kept_only stores at most N+e blocks as well; size for the mask-independent maximum.
    (void)kept_only;
    const int64_t ldw = (int64_t)nblocks(sk) * os_block_stride(sk->b);
    return align256(os_table_bytes(sk, n)) + align256((size_t)m * ldw * 4u) +
           align256((size_t)l * ldw * 4u);
}

os_status os_matmul(const os_sketch* sk, const float* A, int64_t lda, const float* B, int64_t ldb,
                    int b_col_major, int64_t m, int64_t n, int64_t l, const uint8_t* keep_host,
                    int kept_only, float* C, int64_t ldc, void* workspace, size_t ws_bytes,
                    void* stream) {
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    if ((st = check_len(n)) != OS_OK) return st;
    if ((st = check_extent(m)) != OS_OK || (st = check_extent(l)) != OS_OK) return st;
    if ((st = check_matrix(A, m, n, lda)) != OS_OK) return st;
    if (b_col_major) {
        if ((st = check_matrix(B, l, n, ldb)) != OS_OK) return st;
    } else {
        if ((st = check_matrix(B, n, l, ldb, false)) != OS_OK) return st;
    }
    if (!C) return OS_ENULL;
    if (ldc < l) return OS_EINVAL;
    if (!aligned(C, 4)) return OS_EALIGN;

    bool kept[OS_MAX_BLOCKS];
    kept_flags(sk, keep_host, kept);
    BlockList stored, kept_pos;
    int32_t nst = 0, K = 0;
    for (int32_t i = 0; i < nblocks(sk); ++i) {
        if (kept_only && !kept[i]) continue;
        if (kept[i]) kept_pos.idx[K++] = nst;
        stored.idx[nst++] = i;
    }
    for (int32_t i = nst; i < OS_MAX_BLOCKS; ++i) stored.idx[i] = 0;
    for (int32_t i = K; i < OS_MAX_BLOCKS; ++i) kept_pos.idx[i] = 0;
    if (K == 0) return OS_ENOKEEP;

    const size_t need = os_matmul_workspace_bytes(sk, m, n, l, kept_only);
    if (!workspace || !aligned(workspace, 256) || ws_bytes < need) return OS_EWORKSPACE;

    const int32_t bp = os_block_stride(sk->b);
    const int64_t ldw = (int64_t)nst * bp;
    char* ws = static_cast<char*>(workspace);
    uint32_t* table = reinterpret_cast<uint32_t*>(ws);
    float* At = reinterpret_cast<float*>(ws + align256(os_table_bytes(sk, n)));
    float* Bt = reinterpret_cast<float*>(reinterpret_cast<char*>(At) +
                                         align256((size_t)m * nblocks(sk) * bp * 4u));
    hipStream_t s = (hipStream_t)stream;
    const int64_t nt = table_stride(n);

    // Every launch shape is decided before the first launch.
    const osk::ColsPlan plan_a = osk::plan_sketch_cols(m, nst, bp);
    const osk::ColsPlan plan_bc = osk::plan_sketch_cols(l, nst, bp);
    const osk::RowsPlan plan_br = osk::plan_sketch_rows(l, nst, bp);
    if (!plan_a.valid || !(b_col_major ? plan_bc.valid : plan_br.valid) ||
        !osk::plan_gemm_ok(m, l, bp))
        return OS_EINVAL;

    if ((st = fill_table(sk, n, table, s)) != OS_OK) return st;
    if ((st = hip_status(osk::launch_sketch_cols(A, m, n, lda, table, nt, stored, nst, bp, At, ldw,
                                                 plan_a, s))) != OS_OK)
        return st;
    if (b_col_major)
        st = hip_status(osk::launch_sketch_cols(B, l, n, ldb, table, nt, stored, nst, bp, Bt, ldw,
                                                plan_bc, s));
    else
        st = hip_status(osk::launch_sketch_rows(B, n, l, ldb, table, nt, stored, nst, bp, Bt, ldw,
                                                plan_br, s));
    if (st != OS_OK) return st;
    return hip_status(osk::launch_gemm_kept(At, ldw, Bt, ldw, m, l, bp, kept_pos, K,
                                            1.0f / (float)K, C, ldc, s));
}

}  // extern "C"
