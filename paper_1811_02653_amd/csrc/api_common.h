// api_common.h -- argument checks, keep-mask handling and prepared-sketch
// layout shared by the entry points of api.hip and gram.hip.
#pragma once

#include "internal.h"

namespace osk {
namespace api {


using osk::BlockList;

inline thread_local int t_last_hip_error = 0;

inline os_status hip_status(hipError_t e) {
    if (e == hipSuccess) return OS_OK;
    t_last_hip_error = (int)e;
    return OS_EHIP;
}

inline bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

inline os_status check_sketch(const os_sketch* sk) {
    if (!sk) return OS_ENULL;
    if (sk->b < 1 || sk->b > OS_MAX_B || sk->N < 1 || sk->e < 0 ||
        (int64_t)sk->N + sk->e > OS_MAX_BLOCKS)
        return OS_EINVAL;
    if ((sk->h == nullptr) != (sk->sigma == nullptr)) return OS_ENULL;
    return OS_OK;
}

// The sketched dimension n.
inline os_status check_len(int64_t n) { return (n >= 1 && n <= OS_MAX_N) ? OS_OK : OS_EINVAL; }

// The dimension that is not sketched (rows of A, columns of B, m and l).
inline os_status check_extent(int64_t x) { return (x >= 1 && x <= OS_MAX_ROWS) ? OS_OK : OS_EINVAL; }

// vec4: rows are read 16 bytes at a time (base 16-byte aligned, ld a
// multiple of 4); otherwise only 4-byte alignment is needed.
inline os_status check_matrix(const void* p, int64_t rows, int64_t cols, int64_t ld, bool vec4) {
    if (!p) return OS_ENULL;
    if (rows < 1 || cols < 1 || ld < cols) return OS_EINVAL;
    if (vec4 ? (!aligned(p, 16) || (ld & 3)) : !aligned(p, 4)) return OS_EALIGN;
    return OS_OK;
}

inline int32_t nblocks(const os_sketch* sk) { return sk->N + sk->e; }

// Kept flags over the N+e blocks (NULL mask = the first N).
inline void kept_flags(const os_sketch* sk, const uint8_t* keep_host, bool* kept) {
    for (int32_t i = 0; i < nblocks(sk); ++i) kept[i] = keep_host ? keep_host[i] != 0 : i < sk->N;
}

// Stored blocks (all N+e, or only the kept ones, ascending) and the positions
// of the kept blocks among the stored ones.
struct Blocks {
    BlockList stored;
    BlockList kept_pos;
    int32_t nst;
    int32_t K;
};

inline os_status block_sets(const os_sketch* sk, const uint8_t* keep_host, int kept_only, Blocks& bs) {
    bool kept[OS_MAX_BLOCKS];
    kept_flags(sk, keep_host, kept);
    bs.nst = 0;
    bs.K = 0;
    for (int32_t i = 0; i < nblocks(sk); ++i) {
        if (kept_only && !kept[i]) continue;
        if (kept[i]) bs.kept_pos.idx[bs.K++] = bs.nst;
        bs.stored.idx[bs.nst++] = i;
    }
    for (int32_t i = bs.nst; i < OS_MAX_BLOCKS; ++i) bs.stored.idx[i] = 0;
    for (int32_t i = bs.K; i < OS_MAX_BLOCKS; ++i) bs.kept_pos.idx[i] = 0;
    return bs.K > 0 ? OS_OK : OS_ENOKEEP;
}

inline int64_t table_stride(int64_t n) { return osk::round_up(n, 4); }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline size_t table_bytes(const os_sketch* sk, int64_t n) {
    return (size_t)nblocks(sk) * (size_t)table_stride(n) * 4u;
}

// Prepared buffer: the packed table, the bucket lists, then the position
// map inv [N+e][bp] (bucket -> column of the sketch).
inline size_t prepare_bytes(const os_sketch* sk, int64_t n) {
    const int32_t bp = os_block_stride(sk->b);
    return align256(table_bytes(sk, n)) + align256(osk::list_bytes(nblocks(sk), n, bp)) +
           align256((size_t)nblocks(sk) * (size_t)bp * 4u);
}

inline const void* prep_lists(const void* prep, const os_sketch* sk, int64_t n) {
    return static_cast<const char*>(prep) + align256(table_bytes(sk, n));
}

inline const int32_t* prep_inv(const void* prep, const os_sketch* sk, int64_t n) {
    return reinterpret_cast<const int32_t*>(
        static_cast<const char*>(prep) + align256(table_bytes(sk, n)) +
        align256(osk::list_bytes(nblocks(sk), n, os_block_stride(sk->b))));
}

// Table + position map + bucket lists into the prepared buffer.  grouped:
// buckets of similar list lengths share the sketch kernel's 64-bucket
// groups (the sketches' columns then hold the buckets in that order within
// each block; products are unchanged); else the natural order.
inline os_status prepare(const os_sketch* sk, int64_t n, void* prep, hipStream_t s,
                         bool grouped = false) {
    const int64_t nt = table_stride(n);
    const int32_t bp = os_block_stride(sk->b);
    uint32_t* table = static_cast<uint32_t*>(prep);
    hipError_t e = sk->h ? osk::launch_table_explicit(sk->h, sk->sigma, nblocks(sk), n, nt, sk->b,
                                                      table, s)
                         : osk::launch_table_hash(sk->seed, nblocks(sk), n, nt, sk->b, table, s);
    if (e != hipSuccess) return hip_status(e);
    int32_t* inv = const_cast<int32_t*>(prep_inv(prep, sk, n));
    e = grouped ? osk::launch_group_buckets(table, n, nt, nblocks(sk), sk->b, bp, inv, s)
                : osk::launch_identity_inv(nblocks(sk), bp, inv, s);
    if (e != hipSuccess) return hip_status(e);
    void* lists = static_cast<char*>(prep) + align256(table_bytes(sk, n));
    return hip_status(osk::launch_build_lists(table, n, nt, nblocks(sk), bp, lists, s,
                                              grouped && sk->b > 64 ? inv : nullptr));
}

inline os_status check_prep(const os_sketch* sk, int64_t n, const void* prep, size_t prep_bytes) {
    if (!prep) return OS_ENULL;
    if (!aligned(prep, 256)) return OS_EALIGN;
    if (prep_bytes < prepare_bytes(sk, n)) return OS_EWORKSPACE;
    return OS_OK;
}

}  // namespace api
}  // namespace osk
