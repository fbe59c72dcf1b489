// sketch.hip -- count-sketch kernels for gfx950.
//
// Both sketches apply the blocks of S (Eq. (sketch_matrix)) to one operand:
// every input element x at sketched index k is added, with sign
// sigma_i(k), into bucket h_i(k) of every stored block i (Algorithm
// "Calculating Count-sketch of a matrix A", applied block by block as in
// Algorithm "Over sketching A in parallel").  Outputs are bucket-major: row
// j*bp + c of the result holds bucket c of stored block j for every line
// (the layout of S^T X), which is what the block product reads.
//
// Scheme: the count sketch of a matrix Y whose rows are the sketched index
// (Y n x L row-major) is a gather-reduce.  The prepared sketch lists, for
// every (block, bucket), the indices k that hash into the bucket, ascending,
// with their signs (bucket_split).  A group of W/4 lanes produces one bucket
// row for a strip of W columns: it walks the bucket's list, loading the W
// columns of each listed row with 16-byte loads and adding them with their
// signs, in ascending k.  No atomics, no scatter, no cross-lane reduction:
// every output element is summed by one lane and written once.
//
// sketch_rows (S^T B, B row-major) is that gather-reduce directly.
// sketch_cols (A S for A row-major, sketched along its rows) first transposes
// A into the caller's workspace (LDS-tiled, coalesced on both sides) and then
// runs the same gather-reduce on A^T.
//
// Workgroups are ordered strip-major and spread over the XCDs in contiguous
// runs, so the workgroups that read one column strip run on one XCD and
// re-read it from that XCD's L2.
#include "internal.h"

namespace osk {
namespace {

constexpr int kRange = kBucketRange;   // buckets per range list (32)
constexpr int kBatch = kListBatch;     // slack at the end of each block's list

// Spread consecutive task ids over the 8 XCDs in contiguous runs: task T is
// run by the workgroup with linear id L where T = (L % 8) * (tasks / 8) + L / 8,
// so neighbouring tasks share an XCD and its L2.
__device__ __forceinline__ int64_t xcd_task(int64_t L, int64_t tasks) {
    if (tasks % 8 != 0) return L;
    return (L % 8) * (tasks / 8) + L / 8;
}

// Index of the wave within the workgroup, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ __forceinline__ uint64_t lanes_below() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
// Range lists, built for every sketch block i < nblk.  For block i and range
// p of kRange buckets:
//   ent[i*(n+kBatch) + off[i][p] .. off[i][p+1]) = {k, (h - p*kRange) | sign<<31}
// for every k with h_i(k) in [p*kRange, (p+1)*kRange), k ascending.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void count_lists_kernel(const uint32_t* __restrict__ table,
                                                         int64_t n, int64_t nt, int32_t P,
                                                         uint32_t* __restrict__ cnt) {
    const int p = blockIdx.x;
    const int j = blockIdx.y;
    const uint32_t* row = table + (int64_t)j * nt;
    uint32_t c = 0;
    for (int64_t k = threadIdx.x; k < n; k += 64)
        c += (((row[k] & 0x7FFFFFFFu) / kRange) == (uint32_t)p) ? 1u : 0u;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) c += __shfl_xor(c, s);
    if (threadIdx.x == 0) cnt[(int64_t)j * P + p] = c;
}

__global__ __launch_bounds__(64) void fill_lists_kernel(const uint32_t* __restrict__ table, int64_t n,
                                                        int64_t nt, int32_t P,
                                                        const uint32_t* __restrict__ cnt,
                                                        uint32_t* __restrict__ off,
                                                        uint2* __restrict__ ent) {
    const int p = blockIdx.x;
    const int j = blockIdx.y;
    const int lane = threadIdx.x;
    // offset of this range within the block's entries
    uint32_t before = 0;
    for (int q = lane; q < p; q += 64) before += cnt[(int64_t)j * P + q];
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) before += __shfl_xor(before, s);
    if (lane == 0) {
        off[(int64_t)j * (P + 1) + p] = before;
        if (p == P - 1) off[(int64_t)j * (P + 1) + P] = before + cnt[(int64_t)j * P + p];
    }
    const uint32_t* row = table + (int64_t)j * nt;
    uint2* out = ent + (int64_t)j * (n + kBatch) + before;
    const uint64_t below = lanes_below();
    uint32_t pos = 0;
    for (int64_t k0 = 0; k0 < n; k0 += 64) {
        const int64_t k = k0 + lane;
        const uint32_t e = k < n ? row[k] : 0u;
        const uint32_t h = e & 0x7FFFFFFFu;
        const bool mine = k < n && h / kRange == (uint32_t)p;
        const uint64_t mask = __ballot(mine);
        if (mine) {
            const uint32_t at = pos + (uint32_t)__popcll(mask & below);
            out[at] = make_uint2((uint32_t)k, (h - (uint32_t)p * kRange) | (e & 0x80000000u));
        }
        pos += (uint32_t)__popcll(mask);
    }
}

// ---------------------------------------------------------------------------
// Bucket lists: a stable split of every range list into its kRange buckets.
//   boff[i][c] .. boff[i][c+1]   entries of bucket c of block i (boff[i][bp] =
//                                the block's total)
//   bent[i*n + t] = {k, sign as +-1.0f}, k ascending within a bucket
// One wave per (range, block).  Bucket positions share the range list's
// index space: a range's buckets are a permutation of its list.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void bucket_split_kernel(const uint32_t* __restrict__ off,
                                                          const uint2* __restrict__ ent, int64_t n,
                                                          int32_t P, int32_t bp,
                                                          uint32_t* __restrict__ boff,
                                                          uint2* __restrict__ bent,
                                                          float* __restrict__ zero) {
    const int p = blockIdx.x;
    const int64_t blk = blockIdx.y;
    const int lane = threadIdx.x;
    if (p == 0 && blk == 0) zero[lane] = 0.f;   // kZeroFloats = 64 = one wave
    const uint32_t beg = off[blk * (P + 1) + p];
    const uint32_t end = off[blk * (P + 1) + p + 1];
    const uint2* le = ent + blk * (n + kBatch);
    const uint64_t below = lanes_below();

    // entries per bucket: lane c < kRange counts bucket c
    uint32_t count = 0;
    for (uint32_t a = beg; a < end; a += 64) {
        const uint32_t i = a + lane;
        const uint32_t c = i < end ? (le[i].y & (kRange - 1)) : (uint32_t)kRange;
#pragma unroll
        for (int b = 0; b < kRange; ++b) {
            const uint32_t m = (uint32_t)__popcll(__ballot(c == (uint32_t)b));
            if (lane == b) count += m;
        }
    }
    // exclusive prefix over the buckets of the range
    uint32_t incl = count;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    uint32_t next = beg + incl - count;   // next free position of bucket `lane`
    if (lane < kRange && p * kRange + lane < bp) boff[blk * (bp + 1) + p * kRange + lane] = next;
    if (p == P - 1 && lane == 0) boff[blk * (bp + 1) + bp] = end;

    uint2* out = bent + blk * n;
    for (uint32_t a = beg; a < end; a += 64) {
        const uint32_t i = a + lane;
        const bool valid = i < end;
        const uint2 e = valid ? le[i] : make_uint2(0u, 0u);
        const uint32_t c = valid ? (e.y & (kRange - 1)) : (uint32_t)kRange;
        uint32_t at = 0;
#pragma unroll
        for (int b = 0; b < kRange; ++b) {
            const uint64_t mask = __ballot(c == (uint32_t)b);
            const uint32_t start = __shfl(next, b);
            if (c == (uint32_t)b) at = start + (uint32_t)__popcll(mask & below);
            if (lane == b) next += (uint32_t)__popcll(mask);
        }
        if (valid)
            out[at] = make_uint2(e.x, __float_as_uint((e.y & 0x80000000u) ? -1.0f : 1.0f));
    }
}

// ---------------------------------------------------------------------------
// Transpose: Y (n x rows, ld ldy) = X^T for X rows x n (ld ldx, 16-byte rows).
// 64 x 64 tiles through LDS (row stride 65: conflict-free both ways); 256
// threads, four float4 per thread each way.  Columns of Y at or past `rows`
// (up to ldy) are written as zero.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void transpose_kernel(const float* __restrict__ X, int64_t rows,
                                                        int64_t n, int64_t ldx,
                                                        float* __restrict__ Y, int64_t ldy) {
    __shared__ float t[64][65];
    const int tid = threadIdx.x;
    const int64_t row_tiles = (rows + 63) / 64;
    const int64_t k0 = (int64_t)blockIdx.x / row_tiles * 64;   // column tile of X (row tile of Y)
    const int64_t r0 = (int64_t)blockIdx.x % row_tiles * 64;   // row tile of X
    const int sub = tid >> 4;                      // 0..15
    const int c4 = 4 * (tid & 15);                 // 0..60
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = sub + 16 * i;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r0 + r < rows && k0 + c4 < n)
            v = *reinterpret_cast<const float4*>(X + (r0 + r) * ldx + k0 + c4);
        t[r][c4 + 0] = v.x;
        t[r][c4 + 1] = v.y;
        t[r][c4 + 2] = v.z;
        t[r][c4 + 3] = v.w;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int kr = sub + 16 * i;
        const int64_t k = k0 + kr;
        const int64_t col = r0 + c4;
        if (k < n && col < ldy) {
            const float4 v = make_float4(t[c4 + 0][kr], t[c4 + 1][kr], t[c4 + 2][kr], t[c4 + 3][kr]);
            *reinterpret_cast<float4*>(Y + k * ldy + col) = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Gather-reduce: out[(j*bp + c)*ldo + l] = sum_{k in bucket c of block bl[j]}
// sign * Y[k][l] for Y n x L row-major (ld ldy).  A lane group of W/4 lanes
// owns one bucket row of a strip of W columns (one 16-byte column quad per
// lane) and walks that bucket's list U rows at a time, in ascending k; a wave
// holds 64/(W/4) groups (consecutive buckets), a workgroup 4 waves.  Rows past
// the end of a group's list are masked.  kVec: Y 16-byte aligned
// with ldy a multiple of 4 (16-byte loads; quads past L are clamped and never
// stored), else four 4-byte loads per quad.
// ---------------------------------------------------------------------------
template <int W>
struct GatherShape {
    static constexpr int Q = W / 4;       // lanes per group
    static constexpr int G = 64 / Q;      // groups (buckets) per wave
    static constexpr int kBuckets = 4 * G;  // buckets per workgroup
};

template <int W, bool kVec>
__global__ __launch_bounds__(256) void gather_kernel(const float* __restrict__ Y, int64_t n,
                                                     int64_t L, int64_t ldy, int32_t bp, int32_t nst,
                                                     BlockList bl, const uint32_t* __restrict__ boff,
                                                     const uint2* __restrict__ bent,
                                                     const float* __restrict__ zero,
                                                     float* __restrict__ out, int64_t ldo) {
    using Sh = GatherShape<W>;
    constexpr int Q = Sh::Q;
    constexpr int U = 8;           // rows per group per step
    const int lane = threadIdx.x & 63;
    const int g = lane / Q;
    const int q = lane % Q;
    const int64_t strips = (L + W - 1) / W;
    const int64_t groups = (bp + Sh::kBuckets - 1) / Sh::kBuckets;
    const int64_t per_strip = (int64_t)nst * groups;
    const int64_t task = xcd_task(blockIdx.x, strips * per_strip);
    const int64_t strip = task / per_strip;
    const int64_t rem = task % per_strip;
    const int j = (int)(rem / groups);
    // with one group per wave the bucket is wave-uniform: its list is then
    // read with scalar loads
    const int c = (int)(rem % groups) * Sh::kBuckets +
                  (Sh::G == 1 ? wave_id() : (int)(threadIdx.x / Q));
    const bool has = c < bp;
    const int64_t sb = bl.idx[j];
    const uint32_t beg = has ? boff[sb * (bp + 1) + c] : 0u;
    const uint32_t cnt = has ? boff[sb * (bp + 1) + c + 1] - beg : 0u;
    // (an empty list reads entry 0 of the block, always valid, and masks it)
    const uint2* __restrict__ e = bent + sb * n + (cnt > 0 ? beg : 0u);
    const uint32_t last = cnt > 0 ? cnt - 1 : 0u;
    const int64_t col = strip * W + 4 * q;
    const int64_t L4 = (L + 3) / 4 * 4;
    const int64_t lcol = kVec ? min(col, L4 - 4) : col;

    uint32_t most = cnt;           // longest list of the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) most = max(most, (uint32_t)__shfl_xor((int)most, d));

    // Loads are unconditional: a row past the end of a group's list reads the
    // 16 zero bytes at `zero` instead, so no branch sits around a load
    // (branches there make every load wait for the previous ones).
    const float* yq = Y + lcol;
    const uint32_t ld4 = (uint32_t)(ldy * 4);   // row pitch in bytes (< 4 GiB, checked at launch)
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (uint32_t it = 0; it < most; it += U) {
        uint2 en[U];
#pragma unroll
        for (int u = 0; u < U; ++u) en[u] = e[min(it + u, last)];
        float4 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = it + u < cnt;
            if constexpr (kVec) {
                const float* p = reinterpret_cast<const float*>(
                    reinterpret_cast<const char*>(yq) + (uint64_t)en[u].x * ld4);
                x[u] = *reinterpret_cast<const float4*>(ok ? p : zero);
            } else {
                const float* p = Y + (int64_t)en[u].x * ldy;
                x[u].x = *(ok ? p + min(col + 0, L - 1) : zero + 0);
                x[u].y = *(ok ? p + min(col + 1, L - 1) : zero + 1);
                x[u].z = *(ok ? p + min(col + 2, L - 1) : zero + 2);
                x[u].w = *(ok ? p + min(col + 3, L - 1) : zero + 3);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float s = __uint_as_float(en[u].y);   // +-1; masked rows add +-0
            acc.x = fmaf(s, x[u].x, acc.x);
            acc.y = fmaf(s, x[u].y, acc.y);
            acc.z = fmaf(s, x[u].z, acc.z);
            acc.w = fmaf(s, x[u].w, acc.w);
        }
    }
    if (!has || col >= L) return;
    float* o = out + ((int64_t)j * bp + c) * ldo + col;
    if (col + 3 < L) {
        *reinterpret_cast<float4*>(o) = acc;
    } else {
        o[0] = acc.x;
        if (col + 1 < L) o[1] = acc.y;
        if (col + 2 < L) o[2] = acc.z;
    }
}

struct ListView {
    uint32_t* cnt;
    uint32_t* off;
    uint2* ent;
    uint32_t* boff;
    uint2* bent;
    float* zero;     // kZeroFloats zeros (rows past the end of a list read these)
};
constexpr int kZeroFloats = 64;

ListView carve_lists(void* lists, int32_t nblk, int64_t n, int32_t bp) {
    const int64_t P = list_ranges(bp);
    char* base = static_cast<char*>(lists);
    ListView v;
    v.cnt = reinterpret_cast<uint32_t*>(base);
    base += round_up((int64_t)nblk * P * 4, 256);
    v.off = reinterpret_cast<uint32_t*>(base);
    base += round_up((int64_t)nblk * (P + 1) * 4, 256);
    v.ent = reinterpret_cast<uint2*>(base);
    base += round_up((int64_t)nblk * (n + kBatch) * 8, 256);
    v.boff = reinterpret_cast<uint32_t*>(base);
    base += round_up((int64_t)nblk * (bp + 1) * 4, 256);
    v.bent = reinterpret_cast<uint2*>(base);
    base += round_up((int64_t)nblk * n * 8, 256);
    v.zero = reinterpret_cast<float*>(base);
    return v;
}

// Column strip width of the gather: 64 columns (256-byte rows, 4 buckets per
// wave).  Measured on the full-size case against 32 and 256 columns: the
// sketch of a 32768 x 8192 operand takes 1.44 ms at 64, 1.73 ms at 32 and
// 1.51 ms at 256.
constexpr int kStrip = 64;

template <int W>
int64_t gather_tasks(int64_t L, int32_t nst, int32_t bp) {
    const int64_t per = GatherShape<W>::kBuckets;
    return (L + W - 1) / W * nst * ((bp + per - 1) / per);
}

template <int W>
hipError_t launch_gather(const float* Y, int64_t n, int64_t L, int64_t ldy, const BlockList& bl,
                         int32_t nst, int32_t bp, const ListView& v, float* out, int64_t ldo,
                         hipStream_t s) {
    const int64_t tasks = gather_tasks<W>(L, nst, bp);
    const bool vec = (reinterpret_cast<uintptr_t>(Y) & 15) == 0 && (ldy & 3) == 0;
    if (vec)
        hipLaunchKernelGGL((gather_kernel<W, true>), dim3((unsigned)tasks), dim3(256), 0, s, Y, n, L,
                           ldy, bp, nst, bl, v.boff, v.bent, v.zero, out, ldo);
    else
        hipLaunchKernelGGL((gather_kernel<W, false>), dim3((unsigned)tasks), dim3(256), 0, s, Y, n,
                           L, ldy, bp, nst, bl, v.boff, v.bent, v.zero, out, ldo);
    return hipGetLastError();
}

}  // namespace

int32_t list_ranges(int32_t bp) { return (bp + kRange - 1) / kRange; }

size_t list_bytes(int32_t nblk, int64_t n, int32_t bp) {
    const int64_t P = list_ranges(bp);
    return (size_t)(round_up((int64_t)nblk * P * 4, 256) + round_up((int64_t)nblk * (P + 1) * 4, 256) +
                    round_up((int64_t)nblk * (n + kBatch) * 8, 256) +
                    round_up((int64_t)nblk * (bp + 1) * 4, 256) + round_up((int64_t)nblk * n * 8, 256) +
                    kZeroFloats * 4);
}

hipError_t launch_build_lists(const uint32_t* table, int64_t n, int64_t nt, int32_t nblk,
                              int32_t bp, void* lists, hipStream_t s) {
    const int32_t P = list_ranges(bp);
    const ListView v = carve_lists(lists, nblk, n, bp);
    hipLaunchKernelGGL(count_lists_kernel, dim3(P, nblk), dim3(64), 0, s, table, n, nt, P, v.cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fill_lists_kernel, dim3(P, nblk), dim3(64), 0, s, table, n, nt, P, v.cnt,
                       v.off, v.ent);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(bucket_split_kernel, dim3(P, nblk), dim3(64), 0, s, v.off, v.ent, n, P, bp,
                       v.boff, v.bent, v.zero);
    return hipGetLastError();
}

bool plan_sketch_ok(int64_t lines, int32_t nst, int32_t bp, int64_t n) {
    if (lines < 1 || nst < 1 || nst > OS_MAX_BLOCKS || bp < kBlockAlign || bp % kBlockAlign ||
        n < 1 || n > kMaxSketchedLen)
        return false;
    const int64_t tasks = gather_tasks<kStrip>(lines, nst, bp);
    const int64_t tiles = (n + 63) / 64 * ((lines + 63) / 64);
    return tasks <= 0x7fffffff && tiles <= 0x7fffffff;
}

size_t sketch_cols_workspace_bytes(int64_t rows, int64_t n) {
    return (size_t)round_up(n * round_up(rows, 4) * 4, 256);
}

bool plan_sketch_rows_ok(int64_t n, int64_t cols, int64_t ldx, int32_t nst, int32_t bp) {
    return plan_sketch_ok(cols, nst, bp, n) && ldx < (int64_t(1) << 30);
}

hipError_t launch_sketch_rows(const float* X, int64_t n, int64_t cols, int64_t ldx,
                              const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                              const void* lists, float* out, int64_t ldo, hipStream_t s) {
    if (!plan_sketch_rows_ok(n, cols, ldx, nst, bp)) return hipErrorInvalidValue;
    const ListView v = carve_lists(const_cast<void*>(lists), nblk, n, bp);
    return launch_gather<kStrip>(X, n, cols, ldx, bl, nst, bp, v, out, ldo, s);
}

hipError_t launch_sketch_cols(const float* X, int64_t rows, int64_t n, int64_t ldx,
                              const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                              const void* lists, float* out, int64_t ldo, void* workspace,
                              hipStream_t s) {
    if (!plan_sketch_ok(rows, nst, bp, n)) return hipErrorInvalidValue;
    float* Xt = static_cast<float*>(workspace);
    const int64_t ldt = round_up(rows, 4);
    const int64_t tiles = (n + 63) / 64 * ((rows + 63) / 64);
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)tiles), dim3(256), 0, s, X, rows, n, ldx, Xt,
                       ldt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const ListView v = carve_lists(const_cast<void*>(lists), nblk, n, bp);
    return launch_gather<kStrip>(Xt, n, rows, ldt, bl, nst, bp, v, out, ldo, s);
}

}  // namespace osk
