// sketch.hip -- count-sketch kernels for gfx950.
//
// Both kernels apply the blocks of S (Eq. (sketch_matrix)) to one operand:
// every input element x at sketched index k is added, with sign
// sigma_i(k), into bucket h_i(k) of every stored block i (Algorithm
// "Calculating Count-sketch of a matrix A", applied block by block as in
// Algorithm "Over sketching A in parallel").  Outputs are bucket-major: row
// j*bp + c of the result holds bucket c of stored block j for every line
// (the layout of S^T X), which is what the block product reads.
//
// Scheme: the buckets of a block are split into ranges of kRange buckets.
// For every (block, range) a list of the indices k that hash into the range
// is built once per call, in ascending k (build_lists).  One wave owns one
// (block, range): it keeps those kRange buckets for 64 lines in registers
// (lane = line, bucket chosen by a wave-uniform index) and walks its list,
// so every element is added exactly once, in ascending k, with no atomics
// and no two waves touching the same bucket.  (LDS float atomics are slow on
// this chip, so the bucket sums never go through them.)
//
// sketch_rows: X is n x cols row-major and the sketched index is the row:
//   lanes are 64 consecutive columns; a list entry k loads 256 contiguous
//   bytes of row k.  The (block, range) waves of one column strip are
//   scheduled together on one XCD, so the strip is read from HBM once and
//   re-read from that XCD's L2.
// sketch_cols: X is rows x n row-major and the sketched index is the column:
//   a workgroup of 16 waves stages a 64-row x 256-column tile of X through
//   LDS (coalesced reads, transposed, conflict-free layout) and every wave
//   takes the columns of its list from the tile; lanes are the 64 rows.
#include "internal.h"

namespace osk {
namespace {

constexpr int kRange = kBucketRange;   // buckets owned by one wave
constexpr int kBatch = kListBatch;     // list entries fetched per step

// Spread consecutive task ids over the 8 XCDs in contiguous runs: task T is
// run by the workgroup with linear id L where T = (L % 8) * (tasks / 8) + L / 8,
// so neighbouring tasks share an XCD and its L2.
__device__ __forceinline__ int64_t xcd_task(int64_t L, int64_t tasks) {
    if (tasks % 8 != 0) return L;
    return (L % 8) * (tasks / 8) + L / 8;
}

// Index of the wave within the workgroup, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t lanes_below() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
// Bucket lists, built for every sketch block i < nblk.  For block i and
// range p:
//   entries ent[i*nl + off[i][p] .. off[i][p+1]) = {k, (h - p*kRange) | sign<<31}
// for every k with h_i(k) in [p*kRange, (p+1)*kRange), k ascending.
// nl = n + kBatch (room for over-reads of a batch at the end of a list).
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

// Reads kBatch entries starting at list position `at` (uniform) into scalar
// registers.
__device__ __forceinline__ void load_batch(uint2 (&eb)[kBatch], const uint2* __restrict__ ent,
                                           uint32_t at) {
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
        const uint2 e = ent[at + u];
        eb[u] = make_uint2(uniform(e.x), uniform(e.y));
    }
}

__device__ __forceinline__ float entry_sign(uint32_t meta) {
    return (meta & 0x80000000u) ? -1.0f : 1.0f;
}

// The kRange (= 32) buckets of one list range, one line (column or row) per
// lane, live in a 32-wide register vector.  The bucket index is wave-uniform
// and selects a register by relative addressing (s_set_gpr_idx).
typedef float v32f __attribute__((ext_vector_type(32)));
static_assert(kRange == 32, "one register vector holds one bucket range");

__device__ __forceinline__ void bucket_add(v32f& acc, uint32_t c, float x, float s) {
    acc[c & 31u] = fmaf(x, s, acc[c & 31u]);
}

// Sign of a list entry as +-1.0f, built on the scalar unit from bit 31.
__device__ __forceinline__ float entry_sign_bits(uint32_t meta) {
    return __uint_as_float(0x3F800000u | (meta & 0x80000000u));
}

// acc_v[c] += x_v * s for the V register vectors of a wave (V lines per
// lane), c wave-uniform in [0, 32).  One relative-destination window
// (s_set_gpr_idx_on ... DST) covers the V multiply-adds: the destination
// register number of each v_fmac is offset by c.  The vectors are pinned to
// fixed registers (v64.., v96.., ...) so the instruction can name them.
#define OSK_FMAC_REL1(A0, C, X0, S)                                                              \
    asm volatile("s_set_gpr_idx_on %1, gpr_idx(DST)\n\ts_nop 0\n\t"                           \
                 "v_fmac_f32 v64, %2, %3\n\ts_set_gpr_idx_off"                                   \
                 : "+{v[64:95]}"(A0)                                                          \
                 : "s"(C), "v"(X0), "s"(S))
#define OSK_FMAC_REL_AT(REGS, FIRST, A, C, X, S)                                                 \
    asm volatile("s_set_gpr_idx_on %1, gpr_idx(DST)\n\ts_nop 0\n\t"                           \
                 "v_fmac_f32 " FIRST ", %2, %3\n\ts_set_gpr_idx_off"                             \
                 : "+{" REGS "}"(A)                                                          \
                 : "s"(C), "v"(X), "s"(S))
#define OSK_FMAC_REL2(A0, A1, C, X0, X1, S)                                                      \
    asm volatile("s_set_gpr_idx_on %2, gpr_idx(DST)\n\ts_nop 0\n\t"                           \
                 "v_fmac_f32 v64, %3, %5\n\tv_fmac_f32 v96, %4, %5\n\ts_set_gpr_idx_off"        \
                 : "+{v[64:95]}"(A0), "+{v[96:127]}"(A1)                                      \
                 : "s"(C), "v"(X0), "v"(X1), "s"(S))

// ---------------------------------------------------------------------------
// sketch_rows: out[j*bp + c][col] = sum_{k in bucket c of block j} sigma * X[k][col]
// Task = (strip of 128 columns, wave task q = (stored block j, range p)).
// Lane L owns columns 2L and 2L+1 of the strip; row k of the strip is read
// with one 8-byte buffer load per lane at scalar offset k * ldx * 4 (bytes
// past the end of X read as zero).
// ---------------------------------------------------------------------------
constexpr int kRowsCols = 128;

typedef __amdgpu_buffer_rsrc_t rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ __forceinline__ void rows_gather2(float2 (&x)[kBatch], const uint2 (&e)[kBatch],
                                             rsrc_t rs, uint32_t voff, uint32_t ld4) {
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)(e[u].x * ld4), 0);
        x[u] = make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
    }
}

template <bool kFull>
__device__ __forceinline__ void rows_accumulate2(v32f& a0, v32f& a1, const uint2 (&e)[kBatch],
                                                 const float2 (&x)[kBatch], uint32_t valid) {
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
        const bool take = kFull || (uint32_t)u < valid;
        const float x0 = take ? x[u].x : 0.f;
        const float x1 = take ? x[u].y : 0.f;
        const uint32_t c = e[u].y & (uint32_t)(kRange - 1);
        OSK_FMAC_REL2(a0, a1, c, x0, x1, entry_sign_bits(e[u].y));
    }
}

__global__ __launch_bounds__(256) void sketch_rows_kernel(
    const float* __restrict__ X, int64_t n, int64_t cols, int64_t ldx, int32_t bp, int32_t P,
    int32_t Q, BlockList bl, const uint32_t* __restrict__ off, const uint2* __restrict__ ent,
    float* __restrict__ out, int64_t ldo) {
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const int64_t qgroups = (Q + 3) / 4;
    const int64_t strips = (cols + kRowsCols - 1) / kRowsCols;
    const int64_t task = xcd_task(blockIdx.x, strips * qgroups);
    const int64_t strip = task / qgroups;
    const int q = (int)(task % qgroups) * 4 + wave;
    if (q >= Q) return;
    const int j = q / P;
    const int p = q % P;
    const int64_t col0 = strip * kRowsCols;
    // buffer over X from column col0 of row 0 to the end of X
    const float* base = X + col0;
    const uint32_t bytes = (uint32_t)(((n - 1) * ldx + cols - col0) * 4);
    const rsrc_t rs = make_rsrc(base, bytes);
    const uint32_t voff = (uint32_t)lane * 8u;
    const uint32_t ld4 = (uint32_t)(ldx * 4);

    v32f a0 = 0.f, a1 = 0.f;

    const int64_t sb = bl.idx[j];                      // sketch block of stored block j
    const uint2* le = ent + sb * (n + kBatch);
    const uint32_t beg = off[sb * (P + 1) + p];
    const uint32_t end = off[sb * (P + 1) + p + 1];
    // Full batches, two in flight: the loads of batch i+1 are issued before
    // batch i is accumulated.  Then the partial last batch.
    const uint32_t full_end = beg + (end - beg) / kBatch * kBatch;
    uint2 ea[kBatch], eb[kBatch];
    float2 xa[kBatch], xb[kBatch];
    uint32_t at = beg;
    if (at < full_end) {
        load_batch(ea, le, at);
        rows_gather2(xa, ea, rs, voff, ld4);
    }
    while (at < full_end) {
        const uint32_t nb = at + kBatch;
        if (nb < full_end) {
            load_batch(eb, le, nb);
            rows_gather2(xb, eb, rs, voff, ld4);
        }
        rows_accumulate2<true>(a0, a1, ea, xa, kBatch);
        if (nb >= full_end) break;
        const uint32_t nc = nb + kBatch;
        if (nc < full_end) {
            load_batch(ea, le, nc);
            rows_gather2(xa, ea, rs, voff, ld4);
        }
        rows_accumulate2<true>(a0, a1, eb, xb, kBatch);
        at = nc;
    }
    if (full_end < end) {
        load_batch(ea, le, full_end);
        rows_gather2(xa, ea, rs, voff, ld4);
        rows_accumulate2<false>(a0, a1, ea, xa, end - full_end);
    }

    const int64_t colA = col0 + 2 * lane;
    const int64_t obase = (int64_t)j * bp + (int64_t)p * kRange;
    const int cmax = min(kRange, bp - p * kRange);
#pragma unroll
    for (int c = 0; c < kRange; ++c) {
        if (c < cmax) {
            float* o = out + (obase + c) * ldo + colA;
            if (colA + 1 < cols) {
                o[0] = a0[c];
                o[1] = a1[c];
            } else if (colA < cols) {
                o[0] = a0[c];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// sketch_cols: out[j*bp + c][r] = sum_{k in bucket c of block j} sigma * X[r][k]
// Task = (slab of 64 rows, group of 8 wave tasks); a wave task is a range of
// 128 buckets (four consecutive list ranges) of one stored block, held in four
// 32-wide register vectors.  LDS: two tiles [kTileK][65] (k-major; the one
// padding column keeps the transposed writes and the column reads
// conflict-free).
// ---------------------------------------------------------------------------
constexpr int kColsWaves = 8;
constexpr int kColsThreads = 64 * kColsWaves;
constexpr int kTileK = 256;
constexpr int kTileLd = 65;

// Staging of a 64-row x kTileK tile.  Thread (wave w, lane L) covers rows
// 8w + 4g + (L & 3) (g = 0, 1) and the float4s at columns 4(L >> 2) + 64 i
// (i < 4): eight float4 per thread.  Rows past the end read the last row
// (their buckets are never written out).
struct ColsStager {
    const float* src[2];  // X + row_g * ldx + 4 * (lane >> 2)
    int64_t kfirst;       // 4 * (lane >> 2)
    int rl;               // local row of group 0
    __device__ __forceinline__ void init(const float* X, int64_t rows, int64_t ldx, int64_t row0) {
        const int wave = threadIdx.x >> 6;
        const int lane = threadIdx.x & 63;
        rl = 8 * wave + (lane & 3);
        kfirst = 4 * (lane >> 2);
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int64_t row = min(row0 + rl + 4 * g, rows - 1);
            src[g] = X + row * ldx + kfirst;
        }
    }
    __device__ __forceinline__ void load(float4 (&r)[8], int64_t k0, int64_t n) const {
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (k0 + kfirst + 64 * i < n)
                    r[4 * g + i] = *reinterpret_cast<const float4*>(src[g] + k0 + 64 * i);
                else
                    r[4 * g + i] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
    }
    // tile[k][row]: lane L of a wave writes bank (L + const) mod 64, since
    // the row stride kTileLd = 65 is 1 mod 64.
    __device__ __forceinline__ void store(float* tile, const float4 (&r)[8]) const {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            float* t = tile + kfirst * kTileLd + rl + 4 * g;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                t[(64 * i + 0) * kTileLd] = r[4 * g + i].x;
                t[(64 * i + 1) * kTileLd] = r[4 * g + i].y;
                t[(64 * i + 2) * kTileLd] = r[4 * g + i].z;
                t[(64 * i + 3) * kTileLd] = r[4 * g + i].w;
            }
        }
    }
};

// acc[c] += x * s for list slot R of the wave (slot R's 32 buckets live in
// v[64+32R : 95+32R]).
template <int R>
__device__ __forceinline__ void cols_fmac(v32f& acc, uint32_t c, float x, float s) {
    if constexpr (R == 0) OSK_FMAC_REL_AT("v[64:95]", "v64", acc, c, x, s);
    else if constexpr (R == 1) OSK_FMAC_REL_AT("v[96:127]", "v96", acc, c, x, s);
    else if constexpr (R == 2) OSK_FMAC_REL_AT("v[128:159]", "v128", acc, c, x, s);
    else OSK_FMAC_REL_AT("v[160:191]", "v160", acc, c, x, s);
}

// Adds this chunk's share of one list (entries with k < kend) into its 32
// buckets.  Tile reads are issued without branches (entries not taken read a
// clamped, valid tile row and are masked).
template <int R>
__device__ __forceinline__ void cols_consume(v32f& acc, const float* tile,
                                             const uint2* __restrict__ le, uint32_t& at,
                                             uint32_t end, uint32_t kbeg, uint32_t kend, int lane) {
    while (at < end) {
        uint2 eb[kBatch];
        load_batch(eb, le, at);
        int take = 0;
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
            if (at + u < end && eb[u].x < kend) take = u + 1;
        if (take == 0) break;
        float xv[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const uint32_t kk = min(eb[u].x - kbeg, (uint32_t)(kTileK - 1));
            xv[u] = tile[kk * kTileLd + lane];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const float v = (u < take) ? xv[u] : 0.f;
            cols_fmac<R>(acc, eb[u].y & (uint32_t)(kRange - 1), v, entry_sign_bits(eb[u].y));
        }
        at += take;
        if (take < kBatch) break;
    }
}

__global__ __launch_bounds__(kColsThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void sketch_cols_kernel(const float* __restrict__ X, int64_t rows, int64_t n, int64_t ldx,
                        int32_t bp, int32_t P, int32_t Q4, BlockList bl,
                        const uint32_t* __restrict__ off, const uint2* __restrict__ ent,
                        float* __restrict__ out, int64_t ldo) {
    __shared__ __align__(16) float tiles[2][kTileK * kTileLd];
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const int P4 = (P + 3) / 4;                        // 128-bucket ranges per block
    const int64_t qgroups = (Q4 + kColsWaves - 1) / kColsWaves;
    const int64_t slabs = (rows + 63) / 64;
    const int64_t task = xcd_task(blockIdx.x, slabs * qgroups);
    const int64_t slab = task / qgroups;
    const int q = (int)(task % qgroups) * kColsWaves + wave;
    const bool active = q < Q4;                        // idle waves still stage tiles
    const int j = active ? q / P4 : 0;
    const int p4 = active ? q % P4 : 0;
    const int64_t row0 = slab * 64;

    // buckets 32r .. 32r+31 of the wave's range come from list range 4*p4 + r
    v32f a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    const int64_t sb = bl.idx[j];                      // sketch block of stored block j
    const uint2* le = ent + sb * (n + kBatch);
    uint32_t at[4], end[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int pr = 4 * p4 + r;
        const bool has = active && pr < P;
        at[r] = has ? off[sb * (P + 1) + pr] : 0u;
        end[r] = has ? off[sb * (P + 1) + pr + 1] : 0u;
    }

    ColsStager stg;
    stg.init(X, rows, ldx, row0);
    const int64_t chunks = (n + kTileK - 1) / kTileK;
    // sa / sc: staged data of the next two chunks (the loads of chunk t+2 are
    // issued while chunk t is consumed).
    float4 sa[8], sc[8];
    stg.load(sa, 0, n);
    stg.store(tiles[0], sa);
    if (chunks > 1) stg.load(sa, kTileK, n);
    __syncthreads();
    for (int64_t t = 0; t < chunks; t += 2) {
        if (t + 2 < chunks) stg.load(sc, (t + 2) * kTileK, n);
        {
            const uint32_t kb = (uint32_t)(t * kTileK), ke = (uint32_t)min((t + 1) * kTileK, n);
            cols_consume<0>(a0, tiles[0], le, at[0], end[0], kb, ke, lane);
            cols_consume<1>(a1, tiles[0], le, at[1], end[1], kb, ke, lane);
            cols_consume<2>(a2, tiles[0], le, at[2], end[2], kb, ke, lane);
            cols_consume<3>(a3, tiles[0], le, at[3], end[3], kb, ke, lane);
        }
        if (t + 1 < chunks) stg.store(tiles[1], sa);
        __syncthreads();
        if (t + 1 >= chunks) break;
        if (t + 3 < chunks) stg.load(sa, (t + 3) * kTileK, n);
        {
            const uint32_t kb = (uint32_t)((t + 1) * kTileK), ke = (uint32_t)min((t + 2) * kTileK, n);
            cols_consume<0>(a0, tiles[1], le, at[0], end[0], kb, ke, lane);
            cols_consume<1>(a1, tiles[1], le, at[1], end[1], kb, ke, lane);
            cols_consume<2>(a2, tiles[1], le, at[2], end[2], kb, ke, lane);
            cols_consume<3>(a3, tiles[1], le, at[3], end[3], kb, ke, lane);
        }
        if (t + 2 < chunks) stg.store(tiles[0], sc);
        __syncthreads();
    }

    const int64_t row = row0 + lane;
    if (!active || row >= rows) return;
    const int64_t base = (int64_t)j * bp + (int64_t)p4 * 4 * kRange;
    const int cmax = min(4 * kRange, bp - p4 * 4 * kRange);
#pragma unroll
    for (int c = 0; c < 4 * kRange; ++c) {
        if (c < cmax) {
            const float v = c < 32 ? a0[c] : c < 64 ? a1[c - 32] : c < 96 ? a2[c - 64] : a3[c - 96];
            out[(base + c) * ldo + row] = v;
        }
    }
}

}  // namespace

int32_t list_ranges(int32_t bp) { return (bp + kRange - 1) / kRange; }

size_t list_bytes(int32_t nst, int64_t n, int32_t bp) {
    const int64_t P = list_ranges(bp);
    const size_t counts = (size_t)nst * P * 4u;
    const size_t offs = (size_t)nst * (P + 1) * 4u;
    const size_t ents = (size_t)nst * (n + kBatch) * 8u;
    return round_up(counts, 256) + round_up(offs, 256) + round_up(ents, 256);
}

namespace {
struct ListView {
    uint32_t* cnt;
    uint32_t* off;
    uint2* ent;
};
ListView carve_lists(void* lists, int32_t nst, int32_t P) {
    char* base = static_cast<char*>(lists);
    ListView v;
    v.cnt = reinterpret_cast<uint32_t*>(base);
    v.off = reinterpret_cast<uint32_t*>(base + round_up((int64_t)nst * P * 4, 256));
    v.ent = reinterpret_cast<uint2*>(reinterpret_cast<char*>(v.off) +
                                     round_up((int64_t)nst * (P + 1) * 4, 256));
    return v;
}
}  // namespace

hipError_t launch_build_lists(const uint32_t* table, int64_t n, int64_t nt, int32_t nblk,
                              int32_t bp, void* lists, hipStream_t s) {
    const int32_t P = list_ranges(bp);
    const ListView v = carve_lists(lists, nblk, P);
    hipLaunchKernelGGL(count_lists_kernel, dim3(P, nblk), dim3(64), 0, s, table, n, nt, P, v.cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fill_lists_kernel, dim3(P, nblk), dim3(64), 0, s, table, n, nt, P, v.cnt,
                       v.off, v.ent);
    return hipGetLastError();
}

bool plan_sketch_ok(int64_t lines, int32_t nst, int32_t bp, int64_t n) {
    if (lines < 1 || nst < 1 || nst > OS_MAX_BLOCKS || bp < kBlockAlign || bp % kBlockAlign ||
        n < 1)
        return false;
    if (n > kMaxSketchedLen) return false;
    const int64_t Q = (int64_t)nst * list_ranges(bp);
    const int64_t tasks = (lines + 63) / 64 * ((Q + 3) / 4);
    return tasks <= 0x7fffffff;
}

bool plan_sketch_rows_ok(int64_t n, int64_t cols, int64_t ldx, int32_t nst, int32_t bp) {
    // row offsets are 32-bit byte offsets into one buffer resource
    return plan_sketch_ok(cols, nst, bp, n) && ((n - 1) * ldx + cols) * 4 <= 0x7fffffffLL;
}

hipError_t launch_sketch_rows(const float* X, int64_t n, int64_t cols, int64_t ldx,
                              const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                              const void* lists, float* out, int64_t ldo, hipStream_t s) {
    if (!plan_sketch_rows_ok(n, cols, ldx, nst, bp)) return hipErrorInvalidValue;
    const int32_t P = list_ranges(bp);
    const int32_t Q = nst * P;
    const ListView v = carve_lists(const_cast<void*>(lists), nblk, P);
    const int64_t tasks = (cols + kRowsCols - 1) / kRowsCols * ((Q + 3) / 4);
    hipLaunchKernelGGL(sketch_rows_kernel, dim3((unsigned)tasks), dim3(256), 0, s, X, n, cols, ldx,
                       bp, P, Q, bl, v.off, v.ent, out, ldo);
    return hipGetLastError();
}

hipError_t launch_sketch_cols(const float* X, int64_t rows, int64_t n, int64_t ldx,
                              const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                              const void* lists, float* out, int64_t ldo, hipStream_t s) {
    if (!plan_sketch_ok(rows, nst, bp, n)) return hipErrorInvalidValue;
    const int32_t P = list_ranges(bp);
    const int32_t Q = nst * P;
    const ListView v = carve_lists(const_cast<void*>(lists), nblk, P);
    const int32_t Q4 = nst * ((P + 3) / 4);
    const int64_t tasks = (rows + 63) / 64 * ((Q4 + kColsWaves - 1) / kColsWaves);
    hipLaunchKernelGGL(sketch_cols_kernel, dim3((unsigned)tasks), dim3(kColsThreads), 0, s, X, rows,
                       n, ldx, bp, P, Q4, bl, v.off, v.ent, out, ldo);
    return hipGetLastError();
}

}  // namespace osk
