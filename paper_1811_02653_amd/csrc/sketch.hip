// sketch.hip -- count-sketch kernels for gfx950.
//
// Both sketches apply the blocks of S (Eq. (sketch_matrix)) to one operand:
// every input element x at sketched index k is added, with sign sigma_i(k),
// into bucket h_i(k) of every stored block i (Algorithm "Calculating
// Count-sketch of a matrix A", applied block by block as in Algorithm "Over
// sketching A in parallel").
//
// A "line" is a vector over the sketched index: a row of A (m lines of
// length n) or a column of B (l lines of length n).  The sketch of a line is
// a row of the output: out[line][j*bp + c] = bucket c of stored block j
// (line-major; the sketch of A is A S, the sketch of B is (S^T B)^T).
//
// Scheme (read-once): a workgroup owns kLines = 4 lines and keeps ALL their
// buckets -- every stored block -- in registers (a pass covers up to
// 8 * kMaxSlots groups of 64 buckets; wider sketches take several passes).
// It walks the sketched index in windows of kWin = 8192: the window of its
// 4 lines is staged in LDS once as kWin float4 (the 4 lines' values at one
// k side by side), and every lane then adds, for each bucket it owns, the
// window entries hashed into that bucket: one 16-byte LDS read and four FMAs
// per entry.  Each input element is read from HBM once.  No atomics: every
// bucket of every line is summed by one lane, in ascending k.
//
// Which entries a lane adds comes from the prepared sketch, built once per
// (seed or tables, b, N, e, n): for every block i, window w and group q of 64
// consecutive buckets, a lane-interleaved list ("chunks" of 8 entries per
// lane, 1 KiB per chunk) padded to the longest bucket of the group.  An entry
// is 16 bits: the LDS slot of k's window offset (bits 0..14, a fixed
// permutation of the offset, see win_slot) and the sign (bit 15); the
// padding entry points at a zero row.
#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "fp8.h"

namespace osk {
namespace {

constexpr int kWin = kSketchWindow;    // sketched indices per window (8192)
constexpr int kLines = 4;              // lines per workgroup
constexpr int kThreads = 512;          // 8 waves
constexpr int kWaves = kThreads / 64;
constexpr int kPerThread = kWin / kThreads;   // window positions staged per thread (16)
constexpr uint16_t kPad = (uint16_t)kWin;     // entry of the zero row, positive
constexpr int kAhead = 3;              // list chunks of a slot fetched ahead
constexpr int kDist = 1;               // slots ahead whose lists are fetched

// LDS slot of window position p (p < kWin).  Thread t stages the quads of
// positions 2048u + 4t + j (j < 4); they go to slots 2048u + 512j + t, so the
// lanes of one staging write touch consecutive slots.  List entries hold the
// slot of their position.
__device__ __forceinline__ int win_slot(int p) {
    return (p & ~2047) | ((p & 3) << 9) | ((p >> 2) & 511);
}

// f(integral_constant<int, I>) for I = B .. E - 1, unrolled by the compiler
// whatever the size of f's body.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Spread consecutive task ids over the 8 XCDs in contiguous runs: task T is
// run by the workgroup with linear id L where T = (L % 8) * (tasks / 8) + L / 8,
// so neighbouring tasks share an XCD and its L2.
__device__ __forceinline__ int64_t xcd_task(int64_t L, int64_t tasks) {
    if (tasks % 8 != 0) return L;
    return (L % 8) * (tasks / 8) + L / 8;
}

__device__ __forceinline__ uint64_t lanes_below() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ float wave_maxf(float x) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) x = fmaxf(x, __shfl_xor(x, d));
    return x;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) x = max(x, (uint32_t)__shfl_xor((int)x, d));
    return x;
}

// ---------------------------------------------------------------------------
// Prepared lists.  One wave per (window w, block i).
//   hdr[(i*nwin + w)*qn + q] = chunk base (bits 0..15) | chunk count (16..31)
//     of group q (buckets 64q .. 64q+63) within the (i, w) region;
//   ell region (i, w) = RC chunks of 64 lanes x 8 entries; lane L of group q
//     holds the entries of bucket 64q + L at positions 0, 1, ... (entry t in
//     chunk base + t/8, slot t%8), ascending k, then padding.
// The per-group chunk counts sum to at most ceil(kw/8) + qn = RC, because the
// longest bucket of a group holds at most the group's entries.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ell_build_region(const uint32_t* __restrict__ table, int64_t n,
                                                 int64_t nt, int32_t bp, int32_t qn,
                                                 int32_t nwin, int64_t RC,
                                                 uint32_t* __restrict__ hdr,
                                                 uint16_t* __restrict__ ell, int w, int64_t i,
                                                 uint32_t* sm, const int32_t* __restrict__ inv) {
    uint32_t* cnt = sm;            // [bp] counts, then cursors
    uint32_t* qbase = sm + bp;     // [qn] chunk base of each group
    uint32_t* qlen = qbase + qn;   // [qn] chunk count of each group
    const int lane = threadIdx.x;
    const int64_t k0 = (int64_t)w * kWin;
    const int kw = (int)min((int64_t)kWin, n - k0);
    const uint32_t* row = table + i * nt + k0;
    uint32_t* H = hdr + (i * nwin + w) * qn;
    uint16_t* region = ell + (i * nwin + w) * RC * 512;
    // list position of a bucket (the bucket itself unless grouped), the
    // block's map copied to LDS after the counts and group fields
    uint32_t* pos = qlen + qn;
    uint32_t* tab = pos + bp;       // [kWin] the window's table entries
    auto at = [&](uint32_t e) -> uint32_t {
        const uint32_t h = e & 0x7FFFFFFFu;
        return inv ? pos[h] : h;
    };

    for (int c = lane; c < bp; c += 64) {
        cnt[c] = 0;
        if (inv) pos[c] = (uint32_t)inv[i * bp + c];
    }
    for (int t0 = 0; t0 < kw; t0 += 64 * 16) {
        uint32_t e[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) e[u] = row[min(t0 + 64 * u + lane, kw - 1)];
#pragma unroll
        for (int u = 0; u < 16; ++u) tab[t0 + 64 * u + lane] = e[u];
    }
    __syncthreads();
    for (int t = lane; t < kw; t += 64) atomicAdd(&cnt[at(tab[t])], 1u);
    __syncthreads();

    uint32_t base = 0;
    for (int q = 0; q < qn; ++q) {
        const int c = 64 * q + lane;
        const uint32_t x = c < bp ? cnt[c] : 0u;
        const uint32_t nch = (wave_max(x) + 7) / 8;
        if (lane == 0) {
            H[q] = base | (nch << 16);
            qbase[q] = base;
            qlen[q] = nch;
        }
        base += nch;
    }
    __syncthreads();
    for (int c = lane; c < bp; c += 64) cnt[c] = 0;
    __syncthreads();

    // Stable scatter: chunks of 64 consecutive k; lanes holding the same
    // bucket ("peers") are found bit by bit with ballots and ranked by lane.
    int nbits = 1;
    while ((1 << nbits) < bp) ++nbits;
    const uint64_t below = lanes_below();
    for (int t0 = 0; t0 < kw; t0 += 64) {
        const int t = t0 + lane;
        const bool valid = t < kw;
        const uint32_t e = valid ? tab[t] : 0u;
        const uint32_t h = valid ? at(e) : 0u;
        uint64_t peers = __ballot(valid);
        for (int bit = 0; bit < nbits; ++bit) {
            const bool set = (h >> bit) & 1u;
            const uint64_t B = __ballot(valid && set);
            peers &= set ? B : ~B;
        }
        uint32_t pos = 0;
        if (valid) {
            pos = cnt[h] + (uint32_t)__popcll(peers & below);
            const uint32_t chunk = qbase[h >> 6] + pos / 8;
            region[(int64_t)chunk * 512 + (h & 63) * 8 + (pos & 7)] =
                (uint16_t)(win_slot(t) | ((e >> 31) << 15));
        }
        __builtin_amdgcn_wave_barrier();
        // the highest peer advances the bucket's cursor (one writer per bucket)
        if (valid && (peers >> lane) == 1ull) cnt[h] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // padding up to each group's chunk count
    for (int q = 0; q < qn; ++q) {
        const int c = 64 * q + lane;
        const uint32_t have = c < bp ? cnt[c] : 0u;
        const uint32_t len = qlen[q] * 8;
        const uint32_t qb = qbase[q];
        for (uint32_t p = have; p < len; ++p)
            region[(int64_t)(qb + p / 8) * 512 + lane * 8 + (p & 7)] = kPad;
    }
}

// The same region built by kBW waves (bp <= kBWMaxBp): wave v counts
// and scatters its own contiguous part of the window; its cursors start at
// the entries of the earlier parts (an exclusive scan over the waves' counts
// per bucket), so every bucket's list stays in ascending k.  LDS: per-wave
// cursors [kBW][bp], totals [bp], group bases and lengths [qn] each.  The
// single-sketch build takes 16 waves per region for bp <= 1024 and 8 up to
// 2048 (full-size prepare 0.026 ms, against 0.030 with 8 and 0.041 with 4);
// the batch build, which strides over many regions per workgroup, keeps 4
// (8 were 20 % slower there).
constexpr int kBWSingle = 8;
constexpr int kBWWide = 16;            // single-sketch regions with bp <= kBWWideMaxBp
constexpr int kBWWideMaxBp = 1024;
constexpr int kBWBatch = 4;
constexpr int kBWMaxBp = 2048;

template <int kBW>
__device__ __forceinline__ void ell_build_region_waves(const uint32_t* __restrict__ table, int64_t n,
                                                  int64_t nt, int32_t bp, int32_t qn,
                                                  int32_t nwin, int64_t RC,
                                                  uint32_t* __restrict__ hdr,
                                                  uint16_t* __restrict__ ell, int w, int64_t i,
                                                  uint32_t* sm, const int32_t* __restrict__ inv) {
    uint32_t* cur = sm;                 // [kBW][bp] counts, then cursors
    uint32_t* tot = sm + kBW * bp;      // [bp] entries per bucket
    uint32_t* qbase = tot + bp;         // [qn] chunk base of each group
    uint32_t* qlen = qbase + qn;        // [qn] chunk count of each group
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int64_t k0 = (int64_t)w * kWin;
    const int kw = (int)min((int64_t)kWin, n - k0);
    const uint32_t* row = table + i * nt + k0;
    uint32_t* H = hdr + (i * nwin + w) * qn;
    uint16_t* region = ell + (i * nwin + w) * RC * 512;
    // this wave's part of the window: [t_beg, t_end)
    const int part = ((kw + kBW - 1) / kBW + 63) / 64 * 64;
    const int t_beg = min(kw, wv * part);
    const int t_end = min(kw, t_beg + part);
    uint32_t* mine = cur + wv * bp;
    uint32_t* pos = qlen + qn;          // [bp] the block's bucket -> position map
    uint32_t* tab = pos + bp;           // [kWin] the window's table entries
    auto at = [&](uint32_t e) -> uint32_t {
        const uint32_t h = e & 0x7FFFFFFFu;
        return inv ? pos[h] : h;
    };

    for (int c = tid; c < kBW * bp; c += 64 * kBW) cur[c] = 0;
    if (inv)
        for (int c = tid; c < bp; c += 64 * kBW) pos[c] = (uint32_t)inv[i * bp + c];
    {
        // the window's entries to LDS, every load issued before the first store
        constexpr int kU = kWin / (64 * kBW);
        uint32_t e[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) e[u] = row[min(u * 64 * kBW + tid, kw - 1)];
#pragma unroll
        for (int u = 0; u < kU; ++u) tab[u * 64 * kBW + tid] = e[u];
    }
    __syncthreads();
    for (int t = t_beg + lane; t < t_end; t += 64) atomicAdd(&mine[at(tab[t])], 1u);
    __syncthreads();
    for (int c = tid; c < bp; c += 64 * kBW) {
        uint32_t run = 0;
#pragma unroll
        for (int v = 0; v < kBW; ++v) {
            const uint32_t x = cur[v * bp + c];
            cur[v * bp + c] = run;
            run += x;
        }
        tot[c] = run;
    }
    __syncthreads();

    if (wv == 0) {
        uint32_t base = 0;
        for (int q = 0; q < qn; ++q) {
            const int c = 64 * q + lane;
            const uint32_t x = c < bp ? tot[c] : 0u;
            const uint32_t nch = (wave_max(x) + 7) / 8;
            if (lane == 0) {
                H[q] = base | (nch << 16);
                qbase[q] = base;
                qlen[q] = nch;
            }
            base += nch;
        }
    }
    __syncthreads();

    // stable scatter of this wave's part, as in ell_build_region
    int nbits = 1;
    while ((1 << nbits) < bp) ++nbits;
    const uint64_t below = lanes_below();
    for (int t0 = t_beg; t0 < t_end; t0 += 64) {
        const int t = t0 + lane;
        const bool valid = t < t_end;
        const uint32_t e = valid ? tab[t] : 0u;
        const uint32_t h = valid ? at(e) : 0u;
        uint64_t peers = __ballot(valid);
        for (int bit = 0; bit < nbits; ++bit) {
            const bool set = (h >> bit) & 1u;
            const uint64_t B = __ballot(valid && set);
            peers &= set ? B : ~B;
        }
        if (valid) {
            const uint32_t pos = mine[h] + (uint32_t)__popcll(peers & below);
            const uint32_t chunk = qbase[h >> 6] + pos / 8;
            region[(int64_t)chunk * 512 + (h & 63) * 8 + (pos & 7)] =
                (uint16_t)(win_slot(t) | ((e >> 31) << 15));
        }
        __builtin_amdgcn_wave_barrier();
        if (valid && (peers >> lane) == 1ull) mine[h] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // padding up to each group's chunk count, groups spread over the waves
    for (int q = wv; q < qn; q += kBW) {
        const int c = 64 * q + lane;
        const uint32_t have = c < bp ? tot[c] : 0u;
        const uint32_t len = qlen[q] * 8;
        const uint32_t qb = qbase[q];
        for (uint32_t p = have; p < len; ++p)
            region[(int64_t)(qb + p / 8) * 512 + lane * 8 + (p & 7)] = kPad;
    }
}

template <int kW>
__global__ __launch_bounds__(64 * kW) void ell_buildw_kernel(const uint32_t* __restrict__ table,
                                                             int64_t n, int64_t nt, int32_t bp,
                                                             int32_t qn, int32_t nwin, int64_t RC,
                                                             uint32_t* __restrict__ hdr,
                                                             uint16_t* __restrict__ ell,
                                                             const int32_t* __restrict__ inv) {
    extern __shared__ uint32_t sm[];
    ell_build_region_waves<kW>(table, n, nt, bp, qn, nwin, RC, hdr, ell, (int)blockIdx.x,
                               (int64_t)blockIdx.y, sm, inv);
}

__global__ __launch_bounds__(64) void ell_build_kernel(const uint32_t* __restrict__ table,
                                                       int64_t n, int64_t nt, int32_t bp,
                                                       int32_t qn, int32_t nwin, int64_t RC,
                                                       uint32_t* __restrict__ hdr,
                                                       uint16_t* __restrict__ ell,
                                                       const int32_t* __restrict__ inv) {
    extern __shared__ uint32_t sm[];
    ell_build_region(table, n, nt, bp, qn, nwin, RC, hdr, ell, (int)blockIdx.x,
                     (int64_t)blockIdx.y, sm, inv);
}

__global__ __launch_bounds__(64 * kBWBatch) void ell_build_batchw_kernel(
    const PrepDesc* __restrict__ descs, int32_t count, int64_t tasks) {
    extern __shared__ uint32_t sm[];
    for (int64_t t = blockIdx.x; t < tasks; t += gridDim.x) {
        const int32_t p = find_task(descs, count, t, [](const PrepDesc& d) {
            return d.ell_task0;
        });
        const PrepDesc& d = descs[p];
        const int64_t local = t - d.ell_task0;
        ell_build_region_waves<kBWBatch>(d.table, d.n, d.nt, d.bp, d.qn, d.nwin, d.RC, d.hdr,
                                         d.ell, (int)(local % d.nwin), local / d.nwin, sm,
                                         d.inv);
        __syncthreads();
    }
}

// The same for many prepared sketches in one launch: task t (one wave) is
// region (block i, window w) of the descriptor whose ell_task0 range holds
// t; workgroups stride over the tasks.
__global__ __launch_bounds__(64) void ell_build_batch_kernel(const PrepDesc* __restrict__ descs,
                                                             int32_t count, int64_t tasks) {
    extern __shared__ uint32_t sm[];
    for (int64_t t = blockIdx.x; t < tasks; t += gridDim.x) {
        const int32_t p = find_task(descs, count, t, [](const PrepDesc& d) {
            return d.ell_task0;
        });
        const PrepDesc& d = descs[p];
        const int64_t local = t - d.ell_task0;
        ell_build_region(d.table, d.n, d.nt, d.bp, d.qn, d.nwin, d.RC, d.hdr, d.ell,
                         (int)(local % d.nwin), local / d.nwin, sm, d.inv);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Grouping the buckets of each block (one workgroup per block).  The sketch
// kernel's 64 lanes walk the lists of a group of 64 buckets in lockstep, so
// a group costs its longest list in every window.  Any fixed order of the
// buckets within a block serves the product (A's and B's sketches use the
// same order, and C sums over the buckets), so buckets of similar list
// lengths are put in one group: a recursive median split over the groups
// (a k-d partition), level d sorting each node's buckets by their count in
// the windows w with w % D == d (D levels for G = ceil(b / 64) groups), ties
// by their current position, and splitting the node in two halves of whole
// groups.  inv[i * bp + c] = the position of bucket c (c < b) in block i's
// sketch; positions b .. bp - 1 stay empty.
// ---------------------------------------------------------------------------
constexpr int kGroupThreads = 1024;
constexpr int kSortMax = 8192;        // >= OS_MAX_B, a power of two

__global__ __launch_bounds__(kGroupThreads) void group_kernel(const uint32_t* __restrict__ table,
                                                              int64_t n, int64_t nt, int32_t b,
                                                              int32_t bp, int32_t nwin,
                                                              int32_t* __restrict__ inv) {
    __shared__ uint64_t key[kSortMax];
    __shared__ uint32_t feat[kSortMax];
    __shared__ int32_t bucket_at[kSortMax];
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    const uint32_t* row = table + i * nt;
    const int G = (b + 63) / 64;
    int D = 0;
    while ((1 << D) < G) ++D;
    int N = 1;
    while (N < b) N <<= 1;
    for (int p = tid; p < b; p += kGroupThreads) bucket_at[p] = p;
    __syncthreads();
    for (int d = 0; d < D; ++d) {
        for (int c = tid; c < b; c += kGroupThreads) feat[c] = 0;
        __syncthreads();
        for (int64_t w = d; w < nwin; w += D) {
            const int64_t k0 = w * (int64_t)kWin;
            const int64_t k1 = min(n, k0 + kWin);
            // the window's entries: all loads issued before the first atomic
            constexpr int kU = kWin / kGroupThreads;
            uint32_t e[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t k = k0 + u * kGroupThreads + tid;
                e[u] = row[min(k, k1 - 1)];
            }
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (k0 + u * kGroupThreads + tid < k1) atomicAdd(&feat[e[u] & 0x7FFFFFFFu], 1u);
        }
        __syncthreads();
        // key = (first group of the position's level-d node, count, position)
        for (int p = tid; p < N; p += kGroupThreads) {
            uint64_t kk = ~0ull;
            if (p < b) {
                int glo = 0, ghi = G;
                for (int lv = 0; lv < d; ++lv) {
                    const int gm = (glo + ghi) >> 1;
                    if ((p >> 6) < gm)
                        ghi = gm;
                    else
                        glo = gm;
                }
                kk = ((uint64_t)glo << 50) | ((uint64_t)feat[bucket_at[p]] << 14) | (uint64_t)p;
            }
            key[p] = kk;
        }
        __syncthreads();
        // bitonic sort of key[0, N), ascending.  Thread t exchanges the pair
        // (lo, lo + stride), lo = 2t - t % stride.  For strides up to 64 the
        // pairs of wave w lie in entries [128w, 128w + 128), so two such
        // stages in a row need only the wave's own LDS ordering (a wave's
        // LDS instructions execute in program order); a stage that crosses
        // waves (stride >= 128, or several pairs per thread) is fenced by
        // workgroup barriers on both sides.
        bool prev_cross = true;          // (the keys were just written by all waves)
        for (int size = 2; size <= N; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                const bool cross = stride >= 128 || N / 2 > kGroupThreads;
                if (cross || prev_cross) {
                    __syncthreads();
                } else {
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
                prev_cross = cross;
                for (int t = tid; t < N / 2; t += kGroupThreads) {
                    const int lo = 2 * t - (t & (stride - 1));
                    const int hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const uint64_t x = key[lo], y = key[hi];
                    if ((x > y) == up) {
                        key[lo] = y;
                        key[hi] = x;
                    }
                }
            }
        }
        __syncthreads();
        // the bucket now at position p was at position key[p] & 0x3FFF
        for (int p = tid; p < b; p += kGroupThreads) feat[p] = (uint32_t)bucket_at[key[p] & 0x3FFF];
        __syncthreads();
        for (int p = tid; p < b; p += kGroupThreads) bucket_at[p] = (int32_t)feat[p];
        __syncthreads();
    }
    for (int p = tid; p < b; p += kGroupThreads) inv[i * bp + bucket_at[p]] = p;
}

// bucket order of block i: order[i * bp + p] = the bucket at position p
// (p < b), p itself for the empty positions p >= b.
__global__ __launch_bounds__(256) void bucket_order_kernel(const int32_t* __restrict__ inv,
                                                           int32_t b, int32_t bp,
                                                           int32_t* __restrict__ order) {
    const int64_t i = blockIdx.y;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < bp; c += gridDim.x * blockDim.x) {
        if (c < b)
            order[i * bp + inv[i * bp + c]] = c;
        else
            order[i * bp + c] = c;
    }
}

__global__ __launch_bounds__(256) void identity_inv_kernel(int32_t bp, int32_t* __restrict__ inv) {
    const int64_t i = blockIdx.y;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < bp; c += gridDim.x * blockDim.x)
        inv[i * bp + c] = c;
}

// ---------------------------------------------------------------------------
// The sketch kernel.  Thread t stages window positions 2048u + 4t + j
// (u, j < 4) into LDS slots win_slot(k) = 2048u + 512j + t; list entries
// hold those slots.
//   kRowLines = true : lines are rows of X (lines x n, ld ldx).  With vec
//                      (X 16-byte aligned, ldx % 4 == 0, and the window whole
//                      or n a multiple of 4) a line's 4 consecutive positions
//                      come with one 16-byte load (1 KiB per wave,
//                      coalesced): r[4*line + u] holds positions 4t + 2048u
//                      .. +3 of that line.  Otherwise every value is loaded
//                      on its own into the same layout.
//   kRowLines = false: lines are columns of X (n x lines, ld ldx); r[4u + j]
//                      holds X[k][line0 .. line0+3] for position k = 2048u +
//                      4t + j, one 16-byte load when vec (X 16-byte aligned,
//                      ldx % 4 == 0), else four.
// kWeighted (row lines): every value at sketched index k is multiplied by
// sqrt(wd[k]) (a diagonal weight, as in A D^{1/2} S for a Hessian A D A^T);
// w[u] holds the weights of positions 4t + 2048u .. +3.  The weight is
// applied when the window is written to LDS, not when it is loaded, so the
// loads of the next window stay in flight while the current one is summed.
// ---------------------------------------------------------------------------
// Input values are held in registers as loaded (4 consecutive values of a
// line: a float4 for FP32, their 4 bit patterns in a uint2 for BF16) and
// converted to FP32 (exactly) when the window is written to LDS.
// A window's FP32 values and weights are read once: non-temporal loads keep
// them from displacing the bucket lists (which every line group reads) in
// the caches (the FP32 sketch of A 2-5 % faster).
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_stream(const float* __restrict__ p) {
    const f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    return make_float4(t[0], t[1], t[2], t[3]);
}

template <typename TI>
struct RawQuad;
template <>
struct RawQuad<float> {
    using type = float4;
    static __device__ __forceinline__ type load(const float* __restrict__ p) {
        return *reinterpret_cast<const float4*>(p);
    }
    static __device__ __forceinline__ type gather(const float* __restrict__ p,
                                                  const int64_t (&k)[4]) {
        return make_float4(p[k[0]], p[k[1]], p[k[2]], p[k[3]]);
    }
    static __device__ __forceinline__ float value(const type& v, int j) {
        return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
    }
};
template <>
struct RawQuad<__bf16> {
    using type = uint2;
    static __device__ __forceinline__ uint32_t bits(const __bf16* __restrict__ p) {
        return __builtin_bit_cast(uint16_t, *p);
    }
    static __device__ __forceinline__ type load(const __bf16* __restrict__ p) {
        return *reinterpret_cast<const uint2*>(p);
    }
    static __device__ __forceinline__ type gather(const __bf16* __restrict__ p,
                                                  const int64_t (&k)[4]) {
        return make_uint2(bits(p + k[0]) | bits(p + k[1]) << 16,
                          bits(p + k[2]) | bits(p + k[3]) << 16);
    }
    static __device__ __forceinline__ float value(const type& v, int j) {
        const uint32_t w = j < 2 ? v.x : v.y;
        return __uint_as_float((j & 1) ? (w & 0xFFFF0000u) : (w << 16));
    }
};

// Loads pieces p0 .. p1 - 1 of a window (piece 4u + q: r[4q + u] of row
// lines with w[u] at q = 0, r[4u + q] of column lines); all 16 pieces make
// the window.  p0 and p1 are constants where the caller is unrolled.
template <bool kRowLines, bool kWeighted, typename TI, bool kWhole = false>
__device__ __forceinline__ void load_window(typename RawQuad<TI>::type (&r)[kPerThread],
                                            float4 (&w)[4], const TI* __restrict__ X,
                                            int64_t lines, int64_t ldx, int64_t line0, int64_t k0,
                                            int kw, bool vec, const float* __restrict__ wd,
                                            int p0 = 0, int p1 = kPerThread) {
    using R = RawQuad<TI>;
    static_assert(kRowLines || sizeof(TI) == 4, "column lines are read as FP32 only");
    // Every load is unconditional (a branch around a load makes each use wait
    // for all loads in flight): positions past the window's end are clamped to
    // its last index (no entry refers to them) and lines past the matrix to
    // its last line (their sums are never stored).
    const int tid = threadIdx.x;
    const int64_t l1 = min(line0 + 1, lines - 1) - line0;
    const int64_t l2 = min(line0 + 2, lines - 1) - line0;
    const int64_t l3 = min(line0 + 3, lines - 1) - line0;
    if constexpr (kRowLines) {
        const int64_t dl[4] = {0, l1, l2, l3};
        if (vec) {
            // kw is a multiple of 4 here: the last whole quad starts at kw - 4.
            // Uniform line bases plus a 32-bit lane offset (scalar-base
            // addressing: a piece issued late keeps one offset register live,
            // not a 64-bit address).
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t off = (uint32_t)min(4 * tid + 2048 * u, kw - 4);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (4 * u + q < p0 || 4 * u + q >= p1) continue;
                    const TI* base = X + (line0 + dl[q]) * ldx + k0;
                    // (the FP32 load written here, not through R::load: through the
                    // helper the FP32 kernels took 20 more registers and spilled)
                    if constexpr (sizeof(TI) == 4)
                        r[4 * q + u] = load_stream(base + off);
                    else
                        r[4 * q + u] = R::load(base + off);
                    if constexpr (kWeighted)
                        if (q == 0) w[u] = load_stream(wd + k0 + off);
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                int64_t kk[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) kk[j] = k0 + min(4 * tid + 2048 * u + j, kw - 1);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (4 * u + q < p0 || 4 * u + q >= p1) continue;
                    r[4 * q + u] = R::gather(X + (line0 + dl[q]) * ldx, kk);
                    if constexpr (kWeighted)
                        if (q == 0) w[u] = make_float4(wd[kk[0]], wd[kk[1]], wd[kk[2]], wd[kk[3]]);
                }
            }
        }
    } else {
        // r[4u + j] = the 4 lines at position 2048u + 4t + j
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (4 * u + j < p0 || 4 * u + j >= p1) continue;
                const int64_t kk = k0 + min(4 * tid + 2048 * u + j, kw - 1);
                const TI* p = X + kk * ldx + line0;
                if constexpr (kWhole)    // vec and every line group whole
                    r[4 * u + j] = *reinterpret_cast<const float4*>(p);
                else if (vec && l3 == 3)      // uniform
                    r[4 * u + j] = *reinterpret_cast<const float4*>(p);
                else
                    r[4 * u + j] = make_float4(p[0], p[l1], p[l2], p[l3]);
            }
        }
    }
}

__device__ __forceinline__ float comp4(const float4& v, int j) {
    return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
}

// Writes a loaded window into LDS: win[win_slot(k)] = the 4 lines' values at
// window position k (weighted when kWeighted).
template <bool kRowLines, bool kWeighted, typename TI>
__device__ __forceinline__ void stage_window(float4* __restrict__ win,
                                             const typename RawQuad<TI>::type (&r)[kPerThread],
                                             const float4 (&w)[4]) {
    using R = RawQuad<TI>;
    const int tid = threadIdx.x;
    if constexpr (kRowLines) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float4 v = make_float4(R::value(r[u], j), R::value(r[4 + u], j),
                                       R::value(r[8 + u], j), R::value(r[12 + u], j));
                if constexpr (kWeighted) {
                    const float sw = sqrtf(comp4(w[u], j));
                    v.x *= sw;
                    v.y *= sw;
                    v.z *= sw;
                    v.w *= sw;
                }
                win[2048 * u + 512 * j + tid] = v;      // slot of position 2048u + 4t + j
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                win[2048 * u + 512 * j + tid] =
                    make_float4(R::value(r[4 * u + j], 0), R::value(r[4 * u + j], 1),
                                R::value(r[4 * u + j], 2), R::value(r[4 * u + j], 3));
    }
}

// Adds the 8 entries of one chunk (16-bit entries, two per word; sign bit 15
// selects the sign of the FP32 +-1.0 factor).  All eight LDS reads are issued
// before the first FMA so their latencies overlap.
__device__ __forceinline__ void add_chunk(float4& acc, const float4* __restrict__ win, uint4 e) {
    const uint32_t w[4] = {e.x, e.y, e.z, e.w};
    float4 v[8];
    float s[8];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        v[2 * u] = win[w[u] & 0x7FFFu];
        v[2 * u + 1] = win[(w[u] >> 16) & 0x7FFFu];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        s[2 * u] = __uint_as_float(0x3F800000u | ((w[u] << 16) & 0x80000000u));
        s[2 * u + 1] = __uint_as_float(0x3F800000u | (w[u] & 0x80000000u));
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        acc.x = fmaf(s[u], v[u].x, acc.x);
        acc.y = fmaf(s[u], v[u].y, acc.y);
        acc.z = fmaf(s[u], v[u].z, acc.z);
        acc.w = fmaf(s[u], v[u].w, acc.w);
    }
}

// One workgroup of 8 waves fills a CU's LDS, so each SIMD runs 2 waves: the
// compiler may use up to 256 VGPRs per lane.
template <int kSlots, bool kRowLines, bool kWeighted, typename TI, bool kFp8Out, bool kSpread>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 2)))
void sketch_kernel(
    const TI* __restrict__ X, int64_t lines, int64_t n, int64_t ldx, int vec, int32_t bp,
    int32_t qn, int32_t nwin, int32_t nst, BlockList bl, int64_t RC,
    const uint32_t* __restrict__ hdr, const uint4* __restrict__ ell, void* __restrict__ out,
    int64_t ldo, int32_t npass, const float* __restrict__ wd, int32_t obp, int32_t omode,
    int64_t ozlo) {
    __shared__ float4 win[kWin + 1];    // row kWin stays zero
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t groups = (lines + kLines - 1) / kLines;
    const int64_t tasks = groups * npass;
    const int gslots = nst * qn;         // groups of 64 buckets over the stored blocks
    if (tid == 0) win[kWin] = make_float4(0.f, 0.f, 0.f, 0.f);

    // vec for a row-lines window: whole windows always, the last one when n % 4 == 0
    auto vec_at = [&](int64_t k0) {
        return kRowLines ? (vec != 0 && (k0 + kWin <= n || (n & 3) == 0)) : vec != 0;
    };
    // Persistent: workgroup g takes tasks g, g + grid, ... (task = a group
    // of 4 lines and a pass); the first window of its next task is fetched
    // while the last window of the current one is summed, so only the first
    // task of a workgroup waits for its first window.
    //
    // Slot bookkeeping stays out of the scalar path (a scalar load in the
    // slot loop drains every LDS read in flight): lane s of each wave holds,
    // for its slot s, the header index of the slot's bucket group in window
    // 0 (hb, -1 for an unused slot), the region's chunk base in window 0
    // (eb), the group's first output column (col) and how many of its 64
    // buckets exist (lim, 0 for an unused slot).  A window's headers come in
    // with one vector load, issued before the window's values are fetched.
    auto line_of = [&](int64_t it) { return xcd_task(it, tasks) / npass * kLines; };
    struct Meta {
        int32_t hb, eb, col, lim;
    };
    auto meta_of = [&](int64_t it) -> Meta {
        const int ps = (int)(xcd_task(it, tasks) % npass);
        const int G = (ps * kSlots + lane) * kWaves + wave;
        Meta m{-1, 0, 0, 0};
        if (lane < kSlots && G < gslots) {
            const int j = G / qn;
            const int q = G - j * qn;
            const int32_t i = bl.idx[j];
            m.hb = (i * nwin) * qn + q;
            m.eb = (int32_t)((int64_t)i * nwin * RC);
            m.col = j * obp + q * 64;
            m.lim = min(64, obp - q * 64);
        }
        return m;
    };
    auto headers = [&](int32_t hb, int w) -> uint32_t {
        const uint32_t h = hdr[max(hb, 0) + w * qn];     // unconditional: index valid
        return hb >= 0 ? h : 0u;
    };
    typename RawQuad<TI>::type pre[kPerThread];
    float4 wpre[4];
    uint32_t hnext = 0;
    if ((int64_t)blockIdx.x < tasks) {
        hnext = headers(meta_of(blockIdx.x).hb, 0);
        load_window<kRowLines, kWeighted, TI>(pre, wpre, X, lines, ldx, line_of(blockIdx.x), 0,
                                              (int)min((int64_t)kWin, n), vec_at(0), wd);
    }
    for (int64_t it = blockIdx.x; it < tasks; it += gridDim.x) {
    const int64_t task = xcd_task(it, tasks);
    const int64_t line0 = task / npass * kLines;
    const Meta meta = meta_of(it);      // (its loads complete with the window's, before staging)

    float4 acc[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) acc[s] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int w = 0; w < nwin; ++w) {
        __syncthreads();                 // the previous window is no longer read
        stage_window<kRowLines, kWeighted, TI>(win, pre, wpre);
        __syncthreads();
        const uint32_t hv = hnext;       // this window's headers (lane s: slot s)
        // The list chunks of slot s + kDist (up to kAhead of them) are fetched
        // while slot s is summed.  Fetches are unconditional: chunk indices
        // past a slot's count repeat its last chunk, and an unused slot
        // (header 0) reads chunk 0 of block 0's region (never summed).
        const int64_t wrc = (int64_t)w * RC;
        auto slot_list = [&](int s, uint32_t& nch) -> const uint4* {
            const uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)hv, s);
            const int64_t eb = __builtin_amdgcn_readlane(meta.eb, s);
            nch = h >> 16;
            return ell + (eb + wrc + (h & 0xFFFFu)) * 64 + lane;
        };
        auto fetch = [&](uint4 (&d)[kAhead], const uint4* p, uint32_t nch) {
            const uint32_t last = nch > 0 ? nch - 1 : 0;
#pragma unroll
            for (int c = 0; c < kAhead; ++c) d[c] = p[(int64_t)min((uint32_t)c, last) * 64];
        };
        // The next window (this task's, else the first of the next task) is
        // loaded in kPerThread pieces spread over the slots, each issued
        // after the list fetch of its slot: a wave's loads complete in
        // order, so waiting for slot s's list waits only for pieces issued
        // kDist or more slots earlier, not for the whole window.  When no
        // window follows, the pieces read one quad of this window again
        // (every lane the same address; loads stay unconditional).
        int64_t l1 = line0, k1 = (int64_t)(w + 1) * kWin;
        int32_t hb1 = meta.hb;
        int kw1;
        if (w + 1 < nwin) {
            kw1 = (int)min((int64_t)kWin, n - k1);
        } else if (it + gridDim.x < tasks) {
            hb1 = meta_of(it + gridDim.x).hb;
            l1 = line_of(it + gridDim.x);
            k1 = 0;
            kw1 = (int)min((int64_t)kWin, n);
        } else {
            k1 = (int64_t)w * kWin;
            kw1 = (int)min((int64_t)4, n - k1);
        }
        const bool vec1 = vec_at(k1) && kw1 >= 4;
        constexpr int kRing = kDist + 1;
        uint4 lst[kRing][kAhead];
        uint32_t nls[kRing];
        const uint4* pls[kRing];
#pragma unroll
        for (int s = 0; s < kDist && s < kSlots; ++s) {
            pls[s] = slot_list(s, nls[s]);
            fetch(lst[s], pls[s], nls[s]);
        }
        hnext = headers(hb1, (int)(k1 / kWin));
        constexpr int kSpreadSlots = kSlots < kPerThread ? kSlots : kPerThread;
        constexpr int kPer = (kPerThread + kSpreadSlots - 1) / kSpreadSlots;
        // (unrolled at compile time: acc[s] and the ring stay in registers
        // however large the body)
        static_for<0, kSlots>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            if constexpr (s + kDist < kSlots) {
                constexpr int r = (s + kDist) % kRing;
                pls[r] = slot_list(s + kDist, nls[r]);
                fetch(lst[r], pls[r], nls[r]);
            }
            if constexpr (kSpread) {
                if constexpr (s < kSpreadSlots)
                    load_window<kRowLines, kWeighted, TI, true>(
                        pre, wpre, X, lines, ldx, l1, k1, kw1, true, wd, s * kPer,
                        (s + 1) * kPer < kPerThread ? (s + 1) * kPer : kPerThread);
            } else if constexpr (s == 0) {
                load_window<kRowLines, kWeighted, TI>(pre, wpre, X, lines, ldx, l1, k1, kw1, vec1,
                                                      wd);
            }
            constexpr int r = s % kRing;
#pragma unroll
            for (int c = 0; c < kAhead; ++c)
                if ((uint32_t)c < nls[r]) add_chunk(acc[s], win, lst[r][c]);
            for (uint32_t c = kAhead; c < nls[r]; ++c) add_chunk(acc[s], win, pls[r][(int64_t)c * 64]);
        });
    }

    // Output: FP32 (omode 0, blocks obp = bp apart), or the copy the block
    // product reads, blocks obp = b rounded up to 64 apart:
    //   omode 1: BF16, each sum rounded to nearest even; omode 2: also the
    //            residual bf16(x - hi), ozlo values after the high part;
    //   omode 3: FP8 E4M3 codes (bytes) with one E8M0 scale per 64 codes,
    //            i.e. per slot group and line (its max over the wave's 64
    //            lanes); the scale bytes follow the codes (ozlo bytes into
    //            the row), in code order.
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        // lanes below lim hold buckets of the block (the last group may be partial)
        if (lane < __builtin_amdgcn_readlane(meta.lim, s)) {
            const int64_t o0 = line0 * ldo + __builtin_amdgcn_readlane(meta.col, s) + lane;
            const float v[4] = {acc[s].x, acc[s].y, acc[s].z, acc[s].w};
            if (omode == 0) {
                float* o = static_cast<float*>(out) + o0;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (r == 0 || line0 + r < lines) o[r * ldo] = v[r];
            } else if (!kFp8Out) {
                __bf16* o = static_cast<__bf16*>(out) + o0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r == 0 || line0 + r < lines) {
                        const __bf16 hi = (__bf16)v[r];
                        o[r * ldo] = hi;
                        if (omode == 2) o[r * ldo + ozlo] = (__bf16)(v[r] - (float)hi);
                    }
                }
            } else if constexpr (kFp8Out) {
                // (a separate instantiation: this code would make the FP32
                // and BF16 kernels with 20 or more slots spill.)  Every lane
                // of the wave holds a bucket here (lim is 64), so a group's
                // maximum is taken over all 64 lanes; the four lines' maxima
                // run in one interleaved butterfly, so that each step's
                // cross-lane reads overlap.
                const int64_t col = __builtin_amdgcn_readlane(meta.col, s);
                uint8_t* row = static_cast<uint8_t*>(out) + line0 * ldo;
                float a[4];
                int e[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) a[r] = fabsf(v[r]);
#pragma unroll
                for (int d = 1; d < 64; d <<= 1)
#pragma unroll
                    for (int r = 0; r < 4; ++r) a[r] = fmaxf(a[r], __shfl_xor(a[r], d));
#pragma unroll
                for (int r = 0; r < 4; ++r) e[r] = e8m0_exponent(a[r]);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r == 0 || line0 + r < lines) {                // uniform
                        row[r * ldo + col + lane] = (uint8_t)e4m3_rne(ldexpf(v[r], -e[r]));
                        if (lane == 0) row[r * ldo + ozlo + col / 64] = (uint8_t)(e[r] + 127);
                    }
                }
            }
        }
    }
    }   // tasks
}

// Slot counts compiled: 1, 2, 4, 8, 12, 16, 20, 24 (4 registers per slot).
constexpr int kMaxSlots = 24;

// spread: every window is loaded with 16-byte loads -- row lines with vec
// and n a multiple of 4, column lines with vec and every group of 4 lines
// whole -- so the next window's loads can be spread over the slots
// (kSpread).
template <int S, bool R, bool W, typename TI, bool Q8>
hipError_t launch_one(dim3 grid, hipStream_t st, bool spread, const TI* X, int64_t lines,
                      int64_t n, int64_t ldx, int vec, int32_t bp, int32_t qn, int32_t nwin,
                      int32_t nst, const BlockList& bl, int64_t RC, const uint32_t* hdr,
                      const uint4* ell, void* out, int64_t ldo, int32_t npass, const float* wd,
                      int32_t obp, int32_t omode, int64_t ozlo) {
    if (spread) {
        hipLaunchKernelGGL((sketch_kernel<S, R, W, TI, Q8, true>), grid, dim3(kThreads), 0, st, X,
                           lines, n, ldx, vec, bp, qn, nwin, nst, bl, RC, hdr, ell, out, ldo,
                           npass, wd, obp, omode, ozlo);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((sketch_kernel<S, R, W, TI, Q8, false>), grid, dim3(kThreads), 0, st, X,
                       lines, n, ldx, vec, bp, qn, nwin, nst, bl, RC, hdr, ell, out, ldo, npass,
                       wd, obp, omode, ozlo);
    return hipGetLastError();
}

template <bool R, bool W, typename TI, bool Q8 = false>
hipError_t launch_slots(int slots, dim3 grid, hipStream_t st, const TI* X, int64_t lines,
                        int64_t n, int64_t ldx, int vec, int32_t bp, int32_t qn, int32_t nwin,
                        int32_t nst, const BlockList& bl, int64_t RC, const uint32_t* hdr,
                        const uint4* ell, void* out, int64_t ldo, int32_t npass,
                        const float* wd, int32_t obp, int32_t omode, int64_t ozlo) {
    const bool spread = vec && (R ? (n & 3) == 0 : (lines & 3) == 0);
#define OSK_SLOT_CASE(S)                                                                        \
    if (slots <= S)                                                                             \
        return launch_one<S, R, W, TI, Q8>(grid, st, spread, X, lines, n, ldx, vec, bp, qn, nwin, \
                                           nst, bl, RC, hdr, ell, out, ldo, npass, wd, obp, omode, \
                                           ozlo);
    OSK_SLOT_CASE(1)
    OSK_SLOT_CASE(2)
    OSK_SLOT_CASE(4)
    OSK_SLOT_CASE(8)
    OSK_SLOT_CASE(12)
    OSK_SLOT_CASE(16)
    OSK_SLOT_CASE(20)
    if constexpr (!Q8) {        // (FP8 output: at most 20 slots, see sketch_fp8_fusable)
        OSK_SLOT_CASE(24)
    }
#undef OSK_SLOT_CASE
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Transpose: Y (cols x rows, ld ldy) = X^T for X rows x cols (ld ldx): FP32
// to FP32, or BF16 to BF16 (values copied exactly; staged through LDS as
// FP32, which holds every BF16 value).  A workgroup of 512 threads moves
// a 64 x 256 tile of X through LDS (row stride 257 floats: the column reads
// are conflict-free): every row of X contributes 256 consecutive values and
// every row of Y 64, each lane moving 4 values per access.
//   kWhole = true : the wr x wc whole tiles, X aligned to 4 values with
//                   ldx % 4 == 0: vector accesses with no bounds checks and
//                   no branches (a branch between the loads and their LDS
//                   writes, or between the LDS reads and the stores, costs
//                   8-10 % here);
//   kWhole = false: every other tile (the right and bottom strips, or all
//                   tiles when X is not aligned): loads clamped into the
//                   matrix, stores guarded.
// Y is aligned to 4 of its values with ldy % 4 == 0 (checked by the launcher).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ float4 load4(const T* p);

template <>
__device__ __forceinline__ float4 load4<float>(const float* p) {
    return *reinterpret_cast<const float4*>(p);
}

template <>
__device__ __forceinline__ float4 load4<__bf16>(const __bf16* p) {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    const bf16x4 v = *reinterpret_cast<const bf16x4*>(p);
    return make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
}

constexpr int kTrRows = 64;
constexpr int kTrCols = 256;

template <typename TO>
__device__ __forceinline__ void store4(TO* p, const float4& v);

template <>
__device__ __forceinline__ void store4<float>(float* p, const float4& v) {
    *reinterpret_cast<float4*>(p) = v;
}

template <>
__device__ __forceinline__ void store4<__bf16>(__bf16* p, const float4& v) {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    const bf16x4 w = {(__bf16)v.x, (__bf16)v.y, (__bf16)v.z, (__bf16)v.w};
    *reinterpret_cast<bf16x4*>(p) = w;
}

template <typename T, bool kWhole, typename TO>
__global__ __launch_bounds__(512) void transpose_kernel(const T* __restrict__ X, int64_t rows,
                                                        int64_t cols, int64_t ldx,
                                                        TO* __restrict__ Y, int64_t ldy,
                                                        int64_t wr, int64_t wc) {
    __shared__ float t[kTrRows][kTrCols + 1];
    const int tid = threadIdx.x;
    int64_t r0, c0;
    if constexpr (kWhole) {
        const int64_t Tk = xcd_task(blockIdx.x, wr * wc);
        r0 = Tk / wc * kTrRows;
        c0 = Tk % wc * kTrCols;
    } else {
        // the right strip (tile rows < wr, tile columns >= wc), then the
        // bottom strip (tile rows >= wr, every tile column)
        const int64_t C = (cols + kTrCols - 1) / kTrCols;
        const int64_t right = wr * (C - wc);
        const int64_t k = blockIdx.x;
        if (k < right) {
            r0 = k / (C - wc) * kTrRows;
            c0 = (wc + k % (C - wc)) * kTrCols;
        } else {
            r0 = (wr + (k - right) / C) * kTrRows;
            c0 = (k - right) % C * kTrCols;
        }
    }
    // load: row sub + 8i of the tile, columns q .. q+3
    const int sub = tid >> 6;
    const int q = 4 * (tid & 63);
    float4 v[8];
    if constexpr (kWhole) {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = load4<T>(X + (r0 + sub + 8 * i) * ldx + c0 + q);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const T* p = X + min(r0 + sub + 8 * i, rows - 1) * ldx;
            v[i].x = (float)p[min(c0 + q + 0, cols - 1)];
            v[i].y = (float)p[min(c0 + q + 1, cols - 1)];
            v[i].z = (float)p[min(c0 + q + 2, cols - 1)];
            v[i].w = (float)p[min(c0 + q + 3, cols - 1)];
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = sub + 8 * i;
        t[r][q + 0] = v[i].x;
        t[r][q + 1] = v[i].y;
        t[r][q + 2] = v[i].z;
        t[r][q + 3] = v[i].w;
    }
    __syncthreads();
    // store: row cs + 32i of the tile of Y (a column of X), columns p .. p+3
    const int cs = tid >> 4;
    const int p = 4 * (tid & 15);
    float4 w[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int c = cs + 32 * i;
        w[i] = make_float4(t[p][c], t[p + 1][c], t[p + 2][c], t[p + 3][c]);
    }
    const int64_t yc = r0 + p;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t yr = c0 + cs + 32 * i;
        TO* o = Y + yr * ldy + yc;
        if constexpr (kWhole) {
            store4<TO>(o, w[i]);
        } else if (yr < cols) {
            if (yc + 3 < rows) {
                store4<TO>(o, w[i]);
            } else {
                if (yc < rows) o[0] = (TO)w[i].x;
                if (yc + 1 < rows) o[1] = (TO)w[i].y;
                if (yc + 2 < rows) o[2] = (TO)w[i].z;
            }
        }
    }
}

struct Plan {
    int32_t qn;      // groups of 64 buckets per block
    int32_t nwin;    // windows over the sketched dimension
    int64_t RC;      // chunks per (block, window) region
};

Plan plan_of(int64_t n, int32_t bp) {
    Plan p;
    p.qn = (bp + 63) / 64;
    p.nwin = (int32_t)((n + kWin - 1) / kWin);
    p.RC = (min((int64_t)kWin, n) + 7) / 8 + p.qn;
    return p;
}

struct ListView {
    uint32_t* hdr;
    uint4* ell;
};

ListView carve_lists(void* lists, int32_t nblk, int64_t n, int32_t bp) {
    const Plan p = plan_of(n, bp);
    char* base = static_cast<char*>(lists);
    ListView v;
    v.hdr = reinterpret_cast<uint32_t*>(base);
    base += round_up((int64_t)nblk * p.nwin * p.qn * 4, 256);
    v.ell = reinterpret_cast<uint4*>(base);
    return v;
}

// Passes and slots per pass for nst stored blocks.
void pass_plan(int32_t nst, int32_t qn, int32_t* npass, int32_t* slots) {
    const int64_t gs = (int64_t)nst * qn;
    const int64_t per = (int64_t)kWaves * kMaxSlots;
    const int64_t P = (gs + per - 1) / per;
    const int64_t need = (gs + P - 1) / P;               // groups per pass
    *npass = (int32_t)P;
    *slots = (int32_t)((need + kWaves - 1) / kWaves);
}

// X: FP32, or BF16 when bf16 (rows only, unweighted).
// X: FP32, or BF16 when bf16 (rows only, unweighted).  out_mode: 0 = FP32
// sketch (blocks bp apart); 1 = its BF16 rounding, 2 = BF16 and residual
// (nst blocks after), 3 = FP8 codes, then their scales (blocks
// round_up(bp, 64) apart).
hipError_t launch_sketch(bool row_lines, const void* X, bool bf16, int64_t lines, int64_t n,
                         int64_t ldx, const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                         const void* lists, void* out, int64_t ldo, hipStream_t s,
                         const float* wd = nullptr, int out_mode = 0) {
    const Plan p = plan_of(n, bp);
    const ListView v = carve_lists(const_cast<void*>(lists), nblk, n, bp);
    int32_t npass, slots;
    pass_plan(nst, p.qn, &npass, &slots);
    const int64_t groups = (lines + kLines - 1) / kLines;
    // persistent workgroups: one per CU (a window fills a CU's LDS)
    int dev = 0, cus = 0;
    int64_t nwg = groups * npass;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
        nwg = std::min<int64_t>(nwg, cus);
    const dim3 grid((unsigned)nwg);
    if (out_mode < 0 || out_mode > 3) return hipErrorInvalidValue;
    const int32_t obp = out_mode ? p.qn * 64 : bp;
    const int64_t ozlo = out_mode >= 2 ? (int64_t)nst * obp : 0;
    // vec: a quad of 4 values is one aligned load (16 bytes FP32, 8 BF16)
    const uintptr_t quad = bf16 ? 7 : 15;
    const int vec = (reinterpret_cast<uintptr_t>(X) & quad) == 0 && (ldx & 3) == 0 &&
                    (reinterpret_cast<uintptr_t>(wd) & 15) == 0;
    if (out_mode == 3) {          // FP8 copies: rows only, unweighted
        if (!row_lines || wd) return hipErrorInvalidValue;
        if (bf16)
            return launch_slots<true, false, __bf16, true>(
                slots, grid, s, static_cast<const __bf16*>(X), lines, n, ldx, vec, bp, p.qn,
                p.nwin, nst, bl, p.RC, v.hdr, v.ell, out, ldo, npass, nullptr, obp, out_mode, ozlo);
        return launch_slots<true, false, float, true>(
            slots, grid, s, static_cast<const float*>(X), lines, n, ldx, vec, bp, p.qn, p.nwin,
            nst, bl, p.RC, v.hdr, v.ell, out, ldo, npass, nullptr, obp, out_mode, ozlo);
    }
    if (bf16) {
        if (!row_lines || wd) return hipErrorInvalidValue;
        return launch_slots<true, false>(slots, grid, s, static_cast<const __bf16*>(X), lines, n,
                                         ldx, vec, bp, p.qn, p.nwin, nst, bl, p.RC, v.hdr, v.ell,
                                         out, ldo, npass, nullptr, obp, out_mode, ozlo);
    }
    const float* Xf = static_cast<const float*>(X);
    if (wd && row_lines)   // weighted sketches are only taken along rows
        return launch_slots<true, true>(slots, grid, s, Xf, lines, n, ldx, vec, bp, p.qn, p.nwin,
                                        nst, bl, p.RC, v.hdr, v.ell, out, ldo, npass, wd, obp,
                                        out_mode, ozlo);
    if (row_lines)
        return launch_slots<true, false>(slots, grid, s, Xf, lines, n, ldx, vec, bp, p.qn,
                                         p.nwin, nst, bl, p.RC, v.hdr, v.ell, out, ldo, npass,
                                         nullptr, obp, out_mode, ozlo);
    return launch_slots<false, false>(slots, grid, s, Xf, lines, n, ldx, vec, bp, p.qn, p.nwin,
                                      nst, bl, p.RC, v.hdr, v.ell, out, ldo, npass, nullptr, obp,
                                      out_mode, ozlo);
}

}  // namespace

size_t list_bytes(int32_t nblk, int64_t n, int32_t bp) {
    const Plan p = plan_of(n, bp);
    return (size_t)round_up((int64_t)nblk * p.nwin * p.qn * 4, 256) +
           (size_t)nblk * (size_t)p.nwin * (size_t)p.RC * 1024u;
}

void prep_desc_lists(PrepDesc& d, void* lists) {
    const Plan p = plan_of(d.n, d.bp);
    const ListView v = carve_lists(lists, d.nblk, d.n, d.bp);
    d.hdr = v.hdr;
    d.ell = reinterpret_cast<uint16_t*>(v.ell);
    d.qn = p.qn;
    d.nwin = p.nwin;
    d.RC = p.RC;
}

hipError_t launch_lists_batch(const PrepDesc* descs, int32_t count, int64_t tasks,
                              int32_t max_bp, hipStream_t s) {
    if (count < 1 || tasks < 1 || max_bp < 1) return hipErrorInvalidValue;
    const int32_t qn = (max_bp + 63) / 64;
    const unsigned grid = (unsigned)std::min<int64_t>(tasks, int64_t(1) << 20);
    if (max_bp <= kBWMaxBp) {
        const size_t lds = (size_t)((kBWBatch + 2) * max_bp + 2 * qn + kWin) * 4;
        hipLaunchKernelGGL(ell_build_batchw_kernel, dim3(grid), dim3(64 * kBWBatch), lds, s, descs,
                           count, tasks);
    } else {
        const size_t lds = (size_t)(2 * max_bp + 2 * qn + kWin) * 4;
        hipLaunchKernelGGL(ell_build_batch_kernel, dim3(grid), dim3(64), lds, s, descs, count,
                           tasks);
    }
    return hipGetLastError();
}

hipError_t launch_build_lists(const uint32_t* table, int64_t n, int64_t nt, int32_t nblk,
                              int32_t bp, void* lists, hipStream_t s, const int32_t* inv) {
    const Plan p = plan_of(n, bp);
    const ListView v = carve_lists(lists, nblk, n, bp);
    if (bp <= kBWWideMaxBp) {
        const size_t lds = (size_t)((kBWWide + 2) * bp + 2 * p.qn + kWin) * 4;
        hipLaunchKernelGGL(ell_buildw_kernel<kBWWide>, dim3((unsigned)p.nwin, (unsigned)nblk),
                           dim3(64 * kBWWide), lds, s, table, n, nt, bp, p.qn, p.nwin, p.RC, v.hdr,
                           reinterpret_cast<uint16_t*>(v.ell), inv);
    } else if (bp <= kBWMaxBp) {
        const size_t lds = (size_t)((kBWSingle + 2) * bp + 2 * p.qn + kWin) * 4;
        hipLaunchKernelGGL(ell_buildw_kernel<kBWSingle>, dim3((unsigned)p.nwin, (unsigned)nblk),
                           dim3(64 * kBWSingle), lds, s, table, n, nt, bp, p.qn, p.nwin, p.RC, v.hdr,
                           reinterpret_cast<uint16_t*>(v.ell), inv);
    } else {
        const size_t lds = (size_t)(2 * bp + 2 * p.qn + kWin) * 4;
        hipLaunchKernelGGL(ell_build_kernel, dim3((unsigned)p.nwin, (unsigned)nblk), dim3(64), lds,
                           s, table, n, nt, bp, p.qn, p.nwin, p.RC, v.hdr,
                           reinterpret_cast<uint16_t*>(v.ell), inv);
    }
    return hipGetLastError();
}

hipError_t launch_group_buckets(const uint32_t* table, int64_t n, int64_t nt, int32_t nblk,
                                int32_t b, int32_t bp, int32_t* inv, hipStream_t s) {
    if (b < 1 || b > kSortMax || bp < b || nblk < 1) return hipErrorInvalidValue;
    const Plan p = plan_of(n, bp);
    if (b <= 64) {      // one group: nothing to order
        hipLaunchKernelGGL(identity_inv_kernel, dim3((unsigned)((bp + 255) / 256), (unsigned)nblk),
                           dim3(256), 0, s, bp, inv);
    } else {
        hipLaunchKernelGGL(group_kernel, dim3((unsigned)nblk), dim3(kGroupThreads), 0, s, table,
                           n, nt, b, bp, p.nwin, inv);
    }
    return hipGetLastError();
}

hipError_t launch_identity_inv(int32_t nblk, int32_t bp, int32_t* inv, hipStream_t s) {
    hipLaunchKernelGGL(identity_inv_kernel, dim3((unsigned)((bp + 255) / 256), (unsigned)nblk),
                       dim3(256), 0, s, bp, inv);
    return hipGetLastError();
}

hipError_t launch_bucket_order(const int32_t* inv, int32_t nblk, int32_t b, int32_t bp,
                               int32_t* order, hipStream_t s) {
    hipLaunchKernelGGL(bucket_order_kernel, dim3((unsigned)((bp + 255) / 256), (unsigned)nblk),
                       dim3(256), 0, s, inv, b, bp, order);
    return hipGetLastError();
}

bool plan_sketch_ok(int64_t lines, int32_t nst, int32_t bp, int64_t n) {
    if (lines < 1 || nst < 1 || nst > OS_MAX_BLOCKS || bp < kBlockAlign || bp % kBlockAlign ||
        n < 1 || n > kMaxSketchedLen)
        return false;
    const Plan p = plan_of(n, bp);
    int32_t npass, slots;
    pass_plan(nst, p.qn, &npass, &slots);
    const int64_t groups = (lines + kLines - 1) / kLines;
    return groups * npass <= 0x7fffffff && slots <= kMaxSlots;
}

hipError_t launch_sketch_rows(const float* X, int64_t n, int64_t cols, int64_t ldx,
                              const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                              const void* lists, float* out, int64_t ldo, hipStream_t s) {
    if (!plan_sketch_ok(cols, nst, bp, n)) return hipErrorInvalidValue;
    return launch_sketch(false, X, false, cols, n, ldx, bl, nst, nblk, bp, lists, out, ldo, s);
}

bool sketch_rows_in_place_ok(const float* X, int64_t cols, int64_t ldx) {
    return (reinterpret_cast<uintptr_t>(X) & 15) == 0 && (ldx & 3) == 0 && (cols & 3) == 0;
}

hipError_t launch_sketch_rows_q(const float* X, int64_t n, int64_t cols, int64_t ldx,
                                const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                                const void* lists, void* out, int64_t ldo, int split,
                                hipStream_t s) {
    if (!plan_sketch_ok(cols, nst, bp, n)) return hipErrorInvalidValue;
    return launch_sketch(false, X, false, cols, n, ldx, bl, nst, nblk, bp, lists, out, ldo, s,
                         nullptr, split ? 2 : 1);
}

size_t transpose_bytes(int64_t rows, int64_t cols) {
    return (size_t)round_up(cols * round_up(rows, 4) * 4, 256);
}

template <typename T, typename TO>
hipError_t launch_transpose_t(const T* X, int64_t rows, int64_t cols, int64_t ldx, TO* Y,
                              int64_t ldy, hipStream_t s) {
    const int64_t R = (rows + kTrRows - 1) / kTrRows;
    const int64_t C = (cols + kTrCols - 1) / kTrCols;
    if (R * C > 0x7fffffff || ldy % 4 || (reinterpret_cast<uintptr_t>(Y) % (4 * sizeof(TO))))
        return hipErrorInvalidValue;
    const bool vec = (reinterpret_cast<uintptr_t>(X) % (4 * sizeof(T))) == 0 && (ldx & 3) == 0;
    const int64_t wr = vec ? rows / kTrRows : 0;     // whole tiles: wr x wc
    const int64_t wc = vec ? cols / kTrCols : 0;
    if (wr * wc > 0)
        hipLaunchKernelGGL((transpose_kernel<T, true, TO>), dim3((unsigned)(wr * wc)), dim3(512),
                           0, s, X, rows, cols, ldx, Y, ldy, wr, wc);
    if (R * C > wr * wc)
        hipLaunchKernelGGL((transpose_kernel<T, false, TO>), dim3((unsigned)(R * C - wr * wc)),
                           dim3(512), 0, s, X, rows, cols, ldx, Y, ldy, wr, wc);
    return hipGetLastError();
}

hipError_t launch_transpose(const float* X, int64_t rows, int64_t cols, int64_t ldx, float* Y,
                            int64_t ldy, hipStream_t s) {
    return launch_transpose_t(X, rows, cols, ldx, Y, ldy, s);
}

hipError_t launch_transpose_bf16_raw(const void* X, int64_t rows, int64_t cols, int64_t ldx,
                                     void* Y, int64_t ldy, hipStream_t s) {
    return launch_transpose_t(static_cast<const __bf16*>(X), rows, cols, ldx,
                              static_cast<__bf16*>(Y), ldy, s);
}

hipError_t launch_sketch_cols(const float* X, int64_t rows, int64_t n, int64_t ldx,
                              const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                              const void* lists, float* out, int64_t ldo, hipStream_t s,
                              const float* wd) {
    if (!plan_sketch_ok(rows, nst, bp, n)) return hipErrorInvalidValue;
    return launch_sketch(true, X, false, rows, n, ldx, bl, nst, nblk, bp, lists, out, ldo, s, wd);
}

hipError_t launch_sketch_cols_bf16(const void* X, int64_t rows, int64_t n, int64_t ldx,
                                   const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                                   const void* lists, float* out, int64_t ldo, hipStream_t s) {
    if (!plan_sketch_ok(rows, nst, bp, n)) return hipErrorInvalidValue;
    return launch_sketch(true, X, true, rows, n, ldx, bl, nst, nblk, bp, lists, out, ldo, s);
}

hipError_t launch_sketch_cols_q(const void* X, bool x_bf16, int64_t rows, int64_t n, int64_t ldx,
                                const BlockList& bl, int32_t nst, int32_t nblk, int32_t bp,
                                const void* lists, void* out, int64_t ldo, int split,
                                hipStream_t s) {
    if (!plan_sketch_ok(rows, nst, bp, n)) return hipErrorInvalidValue;
    return launch_sketch(true, X, x_bf16, rows, n, ldx, bl, nst, nblk, bp, lists, out, ldo, s,
                         nullptr, split ? 2 : 1);
}

bool sketch_fp8_fusable(int32_t b, int32_t nst) {
    if (round_up(b, 64) != block_stride_fp8(b)) return false;
    // the 24-slot kernel with the FP8 epilogue spills (400 bytes per lane)
    int32_t npass, slots;
    pass_plan(nst, (int32_t)(round_up(b, kBlockAlign) + 63) / 64, &npass, &slots);
    return slots <= 20;
}

hipError_t launch_sketch_cols_fp8(const void* X, bool x_bf16, int64_t rows, int64_t n,
                                  int64_t ldx, const BlockList& bl, int32_t nst, int32_t nblk,
                                  int32_t bp, const void* lists, void* out, int64_t ldo,
                                  hipStream_t s) {
    if (!plan_sketch_ok(rows, nst, bp, n) || !sketch_fp8_fusable(bp, nst))
        return hipErrorInvalidValue;
    return launch_sketch(true, X, x_bf16, rows, n, ldx, bl, nst, nblk, bp, lists, out, ldo, s,
                         nullptr, 3);
}

}  // namespace osk
