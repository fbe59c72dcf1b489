// gemm.hip -- grouped FP32 MFMA product over the kept sketch blocks.
//
// Computes C = scale * sum_{j kept} At_j * Bt_j^T, where At_j (m x bp) and
// Bt_j (l x bp) are the j-th column blocks of the line-major sketches A S
// and (S^T B)^T.
// This is the computation phase and the reduction phase of Algorithm
// "OverSketch" fused into one K loop: the paper's b x b worker products
// A_tilde(i,k) B_tilde(k,j) for the blocks that returned (Fig. (bMM)) are
// summed in registers instead of through storage, and blocks that
// straggled are skipped by walking only the kept-block list.
//
// Design (gfx950; FP32 v_mfma_f32_32x32x2_f32, BF16 v_mfma_f32_32x32x16_bf16,
// FP8 v_mfma_scale_f32_32x32x64_f8f6f4):
//   - 256 x 256 output tile per workgroup of 8 waves, two per SIMD; wave
//     (wm, wn) owns a 128 x 64 sub-tile = 4 x 2 MFMA blocks of 32 x 32 (128
//     accumulators per lane).  With two waves on a SIMD one wave's memory
//     instructions issue while the other's MFMAs keep the pipe busy.
//   - K steps of 128 bytes of every tile row (32 FP32, 64 BF16 or 128 FP8
//     values).  Both operands are K-contiguous; a step's tiles go straight
//     from global memory into LDS (buffer_load_dwordx4 with the lds flag: no
//     VGPR staging, no LDS stores), unpadded, with the 16-byte chunk c of
//     row r at chunk c ^ key(r), key(r) = (r & 7) ^ ((r >> 3) & 1), so the
//     16 rows a fragment read serves at once hit 16 different bank groups.
//     Two step buffers per operand: step t + 1 is loaded into one while
//     step t is read from the other.
//   - Lane half h of every MFMA takes the K values at byte offset 64h + 16q
//     of the step's row (q = quad), so a lane's fragment is one 16-byte LDS
//     read; A and B use the same K order, so the dot products are unchanged
//     (only their summation order differs).
//   - The kept-block list is held in VGPRs and picked with v_readlane.
//   - Workgroup -> tile mapping keeps neighbouring tiles on one XCD (shared
//     L2) and rasterises in groups of kGroupM = 8 tile rows.
#include <algorithm>

#include "internal.h"

namespace osk {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int BM = 256;
constexpr int BN = 256;
constexpr int kStepBytes = 128; // K step: 128 bytes of each tile row (32 FP32 / 64 BF16 values)
// tiles are rasterised in groups of kGroupM tile rows (an XCD's 32
// concurrent tiles then share 8 row blocks of A; 8 measured 0.5 % faster
// than 4 on the full-size product)
constexpr int kGroupM = 8;

__device__ __forceinline__ int64_t xcd_task(int64_t L, int64_t tasks) {
    if (tasks % 8 != 0) return L;
    return (L % 8) * (tasks / 8) + L / 8;
}

// Buffer resource of a matrix starting at p: no stride, no range limit
// (num_records = 2^32 - 1), the gfx9 data format word.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const void* p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, -1, 0x00020000);
}

// ---------------------------------------------------------------------------
// Tiles loaded straight from global memory into LDS (buffer_load_dwordx4
// with the lds flag: no VGPR staging and no LDS store instructions, which
// each cost the MFMA pipe about one slot when issued in the K loop).  A tile
// of BT = 32 kU rows x 128 bytes (one K step) is stored unpadded: the
// 16-byte chunk c of row r sits at chunk c ^ key(r), key(r) = (r & 7) ^
// ((r >> 3) & 1).  A 16-byte fragment read is served 16 lanes (16
// consecutive rows, 256 bytes) at a time over the 64 four-byte banks: rows
// r and r + 8 share their (r & 7) and the parity of their 128-byte row
// offset, and the (r >> 3) term sends them to different chunks, so the 16
// reads of a pass hit 16 different bank groups (with key (r & 7) alone, they
// met in pairs: measured as half the LDS cycles spent in bank conflicts).
// Any 8 consecutive rows also take 8 different chunks.  Load u of wave w
// fills LDS rows 8(kU w + u) .. +7 (1 KiB, 16 bytes per lane): lane l takes
// row r = 8(kU w + u) + l/8 and physical chunk l % 8, i.e. logical chunk
// (l % 8) ^ key(r).  Rows past the matrix end are clamped to its last row
// (they only feed outputs that are not stored).
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ int chunk_key(int r) { return (r & 7) ^ ((r >> 3) & 1); }

// (sub: LDS row r holds matrix row r - sub of the resource, for a tile
// whose rows start sub rows into the LDS array; a multiple of 16, so the
// key is that of r.)
template <int kU>
__device__ __forceinline__ void direct_offsets(uint32_t (&vo)[kU], int64_t ld_bytes, int last,
                                               int wave, int lane, int sub = 0) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int r = 8 * (kU * wave + u) + (lane >> 3);
        const int c = (lane & 7) ^ chunk_key(r);
        vo[u] = (uint32_t)((int64_t)min(r - sub, last) * ld_bytes + 16 * c);
    }
}

// (The builtin exists only for the device target; the host pass of a
// template kernel that names it would silently drop the kernel's launch
// stubs, hence the guard.)
template <int kU>
__device__ __forceinline__ void direct_issue(__amdgpu_buffer_rsrc_t rsrc, float* lds,
                                             const uint32_t (&vo)[kU], uint32_t kbyte, int wave) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
    for (int u = 0; u < kU; ++u)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rsrc, (lds_void*)(lds + (kU * wave + u) * 256), 16, vo[u], kbyte, 0, 0);
#endif
}

// Float offset in a direct tile of the fragment of quad q for tile row
// rbase + 32 i (rbase = a wave's first row + lane % 32; 32 i changes no bit
// of the key): lane half h reads logical chunk 4h + q.
__device__ __forceinline__ int direct_frag_off(int rbase, int q, int lane) {
    return rbase * 32 + 4 * ((4 * (lane >> 5) + q) ^ chunk_key(rbase));
}

__device__ __forceinline__ float comp(const float4& v, int c) {
    return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));


// Operand precisions of the block product.  A K step is 128 bytes of a tile
// row in both: 32 FP32 values or 64 BF16 values.  A fragment is 16 bytes:
// lane half h of quad q holds the K values at byte offset 64h + 16q of the
// step's row (4 FP32 values feeding four 32x32x2 MFMAs, or 8 BF16 values
// feeding one 32x32x16 MFMA); A and B use the same K order.
// A quad's MFMAs come in kParts parts; the K loop issues the next quad's
// fragment reads after kHead parts and leaves the step's last kTail parts
// until after the step's barrier (they keep the MFMA pipe busy while the
// next step's first fragments are read).  Chosen by measurement: FP32 3 and
// 1, BF16 1 and 0 (BF16 3-4 % faster than the compiler's own placement,
// which read each quad's fragments just before its MFMAs; FP32 unchanged).
struct PrecF32 {
    static constexpr int kElem = 4;
    static constexpr int kParts = 4;          // parts of a quad: the four K values kk
    static constexpr int kHead = 3;
    static constexpr int kTail = 1;
    template <int kI, int kJ, int kLo = 0, int kHi = kParts>
    __device__ static __forceinline__ void mfma_quad(v16f (&acc)[kI][kJ], const float4 (&a)[kI],
                                                     const float4 (&b)[kJ]) {
#pragma unroll
        for (int kk = kLo; kk < kHi; ++kk)
#pragma unroll
            for (int i = 0; i < kI; ++i)
#pragma unroll
                for (int j = 0; j < kJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(comp(a[i], kk), comp(b[j], kk),
                                                                     acc[i][j], 0, 0, 0);
    }
};

struct PrecBF16 {
    static constexpr int kElem = 2;
    static constexpr int kParts = 4;          // parts of a quad: the row blocks i (kI = 4)
    static constexpr int kHead = 1;
    static constexpr int kTail = 0;
    template <int kI, int kJ, int kLo = 0, int kHi = kI>
    __device__ static __forceinline__ void mfma_quad(v16f (&acc)[kI][kJ], const float4 (&a)[kI],
                                                     const float4 (&b)[kJ]) {
#pragma unroll
        for (int i = kLo; i < kHi; ++i)
#pragma unroll
            for (int j = 0; j < kJ; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    __builtin_bit_cast(bf16x8, a[i]), __builtin_bit_cast(bf16x8, b[j]), acc[i][j],
                    0, 0, 0);
    }
};

// Terms of the K loop: kept block j contributes nsub terms.  Term 0 pairs
// the A and B columns of the block; with nsub = 3 (split precision), term 1
// pairs A's block with the low part of B's block (lo_off columns further)
// and term 2 the low part of A's block with B's block.
// Per-C-block keep masks (cmask != nullptr, the paper's per-block
// stragglers): C is divided into cblk x cblk blocks, block (I, J) keeps the
// stored blocks j with cmask[(I * nbJ + J) * nstm + j] != 0 and is scaled by
// 1 / (their number); a block that keeps none is written as zero.  Tiles are
// laid on the C-block grid (ceil(cblk / 256) per block side, the last ones
// partial), so every tile lies in one block.
struct CMask {
    const uint8_t* mask;   // DEVICE [nbI][nbJ][nstm], or nullptr (one kept list)
    int64_t cblk;
    int32_t nbJ;
    int32_t nstm;
    int32_t tb;            // tiles per block side
};

// Split K loop (kSplit kernels, for products with few tiles): workgroup
// g = s * tiles + tile runs K steps s * chunk .. min(total, (s + 1) * chunk)
// - 1 of its tile and stores the unscaled partial tile at part + s * m * l
// (row-major, ld l); split_sum_kernel then adds the partials in split order.
struct SplitK {
    float* part;
    int32_t chunk;
};

// kOdd: the K step count may be odd (per-C-block masks, whose count varies
// per tile, with an odd bp / 32; split K loops): an odd last step runs
// alone after the step pairs.
// Eight waves per 256x256 tile, two per SIMD: wave (wm, wn) (wm < 2,
// wn < 4) computes rows 128 wm .. +127 and columns 64 wn .. +63 with 4x2
// MFMA blocks of 32x32 (128 accumulators).  With two waves on a SIMD, one
// wave's memory instructions issue while the other's MFMAs keep the pipe
// busy (one wave per SIMD left the pipe idle for about one MFMA slot per
// memory instruction).
constexpr int kThreadsK = 512;

template <typename P, bool kMask, bool kOdd, bool kSplit = false>
__global__ __launch_bounds__(kThreadsK) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gemm_kept_kernel(const void* __restrict__ At, int64_t ldat, const void* __restrict__ Bt,
                      int64_t ldbt, int64_t m, int64_t l, int32_t bp, BlockList kept,
                      int32_t nkept, int32_t nsub, int64_t lo_off, float scale,
                      float* __restrict__ C, int64_t ldc, int32_t tilesM, int32_t tilesN,
                      CMask cm, SplitK sk) {
    // two K-step buffers per operand, separate arrays so that the compiler
    // can tell the tile loads in flight (into one) from the fragment reads
    // (from the other)
    __shared__ __align__(1024) float As0[BM * 32];
    __shared__ __align__(1024) float As1[BM * 32];
    __shared__ __align__(1024) float Bs0[BN * 32];
    __shared__ __align__(1024) float Bs1[BN * 32];
    __shared__ int32_t klist[kMask ? OS_MAX_BLOCKS + 1 : 1];   // per-tile kept list, count last

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar M0 and selects
    const int wm = wave >> 2;
    const int wn = wave & 3;

    const int64_t ntiles = (int64_t)tilesM * tilesN;
    int32_t split = 0;
    int64_t T;
    if constexpr (kSplit) {
        split = (int32_t)(blockIdx.x / ntiles);
        T = (int64_t)blockIdx.x - (int64_t)split * ntiles;
    } else {
        T = xcd_task(blockIdx.x, ntiles);
    }
    const int64_t group = T / ((int64_t)kGroupM * tilesN);
    const int64_t first_m = group * kGroupM;
    const int64_t gsz = min((int64_t)kGroupM, (int64_t)tilesM - first_m);
    const int64_t in_group = T - group * kGroupM * tilesN;
    const int64_t tm = first_m + in_group % gsz;
    const int64_t tn = in_group / gsz;
    int64_t row0 = tm * BM;
    int64_t col0 = tn * BN;
    if constexpr (kMask) {
        // tile (tm, tn) of the C-block grid: block (I, J), tile (ti, tj) in it
        const int64_t I = tm / cm.tb, J = tn / cm.tb;
        row0 = I * cm.cblk + (tm % cm.tb) * BM;
        col0 = J * cm.cblk + (tn % cm.tb) * BN;
        m = min(m, (I + 1) * cm.cblk);          // rows and columns of this block only
        l = min(l, (J + 1) * cm.cblk);
        if (row0 >= m || col0 >= l) return;     // past a partial block's end (uniform)
        if (tid == 0) {
            const uint8_t* mk = cm.mask + (I * cm.nbJ + J) * cm.nstm;
            int32_t k = 0;
            for (int32_t j = 0; j < cm.nstm; ++j)
                if (mk[j]) klist[k++] = j;
            klist[OS_MAX_BLOCKS] = k;
        }
        __syncthreads();
        nkept = __builtin_amdgcn_readfirstlane(klist[OS_MAX_BLOCKS]);
        if (nkept == 0) {
            for (int64_t r = row0 + (tid >> 6); r < min(m, row0 + BM); r += kThreadsK / 64)
                for (int64_t c = col0 + lane; c < min(l, col0 + BN); c += 64) C[r * ldc + c] = 0.f;
            return;
        }
        scale = 1.0f / (float)nkept;
    }
    // kept stored block of term index j: lane i of kv[q] holds entry 64q + i
    // of the kept list, read once here and picked with v_readlane, so the K
    // loop issues no scalar or LDS load for it (either would make the wave
    // wait for every LDS access in flight)
    int32_t kv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if constexpr (kMask)
            kv[q] = klist[64 * q + lane];
        else
            kv[q] = kept.idx[64 * q + lane];
    }
    auto kept_at = [&](int j) -> int32_t {
        const int32_t r0 = __builtin_amdgcn_readlane(kv[0], j & 63);
        const int32_t r1 = __builtin_amdgcn_readlane(kv[1], j & 63);
        const int32_t r2 = __builtin_amdgcn_readlane(kv[2], j & 63);
        const int32_t r3 = __builtin_amdgcn_readlane(kv[3], j & 63);
        return j < 64 ? r0 : (j < 128 ? r1 : (j < 192 ? r2 : r3));
    };

    v16f acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    constexpr int kStep = kStepBytes / P::kElem;     // K values per step
    const int tpb = bp / kStep;                       // K steps per term
    int t_begin = 0;
    int t_end = nkept * nsub * tpb;                   // this workgroup's K steps
    if constexpr (kSplit) {
        t_begin = split * sk.chunk;
        t_end = min(t_end, t_begin + sk.chunk);
    }
    // byte offsets of the first K column of step `step` in A and in B
    // (terms in order, kStep columns per step)
    auto step_ab = [&](int step, uint32_t& ka, uint32_t& kb) {
        const int term = step / tpb;
        const int j = term / nsub;
        const int sub = term - j * nsub;
        const int64_t c = (int64_t)kept_at(j) * bp + (int64_t)(step % tpb) * kStep;
        ka = (uint32_t)((c + (sub == 2 ? lo_off : 0)) * P::kElem);
        kb = (uint32_t)((c + (sub == 1 ? lo_off : 0)) * P::kElem);
    };

    const __amdgpu_buffer_rsrc_t ra_src =
        tile_rsrc(static_cast<const char*>(At) + row0 * ldat * P::kElem);
    const __amdgpu_buffer_rsrc_t rb_src =
        tile_rsrc(static_cast<const char*>(Bt) + col0 * ldbt * P::kElem);
    // 256 tile rows per operand and step: 4 direct loads per wave
    uint32_t va[4], vb[4];
    direct_offsets<4>(va, ldat * P::kElem, (int)min((int64_t)BM - 1, m - 1 - row0), wave, lane);
    direct_offsets<4>(vb, ldbt * P::kElem, (int)min((int64_t)BN - 1, l - 1 - col0), wave, lane);
    int fa_off[4], fb_off[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        fa_off[q] = direct_frag_off(wm * 128 + (lane & 31), q, lane);
        fb_off[q] = direct_frag_off(wn * 64 + (lane & 31), q, lane);
    }
    auto frag = [&](float4 (&a)[4], float4 (&b)[2], const float* as, const float* bs, int q) {
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const float4*>(as + fa_off[q] + 1024 * i);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const float4*>(bs + fb_off[q] + 1024 * j);
    };
    auto issue = [&](float* as, float* bs, int step) {
        uint32_t ka, kb;
        step_ab(step, ka, kb);
        direct_issue<4>(ra_src, as, va, ka, wave);
        direct_issue<4>(rb_src, bs, vb, kb, wave);
    };

    issue(As0, Bs0, t_begin);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    float4 fa[4], fb[2], ga[4], gb[2];
    frag(fa, fb, As0, Bs0, 0);
    // One K step: the next step's tiles go straight into the other buffers
    // (last read before the previous step's barrier) while this step's four
    // quads run; each quad's fragments are read during the previous quad's
    // MFMAs, after its first kHead parts, and the last quad's final kTail
    // parts run after the step's barrier, behind the reads of the next
    // step's first fragments (scheduling barriers pin this order).  The A
    // tile's loads are issued at the step's start and the B tile's after the
    // first quad, which halves the burst of line requests a CU sends at once
    // (the same loads; 2-3 % faster for BF16, 1 % for FP32); all are waited
    // for at the step's end.
    // Past the last step the tile loaded is step t_end - 1 again, a valid
    // address.  Steps run in pairs (one per buffer); when their count is odd
    // (kOdd kernels only) the last step runs alone after the pairs, from
    // the first buffer, where the last pair loaded it.
    auto quad = [&](float4 (&a)[4], float4 (&b)[2], auto&& reads) {
        P::template mfma_quad<4, 2, 0, P::kHead>(acc, a, b);
        __builtin_amdgcn_sched_barrier(0);
        reads();
        __builtin_amdgcn_sched_barrier(0);
        P::template mfma_quad<4, 2, P::kHead, P::kParts>(acc, a, b);
        __builtin_amdgcn_sched_barrier(0);
    };
    auto kstep = [&](const float* as, const float* bs, float* na, float* nb, int t) {
        uint32_t ka, kb;
        step_ab(min(t + 1, t_end - 1), ka, kb);
        direct_issue<4>(ra_src, na, va, ka, wave);
        __builtin_amdgcn_sched_barrier(0);
        quad(fa, fb, [&] { frag(ga, gb, as, bs, 1); });
        direct_issue<4>(rb_src, nb, vb, kb, wave);
        __builtin_amdgcn_sched_barrier(0);
        quad(ga, gb, [&] { frag(fa, fb, as, bs, 2); });
        quad(fa, fb, [&] { frag(ga, gb, as, bs, 3); });
        P::template mfma_quad<4, 2, 0, P::kParts - P::kTail>(acc, ga, gb);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        frag(fa, fb, na, nb, 0);
        __builtin_amdgcn_sched_barrier(0);
        P::template mfma_quad<4, 2, P::kParts - P::kTail, P::kParts>(acc, ga, gb);
        __builtin_amdgcn_sched_barrier(0);
    };
    int t = t_begin;
    for (; t + 1 < t_end; t += 2) {
        kstep(As0, Bs0, As1, Bs1, t);
        kstep(As1, Bs1, As0, Bs0, t + 1);
    }
    if constexpr (kOdd) {
        if (t < t_end) kstep(As0, Bs0, As1, Bs1, t);
    }

    // 32x32 accumulator layout: register r of lane L holds row
    // 8*(r/4) + 4*(L/32) + r%4 and column L%32 of the block.
    float* out = C;
    int64_t ldo = ldc;
    if constexpr (kSplit) {
        out = sk.part + (int64_t)split * m * l;
        ldo = l;
        scale = 1.0f;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t col = col0 + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + wm * 128 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row < m && col < l) out[row * ldo + col] = acc[i][j][r] * scale;
            }
        }
    }
}

// C = scale * (sum of the nsplit partial products, in split order).
__global__ __launch_bounds__(256) void split_sum_kernel(const float* __restrict__ part,
                                                        int32_t nsplit, int64_t m, int64_t l,
                                                        float scale, float* __restrict__ C,
                                                        int64_t ldc) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m * l) return;
    const int64_t row = i / l;
    float v = 0.f;
    for (int32_t s = 0; s < nsplit; ++s) v += part[(int64_t)s * m * l + i];
    C[row * ldc + (i - row * l)] = v * scale;
}

typedef int i32x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// FP8 (E4M3) operands with one E8M0 scale per 64 K values of a row, on the
// gfx950 scaled MFMA v_mfma_scale_f32_32x32x64_f8f6f4 (FP32 accumulation; the
// hardware multiplies the products by the row scales of A and B).  A row of
// an operand holds its codes, then one scale byte per 64 codes (`scales`
// bytes after the row's start).  The pipeline is gemm_kept_kernel's: eight waves per
// 256 x 256 tile (two per SIMD, 128 x 64 each), K steps of 128 codes (128
// bytes of every tile row) loaded straight into LDS, two step buffers.  A
// step is two substeps, one per 64-value scale block: substep s is one
// scaled MFMA per 32x32 block, lane half h holding the 32 codes at byte
// 64 s + 32 h of the step's row (two 16-byte LDS reads: logical chunks
// 4 s + 2 h and 4 s + 2 h + 1), both halves passing the block's scale.
// Scale bytes: the two of a step sit in one aligned 4-byte word of the row's
// scale area (word at scales + (c / 64 & ~3) for code column c, the step's
// pair in half hsel = (c / 128) & 1); every step each wave loads 64 such
// words straight into LDS, A's rows by waves 0-3 and B's by waves 4-7, laid
// out so that a fragment lane's four A rows (or two B rows) are consecutive
// words: one 16-byte (8-byte) LDS read per lane per step.
// Scale chunks (kChunk, when the block stride is a multiple of 1024 codes
// and rows and the scale area are 16-byte aligned): the scale loads above
// read 64 rows per instruction, one 4-byte piece each, and cost about as
// much as a whole step's tile loads; instead each wave loads 16 bytes of
// its 64 rows (the scales of 8 steps) once per 8 steps, into one of two
// chunk buffers, and each step reads its pair of scale bytes per row from
// there (the chunk for steps 8c .. 8c + 7 is loaded during step 8c - 8).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fp8_frag_off(int rbase, int s, int p, int lane) {
    return rbase * 32 + 4 * ((4 * s + 2 * (lane >> 5) + p) ^ chunk_key(rbase));
}

template <bool kOdd, bool kSplit = false, bool kChunk = false>
__global__ __launch_bounds__(kThreadsK) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gemm_kept_fp8d_kernel(const uint8_t* __restrict__ At, int64_t ldat,
                           const uint8_t* __restrict__ Bt, int64_t ldbt, int64_t scales,
                           int64_t m, int64_t l, int32_t bp, BlockList kept, int32_t nkept,
                           int32_t nsub, int64_t lo_off, float scale, float* __restrict__ C,
                           int64_t ldc, int32_t tilesM, int32_t tilesN, SplitK sk) {
    __shared__ __align__(1024) float As0[BM * 32];
    __shared__ __align__(1024) float As1[BM * 32];
    __shared__ __align__(1024) float Bs0[BN * 32];
    __shared__ __align__(1024) float Bs1[BN * 32];
    // scale words of a step (A's rows, then B's), or two chunk buffers of
    // 16 bytes per row
    __shared__ __align__(16) uint32_t Sc0[kChunk ? 4 : BM + BN];
    __shared__ __align__(16) uint32_t Sc1[kChunk ? 4 : BM + BN];
    __shared__ __align__(16) uint32_t Sq[kChunk ? 2 * 4 * (BM + BN) : 4];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar M0 and selects
    const int wm = wave >> 2;
    const int wn = wave & 3;

    const int64_t ntiles = (int64_t)tilesM * tilesN;
    int32_t split = 0;
    int64_t T;
    if constexpr (kSplit) {
        split = (int32_t)(blockIdx.x / ntiles);
        T = (int64_t)blockIdx.x - (int64_t)split * ntiles;
    } else {
        T = xcd_task(blockIdx.x, ntiles);
    }
    const int64_t group = T / ((int64_t)kGroupM * tilesN);
    const int64_t first_m = group * kGroupM;
    const int64_t gsz = min((int64_t)kGroupM, (int64_t)tilesM - first_m);
    const int64_t in_group = T - group * kGroupM * tilesN;
    const int64_t tm = first_m + in_group % gsz;
    const int64_t tn = in_group / gsz;
    const int64_t row0 = tm * BM;
    const int64_t col0 = tn * BN;

    int32_t kv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) kv[q] = kept.idx[64 * q + lane];
    auto kept_at = [&](int j) -> int32_t {
        const int32_t r0 = __builtin_amdgcn_readlane(kv[0], j & 63);
        const int32_t r1 = __builtin_amdgcn_readlane(kv[1], j & 63);
        const int32_t r2 = __builtin_amdgcn_readlane(kv[2], j & 63);
        const int32_t r3 = __builtin_amdgcn_readlane(kv[3], j & 63);
        return j < 64 ? r0 : (j < 128 ? r1 : (j < 192 ? r2 : r3));
    };

    v16f acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    constexpr int kStep = kStepBytes;                 // 128 codes per step
    const int tpb = bp / kStep;
    int t_begin = 0;
    int t_end = nkept * nsub * tpb;                   // this workgroup's K steps
    if constexpr (kSplit) {
        t_begin = split * sk.chunk;
        t_end = min(t_end, t_begin + sk.chunk);
    }
    // code byte offsets of step `step` in A and B (terms in order)
    auto step_ab = [&](int step, uint32_t& ka, uint32_t& kb) {
        const int term = step / tpb;
        const int j = term / nsub;
        const int sub = term - j * nsub;
        const int64_t c = (int64_t)kept_at(j) * bp + (int64_t)(step % tpb) * kStep;
        ka = (uint32_t)(c + (sub == 2 ? lo_off : 0));
        kb = (uint32_t)(c + (sub == 1 ? lo_off : 0));
    };

    const int alast = (int)min((int64_t)BM - 1, m - 1 - row0);
    const int blast = (int)min((int64_t)BN - 1, l - 1 - col0);
    const __amdgpu_buffer_rsrc_t ra_src = tile_rsrc(At + row0 * ldat);
    const __amdgpu_buffer_rsrc_t rb_src = tile_rsrc(Bt + col0 * ldbt);
    uint32_t va[4], vb[4];
    direct_offsets<4>(va, ldat, alast, wave, lane);
    direct_offsets<4>(vb, ldbt, blast, wave, lane);
    // scale word of this lane's row: word p = 64 (wave % 4) + lane of A's
    // (waves 0-3) or B's (waves 4-7) area holds row (4 consecutive words per
    // A fragment lane: rows wm*128 + 32 i + r; 2 per B fragment lane: rows
    // wn*64 + 32 j + r)
    const int p = 64 * (wave & 3) + lane;
    const bool a_side = wave < 4;
    const int srow = a_side ? (p >> 7) * 128 + 32 * (p & 3) + ((p >> 2) & 31)
                            : (p >> 6) * 64 + 32 * (p & 1) + ((p >> 1) & 31);
    // scale chunks keep rows in their natural order (entry p: row p of A,
    // or row p - 256 of B), so that the 32 lanes of a fragment half read
    // 16-byte-spaced entries (two lanes per bank) instead of 64-byte-spaced
    // ones (sixteen)
    const int crow = kChunk ? 64 * (wave & 3) + lane : srow;
    const uint32_t so = a_side ? (uint32_t)((int64_t)min(crow, alast) * ldat + scales)
                               : (uint32_t)((int64_t)min(crow, blast) * ldbt + scales);
    const __amdgpu_buffer_rsrc_t rs_src = a_side ? ra_src : rb_src;
    const int sbase = a_side ? 64 * (wave & 3) : BM + 64 * (wave & 3);

    // the A tile and (per-step words) the scale words of a step; the B tile
    // is issued on its own
    auto issue_a = [&](float* as, uint32_t* sc, uint32_t ka, uint32_t kb) {
        direct_issue<4>(ra_src, as, va, ka, wave);
#if defined(__HIP_DEVICE_COMPILE__)
        if constexpr (!kChunk) {
            const uint32_t kc = a_side ? ka : kb;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_src, (lds_void*)(sc + sbase), 4, so,
                                                     (kc / kFp8Block) & ~3u, 0, 0);
        }
#else
        (void)sc;
        (void)kb;
#endif
    };
    auto issue = [&](float* as, float* bs, uint32_t* sc, int step) {
        uint32_t ka, kb;
        step_ab(step, ka, kb);
        direct_issue<4>(ra_src, as, va, ka, wave);
        direct_issue<4>(rb_src, bs, vb, kb, wave);
#if defined(__HIP_DEVICE_COMPILE__)
        if constexpr (!kChunk) {
            const uint32_t kc = a_side ? ka : kb;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_src, (lds_void*)(sc + sbase), 4, so,
                                                     (kc / kFp8Block) & ~3u, 0, 0);
        }
#else
        (void)sc;
        (void)so;
        (void)rs_src;
        (void)sbase;
#endif
    };
    // the scale chunk of steps step .. step + 7 (step a multiple of 8) into
    // chunk buffer (step / 8) % 2: 16 bytes of each of the wave's 64 rows
    auto issue_chunk = [&](int step) {
#if defined(__HIP_DEVICE_COMPILE__)
        uint32_t ka, kb;
        step_ab(step, ka, kb);
        const uint32_t kc = a_side ? ka : kb;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs_src, (lds_void*)(Sq + ((step >> 3) & 1) * 4 * (BM + BN) + 4 * sbase), 16, so,
            kc / kFp8Block, 0, 0);
#else
        (void)step;
#endif
    };
    // the half of a step's scale word that holds its pair of scale bytes
    auto hsel = [&](int step, bool a) -> uint32_t {
        uint32_t ka, kb;
        step_ab(step, ka, kb);
        return (((a ? ka : kb) / kStep) & 1u) * 16u;
    };

    int fa_off[2][2], fb_off[2][2];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            fa_off[s2][q] = fp8_frag_off(wm * 128 + (lane & 31), s2, q, lane);
            fb_off[s2][q] = fp8_frag_off(wn * 64 + (lane & 31), s2, q, lane);
        }
    auto as_i32x8 = [](const float4& lo, const float4& hi) -> i32x8 {
        return i32x8{__float_as_int(lo.x), __float_as_int(lo.y), __float_as_int(lo.z),
                     __float_as_int(lo.w), __float_as_int(hi.x), __float_as_int(hi.y),
                     __float_as_int(hi.z), __float_as_int(hi.w)};
    };
    // A fragment of row block i of substep s2; B fragments of substep s2
    auto frag_a = [&](const float* as, int s2, int i) -> i32x8 {
        return as_i32x8(*reinterpret_cast<const float4*>(as + fa_off[s2][0] + 1024 * i),
                        *reinterpret_cast<const float4*>(as + fa_off[s2][1] + 1024 * i));
    };
    auto frag_b = [&](i32x8 (&b)[2], const float* bs, int s2) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
            b[j] = as_i32x8(*reinterpret_cast<const float4*>(bs + fb_off[s2][0] + 1024 * j),
                            *reinterpret_cast<const float4*>(bs + fb_off[s2][1] + 1024 * j));
    };
    const int sa_word = 4 * (wm * 32 + (lane & 31));
    const int sb_word = BM + 2 * (wn * 32 + (lane & 31));
    // the step's pair of scale bytes (substep 0 low, substep 1 high) of the
    // lane's four A rows and two B rows
    uint32_t sa[4], sb[2];
    auto read_scales = [&](const uint32_t* sc, int step) {
        if constexpr (kChunk) {
            const uint16_t* q =
                reinterpret_cast<const uint16_t*>(Sq + ((step >> 3) & 1) * 4 * (BM + BN));
            const int h = step & 7;
#pragma unroll
            for (int i = 0; i < 4; ++i) sa[i] = q[8 * (wm * 128 + 32 * i + (lane & 31)) + h];
#pragma unroll
            for (int j = 0; j < 2; ++j) sb[j] = q[8 * (BM + wn * 64 + 32 * j + (lane & 31)) + h];
        } else {
            const uint4 wa = *reinterpret_cast<const uint4*>(sc + sa_word);
            const uint2 wb = *reinterpret_cast<const uint2*>(sc + sb_word);
            const uint32_t ha = hsel(step, true);
            const uint32_t hb = hsel(step, false);
            sa[0] = wa.x >> ha;
            sa[1] = wa.y >> ha;
            sa[2] = wa.z >> ha;
            sa[3] = wa.w >> ha;
            sb[0] = wb.x >> hb;
            sb[1] = wb.y >> hb;
        }
    };

    issue(As0, Bs0, Sc0, t_begin);
    if constexpr (kChunk) issue_chunk(t_begin);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    i32x8 fa, fb[2], fan, fbn[2];
    fa = frag_a(As0, 0, 0);
    frag_b(fb, Bs0, 0);
    read_scales(Sc0, t_begin);
    // One step: the next step's tiles and scale words go straight into the
    // other buffers while this step runs (the A tile and scales at the step's
    // start, the B tile after a quarter of its MFMAs, as in gemm_kept_kernel:
    // about 2 % faster); the A fragment of the next (substep, row block) is
    // read during the current one's two MFMAs, and substep 1's B fragments
    // during substep 0's last row block.  Steps run in pairs; an odd last
    // step (kOdd) runs alone after them.
    auto kstep = [&](const float* as, const float* bs, float* na, float* nb, uint32_t* nsc,
                     int t) {
        uint32_t ka, kb;
        step_ab(min(t + 1, t_end - 1), ka, kb);
        issue_a(na, nsc, ka, kb);
        if constexpr (kChunk) {
            if ((t & 7) == 0 && t + 8 < t_end) issue_chunk(t + 8);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (s2 == 0 && i == 2) {
                    __builtin_amdgcn_sched_barrier(0);
                    direct_issue<4>(rb_src, nb, vb, kb, wave);
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (i < 3) {
                    fan = frag_a(as, s2, i + 1);
                } else if (s2 == 0) {
                    fan = frag_a(as, 1, 0);
                    frag_b(fbn, bs, 1);
                }
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        fa, fb[j], acc[i][j], 0, 0, 0, (int)((sa[i] >> (8 * s2)) & 0xFFu), 0,
                        (int)((sb[j] >> (8 * s2)) & 0xFFu));
                if (i < 3 || s2 == 0) fa = fan;
            }
            if (s2 == 0) {
                fb[0] = fbn[0];
                fb[1] = fbn[1];
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        fa = frag_a(na, 0, 0);
        frag_b(fb, nb, 0);
        read_scales(nsc, min(t + 1, t_end - 1));
    };
    int t = t_begin;
    for (; t + 1 < t_end; t += 2) {
        kstep(As0, Bs0, As1, Bs1, Sc1, t);
        kstep(As1, Bs1, As0, Bs0, Sc0, t + 1);
    }
    if constexpr (kOdd) {
        if (t < t_end) kstep(As0, Bs0, As1, Bs1, Sc1, t);
    }

    float* out = C;
    int64_t ldo = ldc;
    if constexpr (kSplit) {
        out = sk.part + (int64_t)split * m * l;
        ldo = l;
        scale = 1.0f;
    }

#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t col = col0 + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + wm * 128 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row < m && col < l) out[row * ldo + col] = acc[i][j][r] * scale;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Grouped symmetric block product for a batch of sketched Gram matrices:
//   H_k = scale_k * S_k S_k^T, S_k the line-major sketch (m_k rows) of
//   problem k with only its kept blocks stored, so the sum over the kept
//   blocks runs over its first ksteps * 32 columns (padding columns are
//   zero; ksteps is even, the sketch carrying one more zero step when K*bp/32
//   is odd).  One persistent launch over a tile list that holds the
//   upper-triangle tiles (ti <= tj) of every problem.  Workgroup g takes
//   tiles starts[g] .. starts[g+1] - 1 (a static schedule balanced on the
//   host; every wave reaches its end), computing each with the same FP32
//   MFMA pipeline as above; an off-diagonal tile is also stored
//   transposed (mirror) when `full`.
// kWT = 4: 256 x 256 tiles, eight waves of 128 x 64 (two per SIMD, as in
// gemm_kept_kernel); kWT = 2: 128 x 128 tiles, four waves of 64 x 64 and two
// workgroups per CU (less padding on small problems).
// ---------------------------------------------------------------------------
template <int kWT>
struct TileShape {
    static constexpr int BT = 64 * kWT;                // tile side
    static constexpr int kWaves = 2 * kWT;             // 8 (256 tiles) or 4 (128 tiles)
    static constexpr int kThreads = 64 * kWaves;
    static constexpr int kI = kWT;                     // 32x32 blocks per wave: rows
    static constexpr int kJ = 2;                       //   and columns
    static constexpr int kU = BT / (8 * kWaves);       // direct loads per wave per operand
};


template <int kWT>
__global__ __launch_bounds__(TileShape<kWT>::kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gemm_batch_sym_kernel(const BatchProblem* __restrict__ probs,
                           const int4* __restrict__ tiles, const int32_t* __restrict__ starts,
                           int full) {
    using TS = TileShape<kWT>;
    constexpr int BT = TS::BT;
    constexpr int kU = TS::kU;
    constexpr int kI = TS::kI;
    constexpr int kJ = TS::kJ;
    // direct tiles as in gemm_kept_kernel: separate arrays per buffer
    __shared__ __align__(1024) float As0[BT * 32];
    __shared__ __align__(1024) float As1[BT * 32];
    __shared__ __align__(1024) float Bs0[BT * 32];
    __shared__ __align__(1024) float Bs1[BT * 32];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / (TS::kWaves / 2);      // 2 waves along the rows
    const int wn = wave % (TS::kWaves / 2);      // kWaves / 2 along the columns
    int fa_off[4], fb_off[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        fa_off[q] = direct_frag_off(wm * 32 * kI + (lane & 31), q, lane);
        fb_off[q] = direct_frag_off(wn * 32 * kJ + (lane & 31), q, lane);
    }
    auto frag = [&](float4 (&a)[kI], float4 (&b)[kJ], const float* as, const float* bs, int q) {
#pragma unroll
        for (int i = 0; i < kI; ++i) a[i] = *reinterpret_cast<const float4*>(as + fa_off[q] + 1024 * i);
#pragma unroll
        for (int j = 0; j < kJ; ++j) b[j] = *reinterpret_cast<const float4*>(bs + fb_off[q] + 1024 * j);
    };

    const int32_t w_end = starts[blockIdx.x + 1];
    for (int32_t w = starts[blockIdx.x]; w < w_end; ++w) {
        const int4 tl = tiles[w];
        const BatchProblem pr = probs[tl.x];
        const int64_t m = pr.m;
        const int64_t row0 = (int64_t)tl.y * BT;
        const int64_t col0 = (int64_t)tl.z * BT;
        const int total = pr.ksteps;          // even: the sketch is padded to whole step pairs
        const __amdgpu_buffer_rsrc_t ra_src = tile_rsrc(pr.S + row0 * pr.ld);
        const __amdgpu_buffer_rsrc_t rb_src = tile_rsrc(pr.S + col0 * pr.ld);
        uint32_t va[kU], vb[kU];
        direct_offsets<kU>(va, pr.ld * 4, (int)min((int64_t)BT - 1, m - 1 - row0), wave, lane);
        direct_offsets<kU>(vb, pr.ld * 4, (int)min((int64_t)BT - 1, m - 1 - col0), wave, lane);
        auto issue = [&](float* as, float* bs, int step) {
            direct_issue<kU>(ra_src, as, va, (uint32_t)step * kStepBytes, wave);
            direct_issue<kU>(rb_src, bs, vb, (uint32_t)step * kStepBytes, wave);
        };

        v16f acc[kI][kJ];
#pragma unroll
        for (int i = 0; i < kI; ++i)
#pragma unroll
            for (int j = 0; j < kJ; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();                       // the previous tile's last reads are done
        issue(As0, Bs0, 0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();

        float4 fa[kI], fb[kJ], ga[kI], gb[kJ];
        frag(fa, fb, As0, Bs0, 0);
        // the order of gemm_kept_kernel's K step (FP32 head and tail parts)
        auto quad = [&](float4 (&a)[kI], float4 (&b)[kJ], auto&& reads) {
            PrecF32::mfma_quad<kI, kJ, 0, PrecF32::kHead>(acc, a, b);
            __builtin_amdgcn_sched_barrier(0);
            reads();
            __builtin_amdgcn_sched_barrier(0);
            PrecF32::mfma_quad<kI, kJ, PrecF32::kHead, PrecF32::kParts>(acc, a, b);
            __builtin_amdgcn_sched_barrier(0);
        };
        // (the B tile issued after the first quad, as in gemm_kept_kernel)
        auto kstep = [&](const float* as, const float* bs, float* na, float* nb, int t) {
            const uint32_t kn = (uint32_t)min(t + 1, total - 1) * kStepBytes;
            direct_issue<kU>(ra_src, na, va, kn, wave);
            __builtin_amdgcn_sched_barrier(0);
            quad(fa, fb, [&] { frag(ga, gb, as, bs, 1); });
            direct_issue<kU>(rb_src, nb, vb, kn, wave);
            __builtin_amdgcn_sched_barrier(0);
            quad(ga, gb, [&] { frag(fa, fb, as, bs, 2); });
            quad(fa, fb, [&] { frag(ga, gb, as, bs, 3); });
            PrecF32::mfma_quad<kI, kJ, 0, PrecF32::kParts - PrecF32::kTail>(acc, ga, gb);
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            frag(fa, fb, na, nb, 0);
            __builtin_amdgcn_sched_barrier(0);
            PrecF32::mfma_quad<kI, kJ, PrecF32::kParts - PrecF32::kTail, PrecF32::kParts>(acc, ga,
                                                                                       gb);
            __builtin_amdgcn_sched_barrier(0);
        };
        for (int t = 0; t < total; t += 2) {
            kstep(As0, Bs0, As1, Bs1, t);
            kstep(As1, Bs1, As0, Bs0, t + 1);
        }

        const bool mirror = full && tl.y != tl.z;
#pragma unroll
        for (int i = 0; i < kI; ++i) {
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                const int64_t col = col0 + wn * 32 * kJ + j * 32 + (lane & 31);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t row = row0 + wm * 32 * kI + i * 32 + 8 * (r >> 2) +
                                        4 * (lane >> 5) + (r & 3);
                    if (row < m && col < m) {
                        const float v = acc[i][j][r] * pr.scale;
                        pr.H[row * pr.ldh + col] = v;
                        if (mirror) pr.H[col * pr.ldh + row] = v;
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Mixed-tile form of the batched symmetric product.  Eight waves per
// workgroup, one job at a time; a job is either
//   kind 0: one 256 x 256 tile, waves of 128 x 64 (as gemm_batch_sym_kernel
//           with kWT = 4), or
//   kind 1: one or two 128 x 128 tiles of one problem, waves 0-3 on the
//           first and 4-7 on the second, each wave a 64 x 64 quarter; the
//           LDS tiles hold the first tile's 128 rows then the second's.
// The host gives each upper triangle's interior to kind 0 and its diagonal
// band and ragged last tile column to kind 1, so a diagonal 256 tile (whose
// lower-left quarter is not needed) is three 128 tiles, and a last tile
// column of at most 128 live columns is computed 128 wide.  A job is two
// int4: {problem, kind, tile row, tile col} and {second tile row, second
// tile col, has second, 0}, tile indices in units of 256 (kind 0) or 128
// (kind 1) rows.  In a kind-1 job without a second tile, waves 4-7 load
// nothing and compute nothing; they keep to the barriers.
// ---------------------------------------------------------------------------

// One job's K loop and epilogue for one wave: kI x 2 MFMA blocks of 32 x 32
// whose A rows start at LDS row arow and B rows at brow, output origin
// (orow, ocol).  load: the wave issues its share of the tile loads (offsets
// va / vb against ra / rb); live: it computes and stores.
template <int kI>
__device__ __forceinline__ void mixed_job(float* As0, float* As1, float* Bs0, float* Bs1,
                                          __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rb,
                                          const uint32_t (&va)[4], const uint32_t (&vb)[4],
                                          bool load, bool live, int total, int arow, int brow,
                                          int wave, int lane, const BatchProblem& pr,
                                          int64_t orow, int64_t ocol, bool mirror) {
    constexpr int kJ = 2;
    int fa_off[4], fb_off[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        fa_off[q] = direct_frag_off(arow + (lane & 31), q, lane);
        fb_off[q] = direct_frag_off(brow + (lane & 31), q, lane);
    }
    auto frag = [&](float4 (&a)[kI], float4 (&b)[kJ], const float* as, const float* bs, int q) {
#pragma unroll
        for (int i = 0; i < kI; ++i) a[i] = *reinterpret_cast<const float4*>(as + fa_off[q] + 1024 * i);
#pragma unroll
        for (int j = 0; j < kJ; ++j) b[j] = *reinterpret_cast<const float4*>(bs + fb_off[q] + 1024 * j);
    };
    auto issue = [&](float* as, float* bs, int step) {
        if (load) {
            direct_issue<4>(ra, as, va, (uint32_t)step * kStepBytes, wave);
            direct_issue<4>(rb, bs, vb, (uint32_t)step * kStepBytes, wave);
        }
    };

    v16f acc[kI][kJ];
#pragma unroll
    for (int i = 0; i < kI; ++i)
#pragma unroll
        for (int j = 0; j < kJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();                           // the previous job's last reads are done
    issue(As0, Bs0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    float4 fa[kI], fb[kJ], ga[kI], gb[kJ];
    if (live) frag(fa, fb, As0, Bs0, 0);
    // the order of gemm_kept_kernel's K step (FP32 head and tail parts)
    auto quad = [&](float4 (&a)[kI], float4 (&b)[kJ], auto&& reads) {
        PrecF32::mfma_quad<kI, kJ, 0, PrecF32::kHead>(acc, a, b);
        __builtin_amdgcn_sched_barrier(0);
        reads();
        __builtin_amdgcn_sched_barrier(0);
        PrecF32::mfma_quad<kI, kJ, PrecF32::kHead, PrecF32::kParts>(acc, a, b);
        __builtin_amdgcn_sched_barrier(0);
    };
    // (the B tile issued after the first quad, as in gemm_kept_kernel)
    auto kstep = [&](const float* as, const float* bs, float* na, float* nb, int t) {
        const uint32_t kn = (uint32_t)min(t + 1, total - 1) * kStepBytes;
        if (load) direct_issue<4>(ra, na, va, kn, wave);
        __builtin_amdgcn_sched_barrier(0);
        if (live) quad(fa, fb, [&] { frag(ga, gb, as, bs, 1); });
        if (load) direct_issue<4>(rb, nb, vb, kn, wave);
        __builtin_amdgcn_sched_barrier(0);
        if (live) {
            quad(ga, gb, [&] { frag(fa, fb, as, bs, 2); });
            quad(fa, fb, [&] { frag(ga, gb, as, bs, 3); });
            PrecF32::mfma_quad<kI, kJ, 0, PrecF32::kParts - PrecF32::kTail>(acc, ga, gb);
        }
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (live) {
            frag(fa, fb, na, nb, 0);
            __builtin_amdgcn_sched_barrier(0);
            PrecF32::mfma_quad<kI, kJ, PrecF32::kParts - PrecF32::kTail, PrecF32::kParts>(acc, ga,
                                                                                       gb);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    for (int t = 0; t < total; t += 2) {
        kstep(As0, Bs0, As1, Bs1, t);
        kstep(As1, Bs1, As0, Bs0, t + 1);
    }
    if (!live) return;

    const int64_t m = pr.m;
#pragma unroll
    for (int i = 0; i < kI; ++i) {
#pragma unroll
        for (int j = 0; j < kJ; ++j) {
            const int64_t col = ocol + j * 32 + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = orow + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row < m && col < m) {
                    const float v = acc[i][j][r] * pr.scale;
                    pr.H[row * pr.ldh + col] = v;
                    if (mirror) pr.H[col * pr.ldh + row] = v;
                }
            }
        }
    }
}

__global__ __launch_bounds__(TileShape<4>::kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gemm_batch_mixed_kernel(const BatchProblem* __restrict__ probs,
                             const int4* __restrict__ jobs, const int32_t* __restrict__ starts,
                             int full) {
    constexpr int BT = 256;
    __shared__ __align__(1024) float As0[BT * 32];
    __shared__ __align__(1024) float As1[BT * 32];
    __shared__ __align__(1024) float Bs0[BT * 32];
    __shared__ __align__(1024) float Bs1[BT * 32];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int half = wave >> 2;

    const int32_t w_end = starts[blockIdx.x + 1];
    for (int32_t w = starts[blockIdx.x]; w < w_end; ++w) {
        const int4 j0 = jobs[2 * w];
        const int4 j1 = jobs[2 * w + 1];
        const BatchProblem pr = probs[j0.x];
        const int64_t m = pr.m;
        const bool big = j0.y == 0;
        // this wave's tile: rows ra.. of A's side, rows rb.. of B's side
        bool load = true;
        int64_t ra, rb;
        if (big) {
            ra = (int64_t)j0.z * 256;
            rb = (int64_t)j0.w * 256;
        } else if (half == 0) {
            ra = (int64_t)j0.z * 128;
            rb = (int64_t)j0.w * 128;
        } else {
            load = j1.z != 0;
            ra = (int64_t)(load ? j1.x : j0.z) * 128;
            rb = (int64_t)(load ? j1.y : j0.w) * 128;
        }
        const int span = big ? 256 : 128;
        const int sub = big ? 0 : 128 * half;
        uint32_t va[4], vb[4];
        direct_offsets<4>(va, pr.ld * 4, (int)min((int64_t)span - 1, m - 1 - ra), wave, lane, sub);
        direct_offsets<4>(vb, pr.ld * 4, (int)min((int64_t)span - 1, m - 1 - rb), wave, lane, sub);
        const __amdgpu_buffer_rsrc_t rsa = tile_rsrc(pr.S + ra * pr.ld);
        const __amdgpu_buffer_rsrc_t rsb = tile_rsrc(pr.S + rb * pr.ld);
        const bool mirror = full && ra != rb;
        if (big) {
            const int wm = wave >> 2, wn = wave & 3;
            mixed_job<4>(As0, As1, Bs0, Bs1, rsa, rsb, va, vb, true, true, pr.ksteps, wm * 128,
                         wn * 64, wave, lane, pr, ra + wm * 128, rb + wn * 64, mirror);
        } else {
            const int wm = (wave >> 1) & 1, wn = wave & 1;
            mixed_job<2>(As0, As1, Bs0, Bs1, rsa, rsb, va, vb, load, load, pr.ksteps,
                         sub + wm * 64, sub + wn * 64, wave, lane, pr, ra + wm * 64,
                         rb + wn * 64, mirror);
        }
    }
}

}  // namespace

bool plan_gemm_ok(int64_t m, int64_t l, int32_t bp, int64_t ldat, int64_t ldbt, int elem) {
    const int step = kStepBytes / elem;
    if (m < 1 || l < 1 || bp < step || bp % step) return false;
    if (ldat * elem > kMaxSketchLdBytes || ldbt * elem > kMaxSketchLdBytes) return false;
    const int64_t tilesM = (m + BM - 1) / BM;
    const int64_t tilesN = (l + BN - 1) / BN;
    return tilesM * tilesN <= 0x7fffffff;
}

hipError_t launch_gemm_kept(const float* At, int64_t ldat, const float* Bt, int64_t ldbt,
                            int64_t m, int64_t l, int32_t bp, const BlockList& kept,
                            int32_t nkept, float scale, float* C, int64_t ldc, hipStream_t s) {
    if (!plan_gemm_ok(m, l, bp, ldat, ldbt, 4) || nkept < 1) return hipErrorInvalidValue;
    const int64_t tilesM = (m + BM - 1) / BM;
    const int64_t tilesN = (l + BN - 1) / BN;
    const bool odd = ((int64_t)nkept * (bp / 32)) % 2 != 0;
    auto kern = odd ? gemm_kept_kernel<PrecF32, false, true> : gemm_kept_kernel<PrecF32, false, false>;
    hipLaunchKernelGGL(kern, dim3((unsigned)(tilesM * tilesN)), dim3(kThreadsK), 0, s, At, ldat,
                       Bt, ldbt, m, l, bp, kept, nkept, 1, (int64_t)0, scale, C, ldc,
                       (int32_t)tilesM, (int32_t)tilesN, CMask{nullptr, 0, 0, 0, 1},
                       SplitK{nullptr, 0});
    return hipGetLastError();
}

// Split K loop for products with few tiles: a single 256x256 tile runs on
// one CU, so a small product (for example 256 x 256 over K = 1024) would leave
// the other CUs idle.  Splits aim at kSplitSlots workgroups (the CU count of
// the device this is tuned for) with at least kSplitMinSteps K steps (one
// step pair) each.
constexpr int64_t kSplitSlots = 256;
constexpr int64_t kSplitMinSteps = 2;

namespace {

int64_t tiles_of_product(int64_t m, int64_t l) { return ((m + BM - 1) / BM) * ((l + BN - 1) / BN); }

// Most splits a product of `tiles` tiles over `steps` K steps takes (< 2: none).
int64_t split_bound(int64_t tiles, int64_t steps) {
    if (tiles * 2 > kSplitSlots) return 1;
    return std::min(kSplitSlots / tiles, steps / kSplitMinSteps);
}

}  // namespace

size_t gemm_split_bytes(int64_t m, int64_t l, int64_t max_steps) {
    if (m < 1 || l < 1) return 0;
    const int64_t S = split_bound(tiles_of_product(m, l), max_steps);
    return S >= 2 ? (size_t)S * (size_t)m * (size_t)l * 4u : 0;
}

namespace {

// Splits and steps per split for `total` K steps of an m x l product (false:
// no split: enough tiles, too few steps, or too little partial space).
bool split_plan(int64_t m, int64_t l, int64_t total, const float* part, size_t part_bytes,
                int64_t& S, int64_t& chunk) {
    S = split_bound(tiles_of_product(m, l), total);
    if (S < 2 || !part) return false;
    chunk = (total + S - 1) / S;
    chunk += chunk & 1;                            // whole step pairs, the last split may be odd
    S = (total + chunk - 1) / chunk;               // every split has at least one step
    return S >= 2 && (size_t)S * (size_t)m * (size_t)l * 4u <= part_bytes;
}

hipError_t launch_split_sum(const float* part, int64_t S, int64_t m, int64_t l, float scale,
                            float* C, int64_t ldc, hipStream_t s) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(split_sum_kernel, dim3((unsigned)((m * l + 255) / 256)), dim3(256), 0, s,
                       part, (int32_t)S, m, l, scale, C, ldc);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_kept_split(const float* At, int64_t ldat, const float* Bt, int64_t ldbt,
                                  int64_t m, int64_t l, int32_t bp, const BlockList& kept,
                                  int32_t nkept, float scale, float* C, int64_t ldc, float* part,
                                  size_t part_bytes, hipStream_t s) {
    if (!plan_gemm_ok(m, l, bp, ldat, ldbt, 4) || nkept < 1) return hipErrorInvalidValue;
    int64_t S = 0, chunk = 0;
    if (!split_plan(m, l, (int64_t)nkept * (bp / 32), part, part_bytes, S, chunk))
        return launch_gemm_kept(At, ldat, Bt, ldbt, m, l, bp, kept, nkept, scale, C, ldc, s);
    const int64_t tilesM = (m + BM - 1) / BM;
    const int64_t tilesN = (l + BN - 1) / BN;
    hipLaunchKernelGGL((gemm_kept_kernel<PrecF32, false, true, true>),
                       dim3((unsigned)(S * tilesM * tilesN)), dim3(kThreadsK), 0, s, At, ldat, Bt,
                       ldbt, m, l, bp, kept, nkept, 1, (int64_t)0, scale, C, ldc, (int32_t)tilesM,
                       (int32_t)tilesN, CMask{nullptr, 0, 0, 0, 1}, SplitK{part, (int32_t)chunk});
    return launch_split_sum(part, S, m, l, scale, C, ldc, s);
}

hipError_t launch_gemm_cmask(const float* At, int64_t ldat, const float* Bt, int64_t ldbt,
                             int64_t m, int64_t l, int32_t bp, int32_t nst, const uint8_t* cmask,
                             int64_t cblk, float* C, int64_t ldc, hipStream_t s) {
    if (!plan_gemm_ok(m, l, bp, ldat, ldbt, 4) || cblk < 1 || nst < 1 || nst > OS_MAX_BLOCKS)
        return hipErrorInvalidValue;
    const int64_t nbI = (m + cblk - 1) / cblk, nbJ = (l + cblk - 1) / cblk;
    const int64_t tb = (cblk + BM - 1) / BM;
    const int64_t tilesM = nbI * tb, tilesN = nbJ * tb;
    if (tilesM * tilesN > 0x7fffffff || nbJ > 0x7fffffff) return hipErrorInvalidValue;
    BlockList none;
    for (int j = 0; j < OS_MAX_BLOCKS; ++j) none.idx[j] = 0;
    // a tile's step count is (its kept blocks) * bp / 32: always even when
    // bp / 32 is, and then the unmasked pair loop serves every tile
    auto kern = (bp / 32) % 2 == 0 ? gemm_kept_kernel<PrecF32, true, false>
                                   : gemm_kept_kernel<PrecF32, true, true>;
    hipLaunchKernelGGL(kern, dim3((unsigned)(tilesM * tilesN)), dim3(kThreadsK), 0, s, At, ldat,
                       Bt, ldbt, m, l, bp, none, 0, 1, (int64_t)0, 1.0f, C, ldc, (int32_t)tilesM,
                       (int32_t)tilesN, CMask{cmask, cblk, (int32_t)nbJ, nst, (int32_t)tb},
                       SplitK{nullptr, 0});
    return hipGetLastError();
}

hipError_t launch_gemm_batch_sym(const BatchProblem* probs, const int4* tiles,
                                 const int32_t* starts, int tile, int full, int32_t grid,
                                 hipStream_t s) {
    if (grid < 1) return hipErrorInvalidValue;
    if (tile == 256)
        hipLaunchKernelGGL(gemm_batch_sym_kernel<4>, dim3((unsigned)grid),
                           dim3(TileShape<4>::kThreads), 0, s,
                           probs, tiles, starts, full);
    else if (tile == 128)
        hipLaunchKernelGGL(gemm_batch_sym_kernel<2>, dim3((unsigned)grid),
                           dim3(TileShape<2>::kThreads), 0, s,
                           probs, tiles, starts, full);
    else if (tile == OS_GRAM_MIXED)
        hipLaunchKernelGGL(gemm_batch_mixed_kernel, dim3((unsigned)grid),
                           dim3(TileShape<4>::kThreads), 0, s,
                           probs, tiles, starts, full);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

int batch_sym_blocks_per_cu(int tile) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    if (tile == 256)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gemm_batch_sym_kernel<4>,
                                                         TileShape<4>::kThreads, 0);
    else if (tile == 128)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gemm_batch_sym_kernel<2>,
                                                         TileShape<2>::kThreads, 0);
    else if (tile == OS_GRAM_MIXED)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gemm_batch_mixed_kernel,
                                                         TileShape<4>::kThreads, 0);
    return e == hipSuccess ? n : 0;
}

hipError_t launch_gemm_kept_fp8(const void* At, int64_t ldat, const void* Bt, int64_t ldbt,
                                int64_t scales, int64_t m, int64_t l, int32_t bp,
                                const BlockList& kept, int32_t nkept, int split, int64_t lo_off,
                                float scale, float* C, int64_t ldc, hipStream_t s) {
    if (!plan_gemm_ok(m, l, bp, ldat, ldbt, 1) || nkept < 1) return hipErrorInvalidValue;
    const int64_t tilesM = (m + BM - 1) / BM;
    const int64_t tilesN = (l + BN - 1) / BN;
    const bool odd = ((int64_t)nkept * (split ? 3 : 1) * (bp / kStepBytes)) % 2 != 0;
    // scale chunks of 8 steps: whole chunks per block, 16-byte aligned rows
    // and scale area
    const bool chunk = bp % 1024 == 0 && ldat % 16 == 0 && ldbt % 16 == 0 && scales % 16 == 0;
    // (with chunks the step count is a multiple of 8: never odd)
    auto kern = chunk ? gemm_kept_fp8d_kernel<false, false, true>
                      : (odd ? gemm_kept_fp8d_kernel<true> : gemm_kept_fp8d_kernel<false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)(tilesM * tilesN)), dim3(kThreadsK), 0, s,
                       static_cast<const uint8_t*>(At), ldat, static_cast<const uint8_t*>(Bt),
                       ldbt, scales, m, l, bp, kept, nkept, split ? 3 : 1, lo_off, scale, C, ldc,
                       (int32_t)tilesM, (int32_t)tilesN, SplitK{nullptr, 0});
    return hipGetLastError();
}

hipError_t launch_gemm_kept_fp8_split(const void* At, int64_t ldat, const void* Bt, int64_t ldbt,
                                      int64_t scales, int64_t m, int64_t l, int32_t bp,
                                      const BlockList& kept, int32_t nkept, int split,
                                      int64_t lo_off, float scale, float* C, int64_t ldc,
                                      float* part, size_t part_bytes, hipStream_t s) {
    if (!plan_gemm_ok(m, l, bp, ldat, ldbt, 1) || nkept < 1) return hipErrorInvalidValue;
    int64_t S = 0, chunk = 0;
    const int64_t total = (int64_t)nkept * (split ? 3 : 1) * (bp / kStepBytes);
    if (!split_plan(m, l, total, part, part_bytes, S, chunk))
        return launch_gemm_kept_fp8(At, ldat, Bt, ldbt, scales, m, l, bp, kept, nkept, split,
                                    lo_off, scale, C, ldc, s);
    const int64_t tilesM = (m + BM - 1) / BM;
    const int64_t tilesN = (l + BN - 1) / BN;
    hipLaunchKernelGGL((gemm_kept_fp8d_kernel<true, true>), dim3((unsigned)(S * tilesM * tilesN)),
                       dim3(kThreadsK), 0, s, static_cast<const uint8_t*>(At), ldat,
                       static_cast<const uint8_t*>(Bt), ldbt, scales, m, l, bp, kept, nkept,
                       split ? 3 : 1, lo_off, scale, C, ldc, (int32_t)tilesM, (int32_t)tilesN,
                       SplitK{part, (int32_t)chunk});
    return launch_split_sum(part, S, m, l, scale, C, ldc, s);
}

hipError_t launch_gemm_kept_bf16(const void* At, int64_t ldat, const void* Bt, int64_t ldbt,
                                 int64_t m, int64_t l, int32_t bp, const BlockList& kept,
                                 int32_t nkept, int split, int64_t lo_off, float scale, float* C,
                                 int64_t ldc, hipStream_t s) {
    if (!plan_gemm_ok(m, l, bp, ldat, ldbt, 2) || nkept < 1) return hipErrorInvalidValue;
    const int64_t tilesM = (m + BM - 1) / BM;
    const int64_t tilesN = (l + BN - 1) / BN;
    const bool odd = ((int64_t)nkept * (split ? 3 : 1) * (bp / 64)) % 2 != 0;
    auto kern = odd ? gemm_kept_kernel<PrecBF16, false, true> : gemm_kept_kernel<PrecBF16, false, false>;
    hipLaunchKernelGGL(kern, dim3((unsigned)(tilesM * tilesN)), dim3(kThreadsK), 0, s, At, ldat,
                       Bt, ldbt, m, l, bp, kept, nkept, split ? 3 : 1, lo_off, scale, C, ldc,
                       (int32_t)tilesM, (int32_t)tilesN, CMask{nullptr, 0, 0, 0, 1},
                       SplitK{nullptr, 0});
    return hipGetLastError();
}

hipError_t launch_gemm_kept_bf16_split(const void* At, int64_t ldat, const void* Bt, int64_t ldbt,
                                       int64_t m, int64_t l, int32_t bp, const BlockList& kept,
                                       int32_t nkept, int split, int64_t lo_off, float scale,
                                       float* C, int64_t ldc, float* part, size_t part_bytes,
                                       hipStream_t s) {
    if (!plan_gemm_ok(m, l, bp, ldat, ldbt, 2) || nkept < 1) return hipErrorInvalidValue;
    int64_t S = 0, chunk = 0;
    const int64_t total = (int64_t)nkept * (split ? 3 : 1) * (bp / 64);
    if (!split_plan(m, l, total, part, part_bytes, S, chunk))
        return launch_gemm_kept_bf16(At, ldat, Bt, ldbt, m, l, bp, kept, nkept, split, lo_off,
                                     scale, C, ldc, s);
    const int64_t tilesM = (m + BM - 1) / BM;
    const int64_t tilesN = (l + BN - 1) / BN;
    hipLaunchKernelGGL((gemm_kept_kernel<PrecBF16, false, true, true>),
                       dim3((unsigned)(S * tilesM * tilesN)), dim3(kThreadsK), 0, s, At, ldat, Bt,
                       ldbt, m, l, bp, kept, nkept, split ? 3 : 1, lo_off, scale, C, ldc,
                       (int32_t)tilesM, (int32_t)tilesN, CMask{nullptr, 0, 0, 0, 1},
                       SplitK{part, (int32_t)chunk});
    return launch_split_sum(part, S, m, l, scale, C, ldc, s);
}

}  // namespace osk
