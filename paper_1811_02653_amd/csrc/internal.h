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

// Launch shapes of the sketch kernels, chosen on the host before anything is
// enqueued (valid == false: the shape does not fit; nothing may be launched).
struct ColsPlan {
    bool valid;
    int rw;          // rows owned by one wave (1, 2, 4)
    int g;           // blocks held in LDS per workgroup
    int64_t nslices; // workgroups per row group
    int64_t tasks;   // workgroups
    size_t lds;      // dynamic LDS bytes
};
struct RowsPlan {
    bool valid;
    int wc;          // columns per workgroup strip (power of two <= 64)
    int g;
    int64_t nslices;
    int64_t tasks;
    size_t lds;
};
// rw / g / wc = 0 choose automatically.
ColsPlan plan_sketch_cols(int64_t rows, int32_t nst, int32_t bp, int rw = 0, int g = 0);
RowsPlan plan_sketch_rows(int64_t cols, int32_t nst, int32_t bp, int wc = 0, int g = 0);
bool plan_gemm_ok(int64_t m, int64_t l, int32_t bp);

hipError_t launch_sketch_cols(const float* X, int64_t rows, int64_t n, int64_t ldx,
                              const uint32_t* table, int64_t nt, const BlockList& bl,
                              int32_t nst, int32_t bp, float* out, int64_t ldo,
                              const ColsPlan& plan, hipStream_t s);
hipError_t launch_sketch_rows(const float* X, int64_t n, int64_t cols, int64_t ldx,
                              const uint32_t* table, int64_t nt, const BlockList& bl,
                              int32_t nst, int32_t bp, float* outT, int64_t ldo,
                              const RowsPlan& plan, hipStream_t s);

// C = scale * sum over the kept stored blocks (bl.idx[0 .. nkept)) of
// At_j * Bt_j^T.
hipError_t launch_gemm_kept(const float* At, int64_t ldat, const float* Bt, int64_t ldbt,
                            int64_t m, int64_t l, int32_t bp, const BlockList& kept,
                            int32_t nkept, float scale, float* C, int64_t ldc, hipStream_t s);

}  // namespace osk
