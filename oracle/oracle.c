/*
 * oracle.c -- plain FP64 CPU oracle for OverSketch's sketched matrix product
 *             C ~= A * S * S^T * B  (Gupta, Wang, Courtade, Ramchandran,
 *             "OverSketch: Approximate Matrix Multiplication for the Cloud").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * Everything here is written as plain loops in FP64, in the order the paper
 * states the computation, with no blocking, fusion or reordering:
 *
 *   - oracle_hash_word / oracle_hash: the random choices of the count sketch
 *     (Algorithm "Calculating Count-sketch of a matrix A": flip each column
 *     with probability 1/2, map it uniformly to one of b buckets).  The paper
 *     does not name a random source.  Reading adopted here: a counter-based
 *     generator, SplitMix64 (Steele, Lea & Flood, "Fast splittable
 *     pseudorandom number generators", OOPSLA 2014), evaluated at state
 *     seed + (ctr+1)*0x9E3779B97F4A7C15 with ctr = (block << 40) | index;
 *     bucket = Lemire multiply-shift of the high 32 bits, sign = low bit.
 *     Written here from the published definition of SplitMix64.
 *   - oracle_sketch_cols: A_tilde_i = A * S_i for every count-sketch block
 *     S_i (the count-sketch algorithm applied to the columns of A, one block
 *     at a time, as in the algorithm "Over sketching A in parallel").
 *   - oracle_sketch_rows: B_tilde_i = S_i^T * B (the same sketch applied to
 *     the rows of B; section 4.1 forms A*S and S^T*B with one S).
 *   - oracle_block_product: C = (1/K) * sum over kept blocks i of
 *     A_tilde_i * B_tilde_i (Eq. (sketch_matrix) gives S the factor
 *     N^{-1/2}; Algorithm "OverSketch" keeps any N of the N+e blocks; the
 *     normalisation 1/K with K = number of kept blocks equals 1/N when
 *     K = N, which is the reading used throughout).
 *   - oracle_sampled_entries: single entries C[r][c] by the same definition
 *     (sketch one row of A and one column of B, then the kept-block dot
 *     products), for matrices too large to sketch whole on the CPU.
 *
 * Pins (tests under tests/ marked "not gpu"): SplitMix64's published output
 * stream; the worked count-sketch example n=9, b=3 of section 4.1; sketching
 * the identity reproduces S; exactness when every block is a signed
 * permutation (S_i S_i^T = I); the b=1 rank-one closed form; the exact
 * mean/variance of Lemma 1 by exhaustive enumeration; unbiasedness
 * (Lemma 2); the exact second moment derived from Lemma 1; the Lemma 3 bound
 * and the tail of the main theorem.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ULL

/* Threads the OpenMP loops below run on. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* SplitMix64 output for state value `state` (the generator first advances
 * its state by the golden-ratio increment, then applies this finaliser). */
static uint64_t splitmix64_finalise(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* The j-th output (j = 0, 1, ...) of SplitMix64 seeded with `seed`. */
uint64_t oracle_splitmix64_nth(uint64_t seed, uint64_t j)
{
    return splitmix64_finalise(seed + (j + 1) * GOLDEN_GAMMA);
}

/* 64-bit random word for sketch block `blk`, input index `k`. */
uint64_t oracle_hash_word(uint64_t seed, uint64_t blk, uint64_t k)
{
    uint64_t ctr = (blk << 40) | k;
    return oracle_splitmix64_nth(seed, ctr);
}

/* Bucket h in [0, b) and sign sigma in {-1, +1} for every (block, index):
 * h[blk * n + k], sigma[blk * n + k]. */
void oracle_hash(uint64_t seed, int64_t nblk, int64_t n, int64_t b,
                 int32_t* h, int8_t* sigma)
{
    for (int64_t blk = 0; blk < nblk; ++blk) {
        for (int64_t k = 0; k < n; ++k) {
            uint64_t w = oracle_hash_word(seed, (uint64_t)blk, (uint64_t)k);
            uint64_t hi = w >> 32;                    /* uniform on [0, 2^32) */
            h[blk * n + k] = (int32_t)((hi * (uint64_t)b) >> 32);
            sigma[blk * n + k] = (w & 1ULL) ? (int8_t)-1 : (int8_t)1;
        }
    }
}

/* Count sketch of the columns of A (m x n, row stride lda), block by block:
 * At (m x nblk*b, row-major, dense) with
 *   At[r][blk*b + h[blk][k]] += sigma[blk][k] * A[r][k],  k ascending. */
void oracle_sketch_cols(const double* A, int64_t m, int64_t n, int64_t lda,
                        const int32_t* h, const int8_t* sigma,
                        int64_t nblk, int64_t b, double* At)
{
    int64_t z = nblk * b;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r) {
        double* out = At + r * z;
        for (int64_t j = 0; j < z; ++j) out[j] = 0.0;
        for (int64_t blk = 0; blk < nblk; ++blk) {
            for (int64_t k = 0; k < n; ++k) {
                int64_t c = h[blk * n + k];
                out[blk * b + c] += (double)sigma[blk * n + k] * A[r * lda + k];
            }
        }
    }
}

/* Count sketch of the rows of B (n x l, row stride ldb), block by block:
 * Bt (nblk*b x l, row-major, dense) with
 *   Bt[blk*b + h[blk][k]][j] += sigma[blk][k] * B[k][j],  k ascending. */
void oracle_sketch_rows(const double* B, int64_t n, int64_t l, int64_t ldb,
                        const int32_t* h, const int8_t* sigma,
                        int64_t nblk, int64_t b, double* Bt)
{
    int64_t z = nblk * b;
    memset(Bt, 0, sizeof(double) * (size_t)(z * l));
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < l; ++j) {
        for (int64_t blk = 0; blk < nblk; ++blk) {
            for (int64_t k = 0; k < n; ++k) {
                int64_t c = h[blk * n + k];
                Bt[(blk * b + c) * l + j] += (double)sigma[blk * n + k] * B[k * ldb + j];
            }
        }
    }
}

/* C (m x l) = (1/K) * sum_{blk : keep[blk]} At_blk * Bt_blk with
 * At (m x nblk*b) and Bt (nblk*b x l) dense row-major, K = number of kept
 * blocks.  Kept blocks are summed in ascending order, inner index ascending.
 * Returns K (0 means nothing was kept; C is then left zero). */
int64_t oracle_block_product(const double* At, const double* Bt,
                             int64_t m, int64_t l, int64_t b, int64_t nblk,
                             const uint8_t* keep, double* C)
{
    int64_t z = nblk * b;
    int64_t K = 0;
    for (int64_t blk = 0; blk < nblk; ++blk) K += keep[blk] ? 1 : 0;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r) {
        double* crow = C + r * l;
        for (int64_t j = 0; j < l; ++j) crow[j] = 0.0;
        for (int64_t blk = 0; blk < nblk; ++blk) {
            if (!keep[blk]) continue;
            for (int64_t c = 0; c < b; ++c) {
                double a = At[r * z + blk * b + c];
                const double* brow = Bt + (blk * b + c) * l;
                for (int64_t j = 0; j < l; ++j) crow[j] += a * brow[j];
            }
        }
        if (K > 0)
            for (int64_t j = 0; j < l; ++j) crow[j] /= (double)K;
    }
    return K;
}

/* Entries C[rows[t]][cols[t]] for t < count, by the definition: sketch row
 * rows[t] of A and column cols[t] of B with every kept block, then
 * (1/K) * sum over kept blocks of the b-long dot product.  A is m x n (lda),
 * B is n x l (ldb); h/sigma as in oracle_hash.  scratch needs 2*b doubles
 * per thread; it is allocated here.  Returns K. */
int64_t oracle_sampled_entries(const double* A, int64_t lda, const double* B, int64_t ldb,
                               int64_t n, const int32_t* h, const int8_t* sigma,
                               int64_t nblk, int64_t b, const uint8_t* keep,
                               const int64_t* rows, const int64_t* cols, int64_t count,
                               double* out)
{
    int64_t K = 0;
    for (int64_t blk = 0; blk < nblk; ++blk) K += keep[blk] ? 1 : 0;
    #pragma omp parallel
    {
        double* ta = (double*)malloc(sizeof(double) * (size_t)b);
        double* tb = (double*)malloc(sizeof(double) * (size_t)b);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < count; ++t) {
            int64_t r = rows[t], c = cols[t];
            double acc = 0.0;
            for (int64_t blk = 0; blk < nblk; ++blk) {
                if (!keep[blk]) continue;
                for (int64_t q = 0; q < b; ++q) { ta[q] = 0.0; tb[q] = 0.0; }
                for (int64_t k = 0; k < n; ++k) {
                    int64_t bucket = h[blk * n + k];
                    double s = (double)sigma[blk * n + k];
                    ta[bucket] += s * A[r * lda + k];
                    tb[bucket] += s * B[k * ldb + c];
                }
                for (int64_t q = 0; q < b; ++q) acc += ta[q] * tb[q];
            }
            out[t] = (K > 0) ? acc / (double)K : 0.0;
        }
        free(ta);
        free(tb);
    }
    return K;
}
