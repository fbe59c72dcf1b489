// noalloc.hip -- os_matmul_noalloc: the sketched product for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The workspace os_matmul_prec takes from its caller (prepared sketch,
// sketches of A and B, the transpose of a row-major B, the low-precision
// copies) lives here in one file-scope device array, `scratch`, of
// kScratchBytes.  Each GPU the library runs on holds its own copy of the
// array from module load until the process ends.  Its device address is
// looked up once per device (hipGetSymbolAddress, with that device
// current) and kept; host code only ever passes that address to the
// kernels, never the array's name.  Every kernel of the path writes what
// it later reads (sketches, lists, headers and copies are written whole),
// so nothing is cleared between calls.  All calls on one GPU share the
// array: calls that overlap in time on one GPU (two streams, two host
// threads) race on it and must be serialized by the caller.
#include <mutex>

#include "api_common.h"

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;   // 256 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's `scratch` (looked up on the first call
// on each device), or nullptr with *err set.
void* scratch_on_current_device(hipError_t* err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    *err = hipSuccess;
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

size_t os_noalloc_scratch_bytes(void) { return kScratchBytes; }

os_status os_matmul_noalloc(const os_sketch* sk, const float* A, int64_t lda, const float* B,
                            int64_t ldb, int b_col_major, int64_t m, int64_t n, int64_t l,
                            const uint8_t* keep_host, int kept_only, int precision, float* C,
                            int64_t ldc, void* stream) {
    using namespace osk::api;
    os_status st = check_sketch(sk);
    if (st != OS_OK) return st;
    const size_t need = os_matmul_prec_workspace_bytes(sk, m, n, l, b_col_major, precision);
    if (need == 0) return OS_EINVAL;
    if (need > kScratchBytes) return OS_EWORKSPACE;   // beyond the fixed scratch
    hipError_t e = hipSuccess;
    void* ws = scratch_on_current_device(&e);
    if (!ws) return hip_status(e);
    return os_matmul_prec(sk, A, lda, B, ldb, b_col_major, m, n, l, keep_host, kept_only,
                          precision, C, ldc, ws, kScratchBytes, stream);
}

}  // extern "C"
