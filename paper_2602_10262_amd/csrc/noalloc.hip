// fp8_gemm without any allocation: the split-K partial sums live in a
// fixed-size device array of this library instead of a caller or library
// workspace, for callers that cannot allocate device memory (code under HIP
// graph capture, serving loops, harnesses that forbid allocation).
//
// The array is a file-scope __device__ object; host code never passes its
// name to a kernel (on the host that name is only a stand-in).  The first
// call on a device, with that device current, looks up the array's device
// address with hipGetSymbolAddress and keeps it per device; every kernel
// argument uses that address.  Each GPU holds its own copy of the array until
// the process ends.  Every call on one GPU shares that GPU's copy, so calls
// that overlap in time on one GPU (on different streams, or from different
// threads without ordering) race on it.  Split-K writes every partial sum it
// later reads, so nothing in the array needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "api_util.hpp"

namespace fp8k {

namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;   // 32 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device).
fp8_status scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return set_error(FP8_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch symbol address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FP8_OK;
}

}  // namespace

}  // namespace fp8k

using namespace fp8k;

extern "C" {

size_t fp8_noalloc_scratch_bytes(void) { return kScratchBytes; }

fp8_status fp8_gemm_noalloc(const fp8_gemm_args *args, const fp8_plan *plan, void *stream)
{
    Prepared pr;
    fp8_status st = prepare_dense(args, pr);
    if (st != FP8_OK) return st;
    fp8_plan res;
    st = resolve_plan(pr, plan, res);
    if (st != FP8_OK) return st;
    const size_t need = workspace_bytes(pr, res);
    if (need > kScratchBytes)
        return set_error(FP8_ERR_UNSUPPORTED, "split-K partial sums need " + std::to_string(need) +
                                                  " bytes, beyond the fixed scratch of " +
                                                  std::to_string(kScratchBytes) + " bytes (choose fewer splits)");
    void *ws = nullptr;
    if (need > 0) {
        st = scratch_address(&ws);
        if (st != FP8_OK) return st;
    }
    return run_prepared(pr, res, ws, need, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
