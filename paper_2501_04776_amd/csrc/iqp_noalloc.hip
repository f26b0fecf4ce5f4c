// iqp_expval for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc): the
// workspace is a static device array of kNoAllocBytes that every GPU the
// library runs on holds until the process ends, instead of a caller buffer.
//
// The array's name is a host-side stand-in in host code; its device address
// is taken once per device with hipGetSymbolAddress (with that device
// current) and only that address is passed to the kernels. All calls on one
// GPU share the array: calls that overlap in time on one GPU (on different
// streams, or from different threads) race on it. The forward writes every
// workspace word it later reads, so nothing needs clearing between calls.
#include <mutex>
#include <string>

#include "iqp_plan.h"

namespace iqp {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kNoAllocMaxDevices];

// Device address of `scratch` on the current device, looked up on the first
// call there.
static int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(IQP_ERR_UNSUPPORTED, "device index " + std::to_string(dev) +
                                             " beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(IQP_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return IQP_OK;
}

}  // namespace iqp

using namespace iqp;

extern "C" int iqp_expval_noalloc(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                                  const uint64_t *samples, int precision, double *mean,
                                  double *stderr_, float *phase_save, void *stream) {
    clear_error();
    int st = check_circuit(c);
    if (st) return st;
    const size_t need = iqp_workspace_bytes(IQP_CALL_EXPVAL, c, l, s, 0, precision);
    if (need == 0)  // invalid sizes: the full check below names them
        return expval_call(c, l, ops, s, samples, precision, mean, stderr_, phase_save, nullptr,
                           0, stream, false);
    if (need > kNoAllocBytes)
        return fail(IQP_ERR_WORKSPACE, "iqp_expval_noalloc: these sizes need " +
                                           std::to_string(need) +
                                           " bytes of workspace; the static scratch holds " +
                                           std::to_string(kNoAllocBytes));
    if ((st = check_device())) return st;
    void *ws = nullptr;
    if ((st = scratch_address(&ws))) return st;
    return expval_call(c, l, ops, s, samples, precision, mean, stderr_, phase_save, ws,
                       kNoAllocBytes, stream, false);
}
