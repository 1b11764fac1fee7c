// zolo_pd_noalloc: Zolo-PD with its device workspace in a fixed array of
// this library (one per GPU), for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ variable.  Its name, used in host
// code, is only a host-side stand-in for the symbol, so host code never
// passes it to a kernel or a copy: for each device the library looks up the
// array's device address once (hipGetSymbolAddress, from zolo_create with
// that device current) and uses that pointer as the workspace base.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/zolo.h"
#include "handle.hpp"
#include "pd_core.hpp"

namespace zolo {
namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// The device address of `scratch` on `device` (which must be current);
// looked up once per device.  Returns hipSuccess and *out, or the error.
hipError_t scratch_address(int device, char** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

size_t scratch_bytes() { return kScratchBytes; }

}  // namespace zolo

extern "C" int zolo_pd_noalloc(zolo_handle h, int m, int n, const double* A, int lda, double alpha, double l,
                               int r, double* Qp, int ldq, double* H, int ldh, const zolo_opts* opts_in,
                               zolo_info* info) {
    zolo_opts opts;
    int rc = zolo::check_pd_args(h, m, n, A, lda, alpha, l, r, Qp, ldq, H, ldh, opts_in, &opts);
    if (rc) return zolo::report(info, rc);
    if (zolo::workspace_bytes(h, m, n, r, opts) > zolo::scratch_bytes()) return zolo::report(info, ZOLO_SCRATCH);
    char* base = nullptr;
    if (zolo::scratch_address(h->device, &base) != hipSuccess) return zolo::report(info, ZOLO_HIP);
    return zolo::pd_core(h, base, m, n, A, lda, alpha, l, r, Qp, ldq, H, ldh, opts, info);
}
