// Factor-and-solve for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
// every device byte the call needs comes from one static device array of
// kStaticBytes per GPU, reserved when the library's code object is loaded on
// that GPU and held until the process ends.
#include "pf.h"
#include "pf_internal.h"

#include <mutex>

namespace {

constexpr size_t kStaticBytes = size_t(256) << 20;   // 256 MiB per GPU

// Never named in host code except by hipGetSymbolAddress below: on the host
// the name is a stand-in, not the device address of the array.
__device__ __align__(256) char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices];   // per device: the array's device address
std::mutex g_mu;

// The array's address on the current device (looked up once per device,
// with that device current).
hipError_t scratch_on_current_device(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" int pf_factor_solve_static(const pf_matrix *A, const pf_opts *opts, int32_t nrhs,
                                      const double *f, int64_t ldf, double *x, int64_t ldx,
                                      void *stream, pf_info *info)
{
    void *base = nullptr;
    const hipError_t e = scratch_on_current_device(&base);
    if (e != hipSuccess) {
        pf::note_hip_error(e);
        return PF_EHIP;
    }
    return pf::factor_solve_in(A, opts, (char *)base, kStaticBytes, nrhs, f, ldf, x, ldx,
                               (hipStream_t)stream, info);
}
