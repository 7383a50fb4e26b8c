// fastqsl_q2d_static: fastqsl_q2d with the library's own device scratch instead of a
// caller workspace, for callers that cannot allocate device memory.
//
// The scratch is a file-scope device array of kStaticScratchBytes (64 MiB). Each GPU
// the library runs on holds its own copy from the moment the code object is loaded
// until the process ends. Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a host
// stand-in, not a device address); the address is looked up once per device and
// kept. Every call on one GPU uses that GPU's array, so calls that overlap on one
// GPU (two streams, two threads) race; the call clears every counter it uses itself,
// so what an earlier call left in the array does not matter.
#include <mutex>

#include "fq_internal.h"

namespace {

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The current device's copy of the scratch array, or nullptr.
void *scratch_ptr()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" {

size_t fastqsl_static_scratch_bytes(void) { return kStaticScratchBytes; }

int fastqsl_q2d_static(const fq_field *fields, const fq_plane *planes, int njobs,
                       const fq_params *p, const fq_map *maps, void *stream)
{
    const size_t need = fastqsl_q2d_workspace_size(fields, planes, njobs, p);
    if (need == 0) return FQ_EINVAL;
    if (need > kStaticScratchBytes) return FQ_ENOMEM;
    void *ws = scratch_ptr();
    if (!ws) return FQ_EHIP;
    return fastqsl_q2d(fields, planes, njobs, p, maps, ws, kStaticScratchBytes, stream);
}

}  // extern "C"
