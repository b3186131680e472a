// Device scratch of the allocation-free SP2 solve (sp2_density_matrix_noalloc):
// one file-scope device array, held by every GPU the library runs on until
// the process ends.  Host code never uses the array's name as an address: its
// device address is looked up once per device, with that device current, and
// kept in a table that the solve reads.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc_internal.h"

static __device__ __align__(256) unsigned char scratch[sp2::kStaticScratchBytes];

namespace sp2 {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    return hipSuccess;
}

}  // namespace sp2
