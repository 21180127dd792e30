// Device scratch memory for the entry point that allocates nothing
// (dmrg_sigma_noalloc): a file-scope device array that every GPU the
// library runs on holds for the life of the process.  Host code never
// passes the array's name to a kernel (in host code it is a stand-in, not a
// device address): the address of each device's copy is fetched once with
// hipGetSymbolAddress while that device is current, and only that pointer
// is used.
#include <hip/hip_runtime.h>

#include <mutex>

#include "engine.h"

namespace dmrg {

static __device__ __align__(256) double scratch[kScratchElems];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

void scratch_init(int device) {
    require(device >= 0 && device < kMaxDevices, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    int cur = -1;
    DMRG_HIP(hipGetDevice(&cur));
    require(cur == device, "internal: scratch set-up on a device that is not current", E_STATE);
    void* p = nullptr;
    DMRG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    require(p != nullptr, "hipGetSymbolAddress returned no address for the scratch array", E_HIP);
    g_scratch_ptr[device] = static_cast<double*>(p);
}

double* scratch_ptr(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return nullptr;
    return g_scratch_ptr[device];
}

}  // namespace dmrg
