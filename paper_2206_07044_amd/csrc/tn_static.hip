// Fixed device scratch for the allocation-free compression entry point.
//
// `scratch` is a file-scope device array: every GPU the library runs on holds its own copy for
// the life of the process, at its own address.  The host-side name is only a stand-in, so the
// address of each device's copy is looked up once per device (with that device current) when a
// context is created there, and only that address is ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "tn_static.hpp"

namespace tn {

namespace {

static __device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

std::string static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return "device index beyond the static scratch table";
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_addr[device]) return "";
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return std::string("static scratch address: ") + hipGetErrorString(e);
    g_addr[device] = p;
    return "";
}

void* static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_addr[device];
}

}  // namespace tn
