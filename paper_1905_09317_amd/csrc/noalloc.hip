// Device scratch of the no-allocation entry point (c2f_simulate_noalloc).
//
// One fixed array per device, part of the code object, so that a
// simulation can run without any device allocation: the launch's counters,
// job record, generation tags, arrival planes and work lists are laid out
// inside it by the host runtime.  Host code never passes `scratch` itself
// to a kernel (in host code the name is only a stand-in); it resolves the
// array's device address once per device with hipGetSymbolAddress and uses
// that address everywhere.

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "kernels.h"

namespace c2f {

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;   // device -> address of its copy of the array
std::map<int, std::mutex*> g_scratch_use;
}  // namespace

hipError_t scratch_resolve(int device, void** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = p;
    g_scratch_use[device] = new std::mutex();   // lives as long as the array
    *out = p;
    return hipSuccess;
}

std::mutex& scratch_lock(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return *g_scratch_use.at(device);
}

__global__ void store_job_kernel(Job j, Job* dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = j;
}

hipError_t launch_store_job(const Job& j, Job* dst, hipStream_t s) {
    hipLaunchKernelGGL(store_job_kernel, dim3(1), dim3(64), 0, s, j, dst);
    return hipGetLastError();
}

}  // namespace c2f
