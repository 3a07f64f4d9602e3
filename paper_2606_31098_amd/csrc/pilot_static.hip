// pilot_static.hip -- the fixed device scratch behind pilot_solve_static.
//
// One file-scope device array per GPU, sized kStaticScratchBytes, holds the
// whole workspace of a pilot_solve_static call (descriptors, Gram tables, LM
// states, poses under evaluation, partial sums, pass flags).  In host code the
// array's name is only a stand-in for the symbol: its device address is taken
// once per device with hipGetSymbolAddress (static_scratch_init, called by
// pilot_create with the device current) and every later use goes through that
// address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/pilot.h"
#include "pilot_kernels.h"

namespace pilot {

namespace {

constexpr size_t kStaticScratchBytes = PILOT_STATIC_SCRATCH_BYTES;   // 64 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

__global__ __launch_bounds__(256) void zero_words_kernel(unsigned int *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

}  // namespace

size_t static_scratch_bytes() { return kStaticScratchBytes; }

hipError_t static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void *static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

hipError_t launch_zero_words(void *p, int n_words, hipStream_t s)
{
    if (n_words <= 0) return hipSuccess;
    const int blocks = (n_words + 255) / 256 < 64 ? (n_words + 255) / 256 : 64;
    hipLaunchKernelGGL(zero_words_kernel, dim3(blocks), dim3(256), 0, s, (unsigned int *)p, n_words);
    return hipGetLastError();
}

}  // namespace pilot
