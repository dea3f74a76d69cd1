// Library-held static workspace of the grid kernel, for callers that cannot allocate device memory
// (rebk_solve_ex_static): the partial-sum, reduced-vector and timeout words of one launch live in a
// file-scope device array instead of hipMalloc'd handle memory.  Every device the library runs on
// holds its own copy of the array for the life of the process; host code reaches it only through
// the address hipGetSymbolAddress returns for the current device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "rebk_internal.h"

namespace rebk {
namespace {

__device__ __align__(256) unsigned long long scratch[kStaticScratchWords];

constexpr int kMaxDevices = 64;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

__global__ void __launch_bounds__(256) fill_zero_kernel(unsigned long long* __restrict__ p, size_t n) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) p[q] = 0ull;
}

// ||v||^2 summed in index order by one thread, each square rounded before it is added: the same
// value as the host loop of rebk_solve_ex.
__global__ void sumsq_in_order_kernel(const double* __restrict__ v, int64_t n, double* __restrict__ out) {
#pragma clang fp contract(off)
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (int64_t q = 0; q < n; ++q) {
    const double e = v[q];
    const double sq = e * e;
    s = s + sq;
  }
  *out = s;
}

}  // namespace

hipError_t static_scratch(int device, unsigned long long** ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = (unsigned long long*)p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_fill_zero(unsigned long long* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_sumsq_in_order(const double* v, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sumsq_in_order_kernel, dim3(1), dim3(64), 0, st, v, n, out);
  return hipGetLastError();
}

}  // namespace rebk
