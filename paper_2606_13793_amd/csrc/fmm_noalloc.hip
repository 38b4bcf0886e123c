// The static device workspace of fmm_solve_backward_noalloc, and the two
// small kernels that prepare it on the caller's stream.
//
// `scratch` is a file-scope device array: every GPU that loads the library
// holds its own copy at its own address until the process ends.  In host code
// the name `scratch` is only a host-side stand-in for the symbol, so the
// device address is taken once per device with hipGetSymbolAddress (with that
// device current) and only that address is ever passed to kernels.
#include <mutex>

#include "fmm_internal.h"

namespace fmm {
namespace {

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_base[kMaxDevices] = {};

__global__ __launch_bounds__(256) void k_zero(double* __restrict__ p, long long count) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0.0;
}

// segment records passed by value (kernel arguments are copied at launch and
// kept by a captured graph)
struct SegPack {
  Seg s[kMaxAdjSegs];
};
__global__ void k_put_segs(SegPack pk, int count, Seg* __restrict__ dst) {
  if ((int)threadIdx.x < count) dst[threadIdx.x] = pk.s[threadIdx.x];
}

}  // namespace

hipError_t noalloc_base(int device, void** base) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_base[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_base[device] = p;
  }
  *base = g_base[device];
  return hipSuccess;
}

hipError_t noalloc_zero(double* p, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((count + 255) / 256, 8192);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t noalloc_put_segs(const Seg* segs, int count, Seg* dst, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kMaxAdjSegs) return hipErrorInvalidValue;
  SegPack pk{};
  for (int i = 0; i < count; ++i) pk.s[i] = segs[i];
  hipLaunchKernelGGL(k_put_segs, dim3(1), dim3(64), 0, s, pk, count, dst);
  return hipGetLastError();
}

}  // namespace fmm
