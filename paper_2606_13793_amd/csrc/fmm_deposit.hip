// Cloud-in-cell deposition of particles on the unigrid, the step before the
// solve (Sec. 3: the paper's test particles reach the grid by CIC).
// A particle of mass m at x spreads over the 2^3 cells whose centres lie
// within one cell of it, with the tent weights prod_d (1 - |x_d - x_c,d| / dx),
// and adds m W / dx^3 to their densities.  Shares that fall outside the box
// are dropped (isolated boundaries: nothing exists there).
//
// One thread per particle; the 8 shares are added with FP64 atomics, so the
// order of the additions into a cell, and with it the last bits of a cell
// that several particles reach, varies from run to run.
#include <hip/hip_runtime.h>

#include "fmm_internal.h"

namespace fmm {
namespace {

constexpr int CIC_THREADS = 256;

__global__ __launch_bounds__(CIC_THREADS) void k_cic(int n, long long count, const double* __restrict__ pos,
                                                     const double* __restrict__ mass, double* __restrict__ rho) {
  const long long t = (long long)blockIdx.x * CIC_THREADS + threadIdx.x;
  if (t >= count) return;
  int lo[3];
  double up[3];  // weight of the upper cell along each axis
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // s = x / dx - 1/2: the cell centres below and above x are floor(s), floor(s) + 1
    const double s = pos[3 * t + d] * n - 0.5;
    if (!(s >= -1.0 && s < (double)n)) return;  // reaches no cell (or not a number)
    const double f = floor(s);
    lo[d] = (int)f;
    up[d] = s - f;
  }
  const double m = mass[t] * ((double)n * n * n);
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int i = lo[0] + a;
    if (i < 0 || i >= n) continue;
    const double wa = a ? up[0] : 1.0 - up[0];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = lo[1] + b;
      if (j < 0 || j >= n) continue;
      const double wb = b ? up[1] : 1.0 - up[1];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int k = lo[2] + c;
        if (k < 0 || k >= n) continue;
        const double wc = c ? up[2] : 1.0 - up[2];
        atomicAdd(rho + ((long long)i * n + j) * n + k, m * (wa * wb * wc));
      }
    }
  }
}

}  // namespace

hipError_t launch_cic(int n, long long count, const double* pos, const double* mass, double* rho, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const long long blocks = (count + CIC_THREADS - 1) / CIC_THREADS;
  hipLaunchKernelGGL(k_cic, dim3((unsigned)blocks), dim3(CIC_THREADS), 0, s, n, count, pos, mass, rho);
  return hipGetLastError();
}

}  // namespace fmm
