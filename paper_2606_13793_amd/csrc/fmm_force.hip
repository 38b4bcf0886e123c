// Force from the potential by finite differences, the step after the solve
// (App. C: the host code differentiates phi with a 5-point stencil).  Along
// each axis f = -dphi/dx by fourth-order differences over 5 cells: central
// ones, and in the two layers next to each wall one-sided ones of the same
// order (the box has no cells beyond its walls).  Each is exact for
// polynomials of degree <= 4.
//
// Bandwidth-bound: one thread per cell, 256 consecutive cells of a z line
// per block, so every stencil read of a wave is a contiguous run; the 13
// values a cell reads come mostly from the caches.
#include <hip/hip_runtime.h>

#include "fmm_internal.h"

namespace fmm {
namespace {

constexpr int FD_THREADS = 256;

// 12 dx dphi/dx at position x of a line of n values v(0..n-1) spaced by s
__device__ __forceinline__ double fd12(const double* __restrict__ v, long long s, int x, int n) {
  if (x >= 2 && x <= n - 3) return (v[(x - 2) * s] - v[(x + 2) * s]) + 8.0 * (v[(x + 1) * s] - v[(x - 1) * s]);
  if (x == 1) return -3.0 * v[0] - 10.0 * v[s] + 18.0 * v[2 * s] - 6.0 * v[3 * s] + v[4 * s];
  if (x == 0) return -25.0 * v[0] + 48.0 * v[s] - 36.0 * v[2 * s] + 16.0 * v[3 * s] - 3.0 * v[4 * s];
  const double* w = v + (long long)(n - 1) * s;  // mirrored: the line read backwards from the far wall
  if (x == n - 2) return 3.0 * w[0] + 10.0 * w[-s] - 18.0 * w[-2 * s] + 6.0 * w[-3 * s] - w[-4 * s];
  return 25.0 * w[0] - 48.0 * w[-s] + 36.0 * w[-2 * s] - 16.0 * w[-3 * s] + 3.0 * w[-4 * s];
}

__global__ __launch_bounds__(FD_THREADS) void k_fd_force(int n, const double* __restrict__ phi, double* __restrict__ f) {
  const long long N = (long long)n * n * n;
  const long long u = (long long)blockIdx.x * FD_THREADS + threadIdx.x;
  if (u >= N) return;
  const int k = (int)(u % n), j = (int)((u / n) % n), i = (int)(u / ((long long)n * n));
  const double s = (double)n / 12.0;  // 1 / (12 dx)
  const long long nn = (long long)n * n;
  f[u] = -s * fd12(phi + (u - i * nn), nn, i, n);
  f[N + u] = -s * fd12(phi + (u - (long long)j * n), n, j, n);
  f[2 * N + u] = -s * fd12(phi + (u - k), 1, k, n);
}

}  // namespace

hipError_t launch_fd_force(int n, const double* phi, double* f, hipStream_t s) {
  const long long N = (long long)n * n * n;
  hipLaunchKernelGGL(k_fd_force, dim3((unsigned)((N + FD_THREADS - 1) / FD_THREADS)), dim3(FD_THREADS), 0, s, n, phi,
                     f);
  return hipGetLastError();
}

}  // namespace fmm
