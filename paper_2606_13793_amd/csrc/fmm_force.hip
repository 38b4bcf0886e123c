// Force from the potential by finite differences, the step after the solve
// (App. C: the host code differentiates phi with a 5-point stencil).  Along
// each axis f = -dphi/dx by fourth-order differences over 5 cells: central
// ones, and in the two layers next to each wall one-sided ones of the same
// order (the box has no cells beyond its walls).  Each is exact for
// polynomials of degree <= 4.
//
// Bandwidth-bound, so each phi value should leave HBM once.  A block owns a
// tile of FD_TJ x FD_TK cells of the (y, z) plane and walks FD_CI planes
// along x.  Per plane it stages the tile with a 2-cell margin in LDS, where
// the y and z stencils read it; the x stencil of a cell comes from a
// register window of its own column, phi at x - 2 .. x + 2, which slides by
// one load per plane (the layers next to the x walls read their one-sided
// stencils from memory).  Writes are whole z runs.
#include <hip/hip_runtime.h>

#include "fmm_internal.h"

namespace fmm {
namespace {

constexpr int FD_TK = 64, FD_TJ = 8, FD_CI = 4, FD_THREADS = FD_TK * FD_TJ;
constexpr int FD_HK = FD_TK + 4, FD_HJ = FD_TJ + 4;  // staged plane with its margin

// 12 dx dphi/dx at position x of a line of n values, at(a) = phi at a
template <typename V>
__device__ __forceinline__ double fd12(V at, int x, int n) {
  if (x >= 2 && x <= n - 3) return (at(x - 2) - at(x + 2)) + 8.0 * (at(x + 1) - at(x - 1));
  if (x == 1) return -3.0 * at(0) - 10.0 * at(1) + 18.0 * at(2) - 6.0 * at(3) + at(4);
  if (x == 0) return -25.0 * at(0) + 48.0 * at(1) - 36.0 * at(2) + 16.0 * at(3) - 3.0 * at(4);
  if (x == n - 2) return 3.0 * at(n - 1) + 10.0 * at(n - 2) - 18.0 * at(n - 3) + 6.0 * at(n - 4) - at(n - 5);
  return 25.0 * at(n - 1) - 48.0 * at(n - 2) + 36.0 * at(n - 3) - 16.0 * at(n - 4) + 3.0 * at(n - 5);
}

// Grid: (tiles along z, tiles along y, chunks of FD_CI planes along x).
__global__ __launch_bounds__(FD_THREADS) void k_fd_force(int n, const double* __restrict__ phi, double* __restrict__ f) {
  __shared__ double plane[FD_HJ * FD_HK];
  const long long nn = (long long)n * n, N = nn * n;
  const int tk = threadIdx.x % FD_TK, tj = threadIdx.x / FD_TK;
  const int k0 = blockIdx.x * FD_TK, j0 = blockIdx.y * FD_TJ, i0 = blockIdx.z * FD_CI;
  const int k = k0 + tk, j = j0 + tj;
  const bool mine = k < n && j < n;
  const int i1 = i0 + FD_CI < n ? i0 + FD_CI : n;
  const double s = (double)n / 12.0;  // 1 / (12 dx)
  const long long col = (long long)(mine ? j : 0) * n + (mine ? k : 0);
  // x window: q[d] = phi at x = i - 2 + d of this column (interior planes)
  double q[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    const int x = i0 - 2 + d;
    q[d] = (x >= 0 && x < n) ? phi[x * nn + col] : 0.0;
  }
#pragma unroll 1
  for (int i = i0; i < i1; ++i) {
    // stage plane i, rows j0 - 2 .. j0 + FD_TJ + 1, columns k0 - 2 .. k0 + FD_TK + 1
    __syncthreads();  // the previous plane is consumed
    for (int e = threadIdx.x; e < FD_HJ * FD_HK; e += FD_THREADS) {
      const int hj = e / FD_HK, hk = e - hj * FD_HK;
      const int jj = j0 - 2 + hj, kk = k0 - 2 + hk;
      plane[e] = (jj >= 0 && jj < n && kk >= 0 && kk < n) ? phi[i * nn + (long long)jj * n + kk] : 0.0;
    }
    __syncthreads();
    if (mine) {
      const long long u = i * nn + col;
      // the x walls read their one-sided stencils from memory
      const double fx = (i >= 2 && i <= n - 3) ? (q[0] - q[4]) + 8.0 * (q[3] - q[1])
                                               : fd12([&](int a) { return phi[a * nn + col]; }, i, n);
      // staged cell (jj, kk) sits at row jj - j0 + 2, column kk - k0 + 2
      const double fy = fd12([&](int a) { return plane[(a - j0 + 2) * FD_HK + tk + 2]; }, j, n);
      const double fz = fd12([&](int a) { return plane[(tj + 2) * FD_HK + a - k0 + 2]; }, k, n);
      f[u] = -s * fx;
      f[N + u] = -s * fy;
      f[2 * N + u] = -s * fz;
    }
    // slide the x window by one plane
#pragma unroll
    for (int d = 0; d < 4; ++d) q[d] = q[d + 1];
    const int x = i + 3;
    q[4] = (mine && x < n) ? phi[x * nn + col] : 0.0;
  }
}

}  // namespace

hipError_t launch_fd_force(int n, const double* phi, double* f, hipStream_t s) {
  const dim3 grid((unsigned)((n + FD_TK - 1) / FD_TK), (unsigned)((n + FD_TJ - 1) / FD_TJ),
                  (unsigned)((n + FD_CI - 1) / FD_CI));
  hipLaunchKernelGGL(k_fd_force, grid, dim3(FD_THREADS), 0, s, n, phi, f);
  return hipGetLastError();
}

}  // namespace fmm
