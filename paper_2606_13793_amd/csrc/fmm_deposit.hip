// Cloud-in-cell deposition of particles on the unigrid, the step before the
// solve (Sec. 3: the paper's test particles reach the grid by CIC).
// A particle of mass m at x spreads over the 2^3 cells whose centres lie
// within one cell of it, with the tent weights prod_d (1 - |x_d - x_c,d| / dx),
// and adds m W / dx^3 to their densities.  Shares that fall outside the box
// are dropped (isolated boundaries: nothing exists there).
//
// One thread per particle; the 8 shares are added with FP64 atomics, so the
// order of the additions into a cell, and with it the last bits of a cell
// that several particles reach, varies from run to run.  Particles are
// usually kept in cell order (as AMR codes keep them), and then the lanes of
// a wave mostly share their 8 target cells: a wave first sums the shares of
// each run of consecutive lanes with the same cells (a segmented scan over
// the lanes), and only the last lane of a run adds them to memory.  In random
// order the runs are single lanes and the scan costs a few shuffles.
#include <hip/hip_runtime.h>

#include "fmm_internal.h"

namespace fmm {
namespace {

constexpr int CIC_THREADS = 256;

__global__ __launch_bounds__(CIC_THREADS) void k_cic(int n, long long count, const double* __restrict__ pos,
                                                     const double* __restrict__ mass, double* __restrict__ rho) {
  const long long t = (long long)blockIdx.x * CIC_THREADS + threadIdx.x;
  const int lane = threadIdx.x & 63;
  // every lane of a wave takes part in the shuffles; lanes past the end or
  // whose particle reaches no cell carry a key of their own and zero shares
  bool ok = t < count;
  int lo[3] = {0, 0, 0};
  double up[3] = {0.0, 0.0, 0.0};  // weight of the upper cell along each axis
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // s = x / dx - 1/2: the cell centres below and above x are floor(s), floor(s) + 1
    const double s = ok ? pos[3 * t + d] * n - 0.5 : 0.0;
    if (!(s >= -1.0 && s < (double)n)) ok = false;  // reaches no cell (or not a number)
    const double f = ok ? floor(s) : 0.0;
    lo[d] = (int)f;
    up[d] = s - f;
  }
  const double m = ok ? mass[t] * ((double)n * n * n) : 0.0;
  double v[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const double wa = (c & 4) ? up[0] : 1.0 - up[0];
    const double wb = (c & 2) ? up[1] : 1.0 - up[1];
    const double wc = (c & 1) ? up[2] : 1.0 - up[2];
    v[c] = ok ? m * (wa * wb * wc) : 0.0;
  }
  // lower corner cell, offset by one so that it is >= 0; lanes without a
  // deposit get distinct negative keys
  const int np = n + 2;
  const int key = ok ? ((lo[0] + 1) * np + (lo[1] + 1)) * np + (lo[2] + 1) : -1 - lane;
  // runs of equal keys: the lane where this lane's run starts
  const int prev = __shfl_up(key, 1);
  int start = (lane == 0 || prev != key) ? lane : 0;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(start, d);
    if (lane >= d && o > start) start = o;
  }
  // inclusive sums of the shares within each run
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double o = __shfl_up(v[c], d);
      if (lane - d >= start) v[c] += o;
    }
  }
  const int next = __shfl_down(key, 1);
  const bool last = lane == 63 || next != key;
  if (!ok || !last) return;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int i = lo[0] + ((c >> 2) & 1), j = lo[1] + ((c >> 1) & 1), k = lo[2] + (c & 1);
    if (i < 0 || i >= n || j < 0 || j >= n || k < 0 || k >= n) continue;
    atomicAdd(rho + ((long long)i * n + j) * n + k, v[c]);
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
