// HIP kernels of the unigrid FMM solve for MI355X (gfx950), and the host code
// that launches them.  Included once per expansion order by fmm_p<P>.hip;
// everything but Impl<P> has internal linkage there (each translation unit
// carries its own constant tables and kernels).
//
// Pass order of one solve (Sec. 2 of the paper):
//   k_p2m            rho -> Mhat_F                       eq. (multipole)
//   k_m2m            Mhat_k -> Mhat_{k-1}, k = F..3      eq. (M2M)
//   k_conv (CV_M2L)  Mhat_{k-1} -> Lam_k, k = 3..F       eq. (M2L) over the oct-shared lists
//                                                        (Sec. 2.2), all levels per launch
//   k_l2l            Lhat_{k-1} -> Lhat_k (+=), 4..F-1   eq. (L2L)
//   k_bottom         Mhat_F, Lhat, rho -> phi, g         M2P at the unigrid centres (Sec. 4),
//                                                        L2P and the near field, eq. (direct)
// Every launch spans a table of segments (grids of several levels and/or
// fields); a block finds its segment by binary search over the first blocks.
// The matrix-core kernels (fmm_mfma.h) are generic over FP64 / FP32 / BF16
// operands; the upward pass and the L2L chain are FP64.
//
// Layouts: multipoles and locals are "chunked", [ceil(terms/4)][cells][4], so
// that a matrix-core operand fragment (4 consecutive terms of one cell) is one
// 32-byte load and cells of a z line are contiguous.  Multipole grids carry a
// zero halo of 3 cells per side: the clipped interaction lists of the isolated
// boundary then need no bounds checks.
#pragma once
#include "fmm_internal.h"

#include <cmath>
#include <type_traits>
#include <vector>

namespace fmm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// Calls f(std::integral_constant<int, k>) for k = I, I + 1, ..., N - 1.
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<N, I + 1>(f);
  }
}

#include "fmm_types.h"

// multi-index table for orders <= PDMAX: packed exponents a | b<<8 | c<<16,
// and 1/a!
__constant__ int c_mi_exp[NTMAX];
__constant__ double c_mi_invfact[NTMAX];
// near-field stencil in grid units, offset delta = u - w in [-3,3]^3:
//   c_p2p_phi = -1/max(|delta|, 1),  c_p2p_g = -delta/|delta|^3 (0 at delta = 0)
__constant__ double c_p2p_phi[343];
__constant__ double c_p2p_g[3 * 343];
// the near-field weights of the transposed solve per offset delta:
// (2 c_p2p_phi, -4 c_p2p_g) at [4 delta], read at wave-uniform addresses
__constant__ double c_p2p_adj[4 * 343];

__device__ __forceinline__ int mi_a(int e) { return e & 255; }
__device__ __forceinline__ int mi_b(int e) { return (e >> 8) & 255; }
__device__ __forceinline__ int mi_c(int e) { return (e >> 16) & 255; }

// segment of block b: the last segment whose first block is <= b
__device__ __forceinline__ const Seg& find_seg(const Seg* __restrict__ segs, int nseg, int b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first_block <= b) lo = mid; else hi = mid - 1;
  }
  return segs[lo];
}
template <typename T>
__device__ __forceinline__ const T* io_rho(const IoArg& io, int f) {
  return (const T*)(io.tab ? io.tab[f].rho : io.rho);
}
template <typename T>
__device__ __forceinline__ T* io_phi(const IoArg& io, int f) {
  return (T*)(io.tab ? io.tab[f].phi : io.phi);
}
template <typename T>
__device__ __forceinline__ T* io_g(const IoArg& io, int f) {
  return (T*)(io.tab ? io.tab[f].g : io.g);
}

hipError_t upload_constants_tu() {
  static bool done = false;
  if (done) return hipSuccess;
  int ex[NTMAX];
  double inv[NTMAX];
  for (int a = 0; a <= PDMAX; ++a)
    for (int b = 0; a + b <= PDMAX; ++b)
      for (int c = 0; a + b + c <= PDMAX; ++c) {
        const int t = mi_index(a, b, c);
        ex[t] = a | (b << 8) | (c << 16);
        double f = 1.0;
        for (int i = 2; i <= a; ++i) f *= i;
        for (int i = 2; i <= b; ++i) f *= i;
        for (int i = 2; i <= c; ++i) f *= i;
        inv[t] = 1.0 / f;
      }
  double pp[343], pg[3 * 343], pa[4 * 343];
  for (int t = 0; t < 343; ++t) {
    const int d0 = t / 49 - 3, d1 = (t / 7) % 7 - 3, d2 = t % 7 - 3;
    const double r2 = double(d0 * d0 + d1 * d1 + d2 * d2);
    if (r2 == 0.0) {
      pp[t] = -1.0;
      pg[t] = pg[343 + t] = pg[686 + t] = 0.0;
    } else {
      const double r = std::sqrt(r2);
      pp[t] = -1.0 / r;
      const double i3 = 1.0 / (r2 * r);
      pg[t] = -d0 * i3;
      pg[343 + t] = -d1 * i3;
      pg[686 + t] = -d2 * i3;
    }
    pa[4 * t] = 2.0 * pp[t];
    for (int o = 0; o < 3; ++o) pa[4 * t + 1 + o] = -4.0 * pg[343 * o + t];
  }
  hipError_t e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_mi_exp), ex, sizeof(ex))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_mi_invfact), inv, sizeof(inv))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_p2p_phi), pp, sizeof(pp))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_p2p_g), pg, sizeof(pg))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_p2p_adj), pa, sizeof(pa))) != hipSuccess) return e;
  done = true;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Green's function derivatives at the 343 x 8 unit displacements
//   Rhat = d + (2q - 1)/4,  d in [-3,3]^3, q in {0,1}^3
// (target child q of a cell P, source J = P - d one level up, in units of the
// source cell size).  f = 1/r obeys, for |g| = n >= 1,
//   n r^2 d^g f = -(2n-1) sum_i g_i R_i d^(g-e_i) f - (n-1) sum_i g_i (g_i-1) d^(g-2e_i) f
// (f is harmonic and homogeneous of degree -1); D = -d^g f is stored.
// FP64, once per plan.
// ---------------------------------------------------------------------------
__device__ void green_derivs(double R0, double R1, double R2, int PD, int ND, double* __restrict__ out) {
  const double r2 = R0 * R0 + R1 * R1 + R2 * R2;
  double f[NTMAX];
  f[0] = 1.0 / sqrt(r2);
  for (int n = 1; n <= PD; ++n)
    for (int a = 0; a <= n; ++a)
      for (int b = 0; a + b <= n; ++b) {
        const int c = n - a - b;
        double s1 = 0.0, s2 = 0.0;
        if (a > 0) {
          s1 += a * R0 * f[mi_index(a - 1, b, c)];
          if (a > 1) s2 += a * (a - 1) * f[mi_index(a - 2, b, c)];
        }
        if (b > 0) {
          s1 += b * R1 * f[mi_index(a, b - 1, c)];
          if (b > 1) s2 += b * (b - 1) * f[mi_index(a, b - 2, c)];
        }
        if (c > 0) {
          s1 += c * R2 * f[mi_index(a, b, c - 1)];
          if (c > 1) s2 += c * (c - 1) * f[mi_index(a, b, c - 2)];
        }
        f[mi_index(a, b, c)] = -((2 * n - 1) * s1 + (n - 1) * s2) / (n * r2);
      }
  for (int i = 0; i < ND; ++i) out[i] = -f[i];
}
__global__ void k_dtab(double* __restrict__ out, int PD, int ND) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 343 * 8) return;
  const int dd = t >> 3, q = t & 7;
  const double R0 = double(dd / 49 - 3) + (((q >> 2) & 1) ? 0.25 : -0.25);
  const double R1 = double((dd / 7) % 7 - 3) + (((q >> 1) & 1) ? 0.25 : -0.25);
  const double R2 = double(dd % 7 - 3) + ((q & 1) ? 0.25 : -0.25);
  green_derivs(R0, R1, R2, PD, ND, out + (size_t)t * ND);
}
// The M2P table of FMM-2: Rhat = d + (2 s - 3) / 8 for the unigrid cell at
// s in {0..3}^3 inside its level-F cell (units of that cell's size).
// Layout [343][64][ND].
__global__ void k_dtab2(double* __restrict__ out, int PD, int ND) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 343 * 64) return;
  const int dd = t >> 6, sb = t & 63;
  const double R0 = double(dd / 49 - 3) + (2 * ((sb >> 4) & 3) - 3) / 8.0;
  const double R1 = double((dd / 7) % 7 - 3) + (2 * ((sb >> 2) & 3) - 3) / 8.0;
  const double R2 = double(dd % 7 - 3) + (2 * (sb & 3) - 3) / 8.0;
  green_derivs(R0, R1, R2, PD, ND, out + (size_t)t * ND);
}

// term index -> packed exponents a | b << 8 | c << 16 (the inverse of
// mi_index), and small constant helpers, usable in constant expressions
constexpr __host__ __device__ int mi_exp_of(int t) {
  int n = 0;
  while (nterms(n) <= t) ++n;
  int r = t - nterms(n - 1), a = 0;
  while (r >= n - a + 1) {
    r -= n - a + 1;
    ++a;
  }
  return a | r << 8 | (n - a - r) << 16;
}
constexpr bool mi_exp_inverts_index() {
  for (int t = 0; t < NTMAX; ++t) {
    const int e = mi_exp_of(t);
    if (mi_index(e & 255, (e >> 8) & 255, e >> 16) != t) return false;
  }
  return true;
}
static_assert(mi_exp_inverts_index(), "mi_exp_of inverts mi_index");
constexpr __host__ __device__ double pow3(int k) { return k == 0 ? 1.0 : 3.0 * pow3(k - 1); }
constexpr __host__ __device__ double fact_d(int k) { return k <= 1 ? 1.0 : k * fact_d(k - 1); }

// ---------------------------------------------------------------------------
// P2M: Mhat_F[a] = sum_q rho_{2T+q} (s_q/4)^a / a!,  s_q,i = 1 - 2 q_i.
// (-1)^(q.a) depends on a only through a mod 2, so the 8 signed sums of the
// children are formed once (a Walsh transform) and each term is one product.
// The term loop is unrolled (P fixed): each term's sign pattern and scale are
// compile-time constants.  Terms past nmax are written as zero.
// ---------------------------------------------------------------------------
// Segments: n = unigrid cells per axis, field, b = Mhat_F (or null: not
// written), t = its copy in the compute type CT (mixed precision; null or
// CT = double: none).  256 cells T per block.
// The typed copy of a multipole grid (mixed plans): term chunks of KC, so a
// cell's chunk is KC/4 of the 4-term groups the P2M kernels form.  put<c, NC>
// adds group c to the chunk being filled and stores the chunk in one vector
// store when it is full or c is the last group (zero terms past the last).
template <typename CT>
struct TypedChunk {
  static constexpr int KC = Mf<CT>::IDX != 0 ? Mf<CT>::KC : 1;
  template <int c, int NC>
  __device__ __forceinline__ static void put(double (&tv)[KC], const d4& o, const void* t, long long ncellp,
                                             long long cp) {
    if constexpr (Mf<CT>::IDX != 0) {
      constexpr int j = (4 * c) % KC;
#pragma unroll
      for (int e = 0; e < 4; ++e) tv[j + e] = o[e];
      if constexpr (j + 4 == KC || c == NC - 1) {
#pragma unroll
        for (int e = j + 4; e < KC; ++e) tv[e] = 0.0;
        if (t) store_chunk((typename Mf<CT>::H*)t + ((4 * c / KC) * ncellp + cp) * KC, tv);
      }
    }
  }
};

template <int P, typename TI, typename CT>
__global__ __launch_bounds__(256) void k_p2m(const Seg* __restrict__ segs, int nseg, IoArg io, int NM) {
  constexpr int NT = nterms(P), NC = (NT + 3) / 4;
  const Seg& sg = find_seg(segs, nseg, blockIdx.x);
  const int n = sg.n;
  const TI* __restrict__ rho = io_rho<TI>(io, sg.field);
  double* __restrict__ M = sg.b;
  const int nF = n >> 1, nFp = nF + 6;
  const long long nT = (long long)nF * nF * nF;
  const long long T = (long long)(blockIdx.x - sg.first_block) * 256 + threadIdx.x;
  if (T >= nT) return;
  const int t2 = (int)(T % nF), t1 = (int)((T / nF) % nF), t0 = (int)(T / ((long long)nF * nF));
  double v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const long long u = ((long long)(2 * t0 + ((q >> 2) & 1)) * n + (2 * t1 + ((q >> 1) & 1))) * n + (2 * t2 + (q & 1));
    v[q] = (double)rho[u];
  }
  double S[8];
#pragma unroll
  for (int pat = 0; pat < 8; ++pat) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += (__popc(q & pat) & 1) ? -v[q] : v[q];
    S[pat] = s;
  }
  const long long ncellp = (long long)nFp * nFp * nFp;
  const long long cp = ((long long)(t0 + 3) * nFp + (t1 + 3)) * nFp + (t2 + 3);
  double tv[TypedChunk<CT>::KC];  // the typed chunk being filled
  static_for<NC>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    d4 o;
    static_for<4>([&](auto ec) {
      constexpr int al = 4 * c + decltype(ec)::value;
      double val = 0.0;
      if constexpr (al < NT) {
        constexpr int ex = mi_exp_of(al);
        constexpr int a = ex & 255, b = (ex >> 8) & 255, z = ex >> 16;
        constexpr int pat = ((a & 1) << 2) | ((b & 1) << 1) | (z & 1);
        constexpr double sc = 1.0 / (fact_d(a) * fact_d(b) * fact_d(z) * (double)(1LL << (2 * (a + b + z))));
        if (al < NM) val = sc * S[pat];
      }
      o[decltype(ec)::value] = val;
    });
    if (M) *reinterpret_cast<d4*>(M + (c * ncellp + cp) * 4) = o;
    TypedChunk<CT>::template put<c, NC>(tv, o, sg.t, ncellp, cp);
  });
}

// P2M of FMM-2: Mhat_F[a] = sum_s rho_{4T+s} w_s^a / a!, w_s,i = (3 - 2 s_i) / 8
// over the 64 unigrid cells s of T.  Segments as k_p2m.  FMM-1 plans use it
// for level F - 1, whose cells also hold 4^3 unigrid cells: the same
// multipoles as M2M of the level-F P2M (M2M re-centres exactly), without
// reading the level-F grid.
// Along one axis w takes the values 3/8, 1/8, -1/8, -3/8, so
//   sum_s w_s^k rho_s = (3/8)^k (rho_0 +- rho_3) + (1/8)^k (rho_1 +- rho_2)
// with + for even k and - for odd k: one butterfly per axis turns the 4
// values of each line into these 4 combinations (slot 2 (k odd) + (|w| =
// 1/8)), and each term is then 8 products with the integer weights 3^k of
// its slots, scaled by 8^-|a| / a!.  The term loop is unrolled (P fixed), so
// the slots are register indices known at compile time.
template <int P, typename TI, typename CT>
__global__ __launch_bounds__(256) void k_p2m2(const Seg* __restrict__ segs, int nseg, IoArg io, int NM) {
  constexpr int NT = nterms(P), NC = (NT + 3) / 4;
  const Seg& sg = find_seg(segs, nseg, blockIdx.x);
  const int n = sg.n;
  const TI* __restrict__ rho = io_rho<TI>(io, sg.field);
  double* __restrict__ M = sg.b;
  const int nF = n >> 2, nFp = nF + 6;
  const long long nT = (long long)nF * nF * nF;
  const long long T = (long long)(blockIdx.x - sg.first_block) * 256 + threadIdx.x;
  if (T >= nT) return;
  const int t2 = (int)(T % nF), t1 = (int)((T / nF) % nF), t0 = (int)(T / ((long long)nF * nF));
  double v[64];
#pragma unroll
  for (int sb = 0; sb < 64; ++sb)
    v[sb] = (double)rho[((long long)(4 * t0 + (sb >> 4)) * n + (4 * t1 + ((sb >> 2) & 3))) * n + (4 * t2 + (sb & 3))];
  // butterflies along z (stride 1), y (4), x (16)
#pragma unroll
  for (int st = 1; st <= 16; st *= 4) {
#pragma unroll
    for (int l = 0; l < 64; ++l)
      if (((l / st) & 3) == 0) {
        const double r0 = v[l], r1 = v[l + st], r2 = v[l + 2 * st], r3 = v[l + 3 * st];
        v[l] = r0 + r3;
        v[l + st] = r1 + r2;
        v[l + 2 * st] = r0 - r3;
        v[l + 3 * st] = r1 - r2;
      }
  }
  const long long ncellp = (long long)nFp * nFp * nFp;
  const long long cp = ((long long)(t0 + 3) * nFp + (t1 + 3)) * nFp + (t2 + 3);
  double tv[TypedChunk<CT>::KC];  // the typed chunk being filled
  static_for<NC>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    d4 o;
    static_for<4>([&](auto ec) {
      constexpr int al = 4 * c + decltype(ec)::value;
      double val = 0.0;
      if constexpr (al < NT) {
        constexpr int ex = mi_exp_of(al);
        constexpr int ax = ex & 255, ay = (ex >> 8) & 255, az = ex >> 16;
        constexpr int base = 16 * 2 * (ax & 1) + 4 * 2 * (ay & 1) + 2 * (az & 1);
        double x = 0.0;
        static_for<8>([&](auto mc) {
          constexpr int m = decltype(mc)::value, mx = m >> 2, my = (m >> 1) & 1, mz = m & 1;
          constexpr double wt = pow3(mx ? 0 : ax) * pow3(my ? 0 : ay) * pow3(mz ? 0 : az);
          x = fma(wt, v[base + 16 * mx + 4 * my + mz], x);
        });
        constexpr double sc = 1.0 / (fact_d(ax) * fact_d(ay) * fact_d(az) * (double)(1LL << (3 * (ax + ay + az))));
        if (al < NM) val = sc * x;
      }
      o[decltype(ec)::value] = val;
    });
    *reinterpret_cast<d4*>(M + (c * ncellp + cp) * 4) = o;
    TypedChunk<CT>::template put<c, NC>(tv, o, sg.t, ncellp, cp);
    // (one chunk at a time: the scheduler would otherwise form every term
    // before the first store and hold them all in registers)
    __builtin_amdgcn_sched_barrier(0);
  });
}

// ---------------------------------------------------------------------------
// M2M: Mhat_{k-1}[a] = sum_q sum_{b<=a} 2^-|b| 4^-|g| / g! (-1)^(q.g) Mhat_k[2P+q][b],
// g = a - b.  Block = 8 parents (consecutive in C order, so their children
// are contiguous along z).  Phase 1: thread (chunk c, parent) loads the 4-term
// chunk c of the parent's 8 children and forms, in registers, the signed sums
// W[pat][b] = sum_q (-1)^popc(q & pat) Mhat[2P+q][b] (a Walsh transform over
// q), staged in LDS.  Phase 2: each output term sums its b <= a.
// Segments: n = child grid cells per axis, a = Mhat_k, b = Mhat_{k-1}, t =
// the copy of Mhat_{k-1} in the compute type CT (or null).
// ---------------------------------------------------------------------------
template <int PO>
struct M2MShape {
  static constexpr int NM = nterms(PO), NC = (NM + 3) / 4;
  static constexpr int PAR = NM <= 56 ? 16 : 8;  // parents per block (LDS budget)
  static constexpr int THREADS = ((PAR * NC + 63) / 64) * 64;
  // (b, g) pairs with b + g = a over all terms a: sum_n C(n + 5, 5) = C(PO + 6, 6)
  static constexpr int NE = (PO + 1) * (PO + 2) * (PO + 3) * (PO + 4) * (PO + 5) * (PO + 6) / 720;
};
// Coefficient lists of the M2M terms (plan-time, in device memory): for
// output term a, entries cstart[a] .. cstart[a+1]-1 hold the LDS offset
// 8 b + pat(g) and the coefficient 2^-|b| 4^-|g| / g! for every b <= a,
// g = a - b.
template <int PO, typename CT>
__global__ __launch_bounds__(M2MShape<PO>::THREADS) void k_m2m(const Seg* __restrict__ segs, int nseg,
                                                              const int* __restrict__ cstart,
                                                              const int* __restrict__ coff,
                                                              const double* __restrict__ ccoef, int nmx) {
  constexpr int NM = M2MShape<PO>::NM, NC = M2MShape<PO>::NC, M2M_THREADS = M2MShape<PO>::THREADS;
  constexpr int NE = M2MShape<PO>::NE, M2M_PAR = M2MShape<PO>::PAR;
  constexpr int WS = NM * 8 + 2;  // per-parent stride, padded against bank conflicts
  __shared__ double W[M2M_PAR * WS];
  __shared__ int sstart[NM + 1];
  __shared__ int soff[NE];
  __shared__ double scoef[NE];
  const Seg& sg = find_seg(segs, nseg, blockIdx.x);
  const double* __restrict__ Mc = sg.a;
  double* __restrict__ Mp = sg.b;
  const int nk = sg.n;
  const int np = nk >> 1, nkp = nk + 6, npp = np + 6;
  const long long ncp_c = (long long)nkp * nkp * nkp, ncp_p = (long long)npp * npp * npp;
  const long long nP = (long long)np * np * np;
  const long long P0 = (long long)(blockIdx.x - sg.first_block) * M2M_PAR;
  for (int t = threadIdx.x; t <= NM; t += M2M_THREADS) sstart[t] = cstart[t];
  for (int t = threadIdx.x; t < NE; t += M2M_THREADS) {
    soff[t] = coff[t];
    scoef[t] = ccoef[t];
  }
  // phase 1
  {
    const int pl = threadIdx.x % M2M_PAR, c = threadIdx.x / M2M_PAR;
    const long long P = P0 + pl;
    if (c < NC && P < nP) {
      const int p2 = (int)(P % np), p1 = (int)((P / np) % np), p0 = (int)(P / ((long long)np * np));
      d4 v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const long long cc = ((long long)(2 * p0 + ((q >> 2) & 1) + 3) * nkp + (2 * p1 + ((q >> 1) & 1) + 3)) * nkp +
                             (2 * p2 + (q & 1) + 3);
        v[q] = *reinterpret_cast<const d4*>(Mc + (c * ncp_c + cc) * 4);
      }
      // in-place Walsh transform: index q becomes pattern pat
#pragma unroll
      for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (!(q & bit)) {
            const d4 x = v[q], y = v[q | bit];
            v[q] = x + y;
            v[q | bit] = x - y;
          }
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (4 * c + e < NM) {
#pragma unroll
          for (int pat = 0; pat < 8; ++pat) W[pl * WS + (4 * c + e) * 8 + pat] = v[pat][e];
        }
    }
  }
  __syncthreads();
  // phase 2: thread (term a, parent), parents fastest so lanes share a list
  for (int w = threadIdx.x; w < M2M_PAR * NM; w += M2M_THREADS) {
    const int pl = w % M2M_PAR, al = w / M2M_PAR;
    const long long P = P0 + pl;
    if (P >= nP) continue;
    const double* Wp = W + pl * WS;
    double acc = 0.0;
    // (unrolled so several list entries' LDS reads are in flight; the sum
    // keeps its order)
#pragma unroll 4
    for (int j = sstart[al]; j < sstart[al + 1]; ++j) acc += scoef[j] * Wp[soff[j]];
    const int p2 = (int)(P % np), p1 = (int)((P / np) % np), p0 = (int)(P / ((long long)np * np));
    const long long cp = ((long long)(p0 + 3) * npp + (p1 + 3)) * npp + (p2 + 3);
    const double v = al < nmx ? acc : 0.0;  // truncation at nmax
    Mp[((al >> 2) * ncp_p + cp) * 4 + (al & 3)] = v;
    if constexpr (Mf<CT>::IDX != 0) {
      constexpr int KC = Mf<CT>::KC;
      if (sg.t) ((typename Mf<CT>::H*)sg.t)[((al / KC) * ncp_p + cp) * KC + al % KC] = static_cast<typename Mf<CT>::H>(v);
    }
  }
}

// ---------------------------------------------------------------------------
// Matrix-core M2L / M2P (FP64, v_mfma_f64_16x16x4f64).
//
// Both are sums over the 189 list offsets d of a parity class: with the
// source grid s, a "row" is a cell P of grid s with parity r, and
//   out[P][col] = sum_d sum_a B_d[a][col] Mhat_s[P - d][a]
// where B_d[a][(q, x)] = D[a + x](Rhat_{d,q}) and x is a local term (M2L) or
// one of {0, e_x, e_y, e_z} (M2P).  A wave owns 16 rows; lanes hold
//   A[i][k] = Mhat[row i - d][4c + k]   (lane i + 16k)
//   B[k][j] = D[4c + k + x_j](Rhat_{d, q_j}) from the d's table in LDS (lane j + 16k)
//   D[i][j] at lane j + 16 (i mod 4), element i / 4.
// The d loop stages the next offset's 8 x ND derivative table in LDS while
// the current one is consumed (one barrier per offset).
// ---------------------------------------------------------------------------
// L2P coefficient of local term b for output o of child q, in the units of
// the M2P accumulators (phi = dx^2/2 acc_phi, g_d = -dx/4 acc_gd):
//   phi:  c_b(q) = (2q-1)^b 4^-|b| / b!
//   g_d:  -4 (1 - 2 q_d) b_d c_b(q)
__device__ __forceinline__ double l2p_coef(int bt, int q, int o) {
  const int ex = c_mi_exp[bt];
  const int x = mi_a(ex), y = mi_b(ex), z = mi_c(ex);
  const int q0 = (q >> 2) & 1, q1 = (q >> 1) & 1, q2 = q & 1;
  double c = ldexp(c_mi_invfact[bt], -2 * (x + y + z));
  if (((1 - q0) * x + (1 - q1) * y + (1 - q2) * z) & 1) c = -c;
  if (o == 1) c *= -4.0 * (1 - 2 * q0) * x;
  if (o == 2) c *= -4.0 * (1 - 2 * q1) * y;
  if (o == 3) c *= -4.0 * (1 - 2 * q2) * z;
  return c;
}

// Near-field coefficient of source offset e (w = 2T + e, e in [-2,3]^3) for
// output o of child q (u = 2T + q), delta = u - w = q - e, in accumulator
// units: phi: -2 / max(|delta|, 1);  g_d: 4 delta_d / |delta|^3 (0 at delta = 0).
__device__ __forceinline__ double p2p_coef(int e0, int e1, int e2, int q, int o) {
  const int t = (((q >> 2) & 1) - e0 + 3) * 49 + (((q >> 1) & 1) - e1 + 3) * 7 + ((q & 1) - e2 + 3);
  return o == 0 ? 2.0 * c_p2p_phi[t] : -4.0 * c_p2p_g[(o - 1) * 343 + t];
}

// L2P from the parent level's local, in the units of the bottom accumulators:
// child rp of the parent, unigrid child q of that cell; w = 2 rp + q - 3/2
// (units of dx) is the offset of the unigrid centre from the parent's centre.
//   phi: 1/2 4^-|b| w^b / b!       g_d: 4^-|b| b_d w^(b-e_d) / b!
__device__ __forceinline__ double l2p_parent_coef(int bt, int rp, int q, int o) {
  const int ex = c_mi_exp[bt];
  const int be[3] = {mi_a(ex), mi_b(ex), mi_c(ex)};
  const double w[3] = {2.0 * ((rp >> 2) & 1) + ((q >> 2) & 1) - 1.5, 2.0 * ((rp >> 1) & 1) + ((q >> 1) & 1) - 1.5,
                       2.0 * (rp & 1) + (q & 1) - 1.5};
  const double base = ldexp(c_mi_invfact[bt], -2 * (be[0] + be[1] + be[2]));
  if (o == 0) {
    double mono = 1.0;
    for (int ax = 0; ax < 3; ++ax)
      for (int z = 0; z < be[ax]; ++z) mono *= w[ax];
    return 0.5 * base * mono;
  }
  const int dax = o - 1;
  if (be[dax] == 0) return 0.0;
  double mono = 1.0;
  for (int ax = 0; ax < 3; ++ax)
    for (int z = 0; z < be[ax] - (ax == dax); ++z) mono *= w[ax];
  return base * be[dax] * mono;
}

// FMM-2 (the finest FMM level two above the unigrid, App. A).  A unigrid
// cell sits at s in {0..3}^3 inside its level-F cell of size h = 4 dx; the
// bottom accumulators are in units of dx^3 / h (phi) and -dx^3 / h^2 (g).
// Position s of child q of the level-(F+1) child grp, along axis ax:
__device__ __forceinline__ int sub_pos(int grp, int q, int ax) {
  return 2 * ((grp >> (2 - ax)) & 1) + ((q >> (2 - ax)) & 1);
}
// Evaluation of a local about a centre at offset -w (units of that local's
// cell size, times the factor f of its scale against level F): phi takes
// f w^b / b!, g_d takes f_g b_d w^(b - e_d) / b!.
__device__ __forceinline__ double l2p_w_coef(int bt, const double (&w)[3], double fphi, double fg, int o) {
  const int ex = c_mi_exp[bt];
  const int be[3] = {mi_a(ex), mi_b(ex), mi_c(ex)};
  const int dax = o - 1;
  if (o > 0 && be[dax] == 0) return 0.0;
  double mono = c_mi_invfact[bt];
  for (int ax = 0; ax < 3; ++ax)
    for (int z = 0; z < be[ax] - (o > 0 && ax == dax); ++z) mono *= w[ax];
  return o == 0 ? fphi * mono : fg * be[dax] * mono;
}
// L2P of the own local: w = (2 s - 3) / 8, the unigrid centre from the
// level-F centre in units of h.
__device__ __forceinline__ double l2p2_coef(int bt, int grp, int q, int o) {
  const double w[3] = {(2 * sub_pos(grp, q, 0) - 3) / 8.0, (2 * sub_pos(grp, q, 1) - 3) / 8.0,
                       (2 * sub_pos(grp, q, 2) - 3) / 8.0};
  return l2p_w_coef(bt, w, 1.0, 1.0, o);
}
// L2P from the parent level's local (cell size 2 h, so phi / 2 and g / 4 in
// the accumulator units): the row's cell is child rp of the parent, and
// w = (s - 3/2 + 4 (rp - 1/2)) / 8 in units of 2 h.
__device__ __forceinline__ double l2p2_parent_coef(int bt, int rp, int grp, int q, int o) {
  double w[3];
  for (int ax = 0; ax < 3; ++ax)
    w[ax] = (sub_pos(grp, q, ax) - 1.5 + 4.0 * (((rp >> (2 - ax)) & 1) - 0.5)) / 8.0;
  return l2p_w_coef(bt, w, 0.5, 0.25, o);
}
// Near-field coefficient of FMM-2 for output o of a target u and a source w,
// delta = u - w (units of dx): eq. (direct) in the accumulator units, phi
// 4 (-1 / max(|delta|, 1)), g_d 16 delta_d / |delta|^3 (0 at delta = 0).
__device__ __forceinline__ double p2p2_delta_coef(int d0, int d1, int d2, int o) {
  const double d[3] = {(double)d0, (double)d1, (double)d2};
  const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (o == 0) return r2 == 0.0 ? -4.0 : -4.0 / sqrt(r2);
  return r2 == 0.0 ? 0.0 : 16.0 * d[o - 1] / (r2 * sqrt(r2));
}
// Near field: source k of the 12^3 block (w = 4 T - 4 + k), target
// u = 4 T + s, delta = u - w = s + 4 - k.
__device__ __forceinline__ double p2p2_coef(int k, int grp, int q, int o) {
  const int kk[3] = {k / 144, (k / 12) % 12, k % 12};
  return p2p2_delta_coef(sub_pos(grp, q, 0) + 4 - kk[0], sub_pos(grp, q, 1) + 4 - kk[1],
                         sub_pos(grp, q, 2) + 4 - kk[2], o);
}

#include "fmm_mfma.h"

// ---------------------------------------------------------------------------
// L2L, eq. (L2L), for one level k: Lhat_k[T] += shift of Lhat_{k-1}[parent(T)]
//   Lhat_k[b] += sum_{|b|+|g|<=p} 2^-(|b|+1) 4^-|g| / g! (2q-1)^g Lhat_{k-1}[b+g]
// in the per-parent column layout.  The child q enters only through the sign
// (2q-1)^g = (-1)^((1-q).g), which depends on the parity pattern of g: with
//   S[b][pat] = sum_{g of pattern pat} 2^-(|b|+1) 4^-|g| / g! Lhat_{k-1}[b+g]
// the 8 children's terms b are a sign transform of S[b][.] (one butterfly
// stage per axis), so each coefficient is applied once instead of 8 times.
// A block takes L2L_ROWS cells P of level k - 1 and stages the coefficient
// lists (CSR over (b, pattern)) and the level-(k-1) local of each P in LDS;
// thread (row r, slot s) forms terms b = s, s + 32, ... of P_r's 8 children.
// A wave holds two rows and 32 consecutive terms of each, so every child
// column it reads or writes is a run of up to 32 consecutive doubles (inside
// a degree block the terms of one child are contiguous).
// ---------------------------------------------------------------------------
// Segments: n = cells per axis of level k - 1, a = Lhat_{k-1}, b = Lhat_k.
constexpr int L2L_THREADS = 512, L2L_SLOTS = L2L_THREADS / L2L_ROWS;
template <int P>
__global__ __launch_bounds__(L2L_THREADS) void k_l2l(const Seg* __restrict__ segs, int nseg, const int* __restrict__ cs,
                                             const int* __restrict__ cidx, const double* __restrict__ ccoef) {
  constexpr int NL = nterms(P), RS = loc_stride(P), E = l2l_entries(P), SS = NL + 1;
  static_assert(L2L_SLOTS == 32, "thread = (row, slot) over 16 rows and 32 slots");
  __shared__ int s_cs[8 * NL + 1];
  __shared__ int s_idx[E];
  __shared__ double s_coef[E];
  __shared__ double s_src[L2L_ROWS * SS];  // odd row stride: the rows start in distinct banks
  const Seg& sg = find_seg(segs, nseg, blockIdx.x);
  const double* __restrict__ Lprev = sg.a;
  double* __restrict__ Lk = sg.b;
  const int ns = sg.n, nsp = ns >> 1;
  const long long nps = (long long)ns * ns * ns;
  const long long P0 = (long long)(blockIdx.x - sg.first_block) * L2L_ROWS;
  for (int t = threadIdx.x; t <= 8 * NL; t += L2L_THREADS) s_cs[t] = cs[t];
  for (int t = threadIdx.x; t < E; t += L2L_THREADS) {
    s_idx[t] = cidx[t];
    s_coef[t] = ccoef[t];
  }
  // P's level-(k-1) local sits in its parent's row, in the column block of
  // P's position qP
  for (int e = threadIdx.x; e < L2L_ROWS * NL; e += L2L_THREADS) {
    const int g = e / NL, c = e - g * NL;
    const long long Pc = P0 + g;
    double v = 0.0;
    if (Pc < nps) {
      const int p2 = (int)(Pc % ns), p1 = (int)((Pc / ns) % ns), p0 = (int)(Pc / ((long long)ns * ns));
      const long long PP = ((long long)(p0 >> 1) * nsp + (p1 >> 1)) * nsp + (p2 >> 1);
      const int qP = ((p0 & 1) << 2) | ((p1 & 1) << 1) | (p2 & 1);
      const int ex = c_mi_exp[c];
      v = Lprev[PP * RS + m2l_col(qP, c, mi_a(ex) + mi_b(ex) + mi_c(ex))];
    }
    s_src[g * SS + c] = v;
  }
  __syncthreads();
  const int slot = threadIdx.x % L2L_SLOTS, r = threadIdx.x / L2L_SLOTS;
  const long long Pc = P0 + r;
  if (Pc >= nps) return;
  double* __restrict__ row = Lk + Pc * RS;
  const double* src = s_src + r * SS;
  for (int b = slot; b < NL; b += L2L_SLOTS) {
    const int ex = c_mi_exp[b];
    const int m = mi_a(ex) + mi_b(ex) + mi_c(ex);
    // the 8 child columns, read before the sums so their loads are in flight
    double out[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) out[q] = row[m2l_col(q, b, m)];
    double S[8];
#pragma unroll
    for (int pat = 0; pat < 8; ++pat) {
      double x = 0.0;
#pragma unroll 2
      for (int j = s_cs[8 * b + pat]; j < s_cs[8 * b + pat + 1]; ++j) x = fma(s_coef[j], src[s_idx[j]], x);
      S[pat] = x;
    }
    // axis bit a: child q with q_a = 0 takes (-1)^g_a, with q_a = 1 takes +1
#pragma unroll
    for (int a = 4; a >= 1; a >>= 1)
#pragma unroll
      for (int x = 0; x < 8; ++x)
        if (!(x & a)) {
          const double u = S[x], w = S[x | a];
          S[x] = u - w;
          S[x | a] = u + w;
        }
#pragma unroll
    for (int q = 0; q < 8; ++q) row[m2l_col(q, b, m)] = out[q] + S[q];
  }
}

// ---------------------------------------------------------------------------
// Adjoint (transpose) of the solve: rho_bar = A^T (phi_bar, g_bar), taking the
// passes in reverse order, each the exact transpose of the forward kernel's
// arithmetic in the scaled representation.  With Ybar_T[(q, o)] the scaled
// adjoint outputs of level-F cell T (q child, o in {phi, gx, gy, gz}):
//   Lam_bar_F = L2P^T Ybar,  Lbar_{F-1} = (parent-level L2P)^T Ybar,
//   Lbar_{k-1} = L2L^T Lbar_k (k = F-1..4),
//   Mbar_{k-1} = M2L^T Lbar_k (k = 3..F),  Mbar_F = M2P^T Ybar   (k_conv),
//   Mbar_k += M2M^T Mbar_{k-1} (k = 3..F),
//   rho_bar = P2M^T Mbar_F + near^T Ybar.
// Adjoint locals are stored as chunked padded grids over the parent cells,
// [loc_stride/4][(ns+6)^3][4] with columns in the M2L order, so the
// transposed M2L stages them like multipoles.
// ---------------------------------------------------------------------------

// Ybar: [8^DL chunks][(nF+6)^3][4]: (sphi phi_bar, sg g_bar_x, sg g_bar_y,
// sg g_bar_z) of each unigrid cell of a level-F cell; chunk q (DL = 1) is
// child q, chunk 8 g + q (DL = 2) is child q of the level-(F+1) child g.
template <typename TI, int DL>
__global__ void k_adj_seed(const TI* __restrict__ dphi, const TI* __restrict__ dg, double* __restrict__ Y, int n,
                           double sphi, double sg) {
  const int nF = n >> DL, nFp = nF + 6;
  const long long nT = (long long)nF * nF * nF, N = (long long)n * n * n;
  const long long T = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (T >= nT) return;
  const int t2 = (int)(T % nF), t1 = (int)((T / nF) % nF), t0 = (int)(T / ((long long)nF * nF));
  const long long ncellp = (long long)nFp * nFp * nFp;
  const long long cp = ((long long)(t0 + 3) * nFp + (t1 + 3)) * nFp + (t2 + 3);
#pragma unroll 8
  for (int q = 0; q < (8 << (3 * (DL - 1))); ++q) {
    const int s0 = DL == 1 ? (q >> 2) & 1 : sub_pos(q >> 3, q & 7, 0);
    const int s1 = DL == 1 ? (q >> 1) & 1 : sub_pos(q >> 3, q & 7, 1);
    const int s2 = DL == 1 ? q & 1 : sub_pos(q >> 3, q & 7, 2);
    const long long u = ((long long)((t0 << DL) + s0) * n + ((t1 << DL) + s1)) * n + ((t2 << DL) + s2);
    d4 v;
    v[0] = sphi * (double)dphi[u];
    v[1] = dg ? sg * (double)dg[u] : 0.0;
    v[2] = dg ? sg * (double)dg[N + u] : 0.0;
    v[3] = dg ? sg * (double)dg[2 * N + u] : 0.0;
    *reinterpret_cast<d4*>(Y + (q * ncellp + cp) * 4) = v;
  }
}

// plan-time coefficient tables of the transposed L2P steps:
//   own [NL][32]:      l2p_coef(b, q, o)               at k = 4 q + o
//   par [8][NL][32]:   l2p_parent_coef(b, rp, q, o)
__global__ void k_adj_coef(double* __restrict__ own, double* __restrict__ par, int NL) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 9 * NL * 32) return;
  const int k = id % 32, b = (id / 32) % NL, z = id / (32 * NL);
  if (z == 0)
    own[b * 32 + k] = l2p_coef(b, k >> 2, k & 3);
  else
    par[((z - 1) * NL + b) * 32 + k] = l2p_parent_coef(b, z - 1, k >> 2, k & 3);
}

// The same for FMM-2, per group g of 8 unigrid cells:
//   own [8][NL][32]:     l2p2_coef(b, g, q, o)
//   par [8][8][NL][32]:  l2p2_parent_coef(b, rp, g, q, o)   ([g][rp])
__global__ void k_adj_coef2(double* __restrict__ own, double* __restrict__ par, int NL) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 72 * NL * 32) return;
  const int k = id % 32, b = (id / 32) % NL, z = id / (32 * NL);
  if (z < 8)
    own[(z * NL + b) * 32 + k] = l2p2_coef(b, z, k >> 2, k & 3);
  else
    par[((size_t)(z - 8) * NL + b) * 32 + k] = l2p2_parent_coef(b, (z - 8) & 7, (z - 8) >> 3, k >> 2, k & 3);
}

// L2P^T and (parent-level L2P)^T on the matrix cores (v_mfma_f64_16x16x4f64).
// Block = 16 level-(F-1) cells P (consecutive in C order) = one row tile.
// The K range of a level-F cell is its 8^DL unigrid cells times (phi, g): one
// group of 32 for DL = 1, eight for DL = 2 (group g = the level-(F+1) child).
// The Ybar of the 8 children of the 16 P (256 values each per group) is staged
// in LDS with an odd row stride, and for each 16-column tile of local terms b
//   own[P][(rp, b)] += sum_k cown[g][b][k] Ybar_g[2P + rp][k]      (K = 32)
//   par[P][b]      += sum_{rp, k} cpar[g][rp][b][k] Ybar_g[2P + rp][k]
// own goes to P's row (columns (rp, b) in the M2L order), par, when the
// parent level has locals, to the row of P's parent (column (qP, b)).
//  - FMM-1 (k_adj_l2p1): wave T takes column tile T and runs the 8 children
//    one after the other, so par accumulates in the wave's own registers in a
//    fixed order and a block needs one barrier (after the staging).
//  - FMM-2 (k_adj_l2p<P, 2>): wave rp (of 8) takes child 2P + rp of every P
//    for all tiles, group by group; the 8 waves' par partials are added in
//    LDS in a fixed order.
constexpr int ADJ_L2P_PAR = 16, ADJ_L2P_THREADS = 512, ADJ_L2P_YS = 257;
template <int P>
__global__ __launch_bounds__(64 * ((nterms(P) + 15) / 16)) void k_adj_l2p1(const double* __restrict__ Y,
                                                                           const double* __restrict__ cown,
                                                                           const double* __restrict__ cpar,
                                                                           double* __restrict__ Aown,
                                                                           double* __restrict__ Apar, int nF) {
  constexpr int NL = nterms(P), RS = loc_stride(P), NBT = (NL + 15) / 16, THREADS = 64 * NBT;
  __shared__ double y[ADJ_L2P_PAR * ADJ_L2P_YS];
  const int nP = nF >> 1, nFp = nF + 6, nPp = nP + 6, nPP = nP >> 1, nPPp = nPP + 6;
  const long long ncF = (long long)nFp * nFp * nFp, ncP = (long long)nPp * nPp * nPp,
                  ncPP = (long long)nPPp * nPPp * nPPp;
  const long long nPc = (long long)nP * nP * nP;
  const long long P0 = (long long)blockIdx.x * ADJ_L2P_PAR;
  const int lane = threadIdx.x & 63;
  const int T = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // the wave's column tile
  const int i = lane & 15, kq = lane >> 4;
  // staging: load l = (q, parent, child), children of consecutive parents are
  // contiguous along z
  for (int l = threadIdx.x; l < 8 * ADJ_L2P_PAR * 8; l += THREADS) {
    const int lr = l & 7, pl = (l >> 3) % ADJ_L2P_PAR, q = l / (8 * ADJ_L2P_PAR);
    const long long Pc = P0 + pl;
    d4 v = d4{0, 0, 0, 0};
    if (Pc < nPc) {
      const int p2 = (int)(Pc % nP), p1 = (int)((Pc / nP) % nP), p0 = (int)(Pc / ((long long)nP * nP));
      const long long cT = ((long long)(2 * p0 + ((lr >> 2) & 1) + 3) * nFp + (2 * p1 + ((lr >> 1) & 1) + 3)) * nFp +
                           (2 * p2 + (lr & 1) + 3);
      v = *reinterpret_cast<const d4*>(Y + (q * ncF + cT) * 4);
    }
    double* yy = y + pl * ADJ_L2P_YS + lr * 32 + q * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) yy[e] = v[e];
  }
  // the lane's output rows 4 v + kq: padded-grid cells of P and of its parent,
  // and P's position in the parent
  long long cpo[4], cpp[4];
  int qP[4];
  bool okr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const long long Pc = P0 + 4 * v + kq;
    okr[v] = Pc < nPc;
    const long long Pq = okr[v] ? Pc : 0;
    const int p2 = (int)(Pq % nP), p1 = (int)((Pq / nP) % nP), p0 = (int)(Pq / ((long long)nP * nP));
    cpo[v] = ((long long)(p0 + 3) * nPp + (p1 + 3)) * nPp + (p2 + 3);
    cpp[v] = ((long long)((p0 >> 1) + 3) * nPPp + ((p1 >> 1) + 3)) * nPPp + ((p2 >> 1) + 3);
    qP[v] = ((p0 & 1) << 2) | ((p1 & 1) << 1) | (p2 & 1);
  }
  // the lane's column (B operand); past the last term the loads read the last
  // column (no branch, so they issue together) and the values become zero
  const int bt = 16 * T + i;
  const bool okc = bt < NL;
  const int btc = okc ? bt : NL - 1;
  const int ex = c_mi_exp[btc];
  const int deg = mi_a(ex) + mi_b(ex) + mi_c(ex);
  double bo[8];
#pragma unroll
  for (int kc = 0; kc < 8; ++kc) {
    const double x = cown[btc * 32 + 4 * kc + kq];
    bo[kc] = okc ? x : 0.0;
  }
  __syncthreads();
  const double* ya = y + i * ADJ_L2P_YS + kq;
  d4 ap = d4{0, 0, 0, 0};
#pragma unroll 1
  for (int rp = 0; rp < 8; ++rp) {
    double bp[8];
#pragma unroll
    for (int kc = 0; kc < 8; ++kc) {
      const double x = cpar[((size_t)rp * NL + btc) * 32 + 4 * kc + kq];
      bp[kc] = okc ? x : 0.0;
    }
    d4 ao = d4{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < 8; ++kc) {
      const double a = ya[rp * 32 + 4 * kc];
      ao = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bo[kc], ao, 0, 0, 0);
      ap = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bp[kc], ap, 0, 0, 0);
    }
    if (okc) {
      const int col = m2l_col(rp, bt, deg);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (okr[v]) Aown[((col >> 2) * ncP + cpo[v]) * 4 + (col & 3)] = ao[v];
    }
  }
  if (Apar && okc)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (okr[v]) {
        const int col = m2l_col(qP[v], bt, deg);
        Apar[((col >> 2) * ncPP + cpp[v]) * 4 + (col & 3)] = ap[v];
      }
  // the padding columns of P's row (past 8 NL) stay zero
  if constexpr (RS > 8 * NL) {
    for (int t = threadIdx.x; t < ADJ_L2P_PAR * (RS - 8 * NL) / 4; t += THREADS) {
      const int pl = t % ADJ_L2P_PAR, cc = 2 * NL + t / ADJ_L2P_PAR;
      const long long Pc = P0 + pl;
      if (Pc >= nPc) continue;
      const int p2 = (int)(Pc % nP), p1 = (int)((Pc / nP) % nP), p0 = (int)(Pc / ((long long)nP * nP));
      const long long cp = ((long long)(p0 + 3) * nPp + (p1 + 3)) * nPp + (p2 + 3);
      *reinterpret_cast<d4*>(Aown + (cc * ncP + cp) * 4) = d4{0, 0, 0, 0};
    }
  }
}
template <int P, int DL>
__global__ __launch_bounds__(ADJ_L2P_THREADS) void k_adj_l2p(const double* __restrict__ Y,
                                                             const double* __restrict__ cown,
                                                             const double* __restrict__ cpar,
                                                             double* __restrict__ Aown, double* __restrict__ Apar,
                                                             int nF) {
  static_assert(DL == 2, "FMM-1 runs k_adj_l2p1");
  constexpr int NL = nterms(P), RS = loc_stride(P), NBT = (NL + 15) / 16, NG = 8;
  __shared__ double y[ADJ_L2P_PAR * ADJ_L2P_YS];
  __shared__ double red[8][16][17];
  const int nP = nF >> 1, nFp = nF + 6, nPp = nP + 6, nPP = nP >> 1, nPPp = nPP + 6;
  const long long ncF = (long long)nFp * nFp * nFp, ncP = (long long)nPp * nPp * nPp,
                  ncPP = (long long)nPPp * nPPp * nPPp;
  const long long nPc = (long long)nP * nP * nP;
  const long long P0 = (long long)blockIdx.x * ADJ_L2P_PAR;
  const int lane = threadIdx.x & 63;
  const int rp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = lane & 15, kq = lane >> 4;
  // padded-grid cells of the lane's output rows 4 v + kq
  long long cpo[4];
  bool okr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const long long Pc = P0 + 4 * v + kq;
    okr[v] = Pc < nPc;
    const long long Pq = okr[v] ? Pc : 0;
    const int p2 = (int)(Pq % nP), p1 = (int)((Pq / nP) % nP), p0 = (int)(Pq / ((long long)nP * nP));
    cpo[v] = ((long long)(p0 + 3) * nPp + (p1 + 3)) * nPp + (p2 + 3);
  }
  const double* ya = y + i * ADJ_L2P_YS + rp * 32 + kq;
  // staging of group g: load l = (q, parent, rp), children of consecutive
  // parents are contiguous along z
  auto stage = [&](int g) {
    for (int l = threadIdx.x; l < 8 * ADJ_L2P_PAR * 8; l += ADJ_L2P_THREADS) {
      const int lr = l & 7, pl = (l >> 3) % ADJ_L2P_PAR, q = l / (8 * ADJ_L2P_PAR);
      const long long Pc = P0 + pl;
      d4 v = d4{0, 0, 0, 0};
      if (Pc < nPc) {
        const int p2 = (int)(Pc % nP), p1 = (int)((Pc / nP) % nP), p0 = (int)(Pc / ((long long)nP * nP));
        const long long cT = ((long long)(2 * p0 + ((lr >> 2) & 1) + 3) * nFp + (2 * p1 + ((lr >> 1) & 1) + 3)) * nFp +
                             (2 * p2 + (lr & 1) + 3);
        v = *reinterpret_cast<const d4*>(Y + ((8 * g + q) * ncF + cT) * 4);
      }
      double* yy = y + pl * ADJ_L2P_YS + lr * 32 + q * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) yy[e] = v[e];
    }
  };
  // tile T's own columns to P's row; the 8 waves' parent partials added in
  // LDS in a fixed order, to the row of P's parent
  auto store = [&](int T, const d4& ao, const d4& ap) {
    const int bt = 16 * T + i;
    if (bt < NL) {
      const int ex = c_mi_exp[bt];
      const int col = m2l_col(rp, bt, mi_a(ex) + mi_b(ex) + mi_c(ex));
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (okr[v]) Aown[((col >> 2) * ncP + cpo[v]) * 4 + (col & 3)] = ao[v];
    }
    if (Apar) {
      __syncthreads();  // the staging buffer / previous reduction is consumed
#pragma unroll
      for (int v = 0; v < 4; ++v) red[rp][4 * v + kq][i] = ap[v];
      __syncthreads();
      if (threadIdx.x < 256) {
        const int row = threadIdx.x >> 4, c = threadIdx.x & 15, b2 = 16 * T + c;
        const long long Pc = P0 + row;
        if (b2 < NL && Pc < nPc) {
          double acc = 0.0;
#pragma unroll
          for (int w = 0; w < 8; ++w) acc += red[w][row][c];
          const int p2 = (int)(Pc % nP), p1 = (int)((Pc / nP) % nP), p0 = (int)(Pc / ((long long)nP * nP));
          const int qP = ((p0 & 1) << 2) | ((p1 & 1) << 1) | (p2 & 1);
          const long long cpp = ((long long)((p0 >> 1) + 3) * nPPp + ((p1 >> 1) + 3)) * nPPp + ((p2 >> 1) + 3);
          const int ex = c_mi_exp[b2];
          const int col = m2l_col(qP, b2, mi_a(ex) + mi_b(ex) + mi_c(ex));
          Apar[((col >> 2) * ncPP + cpp) * 4 + (col & 3)] = acc;
        }
      }
    }
  };
  d4 ao[NBT], ap[NBT];
#pragma unroll
  for (int T = 0; T < NBT; ++T) ao[T] = ap[T] = d4{0, 0, 0, 0};
  for (int g = 0; g < NG; ++g) {
    if (g) __syncthreads();  // the previous group is consumed
    stage(g);
    __syncthreads();
    const double* co = cown + (size_t)g * NL * 32;
    const double* cp = cpar + ((size_t)g * 8 + rp) * NL * 32;
#pragma unroll
    for (int T = 0; T < NBT; ++T) {
      const int bt = 16 * T + i;  // the lane's column (B operand)
      const bool okc = bt < NL;
#pragma unroll
      for (int kc = 0; kc < 8; ++kc) {
        const double a = ya[4 * kc];
        const double bo = okc ? co[bt * 32 + 4 * kc + kq] : 0.0;
        const double bp = okc ? cp[bt * 32 + 4 * kc + kq] : 0.0;
        ao[T] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bo, ao[T], 0, 0, 0);
        ap[T] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bp, ap[T], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int T = 0; T < NBT; ++T) store(T, ao[T], ap[T]);
  // the padding columns of P's row (past 8 NL) stay zero
  if constexpr (RS > 8 * NL) {
    for (int t = threadIdx.x; t < ADJ_L2P_PAR * (RS - 8 * NL) / 4; t += ADJ_L2P_THREADS) {
      const int pl = t % ADJ_L2P_PAR, cc = 2 * NL + t / ADJ_L2P_PAR;
      const long long Pc = P0 + pl;
      if (Pc >= nPc) continue;
      const int p2 = (int)(Pc % nP), p1 = (int)((Pc / nP) % nP), p0 = (int)(Pc / ((long long)nP * nP));
      const long long cp = ((long long)(p0 + 3) * nPp + (p1 + 3)) * nPp + (p2 + 3);
      *reinterpret_cast<d4*>(Aown + (cc * ncP + cp) * 4) = d4{0, 0, 0, 0};
    }
  }
}

// L2L^T for one level k: Lbar_{k-1}[P][b'] = sum_q sum_{b + g = b'}
//   2^-(|b|+1) 4^-|g| / g! (2q-1)^g Lbar_k[2P+q][b].
// P's row of Abar_k holds its 8 children; the result goes to P's parent's
// row of Abar_{k-1}.  The child enters only through the sign
// (2q-1)^g = (-1)^(popc(~q & pat(g))), so with the Walsh sums
//   W[b][pat] = sum_q (-1)^(popc(~q & pat)) Lbar_k[2P+q][b]
// (children taken in reverse order, q' = 7 - q, turn ~q into q') each output
// is sum_{b + g = b'} coef W[b][pat(g)]: the M2M's coefficient lists (over
// b <= b', offset 8 b + pat(g), weight 2^-|b| 4^-|g| / g!) at half weight.
// Block = ADJ_L2L_PAR cells P: their rows are staged in LDS with the lists,
// Walsh-transformed in place (thread (P, b)), then thread (P, b') sums.
constexpr int ADJ_L2L_PAR = 8;
template <int PO>
__global__ __launch_bounds__(256) void k_adj_l2l(const double* __restrict__ Ak, double* __restrict__ Akm1, int ns,
                                                 const int* __restrict__ cstart, const int* __restrict__ coff,
                                                 const double* __restrict__ ccoef) {
  constexpr int NL = nterms(PO), NCH = 2 * NL, WS = 8 * NL + 1;  // NCH: 4-column chunks of a row
  constexpr int NE = (PO + 1) * (PO + 2) * (PO + 3) * (PO + 4) * (PO + 5) * (PO + 6) / 720;
  __shared__ double W[ADJ_L2L_PAR * WS];
  __shared__ int sstart[NL + 1];
  __shared__ int soff[NE];
  __shared__ double scoef[NE];
  const long long nps = (long long)ns * ns * ns;
  const int nsp = ns + 6, nh = ns >> 1, nhp = nh + 6;
  const long long nck = (long long)nsp * nsp * nsp, nckm = (long long)nhp * nhp * nhp;
  const long long P0 = (long long)blockIdx.x * ADJ_L2L_PAR;
  for (int t = threadIdx.x; t <= NL; t += 256) sstart[t] = cstart[t];
  for (int t = threadIdx.x; t < NE; t += 256) {
    soff[t] = coff[t];
    scoef[t] = ccoef[t];
  }
  // the rows: thread (P, column chunk), parents fastest (consecutive cells)
#pragma unroll 2
  for (int l = threadIdx.x; l < ADJ_L2L_PAR * NCH; l += 256) {
    const int pl = l % ADJ_L2L_PAR, cc = l / ADJ_L2L_PAR;
    const long long P = P0 + pl;
    d4 v = d4{0, 0, 0, 0};
    if (P < nps) {
      const int p2 = (int)(P % ns), p1 = (int)((P / ns) % ns), p0 = (int)(P / ((long long)ns * ns));
      const long long cp = ((long long)(p0 + 3) * nsp + (p1 + 3)) * nsp + (p2 + 3);
      v = *reinterpret_cast<const d4*>(Ak + (cc * nck + cp) * 4);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int col = 4 * cc + e, m = m2l_col_degree(col);
      const int cin = col - 8 * nterms(m - 1), q = cin / ndeg(m), b = nterms(m - 1) + cin % ndeg(m);
      W[pl * WS + 8 * b + (7 - q)] = v[e];
    }
  }
  __syncthreads();
#pragma unroll 1
  for (int w = threadIdx.x; w < ADJ_L2L_PAR * NL; w += 256) {
    double* x = W + (w % ADJ_L2L_PAR) * WS + 8 * (w / ADJ_L2L_PAR);
    double y[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) y[q] = x[q];
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (!(q & bit)) {
          const double u = y[q], v = y[q | bit];
          y[q] = u + v;
          y[q | bit] = u - v;
        }
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = y[q];
  }
  __syncthreads();
  for (int w = threadIdx.x; w < ADJ_L2L_PAR * NL; w += 256) {
    const int pl = w % ADJ_L2L_PAR, bt2 = w / ADJ_L2L_PAR;
    const long long P = P0 + pl;
    if (P >= nps) continue;
    const double* Wp = W + pl * WS;
    double acc = 0.0;
    for (int j = sstart[bt2]; j < sstart[bt2 + 1]; ++j) acc += scoef[j] * Wp[soff[j]];
    const int p2 = (int)(P % ns), p1 = (int)((P / ns) % ns), p0 = (int)(P / ((long long)ns * ns));
    const int qP = ((p0 & 1) << 2) | ((p1 & 1) << 1) | (p2 & 1);
    const int ex2 = c_mi_exp[bt2];
    const int col = m2l_col(qP, bt2, mi_a(ex2) + mi_b(ex2) + mi_c(ex2));
    const long long cpp = ((long long)((p0 >> 1) + 3) * nhp + ((p1 >> 1) + 3)) * nhp + ((p2 >> 1) + 3);
    Akm1[((col >> 2) * nckm + cpp) * 4 + (col & 3)] = 0.5 * acc;
  }
}

// M2M^T for one level k: Mbar_k[2P+q][b] += sum_{a >= b}
//   2^-|b| 4^-|g| / g! (-1)^(q.g) Mbar_{k-1}[P][a],  g = a - b.
// Block = 16 cells P of level k - 1 (consecutive in C order), whose adjoint
// multipoles are staged in LDS with the plan's coefficient lists (for each
// (b, parity pattern of g): the entries a = b + g and their weights).  Thread
// (parent, b) forms the 8 pattern sums, then the children by a Walsh
// transform.  Segments are not used: one level per launch.
constexpr int ADJ_M2M_PAR = 16, ADJ_M2M_THREADS = 256;
template <int PO>
__global__ __launch_bounds__(ADJ_M2M_THREADS) void k_adj_m2m(const double* __restrict__ Mp, double* __restrict__ Mc,
                                                             int np, const int* __restrict__ lstart,
                                                             const int* __restrict__ la,
                                                             const double* __restrict__ lcoef, int nmx) {
  constexpr int NM = nterms(PO), NC = (NM + 3) / 4, MS = NM | 1;
  constexpr int NE = (PO + 1) * (PO + 2) * (PO + 3) * (PO + 4) * (PO + 5) * (PO + 6) / 720;
  __shared__ double mrow[ADJ_M2M_PAR * MS];
  __shared__ int sstart[NM * 8 + 1];
  __shared__ int sa[NE];
  __shared__ double scoef[NE];
  const int npp = np + 6, nk = 2 * np, nkp = nk + 6;
  const long long ncp = (long long)npp * npp * npp, nck = (long long)nkp * nkp * nkp;
  const long long nps = (long long)np * np * np;
  const long long P0 = (long long)blockIdx.x * ADJ_M2M_PAR;
  for (int t = threadIdx.x; t <= NM * 8; t += ADJ_M2M_THREADS) sstart[t] = lstart[t];
  for (int t = threadIdx.x; t < NE; t += ADJ_M2M_THREADS) {
    sa[t] = la[t];
    scoef[t] = lcoef[t];
  }
  for (int l = threadIdx.x; l < NC * ADJ_M2M_PAR; l += ADJ_M2M_THREADS) {
    const int pl = l % ADJ_M2M_PAR, c = l / ADJ_M2M_PAR;
    const long long P = P0 + pl;
    d4 v = d4{0, 0, 0, 0};
    if (P < nps) {
      const int p2 = (int)(P % np), p1 = (int)((P / np) % np), p0 = (int)(P / ((long long)np * np));
      const long long cp = ((long long)(p0 + 3) * npp + (p1 + 3)) * npp + (p2 + 3);
      v = *reinterpret_cast<const d4*>(Mp + (c * ncp + cp) * 4);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (4 * c + e < NM) mrow[pl * MS + 4 * c + e] = 4 * c + e < nmx ? v[e] : 0.0;  // transpose of the truncation
  }
  __syncthreads();
  for (int w = threadIdx.x; w < ADJ_M2M_PAR * NM; w += ADJ_M2M_THREADS) {
    const int pl = w % ADJ_M2M_PAR, bt = w / ADJ_M2M_PAR;
    const long long P = P0 + pl;
    if (P >= nps) continue;
    const double* mr = mrow + pl * MS;
    double S[8];
#pragma unroll
    for (int pat = 0; pat < 8; ++pat) {
      double x = 0.0;
      for (int j = sstart[bt * 8 + pat]; j < sstart[bt * 8 + pat + 1]; ++j) x += scoef[j] * mr[sa[j]];
      S[pat] = x;
    }
    const int p2 = (int)(P % np), p1 = (int)((P / np) % np), p0 = (int)(P / ((long long)np * np));
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double v = 0.0;
#pragma unroll
      for (int pat = 0; pat < 8; ++pat) v += (__popc(q & pat) & 1) ? -S[pat] : S[pat];
      const long long cc = ((long long)(2 * p0 + ((q >> 2) & 1) + 3) * nkp + (2 * p1 + ((q >> 1) & 1) + 3)) * nkp +
                           (2 * p2 + (q & 1) + 3);
      Mc[((bt >> 2) * nck + cc) * 4 + (bt & 3)] += v;
    }
  }
}

// P2M^T + near^T for the 8 unigrid children w = 2T + q_w of a level-F cell T:
//   rho_bar[w] = sum_a 4^-|a| / a! (-1)^(q_w.a) Mbar_F[T][a]
//     + sum_{e in [-1,1]^3} sum_{(q,o)} p2p_coef(q_w - 2e, q, o) Ybar_{T+e}[(q,o)].
// Thread = cell T, block = 4 x 4 x TZ cells (TZ = blockDim / 16).  The Ybar
// chunks q (4 values each) of the block's cells and their one-cell halo are
// staged in LDS one chunk at a time, so a block needs little LDS and a CU
// holds many; each neighbour's chunk is read once and applied to all 8
// children.  The stencil weights depend only on (e, q, q_w): constant-memory
// reads at wave-uniform addresses (scalar loads, four weights per offset
// contiguous), so the LDS serves only the staged chunks.  The P2M^T part is
// a Walsh transform of 8 signed sums of the cell's terms.
constexpr int ADJ_BOT_TZ = 16;  // cells along z per block (fewer when the grid is smaller)
template <typename TO>
__global__ __launch_bounds__(16 * ADJ_BOT_TZ) void k_adj_bottom(const double* __restrict__ Mb,
                                                                const double* __restrict__ Y, TO* __restrict__ drho,
                                                                int n, int NM) {
  __shared__ d4 ys[36 * (ADJ_BOT_TZ + 2)];
  const int TZ = blockDim.x >> 4, HZ = TZ + 2, nthr = blockDim.x;
  const int nF = n >> 1, nFp = nF + 6;
  const long long ncellp = (long long)nFp * nFp * nFp;
  const int T0x = blockIdx.x * 4, T0y = blockIdx.y * 4, T0z = blockIdx.z * TZ;
  const int tl2 = threadIdx.x % TZ, tl1 = (threadIdx.x / TZ) & 3, tl0 = threadIdx.x / (4 * TZ);
  double acc[8];
#pragma unroll
  for (int qw = 0; qw < 8; ++qw) acc[qw] = 0.0;
  for (int q = 0; q < 8; ++q) {
    __syncthreads();  // the previous chunk is consumed
    for (int c = threadIdx.x; c < 36 * HZ; c += nthr) {
      const int cz = c % HZ, cy = (c / HZ) % 6, cx = c / (6 * HZ);
      // padded coordinates of T = T0 + (cx, cy, cz) - 1, inside [2, nF + 4)
      const long long cp = ((long long)(T0x + cx + 2) * nFp + (T0y + cy + 2)) * nFp + (T0z + cz + 2);
      ys[c] = *reinterpret_cast<const d4*>(Y + (q * ncellp + cp) * 4);
    }
    __syncthreads();
    // delta = u - w = 2e + q - q_w in [-3, 3]^3: the weights of chunk q start
    // at offset qd, and (unrolled) those of (e, q_w) sit at a constant,
    // non-negative distance from there
    const double* cq = c_p2p_adj + 4 * ((((q >> 2) & 1) * 49) + (((q >> 1) & 1) * 7) + (q & 1));
#pragma unroll
    for (int e = 0; e < 27; ++e) {
      const int e0 = e / 9 - 1, e1 = (e / 3) % 3 - 1, e2 = e % 3 - 1;
      const d4 v = ys[((tl0 + e0 + 1) * 6 + (tl1 + e1 + 1)) * HZ + (tl2 + e2 + 1)];
      const int tb = (2 * e0 + 3) * 49 + (2 * e1 + 3) * 7 + (2 * e2 + 3);
#pragma unroll
      for (int qw = 0; qw < 8; ++qw) {
        const int t = tb - (((qw >> 2) & 1) * 49 + ((qw >> 1) & 1) * 7 + (qw & 1));
        const double* cw = cq + 4 * t;
#pragma unroll
        for (int o = 0; o < 4; ++o) acc[qw] = fma(cw[o], v[o], acc[qw]);
      }
    }
  }
  // P2M^T from the adjoint multipoles of the cell
  const int t0 = T0x + tl0, t1 = T0y + tl1, t2 = T0z + tl2;
  const long long cp = ((long long)(t0 + 3) * nFp + (t1 + 3)) * nFp + (t2 + 3);
  double S[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) S[k] = 0.0;
  for (int c = 0; c < (NM + 3) / 4; ++c) {
    const d4 m = *reinterpret_cast<const d4*>(Mb + (c * ncellp + cp) * 4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int a = 4 * c + e;
      if (a < NM) {
        const int ex = c_mi_exp[a];
        const int ax = mi_a(ex), ay = mi_b(ex), az = mi_c(ex);
        const int pat = ((ax & 1) << 2) | ((ay & 1) << 1) | (az & 1);
        const double x = ldexp(c_mi_invfact[a], -2 * (ax + ay + az)) * m[e];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k == pat) S[k] += x;
      }
    }
  }
#pragma unroll
  for (int qw = 0; qw < 8; ++qw) {
    double v = acc[qw];
#pragma unroll
    for (int pat = 0; pat < 8; ++pat) v += (__popc(qw & pat) & 1) ? -S[pat] : S[pat];
    const long long w = ((long long)(2 * t0 + ((qw >> 2) & 1)) * n + (2 * t1 + ((qw >> 1) & 1))) * n +
                        (2 * t2 + (qw & 1));
    drho[w] = (TO)v;
  }
}

// P2M^T of FMM-2 plus the near-field transpose (computed by k_conv as
// CV_P2PT2 into Near, [16][(nF+6)^3][4], column s = 16 s0 + 4 s1 + s2):
//   rho_bar[4T + s] = Near[T][s] + sum_{|a| <= nmax} w_s^a / a! Mbar_F[T][a],
//   w_s,i = (3 - 2 s_i) / 8,
// the transpose of k_p2m2.  A wave takes one level-F cell T (its Mbar row is
// staged in LDS and read by all lanes at once), lane s one unigrid cell; the
// powers of w are formed as the multi-index loops advance.
template <typename TO>
__global__ __launch_bounds__(256) void k_adj_p2mt2(const double* __restrict__ Mb, const double* __restrict__ Near,
                                                   TO* __restrict__ drho, int n, int NM, int nmx) {
  __shared__ double mrow[4][NTMAX];
  const int nF = n >> 2, nFp = nF + 6;
  const long long ncellp = (long long)nFp * nFp * nFp, nT = (long long)nF * nF * nF;
  const int wv = threadIdx.x >> 6, sl = threadIdx.x & 63;
  const long long T = blockIdx.x * 4LL + wv;
  const bool okT = T < nT;
  const long long Tq = okT ? T : 0;
  const int t2 = (int)(Tq % nF), t1 = (int)((Tq / nF) % nF), t0 = (int)(Tq / ((long long)nF * nF));
  const long long cp = ((long long)(t0 + 3) * nFp + (t1 + 3)) * nFp + (t2 + 3);
  for (int a = sl; a < NM; a += 64) mrow[wv][a] = a < nmx ? Mb[((a >> 2) * ncellp + cp) * 4 + (a & 3)] : 0.0;
  __syncthreads();
  if (!okT) return;
  const int s0 = sl >> 4, s1 = (sl >> 2) & 3, s2 = sl & 3;
  const double w0 = (3 - 2 * s0) / 8.0, w1 = (3 - 2 * s1) / 8.0, w2 = (3 - 2 * s2) / 8.0;
  const int P = mi_degree(nmx - 1);  // nmax (nmx = nterms(nmax) >= 1)
  double acc = Near[((sl >> 2) * ncellp + cp) * 4 + (sl & 3)];
  double px = 1.0;
  for (int ax = 0; ax <= P; ++ax) {
    double py = px;
    for (int ay = 0; ax + ay <= P; ++ay) {
      double pz = py;
      for (int az = 0; ax + ay + az <= P; ++az) {
        const int a = mi_index(ax, ay, az);
        acc += c_mi_invfact[a] * pz * mrow[wv][a];
        pz *= w2;
      }
      py *= w1;
    }
    px *= w0;
  }
  const long long u = ((long long)(4 * t0 + s0) * n + (4 * t1 + s1)) * n + (4 * t2 + s2);
  drho[u] = (TO)acc;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
inline unsigned blocks_for(long long work, int per) { return (unsigned)((work + per - 1) / per); }

// B fragments of one convolution (k_conv) in the compute type
template <typename CT>
hipError_t build_conv_table(fmm_plan* pl, int op, void** out, hipStream_t s) {
  using M = Mf<CT>;
  constexpr int EL = 64 / M::OPM;
  const long long cnt = (long long)conv_nfrags(op, pl->p, M::KC) * conv_nslot(op) * EL * M::VPL;
  hipError_t e = hipMalloc(out, cnt * sizeof(typename M::H));
  if (e != hipSuccess) return e;
  pl->bytes += cnt * sizeof(typename M::H);
  hipLaunchKernelGGL((k_expand_conv<CT>), dim3(blocks_for(cnt, 256)), dim3(256), 0, s, pl->dtab, pl->dtab2,
                     (typename M::H*)*out, op, pl->p, pl->ND);
  return hipGetLastError();
}

// (K chunks, first fragment) of each column tile of a convolution kind in
// the compute type, zero-padded by 16 entries (a group may run past the end)
template <typename CT>
hipError_t build_tile_table(fmm_plan* pl, int op, hipStream_t s) {
  constexpr int X = Mf<CT>::IDX, KC = Mf<CT>::KC;
  if (pl->tiletab[op][X]) return hipSuccess;
  const int nt = conv_ntiles(op, pl->p), nb = 2 * (nt + 16);
  // [nt + 16] (K chunks, first fragment) per column tile, then [nt + 16] the
  // first K chunk from which an FP64 transpose's tile has non-zero B entries
  // only in its first 4 columns (none: its chunk count)
  std::vector<int> h(nb + nt + 16, 0);
  for (int t = 0; t < nt; ++t) {
    h[2 * t] = conv_tile_chunks(op, pl->p, t, KC);
    h[2 * t + 1] = conv_frag_offset(op, pl->p, t, KC);
    // multipoles truncated at nmax: M2L needs only the K chunks of the kept
    // terms; the transposes skip column tiles whose terms are all dropped
    if (op == CV_M2L)
      h[2 * t] = std::min(h[2 * t], (pl->NMX + KC - 1) / KC);
    else if (op != CV_P2PT2 && mi_degree(16 * t) > pl->nmax)
      h[2 * t] = 0;
    // the kernel takes the tiles that have a chunk to be a prefix of the group
    if (t > 0 && h[2 * t] > h[2 * t - 2]) return hipErrorInvalidValue;
    h[nb + t] = h[2 * t];
    if (X == 0 && (op == CV_M2LT || op == CV_M2PT || op == CV_M2PT2))
      for (int c = 0; c < h[2 * t]; ++c) {
        // the tile's columns are multipole terms a, sorted by degree; in the
        // transposed M2L, K chunk c holds local columns of degree >= d, where
        // term a has non-zero entries only if |a| + d <= p; the transposed
        // M2Ps use every term (columns past the last term are padding)
        const int d = op == CV_M2LT ? m2l_col_degree(KC * c) : 0;
        int ncol = 0;
        for (int a = 16 * t; a < 16 * t + 16 && a < nterms(pl->p); ++a) ncol += mi_degree(a) + d <= pl->p;
        if (ncol <= 4) {
          h[nb + t] = c;
          break;
        }
      }
  }
  hipError_t e = hipMalloc(&pl->tiletab[op][X], h.size() * sizeof(int));
  if (e != hipSuccess) return e;
  pl->bytes += h.size() * sizeof(int);
  return hipMemcpyAsync(pl->tiletab[op][X], h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice, s) == hipSuccess
             ? hipStreamSynchronize(s)
             : hipGetLastError();
}

template <typename CT>
hipError_t build_tables_t(fmm_plan* pl, bool bottom, bool m2l, hipStream_t s) {
  using M = Mf<CT>;
  using H = typename M::H;
  constexpr int KC = M::KC, OPM = M::OPM, VPL = M::VPL, EL = 64 / OPM, KT = 4 * VPL, X = M::IDX;
  const int NM = pl->NM, NL = pl->NL;
  const long long NCK = (NM + KC - 1) / KC, NLT = (NL + KT - 1) / KT, NPT = kNearK1 / KT;
  hipError_t e;
  if (bottom && !pl->wm2p[X] && pl->dl == 2) {
    // FMM-2: 8 groups of each table, near field over the 12^3 block
    const long long NPT2 = (1728 + KT - 1) / KT;
    const long long n_m2p = 8 * NCK * NSLOT * 2 * EL * VPL, n_l2p = 8 * NLT * 2 * 64 * VPL,
                    n_p2p = 8 * NPT2 * 2 * 64 * VPL;
    if ((e = hipMalloc(&pl->wm2p[X], n_m2p * sizeof(H))) != hipSuccess) return e;
    if ((e = hipMalloc(&pl->wl2p[X], n_l2p * sizeof(H))) != hipSuccess) return e;
    if ((e = hipMalloc(&pl->wl2p2[X], 8 * n_l2p * sizeof(H))) != hipSuccess) return e;
    if ((e = hipMalloc(&pl->wp2p[X], n_p2p * sizeof(H))) != hipSuccess) return e;
    pl->bytes += (n_m2p + 9 * n_l2p + n_p2p) * sizeof(H);
    const long long cnt = n_m2p + 9 * n_l2p + n_p2p;
    hipLaunchKernelGGL((k_expand_bottom2<CT>), dim3(blocks_for(cnt, 256)), dim3(256), 0, s, pl->dtab2,
                       (H*)pl->wm2p[X], (H*)pl->wl2p[X], (H*)pl->wl2p2[X], (H*)pl->wp2p[X], NM, NL, pl->ND);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (bottom && !pl->wm2p[X]) {
    const long long n_m2p = NCK * NSLOT * 2 * EL * VPL, n_l2p = NLT * 2 * 64 * VPL, n_p2p = NPT * 2 * 64 * VPL;
    if ((e = hipMalloc(&pl->wm2p[X], n_m2p * sizeof(H))) != hipSuccess) return e;
    if ((e = hipMalloc(&pl->wl2p[X], n_l2p * sizeof(H))) != hipSuccess) return e;
    if ((e = hipMalloc(&pl->wl2p2[X], 8 * n_l2p * sizeof(H))) != hipSuccess) return e;
    if ((e = hipMalloc(&pl->wp2p[X], n_p2p * sizeof(H))) != hipSuccess) return e;
    pl->bytes += (n_m2p + 9 * n_l2p + n_p2p) * sizeof(H);
    const long long cnt = n_m2p + 9 * n_l2p + n_p2p;
    hipLaunchKernelGGL((k_expand_bottom<CT>), dim3(blocks_for(cnt, 256)), dim3(256), 0, s, pl->dtab,
                       (H*)pl->wm2p[X], (H*)pl->wl2p[X], (H*)pl->wl2p2[X], (H*)pl->wp2p[X], NM, NL, pl->ND);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (m2l && !pl->wm2l[X]) {
    if ((e = build_conv_table<CT>(pl, CV_M2L, &pl->wm2l[X], s)) != hipSuccess) return e;
    if ((e = build_tile_table<CT>(pl, CV_M2L, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// every launch site's compute type: levels k < m2l_low_from and bottoms of
// fields with F <= coarse_fp64_levels run in FP64
hipError_t tables_all(fmm_plan* pl, hipStream_t s) {
  hipLaunchKernelGGL(k_dtab, dim3(blocks_for(343 * 8, 64)), dim3(64), 0, s, pl->dtab, pl->p + 1, pl->ND);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (pl->dl == 2) {
    hipLaunchKernelGGL(k_dtab2, dim3(blocks_for(343 * 64, 64)), dim3(64), 0, s, pl->dtab2, pl->p + 1, pl->ND);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const bool m2l64 = pl->s_conv[0].nseg > 0, m2llow = pl->s_conv[1].nseg > 0;
  const bool bot64 = pl->s_bot[0][0].nseg > 0, botlow = pl->s_bot[1][0].nseg > 0;
  if ((e = build_tables_t<double>(pl, bot64, m2l64, s)) != hipSuccess) return e;
  if (pl->precision == 1) e = build_tables_t<float>(pl, botlow, m2llow, s);
  if (pl->precision == 2) e = build_tables_t<bf16_tag>(pl, botlow, m2llow, s);
  return e;
}

// Sums the split partial results of each segment of a convolution.
// Segments: count = values per part, split, a = partials, b = result.
__global__ __launch_bounds__(256) void k_split_reduce(const Seg* __restrict__ segs, int nseg) {
  const Seg& sg = find_seg(segs, nseg, blockIdx.x);
  const long long cnt = sg.count;
  const long long x = (long long)(blockIdx.x - sg.first_block) * 256 + threadIdx.x;
  if (x >= cnt) return;
  double v = 0.0;
  for (int s = 0; s < sg.split; ++s) v += sg.a[s * cnt + x];
  sg.b[x] = v;
}

template <int P, typename CT, int OP, int NT>
hipError_t launch_conv_nt(fmm_plan* pl, const SegTable& st, const void* W, hipStream_t s) {
  constexpr int G = (conv_ntiles(OP, P) + NT - 1) / NT;
  StageScope sc(pl, ST_M2L, 1, s);
  const int2* tiles = (const int2*)pl->tiletab[OP][Mf<CT>::IDX];
  const auto* w = (const typename Mf<CT>::H*)W;
  const int* lists = OP == CV_P2PT2 ? pl->dlists_p2p : pl->dlists;
  if (st.cz == 8)
    hipLaunchKernelGGL((k_conv<P, CT, OP, NT, 8>), dim3((unsigned)G * st.blocks), dim3(M2L_THREADS), 0, s, st.dev,
                       st.nseg, st.blocks, tiles, w, lists);
  else
    hipLaunchKernelGGL((k_conv<P, CT, OP, NT, 16>), dim3((unsigned)G * st.blocks), dim3(M2L_THREADS), 0, s, st.dev,
                       st.nseg, st.blocks, tiles, w, lists);
  return hipGetLastError();
}

// One launch per convolution site: every column group of every segment.
template <int P, typename CT, int OP>
hipError_t launch_conv(fmm_plan* pl, const SegTable& st, const void* W, hipStream_t s) {
  if (!st.nseg) return hipSuccess;
  if constexpr (OP == CV_M2L)
    if (pl->tune.grp == 1) return launch_conv_nt<P, CT, OP, ConvGroup<CT, 1>::NT>(pl, st, W, s);
  // the FP64 transposed M2L takes one column tile per block, so every tile's
  // narrow K chunks (4-column products) run as such
  if constexpr (OP == CV_M2LT && Mf<CT>::IDX == 0)
    return launch_conv_nt<P, CT, OP, 1>(pl, st, W, s);
  else
    return launch_conv_nt<P, CT, OP, ConvGroup<CT, 0>::NT>(pl, st, W, s);
}

hipError_t launch_split_reduce(fmm_plan* pl, const SegTable& st, hipStream_t s) {
  if (!st.nseg) return hipSuccess;
  hipLaunchKernelGGL(k_split_reduce, dim3(st.blocks), dim3(256), 0, s, st.dev, st.nseg);
  return hipGetLastError();
}

template <int P>
hipError_t launch_l2l_site(fmm_plan* pl, const SegTable& st, hipStream_t s) {
  if (!st.nseg) return hipSuccess;
  hipLaunchKernelGGL(k_l2l<P>, dim3(st.blocks), dim3(L2L_THREADS), 0, s, st.dev, st.nseg, pl->l2l_start, pl->l2l_idx,
                     pl->l2l_coef);
  return hipGetLastError();
}

template <int P, typename CT, typename TI, typename TO>
hipError_t launch_bottom(fmm_plan* pl, int x, IoArg io, hipStream_t s) {
  using H = typename Mf<CT>::H;
  constexpr int X = Mf<CT>::IDX;
  // the tuned tile depth, or 8 when 16-deep tiles would leave compute units
  // idle (few or small fields at this site, e.g. the FP64 bottoms of the
  // coarse fields of a mixed-precision batch)
  int z = pl->tune.bz == 8 ? 1 : 0;
  if (z == 0 && pl->s_bot[x][0].blocks < pl->cus) z = 1;
  if (pl->force_bz) z = pl->force_bz == 8 ? 1 : 0;  // the caller's choice
  if (pl->dl == 2) z = 0;  // FMM-2 launches 8 blocks per tile
  const SegTable& st = pl->s_bot[x][z];
  if (!st.nseg) return hipSuccess;
  // M2P K chunks: those of the multipole terms kept (nmax)
  const int nck = (pl->NMX + Mf<CT>::KC - 1) / Mf<CT>::KC;
  unsigned int* cnt = pl->stamps ? pl->stamp_cnt : nullptr;
  unsigned long long* done = pl->stamps ? pl->stamp_time + 1 : nullptr;
  StageScope sc(pl, ST_BOTTOM, 1, s);
  if (pl->dl == 2) {
    hipLaunchKernelGGL((k_bottom<P, CT, TI, TO, 16, 2>), dim3(st.blocks, 8), dim3(bottom_threads<CT>()), 0, s, st.dev,
                       st.nseg, io, (const H*)pl->wm2p[X], (const H*)pl->wl2p[X], (const H*)pl->wl2p2[X],
                       (const H*)pl->wp2p[X], pl->dlists, nck, cnt, done);
  } else if (z == 0)
    hipLaunchKernelGGL((k_bottom<P, CT, TI, TO, 16, 1>), dim3(st.blocks), dim3(bottom_threads<CT>()), 0, s, st.dev, st.nseg, io,
                       (const H*)pl->wm2p[X], (const H*)pl->wl2p[X], (const H*)pl->wl2p2[X], (const H*)pl->wp2p[X],
                       pl->dlists, nck, cnt, done);
  else
    hipLaunchKernelGGL((k_bottom<P, CT, TI, TO, 8, 1>), dim3(st.blocks), dim3(bottom_threads<CT>()), 0, s, st.dev, st.nseg, io,
                       (const H*)pl->wm2p[X], (const H*)pl->wl2p[X], (const H*)pl->wl2p2[X], (const H*)pl->wp2p[X],
                       pl->dlists, nck, cnt, done);
  return hipGetLastError();
}

// One solve of every field of the plan.  CT is the compute type of the fine
// levels (double for FP64 plans).
template <int P, typename CT, typename TI, typename TO>
hipError_t solve_ct(fmm_plan* pl, IoArg io, hipStream_t s) {
  hipError_t e;
  if (pl->stamps) {
    const int nf = (int)pl->fld.size();
    hipLaunchKernelGGL(k_stamp_start, dim3(blocks_for(nf, 256)), dim3(256), 0, s, pl->stamp_time, pl->stamp_cnt, nf);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    StageScope sc(pl, ST_P2M, 1, s);
    // terms past nmax are written as zero
    if (pl->dl == 2)
      hipLaunchKernelGGL((k_p2m2<P, TI, CT>), dim3(pl->s_p2m.blocks), dim3(256), 0, s, pl->s_p2m.dev, pl->s_p2m.nseg,
                         io, pl->NMX);
    else
      hipLaunchKernelGGL((k_p2m<P, TI, CT>), dim3(pl->s_p2m.blocks), dim3(256), 0, s, pl->s_p2m.dev, pl->s_p2m.nseg,
                         io, pl->NMX);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (pl->s_p2m2.nseg) {
      hipLaunchKernelGGL((k_p2m2<P, TI, CT>), dim3(pl->s_p2m2.blocks), dim3(256), 0, s, pl->s_p2m2.dev,
                         pl->s_p2m2.nseg, io, pl->NMX);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  for (int k = pl->maxF; k >= 3; --k) {
    const SegTable& st = pl->s_m2m[k];
    if (!st.nseg) continue;
    StageScope sc(pl, ST_M2M, 1, s);
    hipLaunchKernelGGL((k_m2m<P, CT>), dim3(st.blocks), dim3(M2MShape<P>::THREADS), 0, s, st.dev, st.nseg,
                       pl->m2m_start, pl->m2m_off, pl->m2m_coef, pl->NMX);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_conv<P, double, CV_M2L>(pl, pl->s_conv[0], pl->wm2l[0], s)) != hipSuccess) return e;
  if ((e = launch_split_reduce(pl, pl->s_red[0], s)) != hipSuccess) return e;
  if constexpr (!std::is_same<CT, double>::value) {
    if ((e = launch_conv<P, CT, CV_M2L>(pl, pl->s_conv[1], pl->wm2l[Mf<CT>::IDX], s)) != hipSuccess) return e;
    if ((e = launch_split_reduce(pl, pl->s_red[1], s)) != hipSuccess) return e;
  }
  // L2L down to level F - 1 of each field; level F's far field is taken from
  // Lhat_{F-1} directly by the bottom kernel
  for (int k = 4; k <= pl->maxF - 1; ++k) {
    StageScope sc(pl, ST_L2L, pl->s_l2l[k].nseg ? 1 : 0, s);
    if ((e = launch_l2l_site<P>(pl, pl->s_l2l[k], s)) != hipSuccess) return e;
  }
  if ((e = launch_bottom<P, double, TI, TO>(pl, 0, io, s)) != hipSuccess) return e;
  if constexpr (!std::is_same<CT, double>::value)
    if ((e = launch_bottom<P, CT, TI, TO>(pl, 1, io, s)) != hipSuccess) return e;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// adjoint solve (field 0)
// ---------------------------------------------------------------------------
// The transposed M2P, and for FMM-2 the transposed near field, in one
// compute type.
template <typename CT>
hipError_t adjoint_bottom_tables(fmm_plan* pl, hipStream_t s) {
  constexpr int X = Mf<CT>::IDX;
  const int op = pl->dl == 2 ? CV_M2PT2 : CV_M2PT;
  hipError_t e;
  if ((e = build_tile_table<CT>(pl, op, s)) != hipSuccess) return e;
  if ((e = build_conv_table<CT>(pl, op, &pl->wt_m2p[X], s)) != hipSuccess) return e;
  if (pl->dl == 2) {
    if ((e = build_tile_table<CT>(pl, CV_P2PT2, s)) != hipSuccess) return e;
    if ((e = build_conv_table<CT>(pl, CV_P2PT2, &pl->wt_p2p[X], s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t adjoint_tables_all(fmm_plan* pl, hipStream_t s) {
  hipError_t e;
  const int NL = pl->NL;
  if (pl->dl == 2)
    hipLaunchKernelGGL(k_adj_coef2, dim3(blocks_for(72LL * NL * 32, 256)), dim3(256), 0, s, pl->adj_l2p,
                       pl->adj_l2p2, NL);
  else
    hipLaunchKernelGGL(k_adj_coef, dim3(blocks_for(9LL * NL * 32, 256)), dim3(256), 0, s, pl->adj_l2p,
                       pl->adj_l2p2, NL);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the transposed M2L of target levels k < klow runs in FP64, the others in
  // the plan's compute type
  const int klow = m2l_low_from(pl);
  const bool lt64 = pl->F >= 3 && klow > 3, ltlow = pl->F >= klow;
  if (lt64) {
    if ((e = build_conv_table<double>(pl, CV_M2LT, &pl->wt_m2l[0], s)) != hipSuccess) return e;
    if ((e = build_tile_table<double>(pl, CV_M2LT, s)) != hipSuccess) return e;
  }
  if (ltlow) {
    if (pl->precision == 1 && ((e = build_conv_table<float>(pl, CV_M2LT, &pl->wt_m2l[1], s)) != hipSuccess ||
                               (e = build_tile_table<float>(pl, CV_M2LT, s)) != hipSuccess))
      return e;
    if (pl->precision == 2 && ((e = build_conv_table<bf16_tag>(pl, CV_M2LT, &pl->wt_m2l[2], s)) != hipSuccess ||
                               (e = build_tile_table<bf16_tag>(pl, CV_M2LT, s)) != hipSuccess))
      return e;
  }
  if (!bottom_low(pl, pl->F)) return adjoint_bottom_tables<double>(pl, s);
  if (pl->precision == 1) return adjoint_bottom_tables<float>(pl, s);
  return adjoint_bottom_tables<bf16_tag>(pl, s);
}

template <int P, typename CT, typename TI, typename TO>
hipError_t backward_ct(fmm_plan* pl, const AdjWs& w, const TI* dphi, const TI* dg, TO* drho, hipStream_t s) {
  constexpr int NL = nterms(P);
  const int n = pl->n, F = pl->F, dl = pl->dl, nF = n >> dl;
  const double dx = pl->dx;
  hipError_t e;
  const long long nT = (long long)nF * nF * nF;
  // the scale of the bottom accumulators (k_bottom): phi = sphi acc, g = sg acc
  if (dl == 2)
    hipLaunchKernelGGL((k_adj_seed<TI, 2>), dim3(blocks_for(nT, 256)), dim3(256), 0, s, dphi, dg, w.ybar, n,
                       0.25 * dx * dx, -0.0625 * dx);
  else
    hipLaunchKernelGGL((k_adj_seed<TI, 1>), dim3(blocks_for(nT, 256)), dim3(256), 0, s, dphi, dg, w.ybar, n,
                       0.5 * dx * dx, -0.25 * dx);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (F >= 3) {
    // transposed L2P of the own local and of the parent level's local
    const long long nP = nT / 8;
    if (dl == 2)
      hipLaunchKernelGGL((k_adj_l2p<P, 2>), dim3(blocks_for(nP, ADJ_L2P_PAR)), dim3(ADJ_L2P_THREADS), 0, s, w.ybar,
                         pl->adj_l2p, pl->adj_l2p2, w.abar[F], F >= 4 ? w.abar[F - 1] : nullptr, nF);
    else
      hipLaunchKernelGGL((k_adj_l2p1<P>), dim3(blocks_for(nP, ADJ_L2P_PAR)), dim3(64 * ((NL + 15) / 16)), 0, s,
                         w.ybar, pl->adj_l2p, pl->adj_l2p2, w.abar[F], F >= 4 ? w.abar[F - 1] : nullptr, nF);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // transposed L2L chain, fine to coarse
    for (int k = F - 1; k >= 4; --k) {
      const int ns = 1 << (k - 1);
      hipLaunchKernelGGL(k_adj_l2l<P>, dim3(blocks_for((long long)ns * ns * ns, ADJ_L2L_PAR)), dim3(256), 0, s,
                         w.abar[k], w.abar[k - 1], ns, pl->m2m_start, pl->m2m_off, pl->m2m_coef);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // transposed M2L of every target level (sources k - 1 receive)
    if ((e = launch_conv<P, double, CV_M2LT>(pl, w.m2lt[0], pl->wt_m2l[0], s)) != hipSuccess) return e;
    if constexpr (!std::is_same<CT, double>::value)
      if ((e = launch_conv<P, CT, CV_M2LT>(pl, w.m2lt[1], pl->wt_m2l[Mf<CT>::IDX], s)) != hipSuccess) return e;
    if ((e = launch_split_reduce(pl, w.m2lt_red, s)) != hipSuccess) return e;
  }
  // transposed M2P at the finest level (and for FMM-2 the transposed near
  // field, on the same pattern over the 27 adjacent cells)
  const bool low = bottom_low(pl, F);
  if (dl == 2) {
    e = low ? launch_conv<P, CT, CV_M2PT2>(pl, w.m2pt, pl->wt_m2p[Mf<CT>::IDX], s)
            : launch_conv<P, double, CV_M2PT2>(pl, w.m2pt, pl->wt_m2p[0], s);
    if (e == hipSuccess)
      e = low ? launch_conv<P, CT, CV_P2PT2>(pl, w.p2pt, pl->wt_p2p[Mf<CT>::IDX], s)
              : launch_conv<P, double, CV_P2PT2>(pl, w.p2pt, pl->wt_p2p[0], s);
  } else {
    e = low ? launch_conv<P, CT, CV_M2PT>(pl, w.m2pt, pl->wt_m2p[Mf<CT>::IDX], s)
            : launch_conv<P, double, CV_M2PT>(pl, w.m2pt, pl->wt_m2p[0], s);
  }
  if (e != hipSuccess) return e;
  // transposed M2M chain, coarse to fine
  for (int k = 3; k <= F; ++k) {
    const int np = 1 << (k - 1);
    hipLaunchKernelGGL((k_adj_m2m<P>), dim3(blocks_for((long long)np * np * np, ADJ_M2M_PAR)), dim3(ADJ_M2M_THREADS),
                       0, s, (const double*)pl->lev[k - 1].M, (double*)pl->lev[k].M, np, pl->m2mt_start,
                       pl->m2mt_a, pl->m2mt_coef, pl->NMX);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (dl == 2) {
    hipLaunchKernelGGL((k_adj_p2mt2<TO>), dim3(blocks_for(nT, 4)), dim3(256), 0, s, (const double*)pl->lev[F].M,
                       w.near, drho, n, pl->NM, pl->NMX);
    return hipGetLastError();
  }
  // nF is a power of two >= 4: the block's z extent divides it
  const int tz = nF < ADJ_BOT_TZ ? nF : ADJ_BOT_TZ;
  dim3 bgrid(nF / 4, nF / 4, nF / tz);
  hipLaunchKernelGGL((k_adj_bottom<TO>), bgrid, dim3(16 * tz), 0, s, (const double*)pl->lev[F].M, w.ybar, drho, n,
                     pl->NMX);
  return hipGetLastError();
}

template <typename T>
__global__ void k_check_finite(const T* __restrict__ x, long long count, int* flag) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < count && !isfinite((double)x[i])) atomicOr(flag, 1);
}

}  // namespace

// ---------------------------------------------------------------------------
// the order's entry points
// ---------------------------------------------------------------------------
template <int P>
hipError_t Impl<P>::upload_constants() {
  return upload_constants_tu();
}

template <int P>
hipError_t Impl<P>::tables(fmm_plan* pl, hipStream_t s) {
  return tables_all(pl, s);
}

template <int P>
hipError_t Impl<P>::solve(fmm_plan* pl, IoArg io, hipStream_t s) {
  switch (pl->precision) {
    case 0: return solve_ct<P, double, double, double>(pl, io, s);
    case 1: return solve_ct<P, float, float, float>(pl, io, s);
    case 2: return solve_ct<P, bf16_tag, float, float>(pl, io, s);
  }
  return hipErrorInvalidValue;
}

template <int P>
hipError_t Impl<P>::backward(fmm_plan* pl, const AdjWs& w, const void* dphi, const void* dg, void* drho,
                             hipStream_t s) {
  switch (pl->precision) {
    case 0: return backward_ct<P, double>(pl, w, (const double*)dphi, (const double*)dg, (double*)drho, s);
    case 1: return backward_ct<P, float>(pl, w, (const float*)dphi, (const float*)dg, (float*)drho, s);
    case 2: return backward_ct<P, bf16_tag>(pl, w, (const float*)dphi, (const float*)dg, (float*)drho, s);
  }
  return hipErrorInvalidValue;
}

template <int P>
hipError_t Impl<P>::adjoint_tables(fmm_plan* pl, hipStream_t s) {
  return adjoint_tables_all(pl, s);
}

// L2L into the finest level of field 0 (the solve leaves Lam_F without it)
template <int P>
hipError_t Impl<P>::finish_locals(fmm_plan* pl, int level, hipStream_t s) {
  if (level < 4 || level != pl->F) return hipSuccess;
  Seg sg{};
  sg.first_block = 0;
  sg.n = 1 << (level - 1);
  sg.a = (const double*)pl->lev[level - 1].L;
  sg.b = (double*)pl->lev[level].L;
  Seg* dev = nullptr;
  hipError_t e = hipMalloc(&dev, sizeof(Seg));
  if (e != hipSuccess) return e;
  if ((e = hipMemcpy(dev, &sg, sizeof(Seg), hipMemcpyHostToDevice)) == hipSuccess) {
    SegTable st;
    st.dev = dev;
    st.nseg = 1;
    st.blocks = (int)blocks_for((long long)sg.n * sg.n * sg.n, L2L_ROWS);
    e = launch_l2l_site<P>(pl, st, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  (void)hipFree(dev);
  return e;
}

template <int P>
hipError_t Impl<P>::check_finite(fmm_plan* pl, const void* rho, int* host_flag, hipStream_t s) {
  const long long N = (long long)pl->n * pl->n * pl->n;
  hipError_t e = hipMemsetAsync(pl->flag, 0, sizeof(int), s);
  if (e != hipSuccess) return e;
  if (pl->precision == 0)
    hipLaunchKernelGGL((k_check_finite<double>), dim3(blocks_for(N, 256)), dim3(256), 0, s, (const double*)rho, N, pl->flag);
  else
    hipLaunchKernelGGL((k_check_finite<float>), dim3(blocks_for(N, 256)), dim3(256), 0, s, (const float*)rho, N, pl->flag);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(host_flag, pl->flag, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace fmm
