// HIP kernels of the unigrid FMM solve for MI355X (gfx950).
//
// Pass order of one solve (Sec. 2 of the paper):
//   k_p2m            rho -> Mhat_F                       eq. (multipole)
//   k_m2m            Mhat_k -> Mhat_{k-1}, k = F..3      eq. (M2M)
//   k_m2l_f64        Mhat_{k-1}, Lhat_{k-1} -> Lhat_k    eq. (M2L) over the oct-shared lists
//                                                        (Sec. 2.2) + eq. (L2L) from the parent
//   k_m2p_f64        Mhat_F, Lhat_F, rho -> phi, g       M2P at the unigrid centres (Sec. 4),
//                                                        L2P and the near field, eq. (direct)
//
// Layouts: multipoles and locals are "chunked", [ceil(terms/4)][cells][4], so
// that a matrix-core operand fragment (4 consecutive terms of one cell) is one
// 32-byte load and cells of a z line are contiguous.  Multipole grids carry a
// zero halo of 3 cells per side: the clipped interaction lists of the isolated
// boundary then need no bounds checks.
#include "fmm_internal.h"

#include <cmath>
#include <vector>

namespace fmm {

typedef double d4 __attribute__((ext_vector_type(4)));

// multi-index table for orders <= PDMAX: packed exponents a | b<<8 | c<<16,
// and 1/a!
__constant__ int c_mi_exp[NTMAX];
__constant__ double c_mi_invfact[NTMAX];
// near-field stencil in grid units, offset delta = u - w in [-3,3]^3:
//   c_p2p_phi = -1/max(|delta|, 1),  c_p2p_g = -delta/|delta|^3 (0 at delta = 0)
__constant__ double c_p2p_phi[343];
__constant__ double c_p2p_g[3 * 343];

__device__ __forceinline__ int mi_a(int e) { return e & 255; }
__device__ __forceinline__ int mi_b(int e) { return (e >> 8) & 255; }
__device__ __forceinline__ int mi_c(int e) { return (e >> 16) & 255; }

hipError_t upload_constants() {
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
  double pp[343], pg[3 * 343];
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
  }
  hipError_t e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_mi_exp), ex, sizeof(ex))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_mi_invfact), inv, sizeof(inv))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_p2p_phi), pp, sizeof(pp))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_p2p_g), pg, sizeof(pg))) != hipSuccess) return e;
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
__global__ void k_dtab(double* __restrict__ out, int PD, int ND) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 343 * 8) return;
  const int dd = t >> 3, q = t & 7;
  const double R0 = double(dd / 49 - 3) + (((q >> 2) & 1) ? 0.25 : -0.25);
  const double R1 = double((dd / 7) % 7 - 3) + (((q >> 1) & 1) ? 0.25 : -0.25);
  const double R2 = double(dd % 7 - 3) + ((q & 1) ? 0.25 : -0.25);
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
  for (int i = 0; i < ND; ++i) out[(size_t)t * ND + i] = -f[i];
}

__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, long long count) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < count) out[i] = (float)in[i];
}

// ---------------------------------------------------------------------------
// P2M: Mhat_F[a] = sum_q rho_{2T+q} (s_q/4)^a / a!,  s_q,i = 1 - 2 q_i.
// (-1)^(q.a) depends on a only through a mod 2, so the 8 signed sums of the
// children are formed once (a Walsh transform) and each term is one product.
// ---------------------------------------------------------------------------
template <typename TI>
__global__ void k_p2m(const TI* __restrict__ rho, double* __restrict__ M, int n, int NM, int NC) {
  const int nF = n >> 1, nFp = nF + 6;
  const long long nT = (long long)nF * nF * nF;
  const long long T = blockIdx.x * (long long)blockDim.x + threadIdx.x;
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
  for (int c = 0; c < NC; ++c) {
    d4 o;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int al = 4 * c + e;
      double val = 0.0;
      if (al < NM) {
        const int ex = c_mi_exp[al];
        const int a = mi_a(ex), b = mi_b(ex), cc = mi_c(ex);
        const int pat = ((a & 1) << 2) | ((b & 1) << 1) | (cc & 1);
        val = ldexp(c_mi_invfact[al], -2 * (a + b + cc)) * S[pat];
      }
      o[e] = val;
    }
    *reinterpret_cast<d4*>(M + (c * ncellp + cp) * 4) = o;
  }
}

// ---------------------------------------------------------------------------
// M2M: Mhat_{k-1}[a] = sum_q sum_{b<=a} 2^-|b| 4^-|g| / g! (-1)^(q.g) Mhat_k[2P+q][b],
// g = a - b.  Block = 4 parents; the Walsh sums of the 8 children per term
// are staged in LDS, then each thread forms terms.
// ---------------------------------------------------------------------------
template <int NMX>
__global__ __launch_bounds__(256) void k_m2m(const double* __restrict__ Mc, double* __restrict__ Mp, int nk, int NM, int NC) {
  __shared__ double W[4][NMX][8];
  const int np = nk >> 1, nkp = nk + 6, npp = np + 6;
  const long long ncp_c = (long long)nkp * nkp * nkp, ncp_p = (long long)npp * npp * npp;
  const long long nP = (long long)np * np * np;
  const long long P0 = (long long)blockIdx.x * 4;
  // phase 1: Walsh sums
  for (int w = threadIdx.x; w < 4 * NM; w += blockDim.x) {
    const int pl = w / NM, b = w % NM;
    const long long P = P0 + pl;
    double v[8];
    if (P < nP) {
      const int p2 = (int)(P % np), p1 = (int)((P / np) % np), p0 = (int)(P / ((long long)np * np));
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const long long cc = ((long long)(2 * p0 + ((q >> 2) & 1) + 3) * nkp + (2 * p1 + ((q >> 1) & 1) + 3)) * nkp +
                             (2 * p2 + (q & 1) + 3);
        v[q] = Mc[((b >> 2) * ncp_c + cc) * 4 + (b & 3)];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = 0.0;
    }
#pragma unroll
    for (int pat = 0; pat < 8; ++pat) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) s += (__popc(q & pat) & 1) ? -v[q] : v[q];
      W[pl][b][pat] = s;
    }
  }
  __syncthreads();
  // phase 2: terms
  for (int w = threadIdx.x; w < 4 * NC * 4; w += blockDim.x) {
    const int pl = w / (NC * 4), al = w % (NC * 4);
    const long long P = P0 + pl;
    if (P >= nP) continue;
    double acc = 0.0;
    if (al < NM) {
      const int ex = c_mi_exp[al];
      const int a = mi_a(ex), b = mi_b(ex), c = mi_c(ex);
      for (int x = 0; x <= a; ++x)
        for (int y = 0; y <= b; ++y)
          for (int z = 0; z <= c; ++z) {
            const int gx = a - x, gy = b - y, gz = c - z;
            const int be = mi_index(x, y, z), ge = mi_index(gx, gy, gz);
            const int pat = ((gx & 1) << 2) | ((gy & 1) << 1) | (gz & 1);
            acc += ldexp(c_mi_invfact[ge], -(x + y + z) - 2 * (gx + gy + gz)) * W[pl][be][pat];
          }
    }
    const int p2 = (int)(P % np), p1 = (int)((P / np) % np), p0 = (int)(P / ((long long)np * np));
    const long long cp = ((long long)(p0 + 3) * npp + (p1 + 3)) * npp + (p2 + 3);
    Mp[((al >> 2) * ncp_p + cp) * 4 + (al & 3)] = acc;
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
// L2L, eq. (L2L), in scaled form for child q of parent P:
//   Lhat_k[b] += sum_{|b|+|g|<=p} 2^-(|b|+1) 4^-|g| / g! (2q-1)^g Lhat_{k-1}[P][b+g]
template <int P>
__device__ __forceinline__ double l2l_term(const double* __restrict__ Lp, long long ncp, long long Pl, int q, int bx,
                                           int by, int bz, int m) {
  const int q0 = (q >> 2) & 1, q1 = (q >> 1) & 1, q2 = q & 1;
  double acc = 0.0;
  for (int gx = 0; gx <= P - m; ++gx)
    for (int gy = 0; gx + gy <= P - m; ++gy)
      for (int gz = 0; gx + gy + gz <= P - m; ++gz) {
        const int bt = mi_index(bx + gx, by + gy, bz + gz);
        double c = ldexp(c_mi_invfact[mi_index(gx, gy, gz)], -2 * (gx + gy + gz)) *
                   Lp[((bt >> 2) * ncp + Pl) * 4 + (bt & 3)];
        if (((1 - q0) * gx + (1 - q1) * gy + (1 - q2) * gz) & 1) c = -c;
        acc += c;
      }
  return ldexp(acc, -(m + 1));
}

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

struct RowCtx {
  long long cell;  // padded linear index in the source grid
  int c0, c1, c2;  // cell coordinates (unpadded)
  bool valid;
};

__device__ __forceinline__ RowCtx row_of(long long gl, long long nlat, int nG, int r, int nsp) {
  RowCtx rc;
  rc.valid = gl < nlat;
  const long long g = rc.valid ? gl : 0;
  const int G2 = (int)(g % nG), G1 = (int)((g / nG) % nG), G0 = (int)(g / ((long long)nG * nG));
  rc.c0 = 2 * G0 + ((r >> 2) & 1);
  rc.c1 = 2 * G1 + ((r >> 1) & 1);
  rc.c2 = 2 * G2 + (r & 1);
  rc.cell = ((long long)(rc.c0 + 3) * nsp + (rc.c1 + 3)) * nsp + (rc.c2 + 3);
  return rc;
}

template <int ND>
__device__ __forceinline__ void stage_load(const double* __restrict__ src, double (&buf)[(8 * ND + 255) / 256]) {
#pragma unroll
  for (int s = 0; s < (8 * ND + 255) / 256; ++s) {
    const int e = threadIdx.x + 256 * s;
    buf[s] = (e < 8 * ND) ? src[e] : 0.0;
  }
}
template <int ND>
__device__ __forceinline__ void stage_store(double* dst, const double (&buf)[(8 * ND + 255) / 256]) {
#pragma unroll
  for (int s = 0; s < (8 * ND + 255) / 256; ++s) {
    const int e = threadIdx.x + 256 * s;
    if (e < 8 * ND) dst[e] = buf[s];
  }
}

// Bottom of the downward pass for the unigrid children of level-F cells:
// columns (q, o), o in {phi, gx, gy, gz}; 32 columns = 2 tiles.  After the
// 189 M2P offsets, two more K blocks run on the matrix cores: L2P (K = local
// terms of the row's own cell) and the near field (K = the 216 unigrid
// densities of the 6^3 block around the row's cell).  phi and g are written
// once.
//
// Data flow: a block owns a tile of BX x BY x BZ level-F cells (all 8 parity
// classes, one wave per class).  For each chunk of 4 multipole terms the
// block stages the multipoles of the tile plus its 3-cell halo in LDS, z
// de-interleaved by parity so that the 16 rows of a fragment (8 z-neighbours
// of one parity x 2 y lines) are two contiguous 256-byte runs.  Every staged
// value then feeds up to 189 x 8 matrix-core ops without touching L2.  The B
// fragments (derivative tables, plan-time fragment order) come from global
// memory and are prefetched one offset ahead.
constexpr int BX = 8, BY = 8, BZ = 16;
constexpr int HX = BX + 6, HY = BY + 6, HZ = BZ + 6, HZ2 = HZ / 2;
constexpr int BOT_MT = (BX / 2) * (BY / 2) * (BZ / 2) / 16;  // row tiles per wave (8)
constexpr int BOT_THREADS = 512;

__device__ __forceinline__ int halo_index(int hx, int hy, int hz) {
  return (((hx * HY + hy) * 2 + (hz & 1)) * HZ2 + (hz >> 1));
}

template <int P, typename TI, typename TO>
__global__ __launch_bounds__(BOT_THREADS, 1) void k_bottom_f64(
    const double* __restrict__ Mh, const double* __restrict__ Lf, const double* __restrict__ Lpar,
    const TI* __restrict__ rho, const double* __restrict__ Wm2p, const double* __restrict__ Wl2p,
    const double* __restrict__ Wl2p2, const double* __restrict__ Wp2p, const int* __restrict__ dlists,
    TO* __restrict__ phi, TO* __restrict__ g, int nF, double sphi, double sg) {
  constexpr int NM = nterms(P), NC = (NM + 3) / 4;
  constexpr int NL = nterms(P), NCL = (NL + 3) / 4;
  __shared__ d4 halo[HX * HY * HZ];
  const int lane = threadIdx.x & 63;
  const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave = parity class (uniform)
  const int i = lane & 15, kq = lane >> 4;
  const int r0 = (r >> 2) & 1, r1 = (r >> 1) & 1, r2 = r & 1;
  const int nFp = nF + 6;
  const long long ncellp = (long long)nFp * nFp * nFp;
  const int tx0 = blockIdx.x * BX, ty0 = blockIdx.y * BY, tz0 = blockIdx.z * BZ;
  // row i of tile m: lattice (gx, gy, gz) = (m >> 1, 2 (m & 1) + (i >> 3), i & 7)
  const int gz = i & 7, gyo = i >> 3;

  d4 acc[BOT_MT][2];
#pragma unroll
  for (int m = 0; m < BOT_MT; ++m) acc[m][0] = acc[m][1] = d4{0, 0, 0, 0};
  const int* dl = dlists + r * NLIST;

  for (int c = 0; c < NC; ++c) {
    __syncthreads();  // previous chunk fully consumed
    for (int h = threadIdx.x; h < HX * HY * HZ; h += BOT_THREADS) {
      const int hz = h % HZ, hy = (h / HZ) % HY, hx = h / (HZ * HY);
      const int px = tx0 + hx, py = ty0 + hy, pz = tz0 + hz;  // padded coordinates
      d4 v = d4{0, 0, 0, 0};
      if (px < nFp && py < nFp && pz < nFp)
        v = *reinterpret_cast<const d4*>(Mh + (c * ncellp + ((long long)px * nFp + py) * nFp + pz) * 4);
      halo[halo_index(hx, hy, hz)] = v;
    }
    __syncthreads();
    const double* hal = reinterpret_cast<const double*>(halo);
    const double* wc = Wm2p + (size_t)c * (343 * 128) + lane;
    // B fragments of offsets it and it + 1 in flight; blocks start at
    // different offsets so that they do not request the same fragment at once
    const int rot = (int)(((blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)) * 37u) % NLIST);
    auto dl_at = [&](int j) { j += rot; return dl[j < NLIST ? j : j - NLIST]; };
    double b0 = wc[(size_t)dl_at(0) * 128], b1 = wc[(size_t)dl_at(0) * 128 + 64];
    double n0 = wc[(size_t)dl_at(1) * 128], n1 = wc[(size_t)dl_at(1) * 128 + 64];
    for (int it = 0; it < NLIST; ++it) {
      const int dd = dl_at(it);
      const int d0 = dd / 49 - 3, d1 = (dd / 7) % 7 - 3, d2 = dd % 7 - 3;
      const double cb0 = b0, cb1 = b1;
      b0 = n0;
      b1 = n1;
      if (it + 2 < NLIST) {
        const int dn = dl_at(it + 2);
        n0 = wc[(size_t)dn * 128];
        n1 = wc[(size_t)dn * 128 + 64];
      }
      // source halo coordinates of row (gx, gy, gz): 3 + 2 g + r - d
      const int zz = 3 + r2 - d2;  // in [1, 6]
      const int zoff = (zz & 1) * HZ2 + gz + (zz >> 1);
#pragma unroll
      for (int m = 0; m < BOT_MT; ++m) {
        const int hx = 3 + 2 * (m >> 1) + r0 - d0;
        const int hy = 3 + 2 * (2 * (m & 1) + gyo) + r1 - d1;
        const double a = hal[((hx * HY + hy) * 2 * HZ2 + zoff) * 4 + kq];
        acc[m][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, cb0, acc[m][0], 0, 0, 0);
        acc[m][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, cb1, acc[m][1], 0, 0, 0);
      }
    }
  }

  const int n = 2 * nF;
  const long long N = (long long)n * n * n;
#pragma unroll
  for (int m = 0; m < BOT_MT; ++m) {
    // the lane's own row (A operand) and its level-F cell, clamped into the grid
    int c0 = tx0 + 2 * (m >> 1) + r0, c1 = ty0 + 2 * (2 * (m & 1) + gyo) + r1, c2 = tz0 + 2 * gz + r2;
    c0 = c0 < nF ? c0 : 0;
    c1 = c1 < nF ? c1 : 0;
    c2 = c2 < nF ? c2 : 0;
    // L2P of the M2L part of the row's own local (stored with its parent P')
    // and of the parent level's full local, evaluated at the unigrid centres
    // (L2L followed by L2P as one exact polynomial evaluation; its B operand
    // depends on the row's parity class r inside P')
    if (Lf) {
      constexpr int RS = loc_stride(P);
      const int nP = nF >> 1;
      const long long Pp = ((long long)(c0 >> 1) * nP + (c1 >> 1)) * nP + (c2 >> 1);
      const double* own = Lf + Pp * RS;
      const double* par = nullptr;
      int qP = 0;
      if (Lpar) {
        const int nPP = nP >> 1;
        const long long PP = ((long long)(c0 >> 2) * nPP + (c1 >> 2)) * nPP + (c2 >> 2);
        par = Lpar + PP * RS;
        qP = (((c0 >> 1) & 1) << 2) | (((c1 >> 1) & 1) << 1) | ((c2 >> 1) & 1);
      }
      const double* w2 = Wl2p2 + (size_t)r * NCL * 128 + lane;
#pragma unroll 1
      for (int c = 0; c < NCL; ++c) {
        const int bt = 4 * c + kq;
        double a = 0.0, ap = 0.0;
        if (bt < NL) {
          const int ex = c_mi_exp[bt];
          const int md = mi_a(ex) + mi_b(ex) + mi_c(ex);
          a = own[m2l_col(r, bt, md)];
          if (par) ap = par[m2l_col(qP, bt, md)];
        }
        acc[m][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Wl2p[c * 128 + lane], acc[m][0], 0, 0, 0);
        acc[m][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Wl2p[c * 128 + 64 + lane], acc[m][1], 0, 0, 0);
        if (par) {
          acc[m][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap, w2[c * 128], acc[m][0], 0, 0, 0);
          acc[m][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap, w2[c * 128 + 64], acc[m][1], 0, 0, 0);
        }
      }
    }
#pragma unroll 1
    for (int c = 0; c < 54; ++c) {
      const int k = 4 * c + kq;
      const int e0 = k / 36 - 2, e1 = (k / 6) % 6 - 2, e2 = k % 6 - 2;
      const int w0 = 2 * c0 + e0, w1 = 2 * c1 + e1, w2 = 2 * c2 + e2;
      const bool in = w0 >= 0 && w1 >= 0 && w2 >= 0 && w0 < n && w1 < n && w2 < n;
      const double a = in ? (double)rho[((long long)w0 * n + w1) * n + w2] : 0.0;
      acc[m][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Wp2p[c * 128 + lane], acc[m][0], 0, 0, 0);
      acc[m][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Wp2p[c * 128 + 64 + lane], acc[m][1], 0, 0, 0);
    }
    // epilogue (f64 layout): element v of tile t is row 4v + kq, column 16t + i
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * v + kq;
      const int o0 = tx0 + 2 * (m >> 1) + r0, o1 = ty0 + 2 * (2 * (m & 1) + (row >> 3)) + r1,
                o2 = tz0 + 2 * (row & 7) + r2;
      if (o0 >= nF || o1 >= nF || o2 >= nF) continue;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int col = 16 * t + i;
        const int q = col >> 2, o = col & 3;
        const long long u = ((long long)(2 * o0 + ((q >> 2) & 1)) * n + (2 * o1 + ((q >> 1) & 1))) * n +
                            (2 * o2 + (q & 1));
        const double val = acc[m][t][v];
        if (o == 0)
          phi[u] = (TO)(sphi * val);
        else if (g)
          g[(o - 1) * N + u] = (TO)(sg * val);
      }
    }
  }
}

// Plan-time expansion of the bottom kernel's B operands into fragment order:
// table[chunk][tile][lane], lane = j + 16 k holds B[k][j] of column 16 tile + j.
//   M2P:  [NC][343 offsets][2][64]  D[a + e_o](Rhat_{d,q}), a = 4 chunk + k (0 past NM)
//   L2P:  [NCL][2][64]              l2p_coef
//   near: [54][2][64]               p2p_coef, source e = decode(4 chunk + k)
__global__ void k_expand_bottom(const double* __restrict__ Dtab, double* __restrict__ Wm2p,
                                double* __restrict__ Wl2p, double* __restrict__ Wp2p, double* __restrict__ Wl2p2,
                                int NM, int NC, int NL, int NCL, int ND) {
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long n_m2p = 343LL * NC * 128, n_l2p = (long long)NCL * 128, n_p2p = 54 * 128;
  const long long n_l2p2 = 8LL * NCL * 128;
  if (id >= n_m2p + n_l2p + n_p2p + n_l2p2) return;
  long long e = id;
  const int lane = (int)(e & 63), t = (int)((e >> 6) & 1);
  const int j = lane & 15, k = lane >> 4;
  const int col = 16 * t + j, q = col >> 2, o = col & 3;
  if (e < n_m2p) {
    const int dd = (int)((e >> 7) % 343), c = (int)((e >> 7) / 343);
    const int al = 4 * c + k;
    double v = 0.0;
    if (al < NM) {
      const int ex = c_mi_exp[al];
      v = Dtab[((size_t)dd * 8 + q) * ND + mi_index(mi_a(ex) + (o == 1), mi_b(ex) + (o == 2), mi_c(ex) + (o == 3))];
    }
    Wm2p[e] = v;
    return;
  }
  e -= n_m2p;
  if (e < n_l2p) {
    const int c = (int)(e >> 7);
    const int bt = 4 * c + k;
    Wl2p[e] = bt < NL ? l2p_coef(bt, q, o) : 0.0;
    return;
  }
  e -= n_l2p;
  if (e < n_p2p) {
    const int c = (int)(e >> 7);
    const int kk = 4 * c + k;
    Wp2p[e] = p2p_coef(kk / 36 - 2, (kk / 6) % 6 - 2, kk % 6 - 2, q, o);
    return;
  }
  e -= n_p2p;
  {
    // parent-level L2P: child rp of the parent, unigrid child q of that cell;
    // w = 2 rp + q - 3/2 (units of dx) is the offset of the unigrid centre from
    // the parent's centre.  phi: 1/2 4^-|b| w^b / b!;  g_d: 4^-|b| b_d w^(b-e_d) / b!
    const int rp = (int)(e / (NCL * 128)), c = (int)((e >> 7) % NCL);
    const int bt = 4 * c + k;
    double v = 0.0;
    if (bt < NL) {
      const int ex = c_mi_exp[bt];
      const int be[3] = {mi_a(ex), mi_b(ex), mi_c(ex)};
      const double w[3] = {2.0 * ((rp >> 2) & 1) + ((q >> 2) & 1) - 1.5, 2.0 * ((rp >> 1) & 1) + ((q >> 1) & 1) - 1.5,
                           2.0 * (rp & 1) + (q & 1) - 1.5};
      const double base = ldexp(c_mi_invfact[bt], -2 * (be[0] + be[1] + be[2]));
      if (o == 0) {
        double mono = 1.0;
        for (int ax = 0; ax < 3; ++ax)
          for (int z = 0; z < be[ax]; ++z) mono *= w[ax];
        v = 0.5 * base * mono;
      } else {
        const int dax = o - 1;
        if (be[dax] > 0) {
          double mono = 1.0;
          for (int ax = 0; ax < 3; ++ax)
            for (int z = 0; z < be[ax] - (ax == dax); ++z) mono *= w[ax];
          v = base * be[dax] * mono;
        }
      }
    }
    Wl2p2[e] = v;
  }
}

// chunk count and first fragment of each tile of an M2L launch, as
// compile-time tables (the helper functions loop and must not run on device)
template <int P, int T0, int NT>
struct TileChunks {
  int v[NT];
  int off[NT];
  constexpr TileChunks() : v(), off() {
    for (int t = 0; t < NT; ++t) {
      v[t] = m2l_tile_chunks(P, T0 + t);
      off[t] = m2l_frag_offset(P, T0 + t);
    }
  }
};

// ---------------------------------------------------------------------------
// M2L, eq. (M2L), over the oct-shared interaction lists (Sec. 2.2), every
// level in one launch per column group.  Rows are cells P of a source grid
// s = k - 1 (one wave per parity class of P); columns are (child q, local
// term b) sorted by |b|; the result is the M2L part Lam_k of the locals of
// the 8 children, Lam_k[2P + q][b] = 2^-(|b|+1) sum_d sum_a D[a+b](Rhat_{d,q}) Mhat_s[P-d][a].
// A block owns an LX^3 tile of grid s plus a 3-cell halo, staged in LDS one
// chunk of 4 multipole terms at a time (z de-interleaved by parity); B
// fragments come from a plan-time fragment-order table, prefetched one
// offset ahead.
// ---------------------------------------------------------------------------
constexpr int LX = 8;
constexpr int LH = LX + 6, LH2 = LH / 2;
constexpr int M2L_MT = (LX / 2) * (LX / 2) * (LX / 2) / 16;  // 4 row tiles per wave
constexpr int M2L_THREADS = 512;
constexpr int MAXLEV = 12;

struct M2LLevels {
  int nlev;
  int first_block[MAXLEV + 1];
  int tiles_per_axis[MAXLEV];
  int ns[MAXLEV];
  const double* M[MAXLEV];
  double* Lam[MAXLEV];
};

__device__ __forceinline__ int lhalo_index(int hx, int hy, int hz) {
  return ((hx * LH + hy) * 2 + (hz & 1)) * LH2 + (hz >> 1);
}

template <int P, int T0, int NT>
__global__ __launch_bounds__(M2L_THREADS, 1) void k_m2l_f64(M2LLevels lv, const double* __restrict__ Wm2l,
                                                           const int* __restrict__ dlists) {
  constexpr int NL = nterms(P);
  constexpr int NCOL = 8 * NL;
  constexpr TileChunks<P, T0, NT> kch{};
  constexpr int CM = kch.v[0];
  __shared__ d4 halo[LH * LH * LH];
  int li = 0;
  while (li + 1 < lv.nlev && (int)blockIdx.x >= lv.first_block[li + 1]) ++li;
  const int tb = (int)blockIdx.x - lv.first_block[li];
  const int tpa = lv.tiles_per_axis[li];
  const int ns = lv.ns[li], nsp = ns + 6;
  const double* __restrict__ Mh = lv.M[li];
  double* __restrict__ Lam = lv.Lam[li];
  const int tx0 = (tb / (tpa * tpa)) * LX, ty0 = ((tb / tpa) % tpa) * LX, tz0 = (tb % tpa) * LX;
  const long long ncellp = (long long)nsp * nsp * nsp;
  const int lane = threadIdx.x & 63;
  const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave = parity class (uniform)
  const int i = lane & 15, kq = lane >> 4;
  const int r0 = (r >> 2) & 1, r1 = (r >> 1) & 1, r2 = r & 1;
  const int gy = i >> 2, gz = i & 3;  // row i of tile m: lattice (m, gy, gz)

  d4 acc[M2L_MT][NT];
#pragma unroll
  for (int m = 0; m < M2L_MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = d4{0, 0, 0, 0};
  const int* dl = dlists + r * NLIST;
  const double* wl = Wm2l + lane;

  for (int c = 0; c < CM; ++c) {
    __syncthreads();
    for (int h = threadIdx.x; h < LH * LH * LH; h += M2L_THREADS) {
      const int hz = h % LH, hy = (h / LH) % LH, hx = h / (LH * LH);
      const int px = tx0 + hx, py = ty0 + hy, pz = tz0 + hz;
      d4 v = d4{0, 0, 0, 0};
      if (px < nsp && py < nsp && pz < nsp)
        v = *reinterpret_cast<const d4*>(Mh + (c * ncellp + ((long long)px * nsp + py) * nsp + pz) * 4);
      halo[lhalo_index(hx, hy, hz)] = v;
    }
    __syncthreads();
    const double* hal = reinterpret_cast<const double*>(halo);
    // Blocks walk the offset list from different starting points (the sum is
    // order-independent) so that concurrent blocks do not all request the same
    // B fragment at once.  B fragments of offsets it and it + 1 are in flight.
    const int rot = (int)((blockIdx.x * 37u) % NLIST);
    auto dl_at = [&](int j) { j += rot; return dl[j < NLIST ? j : j - NLIST]; };
    double b0[NT], b1[NT];
    {
      const int e0 = dl_at(0), e1 = dl_at(1);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        b0[t] = (c < kch.v[t]) ? wl[((size_t)(kch.off[t] + c) * 343 + e0) * 64] : 0.0;
        b1[t] = (c < kch.v[t]) ? wl[((size_t)(kch.off[t] + c) * 343 + e1) * 64] : 0.0;
      }
    }
    for (int it = 0; it < NLIST; ++it) {
      const int dd = dl_at(it);
      const int d0 = dd / 49 - 3, d1 = (dd / 7) % 7 - 3, d2 = dd % 7 - 3;
      double cb[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        cb[t] = b0[t];
        b0[t] = b1[t];
      }
      if (it + 2 < NLIST) {
        const int dn = dl_at(it + 2);
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (c < kch.v[t]) b1[t] = wl[((size_t)(kch.off[t] + c) * 343 + dn) * 64];
      }
      const int zz = 3 + r2 - d2;
      const int zoff = (zz & 1) * LH2 + gz + (zz >> 1);
      const int hy = 3 + 2 * gy + r1 - d1;
#pragma unroll
      for (int m = 0; m < M2L_MT; ++m) {
        const int hx = 3 + 2 * m + r0 - d0;
        const double a = hal[((hx * LH + hy) * 2 * LH2 + zoff) * 4 + kq];
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (c < kch.v[t]) acc[m][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, cb[t], acc[m][t], 0, 0, 0);
      }
    }
  }
  // epilogue (f64 layout): element v of tile t is row 4v + kq, column 16 (T0 + t) + i;
  // locals are stored per source cell in column order, so the 16 lanes of a
  // row write 128 contiguous bytes
  constexpr int RS = loc_stride(P);
  int escale[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = 16 * (T0 + t) + i;
    escale[t] = -(m2l_col_degree(col < NCOL ? col : 0) + 1);
  }
#pragma unroll
  for (int m = 0; m < M2L_MT; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * v + kq;
      const int p0 = tx0 + 2 * m + r0, p1 = ty0 + 2 * (row >> 2) + r1, p2 = tz0 + 2 * (row & 3) + r2;
      if (p0 >= ns || p1 >= ns || p2 >= ns) continue;
      double* dst = Lam + (((long long)p0 * ns + p1) * ns + p2) * RS + 16 * T0 + i;
#pragma unroll
      for (int t = 0; t < NT; ++t) dst[16 * t] = ldexp(acc[m][t][v], escale[t]);
    }
}

// B fragments of the M2L in fragment order: [fragment f][343 offsets][64]
// (the offsets of one fragment are contiguous), fragment f = (tile t, chunk
// c); lane j + 16 k holds D[a + b](Rhat_{d,q}) of column 16 t + j = (q, b) and
// term a = 4 c + k (0 where |a| + |b| > p).
__global__ void k_expand_m2l(const double* __restrict__ Dtab, double* __restrict__ W, int P, int NF, int ND) {
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= 343LL * NF * 64) return;
  const int lane = (int)(id & 63);
  const int dd = (int)((id >> 6) % 343), f = (int)((id >> 6) / 343);
  int t = 0;
  while (m2l_frag_offset(P, t + 1) <= f) ++t;
  const int c = f - m2l_frag_offset(P, t);
  const int j = lane & 15, k = lane >> 4;
  const int col = 16 * t + j, al = 4 * c + k;
  double v = 0.0;
  if (col < 8 * nterms(P) && al < nterms(P)) {
    const int md = m2l_col_degree(col);
    const int cin = col - 8 * nterms(md - 1);
    const int q = cin / ndeg(md);
    const int bex = c_mi_exp[nterms(md - 1) + cin % ndeg(md)];
    const int aex = c_mi_exp[al];
    if (mi_a(aex) + mi_b(aex) + mi_c(aex) + md <= P)
      v = Dtab[((size_t)dd * 8 + q) * ND +
               mi_index(mi_a(aex) + mi_a(bex), mi_b(aex) + mi_b(bex), mi_c(aex) + mi_c(bex))];
  }
  W[id] = v;
}

// ---------------------------------------------------------------------------
// L2L, eq. (L2L), for one level k: Lhat_k[T] += shift of Lhat_{k-1}[parent(T)]
//   Lhat_k[b] += sum_{|b|+|g|<=p} 2^-(|b|+1) 4^-|g| / g! (2q-1)^g Lhat_{k-1}[b+g]
// in the per-parent column layout.  Thread = (cell P of level k-1, column
// (q, b)); lanes run along columns, so loads and stores of the child locals
// are contiguous and, inside a degree block, every lane walks a list of the
// same length.  Lists (CSR over b): coefficient and, packed,
// column base of b+g (column with q = 0) << 9 | ndeg(|b+g|) << 3 | parity of g.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_l2l(const double* __restrict__ Lprev, double* __restrict__ Lk,
                                             const int* __restrict__ cs, const int* __restrict__ cidx,
                                             const double* __restrict__ ccoef, int ns, int NL, int RS) {
  const long long nps = (long long)ns * ns * ns;
  const long long id = blockIdx.x * 256LL + threadIdx.x;
  if (id >= nps * RS) return;
  const long long P = id / RS;
  const int col = (int)(id % RS);
  if (col >= 8 * NL) return;
  const int md = m2l_col_degree(col);
  const int cin = col - 8 * nterms(md - 1);
  const int q = cin / ndeg(md);
  const int bt = nterms(md - 1) + cin % ndeg(md);
  const int p2 = (int)(P % ns), p1 = (int)((P / ns) % ns), p0 = (int)(P / ((long long)ns * ns));
  const int nsp = ns >> 1;
  const long long PP = ((long long)(p0 >> 1) * nsp + (p1 >> 1)) * nsp + (p2 >> 1);
  const int qP = ((p0 & 1) << 2) | ((p1 & 1) << 1) | (p2 & 1);
  const int nq = (~q) & 7;  // axes with q_i = 0
  const double* src = Lprev + PP * RS;
  double acc = 0.0;
  for (int j = cs[bt]; j < cs[bt + 1]; ++j) {
    const int id2 = cidx[j];
    const int cb = id2 >> 9, nd = (id2 >> 3) & 63, pat = id2 & 7;
    const double x = ccoef[j] * src[cb + qP * nd];
    acc += (__popc(nq & pat) & 1) ? -x : x;
  }
  Lk[P * RS + col] += acc;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long work, int per) { return (unsigned)((work + per - 1) / per); }

hipError_t launch_dtab(fmm_plan* pl, hipStream_t s) {
  hipLaunchKernelGGL(k_dtab, dim3(blocks_for(343 * 8, 64)), dim3(64), 0, s, pl->dtab, pl->p + 1, pl->ND);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  {
    const long long cnt = 343LL * pl->NC * 128 + (long long)pl->NCL * 128 + 54 * 128 + 8LL * pl->NCL * 128;
    hipLaunchKernelGGL(k_expand_bottom, dim3(blocks_for(cnt, 256)), dim3(256), 0, s, pl->dtab, pl->wm2p, pl->wl2p,
                       pl->wp2p, pl->wl2p2, pl->NM, pl->NC, pl->NL, pl->NCL, pl->ND);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    const int NF = m2l_nfrags(pl->p);
    const long long cnt = 343LL * NF * 64;
    hipLaunchKernelGGL(k_expand_m2l, dim3(blocks_for(cnt, 256)), dim3(256), 0, s, pl->dtab, pl->wm2l, pl->p, NF,
                       pl->ND);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (pl->dtab32) {
    const long long cnt = 343LL * 8 * pl->ND;
    hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(cnt, 256)), dim3(256), 0, s, pl->dtab, pl->dtab32, cnt);
    e = hipGetLastError();
  }
  return e;
}

template <int P, int G>
static hipError_t launch_m2l_groups(fmm_plan* pl, const M2LLevels& lv, hipStream_t s) {
  if constexpr (G >= m2l_ngroups(P)) {
    return hipSuccess;
  } else {
    constexpr int T0 = m2l_group_start(P, G), T1 = m2l_group_end(P, T0);
    hipLaunchKernelGGL((k_m2l_f64<P, T0, T1 - T0>), dim3(lv.first_block[lv.nlev]), dim3(M2L_THREADS), 0, s, lv,
                       pl->wm2l, pl->dlists);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_m2l_groups<P, G + 1>(pl, lv, s);
  }
}

// L2L for one level k (Lhat_k += shift of Lhat_{k-1}), in place
static hipError_t launch_l2l(fmm_plan* pl, int k, hipStream_t s) {
  const int ns = 1 << (k - 1), RS = loc_stride(pl->p);
  const long long work = (long long)ns * ns * ns * RS;
  hipLaunchKernelGGL(k_l2l, dim3(blocks_for(work, 256)), dim3(256), 0, s, (const double*)pl->lev[k - 1].L,
                     (double*)pl->lev[k].L, pl->l2l_start, pl->l2l_idx, pl->l2l_coef, ns, pl->NL, RS);
  return hipGetLastError();
}

hipError_t finish_locals(fmm_plan* pl, int level, hipStream_t s) {
  if (level >= 4 && level == pl->F) return launch_l2l(pl, level, s);
  return hipSuccess;
}

template <int P, typename TI, typename TO>
static hipError_t solve_fp64(fmm_plan* pl, const TI* rho, TO* phi, TO* g, hipStream_t s) {
  constexpr int NM = nterms(P), NC = (NM + 3) / 4;
  const int n = pl->n, F = pl->F;
  hipError_t e;
  {
    StageScope sc(pl, ST_P2M, 1, s);
    const long long nT = (long long)(n / 2) * (n / 2) * (n / 2);
    hipLaunchKernelGGL((k_p2m<TI>), dim3(blocks_for(nT, 256)), dim3(256), 0, s, rho, (double*)pl->lev[F].M, n, NM, NC);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int k = F; k >= 3; --k) {
    StageScope sc(pl, ST_M2M, 1, s);
    const long long nP = 1LL << (3 * (k - 1));
    hipLaunchKernelGGL((k_m2m<nterms(PMAX)>), dim3(blocks_for(nP, 4)), dim3(256), 0, s, (const double*)pl->lev[k].M,
                       (double*)pl->lev[k - 1].M, 1 << k, NM, NC);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (F >= 3) {
    // M2L of every level k = 3..F at once (sources at s = k - 1)
    M2LLevels lv{};
    lv.nlev = F - 2;
    lv.first_block[0] = 0;
    for (int li = 0; li < lv.nlev; ++li) {
      const int k = li + 3, ns = 1 << (k - 1);
      lv.ns[li] = ns;
      lv.tiles_per_axis[li] = (ns + LX - 1) / LX;
      lv.M[li] = (const double*)pl->lev[k - 1].M;
      lv.Lam[li] = (double*)pl->lev[k].L;
      const int tpa = lv.tiles_per_axis[li];
      lv.first_block[li + 1] = lv.first_block[li] + tpa * tpa * tpa;
    }
    {
      StageScope sc(pl, ST_M2L, m2l_ngroups(P), s);
      if ((e = launch_m2l_groups<P, 0>(pl, lv, s)) != hipSuccess) return e;
    }
    // L2L down to level F - 1; level F's far field is taken from Lhat_{F-1}
    // directly by the bottom kernel
    StageScope sc(pl, ST_L2L, F - 4 > 0 ? F - 4 : 0, s);
    for (int k = 4; k <= F - 1; ++k)
      if ((e = launch_l2l(pl, k, s)) != hipSuccess) return e;
  }
  {
    StageScope sc(pl, ST_BOTTOM, 1, s);
    const int nF = n / 2;
    const double dx = pl->dx;
    const double* Lf = (F >= 3) ? (const double*)pl->lev[F].L : nullptr;
    const double* Lpar = (F >= 4) ? (const double*)pl->lev[F - 1].L : nullptr;
    dim3 bgrid(blocks_for(nF, BX), blocks_for(nF, BY), blocks_for(nF, BZ));
    hipLaunchKernelGGL((k_bottom_f64<P, TI, TO>), bgrid, dim3(BOT_THREADS), 0, s, (const double*)pl->lev[F].M, Lf,
                       Lpar, rho, pl->wm2p, pl->wl2p, pl->wl2p2, pl->wp2p, pl->dlists, phi, g, nF, 0.5 * dx * dx,
                       -0.25 * dx);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename TI, typename TO>
static hipError_t dispatch_p(fmm_plan* pl, const TI* rho, TO* phi, TO* g, hipStream_t s) {
  switch (pl->p) {
    case 1: return solve_fp64<1>(pl, rho, phi, g, s);
    case 2: return solve_fp64<2>(pl, rho, phi, g, s);
    case 3: return solve_fp64<3>(pl, rho, phi, g, s);
    case 4: return solve_fp64<4>(pl, rho, phi, g, s);
    case 5: return solve_fp64<5>(pl, rho, phi, g, s);
    case 6: return solve_fp64<6>(pl, rho, phi, g, s);
    case 7: return solve_fp64<7>(pl, rho, phi, g, s);
    case 8: return solve_fp64<8>(pl, rho, phi, g, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_solve(fmm_plan* pl, const void* rho, void* phi, void* g, hipStream_t s) {
  if (pl->precision == 0)
    return dispatch_p<double, double>(pl, (const double*)rho, (double*)phi, (double*)g, s);
  return hipErrorInvalidValue;
}

hipError_t launch_backward(fmm_plan*, const void*, const void*, void*, hipStream_t) {
  return hipErrorNotSupported;
}

template <typename T>
__global__ void k_check_finite(const T* __restrict__ x, long long count, int* flag) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < count && !isfinite((double)x[i])) atomicOr(flag, 1);
}

hipError_t launch_check_finite(fmm_plan* pl, const void* rho, int* host_flag, hipStream_t s) {
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
