// Matrix-core kernels of the downward pass, generic over the compute type
// (fmm_types.h).  Included by fmm_impl.h (needs its constant tables and
// helpers).
//
// Both kernels are sums over the 189 offsets d of a parity class (Sec. 2.2):
// with the source grid s, a "row" is a cell P of grid s of parity r and
//   out[P][col] = sum_d sum_a B_d[a][col] Mhat_s[P - d][a],
// B_d[a][(q, x)] = D[a + x](Rhat_{d,q}).  For M2L x runs over local terms
// (eq. (M2L)); for M2P x is one of {0, e_x, e_y, e_z} (potential and
// acceleration at the unigrid children).  A block owns a tile of grid s plus a
// 3-cell halo, staged in LDS one chunk of KC multipole terms at a time (z
// de-interleaved by parity), converted from the FP64 multipoles while
// staging; one wave per parity class.  B fragments come from plan-time
// tables in fragment order, two offset groups in flight.
#pragma once

// Lane roles.  kq = lane / 16.  For OPM = 2 the lanes with kq < 2 take the
// first offset of a pair and kq >= 2 the second; each lane holds VPL terms
// starting at term-in-chunk tic.  tl is the lane's slot in a table entry of
// EL = 64 / OPM lanes.
template <typename CT>
struct LaneRole {
  int sel, tic, tl;
  __device__ LaneRole(int lane) {
    const int kq = lane >> 4;
    if (Mf<CT>::OPM == 2) {
      sel = kq >> 1;
      tic = 8 * (kq & 1);
      tl = (lane & 15) | ((kq & 1) << 4);
    } else {
      sel = 0;
      tic = kq;
      tl = lane;
    }
  }
};

// The list entry a lane uses for one offset group.  With one offset per
// MFMA the entry is wave-uniform and is read into a scalar register, so its
// decode runs on the scalar unit; with two (BF16) each lane reads the entry
// of its half of the K range.
struct EntryGroup {
  int e;           // the packed list entry (one offset per MFMA)
  int aoff, boff;  // two offsets per MFMA: the lane's halo and B-table offsets
};

// ---------------------------------------------------------------------------
// Bottom of the downward pass for the unigrid children of level-F cells:
// columns (q, o), o in {phi, gx, gy, gz}; 32 columns = 2 tiles.  After the
// 189 M2P offsets, three more K blocks: L2P of the M2L part of the row's own
// local, L2P from the parent level's full local (L2L then L2P as one exact
// polynomial evaluation), and the near field (the 216 unigrid densities of
// the 6^3 block around the row's cell).  phi and g are written once.
// ---------------------------------------------------------------------------
// Tile of a block: BX x BY x BZ level-F cells (BZ = 16 or 8); per parity
// class a 4 x 4 x BZ2 lattice of rows, BZ2 = BZ / 2, in MT = BZ2 row tiles of
// 16: tile m holds x = m / TPX, y = YPT (m % TPX) + i / BZ2, z = i % BZ2.
constexpr int BX = 8, BY = 8;
constexpr int HX = BX + 6, HY = BY + 6;
// Waves per parity class of a bottom block: with FP64 and BF16 operands two
// waves share a class's row tiles (1024-thread blocks), so a CU holds 16
// waves to hide the operand latencies; FP32 keeps one and fits two 512-thread
// blocks per CU instead.
template <typename CT>
constexpr int bottom_wpr() { return Mf<CT>::IDX == 1 ? 1 : 2; }
template <typename CT>
constexpr int bottom_threads() { return 512 * bottom_wpr<CT>(); }

// K extent of the near-field block of FMM-1: the 6^3 unigrid cells around a
// row's level-F cell, z padded to 8 (K step k: z run (w0, w1) = k / 8 of the
// block, z offset k % 8; offsets 6 and 7 have zero B rows), so that a lane's
// 8 BF16 operands are one z run of the densities staged in LDS.
constexpr int kNearK1 = 6 * 6 * 8;

template <int BZ>
struct BotShape {
  static constexpr int HZ = BZ + 6, HZ2 = HZ / 2, BZ2 = BZ / 2;
  static constexpr int MT = BZ2;             // row tiles per wave
  static constexpr int YPT = 16 / BZ2;       // y values per tile
  static constexpr int TPX = 4 / YPT;        // tiles per x value
};

// LDS halo layout: element (hx, hy, hz, k) at hx XS + hy YS + (hz & 1) HZ2 KC +
// (hz >> 1) KC + k, z de-interleaved by parity.  The 16 rows of an operand
// fragment are 8 z cells x 2 y cells two apart; for FP64 (8-byte reads) an odd
// y stride in doubles spreads them over the LDS banks.  An operand address is
// a per-lane part (fixed for the kernel) + a per-offset part (uniform) + a
// per-row-tile constant, so each offset costs one vector add.
// BF16 (two 16-byte halves of K per cell chunk): the natural y stride is a
// multiple of 128 bytes, so the rows of the two y values of an operand
// fragment would read the same banks.  The halves of a cell's chunk are
// therefore swapped when bit 1 of its halo y index is set (SWZ): a lane
// whose K half is kh reads position kh ^ swz(hy), and the two y rows of a
// fragment (halo y two apart) always take opposite halves.
template <typename CT, int BZ>
struct Halo {
  static constexpr int KC = Mf<CT>::KC, HZ2 = BotShape<BZ>::HZ2;
  static constexpr int NAT = 2 * HZ2 * KC;  // natural y stride (elements)
  static constexpr int YS = Mf<CT>::IDX == 0 ? (NAT | 1) : NAT;
  static constexpr int XS = HY * YS;
  static constexpr int SIZE = HX * XS;
  static constexpr bool SWZ = Mf<CT>::IDX == 2;
  __device__ static int cell(int hx, int hy, int hz) {
    return hx * XS + hy * YS + ((hz & 1) * HZ2 + (hz >> 1)) * KC;
  }
  // element offset, within its cell's chunk, at which K index k is stored
  __device__ static int kpos(int hy, int k) { return SWZ ? k ^ (((hy >> 1) & 1) << 3) : k; }
  // per-offset part: halo cell 3 + r - d of row g = 0 (z by parity plane)
  __device__ static int offset_part(int r0, int r1, int r2, int d0, int d1, int d2) {
    const int zz = 3 + r2 - d2;
    return (3 + r0 - d0) * XS + (3 + r1 - d1) * YS + ((zz & 1) * HZ2 + (zz >> 1)) * KC;
  }
};
// A pointer known to address global memory: loads through it are global
// (vector-memory) loads rather than flat loads, which also hold the LDS
// counter that the matrix-core loops wait on.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// Copies chunk c (KC terms) of an FP64 operand grid, chunked [nc4][np^3][4],
// into the LDS halo of the tile whose padded origin is (x0, y0, z0),
// converting to the compute type; cells past the grid's end read as zero.
// The loads of a batch of cells are all issued before any is stored, so a
// thread waits for memory once per batch instead of once per cell.
template <typename CT, int BZ, int NTHR>
__device__ __forceinline__ void stage_halo(typename Mf<CT>::H* __restrict__ halo, const double* src, int nc4,
                                           long long ncellp, int np, int x0, int y0, int z0, int c) {
  using H = typename Mf<CT>::H;
  using HL = Halo<CT, BZ>;
  constexpr int S4 = Mf<CT>::KC / 4;
  constexpr int HZ = BotShape<BZ>::HZ, NH = HX * HY * HZ, NIT = (NH + NTHR - 1) / NTHR;
  // cells per batch, sized to the registers the kernels leave free: FP64
  // 5 (40 registers in flight), FP32 2 (16), BF16 1 (the 4 loads of a cell)
  constexpr int BATCH = Mf<CT>::IDX == 0 ? 3 : (Mf<CT>::IDX == 1 ? 2 : 1);
  const __attribute__((address_space(1))) d4* g = gmem(reinterpret_cast<const d4*>(src));
#pragma unroll 1
  for (int b0 = 0; b0 < NIT; b0 += BATCH) {
    d4 v[BATCH][S4];
    int to[BATCH], ty[BATCH];
#pragma unroll
    for (int k = 0; k < BATCH; ++k) {
      const int h = threadIdx.x + (b0 + k) * NTHR;
      to[k] = -1;
      ty[k] = 0;
#pragma unroll
      for (int s4 = 0; s4 < S4; ++s4) v[k][s4] = d4{0, 0, 0, 0};
      if (b0 + k < NIT && h < NH) {
        const int hz = h % HZ, hy = (h / HZ) % HY, hx = h / (HZ * HY);
        to[k] = HL::cell(hx, hy, hz);
        ty[k] = hy;
        const int px = x0 + hx, py = y0 + hy, pz = z0 + hz;
        if (px < np && py < np && pz < np) {
          const long long cell = ((long long)px * np + py) * np + pz;
#pragma unroll
          for (int s4 = 0; s4 < S4; ++s4) {
            const int sc = c * S4 + s4;
            if (sc < nc4) v[k][s4] = g[sc * ncellp + cell];
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < BATCH; ++k)
      if (to[k] >= 0) {
#pragma unroll
        for (int s4 = 0; s4 < S4; ++s4)
#pragma unroll
          for (int e = 0; e < 4; ++e) halo[to[k] + HL::kpos(ty[k], 4 * s4 + e)] = static_cast<H>(v[k][s4][e]);
      }
  }
}

// Staging from a grid already held in the compute type (the typed copies of
// mixed-precision plans, chunked [ceil(NM / KC)][np^3][KC]): a cell's chunk is
// KC contiguous elements, copied with 16-byte loads and 16-byte LDS stores and
// no conversion.  The LDS destination and the grid cell of each cell a thread
// copies are the same for every chunk, so they are computed once per block
// (plan) and each chunk only streams (run).  Cells past the grid's end are
// staged as zeros.
template <typename CT, int BZ, int NTHR>
struct TypedStage {
  using H = typename Mf<CT>::H;
  using HL = Halo<CT, BZ>;
  static constexpr int KC = Mf<CT>::KC, NV = KC * (int)sizeof(H) / 16;  // 16-byte pieces per cell chunk
  static constexpr int HZ = BotShape<BZ>::HZ, NH = HX * HY * HZ, NIT = (NH + NTHR - 1) / NTHR;
  // cells loaded before any is stored (registers in flight: 4 NV per cell)
  static constexpr int BATCH = NV == 2 ? 2 : 4;
  int np_, x0_, y0_, z0_;
  __device__ __forceinline__ void plan(int np, int x0, int y0, int z0) {
    np_ = np;
    x0_ = x0;
    y0_ = y0;
    z0_ = z0;
  }
  __device__ __forceinline__ void run(H* __restrict__ halo, const H* src, long long ncellp, int c) const {
    const __attribute__((address_space(1))) u32x4* g = gmem(reinterpret_cast<const u32x4*>(src)) + c * ncellp * NV;
#pragma unroll 1
    for (int b0 = 0; b0 < NIT; b0 += BATCH) {
      u32x4 v[BATCH][NV];
      int to[BATCH], ty[BATCH];
#pragma unroll
      for (int k = 0; k < BATCH; ++k) {
        const int h = threadIdx.x + (b0 + k) * NTHR;
        to[k] = -1;
        ty[k] = 0;
#pragma unroll
        for (int q = 0; q < NV; ++q) v[k][q] = u32x4{0, 0, 0, 0};
        if (b0 + k < NIT && h < NH) {
          const int hz = h % HZ, hy = (h / HZ) % HY, hx = h / (HZ * HY);
          to[k] = HL::cell(hx, hy, hz);
          ty[k] = hy;
          const int px = x0_ + hx, py = y0_ + hy, pz = z0_ + hz;
          if (px < np_ && py < np_ && pz < np_) {
            const long long from = ((long long)px * np_ + py) * np_ + pz;
#pragma unroll
            for (int q = 0; q < NV; ++q) v[k][q] = g[from * NV + q];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < BATCH; ++k)
        if (to[k] >= 0) {
#pragma unroll
          for (int q = 0; q < NV; ++q)
            *reinterpret_cast<u32x4*>(halo + to[k] + HL::kpos(ty[k], q * (16 / (int)sizeof(H)))) = v[k][q];
        }
    }
  }
};

// Operand addresses of two interaction offsets per MFMA (BF16): for parity
// class r and offset pair j (list entries 2 j and 2 j + 1), entry sel of the
// table holds the halo element offset of the offset's operand cells
// (relative to a lane's base address) and the element offset of its B-table
// slot.  Built once per block; a lane then reads its half with one LDS load.
// Built with one pair more than the list holds: the last is the null pair
// (both entries the null offset, zero B rows).
template <typename HL>
__device__ __forceinline__ void build_pair_table(int2* __restrict__ tab, const int* __restrict__ dlists, int npair,
                                                 int slot_elems, int nthr) {
  for (int t = threadIdx.x; t < 8 * npair * 2; t += nthr) {
    const int r = t / (2 * npair), j = (t >> 1) % npair, sel = t & 1;
    const int e = dlists[r * NLIST_PAD + 2 * j + sel];
    // with swizzled K halves, bit 0 (free: offsets are multiples of KC)
    // holds bit 1 of the halo y index 3 + r1 - d1 of the fragment's first row
    const int swz = HL::SWZ ? ((3 + ((r >> 1) & 1) - dl_d1(e)) >> 1) & 1 : 0;
    tab[t] = int2{HL::offset_part((r >> 2) & 1, (r >> 1) & 1, r & 1, dl_d0(e), dl_d1(e), dl_d2(e)) | swz,
                  dl_dd(e) * slot_elems};
  }
}

// per-row-tile constant of an operand address: lattice x = m / TPX and
// y = YPT (m % TPX) of row tile m
template <typename HL, int TPX, int YPT>
__device__ constexpr int tile_part(int m) {
  return 2 * (m / TPX) * HL::XS + 2 * YPT * (m % TPX) * HL::YS;
}

// Segments: n = nF (level-F cells per axis), tpa = tiles along x and y,
// tz = tiles along z, field, a = Mhat_F, c = Lam_F (or null), d = the parent
// level's locals (or null).
// DL = levels between the finest FMM level and the unigrid (App. A).  DL = 1:
// a level-F cell holds 8 unigrid cells, the 32 columns (q, o).  DL = 2
// (FMM-2): it holds 64; blockIdx.y = g picks the level-(F+1) child of the
// row's cell and the columns are the 8 unigrid children q of that child.
// The B tables then hold 8 groups, and the near field is the 12^3 block of
// unigrid cells of the 27 level-F cells around the row's cell.
// put(e, val(e)) for e in [0, count) over the block's threads, FB values
// loaded per thread before any is put, so each thread waits for memory once
// per FB elements instead of once per element.
template <typename H, int THREADS, int FB, typename Val, typename Put>
__device__ __forceinline__ void block_fill(int count, Val&& val, Put&& put) {
#pragma unroll 1
  for (int j0 = threadIdx.x; j0 < count; j0 += FB * THREADS) {
    H v[FB];
#pragma unroll
    for (int u = 0; u < FB; ++u) {
      const int e = j0 + u * THREADS;
      v[u] = e < count ? val(e) : H(0);
    }
#pragma unroll
    for (int u = 0; u < FB; ++u) {
      const int e = j0 + u * THREADS;
      if (e < count) put(e, v[u]);
    }
  }
}

// minimum waves per SIMD (the second launch bound): one 1024-thread block or
// two 512-thread FP32 blocks per CU (4 waves per SIMD, <= 128 registers)
template <typename CT>
constexpr int bottom_min_waves() { return 4; }

// stamp_cnt / stamp_done (or null): per field, the finished blocks and the
// device wall-clock time at which its last block finished.
template <int P, typename CT, typename TI, typename TO, int BZ, int DL>
__global__ __launch_bounds__(bottom_threads<CT>(), bottom_min_waves<CT>()) void k_bottom(
    const Seg* __restrict__ segs, int nseg, IoArg io, const typename Mf<CT>::H* __restrict__ Wm2p,
    const typename Mf<CT>::H* __restrict__ Wl2p, const typename Mf<CT>::H* __restrict__ Wl2p2,
    const typename Mf<CT>::H* __restrict__ Wp2p, const int* __restrict__ dlists, int nck,
    unsigned int* __restrict__ stamp_cnt, unsigned long long* __restrict__ stamp_done) {
  using M = Mf<CT>;
  using H = typename M::H;
  using AF = typename M::AF;
  using Acc = typename M::Acc;
  using S = BotShape<BZ>;
  constexpr int BZ2 = S::BZ2, BOT_MT = S::MT, YPT = S::YPT, TPX = S::TPX;
  constexpr int KC = M::KC, OPM = M::OPM, VPL = M::VPL, EL = 64 / OPM;
  constexpr int NM = nterms(P), NC4 = (NM + 3) / 4;
  constexpr int NL = nterms(P);
  constexpr int NB = 3 << DL, NNEAR = NB * NB * NB;  // near-field block: 6^3 or 12^3 unigrid cells
  constexpr int KT = 4 * VPL, NLT = (NL + KT - 1) / KT;
  constexpr int NPT = DL == 1 ? kNearK1 / KT : (NNEAR + KT - 1) / KT;
  constexpr int NCK = (NM + KC - 1) / KC;
  constexpr int NGRP = (NLIST + OPM - 1) / OPM;
  constexpr int THREADS = bottom_threads<CT>(), MTW = BOT_MT / bottom_wpr<CT>();  // row tiles per wave
  // mixed precision: the level-F multipoles are staged from their typed copy
  constexpr bool TYPED = M::IDX != 0;
  using HL = Halo<CT, BZ>;
  __shared__ __attribute__((aligned(16))) H halo[HL::SIZE];
  // the interaction lists of the 8 parity classes (one offset per MFMA), or
  // the lanes' operand offsets of each offset pair (two per MFMA)
  __shared__ int slist[OPM == 1 ? 8 * NLIST_PAD : 1];
  __shared__ int2 spair[OPM == 2 ? 8 * (NGRP + 1) * 2 : 1];
  // column of local term bt of child q in the locals' M2L layout, for the
  // tail's L2P reads (-1 past the last term)
  __shared__ int scol[8 * NLT * KT];
  // blocks walk the (order-independent) offset sum from different starting
  // points: the lists are stored rotated (one offset per MFMA; the null entry
  // past the end), or the pairs are taken from a rotated index (two)
  const int rot = (int)((blockIdx.x * 37u) % (OPM == 1 ? NLIST : NGRP));
  if constexpr (OPM == 1)
    for (int t = threadIdx.x; t < 8 * NLIST_PAD; t += THREADS) {
      const int cls = t / NLIST_PAD, j = t - cls * NLIST_PAD, jr = j + rot;
      slist[t] = dlists[cls * NLIST_PAD + (j < NLIST ? (jr < NLIST ? jr : jr - NLIST) : NLIST)];
    }
  else
    build_pair_table<HL>(spair, dlists, NGRP + 1, 2 * EL * VPL, THREADS);
  for (int t = threadIdx.x; t < 8 * NLT * KT; t += THREADS) {
    const int q = t / (NLT * KT), bt = t - q * (NLT * KT);
    const int ex = c_mi_exp[bt < NL ? bt : 0];
    scol[t] = bt < NL ? m2l_col(q, bt, mi_a(ex) + mi_b(ex) + mi_c(ex)) : -1;
  }
  const Seg& sg = find_seg(segs, nseg, blockIdx.x);
  const int nF = sg.n;
  // DL = 2: this block's group of unigrid cells, and its part of each B table
  const int grp = DL == 2 ? (int)blockIdx.y : 0;
  if constexpr (DL == 2) {
    Wm2p += (size_t)grp * NCK * NSLOT * 2 * EL * VPL;
    Wl2p += (size_t)grp * NLT * 2 * 64 * VPL;
    Wl2p2 += (size_t)grp * 8 * NLT * 2 * 64 * VPL;
    Wp2p += (size_t)grp * NPT * 2 * 64 * VPL;
  }
  const double* __restrict__ Mh = sg.a;
  const double* __restrict__ Lf = sg.c;
  const double* __restrict__ Lpar = sg.d;
  const TI* __restrict__ rho = io_rho<TI>(io, sg.field);
  TO* __restrict__ phi = io_phi<TO>(io, sg.field);
  TO* __restrict__ g = io_g<TO>(io, sg.field);
  // unigrid cell size; the accumulators are in units of dx^3 / h and
  // -dx^3 / h^2, h = 2^DL dx the level-F cell size
  const double dxf = DL == 1 ? 0.5 / nF : 0.25 / nF;
  const double sphi = (DL == 1 ? 0.5 : 0.25) * dxf * dxf, sgr = (DL == 1 ? -0.25 : -0.0625) * dxf;
  const int lb = blockIdx.x - sg.first_block;
  const int lane = threadIdx.x & 63;
  // wave = parity class r and, of its BOT_MT row tiles, the MTW from m0 (uniform)
  const int r = __builtin_amdgcn_readfirstlane((threadIdx.x >> 6) & 7);
  const int m0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 9) * MTW;
  const int i = lane & 15, kq = lane >> 4;
  const LaneRole<CT> lr(lane);
  const int r0 = (r >> 2) & 1, r1 = (r >> 1) & 1, r2 = r & 1;
  const int nFp = nF + 6;
  const long long ncellp = (long long)nFp * nFp * nFp;
  const int tx0 = (lb / (sg.tpa * sg.tz)) * BX, ty0 = ((lb / sg.tz) % sg.tpa) * BY, tz0 = (lb % sg.tz) * BZ;
  const int gz = i % BZ2, gyo = i / BZ2;
  // per-lane part of the operand addresses: row (gyo, gz), the lane's K slice
  // and the wave's first row tile (MTW is a multiple of TPX, so the tile
  // offset splits into that of m0 and that of the tile within the wave)
  const H* hlane = halo + 2 * gyo * HL::YS + gz * KC + lr.tic + tile_part<HL, TPX, YPT>(m0);
  // swizzled K halves (BF16): the lane's base for swizzle bit 0 and bit 1 of
  // the fragment's first row (its own row is gyo rows of two further on)
  const int kh = lr.tic >> 3;
  const H* hsw0 = halo + 2 * gyo * HL::YS + gz * KC + 8 * (kh ^ (gyo & 1)) + tile_part<HL, TPX, YPT>(m0);
  const H* hsw1 = halo + 2 * gyo * HL::YS + gz * KC + 8 * (kh ^ (gyo & 1) ^ 1) + tile_part<HL, TPX, YPT>(m0);

  Acc acc[MTW][2];
#pragma unroll
  for (int m = 0; m < MTW; ++m) acc[m][0] = acc[m][1] = Acc{0, 0, 0, 0};
  const int* dl = slist + r * NLIST_PAD;  // visible after the first chunk's barrier
  const int2* dp = spair + r * (NGRP + 1) * 2 + lr.sel;
  auto entry = [&](int pos) { return dl[pos]; };  // pos < NLIST_PAD
  // the same entry as a scalar load from the unrotated global list (pos
  // wave-uniform): its value lands in a scalar register, so it ties up no
  // vector register that a pending operand load could also write
  const int* __restrict__ dg = dlists + r * NLIST_PAD;
  auto entry_s = [&](int pos) {
    const int jr = pos + rot;
    return dg[pos < NLIST ? (jr < NLIST ? jr : jr - NLIST) : NLIST];
  };
  TypedStage<CT, BZ, THREADS> ts;
  if constexpr (TYPED) ts.plan(nFp, tx0, ty0, tz0);

  // the M2P K chunks: nck <= ceil(NM / KC), fewer when the multipoles are
  // truncated at nmax < p (the chunks past it hold only zero terms)
  for (int c = 0; c < nck; ++c) {
    __syncthreads();  // previous chunk fully consumed
    if constexpr (TYPED)
      ts.run(halo, (const H*)sg.t, ncellp, c);
    else
      stage_halo<CT, BZ, THREADS>(halo, Mh, NC4, ncellp, nFp, tx0, ty0, tz0, c);
    __syncthreads();
    const H* wc = Wm2p + (size_t)c * NSLOT * 2 * EL * VPL + lr.tl * VPL;
    auto bload = [&](EntryGroup g, int t) {
      if constexpr (OPM == 1)
        return *reinterpret_cast<const AF*>(wc + ((size_t)dl_dd(g.e) * 2 + t) * EL * VPL);
      else
        return *reinterpret_cast<const AF*>(wc + g.boff + t * EL * VPL);
    };
    // A fragments of offset group j: source halo cell of row (gx, gy, gz) is
    // 3 + 2 g + r - d.  Three register slots for the list entries, the B
    // fragments and the A fragments of groups j, j + 1, j + 2 (the loop is
    // unrolled by three, so no slot is copied): B is loaded two groups
    // ahead, A one group ahead, while the current group's products run.
    auto aload = [&](EntryGroup g, AF (&a)[MTW]) {
      const H* base;
      if constexpr (OPM == 1)
        base = hlane + HL::offset_part(r0, r1, r2, dl_d0(g.e), dl_d1(g.e), dl_d2(g.e));
      else if constexpr (HL::SWZ)
        base = ((g.aoff & 1) ? hsw1 : hsw0) + (g.aoff & ~1);
      else
        base = hlane + g.aoff;
#pragma unroll
      for (int m = 0; m < MTW; ++m)
        a[m] = *reinterpret_cast<const AF*>(base + tile_part<HL, TPX, YPT>(m));
    };
    auto group = [&](int j) {
      EntryGroup g;
      if constexpr (OPM == 1) {
        // FP32 keeps the entry in LDS (measured: its loop runs faster so,
        // and without the scheduling fences below)
        g.e = __builtin_amdgcn_readfirstlane(M::IDX == 1 ? entry(j) : entry_s(j));
      } else {
        const int j0 = j + rot;  // wave-uniform; past the groups, the null pair
        const int jr = j < NGRP ? (j0 < NGRP ? j0 : j0 - NGRP) : NGRP;
        const int2 v = dp[2 * jr];
        g.aoff = v.x;
        g.boff = v.y;
      }
      return g;
    };
    EntryGroup es[3];
    AF bs[3][2], as[3][MTW];
    es[0] = group(0);
    bs[0][0] = bload(es[0], 0);
    bs[0][1] = bload(es[0], 1);
    es[1] = group(1);
    bs[1][0] = bload(es[1], 0);
    bs[1][1] = bload(es[1], 1);
    aload(es[0], as[0]);
    // (the list entry of a group is read three groups ahead and used one
    // group later, so the wait for it, which also covers the LDS reads in
    // flight, finds only reads at least one group old.  FP64, BF16: a scalar
    // load; FP32: an LDS read kept in a vector register until its use)
    constexpr bool F32 = M::IDX == 1;
    EntryGroup ahead{};
    int raw = 0;
    if constexpr (F32)
      raw = entry(2 < NGRP ? 2 : NGRP - 1);
    else
      ahead = group(2);
    // (the body is unrolled by three by hand; unrolling the loop itself would
    // hoist every group's table address out of the chunk loop)
    // whole unrolled iterations, the last padded with null groups (zero B
    // rows), so there is no exit inside an iteration and every load is
    // unconditional: each group's products then wait for a fixed number of
    // loads in flight instead of draining them all
#pragma unroll 1
    for (int j = 0; j < NGRP; j += 3) {
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int jj = j + u, cur = u, nx = (u + 1) % 3, nn = (u + 2) % 3;
        // (FP32, measured faster so, keeps a bounds test and the last real
        // group as the prefetch past the end; for the others both are
        // compile-time true)
        if (!F32 || jj < NGRP) {
          if constexpr (F32)
            es[nn].e = __builtin_amdgcn_readfirstlane(raw);
          else
            es[nn] = ahead;
          bs[nn][0] = bload(es[nn], 0);
          bs[nn][1] = bload(es[nn], 1);
          if constexpr (F32)
            raw = entry(jj + 3 < NGRP ? jj + 3 : NGRP - 1);
          else
            ahead = group(jj + 3);
          aload(es[nx], as[nx]);
          // (keep the loads ahead of the products: the scheduler would move
          // them next to their uses and expose their latency)
          if constexpr (!F32) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int m = 0; m < MTW; ++m) {
            acc[m][0] = M::op(as[cur][m], bs[cur][0], acc[m][0]);
            acc[m][1] = M::op(as[cur][m], bs[cur][1], acc[m][1]);
          }
          if constexpr (!F32) __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
  }

  const int n = nF << DL;
  const long long N = (long long)n * n * n;
  constexpr int RS = loc_stride(P);
  // ---- Tail K blocks, after the M2P sum: L2P of the M2L part of each row's
  // own local (stored with its parent), L2P from the parent level's full
  // local, and (FMM-1) the near field.  Their operands are gathered per row
  // and term, which as per-lane loads would issue one address per element;
  // instead the block stages them in the (now free) halo LDS with loads in
  // which consecutive lanes read consecutive elements, and the products run
  // K step by K step over all of the wave's row tiles, so each B fragment is
  // loaded once per step.
  constexpr int TC = BX * BY * BZ, TP = TC / 8;  // the tile's level-F cells, and their parents
  // loads in flight per thread while filling LDS (as the registers allow)
  constexpr int FILLB = M::IDX == 0 ? 2 : 4;
  // tile-local index of the level-F cell of the lane's row in tile m, and of its parent
  auto lcell = [&](int m) { return ((2 * (m / TPX) + r0) * BY + 2 * (YPT * (m % TPX) + gyo) + r1) * BZ + 2 * gz + r2; };
  auto lpar = [&](int m) { return ((m / TPX) * (BY / 2) + YPT * (m % TPX) + gyo) * (BZ / 2) + gz; };
  if constexpr (DL == 1) {
  if (Lf || sg.u) {
    // terms per pass (chunks of KT): the own and parent operands of TC + TP
    // cells fit the halo area; row stride KPS keeps BF16 rows 16-byte aligned
    // and spreads the rows of a fragment over the LDS banks
    constexpr int CPP = M::IDX == 2 ? 1 : 3, KP = CPP * KT, KPS = M::IDX == 2 ? 40 : 13;

    static_assert((TC + TP) * KPS <= HL::SIZE, "tail operands exceed the halo area");
    H* const own = halo;
    H* const par = halo + TC * KPS;
    // the own locals in the compute type, written so by the M2L (or null: FP64)
    const H* const Lt = static_cast<const H*>(sg.u);
    const int nP = nF >> 1, nPP = nP >> 1;
    const H* const w2 = Wl2p2 + (size_t)r * NLT * 2 * 64 * VPL + lane * VPL;
#pragma unroll 1
    for (int c0 = 0; c0 < NLT; c0 += CPP) {
      __syncthreads();  // the area's previous contents fully consumed
      const int k0 = c0 * KT;
      // BF16, FP32: thread t fills term k0 + t % KP of every CPR-th cell from
      // t / KP (the lanes of a wave read consecutive columns of a row; the
      // term's column in the M2L layout is cb + q nd for a cell that is child
      // q of its parent), FILLB loads in flight.  FP64, whose accumulators
      // leave fewer registers, fills one element per thread and step.
      if constexpr (M::IDX != 0) {
        constexpr int CPR = THREADS / KP;
        const int kk = threadIdx.x % KP, cf = threadIdx.x / KP, bt = k0 + kk;
        const bool tok = cf < CPR && bt < NL;
        const int cb = tok ? scol[bt] : 0, nd = tok ? scol[NLT * KT + bt] - cb : 0;
        const auto gLf = gmem(Lf);
        const auto gLt = gmem(Lt);
        const auto gLp = gmem(Lpar);
#pragma unroll 1
        for (int j = 0; j < (TC + CPR - 1) / CPR; j += FILLB) {
          H v[FILLB];
#pragma unroll
          for (int u = 0; u < FILLB; ++u) {
            const int cell = cf + (j + u) * CPR;
            const int g0 = tx0 + cell / (BY * BZ), g1 = ty0 + (cell / BZ) % BY, g2 = tz0 + cell % BZ;
            v[u] = H(0);
            if (tok && cell < TC && g0 < nF && g1 < nF && g2 < nF) {
              const int q = ((g0 & 1) << 2) | ((g1 & 1) << 1) | (g2 & 1);
              const long long x = (((long long)(g0 >> 1) * nP + (g1 >> 1)) * nP + (g2 >> 1)) * RS + cb + q * nd;
              v[u] = Lt ? gLt[x] : static_cast<H>(gLf[x]);
            }
          }
#pragma unroll
          for (int u = 0; u < FILLB; ++u) {
            const int cell = cf + (j + u) * CPR;
            if (cf < CPR && cell < TC) own[cell * KPS + kk] = v[u];
          }
        }
        // (no parent level above F = 3: zero operands, so the products need no branch)
#pragma unroll 1
        for (int j = 0; j < (TP + CPR - 1) / CPR; j += FILLB) {
          H v[FILLB];
#pragma unroll
          for (int u = 0; u < FILLB; ++u) {
            const int pc = cf + (j + u) * CPR;
            const int g0 = (tx0 >> 1) + pc / ((BY / 2) * (BZ / 2)), g1 = (ty0 >> 1) + (pc / (BZ / 2)) % (BY / 2),
                      g2 = (tz0 >> 1) + pc % (BZ / 2);
            v[u] = H(0);
            if (Lpar && tok && pc < TP && g0 < nP && g1 < nP && g2 < nP) {
              const int q = ((g0 & 1) << 2) | ((g1 & 1) << 1) | (g2 & 1);
              v[u] = static_cast<H>(gLp[(((long long)(g0 >> 1) * nPP + (g1 >> 1)) * nPP + (g2 >> 1)) * RS + cb + q * nd]);
            }
          }
#pragma unroll
          for (int u = 0; u < FILLB; ++u) {
            const int pc = cf + (j + u) * CPR;
            if (cf < CPR && pc < TP) par[pc * KPS + kk] = v[u];
          }
        }
      } else {
        const auto gLf = gmem(Lf);
        const auto gLt = gmem(Lt);
        const auto gLp = gmem(Lpar);
        for (int e = threadIdx.x; e < TC * KP; e += THREADS) {
          const int cell = e / KP, kk = e - cell * KP, bt = k0 + kk;
          const int g0 = tx0 + cell / (BY * BZ), g1 = ty0 + (cell / BZ) % BY, g2 = tz0 + cell % BZ;
          H v = H(0);
          if (bt < NL && g0 < nF && g1 < nF && g2 < nF) {
            const int q = ((g0 & 1) << 2) | ((g1 & 1) << 1) | (g2 & 1);
            const long long x = (((long long)(g0 >> 1) * nP + (g1 >> 1)) * nP + (g2 >> 1)) * RS + scol[q * (NLT * KT) + bt];
            if constexpr (M::IDX == 0)
              v = gLf[x];
            else
              v = Lt ? gLt[x] : static_cast<H>(gLf[x]);
          }
          own[cell * KPS + kk] = v;
        }
        // (no parent level above F = 3: zero operands, so the products need no branch)
        for (int e = threadIdx.x; e < TP * KP; e += THREADS) {
          const int pc = e / KP, kk = e - pc * KP, bt = k0 + kk;
          const int g0 = (tx0 >> 1) + pc / ((BY / 2) * (BZ / 2)), g1 = (ty0 >> 1) + (pc / (BZ / 2)) % (BY / 2),
                    g2 = (tz0 >> 1) + pc % (BZ / 2);
          double v = 0.0;
          if (Lpar && bt < NL && g0 < nP && g1 < nP && g2 < nP) {
            const int q = ((g0 & 1) << 2) | ((g1 & 1) << 1) | (g2 & 1);
            v = gLp[(((long long)(g0 >> 1) * nPP + (g1 >> 1)) * nPP + (g2 >> 1)) * RS + scol[q * (NLT * KT) + bt]];
          }
          par[pc * KPS + kk] = static_cast<H>(v);
        }
      }
      __syncthreads();
#pragma unroll 1
      for (int cl = 0; cl < CPP; ++cl) {
        const int c = c0 + cl;
        if (c >= NLT) break;
        AF bo[2], bp[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          bo[t] = *reinterpret_cast<const AF*>(Wl2p + ((size_t)(c * 2 + t) * 64 + lane) * VPL);
          bp[t] = *reinterpret_cast<const AF*>(w2 + (size_t)(c * 2 + t) * 64 * VPL);
        }
        static_for<MTW>([&](auto mi) {
          constexpr int mw = decltype(mi)::value;
          const AF ao = *reinterpret_cast<const AF*>(own + lcell(m0 + mw) * KPS + KT * cl + VPL * kq);
          const AF ap = *reinterpret_cast<const AF*>(par + lpar(m0 + mw) * KPS + KT * cl + VPL * kq);
          acc[mw][0] = M::op(ao, bo[0], acc[mw][0]);
          acc[mw][1] = M::op(ao, bo[1], acc[mw][1]);
          acc[mw][0] = M::op(ap, bp[0], acc[mw][0]);
          acc[mw][1] = M::op(ap, bp[1], acc[mw][1]);
        });
      }
    }
  }
  {
    // Near field: the densities of the tile's unigrid cells and a 2-cell
    // margin, [UX][UY][UZ] from unigrid (2 tx0 - 2, 2 ty0 - 2, 2 tz0 - 2), in
    // the compute type, zero outside the grid and in the two z positions past
    // the margin.  K step k: z run k / 8 = (w0, w1) over the 6 x 6 block, z
    // offset k % 8 (offsets 6 and 7 have zero B rows).
    constexpr int UX = 2 * BX + 4, UY = 2 * BY + 4, UZ = 2 * BZ + 6;
    static_assert(UX * UY * UZ <= HL::SIZE, "near-field block exceeds the halo area");
    H* const ub = halo;
    __syncthreads();
    const int x0 = 2 * tx0 - 2, y0 = 2 * ty0 - 2, z0 = 2 * tz0 - 2;
    const auto grho = gmem(rho);
    block_fill<H, THREADS, FILLB>(
        UX * UY * UZ,
        [&](int e) {
          const int uz = e % UZ, uy = (e / UZ) % UY, ux = e / (UZ * UY);
          const int w0 = x0 + ux, w1 = y0 + uy, w2 = z0 + uz;
          const bool in = uz < UZ - 2 && w0 >= 0 && w1 >= 0 && w2 >= 0 && w0 < n && w1 < n && w2 < n;
          return in ? static_cast<H>(grho[((long long)w0 * n + w1) * n + w2]) : H(0);
        },
        [&](int e, H v) { ub[e] = v; });
    __syncthreads();
    // the lane's row: ub offset of its 6^3 block's corner, per row tile
    auto ubase = [&](int m) {
      return (2 * (2 * (m / TPX) + r0) * UY + 2 * (2 * (YPT * (m % TPX) + gyo) + r1)) * UZ + 2 * (2 * gz + r2);
    };
    AF bn[2], bx[2];
    if constexpr (M::IDX != 0) {
#pragma unroll
      for (int t = 0; t < 2; ++t) bn[t] = *reinterpret_cast<const AF*>(Wp2p + ((size_t)t * 64 + lane) * VPL);
    }
#pragma unroll 1
    for (int c = 0; c < NPT; ++c) {
      // B of step c; FP32 and BF16 also load step c + 1's ahead (FP64 has no
      // registers for it)
      if constexpr (M::IDX == 0) {
#pragma unroll
        for (int t = 0; t < 2; ++t) bn[t] = *reinterpret_cast<const AF*>(Wp2p + ((size_t)(c * 2 + t) * 64 + lane) * VPL);
      } else {
        const int cn = c + 1 < NPT ? c + 1 : c;
#pragma unroll
        for (int t = 0; t < 2; ++t) bx[t] = *reinterpret_cast<const AF*>(Wp2p + ((size_t)(cn * 2 + t) * 64 + lane) * VPL);
      }
      const int k = KT * c + VPL * kq, run = k >> 3;
      const int koff = (run / 6) * (UY * UZ) + (run % 6) * UZ + (k & 7);
      static_for<MTW>([&](auto mi) {
        constexpr int mw = decltype(mi)::value;
        const H* src = ub + ubase(m0 + mw) + koff;
        AF a;
        if constexpr (VPL == 8) {
          // 8 consecutive BF16 from an even element offset: four 4-byte reads
          const unsigned int* s32 = reinterpret_cast<const unsigned int*>(src);
          const u32x4 w = {s32[0], s32[1], s32[2], s32[3]};
          a = __builtin_bit_cast(AF, w);
        } else {
          a = *src;
        }
        acc[mw][0] = M::op(a, bn[0], acc[mw][0]);
        acc[mw][1] = M::op(a, bn[1], acc[mw][1]);
      });
      if constexpr (M::IDX != 0) {
        bn[0] = bx[0];
        bn[1] = bx[1];
      }
    }
  }
  } else {
    // FMM-2: per-row loads of the L2P operands (its tail is dominated by the
    // 12^3 near field, whose B fragments serve all row tiles of the wave)
    // the lane's own row (A operand) of tile m and its level-F cell, clamped into the grid
    auto cell_of = [&](int m, int& c0, int& c1, int& c2) {
      c0 = tx0 + 2 * (m / TPX) + r0;
      c1 = ty0 + 2 * (YPT * (m % TPX) + gyo) + r1;
      c2 = tz0 + 2 * gz + r2;
      c0 = c0 < nF ? c0 : 0;
      c1 = c1 < nF ? c1 : 0;
      c2 = c2 < nF ? c2 : 0;
    };
    // L2P K blocks of row tile m: the M2L part of the own local (stored with
    // the parent P'), then the parent level's full local; UL chunks at a time,
    // their operand loads issued together
    constexpr int UL = M::IDX == 1 ? 2 : 1;
    auto tail = [&](int m, Acc (&am)[2]) __attribute__((always_inline)) {
      int c0, c1, c2;
      cell_of(m, c0, c1, c2);
      if (Lf) {
        const int nP = nF >> 1, nPP = nP >> 1;
        const auto own = gmem(Lf + (((long long)(c0 >> 1) * nP + (c1 >> 1)) * nP + (c2 >> 1)) * RS);
        const auto par =
            gmem(Lpar ? Lpar + (((long long)(c0 >> 2) * nPP + (c1 >> 2)) * nPP + (c2 >> 2)) * RS : Lf);
        const int qP = (((c0 >> 1) & 1) << 2) | (((c1 >> 1) & 1) << 1) | ((c2 >> 1) & 1);
        const int* colr = scol + r * (NLT * KT);
        const int* colq = scol + qP * (NLT * KT);
        const H* w2 = Wl2p2 + (size_t)r * NLT * 2 * 64 * VPL + lane * VPL;
#pragma unroll 1
        for (int cb = 0; cb < NLT; cb += UL) {
          double va[UL][VPL], vp[UL][VPL];
          AF bo[UL][2], bp[UL][2];
#pragma unroll
          for (int u = 0; u < UL; ++u) {
            const int c = cb + u < NLT ? cb + u : 0;
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
              const int bt = KT * c + VPL * kq + v;
              const int co = colr[bt], cq = colq[bt];
              const bool ok = cb + u < NLT && co >= 0;
              va[u][v] = ok ? own[co] : 0.0;
              vp[u][v] = (ok && Lpar) ? par[cq] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              bo[u][t] = *reinterpret_cast<const AF*>(Wl2p + ((size_t)(c * 2 + t) * 64 + lane) * VPL);
              bp[u][t] = Lpar ? *reinterpret_cast<const AF*>(w2 + (size_t)(c * 2 + t) * 64 * VPL) : bo[u][t];
            }
          }
#pragma unroll
          for (int u = 0; u < UL; ++u) {
            if (cb + u < NLT) {
              am[0] = M::op(M::frag(va[u]), bo[u][0], am[0]);
              am[1] = M::op(M::frag(va[u]), bo[u][1], am[1]);
              if (Lpar) {
                am[0] = M::op(M::frag(vp[u]), bp[u][0], am[0]);
                am[1] = M::op(M::frag(vp[u]), bp[u][1], am[1]);
              }
            }
          }
        }
      }
    };
    static_for<MTW>([&](auto mi) { tail(m0 + decltype(mi)::value, acc[decltype(mi)::value]); });
    // FMM-2's near field, 12^3 sources per row: the B fragments of a K step
    // serve every row tile of the wave, so they are loaded once per step
    // instead of once per row tile.  Row cells packed as c0 << 16 | c1 << 8 | c2.
    // K steps in flight, sized to the registers left: FP64 3; FP32 (8 row
    // tiles per wave) and BF16 (8 densities per lane and tile) 1
    constexpr int UN2 = M::IDX == 0 ? 3 : 1;
    int cpk[MTW];
#pragma unroll
    for (int mw = 0; mw < MTW; ++mw) {
      int c0, c1, c2;
      cell_of(m0 + mw, c0, c1, c2);
      cpk[mw] = (c0 << 16) | (c1 << 8) | c2;
    }
    const auto rg = gmem(rho);
#pragma unroll 1
    for (int cb = 0; cb < NPT; cb += UN2) {
      TI va[UN2][MTW][VPL];
      AF bn[UN2][2];
#pragma unroll
      for (int u = 0; u < UN2; ++u) {
        const int c = cb + u < NPT ? cb + u : 0;
#pragma unroll
        for (int t = 0; t < 2; ++t)
          bn[u][t] = *reinterpret_cast<const AF*>(Wp2p + ((size_t)(c * 2 + t) * 64 + lane) * VPL);
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
          const int k = KT * c + VPL * kq + v;
          const int k0 = k / (NB * NB) - 4, k1 = (k / NB) % NB - 4, k2 = k % NB - 4;
          const bool kok = cb + u < NPT && k < NNEAR;
#pragma unroll
          for (int mw = 0; mw < MTW; ++mw) {
            const int w0 = ((cpk[mw] >> 16) << 2) + k0, w1 = (((cpk[mw] >> 8) & 255) << 2) + k1,
                      w2 = ((cpk[mw] & 255) << 2) + k2;
            va[u][mw][v] = (kok && w0 >= 0 && w1 >= 0 && w2 >= 0 && w0 < n && w1 < n && w2 < n)
                               ? rg[((long long)w0 * n + w1) * n + w2]
                               : TI(0);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UN2; ++u) {
        if (cb + u < NPT) {
#pragma unroll
          for (int mw = 0; mw < MTW; ++mw) {
            acc[mw][0] = M::op(M::frag(va[u][mw]), bn[u][0], acc[mw][0]);
            acc[mw][1] = M::op(M::frag(va[u][mw]), bn[u][1], acc[mw][1]);
          }
        }
      }
    }
  }
  // epilogue: element v of tile t is row M::row(v, kq), column 16 t + i
#pragma unroll
  for (int mw = 0; mw < MTW; ++mw) {
    const int m = m0 + mw;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = M::row(v, kq);
      const int o0 = tx0 + 2 * (m / TPX) + r0, o1 = ty0 + 2 * (YPT * (m % TPX) + row / BZ2) + r1,
                o2 = tz0 + 2 * (row % BZ2) + r2;
      if (o0 >= nF || o1 >= nF || o2 >= nF) continue;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int col = 16 * t + i;
        const int q = col >> 2, o = col & 3;
        // unigrid cell: child q of the row's cell (DL = 1), or of its child grp (DL = 2)
        const int u0 = DL == 1 ? 2 * o0 : 4 * o0 + 2 * ((grp >> 2) & 1);
        const int u1 = DL == 1 ? 2 * o1 : 4 * o1 + 2 * ((grp >> 1) & 1);
        const int u2 = DL == 1 ? 2 * o2 : 4 * o2 + 2 * (grp & 1);
        const long long u = ((long long)(u0 + ((q >> 2) & 1)) * n + (u1 + ((q >> 1) & 1))) * n + (u2 + (q & 1));
        const double val = (double)acc[mw][t][v];
        if (o == 0)
          phi[u] = (TO)(sphi * val);
        else if (g)
          g[(o - 1) * N + u] = (TO)(sgr * val);
      }
    }
  }
  if (stamp_cnt) {
    // the field's last block records when the field is complete: its stores
    // are made visible, then one lane counts the block with a global atomic
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      const unsigned int blocks = (unsigned int)(sg.tpa * sg.tpa * sg.tz) * gridDim.y;
      if (atomicAdd(stamp_cnt + sg.field, 1u) == blocks - 1) stamp_done[sg.field] = wall_clock64();
    }
  }
}

// Start of a timed solve: the device wall-clock time, and the per-field
// block counters cleared (a kernel, so the solve can be captured in a graph).
__global__ void k_stamp_start(unsigned long long* __restrict__ time, unsigned int* __restrict__ cnt, int nf) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) time[0] = wall_clock64();
  if (t < nf) cnt[t] = 0;
}

// Plan-time expansion of the bottom kernel's B operands into fragment order,
// converted to the compute type (round to nearest even from FP64).
//   M2P:   [NCK][NSLOT][2 tiles][EL][VPL]  D[a + e_o](Rhat_{d,q}), term a of the
//          chunk for the entry lane (0 past NM and for the null slot)
//   L2P:   [NLT][2][64][VPL]               l2p_coef
//   L2P2:  [8][NLT][2][64][VPL]            parent-level L2P, per parity class
//   near:  [NPT][2][64][VPL]               p2p_coef
// A column 16 t + j is (q, o) = (col / 4, col % 4).
template <typename CT>
__global__ void k_expand_bottom(const double* __restrict__ Dtab, typename Mf<CT>::H* __restrict__ Wm2p,
                                typename Mf<CT>::H* __restrict__ Wl2p, typename Mf<CT>::H* __restrict__ Wl2p2,
                                typename Mf<CT>::H* __restrict__ Wp2p, int NM, int NL, int ND) {
  using M = Mf<CT>;
  using H = typename M::H;
  constexpr int KC = M::KC, OPM = M::OPM, VPL = M::VPL, EL = 64 / OPM, KT = 4 * VPL;
  const int NCK = (NM + KC - 1) / KC, NLT = (NL + KT - 1) / KT, NPT = kNearK1 / KT;
  const long long n_m2p = (long long)NCK * NSLOT * 2 * EL * VPL;
  const long long n_l2p = (long long)NLT * 2 * 64 * VPL, n_l2p2 = 8 * n_l2p, n_p2p = (long long)NPT * 2 * 64 * VPL;
  long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= n_m2p + n_l2p + n_l2p2 + n_p2p) return;
  if (e < n_m2p) {
    const int v = (int)(e % VPL), el = (int)((e / VPL) % EL), t = (int)((e / ((long long)VPL * EL)) % 2);
    const int slot = (int)((e / ((long long)VPL * EL * 2)) % NSLOT), c = (int)(e / ((long long)VPL * EL * 2 * NSLOT));
    const int j = el & 15, col = 16 * t + j, q = col >> 2, o = col & 3;
    const int tic = OPM == 2 ? 8 * (el >> 4) : (el >> 4);
    const int al = c * KC + tic + v;
    double val = 0.0;
    if (al < NM && slot < 343) {
      const int ex = c_mi_exp[al];
      val = Dtab[((size_t)slot * 8 + q) * ND + mi_index(mi_a(ex) + (o == 1), mi_b(ex) + (o == 2), mi_c(ex) + (o == 3))];
    }
    Wm2p[e] = static_cast<H>(val);
    return;
  }
  e -= n_m2p;
  // tail tables share the layout [chunk][t][64 lanes][VPL], lane = j + 16 kq, k = KT chunk + VPL kq + v
  H* out;
  int rp = 0, kind;
  if (e < n_l2p) {
    out = Wl2p;
    kind = 0;
  } else if (e < n_l2p + n_l2p2) {
    e -= n_l2p;
    out = Wl2p2;
    kind = 1;
    rp = (int)(e / n_l2p);
  } else {
    e -= n_l2p + n_l2p2;
    out = Wp2p;
    kind = 2;
  }
  const long long el = kind == 1 ? e % n_l2p : e;
  const int v = (int)(el % VPL), lane = (int)((el / VPL) % 64), t = (int)((el / (VPL * 64)) % 2);
  const int c = (int)(el / (VPL * 64 * 2));
  const int j = lane & 15, kq = lane >> 4, col = 16 * t + j, q = col >> 2, o = col & 3;
  const int k = KT * c + VPL * kq + v;
  double val = 0.0;
  if (kind == 0) {
    if (k < NL) val = l2p_coef(k, q, o);
  } else if (kind == 1) {
    if (k < NL) val = l2p_parent_coef(k, rp, q, o);
  } else {
    const int run = k >> 3, w2 = k & 7;  // the padded near-field order (kNearK1)
    if (k < kNearK1 && w2 < 6) val = p2p_coef(run / 6 - 2, run % 6 - 2, w2 - 2, q, o);
  }
  out[e] = static_cast<H>(val);
}

// The same tables for FMM-2, one set per group g of 8 unigrid cells (the
// children of level-(F+1) child g of a level-F cell):
//   M2P:   [8][NCK][NSLOT][2][EL][VPL]  from Dtab2 [343][64][ND] (Rhat_{d,s})
//   L2P:   [8][NLT][2][64][VPL]         l2p2_coef
//   L2P2:  [8][8][NLT][2][64][VPL]      l2p2_parent_coef
//   near:  [8][NPT2][2][64][VPL]        p2p2_coef over the 12^3 block
template <typename CT>
__global__ void k_expand_bottom2(const double* __restrict__ Dtab2, typename Mf<CT>::H* __restrict__ Wm2p,
                                 typename Mf<CT>::H* __restrict__ Wl2p, typename Mf<CT>::H* __restrict__ Wl2p2,
                                 typename Mf<CT>::H* __restrict__ Wp2p, int NM, int NL, int ND) {
  using M = Mf<CT>;
  using H = typename M::H;
  constexpr int KC = M::KC, OPM = M::OPM, VPL = M::VPL, EL = 64 / OPM, KT = 4 * VPL;
  const int NCK = (NM + KC - 1) / KC, NLT = (NL + KT - 1) / KT, NPT = (1728 + KT - 1) / KT;
  const long long n_m2p = (long long)NCK * NSLOT * 2 * EL * VPL;
  const long long n_l2p = (long long)NLT * 2 * 64 * VPL, n_l2p2 = 8 * n_l2p, n_p2p = (long long)NPT * 2 * 64 * VPL;
  const long long per = n_m2p + n_l2p + n_l2p2 + n_p2p;
  long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= 8 * per) return;
  // region by region, each [8 groups][...]
  if (e < 8 * n_m2p) {
    const int grp = (int)(e / n_m2p);
    const long long x = e % n_m2p;
    const int v = (int)(x % VPL), el = (int)((x / VPL) % EL), t = (int)((x / ((long long)VPL * EL)) % 2);
    const int slot = (int)((x / ((long long)VPL * EL * 2)) % NSLOT), c = (int)(x / ((long long)VPL * EL * 2 * NSLOT));
    const int j = el & 15, col = 16 * t + j, q = col >> 2, o = col & 3;
    const int tic = OPM == 2 ? 8 * (el >> 4) : (el >> 4);
    const int al = c * KC + tic + v;
    double val = 0.0;
    if (al < NM && slot < 343) {
      const int ex = c_mi_exp[al];
      const int sub = (sub_pos(grp, q, 0) << 4) | (sub_pos(grp, q, 1) << 2) | sub_pos(grp, q, 2);
      val = Dtab2[((size_t)slot * 64 + sub) * ND +
                  mi_index(mi_a(ex) + (o == 1), mi_b(ex) + (o == 2), mi_c(ex) + (o == 3))];
    }
    Wm2p[e] = static_cast<H>(val);
    return;
  }
  e -= 8 * n_m2p;
  H* out;
  long long cnt;
  int kind;
  if (e < 8 * n_l2p) {
    out = Wl2p;
    cnt = n_l2p;
    kind = 0;
  } else if (e < 8 * (n_l2p + n_l2p2)) {
    e -= 8 * n_l2p;
    out = Wl2p2;
    cnt = n_l2p2;
    kind = 1;
  } else {
    e -= 8 * (n_l2p + n_l2p2);
    out = Wp2p;
    cnt = n_p2p;
    kind = 2;
  }
  const int grp = (int)(e / cnt);
  const long long x = e % cnt;
  const int rp = kind == 1 ? (int)(x / n_l2p) : 0;
  const long long el = kind == 1 ? x % n_l2p : x;
  const int v = (int)(el % VPL), lane = (int)((el / VPL) % 64), t = (int)((el / (VPL * 64)) % 2);
  const int c = (int)(el / (VPL * 64 * 2));
  const int j = lane & 15, kq = lane >> 4, col = 16 * t + j, q = col >> 2, o = col & 3;
  const int k = KT * c + VPL * kq + v;
  double val = 0.0;
  if (kind == 0) {
    if (k < NL) val = l2p2_coef(k, grp, q, o);
  } else if (kind == 1) {
    if (k < NL) val = l2p2_parent_coef(k, rp, grp, q, o);
  } else {
    if (k < 1728) val = p2p2_coef(k, grp, q, o);
  }
  out[e] = static_cast<H>(val);
}

// ---------------------------------------------------------------------------
// Parity-class convolution on the matrix cores, every level in one launch per
// column group.  Rows are the cells R of a grid s (one wave per parity class
// r of R); for each list offset d of class r the operand cell is X = R - d,
// staged with a 3-cell halo in LDS, and
//   out[R][col] = sum_d sum_k B_d[k][col] in[X][k].
// CV_M2L   (eq. (M2L), Sec. 2.2): R = source parent P of grid k - 1,
//          in = Mhat_{k-1}, col = (child q, local term b) sorted by |b|,
//          B_d[a][(q, b)] = D[a+b](Rhat_{d,q}); the result is the M2L part of
//          the locals of the 8 children, scaled by 2^-(|b|+1) and stored per
//          source cell in column order.
// CV_M2LT  transposed M2L: R = source cell J, X = a target's parent, in = the
//          adjoint locals in that column order, col = multipole term a,
//          B_d[(q, b)][a] = 2^-(|b|+1) D[a+b](Rhat_{-d,q}); stored as an
//          adjoint multipole grid.
// CV_M2PT  transposed M2P: R = level-F cell J, X = a target cell, in = the 32
//          scaled adjoint outputs (q, o) of X, col = a,
//          B_d[(q, o)][a] = D[a + e_o](Rhat_{-d,q}).
// ---------------------------------------------------------------------------
// Conv tile: CX x CX x CZ row-grid cells (the bottom kernel's shapes), per
// parity class 4 x 4 x CZ/2 rows in CMT = CZ/2 row tiles of 16
// (BotShape<CZ>).  CZ = 16, or 8 for launches whose grids are all at most 8
// cells deep (coarse levels), which would leave a 16-deep tile half empty.
constexpr int CX = 8;
constexpr int M2L_THREADS = 512;

// column tiles per group by compute type (accumulator registers: 8 row
// tiles x NT); variant 1 halves them
template <typename CT, int V = 0>
struct ConvGroup {
  static constexpr int WIDE = Mf<CT>::VPL == 8 ? 3 : (sizeof(typename Mf<CT>::Acc) == 32 ? 2 : 4);
  static constexpr int NT = V == 0 ? WIDE : (WIDE + 1) / 2;
};

// Calls f(std::integral_constant<int, k>) for k = N, N - 1, ..., 1.
template <int N, typename F>
__device__ __forceinline__ void count_down(F&& f) {
  f(std::integral_constant<int, N>{});
  if constexpr (N > 1) count_down<N - 1>(f);
}

// Segments: n = row grid cells per axis, tpa = tiles along x and y, tz =
// tiles along z, split = number of blocks sharing a tile (each sums a slice of the offsets), a = operand
// grid (chunked [NK/4][(n+6)^3][4] with a zero margin), b = output (CV_M2L:
// locals [n^3][loc_stride], or split partial sums [split][n^3][loc_stride];
// otherwise chunked padded [NC4][(n+6)^3][4]).
// Grid: ngroups x T blocks, T = the tile blocks of all segments; block b works
// on column group b / T (the heaviest groups first) of tile block b % T.
// tiles[t] = (K chunks, first fragment) of column tile t, zero past the last.
template <int P, typename CT, int OP, int NT, int CZ>
__global__ __launch_bounds__(M2L_THREADS, 1) void k_conv(const Seg* __restrict__ segs, int nseg, int T,
                                                        const int2* __restrict__ tiles,
                                                        const typename Mf<CT>::H* __restrict__ Wt,
                                                        const int* __restrict__ dlists) {
  using M = Mf<CT>;
  using H = typename M::H;
  using AF = typename M::AF;
  using Acc = typename M::Acc;
  constexpr int KC = M::KC, OPM = M::OPM, VPL = M::VPL, EL = 64 / OPM;
  constexpr int NC4 = (conv_nk(OP, P) + 3) / 4;  // 4-term chunks of the operand grid
  constexpr int NCOL = 8 * nterms(P), NTILES = conv_ntiles(OP, P);
  constexpr int NCO = conv_ncols(OP, P);  // output columns (transposes: the chunked output grid's terms)
  constexpr int NOFF = conv_noff(OP), NS = conv_nslot(OP);  // list offsets, B-table slots
  constexpr int NGRP = (NOFF + OPM - 1) / OPM;
  using S = BotShape<CZ>;
  constexpr int CMT = S::MT;  // row tiles per wave
  constexpr int BZ2 = S::BZ2, YPT = S::YPT, TPX = S::TPX;
  using HL = Halo<CT, CZ>;
  // the forward M2L of mixed-precision plans stages the typed multipole copy
  constexpr bool TYPED = OP == CV_M2L && M::IDX != 0;
  __shared__ __attribute__((aligned(16))) H halo[HL::SIZE];
  // the offset lists of the 8 parity classes (one offset per MFMA), or the
  // lanes' operand offsets of each offset pair (two per MFMA)
  __shared__ int slist[OPM == 1 ? 8 * NLIST_PAD : 1];
  __shared__ int2 spair[OPM == 2 ? 8 * (NGRP + 1) * 2 : 1];
  const int grp = (int)blockIdx.x / T;
  const int T0 = grp * NT;
  const int lbk = (int)blockIdx.x - grp * T;
  const Seg& sg = find_seg(segs, nseg, lbk);
  const int split = sg.split;
  const int tbs = lbk - sg.first_block;
  const int tb = tbs / split, part = tbs - tb * split;
  // the rotation of the offset order (of entries, or of pairs) must be the
  // same for every part of a split tile (the parts take consecutive slices of
  // one ordering); the entry lists are stored rotated, the null entry past
  // the end
  const int rot = (int)(((unsigned)(sg.first_block + tb * split) * 37u) % (OPM == 1 ? NOFF : NGRP));
  if constexpr (OPM == 1)
    for (int t = threadIdx.x; t < 8 * NLIST_PAD; t += M2L_THREADS) {
      const int cls = t / NLIST_PAD, j = t - cls * NLIST_PAD, jr = j + rot;
      slist[t] = dlists[cls * NLIST_PAD + (j < NOFF ? (jr < NOFF ? jr : jr - NOFF) : NOFF)];
    }
  else
    build_pair_table<HL>(spair, dlists, NGRP + 1, EL * VPL, M2L_THREADS);
  const int tpa = sg.tpa;
  const int ns = sg.n, nsp = ns + 6;
  const double* __restrict__ src = sg.a;
  double* __restrict__ dst = sg.b;
  int vt[NT], off[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int2 e = tiles[T0 + t];
    vt[t] = e.x;
    off[t] = e.y;
  }
  const int tx0 = (tb / (tpa * sg.tz)) * CX, ty0 = ((tb / sg.tz) % tpa) * CX, tz0 = (tb % sg.tz) * CZ;
  const long long ncellp = (long long)nsp * nsp * nsp;
  const int lane = threadIdx.x & 63;
  const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave = parity class (uniform)
  const int i = lane & 15, kq = lane >> 4;
  const LaneRole<CT> lr(lane);
  const int r0 = (r >> 2) & 1, r1 = (r >> 1) & 1, r2 = r & 1;
  const int gz = i % BZ2, gyo = i / BZ2;  // row i of tile m: lattice (m / TPX, YPT (m % TPX) + gyo, gz)
  // per-lane part of the operand addresses: row (gyo, gz) and the lane's K slice
  const H* hlane = halo + 2 * gyo * HL::YS + gz * KC + lr.tic;
  // swizzled K halves (BF16): the lane's base for swizzle bit 0 and bit 1 of
  // the fragment's first row
  const int kh = lr.tic >> 3;
  const H* hsw0 = halo + 2 * gyo * HL::YS + gz * KC + 8 * (kh ^ (gyo & 1));
  const H* hsw1 = halo + 2 * gyo * HL::YS + gz * KC + 8 * (kh ^ (gyo & 1) ^ 1);

  Acc acc[CMT][NT];
#pragma unroll
  for (int m = 0; m < CMT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = Acc{0, 0, 0, 0};
  // FP64 transposes: from K chunk nar(t) on, column tile t's B entries are
  // zero outside its first 4 columns, so those chunks run the tile as
  // 4-column products (v_mfma_f64_4x4x4f64, four 4 x 4 blocks over the 16
  // rows, a quarter of the 16-column product's work) into acc4, added to the
  // tile at the end.
  //  - transposed M2L (one tile per block): |a| + |b| <= p with |b| large;
  //    the narrow chunks are a suffix of the tile's chunks (NARROW_C);
  //  - transposed M2Ps: the last tile, past the last multipole term, is
  //    narrow in every chunk; its group runs the narrow form throughout
  //    (NARROW_G, when the group's tiles have equal chunk counts).
  constexpr bool NARROW_C = M::IDX == 0 && OP == CV_M2LT && NT == 1;
  constexpr bool NARROW_G = M::IDX == 0 && (OP == CV_M2PT || OP == CV_M2PT2);
  const int* ntab = reinterpret_cast<const int*>(tiles) + 2 * (NTILES + 16);
  const int nar = NARROW_C ? ntab[T0] : 1 << 30;
  const bool gnar = NARROW_G && T0 + NT - 1 < NTILES && vt[0] > 0 && vt[NT - 1] == vt[0] && ntab[T0 + NT - 1] == 0;
  double acc4[NARROW_C || NARROW_G ? CMT : 1];
#pragma unroll
  for (int m = 0; m < (NARROW_C || NARROW_G ? CMT : 1); ++m) acc4[m] = 0.0;

  const int* dl = slist + r * NLIST_PAD;  // visible after the first chunk's barrier
  const int2* dp = spair + r * (NGRP + 1) * 2 + lr.sel;
  auto entry = [&](int pos) { return dl[pos]; };  // pos < NLIST_PAD
  // the same entry as a scalar load from the unrotated global list (pos
  // wave-uniform): its value lands in a scalar register, so it ties up no
  // vector register that a pending operand load could also write
  const int* __restrict__ dg = dlists + r * NLIST_PAD;
  auto entry_s = [&](int pos) {
    const int jr = pos + rot;
    return dg[pos < NOFF ? (jr < NOFF ? jr : jr - NOFF) : NOFF];
  };
  // Packed groups: M2L column tiles of degree p need the single multipole
  // term a = 0, so one K chunk would carry one useful term in KC.  With one
  // offset per MFMA (FP64, FP32) such a group instead packs four offsets into
  // K: lane k-group kq takes offset 4 j + kq, term 0, and its B value from
  // the k-group-0 lane of that offset's fragment.
  constexpr bool CAN_PACK = OPM == 1 && OP == CV_M2L;
  const bool packed = CAN_PACK && m2l_col_degree(16 * T0) == P;

  // One chunk's offset sum.  Three register slots for the list entries, the
  // B fragments and the A fragments of groups j, j + 1, j + 2 (the loop is
  // unrolled by three, so no slot is copied): B is loaded two groups ahead,
  // A one group ahead.  A fragment m of offset d reads halo cell 3 + 2 g + r
  // - d of its rows.
  auto offsets = [&](auto pk, auto na, int c, auto nr) {
    constexpr bool PK = decltype(pk)::value;
    constexpr int NA = decltype(na)::value;  // column tiles with chunk c (the first NA)
    constexpr bool NR = decltype(nr)::value;  // narrow: tile NA - 1's first 4 columns only
    constexpr int NG = PK ? (NOFF + 3) / 4 : NGRP;
    const int ja = part * NG / split, jb = (part + 1) * NG / split;
    const H* wl = Wt + (PK ? i : lr.tl) * VPL;
    // (narrow products: the lane holds the B value of column lane % 4 of its
    // K row, which the 16-column fragment keeps in lane (lane & 48) | (lane & 3))
    const H* wn = Wt + ((lane & 48) | (lane & 3)) * VPL;
    const H* hl = PK ? hlane - lr.tic : hlane;
    auto bload = [&](EntryGroup g, int t) {
      if constexpr (OPM == 1)
        return *reinterpret_cast<const AF*>((NR && t == NA - 1 ? wn : wl) +
                                            ((size_t)(off[t] + c) * NS + dl_dd(g.e)) * EL * VPL);
      else
        return *reinterpret_cast<const AF*>(wl + (size_t)(off[t] + c) * NS * EL * VPL + g.boff);
    };
    auto group = [&](int j) {
      EntryGroup g;
      if constexpr (PK) {
        g.e = entry(j < jb ? 4 * j + kq : NLIST_PAD - 1);
      } else if constexpr (OPM == 1) {
        g.e = __builtin_amdgcn_readfirstlane(entry_s(j < jb ? j : NOFF));
      } else {
        const int j0 = j + rot;  // wave-uniform; past the part's groups, the null pair
        const int jr = j < jb ? (j0 < NGRP ? j0 : j0 - NGRP) : NGRP;
        const int2 v = dp[2 * jr];
        g.aoff = v.x;
        g.boff = v.y;
      }
      return g;
    };
    auto aload = [&](EntryGroup g, AF (&a)[CMT]) {
      const H* base;
      if constexpr (OPM == 1)
        base = hl + HL::offset_part(r0, r1, r2, dl_d0(g.e), dl_d1(g.e), dl_d2(g.e));
      else if constexpr (HL::SWZ)
        base = ((g.aoff & 1) ? hsw1 : hsw0) + (g.aoff & ~1);
      else
        base = hl + g.aoff;
#pragma unroll
      for (int m = 0; m < CMT; ++m)
        a[m] = *reinterpret_cast<const AF*>(base + tile_part<HL, TPX, YPT>(m));
    };
    EntryGroup es[3];
    AF bs[3][NA], as[3][CMT];
    es[0] = group(ja);
    es[1] = group(ja + 1);
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      bs[0][t] = bload(es[0], t);
      bs[1][t] = bload(es[1], t);
    }
    aload(es[0], as[0]);
    // The list entry of a group is read three groups ahead and used one group
    // later: a scalar load may return out of order, so the wait before the
    // first use of its value covers every scalar and LDS read in flight, and
    // this way those are all at least one group old.
    EntryGroup ahead = group(ja + 2);
    // The groups run in whole unrolled iterations, the last padded with null
    // groups (zero B rows): with no exit inside an iteration and every load
    // unconditional, each group's products wait for a fixed number of loads
    // in flight instead of draining them all.
    const int jp = ja + (jb - ja + 2) / 3 * 3;
#pragma unroll 1
    for (int j = ja; j < jp; j += 3) {
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int jj = j + u, cur = u, nx = (u + 1) % 3, nn = (u + 2) % 3;
        es[nn] = ahead;
#pragma unroll
        for (int t = 0; t < NA; ++t) bs[nn][t] = bload(es[nn], t);
        ahead = group(jj + 3);
        aload(es[nx], as[nx]);
        // (keep the loads ahead of the products: the scheduler would move
        // them next to their uses and expose their latency)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int m = 0; m < CMT; ++m)
#pragma unroll
          for (int t = 0; t < NA; ++t) {
            if constexpr (NR)
              if (t == NA - 1) {
                acc4[m] = __builtin_amdgcn_mfma_f64_4x4x4f64(as[cur][m], bs[cur][t], acc4[m], 0, 0, 0);
                continue;
              }
            acc[m][t] = M::op(as[cur][m], bs[cur][t], acc[m][t]);
          }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };

  // Tiles are sorted by degree, so the tiles that have chunk c are a prefix
  // of the group, and its length NA falls as c rises: the chunks with NA
  // tiles, [vt[NA], vt[NA - 1]), run as one loop with branch-free products.
  TypedStage<CT, CZ, M2L_THREADS> ts;
  if constexpr (TYPED) ts.plan(nsp, tx0, ty0, tz0);
  auto chunks = [&](auto pk, auto gn) {
    count_down<NT>([&](auto nac) {
      constexpr int NA = decltype(nac)::value;
      int cb = 0;
      if constexpr (NA < NT) cb = vt[NA];
      for (int c = cb; c < vt[NA - 1]; ++c) {
        __syncthreads();
        if constexpr (TYPED)
          ts.run(halo, (const H*)sg.t, ncellp, c);
        else
          stage_halo<CT, CZ, M2L_THREADS>(halo, src, NC4, ncellp, nsp, tx0, ty0, tz0, c);
        __syncthreads();
        if constexpr (NARROW_C) {
          if (c >= nar)
            offsets(pk, nac, c, std::true_type{});
          else
            offsets(pk, nac, c, std::false_type{});
        } else {
          offsets(pk, nac, c, gn);
        }
      }
    });
  };
  if constexpr (CAN_PACK) {
    if (packed)
      chunks(std::true_type{}, std::false_type{});
    else
      chunks(std::false_type{}, std::false_type{});
  } else if constexpr (NARROW_G) {
    if (gnar)
      chunks(std::false_type{}, std::true_type{});
    else
      chunks(std::false_type{}, std::false_type{});
  } else {
    chunks(std::false_type{}, std::false_type{});
  }
  if constexpr (NARROW_C || NARROW_G) {
    const int tn = NARROW_C ? (nar < vt[0] ? 0 : -1) : (gnar ? NT - 1 : -1);
    // narrow output C_b[i][j] (row 4 b + i, column j) sits in lane 16 i + 4 b + j;
    // the 16-column tile keeps row 4 v + kq, column i in element v of lane 16 kq + i
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (t == tn)
#pragma unroll
        for (int m = 0; m < CMT; ++m)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const double v = __shfl(acc4[m], (lane & 48) | (b << 2) | (lane & 3));
            if ((lane & 12) == 0) acc[m][t][b] += v;  // the tile's columns 0..3
          }
  }
  // epilogue: element v of tile t is row M::row(v, kq), column 16 (T0 + t) + i
  if constexpr (OP == CV_M2L) {
    // the 16 lanes of a row write 128 contiguous bytes
    constexpr int RS = loc_stride(P);
    if (split > 1) dst += (long long)part * ns * ns * ns * RS;
    // the finest level of a low-precision bottom: locals in the compute type
    H* const ut = static_cast<H*>(sg.u);
    int escale[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = 16 * (T0 + t) + i;
      escale[t] = -(m2l_col_degree(col < NCOL ? col : 0) + 1);
    }
#pragma unroll
    for (int m = 0; m < CMT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = M::row(v, kq);
        const int p0 = tx0 + 2 * (m / TPX) + r0, p1 = ty0 + 2 * (YPT * (m % TPX) + row / BZ2) + r1,
                  p2 = tz0 + 2 * (row % BZ2) + r2;
        if (p0 >= ns || p1 >= ns || p2 >= ns) continue;
        const long long x = (((long long)p0 * ns + p1) * ns + p2) * RS + 16 * T0 + i;
        if (ut) {
#pragma unroll
          for (int t = 0; t < NT; ++t)
            if (T0 + t < NTILES) ut[x + 16 * t] = static_cast<H>(ldexp((double)acc[m][t][v], escale[t]));
        } else {
#pragma unroll
          for (int t = 0; t < NT; ++t)
            if (T0 + t < NTILES) dst[x + 16 * t] = ldexp((double)acc[m][t][v], escale[t]);
        }
      }
  } else {
    if (split > 1) dst += (long long)part * ((NCO + 3) / 4) * ncellp * 4;
#pragma unroll
    for (int m = 0; m < CMT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = M::row(v, kq);
        const int p0 = tx0 + 2 * (m / TPX) + r0, p1 = ty0 + 2 * (YPT * (m % TPX) + row / BZ2) + r1,
                  p2 = tz0 + 2 * (row % BZ2) + r2;
        if (p0 >= ns || p1 >= ns || p2 >= ns) continue;
        const long long cp = ((long long)(p0 + 3) * nsp + (p1 + 3)) * nsp + (p2 + 3);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int a = 16 * (T0 + t) + i;
          if (a < NCO) dst[((a >> 2) * ncellp + cp) * 4 + (a & 3)] = (double)acc[m][t][v];
        }
      }
  }
}

// B fragments of the convolutions in fragment order, converted to the compute
// type: [fragment f][NSLOT][EL][VPL], fragment f = (tile t, chunk c); entry
// lane el holds, for column 16 t + (el & 15), the K indices KC c + tic + v
// (0 where the truncation |a| + |b| <= p drops the pair, past the ends, and in
// the null slot).
template <typename CT>
__global__ void k_expand_conv(const double* __restrict__ Dtab, const double* __restrict__ Dtab2,
                              typename Mf<CT>::H* __restrict__ W, int op, int P, int ND) {
  using M = Mf<CT>;
  constexpr int KC = M::KC, OPM = M::OPM, VPL = M::VPL, EL = 64 / OPM;
  const int NF = conv_nfrags(op, P, KC), NS = conv_nslot(op);
  const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (id >= (long long)NF * NS * EL * VPL) return;
  const int v = (int)(id % VPL), el = (int)((id / VPL) % EL);
  const int slot = (int)((id / ((long long)VPL * EL)) % NS), f = (int)(id / ((long long)VPL * EL * NS));
  int t = 0;
  while (conv_frag_offset(op, P, t + 1, KC) <= f) ++t;
  const int c = f - conv_frag_offset(op, P, t, KC);
  const int j = el & 15;
  const int tic = OPM == 2 ? 8 * (el >> 4) : (el >> 4);
  const int col = 16 * t + j, kk = KC * c + tic + v;
  const int NM = nterms(P);
  double val = 0.0;
  if (op == CV_P2PT2) {
    // K = (g, q, o) of a unigrid target u of the adjacent cell W - d, column
    // = unigrid source s of W: the near-field coefficient at delta = u - w
    if (slot < NP2P && kk < 256) {
      const int d[3] = {slot / 9 - 1, (slot / 3) % 3 - 1, slot % 3 - 1};
      const int cq = kk >> 2, o = kk & 3, g = cq >> 3, q = cq & 7;
      const int sw[3] = {(col >> 4) & 3, (col >> 2) & 3, col & 3};
      int dl3[3];
      for (int ax = 0; ax < 3; ++ax) dl3[ax] = -4 * d[ax] + sub_pos(g, q, ax) - sw[ax];
      val = p2p2_delta_coef(dl3[0], dl3[1], dl3[2], o);
    }
  } else if (op == CV_M2PT2) {
    // K = (g, q, o), column = multipole term a, the derivative at the
    // negated offset and the unigrid position of (g, q)
    const int ns = 342 - slot;
    if (slot < 343 && col < NM && kk < 256) {
      const int aex = c_mi_exp[col];
      const int cq = kk >> 2, o = kk & 3, g = cq >> 3, q = cq & 7;
      const int sub = (sub_pos(g, q, 0) << 4) | (sub_pos(g, q, 1) << 2) | sub_pos(g, q, 2);
      val = Dtab2[((size_t)ns * 64 + sub) * ND + mi_index(mi_a(aex) + (o == 1), mi_b(aex) + (o == 2), mi_c(aex) + (o == 3))];
    }
  } else if (slot < 343) {
    if (op == CV_M2L) {
      // K = multipole term a, column (q, b)
      if (col < 8 * NM && kk < NM) {
        const int md = m2l_col_degree(col);
        const int cin = col - 8 * nterms(md - 1);
        const int q = cin / ndeg(md);
        const int bex = c_mi_exp[nterms(md - 1) + cin % ndeg(md)];
        const int aex = c_mi_exp[kk];
        if (mi_a(aex) + mi_b(aex) + mi_c(aex) + md <= P)
          val = Dtab[((size_t)slot * 8 + q) * ND +
                     mi_index(mi_a(aex) + mi_a(bex), mi_b(aex) + mi_b(bex), mi_c(aex) + mi_c(bex))];
      }
    } else {
      // transposes: column = multipole term a, the derivative is taken at the
      // negated offset (slot 342 - slot)
      const int ns = 342 - slot;
      if (col < NM) {
        const int aex = c_mi_exp[col];
        const int ax = mi_a(aex), ay = mi_b(aex), az = mi_c(aex);
        if (op == CV_M2LT) {
          if (kk < 8 * NM) {
            const int md = m2l_col_degree(kk);
            const int cin = kk - 8 * nterms(md - 1);
            const int q = cin / ndeg(md);
            const int bex = c_mi_exp[nterms(md - 1) + cin % ndeg(md)];
            if (ax + ay + az + md <= P)
              val = ldexp(Dtab[((size_t)ns * 8 + q) * ND + mi_index(ax + mi_a(bex), ay + mi_b(bex), az + mi_c(bex))],
                          -(md + 1));
          }
        } else if (kk < 32) {
          const int q = kk >> 2, o = kk & 3;
          val = Dtab[((size_t)ns * 8 + q) * ND + mi_index(ax + (o == 1), ay + (o == 2), az + (o == 3))];
        }
      }
    }
  }
  W[id] = static_cast<typename M::H>(val);
}
