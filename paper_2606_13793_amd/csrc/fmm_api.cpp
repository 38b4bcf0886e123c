// C ABI of the unigrid FMM library: argument validation, plan construction
// and the solve entry points.  Validation happens before any HIP call, so
// invalid arguments are reported identically with or without a device.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fmm.h"
#include "fmm_internal.h"

namespace {

thread_local std::string g_err;
thread_local int g_status = FMM_OK;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  g_status = code;
  return code;
}

int ok() {
  g_err.clear();
  g_status = FMM_OK;
  return FMM_OK;
}

int ilog2_exact(int n) {
  if (n <= 0 || (n & (n - 1)) != 0) return -1;
  int L = 0;
  while ((1 << L) < n) ++L;
  return L;
}

int validate(int n, int p, int isolated, const fmm_options* o) {
  if (isolated == 0)
    return fail(FMM_ERR_UNSUPPORTED, "only isolated (vacuum) boundary conditions are provided (isolated=0 given)");
  if (isolated != 1) return fail(FMM_ERR_INVALID_ARG, "isolated must be 1 (got %d)", isolated);
  const int L = ilog2_exact(n);
  if (L < 3 || L > 10) return fail(FMM_ERR_INVALID_ARG, "n must be a power of two in [8, 1024] (got %d)", n);
  if (p < 1 || p > fmm::PMAX) return fail(FMM_ERR_INVALID_ARG, "p must be in [1, %d] (got %d)", fmm::PMAX, p);
  if (o) {
    if (o->struct_size < (int)sizeof(fmm_options))
      return fail(FMM_ERR_INVALID_ARG, "fmm_options.struct_size %d < %d", o->struct_size, (int)sizeof(fmm_options));
    if (o->precision < FMM_FP64 || o->precision > FMM_BF16)
      return fail(FMM_ERR_INVALID_ARG, "unknown precision %d", o->precision);
    if (o->nmax != -1 && (o->nmax < 0 || o->nmax > p))
      return fail(FMM_ERR_INVALID_ARG, "nmax must be -1 or in [0, p] (got %d)", o->nmax);
    if (o->delta_l != 1 && o->delta_l != 2)
      return fail(FMM_ERR_UNSUPPORTED, "delta_l must be 1 or 2 (got %d)", o->delta_l);
    if (o->delta_l == 2 && L < 4) return fail(FMM_ERR_INVALID_ARG, "delta_l = 2 needs n >= 16 (got %d)", n);
    if (o->coarse_fp64_levels < 0) return fail(FMM_ERR_INVALID_ARG, "coarse_fp64_levels must be >= 0");
    if (o->bottom_tile != 0 && o->bottom_tile != 8 && o->bottom_tile != 16)
      return fail(FMM_ERR_INVALID_ARG, "bottom_tile must be 0, 8 or 16 (got %d)", o->bottom_tile);
    if (o->delta_l == 2 && o->bottom_tile == 8)
      return fail(FMM_ERR_INVALID_ARG, "delta_l = 2 plans run 16-deep bottom tiles (bottom_tile = 8 given)");
  }
  return FMM_OK;
}

// device bytes a plan will allocate (tables once, grids per field)
size_t plan_bytes(const std::vector<int>& ns, int p, int dl) {
  const int NM = fmm::nterms(p), NC = (NM + 3) / 4, NCL = NC, ND = fmm::nterms(p + 1);
  size_t b = (size_t)343 * 8 * ND * sizeof(double) + 8 * fmm::NLIST_PAD * sizeof(int) + 256;
  // FP64 matrix-core tables (the largest set a plan builds)
  b += ((size_t)21 * fmm::NSLOT * 128 + (size_t)NCL * 128 * 9 + 54 * 128) * sizeof(double);
  // delta_l = 2: the 64-position M2P derivative table and 8 groups of bottom tables
  if (dl == 2)
    b += (size_t)343 * 64 * ND * sizeof(double) +
         ((size_t)21 * fmm::NSLOT * 128 + (size_t)NCL * 128 * 9 + 432 * 128) * 8 * sizeof(double);
  b += (size_t)fmm::NSLOT * fmm::conv_nfrags(fmm::CV_M2L, p, 4) * 64 * sizeof(double);
  for (int n : ns) {
    const int F = ilog2_exact(n) - dl;
    for (int k = 2; k <= F; ++k) {
      const size_t nkp = (size_t)(1 << k) + 6;
      b += (size_t)NC * nkp * nkp * nkp * 4 * sizeof(double);
      if (k >= 3) b += ((size_t)1 << (3 * (k - 1))) * fmm::loc_stride(p) * sizeof(double);
    }
  }
  return b;
}

// Frees a plan-owned backward workspace (NULL-safe per buffer) and resets it.
void release_adj(fmm::AdjWs& w) {
  if (w.ybar) (void)hipFree(w.ybar);
  for (auto a : w.abar)
    if (a) (void)hipFree(a);
  if (w.part) (void)hipFree(w.part);
  if (w.near) (void)hipFree(w.near);
  for (fmm::SegTable* st : {&w.m2lt[0], &w.m2lt[1], &w.m2pt, &w.m2lt_red, &w.p2pt})
    if (st->dev) (void)hipFree(st->dev);
  w = fmm::AdjWs{};
}

void release(fmm_plan* pl) {
  if (!pl) return;
  for (auto& r : pl->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto ev : pl->event_pool) (void)hipEventDestroy(ev);
  if (pl->gexec) (void)hipGraphExecDestroy(pl->gexec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  for (auto& f : pl->fld)
    for (auto& lv : f.lev) {
      if (lv.M) (void)hipFree(lv.M);
      if (lv.Mt) (void)hipFree(lv.Mt);
      if (lv.L) (void)hipFree(lv.L);
      if (lv.Lt) (void)hipFree(lv.Lt);
    }
  auto free_st = [](fmm::SegTable& st) {
    if (st.dev) (void)hipFree(st.dev);
    st = fmm::SegTable{};
  };
  free_st(pl->s_p2m);
  free_st(pl->s_p2m2);
  for (auto& st : pl->s_m2m) free_st(st);
  for (auto& st : pl->s_conv) free_st(st);
  for (auto& st : pl->s_l2l) free_st(st);
  for (auto& a : pl->s_bot)
    for (auto& st : a) free_st(st);
  for (auto& st : pl->s_red) free_st(st);
  release_adj(pl->adj);
  if (pl->conv_part) (void)hipFree(pl->conv_part);
  for (auto& row : pl->tiletab)
    for (auto t : row)
      if (t) (void)hipFree(t);
  if (pl->io) (void)hipFree(pl->io);
  if (pl->stamp_time) (void)hipFree(pl->stamp_time);
  if (pl->stamp_cnt) (void)hipFree(pl->stamp_cnt);
  if (pl->dtab) (void)hipFree(pl->dtab);
  if (pl->dtab2) (void)hipFree(pl->dtab2);
  if (pl->dlists) (void)hipFree(pl->dlists);
  for (int x = 0; x < 3; ++x) {
    if (pl->wm2p[x]) (void)hipFree(pl->wm2p[x]);
    if (pl->wl2p[x]) (void)hipFree(pl->wl2p[x]);
    if (pl->wl2p2[x]) (void)hipFree(pl->wl2p2[x]);
    if (pl->wp2p[x]) (void)hipFree(pl->wp2p[x]);
    if (pl->wm2l[x]) (void)hipFree(pl->wm2l[x]);
  }
  for (int x = 0; x < 3; ++x) {
    if (pl->wt_m2l[x]) (void)hipFree(pl->wt_m2l[x]);
    if (pl->wt_m2p[x]) (void)hipFree(pl->wt_m2p[x]);
    if (pl->wt_p2p[x]) (void)hipFree(pl->wt_p2p[x]);
  }
  if (pl->dlists_p2p) (void)hipFree(pl->dlists_p2p);
  if (pl->adj_l2p) (void)hipFree(pl->adj_l2p);
  if (pl->adj_l2p2) (void)hipFree(pl->adj_l2p2);
  if (pl->m2m_start) (void)hipFree(pl->m2m_start);
  if (pl->m2mt_start) (void)hipFree(pl->m2mt_start);
  if (pl->m2mt_a) (void)hipFree(pl->m2mt_a);
  if (pl->m2mt_coef) (void)hipFree(pl->m2mt_coef);
  if (pl->m2m_off) (void)hipFree(pl->m2m_off);
  if (pl->m2m_coef) (void)hipFree(pl->m2m_coef);
  if (pl->l2l_start) (void)hipFree(pl->l2l_start);
  if (pl->l2l_idx) (void)hipFree(pl->l2l_idx);
  if (pl->l2l_coef) (void)hipFree(pl->l2l_coef);
  if (pl->flag) (void)hipFree(pl->flag);
  delete pl;
}

int dev_alloc(fmm_plan* pl, void** ptr, size_t bytes) {
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return fail(FMM_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  }
  pl->bytes += bytes;
  return FMM_OK;
}

// per parity r, the 189 offsets d = P - J of the interaction list (Sec. 2.2):
// parent(J) adjacent to parent(P) and J not adjacent to P gives, per axis,
// d in [r - 3, r + 2], excluding |d| <= 1 on all three axes.  Entries are
// packed (offset index, d + 3 per axis); entry 189 is the null offset (index
// 343, zero weights) with d = r, which keeps halo addresses in range.
std::vector<int> build_dlists() {
  std::vector<int> out;
  auto pack = [](int dd, int d0, int d1, int d2) { return dd | ((d0 + 3) << 9) | ((d1 + 3) << 12) | ((d2 + 3) << 15); };
  for (int r = 0; r < 8; ++r) {
    const int rr[3] = {(r >> 2) & 1, (r >> 1) & 1, r & 1};
    int count = 0;
    for (int dd = 0; dd < 343; ++dd) {
      const int d[3] = {dd / 49 - 3, (dd / 7) % 7 - 3, dd % 7 - 3};
      bool in = true, near = true;
      for (int a = 0; a < 3; ++a) {
        if (d[a] < rr[a] - 3 || d[a] > rr[a] + 2) in = false;
        if (d[a] < -1 || d[a] > 1) near = false;
      }
      if (in && !near) {
        out.push_back(pack(dd, d[0], d[1], d[2]));
        ++count;
      }
    }
    if (count != fmm::NLIST) return {};
    for (int pad = fmm::NLIST; pad < fmm::NLIST_PAD; ++pad) out.push_back(pack(343, rr[0], rr[1], rr[2]));
  }
  return out;
}

// FMM-2's near-field transpose: per parity class the 27 offsets d in
// [-1, 1]^3 of the adjacent finest cells, packed like the interaction lists
// with the compact slot (d0 + 1) 9 + (d1 + 1) 3 + (d2 + 1); the null entry
// (slot 27, zero weights, d = 0) pads each class to NLIST_PAD.
std::vector<int> build_dlists_p2p() {
  std::vector<int> out;
  auto pack = [](int dd, int d0, int d1, int d2) { return dd | ((d0 + 3) << 9) | ((d1 + 3) << 12) | ((d2 + 3) << 15); };
  for (int r = 0; r < 8; ++r) {
    for (int e = 0; e < fmm::NP2P; ++e) out.push_back(pack(e, e / 9 - 1, (e / 3) % 3 - 1, e % 3 - 1));
    for (int pad = fmm::NP2P; pad < fmm::NLIST_PAD; ++pad) out.push_back(pack(fmm::NP2P, 0, 0, 0));
  }
  return out;
}

hipEvent_t take_event(fmm_plan* pl) {
  if (!pl->event_pool.empty()) {
    hipEvent_t e = pl->event_pool.back();
    pl->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

const char* const kStageNames[fmm::ST_COUNT] = {"p2m", "m2m", "m2l", "l2l", "bottom", "solve", "backward"};

}  // namespace

namespace fmm {
StageScope::StageScope(fmm_plan* pl, int stage, int launches, hipStream_t s) : pl_(pl), s_(s) {
  if (!pl->profiling) return;
  StageRec r{stage, launches, take_event(pl), take_event(pl)};
  if (!r.a || !r.b) return;
  if (hipEventRecord(r.a, s) != hipSuccess) return;
  idx_ = (int)pl->recs.size();
  pl->recs.push_back(r);
}
StageScope::~StageScope() {
  if (idx_ >= 0) (void)hipEventRecord(pl_->recs[idx_].b, s_);
}

#define FMM_BY_ORDER(P_, CALL)                 \
  switch (P_) {                                \
    case 1: return Impl<1>::CALL;              \
    case 2: return Impl<2>::CALL;              \
    case 3: return Impl<3>::CALL;              \
    case 4: return Impl<4>::CALL;              \
    case 5: return Impl<5>::CALL;              \
    case 6: return Impl<6>::CALL;              \
    case 7: return Impl<7>::CALL;              \
    case 8: return Impl<8>::CALL;              \
  }                                            \
  return hipErrorInvalidValue;

hipError_t upload_constants(int p) { FMM_BY_ORDER(p, upload_constants()) }
hipError_t launch_tables(fmm_plan* pl, hipStream_t s) { FMM_BY_ORDER(pl->p, tables(pl, s)) }
hipError_t launch_solve(fmm_plan* pl, IoArg io, hipStream_t s) { FMM_BY_ORDER(pl->p, solve(pl, io, s)) }
hipError_t launch_backward(fmm_plan* pl, const AdjWs& w, const void* dphi, const void* dg, void* drho,
                           hipStream_t s) {
  FMM_BY_ORDER(pl->p, backward(pl, w, dphi, dg, drho, s))
}
hipError_t launch_adjoint_tables(fmm_plan* pl, hipStream_t s) { FMM_BY_ORDER(pl->p, adjoint_tables(pl, s)) }
hipError_t launch_check_finite(fmm_plan* pl, const void* rho, int* host_flag, hipStream_t s) {
  FMM_BY_ORDER(pl->p, check_finite(pl, rho, host_flag, s))
}
hipError_t finish_locals(fmm_plan* pl, int level, hipStream_t s) { FMM_BY_ORDER(pl->p, finish_locals(pl, level, s)) }
#undef FMM_BY_ORDER

}  // namespace fmm

namespace {

constexpr int kConvTile = 8;   // row-grid cells along x and y of a k_conv block
constexpr int kConvTileZ = 16; // and along z
constexpr int kBotTile = 8;   // level-F cells along x and y of a k_bottom block

struct SegList {
  std::vector<fmm::Seg> v;
  long long blocks = 0;
  void add(fmm::Seg sg, long long nb) {
    sg.first_block = (int)blocks;
    blocks += nb;
    v.push_back(sg);
  }
};

int upload_segs(fmm_plan* pl, fmm::SegTable& st, const SegList& l) {
  st = fmm::SegTable{};
  if (l.v.empty()) return FMM_OK;
  if (l.blocks > 0x7fffffffLL) return fail(FMM_ERR_INVALID_ARG, "launch of %lld blocks is too large", l.blocks);
  if (dev_alloc(pl, (void**)&st.dev, l.v.size() * sizeof(fmm::Seg))) return FMM_ERR_OUT_OF_MEMORY;
  if (hipMemcpy(st.dev, l.v.data(), l.v.size() * sizeof(fmm::Seg), hipMemcpyHostToDevice) != hipSuccess)
    return fail(FMM_ERR_DEVICE, "segment upload failed");
  st.nseg = (int)l.v.size();
  st.blocks = (int)l.blocks;
  return FMM_OK;
}

long long cdiv(long long a, long long b) { return (a + b - 1) / b; }

// Tiles of M2L launch site x (0: FP64 target levels, 1: low-precision ones)
// over every field, 8-deep when all its row grids are at most 8 cells deep,
// as build_schedule lays them out; a site under 128 tiles splits each tile's
// offset sum over several blocks.
long long conv_site_tiles(const fmm_plan* pl, int x) {
  const int klow = fmm::m2l_low_from(pl);
  bool any = false, shallow = true;
  for (const auto& fd : pl->fld)
    for (int k = 3; k <= fd.F; ++k)
      if ((k >= klow ? 1 : 0) == x) {
        any = true;
        shallow = shallow && (1 << (k - 1)) <= 8;
      }
  long long T = 0;
  for (const auto& fd : pl->fld)
    for (int k = 3; k <= fd.F; ++k)
      if ((k >= klow ? 1 : 0) == x) {
        const long long n = 1LL << (k - 1);
        T += cdiv(n, kConvTile) * cdiv(n, kConvTile) * cdiv(n, shallow ? 8 : kConvTileZ);
      }
  return any ? T : 0;
}

}  // namespace

namespace fmm {
// Whether the finest locals of field fd live only in the compute type
// (Level::Lt): an FMM-1 field whose bottom kernel runs in FP32/BF16, when the
// low-precision M2L launch does not split its offset sums (split partial sums
// are FP64).  Then no FP64 locals are allocated for that level.
bool finest_locals_typed(const fmm_plan* pl, const Field& fd) {
  return pl->dl == 1 && fd.F >= 3 && bottom_low(pl, fd.F) && conv_site_tiles(pl, 1) >= 128;
}
}  // namespace fmm

namespace fmm {
// Segment tables of every launch site of a solve: one launch per stage (and
// per level for the M2M and L2L chains) covers every field of the plan.
int build_schedule(fmm_plan* pl) {
  const int RS = loc_stride(pl->p), klow = m2l_low_from(pl);
  SegList p2m, p2m2, m2m[16], conv[2], l2l[16], bot[2][2];
  for (int f = 0; f < (int)pl->fld.size(); ++f) {
    const Field& fd = pl->fld[f];
    const int F = fd.F, nF = fd.n >> pl->dl;
    Seg sg{};
    sg.n = fd.n;
    sg.field = f;
    // the FP64 level-F multipoles are read only by an FP64 bottom kernel (the
    // level below is formed from the unigrid), so a low-precision bottom
    // gets its typed copy alone
    sg.b = pl->dl == 1 && bottom_low(pl, F) ? nullptr : (double*)fd.lev[F].M;
    sg.t = fd.lev[F].Mt;
    p2m.add(sg, cdiv((long long)nF * nF * nF, 256));
    // FMM-1: the multipoles of level F - 1 straight from the 4^3 unigrid
    // cells of each cell (as FMM-2's P2M), which reads the density instead
    // of the 8x larger level-F grid; M2M then starts at level F - 1
    int top = F;
    if (pl->dl == 1 && F >= 3) {
      Seg s2{};
      s2.n = fd.n;
      s2.field = f;
      s2.b = (double*)fd.lev[F - 1].M;
      s2.t = fd.lev[F - 1].Mt;
      const long long nc = 1LL << (3 * (F - 1));
      p2m2.add(s2, cdiv(nc, 256));
      top = F - 1;
    }
    for (int k = top; k >= 3; --k) {
      Seg m{};
      m.n = 1 << k;
      m.field = f;
      m.a = (const double*)fd.lev[k].M;
      m.b = (double*)fd.lev[k - 1].M;
      m.t = fd.lev[k - 1].Mt;
      // parents per block of k_m2m: 16 up to 56 terms, else 8
      m2m[k].add(m, cdiv(1LL << (3 * (k - 1)), pl->NM <= 56 ? 16 : 8));
    }
    for (int k = 3; k <= F; ++k) {
      Seg c{};
      c.n = 1 << (k - 1);
      c.tpa = (int)cdiv(c.n, kConvTile);
      c.tz = (int)cdiv(c.n, kConvTileZ);
      c.field = f;
      c.split = 1;
      c.a = (const double*)fd.lev[k - 1].M;
      c.b = (double*)fd.lev[k].L;
      c.t = k >= klow ? fd.lev[k - 1].Mt : nullptr;
      c.u = k == F ? fd.lev[F].Lt : nullptr;
      conv[k >= klow ? 1 : 0].add(c, (long long)c.tpa * c.tpa * c.tz);
    }
    for (int k = 4; k <= F - 1; ++k) {
      Seg l{};
      l.n = 1 << (k - 1);
      l.field = f;
      l.a = (const double*)fd.lev[k - 1].L;
      l.b = (double*)fd.lev[k].L;
      l2l[k].add(l, cdiv((long long)l.n * l.n * l.n, fmm::L2L_ROWS));
    }
    for (int z = 0; z < 2; ++z) {
      Seg b{};
      b.n = nF;
      b.tpa = (int)cdiv(nF, kBotTile);
      b.tz = (int)cdiv(nF, z == 0 ? 16 : 8);
      b.field = f;
      b.a = (const double*)fd.lev[F].M;
      b.c = F >= 3 ? (const double*)fd.lev[F].L : nullptr;
      b.d = F >= 4 ? (const double*)fd.lev[F - 1].L : nullptr;
      b.t = fd.lev[F].Mt;
      bot[bottom_low(pl, F) ? 1 : 0][z].add(b, (long long)b.tpa * b.tpa * b.tz);
    }
  }
  // A site whose row grids are all at most 8 cells deep (the coarse FP64
  // levels of mixed-precision plans, small fields) uses 8-deep tiles.
  int cz[2] = {16, 16};
  for (int x = 0; x < 2; ++x) {
    bool shallow = !conv[x].v.empty();
    for (auto& c : conv[x].v) shallow = shallow && c.n <= 8;
    if (!shallow) continue;
    cz[x] = 8;
    SegList sh;
    for (auto c : conv[x].v) {
      c.tz = (int)cdiv(c.n, 8);
      sh.add(c, (long long)c.tpa * c.tpa * c.tz);
    }
    conv[x] = sh;
  }
  // Launch sites with few tiles (the coarse levels of mixed-precision plans,
  // small grids) split each tile's offset sum over several blocks; the
  // partial sums are added in a fixed order afterwards.
  SegList red[2];
  {
    long long part_doubles = 0;
    std::vector<long long> at[2];
    for (int x = 0; x < 2; ++x) {
      long long T = 0;
      for (auto& c : conv[x].v) T += (long long)c.tpa * c.tpa * c.tz;
      const int S = T >= 128 ? 1 : (int)std::min<long long>(16, std::max<long long>(2, 256 / std::max<long long>(T, 1)));
      if (S == 1 || conv[x].v.empty()) continue;
      for (auto& c : conv[x].v) {
        at[x].push_back(part_doubles);
        part_doubles += (long long)S * c.n * c.n * c.n * RS;
      }
      // rebuild the site with the split (split partial sums are FP64: a
      // site that splits never holds a level with typed locals)
      SegList sp;
      for (auto c : conv[x].v) {
        if (c.u) return fail(FMM_ERR_DEVICE, "internal: a split M2L launch with typed finest locals");
        c.split = S;
        sp.add(c, (long long)c.tpa * c.tpa * c.tz * S);
      }
      conv[x] = sp;
    }
    if (part_doubles) {
      if (dev_alloc(pl, (void**)&pl->conv_part, (size_t)part_doubles * sizeof(double))) return FMM_ERR_OUT_OF_MEMORY;
      for (int x = 0; x < 2; ++x)
        for (size_t i = 0; i < at[x].size(); ++i) {
          Seg& c = conv[x].v[i];
          Seg r{};
          r.n = c.n;
          r.split = c.split;
          r.count = (long long)c.n * c.n * c.n * RS;
          r.field = c.field;
          r.a = pl->conv_part + at[x][i];
          r.b = c.b;
          c.b = pl->conv_part + at[x][i];
          red[x].add(r, cdiv((long long)c.n * c.n * c.n * RS, 256));
        }
    }
  }
  // a bottom reads its finest locals in the compute type exactly when the
  // M2L into that level kept them so (an unsplit launch)
  {
    std::vector<void*> lt(pl->fld.size(), nullptr);
    for (auto& cl : conv)
      for (auto& c : cl.v)
        if (c.u) lt[c.field] = c.u;
    pl->lt_live = false;
    for (auto& bs : bot)
      for (auto& bl : bs)
        for (auto& b : bl.v) {
          b.u = lt[b.field];
          pl->lt_live = pl->lt_live || b.u;
        }
  }
  int rc;
  if ((rc = upload_segs(pl, pl->s_p2m, p2m))) return rc;
  if ((rc = upload_segs(pl, pl->s_p2m2, p2m2))) return rc;
  for (int k = 0; k < 16; ++k) {
    if ((rc = upload_segs(pl, pl->s_m2m[k], m2m[k]))) return rc;
    if ((rc = upload_segs(pl, pl->s_l2l[k], l2l[k]))) return rc;
  }
  for (int x = 0; x < 2; ++x) {
    if ((rc = upload_segs(pl, pl->s_conv[x], conv[x]))) return rc;
    pl->s_conv[x].cz = cz[x];
    if ((rc = upload_segs(pl, pl->s_red[x], red[x]))) return rc;
    for (int z = 0; z < 2; ++z)
      if ((rc = upload_segs(pl, pl->s_bot[x][z], bot[x][z]))) return rc;
  }
  return FMM_OK;
}
}  // namespace fmm

namespace {

// Splits of the transposed M2L's offset sums at target level k: a level
// with fewer tiles than about one per compute unit shares each tile among
// several blocks, so its heavy first column group does not leave units idle.
int adj_split(int k) {
  const int n = 1 << (k - 1);
  const long long T = cdiv(n, kConvTile) * cdiv(n, kConvTile) * cdiv(n, kConvTileZ);
  return T >= 256 ? 1 : (int)std::min<long long>(16, std::max<long long>(2, 256 / T));
}

// Bytes of each backward-workspace buffer of a plan.
struct AdjLayout {
  size_t ybar = 0;
  size_t abar[16] = {};
  size_t near = 0;  // FMM-2 only
};
AdjLayout adj_layout(const fmm_plan* pl) {
  AdjLayout l;
  const size_t nFp = (size_t)(pl->n >> pl->dl) + 6;
  l.ybar = ((size_t)8 << (3 * (pl->dl - 1))) * nFp * nFp * nFp * 4 * sizeof(double);
  if (pl->dl == 2) l.near = (size_t)16 * nFp * nFp * nFp * 4 * sizeof(double);
  for (int k = 3; k <= pl->F; ++k) {
    const size_t np = ((size_t)1 << (k - 1)) + 6;
    l.abar[k] = (size_t)fmm::loc_stride(pl->p) * np * np * np * sizeof(double);
  }
  return l;
}

// Doubles of the split transposed M2L's partial sums (every level passes
// through them and is then summed, or copied when not split).
long long adj_part_doubles(const fmm_plan* pl) {
  long long d = 0;
  for (int k = 3; k <= pl->F; ++k) {
    const long long np = (1LL << (k - 1)) + 6;
    d += (long long)adj_split(k) * pl->NC * np * np * np * 4;
  }
  return d;
}

// A segment list of fixed capacity (built without allocating).
struct SegArr {
  fmm::Seg v[fmm::kMaxAdjSegs];
  int n = 0;
  long long blocks = 0;
  void add(fmm::Seg sg, long long nb) {
    sg.first_block = (int)blocks;
    blocks += nb;
    v[n++] = sg;
  }
};
struct AdjSegs {
  SegArr lt[2], pt, ltr, p2pt;
};

// Segments of the transposed convolutions over workspace w: M2L^T rows are
// the sources of every target level (the finest first, so its long blocks
// start first; FP64 levels and low-precision levels in separate launches),
// M2P^T rows the level-F cells.  With w.part every level writes partial sums
// there and the reductions add them into the multipole grids in a fixed
// order; without it every level writes its adjoint multipoles in place.
AdjSegs adj_segments(const fmm_plan* pl, const fmm::AdjWs& w) {
  AdjSegs a;
  const int klow = fmm::m2l_low_from(pl), nF = pl->n >> pl->dl;
  long long at = 0;
  for (int k = pl->F; k >= 3; --k) {
    const int S = w.part ? adj_split(k) : 1;
    fmm::Seg c{};
    c.n = 1 << (k - 1);
    c.tpa = (int)cdiv(c.n, kConvTile);
    c.tz = (int)cdiv(c.n, kConvTileZ);
    c.split = S;
    c.a = w.abar[k];
    if (w.part) {
      const long long cnt = (long long)pl->NC * (c.n + 6) * (c.n + 6) * (c.n + 6) * 4;
      c.b = w.part + at;
      fmm::Seg r{};
      r.split = S;
      r.count = cnt;
      r.a = w.part + at;
      r.b = (double*)pl->lev[k - 1].M;
      a.ltr.add(r, cdiv(cnt, 256));
      at += S * cnt;
    } else {
      c.b = (double*)pl->lev[k - 1].M;
    }
    a.lt[k >= klow ? 1 : 0].add(c, (long long)c.tpa * c.tpa * c.tz * S);
  }
  fmm::Seg c{};
  c.n = nF;
  c.tpa = (int)cdiv(nF, kConvTile);
  c.tz = (int)cdiv(nF, kConvTileZ);
  c.split = 1;
  c.a = w.ybar;
  c.b = (double*)pl->lev[pl->F].M;
  a.pt.add(c, (long long)c.tpa * c.tpa * c.tz);
  if (pl->dl == 2) {  // the near-field transpose: the same rows, into w.near
    c.b = w.near;
    a.p2pt.add(c, (long long)c.tpa * c.tpa * c.tz);
  }
  return a;
}

int upload_arr(fmm_plan* pl, fmm::SegTable& st, const SegArr& l) {
  st = fmm::SegTable{};
  if (!l.n) return FMM_OK;
  if (dev_alloc(pl, (void**)&st.dev, l.n * sizeof(fmm::Seg))) return FMM_ERR_OUT_OF_MEMORY;
  if (hipMemcpy(st.dev, l.v, l.n * sizeof(fmm::Seg), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "segment upload failed");
  }
  st.nseg = l.n;
  st.blocks = (int)l.blocks;
  return FMM_OK;
}

static_assert(fmm::kMaxAdjSegs * 4 * sizeof(fmm::Seg) <= fmm::kNoallocSegBytes, "segment area too small");

}  // namespace

extern "C" {

int fmm_options_default(fmm_options* opt) {
  if (!opt) return fail(FMM_ERR_INVALID_ARG, "opt is NULL");
  std::memset(opt, 0, sizeof(*opt));
  opt->struct_size = (int)sizeof(fmm_options);
  opt->precision = FMM_FP64;
  opt->nmax = -1;
  opt->coarse_fp64_levels = 4;
  opt->delta_l = 1;
  opt->check_finite = 0;
  opt->autotune = 1;
  opt->bottom_tile = 0;
  opt->autotune_cache = nullptr;
  return ok();
}

}  // extern "C"

namespace {

// Plan for one or several fields (a batch) of the same order and precision.
fmm_plan* create_plan(const std::vector<int>& ns, int p, const fmm_options& o, int batch) {
  const size_t need = plan_bytes(ns, p, o.delta_l);
  if (const char* cap = std::getenv("FMM_TEST_MAX_WORKSPACE")) {
    const unsigned long long lim = std::strtoull(cap, nullptr, 10);
    if (need > lim) {
      fail(FMM_ERR_OUT_OF_MEMORY, "plan needs %zu device bytes, over the FMM_TEST_MAX_WORKSPACE cap %llu", need, lim);
      return nullptr;
    }
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(FMM_ERR_DEVICE, "no HIP device: %s", hipGetErrorString(e));
    return nullptr;
  }
  if ((e = fmm::upload_constants(p)) != hipSuccess) {
    fail(FMM_ERR_DEVICE, "constant upload failed: %s", hipGetErrorString(e));
    return nullptr;
  }
  fmm_plan* pl = new (std::nothrow) fmm_plan();
  if (!pl) {
    fail(FMM_ERR_OUT_OF_MEMORY, "host allocation failed");
    return nullptr;
  }
  pl->p = p;
  pl->dl = o.delta_l;
  pl->nmax = (o.nmax < 0) ? p : o.nmax;
  pl->precision = o.precision;
  pl->coarse_fp64_levels = o.coarse_fp64_levels;
  pl->check_finite = o.check_finite;
  pl->force_bz = o.bottom_tile;
  pl->device = dev;
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) pl->cus = cus;
    (void)hipGetLastError();
  }
  pl->batch = batch;
  // multipoles truncated at nmax < p are held in grids of order p whose
  // terms above nmax are zero (P2M and M2M write them as zero), so every
  // kernel runs at the size of order p
  pl->NM = fmm::nterms(p);
  pl->NMX = fmm::nterms(pl->nmax);
  pl->NC = (pl->NM + 3) / 4;
  pl->NL = fmm::nterms(p);
  pl->NCL = (pl->NL + 3) / 4;
  pl->ND = fmm::nterms(p + 1);
  pl->fld.resize(ns.size());
  for (size_t f = 0; f < ns.size(); ++f) {
    fmm::Field& fd = pl->fld[f];
    fd.n = ns[f];
    fd.L = ilog2_exact(ns[f]);
    fd.F = fd.L - pl->dl;
    fd.dx = 1.0 / ns[f];
    if (fd.F > pl->maxF) pl->maxF = fd.F;
  }
  pl->lev = pl->fld[0].lev;
  pl->n = pl->fld[0].n;
  pl->L = pl->fld[0].L;
  pl->F = pl->fld[0].F;
  pl->dx = pl->fld[0].dx;

  auto bail = [&](void) -> fmm_plan* {
    release(pl);
    return nullptr;
  };
  if (dev_alloc(pl, (void**)&pl->dtab, (size_t)343 * 8 * pl->ND * sizeof(double))) return bail();
  if (pl->dl == 2 && dev_alloc(pl, (void**)&pl->dtab2, (size_t)343 * 64 * pl->ND * sizeof(double))) return bail();
  if (dev_alloc(pl, (void**)&pl->dlists, 8 * fmm::NLIST_PAD * sizeof(int))) return bail();
  {
    // L2L coefficient lists: for each local term b and parity pattern of g
    // (start index 8 b + pattern), the terms b + g with |b + g| <= p and
    // coefficient 2^-(|b|+1) 4^-|g| / g! (the sign for child q is
    // (-1)^((1-q).g), applied per pattern by the kernel)
    std::vector<int> start(1, 0), idx;
    std::vector<double> coef;
    auto fact = [](int k) { double f = 1; for (int i = 2; i <= k; ++i) f *= i; return f; };
    std::vector<int> ex(pl->NL * 3);
    for (int a = 0; a <= p; ++a)
      for (int b = 0; a + b <= p; ++b)
        for (int c = 0; a + b + c <= p; ++c) {
          const int t = fmm::mi_index(a, b, c);
          ex[3 * t] = a; ex[3 * t + 1] = b; ex[3 * t + 2] = c;
        }
    for (int t = 0; t < pl->NL; ++t) {
      const int bx = ex[3 * t], by = ex[3 * t + 1], bz = ex[3 * t + 2], m = bx + by + bz;
      for (int pat = 0; pat < 8; ++pat) {
        for (int gx = (pat >> 2) & 1; gx <= p - m; gx += 2)
          for (int gy = (pat >> 1) & 1; gx + gy <= p - m; gy += 2)
            for (int gz = pat & 1; gx + gy + gz <= p - m; gz += 2) {
              const int ng = gx + gy + gz;
              idx.push_back(fmm::mi_index(bx + gx, by + gy, bz + gz));
              coef.push_back(std::ldexp(1.0 / (fact(gx) * fact(gy) * fact(gz)), -(m + 1) - 2 * ng));
            }
        start.push_back((int)idx.size());
      }
    }
    if ((int)idx.size() != fmm::l2l_entries(p)) {  // k_l2l stages exactly this many entries
      fail(FMM_ERR_DEVICE, "L2L coefficient list size");
      return bail();
    }
    if (dev_alloc(pl, (void**)&pl->l2l_start, start.size() * sizeof(int))) return bail();
    if (dev_alloc(pl, (void**)&pl->l2l_idx, idx.size() * sizeof(int))) return bail();
    if (dev_alloc(pl, (void**)&pl->l2l_coef, coef.size() * sizeof(double))) return bail();
    if (hipMemcpy(pl->l2l_start, start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pl->l2l_idx, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pl->l2l_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      fail(FMM_ERR_DEVICE, "upload failed");
      return bail();
    }
  }
  {
    // M2M coefficient lists: for each multipole term a, every b <= a with
    // g = a - b: LDS offset 8 b + parity pattern of g, coefficient
    // 2^-|b| 4^-|g| / g!
    std::vector<int> start(1, 0), off;
    std::vector<double> coef;
    auto fact = [](int k) { double f = 1; for (int i = 2; i <= k; ++i) f *= i; return f; };
    const int P = pl->p;
    std::vector<int> ex(pl->NM * 3);
    for (int a = 0; a <= P; ++a)
      for (int b = 0; a + b <= P; ++b)
        for (int c = 0; a + b + c <= P; ++c) {
          const int t = fmm::mi_index(a, b, c);
          ex[3 * t] = a; ex[3 * t + 1] = b; ex[3 * t + 2] = c;
        }
    for (int t = 0; t < pl->NM; ++t) {
      const int ax = ex[3 * t], ay = ex[3 * t + 1], az = ex[3 * t + 2];
      for (int x = 0; x <= ax; ++x)
        for (int y = 0; y <= ay; ++y)
          for (int z = 0; z <= az; ++z) {
            const int gx = ax - x, gy = ay - y, gz = az - z;
            const int pat = ((gx & 1) << 2) | ((gy & 1) << 1) | (gz & 1);
            off.push_back(8 * fmm::mi_index(x, y, z) + pat);
            coef.push_back(std::ldexp(1.0 / (fact(gx) * fact(gy) * fact(gz)), -(x + y + z) - 2 * (gx + gy + gz)));
          }
      start.push_back((int)off.size());
    }
    // the same pairs grouped for the transposed M2M: for each b and parity
    // pattern of g, the terms a = b + g
    std::vector<int> tstart(1, 0), ta;
    std::vector<double> tcoef;
    for (int t = 0; t < pl->NM; ++t) {
      const int bx = ex[3 * t], by = ex[3 * t + 1], bz = ex[3 * t + 2], bd = bx + by + bz;
      for (int pat = 0; pat < 8; ++pat) {
        for (int gx = 0; gx + bd <= P; ++gx)
          for (int gy = 0; gx + gy + bd <= P; ++gy)
            for (int gz = 0; gx + gy + gz + bd <= P; ++gz) {
              if ((((gx & 1) << 2) | ((gy & 1) << 1) | (gz & 1)) != pat) continue;
              ta.push_back(fmm::mi_index(bx + gx, by + gy, bz + gz));
              tcoef.push_back(std::ldexp(1.0 / (fact(gx) * fact(gy) * fact(gz)), -bd - 2 * (gx + gy + gz)));
            }
        tstart.push_back((int)ta.size());
      }
    }
    if (dev_alloc(pl, (void**)&pl->m2mt_start, tstart.size() * sizeof(int))) return bail();
    if (dev_alloc(pl, (void**)&pl->m2mt_a, ta.size() * sizeof(int))) return bail();
    if (dev_alloc(pl, (void**)&pl->m2mt_coef, tcoef.size() * sizeof(double))) return bail();
    if (hipMemcpy(pl->m2mt_start, tstart.data(), tstart.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pl->m2mt_a, ta.data(), ta.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pl->m2mt_coef, tcoef.data(), tcoef.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      fail(FMM_ERR_DEVICE, "upload failed");
      return bail();
    }
    if (dev_alloc(pl, (void**)&pl->m2m_start, start.size() * sizeof(int))) return bail();
    if (dev_alloc(pl, (void**)&pl->m2m_off, off.size() * sizeof(int))) return bail();
    if (dev_alloc(pl, (void**)&pl->m2m_coef, coef.size() * sizeof(double))) return bail();
    if (hipMemcpy(pl->m2m_start, start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pl->m2m_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pl->m2m_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      fail(FMM_ERR_DEVICE, "upload failed");
      return bail();
    }
  }
  if (dev_alloc(pl, (void**)&pl->flag, 256)) return bail();
  for (auto& fd : pl->fld) {
    for (int k = 2; k <= fd.F; ++k) {
      fmm::Level& lv = fd.lev[k];
      lv.k = k;
      lv.nk = 1 << k;
      lv.nkp = lv.nk + 6;
      lv.ncell = 1LL << (3 * k);
      lv.ncellp = (long long)lv.nkp * lv.nkp * lv.nkp;
      const size_t mb = (size_t)pl->NC * lv.ncellp * 4 * sizeof(double);
      if (dev_alloc(pl, &lv.M, mb)) return bail();
      if (hipMemset(lv.M, 0, mb) != hipSuccess) {
        fail(FMM_ERR_DEVICE, "hipMemset failed");
        return bail();
      }
      if (fmm::typed_level(pl, fd.F, k)) {
        // the copy in the compute type: BF16 chunks of 16 terms, FP32 of 4
        const int kc = pl->precision == 2 ? 16 : 4;
        const size_t tb = (size_t)((pl->NM + kc - 1) / kc) * kc * lv.ncellp * (pl->precision == 2 ? 2 : 4);
        if (dev_alloc(pl, &lv.Mt, tb)) return bail();
        if (hipMemset(lv.Mt, 0, tb) != hipSuccess) {
          fail(FMM_ERR_DEVICE, "hipMemset failed");
          return bail();
        }
      }
      if (k >= 3) {
        // the finest level of a low-precision bottom keeps its locals in the
        // compute type only (Level::Lt)
        const bool typed = k == fd.F && fmm::finest_locals_typed(pl, fd);
        const size_t lb = (size_t)(lv.ncell / 8) * fmm::loc_stride(p) *
                          (!typed ? sizeof(double) : pl->precision == 2 ? 2 : 4);
        void*& dst = typed ? lv.Lt : lv.L;
        if (dev_alloc(pl, &dst, lb)) return bail();
        if (hipMemset(dst, 0, lb) != hipSuccess) {
          fail(FMM_ERR_DEVICE, "hipMemset failed");
          return bail();
        }
      }
    }
  }
  const std::vector<int> dl = build_dlists();
  if (dl.size() != 8 * (size_t)fmm::NLIST_PAD) {
    fail(FMM_ERR_DEVICE, "interaction-list table has %zu entries", dl.size());
    return bail();
  }
  if ((e = hipMemcpy(pl->dlists, dl.data(), dl.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess) {
    fail(FMM_ERR_DEVICE, "upload failed: %s", hipGetErrorString(e));
    return bail();
  }
  if (fmm::build_schedule(pl)) return bail();
  if ((e = fmm::launch_tables(pl, nullptr)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? FMM_ERR_OUT_OF_MEMORY : FMM_ERR_DEVICE, "table precompute failed: %s",
         hipGetErrorString(e));
    return bail();
  }
  if (!batch) {
    // the backward pass's tables: coefficients of the transposed L2P steps
    // (one set per group of 8 unigrid cells), the transposed convolutions'
    // B fragments and, for FMM-2, the near-field transpose's offset lists
    const size_t ng = pl->dl == 2 ? 8 : 1;
    if (dev_alloc(pl, (void**)&pl->adj_l2p, ng * pl->NL * 32 * sizeof(double)) ||
        dev_alloc(pl, (void**)&pl->adj_l2p2, ng * 8 * pl->NL * 32 * sizeof(double)))
      return bail();
    if (pl->dl == 2) {
      const std::vector<int> lp = build_dlists_p2p();
      if (dev_alloc(pl, (void**)&pl->dlists_p2p, lp.size() * sizeof(int))) return bail();
      if ((e = hipMemcpy(pl->dlists_p2p, lp.data(), lp.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess) {
        fail(FMM_ERR_DEVICE, "upload failed: %s", hipGetErrorString(e));
        return bail();
      }
    }
    if ((e = fmm::launch_adjoint_tables(pl, nullptr)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
      (void)hipGetLastError();
      fail(e == hipErrorOutOfMemory ? FMM_ERR_OUT_OF_MEMORY : FMM_ERR_DEVICE, "adjoint tables: %s",
           hipGetErrorString(e));
      return bail();
    }
    pl->adj_tables = 1;
  }
  if (batch) {
    if (dev_alloc(pl, (void**)&pl->io, ns.size() * sizeof(fmm::Io))) return bail();
    if ((e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
      fail(FMM_ERR_DEVICE, "stream creation failed: %s", hipGetErrorString(e));
      return bail();
    }
  }
  ok();
  return pl;
}

// Points the device I/O table at this call's buffers (a no-op when they are
// the ones of the previous call).
int set_io(fmm_plan* pl, const std::vector<fmm::Io>& io) {
  bool same = pl->io_last.size() == io.size();
  for (size_t i = 0; same && i < io.size(); ++i)
    same = io[i].rho == pl->io_last[i].rho && io[i].phi == pl->io_last[i].phi && io[i].g == pl->io_last[i].g;
  if (same) return FMM_OK;
  hipError_t e = hipDeviceSynchronize();  // earlier calls may still read the table
  if (e == hipSuccess) e = hipMemcpy(pl->io, io.data(), io.size() * sizeof(fmm::Io), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "I/O table upload failed: %s", hipGetErrorString(e));
  }
  pl->io_last = io;
  return FMM_OK;
}

// Key of a batch plan in the autotune cache: everything the launch shapes'
// speed depends on (device, field sizes in order, order, truncation,
// precision policy, level offset).  No whitespace inside.
std::string tune_key(const fmm_plan* pl) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, pl->device) == hipSuccess) arch = prop.gcnArchName;
  (void)hipGetLastError();
  for (char& c : arch)
    if (c == ' ' || c == '\t') c = '_';
  std::string k = arch + "/cu" + std::to_string(pl->cus) + "/p" + std::to_string(pl->p) + "/nmax" +
                  std::to_string(pl->nmax) + "/prec" + std::to_string(pl->precision) + "/dl" + std::to_string(pl->dl) +
                  "/kc" + std::to_string(pl->coarse_fp64_levels) + "/n";
  for (size_t f = 0; f < pl->fld.size(); ++f) k += (f ? "," : "") + std::to_string(pl->fld[f].n);
  return k;
}

// Cache lines are "<key> <bottom tile> <grouping> <ms> <ms> <ms> <ms>"; the
// last line with the key wins.  Returns true and fills the choice if found.
bool tune_cache_lookup(const char* path, const std::string& key, fmm::Tuning* t, std::vector<double>* ms) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  bool found = false;
  size_t pos = 0;
  while (pos < text.size()) {
    size_t end = text.find('\n', pos);
    if (end == std::string::npos) end = text.size();
    const std::string line = text.substr(pos, end - pos);
    pos = end + 1;
    const size_t sp = line.find(' ');
    if (sp != key.size() || line.compare(0, sp, key) != 0) continue;
    int bz = 0, grp = -1;
    double m[4] = {0, 0, 0, 0};
    if (std::sscanf(line.c_str() + sp, "%d %d %lf %lf %lf %lf", &bz, &grp, &m[0], &m[1], &m[2], &m[3]) == 6 &&
        (bz == 8 || bz == 16) && (grp == 0 || grp == 1)) {
      t->bz = bz;
      t->grp = grp;
      ms->assign(m, m + 4);
      found = true;
    }
  }
  return found;
}

void tune_cache_store(const char* path, const std::string& key, const fmm::Tuning& t, const std::vector<double>& ms) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %.6f %.6f %.6f %.6f\n", key.c_str(), t.bz, t.grp, ms[0], ms[1], ms[2], ms[3]);
  std::fclose(f);
}

// Launch-shape autotuner of batch plans: every candidate (bottom tile depth,
// M2L column grouping) solves the batch on zero densities, the fastest mean
// of three timed solves wins.  Candidates that cannot differ are skipped
// (FMM-2 and a forced tile depth fix the bottom tile); their slots in
// tune_ms stay 0.
int autotune(fmm_plan* pl) {
  const size_t esz = pl->precision == 0 ? sizeof(double) : sizeof(float);
  std::vector<void*> bufs;
  std::vector<fmm::Io> io(pl->fld.size());
  auto cleanup = [&]() {
    for (void* b : bufs) (void)hipFree(b);
    pl->io_last.clear();
  };
  for (size_t f = 0; f < pl->fld.size(); ++f) {
    const size_t N = (size_t)pl->fld[f].n * pl->fld[f].n * pl->fld[f].n;
    void *r = nullptr, *ph = nullptr, *g = nullptr;
    if (hipMalloc(&r, N * esz) != hipSuccess || hipMalloc(&ph, N * esz) != hipSuccess ||
        hipMalloc(&g, 3 * N * esz) != hipSuccess) {
      (void)hipGetLastError();
      if (r) bufs.push_back(r);
      if (ph) bufs.push_back(ph);
      cleanup();
      return fail(FMM_ERR_OUT_OF_MEMORY, "autotuner buffers do not fit");
    }
    bufs.push_back(r);
    bufs.push_back(ph);
    bufs.push_back(g);
    (void)hipMemset(r, 0, N * esz);
    io[f] = fmm::Io{r, ph, g};
  }
  if (int rc = set_io(pl, io)) {
    cleanup();
    return rc;
  }
  const fmm::Tuning cand[4] = {{16, 0}, {16, 1}, {8, 0}, {8, 1}};
  const int fixed_bz = pl->dl == 2 ? 16 : pl->force_bz;
  hipEvent_t a = nullptr, b = nullptr;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  const fmm::IoArg arg{nullptr, nullptr, nullptr, pl->io};
  const int prof = pl->profiling;
  pl->profiling = 0;
  pl->tune_ms.assign(4, 0.0);
  double best = 1e300;
  fmm::Tuning pick = cand[fixed_bz == 8 ? 2 : 0];
  hipError_t e = hipSuccess;
  for (int c = 0; c < 4 && e == hipSuccess; ++c) {
    if (fixed_bz && cand[c].bz != fixed_bz) continue;
    pl->tune = cand[c];
    e = fmm::launch_solve(pl, arg, pl->cap_stream);
    if (e == hipSuccess) e = hipEventRecord(a, pl->cap_stream);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = fmm::launch_solve(pl, arg, pl->cap_stream);
    if (e == hipSuccess) e = hipEventRecord(b, pl->cap_stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    pl->tune_ms[c] = ms / 3.0;
    if (e == hipSuccess && ms / 3.0 < best) {
      best = ms / 3.0;
      pick = cand[c];
    }
  }
  pl->profiling = prof;
  pl->tune = pick;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  cleanup();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "autotuning failed: %s", hipGetErrorString(e));
  }
  return FMM_OK;
}

}  // namespace

extern "C" {

fmm_plan* fmm_plan_create(int n, int p, int isolated) { return fmm_plan_create_ex(n, p, isolated, nullptr); }

fmm_plan* fmm_plan_create_ex(int n, int p, int isolated, const fmm_options* opt) {
  if (validate(n, p, isolated, opt) != FMM_OK) return nullptr;
  fmm_options o;
  fmm_options_default(&o);
  if (opt) o = *opt;
  return create_plan(std::vector<int>{n}, p, o, 0);
}

fmm_plan* fmm_batch_plan_create(int count, const int* n, int p, int isolated, const fmm_options* opt) {
  if (count < 1 || count > 4096) {
    fail(FMM_ERR_INVALID_ARG, "count must be in [1, 4096] (got %d)", count);
    return nullptr;
  }
  if (!n) {
    fail(FMM_ERR_INVALID_ARG, "n is NULL");
    return nullptr;
  }
  for (int i = 0; i < count; ++i)
    if (validate(n[i], p, isolated, opt) != FMM_OK) return nullptr;
  fmm_options o;
  fmm_options_default(&o);
  if (opt) o = *opt;
  if (o.check_finite) {
    fail(FMM_ERR_UNSUPPORTED, "check_finite is provided for single-field plans only");
    return nullptr;
  }
  fmm_plan* pl = create_plan(std::vector<int>(n, n + count), p, o, 1);
  if (!pl) return nullptr;
  if (pl->dl == 2 || pl->force_bz) pl->tune.bz = pl->dl == 2 ? 16 : pl->force_bz;
  if (o.autotune) {
    const std::string key = o.autotune_cache ? tune_key(pl) : std::string();
    if (o.autotune_cache && tune_cache_lookup(o.autotune_cache, key, &pl->tune, &pl->tune_ms)) {
      pl->tune_cached = 1;
      if (pl->dl == 2 || pl->force_bz) pl->tune.bz = pl->dl == 2 ? 16 : pl->force_bz;
    } else {
      if (autotune(pl) != FMM_OK) {
        const std::string msg = g_err;
        const int code = g_status;
        release(pl);
        fail(code, "%s", msg.c_str());
        return nullptr;
      }
      if (o.autotune_cache) tune_cache_store(o.autotune_cache, key, pl->tune, pl->tune_ms);
    }
  }
  ok();
  return pl;
}

int fmm_batch_solve(fmm_plan* plan, const void* const* rho, void* const* phi, void* const* g, void* stream) {
  if (!plan) return fail(FMM_ERR_INVALID_ARG, "plan is NULL");
  if (!plan->batch) return fail(FMM_ERR_INVALID_ARG, "not a batch plan (use fmm_solve)");
  if (!rho || !phi) return fail(FMM_ERR_INVALID_ARG, "rho and phi must be arrays of device pointers");
  const int cnt = (int)plan->fld.size();
  std::vector<fmm::Io> io(cnt);
  for (int f = 0; f < cnt; ++f) {
    void* gf = g ? g[f] : nullptr;
    if (!rho[f] || !phi[f]) return fail(FMM_ERR_INVALID_ARG, "field %d: rho and phi must not be NULL", f);
    if (rho[f] == phi[f] || (gf && (gf == rho[f] || gf == phi[f])))
      return fail(FMM_ERR_INVALID_ARG, "field %d: rho, phi and g must not alias", f);
    io[f] = fmm::Io{rho[f], phi[f], gf};
  }
  if (int rc = set_io(plan, io)) return rc;
  hipStream_t s = (hipStream_t)stream;
  const fmm::IoArg arg{nullptr, nullptr, nullptr, plan->io};
  hipError_t e;
  if (plan->profiling) {
    // direct launches, so that every stage records its events
    fmm::StageScope whole(plan, fmm::ST_SOLVE, 0, s);
    e = fmm::launch_solve(plan, arg, s);
  } else {
    if (!plan->gexec) {
      e = hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        const hipError_t le = fmm::launch_solve(plan, arg, plan->cap_stream);
        e = hipStreamEndCapture(plan->cap_stream, &plan->graph);
        if (le != hipSuccess) e = le;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&plan->gexec, plan->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        if (plan->graph) (void)hipGraphDestroy(plan->graph);
        plan->graph = nullptr;
        plan->gexec = nullptr;
        return fail(FMM_ERR_DEVICE, "capturing the batch graph failed: %s", hipGetErrorString(e));
      }
    }
    e = hipGraphLaunch(plan->gexec, s);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "batch launch failed: %s", hipGetErrorString(e));
  }
  return ok();
}

int fmm_batch_timestamps(fmm_plan* plan, int enable) {
  if (!plan) return fail(FMM_ERR_INVALID_ARG, "plan is NULL");
  if (!plan->batch) return fail(FMM_ERR_INVALID_ARG, "not a batch plan");
  const int on = enable ? 1 : 0;
  if (on == plan->stamps) return ok();
  if (on && !plan->stamp_time) {
    const size_t nf = plan->fld.size();
    if (dev_alloc(plan, (void**)&plan->stamp_time, (nf + 1) * sizeof(unsigned long long)) ||
        dev_alloc(plan, (void**)&plan->stamp_cnt, nf * sizeof(unsigned int)))
      return FMM_ERR_OUT_OF_MEMORY;
    if (hipMemset(plan->stamp_time, 0, (nf + 1) * sizeof(unsigned long long)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(FMM_ERR_DEVICE, "hipMemset failed");
    }
  }
  // the captured graph holds the bottom kernel's arguments: capture again
  if (hipDeviceSynchronize() != hipSuccess) (void)hipGetLastError();
  if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  plan->gexec = nullptr;
  plan->graph = nullptr;
  plan->stamps = on;
  return ok();
}

int fmm_batch_field_ms(fmm_plan* plan, double* ms, int count) {
  if (!plan) return fail(FMM_ERR_INVALID_ARG, "plan is NULL");
  if (!plan->batch || !plan->stamps) return fail(FMM_ERR_INVALID_ARG, "timestamps are not enabled on this plan");
  const int nf = (int)plan->fld.size();
  if (!ms || count < nf) return fail(FMM_ERR_INVALID_ARG, "ms must hold %d doubles", nf);
  int rate_khz = 0;
  hipError_t e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, plan->device);
  if (e != hipSuccess || rate_khz <= 0) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "device wall-clock rate unavailable");
  }
  std::vector<unsigned long long> t(nf + 1);
  if ((e = hipDeviceSynchronize()) != hipSuccess ||
      (e = hipMemcpy(t.data(), plan->stamp_time, t.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost)) !=
          hipSuccess) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "reading timestamps failed: %s", hipGetErrorString(e));
  }
  for (int f = 0; f < nf; ++f) ms[f] = t[1 + f] >= t[0] ? (double)(t[1 + f] - t[0]) / rate_khz : -1.0;
  return ok();
}

int fmm_batch_info(const fmm_plan* plan, int* count, int* bottom_tile, int* m2l_grouping, double* tune_ms,
                   int ncand) {
  if (!plan) return fail(FMM_ERR_INVALID_ARG, "plan is NULL");
  if (count) *count = (int)plan->fld.size();
  if (bottom_tile) *bottom_tile = plan->tune.bz;
  if (m2l_grouping) *m2l_grouping = plan->tune.grp;
  for (int c = 0; tune_ms && c < ncand; ++c) tune_ms[c] = c < (int)plan->tune_ms.size() ? plan->tune_ms[c] : 0.0;
  return ok();
}

void fmm_plan_destroy(fmm_plan* plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  release(plan);
}

size_t fmm_plan_workspace_bytes(const fmm_plan* plan) { return plan ? plan->bytes : 0; }

int fmm_plan_info(const fmm_plan* plan, int* n, int* p, int* nmax, int* precision, int* finest_level) {
  if (!plan) return fail(FMM_ERR_INVALID_ARG, "plan is NULL");
  if (n) *n = plan->n;
  if (p) *p = plan->p;
  if (nmax) *nmax = plan->nmax;
  if (precision) *precision = plan->precision;
  if (finest_level) *finest_level = plan->F;
  return ok();
}

const char* fmm_last_error(void) { return g_err.c_str(); }

int fmm_last_status(void) { return g_status; }

int fmm_solve(fmm_plan* plan, const void* rho, void* phi, void* g, void* stream) {
  if (!plan) return fail(FMM_ERR_INVALID_ARG, "plan is NULL");
  if (plan->batch) return fail(FMM_ERR_INVALID_ARG, "batch plan: use fmm_batch_solve");
  if (!rho || !phi) return fail(FMM_ERR_INVALID_ARG, "rho and phi must be device pointers (got NULL)");
  if (rho == phi || (g && (g == rho || g == phi))) return fail(FMM_ERR_INVALID_ARG, "rho, phi and g must not alias");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (plan->check_finite) {
    int bad = 0;
    if ((e = fmm::launch_check_finite(plan, rho, &bad, s)) != hipSuccess)
      return fail(FMM_ERR_DEVICE, "finite check failed: %s", hipGetErrorString(e));
    if (bad) return fail(FMM_ERR_NONFINITE, "rho holds NaN or Inf");
  }
  fmm::StageScope whole(plan, fmm::ST_SOLVE, 0, s);
  if ((e = fmm::launch_solve(plan, fmm::IoArg{rho, phi, g, nullptr}, s)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "solve launch failed: %s", hipGetErrorString(e));
  }
  return ok();
}

// Workspace of a plan's backward pass: the scaled adjoint outputs of the
// level-F cells, one adjoint-local grid per level 3..F and the split
// transposed M2L's partial sums, all zeroed once (their margins and padding
// columns are never written); the adjoint multipoles reuse the plan's
// multipole grids.  Allocated by the first fmm_solve_backward call; on
// failure nothing stays allocated.
static int ensure_adjoint(fmm_plan* pl) {
  if (pl->adj_ready) return FMM_OK;
  fmm::AdjWs w;
  const size_t bytes0 = pl->bytes;
  auto bail = [&](int rc) {
    release_adj(w);
    pl->bytes = bytes0;
    return rc;
  };
  auto zalloc = [&](double** ptr, size_t bytes) -> int {
    if (dev_alloc(pl, (void**)ptr, bytes)) return FMM_ERR_OUT_OF_MEMORY;
    if (hipMemset(*ptr, 0, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(FMM_ERR_DEVICE, "hipMemset failed");
    }
    return FMM_OK;
  };
  const AdjLayout lay = adj_layout(pl);
  int rc;
  if ((rc = zalloc(&w.ybar, lay.ybar))) return bail(rc);
  for (int k = 3; k <= pl->F; ++k)
    if ((rc = zalloc(&w.abar[k], lay.abar[k]))) return bail(rc);
  if ((rc = zalloc(&w.part, (size_t)adj_part_doubles(pl) * sizeof(double)))) return bail(rc);
  if (lay.near && (rc = zalloc(&w.near, lay.near))) return bail(rc);
  const AdjSegs sg = adj_segments(pl, w);
  if ((rc = upload_arr(pl, w.m2lt[0], sg.lt[0])) || (rc = upload_arr(pl, w.m2lt[1], sg.lt[1])) ||
      (rc = upload_arr(pl, w.m2pt, sg.pt)) || (rc = upload_arr(pl, w.m2lt_red, sg.ltr)) ||
      (rc = upload_arr(pl, w.p2pt, sg.p2pt)))
    return bail(rc);
  pl->adj = w;
  pl->adj_ready = 1;
  return FMM_OK;
}

// Argument checks shared by both backward entry points.
static int check_backward_args(fmm_plan* plan, const void* dphi, const void* dg, void* drho) {
  if (!plan) return fail(FMM_ERR_INVALID_ARG, "plan is NULL");
  if (plan->batch) return fail(FMM_ERR_UNSUPPORTED, "the backward pass is provided for single-field plans");
  if (!dphi || !drho) return fail(FMM_ERR_INVALID_ARG, "dphi and drho must be device pointers (got NULL)");
  if (drho == dphi || (dg && (dg == drho || dg == dphi))) return fail(FMM_ERR_INVALID_ARG, "buffers must not alias");
  if (!plan->adj_tables) return fail(FMM_ERR_DEVICE, "the plan's backward tables were not built");
  return FMM_OK;
}

int fmm_solve_backward(fmm_plan* plan, const void* dphi, const void* dg, void* drho, void* stream) {
  if (int rc = check_backward_args(plan, dphi, dg, drho)) return rc;
  if (int rc = ensure_adjoint(plan)) return rc;
  fmm::StageScope whole(plan, fmm::ST_BACKWARD, 0, (hipStream_t)stream);
  hipError_t e = fmm::launch_backward(plan, plan->adj, dphi, dg, drho, (hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "backward launch failed: %s", hipGetErrorString(e));
  }
  return ok();
}

// The backward pass with its workspace laid out in the library's static
// device array instead of plan memory: [segment tables | Ybar | adjoint
// locals of levels F..3], each part 256-byte aligned, zeroed by a kernel on
// `stream` at every call; the transposed M2L writes its adjoint multipoles
// in place (no split partial sums).  Only kernels are enqueued.
int fmm_solve_backward_noalloc(fmm_plan* plan, const void* dphi, const void* dg, void* drho, void* stream) {
  if (int rc = check_backward_args(plan, dphi, dg, drho)) return rc;
  hipStream_t s = (hipStream_t)stream;
  const AdjLayout lay = adj_layout(plan);
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t at = fmm::kNoallocSegBytes;
  const size_t y_off = at;
  at += al(lay.ybar);
  size_t a_off[16] = {};
  for (int k = plan->F; k >= 3; --k) {
    a_off[k] = at;
    at += al(lay.abar[k]);
  }
  const size_t n_off = at;
  at += al(lay.near);
  if (at > fmm::kNoallocBytes)
    return fail(FMM_ERR_INVALID_ARG,
                "fmm_solve_backward_noalloc: this plan's backward workspace needs %zu bytes, more than the "
                "%zu-byte static workspace (use fmm_solve_backward)",
                at, fmm::kNoallocBytes);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) {
    (void)hipGetLastError();
    return fail(FMM_ERR_INVALID_ARG, "the current HIP device (%d) is not the plan's (%d)", dev, plan->device);
  }
  void* base = nullptr;
  hipError_t e = fmm::noalloc_base(dev, &base);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "static workspace address: %s", hipGetErrorString(e));
  }
  char* b = (char*)base;
  fmm::AdjWs w;
  w.ybar = (double*)(b + y_off);
  for (int k = 3; k <= plan->F; ++k) w.abar[k] = (double*)(b + a_off[k]);
  if (lay.near) w.near = (double*)(b + n_off);
  const AdjSegs sg = adj_segments(plan, w);
  fmm::Seg* sd = (fmm::Seg*)b;
  int used = 0;
  e = hipSuccess;
  for (auto pr : {std::make_pair(&w.m2lt[0], &sg.lt[0]), std::make_pair(&w.m2lt[1], &sg.lt[1]),
                  std::make_pair(&w.m2pt, &sg.pt), std::make_pair(&w.p2pt, &sg.p2pt)}) {
    fmm::SegTable& st = *pr.first;
    const SegArr& l = *pr.second;
    if (!l.n || e != hipSuccess) continue;
    st.dev = sd + used;
    st.nseg = l.n;
    st.blocks = (int)l.blocks;
    e = fmm::noalloc_put_segs(l.v, l.n, sd + used, s);
    used += l.n;
  }
  if (e == hipSuccess) e = fmm::noalloc_zero(w.ybar, (long long)((at - y_off) / sizeof(double)), s);
  // stage timing would create events: it is off for this call
  const int prof = plan->profiling;
  plan->profiling = 0;
  if (e == hipSuccess) e = fmm::launch_backward(plan, w, dphi, dg, drho, s);
  plan->profiling = prof;
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "backward launch failed: %s", hipGetErrorString(e));
  }
  return ok();
}

int fmm_profile_enable(fmm_plan* plan, int enable) {
  if (!plan) return fail(FMM_ERR_INVALID_ARG, "plan is NULL");
  plan->profiling = enable ? 1 : 0;
  return ok();
}

int fmm_profile_read(fmm_plan* plan, double* ms, int* launches, int nstages) {
  if (!plan) return fail(FMM_ERR_INVALID_ARG, "plan is NULL");
  if (nstages < 0) return fail(FMM_ERR_INVALID_ARG, "nstages < 0");
  for (int s = 0; s < nstages; ++s) {
    if (ms) ms[s] = 0.0;
    if (launches) launches[s] = 0;
  }
  int rc = FMM_OK;
  for (auto& r : plan->recs) {
    float t = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
      (void)hipGetLastError();
      rc = FMM_ERR_DEVICE;
    } else if (r.stage < nstages) {
      if (ms) ms[r.stage] += t;
      if (launches) launches[r.stage] += r.launches;
    }
    plan->event_pool.push_back(r.a);
    plan->event_pool.push_back(r.b);
  }
  plan->recs.clear();
  if (rc != FMM_OK) return fail(rc, "reading profile events failed");
  return ok();
}

const char* fmm_profile_stage_name(int stage) {
  return (stage >= 0 && stage < fmm::ST_COUNT) ? kStageNames[stage] : nullptr;
}

int fmm_multi_index(int P, int* out, size_t count) {
  if (P < 0 || P > fmm::PDMAX) return fail(FMM_ERR_INVALID_ARG, "P must be in [0, %d]", fmm::PDMAX);
  const int nt = fmm::nterms(P);
  if (!out || count < (size_t)(3 * nt)) return fail(FMM_ERR_INVALID_ARG, "out must hold %d ints", 3 * nt);
  for (int a = 0; a <= P; ++a)
    for (int b = 0; a + b <= P; ++b)
      for (int c = 0; a + b + c <= P; ++c) {
        const int t = fmm::mi_index(a, b, c);
        out[3 * t] = a;
        out[3 * t + 1] = b;
        out[3 * t + 2] = c;
      }
  ok();
  return nt;
}

int fmm_deposit_cic(int n, long long count, const double* pos, const double* mass, double* rho, void* stream) {
  const int L = ilog2_exact(n);
  if (L < 3 || L > 10) return fail(FMM_ERR_INVALID_ARG, "n must be a power of two in [8, 1024] (got %d)", n);
  if (count < 0) return fail(FMM_ERR_INVALID_ARG, "count must be >= 0 (got %lld)", count);
  if (count > 0 && (!pos || !mass || !rho)) return fail(FMM_ERR_INVALID_ARG, "pos, mass and rho must be device pointers");
  if (count > (long long)UINT32_MAX * 256) return fail(FMM_ERR_INVALID_ARG, "count %lld is too large", count);
  hipError_t e = fmm::launch_cic(n, count, pos, mass, rho, (hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "CIC launch failed: %s", hipGetErrorString(e));
  }
  return ok();
}

int fmm_fd_force(int n, const double* phi, double* f, void* stream) {
  const int L = ilog2_exact(n);
  if (L < 3 || L > 10) return fail(FMM_ERR_INVALID_ARG, "n must be a power of two in [8, 1024] (got %d)", n);
  if (!phi || !f) return fail(FMM_ERR_INVALID_ARG, "phi and f must be device pointers");
  const size_t N = (size_t)n * n * n;
  const char *pb = (const char*)phi, *fb = (const char*)f;
  if (pb < fb + 3 * N * sizeof(double) && fb < pb + N * sizeof(double))
    return fail(FMM_ERR_INVALID_ARG, "phi and f must not overlap");
  hipError_t e = fmm::launch_fd_force(n, phi, f, (hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(FMM_ERR_DEVICE, "force launch failed: %s", hipGetErrorString(e));
  }
  return ok();
}

int fmm_debug_expansions(fmm_plan* plan, int which, int level, double* out, size_t count) {
  if (!plan) return fail(FMM_ERR_INVALID_ARG, "plan is NULL");
  if (which != 0 && which != 1) return fail(FMM_ERR_INVALID_ARG, "which must be 0 or 1");
  const int lo = which == 0 ? 2 : 3;
  if (level < lo || level > plan->F) return fail(FMM_ERR_INVALID_ARG, "level %d outside [%d, %d]", level, lo, plan->F);
  if (which == 0 && level == plan->F && plan->dl == 1 && fmm::bottom_low(plan, plan->F))
    return fail(FMM_ERR_UNSUPPORTED, "a low-precision bottom keeps the level-%d multipoles in its compute type only", level);
  const fmm::Level& lv = plan->lev[level];
  const int nt = which == 0 ? plan->NMX : plan->NL;
  const int nch = (nt + 3) / 4;
  if (!out || count < (size_t)lv.ncell * nt) return fail(FMM_ERR_INVALID_ARG, "out must hold %lld doubles", lv.ncell * nt);
  const int nk = lv.nk;
  if (which == 0) {
    std::vector<double> host((size_t)nch * lv.ncellp * 4);
    hipError_t e = hipMemcpy(host.data(), lv.M, host.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(FMM_ERR_DEVICE, "copy failed: %s", hipGetErrorString(e));
    for (long long cidx = 0; cidx < lv.ncell; ++cidx) {
      const int c2 = (int)(cidx % nk), c1 = (int)((cidx / nk) % nk), c0 = (int)(cidx / ((long long)nk * nk));
      const long long src = ((long long)(c0 + 3) * lv.nkp + (c1 + 3)) * lv.nkp + (c2 + 3);
      for (int t = 0; t < nt; ++t) out[cidx * nt + t] = host[((size_t)(t >> 2) * lv.ncellp + src) * 4 + (t & 3)];
    }
    return ok();
  }
  if (level == plan->F && plan->lt_live)
    return fail(FMM_ERR_UNSUPPORTED, "a low-precision bottom keeps the level-%d locals in its compute type only", level);
  hipError_t fe = fmm::finish_locals(plan, level, nullptr);
  if (fe == hipSuccess) fe = hipDeviceSynchronize();
  if (fe != hipSuccess) return fail(FMM_ERR_DEVICE, "completing locals failed: %s", hipGetErrorString(fe));
  const int RS = fmm::loc_stride(plan->p), ns = nk / 2;
  std::vector<double> host((size_t)(lv.ncell / 8) * RS);
  hipError_t e = hipMemcpy(host.data(), lv.L, host.size() * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(FMM_ERR_DEVICE, "copy failed: %s", hipGetErrorString(e));
  for (long long cidx = 0; cidx < lv.ncell; ++cidx) {
    const int c2 = (int)(cidx % nk), c1 = (int)((cidx / nk) % nk), c0 = (int)(cidx / ((long long)nk * nk));
    const long long P = ((long long)(c0 >> 1) * ns + (c1 >> 1)) * ns + (c2 >> 1);
    const int q = ((c0 & 1) << 2) | ((c1 & 1) << 1) | (c2 & 1);
    for (int t = 0; t < nt; ++t) {
      int m = 0;
      while (fmm::nterms(m) <= t) ++m;
      out[cidx * nt + t] = host[(size_t)P * RS + fmm::m2l_col(q, t, m)];
    }
  }
  return ok();
}

}  // extern "C"
