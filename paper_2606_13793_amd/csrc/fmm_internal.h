// Internal declarations of the MI355X unigrid FMM library.
//
// Scaled representation (all operators become level-independent matrices):
//   multipole of a level-s cell   Mhat[a] = (-1)^|a| M[a] / (a! h_s^|a| dx^3)
//   local of a level-k cell       Lhat[b] = h_k^(|b|+1) L[b] / dx^3
// with M[a] = sum m (x - c)^a, L[b] = d^b phi at the cell centre, h = cell
// size, dx = 1/n and m = rho dx^3.  Green's function derivatives are taken at
// the unit displacement Rhat = R / h_source, for which eq. (M2L) reads
//   Lhat_k[b] = 2^-(|b|+1) sum_a D[a+b](Rhat) Mhat_{k-1}[a]
// and M2P at the unigrid centres reads
//   phi += dx^2/2 sum_a D[a](Rhat) Mhat_F[a],  g_d += -dx/4 sum_a D[a+e_d](Rhat) Mhat_F[a].
//
// Multi-index order (graded): degree n = 0, 1, ...; inside a degree the x
// exponent ascends, then the y exponent ascends.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <algorithm>
#include <cstdint>
#include <vector>

namespace fmm {

constexpr int PMAX = 8;                   // highest expansion order
constexpr int PDMAX = PMAX + 1;           // highest derivative order (M2P gradient)
constexpr int NTMAX = (PDMAX + 1) * (PDMAX + 2) * (PDMAX + 3) / 6;  // 220

constexpr __host__ __device__ int nterms(int P) { return P < 0 ? 0 : (P + 1) * (P + 2) * (P + 3) / 6; }
constexpr __host__ __device__ int ndeg(int m) { return (m + 1) * (m + 2) / 2; }  // terms of degree m
// entries of the L2L coefficient lists: pairs (b, g) with |b| + |g| <= P
constexpr __host__ __device__ int l2l_entries(int P) {
  int e = 0;
  for (int m = 0; m <= P; ++m) e += ndeg(m) * nterms(P - m);
  return e;
}
// level-(k-1) cells whose child locals one k_l2l block forms
constexpr int L2L_ROWS = 16;

// index of (a, b, c) in the graded order
constexpr __host__ __device__ int mi_index(int a, int b, int c) {
  const int n = a + b + c;
  return nterms(n - 1) + a * (n + 1) - a * (a - 1) / 2 + b;
}

// ---------------------------------------------------------------------------
// M2L column layout: columns (child q, local term b) sorted by the degree m of
// b; inside a degree block the child is the slow index.  Each 16-column MFMA
// tile only needs the multipole terms with |a| <= p - (smallest m in tile),
// which keeps ~86% of the issued MACs useful at p = 6.
// ---------------------------------------------------------------------------
constexpr __host__ __device__ int m2l_ncol(int P) { return 8 * nterms(P); }
constexpr __host__ __device__ int m2l_ntiles(int P) { return (m2l_ncol(P) + 15) / 16; }
// row stride of the local arrays (columns padded to whole tiles)
constexpr __host__ __device__ int loc_stride(int P) { return 16 * m2l_ntiles(P); }
constexpr __host__ __device__ int m2l_col_degree(int col) {
  int m = 0;
  while (col >= 8 * nterms(m)) ++m;
  return m;
}
// column of (child q, local term index bt of degree m) in the M2L layout
constexpr __host__ __device__ int m2l_col(int q, int bt, int m) {
  return 8 * nterms(m - 1) + q * ndeg(m) + (bt - nterms(m - 1));
}
// number of K chunks (of KC multipole terms) tile t needs: terms |a| <= p - m
constexpr __host__ __device__ int m2l_tile_chunks(int P, int t, int KC = 4) {
  return (nterms(P - m2l_col_degree(16 * t)) + KC - 1) / KC;
}
// ---------------------------------------------------------------------------
// The parity-class convolutions of the matrix-core kernel (k_conv):
//   CV_M2L   forward M2L: rows = source cells P, K = multipole terms a,
//            N = local columns (q, b)          (tiles and chunks as above)
//   CV_M2LT  transposed M2L: rows = source cells J, K = adjoint local columns
//            (q, b) of the targets' parents, N = multipole terms a
//   CV_M2PT  transposed M2P: rows = level-F cells J, K = the 32 adjoint
//            outputs (q, o) of a target cell, N = multipole terms a
//   CV_M2PT2 the same for FMM-2 (App. A): K = the 256 adjoint outputs
//            (g, q, o) of the 64 unigrid cells of a target cell
//   CV_P2PT2 transposed near field of FMM-2: rows = level-F cells W, the 27
//            offsets of the adjacent cells, K = the 256 adjoint outputs of
//            an adjacent cell, N = the 64 unigrid (source) cells of W
// The interaction relation is symmetric (J is in the list of P iff P is in
// the list of J), so the first four walk the same per-parity offset lists;
// CV_P2PT2 walks the 27 neighbour offsets.
// ---------------------------------------------------------------------------
enum ConvOp { CV_M2L = 0, CV_M2LT = 1, CV_M2PT = 2, CV_M2PT2 = 3, CV_P2PT2 = 4, CV_NOPS = 5 };
constexpr int NP2P = 27;       // near-field offsets of a finest FMM cell
constexpr int NSLOT_P2P = 28;  // their B-table slots: 27 offsets + the null one
// offsets in a convolution's list, and the B-table slots they index
constexpr __host__ __device__ int conv_noff(int op) { return op == CV_P2PT2 ? NP2P : 189; }
constexpr __host__ __device__ int conv_nslot(int op) { return op == CV_P2PT2 ? NSLOT_P2P : 344; }
// output columns: local columns (M2L), multipole terms, or 64 unigrid cells
constexpr __host__ __device__ int conv_ncols(int op, int P) {
  return op == CV_M2L ? 8 * nterms(P) : (op == CV_P2PT2 ? 64 : nterms(P));
}
// degree of multipole term index a
constexpr __host__ __device__ int mi_degree(int a) {
  int m = 0;
  while (a >= nterms(m)) ++m;
  return m;
}
constexpr __host__ __device__ int conv_nk(int op, int P) {
  return op == CV_M2L ? nterms(P) : (op == CV_M2LT ? loc_stride(P) : (op == CV_M2PT ? 32 : 256));
}
constexpr __host__ __device__ int conv_ntiles(int op, int P) {
  return op == CV_M2L ? m2l_ntiles(P) : (conv_ncols(op, P) + 15) / 16;
}
constexpr __host__ __device__ int conv_tile_chunks(int op, int P, int t, int KC) {
  return op == CV_M2L ? m2l_tile_chunks(P, t, KC)
                      : (op == CV_M2LT ? (8 * nterms(P - mi_degree(16 * t)) + KC - 1) / KC
                                       : (conv_nk(op, P) + KC - 1) / KC);
}
constexpr __host__ __device__ int conv_frag_offset(int op, int P, int t, int KC) {
  int f = 0;
  for (int u = 0; u < t; ++u) f += conv_tile_chunks(op, P, u, KC);
  return f;
}
constexpr __host__ __device__ int conv_nfrags(int op, int P, int KC) {
  return conv_frag_offset(op, P, conv_ntiles(op, P), KC);
}
// launch groups of tiles: at most MAXT tiles (accumulator registers) and, for
// the forward M2L, at most MAXB fragment chunks (balanced launches)
constexpr int conv_group_end(int op, int P, int t0, int KC, int MAXT, int MAXB) {
  int nt = 0, nb = 0, t = t0;
  while (t < conv_ntiles(op, P)) {
    const int c = conv_tile_chunks(op, P, t, KC);
    if (nt > 0 && (nt + 1 > MAXT || (op == CV_M2L && nb + c > MAXB))) break;
    ++nt;
    nb += c;
    ++t;
  }
  return t;
}
constexpr int conv_group_start(int op, int P, int g, int KC, int MAXT, int MAXB) {
  int t = 0;
  for (int i = 0; i < g; ++i) t = conv_group_end(op, P, t, KC, MAXT, MAXB);
  return t;
}
constexpr int conv_ngroups(int op, int P, int KC, int MAXT, int MAXB) {
  int g = 0, t = 0;
  while (t < conv_ntiles(op, P)) { t = conv_group_end(op, P, t, KC, MAXT, MAXB); ++g; }
  return g;
}

// number of interaction-list offsets per parity class (6^3 - 3^3); the
// device lists hold NLIST_PAD entries per class, entry NLIST being a null
// offset (zero weights) used to pad pairs of offsets.  Entries are packed:
// bits 0-8 offset index dd (0..342, 343 = null), then 3 bits each of
// d0 + 3, d1 + 3, d2 + 3.
constexpr int NLIST = 189;
constexpr int NLIST_PAD = 192;
constexpr int NSLOT = 344;  // B-table offset slots: 343 offsets + the null one
__host__ __device__ inline int dl_dd(int e) { return e & 511; }
__host__ __device__ inline int dl_d0(int e) { return ((e >> 9) & 7) - 3; }
__host__ __device__ inline int dl_d1(int e) { return ((e >> 12) & 7) - 3; }
__host__ __device__ inline int dl_d2(int e) { return ((e >> 15) & 7) - 3; }

// ---------------------------------------------------------------------------
// device state of one plan
// ---------------------------------------------------------------------------
struct Level {
  int k = 0;          // level: 2^k cells per axis
  int nk = 0;         // cells per axis
  int nkp = 0;        // padded cells per axis (multipole grids: nk + 6)
  long long ncell = 0;   // nk^3
  long long ncellp = 0;  // nkp^3
  void* M = nullptr;  // multipoles, chunked [NC][ncellp][4], zero halo of 3 cells
  // mixed-precision plans: the same multipoles rounded to the compute type of
  // the kernels that read this level, chunked [ceil(NM/KC)][ncellp][KC] with
  // KC the type's K chunk (16 BF16 / 4 FP32 terms), zero halo; null where no
  // low-precision kernel reads the level
  void* Mt = nullptr;
  // locals of level k >= 3, stored per parent cell P (level k-1) in M2L
  // column order: L[P][m2l_col(q, b)] = Lhat of child 2P + q, term b;
  // row stride loc_stride(p)
  void* L = nullptr;
  // the finest level's M2L part in the compute type of a low-precision
  // bottom kernel (FMM-1), in the layout of L, in place of L (null then);
  // null elsewhere.  Only the bottom kernel reads it, and it rounds its
  // operands to that type anyway.
  void* Lt = nullptr;
};

// one density field of a plan (a single-field plan has one)
struct Field {
  int n = 0, L = 0, F = 0;  // unigrid cells per axis, log2 n, finest FMM level L - 1
  double dx = 0.0;
  Level lev[16];
};

// I/O buffers of one field for one call
struct Io {
  const void* rho;
  void* phi;
  void* g;
};
// I/O as a kernel argument: a single field passes its buffers directly, a
// batch points at a device table indexed by field
struct IoArg {
  const void* rho;
  void* phi;
  void* g;
  const Io* tab;
};

// One segment of a launch that spans several grids (levels and/or fields):
// blocks [first_block, next segment's first_block) work on this grid.  The
// fields' meaning depends on the kernel (see each kernel).
struct Seg {
  int first_block;
  int n;      // grid cells per axis
  int tpa;    // tiles per axis (x and y)
  int field;  // index into the I/O table
  int tz;     // tiles along z
  int split;  // convolutions: blocks sharing one tile, each summing a slice of the offsets
  long long count;  // reductions: values per part
  const double* a;
  double* b;
  const double* c;
  const double* d;
  void* t;  // mixed precision: the typed copy of a (convolutions, bottom) or of b (P2M, M2M), or null
  // M2L into, and the bottom kernel reading, the finest level of a
  // low-precision bottom (FMM-1): those locals in the compute type, which
  // then replace b (M2L) and c (bottom); null otherwise
  void* u;
};
// a segment table in device memory, plus its launch size
struct SegTable {
  Seg* dev = nullptr;
  int nseg = 0;
  int blocks = 0;
  int cz = 16;  // k_conv sites: tile depth along z (8 when every grid is at most 8 deep)
};

// Workspace of one backward pass: the scaled adjoint outputs of the level-F
// cells, the adjoint locals of levels 3..F and, when the transposed M2L
// splits its offset sums over blocks, their partial sums; plus the segment
// tables of the transposed convolutions, which point into it.  A plan owns
// one (fmm_solve_backward); fmm_solve_backward_noalloc lays one out in the
// library's static workspace for each call.
struct AdjWs {
  double* ybar = nullptr;    // [YC][(nF+6)^3][4], YC = 8^dl chunks of (phi, gx, gy, gz)
  double* abar[16] = {};     // level k: [loc_stride/4][(2^(k-1)+6)^3][4]
  double* part = nullptr;    // split partial sums of the transposed M2L (null: unsplit)
  double* near = nullptr;    // FMM-2: the near-field transpose per finest cell, [16][(nF+6)^3][4]
  SegTable m2lt[2], m2pt, m2lt_red, p2pt;
};
// Static workspace of fmm_solve_backward_noalloc (bytes per device) and the
// most segments its tables hold.
constexpr size_t kNoallocBytes = (size_t)96 << 20;
constexpr size_t kNoallocSegBytes = 4096;
constexpr int kMaxAdjSegs = 12;

// launch-shape choices picked by the batch autotuner
struct Tuning {
  int bz = 16;   // bottom tile depth (8 or 16 level-F cells)
  int grp = 0;   // M2L column grouping: 0 wide groups, 1 narrow groups
};

}  // namespace fmm

namespace fmm {
enum Stage { ST_P2M = 0, ST_M2M, ST_M2L, ST_L2L, ST_BOTTOM, ST_SOLVE, ST_BACKWARD, ST_COUNT };
struct StageRec {
  int stage;
  int launches;
  hipEvent_t a, b;
};
}  // namespace fmm

struct fmm_plan {
  int n = 0, p = 0, nmax = 0, L = 0, F = 0;  // of field 0 (the only field of a single plan)
  int dl = 1;  // levels between the finest FMM level and the unigrid (F = L - dl)
  int precision = 0;
  int coarse_fp64_levels = 4;
  int check_finite = 0;
  int force_bz = 0;  // bottom tile depth forced by the caller (0 = the plan's choice)
  int device = 0;
  int cus = 256;  // compute units of the device
  double dx = 0.0;
  // NM multipole terms of order p in the grids and kernels (NC chunks of 4);
  // NMX = terms of order nmax, the ones kept (the others stay zero)
  int NM = 0, NC = 0, NL = 0, NCL = 0, ND = 0, NMX = 0;
  std::vector<fmm::Field> fld;  // the fields; fld[0].lev are field 0's grids
  int maxF = 0;
  fmm::Level* lev = nullptr;    // fld[0].lev
  double* dtab = nullptr;   // [343][8][ND] D[g](Rhat) in FP64
  double* dtab2 = nullptr;  // dl = 2: [343][64][ND] the M2P's D[g](Rhat)
  int* dlists = nullptr;    // [8][NLIST_PAD] packed interaction offsets per parity
  // matrix-core B operands in fragment order, per compute type (index
  // 0 = FP64, 1 = FP32, 2 = BF16); only the types a plan uses are built
  void* wm2p[3] = {nullptr, nullptr, nullptr};   // M2P
  void* wl2p[3] = {nullptr, nullptr, nullptr};   // L2P of the own local
  void* wl2p2[3] = {nullptr, nullptr, nullptr};  // L2P from the parent level
  void* wp2p[3] = {nullptr, nullptr, nullptr};   // near field
  void* wm2l[3] = {nullptr, nullptr, nullptr};   // M2L
  // adjoint tables (built with every single-field plan) and workspace
  // (allocated by the first fmm_solve_backward call)
  int adj_tables = 0;           // the tables below are built
  int adj_ready = 0;            // `adj` is allocated
  fmm::AdjWs adj;
  double* adj_l2p = nullptr;    // [G][NL][32]     L2P coefficients (G = 8^(dl-1) groups of 8 unigrid cells)
  double* adj_l2p2 = nullptr;   // [G][8][NL][32]  parent-level L2P coefficients
  void* wt_m2l[3] = {nullptr, nullptr, nullptr};  // transposed M2L B fragments
  void* wt_m2p[3] = {nullptr, nullptr, nullptr};  // transposed M2P B fragments (CV_M2PT2 for dl = 2)
  void* wt_p2p[3] = {nullptr, nullptr, nullptr};  // dl = 2: transposed near field B fragments
  int* dlists_p2p = nullptr;    // dl = 2: [8][NLIST_PAD] the 27 neighbour offsets (+ null) per parity
  int* m2m_start = nullptr;     // M2M coefficient lists (CSR over multipole terms)
  int* m2m_off = nullptr;       // 8 b + parity pattern of g, for b + g = a
  double* m2m_coef = nullptr;   // 2^-|b| 4^-|g| / g!
  int* m2mt_start = nullptr;    // transposed M2M lists: CSR over (b, parity pattern of g)
  int* m2mt_a = nullptr;        // a = b + g
  double* m2mt_coef = nullptr;  // 2^-|b| 4^-|g| / g!
  int* l2l_start = nullptr;     // L2L coefficient lists (CSR over (local term, parity of g))
  int* l2l_idx = nullptr;       // index of the term b+g
  double* l2l_coef = nullptr;
  int* flag = nullptr;      // device scratch flag (finite check)
  // launch schedule: segment tables of every launch site, built with the plan
  fmm::SegTable s_p2m;
  fmm::SegTable s_p2m2;             // FMM-1: level F - 1 formed from the unigrid (64 cells each)
  bool lt_live = false;             // the M2L writes the finest locals in the compute type (Level::Lt)
  fmm::SegTable s_m2m[16];          // M2M into level k - 1 (index k)
  fmm::SegTable s_conv[2];          // forward M2L: [0] FP64 levels, [1] low-precision levels
  fmm::SegTable s_l2l[16];          // L2L into level k (index k)
  fmm::SegTable s_bot[2][2];        // bottom [FP64 | low][tile depth 16 | 8]
  fmm::SegTable s_red[2];           // reductions of split forward M2L partial sums
  double* conv_part = nullptr;      // partial sums of split forward M2L segments
  // per convolution kind and compute type: (K chunks, first fragment) of
  // every column tile, zero-padded past the last tile
  int* tiletab[fmm::CV_NOPS][3] = {};
  // batches
  int batch = 0;                    // nonzero for fmm_batch_plan_create plans
  fmm::Io* io = nullptr;            // device I/O table, one entry per field
  std::vector<fmm::Io> io_last;     // what the table holds
  fmm::Tuning tune;
  std::vector<double> tune_ms;      // autotuner timings (ms) of each candidate
  int tune_cached = 0;              // the choice came from the autotune cache file
  // per-field completion times (fmm_batch_timestamps): stamp_time[0] the
  // solve's start, stamp_time[1 + f] the end of field f's last bottom block
  // (device wall clock), stamp_cnt[f] the field's finished bottom blocks
  int stamps = 0;
  unsigned long long* stamp_time = nullptr;
  unsigned int* stamp_cnt = nullptr;
  hipStream_t cap_stream = nullptr; // stream the batch graph is captured on
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  size_t bytes = 0;
  // stage profiling
  int profiling = 0;
  std::vector<fmm::StageRec> recs;
  std::vector<hipEvent_t> event_pool;
};

namespace fmm {
// Everything that depends on the expansion order lives in one translation
// unit per order (fmm_p<P>.hip) and is reached through Impl<P>.
template <int P>
struct Impl {
  static hipError_t upload_constants();
  static hipError_t tables(fmm_plan* pl, hipStream_t s);           // derivative and B tables
  static hipError_t solve(fmm_plan* pl, IoArg io, hipStream_t s);  // every field of the plan
  static hipError_t backward(fmm_plan* pl, const AdjWs& w, const void* dphi, const void* dg, void* drho,
                             hipStream_t s);
  static hipError_t adjoint_tables(fmm_plan* pl, hipStream_t s);
  static hipError_t finish_locals(fmm_plan* pl, int level, hipStream_t s);
  static hipError_t check_finite(fmm_plan* pl, const void* rho, int* host_flag, hipStream_t s);
};
extern template struct Impl<1>;
extern template struct Impl<2>;
extern template struct Impl<3>;
extern template struct Impl<4>;
extern template struct Impl<5>;
extern template struct Impl<6>;
extern template struct Impl<7>;
extern template struct Impl<8>;

// the order's entry points, by value of p
hipError_t upload_constants(int p);
hipError_t launch_tables(fmm_plan* pl, hipStream_t s);
// cloud-in-cell deposition (fmm_deposit.hip): rho[n^3] += the CIC densities
// of `count` particles
hipError_t launch_cic(int n, long long count, const double* pos, const double* mass, double* rho, hipStream_t s);
// finite-difference force (fmm_force.hip): f[3][n^3] = -grad(phi) by 5-cell differences
hipError_t launch_fd_force(int n, const double* phi, double* f, hipStream_t s);
hipError_t launch_solve(fmm_plan* pl, IoArg io, hipStream_t s);
hipError_t launch_backward(fmm_plan* pl, const AdjWs& w, const void* dphi, const void* dg, void* drho,
                           hipStream_t s);
// the static workspace of fmm_solve_backward_noalloc on the current device
// (fmm_noalloc.hip): its device address, a zero fill and a segment upload
// that record only kernels on the stream
hipError_t noalloc_base(int device, void** base);
hipError_t noalloc_zero(double* p, long long count, hipStream_t s);
hipError_t noalloc_put_segs(const Seg* segs, int count, Seg* dst, hipStream_t s);
hipError_t launch_adjoint_tables(fmm_plan* pl, hipStream_t s);
hipError_t launch_check_finite(fmm_plan* pl, const void* rho, int* host_flag, hipStream_t s);
// completes the stored locals of `level` of field 0 (the finest level keeps
// only its M2L part during a solve); used before inspecting them
hipError_t finish_locals(fmm_plan* pl, int level, hipStream_t s);

// segment tables of a plan's launch sites (fields, levels and tuning known)
int build_schedule(fmm_plan* pl);
// which levels run in which compute type (same rule for every field)
inline bool bottom_low(const fmm_plan* pl, int F) { return pl->precision != 0 && F > pl->coarse_fp64_levels; }
bool finest_locals_typed(const fmm_plan* pl, const Field& fd);
inline int m2l_low_from(const fmm_plan* pl) {
  return pl->precision == 0 ? 64 : (pl->coarse_fp64_levels + 1 > 3 ? pl->coarse_fp64_levels + 1 : 3);
}
// whether the multipoles of level k (of a field with finest level F) get a
// copy in the compute type: the low-precision bottom reads level F, the
// low-precision M2L into level k + 1 reads level k
inline bool typed_level(const fmm_plan* pl, int F, int k) {
  if (pl->precision == 0) return false;
  return (k == F && bottom_low(pl, F)) || (k < F && k + 1 >= m2l_low_from(pl));
}

// Records an event pair around a stage when the plan is profiling.
class StageScope {
 public:
  StageScope(fmm_plan* pl, int stage, int launches, hipStream_t s);
  ~StageScope();
  StageScope(const StageScope&) = delete;
  StageScope& operator=(const StageScope&) = delete;

 private:
  fmm_plan* pl_;
  hipStream_t s_;
  int idx_ = -1;
};
}  // namespace fmm
