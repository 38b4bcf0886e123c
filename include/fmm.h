/*
 * fmm.h -- C ABI of the MI355X (gfx950) unigrid fast-multipole Poisson solver
 * with isolated (vacuum) boundary conditions.
 *
 * Method: Lee & Teyssier, "A Scalable Fast Multipole Method Poisson Solver for
 * the RAMSES code: I. Unigrid Algorithm".  One upward pass (P2M on the leaf
 * cells, eq. (multipole); M2M through the FMM grids, eq. (M2M), Sec. 2.1) and
 * one downward pass (M2L over the fixed oct-shared interaction lists of
 * Sec. 2.2, eq. (M2L); L2L, eq. (L2L); and at the finest FMM level L2P, M2P
 * at the unigrid cell centres and the near-field direct sum, eq. (direct),
 * Sec. 2.3 and Sec. 4).  Cartesian expansions to order p; the finest FMM
 * grid sits delta_l levels above the unigrid (App. A): 1 (FMM-1, default) or
 * 2 (FMM-2, whose finest FMM cells hold 4^3 unigrid cells and whose near
 * field is the 27 x 64 cells of the adjacent ones).
 *
 * Conventions shared by every entry point
 *  - Grid: unit box [0,1]^3, n cells per axis, cell (i,j,k) centred at
 *    ((i+1/2)/n, (j+1/2)/n, (k+1/2)/n).  Arrays are C order, k fastest:
 *    rho[i][j][k], phi[i][j][k], g[3][i][j][k] (component-major).
 *  - Units: G = 1; the mass of a cell is rho * (1/n)^3.  phi is the
 *    potential sum_w m_w g(x - x_w) with the softened Green's function of
 *    eq. (direct) (g = -1/dx for the cell itself); g = -grad(phi) is the
 *    acceleration.
 *  - Precision: an FMM_FP64 plan takes and returns double; FMM_FP32 and
 *    FMM_BF16 plans take and return float (see fmm_precision).
 *  - Memory: rho, phi, g, dphi, dg and drho are caller-owned DEVICE pointers
 *    (hipMalloc / torch tensors on the plan's device), contiguous, not
 *    aliasing each other.  The plan owns its own workspace.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls only enqueue work; they return before it finishes.  A
 *    nonzero status reports an argument or launch error; errors inside
 *    kernels are not detected.
 *  - Concurrency: a plan's workspace is reused by every call; calls on one
 *    plan that overlap in time (two streams, two threads) race.  Use one plan
 *    per stream.
 *  - Errors: every call returns fmm_status (or NULL for constructors) and
 *    records a message readable with fmm_last_error() in the same thread.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_plan fmm_plan;

typedef enum {
  FMM_OK = 0,
  FMM_ERR_INVALID_ARG = -1,   /* bad size, order, pointer or option */
  FMM_ERR_UNSUPPORTED = -2,   /* well-formed but not provided (periodic BC, delta_l outside {1, 2},
                                 the backward pass of a batch plan, the FP64 export of a grid a
                                 plan keeps in a low compute type only) */
  FMM_ERR_OUT_OF_MEMORY = -3, /* device allocation failed */
  FMM_ERR_DEVICE = -4,        /* HIP runtime error (no device, launch failure) */
  FMM_ERR_NONFINITE = -5      /* rho holds NaN/Inf (only with check_finite) */
} fmm_status;

/*
 * Compute policy.  FMM_FP64: every step in double.  FMM_FP32 / FMM_BF16:
 * the dominant contractions (M2L on fine levels, M2P) run on the matrix cores
 * with FP32 / BF16 operands and FP32 accumulation, while the derivative
 * tables are computed in FP64 on the device and the coarse levels
 * (k <= coarse_fp64_levels) keep FP64 multipoles and locals; I/O is float.
 */
typedef enum { FMM_FP64 = 0, FMM_FP32 = 1, FMM_BF16 = 2 } fmm_precision;

typedef struct {
  int struct_size;          /* sizeof(fmm_options), for forward compatibility */
  int precision;            /* fmm_precision, default FMM_FP64 */
  int nmax;                 /* multipole order, -1 = p (default); 0 <= nmax <= p.  Multipoles
                               are truncated at nmax (Sec. 2.1); M2L and M2P then sum only
                               the kept terms */
  int coarse_fp64_levels;   /* mixed plans: levels k <= this stay FP64; default 4 */
  int delta_l;              /* level offset unigrid -> finest FMM grid: 1 (default) or 2
                               (FMM-2, App. A; n >= 16) */
  int check_finite;         /* nonzero: fmm_solve scans rho for NaN/Inf first (single-field plans) */
  int autotune;             /* batch plans: time the launch-shape candidates at creation; default 1 */
  int bottom_tile;          /* depth (level-F cells along z) of the bottom kernel's tiles: 0 = chosen
                               by the plan (default: 16, or 8 where 16-deep tiles would leave
                               compute units idle, or the autotuner's choice), 8 or 16 to force one
                               (delta_l = 2 plans take 16 only).  Results do not depend on it
                               beyond rounding order. */
  const char* autotune_cache; /* batch plans with autotune: path of a text file that remembers the
                               autotuner's choice per (GPU architecture, compute units, field sizes,
                               p, nmax, precision, delta_l, coarse_fp64_levels).  A plan whose key is
                               in the file takes that choice without timing; otherwise it times the
                               candidates and appends a line.  NULL (default) = always time.  A file
                               that cannot be read is treated as empty; one that cannot be written
                               is left alone (the plan is still created). */
} fmm_options;

/* Fill *opt with the defaults above.  Returns FMM_OK or FMM_ERR_INVALID_ARG. */
int fmm_options_default(fmm_options* opt);

/*
 * Create a plan for an n^3 unigrid solved to expansion order p.
 *   n: power of two, 8 <= n <= 1024 (the finest FMM grid, n/2 cells per axis,
 *      must hold at least one interaction list, Sec. 2.2).
 *   p: 1 <= p <= 8.
 *   isolated: must be 1; the paper's solver handles only isolated boundary
 *      conditions (Sec. 2), so 0 gives FMM_ERR_UNSUPPORTED.
 * Allocates the multipole/local pyramids on the current HIP device and
 * computes the FP64 Green's-function derivative tables there (the fixed
 * interaction geometry of Sec. 2.2).  Synchronous.  Returns NULL on error.
 */
fmm_plan* fmm_plan_create(int n, int p, int isolated);
fmm_plan* fmm_plan_create_ex(int n, int p, int isolated, const fmm_options* opt);

/* Release a plan and its device memory (synchronises the device).  NULL-safe. */
void fmm_plan_destroy(fmm_plan* plan);

/*
 * phi (and g, if not NULL) of the density rho: the solve of Sec. 2 (upward
 * pass P2M, M2M; M2L over the oct-shared lists of Sec. 2.2; downward pass
 * L2L; at the unigrid cells L2P, M2P and the direct near field, Sec. 4;
 * FMM-2 with delta_l = 2, App. A).  Enqueued on `stream`.
 * rho: n^3 values; phi: n^3; g: 3 n^3 or NULL.
 */
int fmm_solve(fmm_plan* plan, const void* rho, void* phi, void* g, void* stream);

/*
 * Vector-Jacobian product of fmm_solve (the transpose of the Sec. 2 solve,
 * FMM-1 and FMM-2): drho = d(<phi, dphi> + <g, dg>)/drho.
 * The solve is linear in rho, so no forward state is needed; the kernels run
 * the transposes of the forward passes in reverse order (P2P^T, L2P^T and
 * M2P^T, then L2L^T and M2L^T from the finest level up, M2M^T down, P2M^T).
 * dphi: n^3 (required); dg: 3 n^3 or NULL (treated as zero); drho: n^3.
 */
int fmm_solve_backward(fmm_plan* plan, const void* dphi, const void* dg, void* drho, void* stream);

/*
 * fmm_solve_backward for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, result and error codes as fmm_solve_backward
 * (up to the rounding order of the transposed M2L's sums), but the call
 * allocates nothing: the backward workspace (the scaled adjoint outputs of
 * the finest FMM cells and the adjoint locals of every level) is laid out in
 * one static device array of the library, 96 MiB (100663296 bytes) per
 * device, which each GPU that loads the library holds until the process
 * ends.  The call enqueues only kernels on `stream`: it clears the part of
 * the array it uses, writes its launch tables there and runs the backward
 * pass.  Plans whose workspace does not fit are rejected with
 * FMM_ERR_INVALID_ARG before anything is enqueued: with m = n / 2^delta_l
 * it needs
 *   4096 + ceil256(8^delta_l (m+6)^3 32) + sum_{k=3..F} ceil256(S (2^(k-1)+6)^3 8)
 *   (+ ceil256(16 (m+6)^3 32) for delta_l = 2)
 * bytes, S = 16 ceil(8 nterms(p) / 16), which fits n <= 32 at every p and
 * n = 64 up to p = 6 (FMM-2: n <= 64 at every p).  The array keeps the last
 * call's contents; every call on a device shares it, so calls that overlap in
 * time on one device (two streams, two threads, two plans) race, and only one
 * may be in flight per device.  The current device must be the plan's.
 * Stage profiling is not recorded for this call.  Single-field plans.
 */
int fmm_solve_backward_noalloc(fmm_plan* plan, const void* dphi, const void* dg, void* drho, void* stream);

/*
 * Batches: several density fields of (possibly different) sizes solved by
 * one plan, each stage of the solve being a single launch over the tiles of
 * every field (the unigrid solve of Sec. 2 applied per field; fields do not
 * interact).  The derivative and B-operand tables are shared.
 *
 * fmm_batch_plan_create: count fields, n[i] as for fmm_plan_create, one order
 *   p and one set of options (check_finite is not provided).  With
 *   opt->autotune (the default) the plan times each launch-shape candidate
 *   (bottom-kernel tile depth 16 or 8, wide or narrow M2L column groups) on
 *   zero densities of the batch and keeps the fastest; this allocates
 *   temporary I/O buffers for every field.  Synchronous.  NULL on error.
 * fmm_batch_solve: rho[i], phi[i] (and g[i], if g is not NULL and g[i] is not
 *   NULL) are device buffers of field i, laid out as for fmm_solve.  The first
 *   call captures the launch sequence into a HIP graph on a stream of the
 *   plan; every call launches that graph on `stream`.  The graph reads the
 *   buffer pointers from a device table: when a call passes different
 *   buffers than the previous one the library synchronises the device and
 *   uploads the table first.  With profiling enabled the stages are launched
 *   directly instead (so that their events are recorded).  fmm_solve and
 *   fmm_solve_backward reject batch plans; fmm_batch_solve rejects single ones.
 * fmm_batch_info: field count, the chosen bottom tile depth and M2L grouping
 *   (0 wide, 1 narrow), and the autotuner's mean milliseconds per candidate
 *   in the order (16, wide), (16, narrow), (8, wide), (8, narrow) for the
 *   first ncand entries of tune_ms (zeros without autotuning, and for the
 *   candidates a delta_l = 2 plan or a forced bottom_tile rules out; the
 *   cached figures when the choice came from opt->autotune_cache).  Any
 *   pointer may be NULL.
 */
fmm_plan* fmm_batch_plan_create(int count, const int* n, int p, int isolated, const fmm_options* opt);

/*
 * Per-field latency of batch solves.  fmm_batch_timestamps(plan, 1) makes
 * every following fmm_batch_solve record, on the device wall clock, its start
 * and the moment each field's last bottom-kernel block has written its
 * phi and g (the field's results are then complete); 0 stops it.  Switching
 * synchronises the device and drops the captured graph (the next solve
 * captures it again); the first enable allocates 12 bytes per field.
 * fmm_batch_field_ms(plan, ms, count) waits for the device and writes, for
 * each of the plan's fields, the milliseconds from the start of the last
 * timed solve to that field's completion (count must be at least the field
 * count).  Both return FMM_ERR_INVALID_ARG for a single-field plan.
 */
int fmm_batch_timestamps(fmm_plan* plan, int enable);
int fmm_batch_field_ms(fmm_plan* plan, double* ms, int count);
int fmm_batch_solve(fmm_plan* plan, const void* const* rho, void* const* phi, void* const* g, void* stream);
int fmm_batch_info(const fmm_plan* plan, int* count, int* bottom_tile, int* m2l_grouping, double* tune_ms,
                   int ncand);

/* Device bytes owned by the plan (tables and pyramids); 0 for NULL. */
size_t fmm_plan_workspace_bytes(const fmm_plan* plan);

/* Plan accessors: n, p, nmax, precision, finest FMM level F = log2(n) - delta_l. */
int fmm_plan_info(const fmm_plan* plan, int* n, int* p, int* nmax, int* precision, int* finest_level);

/* Last error message of the calling thread ("" if none).  Never NULL. */
const char* fmm_last_error(void);

/* Status code of the calling thread's last call (FMM_OK after a success);
 * the way to learn why a constructor returned NULL. */
int fmm_last_status(void);

/*
 * Inspection of the plan's intermediate state after fmm_solve has completed
 * on the device (the caller synchronises the stream first).  Synchronous;
 * it may finish pending work on the plan's buffers (the finest level keeps
 * only its M2L part during a solve), so call it only between solves on the
 * null stream's device.  Copies to HOST
 * memory `out`, as double, the scaled expansions the kernels keep:
 *   which = 0: multipoles of level `level` (2 <= level <= F), nterms(nmax) per cell,
 *              Mhat[a] = (-1)^|a| M[a] / (a! h^|a| dx^3), M[a] = sum m (x - c)^a
 *   which = 1: locals of level `level` (3 <= level <= F),
 *              Lhat[b] = h^(|b|+1) L[b] / dx^3, L[b] = d^b phi at the centre
 * with h = 2^-level the cell size and dx = 1/n.  Layout out[cell][term] with
 * cells of the level in C order and terms in the order of
 * fmm_multi_index().  `count` is the number of doubles `out` holds.
 * A plan whose finest level runs M2P in FP32 or BF16 (delta_l = 1) keeps
 * that level's multipoles and the M2L part of its locals in the compute type
 * only (the level below is formed from the density directly): level F
 * returns FMM_ERR_UNSUPPORTED there, for which = 0 and, unless the M2L of
 * that level splits its offset sums (small grids), for which = 1.
 */
int fmm_debug_expansions(fmm_plan* plan, int which, int level, double* out, size_t count);

/*
 * Cloud-in-cell deposition, the step before a solve (Sec. 3: the paper's test
 * particles reach the grid this way).  A particle of mass m at x adds
 * m W_c / dx^3 to the density of each cell c whose centre lies within one
 * cell of x along every axis, W_c = prod_d (1 - |x_d - x_c,d| / dx).
 *  n      cells per axis, a power of two in [8, 1024] (dx = 1/n)
 *  count  particles, >= 0
 *  pos    DEVICE, count x 3 doubles, (x, y, z) per particle in the unit box;
 *         x runs along the grid's first index
 *  mass   DEVICE, count doubles (G = 1)
 *  rho    DEVICE, n^3 doubles, C order; the densities are ADDED to it (zero
 *         it first for a fresh grid)
 * Shares of cells outside the box are dropped (isolated boundaries); a
 * particle with a coordinate that is not finite deposits nothing.  The
 * shares are added with FP64 atomics, so the last bits of a cell that several
 * particles reach can differ between runs.  Enqueued on `stream`.  Returns
 * FMM_OK, FMM_ERR_INVALID_ARG (n, count or a NULL pointer with count > 0) or
 * FMM_ERR_DEVICE (launch failure).
 */
int fmm_deposit_cic(int n, long long count, const double* pos, const double* mass, double* rho, void* stream);

/*
 * Force from a potential by finite differences, the step after a solve
 * (App. C: the host code differentiates phi with a 5-point stencil).  Along
 * each axis f = -dphi/dx by fourth-order differences over 5 cells, central
 * away from the walls and one-sided of the same order in the two layers
 * next to each wall (the box has no cells beyond them).  This is the host
 * code's force; fmm_solve's g is the exact gradient of the FMM potential.
 *  n    cells per axis, a power of two in [8, 1024]
 *  phi  DEVICE, n^3 doubles, C order (e.g. fmm_solve's phi)
 *  f    DEVICE, 3 x n^3 doubles, component-major like g; must not alias phi
 * Enqueued on `stream`.  Returns FMM_OK, FMM_ERR_INVALID_ARG (n, NULL or
 * aliasing pointers) or FMM_ERR_DEVICE (launch failure).
 */
int fmm_fd_force(int n, const double* phi, double* f, void* stream);

/*
 * Per-stage device timing with HIP events recorded on the solve's stream.
 * fmm_profile_enable(plan, 1) makes every following fmm_solve /
 * fmm_solve_backward record an event pair around each stage; 0 stops it.
 * fmm_profile_read waits for the recorded events, writes for each stage s <
 * nstages the summed milliseconds ms[s] and the number of kernel launches
 * launches[s] they cover (either may be NULL), and clears the record.
 * Stages: 0 P2M, 1 M2M, 2 M2L, 3 L2L, 4 bottom (M2P, L2P and near field),
 * 5 whole solve, 6 whole backward.  Names via fmm_profile_stage_name (NULL
 * past the last stage).  The plan owns the events; recording adds two event
 * records per stage to the stream.
 */
int fmm_profile_enable(fmm_plan* plan, int enable);
int fmm_profile_read(fmm_plan* plan, double* ms, int* launches, int nstages);
const char* fmm_profile_stage_name(int stage);

/* Multi-index order of the expansions: out[3*t + d] = exponent of axis d of
 * term t, for the nterms = (P+1)(P+2)(P+3)/6 terms of order <= P.  `out` holds
 * 3 * nterms ints.  Returns nterms, or FMM_ERR_INVALID_ARG. */
int fmm_multi_index(int P, int* out, size_t count);

#ifdef __cplusplus
}
#endif
#endif /* FMM_H */
