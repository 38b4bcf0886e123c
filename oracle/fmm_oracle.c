/*
 * Plain FP64 CPU oracle for the unigrid FMM Poisson solve with isolated
 * boundary conditions (Lee & Teyssier, "A Scalable Fast Multipole Method
 * Poisson Solver for the RAMSES code: I. Unigrid Algorithm").
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant generator with the HIP solver, and the solver
 * never calls it.
 *
 * Everything is written in the paper's notation with physical (unscaled)
 * quantities, one operator at a time, in the order of Sec. 2:
 *
 *   P2M   eq. (multipole), Sec. 2.1 -- moments of the leaf cells
 *   M2M   eq. (M2M), Sec. 2.1       -- shift of a child's moments to its
 *                                      parent's centre, summed
 *   M2L   eq. (M2L), Sec. 2.3       -- interaction list of Sec. 2.2
 *   L2L   eq. (L2L), Sec. 2.3
 *   L2P / M2P / P2P at the finest FMM level, Sec. 2.3 and Sec. 4
 *         (the finest intermediate field is evaluated at the unigrid cell
 *          centres directly, the near field by eq. (direct))
 *
 * Multi-index notation: for a = (ax, ay, az), x^a = x^ax y^ay z^az,
 * a! = ax! ay! az!, |a| = ax + ay + az.  The paper's symmetric outer-product
 * tensors (after Dehnen 2002) are stored by their distinct components:
 *   multipole  M[a] = sum_i m_i (x_i - c)^a
 *   local      L[b] = d^b Phi / dx^b at the expansion centre
 *   D[g](R)    = d^g g(R) / dR^g with g(R) = -1/|R|
 * and the paper's contraction  (1/n!) T_{n+m} (.) M_n  becomes
 * sum_{|a|=n} D[a+b] M[a] / a!.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *  - R in eq. (M2L) is x_target - x_source: with the (-1)^n factor of the
 *    equation this is the only sign for which M2L followed by L2P
 *    reproduces -m/|x - y|.
 *  - Multipoles run to order nmax (default p) and the M2L truncation is
 *    |a| + |b| <= p, |a| <= nmax: the full order-p Cartesian scheme the
 *    paper says it follows; p = 3, nmax = 2 is the paper's own setting.
 *  - P2M forms moments about each finest FMM cell's centre.  The paper forms
 *    them about the origin, sums them and shifts them with eq. (M2M); both
 *    are the same polynomial identity, but origin moments of order 6 lose
 *    every digit to cancellation on fine grids.
 *  - Interaction lists are shared by the 2^3 cells of an oct (Sec. 2.2,
 *    Fig. 1): a target T at level k takes M2L from every source J at level
 *    k-1 with parent(J) adjacent to parent(parent(T)) and J not adjacent to
 *    parent(T), about T's own centre.  At the finest level the same list of
 *    T_F(u) is summed by M2P at each unigrid centre u, and the near field is
 *    every unigrid cell whose finest FMM cell is adjacent to T_F(u).
 *  - Cells outside the box do not exist (vacuum); lists are clipped.
 *  - Softening, eq. (direct): g = -1/dx only for the cell itself on the grid
 *    (face neighbours sit at exactly dx where both branches agree); the
 *    acceleration of a cell on itself is zero.
 *  - The acceleration returned is -grad(phi) of the FMM potential: L2P
 *    differentiates the local polynomial, M2P uses D up to order nmax + 1,
 *    P2P is the exact pairwise force.
 *  - Level k has 2^k cells per axis; the finest FMM level is F = L - dl,
 *    dl = 1 (FMM-1) or 2 (FMM-2), App. A: a finest FMM cell holds 8^dl
 *    unigrid cells and the near field of a unigrid cell is the 27 x 8^dl
 *    cells of the finest FMM cells adjacent to its own (Sec. 4); locals
 *    exist from level 3, L2L from level 4.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double wall_seconds(void) {
#ifdef _OPENMP
  return omp_get_wtime();
#else
  return 0.0;
#endif
}

#define OR_PMAX 9     /* highest derivative order needed: p + 1, p <= 8 */
#define OR_NTMAX 220  /* number of multi-indices with |a| <= 9 */

typedef long long i64;

/* ------------------------------------------------------------------ */
/* multi-indices                                                        */
/* ------------------------------------------------------------------ */
typedef struct {
  int P, nt;
  int e[OR_NTMAX][3];
  int deg[OR_NTMAX];
  double fact[OR_NTMAX];
  int idx[OR_PMAX + 1][OR_PMAX + 1][OR_PMAX + 1];
} mindex;

static double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= (double)i;
  return f;
}

static int nterms(int P) { return (P + 1) * (P + 2) * (P + 3) / 6; }

/* graded order: degree 0, then degree 1, ...; inside a degree ax descends,
   then ay descends */
static void mi_init(mindex *m, int P) {
  memset(m, 0, sizeof(*m));
  for (int a = 0; a <= OR_PMAX; ++a)
    for (int b = 0; b <= OR_PMAX; ++b)
      for (int c = 0; c <= OR_PMAX; ++c) m->idx[a][b][c] = -1;
  int t = 0;
  for (int n = 0; n <= P; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) {
        int c = n - a - b;
        m->e[t][0] = a; m->e[t][1] = b; m->e[t][2] = c;
        m->deg[t] = n;
        m->fact[t] = factorial(a) * factorial(b) * factorial(c);
        m->idx[a][b][c] = t;
        ++t;
      }
  m->P = P;
  m->nt = t;
}

static double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

static double mono(const double v[3], const int e[3]) {
  return ipow(v[0], e[0]) * ipow(v[1], e[1]) * ipow(v[2], e[2]);
}

static double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  return factorial(n) / (factorial(k) * factorial(n - k));
}

/* ------------------------------------------------------------------ */
/* derivatives of the Green's function                                 */
/* ------------------------------------------------------------------ */
/*
 * D[g](R) = d^g (-1/|R|) for |g| <= P, by the McMurchie-Davidson Hermite
 * recurrence in its point-charge limit (McMurchie & Davidson 1978):
 *   H^(n)_000 = (-1)^n (2n-1)!! / |R|^(2n+1)
 *   H^(n)_{t+1,u,v} = t H^(n+1)_{t-1,u,v} + X H^(n+1)_{t,u,v}   (same in u, v)
 * and d^(t,u,v) (1/|R|) = H^(0)_tuv.
 */
static void dtensor(const double R[3], const mindex *mi, int P, double *D) {
  static const int S = OR_PMAX + 1;
  double H[OR_PMAX + 1][OR_PMAX + 1][OR_PMAX + 1][OR_PMAX + 1];
  (void)S;
  const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  const double r = sqrt(r2);
  double dfact = 1.0; /* (2n-1)!! */
  double rp = 1.0 / r;
  for (int n = 0; n <= P; ++n) {
    if (n > 0) { dfact *= (double)(2 * n - 1); rp /= r2; }
    H[n][0][0][0] = ((n & 1) ? -1.0 : 1.0) * dfact * rp;
  }
  for (int s = 1; s <= P; ++s)
    for (int t = s; t >= 0; --t)
      for (int u = s - t; u >= 0; --u) {
        int v = s - t - u;
        for (int n = 0; n + s <= P; ++n) {
          double h;
          if (t > 0)
            h = (t > 1 ? (t - 1) * H[n + 1][t - 2][u][v] : 0.0) + R[0] * H[n + 1][t - 1][u][v];
          else if (u > 0)
            h = (u > 1 ? (u - 1) * H[n + 1][t][u - 2][v] : 0.0) + R[1] * H[n + 1][t][u - 1][v];
          else
            h = (v > 1 ? (v - 1) * H[n + 1][t][u][v - 2] : 0.0) + R[2] * H[n + 1][t][u][v - 1];
          H[n][t][u][v] = h;
        }
      }
  for (int i = 0; i < nterms(P); ++i)
    D[i] = -H[0][mi->e[i][0]][mi->e[i][1]][mi->e[i][2]];
}

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */
static double centre(int i, int k) { return ((double)i + 0.5) / (double)(1 << k); }

static i64 lin(int i, int j, int l, int nk) { return ((i64)i * nk + j) * nk + l; }

static int inside(int i, int j, int l, int nk) {
  return i >= 0 && j >= 0 && l >= 0 && i < nk && j < nk && l < nk;
}

static int adjacent(int a0, int a1, int a2, int b0, int b1, int b2) {
  return abs(a0 - b0) <= 1 && abs(a1 - b1) <= 1 && abs(a2 - b2) <= 1;
}

/* J (level s) is in the interaction list of P (level s): parent(J) adjacent to
   parent(P) and J not adjacent to P (Sec. 2.2).  Both inside the box. */
static int in_list(int p0, int p1, int p2, int j0, int j1, int j2) {
  return adjacent(p0 >> 1, p1 >> 1, p2 >> 1, j0 >> 1, j1 >> 1, j2 >> 1) &&
         !adjacent(p0, p1, p2, j0, j1, j2);
}

/* ------------------------------------------------------------------ */
/* operators on one cell                                               */
/* ------------------------------------------------------------------ */
/* eq. (multipole): M[a] += m v^a, v = x_cell - centre */
static void op_p2m(const mindex *mi, int ntM, double m, const double v[3], double *M) {
  for (int a = 0; a < ntM; ++a) M[a] += m * mono(v, mi->e[a]);
}

/* eq. (M2M): moments of a child about its centre, shifted to the parent:
   Mp[a] += sum_{b <= a} C(a,b) d^(a-b) Mc[b], d = c_child - c_parent */
static void op_m2m(const mindex *mi, int ntM, const double d[3], const double *Mc, double *Mp) {
  for (int a = 0; a < ntM; ++a) {
    const int *ea = mi->e[a];
    double s = 0.0;
    for (int b = 0; b < ntM; ++b) {
      const int *eb = mi->e[b];
      if (eb[0] > ea[0] || eb[1] > ea[1] || eb[2] > ea[2]) continue;
      int g[3] = {ea[0] - eb[0], ea[1] - eb[1], ea[2] - eb[2]};
      double c = binom(ea[0], eb[0]) * binom(ea[1], eb[1]) * binom(ea[2], eb[2]);
      s += c * mono(d, g) * Mc[b];
    }
    Mp[a] += s;
  }
}

/* eq. (M2L): L[b] += sum_{|a| <= min(nmax, p-|b|)} (-1)^|a| / a! D[a+b](R) M[a] */
static void op_m2l(const mindex *mi, int p, int nmax, const double *D, const double *M, double *L) {
  const int ntL = nterms(p), ntM = nterms(nmax);
  for (int b = 0; b < ntL; ++b) {
    const int *eb = mi->e[b];
    double s = 0.0;
    for (int a = 0; a < ntM; ++a) {
      if (mi->deg[a] + mi->deg[b] > p) continue;
      const int *ea = mi->e[a];
      int g = mi->idx[ea[0] + eb[0]][ea[1] + eb[1]][ea[2] + eb[2]];
      double sg = (mi->deg[a] & 1) ? -1.0 : 1.0;
      s += sg / mi->fact[a] * D[g] * M[a];
    }
    L[b] += s;
  }
}

/* eq. (L2L): Lc[b] += sum_{|b+g| <= p} Lp[b+g] a^g / g!, a = c_child - c_parent */
static void op_l2l(const mindex *mi, int p, const double a[3], const double *Lp, double *Lc) {
  const int ntL = nterms(p);
  for (int b = 0; b < ntL; ++b) {
    const int *eb = mi->e[b];
    double s = 0.0;
    for (int g = 0; g < ntL; ++g) {
      if (mi->deg[b] + mi->deg[g] > p) continue;
      const int *eg = mi->e[g];
      int bg = mi->idx[eb[0] + eg[0]][eb[1] + eg[1]][eb[2] + eg[2]];
      s += Lp[bg] * mono(a, eg) / mi->fact[g];
    }
    Lc[b] += s;
  }
}

/* L2P: phi += sum_b L[b] v^b / b!,  g_d -= sum_{b_d >= 1} L[b] v^(b-e_d)/(b-e_d)! */
static void op_l2p(const mindex *mi, int p, const double v[3], const double *L, double *phi, double g[3]) {
  const int ntL = nterms(p);
  for (int b = 0; b < ntL; ++b) {
    const int *eb = mi->e[b];
    *phi += L[b] * mono(v, eb) / mi->fact[b];
    for (int d = 0; d < 3; ++d) {
      if (eb[d] == 0) continue;
      int e[3] = {eb[0], eb[1], eb[2]};
      e[d] -= 1;
      double f = factorial(e[0]) * factorial(e[1]) * factorial(e[2]);
      g[d] -= L[b] * mono(v, e) / f;
    }
  }
}

/* M2P: phi += sum_a (-1)^|a|/a! D[a](R) M[a],  g_d -= sum_a (-1)^|a|/a! D[a+e_d](R) M[a],
   R = x_target - c_source; D holds orders up to nmax + 1 */
static void op_m2p(const mindex *mi, int nmax, const double *D, const double *M, double *phi, double g[3]) {
  const int ntM = nterms(nmax);
  for (int a = 0; a < ntM; ++a) {
    const int *ea = mi->e[a];
    double w = ((mi->deg[a] & 1) ? -1.0 : 1.0) / mi->fact[a] * M[a];
    *phi += w * D[a];
    g[0] -= w * D[mi->idx[ea[0] + 1][ea[1]][ea[2]]];
    g[1] -= w * D[mi->idx[ea[0]][ea[1] + 1][ea[2]]];
    g[2] -= w * D[mi->idx[ea[0]][ea[1]][ea[2] + 1]];
  }
}

/* eq. (direct): softened Green's function on the grid */
static double green_soft(const double r[3], double dx) {
  double d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  return d > dx ? -1.0 / d : -1.0 / dx;
}

/* ------------------------------------------------------------------ */
/* the solver state                                                     */
/* ------------------------------------------------------------------ */
typedef struct {
  int n, L, F, dl, p, nmax, ntM, ntL;
  double dx;
  mindex mi;       /* orders up to p + 1 */
  double *mass;    /* n^3 */
  double *M[32];   /* level k: 8^k x ntM, k = 2..F */
  double *Lc[32];  /* level k: 8^k x ntL, k = 3..F */
} ostate;

static int ilog2(int n) {
  int L = 0;
  while ((1 << L) < n) ++L;
  return (1 << L) == n ? L : -1;
}

static int st_init(ostate *s, int n, int p, int nmax, int dl) {
  memset(s, 0, sizeof(*s));
  int L = ilog2(n);
  if (dl < 1 || dl > 2 || L < 2 + dl || L > 10 || p < 1 || p > 8 || nmax < 0 || nmax > p) return -1;
  s->n = n; s->L = L; s->F = L - dl; s->dl = dl; s->p = p; s->nmax = nmax;
  s->ntM = nterms(nmax); s->ntL = nterms(p);
  s->dx = 1.0 / n;
  mi_init(&s->mi, p + 1);
  return 0;
}

static void st_free(ostate *s) {
  free(s->mass);
  for (int k = 0; k < 32; ++k) { free(s->M[k]); free(s->Lc[k]); }
}

/* upward pass: P2M on the finest FMM level, then M2M up to level 2 */
static void upward(ostate *s, const double *rho) {
  const int n = s->n, F = s->F, dl = s->dl, ntM = s->ntM;
  const double vol = s->dx * s->dx * s->dx;
  s->mass = (double *)malloc(sizeof(double) * (size_t)n * n * n);
#pragma omp parallel for schedule(static)
  for (i64 u = 0; u < (i64)n * n * n; ++u) s->mass[u] = rho[u] * vol;
  for (int k = 2; k <= F; ++k) {
    i64 nc = (i64)1 << (3 * k);
    s->M[k] = (double *)calloc((size_t)(nc * ntM), sizeof(double));
  }
  const int nF = 1 << F;
#pragma omp parallel for schedule(static)
  for (i64 T = 0; T < (i64)nF * nF * nF; ++T) {
    int t0 = (int)(T / ((i64)nF * nF)), t1 = (int)((T / nF) % nF), t2 = (int)(T % nF);
    double *M = s->M[F] + T * ntM;
    /* the 8^dl unigrid cells of T */
    const int m = (1 << dl) - 1;
    for (int q = 0; q < (1 << (3 * dl)); ++q) {
      int i = (t0 << dl) + ((q >> (2 * dl)) & m), j = (t1 << dl) + ((q >> dl) & m), l = (t2 << dl) + (q & m);
      double v[3] = {centre(i, s->L) - centre(t0, F), centre(j, s->L) - centre(t1, F),
                     centre(l, s->L) - centre(t2, F)};
      op_p2m(&s->mi, ntM, s->mass[lin(i, j, l, n)], v, M);
    }
  }
  for (int k = F; k >= 3; --k) {
    const int np = 1 << (k - 1), nk = 1 << k;
#pragma omp parallel for schedule(static)
    for (i64 P = 0; P < (i64)np * np * np; ++P) {
      int p0 = (int)(P / ((i64)np * np)), p1 = (int)((P / np) % np), p2 = (int)(P % np);
      double *Mp = s->M[k - 1] + P * ntM;
      for (int q = 0; q < 8; ++q) {
        int c0 = 2 * p0 + ((q >> 2) & 1), c1 = 2 * p1 + ((q >> 1) & 1), c2 = 2 * p2 + (q & 1);
        double d[3] = {centre(c0, k) - centre(p0, k - 1), centre(c1, k) - centre(p1, k - 1),
                       centre(c2, k) - centre(p2, k - 1)};
        op_m2m(&s->mi, ntM, d, s->M[k] + lin(c0, c1, c2, nk) * ntM, Mp);
      }
    }
  }
}

/* D tables for the fixed geometry (Sec. 2.2: displacements and Green's
   function derivatives are precomputed).  For a target at level k, descendant
   q of a cell P of level ks = k - sh, and source J = P - d at level ks,
   R = c_k(2^sh P + q) - c_ks(P - d); with P = 0 this is
   centre(q, k) - centre(-d, ks).  Layout [q (8^sh)][d+3 (343)][nterms(P)]. */
static double *geometry_table(const ostate *s, int k, int sh, int P) {
  const int nt = nterms(P), nq = 1 << (3 * sh), m = (1 << sh) - 1;
  (void)s;
  double *tab = (double *)malloc(sizeof(double) * (size_t)nq * 343 * nt);
#pragma omp parallel for schedule(static)
  for (int qd = 0; qd < nq * 343; ++qd) {
    int q = qd / 343, dd = qd % 343;
    int d0 = dd / 49 - 3, d1 = (dd / 7) % 7 - 3, d2 = dd % 7 - 3;
    int q0 = (q >> (2 * sh)) & m, q1 = (q >> sh) & m, q2 = q & m;
    double R[3] = {centre(q0, k) - centre(-d0, k - sh), centre(q1, k) - centre(-d1, k - sh),
                   centre(q2, k) - centre(-d2, k - sh)};
    if (abs(d0) <= 1 && abs(d1) <= 1 && abs(d2) <= 1) {
      for (int i = 0; i < nt; ++i) tab[(size_t)qd * nt + i] = 0.0; /* never used */
    } else {
      dtensor(R, &s->mi, P, tab + (size_t)qd * nt);
    }
  }
  return tab;
}

/* downward pass for the marked cells: M2L from the oct-shared list, then L2L */
static void downward(ostate *s, unsigned char **need) {
  const int F = s->F, p = s->p, ntL = s->ntL, ntM = s->ntM;
  for (int k = 3; k <= F; ++k) {
    const int nk = 1 << k, ns = 1 << (k - 1);
    i64 nc = (i64)1 << (3 * k);
    s->Lc[k] = (double *)calloc((size_t)(nc * ntL), sizeof(double));
    double *tab = geometry_table(s, k, 1, p);
#pragma omp parallel for schedule(dynamic, 64)
    for (i64 T = 0; T < nc; ++T) {
      if (need && !need[k][T]) continue;
      int t0 = (int)(T / ((i64)nk * nk)), t1 = (int)((T / nk) % nk), t2 = (int)(T % nk);
      int p0 = t0 >> 1, p1 = t1 >> 1, p2 = t2 >> 1;
      int q = ((t0 & 1) << 2) | ((t1 & 1) << 1) | (t2 & 1);
      double *L = s->Lc[k] + T * ntL;
      for (int j0 = p0 - 3; j0 <= p0 + 3; ++j0)
        for (int j1 = p1 - 3; j1 <= p1 + 3; ++j1)
          for (int j2 = p2 - 3; j2 <= p2 + 3; ++j2) {
            if (!inside(j0, j1, j2, ns) || !in_list(p0, p1, p2, j0, j1, j2)) continue;
            int dd = (p0 - j0 + 3) * 49 + (p1 - j1 + 3) * 7 + (p2 - j2 + 3);
            op_m2l(&s->mi, p, s->nmax, tab + ((size_t)q * 343 + dd) * nterms(p),
                   s->M[k - 1] + lin(j0, j1, j2, ns) * ntM, L);
          }
      if (k >= 4) {
        double a[3] = {centre(t0, k) - centre(p0, k - 1), centre(t1, k) - centre(p1, k - 1),
                       centre(t2, k) - centre(p2, k - 1)};
        op_l2l(&s->mi, p, a, s->Lc[k - 1] + lin(p0, p1, p2, ns) * ntL, L);
      }
    }
    free(tab);
  }
}

/* finest level: L2P + M2P + P2P at unigrid cell u; T = T_F(u) is the
   finest FMM cell holding u and q the position of u inside it */
static void bottom_cell(const ostate *s, const double *tab, int i, int j, int l, double *phi, double g[3]) {
  const int n = s->n, F = s->F, nF = 1 << F, dl = s->dl, m = (1 << dl) - 1;
  const int t0 = i >> dl, t1 = j >> dl, t2 = l >> dl;
  const int q = ((i & m) << (2 * dl)) | ((j & m) << dl) | (l & m);
  *phi = 0.0; g[0] = g[1] = g[2] = 0.0;
  if (F >= 3) {
    double v[3] = {centre(i, s->L) - centre(t0, F), centre(j, s->L) - centre(t1, F),
                   centre(l, s->L) - centre(t2, F)};
    op_l2p(&s->mi, s->p, v, s->Lc[F] + lin(t0, t1, t2, nF) * s->ntL, phi, g);
  }
  for (int j0 = t0 - 3; j0 <= t0 + 3; ++j0)
    for (int j1 = t1 - 3; j1 <= t1 + 3; ++j1)
      for (int j2 = t2 - 3; j2 <= t2 + 3; ++j2) {
        if (!inside(j0, j1, j2, nF) || !in_list(t0, t1, t2, j0, j1, j2)) continue;
        int dd = (t0 - j0 + 3) * 49 + (t1 - j1 + 3) * 7 + (t2 - j2 + 3);
        op_m2p(&s->mi, s->nmax, tab + ((size_t)q * 343 + dd) * nterms(s->nmax + 1),
               s->M[F] + lin(j0, j1, j2, nF) * s->ntM, phi, g);
      }
  /* near field: every unigrid cell of the finest FMM cells adjacent to T */
  const double xu[3] = {centre(i, s->L), centre(j, s->L), centre(l, s->L)};
  const int side = 1 << dl; /* unigrid cells per finest cell along an axis */
  for (int w0 = (t0 - 1) * side; w0 < (t0 + 2) * side; ++w0)
    for (int w1 = (t1 - 1) * side; w1 < (t1 + 2) * side; ++w1)
      for (int w2 = (t2 - 1) * side; w2 < (t2 + 2) * side; ++w2) {
        if (!inside(w0, w1, w2, n) || !adjacent(t0, t1, t2, w0 >> dl, w1 >> dl, w2 >> dl)) continue;
        double m = s->mass[lin(w0, w1, w2, n)];
        double r[3] = {xu[0] - centre(w0, s->L), xu[1] - centre(w1, s->L), xu[2] - centre(w2, s->L)};
        *phi += m * green_soft(r, s->dx);
        if (w0 == i && w1 == j && w2 == l) continue;
        double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        double inv3 = 1.0 / (d2 * sqrt(d2));
        g[0] -= m * r[0] * inv3; g[1] -= m * r[1] * inv3; g[2] -= m * r[2] * inv3;
      }
}

/* ------------------------------------------------------------------ */
/* exported entry points (called through ctypes by the tests)          */
/* ------------------------------------------------------------------ */
int or_nterms(int P) { return nterms(P); }

/* multi-index table of the oracle's order, [nterms(P)][3] */
int or_multi_index(int P, int *out) {
  if (P < 0 || P > OR_PMAX) return -1;
  mindex mi;
  mi_init(&mi, P);
  for (int t = 0; t < mi.nt; ++t)
    for (int d = 0; d < 3; ++d) out[3 * t + d] = mi.e[t][d];
  return mi.nt;
}

int or_dtensor(const double *R, int P, double *D) {
  if (P < 0 || P > OR_PMAX) return -1;
  mindex mi;
  mi_init(&mi, P);
  dtensor(R, &mi, P, D);
  return 0;
}

/* single-operator entry points (oracle order, physical units) */
int or_op_m2m(int nmax, const double *d, const double *Mc, double *Mp) {
  mindex mi; mi_init(&mi, nmax);
  op_m2m(&mi, nterms(nmax), d, Mc, Mp);
  return 0;
}
int or_op_p2m(int nmax, int npts, const double *m, const double *pos, const double *c, double *M) {
  mindex mi; mi_init(&mi, nmax);
  for (int i = 0; i < npts; ++i) {
    double v[3] = {pos[3 * i] - c[0], pos[3 * i + 1] - c[1], pos[3 * i + 2] - c[2]};
    op_p2m(&mi, nterms(nmax), m[i], v, M);
  }
  return 0;
}
int or_op_m2l(int p, int nmax, const double *R, const double *M, double *L) {
  mindex mi; mi_init(&mi, p + 1);
  double D[OR_NTMAX];
  dtensor(R, &mi, p, D);
  op_m2l(&mi, p, nmax, D, M, L);
  return 0;
}
int or_op_l2l(int p, const double *a, const double *Lp, double *Lc) {
  mindex mi; mi_init(&mi, p + 1);
  op_l2l(&mi, p, a, Lp, Lc);
  return 0;
}
int or_op_l2p(int p, const double *v, const double *L, double *out4) {
  mindex mi; mi_init(&mi, p + 1);
  double phi = 0.0, g[3] = {0, 0, 0};
  op_l2p(&mi, p, v, L, &phi, g);
  out4[0] = phi; out4[1] = g[0]; out4[2] = g[1]; out4[3] = g[2];
  return 0;
}
int or_op_m2p(int nmax, const double *R, const double *M, double *out4) {
  mindex mi; mi_init(&mi, nmax + 1);
  double D[OR_NTMAX];
  dtensor(R, &mi, nmax + 1, D);
  double phi = 0.0, g[3] = {0, 0, 0};
  op_m2p(&mi, nmax, D, M, &phi, g);
  out4[0] = phi; out4[1] = g[0]; out4[2] = g[1]; out4[3] = g[2];
  return 0;
}

/*
 * Full solve.  rho: n^3 density, C order, unit box, G = 1.
 * targets == NULL: phi[n^3], g[3][n^3] for every cell.
 * otherwise:       phi[ntarget], g[3][ntarget] for the listed flat indices;
 *                  only the ancestors of the targets get local expansions.
 * Returns 0, or -1 on invalid arguments.
 */
static int solve_impl(int n, int p, int nmax, int dl, const double *rho, i64 ntarget, const i64 *targets,
                      double *phi, double *g, double *times) {
  ostate s;
  if (st_init(&s, n, p, nmax, dl) != 0) return -1;
  const double t0 = wall_seconds();
  upward(&s, rho);
  const double t1 = wall_seconds();
  const int F = s.F, nF = 1 << F;
  unsigned char *need[32] = {0};
  if (targets) {
    for (int k = 3; k <= F; ++k) need[k] = (unsigned char *)calloc((size_t)1 << (3 * k), 1);
    for (i64 t = 0; t < ntarget; ++t) {
      i64 u = targets[t];
      int i = (int)(u / ((i64)n * n)), j = (int)((u / n) % n), l = (int)(u % n);
      for (int k = F; k >= 3; --k) {
        int sh = s.L - k;
        need[k][lin(i >> sh, j >> sh, l >> sh, 1 << k)] = 1;
      }
    }
  }
  downward(&s, targets ? need : NULL);
  double *tab = geometry_table(&s, s.L, dl, s.nmax + 1); /* targets at level L, sources at F */
  (void)nF;
  if (!targets) {
    const i64 N = (i64)n * n * n;
#pragma omp parallel for schedule(dynamic, 256)
    for (i64 u = 0; u < N; ++u) {
      int i = (int)(u / ((i64)n * n)), j = (int)((u / n) % n), l = (int)(u % n);
      double gg[3];
      bottom_cell(&s, tab, i, j, l, phi + u, gg);
      g[u] = gg[0]; g[N + u] = gg[1]; g[2 * N + u] = gg[2];
    }
  } else {
#pragma omp parallel for schedule(dynamic, 16)
    for (i64 t = 0; t < ntarget; ++t) {
      i64 u = targets[t];
      int i = (int)(u / ((i64)n * n)), j = (int)((u / n) % n), l = (int)(u % n);
      double gg[3];
      bottom_cell(&s, tab, i, j, l, phi + t, gg);
      g[t] = gg[0]; g[ntarget + t] = gg[1]; g[2 * ntarget + t] = gg[2];
    }
  }
  free(tab);
  for (int k = 0; k < 32; ++k) free(need[k]);
  st_free(&s);
  if (times) { times[0] = t1 - t0; times[1] = wall_seconds() - t1; }
  return 0;
}

int or_solve(int n, int p, int nmax, const double *rho, i64 ntarget, const i64 *targets,
             double *phi, double *g) {
  return solve_impl(n, p, nmax, 1, rho, ntarget, targets, phi, g, NULL);
}

/* or_solve with the finest FMM level dl levels above the unigrid (App. A):
   dl = 1 is FMM-1 (or_solve), dl = 2 FMM-2 (n >= 16). */
int or_solve_dl(int n, int p, int nmax, int dl, const double *rho, i64 ntarget, const i64 *targets,
                double *phi, double *g) {
  return solve_impl(n, p, nmax, dl, rho, ntarget, targets, phi, g, NULL);
}

/* or_solve that also reports wall seconds of the upward pass (times[0]) and
   of the downward pass for the requested targets (times[1]). */
int or_solve_timed(int n, int p, int nmax, const double *rho, i64 ntarget, const i64 *targets,
                   double *phi, double *g, double *times) {
  return solve_impl(n, p, nmax, 1, rho, ntarget, targets, phi, g, times);
}

/* or_solve_timed with the finest FMM level dl levels above the unigrid. */
int or_solve_timed_dl(int n, int p, int nmax, int dl, const double *rho, i64 ntarget, const i64 *targets,
                      double *phi, double *g, double *times) {
  return solve_impl(n, p, nmax, dl, rho, ntarget, targets, phi, g, times);
}

/* OpenMP threads the oracle runs with. */
int or_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the number of OpenMP threads of the following calls (n >= 1). */
int or_set_threads(int n) {
  if (n < 1) return -1;
#ifdef _OPENMP
  omp_set_num_threads(n);
#endif
  return 0;
}

/* Multipoles (level 2..F) or locals (level 3..F) of the full solve, in
   physical units and the oracle's multi-index order: out[8^level][nterms]. */
int or_expansions(int n, int p, int nmax, const double *rho, int which, int level, double *out) {
  ostate s;
  if (st_init(&s, n, p, nmax, 1) != 0) return -1;
  if (which == 0 && (level < 2 || level > s.F)) return -1;
  if (which == 1 && (level < 3 || level > s.F)) return -1;
  upward(&s, rho);
  if (which == 1) downward(&s, NULL);
  const i64 nc = (i64)1 << (3 * level);
  if (which == 0) memcpy(out, s.M[level], sizeof(double) * (size_t)(nc * s.ntM));
  else memcpy(out, s.Lc[level], sizeof(double) * (size_t)(nc * s.ntL));
  st_free(&s);
  return 0;
}

/*
 * Cloud-in-cell deposition (Sec. 3: the test particles are put on the grid
 * with CIC).  A particle of mass m at x spreads over the cells c whose centre
 * lies within one cell of it along every axis, with the tent weights
 *   W_c = prod_d max(0, 1 - |x_d - x_c,d| / dx),
 * and rho_c += m W_c / dx^3.  Cells outside the box do not exist (isolated
 * box): their share is dropped.  pos: [count][3] in the unit box.
 */
int or_deposit_cic(int n, i64 count, const double *pos, const double *mass, double *rho) {
  if (ilog2(n) < 0 || count < 0) return -1;
  const double dx = 1.0 / n, inv_vol = (double)n * n * n;
  for (i64 t = 0; t < count; ++t) {
    const double *x = pos + 3 * t;
    int lo[3];
    for (int d = 0; d < 3; ++d) lo[d] = (int)floor(x[d] / dx - 0.5);
    for (int a = lo[0]; a <= lo[0] + 1; ++a)
      for (int b = lo[1]; b <= lo[1] + 1; ++b)
        for (int c = lo[2]; c <= lo[2] + 1; ++c) {
          if (!inside(a, b, c, n)) continue;
          const int cell[3] = {a, b, c};
          double w = 1.0;
          for (int d = 0; d < 3; ++d) {
            const double u = 1.0 - fabs(x[d] - ((double)cell[d] + 0.5) * dx) / dx;
            w *= u > 0.0 ? u : 0.0;
          }
          rho[lin(a, b, c, n)] += mass[t] * w * inv_vol;
        }
  }
  return 0;
}

/*
 * Force from the potential by finite differences, as the host code does
 * after the solve (App. C: a 5-point stencil).  Along each axis, at cell i of
 * n, f = -dphi/dx with the fourth-order differences over 5 cells:
 *   central  (i = 2 .. n-3):  (phi[i-2] - 8 phi[i-1] + 8 phi[i+1] - phi[i+2]) / (12 dx)
 *   i = 1:                    (-3 phi[0] - 10 phi[1] + 18 phi[2] - 6 phi[3] + phi[4]) / (12 dx)
 *   i = 0:                    (-25 phi[0] + 48 phi[1] - 36 phi[2] + 16 phi[3] - 3 phi[4]) / (12 dx)
 * and the mirror images at i = n-2, n-1 (the box has no cells beyond its
 * walls, so the last two layers take one-sided stencils of the same order).
 * Each is exact for polynomials of degree <= 4.  f: [3][n^3].
 */
static double fd_deriv(const double *v, int i, int n, double dx) {
  /* v(k) = phi at position k along the axis */
  if (i >= 2 && i <= n - 3) return (v[i - 2] - 8.0 * v[i - 1] + 8.0 * v[i + 1] - v[i + 2]) / (12.0 * dx);
  if (i == 1) return (-3.0 * v[0] - 10.0 * v[1] + 18.0 * v[2] - 6.0 * v[3] + v[4]) / (12.0 * dx);
  if (i == 0) return (-25.0 * v[0] + 48.0 * v[1] - 36.0 * v[2] + 16.0 * v[3] - 3.0 * v[4]) / (12.0 * dx);
  if (i == n - 2)
    return -(-3.0 * v[n - 1] - 10.0 * v[n - 2] + 18.0 * v[n - 3] - 6.0 * v[n - 4] + v[n - 5]) / (12.0 * dx);
  return -(-25.0 * v[n - 1] + 48.0 * v[n - 2] - 36.0 * v[n - 3] + 16.0 * v[n - 4] - 3.0 * v[n - 5]) / (12.0 * dx);
}

int or_fd_force(int n, const double *phi, double *f) {
  if (ilog2(n) < 0 || n < 8) return -1;
  const double dx = 1.0 / n;
  const i64 N = (i64)n * n * n;
#pragma omp parallel for schedule(static)
  for (i64 u = 0; u < N; ++u) {
    int c[3] = {(int)(u / ((i64)n * n)), (int)((u / n) % n), (int)(u % n)};
    double line[1024];
    for (int d = 0; d < 3; ++d) {
      for (int k = 0; k < n; ++k) {
        int w[3] = {c[0], c[1], c[2]};
        w[d] = k;
        line[k] = phi[lin(w[0], w[1], w[2], n)];
      }
      f[(i64)d * N + u] = -fd_deriv(line, c[d], n, dx);
    }
  }
  return 0;
}

/* O(N^2) direct sum with the same softened Green's function (eq. direct):
   phi_u = sum_w m_w g(x_u - x_w), g_u = -sum_{w != u} m_w (x_u-x_w)/|x_u-x_w|^3.
   targets as in or_solve. */
int or_direct(int n, const double *rho, i64 ntarget, const i64 *targets, double *phi, double *g) {
  int L = ilog2(n);
  if (L < 0) return -1;
  const i64 N = (i64)n * n * n;
  const double dx = 1.0 / n, vol = dx * dx * dx;
  const i64 nt = targets ? ntarget : N;
#pragma omp parallel for schedule(dynamic, 16)
  for (i64 t = 0; t < nt; ++t) {
    i64 u = targets ? targets[t] : t;
    int i = (int)(u / ((i64)n * n)), j = (int)((u / n) % n), l = (int)(u % n);
    double xu[3] = {centre(i, L), centre(j, L), centre(l, L)};
    double ph = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (i64 w = 0; w < N; ++w) {
      int a = (int)(w / ((i64)n * n)), b = (int)((w / n) % n), c = (int)(w % n);
      double m = rho[w] * vol;
      double r[3] = {xu[0] - centre(a, L), xu[1] - centre(b, L), xu[2] - centre(c, L)};
      ph += m * green_soft(r, dx);
      if (w == u) continue;
      double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      double inv3 = 1.0 / (d2 * sqrt(d2));
      g0 -= m * r[0] * inv3; g1 -= m * r[1] * inv3; g2 -= m * r[2] * inv3;
    }
    phi[t] = ph; g[t] = g0; g[nt + t] = g1; g[2 * nt + t] = g2;
  }
  return 0;
}

/*
 * Adjoint (vector-Jacobian product) of or_solve_dl over the full grid:
 * drho = d(<phi, dphi> + <g, dg>)/drho, with the finest FMM level dl levels
 * above the unigrid (dl = 1 FMM-1, dl = 2 FMM-2 of App. A).  The solve is
 * linear in the cell masses m = rho dx^3; each forward operator is transposed
 * and the passes run in reverse: P2P^T, L2P^T and M2P^T at the finest level
 * (each finest FMM cell holds 8^dl unigrid cells, the near field of a
 * unigrid cell is every unigrid cell of the finest FMM cells adjacent to its
 * own), then for k = F..3 L2L^T and M2L^T, then M2M^T for k = 3..F, then
 * P2M^T.  dg may be NULL (treated as zero).
 */
int or_adjoint_dl(int n, int p, int nmax, int dl, const double *dphi, const double *dg, double *drho) {
  ostate s;
  if (st_init(&s, n, p, nmax, dl) != 0) return -1;
  const int F = s.F, Lv = s.L, ntM = s.ntM, ntL = s.ntL;
  const int msk = (1 << dl) - 1, nq = 1 << (3 * dl), reach = (2 << dl) - 1;
  const i64 N = (i64)n * n * n;
  const int nF = 1 << F;
  const double dx = s.dx;
  const mindex *mi = &s.mi;
  double *Mb[32] = {0}, *Lb[32] = {0};
  for (int k = 2; k <= F; ++k) Mb[k] = (double *)calloc((size_t)(((i64)1 << (3 * k)) * ntM), sizeof(double));
  for (int k = 3; k <= F; ++k) Lb[k] = (double *)calloc((size_t)(((i64)1 << (3 * k)) * ntL), sizeof(double));
  double *mb = (double *)calloc((size_t)N, sizeof(double));
#define DGV(d, u) (dg ? dg[(i64)(d) * N + (u)] : 0.0)

  /* P2P^T (gather over the targets u that see w) */
#pragma omp parallel for schedule(dynamic, 256)
  for (i64 w = 0; w < N; ++w) {
    int a = (int)(w / ((i64)n * n)), b = (int)((w / n) % n), c = (int)(w % n);
    double acc = 0.0;
    for (int i = a - reach; i <= a + reach; ++i)
      for (int j = b - reach; j <= b + reach; ++j)
        for (int l = c - reach; l <= c + reach; ++l) {
          if (!inside(i, j, l, n) || !adjacent(i >> dl, j >> dl, l >> dl, a >> dl, b >> dl, c >> dl)) continue;
          i64 u = lin(i, j, l, n);
          double r[3] = {centre(i, Lv) - centre(a, Lv), centre(j, Lv) - centre(b, Lv), centre(l, Lv) - centre(c, Lv)};
          acc += dphi[u] * green_soft(r, dx);
          if (u == w) continue;
          double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
          double inv3 = 1.0 / (d2 * sqrt(d2));
          acc -= (DGV(0, u) * r[0] + DGV(1, u) * r[1] + DGV(2, u) * r[2]) * inv3;
        }
    mb[w] = acc;
  }
  /* L2P^T */
  if (F >= 3) {
#pragma omp parallel for schedule(static)
    for (i64 T = 0; T < (i64)nF * nF * nF; ++T) {
      int t0 = (int)(T / ((i64)nF * nF)), t1 = (int)((T / nF) % nF), t2 = (int)(T % nF);
      for (int q = 0; q < nq; ++q) {
        int i = (t0 << dl) + ((q >> (2 * dl)) & msk), j = (t1 << dl) + ((q >> dl) & msk), l = (t2 << dl) + (q & msk);
        i64 u = lin(i, j, l, n);
        double v[3] = {centre(i, Lv) - centre(t0, F), centre(j, Lv) - centre(t1, F), centre(l, Lv) - centre(t2, F)};
        for (int bb = 0; bb < ntL; ++bb) {
          const int *eb = mi->e[bb];
          double val = dphi[u] * mono(v, eb) / mi->fact[bb];
          for (int d = 0; d < 3; ++d) {
            if (eb[d] == 0) continue;
            int e[3] = {eb[0], eb[1], eb[2]};
            e[d] -= 1;
            val -= DGV(d, u) * mono(v, e) / (factorial(e[0]) * factorial(e[1]) * factorial(e[2]));
          }
          Lb[F][T * ntL + bb] += val;
        }
      }
    }
  }
  /* M2P^T (gather over targets T whose list holds J) */
  {
    double *tab = geometry_table(&s, F + dl, dl, nmax + 1);
    const int ntD = nterms(nmax + 1);
#pragma omp parallel for schedule(dynamic, 64)
    for (i64 J = 0; J < (i64)nF * nF * nF; ++J) {
      int j0 = (int)(J / ((i64)nF * nF)), j1 = (int)((J / nF) % nF), j2 = (int)(J % nF);
      double *Mj = Mb[F] + J * ntM;
      for (int t0 = j0 - 3; t0 <= j0 + 3; ++t0)
        for (int t1 = j1 - 3; t1 <= j1 + 3; ++t1)
          for (int t2 = j2 - 3; t2 <= j2 + 3; ++t2) {
            if (!inside(t0, t1, t2, nF) || !in_list(t0, t1, t2, j0, j1, j2)) continue;
            int dd = (t0 - j0 + 3) * 49 + (t1 - j1 + 3) * 7 + (t2 - j2 + 3);
            for (int q = 0; q < nq; ++q) {
              int i = (t0 << dl) + ((q >> (2 * dl)) & msk), j = (t1 << dl) + ((q >> dl) & msk),
                  l = (t2 << dl) + (q & msk);
              i64 u = lin(i, j, l, n);
              const double *D = tab + ((size_t)q * 343 + dd) * ntD;
              for (int a = 0; a < ntM; ++a) {
                const int *ea = mi->e[a];
                double w = ((mi->deg[a] & 1) ? -1.0 : 1.0) / mi->fact[a];
                double v = dphi[u] * D[a] - DGV(0, u) * D[mi->idx[ea[0] + 1][ea[1]][ea[2]]] -
                           DGV(1, u) * D[mi->idx[ea[0]][ea[1] + 1][ea[2]]] -
                           DGV(2, u) * D[mi->idx[ea[0]][ea[1]][ea[2] + 1]];
                Mj[a] += w * v;
              }
            }
          }
    }
    free(tab);
  }
  /* L2L^T and M2L^T, k = F..3 */
  for (int k = F; k >= 3; --k) {
    const int nk = 1 << k, ns = 1 << (k - 1);
    if (k >= 4) {
#pragma omp parallel for schedule(static)
      for (i64 P = 0; P < (i64)ns * ns * ns; ++P) {
        int p0 = (int)(P / ((i64)ns * ns)), p1 = (int)((P / ns) % ns), p2 = (int)(P % ns);
        double *Lp = Lb[k - 1] + P * ntL;
        for (int q = 0; q < 8; ++q) {
          int c0 = 2 * p0 + ((q >> 2) & 1), c1 = 2 * p1 + ((q >> 1) & 1), c2 = 2 * p2 + (q & 1);
          const double *Lc = Lb[k] + lin(c0, c1, c2, nk) * ntL;
          double a[3] = {centre(c0, k) - centre(p0, k - 1), centre(c1, k) - centre(p1, k - 1),
                         centre(c2, k) - centre(p2, k - 1)};
          /* forward: Lc[b] += Lp[b+g] a^g/g!  =>  Lp[b+g] += Lc[b] a^g/g! */
          for (int bb = 0; bb < ntL; ++bb) {
            const int *eb = mi->e[bb];
            for (int gg = 0; gg < ntL; ++gg) {
              if (mi->deg[bb] + mi->deg[gg] > p) continue;
              const int *eg = mi->e[gg];
              int bg = mi->idx[eb[0] + eg[0]][eb[1] + eg[1]][eb[2] + eg[2]];
              Lp[bg] += Lc[bb] * mono(a, eg) / mi->fact[gg];
            }
          }
        }
      }
    }
    double *tab = geometry_table(&s, k, 1, p);
    const int ntD = nterms(p);
#pragma omp parallel for schedule(dynamic, 64)
    for (i64 J = 0; J < (i64)ns * ns * ns; ++J) {
      int j0 = (int)(J / ((i64)ns * ns)), j1 = (int)((J / ns) % ns), j2 = (int)(J % ns);
      double *Mj = Mb[k - 1] + J * ntM;
      for (int p0 = j0 - 3; p0 <= j0 + 3; ++p0)
        for (int p1 = j1 - 3; p1 <= j1 + 3; ++p1)
          for (int p2 = j2 - 3; p2 <= j2 + 3; ++p2) {
            if (!inside(p0, p1, p2, ns) || !in_list(p0, p1, p2, j0, j1, j2)) continue;
            int dd = (p0 - j0 + 3) * 49 + (p1 - j1 + 3) * 7 + (p2 - j2 + 3);
            for (int q = 0; q < 8; ++q) {
              int c0 = 2 * p0 + ((q >> 2) & 1), c1 = 2 * p1 + ((q >> 1) & 1), c2 = 2 * p2 + (q & 1);
              const double *Lt = Lb[k] + lin(c0, c1, c2, nk) * ntL;
              const double *D = tab + ((size_t)q * 343 + dd) * ntD;
              /* forward: L[b] += (-1)^|a|/a! D[a+b] M[a]  =>  M[a] += (-1)^|a|/a! D[a+b] L[b] */
              for (int a = 0; a < ntM; ++a) {
                const int *ea = mi->e[a];
                double acc = 0.0;
                for (int bb = 0; bb < ntL; ++bb) {
                  if (mi->deg[a] + mi->deg[bb] > p) continue;
                  const int *eb = mi->e[bb];
                  acc += D[mi->idx[ea[0] + eb[0]][ea[1] + eb[1]][ea[2] + eb[2]]] * Lt[bb];
                }
                Mj[a] += ((mi->deg[a] & 1) ? -1.0 : 1.0) / mi->fact[a] * acc;
              }
            }
          }
    }
    free(tab);
  }
  /* M2M^T, k = 3..F: forward Mp[a] += C(a,b) d^(a-b) Mc[b] => Mc[b] += C(a,b) d^(a-b) Mp[a] */
  for (int k = 3; k <= F; ++k) {
    const int nk = 1 << k, np = 1 << (k - 1);
#pragma omp parallel for schedule(static)
    for (i64 C = 0; C < (i64)nk * nk * nk; ++C) {
      int c0 = (int)(C / ((i64)nk * nk)), c1 = (int)((C / nk) % nk), c2 = (int)(C % nk);
      int p0 = c0 >> 1, p1 = c1 >> 1, p2 = c2 >> 1;
      const double *Mp = Mb[k - 1] + lin(p0, p1, p2, np) * ntM;
      double *Mc = Mb[k] + C * ntM;
      double d[3] = {centre(c0, k) - centre(p0, k - 1), centre(c1, k) - centre(p1, k - 1),
                     centre(c2, k) - centre(p2, k - 1)};
      for (int bb = 0; bb < ntM; ++bb) {
        const int *eb = mi->e[bb];
        double acc = 0.0;
        for (int a = 0; a < ntM; ++a) {
          const int *ea = mi->e[a];
          if (eb[0] > ea[0] || eb[1] > ea[1] || eb[2] > ea[2]) continue;
          int gg[3] = {ea[0] - eb[0], ea[1] - eb[1], ea[2] - eb[2]};
          acc += binom(ea[0], eb[0]) * binom(ea[1], eb[1]) * binom(ea[2], eb[2]) * mono(d, gg) * Mp[a];
        }
        Mc[bb] += acc;
      }
    }
  }
  /* P2M^T and the mass-to-density factor */
  const double vol = dx * dx * dx;
#pragma omp parallel for schedule(static)
  for (i64 u = 0; u < N; ++u) {
    int i = (int)(u / ((i64)n * n)), j = (int)((u / n) % n), l = (int)(u % n);
    int t0 = i >> dl, t1 = j >> dl, t2 = l >> dl;
    const double *M = Mb[F] + lin(t0, t1, t2, nF) * ntM;
    double v[3] = {centre(i, Lv) - centre(t0, F), centre(j, Lv) - centre(t1, F), centre(l, Lv) - centre(t2, F)};
    double acc = mb[u];
    for (int a = 0; a < ntM; ++a) acc += mono(v, mi->e[a]) * M[a];
    drho[u] = acc * vol;
  }
#undef DGV
  free(mb);
  for (int k = 0; k < 32; ++k) { free(Mb[k]); free(Lb[k]); }
  st_free(&s);
  return 0;
}

/* or_adjoint_dl for FMM-1 (dl = 1). */
int or_adjoint(int n, int p, int nmax, const double *dphi, const double *dg, double *drho) {
  return or_adjoint_dl(n, p, nmax, 1, dphi, dg, drho);
}

/*
 * Which pass of or_solve accounts for source cell w at target cell u (flat
 * unigrid indices): -1 near field (P2P), F = M2P from the finest FMM level,
 * s in [2, F-1] = M2L from source level s (targets at s + 1).  Returns -2 if
 * no pass counts the pair and -3 if several do.  Used to check that the
 * fields of Sec. 2.2 partition the domain.
 */
static int pair_pass(int n, int dl, i64 u, i64 w) {
  int L = ilog2(n);
  if (L < 2 + dl || dl < 1 || dl > 2) return -4;
  const int F = L - dl;
  int ui[3] = {(int)(u / ((i64)n * n)), (int)((u / n) % n), (int)(u % n)};
  int wi[3] = {(int)(w / ((i64)n * n)), (int)((w / n) % n), (int)(w % n)};
  int count = 0, res = -2;
  if (adjacent(ui[0] >> dl, ui[1] >> dl, ui[2] >> dl, wi[0] >> dl, wi[1] >> dl, wi[2] >> dl)) { ++count; res = -1; }
  if (in_list(ui[0] >> dl, ui[1] >> dl, ui[2] >> dl, wi[0] >> dl, wi[1] >> dl, wi[2] >> dl)) { ++count; res = F; }
  for (int k = 3; k <= F; ++k) {
    int sh = L - (k - 1);
    if (in_list(ui[0] >> sh, ui[1] >> sh, ui[2] >> sh, wi[0] >> sh, wi[1] >> sh, wi[2] >> sh)) { ++count; res = k - 1; }
  }
  return count > 1 ? -3 : res;
}
int or_pair_pass(int n, i64 u, i64 w) { return pair_pass(n, 1, u, w); }

/* Size of the (clipped) interaction list of cell (i,j,l) at level k. */
int or_list_size(int k, int i, int j, int l) {
  const int nk = 1 << k;
  int c = 0;
  for (int a = i - 3; a <= i + 3; ++a)
    for (int b = j - 3; b <= j + 3; ++b)
      for (int d = l - 3; d <= l + 3; ++d)
        if (inside(a, b, d, nk) && in_list(i, j, l, a, b, d)) ++c;
  return c;
}

/* or_pair_pass for one target u against every source w: out[n^3]. */
int or_pair_pass_row(int n, i64 u, int *out) {
  const i64 N = (i64)n * n * n;
#pragma omp parallel for schedule(static)
  for (i64 w = 0; w < N; ++w) out[w] = pair_pass(n, 1, u, w);
  return 0;
}

/* or_pair_pass_row with the finest FMM level dl levels above the unigrid. */
int or_pair_pass_row_dl(int n, int dl, i64 u, int *out) {
  const i64 N = (i64)n * n * n;
#pragma omp parallel for schedule(static)
  for (i64 w = 0; w < N; ++w) out[w] = pair_pass(n, dl, u, w);
  return 0;
}
