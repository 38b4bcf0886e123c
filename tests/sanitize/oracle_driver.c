/*
 * Drives every entry point of the CPU oracle on small seeded inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (the CPU test
 * suite compiles and runs it).  It checks nothing numerical itself (the
 * oracle's pins do that); it only has to run every code path, including the
 * clipped lists at the box walls, targets, FMM-2 and the adjoints, so that
 * the sanitizers see every access.  Exit status 0 on success.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef long long i64;
int or_nterms(int P);
int or_multi_index(int P, int *out);
int or_dtensor(const double *R, int P, double *D);
int or_op_m2m(int nmax, const double *d, const double *Mc, double *Mp);
int or_op_p2m(int nmax, int npts, const double *m, const double *pos, const double *c, double *M);
int or_op_m2l(int p, int nmax, const double *R, const double *M, double *L);
int or_op_l2l(int p, const double *a, const double *Lp, double *Lc);
int or_op_l2p(int p, const double *v, const double *L, double *out4);
int or_op_m2p(int nmax, const double *R, const double *M, double *out4);
int or_solve_dl(int n, int p, int nmax, int dl, const double *rho, i64 ntarget, const i64 *targets, double *phi,
                double *g);
int or_expansions(int n, int p, int nmax, const double *rho, int which, int level, double *out);
int or_direct(int n, const double *rho, i64 ntarget, const i64 *targets, double *phi, double *g);
int or_adjoint_dl(int n, int p, int nmax, int dl, const double *dphi, const double *dg, double *drho);
int or_pair_pass_row_dl(int n, int dl, i64 u, int *out);
int or_list_size(int k, int i, int j, int l);
int or_deposit_cic(int n, i64 count, const double *pos, const double *mass, double *rho);
int or_fd_force(int n, const double *phi, double *f);

static unsigned long long st = 88172645463325252ULL;
static double urand(void) {  /* xorshift64, uniform in [0, 1) */
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return (double)(st >> 11) / 9007199254740992.0;
}

static int check(int rc, const char *what) {
  if (rc != 0) fprintf(stderr, "%s returned %d\n", what, rc);
  return rc != 0;
}

int main(void) {
  int bad = 0;
  const int P = 8, nt = or_nterms(P + 1);
  int *mi = malloc(sizeof(int) * 3 * nt);
  bad |= or_multi_index(P + 1, mi) != nt;
  double R[3] = {2.25, -1.75, 3.25}, D[220], M[220], L[220], out4[4], a3[3] = {0.1, -0.2, 0.3};
  bad |= check(or_dtensor(R, P + 1, D), "dtensor");
  double m[5], pos[15], c[3] = {0.5, 0.5, 0.5};
  for (int i = 0; i < 5; ++i) {
    m[i] = urand();
    for (int d = 0; d < 3; ++d) pos[3 * i + d] = urand();
  }
  bad |= check(or_op_p2m(P, 5, m, pos, c, M), "p2m");
  double Mp[220];
  bad |= check(or_op_m2m(P, a3, M, Mp), "m2m");
  bad |= check(or_op_m2l(P, P, R, M, L), "m2l");
  double Lc[220];
  bad |= check(or_op_l2l(P, a3, L, Lc), "l2l");
  bad |= check(or_op_l2p(P, a3, L, out4), "l2p");
  bad |= check(or_op_m2p(P, R, M, out4), "m2p");
  for (int dl = 1; dl <= 2; ++dl) {
    const int n = 16, N = n * n * n;
    double *rho = malloc(sizeof(double) * N), *phi = malloc(sizeof(double) * N), *g = malloc(sizeof(double) * 3 * N);
    double *dphi = malloc(sizeof(double) * N), *dg = malloc(sizeof(double) * 3 * N), *drho = malloc(sizeof(double) * N);
    for (int u = 0; u < N; ++u) {
      rho[u] = urand();
      dphi[u] = urand() - 0.5;
    }
    for (int u = 0; u < 3 * N; ++u) dg[u] = urand() - 0.5;
    const int p = dl == 1 ? 6 : 4;
    bad |= check(or_solve_dl(n, p, p, dl, rho, 0, NULL, phi, g), "solve");
    bad |= check(or_solve_dl(n, 3, 2, dl, rho, 0, NULL, phi, g), "solve nmax");
    i64 tg[4] = {0, N - 1, 17, (i64)N / 2 + 5};
    bad |= check(or_solve_dl(n, p, p, dl, rho, 4, tg, phi, g), "solve targets");
    bad |= check(or_adjoint_dl(n, p, p, dl, dphi, dg, drho), "adjoint");
    bad |= check(or_adjoint_dl(n, p, p, dl, dphi, NULL, drho), "adjoint phi only");
    int *row = malloc(sizeof(int) * N);
    bad |= check(or_pair_pass_row_dl(n, dl, 1234, row), "pair pass");
    free(row);
    if (dl == 1) {
      double *ex = malloc(sizeof(double) * 512 * nt);
      bad |= check(or_expansions(n, p, p, rho, 0, 3, ex), "expansions M");
      bad |= check(or_expansions(n, p, p, rho, 1, 3, ex), "expansions L");
      free(ex);
      bad |= check(or_direct(n, rho, 4, tg, phi, g), "direct");
      bad |= check(or_fd_force(n, phi, g), "fd force");
      double ppos[3 * 64], pm[64];
      for (int i = 0; i < 64; ++i) {
        pm[i] = urand();
        for (int d = 0; d < 3; ++d) ppos[3 * i + d] = 1.1 * urand() - 0.05; /* some outside the box */
      }
      memset(rho, 0, sizeof(double) * N);
      bad |= check(or_deposit_cic(n, 64, ppos, pm, rho), "cic");
      bad |= or_list_size(3, 0, 0, 0) <= 0;
    }
    free(rho); free(phi); free(g); free(dphi); free(dg); free(drho);
  }
  free(mi);
  if (bad) return 1;
  printf("oracle driver: every entry point ran\n");
  return 0;
}
