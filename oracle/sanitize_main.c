/*
 * Driver for the sanitizer builds of the CPU oracle (test infrastructure).
 *
 * Built together with shasta_oracle.c by the test suite, once with
 * AddressSanitizer and UndefinedBehaviorSanitizer and once with
 * ThreadSanitizer (the OpenMP split over pencils), and run: every call path
 * of the oracle on small grids, every EOS, states the recovery's guard acts
 * on (E <= 0, |M| >= E), thread counts 1 and 4.  A sanitizer report aborts
 * the run; the driver itself checks the conservation ledger of each run
 * (sum U(t) + outflow = sum U(0), the flux form of eq. shasta-geo) and that
 * the thread count does not change a result, and exits non-zero otherwise.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int kind;
  double B;
  double e_H;
  int n;
  const double* te;
  const double* tp;
  double cs2;
  double mass;
} orc_eos;

double orc_pressure(const orc_eos* eos, double e, double nb);
int orc_recover(const orc_eos* eos, double E, double Mx, double My, double Mz, double R,
                double* e_out, double* p_out, double* v_out, double* vx, double* vy,
                double* vz, int* iters_out, int* clamped, int* floored);
void orc_prim_to_cons(const orc_eos* eos, int64_t ncell, const double* e, const double* vx,
                      const double* vy, const double* vz, const double* n, double* E,
                      double* Mx, double* My, double* Mz, double* R);
void orc_cons_to_prim(const orc_eos* eos, int64_t ncell, const double* E, const double* Mx,
                      const double* My, const double* Mz, const double* R, double* e,
                      double* p, double* vx, double* vy, double* vz, double* n);
void orc_fct_1d(int N, const double* U, const double* eps, const double* f, int has_source,
                double lam, double diff, double* unew, double* flux);
void orc_run(const orc_eos* eos, int nx, int ny, int nz, double lam, double diff, int64_t k0,
             int nsteps, double** U, double* ledger, double* maxeps, int64_t* counters,
             int nthreads);
double orc_sum(int64_t n, const double* a);

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double uniform(void) {   /* splitmix64, [0, 1) */
  uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int failures = 0;
static void check(int ok, const char* what) {
  if (!ok) {
    fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

/* one run of nsteps on a random state, with a few guarded cells; returns
 * the fields in U (5 arrays of n cells) */
static void one_run(const orc_eos* eos, int nx, int ny, int nz, int nsteps, int nthreads,
                    double** U, double* ledger) {
  const int64_t n = (int64_t)nx * ny * nz;
  double* prim[5];
  for (int q = 0; q < 5; ++q) prim[q] = (double*)malloc(sizeof(double) * n);
  rng_state = 12345;
  for (int64_t i = 0; i < n; ++i) {
    prim[0][i] = 0.05 + 5.0 * uniform();
    for (int a = 1; a < 4; ++a) prim[a][i] = 0.5 * (uniform() - 0.5);
    prim[4][i] = 0.15 * prim[0][i];
  }
  orc_prim_to_cons(eos, n, prim[0], prim[1], prim[2], prim[3], prim[4], U[0], U[1], U[2],
                   U[3], U[4]);
  U[0][0] = -0.2;                       /* floored */
  U[1][n / 2] = 1.5 * U[0][n / 2];      /* clamped */
  U[0][n - 1] = 0.0;
  double maxeps = 0.0;
  int64_t cnt[4] = {0, 0, 0, 0};
  double s0[5];
  for (int q = 0; q < 5; ++q) s0[q] = orc_sum(n, U[q]);
  for (int q = 0; q < 5; ++q) ledger[q] = 0.0;
  orc_run(eos, nx, ny, nz, 0.4, 1.0, 1, nsteps, U, ledger, &maxeps, cnt, nthreads);
  for (int q = 0; q < 5; ++q) {
    double scale = 0.0;
    for (int64_t i = 0; i < n; ++i) scale += fabs(U[q][i]);
    const double resid = orc_sum(n, U[q]) + ledger[q] - s0[q];
    check(fabs(resid) <= 1e-12 * (scale + fabs(s0[q])) + 1e-300, "conservation ledger");
  }
  check(cnt[0] > 0 && cnt[1] > 0, "guard counted");
  check(maxeps > 0.0 && maxeps < 0.5, "largest Courant number in (0, 1/2)");
  for (int q = 0; q < 5; ++q) free(prim[q]);
}

int main(void) {
  const double te[4] = {0.0, 0.1, 1.7, 1000.0};
  const double tp[4] = {0.0, 0.1 / 3.0, 0.1 / 3.0, (1000.0 - 1.6) / 3.0};
  orc_eos eos[4] = {{0, 0, 0, 0, NULL, NULL, 0, 0},
                    {1, 0.396928, 0.105069, 0, NULL, NULL, 0, 0},
                    {2, 0, 0, 4, te, tp, 0, 0},
                    {3, 0, 0, 0, NULL, NULL, 1.0 / 3.0, 0.938}};
  /* recovery on ordinary and guarded states */
  const double Es[6] = {-1.0, 0.0, 4e-310, 1e-300, 0.7, 9.0};
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 6; ++i)
      for (int m = 0; m < 4; ++m) {
        const double M = (m == 0) ? 0.0 : (m == 1 ? 0.5 : (m == 2 ? 1.0 : 2.0)) * fabs(Es[i]) +
                                              (Es[i] <= 0.0 ? 0.1 : 0.0);
        double e, p, v, vx, vy, vz;
        int it, cl, fl;
        orc_recover(&eos[k], Es[i], 0.6 * M, 0.8 * M, 0.0, 0.1, &e, &p, &v, &vx, &vy, &vz, &it,
                    &cl, &fl);
        check(v >= 0.0 && v < 1.0, "recovered speed in [0, 1)");
      }
  /* the one-dimensional operator with and without source */
  {
    enum { N = 9 };
    double U[N + 6], eps[N + 6], f[N + 6], out[N], flux[2];
    for (int j = 0; j < N + 6; ++j) {
      U[j] = 1.0 + uniform();
      eps[j] = 0.2 * (uniform() - 0.5);
      f[j] = uniform();
    }
    orc_fct_1d(N, U, eps, f, 1, 0.4, 1.0, out, flux);
    orc_fct_1d(N, U, eps, f, 0, 0.2, 0.5, out, NULL);
  }
  /* whole runs: every EOS, a ragged grid, 1 and 4 threads give the same */
  for (int k = 0; k < 4; ++k) {
    const int nx = 11, ny = 7, nz = 5;
    const int64_t n = (int64_t)nx * ny * nz;
    double *U1[5], *U4[5], l1[5], l4[5];
    for (int q = 0; q < 5; ++q) {
      U1[q] = (double*)malloc(sizeof(double) * n);
      U4[q] = (double*)malloc(sizeof(double) * n);
    }
    one_run(&eos[k], nx, ny, nz, 3, 1, U1, l1);
    one_run(&eos[k], nx, ny, nz, 3, 4, U4, l4);
    for (int q = 0; q < 5; ++q) {
      check(memcmp(U1[q], U4[q], sizeof(double) * n) == 0, "thread count independence");
      check(l1[q] == l4[q], "ledger thread count independence");
    }
    double* P[6];
    for (int j = 0; j < 6; ++j) P[j] = (double*)malloc(sizeof(double) * n);
    orc_cons_to_prim(&eos[k], n, U1[0], U1[1], U1[2], U1[3], U1[4], P[0], P[1], P[2], P[3],
                     P[4], P[5]);
    for (int j = 0; j < 6; ++j) free(P[j]);
    for (int q = 0; q < 5; ++q) {
      free(U1[q]);
      free(U4[q]);
    }
  }
  /* a single cell and a thin pencil */
  {
    double a[5][3];
    double* U[5];
    for (int q = 0; q < 5; ++q) U[q] = a[q];
    for (int i = 0; i < 3; ++i) {
      a[0][i] = 2.0;
      a[1][i] = 0.3;
      a[2][i] = a[3][i] = 0.0;
      a[4][i] = 0.2;
    }
    double led[5] = {0, 0, 0, 0, 0}, me = 0.0;
    int64_t cnt[4] = {0, 0, 0, 0};
    orc_run(&eos[0], 1, 1, 1, 0.4, 1.0, 0, 2, U, led, &me, cnt, 2);
    orc_run(&eos[0], 3, 1, 1, 0.4, 1.0, 0, 2, U, led, &me, cnt, 2);
  }
  if (failures) return 1;
  printf("oracle sanitizer run: ok\n");
  return 0;
}
