/*
 * Plain FP64 CPU oracle of one time step of the relativistic SHASTA
 * (Gerhard, Lindenstruth, Bleicher, "Relativistic Hydrodynamics on Graphic
 * Cards", arXiv:1206.0919).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  The product path (the HIP library
 * under paper_1206_0919_amd/) never links, loads or calls it, and the two
 * share no code, header, table or constant generator.
 *
 * Written for a reader holding the paper: every function names the passage it
 * follows.  Slow and plain on purpose: full arrays for every intermediate of
 * the scheme, true divisions, no fusion, no reordering.  Build flags:
 * -O2 -fno-fast-math -ffp-contract=off, so every expression is evaluated
 * exactly as written.
 *
 * Field order everywhere: 0 = E (T^00), 1 = M_x, 2 = M_y, 3 = M_z,
 * 4 = R (the baryon density N of the paper).  Arrays are dense, x fastest:
 * index = x + nx*(y + ny*z).
 *
 * Readings where the paper is silent or ambiguous (each one is listed with
 * its justification in the design notes of the repository):
 *   - one time step = three directional sweeps with the full dt, in the axis
 *     order of the permutation table of the enqueueing listing (Appendix A,
 *     Listing 2), cycling with period 6 steps;
 *   - the predictor (half step, lambda/2) applies transport, antidiffusion and
 *     limiter like the full step (Sec. 3.1, the half-step method; Listing 2);
 *   - the corrector restarts from U^n with the half-step velocity and source
 *     (Sec. 3, eq. shasta-diff, with v taken half a step later; source at
 *     n+1/2);
 *   - boundaries: three halo cells per side (Sec. 3.1, halo cells), filled by
 *     copying the edge cell (outflow) before each half step;
 *   - the eigenframe recovery is a fixed-point iteration (Sec. 3, last
 *     paragraph) started at v0 = M/E, stopped when two iterates differ by at
 *     most 2^-50, at most 200 iterations; an admissibility guard
 *     E >= 1e-300, |M| <= (1 - 1e-10) E (decided on the squares: |M|^2 >
 *     ((1 - 1e-10) E)^2 clamps) is applied inside the recovery only and
 *     counted once per interior cell and time level (n and n+1/2) of each
 *     sweep; the conserved fields are never modified by it;
 *   - the velocity points along M (eq. cf-momentum);
 *   - the constant diff scales the phoenical antiflux (1 by default); the
 *     runs without antiflux are diff = 0 (Sec. 3.1, Sec. 4);
 *   - a tabled EOS is linear between its nodes, the last segment continuing
 *     past the last node (Sec. 3, where the recovery is written for an
 *     arbitrary p(e));
 *   - the baryon-dependent EOS is p = cs2 max(0, e - m n) with the rest-frame
 *     density n = R sqrt(1 - v^2) updated inside the fixed point (Sec. 3, the
 *     recovery of (e, n) from (E, M, R)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_HALO 3               /* halo width, Sec. 3.1 */
#define ORC_E_FLOOR 1e-300       /* guard: smallest E used by the recovery */
#define ORC_M_FRAC (1.0 - 1e-10) /* guard: largest |M|/E used by the recovery */
#define ORC_VTOL (1.0 / 1125899906842624.0) /* 2^-50 */
#define ORC_MAXIT 200

enum { ORC_NF = 5 };

/* Equation of state.  kind 0: ideal ultra-relativistic gas p = e/3
 * (Sec. 2, the ideal-gas closure).  kind 1: bag model with a first order phase
 * transition: p = e/3 below e_H, p = e_H/3 in the mixed phase
 * e_H < e < e_Q = e_H + 4B, p = (e - 4B)/3 above (the paper leaves the EOS
 * open and mentions tabled ones; this is the standard bag closure).
 * kind 2: tabled EOS (Sec. 2 and Sec. 3, last paragraph: a tabulated p(e)
 * read through an interpolation, the reason the recovery is a root search):
 * nodes te[0] = 0 < te[1] < ... < te[n-1] with pressures tp[k], p(e) linear
 * between neighbouring nodes and the last segment continued beyond te[n-1].
 * kind 3: baryon-dependent EOS p(e, n) = cs2 max(0, e - mass n) (Sec. 3,
 * last paragraph: the pressure follows from the energy density and the
 * baryon density of the rest frame): a gas whose pressure comes from the
 * energy above the rest-mass density mass * n, never negative; the recovery
 * then needs n = R sqrt(1 - v^2) at every iterate. */
typedef struct {
  int kind;
  double B;
  double e_H;
  int n;             /* kind 2: number of nodes (>= 2) */
  const double* te;  /* kind 2: node energy densities */
  const double* tp;  /* kind 2: node pressures */
  double cs2;        /* kind 3: dp/de at fixed n */
  double mass;       /* kind 3: rest mass per baryon [GeV] */
} orc_eos;

/* Pressure at rest-frame energy density e and baryon density nb (nb is used
 * by kind 3 only). */
double orc_pressure(const orc_eos* eos, double e, double nb) {
  if (eos->kind == 0) return e / 3.0;
  if (eos->kind == 3) {
    const double internal = e - eos->mass * nb;
    return eos->cs2 * (internal > 0.0 ? internal : 0.0);
  }
  if (eos->kind == 2) {
    /* segment k with te[k] <= e < te[k+1], by bisection over the nodes;
     * k = n-2 for e >= te[n-2] (the last segment, extended) */
    int lo = 0, hi = eos->n - 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (eos->te[mid] <= e) lo = mid; else hi = mid;
    }
    const int k = lo;
    const double slope = (eos->tp[k + 1] - eos->tp[k]) / (eos->te[k + 1] - eos->te[k]);
    return eos->tp[k] + slope * (e - eos->te[k]);
  }
  const double e_Q = eos->e_H + 4.0 * eos->B;
  if (e <= eos->e_H) return e / 3.0;
  if (e < e_Q) return eos->e_H / 3.0;
  return (e - 4.0 * eos->B) / 3.0;
}

/* Counters of guard activations and failures (reductions of the step). */
typedef struct {
  int64_t clamp;   /* |M| lowered to (1-1e-10) E */
  int64_t floor;   /* E raised to the floor */
  int64_t noconv;  /* fixed point did not converge in ORC_MAXIT iterations */
  int64_t nonfinite;
} orc_counters;

/* Eigenframe recovery (Sec. 3, last paragraph: boost to the rest frame by a
 * fixed-point root search).  From E = (e+p) gamma^2 - p and
 * |M| = (e+p) gamma^2 v (eqs. cf-energy, cf-momentum) follows
 * v = |M| / (E + p(e)) with e = E - |M| v; this map is iterated.
 * Outputs e, p, v (speed) and the velocity vector along M.
 * The momentum components are passed as (M_a, M_b, M_c) and |M|^2 is summed
 * as M_a^2 + (M_b^2 + M_c^2): a sweep passes its parallel component first, so
 * the result does not depend on how the two transverse axes are labelled. */
int orc_recover(const orc_eos* eos, double E, double Mx, double My, double Mz,
                double R, double* e_out, double* p_out, double* v_out, double* vx,
                double* vy, double* vz, int* iters_out, int* clamped,
                int* floored) {
  const double M2 = Mx * Mx + (My * My + Mz * Mz);
  const double M = sqrt(M2);
  double Ec = E, Mc = M;
  int fl = 0, cl = 0, conv = 1, it = 0;
  if (!(Ec >= ORC_E_FLOOR)) { Ec = ORC_E_FLOOR; fl = 1; }
  /* the guard compares squares, |M|^2 > ((1-1e-10) E)^2, so that the
   * decision needs no square root */
  const double Mmax = ORC_M_FRAC * Ec;
  if (M2 > Mmax * Mmax) { Mc = Mmax; cl = 1; }
  double v = 0.0;
  if (Mc > 0.0) {
    v = Mc / Ec;
    for (;;) {
      const double e_trial = Ec - Mc * v;
      const double n_trial = R * sqrt(1.0 - v * v);
      const double vn = Mc / (Ec + orc_pressure(eos, e_trial, n_trial));
      ++it;
      const double change = fabs(vn - v);
      v = vn;
      if (change <= ORC_VTOL) break;
      if (it >= ORC_MAXIT) { conv = 0; break; }
    }
  }
  const double e = Ec - Mc * v;
  *e_out = e;
  *p_out = orc_pressure(eos, e, R * sqrt(1.0 - v * v));
  *v_out = v;
  if (M > 0.0) {
    *vx = v * Mx / M;
    *vy = v * My / M;
    *vz = v * Mz / M;
  } else {
    *vx = *vy = *vz = 0.0;
  }
  if (iters_out) *iters_out = it;
  if (clamped) *clamped = cl;
  if (floored) *floored = fl;
  return conv;
}

/* Primitive -> conserved (eqs. cf-density, cf-momentum, cf-energy):
 * N = n gamma, M = (e+p) gamma^2 v, E = (e + p v^2) gamma^2. */
void orc_prim_to_cons(const orc_eos* eos, int64_t ncell, const double* e,
                      const double* vx, const double* vy, const double* vz,
                      const double* n, double* E, double* Mx, double* My,
                      double* Mz, double* R) {
  for (int64_t i = 0; i < ncell; ++i) {
    const double p = orc_pressure(eos, e[i], n[i]);
    const double v2 = vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
    const double g2 = 1.0 / (1.0 - v2);
    const double w = (e[i] + p) * g2;
    E[i] = (e[i] + p * v2) * g2;
    Mx[i] = w * vx[i];
    My[i] = w * vy[i];
    Mz[i] = w * vz[i];
    R[i] = n[i] * sqrt(g2);
  }
}

/* Conserved -> primitive via orc_recover; n = N / gamma = R sqrt(1 - v^2). */
void orc_cons_to_prim(const orc_eos* eos, int64_t ncell, const double* E,
                      const double* Mx, const double* My, const double* Mz,
                      const double* R, double* e, double* p, double* vx,
                      double* vy, double* vz, double* n) {
  for (int64_t i = 0; i < ncell; ++i) {
    double v;
    orc_recover(eos, E[i], Mx[i], My[i], Mz[i], R[i], &e[i], &p[i], &v, &vx[i],
                &vy[i], &vz[i], NULL, NULL, NULL);
    n[i] = R[i] * sqrt(1.0 - v * v);
  }
}

static double orc_sgn(double a) { return (a > 0.0) - (a < 0.0); }

/* One-dimensional SHASTA update of one quantity along one pencil
 * (Sec. 3, eqs. shasta-diff, shasta-geo, the phoenical antidiffusion, the
 * flux limiter and eq. shasta-n).
 *
 * U, eps, f hold N+6 values: index j of the paper sits at position j+3, so
 * that j runs over the halo -3..N+2.  eps_j = lambda' v_j is the local Courant
 * number with the (time-staggered) velocity, f_j the source variable (p for
 * the momentum along the sweep, p v for the energy, unused if !has_source),
 * lam = lambda' = dt'/dx.  diff scales the antidiffusion (Listing 1 constant).
 * Writes U^{new}_j, j = 0..N-1, to unew.  If flux is non-NULL it receives the
 * total (transport + source + antidiffusive) flux through the left interface
 * -1/2 (flux[0]) and the right interface N-1/2 (flux[1]) in cell-sum units;
 * their difference is the change of sum_j U_j (flux form of eq. shasta-geo,
 * which holds because Q+_j + Q-_{j+1} = 1). */
void orc_fct_1d(int N, const double* U, const double* eps, const double* f,
                int has_source, double lam, double diff, double* unew,
                double* flux) {
  const int n = N + 2 * ORC_HALO;
  double* Qp = (double*)calloc((size_t)n, sizeof(double));
  double* Qm = (double*)calloc((size_t)n, sizeof(double));
  double* D = (double*)calloc((size_t)n, sizeof(double));
  double* Uh = (double*)calloc((size_t)n, sizeof(double));
  double* Dh = (double*)calloc((size_t)n, sizeof(double));
  double* A = (double*)calloc((size_t)n, sizeof(double));
#define P(j) ((j) + ORC_HALO)
  /* geometric factors, eq. shasta-diff, for j = -2..N+1 */
  for (int j = -2; j <= N + 1; ++j) {
    Qp[P(j)] = (0.5 - eps[P(j)]) / (1.0 + (eps[P(j + 1)] - eps[P(j)]));
    Qm[P(j)] = (0.5 + eps[P(j)]) / (1.0 - (eps[P(j - 1)] - eps[P(j)]));
  }
  /* Delta_j = U_{j+1} - U_j, j = -3..N+1 */
  for (int j = -3; j <= N + 1; ++j) D[P(j)] = U[P(j + 1)] - U[P(j)];
  /* geometric transport with diffusion, eq. shasta-geo, j = -2..N+1;
   * source term lambda * Delta(f), Delta(f) = -1/2 (f_{j+1} - f_{j-1}) */
  for (int j = -2; j <= N + 1; ++j) {
    const double src =
        has_source ? lam * (-0.5) * (f[P(j + 1)] - f[P(j - 1)]) : 0.0;
    Uh[P(j)] = (0.5 * Qp[P(j)] * Qp[P(j)] * D[P(j)] -
                0.5 * Qm[P(j)] * Qm[P(j)] * D[P(j - 1)]) +
               (Qp[P(j)] + Qm[P(j)]) * U[P(j)] + src;
  }
  /* hat Delta_j = hat U_{j+1} - hat U_j, j = -2..N */
  for (int j = -2; j <= N; ++j) Dh[P(j)] = Uh[P(j + 1)] - Uh[P(j)];
  /* phoenical antidiffusion and the flux limiter, j = -1..N-1 */
  for (int j = -1; j <= N - 1; ++j) {
    const double second = (D[P(j + 1)] + D[P(j - 1)]) - 2.0 * D[P(j)];
    const double Aph = (diff / 8.0) * (Dh[P(j)] - second / 8.0);
    const double s = orc_sgn(Aph);
    const double m = fmin(fmin(s * Dh[P(j + 1)], fabs(Aph)), s * Dh[P(j - 1)]);
    A[P(j)] = s * fmax(0.0, m);
  }
  /* update, eq. shasta-n */
  for (int j = 0; j <= N - 1; ++j) unew[j] = Uh[P(j)] - (A[P(j)] - A[P(j - 1)]);
  if (flux) {
    /* F_{j+1/2} = (1/2 - Q+_j) U_j - 1/2 Q+_j^2 Delta_j
     *             + 1/2 lambda (f_j + f_{j+1}) + A_j */
    const int js[2] = {-1, N - 1};
    for (int k = 0; k < 2; ++k) {
      const int j = js[k];
      double F = (0.5 - Qp[P(j)]) * U[P(j)] - 0.5 * Qp[P(j)] * Qp[P(j)] * D[P(j)];
      if (has_source) F += 0.5 * lam * (f[P(j)] + f[P(j + 1)]);
      flux[k] = F + A[P(j)];
    }
  }
#undef P
  free(Qp); free(Qm); free(D); free(Uh); free(Dh); free(A);
}

/* Outflow halo: the three cells beyond each end copy the edge cell
 * (Sec. 3.1 halo cells; boundary reading in the header). */
static void orc_fill_halo(int N, double* u) {
  for (int g = 1; g <= ORC_HALO; ++g) {
    u[ORC_HALO - g] = u[ORC_HALO];
    u[ORC_HALO + N - 1 + g] = u[ORC_HALO + N - 1];
  }
}

/* One directional sweep of one pencil: half-step predictor and full-step
 * corrector (Sec. 3, eqs. shasta-diff..shasta-n with staggered v and f;
 * Sec. 3.1 half-step method; Listing 2: recovery, lambda/2, propagation).
 * u[q] (q = 0..4) hold the pencil with halo, N+6 values; on return the
 * interior holds U^{n+1}.  axis selects M_axis as the parallel momentum.
 * bflux[q] accumulates right-minus-left boundary flux of the corrector,
 * maxeps the largest |lambda v_axis| seen in the corrector. */
static void orc_sweep_pencil(const orc_eos* eos, int N, int axis, double lam,
                             double diff, double** u, double* bflux,
                             double* maxeps, orc_counters* cnt) {
  const int n = N + 2 * ORC_HALO;
  double* uh[ORC_NF];
  for (int q = 0; q < ORC_NF; ++q) uh[q] = (double*)calloc((size_t)n, sizeof(double));
  double* eps = (double*)calloc((size_t)n, sizeof(double));
  double* fE = (double*)calloc((size_t)n, sizeof(double));
  double* fM = (double*)calloc((size_t)n, sizeof(double));
  const int qpar = 1 + axis;            /* momentum along the sweep */
  const int qt1 = 1 + (axis == 0 ? 1 : 0); /* the two transverse momenta */
  const int qt2 = 1 + (axis == 2 ? 1 : 2);

  /* time level n: halo, then recovery on all N+6 cells; guard activations
   * and failures are counted on the N interior cells only (a halo cell
   * repeats its edge cell) */
  for (int q = 0; q < ORC_NF; ++q) orc_fill_halo(N, u[q]);
  for (int i = 0; i < n; ++i) {
    double e, p, v, vel[3];
    int it, cl, fl;
    const int interior = i >= ORC_HALO && i < ORC_HALO + N;
    if (!orc_recover(eos, u[0][i], u[qpar][i], u[qt1][i], u[qt2][i], u[4][i], &e, &p,
                     &v, &vel[0], &vel[1], &vel[2], &it, &cl, &fl))
      cnt->noconv += interior;
    cnt->clamp += interior * cl;
    cnt->floor += interior * fl;
    eps[i] = (0.5 * lam) * vel[0];
    fE[i] = p * vel[0];
    fM[i] = p;
  }
  /* predictor: U^{n+1/2} = SHASTA(U^n; v^n, f^n; lambda/2) */
  for (int q = 0; q < ORC_NF; ++q) {
    const double* f = (q == 0) ? fE : fM;
    const int src = (q == 0) || (q == qpar);
    orc_fct_1d(N, u[q], eps, f, src, 0.5 * lam, diff, uh[q] + ORC_HALO, NULL);
  }
  /* time level n+1/2: halo, recovery */
  for (int q = 0; q < ORC_NF; ++q) orc_fill_halo(N, uh[q]);
  for (int i = 0; i < n; ++i) {
    double e, p, v, vel[3];
    int it, cl, fl;
    const int interior = i >= ORC_HALO && i < ORC_HALO + N;
    if (!orc_recover(eos, uh[0][i], uh[qpar][i], uh[qt1][i], uh[qt2][i], uh[4][i], &e,
                     &p, &v, &vel[0], &vel[1], &vel[2], &it, &cl, &fl))
      cnt->noconv += interior;
    cnt->clamp += interior * cl;
    cnt->floor += interior * fl;
    eps[i] = lam * vel[0];
    fE[i] = p * vel[0];
    fM[i] = p;
    if (fabs(eps[i]) > *maxeps) *maxeps = fabs(eps[i]);
  }
  /* corrector: U^{n+1} = SHASTA(U^n; v^{n+1/2}, f^{n+1/2}; lambda) */
  double* out = (double*)calloc((size_t)N, sizeof(double));
  for (int q = 0; q < ORC_NF; ++q) {
    const double* f = (q == 0) ? fE : fM;
    const int src = (q == 0) || (q == qpar);
    double fl[2];
    orc_fct_1d(N, u[q], eps, f, src, lam, diff, out, fl);
    bflux[q] += fl[1] - fl[0];
    memcpy(u[q] + ORC_HALO, out, (size_t)N * sizeof(double));
  }
  free(out);
  for (int q = 0; q < ORC_NF; ++q) free(uh[q]);
  free(eps); free(fE); free(fM);
}

/* Axis order of each time step: the permutation table of Listing 2
 * (six permutations of (x, y, z), three sweeps each). */
static const int orc_branch[18] = {0, 1, 2, 0, 2, 1, 2, 0, 1,
                                   2, 1, 0, 1, 2, 0, 1, 0, 2};

int orc_axis_of(int64_t step, int sweep) {
  return orc_branch[3 * (int)(step % 6) + sweep];
}

/* One sweep of the whole grid along one axis.  Every pencil is independent,
 * so the OpenMP split does not change any result.  The boundary flux of each
 * pencil is stored per pencil and summed serially (Neumaier) afterwards, so
 * ledger values do not depend on the thread count either. */
void orc_sweep(const orc_eos* eos, int nx, int ny, int nz, int axis,
               double lam, double diff, double** U, double* ledger,
               double* maxeps, int64_t* counters, int nthreads) {
  const int dims[3] = {nx, ny, nz};
  const int64_t stride[3] = {1, nx, (int64_t)nx * ny};
  const int N = dims[axis];
  const int a1 = (axis == 0) ? 1 : 0;
  const int a2 = (axis == 2) ? 1 : 2;
  const int64_t npen = (int64_t)dims[a1] * dims[a2];
  double* pflux = (double*)calloc((size_t)(npen * ORC_NF), sizeof(double));
  double* pmax = (double*)calloc((size_t)npen, sizeof(double));
  orc_counters tot = {0, 0, 0, 0};
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    orc_counters cnt = {0, 0, 0, 0};
    double* pen[ORC_NF];
    for (int q = 0; q < ORC_NF; ++q)
      pen[q] = (double*)calloc((size_t)(N + 2 * ORC_HALO), sizeof(double));
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t pi = 0; pi < npen; ++pi) {
      const int64_t i1 = pi % dims[a1], i2 = pi / dims[a1];
      const int64_t base = i1 * stride[a1] + i2 * stride[a2];
      for (int q = 0; q < ORC_NF; ++q)
        for (int j = 0; j < N; ++j)
          pen[q][ORC_HALO + j] = U[q][base + j * stride[axis]];
      orc_sweep_pencil(eos, N, axis, lam, diff, pen, &pflux[pi * ORC_NF],
                       &pmax[pi], &cnt);
      for (int q = 0; q < ORC_NF; ++q)
        for (int j = 0; j < N; ++j)
          U[q][base + j * stride[axis]] = pen[q][ORC_HALO + j];
    }
    for (int q = 0; q < ORC_NF; ++q) free(pen[q]);
    /* integer counters: the order of the additions does not matter */
#ifdef _OPENMP
#pragma omp atomic
#endif
    tot.clamp += cnt.clamp;
#ifdef _OPENMP
#pragma omp atomic
#endif
    tot.floor += cnt.floor;
#ifdef _OPENMP
#pragma omp atomic
#endif
    tot.noconv += cnt.noconv;
  }
  for (int q = 0; q < ORC_NF; ++q) {
    double s = 0.0, c = 0.0;
    for (int64_t pi = 0; pi < npen; ++pi) {
      const double x = pflux[pi * ORC_NF + q];
      const double t = s + x;
      c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
      s = t;
    }
    ledger[q] += s + c;
  }
  for (int64_t pi = 0; pi < npen; ++pi)
    if (pmax[pi] > *maxeps) *maxeps = pmax[pi];
  if (counters) {
    counters[0] += tot.clamp;
    counters[1] += tot.floor;
    counters[2] += tot.noconv;
  }
  free(pflux);
  free(pmax);
}

/* nsteps full time steps starting at step index k0 (Listing 2 schedule).
 * lam = dt/dx.  ledger[q] accumulates the net boundary outflow of field q. */
void orc_run(const orc_eos* eos, int nx, int ny, int nz, double lam,
             double diff, int64_t k0, int nsteps, double** U, double* ledger,
             double* maxeps, int64_t* counters, int nthreads) {
  for (int s = 0; s < nsteps; ++s)
    for (int w = 0; w < 3; ++w)
      orc_sweep(eos, nx, ny, nz, orc_axis_of(k0 + s, w), lam, diff, U, ledger,
                maxeps, counters, nthreads);
}

/* Neumaier-compensated sum of one field over the interior. */
double orc_sum(int64_t n, const double* a) {
  double s = 0.0, c = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double t = s + a[i];
    c += (fabs(s) >= fabs(a[i])) ? (s - t) + a[i] : (a[i] - t) + s;
    s = t;
  }
  return s + c;
}

int orc_count_nonfinite(int64_t n, const double* a) {
  int c = 0;
  for (int64_t i = 0; i < n; ++i) c += !isfinite(a[i]);
  return c;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
