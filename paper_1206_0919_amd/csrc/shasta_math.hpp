// Device arithmetic of the relativistic SHASTA step (arXiv:1206.0919).
//
// Every function here is shared by the x-sweep and the y/z-sweep kernels, so
// both organisations of the stencil evaluate identical expressions and their
// results agree bit for bit.  FP contraction is off for the whole library:
// every fused multiply-add is written out.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shasta_internal.hpp"

namespace shasta {

constexpr double kEFloor = 1e-300;       // recovery guard: smallest E
constexpr double kMFrac = 1.0 - 1e-10;   // recovery guard: largest |M|/E
constexpr double kThird = 1.0 / 3.0;

// ------------------------------------------------------------ reciprocal, sqrt
// FP64 reciprocal: hardware estimate (relative error below 5e-8 on gfx950)
// refined by two Newton steps r <- r + r (1 - x r): one step leaves up to
// about 20 ulp, two give the correctly rounded reciprocal on a million
// samples over 120 binades.
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  return r;
}
// FP32 reciprocal: the hardware estimate is accurate to 1 ulp.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// FP64 square root of a positive normal number: reciprocal square root
// estimate (relative error below 6e-8 on gfx950) refined by one coupled
// Newton (Goldschmidt) step for g = sqrt(x), h = 1/(2 sqrt(x)) (then within
// about 40 ulp), then one residual correction g + (x - g^2) h, which on a
// million samples over 120 binades gave the correctly rounded root.
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = 0.5 * y;
  const double r = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  const double d = __builtin_fma(-g, g, x);
  return __builtin_fma(d, h, g);
}

// The same with one refinement step less, for recoveries whose results are
// rounded to FP32 (the sweeps of FP32 fields): the reciprocal within about
// 20 ulp and the root within about 40 ulp of FP64, some 1e-7 of an FP32 ulp.
template <bool kFast>
__device__ __forceinline__ double rcp_r(double x) {
  if constexpr (!kFast) return rcp(x);
  const double r = __builtin_amdgcn_rcp(x);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
template <bool kFast>
__device__ __forceinline__ double sqrt_r(double x) {
  if constexpr (!kFast) return sqrt_pos(x);
  const double y = __builtin_amdgcn_rsq(x);
  const double g = x * y;
  const double r = __builtin_fma(-g, 0.5 * y, 0.5);
  return __builtin_fma(g, r, g);
}

// True if any lane of the wave has pred set (a wave-uniform branch lets the
// rare paths below cost nothing when no lane takes them).
__device__ __forceinline__ bool any_lane(bool pred) {
  return __builtin_amdgcn_ballot_w64(pred) != 0;
}

// -------------------------------------------------------------------- EOS
// Recovery of the rest frame (Sec. 3, last paragraph).  For an EOS that is
// linear on a branch, p = a e + b, the condition v (E + p(E - M v)) = M is a
// quadratic in v whose physical root is v = M w with
//   w = 2 / (K + sqrt(K^2 - 4 a M^2)),  K = (1 + a) E + b   (a > 0),
//   w = 1 / (E + b)                                          (a = 0).
// This is the same root the fixed-point iteration of the paper converges
// to (the root is unique); it is evaluated directly.  The guard of the
// recovery (E >= 1e-300, |M| <= (1 - 1e-10) E) is applied here and counted;
// the conserved fields themselves are never changed.
//
// Inputs: E and the momentum along the sweep (Mpar) and across it (Mt1,
// Mt2).  |M|^2 = Mpar^2 + (Mt1^2 + Mt2^2), symmetric in the transverse pair.
// Outputs: the velocity along the sweep, the pressure, guard flags.
struct Recovered {
  double w;    // v / |M|: velocity component i = w M_i
  double e;    // rest-frame energy density
  double p;    // pressure
  double M2;   // |M|^2 as summed here
  int clamped;
  int floored;
  int noconv;  // the iterative root solve stopped before converging (EOS 3)
};

// w = v/|M_c| and e for p = e/3, on (E, M^2) of moderate size.
template <bool kFast = false>
__device__ __forceinline__ void ideal_root(double E, double M2, double& w,
                                           double& e) {
  // v = 3 M / (2 E + sqrt(4 E^2 - 3 M^2)),  e = E - M v
  const double s = sqrt_r<kFast>(__builtin_fma(4.0 * E, E, -3.0 * M2));
  w = 3.0 * rcp_r<kFast>(__builtin_fma(2.0, E, s));
  e = __builtin_fma(-M2, w, E);
}

// |M|^2 of the recovery on E scaled to Es = E 2^-k: the guard's limit
// ((1 - 1e-10) Es)^2 if |M| was clamped (its square at the original scale
// may underflow, e.g. for E at the floor), else M2 2^-2k.
__device__ __forceinline__ double scaled_m2(double Es, double M2, int k, bool clamped) {
  const double kEs = kMFrac * Es;
  return clamped ? kEs * kEs : __builtin_ldexp(M2, -2 * k);
}

__device__ __forceinline__ void ideal_root_scaled(double E, double M2, bool clamped,
                                                  double& w, double& e) {
  // The root is homogeneous of degree 0 in (E, M): solve on (E, M) scaled
  // by a power of two when the squares would leave the normal range.
  const int k = __builtin_amdgcn_frexp_exp(E);
  const double Es = __builtin_ldexp(E, -k);
  double ws, es;
  ideal_root(Es, scaled_m2(Es, M2, k, clamped), ws, es);
  w = __builtin_ldexp(ws, -k);
  e = __builtin_ldexp(es, k);
}

// Root of a linear EOS branch p = a e + b (a >= 0): w = v/|M| and e.  The
// root is homogeneous of degree 0 in (E, M, b) for w E, so the squares are
// kept in the normal range by a power-of-two scaling of all three.
template <bool kFast = false>
__device__ __forceinline__ void linear_root(double a, double b, double E, double M2,
                                            double& w, double& e) {
  const double K = __builtin_fma(1.0 + a, E, b);
  const double disc = fmax(__builtin_fma(K, K, -4.0 * a * M2), 0.0);
  w = 2.0 * rcp_r<kFast>(K + sqrt_r<kFast>(disc));
  e = __builtin_fma(-M2, w, E);
}
__device__ __forceinline__ void linear_root_scaled(double a, double b, double E, double M2,
                                                   bool clamped, double& w, double& e) {
  const int k = __builtin_amdgcn_frexp_exp(E);
  const double Es = __builtin_ldexp(E, -k);
  double ws, es;
  linear_root(a, __builtin_ldexp(b, -k), Es, scaled_m2(Es, M2, k, clamped), ws, es);
  w = __builtin_ldexp(ws, -k);
  e = __builtin_ldexp(es, k);
}

// Baryon-dependent EOS p = a max(0, e - m n) with n = R sqrt(1 - v^2) (the
// rest-frame baryon density): the recovery condition f(v) = v (E + p) - |M|
// = 0 has no closed form.  f increases with v; its root is |M|/E (a
// pressureless state) exactly when x = e - m n <= 0 there, else it lies on
// the smooth branch p = a x, inside [v0, |M|/E] with v0 the root without rest
// mass (a lower bound: the rest mass lowers p).  The smooth branch is solved
// by Newton's method, safeguarded by bisection of that bracket.  f is
// homogeneous in (E, |M|, m R), so the solve runs on inputs scaled by a power
// of two.  A lane keeps its first iterate whose step (or bracket) is at most
// 4 ulp, so its result does not depend on the other lanes of the wave (at
// most 9 iterations on random states).  At most max_it iterations (16 by
// default); a lane still moving then keeps its last iterate and returns true
// (not converged), which the sweeps count.  mR = m R.
__device__ __forceinline__ bool baryon_root(double a, double mR, double E, double M2,
                                            bool clamped, int max_it, double& w, double& e,
                                            double& p) {
  const int k = __builtin_amdgcn_frexp_exp(E);
  const double Es = __builtin_ldexp(E, -k);
  const double M2s = scaled_m2(Es, M2, k, clamped);
  const double mRs = __builtin_ldexp(mR, -k);
  const bool moving = M2s > 0.0;
  const double Ms = moving ? sqrt_pos(M2s) : 0.0;
  const double vd = Ms * rcp(Es);   // the pressureless root
  const double xd =
      __builtin_fma(-mRs, sqrt_pos(__builtin_fma(-vd, vd, 1.0)), __builtin_fma(-Ms, vd, Es));
  double w0, e0;
  linear_root(a, 0.0, Es, M2s, w0, e0);
  double v = (xd > 0.0) ? Ms * w0 : vd;
  double lo = v, hi = vd;
  bool done = !moving || !(xd > 0.0);
  for (int it = 0; it < max_it; ++it) {
    if (!any_lane(!done)) break;
    const double s = sqrt_pos(__builtin_fma(-v, v, 1.0));
    const double x = __builtin_fma(-mRs, s, __builtin_fma(-Ms, v, Es));
    const double pv = a * x;
    const double f = __builtin_fma(v, Es + pv, -Ms);
    const double dp = a * __builtin_fma(mRs * v, rcp(s), -Ms);
    const double df = __builtin_fma(v, dp, Es + pv);
    lo = (f < 0.0) ? v : lo;
    hi = (f < 0.0) ? hi : v;
    // Newton step if it stays in the closed bracket (at an exact root f = 0
    // and the step is 0), else bisection; done when the step or the bracket
    // is at most 4 ulp
    double vn = __builtin_fma(-f, rcp(df), v);
    vn = (vn >= lo && vn <= hi) ? vn : 0.5 * (lo + hi);
    const double tol = 8.8817841970012523e-16 * v;   // 4 ulp
    const bool conv = fabs(vn - v) <= tol || hi - lo <= tol;
    v = done ? v : vn;
    done = done || conv;
  }
  const double s = sqrt_pos(__builtin_fma(-v, v, 1.0));
  const double es = __builtin_fma(-Ms, v, Es);
  e = __builtin_ldexp(es, k);
  p = __builtin_ldexp(a * fmax(__builtin_fma(-mRs, s, es), 0.0), k);
  w = moving ? __builtin_ldexp(v * rcp(Ms), -k) : 0.0;
  return !done;
}

// Tabled EOS: segment of node e_k that holds e (largest k <= m-2 with
// e_k <= e), by a search with the same trip count in every lane.
__device__ __forceinline__ int table_segment_of_e(const EosParams& eos, double e) {
  const int m = eos.n;
  int k = 0;
  for (int step = 1 << (31 - __builtin_clz(m - 1)); step > 0; step >>= 1)
    if (k + step <= m - 2 && eos.tab[k + step] <= e) k += step;
  return k;
}
__device__ __forceinline__ double table_pressure(const EosParams& eos, double e) {
  const int k = table_segment_of_e(eos, e);
  return __builtin_fma(eos.tab[2 * eos.n + k], e, eos.tab[3 * eos.n + k]);
}


// EOS: 0 = ideal gas p = e/3, 1 = bag model, 2 = tabled p(e), linear between
// nodes, 3 = baryon-dependent p(e, n) (compile-time, as the paper specialises
// its kernels per EOS instead of branching at run time).  R, the fifth
// conserved field, is used by EOS 3 only.  kFast: results rounded to FP32
// afterwards, one refinement step less in the common path (rcp_r, sqrt_r).
template <int EOS, bool kFast = false>
__device__ __forceinline__ Recovered recover(const EosParams& eos, double E,
                                             double Mpar, double Mt1,
                                             double Mt2, double R) {
  Recovered r;
  const double t = Mt1 * Mt1 + Mt2 * Mt2;
  const double M2 = __builtin_fma(Mpar, Mpar, t);
  r.M2 = M2;
  r.noconv = 0;
  r.floored = !(E >= kEFloor);
  const double Ec = r.floored ? kEFloor : E;
  const double kE = kMFrac * Ec;
  const double kE2 = kE * kE;
  r.clamped = M2 > kE2;
  const double M2c = r.clamped ? kE2 : M2;
  double w, e;
  bool rare;
  double ta = 0.0, tb = 0.0;   // tabled EOS: the segment's p = ta e + tb
  if constexpr (EOS == 0) {
    rare = !(Ec > 1e-140 && Ec < 1e140);
    ideal_root<kFast>(Ec, M2c, w, e);
  } else if constexpr (EOS == 3) {
    rare = false;   // the solve is scaled by construction
    r.noconv = baryon_root(eos.cs2, eos.mass * R, Ec, M2, r.clamped, eos.newton_max, w, e,
                           r.p);
  } else if constexpr (EOS == 2) {
    // Tabled EOS: the recovery function v (E + p(E - M v)) - M increases
    // with v, so the root e* lies above node e_k exactly when
    // (E - e_k)(E + p_k) > |M|^2; the largest such k <= m-2 gives the
    // segment (the last one continues past the last node), whose line
    // p = a e + b gives the root in closed form.
    const int m = eos.n;
    const double* te = eos.tab;
    const double* tp = eos.tab + m;
    int k = 0;
    for (int step = 1 << (31 - __builtin_clz(m - 1)); step > 0; step >>= 1) {
      const int j = k + step;
      if (j <= m - 2 && M2c < (Ec - te[j]) * (Ec + tp[j])) k = j;
    }
    ta = eos.tab[2 * m + k];
    tb = eos.tab[3 * m + k];
    rare = !(Ec > 1e-140 && Ec < 1e140);
    linear_root<kFast>(ta, tb, Ec, M2c, w, e);
    r.p = __builtin_fma(ta, e, tb);
  } else {
    // bag model: the recovery function v (E + p(E - M v)) - M increases with
    // v, so its sign at the edges of the mixed phase selects the branch:
    // hadron gas if e* <= e_H, plasma if e* >= e_Q, mixed phase otherwise.
    const double eH = eos.e_H;
    const double eQ = eos.e_H + 4.0 * eos.B;
    const double pc = eos.e_H * kThird;
    const bool hadron = (Ec <= eH) || ((Ec - eH) * (Ec + pc) <= M2c);
    const bool qgp = !hadron && (Ec > eQ) && ((Ec - eQ) * (Ec + pc) >= M2c);
    const bool mixed = !hadron && !qgp;
    const double b = qgp ? -(4.0 * kThird) * eos.B : 0.0;
    const double K = __builtin_fma(4.0 * kThird, Ec, b);
    const double dq =
        0.5 * (K + sqrt_r<kFast>(__builtin_fma(K, K, -(4.0 * kThird) * M2c)));
    const double den = mixed ? (Ec + pc) : dq;
    w = rcp_r<kFast>(den);
    e = __builtin_fma(-M2c, w, Ec);
    r.p = mixed ? pc : __builtin_fma(kThird, e, b);
    rare = hadron && !(Ec > 1e-140);
  }
  if constexpr (EOS == 0) r.p = e * kThird;
  // One wave-uniform branch for both rare paths: scaled root (the squares
  // would leave the normal range; on the bag EOS only in the hadron phase)
  // and clamped |M|: v_i = v M_i / |M| = w M_c M_i / |M|, M_c = |M| unless
  // clamped.
  if (any_lane(rare || r.clamped)) {
    if (rare) {
      if constexpr (EOS == 2) {
        linear_root_scaled(ta, tb, Ec, M2, r.clamped, w, e);
        r.p = __builtin_fma(ta, e, tb);
      } else {
        ideal_root_scaled(Ec, M2, r.clamped, w, e);
        r.p = e * kThird;
      }
    }
    if (r.clamped) w *= kE * rcp(sqrt_pos(M2));
  }
  r.w = w;
  r.e = e;
  return r;
}

// ------------------------------------------------------------ typed helpers
// Fused multiply-add, min, max, |x| and copysign in the precision of their
// operands: the FCT of the FP32 fields runs in FP32 (the unsuffixed builtins
// are the double versions and would promote float operands).
template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}
template <typename T>
__device__ __forceinline__ T fmin_t(T a, T b) {
  if constexpr (sizeof(T) == 4) return __builtin_fminf(a, b);
  else return __builtin_fmin(a, b);
}
template <typename T>
__device__ __forceinline__ T fmax_t(T a, T b) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaxf(a, b);
  else return __builtin_fmax(a, b);
}
template <typename T>
__device__ __forceinline__ T fabs_t(T a) {
  if constexpr (sizeof(T) == 4) return __builtin_fabsf(a);
  else return __builtin_fabs(a);
}
template <typename T>
__device__ __forceinline__ T copysign_t(T a, T b) {
  if constexpr (sizeof(T) == 4) return __builtin_copysignf(a, b);
  else return __builtin_copysign(a, b);
}

// ------------------------------------------------------------ SHASTA pieces
// Geometric factors (eq. shasta-diff) share one reciprocal per interface:
// Q+_j = (1/2 - eps_j) / D_{j+1/2},  Q-_j = (1/2 + eps_j) / D_{j-1/2},
// D_{j+1/2} = 1 + (eps_{j+1} - eps_j).
template <typename T>
__device__ __forceinline__ T interface_rcp(T eps_left, T eps_right) {
  return rcp(T(1) + (eps_right - eps_left));
}

template <typename T>
struct Coef {
  T a;  // 1/2 Q+^2
  T b;  // 1/2 Q-^2
  T c;  // Q+ + Q-
};

template <typename T>
__device__ __forceinline__ Coef<T> coefficients(T eps, T rd_left, T rd_right) {
  const T qp = (T(0.5) - eps) * rd_right;
  const T qm = (T(0.5) + eps) * rd_left;
  Coef<T> k;
  k.a = T(0.5) * (qp * qp);
  k.b = T(0.5) * (qm * qm);
  k.c = qp + qm;
  return k;
}

// Source term lambda' Delta(f), Delta(f) = -1/2 (f_{j+1} - f_{j-1});
// lamsrc = -lambda'/2.
template <typename T>
__device__ __forceinline__ T source(T lamsrc, T f_left, T f_right) {
  return lamsrc * (f_right - f_left);
}

// Transport with diffusion (eq. shasta-geo):
// hat U_j = 1/2 Q+^2 Delta_j - 1/2 Q-^2 Delta_{j-1} + (Q+ + Q-) U_j + src.
template <typename T>
__device__ __forceinline__ T transport(const Coef<T>& k, T src, T d_right,
                                       T d_left, T u) {
  return fma_t(k.a, d_right, fma_t(-k.b, d_left, fma_t(k.c, u, src)));
}

// Second difference of Delta used by the phoenical antidiffusion,
// (d_next + d_prev) - 2 d; 2 d is exact, so the fused form rounds the same.
template <typename T>
__device__ __forceinline__ T second_difference(T d_next, T d_prev, T d) {
  return fma_t(T(-2), d, d_next + d_prev);
}

// Scales of the phoenical antiflux: A^ph = c8 hat Delta + c64 second with
// c8 = diff/8, c64 = -diff/64 (for diff a power of two, as the default 1,
// this rounds exactly as diff/8 (hat Delta - second/8)).
template <typename T>
struct Antidiff {
  T c8, c64;
};
template <typename T>
__device__ __forceinline__ Antidiff<T> antidiff_scales(double diff) {
  return Antidiff<T>{T(diff * 0.125), T(diff * -0.015625)};
}

// Phoenical antidiffusion with the strong flux limiter:
// A^ph_j = diff/8 (hat Delta_j - 1/8 second),  sigma = sgn A^ph_j,
// A_j = sigma max(0, min(sigma hat Delta_{j+1}, |A^ph_j|, sigma hat Delta_{j-1})).
// sigma is taken as copysign(1, A^ph); at A^ph = 0 the result is 0 either way.
// FP32 form, with the same value: for sigma = +1 the limited flux is
// max(0, min(A^ph, lo)) with lo = min(hat Delta_{j+1}, hat Delta_{j-1}), for
// sigma = -1 it is min(0, max(A^ph, hi)) with hi their max; both are the
// median of (0, A^ph, lo or hi), and lo or hi is itself the median of the two
// differences and -sigma infinity.  Two median-of-three instructions replace
// two products, two minima, a maximum and a copysign.
template <typename T>
__device__ __forceinline__ T limited_antiflux(T dh_prev, T dh, T dh_next,
                                             T second, const Antidiff<T>& ad) {
  if constexpr (sizeof(T) == 4) {
    // -A^ph (exactly, rounding is symmetric), so that -sigma infinity is a
    // copysign of it and A^ph a negated operand of the median
    const float naph = fma_t(-ad.c64, second, (-ad.c8) * dh);
    const float toward = __builtin_copysignf(__builtin_inff(), naph);
    const float bound = __builtin_amdgcn_fmed3f(dh_next, dh_prev, toward);
    return __builtin_amdgcn_fmed3f(0.0f, -naph, bound);
  } else {
    const T aph = fma_t(ad.c64, second, ad.c8 * dh);
    const T sg = copysign_t(T(1), aph);
    const T m = fmin_t(fmin_t(sg * dh_next, fabs_t(aph)), sg * dh_prev);
    return copysign_t(fmax_t(T(0), m), aph);
  }
}

// Update (eq. shasta-n): U^{n+1}_j = hat U_j - (A_j - A_{j-1}).
template <typename T>
__device__ __forceinline__ T update(T uhat, T a, T a_prev) {
  return uhat - (a - a_prev);
}

// Net flux through an outflow face in cell-sum units (only the transport
// and source parts are non-zero there): eps U + lambda f.
__device__ __forceinline__ double face_flux(double eps, double u, double lam,
                                            double f) {
  return __builtin_fma(eps, u, lam * f);
}

}  // namespace shasta
