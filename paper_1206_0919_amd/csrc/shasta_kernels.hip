// HIP kernels (gfx950) of the relativistic SHASTA step (arXiv:1206.0919).
//
// One kernel launch = one directional sweep of every event of the batch:
// halo (outflow copy), recovery at U^n, lambda/2 predictor, recovery at
// U^{n+1/2}, lambda corrector from U^n (Sec. 3, eqs. shasta-diff..shasta-n;
// Sec. 3.1 half-step method, halo cells; Listing 2 order).  Each sweep reads
// the five conserved fields once and writes them once; every intermediate
// stays in registers.
//
//  - y and z sweeps (sweep_march): a lane owns one column across the x axis
//    (lanes are consecutive in x, so every load and store is coalesced) and
//    marches along the sweep axis through a software pipeline.  Cell i of
//    U^n enters at iteration i; U^{n+1/2} of cell i-3 and U^{n+1} of cell i-6
//    leave in the same iteration, so each quantity is computed once.
//  - x sweep (sweep_x): a lane owns 4 consecutive cells of the x-fastest
//    array; a wave covers 256 cells of the flattened grid, neighbours come
//    from the adjacent lane through cross-lane shuffles, and the outflow halo
//    of each row is applied cell by cell (rows may start anywhere in a wave).
//
// Both organisations call the same arithmetic (shasta_math.hpp) with the
// same operands, so an x sweep and a y or z sweep of transposed data agree
// bit for bit.
#include <hip/hip_runtime.h>

#include "shasta_internal.hpp"
#include "shasta_math.hpp"

namespace shasta {

struct SweepArgs {
  const EventDesc* ev;
  const Item* items;
  int n_items;
  int parity;          // buffer holding U^n
  void* field_base;    // field arrays (T) start here
  double lam;          // dt / dx
  double diff;         // antidiffusion scale (1: phoenical)
  double* rec;         // reduction records of this sweep, one per block
  EosParams eos;
};

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// acc[0..4] sums, [5..9] ledger, [10] max eps, [11] clamp, [12] floor.
// Deterministic: fixed butterfly within the wave, fixed wave order.
__device__ __forceinline__ void block_record(double (&acc)[13], double* rec) {
  __shared__ double part[kWavesPerBlock][16];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < 13; ++j) {
    const double v = (j == R_MAXEPS) ? wave_max(acc[j]) : wave_sum(acc[j]);
    if (lane == 0) part[wave][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < 13) {
    const int j = threadIdx.x;
    double v = part[0][j];
#pragma unroll
    for (int w = 1; w < kWavesPerBlock; ++w)
      v = (j == R_MAXEPS) ? fmax(v, part[w][j]) : v + part[w][j];
    rec[(size_t)blockIdx.x * R_SIZE + j] = v;
  }
}

// ------------------------------------------------------------ march (y, z)
// Per-field pipeline state.  Index convention at iteration i (cell i of U^n
// just loaded): names give the cell they refer to.
template <typename T>
struct FieldPipe {
  T u1, u2, u3, u4;  // U^n at i-4, i-3, i-2, i-1
  T d1, d2, d3, d4;  // Delta = U_{j+1} - U_j at j = i-5, i-4, i-3, i-2
  T q1, q2, q3;      // second difference of Delta at i-6, i-5, i-4
  T hp1, hp2;        // predictor hat U at i-3, i-2
  T gp1, gp2;        // predictor hat Delta at i-4, i-3
  T ap1;             // predictor antiflux at i-4
  T hc1, hc2;        // corrector hat U at i-6, i-5
  T gc1, gc2;        // corrector hat Delta at i-7, i-6
  T ac1;             // corrector antiflux at i-7
};

template <typename T>
__device__ __forceinline__ void pipe_zero(FieldPipe<T>& f) {
  f.u1 = f.u2 = f.u3 = f.u4 = T(0);
  f.d1 = f.d2 = f.d3 = f.d4 = T(0);
  f.q1 = f.q2 = f.q3 = T(0);
  f.hp1 = f.hp2 = f.gp1 = f.gp2 = f.ap1 = T(0);
  f.hc1 = f.hc2 = f.gc1 = f.gc2 = f.ac1 = T(0);
}

// Predictor stage of one field; returns U^{n+1/2} at cell i-3.
template <typename T>
__device__ __forceinline__ T pipe_predict(FieldPipe<T>& f, T un,
                                          const Coef<T>& k, T src, T diff8,
                                          T& d_new, T& hp_new, T& gp_new,
                                          T& q_new, T& ap_new) {
  d_new = un - f.u4;                                    // Delta_{i-1}
  hp_new = transport(k, src, d_new, f.d4, f.u4);        // hat U_{i-1}
  gp_new = hp_new - f.hp2;                              // hat Delta_{i-2}
  q_new = second_difference(f.d4, f.d2, f.d3);          // at i-3
  ap_new = limited_antiflux(f.gp1, f.gp2, gp_new, q_new, diff8);  // A_{i-3}
  return update(f.hp1, ap_new, f.ap1);                  // U^{n+1/2}_{i-3}
}

// Corrector stage of one field; returns U^{n+1} at cell i-6.
template <typename T>
__device__ __forceinline__ T pipe_correct(FieldPipe<T>& f, const Coef<T>& k,
                                          T src, T diff8, bool left_edge,
                                          T& hc_new, T& gc_new, T& ac_new) {
  hc_new = transport(k, src, f.d2, f.d1, f.u1);         // hat U_{i-4}
  if (left_edge) f.hc2 = hc_new;                        // halo: hat U_{-2} = hat U_{-1}
  gc_new = hc_new - f.hc2;                              // hat Delta_{i-5}
  ac_new = limited_antiflux(f.gc1, f.gc2, gc_new, f.q1, diff8);   // A_{i-6}
  return update(f.hc1, ac_new, f.ac1);                  // U^{n+1}_{i-6}
}

template <typename T>
__device__ __forceinline__ void pipe_shift(FieldPipe<T>& f, T un, T d_new,
                                           T hp_new, T gp_new, T q_new,
                                           T ap_new, T hc_new, T gc_new,
                                           T ac_new) {
  f.u1 = f.u2; f.u2 = f.u3; f.u3 = f.u4; f.u4 = un;
  f.d1 = f.d2; f.d2 = f.d3; f.d3 = f.d4; f.d4 = d_new;
  f.q1 = f.q2; f.q2 = f.q3; f.q3 = q_new;
  f.hp1 = f.hp2; f.hp2 = hp_new;
  f.gp1 = f.gp2; f.gp2 = gp_new;
  f.ap1 = ap_new;
  f.hc1 = f.hc2; f.hc2 = hc_new;
  f.gc1 = f.gc2; f.gc2 = gc_new;
  f.ac1 = ac_new;
}

// AXIS = 1 (y) or 2 (z).
template <typename T, int AXIS, int EOS>
__global__ __launch_bounds__(256) void sweep_march(SweepArgs A) {
  constexpr int QP = 1 + AXIS;                   // momentum along the sweep
  constexpr int QT1 = 1;                         // the transverse momenta
  constexpr int QT2 = (AXIS == 1) ? 3 : 2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int item_id = blockIdx.x * kWavesPerBlock + wave;
  double acc[13];
#pragma unroll
  for (int j = 0; j < 13; ++j) acc[j] = 0.0;

  const Item it = A.items[item_id];
  if (it.ev >= 0) {
    const EventDesc& ev = A.ev[it.ev];
    const int nx = ev.n[0], ny = ev.n[1];
    const int N = ev.n[AXIS];
    const int nb = (AXIS == 1) ? ev.n[2] : ev.n[1];
    const int64_t s_ax = (AXIS == 1) ? (int64_t)nx : (int64_t)nx * ny;
    const int64_t s_b = (AXIS == 1) ? (int64_t)nx * ny : (int64_t)nx;
    const int lx_bits = __builtin_ctz(it.lx);
    int x = it.a + (lane & (it.lx - 1));
    int bb = it.b + (lane >> lx_bits);
    const bool active = (x < nx) && (bb < nb);
    x = min(x, nx - 1);
    bb = min(bb, nb - 1);
    const int64_t col = (int64_t)x + (int64_t)bb * s_b;
    const T* src = reinterpret_cast<const T*>(A.field_base) + ev.off[A.parity] + col;
    T* dst = reinterpret_cast<T*>(A.field_base) + ev.off[A.parity ^ 1] + col;
    const int64_t pitch = ev.pitch;

    const double lam = A.lam;
    const double lamh = 0.5 * lam;
    const T lamsrc_p = T(-0.25 * lam);   // -lambda'/2 with lambda' = lambda/2
    const T lamsrc_c = T(-0.5 * lam);    // -lambda'/2 with lambda' = lambda
    const T diff8 = T(A.diff * 0.125);
    const bool seg_left = (it.s0 == 0), seg_right = (it.s1 == N);

    FieldPipe<T> F[kNF];
#pragma unroll
    for (int q = 0; q < kNF; ++q) pipe_zero(F[q]);
    // shared windows: predictor (time n) and corrector (time n+1/2)
    T ep1 = T(0), ep2 = T(0), rdp2 = T(1);   // eps at i-2, i-1; 1/D at (i-2,i-1)
    T fEp1 = T(0), fEp2 = T(0), fMp1 = T(0), fMp2 = T(0);
    T ec1 = T(0), ec2 = T(0), rdc2 = T(1);   // eps at i-5, i-4; 1/D at (i-5,i-4)
    T fEc1 = T(0), fEc2 = T(0), fMc1 = T(0), fMc2 = T(0);

    const int i_lo = it.s0 - kMarchLag, i_hi = it.s1 + kMarchLag;
    // prefetch queue of two cells
    T qa[kNF], qb[kNF];
    {
      const int64_t o0 = (int64_t)min(max(i_lo, 0), N - 1) * s_ax;
      const int64_t o1 = (int64_t)min(max(i_lo + 1, 0), N - 1) * s_ax;
#pragma unroll
      for (int q = 0; q < kNF; ++q) {
        qa[q] = src[q * pitch + o0];
        qb[q] = src[q * pitch + o1];
      }
    }
    for (int i = i_lo; i < i_hi; ++i) {
      T un[kNF];
#pragma unroll
      for (int q = 0; q < kNF; ++q) { un[q] = qa[q]; qa[q] = qb[q]; }
      {
        const int64_t o2 = (int64_t)min(max(i + 2, 0), N - 1) * s_ax;
#pragma unroll
        for (int q = 0; q < kNF; ++q) qb[q] = src[q * pitch + o2];
      }
      // ---- recovery at U^n of cell i
      const Recovered rn = recover<EOS>(A.eos, double(un[0]), double(un[QP]),
                                   double(un[QT1]), double(un[QT2]));
      const double vn = rn.w * double(un[QP]);
      const T ep_i = T(lamh * vn);
      const T fE_i = T(rn.p * vn);
      const T fM_i = T(rn.p);
      if (active && i >= it.s0 && i < it.s1) {
        acc[R_CLAMP] += rn.clamped;
        acc[R_FLOOR] += rn.floored;
      }
      // ---- predictor coefficients of cell i-1
      const T rdp_new = interface_rcp(ep2, ep_i);
      const Coef<T> kp = coefficients(ep2, rdp2, rdp_new);
      const T sEp = source(lamsrc_p, fEp1, fE_i);
      const T sMp = source(lamsrc_p, fMp1, fM_i);
      // ---- predictor of every field: U^{n+1/2} at cell k = i-3
      T uh[kNF], d_new[kNF], hp_new[kNF], gp_new[kNF], q_new[kNF], ap_new[kNF];
#pragma unroll
      for (int q = 0; q < kNF; ++q) {
        const T s = (q == 0) ? sEp : ((q == QP) ? sMp : T(0));
        uh[q] = pipe_predict(F[q], un[q], kp, s, diff8, d_new[q], hp_new[q],
                             gp_new[q], q_new[q], ap_new[q]);
      }
      // ---- recovery at U^{n+1/2} of cell k (halo cells copy the edge cell)
      const int k = i - 3;
      T ec_k, fEc_k, fMc_k;
      if (k < 0) {
        ec_k = T(0); fEc_k = T(0); fMc_k = T(0);      // replaced at k = 0
      } else if (k >= N) {
        ec_k = ec2; fEc_k = fEc2; fMc_k = fMc2;        // copy of cell N-1
      } else {
        const Recovered rh = recover<EOS>(A.eos, double(uh[0]), double(uh[QP]),
                                     double(uh[QT1]), double(uh[QT2]));
        const double vh = rh.w * double(uh[QP]);
        ec_k = T(lam * vh);
        fEc_k = T(rh.p * vh);
        fMc_k = T(rh.p);
        if (active && k >= it.s0 && k < it.s1) {
          acc[R_CLAMP] += rh.clamped;
          acc[R_FLOOR] += rh.floored;
          acc[R_MAXEPS] = fmax(acc[R_MAXEPS], fabs(double(ec_k)));
        }
      }
      const bool left_edge = (k == 0);
      if (left_edge) {
        ec1 = ec2 = ec_k; fEc1 = fEc2 = fEc_k; fMc1 = fMc2 = fMc_k;
        rdc2 = interface_rcp(ec1, ec2);
      }
      // ---- boundary ledger: flux through the outflow faces (corrector)
      if (active && ((left_edge && seg_left) || (k == N - 1 && seg_right))) {
        const double sg = left_edge ? -1.0 : 1.0;
        const double e64 = double(ec_k);
#pragma unroll
        for (int q = 0; q < kNF; ++q) {
          const double f = (q == 0) ? double(fEc_k) : ((q == QP) ? double(fMc_k) : 0.0);
          acc[R_LEDGER + q] += sg * face_flux(e64, double(F[q].u2), lam, f);
        }
        if (left_edge && k == N - 1) {   // single-cell pencil: both faces
#pragma unroll
          for (int q = 0; q < kNF; ++q) {
            const double f = (q == 0) ? double(fEc_k) : ((q == QP) ? double(fMc_k) : 0.0);
            acc[R_LEDGER + q] += face_flux(e64, double(F[q].u2), lam, f);
          }
        }
      }
      // ---- corrector coefficients of cell i-4
      const T rdc_new = interface_rcp(ec2, ec_k);
      const Coef<T> kc = coefficients(ec2, rdc2, rdc_new);
      const T sEc = source(lamsrc_c, fEc1, fEc_k);
      const T sMc = source(lamsrc_c, fMc1, fMc_k);
      // ---- corrector of every field: U^{n+1} at cell o = i-6
      const int o = i - kMarchLag;
      const bool store = active && (o >= it.s0);
#pragma unroll
      for (int q = 0; q < kNF; ++q) {
        const T s = (q == 0) ? sEc : ((q == QP) ? sMc : T(0));
        T hc_new, gc_new, ac_new;
        const T out = pipe_correct(F[q], kc, s, diff8, left_edge, hc_new,
                                   gc_new, ac_new);
        if (store) {
          dst[q * pitch + (int64_t)o * s_ax] = out;
          acc[R_SUM + q] += double(out);
        }
        pipe_shift(F[q], un[q], d_new[q], hp_new[q], gp_new[q], q_new[q],
                   ap_new[q], hc_new, gc_new, ac_new);
      }
      // ---- shift the shared windows
      ep1 = ep2; ep2 = ep_i; rdp2 = rdp_new;
      fEp1 = fEp2; fEp2 = fE_i; fMp1 = fMp2; fMp2 = fM_i;
      ec1 = ec2; ec2 = ec_k; rdc2 = rdc_new;
      fEc1 = fEc2; fEc2 = fEc_k; fMc1 = fMc2; fMc2 = fMc_k;
    }
  }
  block_record(acc, A.rec);
}

// ------------------------------------------------------------ x sweep
template <typename T>
__device__ __forceinline__ T from_left(T v) { return __shfl_up(v, 1, 64); }
template <typename T>
__device__ __forceinline__ T from_right(T v) { return __shfl_down(v, 1, 64); }

// Neighbours of the 4 owned cells: value of cell k-1 / k+1, where cell -1 is
// the left lane's cell 3 and cell 4 the right lane's cell 0; a cell at the
// start (end) of its row takes the halo value instead.
template <typename T>
__device__ __forceinline__ void neighbours(const T (&v)[kXCells],
                                           const bool (&isL)[kXCells],
                                           const bool (&isR)[kXCells],
                                           const T (&ghostL)[kXCells],
                                           const T (&ghostR)[kXCells],
                                           T (&left)[kXCells],
                                           T (&right)[kXCells]) {
  const T vl = from_left(v[kXCells - 1]);
  const T vr = from_right(v[0]);
#pragma unroll
  for (int k = 0; k < kXCells; ++k) {
    const T l = (k > 0) ? v[k - 1] : vl;
    const T r = (k < kXCells - 1) ? v[k + 1] : vr;
    left[k] = isL[k] ? ghostL[k] : l;
    right[k] = isR[k] ? ghostR[k] : r;
  }
}

// Same with the halo value equal to the cell's own value (outflow copy).
template <typename T>
__device__ __forceinline__ void neighbours_copy(const T (&v)[kXCells],
                                                const bool (&isL)[kXCells],
                                                const bool (&isR)[kXCells],
                                                T (&left)[kXCells],
                                                T (&right)[kXCells]) {
  neighbours(v, isL, isR, v, v, left, right);
}

// One 1-D SHASTA application to the 4 owned cells of one field along x.
// u, ul, ur: U and its neighbours (halo applied), dnext: Delta_{k+1};
// k/kg: coefficients of the cell and of its halo image; s/sg: sources.
template <typename T>
__device__ __forceinline__ void x_fct(const T (&u)[kXCells], const T (&ul)[kXCells],
                                      const T (&ur)[kXCells], const T (&dnext)[kXCells],
                                      const Coef<T> (&k)[kXCells],
                                      const Coef<T> (&kg)[kXCells],
                                      const T (&s)[kXCells], const T (&sg)[kXCells],
                                      const bool (&isL)[kXCells],
                                      const bool (&isR)[kXCells], T diff8,
                                      T (&out)[kXCells]) {
  T uh[kXCells], ug[kXCells], dh[kXCells], sec[kXCells];
#pragma unroll
  for (int j = 0; j < kXCells; ++j) {
    const T dr = ur[j] - u[j];      // Delta_j
    const T dl = u[j] - ul[j];      // Delta_{j-1}
    sec[j] = second_difference(dnext[j], dl, dr);
    uh[j] = transport(k[j], s[j], dr, dl, u[j]);
    // halo image of the transported value: all its inputs equal the edge
    // cell's, so Delta = 0 on both sides and the source vanishes
    const T z = u[j] - u[j];
    ug[j] = transport(kg[j], sg[j], z, z, u[j]);
  }
  // hat Delta_j = hat U_{j+1} - hat U_j
  T uhr[kXCells];
  {
    const T r = from_right(uh[0]);
#pragma unroll
    for (int j = 0; j < kXCells; ++j)
      uhr[j] = isR[j] ? ug[j] : ((j < kXCells - 1) ? uh[j + 1] : r);
  }
#pragma unroll
  for (int j = 0; j < kXCells; ++j) dh[j] = uhr[j] - uh[j];
  // hat Delta_{j-1}, hat Delta_{j+1}
  T dhl[kXCells], dhr[kXCells];
  {
    const T l = from_left(dh[kXCells - 1]);
    const T r = from_right(dh[0]);
#pragma unroll
    for (int j = 0; j < kXCells; ++j) {
      dhl[j] = isL[j] ? (uh[j] - ug[j]) : ((j > 0) ? dh[j - 1] : l);
      dhr[j] = isR[j] ? (ug[j] - ug[j]) : ((j < kXCells - 1) ? dh[j + 1] : r);
    }
  }
  T a[kXCells];
#pragma unroll
  for (int j = 0; j < kXCells; ++j)
    a[j] = limited_antiflux(dhl[j], dh[j], dhr[j], sec[j], diff8);
  {
    const T l = from_left(a[kXCells - 1]);
#pragma unroll
    for (int j = 0; j < kXCells; ++j) {
      const T al = isL[j] ? T(0) : ((j > 0) ? a[j - 1] : l);
      out[j] = update(uh[j], a[j], al);
    }
  }
}

// Coefficients and sources of one half step for the 4 owned cells.
template <typename T>
__device__ __forceinline__ void x_coefficients(const T (&eps)[kXCells],
                                               const T (&fE)[kXCells],
                                               const T (&fM)[kXCells],
                                               const bool (&isL)[kXCells],
                                               const bool (&isR)[kXCells],
                                               T lamsrc, Coef<T> (&k)[kXCells],
                                               Coef<T> (&kg)[kXCells],
                                               T (&sE)[kXCells], T (&sM)[kXCells],
                                               T (&sEg)[kXCells], T (&sMg)[kXCells]) {
  T el[kXCells], er[kXCells], fl[kXCells], fr[kXCells], gl[kXCells], gr[kXCells];
  neighbours_copy(eps, isL, isR, el, er);
  neighbours_copy(fE, isL, isR, fl, fr);
  neighbours_copy(fM, isL, isR, gl, gr);
  T rdr[kXCells];
#pragma unroll
  for (int j = 0; j < kXCells; ++j) rdr[j] = interface_rcp(eps[j], er[j]);
  const T rl_lane = from_left(rdr[kXCells - 1]);
#pragma unroll
  for (int j = 0; j < kXCells; ++j) {
    const T one = interface_rcp(eps[j], eps[j]);   // 1/D of a halo interface
    const T rdl = isL[j] ? one : ((j > 0) ? rdr[j - 1] : rl_lane);
    k[j] = coefficients(eps[j], rdl, rdr[j]);
    kg[j] = coefficients(eps[j], one, one);
    sE[j] = source(lamsrc, fl[j], fr[j]);
    sM[j] = source(lamsrc, gl[j], gr[j]);
    sEg[j] = source(lamsrc, fE[j], fE[j]);
    sMg[j] = source(lamsrc, fM[j], fM[j]);
  }
}

template <typename T, int EOS>
__global__ __launch_bounds__(256) void sweep_x(SweepArgs A) {
  constexpr int QP = 1, QT1 = 2, QT2 = 3;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int item_id = blockIdx.x * kWavesPerBlock + wave;
  double acc[13];
#pragma unroll
  for (int j = 0; j < 13; ++j) acc[j] = 0.0;

  const Item it = A.items[item_id];
  if (it.ev >= 0) {
    const EventDesc& ev = A.ev[it.ev];
    const int nx = ev.n[0];
    const int ncell = (int)ev.ncell;
    const T* src = reinterpret_cast<const T*>(A.field_base) + ev.off[A.parity];
    T* dst = reinterpret_cast<T*>(A.field_base) + ev.off[A.parity ^ 1];
    const int64_t pitch = ev.pitch;
    const double lam = A.lam;
    const double lamh = 0.5 * lam;
    const T lamsrc_p = T(-0.25 * lam);
    const T lamsrc_c = T(-0.5 * lam);
    const T diff8 = T(A.diff * 0.125);

    for (int w = 0; w < it.b; ++w) {
      const int c0 = it.a + w * kXOut;
      if (c0 >= ncell) break;
      const int c1 = min(c0 + kXOut, ncell);
      const int p0 = c0 - kXMargin + kXCells * lane;
      int pc[kXCells];
      bool isL[kXCells], isR[kXCells], own[kXCells];
      {
        int x = min(max(p0, 0), ncell - 1) % nx;
#pragma unroll
        for (int j = 0; j < kXCells; ++j) {
          const int p = p0 + j;
          pc[j] = min(max(p, 0), ncell - 1);
          if (j > 0) x = (x + 1 == nx) ? 0 : x + 1;
          isL[j] = (x == 0);
          isR[j] = (x == nx - 1);
          own[j] = (p >= c0) && (p < c1);
        }
      }
      T u[kNF][kXCells];
#pragma unroll
      for (int q = 0; q < kNF; ++q)
#pragma unroll
        for (int j = 0; j < kXCells; ++j) u[q][j] = src[q * pitch + pc[j]];

      // ---- recovery at U^n
      T ep[kXCells], fE[kXCells], fM[kXCells];
#pragma unroll
      for (int j = 0; j < kXCells; ++j) {
        const Recovered rn = recover<EOS>(A.eos, double(u[0][j]), double(u[QP][j]),
                                     double(u[QT1][j]), double(u[QT2][j]));
        const double v = rn.w * double(u[QP][j]);
        ep[j] = T(lamh * v);
        fE[j] = T(rn.p * v);
        fM[j] = T(rn.p);
        if (own[j]) {
          acc[R_CLAMP] += rn.clamped;
          acc[R_FLOOR] += rn.floored;
        }
      }
      // ---- U^n neighbours (kept for both half steps)
      T ul[kNF][kXCells], ur[kNF][kXCells], dn[kNF][kXCells];
#pragma unroll
      for (int q = 0; q < kNF; ++q) {
        neighbours_copy(u[q], isL, isR, ul[q], ur[q]);
        T dr[kXCells];
#pragma unroll
        for (int j = 0; j < kXCells; ++j) dr[j] = ur[q][j] - u[q][j];
        const T r = from_right(dr[0]);
#pragma unroll
        for (int j = 0; j < kXCells; ++j)
          dn[q][j] = isR[j] ? (u[q][j] - u[q][j]) : ((j < kXCells - 1) ? dr[j + 1] : r);
      }
      // ---- predictor (lambda/2)
      Coef<T> k[kXCells], kg[kXCells];
      T sE[kXCells], sM[kXCells], sEg[kXCells], sMg[kXCells];
      x_coefficients(ep, fE, fM, isL, isR, lamsrc_p, k, kg, sE, sM, sEg, sMg);
      T uh[kNF][kXCells];
#pragma unroll
      for (int q = 0; q < kNF; ++q) {
        T s[kXCells], sg[kXCells];
#pragma unroll
        for (int j = 0; j < kXCells; ++j) {
          s[j] = (q == 0) ? sE[j] : ((q == QP) ? sM[j] : T(0));
          sg[j] = (q == 0) ? sEg[j] : ((q == QP) ? sMg[j] : T(0));
        }
        x_fct(u[q], ul[q], ur[q], dn[q], k, kg, s, sg, isL, isR, diff8, uh[q]);
      }
      // ---- recovery at U^{n+1/2}
      T ec[kXCells], fEc[kXCells], fMc[kXCells];
#pragma unroll
      for (int j = 0; j < kXCells; ++j) {
        const Recovered rh = recover<EOS>(A.eos, double(uh[0][j]), double(uh[QP][j]),
                                     double(uh[QT1][j]), double(uh[QT2][j]));
        const double v = rh.w * double(uh[QP][j]);
        ec[j] = T(lam * v);
        fEc[j] = T(rh.p * v);
        fMc[j] = T(rh.p);
        if (own[j]) {
          acc[R_CLAMP] += rh.clamped;
          acc[R_FLOOR] += rh.floored;
          acc[R_MAXEPS] = fmax(acc[R_MAXEPS], fabs(double(ec[j])));
        }
      }
      // ---- corrector (lambda) from U^n
      x_coefficients(ec, fEc, fMc, isL, isR, lamsrc_c, k, kg, sE, sM, sEg, sMg);
#pragma unroll
      for (int q = 0; q < kNF; ++q) {
        T s[kXCells], sg[kXCells], out[kXCells];
#pragma unroll
        for (int j = 0; j < kXCells; ++j) {
          s[j] = (q == 0) ? sE[j] : ((q == QP) ? sM[j] : T(0));
          sg[j] = (q == 0) ? sEg[j] : ((q == QP) ? sMg[j] : T(0));
        }
        x_fct(u[q], ul[q], ur[q], dn[q], k, kg, s, sg, isL, isR, diff8, out);
#pragma unroll
        for (int j = 0; j < kXCells; ++j) {
          if (own[j]) {
            dst[q * pitch + pc[j]] = out[j];
            acc[R_SUM + q] += double(out[j]);
            const double f = (q == 0) ? double(fEc[j]) : ((q == QP) ? double(fMc[j]) : 0.0);
            const double F = face_flux(double(ec[j]), double(u[q][j]), lam, f);
            if (isR[j]) acc[R_LEDGER + q] += F;
            if (isL[j]) acc[R_LEDGER + q] -= F;
          }
        }
      }
    }
  }
  block_record(acc, A.rec);
}

// ------------------------------------------------------------ step reduction
// One block per event: sums of the last sweep, ledger and counters of the
// three sweeps of the step, in a fixed order; updates the accumulator.
struct FinalizeArgs {
  const EventDesc* ev;
  const double* rec[3];
  int axis[3];
  double* acc;     // A_SIZE doubles per event
  double dt;
};

__global__ __launch_bounds__(256) void finalize_step(FinalizeArgs F) {
  const EventDesc& ev = F.ev[blockIdx.x];
  __shared__ double red[256][13];
  double v[13];
#pragma unroll
  for (int j = 0; j < 13; ++j) v[j] = 0.0;
  double sums3[3][5];
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int q = 0; q < 5; ++q) sums3[s][q] = 0.0;
  for (int s = 0; s < 3; ++s) {
    const int ax = F.axis[s];
    const double* r = F.rec[s] + (size_t)ev.rec_begin[ax] * R_SIZE;
    for (int b = threadIdx.x; b < ev.rec_count[ax]; b += blockDim.x) {
      const double* rb = r + (size_t)b * R_SIZE;
      for (int q = 0; q < 5; ++q) {
        sums3[s][q] += rb[R_SUM + q];
        v[R_LEDGER + q] += rb[R_LEDGER + q];
      }
      v[R_MAXEPS] = fmax(v[R_MAXEPS], rb[R_MAXEPS]);
      v[R_CLAMP] += rb[R_CLAMP];
      v[R_FLOOR] += rb[R_FLOOR];
    }
  }
  // sums of the last sweep; a non-finite sum of any sweep flags the step
  bool bad = false;
  for (int s = 0; s < 3; ++s)
    for (int q = 0; q < 5; ++q) bad = bad || !isfinite(sums3[s][q]);
  for (int q = 0; q < 5; ++q) v[R_SUM + q] = sums3[2][q];
  for (int j = 0; j < 13; ++j) red[threadIdx.x][j] = v[j];
  __shared__ int any_bad;
  if (threadIdx.x == 0) any_bad = 0;
  __syncthreads();
  if (bad) atomicOr(&any_bad, 1);
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w)
      for (int j = 0; j < 13; ++j)
        red[threadIdx.x][j] = (j == R_MAXEPS)
                                  ? fmax(red[threadIdx.x][j], red[threadIdx.x + w][j])
                                  : red[threadIdx.x][j] + red[threadIdx.x + w][j];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* a = F.acc + (size_t)blockIdx.x * A_SIZE;
    for (int q = 0; q < 5; ++q) {
      a[A_SUM + q] = red[0][R_SUM + q];
      a[A_LEDGER + q] += red[0][R_LEDGER + q];
    }
    a[A_MAXEPS] = fmax(a[A_MAXEPS], red[0][R_MAXEPS]);
    a[A_T] += F.dt;
    a[A_CLAMP] += red[0][R_CLAMP];
    a[A_FLOOR] += red[0][R_FLOOR];
    a[A_NONFINITE] += any_bad ? 1.0 : 0.0;
    a[A_STEPS] += 1.0;
  }
}

// ------------------------------------------------------------ init, readout
template <typename T>
__global__ void prim_to_cons(EosParams eos, const double* e, const double* vx,
                             const double* vy, const double* vz, const double* n,
                             T* out, int64_t pitch, int64_t ncell, double* invalid) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ncell;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double ei = e[i], x = vx[i], y = vy[i], z = vz[i], ni = n[i];
    const double v2 = x * x + y * y + z * z;
    bad += !(ei >= 0.0) || !(v2 < 1.0) || !(ni >= 0.0) || !isfinite(ei) || !isfinite(ni);
    double p;
    if (eos.kind == 0) {
      p = ei * kThird;
    } else {
      const double eQ = eos.e_H + 4.0 * eos.B;
      p = (ei <= eos.e_H) ? ei * kThird
                          : ((ei < eQ) ? eos.e_H * kThird : (ei - 4.0 * eos.B) * kThird);
    }
    // eqs. cf-density, cf-momentum, cf-energy
    const double g2 = 1.0 / (1.0 - v2);
    const double wv = (ei + p) * g2;
    out[0 * pitch + i] = T((ei + p * v2) * g2);
    out[1 * pitch + i] = T(wv * x);
    out[2 * pitch + i] = T(wv * y);
    out[3 * pitch + i] = T(wv * z);
    out[4 * pitch + i] = T(ni * sqrt(g2));
  }
  if (bad) atomicAdd(invalid, double(bad));
}

template <typename T>
__global__ void cons_in(const double* E, const double* Mx, const double* My,
                        const double* Mz, const double* R, T* out, int64_t pitch,
                        int64_t ncell) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ncell;
       i += (int64_t)gridDim.x * blockDim.x) {
    out[0 * pitch + i] = T(E[i]);
    out[1 * pitch + i] = T(Mx[i]);
    out[2 * pitch + i] = T(My[i]);
    out[3 * pitch + i] = T(Mz[i]);
    out[4 * pitch + i] = T(R[i]);
  }
}

template <typename T>
__global__ void read_out(EosParams eos, const T* in, int64_t pitch, int64_t ncell,
                         int field, double* dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ncell;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (field < kNF) {
      dst[i] = double(in[field * pitch + i]);
      continue;
    }
    const double E = in[i], Mx = in[pitch + i], My = in[2 * pitch + i],
                 Mz = in[3 * pitch + i], R = in[4 * pitch + i];
    const Recovered r = (eos.kind == 0) ? recover<0>(eos, E, Mx, My, Mz)
                                        : recover<1>(eos, E, Mx, My, Mz);
    double out;
    switch (field) {
      case 5: out = r.e; break;
      case 6: out = r.p; break;
      case 7: out = r.w * Mx; break;
      case 8: out = r.w * My; break;
      case 9: out = r.w * Mz; break;
      default: {
        const double vx = r.w * Mx, vy = r.w * My, vz = r.w * Mz;
        out = R * sqrt(1.0 - (vx * vx + vy * vy + vz * vz));
      }
    }
    dst[i] = out;
  }
}

// Deterministic sums of the five fields of one event: fixed grid, fixed
// per-thread ranges, fixed tree; partial[b*5+q] per block, then one block
// combines them in order.
constexpr int kSumBlocks = 256;

template <typename T>
__global__ __launch_bounds__(256) void sum_fields(const T* in, int64_t pitch,
                                                  int64_t ncell, double* partial) {
  __shared__ double red[256][5];
  double v[5] = {0, 0, 0, 0, 0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ncell;
       i += (int64_t)gridDim.x * blockDim.x)
    for (int q = 0; q < 5; ++q) v[q] += double(in[q * pitch + i]);
  for (int q = 0; q < 5; ++q) red[threadIdx.x][q] = v[q];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 5; ++q) red[threadIdx.x][q] += red[threadIdx.x + w][q];
    __syncthreads();
  }
  if (threadIdx.x < 5) partial[blockIdx.x * 5 + threadIdx.x] = red[0][threadIdx.x];
}

__global__ void combine_sums(const double* partial, int nblocks, double* out) {
  if (threadIdx.x < 5) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[b * 5 + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

__global__ void zero_doubles(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void stream_copy_kernel(const float4* __restrict__ s, float4* __restrict__ d,
                                   int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

__global__ void selftest_kernel(const double* in, double* out, int n, int which) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (which == 0) ? rcp(in[i]) : sqrt_pos(in[i]);
}

// ------------------------------------------------------------ launchers
template <typename T, int EOS>
hipError_t launch_sweep(int axis, const SweepArgs& a, hipStream_t st) {
  const dim3 grid(a.n_items / kWavesPerBlock), block(64 * kWavesPerBlock);
  if (axis == 0)
    hipLaunchKernelGGL((sweep_x<T, EOS>), grid, block, 0, st, a);
  else if (axis == 1)
    hipLaunchKernelGGL((sweep_march<T, 1, EOS>), grid, block, 0, st, a);
  else
    hipLaunchKernelGGL((sweep_march<T, 2, EOS>), grid, block, 0, st, a);
  return hipGetLastError();
}

}  // namespace shasta

// Entry points used by the host library (C++ linkage, internal).
namespace shasta_launch {
using namespace shasta;

hipError_t sweep(int fp32, int axis, const void* args, hipStream_t st) {
  const SweepArgs& a = *static_cast<const SweepArgs*>(args);
  if (a.eos.kind == 0)
    return fp32 ? launch_sweep<float, 0>(axis, a, st) : launch_sweep<double, 0>(axis, a, st);
  return fp32 ? launch_sweep<float, 1>(axis, a, st) : launch_sweep<double, 1>(axis, a, st);
}

hipError_t finalize(const EventDesc* ev, int n_events, const double* const rec[3],
                    const int axis[3], double* acc, double dt, hipStream_t st) {
  FinalizeArgs f;
  f.ev = ev;
  for (int s = 0; s < 3; ++s) { f.rec[s] = rec[s]; f.axis[s] = axis[s]; }
  f.acc = acc;
  f.dt = dt;
  hipLaunchKernelGGL(finalize_step, dim3(n_events), dim3(256), 0, st, f);
  return hipGetLastError();
}

static dim3 grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

hipError_t write_prim(int fp32, EosParams eos, const double* e, const double* vx,
                      const double* vy, const double* vz, const double* n, void* out,
                      int64_t pitch, int64_t ncell, double* invalid, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(prim_to_cons<float>, grid_for(ncell), dim3(256), 0, st, eos, e,
                       vx, vy, vz, n, (float*)out, pitch, ncell, invalid);
  else
    hipLaunchKernelGGL(prim_to_cons<double>, grid_for(ncell), dim3(256), 0, st, eos, e,
                       vx, vy, vz, n, (double*)out, pitch, ncell, invalid);
  return hipGetLastError();
}

hipError_t write_cons(int fp32, const double* E, const double* Mx, const double* My,
                      const double* Mz, const double* R, void* out, int64_t pitch,
                      int64_t ncell, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(cons_in<float>, grid_for(ncell), dim3(256), 0, st, E, Mx, My, Mz,
                       R, (float*)out, pitch, ncell);
  else
    hipLaunchKernelGGL(cons_in<double>, grid_for(ncell), dim3(256), 0, st, E, Mx, My, Mz,
                       R, (double*)out, pitch, ncell);
  return hipGetLastError();
}

hipError_t read(int fp32, EosParams eos, const void* in, int64_t pitch, int64_t ncell,
                int field, double* dst, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(read_out<float>, grid_for(ncell), dim3(256), 0, st, eos,
                       (const float*)in, pitch, ncell, field, dst);
  else
    hipLaunchKernelGGL(read_out<double>, grid_for(ncell), dim3(256), 0, st, eos,
                       (const double*)in, pitch, ncell, field, dst);
  return hipGetLastError();
}

hipError_t zero(double* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_doubles, grid_for(n), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t copy(const void* s, void* d, size_t bytes, hipStream_t st) {
  const int64_t n = (int64_t)(bytes / 16);
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)b), dim3(256), 0, st,
                     (const float4*)s, (float4*)d, n);
  return hipGetLastError();
}

hipError_t selftest(const double* in, double* out, int n, int which, hipStream_t st) {
  hipLaunchKernelGGL(selftest_kernel, dim3((n + 255) / 256), dim3(256), 0, st, in, out,
                     n, which);
  return hipGetLastError();
}

hipError_t sums(int fp32, const void* in, int64_t pitch, int64_t ncell, double* scratch,
                double* out, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(sum_fields<float>, dim3(kSumBlocks), dim3(256), 0, st,
                       (const float*)in, pitch, ncell, scratch);
  else
    hipLaunchKernelGGL(sum_fields<double>, dim3(kSumBlocks), dim3(256), 0, st,
                       (const double*)in, pitch, ncell, scratch);
  hipLaunchKernelGGL(combine_sums, dim3(1), dim3(64), 0, st, scratch, kSumBlocks, out);
  return hipGetLastError();
}

int sum_scratch_doubles() { return kSumBlocks * 5; }

size_t sweep_args_size() { return sizeof(SweepArgs); }

}  // namespace shasta_launch
