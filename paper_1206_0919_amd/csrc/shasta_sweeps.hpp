// Sweep kernels of the relativistic SHASTA step and their launchers, as
// templates.  Each EOS instantiates them in a translation unit of its own
// (sweeps_eos*.hip); shasta_kernels.hip declares those instances extern.
//
// One kernel launch = one directional sweep of every event of the batch:
// halo (outflow copy), recovery at U^n, lambda/2 predictor, recovery at
// U^{n+1/2}, lambda corrector from U^n (Sec. 3, eqs. shasta-diff..shasta-n;
// Sec. 3.1 half-step method, halo cells; Listing 2 order).  Each sweep reads
// the five conserved fields once and writes them once; every intermediate
// stays on chip (registers and LDS).
//
//  - y and z sweeps (sweep_march): a lane owns one column of the transverse
//    plane (lanes are consecutive in x, so every load and store is
//    coalesced) and marches along the sweep axis through a software
//    pipeline split over a producer and a consumer wave.  Cell i of U^n
//    enters at iteration i; U^{n+1/2} of cell i-3 and U^{n+1} of cell i-6
//    leave in the same iteration, so each quantity is computed once.
//  - x sweep (sweep_x): a lane owns kXCells (2) consecutive positions of a
//    window of 64 kXCells positions that holds row pieces with their halos;
//    neighbours come from the adjacent lane through DPP wave shifts.
//
// Both organisations call the same arithmetic (shasta_math.hpp) with the
// same operands, so an x sweep and a y or z sweep of transposed data agree
// bit for bit.
#pragma once
#include <hip/hip_runtime.h>

#include "shasta_internal.hpp"
#include "shasta_math.hpp"

namespace shasta {

// The scheme a sweep kernel is compiled for: the EOS kind in the low bits,
// kNoAntiflux set for the kernels without the phoenical antiflux and its
// limiter (the transport step alone; the result equals diff = 0).
constexpr int kNoAntiflux = 16;
template <int SCHEME>
constexpr int eos_of = SCHEME & 15;
template <int SCHEME>
constexpr bool antiflux_of = (SCHEME & kNoAntiflux) == 0;

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// acc[0..4] sums, [5..9] ledger, [10] max eps, [11] clamp, [12] floor,
// [13] root solves not converged.  One record per work item (at the item's
// record index), written by lane 0: deterministic (fixed butterfly) and
// independent of which block or wave processed the item.
__device__ __forceinline__ void wave_record(const double (&acc)[R_USED], double* rec, int item) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < R_USED; ++j) {
    const double v = (j == R_MAXEPS) ? wave_max(acc[j]) : wave_sum(acc[j]);
    if (lane == 0) rec[(size_t)item * R_SIZE + j] = v;
  }
}

// Work queue of a persistent launch.  The first item of a block (or wave) is
// its index; the next ones come from an atomic counter in the order table.
__device__ __forceinline__ int item_at(const SweepArgs& A, int k) {
  return A.order ? A.order[k] : k;
}

// Block b of a launch runs on XCD b % 8.  Give each XCD a contiguous run of
// blocks, in dispatch order, so that neighbouring work items (which share
// cache lines of misaligned rows and the halo planes of adjacent segments)
// meet in the same L2.  Bijective on [0, gridDim.x).
__device__ __forceinline__ int xcd_block() {
  const int G = gridDim.x, b = blockIdx.x;
  const int q = G >> 3, r = G & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// ------------------------------------------------------------ march (y, z)
// Buffer descriptor of one field array (raw addressing, range checked by the
// hardware: loads beyond num_records return 0, stores beyond are dropped).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
// Byte offset that lies beyond every field array (each is below 2^31 bytes):
// a buffer store there is discarded by the range check, which masks stores
// lane by lane without a branch.
constexpr int kDropOffset = (int)0x80000000u;

template <typename T>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, int off, T v) {
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r, off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b32(
        __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0)), v), r, off, 0, 0);
}

// The march is split over a pair of waves that work on the same 64 columns:
//   producer P: loads U^n, recovery at U^n, lambda/2 predictor -> U^{n+1/2};
//   consumer C: recovery at U^{n+1/2}, lambda corrector from U^n -> U^{n+1},
//               stores, reductions.
// P hands U^n and U^{n+1/2} to C through LDS rings.  The pair meets at a
// barrier every S iterations and C runs S iterations behind P: at trip t P
// writes U^n slot t mod U and U^{n+1/2} slot t mod 2S while C reads U^n
// slot (t - S - 3) mod U and U^{n+1/2} slot (t - S) mod 2S, all written
// before the previous barrier and not rewritten before the next one (this
// needs U >= 2S + 3 ring slots for U^n).
// Each wave carries about half of the pipeline state.
//
// Every windowed quantity lives in a ring of 8 slots: the value of cell p is
// in slot (p - i_lo) & 7.  The loop body is instantiated for the 8 phases, so
// slot indices are compile-time constants and windows never move between
// registers.  At P's iteration i (cell i of U^n consumed): hat U of cell i-1,
// hat Delta of i-2, antiflux and U^{n+1/2} of cell i-3.  At C's iteration i
// (one loop trip later): recovery of U^{n+1/2} at i-3, hat U of cell i-4,
// hat Delta of i-5, antiflux and U^{n+1} of cell i-6.
// Configuration of the march per precision and EOS.  FP64 on the ideal gas
// runs three pairs per SIMD: 168 registers and 23 KB of LDS per pair, which
// needs a barrier every trip (S = 1) and one row of prefetch.  The others
// keep S = 2 and two rows of prefetch: FP32 fits three pairs anyway (four on
// the ideal gas and the bag model, with the producer's LDS re-reads), FP64
// on the bag, tabled and baryon EOS need more registers than three pairs
// allow.
template <typename T, int EOS>
struct MarchCfg {
  static constexpr bool tight = sizeof(T) == 8 && eos_of<EOS> == 0;
  static constexpr int sync = tight ? 1 : 2;        // trips between barriers
  static constexpr int prefetch = tight ? 1 : 2;    // rows P loads ahead
  static constexpr int waves = (sizeof(T) == 8 && eos_of<EOS> != 0) ? 2 : 3;  // per SIMD
  // U^n rows between P and C: at least 2S + 3; eight, so that with loop
  // chunks of 8 trips every slot index is a compile-time constant (the
  // run-time slot arithmetic made the march spill 28-41 scalar registers;
  // FP64 y/z sweeps 182-184 -> 178-181 us on 200^3).
  static constexpr int un_slots = 8;
  // C's boundary ledger: in LDS for FP64 (registers are the limit there), in
  // registers for FP32, whose 8-row ring would otherwise cost it a pair per CU
  static constexpr bool ledger_in_lds = sizeof(T) == 8;
  static_assert(sync == 1 || sync == 2, "the 8-phase loop body needs S in {1, 2}");
  static_assert(un_slots >= 2 * sync + 3, "ring too short for the lag between P and C");
  static_assert(prefetch >= 1 && prefetch <= 3, "register ring of 8: lifetime 4 + prefetch");
};

template <typename T, int S, int U>
struct RingLds {
  T un[U][kNF][64];          // U^n rows, slot = loop trip mod U
  T uh[2 * S][kNF][64];      // U^{n+1/2} rows, slot = loop trip mod 2S
  // C's per-lane FP64 accumulators of the written cells' sums and (FP64)
  // of the boundary ledger: kept in LDS, not in registers, through the whole
  // march (each lane adds only to its own entries, in program order).
  double sum[kNF][64];
  double ledger[sizeof(T) == 8 ? kNF : 1][64];
};

template <typename T, int AXIS, int EOS>
struct MarchCommon {
  static constexpr int QP = 1 + AXIS;            // momentum along the sweep
  static constexpr int QT1 = 1;                  // transverse momenta
  static constexpr int QT2 = (AXIS == 1) ? 3 : 2;
  int N, s0, s1, lane;
  bool active;
  const EosParams* eos;
  double lam, lamh;
  T lamsrc;
  Antidiff<T> ad;         // scales of the phoenical antiflux
  int n_clamp, n_floor;   // recoveries guarded, cells of the segment only
  int n_noconv;           // root solves not converged, cells of the segment only
  double maxeps;          // C only
};

template <typename T, int AXIS, int EOS>
struct MarchP : MarchCommon<T, AXIS, EOS> {
  using C = MarchCommon<T, AXIS, EOS>;
  // FP32: U^n rows i-2 .. i-4 are read back from the LDS ring (written by
  // this wave in earlier trips) and their differences taken again, instead
  // of holding a ring of Delta in registers: 135 -> 115 registers, four
  // pairs per SIMD.  FP64 keeps the register ring (the re-reads slowed the
  // FP64 march, which stays at three pairs per SIMD either way).
  static constexpr bool kReread = sizeof(T) == 4;
  T u[kNF][8], d[kNF][kReread ? 1 : 8], hp[kNF][8], gp[kNF][8], ap[kNF][8];
  T ep[8], fE[8], fM[8], rd[8];
  __amdgpu_buffer_rsrc_t src[kNF];
  int off_col, step_bytes;

  // Registers start at zero, and so do the U^n ring rows P reads back
  // before it has written them (rows before the segment's first trip), so
  // both forms see the same values there.
  template <class Ring>
  __device__ __forceinline__ void init(Ring& L) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      ep[j] = fE[j] = fM[j] = T(0);
      rd[j] = T(1);
#pragma unroll
      for (int q = 0; q < kNF; ++q) {
        u[q][j] = hp[q][j] = gp[q][j] = ap[q][j] = T(0);
        if constexpr (!kReread) d[q][j] = T(0);
      }
    }
    if constexpr (kReread) {
      constexpr int U = MarchCfg<T, EOS>::un_slots;
#pragma unroll
      for (int r = 0; r < U; ++r)
#pragma unroll
        for (int q = 0; q < kNF; ++q) L.un[r][q][this->lane] = T(0);
    }
  }
  template <int PH>
  __device__ __forceinline__ void load(int i) {
    const int o = off_col + min(max(i, 0), this->N - 1) * step_bytes;
#pragma unroll
    for (int q = 0; q < kNF; ++q) u[q][PH & 7] = buf_load<T>(src[q], o);
  }
  // EDGE = false: the caller guarantees that cell i is inside [s0, s1).
  template <int PH, bool EDGE, class Ring>
  __device__ __forceinline__ void iterate(int i, Ring& L, int hslot, int uslot) {
    constexpr int S0 = PH & 7, S1 = (PH - 1) & 7, S2 = (PH - 2) & 7, S3 = (PH - 3) & 7,
                  S4 = (PH - 4) & 7;
    constexpr int QP = C::QP, QT1 = C::QT1, QT2 = C::QT2;
    constexpr int PF = MarchCfg<T, EOS>::prefetch;
    load<PH + PF>(i + PF);  // prefetch
#pragma unroll
    for (int q = 0; q < kNF; ++q) L.un[uslot][q][this->lane] = u[q][S0];
    {
      const Recovered r = recover<eos_of<EOS>, sizeof(T) == 4>(*this->eos, double(u[0][S0]), double(u[QP][S0]),
                                       double(u[QT1][S0]), double(u[QT2][S0]),
                                       double(u[4][S0]));
      const double v = r.w * double(u[QP][S0]);
      ep[S0] = T(this->lamh * v);
      fE[S0] = T(r.p * v);
      fM[S0] = T(r.p);
      if (this->active && (!EDGE || (i >= this->s0 && i < this->s1))) {
        this->n_clamp += r.clamped;
        this->n_floor += r.floored;
        this->n_noconv += r.noconv;
      }
    }
    rd[S0] = interface_rcp(ep[S1], ep[S0]);
    const Coef<T> kp = coefficients(ep[S1], rd[S1], rd[S0]);
    const T sE = source(this->lamsrc, fE[S2], fE[S0]);
    const T sM = source(this->lamsrc, fM[S2], fM[S0]);
    constexpr int U = MarchCfg<T, EOS>::un_slots;
    const int r2 = (uslot + U - 2) % U, r3 = (uslot + U - 3) % U, r4 = (uslot + U - 4) % U;
#pragma unroll
    for (int q = 0; q < kNF; ++q) {
      const T s = (q == 0) ? sE : ((q == QP) ? sM : T(0));
      T d1, d2, d3, d4;                                   // Delta_{i-1} .. Delta_{i-4}
      if constexpr (kReread) {
        const T u2 = L.un[r2][q][this->lane], u3 = L.un[r3][q][this->lane],
                u4 = L.un[r4][q][this->lane];
        d1 = u[q][S0] - u[q][S1];
        d2 = u[q][S1] - u2;
        d3 = u2 - u3;
        d4 = u3 - u4;
      } else {
        d[q][S1] = u[q][S0] - u[q][S1];
        d1 = d[q][S1];
        d2 = d[q][S2];
        d3 = d[q][S3];
        d4 = d[q][S4];
      }
      hp[q][S1] = transport(kp, s, d1, d2, u[q][S1]);                    // hat U_{i-1}
      gp[q][S2] = hp[q][S1] - hp[q][S2];                                 // hat Delta_{i-2}
      const T sec = second_difference(d2, d4, d3);                       // at i-3
      if constexpr (antiflux_of<EOS>)
        ap[q][S3] = limited_antiflux(gp[q][S4], gp[q][S3], gp[q][S2], sec, this->ad);
      else
        ap[q][S3] = T(0);
      L.uh[hslot][q][this->lane] = update(hp[q][S3], ap[q][S3], ap[q][S4]);  // U^{n+1/2}_{i-3}
    }
  }
};

template <typename T, int AXIS, int EOS>
struct MarchC : MarchCommon<T, AXIS, EOS> {
  using C = MarchCommon<T, AXIS, EOS>;
  T u[kNF][8], d[kNF][8], q2[kNF][8], hc[kNF][8], gc[kNF][8], ac[kNF][8];
  T ec[8], fE[8], fM[8], rd[8];
  double led[kNF];   // boundary ledger when it is not kept in LDS
  __amdgpu_buffer_rsrc_t dst[kNF];
  int off_col, step_bytes;

  __device__ __forceinline__ void init() {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      ec[j] = fE[j] = fM[j] = T(0);
      rd[j] = T(1);
#pragma unroll
      for (int q = 0; q < kNF; ++q)
        u[q][j] = d[q][j] = q2[q][j] = hc[q][j] = gc[q][j] = ac[q][j] = T(0);
    }
  }
  // EDGE = false: the caller guarantees 1 <= k <= N-2, k and o inside
  // [s0, s1) (no pencil end, no halo rule, every result is stored).
  template <int PH, bool EDGE, class Ring>
  __device__ __forceinline__ void iterate(int i, Ring& L, int hslot, int uslot) {
    constexpr int S3 = (PH - 3) & 7, S4 = (PH - 4) & 7, S5 = (PH - 5) & 7, S6 = (PH - 6) & 7,
                  S7 = (PH - 7) & 7;
    constexpr int QP = C::QP, QT1 = C::QT1, QT2 = C::QT2;
    const int N = this->N;
    // ---- receive U^n and U^{n+1/2} of cell k = i-3
    T uh[kNF];
#pragma unroll
    for (int q = 0; q < kNF; ++q) {
      u[q][S3] = L.un[uslot][q][this->lane];
      uh[q] = L.uh[hslot][q][this->lane];
      d[q][S4] = u[q][S3] - u[q][S4];                                    // Delta_{i-4}
      q2[q][S5] = second_difference(d[q][S4], d[q][S6], d[q][S5]);      // at i-5
    }
    // ---- recovery at U^{n+1/2} of cell k (halo cells copy the edge cell)
    const int k = i - 3;
    if (EDGE && k < 0) {
      ec[S3] = T(0); fE[S3] = T(0); fM[S3] = T(0);      // replaced at k = 0
    } else if (EDGE && k >= N) {
      ec[S3] = ec[S4]; fE[S3] = fE[S4]; fM[S3] = fM[S4];
    } else {
      const Recovered r = recover<eos_of<EOS>, sizeof(T) == 4>(*this->eos, double(uh[0]), double(uh[QP]),
                                       double(uh[QT1]), double(uh[QT2]), double(uh[4]));
      const double v = r.w * double(uh[QP]);
      ec[S3] = T(this->lam * v);
      fE[S3] = T(r.p * v);
      fM[S3] = T(r.p);
      if (this->active && (!EDGE || (k >= this->s0 && k < this->s1))) {
        this->n_clamp += r.clamped;
        this->n_floor += r.floored;
        this->n_noconv += r.noconv;
        this->maxeps = fmax(this->maxeps, fabs(double(ec[S3])));
      }
    }
    const bool left_edge = EDGE && (k == 0);
    if (EDGE && left_edge) {
      ec[S4] = ec[S5] = ec[S3];
      fE[S4] = fE[S5] = fE[S3];
      fM[S4] = fM[S5] = fM[S3];
      rd[S4] = interface_rcp(ec[S5], ec[S4]);
    }
    // ---- boundary ledger: flux through the outflow faces (corrector)
    if (EDGE && this->active && ((left_edge && this->s0 == 0) || (k == N - 1 && this->s1 == N))) {
      const double e64 = double(ec[S3]);
#pragma unroll
      for (int q = 0; q < kNF; ++q) {
        const double f = (q == 0) ? double(fE[S3]) : ((q == QP) ? double(fM[S3]) : 0.0);
        const double F = face_flux(e64, double(u[q][S3]), this->lam, f);
        if constexpr (MarchCfg<T, EOS>::ledger_in_lds) {
          if (left_edge) L.ledger[q][this->lane] -= F;
          if (k == N - 1) L.ledger[q][this->lane] += F;
        } else {
          if (left_edge) led[q] -= F;
          if (k == N - 1) led[q] += F;
        }
      }
    }
    // ---- corrector of cell i-4 .. U^{n+1} of cell o = i-6
    rd[S3] = interface_rcp(ec[S4], ec[S3]);
    const Coef<T> kc = coefficients(ec[S4], rd[S4], rd[S3]);
    const T sE = source(this->lamsrc, fE[S5], fE[S3]);
    const T sM = source(this->lamsrc, fM[S5], fM[S3]);
    const int o = i - kMarchLag;
    const bool store = this->active && (!EDGE || (o >= this->s0 && o < this->s1));
    const int ooff = off_col + o * step_bytes;
#pragma unroll
    for (int q = 0; q < kNF; ++q) {
      const T s = (q == 0) ? sE : ((q == QP) ? sM : T(0));
      hc[q][S4] = transport(kc, s, d[q][S4], d[q][S5], u[q][S4]);       // hat U_{i-4}
      if (EDGE && left_edge) hc[q][S5] = hc[q][S4];                      // halo: hat U_{-2}
      gc[q][S5] = hc[q][S4] - hc[q][S5];                                 // hat Delta_{i-5}
      if constexpr (antiflux_of<EOS>)
        ac[q][S6] = limited_antiflux(gc[q][S7], gc[q][S6], gc[q][S5], q2[q][S6], this->ad);
      else
        ac[q][S6] = T(0);
      const T out = update(hc[q][S6], ac[q][S6], ac[q][S7]);            // U^{n+1}_{i-6}
      if (store) {
        buf_store<T>(dst[q], ooff, out);
        __hip_atomic_fetch_add(&L.sum[q][this->lane], double(out), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WAVEFRONT);
      }
    }
  }
};

template <typename M>
__device__ __forceinline__ void march_setup(M& m, const SweepArgs& A, const Item& it,
                                            const EventDesc& ev, int axis, int lane) {
  const int nx = ev.n[0], ny = ev.n[1];
  m.N = ev.n[axis];
  const int nb = (axis == 1) ? ev.n[2] : ev.n[1];
  const int s_ax = (axis == 1) ? nx : nx * ny;
  const int s_b = (axis == 1) ? nx * ny : nx;
  int x, bb;
  if (it.lx == kFlatLanes) {
    // 64 consecutive columns of the transverse plane, x fastest, from column
    // it.a on (a wave may cover the end of one row and the start of the next)
    const int g = it.a + lane;
    m.active = g < nx * nb;
    const int gc = min(g, nx * nb - 1);
    bb = gc / nx;
    x = gc - bb * nx;
  } else {
    const int lx_bits = __builtin_ctz(it.lx);
    x = it.a + (lane & (it.lx - 1));
    bb = it.b + (lane >> lx_bits);
    m.active = (x < nx) && (bb < nb);
    x = min(x, nx - 1);
    bb = min(bb, nb - 1);
  }
  m.lane = lane;
  using TT = decltype(m.lamsrc);
  m.off_col = (x + bb * s_b) * (int)sizeof(TT);
  m.step_bytes = s_ax * (int)sizeof(TT);
  m.eos = &A.eos;
  m.lam = A.lam;
  m.lamh = 0.5 * A.lam;
  m.ad = antidiff_scales<TT>(A.diff);
  m.s0 = it.s0;
  m.s1 = it.s1;
  m.n_clamp = 0;
  m.n_floor = 0;
  m.n_noconv = 0;
  m.maxeps = 0.0;
}

// AXIS = 1 (y) or 2 (z).  Block = one producer/consumer pair; it processes
// one work item, or, in a persistent launch, items from the queue until the
// queue is empty.
template <typename T, int AXIS, int EOS, bool PERSIST>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(MarchCfg<T, EOS>::waves)))
void sweep_march(SweepArgs A) {
  constexpr int kSync = MarchCfg<T, EOS>::sync;
  constexpr int kUnSlots = MarchCfg<T, EOS>::un_slots;
  constexpr int kPrefetch = MarchCfg<T, EOS>::prefetch;
  __shared__ RingLds<T, kSync, kUnSlots> L;
  __shared__ double part[16];
  __shared__ int next;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int k = PERSIST ? (int)blockIdx.x : xcd_block(); k < A.n_items;) {
  // wave-uniform: keeps the work item and the buffer descriptors scalar
  const int item = __builtin_amdgcn_readfirstlane(item_at(A, k));
  const Item it = A.items[item];
  double acc[R_USED];
#pragma unroll
  for (int j = 0; j < R_USED; ++j) acc[j] = 0.0;
  if (it.ev >= 0) {
    const EventDesc& ev = A.ev[it.ev];
    const int64_t fbytes = ev.ncell * (int64_t)sizeof(T);
    const T* base = reinterpret_cast<const T*>(A.field_base);
    const int i_lo = it.s0 - kMarchLag;
    const int trips = it.s1 - it.s0 + 2 * kMarchLag + kSync;   // C runs kSync trips behind
    const int N = ev.n[AXIS];
    // A chunk of 8 trips is "interior" when no trip of either wave meets a
    // pencil end, a halo rule or a cell outside the written segment.
    // P at trip t handles cell i = i_lo + t; C handles k = i_lo + t - kSync - 3
    // and o = i_lo + t - kSync - 6.
    auto interior = [&](int j) {
      const int iP0 = i_lo + j, iP1 = i_lo + j + 7;
      const int k0 = i_lo + j - kSync - 3, k1 = k0 + 7;
      const int o0 = i_lo + j - kSync - kMarchLag, o1 = o0 + 7;
      return j >= 1 && iP0 >= it.s0 && iP1 < it.s1 && k0 >= 1 &&
             k1 <= N - 2 && k0 >= it.s0 && k1 < it.s1 && o0 >= it.s0 && o1 < it.s1;
    };
    if (wave == 0) {
      MarchP<T, AXIS, EOS> P;
      march_setup(P, A, it, ev, AXIS, lane);
      P.lamsrc = T(-0.25 * A.lam);   // -lambda'/2 with lambda' = lambda/2
#pragma unroll
      for (int q = 0; q < kNF; ++q)
        P.src[q] = field_rsrc(base + ev.off[A.parity] + q * ev.pitch, fbytes);
      P.init(L);
      P.template load<0>(i_lo);
      if constexpr (kPrefetch >= 2) P.template load<1>(i_lo + 1);
      if constexpr (kPrefetch >= 3) P.template load<2>(i_lo + 2);
#define SHASTA_P(PH, E)                                                        \
  P.template iterate<PH, E>(i + PH, L, PH % (2 * kSync), (j + PH) % kUnSlots);  \
  if constexpr (PH % kSync == kSync - 1) __syncthreads();                      \
  else asm volatile("" ::: "memory");
#define SHASTA_P8(E)                                                           \
  {                                                                            \
    const int i = i_lo + j;                                                    \
    SHASTA_P(0, E) SHASTA_P(1, E) SHASTA_P(2, E) SHASTA_P(3, E)                \
    SHASTA_P(4, E) SHASTA_P(5, E) SHASTA_P(6, E) SHASTA_P(7, E)                \
  }
      int j = 0;
      for (; j < trips && !interior(j); j += 8) SHASTA_P8(true)
      for (; j < trips && interior(j); j += 8) SHASTA_P8(false)
      for (; j < trips; j += 8) SHASTA_P8(true)
#undef SHASTA_P8
#undef SHASTA_P
      acc[R_CLAMP] = P.active ? double(P.n_clamp) : 0.0;
      acc[R_FLOOR] = P.active ? double(P.n_floor) : 0.0;
      acc[R_NOCONV] = P.active ? double(P.n_noconv) : 0.0;
    } else {
      MarchC<T, AXIS, EOS> Cw;
      // FP64 ideal gas (a barrier every trip): the consumer issues ahead of
      // the other waves on its SIMD, since every trip ends at a barrier with
      // its producer and the consumer has the longer trip (y/z sweeps
      // 183-185 -> 174-177 us on 200^3).  With a barrier every two trips
      // (FP32, other EOS) the same priority slowed the sweeps (bag400 FP32
      // 976 -> 1045 us), so they keep the default.
      if constexpr (MarchCfg<T, EOS>::tight) __builtin_amdgcn_s_setprio(2);
      march_setup(Cw, A, it, ev, AXIS, lane);
      Cw.lamsrc = T(-0.5 * A.lam);   // -lambda'/2 with lambda' = lambda
#pragma unroll
      for (int q = 0; q < kNF; ++q)
        Cw.dst[q] = field_rsrc(base + ev.off[A.parity ^ 1] + q * ev.pitch, fbytes);
      Cw.init();
#pragma unroll
      for (int q = 0; q < kNF; ++q) {
        L.sum[q][lane] = 0.0;
        if constexpr (MarchCfg<T, EOS>::ledger_in_lds) L.ledger[q][lane] = 0.0;
        else Cw.led[q] = 0.0;
      }
      // C at trip t handles P's iteration of trip t - kSync (cell
      // i_lo + t - kSync).  Its first kSync trips read ring slots P has not
      // written yet: they produce values only for cells more than 5 cells
      // before the segment, which reach no stored cell, no counter and no
      // ledger entry.
#define SHASTA_C(PH, E)                                                            \
  Cw.template iterate<(PH + 8 - kSync) & 7, E>(                                    \
      i + PH, L, (PH + kSync) % (2 * kSync),                                       \
      (j + PH + 2 * kUnSlots - kSync - 3) % kUnSlots);                             \
  if constexpr (PH % kSync == kSync - 1) __syncthreads();                          \
  else asm volatile("" ::: "memory");
#define SHASTA_C8(E)                                                               \
  {                                                                                \
    const int i = i_lo + j - kSync;                                                \
    SHASTA_C(0, E) SHASTA_C(1, E) SHASTA_C(2, E) SHASTA_C(3, E)                    \
    SHASTA_C(4, E) SHASTA_C(5, E) SHASTA_C(6, E) SHASTA_C(7, E)                    \
  }
      int j = 0;
      for (; j < trips && !interior(j); j += 8) SHASTA_C8(true)
      for (; j < trips && interior(j); j += 8) SHASTA_C8(false)
      for (; j < trips; j += 8) SHASTA_C8(true)
#undef SHASTA_C8
#undef SHASTA_C
      if (Cw.active) {
#pragma unroll
        for (int q = 0; q < kNF; ++q) {
          acc[R_SUM + q] = L.sum[q][lane];
          if constexpr (MarchCfg<T, EOS>::ledger_in_lds) acc[R_LEDGER + q] = L.ledger[q][lane];
          else acc[R_LEDGER + q] = Cw.led[q];
        }
        acc[R_MAXEPS] = Cw.maxeps;
        acc[R_CLAMP] = double(Cw.n_clamp);
        acc[R_FLOOR] = double(Cw.n_floor);
        acc[R_NOCONV] = double(Cw.n_noconv);
      }
    }
  }
  // one record per item: consumer and producer parts summed in a fixed order
  {
    double v[R_USED];
#pragma unroll
    for (int j = 0; j < R_USED; ++j) v[j] = (j == R_MAXEPS) ? wave_max(acc[j]) : wave_sum(acc[j]);
    if (wave == 1 && lane == 0)
      for (int j = 0; j < R_USED; ++j) part[j] = v[j];
    __syncthreads();
    if (wave == 0 && lane == 0) {
      for (int j = 0; j < R_USED; ++j)
        A.rec[(size_t)it.rec * R_SIZE + j] = (j == R_MAXEPS) ? fmax(v[j], part[j]) : v[j] + part[j];
      if (PERSIST) next = atomicAdd(A.counter, 1) + (int)gridDim.x;
    }
    if (!PERSIST) break;
    __syncthreads();
    k = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
  }
  }
}

// ------------------------------------------------------------ x sweep
// A window holds up to 64 kXCells positions, kXCells consecutive ones per lane
// (two: 116 registers in FP64, four waves per SIMD).  It covers
// the cells [c0, c1) of the x-fastest array as row pieces, each preceded and
// followed by 6 halo positions whose loads are clamped to the row (outflow
// copy), exactly as the march treats the ends of a pencil.  The stencil then
// reads plain neighbours (lane-local or from the adjacent lane by a cross-lane
// shuffle); a position next to another row piece sees unrelated data, which
// reaches only halo positions (the step has a 6-cell domain of dependence).
// The only halo rule that is not a plain copy of U^n: at time n+1/2 a halo
// position takes the velocity and sources of its edge cell (read from LDS).
// Neighbour exchange by whole-wave DPP shifts: one VALU move per dword and
// no LDS round trip (against ds_bpermute: x sweep 193 -> 176 us in FP64,
// 302 -> 292 us in FP32).  DPP control 0x138 = wave_shr:1 (lane i takes
// lane i-1), 0x130 = wave_shl:1 (lane i takes lane i+1); the lane without a
// source (0, resp. 63) reads 0.  What lanes 0 and 63 receive from outside
// the wave reaches only the halo positions at the window's ends: a window
// edge is a row-piece edge, and the step's domain of dependence is 6 cells.
template <int CTRL>
__device__ __forceinline__ int dpp_shift(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)dpp_shift<CTRL>((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_shift<CTRL>((int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v) {
  return __builtin_bit_cast(float, dpp_shift<CTRL>(__builtin_bit_cast(int, v)));
}
template <typename T>
__device__ __forceinline__ T from_left(T v) { return dpp_shift<0x138>(v); }
template <typename T>
__device__ __forceinline__ T from_right(T v) { return dpp_shift<0x130>(v); }

template <typename T>
__device__ __forceinline__ void lr(const T (&v)[kXCells], T (&l)[kXCells], T (&r)[kXCells]) {
  const T vl = from_left(v[kXCells - 1]);
  const T vr = from_right(v[0]);
#pragma unroll
  for (int j = 0; j < kXCells; ++j) {
    l[j] = (j > 0) ? v[j - 1] : vl;
    r[j] = (j < kXCells - 1) ? v[j + 1] : vr;
  }
}

// Coefficients and sources of one half step for the 4 owned positions.
template <typename T>
__device__ __forceinline__ void x_coefficients(const T (&eps)[kXCells], const T (&fE)[kXCells],
                                               const T (&fM)[kXCells], T lamsrc,
                                               Coef<T> (&k)[kXCells], T (&sE)[kXCells],
                                               T (&sM)[kXCells]) {
  T el[kXCells], er[kXCells], fl[kXCells], fr[kXCells], gl[kXCells], gr[kXCells];
  lr(eps, el, er);
  lr(fE, fl, fr);
  lr(fM, gl, gr);
  T rdr[kXCells];
#pragma unroll
  for (int j = 0; j < kXCells; ++j) rdr[j] = interface_rcp(eps[j], er[j]);
  const T rl = from_left(rdr[kXCells - 1]);
#pragma unroll
  for (int j = 0; j < kXCells; ++j) {
    k[j] = coefficients(eps[j], (j > 0) ? rdr[j - 1] : rl, rdr[j]);
    sE[j] = source(lamsrc, fl[j], fr[j]);
    sM[j] = source(lamsrc, gl[j], gr[j]);
  }
}

// Differences of U^n around the owned positions p of one field: dl =
// Delta_{p-1}, dr = Delta_p = U_{p+1} - U_p, dn = Delta_{p+1}.  Each Delta is
// formed once, by the lane owning its left cell, and the neighbours' values
// arrive by DPP shifts (three per lane, as for the neighbouring U^n values).
template <typename T>
__device__ __forceinline__ void x_differences(const T (&u)[kXCells], T (&dl)[kXCells],
                                              T (&dr)[kXCells], T (&dn)[kXCells]) {
  const T next = from_right(u[0]);   // U^n of the first position of the next lane
#pragma unroll
  for (int j = 0; j < kXCells; ++j) dr[j] = ((j < kXCells - 1) ? u[j + 1] : next) - u[j];
  const T dl0 = from_left(dr[kXCells - 1]);
  const T dnl = from_right(dr[0]);
#pragma unroll
  for (int j = 0; j < kXCells; ++j) {
    dl[j] = (j > 0) ? dr[j - 1] : dl0;
    dn[j] = (j < kXCells - 1) ? dr[j + 1] : dnl;
  }
}

// One 1-D SHASTA application to the owned positions of one field.
// u: U^n; dl, dr, dn: its differences (x_differences).  AF = false:
// transport only.
template <bool AF, typename T>
__device__ __forceinline__ void x_fct(const T (&u)[kXCells], const T (&dl)[kXCells],
                                      const T (&dr)[kXCells], const T (&dn)[kXCells],
                                      const Coef<T> (&k)[kXCells], const T (&s)[kXCells],
                                      const Antidiff<T>& ad, T (&out)[kXCells]) {
  T uh[kXCells], sec[kXCells];
#pragma unroll
  for (int j = 0; j < kXCells; ++j) {
    sec[j] = second_difference(dn[j], dl[j], dr[j]);
    uh[j] = transport(k[j], s[j], dr[j], dl[j], u[j]);
  }
  if constexpr (!AF) {
#pragma unroll
    for (int j = 0; j < kXCells; ++j) out[j] = update(uh[j], T(0), T(0));
    return;
  }
  T dh[kXCells];
  {
    const T r = from_right(uh[0]);
#pragma unroll
    for (int j = 0; j < kXCells; ++j) dh[j] = ((j < kXCells - 1) ? uh[j + 1] : r) - uh[j];
  }
  T dhl[kXCells], dhr[kXCells];
  lr(dh, dhl, dhr);
  T a[kXCells];
#pragma unroll
  for (int j = 0; j < kXCells; ++j)
    a[j] = limited_antiflux(dhl[j], dh[j], dhr[j], sec[j], ad);
  const T al = from_left(a[kXCells - 1]);
#pragma unroll
  for (int j = 0; j < kXCells; ++j) out[j] = update(uh[j], a[j], (j > 0) ? a[j - 1] : al);
}

// FP32 grid launch: five waves per SIMD (96 registers, 2 % faster than four);
// the other forms spill at that limit and keep the compiler's choice.
template <typename T, int EOS, bool PERSIST>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && !PERSIST ? 5 : 1)))
void sweep_x(SweepArgs A) {
  constexpr int QP = 1, QT1 = 2, QT2 = 3;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __shared__ T halo[kWavesPerBlock][3][kXWindow];
  // per-lane sums of the written cells (0..4) and boundary ledger (5..9),
  // kept in LDS rather than registers through the item; each lane adds to
  // its own entries in program order
  __shared__ double xacc[kWavesPerBlock][10][64];
  double (*const acc10)[64] = xacc[wave];
  // wave-uniform: lets the compiler keep the work item in scalar registers
  for (int kq = __builtin_amdgcn_readfirstlane(
           (int)blockIdx.x * kWavesPerBlock + wave);
       kq < A.n_items;) {
  const int item = __builtin_amdgcn_readfirstlane(item_at(A, kq));
  const Item it = A.items[item];
#pragma unroll
  for (int j = 0; j < 10; ++j) acc10[j][lane] = 0.0;
  double maxeps = 0.0;
  int n_clamp = 0, n_floor = 0, n_noconv = 0;
  if (it.ev >= 0) {
    const EventDesc& ev = A.ev[it.ev];
    const int nx = ev.n[0];
    const T* src = reinterpret_cast<const T*>(A.field_base) + ev.off[A.parity];
    const int64_t pitch = ev.pitch;
    __amdgpu_buffer_rsrc_t dst[kNF];
#pragma unroll
    for (int q = 0; q < kNF; ++q)
      dst[q] = field_rsrc(reinterpret_cast<const T*>(A.field_base) + ev.off[A.parity ^ 1] +
                              q * pitch,
                          ev.ncell * (int64_t)sizeof(T));
    const int2* win = reinterpret_cast<const int2*>(A.xwin) + ev.xwin_begin;
    const double lam = A.lam;
    const double lamh = 0.5 * lam;
    const T lamsrc_p = T(-0.25 * lam);
    const T lamsrc_c = T(-0.5 * lam);
    const Antidiff<T> ad = antidiff_scales<T>(A.diff);
    T* hE = halo[wave][0];
    T* hF = halo[wave][1];
    T* hG = halo[wave][2];

    // ---- map the owned positions of window w to (cell, x) by walking its
    //      row pieces
    struct XMap {
      int cell[kXCells], xs[kXCells];
      bool used[kXCells], out_ok[kXCells];
    };
    auto map_window = [&](int w) {
      const int2 cw = win[w];
      const int c0 = cw.x, c1 = cw.y;
      XMap m;
#pragma unroll
      for (int j = 0; j < kXCells; ++j) {
        m.cell[j] = c0; m.xs[j] = 0; m.used[j] = false; m.out_ok[j] = false;
      }
      int ps = 0, c = c0;
      while (c < c1) {
        const int row0 = c - (c % nx);            // first cell of the row
        const int x0 = c - row0;
        const int len = min(nx - x0, c1 - c);
#pragma unroll
        for (int j = 0; j < kXCells; ++j) {
          const int r = kXCells * lane + j - ps;
          if (r >= 0 && r < len + 2 * kHalo) {
            const int x = x0 - kHalo + r;
            m.xs[j] = x;
            m.cell[j] = row0 + min(max(x, 0), nx - 1);
            m.used[j] = true;
            m.out_ok[j] = (r >= kHalo) && (r < kHalo + len);
          }
        }
        ps += len + 2 * kHalo;
        c += len;
      }
      return m;
    };
    auto load_window = [&](const XMap& m, T (&u)[kNF][kXCells]) {
#pragma unroll
      for (int q = 0; q < kNF; ++q)
#pragma unroll
        for (int j = 0; j < kXCells; ++j) u[q][j] = src[q * pitch + m.cell[j]];
    };
    for (int w = it.a; w < it.a + it.b; ++w) {
      const XMap m = map_window(w);
      T u[kNF][kXCells];
      // loads of the window issue ahead of the other waves' arithmetic
      __builtin_amdgcn_s_setprio(2);
      load_window(m, u);
      __builtin_amdgcn_s_setprio(0);
      const int (&cell)[kXCells] = m.cell;
      const int (&xs)[kXCells] = m.xs;
      const bool (&used)[kXCells] = m.used;
      const bool (&out_ok)[kXCells] = m.out_ok;

      // ---- recovery at U^n
      T ep[kXCells], fE[kXCells], fM[kXCells];
#pragma unroll
      for (int j = 0; j < kXCells; ++j) {
        const Recovered r = recover<eos_of<EOS>, sizeof(T) == 4>(A.eos, double(u[0][j]), double(u[QP][j]),
                                         double(u[QT1][j]), double(u[QT2][j]),
                                         double(u[4][j]));
        const double v = r.w * double(u[QP][j]);
        ep[j] = T(lamh * v);
        fE[j] = T(r.p * v);
        fM[j] = T(r.p);
        n_clamp += out_ok[j] & (r.clamped != 0);
        n_floor += out_ok[j] & (r.floored != 0);
        n_noconv += out_ok[j] & (r.noconv != 0);
      }
      // ---- the differences of U^n of field q are formed again for the
      //      corrector rather than kept in registers (x_differences)
      // ---- predictor (lambda/2)
      Coef<T> k[kXCells];
      T sE[kXCells], sM[kXCells];
      x_coefficients(ep, fE, fM, lamsrc_p, k, sE, sM);
      T uh[kNF][kXCells];
#pragma unroll
      for (int q = 0; q < kNF; ++q) {
        T dl[kXCells], dr[kXCells], dn[kXCells], s[kXCells];
        x_differences(u[q], dl, dr, dn);
#pragma unroll
        for (int j = 0; j < kXCells; ++j) s[j] = (q == 0) ? sE[j] : ((q == QP) ? sM[j] : T(0));
        x_fct<antiflux_of<EOS>>(u[q], dl, dr, dn, k, s, ad, uh[q]);
      }
      // ---- recovery at U^{n+1/2}; halo positions take their edge cell's
      //      values (through the wave's LDS table)
      T ec[kXCells], fEc[kXCells], fMc[kXCells];
#pragma unroll
      for (int j = 0; j < kXCells; ++j) {
        const Recovered r = recover<eos_of<EOS>, sizeof(T) == 4>(A.eos, double(uh[0][j]), double(uh[QP][j]),
                                         double(uh[QT1][j]), double(uh[QT2][j]),
                                         double(uh[4][j]));
        const double v = r.w * double(uh[QP][j]);
        ec[j] = T(lam * v);
        fEc[j] = T(r.p * v);
        fMc[j] = T(r.p);
        n_clamp += out_ok[j] & (r.clamped != 0);
        n_floor += out_ok[j] & (r.floored != 0);
        n_noconv += out_ok[j] & (r.noconv != 0);
        maxeps = out_ok[j] ? fmax(maxeps, fabs(double(ec[j]))) : maxeps;
        // table entry of position p at (p % kXCells) * 64 + p / kXCells:
        // a wave's writes and own-position reads touch distinct banks
        hE[j * 64 + lane] = ec[j];
        hF[j * 64 + lane] = fEc[j];
        hG[j * 64 + lane] = fMc[j];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int j = 0; j < kXCells; ++j) {
        // a halo position reads its edge cell's entry, every other one its own
        const bool ghost = used[j] && (xs[j] < 0 || xs[j] >= nx);
        const int pe = kXCells * lane + j + (ghost ? min(max(xs[j], 0), nx - 1) - xs[j] : 0);
        const int te = (pe % kXCells) * 64 + pe / kXCells;
        ec[j] = hE[te];
        fEc[j] = hF[te];
        fMc[j] = hG[te];
      }
      // the table is rewritten by the next window
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // ---- corrector (lambda) from U^n
      x_coefficients(ec, fEc, fMc, lamsrc_c, k, sE, sM);
#pragma unroll
      for (int q = 0; q < kNF; ++q) {
        T dl[kXCells], dr[kXCells], dn[kXCells], s[kXCells], out[kXCells];
        x_differences(u[q], dl, dr, dn);
#pragma unroll
        for (int j = 0; j < kXCells; ++j) s[j] = (q == 0) ? sE[j] : ((q == QP) ? sM[j] : T(0));
        x_fct<antiflux_of<EOS>>(u[q], dl, dr, dn, k, s, ad, out);
        double sum = acc10[R_SUM + q][lane];
#pragma unroll
        for (int j = 0; j < kXCells; ++j) {
          buf_store<T>(dst[q], out_ok[j] ? cell[j] * (int)sizeof(T) : kDropOffset, out[j]);
          sum += out_ok[j] ? double(out[j]) : 0.0;
        }
        acc10[R_SUM + q][lane] = sum;
      }
      // boundary ledger: flux through the outflow faces (corrector)
#pragma unroll
      for (int j = 0; j < kXCells; ++j) {
        const bool first = out_ok[j] && xs[j] == 0, last = out_ok[j] && xs[j] == nx - 1;
        if (any_lane(first || last)) {
#pragma unroll
          for (int q = 0; q < kNF; ++q) {
            const double f = (q == 0) ? double(fEc[j]) : ((q == QP) ? double(fMc[j]) : 0.0);
            const double F = face_flux(double(ec[j]), double(u[q][j]), lam, f);
            double l = acc10[R_LEDGER + q][lane];
            l = last ? l + F : l;
            l = first ? l - F : l;
            acc10[R_LEDGER + q][lane] = l;
          }
        }
      }
    }
  }
  double acc[R_USED];
#pragma unroll
  for (int j = 0; j < 10; ++j) acc[j] = acc10[j][lane];
  acc[R_MAXEPS] = maxeps;
  acc[R_CLAMP] = double(n_clamp);
  acc[R_FLOOR] = double(n_floor);
  acc[R_NOCONV] = double(n_noconv);
  wave_record(acc, A.rec, it.rec);
  if (!PERSIST) break;
  int nk = 0;
  if (lane == 0) nk = atomicAdd(A.counter, 1) + (int)gridDim.x * kWavesPerBlock;
  kq = __builtin_amdgcn_readfirstlane(__shfl(nk, 0, 64));
  }
}

// ------------------------------------------------------------ launchers
template <typename T, int EOS, bool P>
hipError_t launch_sweep(int axis, const SweepArgs& a, int grid, hipStream_t st) {
  if (axis == 0)
    hipLaunchKernelGGL((sweep_x<T, EOS, P>), dim3(grid), dim3(64 * kWavesPerBlock), 0, st, a);
  else if (axis == 1)
    hipLaunchKernelGGL((sweep_march<T, 1, EOS, P>), dim3(grid), dim3(128), 0, st, a);
  else
    hipLaunchKernelGGL((sweep_march<T, 2, EOS, P>), dim3(grid), dim3(128), 0, st, a);
  return hipGetLastError();
}

// Blocks of the persistent sweep kernel that fit on the whole GPU at once.
template <typename T, int EOS>
int resident_blocks(int axis) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  hipError_t e;
  if (axis == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, sweep_x<T, EOS, true>,
                                                     64 * kWavesPerBlock, 0);
  else if (axis == 1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, sweep_march<T, 1, EOS, true>, 128, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, sweep_march<T, 2, EOS, true>, 128, 0);
  if (e != hipSuccess) return 0;
  return per * cus;
}


// Explicit instances of the sweep launchers (PREFIX empty: definition in the
// translation unit of the EOS; PREFIX extern: declaration elsewhere).
#define SHASTA_SWEEP_INSTANCE(PREFIX, T, S, P) \
  PREFIX template hipError_t launch_sweep<T, S, P>(int, const SweepArgs&, int, hipStream_t);
#define SHASTA_SWEEP_SCHEME(PREFIX, S, P)     \
  SHASTA_SWEEP_INSTANCE(PREFIX, float, S, P)  \
  SHASTA_SWEEP_INSTANCE(PREFIX, double, S, P)
#define SHASTA_RESIDENT_INSTANCE(PREFIX, S)              \
  PREFIX template int resident_blocks<float, S>(int);    \
  PREFIX template int resident_blocks<double, S>(int);

// Schemes per EOS kind e: e with the persistent and the grid launch (kinds
// 0, 1) or the grid launch only (kinds 2, 3), and e | kNoAntiflux with the
// grid launch.
#define SHASTA_SCHEMES_EOS0(PREFIX)            \
  SHASTA_SWEEP_SCHEME(PREFIX, 0, true)         \
  SHASTA_SWEEP_SCHEME(PREFIX, 0, false)        \
  SHASTA_SWEEP_SCHEME(PREFIX, 16, false)       \
  SHASTA_RESIDENT_INSTANCE(PREFIX, 0)
#define SHASTA_SCHEMES_EOS1(PREFIX)            \
  SHASTA_SWEEP_SCHEME(PREFIX, 1, true)         \
  SHASTA_SWEEP_SCHEME(PREFIX, 1, false)        \
  SHASTA_SWEEP_SCHEME(PREFIX, 17, false)       \
  SHASTA_RESIDENT_INSTANCE(PREFIX, 1)
#define SHASTA_SCHEMES_EOS2(PREFIX)            \
  SHASTA_SWEEP_SCHEME(PREFIX, 2, false)        \
  SHASTA_SWEEP_SCHEME(PREFIX, 18, false)
#define SHASTA_SCHEMES_EOS3(PREFIX)            \
  SHASTA_SWEEP_SCHEME(PREFIX, 3, false)        \
  SHASTA_SWEEP_SCHEME(PREFIX, 19, false)

}  // namespace shasta
