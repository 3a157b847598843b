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
//  - x sweep (sweep_x): a lane owns kXCells (2) consecutive positions of a
//    window of 64 kXCells positions that holds row pieces with their halos;
//    neighbours come from the adjacent lane through cross-lane shuffles.
//
// Both organisations call the same arithmetic (shasta_math.hpp) with the
// same operands, so an x sweep and a y or z sweep of transposed data agree
// bit for bit.
#include <hip/hip_runtime.h>

#include <mutex>

#include "shasta_internal.hpp"
#include "shasta_math.hpp"
#include "shasta_sweeps.hpp"

namespace shasta {

// The sweep launchers are compiled in the translation units of their EOS.
SHASTA_SCHEMES_EOS0(extern)
SHASTA_SCHEMES_EOS1(extern)
SHASTA_SCHEMES_EOS2(extern)
SHASTA_SCHEMES_EOS3(extern)

// ------------------------------------------------------------ step reduction
// One block per event: sums of the last sweep, ledger and counters of the
// three sweeps of the step, in a fixed order; updates the accumulator.
struct FinalizeArgs {
  const EventDesc* ev;
  const double* rec[3];
  int axis[3];
  double* acc;     // A_SIZE doubles per event
  double dt;
  int* counters;   // queue counters of the three sweeps, reset for the next step
  double* partial; // R_SIZE doubles per partial
  int* ticket;     // one per event, zero between steps
};

// Entries of a step-reduction partial: the R_USED entries of a sweep record,
// then the non-finite probe.
constexpr int kFinN = R_USED + 1;
constexpr int kProbe = R_USED;

// Adds one record to the thread's partials.  The record entries are those of
// a sweep record; the probe collects x * 0 over the sums of every sweep, which
// stays 0 unless one of them is infinite or NaN.  Sums count only for the
// step's last sweep (the state at the end of the step).
__device__ __forceinline__ void fin_add(const double* r, bool last, double (&v)[kFinN]) {
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    if (last) v[R_SUM + q] += r[R_SUM + q];
    v[kProbe] += r[R_SUM + q] * 0.0;
    v[R_LEDGER + q] += r[R_LEDGER + q];
  }
  v[R_MAXEPS] = fmax(v[R_MAXEPS], r[R_MAXEPS]);
  v[R_CLAMP] += r[R_CLAMP];
  v[R_FLOOR] += r[R_FLOOR];
  v[R_NOCONV] += r[R_NOCONV];
}

// Fixed-order reduction of the block's 256 thread partials (butterfly per
// wave, then the four waves in order); the result is valid in thread 0.
__device__ __forceinline__ void fin_block(double (&v)[kFinN], double (*part)[kFinN]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kFinN; ++j) v[j] = (j == R_MAXEPS) ? wave_max(v[j]) : wave_sum(v[j]);
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < kFinN; ++j) part[wave][j] = v[j];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kFinChunk / 64; ++w)
#pragma unroll
      for (int j = 0; j < kFinN; ++j)
        v[j] = (j == R_MAXEPS) ? fmax(v[j], part[w][j]) : v[j] + part[w][j];
}

// Step reduction.  Block (c, e) reduces records [c * 256, c * 256 + 256) of
// event e (the records of the step's three sweeps, in sweep order) to
// partial c; the block that finishes last, found by a ticket per event,
// combines the partials in index order and updates the event's accumulators.
// The combination order is fixed, so the result does not depend on timing.
// The last block leaves the ticket at zero for the next step.
__global__ __launch_bounds__(kFinChunk) void finalize_step(FinalizeArgs F) {
  const EventDesc& ev = F.ev[blockIdx.y];
  const int c = blockIdx.x;
  __shared__ double part[kFinChunk / 64][kFinN];
  __shared__ int is_last;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 3) F.counters[threadIdx.x] = 0;
  if (c >= ev.fin_count) return;
  double v[kFinN];
#pragma unroll
  for (int j = 0; j < kFinN; ++j) v[j] = 0.0;
  {
    int i = c * kFinChunk + threadIdx.x;
    for (int s = 0; s < 3; ++s) {
      const int n = ev.rec_count[F.axis[s]];
      if (i >= 0 && i < n)
        fin_add(F.rec[s] + (size_t)(ev.rec_begin[F.axis[s]] + i) * R_SIZE, s == 2, v);
      i -= n;
    }
  }
  fin_block(v, part);
  double* mine = F.partial + (size_t)(ev.fin_begin + c) * R_SIZE;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < kFinN; ++j) mine[j] = v[j];
    __threadfence();
    is_last = atomicAdd(F.ticket + blockIdx.y, 1) == ev.fin_count - 1;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
#pragma unroll
  for (int j = 0; j < kFinN; ++j) v[j] = 0.0;
  for (int k = threadIdx.x; k < ev.fin_count; k += kFinChunk) {
    const double* p = F.partial + (size_t)(ev.fin_begin + k) * R_SIZE;
    double r[kFinN];
#pragma unroll
    for (int j = 0; j < kFinN; ++j) r[j] = __builtin_nontemporal_load(p + j);
#pragma unroll
    for (int j = 0; j < kFinN; ++j) v[j] = (j == R_MAXEPS) ? fmax(v[j], r[j]) : v[j] + r[j];
  }
  __syncthreads();  // part[] is reused
  fin_block(v, part);
  if (threadIdx.x == 0) {
    F.ticket[blockIdx.y] = 0;
    bool bad = !(v[kProbe] == 0.0);
    for (int q = 0; q < 5; ++q) bad = bad || !isfinite(v[R_SUM + q]);
    double* a = F.acc + (size_t)blockIdx.y * A_SIZE;
    for (int q = 0; q < 5; ++q) {
      a[A_SUM + q] = v[R_SUM + q];
      a[A_LEDGER + q] += v[R_LEDGER + q];
    }
    a[A_MAXEPS] = fmax(a[A_MAXEPS], v[R_MAXEPS]);
    a[A_T] += F.dt;
    a[A_CLAMP] += v[R_CLAMP];
    a[A_FLOOR] += v[R_FLOOR];
    a[A_NOCONV] += v[R_NOCONV];
    a[A_NONFINITE] += bad ? 1.0 : 0.0;
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
    } else if (eos.kind == 2) {
      p = table_pressure(eos, ei);
    } else if (eos.kind == 3) {
      p = eos.cs2 * fmax(ei - eos.mass * ni, 0.0);
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
    const Recovered r = (eos.kind == 0)   ? recover<0>(eos, E, Mx, My, Mz, R)
                        : (eos.kind == 1) ? recover<1>(eos, E, Mx, My, Mz, R)
                        : (eos.kind == 2) ? recover<2>(eos, E, Mx, My, Mz, R)
                                          : recover<3>(eos, E, Mx, My, Mz, R);
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

// Streaming copy for the bandwidth ceiling: block b copies the contiguous
// chunk [b C, (b + 1) C) of 16-byte elements, each lane keeping four
// independent loads in flight (elements i, i + 256, i + 512, i + 768 of the
// chunk).  On this GPU the contiguous chunks measured 5.3 TB/s against
// 4.5-5.2 TB/s for grid-stride loops (one to eight loads in flight,
// nontemporal or not) and 5.0 TB/s for a device-to-device hipMemcpy.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void stream_copy_kernel(const u32x4* __restrict__ s,
                                                          u32x4* __restrict__ d, int64_t n,
                                                          int64_t chunk) {
  const int64_t b0 = blockIdx.x * chunk;
  const int64_t b1 = (b0 + chunk < n) ? b0 + chunk : n;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 4 * 256) {
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (i + k * 256 < b1) v[k] = s[i + k * 256];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (i + k * 256 < b1) d[i + k * 256] = v[k];
  }
}

// Memory pattern of a y or z sweep without its arithmetic (calibration of
// what that pattern alone allows): one wave per segment of seg_len cells of
// 64 consecutive columns of the transverse plane (x fastest, the march's
// default lane layout), blocks mapped to XCDs as the march maps them.  The
// wave loads the five fields row by row along the axis, one row ahead, from
// kMarchLag cells before its segment to kMarchLag after it (clamped to the
// pencil, as the march's halo), and stores its segment's own rows, so dst
// becomes a copy of src.  Buffer loads and stores are range-checked.
template <typename T, int AXIS>
__global__ __launch_bounds__(64) void march_copy_kernel(const T* src, T* dst, int nx, int ny,
                                                        int nz, int64_t pitch, int seg_len,
                                                        int ngroups) {
  const int item = xcd_block();
  const int grp = item % ngroups, seg = item / ngroups;
  const int lane = threadIdx.x;
  const int N = (AXIS == 1) ? ny : nz;
  const int nb = (AXIS == 1) ? nz : ny;      // rows of the transverse plane
  const int ncol = nx * nb;
  const int g = grp * 64 + lane;
  const bool active = g < ncol;
  const int gc = min(g, ncol - 1);
  const int bb = gc / nx, x = gc - bb * nx;
  const int s_ax = (AXIS == 1) ? nx : nx * ny;
  const int s_b = (AXIS == 1) ? nx * ny : nx;
  const int off_col = (x + bb * s_b) * (int)sizeof(T);
  const int step = s_ax * (int)sizeof(T);
  const int64_t fbytes = (int64_t)nx * ny * nz * (int64_t)sizeof(T);
  __amdgpu_buffer_rsrc_t rs[kNF], rd[kNF];
#pragma unroll
  for (int q = 0; q < kNF; ++q) {
    rs[q] = field_rsrc(src + q * pitch, fbytes);
    rd[q] = field_rsrc(dst + q * pitch, fbytes);
  }
  const int s0 = seg * seg_len, s1 = min(N, s0 + seg_len);
  const int i_lo = s0 - kMarchLag, trips = s1 - s0 + 2 * kMarchLag;
  T v[2][kNF];
  auto load = [&](T (&r)[kNF], int i) {
    const int o = off_col + min(max(i, 0), N - 1) * step;
#pragma unroll
    for (int q = 0; q < kNF; ++q) r[q] = buf_load<T>(rs[q], o);
  };
  auto store = [&](const T (&r)[kNF], int i) {
    if (i < s0 || i >= s1) return;
    const int o = active ? off_col + i * step : kDropOffset;
#pragma unroll
    for (int q = 0; q < kNF; ++q) buf_store<T>(rd[q], o, r[q]);
  };
  load(v[0], i_lo);
  for (int t = 0; t < trips; t += 2) {
    const int i = i_lo + t;
    load(v[1], i + 1);
    store(v[0], i);
    load(v[0], i + 2);
    store(v[1], i + 1);
  }
}

// Recovery self-check: cell i of in = (E, M_x, M_y, M_z, R) -> out =
// (e, p, |v|, clamped + 2 floored + 4 not converged), through the same recover<EOS>() the
// sweeps call (|M|^2 summed as M_x^2 + (M_y^2 + M_z^2)).
template <int EOS>
__global__ void recover_selftest(EosParams eos, const double* in, double* out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* c = in + 5 * (size_t)i;
  const Recovered r = recover<EOS>(eos, c[0], c[1], c[2], c[3], c[4]);
  double* o = out + 4 * (size_t)i;
  o[0] = r.e;
  o[1] = r.p;
  o[2] = r.M2 > 0.0 ? r.w * sqrt(r.M2) : 0.0;   // any range of |M|^2, subnormal too
  o[3] = double(r.clamped + 2 * r.floored + 4 * r.noconv);
}

__global__ void selftest_kernel(const double* in, double* out, int n, int which) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (which == 0) ? rcp(in[i]) : sqrt_pos(in[i]);
}

}  // namespace shasta

// Scratch of the step variant that allocates nothing (shasta_step_noalloc):
// reduction records, step-reduction partials, queue counters and tickets.
// One copy per GPU, alive until the process ends; every call on a GPU shares
// it, so calls that overlap on one GPU race.  Host code never passes this
// name to a kernel or a copy: it is a host-side stand-in, not the device
// address, which static_scratch() looks up per device.
static __device__ __align__(256) unsigned char scratch[shasta::kStaticScratchBytes];

// Entry points used by the host library (C++ linkage, internal).
namespace shasta_launch {
using namespace shasta;

// Device address of this device's copy of the static scratch, looked up once
// per device (with that device current) and kept.
hipError_t static_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex lock;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(lock);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

template <int S>
hipError_t sweep_scheme(int fp32, int axis, const SweepArgs& a, int grid, bool p,
                        hipStream_t st) {
  if (fp32)
    return p ? launch_sweep<float, S, true>(axis, a, grid, st)
             : launch_sweep<float, S, false>(axis, a, grid, st);
  return p ? launch_sweep<double, S, true>(axis, a, grid, st)
           : launch_sweep<double, S, false>(axis, a, grid, st);
}

template <int S>
hipError_t sweep_scheme_grid(int fp32, int axis, const SweepArgs& a, int grid, hipStream_t st) {
  return fp32 ? launch_sweep<float, S, false>(axis, a, grid, st)
              : launch_sweep<double, S, false>(axis, a, grid, st);
}

hipError_t sweep(int fp32, int axis, const void* args, int grid, hipStream_t st) {
  const SweepArgs& a = *static_cast<const SweepArgs*>(args);
  const bool p = a.counter != nullptr;
  // The kernels without antiflux and those of the tabled and baryon EOS
  // exist for the grid launch only (the host never sets a queue for them).
  if (a.no_antiflux || a.eos.kind >= 2) {
    if (p) return hipErrorInvalidValue;
    constexpr int N = kNoAntiflux;
    const int scheme = a.eos.kind | (a.no_antiflux ? N : 0);
    switch (scheme) {
      case N | 0: return sweep_scheme_grid<N | 0>(fp32, axis, a, grid, st);
      case N | 1: return sweep_scheme_grid<N | 1>(fp32, axis, a, grid, st);
      case N | 2: return sweep_scheme_grid<N | 2>(fp32, axis, a, grid, st);
      case N | 3: return sweep_scheme_grid<N | 3>(fp32, axis, a, grid, st);
      case 2: return sweep_scheme_grid<2>(fp32, axis, a, grid, st);
      case 3: return sweep_scheme_grid<3>(fp32, axis, a, grid, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (a.eos.kind) {
    case 0: return sweep_scheme<0>(fp32, axis, a, grid, p, st);
    case 1: return sweep_scheme<1>(fp32, axis, a, grid, p, st);
    default: return hipErrorInvalidValue;
  }
}

int resident(int fp32, int eos_kind, int axis) {
  switch (eos_kind) {
    case 0: return fp32 ? resident_blocks<float, 0>(axis) : resident_blocks<double, 0>(axis);
    case 1: return fp32 ? resident_blocks<float, 1>(axis) : resident_blocks<double, 1>(axis);
    default: return 0;
  }
}

hipError_t finalize(const EventDesc* ev, int n_events, int max_chunks,
                    const double* const rec[3], const int axis[3], double* acc, double dt,
                    int* counters, double* partial, int* ticket, hipStream_t st) {
  FinalizeArgs f;
  f.counters = counters;
  f.partial = partial;
  f.ticket = ticket;
  f.ev = ev;
  for (int s = 0; s < 3; ++s) { f.rec[s] = rec[s]; f.axis[s] = axis[s]; }
  f.acc = acc;
  f.dt = dt;
  hipLaunchKernelGGL(finalize_step, dim3(max_chunks, n_events), dim3(kFinChunk), 0, st, f);
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
  int64_t b = (n + 4 * 256 - 1) / (4 * 256);   // at least four elements per lane
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  const int64_t chunk = (n + b - 1) / b;
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)b), dim3(256), 0, st,
                     (const u32x4*)s, (u32x4*)d, n, chunk);
  return hipGetLastError();
}

hipError_t march_copy(int fp32, const void* s, void* d, int nx, int ny, int nz, int64_t pitch,
                      int axis, int seg_len, hipStream_t st) {
  const int N = (axis == 1) ? ny : nz;
  const int nb = (axis == 1) ? nz : ny;
  const int64_t ngroups = ((int64_t)nx * nb + 63) / 64;
  const int64_t blocks = ngroups * ((N + seg_len - 1) / seg_len);
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  const dim3 g((unsigned)blocks), b(64);
  const int ng = (int)ngroups;
  if (fp32) {
    if (axis == 1)
      hipLaunchKernelGGL((march_copy_kernel<float, 1>), g, b, 0, st, (const float*)s,
                         (float*)d, nx, ny, nz, pitch, seg_len, ng);
    else
      hipLaunchKernelGGL((march_copy_kernel<float, 2>), g, b, 0, st, (const float*)s,
                         (float*)d, nx, ny, nz, pitch, seg_len, ng);
  } else {
    if (axis == 1)
      hipLaunchKernelGGL((march_copy_kernel<double, 1>), g, b, 0, st, (const double*)s,
                         (double*)d, nx, ny, nz, pitch, seg_len, ng);
    else
      hipLaunchKernelGGL((march_copy_kernel<double, 2>), g, b, 0, st, (const double*)s,
                         (double*)d, nx, ny, nz, pitch, seg_len, ng);
  }
  return hipGetLastError();
}

hipError_t selftest_recover(EosParams eos, const double* in, double* out, int n,
                            hipStream_t st) {
  const dim3 g((n + 127) / 128), b(128);
  switch (eos.kind) {
    case 0: hipLaunchKernelGGL(recover_selftest<0>, g, b, 0, st, eos, in, out, n); break;
    case 1: hipLaunchKernelGGL(recover_selftest<1>, g, b, 0, st, eos, in, out, n); break;
    case 2: hipLaunchKernelGGL(recover_selftest<2>, g, b, 0, st, eos, in, out, n); break;
    case 3: hipLaunchKernelGGL(recover_selftest<3>, g, b, 0, st, eos, in, out, n); break;
    default: return hipErrorInvalidValue;
  }
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
