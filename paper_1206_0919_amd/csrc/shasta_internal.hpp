// Layouts shared by the host library and the kernels of the relativistic
// SHASTA step.  Everything here is plain data; no arithmetic of the method.
#pragma once
#include <stdint.h>

namespace shasta {

constexpr int kNF = 5;            // E, M_x, M_y, M_z, R
constexpr int kWavesPerBlock = 4; // 256-thread blocks, each wave independent
#ifndef SHASTA_XCELLS
#define SHASTA_XCELLS 2
#endif
constexpr int kXCells = SHASTA_XCELLS;  // x sweep: consecutive positions per lane
constexpr int kXWindow = 64 * kXCells;  // positions held by one wave
constexpr int kHalo = 6;          // halo of a row piece (two half steps of 3)
constexpr int kMarchLag = 6;      // y/z sweep: output lags input by 6 cells

// One reduction record per block of every sweep (doubles).
enum : int {
  R_SUM = 0,      // 5 sums of the written cells
  R_LEDGER = 5,   // 5 net boundary outflows of the sweep
  R_MAXEPS = 10,  // largest |lambda v| of the corrector
  R_CLAMP = 11,   // recoveries with |M| clamped
  R_FLOOR = 12,   // recoveries with E floored
  R_NOCONV = 13,  // recoveries whose iterative root solve did not converge
  R_USED = 14,    // entries of a record that are written
  R_SIZE = 16
};

// Per-event accumulator (doubles), updated once per step.
enum : int {
  A_SUM = 0,
  A_LEDGER = 5,
  A_MAXEPS = 10,
  A_T = 11,
  A_CLAMP = 12,
  A_FLOOR = 13,
  A_NOCONV = 14,
  A_NONFINITE = 15,
  A_STEPS = 16,
  A_INVALID = 17,  // cells rejected by write_primitive
  A_SIZE = 32
};

struct EventDesc {
  int32_t n[3];        // nx, ny, nz
  int32_t pad0;
  int64_t ncell;
  int64_t off[2];      // element offset of field 0 of buffer 0/1; field q
                       // lives at off[b] + q * pitch
  int64_t pitch;       // elements between consecutive fields
  int32_t rec_begin[3];  // first reduction record of this event, per axis
  int32_t rec_count[3];
  int32_t xwin_begin;    // first x-sweep window of this event
  int32_t xwin_count;
  int32_t fin_begin;     // first partial of the step reduction of this event
  int32_t fin_count;     // its partials (records of the three sweeps / kFinChunk)
};

// Step reduction: one block reduces kFinChunk records to one partial of
// R_SIZE doubles (the R_USED record entries, then the non-finite probe).
constexpr int kFinChunk = 256;

constexpr int kFlatLanes = 1;      // y/z: lane layout of flattened columns

// Work of one wave.
struct Item {
  int32_t ev;   // event index, -1 = padding (wave does nothing)
  int32_t a;    // x sweep: first window (index in the event's windows);
                //          y/z: x origin
  int32_t b;    // x sweep: windows to process; y/z: origin of the other
                //          transverse axis
  int32_t s0;   // y/z: written segment [s0, s1) along the sweep axis
  int32_t s1;
  int32_t lx;   // y/z: lanes along x (16, 32, 64), or kFlatLanes: the wave
                //      takes 64 consecutive columns of the transverse plane
                //      (x fastest) from column a on
  int32_t rec;  // reduction record of the item (records are contiguous per
                // event, whatever order the items are launched in)
  int32_t pad;
};

constexpr int kMaxEosNodes = 1024;   // tabled EOS: most nodes

// Bytes of the static device scratch of the step variant that allocates
// nothing (records, partials, counters and tickets of one handle's step).
constexpr unsigned long kStaticScratchBytes = 16ul << 20;

struct EosParams {
  int32_t kind;  // 0 ideal, 1 bag, 2 table, 3 baryon-dependent
  int32_t n;     // table: nodes m
  double B;      // bag: bag constant
  double e_H;    // bag: hadron edge of the mixed phase
  double cs2;    // baryon: p = cs2 max(0, e - mass n)
  double mass;   // baryon: rest mass per baryon
  // table: 4 m doubles in device memory: node e_k (m), node p_k (m), and the
  // slope a_k and intercept b_k of segment k = [e_k, e_k+1] (p = a e + b;
  // entry m-1 repeats segment m-2, which continues past the last node)
  const double* tab;
  int32_t newton_max;  // baryon: most iterations of the root solve
  int32_t pad;
};

// Kernel arguments of one sweep (built by the host library).
struct SweepArgs {
  const EventDesc* ev;
  const Item* items;
  int n_items;
  int parity;          // buffer holding U^n
  void* field_base;    // field arrays (T) start here
  double lam;          // dt / dx
  double diff;         // antidiffusion scale (1: phoenical)
  double* rec;         // reduction records of this sweep, one per block
  const int32_t* xwin; // x sweep: cell range [c0, c1) of every window (pairs)
  int* counter;        // persistent launch: next work item (null: one block
                       // or wave per item, no queue)
  const int* order;    // persistent launch: items in the order they are taken
  EosParams eos;
  int no_antiflux;     // 1: kernels without antidiffusion (diff = 0)
};

}  // namespace shasta
