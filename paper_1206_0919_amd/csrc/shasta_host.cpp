// Host side of the C ABI declared in include/shasta.h: argument validation,
// device workspace layout, work tables, the time-step schedule (axis
// permutation cycle of Listing 2, ping-pong buffers), HIP-graph replay,
// per-kernel event timing and the tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "shasta.h"
#include "shasta_internal.hpp"

using namespace shasta;

namespace shasta_launch {
hipError_t sweep(int fp32, int axis, const void* args, int grid, hipStream_t st);
int resident(int fp32, int eos_kind, int axis);
hipError_t finalize(const EventDesc* ev, int n_events, int max_chunks,
                    const double* const rec[3], const int axis[3], double* acc, double dt,
                    int* counters, double* partial, int* ticket, hipStream_t st);
hipError_t write_prim(int fp32, EosParams eos, const double* e, const double* vx,
                      const double* vy, const double* vz, const double* n, void* out,
                      int64_t pitch, int64_t ncell, double* invalid, hipStream_t st);
hipError_t write_cons(int fp32, const double* E, const double* Mx, const double* My,
                      const double* Mz, const double* R, void* out, int64_t pitch,
                      int64_t ncell, hipStream_t st);
hipError_t read(int fp32, EosParams eos, const void* in, int64_t pitch, int64_t ncell,
                int field, double* dst, hipStream_t st);
hipError_t zero(double* p, int64_t n, hipStream_t st);
hipError_t copy(const void* s, void* d, size_t bytes, hipStream_t st);
hipError_t march_copy(int fp32, const void* s, void* d, int nx, int ny, int nz, int64_t pitch,
                      int axis, int seg_len, hipStream_t st);
hipError_t selftest(const double* in, double* out, int n, int which, hipStream_t st);
hipError_t selftest_recover(EosParams eos, const double* in, double* out, int n,
                            hipStream_t st);
hipError_t sums(int fp32, const void* in, int64_t pitch, int64_t ncell, double* scratch,
                double* out, hipStream_t st);
int sum_scratch_doubles();
size_t sweep_args_size();
hipError_t static_scratch(void** ptr);
}  // namespace shasta_launch

namespace {

// Baryon-dependent EOS: iterations of the root solve, default and limit.
constexpr int kNewtonDefault = 16;
constexpr int kNewtonLimit = 64;

// Axis order of step k: the permutation table of Listing 2.
const int kBranch[18] = {0, 1, 2, 0, 2, 1, 2, 0, 1, 2, 1, 0, 1, 2, 0, 1, 0, 2};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct ProfRec {
  int cls;
  hipEvent_t a, b;
};

}  // namespace

struct shasta_handle {
  int n_events = 0;
  std::vector<int> dims;  // 3 per event
  double dx = 0.0;
  int precision = 0;
  int bc = 0;
  hipStream_t stream = nullptr;
  EosParams eos{0, 0, 0.0, 0.0, 0.0, 0.0, nullptr, kNewtonDefault, 0};
  std::vector<double> eos_tab;   // tabled EOS: the 4 m doubles of EosParams::tab
  double diff = 1.0;

  // decomposition (0 = automatic per event)
  bool persistent[3] = {false, false, false};
  int xwin = 0;
  int seg[3] = {0, 0, 0};
  int lanes[3] = {0, 0, 0};

  // tables
  std::vector<EventDesc> evd;
  std::vector<int2> xwins;          // x-sweep windows of all events
  std::vector<Item> items[3];
  std::vector<int> order[3];        // items by decreasing estimated cost
  int n_records[3] = {0, 0, 0};
  int64_t item_cap[3] = {0, 0, 0};
  int64_t rec_cap = 0;
  int fin_max = 0;          // most step-reduction partials of one event
  int64_t fin_cap = 0;      // partials the workspace holds

  // workspace layout
  size_t elem = 8;
  size_t field_bytes = 0, off_ev = 0, off_items[3] = {0, 0, 0}, off_rec = 0,
         off_acc = 0, off_scratch = 0, off_xwin = 0, off_cnt = 0, off_order[3] = {0, 0, 0},
         off_part = 0, off_eos = 0, total = 0;
  char* ws = nullptr;
  size_t ws_len = 0;

  std::vector<char> written;
  int64_t step_index = 0;
  int parity = 0;

  // graph
  bool graph_enabled = true;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double graph_dt = -1.0;
  int graph_parity = -1;
  int tables_version = 0, graph_version = -1;

  // profiling
  bool profiling = false;
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> event_pool;
  double prof_ms[4] = {0, 0, 0, 0};
  int64_t prof_n[4] = {0, 0, 0, 0};

  std::string err;
};

namespace {

int fail(shasta_t* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

int hipfail(shasta_t* h, hipError_t e, const char* where) {
  return fail(h, SHASTA_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHECK(h, call)                                 \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return hipfail((h), e_, #call); \
  } while (0)

int64_t ncell_of(const shasta_t* h, int ev) {
  return (int64_t)h->dims[3 * ev] * h->dims[3 * ev + 1] * h->dims[3 * ev + 2];
}

// Lane layout of a y/z sweep when none is set: flattened columns, which leave
// no lane idle but in the last wave of the plane.
int auto_lanes(int, int) { return kFlatLanes; }

int lanes_for(const shasta_t* h, int axis, int ev) {
  const int nx = h->dims[3 * ev];
  const int nb = (axis == 1) ? h->dims[3 * ev + 2] : h->dims[3 * ev + 1];
  return h->lanes[axis] ? h->lanes[axis] : auto_lanes(nx, nb);
}

int64_t columns(const shasta_t* h, int axis, int ev, int lx) {
  const int nx = h->dims[3 * ev];
  const int nb = (axis == 1) ? h->dims[3 * ev + 2] : h->dims[3 * ev + 1];
  if (lx == kFlatLanes) return ((int64_t)nx * nb + 63) / 64;
  const int lb = 64 / lx;
  return (int64_t)((nx + lx - 1) / lx) * ((nb + lb - 1) / lb);
}

// x-sweep windows of one event: consecutive cell ranges [c0, c1) whose row
// pieces, each with a halo of kHalo positions on both sides, fill at most
// kXWindow positions.
void build_xwindows(int nx, int64_t ncell, std::vector<int2>& out) {
  int64_t c = 0;
  while (c < ncell) {
    const int64_t c0 = c;
    int pos = 0;
    while (c < ncell) {
      const int64_t len = std::min<int64_t>(nx - c % nx, ncell - c);
      if (pos + len + 2 * kHalo <= kXWindow) {
        pos += (int)len + 2 * kHalo;
        c += len;
      } else {
        const int take = kXWindow - pos - 2 * kHalo;
        if (take >= 1) c += take;
        break;
      }
    }
    out.push_back(make_int2((int)c0, (int)c));
  }
}

// Build the per-axis work lists.  Every event's list is padded to a whole
// number of blocks so a block never mixes events.
void build_tables(shasta_t* h) {
  const int ne = h->n_events;
  // total waves of full pencils, used by the automatic segment length
  int64_t waves_full[3] = {0, 0, 0};
  for (int ax = 1; ax < 3; ++ax)
    for (int e = 0; e < ne; ++e) waves_full[ax] += columns(h, ax, e, lanes_for(h, ax, e));
  const int64_t target_waves = 2048;  // 2 waves on each of 1024 SIMDs
  for (int ax = 0; ax < 3; ++ax) h->items[ax].clear();
  const int64_t total_windows = (int64_t)h->xwins.size();
  const int auto_xwin = (int)std::max<int64_t>(1, total_windows / 8192);
  // x sweep: guided item sizes.  An item takes ceil(R / (2 * kGuideWaves))
  // windows (R = windows not yet assigned, over all events), capped by the
  // tuned size, so items shrink to single windows toward the end of the
  // launch; launched largest first, the last waves are short and the GPU
  // drains evenly.
  const int64_t kGuideWaves = 2048;   // two waves on each of 1024 SIMDs
  int64_t x_remaining = total_windows;
  for (int ax = 0; ax < 3; ++ax) {
    int rec = 0;
    for (int e = 0; e < ne; ++e) {
      EventDesc& d = h->evd[e];
      const size_t start = h->items[ax].size();
      if (ax == 0) {
        const int64_t nwin = d.xwin_count;
        const int cap = h->xwin ? h->xwin : auto_xwin;
        for (int64_t w = 0; w < nwin;) {
          const int64_t guided = (x_remaining + 2 * kGuideWaves - 1) / (2 * kGuideWaves);
          const int64_t take = std::min<int64_t>({(int64_t)cap, std::max<int64_t>(1, guided),
                                                  nwin - w});
          Item it{};
          it.ev = e;
          it.a = (int32_t)w;
          it.b = (int32_t)take;
          it.rec = rec + (int32_t)(h->items[ax].size() - start);
          h->items[ax].push_back(it);
          w += take;
          x_remaining -= take;
        }
      } else {
        const int N = h->dims[3 * e + ax];
        const int nx = h->dims[3 * e];
        const int nb = (ax == 1) ? h->dims[3 * e + 2] : h->dims[3 * e + 1];
        const int lx = lanes_for(h, ax, e);
        const int lb = (lx == kFlatLanes) ? 0 : 64 / lx;
        int L = h->seg[ax];
        if (L <= 0) {
          const int64_t nseg = std::max<int64_t>(
              1, (target_waves + waves_full[ax] - 1) / std::max<int64_t>(1, waves_full[ax]));
          L = (int)std::max<int64_t>(16, (N + nseg - 1) / nseg);
        }
        L = std::min(L, N);
        if (lx == kFlatLanes) {
          const int ncol = nx * nb;   // below 2^31: the event is
          for (int g0 = 0; g0 < ncol; g0 += 64)
            for (int s0 = 0; s0 < N; s0 += L) {
              Item it{};
              it.ev = e;
              it.a = g0;
              it.b = 0;
              it.s0 = s0;
              it.s1 = std::min(N, s0 + L);
              it.lx = kFlatLanes;
              it.rec = (int32_t)h->items[ax].size();
              h->items[ax].push_back(it);
            }
        } else
        for (int b0 = 0; b0 < nb; b0 += lb)
          for (int x0 = 0; x0 < nx; x0 += lx)
            for (int s0 = 0; s0 < N; s0 += L) {
              Item it{};
              it.ev = e;
              it.a = x0;
              it.b = b0;
              it.s0 = s0;
              it.s1 = std::min(N, s0 + L);
              it.lx = lx;
              it.rec = (int32_t)h->items[ax].size();
              h->items[ax].push_back(it);
            }
      }
      // one reduction record per item
      d.rec_begin[ax] = rec;
      d.rec_count[ax] = (int32_t)(h->items[ax].size() - start);
      rec += d.rec_count[ax];
    }
    h->n_records[ax] = rec;
    // x sweep: launch the largest items first (records stay per event)
    if (ax == 0)
      std::stable_sort(h->items[0].begin(), h->items[0].end(),
                       [](const Item& a, const Item& b) { return a.b > b.b; });
    // queue order of a persistent launch: largest estimated work first
    std::vector<double> cost(h->items[ax].size());
    for (size_t i = 0; i < cost.size(); ++i) {
      const Item& it = h->items[ax][i];
      cost[i] = (ax == 0) ? double(it.b) : double(it.s1 - it.s0 + 2 * kMarchLag);
    }
    h->order[ax].resize(cost.size());
    for (size_t i = 0; i < cost.size(); ++i) h->order[ax][i] = (int)i;
    std::stable_sort(h->order[ax].begin(), h->order[ax].end(),
                     [&](int a, int b) { return cost[a] > cost[b]; });
  }
  // step reduction: kFinChunk records of the three sweeps per partial
  int fin = 0;
  h->fin_max = 0;
  for (int e = 0; e < ne; ++e) {
    EventDesc& d = h->evd[e];
    const int n = d.rec_count[0] + d.rec_count[1] + d.rec_count[2];
    d.fin_begin = fin;
    d.fin_count = std::max(1, (n + kFinChunk - 1) / kFinChunk);
    fin += d.fin_count;
    h->fin_max = std::max(h->fin_max, d.fin_count);
  }
  h->tables_version++;
}

// Capacity of the tables over every decomposition the tuner may choose
// (smallest segment 16, one window per wave), so retuning never needs a
// larger workspace than the one computed at creation.
void table_capacity(const shasta_t* h, int64_t cap[3], int64_t& rec_cap) {
  rec_cap = 0;
  for (int ax = 0; ax < 3; ++ax) {
    int64_t n = 0;
    for (int e = 0; e < h->n_events; ++e) {
      int64_t m;
      if (ax == 0) {
        m = h->evd[e].xwin_count;
      } else {
        const int N = h->dims[3 * e + ax];
        int64_t worst = 0;
        for (int lx : {kFlatLanes, 16, 32, 64}) worst = std::max(worst, columns(h, ax, e, lx));
        m = worst * ((N + 15) / 16);
      }
      n += m;
    }
    cap[ax] = n;
    rec_cap = std::max(rec_cap, n);
  }
}

void layout(shasta_t* h) {
  h->elem = h->precision == SHASTA_FP32_MIXED ? 4 : 8;
  h->evd.assign(h->n_events, EventDesc{});
  int64_t off = 0;  // elements from the field base
  for (int e = 0; e < h->n_events; ++e) {
    EventDesc& d = h->evd[e];
    d.n[0] = h->dims[3 * e];
    d.n[1] = h->dims[3 * e + 1];
    d.n[2] = h->dims[3 * e + 2];
    d.ncell = ncell_of(h, e);
    d.pitch = (d.ncell + 63) / 64 * 64;  // 256/512-byte aligned field arrays
    d.off[0] = off;
    off += kNF * d.pitch;
    d.off[1] = off;
    off += kNF * d.pitch;
  }
  h->field_bytes = align256((size_t)off * h->elem);
  h->xwins.clear();
  for (int e = 0; e < h->n_events; ++e) {
    EventDesc& d = h->evd[e];
    d.xwin_begin = (int32_t)h->xwins.size();
    build_xwindows(d.n[0], d.ncell, h->xwins);
    d.xwin_count = (int32_t)(h->xwins.size() - d.xwin_begin);
  }
  table_capacity(h, h->item_cap, h->rec_cap);
  size_t p = h->field_bytes;
  h->off_ev = p;
  p = align256(p + sizeof(EventDesc) * h->n_events);
  for (int ax = 0; ax < 3; ++ax) {
    h->off_items[ax] = p;
    p = align256(p + sizeof(Item) * (size_t)h->item_cap[ax]);
  }
  h->off_rec = p;
  p = align256(p + 3 * sizeof(double) * R_SIZE * (size_t)h->rec_cap);
  h->off_acc = p;
  p = align256(p + sizeof(double) * A_SIZE * h->n_events);
  h->off_scratch = p;
  p = align256(p + sizeof(double) * shasta_launch::sum_scratch_doubles());
  h->off_xwin = p;
  p = align256(p + sizeof(int2) * h->xwins.size());
  h->off_cnt = p;  // 4 queue counters, then one reduction ticket per event
  p = align256(p + sizeof(int) * (4 + (size_t)h->n_events));
  h->fin_cap = (h->item_cap[0] + h->item_cap[1] + h->item_cap[2]) / kFinChunk + h->n_events;
  h->off_part = p;
  p = align256(p + sizeof(double) * R_SIZE * (size_t)h->fin_cap);
  h->off_eos = p;   // tabled EOS, largest table
  p = align256(p + sizeof(double) * 4 * (size_t)kMaxEosNodes);
  for (int ax = 0; ax < 3; ++ax) {
    h->off_order[ax] = p;
    p = align256(p + sizeof(int) * (size_t)h->item_cap[ax]);
  }
  h->total = p;
}

EventDesc* dev_events(shasta_t* h) { return reinterpret_cast<EventDesc*>(h->ws + h->off_ev); }
Item* dev_items(shasta_t* h, int ax) { return reinterpret_cast<Item*>(h->ws + h->off_items[ax]); }
double* dev_rec(shasta_t* h, int slot) {
  return reinterpret_cast<double*>(h->ws + h->off_rec) + (size_t)slot * R_SIZE * h->rec_cap;
}
double* dev_acc(shasta_t* h, int ev) {
  return reinterpret_cast<double*>(h->ws + h->off_acc) + (size_t)ev * A_SIZE;
}
char* dev_field(shasta_t* h, int ev, int buf) {
  return h->ws + (size_t)h->evd[ev].off[buf] * h->elem;
}

// Copy the tabled EOS into the workspace and point the EOS parameters at it
// (nothing to do for the analytic EOS or before a workspace is bound).
int upload_eos(shasta_t* h) {
  if (h->eos.kind != SHASTA_EOS_TABLE || !h->ws) return SHASTA_OK;
  double* dev = reinterpret_cast<double*>(h->ws + h->off_eos);
  HIPCHECK(h, hipMemcpyAsync(dev, h->eos_tab.data(), sizeof(double) * h->eos_tab.size(),
                             hipMemcpyHostToDevice, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  h->eos.tab = dev;
  return SHASTA_OK;
}

int upload_tables(shasta_t* h) {
  for (int ax = 0; ax < 3; ++ax)
    if ((int64_t)h->items[ax].size() > h->item_cap[ax])
      return fail(h, SHASTA_EWORKSPACE, "work table exceeds the workspace capacity");
  HIPCHECK(h, hipMemcpyAsync(dev_events(h), h->evd.data(), sizeof(EventDesc) * h->n_events,
                             hipMemcpyHostToDevice, h->stream));
  HIPCHECK(h, hipMemcpyAsync(h->ws + h->off_xwin, h->xwins.data(),
                             sizeof(int2) * h->xwins.size(), hipMemcpyHostToDevice, h->stream));
  for (int ax = 0; ax < 3; ++ax) {
    HIPCHECK(h, hipMemcpyAsync(dev_items(h, ax), h->items[ax].data(),
                               sizeof(Item) * h->items[ax].size(), hipMemcpyHostToDevice,
                               h->stream));
    HIPCHECK(h, hipMemcpyAsync(h->ws + h->off_order[ax], h->order[ax].data(),
                               sizeof(int) * h->order[ax].size(), hipMemcpyHostToDevice,
                               h->stream));
  }
  int64_t fin = 0;
  for (int e = 0; e < h->n_events; ++e) fin += h->evd[e].fin_count;
  if (fin > h->fin_cap)
    return fail(h, SHASTA_EWORKSPACE, "reduction partials exceed the workspace capacity");
  // queue counters and reduction tickets start at zero (then the step
  // reduction keeps them there between steps)
  HIPCHECK(h, shasta_launch::zero(reinterpret_cast<double*>(h->ws + h->off_cnt),
                                  (4 + h->n_events + 1) / 2, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  return SHASTA_OK;
}

void drop_graph(shasta_t* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
  h->graph_version = -1;
}

hipEvent_t take_event(shasta_t* h) {
  if (!h->event_pool.empty()) {
    hipEvent_t e = h->event_pool.back();
    h->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Device scratch of the step: reduction records of the three sweeps of a
// step, step-reduction partials, then the queue counters (4 ints) and one
// reduction ticket per event.  Counters and tickets are zero between steps.
struct StepScratch {
  double* rec[3];
  double* partial;
  int* cnt;
  bool may_allocate;   // per-kernel timing events may be created
};

StepScratch workspace_scratch(shasta_t* h) {
  StepScratch sc;
  for (int k = 0; k < 3; ++k) sc.rec[k] = dev_rec(h, k);
  sc.partial = reinterpret_cast<double*>(h->ws + h->off_part);
  sc.cnt = reinterpret_cast<int*>(h->ws + h->off_cnt);
  sc.may_allocate = true;
  return sc;
}

int launch_sweep(shasta_t* h, const StepScratch& sc, int axis, int parity, int slot, double lam,
                 hipStream_t st) {
  SweepArgs a;
  a.ev = dev_events(h);
  a.items = dev_items(h, axis);
  a.n_items = (int)h->items[axis].size();
  a.parity = parity;
  a.field_base = h->ws;
  a.lam = lam;
  a.diff = h->diff;
  a.rec = sc.rec[slot];
  a.xwin = reinterpret_cast<const int32_t*>(h->ws + h->off_xwin);
  a.eos = h->eos;
  a.counter = nullptr;
  a.order = nullptr;
  a.no_antiflux = h->diff == 0.0;
  if (a.n_items == 0) return SHASTA_OK;
  const int per_block = (axis == 0) ? kWavesPerBlock : 1;
  int grid = (a.n_items + per_block - 1) / per_block;
  // the kernels without antiflux and those of the tabled and baryon EOS
  // exist for the grid launch only
  if (h->persistent[axis] && !a.no_antiflux && h->eos.kind <= SHASTA_EOS_BAG) {
    const int res = shasta_launch::resident(h->precision == SHASTA_FP32_MIXED, h->eos.kind, axis);
    if (res > 0 && res < grid) {
      grid = res;
      a.counter = sc.cnt + slot;
      a.order = reinterpret_cast<const int*>(h->ws + h->off_order[axis]);
    }
  }
  const bool prof = h->profiling && st == h->stream && sc.may_allocate;
  ProfRec pr{axis, nullptr, nullptr};
  if (prof) {
    pr.a = take_event(h);
    pr.b = take_event(h);
    if (!pr.a || !pr.b) return fail(h, SHASTA_EHIP, "hipEventCreate failed");
    HIPCHECK(h, hipEventRecord(pr.a, st));
  }
  HIPCHECK(h, shasta_launch::sweep(h->precision == SHASTA_FP32_MIXED, axis, &a, grid, st));
  if (prof) {
    HIPCHECK(h, hipEventRecord(pr.b, st));
    h->prof.push_back(pr);
  }
  return SHASTA_OK;
}

// One time step (three sweeps and the step reduction) enqueued on st.
int enqueue_step(shasta_t* h, const StepScratch& sc, int64_t k, int& parity, double dt,
                 hipStream_t st) {
  const double lam = dt / h->dx;
  const int* perm = &kBranch[3 * (int)(k % 6)];
  for (int w = 0; w < 3; ++w) {
    int rc = launch_sweep(h, sc, perm[w], parity, w, lam, st);
    if (rc) return rc;
    parity ^= 1;
  }
  const double* rec[3] = {sc.rec[0], sc.rec[1], sc.rec[2]};
  const bool prof = h->profiling && st == h->stream && sc.may_allocate;
  ProfRec pr{3, nullptr, nullptr};
  if (prof) {
    pr.a = take_event(h);
    pr.b = take_event(h);
    if (!pr.a || !pr.b) return fail(h, SHASTA_EHIP, "hipEventCreate failed");
    HIPCHECK(h, hipEventRecord(pr.a, st));
  }
  HIPCHECK(h, shasta_launch::finalize(dev_events(h), h->n_events, h->fin_max, rec, perm,
                                      dev_acc(h, 0), dt, sc.cnt, sc.partial, sc.cnt + 4, st));
  if (prof) {
    HIPCHECK(h, hipEventRecord(pr.b, st));
    h->prof.push_back(pr);
  }
  return SHASTA_OK;
}

int capture_cycle(shasta_t* h, double dt) {
  drop_graph(h);
  if (!h->cap_stream)
    HIPCHECK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  HIPCHECK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  int parity = h->parity;
  int rc = SHASTA_OK;
  const StepScratch sc = workspace_scratch(h);
  for (int s = 0; s < 6 && rc == SHASTA_OK; ++s)
    rc = enqueue_step(h, sc, s, parity, dt, h->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hipfail(h, e, "hipStreamEndCapture");
  h->graph = g;
  HIPCHECK(h, hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0));
  h->graph_dt = dt;
  h->graph_parity = h->parity;
  h->graph_version = h->tables_version;
  return SHASTA_OK;
}

hipError_t reset_counters(shasta_t* h, hipStream_t st) {
  return shasta_launch::zero(reinterpret_cast<double*>(h->ws + h->off_cnt), 2, st);
}

int check_ready(shasta_t* h) {
  if (!h->ws) return fail(h, SHASTA_ESTATE, "no workspace bound");
  for (int e = 0; e < h->n_events; ++e)
    if (!h->written[e]) return fail(h, SHASTA_ESTATE, "event " + std::to_string(e) + " not written");
  return SHASTA_OK;
}

int check_event(shasta_t* h, int ev) {
  if (ev < 0 || ev >= h->n_events) return fail(h, SHASTA_EINVAL, "event index out of range");
  return SHASTA_OK;
}

// Status from an event's accumulators: non-finite values first, then root
// solves that did not converge, since the last write.
int health(shasta_t* h, const double* a) {
  if (a[A_NONFINITE] > 0) return fail(h, SHASTA_ENONFINITE, "non-finite values in the fields");
  if (a[A_NOCONV] > 0)
    return fail(h, SHASTA_ENOCONVERGE, std::to_string((long long)a[A_NOCONV]) +
                                           " recoveries stopped before their root converged");
  return SHASTA_OK;
}

int read_acc(shasta_t* h, int ev, double* a) {
  HIPCHECK(h, hipMemcpyAsync(a, dev_acc(h, ev), sizeof(double) * A_SIZE,
                             hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  return SHASTA_OK;
}

int refresh_sums(shasta_t* h, int ev) {
  const EventDesc& d = h->evd[ev];
  HIPCHECK(h, shasta_launch::sums(h->precision == SHASTA_FP32_MIXED, dev_field(h, ev, h->parity),
                                  d.pitch, d.ncell,
                                  reinterpret_cast<double*>(h->ws + h->off_scratch),
                                  dev_acc(h, ev) + A_SUM, h->stream));
  return SHASTA_OK;
}

// One axis' decomposition as the tuner handles it: x: windows per wave (p0);
// y/z: segment length (p0) and lanes along x (p1); persistent launch or not.
struct TuneChoice {
  int p0, p1;
  bool pers;
  float ms;
};

void set_choice(shasta_t* h, int ax, const TuneChoice& c) {
  if (ax == 0) {
    h->xwin = c.p0;
  } else {
    h->seg[ax] = c.p0;
    h->lanes[ax] = c.p1;
  }
  h->persistent[ax] = c.pers;
}

TuneChoice current_choice(const shasta_t* h, int ax) {
  return ax == 0 ? TuneChoice{h->xwin, 0, h->persistent[0], 0.0f}
                 : TuneChoice{h->seg[ax], h->lanes[ax], h->persistent[ax], 0.0f};
}

// Decompositions chosen by the tuner in this process, by device, precision,
// scheme (EOS kind, with or without antiflux) and the grids of the batch.
std::map<std::string, std::array<TuneChoice, 3>>& tune_cache() {
  static std::map<std::string, std::array<TuneChoice, 3>> cache;
  return cache;
}
std::mutex& tune_cache_lock() {
  static std::mutex m;
  return m;
}

int tune_key(shasta_t* h, std::string& key) {
  int dev = 0;
  HIPCHECK(h, hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHECK(h, hipGetDeviceProperties(&prop, dev));
  key = std::string(prop.gcnArchName) + "/" + std::to_string(prop.pciDomainID) + ":" +
        std::to_string(prop.pciBusID) + ":" + std::to_string(prop.pciDeviceID) + "/p" +
        std::to_string(h->precision) + "/e" + std::to_string(h->eos.kind) + "/a" +
        std::to_string(h->diff == 0.0 ? 0 : 1) + "/";
  for (int v : h->dims) key += std::to_string(v) + ",";
  return SHASTA_OK;
}

}  // namespace

extern "C" {

int shasta_create(shasta_t** out, int n_events, const int32_t* dims, double dx_fm,
                  int precision, int bc, void* hip_stream) {
  if (!out) return SHASTA_EINVAL;
  *out = nullptr;
  if (n_events < 1 || !dims) return SHASTA_EINVAL;
  if (!(dx_fm > 0.0) || !std::isfinite(dx_fm)) return SHASTA_EINVAL;
  if (precision != SHASTA_FP64 && precision != SHASTA_FP32_MIXED) return SHASTA_EINVAL;
  if (bc != SHASTA_BC_OUTFLOW) return SHASTA_EINVAL;
  for (int e = 0; e < n_events; ++e) {
    int64_t c = 1;
    for (int a = 0; a < 3; ++a) {
      if (dims[3 * e + a] < 1) return SHASTA_EINVAL;
      c *= dims[3 * e + a];
    }
    // one field array below 2^31 bytes: 32-bit buffer offsets and ranges
    const int64_t elem = precision == SHASTA_FP32_MIXED ? 4 : 8;
    if (c > (2147483647LL - 4096) / elem) return SHASTA_EINVAL;
  }
  shasta_t* h = new (std::nothrow) shasta_t();
  if (!h) return SHASTA_EINVAL;
  h->n_events = n_events;
  h->dims.assign(dims, dims + 3 * n_events);
  h->dx = dx_fm;
  h->precision = precision;
  h->bc = bc;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->written.assign(n_events, 0);
  layout(h);
  build_tables(h);
  *out = h;
  return SHASTA_OK;
}

int shasta_workspace_bytes(const shasta_t* h, size_t* bytes) {
  if (!h || !bytes) return SHASTA_EINVAL;
  *bytes = h->total;
  return SHASTA_OK;
}

int shasta_bind_workspace(shasta_t* h, void* dev_ptr, size_t bytes) {
  if (!h) return SHASTA_EINVAL;
  if (!dev_ptr) return fail(h, SHASTA_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256)
    return fail(h, SHASTA_EWORKSPACE, "workspace not 256-byte aligned");
  if (bytes < h->total)
    return fail(h, SHASTA_EWORKSPACE, "workspace too small: need " + std::to_string(h->total));
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, dev_ptr) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(h, SHASTA_EWORKSPACE, "workspace is not device memory");
  }
  drop_graph(h);
  h->ws = static_cast<char*>(dev_ptr);
  h->ws_len = bytes;
  h->written.assign(h->n_events, 0);
  h->parity = 0;
  int rc = upload_tables(h);
  if (rc) return rc;
  if ((rc = upload_eos(h))) return rc;
  HIPCHECK(h, shasta_launch::zero(dev_acc(h, 0), (int64_t)A_SIZE * h->n_events, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  return SHASTA_OK;
}

int shasta_set_eos(shasta_t* h, int kind, const double* params, int n_params) {
  if (!h) return SHASTA_EINVAL;
  if (kind == SHASTA_EOS_IDEAL) {
    if (n_params != 0) return fail(h, SHASTA_EINVAL, "ideal EOS takes no parameters");
    h->eos = EosParams{0, 0, 0.0, 0.0, 0.0, 0.0, nullptr, kNewtonDefault, 0};
  } else if (kind == SHASTA_EOS_BAG) {
    if (n_params != 2 || !params) return fail(h, SHASTA_EINVAL, "bag EOS takes {B, e_H}");
    const double B = params[0], eH = params[1];
    if (!(B > 0.0) || !(eH > 0.0) || !std::isfinite(B) || !std::isfinite(eH))
      return fail(h, SHASTA_EINVAL, "bag EOS needs B > 0 and e_H > 0");
    h->eos = EosParams{1, 0, B, eH, 0.0, 0.0, nullptr, kNewtonDefault, 0};
  } else if (kind == SHASTA_EOS_TABLE) {
    if (!params || n_params < 4 || n_params % 2 || n_params / 2 > kMaxEosNodes)
      return fail(h, SHASTA_EINVAL, "tabled EOS takes {e_0..e_m-1, p_0..p_m-1}, 2 <= m <= " +
                                        std::to_string(kMaxEosNodes));
    const int m = n_params / 2;
    const double* te = params;
    const double* tp = params + m;
    if (te[0] != 0.0) return fail(h, SHASTA_EINVAL, "tabled EOS: the first node must be e = 0");
    std::vector<double> tab(4 * (size_t)m);
    for (int k = 0; k < m; ++k) {
      if (!std::isfinite(te[k]) || !std::isfinite(tp[k]) || !(tp[k] >= 0.0))
        return fail(h, SHASTA_EINVAL, "tabled EOS: nodes must be finite with p >= 0");
      if (k > 0 && !(te[k] > te[k - 1]))
        return fail(h, SHASTA_EINVAL, "tabled EOS: node energies must increase");
      tab[k] = te[k];
      tab[m + k] = tp[k];
    }
    for (int k = 0; k + 1 < m; ++k) {
      const double a = (tp[k + 1] - tp[k]) / (te[k + 1] - te[k]);
      if (!(a >= 0.0 && a <= 1.0))
        return fail(h, SHASTA_EINVAL, "tabled EOS: slopes dp/de must lie in [0, 1]");
      tab[2 * m + k] = a;
      tab[3 * m + k] = tp[k] - a * te[k];
    }
    tab[3 * m - 1] = tab[3 * m - 2];   // the last segment continues past the last node
    tab[4 * m - 1] = tab[4 * m - 2];
    h->eos_tab.swap(tab);
    h->eos = EosParams{2, m, 0.0, 0.0, 0.0, 0.0, nullptr, kNewtonDefault, 0};
    if (int rc = upload_eos(h)) return rc;
  } else if (kind == SHASTA_EOS_BARYON) {
    if ((n_params != 2 && n_params != 3) || !params)
      return fail(h, SHASTA_EINVAL, "baryon EOS takes {cs2, mass} or {cs2, mass, iterations}");
    const double cs2 = params[0], mass = params[1];
    if (!(cs2 > 0.0 && cs2 <= 1.0) || !(mass >= 0.0) || !std::isfinite(mass))
      return fail(h, SHASTA_EINVAL, "baryon EOS needs 0 < cs2 <= 1 and a finite mass >= 0");
    int iters = kNewtonDefault;
    if (n_params == 3) {
      const double it = params[2];
      if (!(it >= 1.0 && it <= kNewtonLimit) || it != std::floor(it))
        return fail(h, SHASTA_EINVAL, "baryon EOS: iterations must be an integer in [1, " +
                                          std::to_string(kNewtonLimit) + "]");
      iters = (int)it;
    }
    h->eos = EosParams{3, 0, 0.0, 0.0, cs2, mass, nullptr, iters, 0};
  } else {
    return fail(h, SHASTA_EINVAL, "unknown EOS kind");
  }
  drop_graph(h);
  return SHASTA_OK;
}

int shasta_write_primitive(shasta_t* h, int ev, const double* e, const double* vx,
                           const double* vy, const double* vz, const double* n) {
  if (!h) return SHASTA_EINVAL;
  if (int rc = check_event(h, ev)) return rc;
  if (!h->ws) return fail(h, SHASTA_ESTATE, "no workspace bound");
  if (!e || !vx || !vy || !vz || !n) return fail(h, SHASTA_EINVAL, "null field pointer");
  const EventDesc& d = h->evd[ev];
  double* acc = dev_acc(h, ev);
  HIPCHECK(h, shasta_launch::zero(acc, A_SIZE, h->stream));
  HIPCHECK(h, shasta_launch::write_prim(h->precision == SHASTA_FP32_MIXED, h->eos, e, vx, vy, vz,
                                        n, dev_field(h, ev, h->parity), d.pitch, d.ncell,
                                        acc + A_INVALID, h->stream));
  if (int rc = refresh_sums(h, ev)) return rc;
  double a[A_SIZE];
  if (int rc = read_acc(h, ev, a)) return rc;
  h->written[ev] = 1;
  if (a[A_INVALID] > 0)
    return fail(h, SHASTA_EINVAL, std::to_string((long long)a[A_INVALID]) +
                                      " cells violate e >= 0, |v| < 1, n >= 0");
  return SHASTA_OK;
}

int shasta_write_conserved(shasta_t* h, int ev, const double* E, const double* Mx,
                           const double* My, const double* Mz, const double* R) {
  if (!h) return SHASTA_EINVAL;
  if (int rc = check_event(h, ev)) return rc;
  if (!h->ws) return fail(h, SHASTA_ESTATE, "no workspace bound");
  if (!E || !Mx || !My || !Mz || !R) return fail(h, SHASTA_EINVAL, "null field pointer");
  const EventDesc& d = h->evd[ev];
  HIPCHECK(h, shasta_launch::write_cons(h->precision == SHASTA_FP32_MIXED, E, Mx, My, Mz, R,
                                        dev_field(h, ev, h->parity), d.pitch, d.ncell,
                                        h->stream));
  if (int rc = refresh_sums(h, ev)) return rc;
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  h->written[ev] = 1;
  return SHASTA_OK;
}

int shasta_set_step_index(shasta_t* h, int64_t k) {
  if (!h) return SHASTA_EINVAL;
  if (k < 0) return fail(h, SHASTA_EINVAL, "negative step index");
  h->step_index = k;
  return SHASTA_OK;
}

int shasta_get_step_index(const shasta_t* h, int64_t* k) {
  if (!h || !k) return SHASTA_EINVAL;
  *k = h->step_index;
  return SHASTA_OK;
}

int shasta_step(shasta_t* h, double dt_fm, int nsteps) {
  if (!h) return SHASTA_EINVAL;
  if (!(dt_fm > 0.0) || !std::isfinite(dt_fm)) return fail(h, SHASTA_EINVAL, "dt must be > 0");
  const double lam = dt_fm / h->dx;
  if (!(lam < 0.5)) return fail(h, SHASTA_EINVAL, "dt/dx must be < 1/2");
  if (nsteps < 0) return fail(h, SHASTA_EINVAL, "nsteps must be >= 0");
  if (int rc = check_ready(h)) return rc;
  int left = nsteps;
  const bool use_graph = h->graph_enabled && !h->profiling;
  while (left > 0) {
    if (use_graph && h->step_index % 6 == 0 && left >= 6) {
      if (!h->gexec || h->graph_dt != dt_fm || h->graph_parity != h->parity ||
          h->graph_version != h->tables_version) {
        if (int rc = capture_cycle(h, dt_fm)) return rc;
      }
      while (left >= 6) {
        HIPCHECK(h, hipGraphLaunch(h->gexec, h->stream));
        h->step_index += 6;
        left -= 6;
        // 18 sweeps: the buffer parity is back where the cycle started
      }
      continue;
    }
    int parity = h->parity;
    if (int rc = enqueue_step(h, workspace_scratch(h), h->step_index, parity, dt_fm, h->stream))
      return rc;
    h->parity = parity;
    h->step_index += 1;
    left -= 1;
  }
  return SHASTA_OK;
}

int shasta_step_noalloc(shasta_t* h, double dt_fm, int nsteps) {
  if (!h) return SHASTA_EINVAL;
  if (!(dt_fm > 0.0) || !std::isfinite(dt_fm)) return fail(h, SHASTA_EINVAL, "dt must be > 0");
  const double lam = dt_fm / h->dx;
  if (!(lam < 0.5)) return fail(h, SHASTA_EINVAL, "dt/dx must be < 1/2");
  if (nsteps < 0) return fail(h, SHASTA_EINVAL, "nsteps must be >= 0");
  if (int rc = check_ready(h)) return rc;
  // layout of the static scratch for the current work tables: records of the
  // three sweeps, partials, counters and tickets
  size_t nrec = 0, nfin = 0;
  for (int ax = 0; ax < 3; ++ax) nrec = std::max(nrec, (size_t)h->n_records[ax]);
  for (int e = 0; e < h->n_events; ++e) nfin += (size_t)h->evd[e].fin_count;
  const size_t rec_bytes = align256(sizeof(double) * R_SIZE * nrec);
  const size_t part_bytes = align256(sizeof(double) * R_SIZE * nfin);
  const size_t cnt_bytes = align256(sizeof(double) * ((4 + (size_t)h->n_events + 1) / 2));
  const size_t need = 3 * rec_bytes + part_bytes + cnt_bytes;
  if (need > kStaticScratchBytes)
    return fail(h, SHASTA_EINVAL,
                "shasta_step_noalloc: the step needs " + std::to_string(need) +
                    " bytes of scratch, the static scratch holds " +
                    std::to_string(kStaticScratchBytes) +
                    " (fewer events, or more x windows per work item: shasta_set_tiles)");
  if (nsteps == 0) return SHASTA_OK;
  void* base = nullptr;
  HIPCHECK(h, shasta_launch::static_scratch(&base));
  char* p = static_cast<char*>(base);
  StepScratch sc;
  for (int k = 0; k < 3; ++k) sc.rec[k] = reinterpret_cast<double*>(p + k * rec_bytes);
  sc.partial = reinterpret_cast<double*>(p + 3 * rec_bytes);
  sc.cnt = reinterpret_cast<int*>(p + 3 * rec_bytes + part_bytes);
  sc.may_allocate = false;
  // queue counters and tickets start at zero (another call may have left
  // them anywhere); a fill kernel, not a memset, so the call can be captured
  HIPCHECK(h, shasta_launch::zero(reinterpret_cast<double*>(sc.cnt),
                                  (int64_t)(cnt_bytes / sizeof(double)), h->stream));
  for (int s = 0; s < nsteps; ++s) {
    int parity = h->parity;
    if (int rc = enqueue_step(h, sc, h->step_index, parity, dt_fm, h->stream)) return rc;
    h->parity = parity;
    h->step_index += 1;
  }
  return SHASTA_OK;
}

int shasta_read_field(shasta_t* h, int ev, int field, double* dst) {
  if (!h) return SHASTA_EINVAL;
  if (int rc = check_event(h, ev)) return rc;
  if (field < 0 || field > 10) return fail(h, SHASTA_EINVAL, "field index out of range");
  if (!dst) return fail(h, SHASTA_EINVAL, "null destination");
  if (!h->ws || !h->written[ev]) return fail(h, SHASTA_ESTATE, "event not written");
  const EventDesc& d = h->evd[ev];
  HIPCHECK(h, shasta_launch::read(h->precision == SHASTA_FP32_MIXED, h->eos,
                                  dev_field(h, ev, h->parity), d.pitch, d.ncell, field, dst,
                                  h->stream));
  double a[A_SIZE];
  if (int rc = read_acc(h, ev, a)) return rc;
  return health(h, a);
}

int shasta_reduce(shasta_t* h, int ev, double out[12], int64_t counters[4]) {
  if (!h) return SHASTA_EINVAL;
  if (int rc = check_event(h, ev)) return rc;
  if (!out || !counters) return fail(h, SHASTA_EINVAL, "null output");
  if (!h->ws || !h->written[ev]) return fail(h, SHASTA_ESTATE, "event not written");
  double a[A_SIZE];
  if (int rc = read_acc(h, ev, a)) return rc;
  for (int q = 0; q < 5; ++q) {
    out[q] = a[A_SUM + q];
    out[5 + q] = a[A_LEDGER + q];
  }
  out[10] = a[A_MAXEPS];
  out[11] = a[A_T];
  counters[0] = (int64_t)a[A_CLAMP];
  counters[1] = (int64_t)a[A_FLOOR];
  counters[2] = (int64_t)a[A_NOCONV];
  counters[3] = (int64_t)a[A_NONFINITE];
  return health(h, a);
}

int shasta_destroy(shasta_t* h) {
  if (!h) return SHASTA_EINVAL;
  drop_graph(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (auto& p : h->prof) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : h->event_pool) (void)hipEventDestroy(e);
  delete h;
  return SHASTA_OK;
}

const char* shasta_last_error(const shasta_t* h) { return h ? h->err.c_str() : "null handle"; }

const char* shasta_status_str(int status) {
  switch (status) {
    case SHASTA_OK: return "ok";
    case SHASTA_EINVAL: return "invalid argument";
    case SHASTA_ESTATE: return "call out of order";
    case SHASTA_EWORKSPACE: return "workspace missing, too small or misaligned";
    case SHASTA_EHIP: return "HIP runtime error";
    case SHASTA_ENONFINITE: return "non-finite value in the fields";
    case SHASTA_ENOCONVERGE: return "recovery did not converge";
    default: return "unknown status";
  }
}

int shasta_set_tiles(shasta_t* h, int axis, int p0, int p1) {
  if (!h) return SHASTA_EINVAL;
  if (axis < 0 || axis > 2) return fail(h, SHASTA_EINVAL, "axis must be 0, 1 or 2");
  if (p0 < 0) return fail(h, SHASTA_EINVAL, "p0 must be >= 0 (0 = automatic)");
  if (axis == 0) {
    h->xwin = p0;
  } else {
    if (p1 != 0 && p1 != kFlatLanes && p1 != 16 && p1 != 32 && p1 != 64)
      return fail(h, SHASTA_EINVAL,
                  "lanes along x must be 16, 32 or 64, or 1 for flattened columns "
                  "(0 = automatic)");
    if (p0 != 0 && p0 < 16) return fail(h, SHASTA_EINVAL, "segment length must be >= 16");
    h->seg[axis] = p0;
    h->lanes[axis] = p1;
  }
  build_tables(h);
  if (h->ws) return upload_tables(h);
  return SHASTA_OK;
}

int shasta_set_persistent(shasta_t* h, int axis, int enable) {
  if (!h) return SHASTA_EINVAL;
  if (axis < 0 || axis > 2) return fail(h, SHASTA_EINVAL, "axis must be 0, 1 or 2");
  h->persistent[axis] = enable != 0;
  drop_graph(h);
  return SHASTA_OK;
}

int shasta_get_tiles(const shasta_t* h, int axis, int* p0, int* p1) {
  if (!h || !p0 || !p1 || axis < 0 || axis > 2) return SHASTA_EINVAL;
  *p0 = axis == 0 ? h->xwin : h->seg[axis];
  *p1 = axis == 0 ? 0 : h->lanes[axis];
  return SHASTA_OK;
}

int shasta_get_persistent(const shasta_t* h, int axis, int* enable) {
  if (!h || !enable || axis < 0 || axis > 2) return SHASTA_EINVAL;
  *enable = h->persistent[axis] ? 1 : 0;
  return SHASTA_OK;
}

int shasta_autotune(shasta_t* h, double dt_fm, int reps) {
  if (!h) return SHASTA_EINVAL;
  if (!(dt_fm > 0.0) || !(dt_fm / h->dx < 0.5)) return fail(h, SHASTA_EINVAL, "bad dt");
  if (reps < 1) reps = 1;
  if (int rc = check_ready(h)) return rc;
  // a decomposition chosen before for the same device, precision, scheme
  // and grids is taken again without timing
  std::string key;
  if (int rc = tune_key(h, key)) return rc;
  {
    std::lock_guard<std::mutex> g(tune_cache_lock());
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
      for (int ax = 0; ax < 3; ++ax) set_choice(h, ax, it->second[ax]);
      build_tables(h);
      drop_graph(h);
      return upload_tables(h);
    }
  }
  const double lam = dt_fm / h->dx;
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHECK(h, hipEventCreate(&a));
  HIPCHECK(h, hipEventCreate(&b));
  const bool saved_prof = h->profiling;
  h->profiling = false;
  int max_n = 0;
  for (int e = 0; e < h->n_events; ++e)
    for (int ax = 0; ax < 3; ++ax) max_n = std::max(max_n, h->dims[3 * e + ax]);
  // A sweep reads buffer `parity` and writes the other one, so repeated
  // sweeps leave the state untouched; the queue counter of a sweep's slot is
  // reset before every launch (a step does that in its reduction).  `axes`
  // lists the sweeps of one timed unit: one axis alone, or the three axes of
  // a step (all reading the same buffer, in the order of the step).
  auto time_sweeps = [&](const int* axes, int n_axes, float& ms) -> int {
    const StepScratch sc = workspace_scratch(h);
    auto unit = [&]() -> int {
      for (int w = 0; w < n_axes; ++w) {
        HIPCHECK(h, reset_counters(h, h->stream));
        if (int rc = launch_sweep(h, sc, axes[w], h->parity, w, lam, h->stream)) return rc;
      }
      return SHASTA_OK;
    };
    for (int r = 0; r < 2; ++r)
      if (int rc = unit()) return rc;
    // the fastest of three timed blocks: filters clock ramps and interference
    ms = 1e30f;
    for (int t = 0; t < 3; ++t) {
      HIPCHECK(h, hipEventRecord(a, h->stream));
      for (int r = 0; r < reps; ++r)
        if (int rc = unit()) return rc;
      HIPCHECK(h, hipEventRecord(b, h->stream));
      HIPCHECK(h, hipEventSynchronize(b));
      float t_ms = 0.0f;
      HIPCHECK(h, hipEventElapsedTime(&t_ms, a, b));
      ms = std::min(ms, t_ms);
    }
    return SHASTA_OK;
  };
  auto apply = [&](int ax, const TuneChoice& c) -> int {
    set_choice(h, ax, c);
    build_tables(h);
    return upload_tables(h);
  };
  // SHASTA_TUNE_LOG set: every timing goes to stderr
  const bool log = std::getenv("SHASTA_TUNE_LOG") != nullptr;
  auto report = [&](const char* pass, int ax, const TuneChoice& c, float ms) {
    if (log)
      std::fprintf(stderr, "shasta_autotune %s axis %d p0 %d p1 %d persistent %d: %.4f ms\n",
                   pass, ax, c.p0, c.p1, c.pers ? 1 : 0, ms);
  };
  int rc = SHASTA_OK;
  // first pass, per axis: every candidate decomposition (x: windows per
  // wave; y/z: segment length and lanes along x; persistent launch or not)
  // timed on repeated sweeps of that axis alone; then six of them again
  // (below), interleaved, three more times (a candidate keeps its fastest
  // time)
  std::vector<TuneChoice> ranked[3];
  for (int ax = 0; ax < 3 && rc == SHASTA_OK; ++ax) {
    std::vector<TuneChoice> cands;
    for (int pers = 0; pers < 2; ++pers) {
      if (ax == 0) {
        for (int w : {2, 4, 6, 8, 12, 16, 24, 32}) cands.push_back({w, 0, pers != 0, 0.0f});
      } else {
        // segment lengths: whole pencils, pencils cut into 2..8 equal parts,
        // and a few fixed lengths (a segment recomputes 6 cells per side)
        std::vector<int> len;
        for (int parts = 1; parts <= 8; ++parts) len.push_back((max_n + parts - 1) / parts);
        for (int L : {16, 24, 32, 48, 64, 96, 128}) len.push_back(L);
        std::sort(len.begin(), len.end());
        len.erase(std::unique(len.begin(), len.end()), len.end());
        for (int lx : {kFlatLanes, 16, 32, 64})
          for (int L : len)
            if (L >= 16 || L >= max_n) cands.push_back({std::min(L, max_n), lx, pers != 0, 0.0f});
      }
    }
    const int one[1] = {ax};
    for (TuneChoice& c : cands) {
      if ((rc = apply(ax, c))) break;
      if ((rc = time_sweeps(one, 1, c.ms))) break;
      report("sweep", ax, c, c.ms);
    }
    if (rc) break;
    std::stable_sort(cands.begin(), cands.end(),
                     [](const TuneChoice& x, const TuneChoice& y) { return x.ms < y.ms; });
    // the four fastest, then the fastest of up to two further segment
    // lengths (windows per wave for x): a sweep timed alone favours long
    // segments, which in the full step are not always faster
    std::vector<TuneChoice> sel(cands.begin(), cands.begin() + std::min<size_t>(4, cands.size()));
    for (const TuneChoice& c : cands) {
      if (sel.size() >= 6) break;
      bool fresh = true;
      for (const TuneChoice& t : sel) fresh = fresh && t.p0 != c.p0;
      if (fresh) sel.push_back(c);
    }
    for (int round = 0; round < 3 && rc == SHASTA_OK; ++round)
      for (TuneChoice& c : sel) {
        float ms;
        if ((rc = apply(ax, c))) break;
        if ((rc = time_sweeps(one, 1, ms))) break;
        report("sweep-again", ax, c, ms);
        c.ms = std::min(c.ms, ms);
      }
    if (rc) break;
    std::stable_sort(sel.begin(), sel.end(),
                     [](const TuneChoice& x, const TuneChoice& y) { return x.ms < y.ms; });
    ranked[ax] = sel;
    set_choice(h, ax, sel[0]);
  }
  // second pass: a sweep alone, repeated on the same input, does not see
  // what the step's other sweeps leave in the caches, nor their order of
  // reading and writing.  The six kept for each axis are timed again in
  // real time steps (the other axes at their current choice), and the
  // fastest step wins.  The steps advance the state, so the current buffer
  // of every event, its accumulators, the step index and the buffer parity
  // are kept in host memory and put back afterwards.
  if (rc == SHASTA_OK) {
    std::vector<char> saved;
    const int parity0 = h->parity;
    const int64_t step0 = h->step_index;
    size_t total = sizeof(double) * A_SIZE * (size_t)h->n_events;
    for (int e = 0; e < h->n_events; ++e) total += kNF * (size_t)h->evd[e].pitch * h->elem;
    saved.resize(total);
    auto copy_state = [&](bool back) -> int {
      size_t o = 0;
      for (int e = 0; e < h->n_events; ++e) {
        const size_t n = kNF * (size_t)h->evd[e].pitch * h->elem;
        char* dev = dev_field(h, e, parity0);
        HIPCHECK(h, back ? hipMemcpyAsync(dev, saved.data() + o, n, hipMemcpyHostToDevice,
                                          h->stream)
                         : hipMemcpyAsync(saved.data() + o, dev, n, hipMemcpyDeviceToHost,
                                          h->stream));
        o += n;
      }
      const size_t n = sizeof(double) * A_SIZE * (size_t)h->n_events;
      HIPCHECK(h, back ? hipMemcpyAsync(dev_acc(h, 0), saved.data() + o, n,
                                        hipMemcpyHostToDevice, h->stream)
                       : hipMemcpyAsync(saved.data() + o, dev_acc(h, 0), n,
                                        hipMemcpyDeviceToHost, h->stream));
      HIPCHECK(h, hipStreamSynchronize(h->stream));
      return SHASTA_OK;
    };
    auto time_steps = [&](float& ms) -> int {
      const StepScratch sc = workspace_scratch(h);
      auto steps = [&](int n) -> int {
        for (int k = 0; k < n; ++k) {
          int parity = h->parity;
          if (int r = enqueue_step(h, sc, h->step_index, parity, dt_fm, h->stream)) return r;
          h->parity = parity;
          h->step_index += 1;
        }
        return SHASTA_OK;
      };
      if (int r = steps(1)) return r;
      ms = 1e30f;
      for (int t = 0; t < 3; ++t) {
        HIPCHECK(h, hipEventRecord(a, h->stream));
        if (int r = steps(reps)) return r;
        HIPCHECK(h, hipEventRecord(b, h->stream));
        HIPCHECK(h, hipEventSynchronize(b));
        float t_ms = 0.0f;
        HIPCHECK(h, hipEventElapsedTime(&t_ms, a, b));
        ms = std::min(ms, t_ms);
      }
      return SHASTA_OK;
    };
    rc = copy_state(false);
    std::vector<TuneChoice> by_step[3];   // per axis, fastest step first
    for (int ax = 0; ax < 3 && rc == SHASTA_OK; ++ax) {
      const size_t n = std::min<size_t>(6, ranked[ax].size());
      std::vector<float> best(n, 1e30f);
      for (int round = 0; round < 2 && rc == SHASTA_OK; ++round)
        for (size_t i = 0; i < n; ++i) {
          float ms;
          if ((rc = apply(ax, ranked[ax][i]))) break;
          if ((rc = time_steps(ms))) break;
          report("step", ax, ranked[ax][i], ms);
          best[i] = std::min(best[i], ms);
        }
      if (rc) break;
      for (size_t i = 0; i < n; ++i) ranked[ax][i].ms = best[i];
      by_step[ax].assign(ranked[ax].begin(), ranked[ax].begin() + n);
      std::stable_sort(by_step[ax].begin(), by_step[ax].end(),
                       [](const TuneChoice& x, const TuneChoice& y) { return x.ms < y.ms; });
      set_choice(h, ax, by_step[ax][0]);
    }
    // third pass: what one of the y/z sweeps finds in the caches depends on
    // how the other one walked the grid (256^3 FP32: y and z both in
    // 128-cell segments 0.581 ms per step, either one alone 0.605, both whole
    // pencils 0.610), which the axis-by-axis passes cannot see.  For y and
    // for z the fastest candidate and the fastest of another segment length
    // are timed in all four pairs.
    if (rc == SHASTA_OK && by_step[1].size() >= 2 && by_step[2].size() >= 2) {
      TuneChoice two[3][2];
      for (int ax = 1; ax < 3; ++ax) {
        two[ax][0] = by_step[ax][0];
        two[ax][1] = by_step[ax][1];
        for (const TuneChoice& c : by_step[ax])
          if (c.p0 != by_step[ax][0].p0) { two[ax][1] = c; break; }
      }
      float best = 1e30f;
      int by = 0, bz = 0;
      for (int round = 0; round < 2 && rc == SHASTA_OK; ++round)
        for (int iy = 0; iy < 2 && rc == SHASTA_OK; ++iy)
          for (int iz = 0; iz < 2; ++iz) {
            float ms;
            set_choice(h, 1, two[1][iy]);
            if ((rc = apply(2, two[2][iz]))) break;
            if ((rc = time_steps(ms))) break;
            if (log)
              std::fprintf(stderr, "shasta_autotune pair y %d,%d,%d z %d,%d,%d: %.4f ms\n",
                           two[1][iy].p0, two[1][iy].p1, two[1][iy].pers ? 1 : 0,
                           two[2][iz].p0, two[2][iz].p1, two[2][iz].pers ? 1 : 0, ms);
            if (ms < best) { best = ms; by = iy; bz = iz; }
          }
      if (rc == SHASTA_OK) {
        set_choice(h, 1, two[1][by]);
        set_choice(h, 2, two[2][bz]);
      }
    }
    h->parity = parity0;
    h->step_index = step0;
    const int rc_restore = copy_state(true);
    if (rc == SHASTA_OK) rc = rc_restore;
  }
  build_tables(h);
  int rc2 = upload_tables(h);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  h->profiling = saved_prof;
  drop_graph(h);
  if (rc == SHASTA_OK && rc2 == SHASTA_OK) {
    std::array<TuneChoice, 3> c;
    for (int ax = 0; ax < 3; ++ax) c[ax] = current_choice(h, ax);
    std::lock_guard<std::mutex> g(tune_cache_lock());
    tune_cache()[key] = c;
  }
  return rc ? rc : rc2;
}

int shasta_forget_tuning(void) {
  std::lock_guard<std::mutex> g(tune_cache_lock());
  tune_cache().clear();
  return SHASTA_OK;
}

int shasta_set_antidiffusion(shasta_t* h, double diff) {
  if (!h) return SHASTA_EINVAL;
  if (!(diff >= 0.0 && diff <= 1.0)) return fail(h, SHASTA_EINVAL, "diff must lie in [0, 1]");
  h->diff = diff;
  drop_graph(h);   // the captured launches carry the old value
  return SHASTA_OK;
}

int shasta_set_graph(shasta_t* h, int enable) {
  if (!h) return SHASTA_EINVAL;
  h->graph_enabled = enable != 0;
  if (!h->graph_enabled) drop_graph(h);
  return SHASTA_OK;
}

int shasta_set_profiling(shasta_t* h, int enable) {
  if (!h) return SHASTA_EINVAL;
  h->profiling = enable != 0;
  return SHASTA_OK;
}

int shasta_read_profile(shasta_t* h, double ms[4], int64_t launches[4]) {
  if (!h || !ms || !launches) return SHASTA_EINVAL;
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  for (auto& p : h->prof) {
    float t = 0.f;
    HIPCHECK(h, hipEventElapsedTime(&t, p.a, p.b));
    h->prof_ms[p.cls] += t;
    h->prof_n[p.cls] += 1;
    h->event_pool.push_back(p.a);
    h->event_pool.push_back(p.b);
  }
  h->prof.clear();
  for (int c = 0; c < 4; ++c) {
    ms[c] = h->prof_ms[c];
    launches[c] = h->prof_n[c];
    h->prof_ms[c] = 0;
    h->prof_n[c] = 0;
  }
  return SHASTA_OK;
}

int shasta_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
  if (!src || !dst || bytes % 16) return SHASTA_EINVAL;
  if (shasta_launch::copy(src, dst, bytes, static_cast<hipStream_t>(hip_stream)) != hipSuccess)
    return SHASTA_EHIP;
  return SHASTA_OK;
}

int shasta_march_copy(const void* src, void* dst, int nx, int ny, int nz, int64_t pitch,
                      int axis, int seg_len, int precision, void* hip_stream) {
  if (!src || !dst || nx < 1 || ny < 1 || nz < 1 || (axis != 1 && axis != 2) || seg_len < 1 ||
      (precision != SHASTA_FP64 && precision != SHASTA_FP32_MIXED))
    return SHASTA_EINVAL;
  const int64_t ncell = (int64_t)nx * ny * nz;
  const int64_t elem = precision == SHASTA_FP64 ? 8 : 4;
  // one field array below 2^31 bytes: 32-bit buffer offsets, as in the sweeps
  if (pitch < ncell || ncell > 2147483647LL / elem) return SHASTA_EINVAL;
  if (shasta_launch::march_copy(precision == SHASTA_FP32_MIXED, src, dst, nx, ny, nz, pitch,
                                axis, seg_len, static_cast<hipStream_t>(hip_stream)) !=
      hipSuccess)
    return SHASTA_EHIP;
  return SHASTA_OK;
}

int shasta_selftest_math(const double* in, double* out, int n, int which, void* hip_stream) {
  if (!in || !out || n < 0 || (which != 0 && which != 1)) return SHASTA_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (n == 0) return SHASTA_OK;
  if (shasta_launch::selftest(in, out, n, which, st) != hipSuccess) return SHASTA_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return SHASTA_EHIP;
  return SHASTA_OK;
}

int shasta_selftest_recover(shasta_t* h, const double* in, double* out, int n) {
  if (!h) return SHASTA_EINVAL;
  if (!in || !out || n < 0) return fail(h, SHASTA_EINVAL, "null buffer or n < 0");
  if (!h->ws) return fail(h, SHASTA_ESTATE, "no workspace bound");
  if (n == 0) return SHASTA_OK;
  HIPCHECK(h, shasta_launch::selftest_recover(h->eos, in, out, n, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  return SHASTA_OK;
}

}  // extern "C"
