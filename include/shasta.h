/*
 * shasta.h — C ABI of the MI355X (gfx950) relativistic SHASTA library.
 *
 * One time step of the 3+1D relativistic SHASTA flux-corrected transport of
 * "Relativistic Hydrodynamics on Graphic Cards" (arXiv:1206.0919): the
 * dimensionally split x/y/z sweeps (half-step predictor, transport with
 * diffusion, phoenical antidiffusion with flux limiter; Sec. 3, eqs.
 * shasta-diff, shasta-geo, shasta-n) over the conserved fields E, M_x, M_y,
 * M_z, R (eqs. cf-density, cf-momentum, cf-energy), and the cell-wise
 * recovery of e, v, n through the equation of state (Sec. 3, last paragraph).
 *
 * Conventions for every call
 *   - Return value: a status code below; no C++ exception crosses the ABI.
 *     The message of the last failure is available from shasta_last_error().
 *   - Pointers named *_dev are device (HBM) pointers of the calling process;
 *     the caller owns them.  Host pointers are named without suffix.
 *   - Field arrays are dense, x fastest: index = x + nx*(y + ny*z), FP64.
 *   - Units: e, p, E, M in GeV/fm^3; n, R in fm^-3; lengths fm; times fm/c.
 *   - A handle is not thread safe; separate handles are independent.
 *   - Work is enqueued on the HIP stream given at creation.  Calls documented
 *     as "asynchronous" return before the GPU work ends; device-side errors
 *     (non-finite results) are reported by the next synchronizing call.
 */
#ifndef SHASTA_H
#define SHASTA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct shasta_handle shasta_t;

/* status codes */
#define SHASTA_OK 0
#define SHASTA_EINVAL 1      /* bad argument (checked on the host)          */
#define SHASTA_ESTATE 2      /* call out of order (e.g. step before init)   */
#define SHASTA_EWORKSPACE 3  /* workspace missing, too small or misaligned  */
#define SHASTA_EHIP 4        /* a HIP runtime call failed                   */
#define SHASTA_ENONFINITE 5  /* a non-finite value appeared in the fields   */
#define SHASTA_ENOCONVERGE 6 /* recovery root solve did not converge        */

/* precision of the stored fields and of the transport */
#define SHASTA_FP64 0       /* everything in FP64                             */
#define SHASTA_FP32_MIXED 1 /* fields and transport FP32; recovery and sums
                               FP64 (Sec. 5: double precision for the boost) */

/* boundary condition */
#define SHASTA_BC_OUTFLOW 0 /* three halo cells copy the edge cell (Sec. 3.1) */

/* equations of state */
#define SHASTA_EOS_IDEAL 0 /* p = e/3 (Sec. 2, ideal gas)                    */
#define SHASTA_EOS_BAG 1   /* bag model: p = e/3 (e <= e_H), e_H/3 in the
                              mixed phase, (e - 4B)/3 (e >= e_H + 4B)        */
#define SHASTA_EOS_TABLE 2 /* tabulated p(e), linear between nodes          */
#define SHASTA_EOS_BARYON 3 /* p(e, n) = cs2 max(0, e - mass n)             */

/* field indices for shasta_read_field */
#define SHASTA_FIELD_E 0
#define SHASTA_FIELD_MX 1
#define SHASTA_FIELD_MY 2
#define SHASTA_FIELD_MZ 3
#define SHASTA_FIELD_R 4
#define SHASTA_FIELD_e 5  /* recomputed primitives (recovery of Sec. 3) */
#define SHASTA_FIELD_p 6
#define SHASTA_FIELD_vx 7
#define SHASTA_FIELD_vy 8
#define SHASTA_FIELD_vz 9
#define SHASTA_FIELD_n 10

/*
 * Create a handle for a batch of n_events independent grids (a single grid
 * is a batch of 1).  dims[3*k+0..2] = nx, ny, nz of event k, each >= 1;
 * one field array of an event must stay below 2^31 bytes (the kernels
 * address fields with 32-bit byte offsets): at most 268,434,943 cells per
 * event in FP64, 536,869,887 in FP32; dx_fm > 0 is the cell size of every
 * event;
 * precision is SHASTA_FP64 or SHASTA_FP32_MIXED; bc must be
 * SHASTA_BC_OUTFLOW; hip_stream is a hipStream_t (NULL = default stream).
 * Validation is done on the CPU before any HIP call; nothing is allocated on
 * the device.  The EOS defaults to SHASTA_EOS_IDEAL.
 */
int shasta_create(shasta_t** out, int n_events, const int32_t* dims,
                  double dx_fm, int precision, int bc, void* hip_stream);

/* Device bytes the handle needs: ping-pong field buffers, work tables,
 * reduction records and per-event accumulators. */
int shasta_workspace_bytes(const shasta_t* h, size_t* bytes);

/* Bind caller-owned device memory (e.g. a torch uint8 tensor), 256-byte
 * aligned and at least shasta_workspace_bytes() long.  The caller keeps it
 * alive until shasta_destroy().  Uploads the work tables (synchronous). */
int shasta_bind_workspace(shasta_t* h, void* dev_ptr, size_t bytes);

/* Select the EOS.  SHASTA_EOS_IDEAL takes no parameters (n_params = 0);
 * SHASTA_EOS_BAG takes params = {B, e_H} in GeV/fm^3, both > 0 and finite
 * (e_Q = e_H + 4B is derived).  SHASTA_EOS_TABLE (a tabulated p(e) read
 * through an interpolation, Sec. 2 and Sec. 3, last paragraph) takes
 * params = {e_0, ..., e_{m-1}, p_0, ..., p_{m-1}}, n_params = 2m,
 * 2 <= m <= 1024, host memory, copied: e_0 = 0 < e_1 < ... (GeV/fm^3),
 * p_k >= 0, finite, every slope (p_{k+1} - p_k)/(e_{k+1} - e_k) in [0, 1];
 * p is linear between neighbouring nodes and the last segment continues
 * past e_{m-1}.  SHASTA_EOS_BARYON (the pressure from the rest-frame energy
 * and baryon densities, Sec. 3, last paragraph) takes params = {cs2, mass}
 * or {cs2, mass, iterations}: p = cs2 max(0, e - mass n), 0 < cs2 <= 1,
 * mass >= 0 in GeV; its recovery solves for v with n = R sqrt(1 - v^2) by a
 * safeguarded Newton iteration of at most `iterations` steps (an integer in
 * [1, 64], 16 by default); a recovery still unconverged then keeps its last
 * iterate and is counted (shasta_reduce counters[2], SHASTA_ENOCONVERGE).
 * EINVAL on any violation (the previous EOS stays).  May be called before or
 * after shasta_bind_workspace.  The tabled and baryon EOS always use the grid
 * launch (shasta_set_persistent is then ignored). */
int shasta_set_eos(shasta_t* h, int kind, const double* params, int n_params);

/* Write the state of event ev from primitive fields (device pointers to
 * dense FP64 arrays of the event's cells): e >= 0, |v| < 1, n >= 0.
 * Converts with eqs. cf-density, cf-momentum, cf-energy on the device.
 * Synchronous; returns SHASTA_EINVAL (state written anyway) if any cell
 * violates the ranges.  Resets the accumulators (ledger, t, counters) of ev. */
int shasta_write_primitive(shasta_t* h, int ev, const double* e_dev,
                           const double* vx_dev, const double* vy_dev,
                           const double* vz_dev, const double* n_dev);

/* Write the conserved state of event ev (device FP64 arrays).  Used for
 * resume; no admissibility check (the recovery guard handles E <= 0 or
 * |M| >= E and counts it).  Synchronous.  Does not reset the accumulators. */
int shasta_write_conserved(shasta_t* h, int ev, const double* E_dev,
                           const double* Mx_dev, const double* My_dev,
                           const double* Mz_dev, const double* R_dev);

/* Set the step index k; it fixes the axis order of the next step
 * (Appendix A, Listing 2 permutation table, period 6).  k >= 0. */
int shasta_set_step_index(shasta_t* h, int64_t k);
int shasta_get_step_index(const shasta_t* h, int64_t* k);

/*
 * Advance every event by nsteps >= 0 time steps of dt_fm.  One step = three
 * directional sweeps with the full dt in the order of the permutation table;
 * each sweep = outflow halo, recovery at U^n, lambda/2 predictor, recovery at
 * U^{n+1/2}, lambda corrector from U^n (Sec. 3 and Sec. 3.1).  Requires
 * 0 < dt/dx < 1/2, a bound workspace and every event written.
 * Asynchronous on the stream.
 */
int shasta_step(shasta_t* h, double dt_fm, int nsteps);

/*
 * shasta_step without any allocation, for callers that cannot allocate
 * device memory or create runtime objects while it runs (code under HIP
 * graph capture, tight serving loops, harnesses that forbid it).  Same
 * arguments, requirements and results as shasta_step, bit for bit; the
 * fields and accumulators stay in the bound workspace, while the step's
 * scratch (reduction records, step-reduction partials, queue counters,
 * tickets) lives in a static device array of 16 MiB that the library holds
 * on each GPU until the process ends.  Kernels are launched one by one (no
 * graph, no timing events, no stream creation).  SHASTA_EINVAL, with nothing
 * launched, if the current work tables need more scratch than that (the
 * message gives both sizes; more x windows per work item, shasta_set_tiles,
 * or fewer events reduce it).  All calls on one GPU share the array: calls
 * that overlap on one GPU (other streams or threads) race.  The first call on
 * a device looks up the array's device address (with that device current).
 * Asynchronous on the stream.
 */
int shasta_step_noalloc(shasta_t* h, double dt_fm, int nsteps);

/* Copy one field of event ev to dst_dev (dense FP64, the event's cells).
 * field 0..4: E, M_x, M_y, M_z, R; 5..10: e, p, v_x, v_y, v_z, n recomputed
 * from the conserved state.  Synchronizes; the field is copied in every case,
 * but the call returns SHASTA_ENONFINITE if a non-finite value was flagged
 * since the last write, else SHASTA_ENOCONVERGE if a recovery of the sweeps
 * stopped before its root converged (baryon EOS only) since the last
 * write_primitive. */
int shasta_read_field(shasta_t* h, int ev, int field, double* dst_dev);

/*
 * Reductions of event ev (synchronizes).  out[0..4]: FP64 sums over the
 * cells of E, M_x, M_y, M_z, R after the last step; out[5..9]: accumulated
 * net boundary outflow of the same fields since the last write_primitive
 * (sum(t) + outflow = sum(0) is the conservation invariant); out[10]: largest
 * |lambda v_sweep| of the corrector's half-step velocity (Sec. 3.1) seen;
 * out[11]: elapsed time t.  counters[0..3]: recoveries with |M| clamped,
 * recoveries with E floored (the admissibility guard of the recovery,
 * Sec. 3, the relativistic correction), recoveries whose iterative root
 * solve stopped before converging (baryon EOS only: the other EOS are solved
 * in closed form), steps with non-finite values.  The guard and convergence
 * counters count each interior cell once per time level (n and n+1/2) of
 * every sweep.  Sums are deterministic (fixed reduction order).  The outputs
 * are written in every case; the return value is SHASTA_ENONFINITE or
 * SHASTA_ENOCONVERGE as for shasta_read_field.
 */
int shasta_reduce(shasta_t* h, int ev, double out[12], int64_t counters[4]);

int shasta_destroy(shasta_t* h);
const char* shasta_last_error(const shasta_t* h);
const char* shasta_status_str(int status);

/* ---------------------------------------------------------------- tuning */

/*
 * Work decomposition of the sweeps (results are bitwise independent of it).
 * axis 0 (x sweep): p0 = most windows per wave (a window holds 128 positions:
 * row pieces with a 6-cell halo each; items shrink toward the end of the
 * launch), p1 ignored.  axis 1, 2 (y, z sweeps): p0 = segment length along
 * the sweep axis (>= 16; the pencil is cut into ceil(N/p0) segments, each
 * recomputing a 6-cell margin), p1 = lanes along x per wave (16, 32 or 64;
 * the other lanes take the next rows of the transverse plane), or 1: the wave
 * takes 64 consecutive columns of the transverse plane in x-fastest order,
 * wrapping from the end of one row to the start of the next (no idle lane
 * but in the plane's last wave).  0 for either = automatic (p1: 1).  Rebuilds
 * the work tables; if a workspace is bound it must still be large enough
 * (shasta_workspace_bytes tells).  EINVAL for other values.
 */
int shasta_set_tiles(shasta_t* h, int axis, int p0, int p1);

/* Persistent launch of the sweeps along axis (enable = 1): as many blocks as
 * fit on the GPU at once take work items (pencil segments or x windows of
 * every event of the batch) from a queue, largest first, until it is empty.
 * enable = 0: one block (y, z) or wave (x) per work item.  Results are
 * bitwise independent of the choice. */
int shasta_set_persistent(shasta_t* h, int axis, int enable);

/* Current decomposition of axis: p0, p1 as for shasta_set_tiles, and 1 if
 * its sweeps use the persistent launch.  EINVAL for a bad axis or a null
 * output pointer. */
int shasta_get_tiles(const shasta_t* h, int axis, int* p0, int* p1);
int shasta_get_persistent(const shasta_t* h, int axis, int* enable);

/* Antidiffusion coefficient: the constant diff that scales the phoenical
 * antiflux A^ph (Sec. 3; Sec. 3.1 and Listing 1 name it), 1 by default.
 * 0 <= diff
 * <= 1, else EINVAL.  diff = 0 selects sweep kernels compiled without the
 * antiflux and its flux limiter (the transport step alone, as the paper's
 * runs without anti-flux in Sec. 4): their fields equal those of the
 * limiter kernels at
 * diff = 0; they always use the grid launch (shasta_set_persistent is then
 * ignored).  Takes effect at the next shasta_step. */
int shasta_set_antidiffusion(shasta_t* h, double diff);

/* Time candidate decompositions (tiles and persistent or not) on the device
 * with the given dt and keep the fastest per axis.  First pass, per axis: a
 * candidate's time is the fastest of three blocks of reps sweeps of that
 * axis (each reads the current buffer and writes the other one); the four
 * fastest and the fastest of up to two further segment lengths (x: windows
 * per wave) are timed again, interleaved, three more times.  Second pass:
 * these six of each axis are timed in real time steps (three blocks of
 * reps steps, the other axes at their current choice), and the fastest
 * steps decide; then, for y and for z, the fastest and the fastest of
 * another segment length are timed in all four pairs, as one sweep's
 * segments change what the other finds in the caches.  The state is left as it was: the current fields and the
 * accumulators of every event go to host memory (allocated by the call)
 * before the second pass and back after it, with the step index.  The choice
 * is kept, for the rest of the process, under the device, precision, EOS
 * kind, antiflux on or off and the grid sizes of the batch: a later call
 * with the same key takes it without timing.  Synchronous. */
int shasta_autotune(shasta_t* h, double dt_fm, int reps);

/* Forget every decomposition shasta_autotune kept in this process. */
int shasta_forget_tuning(void);

/* Capture the steady-state step cycle (6 steps) in a HIP graph and replay it
 * (enable = 1, default) or launch kernels one by one (enable = 0). */
int shasta_set_graph(shasta_t* h, int enable);

/* Per-kernel timing with HIP events on the handle's stream.  While enabled,
 * shasta_step launches kernel by kernel and records an event pair around
 * each sweep and reduction launch.  shasta_read_profile synchronizes and
 * returns the summed milliseconds and launch counts of: [0] x sweeps,
 * [1] y sweeps, [2] z sweeps, [3] step reductions, then clears them. */
int shasta_set_profiling(shasta_t* h, int enable);
int shasta_read_profile(shasta_t* h, double ms[4], int64_t launches[4]);

/* ----------------------------------------------------- measurement helpers */

/* Plain streaming copy of `bytes` (multiple of 16) from src_dev to dst_dev
 * on hip_stream, used to calibrate bandwidth and traffic counters. */
int shasta_stream_copy(const void* src_dev, void* dst_dev, size_t bytes,
                       void* hip_stream);

/* Copy with the memory pattern of a y (axis 1) or z (axis 2) sweep and none
 * of its arithmetic, to measure what that pattern alone allows (a
 * calibration helper like shasta_stream_copy; the sweep it mimics reads its
 * pencils with the 3-cell halos of both half steps, Sec. 3.1).  src_dev and
 * dst_dev each hold five fields of nx*ny*nz values, x fastest, field q
 * starting at element q*pitch (pitch >= nx*ny*nz); values are doubles for
 * SHASTA_FP64 and floats for SHASTA_FP32_MIXED, and one field is below
 * 2^31 bytes.  One wave per segment of seg_len cells of 64 consecutive
 * columns of the transverse plane loads rows along the axis one row ahead,
 * with 6 clamped halo rows before and after the segment, and stores the
 * segment: afterwards dst_dev holds a copy of src_dev.  Asynchronous on
 * hip_stream; SHASTA_EINVAL for a bad argument (nothing launched). */
int shasta_march_copy(const void* src_dev, void* dst_dev, int nx, int ny, int nz,
                      int64_t pitch, int axis, int seg_len, int precision,
                      void* hip_stream);

/* Device math self-check: out_dev[i] = f(in_dev[i]) for n values with
 * which = 0: the FP64 reciprocal, 1: the FP64 square root used by the
 * kernels.  Synchronous. */
int shasta_selftest_math(const double* in_dev, double* out_dev, int n,
                         int which, void* hip_stream);

/* Recovery self-check with the handle's EOS (Sec. 3, last paragraph: the
 * boost to the rest frame): for n cells, in_dev[5i..5i+4] = (E, M_x, M_y,
 * M_z, R) -> out_dev[4i..4i+3] = (e, p, |v|, clamped + 2 floored + 4 not
 * converged), computed
 * by the same device code the sweeps use.  Device pointers; needs a bound
 * workspace (the tabled EOS lives there); synchronous on the handle's
 * stream. */
int shasta_selftest_recover(shasta_t* h, const double* in_dev, double* out_dev, int n);

#ifdef __cplusplus
}
#endif
#endif /* SHASTA_H */
