/*
 * dpd.h -- C ABI of the MI355X (gfx950) library for one DPD time step of
 * fluid particles and frozen wall particles with phase-field bounce-back
 * (Xu & Meakin, "A phase field approach to no slip boundary conditions in
 * dissipative particle dynamics and other particle models for fluid flow in
 * geometrically complex confined systems").
 *
 * Every entry point returns an int status: DPD_OK (0) or a negative DPD_E_*
 * code; nothing throws or aborts across the ABI.  dpd_last_error() gives a
 * message for the last failure of a context.  Errors detected on the device
 * (non-finite state, a displacement above half a cell in one step) are
 * latched in a device status word and returned by the next dpd_sync() or
 * getter.  A context is used by one host thread at a time.
 *
 * Units: the cutoff rc is the length unit of the paper (Eq. 5) but is a
 * parameter here; mass is 1.  The box is periodic along x, y and z.
 *
 * Memory: unless a struct says otherwise, pointers handed to the library
 * are borrowed for the duration of the call.  Outputs are caller-owned
 * device buffers written asynchronously on the context stream; they are
 * valid once the stream has reached that point (dpd_sync() or any stream
 * synchronisation).  Device memory of a context comes from the caller's
 * allocator when one is given (e.g. PyTorch's caching allocator), from
 * hipMalloc otherwise, and is released by dpd_destroy().
 */
#ifndef DPD_H
#define DPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DPD_OK = 0,
    DPD_E_INVAL = -1,     /* bad argument, shape or inconsistent input */
    DPD_E_NOMEM = -2,     /* device allocation failed */
    DPD_E_DEVICE = -3,    /* no usable gfx950 device, or a HIP runtime error */
    DPD_E_UNSTABLE = -4,  /* non-finite state, or a particle moved > half a cell */
    DPD_E_STATE = -5      /* call not valid in the current state */
};

enum {
    DPD_TYPE_FLUID = 0,
    DPD_TYPE_WALL = 1
};

/* params.flags */
enum {
    DPD_FLAG_NO_MASK = 1,  /* test phi for every particle, not only in cells
                              near the interface (results are identical) */
    DPD_FLAG_SPECULAR = 2, /* specular reflection (Sec. I): only the component
                              of the velocity relative to the wall along the
                              normal grad phi / |grad phi| at the crossing
                              position is reversed, in the new velocity and
                              in the displacement of Eq. 17; without it,
                              bounce-back (Sec. II.C) reverses all of it */
    DPD_FLAG_SPH = 4       /* conservative force of Eq. 22-24 (sr, sa, r0r,
                              r0a) instead of a_ij w */
};

typedef struct dpd_ctx dpd_ctx;

/* Periodic box [0, L[0]) x [0, L[1]) x [0, L[2]). */
typedef struct {
    double L[3];
} dpd_box;

/* Particles (Sec. II.A: positions r_i and velocities v_i, Eq. 1-2; Sec. II.C:
 * fluid particles where phi > 0, frozen wall particles where phi <= 0).
 *   n     number of particles, fluid and wall together
 *   pos   n x 3 float32, row-major, each coordinate in [0, L)
 *   vel   n x 3 float32; for a wall particle, the velocity of its solid
 *         (Sec. II.C, moving walls): a solid keeps its shape and phase
 *         field while it moves, e.g. a plate sliding in its own plane; its
 *         wall particles translate by dt v per step and carry v into the
 *         pair forces, and a reflection uses the velocity of the wall
 *         particle nearest to the crossing position (start-of-step walls
 *         of the 27 cells around it, FP32 pair distance, ties to the
 *         smaller gid): v = -v^t + 2 v_wall, Eq. 17 with v^t - v_wall.
 *         Zero rows: resting walls.  |v| dt must stay below half a cell.
 *   type  n int32, DPD_TYPE_FLUID or DPD_TYPE_WALL
 *   gid   n uint32, a permutation of 0..n-1 naming the particle in the
 *         random-number counter and in every getter's row order; NULL means
 *         gid = row index
 *   on_device  nonzero when the four pointers are device memory */
typedef struct {
    int64_t n;
    const float *pos;
    const float *vel;
    const int32_t *type;
    const uint32_t *gid;
    int32_t on_device;
} dpd_particles;

/* Phase field phi(x) on a periodic node-centred grid (Sec. II.B-C): node
 * (i, j, k) sits at (i h[0], j h[1], k h[2]); n[d] h[d] must equal L[d].
 * data holds n[2] x n[1] x n[0] values (x fastest) of dtype 4 (float32) or
 * 8 (float64); -1 is solid, +1 fluid, the interface is phi = 0.  The grid is
 * copied at create; the discrete phi < 0 test runs in the grid's precision. */
typedef struct {
    int32_t n[3];
    double h[3];
    int32_t dtype;
    const void *data;
    int32_t on_device;
} dpd_phi_grid;

/* DPD parameters (Eq. 4-10 and the Groot-Warren integrator).
 *   a       2 x 2 conservative amplitudes a_ij by type, row-major
 *           {a_ff, a_fw, a_wf, a_ww}; a_fw must equal a_wf; a_ww is unused
 *           (wall-wall pairs never interact)
 *   gamma   dissipative coefficient; sigma = sqrt(2 gamma kBT) (Eq. 8)
 *   kBT     temperature
 *   rc      cutoff; the box must hold at least 3 cells of width >= rc per axis
 *   dt      time step (> 0)
 *   lambda  predictor weight of the modified velocity-Verlet (0.65 typical,
 *           0.5 is plain velocity-Verlet)
 *   g       body force per fluid particle
 *   seed    64-bit key of the random numbers
 *   replica replica id entering the random-number counter (< 65536)
 *   flags   DPD_FLAG_*
 *   sr, sa  with DPD_FLAG_SPH: 2 x 2 strengths S^r_ij, S^a_ij by type of the
 *           attractive-repulsive energy of Eq. 22, E = S^r W(r, r0r) -
 *           S^a W(r, r0a), W the cubic spline of Eq. 23 in 3-D with support
 *           r0 (h = r0/2, alpha_3 = 1/pi); the conservative pair force is
 *           -dE/dr along r_i - r_j (Eq. 24), replacing a_ij w; dissipative
 *           and random forces are unchanged.  Symmetric like a.
 *   r0r, r0a  ranges of the repulsive and attractive parts, 0 < r0 <= rc */
typedef struct {
    double a[4];
    double gamma;
    double kBT;
    double rc;
    double dt;
    double lambda;
    double g[3];
    uint64_t seed;
    uint32_t replica;
    int32_t flags;
    double sr[4];
    double sa[4];
    double r0r;
    double r0a;
} dpd_params;

/* Optional device allocator (e.g. PyTorch's caching allocator through the
 * Python binding).  alloc returns device memory of at least `bytes` bytes
 * aligned to 256 bytes, or NULL; free releases it.  Either may be called
 * from any library call of the context, with the context stream. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, void *stream, void *user);
    void *user;
} dpd_allocator;

/* Create a context on the current HIP device (Sec. II: the problem is the box,
 * the particles, a_ij, gamma, kBT, rc, dt, the body force and the phase field).
 * Validates the inputs (DPD_E_INVAL: shapes, non-finite values, box < 3 cells,
 * asymmetric a, dt <= 0, gid not a permutation, a fluid particle with
 * phi < 0, grid not matching the box), copies them to device memory, sorts
 * the frozen wall particles into their cells once, marks the cells next to
 * the interface, and computes the initial forces f(0) with random-number
 * index k = 0.  hip_stream (a hipStream_t, NULL for the null stream) is the
 * stream of every later call.  alloc may be NULL.  On success *out owns the
 * context; on failure *out is NULL. */
int dpd_create(const dpd_box *box, const dpd_particles *particles,
               const dpd_params *params, const dpd_phi_grid *phi,
               const dpd_allocator *alloc, void *hip_stream, dpd_ctx **out);

/* Advance n >= 0 time steps, asynchronously on the context stream.  One step
 * (Sec. II.A and II.C): the modified velocity-Verlet drift and prediction;
 * for particles whose new position has phi < 0, bounce-back with the
 * reflected position of Eq. 17 (or the start position if that is still in
 * the solid) and v = -v^t; a counting-sort cell list of the new positions;
 * the pairwise conservative + dissipative + random force (Eq. 3-10) with the
 * pair-symmetric counter-based random number xi_ij(k); the velocity update. */
int dpd_step(dpd_ctx *ctx, int64_t n);

/* Forces f at the current state (the force carried into the next step, the
 * sum of Eq. 2 plus the body force), written as n x 3 float32 rows in gid
 * order to the device buffer f_out; wall rows are zero. */
int dpd_forces(dpd_ctx *ctx, float *f_out);

/* Current state in gid order, into device buffers; any pointer may be NULL.
 *   pos     n x 3 float32 positions (walls: fixed, or moved with their solid)
 *   vel     n x 3 float32 velocities (walls: their solid's velocity)
 *   events  n int32: the last step's bounce-back code per particle,
 *           0 none, 1 reflected by Eq. 17, 2 returned to the start position
 *   cell_of n int32: cell index (cz * ncy + cy) * ncx + cx of the position,
 *           cx = min(ncx - 1, floor(fl32(x * fl32(ncx / Lx)))) */
int dpd_get_state(dpd_ctx *ctx, float *pos, float *vel, int32_t *events,
                  int32_t *cell_of);

/* Replace the fluid state: pos, vel, force are n x 3 float32 rows in gid
 * order (wall rows are ignored, except that walls of a box with moving walls
 * take their positions from pos; wall velocities never change), k the index of
 * the random numbers the forces were evaluated with.  Host or device memory
 * per on_device.  Positions must lie in [0, L) and satisfy phi >= 0. */
int dpd_set_state(dpd_ctx *ctx, const float *pos, const float *vel,
                  const float *force, uint64_t k, int32_t on_device);

/* Interacting pairs at the current positions, as seen from each fluid
 * particle i: every (gid_i, gid_j) with j != i in the 27 cells around i and
 * r2 = fma(dz, dz, fma(dy, dy, fl(dx^2))) < fl32(rc^2), where dx is the FP32
 * rounding of the exact minimum-image difference x_i - x_j - s L (s the image
 * shift of the neighbour cell; the coordinate in the last cell is lowered by
 * L, exactly, before the one rounding subtraction).  Fluid-fluid pairs appear in both
 * orders, fluid-wall pairs once.  pairs is a device buffer of cap x 2 uint32
 * (unordered); *count (host) receives the total, which may exceed cap (only
 * cap pairs are written then).  Synchronises the stream. */
int dpd_neighbor_pairs(dpd_ctx *ctx, uint32_t *pairs, int64_t cap, int64_t *count);

/* Binned fluid observables along `axis` (0, 1, 2) in nbins equal bins
 * (Sec. III.A: density, temperature and stream velocity per bin), into the
 * device buffer out of nbins x 5 float64: count, sum v_x, sum v_y, sum v_z,
 * sum |v|^2. */
int dpd_profile(dpd_ctx *ctx, int32_t axis, int32_t nbins, double *out);

/* Counters into host out[10]: steps since create, k, bounce-backs (code 1)
 * and returns to start (code 2) since create, n_fluid, n_wall, cells, grid
 * cubes with a negative corner (the only cubes where phi can be < 0), fluid
 * particles now inside such cubes (those that interpolate phi in a step),
 * displacements above half a cell since create.  Synchronises the stream. */
int dpd_counters(dpd_ctx *ctx, int64_t *out);

/* Per-kernel timing with HIP events on the context stream.  enable = 1
 * starts recording (dpd_step then times each kernel launch), 0 stops.
 * When out is not NULL it receives, for the kernels named by
 * dpd_kernel_name(0..DPD_NUM_KERNELS-1), the summed milliseconds in out_ms
 * and the number of timed launches in out_launches ("scatter" also writes
 * the wall part of the merged cell runs; "pair_codes" writes the coarse
 * position codes of the merged runs that the pair kernel's candidate
 * pre-test reads; "step_persistent" is the one launch of a step under
 * dpd_use_persistent, which then replaces the six step kernels).
 * Synchronises. */
#define DPD_NUM_KERNELS 9
int dpd_kernel_times(dpd_ctx *ctx, int32_t enable, double *out_ms, int64_t *out_launches);
const char *dpd_kernel_name(int32_t i);

/* ---- Batches of independent boxes ----
 * A batch context holds nbox independent systems ("replicas"), each one the
 * whole problem of dpd_create (Sec. II) with its own box, particles, phase
 * field and parameters; a step advances all of them with the same kernels
 * (one launch per kernel for the whole batch).  Replica r of a batch gives
 * bit-identical results to a plain context created from the same inputs.
 * Every box shares the random-number index k; boxes that run the same
 * geometry and seed should differ in params.replica, which enters the
 * counter (Eq. 7).  All phi grids of a batch must have one dtype and all
 * params one flags value.  The arrays boxes, particles, params, grids hold
 * nbox entries each.  dpd_create is dpd_batch_create with nbox = 1. */
int dpd_batch_create(int32_t nbox, const dpd_box *boxes, const dpd_particles *particles,
                     const dpd_params *params, const dpd_phi_grid *grids,
                     const dpd_allocator *alloc, void *hip_stream, dpd_ctx **out);

/* Number of boxes of the context (>= 1), or DPD_E_INVAL for NULL. */
int dpd_replica_count(const dpd_ctx *ctx);

/* Per-box getters and setter: as dpd_forces, dpd_get_state, dpd_set_state,
 * dpd_neighbor_pairs and dpd_profile, for box r (0 <= r < count) with that
 * box's n and gid numbering.  The plain names act on box 0.  set_state sets
 * the context-wide k. */
int dpd_replica_forces(dpd_ctx *ctx, int32_t r, float *f_out);
int dpd_replica_state(dpd_ctx *ctx, int32_t r, float *pos, float *vel, int32_t *events,
                      int32_t *cell_of);
int dpd_replica_set_state(dpd_ctx *ctx, int32_t r, const float *pos, const float *vel,
                          const float *force, uint64_t k, int32_t on_device);
int dpd_replica_pairs(dpd_ctx *ctx, int32_t r, uint32_t *pairs, int64_t cap, int64_t *count);
int dpd_replica_profile(dpd_ctx *ctx, int32_t r, int32_t axis, int32_t nbins, double *out);

/* enable != 0: dpd_step replays one captured HIP graph per step (the launch
 * sequence of a step, captured on first use on a private stream and replayed
 * on the context stream; the random-number index k lives on the device and is
 * advanced inside the graph, so replays draw fresh numbers).  Results are
 * bit-identical to direct launches.  Per-kernel timing, when enabled, uses
 * direct launches.  A captured graph is dropped by set_state and autotune. */
int dpd_use_graph(dpd_ctx *ctx, int32_t enable);

/* enable = 1: run each step as one persistent launch (plus a one-block
 * kernel that clears its counters and advances k) instead of one launch per
 * phase.  Work items (the integrate tiles, the cell-list scan chunks, scatter
 * and per-cell sort ranges, and 256-particle pair-force tiles of every box)
 * are taken in queue order from one device counter; an item of box r waits
 * for the items of the previous phase of box r through per-box arrival
 * counters (each wait bounded; a wait that reaches its bound is reported as
 * DPD_E_DEVICE at the next synchronising call).  Results are bit-identical to
 * the per-phase launches, and it combines with dpd_use_graph.  The
 * persistent launch integrates at most 2 particles per thread, so a context
 * at 4 is set to 2 (see dpd_autotune).  DPD_E_INVAL for
 * contexts with moving walls or boxes on the LDS-staged brick pair kernel;
 * enable = 0 returns to the per-phase launches and keeps the shapes. */
int dpd_use_persistent(dpd_ctx *ctx, int32_t enable);

/* Choose the launch shapes of the integrate kernel (particles per thread:
 * P or 1, with P the context's default, 4 for contexts of at least 2^20
 * fluid particles without moving walls or specular reflection and 2
 * otherwise, and 2 under dpd_use_persistent) and of the pair-force kernel
 * (work-group size, 128 or 256; default 256) by
 * timing `steps` steps of each of the four combinations from the current
 * state: one untimed round of all four, then two timed rounds in opposite
 * orders, each combination keeping its faster time (the first trials of a
 * run are slower, which would favour the last combination tried); the
 * state, k and the step counter are restored after each trial, so
 * the context is left as it was apart from the shapes (results do not depend
 * on them).  If the environment variable DPD_TUNE_CACHE names a file, a
 * choice recorded there for the same device and sizes is used without trials
 * and new choices are appended.  shape_out (host int32[2], may be NULL)
 * receives {particles per thread, work-group size}; ms_out (host double[4],
 * may be NULL) the ms per step of {P/256, 1/256, P/128, 1/128}, -1 when not
 * timed.  Synchronises. */
int dpd_autotune(dpd_ctx *ctx, int32_t steps, int32_t *shape_out, double *ms_out);

/* Replace the parameters of box r (every field of dpd_params; rc and flags
 * must keep their create-time values, since rc fixes the cell grid).  The
 * carried force is not recomputed: the next step uses the new parameters
 * from its force evaluation on.  Invalidates a recorded window. */
int dpd_set_params(dpd_ctx *ctx, int32_t r, const dpd_params *params);

/* Replace the phase-field values of box r (same node count and dtype as at
 * create; host or device memory per on_device) and rebuild the mask of grid
 * cubes next to the interface.  DPD_E_INVAL, with the old grid kept, when a
 * value is not finite or a fluid particle would sit at phi < 0.
 * Invalidates a recorded window. */
int dpd_set_phi(dpd_ctx *ctx, int32_t r, const void *data, int32_t on_device);

/* ---- Adjoint form (single-box contexts) ----
 * A window of `steps` steps from the current positions and velocities, with
 * the carried force first recomputed at them with the current parameters
 * and force index k0 = k: f0 = F(r0, v0; k0) + g (as at create).  The
 * observable is the window-mean stream velocity along x per bin of `axis`
 * (Sec. III.A's velocity profile): profile[b] = (sum over steps t = 1..steps
 * and fluid particles i in bin b after step t of v_x,i) / N_b, with N_b the
 * number of such terms and the bin the FP32 decision
 * clamp(floor(fl(x_axis * fl32(nbins / L_axis))), 0, nbins - 1).
 * profile (device, nbins float64) and counts (device, nbins int64: N_b) may
 * be NULL.  A checkpoint of the fluid state is stored every ckpt steps
 * (1 <= ckpt <= steps, nbins <= 1024); the context ends at the window's last
 * state.  DPD_E_STATE for a batch context; DPD_E_INVAL for moving walls,
 * DPD_FLAG_SPECULAR or DPD_FLAG_SPH (the adjoint covers the a_ij w force and
 * resting walls with bounce-back).
 *
 * dpd_backward: gradients of a loss L(profile) from dL_dprofile (device,
 * nbins float64) by the hand-written adjoint of every step of the window
 * (pair force of Eq. 3-10, the Groot-Warren update and the bounce-back of
 * Eq. 16-17 with the recorded events held fixed, and the starting force),
 * recomputing each ckpt-step segment from its checkpoint.  The bins, pair
 * sets and events are those of the forward window.  grads (host, 6 float64)
 * receives dL/d{a_ff, a_fw, gamma, g_x, g_y, g_z} (gamma through both the
 * dissipative amplitude and sigma = sqrt(2 gamma kBT); the sigma path is
 * omitted where sigma = 0); dL_dphi (device, grid nodes float64 in the
 * grid's layout, may be NULL) receives dL/d(phi node values), nonzero only
 * at the nodes of cubes where a bounce-back of code 1 started or ended.
 * The context's state, k and counters are unchanged.  DPD_E_STATE without a
 * recorded window or after dpd_set_params / dpd_set_phi / dpd_set_state. */
int dpd_window_forward(dpd_ctx *ctx, int32_t steps, int32_t ckpt, int32_t axis,
                       int32_t nbins, double *profile, int64_t *counts);
int dpd_backward(dpd_ctx *ctx, const double *dL_dprofile, double *grads,
                 double *dL_dphi);

/* The trajectory and decisions of the recorded window, for references that
 * hold its discrete decisions fixed (the window as a smooth function of
 * the parameters, Sec. II.C's events frozen) and linearise it around the
 * GPU's own trajectory: the window's steps are recomputed from its
 * checkpoints exactly as dpd_backward recomputes them.  State s of every
 * particle in gid order goes to pos_log, vel_log and frc_log (device,
 * (steps + 1) x n x 3 float32 each): s = 0 is the window's start with its
 * refreshed force f0, s = t + 1 the state after step t, whose positions are
 * those on which step t's cell, pair and bin decisions were taken.  The
 * event codes of step t go to ev_log[t][n] (device, steps x n int32).  Any
 * pointer may be NULL.  Walls: their positions and velocities, zero forces
 * and events.  The context's state, k and counters are unchanged.
 * Synchronises.  DPD_E_STATE without a recorded window or after
 * dpd_set_params / dpd_set_phi / dpd_set_state. */
int dpd_window_trace(dpd_ctx *ctx, float *pos_log, float *vel_log, float *frc_log,
                     int32_t *ev_log);

/* Wait for the context stream and return any latched device error. */
int dpd_sync(dpd_ctx *ctx);

/* Message of the last failure of ctx (or of the last failed create when ctx
 * is NULL); never NULL. */
const char *dpd_last_error(const dpd_ctx *ctx);

/* Release the context and its device memory (synchronises first). */
void dpd_destroy(dpd_ctx *ctx);

/* The pair random numbers of Eq. 7 exactly as the force kernel draws them:
 * for pair m, Philox4x32-10 (Salmon et al., SC'11) with counter
 * (min(gi, gj), max(gi, gj), k & 0xFFFFFFFF, (k >> 32 & 0xFFFF) | replica << 16)
 * and key (seed & 0xFFFFFFFF, seed >> 32); words (device, n x 4 uint32) gets
 * the four output words and xi (device, n float32) the Gaussian
 * sqrt(-2 ln u1) cos(2 pi u2) with u1 = ((w0 >> 9) + 1/2) 2^-23 and
 * u2 = (w1 >> 9) 2^-23.  Either output may be NULL.  gi, gj are device
 * arrays of n uint32.  Runs on hip_stream; for tests and diagnostics. */
int dpd_pair_random(uint64_t seed, uint64_t k, uint32_t replica, const uint32_t *gi,
                    const uint32_t *gj, int64_t n, uint32_t *words, float *xi,
                    void *hip_stream);

/* Device-to-device copy of `bytes` bytes by a plain streaming kernel (no
 * library call), on hip_stream: the reference kernel of known traffic that
 * hardware byte counters are calibrated against. */
int dpd_copy_probe(void *dst, const void *src, size_t bytes, void *hip_stream);

/* VALU calibration kernel of known instruction count, on hip_stream: `waves`
 * wavefronts (a multiple of 4; 256 threads per block) each execute exactly
 * iters x 64 VALU instructions of one kind on eight independent register
 * chains: kind 0 v_fmac_f32, 1 v_mad_u64_u32 (the 32 x 32 -> 64-bit
 * multiply of Philox4x32-10), 2 v_xor_b32, 3 v_log_f32; each thread then
 * writes one float to out (device, waves x 64 floats).  The reference for
 * the issue rate of the vector ALU, as dpd_copy_probe is for HBM bytes.
 * DPD_E_INVAL for a bad kind, waves <= 0, iters < 0 or out NULL. */
int dpd_valu_probe(int32_t kind, int64_t waves, int32_t iters, float *out, void *hip_stream);

/* ---- Snapshots (checkpoint and restart of a run) ----
 * The complete dynamic state of a context: every box's particles in the
 * library's internal cell-sorted order (positions with gids, velocities
 * with the last step's event codes, the forces carried into the next step,
 * wall positions and velocities), the force evaluation index k, the step
 * and event counters.  A context restored from a snapshot continues
 * bit-identically to the one it was taken from (dpd_set_state, which takes
 * gid-ordered rows, re-sorts and so continues only to within rounding).
 * Parameters, phase fields and launch shapes are the context's own and are
 * not in the snapshot. */

/* Bytes of a snapshot of ctx (a host buffer of this size holds one), or
 * DPD_E_INVAL for NULL. */
int64_t dpd_snapshot_size(const dpd_ctx *ctx);

/* dir 0: write ctx's state into blob (host memory, dpd_snapshot_size bytes,
 * owned by the caller); synchronises the stream first.  dir 1: restore
 * ctx's state from blob; the context must have been created from the same
 * boxes (same particle counts, cells and phase-field grids, same resting
 * wall particles), else DPD_E_INVAL and the context is unchanged.  Captured
 * step graphs are dropped on restore.  Synchronises. */
int dpd_snapshot_io(dpd_ctx *ctx, int32_t dir, void *blob);

/* ---- Phase-field relaxation (Sec. II.B, Eq. 13-15) ----
 * Integrates d phi / d t' = lap' phi + phi (1 - phi^2) - kappa |grad' phi|
 * with kappa = div'(grad' phi / |grad' phi|) and grad' = eps grad (Eq. 15)
 * in the pseudo time t' by `iters` explicit Euler steps of length dtau,
 * from the field in phi (a step function -1 solid / +1 fluid in the
 * paper), on the periodic node-centred grid of dpd_phi_grid (n[2] x n[1] x
 * n[0] values, x fastest, node (i, j, k) at (i h[0], j h[1], k h[2])).
 * Differences: the compact 7-point Laplacian; central differences for
 * grad' phi and for the divergence of n = grad' phi / max(|grad' phi|,
 * 0.01), the unit normal wherever |grad' phi| >= 0.01, going linearly to
 * zero where phi is flat.
 *   phi    device, dtype 4 (float32) or 8 (float64) values; input, and the
 *          field after the last step on return
 *   work   device, n[0] n[1] n[2] + 1 values of the same dtype, owned by
 *          the caller, overwritten (ping-pong buffer and one reduction word)
 *   eps    interface coefficient of Eq. 12 (phi = tanh(x / (sqrt(2) eps))
 *          at a plane, Eq. 14); > 0
 *   dtau   pseudo-time step, 0 < dtau <= 1 / (2 sum_a (eps / h[a])^2), the
 *          explicit-Euler bound of the diffusion part
 *   iters  >= 0 steps
 *   residual  host, may be NULL: receives max over nodes of |d phi / d t'|
 *          in the last step (0 when iters = 0); the call then synchronises
 *          hip_stream, otherwise it only enqueues work on it.
 * Needs n[a] >= 1 and n[0] n[1] < 2^31.  DPD_E_INVAL for bad arguments,
 * DPD_E_DEVICE for a HIP error (dpd_last_error(NULL) says which). */
int dpd_phi_relax(void *phi, void *work, int32_t dtype, const int32_t n[3], const double h[3],
                  double eps, double dtau, int32_t iters, double *residual, void *hip_stream);

/* The relaxation of dpd_phi_relax with no workspace argument and no device
 * allocation, for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc).  The
 * ping-pong buffer and the residual word live in a static device array of
 * the library, 64 MiB + 256 bytes, held by each GPU the library runs on
 * until the process ends; grids of at most 16,777,216 float32 or 8,388,608
 * float64 nodes, larger ones DPD_E_INVAL (use dpd_phi_relax).  Results are
 * identical to dpd_phi_relax's.  All calls on one GPU share that array:
 * calls that overlap on one GPU (other streams, other threads) race, and
 * must be serialised by the caller.  Other arguments, errors and the
 * residual as for dpd_phi_relax. */
int dpd_phi_relax_static(void *phi, int32_t dtype, const int32_t n[3], const double h[3],
                         double eps, double dtau, int32_t iters, double *residual,
                         void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* DPD_H */
