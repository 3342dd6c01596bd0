// Host-side launchers of the DPD kernels (defined in kernels.hip).  All take
// the stream to launch on and return the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace dpd {

// Number of scan blocks for n cells (each block scans kScanChunk counts).
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;
// Spare entries after the merged cell runs: the pair kernel reads a few run
// entries past a run's end (and discards them) instead of branching.
constexpr int kIdxSlack = 8;
// Spare entries after the run starts: the pair kernel reads them four at a time.
constexpr int kStartSlack = 4;
inline int scan_blocks(int64_t n) { return (int)((n + kScanChunk - 1) / kScanChunk); }

// Upload: pack host-order rows of one particle class into float4 arrays.
hipError_t launch_pack(hipStream_t s, int64_t n, const float *pos, const float *vel,
                       const uint32_t *gid, const int64_t *rows, float4 *pos4, float4 *vel4,
                       float4 *vt4, float4 *frc4);

// Cell of each position (float4 x,y,z) and its rank within the cell by an
// atomic counter: counting-sort pass 1.
hipError_t launch_bin(hipStream_t s, const KGeom &G, int64_t cell_off, int64_t n,
                      const float4 *pos4, int32_t *cell_of, int32_t *rank_of, int32_t *count);

// Exclusive scan of count[0..ncell) into start[0..ncell] (start[ncell] =
// total), count reset to 0, in two launches: per-block sums, then the
// per-block scans, each block adding the sum of the block sums before it.
hipError_t launch_scan_reduce(hipStream_t s, int64_t ncell, const int32_t *count, int32_t *bsum);
hipError_t launch_scan_down(hipStream_t s, int64_t ncell, int32_t *count, int32_t *start,
                            const int32_t *bsum, const int32_t *wstart, int32_t *start_all,
                            int32_t *fluid_off);

// idx[start[cell_of[p]] + rank_of[p]] = p, then each cell's run sorted by p
// (by the gid bits of key4[p].w when key4 is given), and copied to the fluid
// part of the merged run when idx_all is given.  The scatter also writes the
// wall part of the merged runs when idx_all is given (walls cell-sorted,
// stored at index n + w) and, with dk, advances the force evaluation index.
hipError_t launch_scatter(hipStream_t s, int64_t n, const int32_t *cell_of,
                          const int32_t *rank_of, const int32_t *start, int32_t *idx,
                          int64_t nw = 0, const int32_t *wcell = nullptr,
                          const int32_t *wstart = nullptr, const int32_t *start_all = nullptr,
                          int32_t *idx_all = nullptr, unsigned long long *dk = nullptr);
hipError_t launch_sort_cells(hipStream_t s, int64_t ncell, const int32_t *start, int32_t *idx,
                             const float4 *key4, const int32_t *fluid_off, int32_t *idx_all);
// The walls' per-cell sort by storage index, writing also the global cell of
// every sorted wall position to cell_out.
hipError_t launch_sort_wall_cells(hipStream_t s, int64_t ncell, const int32_t *start,
                                  int32_t *idx, int32_t *cell_out);
// Coarse position codes of the merged runs, cq[t] from pos4[idx_all[t]] for
// t < n (one word per entry), which the pair kernel's candidate pre-test
// reads; n = NF + NW, after the scatter and sort.
hipError_t launch_quant_runs(hipStream_t s, int64_t n, const int32_t *idx_all,
                             const float4 *pos4, uint32_t *cq);


// Write the pad entry (far-away position, zero velocity) at pos4[0], vt4[0];
// with slack given, the kIdxSlack spare run entries name it.
hipError_t launch_set_pad(hipStream_t s, float4 *pos4, float4 *vt4, int32_t *slack, int32_t pad);

// Cell index of each position.
hipError_t launch_cells(hipStream_t s, const KGeom &G, int64_t cell_off, int64_t n,
                        const float4 *pos4, int32_t *cell);

// out[s] = in[idx[s]] for up to three float4 arrays (NULL skipped).
hipError_t launch_permute(hipStream_t s, int64_t n, const int32_t *idx, const float4 *a_in,
                          float4 *a_out, const float4 *b_in, float4 *b_out, const float4 *c_in,
                          float4 *c_out);

// Near-interface mask: one bit per grid cube, set when a corner is negative
// (nwords = ceil(cubes / 32)).
hipError_t launch_cube_mask(hipStream_t s, const KGeom &G, const void *grid, int grid_f64,
                            int64_t nwords, uint32_t *bits);

// Count fluid particles whose grid cube is flagged into *out (added).
hipError_t launch_count_flagged(hipStream_t s, const KGeom &G, int grid_f64, int64_t nf,
                                const float4 *pos4, const uint32_t *bits,
                                unsigned long long *out);

// Count non-finite grid values (create-time validation).
hipError_t launch_check_grid(hipStream_t s, const void *grid, int grid_f64, int64_t count,
                             Status *st);

// Count fluid particles with phi < 0 (create-time validation).
hipError_t launch_check_phi(hipStream_t s, const KGeom &G, const void *grid, int grid_f64,
                            int64_t n, const float4 *pos4, Status *st);

// One launch for a whole step of a batch (k_step_persistent): work items of
// the six phases in queue order with per-box, per-phase arrival counters,
// preceded by a one-block kernel that clears the counters and advances k.
// Arguments of the persistent step, in device memory.
struct PArgs {
  const Box *boxes;
  const PItem *items;
  int nitems;
  int spin_limit;
  const int32_t *need;     // items per (box, phase)
  int32_t *arrive;         // arrivals per (box, phase), zeroed before the launch
  int32_t *head;           // queue counter, zeroed before the launch
  const Tile *itiles, *ftiles;
  float4 *pos4;
  const float4 *vel4, *frc4;
  float4 *vt4;
  int32_t *cell_of, *rank_of, *count;
  const uint32_t *bits;
  int use_mask;
  const void *quad;
  Status *st;
  int64_t NF, NW;
  const int32_t *wcstart, *wcell;
  int32_t *cstart, *bsum, *start_all, *fluid_off, *idx, *idx_all;
  uint32_t *cq;
  int32_t pad, ncell_all;
  float4 *pos_out, *vel_out, *frc_out;
  const unsigned long long *dk;
};
hipError_t launch_step_persistent(hipStream_t s, const PArgs *args, int nitems, int blocks,
                                  int32_t *arrive, int narrive, int32_t *head,
                                  unsigned long long *dk, int grid_f64, int ppt, int reflect,
                                  int sph);
// Resident blocks per CU of the instance the launch would run, or -1.
int persistent_blocks_per_cu(int ppt, int grid_f64, int reflect, int sph);

// The face layout of one box's phase field (PhiQuad in device.h): 16 bytes
// per node for a float32 grid, 32 for float64, into quad.
hipError_t launch_build_quad(hipStream_t s, const KGeom &G, const void *grid, int grid_f64,
                             void *quad);

// Fused drift + predicted velocity + phi test + reflection + binning, over
// tiles of up to ppt x 256 particles (ppt 1, 2 or 4); quad is the base of the
// concatenated phase fields in the face layout, bits of the concatenated
// cube masks.  reflect = 1
// (some box has moving walls or specular reflection) runs the instance with
// those forms: boxes with moving walls look up the solid's velocity among the
// walls (entries NF + w of pos4 and vt4, runs wcstart over the global cells).
hipError_t launch_integrate(hipStream_t s, int ppt, const Box *boxes, const Tile *tiles,
                            int ntiles, float4 *pos4, const float4 *vel4, const float4 *frc4,
                            float4 *vt4, int32_t *cell_of, int32_t *rank_of, int32_t *count,
                            const uint32_t *bits, int use_mask, const void *quad, int grid_f64,
                            Status *st, int64_t NF, const int32_t *wcstart, int reflect);

// Walls of one box from walls_in/vt_in into walls_out/vt_out, advanced by
// dt v (decision-form drift, zero force) when move is set, and binned into
// cells of offset cell_off (cell_of, rank_of, count as launch_bin).
hipError_t launch_wall_move_bin(hipStream_t s, const KGeom &G, float hdt, float dt, int move,
                                int64_t cell_off, int64_t nw, const float4 *walls_in,
                                const float4 *vt_in, float4 *walls_out, float4 *vt_out,
                                int32_t *cell_of, int32_t *rank_of, int32_t *count);

// Wall positions replaced from gid-ordered float32 rows (device memory).
hipError_t launch_import_walls(hipStream_t s, int64_t nw, float4 *walls, const float *pos);

// Pair forces (Eq. 3-10) + body force + velocity update over tiles of up to
// `block` (128 or 256) fluid slots, writing the state in cell-sorted slot
// order.  pos4 and vt4 hold NF fluid entries, the walls and the pad entry
// (index pad).  init = 1: forces only (velocities unchanged).
hipError_t launch_force(hipStream_t s, int block, const Box *boxes, const Tile *tiles,
                        int ntiles, int64_t NF, int32_t pad, int32_t ncell_all, int init,
                        const float4 *pos4, const float4 *vt4, const float4 *vel4,
                        const float4 *frc4, const int32_t *idx, const int32_t *idx_all,
                        const int32_t *start_all, const uint32_t *cq,
                        float4 *pos_out, float4 *vel_out, float4 *frc_out,
                        const unsigned long long *dk, Status *st, int sph);

// The same pair forces, body force and velocity update for the boxes cut
// into bricks: one block per brick stages the brick's cells and a one-cell
// halo in LDS (force_brick.hip).  cstart: fluid slot start of each cell;
// fluid_off: start of each cell's fluid part in the merged run.
hipError_t launch_force_brick(hipStream_t s, const Box *boxes, const Brick *bricks, int nbricks,
                              int64_t NF, int32_t pad, int init, const float4 *pos4,
                              const float4 *vt4, const float4 *vel4, const float4 *frc4,
                              const int32_t *idx_all, const int32_t *start_all,
                              const int32_t *fluid_off, const int32_t *cstart, float4 *pos_out,
                              float4 *vel_out, float4 *frc_out, const unsigned long long *dk,
                              Status *st, int sph);

// Interacting pairs (gid_i, gid_j) from each fluid particle of one box
// (slots [first, first + nf), cells from cell_off).
hipError_t launch_pairs(hipStream_t s, const KGeom &G, const KParams &P, int64_t cell_off,
                        int64_t first, int64_t nf, const float4 *pos4, const int32_t *idx,
                        const int32_t *idx_all, const int32_t *start_all, uint32_t *pairs,
                        int64_t cap, unsigned long long *counter);

// Random numbers of given pairs: Philox words (n x 4) and xi (n), either NULL.
hipError_t launch_pair_random(hipStream_t s, uint64_t seed, uint64_t k, uint32_t replica,
                              const uint32_t *gi, const uint32_t *gj, int64_t n, uint32_t *words,
                              float *xi);

// Export rows by gid.
hipError_t launch_export(hipStream_t s, const KGeom &G, int64_t n, const float4 *pos4,
                         const float4 *vel4, const float4 *frc4, int wall, float *pos,
                         float *vel, float *frc, int32_t *events, int32_t *cell_of);

// Import fluid rows by gid (set_state): pos4[s] = (pos[gid], gid), ...
hipError_t launch_import(hipStream_t s, int64_t nf, float4 *pos4, float4 *vel4, float4 *frc4,
                         const float *pos, const float *vel, const float *frc);

// Fluid profile along an axis: count, sum vx, vy, vz, |v|^2 per bin.
hipError_t launch_profile(hipStream_t s, const KGeom &G, int64_t nf, const float4 *pos4,
                          const float4 *vel4, int axis, int nbins, double *out);

hipError_t launch_fill_zero(hipStream_t s, void *p, size_t bytes);

// One explicit Euler step of the phase-field relaxation (Eq. 15) from src to
// dst (f64: double, else float; n[3] nodes, x fastest; n[0] * n[1] must fit
// in int32).  coef = {eps^2/h_x^2, eps^2/h_y^2, eps^2/h_z^2, eps/(2 h_x),
// eps/(2 h_y), eps/(2 h_z), delta^2, dtau}.  res (device, one word of the
// element size, zeroed by the caller) receives max |rhs| as ordered bits,
// or null.
hipError_t launch_phi_relax(hipStream_t s, int f64, const void *src, void *dst,
                            const int32_t n[3], const double coef[8], void *res);
int64_t phi_relax_blocks(const int32_t n[3]);
hipError_t launch_copy(hipStream_t s, void *dst, const void *src, size_t bytes);

// ---- adjoint form (adjoint.hip) ----
constexpr int kMaxBins = 1024;

// Window observable of one box: per bin (decision form
// clamp(floor(fl(x_axis * scale)), 0, nbins - 1)) the sum of v_x and the
// count, added to sums / counts.
hipError_t launch_obs(hipStream_t s, int64_t nf, const float4 *pos4, const float4 *vel4,
                      int axis, int nbins, float scale, double *sums,
                      unsigned long long *counts);
hipError_t launch_obs_final(hipStream_t s, int nbins, const double *sums,
                            const unsigned long long *counts, double *profile,
                            int64_t *counts_out);
hipError_t launch_loss_weights(hipStream_t s, int nbins, const double *dldp,
                               const unsigned long long *counts, float *lw);
hipError_t launch_vt_from_v(hipStream_t s, int64_t nf, const float4 *vel4, float4 *vt4);
hipError_t launch_set_u64(hipStream_t s, unsigned long long *p, unsigned long long v);

int adj_prep_blocks(int64_t nf);
hipError_t launch_adj_prep(hipStream_t s, const Box *boxes, int64_t nf, int initial,
                           const int32_t *idx, const float4 *pos4, const float4 *vt4,
                           const float4 *rb_s, const float4 *vb_s, const float4 *fb_s,
                           const float *lw, int axis, int nbins, float scale, float4 *rn,
                           float4 *vn, float4 *fbar, double *part_g);
int force_vjp_blocks(int ntiles);
hipError_t launch_force_vjp(hipStream_t s, int block, const Box *boxes, const Tile *tiles,
                            int ntiles, int64_t NF, int32_t pad, const float4 *pos4,
                            const float4 *vt4, const int32_t *idx, const int32_t *idx_all,
                            const int32_t *start_all, const float4 *fbar, const float4 *rn,
                            float4 *rt_out, float4 *vt_out, const unsigned long long *dk0,
                            unsigned long long koff, double *part);
hipError_t launch_integrate_vjp(hipStream_t s, const Box *boxes, int64_t nf, const float4 *pos_t,
                                const float4 *vel_t, const float4 *frc_t, const float4 *vt4,
                                const float4 *rt, const float4 *vtb, const float4 *vn,
                                const void *grid, int grid_f64, double *dphi, float4 *rb_out,
                                float4 *vb_out, float4 *fb_out);
hipError_t launch_reduce_partials(hipStream_t s, int nb_f, const double *part_f, int nb_g,
                                  const double *part_g, double *out);

// Argument checks of dpd_phi_relax (DPD_OK or a DPD_E_* code, with the
// message kept for dpd_last_error(NULL)), and the relaxation itself with
// `work` as the ping-pong buffer (n[0] n[1] n[2] values) followed by the
// residual word.  Defined with the C ABI in api.hip.
int phi_relax_check(const void *phi, int32_t dtype, const int32_t n[3], const double h[3],
                    double eps, double dtau, int32_t iters);
int phi_relax_run(void *phi, void *work, int32_t dtype, const int32_t n[3], const double h[3],
                  double eps, double dtau, int32_t iters, double *residual, void *hip_stream);
// Record a failure message for dpd_last_error(NULL); returns code.
int fail_global(int code, const char *msg);

// VALU calibration: `waves` wavefronts each run `iters` x 64 VALU
// instructions of one kind (0: v_fmac_f32, 1: v_mad_u64_u32, 2: v_xor_b32,
// 3: v_log_f32) on independent registers; out receives one float per thread.
hipError_t launch_valu_probe(hipStream_t s, int kind, int64_t waves, int iters, float *out);

}  // namespace dpd
