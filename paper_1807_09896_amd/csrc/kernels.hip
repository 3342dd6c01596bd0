// Kernels of one DPD time step with phase-field bounce-back on gfx950.
//
// Per-particle state lives in float4 arrays (16-byte loads and stores):
//   pos4 = (x, y, z, gid bits)   vel4 = (v, last event code bits)
//   frc4 = (f, 0)                vt4  = (predicted velocity, event code bits)
// Fluid particles are kept in cell-sorted order: the force kernel writes the
// state of slot s (the s-th particle of the cell list) to slot s of the next
// buffers, so each step's integrate kernel streams a nearly sorted array and
// the force kernel's gathers of neighbour cells hit consecutive addresses.
// Frozen wall particles are sorted by cell once, at create, and stored after
// the fluid in the position and predicted-velocity arrays (index nf + w, with
// zero predicted velocity), so that one merged list per cell (walls first,
// then fluid) serves the neighbour search without a fluid/wall branch.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "kernels.h"

namespace dpd {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int block = kBlock) {
  return (unsigned)((n + block - 1) / block);
}

// ---------------------------------------------------------------------------
// Upload and bookkeeping
// ---------------------------------------------------------------------------
__global__ void k_pack(int64_t n, const float *__restrict__ pos, const float *__restrict__ vel,
                       const uint32_t *__restrict__ gid, const int64_t *__restrict__ rows,
                       float4 *pos4, float4 *vel4, float4 *vt4, float4 *frc4) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t r = rows[p];
  const uint32_t g = gid ? gid[r] : (uint32_t)r;
  pos4[p] = make_float4(pos[3 * r], pos[3 * r + 1], pos[3 * r + 2], __uint_as_float(g));
  if (vel4) {
    const float4 v = make_float4(vel[3 * r], vel[3 * r + 1], vel[3 * r + 2], 0.0f);
    vel4[p] = v;
    if (vt4) vt4[p] = v;
  }
  if (frc4) frc4[p] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_fill_zero(uint32_t *p, size_t nwords) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0u;
}

// Plain streaming copy, 16 bytes per thread per iteration (the traffic
// reference for hardware byte counters).
__global__ void k_copy16(float4 *__restrict__ dst, const float4 *__restrict__ src, size_t n16) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) dst[i] = src[i];
}

// VALU calibration: every thread runs `iters` x 64 VALU instructions of one
// kind on 8 independent register chains (inline assembly, so the count is
// exact), then stores one value so that nothing is dead.  Kinds: 0
// v_fmac_f32, 1 v_mad_u64_u32 (the 32 x 32 -> 64-bit multiply of Philox),
// 2 v_xor_b32, 3 v_log_f32 (a transcendental).
#define DPD_PROBE8(INS) INS(0) INS(1) INS(2) INS(3) INS(4) INS(5) INS(6) INS(7)
template <int KIND>
__global__ __launch_bounds__(256) void k_valu_probe(int iters, float *out) {
  const uint32_t t = threadIdx.x + blockIdx.x * blockDim.x;
  float f[8];
  uint32_t u[8];
  uint64_t w[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    f[k] = (float)(t + k) * 1e-3f + 1.0f;
    u[k] = t * 2654435761u + (uint32_t)k;
    w[k] = (uint64_t)u[k] << 7;
  }
  const float fb = 1.0000001f, fc = 1e-7f;
  const uint32_t ub = 0x9E3779B9u;
  uint64_t cy = 0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int rep = 0; rep < 8; ++rep) {
      if (KIND == 0) {
#define DPD_FMA(k) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(f[k]) : "v"(fb), "v"(fc));
        DPD_PROBE8(DPD_FMA)
#undef DPD_FMA
      } else if (KIND == 1) {
#define DPD_MAD(k) asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(w[k]), "=s"(cy) : "v"(u[k]), "v"(ub));
        DPD_PROBE8(DPD_MAD)
#undef DPD_MAD
      } else if (KIND == 2) {
#define DPD_XOR(k) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(u[k]) : "v"(ub));
        DPD_PROBE8(DPD_XOR)
#undef DPD_XOR
      } else {
#define DPD_LOG(k) asm volatile("v_log_f32 %0, %0" : "+v"(f[k]));
        DPD_PROBE8(DPD_LOG)
#undef DPD_LOG
      }
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) acc += f[k] + (float)u[k] + (float)(uint32_t)w[k];
  out[t] = acc + (float)(uint32_t)cy;
}
#undef DPD_PROBE8

__global__ void k_copy1(uint8_t *__restrict__ dst, const uint8_t *__restrict__ src, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Counting sort into cells
// ---------------------------------------------------------------------------
// Run structure of equal cells across a wavefront (cell < 0: inactive lane).
struct RunInfo {
  unsigned long long heads;
  int len;     // run length, for head lanes
  bool head;
};

__device__ __forceinline__ RunInfo wave_runs(int cell) {
  const int lane = (int)__lane_id();
  const int prev = __shfl_up(cell, 1, 64);
  RunInfo r;
  r.head = lane == 0 || prev != cell;
  r.heads = __ballot(r.head);
  const unsigned long long after = lane == 63 ? 0ull : (r.heads >> (lane + 1));
  r.len = after ? __ffsll((long long)after) : 64 - lane;
  return r;
}

__device__ __forceinline__ int wave_rank(const RunInfo &r, int base) {
  const int lane = (int)__lane_id();
  const unsigned long long upto = lane == 63 ? r.heads : (r.heads & ((2ull << lane) - 1ull));
  const int h = 63 - __clzll((long long)upto);
  return __shfl(base, h, 64) + (lane - h);
}

// Rank of a lane's particle among the particles of its cell c (c < 0: none,
// the result unused), called by every lane of the wavefront: the lanes that
// share a cell (consecutive, as the particles arrive cell-sorted from the
// previous step) take their ranks with one atomic per run of equal cells.
// Ranks come in any order; the per-cell sort orders the cells' runs by
// storage index afterwards.
__device__ __forceinline__ int rank_in_cell(int c, int32_t *__restrict__ count) {
  const RunInfo r = wave_runs(c);
  int base = r.len;
  if (r.head && c >= 0) base = atomicAdd(&count[c], r.len);
  return wave_rank(r, base);
}

// Cell of each of n particles and its rank in that cell.
__global__ void k_bin(const KGeom G, int64_t cell_off, int64_t n, const float4 *__restrict__ pos4,
                      int32_t *__restrict__ cell_of, int32_t *__restrict__ rank_of,
                      int32_t *__restrict__ count) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = -1;
  if (p < n) {
    const float4 x = pos4[p];
    int cx, cy, cz;
    c = (int)cell_off + cell_index(G, x.x, x.y, x.z, cx, cy, cz);
    cell_of[p] = c;
  }
  const int k = rank_in_cell(c, count);
  if (p < n) rank_of[p] = k;
}

__device__ __forceinline__ int block_exclusive_scan(int v, int *lds, int &total) {
  // Hillis-Steele over the block in LDS (kScanThreads entries).
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const int a = t >= off ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += a;
    __syncthreads();
  }
  total = lds[kScanThreads - 1];
  const int incl = lds[t];
  __syncthreads();
  return incl - v;
}

// Sum of count over the chunk [base, min(base + kScanChunk, n)) into *out.
__device__ __forceinline__ void scan_reduce_chunk(int64_t base, int64_t n,
                                                  const int32_t *__restrict__ count,
                                                  int32_t *__restrict__ out, int *lds) {
  int acc = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (i < n) acc += count[i];
  }
  lds[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kScanThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = lds[0];
  __syncthreads();
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(int64_t n,
                                                              const int32_t *__restrict__ count,
                                                              int32_t *__restrict__ bsum) {
  __shared__ int lds[kScanThreads];
  scan_reduce_chunk((int64_t)blockIdx.x * kScanChunk, n, count, bsum + blockIdx.x, lds);
}

// Sum of v over the block (kScanThreads threads, four wavefronts).
__device__ __forceinline__ int block_sum(int v, int *lds) {
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) t += lds[w];
  __syncthreads();
  return t;
}

// Each thread owns kScanItems consecutive cells; the block's cells are read
// through LDS so that global loads and stores stay coalesced.  The block's
// offset is the sum of the block sums bsum[0 .. blockIdx) of k_scan_reduce.  With wall
// offsets wstart (exclusive scan of the static wall counts) it also writes
// the merged runs: start_all[c] = start[c] + wstart[c] begins cell c's run of
// walls then fluid, fluid_off[c] = start_all[c] + (walls in c) its fluid part.
// The chunk [base, min(base + kScanChunk, n)) of the exclusive scan, offset
// by the sum of everything before it; the last chunk (last) also writes the
// entry n after the end.  count is cleared for the next step.
__device__ __forceinline__ void scan_down_chunk(int64_t base, int64_t n, int offset, bool last,
                                                int32_t *__restrict__ count,
                                                int32_t *__restrict__ start,
                                                const int32_t *__restrict__ wstart,
                                                int32_t *__restrict__ start_all,
                                                int32_t *__restrict__ fluid_off, int *tile,
                                                int *lds) {
  for (int k = 0; k < kScanItems; ++k) {
    const int local = k * kScanThreads + threadIdx.x;
    const int64_t i = base + local;
    int v = 0;
    if (i < n) {
      v = count[i];
      count[i] = 0;
    }
    tile[local + local / 32] = v;
  }
  __syncthreads();
  int run = 0;
  const int first = threadIdx.x * kScanItems;
  for (int k = 0; k < kScanItems; ++k) {
    const int local = first + k;
    run += tile[local + local / 32];
  }
  int total;
  int ex = block_exclusive_scan(run, lds, total) + offset;
  for (int k = 0; k < kScanItems; ++k) {
    const int local = first + k;
    const int v = tile[local + local / 32];
    tile[local + local / 32] = ex;
    ex += v;
  }
  __syncthreads();
  for (int k = 0; k < kScanItems; ++k) {
    const int local = k * kScanThreads + threadIdx.x;
    const int64_t i = base + local;
    if (i < n) {
      const int st = tile[local + local / 32];
      start[i] = st;
      if (wstart) {
        const int w0 = wstart[i], w1 = wstart[i + 1];
        start_all[i] = st + w0;
        fluid_off[i] = st + w1;
      }
    }
  }
  if (last && threadIdx.x == kScanThreads - 1) {
    start[n] = offset + total;
    if (wstart) start_all[n] = offset + total + wstart[n];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(
    int64_t n, int32_t *__restrict__ count, int32_t *__restrict__ start,
    const int32_t *__restrict__ bsum, const int32_t *__restrict__ wstart,
    int32_t *__restrict__ start_all, int32_t *__restrict__ fluid_off) {
  __shared__ int tile[kScanChunk + kScanChunk / 32];
  __shared__ int lds[kScanThreads];
  int prior = 0;
  for (int j = (int)threadIdx.x; j < (int)blockIdx.x; j += kScanThreads) prior += bsum[j];
  const int offset = block_sum(prior, lds);
  scan_down_chunk((int64_t)blockIdx.x * kScanChunk, n, offset, blockIdx.x == gridDim.x - 1, count,
                  start, wstart, start_all, fluid_off, tile, lds);
}

// idx[start[cell_of[p]] + rank_of[p]] = p for the n entries.  Threads n ..
// n + nw - 1 write the wall part of the merged runs (wall w, cell-sorted in
// cell wcell[w], is index n + w of the position arrays), and with dk the
// first thread advances the force evaluation index, so that one launch does
// the work of three.
__device__ __forceinline__ void scatter_one(int64_t p, int64_t n, const int32_t *__restrict__ cell_of,
                                            const int32_t *__restrict__ rank_of,
                                            const int32_t *__restrict__ start,
                                            int32_t *__restrict__ idx, int64_t nw,
                                            const int32_t *__restrict__ wcell,
                                            const int32_t *__restrict__ wstart,
                                            const int32_t *__restrict__ start_all,
                                            int32_t *__restrict__ idx_all) {
  if (p < n) {
    idx[start[cell_of[p]] + rank_of[p]] = (int32_t)p;
    return;
  }
  const int64_t w = p - n;
  if (w >= nw) return;
  const int c = wcell[w];
  idx_all[start_all[c] + ((int)w - wstart[c])] = (int32_t)(n + w);
}

__global__ void k_scatter(int64_t n, const int32_t *__restrict__ cell_of,
                          const int32_t *__restrict__ rank_of, const int32_t *__restrict__ start,
                          int32_t *__restrict__ idx, int64_t nw, const int32_t *__restrict__ wcell,
                          const int32_t *__restrict__ wstart,
                          const int32_t *__restrict__ start_all, int32_t *__restrict__ idx_all,
                          unsigned long long *__restrict__ dk) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (dk && p == 0) *dk += 1ull;
  scatter_one(p, n, cell_of, rank_of, start, idx, nw, wcell, wstart, start_all, idx_all);
}

// A cell's run of up to K storage indices (the common case: about four per
// cell at density 4), loaded into registers with independent loads and sorted by a
// fixed insertion network of compare-exchanges, the slots past the run padded
// with a key above every index; written back to idx and, if out, to out.
template <int K>
__device__ __forceinline__ void sort_run_regs(int32_t *__restrict__ idx, int a, int n,
                                              int32_t *__restrict__ out) {
  uint32_t v[K];
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = i < n ? (uint32_t)idx[a + i] : 0xffffffffu;
#pragma unroll
  for (int i = 1; i < K; ++i)
#pragma unroll
    for (int j = i; j > 0; --j) {
      const uint32_t lo = min(v[j - 1], v[j]), hi = max(v[j - 1], v[j]);
      v[j - 1] = lo;
      v[j] = hi;
    }
#pragma unroll
  for (int i = 0; i < K; ++i)
    if (i < n) {
      idx[a + i] = (int32_t)v[i];
      if (out) out[i] = (int32_t)v[i];
    }
}

// Atomic ranks arrive in any order: sort each cell's run by storage index so
// that the cell list, and every sum over it, is deterministic.  With key4 the
// run is sorted by the gid bits of key4[i].w instead, which makes the order
// independent of how the particles were stored before (used when a state is
// loaded from outside).  With idx_all the sorted run is also written to the
// fluid part of the merged run.
// Runs of up to 16 are sorted in registers (sort_run_regs); longer runs, and
// the gid order, by an insertion sort in memory.
template <bool BY_GID>
__device__ __forceinline__ void sort_cell(int64_t c, const int32_t *__restrict__ start,
                                          int32_t *__restrict__ idx,
                                          const float4 *__restrict__ key4,
                                          const int32_t *__restrict__ fluid_off,
                                          int32_t *__restrict__ idx_all) {
  const int a = start[c], b = start[c + 1];
  if (!BY_GID && b - a <= 16) {
    int32_t *out = idx_all ? idx_all + fluid_off[c] : nullptr;
    if (b - a <= 4)
      sort_run_regs<4>(idx, a, b - a, out);
    else if (b - a <= 8)
      sort_run_regs<8>(idx, a, b - a, out);
    else
      sort_run_regs<16>(idx, a, b - a, out);
    return;
  }
  for (int i = a + 1; i < b; ++i) {
    const int v = idx[i];
    const uint32_t kv = BY_GID ? __float_as_uint(key4[v].w) : (uint32_t)v;
    int j = i - 1;
    while (j >= a && (BY_GID ? __float_as_uint(key4[idx[j]].w) : (uint32_t)idx[j]) > kv) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = v;
  }
  if (idx_all) {
    const int o = fluid_off[c];
    for (int i = a; i < b; ++i) idx_all[o + (i - a)] = idx[i];
  }
}

template <bool BY_GID>
__global__ void k_sort_cells(int64_t ncell, const int32_t *__restrict__ start,
                             int32_t *__restrict__ idx, const float4 *__restrict__ key4,
                             const int32_t *__restrict__ fluid_off,
                             int32_t *__restrict__ idx_all) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  sort_cell<BY_GID>(c, start, idx, key4, fluid_off, idx_all);
}

// The walls' per-cell sort (by storage index, as sort_cell), which also
// writes the cell of every sorted position: cell_out[i] = c for i in
// [start[c], start[c + 1]).
__global__ void k_sort_wall_cells(int64_t ncell, const int32_t *__restrict__ start,
                                  int32_t *__restrict__ idx, int32_t *__restrict__ cell_out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  sort_cell<false>(c, start, idx, nullptr, nullptr, nullptr);
  const int a = start[c], b = start[c + 1];
  for (int i = a; i < b; ++i) cell_out[i] = (int32_t)c;
}

// Coarse codes of the merged runs, cq[t] = qcode3(pos4[idx_all[t]]): one
// thread per entry, so that the index reads and code writes coalesce.
__global__ void k_quant_runs(int64_t n, const int32_t *__restrict__ idx_all,
                             const float4 *__restrict__ pos4, uint32_t *__restrict__ cq) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float4 x = pos4[idx_all[t]];
  cq[t] = qcode3(x.x, x.y, x.z);
}

// The pad entry after fluid and walls: a position far outside the box, so
// that it never tests as a neighbour; the spare run-array entries after the
// last run name it.
__global__ void k_set_pad(float4 *pos4, float4 *vt4, int32_t *slack, int32_t pad) {
  *pos4 = make_float4(1e30f, 1e30f, 1e30f, __uint_as_float(0xFFFFFFFFu));
  if (vt4) *vt4 = make_float4(0.f, 0.f, 0.f, 0.f);
  if (slack)
    for (int u = 0; u < kIdxSlack; ++u) slack[u] = pad;
}

__global__ void k_cells(const KGeom G, int64_t cell_off, int64_t n,
                        const float4 *__restrict__ pos4, int32_t *__restrict__ cell) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float4 x = pos4[p];
  int cx, cy, cz;
  cell[p] = (int)cell_off + cell_index(G, x.x, x.y, x.z, cx, cy, cz);
}

__global__ void k_permute(int64_t n, const int32_t *__restrict__ idx, const float4 *a_in,
                          float4 *a_out, const float4 *b_in, float4 *b_out, const float4 *c_in,
                          float4 *c_out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = idx[s];
  if (a_in) a_out[s] = a_in[i];
  if (b_in) b_out[s] = b_in[i];
  if (c_in) c_out[s] = c_in[i];
}

// ---------------------------------------------------------------------------
// Phase field: near-interface mask and create-time check
// ---------------------------------------------------------------------------
// One bit per grid cube (the cube with lower corner node (i, j, k)): set if
// any of its 8 corner nodes is negative.  A trilinear value inside a cube
// whose corners are all >= 0 is >= 0 in the rounding of the decision form
// (each lerp of non-negative values is non-negative), so particles in
// unflagged cubes cannot have phi < 0 and skip the interpolation.
template <typename T>
__global__ void k_cube_mask(const KGeom G, const T *__restrict__ grid, int64_t nwords,
                            uint32_t *__restrict__ bits) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwords) return;
  const int64_t ncube = (int64_t)G.ng[0] * G.ng[1] * G.ng[2];
  const size_t nx = (size_t)G.ng[0], nxy = nx * (size_t)G.ng[1];
  uint32_t word = 0;
  for (int b = 0; b < 32; ++b) {
    const int64_t q = w * 32 + b;
    if (q >= ncube) break;
    const int i = (int)(q % G.ng[0]);
    const int j = (int)((q / G.ng[0]) % G.ng[1]);
    const int k = (int)(q / ((int64_t)G.ng[0] * G.ng[1]));
    const int i1 = i + 1 == G.ng[0] ? 0 : i + 1;
    const int j1 = j + 1 == G.ng[1] ? 0 : j + 1;
    const int k1 = k + 1 == G.ng[2] ? 0 : k + 1;
    bool neg = false;
    for (int dk = 0; dk < 2; ++dk)
      for (int dj = 0; dj < 2; ++dj) {
        const T *row = grid + (size_t)(dk ? k1 : k) * nxy + (size_t)(dj ? j1 : j) * nx;
        neg |= row[i] < (T)0;
        neg |= row[i1] < (T)0;
      }
    if (neg) word |= 1u << b;
  }
  bits[w] = word;
}

// The face layout of the phase field (PhiQuad): node (i, j, k) gets
// (phi(i, j, k), phi(i+1, j, k), phi(i, j+1, k), phi(i+1, j+1, k)).
template <typename T>
__global__ void k_build_quad(const KGeom G, const T *__restrict__ grid, int64_t nodes,
                             typename PhiQuad<T>::type *__restrict__ quad) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nodes) return;
  const int nx = G.ng[0], ny = G.ng[1];
  const int i = (int)(q % nx);
  const int64_t r = q / nx;
  const int j = (int)(r % ny);
  const int64_t k = r / ny;
  const int i1 = i + 1 == nx ? 0 : i + 1;
  const int j1 = j + 1 == ny ? 0 : j + 1;
  const T *row0 = grid + ((size_t)k * ny + j) * nx;
  const T *row1 = grid + ((size_t)k * ny + j1) * nx;
  typename PhiQuad<T>::type v;
  v.x = row0[i];
  v.y = row0[i1];
  v.z = row1[i];
  v.w = row1[i1];
  quad[q] = v;
}

__device__ __forceinline__ bool cube_flagged(const uint32_t *__restrict__ bits, size_t q) {
  return (bits[q >> 5] >> (q & 31)) & 1u;
}

template <typename T>
__global__ void k_check_grid(const T *__restrict__ grid, int64_t count, Status *st) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long bad = 0;
  for (; i < count; i += stride)
    if (!isfinite(grid[i])) ++bad;
  if (bad) atomicAdd(&st->bad_grid, bad);
}

template <typename T>
__global__ void k_check_phi(const KGeom G, const T *__restrict__ grid, int64_t n,
                            const float4 *__restrict__ pos4, Status *st) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float4 x = pos4[p];
  if (phi_at(grid, G, x.x, x.y, x.z) < (T)0) atomicAdd(&st->bad_phi, 1ull);
}

// ---------------------------------------------------------------------------
// Integrate + reflect + bin (Groot-Warren drift, Sec. II.C bounce-back)
//
// Each thread advances two particles (p and p + kBlock of a 2 kBlock tile),
// so that their loads and atomics are in flight together.  Ranks within a
// cell come from one atomic per run of equal cells in a wavefront: the
// particles arrive sorted by their previous cell and most keep it, so runs
// are the common case.
// ---------------------------------------------------------------------------
struct Moved {
  float4 pos;  // new position, gid bits in w
  float4 vt;   // predicted velocity, event code bits in w
  int cell;
};

// Velocity of the solid at a reflection at (x, y, z): that of the wall
// particle nearest to the point among the walls of the 27 cells around its
// cell, nearness by the FP32 pair-decision r2 (with the neighbour cell's
// image shift), ties to the smaller gid; zero where there is none.  Walls
// are at their start-of-step positions: entry NF + w of pos4 and vt4, wall
// runs wcstart over the global cells (box offset co).  The minimum of
// (r2, gid) does not depend on the visiting order, so the walls are taken
// row by row (the three cells of a row are one run, two where it wraps in
// x), four independent loads at a time, with the next row's bounds fetched
// while the current row is searched: a bouncing lane waits for a few loads
// per row instead of one per wall and cell.
__device__ __forceinline__ float4 wall_velocity(const KGeom &G, int co, int64_t NF, float x, float y,
                                             float z, const int32_t *__restrict__ wcstart,
                                             const float4 *__restrict__ pos4,
                                             const float4 *__restrict__ vt4) {
  int cx, cy, cz;
  cell_index(G, x, y, z, cx, cy, cz);
  const float4 *walls = pos4 + NF;
  float best = INFINITY;
  uint32_t best_gid = 0;
  int best_w = -1;
  NeighbourRows rows;
  rows.init(cx, cy, cz);
  int t, te;
  float sx, sy, sz;
  bool more = rows.next(G, wcstart, co, t, te, sx, sy, sz);
  while (more) {
    int t2, te2;
    float sx2, sy2, sz2;
    const bool more2 = rows.next(G, wcstart, co, t2, te2, sx2, sy2, sz2);
    const float ax = sub_nc(x, sx), ay = sub_nc(y, sy), az = sub_nc(z, sz);
    for (int w = t; w < te; w += 4) {
      float4 q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = walls[min(w + u, te - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float r2 = pair_r2(sub_nc(ax, q[u].x), sub_nc(ay, q[u].y), sub_nc(az, q[u].z));
        const uint32_t g = __float_as_uint(q[u].w);
        if (w + u < te && (r2 < best || (r2 == best && g < best_gid))) {
          best = r2;
          best_gid = g;
          best_w = w + u;
        }
      }
    }
    more = more2;
    t = t2;
    te = te2;
    sx = sx2;
    sy = sy2;
    sz = sz2;
  }
  if (best_w < 0) return make_float4(0.f, 0.f, 0.f, 0.f);
  return vt4[NF + best_w];
}

// REFLECT: compiled with the moving-wall and specular forms (the other
// instances keep the register budget of plain bounce-back off resting walls).
template <typename T, bool REFLECT>
__device__ __forceinline__ Moved integrate_one(const KGeom &G, const KParams &P, float4 x,
                                               float4 v, float4 f,
                                               const uint32_t *__restrict__ bits, int use_mask,
                                               const typename PhiQuad<T>::type *__restrict__ quad,
                                               Status *st, int co,
                                               int64_t NF, const int32_t *__restrict__ wcstart,
                                               const float4 *__restrict__ pos4,
                                               const float4 *__restrict__ vt4) {
  float xs = drift1(x.x, v.x, f.x, P.hdt, P.dt, G.L[0]);
  float ys = drift1(x.y, v.y, f.y, P.hdt, P.dt, G.L[1]);
  float zs = drift1(x.z, v.z, f.z, P.hdt, P.dt, G.L[2]);
  float4 vt = make_float4(v.x + P.lamdt * f.x, v.y + P.lamdt * f.y, v.z + P.lamdt * f.z, 0.f);
  {
    const float dx = P.dt * (v.x + P.hdt * f.x), dy = P.dt * (v.y + P.hdt * f.y),
                dz = P.dt * (v.z + P.hdt * f.z);
    const float d2 = dx * dx + dy * dy + dz * dz;
    if (!(d2 <= P.max_disp2)) {
      if (d2 != d2 || isinf(d2))
        atomicAdd(&st->nonfinite, 1ull);
      else
        atomicAdd(&st->unstable, 1ull);
      // keep indices in range for the rest of the step
      if (!(xs >= 0.f && xs <= G.L[0])) xs = x.x;
      if (!(ys >= 0.f && ys <= G.L[1])) ys = x.y;
      if (!(zs >= 0.f && zs <= G.L[2])) zs = x.z;
    }
  }
  int event = 0;
  const GridLoc<T> loc = grid_locate<T>(G, xs, ys, zs);
  if (!use_mask || cube_flagged(bits, cube_index(G, loc))) {
    const T phis = phi_interp_quad<T>(quad, G, loc);
    if (phis < (T)0) {
      // Eq. 16-17: distances beyond and before the interface from atanh(phi)
      const T phit = phi_at_quad<T>(quad, G, x.x, x.y, x.z);
      const T lim = (T)1 - (T)0x1p-20;
      const T a1 = fmin(fmax(-phis, (T)0), lim);
      const T a0 = fmin(fmax(phit, (T)0), lim);
      const T c1 = atanh(a1), c0 = atanh(a0);
      const T sfrac = c1 > (T)0 ? c1 / (c0 + c1) : (T)0;
      const float k2 = (float)((T)2 * sfrac * (T)P.dt);
      // the reversed part u of the velocity relative to the wall: all of it
      // (bounce-back) or its component along the normal (specular)
      float4 vw = make_float4(0.f, 0.f, 0.f, 0.f);
      if (REFLECT && (P.reflect & kReflectMoving))
        vw = wall_velocity(G, co, NF, xs, ys, zs, wcstart, pos4, vt4);
      float ux = v.x - vw.x, uy = v.y - vw.y, uz = v.z - vw.z;
      if (REFLECT && (P.reflect & kReflectSpecular)) {
        T gx, gy, gz;
        phi_grad_quad<T>(quad, G, loc, gx, gy, gz);
        const T gn = sqrt(gx * gx + gy * gy + gz * gz);
        if (gn > (T)0) {
          const T nx = gx / gn, ny = gy / gn, nz = gz / gn;
          const T un = (T)ux * nx + (T)uy * ny + (T)uz * nz;
          ux = (float)(un * nx);
          uy = (float)(un * ny);
          uz = (float)(un * nz);
        }
      }
      float bx = wrap1(xs - k2 * ux, G.L[0]);
      float by = wrap1(ys - k2 * uy, G.L[1]);
      float bz = wrap1(zs - k2 * uz, G.L[2]);
      if (phi_at_quad<T>(quad, G, bx, by, bz) < (T)0) {
        bx = x.x;
        by = x.y;
        bz = x.z;
        event = 2;
      } else {
        event = 1;
      }
      xs = bx;
      ys = by;
      zs = bz;
      vt = make_float4(v.x - 2.f * ux, v.y - 2.f * uy, v.z - 2.f * uz, 0.f);
    }
  }
  vt.w = __int_as_float(event);
  Moved m;
  m.pos = make_float4(xs, ys, zs, x.w);
  m.vt = vt;
  int cx, cy, cz;
  m.cell = cell_index(G, xs, ys, zs, cx, cy, cz);
  return m;
}

// Tile tid of up to PPT x kBlock particles of one box, by one block of
// kBlock threads; each thread advances PPT particles.
template <typename T, int PPT, bool REFLECT>
__device__ __forceinline__ void integrate_tile(
    int tid, const Box *__restrict__ boxes, const Tile *__restrict__ tiles,
    float4 *__restrict__ pos4, const float4 *__restrict__ vel4, const float4 *__restrict__ frc4,
    float4 *__restrict__ vt4, int32_t *__restrict__ cell_of, int32_t *__restrict__ rank_of,
    int32_t *__restrict__ count, const uint32_t *__restrict__ bits_base, int use_mask,
    const typename PhiQuad<T>::type *__restrict__ quad_base, Status *st, int64_t NF,
    const int32_t *__restrict__ wcstart) {
  const Tile tile = tiles[tid];
  const Box &B = boxes[tile.box];
  const KGeom G = B.G;
  const KParams P = B.P;
  const typename PhiQuad<T>::type *quad = quad_base + B.go;
  const uint32_t *bits = bits_base + B.bo;
  const int co = (int)B.co;
  int64_t p[PPT];
  bool a[PPT];
  float4 x[PPT], v[PPT], f[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int local = u * kBlock + (int)threadIdx.x;
    a[u] = local < tile.count;
    p[u] = (int64_t)tile.first + local;
    x[u] = v[u] = f[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (a[u]) {
      x[u] = load_stream(&pos4[p[u]]);
      v[u] = load_stream(&vel4[p[u]]);
      f[u] = load_stream(&frc4[p[u]]);
    }
  }
  Moved m[PPT];
  RunInfo r[PPT];
  int b[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    m[u].cell = -1;
    if (a[u]) {
      m[u] = integrate_one<T, REFLECT>(G, P, x[u], v[u], f[u], bits, use_mask, quad, st, co, NF,
                                       wcstart, pos4, vt4);
      m[u].cell += co;
    }
    r[u] = wave_runs(m[u].cell);
    b[u] = 0;
  }
#pragma unroll
  for (int u = 0; u < PPT; ++u)
    if (r[u].head && m[u].cell >= 0) b[u] = atomicAdd(&count[m[u].cell], r[u].len);
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int k = wave_rank(r[u], b[u]);
    if (a[u]) {
      store_stream(&pos4[p[u]], m[u].pos);
      store_stream(&vt4[p[u]], m[u].vt);
      store_stream(&cell_of[p[u]], m[u].cell);
      store_stream(&rank_of[p[u]], k);
    }
  }
  // event counts: one atomic per wavefront, after the stores (a per-lane
  // atomic on the one counter word put its latency into the step's chain)
  int nbounce = 0, nfall = 0;
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int ev = a[u] ? __float_as_int(m[u].vt.w) : 0;
    nbounce += __popcll(__ballot(ev == 1));
    nfall += __popcll(__ballot(ev == 2));
  }
  if (__lane_id() == 0) {
    if (nbounce) atomicAdd(&st->bounce, (unsigned long long)nbounce);
    if (nfall) atomicAdd(&st->fallback, (unsigned long long)nfall);
  }
}

template <typename T, int PPT, bool REFLECT>
__global__ __launch_bounds__(kBlock) void k_integrate(
    const Box *__restrict__ boxes, const Tile *__restrict__ tiles, int ntiles,
    float4 *__restrict__ pos4, const float4 *__restrict__ vel4, const float4 *__restrict__ frc4,
    float4 *__restrict__ vt4, int32_t *__restrict__ cell_of, int32_t *__restrict__ rank_of,
    int32_t *__restrict__ count, const uint32_t *__restrict__ bits_base, int use_mask,
    const typename PhiQuad<T>::type *__restrict__ quad_base, Status *st, int64_t NF,
    const int32_t *__restrict__ wcstart) {
  const int tid = xcd_block();
  if (tid >= ntiles) return;
  integrate_tile<T, PPT, REFLECT>(tid, boxes, tiles, pos4, vel4, frc4, vt4, cell_of, rank_of, count,
                                  bits_base, use_mask, quad_base, st, NF, wcstart);
}

// Walls of one box re-binned: each is advanced by dt v with move (its solid
// translates: x += dt v per axis in the decision form of the fluid drift
// with zero force, then the single-edge wrap) or kept, written to walls_out
// with its velocity to vt_out, and binned (cell and rank in cell, as k_bin).
__global__ void k_wall_move_bin(const KGeom G, float hdt, float dt, int move, int64_t cell_off,
                                int64_t nw, const float4 *__restrict__ walls_in,
                                const float4 *__restrict__ vt_in, float4 *__restrict__ walls_out,
                                float4 *__restrict__ vt_out, int32_t *__restrict__ cell_of,
                                int32_t *__restrict__ rank_of, int32_t *__restrict__ count) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = -1;
  if (w < nw) {
    float4 x = walls_in[w];
    const float4 v = vt_in[w];
    if (move)
      x = make_float4(drift1(x.x, v.x, 0.f, hdt, dt, G.L[0]), drift1(x.y, v.y, 0.f, hdt, dt, G.L[1]),
                      drift1(x.z, v.z, 0.f, hdt, dt, G.L[2]), x.w);
    walls_out[w] = x;
    vt_out[w] = v;
    int cx, cy, cz;
    c = (int)cell_off + cell_index(G, x.x, x.y, x.z, cx, cy, cz);
    cell_of[w] = c;
  }
  const int k = rank_in_cell(c, count);
  if (w < nw) rank_of[w] = k;
}

// Wall positions from gid-ordered rows (gid in pos4[w].w).
__global__ void k_import_walls(int64_t nw, float4 *__restrict__ walls, const float *__restrict__ pos) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const float4 x = walls[w];
  const size_t g = (size_t)__float_as_uint(x.w);
  walls[w] = make_float4(pos[3 * g], pos[3 * g + 1], pos[3 * g + 2], x.w);
}

// Number of fluid particles whose grid cube is flagged (the particles that
// interpolate phi in a step), one atomic per block.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_count_flagged(const KGeom G, int64_t nf,
                                                          const float4 *__restrict__ pos4,
                                                          const uint32_t *__restrict__ bits,
                                                          unsigned long long *out) {
  __shared__ int lds[kBlock];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int v = 0;
  if (p < nf) {
    const float4 x = pos4[p];
    v = cube_flagged(bits, cube_index(G, grid_locate<T>(G, x.x, x.y, x.z))) ? 1 : 0;
  }
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && lds[0]) atomicAdd(out, (unsigned long long)lds[0]);
}

// ---------------------------------------------------------------------------
// Pair force (Eq. 3-10), body force, velocity update
//
// One thread per fluid particle i, in cell-sorted slot order; a wavefront is
// 64 consecutive particles.  Phase A: the wavefront visits the 9 rows of the
// 27-cell neighbourhood together (the x-neighbours of a row are consecutive
// cells, so a row is one run of merged entries, walls then fluid, or two
// where it wraps in x) and walks each row in lockstep, four run entries per
// lane and pass so that their loads overlap, testing the entries' coarse
// position codes against a bound that keeps every pair of the FP32 cutoff
// decision; kept candidates go to the lane's column of an LDS list
// (slot-major, so the wavefront's appends fall in different banks).  Phase
// B: each lane takes the exact FP32 decision on its listed candidates; the
// random-number and force arithmetic runs only for pairs inside the
// cutoff.  The wavefront runs phase B when any
// lane's list could overflow in the next pass, and once at the end.  Lanes
// never branch apart inside a pass, so the wavefront pays for the longest
// run of each row, not for every lane's row switches.  Sums run in
// candidate order, so runs are deterministic.
// ---------------------------------------------------------------------------
// 26 entries per lane: with 256-thread blocks at six wavefronts per SIMD,
// six blocks' lists (26 KB each) fill a CU's 160 KB of LDS, and most lanes'
// pairs (about 16 plus the pre-test's extras) fit, so most wavefronts run
// the pair pass once, after the walk, instead of twice.
constexpr int kListCap = 26;
constexpr int kBatch = 4;   // = the width of one run-array load

struct Acc {
  float x, y, z;
};

// SPH: compiled with the conservative force of Eq. 22-24 for boxes that use
// it (wall: j is a wall particle, selecting the fluid-wall strengths).
template <bool SPH>
__device__ __forceinline__ void add_pair(Acc &acc, float dx, float dy, float dz, float r2,
                                         float dvx, float dvy, float dvz, float a, bool wall,
                                         const KParams &P, uint32_t gi, uint32_t gj,
                                         uint32_t klo, uint32_t khi) {
  const float rinv = rsqrtf(r2);
  const float r = r2 * rinv;
  const float w = fmaxf(1.0f - r * P.inv_rc, 0.0f);
  const float ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
  const float edv = ex * dvx + ey * dvy + ez * dvz;
  const float xi = pair_gauss(gi, gj, klo, khi, P.key0, P.key1);
  float mag;
  if (SPH && P.sph) {
    const float cr = wall ? P.cr_fw : P.cr_ff, ca = wall ? P.ca_fw : P.ca_ff;
    const float fc = ca * spline_dp(r * P.inv_ha) - cr * spline_dp(r * P.inv_hr);
    mag = fc + w * (P.sigma_rdt * xi - P.gamma * w * edv);
  } else {
    mag = w * (a - P.gamma * w * edv + P.sigma_rdt * xi);
  }
  acc.x += mag * ex;
  acc.y += mag * ey;
  acc.z += mag * ez;
}

// Tile tid by one block of BS threads; list: kListCap x BS words of LDS.
// The walk tests candidates on their coarse codes (cq, one word per
// merged-run entry, in run order) and lists every candidate the bound
// keeps; the pair pass then takes the exact FP32 decision, so the pairs
// summed and their order are those of an exact walk over the same runs.
template <bool INIT, int BS, bool SPH>
__device__ __forceinline__ void force_tile(
    int tid, uint32_t *list, const Box *__restrict__ boxes, const Tile *__restrict__ tiles,
    int64_t NF, int32_t pad, int32_t ncell_all, const float4 *__restrict__ pos4,
    const float4 *__restrict__ vt4, const float4 *__restrict__ vel4,
    const float4 *__restrict__ frc4, const int32_t *__restrict__ idx,
    const int32_t *__restrict__ idx_all, const int32_t *__restrict__ start_all,
    const uint32_t *__restrict__ cq,
    float4 *__restrict__ pos_out, float4 *__restrict__ vel_out, float4 *__restrict__ frc_out,
    const unsigned long long *__restrict__ dk, Status *st) {
  const Tile tile = tiles[tid];
  if ((int)threadIdx.x >= tile.count) return;
  const Box &B = boxes[tile.box];
  const KGeom G = B.G;
  const KParams P = B.P;
  const int co = (int)B.co;
  // force evaluation index k, kept on the device so that a captured step
  // draws new random numbers on every replay
  const unsigned long long kk = *dk;
  const uint32_t klo = (uint32_t)kk;
  const uint32_t khi = ((uint32_t)(kk >> 32) & 0xFFFFu) | (P.replica << 16);
  const int64_t s = (int64_t)tile.first + threadIdx.x;
  const int i = idx[s];
  const float4 pi = pos4[i];
  const float4 vti = vt4[i];
  const uint32_t gi = __float_as_uint(pi.w);
  int cx, cy, cz;
  cell_index(G, pi.x, pi.y, pi.z, cx, cy, cz);
  // pos4 and vt4 hold NF + NW + 1 records (the pad last); the run array and
  // the codes hold NF + NW entries and kIdxSlack spare ones (the run's read
  // as the pad); the run starts hold ncell_all + 1 entries and kStartSlack
  // spare ones
  const Records16 posr(pos4, pad + 1), vtr(vt4, pad + 1);
  const Ints4 runs(idx_all, pad + kIdxSlack);
  const Ints4 codes((const int32_t *)cq, pad + kIdxSlack);
  const Ints4 starts(start_all, ncell_all + 1 + kStartSlack);
  const uint32_t qth = qthresh(P.rc2);
  // this lane's list column as LDS byte offsets: entry q at lane0 + q * BS * 4
  char *const lds = (char *)list;
  const uint32_t lane0 = threadIdx.x * 4u;
  const uint32_t full = lane0 + (uint32_t)((kListCap - kBatch) * BS * 4);
  uint32_t tail = lane0;   // next free entry
  Acc acc = {0.f, 0.f, 0.f};
  // phase B: the listed candidates of this lane, in list (= candidate)
  // order, with the exact decision; the next candidate's data is fetched
  // while the current one is evaluated
  auto flush = [&]() {
    int j = tail > lane0 ? *(const int *)(lds + lane0) : pad;
    float4 pj = posr[j], vtj = vtr[j];
    for (uint32_t q = lane0; q < tail; q += BS * 4u) {
      const uint32_t qn = q + BS * 4u;
      const int jn = qn < tail ? *(const int *)(lds + qn) : pad;
      const float4 pjn = posr[jn], vtjn = vtr[jn];
      const float dx = sep(pi.x, pj.x, G.L[0]);
      const float dy = sep(pi.y, pj.y, G.L[1]);
      const float dz = sep(pi.z, pj.z, G.L[2]);
      const float r2 = dx * dx + dy * dy + dz * dz;
      const bool wall = (int64_t)j >= NF;
      const float a = wall ? P.a_fw : P.a_ff;
      // the pair decision (r2 > 0 also drops coincident particles, whose
      // force is 0)
      const float r2d = pair_r2(dx, dy, dz);
      if (r2d < P.rc2 && r2d > 0.0f)
        add_pair<SPH>(acc, dx, dy, dz, r2, vti.x - vtj.x, vti.y - vtj.y, vti.z - vtj.z, a, wall,
                      P, gi, __float_as_uint(pj.w), klo, khi);
      j = jn;
      pj = pjn;
      vtj = vtjn;
    }
    tail = lane0;
  };
  // Phase A for one neighbour row: the wavefront walks the lane's runs in
  // lockstep, kBatch run entries per lane and pass (run A, then run B where
  // the row wraps; a lane moves to B on its own), with qa / qb the lane's
  // code shifted by the image of run A / B.  Entries past the lane's run are
  // read (other cells' entries, or the pad) but never listed; neither is
  // the lane's own particle.  Phase B runs when a lane's list could
  // overflow in the next pass.
  auto walk = [&](int t, int t_end, int tb, int tb_end, uint32_t qa, uint32_t qb) {
    {
      const bool sw = t >= t_end;
      t = sw ? tb : t;
      t_end = sw ? tb_end : t_end;
      tb = sw ? tb_end : tb;
      qa = sw ? qb : qa;
    }
    for (;;) {
      while (wave_any(t < t_end) && !wave_any(tail > full)) {
        const int rem = t_end - t;
        int jb[kBatch], w[kBatch];
        runs.load(t, jb);
        codes.load(t, w);
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const bool keep = qdist2((uint32_t)w[u], qa) <= qth && jb[u] != i && u < rem;
          *(int *)(lds + tail) = jb[u];
          tail += keep ? (uint32_t)(BS * 4) : 0u;
        }
        t = rem > 0 ? t + kBatch : t;
        const bool sw = t >= t_end && tb < tb_end;
        t = sw ? tb : t;
        t_end = sw ? tb_end : t_end;
        tb = sw ? tb_end : tb;
        qa = sw ? qb : qa;
      }
      if (!wave_any(t < t_end)) break;
      flush();
    }
  };

  const int nx = G.nc[0], ny = G.nc[1], nz = G.nc[2];
  for (int oz = -1; oz <= 1; ++oz) {
    int qz = cz + oz;
    float sz = 0.f;
    if (qz < 0) { qz += nz; sz = -G.L[2]; }
    else if (qz >= nz) { qz -= nz; sz = G.L[2]; }
    const uint32_t cz_code = qshift(pi.z, sz) << 22;
    for (int oy = -1; oy <= 1; ++oy) {
      int qy = cy + oy;
      float sy = 0.f;
      if (qy < 0) { qy += ny; sy = -G.L[1]; }
      else if (qy >= ny) { qy -= ny; sy = G.L[1]; }
      const uint32_t cyz_code = (qshift(pi.y, sy) << 11) | cz_code;
      // the row's x-neighbours [cx-1, cx+1] as run A, plus run B where the
      // row wraps (cell nx-1 seen across the left edge, then cells 0 and 1;
      // or cells nx-2 and nx-1, then cell 0 seen across the right edge)
      const int base = co + (qz * ny + qy) * nx;
      const bool left = cx == 0, right = cx == nx - 1;
      const int a0 = left ? base + nx - 1 : (right ? base + nx - 2 : base + cx - 1);
      int v[4];
      starts.load(a0, v);
      const int ta = v[0], ta_end = left ? v[1] : (right ? v[2] : v[3]);
      int tb = 0, tb_end = 0;
      if (wave_any(left || right)) {
        int w[4];
        starts.load(base, w);
        tb = (left || right) ? w[0] : 0;
        tb_end = left ? w[2] : (right ? w[1] : 0);
      }
      const float sxa = left ? -G.L[0] : 0.f, sxb = right ? G.L[0] : 0.f;
      walk(ta, ta_end, tb, tb_end, qshift(pi.x, sxa) | cyz_code, qshift(pi.x, sxb) | cyz_code);
    }
  }
  flush();
  const float fx = acc.x + P.g[0], fy = acc.y + P.g[1], fz = acc.z + P.g[2];
  const float4 vo = load_stream(&vel4[i]);
  float4 vn;
  if (INIT) {
    vn = make_float4(vo.x, vo.y, vo.z, __int_as_float(0));
  } else {
    const int event = __float_as_int(vti.w);
    if (event) {
      vn = make_float4(vti.x, vti.y, vti.z, __int_as_float(event));
    } else {
      const float4 fo = load_stream(&frc4[i]);
      vn = make_float4(vo.x + P.hdt * (fo.x + fx), vo.y + P.hdt * (fo.y + fy),
                       vo.z + P.hdt * (fo.z + fz), __int_as_float(0));
    }
  }
  if (!(isfinite(fx) && isfinite(fy) && isfinite(fz))) atomicAdd(&st->nonfinite, 1ull);
  store_stream(&pos_out[s], pi);
  store_stream(&vel_out[s], vn);
  store_stream(&frc_out[s], make_float4(fx, fy, fz, 0.f));
}

// Six wavefronts per SIMD: at most 80 VGPRs, so the walk and the pair pass
// run without register spills, and six blocks' lists fit in LDS.
template <bool INIT, int BS, bool SPH>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(6))) void k_force(
    const Box *__restrict__ boxes, const Tile *__restrict__ tiles, int ntiles, int64_t NF,
    int32_t pad, int32_t ncell_all, const float4 *__restrict__ pos4,
    const float4 *__restrict__ vt4, const float4 *__restrict__ vel4,
    const float4 *__restrict__ frc4, const int32_t *__restrict__ idx,
    const int32_t *__restrict__ idx_all, const int32_t *__restrict__ start_all,
    const uint32_t *__restrict__ cq,
    float4 *__restrict__ pos_out, float4 *__restrict__ vel_out, float4 *__restrict__ frc_out,
    const unsigned long long *__restrict__ dk, Status *st) {
  __shared__ uint32_t list[kListCap * BS];
  const int tid = xcd_block();
  if (tid >= ntiles) return;
  force_tile<INIT, BS, SPH>(tid, list, boxes, tiles, NF, pad, ncell_all, pos4, vt4, vel4, frc4,
                            idx, idx_all, start_all, cq, pos_out, vel_out, frc_out, dk, st);
}

// Interacting pairs with the same decision as the force kernel.  Each thread
// counts its pairs, a wavefront reserves room with one atomic, then the
// pairs are written.
__device__ __forceinline__ int pairs_of(const KGeom &G, const KParams &P, int co, int i,
                                        float4 pi, int cx, int cy, int cz,
                                        const float4 *__restrict__ pos4,
                                        const int32_t *__restrict__ idx_all,
                                        const int32_t *__restrict__ start_all, uint32_t *out,
                                        int64_t base, int64_t cap) {
  int n = 0;
  const uint32_t gi = __float_as_uint(pi.w);
  for (int code = 0; code < 27; ++code) {
    const NCell nc = neighbour_cell(G, cx, cy, cz, code);
    const SepAxis ax = sep_axis(pi.x, nc.sx), ay = sep_axis(pi.y, nc.sy),
                  az = sep_axis(pi.z, nc.sz);
    const int t0 = start_all[co + nc.c], t1 = start_all[co + nc.c + 1];
    for (int t = t0; t < t1; ++t) {
      const int j = idx_all[t];
      if (j == i) continue;
      const float4 pj = pos4[j];
      if (pair_r2(sep_d(ax, pj.x), sep_d(ay, pj.y), sep_d(az, pj.z)) < P.rc2) {
        if (out && base + n < cap) {
          out[2 * (base + n)] = gi;
          out[2 * (base + n) + 1] = __float_as_uint(pj.w);
        }
        ++n;
      }
    }
  }
  return n;
}

__global__ __launch_bounds__(kBlock) void k_pairs(
    const KGeom G, const KParams P, int co, int64_t first, int64_t nf,
    const float4 *__restrict__ pos4, const int32_t *__restrict__ idx,
    const int32_t *__restrict__ idx_all, const int32_t *__restrict__ start_all, uint32_t *pairs,
    int64_t cap, unsigned long long *counter) {
  const int64_t s = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = s < first + nf;
  int i = 0, cx = 0, cy = 0, cz = 0;
  float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
  int n = 0;
  if (act) {
    i = idx[s];
    pi = pos4[i];
    cell_index(G, pi.x, pi.y, pi.z, cx, cy, cz);
    n = pairs_of(G, P, co, i, pi, cx, cy, cz, pos4, idx_all, start_all, nullptr, 0, 0);
  }
  // wavefront-inclusive prefix of n, one atomic per wavefront
  const int lane = (int)__lane_id();
  int incl = n;
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  const int total = __shfl(incl, 63, 64);
  unsigned long long base = 0;
  if (lane == 63 && total > 0) base = atomicAdd(counter, (unsigned long long)total);
  base = __shfl(base, 63, 64);
  if (act && pairs && n > 0)
    pairs_of(G, P, co, i, pi, cx, cy, cz, pos4, idx_all, start_all, pairs,
             (int64_t)base + incl - n, cap);
}

// The random numbers of given pairs (the same device functions as the force
// kernel): the four Philox words and xi.
__global__ void k_pair_random(uint32_t key0, uint32_t key1, uint32_t klo, uint32_t khi,
                              const uint32_t *__restrict__ gi, const uint32_t *__restrict__ gj,
                              int64_t n, uint32_t *words, float *xi) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t a = gi[p], b = gj[p];
  if (words) {
    uint32_t c0 = min(a, b), c1 = max(a, b), c2 = klo, c3 = khi;
    philox10(c0, c1, c2, c3, key0, key1);
    words[4 * p] = c0;
    words[4 * p + 1] = c1;
    words[4 * p + 2] = c2;
    words[4 * p + 3] = c3;
  }
  if (xi) xi[p] = pair_gauss(a, b, klo, khi, key0, key1);
}

// ---------------------------------------------------------------------------
// Getters and setters by gid
// ---------------------------------------------------------------------------
__global__ void k_export(const KGeom G, int64_t n, const float4 *__restrict__ pos4,
                         const float4 *__restrict__ vel4, const float4 *__restrict__ frc4,
                         int wall, float *pos, float *vel, float *frc, int32_t *events,
                         int32_t *cell_of) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float4 x = pos4[s];
  const size_t g = (size_t)__float_as_uint(x.w);
  if (pos) {
    pos[3 * g] = x.x;
    pos[3 * g + 1] = x.y;
    pos[3 * g + 2] = x.z;
  }
  float4 v = make_float4(0.f, 0.f, 0.f, __int_as_float(0));
  if (!wall) v = vel4[s];
  else if (vel4) v = make_float4(vel4[s].x, vel4[s].y, vel4[s].z, __int_as_float(0));
  if (vel) {
    vel[3 * g] = v.x;
    vel[3 * g + 1] = v.y;
    vel[3 * g + 2] = v.z;
  }
  if (events) events[g] = __float_as_int(v.w);
  if (frc) {
    float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
    if (!wall) f = frc4[s];
    frc[3 * g] = f.x;
    frc[3 * g + 1] = f.y;
    frc[3 * g + 2] = f.z;
  }
  if (cell_of) {
    int cx, cy, cz;
    cell_of[g] = cell_index(G, x.x, x.y, x.z, cx, cy, cz);
  }
}

__global__ void k_import(int64_t nf, float4 *pos4, float4 *vel4, float4 *frc4,
                         const float *__restrict__ pos, const float *__restrict__ vel,
                         const float *__restrict__ frc) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nf) return;
  const float gbits = pos4[s].w;
  const size_t g = (size_t)__float_as_uint(gbits);
  pos4[s] = make_float4(pos[3 * g], pos[3 * g + 1], pos[3 * g + 2], gbits);
  vel4[s] = make_float4(vel[3 * g], vel[3 * g + 1], vel[3 * g + 2], __int_as_float(0));
  frc4[s] = make_float4(frc[3 * g], frc[3 * g + 1], frc[3 * g + 2], 0.f);
}

__global__ void k_profile(const KGeom G, int64_t nf, const float4 *__restrict__ pos4,
                          const float4 *__restrict__ vel4, int axis, int nbins, double *out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nf) return;
  const float4 x = pos4[s];
  const float4 v = vel4[s];
  const float c = axis == 0 ? x.x : (axis == 1 ? x.y : x.z);
  int b = (int)floorf(c / G.L[axis] * (float)nbins);
  b = b < 0 ? 0 : (b >= nbins ? nbins - 1 : b);
  double *o = out + 5 * (size_t)b;
  atomicAdd(o, 1.0);
  atomicAdd(o + 1, (double)v.x);
  atomicAdd(o + 2, (double)v.y);
  atomicAdd(o + 3, (double)v.z);
  atomicAdd(o + 4, (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z);
}

// ---------------------------------------------------------------------------
// Persistent step: one launch for a whole step of every box of a batch.
// Blocks take work items in queue order from one counter; an item of phase
// p of box r first waits until every item of phase p - 1 of box r has
// arrived (a per-box, per-phase counter), so boxes run through the phases
// independently and no launch boundary separates them.  Every item waits
// only on items earlier in the queue, which blocks that are already running
// have taken, so the waits end whatever the number of resident blocks; each
// is also bounded (spin_limit sleeps), after which the item runs anyway and
// `stalled` reports the step as invalid.  The per-phase bodies are those of
// the per-phase kernels, so results are bit-identical to them.
// ---------------------------------------------------------------------------

// A value the same in every lane, as a scalar: function arguments arrive in
// vector registers, and without this every pointer loaded through them would
// be a per-lane value (vector loads of the arguments, buffer descriptors
// built lane by lane).
template <typename P>
__device__ __forceinline__ P *uniform_ptr(P *p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (P *)(((uint64_t)hi << 32) | lo);
}
// The arguments block, read through the constant address space (scalar loads).
typedef const __attribute__((address_space(4))) PArgs *ArgsPtr;
__device__ __forceinline__ ArgsPtr uniform_args(const PArgs *p) {
  return (ArgsPtr)uniform_ptr(p);
}
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
// A pointer into the block's LDS (the caller's __shared__ array): the cast
// through the local address space lets the compiler use LDS instructions.
template <typename P>
__device__ __forceinline__ P *lds_ptr(P *p) {
  return (P *)(__attribute__((address_space(3))) P *)p;
}

// The phase bodies as separate functions, each register-allocated on its own
// (inlined into one loop, the union of their live ranges would cut the
// kernel to two wavefronts per SIMD); each reads the arguments it needs.
template <typename T, int PPT, bool REFLECT>
__device__ __attribute__((noinline)) void p_integrate(const PArgs *__restrict__ A0, int tile0) {
  const ArgsPtr A = uniform_args(A0);
  const int tile = uniform_int(tile0);
  integrate_tile<T, PPT, REFLECT>(tile, A->boxes, A->itiles, A->pos4, A->vel4, A->frc4, A->vt4,
                                  A->cell_of, A->rank_of, A->count, A->bits, A->use_mask,
                                  (const typename PhiQuad<T>::type *)A->quad, A->st, A->NF,
                                  A->wcstart);
}

// chunk a of box `box`'s cells; its block sum at bsum[b + a]
__device__ __attribute__((noinline)) void p_reduce(const PArgs *__restrict__ A0, int box0,
                                                   int a0, int b0, int *lds0) {
  const ArgsPtr A = uniform_args(A0);
  const int box = uniform_int(box0), a = uniform_int(a0), b = uniform_int(b0);
  int *lds = lds_ptr(lds0);
  const int64_t co = A->boxes[box].co, ncell = A->boxes[box].ncell;
  scan_reduce_chunk(co + (int64_t)a * kScanChunk, co + ncell, A->count, A->bsum + b + a, lds);
}

// the box's fluid starts at slot fo; its chunks before this one add to it
__device__ __attribute__((noinline)) void p_down(const PArgs *__restrict__ A0, int box0, int a0,
                                                 int b0, int *tile0, int *lds0) {
  const ArgsPtr A = uniform_args(A0);
  const int box = uniform_int(box0), a = uniform_int(a0), b = uniform_int(b0);
  int *tile = lds_ptr(tile0), *lds = lds_ptr(lds0);
  const int64_t co = A->boxes[box].co, ncell = A->boxes[box].ncell, fo = A->boxes[box].fo;
  int prior = 0;
  for (int j = (int)threadIdx.x; j < a; j += kScanThreads) prior += A->bsum[b + j];
  const int offset = (int)fo + block_sum(prior, lds);
  const bool last = (int64_t)(a + 1) * kScanChunk >= ncell;
  scan_down_chunk(co + (int64_t)a * kScanChunk, co + ncell, offset, last, A->count, A->cstart,
                  A->wcstart, A->start_all, A->fluid_off, tile, lds);
}

__device__ __attribute__((noinline)) void p_scatter(const PArgs *__restrict__ A0, int a0, int b0) {
  const ArgsPtr A = uniform_args(A0);
  const int a = uniform_int(a0), b = uniform_int(b0);
  for (int64_t p = (int64_t)a + threadIdx.x; p < (int64_t)b; p += kBlock)
    scatter_one(p, A->NF, A->cell_of, A->rank_of, A->cstart, A->idx, A->NW, A->wcell, A->wcstart,
                A->start_all, A->idx_all);
}

__device__ __attribute__((noinline)) void p_sort(const PArgs *__restrict__ A0, int a0, int b0) {
  const ArgsPtr A = uniform_args(A0);
  const int a = uniform_int(a0), b = uniform_int(b0);
  for (int64_t c = (int64_t)a + threadIdx.x; c < (int64_t)b; c += kBlock)
    sort_cell<false>(c, A->cstart, A->idx, nullptr, A->fluid_off, A->idx_all);
  // the coarse codes of the merged-run entries of these cells (walls from
  // the scatter phase, fluid from the loop above)
  __syncthreads();
  const int t0 = uniform_int(A->start_all[a]), t1 = uniform_int(A->start_all[b]);
  for (int t = t0 + (int)threadIdx.x; t < t1; t += kBlock) {
    const float4 x = A->pos4[A->idx_all[t]];
    A->cq[t] = qcode3(x.x, x.y, x.z);
  }
}

template <bool SPH>
__device__ __attribute__((noinline)) void p_force(const PArgs *__restrict__ A0, int tile0,
                                                  uint32_t *list0) {
  const ArgsPtr A = uniform_args(A0);
  const int tile = uniform_int(tile0);
  uint32_t *list = lds_ptr(list0);
  force_tile<false, kBlock, SPH>(tile, list, A->boxes, A->ftiles, A->NF, A->pad,
                                       A->ncell_all, A->pos4, A->vt4, A->vel4, A->frc4, A->idx,
                                       A->idx_all, A->start_all, A->cq, A->pos_out, A->vel_out,
                                       A->frc_out, A->dk, A->st);
}

template <typename T, int PPT, bool REFLECT, bool SPH>
// Six wavefronts per SIMD, as the pair kernel: the pair list (26 KB per
// block) limits a CU to six blocks anyway, and the phase functions are
// allocated separately, the largest (the pair force, 74 VGPRs in its own
// kernel) with a few more registers as a callee.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void
k_step_persistent(const PArgs *__restrict__ A) {
  __shared__ union {
    uint32_t list[kListCap * kBlock];
    struct {
      int tile[kScanChunk + kScanChunk / 32];
      int lds[kScanThreads];
    } scan;
  } sm;
  __shared__ int s_item, s_ok;
  const int t = (int)threadIdx.x;
  const int nitems = A->nitems;
  // The item index and the item are the same in every lane; readfirstlane
  // makes that visible to the compiler, and the loop tests it at its head,
  // so the loop and the phase switch are uniform branches and every barrier
  // runs with all lanes.  (With the index as a per-lane value and the exit
  // in the middle of the loop, the loop was compiled as divergent and
  // rotated so that lanes 1-63 of the first wavefront went back to the top
  // barrier and re-read the index before lane 0 had taken the next one.)
  if (t == 0) s_item = atomicAdd(A->head, 1);
  __syncthreads();
  int it = __builtin_amdgcn_readfirstlane(s_item);
  while (it < nitems) {
    const PItem Iv = A->items[it];
    PItem I;
    I.phase = __builtin_amdgcn_readfirstlane(Iv.phase);
    I.box = __builtin_amdgcn_readfirstlane(Iv.box);
    I.a = __builtin_amdgcn_readfirstlane(Iv.a);
    I.b = __builtin_amdgcn_readfirstlane(Iv.b);
    if (t == 0) {
      int ok = 1;
      if (I.phase != kPhIntegrate) {
        const int dep = I.box * kPhases + I.phase - 1;
        const int need = A->need[dep];
        const int limit = A->spin_limit;
        int spins = 0;
        // relaxed loads while spinning (an acquire would invalidate this
        // XCD's L2 on every iteration); the acquire fence follows the wait
        while (__hip_atomic_load(&A->arrive[dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               need) {
          __builtin_amdgcn_s_sleep(4);
          if (++spins >= limit) {
            ok = 0;
            break;
          }
        }
      }
      s_ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (t == 0 && !__builtin_amdgcn_readfirstlane(s_ok)) atomicAdd(&A->st->stalled, 1ull);
    switch (I.phase) {
      case kPhIntegrate:
        for (int t = I.a; t < I.b; ++t) p_integrate<T, PPT, REFLECT>(A, t);
        break;
      case kPhReduce: p_reduce(A, I.box, I.a, I.b, sm.scan.lds); break;
      case kPhDown: p_down(A, I.box, I.a, I.b, sm.scan.tile, sm.scan.lds); break;
      case kPhScatter: p_scatter(A, I.a, I.b); break;
      case kPhSort: p_sort(A, I.a, I.b); break;
      default:
        for (int t = I.a; t < I.b; ++t) p_force<SPH>(A, t, sm.list);
        break;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (t == 0) {
      __hip_atomic_fetch_add(&A->arrive[I.box * kPhases + I.phase], 1, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
      s_item = atomicAdd(A->head, 1);
    }
    __syncthreads();
    it = __builtin_amdgcn_readfirstlane(s_item);
  }
}

// Before a persistent step: clear the arrival counters and the queue counter
// (a kernel, so that a captured graph holds no memset node) and advance the
// force evaluation index k.
__global__ void k_persist_prep(int32_t *arrive, int n, int32_t *head, unsigned long long *dk) {
  for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) arrive[i] = 0;
  if (threadIdx.x == 0) {
    *head = 0;
    *dk += 1ull;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_pack(hipStream_t s, int64_t n, const float *pos, const float *vel,
                       const uint32_t *gid, const int64_t *rows, float4 *pos4, float4 *vel4,
                       float4 *vt4, float4 *frc4) {
  if (n <= 0) return hipSuccess;
  k_pack<<<grid_for(n), kBlock, 0, s>>>(n, pos, vel, gid, rows, pos4, vel4, vt4, frc4);
  return hipGetLastError();
}

hipError_t launch_bin(hipStream_t s, const KGeom &G, int64_t cell_off, int64_t n,
                      const float4 *pos4, int32_t *cell_of, int32_t *rank_of, int32_t *count) {
  if (n <= 0) return hipSuccess;
  k_bin<<<grid_for(n), kBlock, 0, s>>>(G, cell_off, n, pos4, cell_of, rank_of, count);
  return hipGetLastError();
}

hipError_t launch_scan_reduce(hipStream_t s, int64_t ncell, const int32_t *count, int32_t *bsum) {
  k_scan_reduce<<<scan_blocks(ncell), kScanThreads, 0, s>>>(ncell, count, bsum);
  return hipGetLastError();
}

hipError_t launch_scan_down(hipStream_t s, int64_t ncell, int32_t *count, int32_t *start,
                            const int32_t *bsum, const int32_t *wstart, int32_t *start_all,
                            int32_t *fluid_off) {
  k_scan_down<<<scan_blocks(ncell), kScanThreads, 0, s>>>(ncell, count, start, bsum, wstart,
                                                          start_all, fluid_off);
  return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t s, int64_t n, const int32_t *cell_of,
                          const int32_t *rank_of, const int32_t *start, int32_t *idx,
                          int64_t nw, const int32_t *wcell, const int32_t *wstart,
                          const int32_t *start_all, int32_t *idx_all,
                          unsigned long long *dk) {
  if (!idx_all) nw = 0;
  if (nw > 0 && (!wcell || !wstart || !start_all)) return hipErrorInvalidValue;
  const int64_t total = std::max<int64_t>(n + nw, dk ? 1 : 0);
  if (total <= 0) return hipSuccess;
  k_scatter<<<grid_for(total), kBlock, 0, s>>>(n, cell_of, rank_of, start, idx, nw, wcell, wstart,
                                               start_all, idx_all, dk);
  return hipGetLastError();
}

hipError_t launch_quant_runs(hipStream_t s, int64_t n, const int32_t *idx_all,
                             const float4 *pos4, uint32_t *cq) {
  if (n <= 0) return hipSuccess;
  if (!idx_all || !pos4 || !cq) return hipErrorInvalidValue;
  k_quant_runs<<<grid_for(n), kBlock, 0, s>>>(n, idx_all, pos4, cq);
  return hipGetLastError();
}

hipError_t launch_sort_cells(hipStream_t s, int64_t ncell, const int32_t *start, int32_t *idx,
                             const float4 *key4, const int32_t *fluid_off, int32_t *idx_all) {
  if (key4)
    k_sort_cells<true><<<grid_for(ncell), kBlock, 0, s>>>(ncell, start, idx, key4, fluid_off,
                                                        idx_all);
  else
    k_sort_cells<false><<<grid_for(ncell), kBlock, 0, s>>>(ncell, start, idx, key4, fluid_off,
                                                         idx_all);
  return hipGetLastError();
}

hipError_t launch_sort_wall_cells(hipStream_t s, int64_t ncell, const int32_t *start,
                                  int32_t *idx, int32_t *cell_out) {
  k_sort_wall_cells<<<grid_for(ncell), kBlock, 0, s>>>(ncell, start, idx, cell_out);
  return hipGetLastError();
}

hipError_t launch_wall_move_bin(hipStream_t s, const KGeom &G, float hdt, float dt, int move,
                                int64_t cell_off, int64_t nw, const float4 *walls_in,
                                const float4 *vt_in, float4 *walls_out, float4 *vt_out,
                                int32_t *cell_of, int32_t *rank_of, int32_t *count) {
  if (nw <= 0) return hipSuccess;
  k_wall_move_bin<<<grid_for(nw), kBlock, 0, s>>>(G, hdt, dt, move, cell_off, nw, walls_in, vt_in,
                                                  walls_out, vt_out, cell_of, rank_of, count);
  return hipGetLastError();
}

hipError_t launch_import_walls(hipStream_t s, int64_t nw, float4 *walls, const float *pos) {
  if (nw <= 0) return hipSuccess;
  k_import_walls<<<grid_for(nw), kBlock, 0, s>>>(nw, walls, pos);
  return hipGetLastError();
}

hipError_t launch_set_pad(hipStream_t s, float4 *pos4, float4 *vt4, int32_t *slack, int32_t pad) {
  k_set_pad<<<1, 1, 0, s>>>(pos4, vt4, slack, pad);
  return hipGetLastError();
}

hipError_t launch_cells(hipStream_t s, const KGeom &G, int64_t cell_off, int64_t n,
                        const float4 *pos4, int32_t *cell) {
  if (n <= 0) return hipSuccess;
  k_cells<<<grid_for(n), kBlock, 0, s>>>(G, cell_off, n, pos4, cell);
  return hipGetLastError();
}

hipError_t launch_permute(hipStream_t s, int64_t n, const int32_t *idx, const float4 *a_in,
                          float4 *a_out, const float4 *b_in, float4 *b_out, const float4 *c_in,
                          float4 *c_out) {
  if (n <= 0) return hipSuccess;
  k_permute<<<grid_for(n), kBlock, 0, s>>>(n, idx, a_in, a_out, b_in, b_out, c_in, c_out);
  return hipGetLastError();
}

hipError_t launch_cube_mask(hipStream_t s, const KGeom &G, const void *grid, int grid_f64,
                            int64_t nwords, uint32_t *bits) {
  if (grid_f64)
    k_cube_mask<double><<<grid_for(nwords), kBlock, 0, s>>>(G, (const double *)grid, nwords, bits);
  else
    k_cube_mask<float><<<grid_for(nwords), kBlock, 0, s>>>(G, (const float *)grid, nwords, bits);
  return hipGetLastError();
}

hipError_t launch_count_flagged(hipStream_t s, const KGeom &G, int grid_f64, int64_t nf,
                                const float4 *pos4, const uint32_t *bits,
                                unsigned long long *out) {
  if (nf <= 0) return hipSuccess;
  if (grid_f64)
    k_count_flagged<double><<<grid_for(nf), kBlock, 0, s>>>(G, nf, pos4, bits, out);
  else
    k_count_flagged<float><<<grid_for(nf), kBlock, 0, s>>>(G, nf, pos4, bits, out);
  return hipGetLastError();
}

hipError_t launch_check_grid(hipStream_t s, const void *grid, int grid_f64, int64_t count,
                             Status *st) {
  unsigned blocks = grid_for(count);
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) return hipSuccess;
  if (grid_f64)
    k_check_grid<double><<<blocks, kBlock, 0, s>>>((const double *)grid, count, st);
  else
    k_check_grid<float><<<blocks, kBlock, 0, s>>>((const float *)grid, count, st);
  return hipGetLastError();
}

hipError_t launch_check_phi(hipStream_t s, const KGeom &G, const void *grid, int grid_f64,
                            int64_t n, const float4 *pos4, Status *st) {
  if (n <= 0) return hipSuccess;
  if (grid_f64)
    k_check_phi<double><<<grid_for(n), kBlock, 0, s>>>(G, (const double *)grid, n, pos4, st);
  else
    k_check_phi<float><<<grid_for(n), kBlock, 0, s>>>(G, (const float *)grid, n, pos4, st);
  return hipGetLastError();
}

// Grid of 8k blocks covering n items with the XCD mapping of xcd_block().
inline unsigned xcd_grid(int64_t n, int block) {
  const int64_t nb = (n + block - 1) / block;
  return (unsigned)(((nb + 7) / 8) * 8);
}

hipError_t launch_build_quad(hipStream_t s, const KGeom &G, const void *grid, int grid_f64,
                             void *quad) {
  const int64_t nodes = (int64_t)G.ng[0] * G.ng[1] * G.ng[2];
  if (nodes <= 0) return hipSuccess;
  if (grid_f64)
    k_build_quad<double><<<grid_for(nodes), kBlock, 0, s>>>(G, (const double *)grid, nodes,
                                                            (double4 *)quad);
  else
    k_build_quad<float><<<grid_for(nodes), kBlock, 0, s>>>(G, (const float *)grid, nodes,
                                                           (float4 *)quad);
  return hipGetLastError();
}

hipError_t launch_integrate(hipStream_t s, int ppt, const Box *boxes, const Tile *tiles,
                            int ntiles, float4 *pos4, const float4 *vel4, const float4 *frc4,
                            float4 *vt4, int32_t *cell_of, int32_t *rank_of, int32_t *count,
                            const uint32_t *bits, int use_mask, const void *quad, int grid_f64,
                            Status *st, int64_t NF, const int32_t *wcstart, int reflect) {
  if (ntiles <= 0) return hipSuccess;
  const unsigned nb = (unsigned)(((ntiles + 7) / 8) * 8);
#define DPD_INTEGRATE(T, K, R)                                                                   \
  k_integrate<T, K, R><<<nb, kBlock, 0, s>>>(boxes, tiles, ntiles, pos4, vel4, frc4, vt4,       \
                                             cell_of, rank_of, count, bits, use_mask,           \
                                             (const typename PhiQuad<T>::type *)quad, st, NF,   \
                                             wcstart)
#define DPD_INTEGRATE_T(T, K) \
  if (reflect) DPD_INTEGRATE(T, K, true); else DPD_INTEGRATE(T, K, false)
  if (ppt != 1 && ppt != 2 && ppt != 4) return hipErrorInvalidValue;
  if (grid_f64) {
    if (ppt == 1) { DPD_INTEGRATE_T(double, 1); }
    else if (ppt == 2) { DPD_INTEGRATE_T(double, 2); }
    else { DPD_INTEGRATE_T(double, 4); }
  } else {
    if (ppt == 1) { DPD_INTEGRATE_T(float, 1); }
    else if (ppt == 2) { DPD_INTEGRATE_T(float, 2); }
    else { DPD_INTEGRATE_T(float, 4); }
  }
#undef DPD_INTEGRATE_T
#undef DPD_INTEGRATE
  return hipGetLastError();
}

hipError_t launch_force(hipStream_t s, int block, const Box *boxes, const Tile *tiles,
                        int ntiles, int64_t NF, int32_t pad, int32_t ncell_all, int init,
                        const float4 *pos4,
                        const float4 *vt4, const float4 *vel4, const float4 *frc4,
                        const int32_t *idx, const int32_t *idx_all, const int32_t *start_all,
                        const uint32_t *cq,
                        float4 *pos_out, float4 *vel_out, float4 *frc_out,
                        const unsigned long long *dk, Status *st, int sph) {
  if (ntiles <= 0) return hipSuccess;
  if (!cq) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)(((ntiles + 7) / 8) * 8);
#define DPD_FORCE(I, BS, S)                                                                      \
  k_force<I, BS, S><<<nb, BS, 0, s>>>(boxes, tiles, ntiles, NF, pad, ncell_all, pos4, vt4, vel4, \
                                      frc4, idx, idx_all, start_all, cq, pos_out, vel_out,       \
                                      frc_out, dk, st)
#define DPD_FORCE_S(I, BS) \
  if (sph) DPD_FORCE(I, BS, true); else DPD_FORCE(I, BS, false)
  if (block == 128) {
    if (init) { DPD_FORCE_S(true, 128); } else { DPD_FORCE_S(false, 128); }
  } else {
    if (init) { DPD_FORCE_S(true, 256); } else { DPD_FORCE_S(false, 256); }
  }
#undef DPD_FORCE_S
#undef DPD_FORCE
  return hipGetLastError();
}

hipError_t launch_pairs(hipStream_t s, const KGeom &G, const KParams &P, int64_t cell_off,
                        int64_t first, int64_t nf, const float4 *pos4, const int32_t *idx,
                        const int32_t *idx_all, const int32_t *start_all, uint32_t *pairs,
                        int64_t cap, unsigned long long *counter) {
  if (nf <= 0) return hipSuccess;
  k_pairs<<<grid_for(nf), kBlock, 0, s>>>(G, P, (int)cell_off, first, nf, pos4, idx, idx_all,
                                          start_all, pairs, cap, counter);
  return hipGetLastError();
}

hipError_t launch_pair_random(hipStream_t s, uint64_t seed, uint64_t k, uint32_t replica,
                              const uint32_t *gi, const uint32_t *gj, int64_t n, uint32_t *words,
                              float *xi) {
  if (n <= 0) return hipSuccess;
  const uint32_t khi = ((uint32_t)(k >> 32) & 0xFFFFu) | (replica << 16);
  k_pair_random<<<grid_for(n), kBlock, 0, s>>>((uint32_t)seed, (uint32_t)(seed >> 32),
                                                (uint32_t)k, khi, gi, gj, n, words, xi);
  return hipGetLastError();
}

hipError_t launch_export(hipStream_t s, const KGeom &G, int64_t n, const float4 *pos4,
                         const float4 *vel4, const float4 *frc4, int wall, float *pos,
                         float *vel, float *frc, int32_t *events, int32_t *cell_of) {
  if (n <= 0) return hipSuccess;
  k_export<<<grid_for(n), kBlock, 0, s>>>(G, n, pos4, vel4, frc4, wall, pos, vel, frc, events,
                                          cell_of);
  return hipGetLastError();
}

hipError_t launch_import(hipStream_t s, int64_t nf, float4 *pos4, float4 *vel4, float4 *frc4,
                         const float *pos, const float *vel, const float *frc) {
  if (nf <= 0) return hipSuccess;
  k_import<<<grid_for(nf), kBlock, 0, s>>>(nf, pos4, vel4, frc4, pos, vel, frc);
  return hipGetLastError();
}

hipError_t launch_profile(hipStream_t s, const KGeom &G, int64_t nf, const float4 *pos4,
                          const float4 *vel4, int axis, int nbins, double *out) {
  if (nf <= 0) return hipSuccess;
  k_profile<<<grid_for(nf), kBlock, 0, s>>>(G, nf, pos4, vel4, axis, nbins, out);
  return hipGetLastError();
}

hipError_t launch_step_persistent(hipStream_t s, const PArgs *args, int nitems, int blocks,
                                  int32_t *arrive, int narrive, int32_t *head,
                                  unsigned long long *dk, int grid_f64, int ppt, int reflect,
                                  int sph) {
  if (nitems <= 0) return hipSuccess;
  k_persist_prep<<<1, 256, 0, s>>>(arrive, narrive, head, dk);
  const unsigned nb = (unsigned)std::max(1, std::min(nitems, blocks));
#define DPD_PERSIST(T, P, R, S) k_step_persistent<T, P, R, S><<<nb, kBlock, 0, s>>>(args)
#define DPD_PERSIST_S(T, P, R) \
  if (sph) DPD_PERSIST(T, P, R, true); else DPD_PERSIST(T, P, R, false)
#define DPD_PERSIST_R(T, P) \
  if (reflect) { DPD_PERSIST_S(T, P, true); } else { DPD_PERSIST_S(T, P, false); }
#define DPD_PERSIST_P(T) \
  if (ppt == 1) { DPD_PERSIST_R(T, 1); } else { DPD_PERSIST_R(T, 2); }
  if (grid_f64) {
    DPD_PERSIST_P(double);
  } else {
    DPD_PERSIST_P(float);
  }
#undef DPD_PERSIST_P
#undef DPD_PERSIST_R
#undef DPD_PERSIST_S
#undef DPD_PERSIST
  return hipGetLastError();
}

namespace {
template <typename T, int P, bool R, bool S>
int occupancy_of() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_persistent<T, P, R, S>, kBlock, 0) !=
      hipSuccess)
    return -1;
  return n;
}
template <typename T, int P>
int occupancy_rs(int reflect, int sph) {
  if (reflect) return sph ? occupancy_of<T, P, true, true>() : occupancy_of<T, P, true, false>();
  return sph ? occupancy_of<T, P, false, true>() : occupancy_of<T, P, false, false>();
}
}  // namespace

int persistent_blocks_per_cu(int ppt, int grid_f64, int reflect, int sph) {
  if (grid_f64)
    return ppt == 1 ? occupancy_rs<double, 1>(reflect, sph) : occupancy_rs<double, 2>(reflect, sph);
  return ppt == 1 ? occupancy_rs<float, 1>(reflect, sph) : occupancy_rs<float, 2>(reflect, sph);
}

hipError_t launch_fill_zero(hipStream_t s, void *p, size_t bytes) {
  if (bytes == 0) return hipSuccess;
  const size_t words = (bytes + 3) / 4;
  unsigned blocks = (unsigned)((words + kBlock - 1) / kBlock);
  if (blocks > 4096) blocks = 4096;
  k_fill_zero<<<blocks, kBlock, 0, s>>>((uint32_t *)p, words);
  return hipGetLastError();
}

hipError_t launch_valu_probe(hipStream_t s, int kind, int64_t waves, int iters, float *out) {
  const unsigned blocks = (unsigned)((waves * 64 + 255) / 256);
  if (kind == 0) k_valu_probe<0><<<blocks, 256, 0, s>>>(iters, out);
  else if (kind == 1) k_valu_probe<1><<<blocks, 256, 0, s>>>(iters, out);
  else if (kind == 2) k_valu_probe<2><<<blocks, 256, 0, s>>>(iters, out);
  else k_valu_probe<3><<<blocks, 256, 0, s>>>(iters, out);
  return hipGetLastError();
}

hipError_t launch_copy(hipStream_t s, void *dst, const void *src, size_t bytes) {
  if (bytes == 0) return hipSuccess;
  if ((bytes % 16) == 0 && ((uintptr_t)dst % 16) == 0 && ((uintptr_t)src % 16) == 0) {
    const size_t n16 = bytes / 16;
    unsigned blocks = (unsigned)((n16 + kBlock - 1) / kBlock);
    if (blocks > 8192) blocks = 8192;
    k_copy16<<<blocks, kBlock, 0, s>>>((float4 *)dst, (const float4 *)src, n16);
  } else {
    k_copy1<<<grid_for((int64_t)bytes), kBlock, 0, s>>>((uint8_t *)dst, (const uint8_t *)src,
                                                       bytes);
  }
  return hipGetLastError();
}

}  // namespace dpd
