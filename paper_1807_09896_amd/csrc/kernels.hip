// Kernels of one DPD time step with phase-field bounce-back on gfx950.
//
// Per-particle state lives in float4 arrays (16-byte loads and stores):
//   pos4 = (x, y, z, gid bits)   vel4 = (v, last event code bits)
//   frc4 = (f, 0)                vt4  = (predicted velocity, event code bits)
// Fluid particles are kept in cell-sorted order: the force kernel writes the
// state of slot s (the s-th particle of the cell list) to slot s of the next
// buffers, so each step's integrate kernel streams a nearly sorted array and
// the force kernel's gathers of neighbour cells hit consecutive addresses.
// Frozen wall particles are sorted by cell once, at create.
#include <hip/hip_runtime.h>

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

__global__ void k_copy1(uint8_t *__restrict__ dst, const uint8_t *__restrict__ src, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Counting sort into cells
// ---------------------------------------------------------------------------
__global__ void k_bin(const KGeom G, int64_t n, const float4 *__restrict__ pos4,
                      int32_t *__restrict__ cell_of, int32_t *__restrict__ rank_of,
                      int32_t *__restrict__ count) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float4 x = pos4[p];
  int cx, cy, cz;
  const int c = cell_index(G, x.x, x.y, x.z, cx, cy, cz);
  cell_of[p] = c;
  rank_of[p] = atomicAdd(&count[c], 1);
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

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(int64_t n,
                                                              const int32_t *__restrict__ count,
                                                              int32_t *__restrict__ bsum) {
  __shared__ int lds[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
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
  if (threadIdx.x == 0) bsum[blockIdx.x] = lds[0];
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(int nb, int32_t *__restrict__ bsum) {
  __shared__ int lds[kScanThreads];
  int carry = 0;
  for (int base = 0; base < nb; base += kScanThreads) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    int total;
    const int ex = block_exclusive_scan(v, lds, total);
    if (i < nb) bsum[i] = carry + ex;
    carry += total;
  }
}

// Each thread owns kScanItems consecutive cells; the block's cells are read
// through LDS so that global loads and stores stay coalesced.
__global__ __launch_bounds__(kScanThreads) void k_scan_down(int64_t n, int32_t *__restrict__ count,
                                                            int32_t *__restrict__ start,
                                                            const int32_t *__restrict__ bsum) {
  __shared__ int tile[kScanChunk + kScanChunk / 32];
  __shared__ int lds[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
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
  int ex = block_exclusive_scan(run, lds, total) + bsum[blockIdx.x];
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
    if (i < n) start[i] = tile[local + local / 32];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1)
    start[n] = bsum[blockIdx.x] + total;
}

__global__ void k_scatter(int64_t n, const int32_t *__restrict__ cell_of,
                          const int32_t *__restrict__ rank_of, const int32_t *__restrict__ start,
                          int32_t *__restrict__ idx) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  idx[start[cell_of[p]] + rank_of[p]] = (int32_t)p;
}

// Atomic ranks arrive in any order: sort each cell's run by storage index so
// that the cell list, and every sum over it, is deterministic.
__global__ void k_sort_cells(int64_t ncell, const int32_t *__restrict__ start,
                             int32_t *__restrict__ idx) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int a = start[c], b = start[c + 1];
  for (int i = a + 1; i < b; ++i) {
    const int v = idx[i];
    int j = i - 1;
    while (j >= a && idx[j] > v) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = v;
  }
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
template <typename T>
__global__ void k_mask(const KGeom G, const T *__restrict__ grid, double wx, double wy, double wz,
                       double hx, double hy, double hz, int64_t ncell, uint8_t *mask) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int cx = (int)(c % G.nc[0]);
  const int cy = (int)((c / G.nc[0]) % G.nc[1]);
  const int cz = (int)(c / ((int64_t)G.nc[0] * G.nc[1]));
  const int x0 = (int)floor(cx * wx / hx) - 1, x1 = (int)ceil((cx + 1) * wx / hx) + 1;
  const int y0 = (int)floor(cy * wy / hy) - 1, y1 = (int)ceil((cy + 1) * wy / hy) + 1;
  const int z0 = (int)floor(cz * wz / hz) - 1, z1 = (int)ceil((cz + 1) * wz / hz) + 1;
  const size_t nx = (size_t)G.ng[0], nxy = nx * (size_t)G.ng[1];
  uint8_t m = 0;
  for (int k = z0; k <= z1 && !m; ++k) {
    const size_t kk = (size_t)wrapi(k, G.ng[2]);
    for (int j = y0; j <= y1 && !m; ++j) {
      const T *row = grid + kk * nxy + (size_t)wrapi(j, G.ng[1]) * nx;
      for (int i = x0; i <= x1; ++i) {
        if (row[wrapi(i, G.ng[0])] < (T)0) {
          m = 1;
          break;
        }
      }
    }
  }
  mask[c] = m;
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
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_integrate(
    const KGeom G, const KParams P, int64_t nf, float4 *__restrict__ pos4,
    const float4 *__restrict__ vel4, const float4 *__restrict__ frc4, float4 *__restrict__ vt4,
    int32_t *__restrict__ cell_of, int32_t *__restrict__ rank_of, int32_t *__restrict__ count,
    const uint8_t *__restrict__ mask, int use_mask, const T *__restrict__ grid, Status *st) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nf) return;
  const float4 x = pos4[p];
  const float4 v = vel4[p];
  const float4 f = frc4[p];
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
  int cx, cy, cz;
  int c = cell_index(G, xs, ys, zs, cx, cy, cz);
  int event = 0;
  const bool look = !use_mask || mask[c];
  {
    // one atomic per wavefront for the lookup counter
    const unsigned long long act = __ballot(1);
    const unsigned long long hit = __ballot(look);
    if (__lane_id() == __ffsll((long long)act) - 1 && hit)
      atomicAdd(&st->lookups, (unsigned long long)__popcll(hit));
  }
  if (look) {
    const T phis = phi_at(grid, G, xs, ys, zs);
    if (phis < (T)0) {
      // Eq. 16-17: distances beyond and before the interface from atanh(phi)
      const T phit = phi_at(grid, G, x.x, x.y, x.z);
      const T lim = (T)1 - (T)0x1p-20;
      const T a1 = fmin(fmax(-phis, (T)0), lim);
      const T a0 = fmin(fmax(phit, (T)0), lim);
      const T c1 = atanh(a1), c0 = atanh(a0);
      const T sfrac = c1 > (T)0 ? c1 / (c0 + c1) : (T)0;
      const float k2 = (float)((T)2 * sfrac * (T)P.dt);
      float bx = wrap1(xs - k2 * v.x, G.L[0]);
      float by = wrap1(ys - k2 * v.y, G.L[1]);
      float bz = wrap1(zs - k2 * v.z, G.L[2]);
      if (phi_at(grid, G, bx, by, bz) < (T)0) {
        bx = x.x;
        by = x.y;
        bz = x.z;
        event = 2;
        atomicAdd(&st->fallback, 1ull);
      } else {
        event = 1;
        atomicAdd(&st->bounce, 1ull);
      }
      xs = bx;
      ys = by;
      zs = bz;
      vt = make_float4(-v.x, -v.y, -v.z, 0.f);
      c = cell_index(G, xs, ys, zs, cx, cy, cz);
    }
  }
  vt.w = __int_as_float(event);
  pos4[p] = make_float4(xs, ys, zs, x.w);
  vt4[p] = vt;
  cell_of[p] = c;
  rank_of[p] = atomicAdd(&count[c], 1);
}

// ---------------------------------------------------------------------------
// Pair force (Eq. 3-10), body force, velocity update
// ---------------------------------------------------------------------------
struct Acc {
  float x, y, z;
};

__device__ __forceinline__ void add_pair(Acc &acc, float dx, float dy, float dz, float r2,
                                         float dvx, float dvy, float dvz, float a,
                                         const KParams &P, uint32_t gi, uint32_t gj,
                                         uint32_t klo, uint32_t khi) {
  const float rinv = rsqrtf(r2);
  const float r = r2 * rinv;
  const float w = fmaxf(1.0f - r * P.inv_rc, 0.0f);
  const float ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
  const float edv = ex * dvx + ey * dvy + ez * dvz;
  const float xi = pair_gauss(gi, gj, klo, khi, P.key0, P.key1);
  const float mag = w * (a - P.gamma * w * edv + P.sigma_rdt * xi);
  acc.x += mag * ex;
  acc.y += mag * ey;
  acc.z += mag * ez;
}

template <bool INIT>
__global__ __launch_bounds__(kBlock) void k_force(
    const KGeom G, const KParams P, int64_t nf, const float4 *__restrict__ pos4,
    const float4 *__restrict__ vt4, const float4 *__restrict__ vel4,
    const float4 *__restrict__ frc4, const int32_t *__restrict__ idx,
    const int32_t *__restrict__ cstart, const float4 *__restrict__ wpos4,
    const int32_t *__restrict__ wcstart, float4 *__restrict__ pos_out,
    float4 *__restrict__ vel_out, float4 *__restrict__ frc_out, uint32_t klo, uint32_t khi,
    Status *st) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nf) return;
  const int i = idx[s];
  const float4 pi = pos4[i];
  const float4 vti = vt4[i];
  const uint32_t gi = __float_as_uint(pi.w);
  int cx, cy, cz;
  cell_index(G, pi.x, pi.y, pi.z, cx, cy, cz);
  Acc acc = {0.f, 0.f, 0.f};
  for (int oz = -1; oz <= 1; ++oz) {
    int qz = cz + oz;
    float sz = 0.f;
    if (qz < 0) { qz += G.nc[2]; sz = -G.L[2]; }
    else if (qz >= G.nc[2]) { qz -= G.nc[2]; sz = G.L[2]; }
    for (int oy = -1; oy <= 1; ++oy) {
      int qy = cy + oy;
      float sy = 0.f;
      if (qy < 0) { qy += G.nc[1]; sy = -G.L[1]; }
      else if (qy >= G.nc[1]) { qy -= G.nc[1]; sy = G.L[1]; }
      for (int ox = -1; ox <= 1; ++ox) {
        int qx = cx + ox;
        float sx = 0.f;
        if (qx < 0) { qx += G.nc[0]; sx = -G.L[0]; }
        else if (qx >= G.nc[0]) { qx -= G.nc[0]; sx = G.L[0]; }
        const int c = (qz * G.nc[1] + qy) * G.nc[0] + qx;
        const int f0 = cstart[c], f1 = cstart[c + 1];
        for (int t = f0; t < f1; ++t) {
          const int j = idx[t];
          if (j == i) continue;
          const float4 pj = pos4[j];
          const float dx = sub_nc(pi.x, add_nc(pj.x, sx));
          const float dy = sub_nc(pi.y, add_nc(pj.y, sy));
          const float dz = sub_nc(pi.z, add_nc(pj.z, sz));
          const float r2 = pair_r2(dx, dy, dz);
          if (r2 < P.rc2 && r2 > 0.0f) {
            const float4 vtj = vt4[j];
            add_pair(acc, dx, dy, dz, r2, vti.x - vtj.x, vti.y - vtj.y, vti.z - vtj.z, P.a_ff,
                     P, gi, __float_as_uint(pj.w), klo, khi);
          }
        }
        const int w0 = wcstart[c], w1 = wcstart[c + 1];
        for (int t = w0; t < w1; ++t) {
          const float4 pw = wpos4[t];
          const float dx = sub_nc(pi.x, add_nc(pw.x, sx));
          const float dy = sub_nc(pi.y, add_nc(pw.y, sy));
          const float dz = sub_nc(pi.z, add_nc(pw.z, sz));
          const float r2 = pair_r2(dx, dy, dz);
          if (r2 < P.rc2 && r2 > 0.0f)
            add_pair(acc, dx, dy, dz, r2, vti.x, vti.y, vti.z, P.a_fw, P, gi,
                     __float_as_uint(pw.w), klo, khi);
        }
      }
    }
  }
  const float fx = acc.x + P.g[0], fy = acc.y + P.g[1], fz = acc.z + P.g[2];
  const float4 vo = vel4[i];
  float4 vn;
  if (INIT) {
    vn = make_float4(vo.x, vo.y, vo.z, __int_as_float(0));
  } else {
    const int event = __float_as_int(vti.w);
    if (event) {
      vn = make_float4(vti.x, vti.y, vti.z, __int_as_float(event));
    } else {
      const float4 fo = frc4[i];
      vn = make_float4(vo.x + P.hdt * (fo.x + fx), vo.y + P.hdt * (fo.y + fy),
                       vo.z + P.hdt * (fo.z + fz), __int_as_float(0));
    }
  }
  if (!(isfinite(fx) && isfinite(fy) && isfinite(fz))) atomicAdd(&st->nonfinite, 1ull);
  pos_out[s] = pi;
  vel_out[s] = vn;
  frc_out[s] = make_float4(fx, fy, fz, 0.f);
}

// Interacting pairs with the same decision as the force kernel.
__global__ __launch_bounds__(kBlock) void k_pairs(
    const KGeom G, const KParams P, int64_t nf, const float4 *__restrict__ pos4,
    const int32_t *__restrict__ idx, const int32_t *__restrict__ cstart,
    const float4 *__restrict__ wpos4, const int32_t *__restrict__ wcstart, uint32_t *pairs,
    int64_t cap, unsigned long long *counter) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nf) return;
  const int i = idx[s];
  const float4 pi = pos4[i];
  const uint32_t gi = __float_as_uint(pi.w);
  int cx, cy, cz;
  cell_index(G, pi.x, pi.y, pi.z, cx, cy, cz);
  for (int oz = -1; oz <= 1; ++oz) {
    int qz = cz + oz;
    float sz = 0.f;
    if (qz < 0) { qz += G.nc[2]; sz = -G.L[2]; }
    else if (qz >= G.nc[2]) { qz -= G.nc[2]; sz = G.L[2]; }
    for (int oy = -1; oy <= 1; ++oy) {
      int qy = cy + oy;
      float sy = 0.f;
      if (qy < 0) { qy += G.nc[1]; sy = -G.L[1]; }
      else if (qy >= G.nc[1]) { qy -= G.nc[1]; sy = G.L[1]; }
      for (int ox = -1; ox <= 1; ++ox) {
        int qx = cx + ox;
        float sx = 0.f;
        if (qx < 0) { qx += G.nc[0]; sx = -G.L[0]; }
        else if (qx >= G.nc[0]) { qx -= G.nc[0]; sx = G.L[0]; }
        const int c = (qz * G.nc[1] + qy) * G.nc[0] + qx;
        for (int pass = 0; pass < 2; ++pass) {
          const int t0 = pass ? wcstart[c] : cstart[c];
          const int t1 = pass ? wcstart[c + 1] : cstart[c + 1];
          for (int t = t0; t < t1; ++t) {
            float4 pj;
            if (pass) {
              pj = wpos4[t];
            } else {
              const int j = idx[t];
              if (j == i) continue;
              pj = pos4[j];
            }
            const float dx = sub_nc(pi.x, add_nc(pj.x, sx));
            const float dy = sub_nc(pi.y, add_nc(pj.y, sy));
            const float dz = sub_nc(pi.z, add_nc(pj.z, sz));
            if (pair_r2(dx, dy, dz) < P.rc2) {
              const unsigned long long q = atomicAdd(counter, 1ull);
              if ((int64_t)q < cap) {
                pairs[2 * q] = gi;
                pairs[2 * q + 1] = __float_as_uint(pj.w);
              }
            }
          }
        }
      }
    }
  }
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

hipError_t launch_bin(hipStream_t s, const KGeom &G, int64_t n, const float4 *pos4,
                      int32_t *cell_of, int32_t *rank_of, int32_t *count) {
  if (n <= 0) return hipSuccess;
  k_bin<<<grid_for(n), kBlock, 0, s>>>(G, n, pos4, cell_of, rank_of, count);
  return hipGetLastError();
}

hipError_t launch_scan_reduce(hipStream_t s, int64_t ncell, const int32_t *count, int32_t *bsum) {
  k_scan_reduce<<<scan_blocks(ncell), kScanThreads, 0, s>>>(ncell, count, bsum);
  return hipGetLastError();
}

hipError_t launch_scan_top(hipStream_t s, int nblocks, int32_t *bsum) {
  k_scan_top<<<1, kScanThreads, 0, s>>>(nblocks, bsum);
  return hipGetLastError();
}

hipError_t launch_scan_down(hipStream_t s, int64_t ncell, int32_t *count, int32_t *start,
                            const int32_t *bsum) {
  k_scan_down<<<scan_blocks(ncell), kScanThreads, 0, s>>>(ncell, count, start, bsum);
  return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t s, int64_t n, const int32_t *cell_of,
                          const int32_t *rank_of, const int32_t *start, int32_t *idx) {
  if (n <= 0) return hipSuccess;
  k_scatter<<<grid_for(n), kBlock, 0, s>>>(n, cell_of, rank_of, start, idx);
  return hipGetLastError();
}

hipError_t launch_sort_cells(hipStream_t s, int64_t ncell, const int32_t *start, int32_t *idx) {
  k_sort_cells<<<grid_for(ncell), kBlock, 0, s>>>(ncell, start, idx);
  return hipGetLastError();
}

hipError_t launch_permute(hipStream_t s, int64_t n, const int32_t *idx, const float4 *a_in,
                          float4 *a_out, const float4 *b_in, float4 *b_out, const float4 *c_in,
                          float4 *c_out) {
  if (n <= 0) return hipSuccess;
  k_permute<<<grid_for(n), kBlock, 0, s>>>(n, idx, a_in, a_out, b_in, b_out, c_in, c_out);
  return hipGetLastError();
}

hipError_t launch_mask(hipStream_t s, const KGeom &G, const void *grid, int grid_f64,
                       double wx, double wy, double wz, double hx, double hy, double hz,
                       int64_t ncell, uint8_t *mask) {
  if (grid_f64)
    k_mask<double><<<grid_for(ncell), kBlock, 0, s>>>(G, (const double *)grid, wx, wy, wz, hx,
                                                      hy, hz, ncell, mask);
  else
    k_mask<float><<<grid_for(ncell), kBlock, 0, s>>>(G, (const float *)grid, wx, wy, wz, hx, hy,
                                                     hz, ncell, mask);
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

hipError_t launch_integrate(hipStream_t s, const KGeom &G, const KParams &P, int64_t nf,
                            float4 *pos4, const float4 *vel4, const float4 *frc4, float4 *vt4,
                            int32_t *cell_of, int32_t *rank_of, int32_t *count,
                            const uint8_t *mask, int use_mask, const void *grid, int grid_f64,
                            Status *st) {
  if (nf <= 0) return hipSuccess;
  if (grid_f64)
    k_integrate<double><<<grid_for(nf), kBlock, 0, s>>>(G, P, nf, pos4, vel4, frc4, vt4, cell_of,
                                                        rank_of, count, mask, use_mask,
                                                        (const double *)grid, st);
  else
    k_integrate<float><<<grid_for(nf), kBlock, 0, s>>>(G, P, nf, pos4, vel4, frc4, vt4, cell_of,
                                                       rank_of, count, mask, use_mask,
                                                       (const float *)grid, st);
  return hipGetLastError();
}

hipError_t launch_force(hipStream_t s, const KGeom &G, const KParams &P, int64_t nf, int init,
                        const float4 *pos4, const float4 *vt4, const float4 *vel4,
                        const float4 *frc4, const int32_t *idx, const int32_t *cstart,
                        const float4 *wpos4, const int32_t *wcstart, float4 *pos_out,
                        float4 *vel_out, float4 *frc_out, uint64_t k, Status *st) {
  if (nf <= 0) return hipSuccess;
  const uint32_t klo = (uint32_t)k;
  const uint32_t khi = ((uint32_t)(k >> 32) & 0xFFFFu) | (P.replica << 16);
  if (init)
    k_force<true><<<grid_for(nf), kBlock, 0, s>>>(G, P, nf, pos4, vt4, vel4, frc4, idx, cstart,
                                                  wpos4, wcstart, pos_out, vel_out, frc_out, klo,
                                                  khi, st);
  else
    k_force<false><<<grid_for(nf), kBlock, 0, s>>>(G, P, nf, pos4, vt4, vel4, frc4, idx, cstart,
                                                   wpos4, wcstart, pos_out, vel_out, frc_out,
                                                   klo, khi, st);
  return hipGetLastError();
}

hipError_t launch_pairs(hipStream_t s, const KGeom &G, const KParams &P, int64_t nf,
                        const float4 *pos4, const int32_t *idx, const int32_t *cstart,
                        const float4 *wpos4, const int32_t *wcstart, uint32_t *pairs,
                        int64_t cap, unsigned long long *counter) {
  if (nf <= 0) return hipSuccess;
  k_pairs<<<grid_for(nf), kBlock, 0, s>>>(G, P, nf, pos4, idx, cstart, wpos4, wcstart, pairs,
                                          cap, counter);
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

hipError_t launch_fill_zero(hipStream_t s, void *p, size_t bytes) {
  if (bytes == 0) return hipSuccess;
  const size_t words = (bytes + 3) / 4;
  unsigned blocks = (unsigned)((words + kBlock - 1) / kBlock);
  if (blocks > 4096) blocks = 4096;
  k_fill_zero<<<blocks, kBlock, 0, s>>>((uint32_t *)p, words);
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
