// Pseudo-time relaxation of the phase field (Sec. II.B, Eq. 15):
//   d phi / d t' = lap' phi + phi (1 - phi^2) - kappa |grad' phi|,
//   kappa = div'(grad' phi / |grad' phi|),  grad' = eps grad,
// one explicit Euler step per launch on the periodic node-centred grid of
// the DPD step (x fastest, then y, then z).
//
// Finite differences: the compact 7-point Laplacian, central differences for
// grad' phi and for the divergence of the unit normal n = grad' phi /
// max(|grad' phi|, delta), delta = 0.01 (n goes linearly to zero where phi is
// flat instead of pointing along rounding noise).
//
// Data flow: a block owns a 64 x 16 column of nodes and marches it through a
// chunk of 64 z planes.  phi planes (with a two-node x/y halo) live in an
// LDS ring of four; the x and y components of the normal (one-node halo) in
// a ring of two planes, its z component in the owning thread's registers
// (the divergence needs n_z only in the node's own column).  Each z step
// stores one phi plane into the ring, prepares the
// next plane (each thread's own nodes: the Laplacian and reaction terms and
// |grad' phi| into registers, the unit normal into LDS; the halo normals by
// the first threads) and updates the current plane from its registers and
// the divergence of the normals, with one barrier.  The global loads of a
// plane are issued one step before its LDS store, so their latency overlaps
// a step of work.  Each node's stencil is read once, phi is read from HBM
// about once per node (the x/y halo and the planes before a chunk come from
// L2), and tiles are ordered so that neighbouring tiles run on the same XCD
// and share its L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace dpd {
namespace {

constexpr int kBX = 64, kBY = 16, kTZ = 64;
constexpr int kThreads = 512;
constexpr int kRows = kBY * kBX / kThreads;   // nodes per thread in a plane (rows ty, ty + 4)
constexpr int kRing = 4;                      // phi planes z-1 .. z+2 at step z
constexpr int kPW = kBX + 4, kPH = kBY + 4;   // phi plane with a 2-node halo
constexpr int kNW = kBX + 2, kNH = kBY + 2;   // normal plane with a 1-node halo
constexpr int kPPlane = kPW * kPH;
constexpr int kNPlane = kNW * kNH;
constexpr int kHalo = kNPlane - kBX * kBY;    // normal nodes outside the tile
constexpr int kLoadSlots = (kPPlane + kThreads - 1) / kThreads;

template <typename T>
struct RelaxArgs {
  const T *src;
  T *dst;
  int32_t nx, ny, nz;
  int32_t tiles_x, tiles_y;
  uint32_t tiles;
  T cx, cy, cz;   // eps^2 / h_a^2
  T gx, gy, gz;   // eps / (2 h_a)
  T delta2;
  T dtau;
  void *res;      // max |rhs| as ordered bits (non-negative values), or null
};

__device__ __forceinline__ int wrap(int g, int n) {
  while (g < 0) g += n;
  while (g >= n) g -= n;
  return g;
}

// float: the hardware square root and reciprocal square root (about 1 ulp);
// the rsq argument is at least delta^2, the sqrt argument is a sum of squares
__device__ __forceinline__ float fast_sqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ float fast_rsqrt(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double fast_sqrt(double v) { return sqrt(v); }
__device__ __forceinline__ double fast_rsqrt(double v) { return 1.0 / sqrt(v); }

__device__ __forceinline__ void res_max(void *res, float v) {
  atomicMax((unsigned int *)res, __float_as_uint(v));
}
__device__ __forceinline__ void res_max(void *res, double v) {
  atomicMax((unsigned long long *)res, (unsigned long long)__double_as_longlong(v));
}

// Per step z the block (1) stores phi plane z+2, fetched a step earlier, (2)
// prepares plane z+1: for its own nodes the Laplacian and reaction terms,
// |grad' phi|, phi and the normal's z component stay in registers and the
// normal's x and y components go to LDS; the 148 normal nodes of the halo
// are computed by the first threads; (3) updates plane z from the registers
// prepared a step earlier and the divergence of the normals.  The
// divergence needs n_z only in a node's own column (planes z-1 and z+1), so
// n_z never leaves the thread.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_phi_relax(RelaxArgs<T> a) {
  __shared__ T sphi[kRing * kPPlane];
  __shared__ T sn[2 * 2 * kNPlane];   // [ring slot][x, y component][node]

  // tile of this block: the blocks of one XCD (dispatch is round-robin over
  // the eight XCDs) take a contiguous range of tiles
  const uint32_t b = blockIdx.x, q = a.tiles / 8, r = a.tiles % 8;
  const uint32_t xcd = b % 8, t = xcd * q + min(xcd, r) + b / 8;
  const int tix = (int)(t % (uint32_t)a.tiles_x);
  const uint32_t rest = t / (uint32_t)a.tiles_x;
  const int tiy = (int)(rest % (uint32_t)a.tiles_y), tiz = (int)(rest / (uint32_t)a.tiles_y);
  const int x0 = tix * kBX, y0 = tiy * kBY, z0 = tiz * kTZ;
  const int z1 = min(z0 + kTZ, a.nz);
  const int tid = threadIdx.x;
  const size_t plane = (size_t)a.nx * (size_t)a.ny;

  // this thread's share of a phi plane: LDS index and wrapped in-plane
  // offset.  Only the last slot can fall past the plane; there it repeats
  // the thread's previous slot (same address, same value), so the loads and
  // stores need no guard.
  static_assert(kPPlane > (kLoadSlots - 1) * kThreads, "only the last load slot is partial");
  static_assert(kHalo <= kThreads, "one halo normal per thread at most");
  int lslot[kLoadSlots], loff[kLoadSlots];
#pragma unroll
  for (int s = 0; s < kLoadSlots; ++s) {
    int m = tid + s * kThreads;
    if (m >= kPPlane) m -= kThreads;
    const int ly = m / kPW, lx = m - ly * kPW;
    lslot[s] = m;
    loff[s] = wrap(y0 + ly - 2, a.ny) * a.nx + wrap(x0 + lx - 2, a.nx);
  }
  // this thread's halo normal (tid < kHalo): the rows above and below the
  // tile, then the columns left and right of it; its phi-plane centre
  const bool has_halo = tid < kHalo;
  int hn = 0, hc = 0;
  {
    int lx, ly;
    if (tid < kNW) {
      ly = 0, lx = tid;
    } else if (tid < 2 * kNW) {
      ly = kNH - 1, lx = tid - kNW;
    } else {
      const int k = tid - 2 * kNW;          // 0 .. 2 kBY - 1 for halo threads
      ly = 1 + (k >> 1), lx = (k & 1) ? kNW - 1 : 0;
    }
    hn = has_halo ? ly * kNW + lx : 0;
    hc = has_halo ? (ly + 1) * kPW + lx + 1 : kPW + 1;
  }

  T pre[kLoadSlots];
  auto fetch = [&](int zw) {       // global loads of phi plane zw (wrapped) into registers
    const T *p = a.src + (size_t)zw * plane;
#pragma unroll
    for (int s = 0; s < kLoadSlots; ++s) pre[s] = p[loff[s]];
  };
  auto store = [&](int base) {     // the fetched plane into the ring slot at base
#pragma unroll
    for (int s = 0; s < kLoadSlots; ++s) sphi[base + lslot[s]] = pre[s];
  };

  const int tx = tid % kBX, ty0 = tid / kBX;
  const int x = x0 + tx;
  const bool xin = x < a.nx;
  T rmax = T(0);
  // per own node k: phi on the planes below, at and above the plane being
  // prepared (om, o0, op), the prepared terms of the plane being updated
  // (cur_*) and of the next one (nxt_*), n_z on planes z-1, z and z+1
  T om[kRows], o0[kRows];
  T cur_ph[kRows], cur_base[kRows], cur_gm[kRows];
  T nxt_base[kRows], nxt_gm[kRows];
  T nz_m[kRows], nz_0[kRows], nz_p[kRows];
#pragma unroll
  for (int k = 0; k < kRows; ++k) nz_m[k] = nz_0[k] = nz_p[k] = T(0);
  auto prepare = [&](int pm, int p0, int pp, int nb) {
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int ty = ty0 + k * (kThreads / kBX);
      const int c = (ty + 2) * kPW + tx + 2;
      const T ph = o0[k], zm = om[k], zp = sphi[pp + c];
      const T xm = sphi[p0 + c - 1], xp = sphi[p0 + c + 1];
      const T ym = sphi[p0 + c - kPW], yp = sphi[p0 + c + kPW];
      const T lap = a.cx * (xp - T(2) * ph + xm) + a.cy * (yp - T(2) * ph + ym) +
                    a.cz * (zp - T(2) * ph + zm);
      const T ux = a.gx * (xp - xm), uy = a.gy * (yp - ym), uz = a.gz * (zp - zm);
      const T s2 = ux * ux + uy * uy + uz * uz;
      const T inv = fast_rsqrt(fmax(s2, a.delta2));
      const int m = (ty + 1) * kNW + tx + 1;
      sn[nb + m] = ux * inv;
      sn[nb + kNPlane + m] = uy * inv;
      nz_p[k] = uz * inv;
      nxt_base[k] = lap + ph * (T(1) - ph * ph);
      nxt_gm[k] = fast_sqrt(s2);
      om[k] = ph;
      o0[k] = zp;
    }
    if (has_halo) {
      // the halo needs n_x (columns) or n_y (rows) only; both are written
      const int c = hc;
      const T ux = a.gx * (sphi[p0 + c + 1] - sphi[p0 + c - 1]);
      const T uy = a.gy * (sphi[p0 + c + kPW] - sphi[p0 + c - kPW]);
      const T uz = a.gz * (sphi[pp + c] - sphi[pm + c]);
      const T inv = fast_rsqrt(fmax(ux * ux + uy * uy + uz * uz, a.delta2));
      sn[nb + hn] = ux * inv;
      sn[nb + kNPlane + hn] = uy * inv;
    }
  };
  // explicit Euler update of this thread's nodes of plane z from the
  // prepared terms, the normals' x and y components of plane z at n0 and
  // n_z of planes z-1 and z+1
  auto update = [&](T *zdst, int n0) {
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      // nodes past a ragged grid edge are computed from the wrapped values
      // in LDS like the others, but neither stored nor counted
      const int ty = ty0 + k * (kThreads / kBX);
      const int y = y0 + ty;
      const int cn = (ty + 1) * kNW + tx + 1;
      const T kap = a.gx * (sn[n0 + cn + 1] - sn[n0 + cn - 1]) +
                    a.gy * (sn[n0 + kNPlane + cn + kNW] - sn[n0 + kNPlane + cn - kNW]) +
                    a.gz * (nz_p[k] - nz_m[k]);
      const T rhs = cur_base[k] - kap * cur_gm[k];
      const bool in = xin && y < a.ny;
      // the new value is not read again in this launch: the nontemporal
      // hint lets its line leave the L2 before the planes that neighbouring
      // tiles still read as their halos
      if (in) __builtin_nontemporal_store(cur_ph[k] + a.dtau * rhs, &zdst[(size_t)y * a.nx + x]);
      rmax = in ? fmax(rmax, fabs(rhs)) : rmax;
    }
  };
  auto advance = [&]() {           // the prepared plane becomes the current one
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      cur_ph[k] = om[k];
      cur_base[k] = nxt_base[k];
      cur_gm[k] = nxt_gm[k];
      nz_m[k] = nz_0[k];
      nz_0[k] = nz_p[k];
    }
  };

  // ring slots (element offsets): phi planes z-1 .. z+2 at step z (s3 free),
  // normal x/y planes z (nc) and z+1 (nn)
  int s0 = 0, s1 = kPPlane, s2 = 2 * kPPlane, s3 = 3 * kPPlane;
  int nc = 0, nn = 2 * kNPlane;

  // prologue: phi planes z0-2 .. z0+1 (z0-2 in the slot that plane z0+2
  // takes next), z0+2 in flight; the thread's own phi on z0-2 and z0-1;
  // planes z0-1 and z0 prepared
  fetch(wrap(z0 - 2, a.nz));
  store(s3);
  fetch(wrap(z0 - 1, a.nz));
  store(s0);
  fetch(wrap(z0, a.nz));
  store(s1);
  fetch(wrap(z0 + 1, a.nz));
  store(s2);
  int zf = wrap(z0 + 2, a.nz);     // wrapped index of the plane in flight
  fetch(zf);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int c = (ty0 + k * (kThreads / kBX) + 2) * kPW + tx + 2;
    om[k] = sphi[s3 + c];
    o0[k] = sphi[s0 + c];
  }
  prepare(s3, s0, s1, nn);         // plane z0-1: its n_z is used, its n_x, n_y are not
  advance();
  prepare(s0, s1, s2, nc);         // plane z0
  advance();
  __syncthreads();                 // plane z0-2 (slot s3) is overwritten next
  T *zdst = a.dst + (size_t)z0 * plane;
  for (int z = z0; z < z1; ++z, zdst += plane) {
    // phi: s0 = z-1, s1 = z, s2 = z+1, s3 = free (plane z-2, last read by the
    // preparation of z-1 before the previous step's barriers)
    store(s3);
    zf = zf + 1 == a.nz ? 0 : zf + 1;   // plane z+3
    if (z + 1 < z1) fetch(zf);
    __syncthreads();
    // plane z+1 into the normal slot of z-1, last read by the update of z-1
    // (before this step's barrier); the update of z reads only the normals
    // of z, written before this step's barrier, and registers, so no second
    // barrier is needed
    prepare(s1, s2, s3, nn);
    update(zdst, nc);
    advance();
    const int f = s0;
    s0 = s1; s1 = s2; s2 = s3; s3 = f;
    const int g = nc;
    nc = nn; nn = g;
  }

  if (a.res) {
    // wave maximum, then one atomic per wave (non-negative values order as
    // their bit patterns; a NaN sorts above every finite value)
    for (int o = 32; o > 0; o >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, o));
    if ((tid & 63) == 0) res_max(a.res, rmax);
  }
}

template <typename T>
hipError_t launch_relax_t(hipStream_t s, const void *src, void *dst, const int32_t n[3],
                          const double coef[8], void *res) {
  RelaxArgs<T> a;
  a.src = (const T *)src;
  a.dst = (T *)dst;
  a.nx = n[0];
  a.ny = n[1];
  a.nz = n[2];
  a.tiles_x = (n[0] + kBX - 1) / kBX;
  a.tiles_y = (n[1] + kBY - 1) / kBY;
  const int tiles_z = (n[2] + kTZ - 1) / kTZ;
  a.tiles = (uint32_t)a.tiles_x * (uint32_t)a.tiles_y * (uint32_t)tiles_z;
  a.cx = (T)coef[0];
  a.cy = (T)coef[1];
  a.cz = (T)coef[2];
  a.gx = (T)coef[3];
  a.gy = (T)coef[4];
  a.gz = (T)coef[5];
  a.delta2 = (T)coef[6];
  a.dtau = (T)coef[7];
  a.res = res;
  k_phi_relax<T><<<a.tiles, kThreads, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace

int64_t phi_relax_blocks(const int32_t n[3]) {
  return (int64_t)((n[0] + kBX - 1) / kBX) * ((n[1] + kBY - 1) / kBY) * ((n[2] + kTZ - 1) / kTZ);
}

hipError_t launch_phi_relax(hipStream_t s, int f64, const void *src, void *dst,
                            const int32_t n[3], const double coef[8], void *res) {
  return f64 ? launch_relax_t<double>(s, src, dst, n, coef, res)
             : launch_relax_t<float>(s, src, dst, n, coef, res);
}

}  // namespace dpd
