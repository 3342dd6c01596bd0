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
// Data flow: a block owns a 64 x 8 column of nodes and marches it through a
// chunk of 32 z planes.  phi planes z-1 .. z+2 (with a two-node x/y halo)
// live in an LDS ring of four, the normal planes z-1 .. z+1 (one-node halo)
// in a ring of three; each z step loads one phi plane, computes one normal
// plane and updates one plane.  Each node's normal is computed once per
// block (plus the halo), and phi is read from HBM about once per node (the
// x/y halo and the three planes before a chunk come from L2).  Tiles are
// ordered so that neighbouring tiles run on the same XCD and share its L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace dpd {
namespace {

constexpr int kBX = 64, kBY = 8, kTZ = 32;
constexpr int kThreads = kBX * kBY;
constexpr int kPW = kBX + 4, kPH = kBY + 4;   // phi plane with a 2-node halo
constexpr int kNW = kBX + 2, kNH = kBY + 2;   // normal plane with a 1-node halo
constexpr int kPPlane = kPW * kPH;
constexpr int kNPlane = kNW * kNH;
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

__device__ __forceinline__ float inv_sqrt(float v) { return rsqrtf(v); }
__device__ __forceinline__ double inv_sqrt(double v) { return 1.0 / sqrt(v); }

__device__ __forceinline__ void res_max(void *res, float v) {
  atomicMax((unsigned int *)res, __float_as_uint(v));
}
__device__ __forceinline__ void res_max(void *res, double v) {
  atomicMax((unsigned long long *)res, (unsigned long long)__double_as_longlong(v));
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_phi_relax(RelaxArgs<T> a) {
  __shared__ T sphi[4][kPPlane];
  __shared__ T sn[3][3][kNPlane];   // [ring slot][component][node]

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

  // this thread's share of a phi plane: LDS slot and wrapped in-plane offset
  int lslot[kLoadSlots], loff[kLoadSlots];
#pragma unroll
  for (int s = 0; s < kLoadSlots; ++s) {
    const int m = tid + s * kThreads;
    lslot[s] = -1;
    loff[s] = 0;
    if (m < kPPlane) {
      const int ly = m / kPW, lx = m - ly * kPW;
      lslot[s] = m;
      loff[s] = wrap(y0 + ly - 2, a.ny) * a.nx + wrap(x0 + lx - 2, a.nx);
    }
  }
  auto load_plane = [&](int z) {   // phi plane z into ring slot z mod 4
    const T *p = a.src + (size_t)wrap(z, a.nz) * plane;
    T *d = sphi[z & 3];
#pragma unroll
    for (int s = 0; s < kLoadSlots; ++s)
      if (lslot[s] >= 0) d[lslot[s]] = p[loff[s]];
  };
  auto normals = [&](int z) {      // unit normal on plane z into ring slot z mod 3
    const T *pm = sphi[(z - 1) & 3], *p0 = sphi[z & 3], *pp = sphi[(z + 1) & 3];
    T *n = &sn[(z + 3) % 3][0][0];
    for (int m = tid; m < kNPlane; m += kThreads) {
      const int ly = m / kNW, lx = m - ly * kNW;
      const int c = (ly + 1) * kPW + lx + 1;
      const T ux = a.gx * (p0[c + 1] - p0[c - 1]);
      const T uy = a.gy * (p0[c + kPW] - p0[c - kPW]);
      const T uz = a.gz * (pp[c] - pm[c]);
      const T inv = inv_sqrt(fmax(ux * ux + uy * uy + uz * uz, a.delta2));
      n[m] = ux * inv;
      n[kNPlane + m] = uy * inv;
      n[2 * kNPlane + m] = uz * inv;
    }
  };

  const int tx = tid % kBX, ty = tid / kBX;
  const int x = x0 + tx, y = y0 + ty;
  const bool mine = x < a.nx && y < a.ny;
  T rmax = T(0);
  auto update = [&](int z) {
    if (!mine) return;
    const T *pm = sphi[(z - 1) & 3], *p0 = sphi[z & 3], *pp = sphi[(z + 1) & 3];
    const int c = (ty + 2) * kPW + tx + 2;
    const T ph = p0[c];
    const T xm = p0[c - 1], xp = p0[c + 1], ym = p0[c - kPW], yp = p0[c + kPW];
    const T zm = pm[c], zp = pp[c];
    const T lap = a.cx * (xp - T(2) * ph + xm) + a.cy * (yp - T(2) * ph + ym) +
                  a.cz * (zp - T(2) * ph + zm);
    const T ux = a.gx * (xp - xm), uy = a.gy * (yp - ym), uz = a.gz * (zp - zm);
    const T gm = sqrt(ux * ux + uy * uy + uz * uz);
    const int cn = (ty + 1) * kNW + tx + 1;
    const T *n0 = &sn[(z + 3) % 3][0][0];
    const T *nm = &sn[(z + 2) % 3][2][0], *np = &sn[(z + 4) % 3][2][0];
    const T kap = a.gx * (n0[cn + 1] - n0[cn - 1]) +
                  a.gy * (n0[kNPlane + cn + kNW] - n0[kNPlane + cn - kNW]) +
                  a.gz * (np[cn] - nm[cn]);
    const T rhs = lap + ph * (T(1) - ph * ph) - kap * gm;
    a.dst[(size_t)z * plane + (size_t)y * a.nx + x] = ph + a.dtau * rhs;
    rmax = fmax(rmax, fabs(rhs));
  };

  // prologue: phi planes z0-2 .. z0+1, normals on z0-1 and z0
  for (int z = z0 - 2; z <= z0 + 1; ++z) load_plane(z);
  __syncthreads();
  normals(z0 - 1);
  normals(z0);
  __syncthreads();
  for (int z = z0; z < z1; ++z) {
    load_plane(z + 2);   // overwrites plane z-2, last read before the previous barrier
    __syncthreads();
    normals(z + 1);      // overwrites normals of z-2, no longer read
    __syncthreads();
    update(z);
    __syncthreads();     // plane z-1 is overwritten by the next load
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
