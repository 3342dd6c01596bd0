// Device-side building blocks of the DPD step for gfx950: launch-parameter
// structs, the counter-based random numbers, the discrete decisions (cell of
// a position, pair within the cutoff, phi < 0) and the trilinear phase field.
//
// Decisions are written with contraction disabled so that each FP32 (or FP64)
// operation rounds exactly once, in the order written; the physics arithmetic
// around them is free to contract.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpd {

// Geometry of one box, passed by value to kernels.
struct KGeom {
  float L[3];        // box edges (float32)
  float invw[3];     // fl32(ncell / L): cell decision scale
  int nc[3];         // cells per axis (>= 3)
  int ng[3];         // phi grid nodes per axis (x, y, z)
  float inv_h[3];    // fl32(1 / h) for an FP32 grid
  double inv_h64[3]; // 1 / h for an FP64 grid
  float h[3];        // grid spacing (float32), for gradients
};

// DPD parameters of one box (Eq. 4-10 and the Groot-Warren integrator).
struct KParams {
  float a_ff, a_fw;     // conservative amplitudes, fluid-fluid and fluid-wall
  float gamma;          // dissipative coefficient
  float sigma_rdt;      // sigma / sqrt(dt), sigma = sqrt(2 gamma kBT)
  float rc2;            // fl32(rc^2), the cutoff decision
  float inv_rc;         // 1 / rc
  float dt, hdt;        // dt and fl32(dt / 2)
  float lamdt;          // lambda * dt
  float g[3];           // body force on fluid particles
  float max_disp2;      // (half the smallest cell width)^2
  float dsig_rdt;       // d(sigma / sqrt(dt)) / d gamma = kBT / (sigma sqrt(dt)), 0 if sigma = 0
  uint32_t key0, key1;  // seed words
  uint32_t replica;
  uint32_t reflect;     // kReflectMoving | kReflectSpecular
  // conservative force of Eq. 22-24 (sph = 1): -cr P'(r inv_hr) + ca P'(r inv_ha)
  // by pair type, c = S / (pi h^4)
  uint32_t sph;
  float cr_ff, cr_fw, ca_ff, ca_fw;
  float inv_hr, inv_ha;
};

// Derivative of Eq. 23's cubic spline in v = r / h (3-D), without the
// prefactor: -3 v + 9/4 v^2 (v < 1), -3/4 (2 - v)^2 (v < 2), 0.
__device__ __forceinline__ float spline_dp(float v) {
  const float u = 2.0f - v;
  return v < 1.0f ? v * (2.25f * v - 3.0f) : (v < 2.0f ? -0.75f * u * u : 0.0f);
}

// How a fluid particle that crossed phi = 0 is reflected (Sec. II.C): the
// box's walls move (the velocity of the solid comes from the nearest wall
// particle), and specular instead of bounce-back reflection.
constexpr uint32_t kReflectMoving = 1u;
constexpr uint32_t kReflectSpecular = 2u;

// One box of a batch: its geometry and parameters, and where its slices lie
// in the concatenated arrays (a single box is a batch of one).
struct Box {
  KGeom G;
  KParams P;
  int64_t fo, nf;     // fluid slots [fo, fo + nf)
  int64_t wo, nw;     // walls at position index NF + [wo, wo + nw)
  int64_t co, ncell;  // global cells [co, co + ncell)
  int64_t go;         // first element of the box's phi grid
  int64_t bo;         // first word of the box's cube mask
};

// A run of consecutive particles of one box, the work of one block.
struct Tile {
  int32_t box;
  int32_t first;
  int32_t count;
  int32_t pad;
};

// A brick of cells of one box, the work of one block of the LDS-staged pair
// kernel: home cells [x0, x0 + sx) x [y0, y0 + sy) x [z0, z0 + sz), at most
// kBrickX x kBrickY x kBrickZ.
constexpr int kBrickX = 4, kBrickY = 4, kBrickZ = 4;
struct Brick {
  int32_t box;
  int32_t x0, y0, z0;
  int32_t sx, sy, sz;
  int32_t pad;
};

// Device status counters, read back by the host at sync points.
struct Status {
  unsigned long long bounce;     // bounce-backs by Eq. 17 (code 1)
  unsigned long long fallback;   // returns to the start position (code 2)
  unsigned long long unstable;   // displacement above half a cell
  unsigned long long nonfinite;  // non-finite positions or forces
  unsigned long long bad_phi;    // fluid particles with phi < 0 at create
  unsigned long long bad_grid;   // non-finite phi grid values at create
  unsigned long long lookups;    // phi evaluations at drifted positions
  unsigned long long stalled;    // persistent-step waits that hit their bound
};

// The persistent step (k_step_persistent): work items in queue order, each
// one block's work in one phase of one box.
enum PersistPhase { kPhIntegrate = 0, kPhReduce, kPhDown, kPhScatter, kPhSort, kPhForce, kPhases };
struct PItem {
  int32_t phase, box;
  int32_t a, b;   // tile range [a, b) (integrate, force), chunk index (reduce, down), or range [a, b)
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Ten rounds; each round
// takes the 64-bit products of two counter words with 0xD2511F53 and
// 0xCD9E8D57 and mixes their halves with the other words and the key; the
// key is bumped by 0x9E3779B9, 0xBB67AE85 between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox10(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                         uint32_t &c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Gaussian xi_ij for force evaluation k (Eq. 7).  Counter (min gid, max gid,
// k low word, (k >> 32 & 0xFFFF) | replica << 16), key = seed: the same for
// (i, j) and (j, i).  Box-Muller: u1 = ((x0 >> 9) + 1/2) 2^-23 in (0, 1),
// u2 = (x1 >> 9) 2^-23, xi = sqrt(-2 ln u1) cos(2 pi u2).
__device__ __forceinline__ float pair_gauss(uint32_t gi, uint32_t gj, uint32_t klo,
                                           uint32_t khi_rep, uint32_t key0, uint32_t key1) {
  uint32_t c0 = min(gi, gj), c1 = max(gi, gj), c2 = klo, c3 = khi_rep;
  philox10(c0, c1, c2, c3, key0, key1);
  const float u1 = (float)(c0 >> 9) * 0x1p-23f + 0x1p-24f;
  const float u2 = (float)(c1 >> 9) * 0x1p-23f;
  // -2 ln u1 = -2 ln2 log2 u1 (v_log_f32); cos(2 pi u2) is v_cos_f32(u2),
  // whose argument is in revolutions.
  const float m2ln = fmaxf(-2.0f * 0.693147180559945f * __builtin_amdgcn_logf(u1), 0.0f);
  return __builtin_amdgcn_sqrtf(m2ln) * __builtin_amdgcn_cosf(u2);
}

// ---------------------------------------------------------------------------
// Decisions (no contraction).
// ---------------------------------------------------------------------------

// Cell coordinate: floor(fl(x * invw)) clamped to [0, n - 1] (a NaN maps to
// cell 0 so that no index leaves its array).
__device__ __forceinline__ int cell_coord(float x, float invw, int n) {
#pragma clang fp contract(off)
  const float g = floorf(x * invw);
  return g >= 0.0f ? (g > (float)(n - 1) ? n - 1 : (int)g) : 0;
}

__device__ __forceinline__ int cell_index(const KGeom &G, float x, float y, float z, int &cx,
                                          int &cy, int &cz) {
  cx = cell_coord(x, G.invw[0], G.nc[0]);
  cy = cell_coord(y, G.invw[1], G.nc[1]);
  cz = cell_coord(z, G.invw[2], G.nc[2]);
  return (cz * G.nc[1] + cy) * G.nc[0] + cx;
}

// Single-edge periodic wrap in FP32.
__device__ __forceinline__ float wrap1(float x, float L) {
#pragma clang fp contract(off)
  return x >= L ? x - L : (x < 0.0f ? x + L : x);
}

// Drift of the Groot-Warren step in decision form: w = fl(v + fl(hdt f)),
// x* = fl(x + fl(dt w)), then the single-edge wrap.
__device__ __forceinline__ float drift1(float x, float v, float f, float hdt, float dt, float L) {
#pragma clang fp contract(off)
  const float w = v + hdt * f;
  const float y = x + dt * w;
  return wrap1(y, L);
}

// Pair decision: r2 = fma(dz, dz, fma(dy, dy, fl(dx^2))), in range iff
// r2 < fl32(rc^2), with d per axis the FP32 rounding of the exact
// minimum-image difference x_i - x_j - s L (SepAxis below).
__device__ __forceinline__ float pair_r2(float dx, float dy, float dz) {
#pragma clang fp contract(off)
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

__device__ __forceinline__ float sub_nc(float a, float b) {
#pragma clang fp contract(off)
  return a - b;
}

__device__ __forceinline__ float add_nc(float a, float b) {
#pragma clang fp contract(off)
  return a + b;
}

// Separation along one axis in decision form, for the candidates of a
// neighbour run seen at image shift sL (-L, 0 or +L): the coordinate that
// lies in the last cell (x_i for +L, x_j for -L) is lowered by L first,
// which is exact because it lies in [L/2, L), so d = fl(a - fl(x_j - b)) is
// the exact difference x_i - x_j - s L rounded once (fl(x_j - 0) = x_j).
struct SepAxis {
  float a, b;
};

__device__ __forceinline__ SepAxis sep_axis(float xi, float sL) {
  SepAxis r;
  r.a = sL > 0.f ? sub_nc(xi, sL) : xi;
  r.b = sL < 0.f ? -sL : 0.f;
  return r;
}

__device__ __forceinline__ float sep_d(const SepAxis &s, float xj) {
  return sub_nc(s.a, sub_nc(xj, s.b));
}

// Coarse positions for the candidate pre-test: q = rint(256 x) modulo 2^10
// per axis (256 x is exact in FP32, so |256 x - q| <= 1/2 before the
// modulo), one word per particle: x in bits 0-9, y in 11-20, z in 22-31,
// with bits 10 and 21 set.  Subtracting a lane's code (the same fields,
// those two bits clear) leaves each field's difference modulo 2^10 in its
// own bits (a borrow stops at the set bit above the field); read as signed
// 10-bit values (-512 .. 511) they are exact whenever the true code
// difference lies in that range, i.e. for points less than about 1.99
// apart per axis, whatever the box size.  With a periodic image shift s L rounded the
// same way, the code difference vector dq lies within 3/2 per axis of
// 256 d, d the exact image difference, so |dq| <= 256 |d| + 1.5 sqrt(3): a
// candidate with |dq| beyond 256 rc (1 + 1e-5) + 2.6 is out of range in the
// exact FP32 decision too (whose rounding of r^2 is a few 1e-7).  Farther
// candidates wrap to some other difference; they are at worst kept, and
// the exact decision drops them.
constexpr float kQScale = 256.f;
constexpr uint32_t kQGuard = (1u << 10) | (1u << 21);

__device__ __forceinline__ uint32_t qaxis(float x) {
  return (uint32_t)__float2int_rn(x * kQScale) & 0x3FFu;
}

__device__ __forceinline__ uint32_t qcode3(float x, float y, float z) {
  return qaxis(x) | (qaxis(y) << 11) | (qaxis(z) << 22) | kQGuard;
}

// |dq|^2 of a candidate's code w against the lane's shifted code q.
__device__ __forceinline__ uint32_t qdist2(uint32_t w, uint32_t q) {
  const int d = (int)(w - q);
  const int dx = __builtin_amdgcn_sbfe(d, 0, 10), dy = __builtin_amdgcn_sbfe(d, 11, 10),
            dz = __builtin_amdgcn_sbfe(d, 22, 10);
  return (uint32_t)(dx * dx + dy * dy + dz * dz);
}

// Threshold of the pre-test for cutoff^2 rc2: keep a candidate iff
// qdist2 <= qthresh.  Cutoffs of 1.97 and more (where a hit's code
// difference could leave the 10-bit range) keep every candidate.
__device__ __forceinline__ uint32_t qthresh(float rc2) {
  if (!(rc2 < 3.88f)) return 0xFFFFFFFFu;
  const float r = sqrtf(rc2) * (kQScale * 1.00001f) + 2.6f;
  return (uint32_t)(r * r);
}

// One axis of the lane's own code with the image shift sL of a neighbour row
// applied (10 bits, guard clear).
__device__ __forceinline__ uint32_t qshift(float x, float sL) {
  return ((uint32_t)__float2int_rn(x * kQScale) - (uint32_t)__float2int_rn(sL * kQScale)) &
         0x3FFu;
}

// ---------------------------------------------------------------------------
// Streaming accesses: per-particle records that a step reads or writes once
// (the integrator's own state, the pair kernel's outputs and its own old
// velocity and force).  The nontemporal hint lets their lines leave the L2
// first, so that the neighbour records the pair walk gathers again and again
// stay there.  Values and ordering are those of plain accesses.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 load_stream(const float4 *p) {
  const f32x4 v = __builtin_nontemporal_load((const f32x4 *)p);
  return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void store_stream(float4 *p, const float4 v) {
  __builtin_nontemporal_store(f32x4{v.x, v.y, v.z, v.w}, (f32x4 *)p);
}

__device__ __forceinline__ void store_stream(int32_t *p, int32_t v) {
  __builtin_nontemporal_store(v, p);
}

// ---------------------------------------------------------------------------
// Phase field: trilinear interpolation of the periodic node grid (decision
// form lerp(a, b, t) = fl(a + fl(t fl(b - a))): four lerps in x, two in y,
// one in z), and the gradient of the same interpolant.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T lerp_nc(T a, T b, T t) {
#pragma clang fp contract(off)
  return a + t * (b - a);
}

__device__ __forceinline__ int wrapi(int i, int n) {
  i = i % n;
  return i < 0 ? i + n : i;
}

template <typename T> struct GridScale;
template <> struct GridScale<float> {
  static __device__ __forceinline__ float inv_h(const KGeom &G, int k) { return G.inv_h[k]; }
  static __device__ __forceinline__ float coord(float x) { return x; }
};
template <> struct GridScale<double> {
  static __device__ __forceinline__ double inv_h(const KGeom &G, int k) { return G.inv_h64[k]; }
  static __device__ __forceinline__ double coord(float x) { return (double)x; }
};

// Grid cube holding a point: lower node indices (periodic) and the local
// coordinates t in [0, 1] along each axis (decision form).
template <typename T>
struct GridLoc {
  int i0[3], i1[3];
  T t[3];
};

template <typename T>
__device__ __forceinline__ GridLoc<T> grid_locate(const KGeom &G, float x, float y, float z) {
#pragma clang fp contract(off)
  const float p[3] = {x, y, z};
  GridLoc<T> L;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T g = GridScale<T>::coord(p[k]) * GridScale<T>::inv_h(G, k);
    const T fg = floor(g);
    L.t[k] = g - fg;
    L.i0[k] = wrapi((int)fg, G.ng[k]);
    L.i1[k] = L.i0[k] + 1 == G.ng[k] ? 0 : L.i0[k] + 1;
  }
  return L;
}

// Linear index of the grid cube whose lower corner is node i0.
template <typename T>
__device__ __forceinline__ size_t cube_index(const KGeom &G, const GridLoc<T> &L) {
  return ((size_t)L.i0[2] * (size_t)G.ng[1] + (size_t)L.i0[1]) * (size_t)G.ng[0] + (size_t)L.i0[0];
}

template <typename T>
__device__ __forceinline__ T phi_interp(const T *__restrict__ grid, const KGeom &G,
                                        const GridLoc<T> &L) {
#pragma clang fp contract(off)
  const size_t nx = (size_t)G.ng[0], nxy = nx * (size_t)G.ng[1];
  const T *r00 = grid + (size_t)L.i0[2] * nxy + (size_t)L.i0[1] * nx;
  const T *r01 = grid + (size_t)L.i0[2] * nxy + (size_t)L.i1[1] * nx;
  const T *r10 = grid + (size_t)L.i1[2] * nxy + (size_t)L.i0[1] * nx;
  const T *r11 = grid + (size_t)L.i1[2] * nxy + (size_t)L.i1[1] * nx;
  const T e00 = lerp_nc(r00[L.i0[0]], r00[L.i1[0]], L.t[0]);
  const T e01 = lerp_nc(r01[L.i0[0]], r01[L.i1[0]], L.t[0]);
  const T e10 = lerp_nc(r10[L.i0[0]], r10[L.i1[0]], L.t[0]);
  const T e11 = lerp_nc(r11[L.i0[0]], r11[L.i1[0]], L.t[0]);
  const T y0 = lerp_nc(e00, e01, L.t[1]);
  const T y1 = lerp_nc(e10, e11, L.t[1]);
  return lerp_nc(y0, y1, L.t[2]);
}

// Gradient of the trilinear interpolant at L (the derivative of the
// 8-corner weights), in the grid's precision.
template <typename T>
__device__ __forceinline__ void phi_grad(const T *__restrict__ grid, const KGeom &G,
                                         const GridLoc<T> &L, T &gx, T &gy, T &gz) {
  const size_t nx = (size_t)G.ng[0], nxy = nx * (size_t)G.ng[1];
  const T *r00 = grid + (size_t)L.i0[2] * nxy + (size_t)L.i0[1] * nx;
  const T *r01 = grid + (size_t)L.i0[2] * nxy + (size_t)L.i1[1] * nx;
  const T *r10 = grid + (size_t)L.i1[2] * nxy + (size_t)L.i0[1] * nx;
  const T *r11 = grid + (size_t)L.i1[2] * nxy + (size_t)L.i1[1] * nx;
  // corners c[z][y][x]
  const T c000 = r00[L.i0[0]], c001 = r00[L.i1[0]], c010 = r01[L.i0[0]], c011 = r01[L.i1[0]];
  const T c100 = r10[L.i0[0]], c101 = r10[L.i1[0]], c110 = r11[L.i0[0]], c111 = r11[L.i1[0]];
  const T tx = L.t[0], ty = L.t[1], tz = L.t[2];
  const T ux = (T)1 - tx, uy = (T)1 - ty, uz = (T)1 - tz;
  gx = (uz * (uy * (c001 - c000) + ty * (c011 - c010)) +
        tz * (uy * (c101 - c100) + ty * (c111 - c110))) * GridScale<T>::inv_h(G, 0);
  gy = (uz * (ux * (c010 - c000) + tx * (c011 - c001)) +
        tz * (ux * (c110 - c100) + tx * (c111 - c101))) * GridScale<T>::inv_h(G, 1);
  gz = (uy * (ux * (c100 - c000) + tx * (c101 - c001)) +
        ty * (ux * (c110 - c010) + tx * (c111 - c011))) * GridScale<T>::inv_h(G, 2);
}

template <typename T>
__device__ __forceinline__ T phi_at(const T *__restrict__ grid, const KGeom &G, float x, float y,
                                    float z) {
  return phi_interp(grid, G, grid_locate<T>(G, x, y, z));
}

// The phase field laid out for the lookups of the step: node (i, j, k) holds
// the four values of its x-y face, (phi(i, j, k), phi(i+1, j, k),
// phi(i, j+1, k), phi(i+1, j+1, k)) with periodic neighbours, so that the 8
// corners of a grid cube are two 16-byte (FP32) or 32-byte (FP64) loads.
template <typename T> struct PhiQuad;
template <> struct PhiQuad<float> {
  using type = float4;
};
template <> struct PhiQuad<double> {
  using type = double4;
};

template <typename T>
__device__ __forceinline__ void quad_corners(const typename PhiQuad<T>::type *__restrict__ quad,
                                             const KGeom &G, const GridLoc<T> &L,
                                             typename PhiQuad<T>::type &q0,
                                             typename PhiQuad<T>::type &q1) {
  const size_t nx = (size_t)G.ng[0], nxy = nx * (size_t)G.ng[1];
  const size_t yx = (size_t)L.i0[1] * nx + (size_t)L.i0[0];
  q0 = quad[(size_t)L.i0[2] * nxy + yx];
  q1 = quad[(size_t)L.i1[2] * nxy + yx];
}

// phi_interp from the face layout: the same lerps in the same order.
template <typename T>
__device__ __forceinline__ T phi_interp_quad(const typename PhiQuad<T>::type *__restrict__ quad,
                                             const KGeom &G, const GridLoc<T> &L) {
#pragma clang fp contract(off)
  typename PhiQuad<T>::type q0, q1;
  quad_corners<T>(quad, G, L, q0, q1);
  const T e00 = lerp_nc(q0.x, q0.y, L.t[0]);
  const T e01 = lerp_nc(q0.z, q0.w, L.t[0]);
  const T e10 = lerp_nc(q1.x, q1.y, L.t[0]);
  const T e11 = lerp_nc(q1.z, q1.w, L.t[0]);
  const T y0 = lerp_nc(e00, e01, L.t[1]);
  const T y1 = lerp_nc(e10, e11, L.t[1]);
  return lerp_nc(y0, y1, L.t[2]);
}

template <typename T>
__device__ __forceinline__ T phi_at_quad(const typename PhiQuad<T>::type *__restrict__ quad,
                                         const KGeom &G, float x, float y, float z) {
  return phi_interp_quad<T>(quad, G, grid_locate<T>(G, x, y, z));
}

// phi_grad from the face layout (corners c[z][y][x] as in phi_grad).
template <typename T>
__device__ __forceinline__ void phi_grad_quad(const typename PhiQuad<T>::type *__restrict__ quad,
                                              const KGeom &G, const GridLoc<T> &L, T &gx, T &gy,
                                              T &gz) {
  typename PhiQuad<T>::type q0, q1;
  quad_corners<T>(quad, G, L, q0, q1);
  const T c000 = q0.x, c001 = q0.y, c010 = q0.z, c011 = q0.w;
  const T c100 = q1.x, c101 = q1.y, c110 = q1.z, c111 = q1.w;
  const T tx = L.t[0], ty = L.t[1], tz = L.t[2];
  const T ux = (T)1 - tx, uy = (T)1 - ty, uz = (T)1 - tz;
  gx = (uz * (uy * (c001 - c000) + ty * (c011 - c010)) +
        tz * (uy * (c101 - c100) + ty * (c111 - c110))) * GridScale<T>::inv_h(G, 0);
  gy = (uz * (ux * (c010 - c000) + tx * (c011 - c001)) +
        tz * (ux * (c110 - c100) + tx * (c111 - c101))) * GridScale<T>::inv_h(G, 1);
  gz = (uy * (ux * (c100 - c000) + tx * (c101 - c001)) +
        ty * (ux * (c110 - c010) + tx * (c111 - c011))) * GridScale<T>::inv_h(G, 2);
}

// Minimum-image separation x_i - x_j of two coordinates in [0, L) of a
// pair within the cutoff.  Across the periodic edge the coordinate near L is
// shifted by L first, which is exact (it lies within a factor two of L), so
// the separation carries one rounding of a number below rc rather than the
// rounding of x_i - x_j ~ L (half an ulp of L: 7.6e-6 at L = 168).
__device__ __forceinline__ float sep(float xi, float xj, float L) {
  const float d = xi - xj, h = 0.5f * L;
  const float a = d > h ? xi - L : xi;
  const float b = d < -h ? xj - L : xj;
  return a - b;
}

// Minimum-image component (|d| < L/2 for every pair within the cutoff).
__device__ __forceinline__ float min_image(float d, float L) {
  return d > 0.5f * L ? d - L : (d < -0.5f * L ? d + L : d);
}

// Neighbour cell `code` (0..26) of (cx, cy, cz): wrapped index and the image
// shift s L of its particles as seen from the home cell.
struct NCell {
  int c;
  float sx, sy, sz;
};

__device__ __forceinline__ NCell neighbour_cell(const KGeom &G, int cx, int cy, int cz, int code) {
  const int ox = code % 3 - 1, oy = (code / 3) % 3 - 1, oz = code / 9 - 1;
  int qx = cx + ox, qy = cy + oy, qz = cz + oz;
  NCell n;
  n.sx = 0.f;
  n.sy = 0.f;
  n.sz = 0.f;
  if (qx < 0) { qx += G.nc[0]; n.sx = -G.L[0]; }
  else if (qx >= G.nc[0]) { qx -= G.nc[0]; n.sx = G.L[0]; }
  if (qy < 0) { qy += G.nc[1]; n.sy = -G.L[1]; }
  else if (qy >= G.nc[1]) { qy -= G.nc[1]; n.sy = G.L[1]; }
  if (qz < 0) { qz += G.nc[2]; n.sz = -G.L[2]; }
  else if (qz >= G.nc[2]) { qz -= G.nc[2]; n.sz = G.L[2]; }
  n.c = (qz * G.nc[1] + qy) * G.nc[0] + qx;
  return n;
}

// The 27-cell neighbourhood of a home cell (cx, cy, cz) as contiguous ranges
// of the merged per-cell runs.  Cells x-1, x, x+1 of one (y, z) row are
// consecutive cell indices, so each of the 9 rows is one range, or two where
// the row wraps around x.  The ranges come in the order of the 27 cells (x
// fastest, then y, then z), so candidates are visited in the same order as
// cell by cell, with the image shift s L of each cell.
struct NeighbourRows {
  int cx, cy, cz, oy, oz, pend, base;
  float sy, sz;

  __device__ __forceinline__ void init(int x, int y, int z) {
    cx = x;
    cy = y;
    cz = z;
    oy = -1;
    oz = -1;
    pend = 0;
    base = 0;
    sy = 0.f;
    sz = 0.f;
  }

  // Next range [t, t_end) and its shifts; false when the neighbourhood is done.
  __device__ __forceinline__ bool next(const KGeom &G, const int32_t *__restrict__ start_all,
                                       int co, int &t, int &t_end, float &sx, float &sy_out,
                                       float &sz_out) {
    const int nx = G.nc[0];
    if (pend) {
      // second part of a row that wraps: cells 0, 1 (left edge) or cell 0
      // seen across the right edge
      t = start_all[co + base];
      t_end = start_all[co + base + (pend == 1 ? 2 : 1)];
      sx = pend == 1 ? 0.f : G.L[0];
      pend = 0;
    } else {
      if (oz == 2) return false;
      int qy = cy + oy, qz = cz + oz;
      sy = 0.f;
      sz = 0.f;
      if (qy < 0) { qy += G.nc[1]; sy = -G.L[1]; }
      else if (qy >= G.nc[1]) { qy -= G.nc[1]; sy = G.L[1]; }
      if (qz < 0) { qz += G.nc[2]; sz = -G.L[2]; }
      else if (qz >= G.nc[2]) { qz -= G.nc[2]; sz = G.L[2]; }
      base = (qz * G.nc[1] + qy) * nx;
      if (cx > 0 && cx < nx - 1) {
        t = start_all[co + base + cx - 1];
        t_end = start_all[co + base + cx + 2];
        sx = 0.f;
      } else if (cx == 0) {
        t = start_all[co + base + nx - 1];
        t_end = start_all[co + base + nx];
        sx = -G.L[0];
        pend = 1;
      } else {
        t = start_all[co + base + nx - 2];
        t_end = start_all[co + base + nx];
        sx = 0.f;
        pend = 2;
      }
      if (++oy == 2) {
        oy = -1;
        ++oz;
      }
    }
    sy_out = sy;
    sz_out = sz;
    return true;
  }
};

// Buffer-resource loads.  A buffer resource carries the base address, the
// record stride and the extent; an indexed load takes the record index and
// the memory unit forms the address, so a gather costs no per-lane 64-bit
// address arithmetic.  Word 3 is the gfx9 default (32-bit data format).  The
// extent is the array's true length; every index the kernels form lies
// inside it (the arrays carry spare entries where a pass reads ahead).
typedef int v4i32_t __attribute__((ext_vector_type(4)));
extern "C" __device__ v4i32_t dpd_struct_buffer_load_v4i32(__amdgpu_buffer_rsrc_t rsrc, int vindex,
                                                           int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.v4i32");
constexpr int kBufferWord3 = 0x00020000;

// An array of 16-byte records (float4) read by index.
struct Records16 {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Records16(const float4 *p, int n)
      : r(__builtin_amdgcn_make_buffer_rsrc((void *)p, (short)16, n, kBufferWord3)) {}
  __device__ __forceinline__ float4 operator[](int i) const {
    const v4i32_t v = dpd_struct_buffer_load_v4i32(r, i, 0, 0, 0);
    return make_float4(__int_as_float(v.x), __int_as_float(v.y), __int_as_float(v.z),
                       __int_as_float(v.w));
  }
};

// An int32 array read four entries at a time from any entry.
struct Ints4 {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Ints4(const int32_t *p, int n)
      : r(__builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, 4 * n, kBufferWord3)) {}
  __device__ __forceinline__ void load(int i, int out[4]) const {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, 4 * i, 0, 0);
    out[0] = (int)v[0];
    out[1] = (int)v[1];
    out[2] = (int)v[2];
    out[3] = (int)v[3];
  }
};

// True when the predicate holds on any active lane of the wavefront.
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Map a hardware block index to a logical one so that each of the 8 XCDs
// (which receive blocks round-robin) works on one contiguous eighth of the
// index space and its L2 sees one spatial region.  gridDim.x must be a
// multiple of 8; logical indices past the work are idle.
__device__ __forceinline__ int xcd_block() {
  const int per = (int)(gridDim.x >> 3);
  return (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
}

}  // namespace dpd
