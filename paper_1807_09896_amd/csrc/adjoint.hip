// Adjoint of the DPD step: vector-Jacobian products of the pair force
// (Eq. 3-10), the Groot-Warren update and the phase-field bounce-back
// (Eq. 16-17) with the bounce-back events held at their recorded values,
// plus the window observable (mean v_x per bin) and its adjoint seed.
//
// Notation of one step t (fluid particle i, h = dt/2):
//   w = v + h f,  r* = r + dt w,  vt = v + lambda dt f
//   event 0: r' = r*                      v' = w + h f'
//   event 1: r' = r* - 2 s dt v, s(phi(r*), phi(r))   vt = -v, v' = -v
//   event 2: r' = r                                   vt = -v, v' = -v
//   f'_i = sum_j F_ij(r'_i - r'_j, vt_i - vt_j) + g
// The backward sweep of step t takes the adjoints of (r', v', f') in the
// slot order of step t + 1 and returns the adjoints of (r, v, f) in the
// order of step t, which is the slot order of step t - 1.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace dpd {
namespace {

constexpr int kBlockA = 256;
constexpr int kListCapA = 24;
constexpr int kBatchA = 4;

inline unsigned grid_a(int64_t n) { return (unsigned)((n + kBlockA - 1) / kBlockA); }

// Profile bin in decision form: clamp(floor(fl(x * scale)), 0, nbins - 1).
__device__ __forceinline__ int bin_of(float x, float scale, int nbins) {
#pragma clang fp contract(off)
  const float g = floorf(x * scale);
  return g >= 0.0f ? (g > (float)(nbins - 1) ? nbins - 1 : (int)g) : 0;
}

// Coordinate `axis` of a position held in registers.  The argument is a
// value on purpose: selecting through a reference to global memory lets the
// compiler turn the choice into a choice of load address, which the gfx950
// backend lowers incorrectly for the z case (a load through an address
// register that the z path never writes).
__device__ __forceinline__ float axis_of(const float4 x, int axis) {
  return axis == 0 ? x.x : (axis == 1 ? x.y : x.z);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block sum of three values added to slot[0..2] by thread 0 (a fixed
// summation order: the partial of a block is the same in every run).  Every
// thread of the block must call it.
template <int BS>
__device__ __forceinline__ void block_add3(double a, double b, double c, double *slot) {
  __shared__ double red[3][BS / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = (int)__lane_id(), wv = (int)threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = a;
    red[1][wv] = b;
    red[2][wv] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int q = 0; q < BS / 64; ++q) {
      s0 += red[0][q];
      s1 += red[1][q];
      s2 += red[2][q];
    }
    slot[0] += s0;
    slot[1] += s1;
    slot[2] += s2;
  }
}

// ---------------------------------------------------------------------------
// Window observable
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlockA) void k_obs(int64_t nf, const float4 *__restrict__ pos4,
                                                 const float4 *__restrict__ vel4, int axis,
                                                 int nbins, float scale, double *sums,
                                                 unsigned long long *counts) {
  __shared__ double s_sum[kMaxBins];
  __shared__ unsigned s_cnt[kMaxBins];
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    s_sum[b] = 0.0;
    s_cnt[b] = 0u;
  }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nf; p += stride) {
    const float4 x = pos4[p];
    const int b = bin_of(axis_of(x, axis), scale, nbins);
    atomicAdd(&s_sum[b], (double)vel4[p].x);
    atomicAdd(&s_cnt[b], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    if (s_cnt[b]) {
      atomicAdd(&sums[b], s_sum[b]);
      atomicAdd(&counts[b], (unsigned long long)s_cnt[b]);
    }
  }
}

__global__ void k_obs_final(int nbins, const double *__restrict__ sums,
                            const unsigned long long *__restrict__ counts, double *profile,
                            int64_t *counts_out) {
  const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= nbins) return;
  const unsigned long long c = counts[b];
  if (profile) profile[b] = c ? sums[b] / (double)c : 0.0;
  if (counts_out) counts_out[b] = (int64_t)c;
}

// Adjoint seed: d(mean v_x in bin b)/d(v_x of a term in b) = 1 / N_b.
__global__ void k_loss_weights(int nbins, const double *__restrict__ dldp,
                               const unsigned long long *__restrict__ counts, float *lw) {
  const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= nbins) return;
  const unsigned long long c = counts[b];
  lw[b] = c ? (float)(dldp[b] / (double)c) : 0.0f;
}

__global__ void k_vt_from_v(int64_t nf, const float4 *__restrict__ vel4, float4 *vt4) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nf) return;
  const float4 v = vel4[p];
  vt4[p] = make_float4(v.x, v.y, v.z, __int_as_float(0));
}

__global__ void k_set_u64(unsigned long long *p, unsigned long long v) { *p = v; }

// ---------------------------------------------------------------------------
// Step seed: the adjoint of f' (with the loss term of v' added) moved from
// the slot order of step t + 1 to the order of step t.
//   Fbar_i = fbar'_i + h vbar'_i   (event 0: v' = w + h f')
//   Fbar_i = fbar'_i               (events 1, 2: v' = -v)
// initial = 1: the refreshed starting force f0 = F(r0, v0) + g, whose
// adjoint is already in index order (no permutation, no loss term).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlockA) void k_adj_prep(
    const Box *__restrict__ boxes, int64_t nf, int initial, const int32_t *__restrict__ idx,
    const float4 *__restrict__ pos4, const float4 *__restrict__ vt4,
    const float4 *__restrict__ rb_s, const float4 *__restrict__ vb_s,
    const float4 *__restrict__ fb_s, const float *__restrict__ lw, int axis, int nbins,
    float scale, float4 *__restrict__ rn, float4 *__restrict__ vn, float4 *__restrict__ fbar,
    double *part_g) {
  const KParams P = boxes[0].P;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  if (s < nf) {
    float4 F = fb_s[s];
    if (initial) {
      fbar[s] = F;
    } else {
      const int i = idx[s];
      const int ev = __float_as_int(vt4[i].w);
      float4 vb = vb_s[s];
      const float4 xi = pos4[i];
      vb.x += lw[bin_of(axis_of(xi, axis), scale, nbins)];
      if (ev == 0) {
        F.x += P.hdt * vb.x;
        F.y += P.hdt * vb.y;
        F.z += P.hdt * vb.z;
      }
      fbar[i] = F;
      rn[i] = rb_s[s];
      vn[i] = vb;
    }
    gx = F.x;
    gy = F.y;
    gz = F.z;
  }
  block_add3<kBlockA>(gx, gy, gz, part_g + 3 * (size_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Pair-force VJP.  With d = r_i - r_j, r = |d|, e = d / r, w = 1 - r/rc,
// u = e . (vt_i - vt_j), s = sigma xi / sqrt(dt) and
// F_ij = c e, c = w (a - gamma w u + s), the adjoint mu_ij = Fbar_i - Fbar_j
// (Fbar_j = 0 for a wall: its force is never used) gives
//   rbar_i  += (dc/dd) (e . mu) + c (mu - e (e . mu)) / r
//              dc/dd = -(a - 2 gamma w u + s) e / rc - gamma w^2 (dv - u e) / r
//   vtbar_i += -gamma w^2 e (e . mu)
// gathered per particle over its full neighbour shell (F_ji = -F_ij, and the
// Jacobian is even in d, so both terms of a pair land on i this way), and
// the parameter terms of f_i, with eF = e . Fbar_i:
//   abar    += w eF            (a_ff for a fluid j, a_fw for a wall)
//   gammabar += (-w^2 u + w xi dsigma/dgamma / sqrt(dt)) eF
// Pairs are found with the force kernel's decision at the same positions,
// so the set is the forward's.
// ---------------------------------------------------------------------------
template <int BS>
__global__ __launch_bounds__(BS) void k_force_vjp(
    const Box *__restrict__ boxes, const Tile *__restrict__ tiles, int ntiles, int64_t NF,
    int32_t pad, const float4 *__restrict__ pos4, const float4 *__restrict__ vt4,
    const int32_t *__restrict__ idx, const int32_t *__restrict__ idx_all,
    const int32_t *__restrict__ start_all, const float4 *__restrict__ fbar,
    const float4 *__restrict__ rn, float4 *__restrict__ rt_out, float4 *__restrict__ vt_out,
    const unsigned long long *__restrict__ dk0, unsigned long long koff, double *part) {
  __shared__ uint32_t list[kListCapA * BS];
  const int tid = xcd_block();
  bool act = tid < ntiles;
  Tile tile{0, 0, 0, 0};
  if (act) {
    tile = tiles[tid];
    act = (int)threadIdx.x < tile.count;
  }
  double p_aff = 0.0, p_afw = 0.0, p_gam = 0.0;
  if (act) {
    const Box &B = boxes[tile.box];
    const KGeom G = B.G;
    const KParams P = B.P;
    const int co = (int)B.co;
    const unsigned long long kk = *dk0 + koff;
    const uint32_t klo = (uint32_t)kk;
    const uint32_t khi = ((uint32_t)(kk >> 32) & 0xFFFFu) | (P.replica << 16);
    const int64_t s = (int64_t)tile.first + threadIdx.x;
    const int i = idx[s];
    const float4 pi = pos4[i];
    const float4 vti = vt4[i];
    const float4 Fi = fbar[i];
    const uint32_t gi = __float_as_uint(pi.w);
    int cx, cy, cz;
    cell_index(G, pi.x, pi.y, pi.z, cx, cy, cz);
    uint32_t *mine = list + threadIdx.x;
    float rbx = 0.f, rby = 0.f, rbz = 0.f, vbx = 0.f, vby = 0.f, vbz = 0.f;
    NeighbourRows rows;
    rows.init(cx, cy, cz);
    int t = 0, t_end = 0;
    SepAxis ax = sep_axis(pi.x, 0.f), ay = sep_axis(pi.y, 0.f), az = sep_axis(pi.z, 0.f);
    bool done = false;
    while (!done) {
      int cnt = 0;
      while (cnt <= kListCapA - kBatchA) {
        if (t >= t_end) {
          float sx, sy, sz;
          if (!rows.next(G, start_all, co, t, t_end, sx, sy, sz)) {
            done = true;
            break;
          }
          ax = sep_axis(pi.x, sx);
          ay = sep_axis(pi.y, sy);
          az = sep_axis(pi.z, sz);
          continue;
        }
        int jb[kBatchA];
#pragma unroll
        for (int u = 0; u < kBatchA; ++u) jb[u] = t + u < t_end ? idx_all[t + u] : pad;
        float4 pb[kBatchA];
#pragma unroll
        for (int u = 0; u < kBatchA; ++u) pb[u] = pos4[jb[u]];
#pragma unroll
        for (int u = 0; u < kBatchA; ++u) {
          const float r2 = pair_r2(sep_d(ax, pb[u].x), sep_d(ay, pb[u].y), sep_d(az, pb[u].z));
          if (r2 < P.rc2 && r2 > 0.0f) {
            mine[cnt * BS] = (uint32_t)jb[u];
            ++cnt;
          }
        }
        t += kBatchA;
      }
      for (int q = 0; q < cnt; ++q) {
        const uint32_t j = mine[q * BS];
        const float4 pj = pos4[j];
        const float4 vtj = vt4[j];
        const bool fluid_j = (int64_t)j < NF;
        const float4 Fj = fluid_j ? fbar[j] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float dx = sep(pi.x, pj.x, G.L[0]);
        const float dy = sep(pi.y, pj.y, G.L[1]);
        const float dz = sep(pi.z, pj.z, G.L[2]);
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float rinv = rsqrtf(r2);
        const float r = r2 * rinv;
        const float w = 1.0f - r * P.inv_rc;
        if (!(w > 0.0f)) continue;   // the forward's force is zero there
        const float ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
        const float dvx = vti.x - vtj.x, dvy = vti.y - vtj.y, dvz = vti.z - vtj.z;
        const float u = ex * dvx + ey * dvy + ez * dvz;
        const float xi = pair_gauss(gi, __float_as_uint(pj.w), klo, khi, P.key0, P.key1);
        const float sr = P.sigma_rdt * xi;
        const float a = fluid_j ? P.a_ff : P.a_fw;
        const float c = w * (a - P.gamma * w * u + sr);
        const float mx = Fi.x - Fj.x, my = Fi.y - Fj.y, mz = Fi.z - Fj.z;
        const float em = ex * mx + ey * my + ez * mz;
        const float gw = -(a - 2.0f * P.gamma * w * u + sr) * P.inv_rc * em;
        const float gwu = -P.gamma * w * w;
        const float gu = gwu * rinv * em;
        const float cr = c * rinv;
        rbx += gw * ex + gu * (dvx - u * ex) + cr * (mx - ex * em);
        rby += gw * ey + gu * (dvy - u * ey) + cr * (my - ey * em);
        rbz += gw * ez + gu * (dvz - u * ez) + cr * (mz - ez * em);
        vbx += gwu * em * ex;
        vby += gwu * em * ey;
        vbz += gwu * em * ez;
        const float eF = ex * Fi.x + ey * Fi.y + ez * Fi.z;
        if (fluid_j)
          p_aff += (double)(w * eF);
        else
          p_afw += (double)(w * eF);
        p_gam += (double)((-w * w * u + P.dsig_rdt * w * xi) * eF);
      }
    }
    if (rn) {
      const float4 b = rn[i];
      rbx += b.x;
      rby += b.y;
      rbz += b.z;
    }
    rt_out[i] = make_float4(rbx, rby, rbz, 0.f);
    vt_out[i] = make_float4(vbx, vby, vbz, 0.f);
  }
  block_add3<BS>(p_aff, p_afw, p_gam, part + 3 * (size_t)tid);
}

// Gradient of the trilinear interpolant at a located point (per unit
// length), and bar * (corner weight) added to each of the 8 corner nodes.
template <typename T>
__device__ __forceinline__ void phi_grad_scatter(const T *__restrict__ grid, const KGeom &G,
                                                 const GridLoc<T> &L, T bar, double *dphi,
                                                 T g[3]) {
  const size_t nx = (size_t)G.ng[0], nxy = nx * (size_t)G.ng[1];
  T gx = 0, gy = 0, gz = 0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const T wz = c ? L.t[2] : (T)1 - L.t[2], dwz = c ? (T)1 : (T)-1;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const T wy = b ? L.t[1] : (T)1 - L.t[1], dwy = b ? (T)1 : (T)-1;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T wx = a ? L.t[0] : (T)1 - L.t[0], dwx = a ? (T)1 : (T)-1;
        const size_t node = (size_t)(c ? L.i1[2] : L.i0[2]) * nxy +
                            (size_t)(b ? L.i1[1] : L.i0[1]) * nx + (size_t)(a ? L.i1[0] : L.i0[0]);
        const T p = grid[node];
        gx += p * dwx * wy * wz;
        gy += p * wx * dwy * wz;
        gz += p * wx * wy * dwz;
        if (dphi && bar != (T)0) atomicAdd(&dphi[node], (double)(bar * wx * wy * wz));
      }
    }
  }
  g[0] = gx * GridScale<T>::inv_h(G, 0);
  g[1] = gy * GridScale<T>::inv_h(G, 1);
  g[2] = gz * GridScale<T>::inv_h(G, 2);
}

// ---------------------------------------------------------------------------
// Integrate + bounce-back VJP with the step's events held fixed: from the
// adjoints of r' (rt, pair part included), of vt (vtb) and of v' (vn, loss
// term included) to those of (r, v, f) of step t.  Event 1 differentiates
// Eq. 17's s = c1 / (c0 + c1), c1 = atanh(-phi(r*)), c0 = atanh(phi(r)),
// through the interpolated phi at both points (gradient and node values).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlockA) void k_integrate_vjp(
    const Box *__restrict__ boxes, int64_t nf, const float4 *__restrict__ pos_t,
    const float4 *__restrict__ vel_t, const float4 *__restrict__ frc_t,
    const float4 *__restrict__ vt4, const float4 *__restrict__ rt,
    const float4 *__restrict__ vtb, const float4 *__restrict__ vn, const T *__restrict__ grid_base,
    double *dphi_base, float4 *__restrict__ rb_out, float4 *__restrict__ vb_out,
    float4 *__restrict__ fb_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const Box &B = boxes[0];
  const KGeom G = B.G;
  const KParams P = B.P;
  const int ev = __float_as_int(vt4[i].w);
  const float4 R = rt[i], V = vtb[i], W = vn[i];
  float rb[3], vb[3], fb[3];
  if (ev == 0) {
    const float wb[3] = {P.dt * R.x + W.x, P.dt * R.y + W.y, P.dt * R.z + W.z};
    const float vv[3] = {V.x, V.y, V.z};
    const float rr[3] = {R.x, R.y, R.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      rb[a] = rr[a];
      vb[a] = wb[a] + vv[a];
      fb[a] = P.hdt * wb[a] + P.lamdt * vv[a];
    }
  } else if (ev == 2) {
    rb[0] = R.x;
    rb[1] = R.y;
    rb[2] = R.z;
    vb[0] = -V.x - W.x;
    vb[1] = -V.y - W.y;
    vb[2] = -V.z - W.z;
    fb[0] = fb[1] = fb[2] = 0.f;
  } else {
    const T *grid = grid_base + B.go;
    double *dphi = dphi_base ? dphi_base + B.go : nullptr;
    const float4 x = pos_t[i], v = vel_t[i], f = frc_t[i];
    const float xs = drift1(x.x, v.x, f.x, P.hdt, P.dt, G.L[0]);
    const float ys = drift1(x.y, v.y, f.y, P.hdt, P.dt, G.L[1]);
    const float zs = drift1(x.z, v.z, f.z, P.hdt, P.dt, G.L[2]);
    const GridLoc<T> ls = grid_locate<T>(G, xs, ys, zs);
    const GridLoc<T> lt = grid_locate<T>(G, x.x, x.y, x.z);
    const T phis = phi_interp(grid, G, ls);
    const T phit = phi_interp(grid, G, lt);
    const T lim = (T)1 - (T)0x1p-20;
    const T a1 = fmin(fmax(-phis, (T)0), lim);
    const T a0 = fmin(fmax(phit, (T)0), lim);
    const T c1 = atanh(a1), c0 = atanh(a0);
    const T sfrac = c1 > (T)0 ? c1 / (c0 + c1) : (T)0;
    const float rr[3] = {R.x, R.y, R.z};
    const float vv[3] = {v.x, v.y, v.z};
    // r' = r* - 2 s dt v
    const T sbar = (T)(-2.0f * P.dt) * (T)(vv[0] * rr[0] + vv[1] * rr[1] + vv[2] * rr[2]);
    const float k2 = (float)((T)2 * sfrac * (T)P.dt);
    float rsb[3] = {rr[0], rr[1], rr[2]};
    float rtb[3] = {0.f, 0.f, 0.f};
    if (c1 > (T)0) {
      const T den = c0 + c1;
      const T ds1 = c0 / (den * den), ds0 = -c1 / (den * den);
      const T dp1 = (-phis > (T)0 && -phis < lim) ? (T)-1 / ((T)1 - a1 * a1) : (T)0;
      const T dp0 = (phit > (T)0 && phit < lim) ? (T)1 / ((T)1 - a0 * a0) : (T)0;
      const T pbs = sbar * ds1 * dp1, pbt = sbar * ds0 * dp0;
      T gs[3], gt[3];
      phi_grad_scatter<T>(grid, G, ls, pbs, dphi, gs);
      phi_grad_scatter<T>(grid, G, lt, pbt, dphi, gt);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        rsb[a] += (float)(pbs * gs[a]);
        rtb[a] = (float)(pbt * gt[a]);
      }
    }
    const float vtv[3] = {V.x, V.y, V.z}, vnv[3] = {W.x, W.y, W.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // r* = r + dt w, w = v + h f; vt = -v; v' = -v
      const float wb = P.dt * rsb[a];
      rb[a] = rsb[a] + rtb[a];
      vb[a] = -k2 * rr[a] + wb - vtv[a] - vnv[a];
      fb[a] = P.hdt * wb;
    }
  }
  rb_out[i] = make_float4(rb[0], rb[1], rb[2], 0.f);
  vb_out[i] = make_float4(vb[0], vb[1], vb[2], 0.f);
  fb_out[i] = make_float4(fb[0], fb[1], fb[2], 0.f);
}

// Fixed-order final sums of the per-block partials:
// out = {a_ff, a_fw, gamma} from the pair VJP and {g_x, g_y, g_z}.
__global__ void k_reduce_partials(int nb_f, const double *__restrict__ part_f, int nb_g,
                                  const double *__restrict__ part_g, double *out) {
  const int k = (int)threadIdx.x;
  if (k >= 6) return;
  double s = 0.0;
  if (k < 3) {
    for (int b = 0; b < nb_f; ++b) s += part_f[3 * b + k];
  } else {
    for (int b = 0; b < nb_g; ++b) s += part_g[3 * b + k - 3];
  }
  out[k] = s;
}

}  // namespace

hipError_t launch_obs(hipStream_t s, int64_t nf, const float4 *pos4, const float4 *vel4,
                      int axis, int nbins, float scale, double *sums,
                      unsigned long long *counts) {
  if (nf <= 0) return hipSuccess;
  unsigned nb = grid_a(nf);
  if (nb > 512) nb = 512;
  k_obs<<<nb, kBlockA, 0, s>>>(nf, pos4, vel4, axis, nbins, scale, sums, counts);
  return hipGetLastError();
}

hipError_t launch_obs_final(hipStream_t s, int nbins, const double *sums,
                            const unsigned long long *counts, double *profile,
                            int64_t *counts_out) {
  k_obs_final<<<(nbins + 255) / 256, 256, 0, s>>>(nbins, sums, counts, profile, counts_out);
  return hipGetLastError();
}

hipError_t launch_loss_weights(hipStream_t s, int nbins, const double *dldp,
                               const unsigned long long *counts, float *lw) {
  k_loss_weights<<<(nbins + 255) / 256, 256, 0, s>>>(nbins, dldp, counts, lw);
  return hipGetLastError();
}

hipError_t launch_vt_from_v(hipStream_t s, int64_t nf, const float4 *vel4, float4 *vt4) {
  if (nf <= 0) return hipSuccess;
  k_vt_from_v<<<grid_a(nf), kBlockA, 0, s>>>(nf, vel4, vt4);
  return hipGetLastError();
}

hipError_t launch_set_u64(hipStream_t s, unsigned long long *p, unsigned long long v) {
  k_set_u64<<<1, 1, 0, s>>>(p, v);
  return hipGetLastError();
}

int adj_prep_blocks(int64_t nf) { return nf > 0 ? (int)grid_a(nf) : 0; }

hipError_t launch_adj_prep(hipStream_t s, const Box *boxes, int64_t nf, int initial,
                           const int32_t *idx, const float4 *pos4, const float4 *vt4,
                           const float4 *rb_s, const float4 *vb_s, const float4 *fb_s,
                           const float *lw, int axis, int nbins, float scale, float4 *rn,
                           float4 *vn, float4 *fbar, double *part_g) {
  if (nf <= 0) return hipSuccess;
  k_adj_prep<<<grid_a(nf), kBlockA, 0, s>>>(boxes, nf, initial, idx, pos4, vt4, rb_s, vb_s,
                                            fb_s, lw, axis, nbins, scale, rn, vn, fbar, part_g);
  return hipGetLastError();
}

int force_vjp_blocks(int ntiles) { return ((ntiles + 7) / 8) * 8; }

hipError_t launch_force_vjp(hipStream_t s, int block, const Box *boxes, const Tile *tiles,
                            int ntiles, int64_t NF, int32_t pad, const float4 *pos4,
                            const float4 *vt4, const int32_t *idx, const int32_t *idx_all,
                            const int32_t *start_all, const float4 *fbar, const float4 *rn,
                            float4 *rt_out, float4 *vt_out, const unsigned long long *dk0,
                            unsigned long long koff, double *part) {
  if (ntiles <= 0) return hipSuccess;
  const unsigned nb = (unsigned)force_vjp_blocks(ntiles);
  if (block == 128)
    k_force_vjp<128><<<nb, 128, 0, s>>>(boxes, tiles, ntiles, NF, pad, pos4, vt4, idx, idx_all,
                                        start_all, fbar, rn, rt_out, vt_out, dk0, koff, part);
  else
    k_force_vjp<256><<<nb, 256, 0, s>>>(boxes, tiles, ntiles, NF, pad, pos4, vt4, idx, idx_all,
                                        start_all, fbar, rn, rt_out, vt_out, dk0, koff, part);
  return hipGetLastError();
}

hipError_t launch_integrate_vjp(hipStream_t s, const Box *boxes, int64_t nf, const float4 *pos_t,
                                const float4 *vel_t, const float4 *frc_t, const float4 *vt4,
                                const float4 *rt, const float4 *vtb, const float4 *vn,
                                const void *grid, int grid_f64, double *dphi, float4 *rb_out,
                                float4 *vb_out, float4 *fb_out) {
  if (nf <= 0) return hipSuccess;
  if (grid_f64)
    k_integrate_vjp<double><<<grid_a(nf), kBlockA, 0, s>>>(
        boxes, nf, pos_t, vel_t, frc_t, vt4, rt, vtb, vn, (const double *)grid, dphi, rb_out,
        vb_out, fb_out);
  else
    k_integrate_vjp<float><<<grid_a(nf), kBlockA, 0, s>>>(
        boxes, nf, pos_t, vel_t, frc_t, vt4, rt, vtb, vn, (const float *)grid, dphi, rb_out,
        vb_out, fb_out);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(hipStream_t s, int nb_f, const double *part_f, int nb_g,
                                  const double *part_g, double *out) {
  k_reduce_partials<<<1, 64, 0, s>>>(nb_f, part_f, nb_g, part_g, out);
  return hipGetLastError();
}

}  // namespace dpd
