// Pair force (Eq. 2-10) on LDS-staged cell bricks, with the body force and
// the velocity update of the Groot-Warren step.
//
// A block owns a brick of cells of one box (up to kBrickX x kBrickY x
// kBrickZ).  It stages the brick and a one-cell halo into LDS, once: each
// cell's merged run (walls, then fluid) becomes a contiguous run of staged
// particles in haloed-cell order (x fastest), so the three x-neighbours of a
// row are one contiguous range.  Positions are staged in the brick's frame:
// a column seen across the periodic edge is moved by -L (its coordinates
// lie in [L/2, L), so the move is exact), and a brick whose halo wraps past
// the high edge moves all its other columns by -L instead.  In that frame
// the separation of any staged pair is one FP32 subtraction, and it is the
// exact minimum-image difference rounded once, i.e. the pair decision and
// separation of every other path.
//
// Candidate walk: a task is one home fluid particle and one plane of its
// neighbourhood (three rows, about 36 candidates); 64 tasks run per
// wavefront, four candidates per lane and pass, read from LDS.  An
// interacting pair (r^2 < rc^2) whose partner is a home fluid particle of
// the brick is kept only from the side with the smaller LDS index (Newton's
// third law, Eq. 2: f_ji = -f_ij); pairs with walls or halo particles are
// kept from the home side.  Kept pairs are appended to the wavefront's ring
// queue (ballot + mbcnt), and whenever it holds 64 of them all 64 lanes
// evaluate one pair each: the counter-based random number and the force,
// rounded to a 64-bit fixed-point number (units of 2^-32) and added with
// LDS atomics to the home particle, and negated to a home partner.
//
// Integer sums do not depend on their order: a particle's force is
// 2^-32 sum_j round(2^32 F_ij) + g, whatever the wave schedule, the brick
// decomposition or the pair's owner, and F_ji = -F_ij bit for bit (the
// arithmetic is symmetric in i and j), so results are reproducible run to
// run and the same for a box alone or in a batch.
//
// A brick whose haloed region holds more particles than LDS takes is split
// in two along its longest axis, recursively, down to single cells.
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"

namespace dpd {
namespace {

constexpr int kBT = 256;                 // threads per block
constexpr int kWaves = kBT / 64;
constexpr int kHCmax = (kBrickX + 2) * (kBrickY + 2) * (kBrickZ + 2);
constexpr int kCap = 1152;               // staged particles
constexpr int kHomeCap = 384;            // home fluid particles
constexpr int kQ = 256;                  // per-wavefront ring of kept pairs
constexpr int kStack = 16;               // sub-bricks pending
constexpr int kPass = 4;                 // candidates per lane and pass
constexpr int kStagePer = (kCap + kBT - 1) / kBT;
constexpr int kHomePer = (kHomeCap + kBT - 1) / kBT;
constexpr float kFix = 4294967296.0f;     // 2^32
constexpr float kFixInv = 2.3283064365386963e-10f;   // 2^-32

struct BrickShared {
  // staged particles: position in the brick frame, w = home slot (int bits)
  // of a home fluid particle or -1; kPass spare entries so that a pass may
  // read past the end of a run
  float4 P[kCap + kPass];
  uint32_t gid[kCap];
  int32_t J[kCap];                    // storage index: fluid i, or NF + w for walls
  unsigned long long acc[3 * kHomeCap];   // fixed-point force sums
  int16_t hl[kHomeCap];               // staged index of home slot h
  int16_t hc[kHomeCap];               // haloed cell of home slot h
  int32_t hs[kHomeCap];               // global fluid slot of home slot h
  int32_t cs[kHCmax + 1];             // staged start of each haloed cell's run
  int32_t hstart[kHCmax + 1];         // home-slot start of each haloed cell
  int32_t run[kHCmax];                // merged-run start (start_all) of each haloed cell
  int32_t fslot[kHCmax];              // fluid slot start (cstart) of each home cell
  int16_t nwall[kHCmax];              // walls at the head of each haloed cell's run
  union {
    int16_t ecell[kCap];              // haloed cell of each staged particle (staging)
    uint32_t queue[kWaves][kQ + 64];  // kept pairs (walk); the last 64: discarded appends
  } u;
  int32_t wsum[2][kWaves];
  int32_t stack[kStack][6];
};

// Exclusive scan of a[0..n) and b[0..n) in place, with the totals written to
// a[n] and b[n] (n <= kHCmax); each thread scans a few consecutive entries.
__device__ __forceinline__ void block_scan2(int32_t *a, int32_t *b, int n, int32_t (*wsum)[kWaves]) {
  constexpr int kPer = (kHCmax + kBT - 1) / kBT;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int first = t * kPer;
  int sa = 0, sb = 0;
  int va[kPer], vb[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = first + k;
    va[k] = i < n ? a[i] : 0;
    vb[k] = i < n ? b[i] : 0;
    sa += va[k];
    sb += vb[k];
  }
  int ia = sa, ib = sb;
  for (int off = 1; off < 64; off <<= 1) {
    const int xa = __shfl_up(ia, off, 64), xb = __shfl_up(ib, off, 64);
    if (lane >= off) {
      ia += xa;
      ib += xb;
    }
  }
  if (lane == 63) {
    wsum[0][w] = ia;
    wsum[1][w] = ib;
  }
  __syncthreads();
  int oa = 0, ob = 0, ta = 0, tb = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    const int xa = wsum[0][k], xb = wsum[1][k];
    oa += k < w ? xa : 0;
    ob += k < w ? xb : 0;
    ta += xa;
    tb += xb;
  }
  int ea = oa + ia - sa, eb = ob + ib - sb;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = first + k;
    if (i < n) {
      a[i] = ea;
      b[i] = eb;
    }
    ea += va[k];
    eb += vb[k];
  }
  if (t == 0) {
    a[n] = ta;
    b[n] = tb;
  }
  __syncthreads();
}

// A force component as a 64-bit fixed-point integer in units of 2^-32,
// rounded to nearest (ties to even), so that the value of -f is exactly the
// negation of the value of f.  s = rint(f 2^32) is an integer-valued float;
// hi = floor(s 2^-32) and lo = s - hi 2^32 in [0, 2^32) are exact.
__device__ __forceinline__ long long to_fixed(float f) {
  const float s = __builtin_rintf(f * kFix);
  const float hi = floorf(s * kFixInv);
  const float lo = __builtin_fmaf(-hi, kFix, s);
  return (long long)(((unsigned long long)(uint32_t)(int)hi << 32) | (unsigned long long)(uint32_t)lo);
}

template <bool SPH>
__device__ __forceinline__ void pair_force(const KParams &P, float dx, float dy, float dz,
                                           float4 vti, float4 vtj, bool wall, uint32_t gi,
                                           uint32_t gj, uint32_t klo, uint32_t khi, float &fx,
                                           float &fy, float &fz, float &mag_out) {
  const float r2 = dx * dx + dy * dy + dz * dz;
  const float rinv = rsqrtf(r2);
  const float r = r2 * rinv;
  const float w = fmaxf(1.0f - r * P.inv_rc, 0.0f);
  const float ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
  const float edv = ex * (vti.x - vtj.x) + ey * (vti.y - vtj.y) + ez * (vti.z - vtj.z);
  const float xi = pair_gauss(gi, gj, klo, khi, P.key0, P.key1);
  float mag;
  if (SPH && P.sph) {
    const float cr = wall ? P.cr_fw : P.cr_ff, ca = wall ? P.ca_fw : P.ca_ff;
    const float fc = ca * spline_dp(r * P.inv_ha) - cr * spline_dp(r * P.inv_hr);
    mag = fc + w * (P.sigma_rdt * xi - P.gamma * w * edv);
  } else {
    const float a = wall ? P.a_fw : P.a_ff;
    mag = w * (a - P.gamma * w * edv + P.sigma_rdt * xi);
  }
  fx = mag * ex;
  fy = mag * ey;
  fz = mag * ez;
  mag_out = mag;
}

template <bool INIT, bool SPH>
__global__ __launch_bounds__(kBT) void k_force_brick(
    const Box *__restrict__ boxes, const Brick *__restrict__ bricks, int nbricks, int64_t NF,
    int32_t pad, const float4 *__restrict__ pos4, const float4 *__restrict__ vt4,
    const float4 *__restrict__ vel4, const float4 *__restrict__ frc4,
    const int32_t *__restrict__ idx_all, const int32_t *__restrict__ start_all,
    const int32_t *__restrict__ fluid_off, const int32_t *__restrict__ cstart,
    float4 *__restrict__ pos_out, float4 *__restrict__ vel_out, float4 *__restrict__ frc_out,
    const unsigned long long *__restrict__ dk, Status *st) {
  __shared__ BrickShared S;
  const int b = xcd_block();
  if (b >= nbricks) return;
  const Brick bk = bricks[b];
  const Box &B = boxes[bk.box];
  const KGeom G = B.G;
  const KParams P = B.P;
  const int co = (int)B.co;
  const int nx = G.nc[0], ny = G.nc[1], nz = G.nc[2];
  const unsigned long long kk = *dk;
  const uint32_t klo = (uint32_t)kk;
  const uint32_t khi = ((uint32_t)(kk >> 32) & 0xFFFFu) | (P.replica << 16);
  const Records16 posr(pos4, pad + 1), vtr(vt4, pad + 1), velr(vel4, (int)NF),
      frcr(frc4, (int)NF);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  bool bad = false;      // a non-finite or out-of-range pair force (this thread)
  bool dense = false;    // a single cell whose neighbourhood exceeds LDS

  if (tid == 0) {
    S.stack[0][0] = bk.x0;
    S.stack[0][1] = bk.y0;
    S.stack[0][2] = bk.z0;
    S.stack[0][3] = bk.sx;
    S.stack[0][4] = bk.sy;
    S.stack[0][5] = bk.sz;
  }
  __syncthreads();
  int sp = 1;
  while (sp > 0) {
    --sp;
    const int x0 = S.stack[sp][0], y0 = S.stack[sp][1], z0 = S.stack[sp][2];
    const int sx = S.stack[sp][3], sy = S.stack[sp][4], sz = S.stack[sp][5];
    const int HX = sx + 2, HY = sy + 2, HZ = sz + 2, HC = HX * HY * HZ;
    // frame per axis: the halo wraps past the high edge (every non-wrapped
    // column moves by -L) or not (only the column seen across the low edge
    // moves by -L)
    const bool hix = x0 + sx == nx, hiy = y0 + sy == ny, hiz = z0 + sz == nz;

    // counts of each haloed cell's run and of the fluid of home cells, and
    // the fluid slot start of home cells (one level of global loads)
    for (int c = tid; c < HC; c += kBT) {
      const int a = c % HX, bb = (c / HX) % HY, cc = c / (HX * HY);
      int gx = x0 - 1 + a, gy = y0 - 1 + bb, gz = z0 - 1 + cc;
      gx += gx < 0 ? nx : (gx >= nx ? -nx : 0);
      gy += gy < 0 ? ny : (gy >= ny ? -ny : 0);
      gz += gz < 0 ? nz : (gz >= nz ? -nz : 0);
      const int gc = co + (gz * ny + gy) * nx + gx;
      const bool home = a >= 1 && a <= sx && bb >= 1 && bb <= sy && cc >= 1 && cc <= sz;
      const int r0 = start_all[gc], r1 = start_all[gc + 1], f0 = fluid_off[gc];
      const int fs = home ? cstart[gc] : 0;
      S.run[c] = r0;
      S.nwall[c] = (int16_t)(f0 - r0);
      S.cs[c] = r1 - r0;
      S.hstart[c] = home ? r1 - f0 : 0;
      S.fslot[c] = fs;
    }
    __syncthreads();
    block_scan2(S.cs, S.hstart, HC, S.wsum);
    const int N = S.cs[HC], H = S.hstart[HC];
    if (N > kCap || H > kHomeCap) {
      // split along the longest axis (z, then y, then x on ties)
      if (sx * sy * sz == 1 || sp + 2 > kStack) {
        dense = true;
      } else {
        if (tid == 0) {
          int h0[6] = {x0, y0, z0, sx, sy, sz}, h1[6] = {x0, y0, z0, sx, sy, sz};
          const int ax = (sz >= sy && sz >= sx) ? 2 : (sy >= sx ? 1 : 0);
          const int half = h0[3 + ax] / 2;
          h0[3 + ax] = half;
          h1[ax] += half;
          h1[3 + ax] -= half;
          for (int k = 0; k < 6; ++k) {
            S.stack[sp][k] = h0[k];
            S.stack[sp + 1][k] = h1[k];
          }
        }
        sp += 2;
      }
      __syncthreads();
      continue;
    }
    if (H == 0) {
      __syncthreads();
      continue;
    }

    // the haloed cell of every staged particle
    for (int c = tid; c < HC; c += kBT) {
      const int k0 = S.cs[c], k1 = S.cs[c + 1];
      for (int k = k0; k < k1; ++k) S.u.ecell[k] = (int16_t)c;
    }
    __syncthreads();

    // stage positions in the brick frame (w = -1 for now), gids, storage indices
    {
      int tk[kStagePer], jk[kStagePer];
      float shx[kStagePer], shy[kStagePer], shz[kStagePer];
#pragma unroll
      for (int m = 0; m < kStagePer; ++m) {
        const int k = tid + m * kBT;
        tk[m] = -1;
        shx[m] = shy[m] = shz[m] = 0.f;
        if (k < N) {
          const int c = S.u.ecell[k];
          const int a = c % HX, bb = (c / HX) % HY, cc = c / (HX * HY);
          tk[m] = S.run[c] + (k - S.cs[c]);
          const int gx = x0 - 1 + a, gy = y0 - 1 + bb, gz = z0 - 1 + cc;
          shx[m] = (hix ? gx < nx : gx < 0) ? G.L[0] : 0.f;
          shy[m] = (hiy ? gy < ny : gy < 0) ? G.L[1] : 0.f;
          shz[m] = (hiz ? gz < nz : gz < 0) ? G.L[2] : 0.f;
        }
      }
#pragma unroll
      for (int m = 0; m < kStagePer; ++m) jk[m] = tk[m] >= 0 ? idx_all[tk[m]] : pad;
#pragma unroll
      for (int m = 0; m < kStagePer; ++m) {
        const float4 p = posr[jk[m]];
        const int k = tid + m * kBT;
        if (tk[m] >= 0) {
          S.P[k] = make_float4(sub_nc(p.x, shx[m]), sub_nc(p.y, shy[m]), sub_nc(p.z, shz[m]),
                               __int_as_float(-1));
          S.gid[k] = __float_as_uint(p.w);
          S.J[k] = jk[m];
        }
      }
    }
    __syncthreads();

    // home slots: the fluid part of each home cell's run, in run order
    for (int hcl = tid; hcl < sx * sy * sz; hcl += kBT) {
      const int a = 1 + hcl % sx, bb = 1 + (hcl / sx) % sy, cc = 1 + hcl / (sx * sy);
      const int c = (cc * HY + bb) * HX + a;
      const int h0 = S.hstart[c], nh = S.hstart[c + 1] - h0;
      const int k0 = S.cs[c] + S.nwall[c];
      const int s0 = S.fslot[c];
      for (int e = 0; e < nh; ++e) {
        S.P[k0 + e].w = __int_as_float(h0 + e);
        S.hl[h0 + e] = (int16_t)(k0 + e);
        S.hc[h0 + e] = (int16_t)c;
        S.hs[h0 + e] = s0 + e;
        S.acc[3 * (h0 + e)] = 0ull;
        S.acc[3 * (h0 + e) + 1] = 0ull;
        S.acc[3 * (h0 + e) + 2] = 0ull;
      }
    }
    __syncthreads();

    // this thread's home particles: their state is fetched now and used
    // after the walk
    int hi_[kHomePer];
    float4 vo[kHomePer], fo[kHomePer], vti[kHomePer], po[kHomePer];
#pragma unroll
    for (int m = 0; m < kHomePer; ++m) {
      const int h = tid + m * kBT;
      hi_[m] = h < H ? S.J[S.hl[h]] : 0;
    }
#pragma unroll
    for (int m = 0; m < kHomePer; ++m) {
      po[m] = posr[hi_[m]];
      vo[m] = velr[hi_[m]];
      vti[m] = vtr[hi_[m]];
      fo[m] = INIT ? make_float4(0.f, 0.f, 0.f, 0.f) : frcr[hi_[m]];
    }

    // candidate walk and pair rounds, per wavefront
    {
      uint32_t *const q = S.u.queue[wave];
      uint32_t qh = 0, qt = 0;   // ring head and tail (wavefront-uniform)
      // one round: lane l evaluates queued pair qh + l (if any)
      auto round = [&](int count) {
        const bool act = lane < count;
        const uint32_t e = q[(qh + (uint32_t)lane) & (kQ - 1)];
        const int ki = act ? (int)(e >> 16) : 0, kj = act ? (int)(e & 0xFFFFu) : 0;
        const float4 pi = S.P[ki], pj = S.P[kj];
        const int Ji = S.J[ki], Jj = S.J[kj];
        const uint32_t gi = S.gid[ki], gj = S.gid[kj];
        const float4 vi = vtr[act ? Ji : pad];
        const float4 vj = vtr[act ? Jj : pad];
        if (act) {
          float fx, fy, fz, mag;
          pair_force<SPH>(P, pi.x - pj.x, pi.y - pj.y, pi.z - pj.z, vi, vj, (int64_t)Jj >= NF,
                          gi, gj, klo, khi, fx, fy, fz, mag);
          bad |= !(fabsf(mag) < 1.0e9f);
          const long long cx = to_fixed(fx), cy = to_fixed(fy), cz = to_fixed(fz);
          const int si = __float_as_int(pi.w), sj = __float_as_int(pj.w);
          atomicAdd(&S.acc[3 * si], (unsigned long long)cx);
          atomicAdd(&S.acc[3 * si + 1], (unsigned long long)cy);
          atomicAdd(&S.acc[3 * si + 2], (unsigned long long)cz);
          if (sj >= 0) {
            atomicAdd(&S.acc[3 * sj], (unsigned long long)(-cx));
            atomicAdd(&S.acc[3 * sj + 1], (unsigned long long)(-cy));
            atomicAdd(&S.acc[3 * sj + 2], (unsigned long long)(-cz));
          }
        }
        qh += (uint32_t)count;
      };
      const int ntask = 3 * H;
      for (int base = wave * 64; base < ntask; base += kBT) {
        const int task = base + lane;
        const bool live = task < ntask;
        const int h = live ? task / 3 : 0;
        const int dz = live ? task - 3 * h - 1 : 0;
        const int ki = S.hl[h];
        const float4 a = S.P[ki];
        const int hcell = S.hc[h];
        const int ha = hcell % HX, hb = (hcell / HX) % HY, hcz = hcell / (HX * HY);
        // rows dy = -1, 0, 1 of plane hcz + dz: cells ha - 1 .. ha + 1
        int rb = ((hcz + dz) * HY + hb - 1) * HX + ha - 1;
        int row = live ? 0 : 3;
        int t = live ? S.cs[rb] : 0, tend = live ? S.cs[rb + 3] : 0;
        const uint32_t key = (uint32_t)ki << 16;
        for (;;) {
          // advance lanes whose row is exhausted (skipping empty rows)
          bool need = row < 3 && t >= tend;
          while (wave_any(need)) {
            if (need) {
              ++row;
              rb += HX;
              const bool more = row < 3;
              t = more ? S.cs[rb] : 0;
              tend = more ? S.cs[rb + 3] : 0;
            }
            need = row < 3 && t >= tend;
          }
          if (!wave_any(t < tend)) break;
          // kPass candidates t .. t + kPass - 1 (the spare entries make the
          // reads past a run's end safe; those candidates are masked)
          float4 cq[kPass];
#pragma unroll
          for (int v = 0; v < kPass; ++v) cq[v] = S.P[t + v];
#pragma unroll
          for (int v = 0; v < kPass; ++v) {
            const float r2 = pair_r2(sub_nc(a.x, cq[v].x), sub_nc(a.y, cq[v].y),
                                     sub_nc(a.z, cq[v].z));
            // r2 > 0 drops i itself (and a coincident particle, which exerts
            // no force); a home partner is kept from the lower index only
            const bool keep = (t + v < tend) & (r2 < P.rc2) & (r2 > 0.0f) &
                              ((__float_as_int(cq[v].w) < 0) | (t + v > ki));
            const unsigned long long m = __ballot(keep);
            const uint32_t off = (uint32_t)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            const uint32_t slot = keep ? ((qt + off) & (kQ - 1)) : (uint32_t)(kQ + lane);
            q[slot] = key | (uint32_t)(t + v);
            qt += (uint32_t)__popcll(m);
            // at most 63 pending + 2 x 64 appended < kQ between drains
            if (v & 1)
              while (qt - qh >= 64u) round(64);
          }
          t += kPass;
        }
      }
      while (qt != qh) round((int)min(64u, qt - qh));
    }
    __syncthreads();

    // the sums: forces, velocity update, outputs in cell-sorted slot order
#pragma unroll
    for (int m = 0; m < kHomePer; ++m) {
      const int h = tid + m * kBT;
      if (h >= H) continue;
      const int s = S.hs[h];
      double f3[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long long v = (long long)S.acc[3 * h + c];
        f3[c] = (double)v * 2.3283064365386963e-10 + (double)P.g[c];
      }
      const float fx = (float)f3[0], fy = (float)f3[1], fz = (float)f3[2];
      float4 vn;
      if (INIT) {
        vn = make_float4(vo[m].x, vo[m].y, vo[m].z, __int_as_float(0));
      } else {
        const int event = __float_as_int(vti[m].w);
        if (event) {
          vn = make_float4(vti[m].x, vti[m].y, vti[m].z, __int_as_float(event));
        } else {
          vn = make_float4(vo[m].x + P.hdt * (fo[m].x + fx), vo[m].y + P.hdt * (fo[m].y + fy),
                           vo[m].z + P.hdt * (fo[m].z + fz), __int_as_float(0));
        }
      }
      pos_out[s] = po[m];
      vel_out[s] = vn;
      frc_out[s] = make_float4(fx, fy, fz, 0.f);
    }
    __syncthreads();
  }
  if (bad) atomicAdd(&st->nonfinite, 1ull);
  if (dense && tid == 0) atomicAdd(&st->unstable, 1ull);
}

}  // namespace

hipError_t launch_force_brick(hipStream_t s, const Box *boxes, const Brick *bricks, int nbricks,
                              int64_t NF, int32_t pad, int init, const float4 *pos4,
                              const float4 *vt4, const float4 *vel4, const float4 *frc4,
                              const int32_t *idx_all, const int32_t *start_all,
                              const int32_t *fluid_off, const int32_t *cstart, float4 *pos_out,
                              float4 *vel_out, float4 *frc_out, const unsigned long long *dk,
                              Status *st, int sph) {
  if (nbricks <= 0) return hipSuccess;
  const unsigned nb = (unsigned)(((nbricks + 7) / 8) * 8);
#define DPD_BRICK(I, SP)                                                                       \
  k_force_brick<I, SP><<<nb, kBT, 0, s>>>(boxes, bricks, nbricks, NF, pad, pos4, vt4, vel4,    \
                                           frc4, idx_all, start_all, fluid_off, cstart,        \
                                           pos_out, vel_out, frc_out, dk, st)
  if (init) {
    if (sph) DPD_BRICK(true, true); else DPD_BRICK(true, false);
  } else {
    if (sph) DPD_BRICK(false, true); else DPD_BRICK(false, false);
  }
#undef DPD_BRICK
  return hipGetLastError();
}

}  // namespace dpd
