/*
 * FP64 oracle for one DPD time step of fluid particles and frozen wall
 * particles with phase-field bounce-back at the phi = 0 level set
 * (Xu & Meakin, "A phase field approach to no slip boundary conditions in
 * dissipative particle dynamics ...").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * Plain and slow on purpose: per-particle loops over all candidates, FP64
 * physics, no blocking, no fusion.  Where a floating-point comparison decides
 * an integer (the cell of a particle, whether a pair is within the cutoff,
 * whether a particle crossed phi = 0) the decision is taken in the precision
 * the GPU kernels use, FP32 (or FP64 for an FP64 phi grid), with the op
 * order written out below and no contraction (-ffp-contract=off), so that
 * both sides take the same discrete decisions from the same FP32 inputs.
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes):
 *   - random force sigma*w*xi/sqrt(dt) (Groot-Warren discretisation of Eq. 7)
 *   - modified velocity-Verlet of Groot & Warren with parameter lambda
 *   - d = sqrt(2)eps*atanh(phi) (Eq. 16 prints tanh; Sec. II.C uses atanh)
 *   - Eq. 17 with the start-of-step velocity v^t as printed; if the mirrored
 *     point is still in the solid the particle returns to r^t
 *   - after a bounce v = -v^t and the predicted velocity is -v^t as well
 *   - moving walls (Sec. II.C): a wall particle's velocity is the velocity of
 *     its solid, a body that keeps its shape and phase field while it moves
 *     (a plate sliding in its own plane): wall particles translate with it,
 *     r_w += dt v_w, and carry it as their predicted velocity in the pair
 *     forces.  A reflection takes v_wall from the wall particle nearest to r*
 *     (start-of-step wall positions, the 27-cell neighbourhood of r*'s cell,
 *     the FP32 pair-decision distance, ties to the smaller gid; none: zero),
 *     uses v^t - v_wall in Eq. 17 and leaves v = -v^t + 2 v_wall
 *   - specular reflection (Sec. I): only the component of v^t - v_wall along
 *     the normal n = grad Phi / |grad Phi| at r* is reversed, in the velocity
 *     and in the Eq. 17 displacement; |grad Phi| = 0 falls back to
 *     bounce-back
 *   - atanh arguments clamped to [0, 1 - 2^-20]
 *   - the attractive-repulsive force of Eq. 22-24 replaces a w when enabled:
 *     the conservative force is -dE/dr along r_i - r_j (Eq. 24 prints the
 *     derivative without the minus sign, which would make the repulsive
 *     term attract); dissipative and random forces keep w = 1 - r/rc
 *   - mass 1, box periodic in all three axes, phi grid periodic and
 *     node-centred, trilinear interpolation ("linear interpolation", Sec. II.C)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies by
 * 0xD2511F53 and 0xCD9E8D57 with a Weyl key schedule 0x9E3779B9, 0xBB67AE85.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Pair-symmetric Gaussian xi_ij of Eq. 7 for force evaluation k: the Philox
 * counter is (min gid, max gid, k low word, k bits 32..47 | replica << 16),
 * the key the 64-bit seed.  Box-Muller (1958) on u1 = (x0>>9 + 1/2) 2^-23 in
 * (0,1) and u2 = (x1>>9) 2^-23 in [0,1): xi = sqrt(-2 ln u1) cos(2 pi u2).
 * Swapping i and j gives the same counter, hence xi_ij = xi_ji. */
void orc_uniform_pair(uint64_t seed, uint32_t gi, uint32_t gj, uint64_t k,
                      uint32_t replica, uint32_t out[4])
{
    uint32_t lo = gi < gj ? gi : gj;
    uint32_t hi = gi < gj ? gj : gi;
    uint32_t ctr[4] = {lo, hi, (uint32_t)k,
                       ((uint32_t)(k >> 32) & 0xFFFFu) | (replica << 16)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

double orc_xi(uint64_t seed, uint32_t gi, uint32_t gj, uint64_t k, uint32_t replica)
{
    uint32_t o[4];
    orc_uniform_pair(seed, gi, gj, k, replica, o);
    double u1 = ((double)(o[0] >> 9) + 0.5) * 0x1p-23;
    double u2 = (double)(o[1] >> 9) * 0x1p-23;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * ORC_PI * u2);
}

/* xi for the pairs (gi, gj0 + m), m = 0..count-1, at evaluation k. */
void orc_xi_fill(uint64_t seed, uint32_t gi, uint32_t gj0, int64_t count,
                 uint64_t k, uint32_t replica, double *out)
{
    for (int64_t m = 0; m < count; ++m)
        out[m] = orc_xi(seed, gi, gj0 + (uint32_t)m, k, replica);
}

/* Philox words and xi for arrays of pairs (gi[m], gj[m]) at evaluation k;
 * words (n x 4) or xi (n) may be NULL. */
void orc_pairs_random(uint64_t seed, const uint32_t *gi, const uint32_t *gj, int64_t n,
                      uint64_t k, uint32_t replica, uint32_t *words, double *xi)
{
    #pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < n; ++m) {
        if (words) orc_uniform_pair(seed, gi[m], gj[m], k, replica, words + 4 * m);
        if (xi) xi[m] = orc_xi(seed, gi[m], gj[m], k, replica);
    }
}

/* ------------------------------------------------------------------------
 * Geometry shared by every routine below.
 * ---------------------------------------------------------------------- */
typedef struct {
    double L[3];        /* periodic box edges */
    int32_t nc[3];      /* cells per axis, floor(L/rc) (>= 3) */
    float L32[3];       /* (float)L */
    float invw32[3];    /* (float)(nc/L): cell decision scale */
    int32_t ng[3];      /* phi grid nodes per axis (x, y, z) */
    double h[3];        /* phi grid spacing */
    float inv_h32[3];   /* (float)(1/h) for the FP32 decision */
    double inv_h64[3];  /* 1/h for the FP64 decision */
    const double *phi64;  /* grid values as double, [nz][ny][nx] */
    const float *phi32;   /* FP32 grid, or NULL when the grid is FP64 */
} orc_geom;

typedef struct {
    double a[2][2];     /* a_ij by type (0 fluid, 1 wall), Eq. 4 */
    double gamma;       /* Eq. 6 */
    double kBT;         /* Eq. 8 */
    double rc;          /* cutoff, Eq. 5 */
    double dt;
    double lambda;      /* Groot-Warren predictor weight */
    double g[3];        /* body force on fluid particles */
    uint64_t seed;
    uint32_t replica;
    int32_t specular;   /* 1: specular reflection, 0: bounce-back */
    int32_t sph;        /* 1: conservative force of Eq. 22-24 instead of a w */
    double sr[2][2];    /* S^r_ij: repulsive strengths by type */
    double sa[2][2];    /* S^a_ij: attractive strengths by type */
    double r0r, r0a;    /* their ranges r0^r, r0^a (support of W) */
} orc_params;

static int orc_mod(int a, int n)
{
    int m = a % n;
    return m < 0 ? m + n : m;
}

/* Cell coordinate of an FP32 coordinate: floor(fl(x * invw)) clamped to
 * [0, n-1]. */
static int cell_coord(float x, float invw, int n)
{
    float g = x * invw;
    float fg = floorf(g);
    int c;
    if (fg < 0.0f) c = 0;
    else if (fg > (float)(n - 1)) c = n - 1;
    else c = (int)fg;
    return c;
}

int32_t orc_cell_of(const orc_geom *G, const float x[3])
{
    int cx = cell_coord(x[0], G->invw32[0], G->nc[0]);
    int cy = cell_coord(x[1], G->invw32[1], G->nc[1]);
    int cz = cell_coord(x[2], G->invw32[2], G->nc[2]);
    return (cz * G->nc[1] + cy) * G->nc[0] + cx;
}

/* FP32 periodic wrap by a single box edge; returns the image shift applied. */
static int wrap32(float *x, float L)
{
    if (*x >= L) { *x = *x - L; return -1; }
    if (*x < 0.0f) { *x = *x + L; return 1; }
    return 0;
}

/* ------------------------------------------------------------------------
 * Phase field at a point (Sec. II.C: phi_i by linear interpolation of the
 * finite-difference grid; trilinear in 3-D).  Nodes at (i h_x, j h_y, k h_z),
 * periodic.  The decision forms follow lerp(a, b, t) = a + t (b - a): four
 * lerps along x, two along y, one along z.
 * ---------------------------------------------------------------------- */
static float lerp32(float a, float b, float t) { return a + t * (b - a); }
static double lerp64(double a, double b, double t) { return a + t * (b - a); }

float orc_phi_decide32(const orc_geom *G, const float x[3])
{
    int i0[3], i1[3];
    float t[3];
    for (int k = 0; k < 3; ++k) {
        float g = x[k] * G->inv_h32[k];
        float fg = floorf(g);
        t[k] = g - fg;
        i0[k] = orc_mod((int)fg, G->ng[k]);
        i1[k] = orc_mod(i0[k] + 1, G->ng[k]);
    }
    const float *p = G->phi32;
    const int nx = G->ng[0], ny = G->ng[1];
    float e[2][2];
    for (int dz = 0; dz < 2; ++dz) {
        int kz = dz ? i1[2] : i0[2];
        for (int dy = 0; dy < 2; ++dy) {
            int ky = dy ? i1[1] : i0[1];
            const float *row = p + ((size_t)kz * ny + ky) * nx;
            e[dz][dy] = lerp32(row[i0[0]], row[i1[0]], t[0]);
        }
    }
    float y0 = lerp32(e[0][0], e[0][1], t[1]);
    float y1 = lerp32(e[1][0], e[1][1], t[1]);
    return lerp32(y0, y1, t[2]);
}

double orc_phi_decide64(const orc_geom *G, const float x32[3])
{
    int i0[3], i1[3];
    double t[3];
    for (int k = 0; k < 3; ++k) {
        double g = (double)x32[k] * G->inv_h64[k];
        double fg = floor(g);
        t[k] = g - fg;
        i0[k] = orc_mod((int)fg, G->ng[k]);
        i1[k] = orc_mod(i0[k] + 1, G->ng[k]);
    }
    const double *p = G->phi64;
    const int nx = G->ng[0], ny = G->ng[1];
    double e[2][2];
    for (int dz = 0; dz < 2; ++dz) {
        int kz = dz ? i1[2] : i0[2];
        for (int dy = 0; dy < 2; ++dy) {
            int ky = dy ? i1[1] : i0[1];
            const double *row = p + ((size_t)kz * ny + ky) * nx;
            e[dz][dy] = lerp64(row[i0[0]], row[i1[0]], t[0]);
        }
    }
    double y0 = lerp64(e[0][0], e[0][1], t[1]);
    double y1 = lerp64(e[1][0], e[1][1], t[1]);
    return lerp64(y0, y1, t[2]);
}

/* The phi < 0 test in the precision of the grid. */
static int phi_negative(const orc_geom *G, const float x32[3])
{
    if (G->phi32) return orc_phi_decide32(G, x32) < 0.0f;
    return orc_phi_decide64(G, x32) < 0.0;
}

/* Trilinear interpolant and its exact gradient in FP64 (physics form):
 * Phi(x) = sum_{abc} phi_abc W_a(tx) W_b(ty) W_c(tz), W_0 = 1 - t, W_1 = t. */
double orc_phi64(const orc_geom *G, const double x[3], double grad[3])
{
    int i[3][2];
    double t[3];
    for (int k = 0; k < 3; ++k) {
        double g = x[k] / G->h[k];
        double fg = floor(g);
        t[k] = g - fg;
        i[k][0] = orc_mod((int)fg, G->ng[k]);
        i[k][1] = orc_mod(i[k][0] + 1, G->ng[k]);
    }
    const int nx = G->ng[0], ny = G->ng[1];
    double val = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int c = 0; c < 2; ++c) {
        double wz = c ? t[2] : 1.0 - t[2], dwz = c ? 1.0 : -1.0;
        for (int b = 0; b < 2; ++b) {
            double wy = b ? t[1] : 1.0 - t[1], dwy = b ? 1.0 : -1.0;
            for (int a = 0; a < 2; ++a) {
                double wx = a ? t[0] : 1.0 - t[0], dwx = a ? 1.0 : -1.0;
                double p = G->phi64[((size_t)i[2][c] * ny + i[1][b]) * nx + i[0][a]];
                val += p * wx * wy * wz;
                gx += p * dwx * wy * wz;
                gy += p * wx * dwy * wz;
                gz += p * wx * wy * dwz;
            }
        }
    }
    if (grad) {
        grad[0] = gx / G->h[0];
        grad[1] = gy / G->h[1];
        grad[2] = gz / G->h[2];
    }
    return val;
}

/* ------------------------------------------------------------------------
 * Pair force F_ij = (F^C + F^D + F^R) along e = d/r, d = r_i - r_j
 * (Eq. 3-10 with w_C = w_R = w, w_D = w^2, w = 1 - r/rc, sigma^2 = 2 gamma kBT):
 *   F_ij = [ a_ij w - gamma w^2 (e . (vt_i - vt_j)) + sigma w xi_ij / sqrt(dt) ] e
 * Zero for r >= rc (Eq. 5) and for r = 0.
 * ---------------------------------------------------------------------- */
/* ------------------------------------------------------------------------
 * Smoothing function of Eq. 23 in 3-D (alpha_3 = 1/pi) with support r0:
 * h = r0/2, v = r/h,
 *   W = (1/(pi h^3)) {1 - 3/2 v^2 + 3/4 v^3 (v < 1); 1/4 (2 - v)^3 (v < 2); 0}
 * and its derivative dW/dr.
 * ---------------------------------------------------------------------- */
double orc_sph_w(double r, double r0)
{
    const double h = 0.5 * r0, v = r / h, c = 1.0 / (ORC_PI * h * h * h);
    if (v < 1.0) return c * (1.0 - 1.5 * v * v + 0.75 * v * v * v);
    if (v < 2.0) return c * 0.25 * (2.0 - v) * (2.0 - v) * (2.0 - v);
    return 0.0;
}

double orc_sph_dw(double r, double r0)
{
    const double h = 0.5 * r0, v = r / h, c = 1.0 / (ORC_PI * h * h * h * h);
    if (v < 1.0) return c * (-3.0 * v + 2.25 * v * v);
    if (v < 2.0) return c * (-0.75 * (2.0 - v) * (2.0 - v));
    return 0.0;
}

/* Pair energy of Eq. 22: S^r W(r, r0^r) - S^a W(r, r0^a). */
static double sph_energy(const orc_params *P, double r, int ti, int tj)
{
    return P->sr[ti][tj] * orc_sph_w(r, P->r0r) - P->sa[ti][tj] * orc_sph_w(r, P->r0a);
}

static void pair_force(const orc_params *P, double sigma, double inv_sqrt_dt,
                       const double d[3], const double dv[3], int ti, int tj,
                       uint32_t gi, uint32_t gj, uint64_t k, int noclamp, double out[3])
{
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double w = 1.0 - r / P->rc;
    if (r == 0.0 || (!noclamp && w <= 0.0)) {
        out[0] = out[1] = out[2] = 0.0;
        return;
    }
    double e[3] = {d[0] / r, d[1] / r, d[2] / r};
    double edv = e[0] * dv[0] + e[1] * dv[1] + e[2] * dv[2];
    double xi = orc_xi(P->seed, gi, gj, k, P->replica);
    /* conservative part: a w (Eq. 4), or -dE/dr of Eq. 22 (Eq. 24) */
    double fc = P->a[ti][tj] * w;
    if (P->sph)
        fc = -(P->sr[ti][tj] * orc_sph_dw(r, P->r0r) - P->sa[ti][tj] * orc_sph_dw(r, P->r0a));
    double mag = fc - P->gamma * w * w * edv + sigma * w * xi * inv_sqrt_dt;
    out[0] = mag * e[0];
    out[1] = mag * e[1];
    out[2] = mag * e[2];
}

/* Cells of the FP32 shadow positions and a per-cell member list in particle
 * index order (plain counting sort). */
typedef struct {
    int32_t *cell;    /* n */
    int32_t *start;   /* ncell + 1 */
    int32_t *list;    /* n */
} orc_cells;

static int build_cells(const orc_geom *G, int64_t n, const float *xs, orc_cells *C)
{
    int64_t ncell = (int64_t)G->nc[0] * G->nc[1] * G->nc[2];
    C->cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    C->start = (int32_t *)calloc((size_t)ncell + 1, sizeof(int32_t));
    C->list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *fill = (int32_t *)calloc((size_t)ncell, sizeof(int32_t));
    if (!C->cell || !C->start || !C->list || !fill) return -1;
    for (int64_t p = 0; p < n; ++p) {
        C->cell[p] = orc_cell_of(G, xs + 3 * p);
        C->start[C->cell[p] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) C->start[c + 1] += C->start[c];
    for (int64_t p = 0; p < n; ++p) {
        int32_t c = C->cell[p];
        C->list[C->start[c] + fill[c]++] = (int32_t)p;
    }
    free(fill);
    return 0;
}

static void free_cells(orc_cells *C)
{
    free(C->cell); free(C->start); free(C->list);
}

/* Separation of one FP32 coordinate pair along an axis for image shift s of
 * j (-1, 0, +1): the FP32 rounding of the exact minimum-image difference
 * x_i - x_j - s L.  The coordinate that lies in the last cell (x_i for
 * s = +1, x_j for s = -1) is first lowered by L, which is exact because it
 * lies in [L/2, L) (Sterbenz), so the one subtraction that follows is the
 * only rounding. */
static float sep32(float xi, float xj, int s, float L)
{
    float a = s > 0 ? xi - L : xi;
    float b = s < 0 ? xj - L : xj;
    return a - b;
}

/* FP32 pair decision on shadow positions: with j seen from i's neighbour
 * cell at image shift s (per axis -1, 0, +1), d = sep32 per axis,
 *   r2 = fma(dz, dz, fma(dy, dy, fl(dx^2)))
 * (each fma rounded once), and the pair is in range iff r2 < fl32(rc^2). */
static int pair_in_range32(const orc_geom *G, const float *xi, const float *xj,
                           const int s[3], float rc2)
{
    float dx = sep32(xi[0], xj[0], s[0], G->L32[0]);
    float dy = sep32(xi[1], xj[1], s[1], G->L32[1]);
    float dz = sep32(xi[2], xj[2], s[2], G->L32[2]);
    float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    return r2 < rc2;
}

/* Image shift of neighbour cell coordinate c + o, o in {-1, 0, 1}. */
static int cell_shift(int c, int o, int n, int *wrapped)
{
    int q = c + o;
    if (q < 0) { *wrapped = q + n; return -1; }
    if (q >= n) { *wrapped = q - n; return 1; }
    *wrapped = q;
    return 0;
}

/*
 * Forces at the current state (Eq. 2: f_i = sum_{j != i, r_ij < rc} F_ij,
 * plus the body force g on fluid particles).
 *   mode 0: brute force O(N^2), minimum image, FP64 cutoff test r < rc
 *   mode 1: brute force O(N^2), FP32 decision with the cell-derived image
 *   mode 2: cell list (27 neighbour cells), FP32 decision
 * Modes 1 and 2 visit exactly the same pairs.  Wall particles are frozen,
 * so wall-wall pairs are skipped; with all_particles = 0 only fluid forces
 * are computed (wall rows left zero), with 1 walls get their forces too.
 */
static int forces_impl(const orc_geom *G, const orc_params *P, int64_t n,
                       const double *r, const double *vt, const float *xs,
                       const int32_t *type, const uint32_t *gid, uint64_t k,
                       int mode, int all_particles, int noclamp, double *f)
{
    const double sigma = sqrt(2.0 * P->gamma * P->kBT);
    const double inv_sqrt_dt = 1.0 / sqrt(P->dt);
    const float rc2 = (float)(P->rc * P->rc);
    orc_cells C;
    memset(&C, 0, sizeof C);
    if (mode != 0 && build_cells(G, n, xs, &C) != 0) return -1;
    const int64_t ncx = G->nc[0], ncy = G->nc[1];

    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        if (type[i] != 0 && !all_particles) {
            f[3 * i] = f[3 * i + 1] = f[3 * i + 2] = 0.0;
            continue;
        }
        if (mode == 2) {
            int cx = (int)(C.cell[i] % ncx);
            int cy = (int)((C.cell[i] / ncx) % ncy);
            int cz = (int)(C.cell[i] / (ncx * ncy));
            for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                int wx, wy, wz, s[3];
                s[0] = cell_shift(cx, ox, G->nc[0], &wx);
                s[1] = cell_shift(cy, oy, G->nc[1], &wy);
                s[2] = cell_shift(cz, oz, G->nc[2], &wz);
                int64_t c = ((int64_t)wz * ncy + wy) * ncx + wx;
                for (int32_t q = C.start[c]; q < C.start[c + 1]; ++q) {
                    int64_t j = C.list[q];
                    if (j == i || (type[i] != 0 && type[j] != 0)) continue;
                    if (!pair_in_range32(G, xs + 3 * i, xs + 3 * j, s, rc2)) continue;
                    double d[3], dv[3], F[3];
                    for (int a = 0; a < 3; ++a) {
                        d[a] = r[3 * i + a] - (r[3 * j + a] + s[a] * G->L[a]);
                        dv[a] = vt[3 * i + a] - vt[3 * j + a];
                    }
                    pair_force(P, sigma, inv_sqrt_dt, d, dv, type[i], type[j],
                               gid[i], gid[j], k, noclamp, F);
                    acc[0] += F[0]; acc[1] += F[1]; acc[2] += F[2];
                }
            }
        } else {
            for (int64_t j = 0; j < n; ++j) {
                if (j == i || (type[i] != 0 && type[j] != 0)) continue;
                double d[3], dv[3], F[3];
                if (mode == 0) {
                    for (int a = 0; a < 3; ++a) {
                        double dd = r[3 * i + a] - r[3 * j + a];
                        d[a] = dd - G->L[a] * nearbyint(dd / G->L[a]);
                    }
                    if (sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) >= P->rc) continue;
                } else {
                    /* the image follows from the two particles' cells */
                    int s[3], ok = 1;
                    int ci = C.cell[i], cj = C.cell[j];
                    int cc_i[3] = {(int)(ci % ncx), (int)((ci / ncx) % ncy), (int)(ci / (ncx * ncy))};
                    int cc_j[3] = {(int)(cj % ncx), (int)((cj / ncx) % ncy), (int)(cj / (ncx * ncy))};
                    for (int a = 0; a < 3 && ok; ++a) {
                        int found = 0;
                        for (int o = -1; o <= 1; ++o) {
                            int wq, sh = cell_shift(cc_i[a], o, G->nc[a], &wq);
                            if (wq == cc_j[a]) { s[a] = sh; found = 1; break; }
                        }
                        ok = found;
                    }
                    if (!ok || !pair_in_range32(G, xs + 3 * i, xs + 3 * j, s, rc2)) continue;
                    for (int a = 0; a < 3; ++a)
                        d[a] = r[3 * i + a] - (r[3 * j + a] + s[a] * G->L[a]);
                }
                for (int a = 0; a < 3; ++a) dv[a] = vt[3 * i + a] - vt[3 * j + a];
                pair_force(P, sigma, inv_sqrt_dt, d, dv, type[i], type[j],
                           gid[i], gid[j], k, 0, F);
                acc[0] += F[0]; acc[1] += F[1]; acc[2] += F[2];
            }
        }
        if (type[i] == 0) {
            acc[0] += P->g[0]; acc[1] += P->g[1]; acc[2] += P->g[2];
        }
        f[3 * i] = acc[0]; f[3 * i + 1] = acc[1]; f[3 * i + 2] = acc[2];
    }
    if (mode != 0) free_cells(&C);
    return 0;
}

int orc_forces(const orc_geom *G, const orc_params *P, int64_t n,
               const double *r, const double *vt, const float *xs,
               const int32_t *type, const uint32_t *gid, uint64_t k,
               int mode, int all_particles, double *f)
{
    return forces_impl(G, P, n, r, vt, xs, type, gid, k, mode, all_particles, 0, f);
}

/* Cells of the shadow positions (decision form). */
void orc_cells_of(const orc_geom *G, int64_t n, const float *xs, int32_t *cell)
{
    for (int64_t p = 0; p < n; ++p) cell[p] = orc_cell_of(G, xs + 3 * p);
}

/* Interacting pairs (gid_i, gid_j) seen from every fluid i, FP32 decision
 * on the shadow positions through the 27 neighbour cells.  Fluid-fluid
 * pairs appear in both orders, fluid-wall pairs once.  Returns the count
 * (pairs beyond cap are counted, not written), or -1. */
int64_t orc_pairs(const orc_geom *G, const orc_params *P, int64_t n,
                  const float *xs, const int32_t *type, const uint32_t *gid,
                  uint32_t *out, int64_t cap)
{
    const float rc2 = (float)(P->rc * P->rc);
    orc_cells C;
    if (build_cells(G, n, xs, &C) != 0) return -1;
    const int64_t ncx = G->nc[0], ncy = G->nc[1];
    int64_t count = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] != 0) continue;
        int cx = (int)(C.cell[i] % ncx);
        int cy = (int)((C.cell[i] / ncx) % ncy);
        int cz = (int)(C.cell[i] / (ncx * ncy));
        for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
            int wx, wy, wz, s[3];
            s[0] = cell_shift(cx, ox, G->nc[0], &wx);
            s[1] = cell_shift(cy, oy, G->nc[1], &wy);
            s[2] = cell_shift(cz, oz, G->nc[2], &wz);
            int64_t c = ((int64_t)wz * ncy + wy) * ncx + wx;
            for (int32_t q = C.start[c]; q < C.start[c + 1]; ++q) {
                int64_t j = C.list[q];
                if (j == i) continue;
                if (!pair_in_range32(G, xs + 3 * i, xs + 3 * j, s, rc2)) continue;
                if (count < cap) {
                    out[2 * count] = gid[i];
                    out[2 * count + 1] = gid[j];
                }
                ++count;
            }
        }
    }
    free_cells(&C);
    return count;
}

/* Decision form of the drift: w = fl(v + fl(dt/2 * f)), x* = fl(x + fl(dt * w)),
 * then a single-box wrap.  Returns per-axis image shifts in s. */
static void drift32(const orc_geom *G, const orc_params *P, const float x[3],
                    const float v[3], const float f[3], float out[3], int s[3])
{
    const float hdt = (float)(0.5 * P->dt);
    const float dt = (float)P->dt;
    for (int a = 0; a < 3; ++a) {
        float w = v[a] + hdt * f[a];
        float y = x[a] + dt * w;
        s[a] = wrap32(&y, G->L32[a]);
        out[a] = y;
    }
}

/* Velocity of the solid at a reflection at r* (FP32 shadow y32): that of the
 * wall particle nearest to r* among the walls (at their start-of-step
 * positions xs) in the 27-cell neighbourhood of the cell of y32, nearness by
 * the FP32 pair-decision r2 (image shift of the neighbour cell), ties to the
 * smaller gid; no wall there: zero.  Brute force over all walls. */
static void wall_velocity(const orc_geom *G, int64_t n, const double *v, const float *xs,
                          const int32_t *type, const uint32_t *gid, const float y32[3],
                          double out[3])
{
    const int nx = G->nc[0], ny = G->nc[1], nz = G->nc[2];
    const int ncs[3] = {nx, ny, nz};
    const int32_t c = orc_cell_of(G, y32);
    const int cc[3] = {c % nx, (c / nx) % ny, c / (nx * ny)};
    float best = INFINITY;
    uint32_t best_gid = 0;
    int64_t best_j = -1;
    for (int64_t j = 0; j < n; ++j) {
        if (type[j] == 0) continue;
        int32_t wc = orc_cell_of(G, xs + 3 * j);
        const int wcc[3] = {wc % nx, (wc / nx) % ny, wc / (nx * ny)};
        int near = 1, sh[3];
        for (int a = 0; a < 3; ++a) {
            /* neighbour offset o in {-1, 0, 1} with q = cc + o wrapped; the
             * image shift is -1 below 0 and +1 past the last cell */
            int o = wcc[a] - cc[a];
            if (o == ncs[a] - 1) o = -1;
            else if (o == -(ncs[a] - 1)) o = 1;
            if (o < -1 || o > 1) { near = 0; break; }
            int q = cc[a] + o;
            sh[a] = q < 0 ? -1 : (q >= ncs[a] ? 1 : 0);
        }
        if (!near) continue;
        float ax = y32[0] - (float)sh[0] * G->L32[0];
        float ay = y32[1] - (float)sh[1] * G->L32[1];
        float az = y32[2] - (float)sh[2] * G->L32[2];
        float dx = ax - xs[3 * j], dy = ay - xs[3 * j + 1], dz = az - xs[3 * j + 2];
        float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        if (r2 < best || (r2 == best && gid[j] < best_gid)) {
            best = r2;
            best_gid = gid[j];
            best_j = j;
        }
    }
    for (int a = 0; a < 3; ++a) out[a] = best_j >= 0 ? v[3 * best_j + a] : 0.0;
}

/*
 * One step of the method for every fluid particle (walls frozen):
 *   1. r* = r + dt v + dt^2/2 f,  vt = v + lambda dt f   (Groot-Warren)
 *   2. if phi(r*) < 0: reflect (Sec. II.C, Eq. 16-17):
 *        c1 = atanh(-phi*), c0 = atanh(phi^t),  s = c1 / (c0 + c1)
 *        u = v^t - v_wall (bounce-back) or ((v^t - v_wall) . n) n (specular)
 *        r_bb = r* - 2 s dt u;  if phi(r_bb) < 0 then r_bb = r^t (code 2)
 *        r = r_bb,  v = v^t - 2 u,  vt = v  (code 1 or 2)
 *      (resting walls, bounce-back: u = v^t, v = -v^t)
 *   3. k += 1;  f' = forces(r, vt) with the random numbers of evaluation k
 *   4. non-bounced particles: v = v + dt/2 (f + f');  f = f'
 * Positions r, v, f are FP64 arrays of n*3; xs receives the FP32 shadow
 * positions on which the discrete decisions were taken (x* for particles that
 * did not bounce, fl32(r_bb) for those that did); events receives 0/1/2
 * per particle.  The periodic wrap of r* follows the FP32 decision so that
 * FP64 positions and shadows always name the same image.
 */
int orc_step(const orc_geom *G, const orc_params *P, int64_t n, double *r,
             double *v, double *f, const int32_t *type, const uint32_t *gid,
             uint64_t *k, int32_t *events, float *xs, int mode, double *scratch_vt)
{
    const double dt = P->dt;
    const double delta = 0x1p-20;
    double *vt = scratch_vt;
    double *vold = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *fnew = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!vold || !fnew) { free(vold); free(fnew); return -1; }

    int moving = 0;
    for (int64_t i = 0; i < n; ++i)
        if (type[i] != 0 && (v[3 * i] != 0.0 || v[3 * i + 1] != 0.0 || v[3 * i + 2] != 0.0))
            moving = 1;

    for (int64_t i = 0; i < n; ++i) {
        events[i] = 0;
        for (int a = 0; a < 3; ++a) vold[3 * i + a] = v[3 * i + a];
        if (type[i] != 0) {
            /* a wall particle's velocity is its solid's (moved below) */
            for (int a = 0; a < 3; ++a) vt[3 * i + a] = v[3 * i + a];
            continue;
        }
        float x32[3], v32[3], f32[3], y32[3];
        int s[3];
        for (int a = 0; a < 3; ++a) {
            x32[a] = (float)r[3 * i + a];
            v32[a] = (float)v[3 * i + a];
            f32[a] = (float)f[3 * i + a];
        }
        drift32(G, P, x32, v32, f32, y32, s);
        double rs[3];
        for (int a = 0; a < 3; ++a) {
            rs[a] = r[3 * i + a] + dt * v[3 * i + a] + 0.5 * dt * dt * f[3 * i + a]
                    + s[a] * G->L[a];
            vt[3 * i + a] = v[3 * i + a] + P->lambda * dt * f[3 * i + a];
        }
        if (!phi_negative(G, y32)) {
            for (int a = 0; a < 3; ++a) {
                r[3 * i + a] = rs[a];
                xs[3 * i + a] = y32[a];
            }
            continue;
        }
        /* bounce-back, Eq. 16-17 */
        double rt[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
        double phis = orc_phi64(G, rs, NULL);
        double phit = orc_phi64(G, rt, NULL);
        double a1 = -phis, a0 = phit;
        if (a1 < 0.0) a1 = 0.0;
        if (a1 > 1.0 - delta) a1 = 1.0 - delta;
        if (a0 < 0.0) a0 = 0.0;
        if (a0 > 1.0 - delta) a0 = 1.0 - delta;
        double c1 = atanh(a1), c0 = atanh(a0);
        double sfrac = (c1 > 0.0) ? c1 / (c0 + c1) : 0.0;
        /* the reversed part u of the velocity relative to the wall */
        double vw[3] = {0.0, 0.0, 0.0}, u[3];
        if (moving) wall_velocity(G, n, v, xs, type, gid, y32, vw);
        for (int a = 0; a < 3; ++a) u[a] = v[3 * i + a] - vw[a];
        if (P->specular) {
            double gr[3];
            orc_phi64(G, rs, gr);
            double gn = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
            if (gn > 0.0) {
                double nrm[3] = {gr[0] / gn, gr[1] / gn, gr[2] / gn};
                double un = u[0] * nrm[0] + u[1] * nrm[1] + u[2] * nrm[2];
                for (int a = 0; a < 3; ++a) u[a] = un * nrm[a];
            }
        }
        double rbb[3];
        float bb32[3];
        for (int a = 0; a < 3; ++a) rbb[a] = rs[a] - 2.0 * sfrac * dt * u[a];
        for (int a = 0; a < 3; ++a) {
            bb32[a] = (float)rbb[a];
            int sh = wrap32(&bb32[a], G->L32[a]);
            rbb[a] += sh * G->L[a];
        }
        int code = 1;
        if (phi_negative(G, bb32)) {
            code = 2;
            for (int a = 0; a < 3; ++a) {
                rbb[a] = rt[a];
                bb32[a] = (float)rt[a];
            }
        }
        events[i] = code;
        for (int a = 0; a < 3; ++a) {
            r[3 * i + a] = rbb[a];
            xs[3 * i + a] = bb32[a];
            v[3 * i + a] = v[3 * i + a] - 2.0 * u[a];
            vt[3 * i + a] = v[3 * i + a];
        }
    }

    /* walls translate with their solid: r_w += dt v_w, decided in FP32 as
     * the fluid drift with zero force */
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] == 0) continue;
        float x32[3], v32[3], z32[3] = {0.0f, 0.0f, 0.0f}, y32[3];
        int s[3];
        for (int a = 0; a < 3; ++a) {
            x32[a] = (float)r[3 * i + a];
            v32[a] = (float)v[3 * i + a];
        }
        drift32(G, P, x32, v32, z32, y32, s);
        for (int a = 0; a < 3; ++a) {
            r[3 * i + a] += dt * v[3 * i + a] + s[a] * G->L[a];
            xs[3 * i + a] = y32[a];
        }
    }

    *k += 1;
    int rc = orc_forces(G, P, n, r, vt, xs, type, gid, *k, mode, 0, fnew);
    if (rc == 0) {
        for (int64_t i = 0; i < n; ++i) {
            if (type[i] != 0) continue;
            for (int a = 0; a < 3; ++a) {
                if (events[i] == 0)
                    v[3 * i + a] = vold[3 * i + a] + 0.5 * dt * (f[3 * i + a] + fnew[3 * i + a]);
                f[3 * i + a] = fnew[3 * i + a];
            }
        }
    }
    free(vold);
    free(fnew);
    return rc;
}

/* Conservative potential energy sum_{pairs} a_ij rc/2 (1 - r/rc)^2 (the
 * potential of Eq. 4-5), or the energy of Eq. 22, brute force with minimum
 * image; wall-wall pairs excluded (they are frozen and never interact). */
double orc_potential(const orc_geom *G, const orc_params *P, int64_t n,
                     const double *r, const int32_t *type)
{
    double U = 0.0;
    #pragma omp parallel for reduction(+:U) schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            if (type[i] != 0 && type[j] != 0) continue;
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double dd = r[3 * i + a] - r[3 * j + a];
                dd -= G->L[a] * nearbyint(dd / G->L[a]);
                d2 += dd * dd;
            }
            double rr = sqrt(d2);
            if (rr < P->rc) {
                if (P->sph) {
                    U += sph_energy(P, rr, type[i], type[j]);
                } else {
                    double w = 1.0 - rr / P->rc;
                    U += 0.5 * P->a[type[i]][type[j]] * P->rc * w * w;
                }
            }
        }
    }
    return U;
}

/* Binned fluid observables along one axis (Sec. III.A: density, temperature
 * and stream velocity per bin): count, sum v_x, sum |v|^2 per bin. */
void orc_profile(const orc_geom *G, int64_t n, const double *r, const double *v,
                 const int32_t *type, int axis, int nbins, double *count,
                 double *sum_vx, double *sum_v2, double *sum_v)
{
    for (int b = 0; b < nbins; ++b) {
        count[b] = sum_vx[b] = sum_v2[b] = 0.0;
        if (sum_v) sum_v[3 * b] = sum_v[3 * b + 1] = sum_v[3 * b + 2] = 0.0;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] != 0) continue;
        double x = r[3 * i + axis];
        x -= G->L[axis] * floor(x / G->L[axis]);
        int b = (int)floor(x / G->L[axis] * nbins);
        if (b < 0) b = 0;
        if (b >= nbins) b = nbins - 1;
        count[b] += 1.0;
        sum_vx[b] += v[3 * i];
        sum_v2[b] += v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2];
        if (sum_v) {
            sum_v[3 * b] += v[3 * i];
            sum_v[3 * b + 1] += v[3 * i + 1];
            sum_v[3 * b + 2] += v[3 * i + 2];
        }
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Window of T steps for the gradient checks of the adjoint form.
 *
 * The step of orc_step iterated from (r0, v0) at force index k0, with the
 * carried force refreshed first, f0 = F(r0, v0; k0) + g (pairs decided at
 * fl32(r0)), and the binned profile of v_x over the states after steps
 * 1..T: sums[b] = sum over steps t and fluid particles i in bin b after
 * step t of v_x,i, counts[b] the number of terms.  The bin of a particle is
 * the FP32 decision b = clamp(floor(fl(x_axis * fl32(nbins / L_axis))),
 * 0, nbins - 1) on its FP32 decision position.
 *
 * record = 1: every discrete decision (bounce-back event and its code, the
 * pair set of each force evaluation, the bins) is taken as in orc_step and
 * logged: ev[t n + i], xs_log[3 (t n + i) + a] (the FP32 positions on which
 * step t's pair set and bins are decided) and bin[t n + i].
 * record = 0: the same steps with every decision replayed from the logs, so
 * the profile is a smooth function of a_ij, gamma, g and the phi values
 * near the events (the frozen-event form whose derivative the adjoint
 * computes).  The FP64 positions are kept in the periodic image of the
 * logged decision positions.
 * Pair forces of a decided pair use w = 1 - r/rc without clamping at rc in
 * both modes (replay stays differentiable; record mode differs from
 * orc_step only for pairs within rounding of the cutoff).
 * r_out, v_out (n x 3, may be NULL) receive the final state.  Returns 0, or
 * -1 when an allocation fails.
 * ---------------------------------------------------------------------- */
static int bin_of32(float x, float scale, int nbins)
{
    int b = (int)floorf(x * scale);
    if (b < 0) b = 0;
    if (b >= nbins) b = nbins - 1;
    return b;
}

/* Scratch arrays of one window step (n x 3 doubles, n x 3 floats, n ints). */
typedef struct {
    double *fn, *vt, *vold;
    float *xs;
    int32_t *code;
} win_scratch;

static int win_scratch_alloc(win_scratch *S, int64_t n)
{
    const size_t n3 = 3 * (size_t)(n > 0 ? n : 1);
    S->fn = malloc(sizeof(double) * n3);
    S->vt = malloc(sizeof(double) * n3);
    S->vold = malloc(sizeof(double) * n3);
    S->xs = malloc(sizeof(float) * n3);
    S->code = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    return (S->fn && S->vt && S->vold && S->xs && S->code) ? 0 : -1;
}

static void win_scratch_free(win_scratch *S)
{
    free(S->fn); free(S->vt); free(S->vold); free(S->xs); free(S->code);
}

/* Step t of the window from the state (r, v, f), updated in place: drift
 * and prediction, bounce-back (Eq. 16-17) with the decision taken
 * (record = 1) or read from ev_t (record = 0), the forces at force index k
 * on the pair set decided at the FP32 positions (taken, or read from
 * xs_t), the velocity update, and the step's bin sums added to sums and
 * counts (bins taken, or read from bin_t).  record = 1 writes the step's
 * decisions to ev_t, xs_t and bin_t. */
static int window_step(const orc_geom *G, const orc_params *P, int64_t n, double *r,
                       double *v, double *f, const int32_t *type, const uint32_t *gid,
                       uint64_t k, int axis, int nbins, int record, int32_t *ev_t,
                       float *xs_t, int32_t *bin_t, double *sums, double *counts,
                       win_scratch *S)
{
    const double dt = P->dt;
    const double delta = 0x1p-20;
    const float scale = (float)((double)nbins / G->L[axis]);
    double *fn = S->fn, *vt = S->vt, *vold = S->vold;
    float *xs = S->xs;
    int32_t *code = S->code;
    for (int64_t i = 0; i < n; ++i) {
        double *ri = r + 3 * i, *vi = v + 3 * i, *fi = f + 3 * i;
        for (int a = 0; a < 3; ++a) vold[3 * i + a] = vi[a];
        code[i] = 0;
        if (type[i] != 0) {
            for (int a = 0; a < 3; ++a) {
                vt[3 * i + a] = 0.0;
                xs[3 * i + a] = (float)ri[a];
            }
            continue;
        }
        /* drift and prediction (Groot-Warren) */
        float x32[3], v32[3], f32[3], y32[3];
        int sh[3];
        for (int a = 0; a < 3; ++a) {
            x32[a] = (float)ri[a];
            v32[a] = (float)vi[a];
            f32[a] = (float)fi[a];
        }
        drift32(G, P, x32, v32, f32, y32, sh);
        double rs[3], rt[3];
        for (int a = 0; a < 3; ++a) {
            rt[a] = ri[a];
            rs[a] = ri[a] + dt * vi[a] + 0.5 * dt * dt * fi[a] + sh[a] * G->L[a];
            vt[3 * i + a] = vi[a] + P->lambda * dt * fi[a];
        }
        int c = record ? (phi_negative(G, y32) ? 1 : 0) : ev_t[i];
        float d32[3] = {y32[0], y32[1], y32[2]};
        if (c == 0) {
            for (int a = 0; a < 3; ++a) ri[a] = rs[a];
        } else {
            /* bounce-back, Eq. 16-17 */
            double a1 = -orc_phi64(G, rs, NULL), a0 = orc_phi64(G, rt, NULL);
            if (a1 < 0.0) a1 = 0.0;
            if (a1 > 1.0 - delta) a1 = 1.0 - delta;
            if (a0 < 0.0) a0 = 0.0;
            if (a0 > 1.0 - delta) a0 = 1.0 - delta;
            double c1 = atanh(a1), c0 = atanh(a0);
            double sfrac = c1 > 0.0 ? c1 / (c0 + c1) : 0.0;
            double rbb[3];
            for (int a = 0; a < 3; ++a) {
                rbb[a] = rs[a] - 2.0 * sfrac * dt * vi[a];
                d32[a] = (float)rbb[a];
                rbb[a] += wrap32(&d32[a], G->L32[a]) * G->L[a];
            }
            if (record) c = phi_negative(G, d32) ? 2 : 1;
            for (int a = 0; a < 3; ++a) {
                ri[a] = c == 2 ? rt[a] : rbb[a];
                if (c == 2) d32[a] = (float)rt[a];
                vt[3 * i + a] = -vi[a];
                vi[a] = -vi[a];
            }
        }
        code[i] = c;
        for (int a = 0; a < 3; ++a) xs[3 * i + a] = d32[a];
    }
    if (record) {
        for (int64_t i = 0; i < n; ++i) {
            ev_t[i] = code[i];
            for (int a = 0; a < 3; ++a) xs_t[3 * i + a] = xs[3 * i + a];
        }
    } else {
        /* decisions from the log; positions in the logged image */
        for (int64_t q = 0; q < 3 * n; ++q) {
            const int a = (int)(q % 3);
            xs[q] = xs_t[q];
            r[q] -= G->L[a] * nearbyint((r[q] - (double)xs_t[q]) / G->L[a]);
        }
    }
    if (forces_impl(G, P, n, r, vt, xs, type, gid, k, 2, 0, 1, fn) != 0) return -1;
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] != 0) continue;
        for (int a = 0; a < 3; ++a) {
            if (code[i] == 0)
                v[3 * i + a] = vold[3 * i + a] + 0.5 * dt * (f[3 * i + a] + fn[3 * i + a]);
            f[3 * i + a] = fn[3 * i + a];
        }
        int b;
        if (record) {
            b = bin_of32(xs[3 * i + axis], scale, nbins);
            bin_t[i] = b;
        } else {
            b = bin_t[i];
        }
        sums[b] += v[3 * i];
        counts[b] += 1.0;
    }
    return 0;
}

int orc_window(const orc_geom *G, const orc_params *P, int64_t n,
               const double *r0, const double *v0, const int32_t *type,
               const uint32_t *gid, uint64_t k0, int T, int axis, int nbins,
               int record, int32_t *ev, float *xs_log, int32_t *bin,
               double *sums, double *counts, double *r_out, double *v_out)
{
    const size_t n3 = 3 * (size_t)(n > 0 ? n : 1);
    double *r = malloc(sizeof(double) * n3), *v = malloc(sizeof(double) * n3);
    double *f = malloc(sizeof(double) * n3);
    win_scratch S;
    int rc = -1;
    int ok = win_scratch_alloc(&S, n) == 0;
    if (!r || !v || !f || !ok) goto out;
    for (int b = 0; b < nbins; ++b) sums[b] = counts[b] = 0.0;
    for (int64_t q = 0; q < 3 * n; ++q) {
        r[q] = r0[q];
        v[q] = type[q / 3] == 0 ? v0[q] : 0.0;
        S.xs[q] = (float)r0[q];
    }
    if (forces_impl(G, P, n, r, v, S.xs, type, gid, k0, 2, 0, 1, f) != 0) goto out;
    for (int t = 0; t < T; ++t) {
        if (window_step(G, P, n, r, v, f, type, gid, k0 + (uint64_t)t + 1, axis, nbins, record,
                        ev + (size_t)t * n, xs_log + 3 * (size_t)t * (size_t)n,
                        bin + (size_t)t * n, sums, counts, &S) != 0)
            goto out;
    }
    if (r_out) memcpy(r_out, r, sizeof(double) * 3 * (size_t)n);
    if (v_out) memcpy(v_out, v, sizeof(double) * 3 * (size_t)n);
    rc = 0;
out:
    free(r); free(v); free(f);
    win_scratch_free(&S);
    return rc;
}

/* The window's starting force f0 = F(r0, v0; k0) + g (pairs decided at
 * fl32(r0), w = 1 - r/rc without clamping), as orc_window computes it. */
int orc_window_start_force(const orc_geom *G, const orc_params *P, int64_t n,
                           const double *r0, const double *v0, const int32_t *type,
                           const uint32_t *gid, uint64_t k0, double *f)
{
    const size_t n3 = 3 * (size_t)(n > 0 ? n : 1);
    float *xs = malloc(sizeof(float) * n3);
    double *v = malloc(sizeof(double) * n3);
    if (!xs || !v) { free(xs); free(v); return -1; }
    for (int64_t q = 0; q < 3 * n; ++q) {
        xs[q] = (float)r0[q];
        v[q] = type[q / 3] == 0 ? v0[q] : 0.0;
    }
    int rc = forces_impl(G, P, n, r0, v, xs, type, gid, k0, 2, 0, 1, f);
    free(xs); free(v);
    return rc;
}

/* One step of the window with every decision read from the logs of that
 * step (ev_t, xs_t, bin_t), from the state (r, v, f) updated in place, the
 * new force at force index k; the step's bin sums go to sums and counts
 * (nbins each, overwritten).  The replayed window is this step iterated
 * from f0 of orc_window_start_force with k = k0 + t + 1, so that the window
 * can be linearised step by step around any trajectory. */
int orc_window_step(const orc_geom *G, const orc_params *P, int64_t n, double *r, double *v,
                    double *f, const int32_t *type, const uint32_t *gid, uint64_t k,
                    int axis, int nbins, const int32_t *ev_t, const float *xs_t,
                    const int32_t *bin_t, double *sums, double *counts)
{
    win_scratch S;
    int rc = -1;
    if (win_scratch_alloc(&S, n) == 0) {
        for (int b = 0; b < nbins; ++b) sums[b] = counts[b] = 0.0;
        rc = window_step(G, P, n, r, v, f, type, gid, k, axis, nbins, 0, (int32_t *)ev_t,
                         (float *)xs_t, (int32_t *)bin_t, sums, counts, &S);
    }
    win_scratch_free(&S);
    return rc;
}
