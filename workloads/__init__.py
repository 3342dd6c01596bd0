"""Seeded synthetic inputs for the DPD step with phase-field no-slip walls.

This module builds what a simulation starts from: the periodic box, the
signed distance to the solid, the phase-field grid phi = tanh(d / width) of
the equilibrium profile (Sec. II.B, Eq. 14, with sqrt(2)*eps = width), fluid
particles where phi > 0 and frozen wall particles where phi < 0 (Sec. II.C),
Maxwell velocities, and the DPD parameters of each workload.

It holds none of the time step's arithmetic: no pair forces, no random
numbers of the force, no integration, no interpolation of phi at a particle
and no reflection.  Particles are classified against the grid by the minimum
and maximum of the 8 grid nodes around them, which is a conservative test,
not the method's interpolation.  Both the oracle-based tests and the GPU path
take their inputs from here, so the two never share arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "System", "slab_system", "couette_system", "sph_force", "sinusoid_cylinder_system", "porous_system",
    "sinusoid_slit_system", "replica_systems", "tiny_slab_system",
    "corner_minmax", "maxwell_velocities", "bulk_system",
]


@dataclass
class System:
    """One periodic box of fluid + frozen wall particles and its phase field.

    pos, vel: (N, 3) float32; type: (N,) int32 (0 fluid, 1 wall);
    gid: (N,) uint32, a permutation of 0..N-1;
    phi: (nz, ny, nx) grid of node values, node (i, j, k) at (i*h, j*h, k*h);
    params: a (2x2 list: fluid-fluid, fluid-wall), gamma, kBT, rc, dt, lam,
    g (3,), seed, replica.
    """
    name: str
    L: np.ndarray
    pos: np.ndarray
    vel: np.ndarray
    type: np.ndarray
    gid: np.ndarray
    phi: np.ndarray
    h: np.ndarray
    params: dict
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_fluid(self) -> int:
        return int(np.count_nonzero(self.type == 0))

    @property
    def n_wall(self) -> int:
        return int(np.count_nonzero(self.type == 1))


def default_params(a_ff=25.0, a_fs=25.0, gamma=4.5, kBT=1.0, rc=1.0, dt=0.01,
                   lam=0.65, g=(0.0, 0.0, 0.0), seed=1234, replica=0) -> dict:
    return dict(a=[[float(a_ff), float(a_fs)], [float(a_fs), float(a_fs)]],
                gamma=float(gamma), kBT=float(kBT), rc=float(rc), dt=float(dt),
                lam=float(lam), g=[float(x) for x in g], seed=int(seed),
                replica=int(replica))


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def sph_force(s_ff_r=37.5, s_ff_a=18.75, fs_factor=2.0, r0r=0.73, r0a=1.0):
    """Parameters of the attractive-repulsive conservative force of Eq. 22-24
    (Sec. III.C's values: S^r_ff = 37.5, S^a_ff = 18.75, ranges 0.73 and 1.0,
    fluid-solid strengths `fs_factor` times the fluid-fluid ones), for
    params["sph"]."""
    sr = [[s_ff_r, fs_factor * s_ff_r], [fs_factor * s_ff_r, fs_factor * s_ff_r]]
    sa = [[s_ff_a, fs_factor * s_ff_a], [fs_factor * s_ff_a, fs_factor * s_ff_a]]
    return dict(sr=sr, sa=sa, r0r=float(r0r), r0a=float(r0a))


def _periodic_abs(x, period):
    x = np.mod(x, period)
    return np.minimum(x, period - x)


def _slab_distance(z, lo, hi, Lz):
    """Signed distance to a fluid slab lo < z < hi in a box periodic in z."""
    z = np.mod(z, Lz)
    dist = np.minimum(_periodic_abs(z - lo, Lz), _periodic_abs(z - hi, Lz))
    inside = (z > lo) & (z < hi)
    return np.where(inside, dist, -dist)


def _sinusoid_distance(x, z, base, amp, period, iters=30):
    """Unsigned distance from (x, z) to the curve z = base + amp*sin(2 pi x/period).

    The nearest curve point is found by Newton's method on the squared
    distance, started from the vertical projection; the curve's radius of
    curvature (>= period^2 / (4 pi^2 |amp|)) is large against the distances
    that matter here (phi = tanh(d/0.5) saturates beyond |d| ~ 5).
    """
    k = 2.0 * math.pi / period
    x0 = np.asarray(x, dtype=np.float64)
    z0 = np.asarray(z, dtype=np.float64)
    t = x0.copy()
    for _ in range(iters):
        zc = base + amp * np.sin(k * t)
        dz = amp * k * np.cos(k * t)
        ddz = -amp * k * k * np.sin(k * t)
        gfun = (t - x0) + (zc - z0) * dz
        gpr = 1.0 + dz * dz + (zc - z0) * ddz
        gpr = np.where(gpr > 0.1, gpr, 0.1)
        t = t - gfun / gpr
    zc = base + amp * np.sin(k * t)
    return np.hypot(t - x0, zc - z0)


def _grid_nodes(L, h):
    n = np.rint(np.asarray(L) / np.asarray(h)).astype(np.int64)
    if not np.allclose(n * np.asarray(h), L):
        raise ValueError("box edges must be multiples of the grid spacing")
    return n


def _phi_from_distance(d, width, dtype):
    return np.tanh(d / width).astype(dtype)


def corner_minmax(grid, h, pos):
    """Min and max of the 8 grid nodes of the grid cell holding each position.

    grid is (nz, ny, nx) with node (i, j, k) at (i*hx, j*hy, k*hz), periodic.
    Used only to classify generated particles conservatively.
    """
    nz, ny, nx = grid.shape
    p = np.asarray(pos, dtype=np.float64)
    i0 = np.floor(p[:, 0] / h[0]).astype(np.int64)
    j0 = np.floor(p[:, 1] / h[1]).astype(np.int64)
    k0 = np.floor(p[:, 2] / h[2]).astype(np.int64)
    mn = np.full(p.shape[0], np.inf)
    mx = np.full(p.shape[0], -np.inf)
    for dk in (0, 1):
        kk = np.mod(k0 + dk, nz)
        for dj in (0, 1):
            jj = np.mod(j0 + dj, ny)
            for di in (0, 1):
                ii = np.mod(i0 + di, nx)
                v = grid[kk, jj, ii].astype(np.float64)
                mn = np.minimum(mn, v)
                mx = np.maximum(mx, v)
    return mn, mx


def maxwell_velocities(rng, n, kBT, mass=1.0):
    """Gaussian velocities at temperature kBT with zero net momentum."""
    v = rng.normal(0.0, math.sqrt(kBT / mass), size=(n, 3))
    if n > 1:
        v -= v.mean(axis=0, keepdims=True)
    return v


def _uniform_candidates(rng, L, rho):
    n = int(round(rho * float(np.prod(L))))
    return rng.random((n, 3)) * np.asarray(L)[None, :]


def _fcc_lattice(L, rho):
    """FCC lattice of number density ~rho whose unit cells tile the box."""
    a = (4.0 / rho) ** (1.0 / 3.0)
    n = np.maximum(1, np.rint(np.asarray(L) / a)).astype(np.int64)
    ax = np.asarray(L) / n
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.stack(np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]),
                             indexing="ij"), axis=-1).reshape(-1, 3)
    pts = (g[:, None, :] + base[None, :, :]).reshape(-1, 3) * ax[None, :]
    return pts + 0.25 * ax[None, :]


def _assemble(name, L, fluid, wall, kBT, rng, phi, h, params, meta):
    nf, nw = fluid.shape[0], wall.shape[0]
    pos = np.concatenate([fluid, wall], axis=0)
    pos = np.mod(pos, np.asarray(L)[None, :])
    vel = np.zeros_like(pos)
    vel[:nf] = maxwell_velocities(rng, nf, kBT)
    typ = np.concatenate([np.zeros(nf, np.int32), np.ones(nw, np.int32)])
    # gids are a seeded permutation so that gid order is not storage order
    gid = rng.permutation(nf + nw).astype(np.uint32)
    pos32 = pos.astype(np.float32)
    # float32 rounding can land exactly on L; keep every coordinate in [0, L)
    for k in range(3):
        col = pos32[:, k]
        col[col >= np.float32(L[k])] = np.float32(0.0)
    meta = dict(meta)
    meta.update(n_fluid=int(nf), n_wall=int(nw))
    return System(name=name, L=np.asarray(L, dtype=np.float64), pos=pos32,
                  vel=vel.astype(np.float32), type=typ, gid=gid, phi=phi,
                  h=np.asarray(h, dtype=np.float64), params=params, meta=meta)


def _classify(phi, h, pts, fluid=True):
    """Conservative side test for particles whose analytic distance already
    puts them on one side: fluid needs every surrounding node >= 0 (so the
    interpolated phi cannot be negative), walls every node <= 0."""
    mn, mx = corner_minmax(phi, h, pts)
    if fluid:
        return mn >= 0.0
    return mx <= 0.0


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def slab_system(L=(10.0, 10.0, 10.0), wall=1.5, rho=3.0, h=0.25, width=0.5,
                grid_dtype=np.float64, seed_fluid=0, seed_wall=1, params=None,
                wall_fill="uniform", name="poiseuille_slit"):
    """Plane channel: fluid slab wall < z < Lz - wall, walls elsewhere.

    Plane Poiseuille workload: 10^3 box, density 3, 1.5-thick wall slabs at
    each z end (which wrap into one 3-thick wall), phi = tanh(d/0.5) on a
    0.25-spaced float64 grid.  Walls are random particles at the fluid
    density (as in Sec. III.A, where randomly placed particles with phi < 0
    become the solid); wall_fill="fcc" gives a jittered FCC lattice instead.
    """
    L = np.asarray(L, dtype=np.float64)
    lo, hi = wall, L[2] - wall
    n = _grid_nodes(L, (h, h, h))
    zs = np.arange(n[2]) * h
    d1 = _slab_distance(zs, lo, hi, L[2])
    d = np.broadcast_to(d1[:, None, None], (n[2], n[1], n[0]))
    phi = _phi_from_distance(np.ascontiguousarray(d), width, grid_dtype)
    rng_f = np.random.default_rng(seed_fluid)
    cand = _uniform_candidates(rng_f, L, rho)
    dz = _slab_distance(cand[:, 2], lo, hi, L[2])
    keep = (dz > 0) & _classify(phi, (h, h, h), cand, fluid=True)
    fluid = cand[keep]
    rng_w = np.random.default_rng(seed_wall)
    if wall_fill == "fcc":
        lat = _fcc_lattice(L, rho)
        lat = lat[_slab_distance(lat[:, 2], lo, hi, L[2]) < 0]
        jit = lat + rng_w.uniform(-0.1, 0.1, size=lat.shape)
        ok = _slab_distance(jit[:, 2], lo, hi, L[2]) < 0
        jit[~ok, 2] = lat[~ok, 2]
        wallp = jit
    else:
        c = _uniform_candidates(rng_w, L, rho)
        wallp = c[_slab_distance(c[:, 2], lo, hi, L[2]) < 0]
    wallp = wallp[_classify(phi, (h, h, h), np.mod(wallp, L), fluid=False)]
    params = params or default_params(g=(0.02, 0.0, 0.0))
    rng_v = np.random.default_rng(seed_fluid + 1000)
    return _assemble(name, L, fluid, wallp, params["kBT"], rng_v, phi,
                     (h, h, h), params, dict(lo=lo, hi=hi, width=width))


def couette_system(L=(6.0, 4.0, 7.0), wall=1.5, U=1.0, rho=3.0, h=0.25, grid_dtype=np.float32,
                   seed=50, specular=False, linear_start=True, params=None, name="couette"):
    """Plane Couette flow: the slab channel of `slab_system` without body
    force, the wall below the fluid at rest and the wall above it moving at
    U along x (its wall particles carry that velocity; positions stay
    fixed).  With `linear_start` the fluid starts on the steady profile
    v_x = U (z - wall) / (Lz - 2 wall) plus thermal velocities.  `specular`
    is stored in the parameters (reflection mode)."""
    p = dict(params or default_params(g=(0.0, 0.0, 0.0), seed=seed))
    p["specular"] = bool(specular)
    s = slab_system(L=L, wall=wall, rho=rho, h=h, grid_dtype=grid_dtype, seed_fluid=seed,
                    seed_wall=seed + 1, params=p, wall_fill="uniform", name=name)
    lo, hi = s.meta["lo"], s.meta["hi"]
    z = s.pos[:, 2].astype(np.float64)
    top = (s.type != 0) & (z >= hi)
    vel = s.vel.astype(np.float64)
    vel[top, 0] = U
    if linear_start:
        fl = s.type == 0
        vel[fl, 0] += U * (z[fl] - lo) / (hi - lo)
    s.vel = vel.astype(np.float32)
    s.meta.update(U=float(U), specular=bool(specular))
    return s


def tiny_slab_system(L=(4.0, 4.0, 6.0), wall=1.0, rho=3.0, seed=7, g=(0.05, 0, 0),
                     grid_dtype=np.float32, **kw):
    """A few hundred particles: small enough for O(N^2) checks."""
    p = default_params(g=g, seed=seed, **kw)
    return slab_system(L=L, wall=wall, rho=rho, grid_dtype=grid_dtype,
                       seed_fluid=seed, seed_wall=seed + 1, params=p,
                       wall_fill="uniform", name="tiny_slab")


def _sin_cyl_distance(x, z, Lx, Lz, base, amp, period, radius, cx, cz):
    """Signed distance (fluid > 0) for a channel between z_b = base + amp*sin
    and its mirror z_t = Lz - z_b, periodic in z, minus an optional cylinder
    of `radius` along y centred at (cx, cz)."""
    x = np.asarray(x, dtype=np.float64)
    z = np.mod(np.asarray(z, dtype=np.float64), Lz)
    zb_c = np.mod(z - (base - Lz / 2), Lz) + (base - Lz / 2)
    zt_c = np.mod(z - (Lz - base - Lz / 2), Lz) + (Lz - base - Lz / 2)
    dist = np.minimum(_sinusoid_distance(x, zb_c, base, amp, period),
                      _sinusoid_distance(x, zt_c, Lz - base, -amp, period))
    zb = base + amp * np.sin(2 * math.pi * x / period)
    inside = (z > zb) & (z < Lz - zb)
    d = np.where(inside, dist, -dist)
    if radius > 0:
        dx = np.mod(x - cx + Lx / 2, Lx) - Lx / 2
        d_cyl = np.hypot(dx, z - cz) - radius
        d = np.minimum(d, d_cyl)
    return d


def sinusoid_cylinder_system(L=(40.0, 40.0, 80.0), rho=3.0, h=0.25, width=0.5,
                             base=4.0, amp=2.0, radius=6.0, seed=10, params=None,
                             grid_dtype=np.float32, wall_band=None,
                             name="sinusoid_channel_cylinder"):
    """Sinusoidal channel z = 4 + 2 sin(2 pi x/40) (mirrored at the top) with a
    cylinder of radius 6 along y at the box centre; walls fill phi < 0."""
    L = np.asarray(L, dtype=np.float64)
    n = _grid_nodes(L, (h, h, h))
    xs = np.arange(n[0]) * h
    zs = np.arange(n[2]) * h
    X, Z = np.meshgrid(xs, zs, indexing="xy")          # (nz, nx)
    dxz = _sin_cyl_distance(X, Z, L[0], L[2], base, amp, L[0], radius,
                            L[0] / 2, L[2] / 2)
    d = np.broadcast_to(dxz[:, None, :], (n[2], n[1], n[0]))
    phi = _phi_from_distance(np.ascontiguousarray(d), width, grid_dtype)
    rng = np.random.default_rng(seed)
    cand = _uniform_candidates(rng, L, rho)
    dc = _sin_cyl_distance(cand[:, 0], cand[:, 2], L[0], L[2], base, amp, L[0],
                           radius, L[0] / 2, L[2] / 2)
    fl = (dc > 0) & _classify(phi, (h, h, h), cand, fluid=True)
    wl = (dc < 0) & _classify(phi, (h, h, h), cand, fluid=False)
    if wall_band is not None:
        wl &= dc > -wall_band
    params = params or default_params(g=(0.01, 0.0, 0.0), seed=seed)
    return _assemble(name, L, cand[fl], cand[wl], params["kBT"], rng, phi,
                     (h, h, h), params, dict(base=base, amp=amp, radius=radius))


def stokes_params(g=0.005, dt=0.01, seed=60):
    """Sec. III.A-B's low-temperature fluid: kBT = 0.1, a_ff = a_fs = 1.875,
    gamma = 45 (sigma = 3), body force g along x on the fluid."""
    return default_params(a_ff=1.875, a_fs=1.875, gamma=45.0, kBT=0.1, dt=dt,
                          g=(g, 0.0, 0.0), seed=seed)


def cylinder_array_system(L=28.0, Lz=4.0, solid_fraction=0.1, rho=4.0, h=0.25, width=0.5,
                          wall_band=1.5, seed=61, params=None, grid_dtype=np.float32,
                          name="cylinder_array"):
    """Stokes flow through a square array of parallel cylinders (Sec. III.B):
    one cylinder of radius r = L sqrt(solid_fraction / pi) along z at the
    centre of an L x L cell, periodic in x and y (the array), in a periodic
    slab Lz thick; walls fill the cylinder within `wall_band` of its
    surface; body force along x."""
    L3 = np.asarray([L, L, Lz], dtype=np.float64)
    r = L * math.sqrt(solid_fraction / math.pi)
    n = _grid_nodes(L3, (h, h, h))
    xs = np.arange(n[0]) * h
    ys = np.arange(n[1]) * h

    def dist(x, y):
        dx = np.mod(np.asarray(x) - L / 2 + L / 2, L) - L / 2
        dy = np.mod(np.asarray(y) - L / 2 + L / 2, L) - L / 2
        return np.hypot(dx, dy) - r

    dxy = dist(xs[None, :], ys[:, None])               # (ny, nx)
    d = np.broadcast_to(dxy[None, :, :], (n[2], n[1], n[0]))
    phi = _phi_from_distance(np.ascontiguousarray(d), width, grid_dtype)
    rng = np.random.default_rng(seed)
    cand = _uniform_candidates(rng, L3, rho)
    dc = dist(cand[:, 0], cand[:, 1])
    fl = (dc > 0) & _classify(phi, (h, h, h), cand, fluid=True)
    wl = (dc < 0) & (dc > -wall_band) & _classify(phi, (h, h, h), cand, fluid=False)
    params = params or stokes_params(seed=seed)
    return _assemble(name, L3, cand[fl], cand[wl], params["kBT"], rng, phi,
                     (h, h, h), params, dict(radius=r, solid_fraction=solid_fraction, cell=L))


def sinusoid_slit_system(L=(20.0, 20.0, 20.0), rho=3.0, h=0.25, width=0.5,
                         base=3.0, amp=2.0, wall_band=1.5, seed=40, params=None,
                         grid_dtype=np.float32, name="sinusoid_slit"):
    """Slit with sinusoidal walls z = 3 + 2 sin(2 pi x/20), mirrored at the
    top, and a 1.5-thick band of wall particles (differentiation workload)."""
    return sinusoid_cylinder_system(L=L, rho=rho, h=h, width=width, base=base,
                                    amp=amp, radius=0.0, seed=seed,
                                    params=params or default_params(g=(0.02, 0, 0), seed=seed),
                                    grid_dtype=grid_dtype, wall_band=wall_band,
                                    name=name)


def gaussian_random_field(n, h, corr_len, rng, dtype=np.float32):
    """Periodic Gaussian random field with covariance exp(-r^2 / (2 l^2)).

    White noise on the grid filtered in Fourier space by exp(-k^2 l^2 / 4),
    the square root of the Gaussian spectrum; normalised to unit variance.
    """
    import scipy.fft as sfft
    noise = rng.standard_normal(size=tuple(n[::-1]), dtype=np.float32)
    spec = sfft.rfftn(noise, workers=-1)
    del noise
    kz = 2 * np.pi * np.fft.fftfreq(n[2], d=h).astype(np.float32)
    ky = 2 * np.pi * np.fft.fftfreq(n[1], d=h).astype(np.float32)
    kx = 2 * np.pi * np.fft.rfftfreq(n[0], d=h).astype(np.float32)
    c = np.float32(corr_len * corr_len / 4.0)
    spec *= np.exp(-c * kz * kz)[:, None, None]
    spec *= np.exp(-c * ky * ky)[None, :, None]
    spec *= np.exp(-c * kx * kx)[None, None, :]
    f = sfft.irfftn(spec, s=tuple(n[::-1]), workers=-1).astype(dtype, copy=False)
    del spec
    f -= f.mean()
    f /= f.std()
    return f


def porous_system(Lbox=128.0, rho=4.0, h=0.25, width=0.5, corr_len=6.0,
                  porosity=0.35, wall_band=1.5, seed_field=20, seed_particles=21,
                  params=None, name=None, device=None):
    """Porous medium: a thresholded Gaussian random field (correlation length
    6) with fluid where the field is below its `porosity` quantile; wall
    particles at the fluid density within `wall_band` of the interface.

    The signed distance near the interface is (thr - f)/|grad f| (central
    differences), clipped to +-3, where phi = tanh(d/0.5) is saturated.

    device: a torch device ("cuda") builds the same construction with torch
    on that device (its own seeded generator, so the values differ from the
    numpy path but the statistics are the same); used for the large boxes.
    """
    if device is not None:
        return _porous_system_torch(Lbox, rho, h, width, corr_len, porosity, wall_band,
                                    seed_field, seed_particles, params, name, device)
    L = np.array([Lbox, Lbox, Lbox], dtype=np.float64)
    n = _grid_nodes(L, (h, h, h))
    rng = np.random.default_rng(seed_field)
    f = gaussian_random_field(n, h, corr_len, rng)
    sample = f.reshape(-1)[:: max(1, f.size // 4_000_000)]
    thr = np.float32(np.quantile(sample, porosity))
    g2 = np.zeros_like(f)
    for ax in range(3):
        gax = (np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)) * np.float32(0.5 / h)
        g2 += gax * gax
        del gax
    np.sqrt(g2, out=g2)
    np.maximum(g2, np.float32(1e-6), out=g2)
    d = (thr - f) / g2
    del f, g2
    np.clip(d, -3.0, 3.0, out=d)
    phi = np.tanh(d * np.float32(1.0 / width)).astype(np.float32)
    prng = np.random.default_rng(seed_particles)
    cand = _uniform_candidates(prng, L, rho)
    mn, mx = corner_minmax(phi, (h, h, h), cand)
    fl = mn > 0.0
    dmin, _ = corner_minmax(d, (h, h, h), cand)
    wl = (mx < 0.0) & (dmin > -wall_band)
    del d
    params = params or default_params(a_ff=25.0, a_fs=35.0, g=(0.005, 0, 0),
                                      seed=seed_particles)
    return _assemble(name or f"porous_grf_{int(Lbox)}", L, cand[fl], cand[wl],
                     params["kBT"], prng, phi, (h, h, h), params,
                     dict(porosity=porosity, corr_len=corr_len, threshold=float(thr)))


def replica_systems(count=256, seed=30, rho=3.0, h=0.25, width=0.5,
                    edge_range=(8.0, 24.0), threads=8):
    """Independent replica boxes of uneven size and geometry.

    Edges are drawn per axis uniformly in edge_range and rounded to the grid
    spacing; geometry is a slit (1.5-thick walls), a cylinder along y of
    radius 3-10 (clipped to fit), or a pack of overlapping spheres of radius
    1.5-3 added until the porosity drawn from [0.4, 0.6] is reached.  Each
    replica has its own a in [15, 35], gamma in [3, 6] and g_x in
    [0.005, 0.03]; walls fill phi < 0.  The per-replica draws come from
    generator `seed` in replica order; replica r's geometry and particles
    from generator seed + 1 + r (also its force seed), so replicas are built
    independently (in `threads` threads).
    """
    rng = np.random.default_rng(seed)
    specs = []
    for r in range(count):
        L = np.round(rng.uniform(*edge_range, size=3) / h) * h
        kind = int(rng.integers(0, 3))
        a = float(rng.uniform(15, 35))
        gamma = float(rng.uniform(3, 6))
        gx = float(rng.uniform(0.005, 0.03))
        p = default_params(a_ff=a, a_fs=a, gamma=gamma, g=(gx, 0, 0),
                           seed=seed + 1 + r, replica=r)
        specs.append((r, L, kind, np.random.default_rng(seed + 1 + r), rho, h, width, p))
    if threads and threads > 1 and count > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=threads) as ex:
            return list(ex.map(lambda sp: _replica(*sp), specs))
    return [_replica(*sp) for sp in specs]


def _replica(r, L, kind, rng, rho, h, width, params):
    n = _grid_nodes(L, (h, h, h))
    zs = np.arange(n[2]) * h
    xs = np.arange(n[0]) * h
    ys = np.arange(n[1]) * h
    if kind == 0:
        dfun = lambda p: _slab_distance(p[..., 2], 1.5, L[2] - 1.5, L[2])
        meta = dict(kind="slit")
    elif kind == 1:
        rad = min(float(rng.uniform(3, 10)), min(L[0], L[2]) / 2 - 1.5)
        cx, cz = L[0] / 2, L[2] / 2

        def dfun(p, rad=rad, cx=cx, cz=cz):
            dx = np.mod(p[..., 0] - cx + L[0] / 2, L[0]) - L[0] / 2
            dz = np.mod(p[..., 2] - cz + L[2] / 2, L[2]) - L[2] / 2
            return np.hypot(dx, dz) - rad
        meta = dict(kind="cylinder", radius=rad)
    else:
        # spheres are added until the solid fraction, estimated on 20k
        # random sample points, reaches 1 - porosity
        target = float(rng.uniform(0.4, 0.6))
        samp = rng.random((20000, 3)) * L
        solid = np.zeros(samp.shape[0], dtype=bool)
        centres, radii = [], []
        while True:
            c = rng.random(3) * L
            rr = float(rng.uniform(1.5, 3.0))
            dd = np.mod(samp - c + L / 2, L) - L / 2
            solid |= (dd * dd).sum(-1) < rr * rr
            centres.append(c)
            radii.append(rr)
            if 1.0 - solid.mean() <= target or len(centres) > 2000:
                break
        centres_a = np.array(centres)
        radii_a = np.array(radii)
        from scipy.spatial import cKDTree
        tree = cKDTree(np.mod(centres_a, L), boxsize=L)
        kq = min(16, len(centres))

        def dfun(p, R=radii_a):
            # signed distance to the union: min over the kq nearest centres
            # of |p - c| - r (radii differ by at most 1.5, so a farther
            # centre only matters beyond the 16th neighbour)
            flat = np.mod(p.reshape(-1, 3), L)
            dist, ind = tree.query(flat, k=kq)
            if kq == 1:
                dist, ind = dist[:, None], ind[:, None]
            return (dist - R[ind]).min(axis=1).reshape(p.shape[:-1])
        meta = dict(kind="spheres", porosity_target=target, n_spheres=len(centres))
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    d = dfun(np.stack([X, Y, Z], axis=-1))
    phi = _phi_from_distance(d, width, np.float32)
    cand = _uniform_candidates(rng, L, rho)
    dc = dfun(cand)
    fl = (dc > 0) & _classify(phi, (h, h, h), cand, fluid=True)
    wl = (dc < 0) & _classify(phi, (h, h, h), cand, fluid=False)
    return _assemble(f"replica_{r}", L, cand[fl], cand[wl], params["kBT"], rng,
                     phi, (h, h, h), params, meta)


def bulk_system(L=(8.0, 8.0, 8.0), rho=3.0, h=0.5, seed=3, params=None,
                grid_dtype=np.float32, name="bulk_periodic"):
    """Fully periodic fluid with no walls (phi = +1 everywhere)."""
    L = np.asarray(L, dtype=np.float64)
    n = _grid_nodes(L, (h, h, h))
    phi = np.ones((n[2], n[1], n[0]), dtype=grid_dtype)
    rng = np.random.default_rng(seed)
    cand = _uniform_candidates(rng, L, rho)
    params = params or default_params(seed=seed)
    return _assemble(name, L, cand, np.zeros((0, 3)), params["kBT"], rng, phi,
                     (h, h, h), params, {})


def _porous_system_torch(Lbox, rho, h, width, corr_len, porosity, wall_band, seed_field,
                         seed_particles, params, name, device):
    import torch
    dev = torch.device(device)
    L = np.array([Lbox, Lbox, Lbox], dtype=np.float64)
    n = _grid_nodes(L, (h, h, h))
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed_field))
    shape = (int(n[2]), int(n[1]), int(n[0]))
    f = torch.randn(shape, generator=gen, device=dev, dtype=torch.float32)
    spec = torch.fft.rfftn(f)
    del f
    c = corr_len * corr_len / 4.0
    kz = 2 * math.pi * torch.fft.fftfreq(shape[0], d=h, device=dev)
    ky = 2 * math.pi * torch.fft.fftfreq(shape[1], d=h, device=dev)
    kx = 2 * math.pi * torch.fft.rfftfreq(shape[2], d=h, device=dev)
    spec *= torch.exp(-c * kz * kz)[:, None, None]
    spec *= torch.exp(-c * ky * ky)[None, :, None]
    spec *= torch.exp(-c * kx * kx)[None, None, :]
    f = torch.fft.irfftn(spec, s=shape)
    del spec
    f = (f - f.mean()) / f.std()
    flat = f.reshape(-1)
    sample = flat[:: max(1, flat.numel() // 4_000_000)]
    thr = torch.quantile(sample, porosity)
    g2 = torch.zeros_like(f)
    for ax in range(3):
        gax = (torch.roll(f, -1, dims=ax) - torch.roll(f, 1, dims=ax)) * (0.5 / h)
        g2 += gax * gax
        del gax
    g2 = torch.sqrt(g2).clamp_(min=1e-6)
    d = ((thr - f) / g2).clamp_(-3.0, 3.0)
    del f, g2
    phi = torch.tanh(d * (1.0 / width))
    pgen = torch.Generator(device=dev)
    pgen.manual_seed(int(seed_particles))
    ncand = int(round(rho * float(np.prod(L))))
    cand = torch.rand((ncand, 3), generator=pgen, device=dev, dtype=torch.float64) * float(Lbox)

    def cmm(grid):
        i0 = torch.floor(cand / h).long()
        mn = torch.full((ncand,), float("inf"), device=dev)
        mx = torch.full((ncand,), float("-inf"), device=dev)
        for dz in (0, 1):
            kk = (i0[:, 2] + dz) % shape[0]
            for dy in (0, 1):
                jj = (i0[:, 1] + dy) % shape[1]
                for dx in (0, 1):
                    ii = (i0[:, 0] + dx) % shape[2]
                    v = grid[kk, jj, ii]
                    mn = torch.minimum(mn, v)
                    mx = torch.maximum(mx, v)
        return mn, mx

    mn, mx = cmm(phi)
    fl = mn > 0.0
    dmin, _ = cmm(d)
    wl = (mx < 0.0) & (dmin > -wall_band)
    del d
    fluid = cand[fl].cpu().numpy()
    wall = cand[wl].cpu().numpy()
    nf, nw = fluid.shape[0], wall.shape[0]
    vel = torch.randn((nf, 3), generator=pgen, device=dev, dtype=torch.float64)
    vel = vel - vel.mean(dim=0, keepdim=True)
    perm = torch.randperm(nf + nw, generator=pgen, device=dev)
    phi_np = phi.cpu().numpy()
    del phi
    params = params or default_params(a_ff=25.0, a_fs=35.0, g=(0.005, 0, 0),
                                      seed=seed_particles)
    pos = np.concatenate([fluid, wall], axis=0)
    pos32 = np.mod(pos, Lbox).astype(np.float32)
    pos32[pos32 >= np.float32(Lbox)] = np.float32(0.0)
    velall = np.zeros_like(pos32)
    velall[:nf] = (vel * math.sqrt(params["kBT"])).cpu().numpy().astype(np.float32)
    typ = np.concatenate([np.zeros(nf, np.int32), np.ones(nw, np.int32)])
    return System(name=name or f"porous_grf_{int(Lbox)}", L=L, pos=pos32, vel=velall, type=typ,
                  gid=perm.cpu().numpy().astype(np.uint32), phi=phi_np,
                  h=np.array([h, h, h]), params=params,
                  meta=dict(porosity=porosity, corr_len=corr_len, threshold=float(thr),
                            n_fluid=int(nf), n_wall=int(nw), generator="torch"))


def step_phase_field(n, h, seed, min_len=6.0, margin=0.25):
    """A -1 (solid) / +1 (fluid) step function on the node grid n = (nx, ny,
    nz), spacings h, returned as an array (nz, ny, nx): the sign of
    sum_a A_a cos(2 pi x_a / L_a + p_a) - t over the axes at least `min_len`
    long (A_a, p_a seeded).  Such a field's critical values are the sums
    +-A_x +-A_y +-A_z; the threshold t stays `margin` min(A) away from all of
    them, so the level set has no near-degenerate saddle and every solid and
    fluid feature is as wide as a sizeable part of its box, not a sliver of
    a few nodes.  Axes shorter than `min_len` carry no variation; with none
    long enough, the field is a seeded random step function (for grids
    smaller than the interface itself)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in n)
    L = [nx * h[0], ny * h[1], nz * h[2]]
    use = [a for a in range(3) if L[a] >= min_len]
    if not use:
        return np.where(rng.random((nz, ny, nx)) < 0.5, -1.0, 1.0)
    A = {a: rng.uniform(0.6, 1.4) for a in use}
    crit = [0.0]
    for a in use:
        crit = [c + s * A[a] for c in crit for s in (-1.0, 1.0)]
    lo, hi = min(crit), max(crit)
    gap = margin * min(A.values())
    while True:
        t = rng.uniform(0.5 * lo, 0.5 * hi)
        if all(abs(t - c) >= gap for c in crit):
            break
    f = np.zeros((nz, ny, nx))
    coords = [np.arange(nx) * h[0], np.arange(ny) * h[1], np.arange(nz) * h[2]]
    shape = {0: (1, 1, nx), 1: (1, ny, 1), 2: (nz, 1, 1)}
    for a in use:
        p = rng.uniform(0, 2 * np.pi)
        f = f + A[a] * np.cos(2 * np.pi * coords[a] / L[a] + p).reshape(shape[a])
    return np.where(f > t, 1.0, -1.0)
