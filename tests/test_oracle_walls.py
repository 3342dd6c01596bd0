"""Pins of the oracle's moving walls and specular reflection (Sec. II.C:
v = -v^t + 2 v_wall after a bounce-back, Eq. 17 with v^t - v_wall; Sec. I:
specular reflection reverses only the normal component).

Pinned against what the physics fixes, not against the formulas retyped:
plane Couette flow between a resting and a sliding plate has the linear
closed-form profile (no slip at both interfaces); a fluid and walls that all
move at one velocity stay at it (Galilean invariance, which fails if the
walls' corrugation did not move with them or a reflection ignored the wall
velocity); a specular reflection off a plane keeps the tangential velocity
and the speed relative to the wall exactly and moves the particle only
along the normal; a bounce-back off a moving plate reverses the velocity
relative to the plate.
"""
import numpy as np
import pytest

import oracle
import workloads


def _no_forces(p):
    q = dict(p)
    q["a"] = [[0.0, 0.0], [0.0, 0.0]]
    q["gamma"] = 0.0
    q["kBT"] = 0.0
    q["g"] = (0.0, 0.0, 0.0)
    return q


def _aimed(spec, U=(0.7, -0.4, 0.0), n=24, seed=60):
    """Force-free fluid particles launched into the two plates of a Couette
    slab (the upper plate slides at U), one step apart from their crossing."""
    s = workloads.couette_system(U=1.0, specular=spec, seed=seed, linear_start=False)
    vel = s.vel.copy()
    top = (s.type != 0) & (s.pos[:, 2] >= s.meta["hi"])
    vel[top] = np.asarray(U, np.float32)
    rng = np.random.default_rng(seed)
    fl = np.nonzero(s.type == 0)[0][:n]
    lo, hi = s.meta["lo"], s.meta["hi"]
    pos = s.pos.copy()
    for m, i in enumerate(fl):
        up = m % 2 == 1
        d0 = rng.uniform(0.01, 0.1)
        pos[i, 2] = np.float32(hi - d0 if up else lo + d0)
        vz = (d0 + rng.uniform(0.02, 0.1)) / s.params["dt"]
        vel[i] = np.asarray([rng.uniform(-2, 2), rng.uniform(-2, 2), vz if up else -vz], np.float32)
    # the other fluid particles rest in the middle of the channel
    rest = np.nonzero(s.type == 0)[0][n:]
    vel[rest] = 0.0
    s.pos, s.vel = pos, vel
    p = _no_forces(s.params)
    p["specular"] = spec
    s.params = p
    # the plate's velocity as stored (float32 rows)
    return s, fl, np.asarray(U, np.float32).astype(np.float64)


def test_specular_keeps_tangential_velocity_and_speed():
    s, fl, U = _aimed(spec=True)
    o = oracle.Oracle(s)
    v0 = o.v.copy()
    r0 = o.r.copy()
    ev = o.step(1)
    hit = fl[ev[fl] > 0]
    assert len(hit) >= len(fl) // 2
    hi = s.meta["hi"]
    for i in hit:
        vw = U if r0[i, 2] > 3.5 else np.zeros(3)
        # the plane's normal is z (up to the rounding of the interpolant's
        # gradient): x and y velocity untouched, the normal component
        # relative to the wall reversed, the speed relative to the wall kept
        assert abs(o.v[i, 0] - v0[i, 0]) < 1e-12 and abs(o.v[i, 1] - v0[i, 1]) < 1e-12
        assert abs((o.v[i, 2] - vw[2]) + (v0[i, 2] - vw[2])) < 1e-12
        assert abs(np.linalg.norm(o.v[i] - vw) - np.linalg.norm(v0[i] - vw)) < 1e-12
        if ev[i] == 1:
            # the reflection moves the particle along the normal only: x and
            # y are those of the free flight
            dt = s.params["dt"]
            for a in range(2):
                free = np.mod(r0[i, a] + dt * v0[i, a], s.L[a])
                assert abs(o.r[i, a] - free) < 1e-9 or abs(abs(o.r[i, a] - free) - s.L[a]) < 1e-9


def test_bounce_back_reverses_velocity_relative_to_moving_plate():
    s, fl, U = _aimed(spec=False)
    o = oracle.Oracle(s)
    v0 = o.v.copy()
    r0 = o.r.copy()
    ev = o.step(1)
    hit = fl[ev[fl] > 0]
    assert len(hit) >= len(fl) // 2
    up = [i for i in hit if r0[i, 2] > 3.5]
    assert up, "some particles must reflect off the sliding plate"
    for i in hit:
        vw = U if r0[i, 2] > 3.5 else np.zeros(3)
        assert np.allclose(o.v[i] - vw, -(v0[i] - vw), rtol=0, atol=1e-12)
        if ev[i] == 1:
            # the displacement from the free-flight point is along the
            # velocity relative to the plate
            dt = s.params["dt"]
            free = r0[i] + dt * v0[i]
            d = o.r[i] - free
            d -= np.round(d / s.L) * s.L
            rel = v0[i] - vw
            cross = np.cross(d, rel)
            assert np.linalg.norm(cross) <= 1e-9 * (1 + np.linalg.norm(rel))


def _couette_stats(spec, seed=51, warm=1000, blocks=12, block_steps=500):
    U = 1.0
    s = workloads.couette_system(L=(8.0, 6.0, 7.0), U=U, specular=spec, seed=seed)
    o = oracle.Oracle(s)
    lo, hi = s.meta["lo"], s.meta["hi"]
    o.step(warm)
    nb = 8
    zc = lo + (np.arange(nb) + 0.5) * (hi - lo) / nb
    slopes, vlo, vhi = [], [], []
    fl = o.type == 0
    for _ in range(blocks):
        bs = np.zeros(nb)
        bc = np.zeros(nb)
        for _ in range(block_steps // 10):
            o.step(10)
            z = o.r[fl, 2]
            idx = np.clip(((z - lo) / (hi - lo) * nb).astype(int), 0, nb - 1)
            np.add.at(bs, idx, o.v[fl, 0])
            np.add.at(bc, idx, 1)
        fit = np.polyfit(zc, bs / bc, 1)
        slopes.append(fit[0])
        vlo.append(np.polyval(fit, lo))
        vhi.append(np.polyval(fit, hi))
    se = lambda x: np.std(x, ddof=1) / np.sqrt(len(x))
    return (U, hi - lo, np.mean(slopes), se(slopes), np.mean(vlo), se(vlo), np.mean(vhi), se(vhi))


def test_couette_profile_is_linear_with_no_slip():
    """Plane Couette flow, lower plate at rest, upper plate sliding at U:
    v_x(z) = U (z - z_lo) / (z_hi - z_lo) with the no-slip planes at the
    phi = 0 interfaces (bounce-back, Sec. II.C), within 3 standard errors of
    12 block means over 6000 steps."""
    U, H, slope, s_se, vlo, lo_se, vhi, hi_se = _couette_stats(spec=False)
    assert abs(slope - U / H) < 3 * s_se + 0.01, (slope, s_se)
    assert abs(vlo) < 3 * lo_se + 0.02, (vlo, lo_se)
    assert abs(vhi - U) < 3 * hi_se + 0.02, (vhi, hi_se)


def test_common_motion_is_kept():
    """Fluid and both plates moving at one velocity: the fluid keeps it
    (Galilean invariance of the pair forces and of the moving-wall
    reflection)."""
    s = workloads.couette_system(U=1.0, seed=50, linear_start=False)
    vel = s.vel.copy()
    vel[s.type != 0, 0] = 1.0
    vel[s.type == 0, 0] += 1.0
    s.vel = vel
    o = oracle.Oracle(s)
    fl = o.type == 0
    means = []
    for _ in range(10):
        acc = []
        for _ in range(30):
            o.step(10)
            acc.append(o.v[fl, 0].mean())
        means.append(np.mean(acc))
    m = np.mean(means)
    se = np.std(means, ddof=1) / np.sqrt(len(means))
    assert abs(m - 1.0) < 4 * se + 0.03, (m, se)


def test_resting_walls_unchanged_by_the_moving_wall_path():
    """Zero wall velocities take the resting-wall path: the same state after
    30 steps whether or not the walls carry an explicit zero velocity row."""
    s = workloads.tiny_slab_system()
    a = oracle.Oracle(s)
    a.step(30)
    s2 = workloads.tiny_slab_system()
    v = s2.vel.copy()
    v[s2.type != 0] = -0.0
    s2.vel = v
    b = oracle.Oracle(s2)
    b.step(30)
    assert np.array_equal(a.r, b.r) and np.array_equal(a.v, b.v)


def test_window_rejects_moving_walls_and_specular():
    s = workloads.couette_system(U=1.0, seed=50)
    with pytest.raises(ValueError):
        oracle.Oracle(s).window(2)
    s = workloads.tiny_slab_system()
    p = dict(s.params)
    p["specular"] = True
    with pytest.raises(ValueError):
        oracle.Oracle(s, params=p).window(2)
