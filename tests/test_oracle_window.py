"""Pins of the oracle's window (the reference for the adjoint form).

The window iterates the oracle step; replay holds every discrete decision
(bounce-back events, pair sets, profile bins) at its recorded value, so its
finite differences are the derivative the adjoint computes.  Pinned here:
record mode is the oracle step itself; replay reproduces record bit for
bit; an ideal gas has a closed-form profile and gradient; and central
differences of replay converge at second order (the frozen map is smooth),
also through the bounce-back of Eq. 17 and the phase-field values.
"""
import numpy as np
import pytest

import oracle
import workloads


def _stress(seed=70):
    """Slab channel with hot fluid and particles aimed at the walls, so that
    a few-step window holds bounce-backs (codes 1 and 2)."""
    s = workloads.slab_system(L=(8.0, 6.0, 7.0), wall=1.0, width=0.5, grid_dtype=np.float32,
                              seed_fluid=seed, seed_wall=seed + 1,
                              params=workloads.default_params(g=(0.02, 0.0, 0.0), seed=seed))
    s.vel = (s.vel * 3.0).astype(np.float32)
    rng = np.random.default_rng(seed + 5)
    fl = np.nonzero(s.type == 0)[0]
    pick = rng.choice(fl, size=60, replace=False)
    dt = s.params["dt"]
    for m, i in enumerate(pick):
        d0 = rng.uniform(0.001, 0.3)
        top = m % 2 == 1
        s.pos[i, 2] = np.float32(6.0 - d0 if top else 1.0 + d0)
        vz = (d0 + rng.uniform(0.01, 0.15)) / dt
        s.vel[i, 2] = np.float32(vz if top else -vz)
    return s


def test_record_is_the_oracle_step(oracle_lib):
    s = _stress()
    o = oracle_lib.Oracle(s)
    w = o.window(6, axis=2, nbins=10)
    ev = w["logs"]["ev"]
    assert (ev == 1).sum() > 20
    ref = oracle_lib.Oracle(s)
    for t in range(6):
        e = ref.step(1)
        assert np.array_equal(e, ev[t])
        assert np.array_equal(ref.xs, w["logs"]["xs"][t])
    # the window refreshes f0 and does not clamp w at rc: equal up to pairs
    # within rounding of the cutoff
    assert np.abs(ref.r - w["r"]).max() < 1e-12
    assert np.abs(ref.v - w["v"]).max() < 1e-10
    # profile = mean v_x per bin over the states after steps 1..T
    sums = np.zeros(10)
    cnt = np.zeros(10)
    ref2 = oracle_lib.Oracle(s)
    fl = s.type == 0
    for t in range(6):
        ref2.step(1)
        b = w["logs"]["bin"][t][fl]
        np.add.at(sums, b, ref2.v[fl, 0])
        np.add.at(cnt, b, 1.0)
        z = ref2.xs[fl, 2]
        assert np.array_equal(b, np.clip(np.floor(z * np.float32(10 / 7.0)), 0, 9).astype(int))
    assert np.array_equal(cnt, w["counts"])
    assert np.allclose(sums, w["sums"], rtol=0, atol=1e-9)


def test_replay_reproduces_record(oracle_lib):
    s = _stress(seed=71)
    o = oracle_lib.Oracle(s)
    w = o.window(8, axis=2, nbins=12)
    w2 = o.window(8, axis=2, nbins=12, logs=w["logs"])
    assert np.array_equal(w["sums"], w2["sums"])
    assert np.array_equal(w["r"], w2["r"]) and np.array_equal(w["v"], w2["v"])
    # the state of the Oracle object is left unchanged
    assert np.array_equal(o.r, np.asarray(s.pos, np.float64))


def test_ideal_gas_closed_form(oracle_lib):
    """a = gamma = kBT = 0: every force is the body force, so
    v_x(t) = v_x(0) + t dt g_x and dP_b/dg_x = sum_{t, i in b} t dt / N_b."""
    p = workloads.default_params(a_ff=0.0, a_fs=0.0, gamma=0.0, kBT=0.0, g=(0.05, 0, 0), seed=3)
    s = workloads.bulk_system(L=(6.0, 5.0, 4.0), params=p)
    o = oracle_lib.Oracle(s)
    T, nb = 12, 5
    w = o.window(T, axis=2, nbins=nb)
    dt = p["dt"]
    v0 = np.asarray(s.vel, np.float64)[:, 0]
    sums = np.zeros(nb)
    dsum = np.zeros(nb)
    cnt = np.zeros(nb)
    for t in range(T):
        b = w["logs"]["bin"][t]
        np.add.at(sums, b, v0 + (t + 1) * dt * 0.05)
        np.add.at(dsum, b, (t + 1) * dt)
        np.add.at(cnt, b, 1.0)
    assert np.array_equal(cnt, w["counts"])
    assert np.allclose(w["sums"], sums, rtol=0, atol=1e-11)
    hstep = 1e-4
    prof = []
    for gx in (0.05 + hstep, 0.05 - hstep):
        o.set_params(g=[gx, 0.0, 0.0])
        prof.append(o.window(T, axis=2, nbins=nb, logs=w["logs"])["profile"])
    fd = (prof[0] - prof[1]) / (2 * hstep)
    assert np.allclose(fd, dsum / cnt, rtol=1e-7, atol=1e-9)


def _loss(prof, target):
    return float(((prof - target) ** 2).mean())


def _central(f, h):
    return (f(h) - f(-h)) / (2 * h)


@pytest.mark.parametrize("what", ["a_ff", "a_fs", "gamma", "g_x", "phi"])
def test_frozen_differences_converge_at_second_order(oracle_lib, what):
    s = _stress(seed=72)
    o = oracle_lib.Oracle(s)
    T, nb = 6, 10
    base = o.window(T, axis=2, nbins=nb)
    assert (base["logs"]["ev"] == 1).sum() > 20
    target = base["profile"] * 0.5 + 0.01
    p0 = dict(o.params)
    phi0 = o.phi64.copy()
    # phi direction: smooth bump on the nodes within 0.5 of the lower wall
    z = np.arange(phi0.shape[0]) * s.h[2]
    bump = np.exp(-((z - 1.0) / 0.3) ** 2)[:, None, None] * np.ones_like(phi0)

    def f(h):
        if what == "phi":
            o.set_phi(phi0 + h * bump)
        else:
            p = dict(p0)
            a = [list(r) for r in p0["a"]]
            if what == "a_ff":
                a[0][0] += h
            elif what == "a_fs":
                a[0][1] += h
                a[1][0] += h
            elif what == "gamma":
                p["gamma"] = p0["gamma"] + h
            else:
                p["g"] = [p0["g"][0] + h, 0.0, 0.0]
            p["a"] = a
            o.params = p
            o.cparams = o._make_params(p)
        out = _loss(o.window(T, axis=2, nbins=nb, logs=base["logs"])["profile"], target)
        o.params = dict(p0)
        o.cparams = o._make_params(p0)
        o.set_phi(phi0)
        return out

    # steps small enough that no event's phi(r*) or phi(r^t) crosses the
    # clamps of Eq. 17's atanh arguments (a kink of the frozen map)
    h = {"a_ff": 0.4, "a_fs": 0.4, "gamma": 0.2, "g_x": 0.02, "phi": 1e-3}[what]
    d1, d2, d3 = _central(f, h), _central(f, h / 2), _central(f, h / 4)
    assert d1 != 0.0
    e1, e2 = abs(d1 - d2), abs(d2 - d3)
    # O(h^2): successive differences shrink about fourfold (or sit at rounding)
    assert e2 < 1e-9 * abs(d3) + 1e-15 or 2.5 < e1 / e2 < 6.0, (d1, d2, d3)


def test_window_is_its_step_iterated(oracle_lib):
    """The replayed window equals its one-step map iterated from the
    window's starting force (the form used to linearise it step by step
    around a given trajectory): the same counts and final state bit for
    bit, the same sums up to the order of their additions (the window adds
    every term to one running sum, the steps are summed per step)."""
    s = workloads.tiny_slab_system(seed=19)
    s.vel = (s.vel * 3).astype(np.float32)
    o = oracle_lib.Oracle(s)
    T, nb = 9, 6
    base = o.window(T, axis=2, nbins=nb)
    logs = base["logs"]
    assert (logs["ev"] != 0).sum() > 0
    rep = o.window(T, axis=2, nbins=nb, logs=logs)
    r, v = o.r.copy(), o.v.copy()
    v[o.type != 0] = 0.0
    f = o.window_start_force(r, v, o.k)
    sums = np.zeros(nb)
    counts = np.zeros(nb)
    for t in range(T):
        r, v, f, sm, cn = o.window_step(r, v, f, o.k + t + 1, logs["ev"][t], logs["xs"][t],
                                        logs["bin"][t], axis=2, nbins=nb)
        sums += sm
        counts += cn
    assert np.array_equal(counts, rep["counts"])
    np.testing.assert_allclose(sums, rep["sums"], rtol=1e-13, atol=1e-13)
    assert np.array_equal(r, rep["r"])
    assert np.array_equal(v, rep["v"])
