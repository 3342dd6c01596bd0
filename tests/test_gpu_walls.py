"""Moving walls and specular reflection on the GPU, through the C ABI.

Bars: one step from a common FP32 snapshot against the oracle, with many
reflections off a resting and a sliding plate (events bit-exact, cells,
positions of fluid and walls, velocities, forces: the one-step bar of the
resting-wall parity tests); plane Couette flow has the closed-form linear
profile; common motion of fluid and plates is kept; a box with moving walls
gives the same bits in a batch as alone, under graph replay as with direct
launches, and after the autotuner's trials; the adjoint form refuses both
modes.
"""
import sys

import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu
from test_gpu_parity import _one_step_compare

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dpd():
    require_gpu()
    import paper_1807_09896_amd as dpd
    dpd.load_library()
    return dpd


def _aimed_couette(spec, seed, U=1.0, speed=20.0, band=0.25):
    """Couette slab (upper plate sliding at U along x) with the fluid within
    `band` of a plate sent into it at `speed`: many reflections per step."""
    s = workloads.couette_system(L=(8.0, 6.0, 7.0), U=U, specular=spec, seed=seed)
    rng = np.random.default_rng(seed)
    lo, hi = s.meta["lo"], s.meta["hi"]
    z = s.pos[:, 2]
    fl = s.type == 0
    near_lo = fl & (z - lo < band)
    near_hi = fl & (hi - z < band)
    v = s.vel.copy()
    v[near_lo, 2] = -speed
    v[near_hi, 2] = speed
    v[near_lo | near_hi, 0] += rng.uniform(-3, 3, (near_lo | near_hi).sum()).astype(np.float32)
    s.vel = v
    return s


def _by_gid(s, arr):
    out = np.empty_like(arr)
    out[s.gid] = arr
    return out


@pytest.mark.parametrize("spec", [False, True], ids=["bounce_back", "specular"])
def test_one_step_with_moving_plate(dpd, oracle_lib, spec):
    s = _aimed_couette(spec, seed=61 if spec else 62)
    say("couette", "specular" if spec else "bounce-back", s.n)
    _one_step_compare(dpd, oracle_lib, s)
    # walls: moved by dt v on both sides in the same FP32 decision form
    o = oracle_lib.Oracle(s)
    o.step(1)
    sim = dpd.Simulation(s)
    sim.step(1)
    st = {k: v.cpu().numpy() for k, v in sim.state().items()}
    walls = _by_gid(s, s.type) != 0
    assert np.array_equal(st["pos"][walls], _by_gid(s, o.xs)[walls])
    assert np.array_equal(st["vel"][walls], _by_gid(s, s.vel)[walls])
    ev = st["events"]
    say("events", int((ev > 0).sum()))
    assert (ev > 0).sum() >= 10
    sim.close()


@pytest.mark.parametrize("spec", [False, True], ids=["bounce_back", "specular"])
def test_one_step_mid_run_with_moving_plate(dpd, oracle_lib, spec):
    """Snapshot after 25 oracle steps (the walls have moved): set_state takes
    the wall positions of a box with moving walls."""
    s = _aimed_couette(spec, seed=63 if spec else 64)
    _one_step_compare(dpd, oracle_lib, s, nsteps_before=25)


def _gpu_couette(dpd, spec, seed=70, warm=1000, blocks=12, block_steps=500):
    U = 1.0
    s = workloads.couette_system(L=(24.0, 24.0, 7.0), U=U, specular=spec, seed=seed)
    lo, hi = s.meta["lo"], s.meta["hi"]
    sim = dpd.Simulation(s, graph=True)
    sim.step(warm)
    nbz = 14   # 0.5-wide bins over z; the fluid fills bins 3..10
    zc = (np.arange(nbz) + 0.5) * s.L[2] / nbz
    inside = (zc > lo) & (zc < hi)
    slopes, vlo, vhi = [], [], []
    for _ in range(blocks):
        acc = None
        for _ in range(block_steps // 10):
            sim.step(10)
            p = sim.profile(axis=2, nbins=nbz)
            acc = p if acc is None else acc + p
        a = acc.cpu().numpy()
        m = a[inside, 1] / a[inside, 0]
        fit = np.polyfit(zc[inside], m, 1)
        slopes.append(fit[0])
        vlo.append(np.polyval(fit, lo))
        vhi.append(np.polyval(fit, hi))
    c = sim.counters()
    sim.close()
    se = lambda x: np.std(x, ddof=1) / np.sqrt(len(x))
    return U, hi - lo, np.mean(slopes), se(slopes), np.mean(vlo), se(vlo), np.mean(vhi), se(vhi), c


def test_couette_profile_gpu(dpd):
    """Plane Couette flow, bounce-back: v_x linear from 0 at the resting plate
    to U at the sliding one (no slip at both phi = 0 interfaces)."""
    U, H, slope, s_se, vlo, lo_se, vhi, hi_se, c = _gpu_couette(dpd, spec=False)
    say("slope %.4f +- %.4f (exact %.4f)  v(lo) %.4f +- %.4f  v(hi) %.4f +- %.4f  bounces %d" % (
        slope, s_se, U / H, vlo, lo_se, vhi, hi_se, c["bounce"]))
    assert c["unstable"] == 0 and c["bounce"] > 0
    assert abs(slope - U / H) < 3 * s_se + 0.01
    assert abs(vlo) < 3 * lo_se + 0.02
    assert abs(vhi - U) < 3 * hi_se + 0.02


def test_common_motion_kept_gpu(dpd):
    s = workloads.couette_system(L=(16.0, 12.0, 7.0), U=1.0, seed=71, linear_start=False)
    vel = s.vel.copy()
    vel[s.type != 0, 0] = 1.0
    vel[s.type == 0, 0] += 1.0
    s.vel = vel
    sim = dpd.Simulation(s, graph=True)
    means = []
    for _ in range(10):
        sim.step(300)
        p = sim.profile(axis=2, nbins=1).cpu().numpy()
        means.append(p[0, 1] / p[0, 0])
    sim.close()
    m, se = np.mean(means), np.std(means, ddof=1) / np.sqrt(len(means))
    say("common motion: mean v_x %.4f +- %.4f" % (m, se))
    assert abs(m - 1.0) < 4 * se + 0.03


def _snap(sim, r):
    st = {k: v.cpu().numpy() for k, v in sim.state(r).items()}
    st["force"] = sim.forces(r).cpu().numpy()
    return st


def _same(a, b, what):
    for k in ("pos", "vel", "events", "cell_of", "force"):
        assert np.array_equal(a[k], b[k]), (what, k)


def test_moving_walls_batch_graph_and_autotune(dpd, tmp_path, monkeypatch):
    boxes = [workloads.tiny_slab_system(),
             workloads.couette_system(U=1.0, seed=72),
             workloads.couette_system(U=-0.5, seed=73, specular=True)]
    batch = dpd.Simulation(boxes)
    batch.step(12)
    for r in (1, 2):
        alone = dpd.Simulation(boxes[r])
        alone.step(12)
        _same(_snap(batch, r), _snap(alone, 0), ("batch vs alone", r))
        alone.close()
    graph = dpd.Simulation(boxes, graph=True)
    graph.step(12)
    for r in range(3):
        _same(_snap(graph, r), _snap(batch, r), ("graph", r))
    # the autotuner's trials leave the state (walls included) as it was
    monkeypatch.setenv("DPD_TUNE_CACHE", str(tmp_path / "tune.txt"))
    before = [_snap(graph, r) for r in range(3)]
    graph.autotune(2)
    for r in range(3):
        _same(_snap(graph, r), before[r], ("autotune", r))
    graph.step(5)
    batch.step(5)
    for r in range(3):
        _same(_snap(graph, r), _snap(batch, r), ("after autotune", r))
    graph.close()
    batch.close()


def test_adjoint_refuses_moving_walls_and_specular(dpd):
    from paper_1807_09896_amd.adjoint import Window
    for s in (workloads.couette_system(U=1.0, seed=74),
              workloads.couette_system(U=0.0, seed=75, specular=True)):
        sim = dpd.Simulation(s)
        w = Window(sim, steps=4, ckpt=2)
        with pytest.raises(dpd.DPDError):
            w.run()
        sim.close()
