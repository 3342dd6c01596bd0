"""Both pair-force kernels against the oracle, whichever is the default.

The library computes pair forces either per particle (each lane walks the
27 neighbour cells of its particle from global memory; boxes with fewer
than five cells along an axis always take it) or by LDS-staged cell bricks
(each pair between home particles of a brick evaluated once and added to
both as 64-bit fixed-point sums).  DPD_PAIR_KERNEL, read when a context is
created, selects one of them; these tests create contexts with each.

Bars as in test_gpu_parity: initial forces within 2e-5 F_scale with cell
indices and interacting pair sets bit-exact; one step from a common FP32
snapshot with events and cells bit-exact.  The brick kernel's results do
not depend on the order of its integer sums: mask on and off, repeated
runs, and a box alone or in a batch give identical bits, and the dense box
(cells of up to ~30 particles) goes through the split of bricks whose
neighbourhood overflows LDS.
"""
import os
import sys

import numpy as np
import pytest

import workloads
from gpu_helpers import by_gid, force_scale, require_gpu, sorted_pairs
from test_gpu_parity import SYSTEMS, _one_step_compare, _stress_system

pytestmark = pytest.mark.gpu

FORCE_TOL = 2e-5
KERNELS = ["cells", "bricks"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dpd():
    require_gpu()
    import paper_1807_09896_amd as dpd
    dpd.load_library()
    return dpd


@pytest.fixture
def kernel(request, monkeypatch):
    monkeypatch.setenv("DPD_PAIR_KERNEL", request.param)
    return request.param


@pytest.mark.parametrize("kernel", KERNELS, indirect=True)
@pytest.mark.parametrize("name", ["slab_f64grid", "curved", "dense"])
def test_initial_forces_and_pairs(dpd, oracle_lib, kernel, name):
    s = SYSTEMS[name]()
    say("initial forces", kernel, name, s.n)
    o = oracle_lib.Oracle(s)
    sim = dpd.Simulation(s)
    f_gpu = sim.forces().cpu().numpy().astype(np.float64)
    f_or = by_gid(o, o.f)
    fluid_g = by_gid(o, s.type) == 0
    scale = force_scale(f_or[fluid_g])
    err = np.abs(f_gpu - f_or).max(axis=1)
    say("  max |df| / F_scale %.3g" % (err[fluid_g].max() / scale))
    assert err[fluid_g].max() <= FORCE_TOL * scale
    assert np.all(f_gpu[~fluid_g] == 0)
    st = {k: v.cpu().numpy() for k, v in sim.state().items()}
    assert np.array_equal(st["cell_of"], by_gid(o, o.cells()))
    assert np.array_equal(sorted_pairs(sim.pairs()), sorted_pairs(o.pairs()))
    sim.close()


@pytest.mark.parametrize("kernel", KERNELS, indirect=True)
@pytest.mark.parametrize("name", ["slab_f64grid", "curved", "stress", "dense"])
def test_one_step(dpd, oracle_lib, kernel, name):
    s = SYSTEMS[name]()
    say("one step", kernel, name, s.n)
    n_ev = _one_step_compare(dpd, oracle_lib, s)
    if name == "stress":
        assert n_ev >= 60


@pytest.mark.parametrize("kernel", ["bricks"], indirect=True)
def test_brick_sums_are_order_free(dpd, kernel):
    """Mask on and off and a repeated run: identical bits after 40 steps;
    the same box alone and as box 1 of a batch: identical bits after 20."""
    s = _stress_system(seed=72, vscale=3.0)
    a = dpd.Simulation(s)
    b = dpd.Simulation(s, flags=1)
    c = dpd.Simulation(s)
    for sim in (a, b, c):
        sim.step(40)
    for k in ("pos", "vel", "events"):
        va = a.state()[k].cpu().numpy()
        assert np.array_equal(va, b.state()[k].cpu().numpy()), k
        assert np.array_equal(va, c.state()[k].cpu().numpy()), k
    for sim in (a, b, c):
        sim.close()
    other = workloads.slab_system(seed_fluid=5, seed_wall=6, grid_dtype=np.float32,
                                  params=workloads.default_params(seed=5))
    s2 = _small_curved_box()
    alone = dpd.Simulation(s2)
    batch = dpd.Simulation([other, s2])
    alone.step(20)
    batch.step(20)
    for k in ("pos", "vel", "events"):
        assert np.array_equal(alone.state()[k].cpu().numpy(), batch.state(1)[k].cpu().numpy()), k
    assert np.array_equal(alone.forces().cpu().numpy(), batch.forces(1).cpu().numpy())
    alone.close()
    batch.close()


def _small_curved_box():
    return workloads.sinusoid_cylinder_system(L=(16.0, 5.0, 24.0), base=3.0, amp=1.5, radius=3.0,
                                              seed=31,
                                              params=workloads.default_params(g=(0.01, 0, 0), seed=31))


@pytest.mark.parametrize("kernel", KERNELS, indirect=True)
def test_kernels_agree_on_a_long_run(dpd, kernel):
    """Both kernels keep every fluid particle at phi >= 0 and conserve the
    momentum balance over 300 steps of the stress box (a smoke test of the
    whole step with each kernel; their trajectories differ by rounding)."""
    s = _stress_system(seed=74, vscale=2.0)
    sim = dpd.Simulation(s)
    sim.step(300)
    sim.sync()
    c = sim.counters()
    assert c["unstable"] == 0 and c["bounce"] > 0
    sim.close()
