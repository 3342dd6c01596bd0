"""Stokes flow through a square array of cylinders (Sec. III.B) on the GPU.

Bars: one step on the cylinder-array workload against the oracle at the
standard one-step bar; the viscosity from plane Poiseuille flow (Eq. 19) at
Sec. III.A's low-temperature parameters, then the normalised mean fluid
velocity through arrays of solid fraction 0.05, 0.1 and 0.2 within 15 % of
Eq. 20 (the square-array series, for the two small fractions where it
holds) and of Eq. 21 (the paper's fit of its own DPD results, all three).
The flows run at Reynolds numbers near 1 in batches of 8 independent
replicas; the statistical error of each mean (standard error over the
replicas) must stay below 5 %, so that three standard errors fit inside
the 15 % band, which is the model difference (a 3-D slab here, 2-D in the
paper, and the position of the effective no-slip surface inside the
diffuse interface).  Measured standard errors: 0.5 % (Poiseuille), 0.9 %,
0.7 % and 3.3 % (c = 0.05, 0.1, 0.2).  Measured: 0.95 and 1.07 of Eq. 20
at 0.05 and 0.1; 0.92, 0.96 and 0.93 of Eq. 21.
"""
import math
import sys

import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu
from stokes_forms import eq19_viscosity, eq20, eq21
from test_gpu_parity import _one_step_compare

pytestmark = pytest.mark.gpu

REPLICAS = 8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dpd():
    require_gpu()
    import paper_1807_09896_amd as dpd
    dpd.load_library()
    return dpd


def test_one_step_parity(dpd, oracle_lib):
    s = workloads.cylinder_array_system(solid_fraction=0.1, seed=70)
    s.vel = (s.vel * 4).astype(np.float32)   # hot: reflections off the cylinder in one step
    say("cylinder array", s.n)
    n_ev = _one_step_compare(dpd, oracle_lib, s)
    say("events", n_ev)


def _mean_fluid_vx(dpd, systems, warm, blocks, per, every=20):
    """Per-replica mean fluid x velocity over `blocks` x `per` steps after
    `warm`; returns the grand mean and its standard error over replicas."""
    sim = dpd.Simulation(systems, graph=True)
    sim.step(warm)
    R = len(systems)
    acc = np.zeros((R, 2))
    for _ in range(blocks * per // every):
        sim.step(every)
        for r in range(R):
            p = sim.profile(axis=2, nbins=1, r=r).cpu().numpy()[0]
            acc[r] += p[:2]
    c = sim.counters()
    sim.close()
    assert c["unstable"] == 0
    v = acc[:, 1] / acc[:, 0]
    return v.mean(), v.std(ddof=1) / math.sqrt(R)


def test_cylinder_array_mean_velocity(dpd):
    dt = 0.01
    # viscosity from plane Poiseuille flow, channel 10 wide (Sec. III.A)
    gp = 0.004
    slabs = [workloads.slab_system(L=(12.0, 12.0, 13.0), wall=1.5, rho=4.0, seed_fluid=100 + 2 * k,
                                   seed_wall=101 + 2 * k,
                                   params=workloads.stokes_params(g=gp, dt=dt, seed=200 + k))
             for k in range(REPLICAS)]
    a = (slabs[0].meta["hi"] - slabs[0].meta["lo"]) / 2
    rho = np.mean([s.n_fluid for s in slabs]) / (slabs[0].L[0] * slabs[0].L[1] * 2 * a)
    v, se = _mean_fluid_vx(dpd, slabs, 15000, 10, 2000)
    mu = eq19_viscosity(rho, gp, a, v)
    say("Poiseuille: vbar %.5f +- %.5f, mu %.4f, Re %.2f" % (v, se, mu, rho * v * 2 * a / mu))
    assert se < 0.05 * v
    gc = 0.001
    for c in (0.05, 0.1, 0.2):
        cells = [workloads.cylinder_array_system(solid_fraction=c, seed=300 + k,
                                                 params=workloads.stokes_params(g=gc, dt=dt, seed=400 + k))
                 for k in range(REPLICAS)]
        L, r = cells[0].meta["cell"], cells[0].meta["radius"]
        rho_c = np.mean([s.n_fluid for s in cells]) / ((L * L - math.pi * r * r) * cells[0].L[2])
        v, se = _mean_fluid_vx(dpd, cells, 20000, 10, 2000)
        u = 4 * math.pi * v * mu / (rho_c * gc * L * L)
        say("c %.2f: u %.4f +- %.4f, Eq. 20 %.4f (ratio %.3f), Eq. 21 %.4f (ratio %.3f)" % (
            c, u, u * se / v, eq20(c), u / eq20(c), eq21(c), u / eq21(c)))
        assert se < 0.05 * v
        if c <= 0.1:
            assert abs(u / eq20(c) - 1) < 0.15
        assert abs(u / eq21(c) - 1) < 0.15
