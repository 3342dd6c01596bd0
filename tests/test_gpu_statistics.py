"""Long-run statistical parity of the GPU path with the oracle (Sec. III.A's
binned velocity and density profiles).

Both sides start from the same seeded states and run the same number of
steps; their trajectories decorrelate within about a hundred steps (the
dynamics is chaotic and the two round differently), so only statistics
can agree.  Each replica's profile (mean v_x and number of particles per
bin along z, averaged over samples every 10 steps after a transient) is
one sample.  Replicas are independent, so the standard error of a bin's
mean is the spread over replicas / sqrt(R) (blocks of one replica each).

Bar, per bin of both profiles: |GPU - oracle| <= 3 sqrt(SE_g^2 + SE_o^2).
Because a fixed seed set makes the outcome deterministic, a failure is
reproducible; the joint statistic chi^2 = sum over bins of
(GPU - oracle)^2 / (SE_g^2 + SE_o^2) must also stay below the 0.999
quantile of the chi-square distribution with as many degrees of freedom
(bins x 2), which catches a small shift common to many bins.

Workloads:
- the plane channel (10^3, walls 1.5 thick, density 3, g_x = 0.02,
  FP64 phase field) over the full 1000 steps, sampled from step 200 on, 16
  replicas;
- the geometry of the sinusoidal channel with a cylinder at a size the
  oracle runs in seconds: a 20 x 4 x 24 box, walls z = 3 + 1.5 sin(2 pi x /
  20) mirrored at the top, a cylinder of radius 3 along y at the centre,
  density 3, g_x = 0.02, 1000 steps sampled from step 200 on, 8 replicas.
"""
import math
import sys

import numpy as np
import pytest
from scipy import stats

import workloads
from gpu_helpers import require_gpu

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


def _profiles(dpd, oracle_lib, systems, steps, start, every, zlo, zhi, nb):
    """Per replica: binned mean v_x and mean count per bin over the samples
    at steps start + every, ..., steps, on the GPU (one batch of all
    replicas) and in the oracle."""
    R = len(systems)
    width = (zhi - zlo) / nb

    def bins(z, vx):
        b = np.clip(np.floor((z - zlo) / width).astype(int), 0, nb - 1)
        ok = (z >= zlo) & (z < zhi)
        return (np.bincount(b[ok], minlength=nb), np.bincount(b[ok], weights=vx[ok], minlength=nb))

    nsamp = (steps - start) // every
    cg = np.zeros((R, nb)); vg = np.zeros((R, nb))
    sim = dpd.Simulation(systems)
    sim.step(start)
    gids = [s.gid[s.type == 0] for s in systems]
    for _ in range(nsamp):
        sim.step(every)
        for r, s in enumerate(systems):
            st = sim.state(r)
            p = st["pos"].cpu().numpy()[gids[r]]
            v = st["vel"].cpu().numpy()[gids[r]]
            c, w = bins(p[:, 2].astype(np.float64), v[:, 0].astype(np.float64))
            cg[r] += c; vg[r] += w
    assert sim.counters()["unstable"] == 0
    sim.close()
    co = np.zeros((R, nb)); vo = np.zeros((R, nb))
    for r, s in enumerate(systems):
        o = oracle_lib.Oracle(s)
        fl = s.type == 0
        o.step(start)
        for _ in range(nsamp):
            o.step(every)
            c, w = bins(np.mod(o.r[fl, 2], s.L[2]), o.v[fl, 0])
            co[r] += c; vo[r] += w
    prof_g = np.concatenate([vg / np.maximum(cg, 1), cg / nsamp], axis=1)
    prof_o = np.concatenate([vo / np.maximum(co, 1), co / nsamp], axis=1)
    return prof_g, prof_o


def _check(prof_g, prof_o, label, min_count=5.0):
    """Bins where every replica on both sides holds at least min_count
    particles per sample on average (bins inside a solid hold none)."""
    R, nb2 = prof_g.shape
    nb = nb2 // 2
    full = (prof_g[:, nb:].min(0) >= min_count) & (prof_o[:, nb:].min(0) >= min_count)
    use = np.concatenate([full, full])
    mg, mo = prof_g.mean(0)[use], prof_o.mean(0)[use]
    se2 = prof_g.var(0, ddof=1)[use] / R + prof_o.var(0, ddof=1)[use] / R
    dev = np.abs(mg - mo) / np.sqrt(se2)
    chi2 = float(((mg - mo) ** 2 / se2).sum())
    limit = stats.chi2.ppf(0.999, df=mg.size)
    k = int(full.sum())
    say("%s: %d of %d bins hold fluid" % (label, k, nb))
    say("%s: |d| / SE per bin, v_x:" % label, np.round(dev[:k], 2))
    say("%s: |d| / SE per bin, count:" % label, np.round(dev[k:], 2))
    say("%s: chi2 %.1f (limit %.1f, %d bins)" % (label, chi2, limit, mg.size))
    assert k >= nb // 2
    assert np.all(dev <= 3.0), (label, float(dev.max()))
    assert chi2 < limit


def test_plane_channel_1000_steps(dpd, oracle_lib):
    systems = [workloads.slab_system(seed_fluid=100 + r, seed_wall=200 + r,
                                     params=workloads.default_params(g=(0.02, 0, 0), seed=300 + r))
               for r in range(16)]
    say("plane channel: %d replicas of %d particles" % (len(systems), systems[0].n))
    pg, po = _profiles(dpd, oracle_lib, systems, steps=1000, start=200, every=10, zlo=1.5,
                       zhi=8.5, nb=10)
    _check(pg, po, "plane channel")


def _curved(r):
    return workloads.sinusoid_cylinder_system(
        L=(20.0, 4.0, 24.0), base=3.0, amp=1.5, radius=3.0, seed=500 + r,
        params=workloads.default_params(g=(0.02, 0, 0), seed=600 + r))


def test_sinusoid_and_cylinder_1000_steps(dpd, oracle_lib):
    systems = [_curved(r) for r in range(8)]
    say("sinusoid + cylinder: %d replicas of ~%d particles" % (len(systems), systems[0].n))
    pg, po = _profiles(dpd, oracle_lib, systems, steps=1000, start=200, every=10, zlo=0.0,
                       zhi=24.0, nb=12)
    _check(pg, po, "sinusoid + cylinder")
