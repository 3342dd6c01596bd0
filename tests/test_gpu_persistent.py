"""The persistent step (one launch per step, per-box arrival counters) against
the per-phase launches, through the C ABI.

Bars: bit-identical state, events, cells and forces after 30 steps, for a
batch of seven uneven boxes (direct launches and graph replay, and with the
attractive-repulsive force), for a single box with a float64 phase field,
for boxes whose cells span several scan chunks, and after switching back
and forth mid-run; one timed launch per step; the
contexts it does not serve (moving walls, the brick pair kernel) refused.
"""
import sys

import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu
from test_gpu_batch import _small_batch, _snap

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


def _same(a, b, what):
    for k in ("pos", "vel", "events", "cell_of", "force"):
        assert np.array_equal(a[k], b[k]), (what, k)


def _compare(dpd, boxes, steps, graph, label):
    ref = dpd.Simulation(boxes)
    per = dpd.Simulation(boxes, graph=graph)
    per.use_persistent(True)
    ref.step(steps)
    per.step(steps)
    for r in range(len(boxes)):
        _same(_snap(per, r), _snap(ref, r), (label, r))
    cr, cp = ref.counters(), per.counters()
    say(label, "counters", cp)
    for k in ("bounce", "fallback", "unstable", "k", "steps"):
        assert cr[k] == cp[k], (label, k)
    ref.close()
    per.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_per_phase_launches(dpd, graph):
    boxes = _small_batch()
    say("persistent batch of", len(boxes), "boxes:", [b.n for b in boxes], "graph", graph)
    _compare(dpd, boxes, 30, graph, "batch graph=%s" % graph)


def _sph_slab(r):
    s = workloads.slab_system(seed_fluid=60 + r, seed_wall=70 + r, grid_dtype=np.float32,
                              params=workloads.default_params(seed=80 + r, replica=r))
    p = dict(s.params)
    p["sph"] = workloads.sph_force()
    p["kBT"] = 0.5
    p["dt"] = 0.005
    s.params = p
    return s


def test_attractive_repulsive_batch(dpd):
    boxes = [_sph_slab(r) for r in range(3)]
    say("persistent SPH batch", [b.n for b in boxes])
    _compare(dpd, boxes, 20, False, "sph")


def test_single_box_float64_grid_and_switching(dpd):
    s = workloads.slab_system(seed_fluid=11, seed_wall=12,
                              params=workloads.default_params(g=(0.02, 0, 0), seed=13))
    say("single box", s.n, s.phi.dtype)
    _compare(dpd, [s], 25, False, "slab f64")
    ref = dpd.Simulation(s)
    mix = dpd.Simulation(s)
    ref.step(30)
    mix.step(10)
    mix.use_persistent(True)
    mix.step(10)
    mix.use_persistent(False)
    mix.step(10)
    _same(_snap(mix, 0), _snap(ref, 0), "switching")
    ref.close()
    mix.close()


def test_boxes_with_several_scan_chunks(dpd):
    """Boxes of more than one scan chunk (4096 cells): a 24 x 16 x 24 curved
    box (9216 cells, three chunks) alone and in a batch after a small box,
    so chunk offsets inside a box and box offsets both enter the scan."""
    big = workloads.sinusoid_cylinder_system(
        L=(24.0, 16.0, 24.0), base=3.0, amp=1.5, radius=3.0, seed=77,
        params=workloads.default_params(g=(0.02, 0, 0), seed=78, replica=1))
    small = workloads.slab_system(seed_fluid=79, seed_wall=80, grid_dtype=np.float32,
                                  params=workloads.default_params(seed=81))
    say("multi-chunk boxes", big.n, small.n)
    _compare(dpd, [big], 15, False, "one box, three chunks")
    _compare(dpd, [small, big], 15, True, "batch with a three-chunk box")


def test_one_timed_launch_per_step(dpd):
    boxes = _small_batch()
    sim = dpd.Simulation(boxes)
    sim.use_persistent(True)
    sim.kernel_times(1)
    sim.step(6)
    kt = sim.kernel_times(0)
    say("kernel times", kt)
    assert kt["step_persistent"][1] == 6
    for k in ("integrate_reflect_bin", "scan_reduce", "scan_down", "scatter", "sort_cells",
              "pair_codes", "pair_force"):
        assert kt[k][1] == 0, k
    sim.close()


def test_refused_where_not_served(dpd, monkeypatch):
    from paper_1807_09896_amd.binding import DPDError
    couette = workloads.couette_system(L=(8.0, 6.0, 7.0), seed=3)
    sim = dpd.Simulation(couette)
    with pytest.raises(DPDError):
        sim.use_persistent(True)
    sim.step(2)
    sim.close()
    monkeypatch.setenv("DPD_PAIR_KERNEL", "bricks")
    s = workloads.slab_system(seed_fluid=21, seed_wall=22, grid_dtype=np.float32,
                              params=workloads.default_params(seed=23))
    sim = dpd.Simulation(s)
    with pytest.raises(DPDError):
        sim.use_persistent(True)
    sim.close()
