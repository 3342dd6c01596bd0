"""Batched boxes, HIP-graph replay and the launch-shape autotuner, through
the C ABI, against the plain single-box path and the oracle.

Bars: box r of a batch is bit-identical to the same box run alone (same
replica id) in state, events, forces and pair sets; graph replay is
bit-identical to direct launches; every launch shape gives the same bits;
a sampled box of the full 256-replica batch meets the oracle's one-step bar.
"""
import os
import sys

import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu, sorted_pairs
from test_gpu_parity import _one_step_compare, _stress_system

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


def _small_batch():
    """Seven boxes of uneven size: five replica-generator boxes (slit,
    cylinder, sphere pack), the bounce-back stress slab and a wall-free
    periodic box, all with float32 phase fields."""
    reps = workloads.replica_systems(count=5, seed=40, edge_range=(6.0, 10.0), threads=1)
    stress = _stress_system(seed=72)
    bulk = workloads.bulk_system(L=(5.0, 4.0, 3.0),
                                 params=workloads.default_params(seed=8, replica=9))
    return reps + [stress, bulk]


def _snap(sim, r):
    st = {k: v.cpu().numpy() for k, v in sim.state(r).items()}
    st["force"] = sim.forces(r).cpu().numpy()
    return st


def _assert_same(a, b, what):
    for k in ("pos", "vel", "events", "cell_of", "force"):
        assert np.array_equal(a[k], b[k]), (what, k)


def test_batch_box_equals_box_alone(dpd):
    boxes = _small_batch()
    say("batch of", len(boxes), "boxes:", [b.n for b in boxes])
    batch = dpd.Simulation(boxes)
    assert dpd.dpd_replica_count(batch.ctx) == len(boxes)
    for r, b in enumerate(boxes):
        alone = dpd.Simulation(b)
        _assert_same(_snap(batch, r), _snap(alone, r=0), ("initial", r))
        alone.close()
    batch.step(30)
    bounce = 0
    for r, b in enumerate(boxes):
        alone = dpd.Simulation(b)
        alone.step(30)
        _assert_same(_snap(batch, r), _snap(alone, 0), ("30 steps", r))
        assert np.array_equal(sorted_pairs(batch.pairs(r)), sorted_pairs(alone.pairs()))
        p_b = batch.profile(axis=2, nbins=8, r=r).cpu().numpy()
        p_a = alone.profile(axis=2, nbins=8).cpu().numpy()
        assert np.array_equal(p_b[:, 0], p_a[:, 0])
        assert np.allclose(p_b, p_a, rtol=1e-12, atol=1e-9)
        bounce += alone.counters()["bounce"]
        alone.close()
    c = batch.counters()
    say("batch counters", c)
    assert c["bounce"] == bounce and bounce > 0
    assert c["n_fluid"] == sum(b.n_fluid for b in boxes)
    assert c["unstable"] == 0
    batch.close()


def test_wide_box_tile_order_keeps_bits(dpd):
    """A box more than 56 cell rows wide in y takes its pair-kernel tiles in
    y-bands when it is its context's only box, and in plain order inside a
    batch; the order must not change a bit of the results."""
    wide = workloads.slab_system(L=(16.0, 64.0, 6.0), grid_dtype=np.float32, seed_fluid=61,
                                 seed_wall=62)
    bulk = workloads.bulk_system(L=(5.0, 4.0, 3.0),
                                 params=workloads.default_params(seed=8, replica=9))
    say("wide slab", wide.n, "particles")
    alone = dpd.Simulation(wide)
    batch = dpd.Simulation([wide, bulk])
    alone.step(20)
    batch.step(20)
    _assert_same(_snap(batch, 0), _snap(alone, 0), "20 steps")
    assert np.array_equal(sorted_pairs(batch.pairs(0)), sorted_pairs(alone.pairs()))
    assert alone.counters()["unstable"] == 0
    alone.close()
    batch.close()


def test_replica_id_enters_random_numbers(dpd):
    s = workloads.tiny_slab_system()
    s0 = workloads.tiny_slab_system()
    s1 = workloads.tiny_slab_system()
    s1.params = dict(s1.params, replica=1)
    batch = dpd.Simulation([s, s0, s1])
    batch.step(5)
    a, b, c = _snap(batch, 0), _snap(batch, 1), _snap(batch, 2)
    _assert_same(a, b, "same replica id")
    assert not np.array_equal(a["vel"], c["vel"])
    batch.close()


def test_graph_replay_equals_direct_launches(dpd):
    boxes = _small_batch()
    direct = dpd.Simulation(boxes)
    graph = dpd.Simulation(boxes, graph=True)
    direct.step(25)
    graph.step(25)
    assert graph.counters()["k"] == 25
    for r in range(len(boxes)):
        _assert_same(_snap(graph, r), _snap(direct, r), ("graph", r))
    # set_state drops the captured graph; the next replay starts from it
    st = _snap(direct, 3)
    for sim in (direct, graph):
        sim.set_state(st["pos"], st["vel"], st["force"], 7, r=3)
        sim.step(6)
    for r in range(len(boxes)):
        _assert_same(_snap(graph, r), _snap(direct, r), ("graph after set_state", r))
    assert graph.counters()["k"] == 13
    direct.close()
    graph.close()


def test_autotune_keeps_state_and_every_shape_agrees(dpd, tmp_path):
    boxes = _small_batch()
    ref = dpd.Simulation(boxes)
    ref.step(12)
    want = [_snap(ref, r) for r in range(len(boxes))]
    cache = tmp_path / "tune.txt"
    os.environ["DPD_TUNE_CACHE"] = str(cache)
    try:
        sim = dpd.Simulation(boxes)
        sim.step(2)
        before = [_snap(sim, r) for r in range(len(boxes))]
        c0 = sim.counters()
        shape, ms = sim.autotune(3)
        say("autotune", shape, ms)
        assert shape in [(2, 256), (1, 256), (2, 128), (1, 128)]
        assert all(t > 0 for t in ms)
        c1 = sim.counters()
        assert (c1["k"], c1["steps"], c1["bounce"]) == (c0["k"], c0["steps"], c0["bounce"])
        for r in range(len(boxes)):
            _assert_same(_snap(sim, r), before[r], ("restored", r))
        sim.step(10)
        for r in range(len(boxes)):
            _assert_same(_snap(sim, r), want[r], ("tuned", r))
        sim.close()
        line = cache.read_text().split()
        assert len(line) == 3 and (int(line[1]), int(line[2])) == shape
        sig = line[0]
        # each shape, forced through the cache, gives the same bits
        for ppt, blk in [(2, 256), (1, 256), (2, 128), (1, 128)]:
            cache.write_text("%s %d %d\n" % (sig, ppt, blk))
            sim = dpd.Simulation(boxes)
            got, ms = sim.autotune(1)
            assert got == (ppt, blk) and ms == [-1.0] * 4
            sim.step(12)
            for r in range(len(boxes)):
                _assert_same(_snap(sim, r), want[r], ("shape", ppt, blk, r))
            sim.close()
    finally:
        del os.environ["DPD_TUNE_CACHE"]
    ref.close()


def test_full_batch_sampled_boxes(dpd, oracle_lib):
    """The 256-replica workload in the benchmarked configuration (graph
    replay, autotuned shapes): sampled boxes against the same box alone
    (bit-exact) and one step of the largest against the oracle."""
    boxes = workloads.replica_systems()
    ns = np.array([b.n for b in boxes])
    say("256 replicas: %d particles, %d..%d per box" % (ns.sum(), ns.min(), ns.max()))
    batch = dpd.Simulation(boxes, graph=True)
    shape, ms = batch.autotune(2)
    say("autotune", shape, ms)
    batch.step(20)
    kinds = [b.meta["kind"] for b in boxes]
    sample = sorted({int(ns.argmin()), int(ns.argmax()), kinds.index("spheres"),
                     kinds.index("slit"), kinds.index("cylinder"), len(boxes) - 1})
    for r in sample:
        alone = dpd.Simulation(boxes[r])
        alone.step(20)
        _assert_same(_snap(batch, r), _snap(alone, 0), ("box", r))
        alone.close()
    c = batch.counters()
    say("counters", c)
    assert c["unstable"] == 0
    # one step of the largest box against the oracle: the oracle runs its own
    # 20 steps, its FP32 state is loaded into that box of the batch, and the
    # whole batch (graph replay, tuned shapes) steps once
    r = int(ns.argmax())
    say("oracle one-step on box", r, boxes[r].n)
    _one_step_compare(dpd, oracle_lib, boxes[r], nsteps_before=20, sim=batch, r=r)
    batch.close()
