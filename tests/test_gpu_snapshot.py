"""Snapshots (checkpoint and restart) through the C ABI.

Bars: a batch holding a resting-wall box, a box with a sliding plate and a
box with the attractive-repulsive force, stepped under graph replay,
snapshotted and stepped on, gives bit for bit the same positions,
velocities, event codes, forces and counters as a fresh context restored
from the snapshot and as the same context rewound to it; restoring into a
context of another layout or with other wall particles, or from a blob
that is not a snapshot, fails with DPD_E_INVAL and leaves the context as
it was.
"""
import sys

import numpy as np
import pytest

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


def _boxes():
    slab = workloads.tiny_slab_system()
    slab.vel = (slab.vel * 3).astype(np.float32)
    couette = workloads.couette_system(U=1.0, seed=92)
    sph = workloads.tiny_slab_system(seed=14)
    p = dict(sph.params)
    p["sph"] = workloads.sph_force()
    p["kBT"] = 0.5
    p["dt"] = 0.005
    sph.params = p
    return [slab, couette, sph]


def _state(sim, R):
    out = []
    for r in range(R):
        st = {k: v.cpu().numpy() for k, v in sim.state(r).items()}
        st["force"] = sim.forces(r).cpu().numpy()
        out.append(st)
    c = sim.counters()
    return out, (c["steps"], c["k"], c["bounce"], c["fallback"])


def _same(a, b, what):
    for r, (x, y) in enumerate(zip(a[0], b[0])):
        for k in ("pos", "vel", "events", "cell_of", "force"):
            assert np.array_equal(x[k], y[k]), (what, r, k)
    assert a[1] == b[1], (what, a[1], b[1])


def test_restart_is_bit_identical(dpd):
    boxes = _boxes()
    a = dpd.Simulation(boxes, graph=True)
    a.step(23)
    blob = a.snapshot()
    say("snapshot bytes", blob.nbytes)
    a.step(17)
    ref = _state(a, 3)
    assert ref[1][2] > 0
    b = dpd.Simulation(boxes, graph=True)
    b.step(3)                       # some other state, to be overwritten
    b.restore(blob)
    b.step(17)
    _same(_state(b, 3), ref, "fresh context")
    b.close()
    a.restore(blob)
    a.step(17)
    _same(_state(a, 3), ref, "rewound")
    a.close()


def test_restore_rejects_other_contexts(dpd):
    boxes = _boxes()
    a = dpd.Simulation(boxes)
    a.step(5)
    blob = a.snapshot()
    a.close()
    # other layout: fewer boxes
    c = dpd.Simulation(boxes[:2])
    c.step(2)
    before = _state(c, 2)
    with pytest.raises(dpd.DPDError):
        c.restore(np.resize(blob, c.snapshot().nbytes))
    _same(_state(c, 2), before, "after a rejected restore")
    c.close()
    # same counts, other resting walls
    moved = _boxes()
    s0 = moved[0]
    pos = s0.pos.copy()
    walls = s0.type != 0
    pos[walls, 0] = np.mod(pos[walls, 0] + np.float32(0.125), np.float32(s0.L[0])).astype(np.float32)
    s0.pos = pos
    d = dpd.Simulation([moved[0]])
    e = dpd.Simulation([boxes[0]])
    e.step(3)
    blob_e = e.snapshot()
    e.close()
    with pytest.raises(dpd.DPDError):
        d.restore(blob_e)
    # not a snapshot
    junk = np.zeros_like(blob_e)
    with pytest.raises(dpd.DPDError):
        d.restore(junk)
    d.close()
