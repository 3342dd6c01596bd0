"""Contexts and the phase-field relaxation on a stream other than the
default one: the same bits as on the default stream (direct launches and
graph replay), with the caller ordering its own streams as torch code
does."""
import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpd():
    require_gpu()
    import paper_1807_09896_amd as dpd
    dpd.load_library()
    return dpd


def _snap(sim):
    st = {k: v.cpu().numpy() for k, v in sim.state().items()}
    st["force"] = sim.forces().cpu().numpy()
    return st


def test_steps_on_a_side_stream(dpd):
    import torch
    s = workloads.couette_system(U=1.0, seed=93)
    ref = dpd.Simulation(s)
    ref.step(30)
    want = _snap(ref)
    ref.close()
    side = torch.cuda.Stream()
    for graph in (False, True):
        sim = dpd.Simulation(s, stream=side, graph=graph)
        sim.step(30)
        got = _snap(sim)
        for k in ("pos", "vel", "events", "cell_of", "force"):
            assert np.array_equal(got[k], want[k]), (graph, k)
        sim.close()


def test_phase_field_relaxation_on_a_side_stream(dpd):
    import torch
    h = (0.25, 0.25, 0.25)
    phi0 = torch.tensor(workloads.step_phase_field((66, 20, 40), h, seed=8),
                        dtype=torch.float32, device="cuda")
    eps = 0.5 / np.sqrt(2.0)
    dtau = 0.02
    a = phi0.clone()
    dpd.relax_phi(a, h, eps, dtau, 7)
    b = phi0.clone()
    work = torch.empty(b.numel() + 1, dtype=b.dtype, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    dpd.dpd_phi_relax(b, work, h, eps, dtau, 7, residual=False, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    assert torch.equal(a, b)
