"""The allocation-free phase-field relaxation (dpd_phi_relax_static) against
dpd_phi_relax with a caller workspace, through the C ABI.

The two run the same kernels, so their results must agree bit for bit:
every node and the residual, in float32 and float64, on two calls in a row
where the second relaxes a smaller grid (the static scratch keeps the first
call's contents), with even and odd step counts (the odd count ends with a
copy out of the scratch).  A grid beyond the scratch's 64 MiB is rejected
with DPD_E_INVAL and leaves phi untouched.
"""
import sys

import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu

EPS = 0.5 / np.sqrt(2.0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dpd():
    require_gpu()
    import paper_1807_09896_amd as dpd
    dpd.load_library()
    return dpd


def _dtau(h):
    return 0.5 / (2.0 * sum((EPS / x) ** 2 for x in h))


def _pair(dpd, phi0, h, iters, td):
    import torch
    from paper_1807_09896_amd import binding
    a = torch.tensor(phi0, dtype=td, device="cuda")
    b = a.clone()
    work = torch.empty(a.numel() + 1, dtype=td, device="cuda")
    ra = binding.dpd_phi_relax(a, work, h, EPS, _dtau(h), iters, residual=True)
    rb = binding.dpd_phi_relax_static(b, h, EPS, _dtau(h), iters, residual=True)
    torch.cuda.synchronize()
    return a.cpu().numpy(), ra, b.cpu().numpy(), rb


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_static_scratch_matches_workspace_twice(dpd, dtype):
    import torch
    td = torch.float32 if dtype == "f32" else torch.float64
    cases = [((96, 40, 72), (0.25, 0.25, 0.25), 6, 300),    # first call: larger grid
             ((33, 17, 20), (0.2, 0.3, 0.25), 5, 301)]      # second call: smaller, odd steps
    for n, h, iters, seed in cases:
        say("static scratch", dtype, "grid", n, "steps", iters)
        phi0 = workloads.step_phase_field(n, h, seed=seed)
        a, ra, b, rb = _pair(dpd, phi0, h, iters, td)
        assert a.dtype == b.dtype
        assert np.array_equal(a, b), (n, float(np.abs(a - b).max()))
        assert ra == rb, (ra, rb)
        assert ra > 0.0


def test_static_scratch_rejects_grids_beyond_its_size(dpd):
    import torch
    from paper_1807_09896_amd import binding
    # 257 x 256 x 256 float32 nodes is just over 64 MiB
    phi = torch.ones((256, 256, 257), dtype=torch.float32, device="cuda")
    with pytest.raises(binding.DPDError) as e:
        binding.dpd_phi_relax_static(phi, (0.25, 0.25, 0.25), EPS, _dtau((0.25,) * 3), 2)
    assert e.value.code == binding.DPD_E_INVAL
    assert "scratch" in str(e.value)
    assert bool((phi == 1).all())
    # the largest allowed float64 grid still runs (8,388,608 nodes)
    big = torch.ones((128, 256, 256), dtype=torch.float64, device="cuda")
    r = binding.dpd_phi_relax_static(big, (0.25, 0.25, 0.25), EPS, _dtau((0.25,) * 3), 1)
    torch.cuda.synchronize()
    assert r == 0.0 and bool((big == 1).all())
