"""Phase-field relaxation (Eq. 15) on the GPU, through the C ABI.

Bars: after up to 25 explicit Euler steps from seeded step functions, every
node within 1e-5 of the FP64 oracle in float32 and within 1e-12 in float64,
and the reported residual (max |d phi / d t'| of the last step) within
1e-5 / 1e-12 relative.  The tolerances are the unit roundoff (6e-8, 1.1e-16)
times the amplification of input rounding by the relaxation itself, which
the CPU tests bound by 100 for these inputs, with margin.  Shapes span several 64 x 16 x 64 tiles with ragged
ends, and degenerate grids (one node wide, 1 x 2 x 3); zero, odd and even
step counts; invalid arguments rejected; a sphere keeps its radius over a
long relaxation (the counter term); at the size of the porous workload's
grid (672^3), one step on sampled nodes against the oracle evaluated on
each node's periodic neighbourhood.
"""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu
from oracle import phase_field as pf
from pf_cases import CASES, case_input

pytestmark = pytest.mark.gpu

EPS = 0.5 / np.sqrt(2.0)
TOL = {4: 1e-5, 8: 1e-12}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dpd():
    require_gpu()
    import paper_1807_09896_amd as dpd
    dpd.load_library()
    return dpd


def _gpu_relax(dpd, phi0, h, dtau, iters, dtype):
    import torch
    td = torch.float32 if dtype == 4 else torch.float64
    phi = torch.tensor(phi0, dtype=td, device="cuda")
    work = torch.empty(phi.numel() + 1, dtype=td, device="cuda")
    res = dpd.dpd_phi_relax(phi, work, h, EPS, dtau, iters)
    return phi.cpu().numpy().astype(np.float64), res


@pytest.mark.parametrize("dtype", [4, 8], ids=["f32", "f64"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_parity_with_oracle(dpd, case, dtype):
    phi0, h, iters = case_input(case)
    dtau = 0.5 * pf.max_stable_dtau(h, EPS)
    say("relax", phi0.shape, "dtype", dtype, "steps", iters)
    ref, rres = pf.relax(phi0, h, EPS, dtau, iters)
    out, res = _gpu_relax(dpd, phi0, h, dtau, iters, dtype)
    err = np.abs(out - ref).max()
    say("max err %.3e  residual %.8e vs %.8e" % (err, res, rres))
    assert err <= TOL[dtype]
    assert abs(res - rres) <= TOL[dtype] * max(rres, 1.0)


@pytest.mark.parametrize("iters", [0, 1, 2, 3])
def test_step_counts(dpd, iters):
    """The result lands in phi for odd and even counts (ping-pong buffer);
    zero steps leave phi as it was with residual 0."""
    h = (0.25, 0.25, 0.25)
    phi0 = workloads.step_phase_field((66, 12, 20), h, seed=7)
    dtau = 0.5 * pf.max_stable_dtau(h, EPS)
    ref, rres = pf.relax(phi0, h, EPS, dtau, iters)
    out, res = _gpu_relax(dpd, phi0, h, dtau, iters, 8)
    assert np.abs(out - ref).max() <= 1e-12
    assert abs(res - rres) <= 1e-12 * max(rres, 1.0)
    if iters == 0:
        assert np.array_equal(out, phi0) and res == 0.0


def test_invalid_arguments(dpd):
    import torch
    from paper_1807_09896_amd import binding
    L = dpd.load_library()
    h = (0.25, 0.25, 0.25)
    phi = torch.ones((4, 4, 4), dtype=torch.float32, device="cuda")
    work = torch.empty(65, dtype=torch.float32, device="cuda")
    lim = pf.max_stable_dtau(h, EPS)
    with pytest.raises(dpd.DPDError):
        dpd.dpd_phi_relax(phi, work, h, EPS, 1.01 * lim, 1)
    with pytest.raises(dpd.DPDError):
        dpd.dpd_phi_relax(phi, work, h, -EPS, 0.01, 1)
    with pytest.raises(dpd.DPDError):
        dpd.dpd_phi_relax(phi, work, h, EPS, 0.01, -1)
    with pytest.raises(ValueError):
        dpd.dpd_phi_relax(phi, work[:64], h, EPS, 0.01, 1)
    hh = (C.c_double * 3)(*h)
    for n in ((0, 4, 4), (4, -1, 4)):
        nn = (C.c_int32 * 3)(*n)
        assert L.dpd_phi_relax(binding._ptr(phi), binding._ptr(work), 4, nn, hh, EPS, 0.01, 1,
                               None, None) == binding.DPD_E_INVAL
    nn = (C.c_int32 * 3)(4, 4, 4)
    assert L.dpd_phi_relax(binding._ptr(phi), binding._ptr(work), 2, nn, hh, EPS, 0.01, 1,
                           None, None) == binding.DPD_E_INVAL
    assert torch.all(phi == 1)


def test_sphere_keeps_radius(dpd):
    """A sphere of radius 3 from a step function on a 48^3 grid: the phi = 0
    surface stays at r = 3 over t' = 2..8 (the counter term cancels the
    curvature-driven shrinkage, which would take R^2 down by 4 eps^2 t')."""
    import torch
    Lb, h, R0 = 12.0, 0.25, 3.0
    n = int(Lb / h)
    x = np.arange(n) * h
    c = Lb / 2 + 0.1
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt((X - c) ** 2 + (Y - c) ** 2 + (Z - c) ** 2)
    phi = torch.tensor(np.where(r < R0, 1.0, -1.0), dtype=torch.float32, device="cuda")
    dtau = 0.5 * pf.max_stable_dtau((h, h, h), EPS)
    W = np.sqrt(2.0) * EPS
    radii = []
    done = 0
    for T in (2.0, 8.0):
        it = int(round(T / dtau)) - done
        done += it
        dpd.relax_phi(phi, (h, h, h), EPS, dtau, it)
        p = phi.cpu().numpy().astype(np.float64)
        band = np.abs(p) < 0.9
        radii.append(float((r[band] + W * np.arctanh(p[band])).mean()))
    say("radius at t' = 2, 8:", radii)
    assert abs(radii[1] - radii[0]) < 0.01
    assert abs(radii[1] - R0) < 0.02


def test_full_size_one_step_sampled(dpd):
    """672^3 nodes (the porous workload's grid, float32): one step, 4096
    sampled nodes against the oracle's right-hand side on each node's
    5 x 5 x 5 periodic neighbourhood (the step reads no further)."""
    import torch
    n, h = 672, 0.25
    g = torch.arange(n, device="cuda", dtype=torch.float32) * h
    f = (torch.sin(g / 2.3)[None, None, :] + torch.cos(g / 3.1)[None, :, None] +
         torch.sin(g / 1.7 + 0.4)[:, None, None] * 0.8)
    phi = torch.where(f > 0.2, 1.0, -1.0).to(torch.float32)
    del f
    phi0 = phi.clone()
    dtau = 0.5 * pf.max_stable_dtau((h, h, h), EPS)
    dpd.relax_phi(phi, (h, h, h), EPS, dtau, 1)
    rng = np.random.default_rng(11)
    idx = rng.integers(0, n, size=(4096, 3))
    # patches around the samples, gathered on the device
    off = np.arange(-2, 3)
    kz = (idx[:, 0, None] + off[None, :]) % n
    ky = (idx[:, 1, None] + off[None, :]) % n
    kx = (idx[:, 2, None] + off[None, :]) % n
    tz = torch.tensor(kz, device="cuda")[:, :, None, None]
    ty = torch.tensor(ky, device="cuda")[:, None, :, None]
    tx = torch.tensor(kx, device="cuda")[:, None, None, :]
    patches = phi0[tz, ty, tx].cpu().numpy().astype(np.float64)
    ii = torch.tensor(idx, device="cuda")
    got = phi[ii[:, 0], ii[:, 1], ii[:, 2]]
    got = got.cpu().numpy().astype(np.float64)
    want = np.empty(len(idx))
    for m in range(len(idx)):
        p = patches[m]
        want[m] = p[2, 2, 2] + dtau * pf.rhs(p, (h, h, h), EPS)[2, 2, 2]
    err = np.abs(got - want).max()
    say("sampled max err %.3e, %d interface samples" % (err, int((np.abs(want) < 0.999).sum())))
    assert err <= 1e-5
    assert (np.abs(want) < 0.999).sum() > 50
