"""Pins of the oracle's attractive-repulsive conservative force (Eq. 22-24,
Sec. III.C).

Fixed by the mathematics rather than by retyping the formulas: the
smoothing function of Eq. 23 is normalised (its integral over space is 1
for either range); its derivative is the derivative of the function (finite
differences) and both are continuous where the pieces meet; the force is
minus the gradient of the total energy of Eq. 22 (central differences of
the separately coded energy), which fixes the sign Eq. 24 leaves open; and
pair forces cancel in sum (Newton's third law) without walls.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads


@pytest.mark.parametrize("r0", [0.73, 1.0])
def test_kernel_is_normalised(oracle_lib, r0):
    val, err = integrate.quad(lambda r: 4.0 * np.pi * r * r * oracle.sph_w(r, r0), 0.0, r0,
                              points=[0.5 * r0], epsabs=1e-13, epsrel=1e-13)
    assert abs(val - 1.0) < 1e-10


@pytest.mark.parametrize("r0", [0.73, 1.0])
def test_kernel_derivative_and_smoothness(oracle_lib, r0):
    h = 1e-6
    for r in np.linspace(0.01, r0 * 0.999, 37):
        fd = (oracle.sph_w(r + h, r0) - oracle.sph_w(r - h, r0)) / (2 * h)
        assert abs(fd - oracle.sph_dw(r, r0)) < 1e-6 * (1 + abs(fd))
    # W and dW/dr continuous where the pieces meet (v = 1) and at the support edge
    for rj in (0.5 * r0, r0):
        e = 1e-9
        assert abs(oracle.sph_w(rj - e, r0) - oracle.sph_w(rj + e, r0)) < 1e-6
        assert abs(oracle.sph_dw(rj - e, r0) - oracle.sph_dw(rj + e, r0)) < 1e-6
    assert oracle.sph_w(r0, r0) == 0.0 and oracle.sph_dw(r0 * 1.01, r0) == 0.0


def _sph_system(seed=5, walls=True):
    s = workloads.tiny_slab_system(seed=seed) if walls else workloads.bulk_system(
        L=(4.0, 4.0, 5.0), params=workloads.default_params(seed=seed))
    p = dict(s.params)
    p["sph"] = workloads.sph_force()
    p["kBT"] = 0.0
    p["gamma"] = 0.0
    p["g"] = (0.0, 0.0, 0.0)
    s.params = p
    return s


def test_force_is_minus_energy_gradient(oracle_lib):
    s = _sph_system()
    o = oracle.Oracle(s)
    f = o.forces(k=0, mode=0)
    rng = np.random.default_rng(1)
    fluid = np.nonzero(s.type == 0)[0]
    h = 1e-6
    r0 = o.r.copy()
    for i in rng.choice(fluid, 8, replace=False):
        for a in range(3):
            o.r = r0.copy(); o.r[i, a] += h
            ep = o.potential()
            o.r = r0.copy(); o.r[i, a] -= h
            em = o.potential()
            fd = -(ep - em) / (2 * h)
            assert abs(fd - f[i, a]) < 1e-5 * (1 + abs(f[i, a])), (i, a, fd, f[i, a])
    o.r = r0


def test_pair_forces_cancel_without_walls(oracle_lib):
    s = _sph_system(walls=False)
    o = oracle.Oracle(s)
    f = o.forces(k=0, mode=0)
    assert np.abs(f.sum(axis=0)).max() < 1e-9 * np.abs(f).sum()
    assert np.abs(f).max() > 1.0


def test_window_rejects_sph_force(oracle_lib):
    s = _sph_system()
    with pytest.raises(ValueError):
        oracle.Oracle(s).window(2)
