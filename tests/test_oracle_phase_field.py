"""Pins of the phase-field relaxation oracle (Sec. II.B, Eq. 13-15).

Against what the mathematics fixes, not the stencil retyped:
  - the planar steady state is Eq. 14's tanh profile about the midpoint of
    the initial step, and the discrete solution converges to it at second
    order in the grid spacing;
  - the interface width (-0.9 < phi < 0.9) of that profile is
    2 atanh(0.9) sqrt(2) eps, the paper's "about 3 sqrt(2) eps";
  - without the counter term, a sphere shrinks by mean-curvature flow, the
    sharp-interface law of the Allen-Cahn equation: d R^2 / d t' = -4 eps^2
    in three dimensions;
  - with it, the sphere keeps its radius (the term cancels curvature-driven
    motion, Sec. II.B);
  - the equation is odd in phi.
A dropped or mis-scaled term, a wrong sign of the counter term, a
transposed axis or a wrong spacing fails one of these.
"""
import numpy as np

from oracle import phase_field as pf

EPS = 0.5 / np.sqrt(2.0)   # interface coefficient of the workloads: sqrt(2) eps = 0.5
W = np.sqrt(2.0) * EPS


def _planar(h, L=16.0, T=20.0, axis=2):
    """Slab 4 < x < 12 as a step function along one grid axis; returns the
    relaxed 1-D profile, the node coordinates and Eq. 14 about the step's
    midpoints."""
    n = int(round(L / h))
    x = np.arange(n) * h
    fl = (x > 4.0 + 0.3 * h) & (x < 12.0 + 0.3 * h)
    shape = [1, 1, 1]
    shape[axis] = n
    phi0 = np.where(fl, 1.0, -1.0).reshape(shape)
    hs = [1.0, 1.0, 1.0]
    hs[2 - axis] = h
    dtau = 0.5 * pf.max_stable_dtau(hs, EPS)
    phi, res = pf.relax(phi0, hs, EPS, dtau, int(T / dtau))
    i0, i1 = np.nonzero(fl)[0][[0, -1]]
    xl, xr = 0.5 * (x[i0 - 1] + x[i0]), 0.5 * (x[i1] + x[i1 + 1])
    exact = np.tanh(np.minimum(x - xl, xr - x) / W)
    return phi.reshape(-1), x, exact, res


def test_planar_steady_state_is_eq14_at_second_order():
    e = []
    for h in (0.25, 0.125):
        phi, x, exact, res = _planar(h)
        assert res < 1e-10
        e.append(np.abs(phi - exact).max())
    assert e[1] < 5e-3
    assert 3.5 < e[0] / e[1] < 4.5, e


def test_planar_profile_along_each_axis_is_the_same():
    ref = _planar(0.25, axis=2)[0]
    for axis in (0, 1):
        assert np.allclose(_planar(0.25, axis=axis)[0], ref, rtol=0, atol=1e-13)


def test_interface_width():
    h = 0.0625
    phi, x, _, _ = _planar(h)
    left = x < 8.0
    p, xs = phi[left], x[left]

    def cross(v):
        i = np.nonzero((p[:-1] < v) & (p[1:] >= v))[0][0]
        return xs[i] + (v - p[i]) / (p[i + 1] - p[i]) * h

    width = cross(0.9) - cross(-0.9)
    assert abs(width - 2.0 * np.arctanh(0.9) * W) < 0.01
    assert abs(width - 3.0 * W) < 0.05   # the paper's rounded figure


def _sphere_radius_series(counter_term, times, L=12.0, h=0.25, R0=3.0):
    n = int(round(L / h))
    x = np.arange(n) * h
    c = L / 2 + 0.1
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt((X - c) ** 2 + (Y - c) ** 2 + (Z - c) ** 2)
    phi = np.where(r < R0, 1.0, -1.0)
    dtau = 0.5 * pf.max_stable_dtau((h, h, h), EPS)
    t, out = 0.0, []
    for T in times:
        it = int(round((T - t) / dtau))
        t += it * dtau
        phi, _ = pf.relax(phi, (h, h, h), EPS, dtau, it, counter_term=counter_term)
        # sharp radius from the profile: r + W atanh(phi) over the band
        band = np.abs(phi) < 0.9
        out.append((t, float((r[band] + W * np.arctanh(phi[band])).mean())))
    return out


def test_sphere_without_counter_term_follows_mean_curvature_flow():
    (t1, r1), (t2, r2) = _sphere_radius_series(False, [2.0, 6.0])
    rate = (r2 * r2 - r1 * r1) / (t2 - t1)
    assert abs(rate + 4.0 * EPS * EPS) < 0.05 * 4.0 * EPS * EPS, rate


def test_sphere_with_counter_term_keeps_its_radius():
    (t1, r1), (t2, r2) = _sphere_radius_series(True, [2.0, 8.0])
    assert abs(r2 - r1) < 0.01
    assert abs(r2 - 3.0) < 0.02


def test_odd_in_phi():
    rng = np.random.default_rng(3)
    phi0 = np.where(rng.standard_normal((10, 12, 14)) > 0, 1.0, -1.0)
    a, _ = pf.relax(phi0, (0.25, 0.3, 0.35), EPS, 0.02, 30)
    b, _ = pf.relax(-phi0, (0.25, 0.3, 0.35), EPS, 0.02, 30)
    assert np.array_equal(a, -b)


def test_parity_inputs_are_well_conditioned():
    """The GPU parity inputs: relative input perturbations of 1e-7 move the
    relaxed field by at most 100 times that (no sliver thinner than the
    interface, whose fate rounding would decide), so FP32 rounding of the
    kernels stays within the parity tolerance."""
    from pf_cases import CASES, case_input
    rng = np.random.default_rng(1)
    for i in range(len(CASES)):
        phi0, h, iters = case_input(i)
        dtau = 0.5 * pf.max_stable_dtau(h, EPS)
        a, _ = pf.relax(phi0, h, EPS, dtau, iters)
        for _ in range(2):
            b, _ = pf.relax(phi0 * (1 + 1e-7 * rng.standard_normal(phi0.shape)), h, EPS, dtau, iters)
            assert np.abs(a - b).max() < 100 * 1e-7, i
        assert (np.abs(a) < 0.9).sum() > 0
