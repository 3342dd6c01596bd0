"""FP64 oracle of the phase-field relaxation of Eq. 15 (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
CPU-baseline leg of the benchmark are the only users.  The GPU library never
imports or calls anything here, and this module imports nothing from the
GPU package.

What it computes (Sec. II.B, Eq. 13-15), on the periodic node-centred grid
of the DPD step (node (i, j, k) at (i h0, j h1, k h2), arrays indexed
[k, j, i], x fastest):

    d phi / d t' = lap' phi + phi (1 - phi^2) - kappa |grad' phi|,
    kappa = div' (grad' phi / |grad' phi|),   grad' = eps grad,

integrated in the pseudo time t' from an initial field (a step function
-1 / +1 in the paper) by explicit Euler steps of length dtau.

Discretisation (the paper names a finite-difference grid and no stencil;
these are the readings):
  - lap' phi: the compact 7-point Laplacian, eps^2 sum_a (phi[+a] - 2 phi +
    phi[-a]) / h_a^2;
  - grad' phi: central differences, eps (phi[+a] - phi[-a]) / (2 h_a);
  - the unit normal n = grad' phi / max(|grad' phi|, delta) with
    delta = 0.01: exactly the unit normal wherever |grad' phi| >= delta
    (on the planar profile, everywhere with |phi| < 0.9929), and going
    linearly to zero where phi is flat (the bulk phases) instead of being
    a direction of rounding noise; the map from grad' phi to n then has
    slope <= 1/delta, which bounds how much the counter term amplifies
    rounding where grad' phi passes through zero;
  - kappa: central differences of n, sum_a eps (n_a[+a] - n_a[-a]) / (2 h_a);
  - the counter term kappa |grad' phi| uses the same |grad' phi|.
Pins: the planar steady state is Eq. 14's tanh profile, converging at
second order in h; the interface width of Sec. II.B; a sphere keeps its
radius (the counter term), while without the counter term it shrinks by
mean-curvature flow (the sharp-interface law of the Allen-Cahn equation);
phi -> -phi symmetry.
"""
from __future__ import annotations

import numpy as np

DELTA = 0.01


def _d1(phi, axis, h):
    """Central difference along `axis` (array axes are z, y, x)."""
    return (np.roll(phi, -1, axis=axis) - np.roll(phi, 1, axis=axis)) / (2.0 * h)


def rhs(phi, h, eps, counter_term=True, delta=DELTA):
    """Right-hand side of Eq. 15 at every node.

    h: spacings (h_x, h_y, h_z); eps: the interface coefficient of Eq. 12.
    counter_term=False gives the plain Allen-Cahn form (Eq. 13 in 3-D)."""
    phi = np.asarray(phi, dtype=np.float64)
    axes = (2, 1, 0)  # x, y, z
    lap = np.zeros_like(phi)
    for a, ax in enumerate(axes):
        lap += (np.roll(phi, -1, axis=ax) - 2.0 * phi + np.roll(phi, 1, axis=ax)) / (h[a] * h[a])
    lap *= eps * eps
    out = lap + phi * (1.0 - phi * phi)
    if not counter_term:
        return out
    # grad' phi and its magnitude
    g = [eps * _d1(phi, ax, h[a]) for a, ax in enumerate(axes)]
    gmag = np.sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2])
    # unit normal (regularised where phi is flat) and its divergence
    den = np.maximum(gmag, delta)
    kappa = np.zeros_like(phi)
    for a, ax in enumerate(axes):
        kappa += eps * _d1(g[a] / den, ax, h[a])
    return out - kappa * gmag


def relax(phi0, h, eps, dtau, iters, counter_term=True, delta=DELTA):
    """`iters` explicit Euler steps of Eq. 15 from phi0; returns the field
    and the largest |d phi / d t'| of the last step."""
    phi = np.array(phi0, dtype=np.float64)
    res = 0.0
    for _ in range(iters):
        r = rhs(phi, h, eps, counter_term, delta)
        res = float(np.abs(r).max())
        phi = phi + dtau * r
    return phi, res


def max_stable_dtau(h, eps):
    """Explicit-Euler limit of the diffusion part: dtau <= 1 / (2 sum_a
    (eps / h_a)^2) (the reaction term, slope <= 1, is far less stiff)."""
    return 1.0 / (2.0 * sum((eps / x) ** 2 for x in h))
