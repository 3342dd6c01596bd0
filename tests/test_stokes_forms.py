"""Pins of the closed forms the cylinder-array runs are checked against.

Eq. 20 is the small-concentration series for slow viscous flow
perpendicular to a square array of cylinders (Hasimoto 1959; Sangani and
Acrivos 1982): 4 pi mu U / F = -1/2 ln c - 0.738 + c - 0.887 c^2 +
2.038 c^3 + ..., with F the drag per unit length on a cylinder and U the
superficial velocity.  With the body force on the fluid only, F = rho g L^2
(1 - c) and the mean fluid velocity is U / (1 - c), which is the paper's
normalisation.  The paper writes the same series as ln sqrt(pi / c) - 1.31
and powers of c / pi.
"""
import math

from stokes_forms import eq19_viscosity, eq20, eq21


def test_eq20_is_the_square_array_series():
    for c in (0.01, 0.05, 0.1, 0.2):
        series = -0.5 * math.log(c) - 0.738 + c - 0.887 * c * c + 2.038 * c ** 3
        assert abs(eq20(c) - series) < 2e-3 * max(1.0, c * 10)


def test_eq21_keeps_the_logarithm_and_differs_at_large_fractions():
    assert abs((eq21(1e-4) - eq20(1e-4))) < 1e-3
    assert eq21(0.2) > eq20(0.2) + 0.05


def test_eq19_inverts_the_poiseuille_mean():
    rho, g, a, mu = 4.0, 0.02, 5.0, 1.7
    vbar = rho * g * a * a / (3 * mu)
    assert abs(eq19_viscosity(rho, g, a, vbar) - mu) < 1e-12
