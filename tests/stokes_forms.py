"""Closed forms of Sec. III.A-B used as pins of the DPD flow runs."""
import math


def eq19_viscosity(rho, g, a, vbar):
    """Eq. 19 (mean-velocity form): plane Poiseuille flow of half width a
    under body force g per unit mass has mean velocity rho g a^2 / (3 mu)."""
    return rho * g * a * a / (3.0 * vbar)


def eq20(c):
    """Eq. 20: normalised mean fluid velocity 4 pi vbar mu / (rho g L^2)
    through a square array of cylinders of solid area fraction c (the
    paper's epsilon = pi r^2 / L^2), series truncated after c^3."""
    return (math.log(math.sqrt(math.pi / c)) + c - 1.31 - 8.76 * (c / math.pi) ** 2
            + 63.22 * (c / math.pi) ** 3)


def eq21(c):
    """Eq. 21: the paper's fit of its own DPD results over the whole range."""
    return math.log(math.sqrt(math.pi / c)) + 1.7 * c - 1.31 - 2.15 * c * c + 1.35 * c ** 3
