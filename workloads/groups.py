"""Dimensionless groups of the jet runs (eq. 33-37) used to set up scenarios.

We = rho0 u0^2 R / sigma and Re = rho0 u0 R / mu use the orifice radius R
(eq. 33-34); Oh = sqrt(We)/Re (eq. 35); Fr = u0 / sqrt(g D0) (eq. 36). The
breakup-length correlation (eq. 37) is read as L/D0 = 13 sqrt(We) (1 + 3 Oh):
the printed "30h" is a garbled "3 Oh", which reproduces every correlation entry
of Table 1 to the printed precision.
"""
import math


def weber(rho0, u0, R, sigma):
    return rho0 * u0 * u0 * R / sigma


def reynolds(rho0, u0, R, mu):
    return rho0 * u0 * R / mu


def ohnesorge(We, Re):
    return math.sqrt(We) / Re


def froude(u0, g, D0):
    return u0 / math.sqrt(g * D0)


def breakup_length_correlation(We, Oh):
    """L / D0 from eq. 37."""
    return 13.0 * math.sqrt(We) * (1.0 + 3.0 * Oh)
