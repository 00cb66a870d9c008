"""Gamma-law equation of state (oracle).

Reading (the paper uses a realistic stellar EOS, Sec. 4, which needs tables):
an ideal gas with p = (gamma - 1) rho e and code units in which p = rho T, so
T = (gamma - 1) e and c = sqrt(gamma p / rho).
"""
from __future__ import annotations

import numpy as np


def kinetic(U, dim):
    """Kinetic energy density 0.5 |rho u|^2 / rho."""
    rho = U[0]
    ke = 0.0
    for d in range(dim):
        ke = ke + U[1 + d] * U[1 + d]
    return 0.5 * ke / rho


def pressure(U, dim, gamma):
    return (gamma - 1.0) * (U[1 + dim] - kinetic(U, dim))


def temperature_from_internal(rho_e, rho, gamma):
    return (gamma - 1.0) * rho_e / rho


def sound_speed(rho, p, gamma):
    return np.sqrt(gamma * p / rho)
