"""Advective term A(U): divergence of the hydrodynamic fluxes (oracle).

The paper's A(U) is the divergence of the hydro fluxes (Sec. 2, Eq. 1),
computed in Castro with unsplit PPM.  SDC needs A as a function of the state
alone, so the reading here is a method-of-lines finite-volume operator on a
uniform periodic grid:

* per direction d, piecewise-linear reconstruction of the conserved variables
  with central slopes (smooth mode, slope=0) or monotonized-central slopes
  (slope=1);
* Rusanov (local Lax-Friedrichs) face flux
  F = 1/2 (F(U_L) + F(U_R)) - 1/2 alpha (U_R - U_L), with alpha the local
  max(|u_d| + c) over the two face states, or a frozen constant (alpha > 0);
* A = - sum_d (F_{i+1/2} - F_{i-1/2}) / dx_d.

Arrays are U[comp, *grid] with the grid in C order (z, y, x): direction d
lives on array axis U.ndim - 1 - d.  Hydro source terms are absent.
"""
from __future__ import annotations

import numpy as np

from . import eos


def euler_flux(U, d, dim, gamma):
    """Physical flux of the Euler equations plus passive species, direction d."""
    rho = U[0]
    u_d = U[1 + d] / rho
    p = eos.pressure(U, dim, gamma)
    F = U * u_d[None]
    F[1 + d] = F[1 + d] + p
    F[1 + dim] = F[1 + dim] + p * u_d
    return F, u_d, p


def mc_slope(a, b):
    """Monotonized-central limited slope from one-sided differences a, b."""
    mag = np.minimum(np.minimum(2.0 * np.abs(a), 2.0 * np.abs(b)), 0.5 * np.abs(a + b))
    return np.where(a * b > 0.0, np.sign(a) * mag, 0.0)


def advective_term(U, dim, dx, gamma, slope=1, alpha=-1.0):
    """A(U) on a periodic grid (see module docstring)."""
    A = np.zeros_like(U)
    for d in range(dim):
        ax = U.ndim - 1 - d
        Fh = face_flux(U, d, dim, gamma, slope, alpha)
        A -= (Fh - np.roll(Fh, 1, axis=ax)) / dx[d]
    return A


def face_flux(U, d, dim, gamma, slope=1, alpha=-1.0):
    """Rusanov flux through the face i+1/2 along direction d of every zone
    (periodic grid)."""
    ax = U.ndim - 1 - d
    Um = np.roll(U, 1, axis=ax)
    Up = np.roll(U, -1, axis=ax)
    if slope == 0:
        dU = 0.5 * (Up - Um)
    else:
        dU = mc_slope(U - Um, Up - U)
    UL = U + 0.5 * dU                       # left state at face i+1/2
    UR = np.roll(U - 0.5 * dU, -1, axis=ax)  # right state at face i+1/2
    FL, uL, pL = euler_flux(UL, d, dim, gamma)
    FR, uR, pR = euler_flux(UR, d, dim, gamma)
    if alpha > 0:
        a = alpha
    else:
        cL = eos.sound_speed(UL[0], pL, gamma)
        cR = eos.sound_speed(UR[0], pR, gamma)
        a = np.maximum(np.abs(uL) + cL, np.abs(uR) + cR)[None]
    return 0.5 * (FL + FR) - 0.5 * a * (UR - UL)
