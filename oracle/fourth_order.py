"""Fourth-order finite-volume pieces (oracle; test infrastructure only).

The paper's fourth-order method pairs Simpson's rule in time with the spatial
reconstruction of McCorquodale and Colella (Sec. 2).  The state of Eq. 2 is a
zone average <U>, and so are its advective and reactive terms <A(U)> and
<R(U)>; at second order they may be replaced by functions of the averages,
at fourth order they may not.  This module holds the fourth-order advective
term and the conversions between zone averages and zone-centre (point)
values.

Readings (the paper names the method and gives no formulas):

* Face averages.  Along the face normal d, the average of U over the face at
  i+1/2 is the fourth-order interpolation of the four nearest zone averages:
  7/12 (<U>_i + <U>_{i+1}) - 1/12 (<U>_{i-1} + <U>_{i+2}).
* Face centres.  The value at the centre of that face is its average minus
  1/24 of the sum, over the directions along the face, of the second
  differences of the face averages (the h^2/24 Laplacian of the face).
* Fluxes.  The point flux is the Euler flux of the face-centre value; the
  face-averaged flux adds 1/24 of the transverse second differences of the
  Euler flux of the face averages.  A = -sum_d (<F>_{i+1/2} - <F>_{i-1/2})/h_d.
* No limiter and no Riemann solver: the left and right face states coincide,
  so the Rusanov dissipation of the second-order scheme vanishes.  This is the
  method for smooth flows; the limited variant is outside this reading.
* Averages and centres.  u_c = <u> - 1/24 sum_d delta_d^2 <u> and
  <f> = f_c + 1/24 sum_d delta_d^2 f_c, with delta_d^2 the second difference
  along direction d (u_{i+1} - 2 u_i + u_{i-1}).  Both are exact for
  polynomials of total degree <= 3 and fourth-order accurate otherwise.

Arrays are U[comp, *grid] with the grid in C order (z, y, x): direction d
lives on array axis U.ndim - 1 - d, and the grid is periodic.
"""
from __future__ import annotations

import numpy as np

from .advection import euler_flux


def second_difference(u, ax):
    return np.roll(u, -1, axis=ax) - 2.0 * u + np.roll(u, 1, axis=ax)


def laplacian24(u, dim, skip=None):
    """1/24 of the sum of second differences over the grid directions
    (direction `skip` left out): the h^2/24 Laplacian of the conversions."""
    out = np.zeros_like(u)
    for d in range(dim):
        if d != skip:
            out = out + second_difference(u, u.ndim - 1 - d)
    return out / 24.0


def to_centres(U, dim):
    """Zone-centre values from zone averages."""
    return U - laplacian24(U, dim)


def to_averages(f, dim):
    """Zone averages from zone-centre values."""
    return f + laplacian24(f, dim)


def face_average(U, ax):
    """Average over the face at i+1/2 along array axis `ax` (fourth order)."""
    return (7.0 / 12.0) * (U + np.roll(U, -1, axis=ax)) - (1.0 / 12.0) * (np.roll(U, 1, axis=ax)
                                                                         + np.roll(U, -2, axis=ax))


def advective_term4(U, dim, dx, gamma):
    """Fourth-order <A(U)> on a periodic grid (see the module docstring)."""
    A = np.zeros_like(U)
    for d in range(dim):
        ax = U.ndim - 1 - d
        Uf = face_average(U, ax)                 # face averages at i+1/2
        Uc = Uf - laplacian24(Uf, dim, skip=d)   # face-centre values
        Fc, _, _ = euler_flux(Uc, d, dim, gamma)
        Ff, _, _ = euler_flux(Uf, d, dim, gamma)
        F = Fc + laplacian24(Ff, dim, skip=d)    # face-averaged flux
        A -= (F - np.roll(F, 1, axis=ax)) / dx[d]
    return A
