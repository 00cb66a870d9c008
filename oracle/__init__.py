"""Plain FP64 CPU oracle of the SDC reactive-flow update (test infrastructure).

This package is TEST INFRASTRUCTURE ONLY.  It exists to check the HIP
implementation; only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import or call it.  The product path
(`paper_1910_12578_amd`) never imports it and shares no code with it: the two
meet only in the seeded input generators of `sdc_inputs`.

What it computes (Zingale et al., "The Castro AMR Simulation Code: Current
and Future Developments", Sec. 2):

* the conservative split U_t = A(U) + R(U) (Eq. 1), with A a method-of-lines
  finite-volume advective term (`advection.py`) and R a synthetic Arrhenius
  network (`network.py`);
* the SDC correction update from node m to m+1 (Eq. 2), iterated K times over
  Gauss-Lobatto nodes whose interpolatory quadrature gives the trapezoid
  (2 nodes) and Simpson (3 nodes) integrals (`quadrature.py`, `sdc.py`);
* the implicit reaction equation of Eq. 2 solved per zone by Newton with a
  dense analytic Jacobian and LAPACK LU with partial pivoting (`sdc.py`);
* the gradient of the integrated energy release with respect to the rate
  parameters by complex-step differentiation of the whole run (`adjoint.py`).

Everything is vectorised over zones with NumPy and written for clarity, not
speed.  Where the paper is silent, the readings used are stated in the
docstrings of the function that applies them.

Pins (each function is checked by `tests/test_oracle_*.py` against something
other than itself): quadrature exactness on polynomials, Pade fixed points of
the linear chain, the closed-form exponential solution, IMEX-Euler first
sweep, brute-force Radau integration, exact conservation, measured 2nd/4th
order in time, advective-term invariants and 2nd-order spatial convergence,
Jacobian and gradient against complex step / finite differences.

Parity unpinned (nothing outside this code fixes them): the synthetic
network's realism, the choice of initial iterate, the end-of-step value and
the spatial scheme for A; these follow the readings stated in the sources.
"""
