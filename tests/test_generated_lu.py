"""CPU checks of the generated Newton linear algebra (host build of the device
functions the kernels inline).

The network code generator emits, per topology, the packed Newton matrix and
a fixed-order LU that carries the right-hand side through the elimination
(net_lu_solve) besides the factor-only LU and the transposed solve used by
the adjoint (net_lu, net_solve_t).  Here those functions are cut out of the
generated source, compiled for the host with g++ and run on random matrices
with the network's sparsity pattern: the solution must match a dense LAPACK
solve, the fused solve must give the same bits as factor-then-solve done by
a plain loop over the packed factors, and the pivot guard must reject a
pivot below tau times its column maximum.
"""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import sdc_inputs as si

NETS = [("chain", si.chain_network()),
        ("net7", si.random_network(7, 10, 202)),
        ("net13", si.random_network(13, 20, 302))]


def _pattern(net):
    """Slot map of the packed matrix: structural nonzeros of I - dt dR/dx and
    their LU fill-in, numbered row by row (the generator's packing)."""
    ns = net["nspec"]
    n = ns + 1
    P = np.eye(n, dtype=bool)
    for r in range(net["nreact"]):
        cols = [c for c in net["reactants"][r] if c >= 0] + [ns]
        rows = list(np.nonzero(net["stoich"][r])[0]) + [ns]
        for i in rows:
            for j in cols:
                P[i, j] = True
    S = P.copy()
    for k in range(n):
        for i in range(k + 1, n):
            if S[i, k]:
                for j in range(k + 1, n):
                    if S[k, j]:
                        S[i, j] = True
    slot = -np.ones((n, n), dtype=int)
    slot[S] = np.arange(int(S.sum()))
    return P, slot


def _function(src, name):
    """Text of `template <class MT> ... name(...) {...}` from the generated source."""
    m = re.search(r"template <class MT>\n__device__ __forceinline__ (bool|void) " + name + r"\(", src)
    assert m, name
    return src[m.start():src.index("\n}\n", m.start()) + 3]


@pytest.fixture(scope="module", params=NETS, ids=[n for n, _ in NETS])
def host_lu(request):
    from paper_1910_12578_amd import _binding
    name, net = request.param
    src = _binding.generated_source(dict(dim=1, n=(8,), dx=(0.1,)), net)
    body = "\n".join(_function(src, f) for f in ("net_lu_solve", "net_lu", "net_solve_t"))
    code = ("#include <cmath>\nusing std::fabs; using std::fmax; using std::fma;\n"
            "#define __device__\n#define __forceinline__ inline\n"
            "inline double net_rcp(double d) { return 1.0 / d; }\n" + body +
            '\nextern "C" int lu_solve(double* M, double* r, double tau) { return net_lu_solve<double>(M, r, tau); }\n'
            'extern "C" int lu(double* M, double tau) { return net_lu<double>(M, tau); }\n'
            'extern "C" void solve_t(const double* M, double* r) { net_solve_t<double>(M, r); }\n')
    d = tempfile.mkdtemp(prefix="sdc_lu_")
    cpp, so = os.path.join(d, "lu.cpp"), os.path.join(d, "lu.so")
    with open(cpp, "w") as f:
        f.write(code)
    # -ffp-contract=off: the only fused operations are the explicit fma calls
    subprocess.run(["g++", "-O1", "-ffp-contract=off", "-std=c++17", "-shared", "-fPIC", cpp, "-o", so], check=True)
    lib = ctypes.CDLL(so)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.lu_solve.argtypes = [dp, dp, ctypes.c_double]
    lib.lu.argtypes = [dp, ctypes.c_double]
    lib.solve_t.argtypes = [dp, dp]
    return name, net, lib


def _random_system(net, rng):
    """Diagonally dominant matrix with the network's pattern, packed."""
    P, slot = _pattern(net)
    n = P.shape[0]
    A = np.where(P, rng.uniform(-0.3, 0.3, (n, n)), 0.0)
    A[np.diag_indices(n)] = rng.uniform(1.0, 2.0, n)
    packed = np.zeros(int((slot >= 0).sum()))
    packed[slot[P]] = A[P]
    return A, packed, slot


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def test_fused_lu_solve_matches_dense_solve(host_lu):
    name, net, lib = host_lu
    rng = np.random.default_rng(7)
    for _ in range(20):
        A, packed, _ = _random_system(net, rng)
        b = rng.normal(size=A.shape[0])
        r = b.copy()
        assert lib.lu_solve(_ptr(packed), _ptr(r), 1e-3) == 1
        ref = np.linalg.solve(A, b)
        assert np.max(np.abs(r - ref)) <= 1e-13 * np.max(np.abs(ref)), name


def test_fused_solve_equals_factor_then_solve(host_lu):
    """The right-hand side sees the multipliers in the order a separate
    forward substitution applies them: identical bits."""
    name, net, lib = host_lu
    rng = np.random.default_rng(11)
    A, packed, slot = _random_system(net, rng)
    n = A.shape[0]
    b = rng.normal(size=n)
    r = b.copy()
    lib.lu_solve(_ptr(packed.copy()), _ptr(r), 1e-3)
    F = packed.copy()
    assert lib.lu(_ptr(F), 1e-3) == 1
    y = b.copy()  # forward substitution with the unit-lower factor, k ascending
    for k in range(n):
        for i in range(k + 1, n):
            if slot[i, k] >= 0:
                y[i] = _fma(-F[slot[i, k]], y[k], y[i])
    for k in range(n - 1, -1, -1):  # backward substitution; diagonal slots hold 1/pivot
        for j in range(k + 1, n):
            if slot[k, j] >= 0:
                y[k] = _fma(-F[slot[k, j]], y[j], y[k])
        y[k] *= F[slot[k, k]]
    assert np.array_equal(r, y), name


def _fma(a, b, c):
    """Correctly rounded a * b + c in float64: exact rational arithmetic,
    rounded once."""
    from fractions import Fraction
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def test_transposed_solve_of_the_factors(host_lu):
    name, net, lib = host_lu
    rng = np.random.default_rng(13)
    A, packed, _ = _random_system(net, rng)
    assert lib.lu(_ptr(packed), 1e-3) == 1
    c = rng.normal(size=A.shape[0])
    r = c.copy()
    lib.solve_t(_ptr(packed), _ptr(r))
    ref = np.linalg.solve(A.T, c)
    assert np.max(np.abs(r - ref)) <= 1e-13 * np.max(np.abs(ref)), name


def test_pivot_guard_rejects_small_pivots(host_lu):
    name, net, lib = host_lu
    rng = np.random.default_rng(17)
    A, packed, slot = _random_system(net, rng)
    n = A.shape[0]
    # a column with a structural subdiagonal entry whose pivot row has nothing
    # left of the diagonal (so the pivot is not updated before its step)
    k = next(k for k in range(n) if any(slot[i, k] >= 0 for i in range(k + 1, n))
             and all(slot[k, j] < 0 for j in range(k)))
    packed[slot[k, k]] = 1e-6
    r = np.ones(n)
    assert lib.lu_solve(_ptr(packed.copy()), _ptr(r), 1e-3) == 0
    assert lib.lu_solve(_ptr(packed.copy()), _ptr(np.ones(n)), 0.0) == 1
