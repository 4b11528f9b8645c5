"""Pins of the oracle's transpose-free variant (no A^H, w_k recombined) on the CPU.

The variant is an addition of this library.  What fixes it independently of
its own code: Table 4.2's per-iteration costs at M = I (same matvecs and dots
as Algorithm 7.1, (n-1)/2 more saxpys), finite termination for n >= N, eq. (4.1)
against Algorithm 3.1 (it is the same iteration in exact arithmetic), the
definition w_k = A g_k up to rounding, and, with n = 1 (no inner steps), bitwise
equality with Algorithm 7.1.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import OpCounter, g_n, mlbicg, mlbicgstabt, true_error
from tests.test_oracle_pins import _omega_poly, block, dd_dense, vec


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
def test_table_4_2_operation_counts(n):
    """Per steady cycle: matvec n+1, dot n^2+n+2, saxpy 2n^2+2n+2, scale n (Table 4.2 times n).

    Table 4.2 lists 1 + 1/n matvecs, n + 1 + 2/n dots, 2n + 2 + 2/n saxpys and one
    scaling per iteration; at M = I the preconditioner count equals the matvec count.
    """
    A = workloads.convdiff_2d(12, pe=2.0)
    N = A.shape[0]
    cnt = OpCounter()
    res = mlbicgstabt(A, vec(N, 1), block(N, n, 2), tol=1e-300, maxit=4 * n + 1, counter=cnt, transpose_free=True)
    assert res.flag == 1
    marks = dict((lab[1], c) for lab, c in cnt.marks)
    d = {key: marks[2][key] - marks[1][key] for key in OpCounter.KEYS}
    assert d["matvec"] == n + 1
    assert d["precond"] == n + 1
    assert d["dot"] == n * n + n + 2
    assert d["saxpy"] == 2 * n * n + 2 * n + 2
    assert d["scale"] == n
    assert d["norm"] == n + 1


@pytest.mark.parametrize("N", [4, 7, 12])
@pytest.mark.parametrize("extra", [0, 3])
@pytest.mark.parametrize("complex_", [False, True])
def test_finite_termination(N, extra, complex_):
    """n >= N: r_N = 0, so the N-th iterate is the LU solution."""
    A = dd_dense(N, 10 + N, complex_)
    b = vec(N, 20 + N, complex_)
    Q = block(N, N + extra, 30 + N, complex_)
    res = mlbicgstabt(A, b, Q, tol=1e-10, maxit=10 * N, transpose_free=True)
    assert res.flag == 0
    assert res.iter == N
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) < 1e-10


@pytest.mark.parametrize("n", [2, 3, 5])
@pytest.mark.parametrize("complex_", [False, True])
def test_residual_definition_eq_4_1(n, complex_):
    """r_k = Omega_{g_n(k+1)}(A) hat r_k with hat r_k from Algorithm 3.1 on the same Q (three cycles)."""
    N = 24
    A = dd_dense(N, 40 + n, complex_, dominance=2.5)
    b = vec(N, 41, complex_)
    Q = block(N, n, 42, complex_)
    K = 3 * n
    res = mlbicgstabt(A, b, Q, tol=1e-30, maxit=K, record_x=K, transpose_free=True)
    assert len(res.x_history) == K
    _, rhat = mlbicg(A, b, Q, steps=K)
    for k in range(1, K + 1):
        rk = b - A @ res.x_history[k - 1]
        ref = _omega_poly(A, res.omegas, g_n(n, k + 1), rhat[k])
        tol = 1e-8 * np.linalg.norm(ref) + 1e-13 * np.linalg.norm(b)
        assert np.linalg.norm(rk - ref) < tol, (k, n)


@pytest.mark.parametrize("n", [2, 4, 8])
def test_recombined_w_is_A_g(n):
    """Every recombined w_k equals A g_k to rounding over the first cycles."""
    A = workloads.convdiff_2d(12, pe=3.0)
    N = A.shape[0]
    worst = []

    def obs(event, **st):
        if event == "w":
            w = st["w"]
            worst.append(np.linalg.norm(w - A @ st["g"]) / np.linalg.norm(w))

    mlbicgstabt(A, vec(N, 4), block(N, n, 3), tol=1e-300, maxit=4 * n, observer=obs, transpose_free=True)
    assert len(worst) >= 4 * n
    assert max(worst) < 1e-12


@pytest.mark.parametrize("complex_", [False, True])
def test_n1_equals_algorithm_7_1_bitwise(complex_):
    """With one shadow vector there are no inner steps, so nothing differs."""
    A = workloads.helmholtz_3d(6, pe=2.0, k=3.0, gen=workloads.rng(99, 0)) if complex_ else \
        workloads.convdiff_2d(10, pe=3.0)
    N = A.shape[0]
    b, q = vec(N, 1, complex_), vec(N, 2, complex_)
    a = mlbicgstabt(A, b, q[:, None], tol=1e-10, maxit=500)
    t = mlbicgstabt(A, b, q[:, None], tol=1e-10, maxit=500, transpose_free=True)
    assert a.iter == t.iter and a.flag == t.flag == 0
    assert np.array_equal(a.x, t.x)


@pytest.mark.parametrize("case", ["2d_n4", "2d_n8", "3d_n16", "complex_n8"])
def test_solution_vs_lu(case):
    """Benchmark-shaped systems: the solution meets the tolerance against a sparse LU solve."""
    p = {"2d_n4": lambda: workloads.config1(n=4), "2d_n8": lambda: workloads.config1(n=8),
         "3d_n16": lambda: workloads.config2(n=16, m=16, maxit=4000),
         "complex_n8": lambda: workloads.config5(n=8, m=10)}[case]()
    res = mlbicgstabt(p.A, p.b, p.Q, tol=p.tol, maxit=p.maxit, transpose_free=True)
    assert res.flag == 0
    xs = spla.splu(p.A.tocsc()).solve(p.b)
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) < 1e-7
    assert true_error(p.A, res.x, p.b) < 10 * p.tol


def test_reservoir_drift_is_bounded():
    """On the ill-conditioned block system the recursive residual drifts from the true one
    (the behaviour Section 5.1 reports for the second algorithm); the solution still lies
    within 1e-6 of the LU solve."""
    p = workloads.config3(n=4, grid=(8, 10, 6))
    res = mlbicgstabt(p.A, p.b, p.Q, tol=p.tol, maxit=p.maxit, transpose_free=True)
    assert res.flag == 0 and res.err < p.tol
    xs = spla.splu(p.A.tocsc()).solve(p.b)
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) < 1e-6
    assert true_error(p.A, res.x, p.b) < 1e-7


def test_jacobi_preconditioned_vs_lu():
    """M = diagonal of A (right-applied, as the GPU library does): same solution as LU."""
    p = workloads.config1(n=4)
    d = p.A.diagonal()
    res = mlbicgstabt(p.A, p.b, p.Q, tol=p.tol, maxit=p.maxit, precond=(lambda v: v / d, lambda v: v / np.conj(d)),
                      transpose_free=True)
    assert res.flag == 0
    xs = spla.splu(p.A.tocsc()).solve(p.b)
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) < 1e-7
