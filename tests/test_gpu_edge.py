"""Degenerate systems on the GPU (multi-launch solve and one-workgroup batch) against the oracle.

N = 1; more shadow vectors than unknowns (n > N); a right-hand side that is an eigenvector (exact
after one step); an all-zero matrix with empty index arrays (breakdown at k = 0); a consistent
singular system; an inconsistent singular system, which must not be reported as converged.  The
multi-launch cases are also run without A^H (transpose_free) against the oracle's variant.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from tests.gpu_util import gpu_available, rel, run_gpu

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_1106_3678_amd import binding  # noqa: E402


def problem(name, A, b, Q, maxit=50):
    A = sp.csr_matrix(A)
    return workloads.Problem(name, A, np.asarray(b, float), np.asfortranarray(Q), np.zeros(A.shape[0]), Q.shape[1],
                             1e-10, maxit)


def batch_solve(p):
    dA = binding.to_device(p.A)
    b = torch.from_numpy(p.b).cuda()
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    Q = binding.column_major(p.Q)
    s = binding.Solver(dA, p.n, tol=p.tol, maxit=p.maxit)
    (res,) = binding.solve_batch([s], [b], [x], [Q])
    s.close()
    return res, x.cpu().numpy()


g = np.random.default_rng(404)
A1 = np.diag([1.0, 0.0, 2.0])
A1[0, 1] = 0.5
CASES = [
    problem("N1_n1", [[2.0]], [4.0], np.array([[1.0]])),
    problem("N1_n3", [[2.0]], [4.0], np.array([[1.0, 2.0, 3.0]])),
    problem("N2_n3_eigvec", [[2.0, 1.0], [0.0, 3.0]], [1.0, 1.0], g.standard_normal((2, 3))),
    problem("N5_n7", np.eye(5) * 2 + np.diag(np.ones(4), 1), g.standard_normal(5), g.standard_normal((5, 7))),
    problem("consistent_singular", A1, A1 @ np.ones(3), g.standard_normal((3, 2)), maxit=30),
]


@pytest.mark.parametrize("p", CASES, ids=[c.name for c in CASES])
def test_degenerate_matches_oracle(p):
    o = oracle.mlbicgstabt(p.A, p.b, p.Q, tol=p.tol, maxit=p.maxit)
    for how, (res, x) in (("multi-launch", run_gpu(p)[:2]), ("batch", batch_solve(p))):
        print(f"{p.name} {how}: flag={res.flag} iter={res.iter} | oracle flag={o.flag} iter={o.iter}", flush=True)
        assert res.flag == o.flag
        assert res.iter == o.iter
        if o.flag == 0:
            assert rel(x, o.x) < 1e-10
            assert np.linalg.norm(p.b - p.A @ x) <= 1e-9 * np.linalg.norm(p.b)


def test_zero_matrix_breaks_down_at_once():
    """No entries at all (empty index and value arrays): c_0 = q^H A r_0 = 0, flag -1 at k = 0, x untouched."""
    p = problem("zero", np.zeros((3, 3)), np.ones(3), np.ones((3, 2)))
    assert p.A.nnz == 0
    o = oracle.mlbicgstabt(p.A, p.b, p.Q, tol=p.tol, maxit=p.maxit)
    assert o.flag == -1 and o.iter == 0
    for res, x in (run_gpu(p)[:2], batch_solve(p)):
        assert res.flag == -1 and res.iter == 0 and not x.any()


def test_inconsistent_singular_is_not_converged():
    """b outside the range of a singular A: both paths end without claiming convergence."""
    p = problem("inconsistent_singular", A1, np.ones(3), g.standard_normal((3, 2)), maxit=30)
    o = oracle.mlbicgstabt(p.A, p.b, p.Q, tol=p.tol, maxit=p.maxit)
    assert o.flag != 0
    for res, _ in (run_gpu(p)[:2], batch_solve(p)):
        assert res.flag != 0


@pytest.mark.parametrize("p", CASES, ids=[c.name for c in CASES])
def test_degenerate_transpose_free_matches_oracle(p):
    """The same cases without A^H, against the oracle's transpose-free variant."""
    o = oracle.mlbicgstabt(p.A, p.b, p.Q, tol=p.tol, maxit=p.maxit, transpose_free=True)
    res, x = run_gpu(p, transpose_free=True)[:2]
    print(f"{p.name} transpose-free: flag={res.flag} iter={res.iter} | oracle flag={o.flag} iter={o.iter}", flush=True)
    assert res.flag == o.flag
    assert res.iter == o.iter
    if o.flag == 0:
        assert rel(x, o.x) < 1e-10
        assert np.linalg.norm(p.b - p.A @ x) <= 1e-9 * np.linalg.norm(p.b)


def test_zero_matrix_transpose_free():
    p = problem("zero", np.zeros((3, 3)), np.ones(3), np.ones((3, 2)))
    res, x = run_gpu(p, transpose_free=True)[:2]
    assert res.flag == -1 and res.iter == 0 and not x.any()
