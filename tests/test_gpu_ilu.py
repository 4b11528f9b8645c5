"""ILU(0) right preconditioning (the paper's preconditioner, Section 5) on the GPU against the oracle
preconditioned with oracle.ilu0 (point ILU(0) for CSR, 3x3-block ILU(0) for BSR3).

Same bars as the other parity tests: flag, iteration count within 5%, x_1..x_20 within 1e-8, true
residual below tol, x within 1e-6 -- strict everywhere except the ill-conditioned reservoir system,
whose early iterates the oracle itself moves by up to 120% under a 1e-15 perturbation of b (there
only the flag, the count, the residual and the final x are compared).  Also: a nonzero x_0 (the map y_0 = M x_0), the transpose-free and literal orders,
the 128^3 benchmark operator with n = 4 against the oracle run to convergence, one application of
M^{-1} and M^{-H} element by element (up to 128^3), and the errors.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from oracle.ilu0 import ilu0_precond
from tests.gpu_util import check_against_bars, gpu_available, parity_bars, run_gpu

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_1106_3678_amd import binding  # noqa: E402

ILU = binding.MLB_PRECOND_ILU0


def run_oracle_ilu(p, K=20, transpose_free=False, pre=None):
    return oracle.mlbicgstabt(p.A, p.b, p.Q, x0=p.x0, tol=p.tol, maxit=p.maxit, kappa=p.kappa, record_x=K,
                              precond=pre or ilu0_precond(p.A), transpose_free=transpose_free)


def check_ilu(p, K=20, mode="strict", transpose_free=False, order=0, iterates_cap=1e-6):
    res, x, its = run_gpu(p, record=K, precond=ILU, transpose_free=transpose_free, order=order)
    pre = ilu0_precond(p.A)
    o = run_oracle_ilu(p, K, transpose_free, pre)
    b = parity_bars(p, o, K, mode, precond=pre, transpose_free=transpose_free, n_perturb=6,
                    iterates_cap=iterates_cap)
    check_against_bars(" (ILU(0))", p, res, x, its, o, b, K)
    return res, x, o


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_convdiff2d_32(n):
    check_ilu(workloads.config1(n=n))


@pytest.mark.parametrize("n", [3, 5])
def test_convdiff2d_ragged(n):
    check_ilu(workloads.config1(n=n, m=33))


@pytest.mark.parametrize("n", [1, 4, 16])
def test_convdiff3d(n):
    check_ilu(workloads.config2(n=n, m=20, maxit=4000))


@pytest.mark.parametrize("n", [4, 8])
def test_complex(n):
    check_ilu(workloads.config5(n=n, m=12, maxit=4000))


@pytest.mark.parametrize("grid,n", [((8, 10, 6), 4), ((12, 16, 6), 8), ((9, 14, 7), 4)])
def test_bsr3_block_ilu_well_conditioned(grid, n):
    """Reservoir-shaped systems with the larger diagonal term: block ILU(0), strict bars."""
    check_ilu(workloads.config3(n=n, grid=grid, maxit=4000, accum=1.0))


def test_bsr3_block_ilu_benchmark_conditioning():
    """The benchmark's conditioning (12x16x6, n = 8): the oracle's count does not move under rounding
    here; strict bars."""
    check_ilu(workloads.config3(n=8, grid=(12, 16, 6), maxit=4000))


def test_bsr3_block_ilu_chaotic():
    """8x10x6 at the benchmark's conditioning: rounding alone moves the oracle's own x_1..x_20 by up to
    120% (a near-breakdown early in the iteration), so the iterates bound nothing here; the flag, the
    count (within 15% of the oracle's range), the true residual and the final x (1e-6) are checked."""
    check_ilu(workloads.config3(n=4, grid=(8, 10, 6), maxit=4000), mode="chaotic", iterates_cap=None)


def test_nonzero_initial_guess():
    p = workloads.config2(n=4, m=16, maxit=4000)
    p.x0 = np.random.default_rng(3).standard_normal(p.N)
    check_ilu(p)


@pytest.mark.parametrize("n", [4, 8])
def test_transpose_free(n):
    check_ilu(workloads.config2(n=n, m=16, maxit=4000), transpose_free=True)


def test_literal_order():
    check_ilu(workloads.config2(n=4, m=16, maxit=4000), order=binding.MLB_ORDER_LITERAL)


def test_kappa_guard():
    p = workloads.config1(n=4)
    p.kappa = 0.7
    check_ilu(p)


def test_full_size_convdiff3d_n4():
    """The 128^3 benchmark operator (N = 2,097,152) with ILU(0), n = 4, in the benchmark's launch
    configuration, against the oracle run to convergence."""
    p = workloads.config2(n=4, m=128)
    check_ilu(p)


def _apply_both(p, seed=5):
    """M^{-1} v and M^{-H} v from the library (mlbicgstab_matvec, ops MINV and MINVH: the one-launch
    triangular solves of every application) and from the oracle's ILU(0), for one seeded v; also a
    second MINV of the same v."""
    cplx = np.iscomplexobj(p.A.data)
    g = np.random.default_rng(seed)
    v = g.standard_normal(p.N) + (1j * g.standard_normal(p.N) if cplx else 0.0)
    s = binding.Solver(binding.to_device(p.A), p.n, tol=p.tol, maxit=p.maxit, precond=ILU)
    try:
        x = torch.from_numpy(np.ascontiguousarray(v)).cuda()
        y, yh, y2 = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
        s.matvec(x, y, binding.MLB_OP_MINV)
        s.matvec(x, yh, binding.MLB_OP_MINVH)
        s.matvec(x, y2, binding.MLB_OP_MINV)
        torch.cuda.synchronize()
    finally:
        s.close()
    apply, apply_h = ilu0_precond(p.A)
    return y.cpu().numpy(), yh.cpu().numpy(), y2.cpu().numpy(), apply(v), apply_h(v)


def _random_rows(N, per_row, seed, cplx=False, block=False):
    """A diagonally dominant matrix with about per_row random entries (3x3 blocks when block) a row:
    rows with more than 4 entries on each side of the diagonal, unlike the stencil matrices."""
    g = np.random.default_rng(seed)
    nb = N // 3 if block else N
    rows = np.repeat(np.arange(nb), per_row)
    P = sp.csr_matrix((np.ones(nb * per_row), (rows, g.integers(0, nb, nb * per_row))), shape=(nb, nb))
    P = (P + sp.identity(nb, format="csr")).tocsr()
    P.sum_duplicates()
    P.sort_indices()
    bs = 3 if block else 1
    data = g.standard_normal((P.nnz, bs, bs))
    if cplx:
        data = data + 1j * g.standard_normal((P.nnz, bs, bs))
    rowsum = np.zeros(nb)
    np.add.at(rowsum, np.repeat(np.arange(nb), np.diff(P.indptr)), np.abs(data).sum(axis=(1, 2)))
    for i in range(nb):   # diagonal (blocks) dominant
        for q in range(P.indptr[i], P.indptr[i + 1]):
            if P.indices[q] == i:
                data[q] += (rowsum[i] + 1.0) * np.eye(bs)
    if block:
        A = sp.bsr_matrix((data, P.indices, P.indptr), shape=(3 * nb, 3 * nb))
    else:
        A = sp.csr_matrix((data[:, 0, 0], P.indices, P.indptr), shape=(nb, nb))
    N = A.shape[0]
    dt = np.complex128 if cplx else np.float64
    return workloads.Problem("random_rows", A, np.ones(N, dtype=dt), np.ones((N, 1), dtype=dt), np.zeros(N, dtype=dt),
                             1, 1e-10, 100)


@pytest.mark.parametrize("case", ["2d", "2d_ragged", "3d", "complex", "bsr3", "bsr3_larger", "full_128", "csr_long_rows",
                                  "csr_long_rows_complex", "bsr3_long_rows_complex", "tiny_1", "tiny_7",
                                  "tiny_bsr3_2", "tiny_63"])
def test_apply_against_oracle(case):
    """One application of M^{-1} and of M^{-H} element by element against the oracle's factor and
    triangular solves.  Both sides form the same factor (the same products in the same order, up to
    the fma contraction) and substitute in row order, so they differ by rounding only (9.3e-16 of the
    largest entry at most in these cases); the bar is 1e-12 of it (the achieved value is printed).
    The random-pattern cases have rows with up to 14 entries on a side (the stencils at most 3), so
    the entries past a row's first four, loaded again on every try, are covered too, and complex
    3x3 blocks.  A second application of the
    same v is bitwise the first: each row's sum runs in entry order, whichever wave solves it and
    whenever the values it reads arrive."""
    p = {"2d": lambda: workloads.config1(n=4),
         "2d_ragged": lambda: workloads.config1(n=4, m=33),
         "3d": lambda: workloads.config2(n=4, m=20),
         "complex": lambda: workloads.config5(n=4, m=12),
         "bsr3": lambda: workloads.config3(n=4, grid=(8, 10, 6)),
         "bsr3_larger": lambda: workloads.config3(n=4, grid=(20, 60, 30)),
         "full_128": lambda: workloads.config2(n=4, m=128),
         "csr_long_rows": lambda: _random_rows(3000, 14, 1),
         "csr_long_rows_complex": lambda: _random_rows(2000, 14, 2, cplx=True),
         "bsr3_long_rows_complex": lambda: _random_rows(1200, 12, 3, cplx=True, block=True),
         # every level inside the first 64 positions: one wave, rows waiting on rows of the same wave
         "tiny_1": lambda: _random_rows(1, 1, 5),
         "tiny_7": lambda: _random_rows(7, 4, 6),
         "tiny_bsr3_2": lambda: _random_rows(6, 2, 7, cplx=True, block=True),
         "tiny_63": lambda: _random_rows(63, 5, 8)}[case]()
    y, yh, y2, yo, yho = _apply_both(p)
    for name, a, ref in (("M^-1", y, yo), ("M^-H", yh, yho)):
        err = np.max(np.abs(a - ref)) / np.max(np.abs(ref))
        print(f"{case} {name}: max |gpu - oracle| / max |oracle| = {err:.2e} (bar 1e-12)")
        assert np.all(np.isfinite(a)) and err <= 1e-12, (case, name, err)
    assert np.array_equal(y, y2), case


def test_restart_closes_residual_gap():
    """The reservoir system with ILU(0), n = 8 and the first right-hand side of the sequence
    benchmark (seed 1106): the iteration stops on its recursive residual with the true residual
    above tol.  With max_restarts the library starts again from the x it reached until the true
    residual is below tol; the first run is the same in both (bitwise), the restarted one adds
    iterations and reports the restarts."""
    p = workloads.config3(n=16)
    b = torch.from_numpy(np.random.default_rng(1106).standard_normal(p.N)).cuda()
    Q = binding.column_major(p.Q)[:, :8]
    dA = binding.to_device(p.A)
    out = {}
    for mr in (0, 3):
        x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
        s = binding.Solver(dA, 8, tol=p.tol, maxit=p.maxit, precond=ILU, max_restarts=mr)
        try:
            res = s.solve(b, x, Q)
            torch.cuda.synchronize()
        finally:
            s.close()
        out[mr] = res
        print(f"max_restarts={mr}: flag={res.flag} iter={res.iter} restarts={res.outer_iters} "
              f"err_true={res.err_true:.3e} err_recursive={res.err_recursive:.3e}")
    r0, r3 = out[0], out[3]
    assert r0.flag == 0 and r0.outer_iters == 0
    assert r3.flag == 0 and r3.err_true < p.tol
    if r0.err_true >= p.tol:
        assert r3.outer_iters >= 1 and r3.iter > r0.iter
    else:
        assert r3.outer_iters == 0 and r3.iter == r0.iter and r3.err_true == r0.err_true


def test_wait_give_up_reports_error(monkeypatch):
    """The bounded wait of the one-launch triangular solves, forced from the host: with
    MLB_ILU_MAX_TRIES=1 a row not ready at its first try gives up (stored as a quiet NaN, every
    launch still ends) and the solve returns MLB_EHIP.  On the 32 x 32 grid one wave claims the
    first 64 rows, which span several levels, so some row always waits.  A solver built without
    the limit then solves the same system normally."""
    p = workloads.config1(n=4)
    monkeypatch.setenv("MLB_ILU_MAX_TRIES", "1")
    with pytest.raises(binding.MlbError) as e:
        run_gpu(p, precond=ILU)
    assert e.value.code == binding.MLB_EHIP and "gave up" in str(e.value)
    monkeypatch.delenv("MLB_ILU_MAX_TRIES")
    res, x, _ = run_gpu(p, precond=ILU)
    assert res.flag == 0 and res.err_true < p.tol


def _solver_error(A, opt_precond=ILU, precision=0):
    p = workloads.Problem("e", A, np.ones(A.shape[0]), np.ones((A.shape[0], 1)), np.zeros(A.shape[0]), 1,
                          1e-10, 10)
    with pytest.raises(binding.MlbError) as e:
        run_gpu(p, precond=opt_precond, precision=precision)
    return e.value


def test_errors():
    # no stored diagonal in row 1
    A = sp.csr_matrix(np.array([[2.0, 1.0, 0.0], [1.0, 0.0, 1.0], [0.0, 1.0, 2.0]]))
    A.eliminate_zeros()
    err = _solver_error(A)
    assert err.code == binding.MLB_EINVAL and "diagonal" in str(err)
    # a zero pivot: u_11 = 1 - 1 = 0
    A = sp.csr_matrix(np.array([[1.0, 1.0], [1.0, 1.0]]))
    err = _solver_error(A)
    assert err.code == binding.MLB_EINVAL and "pivot" in str(err)
    # a column stored twice in one row
    A = sp.csr_matrix((np.array([2.0, 1.0, 1.0, 2.0]), np.array([0, 1, 1, 1]), np.array([0, 1, 4])), shape=(2, 2))
    err = _solver_error(A)
    assert err.code == binding.MLB_EINVAL and "twice" in str(err)
    # fp32 refinement is not combined with ILU(0)
    err = _solver_error(sp.identity(4, format="csr"), precision=binding.MLB_PREC_FP32_IR)
    assert err.code == binding.MLB_EUNSUPPORTED
