"""The library's sparse products on their own (mlbicgstab_matvec) against scipy in fp64.

y = A x is the product every step of Algorithm 7.1 forms; y = A^H x is the one that builds
f_s = A^H q_s (Algorithm 4.1, step 2).  Both are plain definitions, so the reference is
scipy's CSR product.  Bar, element by element: |y_i - ref_i| <= 4 k_i u (|A| |x|)_i with k_i
the stored entries of row i and u = 2^-53 (the error bound of a length-k dot product).
Cases cover every SpMV kernel the library picks: wave-local CSR (up to 8 entries a row),
the LDS tile (longer rows), wave-local 3x3 blocks (4 and 8 lanes a block row), the LDS tile
for 3x3 blocks (12 and 24 blocks a row), complex values, ragged sizes, a
solver before and after a solve, an A with no entries, N = 1, and the 128^3 operator of the
benchmark.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from tests.gpu_util import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_1106_3678_amd import binding  # noqa: E402

U = 2.0 ** -53


def _vec(N, seed, cplx):
    g = np.random.default_rng(seed)
    v = g.standard_normal(N)
    return v + 1j * g.standard_normal(N) if cplx else v


def _check(A, y, x):
    A = sp.csr_matrix(A)
    ref = A @ x
    mag = abs(A) @ np.abs(x)
    k = np.diff(A.indptr)
    bound = 4 * np.maximum(k, 1) * U * mag + 1e-300
    err = np.abs(y - ref)
    worst = float(np.max(err / bound)) if len(err) else 0.0
    assert worst <= 1.0, worst
    return worst


def _solver(A, n=4, **kw):
    dA = binding.to_device(A)
    return dA, binding.Solver(dA, n, tol=1e-10, maxit=100, **kw)


def _apply(s, x, op):
    dx = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    dy = torch.full_like(dx, float("nan"))
    s.matvec(dx, dy, op)
    return dy.cpu().numpy()


def _long_rows(N, per_row, seed):
    g = np.random.default_rng(seed)
    rows = np.repeat(np.arange(N), per_row)
    cols = g.integers(0, N, N * per_row)
    A = sp.csr_matrix((g.standard_normal(N * per_row), (rows, cols)), shape=(N, N))
    A.sum_duplicates()
    return A + sp.identity(N, format="csr") * per_row


def _bsr3(nb, per_row, seed, cplx=False):
    """3x3 blocks: the diagonal plus per_row random blocks a block row."""
    g = np.random.default_rng(seed)
    rows = np.repeat(np.arange(nb), per_row)
    P = sp.csr_matrix((np.ones(nb * per_row), (rows, g.integers(0, nb, nb * per_row))), shape=(nb, nb))
    P = (P + sp.identity(nb, format="csr")).tocsr()
    P.sum_duplicates()
    P.sort_indices()
    data = g.standard_normal((P.nnz, 3, 3))
    if cplx:
        data = data + 1j * g.standard_normal((P.nnz, 3, 3))
    return sp.bsr_matrix((data, P.indices, P.indptr), shape=(3 * nb, 3 * nb))


CASES = {
    "bsr3_2_blocks_a_row": lambda: _bsr3(1001, 1, 2),
    "bsr3_12_blocks_a_row": lambda: _bsr3(1001, 11, 3),
    "bsr3_24_blocks_a_row_complex": lambda: _bsr3(517, 23, 4, cplx=True),
    "convdiff2d_33": lambda: workloads.config1(n=4, m=33).A,
    "convdiff3d_16": lambda: workloads.config2(n=4, m=16).A,
    "long_rows_40": lambda: _long_rows(3001, 40, 1),
    "reservoir_8x10x6": lambda: workloads.config3(n=4, grid=(8, 10, 6)).A,
    "helmholtz_10": lambda: workloads.config5(n=4, m=10).A,
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_A_and_AH(case):
    A = CASES[case]()
    cplx = np.iscomplexobj(A.data)
    N = A.shape[0]
    dA, s = _solver(A)
    try:
        for op, M in ((binding.MLB_OP_A, A), (binding.MLB_OP_AH, A.conj().T)):
            x = _vec(N, 7 + op, cplx)
            w = _check(M, _apply(s, x, op), x)
            print(f"{case} op={op}: N={N} worst error / bound {w:.2e}", flush=True)
    finally:
        s.close()


def test_after_a_solve_and_repeated():
    """A finished solve leaves its done flag set; the product still runs, and reruns are bitwise."""
    p = workloads.config1(n=4, m=32)
    dA, s = _solver(p.A)
    try:
        x0 = torch.zeros(p.N, dtype=torch.float64, device="cuda")
        assert s.solve(torch.from_numpy(p.b).cuda(), x0, binding.column_major(p.Q)).flag == 0
        x = _vec(p.N, 3, False)
        y1 = _apply(s, x, binding.MLB_OP_A)
        y2 = _apply(s, x, binding.MLB_OP_A)
        _check(p.A, y1, x)
        assert np.array_equal(y1, y2)
        # the product of the solution is b up to the converged residual
        r = p.b - _apply(s, x0.cpu().numpy(), binding.MLB_OP_A)
        assert np.linalg.norm(r) / np.linalg.norm(p.b) < 1e-9
    finally:
        s.close()


def test_preconditioned_and_transpose_free_solvers():
    """op A is the caller's A in every mode; A^H is held only by the plain iteration."""
    A = workloads.config3(n=4, grid=(8, 10, 6)).A
    x = _vec(A.shape[0], 5, False)
    for kw in ({"precond": binding.MLB_PRECOND_JACOBI}, {"transpose_free": True}):
        dA, s = _solver(A, **kw)
        try:
            _check(A, _apply(s, x, binding.MLB_OP_A), x)
            with pytest.raises(binding.MlbError) as e:
                _apply(s, x, binding.MLB_OP_AH)
            assert e.value.code == binding.MLB_EUNSUPPORTED
        finally:
            s.close()


def test_bad_op_and_shapes():
    A = workloads.config1(n=4, m=8).A
    dA, s = _solver(A)
    try:
        x = torch.zeros(A.shape[0], dtype=torch.float64, device="cuda")
        with pytest.raises(binding.MlbError) as e:
            s.matvec(x, torch.empty_like(x), 4)
        assert e.value.code == binding.MLB_EINVAL
        for op in (binding.MLB_OP_MINV, binding.MLB_OP_MINVH):   # no ILU(0) preconditioner here
            with pytest.raises(binding.MlbError) as e:
                s.matvec(x, torch.empty_like(x), op)
            assert e.value.code == binding.MLB_EUNSUPPORTED
        with pytest.raises(ValueError):
            s.matvec(x[:-1], torch.empty_like(x))
    finally:
        s.close()


def test_full_size_convdiff3d():
    """The 128^3 operator (N = 2,097,152) of the benchmark, both products."""
    A = workloads.config2(n=4, m=128).A
    dA, s = _solver(A)
    try:
        for op, M in ((binding.MLB_OP_A, A), (binding.MLB_OP_AH, A.T)):
            x = _vec(A.shape[0], 11, False)
            print(f"128^3 op={op}: worst error / bound {_check(M, _apply(s, x, op), x):.2e}", flush=True)
    finally:
        s.close()


def test_no_entries_and_one_row():
    """An A with empty index and value arrays gives y = 0 exactly; N = 1 gives the one product."""
    Z = sp.csr_matrix((3, 3))
    assert Z.nnz == 0
    dA, s = _solver(Z, n=2)
    try:
        for op in (binding.MLB_OP_A, binding.MLB_OP_AH):
            y = _apply(s, _vec(3, 1, False), op)
            assert np.array_equal(y, np.zeros(3))
    finally:
        s.close()
    one = sp.csr_matrix(np.array([[2.5 - 1.5j]]))
    dA, s = _solver(one, n=1)
    try:
        x = np.array([0.75 + 2.0j])
        assert _apply(s, x, binding.MLB_OP_A)[0] == (2.5 - 1.5j) * x[0]
        assert _apply(s, x, binding.MLB_OP_AH)[0] == (2.5 + 1.5j) * x[0]
    finally:
        s.close()


def test_fp32_refinement_solver_uses_fp64_products():
    """An fp32-IR solver iterates on an fp32 copy; its products are the fp64 ones, bitwise."""
    p = workloads.config2(n=4, m=16)
    x = _vec(p.N, 9, False)
    ys = []
    for prec in (binding.MLB_PREC_FP64, binding.MLB_PREC_FP32_IR):
        dA, s = _solver(p.A, precision=prec)
        try:
            ys.append([_apply(s, x, op) for op in (binding.MLB_OP_A, binding.MLB_OP_AH)])
        finally:
            s.close()
    _check(p.A, ys[1][0], x)
    _check(p.A.T, ys[1][1], x)
    assert np.array_equal(ys[0][0], ys[1][0]) and np.array_equal(ys[0][1], ys[1][1])
