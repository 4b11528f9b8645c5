"""Pins of the ILU(0) oracle (the preconditioner of the paper's experiments, Section 5), on the CPU.

ILU(0) is fixed by its definition: L unit lower and U upper triangular (by blocks for 3x3-block
matrices), nonzero only on A's pattern, with (L U)_ij = a_ij on that pattern.  The pins:
* that defining identity on convection-diffusion, random sparse, complex and reservoir-shaped block
  matrices (an exact statement, checked to rounding);
* on (block) tridiagonal matrices there is no fill, so ILU(0) is the exact LU: compared with an LU
  without pivoting written here (Doolittle), and ML(n)BiCGStabt preconditioned with it solves
  A M^{-1} y = b with A M^{-1} = I at the first step;
* an independent elimination in another loop order (KIJ, dense, fill dropped outside the pattern)
  gives the same factors;
* planted slips in a copy of the oracle fail these pins.
"""
import os
import sys
import types

import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle import mlbicgstabt
from oracle.ilu0 import factors, ilu0, ilu0_bsr3, ilu0_precond

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "ilu0.py")


def random_sparse_dd(N, density, seed, complex_=False):
    g = np.random.default_rng(seed)
    A = sp.random(N, N, density=density, random_state=np.random.RandomState(seed), format="csr")
    if complex_:
        A = A + 1j * sp.random(N, N, density=density, random_state=np.random.RandomState(seed + 1), format="csr")
    d = np.asarray(abs(A).sum(axis=1)).ravel() + 1.0 + g.random(N)
    return (A + sp.diags(d)).tocsr()


def pattern_identity_error(A, LU, block=1):
    """max |(L U - A)_ij| / max |a_ij| over A's pattern, and whether L + U lives on that pattern."""
    L, U = factors(LU, block)
    P = (L @ U).tocsr()
    As = sp.csr_matrix(A)
    As.sum_duplicates()
    mask = As.copy()
    mask.data = np.ones_like(mask.data)
    diff = (P - As).multiply(mask)
    on_pattern = ((abs(L) + abs(U)) - (abs(L) + abs(U)).multiply(mask.astype(bool)) -
                  sp.identity(A.shape[0]) * 0).nnz == 0
    return abs(diff).max() / abs(As).max(), on_pattern


def doolittle(A):
    """Dense LU without pivoting: A = L U, L unit lower."""
    A = np.array(A, dtype=np.result_type(A.dtype, np.float64))
    N = A.shape[0]
    L, U = np.eye(N, dtype=A.dtype), np.zeros_like(A)
    for i in range(N):
        for j in range(i, N):
            U[i, j] = A[i, j] - L[i, :i] @ U[:i, j]
        for j in range(i + 1, N):
            L[j, i] = (A[j, i] - L[j, :i] @ U[:i, i]) / U[i, i]
    return L, U


def kij_ilu0(A):
    """ILU(0) by dense elimination in KIJ order with every update outside A's pattern dropped."""
    D = np.array(A.toarray(), dtype=np.result_type(A.dtype, np.float64))
    P = A.toarray() != 0
    N = D.shape[0]
    for k in range(N - 1):
        for i in range(k + 1, N):
            if P[i, k]:
                D[i, k] /= D[k, k]
                for j in range(k + 1, N):
                    if P[i, j] and P[k, j]:
                        D[i, j] -= D[i, k] * D[k, j]
    return D


@pytest.mark.parametrize("case", ["convdiff2d", "random", "complex", "helmholtz"])
def test_point_ilu0_defining_identity(case):
    if case == "convdiff2d":
        A = workloads.convdiff_2d(14, pe=5.0)
    elif case == "random":
        A = random_sparse_dd(150, 0.04, 3)
    elif case == "complex":
        A = random_sparse_dd(120, 0.05, 5, complex_=True)
    else:
        A = workloads.helmholtz_3d(6, pe=2.0, k=3.0, gen=workloads.rng(99, 0))
    LU = ilu0(A)
    err, on_pattern = pattern_identity_error(A, LU)
    assert err < 1e-13 and on_pattern
    # the 2D / 3D stencils do fill in, so the identity must fail off the pattern (ILU(0) is not LU)
    if case in ("convdiff2d", "helmholtz"):
        L, U = factors(LU)
        assert abs((L @ U - A)).max() > 1e-6


@pytest.mark.parametrize("complex_", [False, True])
def test_point_ilu0_tridiagonal_is_exact_lu(complex_):
    g = np.random.default_rng(7)
    N = 40
    lo, di, up = g.standard_normal(N - 1), 4 + g.random(N), g.standard_normal(N - 1)
    if complex_:
        lo, up = lo + 1j * g.standard_normal(N - 1), up + 1j * g.standard_normal(N - 1)
    A = sp.diags([lo, di, up], [-1, 0, 1], format="csr")
    L, U = factors(ilu0(A))
    Ld, Ud = doolittle(A.toarray())
    assert np.abs(L.toarray() - Ld).max() < 1e-14 and np.abs(U.toarray() - Ud).max() < 1e-13


@pytest.mark.parametrize("case", ["random", "convdiff2d"])
def test_point_ilu0_matches_kij_elimination(case):
    A = random_sparse_dd(80, 0.06, 11) if case == "random" else workloads.convdiff_2d(9, pe=3.0)
    LU = ilu0(A).toarray()
    D = kij_ilu0(sp.csr_matrix(A))
    mask = sp.csr_matrix(A).toarray() != 0
    assert np.abs((LU - D)[mask]).max() < 1e-13 * np.abs(D).max()
    assert not LU[~mask].any()


@pytest.mark.parametrize("grid,complex_", [((5, 4, 3), False), ((4, 3, 3), True)])
def test_block_ilu0_defining_identity(grid, complex_):
    A = workloads.reservoir_bsr3(*grid, gen=workloads.rng(3, 9))
    if complex_:
        A = sp.bsr_matrix((A.data * (1 + 0.3j), A.indices, A.indptr), shape=A.shape)
    LU = ilu0_bsr3(A)
    err, on_pattern = pattern_identity_error(A, LU, block=3)
    assert err < 1e-12


def test_block_ilu0_block_tridiagonal_is_exact_lu():
    """A block-tridiagonal matrix has no fill: block ILU(0) is the exact block LU, and the scalar L U
    reproduces A everywhere."""
    g = np.random.default_rng(2)
    nb = 12
    blocks, cols, ptr = [], [], [0]
    for i in range(nb):
        for j in (i - 1, i, i + 1):
            if 0 <= j < nb:
                blk = g.standard_normal((3, 3)) + (12 * np.eye(3) if j == i else 0)
                blocks.append(blk)
                cols.append(j)
        ptr.append(len(cols))
    A = sp.bsr_matrix((np.array(blocks), np.array(cols), np.array(ptr)), shape=(3 * nb, 3 * nb))
    L, U = factors(ilu0_bsr3(A), block=3)
    assert abs(L @ U - A).max() < 1e-12
    # block LU, not scalar LU: U's diagonal blocks are full
    assert np.count_nonzero(np.tril(U.toarray(), -1)) > 0


@pytest.mark.parametrize("n", [1, 4])
def test_exact_ilu0_preconditioned_solve_stops_at_first_step(n):
    """With M = A (tridiagonal, so ILU(0) is exact) the iteration runs on A M^{-1} = I: alpha_1 = 1 and
    y_1 = b, so x_1 = M^{-1} b solves the system at k = 1."""
    g = np.random.default_rng(4)
    N = 30
    A = sp.diags([g.standard_normal(N - 1), 5 + g.random(N), g.standard_normal(N - 1)], [-1, 0, 1], format="csr")
    b = g.standard_normal(N)
    Q = np.asfortranarray(g.standard_normal((N, n)))
    res = mlbicgstabt(A, b, Q, tol=1e-10, maxit=20, precond=ilu0_precond(A))
    assert res.flag == 0 and res.iter == 1
    xs = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(res.x - xs) < 1e-12 * np.linalg.norm(xs)


def test_ilu0_precond_applies_inverse_and_adjoint():
    """apply M^{-1} and M^{-H} against dense solves with M = L U from the factors."""
    for A in (workloads.convdiff_2d(8, pe=4.0), random_sparse_dd(60, 0.08, 9, complex_=True),
              workloads.reservoir_bsr3(4, 3, 3, gen=workloads.rng(3, 1))):
        blk = 3 if sp.isspmatrix_bsr(A) else 1
        LU = ilu0_bsr3(A) if blk == 3 else ilu0(A)
        L, U = factors(LU, blk)
        M = (L @ U).toarray()
        mi, mh = ilu0_precond(A)
        v = np.random.default_rng(1).standard_normal(A.shape[0]) + 0j
        assert np.linalg.norm(mi(v) - np.linalg.solve(M, v)) < 1e-10 * np.linalg.norm(np.linalg.solve(M, v))
        assert np.linalg.norm(mh(v) - np.linalg.solve(M.conj().T, v)) < 1e-10 * np.linalg.norm(v)


def test_zero_pivot_raises():
    A = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 1.0]]))
    with pytest.raises(ZeroDivisionError):
        ilu0(A)


MUTATIONS = {
    "drop_update": ("ri[j] = ri[j] - lik * rk[j]", "ri[j] = ri[j]"),
    "no_scaling": ("lik = ri[k] / ukk", "lik = ri[k]"),
    "update_uses_a_not_u": ("if j > k and j in rk:\n                    ri[j] = ri[j] - lik * rk[j]",
                            "if j > k and j in rk:\n                    ri[j] = ri[j] - lik * A[k, j]"),
    "block_side": ("lik = ri[k] @ np.linalg.inv(rk[k])", "lik = np.linalg.inv(rk[k]) @ ri[k]"),
}


def _mutant(name):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert old in text, name
    mod = types.ModuleType(f"ilu0_mutant_{name}")
    mod.__package__ = "oracle"
    sys.modules[mod.__name__] = mod
    try:
        exec(compile(text.replace(old, new), f"<mutant {name}>", "exec"), mod.__dict__)
    finally:
        del sys.modules[mod.__name__]
    return mod


def _pins_hold(mod):
    try:
        for A in (workloads.convdiff_2d(8, pe=3.0), random_sparse_dd(60, 0.08, 3)):
            err, _ = pattern_identity_error(A, mod.ilu0(A))
            if not err < 1e-13:
                return False
        A = workloads.reservoir_bsr3(4, 3, 3, gen=workloads.rng(3, 2))
        err, _ = pattern_identity_error(A, mod.ilu0_bsr3(A), block=3)
        return err < 1e-12
    except Exception:
        return False


def test_unmutated_ilu0_passes():
    assert _pins_hold(sys.modules["oracle.ilu0"])   # the module (the package re-exports a function of that name)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_ilu0_mutation_is_caught(name):
    assert not _pins_hold(_mutant(name))
