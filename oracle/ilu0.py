"""ILU(0), the incomplete LU factorisation without fill that the paper's experiments precondition
with (Section 5).  Test infrastructure only: the GPU library never imports this module.

Definition.  For A with a nonzero (block) diagonal, ILU(0) is M = L U with L unit lower triangular,
U upper triangular, L + U nonzero only where A is, and (L U)_ij = a_ij at every (i, j) where A is
nonzero.  Those equations fix L and U uniquely whenever the pivots u_kk are nonzero.  They are solved
here by Gaussian elimination restricted to A's pattern, row by row (the IKJ order): for row i and
each k < i where a_ik is stored, in increasing k,
    l_ik = a_ik / u_kk,   then   a_ij -= l_ik u_kj   for every stored j > k of row i with u_kj stored;
what is left in row i is l_i* below the diagonal and u_i* on and above it.

3x3-block matrices (BSR with 3x3 blocks) use the same steps on blocks: L has identity diagonal
blocks, U full diagonal blocks, l_ik = a_ik u_kk^{-1} and a_ij -= l_ik u_kj as 3x3 products.

The factors are returned as one matrix with A's sorted pattern (strictly lower part L, the rest U),
and ``ilu0_precond`` gives the pair (apply M^{-1}, apply M^{-H}) the ML(n)BiCGStabt oracle takes,
built from sparse triangular solves of scipy (library primitives).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _rows_sorted(A):
    """Row-wise {col: value} dicts of a CSR matrix (duplicates summed)."""
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.sort_indices()
    return [dict(zip(A.indices[A.indptr[i]:A.indptr[i + 1]].tolist(), A.data[A.indptr[i]:A.indptr[i + 1]]))
            for i in range(A.shape[0])]


def ilu0(A):
    """Point ILU(0) of a square scipy sparse (or dense) matrix; returns the combined factor as CSR with
    A's sorted pattern.  Raises ZeroDivisionError on a zero or missing pivot."""
    A = sp.csr_matrix(A)
    N = A.shape[0]
    dtype = np.result_type(A.dtype, np.float64)
    rows = _rows_sorted(A.astype(dtype))
    for i in range(N):
        ri = rows[i]
        cols = sorted(ri)
        for k in cols:
            if k >= i:
                break
            rk = rows[k]
            ukk = rk.get(k, 0)
            if ukk == 0:
                raise ZeroDivisionError(f"zero pivot in row {k}")
            lik = ri[k] / ukk
            ri[k] = lik
            for j in cols:
                if j > k and j in rk:
                    ri[j] = ri[j] - lik * rk[j]
        if ri.get(i, 0) == 0:
            raise ZeroDivisionError(f"zero pivot in row {i}")
    indptr = np.zeros(N + 1, dtype=np.int64)
    indices, data = [], []
    for i, ri in enumerate(rows):
        cols = sorted(ri)
        indices.extend(cols)
        data.extend(ri[c] for c in cols)
        indptr[i + 1] = len(indices)
    return sp.csr_matrix((np.array(data, dtype=dtype), np.array(indices), indptr), shape=(N, N))


def ilu0_bsr3(A):
    """Block ILU(0) of a BSR matrix with 3x3 blocks; returns the combined factor as BSR with A's sorted
    block pattern (blocks below the diagonal hold L, the others U).  Raises ZeroDivisionError on a
    singular or missing diagonal block."""
    A = sp.bsr_matrix(A, blocksize=(3, 3))
    A.sum_duplicates()
    A.sort_indices()
    nb = A.shape[0] // 3
    dtype = np.result_type(A.dtype, np.float64)
    rows = [dict(zip(A.indices[A.indptr[i]:A.indptr[i + 1]].tolist(),
                     [np.array(b, dtype=dtype) for b in A.data[A.indptr[i]:A.indptr[i + 1]]]))
            for i in range(nb)]
    for i in range(nb):
        ri = rows[i]
        cols = sorted(ri)
        for k in cols:
            if k >= i:
                break
            rk = rows[k]
            if k not in rk or np.linalg.cond(rk[k]) > 1 / np.finfo(float).eps:
                raise ZeroDivisionError(f"singular pivot block in block row {k}")
            lik = ri[k] @ np.linalg.inv(rk[k])
            ri[k] = lik
            for j in cols:
                if j > k and j in rk:
                    ri[j] = ri[j] - lik @ rk[j]
        if i not in ri or np.linalg.cond(ri[i]) > 1 / np.finfo(float).eps:
            raise ZeroDivisionError(f"singular pivot block in block row {i}")
    indptr = np.zeros(nb + 1, dtype=np.int64)
    indices, data = [], []
    for i, ri in enumerate(rows):
        cols = sorted(ri)
        indices.extend(cols)
        data.extend(ri[c] for c in cols)
        indptr[i + 1] = len(indices)
    return sp.bsr_matrix((np.array(data, dtype=dtype).reshape(-1, 3, 3), np.array(indices), indptr),
                         shape=(3 * nb, 3 * nb))


def factors(LU, block=1):
    """(L, U) as scalar CSR matrices from a combined factor: L = unit lower (block) triangle, U = the
    (block) diagonal and above."""
    if block == 1:
        C = sp.csr_matrix(LU)
        L = sp.tril(C, k=-1, format="csr") + sp.identity(C.shape[0], dtype=C.dtype, format="csr")
        U = sp.triu(C, k=0, format="csr")
        return L.tocsr(), U.tocsr()
    B = sp.bsr_matrix(LU)
    nb = B.shape[0] // 3
    rows = np.repeat(np.arange(nb), np.diff(B.indptr))
    low = B.indices < rows
    Lb = sp.bsr_matrix((B.data * low[:, None, None], B.indices, B.indptr), shape=B.shape)
    Ub = sp.bsr_matrix((B.data * (~low)[:, None, None], B.indices, B.indptr), shape=B.shape)
    L = Lb.tocsr() + sp.identity(B.shape[0], dtype=B.dtype, format="csr")
    L.eliminate_zeros()
    U = Ub.tocsr()
    U.eliminate_zeros()
    return L.tocsr(), U.tocsr()


def _splu_solve(lu, dtype, v):
    """lu.solve(v), also for a complex v with a real factor (real and imaginary parts solved apart)."""
    if np.iscomplexobj(v) and not np.issubdtype(dtype, np.complexfloating):
        return lu.solve(np.ascontiguousarray(v.real)) + 1j * lu.solve(np.ascontiguousarray(v.imag))
    return lu.solve(v)


def ilu0_precond(A):
    """(apply M^{-1}, apply M^{-H}) for M = ILU(0) of A (3x3 blocks when A is BSR with 3x3 blocks).

    M^{-1} v = U^{-1} (L^{-1} v); M^{-H} v = L^{-H} (U^{-H} v).  Point factors use scipy's sparse
    triangular solves; the block U, whose diagonal blocks are full, is solved through a sparse LU of U
    (exact for a triangular-by-blocks matrix)."""
    if sp.isspmatrix_bsr(A) and A.blocksize == (3, 3):
        L, U = factors(ilu0_bsr3(A), block=3)
        Ulu = spla.splu(U.tocsc())
        UHlu = spla.splu(U.conj().T.tocsc())
        LH = L.conj().T.tocsr()
        return (lambda v: _splu_solve(Ulu, U.dtype, spla.spsolve_triangular(L, v, lower=True, unit_diagonal=True)),
                lambda v: spla.spsolve_triangular(LH, _splu_solve(UHlu, U.dtype, v), lower=False,
                                                  unit_diagonal=True))
    L, U = factors(ilu0(A))
    LH, UH = L.conj().T.tocsr(), U.conj().T.tocsr()
    return (lambda v: spla.spsolve_triangular(U, spla.spsolve_triangular(L, v, lower=True, unit_diagonal=True),
                                              lower=False),
            lambda v: spla.spsolve_triangular(LH, spla.spsolve_triangular(UH, v, lower=True), lower=False,
                                              unit_diagonal=True))
