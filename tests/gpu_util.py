"""Shared helpers of the GPU parity tests: run the HIP library and the CPU oracle on one problem."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")


def gpu_available():
    return torch.cuda.is_available()


def block_jacobi(A):
    """(apply M^{-1}, apply M^{-H}) for M = the block diagonal of A (3x3 blocks for BSR, else the diagonal),
    built from A's entries with numpy."""
    import scipy.sparse as sp

    if sp.isspmatrix_bsr(A):
        nb = A.shape[0] // 3
        blocks = np.zeros((nb, 3, 3), dtype=A.dtype)
        for r in range(nb):
            for q in range(A.indptr[r], A.indptr[r + 1]):
                if A.indices[q] == r:
                    blocks[r] = A.data[q]
        Minv = np.linalg.inv(blocks)
        MinvH = np.conj(np.transpose(Minv, (0, 2, 1)))
        return (lambda v: np.einsum("rij,rj->ri", Minv, v.reshape(nb, 3)).reshape(-1),
                lambda v: np.einsum("rij,rj->ri", MinvH, v.reshape(nb, 3)).reshape(-1))
    d = A.diagonal()
    return (lambda v: v / d, lambda v: v / np.conj(d))


def run_gpu(p, precision=0, record=0, inner_tol=0.0, maxit=None, kappa=None, precond=0, transpose_free=False,
            order=0):
    """Solve problem p on the GPU; returns (result, x, iterates or None)."""
    from paper_1106_3678_amd import binding

    dA = binding.to_device(p.A)
    cplx = np.iscomplexobj(p.A.data) or np.iscomplexobj(p.b)
    dt = torch.complex128 if cplx else torch.float64
    b = torch.from_numpy(np.ascontiguousarray(p.b.astype(np.complex128 if cplx else np.float64))).cuda()
    x = torch.from_numpy(np.ascontiguousarray(p.x0.astype(np.complex128 if cplx else np.float64))).cuda()
    Q = binding.column_major(p.Q.astype(np.complex128 if cplx else np.float64))
    mi = p.maxit if maxit is None else maxit
    K = min(record, mi)
    it = torch.zeros((K, p.N), dtype=dt, device="cuda") if K else None
    s = binding.Solver(dA, p.n, tol=p.tol, maxit=mi, kappa=p.kappa if kappa is None else kappa,
                       precision=precision, inner_tol=inner_tol, record_iterates=K, iterates=it, precond=precond,
                       transpose_free=transpose_free, order=order)
    try:
        res = s.solve(b, x, Q)
        torch.cuda.synchronize()
    finally:
        s.close()
    xs = x.cpu().numpy()
    its = it.cpu().numpy() if it is not None else None
    return res, xs, its


def run_oracle(p, record=0, maxit=None, kappa=None, precond=0, summation="blas", transpose_free=False):
    pre = block_jacobi(p.A) if precond else None
    return oracle.mlbicgstabt(p.A, p.b, p.Q, x0=p.x0, tol=p.tol, maxit=p.maxit if maxit is None else maxit,
                              kappa=p.kappa if kappa is None else kappa, record_x=record, precond=pre,
                              summation=summation, transpose_free=transpose_free)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def iters_close(a, b):
    """Iteration counts within 5% (at least 1 apart allowed for short runs)."""
    return abs(a - b) <= max(1, int(0.05 * max(a, b)))


def oracle_spread(p, base, K=20, precond=0, transpose_free=False, n_perturb=1):
    """How far the oracle itself moves under rounding-level changes.

    Re-runs the oracle (a) with its inner products summed in other orders
    (correctly rounded, reversed) and (b) with b scaled entrywise by
    (1 + 1e-15 xi), xi ~ N(0, 1), n_perturb times (the k-th perturbed run sums
    in the k-th of the orders blas, exact, reversed).  Returns (max relative
    iterate change over k <= K, max |iteration count change|, max true residual,
    max relative change of the final x).  Two correct fp64 implementations that
    only differ in rounding order cannot be expected to agree better than this.
    """
    it_spread, n_spread, true_max, x_spread = 0.0, 0, oracle.true_error(p.A, base.x, p.b), 0.0
    g = np.random.default_rng(1)
    variants = [("exact", p.b), ("reversed", p.b)]
    for k in range(n_perturb):
        variants.append((("blas", "exact", "reversed")[k % 3], p.b * (1 + 1e-15 * g.standard_normal(p.N))))
    for summation, b in variants:
        o2 = oracle.mlbicgstabt(p.A, b, p.Q, x0=p.x0, tol=p.tol, maxit=p.maxit, kappa=p.kappa, record_x=K,
                                summation=summation, precond=block_jacobi(p.A) if precond else None,
                                transpose_free=transpose_free)
        kk = min(K, o2.iter, base.iter)
        for k in range(kk):
            it_spread = max(it_spread, rel(o2.x_history[k], base.x_history[k]))
        n_spread = max(n_spread, abs(o2.iter - base.iter))
        true_max = max(true_max, oracle.true_error(p.A, o2.x, p.b))
        x_spread = max(x_spread, rel(o2.x, base.x))
    return it_spread, n_spread, true_max, x_spread
