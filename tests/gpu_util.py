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

    precond: 0 (none), 1 (block Jacobi of A) or a pair (apply M^{-1}, apply M^{-H}).
    Re-runs the oracle (a) with its inner products summed in other orders
    (correctly rounded, reversed) and (b) with b scaled entrywise by
    (1 + 1e-15 xi), xi ~ N(0, 1), n_perturb times (the k-th perturbed run sums
    in the k-th of the orders blas, exact, reversed).  Returns a dict: the max
    relative iterate change over k <= K ("iterates"), the max |iteration count
    change| ("iterations") and the range of counts over all runs, base included
    ("iter_min", "iter_max"), the largest true residual ("true_max") and the max
    relative change of the final x ("x").  Two correct fp64 implementations that
    only differ in rounding order cannot be expected to agree better than this.
    """
    it_spread, n_spread, true_max, x_spread = 0.0, 0, oracle.true_error(p.A, base.x, p.b), 0.0
    lo = hi = base.iter
    g = np.random.default_rng(1)
    variants = [("exact", p.b), ("reversed", p.b)]
    for k in range(n_perturb):
        variants.append((("blas", "exact", "reversed")[k % 3], p.b * (1 + 1e-15 * g.standard_normal(p.N))))
    pre = precond if isinstance(precond, tuple) else (block_jacobi(p.A) if precond else None)
    for summation, b in variants:
        o2 = oracle.mlbicgstabt(p.A, b, p.Q, x0=p.x0, tol=p.tol, maxit=p.maxit, kappa=p.kappa, record_x=K,
                                summation=summation, precond=pre, transpose_free=transpose_free)
        kk = min(K, o2.iter, base.iter)
        for k in range(kk):
            it_spread = max(it_spread, rel(o2.x_history[k], base.x_history[k]))
        n_spread = max(n_spread, abs(o2.iter - base.iter))
        lo, hi = min(lo, o2.iter), max(hi, o2.iter)
        true_max = max(true_max, oracle.true_error(p.A, o2.x, p.b))
        x_spread = max(x_spread, rel(o2.x, base.x))
    return {"iterates": it_spread, "iterations": n_spread, "iter_min": lo, "iter_max": hi, "true_max": true_max,
            "x": x_spread}


# Caps on the bars widened to the oracle's rounding spread: whatever the spread, a GPU result keeps its
# first iterates within 1e-6 and its final x within 1e-6 of the oracle's, and its iteration count within
# 15% of the oracle's (mode "sensitive") or of the range the oracle's own perturbed runs took (mode
# "chaotic", for the systems whose count moves by more than 15% under rounding alone).
CAP_ITERATES, CAP_ITERATIONS, CAP_X = 1e-6, 0.15, 1e-6


def parity_bars(p, o, K=20, mode="strict", precond=0, transpose_free=False, n_perturb=24, x_tol=1e-6,
                iterates_cap=CAP_ITERATES):
    """The bars one GPU result is held to against the oracle result o.

    strict   : x_1..x_K within 1e-8, iterations within 5% (at least 1), true residual below tol + 1e-12,
               final x within x_tol.
    sensitive: each bar widened to the oracle's spread under rounding (10x the iterate and x spread,
               2x the count spread, the oracle's own largest true residual), then capped as above.
    chaotic  : as sensitive, but the iteration count must lie in [0.85 min, 1.15 max] of the counts the
               oracle's own runs took.
    iterates_cap=None leaves the iterate bar at 10x the oracle's own spread (for systems whose early
    iterates the oracle itself moves by O(1) under rounding, where no iterate bar can discriminate).
    Returns a dict with iterate bar "it", count range "n_lo".."n_hi", residual bar "res", x bar "x"."""
    n_tol = max(1, int(0.05 * o.iter))
    b = {"it": 1e-8, "n_lo": o.iter - n_tol, "n_hi": o.iter + n_tol, "res": p.tol + 1e-12, "x": x_tol}
    if mode == "strict":
        return b
    s = oracle_spread(p, o, K, precond=precond, transpose_free=transpose_free, n_perturb=n_perturb)
    print(f"  oracle spread: iterates {s['iterates']:.2e} iterations {s['iterations']} "
          f"(range {s['iter_min']}..{s['iter_max']}) true residual {s['true_max']:.2e} x {s['x']:.2e}")
    b["it"] = max(b["it"], 10 * s["iterates"])
    if iterates_cap is not None:
        b["it"] = min(b["it"], iterates_cap)
    b["res"] = max(b["res"], s["true_max"])
    b["x"] = min(max(b["x"], 10 * s["x"]), CAP_X)
    if mode == "sensitive":
        n_tol = min(max(n_tol, 2 * s["iterations"]), max(1, int(CAP_ITERATIONS * o.iter)))
        b["n_lo"], b["n_hi"] = o.iter - n_tol, o.iter + n_tol
    else:
        b["n_lo"], b["n_hi"] = int((1 - CAP_ITERATIONS) * s["iter_min"]), int((1 + CAP_ITERATIONS) * s["iter_max"]) + 1
    return b


def check_against_bars(tag, p, res, x, its, o, b, K=20):
    """Asserts one GPU result against the bars of parity_bars, printing each achieved value beside its bar."""
    kk = min(K, o.iter, res.iter)
    worst_it = max((rel(its[k], o.x_history[k]) for k in range(kk)), default=0.0)
    x_rel = rel(x, o.x)
    print(f"{p.name}{tag}: N={p.N} n={p.n} gpu flag={res.flag} iter={res.iter} err={res.err_recursive:.3e} "
          f"true={res.err_true:.3e} | oracle flag={o.flag} iter={o.iter} err={o.err:.3e}", flush=True)
    print(f"  achieved / bar: iterates {worst_it:.2e} / {b['it']:.0e}, iterations {res.iter} in "
          f"[{b['n_lo']}, {b['n_hi']}], true residual {res.err_true:.2e} / {b['res']:.2e}, "
          f"x {x_rel:.2e} / {b['x']:.0e}", flush=True)
    assert res.flag == o.flag
    assert b["n_lo"] <= res.iter <= b["n_hi"], (res.iter, o.iter, b["n_lo"], b["n_hi"])
    for k in range(kk):
        assert rel(its[k], o.x_history[k]) < b["it"], (k + 1, rel(its[k], o.x_history[k]), b["it"])
    if o.flag == 0:
        assert res.err_true < b["res"], (res.err_true, b["res"])
        assert x_rel < b["x"], (x_rel, b["x"])
