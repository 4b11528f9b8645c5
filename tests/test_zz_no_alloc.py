"""The allocation-free entry point (mlbicgstab_solve_noalloc) against create + solve + destroy.

Both run the same kernels with the same grids, so every result must be bitwise that of the
entry point with its own allocations: x, flag, iteration count and residuals.  Each case makes
two calls in a row, the second on a smaller system, so the second runs over the contents the
first left in the static scratch.
"""
import numpy as np
import pytest

import workloads
from tests.gpu_util import gpu_available, run_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1106_3678_amd import binding  # noqa: E402


def _upload(p):
    cplx = np.iscomplexobj(p.A.data) or np.iscomplexobj(p.b)
    dt = np.complex128 if cplx else np.float64
    dA = binding.to_device(p.A)
    b = torch.from_numpy(np.ascontiguousarray(p.b.astype(dt))).cuda()
    Q = binding.column_major(p.Q.astype(dt))
    return dA, b, Q, (torch.complex128 if cplx else torch.float64)


def _noalloc(p, transpose_free=False, order=0, record=0):
    dA, b, Q, tdt = _upload(p)
    x = torch.from_numpy(np.ascontiguousarray(p.x0.astype(np.complex128 if tdt == torch.complex128 else np.float64))).cuda()
    K = min(record, p.maxit)
    it = torch.zeros((K, p.N), dtype=tdt, device="cuda") if K else None
    print(f"[noalloc] {p.name} N={p.N} n={p.n} tf={transpose_free} order={order}", flush=True)
    res = binding.solve_noalloc(dA, b, x, Q, p.n, tol=p.tol, maxit=p.maxit, kappa=p.kappa, record_iterates=K,
                                iterates=it, transpose_free=transpose_free, order=order)
    torch.cuda.synchronize()
    return res, x.cpu().numpy(), (it.cpu().numpy() if it is not None else None)


def _same(p, transpose_free=False, order=0, record=0):
    r1, x1, i1 = _noalloc(p, transpose_free, order, record)
    r0, x0, i0 = run_gpu(p, record=record, transpose_free=transpose_free, order=order)
    assert r1.flag == r0.flag and r1.iter == r0.iter, (r1.flag, r0.flag, r1.iter, r0.iter)
    assert np.array_equal(x1, x0)
    assert r1.err_recursive == r0.err_recursive and r1.err_true == r0.err_true
    if record:
        assert np.array_equal(i1, i0)
    return r1


CASES = [
    # (larger system, smaller system): the second call reuses the scratch the first left behind
    ("csr_n4", lambda: workloads.config2(n=4, m=40), lambda: workloads.config1(n=4)),
    ("csr_n8_ragged", lambda: workloads.config2(n=8, m=33), lambda: workloads.config2(n=3, m=9)),
    ("complex_n16", lambda: workloads.config5(n=16, m=24), lambda: workloads.config5(n=5, m=10)),
    ("bsr3_n4", lambda: workloads.config3(n=4, grid=(8, 10, 6)), lambda: workloads.config3(n=2, grid=(5, 4, 3))),
]


@pytest.mark.parametrize("name,big,small", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("transpose_free", [False, True])
def test_noalloc_matches_create_solve(name, big, small, transpose_free):
    pb, ps = big(), small()
    assert ps.N < pb.N
    r = _same(pb, transpose_free=transpose_free, record=12)
    assert r.flag in (0, 1)
    _same(ps, transpose_free=transpose_free, record=5)


def test_noalloc_literal_order_and_kappa():
    p = workloads.config2(n=4, m=20)
    p.kappa = 0.7
    _same(p, order=binding.MLB_ORDER_LITERAL, record=8)
    _same(workloads.config1(n=3), order=binding.MLB_ORDER_LITERAL)


def test_noalloc_largest_fitting_system_and_rejection():
    """A 3D system just under the scratch limit runs; one just over it is refused before any work."""
    p = workloads.config2(n=4, m=66)    # 287,496 rows, about 62 MB of scratch with A^H
    r = _same(p)
    assert r.flag == 0
    big = workloads.config2(n=4, m=70)  # 343,000 rows: over the limit with A^H
    dA, b, Q, _ = _upload(big)
    x = torch.zeros(big.N, dtype=torch.float64, device="cuda")
    with pytest.raises(binding.MlbError) as e:
        binding.solve_noalloc(dA, b, x, Q, big.n, tol=big.tol, maxit=big.maxit)
    assert e.value.code == binding.MLB_EUNSUPPORTED and "bytes of scratch" in str(e.value)
    assert not x.any()
    # the same system fits without A^H
    r = _same(big, transpose_free=True)
    assert r.flag == 0


def test_noalloc_restarts_match_create_solve():
    """max_restarts through the allocation-free entry point.  A converged run whose true residual is
    not below tol is made by setting tol between the two residuals of a reference run at 1e-10 (the
    run then stops at the same iteration).  With max_restarts = 2 the solve restarts from its x, with
    every buffer in the static scratch, and the result is bitwise that of create + solve + destroy with
    the same options."""

    def create_solve(p, tol, mr):
        dA, b, Q, tdt = _upload(p)
        x = torch.zeros(p.N, dtype=tdt, device="cuda")
        s = binding.Solver(dA, p.n, tol=tol, maxit=p.maxit, max_restarts=mr)
        try:
            res = s.solve(b, x, Q)
            torch.cuda.synchronize()
        finally:
            s.close()
        return res, x.cpu().numpy()

    checked = 0
    for m, n in ((32, 2), (48, 8), (64, 2), (64, 4)):
        p = workloads.config1(n=n, m=m)
        ref, _ = create_solve(p, 1e-10, 0)
        if not ref.err_true > ref.err_recursive:
            continue
        tol = float(np.sqrt(ref.err_true * ref.err_recursive))
        r0, _ = create_solve(p, tol, 0)
        if not (r0.flag == 0 and r0.err_true >= tol):
            continue
        r2, x2 = create_solve(p, tol, 2)
        dA, b, Q, tdt = _upload(p)
        x = torch.zeros(p.N, dtype=tdt, device="cuda")
        print(f"[noalloc] restarts m={m} n={n} tol={tol:.4e}", flush=True)
        rn = binding.solve_noalloc(dA, b, x, Q, p.n, tol=tol, maxit=p.maxit, max_restarts=2)
        torch.cuda.synchronize()
        print(f"  create/solve: iter={r2.iter} restarts={r2.outer_iters} err_true={r2.err_true:.4e}; "
              f"noalloc: iter={rn.iter} restarts={rn.outer_iters} err_true={rn.err_true:.4e}")
        assert r2.flag == 0 and r2.outer_iters >= 1 and r2.err_true < tol
        assert (rn.flag, rn.iter, rn.outer_iters) == (r2.flag, r2.iter, r2.outer_iters)
        assert np.array_equal(x.cpu().numpy(), x2) and rn.err_true == r2.err_true
        checked += 1
    assert checked >= 1, "no candidate system showed a residual gap"
