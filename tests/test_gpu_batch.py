"""One-workgroup batched solves (mlbicgstab_solve_batch) against the CPU oracle.

Same bars as the multi-launch parity tests (same flag, iteration counts within
5%, x_1..x_20 within 1e-8 relative, true residual below tol, x within 1e-6 of
the oracle's x), plus: every system of a mixed batch gives bitwise the result
it gives in a batch of its own, and ineligible handles are refused.  Systems
created with transpose_free run the transpose-free steps and are checked
against the oracle's transpose-free variant.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from tests.gpu_util import gpu_available, rel, run_oracle

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_1106_3678_amd import binding  # noqa: E402


def prepare(p, record=0, maxit=None, transpose_free=False):
    cplx = np.iscomplexobj(p.A.data) or np.iscomplexobj(p.b)
    dt, nt = (torch.complex128, np.complex128) if cplx else (torch.float64, np.float64)
    dA = binding.to_device(p.A)
    b = torch.from_numpy(np.ascontiguousarray(p.b.astype(nt))).cuda()
    x = torch.from_numpy(np.ascontiguousarray(p.x0.astype(nt))).cuda()
    Q = binding.column_major(p.Q.astype(nt))
    mi = p.maxit if maxit is None else maxit
    K = min(record, mi)
    it = torch.zeros((K, p.N), dtype=dt, device="cuda") if K else None
    s = binding.Solver(dA, p.n, tol=p.tol, maxit=mi, kappa=p.kappa, record_iterates=K, iterates=it,
                       transpose_free=transpose_free)
    return dict(p=p, s=s, b=b, x=x, Q=Q, it=it, dA=dA)


def run_batch(items):
    torch.cuda.synchronize()
    res = binding.solve_batch([d["s"] for d in items], [d["b"] for d in items], [d["x"] for d in items],
                              [d["Q"] for d in items])
    out = []
    for d, r in zip(items, res):
        out.append((r, d["x"].cpu().numpy(), d["it"].cpu().numpy() if d["it"] is not None else None))
        d["s"].close()
    return out


def check(p, r, x, its, K=20, x_tol=1e-6, transpose_free=False):
    o = run_oracle(p, record=K, transpose_free=transpose_free)
    print(f"{p.name}: N={p.N} n={p.n} batch flag={r.flag} iter={r.iter} true={r.err_true:.3e} | "
          f"oracle flag={o.flag} iter={o.iter}", flush=True)
    assert r.flag == o.flag
    assert abs(r.iter - o.iter) <= max(1, int(0.05 * o.iter)), (r.iter, o.iter)
    if its is not None:
        for k in range(min(K, o.iter, r.iter)):
            assert rel(its[k], o.x_history[k]) < 1e-8, (k + 1, rel(its[k], o.x_history[k]))
    if o.flag == 0:
        assert r.err_true < p.tol + 1e-12
        assert rel(x, o.x) < x_tol


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_batch_of_one_convdiff2d(n):
    p = workloads.config1(n=n)
    (r, x, its), = run_batch([prepare(p, record=20)])
    check(p, r, x, its)


@pytest.mark.parametrize("n", [3, 16])
def test_batch_of_one_ragged_and_wide(n):
    """N = 33^2 (ragged against the 512-thread workgroup), odd n; n = 16 on a 3D grid."""
    p = workloads.config1(n=n, m=33) if n == 3 else workloads.config2(n=n, m=12, maxit=4000)
    (r, x, its), = run_batch([prepare(p, record=20)])
    check(p, r, x, its)


def test_batch_of_one_complex():
    p = workloads.config5(n=8, m=10, maxit=4000)
    (r, x, its), = run_batch([prepare(p, record=20)])
    check(p, r, x, its)


def mixed_problems():
    out = []
    for k, (dims, m, n) in enumerate([(2, 20, 2), (3, 9, 4), (2, 45, 8), (3, 14, 1), (2, 31, 4), (3, 11, 16),
                                      (2, 60, 4), (3, 17, 8)]):
        req = workloads.Request(k, 0.0, dims, m, 3.0 + 5 * k, n, 900 + k)
        out.append(workloads.serving_problem(req, maxit=5000))
    return out


def test_mixed_batch_equals_batches_of_one():
    """Systems of different N and n in one launch: bitwise the results of each system alone."""
    probs = mixed_problems()
    alone = [run_batch([prepare(p)])[0] for p in probs]
    mixed = run_batch([prepare(p) for p in probs])
    for p, (ra, xa, _), (rm, xm, _) in zip(probs, alone, mixed):
        assert rm.flag == ra.flag == 0, p.name
        assert rm.iter == ra.iter, p.name
        assert np.array_equal(xm, xa), p.name
    for p, (r, x, _) in zip(probs[:4], mixed[:4]):
        check(p, r, x, None)


def test_batch_matches_multi_launch_solve():
    """The batch kernel and the multi-launch iteration agree to rounding (iterations within 5%)."""
    p = workloads.config2(n=4, m=20, maxit=4000)
    d = prepare(p)
    r_single = d["s"].solve(d["b"], d["x"], d["Q"])
    x_single = d["x"].cpu().numpy()
    d["s"].close()
    (r, x, _), = run_batch([prepare(p)])
    assert r.flag == r_single.flag == 0
    assert abs(r.iter - r_single.iter) <= max(1, int(0.05 * r.iter))
    assert rel(x, x_single) < 1e-6


@pytest.mark.parametrize("N", [4, 7, 12])
def test_batch_finite_termination_dense(N):
    g = np.random.default_rng(N)
    A = sp.csr_matrix(g.standard_normal((N, N)) / np.sqrt(N) + 2 * np.eye(N))
    b = g.standard_normal(N)
    Q = np.asfortranarray(g.standard_normal((N, N + 1)))
    p = workloads.Problem(f"dense{N}", A, b, Q, np.zeros(N), N + 1, 1e-10, 100)
    (r, x, its), = run_batch([prepare(p, record=N)])
    check(p, r, x, its, K=N)
    assert r.iter == N
    assert rel(x, np.linalg.solve(A.toarray(), b)) < 1e-10


def test_batch_flags():
    """Breakdown (c_0 = 0), maxit, zero right-hand side and a converging system in one launch."""
    A = sp.csr_matrix(np.eye(3))
    bad = workloads.Problem("c0", A, np.array([1.0, 0, 0]), np.array([[0.0], [1.0], [0.0]]), np.zeros(3), 1, 1e-10,
                            10)
    p_max = workloads.config1(n=4)
    zero = workloads.config1(n=4)
    zero.b = np.zeros(zero.N)
    ok = workloads.config1(n=2)
    out = run_batch([prepare(bad), prepare(p_max, maxit=7), prepare(zero), prepare(ok)])
    (r0, _, _), (r1, _, _), (r2, x2, _), (r3, x3, _) = out
    assert r0.flag == -1 and r0.iter == 0
    o = run_oracle(p_max, maxit=7)
    assert r1.flag == o.flag == 1 and r1.iter == o.iter == 7
    assert r2.flag == 0 and r2.iter == 0 and not x2.any()
    check(ok, r3, x3, None)


def test_batch_refuses_ineligible():
    """BSR3, fp32-IR and preconditioned handles are refused before anything runs."""
    pb = workloads.config3(n=4, grid=(6, 8, 5))
    d = prepare(workloads.config1(n=4))
    dA = binding.to_device(pb.A)
    s_bsr = binding.Solver(dA, 4, tol=1e-10, maxit=100)
    s_ir = binding.Solver(d["dA"], 4, tol=1e-10, maxit=100, precision=binding.MLB_PREC_FP32_IR)
    for s in (s_bsr, s_ir):
        Qs = d["Q"] if s is s_ir else binding.column_major(pb.Q)
        bs = d["b"] if s is s_ir else torch.from_numpy(pb.b).cuda()
        xs = d["x"] if s is s_ir else torch.zeros(pb.N, dtype=torch.float64, device="cuda")
        with pytest.raises(binding.MlbError) as e:
            binding.solve_batch([d["s"], s], [d["b"], bs], [d["x"], xs], [d["Q"], Qs])
        assert e.value.code == binding.MLB_EUNSUPPORTED
        s.close()
    d["s"].close()


@pytest.mark.parametrize("case", ["2d_n4", "3d_n16", "complex_n8", "dense7"])
def test_batch_transpose_free(case):
    if case == "dense7":
        g = np.random.default_rng(7)
        A = sp.csr_matrix(g.standard_normal((7, 7)) / np.sqrt(7) + 2 * np.eye(7))
        p = workloads.Problem("dense7", A, g.standard_normal(7), np.asfortranarray(g.standard_normal((7, 8))),
                              np.zeros(7), 8, 1e-10, 100)
    else:
        p = {"2d_n4": lambda: workloads.config1(n=4), "3d_n16": lambda: workloads.config2(n=16, m=12, maxit=4000),
             "complex_n8": lambda: workloads.config5(n=8, m=10, maxit=4000)}[case]()
    (r, x, its), = run_batch([prepare(p, record=20, transpose_free=True)])
    check(p, r, x, its, transpose_free=True)
    if case == "dense7":
        assert r.iter == 7


def test_mixed_transpose_free_batch_equals_batches_of_one():
    """Systems with and without A^H in one launch: each bitwise its batch-of-one result."""
    probs = mixed_problems()[:6]
    flags = [k % 2 == 1 for k in range(len(probs))]
    alone = [run_batch([prepare(p, transpose_free=tf)])[0] for p, tf in zip(probs, flags)]
    mixed = run_batch([prepare(p, transpose_free=tf) for p, tf in zip(probs, flags)])
    for p, (ra, xa, _), (rm, xm, _) in zip(probs, alone, mixed):
        assert rm.flag == ra.flag == 0, p.name
        assert rm.iter == ra.iter, p.name
        assert np.array_equal(xm, xa), p.name
