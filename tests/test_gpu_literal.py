"""GPU parity of the literal recurrence order (options.order = MLB_ORDER_LITERAL) against the oracle.

The oracle runs the beta~ and beta loops of Algorithm 7.1 in their sequential order, one
inner product per coefficient; so does this mode (one reduction per coefficient).  Bars as
for the fused order: same flag, iteration counts within 5%, x_1..x_20 within 1e-8 relative,
true residual below tol, x within 1e-6 of the oracle's x; widened to the oracle's own
rounding-level spread on the ill-conditioned block system.  Also: agreement with the fused
order, bitwise reruns, the fp32 refinement mode, the kernel timer, refusal by the batch kernel,
and the 128^3 workload's first iterates in the benchmark's launch configuration.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from tests.gpu_util import check_against_bars, gpu_available, parity_bars, rel, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_1106_3678_amd import binding  # noqa: E402

LIT = binding.MLB_ORDER_LITERAL


def check_literal(p, K=20, x_tol=1e-6, mode="strict", precond=0):
    res, x, its = run_gpu(p, record=K, precond=precond, order=LIT)
    o = run_oracle(p, record=K, precond=precond)
    b = parity_bars(p, o, K, mode, precond=precond, x_tol=x_tol)
    check_against_bars(" (literal)", p, res, x, its, o, b, K)
    return res, x, o


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_convdiff2d_32(n):
    check_literal(workloads.config1(n=n))


@pytest.mark.parametrize("n", [3, 5])
def test_convdiff2d_ragged(n):
    check_literal(workloads.config1(n=n, m=33))


@pytest.mark.parametrize("n", [4, 16])
def test_convdiff3d_small(n):
    check_literal(workloads.config2(n=n, m=16, maxit=4000))


@pytest.mark.parametrize("n", [4, 16])
def test_complex_small(n):
    check_literal(workloads.config5(n=n, m=10, maxit=4000))


@pytest.mark.parametrize("precond", [0, 1])
def test_bsr3_small(precond):
    check_literal(workloads.config3(n=4, grid=(8, 10, 6)), precond=precond,
                  mode="sensitive" if precond else "chaotic")


@pytest.mark.parametrize("N", [4, 7, 12])
def test_finite_termination_dense(N):
    g = np.random.default_rng(N)
    A = sp.csr_matrix(g.standard_normal((N, N)) / np.sqrt(N) + 2 * np.eye(N))
    b = g.standard_normal(N)
    Q = np.asfortranarray(g.standard_normal((N, N + 1)))
    p = workloads.Problem(f"dense{N}", A, b, Q, np.zeros(N), N + 1, 1e-10, 100)
    res, x, _ = check_literal(p, K=N)
    assert res.iter == N
    assert rel(x, np.linalg.solve(A.toarray(), b)) < 1e-10


def test_literal_and_fused_agree():
    """The two orders are the same iteration in exact arithmetic."""
    p = workloads.config2(n=8, m=24)
    rl, xl, il = run_gpu(p, record=20, order=LIT)
    rf, xf, if_ = run_gpu(p, record=20)
    assert rl.flag == rf.flag == 0
    assert abs(rl.iter - rf.iter) <= max(1, int(0.05 * rf.iter))
    for k in range(20):
        assert rel(il[k], if_[k]) < 1e-8
    assert rel(xl, xf) < 1e-6


def test_deterministic_rerun():
    p = workloads.config2(n=4, m=24)
    runs = [run_gpu(p, order=LIT)[:2] for _ in range(3)]
    for res, x in runs[1:]:
        assert res.iter == runs[0][0].iter
        assert np.array_equal(x, runs[0][1])


def test_fp32_refinement():
    p = workloads.config2(n=4, m=24)
    res, x, _ = run_gpu(p, precision=binding.MLB_PREC_FP32_IR, order=LIT)
    assert res.flag == 0 and res.err_true < p.tol
    assert rel(x, run_oracle(p).x) < 1e-6


def test_kernel_timer_and_batch_refusal():
    p = workloads.config1(n=4)
    dA = binding.to_device(p.A)
    b = torch.from_numpy(p.b).cuda()
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    Q = binding.column_major(p.Q)
    s = binding.Solver(dA, 4, tol=p.tol, maxit=p.maxit, order=LIT)
    assert s.solve(b, x, Q).flag == 0
    for k in (binding.MLB_KERNEL_SPMV_STEP, binding.MLB_KERNEL_ALPHA_STEP, binding.MLB_KERNEL_COMBINE,
              binding.MLB_KERNEL_RECOMBINE):
        assert 0 < s.time_kernel(k, 3) < 10
    with pytest.raises(binding.MlbError) as e:
        binding.solve_batch([s], [b], [x], [Q])
    assert e.value.code == binding.MLB_EUNSUPPORTED
    s.close()


def test_full_size_convdiff3d_first_iterates():
    """128^3 (N = 2,097,152), n = 4, literal order, benchmark launch configuration."""
    import oracle as orc

    p = workloads.config2(n=4, m=128)
    res, x, its = run_gpu(p, record=20, order=LIT)
    o = orc.mlbicgstabt(p.A, p.b, p.Q, tol=p.tol, maxit=20, record_x=20)
    worst = max(rel(its[k], o.x_history[k]) for k in range(20))
    print(f"full size literal: iter={res.iter} err_true={res.err_true:.3e} x_1..x_20 worst rel {worst:.2e}")
    for k in range(20):
        assert rel(its[k], o.x_history[k]) < 1e-8, (k + 1, rel(its[k], o.x_history[k]))
    assert res.flag == 0
    true = orc.true_error(p.A, x, p.b)
    assert true < p.tol + 1e-12
    assert abs(true - res.err_true) < 1e-12
