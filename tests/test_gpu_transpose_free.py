"""GPU parity of the transpose-free iteration (options.transpose_free = 1) against the oracle's
transpose-free variant, element by element.

Bars as for Algorithm 7.1 (same flag, iteration counts within 5%, x_1..x_20 within
1e-8 relative, true residual below tol, x within 1e-6 of the oracle's x).  On the
ill-conditioned block system the recursive residual drifts from the true one on
both sides (the drift Section 5.1 reports for the A^H-free second algorithm), so
there each bar is widened to the oracle's own rounding-level spread.  That spread
is sampled over 24 perturbed runs: the drifted final true residual is chaotic under
rounding (2e-11 to 4.3e-9 across 24 oracle runs of the 8x10x6 block-Jacobi case),
so a sample of three understates it.
Also: bitwise reruns, finite termination, the fp32 refinement and preconditioned
modes, sequences and serving (worker and batch paths), the kernel timer, and the
128^3 workload's first iterates in the benchmark's launch configuration.
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


def check_tf(p, K=20, x_tol=1e-6, mode="strict", precond=0):
    res, x, its = run_gpu(p, record=K, precond=precond, transpose_free=True)
    o = run_oracle(p, record=K, precond=precond, transpose_free=True)
    b = parity_bars(p, o, K, mode, precond=precond, transpose_free=True, x_tol=x_tol)
    check_against_bars(" (transpose-free)", p, res, x, its, o, b, K)
    return res, x, o


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_convdiff2d_32(n):
    check_tf(workloads.config1(n=n))


@pytest.mark.parametrize("n", [3, 5])
def test_convdiff2d_ragged(n):
    """N = 33^2 against the 256-thread workgroups; odd n against the n buckets."""
    check_tf(workloads.config1(n=n, m=33))


@pytest.mark.parametrize("n", [4, 16])
def test_convdiff3d_small(n):
    check_tf(workloads.config2(n=n, m=16, maxit=4000))


@pytest.mark.parametrize("n", [4, 16])
def test_complex_small(n):
    check_tf(workloads.config5(n=n, m=10, maxit=4000))


@pytest.mark.parametrize("grid,n", [((8, 10, 6), 4), ((12, 16, 6), 8)])
def test_bsr3_small(grid, n):
    """Benchmark conditioning, no preconditioner: the oracle's own count is chaotic under rounding."""
    check_tf(workloads.config3(n=n, grid=grid), mode="chaotic")


def test_bsr3_block_jacobi():
    check_tf(workloads.config3(n=4, grid=(8, 10, 6)), precond=1, mode="sensitive")


@pytest.mark.parametrize("N", [4, 7, 12])
def test_finite_termination_dense(N):
    g = np.random.default_rng(N)
    A = sp.csr_matrix(g.standard_normal((N, N)) / np.sqrt(N) + 2 * np.eye(N))
    b = g.standard_normal(N)
    Q = np.asfortranarray(g.standard_normal((N, N + 1)))
    p = workloads.Problem(f"dense{N}", A, b, Q, np.zeros(N), N + 1, 1e-10, 100)
    res, x, _ = check_tf(p, K=N)   # (result, x, oracle result)
    assert res.iter == N
    assert rel(x, np.linalg.solve(A.toarray(), b)) < 1e-10


def test_deterministic_rerun():
    p = workloads.config2(n=8, m=24)
    runs = [run_gpu(p, transpose_free=True)[:2] for _ in range(3)]
    for res, x in runs[1:]:
        assert res.iter == runs[0][0].iter
        assert np.array_equal(x, runs[0][1])


def test_fp32_refinement():
    """fp32 inner iteration without A^H inside fp64 refinement: the true residual meets tol."""
    p = workloads.config2(n=4, m=24)
    res, x, _ = run_gpu(p, precision=binding.MLB_PREC_FP32_IR, transpose_free=True)
    print(f"IR transpose-free: flag={res.flag} iter={res.iter} outer={res.outer_iters} true={res.err_true:.3e}")
    assert res.flag == 0 and res.err_true < p.tol
    o = run_oracle(p, transpose_free=True)
    assert rel(x, o.x) < 1e-6


def test_sequence_and_server_match_plain_solves():
    """A fixed-n sequence and a served request give bitwise the plain transpose-free solve."""
    p = workloads.config1(n=4, m=40)
    dA = binding.to_device(p.A)
    b = torch.from_numpy(p.b).cuda()
    Q = binding.column_major(p.Q)
    x0 = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    s = binding.Solver(dA, 4, tol=p.tol, maxit=p.maxit, transpose_free=True)
    r0 = s.solve(b, x0, Q)
    s.close()
    x1 = torch.zeros_like(x0)
    seq = binding.Sequence(dA, 4, 1, 4, 0, tol=p.tol, maxit=p.maxit, transpose_free=True)
    r1, n = seq.solve(b, x1, Q)
    seq.close()
    torch.cuda.synchronize()
    server = binding.Server(budget_bytes=1 << 30, max_inflight=2, small_n_max=-1)   # workers only
    x2 = torch.zeros_like(x0)
    t = server.submit(dA, b, x2, Q, 4, tol=p.tol, maxit=p.maxit, transpose_free=True)
    r2, _ = server.wait(t)
    server.close()
    assert n == 4 and r0.flag == r1.flag == r2.flag == 0
    assert r0.iter == r1.iter == r2.iter
    assert torch.equal(x0, x1) and torch.equal(x0, x2)
    # with the batchers on, the same small request runs in the batch kernel: bitwise a direct batch solve
    s = binding.Solver(dA, 4, tol=p.tol, maxit=p.maxit, transpose_free=True)
    x3 = torch.zeros_like(x0)
    (r3,) = binding.solve_batch([s], [b], [x3], [Q])
    s.close()
    server = binding.Server(budget_bytes=1 << 30, max_inflight=2)
    x4 = torch.zeros_like(x0)
    t = server.submit(dA, b, x4, Q, 4, tol=p.tol, maxit=p.maxit, transpose_free=True)
    r4, _ = server.wait(t)
    server.close()
    assert r3.flag == r4.flag == 0 and r3.iter == r4.iter
    assert torch.equal(x3, x4)


def test_kernel_timer_and_footprint():
    """MLB_KERNEL_RECOMBINE times the recombination pass of either iteration."""
    p = workloads.config2(n=4, m=32)
    dA = binding.to_device(p.A)
    b = torch.from_numpy(p.b).cuda()
    Q = binding.column_major(p.Q)
    for tf in (False, True):
        x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
        s = binding.Solver(dA, 4, tol=p.tol, maxit=p.maxit, transpose_free=tf)
        assert s.solve(b, x, Q).flag == 0
        for k in (binding.MLB_KERNEL_SPMV_STEP, binding.MLB_KERNEL_ALPHA_STEP, binding.MLB_KERNEL_COMBINE,
                  binding.MLB_KERNEL_RECOMBINE):
            ms = s.time_kernel(k, 3)
            print(f"transpose_free={tf} kernel {k}: {1e3 * ms:.1f} us")
            assert 0 < ms < 10
        s.close()


def test_full_size_convdiff3d_first_iterates():
    """128^3 (N = 2,097,152), n = 4, transpose-free, in the benchmark's launch configuration:
    x_1..x_20 against the oracle's variant, then the converged x's true residual on the CPU."""
    import oracle as orc

    p = workloads.config2(n=4, m=128)
    res, x, its = run_gpu(p, record=20, transpose_free=True)
    o = orc.mlbicgstabt(p.A, p.b, p.Q, tol=p.tol, maxit=20, record_x=20, transpose_free=True)
    for k in range(20):
        assert rel(its[k], o.x_history[k]) < 1e-8, (k + 1, rel(its[k], o.x_history[k]))
    assert res.flag == 0
    true = orc.true_error(p.A, x, p.b)
    print(f"full size transpose-free: iter={res.iter} gpu err_true={res.err_true:.3e} cpu-recomputed={true:.3e} "
          f"recursive={res.err_recursive:.3e}")
    assert true < 10 * p.tol
    assert abs(true - res.err_true) < 1e-12
