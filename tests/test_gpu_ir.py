"""fp32-inner / fp64 iterative refinement (MLB_PREC_FP32_IR) against the fp64 oracle.

The refinement loop stops on the TRUE residual ||b - A x|| / ||b|| < tol computed in fp64, so the bar is
that true residual (recomputed here on the CPU) plus the distance of x from the oracle's fp64 solution,
which is printed for every case.  The paper does not discuss precision; this mode is an addition.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import gpu_available, rel, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def check_ir(p, x_tol=1e-6, inner_tol=0.0, precond=0):
    res, x, _ = run_gpu(p, precision=1, inner_tol=inner_tol, precond=precond)
    o = run_oracle(p, precond=precond)
    true_cpu = oracle.true_error(p.A, x, p.b)
    print(f"{p.name}: IR flag={res.flag} inner iters={res.iter} outer={res.outer_iters} fp64 iters={res.fp64_iters} "
          f"true={res.err_true:.3e} (cpu {true_cpu:.3e}) | oracle iter={o.iter} true="
          f"{oracle.true_error(p.A, o.x, p.b):.3e} | rel(x, x_oracle)={rel(x, o.x):.2e}", flush=True)
    assert res.flag == 0
    assert true_cpu < p.tol
    assert abs(true_cpu - res.err_true) < 1e-12
    assert rel(x, o.x) < x_tol
    return res


@pytest.mark.parametrize("n", [1, 4, 8])
def test_ir_convdiff3d(n):
    res = check_ir(workloads.config2(n=n, m=24, maxit=4000))
    assert res.outer_iters >= 2 and res.fp64_iters == 0


def test_ir_convdiff2d():
    check_ir(workloads.config1(n=4))


@pytest.mark.parametrize("grid,n,precond", [((8, 10, 6), 8, 0), ((12, 16, 6), 8, 0), ((8, 10, 6), 8, 1),
                                            ((12, 16, 6), 8, 1)])
def test_ir_reservoir(grid, n, precond):
    """Reservoir-shaped BSR3 systems (cond ~ 1e6): without a preconditioner the fp32 inner solve stagnates
    and the stagnation guard hands the rest to the fp64 iteration; with block Jacobi the refinement
    converges in fp32.  Either way the true residual must reach tol."""
    res = check_ir(workloads.config3(n=n, grid=grid, maxit=20000), x_tol=1e-4, precond=precond)
    assert res.iter < 20000


def test_ir_complex():
    check_ir(workloads.config5(n=8, m=12, maxit=4000))


def test_ir_zero_rhs():
    p = workloads.config1(n=4)
    p.b = np.zeros(p.N)
    res, x, _ = run_gpu(p, precision=1)
    assert res.flag == 0 and res.outer_iters == 0 and not x.any()
