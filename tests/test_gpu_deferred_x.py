"""x updates deferred to the omega pass against per-step updates.

A solve that records no iterates leaves x alone in the alpha passes and applies a cycle's alpha steps
in the omega pass (and, when the solve ends within a cycle, in a flush after the last cycle); a solve
that records iterates updates x at every step.  Both make the same fused multiply-adds in the same
order, so flag, iteration count, x and the true residual are bitwise the same: checked here for the
method's variants and for every place a solve can end (at an inner step, at the half step that ends a
cycle, after the omega step, at maxit within a cycle)."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from tests.gpu_util import gpu_available, run_gpu

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1106_3678_amd import binding  # noqa: E402


def same(p, **kw):
    r0, x0, _ = run_gpu(p, record=0, **kw)   # deferred x updates
    r1, x1, _ = run_gpu(p, record=1, **kw)   # per-step x updates (an iterate record)
    print(f"{p.name} {kw}: flag {r0.flag}/{r1.flag} iter {r0.iter}/{r1.iter} err_true {r0.err_true:.3e}", flush=True)
    assert r0.flag == r1.flag and r0.iter == r1.iter
    assert r0.err_true == r1.err_true
    assert np.array_equal(x0, x1)
    return r0


@pytest.mark.parametrize("case", ["n1", "n4", "n8_s_alpha", "complex_n4", "complex_n6", "bsr3_jacobi", "ilu0",
                                  "literal", "transpose_free", "kappa"])
def test_variants(case):
    kw = {}
    if case == "n1":
        p = workloads.config1(n=1)
    elif case == "n4":
        p = workloads.config1(n=4)
    elif case == "n8_s_alpha":
        p = workloads.config2(n=8, m=16, maxit=4000)
    elif case == "complex_n4":
        p = workloads.config5(n=4, m=10, maxit=4000)
    elif case == "complex_n6":
        p = workloads.config5(n=6, m=10, maxit=4000)
    elif case == "bsr3_jacobi":
        p, kw = workloads.config3(n=4, grid=(8, 10, 6), accum=1.0), {"precond": binding.MLB_PRECOND_JACOBI}
    elif case == "ilu0":
        p, kw = workloads.config2(n=4, m=16, maxit=4000), {"precond": binding.MLB_PRECOND_ILU0}
    elif case == "literal":
        p, kw = workloads.config1(n=4), {"order": binding.MLB_ORDER_LITERAL}
    elif case == "transpose_free":
        p, kw = workloads.config1(n=4), {"transpose_free": True}
    else:
        p, kw = workloads.config1(n=4), {"kappa": 0.7}
    r = same(p, **kw)
    assert r.flag == 0


def test_maxit_within_a_cycle():
    """maxit = 10 with n = 4 ends at the second inner step of the third cycle: two steps pending."""
    r = same(workloads.config2(n=4, m=20), maxit=10)
    assert r.flag == 1 and r.iter == 10


def test_exit_at_the_half_step():
    """n = N = 5: the solve ends at iteration 5, the half step of the first cycle (all n steps pending)."""
    N = 5
    g = np.random.default_rng(77)
    A = sp.csr_matrix(g.standard_normal((N, N)) / np.sqrt(N) + 2 * np.eye(N))
    p = workloads.Problem("half", A, g.standard_normal(N), np.asfortranarray(g.standard_normal((N, N))),
                          np.zeros(N), N, 1e-10, 50)
    r = same(p)
    assert r.flag == 0 and r.iter == N


def test_exit_at_an_inner_step():
    """n = 8 > N = 5: the solve ends at iteration 5, an inner step of the first cycle (five steps pending)."""
    N, n = 5, 8
    g = np.random.default_rng(78)
    A = sp.csr_matrix(g.standard_normal((N, N)) / np.sqrt(N) + 2 * np.eye(N))
    p = workloads.Problem("inner", A, g.standard_normal(N), np.asfortranarray(g.standard_normal((N, n))),
                          np.zeros(N), n, 1e-10, 50)
    r = same(p)
    assert r.flag == 0 and r.iter <= N
