"""Kernel-timing replays leave later solves unchanged; the workspace-size model matches what a solver
allocates."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_1106_3678_amd import binding  # noqa: E402


def test_time_kernel_leaves_later_solves_unchanged():
    p = workloads.config2(n=4, m=24, maxit=4000)
    dA = binding.to_device(p.A)
    b = torch.from_numpy(p.b).cuda()
    Q = binding.column_major(p.Q)
    s = binding.Solver(dA, p.n, tol=p.tol, maxit=p.maxit)
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    r1 = s.solve(b, x, Q)
    x1 = x.cpu().numpy()
    for kind in (binding.MLB_KERNEL_SPMV_STEP, binding.MLB_KERNEL_ALPHA_STEP, binding.MLB_KERNEL_COMBINE):
        ms = s.time_kernel(kind, 2)
        assert 0.0 < ms < 100.0
    x.zero_()
    r2 = s.solve(b, x, Q)
    s.close()
    assert r1.flag == r2.flag == 0 and r1.iter == r2.iter
    assert np.array_equal(x.cpu().numpy(), x1)


@pytest.mark.parametrize("precision,precond", [(0, 0), (1, 0), (0, 1)])
def test_workspace_size_matches_allocation(precision, precond):
    p = workloads.config2(n=8, m=64, maxit=100)
    dA = binding.to_device(p.A)
    opt = binding.mlb_options(p.n, p.tol, p.maxit, 0.0, precision, 0.0, 0, 0, None, precond)
    predicted = binding.mlbicgstab_workspace_size(dA.descriptor(), opt)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    s = binding.Solver(dA, p.n, tol=p.tol, maxit=p.maxit, precision=precision, precond=precond)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    s.close()
    used = free0 - free1
    print(f"precision={precision} precond={precond}: predicted {predicted / 1e6:.1f} MB, allocated {used / 1e6:.1f} MB",
          flush=True)
    assert 0.9 * predicted <= used <= 1.1 * predicted + (64 << 20)
