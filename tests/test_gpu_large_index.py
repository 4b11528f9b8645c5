"""Systems above 2^30 rows: the 32-bit row and entry indices near their limit.

A = 2 I with N = 1.5 * 2^30 = 1,610,612,736 rows and as many stored entries (CSR), and the
same in 3x3 blocks with 2^29 + 7 block rows (BSR3), built on the device together with b and
q (seeded normal draws), so nothing crosses PCIe.  With one shadow
vector the first step of Algorithm 7.1 gives alpha = q^H r_0 / q^H (A r_0) = 1/2 (up to the
rounding of the stored reciprocal of c), so x_1 = b / 2 and r_1 = 0 to rounding: the solve
stops at iteration 1 with flag 0.  The products A x and A^H x are 2 x exactly (one entry a
row, and doubling is exact).  This runs every pass of the iteration (set-up residual,
index validation, the transpose, SpMV steps, vector passes, the reductions) with rows and
entries past 2^30.  Each case needs 180-215 GB of device memory and is skipped where less is free.
"""
import pytest

from tests.gpu_util import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_1106_3678_amd import binding  # noqa: E402

N = 3 * 2 ** 29
CHUNK = 2 ** 27


def check_two_identity(fmt, nrows, need):
    """A = 2I in CSR (one entry a row) or BSR3 (one 3x3 block 2 I_3 a block row), n = 1."""
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 1e9:.0f} GB of free device memory, {free / 1e9:.0f} GB free")
    assert nrows <= binding.MLB_MAX_INDEX
    nb = nrows // 3 if fmt == binding.MLB_BSR3 else nrows
    print(f"N = {nrows} ({nb} index rows): building A = 2I, b and q on the device", flush=True)
    gen = torch.Generator(device="cuda").manual_seed(20110615)
    rp = torch.arange(nb + 1, dtype=torch.int32, device="cuda")
    ci = torch.arange(nb, dtype=torch.int32, device="cuda")
    if fmt == binding.MLB_BSR3:
        val = torch.zeros(nb, 9, dtype=torch.float64, device="cuda")
        val[:, 0::4] = 2.0        # entries (0,0), (1,1), (2,2) of each row-major block
        val = val.reshape(-1)
    else:
        val = torch.full((nb,), 2.0, dtype=torch.float64, device="cuda")
    dA = binding.DeviceMatrix(rp, ci, val, nrows, fmt, binding.MLB_R64)
    b = torch.randn(nrows, dtype=torch.float64, device="cuda", generator=gen)
    Q = torch.randn(nrows, 1, dtype=torch.float64, device="cuda", generator=gen)
    x = torch.zeros(nrows, dtype=torch.float64, device="cuda")
    s = binding.Solver(dA, 1, tol=1e-10, maxit=10)
    try:
        res = s.solve(b, x, Q)
        torch.cuda.synchronize()
        print(f"solve: flag={res.flag} iter={res.iter} err_true={res.err_true:.3e}", flush=True)
        assert res.flag == 0 and res.iter == 1
        assert res.err_true < 1e-15
        # x = b / 2 to a few ulps (alpha = e * (1/c) with c = 2e); compared in chunks so
        # that no temporary of N values is needed beside the solver's workspace
        dev = max(((2 * x[k:k + CHUNK] - b[k:k + CHUNK]).abs() / b[k:k + CHUNK].abs().clamp_min(1e-300)).max().item()
                  for k in range(0, nrows, CHUNK))
        print(f"max relative |2x - b| / |b| = {dev:.2e}", flush=True)
        assert dev < 4e-16
        del Q
        y = torch.empty_like(x)
        for op in (binding.MLB_OP_A, binding.MLB_OP_AH):
            y.fill_(float("nan"))
            s.matvec(x, y, op)
            torch.cuda.synchronize()
            assert all(torch.equal(y[k:k + CHUNK], 2 * x[k:k + CHUNK]) for k in range(0, nrows, CHUNK)), op
        print("A x and A^H x equal 2x bitwise", flush=True)
    finally:
        s.close()
        del dA, rp, ci, val, b, x
        torch.cuda.empty_cache()


def test_two_times_identity_above_2_30_rows():
    """CSR, N = 1.5 * 2^30; about 180 GB of device memory."""
    check_two_identity(binding.MLB_CSR, N, 200 * 10 ** 9)


def test_two_times_identity_bsr3_above_2_30_rows():
    """BSR3, 2^29 + 7 block rows (N = 1,610,612,757, ragged against every tile); about 215 GB."""
    check_two_identity(binding.MLB_BSR3, 3 * (2 ** 29 + 7), 235 * 10 ** 9)
