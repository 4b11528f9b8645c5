"""Sequences of systems with the same A and n chosen from one system to the next (Section 5.2).

Checks: n follows the rule of mlb_sequence_next_n applied to the reported solve times; every
system's result is bitwise that of a fresh solver created with the same n (one workspace and one
A^H serve all n); and every system meets the parity bars against the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import gpu_available, rel

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_1106_3678_amd import binding  # noqa: E402


def systems(count=7, n_max=8):
    """One 3D convection-diffusion matrix, a new right-hand side per system, a fixed N x n_max Q."""
    p = workloads.config2(n=n_max, m=20, maxit=4000)
    g = np.random.default_rng(2024)
    return p, [g.standard_normal(p.N) for _ in range(count)]


def test_sequence_follows_the_rule_and_matches_fresh_solvers():
    n0, n_min, n_max, step = 4, 2, 8, 2
    p, rhs = systems(n_max=n_max)
    dA = binding.to_device(p.A)
    Q = binding.column_major(p.Q)
    seq = binding.Sequence(dA, n0, n_min, n_max, step, tol=p.tol, maxit=p.maxit)
    used, times, xs, its = [], [], [], []
    for bv in rhs:
        b = torch.from_numpy(bv).cuda()
        x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
        res, n = seq.solve(b, x, Q)
        assert res.flag == 0
        used.append(n)
        times.append(res.solve_ms)
        xs.append(x.cpu().numpy())
        its.append(res.iter)
    seq.close()
    print("n used:", used, "solve ms:", [round(t, 2) for t in times], "iterations:", its, flush=True)
    # the rule, replayed from the reported times
    n = n0
    for k in range(len(rhs)):
        assert used[k] == n, (k, used, times)
        n = binding.mlb_sequence_next_n(n, times[k - 1] if k else -1.0, times[k], step, n_min, n_max)
    # each system: bitwise a fresh solver with that n, and the oracle's solution
    for bv, n, x_seq, it in zip(rhs, used, xs, its):
        b = torch.from_numpy(bv).cuda()
        x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
        s = binding.Solver(dA, n, tol=p.tol, maxit=p.maxit)
        r = s.solve(b, x, Q[:, :n])
        s.close()
        assert r.iter == it
        assert np.array_equal(x.cpu().numpy(), x_seq)
        o = oracle.mlbicgstabt(p.A, bv, p.Q[:, :n], tol=p.tol, maxit=p.maxit)
        assert o.flag == 0 and abs(o.iter - it) <= max(1, int(0.05 * o.iter))
        assert rel(x_seq, o.x) < 1e-6


def test_sequence_with_fixed_n():
    """step = 0 keeps n; the sequence's solves equal plain solves."""
    p, rhs = systems(count=3, n_max=4)
    dA = binding.to_device(p.A)
    Q = binding.column_major(p.Q)
    seq = binding.Sequence(dA, 4, 1, 4, 0, tol=p.tol, maxit=p.maxit)
    for bv in rhs:
        b = torch.from_numpy(bv).cuda()
        x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
        res, n = seq.solve(b, x, Q)
        assert n == 4 and res.flag == 0
        x2 = torch.zeros(p.N, dtype=torch.float64, device="cuda")
        s = binding.Solver(dA, 4, tol=p.tol, maxit=p.maxit)
        s.solve(b, x2, Q)
        s.close()
        assert np.array_equal(x.cpu().numpy(), x2.cpu().numpy())
    seq.close()
