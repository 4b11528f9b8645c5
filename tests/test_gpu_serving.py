"""Serving (continuous batching through mlb_server_*): every result in a concurrent mix equals the same
request served alone, a failing request is isolated, and admission respects the HBM budget.  Small CSR
fp64 requests go to the batchers (one-workgroup kernel), the others to the multi-launch workers."""
import time

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from tests.gpu_util import gpu_available, rel

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

from paper_1106_3678_amd import binding  # noqa: E402


def requests(count=14, seed=5):
    """Uneven solves: 2D/3D convection-diffusion of different sizes, n in {2, 4, 8}, fp64 and fp32-IR."""
    g = np.random.default_rng(seed)
    out = []
    for i in range(count):
        dims = 2 + (i % 2)
        m = int(g.integers(12, 70)) if dims == 2 else int(g.integers(8, 22))
        req = workloads.Request(i, 0.0, dims, m, float(g.uniform(0.5, 30)), int(g.choice([2, 4, 8])), 500 + i)
        p = workloads.serving_problem(req, maxit=5000)
        out.append((p, binding.MLB_PREC_FP32_IR if i % 3 == 0 else binding.MLB_PREC_FP64))
    return out


def upload(p):
    dA = binding.to_device(p.A)
    b = torch.from_numpy(p.b).cuda()
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    Q = binding.column_major(p.Q)
    return dA, b, x, Q


def solve_alone(p, prec, small_n_max=0):
    """The request alone in a server of its own (the same routing as in the mix)."""
    dA, b, x, Q = upload(p)
    torch.cuda.synchronize()
    server = binding.Server(budget_bytes=8 << 30, max_inflight=1, small_n_max=small_n_max)
    res, _ = server.wait(server.submit(dA, b, x, Q, p.n, tol=p.tol, maxit=p.maxit, precision=prec))
    server.close()
    return res, x.cpu().numpy()


def solve_multi_launch(p, prec):
    dA, b, x, Q = upload(p)
    s = binding.Solver(dA, p.n, tol=p.tol, maxit=p.maxit, precision=prec)
    res = s.solve(b, x, Q)
    s.close()
    return res, x.cpu().numpy()


def test_mix_equals_alone():
    reqs = requests()
    alone = [solve_alone(p, prec) for p, prec in reqs]
    server = binding.Server(budget_bytes=8 << 30, max_inflight=4)
    bufs = [upload(p) for p, _ in reqs]
    torch.cuda.synchronize()
    tickets = [server.submit(dA, b, x, Q, p.n, tol=p.tol, maxit=p.maxit, precision=prec)
               for (p, prec), (dA, b, x, Q) in zip(reqs, bufs)]
    results = [server.wait(t) for t in tickets]
    st = server.stats()
    server.close()
    print(f"peak concurrency {st.peak_running}, peak footprint {st.peak_used_bytes / 1e6:.1f} MB, "
          f"completed {st.completed}", flush=True)
    assert st.completed == len(reqs)
    for k, ((p, prec), (res_a, x_a), (res_m, tim), (_, _, x_m, _)) in enumerate(zip(reqs, alone, results, bufs)):
        xm = x_m.cpu().numpy()
        print(f"{p.name} prec={prec}: alone flag={res_a.flag} iter={res_a.iter} | mix flag={res_m.flag} "
              f"iter={res_m.iter} true={res_m.err_true:.2e} latency={tim.latency_ms:.1f} ms", flush=True)
        assert res_m.flag == res_a.flag == 0
        assert res_m.iter == res_a.iter
        assert np.array_equal(xm, x_a), k
        assert oracle.true_error(p.A, xm, p.b) < p.tol


def test_workers_only_equal_multi_launch_solves():
    """With the batchers off every request runs the multi-launch iteration: bitwise its plain solve."""
    reqs = requests(count=6, seed=3)
    server = binding.Server(budget_bytes=8 << 30, max_inflight=3, small_n_max=-1)
    bufs = [upload(p) for p, _ in reqs]
    torch.cuda.synchronize()
    tickets = [server.submit(dA, b, x, Q, p.n, tol=p.tol, maxit=p.maxit, precision=prec)
               for (p, prec), (dA, b, x, Q) in zip(reqs, bufs)]
    results = [server.wait(t) for t in tickets]
    server.close()
    for (p, prec), (res, _), (_, _, x, _) in zip(reqs, results, bufs):
        res_a, x_a = solve_multi_launch(p, prec)
        assert res.flag == res_a.flag == 0 and res.iter == res_a.iter
        assert np.array_equal(x.cpu().numpy(), x_a)


def test_batched_requests_match_multi_launch():
    """A small request served by a batcher agrees with the multi-launch solve to rounding."""
    for p, prec in requests(count=4, seed=17):
        if prec != binding.MLB_PREC_FP64:
            continue
        res, x = solve_alone(p, prec)
        res_m, x_m = solve_multi_launch(p, prec)
        assert res.flag == res_m.flag == 0
        assert abs(res.iter - res_m.iter) <= max(1, int(0.05 * res_m.iter))
        assert rel(x, x_m) < 1e-6


def test_failing_request_is_isolated():
    """A breakdown (c_0 = 0) in the mix completes with flag -1 and does not disturb the others."""
    reqs = requests(count=4, seed=9)
    A = sp.csr_matrix(np.eye(3))
    bad = workloads.Problem("c0", A, np.array([1.0, 0, 0]), np.array([[0.0], [1.0], [0.0]]), np.zeros(3), 1,
                            1e-10, 10)
    server = binding.Server(budget_bytes=4 << 30, max_inflight=3)
    items = [(bad, binding.MLB_PREC_FP64)] + reqs
    bufs = [upload(p) for p, _ in items]
    torch.cuda.synchronize()
    tickets = [server.submit(dA, b, x, Q, p.n, tol=p.tol, maxit=p.maxit, precision=prec)
               for (p, prec), (dA, b, x, Q) in zip(items, bufs)]
    results = [server.wait(t) for t in tickets]
    server.close()
    assert results[0][0].flag == -1 and results[0][0].iter == 0
    for (p, prec), (res, _), (_, _, x, _) in zip(items[1:], results[1:], bufs[1:]):
        res_a, x_a = solve_alone(p, prec)
        assert res.flag == 0 and np.array_equal(x.cpu().numpy(), x_a)


def test_smallest_first_order():
    """MLB_SERVE_SMALLEST: with one worker, four large requests and then a small one queued while the first
    large one runs, the small one waits for at most one large run; under MLB_SERVE_FIFO it waits for the
    three large ones queued before it, and with a max_wait_ms below the queueing delay every request has
    aged, so the order is FIFO again.  Every result is bitwise the same in the three orders."""
    big = [workloads.serving_problem(workloads.Request(i, 0.0, 3, 48, 5.0 + i, 4, 900 + i), maxit=5000)
           for i in range(4)]
    small = workloads.serving_problem(workloads.Request(9, 0.0, 2, 20, 3.0, 4, 990), maxit=5000)
    probs = big + [small]
    out = {}
    for tag, order, wait_ms in (("fifo", binding.MLB_SERVE_FIFO, 0.0), ("smallest", binding.MLB_SERVE_SMALLEST, 0.0),
                                ("aged", binding.MLB_SERVE_SMALLEST, 1e-3)):
        bufs = [upload(p) for p in probs]
        torch.cuda.synchronize()
        server = binding.Server(budget_bytes=8 << 30, max_inflight=1, small_n_max=-1, order=order,
                                max_wait_ms=wait_ms)
        t0 = time.perf_counter()
        tickets = [server.submit(dA, b, x, Q, p.n, tol=p.tol, maxit=p.maxit) for p, (dA, b, x, Q) in zip(probs, bufs)]
        submit_ms = (time.perf_counter() - t0) * 1e3
        res = [server.wait(t) for t in tickets]
        server.close()
        tims = [r[1] for r in res]
        print(f"{tag}: submitted in {submit_ms:.2f} ms; queued " +
              ", ".join(f"{t.queued_ms:.1f}" for t in tims) + " ms; run " + ", ".join(f"{t.run_ms:.1f}" for t in tims),
              flush=True)
        assert all(r[0].flag == 0 for r in res)
        assert submit_ms < min(t.run_ms for t in tims[:4])   # all five queued while the first large one ran
        out[tag] = ([b[2].cpu().numpy() for b in bufs], tims)
    f, sm, ag = out["fifo"][1], out["smallest"][1], out["aged"][1]
    assert f[4].queued_ms >= f[1].run_ms + f[2].run_ms + f[3].run_ms
    assert sm[4].queued_ms <= max(t.run_ms for t in sm[:4]) + 5.0
    assert ag[4].queued_ms >= ag[2].run_ms + ag[3].run_ms
    for k in range(5):
        assert np.array_equal(out["fifo"][0][k], out["smallest"][0][k])
        assert np.array_equal(out["fifo"][0][k], out["aged"][0][k])


def test_admission_respects_budget():
    """With a budget that fits about two requests, the footprint in flight never exceeds it."""
    reqs = requests(count=8, seed=13)
    bufs = [upload(p) for p, _ in reqs]
    fps = []
    for (p, prec), (dA, _, _, _) in zip(reqs, bufs):
        opt = binding.mlb_options(p.n, p.tol, p.maxit, 0.0, prec, 0.0, 0, 0, None, 0)
        fps.append(binding.mlbicgstab_workspace_size(dA.descriptor(), opt))
    budget = int(sorted(fps)[-1] + sorted(fps)[-2])
    server = binding.Server(budget_bytes=budget, max_inflight=6)
    torch.cuda.synchronize()
    tickets = [server.submit(dA, b, x, Q, p.n, tol=p.tol, maxit=p.maxit, precision=prec)
               for (p, prec), (dA, b, x, Q) in zip(reqs, bufs)]
    results = [server.wait(t) for t in tickets]
    st = server.stats()
    server.close()
    assert all(r.flag == 0 for r, _ in results)
    assert st.peak_used_bytes <= budget
    # an oversize request is refused at submission
    server = binding.Server(budget_bytes=1024, max_inflight=1)
    p, prec = reqs[-1]
    dA, b, x, Q = bufs[-1]
    with pytest.raises(binding.MlbError) as e:
        server.submit(dA, b, x, Q, p.n, tol=p.tol, maxit=p.maxit, precision=prec)
    assert e.value.code == binding.MLB_ENOMEM
    server.close()


def test_one_request_matches_oracle():
    p, prec = requests(count=2, seed=21)[1]
    server = binding.Server(budget_bytes=1 << 30, max_inflight=2)
    dA, b, x, Q = upload(p)
    torch.cuda.synchronize()
    res, _ = server.wait(server.submit(dA, b, x, Q, p.n, tol=p.tol, maxit=p.maxit, precision=binding.MLB_PREC_FP64))
    server.close()
    o = oracle.mlbicgstabt(p.A, p.b, p.Q, tol=p.tol, maxit=p.maxit)
    assert res.flag == o.flag == 0
    assert abs(res.iter - o.iter) <= max(1, int(0.05 * o.iter))
    assert rel(x.cpu().numpy(), o.x) < 1e-6


def test_sequence_in_server_follows_the_rule_and_matches_fresh_solves():
    """Section 5.2 inside the server: the requests of a sequence share one solver (A^H built once) and
    run in submission order while other requests flow; n follows mlb_sequence_next_n replayed from
    the reported solve times, and each result is bitwise a fresh create + solve with that n."""
    n0, n_min, n_max, step = 4, 2, 8, 2
    p = workloads.config2(n=n_max, m=20, maxit=4000)
    g = np.random.default_rng(77)
    rhs = [g.standard_normal(p.N) for _ in range(7)]
    dA = binding.to_device(p.A)
    Q = binding.column_major(p.Q)
    bs = [torch.from_numpy(v).cuda() for v in rhs]
    xs = [torch.zeros(p.N, dtype=torch.float64, device="cuda") for _ in rhs]
    others = requests(count=6, seed=9)
    obufs = [upload(q) for q, _ in others]
    torch.cuda.synchronize()
    server = binding.Server(budget_bytes=8 << 30, max_inflight=3)
    key = 0x5EC
    tickets, otickets = [], []
    for k, (b, x) in enumerate(zip(bs, xs)):
        tickets.append(server.submit_sequence(key, dA, b, x, Q, n0, n_min, n_max, step, tol=p.tol, maxit=p.maxit))
        if k < len(others):
            (q, prec), (qA, qb, qx, qQ) = others[k], obufs[k]
            otickets.append(server.submit(qA, qb, qx, qQ, q.n, tol=q.tol, maxit=q.maxit, precision=prec))
    results = [server.wait(t) for t in tickets]
    for t in otickets:
        res, _ = server.wait(t)
        assert res.flag == 0
    server.end_sequence(key)
    st = server.stats()
    server.close()
    assert st.used_bytes == 0
    used = [tim.n_used for _, tim in results]
    times = [res.solve_ms for res, _ in results]
    print("n used:", used, "solve ms:", [round(t, 2) for t in times], "iterations:", [r.iter for r, _ in results],
          flush=True)
    n, t_prev = n0, -1.0
    for k in range(len(rhs)):
        assert used[k] == n, (k, used, n)
        n_next = binding.mlb_sequence_next_n(n, t_prev, times[k], step, n_min, n_max)
        t_prev, n = times[k], n_next
    for (res, tim), b, x in zip(results, bs, xs):
        assert res.flag == 0
        xf = torch.zeros(p.N, dtype=torch.float64, device="cuda")
        s = binding.Solver(dA, tim.n_used, tol=p.tol, maxit=p.maxit)
        rf = s.solve(b, xf, Q[:, :tim.n_used])
        s.close()
        assert rf.iter == res.iter and rf.flag == res.flag
        assert torch.equal(xf, x)


def _batched(p, tol):
    dA, b, x, Q = upload(p)
    s = binding.Solver(dA, p.n, tol=tol, maxit=p.maxit)
    try:
        return binding.solve_batch([s], [b], [x], [Q])[0]
    finally:
        s.close()


def _served(p, tol, max_restarts):
    dA, b, x, Q = upload(p)
    torch.cuda.synchronize()
    server = binding.Server(budget_bytes=8 << 30, max_inflight=1)
    try:
        res, _ = server.wait(server.submit(dA, b, x, Q, p.n, tol=tol, maxit=p.maxit, max_restarts=max_restarts))
    finally:
        server.close()
    r = b.cpu().numpy() - p.A @ x.cpu().numpy()
    return res, np.linalg.norm(r) / np.linalg.norm(p.b)


def test_batched_request_restarts_on_residual_gap():
    """A small request on the batched solve that stops on its recursive residual with the true residual
    not below tol.  Such a case is made by setting tol between the two residuals of a run at 1e-10:
    the run then stops at the same iteration (the one before it was still above).  Served with
    max_restarts = 0 the request comes back with the gap.  With max_restarts = 2 the server restarts
    it from its x on the multi-launch iteration.  The result then reports the restart and the added
    iterations, and its true residual (also recomputed here on the CPU) is below tol."""
    checked = 0
    for m, n in ((32, 2), (48, 8), (64, 2), (64, 4)):
        p = workloads.config1(n=n, m=m)
        ref = _batched(p, 1e-10)
        if not ref.err_true > ref.err_recursive:
            continue
        tol = float(np.sqrt(ref.err_true * ref.err_recursive))
        r0, e0 = _served(p, tol, 0)
        if not (r0.flag == 0 and r0.err_true >= tol):
            continue
        r2, e2 = _served(p, tol, 2)
        print(f"m={m} n={n} tol={tol:.4e}: without restarts iter={r0.iter} err_true={r0.err_true:.4e}; "
              f"with: iter={r2.iter} restarts={r2.outer_iters} err_true={r2.err_true:.4e} (CPU {e2:.4e})")
        assert r2.flag == 0 and r2.outer_iters >= 1 and r2.iter > r0.iter
        assert r2.err_true < tol and e2 < 1.01 * tol
        checked += 1
    assert checked >= 1, "no candidate system showed a residual gap"


def test_sequence_argument_errors():
    p = workloads.config1(n=4)
    dA, b, x, Q = upload(p)
    dB = binding.to_device(p.A)
    server = binding.Server(budget_bytes=1 << 30, max_inflight=1)
    try:
        with pytest.raises(binding.MlbError):
            server.submit_sequence(0, dA, b, x, Q, 4, 2, 4, 1)          # key 0
        t = server.submit_sequence(7, dA, b, x, Q, 4, 2, 4, 1)
        with pytest.raises(binding.MlbError):
            server.submit_sequence(7, dB, b, x, Q, 4, 2, 4, 1)          # another A
        with pytest.raises(binding.MlbError):
            server.submit_sequence(7, dA, b, x, Q, 4, 2, 4, 2)          # another rule
        res, tim = server.wait(t)
        assert res.flag == 0 and tim.n_used == 4
        server.end_sequence(7)
        with pytest.raises(binding.MlbError):
            server.end_sequence(7)                                     # already ended
        assert server.stats().used_bytes == 0
    finally:
        server.close()
