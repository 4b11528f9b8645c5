"""Time-to-1e-10 of ML(n)BiCGStab on one MI355X.

One step = one complete solve (setup with A^H q_s, the whole iteration, the
final fp64 true-residual check) with A, b and Q resident in HBM before timing,
x_0 = 0, tol 1e-10.  Default workload: the 3D convection-diffusion system on a
128^3 grid (N = 2,097,152, 14,581,760 nonzeros, CSR fp64), n = 4.  Other
workloads (--workload reservoir: 60x220x85 3x3-block system, BSR3, n = 8;
--workload helmholtz: complex 96^3 system, n = 16) and the fp32-inner /
fp64-refinement mode (--precision ir) use the same step definition.

The default line also carries, under "secondary", one record per other
configuration (the reservoir system in fp64 and fp32-IR, the complex system
with n = 16, the 128^3 system with ILU(0) at n = 1 and n = 4, and the
2000-request serving trace in fp64 and fp32-IR beside the same requests
solved one after another in fp64); --no-extras leaves them out.
Prints one JSON line.  Progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def s_from_alpha(n, transpose_free=False, literal=False, sv=8):
    """Whether the library takes the S column of w_i below its diagonal (q_s^H w_i, s > i) from the next
    alpha pass, so that the SpMV step reduces only c_i = q_i^H w_i: the Gram-form steps with A^H whose
    bucket of n (4, 8, 16, 32) is 8 or 16 with 2 nb + 1 accumulators of sv bytes within 288 bytes (real
    n in 5..16, complex n in 5..8)."""
    nb = 4 if n <= 4 else 8 if n <= 8 else 16 if n <= 16 else 32
    return not transpose_free and not literal and 8 <= nb <= 16 and (2 * nb + 1) * sv <= 288


def spmv_step_bytes(nnz, nbrows, N, n, sv, bsr=False, literal=False, transpose_free=False):
    """Algorithmic bytes of one SpMV-step launch (w_i = A g_i with its shadow dots), averaged over the
    launches i = 0..n-1 of one cycle.

    Matrix: values + column indices + row pointers, each read once; vectors: the gathered input once,
    the columns of Q the epilogue reduces against, and the written w_i.  (The input is already in its
    column of G: the cycle close writes g into G_0 itself.)  With the S column from the alpha pass
    (n <= 16, A^H) and in the literal recurrence order the step reduces only c_i: one column of Q.
    Otherwise it reads n - i columns (s = i..n-1); the transpose-free steps read columns 0..i-1
    instead (v = A g with q_s^H v, s < i): the same count over a cycle, so the same average.
    """
    mat = nnz * ((9 if bsr else 1) * sv + 4) + 4 * (nbrows + 1)
    one = literal or s_from_alpha(n, transpose_free, sv=sv)
    vec_avg = 3.0 if one else sum(1 + (n - i) + 1 for i in range(n)) / n
    return mat + vec_avg * N * sv


def matrix_bytes(nnz, nbrows, sv, bsr=False):
    """Compulsory bytes of one pass over A: values, column indices, row pointers."""
    return nnz * ((9 if bsr else 1) * sv + 4) + 4 * (nbrows + 1)


def vector_passes_per_iter(n, transpose_free=False, sv=8):
    """Vectors of N values the kernels of one iteration read or write, averaged over a cycle of n steps
    (the SpMV's gathered input and output included; each vector counted once per pass).

    The solves bench.py times record no iterates, so the x updates of a cycle are deferred to the omega
    pass.  Per inner step i = 1..n-1: alpha pass 3 + n - i (r, w, n - i columns of Q, r written),
    combination 2 + 2(n - i) + i, recombination 2 + i, SpMV step 2 + (n - i); per cycle end: half step
    3, SpMV of the minimisation step 2, omega pass 5 + 2n (x, u, z, n columns of Q and n of G; x and r
    written), cycle close 2 + 2n, SpMV step 2 + n.  With the S column from the alpha pass
    (s_from_alpha) every SpMV step reads one column of Q: 3.  Transpose-free steps replace the
    recombination and the product of g_k by the product of g (2 + i, its shadow dots) and the
    recombination of g and w (4 + 2i + n - i), and read no F (combination 2 + 2(n - i))."""
    one = s_from_alpha(n, transpose_free, sv=sv)
    total = 0
    for i in range(1, n):
        if transpose_free:
            total += (3 + n - i) + (2 + 2 * (n - i)) + (2 + i) + (4 + 2 * i + n - i)
        else:
            total += (3 + n - i) + (2 + 2 * (n - i) + i) + (2 + i) + (3 if one else 2 + n - i)
    total += 3 + 2 + (5 + 2 * n) + (2 + 2 * n) + (3 if one else 2 + n)
    return total / n


def bytes_per_iter(nnz, nbrows, N, n, sv, bsr=False, transpose_free=False):
    """Algorithmic bytes of one iteration of the kernels as built: (1 + 1/n) passes over A plus the
    vector passes above."""
    return (1 + 1 / n) * matrix_bytes(nnz, nbrows, sv, bsr) + vector_passes_per_iter(n, transpose_free, sv) * N * sv


def copy_rate_gbs(torch, dev, gib=1.0, reps=5):
    """Practical HBM ceiling: a plain elementwise copy kernel over `gib` GiB (read and written once
    per launch; the kernel the counter calibration uses), the best of `reps` launches timed with
    events on the current stream, in GB/s (1e9 B/s)."""
    nel = int(gib * (1 << 30) / 8)
    src = torch.ones(nel, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.mul(src, 1.0, out=dst)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nel * 8 / (best * 1e-3) / 1e9


def measured_traffic(workload, root=ROOT):
    """HBM bytes per SpMV-step launch from the committed rocprofv3 counter summary, or None when
    the kernel source has changed since the counters were taken (or no summary exists)."""
    import hashlib
    import re

    path = os.path.join(root, "profiles", f"spmv_step_{workload}.md")
    src = os.path.join(root, "paper_1106_3678_amd", "csrc", "mlb_spmv.hpp")   # the SpMV kernels
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_t = re.search(r"^traffic_bytes_per_launch: (\d+)", text, re.M)
    m_h = re.search(r"^kernel_source_sha256: ([0-9a-f]+)", text, re.M)
    if not m_t or not m_h:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_h.group(1):
        return None
    return int(m_t.group(1))


def host_info():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "affinity": aff}


def host_threads():
    """Threads for the all-core oracle run: OMP_NUM_THREADS when set (the machine's CPU share), else the
    CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    return int(env) if env.isdigit() and int(env) > 0 else host_info()["affinity"]


def host_add_gbs(threads, mib=512, reps=3):
    """Host memory bandwidth, STREAM-add style: a = b + c over `threads` contiguous slices in parallel
    (numpy releases the GIL), 3 arrays of `mib` MiB moved per pass; the best of `reps` passes, GB/s."""
    from concurrent.futures import ThreadPoolExecutor

    n = mib * (1 << 20) // 8
    a, b, c = np.empty(n), np.ones(n), np.ones(n)
    bounds = np.linspace(0, n, threads + 1).astype(int)
    sl = [slice(bounds[i], bounds[i + 1]) for i in range(threads)]
    best = float("inf")
    with ThreadPoolExecutor(threads) as ex:
        for _ in range(reps + 1):
            t0 = time.perf_counter()
            list(ex.map(lambda q: np.add(b[q], c[q], out=a[q]), sl))
            best = min(best, time.perf_counter() - t0)
    return 3 * n * 8 / best / 1e9


def cpu_baseline(p, iters_gpu, sample_iters, bytes_per_iter, target_s=10.0, add_mib=512):
    """The oracle on this host: a bounded sample of the same solve, on one core and on all the cores
    this process has (BLAS threads; scipy's sparse products stay on one thread).

    A 5-iteration probe sizes the sample to about target_s of single-core time: the whole solve (the
    oracle then runs to its own convergence, and the sample counts as whole only if it converged)
    when that fits in twice target_s, else that many iterations, scaled to the GPU's iteration count.
    `value` is the all-core time; the single-core run is reported beside it, with the host's CPU model
    and an add-kernel bandwidth figure for the bandwidth fraction of the all-core run."""
    from threadpoolctl import threadpool_limits

    import oracle

    def run(maxit, threads):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            o = oracle.mlbicgstabt(p.A, p.b, p.Q, x0=p.x0, tol=p.tol, maxit=maxit, kappa=p.kappa)
            return o, time.perf_counter() - t0

    threads = host_threads()
    o, dt = run(5, 1)
    per_it = dt / max(o.iter, 1)
    whole_fits = per_it * iters_gpu <= 2 * target_s and sample_iters <= 0
    maxit = p.maxit if whole_fits else max(5, min(iters_gpu, int(target_s / per_it),
                                                  sample_iters if sample_iters > 0 else iters_gpu))
    out = {}
    for label, th in (("single", 1), ("all", threads)):
        o, dt = run(maxit, th)
        whole = o.flag == 0
        out[label] = {"seconds": dt if whole else dt / max(o.iter, 1) * iters_gpu, "oracle_flag": int(o.flag),
                      "oracle_iter": int(o.iter), "measured_s": dt, "whole": whole, "threads": th}
    host = host_info()
    add_gbs = host_add_gbs(threads, mib=add_mib)
    a = out["all"]
    bw = bytes_per_iter * a["oracle_iter"] / a["measured_s"] / 1e9
    sample = (f"the whole solve on {threads} threads: the oracle converged (flag 0) at {a['oracle_iter']} "
              f"iterations, setup included" if a["whole"] else
              f"first {a['oracle_iter']} iterations of the same solve on {threads} threads (oracle flag "
              f"{a['oracle_flag']}: not converged) took {a['measured_s']:.2f} s, scaled to the GPU's {iters_gpu} "
              f"iterations")
    return {"value": a["seconds"], "unit": "s", "cores": threads, "kind": "oracle", "sample": sample,
            "oracle_flag": a["oracle_flag"], "oracle_iter": a["oracle_iter"], "whole": a["whole"],
            "single_core": {"value": out["single"]["seconds"], "oracle_flag": out["single"]["oracle_flag"],
                            "oracle_iter": out["single"]["oracle_iter"], "whole": out["single"]["whole"]},
            "host": {**host, "add_bandwidth_gbs": add_gbs, "threads_used": threads},
            "algorithmic_gbs": bw, "bandwidth_frac": bw / add_gbs}


def serving_items(args, torch, workloads, binding):
    """The serving trace's requests, generated and uploaded: (request, problem, A, b, x, Q) each."""
    reqs = workloads.serving_trace(count=args.requests)
    t = time.perf_counter()
    items = []
    for k, r in enumerate(reqs):
        p = workloads.serving_problem(r)
        dA = binding.to_device(p.A)
        b = torch.from_numpy(p.b).cuda()
        x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
        Q = binding.column_major(p.Q)
        items.append((r, p, dA, b, x, Q))
        if (k + 1) % 100 == 0:
            log(f"[bench] generated and uploaded {k + 1}/{len(reqs)} requests ({time.perf_counter() - t:.0f} s)")
    torch.cuda.synchronize()
    return reqs, items


def serve_order(args, binding):
    """The server's pick order for the workers' queue (--serve-order)."""
    return binding.MLB_SERVE_SMALLEST if getattr(args, "serve_order", "fifo") == "smallest" else binding.MLB_SERVE_FIFO


def bench_serving(args, torch, workloads, binding, generated=None, sequential=True):
    """Continuous batching of a Poisson stream of uneven solves (tol 1e-10; --serve-precision picks fp32
    inner / fp64 refinement, as the serving configuration names, or fp64)."""
    reqs, items = generated if generated is not None else serving_items(args, torch, workloads, binding)
    prec = binding.MLB_PREC_FP32_IR if args.serve_precision == "ir" else binding.MLB_PREC_FP64
    mr = args.max_restarts if prec == binding.MLB_PREC_FP64 else 0   # fp32-IR tests the true residual itself
    # warm-up: one request alone (first-use costs of the kernels)
    r0, p0, dA0, b0, x0, Q0 = items[0]
    s = binding.Solver(dA0, p0.n, tol=p0.tol, maxit=p0.maxit, precision=prec)
    s.solve(b0, x0, Q0)
    s.close()
    for it in items:
        it[4].zero_()
    torch.cuda.synchronize()

    server = binding.Server(budget_bytes=int(args.budget_gb * (1 << 30)), max_inflight=args.inflight,
                            small_n_max=args.small_n_max, order=serve_order(args, binding))
    t0 = time.perf_counter()
    tickets = []
    for r, p, dA, b, x, Q in items:
        delay = t0 + r.arrival_s - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets.append(server.submit(dA, b, x, Q, p.n, tol=p.tol, maxit=p.maxit, precision=prec,
                                     transpose_free=args.transpose_free, max_restarts=mr))
    lat, flags, errs, iters = [], [], [], []
    for tk in tickets:
        res, tim = server.wait(tk)
        lat.append(tim.latency_ms)
        flags.append(res.flag)
        errs.append(res.err_true)
        iters.append(res.iter)
    makespan = time.perf_counter() - t0
    st = server.stats()
    server.close()
    log(f"[bench] serving: {len(items)} requests in {makespan:.2f} s, peak concurrency {st.peak_running}, "
        f"peak footprint {st.peak_used_bytes / 1e9:.2f} GB, max true residual {max(errs):.2e}")

    # capacity: the same requests all submitted at once (no arrival gaps)
    for it in items:
        it[4].zero_()
    torch.cuda.synchronize()
    server = binding.Server(budget_bytes=int(args.budget_gb * (1 << 30)), max_inflight=args.inflight,
                            small_n_max=args.small_n_max, order=serve_order(args, binding))
    t2 = time.perf_counter()
    tickets = [server.submit(dA, b, x, Q, p.n, tol=p.tol, maxit=p.maxit, precision=prec,
                             transpose_free=args.transpose_free, max_restarts=mr)
               for r, p, dA, b, x, Q in items]
    sat_flags = [server.wait(tk)[0].flag for tk in tickets]
    saturated = time.perf_counter() - t2
    server.close()
    log(f"[bench] saturated: {len(items)} requests in {saturated:.2f} s ({len(items) / saturated:.1f} solves/s)")

    # the same requests as plain fp64 solves, one after another
    seq, seq_err = float("nan"), float("nan")
    if sequential:
        for it in items:
            it[4].zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        seq_err = 0.0
        for r, p, dA, b, x, Q in items:
            s = binding.Solver(dA, p.n, tol=p.tol, maxit=p.maxit, max_restarts=args.max_restarts)
            res = s.solve(b, x, Q)
            s.close()
            seq_err = max(seq_err, res.err_true)
        seq = time.perf_counter() - t1
        log(f"[bench] sequential plain fp64: {seq:.2f} s, max true residual {seq_err:.2e}")
    lat = np.array(lat)
    return {
        "metric": "batched solves/s", "value": len(items) / makespan, "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": 1e3 * makespan, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 inner / f64 refinement" if args.serve_precision == "ir" else "f64",
        "data": "synthetic",
        "config": {"workload": f"serving_poisson200_{len(items)}req", "requests": len(items),
                   "arrival_rate_per_s": 200.0, "N_range": [int(min(r.N for r in reqs)), int(max(r.N for r in reqs))],
                   "inflight": args.inflight, "budget_gb": args.budget_gb, "tol": 1e-10,
                   "small_n_max": args.small_n_max,
                   "order": "smallest footprint first (max wait 1 s)" if serve_order(args, binding) else "fifo",
                   "variant": "transpose-free (no A^H)" if args.transpose_free else "Algorithm 7.1 (explicit A^H)",
                   "all_converged": bool(all(f == 0 for f in flags)), "max_err_true": float(max(errs)),
                   "total_iterations": int(sum(iters))},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "peak_concurrency": int(st.peak_running), "peak_footprint_bytes": int(st.peak_used_bytes),
        "saturated": {"seconds": saturated, "solves_per_s": len(items) / saturated,
                      "all_converged": bool(all(f == 0 for f in sat_flags))},
        "sequential_fp64": {"seconds": seq, "solves_per_s": len(items) / seq, "max_err_true": seq_err},
    }


def bench_serving_sequences(args, torch, workloads, binding):
    """Serving with repeated matrices (Section 5.2 inside the server): `--matrices` systems drawn like the
    serving trace's, each the A of a sequence of `--systems` right-hand sides; the requests arrive as a
    Poisson stream at 200/s with the sequences interleaved at random.  Run twice on the same requests:
    as sequences (one solver per A, A^H built once, n from 4 by the rule with step 2 in [2, 8]) and as
    independent requests (create, solve, destroy each, n = 4)."""
    g = np.random.default_rng(55)
    base = workloads.serving_trace(count=args.matrices, n_min=args.seq_nmin)
    t = time.perf_counter()
    mats = []
    for r in base:
        p = workloads.serving_problem(r)
        if p.n < 8:   # Q with 8 columns for the rule's n_max
            p = workloads.serving_problem(workloads.Request(r.rid, r.arrival_s, r.dims, r.m, r.pe, 8, r.seed_stream))
        mats.append((p, binding.to_device(p.A), binding.column_major(p.Q)))
    order = np.repeat(np.arange(len(mats)), args.systems)
    g.shuffle(order)
    arrivals = np.cumsum(g.exponential(1 / 200.0, size=len(order)))
    arrivals -= arrivals[0]
    items = []
    for k, mi in enumerate(order):
        p, dA, Q = mats[mi]
        b = torch.from_numpy(g.standard_normal(p.N)).cuda()
        items.append((int(mi), float(arrivals[k]), b, torch.zeros(p.N, dtype=torch.float64, device="cuda")))
    torch.cuda.synchronize()
    log(f"[bench] {len(mats)} matrices, {len(items)} requests generated in {time.perf_counter() - t:.1f} s")

    def run(as_sequences):
        for it in items:
            it[3].zero_()
        torch.cuda.synchronize()
        server = binding.Server(budget_bytes=int(args.budget_gb * (1 << 30)), max_inflight=args.inflight,
                                small_n_max=args.small_n_max, order=serve_order(args, binding))
        t0 = time.perf_counter()
        tickets = []
        for mi, at, b, x in items:
            delay = t0 + at - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            p, dA, Q = mats[mi]
            if as_sequences:
                tickets.append(server.submit_sequence(mi + 1, dA, b, x, Q, 4, 2, 8, 2, tol=p.tol, maxit=p.maxit,
                                                      max_restarts=args.max_restarts))
            else:
                tickets.append(server.submit(dA, b, x, Q[:, :4], 4, tol=p.tol, maxit=p.maxit,
                                             max_restarts=args.max_restarts))
        lat, flags, errs, ns = [], [], [], []
        for tk in tickets:
            res, tim = server.wait(tk)
            lat.append(tim.latency_ms)
            flags.append(res.flag)
            errs.append(res.err_true)
            ns.append(tim.n_used)
        makespan = time.perf_counter() - t0
        if as_sequences:
            for mi in range(len(mats)):
                server.end_sequence(mi + 1)
        server.close()
        lat = np.array(lat)
        out = {"solves_per_s": len(items) / makespan, "makespan_s": makespan,
               "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
               "all_converged": bool(all(f == 0 for f in flags)), "max_err_true": float(max(errs)),
               "n_histogram": {int(v): int(c) for v, c in zip(*np.unique(ns, return_counts=True))}}
        log(f"[bench] {'sequences' if as_sequences else 'independent'}: {out}")
        return out

    run(True)   # warm-up of both paths' kernels
    seqs = run(True)
    indep = run(False)
    return {
        "metric": "batched solves/s, sequences of systems", "value": seqs["solves_per_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": 1e3 * seqs["makespan_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"serving_sequences_{len(mats)}x{args.systems}", "matrices": len(mats),
                   "N_range": [int(min(m[0].N for m in mats)), int(max(m[0].N for m in mats))],
                   "systems_per_matrix": args.systems, "arrival_rate_per_s": 200.0, "inflight": args.inflight,
                   "rule": "n from 4, step 2, in [2, 8]"},
        "sequences": seqs, "independent_n4": indep,
        "p50_ratio_independent_over_sequences": indep["latency_ms"]["p50"] / seqs["latency_ms"]["p50"],
    }


def bench_sequence(args, torch, workloads, binding):
    """A sequence of systems with the same A (3D convection-diffusion, new b each time): total solve time
    with n = 1 (BiCGStab), fixed n, and n chosen from one system to the next (Section 5.2).  --precond
    ilu0 runs every variant with ILU(0), the setting of the paper's Section 5.2 measurements."""
    m = args.m or 128
    n_max = 16
    if args.seq_matrix == "reservoir":
        p = workloads.config3(n=n_max)
        name = f"sequence_reservoir_{args.systems}systems"
        pre = binding.MLB_PRECOND_JACOBI
    else:
        p = workloads.config2(n=n_max, m=m)
        name = f"sequence_convdiff3d_m{m}_{args.systems}systems"
        pre = binding.MLB_PRECOND_NONE
    if args.precond == "ilu0":
        pre = binding.MLB_PRECOND_ILU0
        name += "_ilu0"
    g = np.random.default_rng(1106)
    rhs = [torch.from_numpy(g.standard_normal(p.N)).cuda() for _ in range(args.systems)]
    dA = binding.to_device(p.A)
    Q = binding.column_major(p.Q)
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    out = {}
    for var, n0, lo, hi, step in [("bicgstab_n1", 1, 1, 1, 0), ("fixed_n4", 4, 4, 4, 0), ("fixed_n8", 8, 8, 8, 0),
                                  ("auto_from_n4_step2", 4, 1, n_max, 2)]:
        seq = binding.Sequence(dA, n0, lo, hi, step, tol=p.tol, maxit=p.maxit, precond=pre,
                               max_restarts=args.max_restarts)
        Qv = Q[:, :hi]
        x.zero_()
        seq.solve(rhs[0], x, Qv)   # warm-up (first-use costs), not counted
        seq.close()
        seq = binding.Sequence(dA, n0, lo, hi, step, tol=p.tol, maxit=p.maxit, precond=pre,
                               max_restarts=args.max_restarts)
        total, used, iters, errs, flags = 0.0, [], [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in rhs:
            x.zero_()
            res, n = seq.solve(b, x, Qv)
            total += res.solve_ms
            used.append(n)
            iters.append(int(res.iter))
            errs.append(res.err_true)
            flags.append(int(res.flag))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        seq.close()
        out[var] = {"solve_ms_total": total, "wall_s": wall, "n_used": used, "iterations": iters, "flags": flags,
                    "err_true": errs, "max_err_true": max(errs)}
        log(f"[bench] sequence {var}: {total:.1f} ms over {len(rhs)} systems, n {used}, iterations {iters}")
    base = out["bicgstab_n1"]["solve_ms_total"]
    best = min(v["solve_ms_total"] for k, v in out.items() if k != "bicgstab_n1")
    return {
        "metric": "time-to-1e-10 residual, sequence of systems", "value": out["auto_from_n4_step2"]["wall_s"],
        "unit": "s", "n_gpus": 1, "steps": len(rhs), "warmup": 1,
        "ms_per_step": 1e3 * out["auto_from_n4_step2"]["wall_s"] / len(rhs), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": name, "N": p.N, "tol": p.tol, "max_restarts": args.max_restarts,
                   "preconditioner": {binding.MLB_PRECOND_NONE: "none", binding.MLB_PRECOND_JACOBI: "block Jacobi (right)",
                                      binding.MLB_PRECOND_ILU0: "ILU(0) (right)"}[pre]},
        "variants": out,
        "reduction_vs_bicgstab": {k: 1.0 - v["solve_ms_total"] / base for k, v in out.items() if k != "bicgstab_n1"},
        "best_reduction_vs_bicgstab": 1.0 - best / base,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="convdiff3d",
                    choices=["convdiff3d", "reservoir", "helmholtz", "serving", "sequence", "serving-seq"])
    ap.add_argument("--matrices", type=int, default=200, help="serving-seq: matrices (sequences)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="serving: skip the same requests as sequential fp64 solves")
    ap.add_argument("--seq-nmin", type=float, default=1e3, help="serving-seq: smallest target N of the matrices")
    ap.add_argument("--systems", type=int, default=10, help="sequence: right-hand sides")
    ap.add_argument("--seq-matrix", default="convdiff3d", choices=["convdiff3d", "reservoir"],
                    help="sequence: the matrix (reservoir runs with block Jacobi)")
    ap.add_argument("--requests", type=int, default=2000, help="serving: first requests of the seeded trace")
    ap.add_argument("--inflight", type=int, default=8, help="serving: solves in flight")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serving: HBM admission budget")
    ap.add_argument("--small-n-max", type=int, default=0,
                    help="serving: largest N batched in one-workgroup launches (0 = library default, -1 = none)")
    ap.add_argument("--serve-order", default="fifo", choices=["fifo", "smallest"],
                    help="serving: the workers' pick order (smallest: smallest footprint first, 1 s max wait)")
    ap.add_argument("--serve-precision", default="ir", choices=["fp64", "ir"],
                    help="serving: iteration precision (the serving configuration names fp32-IR)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "ir"])
    ap.add_argument("--n", type=int, default=0, help="number of shadow vectors (0 = the workload's)")
    ap.add_argument("--m", type=int, default=0, help="grid points per dimension (0 = the workload's)")
    ap.add_argument("--inner-tol", type=float, default=0.0)
    ap.add_argument("--max-restarts", type=int, default=2,
                    help="sequence and serving fp64 solves: restarts from the x reached while the true residual "
                         "is not below tol (the single-solve workloads run the paper's stop)")
    ap.add_argument("--velocity", default="constant", choices=["constant", "smooth"],
                    help="convdiff3d: one seeded direction (the benchmark's), or a smooth random direction field")
    ap.add_argument("--order", default="fused", choices=["fused", "literal"],
                    help="recurrence order: Gram-matrix form (fused) or the sequential loops (literal)")
    ap.add_argument("--transpose-free", action="store_true",
                    help="iterate without A^H (beta recurrence from q_s^H A g, w recombined)")
    ap.add_argument("--precond", default="auto", choices=["auto", "none", "jacobi", "ilu0"],
                    help="auto: block Jacobi for the reservoir workload, none otherwise; ilu0: ILU(0)")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="cap on the oracle sample (iterations); 0: about 15 s of CPU time")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary workloads (reservoir fp64 / fp32-IR, complex n = 16, ILU(0), serving)")
    ap.add_argument("--extra-steps", type=int, default=2, help="timed solves per secondary workload")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--calib-copy", type=float, default=0.0,
                    help="also run a plain device copy of this many GiB 3 times (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only; multi-GPU sharding is a design note, "
                                   "not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import workloads
    from paper_1106_3678_amd import binding

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    if args.workload == "serving":
        print(json.dumps(bench_serving(args, torch, workloads, binding, sequential=not args.no_sequential)),
              flush=True)
        return
    if args.workload == "sequence":
        print(json.dumps(bench_sequence(args, torch, workloads, binding)), flush=True)
        return
    if args.workload == "serving-seq":
        print(json.dumps(bench_serving_sequences(args, torch, workloads, binding)), flush=True)
        return
    t = time.perf_counter()
    p, fmt, cplx, grid = make_problem(args.workload, workloads, args.n, args.m, args.velocity)
    nnz = int(p.A.indptr[-1])          # entries (CSR) or 3x3 blocks (BSR3)
    profile_key = {"convdiff3d": f"convdiff3d_m{args.m or 128}_n{p.n}", "reservoir": f"reservoir_n{p.n}",
                   "helmholtz": f"helmholtz_m{args.m or 96}_n{p.n}"}[args.workload]
    if args.precision != "fp64":
        profile_key += "_ir"
    if args.transpose_free:
        profile_key += "_tf"
    if args.order == "literal":
        profile_key += "_literal"
    nbrows = len(p.A.indptr) - 1
    log(f"[bench] generated {p.name}: N={p.N} stored={nnz} in {time.perf_counter() - t:.1f} s")
    use_jacobi = args.precond == "jacobi" or (args.precond == "auto" and args.workload == "reservoir")
    precond = binding.MLB_PRECOND_ILU0 if args.precond == "ilu0" else \
        binding.MLB_PRECOND_JACOBI if use_jacobi else binding.MLB_PRECOND_NONE
    run = timed_solves(torch, binding, p, dev, args.precision, precond, args.transpose_free, args.order,
                       args.steps, args.warmup, args.inner_tol, keep_solver=True)
    solver = run.pop("solver")
    ms, last = run["ms"], run["last"]

    # Dominant kernel (SpMV with its fused combination and shadow dots), timed live with HIP
    # events on the solver's stream, over the workspace of the last solve.
    # value bytes of the iteration that the timed kernel belongs to (fp32 inner iteration for ir)
    sv = (16 if cplx else 8) if args.precision == "fp64" else (8 if cplx else 4)
    ms_spmv = solver.time_kernel(binding.MLB_KERNEL_SPMV_STEP, args.kernel_reps)
    bytes_spmv = spmv_step_bytes(nnz, nbrows, p.N, p.n, sv, bsr=(fmt == "bsr3"), literal=(args.order == "literal"),
                                 transpose_free=args.transpose_free)
    achieved = bytes_spmv / (ms_spmv * 1e-3) / 1e9
    ms_alpha = solver.time_kernel(binding.MLB_KERNEL_ALPHA_STEP, args.kernel_reps)
    ms_comb = solver.time_kernel(binding.MLB_KERNEL_COMBINE, args.kernel_reps)
    ms_recomb = solver.time_kernel(binding.MLB_KERNEL_RECOMBINE, args.kernel_reps)
    log(f"[bench] spmv-step {ms_spmv * 1e3:.1f} us/launch -> {achieved:.0f} GB/s ; alpha {ms_alpha * 1e3:.1f} us ; "
        f"combine {ms_comb * 1e3:.1f} us ; recombine {ms_recomb * 1e3:.1f} us")
    solver.close()
    copy_gbs = copy_rate_gbs(torch, dev)
    log(f"[bench] device copy (practical ceiling): {copy_gbs:.0f} GB/s")
    if args.calib_copy > 0:
        # a plain copy kernel of known size: reads and writes calib-copy GiB per launch
        nel = int(args.calib_copy * (1 << 30) / 8)
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {nel * 8} bytes read and written per launch, 3 launches")
        del src, dst
    # whole solve against the roofline: the kernels' algorithmic bytes over all iterations (fp64 iteration)
    bpi = bytes_per_iter(nnz, nbrows, p.N, p.n, 16 if cplx else 8, bsr=(fmt == "bsr3"),
                         transpose_free=args.transpose_free)
    whole_gbs = bpi * int(last.iter) / (ms * 1e-3) / 1e9 if args.precision == "fp64" else None

    line = {
        "metric": "time-to-1e-10 residual",
        "value": ms / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("c128" if cplx else "f64") if args.precision == "fp64" else
                 ("c64 inner / c128 refinement" if cplx else "f32 inner / f64 refinement"),
        "data": "synthetic",
        "config": {
            "workload": p.name,
            "grid": grid,
            "N": p.N,
            "stored_entries": nnz,
            "format": fmt,
            "n": p.n,
            "tol": p.tol,
            "precision": args.precision,
            "preconditioner": {binding.MLB_PRECOND_ILU0: "ILU(0) (right)", binding.MLB_PRECOND_JACOBI:
                               "block Jacobi (right)"}.get(precond, "none"),
            "variant": "transpose-free (no A^H)" if args.transpose_free else "Algorithm 7.1 (explicit A^H)",
            "recurrence_order": args.order,
            "iterations": int(last.iter),
            "outer_iters": int(last.outer_iters),
            "fp64_iters": int(last.fp64_iters),
            "flag": int(last.flag),
            "err_true": last.err_true,
            "err_recursive": last.err_recursive,
            "setup_ms": last.setup_ms,
            "matrix_setup_ms": run["create_ms"],
        },
        "roofline": {
            "kernel": "k_spmv_csrw / k_spmv_bsrw / k_spmv (SpMV step: w_i = A g_i with " +
                      ("c_i = q_i^H w_i only: literal order)" if args.order == "literal" else
                       "c_i = q_i^H w_i; q_s^H w_i, s > i, in the alpha pass)"
                       if s_from_alpha(p.n, args.transpose_free, sv=sv) else "q_s^H w_i, s >= i)"),
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": measured_traffic(profile_key),
            "bytes_per_launch": bytes_spmv,
            "us_per_launch": ms_spmv * 1e3,
            "copy_ceiling": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
            "whole_solve_bytes_per_iter": bpi,
            "whole_solve_gbs": whole_gbs,
            "whole_solve_frac": whole_gbs / PEAK_HBM_GBS if whole_gbs else None,
            "other_kernels_us": {"alpha": ms_alpha * 1e3, "combine": ms_comb * 1e3, "recombine": ms_recomb * 1e3},
        },
    }
    if not args.no_cpu:
        log("[bench] timing the oracle sample on the host")
        line["cpu_baseline"] = cpu_baseline(p, int(last.iter), args.cpu_iters, bpi)
        log(f"[bench] oracle: {line['cpu_baseline']['sample']}")
    del dA_keep[:]
    if not args.no_extras and args.workload == "convdiff3d" and args.steps > 0:
        line["secondary"] = secondary_workloads(args, torch, workloads, binding, dev)
    print(json.dumps(line), flush=True)


def make_problem(workload, workloads, n=0, m=0, velocity="constant"):
    """(problem, storage, complex?, grid) of a solve workload."""
    if workload == "convdiff3d":
        return workloads.config2(n=n or 4, m=m or 128, velocity=velocity), "csr", False, [m or 128] * 3
    if workload == "reservoir":
        p = workloads.config3(n=n or 8)
        return p, "bsr3", False, list(p.meta["grid"])
    return workloads.config5(n=n or 16, m=m or 96), "csr", True, [m or 96] * 3


dA_keep = []


def timed_solves(torch, binding, p, dev, precision, precond, transpose_free, order, steps, warmup, inner_tol=0.0,
                 keep_solver=False):
    """Upload p, create a solver, run `warmup` untimed and `steps` timed solves from x_0 = 0 (bracketed by
    device synchronisations); returns ms per solve, the last result and the solver set-up time."""
    cplx = np.iscomplexobj(p.A.data)
    dA = binding.to_device(p.A, dev)
    dA_keep.append(dA)
    tdt = torch.complex128 if cplx else torch.float64
    b = torch.from_numpy(p.b.astype(np.complex128 if cplx else np.float64)).to(dev)
    Q = binding.column_major(p.Q, dev)
    x = torch.zeros(p.N, dtype=tdt, device=dev)
    prec = binding.MLB_PREC_FP32_IR if precision == "ir" else binding.MLB_PREC_FP64
    torch.cuda.synchronize()
    t_create = time.perf_counter()
    solver = binding.Solver(dA, p.n, tol=p.tol, maxit=p.maxit, precision=prec, inner_tol=inner_tol,
                            precond=int(precond), transpose_free=transpose_free,
                            order=binding.MLB_ORDER_LITERAL if order == "literal" else binding.MLB_ORDER_FUSED)
    torch.cuda.synchronize()
    create_ms = 1e3 * (time.perf_counter() - t_create)   # validation, A^H (and M^{-1} / fp32 copies)

    def step():
        x.zero_()
        return solver.solve(b, x, Q)

    for w in range(warmup):
        r = step()
        log(f"[bench] {p.name} {precision} warmup {w}: flag={r.flag} iter={r.iter} err_true={r.err_true:.3e} "
            f"solve_ms={r.solve_ms:.1f}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for k, r in enumerate(results):
        log(f"[bench] {p.name} {precision} step {k}: flag={r.flag} iter={r.iter} outer={r.outer_iters} "
            f"fp64_iters={r.fp64_iters} err_rec={r.err_recursive:.3e} err_true={r.err_true:.3e} "
            f"solve_ms={r.solve_ms:.1f} setup_ms={r.setup_ms:.2f}")
    out = {"ms": 1e3 * elapsed / max(steps, 1), "last": results[-1] if results else None, "create_ms": create_ms}
    if keep_solver:
        out["solver"] = solver
    else:
        solver.close()
    return out


def secondary_workloads(args, torch, workloads, binding, dev):
    """The other configurations of the benchmark, one line each, so that every headline claim has a
    measured record: the reservoir system in fp64 and in fp32-IR, the complex Helmholtz system with
    n = 16, the 128^3 system with ILU(0) (the paper's preconditioner) for BiCGStab (n = 1) and ML(4),
    and the serving trace in fp64 and fp32-IR beside the same requests as sequential fp64 solves."""
    out = {}
    for name, wl, precs in (("reservoir_n8", "reservoir", ("fp64", "ir")), ("helmholtz_m96_n16", "helmholtz", ("fp64",))):
        t = time.perf_counter()
        p, fmt, cplx, grid = make_problem(wl, workloads)
        log(f"[bench] secondary: generated {p.name} in {time.perf_counter() - t:.1f} s")
        nnz, nbrows = int(p.A.indptr[-1]), len(p.A.indptr) - 1
        bpi = bytes_per_iter(nnz, nbrows, p.N, p.n, 16 if cplx else 8, bsr=(fmt == "bsr3"))
        rec = {"N": p.N, "n": p.n, "format": fmt, "preconditioner": "block Jacobi (right)" if wl == "reservoir" else
               "none", "steps": args.extra_steps, "warmup": 1}
        for prec in precs:
            r = timed_solves(torch, binding, p, dev, prec,
                             binding.MLB_PRECOND_JACOBI if wl == "reservoir" else binding.MLB_PRECOND_NONE,
                             False, "fused", args.extra_steps, 1)
            last = r["last"]
            e = {"ms_per_solve": r["ms"], "iterations": int(last.iter), "flag": int(last.flag),
                 "err_true": last.err_true, "outer_iters": int(last.outer_iters), "fp64_iters": int(last.fp64_iters)}
            if prec == "fp64":
                e["whole_solve_gbs"] = bpi * int(last.iter) / (r["ms"] * 1e-3) / 1e9
                e["whole_solve_frac"] = e["whole_solve_gbs"] / PEAK_HBM_GBS
                e["ms_per_iter"] = r["ms"] / max(int(last.iter), 1)
            rec[prec] = e
            dA_keep.clear()
            torch.cuda.empty_cache()
        if "ir" in rec:
            rec["ir_vs_fp64_time"] = rec["ir"]["ms_per_solve"] / rec["fp64"]["ms_per_solve"]
        out[name] = rec
    # ILU(0): BiCGStab (n = 1) against ML(4) on the 128^3 system, the setting of Section 5.2
    rec = {"preconditioner": "ILU(0) (right)", "steps": args.extra_steps, "warmup": 1}
    for n in (1, 4):
        p, _, _, _ = make_problem("convdiff3d", workloads, n=n)
        r = timed_solves(torch, binding, p, dev, "fp64", binding.MLB_PRECOND_ILU0, False, "fused", args.extra_steps, 1)
        last = r["last"]
        rec[f"n{n}"] = {"ms_per_solve": r["ms"], "iterations": int(last.iter), "flag": int(last.flag),
                        "err_true": last.err_true, "create_ms": r["create_ms"]}
        dA_keep.clear()
        torch.cuda.empty_cache()
    rec["reduction_n4_vs_bicgstab"] = 1.0 - rec["n4"]["ms_per_solve"] / rec["n1"]["ms_per_solve"]
    out["convdiff3d_m128_ilu0"] = rec
    sargs = argparse.Namespace(**vars(args))
    sargs.transpose_free = False
    generated = serving_items(sargs, torch, workloads, binding)
    seq_rate = None
    for prec in ("fp64", "ir"):
        sargs.serve_precision = prec
        sv = bench_serving(sargs, torch, workloads, binding, generated=generated, sequential=(prec == "fp64"))
        if prec == "fp64":
            seq_rate = sv["sequential_fp64"]["solves_per_s"]
            out["serving_sequential_fp64"] = sv["sequential_fp64"]
        out[f"serving_{prec}"] = {
            "solves_per_s": sv["value"], "latency_ms": sv["latency_ms"], "config": sv["config"],
            "dtype": sv["dtype"], "saturated_solves_per_s": sv["saturated"]["solves_per_s"],
            "speedup_saturated_vs_sequential_fp64": sv["saturated"]["solves_per_s"] / seq_rate}
    return out


if __name__ == "__main__":
    main()
