"""Writes full_size_oracle.json: the CPU oracle run to convergence on the benchmark-size workloads.

Calls only oracle/ (and the seeded generators in workloads/).  For each case it stores the flag,
iteration count, recursive and true residuals, the norm of x, and x at 1024 seeded sample indices
(the whole x of a 2-million-row system is too large to keep), with a SHA-256 of the generated
inputs so that a test can tell whether the generator still produces the same system.

Usage: python tests/golden/make_full_size_oracle.py [case ...]   (about 3 minutes on one core)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "full_size_oracle.json")
N_SAMPLES = 1024

CASES = {
    "convdiff3d_m128_n1": lambda: workloads.config2(n=1, m=128),
    "convdiff3d_m128_n4": lambda: workloads.config2(n=4, m=128),
    "convdiff3d_m128_n8": lambda: workloads.config2(n=8, m=128),
    "convdiff3d_m128_n16": lambda: workloads.config2(n=16, m=128),
    "helmholtz_m96_n16": lambda: workloads.config5(n=16, m=96),
}


def fingerprint(p):
    """SHA-256 over the generated arrays (matrix structure and values, b, Q)."""
    h = hashlib.sha256()
    for a in (p.A.indptr, p.A.indices, p.A.data, p.b, np.asfortranarray(p.Q), p.x0):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def sample_indices(N):
    g = workloads.rng(99, N % 100003)
    return np.sort(g.choice(N, size=min(N_SAMPLES, N), replace=False))


def run(name):
    p = CASES[name]()
    t0 = time.perf_counter()
    o = oracle.mlbicgstabt(p.A, p.b, p.Q, x0=p.x0, tol=p.tol, maxit=p.maxit, kappa=p.kappa)
    dt = time.perf_counter() - t0
    idx = sample_indices(p.N)
    xs = o.x[idx]
    rec = {"name": p.name, "N": int(p.N), "n": int(p.n), "tol": p.tol, "flag": int(o.flag), "iter": int(o.iter),
           "err_recursive": float(o.err), "err_true": oracle.true_error(p.A, o.x, p.b),
           "x_norm": float(np.linalg.norm(o.x)), "sample_idx": idx.tolist(),
           "x_sample_re": np.real(xs).tolist(), "x_sample_im": np.imag(xs).tolist() if np.iscomplexobj(xs) else None,
           "inputs_sha256": fingerprint(p), "oracle_seconds": dt}
    print(f"{name}: flag {o.flag} iter {o.iter} err {o.err:.3e} true {rec['err_true']:.3e} in {dt:.1f} s",
          flush=True)
    return rec


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names or list(CASES):
        data[name] = run(name)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=0)


if __name__ == "__main__":
    main(sys.argv[1:])
