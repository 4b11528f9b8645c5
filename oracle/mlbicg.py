"""ML(n)BiCG, Algorithm 3.1 of the paper (Section 3).  Test infrastructure only.

The paper introduces this BiCG-like method with n left starting vectors
q_1..q_n and one right starting vector only to derive the ML(n)BiCGStab
algorithms, and expects it to be unstable (its shadow sequence
p_k = (A^H)^{g_n(k)} q_{r_n(k)}, eq. (3.1), repeatedly multiplies by A^H).
It is used here, on tiny systems and for few steps, to pin the ML(n)BiCGStabt
oracle: cycle 0 of ML(n)BiCGStabt reproduces these iterates, and every later
residual is Omega_{g_n(k+1)}(A) applied to this method's residual (eq. (4.1)).
It is itself pinned by the relations of Section 3: with n >= N and
q_k = hat r_{k-1} it is FOM, with q_k = A hat r_{k-1} it is GMRES, with n = 1
it is BiCG.

Step k (k = 1, 2, ...):
  alpha_k = p_k^H hat r_{k-1} / p_k^H A hat g_{k-1}
  hat x_k = hat x_{k-1} + alpha_k hat g_{k-1};  hat r_k = hat r_{k-1} - alpha_k A hat g_{k-1}
  for s = max(k-n, 0) .. k-1 (in order):
      beta_s = - p_{s+1}^H A (hat r_k + sum_{t<s} beta_t hat g_t) / p_{s+1}^H A hat g_s
  hat g_k = hat r_k + sum_s beta_s hat g_s
"""
from __future__ import annotations

import numpy as np

from .index import g_n, r_n


def mlbicg(A, b, Q, x0=None, steps=10, q_update=None):
    """Run ``steps`` steps of Algorithm 3.1; returns (xs, rs) with xs[k] = hat x_k, rs[k] = hat r_k.

    q_update(k, hat r_k) may return a vector that replaces q_{k+1} (used for the
    FOM/GMRES relations, where q_k is chosen from hat r_{k-1}); it is called for
    k = 0 before the first step and after every step.
    """
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    dtype = np.result_type(A.dtype, np.asarray(b).dtype, np.asarray(Q).dtype, np.float64)
    A = A.astype(dtype)
    AH = A.conj().T
    Q = np.array(Q, dtype=dtype, copy=True)
    N, n = Q.shape
    x = np.zeros(N, dtype=dtype) if x0 is None else np.array(x0, dtype=dtype, copy=True)
    r = np.asarray(b, dtype=dtype) - A @ x
    if q_update is not None:
        q = q_update(0, r)
        if q is not None:
            Q[:, 0] = q

    def p(k):
        # p_k = (A^H)^{g_n(k)} q_{r_n(k)}, eq. (3.1)
        v = Q[:, r_n(n, k) - 1].copy()
        for _ in range(g_n(n, k)):
            v = AH @ v
        return v

    gs = {0: r.copy()}          # hat g_s
    Ags = {0: A @ r}            # A hat g_s
    xs = [x.copy()]
    rs = [r.copy()]
    for k in range(1, steps + 1):
        pk = p(k)
        alpha = np.vdot(pk, r) / np.vdot(pk, Ags[k - 1])
        x = x + alpha * gs[k - 1]
        r = r - alpha * Ags[k - 1]
        xs.append(x.copy())
        rs.append(r.copy())
        if q_update is not None and k < n:
            q = q_update(k, r)
            if q is not None:
                Q[:, k] = q
        lo = max(k - n, 0)
        betas = {}
        acc = r.copy()
        for s in range(lo, k):
            ps = p(s + 1)
            betas[s] = -np.vdot(ps, A @ acc) / np.vdot(ps, Ags[s])
            acc = acc + betas[s] * gs[s]
        g = r.copy()
        for s in range(lo, k):
            g = g + betas[s] * gs[s]
        gs[k] = g
        Ags[k] = A @ g
        for s in list(gs):
            if s < k - n:
                del gs[s], Ags[s]
    return xs, rs
