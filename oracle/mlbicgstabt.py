"""ML(n)BiCGStabt on the CPU, written from Algorithm 4.1 (Section 4.3) and its
preconditioned form, Algorithm 7.1 (Section 7), with the omega choice of
eq. (5.1).

Test infrastructure only: the GPU library never imports this module.

The iteration is written as the paper states Algorithm 4.1: one loop over
k = 1, 2, ..., with k = j n + i, j = g_n(k), i = r_n(k) (eq. (2.1)).  The
vectors of step k carry the index k: g_k, w_k = A M^{-1} g_k and
c_k = q_{r_n(k+1)}^H w_k are kept by k in small maps that forget every index
older than k - n (no recurrence reaches further back), so the code reads with
the subscripts of the paper rather than with a storage scheme.

What one step computes (u^H v conjugates u; q_1..q_n the shadow vectors,
f_s = M^{-H} A^H q_s for s = 1..n-1, hat v = M^{-1} v):
  alpha_k = e_{k-1} / c_{k-1}, with e_{k-1} = q_{r_n(k)}^H r_{k-1};
  x_k = x_{k-1} + alpha_k hat g_{k-1};
  if i < n:  r_k = r_{k-1} - alpha_k w_{k-1};
  if i = n:  u_k = r_{k-1} - alpha_k w_{k-1};  omega_{j+1} from A hat u_k
             (eq. (5.1), kappa guard when kappa > 0);
             x_k += omega_{j+1} hat u_k;  r_k = u_k - omega_{j+1} A hat u_k;
  beta~ recurrence over s = max(k-n, 0) .. (i < n ? jn - 1 : k - 1):
      beta~_s = -q_{r_n(s+1)}^H z_w / c_s  (z_w starting at r_k, so the first
      coefficient is -e_k / c_s);  z_w += beta~_s w_s;  g += beta~_s g_s;
      then g_k = z_w - (1 / omega) g, with the omega of the cycle the
      recurrence ran over (for j = 0 and i < n the sum is empty and g_k = r_k);
  beta recurrence (i < n only) over s = jn .. k-1, on this cycle's vectors:
      beta_s = -f_{r_n(s+1)}^H g_k / c_s;  g_k += beta_s g_s;
  w_k = A hat g_k;  c_k = q_{r_n(k+1)}^H w_k;  e_k = q_{r_n(k+1)}^H r_k.

Readings of what the algorithm leaves open (the same on the GPU):
  * ||b|| = 0 is replaced by 1.  The stopping test is the recursive residual
    ||r_k|| / ||b|| < tol (strict), checked after every x update; the step
    i = n tests ||u_k|| too, and a solve that meets the tolerance there stops
    with x = x_{k-1} + alpha_k hat g_{k-1} and iteration count k.
  * maxit is tested after the x updates of steps with i < n and after the
    omega update, not on u_k.
  * breakdown (flag -1): c_k, ||A hat u||^2 or omega exactly zero, and, an
    extension of this library, any of them or a residual norm non-finite.
    A breakdown inside step i = n reports k - 1 iterations (x_k was not
    completed); one on c_k reports k.
  * g_k = z_w - (1/omega) g multiplies by the reciprocal, as the algorithm
    writes it.
  * kappa guard (eq. (5.1)): rho = (A hat u)^H u / (||A hat u|| ||u||), and
    omega is scaled by kappa / |rho| when 0 < |rho| < kappa.

Transpose-free variant (``transpose_free=True``; an addition of this
library, the paper prints no such listing): the beta recurrence needs
f_s^H g = q_s^H (A M^{-1} g), so the product v = A M^{-1} g of the vector that
enters it is formed first and carried along: beta_s = -q_s^H v / c_s,
g += beta_s g_s, v += beta_s w_s, and then w_k = v with no further product.
F and A^H are never formed.  Per iteration this costs (n-1)/2 more saxpys
than Algorithm 7.1 and (n-1) N less storage, which are the costs Table 4.2
gives for the paper's second algorithm; that the two are the same algorithm
cannot be checked from the paper, which only cites its listing.  With a
preconditioner, hat g = M^{-1} g is formed once more after the recurrence.

Parity pins (CPU tests): Table 2.1; n = 1 equals an independently written
BiCGStab iterate by iterate (Section 4.3 remark), also with the kappa guard of
eq. (5.1) on systems where the guard fires; the preconditioned iteration equals
the unpreconditioned one on A M^{-1} y = b with x = M^{-1} y (Section 4.3);
finite termination for n >= N against an LU solve; cycle 0 equals
Algorithm 3.1 and every residual satisfies eq. (4.1); FOM/GMRES relations via
Algorithm 3.1 (Section 3); Table 4.3 operation counts per steady cycle.  The
transpose-free variant: Table 4.2 operation counts at M = I, finite
termination, iterates of Algorithm 7.1 in exact arithmetic (agreement to
rounding on well-conditioned systems), and w_k = A M^{-1} g_k up to rounding.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .index import g_n, r_n


class OpCounter:
    """Counts the vector operations the way Table 4.3 does.

    matvec: A v; precond: M^{-1} v; dot: u^H v; saxpy: u + a v;
    scale: u +- v or a v (the table's third column); norm: ||r|| for the
    stopping test (not counted by the table).
    """

    KEYS = ("matvec", "precond", "dot", "saxpy", "scale", "norm")

    def __init__(self):
        self.counts = {k: 0 for k in self.KEYS}
        self.marks = []

    def add(self, key):
        self.counts[key] += 1

    def mark(self, label):
        self.marks.append((label, dict(self.counts)))


@dataclass
class Result:
    x: np.ndarray
    err: float              # recursive ||r|| / ||b|| at exit
    iter: int
    flag: int
    err_history: list = field(default_factory=list)   # err after every x update, indexed by k
    x_history: list = field(default_factory=list)     # x_1 .. x_K (K = record_x)
    omegas: list = field(default_factory=list)        # omega_1, omega_2, ...


def true_error(A, x, b):
    """E(n) of Section 5: ||b - A x|| / ||b|| (||b|| = 0 replaced by 1)."""
    bn = np.linalg.norm(b)
    return float(np.linalg.norm(b - A @ x) / (bn if bn != 0 else 1.0))


class _Ops:
    """The primitive operations one iteration is built from (counted).

    ``summation`` picks the order in which u^H v = sum conj(u_i) v_i is
    accumulated; the paper does not fix it.  "blas" (numpy's vdot) is the
    default; "exact" rounds the sum of the rounded products once (math.fsum),
    "reversed" sums from the last entry.  The alternatives exist to measure how
    much an iteration depends on summation order alone.
    """

    def __init__(self, A, precond, counter, summation="blas"):
        if summation not in ("blas", "exact", "reversed"):
            raise ValueError("summation must be 'blas', 'exact' or 'reversed'")
        self.A = A
        self.precond = precond
        self.counter = counter
        self.summation = summation

    def _c(self, key):
        if self.counter is not None:
            self.counter.add(key)

    def matvec(self, v):
        self._c("matvec")
        return self.A @ v

    def psolve(self, v):
        self._c("precond")
        return v if self.precond is None else self.precond[0](v)

    def dot(self, u, v):
        self._c("dot")
        if self.summation == "blas":
            return np.vdot(u, v)        # u^H v
        if self.summation == "reversed":
            return np.vdot(u[::-1], v[::-1])
        prod = np.conj(u) * v
        if np.iscomplexobj(prod):     # a numpy scalar, so later divisions are numpy's
            return prod.dtype.type(complex(math.fsum(prod.real), math.fsum(prod.imag)))
        return prod.dtype.type(math.fsum(prod))

    def saxpy(self, u, a, v):
        self._c("saxpy")
        return u + a * v

    def scale(self, a, v):
        self._c("scale")
        return a * v

    def norm(self, v):
        self._c("norm")
        return float(np.linalg.norm(v))


def _bad(z):
    return not np.isfinite(z)


def _omega(ops, z, u, kappa):
    """omega_{j+1} of eq. (5.1) from z = A hat u and u; None on breakdown.

    Plain minimisation omega = z^H u / ||z||^2; with kappa > 0 the
    Sleijpen-van der Vorst guard rescales it by kappa / |rho| when the cosine
    rho = z^H u / (||z|| ||u||) is nonzero and below kappa in modulus.
    """
    zz = ops.dot(z, z)
    if zz == 0 or _bad(zz):
        return None
    zu = ops.dot(z, u)
    om = zu / zz
    if kappa > 0:
        rho = zu / (ops.norm(z) * ops.norm(u))
        a = abs(rho)
        if a < kappa and a != 0:
            om = om * kappa / a
    if om == 0 or _bad(om):
        return None
    return om


def mlbicgstabt(A, b, Q, x0=None, tol=1e-10, maxit=1000, kappa=0.0, precond=None,
                record_x=0, counter=None, observer=None, q_update=None, summation="blas",
                transpose_free=False):
    """Solve A x = b with ML(n)BiCGStabt; n is the number of columns of Q.

    A        : matrix-like supporting ``A @ v`` and ``A.conj().T`` (dense or scipy sparse)
    precond  : None for M = I, else a pair (apply M^{-1}, apply M^{-H})
    record_x : keep x_1 .. x_record_x in ``x_history``
    counter  : an OpCounter; ``counter.mark(('cycle', j))`` is recorded when step k = jn + 1 starts
    observer : callable(event, **state), for the biorthogonality tests:
               ("w", k=k, w=w_k, g=g_k, Q=Q) once w_k is formed, and
               ("zw", k=k, zw=z_w, Q=Q) at the end of every beta~ recurrence
    summation: order of the inner-product sums ("blas", "exact", "reversed"); see _Ops
    q_update : test hook realising adaptive shadow vectors (Section 3 FOM/GMRES relations):
               called as q_update(k, r_k) right after r_k is formed while k < n (and with
               k = 0 for r_0); a returned vector replaces q_{k+1} before it is first used.
    transpose_free: the variant described in the module docstring (no A^H, no F)
    """
    dtype = np.result_type(A.dtype, np.asarray(b).dtype, np.asarray(Q).dtype, np.float64)
    b = np.asarray(b, dtype=dtype)
    Q = np.array(Q, dtype=dtype, order="F", copy=True)
    N, n = Q.shape
    if n < 1:
        raise ValueError("n must be >= 1")
    ops = _Ops(A, precond, counter, summation)
    AH = None
    if not transpose_free:
        AH = A.conj().T
        if sp.issparse(A):
            AH = AH.tocsr()

    def q(a):                     # q_a, 1-based as in the paper
        return Q[:, a - 1]

    def f_of(qv):                 # f = M^{-H} A^H q
        f = AH @ qv
        return f if precond is None else precond[1](f)

    x = np.zeros(N, dtype=dtype) if x0 is None else np.array(x0, dtype=dtype, copy=True)
    res = Result(x=x, err=np.inf, iter=0, flag=1)

    def stop(flag, k, err):
        res.x, res.flag, res.iter, res.err = x, flag, k, float(err)
        return res

    def verdict(err, k, test_maxit):
        """The flag the solve ends with after an x update, or None to go on."""
        if _bad(err):
            return -1
        if err < tol:
            return 0
        if test_maxit and k >= maxit:
            return 1
        return None

    # Step 2 of Algorithm 7.1: ||b||, r_0, the early exit, f_1..f_{n-1}.
    bnrm2 = float(np.linalg.norm(b)) or 1.0
    r = b - A @ x
    err = ops.norm(r) / bnrm2
    res.err_history.append(float(err))
    if err < tol:
        return stop(0, 0, err)
    f = {}
    if not transpose_free:
        for a in range(1, n):
            f[a] = f_of(q(a))
    if q_update is not None:
        q_new = q_update(0, r)
        if q_new is not None:
            Q[:, 0] = q_new
            if 1 in f:
                f[1] = f_of(q(1))

    # g_0 = r_0, w_0 = A hat g_0, c_0 = q_1^H w_0, e_0 = q_1^H r_0.
    g = {0: r}
    gh_last = ops.psolve(r)         # hat g of the latest step (the x update reads it)
    w = {0: ops.matvec(gh_last)}
    c = {0: ops.dot(q(1), w[0])}
    if c[0] == 0 or _bad(c[0]):
        return stop(-1, 0, err)
    e = ops.dot(q(1), r)
    if observer is not None:
        observer("w", k=0, w=w[0], g=g[0], Q=Q)
    omega = {}                      # omega_j by cycle, j >= 1

    k = 0
    while True:
        k += 1
        j, i = g_n(n, k), r_n(n, k)
        if counter is not None and i == 1:
            counter.mark(("cycle", j))
        alpha = e / c[k - 1]
        x = ops.saxpy(x, alpha, gh_last)
        if i < n:
            r = ops.saxpy(r, -alpha, w[k - 1])
            err = ops.norm(r) / bnrm2
            res.err_history.append(float(err))
            if k <= record_x:
                res.x_history.append(x.copy())
            flag = verdict(err, k, True)
            if flag is not None:
                return stop(flag, k, err)
            if q_update is not None and k < n:
                q_new = q_update(k, r)
                if q_new is not None:
                    Q[:, k] = q_new
                    if k + 1 in f:
                        f[k + 1] = f_of(q(k + 1))
            lo, hi, om = max(k - n, 0), j * n, omega.get(j)
        else:
            u = ops.saxpy(r, -alpha, w[k - 1])
            err = ops.norm(u) / bnrm2
            if _bad(err):                       # step k did not complete: k - 1 iterations
                return stop(-1, k - 1, err)
            if err < tol:                       # converged on the half step
                res.err_history.append(float(err))
                if k <= record_x:
                    res.x_history.append(x.copy())
                return stop(0, k, err)
            uh = ops.psolve(u)
            z = ops.matvec(uh)
            om = _omega(ops, z, u, kappa)
            if om is None:
                return stop(-1, k - 1, err)
            omega[j + 1] = om
            res.omegas.append(om)
            x = ops.saxpy(x, om, uh)
            r = ops.saxpy(u, -om, z)
            err = ops.norm(r) / bnrm2
            res.err_history.append(float(err))
            if k <= record_x:
                res.x_history.append(x.copy())
            flag = verdict(err, k, True)
            if flag is not None:
                return stop(flag, k, err)
            lo, hi = k - n, k
        e = ops.dot(q(r_n(n, k + 1)), r)        # e_k

        # beta~ recurrence over w_s, g_s, s = lo .. hi-1, then g_k = z_w - (1/omega) g
        if hi > lo:
            zw, gk = r, None
            for s in range(lo, hi):
                bt = -(e if s == lo else ops.dot(q(r_n(n, s + 1)), zw)) / c[s]
                zw = ops.saxpy(zw, bt, w[s])
                gk = ops.scale(bt, g[s]) if gk is None else ops.saxpy(gk, bt, g[s])
            gk = ops.saxpy(zw, -(1.0 / om), gk)
            if observer is not None:
                observer("zw", k=k, zw=zw, Q=Q)
        else:
            gk = r

        # beta recurrence over this cycle's g_s, s = jn .. k-1 (steps i < n), then w_k
        if i < n and transpose_free:
            v = ops.matvec(ops.psolve(gk))      # v = A M^{-1} g, carried along
            for s in range(j * n, k):
                beta = -ops.dot(q(r_n(n, s + 1)), v) / c[s]
                gk = ops.saxpy(gk, beta, g[s])
                v = ops.saxpy(v, beta, w[s])
            gh_last = gk if precond is None else ops.psolve(gk)
            w[k] = v
        else:
            if i < n:
                for s in range(j * n, k):
                    beta = -ops.dot(f[r_n(n, s + 1)], gk) / c[s]
                    gk = ops.saxpy(gk, beta, g[s])
            gh_last = ops.psolve(gk)
            w[k] = ops.matvec(gh_last)
        g[k] = gk
        c[k] = ops.dot(q(r_n(n, k + 1)), w[k])
        if observer is not None:
            observer("w", k=k, w=w[k], g=g[k], Q=Q)
        if c[k] == 0 or _bad(c[k]):
            return stop(-1, k, err)
        for old in [s for s in g if s < k - n]:
            del g[old], w[old], c[old]
