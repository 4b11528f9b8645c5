"""ML(n)BiCGStabt on the CPU: Algorithm 7.1 of the paper (Section 7), the
preconditioned form of Algorithm 4.1 (Section 4.3), in its i/j loop form.

Test infrastructure only: the GPU library never imports this module.

Notation follows the paper.  k = j n + i with 1 <= i <= n (eq. (2.1));
q_1..q_n are the shadow vectors (columns of Q), f_s = M^{-H} A^H q_s for
s = 1..n-1, g_k / w_k = A M^{-1} g_k are the direction vectors and their
images, c_k = q_{r_n(k+1)}^H w_k, e_k = q_{r_n(k+1)}^H r_k, and omega_j is
the minimisation parameter of cycle j (eq. (5.1)).  u^H v conjugates u.

Storage is the one the paper prescribes for its Matlab realisation: the
direction vectors live in two N x n blocks G and W used as ring buffers.
With 0-based column index s, at the start of cycle j column s holds
g_{(j-1)n+s} and w_{(j-1)n+s}; during cycle j column i is overwritten at
step i by g_{jn+i}, w_{jn+i}.  So when step i of cycle j runs its
beta~-recurrence, columns i..n-1 still hold the previous cycle's vectors,
and when it runs its beta-recurrence, columns 0..i-1 already hold this
cycle's.  c is kept in the same ring order.  Only the most recent
preconditioned direction hat g is kept (the x update uses it).

Control flow and exit codes follow the paper's realisation of the method:
  * ||b|| = 0 is replaced by 1; the stopping test is the recursive residual
    ||r_k|| / ||b|| < tol (strict), checked after every x update;
  * flag 0 = converged, 1 = maxit reached (tested after the x updates of the
    inner steps and after the omega step, not after the half step that ends a
    cycle), -1 = breakdown when a c_k or ||A u||^2 or omega is exactly zero;
  * if the half step that ends a cycle already meets the tolerance the solve
    stops there with the half-step x and iteration count k = jn + n.
Extension (not in the paper, shared with the GPU library): a non-finite c_k,
omega or residual norm is also reported as breakdown (-1).

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
BiCGStab iterate by iterate (Section 4.3 remark); finite termination for
n >= N against an LU solve; cycle 0 equals Algorithm 3.1 and every residual
satisfies eq. (4.1); FOM/GMRES relations via Algorithm 3.1 (Section 3);
Table 4.3 operation counts per steady cycle.  The transpose-free variant:
Table 4.2 operation counts at M = I, finite termination, iterates of
Algorithm 7.1 in exact arithmetic (agreement to rounding on well-conditioned
systems), and w_k = A M^{-1} g_k up to rounding.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


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
        if np.iscomplexobj(prod):
            return complex(math.fsum(prod.real), math.fsum(prod.imag))
        return math.fsum(prod)

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


def mlbicgstabt(A, b, Q, x0=None, tol=1e-10, maxit=1000, kappa=0.0, precond=None,
                record_x=0, counter=None, observer=None, q_update=None, summation="blas",
                transpose_free=False):
    """Solve A x = b with ML(n)BiCGStabt; n is the number of columns of Q.

    A        : matrix-like supporting ``A @ v`` and ``A.conj().T`` (dense or scipy sparse)
    precond  : None for M = I, else a pair (apply M^{-1}, apply M^{-H})
    record_x : keep x_1 .. x_record_x in ``x_history``
    counter  : an OpCounter; ``counter.mark(('cycle', j))`` is recorded at the start of every cycle
    observer : callable(event, **state) called at a few points (for biorthogonality tests)
    summation: order of the inner-product sums ("blas", "exact", "reversed"); see _Ops
    q_update : test hook realising adaptive shadow vectors (Section 3 FOM/GMRES relations):
               called as q_update(k, r_k) right after r_k is formed in cycle 0 (and with k = 0
               for r_0); a returned vector replaces q_{k+1} before it is first used.
    transpose_free: the variant described in the module docstring (no A^H, no F)
    """
    A_is_sparse = sp.issparse(A)
    dtype = np.result_type(A.dtype, np.asarray(b).dtype, np.asarray(Q).dtype, np.float64)
    b = np.asarray(b, dtype=dtype)
    Q = np.array(Q, dtype=dtype, order="F", copy=True)
    N, n = Q.shape
    if n < 1:
        raise ValueError("n must be >= 1")
    AH = None
    if not transpose_free:
        AH = A.conj().T
        if A_is_sparse:
            AH = AH.tocsr()
    ops = _Ops(A, precond, counter, summation)

    def apply_mh(v):     # M^{-H} v
        return v if precond is None else precond[1](v)

    x = np.zeros(N, dtype=dtype) if x0 is None else np.array(x0, dtype=dtype, copy=True)
    res = Result(x=x, err=np.inf, iter=0, flag=1)

    def finish(flag, k, err):
        res.x, res.flag, res.iter, res.err = x, flag, k, float(err)
        return res

    def record(k, err):
        res.err_history.append(float(err))
        if k <= record_x:
            res.x_history.append(x.copy())

    # Setup: ||b||, r_0 = b - A x_0, early exit.
    bnrm2 = float(np.linalg.norm(b))
    if bnrm2 == 0.0:
        bnrm2 = 1.0
    r = b - A @ x
    err = ops.norm(r) / bnrm2
    res.err_history.append(float(err))
    if err < tol:
        return finish(0, 0, err)

    # f_s = M^{-H} A^H q_s, s = 1..n-1 (computed once; with q_update, column by column).
    F = np.zeros((N, max(n - 1, 0)), dtype=dtype, order="F")

    def set_shadow(col, q):
        Q[:, col] = q
        if col < n - 1 and not transpose_free:
            F[:, col] = apply_mh(AH @ Q[:, col])

    if not transpose_free:
        for s in range(n - 1):
            F[:, s] = apply_mh(AH @ Q[:, s])
    if q_update is not None:
        q0 = q_update(0, r)
        if q0 is not None:
            set_shadow(0, q0)

    G = np.zeros((N, n), dtype=dtype, order="F")
    W = np.zeros((N, n), dtype=dtype, order="F")
    c = np.zeros(n, dtype=dtype)

    # g_0 = r_0, hat g_0 = M^{-1} r_0, w_0 = A hat g_0, c_0 = q_1^H w_0, e_0 = q_1^H r_0.
    G[:, 0] = r
    ghat = ops.psolve(r)
    W[:, 0] = ops.matvec(ghat)
    c[0] = ops.dot(Q[:, 0], W[:, 0])
    if c[0] == 0 or _bad(c[0]):
        return finish(-1, 0, err)
    e = ops.dot(Q[:, 0], r)
    if observer is not None:
        observer("w", k=0, col=0, Q=Q, W=W, G=G, F=F)

    k = 0
    omega = None
    j = 0
    while True:
        if counter is not None:
            counter.mark(("cycle", j))
        # ---- steps k = jn + i, i = 1..n-1 -----------------------------------
        for i in range(1, n):
            alpha = e / c[i - 1]                       # alpha_{jn+i} = e_{jn+i-1} / c_{jn+i-1}
            x = ops.saxpy(x, alpha, ghat)              # x_{jn+i}
            r = ops.saxpy(r, -alpha, W[:, i - 1])      # r_{jn+i}
            k += 1
            err = ops.norm(r) / bnrm2
            record(k, err)
            if _bad(err):
                return finish(-1, k, err)
            if err < tol:
                return finish(0, k, err)
            if k >= maxit:
                return finish(1, k, err)
            if j == 0 and q_update is not None:
                qn = q_update(k, r)
                if qn is not None:
                    set_shadow(i, qn)
            e = ops.dot(Q[:, i], r)                    # e_{jn+i} = q_{i+1}^H r_{jn+i}
            if j >= 1:
                # beta~ recurrence against the previous cycle's w, g (columns i..n-1)
                bt = -e / c[i]
                zw = ops.saxpy(r, bt, W[:, i])
                g = ops.scale(bt, G[:, i])
                for s in range(i + 1, n):
                    bt = -ops.dot(Q[:, s], zw) / c[s]
                    zw = ops.saxpy(zw, bt, W[:, s])
                    g = ops.saxpy(g, bt, G[:, s])
                g = ops.saxpy(zw, -1.0 / omega, g)    # g = z_w - g / omega_j
                if observer is not None:
                    observer("zw", k=k, col=i, Q=Q, zw=zw)
            elif transpose_free:
                g = r
            if transpose_free:
                # beta recurrence with f_s^H g = q_s^H v, v = A M^{-1} g carried along
                v = ops.matvec(ops.psolve(g))
                for s in range(0, i):
                    beta = -ops.dot(Q[:, s], v) / c[s]
                    g = ops.saxpy(g, beta, G[:, s])
                    v = ops.saxpy(v, beta, W[:, s])
                G[:, i] = g
                ghat = g if precond is None else ops.psolve(g)
                W[:, i] = v                            # w_{jn+i} = A M^{-1} g_{jn+i}, recombined
            else:
                if j >= 1:
                    # beta recurrence against this cycle's g (columns 0..i-1)
                    for s in range(0, i):
                        beta = -ops.dot(F[:, s], g) / c[s]
                        g = ops.saxpy(g, beta, G[:, s])
                else:
                    beta = -ops.dot(F[:, 0], r) / c[0]
                    g = ops.saxpy(r, beta, G[:, 0])
                    for s in range(1, i):
                        beta = -ops.dot(F[:, s], g) / c[s]
                        g = ops.saxpy(g, beta, G[:, s])
                G[:, i] = g
                ghat = ops.psolve(g)
                W[:, i] = ops.matvec(ghat)             # w_{jn+i}
            c[i] = ops.dot(Q[:, i], W[:, i])           # c_{jn+i} = q_{i+1}^H w_{jn+i}
            if observer is not None:
                observer("w", k=k, col=i, Q=Q, W=W, G=G, F=F)
            if c[i] == 0 or _bad(c[i]):
                return finish(-1, k, err)

        # ---- step k = jn + n: half step, then the minimisation step ---------
        alpha = e / c[n - 1]
        x = ops.saxpy(x, alpha, ghat)
        u = ops.saxpy(r, -alpha, W[:, n - 1])          # u_{jn+n}
        err = ops.norm(u) / bnrm2
        if _bad(err):
            return finish(-1, k, err)
        if err < tol:
            k += 1
            record(k, err)
            return finish(0, k, err)
        uhat = ops.psolve(u)
        z = ops.matvec(uhat)                           # A hat u
        zz = ops.dot(z, z)
        if zz == 0 or _bad(zz):
            return finish(-1, k, err)
        rho = ops.dot(z, u)
        omega = rho / zz                               # eq. (5.1), first line
        if kappa > 0:
            rho = rho / (ops.norm(z) * ops.norm(u))
            a = abs(rho)
            if a < kappa and a != 0:
                omega = omega * kappa / a              # guard omega away from zero
        if omega == 0 or _bad(omega):
            return finish(-1, k, err)
        res.omegas.append(omega)
        x = ops.saxpy(x, omega, uhat)                  # x_{jn+n}
        r = ops.saxpy(u, -omega, z)                    # r_{jn+n}
        k += 1
        err = ops.norm(r) / bnrm2
        record(k, err)
        if _bad(err):
            return finish(-1, k, err)
        if err < tol:
            return finish(0, k, err)
        if k >= maxit:
            return finish(1, k, err)

        # ---- close of the cycle: g_{jn+n} from this cycle's w, g (all columns)
        e = ops.dot(Q[:, 0], r)                        # e_{jn+n} = q_1^H r_{jn+n}
        bt = -e / c[0]
        zw = ops.saxpy(r, bt, W[:, 0])
        g = ops.scale(bt, G[:, 0])
        for s in range(1, n):
            bt = -ops.dot(Q[:, s], zw) / c[s]
            zw = ops.saxpy(zw, bt, W[:, s])
            g = ops.saxpy(g, bt, G[:, s])
        g = ops.saxpy(zw, -1.0 / omega, g)
        if observer is not None:
            observer("zw", k=k, col=0, Q=Q, zw=zw)
        G[:, 0] = g
        ghat = ops.psolve(g)
        W[:, 0] = ops.matvec(ghat)                     # w_{jn+n}
        c[0] = ops.dot(Q[:, 0], W[:, 0])               # c_{jn+n} = q_1^H w_{jn+n}
        if observer is not None:
            observer("w", k=k, col=0, Q=Q, W=W, G=G, F=F)
        if c[0] == 0 or _bad(c[0]):
            return finish(-1, k, err)
        j += 1
