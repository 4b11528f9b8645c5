"""Textbook Krylov solvers written independently of the oracle, used to pin it.

* BiCGStab as van der Vorst published it (SIAM J. Sci. Stat. Comput. 13, 1992),
  with shadow residual r~ = q_1 and the usual early exit on ||s||.
* The same BiCGStab with the stabilised choice of omega of Sleijpen and
  van der Vorst (Numer. Algorithms 10, 1995): when the cosine between t = A s
  and s is below kappa in modulus, omega is enlarged by kappa / |cosine|.
* BiCG (Fletcher 1976) with shadow residual r~_0 = q_1.
* FOM and GMRES iterates by brute force: an orthonormal Krylov basis (Arnoldi
  with repeated modified Gram-Schmidt) and a Galerkin solve / least-squares fit.
"""
import numpy as np


def bicgstab(A, b, q, x0=None, tol=1e-10, maxit=100):
    """Returns (xs, iters, flag): xs[k-1] = x after iteration k."""
    A = np.asarray(A.toarray() if hasattr(A, "toarray") else A)
    dt = np.result_type(A.dtype, b.dtype, q.dtype, np.float64)
    x = np.zeros(len(b), dt) if x0 is None else x0.astype(dt).copy()
    bn = np.linalg.norm(b) or 1.0
    r = b - A @ x
    rt = q.astype(dt)
    rho_old = alpha = omega = 1.0
    v = np.zeros_like(x)
    p = np.zeros_like(x)
    xs = []
    for it in range(1, maxit + 1):
        rho = np.vdot(rt, r)
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = A @ p
        alpha = rho / np.vdot(rt, v)
        s = r - alpha * v
        if np.linalg.norm(s) / bn < tol:
            x = x + alpha * p
            xs.append(x.copy())
            return xs, it, 0
        t = A @ s
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        xs.append(x.copy())
        if np.linalg.norm(r) / bn < tol:
            return xs, it, 0
        rho_old = rho
    return xs, maxit, 1


def bicgstab_guarded(A, b, q, kappa, tol=1e-10, maxit=100):
    """BiCGStab with the kappa-guarded omega.  Returns (xs, iters, flag, omegas, fired):
    omegas[m] is the omega used in iteration m + 1, fired[m] whether the guard changed it."""
    A = np.asarray(A.toarray() if hasattr(A, "toarray") else A)
    dt = np.result_type(A.dtype, b.dtype, q.dtype, np.float64)
    x = np.zeros(len(b), dt)
    bn = np.linalg.norm(b) or 1.0
    r = b.astype(dt) - A @ x
    rt = q.astype(dt)
    p = r.copy()
    rho = np.vdot(rt, r)
    xs, omegas, fired = [], [], []
    for it in range(1, maxit + 1):
        v = A @ p
        alpha = rho / np.vdot(rt, v)
        s = r - alpha * v
        if np.linalg.norm(s) / bn < tol:
            x = x + alpha * p
            xs.append(x.copy())
            return xs, it, 0, omegas, fired
        t = A @ s
        ts, tt = np.vdot(t, s), np.vdot(t, t).real
        omega = ts / tt
        cos = abs(ts) / (np.sqrt(tt) * np.linalg.norm(s))
        guard = 0 < cos < kappa
        if guard:
            omega = omega * (kappa / cos)
        omegas.append(omega)
        fired.append(bool(guard))
        x = x + alpha * p + omega * s
        r = s - omega * t
        xs.append(x.copy())
        if np.linalg.norm(r) / bn < tol:
            return xs, it, 0, omegas, fired
        rho_new = np.vdot(rt, r)
        beta = (rho_new / rho) * (alpha / omega)
        rho = rho_new
        p = r + beta * (p - omega * v)
    return xs, maxit, 1, omegas, fired


def bicg(A, b, q, steps):
    """Returns xs[0..steps] (xs[0] = x_0 = 0)."""
    A = np.asarray(A.toarray() if hasattr(A, "toarray") else A)
    dt = np.result_type(A.dtype, b.dtype, q.dtype, np.float64)
    x = np.zeros(len(b), dt)
    r = b.astype(dt) - A @ x
    rt = q.astype(dt).copy()
    p, pt = r.copy(), rt.copy()
    xs = [x.copy()]
    for _ in range(steps):
        Ap = A @ p
        rho = np.vdot(rt, r)
        alpha = rho / np.vdot(pt, Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        rt = rt - np.conj(alpha) * (A.conj().T @ pt)
        beta = np.vdot(rt, r) / rho
        p = r + beta * p
        pt = rt + np.conj(beta) * pt
        xs.append(x.copy())
    return xs


def krylov_basis(A, r0, k):
    """Orthonormal basis of span{r0, A r0, ..., A^{k-1} r0} (Arnoldi, MGS applied twice)."""
    A = np.asarray(A.toarray() if hasattr(A, "toarray") else A)
    V = np.zeros((len(r0), k), dtype=np.result_type(A.dtype, r0.dtype))
    V[:, 0] = r0 / np.linalg.norm(r0)
    for j in range(1, k):
        w = A @ V[:, j - 1]
        for _ in range(2):
            for i in range(j):
                w = w - np.vdot(V[:, i], w) * V[:, i]
        V[:, j] = w / np.linalg.norm(w)
    return V


def fom_iterate(A, b, k):
    """x_k with x_0 = 0: x_k in K_k(A, b), b - A x_k orthogonal to K_k(A, b)."""
    A = np.asarray(A.toarray() if hasattr(A, "toarray") else A)
    V = krylov_basis(A, b, k)
    y = np.linalg.solve(V.conj().T @ A @ V, V.conj().T @ b)
    return V @ y


def gmres_iterate(A, b, k):
    """x_k with x_0 = 0: x_k in K_k(A, b) minimising ||b - A x_k||."""
    A = np.asarray(A.toarray() if hasattr(A, "toarray") else A)
    V = krylov_basis(A, b, k)
    y, *_ = np.linalg.lstsq(A @ V, b, rcond=None)
    return V @ y
