"""The pins are sensitive: each plausible slip planted in a copy of the oracle fails one of them.

The copy is made from the oracle's source text on the CPU; the real oracle is untouched.
"""
import functools
import os
import sys
import types

import numpy as np
import pytest

from oracle import mlbicg
from tests import textbook

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "mlbicgstabt.py")

MUTATIONS = {
    # a dropped term in the beta~ recurrence
    "drop_w_term": ("zw = ops.saxpy(zw, bt, w[s])", "zw = zw"),
    # a wrong sign in g_k = z_w - (1/omega) g
    "sign_omega": ("gk = ops.saxpy(zw, -(1.0 / om), gk)", "gk = ops.saxpy(zw, (1.0 / om), gk)"),
    # an off-by-one index in alpha_k = e_{k-1} / c_{k-1}
    "alpha_index": ("alpha = e / c[k - 1]", "alpha = e / c[max(k - 2, 0)]"),
    # a dropped beta recurrence (no A^H)
    "drop_f_loop": ("beta = -ops.dot(f[r_n(n, s + 1)], gk) / c[s]\n                    gk = ops.saxpy(gk, beta, g[s])",
                    "pass"),
    # a transposed (unconjugated / wrong-side) product for F
    "f_not_transposed": ("f = AH @ qv", "f = A @ qv"),
    # the wrong residual in the omega step
    "omega_r": ("r = ops.saxpy(u, -om, z)", "r = ops.saxpy(r, -om, z)"),
    # an unconjugated inner product
    "no_conj": ("return np.vdot(u, v)", "return np.dot(u, v)"),
    # F = A^H M^{-H} Q instead of M^{-H} A^H Q
    "f_precond_side": ("f = AH @ qv\n        return f if precond is None else precond[1](f)",
                       "f = qv if precond is None else precond[1](qv)\n        return AH @ f"),
    # x += alpha g instead of alpha hat g
    "x_g_not_ghat": ("x = ops.saxpy(x, alpha, gh_last)", "x = ops.saxpy(x, alpha, g[k - 1])"),
    # x += omega u instead of omega hat u
    "x_u_not_uhat": ("x = ops.saxpy(x, om, uh)", "x = ops.saxpy(x, om, u)"),
    # rho of eq. (5.1) normalised by ||z||^2 instead of ||z|| ||u||
    "rho_norm": ("rho = zu / (ops.norm(z) * ops.norm(u))", "rho = zu / (ops.norm(z) * ops.norm(z))"),
    # the guard's factor inverted
    "kappa_factor": ("om = om * kappa / a", "om = om * a / kappa"),
}

# Slips in the transpose-free variant, checked with the same subset run on that variant.
TF_MUTATIONS = {
    # v not carried along the beta recurrence
    "tf_drop_v_update": ("v = ops.saxpy(v, beta, w[s])", "v = v"),
    # a wrong sign of beta
    "tf_beta_sign": ("beta = -ops.dot(q(r_n(n, s + 1)), v) / c[s]", "beta = ops.dot(q(r_n(n, s + 1)), v) / c[s]"),
    # the wrong shadow vector in the beta recurrence
    "tf_q_index": ("beta = -ops.dot(q(r_n(n, s + 1)), v) / c[s]", "beta = -ops.dot(q(r_n(n, s + 2)), v) / c[s]"),
    # the product taken before the beta~ recurrence has formed g
    "tf_product_of_r": ("v = ops.matvec(ops.psolve(gk))", "v = ops.matvec(ops.psolve(r))"),
}


def _mutant(name):
    old, new = {**MUTATIONS, **TF_MUTATIONS}[name]
    text = open(SRC).read()
    assert old in text, name
    mod = types.ModuleType(f"oracle_mutant_{name}")
    mod.__package__ = "oracle"               # its relative import of the index functions
    sys.modules[mod.__name__] = mod          # dataclasses look their module up here
    try:
        exec(compile(text.replace(old, new), f"<mutant {name}>", "exec"), mod.__dict__)
    finally:
        del sys.modules[mod.__name__]
    return mod.mlbicgstabt


def _pins_hold(solve):
    """A compact subset of the CPU pins; returns False as soon as one fails."""
    g = np.random.default_rng(5)
    for cplx in (False, True):
        N = 8
        A = g.standard_normal((N, N)) / np.sqrt(N) + 2.0 * np.eye(N)
        b = g.standard_normal(N)
        Q = g.standard_normal((N, N))
        if cplx:
            A = A + 1j * g.standard_normal((N, N)) / np.sqrt(N)
            b = b + 1j * g.standard_normal(N)
            Q = Q + 1j * g.standard_normal((N, N))
        try:
            res = solve(A, b, Q, tol=1e-10, maxit=80)
        except Exception:
            return False
        xs = np.linalg.solve(A, b)
        if res.flag != 0 or res.iter != N or np.linalg.norm(res.x - xs) > 1e-10 * np.linalg.norm(xs):
            return False
        # n = 1 against BiCGStab
        q = Q[:, 0]
        r1 = solve(A, b, q[:, None], tol=1e-10, maxit=200, record_x=200)
        ref, it, _ = textbook.bicgstab(A, b, q, tol=1e-10, maxit=200)
        if r1.iter != it or np.linalg.norm(r1.x_history[0] - ref[0]) > 1e-10 * np.linalg.norm(ref[0]):
            return False
        # cycles >= 1 against Algorithm 3.1 and eq. (4.1)
        N2, n = 24, 3
        A2 = g.standard_normal((N2, N2)) / np.sqrt(N2) + 2.5 * np.eye(N2)
        b2 = g.standard_normal(N2)
        Q2 = g.standard_normal((N2, n))
        if cplx:
            A2 = A2 + 1j * g.standard_normal((N2, N2)) / np.sqrt(N2)
            Q2 = Q2 + 1j * g.standard_normal((N2, n))
        r2 = solve(A2, b2, Q2, tol=1e-30, maxit=3 * n, record_x=3 * n)
        _, rhat = mlbicg(A2, b2, Q2, steps=3 * n)
        for k in range(1, 3 * n + 1):
            v = rhat[k]
            for m in range((k) // n):
                v = v - r2.omegas[m] * (A2 @ v)
            rk = b2 - A2 @ r2.x_history[k - 1]
            if np.linalg.norm(rk - v) > 1e-8 * np.linalg.norm(v) + 1e-13 * np.linalg.norm(b2):
                return False
        # n = 1 with the kappa guard of eq. (5.1) against the guarded textbook BiCGStab
        N3 = 30
        S = g.standard_normal((N3, N3)) + (1j * g.standard_normal((N3, N3)) if cplx else 0)
        A3 = np.eye(N3) + 0.5 * (S - S.conj().T) / np.sqrt(N3)
        b3 = g.standard_normal(N3) + (1j * g.standard_normal(N3) if cplx else 0)
        q3 = g.standard_normal(N3) + (1j * g.standard_normal(N3) if cplx else 0)
        r3 = solve(A3, b3, q3[:, None], tol=1e-12, maxit=200, kappa=0.7, record_x=200)
        ref, it, _, oms, fired = textbook.bicgstab_guarded(A3, b3, q3, 0.7, tol=1e-12, maxit=200)
        if not any(fired[:8]) or len(r3.omegas) < 8:
            return False
        for k in range(8):
            if abs(r3.omegas[k] - oms[k]) > 1e-8 * abs(oms[k]):
                return False
            if np.linalg.norm(r3.x_history[k] - ref[k]) > 1e-8 * np.linalg.norm(ref[k]):
                return False
        # with M: the iteration on A M^{-1} y = b, x = M^{-1} y (Section 4.3), n = 3, with kappa
        N4, n4 = 12, 3
        A4 = g.standard_normal((N4, N4)) / np.sqrt(N4) + 2.0 * np.eye(N4)
        M4 = np.eye(N4) + 0.3 * g.standard_normal((N4, N4)) / np.sqrt(N4)
        b4 = g.standard_normal(N4)
        Q4 = g.standard_normal((N4, n4))
        if cplx:
            A4 = A4 + 1j * g.standard_normal((N4, N4)) / np.sqrt(N4)
            M4 = M4 + 0.3j * g.standard_normal((N4, N4)) / np.sqrt(N4)
            Q4 = Q4 + 1j * g.standard_normal((N4, n4))
        Mi = np.linalg.inv(M4)
        pre = (lambda v: np.linalg.solve(M4, v), lambda v: np.linalg.solve(M4.conj().T, v))
        for kap in (0.0, 0.7):
            px = solve(A4, b4, Q4, tol=1e-11, maxit=200, kappa=kap, precond=pre, record_x=12)
            py = solve(A4 @ Mi, b4, Q4, tol=1e-11, maxit=200, kappa=kap, record_x=12)
            if px.flag != 0 or py.flag != 0 or px.iter != py.iter:
                return False
            for xk, yk in zip(px.x_history, py.x_history):
                if np.linalg.norm(xk - Mi @ yk) > 1e-10 * np.linalg.norm(Mi @ yk):
                    return False
    return True


def test_unmutated_oracle_passes_the_subset():
    from oracle import mlbicgstabt
    assert _pins_hold(mlbicgstabt)
    assert _pins_hold(functools.partial(mlbicgstabt, transpose_free=True))


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    assert not _pins_hold(_mutant(name)), f"planted slip {name!r} was not caught"


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
@pytest.mark.parametrize("name", sorted(TF_MUTATIONS))
def test_transpose_free_mutation_is_caught(name):
    mutant = functools.partial(_mutant(name), transpose_free=True)
    assert not _pins_hold(mutant), f"planted slip {name!r} was not caught"
