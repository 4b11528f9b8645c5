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
    "drop_w_term": ("zw = ops.saxpy(zw, bt, W[:, s])", "zw = zw"),
    # a wrong sign in g = z_w - g / omega
    "sign_omega": ("g = ops.saxpy(zw, -1.0 / omega, g)    # g = z_w - g / omega_j",
                   "g = ops.saxpy(zw, 1.0 / omega, g)"),
    # an off-by-one ring index in alpha
    "alpha_index": ("alpha = e / c[i - 1]", "alpha = e / c[i % n]"),
    # a dropped beta recurrence (no A^H)
    "drop_f_loop": ("beta = -ops.dot(F[:, s], g) / c[s]\n                        g = ops.saxpy(g, beta, G[:, s])\n                else:",
                    "pass\n                else:"),
    # a transposed (unconjugated / wrong-side) product for F
    "f_not_transposed": ("F[:, s] = apply_mh(AH @ Q[:, s])", "F[:, s] = apply_mh(A @ Q[:, s])"),
    # the wrong residual in the omega step
    "omega_r": ("r = ops.saxpy(u, -omega, z)", "r = ops.saxpy(r, -omega, z)"),
    # an unconjugated inner product
    "no_conj": ("return np.vdot(u, v)", "return np.dot(u, v)"),
}

# Slips in the transpose-free variant, checked with the same subset run on that variant.
TF_MUTATIONS = {
    # v not carried along the beta recurrence
    "tf_drop_v_update": ("v = ops.saxpy(v, beta, W[:, s])", "v = v"),
    # a wrong sign of beta
    "tf_beta_sign": ("beta = -ops.dot(Q[:, s], v) / c[s]", "beta = ops.dot(Q[:, s], v) / c[s]"),
    # the wrong shadow vector in the beta recurrence
    "tf_q_index": ("beta = -ops.dot(Q[:, s], v) / c[s]", "beta = -ops.dot(Q[:, (s + 1) % n], v) / c[s]"),
    # the product taken before the beta~ recurrence has formed g
    "tf_product_of_r": ("v = ops.matvec(ops.psolve(g))", "v = ops.matvec(ops.psolve(r))"),
}


def _mutant(name):
    old, new = {**MUTATIONS, **TF_MUTATIONS}[name]
    text = open(SRC).read()
    assert old in text, name
    mod = types.ModuleType(f"oracle_mutant_{name}")
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
