"""Index functions of Section 2.

For a positive integer n and any integer k the paper defines
g_n(k) = floor((k - 1) / n), rounding toward minus infinity, and
r_n(k) = k - n g_n(k), which takes values in {1, ..., n}.  Writing
k = j n + i with 1 <= i <= n gives g_n(k) = j and r_n(k) = i (eq. (2.1)).
Python's ``//`` is floor division, so it already rounds toward minus
infinity for negative k (C's ``/`` would not).
"""


def g_n(n: int, k: int) -> int:
    if n < 1:
        raise ValueError("n must be a positive integer")
    return (k - 1) // n


def r_n(n: int, k: int) -> int:
    return k - n * g_n(n, k)
