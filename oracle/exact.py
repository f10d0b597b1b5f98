"""Exact rational Gaussian elimination (``fractions.Fraction``).

TEST INFRASTRUCTURE ONLY.  Brute force on tiny integer systems: the result
is the exact solution of eq. (syst), with no rounding at all, so it pins the
floating-point oracle independently of any library.
"""
from __future__ import annotations

from fractions import Fraction


def solve(A, b):
    """Solve A x = b exactly.  A: list of rows (ints or Fractions); b: list.
    Raises ZeroDivisionError if A is singular."""
    n = len(A)
    M = [[Fraction(v) for v in row] + [Fraction(b[i])] for i, row in enumerate(A)]
    for k in range(n):
        p = next((i for i in range(k, n) if M[i][k] != 0), None)
        if p is None:
            raise ZeroDivisionError("singular matrix")
        M[k], M[p] = M[p], M[k]
        for i in range(k + 1, n):
            if M[i][k] != 0:
                t = M[i][k] / M[k][k]
                for j in range(k, n + 1):
                    M[i][j] -= t * M[k][j]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        s = M[i][n] - sum(M[i][j] * x[j] for j in range(i + 1, n))
        x[i] = s / M[i][i]
    return x
