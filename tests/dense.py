"""Dense-matrix helpers for the oracle's pins: build the full matrix a set of
bands stands for, and solve it by routes that share nothing with the oracle's
recurrences (LAPACK with pivoting, exact rational elimination)."""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def tri_dense(a, b, c, cyclic=False):
    n = len(b)
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] = b[i]
        if i > 0:
            A[i, i - 1] = a[i]
        if i < n - 1:
            A[i, i + 1] = c[i]
    if cyclic:
        A[0, n - 1] = a[0]
        A[n - 1, 0] = c[n - 1]
    return A


def penta_dense(a, b, c, d, e, cyclic=False):
    n = len(c)
    A = np.zeros((n, n))
    for i in range(n):
        for off, band in ((-2, a), (-1, b), (0, c), (1, d), (2, e)):
            j = i + off
            if 0 <= j < n:
                A[i, j] = band[i]
            elif cyclic:
                A[i, j % n] = band[i]
    return A


def exact_solve(A, rhs):
    """Gauss-Jordan elimination with partial pivoting in exact rationals."""
    n = len(A)
    M = [[Fraction(A[i][j]) for j in range(n)] + [Fraction(rhs[i])] for i in range(n)]
    for col in range(n):
        piv = max(range(col, n), key=lambda r: abs(M[r][col]))
        if M[piv][col] == 0:
            raise ZeroDivisionError("singular")
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def rel_err(x, ref, axis=0):
    """Per-system relative 2-norm error, max over systems."""
    x, ref = np.asarray(x), np.asarray(ref)
    num = np.linalg.norm(x - ref, axis=axis)
    den = np.linalg.norm(ref, axis=axis)
    return float(np.max(num / np.where(den == 0, 1.0, den)))
