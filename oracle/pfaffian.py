"""Pfaffians of real skew-symmetric matrices.

The paper evaluates <x|phi_Pf> = (N_e/2)! Pf(X) and computes the Pfaffian
with a library (section 3.2.1); that library's real-matrix routine is the
Parlett-Reid reduction with partial pivoting, written out here:

  for k = 0, 2, 4, ...:
    pick p = argmax_{i > k} |A[i, k]| and swap row/column k+1 with p
    (a transposition, so Pf changes sign);
    Pf picks up the pivot A[k, k+1];
    a congruence with a unit lower-triangular Gauss transform removes the
    rest of row/column k and leaves A[k+2:, k+2:] updated by
      tau = A[k, k+2:] / A[k, k+1]
      A[k+2:, k+2:] += tau (x) A[k+2:, k+1] - A[k+2:, k+1] (x) tau.

Pinned (tests/test_oracle_pfaffian.py) by the perfect-matching sum below
for n <= 10, Pf(X)^2 = det(X) (section 3.2.1), Pf(B A B^T) = det B Pf A
(appendix C, Eq. detPf), the 2x2/4x4 closed forms, and the block form
Pf([[0, M], [-M^T, 0]]) = (-1)^{m(m-1)/2} det M.
"""
from __future__ import annotations

import math

import numpy as np


def pfaffian_log(a: np.ndarray) -> tuple[float, float]:
    """Return (sign, log|Pf(a)|); sign is 0.0 and log is -inf when Pf = 0."""
    A = np.array(a, dtype=np.float64, copy=True)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix required")
    if n % 2:
        return 0.0, -math.inf
    sign = 1.0
    logabs = 0.0
    for k in range(0, n - 1, 2):
        p = k + 1 + int(np.argmax(np.abs(A[k + 1:, k])))
        if p != k + 1:
            A[[k + 1, p], :] = A[[p, k + 1], :]
            A[:, [k + 1, p]] = A[:, [p, k + 1]]
            sign = -sign
        piv = A[k, k + 1]
        if piv == 0.0:
            return 0.0, -math.inf
        logabs += math.log(abs(piv))
        if piv < 0:
            sign = -sign
        if k + 2 < n:
            tau = A[k, k + 2:] / piv
            col = A[k + 2:, k + 1].copy()
            A[k + 2:, k + 2:] += np.outer(tau, col) - np.outer(col, tau)
    return sign, logabs


def pfaffian(a: np.ndarray) -> float:
    s, l = pfaffian_log(a)
    return 0.0 if s == 0.0 else s * math.exp(l)


def pfaffian_brute(a: np.ndarray) -> float:
    """Sum over perfect matchings by expansion along the first row (n <= 12)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    if n % 2:
        return 0.0

    def rec(idx: tuple[int, ...]) -> float:
        if not idx:
            return 1.0
        i0 = idx[0]
        total = 0.0
        for pos in range(1, len(idx)):
            j = idx[pos]
            rest = idx[1:pos] + idx[pos + 1:]
            total += (-1.0) ** (pos - 1) * a[i0, j] * rec(rest)
        return total

    return rec(tuple(range(n)))
