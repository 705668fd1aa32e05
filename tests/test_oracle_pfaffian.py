"""Pins for the oracle's Philox generator and Pfaffian (CPU only)."""
import math
import os

import numpy as np
import pytest

from oracle.philox import philox4x32_10, scaled_index, uniform53
from oracle.pfaffian import pfaffian, pfaffian_brute, pfaffian_log

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _skew(n, rng):
    a = rng.standard_normal((n, n))
    return a - a.T


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])


def test_scaled_index_and_uniform_ranges():
    assert scaled_index(0, 7) == 0 and scaled_index(0xFFFFFFFF, 7) == 6
    assert uniform53(0, 0) == 0.0
    assert uniform53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53


@pytest.mark.parametrize("n", [2, 4, 6, 8, 10])
def test_parlett_reid_matches_matching_sum(n):
    rng = np.random.default_rng(n)
    for _ in range(5):
        a = _skew(n, rng)
        assert pfaffian(a) == pytest.approx(pfaffian_brute(a), rel=1e-12, abs=1e-12)


def test_closed_forms_2_and_4():
    a = np.array([[0, 3.0], [-3.0, 0]])
    assert pfaffian(a) == pytest.approx(3.0, rel=1e-15)
    rng = np.random.default_rng(4)
    x = _skew(4, rng)
    expect = x[0, 1] * x[2, 3] - x[0, 2] * x[1, 3] + x[0, 3] * x[1, 2]
    assert pfaffian(x) == pytest.approx(expect, rel=1e-13)


@pytest.mark.parametrize("n", [6, 12, 20, 40])
def test_square_is_determinant(n):
    rng = np.random.default_rng(100 + n)
    a = _skew(n, rng)
    s, l = pfaffian_log(a)
    sd, ld = np.linalg.slogdet(a)
    assert sd > 0
    assert 2 * l == pytest.approx(ld, rel=1e-12, abs=1e-10)


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8])
def test_antiparallel_block_is_det(m):
    rng = np.random.default_rng(m)
    M = rng.standard_normal((m, m))
    X = np.zeros((2 * m, 2 * m))
    X[:m, m:] = M
    X[m:, :m] = -M.T
    expect = (-1) ** (m * (m - 1) // 2) * np.linalg.det(M)
    assert pfaffian(X) == pytest.approx(expect, rel=1e-11)


@pytest.mark.parametrize("n", [4, 8, 14])
def test_congruence_rule(n):
    """Pf(B A B^T) = det(B) Pf(A) (appendix C, Eq. detPf)."""
    rng = np.random.default_rng(7 * n)
    A = _skew(n, rng)
    B = rng.standard_normal((n, n))
    assert pfaffian(B @ A @ B.T) == pytest.approx(np.linalg.det(B) * pfaffian(A), rel=1e-10)


def test_permutation_flips_sign():
    rng = np.random.default_rng(3)
    A = _skew(8, rng)
    P = np.eye(8)[[1, 0, 2, 3, 4, 5, 6, 7]]
    assert pfaffian(P @ A @ P.T) == pytest.approx(-pfaffian(A), rel=1e-13)


def test_odd_and_singular():
    assert pfaffian_log(np.zeros((3, 3)))[0] == 0.0
    z = np.zeros((4, 4))
    z[0, 1], z[1, 0] = 1.0, -1.0
    assert pfaffian(z) == 0.0
    assert math.isinf(pfaffian_log(z)[1])
