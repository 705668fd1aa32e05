"""First-step power-Lanczos estimators (section 3.4).

The first-step state is |psi_1> = (1 + alpha_1 H)|psi>.  Its energy, written
with the Monte Carlo weights rho(x) = |<x|psi>|^2/<psi|psi> (Eq. MC) and the
local quantities F(x, A) = <x|A|psi>/<x|psi>, is

    E_1(alpha) = (h1 + alpha (h20 + h11) + alpha^2 h12) / (1 + 2 alpha h1 + alpha^2 h11)

    h1  = sum_x rho(x) F(x, H)           h11 = sum_x rho(x) F(x, H)^2
    h20 = sum_x rho(x) F(x, H^2)         h12 = sum_x rho(x) F(x, H) F(x, H^2)

(real wave functions: F^dagger = F).  alpha_1 is the stationary point of
E_1, a root of the quadratic dE_1/dalpha = 0; of the two roots the one with
the lower E_1 is the minimum.

F(x, H) is the local energy of measure.py.  F(x, H^2) is written out here
from its definition, <x|H^2|psi>/<x|psi> = sum over two applications of the
Hamiltonian to <x| of the products of matrix elements times psi(x'')/psi(x),
with psi(x'') recomputed from scratch for every end point (the same
label-preserving hops as measure.local_energy, so no extra fermion sign).

THIS MODULE IS TEST INFRASTRUCTURE (see the package docstring).

Pinned (tests/test_oracle_lanczos.py) by exhaustive sums on small rings
against the moments <H^k> = psi^T H^k psi / psi^T psi of the exact-
diagonalisation matrix of ed.py, by E_1(alpha) against the Rayleigh quotient
of (1 + alpha H) psi built with that matrix, and by the optimal alpha against
the Rayleigh-Ritz problem in span{psi, H psi}.
"""
from __future__ import annotations

import math

import numpy as np

from .measure import neighbours
from .wavefunction import Model, log_psi, occupations, skew_table


def _apply_h(m: Model, pos: np.ndarray, nb) -> list[tuple[float, np.ndarray]]:
    """<pos| H = sum over (coefficient, pos') of <pos|H|pos'> <pos'|: the
    diagonal on-site term, then every label-preserving hop of one electron
    to an empty neighbouring spin-orbital with -t."""
    ns = m.n_sites
    nv = occupations(m, pos)
    out = [(float(np.dot(m.U, nv[:ns] * nv[ns:])), pos)]
    for a in range(m.n_elec):
        I = int(pos[a])
        sigma = I // ns
        i = I - sigma * ns
        for j, t in nb[i]:
            J = j + sigma * ns
            if nv[J]:
                continue
            new = pos.copy()
            new[a] = J
            out.append((-t, new))
    return out


def local_h2(m: Model, pos: np.ndarray, A: np.ndarray | None = None) -> float:
    """F(x, H^2) = <x|H^2|psi> / <x|psi>: every two-step path x -> x' -> x''
    of the Hamiltonian, weighted by psi(x'')/psi(x) from scratch."""
    if A is None:
        A = skew_table(m)
    pos = np.asarray(pos, dtype=np.int64)
    nb = neighbours(m)
    s0, l0 = log_psi(m, pos, A)
    if s0 == 0.0:
        raise ZeroDivisionError("psi(x) = 0")
    total = 0.0
    for c1, p1 in _apply_h(m, pos, nb):
        for c2, p2 in _apply_h(m, p1, nb):
            if c1 * c2 == 0.0:
                continue
            s2, l2 = log_psi(m, p2, A)
            if s2 != 0.0:
                total += c1 * c2 * s2 * s0 * math.exp(l2 - l0)
    return total


def moments(f1: np.ndarray, f2: np.ndarray, w: np.ndarray | None = None) -> dict:
    """h1, h11, h20, h12 as weighted averages (weights w, default uniform:
    the Monte Carlo mean over samples drawn from rho)."""
    f1 = np.asarray(f1, dtype=np.float64)
    f2 = np.asarray(f2, dtype=np.float64)
    w = np.full(len(f1), 1.0 / len(f1)) if w is None else np.asarray(w) / np.sum(w)
    return {"h1": float(np.dot(w, f1)), "h11": float(np.dot(w, f1 * f1)),
            "h20": float(np.dot(w, f2)), "h12": float(np.dot(w, f1 * f2))}


def energy(h: dict, alpha: float) -> float:
    """E_1(alpha) from the four moments."""
    num = h["h1"] + alpha * (h["h20"] + h["h11"]) + alpha * alpha * h["h12"]
    den = 1.0 + 2.0 * alpha * h["h1"] + alpha * alpha * h["h11"]
    return num / den


def optimal_alpha(h: dict) -> tuple[float, float]:
    """(alpha_1, E_1(alpha_1)): the root of dE_1/dalpha = 0 with the lower E_1.

    With E_1 = N/D, N = n0 + n1 a + n2 a^2, D = d0 + d1 a + d2 a^2, the
    condition N'D - ND' = 0 is the quadratic
        (n2 d1 - n1 d2) a^2 + 2 (n2 d0 - n0 d2) a + (n1 d0 - n0 d1) = 0
    (the cubic terms cancel)."""
    n0, n1, n2 = h["h1"], h["h20"] + h["h11"], h["h12"]
    d0, d1, d2 = 1.0, 2.0 * h["h1"], h["h11"]
    qa = n2 * d1 - n1 * d2
    qb = 2.0 * (n2 * d0 - n0 * d2)
    qc = n1 * d0 - n0 * d1
    if qa == 0.0:
        roots = [] if qb == 0.0 else [-qc / qb]
    else:
        disc = qb * qb - 4.0 * qa * qc
        if disc < 0.0:
            roots = []
        else:
            sq = math.sqrt(disc)
            roots = [(-qb + sq) / (2.0 * qa), (-qb - sq) / (2.0 * qa)]
    if not roots:
        return 0.0, energy(h, 0.0)
    best = min(roots, key=lambda a: energy(h, a))
    return best, energy(h, best)
