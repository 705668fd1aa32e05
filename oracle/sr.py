"""Stochastic reconfiguration (section 3.3.1) and the SR-CG solve (section 3.3.2).

Given samples mu = 1..N with local energies E_mu and log-derivatives O_mu,k
(estimators of section 3.3.2):

  <E> = (1/N) sum E_mu,  o_k = <O_k> = (1/N) sum O_mu,k,  O~ = O - o
  S_km = <O_k O_m> - <O_k><O_m> = (1/N) sum_mu O~_mu,k O~_mu,m
  g_m  = <H O_m> - <H><O_m>     = (1/N) sum_mu O~_mu,m (E_mu - <E>)
  Delta alpha = -dtau S^-1 g                       (Eq. SR_equation_system)

For real O the real parts in the paper are the values themselves, and the
centred product equals the printed covariance form.  The paper states no
regularisation; the one used (same on both sides) is

  S_reg = S + diag(eps_rel * S_kk + eps_abs), with any parameter whose
  S_kk < freeze frozen (its row/column replaced by the identity, g_k = 0).

S is positive definite and is solved by a Cholesky factorisation, or by the
CG method of Algorithm 1 with the matrix-free product
  S v = (1/N) O~^T (O~ v)   (the z(1) - z(2) form of section 3.3.2),
plus the diagonal shift.

Pinned by: CG = Cholesky; exact S and g by enumeration (exact <E> decreases
for a small step); and the closed-form covariance identity (tests/).
"""
from __future__ import annotations

import numpy as np


def sr_stats(O: np.ndarray, E: np.ndarray) -> dict:
    O = np.asarray(O, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    N = O.shape[0]
    ebar = float(E.mean())
    obar = O.mean(axis=0)
    Oc = O - obar
    S = Oc.T @ Oc / N
    g = Oc.T @ (E - ebar) / N
    return {"E": ebar, "E_var": float(((E - ebar) ** 2).mean()), "obar": obar,
            "Oc": Oc, "S": S, "g": g, "N": N}


def regularize(S: np.ndarray, g: np.ndarray, eps_rel: float, eps_abs: float,
               freeze: float = 1e-12) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    d = np.diag(S).copy()
    keep = d >= freeze
    Sr = S * np.outer(keep, keep)
    shift = np.where(keep, eps_rel * d + eps_abs, 1.0)
    Sr = Sr + np.diag(shift)
    gr = np.where(keep, g, 0.0)
    return Sr, gr, keep


def solve_cholesky(Sr: np.ndarray, b: np.ndarray) -> np.ndarray:
    L = np.linalg.cholesky(Sr)
    y = np.linalg.solve(L, b)
    return np.linalg.solve(L.T, y)


def cg(matvec, b: np.ndarray, x0: np.ndarray, eps: float, kmax: int) -> tuple[np.ndarray, int]:
    """Conjugate gradients for a symmetric positive-definite A (A x = b).

    Textbook derivation (Hestenes and Stiefel): minimise the quadratic
    q(x) = x.A.x / 2 - b.x, whose gradient is -r with r = b - A x.  From x the
    search goes along a direction d: the exact minimum of q on x + s d is at
    s = r.r / d.A.d (for the d built below), after which the residual is
    r - s A d.  The next direction is the new residual made A-conjugate to
    d, r + (r'.r' / r.r) d, so every step minimises q over the whole Krylov
    space seen so far.  The stopping rule is that of Algorithm 1
    (section 3.3.2): stop once |r|^2 < eps^2 |b|^2, or after kmax steps.
    Returns the solution and the number of steps taken."""
    x = np.array(x0, dtype=np.float64, copy=True)
    res = b - matvec(x)
    direction = res.copy()
    res2 = float(res @ res)
    stop2 = eps * eps * float(b @ b)
    steps = 0
    while steps < kmax:
        steps += 1
        a_dir = matvec(direction)
        s = res2 / float(direction @ a_dir)      # exact line minimum
        x += s * direction
        res -= s * a_dir
        res2_next = float(res @ res)
        if res2_next < stop2:
            break
        direction = res + (res2_next / res2) * direction   # A-conjugate to the last
        res2 = res2_next
    return x, steps


def matrix_free_matvec(Oc: np.ndarray, shift: np.ndarray, keep: np.ndarray):
    """v -> S_reg v without forming S: (1/N) O~^T (O~ v) + shift * v."""
    N = Oc.shape[0]
    m = keep.astype(np.float64)

    def mv(v):
        vv = v * m
        return m * (Oc.T @ (Oc @ vv)) / N + shift * v
    return mv


def sr_update(O: np.ndarray, E: np.ndarray, dtau: float, eps_rel: float, eps_abs: float,
              solver: str = "chol", cg_eps: float = 1e-10, cg_kmax: int | None = None,
              freeze: float = 1e-12) -> dict:
    st = sr_stats(O, E)
    Sr, gr, keep = regularize(st["S"], st["g"], eps_rel, eps_abs, freeze)
    if solver == "chol":
        x = solve_cholesky(Sr, gr)
        iters = 0
    else:
        d = np.diag(st["S"])
        shift = np.where(keep, eps_rel * d + eps_abs, 1.0)
        mv = matrix_free_matvec(st["Oc"], shift, keep)
        x, iters = cg(mv, gr, np.zeros_like(gr), cg_eps, cg_kmax or len(gr))
    st.update(dalpha=-dtau * x, x=x, keep=keep, S_reg=Sr, g_reg=gr, cg_iters=iters)
    return st
