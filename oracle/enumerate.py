"""Exhaustive sums over every configuration of a tiny lattice.

Canonical basis (section 3.1.1): the fixed-S^z configuration lists the up
electrons first, then the down electrons, each in ascending site order; with
I = i + Ns*sigma (section 3.2.1) this is ascending spin-orbital order.  The
same order defines the Jordan-Wigner signs of the exact-diagonalisation
basis in ed.py, so psi(x) evaluated here is the component of |psi> on the
ED basis vector of x.

Exact expectation values use rho(x) = |psi(x)|^2 / sum |psi|^2 (Eq. MC).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import measure
from .wavefunction import Model, log_psi, skew_table


def configurations(m: Model) -> list[np.ndarray]:
    ns = m.n_sites
    out = []
    for up in itertools.combinations(range(ns), m.n_up):
        for dn in itertools.combinations(range(ns), m.n_dn):
            out.append(np.array(list(up) + [d + ns for d in dn], dtype=np.int64))
    return out


def amplitudes(m: Model, confs: list[np.ndarray] | None = None) -> np.ndarray:
    """psi(x) for every canonical configuration (relative scale)."""
    if confs is None:
        confs = configurations(m)
    A = skew_table(m)
    sl = [log_psi(m, c, A) for c in confs]
    lmax = max(l for s, l in sl if s != 0.0)
    return np.array([0.0 if s == 0.0 else s * math.exp(l - lmax) for s, l in sl])


def exact_energy(m: Model) -> tuple[float, np.ndarray, np.ndarray, list]:
    """(E_var, probabilities, E_loc per configuration, configurations)."""
    confs = configurations(m)
    psi = amplitudes(m, confs)
    p = psi ** 2
    p /= p.sum()
    A = skew_table(m)
    eloc = np.array([measure.local_energy(m, c, A) if p[k] > 1e-300 else 0.0
                     for k, c in enumerate(confs)])
    return float(np.dot(p, eloc)), p, eloc, confs


def exact_sr(inst, m: Model) -> dict:
    """Exact <E>, <O>, S and g with weights rho(x) (section 3.3.1)."""
    E, p, eloc, confs = exact_energy(m)
    A = skew_table(m)
    keep = [k for k in range(len(confs)) if p[k] > 1e-14]
    O = np.array([measure.log_derivs(inst, m, confs[k], A) for k in keep])
    w = p[keep] / p[keep].sum()
    el = eloc[keep]
    obar = w @ O
    ebar = float(w @ el)
    Oc = O - obar
    S = (Oc * w[:, None]).T @ Oc
    g = Oc.T @ (w * (el - ebar))
    return {"E": ebar, "obar": obar, "S": S, "g": g, "p": w, "O": O, "eloc": el}
