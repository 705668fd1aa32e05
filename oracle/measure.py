"""Local energy and logarithmic derivatives for one configuration.

Local energy (section 3.1.1, Eq. MC): E_loc(x) = sum_x' <x|H|x'> psi(x')/psi(x)
for H = H_T + H_U (Eq. GHam with the on-site term H_U of section 2.3):

  diagonal   sum_i U_i n_iup n_idn
  hopping    for every electron a (site i, spin s) and every bond (i, j) with
             (j, s) empty: -t_ij * psi(x with a moved to j)/psi(x).

The moved electron keeps its label (row of X), so the fermion sign of
c+_j c_i is carried by the Pfaffian itself and no extra sign appears.

Log-derivatives O_k = d ln<x|psi> / d alpha_k (section 3.3.1):

  pair amplitude f_ij (Eq. DiffPf and appendix C): with a the up electron at
  site i and b the down electron at site j, dPf(X)/dF_{(i,up),(j,dn)} =
  -Pf(X) (X^-1)_ab, so O_{f_k} = -sum over class members of (X^-1)_ab;
  Gutzwiller g_k: sum_{i in class} n_iup n_idn (the count D_k(x));
  Jastrow v_k: sum over unordered pairs {i, j} in the class of
  (n_i - 1)(n_j - 1) (the 1/2 of log P_J cancels the double count);
  RBM: O_a = sigma_v, O_b = tanh theta_h, O_W = tanh theta_h sigma_v.

Pinned by finite differences of wavefunction.log_psi and, for the energy, by
the exhaustive <H> against exact diagonalisation (tests/).
"""
from __future__ import annotations

import numpy as np

import math

from .pfaffian import pfaffian_log
from .wavefunction import Model, log_psi, mapped, occupations, skew_table


def neighbours(m: Model) -> list[list[tuple[int, float]]]:
    nb = [[] for _ in range(m.n_sites)]
    for (i, j), t in zip(m.bonds, m.bond_t):
        nb[int(i)].append((int(j), float(t)))
        nb[int(j)].append((int(i), float(t)))
    return nb


def local_energy(m: Model, pos: np.ndarray, A: np.ndarray | None = None) -> float:
    if A is None:
        A = skew_table(m)
    ns = m.n_sites
    pos = np.asarray(pos)
    nv = occupations(m, pos)
    e = float(np.dot(m.U, nv[:ns] * nv[ns:]))
    nb = neighbours(m)
    # psi(x) once; every hop term is psi(x')/psi(x) with psi(x') from scratch
    s0, l0 = log_psi(m, pos, A)
    if s0 == 0.0:
        raise ZeroDivisionError("psi(x) = 0")
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
            s1, l1 = log_psi(m, new, A)
            if s1 != 0.0:
                e += -t * s1 * s0 * math.exp(l1 - l0)
    return e


def log_derivs(inst, m: Model, pos: np.ndarray, A: np.ndarray | None = None) -> np.ndarray:
    """O_k for every parameter of the instance, in the parameter-vector order."""
    if A is None:
        A = skew_table(m)
    ns = m.n_sites
    pos = np.asarray(pos)
    o = inst.offsets()
    out = np.zeros(inst.n_params)
    # f: with the projection terms c_p = w_p Pf(X(q_p(x))),
    # d ln psi / d f_k = sum_p c_p (d ln Pf_p / d f_k) / sum_p c_p, and
    # d ln Pf(X) / dX_ab (a up, b down; X_ba = -X_ab moves with it) = -(X^-1)_ab
    # on the entries whose mapped sites (i, j) carry slot k
    terms = []
    if m.proj_q is None:
        terms.append((1.0, pos))
    else:
        for p in range(len(m.proj_q)):
            terms.append((float(m.proj_w[p]), mapped(m, pos, p)))
    logs = [pfaffian_log(A[np.ix_(y, y)]) for _, y in terms]
    lmax = max(l for s, l in logs if s != 0.0)
    cs = [w * s * math.exp(l - lmax) if s != 0.0 else 0.0 for (w, _), (s, l) in zip(terms, logs)]
    ctot = sum(cs)
    for (w, y), c in zip(terms, cs):
        if c == 0.0:
            continue
        Y = np.linalg.inv(A[np.ix_(y, y)])
        for a in range(m.n_up):
            i = int(y[a])
            for b in range(m.n_up, m.n_elec):
                j = int(y[b]) - ns
                k = int(inst.f_idx[i, j])
                if k >= 0:
                    out[o["f"] + k] += -Y[a, b] * c / ctot
    nv = occupations(m, pos)
    nup, ndn = nv[:ns], nv[ns:]
    for i in range(ns):
        k = int(inst.g_idx[i])
        if k >= 0:
            out[o["g"] + k] += nup[i] * ndn[i]
    mm = nup + ndn - 1.0
    for i in range(ns):
        for j in range(i + 1, ns):
            k = int(inst.v_idx[i, j])
            if k >= 0:
                out[o["v"] + k] += mm[i] * mm[j]
    if m.n_hidden:
        sigma = 2.0 * nv - 1.0
        th = np.tanh(m.b + m.W @ sigma)
        out[o["a"]:o["b"]] = sigma
        out[o["b"]:o["W"]] = th
        out[o["W"]:o["end"]] = np.outer(th, sigma).ravel()
    return out
