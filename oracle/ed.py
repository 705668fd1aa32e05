"""Exact diagonalisation of the Hubbard model in the canonical basis.

H = -sum_{<ij>, s} t_ij (c+_is c_js + c+_js c_is) + sum_i U_i n_iup n_idn
(section 2.3: Eq. GHam with real nearest-neighbour t and the on-site H_U).

Basis state |x> = c+_{I_1} ... c+_{I_N} |0> with I_1 < ... < I_N and
I = i + Ns*sigma.  A hop c+_J c_I (same spin) gives the Jordan-Wigner sign
(-1)^(number of occupied spin-orbitals strictly between I and J).

Pinned by the U = 0 free-fermion energy (sum of the lowest single-particle
levels per spin) and the two-site closed form (U - sqrt(U^2 + 16 t^2)) / 2.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def basis(ns: int, n_up: int, n_dn: int) -> tuple[list[int], list[int]]:
    ups = [sum(1 << s for s in c) for c in itertools.combinations(range(ns), n_up)]
    dns = [sum(1 << s for s in c) for c in itertools.combinations(range(ns), n_dn)]
    return ups, dns


def _hops(masks: list[int], bonds, bond_t):
    """Single-spin hop matrix elements: list of (new, old, amplitude)."""
    index = {m: k for k, m in enumerate(masks)}
    out = []
    for k, m in enumerate(masks):
        for (i, j), t in zip(bonds, bond_t):
            i, j = int(i), int(j)
            for src, dst in ((j, i), (i, j)):
                if (m >> src) & 1 and not (m >> dst) & 1:
                    lo, hi = min(src, dst), max(src, dst)
                    between = bin(m & (((1 << hi) - 1) ^ ((1 << (lo + 1)) - 1))).count("1")
                    sign = -1.0 if between % 2 else 1.0
                    out.append((index[m ^ (1 << src) ^ (1 << dst)], k, -float(t) * sign))
    return out


def hamiltonian(ns: int, n_up: int, n_dn: int, bonds, bond_t, U) -> sp.csr_matrix:
    ups, dns = basis(ns, n_up, n_dn)
    nu, nd = len(ups), len(dns)
    rows, cols, vals = [], [], []
    for new, old, amp in _hops(ups, bonds, bond_t):
        for d in range(nd):
            rows.append(new * nd + d); cols.append(old * nd + d); vals.append(amp)
    for new, old, amp in _hops(dns, bonds, bond_t):
        for u in range(nu):
            rows.append(u * nd + new); cols.append(u * nd + old); vals.append(amp)
    U = np.asarray(U, dtype=np.float64)
    for u, mu in enumerate(ups):
        for d, md in enumerate(dns):
            both = mu & md
            e = sum(U[s] for s in range(ns) if (both >> s) & 1)
            if e:
                rows.append(u * nd + d); cols.append(u * nd + d); vals.append(e)
    dim = nu * nd
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim))


def ground_energy(H: sp.csr_matrix) -> float:
    if H.shape[0] <= 400:
        return float(np.linalg.eigvalsh(H.toarray())[0])
    v0 = np.ones(H.shape[0]) / np.sqrt(H.shape[0])
    w = spla.eigsh(H, k=1, which="SA", tol=1e-13, v0=v0)[0]
    return float(w[0])
