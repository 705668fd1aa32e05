"""log <x|psi> from scratch for psi = P_G P_J [RBM] |phi_AP-Pf>.

Definitions followed (paper arXiv:1711.11418):

* Configuration |x> (section 3.1.1): electron a sits at spin-orbital
  I = i + Ns*sigma (section 3.2.1); electrons 0..n_up-1 are up, the rest down.
* Anti-parallel Pfaffian (Eq. AP-Pf): F_{(i,up),(j,dn)} = f_ij and every other
  F entry is zero.  X_ab = F_{R_a R_b} - F_{R_b R_a} is the N_e x N_e
  skew-symmetric matrix of the electrons' spin-orbitals, and
  <x|phi_Pf> = (N_e/2)! Pf(X); the constant factorial is dropped.
* Gutzwiller (section 3.2.3): log P_G = sum_i g_i n_iup n_idn.
* Jastrow (section 3.2.3): log P_J = 1/2 sum_{i != j} v_ij (n_i - 1)(n_j - 1).
* RBM factor (not in the paper): visible sigma_v = 2 n_v - 1 over the 2 Ns
  spin-orbitals, theta = b + W sigma,
  log psi_RBM = sum_v a_v sigma_v + sum_h log(2 cosh theta_h).
* Quantum-number projection (section 3.2.2, Eqs. momP and pointP): the
  projector sum_p w_p T_p acts on the pair-product part,
  <x|psi> = P_G P_J [RBM] sum_p w_p <x|T_p|phi_Pf>.  With T_p a site
  permutation, <x|T_p|phi_Pf> is the Pfaffian of the configuration whose
  electrons sit on the mapped sites (electron labels, hence the fermion
  sign, kept): Pf(X(q_p(x))), X(y)_ab = A[R_a(y)][R_b(y)] with the site part
  of every spin-orbital sent through the table q_p.  The normalisation
  1/N_g is dropped.

Pinned by the Pfaffian tests, by the exhaustive <H> against exact
diagonalisation and by the zero-variance Slater case (tests/).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .pfaffian import pfaffian_log


@dataclass
class Model:
    """Plain arrays describing one lattice instance and its parameters."""
    n_sites: int
    n_up: int
    n_dn: int
    bonds: np.ndarray      # [nb, 2]
    bond_t: np.ndarray     # [nb]
    U: np.ndarray          # [Ns]
    f: np.ndarray          # [Ns, Ns]
    g: np.ndarray          # [Ns]
    V: np.ndarray          # [Ns, Ns] symmetric, zero diagonal
    a: np.ndarray          # [2Ns]   (empty if no RBM)
    b: np.ndarray          # [M]
    W: np.ndarray          # [M, 2Ns]
    proj_q: np.ndarray | None = None   # [N_P, Ns] site maps (None: no projection)
    proj_w: np.ndarray | None = None   # [N_P] weights

    @property
    def n_elec(self) -> int:
        return self.n_up + self.n_dn

    @property
    def n_hidden(self) -> int:
        return len(self.b)


def expand(inst, params: np.ndarray) -> Model:
    """Parameter vector -> f_ij, g_i, v_ij (and RBM a, b, W) via the index maps."""
    p = np.asarray(params, dtype=np.float64)
    ns = inst.n_sites
    o = inst.offsets()
    pf = p[o["f"]:o["g"]]
    pg = p[o["g"]:o["v"]]
    pv = p[o["v"]:o["a"]]
    f = np.where(inst.f_idx >= 0, pf[np.maximum(inst.f_idx, 0)], 0.0)
    g = np.where(inst.g_idx >= 0, pg[np.maximum(inst.g_idx, 0)], 0.0)
    V = np.where(inst.v_idx >= 0, pv[np.maximum(inst.v_idx, 0)], 0.0)
    np.fill_diagonal(V, 0.0)
    M = inst.n_hidden
    if M:
        a = p[o["a"]:o["b"]].copy()
        b = p[o["b"]:o["W"]].copy()
        W = p[o["W"]:o["end"]].reshape(M, 2 * ns).copy()
    else:
        a = np.zeros(0)
        b = np.zeros(0)
        W = np.zeros((0, 2 * ns))
    pq = getattr(inst, "proj_q", None)
    pw = getattr(inst, "proj_w", None)
    return Model(ns, inst.n_up, inst.n_dn, np.asarray(inst.bonds), inst.bond_t,
                 np.asarray(inst.U, dtype=np.float64), f, g, V, a, b, W,
                 None if pq is None else np.asarray(pq, dtype=np.int64),
                 None if pw is None else np.asarray(pw, dtype=np.float64))


def skew_table(m: Model) -> np.ndarray:
    """A = F - F^T over all 2Ns spin-orbitals, so that X_ab = A[R_a, R_b]."""
    ns = m.n_sites
    F = np.zeros((2 * ns, 2 * ns))
    F[:ns, ns:] = m.f
    return F - F.T


def occupations(m: Model, pos: np.ndarray) -> np.ndarray:
    """n_v for the 2Ns spin-orbitals (v = i + Ns*sigma)."""
    n = np.zeros(2 * m.n_sites)
    n[np.asarray(pos)] = 1.0
    return n


def log_cosh2(x: np.ndarray) -> np.ndarray:
    """log(2 cosh x) = |x| + log1p(exp(-2|x|)), stable for large |x|."""
    ax = np.abs(x)
    return ax + np.log1p(np.exp(-2.0 * ax))


def log_correlators(m: Model, pos: np.ndarray) -> float:
    nv = occupations(m, pos)
    ns = m.n_sites
    nup, ndn = nv[:ns], nv[ns:]
    out = float(np.dot(m.g, nup * ndn))
    mm = nup + ndn - 1.0
    out += 0.5 * float(mm @ m.V @ mm)
    if m.n_hidden:
        sigma = 2.0 * nv - 1.0
        theta = m.b + m.W @ sigma
        out += float(np.dot(m.a, sigma)) + float(np.sum(log_cosh2(theta)))
    return out


def mapped(m: Model, pos: np.ndarray, p: int) -> np.ndarray:
    """Spin-orbitals of the configuration q_p(x): site part through q_p,
    spin kept, electron order kept."""
    ns = m.n_sites
    pos = np.asarray(pos)
    sig = pos // ns
    return m.proj_q[p][pos - sig * ns] + sig * ns


def pair_terms(m: Model, pos: np.ndarray, A: np.ndarray) -> list[tuple[float, float, float]]:
    """(w_p, sign, log|Pf|) of every projection term (one identity term when
    there is no projection)."""
    pos = np.asarray(pos)
    if m.proj_q is None:
        s, l = pfaffian_log(A[np.ix_(pos, pos)])
        return [(1.0, s, l)]
    out = []
    for p in range(len(m.proj_q)):
        y = mapped(m, pos, p)
        s, l = pfaffian_log(A[np.ix_(y, y)])
        out.append((float(m.proj_w[p]), s, l))
    return out


def log_psi(m: Model, pos: np.ndarray, A: np.ndarray | None = None) -> tuple[float, float]:
    """(sign, log|psi(x)|) with electron a at spin-orbital pos[a]."""
    if A is None:
        A = skew_table(m)
    pos = np.asarray(pos)
    terms = [(w, s, l) for w, s, l in pair_terms(m, pos, A) if w != 0.0 and s != 0.0]
    if not terms:
        return 0.0, -math.inf
    lmax = max(l for _, _, l in terms)
    tot = sum(w * s * math.exp(l - lmax) for w, s, l in terms)
    if tot == 0.0:
        return 0.0, -math.inf
    s = 1.0 if tot > 0.0 else -1.0
    return s, lmax + math.log(abs(tot)) + log_correlators(m, pos)


def ratio(m: Model, pos_new: np.ndarray, pos_old: np.ndarray, A: np.ndarray | None = None) -> float:
    """psi(x')/psi(x), both evaluated from scratch."""
    if A is None:
        A = skew_table(m)
    s1, l1 = log_psi(m, pos_new, A)
    s0, l0 = log_psi(m, pos_old, A)
    if s0 == 0.0:
        raise ZeroDivisionError("psi(x) = 0")
    if s1 == 0.0:
        return 0.0
    return s1 * s0 * math.exp(l1 - l0)
