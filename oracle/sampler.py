"""Metropolis sampling of |psi(x)|^2 with a full recomputation per proposal.

Section 3.1.1: configurations are drawn with weight rho(x) ~ |<x|psi>|^2 by a
Markov chain.  Section 3.1.2 / Fig. 5a: the hopping update moves one electron
to another site.  The proposal used here (the same on the GPU):

  draw (r0, r1, r2, r3) = Philox4x32-10(counter = (n, walker id, tag 0));
  electron a = (r0 * N_e) >> 32, spin sigma of a;
  target = empty_sigma[(r1 * (Ns - N_sigma)) >> 32], the k-th entry of the
  walker's list of sites empty for spin sigma;
  u = 53-bit uniform from (r2, r3);
  accept iff u < R^2 with R = psi(x')/psi(x) (real psi; Metropolis rule
  min(1, R^2)).

The proposal is symmetric because Ns - N_sigma is the same before and after a
move.  On acceptance the vacated site takes the target's slot in the empty
list (empty_sigma[k] = old site), electron a keeps its label (row of X).
Initial empty lists hold the empty sites in ascending order.

Exchange update (section 3.1.2, Fig. 5b: two electrons of opposite spin
trade sites), mixed in with probability ex64/64 per proposal:

  the proposal is an exchange iff (r3 & 63) < ex64 (the six low bits of r3,
  which the 53-bit uniform does not use);
  up electron a = (r0 * N_up) >> 32, down electron b = N_up + (r1 * N_dn) >> 32,
  at sites i and j;
  the move (a to j, b to i) is possible iff i != j, no up electron sits on j
  and no down electron on i (both sites singly occupied with opposite
  spins); otherwise the proposal is rejected without a move;
  accept iff u < R^2 as for a hop.

Picking the same pair undoes the move, so the proposal is symmetric.  On
acceptance j takes i's slot in the up list of empty sites and i takes j's
slot in the down list.  Charges per site are unchanged, so the Gutzwiller
and Jastrow factors are too; the Pfaffian and RBM factors change.

Here R comes from two independent Parlett-Reid Pfaffians (no inverse, no
fast update), so it is the plain definition of the ratio.  Trace entries are
(n, a, I', R, accepted, b) with b = -1 for a hop and I' = -1 when no move
was possible.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .philox import proposal_draw, scaled_index, uniform53
from .wavefunction import Model, ratio, skew_table


@dataclass
class Walker:
    pos: np.ndarray            # [N_e] spin-orbital of each electron
    empty: list                # [2] lists of empty sites per spin
    gid: int                   # global walker id (Philox counter word 2)
    n: int = 0                 # proposals made so far (Philox counter words 0-1)
    trace: list = field(default_factory=list)


def make_walker(m: Model, pos: np.ndarray, gid: int, n: int = 0) -> Walker:
    ns = m.n_sites
    pos = np.array(pos, dtype=np.int64)
    occ = np.zeros(2 * ns, dtype=bool)
    occ[pos] = True
    empty = [[s for s in range(ns) if not occ[s]],
             [s for s in range(ns) if not occ[s + ns]]]
    return Walker(pos, empty, gid, n)


def _exchange(m: Model, w: Walker, A: np.ndarray, r: tuple, n_here: int, record: bool) -> bool:
    ns = m.n_sites
    r0, r1, r2, r3 = r
    a = scaled_index(r0, m.n_up)
    b = m.n_up + scaled_index(r1, m.n_dn)
    i = int(w.pos[a])
    j = int(w.pos[b]) - ns
    up = set(int(x) for x in w.pos[:m.n_up])
    dn = set(int(x) - ns for x in w.pos[m.n_up:])
    if i == j or j in up or i in dn:
        if record:
            w.trace.append((n_here, a, -1, 0.0, False, b))
        return False
    new_pos = w.pos.copy()
    new_pos[a] = j
    new_pos[b] = i + ns
    R = ratio(m, new_pos, w.pos, A)
    acc = uniform53(r2, r3) < R * R
    if record:
        w.trace.append((n_here, a, j, R, bool(acc), b))
    if acc:
        w.empty[0][w.empty[0].index(j)] = i
        w.empty[1][w.empty[1].index(i)] = j
        w.pos = new_pos
    return bool(acc)


def step(m: Model, w: Walker, seed: int, A: np.ndarray | None = None,
         record: bool = False, ex64: int = 0) -> bool:
    """One proposal (an exchange with probability ex64/64, else a hop);
    returns True when accepted."""
    if A is None:
        A = skew_table(m)
    ns = m.n_sites
    ne = m.n_elec
    r0, r1, r2, r3 = proposal_draw(seed, w.gid, w.n)
    n_here = w.n
    w.n += 1
    if ex64 and (r3 & 63) < ex64:
        return _exchange(m, w, A, (r0, r1, r2, r3), n_here, record)
    a = scaled_index(r0, ne)
    sigma = 0 if a < m.n_up else 1
    n_sigma = m.n_up if sigma == 0 else m.n_dn
    n_empty = ns - n_sigma
    if n_empty == 0:
        if record:
            w.trace.append((n_here, a, -1, 0.0, False, -1))
        return False
    k = scaled_index(r1, n_empty)
    site_new = w.empty[sigma][k]
    old = int(w.pos[a])
    new_pos = w.pos.copy()
    new_pos[a] = site_new + ns * sigma
    R = ratio(m, new_pos, w.pos, A)
    u = uniform53(r2, r3)
    acc = u < R * R
    if record:
        w.trace.append((n_here, a, int(new_pos[a]), R, bool(acc), -1))
    if acc:
        w.empty[sigma][k] = old - ns * sigma
        w.pos = new_pos
    return bool(acc)


def run(m: Model, w: Walker, n_prop: int, seed: int, record: bool = False,
        ex64: int = 0) -> int:
    A = skew_table(m)
    acc = 0
    for _ in range(n_prop):
        acc += step(m, w, seed, A, record, ex64)
    return acc
