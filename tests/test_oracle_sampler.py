"""Pins for the oracle's Metropolis sampler (CPU only).

The visited-configuration histogram must follow the exhaustive |psi|^2 / Z
(section 3.1.1, Eq. MC), and the chain must be a deterministic function of
the Philox key.
"""
import numpy as np
import pytest
from scipy import stats

from mvmc_inputs import random_configs, workload
from oracle import enumerate as en, sampler
from oracle import wavefunction as wf


def _key(pos, n_up):
    return tuple(sorted(int(x) for x in pos[:n_up])) + tuple(sorted(int(x) for x in pos[n_up:]))


@pytest.mark.parametrize("name,sweeps", [("ring4", 400), ("ring6", 300)])
def test_histogram_matches_exhaustive_distribution(name, sweeps):
    inst = workload(name)["instances"][0]
    m = wf.expand(inst, inst.params0)
    _, p, _, confs = en.exact_energy(m)
    index = {_key(c, m.n_up): k for k, c in enumerate(confs)}
    counts = np.zeros(len(confs))
    pos0 = random_configs(inst, 8, 3)
    A = wf.skew_table(m)
    for w in range(8):
        if wf.log_psi(m, pos0[w], A)[0] == 0.0:
            continue
        wk = sampler.make_walker(m, pos0[w], gid=w)
        for s in range(sweeps + 20):
            for _ in range(m.n_elec):
                sampler.step(m, wk, seed=99, A=A)
            if s >= 20:
                counts[index[_key(wk.pos, m.n_up)]] += 1
    n = counts.sum()
    keep = p * n >= 5
    exp = p[keep] * n
    chi2 = ((counts[keep] - exp) ** 2 / exp).sum()
    dof = keep.sum() - 1
    # successive sweeps are correlated; allow a factor 3 inflation of the variance
    assert chi2 / 3 < stats.chi2.ppf(1 - 1e-4, dof)
    assert counts[~keep].sum() <= 5 * (~keep).sum() + 0.01 * n


def test_chain_is_deterministic_and_replayable():
    inst = workload("ring6")["instances"][0]
    m = wf.expand(inst, inst.params0)
    pos0 = random_configs(inst, 1, 4)[0]
    a = sampler.make_walker(m, pos0, gid=5)
    b = sampler.make_walker(m, pos0, gid=5)
    sampler.run(m, a, 300, seed=7, record=True)
    sampler.run(m, b, 150, seed=7, record=True)
    sampler.run(m, b, 150, seed=7, record=True)
    assert a.trace == b.trace and np.array_equal(a.pos, b.pos)
    c = sampler.make_walker(m, pos0, gid=6)
    sampler.run(m, c, 300, seed=7, record=True)
    assert [t[1] for t in c.trace] != [t[1] for t in a.trace]


@pytest.mark.parametrize("name,sweeps,ex64", [("ring4", 400, 32), ("ring6", 300, 24)])
def test_histogram_with_exchange_updates(name, sweeps, ex64):
    """Hops mixed with exchange proposals (section 3.1.2, Fig. 5b) keep
    |psi|^2 / Z stationary: the symmetric pair choice gives detailed balance."""
    inst = workload(name)["instances"][0]
    m = wf.expand(inst, inst.params0)
    _, p, _, confs = en.exact_energy(m)
    index = {_key(c, m.n_up): k for k, c in enumerate(confs)}
    counts = np.zeros(len(confs))
    pos0 = random_configs(inst, 8, 5)
    A = wf.skew_table(m)
    n_ex = 0
    for w in range(8):
        if wf.log_psi(m, pos0[w], A)[0] == 0.0:
            continue
        wk = sampler.make_walker(m, pos0[w], gid=w)
        for s in range(sweeps + 20):
            for _ in range(m.n_elec):
                sampler.step(m, wk, seed=77, A=A, record=True, ex64=ex64)
            if s >= 20:
                counts[index[_key(wk.pos, m.n_up)]] += 1
        n_ex += sum(1 for t in wk.trace if t[5] >= 0 and t[2] >= 0 and t[4])
    assert n_ex > 0
    n = counts.sum()
    keep = p * n >= 5
    exp = p[keep] * n
    chi2 = ((counts[keep] - exp) ** 2 / exp).sum()
    dof = keep.sum() - 1
    assert chi2 / 3 < stats.chi2.ppf(1 - 1e-4, dof)


def test_exchange_moves_swap_spins_and_keep_charges():
    inst = workload("ring6")["instances"][0]
    m = wf.expand(inst, inst.params0)
    ns = m.n_sites
    pos0 = random_configs(inst, 1, 9)[0]
    wk = sampler.make_walker(m, pos0, gid=3)
    A = wf.skew_table(m)
    seen = 0
    for _ in range(400):
        before = wk.pos.copy()
        sampler.step(m, wk, seed=5, A=A, record=True, ex64=64)
        n, a, inew, R, acc, b = wk.trace[-1]
        assert b >= m.n_up and a < m.n_up
        if acc:
            seen += 1
            i, j = int(before[a]), int(before[b]) - ns
            assert inew == j and int(wk.pos[a]) == j and int(wk.pos[b]) == i + ns
            nb = wf.occupations(m, before)
            na = wf.occupations(m, wk.pos)
            assert np.array_equal(nb[:ns] + nb[ns:], na[:ns] + na[ns:])
        # the empty lists always hold exactly the empty sites of each spin
        occ = wf.occupations(m, wk.pos)
        assert sorted(wk.empty[0]) == [s for s in range(ns) if not occ[s]]
        assert sorted(wk.empty[1]) == [s for s in range(ns) if not occ[s + ns]]
    assert seen > 10
