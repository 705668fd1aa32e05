"""Pins for the oracle's quantum-number projection (section 3.2.2).

The projected amplitude sum_p w_p <x|T_p|phi> is pinned by what the
mathematics fixes independently of the oracle's formula: the exhaustive <H>
equals psi^T H psi / psi^T psi of the Jordan-Wigner matrix (a wrong fermion
sign of a mapped configuration breaks it); a translation eigenstate picks up
the character e^{iK.S} under a translation of the configuration (a wrong map
or weight breaks it); one identity term reproduces the unprojected
amplitude; and the f derivatives match finite differences of log psi.
"""
import math

import numpy as np
import pytest

from mvmc_inputs import random_configs, workload
from oracle import ed, enumerate as en, measure
from oracle import wavefunction as wf


def _inst(name):
    return workload(name)["instances"][0]


@pytest.mark.parametrize("name", ["ring4_proj", "ring4_projpi", "ring6_proj3"])
def test_projected_energy_equals_ed_expectation(name):
    inst = _inst(name)
    m = wf.expand(inst, inst.params0)
    E, p, eloc, confs = en.exact_energy(m)
    psi = en.amplitudes(m, confs)
    H = ed.hamiltonian(m.n_sites, m.n_up, m.n_dn, m.bonds, m.bond_t, m.U)
    assert E == pytest.approx(psi @ (H @ psi) / (psi @ psi), rel=1e-12)
    assert E >= ed.ground_energy(H) - 1e-12


@pytest.mark.parametrize("name,step,char", [("ring4_proj", 1, 1.0), ("ring4_projpi", 1, -1.0),
                                            ("ring6_proj3", 2, 1.0)])
def test_translation_character(name, step, char):
    """psi_P(T_S x) = e^{iK.S} psi_P(x) with T_S x the configuration moved by
    S sites, electron labels kept."""
    inst = _inst(name)
    m = wf.expand(inst, inst.params0)
    A = wf.skew_table(m)
    ns = m.n_sites
    for pos in random_configs(inst, 6, 5):
        sig = pos // ns
        moved = (pos - sig * ns + step) % ns + sig * ns
        s0, l0 = wf.log_psi(m, pos, A)
        s1, l1 = wf.log_psi(m, moved, A)
        assert l1 == pytest.approx(l0, abs=1e-12)
        assert s1 == char * s0


def test_identity_projection_is_the_plain_amplitude():
    inst = _inst("sq4_sub2")
    m = wf.expand(inst, inst.params0)
    A = wf.skew_table(m)
    inst.proj_q = np.arange(inst.n_sites, dtype=np.int32)[None, :]
    inst.proj_w = np.ones(1)
    mp = wf.expand(inst, inst.params0)
    for pos in random_configs(inst, 5, 9):
        assert wf.log_psi(mp, pos, A) == wf.log_psi(m, pos, A)
        assert np.array_equal(measure.log_derivs(inst, mp, pos, A),
                              measure.log_derivs(_inst("sq4_sub2"), m, pos, A))


@pytest.mark.parametrize("name", ["ring4_projpi", "sq4_sub2_proj4"])
def test_projected_f_derivatives_finite_differences(name):
    inst = _inst(name)
    p0 = inst.params0.copy()
    o = inst.offsets()
    h = 1e-6
    for pos in random_configs(inst, 3, 13):
        m = wf.expand(inst, p0)
        d = measure.log_derivs(inst, m, pos)
        for k in range(o["f"], o["g"]):
            pp, pm = p0.copy(), p0.copy()
            pp[k] += h
            pm[k] -= h
            lp = wf.log_psi(wf.expand(inst, pp), pos)[1]
            lm = wf.log_psi(wf.expand(inst, pm), pos)[1]
            fd = (lp - lm) / (2 * h)
            assert d[k] == pytest.approx(fd, rel=1e-5, abs=1e-7), (k, d[k], fd)
