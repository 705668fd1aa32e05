"""Pins for the oracle's wave function, local energy, derivatives, ED and SR.

All CPU-only.  Each check is against something other than the oracle's own
formula: exact diagonalisation, closed forms, finite differences of log psi,
or an identity that a dropped term, wrong sign or transposed index breaks.
"""
import itertools
import math

import numpy as np
import pytest

from mvmc_inputs import random_configs, workload
from mvmc_inputs.instance import (f_map_full, make_instance, ring8_orbitals,
                                  v_map_nn)
from mvmc_inputs.lattice import Lattice, chain
from oracle import ed, enumerate as en, measure, sr
from oracle import wavefunction as wf


def _inst(name):
    return workload(name)["instances"][0]


# ---------------------------------------------------------------- ED pins
def test_ed_two_site_closed_form():
    lat = Lattice("chain", 2, 1, np.array([[0, 0], [1, 0]]), np.array([[0, 1]], dtype=np.int32))
    for U in (0.0, 1.0, 4.0, 10.0):
        H = ed.hamiltonian(2, 1, 1, lat.bonds, [1.0], [U, U])
        assert ed.ground_energy(H) == pytest.approx((U - math.sqrt(U * U + 16)) / 2, abs=1e-12)


@pytest.mark.parametrize("L,n", [(6, 3), (8, 4), (5, 2)])
def test_ed_free_fermions(L, n):
    lat = chain(L)
    H = ed.hamiltonian(L, n, n, lat.bonds, np.ones(L), np.zeros(L))
    eps = np.sort(-2 * np.cos(2 * np.pi * np.arange(L) / L))
    assert ed.ground_energy(H) == pytest.approx(2 * eps[:n].sum(), abs=1e-10)


# --------------------------------------------- energy estimator and signs
@pytest.mark.parametrize("name", ["ring4", "ring6", "ring6_rbm"])
def test_exhaustive_energy_equals_ed_expectation(name):
    """sum rho(x) E_loc(x) = <psi|H|psi>/<psi|psi> with H the Jordan-Wigner
    matrix: pins label-preserving hop ratios, signs and the diagonal term."""
    inst = _inst(name)
    m = wf.expand(inst, inst.params0)
    E, p, eloc, confs = en.exact_energy(m)
    psi = en.amplitudes(m, confs)
    H = ed.hamiltonian(m.n_sites, m.n_up, m.n_dn, m.bonds, m.bond_t, m.U)
    assert E == pytest.approx(psi @ (H @ psi) / (psi @ psi), rel=1e-12)
    assert E >= ed.ground_energy(H) - 1e-12


def test_ring8_zero_variance_slater_case():
    """U = 0, g = v = 0 and f from the eigen-orbitals (Eq. fijSL) make psi an
    exact eigenstate: E_loc equals the free-fermion energy on every weighted x."""
    lat = chain(8)
    phi = ring8_orbitals()
    inst = make_instance("z", lat, 4, 4, 0.0, f_map_full(lat), v_map_nn(lat),
                         g0=0.0, v_nn=0.0, f0=phi @ phi.T)
    m = wf.expand(inst, inst.params0)
    E, p, eloc, confs = en.exact_energy(m)
    e0 = 2 * (-2 - 2 * 2 * math.cos(math.pi / 4))
    w = p > 1e-12
    assert np.max(np.abs(eloc[w] - e0)) < 1e-9
    assert E == pytest.approx(e0, abs=1e-10)


def test_ring8_variational_energy_above_ed():
    inst = workload("ring8_u4")["instances"][0]
    m = wf.expand(inst, inst.params0)
    E, p, eloc, confs = en.exact_energy(m)
    H = ed.hamiltonian(8, 4, 4, m.bonds, m.bond_t, m.U)
    e_ed = ed.ground_energy(H)
    assert e_ed == pytest.approx(-4.603526299989, abs=1e-9)
    assert E > e_ed


# ------------------------------------------------------ correlator forms
def test_gutzwiller_counts_doublons():
    inst = _inst("ring6")
    p = inst.params0.copy()
    o = inst.offsets()
    p[o["v"]:o["a"]] = 0.0
    p[o["g"]] = 0.7
    m = wf.expand(inst, p)
    for pos in random_configs(inst, 20, 5):
        ups = {int(x) for x in pos[:3]}
        dns = {int(x) - 6 for x in pos[3:]}
        assert wf.log_correlators(m, pos) == pytest.approx(0.7 * len(ups & dns), abs=1e-14)


def test_uniform_jastrow_closed_form():
    """v_ij = c for all i != j: 1/2 sum_{i!=j} c m_i m_j = c/2 ((sum m)^2 - sum m^2)."""
    inst = _inst("ring6")
    m = wf.expand(inst, inst.params0)
    c = 0.3
    m.V = c * (np.ones((6, 6)) - np.eye(6))
    m.g = np.zeros(6)
    for pos in random_configs(inst, 20, 6):
        n = np.zeros(6)
        for I in pos:
            n[int(I) % 6] += 1
        mm = n - 1
        assert wf.log_correlators(m, pos) == pytest.approx(c / 2 * (mm.sum() ** 2 - (mm ** 2).sum()),
                                                           abs=1e-13)


def test_rbm_zero_weights_is_constant():
    inst = _inst("ring6_rbm")
    p = inst.params0.copy()
    o = inst.offsets()
    p[o["g"]:o["end"]] = 0.0
    m = wf.expand(inst, p)
    # with g = v = 0 and zero RBM weights the correlator is M log 2 everywhere
    for pos in random_configs(inst, 10, 2):
        assert wf.log_correlators(m, pos) == pytest.approx(12 * math.log(2.0), abs=1e-13)
    # one hidden unit: log(2 cosh(b + sum_v W_v sigma_v)) + sum_v a_v sigma_v
    rng = np.random.default_rng(0)
    m.a = rng.standard_normal(12); m.b = rng.standard_normal(1); m.W = rng.standard_normal((1, 12))
    for pos in random_configs(inst, 5, 3):
        sig = -np.ones(12); sig[np.asarray(pos)] = 1.0
        th = m.b[0] + m.W[0] @ sig
        assert wf.log_correlators(m, pos) == pytest.approx(m.a @ sig + math.log(2 * math.cosh(th)), abs=1e-12)


# ------------------------------------------------------------ derivatives
@pytest.mark.parametrize("name", ["ring6", "sq4_sub2", "ring6_rbm"])
def test_log_derivatives_finite_differences(name):
    inst = _inst(name)
    rng = np.random.default_rng(1)
    p0 = inst.params0 + 0.05 * rng.standard_normal(inst.n_params)
    m0 = wf.expand(inst, p0)
    A0 = wf.skew_table(m0)
    for pos in random_configs(inst, 3, 11):
        if wf.log_psi(m0, pos, A0)[0] == 0.0:
            continue
        O = measure.log_derivs(inst, m0, pos, A0)
        h = 1e-6
        ks = range(inst.n_params) if inst.n_params <= 80 else rng.choice(inst.n_params, 80, replace=False)
        for k in ks:
            pp = p0.copy(); pp[k] += h
            pm = p0.copy(); pm[k] -= h
            lp = wf.log_psi(wf.expand(inst, pp), pos)[1]
            lm = wf.log_psi(wf.expand(inst, pm), pos)[1]
            assert O[k] == pytest.approx((lp - lm) / (2 * h), abs=2e-6, rel=1e-6)


def test_pfaffian_derivative_formula():
    """Eq. DiffPf: d Pf(X)/d x = 1/2 Pf(X) Tr[X^-1 dX/dx]."""
    rng = np.random.default_rng(9)
    a = rng.standard_normal((6, 6)); X = a - a.T
    d = rng.standard_normal((6, 6)); D = d - d.T
    from oracle.pfaffian import pfaffian
    h = 1e-6
    fd = (pfaffian(X + h * D) - pfaffian(X - h * D)) / (2 * h)
    assert fd == pytest.approx(0.5 * pfaffian(X) * np.trace(np.linalg.inv(X) @ D), rel=1e-7)


# --------------------------------------------------------------- SR pins
def test_covariance_identity_and_force():
    rng = np.random.default_rng(2)
    O = rng.standard_normal((500, 7)) + 3.0
    E = rng.standard_normal(500) - 2.0 + 0.3 * O[:, 1]
    st = sr.sr_stats(O, E)
    assert np.allclose(st["S"], np.cov(O.T, bias=True), atol=1e-12)
    g_ref = np.array([np.mean(O[:, k] * E) - np.mean(O[:, k]) * np.mean(E) for k in range(7)])
    assert np.allclose(st["g"], g_ref, atol=1e-12)


def test_cg_equals_cholesky():
    rng = np.random.default_rng(3)
    O = rng.standard_normal((300, 40))
    E = rng.standard_normal(300)
    a = sr.sr_update(O, E, 0.05, 1e-3, 1e-6, solver="chol")
    b = sr.sr_update(O, E, 0.05, 1e-3, 1e-6, solver="cg", cg_eps=1e-12)
    assert np.allclose(a["dalpha"], b["dalpha"], rtol=1e-8, atol=1e-12)


def test_regularisation_freezes_dead_parameters():
    rng = np.random.default_rng(4)
    O = rng.standard_normal((100, 5))
    O[:, 2] = 1.5               # constant column: S_22 = 0
    E = rng.standard_normal(100)
    st = sr.sr_update(O, E, 0.1, 1e-3, 1e-6)
    assert st["dalpha"][2] == 0.0 and not st["keep"][2]


def test_exact_sr_step_lowers_energy_at_first_order():
    """Exact S and g by enumeration: E(alpha + dalpha) - E(alpha) -> 2 g.dalpha
    = -2 dtau g^T S^-1 g < 0 as dtau -> 0 (dE/dalpha_k = 2 g_k)."""
    inst = _inst("ring6")
    m = wf.expand(inst, inst.params0)
    ex = en.exact_sr(inst, m)
    Sr, gr, keep = sr.regularize(ex["S"], ex["g"], 1e-4, 1e-8)
    x = sr.solve_cholesky(Sr, gr)
    errs = []
    for dtau in (1e-3, 1e-4):
        da = -dtau * x
        E1 = en.exact_energy(wf.expand(inst, inst.params0 + da))[0]
        pred = 2 * float(ex["g"] @ da)
        assert pred < 0 and E1 < ex["E"]
        errs.append(abs((E1 - ex["E"]) / pred - 1.0))
    assert errs[0] < 0.05 and errs[1] < errs[0] / 5


def test_force_is_half_energy_gradient():
    inst = _inst("ring4")
    m = wf.expand(inst, inst.params0)
    ex = en.exact_sr(inst, m)
    h = 1e-5
    for k in range(0, inst.n_params, 3):
        pp = inst.params0.copy(); pp[k] += h
        pm = inst.params0.copy(); pm[k] -= h
        dE = (en.exact_energy(wf.expand(inst, pp))[0] - en.exact_energy(wf.expand(inst, pm))[0]) / (2 * h)
        assert dE == pytest.approx(2 * ex["g"][k], abs=1e-7)


# ---------------------------------------------------------------- inputs
def test_parameter_counts():
    assert workload("ring8_u4")["instances"][0].n_params == 66
    assert workload("sq8_u4", n_walkers=4)["instances"][0].n_params == 271
    insts = workload("batch32_ragged", n_walkers=4)["instances"]
    assert len(insts) == 32
    assert all(i.n_elec % 2 == 0 and i.n_up == i.n_dn for i in insts)
