"""Pins for the first-step power-Lanczos oracle (section 3.4).

Exhaustive sums with the exact weights rho(x) must give the moments of the
exact-diagonalisation matrix: h1 = <H>, h11 = h20 = <H^2>, h12 = <H^3>
(completeness of the configuration basis), E_1(alpha) must be the Rayleigh
quotient of (1 + alpha H) psi, and the chosen alpha_1 the minimum of the
Rayleigh-Ritz problem in span{psi, H psi}.  An exact eigenstate has
F(x, H^2) = E0^2 on every configuration.  A dropped diagonal term, a wrong
hop sign or a missing path changes one of these.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from mvmc_inputs import workload
from mvmc_inputs.instance import f_map_full, make_instance, ring8_orbitals, v_map_nn
from mvmc_inputs.lattice import chain
from oracle import ed, enumerate as en, lanczos, measure
from oracle import wavefunction as wf


def _exact(name):
    inst = workload(name)["instances"][0]
    m = wf.expand(inst, inst.params0)
    confs = en.configurations(m)
    psi = en.amplitudes(m, confs)
    H = ed.hamiltonian(m.n_sites, m.n_up, m.n_dn, m.bonds, m.bond_t, m.U).toarray()
    A = wf.skew_table(m)
    keep = [k for k in range(len(confs)) if abs(psi[k]) > 1e-12 * np.max(np.abs(psi))]
    f1 = np.array([measure.local_energy(m, confs[k], A) for k in keep])
    f2 = np.array([lanczos.local_h2(m, confs[k], A) for k in keep])
    w = psi[keep] ** 2
    return m, psi, H, lanczos.moments(f1, f2, w), len(keep) == len(confs)


def _ed_moments(psi, H):
    n = psi @ psi
    hp = H @ psi
    return {"H": psi @ hp / n, "H2": hp @ hp / n, "H3": hp @ (H @ hp) / n}


@pytest.mark.parametrize("name", ["ring4", "ring6"])
def test_moments_equal_exact_diagonalisation(name):
    m, psi, H, h, all_nonzero = _exact(name)
    assert all_nonzero   # every configuration carries weight, so h11 = <H^2> exactly
    ref = _ed_moments(psi, H)
    assert h["h1"] == pytest.approx(ref["H"], rel=1e-11)
    assert h["h20"] == pytest.approx(ref["H2"], rel=1e-11)
    assert h["h11"] == pytest.approx(ref["H2"], rel=1e-11)
    assert h["h12"] == pytest.approx(ref["H3"], rel=1e-11)


@pytest.mark.parametrize("name", ["ring4", "ring6"])
def test_first_step_energy_is_rayleigh_quotient(name):
    m, psi, H, h, _ = _exact(name)
    for alpha in (-0.3, -0.07, 0.0, 0.05, 0.4):
        p1 = psi + alpha * (H @ psi)
        assert lanczos.energy(h, alpha) == pytest.approx(p1 @ (H @ p1) / (p1 @ p1), rel=1e-10)


@pytest.mark.parametrize("name", ["ring4", "ring6"])
def test_optimal_alpha_is_ritz_minimum(name):
    """min over alpha of E_1 is the lowest eigenvalue of the 2 x 2 pencil
    (K, B) on span{psi, H psi}; alpha_1 = c2 / c1 of its eigenvector."""
    m, psi, H, h, _ = _exact(name)
    ref = _ed_moments(psi, H)
    K = np.array([[ref["H"], ref["H2"]], [ref["H2"], ref["H3"]]])
    B = np.array([[1.0, ref["H"]], [ref["H"], ref["H2"]]])
    lam, vec = sla.eigh(K, B)
    alpha, e1 = lanczos.optimal_alpha(h)
    assert e1 == pytest.approx(lam[0], rel=1e-10)
    assert alpha == pytest.approx(vec[1, 0] / vec[0, 0], rel=1e-8)
    e_ed = ed.ground_energy(ed.hamiltonian(m.n_sites, m.n_up, m.n_dn, m.bonds, m.bond_t, m.U))
    assert e_ed - 1e-12 <= e1 <= h["h1"] + 1e-12
    # the minimum of a scan over alpha
    grid = np.linspace(alpha - 0.05, alpha + 0.05, 201)
    assert min(lanczos.energy(h, a) for a in grid) >= e1 - 1e-13


def test_eigenstate_has_constant_local_h2():
    """U = 0, g = v = 0 and f from the ring's eigen-orbitals: psi is an
    eigenstate with E0 = free-fermion energy, so F(x, H^2) = E0^2 and
    E_1(alpha) = E0 for every alpha."""
    lat = chain(8)
    phi = ring8_orbitals()
    inst = make_instance("z", lat, 4, 4, 0.0, f_map_full(lat), v_map_nn(lat),
                         g0=0.0, v_nn=0.0, f0=phi @ phi.T)
    m = wf.expand(inst, inst.params0)
    A = wf.skew_table(m)
    e0 = 2 * (-2 - 2 * 2 * math.cos(math.pi / 4))
    confs = en.configurations(m)
    psi = en.amplitudes(m, confs)
    idx = np.argsort(-np.abs(psi))[:8]
    f2 = [lanczos.local_h2(m, confs[k], A) for k in idx]
    assert np.max(np.abs(np.array(f2) - e0 * e0)) < 1e-8
    h = {"h1": e0, "h11": e0 * e0, "h20": e0 * e0, "h12": e0 ** 3}
    for a in (-0.2, 0.1, 1.0):
        assert lanczos.energy(h, a) == pytest.approx(e0, rel=1e-12)


def test_estimator_is_ratio_of_sample_sums():
    """With any sample weights (here far from rho, so h11 != h20): since
    psi_1(x)/psi(x) = 1 + alpha F(x, H) and <x|H|psi_1>/<x|psi> = F(x, H) +
    alpha F(x, H^2), E_1 is sum w (1 + a F1)(F1 + a F2) / sum w (1 + a F1)^2."""
    inst = workload("ring4")["instances"][0]
    m = wf.expand(inst, inst.params0)
    A = wf.skew_table(m)
    confs = en.configurations(m)
    f1 = np.array([measure.local_energy(m, c, A) for c in confs])
    f2 = np.array([lanczos.local_h2(m, c, A) for c in confs])
    w = np.random.default_rng(3).uniform(0.1, 1.0, len(confs))
    h = lanczos.moments(f1, f2, w)
    assert abs(h["h11"] - h["h20"]) > 1e-3 * abs(h["h20"])
    wn = w / w.sum()
    for a in (-0.4, -0.1, 0.2):
        ref = np.dot(wn, (1 + a * f1) * (f1 + a * f2)) / np.dot(wn, (1 + a * f1) ** 2)
        assert lanczos.energy(h, a) == pytest.approx(ref, rel=1e-12)
