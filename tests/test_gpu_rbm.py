"""The learned correlator: a restricted Boltzmann machine on the
spin-resolved occupations multiplies the Pfaffian-Jastrow-Gutzwiller wave
function and is trained on the GPU by stochastic reconfiguration (section
3.3.1) on the samples the GPU sampler draws, with the library's own
incremental-update, O_k and SR kernels.  What it gains is judged by the exact
variational energy of the trained parameters, evaluated by the oracle's
exhaustive enumeration (6-site ring, U = 8, 400 configurations), against the
same training without the RBM and against exact diagonalisation."""
import numpy as np
import pytest

from mvmc_inputs import workload
from oracle import ed
from oracle import enumerate as en
from oracle import wavefunction as wf

from gpu_common import log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _train(inst, wl, solver):
    from paper_1711_11418_amd import MVMC
    sweeps = wl["sweeps"]
    ctx = MVMC([inst], inst.params0, seed=wl["sampler_seed"], n_slots=sweeps, solver=solver,
               build_s=solver == "chol")
    ctx.sample(wl["warmup"])
    hist = []
    for it in range(wl["sr_iters"]):
        for s in range(sweeps):
            ctx.sample_async(1)
            ctx.measure(s)
        E, _, _ = ctx.build_sr(sweeps)
        hist.append(float(E[0]))
        if it % 20 == 0:
            log(f"  {inst.name} SR step {it}: E_mc = {hist[-1]:.5f}")
        ctx.sr_update(dtau=wl["dtau"], eps_rel=wl["eps_rel"], eps_abs=wl["eps_abs"],
                      solver=solver, cg_tol=1e-8, cg_maxit=2000)
        ctx.sample(5)          # re-equilibrate after the parameter change
    p = ctx.params.cpu().numpy().copy()
    ctx.close()
    return p, hist


def test_rbm_training_gain():
    wl = workload("ring6_u8_gain")
    pj, rbm = wl["instances"]
    lat = pj.lattice
    H = ed.hamiltonian(lat.n_sites, pj.n_up, pj.n_dn, lat.bonds, np.full(len(lat.bonds), pj.t),
                       pj.U)
    E_ed = ed.ground_energy(H)
    E0 = en.exact_energy(wf.expand(pj, pj.params0))[0]
    log(f"[rbm] ring6 U=8: E_ED={E_ed:.6f}, exact E_var at the start {E0:.6f}; "
        f"W={pj.n_walkers} x {wl['sweeps']} sweeps x {wl['sr_iters']} SR steps")
    p_pj, h_pj = _train(pj, wl, "chol")
    p_rbm, h_rbm = _train(rbm, wl, "cg")
    E_pj = en.exact_energy(wf.expand(pj, p_pj))[0]
    E_rbm = en.exact_energy(wf.expand(rbm, p_rbm))[0]
    rel = lambda e: (e - E_ed) / abs(E_ed)
    log(f"  trained Pfaffian-Jastrow:       exact E_var {E_pj:.6f} (rel. error {rel(E_pj):.3e}); "
        f"last MC estimates {np.round(h_pj[-3:], 5)}")
    log(f"  trained Pfaffian-Jastrow x RBM: exact E_var {E_rbm:.6f} (rel. error {rel(E_rbm):.3e}); "
        f"last MC estimates {np.round(h_rbm[-3:], 5)}")
    log(f"  gain {E_pj - E_rbm:.6f} = {(E_pj - E_rbm) / abs(E_ed):.2%} of |E_ED|")
    # both are variational states; the baseline was trained to its plateau
    assert E_pj > E_ed and E_rbm > E_ed - 1e-10
    assert E_pj < E0 and E_pj < -1.94
    # the RBM factor removes most of the remaining error (at least 1% of |E|)
    assert E_rbm < E_pj - 0.01 * abs(E_ed)
    # the Monte Carlo estimates the training saw track the exact energies
    assert abs(np.mean(h_pj[-5:]) - E_pj) < 0.02
    assert abs(np.mean(h_rbm[-5:]) - E_rbm) < 0.05
