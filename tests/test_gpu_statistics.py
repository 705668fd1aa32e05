"""Statistical integration on the GPU: the 8-site ring (64 walkers x 1000
sweeps) must give an energy within 2 standard errors of the exact
variational energy from exhaustive enumeration by the oracle."""
import numpy as np
import pytest

from mvmc_inputs import workload
from oracle import enumerate as en
from oracle import wavefunction as wf

from gpu_common import log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_ring8_energy_within_two_sigma():
    from paper_1711_11418_amd import MVMC
    wl = workload("ring8_u4")
    inst = wl["instances"][0]
    E_exact = en.exact_energy(wf.expand(inst, inst.params0))[0]
    sweeps = 1000
    log(f"[stat] ring8 U=4: W={inst.n_walkers} sweeps={sweeps} seed={wl['sampler_seed']}")
    ctx = MVMC([inst], inst.params0, seed=wl["sampler_seed"], n_slots=sweeps, build_s=False,
               solver="cg")
    ctx.sample(wl["warmup"])
    for s in range(sweeps):
        ctx.sample_async(1)
        ctx.measure(s)
    E = ctx.eloc_of(0, sweeps).cpu().numpy().reshape(sweeps, inst.n_walkers)
    walker_means = E.mean(axis=0)
    mean = walker_means.mean()
    err = walker_means.std(ddof=1) / np.sqrt(inst.n_walkers)
    z = (mean - E_exact) / err
    log(f"  E_mc={mean:.6f} +- {err:.6f}  E_exact={E_exact:.6f}  z={z:+.2f}")
    assert abs(z) < 2.0
    ctx.close()


@pytest.mark.parametrize("precision,refresh", [("mixed", 32), ("fp64", 0)])
def test_sq4_energy_mixed_matches_exact(precision, refresh):
    """4x4 lattice (7 up + 7 down, 2x2-sublattice f): the single-precision
    sampler with a double-precision refresh every 32 proposals (and, as a
    control, the double path) must agree within 2 combined standard errors
    with an independent double-precision chain of the same wave function
    (another Philox key).  The double path itself is pinned to the oracle by
    the trajectory-replay tests."""
    from paper_1711_11418_amd import MVMC
    inst = workload("sq4_sub2")["instances"][0]
    inst.n_walkers = 256
    sweeps = 200
    log(f"[stat-{precision}] sq4 W=256 sweeps={sweeps} refresh={refresh}")
    ctx = MVMC([inst], inst.params0, precision=precision, refresh_every=refresh, seed=99,
               n_slots=sweeps, build_s=False, solver="cg")
    ctx.sample(50)
    for s in range(sweeps):
        ctx.sample_async(1)
        ctx.measure(s)
    E = ctx.eloc_of(0, sweeps).cpu().numpy().reshape(sweeps, inst.n_walkers)
    wm = E.mean(axis=0)
    mean, err = wm.mean(), wm.std(ddof=1) / np.sqrt(inst.n_walkers)
    ctx.close()
    # reference: the same wave function sampled by the double path with another seed
    ref = MVMC([inst], inst.params0, precision="fp64", seed=12345, n_slots=sweeps, build_s=False,
               solver="cg")
    ref.sample(50)
    for s in range(sweeps):
        ref.sample_async(1)
        ref.measure(s)
    E2 = ref.eloc_of(0, sweeps).cpu().numpy().reshape(sweeps, inst.n_walkers).mean(axis=0)
    ref.close()
    m2, e2 = E2.mean(), E2.std(ddof=1) / np.sqrt(inst.n_walkers)
    z = (mean - m2) / np.hypot(err, e2)
    log(f"  {precision}: E={mean:.5f}+-{err:.5f}  fp64 ref {m2:.5f}+-{e2:.5f}  z={z:+.2f}")
    assert abs(z) < 2.0
