"""First-step power-Lanczos on the GPU (section 3.4) against the oracle.

F(x, H) and F(x, H^2) of every walker of a ragged context (1-D rings and
square clusters, N_e 6..30) against the oracle's two applications of H with
every end point recomputed from scratch; the moments, alpha_1 and E_1 against
the oracle's formulas on the same local values.
"""
import numpy as np
import pytest

from mvmc_inputs import workload
from oracle import lanczos, measure
from oracle import wavefunction as wf

from gpu_common import good_configs, log, square_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x1A4C205


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1711_11418_amd import binding
    binding.load()


def _instances():
    insts = [workload(n)["instances"][0] for n in ("ring6", "sq4_sub2", "ring8_u4")]
    insts.append(square_case(6, 15, 2, full_f=False))
    for i, w in zip(insts, (5, 4, 3, 2)):
        i.n_walkers = w
    return insts


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-10), ("mixed", 2e-4)])
def test_local_h2_matches_oracle(precision, rtol):
    """Double: to rounding (1e-10 relative, floor 1e-6 of the largest |F|).
    Mixed: M^-1 held in single precision after a double refresh, so the
    local values carry its rounding (about 1e-6 relative times the
    condition of M): 2e-4 on configurations of condition below 1e4."""
    from paper_1711_11418_amd import MVMC
    insts = _instances()
    params = np.concatenate([i.params0 for i in insts])
    pos0 = [good_configs(i, i.params0, i.n_walkers, 61, cond_max=1e4) for i in insts]
    log(f"[lanczos] {precision}: " + ", ".join(f"Ne={i.n_elec}xW={i.n_walkers}" for i in insts))
    ctx = MVMC(insts, params, precision=precision, seed=SEED, build_s=False, solver="cg")
    ctx.set_state(np.concatenate([p.ravel() for p in pos0]),
                  np.zeros(sum(i.n_walkers for i in insts), dtype=np.int64))
    ctx.measure_h2(0)
    f1 = ctx.f1.cpu().numpy()
    f2 = ctx.f2.cpu().numpy()
    for k, inst in enumerate(insts):
        lay = ctx.layouts[k]
        m = wf.expand(inst, inst.params0)
        A = wf.skew_table(m)
        worst = 0.0
        for w in range(inst.n_walkers):
            e1 = measure.local_energy(m, pos0[k][w], A)
            e2 = lanczos.local_h2(m, pos0[k][w], A)
            g1, g2 = f1[lay.eloc_off + w], f2[lay.eloc_off + w]
            d1 = abs(g1 - e1) / max(abs(e1), 1e-6)
            d2 = abs(g2 - e2) / max(abs(e2), 1e-6)
            worst = max(worst, d1, d2)
            assert d1 <= rtol and d2 <= rtol, (k, w, g1, e1, g2, e2)
        log(f"  instance {k} (Ne={inst.n_elec}): worst relative error {worst:.2e}")
    ctx.close()


def test_moments_alpha_and_energy():
    """Reduction and stationarity quadratic on the device against the
    oracle's formulas applied to the same sampled local values."""
    from paper_1711_11418_amd import MVMC
    insts = _instances()
    for i in insts:
        i.n_walkers = 16
    params = np.concatenate([i.params0 for i in insts])
    slots = 3
    ctx = MVMC(insts, params, seed=SEED, n_slots=slots, build_s=False, solver="cg",
               refresh_every=16)
    ctx.sample(4)
    for s in range(slots):
        ctx.sample(1)
        ctx.measure_h2(s)
    out = ctx.lanczos_first_step(slots)
    f1 = ctx.f1.cpu().numpy()
    f2 = ctx.f2.cpu().numpy()
    for k, inst in enumerate(insts):
        lay = ctx.layouts[k]
        sl = slice(lay.eloc_off, lay.eloc_off + slots * inst.n_walkers)
        h = lanczos.moments(f1[sl], f2[sl])
        alpha, e1 = lanczos.optimal_alpha(h)
        log(f"  instance {k}: h1 {h['h1']:.6f} alpha_1 {alpha:.6f} E_1 {e1:.6f} "
            f"(gpu {out[k, 4]:.6f}, {out[k, 5]:.6f})")
        for j, key in enumerate(("h1", "h11", "h20", "h12")):
            assert out[k, j] == pytest.approx(h[key], rel=1e-12, abs=1e-12)
        assert out[k, 4] == pytest.approx(alpha, rel=1e-9, abs=1e-12)
        assert out[k, 5] == pytest.approx(e1, rel=1e-12)
        assert out[k, 5] <= out[k, 0] + 1e-12 or out[k, 6] == 0
    ctx.close()


def test_rbm_and_oversized_instances_are_refused():
    from paper_1711_11418_amd import MVMC
    from paper_1711_11418_amd.binding import MVMCError
    inst = workload("ring6_rbm")["instances"][0]
    ctx = MVMC([inst], inst.params0, seed=SEED, build_s=False, solver="cg")
    with pytest.raises(MVMCError) as e:
        ctx.measure_h2(0)
    assert e.value.status == 1 and "RBM" in str(e.value)
    ctx.close()
    big = square_case(12, 66, 1, full_f=False)
    ctx = MVMC([big], big.params0, seed=SEED, build_s=False, solver="cg")
    with pytest.raises(MVMCError) as e:
        ctx.measure_h2(0)
    assert e.value.status == 2
    ctx.close()
