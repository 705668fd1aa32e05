"""Ragged batches: several lattice instances of different size in one
context, each with its own statistics and SR step (section 3.3.1,
Eq. SR_equation_system; section 3.3.2 estimators and Algorithm 1), checked
instance by instance against the oracle at the single-instance tolerances;
and a single-precision ragged replay against the rounding bound.
"""
import numpy as np
import pytest

from mvmc_inputs import workload
from oracle import sr as osr

from gpu_common import (good_configs, log, mixed_ratio_stats, oracle_trajectories, square_case)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x5EED1711


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1711_11418_amd import binding
    binding.load()


def _instances():
    insts = [workload(n)["instances"][0] for n in ("ring6", "sq4_sub2", "ring8_u4")]
    insts.append(square_case(6, 15, 24, full_f=False, n_hidden=12))
    for i, w in zip(insts[:3], (16, 40, 24)):
        i.n_walkers = w
    return insts


@pytest.mark.parametrize("solver", ["chol", "cg"])
def test_ragged_sr_per_instance(solver):
    from paper_1711_11418_amd import MVMC
    insts = _instances()
    params = np.concatenate([i.params0 for i in insts])
    slots = 4
    log(f"[batch-sr] {solver}: " + ", ".join(f"Ne={i.n_elec} Np={i.n_params} W={i.n_walkers}"
                                             for i in insts) + f" slots={slots}")
    ctx = MVMC(insts, params, seed=SEED, n_slots=slots, solver=solver, build_s=True,
               refresh_every=16)
    ctx.sample(5)
    for s in range(slots):
        ctx.sample(1)
        ctx.measure(s)
    Os = [ctx.O_of(k, slots).cpu().numpy().copy() for k in range(len(insts))]
    Es = [ctx.eloc_of(k, slots).cpu().numpy().copy() for k in range(len(insts))]
    Eb, Ee, Ev = ctx.build_sr(slots)
    refs = []
    for k, inst in enumerate(insts):
        ref = osr.sr_stats(Os[k], Es[k])
        refs.append(ref)
        wm = Es[k].reshape(slots, inst.n_walkers).mean(axis=0)
        sig = wm.std(ddof=1) / np.sqrt(inst.n_walkers)
        assert Eb[k] == pytest.approx(ref["E"], rel=1e-13)
        assert Ev[k] == pytest.approx(ref["E_var"], rel=1e-10)
        assert Ee[k] == pytest.approx(sig, rel=1e-10)
        S = ctx.S_of(k).cpu().numpy()
        assert np.max(np.abs(S - ref["S"])) <= 1e-12 * np.max(np.abs(ref["S"])), k
        g = ctx.params_of(k, ctx.g).cpu().numpy()
        assert np.max(np.abs(g - ref["g"])) <= 1e-12 * max(np.max(np.abs(ref["g"])), 1e-300) + 1e-15
        Oc = ctx.O_of(k, slots).cpu().numpy()
        assert np.allclose(Oc, ref["Oc"], rtol=0, atol=1e-13 * max(1.0, np.max(np.abs(Os[k]))))
    p0 = ctx.params.cpu().numpy().copy()
    it = ctx.sr_update(dtau=0.05, eps_rel=1e-3, eps_abs=1e-6, solver=solver, cg_tol=1e-12,
                       cg_maxit=2000)
    d_all = ctx.dparams.cpu().numpy()
    for k, inst in enumerate(insts):
        want = osr.sr_update(Os[k], Es[k], 0.05, 1e-3, 1e-6, solver=solver, cg_eps=1e-12,
                             cg_kmax=2000)
        d = ctx.params_of(k, ctx.dparams).cpu().numpy()
        if solver == "chol":
            assert np.allclose(d, want["dalpha"], rtol=1e-8,
                               atol=1e-11 * np.max(np.abs(want["dalpha"]))), k
        else:
            log(f"  instance {k}: cg iterations gpu={it[k]} oracle={want['cg_iters']}")
            assert abs(int(it[k]) - want["cg_iters"]) <= max(3, want["cg_iters"] // 10)
            kappa = np.linalg.cond(want["S_reg"])
            err = np.linalg.norm(d - want["dalpha"]) / np.linalg.norm(want["dalpha"])
            assert err <= 2 * kappa * 1e-12, (k, err, kappa)
    assert np.allclose(ctx.params.cpu().numpy(), p0 + d_all, rtol=0, atol=1e-15)
    ctx.close()


def test_ragged_replay_mixed():
    from paper_1711_11418_amd import MVMC
    insts = _instances()
    for i in insts:
        i.n_walkers = 4
    params = np.concatenate([i.params0 for i in insts])
    pos0 = [good_configs(i, i.params0, i.n_walkers, 17, cond_max=1e4) for i in insts]
    sweeps = 4
    log("[batch-mixed] " + ", ".join(f"Ne={i.n_elec}xW={i.n_walkers}" for i in insts) +
        f" sweeps={sweeps} refresh 32")
    ctx = MVMC(insts, params, seed=SEED, precision="mixed", refresh_every=32, build_s=False,
               solver="cg")
    ctx.set_state(np.concatenate([p.ravel() for p in pos0]),
                  np.zeros(sum(i.n_walkers for i in insts), dtype=np.int64))
    ctx.enable_trace(sweeps * max(i.n_elec for i in insts))
    ctx.sample(sweeps)
    rec = ctx.trace_records()
    for k, inst in enumerate(insts):
        lay = ctx.layouts[k]
        n_prop = sweeps * inst.n_elec
        walkers, m = oracle_trajectories(inst, inst.params0, pos0[k], lay.walker_off, n_prop, SEED)
        sub = rec[lay.walker_off:lay.walker_off + inst.n_walkers]
        st = mixed_ratio_stats(inst, m, sub, walkers, pos0[k], n_prop, SEED, refresh_every=32)
        log(f"  instance {k} (Ne={inst.n_elec}): {st['summary']}")
        assert st["within_bound"], st["summary"]
        assert st["compared"] > 0.5 * n_prop * inst.n_walkers
    ctx.close()
