"""Autotuner of the sweep kernel variant per instance (ragged batch): every
instance ends on a variant that fits it, the chains stay exact after the
re-bucketing (trajectory replay against the oracle's full-recompute chain,
FP64, 1e-10), and a second context reuses the cached choices untimed."""
import numpy as np
import pytest

from mvmc_inputs import workload

from gpu_common import compare_trace, good_configs, log, oracle_trajectories, square_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 4242


def _batch():
    insts = [workload(n)["instances"][0] for n in ("ring6", "sq4_sub2", "ring8_u4")]
    insts.append(square_case(6, 15, 3, full_f=False))
    insts.append(square_case(8, 36, 2, full_f=False))    # N_e = 72: LDS/HBM kernels only
    for i in insts[:3]:
        i.n_walkers = 5
    return insts


def test_autotune_ragged_batch_replay(tmp_path):
    from paper_1711_11418_amd import MVMC
    from paper_1711_11418_amd.binding import SWEEP_VARIANT_NAMES
    insts = _batch()
    params = np.concatenate([i.params0 for i in insts])
    cache = tmp_path / "sweep_variants.txt"
    log("[autotune] " + ", ".join(f"Ne={i.n_elec}xW={i.n_walkers}" for i in insts))
    ctx = MVMC(insts, params, seed=SEED, refresh_every=9)
    before = ctx.sweep_variants()
    ms = ctx.autotune(2, cache)
    after = ctx.sweep_variants()
    log(f"  default {before} -> tuned {after}")
    for k, inst in enumerate(insts):
        row = ms[k]
        timed = [SWEEP_VARIANT_NAMES[v] for v in range(len(row)) if row[v] == row[v]]
        log(f"  Ne={inst.n_elec}: " + ", ".join(f"{SWEEP_VARIANT_NAMES[v]} {row[v]:.3f} ms"
                                               for v in range(len(row)) if row[v] == row[v]))
        assert timed, f"instance {k} was not timed"
        assert after[k] in timed
        best = np.nanargmin(row)
        assert after[k] == SWEEP_VARIANT_NAMES[best]
        if inst.n_elec > 64:
            assert after[k] != "reg"
    assert len(cache.read_text().strip().splitlines()) == len(insts)
    # exact chains after the variant switch
    pos0 = [good_configs(i, i.params0, i.n_walkers, 11) for i in insts]
    ctx.set_state(np.concatenate([p.ravel() for p in pos0]),
                  np.zeros(sum(i.n_walkers for i in insts), dtype=np.int64))
    sweeps = 2
    ctx.enable_trace(sweeps * max(i.n_elec for i in insts))
    ctx.sample(sweeps)
    rec = ctx.trace_records()
    for k, inst in enumerate(insts):
        lay = ctx.layouts[k]
        n_prop = sweeps * inst.n_elec
        walkers, _ = oracle_trajectories(inst, inst.params0, pos0[k], lay.walker_off, n_prop, SEED)
        sub = rec[lay.walker_off:lay.walker_off + inst.n_walkers]
        st = compare_trace(sub, walkers, n_prop, SEED, rtol=1e-10)
        assert st["compared"] == n_prop * inst.n_walkers
    ctx.close()
    # a second context takes the cached choices and times nothing
    ctx2 = MVMC(insts, params, seed=SEED + 1, refresh_every=9)
    ms2 = ctx2.autotune(2, cache)
    assert np.all(np.isnan(ms2))
    assert ctx2.sweep_variants() == after
    ctx2.close()


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_forced_variant_replay(tmp_path, variant):
    """Every LDS, HBM and anti-parallel-block sweep variant, pinned through a
    cache line, replays
    the oracle's chain (FP64, 1e-10) and keeps the inverse equal to inv(X):
    N_e = 72 on the 8x8 lattice, with in-launch refresh stops."""
    from paper_1711_11418_amd import MVMC
    from paper_1711_11418_amd.binding import SWEEP_VARIANT_NAMES
    from oracle import wavefunction as wf
    inst = square_case(8, 36, 3, full_f=False)
    cache = tmp_path / "pin.txt"
    cache.write_text(f"mvmc-sweep 0 {inst.n_elec} {inst.n_sites} 0 {inst.n_walkers} {variant}\n")
    log(f"[variant] {SWEEP_VARIANT_NAMES[variant]} Ne={inst.n_elec} W={inst.n_walkers}")
    ctx = MVMC([inst], inst.params0, seed=SEED, refresh_every=40)
    ms = ctx.autotune(1, cache)
    assert np.all(np.isnan(ms)) and ctx.sweep_variants() == [SWEEP_VARIANT_NAMES[variant]]
    pos0 = good_configs(inst, inst.params0, inst.n_walkers, 13)
    ctx.set_state(pos0.ravel(), np.zeros(inst.n_walkers, dtype=np.int64))
    sweeps = 2
    n_prop = sweeps * inst.n_elec
    ctx.enable_trace(n_prop)
    ctx.sample(sweeps)
    rec = ctx.trace_records()
    walkers, m = oracle_trajectories(inst, inst.params0, pos0, 0, n_prop, SEED)
    st = compare_trace(rec, walkers, n_prop, SEED, rtol=1e-10)
    log(f"  compared {st['compared']} ratios, worst rel err {st['worst_rel']:.2e}")
    assert st["compared"] == n_prop * inst.n_walkers
    pos, _ = ctx.get_state()
    pos = ctx.pos_of(pos, 0).cpu().numpy()
    Y = ctx.Y_of(ctx.get_inverse(), 0).cpu().numpy()
    A = wf.skew_table(m)
    for w in range(inst.n_walkers):
        Yr = np.linalg.inv(A[np.ix_(pos[w], pos[w])])
        assert np.max(np.abs(Y[w] - Yr)) <= 1e-9 * np.max(np.abs(Yr)), w
    ctx.close()
