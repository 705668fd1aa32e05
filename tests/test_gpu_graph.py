"""HIP-graph capture of the sampling path: several replays, each preceded by
eager work (state reset, refresh, synchronisation), must reproduce the eager
run bit for bit (all kernels use fixed-order reductions)."""
import numpy as np
import pytest

from mvmc_inputs import workload

from gpu_common import good_configs, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("name,refresh,schedule,variant", [
    ("sq4_sub2", 0, "buckets", None), ("ring8_u4", 16, "buckets", None),
    ("ring8_u4", 16, "queue", None), ("sq4_sub2", 16, "queue", "ap256"),
    # refresh counted in applied updates (restarted by set_state)
    ("ring8_u4", "3u", "buckets", None), ("sq4_sub2", "3u", "buckets", "ap64"),
    ("ring8_u4", "3u", "queue", None)])
def test_captured_sampling_replays_match_eager(name, refresh, schedule, variant):
    from paper_1711_11418_amd import MVMC
    inst = workload(name)["instances"][0]
    inst.n_walkers = 16
    slots = 4
    pos0 = good_configs(inst, inst.params0, inst.n_walkers, 21)
    zero = np.zeros(inst.n_walkers, dtype=np.int64)
    side = torch.cuda.Stream()
    unit = "updates" if isinstance(refresh, str) else "proposals"
    refresh = int(str(refresh).rstrip("u"))
    log(f"[graph] {name}: W=16 slots={slots} refresh={refresh} ({unit}) {schedule} {variant}")
    with torch.cuda.stream(side):
        eager = MVMC([inst], inst.params0, seed=5, refresh_every=refresh, n_slots=slots,
                     build_s=False, solver="cg", stream=side, schedule=schedule,
                     sweep_variant=variant, refresh_unit=unit)
        eager.set_state(pos0.ravel(), zero)
        for s in range(slots):
            eager.sample_async(2)
            eager.measure(s)
        torch.cuda.synchronize()
        E_ref = eager.eloc_of(0, slots).cpu().numpy().copy()
        O_ref = eager.O_of(0, slots).cpu().numpy().copy()
        eager.close()

        ctx = MVMC([inst], inst.params0, seed=5, refresh_every=refresh, n_slots=slots,
                   build_s=False, solver="cg", stream=side, schedule=schedule,
                   sweep_variant=variant, refresh_unit=unit)
        ctx.set_state(pos0.ravel(), zero)
        torch.cuda.synchronize()
        g = ctx.capture_sampling(2, range(slots))
        for rep in range(3):
            ctx.set_state(pos0.ravel(), zero)      # eager reset + refresh between replays
            torch.cuda.synchronize()
            ctx.eloc.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            E = ctx.eloc_of(0, slots).cpu().numpy()
            O = ctx.O_of(0, slots).cpu().numpy()
            assert np.array_equal(E, E_ref), rep
            assert np.array_equal(O, O_ref), rep
        ctx.close()
