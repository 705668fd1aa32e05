"""Error paths of the C ABI and checkpoint/resume, each forced from the host
(no kernel is made to fault): a singular X, a short or misaligned
workspace, calls out of order, non-finite parameters and ratios (the
double-refresh guard), and a bit-exact resume from mvmc_get_state /
mvmc_set_state.
"""
import ctypes as C

import numpy as np
import pytest

from mvmc_inputs import workload

from gpu_common import good_configs, log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x5EED1711
E_ARG, E_SHAPE, E_WORKSPACE, E_HIP, E_SINGULAR, E_NONFINITE, E_STATE = 1, 2, 3, 4, 5, 6, 7


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1711_11418_amd import binding
    binding.load()


def _ring6(**kw):
    inst = workload("ring6")["instances"][0]
    inst.n_walkers = kw.pop("n_walkers", 8)
    return inst


def test_singular_configuration_is_reported():
    """Site 0 has no pair amplitude (f_0j = 0 for all j), so a configuration
    with an up electron on site 0 has a zero row in X: set_state must
    return MVMC_E_SINGULAR naming the instance and walker."""
    from paper_1711_11418_amd import MVMC
    from paper_1711_11418_amd.binding import MVMCError
    inst = _ring6()
    inst.f_idx[0, :] = -1
    log("[errors] singular X via set_state (ring6, f_0j = 0)")
    ctx = MVMC([inst], inst.params0, seed=SEED, build_s=False, solver="cg")
    pos, cnt = ctx.get_state()
    pos = ctx.pos_of(pos, 0).cpu().numpy().copy()
    pos[3, :3] = [0, 1, 2]                     # up electrons on sites 0, 1, 2
    with pytest.raises(MVMCError) as e:
        ctx.set_state(pos.ravel(), cnt.cpu().numpy())
    assert e.value.status == E_SINGULAR
    assert "instance 0 walker 3" in str(e.value)
    ctx.close()


def test_workspace_too_small_or_misaligned():
    from paper_1711_11418_amd import binding as b
    inst = _ring6()
    cfg = b.make_config([inst], "fp64", 0, SEED, build_s=False, solver="cg")
    sz = b.query_sizes(cfg)
    lib = b.load()
    n = int(sz.workspace_bytes)
    ws = torch.empty(n + 512, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) // 256 * 256
    params = torch.as_tensor(inst.params0).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    log(f"[errors] workspace: need {n} bytes")
    ctx = C.c_void_p()
    rc = lib.mvmc_init_wavefunction(C.byref(ctx), C.byref(cfg), C.c_void_p(base), n - 1,
                                    C.c_void_p(params.data_ptr()), C.c_void_p(stream))
    assert rc == E_WORKSPACE and not ctx.value
    rc = lib.mvmc_init_wavefunction(C.byref(ctx), C.byref(cfg), C.c_void_p(base + 8), n,
                                    C.c_void_p(params.data_ptr()), C.c_void_p(stream))
    assert rc == E_WORKSPACE and not ctx.value
    rc = lib.mvmc_init_wavefunction(C.byref(ctx), C.byref(cfg), C.c_void_p(base), n,
                                    C.c_void_p(params.data_ptr()), C.c_void_p(stream))
    assert rc == 0 and ctx.value
    lib.mvmc_destroy(ctx)


def test_calls_out_of_order_and_bad_arguments():
    from paper_1711_11418_amd import MVMC
    from paper_1711_11418_amd.binding import MVMCError
    inst = _ring6()
    ctx = MVMC([inst], inst.params0, seed=SEED, n_slots=2)
    log("[errors] sr_update before build_sr, bad slot, bad configuration")
    with pytest.raises(MVMCError) as e:
        ctx.sr_update()
    assert e.value.status == E_STATE
    with pytest.raises(MVMCError) as e:
        ctx.measure(2)
    assert e.value.status == E_ARG
    pos, cnt = ctx.get_state()
    bad = ctx.pos_of(pos, 0).cpu().numpy().copy()
    bad[0, 1] = bad[0, 0]                      # two up electrons on one site
    with pytest.raises(MVMCError) as e:
        ctx.set_state(bad.ravel(), cnt.cpu().numpy())
    assert e.value.status == E_ARG
    pos, cnt, emp = ctx.get_state(with_empty=True)
    emp = emp.cpu().numpy().copy()
    emp[0] = pos.cpu().numpy()[0]               # an occupied site in the up list of walker 0
    with pytest.raises(MVMCError) as e:
        ctx.set_state(pos.cpu().numpy(), cnt.cpu().numpy(), emp)
    assert e.value.status == E_ARG and "empty-site list" in str(e.value)
    ctx.close()


@pytest.mark.parametrize("threads,schedule,variant", [(0, "buckets", None), (64, "buckets", None),
                                                      (0, "queue", None), (0, "queue", "ap256")])
def test_nonfinite_parameters_and_ratios(threads, schedule, variant):
    """A NaN parameter is refused by set_params (nothing changes).  A finite
    but huge Gutzwiller factor (g = 800, e^800 overflows) makes every ratio
    that creates a doublon infinite: the guard refreshes in double, retries,
    stops the walker and the synchronising call reports MVMC_E_NONFINITE with
    the instance and walker; set_params with sane values recovers."""
    from paper_1711_11418_amd import MVMC
    from paper_1711_11418_amd.binding import MVMCError
    inst = workload("sq4_sub2")["instances"][0]
    inst.n_walkers = 8
    log(f"[errors] non-finite guard, sweep_threads={threads} {schedule} {variant}")
    ctx = MVMC([inst], inst.params0, seed=SEED, build_s=False, solver="cg",
               sweep_threads=threads, schedule=schedule, sweep_variant=variant)
    p = inst.params0.copy()
    p[inst.offsets()["g"]] = np.nan
    with pytest.raises(MVMCError) as e:
        ctx.set_params(p)
    assert e.value.status == E_NONFINITE and "instance 0" in str(e.value)
    ctx.sample(1)                               # the old parameters still work
    p = inst.params0.copy()
    p[inst.offsets()["g"]:inst.offsets()["v"]] = 800.0
    ctx.set_params(p)
    with pytest.raises(MVMCError) as e:
        ctx.sample(3)
    assert e.value.status == E_NONFINITE
    msg = str(e.value)
    log(f"  {msg}")
    assert "instance 0 walker" in msg and "not finite" in msg
    ctx.set_params(inst.params0)
    acc = ctx.sample(2)
    assert acc[0] > 0
    ctx.close()


@pytest.mark.parametrize("precision,threads,refresh,schedule", [
    ("fp64", 0, 0, "buckets"), ("fp64", 64, 0, "buckets"), ("mixed", 0, 32, "buckets"),
    ("mixed", 128, 32, "buckets"), ("mixed", 0, 32, "queue")])
def test_resume_is_bit_exact(precision, threads, refresh, schedule):
    """Checkpoint after some sweeps, refresh the running context, load the
    checkpoint into a fresh context: both continue with bitwise-identical
    proposal traces (ratios included) and configurations."""
    from paper_1711_11418_amd import MVMC
    inst = workload("sq4_sub2")["instances"][0] if threads == 0 else _ring6()
    inst.n_walkers = 8
    kw = dict(precision=precision, seed=SEED, refresh_every=refresh, sweep_threads=threads,
              build_s=False, solver="cg", schedule=schedule)
    log(f"[resume] {precision} threads={threads} refresh={refresh} {schedule} Ne={inst.n_elec}")
    a = MVMC([inst], inst.params0, **kw)
    a.sample(7)
    pos, cnt, emp = a.get_state(with_empty=True)
    pos_h, cnt_h, emp_h = (x.cpu().numpy().copy() for x in (pos, cnt, emp))
    a.refresh()
    b = MVMC([inst], inst.params0, **kw)
    b.set_state(pos_h, cnt_h, emp_h)
    n_prop = 5 * inst.n_elec
    a.enable_trace(n_prop)
    b.enable_trace(n_prop)
    acc_a = a.sample(5)
    acc_b = b.sample(5)
    ta, tb = a.trace_records(), b.trace_records()
    assert np.array_equal(ta.view(np.uint8), tb.view(np.uint8))
    assert np.array_equal(acc_a, acc_b)
    pa, ca = a.get_state()
    pb, cb = b.get_state()
    assert torch.equal(pa, pb) and torch.equal(ca, cb)
    assert torch.equal(a.get_inverse(), b.get_inverse())
    a.close()
    b.close()
