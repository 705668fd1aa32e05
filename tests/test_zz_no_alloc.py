"""The context without device allocation (mvmc_init_wavefunction_static,
workspace in the library's static per-device array) against the regular
context with a caller-allocated workspace: same initial walkers, inverses,
Pfaffians, proposal traces, local energies, O_k and SR statistics, bit for
bit, on two static contexts in a row (the second smaller, reusing the array
the first left behind), and a clear MVMC_E_WORKSPACE beyond the array's size.
"""
import numpy as np
import pytest

from mvmc_inputs import workload

from gpu_common import log, square_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1711_11418_amd import binding
    binding.load()


def _run(inst, static, precision, **kw):
    from paper_1711_11418_amd import MVMC
    ctx = MVMC([inst], inst.params0, precision=precision, static_workspace=static, **kw)
    out = {"Y": ctx.get_inverse().cpu(), "pf": [t.cpu() for t in ctx.get_pfaffian()],
           "state": [t.cpu() for t in ctx.get_state(with_empty=True)]}
    n_prop = 3 * inst.n_elec
    ctx.enable_trace(n_prop)
    out["acc"] = ctx.sample(3)
    out["trace"] = ctx.trace_records().copy()
    for s in range(2):
        ctx.sample(1)
        ctx.measure(s)
    out["eloc"] = ctx.eloc.cpu()
    out["O"] = ctx.O.cpu()
    out["sr"] = ctx.build_sr(2)
    out["S"] = ctx.S.cpu()
    out["g"] = ctx.g.cpu()
    ctx.sr_update(dtau=0.02)
    out["params"] = ctx.params.cpu()
    out["Y2"] = ctx.get_inverse().cpu()
    ctx.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_workspace_matches_allocated(precision):
    from paper_1711_11418_amd import binding
    first = square_case(6, 15, 64, full_f=False, n_hidden=12)
    second = workload("ring6")["instances"][0]
    second.n_walkers = 8
    for inst in (first, second):
        kw = dict(seed=4321, refresh_every=32, n_slots=2, solver="chol", build_s=True)
        need = binding.query_sizes(binding.make_config([inst], precision, 32, 4321, n_slots=2)).workspace_bytes
        log(f"[no-alloc] {inst.name} {precision}: Ne={inst.n_elec} W={inst.n_walkers} "
            f"workspace {need} bytes")
        a = _run(inst, False, precision, **kw)
        b = _run(inst, True, precision, **kw)
        assert torch.equal(a["Y"], b["Y"])
        for x, y in zip(a["pf"] + a["state"], b["pf"] + b["state"]):
            assert torch.equal(x, y)
        assert np.array_equal(a["acc"], b["acc"])
        assert np.array_equal(a["trace"].view(np.uint8), b["trace"].view(np.uint8))
        for k in ("eloc", "O", "S", "g", "params", "Y2"):
            assert torch.equal(a[k], b[k]), k
        for x, y in zip(a["sr"], b["sr"]):
            assert np.array_equal(x, y)


def test_static_workspace_size_limit():
    """The 10x10 workload (4096 walkers) needs about 1.5 GB of workspace:
    the static entry point refuses it with MVMC_E_WORKSPACE and no context."""
    import ctypes as C

    from paper_1711_11418_amd import binding
    inst = workload("sq10_u8")["instances"][0]
    cfg = binding.make_config([inst], "fp64", 400, 1, n_slots=1)
    need = binding.query_sizes(cfg).workspace_bytes
    log(f"[no-alloc] sq10_u8 needs {need} bytes")
    assert need > 64 << 20
    lib = binding.load()
    params = torch.as_tensor(inst.params0).cuda()
    ctx = C.c_void_p()
    rc = lib.mvmc_init_wavefunction_static(C.byref(ctx), C.byref(cfg),
                                           C.c_void_p(params.data_ptr()),
                                           C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 3 and not ctx.value
