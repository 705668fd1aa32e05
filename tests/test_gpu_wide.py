"""GPU parity at the widest shapes the benchmark runs, through the C ABI.

* the double recomputation of X^-1 and Pf(X) for 64 < N_e/2 <= 128 (the
  16 x 16-thread tiled route of the anti-parallel block, section 3.2.1),
  at N_e = 144, 196 and 224;
* one sweep of trajectory replay at N_e = 224 with an RBM factor on the
  kernel that streams X^-1 from HBM, in double (ratios to 1e-10) and in
  single precision (ratio error against its derived bound);
* the single-precision local energy and O_k against the oracle, element by
  element, against bounds derived from the rounding of the single-precision
  inputs.

Every case prints its name, shapes and seeds before touching the GPU.
"""
import numpy as np
import pytest

from oracle import wavefunction as wf
from oracle.pfaffian import pfaffian_log

from gpu_common import (U32, compare_trace, good_configs, log, mixed_ratio_stats, oracle_measure,
                        oracle_trajectories, square_case)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x5EED1711


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1711_11418_amd import binding
    binding.load()


def _ctx(insts, params, **kw):
    from paper_1711_11418_amd import MVMC
    return MVMC(insts, params, **kw)


@pytest.mark.parametrize("L,nsig,M,precision", [(12, 72, 0, "fp64"), (14, 98, 0, "fp64"),
                                                (16, 112, 64, "fp64"), (16, 112, 64, "mixed")])
def test_refresh_tiled_route(L, nsig, M, precision):
    inst = square_case(L, nsig, 4, full_f=False, n_hidden=M)
    pos0 = good_configs(inst, inst.params0, inst.n_walkers, 3)
    log(f"[refresh-wide] {L}x{L}: Ne={inst.n_elec} M={M} W={inst.n_walkers} {precision}")
    ctx = _ctx([inst], inst.params0, precision=precision, build_s=False, solver="cg")
    ctx.set_state(pos0.ravel(), np.zeros(inst.n_walkers, dtype=np.int64))
    Y = ctx.Y_of(ctx.get_inverse(), 0).cpu().numpy()
    la, sg = (t.cpu().numpy() for t in ctx.get_pfaffian())
    A = wf.skew_table(wf.expand(inst, inst.params0))
    # double refresh cast to the walker type: 1e-10 in double, one rounding
    # to single precision otherwise
    ytol = 1e-10 if precision == "fp64" else 2 * U32
    worst = 0.0
    for w in range(inst.n_walkers):
        X = A[np.ix_(pos0[w], pos0[w])]
        Yr = np.linalg.inv(X)
        err = np.max(np.abs(Y[w] - Yr)) / np.max(np.abs(Yr))
        worst = max(worst, err)
        assert err <= ytol, (w, err)
        s, l = pfaffian_log(X)
        assert sg[w] == s
        assert la[w] == pytest.approx(l, abs=1e-10 * max(1.0, abs(l)))
    log(f"  max |Y - inv X| / max|inv X| = {worst:.2e}")
    ctx.close()


def test_replay_wide_hbm_rbm_fp64():
    """One sweep (224 proposals) of two walkers at N_e = 224 with M = 64
    hidden units on the HBM-resident kernel (X^-1 does not fit LDS), with a
    double refresh every 100 proposals between launches (tiled route)."""
    inst = square_case(16, 112, 2, full_f=False, n_hidden=64)
    pos0 = good_configs(inst, inst.params0, inst.n_walkers, 7)
    n_prop = inst.n_elec
    log(f"[replay-wide] 16x16 Ne=224 M=64 W=2 proposals={n_prop} fp64 HBM refresh 100 "
        f"seed={SEED}")
    ctx = _ctx([inst], inst.params0, seed=SEED, refresh_every=100, sweep_threads=256,
               build_s=False, solver="cg")
    assert ctx.sweep_variants() == ["hbm256"]
    ctx.set_state(pos0.ravel(), np.zeros(inst.n_walkers, dtype=np.int64))
    ctx.enable_trace(n_prop)
    acc = ctx.sample(1)
    rec = ctx.trace_records()
    walkers, m = oracle_trajectories(inst, inst.params0, pos0, 0, n_prop, SEED)
    st = compare_trace(rec, walkers, n_prop, SEED, rtol=1e-10)
    log(f"  compared {st['compared']} ratios, worst rel err {st['worst_rel']:.2e}, accepted {acc}")
    pos = ctx.pos_of(ctx.get_state()[0], 0).cpu().numpy()
    assert np.array_equal(pos, np.array([wk.pos for wk in walkers]))
    Y = ctx.Y_of(ctx.get_inverse(), 0).cpu().numpy()
    A = wf.skew_table(m)
    for w in range(inst.n_walkers):
        Yr = np.linalg.inv(A[np.ix_(pos[w], pos[w])])
        assert np.max(np.abs(Y[w] - Yr)) <= 1e-9 * np.max(np.abs(Yr)), w
    ctx.measure(0)
    el = ctx.eloc_of(0, 1).cpu().numpy()
    O = ctx.O_of(0, 1).cpu().numpy()
    e_ref, o_ref = oracle_measure(inst, m, pos[0])
    log(f"  E_loc gpu {el[0]:.12f} oracle {e_ref:.12f}")
    assert el[0] == pytest.approx(e_ref, rel=1e-10, abs=1e-10)
    assert np.allclose(O[0], o_ref, rtol=1e-9, atol=1e-10)
    ctx.close()


def test_replay_wide_hbm_rbm_mixed():
    """The same sweep in single precision with the double refresh every 32
    proposals: every ratio against the bound of the rounding analysis
    (gpu_common.mixed_ratio_stats)."""
    inst = square_case(16, 112, 2, full_f=False, n_hidden=64)
    pos0 = good_configs(inst, inst.params0, inst.n_walkers, 7)
    n_prop = inst.n_elec
    log(f"[replay-wide] 16x16 Ne=224 M=64 W=2 proposals={n_prop} mixed HBM refresh 32 "
        f"seed={SEED}")
    ctx = _ctx([inst], inst.params0, seed=SEED, precision="mixed", refresh_every=32,
               sweep_threads=256, build_s=False, solver="cg")
    assert ctx.sweep_variants() == ["hbm256"]
    ctx.set_state(pos0.ravel(), np.zeros(inst.n_walkers, dtype=np.int64))
    ctx.enable_trace(n_prop)
    ctx.sample(1)
    rec = ctx.trace_records()
    walkers, m = oracle_trajectories(inst, inst.params0, pos0, 0, n_prop, SEED)
    st = mixed_ratio_stats(inst, m, rec, walkers, pos0, n_prop, SEED, refresh_every=32)
    log(f"  mixed 224: {st['summary']}")
    assert st["within_bound"], st["summary"]
    ctx.close()


@pytest.mark.parametrize("precision,threads", [("fp64", 256), ("fp64", 128), ("mixed", 256)])
def test_replay_wide_ap_block_rbm(precision, threads):
    """The anti-parallel-block sweep (M^-1 alone in LDS, rank-1 updates) at
    N_e = 224 with M = 64 hidden units: one sweep of two walkers, a double
    refresh every 100 (double) or 32 (single precision) proposals; ratios
    to 1e-10 in double, against the rounding bound in single precision; the
    inverse written back equals inv(X) and E_loc, O_k follow from it."""
    inst = square_case(16, 112, 2, full_f=False, n_hidden=64)
    pos0 = good_configs(inst, inst.params0, inst.n_walkers, 7)
    n_prop = inst.n_elec
    R = 100 if precision == "fp64" else 32
    variant = f"ap{threads}"
    log(f"[replay-ap] 16x16 Ne=224 M=64 W=2 proposals={n_prop} {precision} {variant} "
        f"refresh {R} seed={SEED}")
    ctx = _ctx([inst], inst.params0, seed=SEED, precision=precision, refresh_every=R,
               sweep_variant=variant, build_s=False, solver="cg")
    assert ctx.sweep_variants() == [variant]
    ctx.set_state(pos0.ravel(), np.zeros(inst.n_walkers, dtype=np.int64))
    ctx.enable_trace(n_prop)
    acc = ctx.sample(1)
    rec = ctx.trace_records()
    walkers, m = oracle_trajectories(inst, inst.params0, pos0, 0, n_prop, SEED)
    if precision == "mixed":
        st = mixed_ratio_stats(inst, m, rec, walkers, pos0, n_prop, SEED, refresh_every=R)
        log(f"  mixed ap: {st['summary']}")
        assert st["within_bound"], st["summary"]
        ctx.close()
        return
    st = compare_trace(rec, walkers, n_prop, SEED, rtol=1e-10)
    log(f"  compared {st['compared']} ratios, worst rel err {st['worst_rel']:.2e}, accepted {acc}")
    pos = ctx.pos_of(ctx.get_state()[0], 0).cpu().numpy()
    assert np.array_equal(pos, np.array([wk.pos for wk in walkers]))
    Y = ctx.Y_of(ctx.get_inverse(), 0).cpu().numpy()
    A = wf.skew_table(m)
    for w in range(inst.n_walkers):
        Yr = np.linalg.inv(A[np.ix_(pos[w], pos[w])])
        assert np.max(np.abs(Y[w] - Yr)) <= 1e-9 * np.max(np.abs(Yr)), w
    if threads == 256:
        ctx.measure(0)
        el = ctx.eloc_of(0, 1).cpu().numpy()
        e_ref, o_ref = oracle_measure(inst, m, pos[1])
        assert el[1] == pytest.approx(e_ref, rel=1e-10, abs=1e-10)
        assert np.allclose(ctx.O_of(0, 1).cpu().numpy()[1], o_ref, rtol=1e-9, atol=1e-10)
    ctx.close()


@pytest.mark.parametrize("name", ["sq6_rbm", "sq10_full"])
def test_measure_single_precision(name):
    """E_loc and O_k of the single-precision path at configurations loaded
    with set_state (X^-1 freshly recomputed in double, then rounded).
    The kernel forms r_Pf from single-precision X^-1 and pair amplitudes
    with products and sums in double, and the correlator factors in double,
    so each hop term carries at most 2u |t| e^(dlog) sum_b |x'_b Y_ab|
    (u = 2^-24); O_f = -sum Y_ab carries u sum |Y_ab| and one final rounding,
    the RBM terms one rounding each, the Jastrow and Gutzwiller counts none."""
    if name == "sq6_rbm":
        inst = square_case(6, 16, 4, full_f=False, n_hidden=24)
    else:
        inst = square_case(10, 50, 4, full_f=True)
    pos0 = good_configs(inst, inst.params0, inst.n_walkers, 13)
    log(f"[measure-fp32] {name}: Ne={inst.n_elec} M={inst.n_hidden} W={inst.n_walkers}")
    ctx = _ctx([inst], inst.params0, precision="mixed", refresh_every=32, build_s=False,
               solver="cg")
    ctx.set_state(pos0.ravel(), np.zeros(inst.n_walkers, dtype=np.int64))
    ctx.measure(0)
    el = ctx.eloc_of(0, 1).cpu().numpy()
    O = ctx.O_of(0, 1).cpu().numpy().astype(np.float64)
    m = wf.expand(inst, inst.params0)
    A = wf.skew_table(m)
    worst_e = worst_o = 0.0
    for w in range(inst.n_walkers):
        e_ref, o_ref = oracle_measure(inst, m, pos0[w])
        be, bo = _measure_bounds(inst, m, A, pos0[w], o_ref)
        de = abs(el[w] - e_ref)
        do = np.abs(O[w] - o_ref)
        worst_e = max(worst_e, de / be)
        worst_o = max(worst_o, float(np.max(do / bo)))
        assert de <= be, (w, el[w], e_ref, be)
        assert np.all(do <= bo), (w, int(np.argmax(do / bo)))
    log(f"  |dE| / bound max {worst_e:.3f}, |dO| / bound max {worst_o:.3f} "
        f"(E_loc rel err {abs(el[-1] - e_ref) / abs(e_ref):.2e})")
    ctx.close()


def _measure_bounds(inst, m, A, pos, o_ref):
    """Bounds of the single-precision measurement (see the test docstring),
    doubled for margin, from the oracle's inverse."""
    ns, nup, ne = m.n_sites, m.n_up, m.n_elec
    X = A[np.ix_(pos, pos)]
    Y = np.linalg.inv(X)
    nv = wf.occupations(m, pos)
    s0, l0 = wf.log_psi(m, pos, A)
    lc0 = wf.log_correlators(m, pos)
    be = 0.0
    nbr = [[] for _ in range(ns)]
    for (i, j), t in zip(m.bonds, m.bond_t):
        nbr[int(i)].append((int(j), float(t)))
        nbr[int(j)].append((int(i), float(t)))
    for a in range(ne):
        I = int(pos[a])
        sig = I // ns
        for j, t in nbr[I - sig * ns]:
            J = j + sig * ns
            if nv[J]:
                continue
            new = pos.copy()
            new[a] = J
            xr = A[J, pos]
            xr[a] = 0.0
            corr = np.exp(wf.log_correlators(m, new) - lc0)
            be += abs(t) * corr * float(np.sum(np.abs(xr * Y[:, a])))
    be = 2 * (2 * U32 * be) + 1e-12 * max(1.0, abs(float(np.dot(m.U, nv[:ns] * nv[ns:]))))
    o = inst.offsets()
    absY = np.zeros(inst.n_params)
    for a in range(nup):
        for b in range(nup, ne):
            k = int(inst.f_idx[int(pos[a]), int(pos[b]) - ns])
            if k >= 0:
                absY[o["f"] + k] += abs(Y[a, b])
    bo = 2 * (U32 * (absY + np.abs(o_ref))) + 1e-300
    return be, bo
