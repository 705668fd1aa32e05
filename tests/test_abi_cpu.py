"""The C-ABI library loads, exports every declared symbol, and validates
configurations on the host (no GPU needed: these calls touch no device)."""
import os
import re

import numpy as np
import pytest

from mvmc_inputs import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1711_11418_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libmvmc.so is not built (run __graft_entry__.build())")
    return binding


def test_every_declared_symbol_is_exported():
    b = _lib()
    hdr = open(os.path.join(ROOT, "include", "mvmc.h")).read()
    declared = set(re.findall(r"^(?:int|size_t|const char \*)\s*(mvmc_\w+)\(", hdr, re.M))
    assert declared == set(b.ENTRY_POINTS)
    lib = b.load()
    for name in declared:
        assert hasattr(lib, name), name


def test_query_sizes_c2_shapes():
    b = _lib()
    wl = workload("sq8_u4", n_walkers=1024)
    cfg = b.make_config(wl["instances"], "fp64", 256, 7, n_slots=200)
    s = b.query_sizes(cfg)
    assert s.n_walkers == 1024 and s.n_params == 271
    assert s.eloc_elems == 200 * 1024
    lay = b.query_layout(cfg, 0)
    assert lay.O_ld == 320 and lay.n_elec == 64 and lay.n_sites == 64
    assert s.O_elems == 200 * 1024 * 320
    assert s.S_elems == 271 * 271 and s.O_elem_bytes == 8
    assert s.Y_elems == 1024 * 64 * 64


def test_batched_layout_is_contiguous():
    b = _lib()
    insts = workload("batch32_ragged", n_walkers=8)["instances"]
    cfg = b.make_config(insts, "mixed", 32, 7, n_slots=2, build_s=True)
    s = b.query_sizes(cfg)
    offs = [b.query_layout(cfg, k) for k in range(32)]
    assert s.O_elem_bytes == 4
    assert offs[0].param_off == 0 and offs[0].walker_off == 0
    for k in range(1, 32):
        assert offs[k].param_off == offs[k - 1].param_off + offs[k - 1].n_params
        assert offs[k].walker_off == offs[k - 1].walker_off + 8
        assert offs[k].O_off == offs[k - 1].O_off + 2 * 8 * offs[k - 1].O_ld
    assert s.n_params == sum(i.n_params for i in insts)


@pytest.mark.parametrize("mutate,code", [
    (lambda i: setattr(i, "n_dn", i.n_dn - 1), 2),                  # n_up != n_dn
    (lambda i: setattr(i, "n_walkers", 0), 2),
    (lambda i: i.f_idx.__setitem__((0, 0), 10 ** 6), 1),           # slot out of range
    (lambda i: i.v_idx.__setitem__((0, 1), 5), 1),                 # asymmetric Jastrow map
    (lambda i: i.v_idx.__setitem__((2, 2), 0), 1),                 # diagonal Jastrow entry
    (lambda i: i.U.__setitem__(0, np.nan), 6),
])
def test_invalid_descriptors_are_rejected(mutate, code):
    b = _lib()
    inst = workload("ring6")["instances"][0]
    mutate(inst)
    cfg = b.make_config([inst], "fp64", 0, 1)
    with pytest.raises(b.MVMCError) as e:
        b.query_sizes(cfg)
    assert e.value.status == code


def test_cholesky_requires_explicit_s():
    b = _lib()
    inst = workload("ring6")["instances"][0]
    cfg = b.make_config([inst], "fp64", 0, 1, solver="chol", build_s=False)
    with pytest.raises(b.MVMCError):
        b.query_sizes(cfg)


def test_refresh_unit_is_checked():
    """refresh_every counts proposals (0) or applied updates (1); any other
    unit is an argument error, and the update count adds one counter per
    walker to the workspace."""
    b = _lib()
    inst = workload("ring6")["instances"][0]
    sizes = {}
    for unit in ("proposals", "updates"):
        cfg = b.make_config([inst], "mixed", 32, 1, refresh_unit=unit)
        sizes[unit] = b.query_sizes(cfg).workspace_bytes
    assert sizes["proposals"] == sizes["updates"]
    cfg = b.make_config([inst], "mixed", 32, 1)
    cfg.refresh_unit = 2
    with pytest.raises(b.MVMCError) as e:
        b.query_sizes(cfg)
    assert e.value.status == 1


@pytest.mark.parametrize("kw", [dict(sweep_threads=64), dict(sweep_variant="lds64"),
                                dict(sweep_variant="ap128")])
def test_queue_schedule_rejects_other_variants(kw):
    """The persistent queue launch runs the register tier and the 256-thread
    anti-parallel-block sweep only."""
    b = _lib()
    insts = [workload(n)["instances"][0] for n in ("ring6", "sq4_sub2")]
    cfg = b.make_config(insts, "fp64", 16, 1, schedule="queue", **kw)
    with pytest.raises(b.MVMCError) as e:
        b.query_sizes(cfg)
    assert e.value.status == 1


def test_queue_schedule_shapes():
    """Queue schedule: a ragged batch plans (N_e 6..140); an anti-parallel
    block beyond 128 x 128 (N_e > 256) has no in-launch refresh: E_SHAPE."""
    from mvmc_inputs.instance import f_map_sublattice, make_instance, v_map_nn
    from mvmc_inputs.lattice import square
    b = _lib()
    insts = workload("batch32_ragged", n_walkers=8)["instances"]
    cfg = b.make_config(insts, "mixed", 32, 7, n_slots=1, build_s=False, solver="cg",
                        schedule="queue")
    b.query_sizes(cfg)
    lat = square(17)
    big = make_instance("sq17", lat, 130, 130, 4.0, f_map_sublattice(lat, 1, 1), v_map_nn(lat),
                        n_walkers=4)
    cfg = b.make_config([big], "fp64", 16, 1, build_s=False, solver="cg", schedule="queue")
    with pytest.raises(b.MVMCError) as e:
        b.query_sizes(cfg)
    assert e.value.status == 2


def _proj_case():
    inst = workload("sq4_sub2_proj4", n_walkers=8)["instances"][0]
    inst.proj_q = np.array(inst.proj_q, copy=True)
    inst.proj_w = np.array(inst.proj_w, copy=True)
    return inst


def test_projection_layout():
    """A projected instance keeps its N_P inverses M_p^-1 (n x n each) in its
    walker matrix space: Y_ld = max(N_e^2, N_P n^2)."""
    b = _lib()
    from mvmc_inputs.instance import translation_projection
    from mvmc_inputs.lattice import chain
    inst = _proj_case()
    cfg = b.make_config([inst], "fp64", 16, 1)
    lay = b.query_layout(cfg, 0)
    assert lay.Y_ld == 14 * 14 and b.query_sizes(cfg).Y_elems == 8 * 14 * 14
    ring = workload("ring6_proj3", n_walkers=4)["instances"][0]
    ring.proj_q, ring.proj_w = translation_projection(chain(6), [(r, 0) for r in range(6)])
    cfg = b.make_config([ring, inst], "mixed", 16, 1)
    assert b.query_layout(cfg, 0).Y_ld == 6 * 3 * 3 == 54 > 36
    assert b.query_layout(cfg, 1).Y_off == 4 * 54


@pytest.mark.parametrize("mutate,kw,code", [
    (lambda i: i.proj_q.__setitem__((1, 0), i.proj_q[1, 1]), {}, 1),   # not a permutation
    (lambda i: i.proj_q.__setitem__((0, 3), 16), {}, 1),                # site out of range
    (lambda i: setattr(i, "proj_w", np.zeros(4)), {}, 1),                # every weight zero
    (lambda i: i.proj_w.__setitem__(2, np.inf), {}, 6),
    (lambda i: (setattr(i, "proj_q", np.tile(i.proj_q, (9, 1))),
                setattr(i, "proj_w", np.ones(36))), {}, 1),            # N_P > MVMC_MAX_PROJ
    (lambda i: None, dict(exchange_per64=16), 1),                       # hops only
    (lambda i: None, dict(schedule="queue"), 1),                        # buckets only
])
def test_invalid_projections_are_rejected(mutate, kw, code):
    b = _lib()
    inst = _proj_case()
    mutate(inst)
    cfg = b.make_config([inst], "fp64", 16, 1, **kw)
    with pytest.raises(b.MVMCError) as e:
        b.query_sizes(cfg)
    assert e.value.status == code
