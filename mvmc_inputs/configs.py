"""Named workloads: the five benchmark configurations and small test cases.

Each workload is a plain dict:

    instances       list[Instance]      (one, or 32 for the ragged batch)
    precision       "fp64" | "mixed"
    refresh_every   proposals between full double-precision recomputations
                    of the inverse (0 = only after parameter updates)
    sweeps          sweeps per SR iteration (1 sweep = N_e proposals/walker)
    warmup          sweeps before the first sample
    sample_every    sweeps between samples (one sample per walker each time)
    sr_iters        SR iterations
    dtau, eps_rel, eps_abs   SR step and diagonal regularisation
    solver          "chol" | "cg"
    sampler_seed    Philox key for the Metropolis chain

The physical content follows the benchmark descriptions; where a description
leaves a value open the value chosen here is stated next to it.
"""
from __future__ import annotations

import numpy as np

from .instance import (Instance, f_map_full, f_map_sublattice, make_instance,
                       ring8_orbitals, translation_projection, v_map_distance, v_map_nn)
from .lattice import chain, square

INPUT_SEED = 11418


def _c1(n_walkers: int = 64) -> list[Instance]:
    lat = chain(8)
    phi = ring8_orbitals()
    return [make_instance("ring8_U4", lat, 4, 4, 4.0, f_map_full(lat), v_map_nn(lat),
                          g0=-0.5, v_nn=0.1, f0=phi @ phi.T, f_noise=0.01,
                          n_walkers=n_walkers, seed=INPUT_SEED)]


def _c2(n_walkers: int = 1024) -> list[Instance]:
    lat = square(8)
    return [make_instance("sq8_U4", lat, 32, 32, 4.0, f_map_sublattice(lat, 2, 2),
                          v_map_distance(lat), g0=-0.5, v_nn=0.1,
                          n_walkers=n_walkers, seed=INPUT_SEED)]


def _c3(n_walkers: int = 4096) -> list[Instance]:
    lat = square(10)
    return [make_instance("sq10_U8", lat, 50, 50, 8.0, f_map_full(lat), v_map_nn(lat),
                          g0=-1.0, v_nn=0.1, n_walkers=n_walkers, seed=INPUT_SEED)]


def _c4(n_walkers: int = 256, n_inst: int = 32) -> list[Instance]:
    rng = np.random.default_rng(INPUT_SEED)
    out = []
    for k in range(n_inst):
        L = int(rng.integers(4, 13))
        U = float(rng.uniform(2.0, 10.0))
        fill = float(rng.uniform(0.8, 1.0))
        lat = square(L)
        ne = 2 * int(round(fill * lat.n_sites / 2))
        fmap = f_map_sublattice(lat, 2, 2) if L % 2 == 0 else f_map_sublattice(lat, 1, 1)
        out.append(make_instance(f"batch{k:02d}_L{L}_U{U:.2f}", lat, ne // 2, ne // 2, U,
                                 fmap, v_map_nn(lat), g0=-U / 8, v_nn=0.1,
                                 n_walkers=n_walkers, seed=INPUT_SEED + 1 + k))
    return out


def _c5(n_walkers: int = 8192, n_hidden: int = 512) -> list[Instance]:
    lat = square(16)
    name = "sq16_U8_rbm" if n_hidden else "sq16_U8_pj"
    return [make_instance(name, lat, 112, 112, 8.0, f_map_sublattice(lat, 2, 2),
                          v_map_nn(lat), g0=-1.0, v_nn=0.1, n_hidden=n_hidden,
                          rbm_sigma=0.01, n_walkers=n_walkers, seed=INPUT_SEED)]


def _wl(instances, **kw) -> dict:
    d = dict(instances=instances, precision="fp64", refresh_every=0, sweeps=10,
             warmup=100, sample_every=1, sr_iters=10, dtau=0.02, eps_rel=1e-3,
             eps_abs=1e-6, solver="chol", sampler_seed=1711 * 1000)
    d.update(kw)
    return d


def workload(name: str, **overrides) -> dict:
    """Build a named workload; keyword overrides replace defaults (e.g. n_walkers)."""
    nw = overrides.pop("n_walkers", None)
    kw_inst = {} if nw is None else {"n_walkers": nw}
    if name == "ring8_u4":
        d = _wl(_c1(**kw_inst), sweeps=1000, warmup=100, sample_every=1, sr_iters=0,
                sampler_seed=1711 * 1000 + 1)
    elif name == "sq8_u4":
        d = _wl(_c2(**kw_inst), sweeps=200, warmup=100, sample_every=1, sr_iters=10,
                refresh_every=4 * 64, sampler_seed=1711 * 1000 + 2)
    elif name == "sq10_u8":
        d = _wl(_c3(**kw_inst), precision="mixed", refresh_every=32, sweeps=10,
                warmup=100, sample_every=10, sr_iters=10, sampler_seed=1711 * 1000 + 3)
    elif name == "batch32_ragged":
        d = _wl(_c4(**kw_inst), precision="mixed", refresh_every=32, sweeps=10,
                warmup=100, sample_every=1, sr_iters=10, sampler_seed=1711 * 1000 + 4)
    elif name in ("sq16_u8_rbm", "sq16_u8_pj"):
        # the RBM state and its plain Pfaffian-Jastrow twin (same f, g, v start;
        # the RBM parameters are appended); double refresh once per sweep
        hid = {} if name == "sq16_u8_rbm" else {"n_hidden": 0}
        d = _wl(_c5(**kw_inst, **hid), precision="mixed", refresh_every=224, sweeps=10,
                warmup=100, sample_every=10, sr_iters=10, dtau=0.01, solver="cg",
                cg_tol=1e-3, cg_maxit=5000, sampler_seed=1711 * 1000 + 5)
    elif name == "ring4":
        lat = chain(4)
        d = _wl([make_instance("ring4_U4", lat, 2, 2, 4.0, f_map_full(lat), v_map_nn(lat),
                               f_noise=0.05, n_walkers=nw or 16, seed=INPUT_SEED)],
                sweeps=200, warmup=20, sr_iters=0)
    elif name == "ring6":
        lat = chain(6)
        d = _wl([make_instance("ring6_U4", lat, 3, 3, 4.0, f_map_full(lat), v_map_nn(lat),
                               f_noise=0.05, n_walkers=nw or 16, seed=INPUT_SEED)],
                sweeps=200, warmup=20, sr_iters=0)
    elif name == "sq4_sub2":
        lat = square(4)
        d = _wl([make_instance("sq4_U4", lat, 7, 7, 4.0, f_map_sublattice(lat, 2, 2),
                               v_map_distance(lat), f_noise=0.05, n_walkers=nw or 64,
                               seed=INPUT_SEED)], sweeps=20, warmup=10, sr_iters=2)
    elif name == "ring6_rbm":
        lat = chain(6)
        d = _wl([make_instance("ring6_rbm", lat, 3, 3, 4.0, f_map_full(lat), v_map_nn(lat),
                               f_noise=0.05, n_hidden=12, rbm_sigma=0.1,
                               n_walkers=nw or 16, seed=INPUT_SEED)],
                sweeps=100, warmup=20, sr_iters=0)
    elif name == "ring6_u8_gain":
        # 6-site ring at U = 8 with a translation-invariant pair amplitude
        # f(j - i): the same Pfaffian-Jastrow-Gutzwiller start with and
        # without an RBM factor of 12 hidden units (2 per site, weights
        # N(0, 0.01)); the RBM parameters are appended after the shared block
        lat = chain(6)
        pj = make_instance("ring6_U8_pj", lat, 3, 3, 8.0, f_map_sublattice(lat, 1, 1),
                           v_map_nn(lat), n_walkers=nw or 512, seed=INPUT_SEED)
        rbm = make_instance("ring6_U8_rbm", lat, 3, 3, 8.0, f_map_sublattice(lat, 1, 1),
                            v_map_nn(lat), n_hidden=12, rbm_sigma=0.01,
                            n_walkers=nw or 512, seed=INPUT_SEED)
        assert np.array_equal(rbm.params0[:pj.n_params], pj.params0)
        d = _wl([pj, rbm], sweeps=20, warmup=20, sr_iters=80, dtau=0.05,
                sampler_seed=1711 * 1000 + 6)
    elif name in ("ring4_proj", "ring4_projpi", "ring6_proj3"):
        # momentum projection (section 3.2.2): every translation of the
        # 4-site ring at K = 0 or pi, or the translations by 0, 2, 4 sites
        # of the 6-site ring at K = 0
        L = 6 if name == "ring6_proj3" else 4
        lat = chain(L)
        inst = make_instance(f"{name}_U4", lat, L // 2, L // 2, 4.0, f_map_full(lat),
                             v_map_nn(lat), f_noise=0.05, n_walkers=nw or 16, seed=INPUT_SEED)
        steps = [(0, 0), (2, 0), (4, 0)] if L == 6 else [(r, 0) for r in range(4)]
        inst.proj_q, inst.proj_w = translation_projection(
            lat, steps, kx=np.pi if name == "ring4_projpi" else 0.0)
        d = _wl([inst], sweeps=100, warmup=20, sr_iters=0)
    elif name in ("sq4_u4_proj4", "sq4_sub2_proj4"):
        # 4x4 with a 2x2-sublattice pair amplitude and the four translations
        # inside the 2x2 cell at K = 0 (with the sublattice structure this is
        # the full K = 0 momentum projection): half filling for the energy
        # leg, 7 + 7 electrons for parity
        lat = square(4)
        ne = 8 if name == "sq4_u4_proj4" else 7
        inst = make_instance(name, lat, ne, ne, 4.0, f_map_sublattice(lat, 2, 2),
                             v_map_distance(lat), f_noise=0.05, n_walkers=nw or 1024,
                             seed=INPUT_SEED)
        inst.proj_q, inst.proj_w = translation_projection(lat, [(0, 0), (1, 0), (0, 1), (1, 1)])
        d = _wl([inst], sweeps=20, warmup=50, sample_every=1, sr_iters=0, dtau=0.05,
                sampler_seed=1711 * 1000 + 7)
    else:
        raise KeyError(name)
    d["name"] = name
    d.update(overrides)
    return d


WORKLOADS = ("ring8_u4", "sq8_u4", "sq10_u8", "batch32_ragged",
             "sq16_u8_rbm", "sq16_u8_pj", "ring4", "ring6", "sq4_sub2", "ring6_rbm",
             "ring6_u8_gain", "ring4_proj", "ring4_projpi", "ring6_proj3", "sq4_u4_proj4",
             "sq4_sub2_proj4")


def random_configs(inst: Instance, n: int, seed: int) -> np.ndarray:
    """n uniformly drawn electron configurations, shape [n, N_e] int32.

    Electron a < n_up sits at spin-orbital I = site (up); a >= n_up at
    I = site + Ns (down).  Within a spin, sites are in ascending order.
    """
    rng = np.random.default_rng(seed)
    ns = inst.n_sites
    out = np.empty((n, inst.n_elec), dtype=np.int32)
    for w in range(n):
        up = np.sort(rng.choice(ns, inst.n_up, replace=False))
        dn = np.sort(rng.choice(ns, inst.n_dn, replace=False))
        out[w, :inst.n_up] = up
        out[w, inst.n_up:] = dn + ns
    return out
