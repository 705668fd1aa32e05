"""Helpers shared by the GPU parity tests (not collected by itself)."""
from __future__ import annotations

import sys

import numpy as np

from mvmc_inputs import random_configs
from mvmc_inputs.instance import f_map_full, f_map_sublattice, make_instance, v_map_nn
from mvmc_inputs.lattice import square
from oracle import measure, sampler
from oracle import wavefunction as wf
from oracle.philox import proposal_draw, uniform53


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def square_case(L: int, n_sigma: int, n_walkers: int, full_f: bool = True, seed: int = 5,
                n_hidden: int = 0, U: float = 4.0):
    lat = square(L)
    fmap = f_map_full(lat) if full_f else f_map_sublattice(lat, 2, 2)
    return make_instance(f"sq{L}_{n_sigma}", lat, n_sigma, n_sigma, U, fmap, v_map_nn(lat),
                         f_noise=0.05, n_walkers=n_walkers, n_hidden=n_hidden, rbm_sigma=0.05,
                         seed=seed)


def good_configs(inst, params, n: int, seed: int, cond_max: float = 1e5) -> np.ndarray:
    """n configurations whose X has 2-norm condition number below cond_max."""
    m = wf.expand(inst, params)
    A = wf.skew_table(m)
    out = []
    s = seed
    while len(out) < n:
        for pos in random_configs(inst, 64, s):
            X = A[np.ix_(pos, pos)]
            if np.linalg.cond(X) < cond_max:
                out.append(pos)
                if len(out) == n:
                    break
        s += 1
        if s > seed + 200:
            raise RuntimeError("could not find well-conditioned configurations")
    return np.array(out, dtype=np.int32)


def oracle_trajectories(inst, params, pos0: np.ndarray, gid0: int, n_prop: int, seed: int):
    """Run the oracle chain of every walker; returns (walkers, model)."""
    m = wf.expand(inst, params)
    A = wf.skew_table(m)
    ws = []
    for w in range(len(pos0)):
        wk = sampler.make_walker(m, pos0[w], gid=gid0 + w)
        for _ in range(n_prop):
            sampler.step(m, wk, seed, A, record=True)
        ws.append(wk)
    return ws, m


def compare_trace(rec: np.ndarray, walkers, n_prop: int, seed: int, rtol: float = 1e-10,
                  mixed: bool = False, floor: float = 1e-6) -> dict:
    """Compare GPU trace records with oracle traces.

    Ratio error is |R_gpu - R| / max(|R|, floor).  FP64: every decision
    must match and the error stay below rtol.  Mixed (single-precision
    inverse): the error stays below rtol with floor ~ 1e-2, because the dot
    product of row a of X^-1 with the new row of X cancels for small R and
    its single-precision error is absolute; a differing decision is allowed
    only when u lies within the ratio error of R^2, after which that chain
    is no longer compared.
    """
    n_cmp = 0
    worst = 0.0
    diverged = 0
    errors = []
    for w, wk in enumerate(walkers):
        for k in range(n_prop):
            n, a, inew, R, acc = wk.trace[k]
            g = rec[w, k]
            assert int(g["n"]) == n, (w, k, int(g["n"]), n)
            assert int(g["a"]) == a and int(g["i_new"]) == inew, (w, k, g, wk.trace[k])
            if inew < 0:
                continue
            err = abs(float(g["ratio"]) - R) / max(abs(R), floor)
            worst = max(worst, err)
            errors.append(err)
            assert err <= rtol, (w, k, float(g["ratio"]), R, err)
            n_cmp += 1
            if bool(g["accepted"]) != acc:
                if not mixed:
                    raise AssertionError(f"walker {w} proposal {k}: decision differs")
                r = proposal_draw(seed, wk.gid, n)
                u = uniform53(r[2], r[3])
                dR = abs(float(g["ratio"]) - R)
                assert abs(u - R * R) <= 2.5 * dR * (abs(R) + dR) + 1e-15, (w, k, u, R)
                diverged += 1
                break
    return {"compared": n_cmp, "worst_rel": worst, "diverged": diverged, "errors": errors}


def oracle_measure(inst, m, pos):
    A = wf.skew_table(m)
    return measure.local_energy(m, pos, A), measure.log_derivs(inst, m, pos, A)
