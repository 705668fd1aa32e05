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


def oracle_trajectories(inst, params, pos0: np.ndarray, gid0: int, n_prop: int, seed: int,
                        ex64: int = 0):
    """Run the oracle chain of every walker; returns (walkers, model)."""
    m = wf.expand(inst, params)
    A = wf.skew_table(m)
    ws = []
    for w in range(len(pos0)):
        wk = sampler.make_walker(m, pos0[w], gid=gid0 + w)
        for _ in range(n_prop):
            sampler.step(m, wk, seed, A, record=True, ex64=ex64)
        ws.append(wk)
    return ws, m


def exchange_term_scale(m, A, pos, a: int, b: int, inew: int) -> float:
    """Magnitude of the two products whose difference is an exchange ratio:
    with Y the exact inverse of X and M^-1[b'][a'] = Y[n + b'][a'], the
    determinant lemma gives det M'/det M = rho sigma - beta gamma
    (rho: new row a against column a of M^-1; sigma: new column b against
    row b; beta = u . M^-1 c - u_b; gamma = M^-1[b][a]).  Rounding in the
    fast update is relative to |rho sigma| + |beta gamma| times the correlator
    factor, which is what a ratio far below that scale cancels."""
    ns, n = m.n_sites, m.n_up
    X = A[np.ix_(pos, pos)]
    Y = np.linalg.inv(X)
    Mi = Y[n:, :n]
    f = A[:ns, ns:]
    bd = b - n
    si, sj = int(pos[a]), int(pos[b]) - ns
    sdn = np.asarray(pos[n:]) - ns
    sup = np.asarray(pos[:n])
    rn = f[sj, sdn].copy()
    rn[bd] = f[sj, si]
    u = rn - f[si, sdn]
    c = f[sup, si].copy()
    c[a] = f[si, sj]
    rho = rn @ Mi[:, a]
    sig = Mi[bd, :] @ c
    bet = u @ (Mi @ c) - u[bd]
    gam = Mi[bd, a]
    new = np.array(pos).copy()
    new[a], new[b] = sj, si + ns
    corr = np.exp(wf.log_correlators(m, new) - wf.log_correlators(m, pos))
    return float(corr * (abs(rho * sig) + abs(bet * gam)))


def compare_trace(rec: np.ndarray, walkers, n_prop: int, seed: int, rtol: float = 1e-10,
                  floor: float = 1e-6, model=None, pos0=None) -> dict:
    """Compare GPU trace records with oracle traces (double precision).

    Ratio error is |R_gpu - R| / max(|R|, floor); every decision must match
    and the error stay below rtol.  (Single-precision traces are compared by
    mixed_ratio_stats against their rounding bound.)
    """
    n_cmp = 0
    worst = 0.0
    diverged = 0
    errors = []
    A = wf.skew_table(model) if model is not None else None
    for w, wk in enumerate(walkers):
        pos = None if pos0 is None else np.array(pos0[w], dtype=np.int64)
        for k in range(n_prop):
            n, a, inew, R, acc, b = wk.trace[k]
            g = rec[w, k]
            assert int(g["n"]) == n, (w, k, int(g["n"]), n)
            assert int(g["a"]) == a and int(g["i_new"]) == inew, (w, k, g, wk.trace[k])
            assert int(g["b"]) == b, (w, k, int(g["b"]), b)
            if inew < 0:
                continue
            scale = max(abs(R), floor)
            if b >= 0:
                # an exchange ratio is a difference of two products (2 x 2
                # determinant lemma); its rounding is relative to their size
                assert A is not None and pos is not None, "exchange traces need model and pos0"
                scale = max(scale, exchange_term_scale(model, A, pos, a, b, inew))
            if pos is not None and acc:
                if b >= 0:
                    pos[a], pos[b] = inew, int(pos[a]) + model.n_sites
                else:
                    pos[a] = inew
            err = abs(float(g["ratio"]) - R) / scale
            worst = max(worst, err)
            errors.append(err)
            assert err <= rtol, (w, k, float(g["ratio"]), R, err)
            n_cmp += 1
            if bool(g["accepted"]) != acc:
                raise AssertionError(f"walker {w} proposal {k}: decision differs")
    return {"compared": n_cmp, "worst_rel": worst, "diverged": diverged, "errors": errors}


def oracle_measure(inst, m, pos):
    A = wf.skew_table(m)
    return measure.local_energy(m, pos, A), measure.log_derivs(inst, m, pos, A)


U32 = 2.0 ** -24   # unit roundoff of binary32


def mixed_ratio_stats(inst, m, rec, walkers, pos0, n_prop: int, seed: int, refresh_every: int,
                      safety: float = 2.0, refresh_unit: str = "proposals") -> dict:
    """Single-precision ratios against the oracle, proposal by proposal, with
    a first-order forward error bound carried along the oracle's chain.

    Let Y be the exact X^-1 of the current configuration and E the error of
    the single-precision copy the kernel holds (Frobenius norm bounded by e).
    A double refresh leaves e = u |Y|_F (one rounding, u = 2^-24).  For a
    proposal moving electron a to I' with x' the new row of X (x'_a = 0):

      r_Pf = x'.Y[:, a]:  |dr| <= |x'| e + (2 + ceil(n/64)) u sum_b |x'_b Y_ba|
      (E, the rounding of x' and of each product; partial sums of at most
      ceil(n/64) terms in single precision, the rest in double);
      RBM log-ratio in single precision: |dlog| <= sum_h [2 dth_h +
      2u(|theta_h + d_h| + 1) + 2u(|theta_h| + 1) + u |d_h|], d_h the angle
      change and dth_h the drift bound of the single-precision angle;
      |dR| <= e^(dlog_c) |dr| + |R| |dlog|.

    An accepted update Y' = Y + (p q^T - q p^T)/r with p = Y[:, a] and
    q = -Y^T x' + e_a propagates the error to first order as
      e' <= e + 2(e |q| + |p| |dq|)/|r| + 2 |p| |q| |dr| / r^2
            + 3u (|Y'|_F + 2 |p| |q| / |r|)
    with |dq| <= |x'| e + n u | |Y|^T |x'| | (single-precision sums of n
    terms), and each angle drifts by u(|theta_h| + 2|d_h|).  The test bar is
    |R_gpu - R| <= safety * bound (first order: second-order terms are
    neglected).  A differing decision is allowed only when u lies within the
    bound of R^2; that chain is then no longer compared.

    The bound restarts at every double refresh: before proposal n when n is
    a multiple of refresh_every (refresh_unit "proposals"), or right after
    the accepted proposal that makes the walker's count of applied updates
    a multiple of it ("updates"; counted from the first traced proposal,
    which must be the first after set_state or the context's creation)."""
    from oracle.philox import proposal_draw, uniform53
    A = wf.skew_table(m)
    ns = m.n_sites
    ne = m.n_elec
    n_dot = ne // 2
    rel, over, ks = [], [], []
    diverged = 0
    ok = True
    for w, wk in enumerate(walkers):
        pos = np.array(pos0[w], dtype=np.int64)
        lc = wf.log_correlators(m, pos)
        Y = np.linalg.inv(A[np.ix_(pos, pos)])
        e = 0.0
        dth = np.zeros(m.n_hidden)
        k_acc = 0
        n_upd = 0              # applied updates so far (refresh_unit "updates")
        upd_refresh = False    # the last one completed a multiple of refresh_every
        for k in range(n_prop):
            n, a, inew, R, acc, b = wk.trace[k]
            g = rec[w, k]
            assert int(g["n"]) == n and int(g["a"]) == a and int(g["i_new"]) == inew, (w, k)
            nv = wf.occupations(m, pos)
            theta = m.b + m.W @ (2.0 * nv - 1.0) if m.n_hidden else np.zeros(0)
            if refresh_unit == "updates":
                assert k > 0 or n == 0, "update counting needs the trace from the start"
                refreshed = k == 0 or upd_refresh
            else:
                refreshed = k == 0 or (refresh_every and n % refresh_every == 0)
            upd_refresh = False
            if refreshed:
                e = U32 * np.linalg.norm(Y)
                dth = U32 * np.abs(theta)
                k_acc = 0
            if inew < 0:
                continue
            new = pos.copy()
            new[a] = inew
            xr = A[inew, pos].copy()
            xr[a] = 0.0
            lc_new = wf.log_correlators(m, new)
            corr = np.exp(lc_new - lc)
            col = Y[:, a]
            r = float(xr @ col)
            kd = float(np.sum(np.abs(xr * col)))
            nx = np.linalg.norm(xr)
            dr = nx * e + (2 + -(-n_dot // 64)) * U32 * kd
            dlog = 0.0
            d = np.zeros(0)
            if m.n_hidden:
                d = 2.0 * (m.W[:, inew] - m.W[:, int(pos[a])])
                dlog = float(np.sum(2 * dth + 2 * U32 * (np.abs(theta + d) + 1)
                                    + 2 * U32 * (np.abs(theta) + 1) + U32 * np.abs(d)))
            bound = safety * (corr * dr + abs(R) * dlog) + 1e-300
            err = abs(float(g["ratio"]) - R)
            rel.append(err / max(abs(R), 1e-300))
            over.append(err / bound)
            ks.append(k_acc)
            if err > bound:
                ok = False
            if bool(g["accepted"]) != acc:
                rr = proposal_draw(seed, wk.gid, n)
                u = uniform53(rr[2], rr[3])
                if abs(u - R * R) > 2.5 * bound * (abs(R) + bound) + 1e-15:
                    ok = False
                diverged += 1
                break
            if acc:
                q = -(Y.T @ xr)
                q[a] += 1.0
                npv, nq = np.linalg.norm(col), np.linalg.norm(q)
                dq = nx * e + n_dot * U32 * np.linalg.norm(np.abs(Y).T @ np.abs(xr))
                pos = new
                lc = lc_new
                Y = np.linalg.inv(A[np.ix_(pos, pos)])
                e = (e + 2 * (e * nq + npv * dq) / abs(r) + 2 * npv * nq * dr / r ** 2
                     + 3 * U32 * (np.linalg.norm(Y) + 2 * npv * nq / abs(r)))
                if m.n_hidden:
                    dth = dth + U32 * (np.abs(theta) + 2 * np.abs(d))
                k_acc += 1
                n_upd += 1
                upd_refresh = bool(refresh_every) and n_upd % refresh_every == 0
    rel = np.array(rel)
    over = np.array(over)
    ks = np.array(ks)
    summary = (f"compared {len(rel)}, error/bound max {over.max():.3f} median "
               f"{np.median(over):.2e}; rel err median {np.median(rel):.2e} p99 "
               f"{np.percentile(rel, 99):.2e} max {rel.max():.2e}; diverged chains {diverged}")
    return {"within_bound": ok, "summary": summary, "over": over, "rel": rel, "k": ks,
            "compared": len(rel), "diverged": diverged}
