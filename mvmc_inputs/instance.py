"""One Hubbard lattice instance with its variational-parameter index maps.

Parameter vector layout (per instance, float64):

    [ f (n_f) | g (n_g) | v (n_v) | a (2 Ns) | b (M) | W (M x 2 Ns, row-major) ]

The last three blocks exist only when the RBM correlator is on (M > 0).

Index maps follow the expert-mode keyword files of the paper (Table 1:
``Orbital``, ``Gutzwiller``, ``Jastrow``): each entry names the parameter slot
that a pair amplitude f_ij, a Gutzwiller factor g_i or a Jastrow factor v_ij
takes, or -1 when it is held at zero.  The sublattice structure of f_ij
(section 3.2.1, Wsub/Lsub) makes f_ij depend on the sublattice of i and the
displacement j - i only.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .lattice import Lattice


@dataclass
class Instance:
    name: str
    lattice: Lattice
    n_up: int
    n_dn: int
    U: np.ndarray               # [Ns] on-site interaction U_i
    t: float                    # nearest-neighbour hopping amplitude
    f_idx: np.ndarray           # [Ns, Ns] int32
    n_f: int
    g_idx: np.ndarray           # [Ns] int32
    n_g: int
    v_idx: np.ndarray           # [Ns, Ns] int32, symmetric, diagonal -1
    n_v: int
    n_hidden: int               # RBM hidden units M (0 = no RBM)
    n_walkers: int
    params0: np.ndarray = field(repr=False)   # initial parameter vector
    # quantum-number projection (section 3.2.2): site maps q_p [N_P, Ns] and
    # weights w_p [N_P]; None = no projection (one identity term)
    proj_q: np.ndarray | None = field(default=None, repr=False)
    proj_w: np.ndarray | None = field(default=None, repr=False)

    @property
    def n_sites(self) -> int:
        return self.lattice.n_sites

    @property
    def n_elec(self) -> int:
        return self.n_up + self.n_dn

    @property
    def bonds(self) -> np.ndarray:
        return self.lattice.bonds

    @property
    def bond_t(self) -> np.ndarray:
        return np.full(len(self.lattice.bonds), self.t, dtype=np.float64)

    @property
    def n_params(self) -> int:
        return n_params_of(self.n_sites, self.n_f, self.n_g, self.n_v, self.n_hidden)

    def offsets(self) -> dict:
        """Start of each parameter block inside the instance's vector."""
        ns2 = 2 * self.n_sites
        o = {"f": 0, "g": self.n_f, "v": self.n_f + self.n_g}
        o["a"] = o["v"] + self.n_v
        o["b"] = o["a"] + (ns2 if self.n_hidden else 0)
        o["W"] = o["b"] + self.n_hidden
        o["end"] = o["W"] + self.n_hidden * ns2
        return o


def n_params_of(n_sites: int, n_f: int, n_g: int, n_v: int, n_hidden: int) -> int:
    rbm = (2 * n_sites + n_hidden + n_hidden * 2 * n_sites) if n_hidden else 0
    return n_f + n_g + n_v + rbm


# ----------------------------------------------------------------- index maps
def f_map_full(lat: Lattice) -> tuple[np.ndarray, int]:
    n = lat.n_sites
    return np.arange(n * n, dtype=np.int32).reshape(n, n), n * n


def f_map_sublattice(lat: Lattice, sx: int, sy: int) -> tuple[np.ndarray, int]:
    """f_ij = f(sublattice of i, displacement j - i)."""
    if lat.Lx % sx or lat.Ly % sy:
        raise ValueError("sublattice must divide the lattice")
    n = lat.n_sites
    idx = np.empty((n, n), dtype=np.int32)
    for i in range(n):
        xi, yi = lat.coords[i]
        sub = (xi % sx) + sx * (yi % sy)
        for j in range(n):
            dx, dy = lat.displacement(i, j)
            idx[i, j] = sub * n + dx + lat.Lx * dy
    return idx, sx * sy * n


def translation_projection(lat: Lattice, steps: list[tuple[int, int]],
                           kx: float = 0.0, ky: float = 0.0) -> tuple[np.ndarray, np.ndarray]:
    """Site maps and weights of the translations by the given (dx, dy) steps
    with momentum (kx, ky) in {0, pi}: q_p(i) = site of r_i + R_p, weight
    cos(K . R_p) (real characters only)."""
    n = lat.n_sites
    q = np.empty((len(steps), n), dtype=np.int32)
    w = np.empty(len(steps))
    for p, (dx, dy) in enumerate(steps):
        for i in range(n):
            x, y = lat.coords[i]
            q[p, i] = ((x + dx) % lat.Lx) + lat.Lx * ((y + dy) % lat.Ly)
        w[p] = np.cos(kx * dx + ky * dy)
    w[np.abs(w) < 1e-12] = 0.0
    return q, np.round(w)


def g_map_uniform(lat: Lattice) -> tuple[np.ndarray, int]:
    return np.zeros(lat.n_sites, dtype=np.int32), 1


def v_map_nn(lat: Lattice) -> tuple[np.ndarray, int]:
    n = lat.n_sites
    idx = np.full((n, n), -1, dtype=np.int32)
    for i, j in lat.bonds:
        idx[i, j] = idx[j, i] = 0
    return idx, 1


def v_map_distance(lat: Lattice) -> tuple[np.ndarray, int]:
    """One Jastrow slot per minimum-image distance class (min|d|, max|d|)."""
    n = lat.n_sites
    keys = {}
    for i in range(n):
        for j in range(n):
            if i != j:
                dx, dy = lat.min_image(i, j)
                keys[(min(dx, dy), max(dx, dy))] = None
    order = sorted(keys, key=lambda k: (k[0] ** 2 + k[1] ** 2, k))
    cls = {k: c for c, k in enumerate(order)}
    idx = np.full((n, n), -1, dtype=np.int32)
    for i in range(n):
        for j in range(n):
            if i != j:
                dx, dy = lat.min_image(i, j)
                idx[i, j] = cls[(min(dx, dy), max(dx, dy))]
    return idx, len(order)


# -------------------------------------------------------- initial parameters
def free_orbitals(lat: Lattice, n_occ: int, t: float, rng: np.random.Generator,
                  xi_scale: float = 1e-2) -> np.ndarray:
    """Lowest n_occ eigenvectors of -t*hop + xi_scale*diag(xi), xi ~ N(0,1).

    The small random potential picks one state out of the degenerate open
    shell so that the initial pair amplitudes are fixed by the seed.
    """
    n = lat.n_sites
    h = np.zeros((n, n))
    for i, j in lat.bonds:
        h[i, j] -= t
        h[j, i] -= t
    h += xi_scale * np.diag(rng.standard_normal(n))
    _, vec = np.linalg.eigh(h)
    return vec[:, :n_occ]


def ring8_orbitals() -> np.ndarray:
    """Real U = 0 orbitals of the 8-site ring with 4 electrons per spin.

    k = 0, the cos/sin pair at k = pi/4 and cos at k = pi/2 (which picks one
    member of the degenerate k = +-pi/2 shell).
    """
    r = np.arange(8)
    return np.stack([
        np.full(8, 1 / np.sqrt(8)),
        np.sqrt(2 / 8) * np.cos(2 * np.pi * r / 8),
        np.sqrt(2 / 8) * np.sin(2 * np.pi * r / 8),
        np.sqrt(2 / 8) * np.cos(4 * np.pi * r / 8),
    ], axis=1)


def class_average(f: np.ndarray, f_idx: np.ndarray, n_f: int) -> np.ndarray:
    sums = np.zeros(n_f)
    cnt = np.zeros(n_f)
    m = f_idx >= 0
    np.add.at(sums, f_idx[m], f[m])
    np.add.at(cnt, f_idx[m], 1.0)
    return sums / np.maximum(cnt, 1.0)


def make_instance(name: str, lat: Lattice, n_up: int, n_dn: int, U: float,
                  f_map: tuple, v_map: tuple, *, t: float = 1.0,
                  g0: float = -0.5, v_nn: float = 0.1, n_hidden: int = 0,
                  rbm_sigma: float = 0.01, n_walkers: int = 64,
                  f0: np.ndarray | None = None, f_noise: float = 0.0,
                  seed: int = 11418) -> Instance:
    rng = np.random.default_rng(seed)
    ns = lat.n_sites
    f_idx, n_f = f_map
    v_idx, n_v = v_map
    g_idx, n_g = g_map_uniform(lat)
    if n_up != n_dn:
        raise ValueError("the anti-parallel pair amplitude needs n_up == n_dn")
    if f0 is None:
        phi = free_orbitals(lat, n_up, t, rng)
        f0 = phi @ phi.T
    if f_noise:
        f0 = f0 + f_noise * rng.standard_normal(f0.shape)
    p_f = class_average(f0, f_idx, n_f)
    p_g = np.full(n_g, g0)
    p_v = np.zeros(n_v)
    # nearest-neighbour class(es) start at v_nn, every other distance at 0
    for i, j in lat.bonds:
        if v_idx[i, j] >= 0:
            p_v[v_idx[i, j]] = v_nn
    blocks = [p_f, p_g, p_v]
    if n_hidden:
        nv = 2 * ns
        blocks += [rbm_sigma * rng.standard_normal(nv),
                   rbm_sigma * rng.standard_normal(n_hidden),
                   rbm_sigma * rng.standard_normal(n_hidden * nv)]
    params0 = np.concatenate(blocks).astype(np.float64)
    inst = Instance(name, lat, n_up, n_dn, np.full(ns, float(U)), t,
                    f_idx.astype(np.int32), n_f, g_idx, n_g,
                    v_idx.astype(np.int32), n_v, n_hidden, n_walkers, params0)
    assert inst.n_params == len(params0)
    return inst
