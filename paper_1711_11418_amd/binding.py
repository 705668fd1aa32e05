"""Thin Python binding over libmvmc.so (ctypes; argument marshalling only).

PyTorch provides device memory and the stream; every step of the hot path
runs in the library's HIP kernels.  The library must be built
(``python -m paper_1711_11418_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmvmc.so")

MVMC_FP64, MVMC_MIXED = 0, 1
MVMC_SOLVE_CHOL, MVMC_SOLVE_CG = 0, 1

ENTRY_POINTS = (
    "mvmc_query_sizes", "mvmc_query_layout", "mvmc_init_wavefunction", "mvmc_sample_sweeps",
    "mvmc_measure_energy_and_O", "mvmc_build_sr", "mvmc_sr_update", "mvmc_set_params",
    "mvmc_get_state", "mvmc_set_state", "mvmc_get_inverse", "mvmc_get_pfaffian", "mvmc_refresh",
    "mvmc_trace_enable", "mvmc_timing", "mvmc_destroy", "mvmc_last_error", "mvmc_status_string",
    "mvmc_autotune", "mvmc_sweep_variants", "mvmc_s_tiles", "mvmc_set_s_tile",
    "mvmc_peak_probe_bytes", "mvmc_peak_probe", "mvmc_init_wavefunction_static",
    "mvmc_measure_h2", "mvmc_lanczos_first_step",
)
N_SWEEP_VARIANTS = 10
SWEEP_VARIANT_NAMES = ("reg", "lds64", "lds128", "lds256", "hbm64", "hbm128", "hbm256",
                       "ap64", "ap128", "ap256")
PROJ_VARIANT = "proj"   # reported for instances with a quantum-number projection
SCHEDULES = ("buckets", "queue")   # MVMC_SCHED_BUCKETS, MVMC_SCHED_QUEUE
REFRESH_UNITS = ("proposals", "updates")   # MVMC_REFRESH_PROPOSALS, MVMC_REFRESH_UPDATES


class InstanceDesc(C.Structure):
    _fields_ = [
        ("n_sites", C.c_int32), ("n_up", C.c_int32), ("n_dn", C.c_int32), ("n_bonds", C.c_int32),
        ("bond_i", C.POINTER(C.c_int32)), ("bond_j", C.POINTER(C.c_int32)),
        ("bond_t", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double)),
        ("n_f", C.c_int32), ("f_idx", C.POINTER(C.c_int32)),
        ("n_g", C.c_int32), ("g_idx", C.POINTER(C.c_int32)),
        ("n_v", C.c_int32), ("v_idx", C.POINTER(C.c_int32)),
        ("n_hidden", C.c_int32), ("n_walkers", C.c_int32),
        ("n_proj", C.c_int32), ("proj_map", C.POINTER(C.c_int32)),
        ("proj_weight", C.POINTER(C.c_double)),
    ]


class Config(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("refresh_every", C.c_int32), ("seed", C.c_uint64),
        ("n_instances", C.c_int32), ("inst", C.POINTER(InstanceDesc)),
        ("n_slots", C.c_int32), ("solver", C.c_int32), ("build_s", C.c_int32),
        ("sweep_threads", C.c_int32), ("sweep_variant", C.c_int32),
        ("exchange_per64", C.c_int32), ("schedule", C.c_int32), ("refresh_unit", C.c_int32),
    ]


class Sizes(C.Structure):
    _fields_ = [
        ("n_walkers", C.c_int64), ("n_params", C.c_int64), ("eloc_elems", C.c_int64),
        ("O_elems", C.c_int64), ("S_elems", C.c_int64), ("Y_elems", C.c_int64),
        ("pos_elems", C.c_int64), ("empty_elems", C.c_int64),
        ("workspace_bytes", C.c_int64), ("O_elem_bytes", C.c_int32), ("pad", C.c_int32),
    ]


class Layout(C.Structure):
    _fields_ = [
        ("walker_off", C.c_int64), ("n_walkers", C.c_int64), ("param_off", C.c_int64),
        ("n_params", C.c_int64), ("eloc_off", C.c_int64), ("O_off", C.c_int64),
        ("O_ld", C.c_int64), ("S_off", C.c_int64), ("Y_off", C.c_int64), ("pos_off", C.c_int64),
        ("empty_off", C.c_int64), ("n_elec", C.c_int32), ("n_sites", C.c_int32),
        ("Y_ld", C.c_int64),
    ]


TRACE_DTYPE = np.dtype([("n", "<i8"), ("walker", "<i4"), ("a", "<i4"), ("i_new", "<i4"),
                        ("accepted", "<i4"), ("ratio", "<f8"), ("b", "<i4"), ("pad", "<i4")])

_lib = None


class MVMCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mvmc status {status}: {msg}")
        self.status = status


def load() -> C.CDLL:
    """Load libmvmc.so; raises when it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1711_11418_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "mvmc_query_sizes": [C.POINTER(Config), C.POINTER(Sizes)],
        "mvmc_query_layout": [C.POINTER(Config), i32, C.POINTER(Layout)],
        "mvmc_init_wavefunction": [C.POINTER(vp), C.POINTER(Config), vp, C.c_size_t, vp, vp],
        "mvmc_init_wavefunction_static": [C.POINTER(vp), C.POINTER(Config), vp, vp],
        "mvmc_sample_sweeps": [vp, i32, vp],
        "mvmc_measure_energy_and_O": [vp, i32, vp, vp],
        "mvmc_measure_h2": [vp, i32, vp, vp],
        "mvmc_lanczos_first_step": [vp, i32, vp, vp, vp],
        "mvmc_build_sr": [vp, i32, vp, vp, vp, vp, vp, vp, vp],
        "mvmc_sr_update": [vp, vp, vp, vp, dbl, dbl, dbl, i32, dbl, i32, vp, vp, vp],
        "mvmc_set_params": [vp, vp],
        "mvmc_get_state": [vp, vp, vp, vp],
        "mvmc_set_state": [vp, vp, vp, vp],
        "mvmc_get_inverse": [vp, vp],
        "mvmc_get_pfaffian": [vp, vp, vp],
        "mvmc_refresh": [vp],
        "mvmc_trace_enable": [vp, vp, i64],
        "mvmc_timing": [vp, i32, vp, vp],
        "mvmc_destroy": [vp],
        "mvmc_autotune": [vp, i32, C.c_char_p, vp],
        "mvmc_sweep_variants": [vp, vp],
        "mvmc_s_tiles": [vp, vp, vp],
        "mvmc_set_s_tile": [vp, C.c_int32],
        "mvmc_peak_probe_bytes": [],
        "mvmc_peak_probe": [C.c_int32, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.mvmc_peak_probe_bytes.restype = C.c_size_t
    lib.mvmc_last_error.argtypes = [vp]
    lib.mvmc_last_error.restype = C.c_char_p
    lib.mvmc_status_string.argtypes = [C.c_int]
    lib.mvmc_status_string.restype = C.c_char_p
    _lib = lib
    return lib


PEAK_PROBES = ("bf16_mfma", "fp64_mfma", "fp64_fma")


def peak_probe(kind: str) -> float:
    """Attainable TFLOP/s of one instruction class on this GPU
    (mvmc_peak_probe): "bf16_mfma", "fp64_mfma" or "fp64_fma"."""
    import torch
    lib = load()
    buf = torch.empty(int(lib.mvmc_peak_probe_bytes()), dtype=torch.uint8, device="cuda")
    out = C.c_double(0.0)
    stream = torch.cuda.current_stream().cuda_stream
    rc = lib.mvmc_peak_probe(PEAK_PROBES.index(kind), C.c_void_p(buf.data_ptr()),
                             C.c_void_p(stream), C.byref(out))
    if rc != 0:
        raise MVMCError(rc, lib.mvmc_status_string(rc).decode())
    return out.value


class _Desc:
    """Holds the numpy arrays a descriptor points to (kept alive with it)."""

    def __init__(self, inst):
        bonds = np.ascontiguousarray(np.asarray(inst.bonds, dtype=np.int32))
        self.bi = np.ascontiguousarray(bonds[:, 0])
        self.bj = np.ascontiguousarray(bonds[:, 1])
        self.bt = np.ascontiguousarray(np.asarray(inst.bond_t, dtype=np.float64))
        self.U = np.ascontiguousarray(np.asarray(inst.U, dtype=np.float64))
        self.f = np.ascontiguousarray(np.asarray(inst.f_idx, dtype=np.int32).ravel())
        self.g = np.ascontiguousarray(np.asarray(inst.g_idx, dtype=np.int32).ravel())
        self.v = np.ascontiguousarray(np.asarray(inst.v_idx, dtype=np.int32).ravel())
        p32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        p64 = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        pq = getattr(inst, "proj_q", None)
        pw = getattr(inst, "proj_w", None)
        if pq is None:
            self.pq = np.zeros(1, dtype=np.int32)
            self.pw = np.zeros(1, dtype=np.float64)
            n_proj = 0
        else:
            self.pq = np.ascontiguousarray(np.asarray(pq, dtype=np.int32).reshape(-1))
            self.pw = np.ascontiguousarray(np.asarray(pw, dtype=np.float64).reshape(-1))
            n_proj = len(self.pw)
        self.desc = InstanceDesc(int(inst.n_sites), int(inst.n_up), int(inst.n_dn), len(self.bi),
                                 p32(self.bi), p32(self.bj), p64(self.bt), p64(self.U),
                                 int(inst.n_f), p32(self.f), int(inst.n_g), p32(self.g),
                                 int(inst.n_v), p32(self.v), int(inst.n_hidden),
                                 int(inst.n_walkers), n_proj, p32(self.pq), p64(self.pw))


def make_config(instances, precision="fp64", refresh_every=0, seed=1, n_slots=1, solver="chol",
                build_s=True, sweep_threads=0, sweep_variant=None, exchange_per64=0,
                schedule="buckets", refresh_unit="proposals"):
    """sweep_variant: None (automatic) or a name of SWEEP_VARIANT_NAMES forced for
    every instance.  schedule: "buckets" (one launch per variant bucket) or
    "queue" (one persistent launch per call).  refresh_unit: what refresh_every
    counts, "proposals" or "updates" (accepted moves)."""
    descs = [_Desc(i) for i in instances]
    arr = (InstanceDesc * len(descs))(*[d.desc for d in descs])
    cfg = Config(MVMC_FP64 if precision == "fp64" else MVMC_MIXED, int(refresh_every),
                 int(seed), len(descs), C.cast(arr, C.POINTER(InstanceDesc)), int(n_slots),
                 MVMC_SOLVE_CHOL if solver == "chol" else MVMC_SOLVE_CG, int(bool(build_s)),
                 int(sweep_threads),
                 0 if sweep_variant is None else 1 + SWEEP_VARIANT_NAMES.index(sweep_variant),
                 int(exchange_per64), SCHEDULES.index(schedule),
                 REFRESH_UNITS.index(refresh_unit))
    cfg._keep = (descs, arr)   # keep host arrays alive
    return cfg


def query_sizes(cfg) -> Sizes:
    lib = load()
    s = Sizes()
    rc = lib.mvmc_query_sizes(C.byref(cfg), C.byref(s))
    if rc:
        raise MVMCError(rc, lib.mvmc_status_string(rc).decode())
    return s


def query_layout(cfg, k: int) -> Layout:
    lib = load()
    lay = Layout()
    rc = lib.mvmc_query_layout(C.byref(cfg), k, C.byref(lay))
    if rc:
        raise MVMCError(rc, lib.mvmc_status_string(rc).decode())
    return lay


class MVMC:
    """One library context plus the torch buffers it works on."""

    def __init__(self, instances, params, *, precision="fp64", refresh_every=0, seed=1,
                 n_slots=1, solver="chol", build_s=True, sweep_threads=0, sweep_variant=None,
                 exchange_per64=0, schedule="buckets", device="cuda:0", stream=None,
                 static_workspace=False, refresh_unit="proposals"):
        """stream: torch.cuda.Stream for all of the context's work (default: the
        current stream).  A non-default stream is needed for graph capture.
        static_workspace: take the workspace from the library's static device
        array (mvmc_init_wavefunction_static) instead of allocating it.
        refresh_unit: what refresh_every counts, "proposals" or "updates"."""
        import torch
        self.torch = torch
        self.lib = load()
        self.device = torch.device(device)
        self.instances = list(instances)
        self.precision = precision
        self.cfg = make_config(self.instances, precision, refresh_every, seed, n_slots, solver,
                               build_s, sweep_threads, sweep_variant, exchange_per64, schedule,
                               refresh_unit)
        self.sizes = query_sizes(self.cfg)
        self.layouts = [query_layout(self.cfg, k) for k in range(len(self.instances))]
        self.n_inst = len(self.instances)
        odt = torch.float64 if precision == "fp64" else torch.float32
        dev = self.device
        if static_workspace:
            self.ws = None
        else:
            self.ws = torch.empty(int(self.sizes.workspace_bytes) + 256, dtype=torch.uint8,
                                  device=dev)
            self._ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float64)).to(dev).contiguous()
        assert self.params.numel() == self.sizes.n_params
        self.eloc = torch.zeros(int(self.sizes.eloc_elems), dtype=torch.float64, device=dev)
        self.O = torch.zeros(int(self.sizes.O_elems), dtype=odt, device=dev)
        self.S = (torch.zeros(int(self.sizes.S_elems), dtype=odt, device=dev)
                  if build_s else None)
        self.g = torch.zeros(int(self.sizes.n_params), dtype=torch.float64, device=dev)
        self.dparams = torch.zeros_like(self.g)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.ctx = C.c_void_p()
        if static_workspace:
            rc = self.lib.mvmc_init_wavefunction_static(C.byref(self.ctx), C.byref(self.cfg),
                                                        C.c_void_p(self.params.data_ptr()),
                                                        C.c_void_p(self.stream.cuda_stream))
        else:
            rc = self.lib.mvmc_init_wavefunction(C.byref(self.ctx), C.byref(self.cfg),
                                                 C.c_void_p(self._ws_ptr),
                                                 int(self.sizes.workspace_bytes),
                                                 C.c_void_p(self.params.data_ptr()),
                                                 C.c_void_p(self.stream.cuda_stream))
        if rc:
            raise MVMCError(rc, self.lib.mvmc_status_string(rc).decode())
        self._trace = None

    # ------------------------------------------------------------ helpers
    def _check(self, rc):
        if rc:
            msg = self.lib.mvmc_last_error(self.ctx).decode()
            raise MVMCError(rc, msg or self.lib.mvmc_status_string(rc).decode())

    @staticmethod
    def _p(t):
        return None if t is None else C.c_void_p(t.data_ptr())

    def close(self):
        if self.ctx:
            self.lib.mvmc_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------- hot path
    def sample(self, n_sweeps: int) -> np.ndarray:
        """n_sweeps sweeps; returns the accepted proposals per instance since
        the last call that returned them (and clears the counters)."""
        acc = np.zeros(self.n_inst, dtype=np.int64)
        self._check(self.lib.mvmc_sample_sweeps(self.ctx, int(n_sweeps),
                                                acc.ctypes.data_as(C.c_void_p)))
        return acc

    def sample_async(self, n_sweeps: int) -> None:
        self._check(self.lib.mvmc_sample_sweeps(self.ctx, int(n_sweeps), None))

    def capture_sampling(self, n_sweeps: int, slots):
        """HIP graph of [n_sweeps sweeps, measurement into slot s] for s in slots,
        captured on the context's stream (which must not be the default stream)."""
        g = self.torch.cuda.CUDAGraph()
        with self.torch.cuda.graph(g, stream=self.stream):
            for s in slots:
                self.sample_async(n_sweeps)
                self.measure(s)
        return g

    def measure(self, slot: int) -> None:
        self._check(self.lib.mvmc_measure_energy_and_O(self.ctx, int(slot), self._p(self.eloc),
                                                       self._p(self.O)))

    def measure_h2(self, slot: int) -> None:
        """F(x, H) and F(x, H^2) of every walker into slot `slot` of self.f1 /
        self.f2 (first-step power-Lanczos, allocated on first use)."""
        t = self.torch
        if getattr(self, "f1", None) is None:
            self.f1 = t.zeros(int(self.sizes.eloc_elems), dtype=t.float64, device=self.device)
            self.f2 = t.zeros_like(self.f1)
        self._check(self.lib.mvmc_measure_h2(self.ctx, int(slot), self._p(self.f1),
                                             self._p(self.f2)))

    def lanczos_first_step(self, n_used: int) -> np.ndarray:
        """[n_instances][7]: h1, h11, h20, h12, alpha_1, E_1(alpha_1), real roots."""
        out = np.zeros((self.n_inst, 7))
        self._check(self.lib.mvmc_lanczos_first_step(self.ctx, int(n_used), self._p(self.f1),
                                                     self._p(self.f2),
                                                     out.ctypes.data_as(C.c_void_p)))
        return out

    def build_sr(self, n_used: int, with_S: bool = True):
        """SR statistics over the first n_used slots; returns (E_bar, sigma, var E)
        per instance, sigma = std(walker means)/sqrt(W)."""
        E = np.zeros(self.n_inst)
        Er = np.zeros(self.n_inst)
        V = np.zeros(self.n_inst)
        S = self.S if with_S else None
        self._check(self.lib.mvmc_build_sr(self.ctx, int(n_used), self._p(self.eloc),
                                           self._p(self.O), self._p(S), self._p(self.g),
                                           E.ctypes.data_as(C.c_void_p),
                                           Er.ctypes.data_as(C.c_void_p),
                                           V.ctypes.data_as(C.c_void_p)))
        return E, Er, V

    def sr_update(self, dtau=0.02, eps_rel=1e-3, eps_abs=1e-6, solver="chol", cg_tol=1e-10,
                  cg_maxit=1000) -> np.ndarray:
        it = np.zeros(self.n_inst, dtype=np.int32)
        sv = MVMC_SOLVE_CHOL if solver == "chol" else MVMC_SOLVE_CG
        self._check(self.lib.mvmc_sr_update(self.ctx, self._p(self.S), self._p(self.O),
                                            self._p(self.g), float(dtau), float(eps_rel),
                                            float(eps_abs), sv, float(cg_tol), int(cg_maxit),
                                            self._p(self.params), self._p(self.dparams),
                                            it.ctypes.data_as(C.c_void_p)))
        return it

    def set_params(self, params) -> None:
        t = self.torch
        self.params.copy_(t.as_tensor(np.asarray(params, dtype=np.float64)))
        self._check(self.lib.mvmc_set_params(self.ctx, self._p(self.params)))

    # ------------------------------------------------------ state / debug
    def get_state(self, with_empty: bool = False):
        """(configurations int16, counters int64[, empty-site lists int16]) on the device."""
        t = self.torch
        pos = t.empty(int(self.sizes.pos_elems), dtype=t.int16, device=self.device)
        cnt = t.empty(int(self.sizes.n_walkers), dtype=t.int64, device=self.device)
        emp = (t.empty(int(self.sizes.empty_elems), dtype=t.int16, device=self.device)
               if with_empty else None)
        self._check(self.lib.mvmc_get_state(self.ctx, self._p(pos), self._p(cnt), self._p(emp)))
        return (pos, cnt, emp) if with_empty else (pos, cnt)

    def set_state(self, pos, cnt, empty=None) -> None:
        t = self.torch
        pos = t.as_tensor(np.asarray(pos, dtype=np.int16)).to(self.device).contiguous()
        cnt = t.as_tensor(np.asarray(cnt, dtype=np.int64)).to(self.device).contiguous()
        emp = (None if empty is None else
               t.as_tensor(np.asarray(empty, dtype=np.int16)).to(self.device).contiguous())
        self._check(self.lib.mvmc_set_state(self.ctx, self._p(pos), self._p(cnt), self._p(emp)))

    def get_inverse(self):
        t = self.torch
        y = t.empty(int(self.sizes.Y_elems), dtype=t.float64, device=self.device)
        self._check(self.lib.mvmc_get_inverse(self.ctx, self._p(y)))
        return y

    def get_pfaffian(self):
        t = self.torch
        la = t.empty(int(self.sizes.n_walkers), dtype=t.float64, device=self.device)
        sg = t.empty_like(la)
        self._check(self.lib.mvmc_get_pfaffian(self.ctx, self._p(la), self._p(sg)))
        return la, sg

    def refresh(self) -> None:
        self._check(self.lib.mvmc_refresh(self.ctx))

    def enable_trace(self, per_walker: int) -> None:
        t = self.torch
        self._trace = t.zeros(int(self.sizes.n_walkers) * per_walker * TRACE_DTYPE.itemsize,
                              dtype=t.uint8, device=self.device)
        self._trace_cap = per_walker
        self._check(self.lib.mvmc_trace_enable(self.ctx, self._p(self._trace), per_walker))

    def disable_trace(self) -> None:
        self._check(self.lib.mvmc_trace_enable(self.ctx, None, 0))

    def trace_records(self) -> np.ndarray:
        raw = self._trace.cpu().numpy().view(TRACE_DTYPE)
        return raw.reshape(int(self.sizes.n_walkers), self._trace_cap)

    def autotune(self, n_sweeps: int = 3, cache_path: str | None = None) -> np.ndarray:
        """Time every sweep variant per instance and keep the fastest
        (mvmc_autotune); returns [n_instances, 7] milliseconds (NaN = not timed)."""
        ms = np.full((self.n_inst, N_SWEEP_VARIANTS), np.nan)
        path = None if cache_path is None else str(cache_path).encode()
        self._check(self.lib.mvmc_autotune(self.ctx, int(n_sweeps), path,
                                           ms.ctypes.data_as(C.c_void_p)))
        return ms

    def s_tiles(self) -> tuple[list[int], np.ndarray]:
        """Tile side of the split-bf16 S build per instance (0: 64-tile
        kernel) and the milliseconds of the last tuning at sides 128, 192,
        256 ([n_instances, 3], NaN where not timed)."""
        n = self.n_inst
        t = np.zeros(n, np.int32)
        ms = np.zeros((n, 3), np.float64)
        self._check(self.lib.mvmc_s_tiles(self.ctx, t.ctypes.data_as(C.c_void_p),
                                          ms.ctypes.data_as(C.c_void_p)))
        return [int(x) for x in t], ms

    def set_s_tile(self, side: int) -> None:
        """Force the split-bf16 S tile side (128, 192 or 256) of the wide instances."""
        self._check(self.lib.mvmc_set_s_tile(self.ctx, int(side)))

    def sweep_variants(self) -> list[str]:
        v = np.zeros(self.n_inst, dtype=np.int32)
        self._check(self.lib.mvmc_sweep_variants(self.ctx, v.ctypes.data_as(C.c_void_p)))
        return [(SWEEP_VARIANT_NAMES + (PROJ_VARIANT,))[i] for i in v]

    def timing(self, enable: bool):
        ms = np.zeros(6)
        calls = np.zeros(6, dtype=np.int64)
        self._check(self.lib.mvmc_timing(self.ctx, int(enable), ms.ctypes.data_as(C.c_void_p),
                                         calls.ctypes.data_as(C.c_void_p)))
        return ms, calls

    # ------------------------------------------------------ views per instance
    def eloc_of(self, k: int, n_used: int):
        l = self.layouts[k]
        return self.eloc[l.eloc_off:l.eloc_off + n_used * l.n_walkers]

    def O_of(self, k: int, n_used: int):
        l = self.layouts[k]
        rows = n_used * l.n_walkers
        return self.O[l.O_off:l.O_off + rows * l.O_ld].view(rows, l.O_ld)[:, :l.n_params]

    def S_of(self, k: int):
        l = self.layouts[k]
        n = l.n_params
        return self.S[l.S_off:l.S_off + n * n].view(n, n)

    def params_of(self, k: int, t=None):
        l = self.layouts[k]
        t = self.params if t is None else t
        return t[l.param_off:l.param_off + l.n_params]

    def pos_of(self, pos, k: int):
        l = self.layouts[k]
        return pos[l.pos_off:l.pos_off + l.n_walkers * l.n_elec].view(l.n_walkers, l.n_elec)

    def Y_of(self, Y, k: int):
        l = self.layouts[k]
        ne = l.n_elec
        rows = Y[l.Y_off:l.Y_off + l.n_walkers * l.Y_ld].view(l.n_walkers, l.Y_ld)
        return rows[:, :ne * ne].reshape(l.n_walkers, ne, ne)

    def proj_inverses_of(self, Y, k: int, n_proj: int):
        """[walkers, N_P, n, n] view of a projected instance's M_p^-1 blocks
        (entry [b][a]: down electron b, up electron a)."""
        l = self.layouts[k]
        n = l.n_elec // 2
        rows = Y[l.Y_off:l.Y_off + l.n_walkers * l.Y_ld].view(l.n_walkers, l.Y_ld)
        return rows[:, :n_proj * n * n].reshape(l.n_walkers, n_proj, n, n)
