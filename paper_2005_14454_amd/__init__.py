"""MI355X-native Abelian-Higgs lattice evolution (Correia & Martins, section 2).

Python binding of libah.so.  Every step of the path runs in the HIP kernels
behind the C ABI of include/ah.h; this module only marshals arguments.
PyTorch provides device memory (the lattice arena) and the HIP stream.
"""
import ctypes
import math
from dataclasses import dataclass, fields

import numpy as np

from . import _lib
from ._lib import AHError, AH_FP32, AH_FP64, AH_COMPACT, AH_NONCOMPACT, AH_FLAG_NONFINITE, AH_FLAG_UNSTABLE

__all__ = ["Params", "Lattice", "Pool", "AHError", "AH_FP32", "AH_FP64", "AH_COMPACT", "AH_NONCOMPACT",
           "AH_FLAG_NONFINITE", "AH_FLAG_UNSTABLE", "required_bytes", "autotune", "tune_lookup", "tune_set",
           "tune_clear", "tune_save", "tune_load", "pool_footprint", "stability_margin", "read_dump"]


@dataclass
class Params:
    """Lattice and model parameters (section 2 standard choices as defaults).

    precision: "fp64" or "fp32"; gauge_action: "compact" or "noncompact";
    eta_ref <= 0 selects a(dx*N/2) = 1.  damp_gamma > 0 adds an artificial
    damping phase: while eta < eta_damp the friction of the momentum equations
    is the constant damp_gamma instead of the Hubble term."""
    N: int = 64
    precision: str = "fp64"
    gauge_action: str = "compact"
    dx: float = 0.5
    deta: float = 0.1
    lambda0: float = 2.0
    e0: float = 1.0
    sigma: float = 1.0
    m: float = 1.0
    alpha: float = 2.0
    s_early: float = 0.0
    s_late: float = 0.0
    eta_switch: float = math.inf
    eta0: float = 1.0
    eta_ref: float = 0.0
    damp_gamma: float = 0.0
    eta_damp: float = 0.0

    def to_c(self) -> _lib.ah_params:
        c = _lib.ah_params()
        for f in fields(self):
            v = getattr(self, f.name)
            if f.name == "precision":
                v = {"fp64": AH_FP64, "fp32": AH_FP32}[v]
            elif f.name == "gauge_action":
                v = {"compact": AH_COMPACT, "noncompact": AH_NONCOMPACT}[v]
            setattr(c, f.name, v)
        c.reserved = 0
        return c

    @property
    def eta_end(self) -> float:
        return 0.5 * self.dx * self.N


def required_bytes(p: Params) -> int:
    lib = _lib.load()
    n = ctypes.c_size_t()
    _lib.check(lib.ah_required_bytes(ctypes.byref(p.to_c()), ctypes.byref(n)), what="ah_required_bytes")
    return n.value


def stability_margin(p: Params, step: int) -> float:
    """deta * sqrt(max(lambda0, 2 e0^2) f sigma^2 + 12/dx^2) of snapshot `step`; stable below 2."""
    mu = ctypes.c_double()
    _lib.check(_lib.load().ah_stability_margin(ctypes.byref(p.to_c()), step, ctypes.byref(mu)),
               what="ah_stability_margin")
    return mu.value


def _meas_dict(m: _lib.ah_measurement) -> dict:
    return {k: getattr(m, k) for k, _ in _lib.ah_measurement._fields_ if k != "reserved"}


class Lattice:
    """One periodic N^3 lattice resident on the GPU.

    arena="torch": the arena is a torch uint8 tensor owned by this object;
    arena="library": libah hipMallocs and frees it.  stream: a torch.cuda.Stream
    (default: the current stream of the device)."""

    def __init__(self, params: Params, device=None, stream=None, arena: str = "torch"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lattice library has no CPU path")
        lib = _lib.load()
        self.params = params
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._torch = torch
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            cp = params.to_c()
            nbytes = required_bytes(params)
            self._arena = None
            ptr, size = None, 0
            if arena == "torch":
                self._arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
                base = self._arena.data_ptr()
                ptr = (base + 255) // 256 * 256
                size = nbytes
            elif arena != "library":
                raise ValueError("arena must be 'torch' or 'library'")
            h = ctypes.c_void_p()
            _lib.check(lib.ah_create(ctypes.byref(cp), ptr, size, self.stream.cuda_stream, ctypes.byref(h)),
                       what="ah_create")
            self._h = h
        self._lib = lib
        self.N = params.N
        self.V = params.N ** 3

    # -- lifecycle -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            with self._torch.cuda.device(self.device):
                self._lib.ah_destroy(self._h)
            self._h = None
            self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _call(self, fn, *args, what=""):
        with self._torch.cuda.device(self.device):
            _lib.check(fn(self._h, *args), self._h, what)

    # -- evolution -------------------------------------------------------------
    def init(self, seed: int):
        self._call(self._lib.ah_init, ctypes.c_uint64(seed), what="ah_init")

    def step(self, nsteps: int = 1):
        self._call(self._lib.ah_step, nsteps, what="ah_step")

    def measure(self) -> dict:
        m = _lib.ah_measurement()
        self._call(self._lib.ah_measure, ctypes.byref(m), what="ah_measure")
        return _meas_dict(m)

    def step_measured(self, nsteps: int, measure_every: int) -> list:
        """Advance nsteps; snapshots with step % measure_every == 0 that are
        stepped from get their diagnostics in the same pass (list of dicts)."""
        cur = self.step_index
        due = sum(1 for k in range(nsteps) if (cur + k) % measure_every == 0)
        arr = (_lib.ah_measurement * max(due, 1))()
        n = ctypes.c_int32()
        self._call(self._lib.ah_step_measured, nsteps, measure_every, arr, due, ctypes.byref(n),
                   what="ah_step_measured")
        return [_meas_dict(arr[k]) for k in range(n.value)]

    def synchronize(self):
        self._call(self._lib.ah_synchronize, what="ah_synchronize")

    @property
    def step_index(self) -> int:
        s = ctypes.c_int64()
        _lib.check(self._lib.ah_get_step(self._h, ctypes.byref(s)))
        return s.value

    # -- state I/O -------------------------------------------------------------
    def set_state(self, state: np.ndarray, step: int = 0):
        st = np.ascontiguousarray(state, dtype=np.float64)
        if st.size != 10 * self.V:
            raise ValueError(f"state has {st.size} values, expected {10 * self.V}")
        self._call(self._lib.ah_set_state, st.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), step,
                   what="ah_set_state")

    def get_state(self) -> np.ndarray:
        st = np.empty((10, self.V), dtype=np.float64)
        s = ctypes.c_int64()
        self._call(self._lib.ah_get_state, st.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(s),
                   what="ah_get_state")
        return st

    def gather(self, sites) -> np.ndarray:
        """(len(sites), 10) FP64 values of the current snapshot at the listed site indices."""
        s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
        out = np.empty((len(s), 10), dtype=np.float64)
        self._call(self._lib.ah_gather, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(s),
                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), what="ah_gather")
        return out

    def gather_noalloc(self, sites) -> np.ndarray:
        """As gather(), staged in the library's fixed device scratch (no device
        allocation; at most 65536 sites per call)."""
        s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
        out = np.empty((len(s), 10), dtype=np.float64)
        self._call(self._lib.ah_gather_noalloc, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(s),
                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), what="ah_gather_noalloc")
        return out

    def winding(self) -> np.ndarray:
        w = np.empty((3, self.V), dtype=np.int8)
        self._call(self._lib.ah_get_winding, w.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), what="ah_get_winding")
        return w

    def dump(self, path: str, windings: bool = True):
        """Write the current snapshot to `path` (.npz): step index, parameters,
        the ten fields in the lattice's storage precision (so the snapshot
        comes back exactly through `restore`) and the plaquette windings W_ij
        (int8, orientations xy, xz, yz; site index x0 + N (x1 + N x2))."""
        import json
        from dataclasses import asdict
        st = self.get_state()
        out = {"step": np.int64(self.step_index), "params": np.array(json.dumps(asdict(self.params))),
               "fields": st.astype(np.float32) if self.params.precision == "fp32" else st}
        if windings:
            out["windings"] = self.winding()
        np.savez_compressed(path, **out)

    def restore(self, path: str):
        """Load the snapshot of a dump written by `dump` for the same N."""
        d = read_dump(path)
        if d["params"].N != self.N:
            raise ValueError(f"dump is for N = {d['params'].N}, this lattice has N = {self.N}")
        self.set_state(d["fields"].astype(np.float64), d["step"])

    # -- kernel choice ---------------------------------------------------------
    def set_step_config(self, kernel="auto", tile=(0, 0), zchunk=0):
        """kernel: "auto", "site", "tile" or "tile2" (two steps per pass); tile: (tile_x, tile_y);
        zchunk: planes per workgroup."""
        k = {"auto": _lib.AH_KERNEL_AUTO, "site": _lib.AH_KERNEL_SITE, "tile": _lib.AH_KERNEL_TILE,
             "tile2": _lib.AH_KERNEL_TILE2}[kernel]
        c = _lib.ah_step_config(k, tile[0], tile[1], zchunk)
        self._call(self._lib.ah_set_step_config, ctypes.byref(c), what="ah_set_step_config")

    def get_step_config(self) -> dict:
        c = _lib.ah_step_config()
        _lib.check(self._lib.ah_get_step_config(self._h, ctypes.byref(c)))
        name = {_lib.AH_KERNEL_SITE: "site", _lib.AH_KERNEL_TILE: "tile",
                _lib.AH_KERNEL_TILE2: "tile2"}.get(c.kernel, "auto")
        return {"kernel": name, "tile": (c.tile_x, c.tile_y), "zchunk": c.zchunk}

    # -- timing ----------------------------------------------------------------
    def set_timing(self, enable: bool):
        self._call(self._lib.ah_set_timing, 1 if enable else 0, what="ah_set_timing")

    def get_timing(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._call(self._lib.ah_get_timing, ctypes.byref(ms), ctypes.byref(n), what="ah_get_timing")
        return ms.value, n.value

    def get_timing_split(self):
        """(ms, launches) of the timed launches that also formed diagnostics."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._call(self._lib.ah_get_timing_split, ctypes.byref(ms), ctypes.byref(n), what="ah_get_timing_split")
        return ms.value, n.value


def read_dump(path: str) -> dict:
    """Contents of a lattice dump: step, params (Params), fields (10, N^3) and,
    if written, windings (3, N^3).  Plain arrays only; nothing is unpickled."""
    import json
    with np.load(path, allow_pickle=False) as z:
        d = {"step": int(z["step"]), "params": Params(**json.loads(str(z["params"]))), "fields": z["fields"]}
        if "windings" in z.files:
            d["windings"] = z["windings"]
    return d


# ----------------------------------------------------------------- autotuner

def _cfg_dict(c) -> dict:
    return {"kernel": {_lib.AH_KERNEL_SITE: "site", _lib.AH_KERNEL_TILE: "tile",
                       _lib.AH_KERNEL_TILE2: "tile2"}.get(c.kernel, "auto"),
            "tile": (c.tile_x, c.tile_y), "zchunk": c.zchunk}


def autotune(p: Params, steps: int = 5) -> dict:
    """Time the tiled step's tile shapes and z-chunks for (precision, N); record the best."""
    import torch
    lib = _lib.load()
    best = _lib.ah_step_config()
    ms = ctypes.c_double()
    with torch.cuda.device(torch.cuda.current_device()):
        _lib.check(lib.ah_autotune(ctypes.byref(p.to_c()), steps, ctypes.byref(best), ctypes.byref(ms)),
                   what="ah_autotune")
    d = _cfg_dict(best)
    d["ms"] = ms.value
    return d


def tune_lookup(p: Params):
    lib = _lib.load()
    c = _lib.ah_step_config()
    rc = lib.ah_tune_lookup(ctypes.byref(p.to_c()), ctypes.byref(c))
    if rc == _lib.AH_E_AGAIN:
        return None
    _lib.check(rc, what="ah_tune_lookup")
    return _cfg_dict(c)


def tune_set(p: Params, tile, zchunk: int = 0, kernel: str = "tile"):
    """Record a tiling by hand; kernel "tile" (one step per pass) or "tile2" (two)."""
    lib = _lib.load()
    k = {"tile": _lib.AH_KERNEL_TILE, "tile2": _lib.AH_KERNEL_TILE2}[kernel]
    c = _lib.ah_step_config(k, tile[0], tile[1], zchunk)
    _lib.check(lib.ah_tune_set(ctypes.byref(p.to_c()), ctypes.byref(c)), what="ah_tune_set")


def tune_clear():
    _lib.check(_lib.load().ah_tune_clear(), what="ah_tune_clear")


def tune_save(path: str):
    _lib.check(_lib.load().ah_tune_save(path.encode()), what="ah_tune_save")


def tune_load(path: str):
    _lib.check(_lib.load().ah_tune_load(path.encode()), what="ah_tune_load")


def hbm_probe(nbytes: int = 4 << 30, reps: int = 5) -> dict:
    """Achievable HBM bandwidth of the current device (GB/s): streaming copy,
    read-only and write-only kernels over two buffers of nbytes."""
    import torch
    lib = _lib.load()
    c, r, w = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    with torch.cuda.device(torch.cuda.current_device()):
        _lib.check(lib.ah_hbm_probe(nbytes, reps, ctypes.byref(c), ctypes.byref(r), ctypes.byref(w)),
                   what="ah_hbm_probe")
    return {"bytes": nbytes, "copy_GB/s": c.value, "read_GB/s": r.value, "write_GB/s": w.value}


def pool_footprint(p: Params, nsteps: int, measure_every: int) -> int:
    n = ctypes.c_size_t()
    _lib.check(_lib.load().ah_pool_footprint(ctypes.byref(p.to_c()), nsteps, measure_every, ctypes.byref(n)),
               what="ah_pool_footprint")
    return n.value


# ---------------------------------------------------------------------- pool

class Pool:
    """Many lattices resident in one HBM arena, advanced together (one graph
    replay per step).  submit() returns None when the request does not fit now."""

    def __init__(self, hbm_budget: int, max_slots: int = 256, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lattice library has no CPU path")
        self._torch = torch
        self._lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self._lib.ah_pool_create(hbm_budget, max_slots, None, ctypes.byref(h)), what="ah_pool_create")
        self._h = h
        self.max_slots = max_slots
        self._req = {}  # id -> (params, nsteps, measure_every) of the lattices in the pool

    def _call(self, fn, *args, what=""):
        with self._torch.cuda.device(self.device):
            rc = fn(self._h, *args)
        _lib.check(rc, what=what, pool=self._h)

    def close(self):
        if getattr(self, "_h", None):
            with self._torch.cuda.device(self.device):
                self._lib.ah_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, p: Params, seed: int, nsteps: int, measure_every: int = 0):
        rid = ctypes.c_int64()
        with self._torch.cuda.device(self.device):
            rc = self._lib.ah_pool_submit(self._h, ctypes.byref(p.to_c()), ctypes.c_uint64(seed), nsteps,
                                          measure_every, ctypes.byref(rid))
        if rc == _lib.AH_E_AGAIN:
            return None
        _lib.check(rc, what="ah_pool_submit", pool=self._h)
        self._req[rid.value] = (p, nsteps, measure_every)
        return rid.value

    def advance(self, nsteps: int = 1):
        self._call(self._lib.ah_pool_advance, nsteps, what="ah_pool_advance")

    def poll(self, cap: int = 4096):
        ids = (ctypes.c_int64 * cap)()
        n = ctypes.c_int32()
        self._call(self._lib.ah_pool_poll, ids, cap, ctypes.byref(n), what="ah_pool_poll")
        return [ids[k] for k in range(n.value)]

    def poll_async(self, cap: int = 4096):
        """Finished lattices the newest counter copy on the host shows (no wait)."""
        ids = (ctypes.c_int64 * cap)()
        n = ctypes.c_int32()
        self._call(self._lib.ah_pool_poll_async, ids, cap, ctypes.byref(n), what="ah_pool_poll_async")
        return [ids[k] for k in range(n.value)]

    def step_config(self, rid: int) -> dict:
        """Tile shape and z-chunk lattice rid is stepped with."""
        c = _lib.ah_step_config()
        _lib.check(self._lib.ah_pool_step_config(self._h, rid, ctypes.byref(c)), what="ah_pool_step_config",
                   pool=self._h)
        return _cfg_dict(c)

    def progress(self, rid: int):
        s, n = ctypes.c_int64(), ctypes.c_int64()
        self._call(self._lib.ah_pool_progress, rid, ctypes.byref(s), ctypes.byref(n), what="ah_pool_progress")
        return s.value, n.value

    def get_state(self, rid: int, N: int = None) -> np.ndarray:
        """Fields of lattice rid at its current step; the buffer is sized from
        the lattice's own N (a given N must match it)."""
        if rid not in self._req:
            raise KeyError(f"no lattice {rid} in the pool")
        n_own = self._req[rid][0].N
        if N is not None and N != n_own:
            raise ValueError(f"lattice {rid} has N = {n_own}, not {N}")
        st = np.empty((10, n_own ** 3), dtype=np.float64)
        s = ctypes.c_int64()
        self._call(self._lib.ah_pool_get_state, rid, st.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   ctypes.byref(s), what="ah_pool_get_state")
        return st

    def results(self, rid: int):
        """Diagnostics series of a finished lattice; frees its slot."""
        _, nsteps, every = self._req.get(rid, (None, 0, 0))
        cap = (nsteps // every + 1 if every > 0 else 0) + 1
        arr = (_lib.ah_measurement * cap)()
        n = ctypes.c_int32()
        self._call(self._lib.ah_pool_results, rid, arr, cap, ctypes.byref(n), what="ah_pool_results")
        self._req.pop(rid, None)
        return [_meas_dict(arr[k]) for k in range(n.value)]

    def stats(self) -> dict:
        info = _lib.ah_pool_info()
        _lib.check(self._lib.ah_pool_stats(self._h, ctypes.byref(info)), what="ah_pool_stats")
        return {k: getattr(info, k) for k, _ in _lib.ah_pool_info._fields_}

    def synchronize(self):
        self._call(self._lib.ah_pool_synchronize, what="ah_pool_synchronize")
