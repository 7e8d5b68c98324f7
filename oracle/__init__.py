"""Plain FP64 CPU oracle for the Abelian-Higgs leapfrog step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  The GPU library never imports, links or runs this
package; only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the GPU library.

It follows section 2 of Correia & Martins, "Abelian-Higgs cosmic string
evolution with multiple GPUs": the Crank-Nicolson kicks of Pi and E, the
drifts of phi and A, link variables, the covariant Laplacian, the plaquette
field strength, and the diagnostics xi_L, xi_W, <v^2>_phi, <v^2>_omega plus
energy and the Gauss-law residual.  All arithmetic lives in ahref.c; this module only
marshals arguments.

Pins (what fixes the oracle other than itself) live in tests/test_oracle_*.py;
every output has one (closed forms, invariants, brute force, a published
test vector).
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# AHREF_LIB names another build of ahref.c (the planted-mistake tests load
# deliberately broken copies this way)
LIB_PATH = os.environ.get("AHREF_LIB") or os.path.join(HERE, "libahref.so")

NCOMP = 10
COMPONENTS = ("phi_re", "phi_im", "pi_re", "pi_im", "A0", "A1", "A2", "E0", "E1", "E2")


class _Params(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("compact", ctypes.c_int32),
        ("dx", ctypes.c_double), ("deta", ctypes.c_double),
        ("lambda0", ctypes.c_double), ("e0", ctypes.c_double), ("sigma", ctypes.c_double),
        ("m", ctypes.c_double), ("alpha", ctypes.c_double),
        ("s_early", ctypes.c_double), ("s_late", ctypes.c_double), ("eta_switch", ctypes.c_double),
        ("eta0", ctypes.c_double), ("eta_ref", ctypes.c_double),
        ("damp_gamma", ctypes.c_double), ("eta_damp", ctypes.c_double),
    ]


class _Scalars(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("eta", "s", "a", "f", "delta", "omega")]


class _Meas(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("eta", ctypes.c_double), ("a", ctypes.c_double), ("f", ctypes.c_double),
        ("winding_sum_abs", ctypes.c_int64), ("L_W", ctypes.c_double), ("xi_W", ctypes.c_double),
        ("sum_L", ctypes.c_double), ("xi_L", ctypes.c_double), ("R", ctypes.c_double), ("v2_phi", ctypes.c_double),
        ("energy", ctypes.c_double), ("e_kin", ctypes.c_double), ("e_grad", ctypes.c_double),
        ("e_pot", ctypes.c_double), ("e_el", ctypes.c_double), ("e_mag", ctypes.c_double),
        ("gauss_rms", ctypes.c_double), ("gauss_max", ctypes.c_double), ("gauss_rel", ctypes.c_double),
        ("nonfinite", ctypes.c_int64), ("v2_omega", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    dp = P(ctypes.c_double)
    lib.ahref_scalars_at.argtypes = [P(_Params), ctypes.c_int64, P(_Scalars)]
    lib.ahref_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.ahref_splitmix64.restype = ctypes.c_uint64
    lib.ahref_init.argtypes = [P(_Params), ctypes.c_uint64, dp]
    lib.ahref_kick.argtypes = [P(_Params), dp, ctypes.c_int64, dp, dp]
    lib.ahref_step.argtypes = [P(_Params), dp, ctypes.c_int64, ctypes.c_int64]
    lib.ahref_step_sites.argtypes = [P(_Params), dp, ctypes.c_int64, P(ctypes.c_int64), ctypes.c_int64, dp]
    lib.ahref_winding.argtypes = [P(_Params), dp, P(ctypes.c_int32)]
    lib.ahref_winding_sites.argtypes = [P(_Params), dp, P(ctypes.c_int64), ctypes.c_int64, P(ctypes.c_int32)]
    lib.ahref_gauss.argtypes = [P(_Params), dp, ctypes.c_int64, dp]
    lib.ahref_measure.argtypes = [P(_Params), dp, ctypes.c_int64, P(_Meas)]
    lib.ahref_num_threads.restype = ctypes.c_int
    lib.ahref_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


DEFAULTS = dict(N=16, compact=1, dx=0.5, deta=0.1, lambda0=2.0, e0=1.0, sigma=1.0, m=1.0, alpha=2.0,
                s_early=0.0, s_late=0.0, eta_switch=math.inf, eta0=1.0, eta_ref=0.0, damp_gamma=0.0, eta_damp=0.0)


def params(**kw) -> dict:
    """Parameter dict with the paper's standard choices (section 2) as defaults.

    eta_ref <= 0 selects a(eta_end) = 1 with eta_end = dx*N/2 (half light-crossing)."""
    p = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(k)
        p[k] = v
    if p["eta_ref"] <= 0.0:
        p["eta_ref"] = 0.5 * p["dx"] * p["N"]
    return p


def _c(p: dict) -> _Params:
    q = _Params()
    for k, _ in _Params._fields_:
        setattr(q, k, p[k])
    return q


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _state(p: dict, st: np.ndarray) -> np.ndarray:
    V = p["N"] ** 3
    if st.shape != (NCOMP, V) and st.shape != (NCOMP, p["N"], p["N"], p["N"]):
        raise ValueError(f"state shape {st.shape} does not match N={p['N']}")
    if st.dtype != np.float64 or not st.flags["C_CONTIGUOUS"]:
        raise ValueError("state must be a C-contiguous float64 array")
    return st


def scalars(p: dict, n: int) -> dict:
    s = _Scalars()
    _load().ahref_scalars_at(ctypes.byref(_c(p)), n, ctypes.byref(s))
    return {k: getattr(s, k) for k, _ in _Scalars._fields_}


def splitmix64(seed: int, k: int) -> int:
    return int(_load().ahref_splitmix64(seed, k))


def init(p: dict, seed: int) -> np.ndarray:
    """Random-phase initial state (10, N^3) float64."""
    st = np.zeros((NCOMP, p["N"] ** 3), dtype=np.float64)
    _load().ahref_init(ctypes.byref(_c(p)), seed, _dptr(st))
    return st


def kick(p: dict, st: np.ndarray, n: int):
    """Pi^{n+1/2} (2, V) and E^{n+1/2} (3, V) from snapshot n; st unchanged."""
    st = _state(p, st)
    V = p["N"] ** 3
    pin = np.zeros((2, V))
    en = np.zeros((3, V))
    _load().ahref_kick(ctypes.byref(_c(p)), _dptr(st), n, _dptr(pin), _dptr(en))
    return pin, en


def step(p: dict, st: np.ndarray, n0: int, nsteps: int) -> np.ndarray:
    """Return a copy of st advanced from snapshot n0 by nsteps steps."""
    out = np.array(_state(p, st), dtype=np.float64, copy=True, order="C")
    _load().ahref_step(ctypes.byref(_c(p)), _dptr(out), n0, nsteps)
    return out


def step_sites(p: dict, st: np.ndarray, n: int, sites) -> np.ndarray:
    """One step from snapshot n at the listed site indices: (len(sites), 10)."""
    st = _state(p, st)
    sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    out = np.zeros((len(sites), NCOMP))
    _load().ahref_step_sites(ctypes.byref(_c(p)), _dptr(st), n,
                             sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(sites), _dptr(out))
    return out


def winding(p: dict, st: np.ndarray) -> np.ndarray:
    """Plaquette windings (3, V) int32, orientations (0,1), (0,2), (1,2)."""
    st = _state(p, st)
    W = np.zeros((3, p["N"] ** 3), dtype=np.int32)
    _load().ahref_winding(ctypes.byref(_c(p)), _dptr(st), W.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return W


def winding_sites(p: dict, st: np.ndarray, sites) -> np.ndarray:
    """Windings (len(sites), 3) of the plaquettes (0,1), (0,2), (1,2) based at the listed sites."""
    st = _state(p, st)
    sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    W = np.zeros((len(sites), 3), dtype=np.int32)
    _load().ahref_winding_sites(ctypes.byref(_c(p)), _dptr(st), sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                len(sites), W.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return W


def gauss(p: dict, st: np.ndarray, n: int) -> np.ndarray:
    st = _state(p, st)
    G = np.zeros(p["N"] ** 3)
    _load().ahref_gauss(ctypes.byref(_c(p)), _dptr(st), n, _dptr(G))
    return G


def measure(p: dict, st: np.ndarray, n: int) -> dict:
    st = _state(p, st)
    m = _Meas()
    _load().ahref_measure(ctypes.byref(_c(p)), _dptr(st), n, ctypes.byref(m))
    return {k: getattr(m, k) for k, _ in _Meas._fields_}


def num_threads() -> int:
    return int(_load().ahref_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads for the oracle's later calls."""
    _load().ahref_set_threads(int(n))
