"""Test helpers: one parameter set expressed for both the oracle and the GPU binding,
and the field-scaled error norm used for parity (per field f in {phi, Pi, A, E}:
max_x |f_gpu - f_ref| / max_x |f_ref|, reported as the max over fields)."""
import math

import numpy as np

FIELD_GROUPS = {"phi": (0, 1), "pi": (2, 3), "A": (4, 5, 6), "E": (7, 8, 9)}


def both_params(oracle_mod, N, precision="fp64", **kw):
    from paper_2005_14454_amd import Params
    gauge = kw.pop("gauge_action", "compact")
    op = oracle_mod.params(N=N, compact=1 if gauge == "compact" else 0, **kw)
    gp = Params(N=N, precision=precision, gauge_action=gauge, **{k: v for k, v in op.items() if k not in ("N", "compact")})
    return op, gp


def field_scaled_error(got: np.ndarray, ref: np.ndarray) -> dict:
    out = {}
    for name, comps in FIELD_GROUPS.items():
        g = got[list(comps)]
        r = ref[list(comps)]
        scale = np.max(np.abs(r))
        diff = np.max(np.abs(g - r))
        out[name] = diff / scale if scale > 0 else diff
    return out


def max_field_error(got, ref) -> float:
    return max(field_scaled_error(got, ref).values())


def ulp_distance(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.abs(a - b) / np.spacing(np.maximum(np.abs(a), np.abs(b)))


def same_record(a: dict, b: dict) -> bool:
    """Bitwise equality of two measurement dicts (NaN equals NaN)."""
    if a.keys() != b.keys():
        return False
    for k in a:
        x, y = a[k], b[k]
        if isinstance(x, float) and isinstance(y, float):
            if not (x == y or (math.isnan(x) and math.isnan(y))):
                return False
        elif x != y:
            return False
    return True


def close_record(a: dict, b: dict, rtol: float) -> bool:
    """Equality of two measurement dicts up to the rounding of their FP64
    sums (a diagnostics pass over other workgroup shapes adds the same site
    values in another order): integers and flags exactly, every float within
    rtol of the larger magnitude of the pair (NaN equals NaN)."""
    if a.keys() != b.keys():
        return False
    for k in a:
        x, y = a[k], b[k]
        if isinstance(x, float) and isinstance(y, float):
            if math.isnan(x) or math.isnan(y):
                if not (math.isnan(x) and math.isnan(y)):
                    return False
            elif abs(x - y) > rtol * max(abs(x), abs(y)):
                return False
        elif x != y:
            return False
    return True


def run_alone(gp, seed, nsteps, every, tile, zchunk):
    """One lattice run alone through ah_step / ah_measure: its fields after
    nsteps and its diagnostics series (every `every` steps and the last)."""
    import paper_2005_14454_amd as ah
    series = []
    with ah.Lattice(gp) as lat:
        lat.set_step_config("tile", tile, zchunk)
        lat.init(seed)
        for k in range(nsteps + 1):
            if k == nsteps or (every > 0 and k % every == 0):
                series.append(lat.measure())
            if k < nsteps:
                lat.step(1)
        return lat.get_state(), series


def rounding_floor(oracle_mod, N=64, seed=0, nsteps=100):
    """Field-scaled difference after nsteps between the run from the
    random-phase start and the run with phi nudged by one ulp at every site."""
    op = oracle_mod.params(N=N, m=1.0)
    ic = oracle_mod.init(op, seed)
    nudged = ic.copy()
    nudged[0:2] = np.nextafter(nudged[0:2], np.inf)
    a = oracle_mod.step(op, ic, 0, nsteps)
    b = oracle_mod.step(op, nudged, 0, nsteps)
    return field_scaled_error(b, a)
