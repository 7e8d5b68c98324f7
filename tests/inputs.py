"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Only random numbers and shapes live here: no part of the method's
arithmetic.  State arrays are (10, N^3) float64 in the order
phi_re, phi_im, pi_re, pi_im, A0, A1, A2, E0, E1, E2 with site index
idx = x0 + N*(x1 + N*x2).
"""
import numpy as np

NCOMP = 10


def random_state(N: int, seed: int, phi_amp=0.3, pi_amp=0.3, a_amp=0.6, e_amp=0.3) -> np.ndarray:
    """Generic dense state: |phi| ~ 1 with random phase and modulus noise,
    Pi, A, E Gaussian with the given standard deviations."""
    rng = np.random.default_rng(seed)
    V = N ** 3
    st = np.empty((NCOMP, V), dtype=np.float64)
    mod = 1.0 + phi_amp * rng.standard_normal(V)
    ang = rng.uniform(0.0, 2.0 * np.pi, V)
    st[0] = mod * np.cos(ang)
    st[1] = mod * np.sin(ang)
    st[2:4] = pi_amp * rng.standard_normal((2, V))
    st[4:7] = a_amp * rng.standard_normal((3, V))
    st[7:10] = e_amp * rng.standard_normal((3, V))
    return st


def random_gauge(N: int, seed: int) -> np.ndarray:
    """Site gauge angles Lambda uniform on [0, 2 pi)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * np.pi, N ** 3)


def sample_sites(N: int, count: int, seed: int) -> np.ndarray:
    """Distinct site indices, always including the 8 lattice corners and the
    faces' wrap points, plus random interior sites."""
    rng = np.random.default_rng(seed)
    V = N ** 3
    corners = []
    for x2 in (0, N - 1):
        for x1 in (0, N - 1):
            for x0 in (0, N - 1):
                corners.append(x0 + N * (x1 + N * x2))
    rand = rng.choice(V, size=min(count, V), replace=False)
    return np.unique(np.concatenate([np.array(corners, dtype=np.int64), rand.astype(np.int64)]))


def grid(N: int):
    """Integer coordinates (x0, x1, x2) of every site, each of shape (N^3,)."""
    idx = np.arange(N ** 3, dtype=np.int64)
    return idx % N, (idx // N) % N, idx // (N * N)


def near_cut_state(N: int, seed: int, dx: float = 0.5, kmax: int = 1000, eps: float = 1e-4) -> np.ndarray:
    """State whose windings sit on their decision boundaries.

    phi has phase pi ((x0 + x1 + x2) mod 2) + U(-eps, eps), so with a trivial
    link the gauge-invariant link phases lie within ~2 eps of the branch cut
    at +-pi; A_i = 2 pi k / dx with k uniform in [-kmax, kmax] (links near 1,
    but |dx A| up to ~2 pi kmax), plus pi / dx on x-links at odd x1, which
    puts every (x, y) plaquette angle on a half turn.  Pi and E are Gaussian."""
    rng = np.random.default_rng(seed)
    V = N ** 3
    x0, x1, x2 = grid(N)
    st = np.empty((NCOMP, V), dtype=np.float64)
    mod = 1.0 + 0.3 * rng.standard_normal(V)
    ang = np.pi * ((x0 + x1 + x2) % 2) + rng.uniform(-eps, eps, V)
    st[0] = mod * np.cos(ang)
    st[1] = mod * np.sin(ang)
    st[2:4] = 0.3 * rng.standard_normal((2, V))
    k = rng.integers(-kmax, kmax + 1, (3, V))
    st[4:7] = 2.0 * np.pi * k / dx
    st[4] += (np.pi / dx) * (x1 % 2)
    st[7:10] = 0.3 * rng.standard_normal((3, V))
    return st
