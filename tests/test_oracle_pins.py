"""Pins for the FP64 CPU oracle: each test ties one part of the oracle to
something other than the oracle itself -- a closed form, an invariant stated
in section 2 of the paper, a published test vector, brute force on a tiny
lattice, or an independent formulation (forces as minus the gradient of the
lattice Hamiltonian, by autograd).  A plausible slip anywhere in the oracle
(a dropped term, a wrong sign, index or power of dx, a transposed operand)
fails at least one of these.
"""
import math
import os

import numpy as np
import pytest
import torch

from inputs import grid, near_cut_state, random_gauge, random_state, sample_sites

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ helpers

def gauge_transform(st, lam, N, dx):
    """phi, Pi -> e^{i Lambda} phi, e^{i Lambda} Pi; A_i -> A_i + (Lambda^{x+i} - Lambda^x)/dx."""
    out = st.copy()
    c, s = np.cos(lam), np.sin(lam)
    for r, i in ((0, 1), (2, 3)):
        out[r] = c * st[r] - s * st[i]
        out[i] = s * st[r] + c * st[i]
    L = lam.reshape(N, N, N)  # [x2, x1, x0]
    for j in range(3):
        Lp = np.roll(L, -1, axis=2 - j).reshape(-1)
        out[4 + j] = st[4 + j] + (Lp - lam) / dx
    return out


def rel_err(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# ------------------------------------------------------ generator and IC

def test_splitmix64_published_vector(oracle_mod):
    want = [int(l) for l in open(os.path.join(HERE, "golden", "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    got = [oracle_mod.splitmix64(1234567, k) for k in range(5)]
    assert got == want


def test_ic_random_phase_statistics(oracle_mod):
    """Section 2 initial condition: |phi| = sigma, phase uniform, all else zero."""
    N = 24
    p = oracle_mod.params(N=N, sigma=1.7)
    st = oracle_mod.init(p, 7)
    mod = np.hypot(st[0], st[1])
    assert np.allclose(mod, 1.7, rtol=0, atol=4e-16 * 1.7 * 4)
    assert np.all(st[2:] == 0.0)
    ang = np.mod(np.arctan2(st[1], st[0]), 2 * np.pi) / (2 * np.pi)
    from scipy import stats
    assert stats.kstest(ang, "uniform").pvalue > 1e-3
    # the phase of site i is 2 pi u with u = top 53 bits of the i-th generator output
    for i in (0, 1, 5, 1000, N ** 3 - 1):
        u = (oracle_mod.splitmix64(7, i) >> 11) / 2.0 ** 53
        assert abs(ang[i] - u) < 1e-15 or abs(abs(ang[i] - u) - 1.0) < 1e-15
    # different seeds give different fields, same seed the same
    assert np.array_equal(st, oracle_mod.init(p, 7))
    assert not np.array_equal(st, oracle_mod.init(p, 8))


# ----------------------------------------------------------- scalars a1

def test_scalars_definitions(oracle_mod):
    p = oracle_mod.params(N=8, m=2.0, s_early=0.0, s_late=1.0, eta_switch=1.55, eta_ref=4.0)
    s0 = oracle_mod.scalars(p, 0)
    assert s0["eta"] == 1.0 and s0["a"] == (1.0 / 4.0) ** 2 and s0["f"] == 1.0
    assert abs(s0["delta"] - 0.2) < 1e-16 and abs(s0["omega"] - 0.2) < 1e-16
    s6 = oracle_mod.scalars(p, 6)  # eta = 1.6 > eta_switch: s = 1
    a = (1.6 / 4.0) ** 2
    assert abs(s6["f"] - a * a) < 1e-15 and s6["omega"] == 0.0
    # eta_ref default is the half light-crossing time dx N / 2
    q = oracle_mod.params(N=64)
    assert q["eta_ref"] == 16.0


# ------------------------------------------- forces = -grad H (brute force)

def _potential_torch(phr, phi, A, p, f):
    """Lattice Hamiltonian without the momenta, written independently with torch
    rolls: sum_x [ sum_i |U_i phi^{x+i} - phi^x|^2/dx^2 + lambda0 f/4 (|phi|^2-sigma^2)^2
    + 1/(2 e0^2 f) sum_{i<j} B_ij^2 ],  B^2 = 2(1-cos Theta)/dx^4 or Theta^2/dx^4."""
    dx = p["dx"]

    def fwd(t, d):  # t at x + k_d; arrays are indexed [x2, x1, x0]
        return torch.roll(t, shifts=-1, dims=2 - d)

    H = torch.zeros((), dtype=torch.float64)
    for j in range(3):
        ang = -dx * A[j]
        fr, fi = fwd(phr, j), fwd(phi, j)
        ur = torch.cos(ang) * fr - torch.sin(ang) * fi
        ui = torch.cos(ang) * fi + torch.sin(ang) * fr
        H = H + (((ur - phr) ** 2 + (ui - phi) ** 2) / dx ** 2).sum()
    H = H + (p["lambda0"] * f / 4.0 * (phr ** 2 + phi ** 2 - p["sigma"] ** 2) ** 2).sum()
    for i, j in ((0, 1), (0, 2), (1, 2)):
        th = dx * (A[i] + fwd(A[j], i) - fwd(A[i], j) - A[j])
        B2 = 2.0 * (1.0 - torch.cos(th)) / dx ** 4 if p["compact"] else th ** 2 / dx ** 4
        H = H + (B2 / (2.0 * p["e0"] ** 2 * f)).sum()
    return H


@pytest.mark.parametrize("compact", [1, 0])
@pytest.mark.parametrize("expanding", [False, True])
def test_forces_are_minus_grad_H_4cubed(oracle_mod, compact, expanding):
    N = 4
    if expanding:
        # m = 1, s = 1, a(eta0) = 1/2: f = a^2 = 1/4, delta = deta/eta0 = 0.1, omega = 0
        p = oracle_mod.params(N=N, compact=compact, m=1.0, s_early=1.0, s_late=1.0, eta_ref=2.0,
                              lambda0=1.3, e0=0.8, sigma=1.1)
        f, delta, omega = 0.25, 0.1, 0.0
    else:
        p = oracle_mod.params(N=N, compact=compact, m=0.0, lambda0=1.3, e0=0.8, sigma=1.1)
        f, delta, omega = 1.0, 0.0, 0.0
    st = random_state(N, seed=11, a_amp=1.5)
    st[2:4] = 0.0
    st[7:10] = 0.0
    pin, en = oracle_mod.kick(p, st, 0)
    force_pi = pin * (1.0 + delta) / p["deta"]
    force_e = en * (1.0 + omega) / p["deta"]

    t = torch.tensor(st.reshape(10, N, N, N), requires_grad=True)
    H = _potential_torch(t[0], t[1], [t[4], t[5], t[6]], p, f)
    (g,) = torch.autograd.grad(H, t)
    g = g.detach().numpy().reshape(10, -1)
    want_pi = -0.5 * g[0:2]
    want_e = -p["e0"] ** 2 * f * g[4:7]
    assert rel_err(force_pi, want_pi) < 1e-12
    assert rel_err(force_e, want_e) < 1e-12


# ------------------------------------------------- closed-form dynamics

def test_scalar_plane_wave_dispersion(oracle_mod):
    """Free real scalar standing wave: phi^n = cos(k.x) cos(W(n+1/2)deta)/cos(W deta/2)
    with (2/deta) sin(W deta/2) = sqrt(sum_j (2/dx)^2 sin^2(k_j dx/2))."""
    N, dx, deta = 16, 0.5, 0.1
    p = oracle_mod.params(N=N, dx=dx, deta=deta, lambda0=0.0, m=0.0)
    x0, x1, x2 = grid(N)
    k = 2 * np.pi * np.array([1, 2, 3]) / (N * dx)
    kx = k[0] * x0 * dx + k[1] * x1 * dx + k[2] * x2 * dx
    st = np.zeros((10, N ** 3))
    st[0] = np.cos(kx)
    K = math.sqrt(sum((2 / dx) ** 2 * math.sin(kj * dx / 2) ** 2 for kj in k))
    W = 2 / deta * math.asin(deta * K / 2)
    n = 57
    out = oracle_mod.step(p, st, 0, n)
    want = np.cos(kx) * math.cos(W * (n + 0.5) * deta) / math.cos(W * deta / 2)
    assert np.max(np.abs(out[0] - want)) < 1e-12
    assert np.all(out[1] == 0) and np.all(out[4:] == 0)


@pytest.mark.parametrize("compact,eps,tol", [(0, 0.7, 1e-12), (1, 1e-5, 1e-9)])
def test_maxwell_plane_wave_dispersion(oracle_mod, compact, eps, tol):
    """Free transverse gauge wave A_1 = eps cos(k x0 dx), phi = 0: same lattice dispersion
    (exact for the non-compact action, to O((dx eps)^2) for the compact one)."""
    N, dx, deta = 16, 0.5, 0.1
    p = oracle_mod.params(N=N, dx=dx, deta=deta, m=0.0, compact=compact)
    x0, _, _ = grid(N)
    k = 2 * np.pi * 3 / (N * dx)
    st = np.zeros((10, N ** 3))
    st[5] = eps * np.cos(k * x0 * dx)
    K = 2 / dx * abs(math.sin(k * dx / 2))
    W = 2 / deta * math.asin(deta * K / 2)
    n = 45
    out = oracle_mod.step(p, st, 0, n)
    want = eps * np.cos(k * x0 * dx) * math.cos(W * (n + 0.5) * deta) / math.cos(W * deta / 2)
    assert np.max(np.abs(out[5] - want)) / eps < tol
    assert np.all(out[4] == 0) and np.all(out[6] == 0)


@pytest.mark.parametrize("m", [1.0, 2.0])
def test_hubble_damping_telescopes(oracle_mod, m):
    """Zero-force uniform Pi and E decay by prod_k (1-delta_k)/(1+delta_k).  With
    alpha = 2, delta_k = m deta/eta_k and the product telescopes:
    m=1: eta_{-1} eta_0 / (eta_{K-1} eta_K);  m=2: eta_{-2..1} / eta_{K-2..K+1}."""
    N, K, deta = 4, 100, 0.1
    p = oracle_mod.params(N=N, m=m, lambda0=0.0)
    eta = lambda n: 1.0 + n * deta
    if m == 1.0:
        want = eta(-1) * eta(0) / (eta(K - 1) * eta(K))
    else:
        want = (eta(-2) * eta(-1) * eta(0) * eta(1)) / (eta(K - 2) * eta(K - 1) * eta(K) * eta(K + 1))
    # scalar sector: uniform phi, uniform Pi, no gauge field
    st = np.zeros((10, N ** 3))
    st[0], st[1], st[2], st[3] = 0.1, 0.05, 0.3, -0.2
    out = oracle_mod.step(p, st, 0, K)
    assert abs(out[2, 0] / 0.3 - want) < 1e-13 and abs(out[3, 0] / -0.2 - want) < 1e-13
    # gauge sector: phi = 0, uniform E (s = 0 so omega = delta)
    st = np.zeros((10, N ** 3))
    st[7], st[8], st[9] = 0.4, -0.1, 0.25
    out = oracle_mod.step(p, st, 0, K)
    for c, v in ((7, 0.4), (8, -0.1), (9, 0.25)):
        assert abs(out[c, 5] / v - want) < 1e-13
    # s = 1: omega = 0, E is not damped
    p1 = oracle_mod.params(N=N, m=m, lambda0=0.0, s_early=1.0, s_late=1.0)
    out = oracle_mod.step(p1, st, 0, K)
    assert np.all(out[7] == 0.4)


def test_artificial_damping_phase(oracle_mod):
    """A damping phase (friction gamma while eta < eta_damp, then the Hubble
    term again): zero-force uniform Pi and E decay by ((1 - g)/(1 + g))^K1
    with g = gamma deta / 2 over the K1 steps of the phase, then by the
    telescoping Hubble product (m = 1) from there on."""
    N, deta, gamma, eta_damp, K = 4, 0.1, 3.0, 3.05, 60
    p = oracle_mod.params(N=N, m=1.0, lambda0=0.0, damp_gamma=gamma, eta_damp=eta_damp)
    eta = lambda n: 1.0 + n * deta
    K1 = sum(1 for n in range(K) if eta(n) < eta_damp)
    assert K1 == 21
    g = 0.5 * gamma * deta
    want = ((1 - g) / (1 + g)) ** K1 * eta(K1 - 1) * eta(K1) / (eta(K - 1) * eta(K))
    st = np.zeros((10, N ** 3))
    st[0], st[1], st[2], st[3] = 0.1, 0.05, 0.3, -0.2
    out = oracle_mod.step(p, st, 0, K)
    assert abs(out[2, 0] / 0.3 - want) < 1e-13 and abs(out[3, 0] / -0.2 - want) < 1e-13
    st = np.zeros((10, N ** 3))
    st[7], st[9] = 0.4, 0.25
    out = oracle_mod.step(p, st, 0, K)
    assert abs(out[7, 3] / 0.4 - want) < 1e-13 and abs(out[9, 3] / 0.25 - want) < 1e-13
    # damping the random-phase start keeps Gauss's law (s = 0) and drains energy faster than without
    p0 = oracle_mod.params(N=8, m=1.0)
    pd = oracle_mod.params(N=8, m=1.0, damp_gamma=gamma, eta_damp=eta_damp)
    a = oracle_mod.step(p0, oracle_mod.init(p0, 3), 0, 30)
    b = oracle_mod.step(pd, oracle_mod.init(pd, 3), 0, 30)
    ma, mb = oracle_mod.measure(p0, a, 30), oracle_mod.measure(pd, b, 30)
    assert mb["gauss_rel"] < 1e-13 and mb["energy"] < ma["energy"]


@pytest.mark.parametrize("m,s,eta_ref", [(2.0, 1.0, 5.0), (1.0, -1.0, 2.0)])
def test_homogeneous_mode_reduces_to_scalar_recurrence(oracle_mod, m, s, eta_ref):
    """Uniform real phi with A = E = 0: every stencil term cancels and the lattice
    update is the one-site recurrence of a damped anharmonic oscillator whose
    coupling scales as f_n = a_n^{2s} (s = 1: the true equations; s = -1: the
    cores grow as a does)."""
    N = 4
    p = oracle_mod.params(N=N, m=m, s_early=s, s_late=s, eta_ref=eta_ref, sigma=1.0, lambda0=2.0)
    st = np.zeros((10, N ** 3))
    st[0], st[2] = 0.4, 0.1
    out = oracle_mod.step(p, st, 0, 80)
    ph, pi = 0.4, 0.1
    for n in range(80):
        eta = 1.0 + 0.1 * n
        f = ((eta / eta_ref) ** m) ** (2 * s)
        d = m * 0.1 / eta
        pi = ((1 - d) * pi + 0.1 * (-(2.0 * f / 2.0) * (ph * ph - 1.0) * ph)) / (1 + d)
        ph = ph + 0.1 * pi
    assert abs(out[0, 17] - ph) < 1e-13 and abs(out[2, 17] - pi) < 1e-13
    assert np.all(out[0] == out[0, 0]) and np.all(out[1] == 0) and np.all(out[4:] == 0)


# -------------------------------------------------------------- invariants

@pytest.mark.parametrize("m,s", [(0.0, 0.0), (1.0, 0.0), (2.0, 0.0), (2.0, 1.0), (1.0, 1.0)])
def test_vacuum_is_bitwise_static(oracle_mod, m, s):
    N = 6
    p = oracle_mod.params(N=N, m=m, s_early=s, s_late=s, sigma=1.0)
    st = np.zeros((10, N ** 3))
    st[0] = 1.0
    out = oracle_mod.step(p, st, 0, 20)
    assert np.array_equal(out, st)


def test_pure_gauge_is_static(oracle_mod):
    N = 6
    p = oracle_mod.params(N=N, m=1.0)
    st = np.zeros((10, N ** 3))
    st[0] = p["sigma"]
    st = gauge_transform(st, random_gauge(N, 3), N, p["dx"])
    out = oracle_mod.step(p, st, 0, 30)
    assert np.max(np.abs(out - st)) < 1e-12


@pytest.mark.parametrize("m,s", [(0.0, 0.0), (1.0, 0.0), (2.0, 0.0), (0.0, 1.0), (1.0, 1.0)])
def test_gauss_law_exact(oracle_mod, m, s):
    """Section 2: the damping omega = (1-s) delta keeps Gauss's law to machine
    precision.  Holds exactly for s = 0 (any m) and s = 1 with m in {0, 1}."""
    N = 8
    p = oracle_mod.params(N=N, m=m, s_early=s, s_late=s)
    st = oracle_mod.init(p, 5)
    n = 0
    for chunk in (10, 20, 30):
        st = oracle_mod.step(p, st, n, chunk)
        n += chunk
        meas = oracle_mod.measure(p, st, n)
        assert meas["gauss_rel"] < 1e-13, (n, meas["gauss_rel"])


def test_gauss_law_not_exact_for_matter_era_physical_width(oracle_mod):
    """s = 1, m = 2 does not conserve the discrete constraint (the residual grows)."""
    N = 6
    p = oracle_mod.params(N=N, m=2.0, s_early=1.0, s_late=1.0)
    st = oracle_mod.step(p, oracle_mod.init(p, 5), 0, 40)
    assert oracle_mod.measure(p, st, 40)["gauss_rel"] > 1e-6


def test_gauss_residual_detects_violation(oracle_mod):
    """A single-site E perturbation shows up as a dipole in G of exactly +-eps/dx."""
    N = 6
    p = oracle_mod.params(N=N)
    st = np.zeros((10, N ** 3))
    st[0] = 1.0
    st[7, 0] = 0.01  # E_0 at the origin
    G = oracle_mod.gauss(p, st, 3)
    nz = np.flatnonzero(G)
    assert set(nz.tolist()) == {0, 1}
    assert abs(G[0] - 0.02) < 1e-17 and abs(G[1] + 0.02) < 1e-17


@pytest.mark.parametrize("n", [0, 3])
def test_gauss_norms_closed_form(oracle_mod, n):
    """The three Gauss norms of a hand-built state, in closed form.

    phi = sigma everywhere, E_0 = eps at the origin only and Pi = i kappa at
    the origin only.  The residual of section 2's Gauss law is then non-zero
    at two sites: G = eps/dx - c sigma kappa at the origin (divergence minus
    coupled charge) and G = -eps/dx at the +x neighbour (divergence only).
    With a = eps/dx and b = c sigma kappa:
        gauss_max = max(|a - b|, a),
        gauss_rms = sqrt(((a - b)^2 + a^2) / N^3),
        gauss_rel = sqrt((a - b)^2 + a^2) / sqrt(a^2 + a^2 + b^2).
    c is the coupling that keeps the law exact under the kick, 2 e0^2 f_0 at
    the start and 2 e0^2 f_{n-1} (1 + delta_{n-1}) / (1 + omega_{n-1}) after
    it; that this c is the right one is pinned separately by the exactness of
    the law along evolved runs (s = 1 with m = 1 is among them).  dx, e0 and
    sigma differ from 1 and f from 1 (s = 1), so a wrong power of dx, a
    dropped coupling factor, a mean over N instead of N^3 or a relative norm
    without its charge term fails here."""
    N, dx, e0, sigma, deta, eta0, eta_ref = 6, 0.7, 0.8, 1.3, 0.1, 1.0, 2.0
    p = oracle_mod.params(N=N, dx=dx, e0=e0, sigma=sigma, m=1.0, s_early=1.0, s_late=1.0,
                          eta0=eta0, eta_ref=eta_ref, deta=deta)
    eps, kappa = 0.05, 0.2
    st = np.zeros((10, N ** 3))
    st[0] = sigma
    st[7, 0] = eps
    st[3, 0] = kappa
    if n == 0:
        f = (eta0 / eta_ref) ** 2
        c = 2 * e0 ** 2 * f
    else:
        eta = eta0 + (n - 1) * deta
        f = (eta / eta_ref) ** 2
        delta = deta / eta  # (alpha/2) m deta / eta with alpha = 2, m = 1; omega = 0 at s = 1
        c = 2 * e0 ** 2 * f * (1 + delta)
    a, b = eps / dx, c * sigma * kappa
    G = oracle_mod.gauss(p, st, n)
    assert set(np.flatnonzero(G).tolist()) == {0, 1}
    assert abs(G[0] - (a - b)) < 1e-15 and abs(G[1] + a) < 1e-15
    m = oracle_mod.measure(p, st, n)
    assert abs(m["gauss_max"] - max(abs(a - b), a)) < 1e-15
    assert abs(m["gauss_rms"] - math.sqrt(((a - b) ** 2 + a ** 2) / N ** 3)) < 1e-15
    want_rel = math.sqrt((a - b) ** 2 + a ** 2) / math.sqrt(2 * a ** 2 + b ** 2)
    assert abs(m["gauss_rel"] - want_rel) < 1e-14
    # no violation, no denominator: the relative norm is defined as 0
    vac = np.zeros((10, N ** 3))
    vac[0] = sigma
    mv = oracle_mod.measure(p, vac, n)
    assert mv["gauss_rel"] == 0.0 and mv["gauss_rms"] == 0.0 and mv["gauss_max"] == 0.0


@pytest.mark.parametrize("N,dx,sigma,lambda0", [(5, 0.7, 1.3, 1.5), (6, 0.5, 0.6, 2.0)])
def test_xi_L_closed_form_false_vacuum(oracle_mod, N, dx, sigma, lambda0):
    """xi_L of section 2 (sqrt(-mu V / sum_x L_x), mu = 2 pi sigma^2, V the
    comoving volume, the sum carrying the cell volume dx^3) on the symmetric
    state phi = Pi = A = E = 0.  Nothing moves (every force is proportional
    to phi or to a field that is zero), so the Lagrangian density is minus
    the potential, -(lambda0 f / 4) sigma^4, at every site: sum_L =
    -(lambda0 f/4) sigma^4 (N dx)^3 and xi_L = sqrt(8 pi / (lambda0 f sigma^2)),
    independent of N and dx.  sigma, lambda0, dx and f (s = 1, a = 1/2) all
    differ from 1, so a wrong mu, a missing cell or box volume or a dropped
    f fails here."""
    p = oracle_mod.params(N=N, dx=dx, sigma=sigma, lambda0=lambda0, m=1.0, s_early=1.0, s_late=1.0,
                          eta0=1.0, eta_ref=2.0)
    f = 0.25
    m = oracle_mod.measure(p, np.zeros((10, N ** 3)), 0)
    assert abs(m["f"] - f) < 1e-16
    want_L = -(lambda0 * f / 4) * sigma ** 4 * (N * dx) ** 3
    assert abs(m["sum_L"] - want_L) < 1e-13 * abs(want_L)
    assert abs(m["xi_L"] - math.sqrt(8 * math.pi / (lambda0 * f * sigma ** 2))) < 1e-13
    # a positive Lagrangian sum (pure kinetic energy in the vacuum) has no xi_L
    st = np.zeros((10, N ** 3))
    st[0] = sigma
    st[2] = 0.3
    assert math.isnan(oracle_mod.measure(p, st, 0)["xi_L"])


def test_winding_sites_matches_full_winding(oracle_mod):
    """The per-site winding query returns the full winding array's entries."""
    N = 7
    p = oracle_mod.params(N=N)
    for st in (random_state(N, seed=61), near_cut_state(N, seed=62)):
        W = oracle_mod.winding(p, st)
        sites = sample_sites(N, 60, seed=63)
        assert np.array_equal(oracle_mod.winding_sites(p, st, sites), W[:, sites].T)
        assert np.abs(W).sum() > 0


@pytest.mark.parametrize("compact", [1, 0])
def test_gauge_covariance(oracle_mod, compact):
    """step(T_Lambda state) == T_Lambda step(state); diagnostics are invariant."""
    N = 6
    p = oracle_mod.params(N=N, compact=compact, m=1.0)
    st = random_state(N, seed=21)
    lam = random_gauge(N, 22)
    a = oracle_mod.step(p, gauge_transform(st, lam, N, p["dx"]), 3, 5)
    b = gauge_transform(oracle_mod.step(p, st, 3, 5), lam, N, p["dx"])
    assert np.max(np.abs(a - b)) < 1e-12
    ma = oracle_mod.measure(p, gauge_transform(st, lam, N, p["dx"]), 3)
    mb = oracle_mod.measure(p, st, 3)
    assert ma["winding_sum_abs"] == mb["winding_sum_abs"]
    for k in ("energy", "e_kin", "e_grad", "e_pot", "e_el", "e_mag", "sum_L", "gauss_rms"):
        assert abs(ma[k] - mb[k]) <= 1e-12 * max(1.0, abs(mb[k])), k


def test_compact_links_are_periodic_in_A(oracle_mod):
    """Compact U(1): shifting one A by 2 pi/dx changes nothing physical."""
    N = 5
    p = oracle_mod.params(N=N, compact=1)
    st = random_state(N, seed=31)
    st2 = st.copy()
    st2[5, 17] += 2 * np.pi / p["dx"]
    pa, ea = oracle_mod.kick(p, st, 0)
    pb, eb = oracle_mod.kick(p, st2, 0)
    assert np.max(np.abs(pa - pb)) < 1e-12 and np.max(np.abs(ea - eb)) < 1e-12
    assert np.array_equal(oracle_mod.winding(p, st), oracle_mod.winding(p, st2))


def test_energy_conserved_second_order_in_flat_space(oracle_mod):
    """m = 0: the centred energy has no drift and its error falls ~4x when deta halves."""
    N = 8
    errs = []
    for deta in (0.1, 0.05):
        p = oracle_mod.params(N=N, m=0.0, deta=deta, compact=1)
        st = random_state(N, seed=41, phi_amp=0.05, pi_amp=0.1, a_amp=0.1, e_amp=0.05)
        stride = int(round(0.5 / deta))
        e0 = oracle_mod.measure(p, st, 0)["energy"]
        worst = 0.0
        n = 0
        for _ in range(8):
            st = oracle_mod.step(p, st, n, stride)
            n += stride
            worst = max(worst, abs(oracle_mod.measure(p, st, n)["energy"] - e0) / e0)
        errs.append(worst)
    assert errs[0] < 5e-2
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


def test_laplacian_second_order_in_dx(oracle_mod):
    """Section 2: spatial derivatives are O(dx^2).  With smooth phi and A sampled at
    sites and link midpoints, the scalar force at common points converges with
    ratio 4 as dx halves (Richardson)."""
    L = 4.0
    forces = []
    for N in (16, 32, 64):
        dx = L / N
        p = oracle_mod.params(N=N, dx=dx, m=0.0, lambda0=0.0)
        x0, x1, x2 = grid(N)
        X, Y, Z = x0 * dx, x1 * dx, x2 * dx
        w = 2 * np.pi / L
        st = np.zeros((10, N ** 3))
        amp = 1.0 + 0.2 * np.cos(w * X) * np.sin(w * Z)
        ph = 0.7 * np.sin(w * Y + w * Z) + 0.3 * np.cos(w * X)
        st[0], st[1] = amp * np.cos(ph), amp * np.sin(ph)
        st[4] = 0.3 * np.sin(w * (X + dx / 2)) * np.cos(w * Y)
        st[5] = 0.2 * np.cos(w * Z) + 0.1 * np.sin(w * (Y + dx / 2))
        st[6] = 0.25 * np.sin(w * X + w * (Z + dx / 2))
        pin, _ = oracle_mod.kick(p, st, 0)
        F = (pin / p["deta"]).reshape(2, N, N, N)
        s = N // 16
        forces.append(F[:, ::s, ::s, ::s])
    r = np.abs(forces[0] - forces[1]).max() / np.abs(forces[1] - forces[2]).max()
    assert 3.6 < r < 4.4, r


# ---------------------------------------------------------------- windings

def _pair_state(N, sep_axis_len=None):
    x0, x1, x2 = grid(N)
    c1 = (N / 4 + 0.5, N / 2 + 0.5)
    c2 = (3 * N / 4 + 0.5, N / 2 + 0.5)
    th = np.arctan2(x1 - c1[1], x0 - c1[0]) - np.arctan2(x1 - c2[1], x0 - c2[0])
    st = np.zeros((10, N ** 3))
    st[0], st[1] = np.cos(th), np.sin(th)
    return st


def test_winding_string_pair(oracle_mod):
    """A straight string-antistring pair along x2 pierces one (0,1) plaquette of each
    sign per plane: sum |W| = 2N, xi_W = sqrt((N dx)^3 / (2 N dx))."""
    N = 12
    p = oracle_mod.params(N=N)
    st = _pair_state(N)
    W = oracle_mod.winding(p, st)
    assert np.abs(W).sum() == 2 * N
    assert np.all(W[1] == 0) and np.all(W[2] == 0)
    W01 = W[0].reshape(N, N, N)
    assert W01[:, N // 2, N // 4] .tolist() == [1] * N
    assert W01[:, N // 2, 3 * N // 4].tolist() == [-1] * N
    meas = oracle_mod.measure(p, st, 0)
    assert meas["winding_sum_abs"] == 2 * N
    assert abs(meas["L_W"] - 2 * N * 0.5) < 1e-15
    assert abs(meas["xi_W"] - math.sqrt((N * 0.5) ** 3 / (2 * N * 0.5))) < 1e-13


def test_winding_gauge_invariant_and_pure_gauge_zero(oracle_mod):
    N = 12
    p = oracle_mod.params(N=N)
    st = _pair_state(N)
    lam = random_gauge(N, 9)
    assert np.array_equal(oracle_mod.winding(p, gauge_transform(st, lam, N, p["dx"])), oracle_mod.winding(p, st))
    vac = np.zeros((10, N ** 3))
    vac[0] = 1.0
    assert np.all(oracle_mod.winding(p, gauge_transform(vac, lam, N, p["dx"])) == 0)


def test_winding_random_phase_one_third(oracle_mod):
    """Four independent uniform phases around a plaquette wind with probability 1/3,
    so E[sum |W|] = N^3 for a random-phase lattice with A = 0."""
    N = 32
    p = oracle_mod.params(N=N)
    tot = 0
    for seed in (0, 1):
        tot += oracle_mod.measure(p, oracle_mod.init(p, seed), 0)["winding_sum_abs"]
    frac = tot / (2 * 3 * N ** 3)
    assert abs(frac - 1.0 / 3.0) < 0.01, frac


# ------------------------------------------------------------ energy parts

def test_energy_parts_closed_forms(oracle_mod):
    N, dx = 6, 0.5
    vol = N ** 3 * dx ** 3
    # kinetic: uniform phi, uniform Pi, lambda0 = 0, m = 0 -> Pi unchanged by the kick
    p = oracle_mod.params(N=N, m=0.0, lambda0=0.0)
    st = np.zeros((10, N ** 3))
    st[0], st[2], st[3] = 1.0, 0.3, -0.4
    m = oracle_mod.measure(p, st, 0)
    assert abs(m["e_kin"] - 0.25 * vol) < 1e-14 and m["e_grad"] == 0 and m["e_el"] == 0 and m["e_mag"] == 0
    # potential: phi = 0 -> (lambda0 f / 4) sigma^4 per unit volume
    p = oracle_mod.params(N=N, m=0.0, lambda0=2.0, sigma=1.5)
    st = np.zeros((10, N ** 3))
    m = oracle_mod.measure(p, st, 0)
    assert abs(m["e_pot"] - 0.5 * 1.5 ** 4 * vol) < 1e-12
    # electric: phi = 0, uniform E, no forces -> E^2 / (2 e0^2 f)
    p = oracle_mod.params(N=N, m=0.0, e0=0.7)
    st = np.zeros((10, N ** 3))
    st[7], st[9] = 0.2, 0.1
    m = oracle_mod.measure(p, st, 0)
    assert abs(m["e_el"] - 0.05 / (2 * 0.49) * vol) < 1e-14
    # gradient: plane wave phi = exp(i k.x), A = 0: sum_j 4 sin^2(k_j dx/2)/dx^2
    x0, x1, x2 = grid(N)
    k = 2 * np.pi * np.array([1, 0, 2]) / (N * dx)
    ph = k[0] * x0 * dx + k[2] * x2 * dx
    st = np.zeros((10, N ** 3))
    st[0], st[1] = np.cos(ph), np.sin(ph)
    m = oracle_mod.measure(p, st, 0)
    g = sum(4 * math.sin(kj * dx / 2) ** 2 / dx ** 2 for kj in k)
    assert abs(m["e_grad"] - g * vol) < 1e-12 * g * vol
    # magnetic (non-compact): A_1 = eps cos(k x0 dx) gives Theta_01 = dx (A_1^{x+0} - A_1^x) and
    # sum_x Theta^2/dx^4 / 2 * dx^3 = N^3 eps^2 dx sin^2(k dx / 2)
    pn = oracle_mod.params(N=N, m=0.0, compact=0, e0=1.0)
    kk = 2 * np.pi / (N * dx)
    st = np.zeros((10, N ** 3))
    st[5] = 0.3 * np.cos(kk * x0 * dx)
    m = oracle_mod.measure(pn, st, 0)
    want = N ** 3 * 0.3 ** 2 * dx * math.sin(kk * dx / 2) ** 2
    assert abs(m["e_mag"] - want) < 1e-12 * want
    # compact: B^2 = 2 (1 - cos Theta)/dx^4 with a uniform plaquette angle Theta = dx^2 b
    # needs a periodic A with constant curl; instead compare the small-field limit
    pc = oracle_mod.params(N=N, m=0.0, compact=1, e0=1.0)
    st[5] = 1e-4 * np.cos(kk * x0 * dx)
    mc = oracle_mod.measure(pc, st, 0)
    want = N ** 3 * 1e-8 * dx * math.sin(kk * dx / 2) ** 2
    assert abs(mc["e_mag"] - want) < 1e-6 * want


def test_velocity_ratio_plane_wave(oracle_mod):
    """Translation-invariant state phi = exp(i k.x), Pi = c phi, m = 0, |phi| = sigma:
    every density is uniform, so R = |Pi_bar|^2 / sum_j |D_j^+ phi|^2 exactly, with the
    centred momentum Pi_bar = (c - deta K^2 / 2) phi."""
    N, dx, deta = 8, 0.5, 0.1
    p = oracle_mod.params(N=N, m=0.0, dx=dx, deta=deta)
    x0, x1, x2 = grid(N)
    k = 2 * np.pi * np.array([1, 1, 0]) / (N * dx)
    ph = k[0] * x0 * dx + k[1] * x1 * dx
    c = 0.9
    st = np.zeros((10, N ** 3))
    st[0], st[1] = np.cos(ph), np.sin(ph)
    st[2], st[3] = c * st[0], c * st[1]
    K2 = sum(4 * math.sin(kj * dx / 2) ** 2 / dx ** 2 for kj in k)
    R = (c - deta * K2 / 2) ** 2 / K2
    m = oracle_mod.measure(p, st, 0)
    assert abs(m["R"] - R) < 1e-12 * abs(R)
    assert abs(m["v2_phi"] - 2 * R / (1 + R)) < 1e-12
    assert abs(m["e_kin"] - (c - deta * K2 / 2) ** 2 * N ** 3 * dx ** 3) < 1e-10
    # xi_L: -mu V / sum_L with mu = 2 pi sigma^2
    if m["sum_L"] < 0:
        assert abs(m["xi_L"] - math.sqrt(-2 * math.pi * (N * dx) ** 3 / m["sum_L"])) < 1e-12 * m["xi_L"]
    parts = m["e_kin"] - m["e_grad"] - m["e_pot"] + m["e_el"] - m["e_mag"]
    assert abs(m["sum_L"] - parts) < 1e-11 * max(1.0, abs(parts))
    assert abs(m["energy"] - (m["e_kin"] + m["e_grad"] + m["e_pot"] + m["e_el"] + m["e_mag"])) < 1e-11 * m["energy"]


def test_velocity_ratio_weighted_by_lagrangian(oracle_mod):
    """R of section 2 weights |Pi|^2 and |D+ phi|^2 with the site Lagrangian:
    R = sum_x |Pi_bar|^2 L_x / sum_x |D+ phi|^2 L_x.  Plane wave phi = exp(i k x0)
    (|phi| = sigma: no potential), A = E = 0, m = 0, and Pi^{n-1/2} = c(x) phi
    with c = c1 on the lower half of the x2 planes and c2 on the upper half.
    Per site: gradient G = 4 sin^2(k dx/2)/dx^2; the kick adds -deta G phi, so
    the centred momentum is (c - deta G/2) phi; the current J_x = sin(k dx)/dx
    gives E^{n+1/2} = deta 2 e0^2 J_x, so the electric density is
    (E^{n+1/2}/2)^2 / (2 e0^2); no magnetic field.  The Lagrangian differs
    between the halves, so the weighted ratio differs from the plain one."""
    N, dx, deta = 8, 0.5, 0.1
    p = oracle_mod.params(N=N, m=0.0, dx=dx, deta=deta)
    x0, x1, x2 = grid(N)
    k = 2 * np.pi / (N * dx)
    ph = k * x0 * dx
    c = np.where(x2 < N // 2, 2.0, 0.0)
    st = np.zeros((10, N ** 3))
    st[0], st[1] = np.cos(ph), np.sin(ph)
    st[2], st[3] = c * st[0], c * st[1]
    G = 4 * math.sin(k * dx / 2) ** 2 / dx ** 2
    kin = (c - deta * G / 2) ** 2
    Ehalf = deta * 2.0 * math.sin(k * dx) / dx
    el = (Ehalf / 2) ** 2 / 2.0
    L = kin - G + el
    R = float(np.sum(kin * L) / np.sum(G * L))
    assert abs(R - float(np.sum(kin) / (G * N ** 3))) > 0.1  # the weighting matters here
    m = oracle_mod.measure(p, st, 0)
    assert abs(m["R"] - R) < 1e-12 * abs(R), (m["R"], R)
    assert abs(m["v2_phi"] - 2 * R / (1 + R)) < 1e-12
    assert abs(m["sum_L"] - float(np.sum(L)) * dx ** 3) < 1e-12 * abs(float(np.sum(L)) * dx ** 3)


def test_equation_of_state_velocity_single_terms(oracle_mod):
    """<v^2>_omega = (1 + 3 w)/2 with w the L-weighted ratio of pressure to
    energy density.  A state holding one kind of energy only has the textbook
    equation of state of that kind: kinetic w = 1, gradient w = -1/3 (a static
    string's transverse gradients), potential w = -1, electric and magnetic
    radiation w = 1/3.  The stored half-step momenta are chosen so that the
    centred ones are exactly the wanted ones (m = 0, no damping)."""
    N, dx, deta = 6, 0.5, 0.1
    x0, x1, x2 = grid(N)
    # kinetic only: phi = sigma, uniform Pi, no force on Pi, no current
    p = oracle_mod.params(N=N, m=0.0, lambda0=0.0, dx=dx, deta=deta)
    st = np.zeros((10, N ** 3))
    st[0], st[2], st[3] = 1.0, 0.3, -0.4
    assert abs(oracle_mod.measure(p, st, 0)["v2_omega"] - 2.0) < 1e-13
    # potential only: phi = 0 everywhere
    p = oracle_mod.params(N=N, m=0.0, lambda0=2.0, sigma=1.5, dx=dx, deta=deta)
    st = np.zeros((10, N ** 3))
    assert abs(oracle_mod.measure(p, st, 0)["v2_omega"] + 1.0) < 1e-13
    # electric only: phi = 0, uniform E, no curl and no current
    p = oracle_mod.params(N=N, m=0.0, lambda0=0.0, e0=0.7, dx=dx, deta=deta)
    st = np.zeros((10, N ** 3))
    st[7], st[9] = 0.2, 0.1
    assert abs(oracle_mod.measure(p, st, 0)["v2_omega"] - 1.0) < 1e-13
    # magnetic only (compact): A_1 = c x0 with c N dx = 2 pi gives the uniform
    # plaquette angle Theta_01 = 2 pi / N (the wrap differs by 2 pi); no curl
    p = oracle_mod.params(N=N, m=0.0, lambda0=0.0, compact=1, dx=dx, deta=deta)
    st = np.zeros((10, N ** 3))
    st[5] = 2 * np.pi / (N * dx) * x0
    m = oracle_mod.measure(p, st, 0)
    assert abs(m["e_mag"] - N ** 3 * dx ** 3 * (1 - math.cos(2 * math.pi / N)) / dx ** 4) < 1e-12 * m["e_mag"]
    assert abs(m["v2_omega"] - 1.0) < 1e-12
    # gradient only: phi = exp(i q x0), A = 0; Pi^{n-1/2} = -deta F / 2 and
    # E_0^{n-1/2} = -deta e0^2 J_0 make the centred momenta vanish, with the
    # force F = 2 (cos q - 1) phi / dx^2 and the current J_0 = sin q / dx
    q = 2 * np.pi * 2 / N
    e0 = 0.8
    p = oracle_mod.params(N=N, m=0.0, lambda0=0.0, e0=e0, dx=dx, deta=deta)
    st = np.zeros((10, N ** 3))
    st[0], st[1] = np.cos(q * x0), np.sin(q * x0)
    F = 2 * (math.cos(q) - 1) / dx ** 2
    st[2], st[3] = -0.5 * deta * F * st[0], -0.5 * deta * F * st[1]
    st[7] = -deta * e0 ** 2 * math.sin(q) / dx
    m = oracle_mod.measure(p, st, 0)
    assert m["e_kin"] < 1e-25 and m["e_el"] < 1e-25
    assert abs(m["e_grad"] - N ** 3 * dx ** 3 * 2 * (1 - math.cos(q)) / dx ** 2) < 1e-12 * m["e_grad"]
    assert abs(m["v2_omega"]) < 1e-13


def test_equation_of_state_velocity_weighting(oracle_mod):
    """The sums are weighted by the Lagrangian density, which changes sign:
    phi = c uniform (potential energy everywhere) with a centred momentum
    Pi_bar = (u, 0) in the lower half of the box only.  Per site, lower half:
    rho = u^2 + V, p = u^2 - V, L = u^2 - V; upper half: rho = V, p = -V,
    L = -V (V = lambda0/4 (c^2 - sigma^2)^2).  Weighting by rho or not at all
    gives other values."""
    N, dx, deta, lam, c, u = 6, 0.5, 0.1, 2.0, 0.5, 0.6
    p = oracle_mod.params(N=N, m=0.0, lambda0=lam, sigma=1.0, dx=dx, deta=deta)
    x0, x1, x2 = grid(N)
    lower = x2 < N // 2
    F = -0.5 * lam * (c * c - 1.0) * c      # force on Pi (real): -(lambda0/2)(|phi|^2 - sigma^2) phi
    st = np.zeros((10, N ** 3))
    st[0] = c
    st[2] = np.where(lower, u, 0.0) - 0.5 * deta * F
    m = oracle_mod.measure(p, st, 0)
    V = 0.25 * lam * (c * c - 1.0) ** 2
    rho_l, p_l, L_l = u * u + V, u * u - V, u * u - V
    rho_u, p_u, L_u = V, -V, -V
    w = (p_l * L_l + p_u * L_u) / (rho_l * L_l + rho_u * L_u)
    assert abs(m["v2_omega"] - 0.5 * (1 + 3 * w)) < 1e-12
    w_rho = (p_l * rho_l + p_u * rho_u) / (rho_l ** 2 + rho_u ** 2)
    w_flat = (p_l + p_u) / (rho_l + rho_u)
    assert abs(0.5 * (1 + 3 * w_rho) - m["v2_omega"]) > 0.1 and abs(0.5 * (1 + 3 * w_flat) - m["v2_omega"]) > 0.1


def test_nonfinite_counted(oracle_mod):
    N = 4
    p = oracle_mod.params(N=N)
    st = oracle_mod.init(p, 1)
    st[3, 5] = np.nan
    st[8, 9] = np.inf
    assert oracle_mod.measure(p, st, 0)["nonfinite"] == 2


def test_step_sites_matches_full_step(oracle_mod):
    N = 7
    p = oracle_mod.params(N=N, m=2.0)
    st = random_state(N, seed=51)
    full = oracle_mod.step(p, st, 4, 1)
    sites = np.array([0, 6, 48, 49, 342, 170, 57])
    out = oracle_mod.step_sites(p, st, 4, sites)
    assert np.array_equal(out, full[:, sites].T)
