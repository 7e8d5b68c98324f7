/*
 * ahref.c -- plain FP64 CPU oracle for the Abelian-Higgs leapfrog step.
 *
 * TEST INFRASTRUCTURE ONLY (see ahref.h).  Everything here is written
 * site by site straight from the equations of section 2 of Correia &
 * Martins: no blocking, no caching of links or plaquettes between sites,
 * no reordering.  Built with -O2 -fno-fast-math -ffp-contract=off so that
 * every expression is evaluated as written.  OpenMP only splits the site
 * loops over z-planes; every sum is formed per plane and then added in
 * plane order, so results do not depend on the thread count.
 */
#include "ahref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NC 10 /* reals per site */

/* double nearest to 2*pi */
static const double TWO_PI = 6.283185307179586;

/* ---------------------------------------------------------------- scalars */

/* Per-step scalars (section 2, damping coefficients and coupling scaling):
 * a(eta) = (eta/eta_ref)^m with m = d ln a / d ln eta, couplings scaled so
 * that lambda0 and e0^2 appear multiplied by f = a^(2s) in the discrete
 * equations, delta = (alpha/2) (d ln a / d ln eta) deta / eta and
 * omega = delta (1 - s). */
void ahref_scalars_at(const ahref_params* p, int64_t n, ahref_scalars* out)
{
    double eta = p->eta0 + (double)n * p->deta;
    double s = (eta < p->eta_switch) ? p->s_early : p->s_late;
    double a = pow(eta / p->eta_ref, p->m);
    double f = pow(a, 2.0 * s);
    double delta = 0.5 * p->alpha * p->m * p->deta / eta;
    /* artificial damping phase (section 2 mentions the capability): the
     * friction coefficient of the momentum equations is a constant gamma in
     * place of the Hubble term, so its Crank-Nicolson form has delta = gamma deta / 2 */
    if (p->damp_gamma > 0.0 && eta < p->eta_damp) delta = 0.5 * p->damp_gamma * p->deta;
    out->eta = eta;
    out->s = s;
    out->a = a;
    out->f = f;
    out->delta = delta;
    out->omega = (1.0 - s) * delta;
}

/* ------------------------------------------------------------------- RNG */

uint64_t ahref_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* ---------------------------------------------------------- lattice index */

static int64_t site(int N, int x0, int x1, int x2)
{
    return (int64_t)x0 + (int64_t)N * ((int64_t)x1 + (int64_t)N * (int64_t)x2);
}

/* index of x + s*k_d with periodic wrap */
static int64_t shifted(int N, const int x[3], int d, int s)
{
    int y[3] = {x[0], x[1], x[2]};
    y[d] = ((y[d] + s) % N + N) % N;
    return site(N, y[0], y[1], y[2]);
}

static void coords(int N, int64_t i, int x[3])
{
    x[0] = (int)(i % N);
    x[1] = (int)((i / N) % N);
    x[2] = (int)(i / ((int64_t)N * N));
}

/* field component c at site i */
#define FLD(st, V, c, i) ((st)[(int64_t)(c) * (V) + (i)])
#define PHR 0
#define PHI 1
#define PIR 2
#define PII 3
#define AA 4 /* A_j is component AA + j */
#define EE 7 /* E_j is component EE + j */

/* ------------------------------------------------------ links, plaquette */

/* U_j^y = exp(-i dx A_j^y) applied to the complex number (vr, vi) */
static void link_times(double dx, double Aj, double vr, double vi, double* wr, double* wi)
{
    double c = cos(dx * Aj);
    double s = -sin(dx * Aj);
    *wr = c * vr - s * vi;
    *wi = c * vi + s * vr;
}

/* conj(U_j^y) applied to (vr, vi) */
static void conj_link_times(double dx, double Aj, double vr, double vi, double* wr, double* wi)
{
    double c = cos(dx * Aj);
    double s = sin(dx * Aj);
    *wr = c * vr - s * vi;
    *wi = c * vi + s * vr;
}

/* plaquette angle Theta_ij^y = dx (A_i^y + A_j^{y+i} - A_i^{y+j} - A_j^y), i < j */
static double theta(const ahref_params* p, const double* st, int64_t V, const int y[3], int i, int j)
{
    int N = p->N;
    int64_t y0 = site(N, y[0], y[1], y[2]);
    int64_t yi = shifted(N, y, i, +1);
    int64_t yj = shifted(N, y, j, +1);
    double s = FLD(st, V, AA + i, y0) + FLD(st, V, AA + j, yi) - FLD(st, V, AA + i, yj) - FLD(st, V, AA + j, y0);
    return p->dx * s;
}

/* F_ij^y for any ordered pair i != j (antisymmetric) */
static double fstrength(const ahref_params* p, const double* st, int64_t V, const int y[3], int i, int j)
{
    double dx2 = p->dx * p->dx;
    int lo = i < j ? i : j, hi = i < j ? j : i;
    double th = theta(p, st, V, y, lo, hi);
    double F = p->compact ? sin(th) / dx2 : th / dx2;
    return (i < j) ? F : -F;
}

/* ------------------------------------------------------------------ kick */

/* Forces at site x of snapshot (section 2, kick equations):
 *   force_pi = D_j^- D_j^+ phi - (lambda0/2) f (|phi|^2 - sigma^2) phi
 *   force_E_i = -sum_{j != i} (F_ij^x - F_ij^{x-j})/dx + 2 e0^2 f Im[phi^* D_i^+ phi]
 * with the covariant Laplacian and D_i^+ phi built from the links. */
static void site_forces(const ahref_params* p, const ahref_scalars* sc, const double* st,
                        int64_t V, const int x[3], double fpi[2], double fe[3])
{
    int N = p->N;
    double dx = p->dx, dx2 = dx * dx;
    int64_t i0 = site(N, x[0], x[1], x[2]);
    double pr = FLD(st, V, PHR, i0), pim = FLD(st, V, PHI, i0);

    /* covariant Laplacian: sum_j [U_j^x phi^{x+j} - 2 phi^x + conj(U_j^{x-j}) phi^{x-j}] / dx^2 */
    double lr = 0.0, li = 0.0;
    for (int j = 0; j < 3; ++j) {
        int64_t ip = shifted(N, x, j, +1);
        int64_t im = shifted(N, x, j, -1);
        double t1r, t1i, t2r, t2i;
        link_times(dx, FLD(st, V, AA + j, i0), FLD(st, V, PHR, ip), FLD(st, V, PHI, ip), &t1r, &t1i);
        conj_link_times(dx, FLD(st, V, AA + j, im), FLD(st, V, PHR, im), FLD(st, V, PHI, im), &t2r, &t2i);
        lr += t1r - 2.0 * pr + t2r;
        li += t1i - 2.0 * pim + t2i;
    }
    lr /= dx2;
    li /= dx2;
    double pot = 0.5 * p->lambda0 * sc->f * (pr * pr + pim * pim - p->sigma * p->sigma);
    fpi[0] = lr - pot * pr;
    fpi[1] = li - pot * pim;

    for (int i = 0; i < 3; ++i) {
        /* current J_i = Im[conj(phi^x) U_i^x phi^{x+i}] / dx */
        int64_t ip = shifted(N, x, i, +1);
        double wr, wi;
        link_times(dx, FLD(st, V, AA + i, i0), FLD(st, V, PHR, ip), FLD(st, V, PHI, ip), &wr, &wi);
        double J = (pr * wi - pim * wr) / dx;
        /* lattice curl: sum_{j != i} (F_ij^x - F_ij^{x-j}) / dx */
        double C = 0.0;
        for (int j = 0; j < 3; ++j) {
            if (j == i) continue;
            int xm[3] = {x[0], x[1], x[2]};
            xm[j] = (xm[j] - 1 + N) % N;
            C += (fstrength(p, st, V, x, i, j) - fstrength(p, st, V, xm, i, j)) / dx;
        }
        fe[i] = -C + 2.0 * p->e0 * p->e0 * sc->f * J;
    }
}

/* Crank-Nicolson kick at one site:
 * (1+delta) Pi^+ = (1-delta) Pi^- + deta force_pi ; same for E with omega */
static void site_kick(const ahref_params* p, const ahref_scalars* sc, const double* st,
                      int64_t V, const int x[3], double pi_out[2], double e_out[3])
{
    double fpi[2], fe[3];
    int64_t i0 = site(p->N, x[0], x[1], x[2]);
    site_forces(p, sc, st, V, x, fpi, fe);
    for (int c = 0; c < 2; ++c)
        pi_out[c] = ((1.0 - sc->delta) * FLD(st, V, PIR + c, i0) + p->deta * fpi[c]) / (1.0 + sc->delta);
    for (int c = 0; c < 3; ++c)
        e_out[c] = ((1.0 - sc->omega) * FLD(st, V, EE + c, i0) + p->deta * fe[c]) / (1.0 + sc->omega);
}

void ahref_kick(const ahref_params* p, const double* st, int64_t n, double* pi_new, double* e_new)
{
    int N = p->N;
    int64_t V = (int64_t)N * N * N;
    ahref_scalars sc;
    ahref_scalars_at(p, n, &sc);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < N; ++z) {
        for (int y = 0; y < N; ++y) {
            for (int xx = 0; xx < N; ++xx) {
                int x[3] = {xx, y, z};
                int64_t i0 = site(N, xx, y, z);
                double po[2], eo[3];
                site_kick(p, &sc, st, V, x, po, eo);
                pi_new[i0] = po[0];
                pi_new[V + i0] = po[1];
                for (int c = 0; c < 3; ++c) e_new[(int64_t)c * V + i0] = eo[c];
            }
        }
    }
}

/* one full step: kick every site from the snapshot, then drift
 * phi^{n+1} = phi^n + deta Pi^{n+1/2}, A^{n+1} = A^n + deta E^{n+1/2} */
void ahref_step(const ahref_params* p, double* st, int64_t n0, int64_t nsteps)
{
    int N = p->N;
    int64_t V = (int64_t)N * N * N;
    double* pin = (double*)malloc(sizeof(double) * 2 * V);
    double* en = (double*)malloc(sizeof(double) * 3 * V);
    for (int64_t n = n0; n < n0 + nsteps; ++n) {
        ahref_kick(p, st, n, pin, en);
#pragma omp parallel for schedule(static)
        for (int z = 0; z < N; ++z) {
            for (int64_t i = (int64_t)z * N * N; i < (int64_t)(z + 1) * N * N; ++i) {
                for (int c = 0; c < 2; ++c) {
                    FLD(st, V, PIR + c, i) = pin[(int64_t)c * V + i];
                    FLD(st, V, PHR + c, i) = FLD(st, V, PHR + c, i) + p->deta * pin[(int64_t)c * V + i];
                }
                for (int c = 0; c < 3; ++c) {
                    FLD(st, V, EE + c, i) = en[(int64_t)c * V + i];
                    FLD(st, V, AA + c, i) = FLD(st, V, AA + c, i) + p->deta * en[(int64_t)c * V + i];
                }
            }
        }
    }
    free(pin);
    free(en);
}

void ahref_step_sites(const ahref_params* p, const double* st, int64_t n,
                      const int64_t* sites, int64_t count, double* out)
{
    int N = p->N;
    int64_t V = (int64_t)N * N * N;
    ahref_scalars sc;
    ahref_scalars_at(p, n, &sc);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k) {
        int x[3];
        coords(N, sites[k], x);
        double po[2], eo[3];
        site_kick(p, &sc, st, V, x, po, eo);
        double* o = out + NC * k;
        int64_t i0 = sites[k];
        o[PHR] = FLD(st, V, PHR, i0) + p->deta * po[0];
        o[PHI] = FLD(st, V, PHI, i0) + p->deta * po[1];
        o[PIR] = po[0];
        o[PII] = po[1];
        for (int c = 0; c < 3; ++c) {
            o[AA + c] = FLD(st, V, AA + c, i0) + p->deta * eo[c];
            o[EE + c] = eo[c];
        }
    }
}

/* -------------------------------------------------------------------- IC */

void ahref_init(const ahref_params* p, uint64_t seed, double* st)
{
    int N = p->N;
    int64_t V = (int64_t)N * N * N;
    memset(st, 0, sizeof(double) * NC * V);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < N; ++z) {
        for (int64_t i = (int64_t)z * N * N; i < (int64_t)(z + 1) * N * N; ++i) {
            double u = (double)(ahref_splitmix64(seed, (uint64_t)i) >> 11) * 0x1.0p-53;
            double th = u * TWO_PI;
            FLD(st, V, PHR, i) = p->sigma * cos(th);
            FLD(st, V, PHI, i) = p->sigma * sin(th);
        }
    }
}

/* --------------------------------------------------------------- winding */

/* gauge-invariant link phase Y_i(y) = arg(conj(phi^y) U_i^y phi^{y+i}) in (-pi, pi];
 * adding +0.0 to the imaginary part turns -0 into +0 so the cut maps to +pi */
static double link_phase(const ahref_params* p, const double* st, int64_t V, const int y[3], int i)
{
    int64_t y0 = site(p->N, y[0], y[1], y[2]);
    int64_t yi = shifted(p->N, y, i, +1);
    double wr, wi;
    link_times(p->dx, FLD(st, V, AA + i, y0), FLD(st, V, PHR, yi), FLD(st, V, PHI, yi), &wr, &wi);
    double pr = FLD(st, V, PHR, y0), pim = FLD(st, V, PHI, y0);
    double zr = pr * wr + pim * wi;
    double zi = pr * wi - pim * wr;
    return atan2(zi + 0.0, zr);
}

/* winding through plaquette (i,j) at y, i < j (lattice winding after
 * Kajantie et al.): the sum of the gauge-invariant link phases around the
 * plaquette plus the plaquette angle wrapped to (-pi, pi] is a multiple of
 * 2 pi; the multiple is the winding. */
static int32_t plaquette_winding(const ahref_params* p, const double* st, int64_t V, const int y[3], int i, int j)
{
    int N = p->N;
    int yi[3] = {y[0], y[1], y[2]};
    int yj[3] = {y[0], y[1], y[2]};
    yi[i] = (yi[i] + 1) % N;
    yj[j] = (yj[j] + 1) % N;
    double Y1 = link_phase(p, st, V, y, i);
    double Y2 = link_phase(p, st, V, yi, j);
    double Y3 = link_phase(p, st, V, yj, i);
    double Y4 = link_phase(p, st, V, y, j);
    double th = theta(p, st, V, y, i, j);
    double thw = p->compact ? th - TWO_PI * rint(th / TWO_PI) : th;
    double sum = (((Y1 + Y2) - Y3) - Y4) + thw;
    return (int32_t)rint(sum / TWO_PI);
}

static const int PAIRS[3][2] = {{0, 1}, {0, 2}, {1, 2}};

void ahref_winding(const ahref_params* p, const double* st, int32_t* W)
{
    int N = p->N;
    int64_t V = (int64_t)N * N * N;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < N; ++z) {
        for (int y = 0; y < N; ++y) {
            for (int xx = 0; xx < N; ++xx) {
                int x[3] = {xx, y, z};
                int64_t i0 = site(N, xx, y, z);
                for (int q = 0; q < 3; ++q) W[(int64_t)q * V + i0] = plaquette_winding(p, st, V, x, PAIRS[q][0], PAIRS[q][1]);
            }
        }
    }
}

void ahref_winding_sites(const ahref_params* p, const double* st, const int64_t* sites, int64_t count, int32_t* W)
{
    int N = p->N;
    int64_t V = (int64_t)N * N * N;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k) {
        int x[3];
        coords(N, sites[k], x);
        for (int q = 0; q < 3; ++q) W[3 * k + q] = plaquette_winding(p, st, V, x, PAIRS[q][0], PAIRS[q][1]);
    }
}

/* ----------------------------------------------------------------- Gauss */

/* Discrete Gauss law on snapshot n (section 2, Gauss's law with the
 * scaled coupling): G^x = sum_i (E_i^x - E_i^{x-i})/dx - c Im[conj(phi^x) Pi^x]
 * with the stored half-step E and Pi.  The kick preserves G = 0 exactly
 * when c_{n-1/2} = 2 e0^2 f_{n-1} (1+delta_{n-1})/(1+omega_{n-1}); for n = 0
 * c = 2 e0^2 f_0. */
static double gauss_coupling(const ahref_params* p, int64_t n)
{
    ahref_scalars sc;
    if (n <= 0) {
        ahref_scalars_at(p, 0, &sc);
        return 2.0 * p->e0 * p->e0 * sc.f;
    }
    ahref_scalars_at(p, n - 1, &sc);
    return 2.0 * p->e0 * p->e0 * sc.f * (1.0 + sc.delta) / (1.0 + sc.omega);
}

static void site_gauss(const ahref_params* p, const double* st, int64_t V, const int x[3], double c,
                       double* G, double* divE, double* crho)
{
    int N = p->N;
    int64_t i0 = site(N, x[0], x[1], x[2]);
    double d = 0.0;
    for (int i = 0; i < 3; ++i) {
        int64_t im = shifted(N, x, i, -1);
        d += (FLD(st, V, EE + i, i0) - FLD(st, V, EE + i, im)) / p->dx;
    }
    double rho = FLD(st, V, PHR, i0) * FLD(st, V, PII, i0) - FLD(st, V, PHI, i0) * FLD(st, V, PIR, i0);
    *divE = d;
    *crho = c * rho;
    *G = d - c * rho;
}

void ahref_gauss(const ahref_params* p, const double* st, int64_t n, double* G)
{
    int N = p->N;
    int64_t V = (int64_t)N * N * N;
    double c = gauss_coupling(p, n);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < N; ++z) {
        for (int y = 0; y < N; ++y) {
            for (int xx = 0; xx < N; ++xx) {
                int x[3] = {xx, y, z};
                double dv, cr;
                site_gauss(p, st, V, x, c, &G[site(N, xx, y, z)], &dv, &cr);
            }
        }
    }
}

/* ----------------------------------------------------------- measurement */

enum {
    S_KIN, S_GRAD, S_POT, S_EL, S_MAG, S_L, S_KINL, S_GRADL,
    S_G2, S_DIV2, S_CRHO2, S_GMAX, S_WABS, S_NONFIN, S_PL, S_RHOL, S_COUNT
};

/* Site densities of snapshot n with centred momenta (the average of the
 * stored Pi^{n-1/2}, E^{n-1/2} and the kicked Pi^{n+1/2}, E^{n+1/2}),
 * forward covariant differences D_i^+ phi = (U_i phi^{x+i} - phi^x)/dx and
 * forward plaquettes:
 *   kinetic |Pi|^2, gradient sum_i |D_i^+ phi|^2, potential (lambda0 f/4)(|phi|^2-sigma^2)^2,
 *   electric sum_i E_i^2 / (2 e0^2 f), magnetic sum_{i<j} B_ij^2 / (2 e0^2 f)
 *   with B^2 = 2 (1 - cos Theta)/dx^4 (compact) or Theta^2/dx^4.
 * The Lagrangian density is kin - grad - pot + el - mag, the energy density
 * rho = kin + grad + pot + el + mag, and the pressure p (a third of the trace
 * of the spatial stress tensor of the scalar and gauge fields)
 * p = kin - grad/3 - pot + (el + mag)/3. */
static void site_measure(const ahref_params* p, const ahref_scalars* sc, const double* st, int64_t V,
                         const int x[3], double gc, double acc[S_COUNT])
{
    int N = p->N;
    double dx = p->dx, dx2 = dx * dx, dx4 = dx2 * dx2;
    int64_t i0 = site(N, x[0], x[1], x[2]);

    int bad = 0;
    for (int c = 0; c < NC; ++c)
        if (!isfinite(FLD(st, V, c, i0))) bad = 1;
    acc[S_NONFIN] += bad;

    double pin[2], en[3];
    site_kick(p, sc, st, V, x, pin, en);
    double pbr = 0.5 * (FLD(st, V, PIR, i0) + pin[0]);
    double pbi = 0.5 * (FLD(st, V, PII, i0) + pin[1]);
    double kin = pbr * pbr + pbi * pbi;

    double pr = FLD(st, V, PHR, i0), pim = FLD(st, V, PHI, i0);
    double grad = 0.0;
    for (int i = 0; i < 3; ++i) {
        int64_t ip = shifted(N, x, i, +1);
        double wr, wi;
        link_times(dx, FLD(st, V, AA + i, i0), FLD(st, V, PHR, ip), FLD(st, V, PHI, ip), &wr, &wi);
        double dr = (wr - pr) / dx, di = (wi - pim) / dx;
        grad += dr * dr + di * di;
    }
    double m2 = pr * pr + pim * pim - p->sigma * p->sigma;
    double pot = 0.25 * p->lambda0 * sc->f * m2 * m2;

    double inv2e2f = 1.0 / (2.0 * p->e0 * p->e0 * sc->f);
    double el = 0.0;
    for (int i = 0; i < 3; ++i) {
        double eb = 0.5 * (FLD(st, V, EE + i, i0) + en[i]);
        el += eb * eb;
    }
    el *= inv2e2f;
    double mag = 0.0;
    for (int q = 0; q < 3; ++q) {
        double th = theta(p, st, V, x, PAIRS[q][0], PAIRS[q][1]);
        mag += p->compact ? 2.0 * (1.0 - cos(th)) / dx4 : th * th / dx4;
    }
    mag *= inv2e2f;

    double L = kin - grad - pot + el - mag;
    double rho = kin + grad + pot + el + mag;
    double pres = kin - grad / 3.0 - pot + (el + mag) / 3.0;
    acc[S_PL] += pres * L;
    acc[S_RHOL] += rho * L;
    acc[S_KIN] += kin;
    acc[S_GRAD] += grad;
    acc[S_POT] += pot;
    acc[S_EL] += el;
    acc[S_MAG] += mag;
    acc[S_L] += L;
    acc[S_KINL] += kin * L;
    acc[S_GRADL] += grad * L;

    double G, dv, cr;
    site_gauss(p, st, V, x, gc, &G, &dv, &cr);
    acc[S_G2] += G * G;
    acc[S_DIV2] += dv * dv;
    acc[S_CRHO2] += cr * cr;
    if (fabs(G) > acc[S_GMAX]) acc[S_GMAX] = fabs(G);

    for (int q = 0; q < 3; ++q) {
        int32_t w = plaquette_winding(p, st, V, x, PAIRS[q][0], PAIRS[q][1]);
        acc[S_WABS] += (double)(w < 0 ? -w : w);
    }
}

void ahref_measure(const ahref_params* p, const double* st, int64_t n, ahref_meas* out)
{
    int N = p->N;
    int64_t V = (int64_t)N * N * N;
    ahref_scalars sc;
    ahref_scalars_at(p, n, &sc);
    double gc = gauss_coupling(p, n);
    double* plane = (double*)calloc((size_t)N * S_COUNT, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < N; ++z) {
        double* acc = plane + (size_t)z * S_COUNT;
        for (int y = 0; y < N; ++y) {
            for (int xx = 0; xx < N; ++xx) {
                int x[3] = {xx, y, z};
                site_measure(p, &sc, st, V, x, gc, acc);
            }
        }
    }
    double tot[S_COUNT];
    for (int k = 0; k < S_COUNT; ++k) tot[k] = 0.0;
    for (int z = 0; z < N; ++z) {
        for (int k = 0; k < S_COUNT; ++k) {
            if (k == S_GMAX) {
                if (plane[(size_t)z * S_COUNT + k] > tot[k]) tot[k] = plane[(size_t)z * S_COUNT + k];
            } else {
                tot[k] += plane[(size_t)z * S_COUNT + k];
            }
        }
    }
    free(plane);

    double dx3 = p->dx * p->dx * p->dx;
    double vol = pow((double)N * p->dx, 3.0);
    memset(out, 0, sizeof(*out));
    out->step = n;
    out->eta = sc.eta;
    out->a = sc.a;
    out->f = sc.f;
    out->winding_sum_abs = (int64_t)tot[S_WABS];
    out->L_W = p->dx * tot[S_WABS];
    out->xi_W = sqrt(vol / out->L_W);
    out->e_kin = dx3 * tot[S_KIN];
    out->e_grad = dx3 * tot[S_GRAD];
    out->e_pot = dx3 * tot[S_POT];
    out->e_el = dx3 * tot[S_EL];
    out->e_mag = dx3 * tot[S_MAG];
    out->energy = out->e_kin + out->e_grad + out->e_pot + out->e_el + out->e_mag;
    out->sum_L = dx3 * tot[S_L];
    /* xi_L = sqrt(-mu V / sum_x L_x) with mu = 2 pi sigma^2 */
    out->xi_L = (out->sum_L < 0.0) ? sqrt(-TWO_PI * p->sigma * p->sigma * vol / out->sum_L) : NAN;
    out->R = tot[S_KINL] / tot[S_GRADL];
    out->v2_phi = 2.0 * out->R / (1.0 + out->R);
    /* equation-of-state estimator (section 2): w = sum p W / sum rho W with
     * the Lagrangian density as the weight W, <v^2>_omega = (1 + 3 w)/2 */
    out->v2_omega = 0.5 * (1.0 + 3.0 * tot[S_PL] / tot[S_RHOL]);
    out->gauss_rms = sqrt(tot[S_G2] / (double)V);
    out->gauss_max = tot[S_GMAX];
    double den = sqrt(tot[S_DIV2] + tot[S_CRHO2]);
    out->gauss_rel = den > 0.0 ? sqrt(tot[S_G2]) / den : 0.0;
    out->nonfinite = (int64_t)tot[S_NONFIN];
}

int ahref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ahref_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
