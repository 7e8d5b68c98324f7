/*
 * ahref.h -- plain FP64 CPU oracle for the Abelian-Higgs leapfrog step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference
 * that the GPU library is checked against.  It shares no code, header,
 * constant or helper with the GPU library, and the GPU library never calls
 * it.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it.
 *
 * What it computes (Correia & Martins, "Abelian-Higgs cosmic string
 * evolution with multiple GPUs", section 2):
 *   - the staggered leapfrog / Crank-Nicolson update of the scalar momentum
 *     Pi and the electric field E (the two kick equations of section 2),
 *     followed by the drift of phi and A (the two drift equations);
 *   - the link variables U_j = exp(-i dx A_j), the covariant Laplacian
 *     stencil and the plaquette field strength of section 2;
 *   - the diagnostics of section 2: the Lagrangian string-separation
 *     estimator xi_L, the winding estimator xi_W and the Lagrangian-weighted
 *     velocity <v^2>_phi, plus the energy and the discrete Gauss-law
 *     residual.
 *
 * Conventions (the paper is garbled or silent in places; the readings taken
 * are listed in the design notes of the repository):
 *   lattice  x = (x0,x1,x2) in Z_N^3, periodic; idx = x0 + N*(x1 + N*x2)
 *   state    10 arrays of N^3 doubles, in this order:
 *              phi_re, phi_im, pi_re, pi_im, A0, A1, A2, E0, E1, E2
 *            snapshot n: phi, A at eta_n = eta0 + n*deta; Pi, E at eta_n - deta/2
 *   a(eta) = (eta/eta_ref)^m, f = a^(2s), delta = (alpha/2) m deta/eta,
 *   omega = (1-s) delta, s = s_early for eta < eta_switch else s_late.
 */
#ifndef AHREF_H
#define AHREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ahref_params {
    int32_t N;          /* periodic N^3 lattice */
    int32_t compact;    /* 1: F = sin(Theta)/dx^2 ; 0: F = Theta/dx^2 */
    double dx, deta;
    double lambda0, e0, sigma;
    double m;           /* d ln a / d ln eta: 0 flat, 1 radiation, 2 matter */
    double alpha;       /* damping multiplier; 2 gives Crank-Nicolson Hubble friction */
    double s_early, s_late, eta_switch;
    double eta0, eta_ref;
    double damp_gamma;  /* artificial damping phase: friction gamma for eta < eta_damp (0: none) */
    double eta_damp;
} ahref_params;

typedef struct ahref_scalars {
    double eta, s, a, f, delta, omega;
} ahref_scalars;

typedef struct ahref_meas {
    int64_t step;
    double eta, a, f;
    int64_t winding_sum_abs;   /* sum over sites and the 3 orientations of |W| */
    double L_W, xi_W;
    double sum_L, xi_L, R, v2_phi;
    double energy, e_kin, e_grad, e_pot, e_el, e_mag;
    double gauss_rms, gauss_max, gauss_rel;
    int64_t nonfinite;         /* sites with any non-finite field value */
    double v2_omega;           /* equation-of-state velocity estimator */
} ahref_meas;

/* per-step scalars at snapshot n (eta_n = eta0 + n*deta) */
void ahref_scalars_at(const ahref_params* p, int64_t n, ahref_scalars* out);

/* k-th output (k = 0, 1, ...) of SplitMix64 seeded with `seed`:
 * mix(seed + (k+1)*0x9e3779b97f4a7c15) (Steele, Lea & Flood, 2014). */
uint64_t ahref_splitmix64(uint64_t seed, uint64_t k);

/* random-phase initial condition (section 2): phi = sigma*exp(2 pi i u),
 * u = (splitmix64(seed, idx) >> 11) * 2^-53 ; Pi = A = E = 0. */
void ahref_init(const ahref_params* p, uint64_t seed, double* st);

/* kick at snapshot n: Pi^{n+1/2} (2 N^3) and E^{n+1/2} (3 N^3); st unchanged */
void ahref_kick(const ahref_params* p, const double* st, int64_t n,
                double* pi_new, double* e_new);

/* advance st from snapshot n0 by nsteps full steps (kick then drift) */
void ahref_step(const ahref_params* p, double* st, int64_t n0, int64_t nsteps);

/* one step from snapshot n evaluated at `count` listed sites only:
 * out[10*k + c] is component c (state order) of site sites[k] at n+1 */
void ahref_step_sites(const ahref_params* p, const double* st, int64_t n,
                      const int64_t* sites, int64_t count, double* out);

/* plaquette windings W (3 N^3 int32; orientation (0,1), (0,2), (1,2)) */
void ahref_winding(const ahref_params* p, const double* st, int32_t* W);

/* windings of the 3 plaquettes based at each listed site: W[3*k + q] */
void ahref_winding_sites(const ahref_params* p, const double* st, const int64_t* sites, int64_t count, int32_t* W);

/* Gauss residual per site at snapshot n (N^3 doubles) */
void ahref_gauss(const ahref_params* p, const double* st, int64_t n, double* G);

/* all diagnostics of snapshot n */
void ahref_measure(const ahref_params* p, const double* st, int64_t n, ahref_meas* out);

/* OpenMP threads the oracle runs with */
int ahref_num_threads(void);

/* threads for the oracle's later calls (n > 0) */
void ahref_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
