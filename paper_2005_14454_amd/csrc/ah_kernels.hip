// HIP kernels of libah for gfx950: random-phase initial condition, the
// site-parallel reference step, the FP64 diagnostics with their fixed-order
// two-stage reduction, and the per-plaquette winding field.
//
// Discretisation (Correia & Martins, section 2): staggered leapfrog with
// Crank-Nicolson damping; links U_j = exp(-i dx A_j); covariant Laplacian;
// compact plaquette field strength F_ij = sin(Theta_ij)/dx^2.
#include "ah_device.h"
#include "ah_internal.h"

#include <cmath>

namespace ah {
namespace {

// ------------------------------------------------------------ small helpers

// Side and row pitch of the stored lattice: site (x, y, z) is element
// x + P (y + N z) of every field.
struct Dims {
    int N, P;
};
__device__ inline int64_t sidx(Dims D, int x, int y, int z)
{
    return (int64_t)x + (int64_t)D.P * ((int64_t)y + (int64_t)D.N * (int64_t)z);
}
__device__ inline int up(int v, int N) { return v + 1 == N ? 0 : v + 1; }
__device__ inline int dn(int v, int N) { return v == 0 ? N - 1 : v - 1; }

__device__ inline void sincos_t(double x, double* s, double* c) { sincos(x, s, c); }
__device__ inline void sincos_t(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ inline double sin_t(double x) { return sin(x); }
__device__ inline float sin_t(float x) { return sinf(x); }

template <typename R>
__device__ inline const R* gauge(const Fields<R>& f, int d) { return d == 0 ? f.a0 : (d == 1 ? f.a1 : f.a2); }
template <typename R>
__device__ inline const R* elec(const Fields<R>& f, int d) { return d == 0 ? f.e0 : (d == 1 ? f.e1 : f.e2); }

struct C3 {
    int v[3];
};
__device__ inline C3 shift(C3 c, int d, int N, int s)
{
    c.v[d] = s > 0 ? up(c.v[d], N) : dn(c.v[d], N);
    return c;
}
__device__ inline int64_t at(Dims D, const C3& c) { return sidx(D, c.v[0], c.v[1], c.v[2]); }
// coordinates of the dense site index s = x + N (y + N z)
__device__ inline C3 coords(int N, int64_t s)
{
    return C3{{(int)(s % N), (int)((s / N) % N), (int)(s / ((int64_t)N * N))}};
}

// F_ij at site c for an ordered pair i != j, in arithmetic type T
template <typename T, typename R>
__device__ inline T fstrength(const Fields<R>& f, Dims D, int compact, T dx, T inv_dx2, const C3& c, int i, int j)
{
    const int N = D.N;
    int lo = i < j ? i : j, hi = i < j ? j : i;
    const R* Al = gauge(f, lo);
    const R* Ah = gauge(f, hi);
    T th = dx * ((((T)Al[at(D, c)] + (T)Ah[at(D, shift(c, lo, N, 1))]) - (T)Al[at(D, shift(c, hi, N, 1))]) -
                 (T)Ah[at(D, c)]);
    T F = compact ? sin_t(th) * inv_dx2 : th * inv_dx2;
    return i < j ? F : -F;
}

// Kick of Pi and E at one site (section 2, the two Crank-Nicolson kick
// equations) evaluated in arithmetic type T from fields stored as R.
template <typename T, typename R>
__device__ inline void kick_site(const Fields<R>& f, Dims D, int compact, T dx, T sigma2, T cP1, T cP2, T cE1,
                                 T cE2, T lamh, T kappa, const C3& c, T pin[2], T en[3])
{
    const int N = D.N;
    const T inv_dx = (T)1 / dx, inv_dx2 = inv_dx * inv_dx;
    const int64_t i0 = at(D, c);
    const T pr = (T)f.phr[i0], pim = (T)f.phi[i0];
    T lr = 0, li = 0;
    T t1r[3], t1i[3];
    for (int d = 0; d < 3; ++d) {
        const R* Ad = gauge(f, d);
        const int64_t ip = at(D, shift(c, d, N, 1));
        const int64_t im = at(D, shift(c, d, N, -1));
        T s, co;
        sincos_t(dx * (T)Ad[i0], &s, &co);  // U = co - i s
        const T fr = (T)f.phr[ip], fi = (T)f.phi[ip];
        t1r[d] = co * fr + s * fi;
        t1i[d] = co * fi - s * fr;
        T sm, cm;
        sincos_t(dx * (T)Ad[im], &sm, &cm);  // conj U = cm + i sm
        const T gr = (T)f.phr[im], gi = (T)f.phi[im];
        const T t2r = cm * gr - sm * gi, t2i = cm * gi + sm * gr;
        lr += (t1r[d] - (T)2 * pr) + t2r;
        li += (t1i[d] - (T)2 * pim) + t2i;
    }
    const T pot = lamh * (pr * pr + pim * pim - sigma2);
    pin[0] = cP1 * (T)f.pir[i0] + cP2 * (lr * inv_dx2 - pot * pr);
    pin[1] = cP1 * (T)f.pii[i0] + cP2 * (li * inv_dx2 - pot * pim);
    for (int i = 0; i < 3; ++i) {
        const T J = (pr * t1i[i] - pim * t1r[i]) * inv_dx;
        T C = 0;
        for (int j = 0; j < 3; ++j) {
            if (j == i) continue;
            C += fstrength<T>(f, D, compact, dx, inv_dx2, c, i, j) -
                 fstrength<T>(f, D, compact, dx, inv_dx2, shift(c, j, N, -1), i, j);
        }
        en[i] = cE1 * (T)elec(f, i)[i0] + cE2 * (kappa * J - C * inv_dx);
    }
}

// ------------------------------------------------------------------ kernels

__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t k)
{
    // k-th output of SplitMix64 (Steele, Lea & Flood 2014): mix(seed + (k+1) gamma)
    uint64_t z = seed + (k + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

template <typename R>
__global__ void __launch_bounds__(256) k_init(Fields<R> f, Dims D, double sigma, uint64_t seed)
{
    // the phase of site k = x + N (y + N z) is output k of the generator
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)D.N * D.N * D.N) return;
    const int64_t i = at(D, coords(D.N, k));
    const double u = (double)(splitmix64(seed, (uint64_t)k) >> 11) * 0x1.0p-53;
    const double th = u * 6.283185307179586;
    double s, c;
    sincos(th, &s, &c);
    f.phr[i] = (R)(sigma * c);
    f.phi[i] = (R)(sigma * s);
    f.pir[i] = (R)0;
    f.pii[i] = (R)0;
    f.a0[i] = (R)0;
    f.a1[i] = (R)0;
    f.a2[i] = (R)0;
    f.e0[i] = (R)0;
    f.e1[i] = (R)0;
    f.e2[i] = (R)0;
}

// Site-parallel step: one thread per site, every neighbour read from global
// memory.  Kick of Pi and E in place, drift of phi and A into the other
// ping-pong buffer.
template <typename R>
__global__ void __launch_bounds__(256) k_step_site(Fields<R> f, R* __restrict__ ophr, R* __restrict__ ophi,
                                                   R* __restrict__ oa0, R* __restrict__ oa1, R* __restrict__ oa2,
                                                   Dims D, int compact, R dx, R sigma2, R cP1, R cP2, R cE1, R cE2,
                                                   R lamh, R kappa, R deta)
{
    const int N = D.N;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= N || y >= N) return;
    C3 c{{x, y, z}};
    R pin[2], en[3];
    kick_site<R>(f, D, compact, dx, sigma2, cP1, cP2, cE1, cE2, lamh, kappa, c, pin, en);
    const int64_t i0 = at(D, c);
    ophr[i0] = f.phr[i0] + deta * pin[0];
    ophi[i0] = f.phi[i0] + deta * pin[1];
    oa0[i0] = f.a0[i0] + deta * en[0];
    oa1[i0] = f.a1[i0] + deta * en[1];
    oa2[i0] = f.a2[i0] + deta * en[2];
    f.pir[i0] = pin[0];
    f.pii[i0] = pin[1];
    f.e0[i0] = en[0];
    f.e1[i0] = en[1];
    f.e2[i0] = en[2];
}

// ---------------------------------------------------------------- windings

// Gauge-invariant link phase arg(conj(phi^c) U_i^c phi^{c+i}) in (-pi, pi],
// FP64 without contraction so that identical snapshots give identical bits
// up to the last-ulp differences of the link cosine and sine.
template <typename R>
__device__ double link_phase(const Fields<R>& f, Dims D, double dx, const C3& c, int i)
{
#pragma clang fp contract(off)
    const int64_t i0 = at(D, c);
    const int64_t ip = at(D, shift(c, i, D.N, 1));
    double s, co;
    sincos(dx * (double)gauge(f, i)[i0], &s, &co);
    const double ur = co, ui = -s;
    const double vr = (double)f.phr[ip], vi = (double)f.phi[ip];
    const double wr = ur * vr - ui * vi;
    const double wi = ur * vi + ui * vr;
    const double pr = (double)f.phr[i0], pim = (double)f.phi[i0];
    const double zr = pr * wr + pim * wi;
    double zi = pr * wi - pim * wr;
    zi = (zi == 0.0) ? 0.0 : zi;  // -0 -> +0: the branch cut maps to +pi
    return atan2(zi, zr);
}

// Winding through plaquette (i<j) at c: link phases around the plaquette plus
// the plaquette angle wrapped to (-pi, pi] form a multiple of 2 pi.
template <typename R>
__device__ int plaquette_winding(const Fields<R>& f, Dims D, int compact, double dx, const C3& c, int i, int j)
{
#pragma clang fp contract(off)
    const int N = D.N;
    const double two_pi = 6.283185307179586;
    const C3 ci = shift(c, i, N, 1), cj = shift(c, j, N, 1);
    const double Y1 = link_phase(f, D, dx, c, i);
    const double Y2 = link_phase(f, D, dx, ci, j);
    const double Y3 = link_phase(f, D, dx, cj, i);
    const double Y4 = link_phase(f, D, dx, c, j);
    const double a = (double)gauge(f, i)[at(D, c)];
    const double b = (double)gauge(f, j)[at(D, ci)];
    const double cc = (double)gauge(f, i)[at(D, cj)];
    const double d = (double)gauge(f, j)[at(D, c)];
    const double th = dx * (((a + b) - cc) - d);
    const double thw = compact ? th - two_pi * rint(th / two_pi) : th;
    const double sum = (((Y1 + Y2) - Y3) - Y4) + thw;
    return (int)rint(sum / two_pi);
}

template <typename R>
__global__ void __launch_bounds__(256) k_winding(Fields<R> f, Dims D, int compact, double dx, int8_t* __restrict__ w)
{
    // w is dense: plaquette (i, j) of site s at w[q V + s]
    const int64_t V = (int64_t)D.N * D.N * D.N;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < V; s += (int64_t)gridDim.x * blockDim.x) {
        const C3 c = coords(D.N, s);
        w[s] = (int8_t)plaquette_winding(f, D, compact, dx, c, 0, 1);
        w[V + s] = (int8_t)plaquette_winding(f, D, compact, dx, c, 0, 2);
        w[2 * V + s] = (int8_t)plaquette_winding(f, D, compact, dx, c, 1, 2);
    }
}

// ------------------------------------------------------------- diagnostics

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ inline double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// One pass over the snapshot in FP64: centred momenta from a kick that is not
// stored, site densities with forward links and plaquettes, Gauss residual,
// windings.  Each thread walks a fixed grid-stride set of sites; partial
// sums are reduced across the block in a fixed tree and stored per block.
template <typename R>
__global__ void __launch_bounds__(kMeasThreads) k_measure(Fields<R> f, Dims D, int compact, double dx, double sigma2,
                                                          StepCoef cf, MeasConst mc, double* __restrict__ partials)
{
    const int N = D.N;
    const int64_t V = (int64_t)N * N * N;
    const double inv_dx = 1.0 / dx, inv_dx2 = inv_dx * inv_dx, inv_dx4 = inv_dx2 * inv_dx2;
    double acc[M_COUNT];
    for (int k = 0; k < M_COUNT; ++k) acc[k] = 0.0;

    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < V; s += (int64_t)gridDim.x * blockDim.x) {
        const C3 c = coords(N, s);
        const int64_t o = at(D, c);
        const double v[10] = {(double)f.phr[o], (double)f.phi[o], (double)f.pir[o], (double)f.pii[o],
                              (double)f.a0[o],  (double)f.a1[o],  (double)f.a2[o],  (double)f.e0[o],
                              (double)f.e1[o],  (double)f.e2[o]};
        bool bad = false;
        for (int k = 0; k < 10; ++k) bad |= !isfinite(v[k]);
        acc[M_NONFIN] += bad ? 1.0 : 0.0;

        double pin[2], en[3];
        kick_site<double>(f, D, compact, dx, sigma2, cf.cP1, cf.cP2, cf.cE1, cf.cE2, cf.lam_half, cf.kappa, c, pin,
                          en);
        const double pbr = 0.5 * (v[2] + pin[0]), pbi = 0.5 * (v[3] + pin[1]);
        const double kin = pbr * pbr + pbi * pbi;

        const double pr = v[0], pim = v[1];
        double grad = 0.0;
        for (int i = 0; i < 3; ++i) {
            const int64_t ip = at(D, shift(c, i, N, 1));
            double sn, cs;
            sincos(dx * v[4 + i], &sn, &cs);
            const double fr = (double)f.phr[ip], fi = (double)f.phi[ip];
            const double dr = (cs * fr + sn * fi - pr) * inv_dx;
            const double di = (cs * fi - sn * fr - pim) * inv_dx;
            grad += dr * dr + di * di;
        }
        const double m2 = pr * pr + pim * pim - sigma2;
        const double pot = mc.lam_quarter * m2 * m2;
        double el = 0.0;
        for (int i = 0; i < 3; ++i) {
            const double eb = 0.5 * (v[7 + i] + en[i]);
            el += eb * eb;
        }
        el *= mc.inv_2e2f;
        double mag = 0.0;
        const int P[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (int q = 0; q < 3; ++q) {
            const int i = P[q][0], j = P[q][1];
            const double th = dx * ((((double)gauge(f, i)[o] + (double)gauge(f, j)[at(D, shift(c, i, N, 1))]) -
                                     (double)gauge(f, i)[at(D, shift(c, j, N, 1))]) -
                                    (double)gauge(f, j)[o]);
            mag += compact ? 2.0 * (1.0 - cos(th)) * inv_dx4 : th * th * inv_dx4;
        }
        mag *= mc.inv_2e2f;
        const double L = kin - grad - pot + el - mag;
        acc[M_KIN] += kin;
        acc[M_GRAD] += grad;
        acc[M_POT] += pot;
        acc[M_EL] += el;
        acc[M_MAG] += mag;
        acc[M_KINL] += kin * L;
        acc[M_GRADL] += grad * L;
        const double pres = (kin - pot) + ((el + mag) - grad) * (1.0 / 3.0);
        const double rho = ((kin + grad) + pot) + (el + mag);
        acc[M_PL] += pres * L;
        acc[M_RHOL] += rho * L;

        double dv = 0.0;
        for (int i = 0; i < 3; ++i) dv += (v[7 + i] - (double)elec(f, i)[at(D, shift(c, i, N, -1))]) * inv_dx;
        const double crho = mc.gauss_c * (pr * v[3] - pim * v[2]);
        const double G = dv - crho;
        acc[M_G2] += G * G;
        acc[M_DIV2] += dv * dv;
        acc[M_CRHO2] += crho * crho;
        acc[M_GMAX] = fmax(acc[M_GMAX], fabs(G));

        for (int q = 0; q < 3; ++q) acc[M_WABS] += (double)abs(plaquette_winding(f, D, compact, dx, c, P[q][0], P[q][1]));
    }

    __shared__ double red[kMeasThreads / 64][M_COUNT];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < M_COUNT; ++k) {
        const double r = (k == M_GMAX) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[wv][k] = r;
    }
    __syncthreads();
    if (threadIdx.x < M_COUNT) {
        const int k = threadIdx.x;
        double r = red[0][k];
        for (int w = 1; w < kMeasThreads / 64; ++w) r = (k == M_GMAX) ? fmax(r, red[w][k]) : r + red[w][k];
        partials[(int64_t)blockIdx.x * kMeasStride + k] = r;
    }
}

// Second stage: one block folds the per-block records in a fixed order.
__global__ void __launch_bounds__(256) k_measure_final(const double* __restrict__ partials, int nblocks,
                                                       double* __restrict__ result)
{
    __shared__ double red[256];
    fold_records(partials, nblocks, result, red);
}

// Values of the 10 state components at listed sites (dense indices
// x + N (y + N z)): out[10*k + c].
template <typename R>
__global__ void __launch_bounds__(256) k_gather(Fields<R> f, const int64_t* __restrict__ sites, int64_t count,
                                                Dims D, R* __restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int64_t s = sites[k];
    if (s < 0 || s >= (int64_t)D.N * D.N * D.N) return;  // rejected on the host; never read out of bounds
    const int64_t o = at(D, coords(D.N, s));
    const R* comps[10] = {f.phr, f.phi, f.pir, f.pii, f.a0, f.a1, f.a2, f.e0, f.e1, f.e2};
    for (int c = 0; c < 10; ++c) out[10 * k + c] = comps[c][o];
}

}  // namespace

// ------------------------------------------------------------------ launchers

template <typename R>
hipError_t launch_gather(const Fields<R>& f, const int64_t* sites, int64_t count, int N, int P, R* out, hipStream_t s)
{
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_gather<R>, dim3((unsigned)blocks), dim3(256), 0, s, f, sites, count, Dims{N, P}, out);
    return hipGetLastError();
}
template hipError_t launch_gather<double>(const Fields<double>&, const int64_t*, int64_t, int, int, double*,
                                          hipStream_t);
template hipError_t launch_gather<float>(const Fields<float>&, const int64_t*, int64_t, int, int, float*,
                                         hipStream_t);

template <typename R>
hipError_t launch_init(const Fields<R>& f, int N, int P, double sigma, uint64_t seed, hipStream_t s)
{
    const int64_t V = (int64_t)N * N * N;
    const int64_t blocks = (V + 255) / 256;
    hipLaunchKernelGGL(k_init<R>, dim3((unsigned)blocks), dim3(256), 0, s, f, Dims{N, P}, sigma, seed);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_step(const Fields<R>& in, R* ophr, R* ophi, R* oa0, R* oa1, R* oa2, const LatticeConst& L,
                       const StepCoef& c, hipStream_t s)
{
    const int N = L.N;
    dim3 block(64, 4, 1);
    dim3 grid((N + 63) / 64, (N + 3) / 4, N);
    hipLaunchKernelGGL(k_step_site<R>, grid, block, 0, s, in, ophr, ophi, oa0, oa1, oa2, Dims{N, L.P}, L.compact, (R)L.dx,
                       (R)L.sigma2, (R)c.cP1, (R)c.cP2, (R)c.cE1, (R)c.cE2, (R)c.lam_half, (R)c.kappa, (R)L.deta);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_measure(const Fields<R>& f, const LatticeConst& L, const StepCoef& c, const MeasConst& mc,
                          double* partials, double* result, hipStream_t s)
{
    hipLaunchKernelGGL(k_measure<R>, dim3(kMeasBlocks), dim3(kMeasThreads), 0, s, f, Dims{L.N, L.P}, L.compact, L.dx, L.sigma2,
                       c, mc, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_measure_final(partials, kMeasBlocks, result, s);
}

hipError_t launch_measure_final(const double* partials, int nblocks, double* result, hipStream_t s)
{
    hipLaunchKernelGGL(k_measure_final, dim3(1), dim3(256), 0, s, partials, nblocks, result);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_winding(const Fields<R>& f, const LatticeConst& L, int8_t* w, hipStream_t s)
{
    hipLaunchKernelGGL(k_winding<R>, dim3(kMeasBlocks), dim3(256), 0, s, f, Dims{L.N, L.P}, L.compact, L.dx, w);
    return hipGetLastError();
}

#define AH_INSTANTIATE(R)                                                                                          \
    template hipError_t launch_init<R>(const Fields<R>&, int, int, double, uint64_t, hipStream_t);                      \
    template hipError_t launch_step<R>(const Fields<R>&, R*, R*, R*, R*, R*, const LatticeConst&, const StepCoef&, \
                                       hipStream_t);                                                               \
    template hipError_t launch_measure<R>(const Fields<R>&, const LatticeConst&, const StepCoef&, const MeasConst&, \
                                          double*, double*, hipStream_t);                                          \
    template hipError_t launch_winding<R>(const Fields<R>&, const LatticeConst&, int8_t*, hipStream_t);
AH_INSTANTIATE(double)
AH_INSTANTIATE(float)

}  // namespace ah
