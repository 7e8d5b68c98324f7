// Device helpers of the stencil shared by the tiled step kernels: complex
// arithmetic with every fused multiply-add written out, the link variable,
// the plaquette field strength, periodic wrap, XCD-aware tile placement and
// the kick and drift of one site.
//
// Floating-point contraction is off wherever this is included, so each site
// is computed by the same sequence of roundings in every kernel.
#pragma once

#include "ah_internal.h"

#define AH_SINCOS_QUAL __device__
#include "ah_sincos.h"

#pragma clang fp contract(off)

namespace ah {
namespace {

__device__ inline float fm(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// A block-uniform value moved into scalar registers.  What a kernel loads
// from a descriptor or a coefficient row in memory, or converts from it, the
// compiler keeps in vector registers (one copy per lane), which would cost a
// march a wave per SIMD of occupancy.
template <typename T>
__device__ inline T uniform(T v)
{
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    int w[sizeof(T) / 4];
    __builtin_memcpy(w, &v, sizeof(T));
    for (unsigned k = 0; k < sizeof(T) / 4; ++k) w[k] = __builtin_amdgcn_readfirstlane(w[k]);
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}
__device__ inline double fm(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Streaming accesses: Pi and E are read and written once per step at their
// own site, phi and A are written once into the other ping-pong buffer; none
// of it is reused from cache within a step, so they bypass it and leave L2 to
// the phi / A halo lines that neighbouring tiles read again.
template <typename R>
__device__ inline R ld_stream(const R* p)
{
    return __builtin_nontemporal_load(p);
}
template <typename R>
__device__ inline void st_stream(R* p, R v)
{
    __builtin_nontemporal_store(v, p);
}

// base[plane + xy] with a uniform plane offset and a 32-bit in-plane index:
// the load adds the plane base, held in scalar registers, and one vector
// offset, with no 64-bit address arithmetic per access.
template <typename R>
__device__ inline R at(const R* base, int64_t plane, uint32_t xy)
{
    return (base + plane)[xy];
}

template <typename R>
struct Cx {
    R r, i;
};
template <typename R>
__device__ inline Cx<R> cmul(Cx<R> a, Cx<R> b)
{
    return {fm(a.r, b.r, -(a.i * b.i)), fm(a.r, b.i, a.i * b.r)};
}
template <typename R>
__device__ inline Cx<R> cmulc(Cx<R> a, Cx<R> b)  // conj(a) * b
{
    return {fm(a.r, b.r, a.i * b.i), fm(a.r, b.i, -(a.i * b.r))};
}

// FP64 links: the reduced-range sincos (accurate to ~2 ulp for |x| <= 1e9),
// the library routine beyond that (out of line: a link phase past 1e9 is a
// lattice long blown up, and inlined it would cost the march registers)
__device__ __noinline__ double2 sincos_far(double x)
{
    double2 v;
    sincos(x, &v.x, &v.y);
    return v;
}
__device__ inline void sincos_t(double x, double* s, double* c)
{
    if (fabs(x) <= 1e9) {
        sincos_reduced(x, s, c);
    } else {
        const double2 v = sincos_far(x);
        *s = v.x;
        *c = v.y;
    }
}
// FP32 links: the argument is reduced by whole turns with 2 pi split in
// three parts (Cody and Waite; the first two, 6.28125 and 1.9378662109375e-3,
// have at most 8 significant bits, so k times them is exact for |k| < 2^16
// turns), the remainder in [-pi, pi] is converted to turns and given to the
// hardware sine and cosine of one turn.  Within about 3e-7 of the FP64 sine
// and cosine of the same FP32 argument for |x| < 4e5 (the library sincosf is
// within 7e-8 but costs three times the instructions).  Beyond that (a link
// phase that large is a lattice long blown up) the turns are split off in
// FP64.
__device__ inline void sincos_t(float x, float* s, float* c)
{
    float t;
    if (fabsf(x) < 4.0e5f) {
        const float k = __builtin_rintf(x * 0.15915494309189535f);
        float r = fm(-k, 6.28125f, x);
        r = fm(-k, 1.9378662109375e-3f, r);
        r = fm(-k, -2.5590314e-6f, r);
        t = r * 0.15915494309189535f;
    } else {
        const double u = (double)x * 0.15915494309189535;
        t = (float)(u - __builtin_rint(u));
    }
    *s = __builtin_amdgcn_sinf(t);
    *c = __builtin_amdgcn_cosf(t);
}

// link U = exp(-i dx A) = (cos(dx A), -sin(dx A))
template <typename R>
__device__ inline Cx<R> link(R dx, R a)
{
    R s, c;
    sincos_t(dx * a, &s, &c);
    return {c, -s};
}

// -Im(p conj(q)) with p = U_i^x U_j^{x+i}, q = U_i^{x+j} U_j^x: sin(Theta_ij)
template <typename R>
__device__ inline R plaq_sin(Cx<R> ui_x, Cx<R> uj_xi, Cx<R> ui_xj, Cx<R> uj_x)
{
    const Cx<R> p = cmul(ui_x, uj_xi);
    const Cx<R> q = cmul(ui_xj, uj_x);
    return fm(p.r, q.i, -(p.i * q.r));
}

__device__ inline int wrapi(int v, int N)
{
    // v in [-2, 2N + TX]: periodic image in [0, N)
    if (v < 0) return v + N;
    return v < N ? v : v % N;
}

// Whether pool lattice L forms the diagnostics of its snapshot k (every
// measure_every-th and the last), and whether its step k is a two-step pass:
// it has a two-step tiling, neither k nor k+1 is due and both steps remain.
__device__ inline bool measure_due(const PoolLattice& L, int64_t k)
{
    if (k > L.nsteps) return false;
    if (k == L.nsteps) return true;
    return L.measure_every > 0 && (k % L.measure_every) == 0;
}
__device__ inline bool two_step_due(const PoolLattice& L, int64_t k)
{
    return L.two_zchunk > 0 && k + 1 < L.nsteps && !measure_due(L, k) && !measure_due(L, k + 1);
}

// Place tiles so that the blocks the hardware sends to one XCD (block b goes
// to XCD b % 8) cover a contiguous range of tile indices.
__device__ inline int xcd_tile(int b, int nb)
{
    const int per = nb / kXcdCount, rem = nb % kXcdCount;
    const int xcd = b % kXcdCount, k = b / kXcdCount;
    return xcd * per + (xcd < rem ? xcd : rem) + k;
}

// Kick and drift of one site from the values its stencil reads (section 2):
// covariant Laplacian and potential for Pi, lattice curl of the plaquette
// field strength and current for E, Crank-Nicolson damping, then the drift.
// Own column: phi at planes z-1, z, z+1, the site's links U_j^x, the x and y
// links of the site above (x+kz), U_z^{x-kz}, and F_xz, F_yz of the site
// below (carried down the z-march).  Every kernel that steps a site calls
// this, so each site is computed by one sequence of roundings whatever the
// kernel, tile shape or schedule.
template <typename R>
struct SiteNbr {
    Cx<R> ph_xm, ph_xp, ph_ym, ph_yp;  // phi at x -/+ kx, x -/+ ky (plane z)
    Cx<R> ux_xm, uy_ym;                // U_x^{x-kx}, U_y^{x-ky}
    Cx<R> uy_xp, ux_yp, uz_xp, uz_yp;  // U_y^{x+kx}, U_x^{x+ky}, U_z^{x+kx}, U_z^{x+ky}
    Cx<R> ux_xm_yp, uy_xm, uz_xm;      // U_x^{x-kx+ky}, U_y^{x-kx}, U_z^{x-kx}
    Cx<R> ux_ym, uy_xp_ym, uz_ym;      // U_x^{x-ky}, U_y^{x+kx-ky}, U_z^{x-ky}
    Cx<R> ux_xm_zp, uy_ym_zp;          // U_x^{x-kx+kz}, U_y^{x-ky+kz}
};

template <typename R>
struct SiteCoef {
    R inv_dx, inv_dx2, sigma2, cP1, cP2, cE1, cE2, lamh, kappa, deta;
};

template <typename R>
struct SiteOut {
    R pr, pi, e[3];  // Pi^{n+1/2}, E^{n+1/2}
    Cx<R> phi;       // phi^{n+1}
    R a[3];          // A^{n+1}
    R fxz, fyz;      // F_xz, F_yz at x (the carry of the plane above)
};

// Plaquette fields of one site update (each F_ij = sin(Theta_ij) / dx^2):
// those at x, and at x - kx and x - ky, which are the neighbours' own ones.
template <typename R>
struct SiteF {
    R xy, xz, yz;           // at x
    R xy_xm, xz_xm;         // at x - kx
    R xy_ym, yz_ym;         // at x - ky
};

// The plaquettes a site forms at itself (links of planes z and z+1).
template <typename R>
__device__ __forceinline__ void own_plaquettes(const Cx<R> (&Uc)[3], Cx<R> uy_xp, Cx<R> ux_yp, Cx<R> uz_xp,
                                               Cx<R> uz_yp, Cx<R> ux_zp, Cx<R> uy_zp, R inv_dx2, R* fxy, R* fxz,
                                               R* fyz)
{
    *fxy = plaq_sin(Uc[0], uy_xp, ux_yp, Uc[1]) * inv_dx2;
    *fxz = plaq_sin(Uc[0], uz_xp, ux_zp, Uc[2]) * inv_dx2;
    *fyz = plaq_sin(Uc[1], uz_yp, uy_zp, Uc[2]) * inv_dx2;
}

// Kick and drift of one site from its neighbourhood's phi, the links of the
// Laplacian and the plaquette fields.
template <typename R>
__device__ __forceinline__ SiteOut<R> site_update_f(const SiteCoef<R>& k, Cx<R> ph_xm, Cx<R> ph_xp, Cx<R> ph_ym,
                                                    Cx<R> ph_yp, Cx<R> ux_xm, Cx<R> uy_ym, Cx<R> phi_m, Cx<R> phi_c,
                                                    Cx<R> phi_p, const Cx<R> (&Uc)[3], Cx<R> uz_m, const SiteF<R>& F,
                                                    R fxz_m, R fyz_m, R pr_c, R pi_c, const R (&e_c)[3],
                                                    const R (&a_c)[3])
{
    const R inv_dx = k.inv_dx, inv_dx2 = k.inv_dx2;
    // covariant Laplacian: sum_j U_j^x phi^{x+j} + conj(U_j^{x-j}) phi^{x-j} - 2 phi^x
    const Cx<R> fx = cmul(Uc[0], ph_xp), fy = cmul(Uc[1], ph_yp), fz = cmul(Uc[2], phi_p);
    const Cx<R> bx = cmulc(ux_xm, ph_xm), by = cmulc(uy_ym, ph_ym), bz = cmulc(uz_m, phi_m);
    const R lr = ((fx.r + bx.r) + (fy.r + by.r)) + fm(R(-6), phi_c.r, fz.r + bz.r);
    const R li = ((fx.i + bx.i) + (fy.i + by.i)) + fm(R(-6), phi_c.i, fz.i + bz.i);
    // currents J_i = Im[conj(phi) U_i phi^{x+i}] / dx
    const R jx = fm(phi_c.r, fx.i, -(phi_c.i * fx.r)) * inv_dx;
    const R jy = fm(phi_c.r, fy.i, -(phi_c.i * fy.r)) * inv_dx;
    const R jz = fm(phi_c.r, fz.i, -(phi_c.i * fz.r)) * inv_dx;
    // lattice curl C_i = sum_{j != i} (F_ij^x - F_ij^{x-j}) / dx, F_ji = -F_ij
    const R cx = ((F.xy - F.xy_ym) + (F.xz - fxz_m)) * inv_dx;
    const R cy = ((F.yz - fyz_m) - (F.xy - F.xy_xm)) * inv_dx;
    const R cz = -((F.xz - F.xz_xm) + (F.yz - F.yz_ym)) * inv_dx;
    // Crank-Nicolson kick, drift
    const R m2 = fm(phi_c.r, phi_c.r, fm(phi_c.i, phi_c.i, -k.sigma2));
    const R pot = k.lamh * m2;
    SiteOut<R> o;
    o.pr = fm(k.cP1, pr_c, k.cP2 * fm(lr, inv_dx2, -(pot * phi_c.r)));
    o.pi = fm(k.cP1, pi_c, k.cP2 * fm(li, inv_dx2, -(pot * phi_c.i)));
    o.e[0] = fm(k.cE1, e_c[0], k.cE2 * fm(k.kappa, jx, -cx));
    o.e[1] = fm(k.cE1, e_c[1], k.cE2 * fm(k.kappa, jy, -cy));
    o.e[2] = fm(k.cE1, e_c[2], k.cE2 * fm(k.kappa, jz, -cz));
    o.phi = {fm(k.deta, o.pr, phi_c.r), fm(k.deta, o.pi, phi_c.i)};
    o.a[0] = fm(k.deta, o.e[0], a_c[0]);
    o.a[1] = fm(k.deta, o.e[1], a_c[1]);
    o.a[2] = fm(k.deta, o.e[2], a_c[2]);
    o.fxz = F.xz;
    o.fyz = F.yz;
    return o;
}

// The same update forming all seven plaquettes from the neighbourhood's links.
template <typename R>
__device__ __forceinline__ SiteOut<R> site_update(const SiteCoef<R>& k, const SiteNbr<R>& n, Cx<R> phi_m, Cx<R> phi_c,
                                                  Cx<R> phi_p, const Cx<R> (&Uc)[3], Cx<R> ux_zp, Cx<R> uy_zp,
                                                  Cx<R> uz_m, R fxz_m, R fyz_m, R pr_c, R pi_c, const R (&e_c)[3],
                                                  const R (&a_c)[3])
{
    const R inv_dx2 = k.inv_dx2;
    SiteF<R> F;
    own_plaquettes(Uc, n.uy_xp, n.ux_yp, n.uz_xp, n.uz_yp, ux_zp, uy_zp, inv_dx2, &F.xy, &F.xz, &F.yz);
    F.xy_xm = plaq_sin(n.ux_xm, Uc[1], n.ux_xm_yp, n.uy_xm) * inv_dx2;
    F.xy_ym = plaq_sin(n.ux_ym, n.uy_xp_ym, Uc[0], n.uy_ym) * inv_dx2;
    F.xz_xm = plaq_sin(n.ux_xm, Uc[2], n.ux_xm_zp, n.uz_xm) * inv_dx2;
    F.yz_ym = plaq_sin(n.uy_ym, Uc[2], n.uy_ym_zp, n.uz_ym) * inv_dx2;
    return site_update_f(k, n.ph_xm, n.ph_xp, n.ph_ym, n.ph_yp, n.ux_xm, n.uy_ym, phi_m, phi_c, phi_p, Uc, uz_m, F,
                         fxz_m, fyz_m, pr_c, pi_c, e_c, a_c);
}

}  // namespace
}  // namespace ah
