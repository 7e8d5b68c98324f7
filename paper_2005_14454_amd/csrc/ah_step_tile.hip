// Tiled, z-marching leapfrog step and diagnostics for gfx950 (compact gauge
// action), for one lattice and for a pool of lattices.
//
// One workgroup owns a TX x TY tile of the (x0, x1) plane and a chunk of
// x2-planes ("z").  It walks the chunk plane by plane.  For every incoming
// plane it loads A and phi of the tile plus a one-site halo ring once,
// turns A into link variables U_j = exp(-i dx A_j) (one sincos per link,
// shared by all users through LDS), and then updates its own sites:
//   - covariant Laplacian and current from U and phi (section 2);
//   - lattice curl from plaquettes formed as products of four links,
//     F_ij = -Im(U_i^x U_j^{x+i} conj(U_i^{x+j}) conj(U_j^x)) / dx^2, which
//     equals sin(Theta_ij)/dx^2 for the compact action;
//   - Crank-Nicolson kick of Pi and E in place, drift of phi and A into the
//     other ping-pong buffer.
// Every site reads its 10 state values and writes 10 values once per step;
// the halo re-reads hit L2.  Own-column quantities of the planes below and
// above (phi, U_z, F_xz, F_yz) are carried in registers.  Workgroups are
// placed so that each XCD gets a contiguous band of tiles, which keeps halo
// reads inside one L2.
//
// Floating-point contraction is off in this file and every fused multiply-add
// is written out, so each site is computed by the same sequence of roundings
// whatever the tile shape, z-chunk or template instance: results are
// bitwise reproducible across launch configurations.
#include "ah_device.h"
#include "ah_internal.h"
#include "ah_stencil.h"

#pragma clang fp contract(off)

namespace ah {
namespace {


template <typename R, int TX, int TY>
struct TileGeom {
    static constexpr int RW = TX + 2;             // region width (tile + halo)
    static constexpr int RH = TY + 2;             // region height
    static constexpr int RS = RW * RH;            // region sites
    static constexpr int NT = TX * TY;            // threads
    static constexpr int H = 2 * RW + 2 * TY;     // halo ring sites
    static constexpr int HPT = (H + NT - 1) / NT; // halo sites per thread (upper bound)
};

// Per-launch constants of one lattice step (coefficients rounded to R).
template <typename R>
struct StepArgs {
    Fields<R> f;
    R* ophr;
    R* ophi;
    R* oa0;
    R* oa1;
    R* oa2;
    // Pi and E outputs: f's own arrays for an update in place (the measured
    // march needs other ones)
    R* opr;
    R* opi;
    R* oe0;
    R* oe1;
    R* oe2;
    int N, P;  // side, row pitch: site (x, y, z) at x + P (y + N z)
    R dx, sigma2, cP1, cP2, cE1, cE2, lamh, kappa, deta;
};

// Constants of the diagnostics of the snapshot a measured march reads.
struct MeasArgs {
    double dx;          // lattice spacing (FP64, for plaquette angles and links)
    double inv_2e2f;    // 1 / (2 e0^2 f)
    double lam_quarter; // lambda0 f / 4
    double gauss_c;     // coupling of the Gauss residual
};

template <typename R, int TX, int TY>
struct TileShared {
    static constexpr int RS = TileGeom<R, TX, TY>::RS;
    Cx<R> U[2][3][RS];  // links of planes z and z+1 (ring)
    Cx<R> Phi[RS];      // phi of plane z
};

template <typename R, int TX, int TY>
struct MeasShared {
    static constexpr int RS = (TX + 2) * (TY + 2);
    R A[2][3][RS];                      // stored A of the link planes held in the U ring
    float Y[2][3][RS];                  // link phases of planes z (ring of two)
    // FP32 lattices: E_x, E_y of plane z (own sites, and the -x / -y halo)
    // for the Gauss residual
    R E[2][sizeof(R) == 4 ? RS : 1];
    // FP64 lattices: each thread's running diagnostics sums (kept here rather
    // than in registers, which the FP64 measured march runs out of)
    double acc[kMarchSums][sizeof(R) == 8 ? TX * TY : 1];
    double red[TX * TY / 64][M_COUNT];  // block reduction
};

// FP64 link for the windings of FP32 lattices (the stored value, exactly widened)
__device__ inline Cx<double> link64(double dx, double a)
{
    double s, c;
    sincos(dx * a, &s, &c);
    return {c, -s};
}

// atan2(y, x) in FP32 to within 1e-6 rad for max(|x|, |y|) in [1e-30, 1e30]:
// reduction to t = min(|x|, |y|) / max(|x|, |y|) in [0, 1], atan(t) ~ t P(t^2)
// with P of degree 6 fitted by weighted least squares on Chebyshev nodes
// (largest error 3.3e-7 in FP32 over [0, 1]), then the octant and the sign.
// Only the angle of a branch the caller has already made safe is taken from
// it; the cut itself is decided in FP64.
__device__ inline float atan2_fast(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float t = fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(ax, ay));
    const float s = t * t;
    float p = 0.00681175384670496f;
    p = fm(p, s, -0.033604107797145844f);
    p = fm(p, s, 0.07962355017662048f);
    p = fm(p, s, -0.13233335316181183f);
    p = fm(p, s, 0.19807814061641693f);
    p = fm(p, s, -0.3331736922264099f);
    p = fm(p, s, 0.9999961256980896f);
    float a = p * t;
    if (ay > ax) a = 1.57079632679489662f - a;
    if (x < 0.f) a = 3.14159265358979324f - a;
    return copysignf(a, y);
}

// Link phase arg(conj(phi^x) U phi^{x+j}) in (-pi, pi].  z is formed in FP64
// with plain products and sums; its sign decides the branch exactly as an
// FP64 atan2 would (-0 -> +0; atan2_fast keeps the sign of its first
// argument), and the angle itself is evaluated in FP32 on the exactly
// rescaled z: the windings only need it to well below pi.
__device__ inline float link_phase(double pr, double pim, Cx<double> U, double vr, double vi)
{
    const double wr = U.r * vr - U.i * vi;
    const double wi = U.r * vi + U.i * vr;
    const double zr = pr * wr + pim * wi;
    double zi = pr * wi - pim * wr;
    zi = (zi == 0.0) ? 0.0 : zi;
    const double mz = fmax(fabs(zr), fabs(zi));
    if (mz == 0.0) return signbit(zr) ? 3.14159265358979f : 0.0f;
    const int e = ilogb(mz);
    return atan2_fast((float)ldexp(zi, -e), (float)ldexp(zr, -e));
}

// The FP64 evaluation for an FP32 lattice's link near the cut.  It runs for a
// few links in a million, so it is kept out of line: inlined, its FP64 sincos
// raises the register count of the whole measured march.
__device__ __attribute__((noinline)) float link_phase_near_cut(Cx<float> ph, Cx<float> pn, float a, double dx)
{
    return link_phase((double)ph.r, (double)ph.i, link64(dx, (double)a), (double)pn.r, (double)pn.i);
}

// Link phase of an FP32 lattice from z = conj(ph) (U pn), formed in FP32 from
// the link the step itself uses; its angle, taken in FP32, is within
//   |dx A| 2^-22 (rounding of dx A, in the link's phase)
//   + 1e-5        (the link's sine and cosine, within 3e-7; the two complex
//                  products; atan2_fast)
// of the FP64 value, so unless it lies that close to the cut at +-pi it is on
// the same side of it.  Near the cut, where |z| leaves the range in which
// FP32 keeps its relative precision (or is not finite), and where |dx A|
// exceeds 1e5 (so that four phases stay well within pi of the FP64 sum), the
// FP64 evaluation above decides from the stored A.
__device__ inline float link_phase_f(Cx<float> z, Cx<float> ph, Cx<float> pn, float a, double dx)
{
    const float mz = fmaxf(fabsf(z.r), fabsf(z.i));
    const float dxa = fabsf((float)dx * a);
    if (mz > 1e-30f && mz < 1e30f && dxa < 1e5f) {
        const float y = atan2_fast(z.i, z.r);
        if (3.14159265f - fabsf(y) > 1e-5f + 2.4e-7f * dxa) return y;
    }
    return link_phase_near_cut(ph, pn, a, dx);
}

// Winding of a plaquette from its four link phases and its angle (FP64): the
// angle is wrapped to (-pi, pi] by the nearest multiple of 2 pi that the
// division th / 2 pi rounds to (a product with 1 / 2 pi gives the same
// multiple unless the quotient is close to a half turn, where the division
// itself is taken); the total is then within ~1e-5 of a multiple of 2 pi.
__device__ inline int winding_of(float y1, float y2, float y3, float y4, double th)
{
    const double two_pi = 6.283185307179586;
    const double inv_two_pi = 1.0 / two_pi;
    const double q = th * inv_two_pi;
    double r = rint(q);
    if (!(fabs(q - r) < 0.49 && fabs(q) < 1e12)) r = rint(th / two_pi);
    const double thw = th - two_pi * r;
    const double sum = ((((double)y1 + (double)y2) - (double)y3) - (double)y4) + thw;
    return (int)rint(sum * inv_two_pi);
}

// 1 - cos(Theta) of a plaquette from its four links, without cancellation
template <typename R>
__device__ inline R plaq_omc(Cx<R> ui_x, Cx<R> uj_xi, Cx<R> ui_xj, Cx<R> uj_x, R* sn)
{
    const Cx<R> p = cmul(ui_x, uj_xi);
    const Cx<R> q = cmul(ui_xj, uj_x);
    const R c = fm(p.r, q.r, p.i * q.i);
    const R s = fm(p.r, q.i, -(p.i * q.r));
    *sn = s;
    return c > R(0) ? (s * s) / (R(1) + c) : R(1) - c;
}

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

// Walk planes [z0, z1) of the tile whose lower corner is (x0, y0): kick and
// drift every own site (if `write`), and with MEAS also form the diagnostics of
// the snapshot being read (section 2 estimators, energy split, windings, the
// residual of the discrete Gauss law), writing the workgroup's fixed-order
// sums to `record`.  The Gauss residual
// reads E at the -x and -y neighbours, which a neighbouring workgroup of a
// pass that updated E in place could already have overwritten, so a measured
// march that steps writes Pi and E out of place (a.opr .. a.oe2).  E_z of the
// plane below is carried in a register; FP32 passes E_x and E_y of each plane
// through LDS, FP64 (whose LDS holds two workgroups per CU only without that
// exchange) loads the two neighbours with the plane's Pi and E.
// All threads of the workgroup call this with the same arguments; it
// synchronises the workgroup internally.
template <typename R, int TX, int TY, bool MEAS>
__device__ void march_step(TileShared<R, TX, TY>& sh, MeasShared<R, TX, TY>* mx, const StepArgs<R>& a,
                           const MeasArgs& ma, double* __restrict__ record, bool write, int x0, int y0, int z0,
                           int z1)
{
    using G = TileGeom<R, TX, TY>;
    constexpr int RW = G::RW, H = G::H, NT = G::NT;
    static_assert(G::HPT == 1, "halo must fit one extra site per thread");
    auto& sU = sh.U;
    auto& sPhi = sh.Phi;
    const Fields<R>& f = a.f;
    R* __restrict__ ophr = a.ophr;
    R* __restrict__ ophi = a.ophi;
    R* __restrict__ oa0 = a.oa0;
    R* __restrict__ oa1 = a.oa1;
    R* __restrict__ oa2 = a.oa2;
    const int N = a.N;
    const R dx = a.dx, sigma2 = a.sigma2, cP1 = a.cP1, cP2 = a.cP2, cE1 = a.cE1, cE2 = a.cE2;
    const R lamh = a.lamh, kappa = a.kappa, deta = a.deta;
    constexpr bool GAUSS = MEAS;                  // Gauss residual in this march
    constexpr bool GLDS = GAUSS && sizeof(R) == 4;  // its -x / -y E through LDS (FP64: loads)
    R* wpr = a.opr;
    R* wpi = a.opi;
    R* we0 = a.oe0;
    R* we1 = a.oe1;
    R* we2 = a.oe2;

    const R inv_dx = R(1) / dx;
    const R inv_dx2 = inv_dx * inv_dx;
    const int P = a.P;
    const int64_t NN = (int64_t)N * P;  // plane stride

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool active = gx < N && gy < N;
    const int gxw = wrapi(gx, N), gyw = wrapi(gy, N);
    const int64_t own_xy = (int64_t)gxw + (int64_t)P * gyw;
    const uint32_t ob = (uint32_t)own_xy;  // 32-bit in-plane offset (N P < 2^32)
    const int ro = (ly + 1) * RW + (lx + 1);  // own region slot

    // halo ring site of this thread (if any)
    const bool has_halo = tid < H;
    int rh = 0, hrx = 0, hry = 0;
    int64_t halo_xy = 0;
    if (has_halo) {
        if (tid < RW) {
            hrx = tid;
            hry = 0;
        } else if (tid < 2 * RW) {
            hrx = tid - RW;
            hry = TY + 1;
        } else if (tid < 2 * RW + TY) {
            hrx = 0;
            hry = 1 + (tid - 2 * RW);
        } else {
            hrx = TX + 1;
            hry = 1 + (tid - 2 * RW - TY);
        }
        rh = hry * RW + hrx;
        halo_xy = (int64_t)wrapi(x0 - 1 + hrx, N) + (int64_t)P * wrapi(y0 - 1 + hry, N);
    }
    const uint32_t hb = (uint32_t)halo_xy;
    // halo sites whose link phases the windings of the tile read
    const bool halo_top = has_halo && hry == TY + 1 && hrx >= 1 && hrx <= TX;    // Y_x, Y_z
    const bool halo_right = has_halo && hrx == TX + 1 && hry >= 1 && hry <= TY;  // Y_y, Y_z
    // halo sites whose E the Gauss residual of the tile reads: E_x on the -x
    // column, E_y on the -y row
    const bool halo_ex = has_halo && hrx == 0 && hry >= 1 && hry <= TY;
    const bool halo_ey = has_halo && hry == 0 && hrx >= 1 && hrx <= TX;
    const bool halo_e = GLDS && (halo_ex || halo_ey);
    const R* hE = halo_ex ? f.e0 : f.e1;
    const int hEc = halo_ex ? 0 : 1;

    // neighbour slots in the region
    const int rxm = ro - 1, rxp = ro + 1, rym = ro - RW, ryp = ro + RW;
    const int rxm_yp = ro - 1 + RW, rxp_ym = ro + 1 - RW;

    auto plane_of = [&](int z) -> int64_t { return (int64_t)wrapi(z, N) * NN; };

    // ---------------------------------------------------------------- prologue
    // U(z0-1) of the region into slot 1, U(z0) into slot 0, phi(z0) into sPhi.
    // The FP64 plain march reads its own links of planes z and z+1 from LDS
    // where it uses them rather than carrying them from plane to plane in
    // registers (186 rather than 202 registers on 64 x 8, 1% faster).
    constexpr bool ULDS = sizeof(R) == 8;
    Cx<R> Uc[3], Up[3];
    R Ac[3], Ap[3];
    Cx<R> phi_c, phi_p;
    Cx<R> bz_m;  // conj(U_z) phi of the own site one plane below
    R fxz_m, fyz_m;
    // diagnostics state (MEAS): the (x, z) and (y, z) windings of plane z need
    // Y_x, Y_y of plane z+1, so they are completed one plane later from the own
    // link phases of plane z (_b) and the two plaquette angles of plane z
    float yx_b = 0.f, yy_b = 0.f, yz_b = 0.f;
    double thxz_b = 0.0, thyz_b = 0.0;
    // link phase of a link U = exp(-i dx a) between phi values ph and pn
    auto phase = [&](Cx<R> ph, Cx<R> U, Cx<R> pn, R av) -> float {
        if constexpr (sizeof(R) == 8)
            return link_phase(ph.r, ph.i, U, pn.r, pn.i);
        else
            return link_phase_f(cmulc(ph, cmul(U, pn)), ph, pn, av, ma.dx);
    };
    // sums of the march: M_KIN .. M_RHOL (kMarchSums slots, FP64) and the
    // exact counts M_WABS, M_NONFIN (integers); the Gauss sums follow
    double acc_reg[kMarchSums];
    auto acc = [&](int k) -> double& {
        if constexpr (sizeof(R) == 8)
            return mx->acc[k][tid];
        else
            return acc_reg[k];
    };
    int wabs = 0, nonfin = 0;
    if constexpr (MEAS)
        for (int k = 0; k < kMarchSums; ++k) acc(k) = 0.0;
    // Gauss residual (GAUSS): sums of G^2, (div E)^2, (c rho)^2, max |G|, and
    // E_z of the own site one plane below
    double g2 = 0.0, d2 = 0.0, c2 = 0.0, gmax = 0.0;
    R ezm = R(0);
    // FP64: E_x at x - kx and E_y at x - ky of plane z, loaded with the plane's
    // Pi and E (Pi and E go to other buffers, so these are the snapshot's)
    R ex_xm = R(0), ey_ym = R(0);
    const uint32_t ob_xm = gxw == 0 ? ob + (uint32_t)(N - 1) : ob - 1u;
    const uint32_t ob_ym = gyw == 0 ? ob + (uint32_t)(N - 1) * (uint32_t)P : ob - (uint32_t)P;
    const double inv_dx64 = 1.0 / ma.dx;
    {
        const int64_t pm = plane_of(z0 - 1), p0 = plane_of(z0);
        const R* A[3] = {f.a0, f.a1, f.a2};
        Cx<R> um[3];
        for (int d = 0; d < 3; ++d) {
            um[d] = link(dx, at(A[d], pm, ob));
            sU[1][d][ro] = um[d];
            Ac[d] = at(A[d], p0, ob);
            Uc[d] = link(dx, Ac[d]);
            sU[0][d][ro] = Uc[d];
        }
        if (has_halo)
            for (int d = 0; d < 3; ++d) {
                sU[1][d][rh] = link(dx, at(A[d], pm, hb));
                const R ah = at(A[d], p0, hb);
                sU[0][d][rh] = link(dx, ah);
                if constexpr (MEAS) mx->A[0][d][rh] = ah;
            }
        if constexpr (MEAS)
            for (int d = 0; d < 3; ++d) mx->A[0][d][ro] = Ac[d];
        const Cx<R> phi_m{at(f.phr, pm, ob), at(f.phi, pm, ob)};
        phi_c = {at(f.phr, p0, ob), at(f.phi, p0, ob)};
        sPhi[ro] = phi_c;
        if (has_halo) sPhi[rh] = Cx<R>{at(f.phr, p0, hb), at(f.phi, p0, hb)};
        if constexpr (GAUSS) ezm = at(f.e2, pm, ob);
        if constexpr (GLDS) {
            mx->E[0][ro] = at(f.e0, p0, ob);
            mx->E[1][ro] = at(f.e1, p0, ob);
            if (halo_e) mx->E[hEc][rh] = at(hE, p0, hb);
        }

        bz_m = cmulc(um[2], phi_m);
        __syncthreads();
        // F_xz, F_yz of the own column at plane z0-1
        fxz_m = plaq_sin(um[0], sU[1][2][rxp], Uc[0], um[2]) * inv_dx2;
        fyz_m = plaq_sin(um[1], sU[1][2][ryp], Uc[1], um[2]) * inv_dx2;
        __syncthreads();
        // U(z0+1) into slot 1
        const int64_t p1 = plane_of(z0 + 1);
        for (int d = 0; d < 3; ++d) {
            Ap[d] = at(A[d], p1, ob);
            Up[d] = link(dx, Ap[d]);
            sU[1][d][ro] = Up[d];
        }
        if (has_halo)
            for (int d = 0; d < 3; ++d) {
                const R ah = at(A[d], p1, hb);
                sU[1][d][rh] = link(dx, ah);
                if constexpr (MEAS) mx->A[1][d][rh] = ah;
            }
        if constexpr (MEAS)
            for (int d = 0; d < 3; ++d) mx->A[1][d][ro] = Ap[d];
        phi_p = {at(f.phr, p1, ob), at(f.phi, p1, ob)};
        __syncthreads();
    }

    const int64_t pz0 = (int64_t)z0 * NN;
    R pr_c = ld_stream(f.pir + pz0 + ob), pi_c = ld_stream(f.pii + pz0 + ob);
    R e_c[3] = {ld_stream(f.e0 + pz0 + ob), ld_stream(f.e1 + pz0 + ob), ld_stream(f.e2 + pz0 + ob)};
    if constexpr (GAUSS && !GLDS) {
        ex_xm = at(f.e0, pz0, ob_xm);
        ey_ym = at(f.e1, pz0, ob_ym);
    }

    // Operands prefetched for iteration t: A of plane t+2 (own and halo), phi
    // of plane t+1 (halo) and t+2 (own), Pi and E of plane t+1 (own).  The
    // plain march loads them one iteration ahead.  The measured march of FP32
    // lattices holds fewer waves per SIMD (it needs more registers), so it
    // loads them two iterations ahead to keep as many loads in flight; it
    // loads every iteration's operands, the last ones of a chunk from wrapped
    // planes that it does not use.  The FP64 measured march has no registers
    // to hold them across the plane's arithmetic and loads them (LATE) just
    // before they are used, which keeps it at two waves per SIMD.
    constexpr bool D2 = MEAS && sizeof(R) == 4;
    constexpr bool LATE = MEAS && sizeof(R) == 8;
    struct Pre {
        R a[3], ha[3];
        Cx<R> hphi, phi2;
        R pr, pi, e[3];
        R he;          // GLDS: the halo E of plane t+1
        R exm, eym;    // FP64 Gauss: E_x at x - kx, E_y at x - ky of plane t+1
    };
    auto prefetch = [&](int t, Pre& q) {
        const int64_t p2 = plane_of(t + 2), p1 = plane_of(t + 1);
        q.a[0] = at(f.a0, p2, ob);
        q.a[1] = at(f.a1, p2, ob);
        q.a[2] = at(f.a2, p2, ob);
        if (has_halo) {
            q.ha[0] = at(f.a0, p2, hb);
            q.ha[1] = at(f.a1, p2, hb);
            q.ha[2] = at(f.a2, p2, hb);
            q.hphi = {at(f.phr, p1, hb), at(f.phi, p1, hb)};
        }
        if constexpr (GLDS)
            if (halo_e) q.he = at(hE, p1, hb);
        if constexpr (GAUSS && !GLDS) {
            q.exm = at(f.e0, p1, ob_xm);
            q.eym = at(f.e1, p1, ob_ym);
        }
        q.phi2 = {at(f.phr, p2, ob), at(f.phi, p2, ob)};
        q.pr = ld_stream(f.pir + p1 + ob);
        q.pi = ld_stream(f.pii + p1 + ob);
        q.e[0] = ld_stream(f.e0 + p1 + ob);
        q.e[1] = ld_stream(f.e1 + p1 + ob);
        q.e[2] = ld_stream(f.e2 + p1 + ob);
    };
    Pre q1, q2;
    if constexpr (D2) prefetch(z0, q1);

    int cur = 0;
    for (int z = z0; z < z1; ++z) {
        const int nxt = cur ^ 1;
        const bool more = z + 1 < z1;  // is there a next iteration?
        const int zs = (z - z0) & 1;   // link-phase slot of plane z
        // ---- 0. issue the loads of the operands prefetched for the coming
        //         iterations (q1 holds those of this one)
        if constexpr (D2)
            prefetch(z + 1, q2);
        else if (!LATE && more)
            prefetch(z, q1);
        const R* rA = q1.a;  // read at step 3, after the late loads
        const R* hA = q1.ha;
        Cx<R> hphi = q1.hphi;
        if constexpr (LATE) {
            // the halo phi of plane z+1 is needed before the late loads (by the
            // halo link phases of this plane), so it is loaded here
            if (has_halo) {
                const int64_t p1 = plane_of(z + 1);
                hphi = Cx<R>{at(f.phr, p1, hb), at(f.phi, p1, hb)};
            }
        }
        const Cx<R> rphi = phi_p;
        float yx_c = 0.f, yy_c = 0.f, yz_c = 0.f;
        double th_xy = 0.0;
        if constexpr (MEAS) {
            // ---- link phases of plane z on the +x / +y halo
            auto& sY = mx->Y[zs];
            if (halo_top || halo_right) {
                const Cx<R> ph = sPhi[rh];
                const auto& sA = mx->A[cur];
                if (halo_top) sY[0][rh] = phase(ph, sU[cur][0][rh], sPhi[rh + 1], sA[0][rh]);
                if (halo_right) sY[1][rh] = phase(ph, sU[cur][1][rh], sPhi[rh + RW], sA[1][rh]);
                sY[2][rh] = phase(ph, sU[cur][2][rh], hphi, sA[2][rh]);
            }
        }

        // ---- 1. update of the own site at plane z
        {
            if constexpr (ULDS)
                for (int d = 0; d < 3; ++d) {
                    Uc[d] = sU[cur][d][ro];
                    Up[d] = sU[nxt][d][ro];
                }
            if constexpr (GAUSS && !GLDS) {
                // FP64: the Gauss residual of the site first, while few values
                // are live (FP32 forms it with the other diagnostics below)
                if (active) {
                    const double dv = (((double)e_c[0] - (double)ex_xm) * inv_dx64 +
                                       ((double)e_c[1] - (double)ey_ym) * inv_dx64) +
                                      ((double)e_c[2] - (double)ezm) * inv_dx64;
                    const double crho = ma.gauss_c * ((double)phi_c.r * (double)pi_c -
                                                      (double)phi_c.i * (double)pr_c);
                    const double G = dv - crho;
                    g2 += G * G;
                    d2 += dv * dv;
                    c2 += crho * crho;
                    gmax = fmax(gmax, fabs(G));
                }
            }
            const Cx<R> ph_xm = sPhi[rxm], ph_xp = sPhi[rxp], ph_ym = sPhi[rym], ph_yp = sPhi[ryp];
            const Cx<R> ux_xm = sU[cur][0][rxm];  // U_x^{x-kx}
            const Cx<R> uy_ym = sU[cur][1][rym];  // U_y^{x-ky}
            // covariant Laplacian: sum_j U_j^x phi^{x+j} + conj(U_j^{x-j}) phi^{x-j} - 2 phi^x
            const Cx<R> fx = cmul(Uc[0], ph_xp), fy = cmul(Uc[1], ph_yp), fz = cmul(Uc[2], phi_p);
            const Cx<R> bx = cmulc(ux_xm, ph_xm), by = cmulc(uy_ym, ph_ym), bz = bz_m;
            const R lr = ((fx.r + bx.r) + (fy.r + by.r)) + fm(R(-6), phi_c.r, fz.r + bz.r);
            const R li = ((fx.i + bx.i) + (fy.i + by.i)) + fm(R(-6), phi_c.i, fz.i + bz.i);
            // currents J_i = Im[conj(phi) U_i phi^{x+i}] / dx
            const R jx = fm(phi_c.r, fx.i, -(phi_c.i * fx.r)) * inv_dx;
            const R jy = fm(phi_c.r, fy.i, -(phi_c.i * fy.r)) * inv_dx;
            const R jz = fm(phi_c.r, fz.i, -(phi_c.i * fz.r)) * inv_dx;
            if constexpr (MEAS) {
                // own link phases of plane z (FP32 lattices: z = conj(phi) U phi^{x+j}
                // is the forward product of the Laplacian)
                if constexpr (sizeof(R) == 8) {
                    yx_c = link_phase(phi_c.r, phi_c.i, Uc[0], ph_xp.r, ph_xp.i);
                    yy_c = link_phase(phi_c.r, phi_c.i, Uc[1], ph_yp.r, ph_yp.i);
                    yz_c = link_phase(phi_c.r, phi_c.i, Uc[2], phi_p.r, phi_p.i);
                } else {
                    yx_c = link_phase_f(cmulc(phi_c, fx), phi_c, ph_xp, Ac[0], ma.dx);
                    yy_c = link_phase_f(cmulc(phi_c, fy), phi_c, ph_yp, Ac[1], ma.dx);
                    yz_c = link_phase_f(cmulc(phi_c, fz), phi_c, phi_p, Ac[2], ma.dx);
                }
                auto& sY = mx->Y[zs];
                sY[0][ro] = yx_c;
                sY[1][ro] = yy_c;
                sY[2][ro] = yz_c;
                // the (x, z), (y, z) windings at x, plane z-1, now that Y_x, Y_y
                // of plane z are known
                if (active && z > z0) {
                    const auto& sYb = mx->Y[zs ^ 1];
                    wabs += abs(winding_of(yx_b, sYb[2][rxp], yx_c, yz_b, thxz_b)) +
                            abs(winding_of(yy_b, sYb[2][ryp], yy_c, yz_b, thyz_b));
                }
                // plaquette angles at x, plane z, from the stored A
                const auto& sA = mx->A[cur];
                th_xy = ma.dx * ((((double)Ac[0] + (double)sA[1][rxp]) - (double)sA[0][ryp]) - (double)Ac[1]);
                thxz_b = ma.dx * ((((double)Ac[0] + (double)sA[2][rxp]) - (double)Ap[0]) - (double)Ac[2]);
                thyz_b = ma.dx * ((((double)Ac[1] + (double)sA[2][ryp]) - (double)Ap[1]) - (double)Ac[2]);
            }
            // plaquettes at x (F_ij^x, i<j)
            const Cx<R> uy_xp = sU[cur][1][rxp], ux_yp = sU[cur][0][ryp];
            const Cx<R> uz_xp = sU[cur][2][rxp], uz_yp = sU[cur][2][ryp];
            R sxy, sxz, syz, oxy = 0, oxz = 0, oyz = 0;
            if constexpr (MEAS) {
                oxy = plaq_omc(Uc[0], uy_xp, ux_yp, Uc[1], &sxy);
                oxz = plaq_omc(Uc[0], uz_xp, Up[0], Uc[2], &sxz);
                oyz = plaq_omc(Uc[1], uz_yp, Up[1], Uc[2], &syz);
            } else {
                sxy = plaq_sin(Uc[0], uy_xp, ux_yp, Uc[1]);
                sxz = plaq_sin(Uc[0], uz_xp, Up[0], Uc[2]);
                syz = plaq_sin(Uc[1], uz_yp, Up[1], Uc[2]);
            }
            const R fxy = sxy * inv_dx2;
            const R fxz = sxz * inv_dx2;
            const R fyz = syz * inv_dx2;
            // plaquettes at x - kx and x - ky
            const Cx<R> ux_xm_yp = sU[cur][0][rxm_yp], uy_xm = sU[cur][1][rxm], uz_xm = sU[cur][2][rxm];
            const Cx<R> ux_ym = sU[cur][0][rym], uy_xp_ym = sU[cur][1][rxp_ym], uz_ym = sU[cur][2][rym];
            const Cx<R> ux_xm_zp = sU[nxt][0][rxm], uy_ym_zp = sU[nxt][1][rym];
            const R fxy_xm = plaq_sin(ux_xm, Uc[1], ux_xm_yp, uy_xm) * inv_dx2;
            const R fxy_ym = plaq_sin(ux_ym, uy_xp_ym, Uc[0], uy_ym) * inv_dx2;
            const R fxz_xm = plaq_sin(ux_xm, Uc[2], ux_xm_zp, uz_xm) * inv_dx2;
            const R fyz_ym = plaq_sin(uy_ym, Uc[2], uy_ym_zp, uz_ym) * inv_dx2;
            // lattice curl C_i = sum_{j != i} (F_ij^x - F_ij^{x-j}) / dx, F_ji = -F_ij
            const R cx = ((fxy - fxy_ym) + (fxz - fxz_m)) * inv_dx;
            const R cy = ((fyz - fyz_m) - (fxy - fxy_xm)) * inv_dx;
            const R cz = -((fxz - fxz_xm) + (fyz - fyz_ym)) * inv_dx;
            // Crank-Nicolson kick, drift
            const R m2 = fm(phi_c.r, phi_c.r, fm(phi_c.i, phi_c.i, -sigma2));
            const R pot = lamh * m2;
            const R npr = fm(cP1, pr_c, cP2 * fm(lr, inv_dx2, -(pot * phi_c.r)));
            const R npi = fm(cP1, pi_c, cP2 * fm(li, inv_dx2, -(pot * phi_c.i)));
            const R ne0 = fm(cE1, e_c[0], cE2 * fm(kappa, jx, -cx));
            const R ne1 = fm(cE1, e_c[1], cE2 * fm(kappa, jy, -cy));
            const R ne2 = fm(cE1, e_c[2], cE2 * fm(kappa, jz, -cz));
            if (write && active) {
                const int64_t o = (int64_t)z * NN;  // plane offset (uniform); + ob: the site
                st_stream(wpr + o + ob, npr);
                st_stream(wpi + o + ob, npi);
                st_stream(we0 + o + ob, ne0);
                st_stream(we1 + o + ob, ne1);
                st_stream(we2 + o + ob, ne2);
                st_stream(ophr + o + ob, fm(deta, npr, phi_c.r));
                st_stream(ophi + o + ob, fm(deta, npi, phi_c.i));
                st_stream(oa0 + o + ob, fm(deta, ne0, Ac[0]));
                st_stream(oa1 + o + ob, fm(deta, ne1, Ac[1]));
                st_stream(oa2 + o + ob, fm(deta, ne2, Ac[2]));
            }
            if constexpr (MEAS) {
                if (active) {
                    // site densities with centred momenta (average of the stored
                    // half step and the kick), summed in FP64
                    const R v[10] = {phi_c.r, phi_c.i, pr_c, pi_c, Ac[0], Ac[1], Ac[2], e_c[0], e_c[1], e_c[2]};
                    bool bad = false;
                    for (int k = 0; k < 10; ++k) bad |= !isfinite(v[k]);
                    nonfin += bad ? 1 : 0;
                    const R pbr = R(0.5) * (pr_c + npr), pbi = R(0.5) * (pi_c + npi);
                    const double kin = (double)fm(pbr, pbr, pbi * pbi);
                    const R d0r = fx.r - phi_c.r, d0i = fx.i - phi_c.i;
                    const R d1r = fy.r - phi_c.r, d1i = fy.i - phi_c.i;
                    const R d2r = fz.r - phi_c.r, d2i = fz.i - phi_c.i;
                    const double grad =
                        (double)(((d0r * d0r + d0i * d0i) + (d1r * d1r + d1i * d1i) + (d2r * d2r + d2i * d2i)) *
                                 inv_dx2);
                    const double pot_e = ma.lam_quarter * (double)m2 * (double)m2;
                    const R eb0 = R(0.5) * (e_c[0] + ne0), eb1 = R(0.5) * (e_c[1] + ne1),
                            eb2 = R(0.5) * (e_c[2] + ne2);
                    const double el = (double)(eb0 * eb0 + eb1 * eb1 + eb2 * eb2) * ma.inv_2e2f;
                    const double mag = (double)(R(2) * (oxy + oxz + oyz) * (inv_dx2 * inv_dx2)) * ma.inv_2e2f;
                    const double L = kin - grad - pot_e + el - mag;
                    acc(M_KIN) += kin;
                    acc(M_GRAD) += grad;
                    acc(M_POT) += pot_e;
                    acc(M_EL) += el;
                    acc(M_MAG) += mag;
                    acc(M_KINL) += kin * L;
                    acc(M_GRADL) += grad * L;
                    // pressure and energy density for the equation-of-state estimator
                    const double pres = (kin - pot_e) + ((el + mag) - grad) * (1.0 / 3.0);
                    const double rho = ((kin + grad) + pot_e) + (el + mag);
                    acc(M_PL) += pres * L;
                    acc(M_RHOL) += rho * L;
                    if constexpr (GLDS) {
                        // G = sum_i (E_i^x - E_i^{x-i}) / dx - c Im[conj(phi) Pi] of the
                        // snapshot, in FP64 from the exactly widened stored values
                        const double dv = (((double)e_c[0] - (double)mx->E[0][rxm]) * inv_dx64 +
                                           ((double)e_c[1] - (double)mx->E[1][rym]) * inv_dx64) +
                                          ((double)e_c[2] - (double)ezm) * inv_dx64;
                        const double crho = ma.gauss_c * ((double)phi_c.r * (double)pi_c -
                                                          (double)phi_c.i * (double)pr_c);
                        const double G = dv - crho;
                        g2 += G * G;
                        d2 += dv * dv;
                        c2 += crho * crho;
                        gmax = fmax(gmax, fabs(G));
                    }
                }
            }
            fxz_m = fxz;
            fyz_m = fyz;
            bz_m = cmulc(Uc[2], phi_c);  // for plane z+1
        }
        if (!MEAS && !more) break;
        __syncthreads();  // all reads of slot cur and of sPhi (plane z) are done

        if constexpr (MEAS) {
            // winding of the (x, y) plaquette at x, plane z
            if (active) {
                const auto& sY = mx->Y[zs];
                wabs += abs(winding_of(yx_c, sY[1][rxp], sY[0][ryp], yy_c, th_xy));
            }
            yx_b = yx_c;
            yy_b = yy_c;
            yz_b = yz_c;
        }

        if constexpr (LATE) prefetch(z, q1);
        // ---- 3. plane z+2 links into slot cur, plane z+1 phi into sPhi
        Cx<R> Upp[3];
        if (more) {
            for (int d = 0; d < 3; ++d) {
                Upp[d] = link(dx, rA[d]);
                sU[cur][d][ro] = Upp[d];
                if constexpr (MEAS) mx->A[cur][d][ro] = rA[d];
            }
            if (has_halo) {
                for (int d = 0; d < 3; ++d) {
                    sU[cur][d][rh] = link(dx, hA[d]);
                    if constexpr (MEAS) mx->A[cur][d][rh] = hA[d];
                }
                sPhi[rh] = hphi;
            }
            sPhi[ro] = rphi;
            if constexpr (GLDS) {
                mx->E[0][ro] = q1.e[0];
                mx->E[1][ro] = q1.e[1];
                if (halo_e) mx->E[hEc][rh] = q1.he;
            }
        } else if constexpr (MEAS) {
            if (has_halo) sPhi[rh] = hphi;
            sPhi[ro] = rphi;
        }
        __syncthreads();

        if (!more) {
            if constexpr (MEAS) {
                // own Y_x, Y_y of plane z1 complete the (x, z), (y, z) windings
                // of the chunk's last plane
                const Cx<R> px = sPhi[rxp], py = sPhi[ryp];
                const Cx<R> ux_n = ULDS ? sU[nxt][0][ro] : Up[0], uy_n = ULDS ? sU[nxt][1][ro] : Up[1];
                const float yx_n = phase(phi_p, ux_n, px, Ap[0]);
                const float yy_n = phase(phi_p, uy_n, py, Ap[1]);
                if (active) {
                    const auto& sYb = mx->Y[zs];
                    wabs += abs(winding_of(yx_b, sYb[2][rxp], yx_n, yz_b, thxz_b)) +
                            abs(winding_of(yy_b, sYb[2][ryp], yy_n, yz_b, thyz_b));
                }
            }
            break;
        }

        // ---- 5. rotate the own-column registers
        if constexpr (GAUSS) ezm = e_c[2];
        if constexpr (GAUSS && !GLDS) {
            ex_xm = q1.exm;
            ey_ym = q1.eym;
        }
        for (int d = 0; d < 3; ++d) {
            if constexpr (!ULDS) {
                Uc[d] = Up[d];
                Up[d] = Upp[d];
            }
            Ac[d] = Ap[d];
            Ap[d] = q1.a[d];
            e_c[d] = q1.e[d];
        }
        phi_c = phi_p;
        phi_p = q1.phi2;
        pr_c = q1.pr;
        pi_c = q1.pi;
        if constexpr (D2) q1 = q2;
        cur = nxt;
    }

    if constexpr (MEAS) {
        // fixed-order block reduction of the diagnostics into one record
        static_assert(M_KIN == 0 && kMarchSums == M_RHOL + 1, "march sums occupy slots 0 .. M_RHOL");
        auto& red = mx->red;
        const int lane = tid & 63, wv = tid >> 6;
        for (int k = 0; k < kMarchSums; ++k) {
            const double r = wave_sum(acc(k));
            if (lane == 0) red[wv][k] = r;
        }
        const double rw = wave_sum((double)wabs), rn = wave_sum((double)nonfin);
        if (lane == 0) {
            red[wv][M_WABS] = rw;
            red[wv][M_NONFIN] = rn;
        }
        if constexpr (GAUSS) {
            const double v[4] = {wave_sum(g2), wave_sum(d2), wave_sum(c2), wave_max(gmax)};
            if (lane == 0) {
                red[wv][M_G2] = v[0];
                red[wv][M_DIV2] = v[1];
                red[wv][M_CRHO2] = v[2];
                red[wv][M_GMAX] = v[3];
            }
        }
        __syncthreads();
        if (tid < kMeasStride) {
            const bool gslot = tid == M_G2 || tid == M_DIV2 || tid == M_CRHO2 || tid == M_GMAX;
            double r = 0.0;
            if (tid < kMarchSums || tid == M_WABS || tid == M_NONFIN || (GAUSS && gslot)) {
                r = red[0][tid];
                for (int w = 1; w < NT / 64; ++w) r = tid == M_GMAX ? fmax(r, red[w][tid]) : r + red[w][tid];
            }
            record[tid] = r;
        }
    }
}

// Waves per SIMD the compiler must leave room for.  The plain FP32 march
// fits in 128 registers, i.e. four waves per SIMD: two 512-thread workgroups
// per CU, so one can load while the other waits at a barrier.  Left to itself
// the compiler may take a few more registers, which drops a 512-thread tile
// to one workgroup per CU.  FP64 fits two waves per SIMD (its measured march
// only with its sums in LDS and its loads issued late).  Three waves of the
// plain FP64 march on 256-thread tiles, which fit 168 registers only with
// late loads (or spill with early ones), ran slower than two on 64 x 8.  The
// FP32 measured march needs more than 128 registers and is left free.
template <typename R, bool MEAS>
constexpr int kMinWaves = sizeof(R) == 8 ? 2 : (MEAS ? 1 : 4);

// Tile shapes with a measured instance.  Lattices are measured on 64 x 8
// (FP32) and 32 x 8 (FP64) tiles; pool lattices, whose one shape serves both
// nodes, run FP32 shapes of up to 512 threads and FP64 on 32 x 8.  (The
// 1024-thread FP32 shapes would spill; the FP64 measured march fits two
// waves per SIMD only on 32 x 8.)
template <typename R>
constexpr bool has_measured(int tx, int ty)
{
    return sizeof(R) == 8 ? (tx == 32 && ty == 8) : tx * ty <= 512;
}

// One lattice: block b owns tile t = xcd_tile(b) (tx fastest, then ty, then
// z-chunk); with MEAS it writes diagnostics record t, so the records are in
// tile order whatever the launch geometry.
template <typename R, int TX, int TY, bool MEAS>
__global__ void __launch_bounds__(TX* TY, (kMinWaves<R, MEAS>)) k_step_tile(StepArgs<R> a, MeasArgs ma, double* partials, int write,
                                                      int zchunk, int tiles_x, int tiles_y)
{
    __shared__ TileShared<R, TX, TY> sh;
    __shared__ MeasShared<R, TX, MEAS ? TY : 8> mxs;
    const int t0 = xcd_tile(blockIdx.x, gridDim.x);
    int t = t0;
    const int tx = t % tiles_x;
    t /= tiles_x;
    const int ty = t % tiles_y;
    const int tz = t / tiles_y;
    const int z0 = tz * zchunk;
    const int z1 = (z0 + zchunk < a.N) ? z0 + zchunk : a.N;
    if constexpr (MEAS)
        march_step<R, TX, TY, true>(sh, &mxs, a, ma, partials + (int64_t)t0 * kMeasStride, write != 0, tx * TX,
                                    ty * TY, z0, z1);
    else
        march_step<R, TX, TY, false>(sh, nullptr, a, ma, nullptr, true, tx * TX, ty * TY, z0, z1);
}


// Many lattices in one launch: blocks stride over a work list of
// (lattice, tile) items; each lattice reads its own step counter k, takes the
// coefficients of step k from its own FP64 table, and is skipped once it has
// run its steps.  MEAS: only lattices whose snapshot k is due for diagnostics
// (measured step, or measurement alone for the final snapshot); otherwise
// only lattices that are not due.

template <typename R, int TX, int TY, bool MEAS>
__global__ void __launch_bounds__(TX* TY, (kMinWaves<R, MEAS>)) k_step_batch(const PoolLattice* __restrict__ lat,
                                                       const WorkItem* __restrict__ work, int nwork)
{
    __shared__ TileShared<R, TX, TY> sh;
    __shared__ MeasShared<R, TX, MEAS ? TY : 8> mxs;
    // one work item per block; XCD x gets the x-th eighth of the list (the
    // host lays the list out so that this is an equal share of every lattice)
    const int w = xcd_tile(blockIdx.x, nwork);
    const WorkItem it = work[w];
    if (it.lattice < 0) return;
    const PoolLattice& L = lat[it.lattice];
    const int64_t k = L.counter[0];
    const bool due = measure_due(L, k);
    if (MEAS != due) return;                     // uniform across the block
    if (!MEAS && (k >= L.nsteps || two_step_due(L, k))) return;
    const double* row = L.coef + k * kCoefStride;
    const int cur = (int)L.counter[2], curm = (int)L.counter[3];
    StepArgs<R> a;
    a.f = Fields<R>{(R*)L.pp[cur][0], (R*)L.pp[cur][1], (R*)L.mom[curm][0], (R*)L.mom[curm][1], (R*)L.pp[cur][2],
                    (R*)L.pp[cur][3], (R*)L.pp[cur][4], (R*)L.mom[curm][2], (R*)L.mom[curm][3], (R*)L.mom[curm][4]};
    a.ophr = (R*)L.pp[cur ^ 1][0];
    a.ophi = (R*)L.pp[cur ^ 1][1];
    a.oa0 = (R*)L.pp[cur ^ 1][2];
    a.oa1 = (R*)L.pp[cur ^ 1][3];
    a.oa2 = (R*)L.pp[cur ^ 1][4];
    // Pi and E in place, but out of place for the measured march
    const int om = MEAS ? curm ^ 1 : curm;
    a.opr = (R*)L.mom[om][0];
    a.opi = (R*)L.mom[om][1];
    a.oe0 = (R*)L.mom[om][2];
    a.oe1 = (R*)L.mom[om][3];
    a.oe2 = (R*)L.mom[om][4];
    a.N = L.N;
    a.P = L.P;
    a.dx = (R)L.dx;
    a.sigma2 = (R)L.sigma2;
    a.cP1 = (R)row[C_P1];
    a.cP2 = (R)row[C_P2];
    a.cE1 = (R)row[C_E1];
    a.cE2 = (R)row[C_E2];
    a.lamh = (R)row[C_LAMH];
    a.kappa = (R)row[C_KAPPA];
    a.deta = (R)L.deta;
    a = uniform(a);
    const MeasArgs ma = uniform(MeasArgs{L.dx, row[C_INV2E2F], row[C_LAMQ], row[C_GAUSS]});
    // the measured node runs the lattice's measured tiling, the plain node its step tiling
    const int tiles_x = MEAS ? L.mtiles_x : L.tiles_x, tiles_y = MEAS ? L.mtiles_y : L.tiles_y;
    const int zchunk = MEAS ? L.meas_zchunk : L.zchunk;
    int t = it.tile;
    const int tx = t % tiles_x;
    t /= tiles_x;
    const int ty = t % tiles_y;
    const int tz = t / tiles_y;
    const int z0 = uniform(tz * zchunk);
    const int z1 = uniform((z0 + zchunk < L.N) ? z0 + zchunk : L.N);
    const int x0 = uniform(tx * TX), y0 = uniform(ty * TY);
    if constexpr (MEAS)
        march_step<R, TX, TY, true>(sh, &mxs, a, ma, uniform(L.partials + (int64_t)it.tile * kMeasStride),
                                    k < L.nsteps, x0, y0, z0, z1);
    else
        march_step<R, TX, TY, false>(sh, nullptr, a, ma, nullptr, true, x0, y0, z0, z1);
}


// Fold the records of every due lattice into its measurement series (one
// block per lattice, the same fixed order as the single-lattice fold).
__global__ void __launch_bounds__(256) k_fold_batch(const PoolLattice* __restrict__ lat, int nlat)
{
    __shared__ double red[256];
    const PoolLattice& L = lat[blockIdx.x];
    const int64_t k = L.counter[0];
    if (!measure_due(L, k)) return;
    const int64_t slot = L.counter[1];
    if (slot >= L.series_cap) return;
    double* out = L.series + slot * kSeriesStride;
    fold_records(L.partials, L.meas_blocks, out, red);
    if (threadIdx.x == 0) {
        out[M_COUNT] = (double)k;
        L.counter[1] = slot + 1;
    }
}

// Advance the counter of every pool lattice that is not finished by what
// this replay did to it: the final measurement one step; a single step one
// step and the phi/A buffer, and the Pi/E buffer too if it was a measured
// step; a two-step pass two steps and both buffers.
__global__ void k_advance_batch(const PoolLattice* __restrict__ lat, int nlat)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nlat) return;
    const PoolLattice& L = lat[i];
    int64_t* c = L.counter;
    const int64_t k = c[0];
    if (k > L.nsteps) return;
    if (k == L.nsteps) {
        c[0] = k + 1;  // the final measurement: finished
    } else if (two_step_due(L, k)) {
        c[0] = k + 2;
        c[2] ^= 1;
        c[3] ^= 1;
    } else {
        c[0] = k + 1;
        c[2] ^= 1;
        if (measure_due(L, k)) c[3] ^= 1;
    }
}

}  // namespace

template <typename R>
hipError_t launch_step_tile(const Fields<R>& in, const Fields<R>& out, const LatticeConst& L, const StepCoef& c,
                            const TileConfig& tc, const MeasConst* mc, double* partials, bool write, hipStream_t s)
{
    const int N = L.N;
    // a measured step reads E of neighbours that other workgroups update:
    // its Pi and E go to other buffers
    if (mc && write && (out.pir == in.pir || out.pii == in.pii || out.e0 == in.e0 || out.e1 == in.e1 ||
                        out.e2 == in.e2))
        return hipErrorInvalidValue;
    StepArgs<R> a;
    a.f = in;
    a.ophr = out.phr;
    a.ophi = out.phi;
    a.oa0 = out.a0;
    a.oa1 = out.a1;
    a.oa2 = out.a2;
    a.opr = out.pir;
    a.opi = out.pii;
    a.oe0 = out.e0;
    a.oe1 = out.e1;
    a.oe2 = out.e2;
    a.N = N;
    a.P = L.P;
    a.dx = (R)L.dx;
    a.sigma2 = (R)L.sigma2;
    a.cP1 = (R)c.cP1;
    a.cP2 = (R)c.cP2;
    a.cE1 = (R)c.cE1;
    a.cE2 = (R)c.cE2;
    a.lamh = (R)c.lam_half;
    a.kappa = (R)c.kappa;
    a.deta = (R)L.deta;
    MeasArgs ma{L.dx, 0.0, 0.0, 0.0};
    if (mc) {
        ma.inv_2e2f = mc->inv_2e2f;
        ma.lam_quarter = mc->lam_quarter;
        ma.gauss_c = mc->gauss_c;
    }
    const int zc = tc.zchunk > 0 ? tc.zchunk : N;
    // MEASv: whether the shape has a measured instance
#define AH_TILE_CASE(TXv, TYv, MEASv)                                                                              \
    if (tc.tx == TXv && tc.ty == TYv) {                                                                            \
        const int tiles_x = (N + TXv - 1) / TXv, tiles_y = (N + TYv - 1) / TYv;                                   \
        const int nb = tiles_x * tiles_y * ((N + zc - 1) / zc);                                                   \
        if (mc) {                                                                                                  \
            if constexpr (!MEASv) return hipErrorInvalidValue;                                                     \
            else                                                                                                   \
                hipLaunchKernelGGL((k_step_tile<R, TXv, TYv, MEASv>), dim3(nb), dim3(TXv * TYv), 0, s, a, ma,      \
                                   partials, write ? 1 : 0, zc, tiles_x, tiles_y);                                \
        } else {                                                                                                   \
            hipLaunchKernelGGL((k_step_tile<R, TXv, TYv, false>), dim3(nb), dim3(TXv * TYv), 0, s, a, ma, partials, \
                               1, zc, tiles_x, tiles_y);                                                          \
        }                                                                                                          \
        return hipGetLastError();                                                                                 \
    }
    AH_TILE_CASE(64, 8, has_measured<R>(64, 8))
    AH_TILE_CASE(64, 4, has_measured<R>(64, 4))
    AH_TILE_CASE(32, 8, has_measured<R>(32, 8))
    AH_TILE_CASE(128, 4, has_measured<R>(128, 4))
    if constexpr (sizeof(R) == 4) {
        AH_TILE_CASE(64, 16, false)
        AH_TILE_CASE(128, 8, false)
    }
#undef AH_TILE_CASE
    return hipErrorInvalidValue;
}

int step_tile_blocks(int N, const TileConfig& tc)
{
    const int zc = tc.zchunk > 0 ? tc.zchunk : N;
    return ((N + tc.tx - 1) / tc.tx) * ((N + tc.ty - 1) / tc.ty) * ((N + zc - 1) / zc);
}

template <typename R>
hipError_t launch_step_batch(const PoolLattice* lat, const WorkItem* work, int nwork, int tx, int ty, int grid,
                             bool measured, hipStream_t s)
{
    // plain node: the shapes of batch_tile_supported; measured node: the
    // measured march's shape (measured_tile)
    if (measured) {
        int mx = 0, my = 0;
        (void)measured_tile(sizeof(R) == 8 ? AH_FP64 : AH_FP32, &mx, &my);
        if (tx != mx || ty != my) return hipErrorInvalidValue;
        if constexpr (sizeof(R) == 8)
            hipLaunchKernelGGL((k_step_batch<R, 32, 8, true>), dim3(grid), dim3(256), 0, s, lat, work, nwork);
        else
            hipLaunchKernelGGL((k_step_batch<R, 64, 8, true>), dim3(grid), dim3(512), 0, s, lat, work, nwork);
        return hipGetLastError();
    }
    if (!batch_tile_supported(sizeof(R) == 8 ? AH_FP64 : AH_FP32, tx, ty)) return hipErrorInvalidValue;
#define AH_BATCH_CASE(TXv, TYv)                                                                                   \
    if (tx == TXv && ty == TYv) {                                                                                 \
        hipLaunchKernelGGL((k_step_batch<R, TXv, TYv, false>), dim3(grid), dim3(TXv * TYv), 0, s, lat, work, nwork); \
        return hipGetLastError();                                                                                 \
    }
    AH_BATCH_CASE(64, 8)
    AH_BATCH_CASE(64, 4)
    AH_BATCH_CASE(32, 8)
    if constexpr (sizeof(R) == 4) {
        AH_BATCH_CASE(128, 4)
        AH_BATCH_CASE(128, 8)
    }
#undef AH_BATCH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_fold_batch(const PoolLattice* lat, int nlat, hipStream_t s)
{
    hipLaunchKernelGGL(k_fold_batch, dim3(nlat), dim3(256), 0, s, lat, nlat);
    return hipGetLastError();
}

hipError_t launch_advance_batch(const PoolLattice* lat, int nlat, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance_batch, dim3((nlat + 63) / 64), dim3(64), 0, s, lat, nlat);
    return hipGetLastError();
}

template hipError_t launch_step_batch<double>(const PoolLattice*, const WorkItem*, int, int, int, int, bool,
                                              hipStream_t);
template hipError_t launch_step_batch<float>(const PoolLattice*, const WorkItem*, int, int, int, int, bool,
                                             hipStream_t);

template hipError_t launch_step_tile<double>(const Fields<double>&, const Fields<double>&, const LatticeConst&,
                                             const StepCoef&, const TileConfig&, const MeasConst*, double*, bool,
                                             hipStream_t);
template hipError_t launch_step_tile<float>(const Fields<float>&, const Fields<float>&, const LatticeConst&,
                                            const StepCoef&, const TileConfig&, const MeasConst*, double*, bool,
                                            hipStream_t);

}  // namespace ah
