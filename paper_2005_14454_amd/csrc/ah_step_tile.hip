// Tiled, z-marching leapfrog step for gfx950 (compact gauge action).
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
#include "ah_internal.h"

#pragma clang fp contract(off)

namespace ah {
namespace {

__device__ inline float fm(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fm(double a, double b, double c) { return __builtin_fma(a, b, c); }

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

__device__ inline void sincos_t(double x, double* s, double* c) { sincos(x, s, c); }
__device__ inline void sincos_t(float x, float* s, float* c) { sincosf(x, s, c); }

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
    // v in [-1, 2N + TX]: periodic image in [0, N)
    if (v < 0) return v + N;
    return v < N ? v : v % N;
}

// Place tiles so that the blocks the hardware sends to one XCD (block b goes
// to XCD b % 8) cover a contiguous range of tile indices.
__device__ inline int xcd_tile(int b, int nb)
{
    constexpr int kXcd = 8;
    const int per = nb / kXcd, rem = nb % kXcd;
    const int xcd = b % kXcd, k = b / kXcd;
    return xcd * per + (xcd < rem ? xcd : rem) + k;
}

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
    int N;
    R dx, sigma2, cP1, cP2, cE1, cE2, lamh, kappa, deta;
};

template <typename R, int TX, int TY>
struct TileShared {
    static constexpr int RS = TileGeom<R, TX, TY>::RS;
    Cx<R> U[2][3][RS];  // links of planes z and z+1 (ring)
    Cx<R> Phi[RS];      // phi of plane z
};

// Walk planes [z0, z1) of the tile whose lower corner is (x0, y0): kick and
// drift every own site.  All threads of the workgroup must call this with
// the same arguments; it synchronises the workgroup internally.
template <typename R, int TX, int TY>
__device__ void march_step(TileShared<R, TX, TY>& sh, const StepArgs<R>& a, int x0, int y0, int z0, int z1)
{
    using G = TileGeom<R, TX, TY>;
    constexpr int RW = G::RW, H = G::H;
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

    const R inv_dx = R(1) / dx;
    const R inv_dx2 = inv_dx * inv_dx;
    const int64_t NN = (int64_t)N * N;

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool active = gx < N && gy < N;
    const int64_t own_xy = (int64_t)wrapi(gx, N) + (int64_t)N * wrapi(gy, N);
    const int ro = (ly + 1) * RW + (lx + 1);  // own region slot

    // halo ring site of this thread (if any)
    const bool has_halo = tid < H;
    int rh = 0;
    int64_t halo_xy = 0;
    if (has_halo) {
        int rx, ry;
        if (tid < RW) {
            rx = tid;
            ry = 0;
        } else if (tid < 2 * RW) {
            rx = tid - RW;
            ry = TY + 1;
        } else if (tid < 2 * RW + TY) {
            rx = 0;
            ry = 1 + (tid - 2 * RW);
        } else {
            rx = TX + 1;
            ry = 1 + (tid - 2 * RW - TY);
        }
        rh = ry * RW + rx;
        halo_xy = (int64_t)wrapi(x0 - 1 + rx, N) + (int64_t)N * wrapi(y0 - 1 + ry, N);
    }

    // neighbour slots in the region
    const int rxm = ro - 1, rxp = ro + 1, rym = ro - RW, ryp = ro + RW;
    const int rxm_yp = ro - 1 + RW, rxp_ym = ro + 1 - RW;

    auto plane_of = [&](int z) -> int64_t { return (int64_t)wrapi(z, N) * NN; };

    // ---------------------------------------------------------------- prologue
    // U(z0-1) of the region into slot 1, U(z0) into slot 0, phi(z0) into sPhi.
    Cx<R> Uc[3], Up[3];
    R Ac[3], Ap[3];
    Cx<R> phi_m, phi_c, phi_p;
    Cx<R> uz_m;
    R fxz_m, fyz_m;
    {
        const int64_t pm = plane_of(z0 - 1), p0 = plane_of(z0);
        const R* A[3] = {f.a0, f.a1, f.a2};
        Cx<R> um[3];
        for (int d = 0; d < 3; ++d) {
            um[d] = link(dx, A[d][pm + own_xy]);
            sU[1][d][ro] = um[d];
            Ac[d] = A[d][p0 + own_xy];
            Uc[d] = link(dx, Ac[d]);
            sU[0][d][ro] = Uc[d];
        }
        if (has_halo)
            for (int d = 0; d < 3; ++d) {
                sU[1][d][rh] = link(dx, A[d][pm + halo_xy]);
                sU[0][d][rh] = link(dx, A[d][p0 + halo_xy]);
            }
        phi_m = {f.phr[pm + own_xy], f.phi[pm + own_xy]};
        phi_c = {f.phr[p0 + own_xy], f.phi[p0 + own_xy]};
        sPhi[ro] = phi_c;
        if (has_halo) sPhi[rh] = Cx<R>{f.phr[p0 + halo_xy], f.phi[p0 + halo_xy]};
        uz_m = um[2];
        __syncthreads();
        // F_xz, F_yz of the own column at plane z0-1
        fxz_m = plaq_sin(um[0], sU[1][2][rxp], Uc[0], um[2]) * inv_dx2;
        fyz_m = plaq_sin(um[1], sU[1][2][ryp], Uc[1], um[2]) * inv_dx2;
        __syncthreads();
        // U(z0+1) into slot 1
        const int64_t p1 = plane_of(z0 + 1);
        for (int d = 0; d < 3; ++d) {
            Ap[d] = A[d][p1 + own_xy];
            Up[d] = link(dx, Ap[d]);
            sU[1][d][ro] = Up[d];
        }
        if (has_halo)
            for (int d = 0; d < 3; ++d) sU[1][d][rh] = link(dx, A[d][p1 + halo_xy]);
        phi_p = {f.phr[p1 + own_xy], f.phi[p1 + own_xy]};
        __syncthreads();
    }

    R pr_c = f.pir[(int64_t)z0 * NN + own_xy], pi_c = f.pii[(int64_t)z0 * NN + own_xy];
    R e_c[3] = {f.e0[(int64_t)z0 * NN + own_xy], f.e1[(int64_t)z0 * NN + own_xy], f.e2[(int64_t)z0 * NN + own_xy]};

    int cur = 0;
    for (int z = z0; z < z1; ++z) {
        const int nxt = cur ^ 1;
        const bool more = z + 1 < z1;  // is there a next iteration?
        // ---- 0. issue loads for the preparation of the next plane and the
        //         own values of the next iteration
        R rA[3] = {0, 0, 0}, hA[3] = {0, 0, 0};
        Cx<R> rphi{0, 0}, hphi{0, 0}, phi_pp{0, 0};
        R n_pr = 0, n_pi = 0, n_e[3] = {0, 0, 0};
        if (more) {
            const int64_t p2 = plane_of(z + 2), p1 = plane_of(z + 1), pn = (int64_t)(z + 1) * NN;
            rA[0] = f.a0[p2 + own_xy];
            rA[1] = f.a1[p2 + own_xy];
            rA[2] = f.a2[p2 + own_xy];
            if (has_halo) {
                hA[0] = f.a0[p2 + halo_xy];
                hA[1] = f.a1[p2 + halo_xy];
                hA[2] = f.a2[p2 + halo_xy];
                hphi = {f.phr[p1 + halo_xy], f.phi[p1 + halo_xy]};
            }
            phi_pp = {f.phr[p2 + own_xy], f.phi[p2 + own_xy]};
            n_pr = f.pir[pn + own_xy];
            n_pi = f.pii[pn + own_xy];
            n_e[0] = f.e0[pn + own_xy];
            n_e[1] = f.e1[pn + own_xy];
            n_e[2] = f.e2[pn + own_xy];
        }
        rphi = phi_p;

        // ---- 1. update of the own site at plane z
        {
            const Cx<R> ph_xm = sPhi[rxm], ph_xp = sPhi[rxp], ph_ym = sPhi[rym], ph_yp = sPhi[ryp];
            const Cx<R> ux_xm = sU[cur][0][rxm];  // U_x^{x-kx}
            const Cx<R> uy_ym = sU[cur][1][rym];  // U_y^{x-ky}
            // covariant Laplacian: sum_j U_j^x phi^{x+j} + conj(U_j^{x-j}) phi^{x-j} - 2 phi^x
            const Cx<R> fx = cmul(Uc[0], ph_xp), fy = cmul(Uc[1], ph_yp), fz = cmul(Uc[2], phi_p);
            const Cx<R> bx = cmulc(ux_xm, ph_xm), by = cmulc(uy_ym, ph_ym), bz = cmulc(uz_m, phi_m);
            const R lr = ((fx.r + bx.r) + (fy.r + by.r)) + fm(R(-6), phi_c.r, fz.r + bz.r);
            const R li = ((fx.i + bx.i) + (fy.i + by.i)) + fm(R(-6), phi_c.i, fz.i + bz.i);
            // currents J_i = Im[conj(phi) U_i phi^{x+i}] / dx
            const R jx = fm(phi_c.r, fx.i, -(phi_c.i * fx.r)) * inv_dx;
            const R jy = fm(phi_c.r, fy.i, -(phi_c.i * fy.r)) * inv_dx;
            const R jz = fm(phi_c.r, fz.i, -(phi_c.i * fz.r)) * inv_dx;
            // plaquettes at x (F_ij^x, i<j)
            const Cx<R> uy_xp = sU[cur][1][rxp], ux_yp = sU[cur][0][ryp];
            const Cx<R> uz_xp = sU[cur][2][rxp], uz_yp = sU[cur][2][ryp];
            const R fxy = plaq_sin(Uc[0], uy_xp, ux_yp, Uc[1]) * inv_dx2;
            const R fxz = plaq_sin(Uc[0], uz_xp, Up[0], Uc[2]) * inv_dx2;
            const R fyz = plaq_sin(Uc[1], uz_yp, Up[1], Uc[2]) * inv_dx2;
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
            const R pot = lamh * fm(phi_c.r, phi_c.r, fm(phi_c.i, phi_c.i, -sigma2));
            const R npr = fm(cP1, pr_c, cP2 * fm(lr, inv_dx2, -(pot * phi_c.r)));
            const R npi = fm(cP1, pi_c, cP2 * fm(li, inv_dx2, -(pot * phi_c.i)));
            const R ne0 = fm(cE1, e_c[0], cE2 * fm(kappa, jx, -cx));
            const R ne1 = fm(cE1, e_c[1], cE2 * fm(kappa, jy, -cy));
            const R ne2 = fm(cE1, e_c[2], cE2 * fm(kappa, jz, -cz));
            if (active) {
                const int64_t o = (int64_t)z * NN + own_xy;
                f.pir[o] = npr;
                f.pii[o] = npi;
                f.e0[o] = ne0;
                f.e1[o] = ne1;
                f.e2[o] = ne2;
                ophr[o] = fm(deta, npr, phi_c.r);
                ophi[o] = fm(deta, npi, phi_c.i);
                oa0[o] = fm(deta, ne0, Ac[0]);
                oa1[o] = fm(deta, ne1, Ac[1]);
                oa2[o] = fm(deta, ne2, Ac[2]);
            }
            fxz_m = fxz;
            fyz_m = fyz;
        }
        if (!more) break;
        __syncthreads();  // all reads of slot cur and of sPhi (plane z) are done

        // ---- 3. plane z+2 links into slot cur, plane z+1 phi into sPhi
        Cx<R> Upp[3];
        for (int d = 0; d < 3; ++d) {
            Upp[d] = link(dx, rA[d]);
            sU[cur][d][ro] = Upp[d];
        }
        if (has_halo) {
            for (int d = 0; d < 3; ++d) sU[cur][d][rh] = link(dx, hA[d]);
            sPhi[rh] = hphi;
        }
        sPhi[ro] = rphi;
        __syncthreads();

        // ---- 5. rotate the own-column registers
        uz_m = Uc[2];
        for (int d = 0; d < 3; ++d) {
            Uc[d] = Up[d];
            Up[d] = Upp[d];
            Ac[d] = Ap[d];
            Ap[d] = rA[d];
            e_c[d] = n_e[d];
        }
        phi_m = phi_c;
        phi_c = phi_p;
        phi_p = phi_pp;
        pr_c = n_pr;
        pi_c = n_pi;
        cur = nxt;
    }
}

// One lattice: block b owns tile xcd_tile(b) (tx fastest, then ty, then z-chunk).
template <typename R, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) k_step_tile(StepArgs<R> a, int zchunk, int tiles_x, int tiles_y)
{
    __shared__ TileShared<R, TX, TY> sh;
    int t = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = t % tiles_x;
    t /= tiles_x;
    const int ty = t % tiles_y;
    const int tz = t / tiles_y;
    const int z0 = tz * zchunk;
    const int z1 = (z0 + zchunk < a.N) ? z0 + zchunk : a.N;
    march_step<R, TX, TY>(sh, a, tx * TX, ty * TY, z0, z1);
}

// Many lattices in one launch: blocks stride over a work list of
// (lattice, tile) items; each lattice reads its own step counter, skips the
// work once it has run its steps, and takes the coefficients of its current
// step from its own FP64 table.
template <typename R, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) k_step_batch(const PoolLattice* __restrict__ lat,
                                                       const WorkItem* __restrict__ work, int nwork)
{
    __shared__ TileShared<R, TX, TY> sh;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const WorkItem it = work[w];
        const PoolLattice& L = lat[it.lattice];
        const int64_t k = *L.counter;
        if (k >= L.nsteps) continue;  // uniform across the block
        const double* row = L.coef + k * kCoefStride;
        const int cur = (int)(k & 1);
        StepArgs<R> a;
        a.f = Fields<R>{(R*)L.pp[cur][0], (R*)L.pp[cur][1], (R*)L.mom[0], (R*)L.mom[1], (R*)L.pp[cur][2],
                        (R*)L.pp[cur][3], (R*)L.pp[cur][4], (R*)L.mom[2], (R*)L.mom[3], (R*)L.mom[4]};
        a.ophr = (R*)L.pp[cur ^ 1][0];
        a.ophi = (R*)L.pp[cur ^ 1][1];
        a.oa0 = (R*)L.pp[cur ^ 1][2];
        a.oa1 = (R*)L.pp[cur ^ 1][3];
        a.oa2 = (R*)L.pp[cur ^ 1][4];
        a.N = L.N;
        a.dx = (R)L.dx;
        a.sigma2 = (R)L.sigma2;
        a.cP1 = (R)row[C_P1];
        a.cP2 = (R)row[C_P2];
        a.cE1 = (R)row[C_E1];
        a.cE2 = (R)row[C_E2];
        a.lamh = (R)row[C_LAMH];
        a.kappa = (R)row[C_KAPPA];
        a.deta = (R)L.deta;
        int t = it.tile;
        const int tx = t % L.tiles_x;
        t /= L.tiles_x;
        const int ty = t % L.tiles_y;
        const int tz = t / L.tiles_y;
        const int z0 = tz * L.zchunk;
        const int z1 = (z0 + L.zchunk < L.N) ? z0 + L.zchunk : L.N;
        march_step<R, TX, TY>(sh, a, tx * TX, ty * TY, z0, z1);
        __syncthreads();  // LDS is reused by the next item
    }
}

}  // namespace

template <typename R>
hipError_t launch_step_tile(const Fields<R>& in, R* ophr, R* ophi, R* oa0, R* oa1, R* oa2, const LatticeConst& L,
                            const StepCoef& c, const TileConfig& tc, hipStream_t s)
{
    const int N = L.N;
    StepArgs<R> a;
    a.f = in;
    a.ophr = ophr;
    a.ophi = ophi;
    a.oa0 = oa0;
    a.oa1 = oa1;
    a.oa2 = oa2;
    a.N = N;
    a.dx = (R)L.dx;
    a.sigma2 = (R)L.sigma2;
    a.cP1 = (R)c.cP1;
    a.cP2 = (R)c.cP2;
    a.cE1 = (R)c.cE1;
    a.cE2 = (R)c.cE2;
    a.lamh = (R)c.lam_half;
    a.kappa = (R)c.kappa;
    a.deta = (R)L.deta;
#define AH_TILE_CASE(TXv, TYv)                                                                                   \
    if (tc.tx == TXv && tc.ty == TYv) {                                                                          \
        const int tiles_x = (N + TXv - 1) / TXv, tiles_y = (N + TYv - 1) / TYv;                                 \
        const int zc = tc.zchunk > 0 ? tc.zchunk : N;                                                           \
        const int tiles_z = (N + zc - 1) / zc;                                                                  \
        const int nb = tiles_x * tiles_y * tiles_z;                                                             \
        hipLaunchKernelGGL((k_step_tile<R, TXv, TYv>), dim3(nb), dim3(TXv * TYv), 0, s, a, zc, tiles_x, tiles_y);  \
        return hipGetLastError();                                                                               \
    }
    AH_TILE_CASE(64, 8)
    AH_TILE_CASE(64, 4)
    AH_TILE_CASE(32, 8)
    if constexpr (sizeof(R) == 4) {
        AH_TILE_CASE(64, 16)
    }
#undef AH_TILE_CASE
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_step_batch(const PoolLattice* lat, const WorkItem* work, int nwork, int tx, int ty, int grid,
                             hipStream_t s)
{
#define AH_BATCH_CASE(TXv, TYv)                                                                               \
    if (tx == TXv && ty == TYv) {                                                                             \
        hipLaunchKernelGGL((k_step_batch<R, TXv, TYv>), dim3(grid), dim3(TXv * TYv), 0, s, lat, work, nwork); \
        return hipGetLastError();                                                                            \
    }
    AH_BATCH_CASE(64, 8)
    AH_BATCH_CASE(64, 4)
    AH_BATCH_CASE(32, 8)
    if constexpr (sizeof(R) == 4) {
        AH_BATCH_CASE(64, 16)
    }
#undef AH_BATCH_CASE
    return hipErrorInvalidValue;
}

template hipError_t launch_step_batch<double>(const PoolLattice*, const WorkItem*, int, int, int, int, hipStream_t);
template hipError_t launch_step_batch<float>(const PoolLattice*, const WorkItem*, int, int, int, int, hipStream_t);

template hipError_t launch_step_tile<double>(const Fields<double>&, double*, double*, double*, double*, double*,
                                             const LatticeConst&, const StepCoef&, const TileConfig&, hipStream_t);
template hipError_t launch_step_tile<float>(const Fields<float>&, float*, float*, float*, float*, float*,
                                            const LatticeConst&, const StepCoef&, const TileConfig&, hipStream_t);

}  // namespace ah
