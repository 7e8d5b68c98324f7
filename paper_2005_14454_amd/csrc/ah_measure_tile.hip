// Tiled, z-marching diagnostics pass for gfx950 (compact gauge action).
//
// Same walk as the tiled step: a workgroup owns a TX x TY tile and a chunk
// of x2-planes, and shares per-site quantities of the current and next plane
// through LDS, so that every transcendental is evaluated once per site:
//   - links U_j = exp(-i dx A_j)        (one FP64 sincos per link)
//   - link phases Y_j = arg(conj(phi^x) U_j^x phi^{x+j})  (one FP64 atan2 per link)
// For its own sites a workgroup forms, in FP64 whatever the storage type:
//   - the centred momenta from a kick that is not stored (section 2 kick
//     equations), the site energy densities and the Lagrangian density;
//   - the Gauss residual with the stored half-step fields;
//   - the three plaquette windings: link phases around the plaquette plus
//     the plaquette angle wrapped to (-pi, pi] make a multiple of 2 pi.
// Link phases and plaquette angles use no contraction, so windings follow
// the same rounding sequence as a plain evaluation of the definition.
// Per-thread sums go through a fixed tree to one record per workgroup; the
// caller folds the records in a fixed order.
#include "ah_device.h"
#include "ah_internal.h"

#pragma clang fp contract(off)

namespace ah {
namespace {

struct Cd {
    double r, i;
};
__device__ inline Cd cmul(Cd a, Cd b) { return {fma(a.r, b.r, -(a.i * b.i)), fma(a.r, b.i, a.i * b.r)}; }
__device__ inline Cd cmulc(Cd a, Cd b) { return {fma(a.r, b.r, a.i * b.i), fma(a.r, b.i, -(a.i * b.r))}; }

__device__ inline Cd link(double dx, double a)
{
    double s, c;
    sincos(dx * a, &s, &c);
    return {c, -s};
}

// sin and 1 - cos of the plaquette angle from the four links:
// exp(-i Theta) = U_i^x U_j^{x+i} conj(U_i^{x+j} U_j^x)
__device__ inline void plaq(Cd ui_x, Cd uj_xi, Cd ui_xj, Cd uj_x, double* sn, double* omc)
{
    const Cd p = cmul(ui_x, uj_xi);
    const Cd q = cmul(ui_xj, uj_x);
    const double c = fma(p.r, q.r, p.i * q.i);
    const double s = fma(p.r, q.i, -(p.i * q.r));
    *sn = s;
    // 1 - cos without cancellation for small angles
    *omc = c > 0.0 ? (s * s) / (1.0 + c) : 1.0 - c;
}
__device__ inline double plaq_sin(Cd ui_x, Cd uj_xi, Cd ui_xj, Cd uj_x)
{
    const Cd p = cmul(ui_x, uj_xi);
    const Cd q = cmul(ui_xj, uj_x);
    return fma(p.r, q.i, -(p.i * q.r));
}

// arg(conj(phx) U phn) in (-pi, pi]; plain products and sums, -0 -> +0
__device__ inline double link_phase(Cd phx, Cd U, Cd phn)
{
    const double wr = U.r * phn.r - U.i * phn.i;
    const double wi = U.r * phn.i + U.i * phn.r;
    const double zr = phx.r * wr + phx.i * wi;
    double zi = phx.r * wi - phx.i * wr;
    zi = (zi == 0.0) ? 0.0 : zi;
    return atan2(zi, zr);
}

__device__ inline int winding(double y1, double y2, double y3, double y4, double th)
{
    const double two_pi = 6.283185307179586;
    const double thw = th - two_pi * rint(th / two_pi);
    const double sum = (((y1 + y2) - y3) - y4) + thw;
    return (int)rint(sum / two_pi);
}

__device__ inline int wrapi(int v, int N)
{
    if (v < 0) return v + N;
    return v < N ? v : v % N;
}

__device__ inline int xcd_tile(int b, int nb)
{
    constexpr int kXcd = 8;
    const int per = nb / kXcd, rem = nb % kXcd;
    const int xcd = b % kXcd, k = b / kXcd;
    return xcd * per + (xcd < rem ? xcd : rem) + k;
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

template <int TX, int TY>
struct MeasShared {
    static constexpr int RS = (TX + 2) * (TY + 2);
    Cd U[2][3][RS];     // links of planes z and z+1
    Cd Phi[2][RS];      // phi of planes z and z+1
    double Y[3][RS];    // link phases of plane z
    double red[TX * TY / 64][M_COUNT];
};

// Diagnostics of the planes [z0, z1) of the tile at (x0, y0); the workgroup's
// fixed-order sums go to record[0 .. M_COUNT).  Every thread of the workgroup
// calls this with the same arguments.
template <typename R, int TX, int TY>
__device__ void march_measure(MeasShared<TX, TY>& sh, const Fields<R>& f, int N, double dx, double sigma2,
                              const StepCoef& cf, const MeasConst& mc, int x0, int y0, int z0, int z1,
                              double* __restrict__ record)
{
    constexpr int RW = TX + 2, H = 2 * RW + 2 * TY, NT = TX * TY;
    static_assert(H <= NT, "halo must fit one extra site per thread");
    auto& sU = sh.U;
    auto& sPhi = sh.Phi;
    auto& sY = sh.Y;

    const double inv_dx = 1.0 / dx, inv_dx2 = inv_dx * inv_dx, inv_dx4 = inv_dx2 * inv_dx2;
    const int64_t NN = (int64_t)N * N;

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool active = gx < N && gy < N;
    const int gxw = wrapi(gx, N), gyw = wrapi(gy, N);
    const int64_t own_xy = (int64_t)gxw + (int64_t)N * gyw;
    const int64_t xm_xy = (int64_t)wrapi(gxw - 1, N) + (int64_t)N * gyw;
    const int64_t ym_xy = (int64_t)gxw + (int64_t)N * wrapi(gyw - 1, N);
    const int64_t xp_xy = (int64_t)wrapi(gxw + 1, N) + (int64_t)N * gyw;
    const int64_t yp_xy = (int64_t)gxw + (int64_t)N * wrapi(gyw + 1, N);
    const int ro = (ly + 1) * RW + (lx + 1);

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
        halo_xy = (int64_t)wrapi(x0 - 1 + hrx, N) + (int64_t)N * wrapi(y0 - 1 + hry, N);
    }
    // halo sites whose link phases the plaquettes of the tile need
    const bool halo_top = has_halo && hry == TY + 1 && hrx >= 1 && hrx <= TX;    // needs Y_x, Y_z
    const bool halo_right = has_halo && hrx == TX + 1 && hry >= 1 && hry <= TY;  // needs Y_y, Y_z

    const int rxm = ro - 1, rxp = ro + 1, rym = ro - RW, ryp = ro + RW;
    const int rxm_yp = ro - 1 + RW, rxp_ym = ro + 1 - RW;
    auto plane_of = [&](int z) -> int64_t { return (int64_t)wrapi(z, N) * NN; };
    const R* A[3] = {f.a0, f.a1, f.a2};

    double acc[M_COUNT];
    for (int k = 0; k < M_COUNT; ++k) acc[k] = 0.0;

    // ---------------------------------------------------------------- prologue
    Cd Uc[3], Up[3];
    double Ac[3], Ap[3];
    Cd phi_m, phi_c, phi_p;
    Cd uz_m;
    double fxz_m, fyz_m, ez_m;
    double yx_c, yy_c;  // own link phases Y_x, Y_y of the current plane
    {
        const int64_t pm = plane_of(z0 - 1), p0 = plane_of(z0), p1 = plane_of(z0 + 1);
        Cd um[3];
        for (int d = 0; d < 3; ++d) {
            um[d] = link(dx, (double)A[d][pm + own_xy]);
            sU[1][d][ro] = um[d];
            Ac[d] = (double)A[d][p0 + own_xy];
            Uc[d] = link(dx, Ac[d]);
            sU[0][d][ro] = Uc[d];
        }
        if (has_halo)
            for (int d = 0; d < 3; ++d) {
                sU[1][d][rh] = link(dx, (double)A[d][pm + halo_xy]);
                sU[0][d][rh] = link(dx, (double)A[d][p0 + halo_xy]);
            }
        phi_m = {(double)f.phr[pm + own_xy], (double)f.phi[pm + own_xy]};
        phi_c = {(double)f.phr[p0 + own_xy], (double)f.phi[p0 + own_xy]};
        sPhi[0][ro] = phi_c;
        if (has_halo) sPhi[0][rh] = Cd{(double)f.phr[p0 + halo_xy], (double)f.phi[p0 + halo_xy]};
        ez_m = (double)f.e2[pm + own_xy];
        uz_m = um[2];
        __syncthreads();
        fxz_m = plaq_sin(um[0], sU[1][2][rxp], Uc[0], um[2]) * inv_dx2;
        fyz_m = plaq_sin(um[1], sU[1][2][ryp], Uc[1], um[2]) * inv_dx2;
        yx_c = link_phase(phi_c, Uc[0], sPhi[0][rxp]);
        yy_c = link_phase(phi_c, Uc[1], sPhi[0][ryp]);
        __syncthreads();
        for (int d = 0; d < 3; ++d) {
            Ap[d] = (double)A[d][p1 + own_xy];
            Up[d] = link(dx, Ap[d]);
            sU[1][d][ro] = Up[d];
        }
        if (has_halo)
            for (int d = 0; d < 3; ++d) sU[1][d][rh] = link(dx, (double)A[d][p1 + halo_xy]);
        phi_p = {(double)f.phr[p1 + own_xy], (double)f.phi[p1 + own_xy]};
        sPhi[1][ro] = phi_p;
        if (has_halo) sPhi[1][rh] = Cd{(double)f.phr[p1 + halo_xy], (double)f.phi[p1 + halo_xy]};
        __syncthreads();
    }

    int cur = 0;
    for (int z = z0; z < z1; ++z) {
        const int nxt = cur ^ 1;
        const bool more = z + 1 < z1;
        const int64_t pz = (int64_t)z * NN;
        // ---- loads: own values of plane z, neighbours for Gauss and plaquette
        //      angles, and the region of plane z+2 for the preparation step
        double v[10];
        v[0] = phi_c.r;
        v[1] = phi_c.i;
        v[2] = (double)f.pir[pz + own_xy];
        v[3] = (double)f.pii[pz + own_xy];
        v[4] = Ac[0];
        v[5] = Ac[1];
        v[6] = Ac[2];
        v[7] = (double)f.e0[pz + own_xy];
        v[8] = (double)f.e1[pz + own_xy];
        v[9] = (double)f.e2[pz + own_xy];
        const double ex_xm = (double)f.e0[pz + xm_xy], ey_ym = (double)f.e1[pz + ym_xy];
        const double ay_xp = (double)f.a1[pz + xp_xy], ax_yp = (double)f.a0[pz + yp_xy];
        const double az_xp = (double)f.a2[pz + xp_xy], az_yp = (double)f.a2[pz + yp_xy];
        double rA[3] = {0, 0, 0}, hA[3] = {0, 0, 0};
        Cd rphi{0, 0}, hphi{0, 0};
        if (more) {
            const int64_t p2 = plane_of(z + 2);
            for (int d = 0; d < 3; ++d) rA[d] = (double)A[d][p2 + own_xy];
            rphi = {(double)f.phr[p2 + own_xy], (double)f.phi[p2 + own_xy]};
            if (has_halo) {
                for (int d = 0; d < 3; ++d) hA[d] = (double)A[d][p2 + halo_xy];
                hphi = {(double)f.phr[p2 + halo_xy], (double)f.phi[p2 + halo_xy]};
            }
        }

        // ---- (a) link phases of plane z: own and the +x / +y halo
        const double yz_c = link_phase(phi_c, Uc[2], phi_p);
        sY[0][ro] = yx_c;
        sY[1][ro] = yy_c;
        sY[2][ro] = yz_c;
        if (halo_top || halo_right) {
            const Cd ph = sPhi[cur][rh];
            if (halo_top) sY[0][rh] = link_phase(ph, sU[cur][0][rh], sPhi[cur][rh + 1]);
            if (halo_right) sY[1][rh] = link_phase(ph, sU[cur][1][rh], sPhi[cur][rh + RW]);
            sY[2][rh] = link_phase(ph, sU[cur][2][rh], sPhi[nxt][rh]);
        }
        __syncthreads();

        // ---- (b) own site: kick, densities, Gauss residual, windings
        // own link phases of plane z+1 (used here and carried)
        const double yx_n = link_phase(phi_p, Up[0], sPhi[nxt][rxp]);
        const double yy_n = link_phase(phi_p, Up[1], sPhi[nxt][ryp]);
        {
            const Cd ph_xm = sPhi[cur][rxm], ph_xp = sPhi[cur][rxp], ph_ym = sPhi[cur][rym], ph_yp = sPhi[cur][ryp];
            const Cd ux_xm = sU[cur][0][rxm], uy_ym = sU[cur][1][rym];
            const Cd fx = cmul(Uc[0], ph_xp), fy = cmul(Uc[1], ph_yp), fz = cmul(Uc[2], phi_p);
            const Cd bx = cmulc(ux_xm, ph_xm), by = cmulc(uy_ym, ph_ym), bz = cmulc(uz_m, phi_m);
            const double lr = ((fx.r + bx.r) + (fy.r + by.r)) + fma(-6.0, phi_c.r, fz.r + bz.r);
            const double li = ((fx.i + bx.i) + (fy.i + by.i)) + fma(-6.0, phi_c.i, fz.i + bz.i);
            const double jx = fma(phi_c.r, fx.i, -(phi_c.i * fx.r)) * inv_dx;
            const double jy = fma(phi_c.r, fy.i, -(phi_c.i * fy.r)) * inv_dx;
            const double jz = fma(phi_c.r, fz.i, -(phi_c.i * fz.r)) * inv_dx;
            const Cd uy_xp = sU[cur][1][rxp], ux_yp = sU[cur][0][ryp];
            const Cd uz_xp = sU[cur][2][rxp], uz_yp = sU[cur][2][ryp];
            double sxy, sxz, syz, oxy, oxz, oyz;
            plaq(Uc[0], uy_xp, ux_yp, Uc[1], &sxy, &oxy);
            plaq(Uc[0], uz_xp, Up[0], Uc[2], &sxz, &oxz);
            plaq(Uc[1], uz_yp, Up[1], Uc[2], &syz, &oyz);
            const double fxy = sxy * inv_dx2, fxz = sxz * inv_dx2, fyz = syz * inv_dx2;
            const Cd ux_xm_yp = sU[cur][0][rxm_yp], uy_xm = sU[cur][1][rxm], uz_xm = sU[cur][2][rxm];
            const Cd ux_ym = sU[cur][0][rym], uy_xp_ym = sU[cur][1][rxp_ym], uz_ym = sU[cur][2][rym];
            const Cd ux_xm_zp = sU[nxt][0][rxm], uy_ym_zp = sU[nxt][1][rym];
            const double fxy_xm = plaq_sin(ux_xm, Uc[1], ux_xm_yp, uy_xm) * inv_dx2;
            const double fxy_ym = plaq_sin(ux_ym, uy_xp_ym, Uc[0], uy_ym) * inv_dx2;
            const double fxz_xm = plaq_sin(ux_xm, Uc[2], ux_xm_zp, uz_xm) * inv_dx2;
            const double fyz_ym = plaq_sin(uy_ym, Uc[2], uy_ym_zp, uz_ym) * inv_dx2;
            const double cx = ((fxy - fxy_ym) + (fxz - fxz_m)) * inv_dx;
            const double cy = ((fyz - fyz_m) - (fxy - fxy_xm)) * inv_dx;
            const double cz = -((fxz - fxz_xm) + (fyz - fyz_ym)) * inv_dx;
            const double m2 = fma(phi_c.r, phi_c.r, fma(phi_c.i, phi_c.i, -sigma2));
            const double pot_force = cf.lam_half * m2;
            const double npr = fma(cf.cP1, v[2], cf.cP2 * fma(lr, inv_dx2, -(pot_force * phi_c.r)));
            const double npi = fma(cf.cP1, v[3], cf.cP2 * fma(li, inv_dx2, -(pot_force * phi_c.i)));
            const double ne0 = fma(cf.cE1, v[7], cf.cE2 * fma(cf.kappa, jx, -cx));
            const double ne1 = fma(cf.cE1, v[8], cf.cE2 * fma(cf.kappa, jy, -cy));
            const double ne2 = fma(cf.cE1, v[9], cf.cE2 * fma(cf.kappa, jz, -cz));

            if (active) {
                bool bad = false;
                for (int k = 0; k < 10; ++k) bad |= !isfinite(v[k]);
                acc[M_NONFIN] += bad ? 1.0 : 0.0;
                const double pbr = 0.5 * (v[2] + npr), pbi = 0.5 * (v[3] + npi);
                const double kin = pbr * pbr + pbi * pbi;
                double grad = 0.0;
                {
                    const double d0r = fx.r - phi_c.r, d0i = fx.i - phi_c.i;
                    const double d1r = fy.r - phi_c.r, d1i = fy.i - phi_c.i;
                    const double d2r = fz.r - phi_c.r, d2i = fz.i - phi_c.i;
                    grad = ((d0r * d0r + d0i * d0i) + (d1r * d1r + d1i * d1i) + (d2r * d2r + d2i * d2i)) * inv_dx2;
                }
                const double pot = mc.lam_quarter * m2 * m2;
                const double eb0 = 0.5 * (v[7] + ne0), eb1 = 0.5 * (v[8] + ne1), eb2 = 0.5 * (v[9] + ne2);
                const double el = (eb0 * eb0 + eb1 * eb1 + eb2 * eb2) * mc.inv_2e2f;
                const double mag = (2.0 * (oxy + oxz + oyz) * inv_dx4) * mc.inv_2e2f;
                const double L = kin - grad - pot + el - mag;
                acc[M_KIN] += kin;
                acc[M_GRAD] += grad;
                acc[M_POT] += pot;
                acc[M_EL] += el;
                acc[M_MAG] += mag;
                acc[M_L] += L;
                acc[M_KINL] += kin * L;
                acc[M_GRADL] += grad * L;

                const double dv = ((v[7] - ex_xm) * inv_dx + (v[8] - ey_ym) * inv_dx) + (v[9] - ez_m) * inv_dx;
                const double crho = mc.gauss_c * (phi_c.r * v[3] - phi_c.i * v[2]);
                const double G = dv - crho;
                acc[M_G2] += G * G;
                acc[M_DIV2] += dv * dv;
                acc[M_CRHO2] += crho * crho;
                acc[M_GMAX] = fmax(acc[M_GMAX], fabs(G));

                const double th_xy = dx * (((v[4] + ay_xp) - ax_yp) - v[5]);
                const double th_xz = dx * (((v[4] + az_xp) - Ap[0]) - v[6]);
                const double th_yz = dx * (((v[5] + az_yp) - Ap[1]) - v[6]);
                const int wxy = winding(yx_c, sY[1][rxp], sY[0][ryp], yy_c, th_xy);
                const int wxz = winding(yx_c, sY[2][rxp], yx_n, yz_c, th_xz);
                const int wyz = winding(yy_c, sY[2][ryp], yy_n, yz_c, th_yz);
                acc[M_WABS] += (double)(abs(wxy) + abs(wxz) + abs(wyz));
            }
            fxz_m = fxz;
            fyz_m = fyz;
        }
        if (!more) break;
        __syncthreads();

        // ---- (c) plane z+2 into the slots of plane z
        Cd Upp[3];
        for (int d = 0; d < 3; ++d) {
            Upp[d] = link(dx, rA[d]);
            sU[cur][d][ro] = Upp[d];
        }
        sPhi[cur][ro] = rphi;
        if (has_halo) {
            for (int d = 0; d < 3; ++d) sU[cur][d][rh] = link(dx, hA[d]);
            sPhi[cur][rh] = hphi;
        }
        __syncthreads();

        uz_m = Uc[2];
        ez_m = v[9];
        for (int d = 0; d < 3; ++d) {
            Uc[d] = Up[d];
            Up[d] = Upp[d];
            Ac[d] = Ap[d];
            Ap[d] = rA[d];
        }
        phi_m = phi_c;
        phi_c = phi_p;
        phi_p = rphi;
        yx_c = yx_n;
        yy_c = yy_n;
        cur = nxt;
    }

    // ---- fixed-order block reduction into one record per workgroup
    auto& red = sh.red;
    const int lane = tid & 63, wv = tid >> 6;
    for (int k = 0; k < M_COUNT; ++k) {
        const double r = (k == M_GMAX) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[wv][k] = r;
    }
    __syncthreads();
    if (tid < M_COUNT) {
        double r = red[0][tid];
        for (int w = 1; w < NT / 64; ++w) r = (tid == M_GMAX) ? fmax(r, red[w][tid]) : r + red[w][tid];
        record[tid] = r;
    }
}

// One lattice: block b measures tile t = xcd_tile(b) and writes record t, so
// the records are in tile order whatever the launch geometry.
template <typename R, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) k_measure_tile(Fields<R> f, int N, int zchunk, int tiles_x, int tiles_y,
                                                         double dx, double sigma2, StepCoef cf, MeasConst mc,
                                                         double* __restrict__ partials)
{
    __shared__ MeasShared<TX, TY> sh;
    const int t0 = xcd_tile(blockIdx.x, gridDim.x);
    int t = t0;
    const int tx = t % tiles_x;
    t /= tiles_x;
    const int ty = t % tiles_y;
    const int tz = t / tiles_y;
    const int z0 = tz * zchunk;
    const int z1 = (z0 + zchunk < N) ? z0 + zchunk : N;
    march_measure<R, TX, TY>(sh, f, N, dx, sigma2, cf, mc, tx * TX, ty * TY, z0, z1,
                             partials + (int64_t)t0 * kMeasStride);
}

__device__ inline bool measure_due(const PoolLattice& L, int64_t k)
{
    if (k > L.nsteps) return false;
    if (k == L.nsteps) return true;
    return L.measure_every > 0 && (k % L.measure_every) == 0;
}

// Diagnostics of every pool lattice whose current snapshot is due.
template <typename R>
__global__ void __launch_bounds__(kMeasTileX* kMeasTileY) k_measure_batch(const PoolLattice* __restrict__ lat,
                                                                          const WorkItem* __restrict__ work,
                                                                          int nwork)
{
    __shared__ MeasShared<kMeasTileX, kMeasTileY> sh;
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const WorkItem it = work[w];
        const PoolLattice& L = lat[it.lattice];
        const int64_t k = L.counter[0];
        if (!measure_due(L, k)) continue;
        const double* row = L.coef + k * kCoefStride;
        StepCoef cf{row[C_P1], row[C_P2], row[C_E1], row[C_E2], row[C_LAMH], row[C_KAPPA]};
        MeasConst mc{row[C_INV2E2F], row[C_LAMQ], row[C_GAUSS]};
        const int cur = (int)(k & 1);
        const Fields<R> f{(R*)L.pp[cur][0], (R*)L.pp[cur][1], (R*)L.mom[0], (R*)L.mom[1], (R*)L.pp[cur][2],
                          (R*)L.pp[cur][3], (R*)L.pp[cur][4], (R*)L.mom[2], (R*)L.mom[3], (R*)L.mom[4]};
        const int tiles_x = (L.N + kMeasTileX - 1) / kMeasTileX, tiles_y = (L.N + kMeasTileY - 1) / kMeasTileY;
        int t = it.tile;
        const int tx = t % tiles_x;
        t /= tiles_x;
        const int ty = t % tiles_y;
        const int tz = t / tiles_y;
        const int z0 = tz * L.meas_zchunk;
        const int z1 = (z0 + L.meas_zchunk < L.N) ? z0 + L.meas_zchunk : L.N;
        march_measure<R, kMeasTileX, kMeasTileY>(sh, f, L.N, L.dx, L.sigma2, cf, mc, tx * kMeasTileX,
                                                 ty * kMeasTileY, z0, z1, L.partials + (int64_t)it.tile * kMeasStride);
        __syncthreads();
    }
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

// Advance the step counter of every pool lattice that is not finished.
__global__ void k_advance_batch(const PoolLattice* __restrict__ lat, int nlat)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nlat) return;
    const int64_t k = lat[i].counter[0];
    if (k <= lat[i].nsteps) lat[i].counter[0] = k + 1;
}

}  // namespace

int measure_tile_blocks(int N, int zchunk)
{
    const int tiles = ((N + kMeasTileX - 1) / kMeasTileX) * ((N + kMeasTileY - 1) / kMeasTileY);
    return tiles * ((N + zchunk - 1) / zchunk);
}

template <typename R>
hipError_t launch_measure_tile(const Fields<R>& f, const LatticeConst& L, const StepCoef& c, const MeasConst& mc,
                               int zchunk, double* partials, double* result, hipStream_t s)
{
    const int N = L.N;
    const int tiles_x = (N + kMeasTileX - 1) / kMeasTileX, tiles_y = (N + kMeasTileY - 1) / kMeasTileY;
    const int nb = measure_tile_blocks(N, zchunk);
    hipLaunchKernelGGL((k_measure_tile<R, kMeasTileX, kMeasTileY>), dim3(nb), dim3(kMeasTileX * kMeasTileY), 0, s,
                       f, N, zchunk, tiles_x, tiles_y, L.dx, L.sigma2, c, mc, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_measure_final(partials, nb, result, s);
}

template <typename R>
hipError_t launch_measure_batch(const PoolLattice* lat, const WorkItem* work, int nwork, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_measure_batch<R>), dim3(grid), dim3(kMeasTileX * kMeasTileY), 0, s, lat, work, nwork);
    return hipGetLastError();
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

template hipError_t launch_measure_batch<double>(const PoolLattice*, const WorkItem*, int, int, hipStream_t);
template hipError_t launch_measure_batch<float>(const PoolLattice*, const WorkItem*, int, int, hipStream_t);

template hipError_t launch_measure_tile<double>(const Fields<double>&, const LatticeConst&, const StepCoef&,
                                                const MeasConst&, int, double*, double*, hipStream_t);
template hipError_t launch_measure_tile<float>(const Fields<float>&, const LatticeConst&, const StepCoef&,
                                               const MeasConst&, int, double*, double*, hipStream_t);

}  // namespace ah
