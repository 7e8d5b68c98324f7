// Two leapfrog steps per pass over HBM: a temporally blocked z-march for
// gfx950 (compact gauge action).
//
// The step is a memory-bound stencil (section 5 of the paper): one step
// reads 10 and writes 10 reals per site.  Here a workgroup advances its
// TX x TY tile by two steps while reading the snapshot n once and writing
// snapshot n+2 once, so HBM moves half the bytes of two single steps.
//
// Step n -> n+1 ("stage 1") is computed on the tile plus a one-site ring
// (region R1, (TX+2) x (TY+2)), which needs links and phi of snapshot n on a
// two-site ring (region R2, (TX+4) x (TY+4)).  Step n+1 -> n+2 ("stage 2")
// is computed on the tile from stage 1's values in LDS.  The workgroup walks
// its z-chunk plane by plane with stage 2 one plane behind stage 1:
//   (a) stage 1 at plane p on R1 (tile threads and ring threads);
//   (b) barrier;
//   (c) stage 2 at plane p-1 on the tile, stores of snapshot n+2;
//       links of plane p+2 and phi of plane p+1 for stage 1 into LDS;
//   (d) barrier.
// Stage 1 reads Pi and E of snapshot n on the ring too, which the
// neighbouring workgroups' stage 2 would overwrite in place, so Pi and E are
// double-buffered: the pass reads (phi, A, Pi, E) from one set of buffers
// and writes all ten to the other.
//
// Each site of either stage is computed by site_update, the same sequence of
// roundings as the single-step march, so two steps here are bitwise equal
// to two single steps.
#include "ah_internal.h"
#include "ah_stencil.h"

#pragma clang fp contract(off)

namespace ah {
namespace {

template <int TX, int TY>
struct Geom2 {
    static constexpr int W1 = TX + 2, H1 = TY + 2, S1 = W1 * H1;  // R1: tile + 1-site ring
    static constexpr int W2 = TX + 4, H2 = TY + 4, S2 = W2 * H2;  // R2: tile + 2-site ring
    static constexpr int NT = TX * TY;                            // tile threads
    static constexpr int NRING = S1 - NT;                         // R1 ring sites
    static constexpr int NTH = NT + (NRING + 63) / 64 * 64;       // threads (ring in whole waves)
    static constexpr int NOUT = S2 - S1;                          // R2 outer ring sites
    static_assert(NOUT <= NTH, "one outer-ring site per thread at most");
};

// LDS of one workgroup.  Stage-1 links and phi live on R2, stage-2 ones on
// R1.  x and y links are kept for two planes (p and p+1: the plaquettes at
// x-kx and x-ky reach one plane up), z links and phi for one.
template <typename R, int TX, int TY>
struct Shared2 {
    using G = Geom2<TX, TY>;
    Cx<R> u0x[2][G::S2], u0y[2][G::S2], u0z[G::S2], p0[G::S2];
    Cx<R> u1x[2][G::S1], u1y[2][G::S1], u1z[G::S1], p1[G::S1];
    // stage-1 results at the tile sites that stage 2 takes one plane later
    // (Pi, E of snapshot n+1/2 and A of snapshot n+1), by plane parity
    R h1[2][8][G::NT];
};

template <typename R>
struct Step2Args {
    Fields<R> in;   // snapshot n
    Fields<R> out;  // snapshot n+2
    int N, P;  // side, row pitch: site (x, y, z) at x + P (y + N z)
    SiteCoef<R> k0, k1;  // coefficients of steps n and n+1
    R dx;
};

// Neighbourhood of the site at index c of a region of width W whose links
// (x, y, z of plane z; x, y of plane z+1) and phi (plane z) are in LDS.
template <typename R, int W>
__device__ __forceinline__ SiteNbr<R> gather_nbr(int c, const Cx<R>* ux, const Cx<R>* uy, const Cx<R>* uz,
                                                 const Cx<R>* ph, const Cx<R>* uxp, const Cx<R>* uyp)
{
    SiteNbr<R> n;
    n.ph_xm = ph[c - 1];
    n.ph_xp = ph[c + 1];
    n.ph_ym = ph[c - W];
    n.ph_yp = ph[c + W];
    n.ux_xm = ux[c - 1];
    n.uy_ym = uy[c - W];
    n.uy_xp = uy[c + 1];
    n.ux_yp = ux[c + W];
    n.uz_xp = uz[c + 1];
    n.uz_yp = uz[c + W];
    n.ux_xm_yp = ux[c - 1 + W];
    n.uy_xm = uy[c - 1];
    n.uz_xm = uz[c - 1];
    n.ux_ym = ux[c - W];
    n.uy_xp_ym = uy[c + 1 - W];
    n.uz_ym = uz[c - W];
    n.ux_xm_zp = uxp[c - 1];
    n.uy_ym_zp = uyp[c - W];
    return n;
}

template <int TX, int TY>
constexpr int kStep2Threads = Geom2<TX, TY>::NTH;
// Waves per SIMD the register allocation leaves room for: FP64 two (its
// stage state needs up to 256 registers); FP32 three (168 registers: one
// 11-wave 64 x 8 or two 7-wave 64 x 4 workgroups per CU), four for the
// 6-wave 32 x 8 workgroup (128 registers; the pool's instance then spills
// a few bytes and still runs faster).
template <typename R, int TX, int TY>
constexpr int kStep2MinWaves = sizeof(R) == 8 ? 2 : (Geom2<TX, TY>::NTH <= 384 ? 4 : 3);

// Two steps of planes [z0, z1) of the tile whose lower corner is (x0, y0).
// All threads of the workgroup call this with the same arguments.
template <typename R, int TX, int TY>
__device__ __forceinline__ void march2(Shared2<R, TX, TY>& sh, const Step2Args<R>& a, int x0, int y0, int z0, int z1)
{
    using G = Geom2<TX, TY>;
    constexpr int W1 = G::W1, H1 = G::H1, W2 = G::W2, H2 = G::H2, NT = G::NT;

    const int N = a.N, P = a.P;
    const int64_t NN = (int64_t)N * P;  // plane stride
    const R dx = a.dx;
    const Fields<R>& f = a.in;
    // 1/dx and 1/dx^2 formed on the device as the single-step march forms them
    SiteCoef<R> k0 = a.k0, k1 = a.k1;
    k0.inv_dx = k1.inv_dx = R(1) / dx;
    k0.inv_dx2 = k1.inv_dx2 = k0.inv_dx * k0.inv_dx;

    // ---- roles: R1 position (stage 1) of every thread that has one; tile
    //      threads also own a stage-2 site; threads < NOUT one R2 outer site
    const int tid = threadIdx.x;
    const bool is_tile = tid < NT;
    int rx = 0, ry = 0;
    bool has1 = true;
    if (is_tile) {
        rx = tid % TX + 1;
        ry = tid / TX + 1;
    } else {
        const int r = tid - NT;
        if (r < W1) {
            rx = r;
            ry = 0;
        } else if (r < 2 * W1) {
            rx = r - W1;
            ry = H1 - 1;
        } else if (r < 2 * W1 + TY) {
            rx = 0;
            ry = 1 + (r - 2 * W1);
        } else if (r < G::NRING) {
            rx = W1 - 1;
            ry = 1 + (r - 2 * W1 - TY);
        } else {
            has1 = false;  // padding lane of the last ring wave
        }
    }
    const bool has_out = tid < G::NOUT;
    int ox = 0, oy = 0;
    if (has_out) {
        if (tid < W2) {
            ox = tid;
            oy = 0;
        } else if (tid < 2 * W2) {
            ox = tid - W2;
            oy = H2 - 1;
        } else if (tid < 2 * W2 + (H2 - 2)) {
            ox = 0;
            oy = 1 + (tid - 2 * W2);
        } else {
            ox = W2 - 1;
            oy = 1 + (tid - 2 * W2 - (H2 - 2));
        }
    }
    const int c1 = rx + W1 * ry;              // R1 index of the stage-1 site
    const int c2 = (rx + 1) + W2 * (ry + 1);  // its R2 index
    const int co = ox + W2 * oy;              // R2 index of the outer site
    const int64_t xy1 = has1 ? (int64_t)wrapi(x0 - 1 + rx, N) + (int64_t)P * wrapi(y0 - 1 + ry, N) : 0;
    const int64_t xyo = (int64_t)wrapi(x0 - 2 + ox, N) + (int64_t)P * wrapi(y0 - 2 + oy, N);
    const int gx = x0 + rx - 1, gy = y0 + ry - 1;
    const bool active = is_tile && gx < N && gy < N;
    const int64_t own_xy = xy1;

    auto plane_of = [&](int z) -> int64_t { return (int64_t)wrapi(z, N) * NN; };
    const R* A[3] = {f.a0, f.a1, f.a2};

    // ---- stage-1 column state (snapshot n at the stage-1 site).  The
    //      site's own links of planes p and p+1 are read back from LDS.
    R ac[3], ap[3];          // A at planes p, p+1
    Cx<R> upz;               // U_z at plane p+1 (into LDS once plane p is done)
    Cx<R> uz_m;              // U_z at plane p-1
    R fxz_m = 0, fyz_m = 0;  // F_xz, F_yz at plane p-1
    Cx<R> phm, phc, php;     // phi at planes p-1, p, p+1
    R pr, pi, e[3];          // Pi, E at plane p
    Cx<R> uo_z;              // outer site: U_z of the plane above the one in u0z
    // ---- stage-2 column state (snapshot n+1 at the tile site); the site's
    //      Pi, E and A come from stage 1 through LDS
    Cx<R> vz_m = {};         // U_z^{n+1} at q-1
    R gxz_m = 0, gyz_m = 0;  // F^{n+1}_xz, F^{n+1}_yz at q-1
    Cx<R> chm = {};          // phi^{n+1} at q-1
    // stage-1 phi and U_z of plane p, into LDS when stage 2 has finished with
    // plane p-1 (its x, y links go there at once)
    Cx<R> s1phi = {}, s1z = {};

    // ------------------------------------------------------------ prologue
    // plane zm = z0-2: U_z on R2 into u0z (for F^n at z0-2), own x, y links
    {
        const int64_t pm2 = plane_of(z0 - 2), pm1 = plane_of(z0 - 1), p0 = plane_of(z0);
        Cx<R> um2[3];
        if (has1) {
            for (int d = 0; d < 3; ++d) um2[d] = link(dx, A[d][pm2 + own_xy]);
            sh.u0z[c2] = um2[2];
            uz_m = um2[2];
        }
        if (has_out) sh.u0z[co] = link(dx, A[2][pm2 + xyo]);
        // plane z0-1 links: x, y into their slot, z held
        const int s_m1 = (z0 - 1) & 1, s_0 = z0 & 1;
        Cx<R> uc[3];
        if (has1) {
            for (int d = 0; d < 3; ++d) {
                ac[d] = A[d][pm1 + own_xy];
                uc[d] = link(dx, ac[d]);
            }
            sh.u0x[s_m1][c2] = uc[0];
            sh.u0y[s_m1][c2] = uc[1];
            phm = Cx<R>{f.phr[pm2 + own_xy], f.phi[pm2 + own_xy]};
            phc = Cx<R>{f.phr[pm1 + own_xy], f.phi[pm1 + own_xy]};
            php = Cx<R>{f.phr[p0 + own_xy], f.phi[p0 + own_xy]};
            sh.p0[c2] = phc;
        }
        Cx<R> uo_m1z = {};
        if (has_out) {
            sh.u0x[s_m1][co] = link(dx, A[0][pm1 + xyo]);
            sh.u0y[s_m1][co] = link(dx, A[1][pm1 + xyo]);
            uo_m1z = link(dx, A[2][pm1 + xyo]);
            sh.p0[co] = Cx<R>{f.phr[pm1 + xyo], f.phi[pm1 + xyo]};
        }
        __syncthreads();
        // F^n_xz, F^n_yz at z0-2 of the stage-1 site
        if (has1) {
            fxz_m = plaq_sin(um2[0], sh.u0z[c2 + 1], uc[0], um2[2]) * k0.inv_dx2;
            fyz_m = plaq_sin(um2[1], sh.u0z[c2 + W2], uc[1], um2[2]) * k0.inv_dx2;
        }
        __syncthreads();
        // U_z of z0-1 into u0z; plane z0 links: x, y into their slot, z held
        if (has1) {
            sh.u0z[c2] = uc[2];
            for (int d = 0; d < 3; ++d) ap[d] = A[d][p0 + own_xy];
            sh.u0x[s_0][c2] = link(dx, ap[0]);
            sh.u0y[s_0][c2] = link(dx, ap[1]);
            upz = link(dx, ap[2]);
            pr = f.pir[pm1 + own_xy];
            pi = f.pii[pm1 + own_xy];
            e[0] = f.e0[pm1 + own_xy];
            e[1] = f.e1[pm1 + own_xy];
            e[2] = f.e2[pm1 + own_xy];
        }
        if (has_out) {
            sh.u0z[co] = uo_m1z;
            sh.u0x[s_0][co] = link(dx, A[0][p0 + xyo]);
            sh.u0y[s_0][co] = link(dx, A[1][p0 + xyo]);
            uo_z = link(dx, A[2][p0 + xyo]);
        }
        __syncthreads();
    }

    // Operands loaded one iteration ahead: A of plane p+2 (stage-1 site and
    // outer site), phi of plane p+2 (stage-1 site) and p+1 (outer site), Pi
    // and E of plane p+1 (stage-1 site).
    R na[3] = {0, 0, 0}, noa[3] = {0, 0, 0}, npr = 0, npi = 0, ne[3] = {0, 0, 0};
    Cx<R> nph = {}, noph = {};

    for (int p = z0 - 1; p <= z1; ++p) {
        const bool more = p < z1;
        if (more) {
            const int64_t p2 = plane_of(p + 2), p1 = plane_of(p + 1);
            if (has1) {
                for (int d = 0; d < 3; ++d) na[d] = A[d][p2 + own_xy];
                nph = Cx<R>{f.phr[p2 + own_xy], f.phi[p2 + own_xy]};
                npr = f.pir[p1 + own_xy];
                npi = f.pii[p1 + own_xy];
                ne[0] = f.e0[p1 + own_xy];
                ne[1] = f.e1[p1 + own_xy];
                ne[2] = f.e2[p1 + own_xy];
            }
            if (has_out) {
                for (int d = 0; d < 3; ++d) noa[d] = A[d][p2 + xyo];
                noph = Cx<R>{f.phr[p1 + xyo], f.phi[p1 + xyo]};
            }
        }
        const int sp = p & 1, sq = sp ^ 1;  // LDS slots of planes p (and p+2) and p+1 (and p-1)

        // ---- (a) stage 1 at plane p; the previous plane's phi and U_z of
        //      snapshot n+1 go into LDS first (stage 2 reads them this time)
        if (has1) {
            if (p > z0 - 1) {
                if (is_tile) chm = sh.p1[c1];  // phi^{n+1} of plane p-2, before it is replaced
                sh.p1[c1] = s1phi;
                sh.u1z[c1] = s1z;
            }
            const Cx<R> uc[3] = {sh.u0x[sp][c2], sh.u0y[sp][c2], sh.u0z[c2]};
            const SiteNbr<R> nb = gather_nbr<R, W2>(c2, sh.u0x[sp], sh.u0y[sp], sh.u0z, sh.p0, sh.u0x[sq], sh.u0y[sq]);
            const SiteOut<R> o = site_update(k0, nb, phm, phc, php, uc, sh.u0x[sq][c2], sh.u0y[sq][c2], uz_m, fxz_m,
                                             fyz_m, pr, pi, e, ac);
            fxz_m = o.fxz;
            fyz_m = o.fyz;
            if (is_tile) {
                R* h = &sh.h1[sp][0][tid];
                h[0 * NT] = o.pr;
                h[1 * NT] = o.pi;
                for (int d = 0; d < 3; ++d) {
                    h[(2 + d) * NT] = o.e[d];
                    h[(5 + d) * NT] = o.a[d];
                }
            }
            s1phi = o.phi;
            sh.u1x[sp][c1] = link(dx, o.a[0]);
            sh.u1y[sp][c1] = link(dx, o.a[1]);
            s1z = link(dx, o.a[2]);
        }
        __syncthreads();

        // ---- (c) stage 2 at plane q = p-1 on the tile
        if (is_tile && p >= z0) {
            const int q = p - 1;
            const int c = c1;
            const Cx<R> vc[3] = {sh.u1x[sq][c], sh.u1y[sq][c], sh.u1z[c]};
            if (p == z0) {
                // plane z0-1 is not stepped here: its F^{n+1}_xz, F^{n+1}_yz
                // start the stage-2 carry
                gxz_m = plaq_sin(vc[0], sh.u1z[c + 1], sh.u1x[sp][c], vc[2]) * k1.inv_dx2;
                gyz_m = plaq_sin(vc[1], sh.u1z[c + W1], sh.u1y[sp][c], vc[2]) * k1.inv_dx2;
            } else {
                const R* h = &sh.h1[sq][0][tid];
                const R qe[3] = {h[2 * NT], h[3 * NT], h[4 * NT]};
                const R bc[3] = {h[5 * NT], h[6 * NT], h[7 * NT]};
                const SiteNbr<R> nb = gather_nbr<R, W1>(c, sh.u1x[sq], sh.u1y[sq], sh.u1z, sh.p1, sh.u1x[sp], sh.u1y[sp]);
                const SiteOut<R> o = site_update(k1, nb, chm, sh.p1[c], s1phi, vc, sh.u1x[sp][c], sh.u1y[sp][c], vz_m,
                                                 gxz_m, gyz_m, h[0], h[NT], qe, bc);
                gxz_m = o.fxz;
                gyz_m = o.fyz;
                if (active) {
                    const int64_t oq = (int64_t)q * NN + own_xy;
                    const Fields<R>& w = a.out;
                    st_stream(w.pir + oq, o.pr);
                    st_stream(w.pii + oq, o.pi);
                    st_stream(w.e0 + oq, o.e[0]);
                    st_stream(w.e1 + oq, o.e[1]);
                    st_stream(w.e2 + oq, o.e[2]);
                    st_stream(w.phr + oq, o.phi.r);
                    st_stream(w.phi + oq, o.phi.i);
                    st_stream(w.a0 + oq, o.a[0]);
                    st_stream(w.a1 + oq, o.a[1]);
                    st_stream(w.a2 + oq, o.a[2]);
                }
            }
            vz_m = vc[2];
        }
        if (!more) break;

        // ---- stage-1 operands of plane p+1: U_z of p+1 and phi of p+1 into
        //      LDS, links of plane p+2 (x, y into slot sp, z held)
        if (has1) {
            uz_m = sh.u0z[c2];
            sh.u0z[c2] = upz;
            sh.p0[c2] = php;
            for (int d = 0; d < 3; ++d) {
                ac[d] = ap[d];
                ap[d] = na[d];
            }
            sh.u0x[sp][c2] = link(dx, na[0]);
            sh.u0y[sp][c2] = link(dx, na[1]);
            upz = link(dx, na[2]);
            phm = phc;
            phc = php;
            php = nph;
            pr = npr;
            pi = npi;
            for (int d = 0; d < 3; ++d) e[d] = ne[d];
        }
        if (has_out) {
            sh.u0z[co] = uo_z;
            sh.p0[co] = noph;
            sh.u0x[sp][co] = link(dx, noa[0]);
            sh.u0y[sp][co] = link(dx, noa[1]);
            uo_z = link(dx, noa[2]);
        }
        __syncthreads();
    }
}

// One lattice: tile t = xcd_tile(b) (tx fastest, then ty, then z-chunk).
template <typename R, int TX, int TY>
__global__ void __launch_bounds__((kStep2Threads<TX, TY>), (kStep2MinWaves<R, TX, TY>))
    k_step2_tile(Step2Args<R> a, int zchunk, int tiles_x, int tiles_y)
{
    __shared__ Shared2<R, TX, TY> sh;
    int t = xcd_tile(blockIdx.x, gridDim.x);
    const int x0 = (t % tiles_x) * TX;
    t /= tiles_x;
    const int y0 = (t % tiles_y) * TY;
    const int z0 = (t / tiles_y) * zchunk;
    const int z1 = (z0 + zchunk < a.N) ? z0 + zchunk : a.N;
    march2<R, TX, TY>(sh, a, x0, y0, z0, z1);
}

// Pool lattices that take a two-step pass at their step k (two_step_due):
// one block per (lattice, tile) work item, XCD x the x-th eighth of the list
// as in the single-step batch kernel; snapshot k of the current buffers to
// snapshot k+2 in the other ones, with the coefficients of rows k and k+1 of
// the lattice's table.
template <typename R, int TX, int TY>
__global__ void __launch_bounds__((kStep2Threads<TX, TY>), (kStep2MinWaves<R, TX, TY>))
    k_step2_batch(const PoolLattice* __restrict__ lat, const WorkItem* __restrict__ work, int nwork)
{
    __shared__ Shared2<R, TX, TY> sh;
    const WorkItem it = work[xcd_tile(blockIdx.x, nwork)];
    if (it.lattice < 0) return;
    const PoolLattice& L = lat[it.lattice];
    const int64_t k = L.counter[0];
    if (!two_step_due(L, k)) return;  // uniform across the block
    const int cur = (int)L.counter[2], curm = (int)L.counter[3];
    Step2Args<R> a;
    a.in = Fields<R>{(R*)L.pp[cur][0], (R*)L.pp[cur][1], (R*)L.mom[curm][0], (R*)L.mom[curm][1], (R*)L.pp[cur][2],
                     (R*)L.pp[cur][3], (R*)L.pp[cur][4], (R*)L.mom[curm][2], (R*)L.mom[curm][3], (R*)L.mom[curm][4]};
    const int o = cur ^ 1, om = curm ^ 1;
    a.out = Fields<R>{(R*)L.pp[o][0], (R*)L.pp[o][1], (R*)L.mom[om][0], (R*)L.mom[om][1], (R*)L.pp[o][2],
                      (R*)L.pp[o][3], (R*)L.pp[o][4], (R*)L.mom[om][2], (R*)L.mom[om][3], (R*)L.mom[om][4]};
    a.N = L.N;
    a.P = L.P;
    a.dx = (R)L.dx;
    const double* row = L.coef + k * kCoefStride;
    for (int j = 0; j < 2; ++j, row += kCoefStride) {
        SiteCoef<R>& c = j ? a.k1 : a.k0;
        c.inv_dx = c.inv_dx2 = R(0);  // formed in the march
        c.sigma2 = (R)L.sigma2;
        c.cP1 = (R)row[C_P1];
        c.cP2 = (R)row[C_P2];
        c.cE1 = (R)row[C_E1];
        c.cE2 = (R)row[C_E2];
        c.lamh = (R)row[C_LAMH];
        c.kappa = (R)row[C_KAPPA];
        c.deta = (R)L.deta;
    }
    a = uniform(a);
    int t = it.tile;
    const int x0 = uniform((t % L.two_tiles_x) * TX);
    t /= L.two_tiles_x;
    const int y0 = uniform((t % L.two_tiles_y) * TY);
    const int z0 = uniform((t / L.two_tiles_y) * L.two_zchunk);
    const int z1 = uniform((z0 + L.two_zchunk < L.N) ? z0 + L.two_zchunk : L.N);
    march2<R, TX, TY>(sh, a, x0, y0, z0, z1);
}

}  // namespace

template <typename R>
hipError_t launch_step2_tile(const Fields<R>& in, const Fields<R>& out, const LatticeConst& L, const StepCoef& c0,
                             const StepCoef& c1, const TileConfig& tc, hipStream_t s)
{
    const int N = L.N;
    Step2Args<R> a;
    a.in = in;
    a.out = out;
    a.N = N;
    a.P = L.P;
    a.dx = (R)L.dx;
    for (int j = 0; j < 2; ++j) {
        const StepCoef& c = j ? c1 : c0;
        SiteCoef<R>& k = j ? a.k1 : a.k0;
        k.inv_dx = k.inv_dx2 = R(0);  // formed in the kernel
        k.sigma2 = (R)L.sigma2;
        k.cP1 = (R)c.cP1;
        k.cP2 = (R)c.cP2;
        k.cE1 = (R)c.cE1;
        k.cE2 = (R)c.cE2;
        k.lamh = (R)c.lam_half;
        k.kappa = (R)c.kappa;
        k.deta = (R)L.deta;
    }
    const int zc = tc.zchunk > 0 ? tc.zchunk : N;
#define AH_STEP2_CASE(TXv, TYv)                                                                                   \
    if (tc.tx == TXv && tc.ty == TYv) {                                                                           \
        const int tiles_x = (N + TXv - 1) / TXv, tiles_y = (N + TYv - 1) / TYv;                                  \
        const int nb = tiles_x * tiles_y * ((N + zc - 1) / zc);                                                  \
        hipLaunchKernelGGL((k_step2_tile<R, TXv, TYv>), dim3(nb), dim3(Geom2<TXv, TYv>::NTH), 0, s, a, zc,       \
                           tiles_x, tiles_y);                                                                     \
        return hipGetLastError();                                                                                \
    }
    AH_STEP2_CASE(32, 8)
    AH_STEP2_CASE(64, 4)
    if constexpr (sizeof(R) == 4) {
        AH_STEP2_CASE(64, 8)  // FP64 would need more LDS than a CU has
    }
#undef AH_STEP2_CASE
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_step2_batch(const PoolLattice* lat, const WorkItem* work, int nwork, int tx, int ty, int grid,
                              hipStream_t s)
{
    if (!tile2_supported(sizeof(R) == 8 ? AH_FP64 : AH_FP32, tx, ty)) return hipErrorInvalidValue;
#define AH_STEP2_BATCH_CASE(TXv, TYv)                                                                             \
    if (tx == TXv && ty == TYv) {                                                                                 \
        hipLaunchKernelGGL((k_step2_batch<R, TXv, TYv>), dim3(grid), dim3(Geom2<TXv, TYv>::NTH), 0, s, lat, work, \
                           nwork);                                                                                \
        return hipGetLastError();                                                                                 \
    }
    AH_STEP2_BATCH_CASE(32, 8)
    AH_STEP2_BATCH_CASE(64, 4)
    if constexpr (sizeof(R) == 4) {
        AH_STEP2_BATCH_CASE(64, 8)
    }
#undef AH_STEP2_BATCH_CASE
    return hipErrorInvalidValue;
}
template hipError_t launch_step2_batch<double>(const PoolLattice*, const WorkItem*, int, int, int, int, hipStream_t);
template hipError_t launch_step2_batch<float>(const PoolLattice*, const WorkItem*, int, int, int, int, hipStream_t);

template hipError_t launch_step2_tile<double>(const Fields<double>&, const Fields<double>&, const LatticeConst&,
                                              const StepCoef&, const StepCoef&, const TileConfig&, hipStream_t);
template hipError_t launch_step2_tile<float>(const Fields<float>&, const Fields<float>&, const LatticeConst&,
                                             const StepCoef&, const StepCoef&, const TileConfig&, hipStream_t);

}  // namespace ah
