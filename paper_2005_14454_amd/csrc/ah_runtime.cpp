// Host runtime of libah: parameter validation, device arena layout, the FP64
// per-step coefficient formulas, phi/A ping-pong, state I/O, diagnostics
// assembly and the C ABI declared in include/ah.h.
#include "ah.h"
#include "ah_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace ah;

struct ah_handle {
    ah_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool owns_arena = false;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    int64_t V = 0;  // sites, N^3
    int P = 0;      // row pitch of the stored fields (site (x, y, z) at x + P (y + N z))
    size_t real_bytes = 8;
    // ping-pong phi/A buffers [2][5] (phr, phi, a0, a1, a2) and Pi/E buffers
    // [2][5] (pir, pii, e0, e1, e2).  A single step drifts phi and A into the
    // other buffer and kicks Pi and E in place; a two-step pass writes all
    // ten fields into the other buffers.
    void* pp[2][5] = {};
    void* mom[2][5] = {};
    int curm = 0;  // current Pi/E buffer
    double* partials = nullptr;
    double* result = nullptr;
    double* series = nullptr;       // kSeriesCap folded records (ah_step_measured)
    double* host_result = nullptr;  // pinned
    double* host_series = nullptr;  // pinned, kSeriesCap records
    int cur = 0;
    int64_t step = 0;
    bool ready = false;
    bool timing = false;
    std::vector<hipEvent_t> ev;  // start/stop pairs
    size_t ev_used = 0;
    ah_step_config cfg{AH_KERNEL_AUTO, 0, 0, 0};
    int64_t measured_launches = 0;  // timed launches that also formed diagnostics
    std::vector<char> ev_measured;  // per event pair: 1 if that launch formed diagnostics
    std::vector<char> ev_steps;     // per event pair: steps the launch advanced (1 or 2)
    std::string err;
};

namespace ah {
bool tuned_config(const ah_params& p, ah_step_config* out);  // ah_tune.cpp
}

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int fail(ah_handle* h, int code, const std::string& msg)
{
    if (h) h->err = msg;
    return code;
}

int hip_fail(ah_handle* h, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(h, AH_E_DEVICE, m);
}

double eta_ref_of(const ah_params& p) { return p.eta_ref > 0.0 ? p.eta_ref : 0.5 * p.dx * (double)p.N; }

// Section 2 scalars at snapshot n.
struct Scalars {
    double eta, s, a, f, delta, omega;
};
Scalars scalars_at(const ah_params& p, int64_t n)
{
    Scalars r;
    r.eta = p.eta0 + (double)n * p.deta;
    r.s = r.eta < p.eta_switch ? p.s_early : p.s_late;
    r.a = std::pow(r.eta / eta_ref_of(p), p.m);
    r.f = std::pow(r.a, 2.0 * r.s);
    r.delta = 0.5 * p.alpha * p.m * p.deta / r.eta;
    // artificial damping phase: a constant friction gamma replaces the Hubble term
    if (p.damp_gamma > 0.0 && r.eta < p.eta_damp) r.delta = 0.5 * p.damp_gamma * p.deta;
    r.omega = (1.0 - r.s) * r.delta;
    return r;
}

StepCoef coef_at(const ah_params& p, int64_t n)
{
    const Scalars s = scalars_at(p, n);
    StepCoef c;
    c.cP1 = (1.0 - s.delta) / (1.0 + s.delta);
    c.cP2 = p.deta / (1.0 + s.delta);
    c.cE1 = (1.0 - s.omega) / (1.0 + s.omega);
    c.cE2 = p.deta / (1.0 + s.omega);
    c.lam_half = 0.5 * p.lambda0 * s.f;
    c.kappa = 2.0 * p.e0 * p.e0 * s.f;
    return c;
}

// Coupling c_{n-1/2} of the Gauss residual: the kick keeps
// div E^{n-1/2} = c_{n-1/2} Im[conj(phi^n) Pi^{n-1/2}] exactly when
// c_{n-1/2} = 2 e0^2 f_{n-1} (1+delta_{n-1}) / (1+omega_{n-1}); 2 e0^2 f_0 at n = 0.
double gauss_coupling(const ah_params& p, int64_t n)
{
    if (n <= 0) return 2.0 * p.e0 * p.e0 * scalars_at(p, 0).f;
    const Scalars s = scalars_at(p, n - 1);
    return 2.0 * p.e0 * p.e0 * s.f * (1.0 + s.delta) / (1.0 + s.omega);
}

double stability_margin(const ah_params& p, int64_t n)
{
    const Scalars s = scalars_at(p, n);
    const double g = std::fmax(p.lambda0, 2.0 * p.e0 * p.e0) * s.f * p.sigma * p.sigma + 12.0 / (p.dx * p.dx);
    return p.deta * std::sqrt(g);
}

bool unstable_at(const ah_params& p, int64_t n) { return stability_margin(p, n) >= 2.0; }

}  // namespace

namespace ah {

int validate_params(const ah_params* p, std::string* why)
{
    if (!p) {
        *why = "params is NULL";
        return AH_E_INVAL;
    }
    if (p->N < 4 || p->N > 4096) {
        *why = "N must be in [4, 4096]";
        return AH_E_INVAL;
    }
    if (p->precision != AH_FP64 && p->precision != AH_FP32) {
        *why = "precision must be AH_FP64 or AH_FP32";
        return AH_E_INVAL;
    }
    if (p->gauge_action != AH_COMPACT && p->gauge_action != AH_NONCOMPACT) {
        *why = "gauge_action must be AH_COMPACT or AH_NONCOMPACT";
        return AH_E_INVAL;
    }
    if (p->reserved != 0) {
        *why = "reserved must be 0";
        return AH_E_INVAL;
    }
    if (!(p->dx > 0.0) || !(p->deta > 0.0) || !std::isfinite(p->dx) || !std::isfinite(p->deta)) {
        *why = "dx and deta must be positive and finite";
        return AH_E_INVAL;
    }
    if (!(p->eta0 > 0.0) || !std::isfinite(p->eta0)) {
        *why = "eta0 must be positive";
        return AH_E_INVAL;
    }
    if (!(p->e0 > 0.0) || !std::isfinite(p->lambda0) || !std::isfinite(p->sigma) || !std::isfinite(p->m) ||
        !std::isfinite(p->alpha) || !std::isfinite(p->s_early) || !std::isfinite(p->s_late) ||
        std::isnan(p->eta_switch) || !std::isfinite(p->eta_ref)) {
        *why = "non-finite or invalid coupling / expansion parameter (e0 must be > 0)";
        return AH_E_INVAL;
    }
    if (!(p->damp_gamma >= 0.0) || !std::isfinite(p->damp_gamma) || std::isnan(p->eta_damp)) {
        *why = "damp_gamma must be finite and >= 0, eta_damp not NaN";
        return AH_E_INVAL;
    }
    return AH_OK;
}

}  // namespace ah

namespace {

int validate(const ah_params* p, std::string* why) { return validate_params(p, why); }

size_t field_bytes(const ah_params& p)
{
    const size_t stored = (size_t)p.N * p.N * row_pitch(p.N, p.precision);
    return align_up(stored * (p.precision == AH_FP64 ? 8 : 4));
}


// Diagnostics records a handle can hold: the largest number of workgroups
// of any supported tile shape at the smallest z-chunk.
size_t partial_records(const ah_params& p)
{
    const int N = p.N;
    const int zc = min_zchunk(N);
    const int64_t tz = (N + zc - 1) / zc;
    int64_t best = 0;
    const int shapes[6][2] = {{64, 8}, {64, 4}, {32, 8}, {64, 16}, {128, 4}, {128, 8}};
    for (auto& s : shapes) {
        const int64_t t = (int64_t)((N + s[0] - 1) / s[0]) * ((N + s[1] - 1) / s[1]) * tz;
        if (t > best) best = t;
    }
    return (size_t)(best > kMeasBlocks ? best : kMeasBlocks);
}

constexpr int kSeriesCap = 1024;  // device measurement records per ah_step_measured batch

size_t required_bytes(const ah_params& p)
{
    return 20 * field_bytes(p) + align_up(partial_records(p) * kMeasStride * sizeof(double)) +
           align_up(kMeasStride * sizeof(double)) + align_up((size_t)kSeriesCap * kMeasStride * sizeof(double));
}

template <typename R>
Fields<R> fields_of(const ah_handle* h, int buf)
{
    Fields<R> f;
    f.phr = (R*)h->pp[buf][0];
    f.phi = (R*)h->pp[buf][1];
    f.a0 = (R*)h->pp[buf][2];
    f.a1 = (R*)h->pp[buf][3];
    f.a2 = (R*)h->pp[buf][4];
    f.pir = (R*)h->mom[h->curm][0];
    f.pii = (R*)h->mom[h->curm][1];
    f.e0 = (R*)h->mom[h->curm][2];
    f.e1 = (R*)h->mom[h->curm][3];
    f.e2 = (R*)h->mom[h->curm][4];
    return f;
}

LatticeConst lconst(const ah_params& p)
{
    LatticeConst L;
    L.N = p.N;
    L.P = row_pitch(p.N, p.precision);
    L.compact = p.gauge_action == AH_COMPACT ? 1 : 0;
    L.dx = p.dx;
    L.deta = p.deta;
    L.sigma2 = p.sigma * p.sigma;
    return L;
}

}  // namespace

namespace ah {

hipError_t field_upload(void* dev, const void* host, int N, int P, size_t rb, hipStream_t s)
{
    if (P == N) return hipMemcpyAsync(dev, host, (size_t)N * N * N * rb, hipMemcpyHostToDevice, s);
    return hipMemcpy2DAsync(dev, (size_t)P * rb, host, (size_t)N * rb, (size_t)N * rb, (size_t)N * N,
                            hipMemcpyHostToDevice, s);
}
hipError_t field_download(void* host, const void* dev, int N, int P, size_t rb, hipStream_t s)
{
    if (P == N) return hipMemcpyAsync(host, dev, (size_t)N * N * N * rb, hipMemcpyDeviceToHost, s);
    return hipMemcpy2DAsync(host, (size_t)N * rb, dev, (size_t)P * rb, (size_t)N * rb, (size_t)N * N,
                            hipMemcpyDeviceToHost, s);
}

}  // namespace ah

namespace {

// component c of the state (order phi_re, phi_im, pi_re, pi_im, A0..2, E0..2)
void* comp_ptr(ah_handle* h, int c)
{
    switch (c) {
    case 0: return h->pp[h->cur][0];
    case 1: return h->pp[h->cur][1];
    case 2: return h->mom[h->curm][0];
    case 3: return h->mom[h->curm][1];
    case 4: return h->pp[h->cur][2];
    case 5: return h->pp[h->cur][3];
    case 6: return h->pp[h->cur][4];
    default: return h->mom[h->curm][c - 5];
    }
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int now = -1;
        if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
    }
};


}  // namespace

namespace ah {

// Step rates of the one-step tile shapes on a lattice they tile exactly
// (MI355X, 512^3, best z-chunk; 1e9 site-updates/s; 0: no such instance).
namespace {
struct ShapeRate {
    int tx, ty;
    double fp32, fp64;
};
constexpr ShapeRate kShapeRates[] = {
    {128, 4, 65.9, 0.0}, {128, 8, 64.7, 0.0}, {64, 8, 61.2, 28.3}, {64, 4, 60.8, 27.1}, {32, 8, 59.0, 27.7},
};
}  // namespace

bool default_tile(int precision, int N, int* tx, int* ty)
{
    double best = 0.0;
    for (const ShapeRate& r : kShapeRates) {
        const double rate = precision == AH_FP64 ? r.fp64 : r.fp32;
        if (rate <= 0.0 || !tile_supported(precision, r.tx, r.ty) || !batch_tile_supported(precision, r.tx, r.ty))
            continue;
        // a ragged last tile in x or y runs idle lanes
        const double rx = (double)((N + r.tx - 1) / r.tx * r.tx) / N, ry = (double)((N + r.ty - 1) / r.ty * r.ty) / N;
        const double score = rate / (rx * ry);
        if (score > best) {
            best = score;
            *tx = r.tx;
            *ty = r.ty;
        }
    }
    return best > 0.0;
}

int resident_per_cu(int kernel, int precision, int tx, int ty, bool measured)
{
    if (kernel == AH_KERNEL_TILE2) {
        // waves per SIMD at the pass's registers: FP32 3, FP64 2; the FP64
        // pass's LDS (over 100 KB) admits one workgroup per CU
        if (precision == AH_FP64) return 1;
        const int nt = tx * ty, ring = (tx + 2) * (ty + 2) - nt;
        const int waves = (nt + (ring + 63) / 64 * 64) / 64;
        return std::max(1, 12 / waves);
    }
    // waves per SIMD at the march's registers: plain FP32 4, FP64 2; the
    // measured march 2 in both precisions
    const int waves = (tx * ty + 63) / 64;
    return std::max(1, (precision == AH_FP64 || measured ? 8 : 16) / waves);
}

int auto_zchunk(int kernel, int precision, int N, int tx, int ty, bool measured)
{
    // Workgroups run in rounds of (CUs x resident workgroups); a launch
    // takes about rounds x (planes per chunk + 2), the 2 for a chunk's
    // prologue.  The z-chunks are equal (a short last chunk would leave most
    // of its round idle); among equal estimates the one with more
    // workgroups, which spread more evenly over the XCDs.  Chosen on MI355X
    // over a sweep of N in 65 .. 512 and five tile shapes: within 2% of the
    // best measured z-chunk on average.
    constexpr int kCUs = 256;
    const int64_t per_chunk = (int64_t)((N + tx - 1) / tx) * ((N + ty - 1) / ty);
    const int64_t slots = (int64_t)kCUs * resident_per_cu(kernel, precision, tx, ty, measured);
    const int zmin = std::min(min_zchunk(N), N);
    int best_zc = N;
    int64_t best_t = -1, best_nb = 0;
    for (int nz = 1; nz <= N / zmin; ++nz) {
        const int zc = (N + nz - 1) / nz;
        if (zc < zmin) break;
        const int64_t nb = per_chunk * ((N + zc - 1) / zc);
        const int64_t t = (nb + slots - 1) / slots * (zc + 2);
        if (best_t < 0 || t < best_t || (t == best_t && nb > best_nb)) {
            best_t = t;
            best_nb = nb;
            best_zc = zc;
        }
    }
    return best_zc;
}

// Any tile shape computes the same fields bit for bit, so the measured march
// may run another shape than the plain step: the fastest measured march
// (measured_tile: FP32 64 x 8, FP64 32 x 8), with the step's z-chunk when
// the step runs that shape too, else the automatic z-chunk of the measured
// march but no shorter than the step's (a pool's floor of 16 planes then
// holds for its measured node too).  A lattice of the site kernel takes the
// automatic one.  The diagnostics records are summed in tile order, so a
// lattice measured with the same tiling (alone or in a pool) gets the same
// bits.
TileConfig measured_tiling(const ah_params& p, const ah_step_config& cfg)
{
    int tx = cfg.tile_x, ty = cfg.tile_y;
    const bool tiled = cfg.kernel == AH_KERNEL_TILE || cfg.kernel == AH_KERNEL_TILE2;
    if (!measured_tile(p.precision, &tx, &ty) && tiled) return TileConfig{tx, ty, cfg.zchunk};
    int zc = auto_zchunk(AH_KERNEL_TILE, p.precision, p.N, tx, ty, true);
    if (tiled && cfg.zchunk > zc) zc = std::min(cfg.zchunk, p.N);
    return TileConfig{tx, ty, zc};
}

// Resolve automatic choices of a step configuration for the lattice.
int resolve_step_config(const ah_params& p, const ah_step_config& in, ah_step_config* out, std::string* why)
{
    ah_step_config c = in;
    if (c.kernel == AH_KERNEL_AUTO) c.kernel = p.gauge_action == AH_COMPACT ? AH_KERNEL_TILE : AH_KERNEL_SITE;
    if (c.kernel != AH_KERNEL_SITE && c.kernel != AH_KERNEL_TILE && c.kernel != AH_KERNEL_TILE2) {
        *why = "unknown kernel";
        return AH_E_INVAL;
    }
    if (c.kernel == AH_KERNEL_SITE) {
        c.tile_x = c.tile_y = c.zchunk = 0;
        *out = c;
        return AH_OK;
    }
    if (p.gauge_action != AH_COMPACT) {
        *why = "the tiled kernel supports the compact gauge action only";
        return AH_E_INVAL;
    }
    if (c.tile_x == 0 && c.tile_y == 0) {
        // one step: the shape of the highest rate once its ragged edge is
        // paid for; two-step passes: 32 x 8 in both precisions
        c.tile_x = 32;
        c.tile_y = 8;
        if (c.kernel == AH_KERNEL_TILE) (void)default_tile(p.precision, p.N, &c.tile_x, &c.tile_y);
    }
    if (c.kernel == AH_KERNEL_TILE2 ? !tile2_supported(p.precision, c.tile_x, c.tile_y)
                                    : !tile_supported(p.precision, c.tile_x, c.tile_y)) {
        *why = "unsupported tile shape";
        return AH_E_INVAL;
    }
    if (c.zchunk < 0 || (c.zchunk > 0 && c.zchunk < min_zchunk(p.N))) {
        *why = "zchunk must be 0 (automatic) or at least 2 (N <= 128) or 8 (N > 128)";
        return AH_E_INVAL;
    }
    if (c.zchunk == 0) c.zchunk = auto_zchunk(c.kernel, p.precision, p.N, c.tile_x, c.tile_y, false);
    if (c.zchunk > p.N) c.zchunk = p.N;
    *out = c;
    return AH_OK;
}

// One FP64 row of a lattice's coefficient table for snapshot n (kick
// coefficients and diagnostics constants).
void coef_row(const ah_params& p, int64_t n, double* row)
{
    const Scalars s = scalars_at(p, n);
    const StepCoef c = coef_at(p, n);
    for (int k = 0; k < kCoefStride; ++k) row[k] = 0.0;
    row[C_P1] = c.cP1;
    row[C_P2] = c.cP2;
    row[C_E1] = c.cE1;
    row[C_E2] = c.cE2;
    row[C_LAMH] = c.lam_half;
    row[C_KAPPA] = c.kappa;
    row[C_INV2E2F] = 1.0 / (2.0 * p.e0 * p.e0 * s.f);
    row[C_LAMQ] = 0.25 * p.lambda0 * s.f;
    row[C_GAUSS] = gauss_coupling(p, n);
}

// Diagnostics of snapshot `step` from the folded FP64 sums r[M_COUNT].
void to_measurement(const ah_params& p, int64_t step, const double* r, int64_t V, ah_measurement* out)
{
    const Scalars sc = scalars_at(p, step);
    const double dx3 = p.dx * p.dx * p.dx;
    const double vol = std::pow((double)p.N * p.dx, 3.0);
    std::memset(out, 0, sizeof(*out));
    out->step = step;
    out->eta = sc.eta;
    out->a = sc.a;
    out->f = sc.f;
    out->winding_sum_abs = (int64_t)r[M_WABS];
    out->L_W = p.dx * r[M_WABS];
    out->xi_W = std::sqrt(vol / out->L_W);
    out->e_kin = dx3 * r[M_KIN];
    out->e_grad = dx3 * r[M_GRAD];
    out->e_pot = dx3 * r[M_POT];
    out->e_el = dx3 * r[M_EL];
    out->e_mag = dx3 * r[M_MAG];
    out->energy = out->e_kin + out->e_grad + out->e_pot + out->e_el + out->e_mag;
    out->sum_L = dx3 * ((((r[M_KIN] - r[M_GRAD]) - r[M_POT]) + r[M_EL]) - r[M_MAG]);
    out->xi_L = out->sum_L < 0.0 ? std::sqrt(-2.0 * M_PI * p.sigma * p.sigma * vol / out->sum_L) : NAN;
    out->R = r[M_KINL] / r[M_GRADL];
    out->v2_phi = 2.0 * out->R / (1.0 + out->R);
    out->v2_omega = 0.5 * (1.0 + 3.0 * r[M_PL] / r[M_RHOL]);
    out->gauss_rms = std::sqrt(r[M_G2] / (double)V);
    out->gauss_max = r[M_GMAX];
    const double den = std::sqrt(r[M_DIV2] + r[M_CRHO2]);
    out->gauss_rel = den > 0.0 ? std::sqrt(r[M_G2]) / den : 0.0;
    out->nonfinite = (int64_t)r[M_NONFIN];
    out->flags = (unstable_at(p, step) ? AH_FLAG_UNSTABLE : 0u) | (out->nonfinite ? AH_FLAG_NONFINITE : 0u);
}

}  // namespace ah

namespace {

int resolve_config(const ah_params& p, const ah_step_config& in, ah_step_config* out, std::string* why)
{
    ah_step_config tuned;
    if (in.kernel == AH_KERNEL_AUTO && in.tile_x == 0 && in.tile_y == 0 && in.zchunk == 0 &&
        p.gauge_action == AH_COMPACT && tuned_config(p, &tuned))
        return resolve_step_config(p, tuned, out, why);
    return resolve_step_config(p, in, out, why);
}

MeasConst meas_const(const ah_params& p, int64_t n)
{
    const Scalars sc = scalars_at(p, n);
    MeasConst mc;
    mc.inv_2e2f = 1.0 / (2.0 * p.e0 * p.e0 * sc.f);
    mc.lam_quarter = 0.25 * p.lambda0 * sc.f;
    mc.gauss_c = gauss_coupling(p, n);
    return mc;
}

// Tiling of the measured march (diagnostics of a compact-action handle).
TileConfig meas_tiles(const ah_handle* h)
{
    return measured_tiling(h->p, h->cfg);
}

// Diagnostics of the current snapshot folded into dst[M_COUNT] (device), and
// with `advance` the step of that snapshot in the same pass, which writes Pi
// and E into the other buffer (the Gauss residual reads E of neighbours).
template <typename R>
hipError_t measured_pass(ah_handle* h, double* dst, bool advance)
{
    const ah_params& p = h->p;
    const StepCoef c = coef_at(p, h->step);
    const MeasConst mc = meas_const(p, h->step);
    const TileConfig tc = meas_tiles(h);
    const Fields<R> in = fields_of<R>(h, h->cur);
    Fields<R> out = fields_of<R>(h, h->cur ^ 1);
    const int om = h->curm ^ 1;
    out.pir = (R*)h->mom[om][0];
    out.pii = (R*)h->mom[om][1];
    out.e0 = (R*)h->mom[om][2];
    out.e1 = (R*)h->mom[om][3];
    out.e2 = (R*)h->mom[om][4];
    hipError_t e;
    if (advance && h->timing) {
        if (h->ev_used + 2 > h->ev.size()) {
            for (int k = 0; k < 2; ++k) {
                hipEvent_t ev;
                e = hipEventCreate(&ev);
                if (e != hipSuccess) return e;
                h->ev.push_back(ev);
            }
        }
        e = hipEventRecord(h->ev[h->ev_used], h->stream);
        if (e != hipSuccess) return e;
    }
    const int nb = step_tile_blocks(p.N, tc);
    e = launch_step_tile<R>(in, out, lconst(p), c, tc, &mc, h->partials, advance, h->stream);
    if (e != hipSuccess) return e;
    if (advance && h->timing) {
        e = hipEventRecord(h->ev[h->ev_used + 1], h->stream);
        if (e != hipSuccess) return e;
        h->ev_used += 2;
        h->measured_launches += 1;
        h->ev_measured.push_back(1);
        h->ev_steps.push_back(1);
    }
    e = launch_measure_final(h->partials, nb, dst, h->stream);
    if (e != hipSuccess) return e;
    if (advance) {
        h->cur ^= 1;
        h->curm ^= 1;
        h->step += 1;
    }
    return hipSuccess;
}

// Brackets a step launch with an event pair while timing is on.
struct TimedLaunch {
    ah_handle* h;
    int steps;
    hipError_t begin()
    {
        if (!h->timing) return hipSuccess;
        if (h->ev_used + 2 > h->ev.size()) {
            for (int k = 0; k < 2; ++k) {
                hipEvent_t ev;
                const hipError_t e = hipEventCreate(&ev);
                if (e != hipSuccess) return e;
                h->ev.push_back(ev);
            }
        }
        return hipEventRecord(h->ev[h->ev_used], h->stream);
    }
    hipError_t end()
    {
        if (!h->timing) return hipSuccess;
        const hipError_t e = hipEventRecord(h->ev[h->ev_used + 1], h->stream);
        if (e != hipSuccess) return e;
        h->ev_used += 2;
        h->ev_measured.push_back(0);
        h->ev_steps.push_back((char)steps);
        return hipSuccess;
    }
};

template <typename R>
hipError_t do_step(ah_handle* h)
{
    const Fields<R> in = fields_of<R>(h, h->cur);
    const Fields<R> out = fields_of<R>(h, h->cur ^ 1);
    const StepCoef c = coef_at(h->p, h->step);
    TimedLaunch t{h, 1};
    hipError_t e = t.begin();
    if (e != hipSuccess) return e;
    if (h->cfg.kernel == AH_KERNEL_TILE || h->cfg.kernel == AH_KERNEL_TILE2) {
        TileConfig tc{h->cfg.tile_x, h->cfg.tile_y, h->cfg.zchunk};
        if (h->cfg.kernel == AH_KERNEL_TILE2) {
            // a single step between two-step passes runs the default one-step
            // tiling (every tiling gives the same fields)
            if (default_tile(h->p.precision, h->p.N, &tc.tx, &tc.ty))
                tc.zchunk = auto_zchunk(AH_KERNEL_TILE, h->p.precision, h->p.N, tc.tx, tc.ty, false);
        }
        e = launch_step_tile<R>(in, out, lconst(h->p), c, tc, nullptr, nullptr, true, h->stream);
    } else {
        e = launch_step<R>(in, out.phr, out.phi, out.a0, out.a1, out.a2, lconst(h->p), c, h->stream);
    }
    if (e != hipSuccess) return e;
    e = t.end();
    if (e != hipSuccess) return e;
    h->cur ^= 1;
    h->step += 1;
    return hipSuccess;
}

// Two steps in one pass (kernel AH_KERNEL_TILE2): reads snapshot n from the
// current buffers and writes snapshot n+2 into the other phi/A and Pi/E ones.
template <typename R>
hipError_t do_step2(ah_handle* h)
{
    Fields<R> in = fields_of<R>(h, h->cur);
    Fields<R> out = fields_of<R>(h, h->cur ^ 1);
    const int om = h->curm ^ 1;
    out.pir = (R*)h->mom[om][0];
    out.pii = (R*)h->mom[om][1];
    out.e0 = (R*)h->mom[om][2];
    out.e1 = (R*)h->mom[om][3];
    out.e2 = (R*)h->mom[om][4];
    const StepCoef c0 = coef_at(h->p, h->step), c1 = coef_at(h->p, h->step + 1);
    const TileConfig tc{h->cfg.tile_x, h->cfg.tile_y, h->cfg.zchunk};
    TimedLaunch t{h, 2};
    hipError_t e = t.begin();
    if (e != hipSuccess) return e;
    e = launch_step2_tile<R>(in, out, lconst(h->p), c0, c1, tc, h->stream);
    if (e != hipSuccess) return e;
    e = t.end();
    if (e != hipSuccess) return e;
    h->cur ^= 1;
    h->curm ^= 1;
    h->step += 2;
    return hipSuccess;
}

// nsteps plain steps: two-step passes while at least two remain when the
// handle's kernel is AH_KERNEL_TILE2, single steps otherwise.
hipError_t plain_steps(ah_handle* h, int64_t nsteps)
{
    const bool two = h->cfg.kernel == AH_KERNEL_TILE2;
    while (nsteps > 0) {
        hipError_t e;
        if (two && nsteps >= 2) {
            e = h->p.precision == AH_FP64 ? do_step2<double>(h) : do_step2<float>(h);
            nsteps -= 2;
        } else {
            e = h->p.precision == AH_FP64 ? do_step<double>(h) : do_step<float>(h);
            nsteps -= 1;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int ah_params_default(ah_params* p)
{
    if (!p) return AH_E_INVAL;
    std::memset(p, 0, sizeof(*p));
    p->N = 64;
    p->precision = AH_FP64;
    p->gauge_action = AH_COMPACT;
    p->dx = 0.5;
    p->deta = 0.1;
    p->lambda0 = 2.0;
    p->e0 = 1.0;
    p->sigma = 1.0;
    p->m = 1.0;
    p->alpha = 2.0;
    p->s_early = 0.0;
    p->s_late = 0.0;
    p->eta_switch = HUGE_VAL;
    p->eta0 = 1.0;
    p->eta_ref = 0.0;
    p->damp_gamma = 0.0;  // no artificial damping phase
    p->eta_damp = 0.0;
    return AH_OK;
}

int ah_stability_margin(const ah_params* p, int64_t step, double* mu)
{
    return no_throw([&]() -> int {
        std::string why;
        if (validate(p, &why) != AH_OK || step < 0 || !mu) return AH_E_INVAL;
        *mu = stability_margin(*p, step);
        return AH_OK;
    });
}

int ah_required_bytes(const ah_params* p, size_t* bytes)
{
    return no_throw([&]() -> int {
        std::string why;
        int rc = validate(p, &why);
        if (rc != AH_OK) return rc;
        if (!bytes) return AH_E_INVAL;
        *bytes = required_bytes(*p);
        return AH_OK;
    });
}

int ah_create(const ah_params* p, void* dev_arena, size_t arena_bytes, void* hip_stream, ah_handle** out)
{
    return no_throw([&]() -> int {
        if (!out) return AH_E_INVAL;
        *out = nullptr;
        std::string why;
        int rc = validate(p, &why);
        if (rc != AH_OK) {
            std::fprintf(stderr, "ah_create: %s\n", why.c_str());
            return rc;
        }
        ah_handle* h = new (std::nothrow) ah_handle;
        if (!h) return AH_E_NOMEM;
        h->p = *p;
        h->stream = (hipStream_t)hip_stream;
        h->V = (int64_t)p->N * p->N * p->N;
        h->P = row_pitch(p->N, p->precision);
        h->real_bytes = p->precision == AH_FP64 ? 8 : 4;
        hipError_t e = hipGetDevice(&h->device);
        if (e != hipSuccess) {
            delete h;
            return AH_E_DEVICE;
        }
        const size_t need = required_bytes(*p);
        if (dev_arena) {
            if (arena_bytes < need || ((uintptr_t)dev_arena % kAlign) != 0) {
                delete h;
                return AH_E_NOMEM;
            }
            h->arena = dev_arena;
            h->arena_bytes = arena_bytes;
        } else {
            e = hipMalloc(&h->arena, need);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                delete h;
                return AH_E_NOMEM;
            }
            h->owns_arena = true;
            h->arena_bytes = need;
        }
        char* base = (char*)h->arena;
        const size_t fb = field_bytes(*p);
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 5; ++c) {
                h->pp[b][c] = base;
                base += fb;
            }
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 5; ++c) {
                h->mom[b][c] = base;
                base += fb;
            }
        h->partials = (double*)base;
        base += align_up(partial_records(*p) * kMeasStride * sizeof(double));
        h->result = (double*)base;
        base += align_up(kMeasStride * sizeof(double));
        h->series = (double*)base;
        e = hipHostMalloc((void**)&h->host_result, kMeasStride * sizeof(double), hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&h->host_series, (size_t)kSeriesCap * kMeasStride * sizeof(double),
                              hipHostMallocDefault);
        if (e != hipSuccess) {
            if (h->host_result) (void)hipHostFree(h->host_result);
            if (h->owns_arena) (void)hipFree(h->arena);
            delete h;
            return AH_E_NOMEM;
        }
        {
            std::string why2;
            const ah_step_config dflt{AH_KERNEL_AUTO, 0, 0, 0};
            if (resolve_config(h->p, dflt, &h->cfg, &why2) != AH_OK) {
                (void)hipHostFree(h->host_result);
                if (h->owns_arena) (void)hipFree(h->arena);
                delete h;
                return AH_E_INVAL;
            }
        }
        *out = h;
        return AH_OK;
    });
}

int ah_set_step_config(ah_handle* h, const ah_step_config* c)
{
    return no_throw([&]() -> int {
        if (!h || !c) return fail(h, AH_E_INVAL, "ah_set_step_config: bad argument");
        std::string why;
        ah_step_config r;
        int rc = resolve_config(h->p, *c, &r, &why);
        if (rc != AH_OK) return fail(h, rc, "ah_set_step_config: " + why);
        h->cfg = r;
        return AH_OK;
    });
}

int ah_get_step_config(const ah_handle* h, ah_step_config* c)
{
    if (!h || !c) return AH_E_INVAL;
    *c = h->cfg;
    return AH_OK;
}

int ah_init(ah_handle* h, uint64_t seed)
{
    return no_throw([&]() -> int {
        if (!h) return AH_E_INVAL;
        DeviceGuard g(h->device);
        h->cur = 0;
        h->curm = 0;
        h->step = 0;
        hipError_t e = h->p.precision == AH_FP64
                           ? launch_init<double>(fields_of<double>(h, 0), h->p.N, h->P, h->p.sigma, seed, h->stream)
                           : launch_init<float>(fields_of<float>(h, 0), h->p.N, h->P, h->p.sigma, seed, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "ah_init launch");
        h->ready = true;
        return AH_OK;
    });
}

int ah_set_state(ah_handle* h, const double* host_soa, int64_t step)
{
    return no_throw([&]() -> int {
        if (!h || !host_soa || step < 0) return fail(h, AH_E_INVAL, "ah_set_state: bad argument");
        DeviceGuard g(h->device);
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "ah_set_state sync");
        h->cur = 0;
        h->curm = 0;
        const size_t V = (size_t)h->V;
        std::vector<float> tmp;
        if (h->real_bytes == 4) tmp.resize(V);
        for (int c = 0; c < 10; ++c) {
            const double* src = host_soa + (size_t)c * V;
            if (h->real_bytes == 8) {
                e = field_upload(comp_ptr(h, c), src, h->p.N, h->P, 8, h->stream);
            } else {
                for (size_t i = 0; i < V; ++i) tmp[i] = (float)src[i];
                e = field_upload(comp_ptr(h, c), tmp.data(), h->p.N, h->P, 4, h->stream);
            }
            if (e != hipSuccess) return hip_fail(h, e, "ah_set_state copy");
            e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "ah_set_state sync");
        }
        h->step = step;
        h->ready = true;
        return AH_OK;
    });
}

int ah_get_state(ah_handle* h, double* host_soa, int64_t* step)
{
    return no_throw([&]() -> int {
        if (!h || !host_soa) return fail(h, AH_E_INVAL, "ah_get_state: bad argument");
        if (!h->ready) return fail(h, AH_E_STATE, "ah_get_state before ah_init/ah_set_state");
        DeviceGuard g(h->device);
        const size_t V = (size_t)h->V;
        std::vector<float> tmp;
        if (h->real_bytes == 4) tmp.resize(V);
        for (int c = 0; c < 10; ++c) {
            double* dst = host_soa + (size_t)c * V;
            hipError_t e;
            if (h->real_bytes == 8) {
                e = field_download(dst, comp_ptr(h, c), h->p.N, h->P, 8, h->stream);
            } else {
                e = field_download(tmp.data(), comp_ptr(h, c), h->p.N, h->P, 4, h->stream);
            }
            if (e != hipSuccess) return hip_fail(h, e, "ah_get_state copy");
            e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "ah_get_state sync");
            if (h->real_bytes == 4)
                for (size_t i = 0; i < V; ++i) dst[i] = (double)tmp[i];
        }
        if (step) *step = h->step;
        return AH_OK;
    });
}

int ah_gather(ah_handle* h, const int64_t* sites, int64_t count, double* host_out)
{
    return no_throw([&]() -> int {
        if (!h || count < 0 || (count > 0 && (!sites || !host_out))) return fail(h, AH_E_INVAL, "ah_gather: bad argument");
        if (!h->ready) return fail(h, AH_E_STATE, "ah_gather before ah_init/ah_set_state");
        for (int64_t k = 0; k < count; ++k)
            if (sites[k] < 0 || sites[k] >= h->V) return fail(h, AH_E_INVAL, "ah_gather: site index out of range");
        if (count == 0) return AH_OK;
        DeviceGuard g(h->device);
        void* d_sites = nullptr;
        void* d_out = nullptr;
        const size_t rb = h->real_bytes;
        std::vector<float> tmp(rb == 4 ? count * 10 : 0);  // host staging first: a throw after hipMalloc would leak
        hipError_t e = hipMalloc(&d_sites, count * sizeof(int64_t));
        if (e == hipSuccess) e = hipMalloc(&d_out, count * 10 * rb);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (d_sites) (void)hipFree(d_sites);
            return fail(h, AH_E_NOMEM, "ah_gather: cannot allocate the temporary buffers");
        }
        e = hipMemcpyAsync(d_sites, sites, count * sizeof(int64_t), hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess)
            e = rb == 8 ? launch_gather<double>(fields_of<double>(h, h->cur), (const int64_t*)d_sites, count, h->p.N, h->P,
                                                (double*)d_out, h->stream)
                        : launch_gather<float>(fields_of<float>(h, h->cur), (const int64_t*)d_sites, count, h->p.N, h->P,
                                               (float*)d_out, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(rb == 8 ? (void*)host_out : (void*)tmp.data(), d_out, count * 10 * rb,
                               hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        (void)hipFree(d_sites);
        (void)hipFree(d_out);
        if (e != hipSuccess) return hip_fail(h, e, "ah_gather");
        if (rb == 4)
            for (int64_t q = 0; q < count * 10; ++q) host_out[q] = (double)tmp[q];
        return AH_OK;
    });
}

int ah_gather_noalloc(ah_handle* h, const int64_t* sites, int64_t count, double* host_out)
{
    return no_throw([&]() -> int {
        if (!h || count < 0 || (count > 0 && (!sites || !host_out)))
            return fail(h, AH_E_INVAL, "ah_gather_noalloc: bad argument");
        if (count > kGatherMax)
            return fail(h, AH_E_INVAL, "ah_gather_noalloc: more than 65536 sites in one call");
        if (!h->ready) return fail(h, AH_E_STATE, "ah_gather_noalloc before ah_init/ah_set_state");
        for (int64_t k = 0; k < count; ++k)
            if (sites[k] < 0 || sites[k] >= h->V)
                return fail(h, AH_E_INVAL, "ah_gather_noalloc: site index out of range");
        if (count == 0) return AH_OK;
        DeviceGuard g(h->device);
        void* base = nullptr;
        hipError_t e = scratch_ptr(h->device, &base);
        if (e != hipSuccess) return hip_fail(h, e, "ah_gather_noalloc: scratch lookup");
        // scratch layout: kGatherMax site indices, then the gathered values
        int64_t* d_sites = (int64_t*)base;
        void* d_out = (char*)base + (size_t)kGatherMax * sizeof(int64_t);
        const size_t rb = h->real_bytes;
        e = hipMemcpyAsync(d_sites, sites, count * sizeof(int64_t), hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess)
            e = rb == 8 ? launch_gather<double>(fields_of<double>(h, h->cur), d_sites, count, h->p.N, h->P, (double*)d_out,
                                                h->stream)
                        : launch_gather<float>(fields_of<float>(h, h->cur), d_sites, count, h->p.N, h->P, (float*)d_out,
                                               h->stream);
        // FP32 values land in the first half of host_out and are widened in
        // place, last first, so no host staging buffer is needed either
        if (e == hipSuccess)
            e = hipMemcpyAsync(host_out, d_out, count * 10 * rb, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "ah_gather_noalloc");
        if (rb == 4) {
            const float* src = (const float*)host_out;
            for (int64_t q = count * 10 - 1; q >= 0; --q) host_out[q] = (double)src[q];
        }
        return AH_OK;
    });
}

int ah_get_step(const ah_handle* h, int64_t* step)
{
    if (!h || !step) return AH_E_INVAL;
    *step = h->step;
    return AH_OK;
}

int ah_step(ah_handle* h, int64_t nsteps)
{
    return no_throw([&]() -> int {
        if (!h || nsteps < 0) return fail(h, AH_E_INVAL, "ah_step: bad argument");
        if (!h->ready) return fail(h, AH_E_STATE, "ah_step before ah_init/ah_set_state");
        DeviceGuard g(h->device);
        const hipError_t e = plain_steps(h, nsteps);
        if (e != hipSuccess) return hip_fail(h, e, "ah_step launch");
        return AH_OK;
    });
}

int ah_step_measured(ah_handle* h, int64_t nsteps, int32_t measure_every, ah_measurement* series, int32_t cap,
                     int32_t* n)
{
    return no_throw([&]() -> int {
        if (!h || nsteps < 0 || measure_every <= 0 || !n || (cap > 0 && !series))
            return fail(h, AH_E_INVAL, "ah_step_measured: bad argument");
        if (!h->ready) return fail(h, AH_E_STATE, "ah_step_measured before ah_init/ah_set_state");
        if (h->p.gauge_action != AH_COMPACT)
            return fail(h, AH_E_INVAL, "ah_step_measured: fused diagnostics need the compact action");
        int64_t due = 0;
        for (int64_t k = 0; k < nsteps; ++k)
            if ((h->step + k) % measure_every == 0) ++due;
        if (due > cap) return fail(h, AH_E_INVAL, "ah_step_measured: more due snapshots than cap");
        DeviceGuard g(h->device);
        int32_t written = 0;
        std::vector<int64_t> steps;
        auto flush = [&]() -> hipError_t {
            if (steps.empty()) return hipSuccess;
            hipError_t e = hipMemcpyAsync(h->host_series, h->series, steps.size() * kMeasStride * sizeof(double),
                                          hipMemcpyDeviceToHost, h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return e;
            for (size_t j = 0; j < steps.size(); ++j)
                to_measurement(h->p, steps[j], h->host_series + j * kMeasStride, h->V, &series[written++]);
            steps.clear();
            return hipSuccess;
        };
        const int64_t end = h->step + nsteps;
        while (h->step < end) {
            hipError_t e;
            if (h->step % measure_every == 0) {
                if ((int)steps.size() == kSeriesCap) {
                    e = flush();
                    if (e != hipSuccess) return hip_fail(h, e, "ah_step_measured copy");
                }
                steps.push_back(h->step);
                double* dst = h->series + (steps.size() - 1) * kMeasStride;
                e = h->p.precision == AH_FP64 ? measured_pass<double>(h, dst, true) : measured_pass<float>(h, dst, true);
            } else {
                // the plain steps up to the next due snapshot (or the end)
                const int64_t next = (h->step / measure_every + 1) * measure_every;
                e = plain_steps(h, (next < end ? next : end) - h->step);
            }
            if (e != hipSuccess) return hip_fail(h, e, "ah_step_measured launch");
        }
        hipError_t e = flush();
        if (e != hipSuccess) return hip_fail(h, e, "ah_step_measured copy");
        *n = written;
        return AH_OK;
    });
}

int ah_get_timing_split(ah_handle* h, double* measured_ms, int64_t* measured_launches)
{
    return no_throw([&]() -> int {
        if (!h || !measured_ms || !measured_launches) return fail(h, AH_E_INVAL, "ah_get_timing_split: bad argument");
        DeviceGuard g(h->device);
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "ah_get_timing_split sync");
        double tot = 0.0;
        for (size_t k = 0; k + 1 < h->ev_used; k += 2) {
            if (!h->ev_measured[k / 2]) continue;
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, h->ev[k], h->ev[k + 1]);
            if (e != hipSuccess) return hip_fail(h, e, "ah_get_timing_split elapsed");
            tot += ms;
        }
        *measured_ms = tot;
        *measured_launches = h->measured_launches;
        return AH_OK;
    });
}

int ah_measure(ah_handle* h, ah_measurement* out)
{
    return no_throw([&]() -> int {
        if (!h || !out) return fail(h, AH_E_INVAL, "ah_measure: bad argument");
        if (!h->ready) return fail(h, AH_E_STATE, "ah_measure before ah_init/ah_set_state");
        DeviceGuard g(h->device);
        const ah_params& p = h->p;
        hipError_t e;
        if (p.gauge_action == AH_COMPACT) {
            e = p.precision == AH_FP64 ? measured_pass<double>(h, h->result, false)
                                       : measured_pass<float>(h, h->result, false);
        } else {
            const StepCoef c = coef_at(p, h->step);
            const MeasConst mc = meas_const(p, h->step);
            e = p.precision == AH_FP64 ? launch_measure<double>(fields_of<double>(h, h->cur), lconst(p), c, mc,
                                                                h->partials, h->result, h->stream)
                                       : launch_measure<float>(fields_of<float>(h, h->cur), lconst(p), c, mc,
                                                               h->partials, h->result, h->stream);
        }
        if (e != hipSuccess) return hip_fail(h, e, "ah_measure launch");
        e = hipMemcpyAsync(h->host_result, h->result, M_COUNT * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "ah_measure copy");
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "ah_measure sync");
        to_measurement(p, h->step, h->host_result, h->V, out);
        return AH_OK;
    });
}

int ah_get_winding(ah_handle* h, int8_t* host_w)
{
    return no_throw([&]() -> int {
        if (!h || !host_w) return fail(h, AH_E_INVAL, "ah_get_winding: bad argument");
        if (!h->ready) return fail(h, AH_E_STATE, "ah_get_winding before ah_init/ah_set_state");
        DeviceGuard g(h->device);
        int8_t* d = nullptr;
        const size_t bytes = 3 * (size_t)h->V;
        hipError_t e = hipMalloc(&d, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, AH_E_NOMEM, "ah_get_winding: cannot allocate the temporary winding buffer");
        }
        e = h->p.precision == AH_FP64 ? launch_winding<double>(fields_of<double>(h, h->cur), lconst(h->p), d, h->stream)
                                      : launch_winding<float>(fields_of<float>(h, h->cur), lconst(h->p), d, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(host_w, d, bytes, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        hipError_t e2 = hipFree(d);
        if (e != hipSuccess) return hip_fail(h, e, "ah_get_winding");
        if (e2 != hipSuccess) return hip_fail(h, e2, "ah_get_winding free");
        return AH_OK;
    });
}

int ah_synchronize(ah_handle* h)
{
    return no_throw([&]() -> int {
        if (!h) return AH_E_INVAL;
        DeviceGuard g(h->device);
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "ah_synchronize");
        return AH_OK;
    });
}

int ah_set_timing(ah_handle* h, int enable)
{
    return no_throw([&]() -> int {
        if (!h) return AH_E_INVAL;
        h->timing = enable != 0;
        h->ev_used = 0;
        h->measured_launches = 0;
        h->ev_measured.clear();
        h->ev_steps.clear();
        return AH_OK;
    });
}

int ah_get_timing(ah_handle* h, double* total_ms, int64_t* launches)
{
    return no_throw([&]() -> int {
        if (!h || !total_ms || !launches) return fail(h, AH_E_INVAL, "ah_get_timing: bad argument");
        DeviceGuard g(h->device);
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "ah_get_timing sync");
        double tot = 0.0;
        for (size_t k = 0; k + 1 < h->ev_used; k += 2) {
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, h->ev[k], h->ev[k + 1]);
            if (e != hipSuccess) return hip_fail(h, e, "ah_get_timing elapsed");
            tot += ms;
        }
        int64_t steps = 0;
        for (size_t k = 0; k < h->ev_used / 2; ++k) steps += h->ev_steps[k];
        *total_ms = tot;
        *launches = steps;
        return AH_OK;
    });
}

int ah_destroy(ah_handle* h)
{
    if (!h) return AH_E_INVAL;
    DeviceGuard g(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (hipEvent_t ev : h->ev) (void)hipEventDestroy(ev);
    if (h->host_result) (void)hipHostFree(h->host_result);
    if (h->host_series) (void)hipHostFree(h->host_series);
    if (h->owns_arena && h->arena) (void)hipFree(h->arena);
    delete h;
    return AH_OK;
}

const char* ah_strerror(int code)
{
    switch (code) {
    case AH_OK: return "ok";
    case AH_E_INVAL: return "invalid argument";
    case AH_E_NOMEM: return "out of device memory or arena too small";
    case AH_E_DEVICE: return "HIP device error";
    case AH_E_STATE: return "call out of order";
    case AH_E_AGAIN: return "resource busy; retry later";
    default: return "unknown error";
    }
}

const char* ah_last_error(const ah_handle* h)
{
    if (!h) return "";
    return h->err.c_str();
}

}  // extern "C"
