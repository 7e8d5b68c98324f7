// Internal declarations shared by the host runtime and the HIP kernels of libah.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ah.h"

namespace ah {

// Runs the body of a C-ABI entry point: an exception from the host containers
// it uses (host memory exhausted, a size past what a container can hold)
// becomes AH_E_NOMEM instead of crossing the ABI.
template <typename F>
inline int no_throw(F&& body) noexcept
{
    try {
        return body();
    } catch (...) {
        return AH_E_NOMEM;
    }
}

// Structure-of-arrays field pointers of one lattice snapshot.  phi and A come
// from the current ping-pong buffer, Pi and E are single buffers updated in
// place; the drift writes phi and A into the other ping-pong buffer.
template <typename R>
struct Fields {
    R* phr;
    R* phi;
    R* pir;
    R* pii;
    R* a0;
    R* a1;
    R* a2;
    R* e0;
    R* e1;
    R* e2;
};

// Per-step scalars of the update, formed on the host in FP64 and rounded to
// the storage type (kick: X^{n+1/2} = c1 X^{n-1/2} + c2 force).
struct StepCoef {
    double cP1, cP2;   // (1-delta)/(1+delta), deta/(1+delta)
    double cE1, cE2;   // (1-omega)/(1+omega), deta/(1+omega)
    double lam_half;   // lambda0 f / 2
    double kappa;      // 2 e0^2 f
};

// Stored layout of every field of a lattice: site (x, y, z) at element
// x + P (y + N z), with the row pitch P >= N a whole number of 128-byte cache
// lines.  Every row then starts on a line, and a tile's rows are read as
// whole lines whatever N is; the P - N elements that end a row are never
// read or written.
inline int row_pitch(int N, int precision)
{
    const int per_line = precision == AH_FP64 ? 16 : 32;
    return (N + per_line - 1) / per_line * per_line;
}

// Lattice-wide constants.
struct LatticeConst {
    int N;
    int P;  // row pitch (row_pitch(N, precision))
    int compact;
    double dx, deta, sigma2;
};

// Diagnostics reduction slots (FP64 sums over sites unless noted).  The
// Lagrangian sum is kin - grad - pot + el - mag of the first five, so it has
// no slot of its own.
enum MeasSlot {
    M_KIN = 0,   // |Pi_bar|^2
    M_GRAD,      // sum_i |D_i^+ phi|^2
    M_POT,       // lambda0 f/4 (|phi|^2 - sigma^2)^2
    M_EL,        // sum_i E_bar_i^2 / (2 e0^2 f)
    M_MAG,       // sum_{i<j} B_ij^2 / (2 e0^2 f)
    M_KINL,      // |Pi_bar|^2 L
    M_GRADL,     // sum_i |D_i^+ phi|^2 L
    M_PL,        // p L, with the pressure p = kin - grad/3 - pot + (el + mag)/3
    M_RHOL,      // rho L, with the energy density rho = kin + grad + pot + el + mag
    M_G2,        // G^2
    M_DIV2,      // (div E)^2
    M_CRHO2,     // (c rho)^2
    M_GMAX,      // max |G|   (max-reduced)
    M_WABS,      // sum_{i<j} |W_ij|  (exact integer in FP64)
    M_NONFIN,    // count of sites with a non-finite value
    M_COUNT
};
constexpr int kMarchSums = M_RHOL + 1;  // FP64 sums the measured march forms: slots 0 .. M_RHOL
constexpr int kMeasStride = 16;        // doubles per partial record
static_assert(M_COUNT <= kMeasStride, "a record holds every slot");
constexpr int kMeasBlocks = 2048;      // fixed grid of the measurement kernel
constexpr int kMeasThreads = 256;

struct MeasConst {
    double inv_2e2f;   // 1 / (2 e0^2 f)
    double lam_quarter;// lambda0 f / 4
    double gauss_c;    // coupling of the Gauss residual
};

// Tiled step kernel shape: TX x TY sites per workgroup, zchunk x2-planes per
// workgroup (0 = the whole lattice).
struct TileConfig {
    int tx, ty, zchunk;
};

// Tile shapes the tiled kernels are built for (the 1024-thread ones for FP32 only).
inline bool tile_supported(int precision, int tx, int ty)
{
    if (tx == 64 && (ty == 8 || ty == 4)) return true;
    if (tx == 32 && ty == 8) return true;
    if (tx == 128 && ty == 4) return true;
    if ((tx == 64 && ty == 16) || (tx == 128 && ty == 8)) return precision == AH_FP32;
    return false;
}

// Tile shapes of the two-step pass (its LDS holds two regions of links per
// workgroup, so the FP64 shapes are the smaller ones).
inline bool tile2_supported(int precision, int tx, int ty)
{
    if ((tx == 32 && ty == 8) || (tx == 64 && ty == 4)) return true;
    return tx == 64 && ty == 8 && precision == AH_FP32;
}

// Tile shapes of the pool's batched plain step (its measured step runs the
// measured march's shape, measured_tile).
inline bool batch_tile_supported(int precision, int tx, int ty)
{
    if ((tx == 64 && (ty == 8 || ty == 4)) || (tx == 32 && ty == 8)) return true;
    return precision == AH_FP32 && tx == 128 && (ty == 4 || ty == 8);
}

// Default one-step tile shape for side N; false if none applies.
bool default_tile(int precision, int N, int* tx, int* ty);
// Workgroups of a tiled launch one CU holds at once (measured: the march
// that also forms the diagnostics).
int resident_per_cu(int kernel, int precision, int tx, int ty, bool measured);
// Automatic z-chunk of a tiled launch.
int auto_zchunk(int kernel, int precision, int N, int tx, int ty, bool measured);
// Tiling of the measured march of a lattice stepped with cfg (resolved).
TileConfig measured_tiling(const ah_params& p, const ah_step_config& cfg);

// Smallest z-chunk the tiled kernels accept for a lattice of side N.  Short
// chunks pay for themselves only on small lattices, which they give enough
// workgroups (64^3 FP32 on MI355X: 2-plane chunks step in 11.4 us, 8-plane
// ones in 22 us); larger lattices keep at least 8 planes, which bounds the
// diagnostics records a handle holds.
inline int min_zchunk(int N) { return N <= 128 ? 2 : 8; }

// Tile shape for the measured march of a lattice stepped on (tx, ty): the
// fastest measured march, FP32 64 x 8 and FP64 32 x 8 (the 1024-thread FP32
// and 512-thread FP64 shapes would spill registers).  Returns whether it
// changed.
inline bool measured_tile(int precision, int* tx, int* ty)
{
    const int mx = precision == AH_FP64 ? 32 : 64, my = 8;
    const bool changed = mx != *tx || my != *ty;
    *tx = mx;
    *ty = my;
    return changed;
}

// ---- lattice pool (many independent lattices advanced by one launch) ------
// Row layout of a lattice's per-step FP64 coefficient table.
enum CoefSlot { C_P1 = 0, C_P2, C_E1, C_E2, C_LAMH, C_KAPPA, C_INV2E2F, C_LAMQ, C_GAUSS, kCoefStride = 10 };

// Device-resident descriptor of one pool lattice (plain data; uploaded by the host).
struct PoolLattice {
    void* pp[2][5];        // ping-pong phi_re, phi_im, A0, A1, A2; counter[2] names the current one
    void* mom[2][5];       // Pi_re, Pi_im, E0, E1, E2; counter[3] names the current one (updated in place by a
                           // plain single step; a two-step pass and a measured step write the other)
    const double* coef;    // (nsteps + 1) rows of kCoefStride doubles
    int64_t* counter;      // kCounterWords words: local step k, measurements taken, phi/A buffer, Pi/E buffer
    double* partials;      // diagnostics records of this lattice
    double* series;        // measurement records: kSeriesStride doubles each
    int64_t nsteps;        // steps to run; the lattice is finished when counter[0] == nsteps + 1
    int64_t series_cap;
    int N, tiles_x, tiles_y, zchunk;     // step tiling
    int meas_zchunk, meas_blocks, measure_every, precision;
    int P;                   // row pitch
    int mtiles_x, mtiles_y;  // tiling of the measured step (measured_tile), z-chunks of meas_zchunk
    int two_tiles_x, two_tiles_y, two_zchunk;  // tiling of the two-step pass; two_zchunk == 0: none
    int compact;
    double dx, deta, sigma2;
};
struct WorkItem {
    int lattice, tile;  // lattice < 0: an empty item (padding)
};
constexpr int kXcdCount = 8;           // XCDs of the device; block b runs on XCD b % 8
constexpr int kCounterWords = 4;       // int64 words of a pool lattice's counter
constexpr int kSeriesStride = 18;      // M_COUNT sums + step index + pad
static_assert(M_COUNT + 1 <= kSeriesStride, "a series record holds the sums and the step index");

// ---- fixed device scratch (ah_scratch.hip) ---------------------------------
// Sites one ah_gather_noalloc call may ask for, and the scratch that holds
// their indices and their FP64-sized values.
constexpr int64_t kGatherMax = 65536;
constexpr size_t kScratchBytes = (size_t)kGatherMax * sizeof(int64_t) + (size_t)kGatherMax * 10 * sizeof(double);
// Device address of `device`'s copy of the scratch (looked up on the first
// call for that device, with it current).
hipError_t scratch_ptr(int device, void** out);

// Copies between a dense host array of N^3 values (x fastest) and a stored
// field of row pitch P, element size rb, enqueued on s (ah_runtime.cpp).
hipError_t field_upload(void* dev, const void* host, int N, int P, size_t rb, hipStream_t s);
hipError_t field_download(void* host, const void* dev, int N, int P, size_t rb, hipStream_t s);

// ---- launchers (ah_kernels.hip, ah_step_tile.hip) -------------------------
template <typename R>
hipError_t launch_init(const Fields<R>& f, int N, int P, double sigma, uint64_t seed, hipStream_t s);

template <typename R>
hipError_t launch_step(const Fields<R>& in, R* ophr, R* ophi, R* oa0, R* oa1, R* oa2,
                       const LatticeConst& L, const StepCoef& c, hipStream_t s);

// Tiled step from `in` to `out`: phi and A into out's (other) buffers, Pi
// and E into out's, which may be in's (an update in place).  With mc !=
// nullptr also the diagnostics of the snapshot read, Gauss residual included
// (one record per workgroup into partials, in tile order); a measured step
// then needs Pi and E out of place (else hipErrorInvalidValue).  write =
// false leaves the fields untouched (diagnostics only).
template <typename R>
hipError_t launch_step_tile(const Fields<R>& in, const Fields<R>& out, const LatticeConst& L, const StepCoef& c,
                            const TileConfig& tc, const MeasConst* mc, double* partials, bool write, hipStream_t s);

// Two steps in one pass: snapshot n of `in` to snapshot n+2 of `out` (all
// ten fields in other buffers), with the coefficients of steps n and n+1.
template <typename R>
hipError_t launch_step2_tile(const Fields<R>& in, const Fields<R>& out, const LatticeConst& L, const StepCoef& c0,
                             const StepCoef& c1, const TileConfig& tc, hipStream_t s);

// workgroups (= diagnostics records) of one tiled launch
int step_tile_blocks(int N, const TileConfig& tc);


template <typename R>
hipError_t launch_step_batch(const PoolLattice* lat, const WorkItem* work, int nwork, int tx, int ty, int grid,
                             bool measured, hipStream_t s);
// the pool's two-step pass (ah_step2.hip): lattices whose step k takes one
template <typename R>
hipError_t launch_step2_batch(const PoolLattice* lat, const WorkItem* work, int nwork, int tx, int ty, int grid,
                              hipStream_t s);

template <typename R>
hipError_t launch_measure(const Fields<R>& f, const LatticeConst& L, const StepCoef& c,
                          const MeasConst& mc, double* partials, double* result, hipStream_t s);

// second-stage fold of nblocks per-workgroup records into result[M_COUNT]
hipError_t launch_measure_final(const double* partials, int nblocks, double* result, hipStream_t s);

hipError_t launch_fold_batch(const PoolLattice* lat, int nlat, hipStream_t s);
hipError_t launch_advance_batch(const PoolLattice* lat, int nlat, hipStream_t s);

template <typename R>
hipError_t launch_gather(const Fields<R>& f, const int64_t* sites, int64_t count, int N, int P, R* out, hipStream_t s);

template <typename R>
hipError_t launch_winding(const Fields<R>& f, const LatticeConst& L, int8_t* w, hipStream_t s);

}  // namespace ah
