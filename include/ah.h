/*
 * ah.h -- C ABI of the MI355X Abelian-Higgs lattice library (libah.so).
 *
 * One handle evolves one periodic comoving N^3 lattice of the U(1)
 * Abelian-Higgs model in a flat FRW background, in temporal gauge, with the
 * staggered leapfrog / Crank-Nicolson discretisation of Correia & Martins,
 * "Abelian-Higgs cosmic string evolution with multiple GPUs", section 2:
 *
 *   (1+delta) Pi^{n+1/2}  = (1-delta) Pi^{n-1/2}
 *                            + deta [ D_j^- D_j^+ phi^n - (lambda0/2) f_n (|phi^n|^2 - sigma^2) phi^n ]
 *   (1+omega) E_i^{n+1/2} = (1-omega) E_i^{n-1/2}
 *                            + deta [ -sum_{j!=i} d_j^- F_ij^n + 2 e0^2 f_n Im(phi^* D_i^+ phi)^n ]
 *   phi^{n+1} = phi^n + deta Pi^{n+1/2},   A_i^{n+1} = A_i^n + deta E_i^{n+1/2}
 *
 * with links U_j = exp(-i dx A_j), the covariant Laplacian
 * D_j^- D_j^+ phi^x = sum_j [U_j^x phi^{x+j} - 2 phi^x + conj(U_j^{x-j}) phi^{x-j}] / dx^2,
 * the compact plaquette field strength F_ij = sin(Theta_ij)/dx^2 with
 * Theta_ij^x = dx (A_i^x + A_j^{x+i} - A_i^{x+j} - A_j^x) (or Theta/dx^2 for
 * the non-compact action), a(eta) = (eta/eta_ref)^m, f = a^(2s),
 * delta = (alpha/2) m deta/eta (damp_gamma deta/2 during an optional
 * artificial damping phase) and omega = (1-s) delta (section 2, damping
 * coefficients and coupling scaling).
 *
 * Diagnostics (section 2, string-separation and velocity estimators):
 * xi_W from gauge-invariant plaquette windings, xi_L from the Lagrangian
 * sum, <v^2>_phi = 2R/(1+R) with the Lagrangian-weighted ratio R,
 * <v^2>_omega = (1 + 3w)/2 with w the Lagrangian-weighted ratio of the
 * pressure kin - grad/3 - pot + (el + mag)/3 to the energy density (the
 * paper leaves p, rho and the weight undefined; this is the reading taken),
 * plus the energy split and the discrete Gauss-law residual.
 *
 * Conventions
 *   - site index idx = x0 + N*(x1 + N*x2); periodic in all three directions.
 *   - host state buffers are structure-of-arrays FP64, 10*N^3 doubles, in the
 *     component order phi_re, phi_im, pi_re, pi_im, A0, A1, A2, E0, E1, E2;
 *     they are owned by the caller and only read or written during the call.
 *   - snapshot n holds phi, A at eta_n = eta0 + n*deta and Pi, E at eta_n - deta/2.
 *   - every function returns AH_OK (0) or a negative AH_E_* code and never
 *     throws across the ABI; ah_last_error() gives the text of the last error
 *     on a handle (including the HIP error string for AH_E_DEVICE).
 *   - numerical trouble (blow-up) is not an error: it is reported in
 *     ah_measurement.flags and .nonfinite.
 *   - threading: a handle must be used from one host thread at a time;
 *     distinct handles are independent.
 *   - all device work of a handle is enqueued on the HIP stream given at
 *     creation (NULL = the null stream).  Calls documented "asynchronous"
 *     return before the GPU has finished; kernel errors surface at the next
 *     synchronising call.
 */
#ifndef AH_H
#define AH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define AH_OK 0
#define AH_E_INVAL (-1)  /* bad argument or parameter */
#define AH_E_NOMEM (-2)  /* device allocation failed or arena too small */
#define AH_E_DEVICE (-3) /* HIP runtime error; see ah_last_error */
#define AH_E_STATE (-4)  /* call out of order (e.g. step before init) */
#define AH_E_AGAIN (-5)  /* resource busy or full now; retry later */

#define AH_FP64 0
#define AH_FP32 1

#define AH_COMPACT 0    /* F = sin(Theta)/dx^2 (compact Wilson action) */
#define AH_NONCOMPACT 1 /* F = Theta/dx^2 */

#define AH_FLAG_UNSTABLE 1u  /* leapfrog stability margin deta*sqrt(max(lambda0,2e0^2) f sigma^2 + 12/dx^2) >= 2 */
#define AH_FLAG_NONFINITE 2u /* some field value is NaN or Inf */

/* --------------------------------------------------------------- params */
typedef struct ah_params {
    int32_t N;            /* lattice side, N >= 4 */
    int32_t precision;    /* AH_FP64 or AH_FP32: type of the stored fields and of the step arithmetic */
    int32_t gauge_action; /* AH_COMPACT or AH_NONCOMPACT */
    int32_t reserved;     /* must be 0 */
    double dx, deta;      /* lattice spacing and conformal time step (section 2: 0.5, 0.1) */
    double lambda0, e0, sigma; /* couplings and vacuum expectation value (section 2: 2, 1, 1) */
    double m;             /* d ln a / d ln eta: 0 flat, 1 radiation, 2 matter */
    double alpha;         /* damping multiplier; 2 is Crank-Nicolson Hubble friction */
    double s_early, s_late, eta_switch; /* s = s_early for eta < eta_switch, else s_late */
    double eta0;          /* initial conformal time (section 2: 1) */
    double eta_ref;       /* a(eta_ref) = 1; <= 0 selects the half light-crossing time dx*N/2 */
    double damp_gamma;    /* artificial damping phase: while eta < eta_damp the momentum equations */
    double eta_damp;      /*   have the constant friction damp_gamma in place of the Hubble term
                           *   (delta = damp_gamma deta / 2, omega = (1 - s) delta); 0: no such phase */
} ah_params;

/* Fill *p with the paper's standard choices (section 2): N = 64, FP64,
 * compact, dx = 0.5, deta = 0.1, lambda0 = 2, e0 = 1, sigma = 1, m = 1,
 * alpha = 2, s = 0 throughout, eta0 = 1, eta_ref = dx*N/2, no damping phase. */
int ah_params_default(ah_params* p);

/* ---------------------------------------------------------- measurement */
typedef struct ah_measurement {
    int64_t step;               /* snapshot index n */
    double eta, a, f;           /* eta_n, a(eta_n), f_n = a^(2 s_n) */
    int64_t winding_sum_abs;    /* sum over sites and orientations i<j of |W_ij| (exact) */
    double L_W, xi_W;           /* dx * winding_sum_abs ; sqrt((N dx)^3 / L_W) */
    double sum_L, xi_L;         /* dx^3 sum_x L_x ; sqrt(-2 pi sigma^2 (N dx)^3 / sum_L) (NaN if sum_L >= 0) */
    double R, v2_phi;           /* sum |Pi|^2 L / sum |D+phi|^2 L ; 2R/(1+R) */
    double energy, e_kin, e_grad, e_pot, e_el, e_mag; /* dx^3-weighted sums with centred momenta */
    double gauss_rms, gauss_max, gauss_rel; /* norms of the Gauss residual G^x */
    int64_t nonfinite;          /* sites with a non-finite field value */
    uint32_t flags;             /* AH_FLAG_* */
    uint32_t reserved;
    double v2_omega;            /* (1 + 3 w)/2, w = sum p L / sum rho L: equation-of-state estimator */
} ah_measurement;

typedef struct ah_handle ah_handle;

/* Leapfrog stability margin of snapshot `step` (host arithmetic only, no
 * device work): mu = deta * sqrt(max(lambda0, 2 e0^2) f sigma^2 + 12/dx^2),
 * the largest angular frequency of the linearised update times deta.  The
 * explicit scheme is stable for mu < 2; ah_measure sets AH_FLAG_UNSTABLE when
 * mu >= 2.  AH_E_INVAL on bad parameters or step < 0. */
int ah_stability_margin(const ah_params* p, int64_t step, double* mu);

/* Device bytes one lattice needs: 20 field arrays (the 10 state fields twice:
 * a single step drifts phi and A into the other buffer, a two-step pass and
 * a measured step write all ten) of N^3 reals each, plus reduction scratch.
 * AH_E_INVAL on bad params. */
int ah_required_bytes(const ah_params* p, size_t* bytes);

/* Create a handle on the current HIP device.
 *   dev_arena == NULL: the library allocates (hipMalloc) and owns the memory.
 *   else: dev_arena is device memory of at least ah_required_bytes bytes,
 *         256-byte aligned, owned by the caller, which keeps it alive until
 *         ah_destroy returns (AH_E_NOMEM if arena_bytes is too small).
 *   hip_stream: a hipStream_t (NULL = null stream) on which all work runs.
 * The lattice is uninitialised until ah_init or ah_set_state. */
int ah_create(const ah_params* p, void* dev_arena, size_t arena_bytes, void* hip_stream, ah_handle** out);

/* Random-phase initial condition at eta0, step 0 (section 2): phi = sigma
 * exp(2 pi i u_x) with u_x = (SplitMix64(seed) output number idx >> 11) *
 * 2^-53 evaluated in FP64 (rounded to the storage type), Pi = A = E = 0.
 * Asynchronous. */
int ah_init(ah_handle* h, uint64_t seed);

/* Upload a host FP64 SoA state (10*N^3 doubles, see conventions) as snapshot
 * `step` (>= 0).  Values are rounded to the storage type.  Synchronous. */
int ah_set_state(ah_handle* h, const double* host_soa, int64_t step);

/* Download the current snapshot as FP64 SoA (10*N^3 doubles) and its step
 * index (step may be NULL).  Synchronous. */
int ah_get_state(ah_handle* h, double* host_soa, int64_t* step);

/* Values of the current snapshot at `count` listed site indices (each in
 * [0, N^3), else AH_E_INVAL before any device work): host_out[10*k + c] is
 * component c (state order) of site sites[k], widened to FP64.  For
 * spot-checking lattices too large to download.  Allocates two temporary
 * device buffers (count*8 and count*10*sizeof(real) bytes).  Synchronous. */
int ah_gather(ah_handle* h, const int64_t* sites, int64_t count, double* host_out);

/* ah_gather without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, checks and results as ah_gather, with
 * count <= 65536 (AH_E_INVAL above that, before any device work).  The site
 * indices and gathered values are staged in a fixed device scratch array of
 * 5.5 MB per GPU, held by the library until the process ends; the call makes
 * no device (or host) allocation.  Every call on a GPU uses that GPU's one
 * array, so calls that overlap on one GPU (from several host threads, or on
 * several streams) race: the caller serialises them.  Synchronous. */
int ah_gather_noalloc(ah_handle* h, const int64_t* sites, int64_t count, double* host_out);

/* Current snapshot index (host-side counter; no synchronisation). */
int ah_get_step(const ah_handle* h, int64_t* step);

/* Advance nsteps (>= 0) full leapfrog steps (kick + drift).  Asynchronous.
 * AH_E_STATE before ah_init/ah_set_state. */
int ah_step(ah_handle* h, int64_t nsteps);

/* Advance nsteps steps; the snapshots n with n % measure_every == 0 among
 * the ones stepped from (current .. current+nsteps-1) get their diagnostics
 * in the same pass as their step (the diagnostics read what the step reads).
 * Writes those records to series (cap >= their number, else AH_E_INVAL) and
 * their count to *n.  The records equal what ah_measure returns on the same
 * snapshots.  Compact action only.  Synchronous at the end. */
int ah_step_measured(ah_handle* h, int64_t nsteps, int32_t measure_every, ah_measurement* series, int32_t cap,
                     int32_t* n);

/* The part of ah_get_timing that belongs to launches which also formed
 * diagnostics (ah_step_measured): their summed time (ms) and number, so
 * that callers can separate plain and measured steps.  Synchronises. */
int ah_get_timing_split(ah_handle* h, double* measured_ms, int64_t* measured_launches);

/* All diagnostics of the current snapshot, summed in FP64 in a fixed order
 * (bitwise reproducible for a given handle configuration).  Site densities
 * are formed in the storage precision; link phases, plaquette angles and
 * windings in FP64 from the stored values, so windings are exact for FP32
 * lattices too.  The snapshot is not modified.  Synchronous. */
int ah_measure(ah_handle* h, ah_measurement* out);

/* Per-plaquette windings of the current snapshot: 3*N^3 int8 values,
 * orientation-major ((0,1), (0,2), (1,2)), site index inside.  Allocates a
 * temporary device buffer of 3*N^3 bytes.  Synchronous. */
int ah_get_winding(ah_handle* h, int8_t* host_w);

/* ------------------------------------------------------ step kernel choice */
#define AH_KERNEL_AUTO 0 /* tiled kernel for the compact action, site kernel otherwise */
#define AH_KERNEL_SITE 1 /* one thread per site, every neighbour read from global memory */
#define AH_KERNEL_TILE 2 /* z-marching tiles with links shared through LDS (compact action only) */
#define AH_KERNEL_TILE2 3 /* as AH_KERNEL_TILE, with two steps per pass over the fields wherever two plain
                           * steps follow each other: the step n -> n+1 is formed on the tile plus a
                           * one-site ring and kept in LDS, the step n+1 -> n+2 on the tile from it, so
                           * the fields are read and written once per two steps.  Bitwise equal to two
                           * single steps.  Tiles (32,8), (64,4), FP32 also (64,8); a single plain step
                           * it leaves (an odd count) runs the tiled kernel on its default tiling, the
                           * measured steps on the measured march's tiling */

/* Performance knobs of the step; they do not change the equations.  The
 * tiled kernel gives bitwise-identical results for every tile shape and
 * z-chunk; the site kernel agrees with it to rounding. */
typedef struct ah_step_config {
    int32_t kernel;         /* AH_KERNEL_* */
    int32_t tile_x, tile_y; /* tiled kernel: (64,8), (64,4), (32,8), (128,4) (FP32 also (64,16), (128,8));
                             * two-step kernel: see AH_KERNEL_TILE2; 0,0 = default: the shape of the
                             * highest measured rate once the idle lanes of a ragged last tile are
                             * counted (one step), (32,8) (two steps) */
    int32_t zchunk;         /* x2-planes per workgroup of the tiled kernel; 0 = automatic: equal chunks,
                             * the count that minimises (rounds of resident workgroups) x (planes per
                             * chunk + 2); else >= 2 for N <= 128 and >= 8 above (the last chunk of a
                             * column may be shorter) */
} ah_step_config;

/* Select the step kernel; AH_E_INVAL for an unsupported combination. */
int ah_set_step_config(ah_handle* h, const ah_step_config* c);

/* The configuration in use, with automatic choices resolved. */
int ah_get_step_config(const ah_handle* h, ah_step_config* c);

/* Wait for all work enqueued on the handle's stream. */
int ah_synchronize(ah_handle* h);

/* Step-kernel timing with HIP events on the handle's stream.  While enabled
 * every step-kernel launch is bracketed by an event pair; ah_get_timing
 * synchronises and returns the summed kernel time (ms) and the number of
 * steps those launches advanced since the last enable (a two-step pass counts
 * two), so total_ms / launches is the kernel time per step.  Lattice results
 * do not change. */
int ah_set_timing(ah_handle* h, int enable);
int ah_get_timing(ah_handle* h, double* total_ms, int64_t* launches);

/* Free what the library allocated; the handle is invalid afterwards. */
int ah_destroy(ah_handle* h);

/* ------------------------------------------------------------- autotuner */
/* Time every supported tile shape and z-chunk of the tiled step, with one
 * and with two steps per pass (AH_KERNEL_TILE, AH_KERNEL_TILE2), for
 * (p->precision, p->N) on a scratch lattice (library-allocated: 20 N^3 reals,
 * freed before returning; `steps` timed steps per candidate) and record the
 * fastest per step in the process-wide tuning table.  Handles created afterwards with
 * the automatic configuration, and lattices submitted to a pool, use the
 * recorded choice.  Synchronous.  AH_E_INVAL for the non-compact action. */
int ah_autotune(const ah_params* p, int32_t steps, ah_step_config* best, double* best_ms);

/* Recorded choice for (p->precision, p->N); AH_E_AGAIN if none. */
int ah_tune_lookup(const ah_params* p, ah_step_config* out);

/* Record a choice by hand: kernel AH_KERNEL_TILE or AH_KERNEL_TILE2, a tile
 * shape that kernel supports for the precision, zchunk 0 (automatic) or at
 * least the minimum of ah_step_config.zchunk; AH_E_INVAL otherwise.  Pool
 * lattices take the tile shape of a two-step entry and step once per replay. */
int ah_tune_set(const ah_params* p, const ah_step_config* c);

/* Forget every recorded choice. */
int ah_tune_clear(void);

/* Save / load the tuning table as JSON (one entry per line:
 * {"precision": "fp32", "N": 128, "tile_x": 64, "tile_y": 8, "zchunk": 32, "ms": 0.01, "kernel": "tile"};
 * "kernel" is "tile" or "tile2", "tile" when absent).
 * Loading adds to (and overrides entries of) the table.  AH_E_INVAL if the
 * file cannot be opened or holds an entry that does not parse or that
 * ah_tune_set would refuse; the table is then unchanged. */
int ah_tune_save(const char* path);
int ah_tune_load(const char* path);

/* --------------------------------------------------------- lattice pool */
/* A pool keeps many independent lattices (any N, precision, expansion
 * history; compact action) resident in one device arena and advances all
 * active ones together: each ah_pool_advance step is one replay of a HIP
 * graph holding the measured step of the lattices whose snapshot is due (it
 * forms every diagnostic, the Gauss residual included) and its fixed-order
 * fold, the plain step of every other active lattice (one kernel node per precision and
 * tile shape, one block per (lattice, tile) work item) and a counter update;
 * an FP32 lattice whose next two snapshots are both not due takes a
 * two-step pass instead (AH_KERNEL_TILE2; 64 x 8 unless its tuning entry
 * names another two-step shape), which advances it by two steps in that
 * replay.  Pool lattices run the tuned one-step (else the default) tile
 * shape with z-chunks of at least 16 planes (ah_pool_step_config reports
 * them), and their measured steps the measured march's tiling, as a lattice
 * alone does.  Every lattice takes the coefficients of its own step from its own
 * FP64 table, so its fields and diagnostics are bitwise identical to the
 * same lattice run alone through ah_step / ah_measure with the same tiling.
 * Requests enter and leave between advances (continuous batching); the
 * graph is captured again only when a node's work list outgrows its
 * capacity (or shrinks far below it) or a new node is needed.  A pool is
 * used from one host thread at a time. */
typedef struct ah_pool ah_pool;

typedef struct ah_pool_info {
    size_t budget;          /* arena bytes */
    size_t bytes_in_use;    /* sum of admitted footprints */
    size_t largest_free;    /* largest contiguous free block */
    int32_t active;         /* lattices admitted and not yet collected */
    int32_t max_slots;
    int64_t graph_launches; /* steps issued so far */
    int64_t graph_captures; /* times the per-step graph was captured */
} ah_pool_info;

/* Create a pool with a device arena of hbm_budget bytes (hipMalloc'd and
 * owned by the pool) and at most max_slots lattices.  hip_stream == NULL: the
 * pool creates its own stream (graph capture needs a non-null stream). */
int ah_pool_create(size_t hbm_budget, int32_t max_slots, void* hip_stream, ah_pool** out);

/* Device bytes a request occupies in a pool: fields (20 arrays of N^2 rows
 * of the pitched length: phi, A, Pi and E each double-buffered), diagnostics
 * records, the (nsteps+1)-row coefficient table, the series. */
int ah_pool_footprint(const ah_params* p, int64_t nsteps, int32_t measure_every, size_t* bytes);

/* Admit a lattice: random-phase IC from `seed` (as ah_init), `nsteps` steps,
 * diagnostics of snapshots 0, measure_every, 2 measure_every, ... and always
 * of the final snapshot (measure_every = 0: the final one only).  Returns the
 * request id.  AH_E_AGAIN when no slot or not enough contiguous free memory is
 * available now; AH_E_NOMEM when the request exceeds the whole budget.  The
 * uploads and the initial condition are queued on the pool stream after the
 * replays already there (through pinned staging; the call does not wait for
 * them unless a coefficient table exceeds 16 MB). */
int ah_pool_submit(ah_pool* pool, const ah_params* p, uint64_t seed, int64_t nsteps, int32_t measure_every,
                   int64_t* id);

/* Enqueue nsteps graph replays (one step of every active lattice each) and a
 * copy of the step counters behind them.  Asynchronous, with at most eight
 * replays queued ahead of the host: past that it waits until the GPU has
 * reached a replay four or more behind the newest (never for the whole
 * queue).  A set of lattices changed by submit or results gets a new graph
 * here, built while earlier replays still run. */
int ah_pool_advance(ah_pool* pool, int32_t nsteps);

/* Ids of lattices that finished since the last poll (at most cap; *n is the
 * number written).  Synchronises with the pool stream. */
int ah_pool_poll(ah_pool* pool, int64_t* done_ids, int32_t cap, int32_t* n);

/* As ah_pool_poll without waiting: reports the lattices that the newest
 * counter copy already on the host shows finished (the copies queued by
 * ah_pool_advance land as the GPU reaches them).  For serving loops that keep
 * the GPU busy while they admit and collect requests. */
int ah_pool_poll_async(ah_pool* pool, int64_t* done_ids, int32_t cap, int32_t* n);

/* Tile shape and z-chunk a request is stepped with (kernel AH_KERNEL_TILE).
 * The pool takes the tuned configuration of the request's (precision, N), or
 * the default one, with z-chunks of at least 16 planes and one tile shape
 * for its plain and measured steps.  Host only.  AH_E_INVAL for an unknown id. */
int ah_pool_step_config(const ah_pool* pool, int64_t id, ah_step_config* out);

/* Current step of a request and its target (nsteps may be NULL). */
int ah_pool_progress(ah_pool* pool, int64_t id, int64_t* step, int64_t* nsteps);

/* Current snapshot of a request as FP64 SoA and its step: host_soa must hold
 * 10 N^3 doubles for the N that request was submitted with (the call writes
 * that many; it cannot check the buffer).  Synchronous.  AH_E_INVAL for an
 * unknown id. */
int ah_pool_get_state(ah_pool* pool, int64_t id, double* host_soa, int64_t* step);

/* Measurement series of a finished request (at most cap records; *n written)
 * and release of its slot and memory.  A request with measure_every = k > 0
 * has nsteps/k + 2 records at most (every k-th step and the final one); with
 * k = 0, one.  AH_E_AGAIN if it has not finished.  For a request a poll has
 * reported, the series is read on a side stream without waiting for the
 * replays queued on the pool stream. */
int ah_pool_results(ah_pool* pool, int64_t id, ah_measurement* series, int32_t cap, int32_t* n);

/* Occupancy figures. */
int ah_pool_stats(const ah_pool* pool, ah_pool_info* info);

/* Wait for all work enqueued on the pool stream. */
int ah_pool_synchronize(ah_pool* pool);

/* Text of the last error on the pool ("" if none). */
const char* ah_pool_last_error(const ah_pool* pool);

/* Free the arena and everything else the pool holds. */
int ah_pool_destroy(ah_pool* pool);

/* ------------------------------------------------------ bandwidth probe */
/* Achievable HBM bandwidth of the current device, the reference the step's
 * bytes per second are read against besides the nominal peak: streaming
 * copy (bytes read + written), read-only and write-only kernels over two
 * library-allocated buffers of `bytes` each (>= 1 MiB; freed before
 * returning), `reps` timed launches per launch shape, best shape reported, in
 * GB/s (1e9 bytes/s).  Synchronous; AH_E_NOMEM if the buffers do not fit. */
int ah_hbm_probe(size_t bytes, int32_t reps, double* copy_gbps, double* read_gbps, double* write_gbps);

/* Static description of an error code. */
const char* ah_strerror(int code);

/* Text of the last error on h ("" if none); valid until the next call on h. */
const char* ah_last_error(const ah_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* AH_H */
