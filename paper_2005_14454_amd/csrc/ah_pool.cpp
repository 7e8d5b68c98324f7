// Lattice pool of libah: many independent lattices of different sizes,
// precisions and expansion histories resident in one HBM arena and advanced
// together, one graph launch per step.
//
// Each lattice owns its fields, a per-step FP64 coefficient table, its
// diagnostics records and its measurement series inside the arena, plus a
// descriptor and a counter (step, measurements taken, buffer parities) in
// pool metadata.  The graph replayed per step is
//     measured step (lattices whose snapshot is due) -> fold
//     -> single step and two-step pass (one node per precision and tile
//     shape) -> advance counters
// and every kernel reads the lattice's own counter, so the same graph serves
// every step until the set of lattices changes.
//
// The host never drains the stream in the serving path: uploads (coefficient
// tables, descriptors, work lists) go through a pinned staging ring and are
// ordered on the pool stream after the replays already queued; each advance
// queues a copy of the step counters into pinned memory behind an event, and
// ah_pool_poll_async reads the newest copy that has landed; series downloads
// run on a side stream.  At most kMaxInflight replays are queued ahead of the
// host, so a request admitted now joins within that many steps.
#include "ah.h"
#include "ah_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

using namespace ah;

namespace ah {
// shared with the single-lattice runtime (ah_runtime.cpp)
int resolve_step_config(const ah_params& p, const ah_step_config& in, ah_step_config* out, std::string* why);
int validate_params(const ah_params* p, std::string* why);
void coef_row(const ah_params& p, int64_t n, double* row);
void to_measurement(const ah_params& p, int64_t step, const double* r, int64_t V, ah_measurement* out);
bool tuned_config(const ah_params& p, ah_step_config* out);
}  // namespace ah

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

constexpr int64_t kMaxInflight = 8;  // graph replays queued ahead of the host
constexpr int kSnapshots = 16;       // counter copies in flight (> kMaxInflight)
constexpr size_t kStageBytes = 32u << 20;

struct Slot {
    bool used = false;
    int64_t id = -1;
    int64_t seq = 0;  // admission order: counter copies issued before it do not describe it
    ah_params p{};
    int64_t nsteps = 0;
    int measure_every = 0;
    size_t off = 0, bytes = 0;
    ah_step_config cfg{};
    TileConfig meas{};  // tiling of the measured step
    TileConfig two{};   // tiling of the two-step pass (zchunk 0: none)
    PoolLattice d{};
    bool reported = false;
};

struct Footprint {
    size_t field, fields, partials, coef, series, total;
    TileConfig meas;  // tiling of the measured step
    int meas_blocks;
    int64_t series_cap;
};

// Bytes of one pool lattice (20 fields: phi and A ping-pong, and so do Pi
// and E, which a two-step pass and a measured step write out of place);
// total = SIZE_MAX when nsteps is too large for its coefficient table to be
// addressed at all.
Footprint footprint(const ah_params& p, const ah_step_config& cfg, const TileConfig& two, int64_t nsteps,
                    int measure_every)
{
    Footprint f{};
    if ((uint64_t)nsteps >= (SIZE_MAX / 4) / (kCoefStride * sizeof(double))) {
        f.total = SIZE_MAX;
        return f;
    }
    const size_t stored = (size_t)p.N * p.N * row_pitch(p.N, p.precision);
    f.field = align_up(stored * (p.precision == AH_FP64 ? 8 : 4));
    f.fields = 20 * f.field;
    f.meas = measured_tiling(p, cfg);
    f.meas_blocks = step_tile_blocks(p.N, f.meas);
    f.partials = align_up((size_t)f.meas_blocks * kMeasStride * sizeof(double));
    f.coef = align_up((size_t)(nsteps + 1) * kCoefStride * sizeof(double));
    f.series_cap = (measure_every > 0 ? nsteps / measure_every + 1 : 0) + 1;
    f.series = align_up((size_t)f.series_cap * kSeriesStride * sizeof(double));
    f.total = f.fields + f.partials + f.coef + f.series;
    return f;
}

}  // namespace

struct StageChunk {
    size_t off, len;
    hipEvent_t ev;
};
struct Snapshot {
    int64_t* h = nullptr;    // pinned copy of the counters
    hipEvent_t ev = nullptr;
    int64_t launches = 0;    // replays queued before the copy
    int64_t seq = 0;         // admissions made before the copy
};
struct Retired {
    hipGraphExec_t exec;
    hipGraph_t graph;
    void* buf;
    hipEvent_t ev;  // recorded after the last work that could use them
};

// A node group of the pool graph: kind 1 the plain single step, kind 2 the
// measured step and kind 3 the two-step pass of one precision and tile
// shape.
struct GroupKey {
    int kind, precision, tx, ty;
    bool operator<(const GroupKey& o) const
    {
        return std::tie(kind, precision, tx, ty) < std::tie(o.kind, o.precision, o.tx, o.ty);
    }
};
struct NodeGroup {
    size_t off, cap;  // region of the work list (items); a step group's cap is a multiple of kXcdCount
};

struct ah_pool {
    int device = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    hipStream_t side = nullptr;  // series downloads of finished lattices
    char* stage = nullptr;       // pinned staging ring for uploads
    size_t stage_head = 0;
    std::deque<StageChunk> stage_busy;
    std::vector<hipEvent_t> free_events;
    std::vector<Snapshot> snaps;
    std::deque<int> snap_order;           // issued, not yet read, oldest first
    std::vector<int64_t> host_counters;   // newest counters read back
    int64_t launches_done = 0;            // replays known to have finished
    int64_t seq = 0;                      // admissions so far
    std::vector<Retired> retired;
    void* arena = nullptr;
    size_t budget = 0;
    std::vector<std::pair<size_t, size_t>> free_list;  // (offset, size), sorted by offset
    std::vector<Slot> slots;
    int64_t next_id = 1;
    PoolLattice* d_lat = nullptr;
    int64_t* d_counters = nullptr;
    WorkItem* d_work = nullptr;
    size_t work_cap = 0;
    std::map<GroupKey, NodeGroup> groups;  // work-list regions of the captured graph's nodes
    int64_t graph_captures = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool dirty = true;
    int64_t graph_launches = 0;
    std::string err;
};

namespace {

int pfail(ah_pool* P, int code, const std::string& m)
{
    if (P) P->err = m;
    return code;
}
int phip(ah_pool* P, hipError_t e, const char* what)
{
    return pfail(P, AH_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

struct Guard {
    int prev = -1;
    explicit Guard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~Guard()
    {
        int now = -1;
        if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
    }
};

bool arena_alloc(ah_pool* P, size_t bytes, size_t* off)
{
    for (size_t i = 0; i < P->free_list.size(); ++i) {
        auto& b = P->free_list[i];
        if (b.second >= bytes) {
            *off = b.first;
            b.first += bytes;
            b.second -= bytes;
            if (b.second == 0) P->free_list.erase(P->free_list.begin() + i);
            return true;
        }
    }
    return false;
}

void arena_free(ah_pool* P, size_t off, size_t bytes)
{
    P->free_list.push_back({off, bytes});
    std::sort(P->free_list.begin(), P->free_list.end());
    std::vector<std::pair<size_t, size_t>> merged;
    for (auto& b : P->free_list) {
        if (!merged.empty() && merged.back().first + merged.back().second == b.first)
            merged.back().second += b.second;
        else
            merged.push_back(b);
    }
    P->free_list.swap(merged);
}

size_t largest_free(const ah_pool* P)
{
    size_t m = 0;
    for (auto& b : P->free_list) m = std::max(m, b.second);
    return m;
}

hipError_t take_event(ah_pool* P, hipEvent_t* ev)
{
    if (!P->free_events.empty()) {
        *ev = P->free_events.back();
        P->free_events.pop_back();
        return hipSuccess;
    }
    return hipEventCreateWithFlags(ev, hipEventDisableTiming);
}

// Release staging chunks whose copies have run (wait = also the oldest one).
hipError_t stage_reclaim(ah_pool* P, bool wait)
{
    while (!P->stage_busy.empty()) {
        StageChunk& c = P->stage_busy.front();
        hipError_t e = wait ? hipEventSynchronize(c.ev) : hipEventQuery(c.ev);
        if (e == hipErrorNotReady) return hipSuccess;
        if (e != hipSuccess) return e;
        P->free_events.push_back(c.ev);
        P->stage_busy.pop_front();
        wait = false;
    }
    return hipSuccess;
}

// Upload n bytes from host memory to device memory dst on the pool stream,
// through the staging ring (waiting only for staging space, which earlier
// copies free as they run).  Copies larger than half the ring go directly
// and wait for the stream.
hipError_t stage_upload(ah_pool* P, void* dst, const void* src, size_t n)
{
    if (n == 0) return hipSuccess;
    hipError_t e;
    if (n > kStageBytes / 2) {
        e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, P->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
        return e;
    }
    const size_t len = align_up(n);
    if (P->stage_head + len > kStageBytes) P->stage_head = 0;
    const size_t lo = P->stage_head, hi = lo + len;
    for (;;) {
        bool overlap = false;
        for (const StageChunk& c : P->stage_busy)
            if (c.off < hi && lo < c.off + c.len) overlap = true;
        if (!overlap) break;
        e = stage_reclaim(P, true);
        if (e != hipSuccess) return e;
    }
    std::memcpy(P->stage + lo, src, n);
    e = hipMemcpyAsync(dst, P->stage + lo, n, hipMemcpyHostToDevice, P->stream);
    hipEvent_t ev = nullptr;
    if (e == hipSuccess) e = take_event(P, &ev);
    if (e == hipSuccess) e = hipEventRecord(ev, P->stream);
    if (e != hipSuccess) return e;
    P->stage_busy.push_back({lo, len, ev});
    P->stage_head = hi;
    return hipSuccess;
}

// Read the counter copies that have landed (wait = block for the oldest
// one); the newest becomes the host's view of every lattice admitted before it.
hipError_t read_snapshots(ah_pool* P, bool wait)
{
    while (!P->snap_order.empty()) {
        Snapshot& sn = P->snaps[P->snap_order.front()];
        hipError_t e = wait ? hipEventSynchronize(sn.ev) : hipEventQuery(sn.ev);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) return e;
        for (size_t i = 0; i < P->slots.size(); ++i)
            if (P->slots[i].used && P->slots[i].seq <= sn.seq) {
                for (int w = 0; w < kCounterWords; ++w)
                    P->host_counters[kCounterWords * i + w] = sn.h[kCounterWords * i + w];
            }
        P->launches_done = std::max(P->launches_done, sn.launches);
        P->snap_order.pop_front();
        wait = false;
    }
    // retired graphs and buffers whose last user has run
    for (size_t k = 0; k < P->retired.size();) {
        Retired& r = P->retired[k];
        const hipError_t q = hipEventQuery(r.ev);
        if (q == hipSuccess) {
            if (r.exec) (void)hipGraphExecDestroy(r.exec);
            if (r.graph) (void)hipGraphDestroy(r.graph);
            if (r.buf) (void)hipFree(r.buf);
            P->free_events.push_back(r.ev);
            P->retired.erase(P->retired.begin() + k);
        } else {
            ++k;
        }
    }
    return hipSuccess;
}

// Queue a copy of the counters behind the replays queued so far.
hipError_t queue_snapshot(ah_pool* P)
{
    if ((int)P->snap_order.size() >= kSnapshots) {
        hipError_t e = read_snapshots(P, true);
        if (e != hipSuccess) return e;
    }
    int j = 0;
    for (; j < kSnapshots; ++j) {
        bool busy = false;
        for (int k : P->snap_order) busy |= (k == j);
        if (!busy) break;
    }
    Snapshot& sn = P->snaps[j];
    hipError_t e = hipMemcpyAsync(sn.h, P->d_counters, kCounterWords * P->slots.size() * sizeof(int64_t), hipMemcpyDeviceToHost,
                                  P->stream);
    if (e == hipSuccess) e = hipEventRecord(sn.ev, P->stream);
    if (e != hipSuccess) return e;
    sn.launches = P->graph_launches;
    sn.seq = P->seq;
    P->snap_order.push_back(j);
    return hipSuccess;
}

// Keep a graph (or a buffer) until the work queued so far has run.
hipError_t retire(ah_pool* P, hipGraphExec_t exec, hipGraph_t graph, void* buf)
{
    hipEvent_t ev = nullptr;
    hipError_t e = take_event(P, &ev);
    if (e == hipSuccess) e = hipEventRecord(ev, P->stream);
    if (e != hipSuccess) return e;
    P->retired.push_back({exec, graph, buf, ev});
    return hipSuccess;
}

// Rebuild descriptors and work lists, and the per-step graph when its
// node layout no longer fits.  Nothing here waits for the stream: the
// uploads are ordered after the replays already queued, which keep reading
// the old descriptors and lists until then.
//
// The graph has one step node (plain, measured, two-step) per (precision,
// tile shape), each over a fixed-capacity region
// of the work list whose unused items are empty.  An admission or a release
// that fits the captured capacities only rewrites the lists; a new group or
// a list beyond its capacity (or far below it) captures anew, with room for
// growth.
int rebuild(ah_pool* P)
{
    hipError_t e;
    const int nslot = (int)P->slots.size();
    std::vector<PoolLattice> desc(nslot);
    for (int i = 0; i < nslot; ++i) {
        if (P->slots[i].used) {
            desc[i] = P->slots[i].d;
        } else {
            std::memset(&desc[i], 0, sizeof(PoolLattice));
            desc[i].nsteps = -1;
            desc[i].counter = P->d_counters + kCounterWords * i;
        }
    }
    // the lists each group needs now: step items per (precision, tile shape)
    // in kXcdCount bands
    std::map<GroupKey, std::array<std::vector<WorkItem>, kXcdCount>> step_need;
    // step groups: kind 1 the plain step per (precision, tile shape), kind 2
    // the measured step per (precision, measured tile shape), kind 3 the
    // two-step pass per (precision, tile shape)
    std::map<GroupKey, std::vector<int>> by_shape;
    for (int i = 0; i < nslot; ++i) {
        const Slot& s = P->slots[i];
        if (!s.used) continue;
        by_shape[GroupKey{1, s.p.precision, s.cfg.tile_x, s.cfg.tile_y}].push_back(i);
        by_shape[GroupKey{2, s.p.precision, s.meas.tx, s.meas.ty}].push_back(i);
        if (s.two.zchunk > 0) by_shape[GroupKey{3, s.p.precision, s.two.tx, s.two.ty}].push_back(i);
    }
    // The step kernels run one block per item and give XCD x (which runs
    // blocks x, x+8, ...) the x-th eighth of the list.  So that every XCD
    // gets an equal share of every lattice, with neighbouring tiles (which
    // read each other's halo) in the same L2, each lattice's tiles, in index
    // order, are cut into eight contiguous runs, run x goes to band x, bands
    // list the lattices with the longest z-marches first.
    for (auto& kv : by_shape) {
        const int kind = kv.first.kind;
        auto zc_of = [&](const PoolLattice& d) {
            return kind == 2 ? d.meas_zchunk : (kind == 3 ? d.two_zchunk : d.zchunk);
        };
        auto tiles_of = [&](const PoolLattice& d) {
            return kind == 2 ? d.mtiles_x * d.mtiles_y : (kind == 3 ? d.two_tiles_x * d.two_tiles_y : d.tiles_x * d.tiles_y);
        };
        std::vector<int> order = kv.second;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const PoolLattice &da = P->slots[a].d, &db = P->slots[b].d;
            return std::min(zc_of(da), da.N) > std::min(zc_of(db), db.N);  // planes per item
        });
        auto& band = step_need[kv.first];
        for (int i : order) {
            const PoolLattice& d = P->slots[i].d;
            const int tiles_z = (d.N + zc_of(d) - 1) / zc_of(d);
            const int nt = tiles_of(d) * tiles_z;
            for (int x = 0; x < kXcdCount; ++x) {
                const int t0 = (int)((int64_t)nt * x / kXcdCount), t1 = (int)((int64_t)nt * (x + 1) / kXcdCount);
                for (int t = t0; t < t1; ++t) band[x].push_back({i, t});
            }
        }
    }
    // items each group needs (a step group: kXcdCount bands of the longest band's length)
    std::map<GroupKey, size_t> need;
    for (auto& kv : step_need) {
        size_t len = 0;
        for (auto& b : kv.second) len = std::max(len, b.size());
        need[kv.first] = len * kXcdCount;
    }
    size_t need_total = 0, cap_total = 0;
    bool fits = P->exec != nullptr;
    for (auto& kv : need) {
        need_total += kv.second;
        auto it = P->groups.find(kv.first);
        if (it == P->groups.end() || it->second.cap < kv.second) fits = false;
    }
    for (auto& kv : P->groups) cap_total += kv.second.cap;
    if (cap_total > 4 * std::max<size_t>(need_total, 4096)) fits = false;  // mostly empty: shrink
    if (!fits) {
        // capacities with room for growth (groups that emptied keep a small
        // one), laid out one after another
        std::map<GroupKey, NodeGroup> groups;
        size_t off = 0;
        auto add = [&](const GroupKey& k, size_t n) {
            const size_t unit = (size_t)kXcdCount * 32;
            size_t cap = std::max<size_t>(n + n / 4, unit);
            cap = (cap + unit - 1) / unit * unit;
            groups[k] = NodeGroup{off, cap};
            off += cap;
        };
        for (auto& kv : need) add(kv.first, kv.second);
        for (auto& kv : P->groups)
            if (!need.count(kv.first)) add(kv.first, 0);
        if (off > P->work_cap) {
            // the queued replays may still read the old list: it is freed once they have run
            if (P->d_work) {
                e = retire(P, nullptr, nullptr, P->d_work);
                if (e != hipSuccess) return phip(P, e, "pool work list retire");
            }
            P->d_work = nullptr;
            P->work_cap = 0;
            e = hipMalloc(&P->d_work, off * sizeof(WorkItem));
            if (e != hipSuccess) return phip(P, e, "pool work list allocation");
            P->work_cap = off;
        }
        P->groups = groups;
    }
    // the whole list, every group at its offset, unused items empty
    size_t total = 0;
    for (auto& kv : P->groups) total = std::max(total, kv.second.off + kv.second.cap);
    std::vector<WorkItem> work(total, WorkItem{-1, 0});
    for (auto& kv : step_need) {
        const NodeGroup& g = P->groups[kv.first];
        const size_t per_band = g.cap / kXcdCount;
        for (int x = 0; x < kXcdCount; ++x)
            std::copy(kv.second[x].begin(), kv.second[x].end(), work.begin() + g.off + x * per_band);
    }
    e = stage_upload(P, P->d_lat, desc.data(), nslot * sizeof(PoolLattice));
    if (e == hipSuccess && total) e = stage_upload(P, P->d_work, work.data(), total * sizeof(WorkItem));
    if (e != hipSuccess) return phip(P, e, "pool descriptor upload");
    P->dirty = false;
    if (fits) return AH_OK;

    if (P->exec || P->graph) {
        e = retire(P, P->exec, P->graph, nullptr);
        if (e != hipSuccess) return phip(P, e, "pool graph retire");
    }
    P->exec = nullptr;
    P->graph = nullptr;
    P->dirty = true;  // until a graph is instantiated
    e = hipStreamBeginCapture(P->stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return phip(P, e, "pool graph capture begin");
    hipError_t le = hipSuccess;
    // measured steps of the due lattices, their fold, the plain steps of all
    // others, the counter update
    for (int measured = 1; measured >= 0; --measured) {
        for (auto& kv : P->groups) {
            if (kv.first.kind != (measured ? 2 : 1) || le != hipSuccess) continue;
            const GroupKey& k = kv.first;
            const NodeGroup& g = kv.second;
            const int grid = (int)g.cap;  // one block per work item
            le = k.precision == AH_FP64 ? launch_step_batch<double>(P->d_lat, P->d_work + g.off, (int)g.cap, k.tx,
                                                                    k.ty, grid, measured != 0, P->stream)
                                        : launch_step_batch<float>(P->d_lat, P->d_work + g.off, (int)g.cap, k.tx, k.ty,
                                                                   grid, measured != 0, P->stream);
        }
        if (measured && le == hipSuccess) le = launch_fold_batch(P->d_lat, nslot, P->stream);
    }
    for (auto& kv : P->groups) {
        if (kv.first.kind != 3 || le != hipSuccess) continue;
        const GroupKey& k = kv.first;
        const NodeGroup& g = kv.second;
        le = k.precision == AH_FP64
                 ? launch_step2_batch<double>(P->d_lat, P->d_work + g.off, (int)g.cap, k.tx, k.ty, (int)g.cap, P->stream)
                 : launch_step2_batch<float>(P->d_lat, P->d_work + g.off, (int)g.cap, k.tx, k.ty, (int)g.cap, P->stream);
    }
    if (le == hipSuccess) le = launch_advance_batch(P->d_lat, nslot, P->stream);
    e = hipStreamEndCapture(P->stream, &P->graph);
    if (le != hipSuccess) return phip(P, le, "pool graph capture launch");
    if (e != hipSuccess) return phip(P, e, "pool graph capture end");
    e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return phip(P, e, "pool graph instantiate");
    ++P->graph_captures;
    P->dirty = false;
    return AH_OK;
}

}  // namespace

extern "C" {

int ah_pool_create(size_t hbm_budget, int32_t max_slots, void* hip_stream, ah_pool** out)
{
    return no_throw([&]() -> int {
        if (!out || max_slots <= 0 || max_slots > 65536 || hbm_budget < kAlign) return AH_E_INVAL;
        *out = nullptr;
        ah_pool* P = new (std::nothrow) ah_pool;
        if (!P) return AH_E_NOMEM;
        if (hipGetDevice(&P->device) != hipSuccess) {
            delete P;
            return AH_E_DEVICE;
        }
        hipError_t e;
        if (hip_stream) {
            P->stream = (hipStream_t)hip_stream;
        } else {
            e = hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                delete P;
                return AH_E_DEVICE;
            }
            P->owns_stream = true;
        }
        P->budget = hbm_budget / kAlign * kAlign;
        e = hipMalloc(&P->arena, P->budget);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (P->owns_stream) (void)hipStreamDestroy(P->stream);
            delete P;
            return AH_E_NOMEM;
        }
        P->free_list.push_back({0, P->budget});
        P->slots.resize(max_slots);
        e = hipMalloc(&P->d_lat, max_slots * sizeof(PoolLattice));
        if (e == hipSuccess) e = hipMalloc(&P->d_counters, kCounterWords * max_slots * sizeof(int64_t));
        if (e == hipSuccess) e = hipMemset(P->d_counters, 0, kCounterWords * max_slots * sizeof(int64_t));
        if (e == hipSuccess) e = hipHostMalloc((void**)&P->stage, kStageBytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking);
        P->snaps.resize(kSnapshots);
        for (int j = 0; j < kSnapshots && e == hipSuccess; ++j) {
            e = hipHostMalloc((void**)&P->snaps[j].h, kCounterWords * max_slots * sizeof(int64_t), hipHostMallocDefault);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&P->snaps[j].ev, hipEventDisableTiming);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            (void)ah_pool_destroy(P);
            return AH_E_NOMEM;
        }
        P->host_counters.assign(kCounterWords * (size_t)max_slots, 0);
        *out = P;
        return AH_OK;
    });
}

// Tile configuration of a pool lattice: the tuned one-step configuration if
// the pool's step is built for its shape (a two-step entry lends its tile
// shape, with the automatic z-chunk), else the default, as for a lattice run
// alone; z-chunks of at least 16 planes.  The measured node runs the
// measured march's tiling (measured_tiling), as a lattice alone does.  FP32
// lattices also take two-step passes wherever neither of two snapshots is
// due (two): on the tuned two-step tile shape, else 64 x 8, with the
// automatic z-chunk of at least 16 planes; on MI355X the pass beats the
// single step at every FP32 size measured (65 .. 512) and loses at every
// FP64 size.
// The pool supplies much of the parallelism that short z-chunks buy a
// lattice run alone; 16 planes keep enough work items for ensembles of small
// lattices (measured on MI355X: 128 lattices of N in {32, 48, 64} run 11%
// faster than with 64-plane chunks, a mix of N in 64 .. 256 2% faster; 8
// and 32 planes are slower than 16).
static int pool_config(const ah_params& p, ah_step_config* cfg, TileConfig* two, std::string* why)
{
    ah_step_config t{AH_KERNEL_TILE, 0, 0, 0};
    int two_tx = 64, two_ty = 8;
    if (tuned_config(p, &t)) {
        if (t.kernel == AH_KERNEL_TILE2) {
            two_tx = t.tile_x;
            two_ty = t.tile_y;
            t.zchunk = 0;
        }
        t.kernel = AH_KERNEL_TILE;
        if (!batch_tile_supported(p.precision, t.tile_x, t.tile_y)) t = ah_step_config{AH_KERNEL_TILE, 0, 0, 0};
    }
    const int rc = resolve_step_config(p, t, cfg, why);
    if (rc != AH_OK) return rc;
    auto floor16 = [&](int zc) { return std::min(std::max(zc, 16), p.N); };
    cfg->zchunk = floor16(cfg->zchunk);
    *two = TileConfig{0, 0, 0};
    if (p.precision == AH_FP32 && tile2_supported(p.precision, two_tx, two_ty))
        *two = TileConfig{two_tx, two_ty, floor16(auto_zchunk(AH_KERNEL_TILE2, p.precision, p.N, two_tx, two_ty, false))};
    return AH_OK;
}

int ah_pool_footprint(const ah_params* p, int64_t nsteps, int32_t measure_every, size_t* bytes)
{
    return no_throw([&]() -> int {
        std::string why;
        if (validate_params(p, &why) != AH_OK || nsteps < 0 || measure_every < 0 || !bytes) return AH_E_INVAL;
        if (p->gauge_action != AH_COMPACT) return AH_E_INVAL;
        ah_step_config cfg;
        TileConfig two;
        if (pool_config(*p, &cfg, &two, &why) != AH_OK) return AH_E_INVAL;
        const size_t total = footprint(*p, cfg, two, nsteps, measure_every).total;
        if (total == SIZE_MAX) return AH_E_INVAL;
        *bytes = total;
        return AH_OK;
    });
}

int ah_pool_submit(ah_pool* P, const ah_params* p, uint64_t seed, int64_t nsteps, int32_t measure_every,
                   int64_t* id)
{
    return no_throw([&]() -> int {
        if (!P || !p || !id || nsteps < 0 || measure_every < 0) return pfail(P, AH_E_INVAL, "ah_pool_submit: bad argument");
        std::string why;
        int rc = validate_params(p, &why);
        if (rc != AH_OK) return pfail(P, rc, "ah_pool_submit: " + why);
        ah_step_config cfg{AH_KERNEL_TILE, 0, 0, 0};
        if (p->gauge_action != AH_COMPACT) return pfail(P, AH_E_INVAL, "ah_pool_submit: the pool runs the compact action");
        TileConfig two;
        rc = pool_config(*p, &cfg, &two, &why);
        if (rc != AH_OK) return pfail(P, rc, "ah_pool_submit: " + why);
        const Footprint fp = footprint(*p, cfg, two, nsteps, measure_every);
        if (fp.total > P->budget) return pfail(P, AH_E_NOMEM, "ah_pool_submit: request larger than the pool budget");
        int slot = -1;
        for (int i = 0; i < (int)P->slots.size(); ++i)
            if (!P->slots[i].used) {
                slot = i;
                break;
            }
        if (slot < 0) return pfail(P, AH_E_AGAIN, "ah_pool_submit: no free slot");
        if (largest_free(P) < fp.total) return pfail(P, AH_E_AGAIN, "ah_pool_submit: not enough free memory now");
        // the coefficient table before anything is taken, so that a host
        // allocation failure leaves the pool as it was
        std::vector<double> rows((size_t)(nsteps + 1) * kCoefStride, 0.0);
        for (int64_t k = 0; k <= nsteps; ++k) coef_row(*p, k, rows.data() + k * kCoefStride);
        size_t off;
        if (!arena_alloc(P, fp.total, &off)) return pfail(P, AH_E_AGAIN, "ah_pool_submit: not enough free memory now");
        Guard g(P->device);

        Slot& s = P->slots[slot];
        s = Slot{};
        s.used = true;
        s.id = P->next_id++;
        s.seq = ++P->seq;
        for (int w = 0; w < kCounterWords; ++w) P->host_counters[kCounterWords * slot + w] = 0;
        s.p = *p;
        s.nsteps = nsteps;
        s.measure_every = measure_every;
        s.off = off;
        s.bytes = fp.total;
        s.cfg = cfg;
        s.meas = fp.meas;
        s.two = two;
        char* base = (char*)P->arena + off;
        PoolLattice& d = s.d;
        std::memset(&d, 0, sizeof(d));
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 5; ++c) {
                d.pp[b][c] = base;
                base += fp.field;
            }
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 5; ++c) {
                d.mom[b][c] = base;
                base += fp.field;
            }
        d.partials = (double*)base;
        base += fp.partials;
        double* coef = (double*)base;
        d.coef = coef;
        base += fp.coef;
        d.series = (double*)base;
        d.counter = P->d_counters + kCounterWords * slot;
        d.nsteps = nsteps;
        d.series_cap = fp.series_cap;
        d.N = p->N;
        d.P = row_pitch(p->N, p->precision);
        d.tiles_x = (p->N + cfg.tile_x - 1) / cfg.tile_x;
        d.tiles_y = (p->N + cfg.tile_y - 1) / cfg.tile_y;
        d.zchunk = cfg.zchunk;
        d.mtiles_x = (p->N + fp.meas.tx - 1) / fp.meas.tx;
        d.mtiles_y = (p->N + fp.meas.ty - 1) / fp.meas.ty;
        d.meas_zchunk = fp.meas.zchunk;
        d.meas_blocks = fp.meas_blocks;
        if (two.zchunk > 0) {
            d.two_tiles_x = (p->N + two.tx - 1) / two.tx;
            d.two_tiles_y = (p->N + two.ty - 1) / two.ty;
            d.two_zchunk = two.zchunk;
        }
        d.measure_every = measure_every;
        d.precision = p->precision;
        d.compact = 1;
        d.dx = p->dx;
        d.deta = p->deta;
        d.sigma2 = p->sigma * p->sigma;

        // enqueued on the pool stream after the graph replays already queued
        // (the slot's previous lattice, if any, has finished, so they leave
        // its memory and counter alone); nothing waits for them
        hipError_t e = stage_upload(P, coef, rows.data(), rows.size() * sizeof(double));
        if (e == hipSuccess) e = hipMemsetAsync(d.counter, 0, kCounterWords * sizeof(int64_t), P->stream);
        if (e == hipSuccess) {
            Fields<double> f64;
            Fields<float> f32;
            if (p->precision == AH_FP64) {
                f64 = Fields<double>{(double*)d.pp[0][0], (double*)d.pp[0][1], (double*)d.mom[0][0],
                                     (double*)d.mom[0][1], (double*)d.pp[0][2], (double*)d.pp[0][3],
                                     (double*)d.pp[0][4], (double*)d.mom[0][2], (double*)d.mom[0][3],
                                     (double*)d.mom[0][4]};
                e = launch_init<double>(f64, p->N, d.P, p->sigma, seed, P->stream);
            } else {
                f32 = Fields<float>{(float*)d.pp[0][0], (float*)d.pp[0][1], (float*)d.mom[0][0], (float*)d.mom[0][1],
                                    (float*)d.pp[0][2], (float*)d.pp[0][3], (float*)d.pp[0][4], (float*)d.mom[0][2],
                                    (float*)d.mom[0][3], (float*)d.mom[0][4]};
                e = launch_init<float>(f32, p->N, d.P, p->sigma, seed, P->stream);
            }
        }
        if (e != hipSuccess) {
            arena_free(P, s.off, s.bytes);
            s = Slot{};
            return phip(P, e, "ah_pool_submit");
        }
        P->dirty = true;
        *id = s.id;
        return AH_OK;
    });
}

int ah_pool_advance(ah_pool* P, int32_t nsteps)
{
    return no_throw([&]() -> int {
        if (!P || nsteps < 0) return pfail(P, AH_E_INVAL, "ah_pool_advance: bad argument");
        Guard g(P->device);
        if (P->dirty) {
            int rc = rebuild(P);
            if (rc != AH_OK) return rc;
        }
        hipError_t e = hipSuccess;
        for (int32_t k = 0; k < nsteps; ++k) {
            // keep at most kMaxInflight replays queued ahead of the host: wait
            // for the counter copy queued after an earlier replay (one is
            // queued every kMaxInflight / 2 replays, so the wait leaves at
            // least that many queued)
            while (e == hipSuccess && P->graph_launches - P->launches_done >= kMaxInflight) {
                if (P->snap_order.empty()) e = queue_snapshot(P);
                if (e == hipSuccess) e = read_snapshots(P, true);
            }
            if (e == hipSuccess) e = hipGraphLaunch(P->exec, P->stream);
            if (e != hipSuccess) return phip(P, e, "ah_pool_advance graph launch");
            ++P->graph_launches;
            if (k + 1 < nsteps && P->graph_launches % (kMaxInflight / 2) == 0) {
                e = queue_snapshot(P);
                if (e != hipSuccess) return phip(P, e, "ah_pool_advance counter copy");
            }
        }
        if (nsteps > 0) {
            e = queue_snapshot(P);
            if (e == hipSuccess) e = stage_reclaim(P, false);
            if (e != hipSuccess) return phip(P, e, "ah_pool_advance counter copy");
        }
        return AH_OK;
    });
}

// Ids of lattices the host view shows finished and not yet reported.
static int report_done(ah_pool* P, int64_t* done_ids, int32_t cap, int32_t* n)
{
    int32_t k = 0;
    for (size_t i = 0; i < P->slots.size(); ++i) {
        Slot& s = P->slots[i];
        if (!s.used || s.reported) continue;
        if (P->host_counters[kCounterWords * i] == s.nsteps + 1) {
            if (k < cap) {
                done_ids[k] = s.id;
                s.reported = true;
            }
            ++k;
        }
    }
    *n = k < cap ? k : cap;
    return AH_OK;
}

int ah_pool_poll(ah_pool* P, int64_t* done_ids, int32_t cap, int32_t* n)
{
    return no_throw([&]() -> int {
        if (!P || !n || (cap > 0 && !done_ids)) return pfail(P, AH_E_INVAL, "ah_pool_poll: bad argument");
        Guard g(P->device);
        hipError_t e = queue_snapshot(P);
        if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
        if (e == hipSuccess) e = read_snapshots(P, true);
        if (e != hipSuccess) return phip(P, e, "ah_pool_poll");
        return report_done(P, done_ids, cap, n);
    });
}

int ah_pool_poll_async(ah_pool* P, int64_t* done_ids, int32_t cap, int32_t* n)
{
    return no_throw([&]() -> int {
        if (!P || !n || (cap > 0 && !done_ids)) return pfail(P, AH_E_INVAL, "ah_pool_poll_async: bad argument");
        Guard g(P->device);
        hipError_t e = read_snapshots(P, false);
        if (e != hipSuccess) return phip(P, e, "ah_pool_poll_async");
        return report_done(P, done_ids, cap, n);
    });
}

static Slot* find_slot(ah_pool* P, int64_t id, int* index)
{
    for (size_t i = 0; i < P->slots.size(); ++i)
        if (P->slots[i].used && P->slots[i].id == id) {
            if (index) *index = (int)i;
            return &P->slots[i];
        }
    return nullptr;
}

int ah_pool_step_config(const ah_pool* P, int64_t id, ah_step_config* out)
{
    if (!P || !out) return AH_E_INVAL;
    for (const Slot& s : P->slots)
        if (s.used && s.id == id) {
            *out = s.cfg;
            return AH_OK;
        }
    return AH_E_INVAL;
}

int ah_pool_progress(ah_pool* P, int64_t id, int64_t* step, int64_t* nsteps)
{
    return no_throw([&]() -> int {
        if (!P || !step) return pfail(P, AH_E_INVAL, "ah_pool_progress: bad argument");
        int i;
        Slot* s = find_slot(P, id, &i);
        if (!s) return pfail(P, AH_E_INVAL, "ah_pool_progress: unknown id");
        Guard g(P->device);
        int64_t c[kCounterWords];
        hipError_t e = hipMemcpyAsync(c, P->d_counters + kCounterWords * i, sizeof(c), hipMemcpyDeviceToHost, P->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
        if (e != hipSuccess) return phip(P, e, "ah_pool_progress");
        *step = std::min(c[0], s->nsteps);
        if (nsteps) *nsteps = s->nsteps;
        return AH_OK;
    });
}

int ah_pool_get_state(ah_pool* P, int64_t id, double* host_soa, int64_t* step)
{
    return no_throw([&]() -> int {
        if (!P || !host_soa) return pfail(P, AH_E_INVAL, "ah_pool_get_state: bad argument");
        int i;
        Slot* s = find_slot(P, id, &i);
        if (!s) return pfail(P, AH_E_INVAL, "ah_pool_get_state: unknown id");
        Guard g(P->device);
        int64_t c[kCounterWords];
        hipError_t e = hipMemcpyAsync(c, P->d_counters + kCounterWords * i, sizeof(c), hipMemcpyDeviceToHost, P->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
        if (e != hipSuccess) return phip(P, e, "ah_pool_get_state");
        const int64_t k = std::min(c[0], s->nsteps);
        const int cur = (int)c[2], curm = (int)c[3];  // the buffers of snapshot k
        const size_t V = (size_t)s->p.N * s->p.N * s->p.N;
        const size_t rb = s->p.precision == AH_FP64 ? 8 : 4;
        void* const* m = s->d.mom[curm];
        void* comps[10] = {s->d.pp[cur][0], s->d.pp[cur][1], m[0], m[1], s->d.pp[cur][2],
                           s->d.pp[cur][3], s->d.pp[cur][4], m[2], m[3], m[4]};
        std::vector<float> tmp(rb == 4 ? V : 0);
        for (int cc = 0; cc < 10; ++cc) {
            double* dst = host_soa + cc * V;
            e = field_download(rb == 8 ? (void*)dst : (void*)tmp.data(), comps[cc], s->p.N, s->d.P, rb, P->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
            if (e != hipSuccess) return phip(P, e, "ah_pool_get_state copy");
            if (rb == 4)
                for (size_t q = 0; q < V; ++q) dst[q] = (double)tmp[q];
        }
        if (step) *step = k;
        return AH_OK;
    });
}

int ah_pool_results(ah_pool* P, int64_t id, ah_measurement* series, int32_t cap, int32_t* n)
{
    return no_throw([&]() -> int {
        if (!P || !n || (cap > 0 && !series)) return pfail(P, AH_E_INVAL, "ah_pool_results: bad argument");
        int i;
        Slot* s = find_slot(P, id, &i);
        if (!s) return pfail(P, AH_E_INVAL, "ah_pool_results: unknown id");
        Guard g(P->device);
        hipError_t e;
        int64_t c[kCounterWords];
        for (int w = 0; w < kCounterWords; ++w) c[w] = P->host_counters[kCounterWords * i + w];
        if (c[0] != s->nsteps + 1) {
            // not seen finished yet: read the counters after the queued work
            e = hipMemcpyAsync(c, P->d_counters + kCounterWords * i, sizeof(c), hipMemcpyDeviceToHost, P->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
            if (e != hipSuccess) return phip(P, e, "ah_pool_results");
            if (c[0] != s->nsteps + 1) return pfail(P, AH_E_AGAIN, "ah_pool_results: the lattice has not finished");
        }
        // a finished lattice is no longer written, so its series is read on
        // the side stream while the pool stream runs on
        const int64_t nm = std::min(c[1], s->d.series_cap);
        std::vector<double> raw((size_t)nm * kSeriesStride);
        if (nm > 0) {
            e = hipMemcpyAsync(raw.data(), s->d.series, raw.size() * sizeof(double), hipMemcpyDeviceToHost, P->side);
            if (e == hipSuccess) e = hipStreamSynchronize(P->side);
            if (e != hipSuccess) return phip(P, e, "ah_pool_results copy");
        }
        const int64_t V = (int64_t)s->p.N * s->p.N * s->p.N;
        const int32_t m = (int32_t)std::min<int64_t>(nm, cap);
        for (int32_t k = 0; k < m; ++k)
            to_measurement(s->p, (int64_t)raw[(size_t)k * kSeriesStride + M_COUNT], raw.data() + (size_t)k * kSeriesStride,
                           V, &series[k]);
        *n = m;
        arena_free(P, s->off, s->bytes);
        *s = Slot{};
        P->dirty = true;
        return AH_OK;
    });
}

int ah_pool_stats(const ah_pool* P, ah_pool_info* info)
{
    if (!P || !info) return AH_E_INVAL;
    std::memset(info, 0, sizeof(*info));
    info->budget = P->budget;
    size_t used = 0;
    for (const Slot& s : P->slots)
        if (s.used) {
            used += s.bytes;
            info->active += 1;
        }
    info->bytes_in_use = used;
    info->largest_free = largest_free(P);
    info->max_slots = (int32_t)P->slots.size();
    info->graph_launches = P->graph_launches;
    info->graph_captures = P->graph_captures;
    return AH_OK;
}

int ah_pool_synchronize(ah_pool* P)
{
    return no_throw([&]() -> int {
        if (!P) return AH_E_INVAL;
        Guard g(P->device);
        hipError_t e = hipStreamSynchronize(P->stream);
        if (e == hipSuccess) e = read_snapshots(P, true);
        if (e != hipSuccess) return phip(P, e, "ah_pool_synchronize");
        return AH_OK;
    });
}

const char* ah_pool_last_error(const ah_pool* P) { return P ? P->err.c_str() : ""; }

int ah_pool_destroy(ah_pool* P)
{
    if (!P) return AH_E_INVAL;
    Guard g(P->device);
    if (P->stream) (void)hipStreamSynchronize(P->stream);
    if (P->side) (void)hipStreamSynchronize(P->side);
    for (Retired& r : P->retired) {
        if (r.exec) (void)hipGraphExecDestroy(r.exec);
        if (r.graph) (void)hipGraphDestroy(r.graph);
        if (r.buf) (void)hipFree(r.buf);
        (void)hipEventDestroy(r.ev);
    }
    for (StageChunk& c : P->stage_busy) (void)hipEventDestroy(c.ev);
    for (hipEvent_t ev : P->free_events) (void)hipEventDestroy(ev);
    for (Snapshot& sn : P->snaps) {
        if (sn.h) (void)hipHostFree(sn.h);
        if (sn.ev) (void)hipEventDestroy(sn.ev);
    }
    if (P->stage) (void)hipHostFree(P->stage);
    if (P->side) (void)hipStreamDestroy(P->side);
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->d_work) (void)hipFree(P->d_work);
    if (P->d_lat) (void)hipFree(P->d_lat);
    if (P->d_counters) (void)hipFree(P->d_counters);
    if (P->arena) (void)hipFree(P->arena);
    if (P->owns_stream) (void)hipStreamDestroy(P->stream);
    delete P;
    return AH_OK;
}

}  // extern "C"
