// Autotuner of libah: picks the kernel (one step per pass, or two), the tile
// shape and the z-chunk of the tiled step for a (precision, N) by timing
// candidates on a scratch lattice, and keeps the choices in a process-wide
// table that can be saved to and loaded from a small JSON file (one entry
// per line).
#include "ah.h"
#include "ah_internal.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

namespace {

struct Entry {
    ah_step_config cfg;
    double ms;
};
std::mutex g_mu;
std::map<std::pair<int, int>, Entry> g_table;  // (precision, N) -> choice

}  // namespace

namespace ah {
// A table entry names a supported tile shape for its precision and a z-chunk
// that is automatic (0) or at least the minimum.
static bool valid_entry(int precision, int N, const ah_step_config& c)
{
    const bool shape = c.kernel == AH_KERNEL_TILE    ? tile_supported(precision, c.tile_x, c.tile_y)
                       : c.kernel == AH_KERNEL_TILE2 ? tile2_supported(precision, c.tile_x, c.tile_y)
                                                     : false;
    return (precision == AH_FP32 || precision == AH_FP64) && N >= 4 && shape && c.zchunk >= 0 &&
           (c.zchunk == 0 || c.zchunk >= min_zchunk(N));
}

bool tuned_config(const ah_params& p, ah_step_config* out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find({p.precision, p.N});
    if (it == g_table.end()) return false;
    *out = it->second.cfg;
    if (out->zchunk > p.N) out->zchunk = p.N;
    return true;
}
}  // namespace ah

using ah::no_throw;

extern "C" {

int ah_autotune(const ah_params* p, int32_t steps, ah_step_config* best, double* best_ms)
{
    return no_throw([&]() -> int {
        if (!p || steps <= 0) return AH_E_INVAL;
        if (p->gauge_action != AH_COMPACT) return AH_E_INVAL;
        ah_handle* h = nullptr;
        int rc = ah_create(p, nullptr, 0, nullptr, &h);
        if (rc != AH_OK) return rc;
        rc = ah_init(h, 0);
        // (kernel, tile x, tile y): single steps on every tile shape, two-step
        // passes on theirs (timed per step)
        std::vector<std::tuple<int, int, int>> shapes = {{AH_KERNEL_TILE, 64, 8}, {AH_KERNEL_TILE, 64, 4},
                                                         {AH_KERNEL_TILE, 32, 8}, {AH_KERNEL_TILE, 128, 4},
                                                         {AH_KERNEL_TILE2, 32, 8}, {AH_KERNEL_TILE2, 64, 4}};
        if (p->precision == AH_FP32) {
            shapes.push_back({AH_KERNEL_TILE, 64, 16});
            shapes.push_back({AH_KERNEL_TILE, 128, 8});
            shapes.push_back({AH_KERNEL_TILE2, 64, 8});
        }
        // the automatic z-chunk and equal chunks of 1 .. 32 per column
        std::vector<int> zcs = {0};
        for (int nz : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32}) {
            const int zc = (p->N + nz - 1) / nz;
            if (zc >= ah::min_zchunk(p->N) && std::find(zcs.begin(), zcs.end(), zc) == zcs.end()) zcs.push_back(zc);
        }
        ah_step_config bcfg{};
        double bms = 1e300;
        for (auto& t : shapes) {
            for (int zc : zcs) {
                if (rc != AH_OK) break;
                ah_step_config c{std::get<0>(t), std::get<1>(t), std::get<2>(t), zc};
                if (ah_set_step_config(h, &c) != AH_OK) continue;
                rc = ah_step(h, 2);
                if (rc == AH_OK) rc = ah_set_timing(h, 1);
                if (rc == AH_OK) rc = ah_step(h, steps);
                double ms = 0.0;
                int64_t n = 0;
                if (rc == AH_OK) rc = ah_get_timing(h, &ms, &n);
                if (rc == AH_OK) rc = ah_set_timing(h, 0);
                if (rc == AH_OK && n > 0 && ms / n < bms) {
                    bms = ms / n;
                    (void)ah_get_step_config(h, &bcfg);
                }
            }
        }
        ah_destroy(h);
        if (rc != AH_OK) return rc;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            g_table[{p->precision, p->N}] = Entry{bcfg, bms};
        }
        if (best) *best = bcfg;
        if (best_ms) *best_ms = bms;
        return AH_OK;
    });
}

int ah_tune_lookup(const ah_params* p, ah_step_config* out)
{
    return no_throw([&]() -> int {
        if (!p || !out) return AH_E_INVAL;
        return ah::tuned_config(*p, out) ? AH_OK : AH_E_AGAIN;
    });
}

int ah_tune_set(const ah_params* p, const ah_step_config* c)
{
    return no_throw([&]() -> int {
        if (!p || !c) return AH_E_INVAL;
        if (!ah::valid_entry(p->precision, p->N, *c)) return AH_E_INVAL;
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[{p->precision, p->N}] = Entry{*c, 0.0};
        return AH_OK;
    });
}

int ah_tune_clear(void)
{
    return no_throw([&]() -> int {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table.clear();
        return AH_OK;
    });
}

int ah_tune_save(const char* path)
{
    return no_throw([&]() -> int {
        if (!path) return AH_E_INVAL;
        FILE* f = std::fopen(path, "w");
        if (!f) return AH_E_INVAL;
        std::lock_guard<std::mutex> lk(g_mu);
        std::fprintf(f, "{\"version\": 1, \"entries\": [\n");
        size_t i = 0;
        for (auto& kv : g_table) {
            std::fprintf(f,
                         "{\"precision\": \"%s\", \"N\": %d, \"tile_x\": %d, \"tile_y\": %d, \"zchunk\": %d, "
                         "\"ms\": %.6g, \"kernel\": \"%s\"}%s\n",
                         kv.first.first == AH_FP64 ? "fp64" : "fp32", kv.first.second, kv.second.cfg.tile_x,
                         kv.second.cfg.tile_y, kv.second.cfg.zchunk, kv.second.ms,
                         kv.second.cfg.kernel == AH_KERNEL_TILE2 ? "tile2" : "tile", ++i < g_table.size() ? "," : "");
        }
        std::fprintf(f, "]}\n");
        std::fclose(f);
        return AH_OK;
    });
}

int ah_tune_load(const char* path)
{
    return no_throw([&]() -> int {
        if (!path) return AH_E_INVAL;
        FILE* f = std::fopen(path, "r");
        if (!f) return AH_E_INVAL;
        // every entry line is checked before any is taken: a file with a bad
        // entry changes nothing
        char line[512];
        std::vector<std::pair<std::pair<int, int>, Entry>> got;
        bool bad = false;
        while (std::fgets(line, sizeof(line), f)) {
            if (!std::strstr(line, "\"precision\"")) continue;
            char prec[8] = {0};
            int N, tx, ty, zc;
            double ms;
            if (std::sscanf(line, " {\"precision\": \"%7[a-z0-9]\", \"N\": %d, \"tile_x\": %d, \"tile_y\": %d, \"zchunk\": %d, \"ms\": %lf",
                            prec, &N, &tx, &ty, &zc, &ms) != 6) {
                bad = true;
                continue;
            }
            const int pr = std::strcmp(prec, "fp64") == 0 ? AH_FP64 : (std::strcmp(prec, "fp32") == 0 ? AH_FP32 : -1);
            // an entry without a kernel field is a single-step one
            const int kern = std::strstr(line, "\"kernel\": \"tile2\"") ? AH_KERNEL_TILE2 : AH_KERNEL_TILE;
            const ah_step_config c{kern, tx, ty, zc};
            if (!ah::valid_entry(pr, N, c)) {
                bad = true;
                continue;
            }
            got.push_back({{pr, N}, Entry{c, ms}});
        }
        std::fclose(f);
        if (bad) return AH_E_INVAL;
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto& kv : got) g_table[kv.first] = kv.second;
        return AH_OK;
    });
}

}  // extern "C"
