// tune.hip -- the autotuner of the step kernels' tile shape.
//
// Every candidate shape is timed on the caller's own lattice(s) with launches
// that read the current buffer and write the other one without swapping them,
// so tuning never changes the state (and results do not depend on the shape
// anyway). The fastest shape is applied and remembered per (GPU architecture,
// form, dtype, size): in memory for the process, and, when the environment
// variable LBM_TUNE_CACHE names a file, in that file as one JSON object per
// line (later lines override earlier ones).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "host.h"
#include "tune.h"

namespace lbm {

namespace {

std::mutex g_mu;
std::map<std::string, TileCand> g_cache;
bool g_loaded = false;

const char* cache_path() { return std::getenv("LBM_TUNE_CACHE"); }

void load_cache_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char* p = cache_path();
    if (!p) return;
    FILE* f = std::fopen(p, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        char key[256];
        TileCand c{};
        float us = 0;
        if (std::sscanf(line,
                        "{\"key\": \"%255[^\"]\", \"vx\": %d, \"nw\": %d, \"h\": %d, \"flags\": %d, \"ch\": %d, "
                        "\"us\": %f}",
                        key, &c.vx, &c.nw, &c.h, &c.flags, &c.ch, &us) == 7)
            g_cache[key] = c;
    }
    std::fclose(f);
}

}  // namespace

std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

bool tune_cache_get(const std::string& key, TileCand* out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return false;
    *out = it->second;
    return true;
}

void tune_cache_put(const std::string& key, const TileCand& c, float us)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    g_cache[key] = c;
    if (const char* p = cache_path()) {
        if (FILE* f = std::fopen(p, "a")) {
            std::fprintf(f,
                         "{\"key\": \"%s\", \"vx\": %d, \"nw\": %d, \"h\": %d, \"flags\": %d, \"ch\": %d, "
                         "\"us\": %.3f}\n",
                         key.c_str(), c.vx, c.nw, c.h, c.flags, c.ch, us);
            std::fclose(f);
        }
    }
}

std::vector<TileCand> lattice_candidates(int dtype)
{
    std::vector<TileCand> v;
    const int vxs[] = {1, 2, 4};
    const int nws[] = {4, 8, 16};
    for (int vx : vxs)
        for (int nw : nws)
            for (int nts = 0; nts < 2; ++nts)
                v.push_back({vx, nw, 8, LBM_TILE_VSTACK | (nts ? LBM_TILE_NT_STORE : 0), 0});
    // two steps per launch (32-row tiles: one column per lane, 4-byte or
    // smaller storage)
    for (int vx : {1, 2})
        for (int nw : {12, 16, 32})
            for (int nts = 0; nts < 2; ++nts)
                if (nw < 32 || (vx == 1 && dtype != LBM_F64))
                    v.push_back({vx, nw, 8, LBM_TILE_VSTACK | LBM_TILE_TWO_STEP | (nts ? LBM_TILE_NT_STORE : 0), 0});
    // march form: prefetched, row-band order
    for (int vx : {1, 2})
        for (int h : {4, 8})
            for (int f : {LBM_TILE_PREFETCH2 | LBM_TILE_NT_STORE | LBM_TILE_ROWBAND,
                          LBM_TILE_PREFETCH | LBM_TILE_NT_STORE | LBM_TILE_ROWBAND})
                v.push_back({vx, 4, h, f, 0});
    return v;
}

// Batched kernels: vertical-stack shape, non-temporal stores, the tiles per
// work item (carried in the h field) and the items per XCD chunk.
std::vector<TileCand> pool_candidates(int dtype)
{
    std::vector<TileCand> v;
    for (int vx : {1, 2, 4})
        for (int nw : {4, 8, 16})
            for (int nts = 0; nts < 2; ++nts)
                for (int per : {1, 2})
                    for (int ch : {8, 32}) v.push_back({vx, nw, per, nts ? LBM_TILE_NT_STORE : 0, ch});
    // two steps per launch
    for (int vx : {1, 2})
        for (int nw : {12, 16})
            for (int per : {1, 2})
                for (int ch : {8, 32}) v.push_back({vx, nw, per, LBM_TILE_TWO_STEP | LBM_TILE_NT_STORE, ch});
    (void)dtype;
    return v;
}

// Time `reps` launches of each candidate (after two warm-up launches) with
// HIP events on `st`; returns the index of the fastest and its time per
// launch in microseconds. `launch(c)` enqueues one launch of candidate c.
int time_candidates(const std::vector<TileCand>& cands, int reps, hipStream_t st,
                    const std::function<hipError_t(const TileCand&)>& launch, float* best_us)
{
    if (cands.empty()) return -1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
    // Warm the device up first (clocks, caches), then time every candidate
    // in two passes and keep each one's faster pass, so that the order of
    // the candidates does not decide between shapes a few percent apart.
    for (int w = 0; w < std::max(10, 4 * reps); ++w)
        if (launch(cands[0]) != hipSuccess) {
            (void)hipGetLastError();
            break;
        }
    std::vector<float> t(cands.size(), -1.0f);
    for (int pass = 0; pass < 2; ++pass)
        for (size_t k = 0; k < cands.size(); ++k) {
            if (pass > 0 && t[k] < 0) continue;  // unsupported in the first pass
            hipError_t e = launch(cands[k]);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(cands[k]);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                (void)hipGetLastError();  // an unsupported candidate is skipped
                continue;
            }
            const float us = 1e3f * ms / reps;
            if (t[k] < 0 || us < t[k]) t[k] = us;
        }
    // Refine: the few fastest shapes are often within a percent of each
    // other, closer than one short timing resolves; time them again in
    // interleaved rounds and keep the lowest median.
    std::vector<int> order;
    for (size_t k = 0; k < cands.size(); ++k)
        if (t[k] >= 0) order.push_back((int)k);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return t[a] < t[b]; });
    if (order.size() > 4) order.resize(4);
    std::vector<std::vector<float>> rounds(order.size(), std::vector<float>{});
    for (size_t k = 0; k < order.size(); ++k) rounds[k].push_back(t[order[k]]);
    for (int round = 0; round < 3; ++round)
        for (size_t k = 0; k < order.size(); ++k) {
            const TileCand& c = cands[order[k]];
            hipError_t e = launch(c);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(c);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                continue;
            }
            rounds[k].push_back(1e3f * ms / reps);
        }
    int best = -1;
    float best_med = 0.0f;
    for (size_t k = 0; k < order.size(); ++k) {
        std::vector<float> v = rounds[k];
        std::sort(v.begin(), v.end());
        const float med = v[v.size() / 2];
        if (best < 0 || med < best_med) {
            best = order[k];
            best_med = med;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_us) *best_us = best >= 0 ? best_med : 0.0f;
    return best;
}

}  // namespace lbm
