// Launch-shape autotuner.  A tunable launch offers a few variants (tile shapes,
// work splits); the first time a key (kernel, data type, size class) is met,
// every variant is run once to warm up and then timed over three launches with
// HIP events on the caller's stream, and the fastest is kept.  Size classes
// are quarter octaves (size_class), so meshes of nearby sizes share one timing:
// a server meeting hundreds of sizes would otherwise time every variant for
// each of them.  The timing runs outside the lock; when two threads time one
// key at once, both use the first winner stored, so every launch of a key in
// a process takes the same variant.  Winners are cached for the process and,
// when PBM_TUNE_CACHE names a file, read from and appended to it ("key variant"
// per line) so later processes skip the timing.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <string>

#include "pbm_internal.h"

namespace pbm {

namespace {
std::mutex g_mu;
std::map<std::string, int> g_cache;
bool g_loaded = false;

void load_file()
{
    if (g_loaded) return;
    g_loaded = true;
    const char *path = std::getenv("PBM_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string k;
    int v;
    while (f >> k >> v) g_cache[k] = v;
}
}  // namespace

std::string size_class(long long n)
{
    // round(4 log2 n): classes 19% apart
    const int c = n > 0 ? (int)std::lround(4.0 * std::log2((double)n)) : 0;
    return "c" + std::to_string(c);
}

int autotune_pick(const std::string &key, int nvariants, const std::function<void(int)> &run, hipStream_t st)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_file();
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            if (it->second >= 0 && it->second < nvariants) return it->second;
            g_cache.erase(it);   // a stale or corrupt file entry: time the variants again
        }
    }
    hipEvent_t a, b;
    HIPCHECK(hipEventCreate(&a));
    HIPCHECK(hipEventCreate(&b));
    int best = 0;
    float best_ms = 1e30f;
    for (int v = 0; v < nvariants; ++v) {
        run(v);
        HIPCHECK(hipEventRecord(a, st));
        for (int r = 0; r < 3; ++r) run(v);
        HIPCHECK(hipEventRecord(b, st));
        HIPCHECK(hipEventSynchronize(b));
        float ms = 0.0f;
        HIPCHECK(hipEventElapsedTime(&ms, a, b));
        if (ms < best_ms) { best_ms = ms; best = v; }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::lock_guard<std::mutex> lk(g_mu);
    auto ins = g_cache.emplace(key, best);
    if (ins.second) {
        if (const char *path = std::getenv("PBM_TUNE_CACHE")) {
            std::ofstream f(path, std::ios::app);
            f << key << " " << best << "\n";
        }
    }
    return ins.first->second;
}

}  // namespace pbm
