// autotune.cpp -- the schedule cache (autotune.hpp).
#include "autotune.hpp"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

namespace gsapi {

namespace {

std::mutex g_mu;
std::map<std::string, TuneEntry> g_cache;
std::string g_loaded_from = "\x01";     // file the cache was last merged from ("" = none)

const char* cache_path() {
    const char* p = std::getenv("GS_AUTOTUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// When GS_AUTOTUNE_CACHE names another file than last time (or none), the cache
// switches to it: the entries held so far are dropped and those of the file are
// read, as written by save(): one per line,
//   "key": {"schedule": S, "tiles_per_task": T, "largest_first": F, "grid": G, "ms": M},
void load() {
    const char* path = cache_path();
    const std::string now = path ? path : "";
    if (now == g_loaded_from) return;
    g_loaded_from = now;
    g_cache.clear();
    if (!path) return;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        const size_t q0 = line.find('"');
        const size_t q1 = (q0 == std::string::npos) ? q0 : line.find('"', q0 + 1);
        const size_t br = (q1 == std::string::npos) ? q1 : line.find('{', q1);
        if (br == std::string::npos) continue;
        TuneEntry e;
        if (std::sscanf(line.c_str() + br,
                        "{\"schedule\": %d, \"tiles_per_task\": %d, \"largest_first\": %d, \"grid\": %d, \"ms\": %lf}",
                        &e.schedule, &e.tiles_per_task, &e.largest_first, &e.grid, &e.ms) == 5)
            g_cache[line.substr(q0 + 1, q1 - q0 - 1)] = e;
    }
}

void save() {
    const char* path = cache_path();
    if (!path) return;
    std::ostringstream os;
    os << "{\n";
    size_t i = 0;
    for (const auto& [k, e] : g_cache) {
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "{\"schedule\": %d, \"tiles_per_task\": %d, \"largest_first\": %d, \"grid\": %d, \"ms\": %.6g}",
                      e.schedule, e.tiles_per_task, e.largest_first, e.grid, e.ms);
        os << "  \"" << k << "\": " << buf << (++i < g_cache.size() ? ",\n" : "\n");
    }
    os << "}\n";
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out) return;
        out << os.str();
    }
    std::rename(tmp.c_str(), path);
}

}  // namespace

std::string tune_device_key(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return arch + "/cu" + std::to_string(prop.multiProcessorCount);
}

bool tune_lookup(const std::string& key, TuneEntry& e) {
    std::lock_guard<std::mutex> g(g_mu);
    load();
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return false;
    e = it->second;
    return true;
}

void tune_store(const std::string& key, const TuneEntry& e) {
    std::lock_guard<std::mutex> g(g_mu);
    load();
    g_cache[key] = e;
    save();
}

}  // namespace gsapi
