// autotune.hpp -- measured choice of launch schedules, cached per device and shape.
//
// Entries map a key (device, then the shapes of the work) to the schedule that
// measured fastest.  The cache lives in the process; if GS_AUTOTUNE_CACHE names
// a file, it is read from there on first use and rewritten after every new entry
// (a flat JSON object, written by this file only).  Pointing GS_AUTOTUNE_CACHE at
// another file (or unsetting it) switches to that file's entries (or to an empty
// cache in the process).
#pragma once

#include <string>

namespace gsapi {

// Batch entries: the schedule, task size, task order and grid.  Plan entries reuse
// the fields: schedule = cache-hint bits of the passes, tiles_per_task = rounds of
// co-resident blocks of the fused pass.
struct TuneEntry {
    int schedule = 0, tiles_per_task = 1, largest_first = 1, grid = 0;
    double ms = 0.0;
};

// Identifies the device: architecture name and compute-unit count.
std::string tune_device_key(int device);
bool tune_lookup(const std::string& key, TuneEntry& e);
void tune_store(const std::string& key, const TuneEntry& e);

}  // namespace gsapi
