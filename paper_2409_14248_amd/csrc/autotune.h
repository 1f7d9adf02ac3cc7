// autotune.h -- the batched plan's tile-configuration cache: a JSON file of
// the configurations the autotuner chose, keyed by the device architecture,
// the network shape, the dtype, the PDE kind and the instance and point
// counts in powers of two, so that a later plan of the same kind of batch
// reuses the choice instead of timing every candidate again.
#pragma once

#include <stdint.h>

#include <string>

#include "runtime_internal.h"

namespace hrk {

struct TunedCfg {
    int slice_pts;   // points per gradient slice
    int dw_ii;       // inputs per wave of the gradient kernel (0: automatic)
    double ms;       // the measured step time of that choice
};

// Path of the cache file: $HRKAN_AUTOTUNE_CACHE if set (an empty value turns
// the cache off: returns ""), else $XDG_CACHE_HOME/hrkan/autotune.json, else
// $HOME/.cache/hrkan/autotune.json, else "".
std::string tune_cache_path();

// The key of a batch: "<arch>|w=2,32,32,1|G=10|k=3|m=4|dtype=1|S=1|kind=1|inst=2^8|pts=2^23".
std::string tune_key(const char *arch, const NetInfo &ni, int kind, int n_inst, int64_t total_points);

// Look the key up; false if the file or the entry is missing or malformed.
bool tune_lookup(const std::string &path, const std::string &key, TunedCfg *out);

// Add or replace the entry and rewrite the file (written to a temporary file
// and renamed into place, so readers never see a partial file). Failures
// are ignored: the cache only saves time.
void tune_store(const std::string &path, const std::string &key, const TunedCfg &cfg);

}  // namespace hrk
