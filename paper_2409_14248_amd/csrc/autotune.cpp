// autotune.cpp -- the batched plan's tile-configuration cache (autotune.h).
//
// File format (valid JSON, one entry per line so that it is read back with
// a line scanner; no other JSON is accepted):
//   {
//     "hrkan_autotune": 1,
//     "entries": {
//       "<key>": {"slice_pts": 1024, "dw_ii": 0, "ms": 36.9},
//       ...
//     }
//   }
#include "autotune.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <sys/stat.h>
#include <unistd.h>

namespace hrk {

namespace {

std::mutex g_mu;

int log2_ceil(int64_t v)
{
    int e = 0;
    while (((int64_t)1 << e) < v && e < 62) ++e;
    return e;
}

// Every entry of the file, key -> line fields.
std::map<std::string, TunedCfg> read_all(const std::string &path)
{
    std::map<std::string, TunedCfg> m;
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return m;
    char line[1024];
    while (fgets(line, sizeof line, f)) {
        const char *q0 = strchr(line, '"');
        if (!q0) continue;
        const char *q1 = strchr(q0 + 1, '"');
        if (!q1) continue;
        const char *body = strstr(q1, "{\"slice_pts\":");
        if (!body) continue;
        TunedCfg c{};
        if (sscanf(body, "{\"slice_pts\": %d, \"dw_ii\": %d, \"ms\": %lf}", &c.slice_pts, &c.dw_ii, &c.ms) != 3)
            continue;
        m[std::string(q0 + 1, q1)] = c;
    }
    fclose(f);
    return m;
}

void make_dirs(const std::string &path)
{
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
}

}  // namespace

std::string tune_cache_path()
{
    if (const char *e = getenv("HRKAN_AUTOTUNE_CACHE")) return std::string(e);
    if (const char *x = getenv("XDG_CACHE_HOME"); x && *x) return std::string(x) + "/hrkan/autotune.json";
    if (const char *h = getenv("HOME"); h && *h) return std::string(h) + "/.cache/hrkan/autotune.json";
    return std::string();
}

std::string tune_key(const char *arch, const NetInfo &ni, int kind, int n_inst, int64_t total_points)
{
    std::string k = arch && *arch ? arch : "unknown";
    // the architecture name may carry feature suffixes ("gfx950:sramecc+:xnack-"); keep them
    for (char &ch : k)
        if (ch == '"' || ch == '|' || ch == '\\') ch = '_';
    k += "|w=";
    for (int l = 0; l <= ni.L; ++l) k += (l ? "," : "") + std::to_string(ni.w[l]);
    k += "|G=" + std::to_string(ni.G) + "|k=" + std::to_string(ni.k) + "|m=" + std::to_string(ni.m);
    k += "|dtype=" + std::to_string(ni.dtype) + "|S=" + std::to_string(ni.S) + "|kind=" + std::to_string(kind);
    k += "|inst=2^" + std::to_string(log2_ceil(n_inst)) + "|pts=2^" + std::to_string(log2_ceil(total_points));
    return k;
}

bool tune_lookup(const std::string &path, const std::string &key, TunedCfg *out)
{
    if (path.empty()) return false;
    std::lock_guard<std::mutex> lock(g_mu);
    const auto m = read_all(path);
    const auto it = m.find(key);
    if (it == m.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const std::string &path, const std::string &key, const TunedCfg &cfg)
{
    if (path.empty()) return;
    std::lock_guard<std::mutex> lock(g_mu);
    auto m = read_all(path);
    m[key] = cfg;
    make_dirs(path);
    const std::string tmp = path + ".tmp." + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n  \"hrkan_autotune\": 1,\n  \"entries\": {\n");
    size_t i = 0;
    for (const auto &kv : m) {
        fprintf(f, "    \"%s\": {\"slice_pts\": %d, \"dw_ii\": %d, \"ms\": %.6g}%s\n", kv.first.c_str(),
                kv.second.slice_pts, kv.second.dw_ii, kv.second.ms, ++i < m.size() ? "," : "");
    }
    fprintf(f, "  }\n}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path.c_str()) != 0) (void)unlink(tmp.c_str());
}

}  // namespace hrk
