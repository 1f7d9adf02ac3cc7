// profile.cpp -- optional per-kernel timing with HIP events.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "runtime_internal.h"

namespace hrk {

namespace {
struct Rec {
    std::string name;
    hipEvent_t a, b;
};
bool g_on = false;
std::vector<Rec> g_recs;
}  // namespace

bool prof_on() { return g_on; }

ProfScope::ProfScope(const char *name, int layer, hipStream_t st, bool bc) : st_(st), idx_(-1)
{
    if (!g_on) return;
    Rec r;
    r.name = layer >= 0 ? std::string(name) + "_l" + std::to_string(layer) : std::string(name);
    if (bc) r.name += "_bc";
    if (hipEventCreate(&r.a) != hipSuccess) return;
    if (hipEventCreate(&r.b) != hipSuccess) {
        (void)hipEventDestroy(r.a);
        return;
    }
    (void)hipEventRecord(r.a, st);
    g_recs.push_back(r);
    idx_ = (int)g_recs.size() - 1;
}

ProfScope::~ProfScope()
{
    if (idx_ >= 0) (void)hipEventRecord(g_recs[idx_].b, st_);
}

}  // namespace hrk

using namespace hrk;

extern "C" {

int hrkan_profile_enable(int32_t on)
{
    g_on = on != 0;
    return HRKAN_OK;
}

int hrkan_profile_read(char *buf, size_t buflen)
{
    if (!buf || buflen == 0) return fail(HRKAN_ERR_INVALID_ARG, "buf is NULL or empty");
    std::map<std::string, std::pair<long, double>> agg;
    int rc = HRKAN_OK;
    for (auto &r : g_recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) rc = hip_fail(e, "profile event");
        auto &v = agg[r.name];
        v.first += 1;
        v.second += ms;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_recs.clear();
    std::string out;
    char line[160];
    for (auto &kv : agg) {
        snprintf(line, sizeof line, "%s %ld %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
        out += line;
    }
    snprintf(buf, buflen, "%s", out.c_str());
    return rc;
}

}  // extern "C"
