// Diagnostic kernel timing: when enabled, hot kernels are bracketed by HIP
// events recorded on the caller's stream; durations are summed per kernel name
// when read.  Off by default (no events recorded).
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "timing.hpp"

namespace sph {
namespace {

struct Slot {
    std::string name;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    size_t used = 0;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Slot> g_slots;

Slot &slot(const char *name) {
    for (auto &s : g_slots)
        if (s.name == name) return s;
    g_slots.push_back(Slot{name, {}, 0});
    return g_slots.back();
}

}  // namespace

bool timing_on() { return g_on; }

TimedRegion::TimedRegion(const char *name, hipStream_t s) : stream(s) {
    if (!g_on || !name) return;
    std::lock_guard<std::mutex> lk(g_mu);
    Slot &sl = slot(name);
    if (sl.used == sl.pool.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
        sl.pool.push_back({a, b});
    }
    auto &p = sl.pool[sl.used++];
    start = p.first;
    stop = p.second;
    (void)hipEventRecord(start, stream);
}

TimedRegion::~TimedRegion() {
    if (stop) (void)hipEventRecord(stop, stream);
}

}  // namespace sph

using namespace sph;

extern "C" int sph_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return SPH_OK;
}

extern "C" int sph_timing_read(const char *kernel, double *total_ms, int64_t *launches) {
    clear_error();
    if (!kernel || !total_ms || !launches) return fail(SPH_ERR_INVALID_ARG, "null pointer");
    std::lock_guard<std::mutex> lk(g_mu);
    *total_ms = 0.0;
    *launches = 0;
    for (auto &s : g_slots) {
        if (s.name != kernel) continue;
        for (size_t i = 0; i < s.used; ++i) {
            SPH_HIP_TRY(hipEventSynchronize(s.pool[i].second));
            float ms = 0.f;
            SPH_HIP_TRY(hipEventElapsedTime(&ms, s.pool[i].first, s.pool[i].second));
            *total_ms += ms;
        }
        *launches = (int64_t)s.used;
    }
    return SPH_OK;
}

extern "C" int sph_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &s : g_slots) {
        for (size_t i = 0; i < s.used; ++i) (void)hipEventSynchronize(s.pool[i].second);
        s.used = 0;
    }
    return SPH_OK;
}
