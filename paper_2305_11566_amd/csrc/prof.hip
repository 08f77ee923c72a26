// Optional per-stage timing with HIP events, recorded on the stream each
// kernel is launched on (for the benchmark's roofline figures).
#include <atomic>
#include <mutex>
#include <vector>

#include "prof.h"

namespace sv {

static std::mutex g_mu;
static std::atomic<bool> g_on{false};
static std::atomic<int> g_rep{1};
static int g_max = 0;
static std::vector<hipEvent_t> g_ev[PROF_NSTAGES];  // 2 * max per stage
static int g_count[PROF_NSTAGES];                   // event pairs recorded
static int g_launches[PROF_NSTAGES];                // launches inside them

static void free_events() {
    for (int s = 0; s < PROF_NSTAGES; ++s) {
        for (hipEvent_t e : g_ev[s]) (void)hipEventDestroy(e);
        g_ev[s].clear();
        g_count[s] = 0;
        g_launches[s] = 0;
    }
}

void prof_mark(int stage, int which, hipStream_t st) {
    if (!g_on.load()) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on.load() || stage < 0 || stage >= PROF_NSTAGES) return;
    const int i = g_count[stage];
    if (i >= g_max) return;
    (void)hipEventRecord(g_ev[stage][2 * i + which], st);
    if (which == 1) {
        g_count[stage] = i + 1;
        g_launches[stage] += g_rep.load();
    }
}

int prof_repeat() { return g_on.load() ? g_rep.load() : 1; }

}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_profile_enable(int max_calls) {
    std::lock_guard<std::mutex> lk(g_mu);
    free_events();
    g_on = false;
    if (max_calls <= 0) return SV_OK;
    if (max_calls > 4096) return SV_ERR_RANGE;
    for (int s = 0; s < PROF_NSTAGES; ++s) {
        g_ev[s].resize(2 * (size_t)max_calls);
        for (auto &e : g_ev[s]) SV_HIP(hipEventCreate(&e));
    }
    g_max = max_calls;
    g_on = true;
    return SV_OK;
}

sv_status sv_profile_repeat(int repeat) {
    if (repeat < 1 || repeat > 64) return SV_ERR_RANGE;
    std::lock_guard<std::mutex> lk(g_mu);
    g_rep = repeat;
    return SV_OK;
}

sv_status sv_profile_read(float *ms_sum, int *counts) {
    if (!ms_sum || !counts) return SV_ERR_NULL;
    std::lock_guard<std::mutex> lk(g_mu);
    for (int s = 0; s < PROF_NSTAGES; ++s) {
        float tot = 0.f;
        for (int i = 0; i < g_count[s]; ++i) {
            SV_HIP(hipEventSynchronize(g_ev[s][2 * i + 1]));
            float ms = 0.f;
            SV_HIP(hipEventElapsedTime(&ms, g_ev[s][2 * i], g_ev[s][2 * i + 1]));
            tot += ms;
        }
        ms_sum[s] = tot;
        counts[s] = g_launches[s];
        g_count[s] = 0;
        g_launches[s] = 0;
    }
    return SV_OK;
}

}  // extern "C"
