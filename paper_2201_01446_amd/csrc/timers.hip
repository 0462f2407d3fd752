// timers.hip -- optional per-kernel timing with HIP events recorded on the
// stream each kernel is launched on (off by default; see dp_timers_enable).

#include "dp_internal.h"

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace dp {

namespace {
struct Rec {
    const char *name;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
thread_local bool t_quiet = false;   // no events from this thread (dp_compute_noalloc)

hipEvent_t get_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

TimerScope::TimerScope(const char *name, hipStream_t st) : name_(name), st_(st)
{
    if (t_quiet) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    a_ = get_event();
    b_ = get_event();
    if (a_ && b_) (void)hipEventRecord(a_, st_);
}

TimerScope::~TimerScope()
{
    if (!a_ || !b_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipEventRecord(b_, st_);
    g_recs.push_back(Rec{name_, a_, b_});
}

void timers_quiet(bool on) { t_quiet = on; }

}  // namespace dp

using namespace dp;

extern "C" {

dp_status dp_timers_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return DP_OK;
}

dp_status dp_timers_read(int max_names, char *names, double *total_ms, int *counts, int *n_names)
{
    std::lock_guard<std::mutex> lk(g_mu);
    std::map<std::string, std::pair<double, int>> agg;
    for (Rec &r : g_recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "timer event");
        auto &v = agg[r.name];
        v.first += ms;
        v.second += 1;
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    int k = 0;
    for (auto &kv : agg) {
        if (k >= max_names) break;
        if (names) {
            std::strncpy(names + 32 * k, kv.first.c_str(), 31);
            names[32 * k + 31] = 0;
        }
        if (total_ms) total_ms[k] = kv.second.first;
        if (counts) counts[k] = kv.second.second;
        k++;
    }
    if (n_names) *n_names = k;
    return DP_OK;
}

}  // extern "C"
