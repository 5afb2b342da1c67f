// Optional per-kernel event timing (include/bgv_profile.h): host-side registry of
// (start, stop) HIP event pairs attached to library launches.  Completed pairs are
// harvested as new events are needed, so the number of live events stays near the
// number of launches in flight instead of growing with the length of the run.
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bgv_profile.h"
#include "common.h"

namespace bgv {

namespace {
struct KStat {
    int64_t launches = 0;
    double total_ms = 0.0;
};
struct Pending {
    KStat *stat;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::string g_filter;  // record only kernels whose name starts with this ("" = all)
int64_t g_every = 1;   // record one in g_every of the launches that pass the filter
int64_t g_seen = 0;
std::map<std::string, KStat> g_stats;
std::deque<Pending> g_pending;  // in launch order
std::vector<hipEvent_t> g_pool;
std::vector<std::string> g_names;
constexpr size_t kMaxEvents = 1024;  // created events before waiting on the oldest pair

size_t g_created = 0;

void harvest(const Pending &p) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        p.stat->total_ms += ms;
        p.stat->launches += 1;
    }
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
}

// Harvest finished pairs from the front (non-blocking), or the oldest one (blocking)
// when the event budget is exhausted.
void reclaim(bool must) {
    while (!g_pending.empty() && hipEventQuery(g_pending.front().b) == hipSuccess) {
        harvest(g_pending.front());
        g_pending.pop_front();
    }
    if (must && g_pool.empty() && !g_pending.empty()) {
        harvest(g_pending.front());
        g_pending.pop_front();
    }
}

hipEvent_t take_event() {
    if (g_pool.empty()) reclaim(g_created >= kMaxEvents);
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ++g_created;
    return e;
}

void resolve_all() {
    while (!g_pending.empty()) {
        harvest(g_pending.front());
        g_pending.pop_front();
    }
}
}  // namespace

bool prof_on() { return g_on; }

bool prof_take(const char *name, ProfPair *p) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_filter.empty() && std::strncmp(name, g_filter.c_str(), g_filter.size()) != 0) return false;
    if (g_every > 1 && (g_seen++ % g_every) != 0) return false;
    hipEvent_t a = take_event();
    if (!a) return false;
    hipEvent_t b = take_event();
    if (!b) {
        g_pool.push_back(a);
        return false;
    }
    p->start = a;
    p->stop = b;
    p->stat = &g_stats[name];
    return true;
}

void prof_commit(const ProfPair &p) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back({static_cast<KStat *>(p.stat), p.start, p.stop});
}

}  // namespace bgv

using namespace bgv;

extern "C" void bgv_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
}

extern "C" void bgv_profile_filter(const char *prefix) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_filter = prefix ? prefix : "";
}

extern "C" void bgv_profile_sample(int every) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_every = every > 1 ? every : 1;
    g_seen = 0;
}

extern "C" void bgv_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    resolve_all();
    g_stats.clear();
    g_names.clear();
    prof_reset_counters();
}

extern "C" int bgv_profile_counter(const char *name, uint64_t *value) {
    if (!name || !value) return -1;
    return prof_read_counter(name, value);
}

extern "C" int bgv_profile_count(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    resolve_all();
    g_names.clear();
    for (auto &kv : g_stats) g_names.push_back(kv.first);
    return (int)g_names.size();
}

extern "C" int bgv_profile_get(int idx, const char **name, int64_t *launches, double *total_ms) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (idx < 0 || idx >= (int)g_names.size()) return -1;
    auto it = g_stats.find(g_names[idx]);
    if (it == g_stats.end()) return -1;
    if (name) *name = g_names[idx].c_str();
    if (launches) *launches = it->second.launches;
    if (total_ms) *total_ms = it->second.total_ms;
    return 0;
}
