// Optional per-kernel event timing (include/bgv_profile.h): host-side registry of
// (start, stop) HIP event pairs recorded around library launches.
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bgv_profile.h"
#include "common.h"

namespace bgv {

namespace {
struct Pending {
    hipEvent_t a, b;
};
struct KStat {
    int64_t launches = 0;
    double total_ms = 0.0;
    std::vector<Pending> pending;
};
std::mutex g_mu;
bool g_on = false;
std::map<std::string, KStat> g_stats;
std::vector<hipEvent_t> g_pool;
std::vector<std::string> g_names;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void resolve_all() {
    for (auto &kv : g_stats) {
        for (auto &p : kv.second.pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                kv.second.total_ms += ms;
                kv.second.launches += 1;
            }
            g_pool.push_back(p.a);
            g_pool.push_back(p.b);
        }
        kv.second.pending.clear();
    }
}
}  // namespace

bool prof_on() { return g_on; }

struct Token {
    std::string name;
    hipEvent_t a;
};

void *prof_begin(const char *name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t a = take_event();
    if (!a) return nullptr;
    hipEventRecord(a, s);
    return new Token{name, a};
}

void prof_end(void *token, hipStream_t s) {
    Token *t = static_cast<Token *>(token);
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = take_event();
    if (b) {
        hipEventRecord(b, s);
        g_stats[t->name].pending.push_back({t->a, b});
    } else {
        g_pool.push_back(t->a);
    }
    delete t;
}

}  // namespace bgv

using namespace bgv;

extern "C" void bgv_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
}

extern "C" void bgv_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    resolve_all();
    g_stats.clear();
    g_names.clear();
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
