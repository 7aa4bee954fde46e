// Optional per-kernel timing: when enabled, every kernel the library launches
// is bracketed by a pair of HIP events recorded on its own stream, and
// tqp_profile_collect() turns the pairs into per-kernel launch counts and
// total milliseconds.  Disabled (the default) it costs one branch per launch.
#include <mutex>
#include <string>
#include <vector>
#include <stdio.h>
#include <string.h>

#include "tqp_internal.hpp"

namespace tqp {

namespace {
struct Pending {
    const char *name;
    hipEvent_t a, b;
};
struct Acc {
    std::string name;
    long long count;
    double ms;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::vector<Acc> g_acc;

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
}  // namespace

bool profile_on() { return g_on; }

ProfScope::ProfScope(const char *name, hipStream_t s) : name_(name), s_(s) {
    if (!g_on) return;
    std::lock_guard<std::mutex> g(g_mu);
    a_ = take_event();
    b_ = take_event();
    if (a_) (void)hipEventRecord(a_, s_);
}

ProfScope::~ProfScope() {
    if (!a_ || !b_) return;
    (void)hipEventRecord(b_, s_);
    std::lock_guard<std::mutex> g(g_mu);
    g_pending.push_back({name_, a_, b_});
}

}  // namespace tqp

using namespace tqp;

TQP_API void tqp_profile_enable(int on) {
    std::lock_guard<std::mutex> g(g_mu);
    g_on = on != 0;
}

TQP_API void tqp_profile_reset(void) {
    std::lock_guard<std::mutex> g(g_mu);
    for (auto &p : g_pending) {
        (void)hipEventSynchronize(p.b);
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
    g_acc.clear();
}

TQP_API int tqp_profile_collect(char *buf, size_t len) {
    std::lock_guard<std::mutex> g(g_mu);
    for (auto &p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            bool found = false;
            for (auto &a : g_acc)
                if (a.name == p.name) {
                    a.count++;
                    a.ms += ms;
                    found = true;
                    break;
                }
            if (!found) g_acc.push_back({p.name, 1, double(ms)});
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
    std::string out;
    char line[256];
    for (auto &a : g_acc) {
        snprintf(line, sizeof line, "%s %lld %.6f\n", a.name.c_str(), a.count, a.ms);
        out += line;
    }
    if (buf && len > 0) {
        size_t k = out.size() < len - 1 ? out.size() : len - 1;
        memcpy(buf, out.data(), k);
        buf[k] = 0;
    }
    return int(out.size() + 1);
}
