// Per-kernel event tracing: while enabled, launches wrapped in a TraceScope
// are bracketed by HIP events on their own stream, together with the
// algorithmic bytes and flops of that launch.  sv_trace_report aggregates
// durations by kernel name.
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sv_internal.h"

namespace sv {

struct TRec {
    const char *name;
    double bytes, flops;
    hipEvent_t e0, e1;
};

static std::mutex g_mu;
static bool g_on = false;
static std::vector<TRec> g_recs;
static std::vector<hipEvent_t> g_pool;

bool trace_on() { return g_on; }

bool trace_set(bool on) {
    std::lock_guard<std::mutex> lk(g_mu);
    const bool was = g_on;
    g_on = on;
    return was;
}

static hipEvent_t get_event() {
    hipEvent_t e = nullptr;
    if (!g_pool.empty()) {
        e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

TraceScope::TraceScope(hipStream_t st, const char *name, double bytes, double flops)
    : st_(st), name_(name), bytes_(bytes), flops_(flops) {
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    e0_ = get_event();
    if (e0_) hipEventRecord(e0_, st_);
}

TraceScope::~TraceScope() {
    if (!e0_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t e1 = get_event();
    if (!e1) return;
    hipEventRecord(e1, st_);
    g_recs.push_back({name_, bytes_, flops_, e0_, e1});
}

static void recycle() {
    for (auto &r : g_recs) {
        g_pool.push_back(r.e0);
        g_pool.push_back(r.e1);
    }
    g_recs.clear();
}

}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_trace_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (on) {
        hipDeviceSynchronize();
        recycle();
    }
    g_on = on != 0;
    return SV_OK;
}

int sv_trace_report(char *buf, int len) {
    std::lock_guard<std::mutex> lk(g_mu);
    hipDeviceSynchronize();
    struct Agg {
        int n = 0;
        double ms = 0, bytes = 0, flops = 0;
    };
    std::map<std::string, Agg> agg;
    for (auto &r : g_recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) continue;
        Agg &a = agg[r.name];
        a.n += 1;
        a.ms += ms;
        a.bytes += r.bytes;
        a.flops += r.flops;
    }
    std::string out;
    char line[256];
    for (auto &kv : agg) {
        snprintf(line, sizeof line, "%s %d %.6f %.6e %.6e\n", kv.first.c_str(), kv.second.n, kv.second.ms,
                 kv.second.bytes, kv.second.flops);
        out += line;
    }
    if (buf && len > 0) {
        strncpy(buf, out.c_str(), (size_t)len - 1);
        buf[len - 1] = 0;
    }
    return (int)out.size();
}

}  // extern "C"
