// Autotuner support: a process-wide cache of tuned launch parameters, keyed
// by operation and shape, optionally persisted to the text file named by
// SV_TUNE_CACHE (one "key v0 v1 ..." line per entry), and a stream timer.
// SV_AUTOTUNE=0 disables tuning (defaults are used).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "sv_internal.h"

namespace sv {

int default_max_local(sv_dtype dt) { return dt == SV_C128 ? 12 : 13; }

static std::mutex g_tmu;
static std::map<std::string, std::vector<int>> g_tune;
static bool g_loaded = false;

static void load_file() {
    if (g_loaded) return;
    g_loaded = true;
    const char *path = getenv("SV_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        std::istringstream is(line);
        std::string key;
        if (!(is >> key)) continue;
        std::vector<int> v;
        int x;
        while (is >> x) v.push_back(x);
        g_tune[key] = v;
    }
    fclose(f);
}

bool autotune_enabled() {
    const char *e = getenv("SV_AUTOTUNE");
    return !(e && e[0] == '0');
}

bool tune_lookup(const std::string &key, std::vector<int> &out) {
    std::lock_guard<std::mutex> lk(g_tmu);
    load_file();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    out = it->second;
    return true;
}

void tune_store(const std::string &key, const std::vector<int> &v) {
    std::lock_guard<std::mutex> lk(g_tmu);
    load_file();
    g_tune[key] = v;
    const char *path = getenv("SV_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    for (auto &kv : g_tune) {
        fprintf(f, "%s", kv.first.c_str());
        for (int x : kv.second) fprintf(f, " %d", x);
        fprintf(f, "\n");
    }
    fclose(f);
}

sv_status time_stream(hipStream_t st, int reps, float *ms_out, const std::function<sv_status()> &fn) {
    hipEvent_t e0, e1;
    SV_HIP(hipEventCreate(&e0));
    SV_HIP(hipEventCreate(&e1));
    sv_status s = fn();   // warm-up
    if (s == SV_OK) {
        hipEventRecord(e0, st);
        for (int i = 0; i < reps && s == SV_OK; ++i) s = fn();
        hipEventRecord(e1, st);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        *ms_out = ms / reps;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return s;
}

}  // namespace sv

using namespace sv;

extern "C" sv_status sv_tune_set(const char *key, const int *vals, int n) {
    if (!key || !key[0] || n < 0 || (n > 0 && !vals)) return fail(SV_EINVAL, "bad tuning entry");
    std::lock_guard<std::mutex> lk(g_tmu);
    load_file();
    if (n == 0) g_tune.erase(key);
    else g_tune[key] = std::vector<int>(vals, vals + n);
    return SV_OK;
}

extern "C" int sv_tune_report(char *buf, int len) {
    std::lock_guard<std::mutex> lk(g_tmu);
    std::string out;
    for (auto &kv : g_tune) {
        out += kv.first;
        for (int x : kv.second) out += " " + std::to_string(x);
        out += "\n";
    }
    if (buf && len > 0) {
        strncpy(buf, out.c_str(), (size_t)len - 1);
        buf[len - 1] = 0;
    }
    return (int)out.size();
}
