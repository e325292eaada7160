// Internal declarations shared by the HIP sources of libsv.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/sv.h"

struct sv_state_s {
    int n = 0;
    sv_dtype dt = SV_C64;
    void *data = nullptr;
    bool owned = false;
    hipStream_t stream = nullptr;
    int device = 0;
    // grow-only device scratch arenas owned by the handle
    void *scratch = nullptr;      // large: GEMM outputs, staged host data
    size_t scratch_bytes = 0;
    void *small = nullptr;        // small: reduction partials, tables, descriptors
    size_t small_bytes = 0;
    void *pinned = nullptr;       // pinned host staging
    size_t pinned_bytes = 0;
};

namespace sv {

// ---- error reporting ---------------------------------------------------
sv_status fail(sv_status code, const char *fmt, ...);
sv_status hip_fail(hipError_t e, const char *what);
void clear_error();

#define SV_HIP(call)                                   \
    do {                                               \
        hipError_t _e = (call);                        \
        if (_e != hipSuccess) return sv::hip_fail(_e, #call); \
    } while (0)

#define SV_TRY(call)                                   \
    do {                                               \
        sv_status _s = (call);                         \
        if (_s != SV_OK) return _s;                    \
    } while (0)

// ---- device buffers owned by a state --------------------------------------
sv_status ensure_scratch(sv_state s, size_t bytes);
sv_status ensure_small(sv_state s, size_t bytes);
sv_status ensure_pinned(sv_state s, size_t bytes);
// host -> device copy of borrowed host memory; completes before returning
sv_status upload(sv_state s, void *dst, const void *src, size_t bytes);
sv_status download(sv_state s, void *dst, const void *src, size_t bytes);

inline size_t amp_bytes(sv_dtype dt) { return dt == SV_C128 ? 16 : 8; }
inline uint64_t dim_of(int n) { return (uint64_t)1 << n; }

// ---- validation helpers -----------------------------------------------
sv_status check_state(sv_state s);
sv_status check_qubits(sv_state s, const int *qs, int nq, const int *ctrls, const int *ctrl_vals,
                       int n_ctrls, uint64_t *cmask, uint64_t *cval);

// ---- launchers used across files -----------------------------------------
// FP64 sum of |a_i|^2 over (i & mask) == value, result left in device memory at *dev_out
sv_status norm2_device(sv_state s, uint64_t mask, uint64_t value, double *dev_out);
// in-place bit reversal of the register [lo, lo+m)
sv_status bitrev_register(sv_state s, int lo, int m, uint64_t fix_mask, uint64_t fix_val);

// ---- fused passes (sv_fused.hip) ---------------------------------------
struct QftSpec {
    int lo, m;
    int inverse;       // 0: cascade (natural in -> bit-reversed out); 1: its inverse
    uint64_t fix_mask, fix_val;  // restrict the transform to indices with (i & fix_mask) == fix_val
};
sv_status run_qft_cascade(sv_state s, const QftSpec &q, int max_local);
sv_status run_hadamards(sv_state s, int lo, int m, uint64_t fix_mask, uint64_t fix_val);

// ---- tuning (sv_tune.cpp) ---------------------------------------------------
int default_max_local(sv_dtype dt);
bool autotune_enabled();
bool tune_lookup(const std::string &key, std::vector<int> &out);
void tune_store(const std::string &key, const std::vector<int> &v);
// mean duration of fn() over `reps` runs on stream st (after one warm-up run)
sv_status time_stream(hipStream_t st, int reps, float *ms_out, const std::function<sv_status()> &fn);

// ---- per-kernel tracing (sv_trace.cpp) ------------------------------------
bool trace_on();
bool trace_set(bool on);   // returns the previous setting
class TraceScope {
  public:
    TraceScope(hipStream_t st, const char *name, double bytes, double flops);
    ~TraceScope();

  private:
    hipStream_t st_;
    const char *name_;
    double bytes_, flops_;
    hipEvent_t e0_ = nullptr;
};

// bit deposit helpers (host)
inline int popcount64(uint64_t x) { return __builtin_popcountll(x); }

}  // namespace sv
