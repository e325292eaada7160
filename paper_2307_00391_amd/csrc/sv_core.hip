// State handles, initialisation, one-qubit gates, bit-exact permutations,
// FP64 reductions and post-selection.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

static thread_local std::string g_err;

sv_status fail(sv_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

sv_status hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? SV_ENOMEM : SV_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

static sv_status grow(void **p, size_t *have, size_t need) {
    if (*have >= need) return SV_OK;
    if (*p) {
        SV_HIP(hipFree(*p));
        *p = nullptr;
        *have = 0;
    }
    size_t sz = std::max<size_t>(need, 1 << 16);
    SV_HIP(hipMalloc(p, sz));
    *have = sz;
    return SV_OK;
}

sv_status ensure_scratch(sv_state s, size_t bytes) {
    if (s->scratch_bytes < bytes) SV_HIP(hipStreamSynchronize(s->stream));
    return grow(&s->scratch, &s->scratch_bytes, bytes);
}
sv_status ensure_small(sv_state s, size_t bytes) {
    if (s->small_bytes < bytes) SV_HIP(hipStreamSynchronize(s->stream));
    return grow(&s->small, &s->small_bytes, bytes);
}
sv_status ensure_pinned(sv_state s, size_t bytes) {
    if (s->pinned_bytes >= bytes) return SV_OK;
    SV_HIP(hipStreamSynchronize(s->stream));
    if (s->pinned) SV_HIP(hipHostFree(s->pinned));
    s->pinned = nullptr;
    s->pinned_bytes = 0;
    size_t sz = std::max<size_t>(bytes, 1 << 16);
    SV_HIP(hipHostMalloc(&s->pinned, sz, hipHostMallocDefault));
    s->pinned_bytes = sz;
    return SV_OK;
}

sv_status upload(sv_state s, void *dst, const void *src, size_t bytes) {
    if (!bytes) return SV_OK;
    SV_TRY(ensure_pinned(s, bytes));
    SV_HIP(hipStreamSynchronize(s->stream));   // the staging buffer may still be in use
    memcpy(s->pinned, src, bytes);
    SV_HIP(hipMemcpyAsync(dst, s->pinned, bytes, hipMemcpyHostToDevice, s->stream));
    SV_HIP(hipStreamSynchronize(s->stream));
    return SV_OK;
}

sv_status download(sv_state s, void *dst, const void *src, size_t bytes) {
    if (!bytes) return SV_OK;
    SV_TRY(ensure_pinned(s, bytes));
    SV_HIP(hipMemcpyAsync(s->pinned, src, bytes, hipMemcpyDeviceToHost, s->stream));
    SV_HIP(hipStreamSynchronize(s->stream));
    memcpy(dst, s->pinned, bytes);
    return SV_OK;
}

sv_status check_state(sv_state s) {
    if (!s || !s->data) return fail(SV_EINVAL, "null state");
    return SV_OK;
}

// Validates target qubits qs[0..nq) and controls; returns the control mask/value.
sv_status check_qubits(sv_state s, const int *qs, int nq, const int *ctrls, const int *ctrl_vals,
                       int n_ctrls, uint64_t *cmask, uint64_t *cval) {
    if (n_ctrls < 0 || n_ctrls > 32) return fail(SV_EINVAL, "n_ctrls %d out of range", n_ctrls);
    if (n_ctrls && !ctrls) return fail(SV_EINVAL, "ctrls is NULL");
    uint64_t used = 0, m = 0, v = 0;
    for (int i = 0; i < nq; ++i) {
        if (qs[i] < 0 || qs[i] >= s->n) return fail(SV_EINVAL, "qubit %d out of range [0,%d)", qs[i], s->n);
        if (used >> qs[i] & 1) return fail(SV_EINVAL, "qubit %d repeated", qs[i]);
        used |= 1ull << qs[i];
    }
    for (int i = 0; i < n_ctrls; ++i) {
        int c = ctrls[i];
        if (c < 0 || c >= s->n) return fail(SV_EINVAL, "control %d out of range [0,%d)", c, s->n);
        if (used >> c & 1) return fail(SV_EINVAL, "control %d repeats a gate qubit", c);
        used |= 1ull << c;
        int val = ctrl_vals ? ctrl_vals[i] : 1;
        if (val != 0 && val != 1) return fail(SV_EINVAL, "control value %d not 0/1", val);
        m |= 1ull << c;
        v |= (uint64_t)val << c;
    }
    *cmask = m;
    *cval = v;
    return SV_OK;
}

static Ins make_ins(uint64_t mask, uint64_t val) {
    Ins f;
    memset(&f, 0, sizeof f);
    f.nf = 0;
    for (int q = 0; q < 64; ++q)
        if (mask >> q & 1) f.pos[f.nf++] = (uint8_t)q;
    f.fval = val & mask;
    return f;
}

static inline unsigned grid_for(uint64_t items, int per_thread, int block = 256, unsigned cap = 1u << 20) {
    uint64_t g = (items + (uint64_t)block * per_thread - 1) / ((uint64_t)block * per_thread);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

template <typename R>
__global__ void k_fill_basis(cvec<R> *__restrict__ psi, uint64_t dim, uint64_t index) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride)
        psi[i] = cmake<R>(i == index ? (R)1 : (R)0, (R)0);
}

// psi[i] = b[x] * scale for i = x + 2^n_s y with y < 2^c, all higher bits 0
template <typename R>
__global__ void k_init_b(cvec<R> *__restrict__ psi, uint64_t dim, const double2 *__restrict__ b, int n_s,
                         uint64_t ylimit, double scale) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t xm = (1ull << n_s) - 1ull;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride) {
        cvec<R> z = cmake<R>((R)0, (R)0);
        if ((i >> n_s) < ylimit) {
            const double2 v = b[i & xm];
            z = cmake<R>((R)(v.x * scale), (R)(v.y * scale));
        }
        psi[i] = z;
    }
}

template <typename R>
__global__ void k_from_f64(cvec<R> *__restrict__ psi, const double2 *__restrict__ src, uint64_t count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        psi[i] = cmake<R>((R)src[i].x, (R)src[i].y);
}

template <typename R>
__global__ void k_to_f64(double2 *__restrict__ dst, const cvec<R> *__restrict__ psi, uint64_t count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        dst[i] = make_double2((double)psi[i].x, (double)psi[i].y);
}

enum GateKind { GK_DENSE = 0, GK_X = 1, GK_DIAG = 2, GK_PHASE1 = 3 };

// One-qubit gate on pairs (i0, i0 | tbit); i0 enumerates the indices with the
// target bit 0 and every control bit at its required value.
template <typename R, int KIND>
__global__ __launch_bounds__(256) void k_gate(cvec<R> *__restrict__ psi, uint64_t count, Ins f, uint64_t tbit,
                                              cvec<R> u00, cvec<R> u01, cvec<R> u10, cvec<R> u11) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count; p += stride) {
        const uint64_t i0 = expand(p, f);
        if (KIND == GK_PHASE1) {              // only the |1> amplitude changes: f pins the target to 1
            psi[i0] = cmul<R>(u11, psi[i0]);
            continue;
        }
        const uint64_t i1 = i0 | tbit;
        const cvec<R> a0 = psi[i0], a1 = psi[i1];
        if (KIND == GK_DENSE) {
            psi[i0] = cmac2<R>(u00, a0, u01, a1);
            psi[i1] = cmac2<R>(u10, a0, u11, a1);
        } else if (KIND == GK_X) {
            psi[i0] = a1;
            psi[i1] = a0;
        } else {
            psi[i0] = cmul<R>(u00, a0);
            psi[i1] = cmul<R>(u11, a1);
        }
    }
}

// SWAP of two qubits: f pins q1 = 1, q2 = 0 (and the controls); the partner
// index flips both bits.
template <typename R>
__global__ __launch_bounds__(256) void k_swap(cvec<R> *__restrict__ psi, uint64_t count, Ins f, uint64_t flip) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count; p += stride) {
        const uint64_t i = expand(p, f), j = i ^ flip;
        const cvec<R> a = psi[i], b = psi[j];
        psi[i] = b;
        psi[j] = a;
    }
}

// Per-block FP64 partial sums of |psi_i|^2 over the enumerated subspace.  Each
// block owns a contiguous chunk of the enumeration, so the summation order
// (and therefore the result) depends only on the sizes.
template <typename R>
__global__ __launch_bounds__(256) void k_norm_partial(const cvec<R> *__restrict__ psi, uint64_t count,
                                                      uint64_t chunk, Ins f, double *__restrict__ part) {
    __shared__ double ws[4];
    const uint64_t beg = (uint64_t)blockIdx.x * chunk;
    const uint64_t end = beg + chunk < count ? beg + chunk : count;
    double acc = 0.0;
    for (uint64_t p = beg + threadIdx.x; p < end; p += blockDim.x) {
        const cvec<R> a = psi[expand(p, f)];
        acc += (double)a.x * (double)a.x + (double)a.y * (double)a.y;
    }
    acc = wave_sum_f64(acc);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// Sums `count` partials (strided) in a fixed order into out[0].
__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ part, int count, int stride,
                                                      double *__restrict__ out) {
    __shared__ double ws[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) acc += part[(size_t)i * stride];
    acc = wave_sum_f64(acc);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

template <typename R>
__global__ void k_gather_f64(double2 *__restrict__ out, const cvec<R> *__restrict__ psi, uint64_t count, Ins f,
                             const double *__restrict__ prob) {
    const double sc = 1.0 / sqrt(prob[0]);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count; p += stride) {
        const cvec<R> a = psi[expand(p, f)];
        out[p] = make_double2((double)a.x * sc, (double)a.y * sc);
    }
}

template <typename R>
__global__ void k_gather_dev(cvec<R> *__restrict__ out, const cvec<R> *__restrict__ psi, uint64_t count, Ins f,
                             const double *__restrict__ prob) {
    const R sc = (R)(1.0 / sqrt(prob[0]));
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count; p += stride) {
        const cvec<R> a = psi[expand(p, f)];
        out[p] = cmake<R>(a.x * sc, a.y * sc);
    }
}

// Uniformly controlled Ry on `tbit`: f pins the target to 0 (plus an optional
// extra control); the register value v = (i >> reg_lo) & rmask selects
// (c, s) = cs[v].
template <typename R>
__global__ __launch_bounds__(256) void k_uniform_ry(cvec<R> *__restrict__ psi, uint64_t count, Ins f,
                                                    uint64_t tbit, int reg_lo, uint64_t rmask,
                                                    const cvec<R> *__restrict__ cs) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count; p += stride) {
        const uint64_t i0 = expand(p, f), i1 = i0 | tbit;
        const cvec<R> r = cs[(i0 >> reg_lo) & rmask];
        const cvec<R> a0 = psi[i0], a1 = psi[i1];
        psi[i0] = cmake<R>(r.x * a0.x - r.y * a1.x, r.x * a0.y - r.y * a1.y);
        psi[i1] = cmake<R>(r.y * a0.x + r.x * a1.x, r.y * a0.y + r.x * a1.y);
    }
}

// In-place bit reversal of the register [lo, lo+m): each index whose
// reversed register value is larger swaps with its mirror.
template <typename R>
__global__ __launch_bounds__(256) void k_bitrev(cvec<R> *__restrict__ psi, uint64_t count, Ins f, int lo, int m) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t rm = ((1ull << m) - 1ull);
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count; p += stride) {
        const uint64_t i = expand(p, f);
        const uint64_t v = (i >> lo) & rm;
        const uint64_t r = __brevll(v) >> (64 - m);
        if (r > v) {
            const uint64_t j = (i & ~(rm << lo)) | (r << lo);
            const cvec<R> a = psi[i], b = psi[j];
            psi[i] = b;
            psi[j] = a;
        }
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <typename R> static inline cvec<R> hc(const double *u) {
    cvec<R> z;
    z.x = (R)u[0];
    z.y = (R)u[1];
    return z;
}

// Reduction partials of norm2_into: at most this many blocks.
constexpr int NORM_MAX_PARTS = 4096;

static uint64_t norm_blocks(uint64_t count) {
    const uint64_t per_block = 256 * 64;
    const uint64_t nb = (count + per_block - 1) / per_block;
    return nb > (uint64_t)NORM_MAX_PARTS ? (uint64_t)NORM_MAX_PARTS : (nb ? nb : 1);
}

// FP64 sum of |a_i|^2 over (i & mask) == value into dev_out[0], with `part`
// (device, norm_blocks(count) doubles) holding the per-block partials.
static sv_status norm2_into(sv_state s, uint64_t mask, uint64_t value, double *part, double *dev_out) {
    const Ins f = make_ins(mask, value);
    const uint64_t count = dim_of(s->n - popcount64(mask));
    const uint64_t nb = norm_blocks(count);
    const uint64_t chunk = (count + nb - 1) / nb;
    if (s->dt == SV_C64)
        {
            TraceScope _ts(s->stream, "norm_partial_c64", (double)count * 8, 0.0);
            hipLaunchKernelGGL(k_norm_partial<float>, dim3((unsigned)nb), dim3(256), 0, s->stream,
                           (const float2 *)s->data, count, chunk, f, part);
        }
    else
        {
            TraceScope _ts(s->stream, "norm_partial_c128", (double)count * 16, 0.0);
            hipLaunchKernelGGL(k_norm_partial<double>, dim3((unsigned)nb), dim3(256), 0, s->stream,
                           (const double2 *)s->data, count, chunk, f, part);
        }
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s->stream, (const double *)part, (int)nb, 1, dev_out);
    SV_HIP(hipGetLastError());
    return SV_OK;
}

sv_status norm2_device(sv_state s, uint64_t mask, uint64_t value, double *dev_out) {
    const uint64_t nb = norm_blocks(dim_of(s->n - popcount64(mask)));
    SV_TRY(ensure_small(s, (nb + 8) * sizeof(double)));
    return norm2_into(s, mask, value, (double *)s->small + 8, dev_out);
}

// Workspace of the allocation-free post-selection: the reduction partials
// (NORM_MAX_PARTS doubles) and the probability in the slot after them.  Each
// device holds its own copy until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returns for that device.
constexpr int NOALLOC_SLOTS = NORM_MAX_PARTS + 64;
static __device__ __align__(256) double scratch[NOALLOC_SLOTS];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_noalloc_mu;
static double *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of `scratch` on `dev`, looked up once per device with that
// device current (the caller's current device is restored)
static sv_status noalloc_workspace(int dev, double **out) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(SV_EDEVICE, "device %d beyond the workspace table", dev);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        int cur = 0;
        SV_HIP(hipGetDevice(&cur));
        if (cur != dev) SV_HIP(hipSetDevice(dev));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) SV_HIP(hipSetDevice(cur));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_noalloc_ptr[dev] = (double *)ptr;
    }
    *out = g_noalloc_ptr[dev];
    return SV_OK;
}

sv_status bitrev_register(sv_state s, int lo, int m, uint64_t fix_mask, uint64_t fix_val) {
    if (m < 2) return SV_OK;
    const uint64_t reg = ((1ull << m) - 1ull) << lo;
    if (fix_mask & reg) return fail(SV_EINVAL, "bit reversal: fixed bits overlap the register");
    const Ins f = make_ins(fix_mask, fix_val);
    const uint64_t count = dim_of(s->n - popcount64(fix_mask));
    const unsigned g = grid_for(count, 4);
    if (s->dt == SV_C64)
        {
            TraceScope _ts(s->stream, "bitrev_c64", (double)count * 16, 0.0);
            hipLaunchKernelGGL(k_bitrev<float>, dim3(g), dim3(256), 0, s->stream, (float2 *)s->data, count, f, lo, m);
        }
    else
        {
            TraceScope _ts(s->stream, "bitrev_c128", (double)count * 32, 0.0);
            hipLaunchKernelGGL(k_bitrev<double>, dim3(g), dim3(256), 0, s->stream, (double2 *)s->data, count, f, lo, m);
        }
    SV_HIP(hipGetLastError());
    return SV_OK;
}

template <typename R>
static sv_status launch_gate(sv_state s, int target, const double *u, uint64_t cmask, uint64_t cval) {
    const uint64_t tbit = 1ull << target;
    const bool is_x = u[0] == 0 && u[1] == 0 && u[2] == 1 && u[3] == 0 && u[4] == 1 && u[5] == 0 &&
                      u[6] == 0 && u[7] == 0;
    const bool diag = u[2] == 0 && u[3] == 0 && u[4] == 0 && u[5] == 0;
    const bool u00_one = u[0] == 1 && u[1] == 0;
    const int nfixed = popcount64(cmask) + 1;
    const uint64_t count = dim_of(s->n - nfixed);
    cvec<R> *psi = (cvec<R> *)s->data;
    const cvec<R> u00 = hc<R>(u), u01 = hc<R>(u + 2), u10 = hc<R>(u + 4), u11 = hc<R>(u + 6);
    const unsigned g = grid_for(count, 4);
    if (diag && u00_one) {
        if (u[6] == 1 && u[7] == 0) return SV_OK;    // identity
        const Ins f = make_ins(cmask | tbit, cval | tbit);
        {
            TraceScope _ts(s->stream, "gate_phase", (double)count * 2 * sizeof(cvec<R>), 0.0);
            hipLaunchKernelGGL((k_gate<R, GK_PHASE1>), dim3(g), dim3(256), 0, s->stream, psi, count, f, tbit, u00, u01,
                           u10, u11);
        }
    } else {
        const Ins f = make_ins(cmask | tbit, cval);
        if (is_x)
            {
                TraceScope _ts(s->stream, "gate_x", (double)count * 4 * sizeof(cvec<R>), 0.0);
                hipLaunchKernelGGL((k_gate<R, GK_X>), dim3(g), dim3(256), 0, s->stream, psi, count, f, tbit, u00, u01,
                               u10, u11);
            }
        else if (diag)
            {
                TraceScope _ts(s->stream, "gate_diag", (double)count * 4 * sizeof(cvec<R>), 0.0);
                hipLaunchKernelGGL((k_gate<R, GK_DIAG>), dim3(g), dim3(256), 0, s->stream, psi, count, f, tbit, u00, u01,
                               u10, u11);
            }
        else
            {
                TraceScope _ts(s->stream, "gate_dense", (double)count * 4 * sizeof(cvec<R>), (double)count * 28);
                hipLaunchKernelGGL((k_gate<R, GK_DENSE>), dim3(g), dim3(256), 0, s->stream, psi, count, f, tbit, u00,
                               u01, u10, u11);
            }
    }
    SV_HIP(hipGetLastError());
    return SV_OK;
}

}  // namespace sv

using namespace sv;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *sv_last_error(void) { return g_err.c_str(); }

const char *sv_version(void) {
    return "libsv (HIP, gfx950) built " __DATE__ " " __TIME__;
}

sv_status sv_alloc(sv_state *out, int n_qubits, sv_dtype dt, void *device_buf, void *hip_stream) {
    clear_error();
    if (!out) return fail(SV_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d out of range [1,34]", n_qubits);
    if (dt != SV_C64 && dt != SV_C128) return fail(SV_EINVAL, "bad dtype %d", (int)dt);
    sv_state s = new sv_state_s();
    s->n = n_qubits;
    s->dt = dt;
    s->stream = (hipStream_t)hip_stream;
    hipGetDevice(&s->device);
    const size_t bytes = dim_of(n_qubits) * amp_bytes(dt);
    if (device_buf) {
        s->data = device_buf;
        s->owned = false;
    } else {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && bytes > free_b) {
            delete s;
            return fail(SV_ENOMEM, "state of %zu bytes exceeds free device memory (%zu)", bytes, free_b);
        }
        hipError_t e = hipMalloc(&s->data, bytes);
        if (e != hipSuccess) {
            delete s;
            return hip_fail(e, "hipMalloc(state)");
        }
        s->owned = true;
    }
    *out = s;
    return SV_OK;
}

sv_status sv_free(sv_state s) {
    if (!s) return SV_OK;
    hipStreamSynchronize(s->stream);
    if (s->owned && s->data) hipFree(s->data);
    if (s->scratch) hipFree(s->scratch);
    if (s->small) hipFree(s->small);
    if (s->pinned) hipHostFree(s->pinned);
    delete s;
    return SV_OK;
}

void *sv_data(sv_state s) { return s ? s->data : nullptr; }
int sv_num_qubits(sv_state s) { return s ? s->n : 0; }
sv_dtype sv_get_dtype(sv_state s) { return s ? s->dt : SV_C64; }

sv_status sv_set_stream(sv_state s, void *hip_stream) {
    SV_TRY(check_state(s));
    s->stream = (hipStream_t)hip_stream;
    return SV_OK;
}

sv_status sv_init_basis(sv_state s, uint64_t index) {
    clear_error();
    SV_TRY(check_state(s));
    const uint64_t dim = dim_of(s->n);
    if (index >= dim) return fail(SV_EINVAL, "basis index out of range");
    const unsigned g = grid_for(dim, 8);
    if (s->dt == SV_C64)
        hipLaunchKernelGGL(k_fill_basis<float>, dim3(g), dim3(256), 0, s->stream, (float2 *)s->data, dim, index);
    else
        hipLaunchKernelGGL(k_fill_basis<double>, dim3(g), dim3(256), 0, s->stream, (double2 *)s->data, dim, index);
    SV_HIP(hipGetLastError());
    return SV_OK;
}

sv_status sv_init_b(sv_state s, const double *b, int n_s, int n_clock_superpose) {
    clear_error();
    SV_TRY(check_state(s));
    if (!b) return fail(SV_EINVAL, "b is NULL");
    if (n_s < 0 || n_clock_superpose < 0 || n_s + n_clock_superpose > s->n)
        return fail(SV_EINVAL, "n_s %d + clock %d exceeds %d qubits", n_s, n_clock_superpose, s->n);
    const uint64_t N = dim_of(n_s);
    double nrm = 0.0;
    for (uint64_t j = 0; j < 2 * N; ++j) nrm += b[j] * b[j];
    nrm = sqrt(nrm);
    if (!(nrm > 0.0) || !isfinite(nrm)) return fail(SV_EZERONORM, "|b| = 0 or not finite");
    SV_TRY(ensure_small(s, 64 + N * sizeof(double2)));
    double2 *db = (double2 *)((char *)s->small + 64);
    SV_TRY(upload(s, db, b, N * sizeof(double2)));
    const double scale = 1.0 / (nrm * sqrt((double)dim_of(n_clock_superpose)));
    const uint64_t dim = dim_of(s->n);
    const unsigned g = grid_for(dim, 8);
    if (s->dt == SV_C64)
        {
            TraceScope _ts(s->stream, "init_b_c64", (double)dim * 8, 0.0);
            hipLaunchKernelGGL(k_init_b<float>, dim3(g), dim3(256), 0, s->stream, (float2 *)s->data, dim,
                           (const double2 *)db, n_s, dim_of(n_clock_superpose), scale);
        }
    else
        {
            TraceScope _ts(s->stream, "init_b_c128", (double)dim * 16, 0.0);
            hipLaunchKernelGGL(k_init_b<double>, dim3(g), dim3(256), 0, s->stream, (double2 *)s->data, dim,
                           (const double2 *)db, n_s, dim_of(n_clock_superpose), scale);
        }
    SV_HIP(hipGetLastError());
    SV_HIP(hipStreamSynchronize(s->stream));   // db lives in the small arena
    return SV_OK;
}

sv_status sv_set_state(sv_state s, const double *host) {
    clear_error();
    SV_TRY(check_state(s));
    if (!host) return fail(SV_EINVAL, "host is NULL");
    const uint64_t dim = dim_of(s->n);
    if (s->dt == SV_C128) return upload(s, s->data, host, dim * 16);
    SV_TRY(ensure_scratch(s, dim * 16));
    SV_TRY(upload(s, s->scratch, host, dim * 16));
    hipLaunchKernelGGL(k_from_f64<float>, dim3(grid_for(dim, 8)), dim3(256), 0, s->stream, (float2 *)s->data,
                       (const double2 *)s->scratch, dim);
    SV_HIP(hipGetLastError());
    SV_HIP(hipStreamSynchronize(s->stream));
    return SV_OK;
}

sv_status sv_get_state(sv_state s, double *host) {
    clear_error();
    SV_TRY(check_state(s));
    if (!host) return fail(SV_EINVAL, "host is NULL");
    const uint64_t dim = dim_of(s->n);
    if (s->dt == SV_C128) return download(s, host, s->data, dim * 16);
    SV_TRY(ensure_scratch(s, dim * 16));
    hipLaunchKernelGGL(k_to_f64<float>, dim3(grid_for(dim, 8)), dim3(256), 0, s->stream, (double2 *)s->scratch,
                       (const float2 *)s->data, dim);
    SV_HIP(hipGetLastError());
    return download(s, host, s->scratch, dim * 16);
}

sv_status sv_apply_gate(sv_state s, int target, const double u[8], const int *ctrls, const int *ctrl_vals,
                        int n_ctrls) {
    clear_error();
    SV_TRY(check_state(s));
    if (!u) return fail(SV_EINVAL, "u is NULL");
    for (int i = 0; i < 8; ++i)
        if (!isfinite(u[i])) return fail(SV_EINVAL, "u has a non-finite entry");
    uint64_t cm, cv;
    SV_TRY(check_qubits(s, &target, 1, ctrls, ctrl_vals, n_ctrls, &cm, &cv));
    return s->dt == SV_C64 ? launch_gate<float>(s, target, u, cm, cv) : launch_gate<double>(s, target, u, cm, cv);
}

sv_status sv_apply_swap(sv_state s, int q1, int q2, const int *ctrls, const int *ctrl_vals, int n_ctrls) {
    clear_error();
    SV_TRY(check_state(s));
    int qs[2] = {q1, q2};
    uint64_t cm, cv;
    SV_TRY(check_qubits(s, qs, 2, ctrls, ctrl_vals, n_ctrls, &cm, &cv));
    const uint64_t b1 = 1ull << q1, b2 = 1ull << q2;
    const Ins f = make_ins(cm | b1 | b2, cv | b1);
    const uint64_t count = dim_of(s->n - popcount64(cm) - 2);
    const unsigned g = grid_for(count, 4);
    if (s->dt == SV_C64)
        {
            TraceScope _ts(s->stream, "swap_c64", (double)count * 32, 0.0);
            hipLaunchKernelGGL(k_swap<float>, dim3(g), dim3(256), 0, s->stream, (float2 *)s->data, count, f, b1 | b2);
        }
    else
        {
            TraceScope _ts(s->stream, "swap_c128", (double)count * 64, 0.0);
            hipLaunchKernelGGL(k_swap<double>, dim3(g), dim3(256), 0, s->stream, (double2 *)s->data, count, f, b1 | b2);
        }
    SV_HIP(hipGetLastError());
    return SV_OK;
}

sv_status sv_apply_uniform_ry(sv_state s, int target, int reg_lo, int m, const double *cs, int extra_ctrl,
                              int extra_val) {
    clear_error();
    SV_TRY(check_state(s));
    if (!cs) return fail(SV_EINVAL, "cs is NULL");
    if (m < 1 || reg_lo < 0 || reg_lo + m > s->n) return fail(SV_EINVAL, "register out of range");
    if (target < 0 || target >= s->n || (target >= reg_lo && target < reg_lo + m))
        return fail(SV_EINVAL, "target %d invalid", target);
    uint64_t fm = 1ull << target, fv = 0;
    if (extra_ctrl >= 0) {
        if (extra_ctrl >= s->n || extra_ctrl == target || (extra_ctrl >= reg_lo && extra_ctrl < reg_lo + m))
            return fail(SV_EINVAL, "extra control %d invalid", extra_ctrl);
        fm |= 1ull << extra_ctrl;
        fv |= (uint64_t)(extra_val ? 1 : 0) << extra_ctrl;
    }
    const uint64_t M = dim_of(m);
    const size_t tb = M * amp_bytes(s->dt);
    SV_TRY(ensure_small(s, 64 + tb));
    void *dt = (char *)s->small + 64;
    if (s->dt == SV_C64) {
        std::vector<float> tmp(2 * M);
        for (uint64_t i = 0; i < 2 * M; ++i) tmp[i] = (float)cs[i];
        SV_TRY(upload(s, dt, tmp.data(), tb));
    } else {
        SV_TRY(upload(s, dt, cs, tb));
    }
    const Ins f = make_ins(fm, fv);
    const uint64_t count = dim_of(s->n - popcount64(fm));
    const unsigned g = grid_for(count, 4);
    if (s->dt == SV_C64)
        {
            TraceScope _ts(s->stream, "uniform_ry_c64", (double)count * 32, 0.0);
            hipLaunchKernelGGL(k_uniform_ry<float>, dim3(g), dim3(256), 0, s->stream, (float2 *)s->data, count, f,
                           1ull << target, reg_lo, M - 1, (const float2 *)dt);
        }
    else
        {
            TraceScope _ts(s->stream, "uniform_ry_c128", (double)count * 64, 0.0);
            hipLaunchKernelGGL(k_uniform_ry<double>, dim3(g), dim3(256), 0, s->stream, (double2 *)s->data, count, f,
                           1ull << target, reg_lo, M - 1, (const double2 *)dt);
        }
    SV_HIP(hipGetLastError());
    SV_HIP(hipStreamSynchronize(s->stream));   // the table lives in the small arena
    return SV_OK;
}

sv_status sv_norm2(sv_state s, uint64_t mask, uint64_t value, double *out) {
    clear_error();
    SV_TRY(check_state(s));
    if (!out) return fail(SV_EINVAL, "out is NULL");
    if (mask >> s->n) return fail(SV_EINVAL, "mask has bits beyond the state");
    if (value & ~mask) return fail(SV_EINVAL, "value has bits outside mask");
    SV_TRY(ensure_small(s, 4096 * sizeof(double) + 64));
    double *dres = (double *)s->small;
    SV_TRY(norm2_device(s, mask, value, dres));
    return download(s, out, dres, sizeof(double));
}

sv_status sv_postselect(sv_state s, uint64_t mask, uint64_t value, double *prob, void *out, int out_on_device) {
    clear_error();
    SV_TRY(check_state(s));
    if (mask >> s->n) return fail(SV_EINVAL, "mask has bits beyond the state");
    if (value & ~mask) return fail(SV_EINVAL, "value has bits outside mask");
    SV_TRY(ensure_small(s, 4096 * sizeof(double) + 64));
    double *dres = (double *)s->small;
    SV_TRY(norm2_device(s, mask, value, dres));
    double p = 0.0;
    SV_TRY(download(s, &p, dres, sizeof(double)));
    if (prob) *prob = p;
    if (!(p > 0.0)) return fail(SV_EZERONORM, "post-selected outcome has probability 0");
    if (!out) return SV_OK;
    const uint64_t count = dim_of(s->n - popcount64(mask));
    const Ins f = make_ins(mask, value);
    const unsigned g = grid_for(count, 4);
    if (out_on_device) {
        if (s->dt == SV_C64)
            hipLaunchKernelGGL(k_gather_dev<float>, dim3(g), dim3(256), 0, s->stream, (float2 *)out,
                               (const float2 *)s->data, count, f, (const double *)dres);
        else
            hipLaunchKernelGGL(k_gather_dev<double>, dim3(g), dim3(256), 0, s->stream, (double2 *)out,
                               (const double2 *)s->data, count, f, (const double *)dres);
        SV_HIP(hipGetLastError());
        return SV_OK;
    }
    SV_TRY(ensure_scratch(s, count * sizeof(double2)));
    if (s->dt == SV_C64)
        hipLaunchKernelGGL(k_gather_f64<float>, dim3(g), dim3(256), 0, s->stream, (double2 *)s->scratch,
                           (const float2 *)s->data, count, f, (const double *)dres);
    else
        hipLaunchKernelGGL(k_gather_f64<double>, dim3(g), dim3(256), 0, s->stream, (double2 *)s->scratch,
                           (const double2 *)s->data, count, f, (const double *)dres);
    SV_HIP(hipGetLastError());
    return download(s, out, s->scratch, count * sizeof(double2));
}

sv_status sv_postselect_noalloc(sv_state s, uint64_t mask, uint64_t value, double *prob_dev, void *out_dev) {
    clear_error();
    SV_TRY(check_state(s));
    if (!prob_dev) return fail(SV_EINVAL, "prob_dev is NULL");
    if (mask >> s->n) return fail(SV_EINVAL, "mask has bits beyond the state");
    if (value & ~mask) return fail(SV_EINVAL, "value has bits outside mask");
    const uint64_t count = dim_of(s->n - popcount64(mask));
    if (norm_blocks(count) > (uint64_t)NORM_MAX_PARTS)
        return fail(SV_EINVAL, "reduction needs %llu partials, workspace holds %d",
                    (unsigned long long)norm_blocks(count), NORM_MAX_PARTS);
    double *ws = nullptr;
    SV_TRY(noalloc_workspace(s->device, &ws));
    // every partial slot the reduction reads is written by its own block first,
    // so the workspace needs no clearing between calls
    SV_TRY(norm2_into(s, mask, value, ws, prob_dev));
    if (!out_dev) return SV_OK;
    const Ins f = make_ins(mask, value);
    const unsigned g = grid_for(count, 4);
    if (s->dt == SV_C64)
        hipLaunchKernelGGL(k_gather_dev<float>, dim3(g), dim3(256), 0, s->stream, (float2 *)out_dev,
                           (const float2 *)s->data, count, f, (const double *)prob_dev);
    else
        hipLaunchKernelGGL(k_gather_dev<double>, dim3(g), dim3(256), 0, s->stream, (double2 *)out_dev,
                           (const double2 *)s->data, count, f, (const double *)prob_dev);
    SV_HIP(hipGetLastError());
    return SV_OK;
}

}  // extern "C"
