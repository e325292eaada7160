// QSP-1: binary-tree state preparation (appendix "Quantum State
// Preparation"; the Grover-Rudolph tree in Prakash's form).
//
// Tree over the register value r of [q_lo, q_lo + m): leaves carry |b_r|^2,
// inner nodes the sum of their children.  Level l decides qubit
// q_lo + m - 1 - l (most significant first); node p of level l is the value of
// the l qubits above it.  Each node with weight w > 0 is an Ry(t) with
// cos^2(t/2) = zero-child / w, controlled on those qubits taking the value p;
// a final diagonal restores arg(b_r).
//
//   mode 0: the circuit on the state: |0...0>, one Ry on the top qubit, then
//           per level one uniformly controlled Ry pass (every node of the
//           level is one control value), then the phase diagonal pass;
//   mode 1: the same circuit applied to |0...0> in one write pass: each
//           amplitude is the product of the rotation entries on its tree
//           path times its phase (a thread expands the subtree below one
//           node of level m - 5 in registers); zero outside the register.
#include <math.h>

#include <complex>
#include <vector>

#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

// heap-ordered (cos, sin) of every node, node k = 2^l + p at 2k, 2k + 1.
// A thread owns the 2^C leaves below one node of level m - C: it walks the
// m - C levels above that node once, then expands its subtree in registers.
// The leaves of a block's QSP_NT subtrees (QSP_NT 2^C consecutive register
// values) go through LDS (one pad element per thread, so the row writes are
// conflict-free) and leave in register order, so that each store and each
// phase-table read of a wavefront covers consecutive addresses.
constexpr int QSP_NT = 128;

template <typename R, int C>
__global__ __launch_bounds__(QSP_NT) void k_qsp_tree(cvec<R> *__restrict__ psi, int q_lo, int m,
                                                     const R *__restrict__ cs, const cvec<R> *__restrict__ ph) {
    constexpr int L = 1 << C, LP = L + 1;
    __shared__ R leaves[QSP_NT * LP];
    const uint64_t nsub = 1ull << (m - C);          // subtrees
    const uint64_t R_ = 1ull << m;
    for (uint64_t t0 = (uint64_t)blockIdx.x * QSP_NT; t0 < nsub; t0 += (uint64_t)gridDim.x * QSP_NT) {
        const uint64_t t = t0 + threadIdx.x;
        if (t < nsub) {
            R a = 1;
            uint64_t node = 1;
            for (int l = 0; l < m - C; ++l) {
                const uint64_t bit = (t >> (m - C - 1 - l)) & 1ull;
                a *= cs[2 * node + bit];
                node = 2 * node + bit;
            }
            R v[L];
            v[0] = a;
#pragma unroll
            for (int l = 0; l < C; ++l) {
                // the 2^l values of this level, at nodes (node << l) + q, split into their children
#pragma unroll
                for (int q = (1 << l) - 1; q >= 0; --q) {
                    const uint64_t nd = (node << l) + (uint64_t)q;
                    const R x = v[q];
                    v[2 * q] = x * cs[2 * nd];
                    v[2 * q + 1] = x * cs[2 * nd + 1];
                }
            }
#pragma unroll
            for (int j = 0; j < L; ++j) leaves[threadIdx.x * LP + j] = v[j];
        }
        __syncthreads();
        // leaf e of the block is register value (t0 << C) + e
        const uint64_t rbase = t0 << C;
        for (int e = threadIdx.x; e < QSP_NT * L; e += QSP_NT) {
            const uint64_t r = rbase + (uint64_t)e;
            if (r >= R_) break;
            const R x = leaves[(e >> C) * LP + (e & (L - 1))];
            const cvec<R> p = ph[r];
            psi[r << q_lo] = cmake<R>(x * p.x, x * p.y);
        }
        __syncthreads();
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_zero(cvec<R> *__restrict__ psi, uint64_t dim) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride) psi[i] = cmake<R>(0, 0);
}

// psi[i] *= ph[register value of i] (a diagonal gate on the register)
template <typename R>
__global__ __launch_bounds__(256) void k_reg_phase(cvec<R> *__restrict__ psi, uint64_t dim, int q_lo, int m,
                                                   const cvec<R> *__restrict__ ph) {
    const uint64_t rmask = (1ull << m) - 1ull;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride)
        psi[i] = cmul<R>(psi[i], ph[(i >> q_lo) & rmask]);
}

static unsigned grid_of(uint64_t items) {
    uint64_t g = (items + 1023) / 1024;
    if (g < 1) g = 1;
    if (g > (1u << 20)) g = 1u << 20;
    return (unsigned)g;
}

template <typename R>
static sv_status upload_tables(sv_state s, const std::vector<double> &cs, const std::vector<double> &ph, void **dcs,
                               void **dph) {
    const size_t ncs = cs.size(), nph = ph.size();
    const size_t bcs = ncs * sizeof(R), bph = nph * sizeof(R);
    const size_t off = (bcs + 255) & ~(size_t)255;
    SV_TRY(ensure_scratch(s, off + bph));
    std::vector<R> tmp(ncs > nph ? ncs : nph);
    for (size_t i = 0; i < ncs; ++i) tmp[i] = (R)cs[i];
    SV_TRY(upload(s, s->scratch, tmp.data(), bcs));
    for (size_t i = 0; i < nph; ++i) tmp[i] = (R)ph[i];
    SV_TRY(upload(s, (char *)s->scratch + off, tmp.data(), bph));
    *dcs = s->scratch;
    *dph = (char *)s->scratch + off;
    return SV_OK;
}

}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_qsp_prepare(sv_state s, const double *b, int q_lo, int m, int mode) {
    clear_error();
    SV_TRY(check_state(s));
    if (!b) return fail(SV_EINVAL, "b is NULL");
    if (m < 1 || m > 26 || q_lo < 0 || q_lo + m > s->n)
        return fail(SV_EINVAL, "register [%d, %d) outside the state (or wider than 26 qubits)", q_lo, q_lo + m);
    if (mode != 0 && mode != 1) return fail(SV_EINVAL, "mode must be 0 or 1");
    const uint64_t R = 1ull << m, dim = dim_of(s->n);
    // tree weights (FP64, heap order) and the rotation of every node
    std::vector<double> w(2 * R, 0.0);
    double tot = 0.0;
    for (uint64_t r = 0; r < R; ++r) {
        const double re = b[2 * r], im = b[2 * r + 1];
        if (!std::isfinite(re) || !std::isfinite(im)) return fail(SV_EINVAL, "b has a non-finite entry");
        w[R + r] = re * re + im * im;
        tot += w[R + r];
    }
    if (!(tot > 0.0)) return fail(SV_EZERONORM, "|b| = 0");
    for (uint64_t k = R - 1; k >= 1; --k) w[k] = w[2 * k] + w[2 * k + 1];
    std::vector<double> cs(2 * R, 0.0);     // (cos, sin) of node k at 2k, 2k + 1 (k >= 1)
    for (uint64_t k = 1; k < R; ++k) {
        if (w[k] > 0.0) {
            cs[2 * k] = sqrt(w[2 * k] / w[k]);
            cs[2 * k + 1] = sqrt(w[2 * k + 1] / w[k]);
        } else {
            cs[2 * k] = 1.0;                    // no gate
            cs[2 * k + 1] = 0.0;
        }
    }
    std::vector<double> ph(2 * R);
    for (uint64_t r = 0; r < R; ++r) {
        const double a = w[R + r] > 0.0 ? atan2(b[2 * r + 1], b[2 * r]) : 0.0;
        ph[2 * r] = cos(a);
        ph[2 * r + 1] = sin(a);
    }
    const bool f32 = s->dt == SV_C64;
    if (mode == 1) {
        void *dcs = nullptr, *dph = nullptr;
        SV_TRY(f32 ? upload_tables<float>(s, cs, ph, &dcs, &dph) : upload_tables<double>(s, cs, ph, &dcs, &dph));
        if (R != dim) {   // qubits outside the register: |0>
            TraceScope tz(s->stream, "qsp_zero", (double)dim * amp_bytes(s->dt), 0.0);
            if (f32)
                hipLaunchKernelGGL(k_zero<float>, dim3(grid_of(dim)), dim3(256), 0, s->stream, (float2 *)s->data, dim);
            else
                hipLaunchKernelGGL(k_zero<double>, dim3(grid_of(dim)), dim3(256), 0, s->stream, (double2 *)s->data,
                                   dim);
        }
        // algorithmic bytes: the register written once, its (cos, sin) tree and phase table read once
        TraceScope ts(s->stream, "qsp_tree", (double)R * (2.0 * amp_bytes(s->dt) + amp_bytes(s->dt)), 0.0);
        const uint64_t nsub = R >> (m < 5 ? m : 5);
        const uint64_t nblk = (nsub + QSP_NT - 1) / QSP_NT;
        const dim3 g((unsigned)(nblk < (1u << 20) ? nblk : (1u << 20)));
#define SV_QSP_LAUNCH(Cb)                                                                                       \
    do {                                                                                                        \
        if (f32)                                                                                                \
            hipLaunchKernelGGL((k_qsp_tree<float, Cb>), g, dim3(QSP_NT), 0, s->stream, (float2 *)s->data, q_lo, m, \
                               (const float *)dcs, (const float2 *)dph);                                       \
        else                                                                                                    \
            hipLaunchKernelGGL((k_qsp_tree<double, Cb>), g, dim3(QSP_NT), 0, s->stream, (double2 *)s->data, q_lo, m, \
                               (const double *)dcs, (const double2 *)dph);                                     \
    } while (0)
        switch (m < 5 ? m : 5) {
        case 1: SV_QSP_LAUNCH(1); break;
        case 2: SV_QSP_LAUNCH(2); break;
        case 3: SV_QSP_LAUNCH(3); break;
        case 4: SV_QSP_LAUNCH(4); break;
        default: SV_QSP_LAUNCH(5); break;
        }
#undef SV_QSP_LAUNCH
        SV_HIP(hipGetLastError());
        SV_HIP(hipStreamSynchronize(s->stream));   // the tables live in the scratch arena
        return SV_OK;
    }
    // mode 0: the circuit, level by level
    SV_TRY(sv_init_basis(s, 0));
    const int top = q_lo + m - 1;
    {
        const double c = cs[2], sn = cs[3];
        const double ry[8] = {c, 0.0, -sn, 0.0, sn, 0.0, c, 0.0};
        SV_TRY(sv_apply_gate(s, top, ry, nullptr, nullptr, 0));
    }
    std::vector<double> lv;
    for (int l = 1; l < m; ++l) {
        // control register: the l qubits above the target, value v = node p
        const uint64_t P = 1ull << l;
        lv.assign(2 * P, 0.0);
        for (uint64_t p = 0; p < P; ++p) {
            lv[2 * p] = cs[2 * (P + p)];
            lv[2 * p + 1] = cs[2 * (P + p) + 1];
        }
        SV_TRY(sv_apply_uniform_ry(s, top - l, top - l + 1, l, lv.data(), -1, 0));
    }
    void *dcs = nullptr, *dph = nullptr;
    std::vector<double> none(2, 0.0);
    SV_TRY(f32 ? upload_tables<float>(s, none, ph, &dcs, &dph) : upload_tables<double>(s, none, ph, &dcs, &dph));
    {
        TraceScope ts(s->stream, "reg_phase", 2.0 * (double)dim * amp_bytes(s->dt), 0.0);
        if (f32)
            hipLaunchKernelGGL(k_reg_phase<float>, dim3(grid_of(dim)), dim3(256), 0, s->stream, (float2 *)s->data, dim,
                               q_lo, m, (const float2 *)dph);
        else
            hipLaunchKernelGGL(k_reg_phase<double>, dim3(grid_of(dim)), dim3(256), 0, s->stream, (double2 *)s->data,
                               dim, q_lo, m, (const double2 *)dph);
    }
    SV_HIP(hipGetLastError());
    SV_HIP(hipStreamSynchronize(s->stream));
    return SV_OK;
}

}  // extern "C"
