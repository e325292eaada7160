// Controlled dense unitary on a register of m qubits [lo, lo + m) as a
// complex GEMM on the matrix cores (MFMA): every amplitude row whose control
// bits match is a length-2^m vector v, replaced by U v.  Rows are gathered
// straight from the state (row r starts at pdep(r, row_mask) | row_fix, its
// element k at stride 2^lo), multiplied out of place into a compact buffer
// and scattered back.  complex64 uses v_mfma_f32_16x16x4f32 (FP32 in, FP32 accumulate);
// complex128 uses v_mfma_f64_16x16x4f64.  A complex product is four real
// MFMAs: re += ar br - ai bi, im += ar bi + ai br.
#include <string.h>

#include <string>
#include <vector>

#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename R> struct MfmaT;
// Operands of both: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16].
// Results: the FP32 form keeps four consecutive rows per lane group
// (row 4 (l / 16) + v), the FP64 form interleaves them (row l / 16 + 4 v);
// the column is l % 16 in both.
template <> struct MfmaT<float> {
    using acc = floatx4;
    static __device__ __forceinline__ acc mfma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) * 4 + v; }
};
template <> struct MfmaT<double> {
    using acc = doublex4;
    static __device__ __forceinline__ acc mfma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

constexpr int GBM = 64, GBN = 64, GBK = 16;

template <typename R>
struct GemmArgs {
    const cvec<R> *in;   // rows of length K
    cvec<R> *out;        // M x N, row-major, compact
    const cvec<R> *U;    // B(kk, n) = trans ? U[kk * N + n] : U[n * K + kk]  (conj if conjb)
    uint64_t M;
    int N, K;
    uint64_t row_mask, row_fix;   // row r starts at pdep(r, row_mask) | row_fix
    int ksh;                      // element k of a row at offset k << ksh
    int trans, conjb;
};

// 256 threads: 4 waves as 2 x 2, each wave a 32 x 32 output block made of
// 2 x 2 MFMA 16 x 16 tiles.  Operands are staged in LDS as separate real and
// imaginary planes, k-major, so the 16 lanes that share a k read 16
// consecutive words; the next k step's operands are in flight (in
// registers) while a step's MFMAs run.
template <typename R>
__global__ __launch_bounds__(256) void k_cgemm(GemmArgs<R> A) {
    using M_ = MfmaT<R>;
    using acc_t = typename M_::acc;
    __shared__ R As_re[GBK][GBM], As_im[GBK][GBM], Bs_re[GBK][GBN], Bs_im[GBK][GBN];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const uint64_t row0 = (uint64_t)blockIdx.x * GBM;
    const int n0 = blockIdx.y * GBN;

    // this thread's A-load row and its base offset in the state: four
    // threads along k per row when the row is contiguous (ksh = 0), else one
    // row per lane, so that a wavefront reads 64 neighbouring rows
    const int a_row = A.ksh ? (tid & 63) : tid >> 2, a_k = A.ksh ? (tid >> 6) * 4 : (tid & 3) * 4;
    const uint64_t ar = row0 + a_row;
    const bool a_ok = ar < A.M;
    const uint64_t a_base = a_ok ? (pdep64(ar, A.row_mask) | A.row_fix) : 0;

    acc_t acc_re[2][2], acc_im[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int v = 0; v < 4; ++v) acc_re[i][j][v] = acc_im[i][j][v] = (R)0;

    const R csgn = A.conjb ? (R)-1 : (R)1;
    // The next k step's operands are loaded into registers while this step's
    // MFMAs run, and written to the LDS after the step's closing barrier.
    // Thread roles: A rows as above; B as (n, four k) or (k, four n).
    const int b_n = A.trans ? (tid & 15) * 4 : tid >> 2, b_k = A.trans ? tid >> 4 : (tid & 3) * 4;
    cvec<R> pa[4], pb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kk = k0 + a_k + i;
            pa[i] = cmake<R>((R)0, (R)0);
            if (a_ok && kk < A.K) pa[i] = A.in[a_base + ((uint64_t)kk << A.ksh)];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            pb[i] = cmake<R>((R)0, (R)0);
            if (!A.trans) {
                const int kk = k0 + b_k + i, nn = n0 + b_n;
                if (kk < A.K && nn < A.N) pb[i] = A.U[(uint64_t)nn * A.K + kk];
            } else {
                const int kk = k0 + b_k, nn = n0 + b_n + i;
                if (kk < A.K && nn < A.N) pb[i] = A.U[(uint64_t)kk * A.N + nn];
            }
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < A.K; k0 += GBK) {
        // A tile: 64 rows x 16 k; B tile: 16 k x 64 n
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            As_re[a_k + i][a_row] = pa[i].x;
            As_im[a_k + i][a_row] = pa[i].y;
            const int bk = A.trans ? b_k : b_k + i, bn = A.trans ? b_n + i : b_n;
            Bs_re[bk][bn] = pb[i].x;
            Bs_im[bk][bn] = csgn * pb[i].y;
        }
        __syncthreads();
        if (k0 + GBK < A.K) fetch(k0 + GBK);
#pragma unroll
        for (int kc = 0; kc < GBK / 4; ++kc) {
            const int kr = kc * 4 + (lane >> 4), li = lane & 15;
            R ar_[2], ai_[2], br_[2], bi_[2];
            for (int i = 0; i < 2; ++i) {
                ar_[i] = As_re[kr][wm * 32 + i * 16 + li];
                ai_[i] = As_im[kr][wm * 32 + i * 16 + li];
                br_[i] = Bs_re[kr][wn * 32 + i * 16 + li];
                bi_[i] = Bs_im[kr][wn * 32 + i * 16 + li];
            }
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    acc_re[i][j] = M_::mfma(ar_[i], br_[j], acc_re[i][j]);
                    acc_re[i][j] = M_::mfma(-ai_[i], bi_[j], acc_re[i][j]);
                    acc_im[i][j] = M_::mfma(ar_[i], bi_[j], acc_im[i][j]);
                    acc_im[i][j] = M_::mfma(ai_[i], br_[j], acc_im[i][j]);
                }
        }
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int v = 0; v < 4; ++v) {
                const uint64_t r = row0 + wm * 32 + i * 16 + M_::row(lane, v);
                const int c = n0 + wn * 32 + j * 16 + (lane & 15);
                if (r < A.M && c < A.N) A.out[r * A.N + c] = cmake<R>(acc_re[i][j][v], acc_im[i][j][v]);
            }
}

// The same product with one wavefront per 16 x 16 output tile and no LDS:
// each lane loads its MFMA operands straight from memory (A[row][k] for row
// l % 16, k = l / 16 of each 4-wide k step, and B[k][col] alike).  For small
// products (the basis changes of a Kronecker plan: 256 x 256 x 256) the
// 64 x 64 block tiles leave most of the chip idle; here every tile is a
// wavefront.  The k steps and the four real MFMAs of a complex product run in
// the same order as in k_cgemm, so both give the same bits.
template <typename R>
__global__ __launch_bounds__(256) void k_cgemm_w(GemmArgs<R> A) {
    using M_ = MfmaT<R>;
    using acc_t = typename M_::acc;
    const int lane = threadIdx.x & 63;
    const uint64_t tiles_n = (uint64_t)((A.N + 15) / 16);
    const uint64_t tile = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint64_t tm = tile / tiles_n, tn = tile % tiles_n;
    if (tm * 16 >= A.M) return;                       // the whole wavefront (no barriers below)
    const uint64_t r = tm * 16 + (lane & 15);
    const int c = (int)(tn * 16) + (lane & 15);
    const int kq = lane >> 4;
    const bool r_ok = r < A.M, c_ok = c < A.N;
    const uint64_t a_base = r_ok ? (pdep64(r, A.row_mask) | A.row_fix) : 0;
    const R csgn = A.conjb ? (R)-1 : (R)1;
    acc_t acc_re, acc_im;
    for (int v = 0; v < 4; ++v) acc_re[v] = acc_im[v] = (R)0;
#pragma unroll 4
    for (int k0 = 0; k0 < A.K; k0 += 4) {
        const int kk = k0 + kq;
        cvec<R> a = cmake<R>((R)0, (R)0), b = cmake<R>((R)0, (R)0);
        if (r_ok && kk < A.K) a = A.in[a_base + ((uint64_t)kk << A.ksh)];
        if (c_ok && kk < A.K) b = A.trans ? A.U[(uint64_t)kk * A.N + c] : A.U[(uint64_t)c * A.K + kk];
        acc_re = M_::mfma(a.x, b.x, acc_re);
        acc_re = M_::mfma(-a.y, csgn * b.y, acc_re);
        acc_im = M_::mfma(a.x, csgn * b.y, acc_im);
        acc_im = M_::mfma(a.y, b.x, acc_im);
    }
    for (int v = 0; v < 4; ++v) {
        const uint64_t rr = tm * 16 + M_::row(lane, v);
        if (rr < A.M && c_ok) A.out[rr * A.N + c] = cmake<R>(acc_re[v], acc_im[v]);
    }
}

template <typename R>
__global__ void k_scatter_rows(cvec<R> *__restrict__ psi, const cvec<R> *__restrict__ src, uint64_t M, int mbits,
                               uint64_t row_mask, uint64_t row_fix, int ksh) {
    const uint64_t total = M << mbits;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t cm = (1ull << mbits) - 1ull;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const uint64_t r = i >> mbits;
        psi[(pdep64(r, row_mask) | row_fix) + ((i & cm) << ksh)] = src[i];
    }
}

// host: Out(M x N) = rows(In) * B, with B as described in GemmArgs
template <typename R>
static sv_status cgemm_ks(hipStream_t st, const cvec<R> *in, cvec<R> *out, const cvec<R> *U, uint64_t M, int N,
                          int K, uint64_t row_mask, uint64_t row_fix, int ksh, int trans, int conjb) {
    GemmArgs<R> a;
    a.in = in;
    a.out = out;
    a.U = U;
    a.M = M;
    a.N = N;
    a.K = K;
    a.row_mask = row_mask;
    a.row_fix = row_fix;
    a.ksh = ksh;
    a.trans = trans;
    a.conjb = conjb;
    const uint64_t gm = (M + GBM - 1) / GBM;
    const unsigned gn = (unsigned)((N + GBN - 1) / GBN);
    if (gm > 0x7fffffffull) return fail(SV_EUNSUPPORTED, "GEMM with too many rows");
    const uint64_t wtiles = ((M + 15) / 16) * (uint64_t)((N + 15) / 16);
    const uint64_t wblocks = (wtiles + 3) / 4;
    // the tile shape: 64 x 64 per workgroup (0) or 16 x 16 per wavefront (1).
    // Tuned per shape by timing both on this call's operands (the product is
    // out of place, so it can be run twice), cached; without tuning, the
    // wavefront tiles wherever the workgroup tiles would not fill the chip.
    const std::string key = std::string("cgemm/") + (sizeof(R) == 4 ? "c64/" : "c128/") + std::to_string(M) + "/" +
                            std::to_string(N) + "/" + std::to_string(K) + "/" + std::to_string(trans) +
                            (ksh ? "/s" + std::to_string(ksh) : std::string());
    auto launch = [&](int shape) -> sv_status {
        TraceScope _ts(st, "cgemm", ((double)M * (N + K) + (double)N * K) * sizeof(cvec<R>), 8.0 * (double)M * N * K);
        if (shape == 1) {
            if (wblocks > 0x7fffffffull) return fail(SV_EUNSUPPORTED, "GEMM with too many tiles");
            hipLaunchKernelGGL(k_cgemm_w<R>, dim3((unsigned)wblocks), dim3(256), 0, st, a);
        } else {
            hipLaunchKernelGGL(k_cgemm<R>, dim3((unsigned)gm, gn), dim3(256), 0, st, a);
        }
        SV_HIP(hipGetLastError());
        return SV_OK;
    };
    std::vector<int> cached;
    int shape = gm * gn < 256 ? 1 : 0;
    if (tune_lookup(key, cached) && cached.size() == 1 && (cached[0] == 0 || cached[0] == 1)) {
        shape = cached[0];
    } else if (autotune_enabled() && wblocks <= 0x7fffffffull) {
        float best = 1e30f;
        for (int c = 0; c < 2; ++c) {
            float ms = 0.f;
            SV_TRY(time_stream(st, 2, &ms, [&]() { return launch(c); }));
            if (ms < best) {
                best = ms;
                shape = c;
            }
        }
        tune_store(key, {shape});
    }
    return launch(shape);
}

template <typename R>
sv_status cgemm(hipStream_t st, const cvec<R> *in, cvec<R> *out, const cvec<R> *U, uint64_t M, int N, int K,
                uint64_t row_mask, uint64_t row_fix, int trans, int conjb) {
    return cgemm_ks<R>(st, in, out, U, M, N, K, row_mask, row_fix, 0, trans, conjb);
}
template sv_status cgemm<float>(hipStream_t, const float2 *, float2 *, const float2 *, uint64_t, int, int, uint64_t,
                                uint64_t, int, int);
template sv_status cgemm<double>(hipStream_t, const double2 *, double2 *, const double2 *, uint64_t, int, int,
                                 uint64_t, uint64_t, int, int);

// the register [lo, lo + m), controls cmask fixed to cval
template <typename R>
static sv_status ctrl_mask_unitary_at(sv_state s, const cvec<R> *U, int lo, int m, uint64_t cmask, uint64_t cval,
                                      int adjoint) {
    const uint64_t all = (s->n >= 64) ? ~0ull : ((1ull << s->n) - 1ull);
    // rows: every value of the bits outside the register and the controls,
    // with the controls fixed to cval
    const uint64_t row_mask = all & ~(((1ull << m) - 1ull) << lo) & ~cmask;
    const uint64_t row_fix = cval & cmask;
    const uint64_t M = dim_of(popcount64(row_mask));
    const int N = 1 << m;
    SV_TRY(ensure_scratch(s, (size_t)M * N * sizeof(cvec<R>)));
    cvec<R> *out = (cvec<R> *)s->scratch;
    SV_TRY(cgemm_ks<R>(s->stream, (const cvec<R> *)s->data, out, U, M, N, N, row_mask, row_fix, lo, adjoint, adjoint));
    const uint64_t total = M * (uint64_t)N;
    uint64_t g = (total + 1023) / 1024;
    if (g > (1u << 20)) g = 1u << 20;
    {
        TraceScope _ts(s->stream, "scatter_rows", 2.0 * (double)total * sizeof(cvec<R>), 0.0);
        hipLaunchKernelGGL(k_scatter_rows<R>, dim3((unsigned)g), dim3(256), 0, s->stream, (cvec<R> *)s->data,
                       (const cvec<R> *)out, M, m, row_mask, row_fix, lo);
    }
    SV_HIP(hipGetLastError());
    return SV_OK;
}

template <typename R>
sv_status ctrl_mask_unitary_impl(sv_state s, const cvec<R> *U, int m, uint64_t cmask, uint64_t cval, int adjoint) {
    return ctrl_mask_unitary_at<R>(s, U, 0, m, cmask, cval, adjoint);
}
template sv_status ctrl_mask_unitary_impl<float>(sv_state, const float2 *, int, uint64_t, uint64_t, int);
template sv_status ctrl_mask_unitary_impl<double>(sv_state, const double2 *, int, uint64_t, uint64_t, int);

template <typename R>
sv_status ctrl_unitary_impl(sv_state s, const cvec<R> *U, int m, int ctrl, int ctrl_val, int adjoint) {
    const uint64_t cm = ctrl >= 0 ? 1ull << ctrl : 0ull;
    return ctrl_mask_unitary_impl<R>(s, U, m, cm, ctrl_val ? cm : 0ull, adjoint);
}
template sv_status ctrl_unitary_impl<float>(sv_state, const float2 *, int, int, int, int);
template sv_status ctrl_unitary_impl<double>(sv_state, const double2 *, int, int, int, int);

}  // namespace sv

using namespace sv;

extern "C" sv_status sv_apply_ctrl_unitary(sv_state s, const void *U, int sys_lo, int m, int ctrl, int ctrl_val,
                                           int adjoint) {
    clear_error();
    SV_TRY(check_state(s));
    if (!U) return fail(SV_EINVAL, "U is NULL");
    if (m < 1 || sys_lo < 0 || sys_lo + m > s->n) return fail(SV_EINVAL, "register [%d,%d) outside the state", sys_lo, sys_lo + m);
    if (ctrl >= s->n || (ctrl >= sys_lo && ctrl < sys_lo + m)) return fail(SV_EINVAL, "control %d invalid", ctrl);
    if (m > 16) return fail(SV_EUNSUPPORTED, "dense register of %d qubits", m);
    const uint64_t cm = ctrl >= 0 ? 1ull << ctrl : 0ull, cv = ctrl_val ? cm : 0ull;
    if (s->dt == SV_C64)
        return ctrl_mask_unitary_at<float>(s, (const float2 *)U, sys_lo, m, cm, cv, adjoint ? 1 : 0);
    return ctrl_mask_unitary_at<double>(s, (const double2 *)U, sys_lo, m, cm, cv, adjoint ? 1 : 0);
}
