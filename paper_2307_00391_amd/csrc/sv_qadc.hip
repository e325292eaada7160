// QPP nonlinear transform (appendix "Nonlinear transform", steps 1-5): the
// amplitudes u'_s of a real 2^n-point state are turned into (u'_s)^2 on the
// amplitude of an output qubit, by a SWAP test against the address, amplitude
// estimation of the test's success probability (1 + u_s^2)/2 = sin^2(pi beta_s)
// by phase estimation, a rotation driven by the estimated phase and the
// uncompute.
//
// Layout: ua [0, n) (the loaded amplitudes), a1 [n, 2n) (the address copy),
// add [2n, 3n) (the address), a2 = 3n (the SWAP-test qubit), ub [3n+1,
// 3n+1+r) (the phase-estimation register), up = 3n+1+r (the output qubit).
//
// Operators: U_V is the real Householder reflection I - 2 v v^T / (v^T v),
// v = e_0 + sigma zeta (sigma = sign of zeta_0, +1 at 0), so U_V|0> =
// -sigma zeta; T = H(a2) CSWAP(ua <-> a1 | a2) H(a2); W = T U_V, W^dagger =
// U_V T.  The iterate is Q = -W S_0 W^dagger S_chi, S_chi the sign flip of
// a2 = 0, S_0 the sign flip of (ua = 0, a1 = address, a2 = 0).  The rotation
// on up for ub = y has sine -cos(2 pi y / 2^r) and cosine |sin(2 pi y / 2^r)|.
//
//   mode 0: gate by gate: Hadamards, CNOT copies, the dense U_V on the matrix
//           cores, the SWAP test and the reflections as fused gate passes,
//           2^r - 1 controlled iterates for phase estimation and as many for
//           its uncompute;
//   mode 1: the controlled powers fused: a (add, ub, up) column of the state
//           holds a 2^(2n+1)-amplitude (ua, a1, a2) block on which the
//           controlled Q^(2^k) of every clock bit k compose to Q^t, t the
//           column's ub value.  One workgroup keeps the block in LDS and
//           applies Q^t there (Q^dagger for the uncompute), reduced by exact
//           identities of its factors to two SWAP tests around t reflections
//           of one N-entry line (k_qadc_power), so the 2^r - 1 iterates cost
//           one read and one write of the state.  U_V is one pass of the
//           reflection on each ua row (k_qadc_loader); the remaining steps
//           are the mode-0 gates.
#include <math.h>
#include <stdlib.h>

#include <cmath>
#include <vector>

#include "sv_device.h"
#include "sv_hhl_internal.h"
#include "sv_internal.h"

namespace sv {

template <typename R>
sv_status ctrl_unitary_impl(sv_state s, const cvec<R> *U, int m, int ctrl, int ctrl_val, int adjoint);

struct QadcArgs {
    int n, r;
    uint64_t ncols;      // 2^(n + r + 1) columns (add, ub, up)
    int inverse;         // 0: Q^t, 1: (Q^dagger)^t
};

// The block in LDS: entry (ua = i, a1 = j) of row a2 at a2 N P + j P + i with
// the padded row pitch P = N + 1, so that the SWAP test's transposed reads
// (j, i) of consecutive i fall in distinct banks.

// Sum over aligned groups of N lanes (N a power of two <= 64), every lane of
// a group getting the group's sum.  Within a 16-lane row the partners come by
// DPP (lane xor 1 and xor 2 inside each quad, then the half-row and row
// mirrors), which needs no LDS round trip; 32- and 64-lane groups add the
// other rows by shuffles.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <typename R, int N>
__device__ __forceinline__ R group_sum(R x) {
    if (N >= 2) x += dpp_move<0xB1>(x);      // quad_perm [1, 0, 3, 2]
    if (N >= 4) x += dpp_move<0x4E>(x);      // quad_perm [2, 3, 0, 1]
    if (N >= 8) x += dpp_move<0x141>(x);     // row_half_mirror
    if (N >= 16) x += dpp_move<0x140>(x);    // row_mirror
    if (N >= 32) x += __shfl_xor(x, 16);
    if (N >= 64) x += __shfl_xor(x, 32);
    return x;
}

// x <- x - 2 w (w . x) over the N lanes of a line
template <typename R, int N>
__device__ __forceinline__ cvec<R> reflect_line(cvec<R> x, R w, R w2) {
    const R dx = group_sum<R, N>(w * x.x), dy = group_sum<R, N>(w * x.y);
    return cmake<R>(x.x - w2 * dx, x.y - w2 * dy);
}

// T = H(a2) CSWAP(ua <-> a1 | a2) H(a2) on the pairs (i, j), (j, i), i < j
// (the identity on i == j).  neg_before: the sign of row 1 first (-S_chi);
// neg_after: the same sign last.
template <typename R>
__device__ __forceinline__ void qadc_swap_test(cvec<R> *__restrict__ row0, cvec<R> *__restrict__ row1, int n,
                                               bool neg_before, bool neg_after) {
    const uint32_t N = 1u << n, B = N * N, P = N + 1u;
    const R h = (R)0.5;
    for (uint32_t f = threadIdx.x; f < B; f += blockDim.x) {
        const uint32_t i = f & (N - 1u), j = f >> n;
        const uint32_t e = i + j * P;
        if (i == j) {
            if (neg_before != neg_after) row1[e] = cmake<R>(-row1[e].x, -row1[e].y);
            continue;
        }
        if (i > j) continue;
        const uint32_t et = j + i * P;
        const cvec<R> p = row0[e], q = row0[et];
        cvec<R> Pv = row1[e], Qv = row1[et];
        if (neg_before) {
            Pv = cmake<R>(-Pv.x, -Pv.y);
            Qv = cmake<R>(-Qv.x, -Qv.y);
        }
        const cvec<R> spP = cmake<R>(p.x + Pv.x, p.y + Pv.y), sqQ = cmake<R>(q.x + Qv.x, q.y + Qv.y);
        const cvec<R> dqQ = cmake<R>(q.x - Qv.x, q.y - Qv.y), dpP = cmake<R>(p.x - Pv.x, p.y - Pv.y);
        const R s1 = neg_after ? -h : h;
        row0[e] = cmake<R>(h * (spP.x + dqQ.x), h * (spP.y + dqQ.y));
        row0[et] = cmake<R>(h * (sqQ.x + dpP.x), h * (sqQ.y + dpP.y));
        row1[e] = cmake<R>(s1 * (spP.x - dqQ.x), s1 * (spP.y - dqQ.y));
        row1[et] = cmake<R>(s1 * (sqQ.x - dpP.x), s1 * (sqQ.y - dpP.y));
    }
}

// One column per workgroup: rows a2 = 0 and a2 = 1 of the (ua, a1) block,
// row 1 right after row 0.  Q^t is applied through three exact identities of
// its factors: U_V^2 = I, so U_V S_0 U_V is the identity except on the
// (a2 = 0, a1 = s) column, where it is the reflection I - 2 w w^T about
// w = U_V|0>; T^2 = I; and T (-S_chi) T = Z(a2) SWAP(ua, a1).  Hence
//   Q^t = T . R . (Z SWAP) . R . ... . (Z SWAP) . R . T . (-S_chi)
// with t reflections R.  A reflection after k swaps acts on column s of the
// stored a2 = 0 plane for even k and on row s for odd k, and the (t - 1)
// swaps, pushed through the closing T, leave one sign of row 1 when t - 1 is
// odd.  The column and the row (2N - 1 entries) stay in the registers of N
// lanes of the first wavefront for all t reflections, each a dot product
// reduced across the lanes and an update.  (Q^dagger)^t is the same sequence with
// -S_chi moved to the end.
template <typename R, int NL>
__global__ __launch_bounds__(256) void k_qadc_power(cvec<R> *__restrict__ psi, const R *__restrict__ vhh, QadcArgs a) {
    extern __shared__ unsigned char lds_raw[];
    constexpr int n = NL;
    constexpr uint32_t N = 1u << NL, B = N * N, P = N + 1u;
    cvec<R> *row0 = reinterpret_cast<cvec<R> *>(lds_raw);
    cvec<R> *row1 = row0 + N * P;
    for (uint64_t col = blockIdx.x; col < a.ncols; col += gridDim.x) {
        const uint32_t s = (uint32_t)(col & (N - 1u));
        const uint32_t t = (uint32_t)((col >> n) & ((1ull << a.r) - 1ull));
        if (t == 0) continue;                        // Q^0: the column is left as it is
        const uint64_t hi = col >> n;                // (ub, up), placed above a2
        const uint64_t base = ((uint64_t)s << (2 * n)) | (hi << (3 * n + 1));
        const uint64_t off1 = 1ull << (3 * n);
        for (uint32_t e = threadIdx.x; e < B; e += blockDim.x) {
            const uint32_t l = (e & (N - 1u)) + (e >> n) * P;
            row0[l] = psi[base | e];
            row1[l] = psi[base | off1 | e];
        }
        __syncthreads();
        qadc_swap_test<R>(row0, row1, n, !a.inverse, false);
        __syncthreads();
        if (threadIdx.x < N) {
            const uint32_t i = threadIdx.x;
            const R c = vhh[N];
            const R w = (i == 0 ? (R)1 : (R)0) - c * vhh[i] * vhh[0];   // U_V|0>
            const R w2 = w + w;
            cvec<R> cl = row0[i + s * P];            // column s: (i, s)
            cvec<R> rw = row0[s + i * P];            // row s: (s, i)
            // reflections alternate: column s (even k), row s (odd k); lane s
            // holds the shared entry (s, s) in both
            for (uint32_t k = 0; k + 1 < t; k += 2) {
                cl = reflect_line<R, N>(cl, w, w2);
                if (i == s) rw = cl;
                rw = reflect_line<R, N>(rw, w, w2);
                if (i == s) cl = rw;
            }
            if (t & 1u) {
                cl = reflect_line<R, N>(cl, w, w2);
                if (i == s) rw = cl;
            }
            row0[i + s * P] = cl;
            row0[s + i * P] = rw;
        }
        __syncthreads();
        qadc_swap_test<R>(row0, row1, n, false, (((t - 1u) & 1u) != 0u) != (a.inverse != 0));
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < B; e += blockDim.x) {
            const uint32_t l = (e & (N - 1u)) + (e >> n) * P;
            psi[base | e] = row0[l];
            psi[base | off1 | e] = row1[l];
        }
        __syncthreads();
    }
}

// The same Q^t for n = 3 and 4, with 64 / N columns of equal t in one
// wavefront: the (address, up) pairs sharing a ub value t are consecutive in
// groups of G = 64 / N, lane l works on line entry l mod N of column l / N, and
// the DPP sums stay inside each N-lane group, so every lane of the wave takes
// part in the reflections (one column per wave left 64 - N lanes idle).
template <typename R, int NL>
__global__ __launch_bounds__(64) void k_qadc_power_packed(cvec<R> *__restrict__ psi, const R *__restrict__ vhh,
                                                          QadcArgs a) {
    extern __shared__ unsigned char lds_raw[];
    constexpr int n = NL;
    constexpr uint32_t N = 1u << NL, B = N * N, P = N + 1u, G = 64u / N;
    constexpr uint32_t per_t = 2u * N / G;           // groups per ub value
    cvec<R> *blk = reinterpret_cast<cvec<R> *>(lds_raw);       // G blocks of 2 N P entries
    const uint64_t ngroups = (1ull << a.r) * per_t;
    const uint64_t off1 = 1ull << (3 * n);
    for (uint64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const uint32_t t = (uint32_t)(grp / per_t);
        if (t == 0) continue;                        // Q^0: the columns are left as they are
        const uint32_t c0 = (uint32_t)(grp % per_t) * G;          // first (address, up) pair
        // column j of the group: address (c0 + j) mod N, up = (c0 + j) / N
        for (uint32_t e = threadIdx.x; e < G * B; e += 64) {
            const uint32_t j = e / B, f = e % B, cc = c0 + j;
            const uint64_t base = ((uint64_t)(cc & (N - 1u)) << (2 * n)) |
                                  (((uint64_t)t | ((uint64_t)(cc >> n) << a.r)) << (3 * n + 1));
            const uint32_t l = j * 2u * N * P + (f & (N - 1u)) + (f >> n) * P;
            blk[l] = psi[base | f];
            blk[l + N * P] = psi[base | off1 | f];
        }
        __syncthreads();
        for (uint32_t j = 0; j < G; ++j)
            qadc_swap_test<R>(blk + j * 2u * N * P, blk + j * 2u * N * P + N * P, n, !a.inverse, false);
        __syncthreads();
        {
            const uint32_t l = threadIdx.x, j = l >> n, i = l & (N - 1u);
            const uint32_t sj = (c0 + j) & (N - 1u);
            cvec<R> *X = blk + j * 2u * N * P;
            const R c = vhh[N];
            const R w = (i == 0 ? (R)1 : (R)0) - c * vhh[i] * vhh[0];   // U_V|0>
            const R w2 = w + w;
            cvec<R> cl = X[i + sj * P];              // column sj: (i, sj)
            cvec<R> rw = X[sj + i * P];              // row sj: (sj, i)
            for (uint32_t k = 0; k + 1 < t; k += 2) {
                cl = reflect_line<R, N>(cl, w, w2);
                if (i == sj) rw = cl;
                rw = reflect_line<R, N>(rw, w, w2);
                if (i == sj) cl = rw;
            }
            if (t & 1u) {
                cl = reflect_line<R, N>(cl, w, w2);
                if (i == sj) rw = cl;
            }
            X[i + sj * P] = cl;
            X[sj + i * P] = rw;
        }
        __syncthreads();
        const bool neg = (((t - 1u) & 1u) != 0u) != (a.inverse != 0);
        for (uint32_t j = 0; j < G; ++j)
            qadc_swap_test<R>(blk + j * 2u * N * P, blk + j * 2u * N * P + N * P, n, false, neg);
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < G * B; e += 64) {
            const uint32_t j = e / B, f = e % B, cc = c0 + j;
            const uint64_t base = ((uint64_t)(cc & (N - 1u)) << (2 * n)) |
                                  (((uint64_t)t | ((uint64_t)(cc >> n) << a.r)) << (3 * n + 1));
            const uint32_t l = j * 2u * N * P + (f & (N - 1u)) + (f >> n) * P;
            psi[base | f] = blk[l];
            psi[base | off1 | f] = blk[l + N * P];
        }
        __syncthreads();
    }
}

// U_V on the ua register ([0, n), contiguous) of every row in one pass: each
// aligned group of N lanes holds one row, forms v.z with DPP sums and writes
// z - c v (v.z).  The state has at least 64 amplitudes, a multiple of the
// 64-lane stride, so every group runs its loop trips together.
template <typename R, int NL>
__global__ __launch_bounds__(256) void k_qadc_loader(cvec<R> *__restrict__ psi, const R *__restrict__ vhh,
                                                     uint64_t total) {
    constexpr uint32_t N = 1u << NL;
    const uint32_t i = threadIdx.x & (N - 1u);
    const R c = vhh[N], vi = vhh[i];
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (uint64_t)gridDim.x * blockDim.x) {
        cvec<R> z = psi[idx];
        const R dx = c * group_sum<R, N>(vi * z.x), dy = c * group_sum<R, N>(vi * z.y);
        z.x -= vi * dx;
        z.y -= vi * dy;
        psi[idx] = z;
    }
}

namespace {

struct Layout {
    int n, r;
    int ua() const { return 0; }
    int a1() const { return n; }
    int add() const { return 2 * n; }
    int a2() const { return 3 * n; }
    int ub() const { return 3 * n + 1; }
    int up() const { return 3 * n + 1 + r; }
};

// the Householder vector v = e_0 + sigma zeta of the loader, FP64
void loader_vector(const std::vector<double> &zeta, std::vector<double> &v, double &c) {
    const double sigma = zeta[0] >= 0.0 ? 1.0 : -1.0;
    v.resize(zeta.size());
    double vv = 0.0;
    for (size_t i = 0; i < zeta.size(); ++i) {
        v[i] = sigma * zeta[i] + (i == 0 ? 1.0 : 0.0);
        vv += v[i] * v[i];
    }
    c = 2.0 / vv;
}

sv_gate gate_u(int target, double a, double b, double cc, double d) {
    sv_gate g{};
    g.kind = SV_GATE_U;
    g.target = target;
    g.u[0] = a;
    g.u[2] = b;
    g.u[4] = cc;
    g.u[6] = d;
    return g;
}
sv_gate gate_ctrl(sv_gate g, int ctrl, int val) {
    g.ctrls[g.n_ctrls] = ctrl;
    g.ctrl_vals[g.n_ctrls] = val;
    ++g.n_ctrls;
    return g;
}

// SV_QADC_PACKED=0 keeps one column per workgroup for every address width
int packed_env() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("SV_QADC_PACKED");
        v = (e && atoi(e) == 0) ? 0 : 1;
    }
    return v;
}

class Qadc {
public:
    Qadc(sv_state s, int n, int r) : s_(s), L{n, r} {}

    sv_status prepare(const std::vector<double> &zeta) {
        std::vector<double> v;
        double c;
        loader_vector(zeta, v, c);
        const int N = 1 << L.n;
        const size_t eb = amp_bytes(s_->dt);
        // dense U_V in the state's precision (mode 0)
        SV_TRY(U_.ensure((size_t)N * N * eb));
        if (s_->dt == SV_C64) {
            std::vector<float2> U((size_t)N * N);
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j) U[(size_t)i * N + j] = make_float2((float)((i == j) - c * v[i] * v[j]), 0.f);
            SV_TRY(upload(s_, U_.p, U.data(), U.size() * sizeof(float2)));
            std::vector<float> vh(N + 1);
            for (int i = 0; i < N; ++i) vh[i] = (float)v[i];
            vh[N] = (float)c;
            SV_TRY(vh_.ensure(vh.size() * sizeof(float)));
            SV_TRY(upload(s_, vh_.p, vh.data(), vh.size() * sizeof(float)));
        } else {
            std::vector<double2> U((size_t)N * N);
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j) U[(size_t)i * N + j] = make_double2((i == j) - c * v[i] * v[j], 0.0);
            SV_TRY(upload(s_, U_.p, U.data(), U.size() * sizeof(double2)));
            std::vector<double> vh(v);
            vh.push_back(c);
            SV_TRY(vh_.ensure(vh.size() * sizeof(double)));
            SV_TRY(upload(s_, vh_.p, vh.data(), vh.size() * sizeof(double)));
        }
        return SV_OK;
    }

    // the queued gates, as one fused circuit
    sv_status flush() {
        if (q_.empty()) return SV_OK;
        sv_status st = sv_apply_circuit(s_, q_.data(), (int)q_.size(), 0);
        q_.clear();
        return st;
    }
    void h(int q) {
        const double k = M_SQRT1_2;
        q_.push_back(gate_u(q, k, k, k, -k));
    }
    void copy_address() {
        for (int j = 0; j < L.n; ++j) {
            sv_gate g{};
            g.kind = SV_GATE_X;
            g.target = L.a1() + j;
            q_.push_back(gate_ctrl(g, L.add() + j, 1));
        }
    }
    void swap_test() {
        h(L.a2());
        for (int j = 0; j < L.n; ++j) {
            sv_gate g{};
            g.kind = SV_GATE_SWAP;
            g.target = L.ua() + j;
            g.target2 = L.a1() + j;
            q_.push_back(gate_ctrl(g, L.a2(), 1));
        }
        h(L.a2());
    }
    sv_status loader() {
        SV_TRY(flush());
        if (fused_ && L.n <= 6) {
            if (s_->dt == SV_C64) return launch_loader<float>();
            return launch_loader<double>();
        }
        if (s_->dt == SV_C64) return ctrl_unitary_impl<float>(s_, (const float2 *)U_.p, L.n, -1, 0, 0);
        return ctrl_unitary_impl<double>(s_, (const double2 *)U_.p, L.n, -1, 0, 0);
    }
    template <typename R, int NL>
    sv_status loader_one() {
        const uint64_t total = dim_of(s_->n);
        uint64_t g = total / 256;
        if (g < 1) g = 1;
        if (g > (1u << 20)) g = 1u << 20;
        TraceScope ts(s_->stream, "qadc_loader", 2.0 * (double)total * sizeof(cvec<R>), 16.0 * (double)total);
        hipLaunchKernelGGL((k_qadc_loader<R, NL>), dim3((unsigned)g), dim3(256), 0, s_->stream, (cvec<R> *)s_->data,
                           (const R *)vh_.p, total);
        SV_HIP(hipGetLastError());
        return SV_OK;
    }
    template <typename R>
    sv_status launch_loader() {
        switch (L.n) {
        case 1: return loader_one<R, 1>();
        case 2: return loader_one<R, 2>();
        case 3: return loader_one<R, 3>();
        case 4: return loader_one<R, 4>();
        case 5: return loader_one<R, 5>();
        default: return loader_one<R, 6>();
        }
    }
    sv_status W() {
        SV_TRY(loader());
        swap_test();
        return SV_OK;
    }
    sv_status W_dagger() {
        swap_test();
        return loader();
    }
    void s_chi(int c) { q_.push_back(gate_ctrl(gate_u(L.a2(), -1, 0, 0, 1), c, 1)); }
    sv_status s_0(int c) {
        copy_address();
        SV_TRY(flush());
        int ctrls[32], vals[32];
        int k = 0;
        for (int j = 0; j < 2 * L.n; ++j) {
            ctrls[k] = L.ua() + j;      // ua then a1: bits [0, 2n)
            vals[k++] = 0;
        }
        ctrls[k] = c;
        vals[k++] = 1;
        const double flip0[8] = {-1, 0, 0, 0, 0, 0, 1, 0};
        SV_TRY(sv_apply_gate(s_, L.a2(), flip0, ctrls, vals, k));
        copy_address();
        return SV_OK;
    }
    sv_status controlled_q(int c, bool inverse) {
        if (!inverse) {
            s_chi(c);
            SV_TRY(W_dagger());
            SV_TRY(s_0(c));
            SV_TRY(W());
        } else {
            SV_TRY(W_dagger());
            SV_TRY(s_0(c));
            SV_TRY(W());
            s_chi(c);
        }
        q_.push_back(gate_u(c, 1, 0, 0, -1));   // the iterate's minus sign, on its control
        return SV_OK;
    }

    template <typename R, int NL>
    sv_status launch_one(const QadcArgs &a, size_t lds, int nt, unsigned g) {
        if (lds > 65536)
            SV_HIP(hipFuncSetAttribute((const void *)k_qadc_power<R, NL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds));
        hipLaunchKernelGGL((k_qadc_power<R, NL>), dim3(g), dim3(nt), lds, s_->stream, (cvec<R> *)s_->data,
                           (const R *)vh_.p, a);
        return SV_OK;
    }
    template <typename R, int NL>
    sv_status launch_packed(const QadcArgs &a) {
        constexpr uint32_t N = 1u << NL, G = 64u / N;
        const size_t lds = (size_t)G * 2 * N * (N + 1) * sizeof(cvec<R>);
        uint64_t groups = (1ull << a.r) * (2ull * N / G);
        if (groups > (1u << 20)) groups = 1u << 20;
        hipLaunchKernelGGL((k_qadc_power_packed<R, NL>), dim3((unsigned)groups), dim3(64), lds, s_->stream,
                           (cvec<R> *)s_->data, (const R *)vh_.p, a);
        return SV_OK;
    }
    template <typename R>
    sv_status launch_power(const QadcArgs &a, size_t lds, int nt, unsigned g) {
        if (packed_env()) {
            if (a.n == 3) return launch_packed<R, 3>(a);
            if (a.n == 4) return launch_packed<R, 4>(a);
        }
        switch (a.n) {
        case 1: return launch_one<R, 1>(a, lds, nt, g);
        case 2: return launch_one<R, 2>(a, lds, nt, g);
        case 3: return launch_one<R, 3>(a, lds, nt, g);
        case 4: return launch_one<R, 4>(a, lds, nt, g);
        case 5: return launch_one<R, 5>(a, lds, nt, g);
        case 6: return launch_one<R, 6>(a, lds, nt, g);
        default: return fail(SV_EUNSUPPORTED, "fused powers need n <= 6");
        }
    }

    // every controlled power of the iterate at once: Q^t on the column with ub = t
    sv_status fused_powers(bool inverse) {
        SV_TRY(flush());
        QadcArgs a;
        a.n = L.n;
        a.r = L.r;
        a.ncols = dim_of(L.n + L.r + 1);
        a.inverse = inverse ? 1 : 0;
        const int N = 1 << L.n;
        const size_t eb = amp_bytes(s_->dt);
        const size_t lds = 2 * (size_t)N * (N + 1) * eb;
        // one wavefront per column up to n = 4 (a 512-amplitude block), four above
        const int nt = L.n <= 4 ? 64 : 256;
        uint64_t g = a.ncols;
        if (g > (1u << 20)) g = 1u << 20;
        // per launch: every (add, up) pair runs t = 0 .. 2^r - 1 reflections of
        // 8 N flops each; every column with t > 0 two SWAP tests of 12 N^2 flops
        const double M = (double)(1ull << L.r);
        const double refl = (M - 1.0) * M / 2.0 * (double)(2ull * N);
        const double cols = (double)a.ncols * (M - 1.0) / M;
        TraceScope ts(s_->stream, "qadc_power", 2.0 * cols * 2.0 * N * N * eb, refl * 8.0 * N + cols * 24.0 * N * N);
        if (s_->dt == SV_C64) SV_TRY(launch_power<float>(a, lds, nt, (unsigned)g));
        else SV_TRY(launch_power<double>(a, lds, nt, (unsigned)g));
        SV_HIP(hipGetLastError());
        return SV_OK;
    }

    sv_status run(int mode, int avg, const std::vector<double> &zeta, double *sq_out, sv_qadc_result *res) {
        fused_ = mode == 1;
        SV_TRY(prepare(zeta));
        SV_TRY(sv_init_basis(s_, 0));
        const int n = L.n, r = L.r;
        const uint64_t M = 1ull << r;
        for (int j = 0; j < n; ++j) h(L.add() + j);                  // step 1
        copy_address();
        SV_TRY(W());                                                 // steps 2-3
        for (int k = 0; k < r; ++k) h(L.ub() + k);                   // step 4
        if (mode == 1) {
            SV_TRY(fused_powers(false));
        } else {
            for (int k = 0; k < r; ++k)
                for (uint64_t i = 0; i < (1ull << k); ++i) SV_TRY(controlled_q(L.ub() + k, false));
        }
        SV_TRY(flush());
        SV_TRY(sv_qft(s_, L.ub(), r, 1, 1, 0));
        std::vector<double> cs(2 * M);                               // step 5
        for (uint64_t y = 0; y < M; ++y) {
            const double ang = 2.0 * M_PI * (double)y / (double)M;
            cs[2 * y] = fabs(sin(ang));
            cs[2 * y + 1] = -cos(ang);
        }
        SV_TRY(sv_apply_uniform_ry(s_, L.up(), L.ub(), r, cs.data(), -1, 0));
        SV_TRY(sv_qft(s_, L.ub(), r, 0, 1, 0));                      // undo phase estimation
        if (mode == 1) {
            SV_TRY(fused_powers(true));
        } else {
            for (int k = r - 1; k >= 0; --k)
                for (uint64_t i = 0; i < (1ull << k); ++i) SV_TRY(controlled_q(L.ub() + k, true));
        }
        for (int k = 0; k < r; ++k) h(L.ub() + k);
        SV_TRY(W_dagger());
        copy_address();
        SV_TRY(flush());
        // the squares: the up = 1 block with every ancilla at 0, times sqrt(N)
        const uint64_t upbit = 1ull << L.up();
        const uint64_t all = dim_of(s_->n) - 1ull;
        const uint64_t addmask = ((1ull << n) - 1ull) << L.add();
        const int N = 1 << n;
        double p = 0.0;
        SV_TRY(sv_norm2(s_, all & ~addmask, upbit, &p));
        res->p_sq = p;
        SV_TRY(sv_norm2(s_, upbit, upbit, &res->p_up));
        if (sq_out) {
            if (p > 0.0) {
                std::vector<double> z(2 * (size_t)N);
                SV_TRY(sv_postselect(s_, all & ~addmask, upbit, &p, z.data(), 0));
                const double k = sqrt(p * (double)N);
                for (int i = 0; i < N; ++i) sq_out[i] = z[2 * i] * k;
            } else {
                for (int i = 0; i < N; ++i) sq_out[i] = 0.0;
            }
        }
        res->avg = 0.0;
        if (avg) {
            SV_TRY(run_hadamards(s_, L.add(), n, 0, 0));             // U_avg
            double p0 = 0.0;
            SV_TRY(sv_norm2(s_, all, upbit, &p0));
            if (p0 > 0.0) {
                double z[2];
                SV_TRY(sv_postselect(s_, all, upbit, &p0, z, 0));
                res->avg = z[0] * sqrt(p0);
            }
        }
        return SV_OK;
    }

private:
    sv_state s_;
    Layout L;
    DevBuf U_, vh_;
    std::vector<sv_gate> q_;
    bool fused_ = false;     // mode 1: U_V as the one-pass reflection kernel
};

}  // namespace
}  // namespace sv

using namespace sv;

extern "C" sv_status sv_qadc_square(sv_state s, const double *u, int n, int r, int mode, int avg, double *sq_out,
                                    sv_qadc_result *res) {
    clear_error();
    SV_TRY(check_state(s));
    if (!u || !res) return fail(SV_EINVAL, "u and res must not be NULL");
    if (n < 1 || n > 10) return fail(SV_EINVAL, "n = %d outside 1..10", n);
    if (r < 1 || r > 16) return fail(SV_EINVAL, "r = %d outside 1..16", r);
    if (3 * n + r + 2 != s->n)
        return fail(SV_EINVAL, "the state has %d qubits; 3n + r + 2 = %d", s->n, 3 * n + r + 2);
    if (mode != 0 && mode != 1) return fail(SV_EINVAL, "mode must be 0 or 1");
    if (mode == 1 && n > 6) return fail(SV_EUNSUPPORTED, "mode 1 keeps the 2^(2n+1) block in LDS: n <= 6");
    const int N = 1 << n;
    std::vector<double> zeta(u, u + N);
    double nrm = 0.0;
    for (int i = 0; i < N; ++i) {
        if (!std::isfinite(zeta[i])) return fail(SV_EINVAL, "u[%d] is not finite", i);
        nrm += zeta[i] * zeta[i];
    }
    if (nrm == 0.0) return fail(SV_EZERONORM, "u = 0");
    nrm = sqrt(nrm);
    for (double &z : zeta) z /= nrm;
    Qadc q(s, n, r);
    SV_TRY(q.run(mode, avg, zeta, sq_out, res));
    SV_HIP(hipStreamSynchronize(s->stream));
    return SV_OK;
}
