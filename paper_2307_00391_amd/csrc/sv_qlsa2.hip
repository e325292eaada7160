// QLSA-2: a linear-systems solver by a linear combination of unitaries over a
// qubitized walk (main text, "Quantum Linear Systems Algorithm": the second
// family of solvers, whose construction the paper takes from the cited work
// of Childs, Kothari and Somma and does not spell out).
//
// The odd polynomial g(x) = (1 - (1 - x^2)^B) / x = sum_j alpha_j T_{2j+1}(x),
// alpha_j = 4 (-1)^j sum_{i>j} C(2B, B+i) / 4^B, approximates 1/x on
// 1/kappa <= |x| <= 1.  A~ = A / max|lambda| is block-encoded on one walk
// qubit, U = [[A~, S], [S, -A~]] with S = sqrt(I - A~^2), and the walk
// W = (Z on the walk qubit) U has T_k(A~) as the walk-0 block of W^k.  With
// the select register (J = 2^s terms) prepared in sqrt(|alpha_j| / |alpha|_1),
// SELECT W^(2j+1), the signs (-1)^j as one Z on the lowest select qubit and
// PREP^dagger, the select = 0, walk = 0 block is g(A~) b^ / |alpha|_1.
//
// Layout: bits [0, n_s) system, bit n_s the walk qubit, [n_s + 1, n_s + 1 + s)
// the select register.
//   mode 0: the circuit in the computational basis: PREP and PREP^dagger as
//           the QSP-1 tree of uniformly controlled Ry passes on the select
//           register, W once and one controlled W^(2^(m+1)) per select qubit
//           as dense unitaries of the (walk, system) register on the matrix
//           cores (built in FP64 from the eigen-decomposition of A), the sign
//           gate, post-selection;
//   mode 1: the same circuit with the system register held in the eigenbasis
//           of A, where W^(2j+1) is a rotation of the walk qubit by (2j+1)
//           theta_k, theta_k = arccos(lambda~_k): one pass writes the state
//           after PREP, SELECT and the signs, a second forms the select = 0
//           projection of PREP^dagger (an FP64 sum over the select values).
#include <math.h>

#include <vector>

#include "sv_device.h"
#include "sv_hhl_internal.h"
#include "sv_internal.h"

namespace sv {

template <typename R>
sv_status cgemm(hipStream_t st, const cvec<R> *in, cvec<R> *out, const cvec<R> *U, uint64_t M, int N, int K,
                uint64_t row_mask, uint64_t row_fix, int trans, int conjb);
template <typename R>
sv_status ctrl_unitary_impl(sv_state s, const cvec<R> *U, int m, int ctrl, int ctrl_val, int adjoint);
template <typename R>
sv_status ctrl_mask_unitary_impl(sv_state s, const cvec<R> *U, int m, uint64_t cmask, uint64_t cval, int adjoint);

static unsigned grid_for(uint64_t items) {
    uint64_t g = (items + 255) / 256;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

// alpha_j, j < J (zero for j >= B): t_i = C(2B, B+i) / 4^B from
// t_0 = prod_{k<=B} (2k - 1) / (2k) and t_{i+1} = t_i (B - i) / (B + i + 1),
// tails summed from the small end
static void cheb_coeffs(int B, int J, std::vector<double> &alpha) {
    std::vector<double> tail((size_t)B + 2, 0.0);
    double t = 1.0;
    for (int k = 1; k <= B; ++k) t *= (2.0 * k - 1.0) / (2.0 * k);
    std::vector<double> term((size_t)B + 1);
    term[0] = t;
    for (int i = 0; i < B; ++i) term[i + 1] = term[i] * (double)(B - i) / (double)(B + i + 1);
    double acc = 0.0;
    for (int i = B; i >= 0; --i) {
        acc += term[i];
        tail[i] = acc;
    }
    alpha.assign(J, 0.0);
    for (int j = 0; j < J && j + 1 <= B; ++j) alpha[j] = ((j & 1) ? -4.0 : 4.0) * tail[j + 1];
}

// the QSP-1 tree for real non-negative amplitudes w on the register
// [q_lo, q_lo + m) of the current state (no initialisation), or its adjoint
static sv_status tree_circuit(sv_state s, const std::vector<double> &amp, int q_lo, int m, bool adjoint) {
    const uint64_t R = 1ull << m;
    std::vector<double> w(2 * R, 0.0);
    for (uint64_t r = 0; r < R; ++r) w[R + r] = amp[r] * amp[r];
    for (uint64_t k = R - 1; k >= 1; --k) w[k] = w[2 * k] + w[2 * k + 1];
    const double sg = adjoint ? -1.0 : 1.0;
    const int top = q_lo + m - 1;
    std::vector<double> lv;
    for (int li = 0; li < m; ++li) {
        const int l = adjoint ? m - 1 - li : li;
        const uint64_t P = 1ull << l;
        lv.assign(2 * P, 0.0);
        for (uint64_t p = 0; p < P; ++p) {
            const uint64_t node = P + p;
            if (w[node] > 0.0) {
                lv[2 * p] = sqrt(w[2 * node] / w[node]);
                lv[2 * p + 1] = sg * sqrt(w[2 * node + 1] / w[node]);
            } else {
                lv[2 * p] = 1.0;
                lv[2 * p + 1] = 0.0;
            }
        }
        if (l == 0) {
            const double u[8] = {lv[0], 0.0, -lv[1], 0.0, lv[1], 0.0, lv[0], 0.0};
            SV_TRY(sv_apply_gate(s, top, u, nullptr, nullptr, 0));
        } else {
            SV_TRY(sv_apply_uniform_ry(s, top - l, top - l + 1, l, lv.data(), -1, 0));
        }
    }
    return SV_OK;
}

// turn fraction (64-bit) of theta_k / 2 pi, theta_k = arccos(lambda_k / lmax)
static void walk_turns(const std::vector<double> &lam, double lmax, std::vector<uint64_t> &t) {
    t.resize(lam.size());
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (size_t k = 0; k < lam.size(); ++k) {
        long double x = (long double)lam[k] / (long double)lmax;
        if (x > 1.0L) x = 1.0L;
        if (x < -1.0L) x = -1.0L;
        const long double f = acosl(x) / two_pi;              // in [0, 1/2]
        t[k] = (uint64_t)llroundl(ldexpl(f, 63)) << 1;         // f 2^64, even (exact for f = 1/2)
    }
}

// (cos, sin) of the power-k walk angle as FP64, one row of E per block (c) and (s)
__global__ void k_walk_cs(double2 *__restrict__ Ec, double2 *__restrict__ Es, const uint64_t *__restrict__ t,
                          uint64_t power, int N) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
        const double2 e = turn_phase_f64(t[k] * power);
        Ec[k] = make_double2(e.x, 0.0);
        Es[k] = make_double2(e.y, 0.0);
    }
}

// W^k = [[P, Q], [-Q, P]] with P = V C V^H, Q = V S V^H, in the state's dtype;
// row/column index = (walk << n_s) | x
template <typename R>
__global__ void k_walk_assemble(cvec<R> *__restrict__ Wk, const double2 *__restrict__ P, const double2 *__restrict__ Q,
                                int N) {
    const uint64_t M = 2ull * N, total = M * M;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = i / M, c = i % M;
        const uint64_t ra = r / N, ca = c / N, rx = r % N, cx = c % N;
        double2 v = (ra == ca) ? P[rx * N + cx] : Q[rx * N + cx];
        if (ra == 1 && ca == 0) v = make_double2(-v.x, -v.y);
        Wk[i] = cmake<R>((R)v.x, (R)v.y);
    }
}

// mode 1: the state after PREP, SELECT and the signs, in the eigen frame:
// psi[j][walk][k] = (-1)^j p_j beta_k (cos, -sin)((2j+1) theta_k)
template <typename R>
__global__ __launch_bounds__(256) void k_cheb_select(cvec<R> *__restrict__ psi, const double2 *__restrict__ beta,
                                                     const double *__restrict__ pj, const uint64_t *__restrict__ t,
                                                     int n_s, uint64_t J) {
    const uint64_t N = 1ull << n_s, total = J * N;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const uint64_t j = i >> n_s, k = i & (N - 1);
        const double2 bk = beta[k];
        const double a = ((j & 1) ? -1.0 : 1.0) * pj[j];
        const cvec<R> e = turn_phase<R>(t[k] * (2 * j + 1));
        const cvec<R> amp = cmake<R>((R)(a * bk.x), (R)(a * bk.y));
        const uint64_t base = (j << (n_s + 1)) | k;
        psi[base] = cmake<R>(e.x * amp.x, e.x * amp.y);
        psi[base | N] = cmake<R>(-e.y * amp.x, -e.y * amp.y);
    }
}

// The select = 0 projection of PREP^dagger, z_k = sum_r p_r psi[(r << shift) | k]
// with p_r = pw[r >> wshift] (FP64, fixed order), in two passes.  Pass 1: block (x, y) takes the columns
// [y W, y W + W), W = min(N, 256), and the select rows [x L, x L + L); its 256
// threads read 256 / W rows per step, consecutive threads at consecutive
// addresses when shift = n_s; part[x][k] holds the block's sum.
template <typename R>
__global__ __launch_bounds__(256) void k_select_partial(const cvec<R> *__restrict__ psi, const double *__restrict__ pr,
                                                        double2 *__restrict__ part, int n_s, int shift, int wshift,
                                                        uint64_t nsel, uint64_t rows) {
    __shared__ double sr[256], si[256];
    const int lw = n_s < 8 ? n_s : 8;
    const uint64_t W = 1ull << lw, P = 256u >> lw;
    const uint64_t lane = threadIdx.x & (W - 1), sub = threadIdx.x >> lw;
    const uint64_t col = ((uint64_t)blockIdx.y << lw) | lane;
    const uint64_t r0 = (uint64_t)blockIdx.x * rows, r1 = r0 + rows < nsel ? r0 + rows : nsel;
    double ar = 0.0, ai = 0.0;
    for (uint64_t r = r0 + sub; r < r1; r += P) {
        const cvec<R> v = psi[(r << shift) | col];
        const double w = pr[r >> wshift];
        ar += w * (double)v.x;
        ai += w * (double)v.y;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    if (sub == 0) {
        double tr = 0.0, ti = 0.0;
        for (uint64_t q = 0; q < P; ++q) {
            tr += sr[(q << lw) | lane];
            ti += si[(q << lw) | lane];
        }
        part[((uint64_t)blockIdx.x << n_s) | col] = make_double2(tr, ti);
    }
}

// Pass 2: one block per column k sums part[x][k] over the chunks x (each
// thread a fixed stride of chunks, then a fixed-shape tree)
__global__ __launch_bounds__(256) void k_select_finish(const double2 *__restrict__ part, double2 *__restrict__ z,
                                                       int n_s, unsigned chunks) {
    __shared__ double sr[4], si[4];
    const uint64_t k = blockIdx.x;
    double ar = 0.0, ai = 0.0;
    for (unsigned x = threadIdx.x; x < chunks; x += blockDim.x) {
        const double2 v = part[((uint64_t)x << n_s) | k];
        ar += v.x;
        ai += v.y;
    }
    ar = wave_sum_f64(ar);
    ai = wave_sum_f64(ai);
    if ((threadIdx.x & 63) == 0) {
        sr[threadIdx.x >> 6] = ar;
        si[threadIdx.x >> 6] = ai;
    }
    __syncthreads();
    if (threadIdx.x == 0) z[k] = make_double2((sr[0] + sr[1]) + (sr[2] + sr[3]), (si[0] + si[1]) + (si[2] + si[3]));
}

// z (N FP64 entries, device) from the state: chunking chosen for about 2048
// blocks in pass 1; the partial sums take at most 2^20 complex entries
template <typename R>
static sv_status select_project(sv_state s, const double *pr, double2 *z, int n_s, int shift, int wshift,
                                uint64_t nsel, const char *label) {
    const hipStream_t st = s->stream;
    const int lw = n_s < 8 ? n_s : 8;
    const uint64_t N = 1ull << n_s, P = 256u >> lw, gy = N >> lw;
    uint64_t chunks = 2048 / gy;
    if (chunks < 1) chunks = 1;
    const uint64_t steps = (nsel + P - 1) / P;
    if (chunks > steps) chunks = steps;
    const uint64_t rows = ((nsel + chunks - 1) / chunks + P - 1) / P * P;
    chunks = (nsel + rows - 1) / rows;
    DevBuf part;
    SV_TRY(part.alloc(chunks * N * sizeof(double2)));
    {
        TraceScope ts(st, label, (double)(nsel * N) * sizeof(cvec<R>), 0.0);
        hipLaunchKernelGGL(k_select_partial<R>, dim3((unsigned)chunks, (unsigned)gy), dim3(256), 0, st,
                           (const cvec<R> *)s->data, pr, (double2 *)part.p, n_s, shift, wshift, nsel, rows);
        hipLaunchKernelGGL(k_select_finish, dim3((unsigned)N), dim3(256), 0, st, (const double2 *)part.p, z, n_s,
                           (unsigned)chunks);
    }
    SV_HIP(hipGetLastError());
    // the partial buffer is released by its destructor: wait for the kernels first
    SV_HIP(hipStreamSynchronize(st));
    return SV_OK;
}

// Fourier form, eigen frame: psi[r][k] = p_m beta_k i sign(z) e^{-i lambda~_k y_j z_k}
// for r = j + 2^sy m, y_j = j dy, z_k = k dz with k = m + 1 (m < K) or m - 2K (the
// PREP amplitude p_m depends on m only).
// complex128: the argument -lambda~_k (j dy k dz) in FP64 and an FP64 sincos;
// complex64: the phase as an exact 64-bit turn count, -F_k j k mod 2^64 with
// F_k = lambda~_k dy dz / 2 pi in units of 2^-64 turns, and an FP32 sincospi.
// The factor i sign(z) swaps the components.
template <typename R>
__global__ __launch_bounds__(256) void k_fourier_select(cvec<R> *__restrict__ psi, const double2 *__restrict__ beta,
                                                        const double *__restrict__ pr, const double *__restrict__ lamt,
                                                        const uint64_t *__restrict__ F, int n_s, int sy, int sz,
                                                        double dy, double dz) {
    const uint64_t N = 1ull << n_s, total = (1ull << (sy + sz)) << n_s;
    const int64_t K = (int64_t)1 << (sz - 1);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const uint64_t r = i >> n_s, k = i & (N - 1);
        const int64_t j = (int64_t)(r & ((1ull << sy) - 1ull));
        const int64_t m = (int64_t)(r >> sy);
        const int64_t kk = m < K ? m + 1 : m - 2 * K;
        cvec<R> e;
        if (sizeof(R) == 8) {
            const double t = (double)j * dy * (double)kk * dz;
            double sd, cd;
            sincos(-lamt[k] * t, &sd, &cd);
            e = cmake<R>((R)cd, (R)sd);
        } else {
            e = turn_phase<R>((uint64_t)0 - F[k] * (uint64_t)(j * kk));
        }
        const double2 bk = beta[k];
        const double a = pr[m];
        const R ar = (R)(a * bk.x), ai = (R)(a * bk.y);
        const R xr = e.x * ar - e.y * ai, xi = e.x * ai + e.y * ar;
        psi[i] = kk > 0 ? cmake<R>(-xi, xr) : cmake<R>(xi, -xr);
    }
}

template <typename R>
__global__ void k_round_unitary(cvec<R> *__restrict__ out, const double2 *__restrict__ in, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = cmake<R>((R)in[i].x, (R)in[i].y);
}

// Fourier form, gate by gate in the computational basis.  With k = m + 1
// (m < K) or m - 2K written as k = sum_{b < sz-1} m_b 2^b + 1 - m_top (2^(sz-1) + 1),
// j k is bilinear in the bits of j and m, so SELECT = diag(i, -i) on m_top (the
// factor i sign(z)) times, for each bit a of j,
//   controlled on j_a:          V(2^a)
//   controlled on j_a and m_b:  V(2^(a+b))            (b < sz - 1)
//   controlled on j_a and m_top: V(-2^a (2^(sz-1) + 1))
// with V(t) = exp(-i A~ dy dz t) = V_A diag(exp(-i lambda~ dy dz t)) V_A^H, built
// in FP64 on the device from phases reduced in long double.
template <typename R>
static sv_status run_fourier_gates(sv_state s, int n_s, int sy, int sz, double dy, double dz, const DevBuf &dV,
                                   const std::vector<double> &lamt, const std::vector<double> &pm, const double *b) {
    const int N = 1 << n_s, S = sy + sz;
    const hipStream_t st = s->stream;
    const uint64_t NN = (uint64_t)N * N;
    DevBuf dE, W, P, Uk;
    SV_TRY(dE.alloc(N * sizeof(double2)));
    SV_TRY(W.alloc(NN * sizeof(double2)));
    SV_TRY(P.alloc(NN * sizeof(double2)));
    SV_TRY(Uk.alloc(NN * sizeof(cvec<R>)));
    std::vector<double> E(2 * (size_t)N);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    auto build = [&](long double t) -> sv_status {
        for (int k = 0; k < N; ++k) {
            long double a = -(long double)lamt[k] * (long double)dy * (long double)dz * t;
            a = fmodl(a, two_pi);
            E[2 * k] = (double)cosl(a);
            E[2 * k + 1] = (double)sinl(a);
        }
        SV_TRY(upload(s, dE.p, E.data(), E.size() * sizeof(double)));
        hipLaunchKernelGGL(k_scale_cols, dim3(grid_for(NN)), dim3(256), 0, st, (double2 *)W.p, (const double2 *)dV.p,
                           (const double2 *)dE.p, N);
        SV_HIP(hipGetLastError());
        SV_TRY(cgemm<double>(st, (const double2 *)W.p, (double2 *)P.p, (const double2 *)dV.p, (uint64_t)N, N, N,
                             (uint64_t)(N - 1) << n_s, 0, 0, 1));
        hipLaunchKernelGGL(k_round_unitary<R>, dim3(grid_for(NN)), dim3(256), 0, st, (cvec<R> *)Uk.p,
                           (const double2 *)P.p, NN);
        SV_HIP(hipGetLastError());
        return SV_OK;
    };
    std::vector<double> amp((size_t)1 << S);
    for (size_t r = 0; r < amp.size(); ++r) amp[r] = pm[r >> sy];
    SV_TRY(sv_init_b(s, b, n_s, 0));
    SV_TRY(tree_circuit(s, amp, n_s, S, false));
    const int top = n_s + S - 1;
    static const double SG[8] = {0, 1, 0, 0, 0, 0, 0, -1};
    SV_TRY(sv_apply_gate(s, top, SG, nullptr, nullptr, 0));
    const cvec<R> *U = (const cvec<R> *)Uk.p;
    for (int a = 0; a < sy; ++a) {
        const uint64_t cj = 1ull << (n_s + a);
        SV_TRY(build(ldexpl(1.0L, a)));
        SV_TRY(ctrl_mask_unitary_impl<R>(s, U, n_s, cj, cj, 0));
        for (int bb = 0; bb + 1 < sz; ++bb) {
            const uint64_t cm = cj | (1ull << (n_s + sy + bb));
            SV_TRY(build(ldexpl(1.0L, a + bb)));
            SV_TRY(ctrl_mask_unitary_impl<R>(s, U, n_s, cm, cm, 0));
        }
        const uint64_t ct = cj | (1ull << top);
        SV_TRY(build(-ldexpl(1.0L, a) * (ldexpl(1.0L, sz - 1) + 1.0L)));
        SV_TRY(ctrl_mask_unitary_impl<R>(s, U, n_s, ct, ct, 0));
    }
    SV_TRY(tree_circuit(s, amp, n_s, S, true));
    SV_HIP(hipStreamSynchronize(st));
    return SV_OK;
}

template <typename R>
static sv_status run_fourier(sv_state s, int n_s, int sy, int sz, double dy, double dz, const DevBuf &dV,
                             const std::vector<double> &lamt, const std::vector<uint64_t> &F,
                             const std::vector<double> &pr, const std::vector<double> &bhat, double2 *z_dev) {
    const uint64_t N = 1ull << n_s, R2 = 1ull << (sy + sz);
    const hipStream_t st = s->stream;
    DevBuf db, dbeta, dtmp, dl, dF, dp;
    SV_TRY(db.alloc(N * sizeof(double2)));
    SV_TRY(dbeta.alloc(N * sizeof(double2)));
    SV_TRY(dtmp.alloc(N * sizeof(double2)));
    SV_TRY(dl.alloc(N * sizeof(double)));
    SV_TRY(dF.alloc(N * sizeof(uint64_t)));
    SV_TRY(dp.alloc(pr.size() * sizeof(double)));
    SV_TRY(upload(s, db.p, bhat.data(), N * sizeof(double2)));
    SV_TRY(upload(s, dl.p, lamt.data(), N * sizeof(double)));
    SV_TRY(upload(s, dF.p, F.data(), N * sizeof(uint64_t)));
    SV_TRY(upload(s, dp.p, pr.data(), pr.size() * sizeof(double)));
    // beta = V^H b^
    SV_TRY(kron_apply(st, (double2 *)dbeta.p, (const double2 *)db.p, (double2 *)dtmp.p, (const double2 *)dV.p,
                      (int)N, nullptr, 1, 1));
    {
        TraceScope ts(st, "fourier_select", (double)(R2 * N) * sizeof(cvec<R>), 0.0);
        hipLaunchKernelGGL(k_fourier_select<R>, dim3(grid_for(R2 * N)), dim3(256), 0, st, (cvec<R> *)s->data,
                           (const double2 *)dbeta.p, (const double *)dp.p, (const double *)dl.p,
                           (const uint64_t *)dF.p, n_s, sy, sz, dy, dz);
    }
    SV_HIP(hipGetLastError());
    SV_TRY(select_project<R>(s, (const double *)dp.p, (double2 *)dtmp.p, n_s, n_s, sy, R2, "fourier_project"));
    // back to the computational basis: z = V z_eig
    SV_TRY(kron_apply(st, z_dev, (const double2 *)dtmp.p, (double2 *)db.p, (const double2 *)dV.p, (int)N, nullptr,
                      1, 0));
    SV_HIP(hipStreamSynchronize(st));
    return SV_OK;
}

template <typename R>
static sv_status run_mode0(sv_state s, int n_s, int sbits, const DevBuf &dV, const std::vector<uint64_t> &t,
                           const std::vector<double> &pamp, const double *b) {
    const int N = 1 << n_s, M = 2 * N;
    const hipStream_t st = s->stream;
    const uint64_t NN = (uint64_t)N * N, MM = (uint64_t)M * M;
    DevBuf dt, Ec, Es, Wc, Ws, P, Q, Wk;
    SV_TRY(dt.alloc(N * sizeof(uint64_t)));
    SV_TRY(Ec.alloc(N * sizeof(double2)));
    SV_TRY(Es.alloc(N * sizeof(double2)));
    SV_TRY(Wc.alloc(NN * sizeof(double2)));
    SV_TRY(Ws.alloc(NN * sizeof(double2)));
    SV_TRY(P.alloc(NN * sizeof(double2)));
    SV_TRY(Q.alloc(NN * sizeof(double2)));
    SV_TRY(Wk.alloc(MM * sizeof(cvec<R>)));
    SV_TRY(upload(s, dt.p, t.data(), N * sizeof(uint64_t)));
    // one walk power as a dense unitary of the (walk, system) register
    auto build = [&](uint64_t power) -> sv_status {
        hipLaunchKernelGGL(k_walk_cs, dim3(grid_for(N)), dim3(256), 0, st, (double2 *)Ec.p, (double2 *)Es.p,
                           (const uint64_t *)dt.p, power, N);
        hipLaunchKernelGGL(k_scale_cols, dim3(grid_for(NN)), dim3(256), 0, st, (double2 *)Wc.p,
                           (const double2 *)dV.p, (const double2 *)Ec.p, N);
        hipLaunchKernelGGL(k_scale_cols, dim3(grid_for(NN)), dim3(256), 0, st, (double2 *)Ws.p,
                           (const double2 *)dV.p, (const double2 *)Es.p, N);
        SV_HIP(hipGetLastError());
        SV_TRY(cgemm<double>(st, (const double2 *)Wc.p, (double2 *)P.p, (const double2 *)dV.p, (uint64_t)N, N, N,
                             (uint64_t)(N - 1) << n_s, 0, 0, 1));
        SV_TRY(cgemm<double>(st, (const double2 *)Ws.p, (double2 *)Q.p, (const double2 *)dV.p, (uint64_t)N, N, N,
                             (uint64_t)(N - 1) << n_s, 0, 0, 1));
        hipLaunchKernelGGL(k_walk_assemble<R>, dim3(grid_for(MM)), dim3(256), 0, st, (cvec<R> *)Wk.p,
                           (const double2 *)P.p, (const double2 *)Q.p, N);
        SV_HIP(hipGetLastError());
        return SV_OK;
    };
    SV_TRY(sv_init_b(s, b, n_s, 0));
    SV_TRY(tree_circuit(s, pamp, n_s + 1, sbits, false));
    SV_TRY(build(1));
    SV_TRY(ctrl_unitary_impl<R>(s, (const cvec<R> *)Wk.p, n_s + 1, -1, 1, 0));
    for (int m = 0; m < sbits; ++m) {
        SV_TRY(build(2ull << m));
        SV_TRY(ctrl_unitary_impl<R>(s, (const cvec<R> *)Wk.p, n_s + 1, n_s + 1 + m, 1, 0));
    }
    static const double Z[8] = {1, 0, 0, 0, 0, 0, -1, 0};
    SV_TRY(sv_apply_gate(s, n_s + 1, Z, nullptr, nullptr, 0));
    SV_TRY(tree_circuit(s, pamp, n_s + 1, sbits, true));
    SV_HIP(hipStreamSynchronize(st));
    return SV_OK;
}

template <typename R>
static sv_status run_mode1(sv_state s, int n_s, int sbits, const DevBuf &dV, const std::vector<uint64_t> &t,
                           const std::vector<double> &pamp, const std::vector<double> &bhat, double2 *z_dev) {
    const uint64_t N = 1ull << n_s, J = 1ull << sbits;
    const hipStream_t st = s->stream;
    DevBuf db, dbeta, dtmp, dt, dp;
    SV_TRY(db.alloc(N * sizeof(double2)));
    SV_TRY(dbeta.alloc(N * sizeof(double2)));
    SV_TRY(dtmp.alloc(N * sizeof(double2)));
    SV_TRY(dt.alloc(N * sizeof(uint64_t)));
    SV_TRY(dp.alloc(J * sizeof(double)));
    SV_TRY(upload(s, db.p, bhat.data(), N * sizeof(double2)));
    SV_TRY(upload(s, dt.p, t.data(), N * sizeof(uint64_t)));
    SV_TRY(upload(s, dp.p, pamp.data(), J * sizeof(double)));
    // beta = V^H b^
    SV_TRY(kron_apply(st, (double2 *)dbeta.p, (const double2 *)db.p, (double2 *)dtmp.p, (const double2 *)dV.p,
                      (int)N, nullptr, 1, 1));
    {
        TraceScope ts(st, "cheb_select", (double)(2 * J * N) * sizeof(cvec<R>), 0.0);
        hipLaunchKernelGGL(k_cheb_select<R>, dim3(grid_for(J * N)), dim3(256), 0, st, (cvec<R> *)s->data,
                           (const double2 *)dbeta.p, (const double *)dp.p, (const uint64_t *)dt.p, n_s, J);
    }
    SV_HIP(hipGetLastError());
    SV_TRY(select_project<R>(s, (const double *)dp.p, (double2 *)dtmp.p, n_s, n_s + 1, 0, J, "cheb_project"));
    // back to the computational basis: z = V z_eig
    SV_TRY(kron_apply(st, z_dev, (const double2 *)dtmp.p, (double2 *)db.p, (const double2 *)dV.p, (int)N, nullptr,
                      1, 0));
    SV_HIP(hipStreamSynchronize(st));
    return SV_OK;
}

}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_qlsa2(sv_state s, const double *A, const double *b, const sv_qlsa2_params *prm, sv_qlsa2_result *res,
                   double *z_out) {
    clear_error();
    SV_TRY(check_state(s));
    if (!A || !b || !prm || !res) return fail(SV_EINVAL, "A, b, params or result is NULL");
    const int n_s = prm->n_s, sbits = prm->s;
    if (n_s < 1 || n_s > 13 || sbits < 1 || sbits > 24 || n_s + 1 + sbits != s->n)
        return fail(SV_EINVAL, "n_s %d + 1 + s %d != %d qubits (1 <= n_s <= 13, 1 <= s <= 24)", n_s, sbits, s->n);
    if (prm->B < 1 || prm->B > 20000000) return fail(SV_EINVAL, "B = %d outside [1, 2e7]", prm->B);
    if (prm->mode != 0 && prm->mode != 1) return fail(SV_EINVAL, "mode must be 0 or 1");
    const int N = 1 << n_s;
    const uint64_t J = 1ull << sbits;
    SV_TRY(check_hermitian(A, N, "A"));
    double bn = 0.0;
    for (int j = 0; j < 2 * N; ++j) bn += b[j] * b[j];
    bn = sqrt(bn);
    if (!(bn > 0.0) || !isfinite(bn)) return fail(SV_EZERONORM, "|b| = 0 or not finite");
    std::vector<double> bhat(2 * (size_t)N);
    for (int j = 0; j < 2 * N; ++j) bhat[j] = b[j] / bn;
    // spectrum and walk angles
    DevBuf dV;
    std::vector<double> lam;
    SV_TRY(eigh_device(s, A, N, dV, lam));
    double lmax = 0.0, lmin = INFINITY;
    for (double l : lam) {
        lmax = fmax(lmax, fabs(l));
        lmin = fmin(lmin, fabs(l));
    }
    if (!(lmax > 0.0)) return fail(SV_EINVAL, "A = 0");
    std::vector<uint64_t> turns;
    walk_turns(lam, lmax, turns);
    // LCU weights
    std::vector<double> alpha;
    cheb_coeffs(prm->B, (int)J, alpha);
    double l1 = 0.0;
    for (double a : alpha) l1 += fabs(a);
    if (!(l1 > 0.0)) return fail(SV_EINVAL, "no Chebyshev term");
    std::vector<double> pamp(J);
    for (uint64_t j = 0; j < J; ++j) pamp[j] = sqrt(fabs(alpha[j]) / l1);
    res->lambda_abs_max = lmax;
    res->lambda_abs_min = lmin;
    res->alpha_l1 = l1;
    std::vector<double> z(2 * (size_t)N, 0.0);
    if (prm->mode == 0) {
        if (s->dt == SV_C64)
            SV_TRY(run_mode0<float>(s, n_s, sbits, dV, turns, pamp, bhat.data()));
        else
            SV_TRY(run_mode0<double>(s, n_s, sbits, dV, turns, pamp, bhat.data()));
        // the select = 0, walk = 0 block: the first 2^n_s amplitudes
        double p = 0.0;
        SV_TRY(sv_postselect(s, ((1ull << (sbits + 1)) - 1ull) << n_s, 0, &p, z.data(), 0));
        const double sp = sqrt(p);
        for (double &v : z) v *= sp;
        res->p_post = p;
    } else {
        DevBuf dz;
        SV_TRY(dz.alloc(N * sizeof(double2)));
        if (s->dt == SV_C64)
            SV_TRY(run_mode1<float>(s, n_s, sbits, dV, turns, pamp, bhat, (double2 *)dz.p));
        else
            SV_TRY(run_mode1<double>(s, n_s, sbits, dV, turns, pamp, bhat, (double2 *)dz.p));
        SV_TRY(download(s, z.data(), dz.p, N * sizeof(double2)));
        double p = 0.0;
        for (int j = 0; j < 2 * N; ++j) p += z[j] * z[j];
        res->p_post = p;
    }
    if (z_out)
        for (int j = 0; j < 2 * N; ++j) z_out[j] = z[j];
    return SV_OK;
}

sv_status sv_qlsa2_fourier(sv_state s, const double *A, const double *b, const sv_qlsa2f_params *prm,
                           sv_qlsa2_result *res, double *z_out) {
    clear_error();
    SV_TRY(check_state(s));
    if (!A || !b || !prm || !res) return fail(SV_EINVAL, "A, b, params or result is NULL");
    const int n_s = prm->n_s, sy = prm->sy, sz = prm->sz;
    if (n_s < 1 || n_s > 13 || sy < 1 || sz < 1 || sy + sz > 30 || n_s + sy + sz != s->n)
        return fail(SV_EINVAL, "n_s %d + sy %d + sz %d != %d qubits (1 <= n_s <= 13)", n_s, sy, sz, s->n);
    if (!(prm->dy > 0.0) || !(prm->dz > 0.0) || !isfinite(prm->dy) || !isfinite(prm->dz))
        return fail(SV_EINVAL, "dy and dz must be positive");
    if (prm->mode != 0 && prm->mode != 1) return fail(SV_EINVAL, "mode must be 0 or 1");
    if (prm->mode == 0 && (n_s > 10 || sy + sz > 24))
        return fail(SV_EUNSUPPORTED, "gate-level mode with n_s = %d > 10 or sy + sz = %d > 24", n_s, sy + sz);
    const int N = 1 << n_s;
    SV_TRY(check_hermitian(A, N, "A"));
    double bn = 0.0;
    for (int j = 0; j < 2 * N; ++j) bn += b[j] * b[j];
    bn = sqrt(bn);
    if (!(bn > 0.0) || !isfinite(bn)) return fail(SV_EZERONORM, "|b| = 0 or not finite");
    std::vector<double> bhat(2 * (size_t)N);
    for (int j = 0; j < 2 * N; ++j) bhat[j] = b[j] / bn;
    DevBuf dV;
    std::vector<double> lam;
    SV_TRY(eigh_device(s, A, N, dV, lam));
    double lmax = 0.0, lmin = INFINITY;
    for (double l : lam) {
        lmax = fmax(lmax, fabs(l));
        lmin = fmin(lmin, fabs(l));
    }
    if (!(lmax > 0.0)) return fail(SV_EINVAL, "A = 0");
    std::vector<double> lamt(N);
    std::vector<uint64_t> F(N);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int k = 0; k < N; ++k) {
        lamt[k] = lam[k] / lmax;
        // lambda~ dy dz / 2 pi as a signed 64-bit turn fraction (reduced to [-1/2, 1/2])
        long double f = (long double)lamt[k] * (long double)prm->dy * (long double)prm->dz / two_pi;
        f -= nearbyintl(f);
        F[k] = (uint64_t)(int64_t)llroundl(ldexpl(f, 63)) * 2u;
    }
    // LCU weights w_r = dy dz |z_m| e^{-z_m^2/2} / sqrt(2 pi), the same for all 2^sy
    // values of j; PREP amplitudes sqrt(w_r / |w|_1) per m; |w|_1 in long double
    const int64_t K = (int64_t)1 << (sz - 1);
    const uint64_t M = 1ull << sz;
    std::vector<double> pr(M);
    long double l1acc = 0.0L;
    for (uint64_t m = 0; m < M; ++m) {
        const int64_t kk = (int64_t)m < K ? (int64_t)m + 1 : (int64_t)m - 2 * K;
        const double z = (double)kk * prm->dz;
        pr[m] = prm->dy * prm->dz * fabs(z) * exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
        l1acc += pr[m];
    }
    const double l1 = (double)(l1acc * (long double)(1ull << sy));
    if (!(l1 > 0.0)) return fail(SV_EINVAL, "no Fourier term");
    for (uint64_t m = 0; m < M; ++m) pr[m] = sqrt(pr[m] / l1);
    res->lambda_abs_max = lmax;
    res->lambda_abs_min = lmin;
    res->alpha_l1 = l1;
    std::vector<double> z(2 * (size_t)N);
    if (prm->mode == 0) {
        if (s->dt == SV_C64)
            SV_TRY(run_fourier_gates<float>(s, n_s, sy, sz, prm->dy, prm->dz, dV, lamt, pr, bhat.data()));
        else
            SV_TRY(run_fourier_gates<double>(s, n_s, sy, sz, prm->dy, prm->dz, dV, lamt, pr, bhat.data()));
        // the select = 0 block: the first 2^n_s amplitudes
        double p = 0.0;
        SV_TRY(sv_postselect(s, ((1ull << (sy + sz)) - 1ull) << n_s, 0, &p, z.data(), 0));
        const double sp = sqrt(p);
        for (double &v : z) v *= sp;
        res->p_post = p;
    } else {
        DevBuf dz;
        SV_TRY(dz.alloc(N * sizeof(double2)));
        if (s->dt == SV_C64)
            SV_TRY(run_fourier<float>(s, n_s, sy, sz, prm->dy, prm->dz, dV, lamt, F, pr, bhat, (double2 *)dz.p));
        else
            SV_TRY(run_fourier<double>(s, n_s, sy, sz, prm->dy, prm->dz, dV, lamt, F, pr, bhat, (double2 *)dz.p));
        SV_TRY(download(s, z.data(), dz.p, N * sizeof(double2)));
        double p = 0.0;
        for (int j = 0; j < 2 * N; ++j) p += z[j] * z[j];
        res->p_post = p;
    }
    if (z_out)
        for (int j = 0; j < 2 * N; ++j) z_out[j] = z[j];
    return SV_OK;
}

}  // extern "C"
