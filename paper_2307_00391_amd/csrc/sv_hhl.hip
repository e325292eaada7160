// HHL (QLSA-1) on the state vector.
//
// Register layout: bits [0, n_s) system x, [n_s, n_s + n_c) clock, bit
// n_s + n_c ancilla.  Both modes simulate the same circuit:
//   |0>_a H|0>_c |b^>  ->  controlled U_k = exp(i A T0 2^k)  ->  inverse QFT
//   ->  Ry(theta_y), sin(theta_y/2) = 1/y  ->  QFT  ->  controlled U_k^H
//   ->  H on the clock  ->  post-select a = 1, clock = 0.
// The QFT's final bit reversal is never materialised in the middle of the
// circuit: the clock qubit that controls U_k is relabelled n_c-1-k instead
// (a bit reversal commutes with the Hadamard layer and maps the control of
// U_k from bit k to bit n_c-1-k), so the cascades run without swaps.
//
// mode 0 (gate-faithful): every controlled U_k is a dense 2^n_s x 2^n_s
// matrix, built in FP64 as V diag(exp(2 pi i frac(phi_j 2^k))) V^H and
// applied to the state rows on the matrix cores; all steps act on the whole
// state; a final bit reversal restores the textbook clock order.
// mode 1 (eigen-frame): the system register is held in the eigenbasis of A
// (beta = V^H b, x = V z): the controlled U_k are diagonal, so the state
// after phase estimation is written directly; the inverse QFT runs on the
// ancilla = 0 half, the rotation writes the ancilla = 1 half, the QFT runs
// on that half, and the conjugate phases, Hadamards and clock = 0
// projection are one reduction over the clock register.
#include <math.h>
#include <string.h>

#include <stdlib.h>

#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

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
sv_status pipe_run(sv_state s, int n_s, int n_c, bool sgn, uint64_t gcut, const double2 *beta, const uint64_t *F,
                   double *part,
                   double2 *zpart, uint64_t *nparts);

// --------------------------------------------------------------------------
// small FP64 kernels
// --------------------------------------------------------------------------

__global__ void k_transpose_c128(double2 *__restrict__ out, const double2 *__restrict__ in, int N) {
    const uint64_t total = (uint64_t)N * N;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = i / N, c = i % N;
        out[c * N + r] = in[i];
    }
}

// W[r][j] = V[r][j] * E[j]
__global__ void k_scale_cols(double2 *__restrict__ W, const double2 *__restrict__ V, const double2 *__restrict__ E,
                             int N) {
    const uint64_t total = (uint64_t)N * N;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const double2 v = V[i], e = E[i % N];
        W[i] = make_double2(v.x * e.x - v.y * e.y, v.x * e.y + v.y * e.x);
    }
}

// real column-major eigenvectors -> complex row-major V
__global__ void k_real_cm_to_complex(double2 *__restrict__ V, const double *__restrict__ Acm, int N) {
    const uint64_t total = (uint64_t)N * N;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = i / N, j = i % N;
        V[i] = make_double2(Acm[j * N + r], 0.0);
    }
}

__global__ void k_real_to_complex(double2 *__restrict__ out, const double *__restrict__ in, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = make_double2(in[i], 0.0);
}

__global__ void k_c128_to_c64(float2 *__restrict__ out, const double2 *__restrict__ in, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

// One axis of a Kronecker basis change on a (n_hi x n_lo) array:
//   axis 0: out[a][q] = sum_c op(V)[c -> q] in[a][c]   (V is n_lo x n_lo)
//   axis 1: out[p][b] = sum_r op(V)[r -> p] in[r][b]   (V is n_hi x n_hi)
// op(V)[c -> q] = conj(V[c][q]) for the adjoint (V^H in), V[q][c] otherwise.
__global__ void k_axis_transform(double2 *__restrict__ out, const double2 *__restrict__ in,
                                 const double2 *__restrict__ V, int n_hi, int n_lo, int axis, int adjoint) {
    const uint64_t total = (uint64_t)n_hi * n_lo;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t a = i / n_lo, q = i % n_lo;
        const int L = axis ? n_hi : n_lo;
        const uint64_t o = axis ? a : q;        // output index along the axis
        double re = 0.0, im = 0.0;
        for (int c = 0; c < L; ++c) {
            const double2 x = axis ? in[(uint64_t)c * n_lo + q] : in[a * n_lo + c];
            double2 v;
            if (adjoint) {
                v = V[(uint64_t)c * L + o];
                v.y = -v.y;
            } else {
                v = V[o * L + c];
            }
            re += v.x * x.x - v.y * x.y;
            im += v.x * x.y + v.y * x.x;
        }
        out[i] = make_double2(re, im);
    }
}

// F[j][k] = frac(phi_j 2^k) as a 64-bit fraction of a turn, phi_j = lam_j T0 / 2 pi:
// the same IEEE operations as the host-side table (product, quotient, exact
// scaling by 2^k, exact floor), so both give the same bits
__global__ void k_turn_table(uint64_t *__restrict__ F, const double *__restrict__ lam, double T0, int n_c,
                             uint64_t N) {
    const uint64_t total = N * (uint64_t)n_c;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = i / n_c;
        const int k = (int)(i % n_c);
        const double phi = lam[j] * T0 / (2.0 * M_PI);
        const double x = ldexp(phi, k);
        const double f = x - floor(x);
        const double sc = ldexp(f, 64);
        F[i] = sc >= 18446744073709551616.0 ? 0ull : (uint64_t)sc;
    }
}

// ---- eigen-frame kernels ---------------------------------------------------
// Thread layout: 64 consecutive eigen-indices j per wave, 4 waves splitting a
// chunk of clock values; each thread walks its clock values in Gray-code
// order so the phase sum changes by one table entry per step.  The phase of
// clock index s (relabelled, see above) for eigen-index j is
// sum_k bit(s, n_c-1-k) F[j][k] (exact 64-bit turn fractions).
constexpr int EIG_MAXC = 24;

template <typename R>
__global__ __launch_bounds__(256) void k_eig_init(cvec<R> *__restrict__ psi, const double2 *__restrict__ beta,
                                                  const uint64_t *__restrict__ F, uint64_t N, int n_s, int n_c,
                                                  int log_len, double scale) {
    __shared__ uint64_t Fs[EIG_MAXC][64];
    const int lane = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const uint64_t j = (uint64_t)blockIdx.x * 64 + lane;
    const bool ok = j < N;
    if (rg == 0)
        for (int k = 0; k < n_c; ++k) Fs[k][lane] = ok ? F[j * n_c + k] : 0ull;
    __syncthreads();
    if (!ok) return;
    const uint64_t len = 1ull << log_len;
    const uint64_t s0 = ((uint64_t)blockIdx.y * 4 + rg) << log_len;
    uint64_t th = 0;
    for (int b = log_len; b < n_c; ++b)
        if (s0 >> b & 1) th += Fs[n_c - 1 - b][lane];
    const double2 bj = beta[j];
    const cvec<R> bv = cmake<R>((R)(bj.x * scale), (R)(bj.y * scale));
    uint64_t g = 0;
    for (uint64_t step = 0; step < len; ++step) {
        if (step) {
            const int b = __builtin_ctzll(step);
            g ^= 1ull << b;
            const uint64_t f = Fs[n_c - 1 - b][lane];
            th += (g >> b & 1) ? f : (0ull - f);
        }
        psi[((s0 | g) << n_s) | j] = cmul<R>(bv, turn_phase<R>(th));
    }
}

// ancilla = 1 half <- s_y * (ancilla = 0 half); FP64 partial sums of
// |s_y a|^2 (P(a=1)) and |a|^2 (c_y^2 + s_y^2) (total norm)
template <typename R>
__global__ __launch_bounds__(256) void k_eig_ry(cvec<R> *__restrict__ psi, const double2 *__restrict__ cs,
                                                uint64_t half, int n_s, uint64_t ymask, uint64_t abit, uint64_t chunk,
                                                double *__restrict__ part) {
    __shared__ double ws[2][4];
    const uint64_t beg = (uint64_t)blockIdx.x * chunk;
    const uint64_t end = beg + chunk < half ? beg + chunk : half;
    double pa = 0.0, nt = 0.0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const double2 t = cs[(i >> n_s) & ymask];
        const cvec<R> a = psi[i];
        const R sr = (R)t.y;
        psi[i | abit] = cmake<R>(sr * a.x, sr * a.y);
        const double a2 = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
        pa += t.y * t.y * a2;
        nt += (t.x * t.x + t.y * t.y) * a2;
    }
    pa = wave_sum_f64(pa);
    nt = wave_sum_f64(nt);
    if ((threadIdx.x & 63) == 0) {
        ws[0][threadIdx.x >> 6] = pa;
        ws[1][threadIdx.x >> 6] = nt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = (ws[0][0] + ws[0][1]) + (ws[0][2] + ws[0][3]);
        part[2 * blockIdx.x + 1] = (ws[1][0] + ws[1][1]) + (ws[1][2] + ws[1][3]);
    }
}

// z partials: part[(by * 4 + rg) * N + j] = sum over this thread's clock
// values of psi[a=1, s, j] * exp(-2 pi i phase(s, j)), in FP64
template <typename R>
__global__ __launch_bounds__(256) void k_eig_project(const cvec<R> *__restrict__ psi, const uint64_t *__restrict__ F,
                                                     uint64_t N, int n_s, int n_c, int log_len, uint64_t abit,
                                                     double2 *__restrict__ part) {
    __shared__ uint64_t Fs[EIG_MAXC][64];
    const int lane = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const uint64_t j = (uint64_t)blockIdx.x * 64 + lane;
    const bool ok = j < N;
    if (rg == 0)
        for (int k = 0; k < n_c; ++k) Fs[k][lane] = ok ? F[j * n_c + k] : 0ull;
    __syncthreads();
    if (!ok) return;
    const uint64_t len = 1ull << log_len;
    const uint64_t s0 = ((uint64_t)blockIdx.y * 4 + rg) << log_len;
    uint64_t th = 0;
    for (int b = log_len; b < n_c; ++b)
        if (s0 >> b & 1) th += Fs[n_c - 1 - b][lane];
    double zr = 0.0, zi = 0.0;
    uint64_t g = 0;
    for (uint64_t step = 0; step < len; ++step) {
        if (step) {
            const int b = __builtin_ctzll(step);
            g ^= 1ull << b;
            const uint64_t f = Fs[n_c - 1 - b][lane];
            th += (g >> b & 1) ? f : (0ull - f);
        }
        const cvec<R> a = psi[abit | ((s0 | g) << n_s) | j];
        const cvec<R> e = turn_phase<R>(0ull - th);
        const cvec<R> p = cmul<R>(a, e);
        zr += (double)p.x;
        zi += (double)p.y;
    }
    part[((uint64_t)blockIdx.y * 4 + rg) * N + j] = make_double2(zr, zi);
}

// z[j] = scale * sum over the partial rows of column j: four interleaved
// accumulators (rows r = k mod 4) keep four loads in flight per thread, and
// are combined in a fixed order
__global__ void k_sum_cols(double2 *__restrict__ z, const double2 *__restrict__ part, uint64_t N, int rows,
                           double scale) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (uint64_t)gridDim.x * blockDim.x) {
        double re[4] = {0.0, 0.0, 0.0, 0.0}, im[4] = {0.0, 0.0, 0.0, 0.0};
        int r = 0;
        for (; r + 4 <= rows; r += 4) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double2 p = part[(uint64_t)(r + k) * N + j];
                re[k] += p.x;
                im[k] += p.y;
            }
        }
        for (int k = 0; r < rows; ++r, ++k) {
            const double2 p = part[(uint64_t)r * N + j];
            re[k] += p.x;
            im[k] += p.y;
        }
        z[j] = make_double2(((re[0] + re[1]) + (re[2] + re[3])) * scale, ((im[0] + im[1]) + (im[2] + im[3])) * scale);
    }
}

// --------------------------------------------------------------------------
// host helpers
// --------------------------------------------------------------------------

// One rocBLAS handle (rocSOLVER's eigen-solvers) for the process.  A lease
// holds its lock from setting the stream until the lease ends, so that two
// host threads cannot move the handle to another stream in the middle of
// each other's library call.
static std::mutex g_blas_mu;
static rocblas_handle g_blas = nullptr;

struct BlasLease {
    std::unique_lock<std::mutex> lk;
    rocblas_handle h = nullptr;
};

static sv_status blas_lease(hipStream_t st, BlasLease &L) {
    L.lk = std::unique_lock<std::mutex>(g_blas_mu);
    if (!g_blas && rocblas_create_handle(&g_blas) != rocblas_status_success)
        return fail(SV_EDEVICE, "rocblas_create_handle failed");
    if (rocblas_set_stream(g_blas, st) != rocblas_status_success) return fail(SV_EDEVICE, "rocblas_set_stream failed");
    L.h = g_blas;
    return SV_OK;
}

static unsigned grid1(uint64_t items) {
    uint64_t g = (items + 255) / 256;
    if (g < 1) g = 1;
    if (g > (1u << 16)) g = 1u << 16;
    return (unsigned)g;
}

DevBuf::~DevBuf() {
    if (p) hipFree(p);
}
sv_status DevBuf::alloc(size_t nbytes) {
    if (p) hipFree(p);
    p = nullptr;
    bytes = 0;
    if (!nbytes) return SV_OK;
    SV_HIP(hipMalloc(&p, nbytes));
    bytes = nbytes;
    return SV_OK;
}

sv_status check_hermitian(const double *A, int N, const char *name) {
    double amax = 0.0, dmax = 0.0;
    for (int r = 0; r < N; ++r)
        for (int c = 0; c < N; ++c) {
            const double *x = A + 2 * ((size_t)r * N + c), *y = A + 2 * ((size_t)c * N + r);
            if (!isfinite(x[0]) || !isfinite(x[1])) return fail(SV_EINVAL, "%s has a non-finite entry", name);
            amax = fmax(amax, hypot(x[0], x[1]));
            dmax = fmax(dmax, hypot(x[0] - y[0], x[1] + y[1]));
        }
    if (dmax > 1e-12 * amax) return fail(SV_ENOTHERMITIAN, "%s is not Hermitian (|A - A^H| = %g)", name, dmax);
    return SV_OK;
}

// Residual check of an eigen-decomposition with one fixed pseudo-random
// vector x: V must preserve its norm and A (V x) must equal V (lam .* x).
// O(N^2) on the host; catches non-finite or non-orthonormal eigenvectors.
static bool eig_residual_ok(const double *A, int N, const std::vector<double> &lam, const std::vector<double> &V,
                            double *worst) {
    std::vector<double> x(2 * (size_t)N), y(2 * (size_t)N, 0.0), z(2 * (size_t)N, 0.0);
    uint64_t st = 0x9e3779b97f4a7c15ull;
    double xn = 0.0, amax = 0.0;
    for (size_t i = 0; i < 2 * (size_t)N; ++i) {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        x[i] = (double)(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        xn += x[i] * x[i];
    }
    for (int r = 0; r < N; ++r)
        for (int j = 0; j < N; ++j) {
            const double *v = &V[2 * ((size_t)r * N + j)];
            if (!isfinite(v[0]) || !isfinite(v[1])) return false;
            const double xr = x[2 * j], xi = x[2 * j + 1];
            y[2 * r] += v[0] * xr - v[1] * xi;            // y = V x
            y[2 * r + 1] += v[0] * xi + v[1] * xr;
            z[2 * r] += lam[j] * (v[0] * xr - v[1] * xi);  // z = V (lam .* x)
            z[2 * r + 1] += lam[j] * (v[0] * xi + v[1] * xr);
        }
    double yn = 0.0, rn = 0.0;
    for (int r = 0; r < N; ++r) {
        yn += y[2 * r] * y[2 * r] + y[2 * r + 1] * y[2 * r + 1];
        double ar = 0.0, ai = 0.0;
        for (int c = 0; c < N; ++c) {
            const double *a = &A[2 * ((size_t)r * N + c)];
            amax = fmax(amax, fabs(a[0]) + fabs(a[1]));
            ar += a[0] * y[2 * c] - a[1] * y[2 * c + 1];
            ai += a[0] * y[2 * c + 1] + a[1] * y[2 * c];
        }
        rn += (ar - z[2 * r]) * (ar - z[2 * r]) + (ai - z[2 * r + 1]) * (ai - z[2 * r + 1]);
    }
    const double lmax = fmax(fabs(lam.front()), fabs(lam.back()));
    const double e1 = fabs(sqrt(yn) - sqrt(xn)) / sqrt(xn), e2 = sqrt(rn) / (sqrt(xn) * fmax(lmax, amax));
    *worst = fmax(e1, e2);
    return isfinite(*worst) && e1 < 1e-10 && e2 < 1e-10 * sqrt((double)N);
}

// Hermitian eigen-decomposition in FP64 on the device (rocSOLVER), validated
// by eig_residual_ok.  Real symmetric input goes to the real solvers, and a
// real tridiagonal matrix first to the tridiagonal divide and conquer (no
// reduction to tridiagonal form, which dominates the dense solvers' time).
// The solvers are tried in order (divide and conquer, Jacobi, QR iteration)
// until one passes the check; SV_EIGH_ORDER (comma-separated names) can
// override the order.  dV receives V row-major (column j = eigenvector j);
// lam ascending.
enum EigSolver { ES_ZHEEVD, ES_ZHEEVJ, ES_ZHEEV, ES_DSYEVD, ES_DSYEVJ, ES_DSYEV, ES_DSTEDC };
constexpr int ES_COUNT = 7;
static const char *es_name(int e) {
    static const char *n[] = {"zheevd", "zheevj", "zheev", "dsyevd", "dsyevj", "dsyev", "dstedc"};
    return n[e];
}

// zero outside the diagonal and the first off-diagonals (real and imaginary parts)
bool is_tridiagonal(const double *A, int N) {
    for (int r = 0; r < N; ++r)
        for (int c = 0; c < N; ++c)
            if ((c > r + 1 || r > c + 1) && (A[2 * ((size_t)r * N + c)] != 0.0 || A[2 * ((size_t)r * N + c) + 1] != 0.0))
                return false;
    return true;
}

static thread_local std::string g_eigh_used;

sv_status eigh_device(sv_state s, const double *A, int N, DevBuf &dV, std::vector<double> &lam) {
    bool real = true;
    for (size_t i = 0; i < (size_t)N * N && real; ++i) real = A[2 * i + 1] == 0.0;
    const bool tri = real && N > 1 && is_tridiagonal(A, N);
    std::vector<int> order;
    if (const char *env = getenv("SV_EIGH_ORDER")) {
        std::string e(env);
        size_t pos = 0;
        while (pos <= e.size()) {
            size_t q = e.find(',', pos);
            if (q == std::string::npos) q = e.size();
            std::string name = e.substr(pos, q - pos);
            for (int k = 0; k < ES_COUNT; ++k)
                if (name == es_name(k) && (k == ES_DSTEDC ? tri : (real || k < 3))) order.push_back(k);
            pos = q + 1;
        }
    }
    if (order.empty()) {
        if (tri) order = {ES_DSTEDC, ES_DSYEVD, ES_DSYEVJ, ES_ZHEEVJ, ES_DSYEV};
        else if (real) order = {ES_DSYEVD, ES_DSYEVJ, ES_ZHEEVJ, ES_DSYEV};
        else order = {ES_ZHEEVD, ES_ZHEEVJ, ES_ZHEEV};
    }
    // the tridiagonal solver's input: the diagonal and the off-diagonal
    std::vector<double> td, te;
    if (tri) {
        td.resize(N);
        te.assign(N, 0.0);
        for (int i = 0; i < N; ++i) td[i] = A[2 * ((size_t)i * N + i)];
        for (int i = 0; i + 1 < N; ++i) te[i] = A[2 * ((size_t)i * N + i + 1)];
    }
    // rocSOLVER is column-major: the row-major conj(A) is A in column-major order
    std::vector<double> Ac(2 * (size_t)N * N), Ar;
    for (size_t i = 0; i < (size_t)N * N; ++i) {
        Ac[2 * i] = A[2 * i];
        Ac[2 * i + 1] = -A[2 * i + 1];
    }
    if (real) {
        Ar.resize((size_t)N * N);
        for (size_t i = 0; i < (size_t)N * N; ++i) Ar[i] = A[2 * i];   // symmetric: row-major == column-major
    }
    DevBuf dA, dD, dE, dInfo, dRes, dSweeps;
    SV_TRY(dA.alloc((size_t)N * N * sizeof(double2)));
    SV_TRY(dD.alloc(N * sizeof(double)));
    SV_TRY(dE.alloc(N * sizeof(double)));
    SV_TRY(dInfo.alloc(sizeof(int)));
    SV_TRY(dRes.alloc(sizeof(double)));
    SV_TRY(dSweeps.alloc(sizeof(int)));
    SV_TRY(dV.alloc((size_t)N * N * sizeof(double2)));
    BlasLease lease;
    SV_TRY(blas_lease(s->stream, lease));
    const rocblas_handle h = lease.h;
    std::vector<double> Vh(2 * (size_t)N * N);
    double worst = 0.0;
    std::string tried;
    for (int e : order) {
        const bool rs_real = e >= ES_DSYEVD;
        if (e == ES_DSTEDC) {
            SV_TRY(upload(s, dD.p, td.data(), N * sizeof(double)));
            SV_TRY(upload(s, dE.p, te.data(), N * sizeof(double)));
        } else if (rs_real) {
            SV_TRY(upload(s, dA.p, Ar.data(), Ar.size() * sizeof(double)));
        } else {
            SV_TRY(upload(s, dA.p, Ac.data(), Ac.size() * sizeof(double)));
        }
        rocblas_double_complex *zA = (rocblas_double_complex *)dA.p;
        double *rA = (double *)dA.p, *D = (double *)dD.p, *E = (double *)dE.p;
        rocblas_int *info_p = (rocblas_int *)dInfo.p;
        rocblas_status rs = rocblas_status_not_implemented;
        switch (e) {
        case ES_ZHEEVD: rs = rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, N, zA, N, D, E, info_p); break;
        case ES_ZHEEV: rs = rocsolver_zheev(h, rocblas_evect_original, rocblas_fill_upper, N, zA, N, D, E, info_p); break;
        case ES_ZHEEVJ:
            rs = rocsolver_zheevj(h, rocblas_esort_ascending, rocblas_evect_original, rocblas_fill_upper, N, zA, N, 0.0,
                                  (double *)dRes.p, 100, (rocblas_int *)dSweeps.p, D, info_p);
            break;
        case ES_DSYEVD: rs = rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, N, rA, N, D, E, info_p); break;
        case ES_DSYEV: rs = rocsolver_dsyev(h, rocblas_evect_original, rocblas_fill_upper, N, rA, N, D, E, info_p); break;
        case ES_DSYEVJ:
            rs = rocsolver_dsyevj(h, rocblas_esort_ascending, rocblas_evect_original, rocblas_fill_upper, N, rA, N, 0.0,
                                  (double *)dRes.p, 100, (rocblas_int *)dSweeps.p, D, info_p);
            break;
        case ES_DSTEDC:   // eigenvectors of the tridiagonal matrix itself, column-major into dA
            rs = rocsolver_dstedc(h, rocblas_evect_tridiagonal, N, D, E, rA, N, info_p);
            break;
        }
        tried += std::string(tried.empty() ? "" : ",") + es_name(e);
        if (rs != rocblas_status_success) continue;
        int info = 0;
        lam.resize(N);
        SV_TRY(download(s, lam.data(), dD.p, N * sizeof(double)));
        SV_TRY(download(s, &info, dInfo.p, sizeof(int)));
        if (info != 0) continue;
        if (rs_real)
            hipLaunchKernelGGL(k_real_cm_to_complex, dim3(grid1((uint64_t)N * N)), dim3(256), 0, s->stream,
                               (double2 *)dV.p, (const double *)dA.p, N);
        else   // column-major eigenvectors read row-major are V^T; transpose to V
            hipLaunchKernelGGL(k_transpose_c128, dim3(grid1((uint64_t)N * N)), dim3(256), 0, s->stream,
                               (double2 *)dV.p, (const double2 *)dA.p, N);
        SV_HIP(hipGetLastError());
        SV_TRY(download(s, Vh.data(), dV.p, Vh.size() * sizeof(double)));
        if (eig_residual_ok(A, N, lam, Vh, &worst)) {
            g_eigh_used = es_name(e);
            return SV_OK;
        }
    }
    return fail(SV_EDEVICE, "no eigen-solver passed the residual check for N = %d (tried %s; last residual %g)", N,
                tried.c_str(), worst);
}

const char *eigh_last_solver() { return g_eigh_used.c_str(); }

// Several real symmetric N x N matrices at once: one strided-batched
// divide-and-conquer call, each result validated by eig_residual_ok; a
// matrix whose result fails the check goes through eigh_device alone.
sv_status eigh_device_batched(sv_state s, const std::vector<const double *> &As, int N, std::vector<DevBuf *> &dVs,
                              std::vector<std::vector<double>> &lams) {
    const int cnt = (int)As.size();
    lams.assign(cnt, {});
    if (!cnt) return SV_OK;
    const size_t NN = (size_t)N * N;
    std::vector<double> Ar(NN * cnt);
    for (int i = 0; i < cnt; ++i)
        for (size_t k = 0; k < NN; ++k) Ar[i * NN + k] = As[i][2 * k];   // symmetric: row- = column-major
    DevBuf dA, dD, dE, dInfo;
    SV_TRY(dA.alloc(NN * cnt * sizeof(double)));
    SV_TRY(dD.alloc((size_t)N * cnt * sizeof(double)));
    SV_TRY(dE.alloc((size_t)N * cnt * sizeof(double)));
    SV_TRY(dInfo.alloc(cnt * sizeof(int)));
    SV_TRY(upload(s, dA.p, Ar.data(), Ar.size() * sizeof(double)));
    BlasLease lease;
    SV_TRY(blas_lease(s->stream, lease));
    const rocblas_handle h = lease.h;
    const rocblas_status rs = rocsolver_dsyevd_strided_batched(
        h, rocblas_evect_original, rocblas_fill_upper, N, (double *)dA.p, N, (rocblas_stride)NN, (double *)dD.p,
        (rocblas_stride)N, (double *)dE.p, (rocblas_stride)N, (rocblas_int *)dInfo.p, cnt);
    std::vector<double> D((size_t)N * cnt);
    std::vector<int> info(cnt, 1);
    if (rs == rocblas_status_success) {
        SV_TRY(download(s, D.data(), dD.p, D.size() * sizeof(double)));
        SV_TRY(download(s, info.data(), dInfo.p, cnt * sizeof(int)));
    }
    std::vector<double> Vh(2 * NN);
    lease.lk.unlock();          // eigh_device below takes the handle itself
    for (int i = 0; i < cnt; ++i) {
        bool ok = rs == rocblas_status_success && info[i] == 0;
        if (ok) {
            lams[i].assign(D.begin() + (size_t)i * N, D.begin() + (size_t)(i + 1) * N);
            SV_TRY(dVs[i]->alloc(NN * sizeof(double2)));
            hipLaunchKernelGGL(k_real_cm_to_complex, dim3(grid1(NN)), dim3(256), 0, s->stream, (double2 *)dVs[i]->p,
                               (const double *)dA.p + (size_t)i * NN, N);
            SV_HIP(hipGetLastError());
            SV_TRY(download(s, Vh.data(), dVs[i]->p, Vh.size() * sizeof(double)));
            double worst = 0.0;
            ok = eig_residual_ok(As[i], N, lams[i], Vh, &worst);
        }
        if (ok) {
            g_eigh_used = "dsyevd_strided_batched";
        } else {
            SV_TRY(eigh_device(s, As[i], N, *dVs[i], lams[i]));
        }
    }
    return SV_OK;
}

// turn fractions frac(phi_j 2^k), phi_j = lam_j T0 / 2 pi, as 64-bit fixed point
void turn_table(const std::vector<double> &lam, double T0, int n_c, std::vector<uint64_t> &F) {
    const size_t N = lam.size();
    F.assign(N * n_c, 0);
    for (size_t j = 0; j < N; ++j) {
        const double phi = lam[j] * T0 / (2.0 * M_PI);
        for (int k = 0; k < n_c; ++k) {
            const double x = ldexp(phi, k);
            const double f = x - floor(x);   // exact
            const double sc = ldexp(f, 64);
            F[j * n_c + k] = sc >= 18446744073709551616.0 ? 0ull : (uint64_t)sc;
        }
    }
}

// (cos, sin) of the inversion rotation for every clock value: sin = 1/y,
// y >= 1; a signed clock reads y >= 2^(n_c-1) as y - 2^n_c (two's complement).
// gcut >= 1 gives the gapped-phase-estimation flag instead: sin = 1 (Ry(pi))
// where |y| >= gcut, sin = 0 elsewhere.
void inversion_table(int n_c, std::vector<double> &cs, bool sgn, uint64_t gcut) {
    const size_t M = (size_t)1 << n_c;
    cs.assign(2 * M, 0.0);
    cs[0] = 1.0;
    for (size_t y = 1; y < M; ++y) {
        const double ys = (sgn && y >= M / 2) ? (double)y - (double)M : (double)y;
        const double sv = gcut ? (fabs(ys) >= (double)gcut ? 1.0 : 0.0) : 1.0 / ys;
        cs[2 * y] = sqrt(1.0 - sv * sv);
        cs[2 * y + 1] = sv;
    }
}

// basis change out = (V_hi (x) V_lo)^(H) in on FP64 device vectors (V_lo may be null: dense V_hi)
sv_status kron_apply(hipStream_t st, double2 *out, const double2 *in, double2 *tmp, const double2 *V_hi, int n_hi,
                     const double2 *V_lo, int n_lo, int adjoint) {
    const uint64_t total = (uint64_t)n_hi * n_lo;
    if (V_lo && n_lo > 1) {
        hipLaunchKernelGGL(k_axis_transform, dim3(grid1(total)), dim3(256), 0, st, tmp, in, V_lo, n_hi, n_lo, 0,
                           adjoint);
        in = tmp;
    }
    hipLaunchKernelGGL(k_axis_transform, dim3(grid1(total)), dim3(256), 0, st, out, in, V_hi, n_hi, n_lo, 1, adjoint);
    SV_HIP(hipGetLastError());
    return SV_OK;
}

// out[q][c] = conj(in[c][q]) for an n x n row-major matrix
__global__ void k_conj_transpose(double2 *__restrict__ out, const double2 *__restrict__ in, int n) {
    const uint64_t total = (uint64_t)n * n;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t q = i / n, c = i % n;
        const double2 v = in[c * n + q];
        out[i] = make_double2(v.x, -v.y);
    }
}


// Dense basis change, FP64, reading V once from HBM.
// Dense basis change, FP64, reading V once from HBM.
__device__ __forceinline__ double2 vmul_acc(double v, double2 z, double2 a) {
    return make_double2(fma(v, z.x, a.x), fma(v, z.y, a.y));
}
__device__ __forceinline__ double2 vmul_acc(double2 v, double2 z, double2 a) {
    return make_double2(fma(v.x, z.x, fma(-v.y, z.y, a.x)), fma(v.x, z.y, fma(v.y, z.x, a.y)));
}
// conj(v) * z + a
__device__ __forceinline__ double2 vcmul_acc(double v, double2 z, double2 a) { return vmul_acc(v, z, a); }
__device__ __forceinline__ double2 vcmul_acc(double2 v, double2 z, double2 a) {
    return make_double2(fma(v.x, z.x, fma(v.y, z.y, a.x)), fma(v.x, z.y, fma(-v.y, z.x, a.y)));
}

// k_gemv_rows: the partial sums part[i][s] = sum_{j in segment s} V[i][j] z[j]
// over segments of 1024 columns.  A block of four wavefronts takes 16 rows
// (four per wavefront) of one segment, with z's segment in LDS; each lane
// reads 16 entries of each of its wavefront's rows, 1 KiB of a row per
// wavefront load (two real entries, or one complex entry, per lane).  Blocks are numbered segment-fastest,
// so the blocks in flight read whole rows of a few row groups, as a linear
// sweep of V would (per-row streams spread over all of V read at half speed).
constexpr int GV_SEG = 1024, GV_ROWS = 16;

template <typename VT>
__global__ __launch_bounds__(256) void k_gemv_rows(double2 *__restrict__ part, const VT *__restrict__ V,
                                                   const double2 *__restrict__ z, uint64_t N, int nseg) {
    __shared__ double2 zs[GV_SEG];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t rg = (uint64_t)blockIdx.x / nseg;
    const int seg = (int)((uint64_t)blockIdx.x % nseg);
    const uint64_t j0 = (uint64_t)seg * GV_SEG;
    const int J = (int)(N - j0 < (uint64_t)GV_SEG ? N - j0 : (uint64_t)GV_SEG);
    for (int t = threadIdx.x; t < J; t += 256) zs[t] = z[j0 + t];
    __syncthreads();
    const uint64_t r0 = rg * GV_ROWS + (uint64_t)w * 4;
    double2 acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = make_double2(0.0, 0.0);
    const int nr = r0 >= N ? 0 : (N - r0 < 4 ? (int)(N - r0) : 4);
    if (sizeof(VT) == sizeof(double) && (N & 1) == 0) {
        // a real V with an even row length: two entries (16 B) per lane and
        // load, 1 KiB of a row per wavefront instruction; J is even too
#pragma unroll 2
        for (int t = 2 * lane; t < J; t += 128) {
            const double2 z0 = zs[t], z1 = zs[t + 1];
            const double2 *col = reinterpret_cast<const double2 *>(V + r0 * N + j0 + t);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r < nr) {
                    const double2 v = col[(uint64_t)r * (N / 2)];
                    acc[r] = vmul_acc(v.y, z1, vmul_acc(v.x, z0, acc[r]));
                }
        }
    } else {
#pragma unroll 4
        for (int t = lane; t < J; t += 64) {
            const double2 zt = zs[t];
            const VT *col = V + r0 * N + j0 + t;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r < nr) acc[r] = vmul_acc(col[(uint64_t)r * N], zt, acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double re = wave_sum_f64(acc[r].x), im = wave_sum_f64(acc[r].y);
        if (lane == 0 && r < nr) part[(r0 + r) * nseg + seg] = make_double2(re, im);
    }
}

// out[i] = sum over s of part[i][s], in segment order
__global__ void k_gemv_reduce(double2 *__restrict__ out, const double2 *__restrict__ part, uint64_t N, int nseg) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int sg = 0; sg < nseg; ++sg) {
            const double2 v = part[i * nseg + sg];
            re += v.x;
            im += v.y;
        }
        out[i] = make_double2(re, im);
    }
}

// k_gemv_cols: out[j] = sum_i conj(V[i][j]) b[i].  A block of four wavefronts
// takes 64 columns, one per lane; wavefront w sums the rows i = w mod 4 (each
// load a 512 B or 1 KiB row segment), and the four partial sums are added in
// a fixed order.
template <typename VT>
__global__ __launch_bounds__(256) void k_gemv_cols(double2 *__restrict__ out, const VT *__restrict__ V,
                                                   const double2 *__restrict__ b, uint64_t N);

// the same for a real V with an even row length, two columns per lane (one
// 16 B load per row, 1 KiB of a row per wavefront instruction, 128 columns
// per block); every column's sum runs in the same order as above
__global__ __launch_bounds__(256) void k_gemv_cols2(double2 *__restrict__ out, const double *__restrict__ V,
                                                    const double2 *__restrict__ b, uint64_t N) {
    __shared__ double2 part[3][2][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t j = (uint64_t)blockIdx.x * 128 + 2 * (uint64_t)lane;
    const bool ok = j < N;
    double2 a0 = make_double2(0.0, 0.0), a1 = make_double2(0.0, 0.0);
    if (ok) {
        const double2 *V2 = reinterpret_cast<const double2 *>(V);
#pragma unroll 8
        for (uint64_t i = w; i < N; i += 4) {
            const double2 v = V2[(i * N + j) >> 1];
            const double2 bi = b[i];
            a0 = vcmul_acc(v.x, bi, a0);
            a1 = vcmul_acc(v.y, bi, a1);
        }
    }
    if (w > 0) {
        part[w - 1][0][lane] = a0;
        part[w - 1][1][lane] = a1;
    }
    __syncthreads();
    if (w == 0 && ok) {
        const double2 p1 = part[0][0][lane], p2 = part[1][0][lane], p3 = part[2][0][lane];
        const double2 q1 = part[0][1][lane], q2 = part[1][1][lane], q3 = part[2][1][lane];
        out[j] = make_double2((a0.x + p1.x) + (p2.x + p3.x), (a0.y + p1.y) + (p2.y + p3.y));
        out[j + 1] = make_double2((a1.x + q1.x) + (q2.x + q3.x), (a1.y + q1.y) + (q2.y + q3.y));
    }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_gemv_cols(double2 *__restrict__ out, const VT *__restrict__ V,
                                                   const double2 *__restrict__ b, uint64_t N) {
    __shared__ double2 part[3][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t j = (uint64_t)blockIdx.x * 64 + lane;
    const bool ok = j < N;
    double2 acc = make_double2(0.0, 0.0);
    if (ok) {
#pragma unroll 8
        for (uint64_t i = w; i < N; i += 4) acc = vcmul_acc(V[i * N + j], b[i], acc);
    }
    if (w > 0) part[w - 1][lane] = acc;
    __syncthreads();
    if (w == 0 && ok) {
        const double2 p1 = part[0][lane], p2 = part[1][lane], p3 = part[2][lane];
        out[j] = make_double2((acc.x + p1.x) + (p2.x + p3.x), (acc.y + p1.y) + (p2.y + p3.y));
    }
}

// the dense basis change: out = V in (forward) or V^H in (adjoint), V N x N
// row-major FP64, real (Vr) or complex (Vc); part holds N * ceil(N / 1024)
// complex partial sums (forward only)
static sv_status gemv_apply(hipStream_t st, double2 *out, const double2 *in, const double *Vr, const double2 *Vc,
                            uint64_t N, int adjoint, double2 *part) {
    const double bytes = (double)N * (double)N * (Vr ? sizeof(double) : sizeof(double2));
    TraceScope _ts(st, adjoint ? "gemv_vh" : "gemv_v", bytes, 8.0 * (double)N * (double)N);
    if (adjoint) {
        const unsigned g = (unsigned)((N + 63) / 64);
        if (Vr && (N & 1) == 0)
            hipLaunchKernelGGL(k_gemv_cols2, dim3((unsigned)((N + 127) / 128)), dim3(256), 0, st, out, Vr, in, N);
        else if (Vr)
            hipLaunchKernelGGL(k_gemv_cols<double>, dim3(g), dim3(256), 0, st, out, Vr, in, N);
        else
            hipLaunchKernelGGL(k_gemv_cols<double2>, dim3(g), dim3(256), 0, st, out, Vc, in, N);
    } else {
        const int nseg = (int)((N + GV_SEG - 1) / GV_SEG);
        const uint64_t blocks = ((N + GV_ROWS - 1) / GV_ROWS) * (uint64_t)nseg;
        if (blocks > 0x7fffffffull) return fail(SV_EUNSUPPORTED, "GEMV of %llu rows", (unsigned long long)N);
        if (Vr) hipLaunchKernelGGL(k_gemv_rows<double>, dim3((unsigned)blocks), dim3(256), 0, st, part, Vr, in, N, nseg);
        else hipLaunchKernelGGL(k_gemv_rows<double2>, dim3((unsigned)blocks), dim3(256), 0, st, part, Vc, in, N, nseg);
        hipLaunchKernelGGL(k_gemv_reduce, dim3(grid1(N)), dim3(256), 0, st, out, (const double2 *)part, N, nseg);
    }
    SV_HIP(hipGetLastError());
    return SV_OK;
}

static size_t gemv_part_bytes(uint64_t N) { return (size_t)N * ((N + GV_SEG - 1) / GV_SEG) * sizeof(double2); }

static int ilog2(uint64_t v) { return 63 - __builtin_clzll(v); }

// The basis change of a plan: out = (V_hi (x) V_lo) in, or with the conjugate
// transposes (adjoint).  The vector is the row-major n_hi x n_lo matrix X.
// Kronecker plans: two complex FP64 GEMMs on the matrix cores (k_cgemm):
//   low axis:  each row x_r of X -> V_lo x_r (forward) or V_lo^H x_r
//              (k_cgemm with B(k, n) = V_lo[n][k], or conj(V_lo[k][n]));
//   high axis: V_hi Y or V_hi^H Y, the rows of V_hi (or of its stored
//              conjugate transpose) times Y.
// Dense plans: one GEMV over V (real, a caller's eigenbasis, or complex).
static sv_status kron_apply_frame(sv_state s, double2 *out, const double2 *in, double2 *tmp, const EigFrame &E,
                                  int adjoint, DevBuf &gpart) {
    const hipStream_t st = s->stream;
    const uint64_t nh = (uint64_t)E.n_hi, nl = (uint64_t)E.n_lo;
    if (E.Vr || nl <= 1) {
        const uint64_t N = nh * nl;
        if (!adjoint) SV_TRY(gpart.ensure(gemv_part_bytes(N)));
        return gemv_apply(st, out, in, E.Vr, E.Vr ? nullptr : (const double2 *)E.V_hi.p, N, adjoint,
                          (double2 *)gpart.p);
    }
    SV_TRY(cgemm<double>(st, in, tmp, (const double2 *)E.V_lo.p, nh, (int)nl, (int)nl, (nh - 1) << ilog2(nl), 0,
                         adjoint, adjoint));
    const double2 *W = (const double2 *)(adjoint ? E.VH_hi.p : E.V_hi.p);
    return cgemm<double>(st, W, out, tmp, nh, (int)nl, (int)nh, (nh - 1) << ilog2(nh), 0, 1, 0);
}

static int pick_log_len(uint64_t N, int n_c) {
    // enough workgroups to fill the chip: ~8 per CU over the column blocks
    const uint64_t colblocks = (N + 63) / 64;
    int L = 0;
    while (L < n_c - 2 && (((1ull << n_c) >> (L + 2)) * colblocks) > 8192) ++L;
    if (L > n_c - 2) L = n_c - 2 > 0 ? n_c - 2 : 0;
    if (n_c < 2) L = 0;
    return L;
}

// device workspaces of a plan, grown on demand and reused by every solve
struct Workspace {
    DevBuf F, cs, beta, tmp, tmp2, z, x, part, zpart, sum, E, W, U64, Uk, gpart;
};

static sv_status need(DevBuf &b, size_t bytes) { return b.ensure(bytes); }
static sv_status eig_finish(sv_state s, const EigFrame &E, Workspace &w, uint64_t N, sv_hhl_result *res,
                            double *x_out, bool dev, double2 *x_dev);

// |v|^2 of an FP64 complex device vector, first level: block b sums the
// contiguous chunk [b*chunk, (b+1)*chunk) into tmp[b]
__global__ __launch_bounds__(256) void k_vec_norm2(const double2 *__restrict__ v, uint64_t n, uint64_t chunk,
                                                   double *__restrict__ tmp) {
    __shared__ double red[4];
    const uint64_t beg = (uint64_t)blockIdx.x * chunk;
    const uint64_t end = beg + chunk < n ? beg + chunk : n;
    double a = 0.0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += 256) a += v[i].x * v[i].x + v[i].y * v[i].y;
    a = wave_sum_f64(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) tmp[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[0] = |v|^2 in a fixed order: 64 chunk sums (tmp holds >= 64 doubles),
// then their sum in one workgroup
static void vec_norm2(hipStream_t st, const double2 *v, uint64_t n, double *tmp, double *out) {
    const unsigned nb = 64;
    const uint64_t chunk = (n + nb - 1) / nb;
    hipLaunchKernelGGL(k_vec_norm2, dim3(nb), dim3(256), 0, st, v, n, chunk, tmp);
    hipLaunchKernelGGL(k_sum_partials_strided, dim3(1), dim3(256), 0, st, (const double *)tmp, (int)nb, 1, out);
}

// out = in / sqrt(nrm[0]) (nrm on the device)
__global__ void k_vec_normalise(double2 *__restrict__ out, const double2 *__restrict__ in, uint64_t n,
                                const double *__restrict__ nrm) {
    const double sc = 1.0 / sqrt(nrm[0]);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = make_double2(in[i].x * sc, in[i].y * sc);
}

template <typename R>
static sv_status eig_frame_run(sv_state s, const EigFrame &E, Workspace &w, const std::vector<double> &bhat, int n_c, bool sgn,
                               uint64_t gcut, double T0, bool fused, sv_hhl_result *res, double *x_out,
                               const double2 *b_dev = nullptr, double2 *x_dev = nullptr) {
    const int n_s = E.n_s;
    const uint64_t N = dim_of(n_s);
    const int anc = n_s + n_c;
    const uint64_t abit = 1ull << anc;
    const hipStream_t st = s->stream;

    const int L = pick_log_len(N, n_c);
    if (((1ull << n_c) >> L) < 4) return fail(SV_EUNSUPPORTED, "eigen-frame mode needs n_c >= 2");
    const dim3 g2((unsigned)((N + 63) / 64), (unsigned)(((1ull << n_c) >> L) / 4));
    const uint64_t half = dim_of(n_s + n_c);
    uint64_t nb = (half + 256 * 64 - 1) / (256 * 64);
    if (nb > 4096) nb = 4096;
    const uint64_t chunk = (half + nb - 1) / nb;

    SV_TRY(need(w.F, N * n_c * sizeof(uint64_t)));
    SV_TRY(need(w.beta, N * sizeof(double2)));
    SV_TRY(need(w.tmp, N * sizeof(double2)));
    SV_TRY(need(w.z, N * sizeof(double2)));
    SV_TRY(need(w.x, N * sizeof(double2)));
    SV_TRY(need(w.part, 2 * nb * sizeof(double)));
    SV_TRY(need(w.zpart, (size_t)g2.y * 4 * N * sizeof(double2)));
    SV_TRY(need(w.sum, 4 * sizeof(double)));
    hipLaunchKernelGGL(k_turn_table, dim3(grid1(N * n_c)), dim3(256), 0, st, (uint64_t *)w.F.p,
                       (const double *)E.lam_dev.p, T0, n_c, N);
    SV_HIP(hipGetLastError());
    const bool dev = b_dev != nullptr;
    if (dev) {
        // b on the device: its norm (w.sum[2]) and b^ there
        SV_TRY(need(w.tmp2, 512 * sizeof(double)));
        vec_norm2(st, b_dev, N, (double *)w.tmp2.p, (double *)w.sum.p + 2);
        hipLaunchKernelGGL(k_vec_normalise, dim3(grid1(N)), dim3(256), 0, st, (double2 *)w.x.p, b_dev, N,
                           (const double *)w.sum.p + 2);
        SV_HIP(hipGetLastError());
    } else {
        SV_TRY(upload(s, w.x.p, bhat.data(), N * sizeof(double2)));
    }
    // beta = V^H b^
    SV_TRY(kron_apply_frame(s, (double2 *)w.beta.p, (const double2 *)w.x.p, (double2 *)w.tmp.p, E, 1, w.gpart));

    if (fused && pipe_supported(n_s, n_c)) {
        // fused three-kernel pipeline: (state + inverse QFT on the low clock bits),
        // (inverse QFT high + rotation), (uncompute projected on clock 0)
        const uint64_t nbp = pipe_b_blocks(n_s, n_c, sizeof(cvec<R>));
        const int rows = pipe_c_rows(n_c);
        SV_TRY(need(w.part, 2 * nbp * sizeof(double)));
        SV_TRY(need(w.zpart, (size_t)rows * N * sizeof(double2)));
        uint64_t nparts = 0;
        SV_TRY(pipe_run<R>(s, n_s, n_c, sgn, gcut, (const double2 *)w.beta.p, (const uint64_t *)w.F.p, (double *)w.part.p,
                           (double2 *)w.zpart.p, &nparts));
        if (nparts > nbp) return fail(SV_EDEVICE, "pipeline partial count exceeds its buffer");
        SV_TRY(need(w.tmp2, 512 * sizeof(double)));
        sum_partials(st, (const double *)w.part.p, nparts, 2, (double *)w.tmp2.p, (double *)w.sum.p);
        sum_partials(st, (const double *)w.part.p + 1, nparts, 2, (double *)w.tmp2.p + 256, (double *)w.sum.p + 1);
        // 2^(-n_c/2) of the final Hadamard layer, and 2^(-g1/2) the fused forward
        // transform on the low clock group leaves out of its butterflies
        const int g1 = (n_c + 1) / 2;
        hipLaunchKernelGGL(k_sum_cols, dim3(grid1(N)), dim3(256), 0, st, (double2 *)w.z.p,
                           (const double2 *)w.zpart.p, N, rows, exp2(-0.5 * (n_c + g1)));
        SV_HIP(hipGetLastError());
        return eig_finish(s, E, w, N, res, x_out, dev, x_dev);
    }
    std::vector<double> cs;
    inversion_table(n_c, cs, sgn, gcut);
    SV_TRY(need(w.cs, cs.size() * sizeof(double)));
    SV_TRY(upload(s, w.cs.p, cs.data(), cs.size() * sizeof(double)));
    // 1. the state after phase estimation, written directly (ancilla = 0 half)
    {
        TraceScope _ts(st, "eig_init", (double)half * sizeof(cvec<R>), 0.0);
        hipLaunchKernelGGL(k_eig_init<R>, g2, dim3(256), 0, st, (cvec<R> *)s->data, (const double2 *)w.beta.p,
                           (const uint64_t *)w.F.p, N, n_s, n_c, L, 1.0 / sqrt((double)(1ull << n_c)));
    }
    SV_HIP(hipGetLastError());
    // 2. inverse QFT cascade on the clock, ancilla = 0 half
    SV_TRY(run_qft_cascade(s, QftSpec{n_s, n_c, 1, abit, 0}, 0));
    // 3. eigenvalue inversion: ancilla = 1 half <- s_y (ancilla = 0 half)
    {
        TraceScope _ts(st, "eig_ry", 2.0 * (double)half * sizeof(cvec<R>), 0.0);
        hipLaunchKernelGGL(k_eig_ry<R>, dim3((unsigned)nb), dim3(256), 0, st, (cvec<R> *)s->data,
                           (const double2 *)w.cs.p, half, n_s, (1ull << n_c) - 1ull, abit, chunk, (double *)w.part.p);
    }
    hipLaunchKernelGGL(k_sum_partials_strided, dim3(1), dim3(256), 0, st, (const double *)w.part.p, (int)nb, 2,
                       (double *)w.sum.p);
    hipLaunchKernelGGL(k_sum_partials_strided, dim3(1), dim3(256), 0, st, (const double *)w.part.p + 1, (int)nb, 2,
                       (double *)w.sum.p + 1);
    SV_HIP(hipGetLastError());
    // 4. QFT cascade on the clock, ancilla = 1 half
    SV_TRY(run_qft_cascade(s, QftSpec{n_s, n_c, 0, abit, abit}, 0));
    // 5. conjugate phases + Hadamards + clock = 0 projection
    {
        TraceScope _ts(st, "eig_project", (double)half * sizeof(cvec<R>), 0.0);
        hipLaunchKernelGGL(k_eig_project<R>, g2, dim3(256), 0, st, (const cvec<R> *)s->data,
                           (const uint64_t *)w.F.p, N, n_s, n_c, L, abit, (double2 *)w.zpart.p);
    }
    hipLaunchKernelGGL(k_sum_cols, dim3(grid1(N)), dim3(256), 0, st, (double2 *)w.z.p, (const double2 *)w.zpart.p, N,
                       (int)(g2.y * 4), 1.0 / sqrt((double)(1ull << n_c)));
    SV_HIP(hipGetLastError());
    return eig_finish(s, E, w, N, res, x_out, dev, x_dev);
}

// x = V z on the device, then P(a=1, clock=0) = |z|^2 and the normalised x on the host
static sv_status eig_finish(sv_state s, const EigFrame &E, Workspace &w, uint64_t N, sv_hhl_result *res,
                            double *x_out, bool dev, double2 *x_dev) {
    const hipStream_t st = s->stream;
    SV_TRY(kron_apply_frame(s, (double2 *)w.x.p, (const double2 *)w.z.p, (double2 *)w.tmp.p, E, 0, w.gpart));
    if (dev) {
        // p = |x|^2 (w.sum[3]) and the normalised x on the device; only the scalars come back
        SV_TRY(need(w.tmp2, 512 * sizeof(double)));
        vec_norm2(st, (const double2 *)w.x.p, N, (double *)w.tmp2.p, (double *)w.sum.p + 3);
        if (x_dev)
            hipLaunchKernelGGL(k_vec_normalise, dim3(grid1(N)), dim3(256), 0, st, x_dev, (const double2 *)w.x.p, N,
                               (const double *)w.sum.p + 3);
        SV_HIP(hipGetLastError());
        std::vector<double> sums(4);
        SV_TRY(download(s, sums.data(), w.sum.p, 4 * sizeof(double)));
        res->p_post = sums[3];
        res->p_anc = sums[0];
        res->norm_total = sums[1];
        if (!(sums[2] > 0.0) || !isfinite(sums[2])) return fail(SV_EZERONORM, "|b| = 0 or not finite");
        if (!(sums[3] > 0.0)) return fail(SV_EZERONORM, "post-selected outcome has probability 0");
        return SV_OK;
    }
    std::vector<double> sums(2), xz(2 * N);
    SV_TRY(download(s, sums.data(), w.sum.p, 2 * sizeof(double)));
    SV_TRY(download(s, xz.data(), w.x.p, N * sizeof(double2)));
    double p = 0.0;
    for (uint64_t j = 0; j < N; ++j) p += xz[2 * j] * xz[2 * j] + xz[2 * j + 1] * xz[2 * j + 1];
    res->p_post = p;
    res->p_anc = sums[0];
    res->norm_total = sums[1];
    if (!(p > 0.0)) return fail(SV_EZERONORM, "post-selected outcome has probability 0");
    if (x_out) {
        const double inv = 1.0 / sqrt(p);
        for (uint64_t j = 0; j < 2 * N; ++j) x_out[j] = xz[j] * inv;
    }
    return SV_OK;
}

// V = V_hi (x) V_lo as a dense row-major matrix
__global__ void k_kron_matrix(double2 *__restrict__ V, const double2 *__restrict__ Vh, const double2 *__restrict__ Vl,
                              int nh, int nl) {
    const uint64_t N = (uint64_t)nh * nl, total = N * N;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t row = i / N, col = i % N;
        const double2 a = Vh[(row / nl) * nh + col / nl], b = Vl[(row % nl) * nl + col % nl];
        V[i] = make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
    }
}

template <typename R>
static sv_status gate_faithful_run(sv_state s, const double2 *dV, const std::vector<double> &lam, Workspace &w, bool sgn,
                                   uint64_t gcut, int n_s, int n_c, double T0, const double *b, sv_hhl_result *res,
                                   double *x_out) {
    const int N = 1 << n_s;
    const hipStream_t st = s->stream;
    // U_k = V diag(E_k) V^H for k = 0..n_c-1, FP64, then rounded to the state's precision
    std::vector<double> Ek(2 * (size_t)N * n_c);
    for (int k = 0; k < n_c; ++k)
        for (int j = 0; j < N; ++j) {
            const double phi = lam[j] * T0 / (2.0 * M_PI);
            const double x = ldexp(phi, k), f = x - floor(x);
            Ek[2 * ((size_t)k * N + j)] = cos(2.0 * M_PI * f);
            Ek[2 * ((size_t)k * N + j) + 1] = sin(2.0 * M_PI * f);
        }
    const uint64_t NN = (uint64_t)N * N;
    SV_TRY(need(w.E, Ek.size() * sizeof(double)));
    SV_TRY(need(w.W, NN * sizeof(double2)));
    SV_TRY(need(w.U64, NN * sizeof(double2)));
    SV_TRY(need(w.Uk, (size_t)n_c * NN * sizeof(cvec<R>)));
    SV_TRY(upload(s, w.E.p, Ek.data(), Ek.size() * sizeof(double)));
    for (int k = 0; k < n_c; ++k) {
        hipLaunchKernelGGL(k_scale_cols, dim3(grid1(NN)), dim3(256), 0, st, (double2 *)w.W.p, dV,
                           (const double2 *)w.E.p + (size_t)k * N, N);
        double2 *dst = std::is_same<R, double>::value ? (double2 *)w.Uk.p + (size_t)k * NN : (double2 *)w.U64.p;
        SV_TRY(cgemm<double>(st, (const double2 *)w.W.p, dst, dV, (uint64_t)N, N, N, (uint64_t)(N - 1) << n_s, 0, 0,
                             1));
        if (!std::is_same<R, double>::value)
            hipLaunchKernelGGL(k_c128_to_c64, dim3(grid1(NN)), dim3(256), 0, st, (float2 *)w.Uk.p + (size_t)k * NN,
                               (const double2 *)w.U64.p, NN);
    }
    SV_HIP(hipGetLastError());
    const cvec<R> *U = (const cvec<R> *)w.Uk.p;

    SV_TRY(sv_init_b(s, b, n_s, n_c));
    for (int k = 0; k < n_c; ++k) SV_TRY(ctrl_unitary_impl<R>(s, U + (size_t)k * NN, n_s, n_s + (n_c - 1 - k), 1, 0));
    SV_TRY(run_qft_cascade(s, QftSpec{n_s, n_c, 1, 0, 0}, 0));
    std::vector<double> cs;
    inversion_table(n_c, cs, sgn, gcut);
    SV_TRY(sv_apply_uniform_ry(s, n_s + n_c, n_s, n_c, cs.data(), -1, 0));
    SV_TRY(run_qft_cascade(s, QftSpec{n_s, n_c, 0, 0, 0}, 0));
    for (int k = n_c - 1; k >= 0; --k)
        SV_TRY(ctrl_unitary_impl<R>(s, U + (size_t)k * NN, n_s, n_s + (n_c - 1 - k), 1, 1));
    SV_TRY(run_hadamards(s, n_s, n_c, 0, 0));
    SV_TRY(bitrev_register(s, n_s, n_c, 0, 0));

    const uint64_t abit = 1ull << (n_s + n_c), cmask = ((1ull << n_c) - 1ull) << n_s;
    SV_TRY(sv_norm2(s, abit, abit, &res->p_anc));
    SV_TRY(sv_norm2(s, 0, 0, &res->norm_total));
    return sv_postselect(s, abit | cmask, abit, &res->p_post, x_out, 0);
}

static sv_status check_params(sv_state s, const sv_hhl_params *prm, sv_hhl_result *res) {
    if (!prm || !res) return fail(SV_EINVAL, "params/result is NULL");
    if (prm->signed_clock != 0 && prm->signed_clock != 1) return fail(SV_EINVAL, "signed_clock must be 0 or 1");
    if (prm->n_s < 1 || prm->n_c < 1 || prm->n_s + prm->n_c + 1 != s->n)
        return fail(SV_EINVAL, "n_s %d + n_c %d + 1 != %d qubits", prm->n_s, prm->n_c, s->n);
    if (!(prm->T0 > 0.0) || !isfinite(prm->T0)) return fail(SV_EINVAL, "T0 must be positive");
    if (prm->mode < 0 || prm->mode > 2) return fail(SV_EINVAL, "mode must be 0, 1 or 2");
    if (prm->n_c > EIG_MAXC) return fail(SV_EUNSUPPORTED, "n_c %d > %d", prm->n_c, EIG_MAXC);
    return SV_OK;
}

static sv_status normalise_b(const double *b, uint64_t N, std::vector<double> &bhat) {
    double nrm = 0.0;
    for (uint64_t j = 0; j < 2 * N; ++j) nrm += b[j] * b[j];
    nrm = sqrt(nrm);
    if (!(nrm > 0.0) || !isfinite(nrm)) return fail(SV_EZERONORM, "|b| = 0 or not finite");
    bhat.resize(2 * N);
    for (uint64_t j = 0; j < 2 * N; ++j) bhat[j] = b[j] / nrm;
    return SV_OK;
}

}  // namespace sv

struct sv_hhl_plan_s {
    sv::EigFrame E;
    sv::DevBuf V_dense;     // V_hi (x) V_lo, built on first gate-faithful run of a Kronecker plan
    sv::Workspace w;
    // the spectrum's range and whether it holds a zero, from E.lam (fixed once
    // prepared), computed on first use instead of on every solve
    bool have_range = false, has_zero = false;
    double lam_lo = 0.0, lam_hi = 0.0;
    void range() {
        if (have_range) return;
        lam_lo = lam_hi = E.lam[0];
        for (double v : E.lam) {
            lam_lo = fmin(lam_lo, v);
            lam_hi = fmax(lam_hi, v);
            if (!(v != 0.0)) has_zero = true;
        }
        have_range = true;
    }
};

using namespace sv;

extern "C" {

const char *sv_last_eigensolver(void) { return eigh_last_solver(); }

sv_status sv_hhl_prepare(sv_hhl_plan *out, sv_state s, const double *A_hi, int m_hi, const double *A_lo, int m_lo) {
    clear_error();
    if (!out) return fail(SV_EINVAL, "out is NULL");
    *out = nullptr;
    SV_TRY(check_state(s));
    if (!A_hi || m_hi < 1 || m_lo < 0 || (m_lo > 0 && !A_lo)) return fail(SV_EINVAL, "bad operator arguments");
    if (m_hi > 13 || m_lo > 13) return fail(SV_EUNSUPPORTED, "factor larger than 2^13");
    const int nh = 1 << m_hi, nl = 1 << m_lo;
    SV_TRY(check_hermitian(A_hi, nh, m_lo ? "A_hi" : "A"));
    if (m_lo) SV_TRY(check_hermitian(A_lo, nl, "A_lo"));
    sv_hhl_plan p = new sv_hhl_plan_s();
    p->E.n_s = m_hi + m_lo;
    p->E.n_hi = nh;
    p->E.n_lo = nl;
    sv_status st = eigh_device(s, A_hi, nh, p->E.V_hi, p->E.lam);
    if (st == SV_OK && m_lo) {
        std::vector<double> mu = p->E.lam, nu;
        st = eigh_device(s, A_lo, nl, p->E.V_lo, nu);
        if (st == SV_OK) {
            p->E.lam.resize((size_t)nh * nl);
            for (int a = 0; a < nh; ++a)
                for (int q = 0; q < nl; ++q) p->E.lam[(size_t)a * nl + q] = mu[a] + nu[q];
        }
    }
    // V_hi^H: the rows of the high-axis GEMM of the V^H basis change (Kronecker plans)
    if (st == SV_OK && m_lo) st = p->E.VH_hi.alloc((size_t)nh * nh * sizeof(double2));
    if (st == SV_OK && m_lo) {
        hipLaunchKernelGGL(k_conj_transpose, dim3(grid1((uint64_t)nh * nh)), dim3(256), 0, s->stream,
                           (double2 *)p->E.VH_hi.p, (const double2 *)p->E.V_hi.p, nh);
        const hipError_t he = hipGetLastError();
        if (he != hipSuccess) st = hip_fail(he, "k_conj_transpose");
    }
    if (st == SV_OK) st = p->E.lam_dev.alloc(p->E.lam.size() * sizeof(double));
    if (st == SV_OK) st = upload(s, p->E.lam_dev.p, p->E.lam.data(), p->E.lam.size() * sizeof(double));
    if (st != SV_OK) {
        delete p;
        return st;
    }
    *out = p;
    return SV_OK;
}

sv_status sv_hhl_prepare_eig(sv_hhl_plan *out, sv_state s, const double *V_dev, const double *lam, int n_s) {
    clear_error();
    if (!out) return fail(SV_EINVAL, "out is NULL");
    *out = nullptr;
    SV_TRY(check_state(s));
    if (!V_dev || !lam) return fail(SV_EINVAL, "V_dev/lam is NULL");
    if (n_s < 1 || n_s > 16) return fail(SV_EINVAL, "n_s = %d outside [1, 16]", n_s);
    const uint64_t N = dim_of(n_s);
    for (uint64_t j = 0; j < N; ++j)
        if (!isfinite(lam[j])) return fail(SV_EINVAL, "eigenvalue %llu is not finite", (unsigned long long)j);
    sv_hhl_plan p = new sv_hhl_plan_s();
    p->E.n_s = n_s;
    p->E.n_hi = (int)N;
    p->E.n_lo = 1;
    p->E.lam.assign(lam, lam + N);
    p->E.Vr = V_dev;
    sv_status st = p->E.lam_dev.alloc(N * sizeof(double));
    if (st == SV_OK) st = upload(s, p->E.lam_dev.p, lam, N * sizeof(double));
    // orthogonality probe through the basis-change kernels: V V^T r = r for a
    // fixed pseudo-random r (splitmix64 draws in [-1, 1))
    if (st == SV_OK) {
        std::vector<double> r(2 * N), u(2 * N);
        uint64_t x = 0x9e3779b97f4a7c15ull;
        for (uint64_t i = 0; i < 2 * N; ++i) {
            x += 0x9e3779b97f4a7c15ull;
            uint64_t z = x;
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
            z ^= z >> 31;
            r[i] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
        }
        DevBuf dr, dt, du, dp;
        st = dr.alloc(N * sizeof(double2));
        if (st == SV_OK) st = dt.alloc(N * sizeof(double2));
        if (st == SV_OK) st = du.alloc(N * sizeof(double2));
        if (st == SV_OK) st = dp.alloc(gemv_part_bytes(N));
        if (st == SV_OK) st = upload(s, dr.p, r.data(), N * sizeof(double2));
        if (st == SV_OK)
            st = gemv_apply(s->stream, (double2 *)dt.p, (const double2 *)dr.p, V_dev, nullptr, N, 1, nullptr);
        if (st == SV_OK)
            st = gemv_apply(s->stream, (double2 *)du.p, (const double2 *)dt.p, V_dev, nullptr, N, 0, (double2 *)dp.p);
        if (st == SV_OK) st = download(s, u.data(), du.p, N * sizeof(double2));
        if (st == SV_OK) {
            double e2 = 0.0, r2 = 0.0;
            for (uint64_t i = 0; i < 2 * N; ++i) {
                e2 += (u[i] - r[i]) * (u[i] - r[i]);
                r2 += r[i] * r[i];
            }
            if (!(e2 <= 1e-20 * r2)) st = fail(SV_EINVAL, "V is not orthogonal (|V V^T r - r| / |r| = %g)", sqrt(e2 / r2));
        }
    }
    // the gate-faithful mode needs the complex V (small operators only)
    if (st == SV_OK && n_s <= 13) {
        st = p->E.V_hi.alloc(N * N * sizeof(double2));
        if (st == SV_OK) {
            hipLaunchKernelGGL(k_real_to_complex, dim3(grid1(N * N)), dim3(256), 0, s->stream, (double2 *)p->E.V_hi.p,
                               V_dev, N * N);
            const hipError_t he = hipGetLastError();
            if (he != hipSuccess) st = hip_fail(he, "k_real_to_complex");
        }
    }
    if (st != SV_OK) {
        delete p;
        return st;
    }
    *out = p;
    return SV_OK;
}

sv_status sv_hhl_plan_spectrum(sv_hhl_plan p, double *lambda_min, double *lambda_max) {
    if (!p) return fail(SV_EINVAL, "null plan");
    p->range();
    if (lambda_min) *lambda_min = p->lam_lo;
    if (lambda_max) *lambda_max = p->lam_hi;
    return SV_OK;
}

// the solve on a prepared operator: gcut = 0 the HHL inversion, gcut >= 1 the
// gapped-phase-estimation flag (which allows a zero eigenvalue on a signed
// clock and lambda_min = 0 on an unsigned one)
static sv_status hhl_run_impl(sv_hhl_plan p, sv_state s, const double *b, const sv_hhl_params *prm, uint64_t gcut,
                              sv_hhl_result *res, double *x_out, const double2 *b_dev = nullptr,
                              double2 *x_dev = nullptr) {
    if (!p) return fail(SV_EINVAL, "null plan");
    SV_TRY(check_state(s));
    SV_TRY(check_params(s, prm, res));
    if (!b && !b_dev) return fail(SV_EINVAL, "b is NULL");
    if (prm->n_s != p->E.n_s) return fail(SV_EINVAL, "plan has n_s = %d, params n_s = %d", p->E.n_s, prm->n_s);
    if (b_dev && prm->mode == 0) return fail(SV_EUNSUPPORTED, "device-resident b and x need mode 1 or 2");
    const uint64_t N = dim_of(p->E.n_s);
    std::vector<double> bhat;
    if (!b_dev) SV_TRY(normalise_b(b, N, bhat));
    SV_TRY(sv_hhl_plan_spectrum(p, &res->lambda_min, &res->lambda_max));
    const bool sgn = prm->signed_clock == 1;
    if (gcut == 0) {
        if (!sgn && !(res->lambda_min > 0.0))
            return fail(SV_ENOTPOSDEF, "lambda_min = %g <= 0 (unsigned clock)", res->lambda_min);
        if (sgn && p->has_zero) return fail(SV_EINVAL, "A is singular (a zero eigenvalue)");
    } else if (!sgn && !(res->lambda_min >= 0.0)) {
        return fail(SV_ENOTPOSDEF, "lambda_min = %g < 0 (unsigned clock)", res->lambda_min);
    }
    if (prm->mode >= 1) {
        const bool fused = prm->mode == 1;
        return s->dt == SV_C64
                   ? eig_frame_run<float>(s, p->E, p->w, bhat, prm->n_c, sgn, gcut, prm->T0, fused, res, x_out,
                                          b_dev, x_dev)
                   : eig_frame_run<double>(s, p->E, p->w, bhat, prm->n_c, sgn, gcut, prm->T0, fused, res, x_out,
                                           b_dev, x_dev);
    }
    // gate-faithful: dense eigenvectors
    if (p->E.n_s > 13 || !p->E.V_hi.p) return fail(SV_EUNSUPPORTED, "gate-faithful mode with n_s = %d > 13", p->E.n_s);
    const double2 *dV = (const double2 *)p->E.V_hi.p;
    if (p->E.n_lo > 1) {
        if (!p->V_dense.p) {
            SV_TRY(p->V_dense.ensure(N * N * sizeof(double2)));
            hipLaunchKernelGGL(k_kron_matrix, dim3(grid1(N * N)), dim3(256), 0, s->stream, (double2 *)p->V_dense.p,
                               (const double2 *)p->E.V_hi.p, (const double2 *)p->E.V_lo.p, p->E.n_hi, p->E.n_lo);
            SV_HIP(hipGetLastError());
        }
        dV = (const double2 *)p->V_dense.p;
    }
    if (s->dt == SV_C64)
        return gate_faithful_run<float>(s, dV, p->E.lam, p->w, sgn, gcut, p->E.n_s, prm->n_c, prm->T0, bhat.data(),
                                        res, x_out);
    return gate_faithful_run<double>(s, dV, p->E.lam, p->w, sgn, gcut, p->E.n_s, prm->n_c, prm->T0, bhat.data(), res,
                                     x_out);
}

sv_status sv_hhl_run(sv_hhl_plan p, sv_state s, const double *b, const sv_hhl_params *prm, sv_hhl_result *res,
                     double *x_out) {
    clear_error();
    return hhl_run_impl(p, s, b, prm, 0, res, x_out);
}

sv_status sv_hhl_run_device(sv_hhl_plan p, sv_state s, const void *b_dev, const sv_hhl_params *prm,
                            sv_hhl_result *res, void *x_dev) {
    clear_error();
    if (!b_dev) return fail(SV_EINVAL, "b_dev is NULL");
    return hhl_run_impl(p, s, nullptr, prm, 0, res, nullptr, (const double2 *)b_dev, (double2 *)x_dev);
}

sv_status sv_hhl_plan_free(sv_hhl_plan p) {
    if (p) {
        hipDeviceSynchronize();
        delete p;
    }
    return SV_OK;
}

sv_status sv_hhl(sv_state s, const double *A, const double *b, const sv_hhl_params *prm, sv_hhl_result *res,
                 double *x_out) {
    clear_error();
    SV_TRY(check_state(s));
    SV_TRY(check_params(s, prm, res));
    if (!A || !b) return fail(SV_EINVAL, "A/b is NULL");
    if (prm->n_s > 13) return fail(SV_EUNSUPPORTED, "dense A with n_s = %d (use sv_hhl_kron)", prm->n_s);
    std::vector<double> bhat;
    SV_TRY(normalise_b(b, dim_of(prm->n_s), bhat));
    sv_hhl_plan p = nullptr;
    SV_TRY(sv_hhl_prepare(&p, s, A, prm->n_s, nullptr, 0));
    sv_status st = sv_hhl_run(p, s, b, prm, res, x_out);
    std::string keep = sv_last_error();
    sv_hhl_plan_free(p);
    if (st != SV_OK) fail(st, "%s", keep.c_str());
    return st;
}

static sv_status gpe_check(sv_state s, const sv_gpe_params *g, sv_hhl_params &prm, sv_hhl_result *res) {
    if (!g) return fail(SV_EINVAL, "params is NULL");
    prm = sv_hhl_params{g->n_s, g->n_c, g->T0, g->mode, g->signed_clock};
    SV_TRY(check_params(s, &prm, res));
    const uint64_t top = prm.signed_clock ? (1ull << (prm.n_c - 1)) : (1ull << prm.n_c);
    if (g->cut < 1 || g->cut >= top)
        return fail(SV_EINVAL, "cut %llu outside [1, %llu)", (unsigned long long)g->cut, (unsigned long long)top);
    return SV_OK;
}

sv_status sv_gapped_pe_run(sv_hhl_plan p, sv_state s, const double *b, const sv_gpe_params *g, sv_hhl_result *res,
                           double *x_out) {
    clear_error();
    SV_TRY(check_state(s));
    sv_hhl_params prm;
    SV_TRY(gpe_check(s, g, prm, res));
    return hhl_run_impl(p, s, b, &prm, g->cut, res, x_out);
}

sv_status sv_gapped_pe(sv_state s, const double *A, const double *b, const sv_gpe_params *g, sv_hhl_result *res,
                       double *x_out) {
    clear_error();
    SV_TRY(check_state(s));
    sv_hhl_params prm;
    SV_TRY(gpe_check(s, g, prm, res));
    if (!A || !b) return fail(SV_EINVAL, "A/b is NULL");
    if (prm.n_s > 13) return fail(SV_EUNSUPPORTED, "dense A with n_s = %d (use sv_gapped_pe_run on a plan)", prm.n_s);
    std::vector<double> bhat;
    SV_TRY(normalise_b(b, dim_of(prm.n_s), bhat));
    sv_hhl_plan p = nullptr;
    SV_TRY(sv_hhl_prepare(&p, s, A, prm.n_s, nullptr, 0));
    sv_status st = hhl_run_impl(p, s, b, &prm, g->cut, res, x_out);
    std::string keep = sv_last_error();
    sv_hhl_plan_free(p);
    if (st != SV_OK) fail(st, "%s", keep.c_str());
    return st;
}

sv_status sv_hhl_kron(sv_state s, const double *A_hi, int m_hi, const double *A_lo, int m_lo, const double *b,
                      const sv_hhl_params *prm, sv_hhl_result *res, double *x_out) {
    clear_error();
    SV_TRY(check_state(s));
    SV_TRY(check_params(s, prm, res));
    if (!A_hi || !A_lo || !b) return fail(SV_EINVAL, "A_hi/A_lo/b is NULL");
    if (m_hi < 1 || m_lo < 1 || m_hi + m_lo != prm->n_s) return fail(SV_EINVAL, "m_hi + m_lo != n_s");
    std::vector<double> bhat;
    SV_TRY(normalise_b(b, dim_of(prm->n_s), bhat));
    sv_hhl_plan p = nullptr;
    SV_TRY(sv_hhl_prepare(&p, s, A_hi, m_hi, A_lo, m_lo));
    sv_status st = sv_hhl_run(p, s, b, prm, res, x_out);
    std::string keep = sv_last_error();
    sv_hhl_plan_free(p);
    if (st != SV_OK) fail(st, "%s", keep.c_str());
    return st;
}

}  // extern "C"
