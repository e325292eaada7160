// Cheap spectrum features: the extreme eigenvalues of a Hermitian matrix by
// Lanczos iteration on the GPU (full reorthogonalisation, every coefficient
// kept in device memory, no host round trip per step), then Sturm-sequence
// bisection of the small Lanczos tridiagonal matrix on the host.
//
// Per step j (q_j the current unit vector, Q = [q_0 .. q_j]):
//   w = A q_j                                  one wavefront per matrix row
//   twice: h = Q^H w,  w -= Q h                classical Gram-Schmidt, repeated
//   alpha_j = Re(h_j of both passes)
//   beta_j = |w|,  q_{j+1} = w / beta_j        one workgroup
#include <math.h>

#include <vector>

#include "sv_device.h"
#include "sv_hhl_internal.h"
#include "sv_internal.h"

namespace sv {

constexpr int LZ_MAX_N = 8192;

// w[r] = sum_c A[r][c] q[c]; 4 rows per 256-thread workgroup
__global__ __launch_bounds__(256) void k_lz_matvec(const double2 *__restrict__ A, const double2 *__restrict__ q,
                                                   double2 *__restrict__ w, int N) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= N) return;   // uniform per wavefront
    const double2 *a = A + (size_t)row * N;
    double sr = 0.0, si = 0.0;
    for (int c = lane; c < N; c += 64) {
        const double2 x = a[c], y = q[c];
        sr += x.x * y.x - x.y * y.y;
        si += x.x * y.y + x.y * y.x;
    }
    sr = wave_sum_f64(sr);
    si = wave_sum_f64(si);
    if (lane == 0) w[row] = make_double2(sr, si);
}

// banded form: w[r] = sum_d B[d][r] q[r + d - bw] for a Hermitian matrix of
// half-bandwidth bw stored by diagonals (B[d][r] = A[r][r + d - bw], zero
// outside the matrix); one thread per row
__global__ __launch_bounds__(256) void k_lz_matvec_band(const double2 *__restrict__ Bd, const double2 *__restrict__ q,
                                                        double2 *__restrict__ w, int N, int bw) {
    const int row = blockIdx.x * 256 + threadIdx.x;
    if (row >= N) return;
    double sr = 0.0, si = 0.0;
    for (int d = 0; d <= 2 * bw; ++d) {
        const int c = row + d - bw;
        if (c < 0 || c >= N) continue;
        const double2 x = Bd[(size_t)d * N + row], y = q[c];
        sr += x.x * y.x - x.y * y.y;
        si += x.x * y.y + x.y * y.x;
    }
    w[row] = make_double2(sr, si);
}

__device__ __forceinline__ double block_sum_256(double v, double *ws) {
    v = wave_sum_f64(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    return (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// h[i] = <q_i, w> for i = blockIdx.x (one workgroup per basis vector)
__global__ __launch_bounds__(256) void k_lz_dots(const double2 *__restrict__ Q, const double2 *__restrict__ w,
                                                 double2 *__restrict__ h, int N) {
    __shared__ double ws[4];
    const double2 *q = Q + (size_t)blockIdx.x * N;
    double re = 0.0, im = 0.0;
    for (int r = threadIdx.x; r < N; r += 256) {
        const double2 a = q[r], b = w[r];
        re += a.x * b.x + a.y * b.y;
        im += a.x * b.y - a.y * b.x;
    }
    re = block_sum_256(re, ws);
    im = block_sum_256(im, ws);
    if (threadIdx.x == 0) h[blockIdx.x] = make_double2(re, im);
}

// w -= sum_{i <= j} h[i] q_i; the first pass sets alpha[j], the second adds to it
__global__ __launch_bounds__(256) void k_lz_update(const double2 *__restrict__ Q, double2 *__restrict__ w,
                                                   const double2 *__restrict__ h, int j, int N,
                                                   double *__restrict__ alpha, int second) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) alpha[j] = (second ? alpha[j] : 0.0) + h[j].x;
    if (r >= N) return;
    double2 v = w[r];
    for (int i = 0; i <= j; ++i) {
        const double2 c = h[i], q = Q[(size_t)i * N + r];
        v.x -= c.x * q.x - c.y * q.y;
        v.y -= c.x * q.y + c.y * q.x;
    }
    w[r] = v;
}

// beta[j] = |w|, q_next = w / beta[j] (zero if w vanished); one workgroup of 1024
__global__ __launch_bounds__(1024) void k_lz_norm_scale(const double2 *__restrict__ w, double2 *__restrict__ qn,
                                                        double *__restrict__ beta, int j, int N) {
    __shared__ double ws[16];
    double s = 0.0;
    for (int r = threadIdx.x; r < N; r += 1024) s += w[r].x * w[r].x + w[r].y * w[r].y;
    s = wave_sum_f64(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += ws[i];
    const double b = sqrt(t);
    if (threadIdx.x == 0) beta[j] = b;
    const double inv = b > 0.0 ? 1.0 / b : 0.0;
    for (int r = threadIdx.x; r < N; r += 1024) qn[r] = make_double2(w[r].x * inv, w[r].y * inv);
}

// extreme eigenvalue of the symmetric tridiagonal (a, b) by bisection on the
// Sturm count (number of eigenvalues below x = negative pivots of T - x I)
static double sturm_extreme(const std::vector<double> &a, const std::vector<double> &b, bool smallest) {
    const int k = (int)a.size();
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {   // Gershgorin interval
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < k ? fabs(b[i]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
    }
    auto below = [&](double x) {
        int c = 0;
        double d = a[0] - x;
        if (d < 0) ++c;
        for (int i = 1; i < k; ++i) {
            d = a[i] - x - b[i - 1] * b[i - 1] / (d != 0.0 ? d : 1e-300);
            if (d < 0) ++c;
        }
        return c;
    };
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (smallest ? below(mid) >= 1 : below(mid) >= k) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// the Lanczos iteration and the Sturm bisection of its tridiagonal matrix;
// matvec(q, w) enqueues w = A q on st
template <typename MV>
static sv_status lanczos_run(hipStream_t st, int N, int iters, uint64_t seed, double *lambda_min, double *lambda_max,
                             MV matvec) {
    const int k = iters < N ? iters : N;
    // seeded start vector: xorshift64* stream, uniform in [-1/2, 1/2), normalised
    std::vector<double> q0(2 * (size_t)N, 0.0);
    uint64_t x = seed ^ 0x9e3779b97f4a7c15ull;
    double nrm = 0.0;
    for (int i = 0; i < N; ++i) {
        x ^= x >> 12;
        x ^= x << 25;
        x ^= x >> 27;
        const double r = (double)((x * 0x2545f4914f6cdd1dull) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        q0[2 * i] = r;
        nrm += r * r;
    }
    nrm = sqrt(nrm);
    if (!(nrm > 0.0)) q0[0] = nrm = 1.0;
    for (int i = 0; i < N; ++i) q0[2 * i] /= nrm;
    DevBuf dQ, dw, dh, dab;
    SV_TRY(dQ.alloc((size_t)(k + 1) * N * sizeof(double2)));
    SV_TRY(dw.alloc((size_t)N * sizeof(double2)));
    SV_TRY(dh.alloc((size_t)(k + 1) * sizeof(double2)));
    SV_TRY(dab.alloc(2 * (size_t)k * sizeof(double)));
    double2 *Q = (double2 *)dQ.p, *w = (double2 *)dw.p, *h = (double2 *)dh.p;
    double *alpha = (double *)dab.p, *beta = alpha + k;
    SV_HIP(hipMemcpyAsync(Q, q0.data(), (size_t)N * sizeof(double2), hipMemcpyHostToDevice, st));
    SV_HIP(hipMemsetAsync(dab.p, 0, 2 * (size_t)k * sizeof(double), st));
    const int vec_grid = (N + 255) / 256;
    for (int j = 0; j < k; ++j) {
        const double2 *qj = Q + (size_t)j * N;
        matvec(qj, w);
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(k_lz_dots, dim3(j + 1), dim3(256), 0, st, (const double2 *)Q, (const double2 *)w, h,
                               N);
            hipLaunchKernelGGL(k_lz_update, dim3(vec_grid), dim3(256), 0, st, (const double2 *)Q, w,
                               (const double2 *)h, j, N, alpha, pass);
        }
        if (j + 1 < k)
            hipLaunchKernelGGL(k_lz_norm_scale, dim3(1), dim3(1024), 0, st, (const double2 *)w, Q + (size_t)(j + 1) * N,
                               beta, j, N);
        SV_HIP(hipGetLastError());
    }
    std::vector<double> ab(2 * (size_t)k);
    SV_HIP(hipMemcpyAsync(ab.data(), dab.p, ab.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    SV_HIP(hipStreamSynchronize(st));
    // truncate at the first (numerical) breakdown: the Krylov space is invariant there
    double amax = 0.0;
    for (int j = 0; j < k; ++j) amax = fmax(amax, fabs(ab[j]));
    int m = k;
    for (int j = 0; j + 1 < k; ++j)
        if (!(ab[k + j] > 1e-13 * amax)) {
            m = j + 1;
            break;
        }
    std::vector<double> a(ab.begin(), ab.begin() + m), b(ab.begin() + k, ab.begin() + k + (m - 1));
    for (double v : a)
        if (!isfinite(v)) return fail(SV_EDEVICE, "Lanczos produced a non-finite coefficient");
    *lambda_min = sturm_extreme(a, b, true);
    *lambda_max = sturm_extreme(a, b, false);
    return SV_OK;
}

}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_spectrum_lanczos(const double *A, int N, int iters, uint64_t seed, double *lambda_min,
                              double *lambda_max, void *hip_stream) {
    clear_error();
    if (!A || !lambda_min || !lambda_max || iters < 1) return fail(SV_EINVAL, "bad Lanczos arguments");
    if (N < 1 || N > LZ_MAX_N) return fail(SV_EINVAL, "N = %d outside 1..%d", N, LZ_MAX_N);
    SV_TRY(check_hermitian(A, N, "A"));
    const hipStream_t st = (hipStream_t)hip_stream;
    DevBuf dA;
    SV_TRY(dA.alloc((size_t)N * N * sizeof(double2)));
    SV_HIP(hipMemcpyAsync(dA.p, A, (size_t)N * N * sizeof(double2), hipMemcpyHostToDevice, st));
    const int rows_grid = (N + 3) / 4;
    return lanczos_run(st, N, iters, seed, lambda_min, lambda_max, [&](const double2 *q, double2 *w) {
        hipLaunchKernelGGL(k_lz_matvec, dim3(rows_grid), dim3(256), 0, st, (const double2 *)dA.p, q, w, N);
    });
}

sv_status sv_spectrum_lanczos_band(const double *band, int N, int bw, int iters, uint64_t seed, double *lambda_min,
                                   double *lambda_max, void *hip_stream) {
    clear_error();
    if (!band || !lambda_min || !lambda_max || iters < 1 || bw < 0) return fail(SV_EINVAL, "bad Lanczos arguments");
    if (N < 1 || N > LZ_MAX_N || bw >= N) return fail(SV_EINVAL, "N = %d (1..%d), bw = %d", N, LZ_MAX_N, bw);
    // Hermitian: B[bw + e][r] = conj(B[bw - e][r + e]) for every stored pair
    double amax = 0.0, dmax = 0.0;
    for (int d = 0; d <= 2 * bw; ++d)
        for (int r = 0; r < N; ++r) {
            const double *x = band + 2 * ((size_t)d * N + r);
            if (!isfinite(x[0]) || !isfinite(x[1])) return fail(SV_EINVAL, "band has a non-finite entry");
            const int c = r + d - bw;
            if (c < 0 || c >= N) continue;
            const double *y = band + 2 * ((size_t)(2 * bw - d) * N + c);
            amax = fmax(amax, hypot(x[0], x[1]));
            dmax = fmax(dmax, hypot(x[0] - y[0], x[1] + y[1]));
        }
    if (dmax > 1e-12 * amax) return fail(SV_ENOTHERMITIAN, "band is not Hermitian (|B - B^H| = %g)", dmax);
    const hipStream_t st = (hipStream_t)hip_stream;
    DevBuf dB;
    const size_t bytes = (size_t)(2 * bw + 1) * N * sizeof(double2);
    SV_TRY(dB.alloc(bytes));
    SV_HIP(hipMemcpyAsync(dB.p, band, bytes, hipMemcpyHostToDevice, st));
    const int grid = (N + 255) / 256;
    return lanczos_run(st, N, iters, seed, lambda_min, lambda_max, [&](const double2 *q, double2 *w) {
        hipLaunchKernelGGL(k_lz_matvec_band, dim3(grid), dim3(256), 0, st, (const double2 *)dB.p, q, w, N, bw);
    });
}

}  // extern "C"
