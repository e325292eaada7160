// Internal pieces of the HHL drivers shared by sv_hhl.hip and sv_batch.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

// owning device buffer (freed with hipFree after a device-wide sync point)
struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    size_t bytes = 0;
    sv_status alloc(size_t bytes);
    sv_status ensure(size_t need) { return need <= bytes && p ? SV_OK : alloc(need); }
};

// per-solve operands of the fused eigen-frame kernels (one solve: passed by
// value; a batch: a device array indexed by blockIdx.z)
struct PipeSolve {
    void *psi;              // the state
    const double2 *beta;    // V^H b^ (FP64)
    const uint64_t *F;      // turn table [N][n_c]
    double *part;           // k_pipe_b partial sums (2 per block)
    double2 *zpart;         // k_pipe_c partial column sums [2^g2][N]
};

// the last step of a batched solve: FP64 sums of P(a=1) and the norm, the
// post-selected eigen-coefficients z_j (column sums of the clock projection),
// p_post = |z|^2 and F = |<x_C|x_Q>| = |sum conj(c_j) z_j| / |z|
struct FinishJob {
    const double *part;     // k_pipe_b partials, 2 per block (or queue item)
    uint64_t nparts;
    const double2 *zpart;   // [rows][N]
    int rows;
    uint64_t N;
    double scale;           // 2^(-(n_c + g1)/2)
    const double2 *cexact;  // normalised eigen-coefficients of A^{-1} b
    double *out;            // p_post, p_anc, norm_total, fidelity
};

__device__ __forceinline__ double finish_block_sum(double v, double *ws) {
    v = wave_sum_f64(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    return (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// one block of 256 threads per solve; fixed summation order
__device__ __forceinline__ void batch_finish_body(const FinishJob &J) {
    __shared__ double ws[4];
    double pa = 0.0, nt = 0.0, pp = 0.0, orr = 0.0, oi = 0.0;
    for (uint64_t i = threadIdx.x; i < J.nparts; i += blockDim.x) {
        pa += J.part[2 * i];
        nt += J.part[2 * i + 1];
    }
    for (uint64_t j = threadIdx.x; j < J.N; j += blockDim.x) {
        double zr = 0.0, zi = 0.0;
        for (int r = 0; r < J.rows; ++r) {
            const double2 v = J.zpart[(uint64_t)r * J.N + j];
            zr += v.x;
            zi += v.y;
        }
        zr *= J.scale;
        zi *= J.scale;
        pp += zr * zr + zi * zi;
        const double2 c = J.cexact[j];
        orr += c.x * zr + c.y * zi;      // conj(c) z
        oi += c.x * zi - c.y * zr;
    }
    pa = finish_block_sum(pa, ws);
    nt = finish_block_sum(nt, ws);
    pp = finish_block_sum(pp, ws);
    orr = finish_block_sum(orr, ws);
    oi = finish_block_sum(oi, ws);
    if (threadIdx.x == 0) {
        J.out[0] = pp;
        J.out[1] = pa;
        J.out[2] = nt;
        J.out[3] = pp > 0.0 ? sqrt(orr * orr + oi * oi) / sqrt(pp) : 0.0;
    }
}

// A batch as one persistent kernel over device work queues.  Every solve
// has four phases: the k_pipe_a tiles, the k_pipe_b tiles, the k_pipe_c
// tiles (each item a run of consecutive column blocks of one clock-group
// value) and the finish; an item of phase p > 0 waits until every item of
// phase p - 1 of its solve is done (one counter per solve and phase).  The
// solves are spread over one queue per XCC; a queue's items are numbered
// phase-major, so a wait only ever targets items taken before.
struct QueueClassIn {
    int n_s, n_c;
    int cl[3];              // log2 columns per tile of the three kernels
};
struct PipeQueue {
    const void *d_cls = nullptr;        // class table (launch parameters per phase)
    const void *d_solves = nullptr;     // solve table
    const uint64_t *d_items = nullptr;  // item codes: phase (2 bits), solve (20), wait target (21), index (21)
    uint32_t nitems = 0, nsolves = 0;
    int nq = 1;                         // queues (one per XCC)
    uint32_t qstart[9] = {};            // item range of every queue
    int xcc[8] = {-1, -1, -1, -1, -1, -1, -1, -1};   // the XCC serving each queue (-1: any)
    unsigned *cnt = nullptr;            // counters (pipe_queue_counters); zeroed before a run
    unsigned *flag = nullptr;           // set (never cleared by the kernel) if a bounded wait expired
    int blocks = 0;                     // resident blocks of 256 threads
    int gmax = 8;                       // widest clock group the kernel form carries (6 or 8)
    uint64_t wait_ticks = 0;            // bound of one dependency wait (wall-clock ticks)
    size_t lds = 0;
    std::vector<uint64_t> nparts;       // k_pipe_b partial pairs of every solve
    uint64_t items_per_phase[4] = {0, 0, 0, 0};
    double bytes = 0.0;                 // algorithmic HBM bytes of one run
};
// counters the queue needs for `nsolves` solves: three per solve, eight
// queue heads, the count of finished solves (the last)
inline size_t pipe_queue_counters(int nsolves) { return 3 * (size_t)nsolves + 8 + 1; }
// plan and upload the queue (descriptors into `desc`); solve k uses class solve_cls[k]
template <typename R>
sv_status pipe_queue_build(sv_state ctx, hipStream_t st, PipeQueue &q, DevBuf &desc,
                           const std::vector<QueueClassIn> &cls, const std::vector<int> &solve_cls,
                           const std::vector<PipeSolve> &solves, unsigned *cnt, unsigned *flag);
// one launch over every item; the counters must be zero
template <typename R>
sv_status pipe_queue_launch(hipStream_t st, const PipeQueue &q, const FinishJob *d_fin);

template <typename R>
sv_status pipe_config(hipStream_t st, int n_s, int n_c, const PipeSolve *tune_on, int cl[3], int nt[3]);
template <typename R>
sv_status pipe_run_batch(hipStream_t st, int n_s, int n_c, const int cl[3], const int nt[3],
                         const PipeSolve *dev_solves, int nsolves, uint64_t *nparts);
int pipe_supported(int n_s, int n_c);
uint64_t pipe_b_blocks_for(int n_s, int n_c, int cl);
uint64_t pipe_b_blocks(int n_s, int n_c, size_t elem);
int pipe_c_rows(int n_c);

// W[r][j] = V[r][j] * E[j] for an N x N row-major V (sv_hhl.hip)
__global__ void k_scale_cols(double2 *__restrict__ W, const double2 *__restrict__ V, const double2 *__restrict__ E,
                             int N);

// F[j][k] = frac(lam_j T0 / 2 pi 2^k) as 64-bit turn fractions (sv_hhl.hip)
__global__ void k_turn_table(uint64_t *__restrict__ F, const double *__restrict__ lam, double T0, int n_c,
                             uint64_t N);

// eigen-decomposition of A = A_hi (x) I + I (x) A_lo (dense A: n_lo = 1, V_lo empty)
struct EigFrame {
    int n_s = 0, n_hi = 0, n_lo = 1;
    DevBuf V_hi, V_lo;            // FP64 complex, row-major, column j = eigenvector j
    DevBuf VH_hi;                 // V_hi^H (Kronecker plans: the rows of the high-axis GEMM of V^H)
    DevBuf lam_dev;               // the eigenvalues on the device (FP64)
    std::vector<double> lam;      // ascending for dense; mu_p + nu_q (p major) for Kronecker
    const double *Vr = nullptr;   // a caller's real orthogonal V (device, row-major, borrowed):
                                  // the basis change then runs as two FP64 GEMVs over it
};

sv_status check_hermitian(const double *A, int N, const char *name);
bool is_tridiagonal(const double *A, int N);
sv_status eigh_device(sv_state s, const double *A, int N, DevBuf &dV, std::vector<double> &lam);
sv_status eigh_device_batched(sv_state s, const std::vector<const double *> &As, int N, std::vector<DevBuf *> &dVs,
                              std::vector<std::vector<double>> &lams);
void turn_table(const std::vector<double> &lam, double T0, int n_c, std::vector<uint64_t> &F);
void inversion_table(int n_c, std::vector<double> &cs, bool sgn = false, uint64_t gcut = 0);
sv_status kron_apply(hipStream_t st, double2 *out, const double2 *in, double2 *tmp, const double2 *V_hi, int n_hi,
                     const double2 *V_lo, int n_lo, int adjoint);
const char *eigh_last_solver();

// fixed-order sum of `count` partials spaced `stride` apart into out[0]
static __global__ __launch_bounds__(256) void k_sum_partials_strided(const double *__restrict__ part, int count,
                                                                     int stride, double *__restrict__ out) {
    __shared__ double ws[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) acc += part[(size_t)i * stride];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// first level of a two-level fixed-order sum: block b sums the strided
// entries [b*chunk, (b+1)*chunk) of `part` into tmp[b]
static __global__ __launch_bounds__(256) void k_sum_chunks(const double *__restrict__ part, uint64_t count,
                                                           int stride, uint64_t chunk, double *__restrict__ tmp) {
    __shared__ double ws[4];
    const uint64_t beg = (uint64_t)blockIdx.x * chunk;
    const uint64_t end = beg + chunk < count ? beg + chunk : count;
    double acc = 0.0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += blockDim.x) acc += part[i * stride];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) tmp[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// out[0] = sum of count strided partials, fixed order; tmp holds >= 256 doubles
static inline void sum_partials(hipStream_t st, const double *part, uint64_t count, int stride, double *tmp,
                                double *out) {
    uint64_t nb = (count + 4095) / 4096;
    if (nb > 256) nb = 256;
    if (nb < 1) nb = 1;
    const uint64_t chunk = (count + nb - 1) / nb;
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)nb), dim3(256), 0, st, part, count, stride, chunk, tmp);
    hipLaunchKernelGGL(k_sum_partials_strided, dim3(1), dim3(256), 0, st, (const double *)tmp, (int)nb, 1, out);
}

}  // namespace sv
