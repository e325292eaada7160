// Batched T0 sweep: many HHL instances of uneven size (each with its own
// grid of T0 values) solved by the fused eigen-frame kernels, recorded once
// as a hipGraph and replayed.
//
// Per instance (classical preprocessing, once): FP64 eigen-decomposition,
// beta = V^H b^, and the eigen-basis coefficients of the exact solution
// A^{-1} b (beta_j / lambda_j, normalised) for the fidelity.
// Per solve (instance, T0), inside the graph:
//   turn tables (all solves, one kernel; it also clears the queue counters)
//   -> the three pipeline kernels' tiles and the finish, in one of two forms:
//      * work queues: one persistent kernel; the solves are spread over one
//        queue per XCC, each item a run of tiles of one phase of one solve,
//        ordered by a done counter per solve and phase
//      * side streams: per (n_s, n_c) class the three pipeline kernels with
//        blockIdx.z = solve, the classes over four streams (parallel branches
//        of the graph) so that small classes overlap instead of each paying
//        its launch latency in series, then one finishing kernel
//      prepare times both and keeps the faster (or the one SV_BATCH_QUEUE
//      names)
//   the finish: FP64 sums of P(a=1) and the norm, the post-selected
//   eigen-coefficients z_j (column sums of the clock projection),
//   p_post = |z|^2 and F = |<x_C|x_Q>| = |sum conj(c_j) z_j| / |z|, all in
//   FP64, fixed summation order.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "sv_device.h"
#include "sv_hhl_internal.h"
#include "sv_internal.h"

namespace sv {

struct TurnJob {
    const double *lam;
    uint64_t *F;
    double T0;
    int n_c;
    uint64_t N;
};

// all turn tables of the batch (blockIdx.y = solve); also clears the work
// queue's counters for the launch that follows
__global__ void k_turn_batch(const TurnJob *__restrict__ jobs, unsigned *__restrict__ cnt, uint64_t ncnt) {
    for (uint64_t i = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x; i < ncnt;
         i += (uint64_t)gridDim.x * gridDim.y * blockDim.x)
        cnt[i] = 0u;
    const TurnJob J = jobs[blockIdx.y];
    const uint64_t total = J.N * (uint64_t)J.n_c;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = i / J.n_c;
        const int k = (int)(i % J.n_c);
        const double phi = J.lam[j] * J.T0 / (2.0 * M_PI);
        const double x = ldexp(phi, k);
        const double f = x - floor(x);
        const double sc = ldexp(f, 64);
        J.F[i] = sc >= 18446744073709551616.0 ? 0ull : (uint64_t)sc;
    }
}

// the finish of every solve, one block each (the stream path)
__global__ __launch_bounds__(256) void k_batch_finish(const FinishJob *__restrict__ jobs) {
    batch_finish_body(jobs[blockIdx.x]);
}

}  // namespace sv

using namespace sv;

struct sv_batch_s {
    sv_dtype dt = SV_C64;
    hipStream_t stream = nullptr;
    sv_state_s ctx;                       // staging buffers for uploads (no amplitudes)
    int n_solves = 0;
    std::vector<DevBuf *> bufs;           // every device allocation of the batch
    DevBuf *arena = nullptr;              // states, tables, partials
    DevBuf *desc = nullptr;               // descriptor arrays
    const TurnJob *d_turn = nullptr;
    const FinishJob *d_finish = nullptr;     // the finish jobs of the stream form
    const FinishJob *d_finish_q = nullptr;   // the same for the work-queue form (its own partial counts)
    double *d_out = nullptr;
    struct Class {
        int n_s, n_c, cl[3], nt[3];
        const PipeSolve *d_solves;
        int count;
        uint64_t nparts;      // k_pipe_b partial pairs per solve, as laid out for the finish
    };
    std::vector<Class> classes;
    // the launch form: every solve in one persistent kernel over per-XCC
    // work queues, or the classes' kernels on side streams; chosen by timing
    // both at prepare unless SV_BATCH_QUEUE is 1 or 0
    bool use_queue = true;
    bool have_queue = false;
    float form_ms[2] = {0.f, 0.f};           // timed graph replays: streams, queue (0: not timed)
    PipeQueue queue;
    DevBuf qdesc;
    unsigned *d_cnt = nullptr;            // queue counters (cleared by the turn-table kernel)
    uint64_t n_cnt = 0;
    unsigned *d_flag = nullptr;           // set if a queue wait expired
    // the classes are independent: they run on kSide streams forked after the
    // turn tables and joined before the finish (in the graph: parallel branches)
    static constexpr int kSide = 4;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {};
    std::vector<int> lane[kSide];          // class indices per side stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t own_stream = nullptr;
    ~sv_batch_s() {
        // a replayed graph with side-stream branches kept the batch's memory
        // from being released unless the device was idle when the graph and
        // then the buffers went (prepare/replay/free loops lost one arena per
        // batch otherwise)
        hipDeviceSynchronize();
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        hipDeviceSynchronize();
        for (int i = 0; i < kSide; ++i) {
            if (join[i]) hipEventDestroy(join[i]);
            if (side[i]) hipStreamDestroy(side[i]);
        }
        if (fork) hipEventDestroy(fork);
        if (own_stream) hipStreamDestroy(own_stream);
        for (auto *b : bufs) delete b;
        if (ctx.pinned) hipHostFree(ctx.pinned);
        if (ctx.small) hipFree(ctx.small);
        if (ctx.scratch) hipFree(ctx.scratch);
    }
};

namespace sv {

template <typename R>
static sv_status enqueue_batch(sv_batch b) {
    const hipStream_t st = b->stream;
    hipLaunchKernelGGL(k_turn_batch, dim3(64, b->n_solves), dim3(256), 0, st, b->d_turn, b->d_cnt, b->n_cnt);
    SV_HIP(hipGetLastError());
    if (b->use_queue) return pipe_queue_launch<R>(st, b->queue, b->d_finish_q);
    SV_HIP(hipEventRecord(b->fork, st));
    for (int i = 0; i < sv_batch_s::kSide; ++i) {
        if (b->lane[i].empty()) continue;
        SV_HIP(hipStreamWaitEvent(b->side[i], b->fork, 0));
        for (int ci : b->lane[i]) {
            const auto &c = b->classes[ci];
            uint64_t np = 0;
            SV_TRY(pipe_run_batch<R>(b->side[i], c.n_s, c.n_c, c.cl, c.nt, c.d_solves, c.count, &np));
            if (np != c.nparts) return fail(SV_EDEVICE, "partial count %llu != %llu", (unsigned long long)np,
                                            (unsigned long long)c.nparts);
        }
        SV_HIP(hipEventRecord(b->join[i], b->side[i]));
        SV_HIP(hipStreamWaitEvent(st, b->join[i], 0));
    }
    hipLaunchKernelGGL(k_batch_finish, dim3(b->n_solves), dim3(256), 0, st, b->d_finish);
    SV_HIP(hipGetLastError());
    return SV_OK;
}

}  // namespace sv

extern "C" {

sv_status sv_batch_prepare(sv_batch *out, sv_dtype dt, void *hip_stream, const sv_batch_instance *inst, int n_inst) {
    clear_error();
    if (!out) return fail(SV_EINVAL, "out is NULL");
    *out = nullptr;
    if (!inst || n_inst < 1) return fail(SV_EINVAL, "no instances");
    if (dt != SV_C64 && dt != SV_C128) return fail(SV_EINVAL, "bad dtype");
    const size_t e = amp_bytes(dt);
    // validate
    int total = 0;
    for (int i = 0; i < n_inst; ++i) {
        const sv_batch_instance &I = inst[i];
        if (!I.A || !I.b || !I.t0 || I.n_t0 < 1) return fail(SV_EINVAL, "instance %d: missing data", i);
        if (I.n_s < 1 || I.n_s > 13 || !pipe_supported(I.n_s, I.n_c) || I.n_s + I.n_c + 1 > 32)
            return fail(SV_EUNSUPPORTED, "instance %d: n_s %d, n_c %d outside the batched path", i, I.n_s, I.n_c);
        for (int t = 0; t < I.n_t0; ++t)
            if (!(I.t0[t] > 0.0) || !isfinite(I.t0[t])) return fail(SV_EINVAL, "instance %d: T0 must be > 0", i);
        total += I.n_t0;
    }
    if (total > 65535) return fail(SV_EUNSUPPORTED, "more than 65535 solves in one batch");
    sv_batch b = new sv_batch_s();
    b->dt = dt;
    b->stream = (hipStream_t)hip_stream;
    if (!b->stream) {   // graphs are captured from a stream of our own, not the null stream
        hipError_t he = hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking);
        if (he != hipSuccess) {
            delete b;
            return hip_fail(he, "hipStreamCreateWithFlags");
        }
        b->stream = b->own_stream;
    }
    b->ctx.stream = b->stream;
    b->ctx.dt = dt;
    b->n_solves = total;
    hipGetDevice(&b->ctx.device);
    auto fail_del = [&](sv_status s) {
        delete b;
        return s;
    };
    // --- eigen-decompositions: dense real symmetric instances of one size in
    // one batched call, the others one at a time
    std::vector<DevBuf *> V(n_inst), lamd(n_inst), beta(n_inst), cex(n_inst);
    std::vector<std::vector<double>> lams(n_inst);
    std::map<int, std::vector<int>> real_by_n;
    for (int i = 0; i < n_inst; ++i) {
        const sv_batch_instance &I = inst[i];
        const int N = 1 << I.n_s;
        sv_status st = check_hermitian(I.A, N, "A");
        if (st != SV_OK) return fail_del(st);
        V[i] = new DevBuf();
        lamd[i] = new DevBuf();
        beta[i] = new DevBuf();
        cex[i] = new DevBuf();
        b->bufs.push_back(V[i]);
        b->bufs.push_back(lamd[i]);
        b->bufs.push_back(beta[i]);
        b->bufs.push_back(cex[i]);
        bool real = true;
        for (size_t k = 0; k < (size_t)N * N && real; ++k) real = I.A[2 * k + 1] == 0.0;
        // dense real instances of one size share a strided-batched solve;
        // tridiagonal ones (and complex ones) go one at a time, the
        // tridiagonal ones to the tridiagonal divide and conquer
        if (real && N > 1 && !is_tridiagonal(I.A, N)) {
            real_by_n[N].push_back(i);
        } else {
            st = eigh_device(&b->ctx, I.A, N, *V[i], lams[i]);
            if (st != SV_OK) return fail_del(st);
        }
    }
    for (auto &kv : real_by_n) {
        std::vector<const double *> As;
        std::vector<DevBuf *> dVs;
        std::vector<std::vector<double>> ls;
        for (int i : kv.second) {
            As.push_back(inst[i].A);
            dVs.push_back(V[i]);
        }
        sv_status st = eigh_device_batched(&b->ctx, As, kv.first, dVs, ls);
        if (st != SV_OK) return fail_del(st);
        for (size_t q = 0; q < kv.second.size(); ++q) lams[kv.second[q]] = std::move(ls[q]);
    }
    // --- per instance: beta = V^H b^ and the exact-solution coefficients
    for (int i = 0; i < n_inst; ++i) {
        const sv_batch_instance &I = inst[i];
        const int N = 1 << I.n_s;
        sv_status st = SV_OK;
        const std::vector<double> &lam = lams[i];
        if (!(lam[0] > 0.0)) return fail_del(fail(SV_ENOTPOSDEF, "instance %d: lambda_min <= 0", i));
        double nb = 0.0;
        for (int j = 0; j < 2 * N; ++j) nb += I.b[j] * I.b[j];
        nb = sqrt(nb);
        if (!(nb > 0.0)) return fail_del(fail(SV_EZERONORM, "instance %d: |b| = 0", i));
        std::vector<double> bh(2 * (size_t)N);
        for (int j = 0; j < 2 * N; ++j) bh[j] = I.b[j] / nb;
        DevBuf tmp, bdev;
        if ((st = tmp.alloc(N * sizeof(double2))) != SV_OK || (st = bdev.alloc(N * sizeof(double2))) != SV_OK ||
            (st = beta[i]->alloc(N * sizeof(double2))) != SV_OK || (st = lamd[i]->alloc(N * sizeof(double))) != SV_OK ||
            (st = cex[i]->alloc(N * sizeof(double2))) != SV_OK)
            return fail_del(st);
        if ((st = upload(&b->ctx, bdev.p, bh.data(), bh.size() * sizeof(double))) != SV_OK) return fail_del(st);
        if ((st = upload(&b->ctx, lamd[i]->p, lam.data(), N * sizeof(double))) != SV_OK) return fail_del(st);
        if ((st = kron_apply(b->stream, (double2 *)beta[i]->p, (const double2 *)bdev.p, (double2 *)tmp.p,
                             (const double2 *)V[i]->p, N, nullptr, 1, 1)) != SV_OK)
            return fail_del(st);
        std::vector<double> bt(2 * (size_t)N);
        if ((st = download(&b->ctx, bt.data(), beta[i]->p, bt.size() * sizeof(double))) != SV_OK) return fail_del(st);
        double cn = 0.0;
        for (int j = 0; j < N; ++j) {
            bt[2 * j] /= lam[j];
            bt[2 * j + 1] /= lam[j];
            cn += bt[2 * j] * bt[2 * j] + bt[2 * j + 1] * bt[2 * j + 1];
        }
        cn = sqrt(cn);
        for (auto &v : bt) v /= cn;
        if ((st = upload(&b->ctx, cex[i]->p, bt.data(), bt.size() * sizeof(double))) != SV_OK) return fail_del(st);
    }
    // --- arena layout: per solve state, F, part, zpart, out
    struct SolveLay {
        int inst, t;
        size_t psi, F, part, zpart;
        uint64_t nparts_max;
    };
    std::vector<SolveLay> lay;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        size_t o = off;
        off += bytes;
        return o;
    };
    for (int i = 0; i < n_inst; ++i) {
        const sv_batch_instance &I = inst[i];
        const uint64_t N = dim_of(I.n_s);
        for (int t = 0; t < I.n_t0; ++t) {
            SolveLay L;
            L.inst = i;
            L.t = t;
            L.psi = take(dim_of(I.n_s + I.n_c + 1) * e);
            L.F = take(N * I.n_c * sizeof(uint64_t));
            L.nparts_max = pipe_b_blocks(I.n_s, I.n_c, e);
            L.part = take(2 * L.nparts_max * sizeof(double));
            L.zpart = take((size_t)pipe_c_rows(I.n_c) * N * sizeof(double2));
            lay.push_back(L);
        }
    }
    const size_t out_off = take((size_t)total * 4 * sizeof(double));
    const uint64_t n_cnt = pipe_queue_counters(total);
    const size_t cnt_off = take(n_cnt * sizeof(unsigned));
    const size_t flag_off = take(sizeof(unsigned));
    b->arena = new DevBuf();
    b->bufs.push_back(b->arena);
    sv_status st = b->arena->alloc(off);
    if (st != SV_OK) return fail_del(st);
    char *base = (char *)b->arena->p;
    b->d_out = (double *)(base + out_off);
    b->d_cnt = (unsigned *)(base + cnt_off);
    b->n_cnt = n_cnt;
    b->d_flag = (unsigned *)(base + flag_off);
    {
        const hipError_t me = hipMemsetAsync(b->d_flag, 0, sizeof(unsigned), b->stream);
        if (me != hipSuccess) return fail_del(hip_fail(me, "hipMemsetAsync"));
    }
    int form = -1;     // -1: time both
    {
        const char *qe = getenv("SV_BATCH_QUEUE");
        if (qe && *qe) form = atoi(qe) != 0 ? 1 : 0;
    }
    // --- classes by (n_s, n_c)
    std::map<std::pair<int, int>, std::vector<int>> cls;
    for (int k = 0; k < total; ++k) cls[{inst[lay[k].inst].n_s, inst[lay[k].inst].n_c}].push_back(k);
    // host descriptors
    std::vector<TurnJob> turn(total);
    std::vector<FinishJob> fin(total);
    std::vector<PipeSolve> solves;
    for (int k = 0; k < total; ++k) {
        const SolveLay &L = lay[k];
        const sv_batch_instance &I = inst[L.inst];
        turn[k] = TurnJob{(const double *)lamd[L.inst]->p, (uint64_t *)(base + L.F), I.t0[L.t], I.n_c,
                          dim_of(I.n_s)};
    }
    std::vector<std::pair<int, int>> class_keys;
    std::vector<std::vector<int>> class_members;
    for (auto &kv : cls) {
        class_keys.push_back(kv.first);
        class_members.push_back(kv.second);
    }
    // descriptor arena: turn jobs, finish jobs, per-class solve arrays
    b->desc = new DevBuf();
    b->bufs.push_back(b->desc);
    const size_t dbytes = total * (sizeof(TurnJob) + 2 * sizeof(FinishJob) + sizeof(PipeSolve)) + 4096;
    if ((st = b->desc->alloc(dbytes)) != SV_OK) return fail_del(st);
    char *dbase = (char *)b->desc->p;
    b->d_turn = (const TurnJob *)dbase;
    b->d_finish = (const FinishJob *)(dbase + ((total * sizeof(TurnJob) + 255) & ~(size_t)255));
    b->d_finish_q = (const FinishJob *)((const char *)b->d_finish + ((total * sizeof(FinishJob) + 255) & ~(size_t)255));
    char *dsol = (char *)b->d_finish_q + ((total * sizeof(FinishJob) + 255) & ~(size_t)255);
    if ((st = upload(&b->ctx, (void *)b->d_turn, turn.data(), total * sizeof(TurnJob))) != SV_OK) return fail_del(st);
    hipLaunchKernelGGL(k_turn_batch, dim3(64, total), dim3(256), 0, b->stream, b->d_turn, b->d_cnt, b->n_cnt);
    {
        const hipError_t ke = hipGetLastError();
        if (ke != hipSuccess) return fail_del(hip_fail(ke, "k_turn_batch"));
    }
    size_t sol_off = 0;
    std::vector<QueueClassIn> qcls;
    std::vector<int> qsolve_cls(total, 0);
    std::vector<PipeSolve> qsolves(total);
    for (size_t c = 0; c < class_keys.size(); ++c) {
        const int n_s = class_keys[c].first, n_c = class_keys[c].second;
        std::vector<PipeSolve> ps;
        for (int k : class_members[c]) {
            const SolveLay &L = lay[k];
            ps.push_back(PipeSolve{base + L.psi, (const double2 *)beta[L.inst]->p, (const uint64_t *)(base + L.F),
                                   (double *)(base + L.part), (double2 *)(base + L.zpart)});
        }
        sv_batch_s::Class C;
        C.n_s = n_s;
        C.n_c = n_c;
        C.count = (int)ps.size();
        C.d_solves = (const PipeSolve *)(dsol + sol_off);
        sol_off += ps.size() * sizeof(PipeSolve);
        if ((st = upload(&b->ctx, (void *)C.d_solves, ps.data(), ps.size() * sizeof(PipeSolve))) != SV_OK)
            return fail_del(st);
        // launch configuration: cached or tuned on the first solve of the class
        st = dt == SV_C64 ? pipe_config<float>(b->stream, n_s, n_c, &ps[0], C.cl, C.nt)
                          : pipe_config<double>(b->stream, n_s, n_c, &ps[0], C.cl, C.nt);
        if (st != SV_OK) return fail_del(st);
        const uint64_t np = pipe_b_blocks_for(n_s, n_c, C.cl[1]);
        if (np > pipe_b_blocks(n_s, n_c, e)) return fail_del(fail(SV_EDEVICE, "partials exceed their buffer"));
        C.nparts = np;
        for (size_t q = 0; q < class_members[c].size(); ++q) {
            const int k = class_members[c][q];
            const SolveLay &L = lay[k];
            const int g1 = (n_c + 1) / 2;
            fin[k] = FinishJob{(const double *)(base + L.part), np, (const double2 *)(base + L.zpart),
                               pipe_c_rows(n_c), dim_of(n_s), exp2(-0.5 * (n_c + g1)),
                               (const double2 *)cex[L.inst]->p, b->d_out + 4 * (size_t)k};
            qsolve_cls[k] = (int)c;
            qsolves[k] = ps[q];
        }
        qcls.push_back(QueueClassIn{n_s, n_c, {C.cl[0], C.cl[1], C.cl[2]}});
        b->classes.push_back(C);
    }
    if ((st = upload(&b->ctx, (void *)b->d_finish, fin.data(), total * sizeof(FinishJob))) != SV_OK)
        return fail_del(st);
    if (form != 0) {
        st = dt == SV_C64 ? pipe_queue_build<float>(&b->ctx, b->stream, b->queue, b->qdesc, qcls, qsolve_cls,
                                                    qsolves, b->d_cnt, b->d_flag)
                          : pipe_queue_build<double>(&b->ctx, b->stream, b->queue, b->qdesc, qcls, qsolve_cls,
                                                     qsolves, b->d_cnt, b->d_flag);
        if (st == SV_OK) {
            b->have_queue = true;
            for (int k = 0; k < total; ++k) fin[k].nparts = b->queue.nparts[k];
            if ((st = upload(&b->ctx, (void *)b->d_finish_q, fin.data(), total * sizeof(FinishJob))) != SV_OK)
                return fail_del(st);
        } else if (form == 1 || st != SV_EUNSUPPORTED) {
            return fail_del(st);
        } else {
            clear_error();      // a shape the queue does not carry: the stream form
        }
    }
    // side streams (default priority) and the fork/join events; classes go to
    // the least-loaded stream, largest first, weighed by amplitudes plus a
    // fixed cost per class for its three launches
    {
        for (int i = 0; i < sv_batch_s::kSide; ++i) {
            hipError_t e1 = hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking);
            if (e1 != hipSuccess) return fail_del(hip_fail(e1, "hipStreamCreateWithFlags"));
            e1 = hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming);
            if (e1 != hipSuccess) return fail_del(hip_fail(e1, "hipEventCreateWithFlags"));
        }
        hipError_t e2 = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e2 != hipSuccess) return fail_del(hip_fail(e2, "hipEventCreateWithFlags"));
        std::vector<int> order(b->classes.size());
        std::vector<double> wgt(b->classes.size());
        for (size_t i = 0; i < order.size(); ++i) {
            const auto &c = b->classes[i];
            order[i] = (int)i;
            wgt[i] = (double)c.count * (double)dim_of(c.n_s + c.n_c) + (double)(1u << 20);
        }
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return wgt[x] > wgt[y]; });
        double load[sv_batch_s::kSide] = {};
        for (int ci : order) {
            int best = 0;
            for (int i = 1; i < sv_batch_s::kSide; ++i)
                if (load[i] < load[best]) best = i;
            b->lane[best].push_back(ci);
            load[best] += wgt[ci];
        }
    }
    // record the whole sweep in a graph, in the given launch form (event
    // tracing is paused while capturing)
    auto capture = [&](bool q, hipGraph_t *g, hipGraphExec_t *ex) -> sv_status {
        b->use_queue = q;
        SV_HIP(hipStreamSynchronize(b->stream));
        const bool tr = trace_set(false);
        hipError_t he = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (he != hipSuccess) {
            trace_set(tr);
            return hip_fail(he, "hipStreamBeginCapture");
        }
        sv_status cs = dt == SV_C64 ? enqueue_batch<float>(b) : enqueue_batch<double>(b);
        he = hipStreamEndCapture(b->stream, g);
        trace_set(tr);
        if (cs != SV_OK) return cs;
        if (he != hipSuccess) return hip_fail(he, "hipStreamEndCapture");
        he = hipGraphInstantiate(ex, *g, nullptr, nullptr, 0);
        if (he != hipSuccess) return hip_fail(he, "hipGraphInstantiate");
        return SV_OK;
    };
    // the launch form: as asked; else the cached choice for this mix of
    // shape classes; else the faster graph replay (both forms captured and
    // replayed alternately, after an untimed replay each; best of three
    // rounds), cached; with tuning off, the side streams
    bool timed = false;
    if (form >= 0 || !b->have_queue) {
        b->use_queue = form != 0 && b->have_queue;
    } else {
        std::string key = std::string("batchform/") + (dt == SV_C64 ? "c64" : "c128");
        for (const auto &c : b->classes)
            key += "/" + std::to_string(c.n_s) + "." + std::to_string(c.n_c) + "x" + std::to_string(c.count);
        std::vector<int> cached;
        if (tune_lookup(key, cached) && cached.size() == 1) {
            b->use_queue = cached[0] == 1;
        } else if (!autotune_enabled()) {
            b->use_queue = false;
        } else {
            timed = true;
            hipGraph_t g[2] = {};
            hipGraphExec_t ex[2] = {};
            for (int f = 0; f < 2 && st == SV_OK; ++f) st = capture(f == 1, &g[f], &ex[f]);
            const bool tr0 = trace_set(false);
            for (int r = 0; r < 3 && st == SV_OK; ++r)
                for (int f = 0; f < 2 && st == SV_OK; ++f) {
                    float ms = 0.f;
                    st = time_stream(b->stream, 2, &ms, [&]() -> sv_status {
                        SV_HIP(hipGraphLaunch(ex[f], b->stream));
                        return SV_OK;
                    });
                    if (st == SV_OK && (r == 0 || ms < b->form_ms[f])) b->form_ms[f] = ms;
                }
            trace_set(tr0);
            const int keep = st == SV_OK && b->form_ms[1] < b->form_ms[0] ? 1 : 0;
            // the replays above must be over before a graph goes (see the
            // destructor)
            hipDeviceSynchronize();
            for (int f = 0; f < 2; ++f) {
                if (f == keep && st == SV_OK) continue;
                if (ex[f]) hipGraphExecDestroy(ex[f]);
                if (g[f]) hipGraphDestroy(g[f]);
            }
            if (st != SV_OK) return fail_del(st);
            b->use_queue = keep == 1;
            b->graph = g[keep];
            b->exec = ex[keep];
            tune_store(key, {keep});
        }
    }
    if (!timed) {
        st = capture(b->use_queue, &b->graph, &b->exec);
        if (st != SV_OK) return fail_del(st);
    }
    *out = b;
    return SV_OK;
}

sv_status sv_batch_run(sv_batch b, int use_graph, double *results) {
    clear_error();
    if (!b) return fail(SV_EINVAL, "null batch");
    if (use_graph) {
        SV_HIP(hipGraphLaunch(b->exec, b->stream));
    } else {
        SV_TRY(b->dt == SV_C64 ? enqueue_batch<float>(b) : enqueue_batch<double>(b));
    }
    if (results) {
        SV_TRY(download(&b->ctx, results, b->d_out, (size_t)b->n_solves * 4 * sizeof(double)));
        // a wait of the work queue that expired (this run or an earlier one
        // without results) leaves the flag set: the results are not trusted
        if (b->use_queue) {
            unsigned flag = 0, finished = 0;
            SV_TRY(download(&b->ctx, &flag, b->d_flag, sizeof(unsigned)));
            SV_TRY(download(&b->ctx, &finished, b->d_cnt + b->n_cnt - 1, sizeof(unsigned)));
            if (flag) return fail(SV_EDEVICE, "a work-queue dependency wait expired; the results are invalid");
            if (finished != (unsigned)b->n_solves)
                return fail(SV_EDEVICE, "the work queues finished %u of %d solves", finished, b->n_solves);
        }
    } else {
        SV_HIP(hipStreamSynchronize(b->stream));
    }
    return SV_OK;
}

int sv_batch_num_solves(sv_batch b) { return b ? b->n_solves : 0; }

int sv_batch_form(sv_batch b, float *ms_streams, float *ms_queue) {
    if (!b) return -1;
    if (ms_streams) *ms_streams = b->form_ms[0];
    if (ms_queue) *ms_queue = b->form_ms[1];
    return b->use_queue ? 1 : 0;
}

sv_status sv_batch_free(sv_batch b) {
    if (b) {
        hipStreamSynchronize(b->stream);
        delete b;
    }
    return SV_OK;
}

sv_status sv_hhl_batch(sv_dtype dt, void *hip_stream, const sv_batch_instance *inst, int n_inst, double *results) {
    sv_batch b = nullptr;
    SV_TRY(sv_batch_prepare(&b, dt, hip_stream, inst, n_inst));
    sv_status st = sv_batch_run(b, 1, results);
    sv_batch_free(b);
    return st;
}

}  // extern "C"
