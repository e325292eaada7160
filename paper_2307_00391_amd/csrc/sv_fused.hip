// LDS-fused passes: a circuit is cut into passes; each pass stages tiles of
// 2^k amplitudes (k "local" qubits) in LDS, applies every gate it can there
// and writes the tile back, so a run of gates costs one HBM round trip.
//
// Tile layout: the local qubits are the low c bits of the index plus a set
// of higher "gathered" bits.  The low bits keep HBM accesses contiguous
// (2^c amplitudes per segment); the gathered bits are the targets the pass
// needs.  All other bits are fixed per tile (the tile id is deposited into
// them), so controls and phases on them are uniform over a workgroup.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

constexpr int FUSE_BLOCK = 256;
constexpr int MAX_HI = 20;

enum OpType { OP_U = 0, OP_X = 1, OP_SWAP = 2, OP_PHASE = 3 };

struct FOp {
    int type;
    int p0, p1;            // tile positions of the target(s)
    int pad;
    uint64_t lmask, lval;  // condition on local bits (tile coordinates)
    uint64_t gmask, gval;  // condition on non-local bits (global coordinates)
    uint64_t turns;        // OP_PHASE: phase as a fraction of a turn, 2^-64 units
    double u[8];           // OP_U
};

struct FPass {
    uint64_t nl_mask;      // non-local, non-fixed bits (the tile id is deposited here)
    uint64_t fix_val;      // fixed non-local bits
    int k, c, r;           // local count, low contiguous bits, gathered high bits
    int nops, op_off;
    int hpos[MAX_HI];      // global positions of the gathered bits, ascending
};

// global offset of tile coordinate t
__device__ __forceinline__ uint64_t scatter_t(uint32_t t, int c, int r, const int *__restrict__ hpos) {
    uint64_t g = t & ((1u << c) - 1u);
    uint32_t h = t >> c;
    for (int i = 0; i < r; ++i)
        if (h >> i & 1u) g |= 1ull << hpos[i];
    return g;
}

__device__ __forceinline__ uint32_t insert0(uint32_t p, int pos) {
    return ((p >> pos) << (pos + 1)) | (p & ((1u << pos) - 1u));
}

template <typename R>
__global__ __launch_bounds__(FUSE_BLOCK) void k_fused(cvec<R> *__restrict__ psi, const FPass *__restrict__ passes,
                                                       int pi, const FOp *__restrict__ ops) {
    extern __shared__ unsigned char smem_raw[];
    cvec<R> *tile = reinterpret_cast<cvec<R> *>(smem_raw);
    const FPass &P = passes[pi];
    const int k = P.k, c = P.c, r = P.r;
    const uint32_t T = 1u << k;
    const uint64_t tid = (uint64_t)blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
    const uint64_t base = pdep64(tid, P.nl_mask) | P.fix_val;
    const int *hpos = P.hpos;

    for (uint32_t t = threadIdx.x; t < T; t += FUSE_BLOCK) tile[t] = psi[base | scatter_t(t, c, r, hpos)];
    __syncthreads();

    const FOp *op0 = ops + P.op_off;
    int o = 0;
    while (o < P.nops) {
        const int type = op0[o].type;
        if (type == OP_PHASE) {
            int e = o;
            while (e < P.nops && op0[e].type == OP_PHASE) ++e;
            for (uint32_t t = threadIdx.x; t < T; t += FUSE_BLOCK) {
                uint64_t acc = 0;
                for (int q = o; q < e; ++q) {
                    const FOp &f = op0[q];
                    if ((base & f.gmask) == f.gval && (t & f.lmask) == f.lval) acc += f.turns;
                }
                if (acc) tile[t] = cmul<R>(tile[t], turn_phase<R>(acc));
            }
            o = e;
        } else {
            const FOp &f = op0[o];
            if ((base & f.gmask) == f.gval) {
                if (type == OP_SWAP) {
                    // elements with bit p0 = 1, p1 = 0 exchange with their mirror
                    const int lo_p = f.p0 < f.p1 ? f.p0 : f.p1, hi_p = f.p0 < f.p1 ? f.p1 : f.p0;
                    const uint32_t flip = (1u << f.p0) | (1u << f.p1);
                    for (uint32_t p = threadIdx.x; p < T / 4; p += FUSE_BLOCK) {
                        uint32_t t = insert0(insert0(p, lo_p), hi_p) | (1u << f.p0);
                        if ((t & f.lmask) != f.lval) continue;
                        const uint32_t u = t ^ flip;
                        const cvec<R> a = tile[t], b = tile[u];
                        tile[t] = b;
                        tile[u] = a;
                    }
                } else {
                    const cvec<R> u00 = cmake<R>((R)f.u[0], (R)f.u[1]), u01 = cmake<R>((R)f.u[2], (R)f.u[3]);
                    const cvec<R> u10 = cmake<R>((R)f.u[4], (R)f.u[5]), u11 = cmake<R>((R)f.u[6], (R)f.u[7]);
                    const uint32_t tb = 1u << f.p0;
                    for (uint32_t p = threadIdx.x; p < T / 2; p += FUSE_BLOCK) {
                        const uint32_t t0 = insert0(p, f.p0);
                        if ((t0 & f.lmask) != f.lval) continue;
                        const cvec<R> a0 = tile[t0], a1 = tile[t0 | tb];
                        if (type == OP_X) {
                            tile[t0] = a1;
                            tile[t0 | tb] = a0;
                        } else {
                            tile[t0] = cmac2<R>(u00, a0, u01, a1);
                            tile[t0 | tb] = cmac2<R>(u10, a0, u11, a1);
                        }
                    }
                }
            }
            ++o;
        }
        __syncthreads();
    }

    for (uint32_t t = threadIdx.x; t < T; t += FUSE_BLOCK) psi[base | scatter_t(t, c, r, hpos)] = tile[t];
}

// One group of the QFT cascade on the register [lo, lo+m): local qubits are
// the low c bits and the r register bits starting at global position gpos0
// (register-relative j0).  Each register qubit j of the group gets a
// Hadamard fused with all controlled phases whose target is j:
//   forward cascade (QFT without swaps): for j = j0+r-1 .. j0,
//     H(j), then phase 2 pi (v mod 2^j) / 2^(j+1) on bit j = 1
//   inverse cascade: for j = j0 .. j0+r-1, conjugate phase first, then H(j)
// where v is the register value of the amplitude.  Phases are accumulated
// as exact 64-bit fractions of a turn.
struct QftPassArgs {
    uint64_t nl_mask, fix_val;
    int k, c, gpos0, r;     // local = [0,c) U [gpos0, gpos0 + r)   (r = 0: local = [0,c))
    int lo, j0, jn;          // register base and the register bits of this group: [j0, j0 + jn)
    int tpos0;               // tile position of register bit j0
    int inverse;
};

template <typename R>
__global__ __launch_bounds__(FUSE_BLOCK) void k_qft_pass(cvec<R> *__restrict__ psi, QftPassArgs A) {
    extern __shared__ unsigned char smem_raw[];
    cvec<R> *tile = reinterpret_cast<cvec<R> *>(smem_raw);
    const uint32_t T = 1u << A.k;
    const uint64_t tid = (uint64_t)blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
    const uint64_t base = pdep64(tid, A.nl_mask) | A.fix_val;
    const uint64_t cm = (1ull << A.c) - 1ull;
    auto gidx = [&](uint32_t t) -> uint64_t {
        return base | ((uint64_t)t & cm) | (A.r ? ((uint64_t)(t >> A.c) << A.gpos0) : 0ull);
    };
    for (uint32_t t = threadIdx.x; t < T; t += FUSE_BLOCK) tile[t] = psi[gidx(t)];
    __syncthreads();

    const R h = (R)0.70710678118654752440;
    for (int s = 0; s < A.jn; ++s) {
        const int jr = A.inverse ? s : A.jn - 1 - s;       // position inside the group
        const int j = A.j0 + jr;                            // register-relative qubit
        const int pos = A.tpos0 + jr;                       // tile position
        const uint32_t tb = 1u << pos;
        const uint64_t lowmask = (1ull << j) - 1ull;
        for (uint32_t p = threadIdx.x; p < T / 2; p += FUSE_BLOCK) {
            const uint32_t t0 = insert0(p, pos);
            cvec<R> a0 = tile[t0], a1 = tile[t0 | tb];
            const uint64_t vlow = (gidx(t0) >> A.lo) & lowmask;
            const uint64_t turns = j ? (vlow << (63 - j)) : 0ull;
            if (A.inverse) {
                if (turns) a1 = cmul<R>(a1, turn_phase<R>(0ull - turns));
                tile[t0] = cmake<R>((a0.x + a1.x) * h, (a0.y + a1.y) * h);
                tile[t0 | tb] = cmake<R>((a0.x - a1.x) * h, (a0.y - a1.y) * h);
            } else {
                cvec<R> b1 = cmake<R>((a0.x - a1.x) * h, (a0.y - a1.y) * h);
                if (turns) b1 = cmul<R>(b1, turn_phase<R>(turns));
                tile[t0] = cmake<R>((a0.x + a1.x) * h, (a0.y + a1.y) * h);
                tile[t0 | tb] = b1;
            }
        }
        __syncthreads();
    }
    for (uint32_t t = threadIdx.x; t < T; t += FUSE_BLOCK) psi[gidx(t)] = tile[t];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static int g_lds_limit = 0;

static int lds_limit_bytes() {
    if (g_lds_limit) return g_lds_limit;
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    int lim = 65536;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.sharedMemPerBlock > 0)
        lim = (int)prop.sharedMemPerBlock;
    if (lim > 147456) lim = 147456;   // the largest power-of-two tile (128 KiB) plus headroom
    bool ok = hipFuncSetAttribute((const void *)k_fused<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) ==
              hipSuccess;
    ok &= hipFuncSetAttribute((const void *)k_fused<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) ==
          hipSuccess;
    ok &= hipFuncSetAttribute((const void *)k_qft_pass<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) ==
          hipSuccess;
    ok &= hipFuncSetAttribute((const void *)k_qft_pass<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) ==
          hipSuccess;
    (void)hipGetLastError();
    if (!ok) lim = 65536;
    g_lds_limit = lim;
    return lim;
}

static int low_bits_for(sv_dtype dt) { return dt == SV_C128 ? 3 : 4; }   // 128-byte segments

static int clamp_k(sv_state s, int max_local) {
    int k = max_local > 0 ? max_local : default_max_local(s->dt);
    const int bytes = (int)amp_bytes(s->dt);
    while (k > 1 && (1 << k) * bytes > lds_limit_bytes()) --k;
    if (k > s->n) k = s->n;
    return k;
}

static inline dim3 tile_grid(uint64_t tiles) {
    if (tiles <= 0x7fffffffull) return dim3((unsigned)tiles);
    return dim3(1u << 30, (unsigned)(tiles >> 30));
}

struct PGate {
    int kind;          // 0 dense U, 1 X, 2 SWAP, 3 diagonal (phases)
    int t0, t1;
    uint64_t cmask, cval;
    uint64_t qubits;   // all qubits touched (targets + controls)
    uint64_t need;     // qubits that must be local
    double u[8];
};

static bool unit_modulus(double re, double im) { return fabs(re * re + im * im - 1.0) < 1e-13; }

static uint64_t angle_turns(double re, double im) {
    // arg(re + i im) as a fraction of a turn in [-1/2, 1/2), rounded to 2^-64
    long double a = atan2l((long double)im, (long double)re) / (2.0L * 3.14159265358979323846264338327950288L);
    if (a >= 0.5L) a -= 1.0L;
    return (uint64_t)(int64_t)llroundl(ldexpl(a, 64));
}

static sv_status to_pgates(sv_state s, const sv_gate *gates, int n_gates, std::vector<PGate> &out) {
    out.clear();
    out.reserve(n_gates);
    for (int i = 0; i < n_gates; ++i) {
        const sv_gate &g = gates[i];
        PGate p;
        memset(&p, 0, sizeof p);
        if (g.n_ctrls < 0 || g.n_ctrls > SV_MAX_CTRLS) return fail(SV_EINVAL, "gate %d: n_ctrls out of range", i);
        int qs[2] = {g.target, g.target2};
        int nq = g.kind == SV_GATE_SWAP ? 2 : 1;
        if (g.kind != SV_GATE_U && g.kind != SV_GATE_X && g.kind != SV_GATE_SWAP)
            return fail(SV_EINVAL, "gate %d: unknown kind %d", i, g.kind);
        sv_status st = check_qubits(s, qs, nq, g.ctrls, g.ctrl_vals, g.n_ctrls, &p.cmask, &p.cval);
        if (st != SV_OK) return fail(st, "gate %d: %s", i, sv_last_error());
        p.t0 = g.target;
        p.t1 = nq == 2 ? g.target2 : -1;
        p.qubits = p.cmask | (1ull << g.target) | (nq == 2 ? 1ull << g.target2 : 0);
        if (g.kind == SV_GATE_X) {
            p.kind = 1;
            p.need = 1ull << g.target;
        } else if (g.kind == SV_GATE_SWAP) {
            p.kind = 2;
            p.need = (1ull << g.target) | (1ull << g.target2);
        } else {
            memcpy(p.u, g.u, sizeof p.u);
            for (int j = 0; j < 8; ++j)
                if (!isfinite(p.u[j])) return fail(SV_EINVAL, "gate %d: non-finite matrix entry", i);
            const bool diag = p.u[2] == 0 && p.u[3] == 0 && p.u[4] == 0 && p.u[5] == 0 &&
                              unit_modulus(p.u[0], p.u[1]) && unit_modulus(p.u[6], p.u[7]);
            p.kind = diag ? 3 : 0;
            p.need = diag ? 0 : 1ull << g.target;
        }
        out.push_back(p);
    }
    return SV_OK;
}

struct HostPass {
    FPass hdr;
    std::vector<FOp> ops;
};

static int ops_of(const PGate &g) {
    if (g.kind != 3) return 1;
    int c = 0;
    if (!(g.u[0] == 1 && g.u[1] == 0)) ++c;
    if (!(g.u[6] == 1 && g.u[7] == 0)) ++c;
    return c;
}

static void finish_layout(int n, int k, uint64_t L, HostPass &hp) {
    // fill the local set up to k with the lowest free bits
    for (int q = 0; q < n && popcount64(L) < k; ++q) L |= 1ull << q;
    int c = 0;
    while (c < n && (L >> c & 1)) ++c;
    hp.hdr.c = c;
    hp.hdr.k = popcount64(L);
    hp.hdr.r = 0;
    for (int q = c; q < n; ++q)
        if (L >> q & 1) hp.hdr.hpos[hp.hdr.r++] = q;
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    hp.hdr.nl_mask = all & ~L;
    hp.hdr.fix_val = 0;
}

static int tile_pos(uint64_t L, int q) { return popcount64(L & ((1ull << q) - 1ull)); }

static uint64_t to_tile_mask(uint64_t L, uint64_t gm) {
    uint64_t r = 0;
    for (int q = 0; q < 64; ++q)
        if ((gm >> q & 1) && (L >> q & 1)) r |= 1ull << tile_pos(L, q);
    return r;
}

static void emit_ops(const PGate &g, uint64_t L, std::vector<FOp> &ops) {
    FOp f;
    memset(&f, 0, sizeof f);
    const uint64_t lc = g.cmask & L, gc = g.cmask & ~L;
    f.lmask = to_tile_mask(L, lc);
    f.lval = to_tile_mask(L, g.cval & lc);
    f.gmask = gc;
    f.gval = g.cval & gc;
    if (g.kind == 3) {
        // diag(u00, u11): phase on target = 0 and on target = 1 (with the controls)
        const uint64_t tb = 1ull << g.t0;
        for (int b = 0; b < 2; ++b) {
            const double re = g.u[6 * b], im = g.u[6 * b + 1];
            if (re == 1 && im == 0) continue;
            FOp h = f;
            h.type = OP_PHASE;
            if (L & tb) {
                h.lmask |= 1ull << tile_pos(L, g.t0);
                if (b) h.lval |= 1ull << tile_pos(L, g.t0);
            } else {
                h.gmask |= tb;
                if (b) h.gval |= tb;
            }
            h.turns = angle_turns(re, im);
            ops.push_back(h);
        }
        return;
    }
    f.type = g.kind == 0 ? OP_U : g.kind == 1 ? OP_X : OP_SWAP;
    f.p0 = tile_pos(L, g.t0);
    f.p1 = g.kind == 2 ? tile_pos(L, g.t1) : 0;
    memcpy(f.u, g.u, sizeof f.u);
    ops.push_back(f);
}

constexpr int MAX_OPS_PER_PASS = 96;

static void plan(int n, int kmax, int c0, const std::vector<PGate> &gates, std::vector<HostPass> &passes) {
    passes.clear();
    std::vector<char> done(gates.size(), 0);
    size_t left = gates.size();
    const uint64_t low = (1ull << std::min(c0, n)) - 1ull;
    while (left) {
        uint64_t L = low, blocked = 0;
        std::vector<int> take;
        int nops = 0;
        for (size_t i = 0; i < gates.size(); ++i) {
            if (done[i]) continue;
            const PGate &g = gates[i];
            if (g.qubits & blocked) {
                blocked |= g.qubits;
                continue;
            }
            const uint64_t L2 = L | g.need;
            const int no = ops_of(g);
            if (popcount64(L2) <= kmax && nops + no <= MAX_OPS_PER_PASS) {
                L = L2;
                nops += no;
                take.push_back((int)i);
            } else {
                blocked |= g.qubits;
            }
        }
        HostPass hp;
        memset(&hp.hdr, 0, sizeof hp.hdr);
        finish_layout(n, kmax, L, hp);
        uint64_t Lfinal = ~hp.hdr.nl_mask & ((n >= 64) ? ~0ull : ((1ull << n) - 1ull));
        for (int i : take) {
            emit_ops(gates[i], Lfinal, hp.ops);
            done[i] = 1;
            --left;
        }
        if (!hp.ops.empty()) passes.push_back(std::move(hp));
    }
}

template <typename R>
static sv_status launch_passes(sv_state s, std::vector<HostPass> &passes) {
    if (passes.empty()) return SV_OK;
    size_t nops = 0;
    for (auto &p : passes) nops += p.ops.size();
    const size_t hbytes = passes.size() * sizeof(FPass);
    const size_t obytes = std::max<size_t>(nops, 1) * sizeof(FOp);
    std::vector<unsigned char> blob(hbytes + obytes);
    size_t off = 0;
    for (size_t i = 0; i < passes.size(); ++i) {
        passes[i].hdr.nops = (int)passes[i].ops.size();
        passes[i].hdr.op_off = (int)off;
        memcpy(blob.data() + hbytes + off * sizeof(FOp), passes[i].ops.data(), passes[i].ops.size() * sizeof(FOp));
        off += passes[i].ops.size();
        memcpy(blob.data() + i * sizeof(FPass), &passes[i].hdr, sizeof(FPass));
    }
    void *dev = nullptr;
    SV_HIP(hipMallocAsync(&dev, blob.size(), s->stream));
    sv_status st = upload(s, dev, blob.data(), blob.size());
    if (st != SV_OK) {
        hipFreeAsync(dev, s->stream);
        return st;
    }
    const FPass *dp = (const FPass *)dev;
    const FOp *dops = (const FOp *)((unsigned char *)dev + hbytes);
    for (size_t i = 0; i < passes.size(); ++i) {
        const FPass &h = passes[i].hdr;
        const uint64_t tiles = dim_of(s->n - h.k);
        const size_t lds = ((size_t)1 << h.k) * sizeof(cvec<R>);
        {
            TraceScope _ts(s->stream, "fused_pass", 2.0 * (double)dim_of(s->n) * sizeof(cvec<R>), 0.0);
            hipLaunchKernelGGL(k_fused<R>, tile_grid(tiles), dim3(FUSE_BLOCK), lds, s->stream, (cvec<R> *)s->data, dp,
                           (int)i, dops);
        }
    }
    hipError_t e = hipGetLastError();
    hipFreeAsync(dev, s->stream);
    if (e != hipSuccess) return hip_fail(e, "k_fused launch");
    return SV_OK;
}

sv_status run_hadamards(sv_state s, int lo, int m, uint64_t fix_mask, uint64_t fix_val) {
    // a layer of Hadamards restricted to (i & fix_mask) == fix_val, as fused passes
    std::vector<PGate> gs;
    const double h = 0.70710678118654752440;
    for (int j = 0; j < m; ++j) {
        PGate p;
        memset(&p, 0, sizeof p);
        p.kind = 0;
        p.t0 = lo + j;
        p.t1 = -1;
        p.cmask = fix_mask;
        p.cval = fix_val;
        p.qubits = (1ull << (lo + j)) | fix_mask;
        p.need = 1ull << (lo + j);
        const double u[8] = {h, 0, h, 0, h, 0, -h, 0};
        memcpy(p.u, u, sizeof u);
        gs.push_back(p);
    }
    const int k = clamp_k(s, 0);
    std::vector<HostPass> passes;
    plan(s->n, k, std::min(low_bits_for(s->dt), k - 2), gs, passes);
    return s->dt == SV_C64 ? launch_passes<float>(s, passes) : launch_passes<double>(s, passes);
}

template <typename R>
static sv_status qft_cascade_impl(sv_state s, const QftSpec &q, int max_local) {
    const int n = s->n;
    const int kmax = clamp_k(s, max_local);
    const int c0 = std::min(low_bits_for(s->dt), kmax - 1);
    const uint64_t all = (1ull << n) - 1ull;
    // group sizes: as many register bits per pass as fit next to the low bits
    // a register that lies inside the lowest kmax bits is transformed in one pass
    const int gmax = (q.lo + q.m <= kmax) ? q.m : std::max(1, kmax - c0);
    std::vector<std::pair<int, int>> groups;   // (j0, count), in application order
    if (!q.inverse) {
        int top = q.m;
        while (top > 0) {
            int cnt = std::min(gmax, top);
            groups.push_back({top - cnt, cnt});
            top -= cnt;
        }
    } else {
        int bot = 0;
        while (bot < q.m) {
            int cnt = std::min(gmax, q.m - bot);
            groups.push_back({bot, cnt});
            bot += cnt;
        }
    }
    const int nfix = popcount64(q.fix_mask);
    for (auto &gr : groups) {
        QftPassArgs A;
        memset(&A, 0, sizeof A);
        A.lo = q.lo;
        A.j0 = gr.first;
        A.jn = gr.second;
        A.inverse = q.inverse;
        const int gpos0 = q.lo + gr.first;
        // local set: [0, c) U [gpos0, gpos0 + jn) with |local| <= kmax
        int c = std::min(kmax - gr.second, gpos0);
        if (c < 0) c = 0;
        uint64_t L;
        const uint64_t lowm = (1ull << c) - 1ull;
        if ((lowm | (((1ull << gr.second) - 1ull) << gpos0)) & q.fix_mask)
            return fail(SV_EINVAL, "qft: a restricted bit overlaps the pass's local qubits");
        if (c == gpos0) {
            // contiguous: [0, gpos0 + jn)
            A.c = gpos0 + gr.second;
            A.r = 0;
            A.gpos0 = 0;
            A.tpos0 = gpos0;
            L = (1ull << A.c) - 1ull;
        } else {
            A.c = c;
            A.r = gr.second;
            A.gpos0 = gpos0;
            A.tpos0 = c;
            L = ((1ull << c) - 1ull) | (((1ull << gr.second) - 1ull) << gpos0);
        }
        if (L & q.fix_mask) return fail(SV_EINVAL, "qft: restriction bit inside the register");
        A.k = popcount64(L);
        A.nl_mask = all & ~L & ~q.fix_mask;
        A.fix_val = q.fix_val;
        const uint64_t tiles = dim_of(n - A.k - nfix);
        const size_t lds = ((size_t)1 << A.k) * sizeof(cvec<R>);
        {
            TraceScope _ts(s->stream, "qft_pass", 2.0 * (double)dim_of(n - nfix) * sizeof(cvec<R>), 0.0);
            hipLaunchKernelGGL(k_qft_pass<R>, tile_grid(tiles), dim3(FUSE_BLOCK), lds, s->stream, (cvec<R> *)s->data, A);
        }
    }
    SV_HIP(hipGetLastError());
    return SV_OK;
}

sv_status run_qft_cascade(sv_state s, const QftSpec &q, int max_local) {
    if (q.m < 1 || q.lo < 0 || q.lo + q.m > s->n) return fail(SV_EINVAL, "qft register out of range");
    return s->dt == SV_C64 ? qft_cascade_impl<float>(s, q, max_local) : qft_cascade_impl<double>(s, q, max_local);
}

}  // namespace sv

using namespace sv;

extern "C" {

int sv_plan_passes(int n_qubits, sv_dtype dt, const sv_gate *gates, int n_gates, int max_local) {
    sv_state_s tmp;
    tmp.n = n_qubits;
    tmp.dt = dt;
    tmp.data = (void *)1;
    std::vector<PGate> pg;
    if (to_pgates(&tmp, gates, n_gates, pg) != SV_OK) return -1;
    int k = max_local > 0 ? max_local : default_max_local(dt);
    if (k > n_qubits) k = n_qubits;
    std::vector<HostPass> passes;
    plan(n_qubits, k, std::min(low_bits_for(dt), k - 2), pg, passes);
    return (int)passes.size();
}

sv_status sv_apply_circuit(sv_state s, const sv_gate *gates, int n_gates, int max_local) {
    clear_error();
    SV_TRY(check_state(s));
    if (n_gates < 0 || (n_gates && !gates)) return fail(SV_EINVAL, "bad gate list");
    if (!n_gates) return SV_OK;
    std::vector<PGate> pg;
    SV_TRY(to_pgates(s, gates, n_gates, pg));
    const int k = clamp_k(s, max_local);
    if (k < 3) return fail(SV_EUNSUPPORTED, "state too small for fused passes");
    std::vector<HostPass> passes;
    plan(s->n, k, std::max(0, std::min(low_bits_for(s->dt), k - 2)), pg, passes);
    return s->dt == SV_C64 ? launch_passes<float>(s, passes) : launch_passes<double>(s, passes);
}

sv_status sv_qft(sv_state s, int q_lo, int m, int inverse, int swaps, int max_local) {
    clear_error();
    SV_TRY(check_state(s));
    if (m < 1 || q_lo < 0 || q_lo + m > s->n) return fail(SV_EINVAL, "register [%d,%d) outside the state", q_lo, q_lo + m);
    QftSpec q{q_lo, m, inverse ? 1 : 0, 0, 0};
    if (inverse && swaps) SV_TRY(bitrev_register(s, q_lo, m, 0, 0));
    SV_TRY(run_qft_cascade(s, q, max_local));
    if (!inverse && swaps) SV_TRY(bitrev_register(s, q_lo, m, 0, 0));
    return SV_OK;
}

}  // extern "C"
