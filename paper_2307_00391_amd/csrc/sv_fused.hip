// LDS-fused passes: a circuit is cut into passes; each pass stages tiles of
// 2^k amplitudes (k "local" qubits) in LDS, applies every gate it can there
// and writes the tile back, so a run of gates costs one HBM round trip.
//
// Tile layout: the local qubits are the low c bits of the index plus a set
// of higher "gathered" bits.  The low bits keep HBM accesses contiguous
// (2^c amplitudes per segment); the gathered bits are the targets the pass
// needs.  All other bits are fixed per tile (the tile id is deposited into
// them), so controls and phases on them are uniform over a workgroup.
//
// Inside a tile the gates run from registers: the pass's gate list is cut
// into segments whose targets fall in at most RB tile positions S.  For a
// segment every thread holds the 2^RB amplitudes that differ only in S (its
// other tile bits come from the thread index), applies the segment's gates
// without any exchange, and hands the tile back through LDS.  The LDS
// layout is XOR-swizzled so that threads whose amplitudes sit 2^p apart hit
// distinct banks.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
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

// an op as a segment runs it: targets as register bits, its local condition
// split into the register part and the part fixed per thread
struct ROp {
    int type;
    int j0, j1;            // register bits of the target(s)
    uint32_t rmask, rval;  // condition on the register index
    uint32_t tmask, tval;  // condition on the tile bits outside the segment's set
    uint32_t onm;          // bit m set: register index m meets the register condition
    uint64_t gmask, gval;  // condition on non-local bits
    double u[8];           // OP_U matrix; OP_PHASE: (cos, sin) of the phase in u[0], u[1]
};

constexpr int MAX_RB = 5;

struct FSeg {
    int pos[MAX_RB];       // tile positions held in registers (register bit i = pos[i]), ascending
    int nops, op_off;
    // LDS byte offsets (swz of the tile bits times the amplitude size) that
    // register index m is read from and written to.  They differ from the
    // slot of m itself where the segment's register permutations at its
    // start or end (register-controlled NOTs that commute there) were
    // folded into them.
    uint32_t off[1 << MAX_RB];
    uint32_t offw[1 << MAX_RB];
};

struct FPass {
    uint64_t nl_mask;      // non-local, non-fixed bits (the tile id is deposited here)
    uint64_t fix_val;      // fixed non-local bits
    int k, c, r;           // local count, low contiguous bits, gathered high bits
    int nseg, seg_off;
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

// LDS slot of tile coordinate t: the bank index (the low e = log2(256 B /
// elem) bits) is XOR-ed with the folded higher bits.  The segment tables
// are built on the host with the same function.
__host__ __device__ __forceinline__ uint32_t swz_e(uint32_t t, int e) {
    const uint32_t m = (1u << e) - 1u;
    const uint32_t h = t >> e;
    return t ^ ((h ^ (h >> e) ^ (h >> (2 * e))) & m);
}
template <typename R>
__device__ __forceinline__ uint32_t swz(uint32_t t) {
    return swz_e(t, sizeof(cvec<R>) == 8 ? 5 : 4);
}

__device__ __forceinline__ uint32_t pdep32(uint32_t v, uint32_t mask) {
    uint32_t r = 0;
    for (uint32_t b = 1; mask; b <<= 1) {
        const uint32_t low = mask & (0u - mask);
        if (v & b) r |= low;
        mask ^= low;
    }
    return r;
}

template <typename R>
__device__ __forceinline__ cvec<R> csel(bool c, cvec<R> a, cvec<R> b) {
    return cmake<R>(c ? a.x : b.x, c ? a.y : b.y);
}

// The register-bit condition of an op is uniform.  Without one every pair
// is updated (no branches, so the pairs interleave); with one, a uniform
// branch per pair (on the op's precomputed mask of the register indices
// that meet it) skips the pairs it leaves alone.
template <typename R, int RB, int J>
__device__ __forceinline__ void reg_u(cvec<R> (&v)[1 << RB], const ROp &f) {
    const cvec<R> u00 = cmake<R>((R)f.u[0], (R)f.u[1]), u01 = cmake<R>((R)f.u[2], (R)f.u[3]);
    const cvec<R> u10 = cmake<R>((R)f.u[4], (R)f.u[5]), u11 = cmake<R>((R)f.u[6], (R)f.u[7]);
    if (f.rmask == 0) {
#pragma unroll
        for (int m = 0; m < (1 << RB); ++m) {
            if (m & (1 << J)) continue;
            const cvec<R> a0 = v[m], a1 = v[m | (1 << J)];
            v[m] = cmac2<R>(u00, a0, u01, a1);
            v[m | (1 << J)] = cmac2<R>(u10, a0, u11, a1);
        }
    } else {
        const uint32_t on = f.onm;
#pragma unroll
        for (int m = 0; m < (1 << RB); ++m) {
            if (m & (1 << J)) continue;
            if (!(on >> m & 1u)) continue;
            const cvec<R> a0 = v[m], a1 = v[m | (1 << J)];
            v[m] = cmac2<R>(u00, a0, u01, a1);
            v[m | (1 << J)] = cmac2<R>(u10, a0, u11, a1);
        }
    }
}

// A conditional swap in place on the bits, d = (a ^ b) & mask, a ^= d,
// b ^= d: three instructions per pair of words (the AND folds into one
// three-input bit op), where selects of both words into fresh registers and
// moves back took four, with no register permutation for the compiler to resolve
__device__ __forceinline__ void cswap_bits(float &a, float &b, uint32_t mask) {
    const uint32_t x = __builtin_bit_cast(uint32_t, a), y = __builtin_bit_cast(uint32_t, b);
    const uint32_t d = (x ^ y) & mask;
    a = __builtin_bit_cast(float, x ^ d);
    b = __builtin_bit_cast(float, y ^ d);
}
__device__ __forceinline__ void cswap_bits(double &a, double &b, uint32_t mask) {
    const uint64_t m64 = mask ? ~0ull : 0ull;
    const uint64_t x = __builtin_bit_cast(uint64_t, a), y = __builtin_bit_cast(uint64_t, b);
    const uint64_t d = (x ^ y) & m64;
    a = __builtin_bit_cast(double, x ^ d);
    b = __builtin_bit_cast(double, y ^ d);
}

template <typename R, int RB, int J>
__device__ __forceinline__ void reg_x(cvec<R> (&v)[1 << RB], const ROp &f) {
    const uint32_t on = f.onm;
#pragma unroll
    for (int m = 0; m < (1 << RB); ++m) {
        if (m & (1 << J)) continue;
        const uint32_t mask = 0u - (on >> m & 1u);
        cswap_bits(v[m].x, v[m | (1 << J)].x, mask);
        cswap_bits(v[m].y, v[m | (1 << J)].y, mask);
    }
}

template <typename R, int RB>
__device__ __forceinline__ void reg_phase(cvec<R> (&v)[1 << RB], const ROp &f) {
    const cvec<R> ph = cmake<R>((R)f.u[0], (R)f.u[1]);
    const uint32_t on = f.onm;
#pragma unroll
    for (int m = 0; m < (1 << RB); ++m)
        if (on >> m & 1u) v[m] = cmul<R>(v[m], ph);
}

template <typename R, int RB>
__device__ __forceinline__ void reg_apply(cvec<R> (&v)[1 << RB], const ROp &f) {
    switch (f.type) {
    case OP_PHASE: reg_phase<R, RB>(v, f); break;
    case OP_X:
        switch (f.j0) {
        case 0: reg_x<R, RB, 0>(v, f); break;
        case 1: reg_x<R, RB, 1 < RB ? 1 : 0>(v, f); break;
        case 2: reg_x<R, RB, 2 < RB ? 2 : 0>(v, f); break;
        case 3: reg_x<R, RB, 3 < RB ? 3 : 0>(v, f); break;
        default: reg_x<R, RB, 4 < RB ? 4 : 0>(v, f); break;
        }
        break;
    default:
        switch (f.j0) {
        case 0: reg_u<R, RB, 0>(v, f); break;
        case 1: reg_u<R, RB, 1 < RB ? 1 : 0>(v, f); break;
        case 2: reg_u<R, RB, 2 < RB ? 2 : 0>(v, f); break;
        case 3: reg_u<R, RB, 3 < RB ? 3 : 0>(v, f); break;
        default: reg_u<R, RB, 4 < RB ? 4 : 0>(v, f); break;
        }
        break;
    }
}

// LDS access by byte address.  The kernels that use these have no static LDS,
// so their dynamic area starts at address 0 (the host checks this): a slot's
// byte offset, formed by XOR, is then its address with no base added.
template <typename R> using v2r = R __attribute__((ext_vector_type(2)));
template <typename T> using lptr = __attribute__((address_space(3))) T *;
template <typename R>
__device__ __forceinline__ cvec<R> lds_ld(uint32_t a) {
    const v2r<R> x = *(lptr<v2r<R>>)(uintptr_t)a;
    return cmake<R>(x.x, x.y);
}
template <typename R>
__device__ __forceinline__ void lds_st(uint32_t a, cvec<R> v) {
    v2r<R> x;
    x.x = v.x;
    x.y = v.y;
    *(lptr<v2r<R>>)(uintptr_t)a = x;
}

// One fused pass.  Blocks walk the tiles tile = block + i * (blocks in the
// grid): the grid is what the device holds at once, or one tile per block
// when that covers them all.  (Reading the next tile into registers during
// this tile's segments cost more in registers than it hid.)
template <typename R, int RB, int NT = FUSE_BLOCK>
__global__ __launch_bounds__(NT) void k_fused(cvec<R> *__restrict__ psi, const FPass *__restrict__ passes,
                                                       int pi, const FSeg *__restrict__ segs,
                                                       const ROp *__restrict__ ops, uint64_t ntiles) {
    extern __shared__ unsigned char smem_raw[];
    cvec<R> *tile = reinterpret_cast<cvec<R> *>(smem_raw);
    const FPass &P = passes[pi];
    const int k = P.k, c = P.c, r = P.r;
    const uint32_t T = 1u << k;
    const uint64_t tstride = (uint64_t)gridDim.x * gridDim.y;
    const int *hpos = P.hpos;

    // HBM <-> LDS with U loads in flight per thread.  scatter_t is a bit
    // deposit, so the thread's part (bits below log2 NT), the part of
    // the unrolled index u and that of the outer step t0 combine by OR; the
    // offsets of u's bits are formed once and combined per load (uniform
    // values: a table of all U combinations held 48 more vector registers
    // through the whole kernel).
    constexpr int U = sizeof(R) == 4 ? 16 : 8;
    constexpr int LB = NT == 512 ? 9 : 8, LU = sizeof(R) == 4 ? 4 : 3;      // log2 NT, log2 U
    const uint64_t gthr = scatter_t(threadIdx.x & (T - 1u), c, r, hpos);
    // swz is XOR-linear too: the LDS slot of t0 + u 256 + thread is
    // swz(thread) ^ swz(t0) ^ swz(u 256)
    const uint32_t sthr = swz<R>(threadIdx.x);
    const bool big = T >= NT * U;
    // the offsets of the bits of u (HBM and LDS), combined per load
    uint64_t hb[LU];
    uint32_t hs[LU];
#pragma unroll
    for (int i = 0; i < LU; ++i) {
        hb[i] = big ? scatter_t(1u << (LB + i), c, r, hpos) : 0;
        hs[i] = swz<R>(1u << (LB + i)) * (uint32_t)sizeof(cvec<R>);
    }
    auto uoff = [&](int u) {
        uint64_t o = 0;
#pragma unroll
        for (int i = 0; i < LU; ++i)
            if (u >> i & 1) o |= hb[i];
        return o;
    };
    auto uswz = [&](int u) {
        uint32_t w = 0;
#pragma unroll
        for (int i = 0; i < LU; ++i)
            if (u >> i & 1) w ^= hs[i];
        return w;
    };
    for (uint64_t tl = (uint64_t)blockIdx.x + (uint64_t)blockIdx.y * gridDim.x; tl < ntiles; tl += tstride) {
        const uint64_t base = pdep64(tl, P.nl_mask) | P.fix_val;
        if (big) {
            for (uint32_t t0 = 0; t0 < T; t0 += NT * U) {
                const uint64_t g0 = base | gthr | scatter_t(t0, c, r, hpos);
                const uint32_t s0 = (sthr ^ swz<R>(t0)) * (uint32_t)sizeof(cvec<R>);
                cvec<R> buf[U];
#pragma unroll
                for (int u = 0; u < U; ++u) buf[u] = psi[g0 | uoff(u)];
#pragma unroll
                for (int u = 0; u < U; ++u) lds_st<R>(s0 ^ uswz(u), buf[u]);
            }
        } else {
            for (uint32_t t = threadIdx.x; t < T; t += NT) tile[swz<R>(t)] = psi[base | scatter_t(t, c, r, hpos)];
        }
        __syncthreads();

        const uint32_t lines = T >> RB;                  // register lines per tile
        for (int sg = 0; sg < P.nseg; ++sg) {
            const FSeg &S = segs[P.seg_off + sg];
            // swz is XOR-linear and bt and the register bits are disjoint, so the
            // slot of bt | (bits of m) is swz(bt) ^ S.off[m] (the table is uniform,
            // in bytes, as the slot is used)
            uint32_t off[1 << RB];
#pragma unroll
            for (int m = 0; m < (1 << RB); ++m) off[m] = S.off[m];
            const ROp *op0 = ops + S.op_off;
            for (uint32_t line = threadIdx.x; line < lines; line += NT) {
                // the tile bits outside the register positions: the line index
                // with a zero inserted at each position, lowest first
                uint32_t bt = line;
#pragma unroll
                for (int i = 0; i < RB; ++i) bt = insert0(bt, S.pos[i]);
                const uint32_t sbt = swz<R>(bt) * (uint32_t)sizeof(cvec<R>);
                cvec<R> v[1 << RB];
#pragma unroll
                for (int m = 0; m < (1 << RB); ++m) v[m] = lds_ld<R>(sbt ^ off[m]);
                for (int o = 0; o < S.nops; ++o) {
                    const ROp &f = op0[o];
                    if ((base & f.gmask) != f.gval || (bt & f.tmask) != f.tval) continue;
                    reg_apply<R, RB>(v, f);
                }
#pragma unroll
                for (int m = 0; m < (1 << RB); ++m) lds_st<R>(sbt ^ S.offw[m], v[m]);
            }
            __syncthreads();
        }

        if (big) {
            for (uint32_t t0 = 0; t0 < T; t0 += NT * U) {
                const uint64_t g0 = base | gthr | scatter_t(t0, c, r, hpos);
                const uint32_t s0 = (sthr ^ swz<R>(t0)) * (uint32_t)sizeof(cvec<R>);
                cvec<R> buf[U];
#pragma unroll
                for (int u = 0; u < U; ++u) buf[u] = lds_ld<R>(s0 ^ uswz(u));
#pragma unroll
                for (int u = 0; u < U; ++u) psi[g0 | uoff(u)] = buf[u];
            }
        } else {
            for (uint32_t t = threadIdx.x; t < T; t += NT) psi[base | scatter_t(t, c, r, hpos)] = tile[swz<R>(t)];
        }
        // the next tile is written into the LDS this one was read from
        if (tl + tstride < ntiles) __syncthreads();
    }
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
    constexpr int U = sizeof(R) == 4 ? 16 : 8;
    if (T >= FUSE_BLOCK * U) {
        for (uint32_t t0 = threadIdx.x; t0 < T; t0 += FUSE_BLOCK * U) {
            cvec<R> buf[U];
#pragma unroll
            for (int u = 0; u < U; ++u) buf[u] = psi[gidx(t0 + u * FUSE_BLOCK)];
#pragma unroll
            for (int u = 0; u < U; ++u) tile[t0 + u * FUSE_BLOCK] = buf[u];
        }
    } else {
        for (uint32_t t = threadIdx.x; t < T; t += FUSE_BLOCK) tile[t] = psi[gidx(t)];
    }
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
    if (T >= FUSE_BLOCK * U) {
        for (uint32_t t0 = threadIdx.x; t0 < T; t0 += FUSE_BLOCK * U) {
            cvec<R> buf[U];
#pragma unroll
            for (int u = 0; u < U; ++u) buf[u] = tile[t0 + u * FUSE_BLOCK];
#pragma unroll
            for (int u = 0; u < U; ++u) psi[gidx(t0 + u * FUSE_BLOCK)] = buf[u];
        }
    } else {
        for (uint32_t t = threadIdx.x; t < T; t += FUSE_BLOCK) psi[gidx(t)] = tile[t];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static int g_lds_limit = 0;
static bool g_fused_lds_at_0 = false;   // k_fused has no static LDS: its tile starts at address 0

static int lds_limit_bytes() {
    if (g_lds_limit) return g_lds_limit;
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    int lim = 65536;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.sharedMemPerBlock > 0)
        lim = (int)prop.sharedMemPerBlock;
    if (lim > 147456) lim = 147456;   // the largest power-of-two tile (128 KiB) plus headroom
    bool ok = true;
    const void *fk[] = {(const void *)k_fused<float, 5>, (const void *)k_fused<float, 4>,
                        (const void *)k_fused<float, 4, 512>, (const void *)k_fused<float, 3>,
                        (const void *)k_fused<double, 4>, (const void *)k_fused<double, 3>};
    for (const void *f : fk) ok &= hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) == hipSuccess;
    ok &= hipFuncSetAttribute((const void *)k_qft_pass<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) ==
          hipSuccess;
    ok &= hipFuncSetAttribute((const void *)k_qft_pass<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) ==
          hipSuccess;
    bool at0 = true;
    for (const void *f : fk) {
        hipFuncAttributes fa;
        if (hipFuncGetAttributes(&fa, f) != hipSuccess || fa.sharedSizeBytes != 0) at0 = false;
    }
    (void)hipGetLastError();
    if (!ok) lim = 65536;
    g_fused_lds_at_0 = at0;
    g_lds_limit = lim;
    return lim;
}

// low index bits every pass keeps local (contiguous HBM segments of 2^c
// amplitudes): 256-byte segments by default; SV_FUSED_LOWBITS (2..10) overrides
static int low_bits_for(sv_dtype dt) {
    if (const char *e = getenv("SV_FUSED_LOWBITS")) {
        const int v = atoi(e);
        if (v >= 2 && v <= 10) return v;
    }
    return dt == SV_C128 ? 4 : 5;
}

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
    // a gate needs at most two local bits besides the low run, so every pass
    // takes at least the first gate left (callers pass c0 <= kmax - 2)
    c0 = std::max(0, std::min(c0, kmax - 2));
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

// tile positions a gate must hold in registers
static uint32_t op_targets(const FOp &f) {
    if (f.type == OP_PHASE) return 0;
    if (f.type == OP_SWAP) return (1u << f.p0) | (1u << f.p1);
    return 1u << f.p0;
}

static uint32_t compress_bits(uint32_t x, uint32_t S) {   // tile bits in S -> register bits
    uint32_t r = 0;
    int j = 0;
    for (int p = 0; p < 32; ++p)
        if (S >> p & 1) {
            if (x >> p & 1) r |= 1u << j;
            ++j;
        }
    return r;
}

// bit m set for the register indices m < 2^RB with (m & rmask) == rval
static uint32_t on_mask(uint32_t rmask, uint32_t rval, int RB) {
    uint32_t on = 0;
    for (uint32_t m = 0; m < (1u << RB); ++m)
        if ((m & rmask) == rval) on |= 1u << m;
    return on;
}

// Register-controlled NOTs at either end of a segment permute the register
// indices only, so they need no arithmetic: those that commute to the start
// (with every op before them that is not moved) become the read offsets,
// those that commute to the end the write offsets, and both leave the op
// list.  A NOT moves only if its condition is on register bits alone (no
// tile or non-local control); an op touches its target and condition bits,
// a phase every register bit.  If P is the product of the leading NOTs in
// program order, register m holds the amplitude of P^-1(m) after them; if T
// is that of the trailing ones, the value in register m ends at T(m).
static void fold_permutations(FSeg &g, std::vector<ROp> &rops, int RB) {
    const size_t n = (size_t)g.nops, b0 = (size_t)g.op_off;
    const uint32_t all = (1u << RB) - 1u;
    auto movable = [](const ROp &f) { return f.type == OP_X && f.tmask == 0 && f.gmask == 0; };
    auto touched = [&](const ROp &f) { return f.type == OP_PHASE ? all : ((1u << f.j0) | f.rmask); };
    auto xmap = [](const ROp &f, uint32_t m) { return (m & f.rmask) == f.rval ? m ^ (1u << f.j0) : m; };
    std::vector<char> lead(n, 0), trail(n, 0);
    uint32_t blocked = 0;
    for (size_t i = 0; i < n; ++i) {
        const ROp &f = rops[b0 + i];
        if (movable(f) && !(touched(f) & blocked))
            lead[i] = 1;
        else
            blocked |= touched(f);
    }
    blocked = 0;
    for (size_t i = n; i-- > 0;) {
        const ROp &f = rops[b0 + i];
        if (lead[i]) continue;
        if (movable(f) && !(touched(f) & blocked))
            trail[i] = 1;
        else
            blocked |= touched(f);
    }
    uint32_t base[1 << MAX_RB];
    for (uint32_t m = 0; m <= all; ++m) base[m] = g.off[m];
    for (uint32_t m = 0; m <= all; ++m) {
        uint32_t p = m;      // P^-1(m): the leading NOTs from the last to the first
        for (size_t i = n; i-- > 0;)
            if (lead[i]) p = xmap(rops[b0 + i], p);
        uint32_t q = m;      // T(m), where the value in register m ends: the trailing NOTs from the first
        for (size_t i = 0; i < n; ++i)
            if (trail[i]) q = xmap(rops[b0 + i], q);
        g.off[m] = base[p];
        g.offw[m] = base[q];
    }
    size_t w = b0;
    for (size_t i = 0; i < n; ++i)
        if (!lead[i] && !trail[i]) rops[w++] = rops[b0 + i];
    rops.resize(w);
    g.nops = (int)(w - b0);
}

// cut a pass's gate list into register segments of at most RB target
// positions.  Gates that touch disjoint qubits commute, so a segment takes
// every gate that is ready (all earlier gates it does not commute with are
// placed) and whose targets fit, in program order, not only a contiguous run.
static void segment_pass(const HostPass &hp, int RB, int swz_bits, std::vector<FSeg> &segs, std::vector<ROp> &rops) {
    const int k = hp.hdr.k;
    const std::vector<FOp> &ops = hp.ops;
    const size_t n = ops.size();
    // conflict: a target of one is a target or a local control of the other
    // (controls on non-local bits never coincide with a target: targets are local)
    std::vector<std::vector<int>> pred(n);
    for (size_t b = 0; b < n; ++b) {
        const uint32_t tb = op_targets(ops[b]), qb = tb | (uint32_t)ops[b].lmask;
        for (size_t a = 0; a < b; ++a) {
            const uint32_t ta = op_targets(ops[a]), qa = ta | (uint32_t)ops[a].lmask;
            if ((ta & qb) || (tb & qa)) pred[b].push_back((int)a);
        }
    }
    std::vector<char> done(n, 0);
    size_t left = n;
    while (left) {
        uint32_t S = 0;
        std::vector<int> seg;
        for (bool progress = true; progress;) {
            progress = false;
            for (size_t b = 0; b < n; ++b) {
                if (done[b]) continue;
                bool ready = true;
                for (int a : pred[b])
                    if (!done[a]) {
                        ready = false;
                        break;
                    }
                if (!ready || popcount64(S | op_targets(ops[b])) > RB) continue;
                S |= op_targets(ops[b]);
                done[b] = 1;
                --left;
                seg.push_back((int)b);
                progress = true;
            }
        }
        // fill with the highest free positions: the threads of a wavefront then
        // differ in the low tile bits (contiguous LDS slots)
        for (int p = k - 1; p >= 0 && popcount64(S) < RB; --p) S |= 1u << p;
        FSeg g;
        memset(&g, 0, sizeof g);
        int npos = 0;
        for (int p = 0; p < k; ++p)
            if (S >> p & 1) g.pos[npos++] = p;
        for (int m = 0; m < (1 << RB); ++m) {
            uint32_t o = 0;
            for (int i = 0; i < RB; ++i)
                if (m >> i & 1) o |= 1u << g.pos[i];
            g.off[m] = swz_e(o, swz_bits) * (swz_bits == 5 ? 8u : 16u);   // bytes
        }
        g.op_off = (int)rops.size();
        g.nops = (int)seg.size();
        for (int q : seg) {
            const FOp &f = ops[q];
            ROp o;
            memset(&o, 0, sizeof o);
            o.type = f.type;
            o.j0 = f.type == OP_PHASE ? 0 : __builtin_ctz(compress_bits(1u << f.p0, S));
            o.j1 = f.type == OP_SWAP ? __builtin_ctz(compress_bits(1u << f.p1, S)) : 0;
            o.rmask = compress_bits((uint32_t)f.lmask & S, S);
            o.rval = compress_bits((uint32_t)f.lval & S, S);
            o.tmask = (uint32_t)f.lmask & ~S;
            o.tval = (uint32_t)f.lval & ~S;
            o.onm = on_mask(o.rmask, o.rval, RB);
            o.gmask = f.gmask;
            o.gval = f.gval;
            if (f.type == OP_PHASE) {
                const long double a = ldexpl((long double)(int64_t)f.turns, -64) * 2.0L * 3.14159265358979323846264338327950288L;
                o.u[0] = (double)cosl(a);
                o.u[1] = (double)sinl(a);
            } else {
                memcpy(o.u, f.u, sizeof o.u);
            }
            if (f.type == OP_SWAP) {
                // SWAP(a, b) = CX(a -> b) CX(b -> a) CX(a -> b), each an X on
                // a register bit controlled by the other
                const int a = o.j0, b = o.j1;
                ROp x = o;
                x.type = OP_X;
                for (int r = 0; r < 3; ++r) {
                    const int tgt = r == 1 ? a : b, ctl = r == 1 ? b : a;
                    x.j0 = tgt;
                    x.j1 = 0;
                    x.rmask = o.rmask | (1u << ctl);
                    x.rval = o.rval | (1u << ctl);
                    x.onm = on_mask(x.rmask, x.rval, RB);
                    rops.push_back(x);
                }
                g.nops += 2;
                continue;
            }
            rops.push_back(o);
        }
        fold_permutations(g, rops, RB);
        segs.push_back(g);
    }
}

// amplitudes per thread in a segment: 2^5 (complex64) or 2^4 (complex128);
// SV_FUSED_RB (3..5, complex128 at most 4) overrides
static int reg_bits_for(sv_dtype dt, int k) {
    int rb = dt == SV_C128 ? 4 : 5;
    if (const char *e = getenv("SV_FUSED_RB")) {
        const int v = atoi(e);
        if (v >= 3 && v <= (dt == SV_C128 ? 4 : 5)) rb = v;
    }
    return rb < k ? rb : k;
}

// persistent fused passes (the blocks the device holds at once walk the
// tiles); SV_FUSED_PERSIST=0 launches one block per tile
static int fused_persist_env() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("SV_FUSED_PERSIST");
        v = (e && atoi(e) == 0) ? 0 : 1;
    }
    return v;
}

template <typename R, int RB, int NT = FUSE_BLOCK>
static void launch_fused(uint64_t tiles, size_t lds, hipStream_t st, cvec<R> *psi, const FPass *dp, int i,
                         const FSeg *ds, const ROp *dops) {
    dim3 grid = tile_grid(tiles);
    if (fused_persist_env()) {
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_fused<R, RB, NT>, NT, lds);
        (void)hipGetLastError();
        const uint64_t slots = (uint64_t)(cus > 0 ? cus : 1) * (uint64_t)(per > 0 ? per : 1);
        if (slots < tiles) grid = dim3((unsigned)slots);
    }
    hipLaunchKernelGGL((k_fused<R, RB, NT>), grid, dim3(NT), lds, st, psi, dp, i, ds, dops, tiles);
}

// rb_req: amplitudes per thread in a segment as 2^rb_req (the fusion tuner's
// choice), 0 for the default of reg_bits_for
template <typename R>
static sv_status launch_passes(sv_state s, std::vector<HostPass> &passes, int rb_req = 0) {
    if (passes.empty()) return SV_OK;
    lds_limit_bytes();
    if (!g_fused_lds_at_0) return fail(SV_EDEVICE, "the fused-pass kernels carry static LDS; their tile addressing needs none");
    int RB = reg_bits_for(s->dt, passes[0].hdr.k);
    if (rb_req > 0) {
        if (rb_req < 3 || rb_req > (sizeof(R) == 4 ? 5 : 4)) return fail(SV_EINVAL, "%d register bits per segment line", rb_req);
        RB = std::min(rb_req, passes[0].hdr.k);
    }
    if (RB < 3) return fail(SV_EUNSUPPORTED, "state too small for fused passes");
    std::vector<FSeg> segs;
    std::vector<ROp> rops;
    for (auto &p : passes) {
        if (p.hdr.k < RB) return fail(SV_EDEVICE, "pass with %d local qubits (< %d)", p.hdr.k, RB);
        p.hdr.seg_off = (int)segs.size();
        segment_pass(p, RB, sizeof(R) == 4 ? 5 : 4, segs, rops);
        p.hdr.nseg = (int)segs.size() - p.hdr.seg_off;
    }
    const size_t hbytes = passes.size() * sizeof(FPass);
    const size_t sbytes = std::max<size_t>(segs.size(), 1) * sizeof(FSeg);
    const size_t obytes = std::max<size_t>(rops.size(), 1) * sizeof(ROp);
    const size_t soff = (hbytes + 255) & ~(size_t)255, ooff = (soff + sbytes + 255) & ~(size_t)255;
    std::vector<unsigned char> blob(ooff + obytes, 0);
    for (size_t i = 0; i < passes.size(); ++i) memcpy(blob.data() + i * sizeof(FPass), &passes[i].hdr, sizeof(FPass));
    memcpy(blob.data() + soff, segs.data(), segs.size() * sizeof(FSeg));
    memcpy(blob.data() + ooff, rops.data(), rops.size() * sizeof(ROp));
    void *dev = nullptr;
    SV_HIP(hipMallocAsync(&dev, blob.size(), s->stream));
    sv_status st = upload(s, dev, blob.data(), blob.size());
    if (st != SV_OK) {
        hipFreeAsync(dev, s->stream);
        return st;
    }
    const FPass *dp = (const FPass *)dev;
    const FSeg *ds = (const FSeg *)((unsigned char *)dev + soff);
    const ROp *dops = (const ROp *)((unsigned char *)dev + ooff);
    for (size_t i = 0; i < passes.size(); ++i) {
        const FPass &h = passes[i].hdr;
        const uint64_t tiles = dim_of(s->n - h.k);
        const size_t lds = ((size_t)1 << h.k) * sizeof(cvec<R>);
        TraceScope _ts(s->stream, "fused_pass", 2.0 * (double)dim_of(s->n) * sizeof(cvec<R>), 0.0);
        cvec<R> *psi = (cvec<R> *)s->data;
        // complex64 lines of 16 amplitudes on tiles of 2^13 or more: 512
        // threads, so that each has one line per segment and two workgroups
        // of a 64 KiB tile keep four waves on every SIMD
        if (RB == 5 && sizeof(R) == 4) launch_fused<float, 5>(tiles, lds, s->stream, (cvec<float> *)psi, dp, (int)i, ds, dops);
        else if (RB >= 4 && sizeof(R) == 4 && (1u << (h.k - 4)) >= 512u)
            launch_fused<float, 4, 512>(tiles, lds, s->stream, (cvec<float> *)psi, dp, (int)i, ds, dops);
        else if (RB >= 4) launch_fused<R, 4>(tiles, lds, s->stream, psi, dp, (int)i, ds, dops);
        else launch_fused<R, 3>(tiles, lds, s->stream, psi, dp, (int)i, ds, dops);
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

namespace sv {

// The fusion autotuner (sv_apply_circuit with max_local = 0, states of 2^22
// amplitudes and more): the candidates are k local qubits in {K-1, K} (K the
// default, bounded by the LDS) times c contiguous low bits in {C-1, C, C+1}
// (C the default, c <= k - 2) times rb register bits per segment line (the
// default and one fewer).  Each candidate's plan is made for the whole
// circuit and its first passes are timed on a scratch copy of the state (the
// state itself is not touched): the first pass, plus the mean of up to eight
// others spread over the plan times their number.  When the two best
// estimates are within 10 %, both run their whole plan, and the faster is kept.  Cached per dtype, size and circuit
// structure (gate kinds and qubits, not angles) as (k, c, rb); an entry of
// (k, c) takes the default rb.  SV_FUSED_LOWBITS pins c and skips the tuning.
static uint64_t circuit_signature(const std::vector<PGate> &pg) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix(pg.size());
    for (const PGate &g : pg) {
        mix((uint64_t)g.kind);
        mix((uint64_t)(int64_t)g.t0);
        mix((uint64_t)(int64_t)g.t1);
        mix(g.cmask);
        mix(g.cval);
        mix(g.need);
    }
    return h;
}

sv_status fusion_config(sv_state s, const std::vector<PGate> &pg, int &k, int &c, int &rb) {
    if (s->n < 22 || getenv("SV_FUSED_LOWBITS")) return SV_OK;
    char sig[32];
    snprintf(sig, sizeof sig, "%016llx", (unsigned long long)circuit_signature(pg));
    const std::string key = std::string("fused/") + (s->dt == SV_C64 ? "c64/" : "c128/") + std::to_string(s->n) + "/" + sig;
    std::vector<int> cached;
    if (tune_lookup(key, cached) && (cached.size() == 2 || cached.size() == 3)) {
        k = cached[0];
        c = cached[1];
        rb = cached.size() == 3 ? cached[2] : 0;
        return SV_OK;
    }
    if (!autotune_enabled()) return SV_OK;
    const size_t bytes = dim_of(s->n) * amp_bytes(s->dt);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || free_b < bytes + bytes / 16) return SV_OK;
    void *scratch = nullptr;
    if (hipMalloc(&scratch, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return SV_OK;
    }
    sv_state t = new sv_state_s();
    t->n = s->n;
    t->dt = s->dt;
    t->data = scratch;
    t->owned = false;
    t->stream = s->stream;
    t->device = s->device;
    sv_status st = SV_OK;
    if (hipMemcpyAsync(scratch, s->data, bytes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
        st = fail(SV_EDEVICE, "scratch copy for the fusion tuner");
    // Candidates: tile depth k, contiguous low bits c and register bits per
    // segment line rb.  Fewer register bits mean more segments but far fewer
    // registers, so a smaller tile can run three or more workgroups per CU.
    // A plan's time is estimated from its first pass (which holds the most
    // ops) plus a sample of the others scaled to their number.
    const int K = k, C = c, RB0 = s->dt == SV_C64 ? 5 : 4;
    struct Cand {
        float est;
        int k, c, rb;
    };
    std::vector<Cand> cands;
    float best = 1e30f;
    for (int rr = RB0; rr >= RB0 - 1 && st == SV_OK; --rr) {
        for (int kk = K - 1; kk <= K && st == SV_OK; ++kk) {
            if (kk < 3 || kk < rr) continue;
            for (int cc = C - 1; cc <= C + 1 && st == SV_OK; ++cc) {
                if (cc < 0 || cc > kk - 2) continue;
                std::vector<HostPass> passes;
                plan(s->n, kk, cc, pg, passes);
                if (passes.empty()) continue;
                // the first pass, and up to eight of the others spread evenly
                // over the plan (pass times vary several-fold along it)
                const size_t N = passes.size(), S = N - 1 < 8 ? N - 1 : 8;
                std::vector<HostPass> first(passes.begin(), passes.begin() + 1), sample;
                for (size_t j = 0; j < S; ++j) sample.push_back(passes[1 + j * (N - 1) / S]);
                float ms0 = 0.f, ms1 = 0.f;
                st = time_stream(s->stream, 1, &ms0, [&]() {
                    return s->dt == SV_C64 ? launch_passes<float>(t, first, rr) : launch_passes<double>(t, first, rr);
                });
                if (st == SV_OK && S > 0)
                    st = time_stream(s->stream, 1, &ms1, [&]() {
                        return s->dt == SV_C64 ? launch_passes<float>(t, sample, rr) : launch_passes<double>(t, sample, rr);
                    });
                const float est = ms0 + (S > 0 ? ms1 * (float)(N - 1) / (float)S : 0.f);
                if (st == SV_OK) cands.push_back({est, kk, cc, rr});
            }
        }
    }
    // the two best estimates, when within 10 % of each other (closer than the
    // sample can tell apart), both run their whole plan, and the faster is kept
    std::sort(cands.begin(), cands.end(), [](const Cand &x, const Cand &y) { return x.est < y.est; });
    const size_t nfull = cands.size() > 1 && cands[1].est <= 1.1f * cands[0].est ? 2 : 1;
    if (nfull == 1 && !cands.empty()) {
        k = cands[0].k;
        c = cands[0].c;
        rb = cands[0].rb;
    }
    for (size_t i = 0; i < cands.size() && i < nfull && nfull > 1 && st == SV_OK; ++i) {
        const Cand &cd = cands[i];
        std::vector<HostPass> passes;
        plan(s->n, cd.k, cd.c, pg, passes);
        float ms = 0.f;
        st = time_stream(s->stream, 1, &ms, [&]() {
            return s->dt == SV_C64 ? launch_passes<float>(t, passes, cd.rb) : launch_passes<double>(t, passes, cd.rb);
        });
        if (st == SV_OK && ms < best) {
            best = ms;
            k = cd.k;
            c = cd.c;
            rb = cd.rb;
        }
    }
    hipStreamSynchronize(s->stream);
    sv_free(t);
    hipFree(scratch);
    if (st != SV_OK) return st;
    tune_store(key, {k, c, rb});
    return SV_OK;
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
    int k = clamp_k(s, max_local);
    if (k < 3) return fail(SV_EUNSUPPORTED, "state too small for fused passes");
    int c = std::max(0, std::min(low_bits_for(s->dt), k - 2)), rb = 0;
    if (max_local == 0) SV_TRY(fusion_config(s, pg, k, c, rb));
    std::vector<HostPass> passes;
    plan(s->n, k, c, pg, passes);
    return s->dt == SV_C64 ? launch_passes<float>(s, passes, rb) : launch_passes<double>(s, passes, rb);
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
