// Eigen-frame HHL as three fused column-tile kernels.
//
// The clock register [n_s, n_s + n_c) is split into a low group G1 =
// register bits [0, g1) and a high group G2 = [g1, n_c) (g1, g2 <= 10).  A
// tile holds C consecutive system columns j (contiguous in memory) times the
// 2^g clock values of one group, for one setting of the other group's bits
// (and the ancilla).
//
//   k_pipe_a: generate the state after phase estimation (product state over
//             the clock bits, relabelled so the cascades need no swaps), then
//             the inverse-QFT cascade on G1 (butterflies in registers, RA
//             bits at a time, one LDS exchange).  The G1 stages act on G1
//             qubits only, so the result is still a product between the
//             groups: psi(j, y1, y2) = T_j(y1) * B_j(y2), with T_j the G1
//             transform of the column's G1 factor and B_j(y2) the product of
//             the phases of the set G2 bits.  k_pipe_a therefore runs for
//             y2 = 0 only and leaves T in the clock rows y1 < 2^g1 of the
//             ancilla = 0 half, and stages every column's clock-bit phases.
//   k_pipe_b: the inverse-QFT cascade on G2 of T_j(y1) B_j(y2): each stage
//             maps a product state over the G2 bits to another, so the
//             cascade's output is T_j(y1) times a product of one factor per
//             G2 bit, formed directly; then eigenvalue inversion
//             a1 = (1/y) a0 (FP64 sums of P(a=1) and the norm)
//                                                     -> ancilla = 1 half
//   k_pipe_c: the uncompute projected on clock 0 (the QFT on the whole
//             clock, the conjugate phases, the Hadamard layer onto |0>), as
//             a contraction of the half against the transposed QFT applied
//             to the phase product state, itself a closed-form product
//                                                     -> FP64 partial sums
//
// Cascade stages on register qubit j (relative to the clock register):
//   inverse: a1 *= conj(phase), then (a0 + a1, a0 - a1)/sqrt 2
//   forward: (a0 + a1, (a0 - a1) * phase)/sqrt 2
// with phase = exp(2 pi i (v mod 2^j) / 2^(j+1)), v the register value: the
// controlled phases of the textbook QFT circuit that target qubit j.  The
// local part comes from a table of 2^g roots of unity, the part due to bits
// outside the tile is one exact-turn phase per stage and tile.
#include <math.h>

#include <algorithm>
#include <string>
#include <vector>

#include "sv_device.h"
#include "sv_hhl_internal.h"
#include "sv_internal.h"

namespace sv {


struct PipeArgs {
    uint64_t N;          // 2^n_s columns
    int n_s, n_c;
    int g1, g2;          // clock groups
    int cl;              // log2 of the columns per tile
    uint64_t abit;       // ancilla bit
    double scale;        // 2^(-n_c/2)
    int sgn;             // signed (two's-complement) clock for the inversion
    uint64_t gcut;       // 0: inversion sin = 1/y; >= 1: gapped-phase-estimation flag, sin = [|y| >= gcut]
    int pslog, iters;    // work-queue items: log2 of the column-block stride in blocks (0);
                         // column blocks per item
};

// HBM pointers of a solve, in the global address space: the pointers come
// from a descriptor, so without the cast every access would be a flat
// instruction, which also counts against the LDS wait counter.
template <typename T> using gptr = __attribute__((address_space(1))) T *;

// complex loads and stores through a global pointer (a native two-element
// vector, so no class member is needed on an address-space-qualified object)
template <typename R> using v2_t = R __attribute__((ext_vector_type(2)));
template <typename R>
__device__ __forceinline__ cvec<R> gld(const cvec<R> *p, uint64_t i) {
    const v2_t<R> x = ((gptr<const v2_t<R>>)p)[i];
    return cmake<R>(x.x, x.y);
}
template <typename R>
__device__ __forceinline__ void gst(cvec<R> *p, uint64_t i, cvec<R> v) {
    v2_t<R> x;
    x.x = v.x;
    x.y = v.y;
    ((gptr<v2_t<R>>)p)[i] = x;
}

// non-temporal forms for the ancilla = 1 half, written by k_pipe_b and read
// back only by k_pipe_c after every tile is written: far more than the L2
// and MALL hold, so they are streamed (the nt bit) instead of cached
template <typename R>
__device__ __forceinline__ void gst_nt(cvec<R> *p, uint64_t i, cvec<R> v) {
    v2_t<R> x;
    x.x = v.x;
    x.y = v.y;
    __builtin_nontemporal_store(x, &((gptr<v2_t<R>>)p)[i]);
}
template <typename R>
__device__ __forceinline__ cvec<R> gld_nt(const cvec<R> *p, uint64_t i) {
    const v2_t<R> x = __builtin_nontemporal_load(&((gptr<const v2_t<R>>)p)[i]);
    return cmake<R>(x.x, x.y);
}

// the solve of this block: the kernel argument, or entry blockIdx.z of a batch
__device__ __forceinline__ PipeSolve solve_of(const PipeSolve &one, const PipeSolve *many) {
    if (!many) return one;
    const gptr<const PipeSolve> m = (gptr<const PipeSolve>)many + blockIdx.z;
    PipeSolve r;
    r.psi = m->psi;
    r.beta = m->beta;
    r.F = m->F;
    r.part = m->part;
    r.zpart = m->zpart;
    return r;
}

template <typename R>
__device__ __forceinline__ cvec<R> cconjmul(cvec<R> a, cvec<R> b) {   // a * conj(b)
    return cmake<R>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

__device__ __forceinline__ float ffma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double ffma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One cascade stage on a register line v[0..2^RL): pairs differ in bit kb of
// the register index.  tw is the stage's twiddle table (entry m = phase for
// the register bits below the stage's qubit equal to m); tidx(k) gives that
// m for element k.  The 1/sqrt(2) of the Hadamard is left out here and
// applied once per group by the caller (butterflies are add/sub only).
// has_tw = false for the lowest qubit of the register (phase 1).
// The inverse butterfly forms v0 = a0 + a1 conj(w) with four FMAs and
// v1 = 2 a0 - v0 with two more (six operations instead of eight).
template <typename R, int RL, bool INV, typename TIDX>
__device__ __forceinline__ void stage(cvec<R> (&v)[1 << RL], int kb, const cvec<R> *__restrict__ tw, bool has_tw,
                                      TIDX tidx) {
#pragma unroll
    for (int k0 = 0; k0 < (1 << RL); ++k0) {
        if (k0 & (1 << kb)) continue;
        const int k1 = k0 | (1 << kb);
        cvec<R> a0 = v[k0], a1 = v[k1];
        if (INV) {
            if (has_tw) {
                const cvec<R> w = tw[tidx(k0)];
                const R rx = ffma(a1.x, w.x, ffma(a1.y, w.y, a0.x));
                const R ry = ffma(a1.y, w.x, ffma(-a1.x, w.y, a0.y));
                v[k0] = cmake<R>(rx, ry);
                v[k1] = cmake<R>(ffma((R)2, a0.x, -rx), ffma((R)2, a0.y, -ry));
            } else {
                v[k0] = cmake<R>(a0.x + a1.x, a0.y + a1.y);
                v[k1] = cmake<R>(a0.x - a1.x, a0.y - a1.y);
            }
        } else {
            const cvec<R> d = cmake<R>(a0.x - a1.x, a0.y - a1.y);
            v[k0] = cmake<R>(a0.x + a1.x, a0.y + a1.y);
            v[k1] = has_tw ? cmul<R>(d, tw[tidx(k0)]) : d;
        }
    }
}

// Two forward stages at once (radix 4): the stage on bit kb + 1, then the
// stage on bit kb, for every group of four elements that differ in those two
// bits.  With m the group's twiddle index (the same for both stages: the
// bit-kb-clear entry of the upper stage), t = tlo[m], T = thi[m], and the
// upper stage's twiddle for bit kb set equal to i T, the four outputs are
//   z00 = s0 + s1, z01 = (s0 - s1) t, z10 = T (d0 + i d1), z11 = T t (d0 - i d1)
// with s0, d0 = x00 +- x10 and s1, d1 = x01 +- x11 (x_ab: bit kb + 1 = a,
// bit kb = b); tt[m] = T t.  Three twiddle products per four elements
// instead of four.
template <typename R, int RL, typename TIDX>
__device__ __forceinline__ void stage4f(cvec<R> (&v)[1 << RL], int kb, const cvec<R> *__restrict__ tlo,
                                        const cvec<R> *__restrict__ thi, const cvec<R> *__restrict__ tt, TIDX tidx) {
    const int b0 = 1 << kb, b1 = 2 << kb;
#pragma unroll
    for (int k = 0; k < (1 << RL); ++k) {
        if (k & (b0 | b1)) continue;
        const cvec<R> x00 = v[k], x01 = v[k | b0], x10 = v[k | b1], x11 = v[k | b0 | b1];
        const int m = tidx(k);
        const cvec<R> s0 = cmake<R>(x00.x + x10.x, x00.y + x10.y), d0 = cmake<R>(x00.x - x10.x, x00.y - x10.y);
        const cvec<R> s1 = cmake<R>(x01.x + x11.x, x01.y + x11.y), d1 = cmake<R>(x01.x - x11.x, x01.y - x11.y);
        v[k] = cmake<R>(s0.x + s1.x, s0.y + s1.y);
        v[k | b0] = cmul<R>(cmake<R>(s0.x - s1.x, s0.y - s1.y), tlo[m]);
        v[k | b1] = cmul<R>(cmake<R>(d0.x - d1.y, d0.y + d1.x), thi[m]);
        v[k | b0 | b1] = cmul<R>(cmake<R>(d0.x + d1.y, d0.y - d1.x), tt[m]);
    }
}

// The forward cascade over stages hi down to lo of a register line, in
// radix-4 pairs from the top (a last single stage when the count is odd);
// tables at tw_off(jb) of TW (twiddles) and TT (pair products), with stage
// jb acting on line bit jb - lo_bit and tidx(jb, k) its twiddle index.
template <typename R, int RL, int HI, int LO, int LOBIT, typename TIDX>
__device__ __forceinline__ void fwd_cascade(cvec<R> (&v)[1 << RL], const cvec<R> *TW, const cvec<R> *TT, TIDX tidx) {
#pragma unroll
    for (int jb = HI; jb >= LO; jb -= 2) {
        if (jb - 1 >= LO) {
            const int lo = jb - 1;
            stage4f<R, RL>(v, lo - LOBIT, TW + ((1 << lo) - 1), TW + ((1 << jb) - 1), TT + ((1 << lo) - 1),
                           [&](int k) { return tidx(lo, k); });
        } else {
            stage<R, RL, false>(v, jb - LOBIT, TW + ((1 << jb) - 1), true, [&](int k) { return tidx(jb, k); });
        }
    }
}

// Twiddle tables of one group, stage jb at offset 2^jb - 1 (2^jb entries):
// entry m = exp(2 pi i (vlow + m 2^gbase) / 2^(gbase + jb + 1)), where vlow
// (< 2^gbase) are the register bits below the group, fixed for the tile.
template <typename R>
__device__ __forceinline__ void fill_twiddles(cvec<R> *TW, int g, int gbase, uint64_t vlow) {
    for (int i = threadIdx.x; i < (1 << g) - 1; i += blockDim.x) {
        int jb = 0;
        while ((2 << jb) - 1 <= i) ++jb;
        const uint64_t m = (uint64_t)(i - ((1 << jb) - 1));
        const int j = gbase + jb;
        TW[i] = turn_phase<R>((vlow + (m << gbase)) << (63 - j));
    }
}
__device__ __forceinline__ int tw_off(int jb) { return (1 << jb) - 1; }

// The radix-4 pair products at offset 2^jb - 1 for jb <= g - 2: entry m is
// (stage jb + 1 twiddle m) x (stage jb twiddle m), formed as one exact turn count
template <typename R>
__device__ __forceinline__ void fill_pair_twiddles(cvec<R> *TT, int g, int gbase, uint64_t vlow) {
    for (int i = threadIdx.x; i < (1 << (g - 1)) - 1; i += blockDim.x) {
        int jb = 0;
        while ((2 << jb) - 1 <= i) ++jb;
        const uint64_t m = (uint64_t)(i - ((1 << jb) - 1));
        const int j = gbase + jb;
        const uint64_t X = vlow + (m << gbase);
        TT[i] = turn_phase<R>((X << (63 - j)) + (X << (62 - j)));
    }
}

// tile decomposition: column block and the setting of the other group's bits
__device__ __forceinline__ void tile_coords(const PipeArgs &A, uint64_t &j0, uint64_t &o) {
    const uint64_t nb = A.N >> A.cl;
    const uint64_t tid = (uint64_t)blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
    j0 = (tid % nb) << A.cl;
    o = tid / nb;
}

// ---------------------------------------------------------------------------
// k_pipe_a: phase-estimation state + inverse cascade on G1
// ---------------------------------------------------------------------------
template <typename R, int RA, int RB, int NT>
__device__ __forceinline__ void pipe_a_body(const PipeArgs &A, const PipeSolve &S, uint64_t j0, uint64_t o) {
    constexpr int G = RA + RB;
    cvec<R> *__restrict__ psi = (cvec<R> *)S.psi;
    const double2 *__restrict__ beta = S.beta;
    const gptr<const uint64_t> __restrict__ F = (gptr<const uint64_t>)S.F;
    extern __shared__ unsigned char smem_raw[];
    const int C = 1 << A.cl;
    cvec<R> *tile = reinterpret_cast<cvec<R> *>(smem_raw);          // [2^G][C]
    cvec<R> *TW = tile + ((size_t)C << G);                           // [2^G - 1] (+1 pad)
    cvec<R> *om = TW + (1 << G);                                     // [G][C] exp(2 pi i F) of the local bits
    cvec<R> *cc = om + G * C;                                        // [C] column constants
    const int n_c = A.n_c;
    fill_twiddles<R>(TW, G, 0, 0);
    // the tile holds clock index s = (o << G) | l; bit b of s carries F[j][n_c-1-b].
    // The G Hadamards below omit their 1/sqrt(2): 2^(-G/2) joins the amplitude scale.
    const double sc = A.scale * exp2(-0.5 * G);
    for (int c = threadIdx.x; c < C; c += NT) {
        const uint64_t j = j0 + c;
        uint64_t th = 0;
        for (int b = G; b < n_c; ++b)
            if (o >> (b - G) & 1) th += F[j * n_c + (n_c - 1 - b)];
        const cvec<R> ph = turn_phase<R>(th);
        const double2 bj = gld<double>(beta, j);
        cc[c] = cmul<R>(cmake<R>((R)(bj.x * sc), (R)(bj.y * sc)), ph);
        for (int b = 0; b < G; ++b) om[b * C + c] = turn_phase<R>(F[j * n_c + (n_c - 1 - b)]);
    }
    // the clock-bit phases of every column for k_pipe_b and k_pipe_c, staged in
    // clock rows 2^g1 + r (r < n_c) of the ancilla = 0 half, which the solve
    // leaves unused otherwise (only the rows below 2^g1 hold the G1 table):
    // row 2^g1 + r holds G2 bit r for r < g2 and G1 bit r - g2 after that
    const int g2 = n_c - G;
    for (int e = threadIdx.x; e < n_c * C; e += NT) {
        const int r = e / C, c = e - r * C;
        const uint64_t j = j0 + c;
        const int q = r < g2 ? n_c - 1 - (G + r) : n_c - 1 - (r - g2);
        gst<R>(psi, ((((uint64_t)1 << G) + (uint64_t)r) << A.n_s) + j, turn_phase<R>(F[j * n_c + q]));
    }
    __syncthreads();
    // phase A: line = (c, l_hi), register index = bits [0, RA)
    const int nla = C << RB;
    for (int line = threadIdx.x; line < nla; line += NT) {
        const int c = line & (C - 1), lhi = line >> A.cl;
        cvec<R> v[1 << RA];
        cvec<R> base = cc[c];
        for (int b = 0; b < RB; ++b)
            if (lhi >> b & 1) base = cmul<R>(base, om[(RA + b) * C + c]);
        v[0] = base;
#pragma unroll
        for (int b = 0; b < RA; ++b) {
            const cvec<R> w = om[b * C + c];
#pragma unroll
            for (int k = 0; k < (1 << b); ++k) v[k | (1 << b)] = cmul<R>(v[k], w);
        }
#pragma unroll
        for (int jb = 0; jb < RA; ++jb)
            stage<R, RA, true>(v, jb, TW + tw_off(jb), jb > 0, [&](int k) { return k & ((1 << jb) - 1); });
        cvec<R> *lt = tile + ((lhi << RA) << A.cl) + c;
#pragma unroll
        for (int k = 0; k < (1 << RA); ++k) lt[k << A.cl] = v[k];
    }
    __syncthreads();
    // phase B: line = (c, l_lo), register index = bits [RA, G)
    const int nlb = C << RA;
    for (int line = threadIdx.x; line < nlb; line += NT) {
        const int c = line & (C - 1), llo = line >> A.cl;
        cvec<R> v[1 << RB];
        cvec<R> *lt = tile + (llo << A.cl) + c;
#pragma unroll
        for (int k = 0; k < (1 << RB); ++k) v[k] = lt[(k << RA) << A.cl];
#pragma unroll
        for (int jb = RA; jb < G; ++jb)
            stage<R, RB, true>(v, jb - RA, TW + tw_off(jb), true,
                               [&](int k) { return llo + ((k & ((1 << (jb - RA)) - 1)) << RA); });
        // clock index (o << G) + (k << RA) + llo: a base for the line and a stride for k
        cvec<R> *p = psi + (((((o << G) + (uint64_t)llo) << A.n_s)) + j0 + c);
        const uint64_t ks = 1ull << (RA + A.n_s);
#pragma unroll
        for (int k = 0; k < (1 << RB); ++k) gst<R>(p, k * ks, v[k]);
    }
}

template <typename R, int RA, int RB, int NT>
__global__ __launch_bounds__(NT) void k_pipe_a(PipeArgs A, PipeSolve one, const PipeSolve *__restrict__ many) {
    uint64_t j0, o;
    tile_coords(A, j0, o);
    pipe_a_body<R, RA, RB, NT>(A, solve_of(one, many), j0, o);
}

// ---------------------------------------------------------------------------
// k_pipe_b: inverse cascade on G2 and the inversion rotation
// ---------------------------------------------------------------------------
// Writes the state after the rotation (the ancilla = 1 half), as
// 2^-G2 s_y a(y): the forward cascade of the uncompute that follows is left
// to k_pipe_c, which needs only its projection.  In the half the clock's two
// groups trade places: clock value y1 + (y2 << g1) is row y2 + (y1 << g2), so
// the rows of a tile (one G1 value) form one block of 2^g2 rows, which
// streams faster than rows 2^g1 apart (a relabelling of the clock qubits in
// memory; both kernels use it).  Tile: columns [j0, j0 + C)
// at G1 value o; a work-queue item (PERS) runs A.iters column blocks j0 + it 2^(pslog + cl).
// The FP64 partial pair goes to slot `slot`.
template <typename R, int RA, int RB, int NT, bool PERS>
__device__ __forceinline__ void pipe_b_body(const PipeArgs &A, const PipeSolve &S, uint64_t j0, uint64_t o,
                                            uint64_t slot) {
    constexpr int G = RA + RB;
    cvec<R> *__restrict__ psi = (cvec<R> *)S.psi;
    const gptr<double> __restrict__ part = (gptr<double>)S.part;
    extern __shared__ unsigned char smem_raw[];
    const int C = 1 << A.cl;
    cvec<R> *TW = reinterpret_cast<cvec<R> *>(smem_raw);            // [2^G] twiddles of G2 at G1 value o
    R *s2t = reinterpret_cast<R *>(TW + (1 << G));                  // [2^G] s_y^2 2^-G
    R *srt = s2t + (1 << G);                                         // [2^G] s_y 2^-G
    // two sets (alternate tiles) of the column data: om[G][C] the phases of
    // the G2 bits (staged by k_pipe_a in clock rows 2^g1 + b), then tT[C] the
    // G1 table entries T_j(o)
    const int ncd = (G + 1) * C;
    cvec<R> *cd = reinterpret_cast<cvec<R> *>(srt + (1 << G));
    __shared__ double red[2][NT / 64];
    const int iters = PERS ? A.iters : 1;
    const uint64_t jstep = PERS ? 1ull << (A.pslog + A.cl) : 0;
    const int g1 = A.g1, n_c = A.n_c;
    auto col_data = [&](int e, uint64_t j) -> cvec<R> {
        const int b = e / C, cq = e - b * C;
        return b < G ? gld<R>(psi, ((((uint64_t)1 << g1) + (uint64_t)b) << A.n_s) + j + cq)
                     : gld<R>(psi, (o << A.n_s) | (j + cq));
    };
    // read before the twiddles are built, so that their latency overlaps that work
    for (int e = threadIdx.x; e < ncd; e += NT) cd[e] = col_data(e, j0);
    fill_twiddles<R>(TW, G, g1, o);
    // rotation of clock value y = o + l 2^g1 (natural order after the inverse
    // transform): sin = 1/y (y >= 1).  The G Hadamards of the inverse cascade
    // and the G of the forward one omit their 1/sqrt(2) each, so 2^-G is
    // folded into the rotation (and into the FP64 weights of the sums, taken
    // where the amplitudes are 2^(G/2) too large).
    const double fold = exp2(-(double)G);
    for (int l = threadIdx.x; l < (1 << G); l += NT) {
        const uint64_t y = o | ((uint64_t)l << g1);
        const double ys = (A.sgn && (y >> (n_c - 1))) ? (double)y - exp2((double)n_c) : (double)y;
        const double sd = !y ? 0.0 : A.gcut ? (fabs(ys) >= (double)A.gcut ? 1.0 : 0.0) : 1.0 / ys;
        s2t[l] = (R)(sd * sd * fold);
        srt[l] = (R)(sd * fold);
    }
    __syncthreads();
    const int nl = C << RA;
    // clock value o + (l << g1), l = llo + (k << RA), is row l + (o << g2) of
    // the half: a base for the line and a stride for k
    const uint64_t ks = 1ull << (RA + A.n_s);
    double pa = 0.0, nt = 0.0;
    for (int it = 0; it < iters; ++it) {
        const bool more = PERS && it + 1 < iters;
        const cvec<R> *om = cd + (it & 1) * ncd, *tT = om + G * C;
        // the inverse-QFT output on the G2 register of column j at
        // y = o + l 2^g1, l = llo + (k << RA), from its closed form.  The
        // input of the G2 stages is T_j(o) times a product state over the G2
        // bits (phase w_b on bit b), and inverse stage b maps a product state
        // to a product state: after all of them the amplitude is
        //   T_j(o) prod_b (1 + (-1)^(l_b) w_b conj(tw_b(l mod 2^b))),
        // tw_b the stage's twiddle.  The factors of the low RA bits are the
        // line's, those of the RB high bits branch into the line's 2^RB
        // entries (a product tree, one level per bit).
        for (int line = threadIdx.x; line < nl; line += NT) {
            int c = line & (C - 1), llo = line >> A.cl;
            // a wavefront takes 16 columns of four lines, so that each store
            // instruction writes four rows of 128 B: that pattern streams
            // faster than one row of 512 B
            if (RA >= 2 && A.cl >= 4) {
                const int wv = line >> 6;
                c = (line & 15) | ((wv & ((1 << (A.cl - 4)) - 1)) << 4);
                llo = ((line >> 4) & 3) | ((wv >> (A.cl - 4)) << 2);
            }
            cvec<R> v[1 << RB];
            cvec<R> p = tT[c];
#pragma unroll
            for (int b = 0; b < RA; ++b) {
                const cvec<R> q = cconjmul<R>(om[b * C + c], TW[tw_off(b) + (llo & ((1 << b) - 1))]);
                const cvec<R> f = (llo >> b & 1) ? cmake<R>((R)1 - q.x, -q.y) : cmake<R>((R)1 + q.x, q.y);
                p = cmul<R>(p, f);
            }
            v[0] = p;
#pragma unroll
            for (int bb = 0; bb < RB; ++bb) {
                const cvec<R> w = om[(RA + bb) * C + c];
#pragma unroll
                for (int m = 0; m < (1 << bb); ++m) {
                    const cvec<R> q = cconjmul<R>(w, TW[tw_off(RA + bb) + llo + (m << RA)]);
                    const cvec<R> a = v[m];
                    v[m] = cmul<R>(a, cmake<R>((R)1 + q.x, q.y));
                    v[m + (1 << bb)] = cmul<R>(a, cmake<R>((R)1 - q.x, -q.y));
                }
            }
            // |a|^2 summed over the line in the amplitude precision (weighted by
            // s_y^2 for P(a = 1); the rotation keeps each pair's norm, so the
            // total is the plain sum), then accumulated in FP64
            R lpa = 0, lnt = 0;
            const R *s2l = s2t + llo, *srl = srt + llo;
            cvec<R> *ps = psi + (A.abit + (((uint64_t)llo + (o << G)) << A.n_s) + j0 + c);
#pragma unroll
            for (int k = 0; k < (1 << RB); ++k) {
                const R a2 = v[k].x * v[k].x + v[k].y * v[k].y;
                lpa += s2l[k << RA] * a2;
                lnt += a2;
                const R sr = srl[k << RA];
                gst_nt<R>(ps, k * ks, cmake<R>(v[k].x * sr, v[k].y * sr));
            }
            pa += (double)lpa;
            nt += (double)lnt * fold;
        }
        // an item's run: the next tile's column data go to the other set, last
        // read in the previous tile (before the last barrier).  (Reading them
        // into registers during the tile cost the work-queue kernel more in
        // spills than it hid.)
        if (more) {
            cvec<R> *nxt = cd + ((it + 1) & 1) * ncd;
            for (int e = threadIdx.x; e < ncd; e += NT) nxt[e] = col_data(e, j0 + jstep);
            __syncthreads();
        }
        j0 += jstep;
    }
    pa = wave_sum_f64(pa);
    nt = wave_sum_f64(nt);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = pa;
        red[1][threadIdx.x >> 6] = nt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sp = 0.0, sn = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
            sp += red[0][w];
            sn += red[1][w];
        }
        part[2 * slot] = sp;
        part[2 * slot + 1] = sn;
    }
}

template <typename R, int RA, int RB, int NT>
__global__ __launch_bounds__(NT) void k_pipe_b(PipeArgs A, PipeSolve one, const PipeSolve *__restrict__ many) {
    uint64_t j0, o;
    tile_coords(A, j0, o);               // o = value of the G1 bits
    pipe_b_body<R, RA, RB, NT, false>(A, solve_of(one, many), j0, o,
                                      (uint64_t)blockIdx.x + (uint64_t)blockIdx.y * gridDim.x);
}


// ---------------------------------------------------------------------------
// k_pipe_c: forward cascade on the clock, conjugate phases, clock sum
// (the missing 2^(-G/2) of the G1 Hadamards is applied with the final scale)
// ---------------------------------------------------------------------------
// Only the clock sum of each transformed column is needed,
//   z = sum_y ph(y) (F v)(y),
// F the forward cascade on the whole clock (the QFT of the uncompute, from
// the top bit down) and ph(y) = prod_b om_b^(y_b) the conjugate phases of
// the controlled powers, a product over the clock bits.  Moved onto the
// input, z = sum_y v(y) K(y) with K the transposed cascade applied to ph.  A
// transposed stage on bit b maps the pair (p0, p1) to (p0 + t p1, p0 - t p1),
// t = exp(2 pi i (y mod 2^b) / 2^(b+1)) its twiddle; run from bit 0 upwards
// on a product state it leaves
//   K(y) = prod_b (1 + (-1)^(y_b) t_b(y mod 2^b) om_b),
// so no transform is formed.  A thread takes a line: one column, one value lo
// of the clock bits below L = n_c - RB, the 2^RB values of the top RB bits.
// It contracts the line from its top bit down, each step halving it,
//   u(m) = (v(m) + v(m + h)) + q (v(m) - v(m + h)),  q = t_b(lo + m 2^L) om_b,
// and multiplies what is left by the factors of the bits below L.  With
// lo = llo + (o << RA): the tile is columns [j0, j0 + C) at o (< 2^g2), its
// lines the 2^RA values llo; a work-queue item (PERS) runs A.iters column
// blocks j0 + it 2^(pslog + cl).  The threads exchange only the column sums.
// cos(2 pi k / 32) and sin(2 pi k / 32): the roots of the line bits in
// k_pipe_c (RB <= 5), folded into the code as constants
__device__ constexpr double cos32(int k) {
    // cos(j pi / 16), j = 0..8
    constexpr double c[9] = {1.0,
                             0.98078528040323044913,
                             0.92387953251128675613,
                             0.83146961230254523708,
                             0.70710678118654752440,
                             0.55557023301960222474,
                             0.38268343236508977173,
                             0.19509032201612826785,
                             0.0};
    k &= 31;
    return k <= 8 ? c[k] : k <= 16 ? -c[16 - k] : k <= 24 ? -c[k - 16] : c[32 - k];
}
__device__ constexpr double sin32(int k) { return cos32(k - 8); }

template <typename R, int RA, int RB, int NT, bool PERS>
__device__ __forceinline__ void pipe_c_body(const PipeArgs &A, const PipeSolve &S, uint64_t j0, uint64_t o) {
    constexpr int G = RA + RB;           // = g1
    static_assert(RB <= 5, "the line bits' roots are 32nd roots of unity");
    const cvec<R> *__restrict__ psi = (const cvec<R> *)S.psi;
    double2 *__restrict__ zpart = S.zpart;
    extern __shared__ unsigned char smem_raw[];
    const int C = 1 << A.cl;
    const int n_c = A.n_c, g2 = n_c - G, L = n_c - RB;
    // LDS: the twiddles of the low bits t_b(x) (b < RA), per o the twiddles
    // of the bits [RA, L) and the line's base phases exp(2 pi i lo / 2^(b+1))
    // (b >= L), then two sets (alternate tiles) of the column phases
    // om[n_c][C] and of the threads' partial sums
    cvec<R> *TWa = reinterpret_cast<cvec<R> *>(smem_raw);           // [2^RA]
    cvec<R> *T2 = TWa + (1 << RA);                                   // [g2][2^RA]
    cvec<R> *T3 = T2 + (g2 << RA);                                   // [RB][2^RA]
    const int nph = n_c * C;
    cvec<R> *phs = T3 + (RB << RA);                                  // [2][n_c][C]
    const size_t zoff = (((size_t)((unsigned char *)(phs + 2 * nph) - smem_raw)) + 15) & ~(size_t)15;
    double2 *zs = reinterpret_cast<double2 *>(smem_raw + zoff);      // [2][NT]
    const int iters = PERS ? A.iters : 1;
    const uint64_t jstep = PERS ? 1ull << (A.pslog + A.cl) : 0;
    const int nl = C << RA;
    // every line of a thread has the thread's column (the line stride NT is a multiple of C)
    const int c = threadIdx.x & (C - 1);
    // clock value y = lo + (k << L) is row (y >> g1) + ((y mod 2^g1) << g2) of
    // the half (k_pipe_b's layout); k's bits lie above g1, so a line is a
    // base row and a stride for k
    const uint64_t ks = 1ull << (L - G + A.n_s);
    // conjugate phase of clock bit b (= e / C) of the column at j: staged by
    // k_pipe_a in clock row 2^g1 + g2 + b (G1 bits) or 2^g1 + b - g1 (G2
    // bits) of the ancilla = 0 half
    auto col_phase = [&](int e, uint64_t j) -> cvec<R> {
        const int b = e / C, cq = e - b * C;
        const int r = b < G ? g2 + b : b - G;
        const cvec<R> w = gld<R>(psi, ((((uint64_t)1 << G) + (uint64_t)r) << A.n_s) + j + cq);
        return cmake<R>(w.x, -w.y);
    };
    for (int e = threadIdx.x; e < nph; e += NT) phs[e] = col_phase(e, j0);
    fill_twiddles<R>(TWa, RA, 0, 0);
    for (int e = threadIdx.x; e < ((g2 + RB) << RA); e += NT) {
        const int i = e >> RA, llo = e & ((1 << RA) - 1);
        if (i < g2) {
            // bit b = RA + i: t_b(lo mod 2^b), lo mod 2^b = llo + ((o mod 2^i) << RA)
            const int b = RA + i;
            const uint64_t x = (uint64_t)llo + ((o & ((1ull << i) - 1)) << RA);
            T2[e] = turn_phase<R>(x << (63 - b));
        } else {
            // bit b = L + kb: exp(2 pi i lo / 2^(b+1))
            const int b = L + (i - g2);
            T3[((i - g2) << RA) + llo] = turn_phase<R>(((uint64_t)llo + (o << RA)) << (63 - b));
        }
    }
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        const bool more = PERS && it + 1 < iters;
        const cvec<R> *om = phs + (it & 1) * nph;
        // lines are read where they are used: lines held in registers across
        // the table set-up or the previous tile cost more in occupancy than
        // they hide
        double zr = 0.0, zi = 0.0;
        for (int line = threadIdx.x; line < nl; line += NT) {
            const int llo = line >> A.cl;
            cvec<R> v[1 << RB];
            const uint64_t y = (o << RA) + (uint64_t)llo;
            const uint64_t row = (y >> G) + ((y & ((1ull << G) - 1)) << g2);
            const cvec<R> *p = psi + (A.abit + (row << A.n_s) + j0 + c);
#pragma unroll
            for (int k = 0; k < (1 << RB); ++k) v[k] = gld_nt<R>(p, k * ks);
            // the line's bits, top first: q = om_b exp(2 pi i lo / 2^(b+1)) times
            // the root exp(2 pi i m / 2^(kb+1)) of the line bits below
#pragma unroll
            for (int kb = RB - 1; kb >= 0; --kb) {
                const int h = 1 << kb;
                const cvec<R> Q = cmul<R>(om[(L + kb) * C + c], T3[(kb << RA) + llo]);
#pragma unroll
                for (int m = 0; m < h; ++m) {
                    const int r = m << (4 - kb);
                    const cvec<R> q = r == 0   ? Q
                                      : r == 8 ? cmake<R>(-Q.y, Q.x)
                                               : cmul<R>(Q, cmake<R>((R)cos32(r), (R)sin32(r)));
                    const cvec<R> a = v[m], b = v[m + h];
                    const R sx = a.x + b.x, sy = a.y + b.y, dx = a.x - b.x, dy = a.y - b.y;
                    v[m] = cmake<R>(ffma(q.x, dx, ffma(-q.y, dy, sx)), ffma(q.x, dy, ffma(q.y, dx, sy)));
                }
            }
            // the factors of the bits below L: the low RA bits (bit 0: twiddle
            // 1), then the g2 bits of o
            cvec<R> f = cmake<R>((R)1, (R)0);
#pragma unroll
            for (int b = 0; b < RA; ++b) {
                const cvec<R> w = om[b * C + c];
                const cvec<R> q = b == 0 ? w : cmul<R>(w, TWa[tw_off(b) + (llo & ((1 << b) - 1))]);
                f = cmul<R>(f, (llo >> b & 1) ? cmake<R>((R)1 - q.x, -q.y) : cmake<R>((R)1 + q.x, q.y));
            }
            for (int i = 0; i < g2; ++i) {
                const cvec<R> q = cmul<R>(om[(RA + i) * C + c], T2[(i << RA) + llo]);
                f = cmul<R>(f, (o >> i & 1) ? cmake<R>((R)1 - q.x, -q.y) : cmake<R>((R)1 + q.x, q.y));
            }
            const cvec<R> u = cmul<R>(v[0], f);
            zr += (double)u.x;
            zi += (double)u.y;
        }
        // an item's run: the next tile's phases go to the other set, last read
        // in the previous tile (before the last barrier)
        if (more) {
            cvec<R> *nxt = phs + ((it + 1) & 1) * nph;
            for (int e = threadIdx.x; e < nph; e += NT) nxt[e] = col_phase(e, j0 + jstep);
        }
        double2 *zt = zs + (it & 1) * NT;
        zt[threadIdx.x] = make_double2(zr, zi);
        __syncthreads();
        for (int cq = threadIdx.x; cq < C; cq += NT) {
            double r = 0.0, i = 0.0;
            for (int t = cq; t < NT; t += C) {
                r += zt[t].x;
                i += zt[t].y;
            }
            gst<double>(zpart, o * A.N + j0 + cq, make_double2(r, i));
        }
        j0 += jstep;
    }
}

template <typename R, int RA, int RB, int NT>
__global__ __launch_bounds__(NT) void k_pipe_c(PipeArgs A, PipeSolve one, const PipeSolve *__restrict__ many) {
    uint64_t j0, o;
    tile_coords(A, j0, o);               // o = value of the G2 bits
    pipe_c_body<R, RA, RB, NT, false>(A, solve_of(one, many), j0, o);
}


// ---------------------------------------------------------------------------
// a batch as one persistent kernel over device work queues
// ---------------------------------------------------------------------------
struct QClass {
    PipeArgs A[3];            // launch parameters of the three kernels' items
    int g[3];                 // the group each transforms: g1, g2, g1
    uint32_t per_o[3];        // items per value of the other clock group
};
struct QSolve {
    PipeSolve S;
    uint32_t cls;
    uint32_t items[3];        // items of the three kernels (the finish waits for the last)
};
constexpr int kMaxQueues = 8;
struct QueueArgs {
    const QClass *cls;
    const QSolve *solves;
    const uint64_t *items;    // the queues' item codes, queue after queue
    const FinishJob *fin;
    unsigned *cnt;            // [3 nsolves] done counters, [kMaxQueues] heads, finished solves
    unsigned *flag;
    uint64_t wait_ticks;      // bound of one dependency wait, in wall-clock ticks
    uint32_t nsolves;
    int local;                // 1: one queue per XCC, served by that XCC's blocks; 0: one queue for all
                              // blocks, with device-scope synchronisation
    uint32_t qstart[kMaxQueues + 1];
    int qof[16];              // local: the queue of every XCC id (-1: none)
};

// the accelerator complex die (its own L2) the wave runs on
__device__ __forceinline__ int xcc_id() { return (int)(__builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) & 15u); }

// Wait for *c >= target, bounded by `ticks` of the constant-rate wall clock
// (a quarter second): on expiry the flag is set and the item runs anyway,
// and once the flag is set no wait blocks any more, so every block drains.
// Then the acquire: a queue served by one XCC shares that XCC's L2 with its
// producers, so only the CU's vector L1 is invalidated (a line there may
// hold data another phase has since rewritten); otherwise the device-scope
// acquire (L1 and the XCC's L2).  The block barrier follows.
__device__ __forceinline__ void queue_wait(unsigned *c, unsigned target, unsigned *flag, uint64_t ticks, bool local) {
    if (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (wall_clock64() - t0 > ticks) {
                __hip_atomic_fetch_or(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    if (local) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        asm volatile("buffer_inv sc0" ::: "memory");
    } else {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
}

template <typename R, int G>
__device__ __forceinline__ void queue_item(int ph, const PipeArgs &A, const PipeSolve &S, uint64_t j0, uint64_t o,
                                           uint64_t slot) {
    constexpr int RA = (G + 1) / 2, RB = G / 2;     // the register split of dispatch_g
    if (ph == 0)
        pipe_a_body<R, RA, RB, 256>(A, S, j0, o);
    else if (ph == 1)
        pipe_b_body<R, RA, RB, 256, true>(A, S, j0, o, slot);
    else
        pipe_c_body<R, RA, RB, 256, true>(A, S, j0, o);
}

// Every block serves one queue and takes its items from the queue's head
// until it is empty; the next item's code and the position of the one after
// it are fetched while the current one runs.  An item code holds the phase (bits 62-63: 0-2 the three
// kernels, 3 the finish), the solve (bits 42-61), the number of items of the
// previous phase of the solve that it waits for (bits 21-41) and the item's
// index within its phase of the solve (bits 0-20).  With one queue per XCC, a block reads the XCC it runs on and
// serves that XCC's queue: every producer and consumer of a solve then
// share one L2, and no L2 write-back or invalidation is needed (the XCCs
// present are probed when the queues are built; dispatch spreads the
// blocks of a launch over all of them, from a starting XCC that varies
// between launches).  GMAX bounds the clock groups of the batch: the registers of
// a kernel are those of its widest group, so batches of groups <= 6 bits
// get a form without the 7- and 8-bit bodies, held to four waves per SIMD
// for complex64 (128 VGPRs, a few spilled) and two for complex128 (256).
template <typename R, int GMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GMAX == 6 ? (sizeof(R) == 4 ? 4 : 2) : 1))) void
k_pipe_queue(QueueArgs Q) {
    __shared__ uint64_t sh_code;
    const bool local = Q.local != 0;
    const int q = local ? Q.qof[xcc_id()] : 0;
    if (q < 0) return;
    unsigned *const head = Q.cnt + 3 * (size_t)Q.nsolves + q;
    unsigned *const finished = Q.cnt + 3 * (size_t)Q.nsolves + kMaxQueues;
    const uint32_t base = Q.qstart[q], nitems = Q.qstart[q + 1] - base;
    // thread 0: the code of the block's next item (~0: none left) and the
    // queue position of the one after, both in flight during an item
    uint64_t next_code = ~0ull;
    uint32_t pend = 0;
    if (threadIdx.x == 0) {
        const uint32_t i = __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (i < nitems) next_code = Q.items[base + i];
        pend = i < nitems ? __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : nitems;
    }
    for (;;) {
        if (threadIdx.x == 0) {
            const uint64_t code = next_code;
            if (code != ~0ull) {
                next_code = pend < nitems ? Q.items[base + pend] : ~0ull;
                if (pend < nitems) pend = __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned ph = (unsigned)(code >> 62), sv = (unsigned)(code >> 42) & 0xFFFFFu;
                if (ph > 0)
                    queue_wait(Q.cnt + 3 * (size_t)sv + ph - 1, (unsigned)(code >> 21) & 0x1FFFFFu, Q.flag,
                               Q.wait_ticks, local);
            }
            sh_code = code;
        }
        // also the barrier between the last item's LDS reads and this one's writes
        __syncthreads();
        const uint64_t code = sh_code;
        if (code == ~0ull) break;
        const int ph = (int)(code >> 62);
        const uint32_t sv = (uint32_t)(code >> 42) & 0xFFFFFu;
        const uint64_t t = code & 0x1FFFFFu;
        if (ph == 3) {
            batch_finish_body(Q.fin[sv]);
            if (threadIdx.x == 0) __hip_atomic_fetch_add(finished, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        const QSolve &qs = Q.solves[sv];
        const QClass &c = Q.cls[qs.cls];
        const PipeArgs A = c.A[ph];
        const PipeSolve S = qs.S;
        const uint64_t per = c.per_o[ph];
        const uint64_t o = t / per;
        const uint64_t j0 = ((t - o * per) * (uint64_t)A.iters) << A.cl;
        switch (c.g[ph]) {
        case 1: queue_item<R, 1>(ph, A, S, j0, o, t); break;
        case 2: queue_item<R, 2>(ph, A, S, j0, o, t); break;
        case 3: queue_item<R, 3>(ph, A, S, j0, o, t); break;
        case 4: queue_item<R, 4>(ph, A, S, j0, o, t); break;
        case 5: queue_item<R, 5>(ph, A, S, j0, o, t); break;
        case 6: queue_item<R, 6>(ph, A, S, j0, o, t); break;
        case 7:
            if (GMAX >= 7) queue_item<R, 7>(ph, A, S, j0, o, t);
            break;
        default:
            if (GMAX >= 8) queue_item<R, 8>(ph, A, S, j0, o, t);
            break;
        }
        // publish the item: every wave's stores complete (the block barrier
        // alone waits for LDS traffic only): in the XCC's L2 for a local
        // queue, else released at device scope; then one thread counts it
        if (local) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_s_waitcnt(0);
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(Q.cnt + 3 * (size_t)sv + ph, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// the XCC of every block of a grid (one wave per block)
__global__ void k_xcc_probe(int *__restrict__ out) {
    if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------

template <typename R, int RA, int RB, int NT>
static sv_status launch_pipe(int which, hipStream_t st, const PipeSolve &one, const PipeSolve *many,
                             const PipeArgs &A, dim3 grid, size_t lds) {
    // tiles above 64 KiB need a larger dynamic LDS limit; the request plus the
    // kernels' static LDS must stay within the 160 KiB of a workgroup
    constexpr int kLim = 144 * 1024;
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e0 = hipFuncSetAttribute((const void *)k_pipe_a<R, RA, RB, NT>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, kLim);
        hipError_t e1 = hipFuncSetAttribute((const void *)k_pipe_b<R, RA, RB, NT>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, kLim);
        hipError_t e2 = hipFuncSetAttribute((const void *)k_pipe_c<R, RA, RB, NT>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, kLim);
        (void)hipGetLastError();
        if (e0 != hipSuccess || e1 != hipSuccess || e2 != hipSuccess)
            return fail(SV_EDEVICE, "cannot raise the LDS limit of the pipeline kernels");
        attr_done = true;
    }
    if (lds > (size_t)kLim) return fail(SV_EUNSUPPORTED, "pipeline tile needs %zu bytes of LDS", lds);
    // algorithmic bytes: the ancilla half is 2^(n_s + n_c) amplitudes; the G1
    // table 2^(n_s + g1)
    const double half = (double)A.N * (double)(1ull << A.n_c) * sizeof(cvec<R>) * grid.z;
    const double table = (double)A.N * (double)(1ull << A.g1) * sizeof(cvec<R>) * grid.z;
    if (which == 0) {
        TraceScope ts(st, "pipe_a_init_iqft", table, 0.0);
        hipLaunchKernelGGL((k_pipe_a<R, RA, RB, NT>), grid, dim3(NT), lds, st, A, one, many);
    } else if (which == 1) {
        TraceScope ts(st, "pipe_b_iqft_ry", half + table, 0.0);
        hipLaunchKernelGGL((k_pipe_b<R, RA, RB, NT>), grid, dim3(NT), lds, st, A, one, many);
    } else {
        TraceScope ts(st, "pipe_c_qft_project", half, 0.0);
        hipLaunchKernelGGL((k_pipe_c<R, RA, RB, NT>), grid, dim3(NT), lds, st, A, one, many);
    }
    SV_HIP(hipGetLastError());
    return SV_OK;
}

template <typename R, int RA, int RB>
static sv_status launch_nt(int which, hipStream_t st, const PipeSolve &one, const PipeSolve *many,
                           const PipeArgs &A, int nt, dim3 grid, size_t lds) {
    if (nt == 512) return launch_pipe<R, RA, RB, 512>(which, st, one, many, A, grid, lds);
    return launch_pipe<R, RA, RB, 256>(which, st, one, many, A, grid, lds);
}

template <typename R>
static sv_status dispatch_g(int which, hipStream_t st, const PipeSolve &one, const PipeSolve *many,
                            const PipeArgs &A, int g, int nt, dim3 grid, size_t lds) {
    switch (g) {
    case 1: return launch_nt<R, 1, 0>(which, st, one, many, A, nt, grid, lds);
    case 2: return launch_nt<R, 1, 1>(which, st, one, many, A, nt, grid, lds);
    case 3: return launch_nt<R, 2, 1>(which, st, one, many, A, nt, grid, lds);
    case 4: return launch_nt<R, 2, 2>(which, st, one, many, A, nt, grid, lds);
    case 5: return launch_nt<R, 3, 2>(which, st, one, many, A, nt, grid, lds);
    case 6: return launch_nt<R, 3, 3>(which, st, one, many, A, nt, grid, lds);
    case 7: return launch_nt<R, 4, 3>(which, st, one, many, A, nt, grid, lds);
    case 8: return launch_nt<R, 4, 4>(which, st, one, many, A, nt, grid, lds);
    case 9: return launch_nt<R, 5, 4>(which, st, one, many, A, nt, grid, lds);
    case 10: return launch_nt<R, 5, 5>(which, st, one, many, A, nt, grid, lds);
    }
    return fail(SV_EUNSUPPORTED, "clock group of %d bits", g);
}

int pipe_supported(int n_s, int n_c) { return n_c >= 2 && n_c <= 20 && n_s >= 0; }

static const int PIPE_LDS_LIMIT = 144 * 1024;

// columns per tile for a group of g bits by default (tile of at most 2^13
// c64 / 2^12 c128 amplitudes)
static int default_cl(int n_s, int g, size_t elem) {
    const int tile_log = elem == 8 ? 13 : 12;
    int cl = tile_log - g;
    if (cl > 6) cl = 6;
    if (cl > n_s) cl = n_s;
    if (cl < 0) cl = 0;
    return cl;
}

static size_t pipe_lds(int which, int cl, int g, int n_c, size_t e, int nt) {
    const size_t C = (size_t)1 << cl;
    const size_t RA = (size_t)(g + 1) / 2, RB = (size_t)g / 2, g2 = (size_t)(n_c - g);
    if (which == 0)        // the tile, the twiddles, the column phases and constants
        return ((C << g) + ((size_t)1 << g) + (size_t)(g + 1) * C) * e;
    if (which == 1)        // the twiddles, two rotation tables, two sets of column data
        return ((size_t)1 << g) * e + 2 * ((size_t)1 << g) * (e / 2) + 2 * (size_t)(g + 1) * C * e;
    // k_pipe_c: the twiddle tables, two sets of column phases and of partial sums
    return (((size_t)1 << RA) + ((g2 + RB) << RA) + 2 * (size_t)n_c * C) * e + 2 * (size_t)nt * sizeof(double2) + 16;
}

struct PipePlan {
    PipeArgs A[3];
    int nt[3];
    dim3 grid[3];
    size_t lds[3];
};

static void make_plan(PipePlan &P, int n_s, int n_c, size_t e, const int cl[3], const int nt[3], int nsolves) {
    PipeArgs A;
    A.N = dim_of(n_s);
    A.n_s = n_s;
    A.n_c = n_c;
    A.g1 = (n_c + 1) / 2;
    A.g2 = n_c - A.g1;
    A.abit = 1ull << (n_s + n_c);
    A.scale = 1.0 / sqrt((double)(1ull << n_c));
    A.sgn = 0;
    A.gcut = 0;
    A.pslog = 0;
    A.iters = 1;
    for (int w = 0; w < 3; ++w) {
        const int g = w == 1 ? A.g2 : A.g1;
        P.A[w] = A;
        P.A[w].cl = cl[w];
        P.nt[w] = nt[w];
        // k_pipe_a writes the G1 table only (G2 value 0)
        const uint64_t tiles = w == 0 ? (A.N >> cl[w]) : (A.N >> cl[w]) << (n_c - g);
        P.grid[w] = tiles <= 0x7fffffffull ? dim3((unsigned)tiles, 1, nsolves)
                                           : dim3(1u << 30, (unsigned)(tiles >> 30), nsolves);
        P.lds[w] = pipe_lds(w, cl[w], g, n_c, e, nt[w]);
    }
}

template <typename R>
static sv_status run_one(hipStream_t st, const PipePlan &P, int w, const PipeSolve &one, const PipeSolve *many) {
    const int g = w == 1 ? P.A[w].g2 : P.A[w].g1;
    return dispatch_g<R>(w, st, one, many, P.A[w], g, P.nt[w], P.grid[w], P.lds[w]);
}

// The autotuner: per (dtype, n_s, n_c) time every feasible (columns per
// tile, threads per workgroup) for each of the three kernels on the real
// operands of one solve (each kernel is idempotent given its input half)
// and keep the fastest; results live in the process-wide tuning cache.
template <typename R>
static sv_status tune_pipe(hipStream_t st, int n_s, int n_c, const PipeSolve &one, int cl_out[3],
                           int nt_out[3]) {
    const size_t e = sizeof(cvec<R>);
    const int g1 = (n_c + 1) / 2, g2 = n_c - g1;
    for (int w = 0; w < 3; ++w) {
        cl_out[w] = default_cl(n_s, w == 1 ? g2 : g1, e);
        nt_out[w] = 256;
    }
    for (int w = 0; w < 3; ++w) {
        const int g = w == 1 ? g2 : g1;
        // up to 128 columns: k_pipe_c's loads then cover 1 KiB of a row per
        // instruction (its 64-column tiles read the half about 3 % more slowly).
        // Every candidate is timed in two alternating rounds and keeps its
        // faster one: single timings of a few-millisecond kernel differ by
        // more than the candidates do.
        std::vector<std::pair<int, int>> cand;
        for (int cl = 3; cl <= 7; ++cl) {
            if (cl > n_s) break;
            for (int nt : {256, 512})
                if (pipe_lds(w, cl, g, n_c, e, nt) <= (size_t)PIPE_LDS_LIMIT) cand.push_back({cl, nt});
        }
        std::vector<float> tbest(cand.size(), 1e30f);
        for (int round = 0; round < 2; ++round)
            for (size_t i = 0; i < cand.size(); ++i) {
                int cls[3] = {cl_out[0], cl_out[1], cl_out[2]}, nts[3] = {nt_out[0], nt_out[1], nt_out[2]};
                cls[w] = cand[i].first;
                nts[w] = cand[i].second;
                PipePlan P;
                make_plan(P, n_s, n_c, e, cls, nts, 1);
                float ms = 0.f;
                SV_TRY(time_stream(st, 2, &ms, [&]() { return run_one<R>(st, P, w, one, nullptr); }));
                if (ms < tbest[i]) tbest[i] = ms;
            }
        int bcl = cl_out[w], bnt = nt_out[w];
        float best = 1e30f;
        for (size_t i = 0; i < cand.size(); ++i)
            if (tbest[i] < best) {
                best = tbest[i];
                bcl = cand[i].first;
                bnt = cand[i].second;
            }
        cl_out[w] = bcl;
        nt_out[w] = bnt;
        // the next kernel reads what this one writes: leave its output in place
        PipePlan P;
        make_plan(P, n_s, n_c, e, cl_out, nt_out, 1);
        SV_TRY(run_one<R>(st, P, w, one, nullptr));
    }
    return SV_OK;
}

// launch parameters for a shape: cached, tuned on `one` if allowed, else defaults
template <typename R>
static sv_status pipe_config_impl(hipStream_t st, int n_s, int n_c, const PipeSolve *tune_on, int cl[3],
                                  int nt[3]) {
    const size_t e = sizeof(cvec<R>);
    const int g1 = (n_c + 1) / 2, g2 = n_c - g1;
    const std::string key = std::string("eigpipe/") + (e == 8 ? "c64/" : "c128/") + std::to_string(n_s) + "/" +
                            std::to_string(n_c);
    std::vector<int> cached;
    if (tune_lookup(key, cached) && cached.size() == 6) {
        for (int w = 0; w < 3; ++w) {
            cl[w] = cached[2 * w];
            nt[w] = cached[2 * w + 1];
        }
        return SV_OK;
    }
    if (tune_on && autotune_enabled()) {
        SV_TRY(tune_pipe<R>(st, n_s, n_c, *tune_on, cl, nt));
        tune_store(key, {cl[0], nt[0], cl[1], nt[1], cl[2], nt[2]});
        return SV_OK;
    }
    for (int w = 0; w < 3; ++w) {
        cl[w] = default_cl(n_s, w == 1 ? g2 : g1, e);
        nt[w] = 256;
    }
    return SV_OK;
}

template <typename R>
sv_status pipe_config(hipStream_t st, int n_s, int n_c, const PipeSolve *tune_on, int cl[3], int nt[3]) {
    return pipe_config_impl<R>(st, n_s, n_c, tune_on, cl, nt);
}

template <typename R>
sv_status pipe_run(sv_state s, int n_s, int n_c, bool sgn, uint64_t gcut, const double2 *beta, const uint64_t *F,
                   double *part, double2 *zpart, uint64_t *nparts) {
    const size_t e = sizeof(cvec<R>);
    PipeSolve one{s->data, beta, F, part, zpart};
    int cl[3], nt[3];
    SV_TRY(pipe_config_impl<R>(s->stream, n_s, n_c, &one, cl, nt));
    PipePlan P;
    make_plan(P, n_s, n_c, e, cl, nt, 1);
    for (int w = 0; w < 3; ++w) {
        P.A[w].sgn = sgn ? 1 : 0;
        P.A[w].gcut = gcut;
    }
    *nparts = (uint64_t)P.grid[1].x * P.grid[1].y;
    for (int w = 0; w < 3; ++w) SV_TRY(run_one<R>(s->stream, P, w, one, nullptr));
    return SV_OK;
}
template sv_status pipe_run<float>(sv_state, int, int, bool, uint64_t, const double2 *, const uint64_t *, double *,
                                   double2 *, uint64_t *);
template sv_status pipe_run<double>(sv_state, int, int, bool, uint64_t, const double2 *, const uint64_t *,
                                    double *, double2 *, uint64_t *);

// a class of solves sharing (n_s, n_c): the three kernels once each, blockIdx.z = solve
template <typename R>
sv_status pipe_run_batch(hipStream_t st, int n_s, int n_c, const int cl[3], const int nt[3],
                         const PipeSolve *dev_solves, int nsolves, uint64_t *nparts) {
    const size_t e = sizeof(cvec<R>);
    if (nsolves < 1 || nsolves > 65535) return fail(SV_EINVAL, "batch of %d solves", nsolves);
    PipePlan P;
    make_plan(P, n_s, n_c, e, cl, nt, nsolves);
    *nparts = (uint64_t)P.grid[1].x * P.grid[1].y;
    PipeSolve none{};
    for (int w = 0; w < 3; ++w) SV_TRY(run_one<R>(st, P, w, none, dev_solves));
    return SV_OK;
}
template sv_status pipe_run_batch<float>(hipStream_t, int, int, const int *, const int *, const PipeSolve *, int,
                                         uint64_t *);
template sv_status pipe_run_batch<double>(hipStream_t, int, int, const int *, const int *, const PipeSolve *, int,
                                          uint64_t *);
template sv_status pipe_config<float>(hipStream_t, int, int, const PipeSolve *, int *, int *);
template sv_status pipe_config<double>(hipStream_t, int, int, const PipeSolve *, int *, int *);

// ---------------------------------------------------------------------------
// the work queues' plan: items of about 2^15 amplitudes (runs of consecutive
// column blocks for k_pipe_b and k_pipe_c); the solves spread over one
// queue per XCC, each queue numbered phase-major, its solves largest first
// ---------------------------------------------------------------------------
template <typename R>
sv_status pipe_queue_build(sv_state ctx, hipStream_t st, PipeQueue &q, DevBuf &desc,
                           const std::vector<QueueClassIn> &cls, const std::vector<int> &solve_cls,
                           const std::vector<PipeSolve> &solves, unsigned *cnt, unsigned *flag) {
    (void)st;
    const size_t e = sizeof(cvec<R>);
    const int ns = (int)solves.size();
    if (ns < 1 || ns >= (1 << 20) || solve_cls.size() != solves.size())
        return fail(SV_EINVAL, "work queue of %d solves", ns);
    constexpr int kLim = 144 * 1024;
    static bool attr_done = false;
    if (!attr_done) {
        const hipError_t h6 =
            hipFuncSetAttribute((const void *)k_pipe_queue<R, 6>, hipFuncAttributeMaxDynamicSharedMemorySize, kLim);
        const hipError_t h8 =
            hipFuncSetAttribute((const void *)k_pipe_queue<R, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, kLim);
        (void)hipGetLastError();
        if (h6 != hipSuccess || h8 != hipSuccess) return fail(SV_EDEVICE, "cannot raise the LDS limit of the queue kernel");
        attr_done = true;
    }
    std::vector<QClass> qc(cls.size());
    size_t lds = 0;
    int gmax = 1;
    for (size_t k = 0; k < cls.size(); ++k) {
        const QueueClassIn &ci = cls[k];
        const int nt[3] = {256, 256, 256};
        PipePlan P;
        make_plan(P, ci.n_s, ci.n_c, e, ci.cl, nt, 1);
        for (int w = 0; w < 3; ++w) {
            PipeArgs A = P.A[w];
            const int g = w == 1 ? A.g2 : A.g1;
            // tiles of at most 2^11 amplitudes: LDS for four blocks per CU
            while (A.cl > 0 && ((1ull << A.cl) << g) > (1ull << 11)) --A.cl;
            const uint64_t C = 1ull << A.cl, nb = A.N >> A.cl;
            int iters = 1;
            // a run of column blocks reads each next block's column data ahead
            if (w > 0)
                while ((uint64_t)iters < nb && (((uint64_t)iters * 2 * C) << g) <= (1ull << 15)) iters *= 2;
            A.pslog = 0;
            A.iters = iters;
            qc[k].A[w] = A;
            qc[k].g[w] = g;
            if (g > gmax) gmax = g;
            qc[k].per_o[w] = (uint32_t)(nb / (uint64_t)iters);
            const size_t b = pipe_lds(w, A.cl, g, A.n_c, e, 256);
            if (b > lds) lds = b;
        }
    }
    if (lds > (size_t)kLim) return fail(SV_EUNSUPPORTED, "queue items need %zu bytes of LDS", lds);
    std::vector<QSolve> qs(ns);
    std::vector<double> cost(ns);
    q.nparts.assign(ns, 0);
    double bytes = 0.0;
    for (int k = 0; k < ns; ++k) {
        const QClass &c = qc[solve_cls[k]];
        qs[k].S = solves[k];
        qs[k].cls = (uint32_t)solve_cls[k];
        const int g1 = c.A[0].g1, g2 = c.A[0].g2;
        qs[k].items[0] = c.per_o[0];
        qs[k].items[1] = c.per_o[1] << g1;
        qs[k].items[2] = c.per_o[2] << g2;
        q.nparts[k] = qs[k].items[1];
        if (q.nparts[k] > pipe_b_blocks(c.A[0].n_s, c.A[0].n_c, e))
            return fail(SV_EDEVICE, "queue partials exceed their buffer");
        const double half = (double)c.A[0].N * (double)(1ull << c.A[0].n_c) * e;
        const double table = (double)c.A[0].N * (double)(1ull << g1) * e;
        cost[k] = 2.0 * half + 2.0 * table;
        bytes += cost[k];
    }
    // resident blocks, and the XCC each of them lands on
    // the queue kernel carries bodies for clock groups of up to 8 bits; a
    // batch with wider groups runs its classes' own kernels instead
    if (gmax > 8) return fail(SV_EUNSUPPORTED, "work queue for clock groups of %d bits", gmax);
    q.gmax = gmax <= 6 ? 6 : 8;
    const void *kfn = q.gmax == 6 ? (const void *)k_pipe_queue<R, 6> : (const void *)k_pipe_queue<R, 8>;
    int per_cu = 0, dev = 0, ncu = 0, khz = 0;
    SV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, 256, lds));
    SV_HIP(hipGetDevice(&dev));
    SV_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    SV_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (per_cu < 1) return fail(SV_EUNSUPPORTED, "the queue kernel does not fit a CU with %zu bytes of LDS", lds);
    q.wait_ticks = (uint64_t)(khz > 0 ? khz : 100000) * 250;     // 0.25 s
    q.blocks = per_cu * ncu;
    std::vector<int> ids(q.blocks);
    {
        DevBuf probe;
        SV_TRY(probe.alloc(ids.size() * sizeof(int)));
        hipLaunchKernelGGL(k_xcc_probe, dim3((unsigned)q.blocks), dim3(256), 0, ctx->stream, (int *)probe.p);
        SV_HIP(hipGetLastError());
        SV_TRY(download(ctx, ids.data(), probe.p, ids.size() * sizeof(int)));
    }
    // queues: one per XCC that the probe's blocks landed on (each held an
    // even share of them), else one queue with device-scope synchronisation
    std::vector<int> distinct, count;
    for (int b = 0; b < q.blocks; ++b) {
        const auto it = std::find(distinct.begin(), distinct.end(), ids[b]);
        if (it == distinct.end()) {
            distinct.push_back(ids[b]);
            count.push_back(1);
        } else {
            ++count[it - distinct.begin()];
        }
    }
    const int D = (int)distinct.size();
    // SV_QUEUE_LOCAL=0 forces the single queue with device-scope
    // synchronisation (the fallback), so that it can be tested on any box
    const char *lenv = getenv("SV_QUEUE_LOCAL");
    bool even = D >= 1 && D <= kMaxQueues && !(lenv && atoi(lenv) == 0);
    for (int i = 0; i < D && even; ++i) even = distinct[i] >= 0 && distinct[i] < 16 && count[i] * D >= q.blocks / 2;
    if (even) {
        std::sort(distinct.begin(), distinct.end());
        q.nq = D;
        for (int i = 0; i < D; ++i) q.xcc[i] = distinct[i];
    } else {
        q.nq = 1;
        q.xcc[0] = -1;
    }
    // solves to queues, longest first to the least loaded queue
    std::vector<int> order(ns);
    for (int k = 0; k < ns; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<std::vector<int>> members(q.nq);
    std::vector<double> load(q.nq, 0.0);
    for (int k : order) {
        int best = 0;
        for (int i = 1; i < q.nq; ++i)
            if (load[i] < load[best]) best = i;
        members[best].push_back(k);
        load[best] += cost[k];
    }
    // each queue phase-major, its solves largest first; a code carries the
    // item count its wait targets (that of the solve's previous phase)
    for (int k = 0; k < ns; ++k)
        for (int ph = 0; ph < 3; ++ph)
            if (qs[k].items[ph] >= (1u << 21))
                return fail(SV_EUNSUPPORTED, "%u items in one phase of a solve", qs[k].items[ph]);
    std::vector<uint64_t> items;
    for (int i = 0; i < q.nq; ++i) {
        q.qstart[i] = (uint32_t)items.size();
        for (int ph = 0; ph < 3; ++ph)
            for (int k : members[i]) {
                q.items_per_phase[ph] += qs[k].items[ph];
                const uint64_t wait = ph > 0 ? qs[k].items[ph - 1] : 0;
                for (uint64_t t = 0; t < qs[k].items[ph]; ++t)
                    items.push_back(((uint64_t)ph << 62) | ((uint64_t)k << 42) | (wait << 21) | t);
            }
        for (int k : members[i]) items.push_back((3ull << 62) | ((uint64_t)k << 42) | ((uint64_t)qs[k].items[2] << 21));
        if (items.size() >= 0xffffffffull) return fail(SV_EUNSUPPORTED, "work queue of %zu items", items.size());
    }
    q.qstart[q.nq] = (uint32_t)items.size();
    q.items_per_phase[3] = (uint64_t)ns;
    // descriptors: classes, solves, item codes
    const size_t o_cls = 0, o_sol = (qc.size() * sizeof(QClass) + 255) & ~(size_t)255;
    const size_t o_items = o_sol + ((qs.size() * sizeof(QSolve) + 255) & ~(size_t)255);
    SV_TRY(desc.alloc(o_items + items.size() * sizeof(uint64_t)));
    char *d = (char *)desc.p;
    SV_TRY(upload(ctx, d + o_cls, qc.data(), qc.size() * sizeof(QClass)));
    SV_TRY(upload(ctx, d + o_sol, qs.data(), qs.size() * sizeof(QSolve)));
    SV_TRY(upload(ctx, d + o_items, items.data(), items.size() * sizeof(uint64_t)));
    q.d_cls = d + o_cls;
    q.d_solves = d + o_sol;
    q.d_items = (const uint64_t *)(d + o_items);
    q.nitems = (uint32_t)items.size();
    q.nsolves = (uint32_t)ns;
    q.cnt = cnt;
    q.flag = flag;
    q.lds = lds;
    q.bytes = bytes;
    return SV_OK;
}

template <typename R>
sv_status pipe_queue_launch(hipStream_t st, const PipeQueue &q, const FinishJob *d_fin) {
    QueueArgs Q;
    Q.cls = (const QClass *)q.d_cls;
    Q.solves = (const QSolve *)q.d_solves;
    Q.items = q.d_items;
    Q.fin = d_fin;
    Q.cnt = q.cnt;
    Q.flag = q.flag;
    Q.wait_ticks = q.wait_ticks;
    Q.nsolves = q.nsolves;
    Q.local = q.xcc[0] >= 0 ? 1 : 0;
    for (int i = 0; i <= kMaxQueues; ++i) Q.qstart[i] = i <= q.nq ? q.qstart[i] : q.qstart[q.nq];
    for (int i = 0; i < 16; ++i) Q.qof[i] = -1;
    if (Q.local)
        for (int i = 0; i < q.nq; ++i) Q.qof[q.xcc[i]] = i;
    TraceScope ts(st, "pipe_queue", q.bytes, 0.0);
    if (q.gmax == 6)
        hipLaunchKernelGGL((k_pipe_queue<R, 6>), dim3((unsigned)q.blocks), dim3(256), q.lds, st, Q);
    else
        hipLaunchKernelGGL((k_pipe_queue<R, 8>), dim3((unsigned)q.blocks), dim3(256), q.lds, st, Q);
    SV_HIP(hipGetLastError());
    return SV_OK;
}
template sv_status pipe_queue_build<float>(sv_state, hipStream_t, PipeQueue &, DevBuf &,
                                           const std::vector<QueueClassIn> &, const std::vector<int> &,
                                           const std::vector<PipeSolve> &, unsigned *, unsigned *);
template sv_status pipe_queue_build<double>(sv_state, hipStream_t, PipeQueue &, DevBuf &,
                                            const std::vector<QueueClassIn> &, const std::vector<int> &,
                                            const std::vector<PipeSolve> &, unsigned *, unsigned *);
template sv_status pipe_queue_launch<float>(hipStream_t, const PipeQueue &, const FinishJob *);
template sv_status pipe_queue_launch<double>(hipStream_t, const PipeQueue &, const FinishJob *);

uint64_t pipe_b_blocks_for(int n_s, int n_c, int cl) {
    const int g1 = (n_c + 1) / 2;
    return (dim_of(n_s) >> cl) << g1;
}

// upper bounds of the k_pipe_b block count (one FP64 partial pair each) and
// the k_pipe_c partial rows, over every configuration the tuner may pick
uint64_t pipe_b_blocks(int n_s, int n_c, size_t elem) {
    (void)elem;
    return pipe_b_blocks_for(n_s, n_c, n_s < 3 ? n_s : 3);
}
int pipe_c_rows(int n_c) { return 1 << (n_c - (n_c + 1) / 2); }

}  // namespace sv
