// QPP: velocity gradients of an amplitude-encoded profile (main text,
// "Quantum Post-processing Protocol"; appendix "Velocity gradients").
//
// LCU form.  The zero-wall central difference (D u)_j = (u_{j+1} - u_{j-1})/2h
// on the N = 2^m points of a register is 4h D = C + C R0 - C^T - R0 C^T with
// the cyclic shift (C u)_j = u_{(j+1) mod N} and R0 = I - 2|0><0|: four
// unitaries of equal weight, selected by two qubits.  The circuit is
// V^dagger G V with V = H (x) H on the select qubits and G = sum_i |i><i| (x) U_i;
// from select |00> its select-|00> block is h D u.
//   mode 0: the circuit gate by gate (Hadamards; C and C^T as cascades of
//           multi-controlled X; R0 as a multi-controlled phase; the two minus
//           signs as one Z on the high select qubit);
//   mode 1: the whole circuit in one pass: tiles holding every register and
//           select value of a few columns are staged in LDS, and each thread
//           forms the four select outputs of one register point from the
//           select values at its two neighbours.  A register too wide for one
//           tile is cut into chunks of its low bits: a first kernel copies the
//           two outside neighbours of every chunk (all select values) into
//           scratch memory, so the in-place tile pass can read them after the
//           neighbouring tiles have been overwritten.
//
// Spectral form.  Inverse QFT on the register, the wavenumber diagonal
// Lambda_k as the |1> block of a rotation of one more qubit (controlled on the
// register value; its table is computed in the kernel), then the QFT.
#include <math.h>

#include <vector>

#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

// ----------------------------------------------------------------- LCU, fused

struct LcuArgs {
    uint64_t tmask;      // index bits held by one tile (register, select, lowest others)
    uint64_t omask;      // the remaining index bits (tile number)
    int tb;              // log2 tile size
    int rq, rs;          // rank of the register's lowest bit / select's lowest bit inside a tile index
    int m;               // register qubits
    int cb;              // register bits inside a tile (cb < m: the register is chunked)
    int q_lo;
    uint64_t sb1, sb2;   // the two select bits of a global index
    uint64_t ntiles;
    int contig;          // the tile bits are the lowest tb bits: no bit deposit needed
};

// global index of tile element t of tile `tid`
__device__ __forceinline__ uint64_t lcu_index(const LcuArgs &a, uint64_t tid, uint64_t t) {
    return a.contig ? (tid << a.tb) | t : pdep64(tid, a.omask) | pdep64(t, a.tmask);
}

// index of the chunk-halo pair of the global index g: g without the low cb
// register bits (the bits of a point inside its chunk)
__device__ __forceinline__ uint64_t halo_slot(uint64_t g, int q_lo, int cb) {
    return ((g >> (q_lo + cb)) << q_lo) | (g & ((1ull << q_lo) - 1ull));
}

// the two outside neighbours of every chunk, for every select value and column:
// halo[2 t] = point chunk 2^cb - 1, halo[2 t + 1] = point (chunk + 1) 2^cb (cyclic)
template <typename R>
__global__ __launch_bounds__(256) void k_lcu_halo(const cvec<R> *__restrict__ psi, cvec<R> *__restrict__ halo,
                                                  uint64_t nslots, int q_lo, int m, int cb) {
    const uint64_t N = 1ull << m, rmask = (N - 1ull) << q_lo;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nslots; t += stride) {
        const uint64_t g0 = ((t >> q_lo) << (q_lo + cb)) | (t & ((1ull << q_lo) - 1ull));
        const uint64_t first = ((g0 & rmask) >> q_lo);           // chunk * 2^cb
        const uint64_t dn = (first + N - 1ull) & (N - 1ull), up = (first + (1ull << cb)) & (N - 1ull);
        const uint64_t rest = g0 & ~rmask;
        halo[2 * t] = psi[rest | (dn << q_lo)];
        halo[2 * t + 1] = psi[rest | (up << q_lo)];
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_lcu(cvec<R> *__restrict__ psi, const cvec<R> *__restrict__ halo, LcuArgs a) {
    extern __shared__ unsigned char lds_raw[];
    cvec<R> *tile = reinterpret_cast<cvec<R> *>(lds_raw);
    const uint32_t T = 1u << a.tb, jm = (1u << a.cb) - 1u;     // points of one chunk
    const uint64_t Nm = (1ull << a.m) - 1ull;                    // last point of the register
    const bool chunked = a.cb < a.m;
    const uint32_t rmask = jm << a.rq;
    for (uint64_t tid = blockIdx.x; tid < a.ntiles; tid += gridDim.x) {
        const uint64_t base = lcu_index(a, tid, 0);
        for (uint32_t t = threadIdx.x; t < T; t += blockDim.x) tile[t] = psi[a.contig ? base | t : base | pdep64(t, a.tmask)];
        __syncthreads();
        // one thread per (column, register point): tile indices with select = 0
        for (uint32_t q = threadIdx.x; q < (T >> 2); q += blockDim.x) {
            // insert the two select bits (zero) at rank rs
            const uint32_t t0 = ((q >> a.rs) << (a.rs + 2)) | (q & ((1u << a.rs) - 1u));
            const uint32_t j = (t0 & rmask) >> a.rq;
            const uint32_t col = t0 & ~rmask;
            const uint32_t up = col | (((j + 1u) & jm) << a.rq), dn = col | (((j + jm) & jm) << a.rq);
            const uint32_t s1 = 1u << a.rs, s2 = 2u << a.rs;
            const uint64_t g = a.contig ? base | t0 : base | pdep64(t0, a.tmask);   // select 0, this point
            const uint64_t g1 = a.sb1, g2 = a.sb2;
            const uint64_t jg = ((g >> a.q_lo) & Nm);                     // the point's register value
            // the select values at the two neighbours (from the halo copy at a chunk edge)
            cvec<R> u0, u1, u2, u3, d0, d1, d2, d3;
            if (chunked && j == jm) {
                u0 = halo[2 * halo_slot(g, a.q_lo, a.cb) + 1];
                u1 = halo[2 * halo_slot(g | g1, a.q_lo, a.cb) + 1];
                u2 = halo[2 * halo_slot(g | g2, a.q_lo, a.cb) + 1];
                u3 = halo[2 * halo_slot(g | g1 | g2, a.q_lo, a.cb) + 1];
            } else {
                u0 = tile[up], u1 = tile[up | s1], u2 = tile[up | s2], u3 = tile[up | s1 | s2];
            }
            if (chunked && j == 0) {
                d0 = halo[2 * halo_slot(g, a.q_lo, a.cb)];
                d1 = halo[2 * halo_slot(g | g1, a.q_lo, a.cb)];
                d2 = halo[2 * halo_slot(g | g2, a.q_lo, a.cb)];
                d3 = halo[2 * halo_slot(g | g1 | g2, a.q_lo, a.cb)];
            } else {
                d0 = tile[dn], d1 = tile[dn | s1], d2 = tile[dn | s2], d3 = tile[dn | s1 | s2];
            }
            // V at the two neighbours: w_0, w_1 at j + 1 (used by C, C R0), w_2, w_3 at j - 1
            const R h = (R)0.5;
            cvec<R> y0 = cmake<R>(h * (u0.x + u1.x + u2.x + u3.x), h * (u0.y + u1.y + u2.y + u3.y));
            cvec<R> y1 = cmake<R>(h * (u0.x - u1.x + u2.x - u3.x), h * (u0.y - u1.y + u2.y - u3.y));
            cvec<R> y2 = cmake<R>(h * (d0.x + d1.x - d2.x - d3.x), h * (d0.y + d1.y - d2.y - d3.y));
            cvec<R> y3 = cmake<R>(h * (d0.x - d1.x - d2.x + d3.x), h * (d0.y - d1.y - d2.y + d3.y));
            // G: C R0 flips the sign of the value that wrapped from 0; -C^T; -R0 C^T flips at j = 0
            if (jg == Nm) y1 = cmake<R>(-y1.x, -y1.y);
            y2 = cmake<R>(-y2.x, -y2.y);
            if (jg != 0) y3 = cmake<R>(-y3.x, -y3.y);
            // V^dagger
            psi[g] = cmake<R>(h * (y0.x + y1.x + y2.x + y3.x), h * (y0.y + y1.y + y2.y + y3.y));
            psi[g | g1] = cmake<R>(h * (y0.x - y1.x + y2.x - y3.x), h * (y0.y - y1.y + y2.y - y3.y));
            psi[g | g2] = cmake<R>(h * (y0.x + y1.x - y2.x - y3.x), h * (y0.y + y1.y - y2.y - y3.y));
            psi[g | g1 | g2] = cmake<R>(h * (y0.x - y1.x - y2.x + y3.x), h * (y0.y - y1.y - y2.y + y3.y));
        }
        __syncthreads();
    }
}

// log2 of the largest LDS tile the fused LCU pass stages (64 KiB)
static int lcu_max_tile_bits(sv_dtype dt) { return dt == SV_C128 ? 12 : 13; }

static sv_status lcu_fused(sv_state s, int q_lo, int m, int sel_lo) {
    const int n = s->n;
    const int cap = lcu_max_tile_bits(s->dt);
    const int cb = m + 2 <= cap ? m : cap - 2;      // register bits per tile
    const int need = cb + 2;
    int tb = need < 10 ? 10 : need;
    if (tb > n) tb = n;
    uint64_t tmask = (((1ull << cb) - 1ull) << q_lo) | (3ull << sel_lo);
    // fill the tile with the lowest remaining bits
    for (int b = 0, extra = tb - need; b < n && extra > 0; ++b)
        if (!((tmask >> b) & 1ull)) {
            tmask |= 1ull << b;
            --extra;
        }
    const uint64_t all = dim_of(n) - 1ull;
    LcuArgs a;
    a.tmask = tmask;
    a.omask = all & ~tmask;
    a.tb = tb;
    a.rq = popcount64(tmask & ((1ull << q_lo) - 1ull));
    a.rs = popcount64(tmask & ((1ull << sel_lo) - 1ull));
    a.m = m;
    a.cb = cb;
    a.q_lo = q_lo;
    a.sb1 = 1ull << sel_lo;
    a.sb2 = 2ull << sel_lo;
    a.ntiles = 1ull << (n - tb);
    a.contig = tmask == ((1ull << tb) - 1ull) ? 1 : 0;
    const size_t lds = ((size_t)1 << tb) * amp_bytes(s->dt);
    const unsigned grid = (unsigned)(a.ntiles < 4096 ? a.ntiles : 4096);
    void *halo = nullptr;
    if (cb < m) {
        // one pair per (column, chunk, select value): 2^(n - cb) slots
        const uint64_t nslots = dim_of(n - cb);
        SV_TRY(ensure_scratch(s, 2 * nslots * amp_bytes(s->dt)));
        halo = s->scratch;
        uint64_t hg = (nslots + 255) / 256;
        if (hg > 65536) hg = 65536;
        TraceScope th(s->stream, "lcu_halo", 4.0 * (double)nslots * amp_bytes(s->dt), 0.0);
        if (s->dt == SV_C64)
            hipLaunchKernelGGL(k_lcu_halo<float>, dim3((unsigned)hg), dim3(256), 0, s->stream,
                               (const float2 *)s->data, (float2 *)halo, nslots, q_lo, m, cb);
        else
            hipLaunchKernelGGL(k_lcu_halo<double>, dim3((unsigned)hg), dim3(256), 0, s->stream,
                               (const double2 *)s->data, (double2 *)halo, nslots, q_lo, m, cb);
        SV_HIP(hipGetLastError());
    }
    TraceScope ts(s->stream, "lcu_derivative", 2.0 * (double)dim_of(n) * amp_bytes(s->dt), 0.0);
    if (s->dt == SV_C64)
        hipLaunchKernelGGL(k_lcu<float>, dim3(grid), dim3(256), lds, s->stream, (float2 *)s->data,
                           (const float2 *)halo, a);
    else
        hipLaunchKernelGGL(k_lcu<double>, dim3(grid), dim3(256), lds, s->stream, (double2 *)s->data,
                           (const double2 *)halo, a);
    SV_HIP(hipGetLastError());
    return SV_OK;
}

// ------------------------------------------------------------- LCU, gate mode

static const double GX[8] = {0, 0, 1, 0, 1, 0, 0, 0};

// cyclic shift of the register under the select controls: down (k -> k - 1, the
// operator C) flips bit b when every lower bit is 0; up (C^T) when every lower bit is 1.
static sv_status shift_gates(sv_state s, int q_lo, int m, bool down, const int *sc, const int *sv) {
    int ctrls[34], vals[34];
    for (int b = m - 1; b >= 0; --b) {
        int c = 0;
        for (int l = 0; l < b; ++l) {
            ctrls[c] = q_lo + l;
            vals[c++] = down ? 0 : 1;
        }
        ctrls[c] = sc[0];
        vals[c++] = sv[0];
        ctrls[c] = sc[1];
        vals[c++] = sv[1];
        SV_TRY(sv_apply_gate(s, q_lo + b, GX, ctrls, vals, c));
    }
    return SV_OK;
}

// R0 = I - 2|0><0| on the register under the select controls
static sv_status reflect_gate(sv_state s, int q_lo, int m, const int *sc, const int *sv) {
    static const double ZN[8] = {-1, 0, 0, 0, 0, 0, 1, 0};   // diag(-1, 1)
    int ctrls[34], vals[34], c = 0;
    for (int l = 1; l < m; ++l) {
        ctrls[c] = q_lo + l;
        vals[c++] = 0;
    }
    ctrls[c] = sc[0];
    vals[c++] = sv[0];
    ctrls[c] = sc[1];
    vals[c++] = sv[1];
    return sv_apply_gate(s, q_lo, ZN, ctrls, vals, c);
}

static sv_status lcu_gates(sv_state s, int q_lo, int m, int sel_lo) {
    const double r = 0.70710678118654752440;
    const double H[8] = {r, 0, r, 0, r, 0, -r, 0};
    static const double Z[8] = {1, 0, 0, 0, 0, 0, -1, 0};
    SV_TRY(sv_apply_gate(s, sel_lo, H, nullptr, nullptr, 0));
    SV_TRY(sv_apply_gate(s, sel_lo + 1, H, nullptr, nullptr, 0));
    const int sc[2] = {sel_lo, sel_lo + 1};
    for (int i = 0; i < 4; ++i) {
        const int sv[2] = {i & 1, i >> 1};
        switch (i) {
        case 0: SV_TRY(shift_gates(s, q_lo, m, true, sc, sv)); break;                   // C
        case 1: SV_TRY(reflect_gate(s, q_lo, m, sc, sv));                               // C R0
                SV_TRY(shift_gates(s, q_lo, m, true, sc, sv)); break;
        case 2: SV_TRY(shift_gates(s, q_lo, m, false, sc, sv)); break;                  // (-) C^T
        default: SV_TRY(shift_gates(s, q_lo, m, false, sc, sv));                        // (-) R0 C^T
                 SV_TRY(reflect_gate(s, q_lo, m, sc, sv)); break;
        }
    }
    SV_TRY(sv_apply_gate(s, sel_lo + 1, Z, nullptr, nullptr, 0));                      // the two minus signs
    SV_TRY(sv_apply_gate(s, sel_lo, H, nullptr, nullptr, 0));
    return sv_apply_gate(s, sel_lo + 1, H, nullptr, nullptr, 0);
}

// ----------------------------------------------------------- spectral diagonal

// For each register value k: (a0, a1) on qubit anc <- e^{i arg Lambda_k} Ry(t_k) (a0, a1),
// sin(t_k/2) = |k'| / (N/2 - 1), k' = k (k < N/2) or k - N (k > N/2); arg = +-pi/2, so the
// phase is an exact multiplication by +-i.  k = 0 and k = N/2 are the identity.
template <typename R>
__global__ __launch_bounds__(256) void k_wavenumber_ry(cvec<R> *__restrict__ psi, uint64_t npairs, int anc,
                                                       int q_lo, int m) {
    const uint64_t N = 1ull << m, half = N >> 1;
    const double den = (double)(half - 1);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npairs; p += stride) {
        const uint64_t i0 = ((p >> anc) << (anc + 1)) | (p & ((1ull << anc) - 1ull));
        const uint64_t k = (i0 >> q_lo) & (N - 1);
        if (k == 0 || k == half) continue;
        const uint64_t i1 = i0 | (1ull << anc);
        const bool pos = k < half;
        const double sd = (double)(pos ? k : N - k) / den;   // exactly 1 at the largest |k'|
        const R sn = (R)sd, cs = (R)sqrt(fmax(0.0, 1.0 - sd * sd));
        const cvec<R> a0 = psi[i0], a1 = psi[i1];
        const cvec<R> b0 = cmake<R>(cs * a0.x - sn * a1.x, cs * a0.y - sn * a1.y);
        const cvec<R> b1 = cmake<R>(sn * a0.x + cs * a1.x, sn * a0.y + cs * a1.y);
        // times +i: (x, y) -> (-y, x); times -i: (x, y) -> (y, -x)
        psi[i0] = pos ? cmake<R>(-b0.y, b0.x) : cmake<R>(b0.y, -b0.x);
        psi[i1] = pos ? cmake<R>(-b1.y, b1.x) : cmake<R>(b1.y, -b1.x);
    }
}

}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_lcu_derivative(sv_state s, int q_lo, int m, int sel_lo, int mode) {
    clear_error();
    SV_TRY(check_state(s));
    if (m < 1 || q_lo < 0 || q_lo + m > s->n)
        return fail(SV_EINVAL, "register [%d, %d) outside the %d-qubit state", q_lo, q_lo + m, s->n);
    if (m > 30) return fail(SV_EINVAL, "register wider than 30 qubits");
    if (sel_lo < 0 || sel_lo + 2 > s->n)
        return fail(SV_EINVAL, "select qubits [%d, %d) outside the state", sel_lo, sel_lo + 2);
    if (sel_lo + 2 > q_lo && sel_lo < q_lo + m) return fail(SV_EINVAL, "select qubits overlap the register");
    if (mode == 0) return lcu_gates(s, q_lo, m, sel_lo);
    if (mode == 1) return lcu_fused(s, q_lo, m, sel_lo);
    return fail(SV_EINVAL, "mode must be 0 or 1");
}

sv_status sv_spectral_derivative(sv_state s, int q_lo, int m, int anc, int max_local) {
    clear_error();
    SV_TRY(check_state(s));
    if (m < 2 || q_lo < 0 || q_lo + m > s->n)
        return fail(SV_EINVAL, "register [%d, %d) outside the state or narrower than 2 qubits", q_lo, q_lo + m);
    if (m > 30) return fail(SV_EINVAL, "register wider than 30 qubits");
    if (anc < 0 || anc >= s->n || (anc >= q_lo && anc < q_lo + m))
        return fail(SV_EINVAL, "qubit %d is outside the state or inside the register", anc);
    SV_TRY(sv_qft(s, q_lo, m, 1, 1, max_local));
    {
        const uint64_t np = dim_of(s->n - 1);
        uint64_t g = (np + 1023) / 1024;
        if (g > (1u << 20)) g = 1u << 20;
        TraceScope ts(s->stream, "wavenumber_ry", 2.0 * (double)dim_of(s->n) * amp_bytes(s->dt), 0.0);
        if (s->dt == SV_C64)
            hipLaunchKernelGGL(k_wavenumber_ry<float>, dim3((unsigned)g), dim3(256), 0, s->stream, (float2 *)s->data,
                               np, anc, q_lo, m);
        else
            hipLaunchKernelGGL(k_wavenumber_ry<double>, dim3((unsigned)g), dim3(256), 0, s->stream,
                               (double2 *)s->data, np, anc, q_lo, m);
        SV_HIP(hipGetLastError());
    }
    return sv_qft(s, q_lo, m, 0, 1, max_local);
}

}  // extern "C"
