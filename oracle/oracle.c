/*
 * oracle.c -- plain, slow, FP64 CPU reference for the HHL state-vector path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it (through oracle/__init__.py).
 *
 * Conventions (shared by definition, not by code, with the GPU library):
 *   - a state on n qubits is 2^n complex doubles; qubit q is bit q of the
 *     basis index (fixed by the paper's worked example U = H_1 (x) X_0 in the
 *     appendix "QFlowS - a brief overview", whose 4x4 matrix only matches
 *     the Kronecker product if qubit 1 is the most significant bit);
 *   - a one-qubit gate u is row-major 2x2: (a0,a1) <- (u00 a0 + u01 a1,
 *     u10 a0 + u11 a1) on the pair of indices that differ only in bit q
 *     (the "algebraic" gate application of the same appendix);
 *   - HHL register layout: bits [0,n_s) system x, [n_s,n_s+n_c) clock y,
 *     bit n_s+n_c the ancilla a.
 *
 * Every loop here is written for clarity; the only parallelism is an
 * OpenMP "parallel for" over iterations that are independent by
 * construction (they touch disjoint amplitudes), which leaves every
 * floating-point result bit-identical to the serial loop.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* True when every control qubit of index i holds its required value. */
static int controls_match(uint64_t i, const int *ctrls, const int *cvals, int nctrl)
{
    for (int c = 0; c < nctrl; ++c)
        if ((int)((i >> ctrls[c]) & 1u) != (cvals ? cvals[c] : 1))
            return 0;
    return 1;
}

static int check_qubits(int n, int target, const int *ctrls, int nctrl)
{
    if (n < 1 || n > 40 || target < 0 || target >= n) return ORC_EINVAL;
    for (int c = 0; c < nctrl; ++c) {
        if (ctrls[c] < 0 || ctrls[c] >= n || ctrls[c] == target) return ORC_EINVAL;
        for (int d = 0; d < c; ++d)
            if (ctrls[d] == ctrls[c]) return ORC_EINVAL;
    }
    return ORC_OK;
}

/*
 * One-qubit gate u (row-major 2x2, interleaved re/im: 8 doubles) on qubit
 * `target`, applied only where the control qubits match.  This is the pair
 * update of the appendix's algebraic gate rule: for each index i0 with bit
 * `target` clear, i1 = i0 | 2^target, the pair (psi[i0], psi[i1]) is
 * multiplied by u.
 */
int orc_apply_gate(cplx *psi, int n, int target, const double *u8,
                   const int *ctrls, const int *cvals, int nctrl)
{
    if (check_qubits(n, target, ctrls, nctrl) != ORC_OK) return ORC_EINVAL;
    const cplx u00 = u8[0] + I * u8[1], u01 = u8[2] + I * u8[3];
    const cplx u10 = u8[4] + I * u8[5], u11 = u8[6] + I * u8[7];
    const uint64_t dim = (uint64_t)1 << n, bit = (uint64_t)1 << target;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i0 = (uint64_t)ii;
        if (i0 & bit) continue;
        if (!controls_match(i0, ctrls, cvals, nctrl)) continue;
        uint64_t i1 = i0 | bit;
        cplx a0 = psi[i0], a1 = psi[i1];
        psi[i0] = u00 * a0 + u01 * a1;
        psi[i1] = u10 * a0 + u11 * a1;
    }
    return ORC_OK;
}

/*
 * Exchange of qubits q1 and q2 (the SWAP gate), restricted to indices whose
 * control qubits match.  A pure permutation: amplitudes are moved, never
 * combined, so the result is bit-exact.
 */
int orc_apply_swap(cplx *psi, int n, int q1, int q2, const int *ctrls,
                   const int *cvals, int nctrl)
{
    if (check_qubits(n, q1, ctrls, nctrl) != ORC_OK) return ORC_EINVAL;
    if (check_qubits(n, q2, ctrls, nctrl) != ORC_OK || q1 == q2) return ORC_EINVAL;
    const uint64_t dim = (uint64_t)1 << n;
    const uint64_t b1 = (uint64_t)1 << q1, b2 = (uint64_t)1 << q2;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i = (uint64_t)ii;
        /* visit each exchanged pair once: from the member with q1 set, q2 clear */
        if (!(i & b1) || (i & b2)) continue;
        if (!controls_match(i, ctrls, cvals, nctrl)) continue;
        uint64_t j = (i & ~b1) | b2;
        cplx t = psi[i];
        psi[i] = psi[j];
        psi[j] = t;
    }
    return ORC_OK;
}

/*
 * Quantum Fourier transform on the register of qubits [lo, lo+m), written
 * out as its definition (the DFT kernels of the appendix on velocity
 * gradients): QFT|j> = 2^{-m/2} sum_k exp(+2 pi i j k / 2^m) |k>, the
 * inverse uses exp(-2 pi i j k / 2^m).  Output is in natural index order.
 * The phase angle is reduced exactly in integers, (j k mod 2^m) / 2^m,
 * before the cosine/sine, so no precision is lost for large m.
 */
int orc_qft(cplx *psi, int n, int lo, int m, int inverse)
{
    if (n < 1 || n > 40 || m < 1 || lo < 0 || lo + m > n) return ORC_EINVAL;
    const uint64_t M = (uint64_t)1 << m, dim = (uint64_t)1 << n;
    const uint64_t mask = (M - 1) << lo;
    const double sgn = inverse ? -1.0 : 1.0, scale = 1.0 / sqrt((double)M);
    cplx *tw = (cplx *)malloc(sizeof(cplx) * M);
    if (!tw) return ORC_ENOMEM;
    for (uint64_t r = 0; r < M; ++r)
        tw[r] = cos(2.0 * ORC_PI * (double)r / (double)M) +
                I * sgn * sin(2.0 * ORC_PI * (double)r / (double)M);
    const uint64_t ncol = dim / M;
    int err = ORC_OK;
#pragma omp parallel
    {
        cplx *in = (cplx *)malloc(sizeof(cplx) * M);
        if (!in) {
#pragma omp atomic write
            err = ORC_ENOMEM;
        }
#pragma omp for schedule(static)
        for (int64_t cc = 0; cc < (int64_t)ncol; ++cc) {
            if (!in) continue;
            /* spread the column index over the bits outside the register */
            uint64_t c = (uint64_t)cc;
            uint64_t base = (c & (((uint64_t)1 << lo) - 1)) | ((c >> lo) << (lo + m));
            for (uint64_t j = 0; j < M; ++j) in[j] = psi[base | (j << lo)];
            for (uint64_t k = 0; k < M; ++k) {
                cplx acc = 0;
                for (uint64_t j = 0; j < M; ++j) acc += tw[(j * k) & (M - 1)] * in[j];
                psi[base | (k << lo)] = scale * acc;
            }
        }
        free(in);
    }
    (void)mask;
    free(tw);
    return err;
}

/*
 * Controlled dense unitary on the contiguous register [lo, lo+m): for every
 * basis setting of the other qubits with qubit `ctrl` equal to `cval`
 * (ctrl < 0: no control), the 2^m sub-vector v is replaced by U v (or U^H v
 * when `adjoint`).  U is row-major, 2^m x 2^m, interleaved complex.
 */
int orc_apply_ctrl_unitary(cplx *psi, int n, const cplx *U, int lo, int m,
                           int ctrl, int cval, int adjoint)
{
    if (n < 1 || n > 40 || m < 1 || lo < 0 || lo + m > n) return ORC_EINVAL;
    if (ctrl >= n || (ctrl >= lo && ctrl < lo + m)) return ORC_EINVAL;
    const uint64_t M = (uint64_t)1 << m, dim = (uint64_t)1 << n;
    const uint64_t ncol = dim / M;
    int err = ORC_OK;
#pragma omp parallel
    {
        cplx *in = (cplx *)malloc(sizeof(cplx) * M);
        if (!in) {
#pragma omp atomic write
            err = ORC_ENOMEM;
        }
#pragma omp for schedule(static)
        for (int64_t cc = 0; cc < (int64_t)ncol; ++cc) {
            if (!in) continue;
            uint64_t c = (uint64_t)cc;
            uint64_t base = (c & (((uint64_t)1 << lo) - 1)) | ((c >> lo) << (lo + m));
            if (ctrl >= 0 && (int)((base >> ctrl) & 1u) != cval) continue;
            for (uint64_t j = 0; j < M; ++j) in[j] = psi[base | (j << lo)];
            for (uint64_t r = 0; r < M; ++r) {
                cplx acc = 0;
                for (uint64_t j = 0; j < M; ++j)
                    acc += (adjoint ? conj(U[j * M + r]) : U[r * M + j]) * in[j];
                psi[base | (r << lo)] = acc;
            }
        }
        free(in);
    }
    return err;
}

/* sum of |psi_i|^2 over indices with (i & mask) == value, in FP64 */
double orc_norm2(const cplx *psi, int n, uint64_t mask, uint64_t value)
{
    const uint64_t dim = (uint64_t)1 << n;
    double s = 0.0;
    for (uint64_t i = 0; i < dim; ++i)
        if ((i & mask) == value) s += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
    return s;
}

/*
 * Post-selection on the qubits in `mask` having the values in `value`: the
 * probability p of that outcome, and (if out != NULL) the surviving
 * amplitudes, in increasing index order, divided by sqrt(p).
 * Returns ORC_EINVAL when p == 0.
 */
int orc_postselect(const cplx *psi, int n, uint64_t mask, uint64_t value,
                   double *prob, cplx *out)
{
    if ((value & ~mask) != 0) return ORC_EINVAL;
    const uint64_t dim = (uint64_t)1 << n;
    double p = orc_norm2(psi, n, mask, value);
    if (prob) *prob = p;
    if (!(p > 0.0)) return ORC_EINVAL;
    if (out) {
        const double inv = 1.0 / sqrt(p);
        uint64_t k = 0;
        for (uint64_t i = 0; i < dim; ++i)
            if ((i & mask) == value) out[k++] = psi[i] * inv;
    }
    return ORC_OK;
}

/*
 * Eigen-decomposition of a Hermitian N x N matrix (row-major) by the cyclic
 * Jacobi method: repeated 2x2 unitary rotations J, each zeroing one
 * off-diagonal pair (p,q), until the off-diagonal mass is negligible.
 * For a pivot a_pq = r e^{i alpha}, J = diag(1, e^{-i alpha}) R, with R the
 * real Jacobi rotation (c, s; -s, c) that annihilates the now-real pair.
 * On return lam[j] (ascending) and column j of V (row-major) are the
 * eigen-pairs: A V = V diag(lam).
 */
int orc_eigh(int N, const cplx *A_in, double *lam, cplx *V)
{
    if (N < 1 || N > 8192) return ORC_EINVAL;
    cplx *A = (cplx *)malloc(sizeof(cplx) * (size_t)N * N);
    if (!A) return ORC_ENOMEM;
    memcpy(A, A_in, sizeof(cplx) * (size_t)N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) V[(size_t)i * N + j] = (i == j) ? 1.0 : 0.0;

    double fro = 0.0;
    for (size_t k = 0; k < (size_t)N * N; ++k) fro += creal(A[k] * conj(A[k]));
    fro = sqrt(fro);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < N; ++p)
            for (int q = p + 1; q < N; ++q) off += 2.0 * creal(A[(size_t)p * N + q] * conj(A[(size_t)p * N + q]));
        if (sqrt(off) <= 1e-15 * fro || fro == 0.0) break;
        for (int p = 0; p < N - 1; ++p) {
            for (int q = p + 1; q < N; ++q) {
                cplx apq = A[(size_t)p * N + q];
                double r = cabs(apq);
                if (r == 0.0) continue;
                double app = creal(A[(size_t)p * N + p]), aqq = creal(A[(size_t)q * N + q]);
                cplx ph = conj(apq) / r; /* e^{-i alpha} */
                double theta = (aqq - app) / (2.0 * r);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* J on the (p,q) plane: [[c, s], [-s ph, c ph]] */
                cplx Jpp = c, Jpq = s, Jqp = -s * ph, Jqq = c * ph;
                /* A <- A J (columns p, q) */
                for (int k = 0; k < N; ++k) {
                    cplx akp = A[(size_t)k * N + p], akq = A[(size_t)k * N + q];
                    A[(size_t)k * N + p] = akp * Jpp + akq * Jqp;
                    A[(size_t)k * N + q] = akp * Jpq + akq * Jqq;
                }
                /* A <- J^H A (rows p, q) */
                for (int k = 0; k < N; ++k) {
                    cplx apk = A[(size_t)p * N + k], aqk = A[(size_t)q * N + k];
                    A[(size_t)p * N + k] = conj(Jpp) * apk + conj(Jqp) * aqk;
                    A[(size_t)q * N + k] = conj(Jpq) * apk + conj(Jqq) * aqk;
                }
                A[(size_t)p * N + q] = 0.0;
                A[(size_t)q * N + p] = 0.0;
                /* V <- V J */
                for (int k = 0; k < N; ++k) {
                    cplx vkp = V[(size_t)k * N + p], vkq = V[(size_t)k * N + q];
                    V[(size_t)k * N + p] = vkp * Jpp + vkq * Jqp;
                    V[(size_t)k * N + q] = vkp * Jpq + vkq * Jqq;
                }
            }
        }
    }
    for (int j = 0; j < N; ++j) lam[j] = creal(A[(size_t)j * N + j]);
    /* sort ascending (selection sort keeps it obvious) */
    for (int a = 0; a < N; ++a) {
        int best = a;
        for (int b = a + 1; b < N; ++b)
            if (lam[b] < lam[best]) best = b;
        if (best != a) {
            double tl = lam[a]; lam[a] = lam[best]; lam[best] = tl;
            for (int k = 0; k < N; ++k) {
                cplx tv = V[(size_t)k * N + a];
                V[(size_t)k * N + a] = V[(size_t)k * N + best];
                V[(size_t)k * N + best] = tv;
            }
        }
    }
    free(A);
    return ORC_OK;
}

/*
 * The phase of eigen-component j under U^(2^k) = exp(i A T0 2^k):
 * phi_j = lam_j T0 / (2 pi) is formed once in FP64 and the clock bit k
 * contributes exp(2 pi i frac(phi_j 2^k)); multiplying by 2^k and taking
 * the fractional part are exact in binary floating point.
 */
static double frac_phase(double phi, int k)
{
    double x = ldexp(phi, k);
    return x - floor(x);
}

/*
 * U_k = V diag(exp(2 pi i frac(phi_j 2^k))) V^H on the system register,
 * written out as a dense matrix.
 */
static void build_uk(int N, const cplx *V, const double *phi, int k, cplx *Uk)
{
    for (int r = 0; r < N; ++r)
        for (int c = 0; c < N; ++c) {
            cplx acc = 0;
            for (int j = 0; j < N; ++j) {
                double f = frac_phase(phi[j], k);
                cplx e = cos(2.0 * ORC_PI * f) + I * sin(2.0 * ORC_PI * f);
                acc += V[(size_t)r * N + j] * e * conj(V[(size_t)c * N + j]);
            }
            Uk[(size_t)r * N + c] = acc;
        }
}

/*
 * HHL (QLSA-1) as a gate-level circuit, step by step:
 *   1. |0>_a |0>_c |b/|b|>_s
 *   2. Hadamard on every clock qubit
 *   3. eigen-decomposition A = V diag(lam) V^H; phi_j = lam_j T0 / (2 pi)
 *   4. for k = 0..n_c-1: controlled on clock qubit k, apply U_k = exp(i A T0 2^k)
 *      on the system register (phase estimation with e^{i A T0}, least count
 *      2^{-n_c} on lam T0 / 2 pi)
 *   5. inverse QFT on the clock register
 *   6. eigenvalue inversion: for clock value y >= 1, rotate the ancilla by
 *      Ry(theta_y) with sin(theta_y / 2) = C / lam~_y = 1 / y (y read as a
 *      two's-complement value with signed_clock, for indefinite A), where
 *      lam~_y = 2 pi y / (2^n_c T0) and C = 2 pi / (2^n_c T0) is the least
 *      count; y = 0 is left untouched
 *   7. uncompute: QFT on the clock, controlled U_k^H for k = n_c-1..0,
 *      Hadamard on every clock qubit
 *   8. post-select ancilla = 1 and clock = 0
 * Outputs: the whole final state psi (2^(n_s+n_c+1)), the normalised
 * post-selected system vector x (2^n_s), p_post = P(a=1, y=0) and
 * p_anc = P(a=1).
 */
static int hhl_circuit(int n_s, int n_c, double T0, const cplx *A, const cplx *b, cplx *psi, cplx *x_out,
                       double *p_post, double *p_anc, int signed_clock, uint64_t cut);

int orc_hhl(int n_s, int n_c, double T0, const cplx *A, const cplx *b,
            cplx *psi, cplx *x_out, double *p_post, double *p_anc, int signed_clock)
{
    return hhl_circuit(n_s, n_c, T0, A, b, psi, x_out, p_post, p_anc, signed_clock, 0);
}

/*
 * Gapped phase estimation (GPE; the building block of the variable-time
 * solver in the cited Childs-Kothari-Somma construction, which QLSA-2 names):
 * the circuit of orc_hhl with step 6 replaced by a flag.  After the inverse
 * QFT, every clock value y with |y| >= cut (y read as a two's-complement value
 * with signed_clock) rotates the flag qubit (the ancilla position) by
 * Ry(pi), |0> -> |1>; the others leave it alone.  The phase estimation is
 * then uncomputed (step 7).  An eigenvector whose estimate lies well above
 * the cut ends with flag 1 and the clock back at 0, one well below it with
 * flag 0; near the cut the two branches mix and part of the amplitude stays
 * on clock values != 0.  Outputs as orc_hhl: x is the normalised flag = 1,
 * clock = 0 system vector, p_post = P(flag = 1, clock = 0), p_anc = P(flag = 1).
 * cut >= 1.
 */
int orc_gapped_pe(int n_s, int n_c, double T0, const cplx *A, const cplx *b, cplx *psi, cplx *x_out,
                  double *p_post, double *p_anc, int signed_clock, uint64_t cut)
{
    if (cut < 1) return ORC_EINVAL;
    return hhl_circuit(n_s, n_c, T0, A, b, psi, x_out, p_post, p_anc, signed_clock, cut);
}

/* the HHL circuit; cut = 0 takes the inversion rotation of step 6, cut >= 1
 * the gapped-phase-estimation flag */
static int hhl_circuit(int n_s, int n_c, double T0, const cplx *A, const cplx *b, cplx *psi, cplx *x_out,
                       double *p_post, double *p_anc, int signed_clock, uint64_t cut)
{
    if (n_s < 1 || n_c < 1 || n_s + n_c + 1 > 30 || !(T0 > 0.0)) return ORC_EINVAL;
    const int N = 1 << n_s, n = n_s + n_c + 1;
    const uint64_t dim = (uint64_t)1 << n;
    const int anc = n_s + n_c;

    double bn = 0.0;
    for (int j = 0; j < N; ++j) bn += creal(b[j] * conj(b[j]));
    bn = sqrt(bn);
    if (!(bn > 0.0)) return ORC_EINVAL;

    /* 1. initial state */
    memset(psi, 0, sizeof(cplx) * dim);
    for (int j = 0; j < N; ++j) psi[j] = b[j] / bn;

    /* 2. Hadamards on the clock */
    const double h = 1.0 / sqrt(2.0);
    const double H8[8] = {h, 0, h, 0, h, 0, -h, 0};
    for (int k = 0; k < n_c; ++k) orc_apply_gate(psi, n, n_s + k, H8, NULL, NULL, 0);

    /* 3. spectrum */
    double *lam = (double *)malloc(sizeof(double) * N);
    double *phi = (double *)malloc(sizeof(double) * N);
    cplx *V = (cplx *)malloc(sizeof(cplx) * (size_t)N * N);
    cplx *Uk = (cplx *)malloc(sizeof(cplx) * (size_t)N * N);
    if (!lam || !phi || !V || !Uk) {
        free(lam); free(phi); free(V); free(Uk);
        return ORC_ENOMEM;
    }
    orc_eigh(N, A, lam, V);
    for (int j = 0; j < N; ++j) phi[j] = lam[j] * T0 / (2.0 * ORC_PI);

    /* 4. controlled powers of exp(i A T0) */
    for (int k = 0; k < n_c; ++k) {
        build_uk(N, V, phi, k, Uk);
        orc_apply_ctrl_unitary(psi, n, Uk, 0, n_s, n_s + k, 1, 0);
    }

    /* 5. inverse QFT on the clock */
    orc_qft(psi, n, n_s, n_c, 1);

    /* 6. controlled-Ry eigenvalue inversion, one clock value at a time; with
     *    a signed clock the values y >= 2^(n_c-1) stand for y - 2^n_c (two's
     *    complement), so negative eigenvalues invert with their sign */
    const uint64_t Y = (uint64_t)1 << n_c;
    for (uint64_t y = 1; y < Y; ++y) {
        const double ys = (signed_clock && y >= Y / 2) ? (double)y - (double)Y : (double)y;
        double s, c;
        if (cut == 0) {
            s = 1.0 / ys;
            c = sqrt(1.0 - s * s);
        } else if (fabs(ys) >= (double)cut) {    /* flag: Ry(pi) */
            s = 1.0;
            c = 0.0;
        } else {
            continue;
        }
        for (uint64_t x = 0; x < (uint64_t)N; ++x) {
            uint64_t i0 = x | (y << n_s), i1 = i0 | ((uint64_t)1 << anc);
            cplx a0 = psi[i0], a1 = psi[i1];
            psi[i0] = c * a0 - s * a1;
            psi[i1] = s * a0 + c * a1;
        }
    }

    /* 7. uncompute the phase estimation */
    orc_qft(psi, n, n_s, n_c, 0);
    for (int k = n_c - 1; k >= 0; --k) {
        build_uk(N, V, phi, k, Uk);
        orc_apply_ctrl_unitary(psi, n, Uk, 0, n_s, n_s + k, 1, 1);
    }
    for (int k = 0; k < n_c; ++k) orc_apply_gate(psi, n, n_s + k, H8, NULL, NULL, 0);

    /* 8. post-selection */
    const uint64_t amask = (uint64_t)1 << anc, cmask = (Y - 1) << n_s;
    double pa = orc_norm2(psi, n, amask, amask);
    if (p_anc) *p_anc = pa;
    double pp = 0.0;
    int rc = orc_postselect(psi, n, amask | cmask, amask, &pp, x_out);
    if (p_post) *p_post = pp;
    free(lam); free(phi); free(V); free(Uk);
    return rc;
}

/*
 * QSP-1: the binary-tree state preparation of the appendix "Quantum State
 * Preparation" (Grover-Rudolph tree in the form of Prakash), written as the
 * circuit it describes.  From |0...0> it prepares b / |b| on the register
 * [q_lo, q_lo + m) (register value r = sum of bit j of r times qubit q_lo + j).
 *
 * Tree: the leaves are the weights |b_r|^2; an inner node's weight is the sum
 * of its two children.  Level l (0 = root) decides qubit q_lo + m - 1 - l, the
 * register's most significant qubit first, so a node at level l is the value
 * p of the l qubits above that one (p's most significant bit is the top
 * qubit).  For every node with weight w > 0 the circuit applies
 * Ry(t) = [[cos t/2, -sin t/2], [sin t/2, cos t/2]], controlled on those l
 * qubits taking the values of p, with cos^2(t/2) = (zero child) / w: the
 * node's amplitude splits into its children's amplitudes.  A node of weight
 * 0 gets no gate.  After the last level the amplitudes are |b_r| / |b|; one
 * phase gate per basis state restores arg(b_r), a diag(e^{i a}, 1) or
 * diag(1, e^{i a}) on qubit q_lo controlled on the other register qubits.
 *
 * levels < m stops after that many levels (no phases): the intermediate
 * states of the appendix's worked example.
 */
int orc_qsp(cplx *psi, int n, int q_lo, int m, const cplx *b, int levels)
{
    if (m < 1 || q_lo < 0 || q_lo + m > n || m > 24) return ORC_EINVAL;
    const uint64_t R = (uint64_t)1 << m, dim = (uint64_t)1 << n;
    double *w = (double *)calloc(2 * R, sizeof(double));   /* heap order: node (l, p) at 2^l + p */
    if (!w) return ORC_ENOMEM;
    double tot = 0.0;
    for (uint64_t r = 0; r < R; ++r) {
        w[R + r] = creal(b[r]) * creal(b[r]) + cimag(b[r]) * cimag(b[r]);
        tot += w[R + r];
    }
    if (!(tot > 0.0)) { free(w); return ORC_EINVAL; }
    for (uint64_t k = R - 1; k >= 1; --k) w[k] = w[2 * k] + w[2 * k + 1];
    for (uint64_t i = 0; i < dim; ++i) psi[i] = 0.0;
    psi[0] = 1.0;
    int ctrls[32], cvals[32];
    const int L = levels < 0 || levels > m ? m : levels;
    for (int l = 0; l < L; ++l) {
        const int t = q_lo + m - 1 - l;
        for (int j = 0; j < l; ++j) ctrls[j] = q_lo + m - 1 - j;   /* the qubits above t */
        for (uint64_t p = 0; p < ((uint64_t)1 << l); ++p) {
            const uint64_t node = ((uint64_t)1 << l) + p;
            if (!(w[node] > 0.0)) continue;
            const double c = sqrt(w[2 * node] / w[node]), s = sqrt(w[2 * node + 1] / w[node]);
            for (int j = 0; j < l; ++j) cvals[j] = (int)((p >> (l - 1 - j)) & 1);
            const double ry[8] = {c, 0.0, -s, 0.0, s, 0.0, c, 0.0};
            int rc = orc_apply_gate(psi, n, t, ry, ctrls, cvals, l);
            if (rc != ORC_OK) { free(w); return rc; }
        }
    }
    if (L == m) {
        for (uint64_t r = 0; r < R; ++r) {
            if (w[R + r] == 0.0) continue;
            const double a = carg(b[r]);
            if (a == 0.0) continue;
            const cplx e = cexp(I * a);
            double u[8] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
            if (r & 1) { u[6] = creal(e); u[7] = cimag(e); }
            else { u[0] = creal(e); u[1] = cimag(e); }
            for (int j = 1; j < m; ++j) { ctrls[j - 1] = q_lo + j; cvals[j - 1] = (int)((r >> j) & 1); }
            int rc = orc_apply_gate(psi, n, q_lo, u, ctrls, cvals, m - 1);
            if (rc != ORC_OK) { free(w); return rc; }
        }
    }
    free(w);
    return ORC_OK;
}

/*
 * QPP velocity gradient by a linear combination of unitaries (appendix
 * "Velocity gradients - LCU method").
 *
 * The finite-difference operator is the central first difference on the
 * register's N = 2^m points with zero Dirichlet walls,
 *     (D u)_j = (u_{j+1} - u_{j-1}) / 2h,   u_{-1} = u_N = 0.
 * The paper does not spell out the unitaries; the decomposition used here:
 * with the cyclic shift (C u)_j = u_{(j+1) mod N} and the reflection
 * R0 = I - 2|0><0|, the truncated shift (S u)_j = u_{j+1} (0 past the end)
 * is (C + C R0) / 2, so
 *     4h D = 2 S - 2 S^T = C + C R0 - C^T - R0 C^T:
 * four unitaries U_0..U_3 = C, C R0, -C^T, -R0 C^T with equal weights.
 * The appendix's steps on the two select qubits [sel_lo, sel_lo + 2)
 * (select value i = bit sel_lo + 2 bit sel_lo+1):
 *     V  = H (x) H          (the equal-weight state of the coefficients),
 *     G  = sum_i |i><i| (x) U_i on the register,
 *     V^dagger = H (x) H.
 * G is written out as the action of each U_i on the register amplitudes.
 * A select register that starts in |00> ends with h D |phi> in its |00>
 * component.
 */
int orc_lcu_derivative(cplx *psi, int n, int q_lo, int m, int sel_lo)
{
    if (n < 3 || n > 40 || m < 1 || q_lo < 0 || q_lo + m > n) return ORC_EINVAL;
    if (sel_lo < 0 || sel_lo + 2 > n) return ORC_EINVAL;
    if (sel_lo + 2 > q_lo && sel_lo < q_lo + m) return ORC_EINVAL;    /* overlaps the register */
    const double r = 1.0 / sqrt(2.0);
    const double h[8] = {r, 0.0, r, 0.0, r, 0.0, -r, 0.0};
    int rc;
    if ((rc = orc_apply_gate(psi, n, sel_lo, h, NULL, NULL, 0)) != ORC_OK) return rc;
    if ((rc = orc_apply_gate(psi, n, sel_lo + 1, h, NULL, NULL, 0)) != ORC_OK) return rc;
    const uint64_t dim = (uint64_t)1 << n, N = (uint64_t)1 << m, rmask = (N - 1) << q_lo;
    cplx *src = (cplx *)malloc(sizeof(cplx) * dim);
    if (!src) return ORC_ENOMEM;
    memcpy(src, psi, sizeof(cplx) * dim);
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        const uint64_t i = (uint64_t)ii;
        const int sel = (int)((i >> sel_lo) & 3u);
        const uint64_t j = (i >> q_lo) & (N - 1), rest = i & ~rmask;
        const uint64_t up = (j + 1) & (N - 1), dn = (j + N - 1) & (N - 1);
        cplx v;
        switch (sel) {
        case 0: v = src[rest | (up << q_lo)]; break;                              /* C       */
        case 1: v = (up == 0 ? -1.0 : 1.0) * src[rest | (up << q_lo)]; break;      /* C R0    */
        case 2: v = -src[rest | (dn << q_lo)]; break;                             /* -C^T    */
        default: v = -(j == 0 ? -1.0 : 1.0) * src[rest | (dn << q_lo)]; break;     /* -R0 C^T */
        }
        psi[i] = v;
    }
    free(src);
    if ((rc = orc_apply_gate(psi, n, sel_lo, h, NULL, NULL, 0)) != ORC_OK) return rc;
    return orc_apply_gate(psi, n, sel_lo + 1, h, NULL, NULL, 0);
}

/*
 * QPP velocity gradient in spectral space (appendix "Velocity gradients -
 * spectral method"), in the order its text gives: the inverse QFT on the
 * register (kernel exp(-2 pi i j k / N)), the diagonal
 *     Lambda_k = 2 pi i k (k < N/2),  0 (k = N/2),  2 pi i (k - N) (k > N/2),
 * then the QFT back.  Lambda is not unitary: it is applied as the |1> block
 * of a rotation of qubit `anc` controlled on the register value k,
 *     e^{i arg Lambda_k} Ry(t_k),  sin(t_k / 2) = |Lambda_k| / Lambda_max,
 * with Lambda_max = 2 pi (N/2 - 1), one multi-controlled gate per k.
 * With anc starting in |0>, its |1> component at the end is
 * F Lambda F^-1 phi / Lambda_max: d/dy of phi on the periodic grid y_j = j/N.
 * Needs m >= 2 (for N = 2 every Lambda_k is 0).
 */
int orc_spectral_derivative(cplx *psi, int n, int q_lo, int m, int anc)
{
    if (n < 3 || n > 40 || m < 2 || m > 30 || q_lo < 0 || q_lo + m > n) return ORC_EINVAL;
    if (anc < 0 || anc >= n || (anc >= q_lo && anc < q_lo + m)) return ORC_EINVAL;
    const uint64_t N = (uint64_t)1 << m;
    int rc = orc_qft(psi, n, q_lo, m, 1);
    if (rc != ORC_OK) return rc;
    const double lmax = 2.0 * ORC_PI * ((double)(N / 2) - 1.0);
    int ctrls[30], cvals[30];
    for (int b = 0; b < m; ++b) ctrls[b] = q_lo + b;
    for (uint64_t k = 0; k < N; ++k) {
        double mag, arg;
        if (k < N / 2) { mag = 2.0 * ORC_PI * (double)k; arg = ORC_PI / 2; }
        else if (k == N / 2) { mag = 0.0; arg = 0.0; }
        else { mag = 2.0 * ORC_PI * (double)(N - k); arg = -ORC_PI / 2; }
        if (mag == 0.0) continue;                                   /* identity */
        const double s = mag / lmax, c = sqrt(fmax(0.0, 1.0 - s * s));
        const cplx e = cexp(I * arg);
        const cplx u00 = c * e, u01 = -s * e, u10 = s * e, u11 = c * e;
        const double u[8] = {creal(u00), cimag(u00), creal(u01), cimag(u01),
                             creal(u10), cimag(u10), creal(u11), cimag(u11)};
        for (int b = 0; b < m; ++b) cvals[b] = (int)((k >> b) & 1u);
        if ((rc = orc_apply_gate(psi, n, anc, u, ctrls, cvals, m)) != ORC_OK) return rc;
    }
    return orc_qft(psi, n, q_lo, m, 0);
}

/*
 * The QSP-1 tree circuit of orc_qsp applied to the register [q_lo, q_lo + m)
 * of an arbitrary state (no initialisation), or its adjoint (inverse != 0:
 * the phase diagonal conjugated first, then the rotations transposed in
 * reverse order).  On a register in |0...0> the forward circuit prepares
 * b / |b| there.  Used as the PREP step of the LCU solver below.
 */
int orc_qsp_apply(cplx *psi, int n, int q_lo, int m, const cplx *b, int inverse)
{
    if (m < 1 || q_lo < 0 || q_lo + m > n || m > 24) return ORC_EINVAL;
    const uint64_t R = (uint64_t)1 << m;
    double *w = (double *)calloc(2 * R, sizeof(double));
    if (!w) return ORC_ENOMEM;
    double tot = 0.0;
    for (uint64_t r = 0; r < R; ++r) {
        w[R + r] = creal(b[r]) * creal(b[r]) + cimag(b[r]) * cimag(b[r]);
        tot += w[R + r];
    }
    if (!(tot > 0.0)) { free(w); return ORC_EINVAL; }
    for (uint64_t k = R - 1; k >= 1; --k) w[k] = w[2 * k] + w[2 * k + 1];
    int ctrls[32], cvals[32], rc = ORC_OK;
    /* the phase diagonal: diag(e^{i a}, 1) or diag(1, e^{i a}) on qubit q_lo
     * controlled on the other register qubits taking the value of r */
    for (int pass = 0; pass < 2 && rc == ORC_OK; ++pass) {
        const int phase_now = inverse ? pass == 0 : pass == 1;
        if (phase_now) {
            for (uint64_t r = 0; r < R && rc == ORC_OK; ++r) {
                if (w[R + r] == 0.0) continue;
                const double a = carg(b[r]) * (inverse ? -1.0 : 1.0);
                if (a == 0.0) continue;
                const cplx e = cexp(I * a);
                double u[8] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
                if (r & 1) { u[6] = creal(e); u[7] = cimag(e); }
                else { u[0] = creal(e); u[1] = cimag(e); }
                for (int j = 1; j < m; ++j) { ctrls[j - 1] = q_lo + j; cvals[j - 1] = (int)((r >> j) & 1); }
                rc = orc_apply_gate(psi, n, q_lo, u, ctrls, cvals, m - 1);
            }
        } else {
            for (int li = 0; li < m && rc == ORC_OK; ++li) {
                const int l = inverse ? m - 1 - li : li;        /* tree level */
                const int t = q_lo + m - 1 - l;
                for (int j = 0; j < l; ++j) ctrls[j] = q_lo + m - 1 - j;
                for (uint64_t p = 0; p < ((uint64_t)1 << l) && rc == ORC_OK; ++p) {
                    const uint64_t node = ((uint64_t)1 << l) + p;
                    if (!(w[node] > 0.0)) continue;
                    const double c = sqrt(w[2 * node] / w[node]), sn = sqrt(w[2 * node + 1] / w[node]);
                    const double sg = inverse ? -1.0 : 1.0;
                    for (int j = 0; j < l; ++j) cvals[j] = (int)((p >> (l - 1 - j)) & 1);
                    const double ry[8] = {c, 0.0, -sg * sn, 0.0, sg * sn, 0.0, c, 0.0};
                    rc = orc_apply_gate(psi, n, t, ry, ctrls, cvals, l);
                }
            }
        }
    }
    free(w);
    return rc;
}

/*
 * Chebyshev coefficients of the linear-systems solver by a linear
 * combination of unitaries (QLSA-2, built from the cited work of Childs,
 * Kothari and Somma, since the paper defers its details): the odd function
 *     g(x) = (1 - (1 - x^2)^B) / x = sum_{j=0}^{B-1} alpha_j T_{2j+1}(x),
 *     alpha_j = 4 (-1)^j sum_{i=j+1}^{B} C(2B, B+i) / 4^B,
 * approximates 1/x on [-1, -1/kappa] u [1/kappa, 1] to within (1 - 1/kappa^2)^B kappa.
 * alpha[0..J) are written (zero for j >= B).  The binomial weights
 * t_i = C(2B, B+i)/4^B come from t_0 = prod_{k=1}^{B} (2k-1)/(2k) and
 * t_{i+1} = t_i (B-i)/(B+i+1); the tails are summed from the small end.
 */
int orc_cks_coeffs(int B, int J, double *alpha)
{
    if (B < 1 || B > 20000000 || J < 1) return ORC_EINVAL;
    double *t = (double *)malloc(sizeof(double) * ((size_t)B + 2));
    if (!t) return ORC_ENOMEM;
    double t0 = 1.0;
    for (int k = 1; k <= B; ++k) t0 *= (2.0 * k - 1.0) / (2.0 * k);
    t[0] = t0;
    for (int i = 0; i < B; ++i) t[i + 1] = t[i] * (double)(B - i) / (double)(B + i + 1);
    t[B + 1] = 0.0;
    /* tail[i] = sum_{i' >= i} t_i', overwriting t from the top */
    double acc = 0.0;
    for (int i = B; i >= 0; --i) { acc += t[i]; t[i] = acc; }
    for (int j = 0; j < J; ++j) {
        const double tail = j + 1 <= B ? t[j + 1] : 0.0;
        alpha[j] = 4.0 * ((j & 1) ? -1.0 : 1.0) * tail;
    }
    free(t);
    return ORC_OK;
}

/*
 * QLSA-2 by Chebyshev LCU, gate level, in the order of the construction:
 *   layout: bits [0, n_s) system, bit n_s the walk qubit, bits
 *   [n_s + 1, n_s + 1 + s) the select register (J = 2^s terms);
 *   1. |0>_sel |0>_walk |b / |b|>;
 *   2. A~ = A / max|lambda|; U = [[A~, S], [S, -A~]] with S = sqrt(I - A~^2)
 *      (walk qubit = the high bit of the (walk, system) register), a block
 *      encoding of A~; the walk W = (Z on the walk qubit) U, whose walk-0 block
 *      of W^k is the Chebyshev polynomial T_k(A~);
 *   3. PREP: the QSP-1 tree on the select register with amplitudes
 *      sqrt(|alpha_j| / sum |alpha|);
 *   4. SELECT: W^(2j+1) on the (walk, system) register where the select
 *      register holds j;
 *   5. the signs (-1)^j: Z on the lowest select qubit;
 *   6. PREP^dagger;
 *   7. post-select select = 0 and walk = 0: z = the first 2^n_s amplitudes,
 *      z = sum_j alpha_j T_{2j+1}(A~) b^ / sum |alpha|, p = |z|^2.
 */
int orc_qlsa2(int n_s, int s, int B, const cplx *A, const cplx *b, cplx *psi, cplx *z_out, double *p_post)
{
    if (n_s < 1 || s < 1 || n_s + 1 + s > 26 || B < 1) return ORC_EINVAL;
    const int N = 1 << n_s, M = 2 * N, n = n_s + 1 + s, J = 1 << s;
    const uint64_t dim = (uint64_t)1 << n;
    double bn = 0.0;
    for (int j = 0; j < N; ++j) bn += creal(b[j] * conj(b[j]));
    bn = sqrt(bn);
    if (!(bn > 0.0)) return ORC_EINVAL;
    double *lam = (double *)malloc(sizeof(double) * N);
    double *alpha = (double *)malloc(sizeof(double) * J);
    cplx *V = (cplx *)malloc(sizeof(cplx) * (size_t)N * N);
    cplx *W = (cplx *)malloc(sizeof(cplx) * (size_t)M * M);
    cplx *pamp = (cplx *)malloc(sizeof(cplx) * J);
    cplx *u = (cplx *)malloc(sizeof(cplx) * M), *v = (cplx *)malloc(sizeof(cplx) * M);
    int rc = ORC_OK;
    if (!lam || !alpha || !V || !W || !pamp || !u || !v) { rc = ORC_ENOMEM; goto done; }
    /* 1 */
    memset(psi, 0, sizeof(cplx) * dim);
    for (int j = 0; j < N; ++j) psi[j] = b[j] / bn;
    /* 2: the walk operator */
    if ((rc = orc_eigh(N, A, lam, V)) != ORC_OK) goto done;
    {
        double lmax = 0.0;
        for (int k = 0; k < N; ++k) lmax = fmax(lmax, fabs(lam[k]));
        if (!(lmax > 0.0)) { rc = ORC_EINVAL; goto done; }
        for (int r = 0; r < N; ++r)
            for (int c = 0; c < N; ++c) {
                cplx a = 0, sq = 0;
                for (int k = 0; k < N; ++k) {
                    const double lt = lam[k] / lmax;
                    const cplx vv = V[(size_t)r * N + k] * conj(V[(size_t)c * N + k]);
                    a += lt * vv;
                    sq += sqrt(fmax(0.0, 1.0 - lt * lt)) * vv;
                }
                /* U = [[a, sq], [sq, -a]]; W = Z_walk U negates the walk = 1 rows */
                W[(size_t)r * M + c] = a;
                W[(size_t)r * M + (N + c)] = sq;
                W[(size_t)(N + r) * M + c] = -sq;
                W[(size_t)(N + r) * M + (N + c)] = a;
            }
    }
    /* 3: PREP */
    if ((rc = orc_cks_coeffs(B, J, alpha)) != ORC_OK) goto done;
    {
        double l1 = 0.0;
        for (int j = 0; j < J; ++j) l1 += fabs(alpha[j]);
        for (int j = 0; j < J; ++j) pamp[j] = sqrt(fabs(alpha[j]) / l1);
    }
    if ((rc = orc_qsp_apply(psi, n, n_s + 1, s, pamp, 0)) != ORC_OK) goto done;
    /* 4: SELECT, W applied 2j + 1 times to the (walk, system) vector of select value j */
    for (int j = 0; j < J; ++j) {
        const uint64_t off = (uint64_t)j << (n_s + 1);
        for (int i = 0; i < M; ++i) u[i] = psi[off + i];
        for (int rep = 0; rep < 2 * j + 1; ++rep) {
            for (int r = 0; r < M; ++r) {
                cplx acc = 0;
                for (int c = 0; c < M; ++c) acc += W[(size_t)r * M + c] * u[c];
                v[r] = acc;
            }
            memcpy(u, v, sizeof(cplx) * M);
        }
        for (int i = 0; i < M; ++i) psi[off + i] = u[i];
    }
    /* 5: signs */
    {
        const double z8[8] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0, 0.0};
        if ((rc = orc_apply_gate(psi, n, n_s + 1, z8, NULL, NULL, 0)) != ORC_OK) goto done;
    }
    /* 6: PREP^dagger */
    if ((rc = orc_qsp_apply(psi, n, n_s + 1, s, pamp, 1)) != ORC_OK) goto done;
    /* 7 */
    {
        double pp = 0.0;
        for (int k = 0; k < N; ++k) {
            z_out[k] = psi[k];
            pp += creal(psi[k] * conj(psi[k]));
        }
        *p_post = pp;
    }
done:
    free(lam); free(alpha); free(V); free(W); free(pamp); free(u); free(v);
    return rc;
}

/*
 * QLSA-2, Fourier form (the cited Childs-Kothari-Somma construction; the
 * paper defers it): the integral representation
 *     1/x = (i / sqrt(2 pi)) int_0^inf dy int_-inf^inf dz z e^{-z^2/2} e^{-i x y z}
 * discretised as h(x) = sum_{j,k} w_jk i sign(z_k) e^{-i x y_j z_k} with
 *     y_j = j dy (j < 2^sy),  z_k = k dz,  k = m + 1 (m < K) or m - 2K (m >= K),
 *     K = 2^(sz - 1),  w_jk = dy dz |z_k| e^{-z_k^2 / 2} / sqrt(2 pi),
 * an LCU of the unitaries i sign(z_k) exp(-i A~ y_j z_k), A~ = A / max|lambda|.
 *   layout: bits [0, n_s) system, [n_s, n_s + sy) the j register,
 *   [n_s + sy, n_s + sy + sz) the m register (select value r = j + 2^sy m);
 *   1. |0>_sel |b^>;  2. PREP: the QSP-1 tree with sqrt(w_r / |w|_1);
 *   3. SELECT: the unitary of term r on the system sub-vector of select r,
 *      exp(-i A~ t) = V diag(e^{-i lambda~ t}) V^dagger (the oracle's eigensolver);
 *   4. PREP^dagger;  5. post-select select = 0: z = h(A~) b^ / |w|_1.
 */
int orc_qlsa2_fourier(int n_s, int sy, int sz, double dy, double dz, const cplx *A, const cplx *b, cplx *psi,
                      cplx *z_out, double *p_post)
{
    if (n_s < 1 || sy < 1 || sz < 1 || n_s + sy + sz > 26 || !(dy > 0.0) || !(dz > 0.0)) return ORC_EINVAL;
    const int N = 1 << n_s, n = n_s + sy + sz, S = sy + sz;
    const uint64_t dim = (uint64_t)1 << n, R = (uint64_t)1 << S, Jn = (uint64_t)1 << sy;
    const int64_t K = (int64_t)1 << (sz - 1);
    double bn = 0.0;
    for (int j = 0; j < N; ++j) bn += creal(b[j] * conj(b[j]));
    bn = sqrt(bn);
    if (!(bn > 0.0)) return ORC_EINVAL;
    double *lam = (double *)malloc(sizeof(double) * N);
    cplx *V = (cplx *)malloc(sizeof(cplx) * (size_t)N * N);
    cplx *pamp = (cplx *)malloc(sizeof(cplx) * R);
    cplx *u = (cplx *)malloc(sizeof(cplx) * N), *v = (cplx *)malloc(sizeof(cplx) * N);
    int rc = ORC_OK;
    double lmax = 0.0, l1 = 0.0;
    if (!lam || !V || !pamp || !u || !v) { rc = ORC_ENOMEM; goto done; }
    memset(psi, 0, sizeof(cplx) * dim);
    for (int j = 0; j < N; ++j) psi[j] = b[j] / bn;
    if ((rc = orc_eigh(N, A, lam, V)) != ORC_OK) goto done;
    for (int k = 0; k < N; ++k) lmax = fmax(lmax, fabs(lam[k]));
    if (!(lmax > 0.0)) { rc = ORC_EINVAL; goto done; }
    /* the LCU weights */
    for (uint64_t r = 0; r < R; ++r) {
        const int64_t m = (int64_t)(r >> sy);
        const int64_t k = m < K ? m + 1 : m - 2 * K;
        const double zk = (double)k * dz;
        const double w = dy * dz * fabs(zk) * exp(-0.5 * zk * zk) / sqrt(2.0 * ORC_PI);
        pamp[r] = w;
        l1 += w;
    }
    for (uint64_t r = 0; r < R; ++r) pamp[r] = sqrt(creal(pamp[r]) / l1);
    /* PREP */
    if ((rc = orc_qsp_apply(psi, n, n_s, S, pamp, 0)) != ORC_OK) goto done;
    /* SELECT */
    for (uint64_t r = 0; r < R; ++r) {
        const uint64_t j = r & (Jn - 1);
        const int64_t m = (int64_t)(r >> sy);
        const int64_t k = m < K ? m + 1 : m - 2 * K;
        const double t = (double)j * dy * (double)k * dz;
        const cplx sgn = k > 0 ? I : -I;
        const uint64_t off = r << n_s;
        /* u = V^dagger psi_r, scaled by e^{-i lambda~ t}, then V u */
        for (int a = 0; a < N; ++a) {
            cplx acc = 0;
            for (int c = 0; c < N; ++c) acc += conj(V[(size_t)c * N + a]) * psi[off + c];
            u[a] = acc * cexp(-I * (lam[a] / lmax) * t);
        }
        for (int c = 0; c < N; ++c) {
            cplx acc = 0;
            for (int a = 0; a < N; ++a) acc += V[(size_t)c * N + a] * u[a];
            v[c] = sgn * acc;
        }
        for (int c = 0; c < N; ++c) psi[off + c] = v[c];
    }
    /* PREP^dagger */
    if ((rc = orc_qsp_apply(psi, n, n_s, S, pamp, 1)) != ORC_OK) goto done;
    {
        double pp = 0.0;
        for (int k = 0; k < N; ++k) {
            z_out[k] = psi[k];
            pp += creal(psi[k] * conj(psi[k]));
        }
        *p_post = pp;
    }
done:
    free(lam); free(V); free(pamp); free(u); free(v);
    return rc;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the following calls (the CPU baseline times 1 and all) */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
