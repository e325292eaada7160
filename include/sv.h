/*
 * sv.h -- C ABI of the MI355X state-vector library for gate-level HHL
 * (QLSA-1) as used for the Poiseuille / Couette flow systems of
 * "Hybrid quantum algorithms for flow problems" (arXiv:2307.00391).
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - A state on n qubits is a device array of 2^n complex amplitudes,
 *    interleaved (re, im): float2 for SV_C64, double2 for SV_C128.
 *    Qubit q is bit q of the basis index.  This order is the one fixed by
 *    the paper's worked two-qubit example U = H_1 (x) X_0 (appendix
 *    "QFlowS - a brief overview", gates and circuits); it is the reverse of
 *    the stride 2^(n-q-1) written in the same paragraph's Hadamard rule.
 *  - HHL register layout: bits [0, n_s) system register x, bits
 *    [n_s, n_s + n_c) clock register y, bit n_s + n_c the ancilla a.
 *  - One-qubit gates are row-major 2x2 complex matrices given as 8 host
 *    doubles (u00re, u00im, u01re, u01im, u10re, u10im, u11re, u11im) and act
 *    on each index pair (i0, i1 = i0 | 2^target) as
 *    (a_i0, a_i1) <- (u00 a_i0 + u01 a_i1, u10 a_i0 + u11 a_i1)
 *    (the "algebraic" pair update of the same appendix).  Gate matrices are
 *    taken in FP64; the SV_C64 path rounds them to FP32 once.
 *  - Every call enqueues its kernels on the state's HIP stream (borrowed;
 *    NULL = the null stream).  Calls that hand back host scalars or host
 *    vectors synchronise that stream before returning.
 *  - All functions return sv_status.  On a validation error nothing is
 *    enqueued and the state is unchanged; sv_last_error() returns a
 *    thread-local description of the last failure.
 *  - Pointers passed in are borrowed for the duration of the call only
 *    (device inputs must stay live until the stream has drained).
 *    The library owns sv_state handles and any buffer it allocated.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SV_OK = 0,
    SV_EINVAL = -1,          /* bad argument: qubit out of range, duplicate qubits, sizes */
    SV_ENOMEM = -2,          /* device allocation failed (or state larger than device memory) */
    SV_EDEVICE = -3,         /* HIP / library runtime error */
    SV_ENOTHERMITIAN = -4,   /* |A - A^H|_max > 1e-12 |A|_max */
    SV_ENOTPOSDEF = -5,      /* lambda_min <= 0 (the clock register is unsigned) */
    SV_EZERONORM = -6,       /* |b| = 0, or a post-selected outcome of probability 0 */
    SV_EUNSUPPORTED = -7     /* valid request outside what the library implements */
} sv_status;

typedef enum { SV_C64 = 1, SV_C128 = 2 } sv_dtype;

typedef struct sv_state_s *sv_state;   /* opaque; owned by the library */

/* ------------------------------------------------------------------------
 * State management
 * --------------------------------------------------------------------- */

/* Create a state of n_qubits (1..34) amplitudes of type dt.
 * device_buf: borrowed device memory of at least 2^n * sizeof(amplitude)
 * bytes (e.g. a torch tensor's storage), or NULL to let the library
 * allocate it (freed by sv_free).  hip_stream: a hipStream_t, or NULL.
 * The contents are left as found (use sv_init_basis / sv_init_b).
 * Errors: SV_EINVAL (n out of range), SV_ENOMEM, SV_EDEVICE. */
sv_status sv_alloc(sv_state *out, int n_qubits, sv_dtype dt, void *device_buf, void *hip_stream);

/* Release the handle (and the buffer if the library allocated it). */
sv_status sv_free(sv_state s);

/* Device pointer of the amplitudes, qubit count, dtype. */
void *sv_data(sv_state s);
int sv_num_qubits(sv_state s);
sv_dtype sv_get_dtype(sv_state s);
sv_status sv_set_stream(sv_state s, void *hip_stream);

/* |index>: one amplitude 1, all others 0. */
sv_status sv_init_basis(sv_state s, uint64_t index);

/* HHL initial state |0>_a (H^{(x)c}|0>)_clock |b/|b|>_system, where the
 * system register is bits [0, n_s) and c = n_clock_superpose clock qubits
 * occupy bits [n_s, n_s + c) (c = 0: the clock stays |0>).  All other bits
 * are |0>.  b: host, 2^n_s complex FP64 interleaved, not necessarily
 * normalised (state preparation, main text "Quantum State Preparation";
 * the clock superposition is the first layer of phase estimation).
 * Errors: SV_EINVAL (n_s + c > n), SV_EZERONORM (|b| = 0). */
sv_status sv_init_b(sv_state s, const double *b, int n_s, int n_clock_superpose);

/* Copy the whole state from / to host memory as complex FP64 interleaved
 * (2 * 2^n doubles); the SV_C64 path converts on the device. */
sv_status sv_set_state(sv_state s, const double *host);
sv_status sv_get_state(sv_state s, double *host);

/* ------------------------------------------------------------------------
 * Gates (appendix "QFlowS - a brief overview": gates applied as algebraic
 * pair updates without forming 2^n x 2^n matrices)
 * --------------------------------------------------------------------- */

/* One-qubit gate u on `target`, applied where every control qubit ctrls[i]
 * equals ctrl_vals[i] (ctrl_vals NULL: all 1).  A c-controlled gate touches
 * 2^(n-c) amplitudes.  When u is exactly X = [[0,1],[1,0]] the update is a
 * pure exchange of amplitudes (bit-exact); when u is diagonal only the
 * amplitudes whose phase changes are rewritten.
 * Errors: SV_EINVAL (qubit out of range or repeated, n_ctrls > 32). */
sv_status sv_apply_gate(sv_state s, int target, const double u[8], const int *ctrls,
                        const int *ctrl_vals, int n_ctrls);

/* Exchange of qubits q1 and q2 where the controls match (bit-exact). */
sv_status sv_apply_swap(sv_state s, int q1, int q2, const int *ctrls, const int *ctrl_vals,
                        int n_ctrls);

/* A gate of a circuit passed to sv_apply_circuit. */
typedef enum {
    SV_GATE_U = 0,      /* dense one-qubit u on target (diagonal u allowed) */
    SV_GATE_X = 1,      /* bit-exact X on target (with controls: CNOT, Toffoli, ...) */
    SV_GATE_SWAP = 2    /* bit-exact exchange of target and target2 */
} sv_gate_kind;

#define SV_MAX_CTRLS 8
typedef struct {
    int kind;                        /* sv_gate_kind */
    int target, target2;             /* target2 only for SV_GATE_SWAP */
    int n_ctrls;
    int ctrls[SV_MAX_CTRLS];
    int ctrl_vals[SV_MAX_CTRLS];
    double u[8];                     /* SV_GATE_U only */
} sv_gate;

/* Apply gates[0..n_gates) in order.  The library groups the circuit into
 * passes: each pass stages tiles of 2^k amplitudes (k "local" qubits: the
 * lowest few bits plus the targets it needs) in LDS and applies every gate
 * it can there, so a run of g gates costs one read and one write of the
 * state instead of g.  Gates are only moved past gates on disjoint qubits;
 * the result equals the in-order product.  max_local <= 0 lets the
 * autotuner choose k.  A pass runs as many workgroups as the device holds at
 * once, each walking a strided run of tiles; SV_FUSED_PERSIST=0 launches one
 * workgroup per tile instead (same results, bit for bit). */
sv_status sv_apply_circuit(sv_state s, const sv_gate *gates, int n_gates, int max_local);

/* Number of fused passes sv_apply_circuit would run (planning only). */
int sv_plan_passes(int n_qubits, sv_dtype dt, const sv_gate *gates, int n_gates, int max_local);

/* Controlled dense unitary on the contiguous register [sys_lo, sys_lo + m):
 * for every setting of the other qubits with qubit ctrl == ctrl_val
 * (ctrl < 0: unconditional) the 2^m sub-vector v becomes U v, or U^H v if
 * `adjoint`.  U: device, 2^m x 2^m, row-major, in the state's dtype.  This
 * is the controlled-U^(2^k) of phase estimation (main text: the operator is
 * exponentiated as exp(i A T0)), computed as a complex GEMM on the matrix
 * cores; element k of a row sits at stride 2^sys_lo, so for sys_lo > 0 the
 * GEMM reads 64 neighbouring rows per wavefront instead of a contiguous row.
 * Errors: SV_EINVAL (register outside the state, ctrl inside it),
 * SV_EUNSUPPORTED (m > 16), SV_ENOMEM (the staging buffer of rows x 2^m
 * amplitudes that the product is written to before the scatter). */
sv_status sv_apply_ctrl_unitary(sv_state s, const void *U, int sys_lo, int m, int ctrl,
                                int ctrl_val, int adjoint);

/* Quantum Fourier transform on qubits [q_lo, q_lo + m):
 * QFT|j> = 2^(-m/2) sum_k exp(+2 pi i j k / 2^m) |k>, inverse with
 * exp(-2 pi i j k / 2^m) (QFT / IQFT kernels of the appendix on spectral
 * velocity gradients).  swaps = 1 gives exact DFT index order (the
 * textbook final bit reversal, bit-exact); swaps = 0 leaves the register
 * bit-reversed (the QFT) or expects it bit-reversed (the inverse).
 * max_local as in sv_apply_circuit. */
sv_status sv_qft(sv_state s, int q_lo, int m, int inverse, int swaps, int max_local);

/* Uniformly controlled Ry: for each value v of the register [reg_lo,
 * reg_lo + m), rotate qubit `target` by the real 2x2 [[c_v, -s_v], [s_v, c_v]]
 * with (c_v, s_v) = cs[2v], cs[2v+1] (host FP64, 2^(m+1) doubles).  With
 * s_v = C / lambda~_v this is the eigenvalue-inversion rotation of HHL.
 * extra_ctrl >= 0 restricts it to indices whose qubit extra_ctrl equals
 * extra_val. */
sv_status sv_apply_uniform_ry(sv_state s, int target, int reg_lo, int m, const double *cs,
                              int extra_ctrl, int extra_val);

/* ------------------------------------------------------------------------
 * Measurement-side reductions (FP64 accumulation)
 * --------------------------------------------------------------------- */

/* sum |a_i|^2 over indices with (i & mask) == value, accumulated in FP64
 * with a fixed reduction order (repeatable bit for bit). */
sv_status sv_norm2(sv_state s, uint64_t mask, uint64_t value, double *out);

/* Post-selection of the outcome (i & mask) == value (main text: the
 * post-selected state of the QLSA output).  *prob = its probability (FP64).
 * out (may be NULL): 2^(n - popcount(mask)) complex amplitudes in
 * increasing index order, divided by sqrt(prob); complex FP64 on the host
 * if out_on_device == 0, else the state's dtype on the device.
 * Errors: SV_EINVAL (value outside mask), SV_EZERONORM (prob == 0). */
sv_status sv_postselect(sv_state s, uint64_t mask, uint64_t value, double *prob, void *out,
                        int out_on_device);

/* The post-selection of sv_postselect with every result left on the device,
 * for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  It calls no
 * hipMalloc, hipFree or allocating library routine and never synchronises.
 *   prob_dev: device, 1 double (caller-owned): P((i & mask) == value), FP64,
 *             summed in the same fixed order as sv_postselect (the same bits).
 *   out_dev:  device (caller-owned, may be NULL): 2^(n - popcount(mask))
 *             amplitudes in the state's dtype, increasing index order, divided
 *             by sqrt(*prob_dev).  A zero probability is not detected (the
 *             call is asynchronous): out_dev then holds inf/NaN; check *prob_dev.
 * Workspace: a fixed array of 4096 + 64 doubles (33 KiB) per device in the
 * library's static device memory, held until the process ends; the reduction
 * never needs more than 4096 partial sums, so every state size fits.  Calls
 * that overlap on one device (different host threads or streams) share that
 * array and race; serialise them.  Enqueued on the state's stream.
 * Errors: SV_EINVAL (NULL prob_dev, value outside mask), SV_EDEVICE. */
sv_status sv_postselect_noalloc(sv_state s, uint64_t mask, uint64_t value, double *prob_dev, void *out_dev);

/* ------------------------------------------------------------------------
 * HHL (QLSA-1, main text "Quantum Linear Systems Algorithm"; phase
 * estimation with exp(i A T0) and least count 2^-n_c, "Flow simulation
 * results")
 * --------------------------------------------------------------------- */

typedef struct {
    int n_s;       /* system qubits: A is 2^n_s x 2^n_s */
    int n_c;       /* clock (phase-estimation) qubits */
    double T0;     /* clock bit k applies exp(i A T0 2^k); y = 2^n_c lambda T0 / 2 pi */
    int mode;      /* 0: gate-faithful (dense controlled-U_k on the matrix cores, every
                      step on the full state);
                      1: eigen-frame, fused: the system register is held in the eigenbasis
                      of A, so the controlled-U_k are diagonal; the state after phase
                      estimation is generated inside the first inverse-QFT kernel, the
                      rotation sits between the two halves of the clock transforms, and
                      the uncompute ends in the clock = 0 projection: three passes over
                      half the state (n_c <= 20; larger n_c runs as mode 2);
                      2: eigen-frame, one kernel per step (state write, inverse QFT on
                      the ancilla = 0 half, rotation into the ancilla = 1 half, QFT there,
                      projection) */
    int signed_clock;  /* 0: unsigned clock, A must be positive definite;
                          1: two's-complement clock, y >= 2^(n_c-1) stands for
                          y - 2^n_c, so negative eigenvalues invert with their sign
                          (A Hermitian and non-singular, e.g. the Hermitian dilation
                          [[0, M], [M^H, 0]] of a non-Hermitian M); choose T0 so
                          that |lambda| T0 / 2 pi < 1/2 */
} sv_hhl_params;

typedef struct {
    double p_post;      /* P(ancilla = 1, clock = 0), FP64 */
    double p_anc;       /* P(ancilla = 1) after the inversion rotation, FP64 */
    double norm_total;  /* squared norm of the state after the rotation, FP64 */
    double lambda_min, lambda_max;   /* spectrum edges of A (FP64 eigen-decomposition) */
} sv_hhl_result;

/* Solve A x = b by simulating the HHL circuit on the state s, which must
 * hold n_s + n_c + 1 qubits.  Steps: |0>_a H^{(x)n_c}|0>_c |b^>_s; for
 * k = 0..n_c-1 controlled on clock bit k apply U_k = V diag(exp(2 pi i
 * frac(phi_j 2^k))) V^H with phi_j = lambda_j T0 / 2 pi (FP64
 * eigen-decomposition A = V diag(lambda) V^H); inverse QFT on the clock;
 * for clock value y >= 1 rotate the ancilla by Ry(theta_y) with
 * sin(theta_y / 2) = 1 / y (inversion constant C = least count
 * 2 pi / (2^n_c T0)), y = 0 untouched; QFT; controlled U_k^H for
 * k = n_c-1..0; H^{(x)n_c}; post-select ancilla = 1, clock = 0.
 * A: host, 2^n_s x 2^n_s complex FP64 row-major, Hermitian.  b: host,
 * 2^n_s complex FP64.  x_out (may be NULL): host, 2^n_s complex FP64, the
 * post-selected system vector divided by sqrt(p_post) (global phase as the
 * circuit leaves it).  After mode 0 the state holds the final circuit state;
 * after modes 1 and 2 its contents are unspecified.
 * Errors: SV_EINVAL, SV_ENOTHERMITIAN, SV_ENOTPOSDEF, SV_EZERONORM (|b| = 0 or
 * p_post = 0), SV_ENOTPOSDEF (lambda_min <= 0 with signed_clock = 0), SV_EINVAL
 * (a zero eigenvalue with signed_clock = 1), SV_ENOMEM, SV_EDEVICE. */
sv_status sv_hhl(sv_state s, const double *A, const double *b, const sv_hhl_params *prm,
                 sv_hhl_result *res, double *x_out);

typedef struct {
    int n_s, n_c;      /* system and clock qubits */
    double T0;         /* as sv_hhl_params */
    int mode;          /* 0, 1, 2 as sv_hhl_params */
    int signed_clock;  /* as sv_hhl_params (a zero eigenvalue is allowed here) */
    uint64_t cut;      /* flag clock values with |y| >= cut: 1 <= cut < 2^n_c,
                          or < 2^(n_c-1) with a signed clock */
} sv_gpe_params;

/* Gapped phase estimation: the building block of the variable-time
 * linear-systems solver in the Childs-Kothari-Somma construction that the
 * paper names for QLSA-2.  It decides, coherently and per eigenvector of A,
 * whether |lambda| T0 2^n_c / 2 pi lies above or below the cut, with a gap of
 * a few clock units in which both answers mix.  The circuit is that of
 * sv_hhl with the inversion rotation replaced by a flag on the ancilla
 * position: Ry(pi), |0> -> |1>, for clock values |y| >= cut, nothing
 * elsewhere; then the phase estimation is uncomputed.  An eigenvector whose
 * estimate lies well above the cut ends with flag 1 and clock 0, one well
 * below it with flag 0 and clock 0.  The state must hold n_s + n_c + 1 qubits
 * (flag bit n_s + n_c).
 * Results as sv_hhl: p_post = P(flag = 1, clock = 0), p_anc = P(flag = 1),
 * x_out the normalised flag = 1, clock = 0 system vector; after mode 0 the
 * state holds the final circuit state (the flag = 0, clock = 0 block is the
 * other branch).  A: host, 2^n_s x 2^n_s complex FP64 row-major, Hermitian,
 * n_s <= 13; b: host, 2^n_s complex FP64.
 * Errors: SV_EINVAL (sizes, T0, cut out of range), SV_ENOTHERMITIAN,
 * SV_ENOTPOSDEF (a negative eigenvalue on an unsigned clock), SV_EZERONORM
 * (|b| = 0, or no amplitude with flag 1 at clock 0), SV_ENOMEM, SV_EDEVICE. */
sv_status sv_gapped_pe(sv_state s, const double *A, const double *b, const sv_gpe_params *prm,
                       sv_hhl_result *res, double *x_out);

/* Classical preprocessing and the quantum solve, split so the FP64
 * eigen-decomposition is computed once per operator and reused for every
 * right-hand side and every T0 (the hybrid loop of the paper's Fig. 1b: the
 * parameters beta, here the spectrum and T0, are prepared classically).
 * sv_hhl_prepare: A = A_hi (x) I + I (x) A_lo with A_hi 2^m_hi and A_lo
 * 2^m_lo square (host, complex FP64 row-major, Hermitian), or the dense
 * A = A_hi when A_lo == NULL and m_lo == 0.  Uses the stream and staging
 * buffers of s; the plan then serves any state with n_s = m_hi + m_lo
 * system qubits on the same device.  Errors: SV_EINVAL, SV_ENOTHERMITIAN,
 * SV_EUNSUPPORTED (a factor above 2^13), SV_EDEVICE (no eigen-solver result
 * passed the residual check), SV_ENOMEM. */
typedef struct sv_hhl_plan_s *sv_hhl_plan;
sv_status sv_hhl_prepare(sv_hhl_plan *out, sv_state s, const double *A_hi, int m_hi, const double *A_lo,
                         int m_lo);
/* A plan from an eigen-decomposition the caller has already computed:
 * A = V diag(lam) V^T with V real orthogonal (the classical preprocessing of
 * the hybrid loop, done outside the library).  For operators whose
 * eigenbasis is dense and too large for sv_hhl_prepare's solvers (n_s up to
 * 16: a 2^16 x 2^16 V is 32 GiB): the basis changes of modes 1 and 2 then run
 * as two FP64 matrix-vector products over V, each reading V once from HBM.
 *   V_dev: device, 2^n_s x 2^n_s FP64 row-major, column j the eigenvector of
 *          lam[j]; borrowed for the plan's lifetime (not copied), unchanged.
 *   lam:   host, 2^n_s FP64 eigenvalues (any order, copied).
 * Checked: V V^T r = r to 1e-10 relative for a fixed pseudo-random r.  Mode 0
 * (gate-faithful) is available for n_s <= 13.  Errors: SV_EINVAL (sizes, NULL,
 * non-finite lam, V not orthogonal), SV_ENOMEM, SV_EDEVICE. */
sv_status sv_hhl_prepare_eig(sv_hhl_plan *out, sv_state s, const double *V_dev, const double *lam, int n_s);
/* One HHL solve on a prepared operator; arguments and results as sv_hhl.
 * The plan keeps device workspaces between calls: calls sharing a plan must
 * not overlap. */
sv_status sv_hhl_run(sv_hhl_plan p, sv_state s, const double *b, const sv_hhl_params *prm,
                     sv_hhl_result *res, double *x_out);
/* sv_hhl_run with the right-hand side and the solution in device memory, so
 * that a solve moves no vector over PCIe: b_dev is a device array of 2^n_s
 * complex FP64 (interleaved, need not be normalised; its norm is reduced on
 * the device), x_dev (may be NULL) a device array of 2^n_s complex FP64 that
 * receives the normalised post-selected vector; both are borrowed and stay on
 * the state's stream.  Only the result scalars are copied back (the call
 * synchronises the stream).  Modes 1 and 2 only (mode 0 starts from a host
 * b); other arguments, results and errors as sv_hhl_run, with SV_EUNSUPPORTED
 * for mode 0 and SV_EZERONORM when |b| = 0 or p_post = 0. */
sv_status sv_hhl_run_device(sv_hhl_plan p, sv_state s, const void *b_dev, const sv_hhl_params *prm,
                            sv_hhl_result *res, void *x_dev);
/* Smallest and largest eigenvalue of the prepared operator (FP64). */
sv_status sv_hhl_plan_spectrum(sv_hhl_plan p, double *lambda_min, double *lambda_max);
sv_status sv_hhl_plan_free(sv_hhl_plan p);

/* Gapped phase estimation on a prepared operator (sv_hhl_prepare, including
 * the Kronecker-sum form, so n_s is bounded by the plan, not by 13): arguments,
 * results and errors as sv_gapped_pe, with the plan's errors as sv_hhl_run. */
sv_status sv_gapped_pe_run(sv_hhl_plan p, sv_state s, const double *b, const sv_gpe_params *prm,
                           sv_hhl_result *res, double *x_out);

/* HHL for a separable operator A = A_hi (x) I + I (x) A_lo (a Laplacian /
 * Poisson operator on a 2-D tensor grid, main text: "d-dimensional Laplace,
 * Poisson and heat equations"), A_hi 2^m_hi square acting on system bits
 * [m_lo, n_s), A_lo 2^m_lo square on bits [0, m_lo), n_s = m_hi + m_lo.
 * The eigen-decomposition is taken factor by factor (V = V_hi (x) V_lo,
 * lambda = mu_p + nu_q), so n_s = 16 needs two 256-point solves instead of
 * one 65536-point one.  Only mode 1 is implemented for n_s > 12.
 * Other arguments and results as sv_hhl. */
sv_status sv_hhl_kron(sv_state s, const double *A_hi, int m_hi, const double *A_lo, int m_lo,
                      const double *b, const sv_hhl_params *prm, sv_hhl_result *res,
                      double *x_out);

/* ------------------------------------------------------------------------
 * Instrumentation
 * --------------------------------------------------------------------- */

/* Per-kernel tracing: while enabled, each state-vector kernel launch is
 * bracketed by HIP events recorded on the stream it runs on, together with
 * the algorithmic bytes (reads + writes the operation must make) and flops
 * of that launch.  on != 0 clears earlier records and starts recording. */
sv_status sv_trace_enable(int on);

/* Synchronises the device and writes one line per kernel name,
 * "name launches total_ms algorithmic_bytes flops", into buf (NUL
 * terminated, truncated to len).  Returns the full report length. */
int sv_trace_report(char *buf, int len);

/* The autotuner's current choices, one line per tuned shape:
 * "op/dtype/shape... values".  Tuning runs on first use of a shape
 * (SV_AUTOTUNE=0: defaults); SV_TUNE_CACHE=<file> persists the choices.
 *   eigpipe/<dtype>/<n_s>/<n_c>  fused eigen-frame kernels: (log2 columns
 *       per tile, threads per workgroup) for each of the three kernels;
 *   cgemm/<dtype>/<M>/<N>/<K>/<trans>  the matrix-core GEMM's tile shape:
 *       0 = 64 x 64 per workgroup, 1 = 16 x 16 per wavefront;
 *   fused/<dtype>/<n>/<circuit>  sv_apply_circuit with max_local = 0: (k
 *       local qubits, c contiguous low bits, rb register bits per segment
 *       line: 5 or 4 for complex64, 4 or 3 for complex128) per circuit
 *       structure; an entry of (k, c) takes the default rb.
 * Returns the report length. */
int sv_tune_report(char *buf, int len);
/* Sets (n > 0: vals[0..n)) or removes (n == 0) one tuning entry, with the key
 * format of sv_tune_report: pins a configuration (tests run every candidate
 * this way).  A pinned entry is used as it is.  Errors: SV_EINVAL. */
sv_status sv_tune_set(const char *key, const int *vals, int n);

/* Name of the rocSOLVER routine whose eigen-decomposition was used by the
 * calling thread's last HHL call (each result is accepted only after a
 * residual check A V x = V diag(lambda) x, |V x| = |x| on a fixed vector;
 * real symmetric A goes to the real routines).  "" before the first call. */
const char *sv_last_eigensolver(void);

/* QSP-1, the binary-tree state preparation of the appendix "Quantum State
 * Preparation" (Grover-Rudolph, in Prakash's binary-tree form): prepares
 * b / |b| on the register [q_lo, q_lo + m) (register value r: bit j of r is
 * qubit q_lo + j), every other qubit |0>, overwriting the whole state.
 * Tree: leaf r carries |b_r|^2, an inner node the sum of its two children;
 * level l (0 = root) decides qubit q_lo + m - 1 - l, and node p of level l
 * (the value of the l qubits above it) is the gate
 * Ry(t) = [[cos t/2, -sin t/2], [sin t/2, cos t/2]] with
 * cos^2(t/2) = zero-child / node weight, controlled on those qubits taking
 * the value p (no gate for a node of weight 0).  A diagonal over the
 * register then restores arg(b_r).  All angles are computed on the host in
 * FP64 and rounded once to the state's precision.
 *   mode 0: the circuit gate by gate: |0...0>, one Ry on the top qubit, one
 *           uniformly controlled Ry pass per further level, the diagonal;
 *   mode 1: the same circuit applied to |0...0> in one write pass (each
 *           amplitude is the product of the rotation entries on its path).
 * b: host, 2^m complex FP64 interleaved, borrowed.  1 <= m <= 26.
 * Synchronises the state's stream.  Errors: SV_EINVAL (register, mode,
 * non-finite b), SV_EZERONORM (b = 0), SV_ENOMEM. */
sv_status sv_qsp_prepare(sv_state s, const double *b, int q_lo, int m, int mode);

/* QPP velocity gradient by a linear combination of unitaries (appendix
 * "Velocity gradients - LCU method"; the derivative module of the main
 * text's "Quantum Post-processing Protocol").  The finite-difference
 * operator is the central first difference with zero Dirichlet walls on the
 * N = 2^m points of the register [q_lo, q_lo + m) (point j = register value
 * j): (D u)_j = (u_{j+1} - u_{j-1}) / 2h, u_{-1} = u_N = 0.  With the cyclic
 * shift (C u)_j = u_{(j+1) mod N} and R0 = I - 2|0><0|, 4h D = C + C R0 - C^T
 * - R0 C^T: four unitaries of equal weight.  The circuit on the select
 * qubits [sel_lo, sel_lo + 2) (select value i = bit sel_lo + 2 * bit
 * sel_lo+1) is V^dagger G V, V = H (x) H, G = sum_i |i><i| (x) U_i with
 * U = (C, C R0, -C^T, -R0 C^T).  It is unitary and acts on any input; from
 * select |00> the select-|00> block becomes h D u = (S - S^T) u / 2 (S the
 * truncated shift), so the probability of select = 00 is h^2 |D u|^2 / |u|^2.
 *   mode 0: gate by gate (Hadamards, multi-controlled X cascades for C and
 *           C^T, a multi-controlled phase for R0, one Z for the signs);
 *   mode 1: the whole circuit in one read and one write of the state (LDS
 *           tiles).  A register wider than 11 qubits (complex64) or 10
 *           (complex128) is cut into chunks of its low bits, and a first
 *           small kernel copies the two outside neighbours of every chunk
 *           into the state's scratch memory (2^(n - 10) or 2^(n - 9)
 *           amplitudes).
 * Errors: SV_EINVAL (register or select outside the state, overlapping,
 * m > 30, mode), SV_ENOMEM (scratch). */
sv_status sv_lcu_derivative(sv_state s, int q_lo, int m, int sel_lo, int mode);

/* QPP velocity gradient in spectral space (appendix "Velocity gradients -
 * spectral method"), in the order its text gives: inverse QFT on the
 * register [q_lo, q_lo + m) (exact index order), the wavenumber diagonal
 * Lambda_k = 2 pi i k (k < N/2), 0 (k = N/2), 2 pi i (k - N) (k > N/2), and
 * the QFT back.  Lambda is applied as the |1> block of a rotation of qubit
 * `anc` controlled on the register value k: e^{i arg Lambda_k} Ry(t_k) with
 * sin(t_k/2) = |Lambda_k| / Lambda_max, Lambda_max = 2 pi (N/2 - 1).  From
 * anc = |0>, the anc = 1 block ends as (du/dy) / Lambda_max on the periodic
 * grid y_j = j / N.  max_local as in sv_apply_circuit.
 * Errors: SV_EINVAL (m < 2 or > 30, register outside the state, anc inside
 * the register or outside the state). */
sv_status sv_spectral_derivative(sv_state s, int q_lo, int m, int anc, int max_local);

/* QPP nonlinear transform (appendix "Nonlinear transform", steps 1-5): the
 * amplitudes of a real 2^n-point state zeta = u/|u| become their squares on
 * an output qubit.  Qubits of the state (3n + r + 2 in all): ua [0, n) (the
 * loaded amplitudes), a1 [n, 2n) (the address copy), add [2n, 3n) (the
 * address), a2 = 3n (the SWAP-test qubit), ub [3n+1, 3n+1+r) (phase
 * estimation), up = 3n+1+r (the output).  The circuit, from |0...0>:
 *   1. H on add, CNOT add_j -> a1_j;
 *   2-3. W = T U_V: U_V loads zeta on ua (the real Householder reflection
 *      I - 2 v v^T / v^T v, v = e_0 + sigma zeta, sigma = +1 if zeta_0 >= 0
 *      else -1, so U_V|0> = -sigma zeta), T = H(a2) CSWAP(ua <-> a1 | a2)
 *      H(a2), the SWAP test, whose a2 = 0 part has probability
 *      (1 + zeta_s^2) / 2 = sin^2(pi beta_s) at address s;
 *   4. phase estimation on ub of the amplitude-estimation iterate
 *      Q = -W S_0 W^H S_chi (S_chi: sign of a2 = 0; S_0: sign of ua = 0,
 *      a1 = address, a2 = 0): H on ub, controlled Q^(2^k), inverse QFT;
 *   5. Ry on up for ub = y with sine -cos(2 pi y / 2^r) (cosine |sin|), then
 *      phase estimation, W and the address copy undone.
 * The up = 1 amplitude at address s with every ancilla at 0 is
 * g_s / sqrt(2^n), g_s = zeta_s^2 when beta_s lies on the 2^-r grid and
 * within 2 / 2^r of it otherwise.
 *   mode 0: gate by gate (U_V on the matrix cores, 2^r - 1 controlled
 *           iterates and as many inverse ones);
 *   mode 1: each (add, ub, up) column's controlled powers applied as Q^t
 *           (t = its ub value) in LDS in one pass, and the same for the
 *           uncompute; n <= 6.
 * avg != 0 ends with U_avg = H on add, so the up = 1, all-zero amplitude is
 * (1/2^n) sum_s g_s.  u: host, 2^n FP64 values, borrowed.  sq_out (host,
 * 2^n doubles, may be NULL): sqrt(2^n) times the real part of the up = 1,
 * ancillas = 0 amplitudes, i.e. g_s.  The final state stays in s.
 * Synchronises the state's stream.  Errors: SV_EINVAL (n outside 1..10, r
 * outside 1..16, 3n + r + 2 != the state's qubits, mode, non-finite u),
 * SV_EZERONORM (u = 0), SV_EUNSUPPORTED (mode 1 with n > 6), SV_ENOMEM. */
typedef struct {
    double p_sq;   /* P(up = 1, every ancilla 0) before U_avg = (1/2^n) sum_s g_s^2 */
    double p_up;   /* P(up = 1) before U_avg */
    double avg;    /* with avg: the real up = 1, all-zero amplitude after U_avg */
} sv_qadc_result;
sv_status sv_qadc_square(sv_state s, const double *u, int n, int r, int mode, int avg, double *sq_out,
                         sv_qadc_result *res);

/* ------------------------------------------------------------------------
 * QLSA-2 (main text, "Quantum Linear Systems Algorithm": the solver family
 * built on a linear combination of unitaries, after the cited work of
 * Childs, Kothari and Somma; the paper defers the construction, which is
 * taken here in its Chebyshev form)
 * --------------------------------------------------------------------- */

typedef struct {
    int n_s;    /* system qubits: A is 2^n_s x 2^n_s (1..13) */
    int s;      /* select qubits: J = 2^s Chebyshev terms (1..24) */
    int B;      /* the polynomial (1 - (1 - x^2)^B) / x; B >= kappa^2 ln(kappa / eps)
                   makes it eps-close to 1/x on 1/kappa <= |x| <= 1 (1..2e7) */
    int mode;   /* 0: the circuit in the computational basis (PREP as the QSP-1 tree
                      of uniformly controlled Ry passes, W once and one controlled
                      W^(2^(m+1)) per select qubit as dense unitaries of the
                      (walk, system) register on the matrix cores, the sign gate,
                      PREP^dagger);
                   1: the same circuit with the system register in the eigenbasis
                      of A: one pass writes the state after PREP, SELECT and the
                      signs, one FP64 reduction forms the select = 0 projection */
} sv_qlsa2_params;

typedef struct {
    double p_post;          /* P(select = 0, walk = 0), FP64 */
    double lambda_abs_max;  /* max |lambda(A)|: A~ = A / lambda_abs_max */
    double lambda_abs_min;  /* min |lambda(A)|: kappa = lambda_abs_max / lambda_abs_min */
    double alpha_l1;        /* sum_j |alpha_j| of the J terms used */
} sv_qlsa2_result;

/* Solve A x = b with the Chebyshev LCU solver on the state s, which must have
 * n_s + 1 + s qubits: bits [0, n_s) system, bit n_s the walk qubit, bits
 * [n_s + 1, n_s + 1 + s) the select register.  A~ = A / max|lambda| is
 * block-encoded as U = [[A~, S], [S, -A~]], S = sqrt(I - A~^2) (walk qubit =
 * the high bit of the (walk, system) register); the walk W = (Z on the walk
 * qubit) U has T_k(A~) as its walk = 0 block of W^k.  alpha_j = 4 (-1)^j
 * sum_{i=j+1}^{B} C(2B, B+i) / 4^B, j < J (zero for j >= B), so that
 * sum_j alpha_j T_{2j+1}(x) is (1 - (1 - x^2)^B) / x when J >= B.  The circuit:
 * |0>_sel |0>_walk |b^>, PREP (select amplitudes sqrt(|alpha_j| / |alpha|_1)),
 * SELECT W^(2j+1), Z on the lowest select qubit (the signs), PREP^dagger.
 * z_out (host, 2^n_s complex FP64 interleaved, may be NULL) receives the
 * select = 0, walk = 0 amplitudes, unnormalised and in the computational
 * basis: z = sum_j alpha_j T_{2j+1}(A~) b^ / |alpha|_1, p_post = |z|^2.
 * A: host, 2^n_s x 2^n_s complex FP64 row-major, Hermitian, non-zero.
 * After mode 0 the state holds the final circuit state; after mode 1 it holds
 * the state after the signs, in the eigen frame.  Synchronises the stream.
 * Errors: SV_EINVAL (sizes, B, mode, A = 0), SV_ENOTHERMITIAN,
 * SV_EZERONORM (b = 0), SV_ENOMEM, SV_EDEVICE. */
sv_status sv_qlsa2(sv_state s, const double *A, const double *b, const sv_qlsa2_params *prm,
                   sv_qlsa2_result *res, double *z_out);

typedef struct {
    int n_s;        /* system qubits (1..13; 1..10 in mode 0) */
    int sy, sz;     /* select registers: j < 2^sy, and m < 2^sz for z_k (sy + sz <= 30; <= 24 in mode 0) */
    double dy, dz;  /* grid steps of the two integrals */
    int mode;       /* 0: the circuit in the computational basis; 1: the eigen frame */
} sv_qlsa2f_params;

/* QLSA-2 in Fourier form: the integral representation
 * 1/x = (i / sqrt(2 pi)) int_0^inf dy int dz z e^{-z^2/2} e^{-i x y z}, discretised
 * as h(x) = sum_{j,k} w_jk i sign(z_k) e^{-i x y_j z_k}, y_j = j dy (j < 2^sy),
 * z_k = k dz with k = m + 1 (m < 2^(sz-1)) or m - 2^sz, w_jk = dy dz |z_k|
 * e^{-z_k^2/2} / sqrt(2 pi): a linear combination of the unitaries
 * i sign(z_k) exp(-i A~ y_j z_k), A~ = A / max|lambda|.  The state must have
 * n_s + sy + sz qubits: bits [0, n_s) system, [n_s, n_s + sy) the j register,
 * [n_s + sy, n_s + sy + sz) the m register.  The circuit (PREP with
 * sqrt(w / |w|_1), SELECT, PREP^dagger, post-selection of select = 0) runs
 *   mode 0: gate by gate in the computational basis: PREP and PREP^dagger as
 *           the QSP-1 tree of uniformly controlled Ry passes; SELECT as
 *           diag(i, -i) on the top m qubit (the factor i sign(z)) and, since
 *           j k is bilinear in the bits of j and m, sy (sz + 1) singly or
 *           doubly controlled dense exp(-i A~ dy dz t) on the matrix cores;
 *           the state holds the final circuit state afterwards;
 *   mode 1: with the system register in the eigenbasis of A: one pass writes
 *           the state after SELECT, one FP64 reduction forms the select = 0
 *           projection; the state's contents are unspecified afterwards.
 * z_out as in sv_qlsa2: z = h(A~) b^ / |w|_1 in the computational basis,
 * p_post = |z|^2; alpha_l1 of the result holds |w|_1.  Synchronises the stream.
 * Errors: SV_EINVAL (sizes, steps, A = 0), SV_ENOTHERMITIAN, SV_EZERONORM,
 * SV_EUNSUPPORTED (mode 0 beyond its sizes), SV_ENOMEM, SV_EDEVICE. */
sv_status sv_qlsa2_fourier(sv_state s, const double *A, const double *b, const sv_qlsa2f_params *prm,
                           sv_qlsa2_result *res, double *z_out);

/* ------------------------------------------------------------------------
 * Batched T0 sweep (the T Q phase-diagram scans of Fig. 3c and the T0*-kappa
 * study of Fig. 4b): many HHL instances of uneven size, each over its own
 * list of T0 values, solved in the fused eigen-frame mode and recorded once
 * as a hipGraph that is replayed.  Two launch forms (the Quantum Flow
 * Simulator section's many parallel runs): one persistent kernel that takes
 * every solve's tiles from per-XCC device work queues, with a dependency
 * counter per solve and phase; or one launch per kernel and shape class on
 * side streams.
 * --------------------------------------------------------------------- */
typedef struct {
    int n_s, n_c;          /* 1 <= n_s <= 13, 2 <= n_c <= 20, n_s + n_c + 1 <= 32 */
    const double *A;       /* host, 2^n_s x 2^n_s complex FP64 row-major, Hermitian positive definite */
    const double *b;       /* host, 2^n_s complex FP64 */
    int n_t0;              /* number of T0 values (>= 1) */
    const double *t0;      /* host, n_t0 values > 0 */
} sv_batch_instance;

typedef struct sv_batch_s *sv_batch;

/* Classical preprocessing for every instance (FP64 eigen-decomposition,
 * beta = V^H b^, the eigen-coefficients of the exact solution A^{-1} b),
 * device buffers for every (instance, T0) state, launch configurations per
 * shape class (autotuned on first use), and the captured graph.  All inputs
 * are copied; the caller's arrays may be freed on return.  hip_stream NULL:
 * the batch creates and owns a stream.  The launch form is the faster of
 * the two in graph replays (both forms captured, replayed alternately after
 * an untimed replay each, best of three rounds of two), remembered in
 * the tuning cache under key "batchform/<c64|c128>/<n_s>.<n_c>x<solves>/..."
 * (one entry per shape class, in increasing (n_s, n_c)); with autotuning
 * off (SV_AUTOTUNE=0) and no cached choice, the side streams.  The
 * environment variable SV_BATCH_QUEUE = 1 (the work queues) or 0 (the side
 * streams) overrides both.  The queue
 * kernel serves one queue per XCC with that XCC's blocks, so the producers
 * and consumers of a solve share one L2; a dependency wait is bounded (a
 * quarter second), and an expired wait or an undrained queue makes
 * sv_batch_run fail with SV_EDEVICE instead of hanging.  SV_QUEUE_LOCAL=0
 * forces a single queue for all blocks with device-scope synchronisation
 * (the fallback for an XCC layout the probe does not recognise).  In the stream form
 * the shape classes run on four side streams of default priority that the
 * batch owns, forked from and joined back into its stream (parallel branches
 * of the graph).  Either way the batch's work stays ordered on its stream.
 * Errors: SV_EINVAL, SV_EUNSUPPORTED, SV_ENOTHERMITIAN, SV_ENOTPOSDEF,
 * SV_EZERONORM, SV_ENOMEM, SV_EDEVICE. */
sv_status sv_batch_prepare(sv_batch *out, sv_dtype dt, void *hip_stream, const sv_batch_instance *inst,
                           int n_inst);

/* Run every solve of the batch (use_graph != 0: replay the graph; 0: the same
 * launches eagerly).  results (may be NULL): host, 4 doubles per solve in
 * instance-major, T0-minor order: P(a=1, clock=0), P(a=1), the norm after the
 * rotation, and the fidelity |<x_C|x_Q>| against x_C = A^{-1} b / |A^{-1} b|,
 * all accumulated in FP64.  Synchronises the batch's stream. */
sv_status sv_batch_run(sv_batch b, int use_graph, double *results);
int sv_batch_num_solves(sv_batch b);
/* The batch's launch form: 1 the work-queue kernel, 0 the side streams, -1
 * for a NULL batch.  ms_streams / ms_queue (may be NULL): the graph
 * replay times of the two forms measured at prepare (0 when not timed: pinned,
 * cached, or tuning off). */
int sv_batch_form(sv_batch b, float *ms_streams, float *ms_queue);
sv_status sv_batch_free(sv_batch b);

/* prepare + one graph replay + free */
sv_status sv_hhl_batch(sv_dtype dt, void *hip_stream, const sv_batch_instance *inst, int n_inst,
                       double *results);

/* ------------------------------------------------------------------------
 * Learned T0: a 5 -> 64 -> 64 -> 1 perceptron with exact (erf) GELU
 * activations in FP32 whose input is the spectrum features of an instance and
 * whose output predicts log(T0 lambda_max / 2 pi) (the "QPE optimizer" of the
 * main text, which estimates T0* from kappa, generalised to several cheap
 * features).  Parameter layout (SV_MLP_PARAMS floats): W1[64][5], b1[64],
 * W2[64][64], b2[64], W3[64], b3.  All pointers are device pointers;
 * calls run on hip_stream (NULL = null stream).
 * --------------------------------------------------------------------- */
#define SV_MLP_IN 5
#define SV_MLP_HIDDEN 64
#define SV_MLP_PARAMS 4609

/* y[i] = net(X[i, 0..5)) for i < B (B = 0: nothing, X and y may be NULL).
 * Errors: SV_EINVAL. */
sv_status sv_mlp_forward(const float *params, const float *X, int B, float *y, void *hip_stream);

/* Gradient of the mean squared error L = mean_i (net(X_i) - t_i)^2 with
 * respect to the parameters (grad, SV_MLP_PARAMS floats, overwritten) and L
 * itself (loss, 1 float).  Per-block partial gradients are summed in a fixed
 * order (repeatable bit for bit). */
sv_status sv_mlp_backward(const float *params, const float *X, const float *t, int B, float *grad, float *loss,
                          void *hip_stream);

/* One Adam step (step >= 1 is the 1-based step count used for bias
 * correction) on n parameters with first/second moment buffers m, v. */
sv_status sv_mlp_adam(float *params, float *m, float *v, const float *grad, int n, int step, float lr,
                      float beta1, float beta2, float eps, void *hip_stream);

/* Extreme eigenvalues of a Hermitian matrix (host, complex FP64 row-major,
 * 1 <= N <= 8192) by Lanczos iteration on the GPU: a seeded start vector
 * (xorshift64* stream, uniform entries), min(iters, N) steps with full
 * reorthogonalisation (two classical Gram-Schmidt passes per step), then
 * Sturm-sequence bisection of the Lanczos tridiagonal matrix on the host.
 * These are the cheap spectrum features of the learned T0; the paper bounds
 * the same two quantities from the trace (Wolkowicz-Styan, Sec. 3.2).
 * Runs on hip_stream (NULL = null stream) and synchronises it.  Errors:
 * SV_EINVAL, SV_ENOTHERMITIAN, SV_ENOMEM, SV_EDEVICE. */
sv_status sv_spectrum_lanczos(const double *A, int N, int iters, uint64_t seed, double *lambda_min,
                              double *lambda_max, void *hip_stream);
/* sv_spectrum_lanczos for a banded Hermitian matrix given by its 2 bw + 1
 * diagonals (host, complex FP64, band[d][r] = A[r][r + d - bw], entries
 * outside the matrix ignored; bw = 1 for the tridiagonal systems of the flow
 * problems): each Lanczos step's matrix-vector product costs O(N bw) instead
 * of O(N^2), and only the band crosses PCIe.  The same start vector, steps
 * and bisection.  Errors: SV_EINVAL (sizes, bw >= N, non-finite entries),
 * SV_ENOTHERMITIAN, SV_ENOMEM, SV_EDEVICE. */
sv_status sv_spectrum_lanczos_band(const double *band, int N, int bw, int iters, uint64_t seed, double *lambda_min,
                                   double *lambda_max, void *hip_stream);

/* Last error message of the calling thread ("" if none). */
const char *sv_last_error(void);

/* Library build string (target, compiler) for reports. */
const char *sv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SV_H */
