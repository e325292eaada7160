"""FP64 CPU oracle for the HHL state-vector path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product library never imports it, and it
shares no code with it.

The numerical work lives in oracle.c (plain loops, FP64); this module only
marshals numpy arrays.  `mlp` holds the FP64 reference of the T0 predictor.
States are numpy complex128 arrays of length 2^n, qubit q = bit q of the index.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_c128p = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_apply_gate.argtypes = [_c128p, ctypes.c_int, ctypes.c_int, _f64p, ip, ip, ctypes.c_int]
    lib.orc_apply_swap.argtypes = [_c128p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip, ctypes.c_int]
    lib.orc_qft.argtypes = [_c128p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.orc_apply_ctrl_unitary.argtypes = [_c128p, ctypes.c_int, _c128p, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.orc_qsp.argtypes = [_c128p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c128p, ctypes.c_int]
    lib.orc_lcu_derivative.argtypes = [_c128p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.orc_spectral_derivative.argtypes = [_c128p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.orc_qsp_apply.argtypes = [_c128p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c128p, ctypes.c_int]
    lib.orc_cks_coeffs.argtypes = [ctypes.c_int, ctypes.c_int, _f64p]
    lib.orc_qlsa2.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _c128p, _c128p, _c128p, _c128p,
                              ctypes.POINTER(ctypes.c_double)]
    lib.orc_qlsa2_fourier.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      _c128p, _c128p, _c128p, _c128p, ctypes.POINTER(ctypes.c_double)]
    lib.orc_norm2.argtypes = [_c128p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    lib.orc_norm2.restype = ctypes.c_double
    lib.orc_postselect.argtypes = [_c128p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    lib.orc_eigh.argtypes = [ctypes.c_int, _c128p, _f64p, _c128p]
    lib.orc_hhl.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _c128p, _c128p, _c128p, _c128p,
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    lib.orc_gapped_pe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _c128p, _c128p, _c128p, _c128p,
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                  ctypes.c_uint64]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def _ints(xs):
    xs = list(xs or [])
    arr = (ctypes.c_int * max(1, len(xs)))(*xs)
    return arr, len(xs)


def _nqubits(psi):
    n = int(psi.size).bit_length() - 1
    if psi.size != 1 << n:
        raise ValueError("state length must be a power of two")
    return n


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls (results do not depend on it)."""
    _load().orc_set_num_threads(int(n))


def apply_gate(psi, target, u, ctrls=(), cvals=None):
    """psi <- (controlled) one-qubit gate u (2x2 complex) on `target`, in place."""
    lib = _load()
    u8 = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(2, 2)).view(np.float64).ravel()
    c, nc = _ints(ctrls)
    v, _ = _ints(cvals if cvals is not None else [1] * len(list(ctrls)))
    _check(lib.orc_apply_gate(psi, _nqubits(psi), int(target), np.ascontiguousarray(u8), c, v, nc), "apply_gate")
    return psi


def apply_swap(psi, q1, q2, ctrls=(), cvals=None):
    lib = _load()
    c, nc = _ints(ctrls)
    v, _ = _ints(cvals if cvals is not None else [1] * len(list(ctrls)))
    _check(lib.orc_apply_swap(psi, _nqubits(psi), int(q1), int(q2), c, v, nc), "apply_swap")
    return psi


def qft(psi, lo, m, inverse=False):
    _check(_load().orc_qft(psi, _nqubits(psi), int(lo), int(m), int(bool(inverse))), "qft")
    return psi


def apply_ctrl_unitary(psi, U, lo, m, ctrl=-1, cval=1, adjoint=False):
    U = np.ascontiguousarray(U, dtype=np.complex128)
    _check(_load().orc_apply_ctrl_unitary(psi, _nqubits(psi), U, int(lo), int(m), int(ctrl), int(cval),
                                          int(bool(adjoint))), "apply_ctrl_unitary")
    return psi


def norm2(psi, mask=0, value=0):
    return float(_load().orc_norm2(psi, _nqubits(psi), int(mask), int(value)))


def postselect(psi, mask, value, want_vector=True):
    n = _nqubits(psi)
    p = ctypes.c_double(0.0)
    out = None
    ptr = None
    if want_vector:
        out = np.zeros(1 << (n - bin(int(mask)).count("1")), dtype=np.complex128)
        ptr = out.ctypes.data_as(ctypes.c_void_p)
    rc = _load().orc_postselect(psi, n, int(mask), int(value), ctypes.byref(p), ptr)
    if rc != 0 and p.value != 0.0:
        _check(rc, "postselect")
    return p.value, out


def eigh(A):
    A = np.ascontiguousarray(A, dtype=np.complex128)
    N = A.shape[0]
    lam = np.zeros(N, dtype=np.float64)
    V = np.zeros((N, N), dtype=np.complex128)
    _check(_load().orc_eigh(N, A, lam, V), "eigh")
    return lam, V


def qsp(n, q_lo, b, levels=-1):
    """QSP-1 binary-tree preparation of b on the register [q_lo, q_lo + m)
    of an n-qubit state from |0...0> (see oracle.c); returns the state."""
    b = np.ascontiguousarray(np.asarray(b, dtype=np.complex128))
    m = b.size.bit_length() - 1
    if b.size != 1 << m:
        raise ValueError("b must have 2^m entries")
    psi = np.zeros(1 << n, dtype=np.complex128)
    _check(_load().orc_qsp(psi, int(n), int(q_lo), int(m), b, int(levels)), "qsp")
    return psi


def hhl(A, b, n_c, T0, signed_clock=False):
    """Gate-level HHL (see oracle.c): returns (psi, x, p_post, p_anc).
    signed_clock reads the clock as a two's-complement value (indefinite A)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    N = A.shape[0]
    n_s = N.bit_length() - 1
    if N != 1 << n_s or b.shape != (N,):
        raise ValueError("A must be 2^n_s square and b of length 2^n_s")
    psi = np.zeros(1 << (n_s + n_c + 1), dtype=np.complex128)
    x = np.zeros(N, dtype=np.complex128)
    pp, pa = ctypes.c_double(0), ctypes.c_double(0)
    _check(_load().orc_hhl(n_s, int(n_c), float(T0), A, b, psi, x, ctypes.byref(pp), ctypes.byref(pa),
                           int(bool(signed_clock))), "hhl")
    return psi, x, pp.value, pa.value


def gapped_pe(A, b, n_c, T0, cut, signed_clock=False):
    """Gapped phase estimation (see oracle.c): the HHL circuit with the flag
    Ry(pi) on clock values |y| >= cut in place of the inversion rotation.
    Returns (psi, x, p_post, p_anc): x the normalised flag = 1, clock = 0
    system vector, p_post = P(flag = 1, clock = 0), p_anc = P(flag = 1)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    N = A.shape[0]
    n_s = N.bit_length() - 1
    if N != 1 << n_s or b.shape != (N,):
        raise ValueError("A must be 2^n_s square and b of length 2^n_s")
    psi = np.zeros(1 << (n_s + n_c + 1), dtype=np.complex128)
    x = np.zeros(N, dtype=np.complex128)
    pp, pa = ctypes.c_double(0), ctypes.c_double(0)
    _check(_load().orc_gapped_pe(n_s, int(n_c), float(T0), A, b, psi, x, ctypes.byref(pp), ctypes.byref(pa),
                                 int(bool(signed_clock)), ctypes.c_uint64(int(cut))), "gapped_pe")
    return psi, x, pp.value, pa.value


def lcu_derivative(psi, q_lo, m, sel_lo):
    """QPP finite-difference gradient by LCU on the register [q_lo, q_lo + m)
    with the two select qubits [sel_lo, sel_lo + 2) (see oracle.c), in place.
    From select |00>, the select-|00> block ends as (S - S^T) phi / 2 = h D phi."""
    _check(_load().orc_lcu_derivative(psi, _nqubits(psi), int(q_lo), int(m), int(sel_lo)), "lcu_derivative")
    return psi


def spectral_derivative(psi, q_lo, m, anc):
    """QPP spectral gradient on the register [q_lo, q_lo + m) with the
    block-encoding qubit `anc` (see oracle.c), in place.  From anc = |0>,
    the anc = 1 block ends as dphi/dy / (2 pi (2^(m-1) - 1)), y_j = j / 2^m."""
    _check(_load().orc_spectral_derivative(psi, _nqubits(psi), int(q_lo), int(m), int(anc)),
           "spectral_derivative")
    return psi


def qsp_apply(psi, q_lo, b, inverse=False):
    """The QSP-1 tree circuit for b on the register [q_lo, q_lo + m) of an
    arbitrary state (or its adjoint), in place."""
    b = np.ascontiguousarray(np.asarray(b, dtype=np.complex128))
    m = b.size.bit_length() - 1
    if b.size != 1 << m:
        raise ValueError("b must have 2^m entries")
    _check(_load().orc_qsp_apply(psi, _nqubits(psi), int(q_lo), int(m), b, int(bool(inverse))), "qsp_apply")
    return psi


def cks_coeffs(B, J):
    """alpha_j (j < J) of g(x) = (1 - (1 - x^2)^B) / x = sum_j alpha_j T_{2j+1}(x)."""
    out = np.zeros(int(J), dtype=np.float64)
    _check(_load().orc_cks_coeffs(int(B), int(J), out), "cks_coeffs")
    return out


def qlsa2(A, b, s, B):
    """QLSA-2 by Chebyshev LCU (see oracle.c): returns (psi, z, p_post) with
    z the post-selected (select = 0, walk = 0) amplitudes, unnormalised."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    N = A.shape[0]
    n_s = N.bit_length() - 1
    if N != 1 << n_s or b.shape != (N,):
        raise ValueError("A must be 2^n_s square and b of length 2^n_s")
    psi = np.zeros(1 << (n_s + 1 + int(s)), dtype=np.complex128)
    z = np.zeros(N, dtype=np.complex128)
    p = ctypes.c_double(0.0)
    _check(_load().orc_qlsa2(n_s, int(s), int(B), A, b, psi, z, ctypes.byref(p)), "qlsa2")
    return psi, z, p.value


def qlsa2_fourier(A, b, sy, sz, dy, dz):
    """QLSA-2 in Fourier form (see oracle.c): returns (psi, z, p_post), z the
    post-selected (select = 0) amplitudes, unnormalised."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    N = A.shape[0]
    n_s = N.bit_length() - 1
    if N != 1 << n_s or b.shape != (N,):
        raise ValueError("A must be 2^n_s square and b of length 2^n_s")
    psi = np.zeros(1 << (n_s + int(sy) + int(sz)), dtype=np.complex128)
    z = np.zeros(N, dtype=np.complex128)
    p = ctypes.c_double(0.0)
    _check(_load().orc_qlsa2_fourier(n_s, int(sy), int(sz), float(dy), float(dz), A, b, psi, z, ctypes.byref(p)),
           "qlsa2_fourier")
    return psi, z, p.value


def qadc_loader(zeta):
    """U_V of the nonlinear transform (appendix "Nonlinear transform", step 2):
    any unitary that loads the amplitudes from |0> will do; this one is the
    real Householder reflection I - 2 v v^T / (v^T v), v = e_0 + sigma zeta,
    sigma = +1 if zeta_0 >= 0 else -1, so U_V|0> = -sigma zeta.  It is
    symmetric and its own inverse."""
    zeta = np.asarray(zeta, dtype=np.float64)
    sigma = 1.0 if zeta[0] >= 0.0 else -1.0
    v = sigma * zeta
    v[0] += 1.0
    return np.eye(zeta.size) - 2.0 * np.outer(v, v) / np.dot(v, v)


def qadc_square(u, r, avg=True):
    """The QPP nonlinear transform sum_k u'_k |k> -> sum_k (u'_k)^2 |k>
    (appendix "Nonlinear transform", steps 1-5), gate by gate.  u: 2^n real
    values (normalised here); r: qubits of the phase-estimation register.
    Qubits: ua [0, n), a1 [n, 2n), add [2n, 3n), a2 = 3n, ub [3n+1, 3n+1+r),
    up = 3n+1+r.  Returns the final state (after U_avg = H on add if `avg`).

    Step 1: H on add, then CNOT add_j -> a1_j copies the address.
    Steps 2-3, W: U_V on ua, then the SWAP test of ua and a1 on a2 (H,
    controlled swaps, H); the a2 = 0 part of W|0, s, 0> has probability
    (1 + u_s^2) / 2 = sin^2(pi beta_s).
    Step 4: phase estimation of the amplitude-estimation iterate
    Q = -W S_0 W^dagger S_chi on ub (H, controlled Q^(2^k), inverse QFT).
    S_chi flips the sign of a2 = 0; S_0 flips the sign of ua = 0, a1 = s,
    a2 = 0 (the conditional phase shift of the appendix), written as CNOTs
    add -> a1 around a phase on ua = a1 = a2 = 0.  Q's eigenphases are
    +-beta_s, so ub holds beta_s or 1 - beta_s.
    Step 5: Ry on up with sine -cos(2 pi y / 2^r) = 2 sin^2(pi y/2^r) - 1
    for ub = y (u_s^2 at the exact phase), then phase estimation, W and the
    address copy undone, so the up = 1, ancillas = 0 block holds the squares."""
    u = np.asarray(u, dtype=np.float64)
    N = u.size
    n = N.bit_length() - 1
    if N != 1 << n or n < 1 or r < 1:
        raise ValueError("u must have 2^n >= 2 entries and r >= 1")
    UV = qadc_loader(u / np.linalg.norm(u)).astype(np.complex128)
    ua, a1, add = list(range(n)), list(range(n, 2 * n)), list(range(2 * n, 3 * n))
    a2, ub0, up = 3 * n, 3 * n + 1, 3 * n + 1 + r
    ub = list(range(ub0, ub0 + r))
    psi = np.zeros(1 << (up + 1), dtype=np.complex128)
    psi[0] = 1.0
    H = np.array([[1, 1], [1, -1]]) / math.sqrt(2.0)
    X = np.array([[0, 1], [1, 0]])
    Z = np.diag([1.0, -1.0])
    FLIP0 = np.diag([-1.0, 1.0])

    def copy_address():
        for j in range(n):
            apply_gate(psi, a1[j], X, [add[j]])

    def swap_test():
        apply_gate(psi, a2, H)
        for j in range(n):
            apply_swap(psi, ua[j], a1[j], [a2])
        apply_gate(psi, a2, H)

    def W():
        apply_ctrl_unitary(psi, UV, 0, n)
        swap_test()

    def W_dagger():
        swap_test()
        apply_ctrl_unitary(psi, UV, 0, n, adjoint=True)

    def S_chi(c):
        apply_gate(psi, a2, FLIP0, [c])

    def S_0(c):
        copy_address()
        apply_gate(psi, a2, FLIP0, ua + a1 + [c], [0] * (2 * n) + [1])
        copy_address()

    def controlled_Q(c, inverse):
        if not inverse:          # Q = -W S_0 W^dagger S_chi
            S_chi(c)
            W_dagger()
            S_0(c)
            W()
        else:                    # Q^dagger = -S_chi W S_0 W^dagger
            W_dagger()
            S_0(c)
            W()
            S_chi(c)
        apply_gate(psi, c, Z)    # the minus sign, on the control

    for q in add:                                   # step 1
        apply_gate(psi, q, H)
    copy_address()
    W()                                             # steps 2-3
    for q in ub:                                    # step 4
        apply_gate(psi, q, H)
    for k in range(r):
        for _ in range(1 << k):
            controlled_Q(ub[k], False)
    qft(psi, ub0, r, inverse=True)
    M = 1 << r
    for y in range(M):                              # step 5
        f = -math.cos(2.0 * math.pi * y / M)
        c = abs(math.sin(2.0 * math.pi * y / M))
        apply_gate(psi, up, np.array([[c, -f], [f, c]]), ub, [(y >> b) & 1 for b in range(r)])
    qft(psi, ub0, r, inverse=False)                 # undo phase estimation
    for k in reversed(range(r)):
        for _ in range(1 << k):
            controlled_Q(ub[k], True)
    for q in ub:
        apply_gate(psi, q, H)
    W_dagger()
    copy_address()
    if avg:
        for q in add:
            apply_gate(psi, q, H)
    return psi
