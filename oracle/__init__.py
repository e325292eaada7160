"""FP64 CPU oracle for the HHL state-vector path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product library never imports it, and it
shares no code with it.

The numerical work lives in oracle.c (plain loops, FP64); this module only
marshals numpy arrays.  `mlp` holds the FP64 reference of the T0 predictor.
States are numpy complex128 arrays of length 2^n, qubit q = bit q of the index.
"""
import ctypes
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
