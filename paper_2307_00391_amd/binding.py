"""Thin ctypes binding to libsv.so (declared in include/sv.h).

Functions keep the C names and only marshal arguments; every step of the
simulation runs in the library's HIP kernels.  PyTorch provides device
memory and the stream.  If libsv.so is missing the import of any entry
point raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsv.so")

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE = 0, -1, -2, -3
SV_ENOTHERMITIAN, SV_ENOTPOSDEF, SV_EZERONORM, SV_EUNSUPPORTED = -4, -5, -6, -7
SV_C64, SV_C128 = 1, 2
SV_GATE_U, SV_GATE_X, SV_GATE_SWAP = 0, 1, 2
SV_MAX_CTRLS = 8

_STATUS_NAMES = {0: "SV_OK", -1: "SV_EINVAL", -2: "SV_ENOMEM", -3: "SV_EDEVICE", -4: "SV_ENOTHERMITIAN",
                 -5: "SV_ENOTPOSDEF", -6: "SV_EZERONORM", -7: "SV_EUNSUPPORTED"}


class SvError(RuntimeError):
    def __init__(self, status, what, msg):
        super().__init__(f"{what}: {_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class sv_gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("target", ctypes.c_int), ("target2", ctypes.c_int),
                ("n_ctrls", ctypes.c_int), ("ctrls", ctypes.c_int * SV_MAX_CTRLS),
                ("ctrl_vals", ctypes.c_int * SV_MAX_CTRLS), ("u", ctypes.c_double * 8)]


class sv_hhl_params(ctypes.Structure):
    _fields_ = [("n_s", ctypes.c_int), ("n_c", ctypes.c_int), ("T0", ctypes.c_double), ("mode", ctypes.c_int),
                ("signed_clock", ctypes.c_int)]


class sv_hhl_result(ctypes.Structure):
    _fields_ = [("p_post", ctypes.c_double), ("p_anc", ctypes.c_double), ("norm_total", ctypes.c_double),
                ("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double)]


class sv_qlsa2_params(ctypes.Structure):
    _fields_ = [("n_s", ctypes.c_int), ("s", ctypes.c_int), ("B", ctypes.c_int), ("mode", ctypes.c_int)]


class sv_qlsa2_result(ctypes.Structure):
    _fields_ = [("p_post", ctypes.c_double), ("lambda_abs_max", ctypes.c_double),
                ("lambda_abs_min", ctypes.c_double), ("alpha_l1", ctypes.c_double)]


class sv_gpe_params(ctypes.Structure):
    _fields_ = [("n_s", ctypes.c_int), ("n_c", ctypes.c_int), ("T0", ctypes.c_double), ("mode", ctypes.c_int),
                ("signed_clock", ctypes.c_int), ("cut", ctypes.c_uint64)]


class sv_qlsa2f_params(ctypes.Structure):
    _fields_ = [("n_s", ctypes.c_int), ("sy", ctypes.c_int), ("sz", ctypes.c_int), ("dy", ctypes.c_double),
                ("dz", ctypes.c_double), ("mode", ctypes.c_int)]


class sv_qadc_result(ctypes.Structure):
    _fields_ = [("p_sq", ctypes.c_double), ("p_up", ctypes.c_double), ("avg", ctypes.c_double)]


class sv_batch_instance(ctypes.Structure):
    _fields_ = [("n_s", ctypes.c_int), ("n_c", ctypes.c_int), ("A", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("n_t0", ctypes.c_int), ("t0", ctypes.c_void_p)]


SV_MLP_IN, SV_MLP_HIDDEN, SV_MLP_PARAMS = 5, 64, 4609

_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_U64 = ctypes.c_uint64
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)

# name -> (argtypes, restype); optional entries are bound when the library exports them
_SIGS = {
    "sv_alloc": ([ctypes.POINTER(_P), _I, _I, _P, _P], _I),
    "sv_free": ([_P], _I),
    "sv_data": ([_P], _P),
    "sv_num_qubits": ([_P], _I),
    "sv_get_dtype": ([_P], _I),
    "sv_set_stream": ([_P, _P], _I),
    "sv_init_basis": ([_P, _U64], _I),
    "sv_init_b": ([_P, _P, _I, _I], _I),
    "sv_set_state": ([_P, _P], _I),
    "sv_get_state": ([_P, _P], _I),
    "sv_apply_gate": ([_P, _I, _P, _P, _P, _I], _I),
    "sv_apply_swap": ([_P, _I, _I, _P, _P, _I], _I),
    "sv_apply_circuit": ([_P, _P, _I, _I], _I),
    "sv_plan_passes": ([_I, _I, _P, _I, _I], _I),
    "sv_apply_ctrl_unitary": ([_P, _P, _I, _I, _I, _I, _I], _I),
    "sv_qft": ([_P, _I, _I, _I, _I, _I], _I),
    "sv_apply_uniform_ry": ([_P, _I, _I, _I, _P, _I, _I], _I),
    "sv_norm2": ([_P, _U64, _U64, _DP], _I),
    "sv_postselect": ([_P, _U64, _U64, _DP, _P, _I], _I),
    "sv_postselect_noalloc": ([_P, _U64, _U64, _P, _P], _I),
    "sv_hhl": ([_P, _P, _P, ctypes.POINTER(sv_hhl_params), ctypes.POINTER(sv_hhl_result), _P], _I),
    "sv_hhl_kron": ([_P, _P, _I, _P, _I, _P, ctypes.POINTER(sv_hhl_params), ctypes.POINTER(sv_hhl_result), _P], _I),
    "sv_hhl_prepare": ([ctypes.POINTER(_P), _P, _P, _I, _P, _I], _I),
    "sv_hhl_run": ([_P, _P, _P, ctypes.POINTER(sv_hhl_params), ctypes.POINTER(sv_hhl_result), _P], _I),
    "sv_hhl_prepare_eig": ([ctypes.POINTER(_P), _P, _P, _P, _I], _I),
    "sv_hhl_plan_spectrum": ([_P, _DP, _DP], _I),
    "sv_hhl_plan_free": ([_P], _I),
    "sv_last_eigensolver": ([], ctypes.c_char_p),
    "sv_qsp_prepare": ([_P, _P, _I, _I, _I], _I),
    "sv_lcu_derivative": ([_P, _I, _I, _I, _I], _I),
    "sv_qlsa2": ([_P, _P, _P, _P, _P, _P], _I),
    "sv_qlsa2_fourier": ([_P, _P, _P, _P, _P, _P], _I),
    "sv_hhl_run_device": ([_P, _P, _P, _P, _P, _P], _I),
    "sv_gapped_pe": ([_P, _P, _P, _P, _P, _P], _I),
    "sv_gapped_pe_run": ([_P, _P, _P, _P, _P, _P], _I),
    "sv_spectral_derivative": ([_P, _I, _I, _I, _I], _I),
    "sv_qadc_square": ([_P, _DP, _I, _I, _I, _I, _DP, ctypes.POINTER(sv_qadc_result)], _I),
    "sv_batch_prepare": ([ctypes.POINTER(_P), _I, _P, ctypes.POINTER(sv_batch_instance), _I], _I),
    "sv_batch_run": ([_P, _I, _P], _I),
    "sv_batch_num_solves": ([_P], _I),
    "sv_batch_form": ([_P, _P, _P], _I),
    "sv_batch_free": ([_P], _I),
    "sv_hhl_batch": ([_I, _P, ctypes.POINTER(sv_batch_instance), _I, _P], _I),
    "sv_mlp_forward": ([_P, _P, _I, _P, _P], _I),
    "sv_mlp_backward": ([_P, _P, _P, _I, _P, _P, _P], _I),
    "sv_mlp_adam": ([_P, _P, _P, _P, _I, _I, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P],
                    _I),
    "sv_spectrum_lanczos": ([_P, _I, _I, _U64, _DP, _DP, _P], _I),
    "sv_spectrum_lanczos_band": ([_P, _I, _I, _I, _U64, _DP, _DP, _P], _I),
    "sv_trace_enable": ([_I], _I),
    "sv_tune_report": ([ctypes.c_char_p, _I], _I),
    "sv_tune_set": ([ctypes.c_char_p, _P, _I], _I),
    "sv_trace_report": ([ctypes.c_char_p, _I], _I),
    "sv_last_error": ([], ctypes.c_char_p),
    "sv_version": ([], ctypes.c_char_p),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libsv.so; raises FileNotFoundError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} is missing: run `python -m paper_2307_00391_amd.build` "
                                "(there is no CPU fallback)")
    # torch first: the library then binds to the HIP runtime torch has loaded
    # (one runtime per process, so torch's streams and memory are the
    # library's); loaded the other way round, two runtimes would coexist
    _torch()
    L = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        fn = getattr(L, name, None)
        if fn is None:          # reported by missing_exports(); calling it raises AttributeError
            continue
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def missing_exports():
    """Entry points declared in include/sv.h that the loaded library lacks."""
    L = lib()
    return [n for n in _SIGS if getattr(L, n, None) is None]


def last_error() -> str:
    return lib().sv_last_error().decode()


def _check(st, what):
    if st != SV_OK:
        raise SvError(st, what, last_error())


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    """complex/real array -> contiguous interleaved float64 view"""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    return a, a.view(np.float64)


def _ints(xs):
    xs = [int(v) for v in (xs or [])]
    arr = (ctypes.c_int * max(1, len(xs)))(*xs)
    return arr, len(xs)


def _torch():
    import torch
    return torch


# --------------------------------------------------------------------------
# entry points (same names as the C ABI)
# --------------------------------------------------------------------------

def sv_alloc(n_qubits, dtype=SV_C64, device_buf=None, stream=None):
    h = ctypes.c_void_p()
    _check(lib().sv_alloc(ctypes.byref(h), int(n_qubits), int(dtype), device_buf, stream), "sv_alloc")
    return h


def sv_free(h):
    _check(lib().sv_free(h), "sv_free")


def sv_init_basis(h, index):
    _check(lib().sv_init_basis(h, int(index)), "sv_init_basis")


def sv_init_b(h, b, n_s, n_clock_superpose=0):
    _, bf = _f64(b)
    _check(lib().sv_init_b(h, _ptr(bf), int(n_s), int(n_clock_superpose)), "sv_init_b")


def sv_set_state(h, psi):
    _, f = _f64(psi)
    _check(lib().sv_set_state(h, _ptr(f)), "sv_set_state")


def sv_get_state(h, n):
    out = np.zeros(1 << n, dtype=np.complex128)
    _check(lib().sv_get_state(h, _ptr(out)), "sv_get_state")
    return out


def sv_apply_gate(h, target, u, ctrls=(), ctrl_vals=None):
    _, uf = _f64(np.asarray(u).reshape(2, 2))
    c, nc = _ints(ctrls)
    v, _ = _ints(ctrl_vals if ctrl_vals is not None else [1] * nc)
    _check(lib().sv_apply_gate(h, int(target), _ptr(uf), c, v, nc), "sv_apply_gate")


def sv_apply_swap(h, q1, q2, ctrls=(), ctrl_vals=None):
    c, nc = _ints(ctrls)
    v, _ = _ints(ctrl_vals if ctrl_vals is not None else [1] * nc)
    _check(lib().sv_apply_swap(h, int(q1), int(q2), c, v, nc), "sv_apply_swap")


def make_gates(gates):
    """Gate list -> ctypes array of sv_gate.  Entries:
    ("u", target, 2x2[, ctrls, cvals]) | ("x", target[, ctrls, cvals]) |
    ("cx", control, target) | ("swap", q1, q2[, ctrls, cvals])"""
    arr = (sv_gate * max(1, len(gates)))()
    for i, g in enumerate(gates):
        s = arr[i]
        kind = g[0]
        ctrls, cvals = (), None
        if kind == "u":
            s.kind, s.target = SV_GATE_U, int(g[1])
            u = np.ascontiguousarray(np.asarray(g[2], dtype=np.complex128).reshape(2, 2)).view(np.float64).ravel()
            for j in range(8):
                s.u[j] = float(u[j])
            if len(g) > 3:
                ctrls, cvals = g[3], g[4]
        elif kind == "x":
            s.kind, s.target = SV_GATE_X, int(g[1])
            if len(g) > 2:
                ctrls, cvals = g[2], g[3]
        elif kind == "cx":
            s.kind, s.target = SV_GATE_X, int(g[2])
            ctrls, cvals = (int(g[1]),), (1,)
        elif kind == "swap":
            s.kind, s.target, s.target2 = SV_GATE_SWAP, int(g[1]), int(g[2])
            if len(g) > 3:
                ctrls, cvals = g[3], g[4]
        else:
            raise ValueError(f"unknown gate kind {kind}")
        ctrls = list(ctrls or ())
        cvals = list(cvals) if cvals is not None else [1] * len(ctrls)
        if len(ctrls) > SV_MAX_CTRLS:
            raise ValueError("too many controls")
        s.n_ctrls = len(ctrls)
        for j, (cq, cv) in enumerate(zip(ctrls, cvals)):
            s.ctrls[j], s.ctrl_vals[j] = int(cq), int(cv)
    return arr


def sv_apply_circuit(h, gates, max_local=0):
    arr = gates if isinstance(gates, ctypes.Array) else make_gates(gates)
    n = len(arr) if isinstance(gates, ctypes.Array) else len(gates)
    _check(lib().sv_apply_circuit(h, arr, n, int(max_local)), "sv_apply_circuit")


def sv_plan_passes(n_qubits, dtype, gates, max_local=0):
    arr = make_gates(gates)
    return int(lib().sv_plan_passes(int(n_qubits), int(dtype), arr, len(gates), int(max_local)))


def sv_apply_ctrl_unitary(h, U_dev, sys_lo, m, ctrl=-1, ctrl_val=1, adjoint=False):
    """U_dev: device tensor (2^m x 2^m, the state's dtype, row-major)."""
    _check(lib().sv_apply_ctrl_unitary(h, _ptr(U_dev), int(sys_lo), int(m), int(ctrl), int(ctrl_val),
                                       int(bool(adjoint))), "sv_apply_ctrl_unitary")


def sv_qft(h, q_lo, m, inverse=False, swaps=True, max_local=0):
    _check(lib().sv_qft(h, int(q_lo), int(m), int(bool(inverse)), int(bool(swaps)), int(max_local)), "sv_qft")


def sv_apply_uniform_ry(h, target, reg_lo, m, cs, extra_ctrl=-1, extra_val=0):
    cs = np.ascontiguousarray(np.asarray(cs, dtype=np.float64).reshape(-1))
    if cs.size != 2 << m:
        raise ValueError("cs must hold 2^(m+1) doubles")
    _check(lib().sv_apply_uniform_ry(h, int(target), int(reg_lo), int(m), _ptr(cs), int(extra_ctrl),
                                     int(extra_val)), "sv_apply_uniform_ry")


def sv_norm2(h, mask=0, value=0):
    out = ctypes.c_double()
    _check(lib().sv_norm2(h, int(mask), int(value), ctypes.byref(out)), "sv_norm2")
    return out.value


def sv_postselect(h, n, mask, value, want_vector=True):
    p = ctypes.c_double()
    out = None
    if want_vector:
        out = np.zeros(1 << (n - bin(int(mask)).count("1")), dtype=np.complex128)
    _check(lib().sv_postselect(h, int(mask), int(value), ctypes.byref(p), _ptr(out), 0), "sv_postselect")
    return p.value, out


def sv_postselect_device(h, mask, value, out_dev=None):
    """sv_postselect with the vector left on the device (out_on_device = 1):
    out_dev is a contiguous tensor of the state's dtype, 2^(n - popcount(mask))
    entries; returns the probability."""
    p = ctypes.c_double()
    _check(lib().sv_postselect(h, int(mask), int(value), ctypes.byref(p), _ptr(out_dev), 1), "sv_postselect")
    return p.value


def sv_postselect_noalloc(h, mask, value, prob_dev, out_dev=None):
    """prob_dev: device tensor of >= 1 float64 (written asynchronously);
    out_dev: device tensor of the state's dtype or None."""
    _check(lib().sv_postselect_noalloc(h, int(mask), int(value), _ptr(prob_dev), _ptr(out_dev)),
           "sv_postselect_noalloc")


def sv_hhl(h, A, b, n_c, T0, mode=0, signed_clock=False):
    A, Af = _f64(A)
    b, bf = _f64(b)
    N = A.shape[0]
    n_s = N.bit_length() - 1
    prm = sv_hhl_params(n_s, int(n_c), float(T0), int(mode), int(bool(signed_clock)))
    res = sv_hhl_result()
    x = np.zeros(N, dtype=np.complex128)
    _check(lib().sv_hhl(h, _ptr(Af), _ptr(bf), ctypes.byref(prm), ctypes.byref(res), _ptr(x)), "sv_hhl")
    return x, res


def sv_qlsa2(h, A, b, s, B, mode=1):
    """QLSA-2 (Chebyshev LCU): returns (z, result), z the post-selected
    (select = 0, walk = 0) amplitudes, unnormalised, computational basis."""
    A, Af = _f64(A)
    b, bf = _f64(b)
    N = A.shape[0]
    n_s = N.bit_length() - 1
    prm = sv_qlsa2_params(n_s, int(s), int(B), int(mode))
    res = sv_qlsa2_result()
    z = np.zeros(N, dtype=np.complex128)
    _check(lib().sv_qlsa2(h, _ptr(Af), _ptr(bf), ctypes.byref(prm), ctypes.byref(res), _ptr(z)), "sv_qlsa2")
    return z, res


def sv_gapped_pe(h, A, b, n_c, T0, cut, mode=1, signed_clock=0):
    """Gapped phase estimation: returns (x, result), x the normalised flag = 1,
    clock = 0 system vector (result fields as sv_hhl)."""
    A, Af = _f64(A)
    b, bf = _f64(b)
    N = A.shape[0]
    n_s = N.bit_length() - 1
    prm = sv_gpe_params(n_s, int(n_c), float(T0), int(mode), int(signed_clock), int(cut))
    res = sv_hhl_result()
    x = np.zeros(N, dtype=np.complex128)
    _check(lib().sv_gapped_pe(h, _ptr(Af), _ptr(bf), ctypes.byref(prm), ctypes.byref(res), _ptr(x)),
           "sv_gapped_pe")
    return x, res


def sv_gapped_pe_run(plan, h, b, n_c, T0, cut, mode=1, signed_clock=0):
    """Gapped phase estimation on a prepared operator: returns (x, result)."""
    b, bf = _f64(b)
    n_s = b.size.bit_length() - 1
    prm = sv_gpe_params(n_s, int(n_c), float(T0), int(mode), int(signed_clock), int(cut))
    res = sv_hhl_result()
    x = np.zeros(b.size, dtype=np.complex128)
    _check(lib().sv_gapped_pe_run(plan, h, _ptr(bf), ctypes.byref(prm), ctypes.byref(res), _ptr(x)),
           "sv_gapped_pe_run")
    return x, res


def sv_qlsa2_fourier(h, A, b, sy, sz, dy, dz, mode=1):
    """QLSA-2 in Fourier form: returns (z, result), z as in sv_qlsa2."""
    A, Af = _f64(A)
    b, bf = _f64(b)
    N = A.shape[0]
    n_s = N.bit_length() - 1
    prm = sv_qlsa2f_params(n_s, int(sy), int(sz), float(dy), float(dz), int(mode))
    res = sv_qlsa2_result()
    z = np.zeros(N, dtype=np.complex128)
    _check(lib().sv_qlsa2_fourier(h, _ptr(Af), _ptr(bf), ctypes.byref(prm), ctypes.byref(res), _ptr(z)),
           "sv_qlsa2_fourier")
    return z, res


def sv_hhl_kron(h, A_hi, A_lo, b, n_c, T0, mode=1):
    A_hi, Ahf = _f64(A_hi)
    A_lo, Alf = _f64(A_lo)
    b, bf = _f64(b)
    m_hi = A_hi.shape[0].bit_length() - 1
    m_lo = A_lo.shape[0].bit_length() - 1
    prm = sv_hhl_params(m_hi + m_lo, int(n_c), float(T0), int(mode), 0)
    res = sv_hhl_result()
    x = np.zeros(b.size, dtype=np.complex128)
    _check(lib().sv_hhl_kron(h, _ptr(Ahf), m_hi, _ptr(Alf), m_lo, _ptr(bf), ctypes.byref(prm), ctypes.byref(res),
                             _ptr(x)), "sv_hhl_kron")
    return x, res


def sv_trace_enable(on=True):
    _check(lib().sv_trace_enable(int(bool(on))), "sv_trace_enable")


def sv_trace_report():
    """{kernel: {"launches", "ms", "bytes", "flops"}} for the records since sv_trace_enable(1)."""
    n = lib().sv_trace_report(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib().sv_trace_report(buf, n + 1)
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms, by, fl = line.split()
        out[name] = {"launches": int(cnt), "ms": float(ms), "bytes": float(by), "flops": float(fl)}
    return out


def sv_tune_report():
    n = lib().sv_tune_report(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib().sv_tune_report(buf, n + 1)
    return buf.value.decode()


def sv_tune_set(key, vals=()):
    """Pin (vals) or remove (empty vals) one tuning-cache entry."""
    vals = [int(v) for v in vals]
    arr = (ctypes.c_int * max(1, len(vals)))(*vals)
    _check(lib().sv_tune_set(key.encode(), ctypes.cast(arr, ctypes.c_void_p), len(vals)), "sv_tune_set")


def sv_last_eigensolver():
    return lib().sv_last_eigensolver().decode()


def sv_hhl_prepare(h, A_hi, A_lo=None):
    """Plan for A (A_lo None) or for A_hi (x) I + I (x) A_lo."""
    A_hi, Ahf = _f64(A_hi)
    m_hi = A_hi.shape[0].bit_length() - 1
    m_lo, Alf = 0, None
    if A_lo is not None:
        A_lo, Alf = _f64(A_lo)
        m_lo = A_lo.shape[0].bit_length() - 1
    p = ctypes.c_void_p()
    _check(lib().sv_hhl_prepare(ctypes.byref(p), h, _ptr(Ahf), m_hi, _ptr(Alf), m_lo), "sv_hhl_prepare")
    return p


def sv_hhl_prepare_eig(h, V_dev, lam):
    """V_dev: contiguous float64 device tensor (N x N, column j = eigenvector of
    lam[j]), kept alive by the caller for the plan's lifetime; lam: N floats."""
    lam = np.ascontiguousarray(np.asarray(lam, dtype=np.float64))
    n_s = lam.size.bit_length() - 1
    torch = _torch()
    if not (isinstance(V_dev, torch.Tensor) and V_dev.is_cuda and V_dev.dtype == torch.float64
            and V_dev.is_contiguous() and V_dev.numel() == lam.size * lam.size):
        raise ValueError("V_dev must be a contiguous float64 CUDA tensor of N x N entries")
    p = ctypes.c_void_p()
    _check(lib().sv_hhl_prepare_eig(ctypes.byref(p), h, ctypes.c_void_p(V_dev.data_ptr()),
                                    lam.ctypes.data_as(ctypes.c_void_p), n_s), "sv_hhl_prepare_eig")
    return p


def sv_hhl_run(plan, h, b, n_c, T0, mode=1, signed_clock=False):
    b, bf = _f64(b)
    n_s = b.size.bit_length() - 1
    prm = sv_hhl_params(n_s, int(n_c), float(T0), int(mode), int(bool(signed_clock)))
    res = sv_hhl_result()
    x = np.zeros(b.size, dtype=np.complex128)
    _check(lib().sv_hhl_run(plan, h, _ptr(bf), ctypes.byref(prm), ctypes.byref(res), _ptr(x)), "sv_hhl_run")
    return x, res


def sv_hhl_run_device(plan, h, b_dev, n_c, T0, mode=1, signed_clock=False, x_dev=None):
    """sv_hhl_run with b and x as device tensors (complex128, 2^n_s entries, on
    the state's device); returns the result (x lands in x_dev when given)."""
    n = int(b_dev.numel())
    n_s = n.bit_length() - 1
    prm = sv_hhl_params(n_s, int(n_c), float(T0), int(mode), int(bool(signed_clock)))
    res = sv_hhl_result()
    xp = ctypes.c_void_p(x_dev.data_ptr()) if x_dev is not None else None
    _check(lib().sv_hhl_run_device(plan, h, ctypes.c_void_p(b_dev.data_ptr()), ctypes.byref(prm), ctypes.byref(res),
                                   xp), "sv_hhl_run_device")
    return res


def sv_hhl_plan_spectrum(plan):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(lib().sv_hhl_plan_spectrum(plan, ctypes.byref(lo), ctypes.byref(hi)), "sv_hhl_plan_spectrum")
    return lo.value, hi.value


def sv_hhl_plan_free(plan):
    _check(lib().sv_hhl_plan_free(plan), "sv_hhl_plan_free")


def sv_version():
    return lib().sv_version().decode()


def sv_qsp_prepare(h, b, q_lo=0, mode=1):
    """QSP-1 binary-tree preparation of b / |b| on the register [q_lo, q_lo + m)."""
    b, bf = _f64(b)
    m = b.size.bit_length() - 1
    if b.size != 1 << m:
        raise ValueError("b must have 2^m entries")
    _check(lib().sv_qsp_prepare(h, _ptr(bf), int(q_lo), m, int(mode)), "sv_qsp_prepare")


def sv_lcu_derivative(h, q_lo, m, sel_lo, mode=1):
    """QPP LCU central-difference gradient on [q_lo, q_lo + m) with select
    qubits [sel_lo, sel_lo + 2); mode 0 gate by gate, 1 one fused pass."""
    _check(lib().sv_lcu_derivative(h, int(q_lo), int(m), int(sel_lo), int(mode)), "sv_lcu_derivative")


def sv_spectral_derivative(h, q_lo, m, anc, max_local=0):
    """QPP spectral gradient on [q_lo, q_lo + m), Lambda block-encoded on `anc`."""
    _check(lib().sv_spectral_derivative(h, int(q_lo), int(m), int(anc), int(max_local)),
           "sv_spectral_derivative")


def sv_qadc_square(h, u, r, mode=1, avg=True):
    """QPP nonlinear transform of the real 2^n-point u on a (3n + r + 2)-qubit
    state.  Returns (g, result): g[s] ~ (u_s / |u|)^2."""
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).ravel())
    n = u.size.bit_length() - 1
    if u.size != 1 << n:
        raise ValueError("u must have 2^n entries")
    g = np.zeros(u.size)
    res = sv_qadc_result()
    _check(lib().sv_qadc_square(h, u.ctypes.data_as(_DP), n, int(r), int(mode), int(bool(avg)),
                                g.ctypes.data_as(_DP), ctypes.byref(res)), "sv_qadc_square")
    return g, res


# --------------------------------------------------------------------------
# batched T0 sweeps
# --------------------------------------------------------------------------

def _dtype_code(dtype):
    return SV_C64 if dtype in ("c64", SV_C64) else SV_C128


def _batch_instances(instances):
    """instances: iterable of (A, b, n_c, t0_list).  Returns the ctypes array
    and the host arrays it points into (kept alive by the caller)."""
    keep, arr = [], (sv_batch_instance * max(1, len(instances)))()
    for i, (A, b, n_c, t0) in enumerate(instances):
        A, Af = _f64(A)
        b, bf = _f64(b)
        t0 = np.ascontiguousarray(np.atleast_1d(np.asarray(t0, dtype=np.float64)))
        keep += [A, Af, b, bf, t0]
        n_s = b.size.bit_length() - 1
        arr[i] = sv_batch_instance(n_s, int(n_c), Af.ctypes.data, bf.ctypes.data, t0.size, t0.ctypes.data)
    return arr, keep


def sv_batch_prepare(instances, dtype="c64", stream=None):
    arr, keep = _batch_instances(instances)
    h = ctypes.c_void_p()
    _check(lib().sv_batch_prepare(ctypes.byref(h), _dtype_code(dtype), stream, arr, len(instances)),
           "sv_batch_prepare")
    del keep
    return h


def sv_batch_num_solves(b):
    return int(lib().sv_batch_num_solves(b))


def sv_batch_form(b):
    """(form, ms_streams, ms_queue): 1 = the work-queue kernel, 0 = side
    streams; the graph replay times measured at prepare (0 when not timed)."""
    ms = (ctypes.c_float * 2)()
    a = ctypes.addressof(ms)
    f = int(lib().sv_batch_form(b, a, a + ctypes.sizeof(ctypes.c_float)))
    return f, float(ms[0]), float(ms[1])


def sv_batch_run(b, use_graph=True, want_results=True):
    """-> (n_solves, 4) array of [p_post, p_anc, norm_total, fidelity] or None"""
    out = np.zeros((sv_batch_num_solves(b), 4)) if want_results else None
    _check(lib().sv_batch_run(b, int(bool(use_graph)), _ptr(out)), "sv_batch_run")
    return out


def sv_batch_free(b):
    _check(lib().sv_batch_free(b), "sv_batch_free")


def sv_hhl_batch(instances, dtype="c64", stream=None):
    arr, keep = _batch_instances(instances)
    out = np.zeros((sum(np.atleast_1d(t).size for *_, t in instances), 4))
    _check(lib().sv_hhl_batch(_dtype_code(dtype), stream, arr, len(instances), _ptr(out)), "sv_hhl_batch")
    del keep
    return out


# --------------------------------------------------------------------------
# learned-T0 perceptron (device tensors, float32)
# --------------------------------------------------------------------------

def _stream_ptr(stream):
    if stream is None:
        return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f32(t, n=None):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def sv_mlp_forward(params, X, y=None, stream=None):
    torch = _torch()
    B = X.shape[0]
    if X.shape[1:] != (SV_MLP_IN,):
        raise ValueError("X must be (B, 5)")
    if y is None:
        y = torch.empty(B, dtype=torch.float32, device=X.device)
    _check(lib().sv_mlp_forward(_dev_f32(params, SV_MLP_PARAMS), _dev_f32(X), B, _dev_f32(y, B),
                                _stream_ptr(stream)), "sv_mlp_forward")
    return y


def sv_mlp_backward(params, X, t, grad=None, loss=None, stream=None):
    torch = _torch()
    B = X.shape[0]
    if X.shape[1:] != (SV_MLP_IN,):
        raise ValueError("X must be (B, 5)")
    if grad is None:
        grad = torch.empty(SV_MLP_PARAMS, dtype=torch.float32, device=X.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib().sv_mlp_backward(_dev_f32(params, SV_MLP_PARAMS), _dev_f32(X), _dev_f32(t, B), B,
                                 _dev_f32(grad, SV_MLP_PARAMS), _dev_f32(loss, 1), _stream_ptr(stream)),
           "sv_mlp_backward")
    return grad, loss


def sv_mlp_adam(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    n = params.numel()
    _check(lib().sv_mlp_adam(_dev_f32(params), _dev_f32(m, n), _dev_f32(v, n), _dev_f32(grad, n), n, int(step),
                             lr, beta1, beta2, eps, _stream_ptr(stream)), "sv_mlp_adam")


def sv_spectrum_lanczos(A, iters=96, seed=0, stream=None):
    A, Af = _f64(A)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(lib().sv_spectrum_lanczos(_ptr(Af), A.shape[0], int(iters), int(seed), ctypes.byref(lo),
                                     ctypes.byref(hi), _stream_ptr(stream)), "sv_spectrum_lanczos")
    return lo.value, hi.value


def band_of(A, bw):
    """The 2 bw + 1 diagonals of A as the band layout of sv_spectrum_lanczos_band:
    band[d][r] = A[r][r + d - bw] (zero outside the matrix)."""
    A = np.asarray(A)
    N = A.shape[0]
    band = np.zeros((2 * bw + 1, N), dtype=np.complex128)
    for d in range(2 * bw + 1):
        off = d - bw
        diag = np.diagonal(A, off)
        if off >= 0:
            band[d, :N - off] = diag
        else:
            band[d, -off:] = diag
    return band


def sv_spectrum_lanczos_band(band, iters=96, seed=0, stream=None):
    band, bf = _f64(band)
    nd, N = band.shape
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(lib().sv_spectrum_lanczos_band(_ptr(bf), int(N), int((nd - 1) // 2), int(iters), int(seed),
                                          ctypes.byref(lo), ctypes.byref(hi), _stream_ptr(stream)),
           "sv_spectrum_lanczos_band")
    return lo.value, hi.value


# --------------------------------------------------------------------------
# convenience: a state whose memory is a torch tensor on the current device
# --------------------------------------------------------------------------

class State:
    def __init__(self, n, dtype="c64", device=None, stream=None):
        torch = _torch()
        self.n = int(n)
        self.dt = SV_C64 if dtype in ("c64", SV_C64, torch.complex64) else SV_C128
        tdt = torch.complex64 if self.dt == SV_C64 else torch.complex128
        self.tensor = torch.empty(1 << self.n, dtype=tdt, device=device or "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.tensor.device)
        self.h = sv_alloc(self.n, self.dt, ctypes.c_void_p(self.tensor.data_ptr()),
                          ctypes.c_void_p(self.stream.cuda_stream))

    def close(self):
        if self.h is not None:
            sv_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self):
        return sv_get_state(self.h, self.n)

    def set(self, psi):
        sv_set_state(self.h, psi)
