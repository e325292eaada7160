"""Host-side quality metrics and work counts (FP64).

Quality (paper, main text "Flow simulation results" and the Couette
appendix): fidelity F = |<u_Q|u_C>| of the normalised quantum and classical
solutions, the QLSA error |u_Q - u_C|, and the RMS error against an
analytic profile.

Work counts define the throughput figures: a gate acting on n qubits with c
controls performs 2^(n-c) amplitude updates; algorithmic bytes are the reads
and writes an operation must make (one read and one write per touched
amplitude).
"""
from __future__ import annotations

import numpy as np


def _unit(v):
    v = np.asarray(v, dtype=np.complex128)
    return v / np.linalg.norm(v)


def fidelity(x_q, x_c) -> float:
    return float(abs(np.vdot(_unit(x_c), _unit(x_q))))


def qlsa_error(x_q, x_c) -> float:
    """|x_Q - x_C| after aligning the global phase of x_Q to x_C."""
    q, c = _unit(x_q), _unit(x_c)
    ph = np.vdot(q, c)
    ph = ph / abs(ph) if abs(ph) > 0 else 1.0
    return float(np.linalg.norm(q * ph - c))


def rms_error(x_q, profile) -> float:
    q, c = _unit(x_q), _unit(profile)
    ph = np.vdot(q, c)
    ph = ph / abs(ph) if abs(ph) > 0 else 1.0
    return float(np.sqrt(np.mean(np.abs(q * ph - c) ** 2)))


def kron_solve(A_hi, A_lo, b):
    """Classical solution of (A_hi (x) I + I (x) A_lo) x = b through the
    factor eigen-decompositions (numpy)."""
    mu, P = np.linalg.eigh(A_hi)
    nu, Q = np.linalg.eigh(A_lo)
    B = np.asarray(b, dtype=np.complex128).reshape(len(mu), len(nu))
    Bt = P.conj().T @ B @ Q.conj()
    Xt = Bt / (mu[:, None] + nu[None, :])
    return (P @ Xt @ Q.T).reshape(-1)


def hhl_updates(n_s: int, n_c: int, mode: int) -> dict:
    """Gate-amplitude updates of one HHL solve, counted gate by gate over
    the gates the mode applies (n = n_s + n_c + 1).

    mode 0 (gate-faithful, whole state): n_c Hadamards, n_c controlled-U_k,
    inverse QFT (n_c H, n_c(n_c-1)/2 controlled phases), the 2^n_c - 1
    inversion rotations (n_c controls each), QFT, n_c controlled-U_k^H,
    n_c Hadamards.
    mode 1 (eigen-frame): the same gates before the rotation act on the
    ancilla = 0 half only (the ancilla = 1 half is zero), those after it on
    the ancilla = 1 half only (the other half is discarded by the
    post-selection); the final Hadamard layer is evaluated only for the
    clock = 0 outcome it is projected on, counted as one update per
    amplitude of the half.
    """
    n = n_s + n_c + 1
    full, half, quarter = 2.0 ** n, 2.0 ** (n - 1), 2.0 ** (n - 2)
    cps = n_c * (n_c - 1) / 2
    rot = (2.0 ** n_c - 1) * 2.0 ** (n - n_c)
    if mode == 0:
        parts = {"hadamards": 2 * n_c * full, "controlled_u": 2 * n_c * half, "qft_h": 2 * n_c * full,
                 "qft_cphase": 2 * cps * half, "rotation": rot}
    else:
        parts = {"hadamards": n_c * half + half, "controlled_u": 2 * n_c * quarter, "qft_h": 2 * n_c * half,
                 "qft_cphase": 2 * cps * quarter, "rotation": rot}
    parts["total"] = sum(parts.values())
    return parts


def probe_updates(n: int, layers: int) -> float:
    """U3 on every qubit then CNOT(q -> q+1) for q = 0..n-2, per layer."""
    return layers * (n * 2.0 ** n + (n - 1) * 2.0 ** (n - 1))
