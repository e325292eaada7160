"""Gapped phase estimation (GPE), the building block of the variable-time
solver in the Childs-Kothari-Somma construction that the paper names for
QLSA-2: per eigenvector of A, a flag that is 1 when |lambda| >= 2 eps and 0
when |lambda| <= eps, each up to an amplitude delta.

Parameter rule (signed clock of n_c qubits, T0 = pi / (2 lambda_max), so an
eigenvalue sits at the clock value y = lambda T0 2^n_c / 2 pi with
|y| <= 2^n_c / 4, far from the wrap):
    u   = eps 2^n_c / (4 lambda_max)    the clock value of |lambda| = eps;
    cut = ceil(1.5 u)                   the flag is Ry(pi) on |y| >= cut;
both sides of the gap are then at least u/2 - 1/2 clock units from the cut,
and the phase-estimation (Fejer) mass beyond a distance D on the two sides is
below 2 x 1.2 / (pi^2 (D - 1/2)) (the factor 1.2 covers the finite clock);
asking that to be <= delta^2 gives u >= 1 + 4.8 / (pi^2 delta^2), hence
n_c = ceil(log2(4 lambda_max u / eps)).
The library's `sv_gapped_pe` runs the circuit; this module only chooses the
parameters and marshals the call.
"""
from __future__ import annotations

import math

import numpy as np

from . import binding as B


def parameters(eps: float, delta: float, lam_max: float):
    """(n_c, T0, cut) for the gap (eps, 2 eps) at wrong-flag amplitude delta."""
    if not (0 < eps and 2 * eps <= lam_max and 0 < delta < 1):
        raise ValueError("need 0 < eps, 2 eps <= lam_max, 0 < delta < 1")
    u_min = 1.0 + 4.8 / (math.pi ** 2 * delta ** 2)
    n_c = max(3, math.ceil(math.log2(4.0 * lam_max * u_min / eps)))
    T0 = math.pi / (2.0 * lam_max)
    u = eps * (1 << n_c) / (4.0 * lam_max)
    cut = math.ceil(1.5 * u)
    return n_c, T0, cut


def run(A, b, eps: float, delta: float, dtype: str = "c64", mode: int = 1):
    """GPE of b over A's spectrum: returns (x_flag1, result, (n_c, T0, cut))."""
    A = np.asarray(A)
    N = A.shape[0]
    n_s = N.bit_length() - 1
    lam_max = float(np.abs(np.linalg.eigvalsh(A)).max())
    n_c, T0, cut = parameters(eps, delta, lam_max)
    st = B.State(n_s + n_c + 1, dtype)
    try:
        x, res = B.sv_gapped_pe(st.h, A, b, n_c, T0, cut, mode, 1)
    finally:
        st.close()
    return x, res, (n_c, T0, cut)
