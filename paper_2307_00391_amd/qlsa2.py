"""QLSA-2 (Chebyshev, and Fourier form, linear combinations of unitaries) next
to QLSA-1 (HHL) on the paper's steady channel-flow systems.

Parameters of the Chebyshev solver from the condition number and a target
error (after the cited Childs-Kothari-Somma analysis):
    B  = ceil(kappa^2 ln(kappa / eps))   makes (1 - (1 - x^2)^B)/x eps-close
                                          to 1/x on 1/kappa <= |x| <= 1;
    j0 = ceil(sqrt(B ln(4 B / eps)))     Chebyshev terms kept (J = 2^s > j0).
The library's `sv_qlsa2` runs the circuit; this module only chooses the
parameters, marshals the inputs and compares the outputs with A^-1 b.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import binding as B
from . import inputs


def parameters(kappa: float, eps: float):
    """(B, s): the polynomial degree parameter and the select-register width."""
    Bdeg = max(1, math.ceil(kappa * kappa * math.log(kappa / eps)))
    j0 = math.ceil(math.sqrt(Bdeg * math.log(4 * Bdeg / eps)))
    s = max(1, math.ceil(math.log2(j0 + 1)))
    return Bdeg, s


def fourier_parameters(kappa: float, eps: float):
    """(sy, sz, dy, dz) of the Fourier form, each of three error terms below eps / 3:
    y-cut Y = kappa sqrt(2 ln(3 kappa / eps)) (the tail (1/x) e^{-x^2 Y^2 / 2});
    dy = 2 sqrt(eps) (the left sum of x y e^{-x^2 y^2 / 2} from y = 0 is off by dy^2 x / 12);
    2^sy >= Y / dy, so the sum runs to Y' = 2^sy dy >= Y;
    z-cut Z = sqrt(2 ln(6 Y' / (sqrt(2 pi) eps))) (the Gaussian tail over y <= Y');
    dz = 2 pi / (Y' + 2 Z) (the first alias of the z-sum lies 2 pi / dz - x y >= 2 Z away);
    2^(sz - 1) >= Z / dz."""
    Y = kappa * math.sqrt(2.0 * math.log(3.0 * kappa / eps))
    dy = 2.0 * math.sqrt(eps)
    sy = max(1, math.ceil(math.log2(Y / dy)))
    Yr = (1 << sy) * dy
    Z = math.sqrt(2.0 * math.log(6.0 * Yr / (math.sqrt(2.0 * math.pi) * eps)))
    dz = 2.0 * math.pi / (Yr + 2.0 * Z)
    sz = max(1, math.ceil(math.log2(Z / dz))) + 1
    return sy, sz, dy, dz


def fourier_terms(sy: int, sz: int, dy: float, dz: float):
    """(w, t, sign): weights, times y_j z_k and the sign of z_k of every select value r = j + 2^sy m."""
    J, K = 1 << sy, 1 << (sz - 1)
    r = np.arange(J * 2 * K)
    j, m = r & (J - 1), r >> sy
    k = np.where(m < K, m + 1, m - 2 * K)
    z = k * dz
    w = dy * dz * np.abs(z) * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)
    return w, j * dy * z, np.sign(k)


def solve(A, b, eps: float, dtype: str = "c64", mode: int = 1, kappa: float | None = None):
    """Run QLSA-2 for A x = b at target error eps; returns (x_unit, result, s, B, seconds)."""
    A = np.asarray(A)
    N = A.shape[0]
    n_s = N.bit_length() - 1
    if kappa is None:
        lam = np.abs(np.linalg.eigvalsh(A))
        kappa = lam.max() / lam.min()
    Bdeg, s = parameters(kappa, eps)
    st = B.State(n_s + 1 + s, dtype)
    try:
        t = time.perf_counter()
        z, res = B.sv_qlsa2(st.h, A, b, s, Bdeg, mode)
        el = time.perf_counter() - t
    finally:
        st.close()
    return z / np.linalg.norm(z), res, s, Bdeg, el


def solve_fourier(A, b, eps: float, dtype: str = "c64", kappa: float | None = None):
    """QLSA-2 in Fourier form at target error eps; returns (x_unit, result, (sy, sz, dy, dz), seconds)."""
    A = np.asarray(A)
    N = A.shape[0]
    n_s = N.bit_length() - 1
    if kappa is None:
        lam = np.abs(np.linalg.eigvalsh(A))
        kappa = lam.max() / lam.min()
    sy, sz, dy, dz = fourier_parameters(kappa, eps)
    st = B.State(n_s + sy + sz, dtype)
    try:
        t = time.perf_counter()
        z, res = B.sv_qlsa2_fourier(st.h, A, b, sy, sz, dy, dz)
        el = time.perf_counter() - t
    finally:
        st.close()
    return z / np.linalg.norm(z), res, (sy, sz, dy, dz), el


def A_kappa(A):
    lam = np.abs(np.linalg.eigvalsh(np.asarray(A)))
    return float(lam.max() / lam.min())


def fidelity(x, ref):
    return float(abs(np.vdot(x / np.linalg.norm(x), ref / np.linalg.norm(ref))))


def compare(N: int = 16, eps_list=(1e-1, 1e-2, 1e-3, 1e-4), n_cs=(6, 8, 10, 12), dtype: str = "c64"):
    """Poiseuille (N interior points): QLSA-1 at textbook T0 for several clock
    sizes, QLSA-2 (both modes) for several target errors."""
    sysm = inputs.poiseuille(N)
    A, b = sysm.A, sysm.b
    n_s = N.bit_length() - 1
    x = np.linalg.solve(A, b)
    rows = []
    for n_c in n_cs:
        st = B.State(n_s + n_c + 1, dtype)
        T0 = inputs.t0_top_of_clock(sysm.lambda_max, n_c)
        B.sv_hhl(st.h, A, b, n_c, T0, 1)                    # first use: tuning
        t = time.perf_counter()
        xq, res = B.sv_hhl(st.h, A, b, n_c, T0, 1)
        el = time.perf_counter() - t
        st.close()
        rows.append({"solver": "QLSA-1", "n_c": n_c, "qubits": n_s + n_c + 1, "p_post": res.p_post,
                     "one_minus_F": 1 - fidelity(xq, x), "seconds": el})
        print(f"[qlsa] QLSA-1 n_c {n_c:2d}: {n_s + n_c + 1} qubits, 1-F {rows[-1]['one_minus_F']:.2e}, "
              f"p {res.p_post:.2e}, {el * 1e3:.2f} ms", flush=True)
    for eps in eps_list:
        for mode in (1, 0):
            solve(A, b, eps, dtype, mode)                     # first use
            xq, res, s, Bdeg, el = solve(A, b, eps, dtype, mode)
            rows.append({"solver": "QLSA-2", "mode": mode, "eps": eps, "B": Bdeg, "s": s,
                         "qubits": n_s + 1 + s, "p_post": res.p_post, "one_minus_F": 1 - fidelity(xq, x),
                         "seconds": el})
            print(f"[qlsa] QLSA-2 mode {mode} eps {eps:.0e}: B {Bdeg}, s {s}, {n_s + 1 + s} qubits, "
                  f"1-F {rows[-1]['one_minus_F']:.2e}, p {res.p_post:.2e}, {el * 1e3:.2f} ms", flush=True)
        if N.bit_length() - 1 + sum(fourier_parameters(A_kappa(A), eps)[:2]) <= 30:
            solve_fourier(A, b, eps, dtype)                          # first use
            xq, res, (sy, sz, dy, dz), el = solve_fourier(A, b, eps, dtype)
            rows.append({"solver": "QLSA-2 Fourier", "eps": eps, "sy": sy, "sz": sz, "qubits": n_s + sy + sz,
                         "p_post": res.p_post, "one_minus_F": 1 - fidelity(xq, x), "seconds": el})
            print(f"[qlsa] QLSA-2 Fourier eps {eps:.0e}: sy {sy}, sz {sz}, {n_s + sy + sz} qubits, "
                  f"1-F {rows[-1]['one_minus_F']:.2e}, p {res.p_post:.2e}, {el * 1e3:.2f} ms", flush=True)
    return rows


def _main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="QLSA-1 and QLSA-2 on the Poiseuille system")
    ap.add_argument("--N", type=int, default=16)
    ap.add_argument("--dtype", default="c64")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    rows = compare(a.N, dtype=a.dtype)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    _main()
