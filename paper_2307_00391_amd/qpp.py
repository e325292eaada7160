"""QPP: the viscous dissipation rate eps = nu <(du/dy)^2> of a channel-flow
solution, read from its amplitude encoding (main text, "Quantum
Post-processing Protocol"; appendix "Velocity gradients").

The velocity comes from the library's HHL (the U_V oracle of the main text is
QLSA-1 here), as a unit vector x plus its length |u| = |b| sqrt(p_post) / C
(C the least count).  The derivative module is the LCU circuit of
`sv_lcu_derivative` on a fresh (n_s + 2)-qubit state holding x: from select
|00>, the probability of select = 00 afterwards is

    p_D = h^2 |D x|^2,   D the zero-wall central difference,

so the grid average of the squared gradient is <(Du)^2> = |u|^2 p_D / (h^2 N)
and eps = nu |u|^2 p_D / (h^2 N).  The paper runs the derivative module and
the solver as separate circuits as well.  Its QADC-based squaring (SWAP test,
a phase estimation of a further operator, digital-to-analog conversion) is
not built: the sum of squared gradients is exactly the post-selection
probability above, which the state-vector simulation yields in FP64.

For periodic profiles the spectral derivative (`sv_spectral_derivative`)
gives <u'^2> = |u|^2 p_S Lambda_max^2 / N the same way, with p_S the
probability of the block-encoding qubit reading 1.

Everything here is marshalling around the library's kernels; the classical
and analytical references are the comparison of the main text's
dissipation-versus-Re figure.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import binding as B
from . import flow


def central_difference(N: int, h: float) -> np.ndarray:
    """(D u)_j = (u_{j+1} - u_{j-1}) / 2h with u_{-1} = u_N = 0."""
    return (np.eye(N, k=1) - np.eye(N, k=-1)) / (2.0 * h)


def dissipation_fd(u: np.ndarray, h: float, nu: float) -> float:
    """nu times the grid average of (D u)^2 (the classical post-processing
    applied to every solution in the comparison)."""
    g = central_difference(u.size, h) @ np.asarray(u, dtype=float)
    return float(nu * np.mean(g * g))


def dissipation_poiseuille_steady(Re: float, dpdx: float = -1.0) -> float:
    """Steady Poiseuille u = -(Re dpdx / 2) y (1 - y): eps = nu * int_0^1 u'^2 dy
    = Re dpdx^2 / 12 with nu = 1 / Re."""
    return Re * dpdx * dpdx / 12.0


def lcu_gradient_probability(x: np.ndarray, dtype: str = "c64", mode: int = 1) -> float:
    """p_D = probability of select = 00 after the LCU derivative of the unit
    vector x (length 2^m) on a fresh (m + 2)-qubit state."""
    x = np.asarray(x, dtype=np.complex128)
    m = x.size.bit_length() - 1
    if x.size != 1 << m:
        raise ValueError("x must have 2^m entries")
    st = B.State(m + 2, dtype)
    try:
        B.sv_init_b(st.h, x, m, 0)
        B.sv_lcu_derivative(st.h, 0, m, m, mode)
        return B.sv_norm2(st.h, 3 << m, 0)
    finally:
        st.close()


def spectral_gradient_probability(x: np.ndarray, dtype: str = "c64") -> float:
    """p_S = probability of the block-encoding qubit reading 1 after the
    spectral derivative of the unit vector x on a fresh (m + 1)-qubit state."""
    x = np.asarray(x, dtype=np.complex128)
    m = x.size.bit_length() - 1
    if x.size != 1 << m:
        raise ValueError("x must have 2^m entries")
    st = B.State(m + 1, dtype)
    try:
        B.sv_init_b(st.h, x, m, 0)
        B.sv_spectral_derivative(st.h, 0, m, m)
        return B.sv_norm2(st.h, 1 << m, 1 << m)
    finally:
        st.close()


def mean_square_gradient_spectral(x: np.ndarray, norm_u: float, dtype: str = "c64") -> float:
    """<u'^2> on the periodic grid y_j = j / N from the spectral derivative."""
    m = np.asarray(x).size.bit_length() - 1
    lmax = 2 * math.pi * ((1 << (m - 1)) - 1)
    return norm_u ** 2 * spectral_gradient_probability(x, dtype) * lmax ** 2 / (1 << m)


@dataclass
class QPPResult:
    Re: float
    eps_quantum: float          # LCU derivative of the HHL solution
    eps_classical: float        # the same post-processing on the classical solution
    eps_analytic: float         # the continuous steady value
    p_post: float               # HHL post-selection probability (last step)
    p_grad: float               # LCU select = 00 probability
    steps: int
    u_quantum: np.ndarray
    u_classical: np.ndarray


def poiseuille_dissipation(Re: float, N: int = 8, n_c: int = 8, dt: float | None = None, dtype: str = "c64",
                           mode: int = 1, tol: float = 1e-6, max_steps: int = 400) -> QPPResult:
    """Near-steady Poiseuille flow by iterative BE with one HHL solve per step
    (`flow.iterative_be`), then the QPP derivative of the last HHL output.
    dt defaults to Re / 4 (the decay time of the slowest mode is Re / pi^2);
    the march stops when a step changes u by at most tol times the steady
    centre-line velocity Re |dp/dx| / 8."""
    dt = Re / 4.0 if dt is None else dt
    ch = flow.channel("poiseuille", N=N, Re=Re, dt=dt)
    h = 1.0 / (N + 1)
    scale = max(1.0, Re * abs(ch.dpdx) / 8.0)
    run = flow.iterative_be(ch, n_c, max_steps=max_steps, tol=tol * scale, dtype=dtype, mode=mode)
    uq = run.u[-1]
    nu = 1.0 / Re
    norm_u = float(np.linalg.norm(uq))
    p_grad = lcu_gradient_probability(uq / norm_u, dtype, mode)
    eps_q = nu * norm_u ** 2 * p_grad / (h * h * N)
    steps = len(run.residual)
    uc = flow.classical_be(ch, steps)[-1]
    return QPPResult(Re, eps_q, dissipation_fd(uc, h, nu), dissipation_poiseuille_steady(Re, ch.dpdx),
                     run.p_post[-1], p_grad, steps, uq, uc)


def sweep_re(Res=(1.0, 10.0, 100.0, 1000.0), N: int = 8, n_cs=(6, 8, 10, 12), dtype: str = "c64", mode: int = 1):
    rows = []
    for n_c in n_cs:
        for Re in Res:
            r = poiseuille_dissipation(Re, N=N, n_c=n_c, dtype=dtype, mode=mode)
            rows.append({"n_c": n_c, "Re": Re, "steps": r.steps, "eps_quantum": r.eps_quantum,
                         "eps_classical": r.eps_classical, "eps_analytic": r.eps_analytic,
                         "rel_err_vs_classical": abs(r.eps_quantum - r.eps_classical) / r.eps_classical,
                         "p_post": r.p_post, "p_grad": r.p_grad})
            print(f"[qpp] n_c {n_c:2d} Re {Re:7.1f}: eps Q {r.eps_quantum:.6e} FD {r.eps_classical:.6e} "
                  f"an {r.eps_analytic:.6e} rel {rows[-1]['rel_err_vs_classical']:.2e} ({r.steps} steps)",
                  flush=True)
    return rows


def _main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="QPP dissipation of near-steady Poiseuille flow versus Re")
    ap.add_argument("--N", type=int, default=8)
    ap.add_argument("--n-c", type=int, nargs="+", default=[6, 8, 10, 12])
    ap.add_argument("--re", type=float, nargs="+", default=[1.0, 10.0, 100.0, 1000.0])
    ap.add_argument("--dtype", default="c64")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    rows = sweep_re(a.re, a.N, a.n_c, a.dtype)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    _main()
