"""Unsteady channel flow by iterative backward Euler, one HHL solve per step.

The main text's iterative BE scheme (QLSA-1 on the A_be1 system; the
temporal discretisation of the appendix on finite differences):

    (u^{j+1} - u^j) / dt = A u^{j+1} + f,   A = (1/Re) d^2/dy^2 (central differences)
    A_be1 u^{j+1} = b_be1,   A_be1 = I - A dt,   b_be1 = u^j + f dt (+ wall terms)

solved at every step by the library's HHL (the circuit on the GPU), until the
change between steps falls below a tolerance (the paper uses 1e-6).  HHL
returns a unit vector; the length of the solution comes from the
post-selection probability: the post-selected vector is C A_be1^{-1} b^ with
C the least count 2 pi / (2^n_c T0), so |A_be1^{-1} b| = |b| sqrt(p_post) / C
(exact for exact phase estimation, otherwise the HHL estimate itself).

Flows (walls at y = 0 and y = 1, N interior points, h = 1 / (N + 1)):
  Poiseuille start-up: u(y, 0) = 1, u(0) = u(1) = 0, f = -dp/dx; the
    analytical solution is the series of the main text's QSP section.
  Couette start-up: u(y, 0) = 0, u(0) = 0, u(1) = 1, f = 0;
    u = y + sum_k 2 (-1)^k / (k pi) sin(k pi y) exp(-(k pi)^2 t / Re).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import binding as B


@dataclass
class Channel:
    kind: str
    N: int
    Re: float
    dt: float
    dpdx: float
    y: np.ndarray
    A_be1: np.ndarray       # I - A dt
    src: np.ndarray         # f dt + wall terms, added to u^j every step
    u0: np.ndarray


def channel(kind: str = "poiseuille", N: int = 16, Re: float = 10.0, dt: float = 0.1, dpdx: float = -1.0) -> Channel:
    if N < 2 or N & (N - 1):
        raise ValueError("N must be a power of two >= 2")
    h = 1.0 / (N + 1)
    y = h * np.arange(1, N + 1)
    L = (np.diag(np.full(N, -2.0)) + np.diag(np.ones(N - 1), 1) + np.diag(np.ones(N - 1), -1)) / (h * h)
    A = L / Re
    A_be1 = np.eye(N) - dt * A
    src = np.zeros(N)
    if kind == "poiseuille":
        src += -dpdx * dt
        u0 = np.ones(N)
    elif kind == "couette":
        src[-1] += dt / (Re * h * h)          # moving wall u(1) = 1 folded into the last equation
        u0 = np.zeros(N)
    else:
        raise ValueError(kind)
    return Channel(kind, N, Re, dt, dpdx, y, A_be1, src, u0)


def analytic(ch: Channel, t: float, kmax: int = 4001) -> np.ndarray:
    """The series solutions (main text, QSP section, for Poiseuille; the
    classical start-up series for Couette)."""
    y, Re = ch.y, ch.Re
    k = np.arange(1, kmax + 1)[:, None]
    decay = np.exp(-t / Re * (k * math.pi) ** 2)
    if ch.kind == "poiseuille":
        coef = 2 * (1 - (-1.0) ** k) / (k * math.pi) * (1 + ch.dpdx * Re / (k * math.pi) ** 2)
        return (coef * np.sin(k * math.pi * y) * decay).sum(0) - 0.5 * Re * ch.dpdx * y * (1 - y)
    return y + (2 * (-1.0) ** k / (k * math.pi) * np.sin(k * math.pi * y) * decay).sum(0)


def classical_be(ch: Channel, steps: int) -> np.ndarray:
    """The same scheme with a direct solve per step (the classical CFD reference)."""
    u = ch.u0.copy()
    out = [u]
    for _ in range(steps):
        u = np.linalg.solve(ch.A_be1, u + ch.src)
        out.append(u)
    return np.array(out)


@dataclass
class BERun:
    u: np.ndarray                     # (steps + 1, N)
    residual: list = field(default_factory=list)
    p_post: list = field(default_factory=list)
    converged_at: int = -1


def iterative_be(ch: Channel, n_c: int, max_steps: int = 400, tol: float = 1e-6, dtype: str = "c64", mode: int = 1,
                 T0: float | None = None) -> BERun:
    """March with one HHL solve per step until |u^{j+1} - u^j|_inf <= tol."""
    n_s = ch.N.bit_length() - 1
    st = B.State(n_s + n_c + 1, dtype)
    plan = B.sv_hhl_prepare(st.h, ch.A_be1)
    try:
        lmin, lmax = B.sv_hhl_plan_spectrum(plan)
        if T0 is None:
            T0 = 2 * math.pi * (1 - 2.0 ** -n_c) / lmax
        C = 2 * math.pi / (2 ** n_c * T0)
        u = ch.u0.copy()
        hist = [u]
        run = BERun(u=None)
        for j in range(max_steps):
            b = u + ch.src
            x, res = B.sv_hhl_run(plan, st.h, b, n_c, T0, mode)
            un = np.linalg.norm(b) * math.sqrt(res.p_post) / C * x.real
            run.p_post.append(res.p_post)
            r = float(np.abs(un - u).max())
            run.residual.append(r)
            u = un
            hist.append(u)
            if r <= tol:
                run.converged_at = j + 1
                break
        run.u = np.array(hist)
        return run
    finally:
        B.sv_hhl_plan_free(plan)
        st.close()


def rms(a, b):
    return float(np.sqrt(np.mean((np.asarray(a) - np.asarray(b)) ** 2)))


def one_shot_system(ch: Channel, scheme: str, m: int, p: int):
    """The unrolled systems of the appendix on finite differences: blocks
    u^0 .. u^{m+p} of the field, row 0 u^0 = u_in, rows 1..m one time step,
    rows m+1..m+p the copies u^i - u^{i-1} = 0 that lift the post-selection
    probability.  FE: u^i - (I + A dt) u^{i-1} = f dt; BE: (I - A dt) u^i -
    u^{i-1} = f dt (A_be1 = I - A dt).  Returns (A_os, b_os)."""
    N = ch.N
    K = m + p + 1
    I = np.eye(N)
    Adt = I - ch.A_be1                    # A dt
    A_os = np.zeros((K * N, K * N))
    b_os = np.zeros(K * N)
    A_os[:N, :N] = I
    b_os[:N] = ch.u0
    for i in range(1, K):
        r = slice(i * N, (i + 1) * N)
        prev = slice((i - 1) * N, i * N)
        if i <= m:
            if scheme == "fe":
                A_os[r, r] = I
                A_os[r, prev] = -(I + Adt)
            elif scheme == "be":
                A_os[r, r] = ch.A_be1
                A_os[r, prev] = -I
            else:
                raise ValueError(scheme)
            b_os[r] = ch.src
        else:
            A_os[r, r] = I
            A_os[r, prev] = -I
    return A_os, b_os


@dataclass
class OneShot:
    u: np.ndarray          # (m + p + 1, N) from the HHL solution
    u_classical: np.ndarray
    p_post: float
    fidelity: float


def one_shot(ch: Channel, scheme: str, m: int, p: int, n_c: int, dtype: str = "c64", mode: int = 1) -> OneShot:
    """Solve the unrolled system in one HHL run: the system is not Hermitian,
    so its Hermitian dilation H = [[0, A], [A^T, 0]] with right-hand side
    [b; 0] is solved with a signed clock (H has eigenvalues +-sigma, the
    singular values of A), and the lower half of the solution is A^-1 b.
    The length again comes from p_post."""
    A_os, b_os = one_shot_system(ch, scheme, m, p)
    n = A_os.shape[0]
    if n & (n - 1):
        raise ValueError("(m + p + 1) N must be a power of two")
    H = np.block([[np.zeros((n, n)), A_os], [A_os.T, np.zeros((n, n))]])
    bb = np.concatenate([b_os, np.zeros(n)])
    n_s = (2 * n).bit_length() - 1
    smax = np.linalg.norm(A_os, 2)
    T0 = 2 * math.pi * 0.45 / smax
    st = B.State(n_s + n_c + 1, dtype)
    try:
        x, res = B.sv_hhl(st.h, H, bb, n_c, T0, mode, signed_clock=True)
    finally:
        st.close()
    C = 2 * math.pi / (2 ** n_c * T0)
    full = np.linalg.norm(bb) * math.sqrt(res.p_post) / C * x.real
    u = full[n:].reshape(m + p + 1, ch.N)
    uc = np.linalg.solve(A_os, b_os).reshape(m + p + 1, ch.N)
    xc = uc.ravel() / np.linalg.norm(uc)
    F = abs(np.vdot(xc, x[n:])) / np.linalg.norm(x[n:])
    return OneShot(u, uc, res.p_post, float(F))


def sweep_clock_qubits(kind="poiseuille", N=16, Re=10.0, dt=0.5, n_cs=range(4, 17), dtype="c64", tol=1e-6,
                       max_steps=600, log=print):
    """Converged iterative-BE profiles for several clock sizes (the main
    text's Q_PE study): rms and centre-line errors against the exact steady
    profile, steps to convergence, wall time per step."""
    import time
    ch = channel(kind, N, Re, dt)
    steady = -0.5 * Re * ch.dpdx * ch.y * (1 - ch.y) if kind == "poiseuille" else ch.y
    mid = N // 2
    rows = []
    for n_c in n_cs:
        t = time.perf_counter()
        run = iterative_be(ch, n_c, max_steps=max_steps, tol=tol, dtype=dtype)
        el = time.perf_counter() - t
        steps = len(run.residual)
        rows.append({"n_c": int(n_c), "qubits": int(N.bit_length() - 1 + n_c + 1), "steps": steps,
                     "converged": run.converged_at > 0, "eps_rms": rms(run.u[-1], steady),
                     "centre_err": float(run.u[-1][mid] - steady[mid]),
                     "ms_per_step": 1e3 * el / max(steps, 1), "p_post_last": run.p_post[-1]})
        log(f"[flow] n_c {n_c:2d}: {steps} steps, eps_rms {rows[-1]['eps_rms']:.3e}, "
            f"centre {rows[-1]['centre_err']:+.3e}, {rows[-1]['ms_per_step']:.2f} ms/step")
    return {"kind": kind, "N": N, "Re": Re, "dt": dt, "dtype": dtype, "tol": tol, "rows": rows}


def sweep_one_shot(kind="poiseuille", N=4, Re=10.0, dt=0.18, m=27, p=4, n_cs=range(6, 15), dtype="c64",
                   log=print):
    """One-shot FE and BE (dilated, signed clock) for several clock sizes:
    the final block against the classical solution of the same system and
    against the analytical series, and the fidelity of the whole solution."""
    import time
    ch = channel(kind, N, Re, dt)
    ua = analytic(ch, m * dt)
    rows = []
    for scheme in ("fe", "be"):
        for n_c in n_cs:
            t = time.perf_counter()
            r = one_shot(ch, scheme, m, p, n_c, dtype)
            el = time.perf_counter() - t
            rows.append({"scheme": scheme, "n_c": int(n_c), "eps_rms_vs_classical": rms(r.u[-1], r.u_classical[-1]),
                         "eps_rms_vs_analytic": rms(r.u[-1], ua),
                         "classical_vs_analytic": rms(r.u_classical[-1], ua), "fidelity": r.fidelity,
                         "p_post": r.p_post, "seconds": el})
            log(f"[one-shot] {scheme} n_c {n_c:2d}: rms vs classical {rows[-1]['eps_rms_vs_classical']:.3e}, "
                f"vs analytic {rows[-1]['eps_rms_vs_analytic']:.3e}, F {r.fidelity:.5f}, p {r.p_post:.2e}")
    return {"kind": kind, "N": N, "Re": Re, "dt": dt, "m": m, "p": p, "dtype": dtype, "rows": rows}


if __name__ == "__main__":
    import argparse
    import json
    import os
    ap = argparse.ArgumentParser(description="iterative backward Euler with one HHL solve per step")
    ap.add_argument("--kind", default="poiseuille")
    ap.add_argument("--N", type=int, default=16)
    ap.add_argument("--Re", type=float, default=10.0)
    ap.add_argument("--dt", type=float, default=0.5)
    ap.add_argument("--nc-min", type=int, default=4)
    ap.add_argument("--nc-max", type=int, default=16)
    ap.add_argument("--dtype", default="c64")
    ap.add_argument("--out", default="flow_sweep.json")
    ap.add_argument("--one-shot", action="store_true", help="the unrolled FE/BE systems (N=4, m=27, p=4)")
    a = ap.parse_args()
    if a.one_shot:
        res = sweep_one_shot(a.kind, n_cs=range(a.nc_min, a.nc_max + 1), dtype=a.dtype,
                             log=lambda s: print(s, flush=True))
    else:
        res = sweep_clock_qubits(a.kind, a.N, a.Re, a.dt, range(a.nc_min, a.nc_max + 1), a.dtype,
                                 log=lambda s: print(s, flush=True))
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
