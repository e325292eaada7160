"""Seeded synthetic inputs for the HHL state-vector path.

This module only *generates inputs*: the linear systems (A, b), the T0
choices and grids, and random circuits.  It contains none of the simulator's
arithmetic (no gate application, phase estimation or inversion), so both the
GPU library's tests and the FP64 oracle can draw from it.

Workloads (all synthetic; the paper publishes no dataset):
  * Poiseuille / Couette steady systems: second-order central difference
    Laplacian (paper, appendix "Finite difference", eq. CDS) on N interior
    points, h = 1/(N+1), Dirichlet walls folded into b.  The steady limits of
    the flow equation (main text eq. 3) are the parabola y(1-y) (Poiseuille,
    constant pressure gradient) and the line y (Couette, moving top wall).
  * random SPD tridiagonal matrices with a prescribed condition number
    (the T0 / kappa sweep family of the "QPE optimizer" study, Fig. 4b).
  * a 2-D separable Laplacian (paper: "d-dimensional" Laplace/Poisson) plus
    a random symmetric perturbation, as a Kronecker sum, kappa = 1000.
  * random U3 + CNOT-ladder layers (pure gate-throughput probe).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.linalg import eigvalsh_tridiagonal
from scipy.optimize import brentq

SEED_BASE = 230700391


def seed_for(config: int, instance: int = 0) -> int:
    return SEED_BASE + 1000 * int(config) + int(instance)


def rng_for(config: int, instance: int = 0) -> np.random.Generator:
    return np.random.default_rng(seed_for(config, instance))


# --------------------------------------------------------------------------
# finite-difference flow systems
# --------------------------------------------------------------------------

def laplacian_1d(N: int, h: float | None = None) -> np.ndarray:
    """tridiag(-1, 2, -1) / h^2: the SPD form of minus the central-difference
    second derivative on N interior points (h = 1/(N+1) by default)."""
    if h is None:
        h = 1.0 / (N + 1)
    A = np.zeros((N, N))
    idx = np.arange(N)
    A[idx, idx] = 2.0
    A[idx[:-1], idx[:-1] + 1] = -1.0
    A[idx[1:], idx[1:] - 1] = -1.0
    return A / (h * h)


def laplacian_1d_lambda_max(N: int) -> float:
    """Largest eigenvalue of tridiag(-1,2,-1)/h^2 (closed form)."""
    h = 1.0 / (N + 1)
    return 4.0 * math.sin(N * math.pi / (2 * (N + 1))) ** 2 / (h * h)


def laplacian_1d_lambda_min(N: int) -> float:
    h = 1.0 / (N + 1)
    return 4.0 * math.sin(math.pi / (2 * (N + 1))) ** 2 / (h * h)


def grid_points(N: int) -> np.ndarray:
    return np.arange(1, N + 1) / (N + 1)


@dataclass
class LinearSystem:
    name: str
    A: np.ndarray            # Hermitian, FP64
    b: np.ndarray            # FP64 (complex allowed), not normalised
    lambda_max: float
    lambda_min: float
    profile: np.ndarray | None = None   # analytic steady profile at the grid points


def poiseuille(N: int = 16) -> LinearSystem:
    """Steady Poiseuille flow: -u'' = const with u(0)=u(1)=0; b uniform.
    Normalised, the pressure-gradient sign and Re drop out."""
    A = laplacian_1d(N)
    b = np.ones(N)
    y = grid_points(N)
    return LinearSystem("poiseuille", A, b, laplacian_1d_lambda_max(N),
                        laplacian_1d_lambda_min(N), y * (1.0 - y))


def couette(N: int = 256, u_wall: float = 1.0) -> LinearSystem:
    """Steady Couette flow: -u'' = 0, u(0)=0, u(1)=u_wall; the wall value
    enters b at the last interior point as u_wall / h^2."""
    h = 1.0 / (N + 1)
    A = laplacian_1d(N)
    b = np.zeros(N)
    b[-1] = u_wall / (h * h)
    y = grid_points(N)
    return LinearSystem("couette", A, b, laplacian_1d_lambda_max(N),
                        laplacian_1d_lambda_min(N), u_wall * y)


def t0_top_of_clock(lambda_max: float, n_c: int) -> float:
    """T0 = 2 pi (1 - 2^-n_c) / lambda_max: puts lambda_max on the largest
    clock value y = 2^n_c - 1 when clock bit k applies exp(i A T0 2^k)."""
    return 2.0 * math.pi * (1.0 - 2.0 ** (-n_c)) / lambda_max


def t0_grid(lambda_max: float, count: int = 16) -> np.ndarray:
    """Log grid around 2 pi / lambda_max: factors 2^(-1 + 3 m / 15), m = 0..15
    (0.5x .. 4x)."""
    m = np.arange(count)
    return (2.0 * math.pi / lambda_max) * 2.0 ** (-1.0 + 3.0 * m / (count - 1))


# --------------------------------------------------------------------------
# random SPD tridiagonal family (T0 / kappa sweep)
# --------------------------------------------------------------------------

def _tridiag(d: np.ndarray, e: np.ndarray) -> np.ndarray:
    A = np.diag(d)
    A += np.diag(e, 1) + np.diag(e, -1)
    return A


def random_spd_tridiag(rng: np.random.Generator, N: int, kappa: float):
    """Diagonal d_j ~ U[2,4], weights w_j ~ U[0.5,1], off-diagonals
    -s w_j sqrt(d_j d_{j+1}); s is bisected so that cond(A) = kappa
    (cond grows monotonically with s from cond(diag(d)) <= 2)."""
    d = rng.uniform(2.0, 4.0, N)
    w = rng.uniform(0.5, 1.0, N - 1)
    base = -w * np.sqrt(d[:-1] * d[1:])

    def extremes(s):
        off = s * base
        lo_ = eigvalsh_tridiagonal(d, off, select="i", select_range=(0, 0))[0]
        hi_ = eigvalsh_tridiagonal(d, off, select="i", select_range=(N - 1, N - 1))[0]
        return lo_, hi_

    def cond(s):
        lo_, hi_ = extremes(s)
        if lo_ <= 0:
            return math.inf
        return hi_ / lo_

    lo, hi = 0.0, 1.0
    while cond(hi) < kappa:        # widen if needed (rare)
        hi *= 2.0
        if hi > 64:
            break
    if cond(lo) >= kappa:
        s = 0.0
    elif cond(hi) <= kappa:
        s = hi
    else:
        # log cond(s) - log kappa changes sign on [lo, hi]; cond is infinite
        # past the loss of definiteness, which brentq only sees as "large"
        def f(s_):
            c = cond(s_)
            return (math.log(c) if math.isfinite(c) else 800.0) - math.log(kappa)
        s = brentq(f, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=200)
    A = _tridiag(d, s * base)
    lmin, lmax = extremes(s)
    return A, float(lmin), float(lmax)


@dataclass
class SweepInstance:
    index: int
    n_s: int
    n_c: int
    kappa_target: float
    A: np.ndarray
    b: np.ndarray
    lambda_min: float
    lambda_max: float
    t0: np.ndarray          # the T0 grid for this instance


def sweep_instances(count: int = 64, config: int = 2, n_s_range=(4, 10), n_c_range=(8, 12),
                    kappa_log10=(1.0, 4.0), t0_count: int = 16, first: int = 0):
    """Instances of the batched T0 sweep: n_s ~ U{n_s_range}, n_c ~ U{n_c_range},
    kappa log-uniform, b ~ N(0, I); one seed per instance."""
    out = []
    for i in range(first, first + count):
        rng = rng_for(config, i)
        n_s = int(rng.integers(n_s_range[0], n_s_range[1] + 1))
        n_c = int(rng.integers(n_c_range[0], n_c_range[1] + 1))
        kappa = float(10.0 ** rng.uniform(*kappa_log10))
        A, lmin, lmax = random_spd_tridiag(rng, 1 << n_s, kappa)
        b = rng.standard_normal(1 << n_s)
        out.append(SweepInstance(i, n_s, n_c, kappa, A, b, lmin, lmax, t0_grid(lmax, t0_count)))
    return out


# --------------------------------------------------------------------------
# 2-D separable system (Kronecker sum), kappa = 1000
# --------------------------------------------------------------------------

@dataclass
class KronSystem:
    A_hi: np.ndarray     # acts on the high half of the system index
    A_lo: np.ndarray     # acts on the low half
    b: np.ndarray
    lambda_min: float
    lambda_max: float

    def dense(self) -> np.ndarray:
        """A = A_hi (x) I + I (x) A_lo (only for small sizes)."""
        n_hi, n_lo = self.A_hi.shape[0], self.A_lo.shape[0]
        return np.kron(self.A_hi, np.eye(n_lo)) + np.kron(np.eye(n_hi), self.A_lo)


def kron_laplacian_system(rng: np.random.Generator, m_hi: int, m_lo: int, kappa: float = 1000.0,
                          pert_norm: float = 0.1, band: int = 2) -> KronSystem:
    """2-D five-point Laplacian on a 2^m_hi x 2^m_lo grid, written as
    L_hi (x) I + I (x) L_lo and scaled so lambda_max = 1, plus a random real
    symmetric banded perturbation E_hi (x) I + I (x) E_lo with spectral norm
    `pert_norm`, plus a shift sigma I fixing cond(A) = kappa exactly."""
    n_hi, n_lo = 1 << m_hi, 1 << m_lo
    L_hi, L_lo = laplacian_1d(n_hi, 1.0), laplacian_1d(n_lo, 1.0)
    scale = 1.0 / (np.linalg.eigvalsh(L_hi)[-1] + np.linalg.eigvalsh(L_lo)[-1])
    L_hi, L_lo = L_hi * scale, L_lo * scale

    def band_sym(n):
        E = np.zeros((n, n))
        for k in range(band + 1):
            v = rng.standard_normal(n - k)
            E += np.diag(v, k) + (np.diag(v, -k) if k else 0)
        return E

    E_hi, E_lo = band_sym(n_hi), band_sym(n_lo)
    e_hi, e_lo = np.linalg.eigvalsh(E_hi), np.linalg.eigvalsh(E_lo)
    enorm = max(abs(e_hi[-1] + e_lo[-1]), abs(e_hi[0] + e_lo[0]))
    E_hi, E_lo = E_hi * (pert_norm / enorm), E_lo * (pert_norm / enorm)
    B_hi, B_lo = L_hi + E_hi, L_lo + E_lo
    m_hi_ev, m_lo_ev = np.linalg.eigvalsh(B_hi), np.linalg.eigvalsh(B_lo)
    lmin, lmax = m_hi_ev[0] + m_lo_ev[0], m_hi_ev[-1] + m_lo_ev[-1]
    sigma = (lmax - kappa * lmin) / (kappa - 1.0)
    B_hi = B_hi + 0.5 * sigma * np.eye(n_hi)
    B_lo = B_lo + 0.5 * sigma * np.eye(n_lo)
    b = rng.standard_normal(n_hi * n_lo)
    return KronSystem(B_hi, B_lo, b, float(lmin + sigma), float(lmax + sigma))


# --------------------------------------------------------------------------
# random circuits
# --------------------------------------------------------------------------

def u3(theta: float, phi: float, lam: float) -> np.ndarray:
    """U3 in the OpenQASM convention (the paper does not define U3)."""
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -np.exp(1j * lam) * s],
                     [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]], dtype=np.complex128)


def random_unitary(rng: np.random.Generator, dim: int) -> np.ndarray:
    """Haar-like random unitary from the QR of a complex Gaussian matrix."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def random_state(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def probe_layers(rng: np.random.Generator, n: int, layers: int):
    """Gate list of the bandwidth probe: per layer, U3 with angles ~ U[0, 2 pi)
    on every qubit, then CNOT(q -> q+1) for q = 0..n-2.
    Entries: ("u", target, 2x2) or ("cx", control, target)."""
    gates = []
    for _ in range(layers):
        for q in range(n):
            th, ph, la = rng.uniform(0.0, 2.0 * math.pi, 3)
            gates.append(("u", q, u3(th, ph, la)))
        for q in range(n - 1):
            gates.append(("cx", q, q + 1))
    return gates


def random_circuit(rng: np.random.Generator, n: int, count: int, max_ctrls: int = 2):
    """Random mix of controlled one-qubit gates, CNOT/Toffoli and SWAPs."""
    gates = []
    for _ in range(count):
        kind = rng.integers(0, 4)
        qs = rng.permutation(n)
        nc = int(rng.integers(0, min(max_ctrls, n - 2) + 1))
        if kind <= 1:
            ctrls = [int(q) for q in qs[1:1 + nc]]
            cvals = [int(v) for v in rng.integers(0, 2, nc)]
            gates.append(("u", int(qs[0]), random_unitary(rng, 2), ctrls, cvals))
        elif kind == 2:
            ctrls = [int(q) for q in qs[1:1 + nc]]
            cvals = [int(v) for v in rng.integers(0, 2, nc)]
            gates.append(("x", int(qs[0]), ctrls, cvals))
        else:
            nc2 = min(nc, n - 2)
            ctrls = [int(q) for q in qs[2:2 + nc2]]
            cvals = [int(v) for v in rng.integers(0, 2, nc2)]
            gates.append(("swap", int(qs[0]), int(qs[1]), ctrls, cvals))
    return gates
