"""Closed form of the whole HHL circuit (test helper, numpy FP64).

With A = V diag(lam) V^H, beta = V^H b/|b|, phi_j = lam_j T0 / 2 pi and
M = 2^n_c, phase estimation leaves |alpha_{y|j}|^2 = K(phi_j - y/M) (Fejer
kernel [sin(pi M d) / (M sin(pi d))]^2), the rotation multiplies the
ancilla-1 branch by 1/y (y >= 1) and the uncompute + clock = 0 projection
returns sum_y |alpha_{y|j}|^2 / y; so the post-selected vector is
proportional to V (beta * g) with g_j = sum_{y>=1} K(phi_j - y/M) / y,
and p = sum_j |beta_j g_j|^2.  Pinned against the gate-level oracle in
test_oracle_hhl.py.
"""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def fejer(delta, M):
    d = np.asarray(delta, dtype=np.float64)
    s = np.sin(np.pi * d)
    out = np.ones_like(d)
    nz = np.abs(s) > 1e-300
    out[nz] = (np.sin(np.pi * M * d[nz]) / (M * s[nz])) ** 2
    return out


def g_of_phi(phi, n_c, chunk=64, signed=False):
    """g(phi) = sum_{y=1}^{M-1} K(phi - y/M) / y, vectorised in chunks of phi.
    signed: clock values y >= M/2 invert as y - M (K has period 1 in phi)."""
    M = 1 << n_c
    y = np.arange(1, M, dtype=np.float64)
    ys = np.where(y >= M // 2, y - M, y) if signed else y
    phi = np.asarray(phi, dtype=np.float64)
    out = np.empty_like(phi)
    for a in range(0, phi.size, chunk):
        d = phi[a:a + chunk, None] - y[None, :] / M
        out[a:a + chunk] = (fejer(d, M) / ys[None, :]).sum(axis=1)
    return out


def g_h_of_phi_wide(phi, n_c, chunk=32, workers=None):
    """(g, h) per eigenphase for wide clocks (n_c up to 15 on 2^16 phases):
    g = sum_{y>=1} K(phi - y/M) / y as in g_of_phi, and
    h = sum_{y>=1} K(phi - y/M) / y^2, the ancilla-1 weight (the rotation's
    |1> amplitude is 1/y).  Written with u = M phi once: K(phi - y/M) =
    sin^2(pi r) / (M^2 sin^2(pi (u - y) / M)) with r = u - rint(u), so the
    numerator's argument reduction is exact and numerator and denominator
    come from the same rounded u (no cancellation error near the clock grid).
    Phases with u an exact integer (K = 1 at y = u, 0 elsewhere) are handled
    apart.  Numpy releases the GIL in the ufuncs: chunks run on threads."""
    M = 1 << n_c
    y = np.arange(1, M, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    u = phi * M
    r = u - np.rint(u)
    g = np.empty_like(phi)
    h = np.empty_like(phi)

    def work(a):
        uu = u[a:a + chunk, None]
        s = np.sin((uu - y[None, :]) * (math.pi / M))
        num = np.sin(math.pi * r[a:a + chunk]) ** 2 / (M * M)
        with np.errstate(divide="ignore", invalid="ignore"):   # exact-grid rows, replaced below
            w = 1.0 / (s * s)
            g[a:a + chunk] = num * (w / y[None, :]).sum(axis=1)
            h[a:a + chunk] = num * (w / (y * y)[None, :]).sum(axis=1)

    with ThreadPoolExecutor(workers or min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(work, range(0, phi.size, chunk)))
    exact = r == 0.0
    if exact.any():
        yy = np.mod(np.rint(u[exact]), M)
        g[exact] = np.where(yy >= 1, 1.0 / np.maximum(yy, 1), 0.0)
        h[exact] = np.where(yy >= 1, 1.0 / np.maximum(yy, 1) ** 2, 0.0)
    return g, h


def hhl_closed_form(A, b, n_c, T0, signed=False):
    lam, V = np.linalg.eigh(A)
    beta = V.conj().T @ (b / np.linalg.norm(b))
    g = g_of_phi(lam * T0 / (2 * math.pi), n_c, signed=signed)
    z = V @ (beta * g)
    p = float(np.sum(np.abs(beta * g) ** 2))
    return z / math.sqrt(p), p


def hhl_probabilities(A, b, n_c, T0):
    """(p_post, p_anc) of the unsigned-clock circuit: P(a = 1, clock = 0) =
    sum_j |beta_j g_j|^2 and P(a = 1) = sum_j |beta_j|^2 h_j, with g, h as in
    g_h_of_phi_wide (the ancilla-1 probability of clock value y is 1/y^2, and
    phase estimation puts K(phi_j - y/M) of eigencomponent j on y)."""
    lam, V = np.linalg.eigh(A)
    beta = V.conj().T @ (b / np.linalg.norm(b))
    g, h = g_h_of_phi_wide(lam * T0 / (2 * math.pi), n_c)
    return float(np.sum(np.abs(beta * g) ** 2)), float(np.sum(np.abs(beta) ** 2 * h))


def hhl_closed_form_kron(A_hi, A_lo, b, n_c, T0):
    """Same for A = A_hi (x) I + I (x) A_lo via the factor decompositions."""
    mu, P = np.linalg.eigh(A_hi)
    nu, Q = np.linalg.eigh(A_lo)
    Bm = (np.asarray(b, dtype=np.complex128) / np.linalg.norm(b)).reshape(len(mu), len(nu))
    beta = P.conj().T @ Bm @ Q.conj()
    lam = mu[:, None] + nu[None, :]
    g = g_of_phi((lam * T0 / (2 * math.pi)).ravel(), n_c).reshape(lam.shape)
    Z = beta * g
    p = float(np.sum(np.abs(Z) ** 2))
    X = P @ Z @ Q.T
    return X.reshape(-1) / math.sqrt(p), p


def gpe_weights(phi, n_c, cut, signed=False):
    """Gapped phase estimation: (g, h) per eigenphase, g = sum over the clock
    values with |y| >= cut of K(phi - y/M) (the flag = 1, clock = 0 amplitude
    after the uncompute: each flagged y returns to clock 0 with amplitude
    |alpha_y|^2), h the same sum over the other values (flag = 0)."""
    M = 1 << n_c
    y = np.arange(M, dtype=np.float64)
    ys = np.where(y >= M // 2, y - M, y) if signed else y
    flag = np.abs(ys) >= cut
    d = np.asarray(phi, dtype=np.float64)[:, None] - y[None, :] / M
    K = fejer(d, M)
    return (K * flag[None, :]).sum(axis=1), (K * ~flag[None, :]).sum(axis=1)


def gpe_closed_form(A, b, n_c, T0, cut, signed=False):
    """(z1, z0, p_post, p_flag): the flag = 1 and flag = 0 system vectors at
    clock 0 (unnormalised amplitudes), P(flag = 1, clock = 0) and P(flag = 1)."""
    lam, V = np.linalg.eigh(A)
    beta = V.conj().T @ (b / np.linalg.norm(b))
    g, h = gpe_weights(lam * T0 / (2 * math.pi), n_c, cut, signed)
    z1, z0 = V @ (beta * g), V @ (beta * h)
    return z1, z0, float(np.sum(np.abs(beta * g) ** 2)), float(np.sum(np.abs(beta) ** 2 * g))


def qadc_weights(u, r):
    """The QPP nonlinear transform: for each address s, the up = 1 amplitude
    with every ancilla back at 0, times sqrt(N).  Amplitude estimation of the
    SWAP test's a2 = 0 probability (1 + u_s^2) / 2 = sin^2(pi beta_s) puts
    clock value y on the phase-estimation register with probability
    K(beta_s - y/M) (the iterate's second eigenphase -beta_s gives the same
    weights at M - y, where the rotation is the same), the rotation multiplies
    the up = 1 part by f(y) = -cos(2 pi y / M), and the uncompute returns each
    y to 0 with amplitude conj(alpha_y): g_s = sum_y K(beta_s - y/M) f(y)."""
    u = np.asarray(u, dtype=np.float64)
    z = u / np.linalg.norm(u)
    M = 1 << r
    beta = np.arcsin(np.sqrt((1.0 + z * z) / 2.0)) / math.pi
    y = np.arange(M, dtype=np.float64)
    return (fejer(beta[:, None] - y[None, :] / M, M) * (-np.cos(2 * math.pi * y / M))[None, :]).sum(axis=1)
