"""Pins of the oracle's signed clock (two's-complement eigenvalue inversion,
for indefinite Hermitian A such as the Hermitian dilation of a non-symmetric
system): exact inversion when every eigenphase lies on the clock grid
(positive and negative), the closed form for generic spectra, and the
dilation [[0, A], [A^T, 0]] returning [0; A^-1 b]."""
import math

import numpy as np
import pytest

import oracle
from tests.closed_form import hhl_closed_form


def _on_grid(rng, N, n_c, T0, ks):
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    lam = np.asarray(ks, dtype=float) * 2 * math.pi / (T0 * 2 ** n_c)
    return (Q * lam) @ Q.T, lam


@pytest.mark.parametrize("N,n_c", [(4, 4), (8, 5)])
def test_exact_inversion_with_negative_eigenvalues(N, n_c):
    rng = np.random.default_rng(N)
    T0 = 0.7
    M = 2 ** n_c
    ks = np.concatenate([rng.choice(np.arange(-M // 2 + 1, 0), size=N // 2, replace=False),
                         rng.choice(np.arange(1, M // 2), size=N // 2, replace=False)])
    A, lam = _on_grid(rng, N, n_c, T0, ks)
    b = rng.standard_normal(N)
    _, x, p, _ = oracle.hhl(A, b, n_c, T0, signed_clock=True)
    xc = np.linalg.solve(A, b)
    xc /= np.linalg.norm(xc)
    assert np.abs(x - xc).max() <= 1e-12
    # p = |C A^-1 b^|^2 with C the least count
    C = 2 * math.pi / (M * T0)
    assert abs(p - C * C * np.linalg.norm(np.linalg.solve(A, b / np.linalg.norm(b))) ** 2) <= 1e-12
    # the unsigned clock inverts the negative ones as M + k: not A^-1 b
    _, xu, _, _ = oracle.hhl(A, b, n_c, T0, signed_clock=False)
    assert np.abs(xu - xc).max() > 1e-3


def test_signed_closed_form_generic_spectrum():
    rng = np.random.default_rng(5)
    N, n_c = 8, 6
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    lam = np.concatenate([rng.uniform(-3, -0.5, 4), rng.uniform(0.5, 3, 4)])
    A = (Q * lam) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    T0 = 2 * math.pi * 0.45 / 3.0
    _, x, p, _ = oracle.hhl(A, b, n_c, T0, signed_clock=True)
    xr, pr = hhl_closed_form(A, b, n_c, T0, signed=True)
    assert np.abs(x - xr).max() <= 1e-12 and abs(p - pr) <= 1e-12


def test_dilation_solves_the_nonsymmetric_system():
    rng = np.random.default_rng(9)
    N, n_c, T0 = 4, 5, 0.9
    M = 2 ** n_c
    # A = U diag(s) W^T with singular values on the clock grid: the dilation's
    # eigenvalues are +-s, all on the grid
    U, _ = np.linalg.qr(rng.standard_normal((N, N)))
    W, _ = np.linalg.qr(rng.standard_normal((N, N)))
    s = np.array([3, 5, 7, 11]) * 2 * math.pi / (T0 * M)
    A = (U * s) @ W.T
    H = np.block([[np.zeros((N, N)), A], [A.T, np.zeros((N, N))]])
    b = rng.standard_normal(N)
    _, x, _, _ = oracle.hhl(H, np.concatenate([b, np.zeros(N)]), n_c, T0, signed_clock=True)
    xc = np.linalg.solve(A, b)
    xc /= np.linalg.norm(xc)
    assert np.abs(x[:N]).max() <= 1e-12
    assert np.abs(x[N:] - xc).max() <= 1e-12
