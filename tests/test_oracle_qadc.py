"""Pins of the QPP nonlinear-transform oracle (appendix "Nonlinear
transform": address register, SWAP test, amplitude estimation by phase
estimation, a rotation from the estimated phase, the uncompute).

Pinned against the mathematics, not against the oracle's own steps:
- the up = 1, ancillas = 0 amplitude of address s is g_s / sqrt(N), with g_s
  the Fejer-weighted mean of f(y) = -cos(2 pi y / M) around the eigenphase
  beta_s of the amplitude-estimation iterate, sin^2(pi beta_s) = (1 + u_s^2)/2
  (written out in tests/closed_form.py), and also its Fourier-series
  closed form -((M - 1) cos 2 pi beta + cos 2 pi (M - 1) beta) / M;
- at an exact phase (u_s = 0: beta = 1/4; u_s = +-1: beta = 1/2) the
  transform is exact, so a basis-vector input gives a fully known final
  state;
- |g_s - u_s^2| <= 2 / M, g depends on u_s^2 only, the state stays
  normalised, and U_avg puts (1/N) sum_s g_s on address 0.
Planted mistakes (S_chi on a2 = 1, the iterate's minus sign dropped, S_0
without the address copy, the rotation's sine of the wrong sign) each fail
the closed-form pin."""
import math

import numpy as np
import pytest

import oracle
from tests.closed_form import qadc_weights


def _layout(n, r):
    return 3 * n + 1 + r          # the up qubit; add = [2n, 3n)


def _amps(psi, n, r):
    up = _layout(n, r)
    N = 1 << n
    return np.array([psi[(1 << up) | (s << (2 * n))] for s in range(N)]) * math.sqrt(N)


def _g_cos(u, r):
    z = np.asarray(u, dtype=np.float64) / np.linalg.norm(u)
    M = 1 << r
    beta = np.arcsin(np.sqrt((1.0 + z * z) / 2.0)) / math.pi
    return -((M - 1) * np.cos(2 * math.pi * beta) + np.cos(2 * math.pi * (M - 1) * beta)) / M


@pytest.mark.parametrize("n,r,seed", [(1, 2, 0), (1, 5, 1), (2, 3, 2), (2, 4, 3), (2, 6, 4), (3, 3, 5)])
def test_qadc_closed_form(n, r, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(1 << n)
    u[rng.integers(1 << n)] = 0.0
    psi = oracle.qadc_square(u, r, avg=False)
    a = _amps(psi, n, r)
    g = qadc_weights(u, r)
    assert np.abs(a - g).max() < 1e-12
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12


@pytest.mark.parametrize("r", [2, 3, 5, 8, 11])
def test_qadc_fejer_sum_equals_its_fourier_series(r):
    u = np.random.default_rng(r).standard_normal(64)
    assert np.abs(qadc_weights(u, r) - _g_cos(u, r)).max() < 1e-13


@pytest.mark.parametrize("n,r,j", [(1, 2, 1), (2, 3, 2), (2, 4, 0)])
def test_qadc_exact_on_basis_vectors(n, r, j):
    N = 1 << n
    u = np.zeros(N)
    u[j] = -1.0
    psi = oracle.qadc_square(u, r, avg=False)
    want = np.zeros_like(psi)
    up = _layout(n, r)
    for s in range(N):
        want[(s << (2 * n)) | ((1 << up) if s == j else 0)] = 1.0 / math.sqrt(N)
    assert np.abs(psi - want).max() < 1e-12


@pytest.mark.parametrize("r", [3, 4, 6])
def test_qadc_error_bound_and_sign_invariance(r):
    rng = np.random.default_rng(10 + r)
    u = rng.standard_normal(4)
    z2 = (u / np.linalg.norm(u)) ** 2
    a = _amps(oracle.qadc_square(u, r, avg=False), 2, r).real
    assert np.abs(a - z2).max() <= 2.0 / (1 << r)
    flip = u * np.array([1, -1, -1, 1])
    b = _amps(oracle.qadc_square(flip, r, avg=False), 2, r).real
    assert np.abs(a - b).max() < 1e-12


def test_qadc_average():
    n, r = 2, 4
    u = np.random.default_rng(5).standard_normal(1 << n)
    psi = oracle.qadc_square(u, r, avg=True)
    got = psi[1 << _layout(n, r)]
    assert abs(got - qadc_weights(u, r).sum() / (1 << n)) < 1e-12


def test_qadc_loader():
    rng = np.random.default_rng(6)
    for z0 in (0.3, -0.4, 0.0):
        z = rng.standard_normal(8)
        z[0] = z0
        z /= np.linalg.norm(z)
        U = oracle.qadc_loader(z)
        assert np.abs(U @ U - np.eye(8)).max() < 1e-14 and np.abs(U - U.T).max() < 1e-15
        sigma = 1.0 if z[0] >= 0 else -1.0
        assert np.abs(U[:, 0] + sigma * z).max() < 1e-15
