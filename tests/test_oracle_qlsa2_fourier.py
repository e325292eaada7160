"""Pins of the QLSA-2 Fourier-form oracle: the discretised integral
representation is eps-close to 1/x for the parameter rule, and the circuit
(PREP, SELECT of i sign(z_k) exp(-i A~ y_j z_k), PREP^dagger, post-selection)
equals sum_r w_r U_r b^ / |w|_1 computed with scipy's matrix exponential
(independent of the oracle's eigensolver); the solution approaches A^-1 b."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from paper_2307_00391_amd import qlsa2


def _h(x, sy, sz, dy, dz):
    w, t, sg = qlsa2.fourier_terms(sy, sz, dy, dz)
    return (w[None, :] * 1j * sg[None, :] * np.exp(-1j * np.outer(x, t))).sum(1)


@pytest.mark.parametrize("kappa,eps", [(4.0, 5e-2), (10.0, 1e-2), (3.0, 1e-3)])
def test_parameter_rule_error_bound(kappa, eps):
    sy, sz, dy, dz = qlsa2.fourier_parameters(kappa, eps)
    x = np.concatenate([np.linspace(-1, -1 / kappa, 150), np.linspace(1 / kappa, 1, 150)])
    err = np.abs(_h(x, sy, sz, dy, dz) - 1 / x).max()
    assert err <= eps, err


def _herm(rng, N, kind):
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    if kind == "spd":
        return (Q * np.linspace(1.0, 4.0, N)) @ Q.T
    if kind == "indefinite":
        return Q @ np.diag(np.linspace(-3.0, 2.0, N) + 0.2) @ Q.T
    H = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    return H + H.conj().T


@pytest.mark.parametrize("kind", ["spd", "indefinite", "complex"])
@pytest.mark.parametrize("sy,sz,dy,dz", [(1, 1, 0.7, 0.9), (2, 2, 0.4, 0.6), (3, 3, 0.3, 0.5)])
def test_circuit_matches_matrix_exponentials(kind, sy, sz, dy, dz):
    rng = np.random.default_rng(sy * 10 + sz)
    N = 8
    A = _herm(rng, N, kind)
    b = rng.standard_normal(N) + (1j * rng.standard_normal(N) if kind == "complex" else 0)
    psi, z, p = oracle.qlsa2_fourier(A, b, sy, sz, dy, dz)
    At = A / np.abs(np.linalg.eigvalsh(A)).max()
    w, t, sg = qlsa2.fourier_terms(sy, sz, dy, dz)
    bh = b / np.linalg.norm(b)
    want = sum(w[r] * 1j * sg[r] * (expm(-1j * At * t[r]) @ bh) for r in range(w.size)) / w.sum()
    np.testing.assert_allclose(z, want, rtol=0, atol=1e-12)
    assert abs(p - np.linalg.norm(want) ** 2) < 1e-13
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-12


def test_solution_approaches_inverse():
    rng = np.random.default_rng(2)
    N, kappa, eps = 8, 4.0, 1e-2
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    A = (Q * np.exp(np.linspace(0, math.log(kappa), N))) @ Q.T
    b = rng.standard_normal(N)
    sy, sz, dy, dz = qlsa2.fourier_parameters(kappa, eps)
    _, z, p = oracle.qlsa2_fourier(A, b, sy, sz, dy, dz)
    x = np.linalg.solve(A, b)
    F = abs(np.vdot(z / np.linalg.norm(z), x / np.linalg.norm(x)))
    assert F >= 1 - 1e-4, F
