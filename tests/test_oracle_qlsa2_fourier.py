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


def _terms(sy, sz, dy, dz):
    """The select values written out one by one: r = j + 2^sy m, y = j dy, z = k dz
    with k = 1 .. 2^(sz-1) for m < 2^(sz-1) and k = -2^(sz-1) .. -1 above."""
    J, K = 1 << sy, 1 << (sz - 1)
    w, t, sg = [], [], []
    for r in range(J * 2 * K):
        j, m = r % J, r // J
        k = m + 1 if m < K else m - 2 * K
        z = k * dz
        w.append(dy * dz * abs(z) * math.exp(-z * z / 2) / math.sqrt(2 * math.pi))
        t.append(j * dy * z)
        sg.append(1.0 if k > 0 else -1.0)
    return np.array(w), np.array(t), np.array(sg)


@pytest.mark.parametrize("sy,sz,dy,dz", [(1, 1, 0.7, 0.9), (3, 4, 0.3, 0.2), (5, 2, 0.1, 1.3)])
def test_fourier_terms_written_out(sy, sz, dy, dz):
    got = qlsa2.fourier_terms(sy, sz, dy, dz)
    for g, want in zip(got, _terms(sy, sz, dy, dz)):
        np.testing.assert_allclose(g, want, rtol=1e-15, atol=0)


def test_weights_integrate_to_the_gaussian_moment():
    """sum over z of dz |z| e^{-z^2/2} / sqrt(2 pi) -> sqrt(2 / pi), the same for every y:
    |w|_1 = 2^sy dy sqrt(2 / pi) up to the midpoint-free Riemann error O(dz^2)."""
    sy, sz, dy, dz = 3, 12, 0.5, 0.004
    w, _, _ = qlsa2.fourier_terms(sy, sz, dy, dz)
    want = (1 << sy) * dy * math.sqrt(2 / math.pi)
    assert abs(w.sum() - want) <= 1e-5 * want


@pytest.mark.parametrize("kind", ["spd", "indefinite", "complex"])
@pytest.mark.parametrize("sy,sz,dy,dz", [(1, 1, 0.7, 0.9), (2, 2, 0.4, 0.6), (3, 3, 0.3, 0.5)])
def test_circuit_matches_matrix_exponentials(kind, sy, sz, dy, dz):
    rng = np.random.default_rng(sy * 10 + sz)
    N = 8
    A = _herm(rng, N, kind)
    b = rng.standard_normal(N) + (1j * rng.standard_normal(N) if kind == "complex" else 0)
    psi, z, p = oracle.qlsa2_fourier(A, b, sy, sz, dy, dz)
    At = A / np.abs(np.linalg.eigvalsh(A)).max()
    w, t, sg = _terms(sy, sz, dy, dz)
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
