"""Pins of the QLSA-2 oracle (Chebyshev linear combination of unitaries, after
the cited Childs-Kothari-Somma construction; the paper defers the details):
the coefficients against exact integer binomials, the exact Chebyshev
identity of the truncated inverse, its error bound, the select-register
preparation against the pinned QSP-1 tree, and the whole circuit against
the matrix Chebyshev recurrence (no eigen-decomposition) and against A^-1 b."""
import math
from fractions import Fraction

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

import oracle


def _alpha_exact(B, J):
    out = []
    for j in range(J):
        tail = sum(Fraction(math.comb(2 * B, B + i), 4 ** B) for i in range(j + 1, B + 1))
        out.append(float(4 * (-1) ** j * tail))
    return np.array(out)


@pytest.mark.parametrize("B", [1, 2, 3, 7, 20, 45])
def test_coefficients_exact_binomials(B):
    J = B + 3
    got = oracle.cks_coeffs(B, J)
    want = _alpha_exact(B, J)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-300)
    assert np.all(got[B:] == 0.0)


@pytest.mark.parametrize("B", [1, 4, 25, 200])
def test_chebyshev_identity(B):
    """sum_{j<B} alpha_j T_{2j+1}(x) = (1 - (1 - x^2)^B) / x exactly."""
    a = oracle.cks_coeffs(B, B)
    c = np.zeros(2 * B)
    c[1::2] = a
    x = np.concatenate([np.linspace(-1, -0.01, 50), np.linspace(0.01, 1, 50)])
    want = (1 - (1 - x * x) ** B) / x
    np.testing.assert_allclose(C.chebval(x, c), want, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("kappa,eps", [(4.0, 1e-3), (10.0, 1e-4), (30.0, 1e-2)])
def test_error_bound_of_the_degree_rule(kappa, eps):
    """With B = ceil(kappa^2 ln(kappa / eps)), |g(x) - 1/x| <= eps on 1/kappa <= |x| <= 1."""
    B = math.ceil(kappa ** 2 * math.log(kappa / eps))
    x = np.linspace(1 / kappa, 1, 2001)
    err = np.abs((1 - (1 - x * x) ** B) / x - 1 / x).max()
    assert err <= eps


def test_qsp_apply_matches_qsp_and_inverts():
    rng = np.random.default_rng(4)
    n, q_lo, m = 7, 2, 4
    b = rng.standard_normal(1 << m) + 1j * rng.standard_normal(1 << m)
    b[3] = 0
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    np.testing.assert_allclose(oracle.qsp_apply(psi.copy(), q_lo, b), oracle.qsp(n, q_lo, b), atol=1e-14)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.linalg.norm(v)
    w = oracle.qsp_apply(oracle.qsp_apply(v.copy(), q_lo, b), q_lo, b, inverse=True)
    np.testing.assert_allclose(w, v, atol=1e-13)


def _cheb_matrix_sum(At, alpha, b):
    """sum_j alpha_j T_{2j+1}(At) b by the recurrence T_{k+1} = 2 At T_k - T_{k-1}."""
    Tprev, Tcur = b.copy(), At @ b           # T_0 b, T_1 b
    out = alpha[0] * Tcur
    for j in range(1, alpha.size):
        for _ in range(2):                  # advance two degrees: 2j - 1 -> 2j + 1
            Tprev, Tcur = Tcur, 2 * At @ Tcur - Tprev
        out = out + alpha[j] * Tcur
    return out


def _spd(rng, N, kappa):
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    lam = np.exp(np.linspace(0, math.log(kappa), N))
    return (Q * lam) @ Q.T


@pytest.mark.parametrize("kind", ["spd", "indefinite", "complex"])
@pytest.mark.parametrize("s,B", [(1, 3), (3, 12), (5, 40)])
def test_circuit_matches_matrix_chebyshev(kind, s, B):
    rng = np.random.default_rng(10 * s + B)
    N = 8
    if kind == "spd":
        A = _spd(rng, N, 5.0)
    elif kind == "indefinite":
        Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
        A = Q @ np.diag(np.linspace(-2.0, 3.0, N) + 0.15) @ Q.T
    else:
        H = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
        A = H + H.conj().T
    b = rng.standard_normal(N) + (1j * rng.standard_normal(N) if kind == "complex" else 0)
    psi, z, p = oracle.qlsa2(A, b, s, B)
    At = A / np.abs(np.linalg.eigvalsh(A)).max()
    alpha = oracle.cks_coeffs(B, 1 << s)
    want = _cheb_matrix_sum(At, alpha, b / np.linalg.norm(b)) / np.abs(alpha).sum()
    np.testing.assert_allclose(z, want, rtol=0, atol=1e-12)
    assert abs(p - np.linalg.norm(want) ** 2) < 1e-13
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-12


def test_solution_approaches_inverse():
    """B and J from the error bound: the normalised output is A^-1 b to O(eps)."""
    rng = np.random.default_rng(7)
    N, kappa, eps = 8, 6.0, 1e-3
    A = _spd(rng, N, kappa)
    b = rng.standard_normal(N)
    B = math.ceil(kappa ** 2 * math.log(kappa / eps))
    j0 = math.ceil(math.sqrt(B * math.log(4 * B / eps)))
    s = max(1, math.ceil(math.log2(j0 + 1)))
    _, z, p = oracle.qlsa2(A, b, s, B)
    x = np.linalg.solve(A, b)
    F = abs(np.vdot(z / np.linalg.norm(z), x / np.linalg.norm(x)))
    assert F >= 1 - 1e-5, F
    assert p > 0
