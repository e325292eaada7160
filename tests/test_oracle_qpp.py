"""Pins of the QPP gradient oracles (appendix "Velocity gradients - LCU
method" and "- spectral method") against closed forms: the block structure
of the LCU circuit worked out by hand, exactness of central differences on a
quadratic with zero walls, exactness of spectral differentiation on
trigonometric polynomials, the Nyquist mode, norm preservation, and the
U_avg = H^(x)m sum of amplitudes (main text, QPP section)."""
import numpy as np
import pytest

import oracle


def _rand_state(rng, n):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def _embed(phi, n, q_lo):
    """phi on register [q_lo, q_lo + m), every other qubit |0>."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    for j, a in enumerate(phi):
        psi[j << q_lo] = a
    return psi


def _block(psi, q_lo, m, fixed):
    """Register amplitudes at the other qubits' values given by `fixed`."""
    return np.array([psi[fixed | (j << q_lo)] for j in range(1 << m)])


def _shift(N):
    """(S u)_j = u_{j+1}, zero past the end (textbook truncated shift)."""
    return np.eye(N, k=1)


# ------------------------------------------------------------------ LCU

@pytest.mark.parametrize("m,q_lo,sel_lo", [(1, 0, 1), (2, 0, 2), (3, 0, 3), (4, 2, 0), (5, 0, 5), (3, 1, 5)])
def test_lcu_blocks_closed_form(m, q_lo, sel_lo):
    """From select |00>, the four select blocks are (by hand):
    00: (S - S^T)/2 = h D;  01: (|N-1><0| - |0><N-1|)/2;
    10: (S + S^T)/2;        11: (|N-1><0| + |0><N-1|)/2."""
    rng = np.random.default_rng(7 + m)
    N = 1 << m
    n = max(q_lo + m, sel_lo + 2)
    phi = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    phi /= np.linalg.norm(phi)
    psi = oracle.lcu_derivative(_embed(phi, n, q_lo), q_lo, m, sel_lo)
    S = _shift(N)
    corner_a = np.zeros((N, N)); corner_a[N - 1, 0] = 1.0
    corner_b = np.zeros((N, N)); corner_b[0, N - 1] = 1.0
    want = {0: 0.5 * (S - S.T), 1: 0.5 * (corner_a - corner_b), 2: 0.5 * (S + S.T), 3: 0.5 * (corner_a + corner_b)}
    for sel, M in want.items():
        got = _block(psi, q_lo, m, sel << sel_lo)
        np.testing.assert_allclose(got, M @ phi, rtol=0, atol=1e-14)
    # nothing else is populated
    tot = sum(np.linalg.norm(_block(psi, q_lo, m, s << sel_lo)) ** 2 for s in range(4))
    assert abs(tot - 1.0) < 1e-13


@pytest.mark.parametrize("m", [2, 3, 4, 6, 8])
def test_lcu_exact_on_poiseuille_quadratic(m):
    """Central differences are exact on a quadratic, and the profile
    y(1 - y) vanishes at the walls, so h D u = h (1 - 2 y_j) exactly."""
    N = 1 << m
    h = 1.0 / (N + 1)
    y = h * np.arange(1, N + 1)
    u = y * (1 - y)
    nu = np.linalg.norm(u)
    psi = oracle.lcu_derivative(_embed(u / nu, m + 2, 0), 0, m, m)
    got = _block(psi, 0, m, 0) * nu / h
    np.testing.assert_allclose(got.real, 1 - 2 * y, rtol=0, atol=1e-12)
    assert np.max(np.abs(got.imag)) < 1e-15
    # probability of the select-|00> outcome = h^2 |D u|^2 / |u|^2
    p = oracle.norm2(psi, 3 << m, 0)
    assert abs(p - h * h * np.sum((1 - 2 * y) ** 2) / nu ** 2) < 1e-14


def test_lcu_unitary_on_any_input():
    """The circuit is V^dagger G V with unitary parts: norms are kept for a
    state with every select value populated, and two inputs keep their
    inner product."""
    rng = np.random.default_rng(3)
    a, b = _rand_state(rng, 7), _rand_state(rng, 7)
    ip = np.vdot(a, b)
    oa = oracle.lcu_derivative(a.copy(), 1, 4, 5)
    ob = oracle.lcu_derivative(b.copy(), 1, 4, 5)
    assert abs(np.linalg.norm(oa) - 1.0) < 1e-13
    assert abs(np.vdot(oa, ob) - ip) < 1e-13


def test_lcu_rejects_overlap():
    psi = np.zeros(1 << 6, dtype=np.complex128)
    psi[0] = 1
    with pytest.raises(oracle.OracleError):
        oracle.lcu_derivative(psi, 0, 4, 3)


def test_uavg_sums_the_gradient():
    """U_avg = H on every register qubit puts sum_j w_j / sqrt(N) on |0>.
    For the zero-wall central difference the sum telescopes:
    sum_j (D u)_j = (u_{N-1} - u_0) / 2h."""
    rng = np.random.default_rng(11)
    m = 5
    N = 1 << m
    h = 1.0 / (N + 1)
    u = rng.standard_normal(N)
    nu = np.linalg.norm(u)
    psi = oracle.lcu_derivative(_embed(u / nu, m + 2, 0), 0, m, m)
    r = 1 / np.sqrt(2)
    H = np.array([[r, r], [r, -r]])
    for q in range(m):
        oracle.apply_gate(psi, q, H)
    s = psi[0] * np.sqrt(N) * nu / h
    assert abs(s - (u[N - 1] - u[0]) / (2 * h)) < 1e-11


# ------------------------------------------------------------- spectral

def _lmax(m):
    return 2 * np.pi * ((1 << (m - 1)) - 1)


@pytest.mark.parametrize("m,q_lo,anc", [(2, 0, 2), (3, 1, 0), (5, 0, 5), (6, 0, 6), (7, 1, 0)])
def test_spectral_exact_on_trig_polynomial(m, q_lo, anc):
    """For phi_j = sum_p a_p exp(2 pi i p j / N), |p| < N/2, the anc = 1 block
    is sum_p 2 pi i p a_p exp(2 pi i p j / N) / Lambda_max exactly."""
    rng = np.random.default_rng(100 + m)
    N = 1 << m
    n = max(q_lo + m, anc + 1)
    ps = np.arange(-(N // 2) + 1, N // 2)
    a = rng.standard_normal(ps.size) + 1j * rng.standard_normal(ps.size)
    j = np.arange(N)
    E = np.exp(2j * np.pi * np.outer(j, ps) / N)
    phi = E @ a
    d = E @ (2j * np.pi * ps * a)
    nrm = np.linalg.norm(phi)
    psi = oracle.spectral_derivative(_embed(phi / nrm, n, q_lo), q_lo, m, anc)
    got = _block(psi, q_lo, m, 1 << anc) * nrm * _lmax(m)
    np.testing.assert_allclose(got, d, rtol=0, atol=1e-11 * np.max(np.abs(d)))
    assert abs(np.linalg.norm(psi) - 1) < 1e-13


def test_spectral_sine_gives_cosine():
    m = 6
    N = 1 << m
    y = np.arange(N) / N
    u = np.sin(2 * np.pi * 3 * y)
    nu = np.linalg.norm(u)
    psi = oracle.spectral_derivative(_embed(u / nu, m + 1, 0), 0, m, m)
    got = _block(psi, 0, m, 1 << m) * nu * _lmax(m)
    np.testing.assert_allclose(got.real, 6 * np.pi * np.cos(2 * np.pi * 3 * y), rtol=0, atol=1e-11)
    assert np.max(np.abs(got.imag)) < 1e-11


def test_spectral_nyquist_and_constant_vanish():
    """Lambda is 0 at k = 0 and k = N/2: a constant and (-1)^j have zero
    derivative, so the anc = 1 block is empty."""
    m = 4
    N = 1 << m
    for u in (np.ones(N), (-1.0) ** np.arange(N)):
        psi = oracle.spectral_derivative(_embed(u / np.linalg.norm(u), m + 1, 0), 0, m, m)
        assert oracle.norm2(psi, 1 << m, 1 << m) < 1e-28


def test_spectral_matches_numpy_fft():
    """Library route for the same definition: ifft(Lambda * fft(u))."""
    rng = np.random.default_rng(5)
    m = 5
    N = 1 << m
    u = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    u /= np.linalg.norm(u)
    k = np.arange(N)
    lam = np.where(k < N // 2, 2j * np.pi * k, np.where(k == N // 2, 0, 2j * np.pi * (k - N)))
    want = np.fft.ifft(lam * np.fft.fft(u))
    psi = oracle.spectral_derivative(_embed(u, m + 1, 0), 0, m, m)
    np.testing.assert_allclose(_block(psi, 0, m, 1 << m) * _lmax(m), want, rtol=0, atol=1e-11)


def test_spectral_rejects_small_register():
    psi = np.zeros(8, dtype=np.complex128)
    psi[0] = 1
    with pytest.raises(oracle.OracleError):
        oracle.spectral_derivative(psi, 0, 1, 2)
