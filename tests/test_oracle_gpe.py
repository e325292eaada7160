"""Pins of the gapped-phase-estimation oracle (the building block of the
variable-time solver in the cited Childs-Kothari-Somma construction that the
paper's QLSA-2 names): the HHL circuit with a flag Ry(pi) on clock values
|y| >= cut in place of the inversion rotation, then the uncompute.

Pinned against the mathematics, with numpy's eigh (not the oracle's Jacobi
solver): after phase estimation the clock holds alpha_y with |alpha_y|^2 =
K(phi - y/M) (Fejer kernel), and the uncompute returns each clock value to 0
with amplitude conj(alpha_y), so the flag = 1, clock = 0 amplitude of
eigenvector j is g_j = sum_{|y| >= cut} K(phi_j - y/M) and the flag = 0 one
h_j = the sum over the rest; P(flag = 1) = sum_j |beta_j|^2 g_j.  On a clock
grid (lam_j T0 M / 2 pi integer) the estimate is exact: the flag = 1 output is
the projection of b onto the eigenvectors with |y_j| >= cut, and nothing stays
on clock values != 0."""
import math

import numpy as np
import pytest

import oracle
from paper_2307_00391_amd import inputs
from tests.closed_form import gpe_closed_form


def _blocks(psi, n_s, n_c):
    N, M = 1 << n_s, 1 << n_c
    st = psi.reshape(2, M, N)              # [flag][clock][system]
    return st[1, 0], st[0, 0], st[:, 1:]


@pytest.mark.parametrize("kind,signed,n_s,n_c,cut", [("spd", False, 3, 5, 9), ("spd", False, 2, 6, 20),
                                                     ("indefinite", True, 3, 5, 4), ("complex", True, 3, 6, 11)])
def test_gpe_matches_fejer_closed_form(kind, signed, n_s, n_c, cut):
    rng = np.random.default_rng(n_s * 10 + n_c + cut)
    N = 1 << n_s
    if kind == "spd":
        A, lmin, lmax = inputs.random_spd_tridiag(rng, N, 30.0)
        T0 = inputs.t0_top_of_clock(lmax, n_c) * 0.9
    else:
        if kind == "indefinite":
            Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
            A = Q @ np.diag(np.linspace(-2.0, 3.0, N) + 0.13) @ Q.T
        else:
            Z = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
            A = Z + Z.conj().T
        T0 = 0.45 * 2 * math.pi / np.abs(np.linalg.eigvalsh(A)).max()
    b = rng.standard_normal(N) + (1j * rng.standard_normal(N) if kind == "complex" else 0)
    psi, x, p_post, p_flag = oracle.gapped_pe(A, b, n_c, T0, cut, signed)
    z1, z0, pp, pf = gpe_closed_form(A, b, n_c, T0, cut, signed)
    f1, f0, _ = _blocks(psi, n_s, n_c)
    np.testing.assert_allclose(f1, z1, rtol=0, atol=1e-12)
    np.testing.assert_allclose(f0, z0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(x, z1 / np.linalg.norm(z1), rtol=0, atol=1e-11)
    assert abs(p_post - pp) < 1e-12 and abs(p_flag - pf) < 1e-12
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12
    assert 0 < p_post <= p_flag < 1


@pytest.mark.parametrize("signed", [False, True])
def test_gpe_exact_on_clock_grid(signed):
    rng = np.random.default_rng(31 + signed)
    n_s, n_c, T0 = 3, 5, 0.6
    N, M = 1 << n_s, 1 << n_c
    yj = np.array([1, 3, 5, 8, 9, 12, 14, 15]) * (np.where(rng.random(N) < 0.5, -1, 1) if signed else 1)
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    A = Q @ np.diag(2 * math.pi * yj / (M * T0)) @ Q.T
    A = (A + A.T) / 2
    b = rng.standard_normal(N)
    cut = 8
    psi, x, p_post, p_flag = oracle.gapped_pe(A, b, n_c, T0, cut, signed)
    beta = Q.T @ (b / np.linalg.norm(b))
    big = np.abs(yj) >= cut
    f1, f0, rest = _blocks(psi, n_s, n_c)
    np.testing.assert_allclose(f1, Q @ (beta * big), atol=1e-12)
    np.testing.assert_allclose(f0, Q @ (beta * ~big), atol=1e-12)
    assert np.abs(rest).max() < 1e-12
    assert abs(p_post - np.sum(beta[big] ** 2)) < 1e-12 and abs(p_flag - p_post) < 1e-12


def test_gpe_wrong_flag_within_the_fejer_tail_bound():
    """One eigenvector with its estimate y_t at distance D from the cut: the
    wrong flag's probability is the Fejer mass at circular distances >= D on
    one side and beyond the clock's wrap on the other, each side below
    1/(pi^2 (D - 1/2)) in the continuum limit (x 1.2 for the finite M);
    on the grid (integer y_t) the flag is exact."""
    n_c, cut, T0 = 7, 20, 1.0
    M = 1 << n_c
    for yt in np.arange(3.0, 60.0, 0.5):
        A = np.diag([2 * math.pi * yt / (M * T0), 1.0])
        _, _, _, p = oracle.gapped_pe(A, np.array([1.0, 0.0]), n_c, T0, cut)
        if yt == int(yt):
            assert abs(p - (1.0 if yt >= cut else 0.0)) < 1e-12, yt
        elif yt < cut:
            if cut - yt < 1:            # within half a clock unit of the cut: no bound
                continue
            bound = 1 / (math.pi ** 2 * (cut - yt - 0.5)) + 1 / (math.pi ** 2 * (yt + 0.5))
            assert p <= 1.2 * bound, (yt, p, bound)
        else:
            bound = 1 / (math.pi ** 2 * (yt - cut + 0.5)) + 1 / (math.pi ** 2 * (M - yt - 0.5))
            assert 1 - p <= 1.2 * bound, (yt, 1 - p, bound)


def test_gpe_rejects_cut_zero():
    with pytest.raises(oracle.OracleError):
        oracle.gapped_pe(np.eye(2), np.ones(2), 3, 1.0, 0)
