"""GPU parity of QLSA-2 (Chebyshev LCU over a qubitized walk) against the
oracle: both library modes (the circuit in the computational basis with
dense controlled walk powers, and the eigen-frame form), complex128 to 1e-12
and complex64 to 1e-5 relative to the largest amplitude; the full final state
of mode 0; at sizes beyond the oracle's repeated walk products, the matrix
Chebyshev recurrence that pins the oracle; the Poiseuille solve against A^-1 b;
error paths."""
import math

import numpy as np
import pytest

import oracle
from paper_2307_00391_amd import binding as B
from paper_2307_00391_amd import inputs

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _matrix(kind, rng, N):
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    if kind == "spd":
        return (Q * np.exp(np.linspace(0, math.log(5.0), N))) @ Q.T
    if kind == "indefinite":
        return Q @ np.diag(np.linspace(-2.0, 3.0, N) + 0.15) @ Q.T
    H = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    return H + H.conj().T


def _cheb_reference(A, b, s, Bdeg):
    """sum_j alpha_j T_{2j+1}(A~) b^ / |alpha|_1 by the matrix recurrence."""
    At = A / np.abs(np.linalg.eigvalsh(A)).max()
    alpha = oracle.cks_coeffs(Bdeg, 1 << s)
    bh = b / np.linalg.norm(b)
    Tprev, Tcur = bh.astype(np.complex128), At @ bh
    out = alpha[0] * Tcur
    for j in range(1, alpha.size):
        for _ in range(2):
            Tprev, Tcur = Tcur, 2 * At @ Tcur - Tprev
        out = out + alpha[j] * Tcur
    return out / np.abs(alpha).sum()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("kind", ["spd", "indefinite", "complex"])
@pytest.mark.parametrize("n_s,s,Bdeg", [(1, 1, 2), (3, 3, 12), (4, 5, 40), (3, 2, 300)])
def test_qlsa2_matches_oracle(dt, mode, kind, n_s, s, Bdeg):
    rng = np.random.default_rng(100 * n_s + 10 * s + len(kind))
    N = 1 << n_s
    A = _matrix(kind, rng, N)
    b = rng.standard_normal(N) + (1j * rng.standard_normal(N) if kind == "complex" else 0)
    psi_ref, z_ref, p_ref = oracle.qlsa2(A, b, s, Bdeg)
    st = B.State(n_s + 1 + s, dt)
    z, res = B.sv_qlsa2(st.h, A, b, s, Bdeg, mode)
    scale = np.abs(z_ref).max()
    assert np.abs(z - z_ref).max() <= TOL[dt] * scale
    assert abs(res.p_post - p_ref) <= 10 * TOL[dt] * p_ref
    if mode == 0:
        got = st.get()
        assert np.abs(got - psi_ref).max() <= TOL[dt] * np.abs(psi_ref).max()
    st.close()
    assert abs(res.lambda_abs_max - np.abs(np.linalg.eigvalsh(A)).max()) <= 1e-12 * res.lambda_abs_max


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("mode", [0, 1])
def test_qlsa2_larger_against_matrix_chebyshev(dt, mode):
    """n_s = 7, 2^9 terms: beyond the oracle's repeated walk products; the
    reference is the matrix recurrence that pins the oracle."""
    rng = np.random.default_rng(5)
    n_s, s, Bdeg = 7, 9, 4000
    A = _matrix("indefinite", rng, 1 << n_s)
    b = rng.standard_normal(1 << n_s)
    want = _cheb_reference(A, b, s, Bdeg)
    st = B.State(n_s + 1 + s, dt)
    z, res = B.sv_qlsa2(st.h, A, b, s, Bdeg, mode)
    st.close()
    assert np.abs(z - want).max() <= 10 * TOL[dt] * np.abs(want).max()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_qlsa2_poiseuille_solution(dt):
    """The paper's Poiseuille system (16 points, kappa = 116): B and J from
    eps = 1e-3; the output is A^-1 b (the parabola) to O(eps)."""
    sysm = inputs.poiseuille(16)
    A = sysm.A
    b = sysm.b
    lam = np.linalg.eigvalsh(A)
    kappa = lam.max() / lam.min()
    eps = 1e-3
    Bdeg = math.ceil(kappa ** 2 * math.log(kappa / eps))
    j0 = math.ceil(math.sqrt(Bdeg * math.log(4 * Bdeg / eps)))
    s = math.ceil(math.log2(j0 + 1))
    st = B.State(4 + 1 + s, dt)
    z, res = B.sv_qlsa2(st.h, A, b, s, Bdeg, 1)
    st.close()
    x = np.linalg.solve(A, b)
    F = abs(np.vdot(z / np.linalg.norm(z), x / np.linalg.norm(x)))
    assert F >= 1 - 1e-5, F
    y = np.arange(1, 17) / 17
    prof = (z / np.linalg.norm(z)).real
    prof *= np.sign(prof[8])
    want = y * (1 - y) / np.linalg.norm(y * (1 - y))
    assert np.abs(prof - want).max() <= 5e-3


def test_qlsa2_modes_agree_c64_16_qubits():
    rng = np.random.default_rng(9)
    n_s, s, Bdeg = 6, 9, 2000
    A = _matrix("spd", rng, 1 << n_s)
    b = rng.standard_normal(1 << n_s)
    out = []
    for mode in (0, 1):
        st = B.State(n_s + 1 + s, "c64")
        z, _ = B.sv_qlsa2(st.h, A, b, s, Bdeg, mode)
        st.close()
        out.append(z)
    assert np.abs(out[0] - out[1]).max() <= 1e-5 * np.abs(out[1]).max()


def test_qlsa2_errors():
    A = np.diag([1.0, 2.0, 3.0, 4.0])
    b = np.ones(4)
    st = B.State(5, "c64")
    try:
        with pytest.raises(B.SvError):
            B.sv_qlsa2(st.h, A, b, 3, 10, 1)          # 2 + 1 + 3 != 5
        with pytest.raises(B.SvError):
            B.sv_qlsa2(st.h, A, b, 2, 0, 1)           # B = 0
        with pytest.raises(B.SvError):
            B.sv_qlsa2(st.h, A, b, 2, 10, 2)          # mode
        with pytest.raises(B.SvError):
            B.sv_qlsa2(st.h, A + np.triu(np.ones((4, 4)), 1), b, 2, 10, 1)   # not Hermitian
        with pytest.raises(B.SvError):
            B.sv_qlsa2(st.h, A, np.zeros(4), 2, 10, 1)
    finally:
        st.close()
