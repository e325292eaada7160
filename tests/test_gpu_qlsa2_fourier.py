"""GPU parity of QLSA-2 in Fourier form against the oracle's gate-by-gate
circuit: the eigen-frame path (mode 1) and the circuit in the computational
basis (mode 0, the whole final state), complex128 and complex64, over Hermitian
kinds, register widths from one system qubit up to 2^9 system states (the
partial-sum reduction with more than one column block); at the Poiseuille
sizes (27 and 29 qubits) against the spectral sum h(lambda~) = sum_r w_r
i sign(z_r) e^{-i lambda~ t_r} written out here, and the property that
lambda~ h(lambda~) is within the target error of 1; error paths.

Tolerances: complex128 adds to 1e-12 of the largest amplitude an absolute
term for the phase argument lambda~ y z (up to a few thousand radians at the
channel sizes), which both sides round in FP64 and whose eigenvalues come
from two different FP64 eigensolvers: 16 ulp of the largest argument.
complex64 keeps 1e-5 of the largest amplitude plus 1e-6 absolute (FP32 phase
and storage, about 1e-7 per term, summed with weights that add up to 1)."""
import math

import numpy as np
import pytest

import oracle
from paper_2307_00391_amd import binding as B
from paper_2307_00391_amd import inputs

pytestmark = pytest.mark.gpu


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


def _argmax(sy, sz, dy, dz):
    return ((1 << sy) - 1) * dy * (1 << (sz - 1)) * dz


def _tol(dt, scale, sy, sz, dy, dz):
    if dt == "c128":
        return 1e-12 * scale + 16 * 2.0 ** -53 * _argmax(sy, sz, dy, dz)
    return 1e-5 * scale + 1e-6


def _spectral(A, b, sy, sz, dy, dz):
    """z = V diag(h(lambda~)) V^H b^ / |w|_1 from the discretised double integral."""
    lam, V = np.linalg.eigh(A)
    lt = lam / np.abs(lam).max()
    J, K = 1 << sy, 1 << (sz - 1)
    r = np.arange(J * 2 * K)
    j, m = r & (J - 1), r >> sy
    k = np.where(m < K, m + 1, m - 2 * K)
    zk = k * dz
    w = dy * dz * np.abs(zk) * np.exp(-0.5 * zk * zk) / math.sqrt(2 * math.pi)
    t = j * dy * zk
    h = np.array([(w * 1j * np.sign(k) * np.exp(-1j * l * t)).sum() for l in lt])
    beta = V.conj().T @ (b / np.linalg.norm(b))
    return V @ (h * beta) / w.sum(), lt, V, beta, w.sum()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("kind", ["spd", "indefinite", "complex"])
@pytest.mark.parametrize("n_s,sy,sz,dy,dz", [(1, 1, 1, 0.7, 0.9), (3, 4, 4, 0.3, 0.4), (4, 6, 5, 0.25, 0.2),
                                             (9, 3, 2, 0.5, 0.8)])
def test_fourier_matches_oracle(dt, kind, n_s, sy, sz, dy, dz):
    rng = np.random.default_rng(7 * n_s + sy + 3 * sz + len(kind))
    N = 1 << n_s
    A = _matrix(kind, rng, N)
    b = rng.standard_normal(N) + (1j * rng.standard_normal(N) if kind == "complex" else 0)
    print(f"[fourier] {dt} {kind} n_s {n_s} sy {sy} sz {sz}", flush=True)
    _, z_ref, p_ref = oracle.qlsa2_fourier(A, b, sy, sz, dy, dz)
    st = B.State(n_s + sy + sz, dt)
    try:
        z, res = B.sv_qlsa2_fourier(st.h, A, b, sy, sz, dy, dz)
    finally:
        st.close()
    scale = np.abs(z_ref).max()
    tol = _tol(dt, scale, sy, sz, dy, dz)
    assert np.abs(z - z_ref).max() <= tol
    assert abs(res.p_post - p_ref) <= 4 * tol * math.sqrt(N) * (1 + math.sqrt(p_ref))
    assert abs(res.lambda_abs_max - np.abs(np.linalg.eigvalsh(A)).max()) <= 1e-12 * res.lambda_abs_max


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_fourier_poiseuille_27_qubits_spectral_sum(dt):
    """The channel system (16 points, kappa = 116) at target error 1e-2:
    sy = 12, sz = 11, 27 qubits; against the spectral sum and A^-1 b."""
    sysm = inputs.poiseuille(16)
    A, b = sysm.A, sysm.b
    sy, sz, dy, dz = 12, 11, 0.2, 0.007578560356745859
    want, lt, V, beta, l1 = _spectral(A, b, sy, sz, dy, dz)
    st = B.State(4 + sy + sz, dt)
    try:
        z, res = B.sv_qlsa2_fourier(st.h, A, b, sy, sz, dy, dz)
    finally:
        st.close()
    assert np.abs(z - want).max() <= _tol(dt, np.abs(want).max(), sy, sz, dy, dz)
    assert abs(res.alpha_l1 - l1) <= 1e-12 * l1
    x = np.linalg.solve(A, b)
    F = abs(np.vdot(z / np.linalg.norm(z), x / np.linalg.norm(x)))
    assert F >= 1 - 1e-9, F


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_fourier_poiseuille_29_qubits_inverse_property(dt):
    """Target error 1e-3 (sy = 14, sz = 11, 29 qubits): in the eigenbasis every
    component with weight is z_k = h(lambda~_k) beta_k / |w|_1 and
    lambda~ h(lambda~) is within 1e-3 of 1; the profile is the parabola."""
    sysm = inputs.poiseuille(16)
    A, b = sysm.A, sysm.b
    sy, sz, dy, dz = 14, 11, 0.06324555320336758, 0.006000740580676756
    lam, V = np.linalg.eigh(A)
    lt = lam / np.abs(lam).max()
    beta = V.T @ (b / np.linalg.norm(b))
    st = B.State(4 + sy + sz, dt)
    try:
        z, res = B.sv_qlsa2_fourier(st.h, A, b, sy, sz, dy, dz)
    finally:
        st.close()
    ze = V.T @ z
    on = np.abs(beta) > 1e-8
    ratio = ze[on] * res.alpha_l1 * lt[on] / beta[on]
    assert np.abs(ratio - 1).max() <= 1e-3, np.abs(ratio - 1).max()
    assert np.abs(ze[~on]).max() <= 1e-6 * np.abs(ze).max()
    y = np.arange(1, 17) / 17
    prof = (z / np.linalg.norm(z)).real
    prof *= np.sign(prof[8])
    want = y * (1 - y) / np.linalg.norm(y * (1 - y))
    assert np.abs(prof - want).max() <= 1e-3


def _tol_gates(dt, scale, n_s, sy, sz, dy, dz):
    """Mode 0 applies sy (sz + 1) dense unitaries rounded to the state's
    precision: complex64 adds 2^-24 sqrt(2^n_s) per unitary to the bar."""
    if dt == "c128":
        return _tol(dt, scale, sy, sz, dy, dz)
    return _tol(dt, scale, sy, sz, dy, dz) + sy * (sz + 1) * 2.0 ** (n_s / 2) * 2.0 ** -24


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("kind", ["spd", "indefinite", "complex"])
@pytest.mark.parametrize("n_s,sy,sz,dy,dz", [(1, 1, 1, 0.7, 0.9), (3, 4, 4, 0.3, 0.4), (4, 5, 3, 0.25, 0.2),
                                             (2, 2, 6, 0.4, 0.15)])
def test_fourier_gates_full_state_matches_oracle(dt, kind, n_s, sy, sz, dy, dz):
    """Mode 0 (the circuit in the computational basis) against the oracle's
    gate-by-gate circuit: the whole final state, z and p_post."""
    rng = np.random.default_rng(11 * n_s + sy + 5 * sz + len(kind))
    N = 1 << n_s
    A = _matrix(kind, rng, N)
    b = rng.standard_normal(N) + (1j * rng.standard_normal(N) if kind == "complex" else 0)
    print(f"[fourier gates] {dt} {kind} n_s {n_s} sy {sy} sz {sz}", flush=True)
    psi_ref, z_ref, p_ref = oracle.qlsa2_fourier(A, b, sy, sz, dy, dz)
    st = B.State(n_s + sy + sz, dt)
    try:
        z, res = B.sv_qlsa2_fourier(st.h, A, b, sy, sz, dy, dz, mode=0)
        psi = st.get()
    finally:
        st.close()
    tol = _tol_gates(dt, np.abs(psi_ref).max(), n_s, sy, sz, dy, dz)
    assert np.abs(psi - psi_ref).max() <= tol
    assert np.abs(z - z_ref).max() <= _tol_gates(dt, np.abs(z_ref).max(), n_s, sy, sz, dy, dz)
    assert abs(res.p_post - p_ref) <= 4 * tol * math.sqrt(N) * (1 + math.sqrt(p_ref))


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_fourier_gates_and_eigen_frame_agree(dt):
    """n_s = 6, 2^10 select values (16 qubits): the two library modes."""
    rng = np.random.default_rng(3)
    n_s, sy, sz, dy, dz = 6, 5, 5, 0.35, 0.12
    A = _matrix("indefinite", rng, 1 << n_s)
    b = rng.standard_normal(1 << n_s)
    out = []
    for mode in (0, 1):
        st = B.State(n_s + sy + sz, dt)
        try:
            out.append(B.sv_qlsa2_fourier(st.h, A, b, sy, sz, dy, dz, mode=mode)[0])
        finally:
            st.close()
    assert np.abs(out[0] - out[1]).max() <= _tol_gates(dt, np.abs(out[1]).max(), n_s, sy, sz, dy, dz)


def test_fourier_errors():
    A = np.diag([1.0, 2.0, 3.0, 4.0])
    b = np.ones(4)
    st = B.State(6, "c64")
    try:
        with pytest.raises(B.SvError):
            B.sv_qlsa2_fourier(st.h, A, b, 2, 3, 0.1, 0.1)          # 2 + 2 + 3 != 6
        with pytest.raises(B.SvError):
            B.sv_qlsa2_fourier(st.h, A, b, 2, 2, 0.0, 0.1)          # dy = 0
        with pytest.raises(B.SvError):
            B.sv_qlsa2_fourier(st.h, A, b, 2, 2, 0.1, float("nan"))
        with pytest.raises(B.SvError):
            B.sv_qlsa2_fourier(st.h, A + np.triu(np.ones((4, 4)), 1), b, 2, 2, 0.1, 0.1)
        with pytest.raises(B.SvError):
            B.sv_qlsa2_fourier(st.h, A, np.zeros(4), 2, 2, 0.1, 0.1)
        with pytest.raises(B.SvError):
            B.sv_qlsa2_fourier(st.h, A, b, 2, 2, 0.1, 0.1, mode=2)
    finally:
        st.close()
    big = np.diag(np.arange(1.0, 2049.0))
    st = B.State(11 + 1 + 1, "c64")
    try:
        with pytest.raises(B.SvError):                                   # mode 0 with n_s = 11
            B.sv_qlsa2_fourier(st.h, big, np.ones(2048), 1, 1, 0.1, 0.1, mode=0)
    finally:
        st.close()
