"""GPU parity of the signed (two's-complement) clock in all three HHL modes
against the oracle's gate-level circuit, the fused mode at a larger clock
against the signed closed form, and the Hermitian dilation of a
non-symmetric system."""
import math

import numpy as np
import pytest

import oracle
from paper_2307_00391_amd import binding as B
from tests.closed_form import hhl_closed_form

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _indefinite(rng, N, complex_=True):
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + (1j * rng.standard_normal((N, N)) if complex_ else 0))
    lam = np.concatenate([rng.uniform(-3.0, -0.4, N // 2), rng.uniform(0.4, 3.0, N - N // 2)])
    A = (Q * lam) @ Q.conj().T
    return 0.5 * (A + A.conj().T), np.abs(lam).max()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("n_s,n_c", [(2, 5), (4, 6), (5, 8)])
def test_signed_matches_oracle(dt, mode, n_s, n_c):
    rng = np.random.default_rng(10 * n_s + n_c)
    A, amax = _indefinite(rng, 1 << n_s)
    b = rng.standard_normal(1 << n_s) + 1j * rng.standard_normal(1 << n_s)
    T0 = 2 * math.pi * 0.45 / amax
    psi_r, x_r, pp_r, pa_r = oracle.hhl(A, b, n_c, T0, signed_clock=True)
    st = B.State(n_s + n_c + 1, dt)
    x, res = B.sv_hhl(st.h, A, b, n_c, T0, mode, signed_clock=True)
    if mode == 0:
        assert np.abs(st.get() - psi_r).max() <= TOL[dt]
    st.close()
    assert np.abs(x - x_r).max() <= TOL[dt] / math.sqrt(pp_r) + TOL[dt]
    assert abs(res.p_post - pp_r) <= TOL[dt]
    assert abs(res.p_anc - pa_r) <= TOL[dt]


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_signed_fused_large_clock_closed_form(dt):
    rng = np.random.default_rng(77)
    A, amax = _indefinite(rng, 16, complex_=False)
    b = rng.standard_normal(16)
    n_c = 13
    T0 = 2 * math.pi * 0.45 / amax
    xr, pr = hhl_closed_form(A, b, n_c, T0, signed=True)
    st = B.State(4 + n_c + 1, dt)
    x, res = B.sv_hhl(st.h, A, b, n_c, T0, 1, signed_clock=True)
    st.close()
    tol = 1e-11 if dt == "c128" else 2e-5
    assert np.abs(x - xr).max() <= tol and abs(res.p_post - pr) <= tol


def test_dilation_of_a_nonsymmetric_system():
    rng = np.random.default_rng(5)
    N, n_c = 8, 9
    M = rng.standard_normal((N, N)) + 3 * np.eye(N)
    H = np.block([[np.zeros((N, N)), M], [M.T, np.zeros((N, N))]])
    smax = np.linalg.svd(M, compute_uv=False).max()
    T0 = 2 * math.pi * 0.45 / smax
    b = rng.standard_normal(N)
    bb = np.concatenate([b, np.zeros(N)])
    _, x_r, pp_r, _ = oracle.hhl(H, bb, n_c, T0, signed_clock=True)
    st = B.State(4 + n_c + 1, "c128")
    x, res = B.sv_hhl(st.h, H, bb, n_c, T0, 1, signed_clock=True)
    st.close()
    assert np.abs(x - x_r).max() <= 1e-11 and abs(res.p_post - pp_r) <= 1e-12
    # the lower half approximates M^-1 b (phase estimation error only)
    xc = np.linalg.solve(M, b)
    xc /= np.linalg.norm(xc)
    assert abs(abs(np.vdot(xc, x[N:])) / np.linalg.norm(x[N:]) - 1.0) < 0.05


def test_signed_error_paths():
    st = B.State(2 + 4 + 1, "c64")
    A = np.diag([1.0, -1.0, 2.0, 0.0])
    with pytest.raises(B.SvError) as e:
        B.sv_hhl(st.h, A, np.ones(4), 4, 0.5, 1, signed_clock=True)
    assert e.value.status == B.SV_EINVAL
    with pytest.raises(B.SvError) as e:
        B.sv_hhl(st.h, np.diag([1.0, -1.0, 2.0, 3.0]), np.ones(4), 4, 0.5, 1, signed_clock=False)
    assert e.value.status == B.SV_ENOTPOSDEF
    st.close()
