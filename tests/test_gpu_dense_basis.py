"""HHL on a prepared eigen-decomposition with a dense real eigenbasis
(sv_hhl_prepare_eig): the basis changes run as FP64 matrix-vector products
over V.

* small operators (n_s = 5): A = V diag(lam) V^T from a random orthogonal V,
  every mode against the gate-level oracle on the dense A;
* n_s = 12 against the closed form;
* 32 qubits (n_s = 16, n_c = 15): V = H (P_hi (x) P_lo), the eigenbasis of the
  Kronecker-sum operator of the 32-qubit workload turned by a Householder
  reflection H = I - 2 w w^T / |w|^2 about a dense random w, so that
  A = V diag(lam) V^T is a dense, non-separable 2^16 x 2^16 operator with the
  same spectrum (kappa = 1000).  V (32 GiB) is formed on the device; the
  closed form runs through the factors on the host.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2307_00391_amd import binding as B
from paper_2307_00391_amd import inputs
from tests.closed_form import g_h_of_phi_wide

pytestmark = pytest.mark.gpu

REL = {"c64": 1e-5, "c128": 1e-10}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _orthogonal(rng, N):
    Q, R = np.linalg.qr(rng.standard_normal((N, N)))
    return Q * np.sign(np.diag(R))[None, :]


def _closed_form(V, lam, b, n_c, T0):
    beta = V.T @ (b / np.linalg.norm(b))
    g, h = g_h_of_phi_wide(lam * T0 / (2 * math.pi), n_c, workers=4)
    z = beta * g
    p = float(np.sum(np.abs(z) ** 2))
    return V @ z / math.sqrt(p), p, float(np.sum(np.abs(beta) ** 2 * h))


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_small_dense_basis_against_oracle(dt):
    import torch
    rng = np.random.default_rng(501)
    n_s, n_c = 5, 7
    N = 1 << n_s
    V = _orthogonal(rng, N)
    lam = rng.uniform(1.0, 80.0, N)
    A = (V * lam) @ V.T
    A = 0.5 * (A + A.T)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    T0 = inputs.t0_top_of_clock(lam.max(), n_c) * 0.9
    psi_r, x_r, pp_r, pa_r = oracle.hhl(A, b, n_c, T0)
    Vd = torch.tensor(V, dtype=torch.float64, device="cuda")
    st = B.State(n_s + n_c + 1, dt)
    plan = B.sv_hhl_prepare_eig(st.h, Vd, lam)
    try:
        lo, hi = B.sv_hhl_plan_spectrum(plan)
        assert lo == lam.min() and hi == lam.max()
        for mode in (0, 1, 2):
            x, res = B.sv_hhl_run(plan, st.h, b, n_c, T0, mode)
            tol = 1e-12 if dt == "c128" else max(1e-5, 2e-6 / math.sqrt(pp_r))
            assert np.abs(x - x_r).max() <= tol, (mode, np.abs(x - x_r).max())
            assert abs(res.p_post - pp_r) <= (1e-12 if dt == "c128" else 1e-5)
            assert abs(res.p_anc - pa_r) <= (1e-12 if dt == "c128" else 1e-5)
            if mode == 0:
                assert np.abs(st.get() - psi_r).max() <= (1e-12 if dt == "c128" else 1e-5)
            else:
                assert np.linalg.norm(x - x_r) <= REL[dt]
    finally:
        B.sv_hhl_plan_free(plan)
        st.close()


def test_dense_basis_n12_against_closed_form():
    import torch
    rng = np.random.default_rng(502)
    n_s, n_c = 12, 9
    N = 1 << n_s
    V = _orthogonal(rng, N)
    lam = np.exp(rng.uniform(0.0, math.log(500.0), N))
    b = rng.standard_normal(N)
    T0 = inputs.t0_top_of_clock(lam.max(), n_c) * 0.8
    x_r, pp_r, pa_r = _closed_form(V, lam, b, n_c, T0)
    Vd = torch.tensor(V, dtype=torch.float64, device="cuda")
    for dt in ("c64", "c128"):
        st = B.State(n_s + n_c + 1, dt)
        plan = B.sv_hhl_prepare_eig(st.h, Vd, lam)
        try:
            for mode in (1, 2):
                x, res = B.sv_hhl_run(plan, st.h, b, n_c, T0, mode)
                rel = np.linalg.norm(x - x_r)
                assert rel <= REL[dt], (dt, mode, rel)
                assert abs(res.p_post - pp_r) <= 2 * REL[dt] * pp_r
                assert abs(res.p_anc - pa_r) <= 2 * REL[dt] * pa_r
        finally:
            B.sv_hhl_plan_free(plan)
            st.close()


def test_dense_basis_rejects_non_orthogonal_and_mode0_beyond_13():
    import torch
    rng = np.random.default_rng(503)
    N = 16
    V = _orthogonal(rng, N)
    V[3, 5] += 1e-3
    st = B.State(4 + 4 + 1, "c128")
    with pytest.raises(B.SvError) as e:
        B.sv_hhl_prepare_eig(st.h, torch.tensor(V, dtype=torch.float64, device="cuda"), np.ones(N))
    assert e.value.status == B.SV_EINVAL
    st.close()


@pytest.fixture(scope="module")
def dense32():
    """The 32-qubit dense-basis workload and its closed form."""
    m_hi = m_lo = 8
    n_c = 15
    ks = inputs.kron_laplacian_system(inputs.rng_for(3, 0), m_hi, m_lo, kappa=1000.0)
    T0 = inputs.t0_top_of_clock(ks.lambda_max, n_c)
    mu, P = np.linalg.eigh(ks.A_hi)
    nu, Q = np.linalg.eigh(ks.A_lo)
    lam = (mu[:, None] + nu[None, :]).ravel()
    w = inputs.rng_for(3, 3).standard_normal(1 << 16)
    bh = ks.b / np.linalg.norm(ks.b)
    c = bh - 2.0 * w * (w @ bh) / (w @ w)
    beta = (P.T @ c.reshape(256, 256) @ Q).ravel()
    g, h = g_h_of_phi_wide(lam * T0 / (2 * math.pi), n_c)
    z = beta * g
    p_post = float(np.sum(z ** 2))
    p_anc = float(np.sum(beta ** 2 * h))
    y = (P @ z.reshape(256, 256) @ Q.T).ravel()
    x = (y - 2.0 * w * (w @ y) / (w @ w)) / math.sqrt(p_post)
    return dict(ks=ks, n_c=n_c, T0=T0, P=P, Q=Q, lam=lam, w=w, x=x, p_post=p_post, p_anc=p_anc)


def _dense_V(case):
    """V = (I - 2 w w^T / |w|^2)(P (x) Q) on the device, FP64, 32 GiB."""
    import torch
    P = torch.tensor(case["P"], dtype=torch.float64, device="cuda")
    Q = torch.tensor(case["Q"], dtype=torch.float64, device="cuda")
    w = torch.tensor(case["w"], dtype=torch.float64, device="cuda")
    V = torch.kron(P, Q)
    u = torch.mv(V.t(), w)
    V.addr_(w, u, alpha=-2.0 / float(torch.dot(w, w)))
    return V


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_dense_basis_32_qubits(dense32, dt):
    import torch
    c = dense32
    n = 16 + c["n_c"] + 1
    need = (1 << 32) * 8 + (1 << n) * (8 if dt == "c64" else 16)
    if torch.cuda.mem_get_info()[0] < need * 1.1:
        pytest.skip("not enough device memory")
    V = _dense_V(c)
    st = B.State(n, dt)
    plan = B.sv_hhl_prepare_eig(st.h, V, c["lam"])
    try:
        x, res = B.sv_hhl_run(plan, st.h, c["ks"].b, c["n_c"], c["T0"], 1)
    finally:
        B.sv_hhl_plan_free(plan)
        st.close()
        del V
        torch.cuda.empty_cache()
    rel = np.linalg.norm(x - c["x"])
    print(f"dense 32q {dt}: rel-l2 {rel:.3e} p_post {res.p_post:.9e} ({c['p_post']:.9e})", flush=True)
    assert rel <= REL[dt]
    assert np.abs(x - c["x"]).max() <= (1e-5 if dt == "c64" else 1e-12)
    assert abs(res.p_post - c["p_post"]) <= REL[dt] * c["p_post"]
    assert abs(res.p_anc - c["p_anc"]) <= REL[dt] * c["p_anc"]
