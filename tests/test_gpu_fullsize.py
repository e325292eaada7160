"""Full-size GPU checks (the sizes bench.py times), where the oracle cannot run.

* 32-qubit HHL (n_s = 16 Kronecker-sum Laplacian + perturbation, kappa = 1000,
  n_c = 15): the post-selected amplitudes are compared, on 4096 sampled
  eigen-components, with the circuit's closed form (pinned against the
  oracle in test_oracle_hhl.py); complex64 to 1e-5 and complex128 to 1e-12
  in state-amplitude units.
* 33-qubit U3 + CNOT-ladder probe: the norm is preserved and the circuit
  followed by its inverse returns |0...0>; and, through the same fused
  passes, the probe's 20 U3 layers followed by one CNOT ladder, whose output
  has a closed form (a product state permuted by the ladder), on 4096
  sampled amplitudes.
"""
import math

import numpy as np
import pytest

from paper_2307_00391_amd import binding as B
from paper_2307_00391_amd import inputs
from tests.closed_form import g_of_phi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _free_mem():
    import torch
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("dt,tol,mode,device", [("c64", 1e-5, 1, True), ("c64", 1e-5, 1, False),
                                                ("c128", 1e-12, 1, False), ("c64", 1e-5, 2, False)])
def test_hhl_32_qubits_against_closed_form(dt, tol, mode, device):
    """device: b and x in HBM (sv_hhl_run_device), as the benchmark times it."""
    m_hi = m_lo = 8
    n_c = 15
    n = m_hi + m_lo + n_c + 1
    need = (1 << n) * (8 if dt == "c64" else 16)
    if _free_mem() < need * 1.1:
        pytest.skip("not enough device memory")
    ks = inputs.kron_laplacian_system(inputs.rng_for(3, 0), m_hi, m_lo, kappa=1000.0)
    T0 = inputs.t0_top_of_clock(ks.lambda_max, n_c)
    st = B.State(n, dt)
    plan = B.sv_hhl_prepare(st.h, ks.A_hi, ks.A_lo)
    if device:
        import torch
        b_dev = torch.tensor(np.asarray(ks.b, dtype=np.complex128), device="cuda")
        x_dev = torch.empty(1 << (m_hi + m_lo), dtype=torch.complex128, device="cuda")
        res = B.sv_hhl_run_device(plan, st.h, b_dev, n_c, T0, mode, x_dev=x_dev)
        x = x_dev.cpu().numpy()
    else:
        x, res = B.sv_hhl_run(plan, st.h, ks.b, n_c, T0, mode)
    B.sv_hhl_plan_free(plan)
    st.close()
    # eigen-basis view of the GPU result: z = V^H x sqrt(p)
    mu, P = np.linalg.eigh(ks.A_hi)
    nu, Q = np.linalg.eigh(ks.A_lo)
    X = x.reshape(1 << m_hi, 1 << m_lo)
    Z_gpu = (P.conj().T @ X @ Q.conj()) * math.sqrt(res.p_post)
    Bm = (ks.b / np.linalg.norm(ks.b)).reshape(1 << m_hi, 1 << m_lo)
    beta = P.conj().T @ Bm @ Q.conj()
    lam = mu[:, None] + nu[None, :]
    rng = np.random.default_rng(32)
    idx = rng.choice(lam.size, size=4096, replace=False)
    idx = np.union1d(idx, [0, lam.size - 1, int(np.argmax(np.abs(beta).ravel()))])
    g = g_of_phi(lam.ravel()[idx] * T0 / (2 * math.pi), n_c, chunk=128)
    z_true = beta.ravel()[idx] * g
    err = np.abs(Z_gpu.ravel()[idx] - z_true).max()
    assert err <= tol, err
    assert abs(res.lambda_min - lam.min()) <= 1e-12 * lam.max()
    assert abs(res.norm_total - 1.0) <= (1e-5 if dt == "c64" else 1e-12)
    assert 0 < res.p_post <= res.p_anc <= 1.0


def test_probe_33_qubits_norm_and_roundtrip():
    q, layers = 33, 20
    if _free_mem() < (1 << q) * 8 * 1.1:
        pytest.skip("not enough device memory")
    gates = inputs.probe_layers(inputs.rng_for(3, 1000), q, layers)
    inv = []
    for g in reversed(gates):
        inv.append(("u", g[1], np.conj(g[2]).T) if g[0] == "u" else g)
    st = B.State(q, "c64")
    B.sv_init_basis(st.h, 0)
    B.sv_apply_circuit(st.h, gates)
    assert abs(B.sv_norm2(st.h) - 1.0) <= 1e-5
    B.sv_apply_circuit(st.h, inv)
    p0 = B.sv_norm2(st.h, (1 << q) - 1, 0)
    assert p0 >= 1.0 - 1e-4, p0
    st.close()


def test_probe_33_qubits_product_state_closed_form():
    """The probe's U3 gates (20 layers on all 33 qubits) and then one CNOT
    ladder q -> q+1, q = 0..31.  The U3 layers leave the product state
    (x)_q m_q with m_q = (product of qubit q's 20 gates)|0>; the ladder maps
    |x> to |y> with y_k = x_0 ^ ... ^ x_k, so the output amplitude at y is
    prod_q m_q[y_q ^ y_(q-1)] (y_(-1) = 0)."""
    torch = pytest.importorskip("torch")
    q, layers = 33, 20
    if _free_mem() < (1 << q) * 8 * 1.1:
        pytest.skip("not enough device memory")
    full = inputs.probe_layers(inputs.rng_for(3, 1000), q, layers)
    us = [g for g in full if g[0] == "u"]
    ladder = [("cx", k, k + 1) for k in range(q - 1)]
    m = [np.array([1.0, 0.0], dtype=np.complex128) for _ in range(q)]
    for _, t, u in us:
        m[t] = u @ m[t]
    st = B.State(q, "c64")
    B.sv_init_basis(st.h, 0)
    B.sv_apply_circuit(st.h, us + ladder)
    rng = np.random.default_rng(33)
    ys = np.unique(np.concatenate([rng.integers(0, 1 << q, size=4096, dtype=np.int64), [0, (1 << q) - 1]]))
    got = st.tensor[torch.as_tensor(ys, device=st.tensor.device)].cpu().numpy().astype(np.complex128)
    st.close()
    bits = (ys[:, None] >> np.arange(q)[None, :]) & 1
    xs = bits ^ np.concatenate([np.zeros((ys.size, 1), dtype=np.int64), bits[:, :-1]], axis=1)
    want = np.ones(ys.size, dtype=np.complex128)
    for k in range(q):
        want *= np.where(xs[:, k] == 1, m[k][1], m[k][0])
    scale = np.abs(want).max()
    err = np.abs(got - want).max()
    assert err <= 1e-4 * scale, (err, scale)
