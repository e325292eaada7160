"""Full-size GPU checks (the sizes bench.py times), where the oracle cannot run.

* 32-qubit HHL (n_s = 16 Kronecker-sum Laplacian + perturbation, kappa = 1000,
  n_c = 15): the whole normalised post-selected vector (2^16 entries) against
  the circuit's closed form over every eigencomponent (pinned against the
  oracle in test_oracle_hhl.py), by relative l2 (1e-5 complex64, 1e-10
  complex128) and max-abs; p_post and P(a = 1) relative to their closed
  forms; the complex64 x against the complex128 x.
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
from tests.closed_form import g_h_of_phi_wide

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


# relative-l2 bars on the whole post-selected vector and relative bars on the
# probabilities: FP32 amplitudes carry ~1e-7 relative rounding per operation
# over the ~30 dependent butterfly and rotation stages; FP64 stays near 1e-13.
REL = {"c64": 1e-5, "c128": 1e-10}


@pytest.fixture(scope="module")
def hhl32_case():
    """The 32-qubit workload and its closed form over all 2^16 eigencomponents:
    x = V (beta g) / sqrt(p), p = sum |beta g|^2, p_anc = sum |beta|^2 h."""
    m_hi = m_lo = 8
    n_c = 15
    ks = inputs.kron_laplacian_system(inputs.rng_for(3, 0), m_hi, m_lo, kappa=1000.0)
    T0 = inputs.t0_top_of_clock(ks.lambda_max, n_c)
    mu, P = np.linalg.eigh(ks.A_hi)
    nu, Q = np.linalg.eigh(ks.A_lo)
    Bm = (ks.b / np.linalg.norm(ks.b)).reshape(1 << m_hi, 1 << m_lo)
    beta = P.conj().T @ Bm @ Q.conj()
    lam = mu[:, None] + nu[None, :]
    g, h = g_h_of_phi_wide((lam * T0 / (2 * math.pi)).ravel(), n_c)
    Z = beta * g.reshape(lam.shape)
    p_post = float(np.sum(np.abs(Z) ** 2))
    p_anc = float(np.sum(np.abs(beta) ** 2 * h.reshape(lam.shape)))
    x_true = (P @ Z @ Q.T).reshape(-1) / math.sqrt(p_post)
    return dict(ks=ks, n_c=n_c, T0=T0, m_hi=m_hi, m_lo=m_lo, lam=lam, x=x_true, p_post=p_post,
                p_anc=p_anc, got={})


def _run32(case, dt, mode, device):
    ks, n_c, T0 = case["ks"], case["n_c"], case["T0"]
    n_s = case["m_hi"] + case["m_lo"]
    n = n_s + n_c + 1
    need = (1 << n) * (8 if dt == "c64" else 16)
    if _free_mem() < need * 1.1:
        pytest.skip("not enough device memory")
    st = B.State(n, dt)
    plan = B.sv_hhl_prepare(st.h, ks.A_hi, ks.A_lo)
    try:
        if device:
            import torch
            b_dev = torch.tensor(np.asarray(ks.b, dtype=np.complex128), device="cuda")
            x_dev = torch.empty(1 << n_s, dtype=torch.complex128, device="cuda")
            res = B.sv_hhl_run_device(plan, st.h, b_dev, n_c, T0, mode, x_dev=x_dev)
            x = x_dev.cpu().numpy()
        else:
            x, res = B.sv_hhl_run(plan, st.h, ks.b, n_c, T0, mode)
    finally:
        B.sv_hhl_plan_free(plan)
        st.close()
    return x, res


@pytest.mark.parametrize("dt,mode,device", [("c64", 1, True), ("c64", 1, False), ("c128", 1, False),
                                            ("c64", 2, False)])
def test_hhl_32_qubits_against_closed_form(hhl32_case, dt, mode, device):
    """device: b and x in HBM (sv_hhl_run_device), as the benchmark times it.
    The whole normalised x (2^16 entries) against the closed form: relative
    l2 and max-abs; p_post and p_anc relative to their closed forms."""
    c = hhl32_case
    x, res = _run32(c, dt, mode, device)
    c["got"][(dt, mode, device)] = x
    rel = np.linalg.norm(x - c["x"]) / np.linalg.norm(c["x"])
    amax = np.abs(x - c["x"]).max()
    print(f"32q {dt} mode {mode} device {device}: rel-l2 {rel:.3e} max-abs {amax:.3e} "
          f"p_post {res.p_post:.9e} (closed form {c['p_post']:.9e}) p_anc {res.p_anc:.9e} ({c['p_anc']:.9e})",
          flush=True)
    assert rel <= REL[dt], rel
    assert amax <= (1e-5 if dt == "c64" else 1e-12), amax
    assert abs(res.p_post - c["p_post"]) <= REL[dt] * c["p_post"], (res.p_post, c["p_post"])
    assert abs(res.p_anc - c["p_anc"]) <= REL[dt] * c["p_anc"], (res.p_anc, c["p_anc"])
    assert abs(res.lambda_min - c["lam"].min()) <= 1e-12 * c["lam"].max()
    assert abs(res.norm_total - 1.0) <= (1e-5 if dt == "c64" else 1e-12)


def test_hhl_32_qubits_c64_against_c128(hhl32_case):
    """The mixed-precision claim at full size: the complex64 solve's x within
    the FP32 bars of the complex128 solve's x (both from the same plan kind,
    b and x on the host)."""
    c = hhl32_case
    x64 = c["got"].get(("c64", 1, False))
    if x64 is None:
        x64, _ = _run32(c, "c64", 1, False)
    x128 = c["got"].get(("c128", 1, False))
    if x128 is None:
        x128, _ = _run32(c, "c128", 1, False)
    rel = np.linalg.norm(x64 - x128) / np.linalg.norm(x128)
    print(f"32q c64 vs c128: rel-l2 {rel:.3e} max-abs {np.abs(x64 - x128).max():.3e}", flush=True)
    assert rel <= REL["c64"]
    assert np.abs(x64 - x128).max() <= 1e-5


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
