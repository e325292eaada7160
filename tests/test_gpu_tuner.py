"""The autotuner's candidates give the same results.

Every configuration the tuner can pick is pinned through sv_tune_set (or the
explicit max_local / SV_FUSED_LOWBITS of the fused passes) and run:
* the eigen-frame kernels: every (log2 columns per tile, threads) of each of
  the three kernels, for single solves and for a batch,
  against the oracle at the usual bars;
* the matrix-core GEMM: both tile shapes, bit for bit against each other
  (same k order) and against the oracle;
* the fused gate passes: every (k local qubits, c contiguous low bits), bit
  for bit on a permutation circuit and against the oracle on a general one;
  the tuner's own pick (max_local = 0) too;
* SV_AUTOTUNE=0 (the default configurations) in a child process.
"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2307_00391_amd import binding as B
from paper_2307_00391_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _default_cl(n_s, g, dt):
    return max(0, min(6, n_s, (13 if dt == "c64" else 12) - g))


def _pipe_candidates(n_s, n_c, dt):
    g1 = (n_c + 1) // 2
    g2 = n_c - g1
    base = []
    for w in range(3):
        base += [_default_cl(n_s, g2 if w == 1 else g1, dt), 256]
    out = []
    for w in range(3):
        for cl in range(3, 8):
            if cl > n_s:
                break
            for nt in (256, 512):
                v = list(base)
                v[2 * w], v[2 * w + 1] = cl, nt
                out.append(v)
    return out


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n_s,n_c", [(6, 9), (5, 12), (8, 7)])
def test_pipeline_candidates_single_solves(dt, n_s, n_c):
    rng = np.random.default_rng(700 + 16 * n_s + n_c)
    A, _, lmax = inputs.random_spd_tridiag(rng, 1 << n_s, 150.0)
    b = rng.standard_normal(1 << n_s)
    T0 = inputs.t0_top_of_clock(lmax, n_c) * 0.87
    _, x_r, pp_r, pa_r = oracle.hhl(A, b, n_c, T0)
    key = f"eigpipe/{dt}/{n_s}/{n_c}"
    tol = TOL[dt] if dt == "c128" else max(1e-5, 2e-6 / math.sqrt(pp_r))
    ran = 0
    try:
        for v in _pipe_candidates(n_s, n_c, dt):
            B.sv_tune_set(key, v)
            st = B.State(n_s + n_c + 1, dt)
            try:
                x, res = B.sv_hhl(st.h, A, b, n_c, T0, 1)
            except B.SvError as e:                     # a tile that does not fit the LDS
                assert e.status == B.SV_EUNSUPPORTED and "LDS" in str(e), (v, str(e))
                continue
            finally:
                st.close()
            ran += 1
            assert np.abs(x - x_r).max() <= tol, (v, np.abs(x - x_r).max())
            assert abs(res.p_post - pp_r) <= TOL[dt], v
            assert abs(res.p_anc - pa_r) <= TOL[dt], v
    finally:
        B.sv_tune_set(key, [])
    assert ran >= 12


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_pipeline_candidates_batch(dt):
    n_s, n_c = 5, 8
    rng = np.random.default_rng(731)
    A, _, lmax = inputs.random_spd_tridiag(rng, 1 << n_s, 60.0)
    b = rng.standard_normal(1 << n_s)
    t0s = inputs.t0_grid(lmax)[::5]
    ref = [oracle.hhl(A, b, n_c, T0) for T0 in t0s]
    key = f"eigpipe/{dt}/{n_s}/{n_c}"
    try:
        for v in _pipe_candidates(n_s, n_c, dt)[::2]:
            B.sv_tune_set(key, v)
            try:
                res = B.sv_hhl_batch([(A, b, n_c, t0s)], dt)
            except B.SvError as e:
                assert e.status == B.SV_EUNSUPPORTED and "LDS" in str(e), (v, str(e))
                continue
            for k, (_, _, pp, pa) in enumerate(ref):
                assert abs(res[k, 0] - pp) <= TOL[dt] and abs(res[k, 1] - pa) <= TOL[dt], (v, k)
    finally:
        B.sv_tune_set(key, [])


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,m,ctrl,adj", [(14, 8, 13, 0), (14, 8, 9, 1), (12, 4, -1, 0), (17, 6, 16, 1)])
def test_gemm_tile_shapes_bitwise(dt, n, m, ctrl, adj):
    import torch
    rng = np.random.default_rng(800 + n + m + adj)
    U = inputs.random_unitary(rng, 1 << m)
    psi0 = inputs.random_state(rng, n)
    if dt == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    Ur = U.astype(np.complex64).astype(np.complex128) if dt == "c64" else U
    ref = oracle.apply_ctrl_unitary(psi0.copy(), Ur, 0, m, ctrl, 1, bool(adj))
    dU = torch.tensor(U, dtype=torch.complex64 if dt == "c64" else torch.complex128, device="cuda")
    rows = 1 << (n - m - (1 if ctrl >= 0 else 0))
    key = f"cgemm/{dt}/{rows}/{1 << m}/{1 << m}/{adj}"
    outs = []
    try:
        for shape in (0, 1):
            B.sv_tune_set(key, [shape])
            s = B.State(n, dt)
            s.set(psi0)
            B.sv_apply_ctrl_unitary(s.h, dU, 0, m, ctrl, 1, bool(adj))
            outs.append(s.get())
            s.close()
    finally:
        B.sv_tune_set(key, [])
    assert np.array_equal(outs[0], outs[1])
    assert np.abs(outs[0] - ref).max() <= TOL[dt]


def _oracle_apply(psi, g):
    if g[0] == "u":
        oracle.apply_gate(psi, g[1], g[2], *(g[3:5] if len(g) > 3 else ((), None)))
    elif g[0] == "x":
        oracle.apply_gate(psi, g[1], X, *(g[2:4] if len(g) > 2 else ((), None)))
    else:
        oracle.apply_swap(psi, g[1], g[2], *(g[3:5] if len(g) > 3 else ((), None)))


def _fusion_candidates(dt):
    K = 13 if dt == "c64" else 12
    C = 5 if dt == "c64" else 4
    RB = 5 if dt == "c64" else 4
    return [(k, c, rb) for rb in (RB, RB - 1) for k in (K - 1, K) for c in (C - 1, C, C + 1) if c <= k - 2]


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_fusion_candidates(dt, monkeypatch):
    n = 22
    rng = np.random.default_rng(900)
    psi0 = inputs.random_state(rng, n)
    if dt == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    gates = inputs.random_circuit(rng, n, 48, max_ctrls=2)
    perm = [g for g in inputs.random_circuit(np.random.default_rng(901), n, 60, max_ctrls=2) if g[0] != "u"]
    ref = psi0.copy()
    for g in gates:
        _oracle_apply(ref, g)
    ref_p = psi0.copy()
    for g in perm:
        _oracle_apply(ref_p, g)
    outs_p = []
    for k, c, rb in _fusion_candidates(dt):
        monkeypatch.setenv("SV_FUSED_LOWBITS", str(c))
        monkeypatch.setenv("SV_FUSED_RB", str(rb))
        s = B.State(n, dt)
        s.set(psi0)
        B.sv_apply_circuit(s.h, gates, k)
        assert np.abs(s.get() - ref).max() <= TOL[dt], (k, c, rb)
        s.set(psi0)
        B.sv_apply_circuit(s.h, perm, k)
        outs_p.append(s.get())
        s.close()
    for o in outs_p:
        assert np.array_equal(o, ref_p)
    # the tuner's own choice
    monkeypatch.delenv("SV_FUSED_LOWBITS")
    monkeypatch.delenv("SV_FUSED_RB")
    s = B.State(n, dt)
    s.set(psi0)
    B.sv_apply_circuit(s.h, gates, 0)
    assert np.abs(s.get() - ref).max() <= TOL[dt]
    s.close()
    assert any(ln.startswith(f"fused/{dt}/{n}/") for ln in B.sv_tune_report().splitlines())


def test_defaults_without_tuning_in_a_child_process():
    """SV_AUTOTUNE=0: the default configurations of every tuned knob."""
    code = r'''
import numpy as np, oracle, math
from paper_2307_00391_amd import binding as B, inputs
B.lib()
rng = np.random.default_rng(950)
A, _, lmax = inputs.random_spd_tridiag(rng, 64, 80.0)
b = rng.standard_normal(64)
T0 = inputs.t0_top_of_clock(lmax, 10) * 0.9
_, x_r, pp_r, _ = oracle.hhl(A, b, 10, T0)
for dt, tol in (("c128", 1e-12), ("c64", 1e-5)):
    st = B.State(6 + 10 + 1, dt)
    x, res = B.sv_hhl(st.h, A, b, 10, T0, 1)
    assert np.abs(x - x_r).max() <= max(tol, (2e-6 / math.sqrt(pp_r)) if dt == "c64" else tol), dt
    x0, res0 = B.sv_hhl(st.h, A, b, 10, T0, 0)
    assert np.abs(x0 - x_r).max() <= max(tol, (2e-6 / math.sqrt(pp_r)) if dt == "c64" else tol), dt
    st.close()
assert B.sv_tune_report().strip() == "", B.sv_tune_report()
print("defaults ok")
'''
    env = dict(os.environ, SV_AUTOTUNE="0")
    env.pop("SV_TUNE_CACHE", None)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "defaults ok" in r.stdout, r.stdout + r.stderr
