"""GPU parity: gates, permutations, fused passes, QFT, uniform Ry, reductions.

Every case runs the HIP library through the C ABI and compares with the FP64
oracle on the same seeded input: max-abs <= 1e-12 for complex128, <= 1e-5 for
complex64; permutations are compared bit for bit.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2307_00391_amd import binding as B
from paper_2307_00391_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _state(n, dt, psi=None):
    s = B.State(n, dt)
    if psi is not None:
        s.set(psi)
    return s


def _oracle_apply(psi, g):
    if g[0] == "u":
        oracle.apply_gate(psi, g[1], g[2], *(g[3:5] if len(g) > 3 else ((), None)))
    elif g[0] == "x":
        oracle.apply_gate(psi, g[1], X, *(g[2:4] if len(g) > 2 else ((), None)))
    elif g[0] == "cx":
        oracle.apply_gate(psi, g[2], X, [g[1]], [1])
    else:
        oracle.apply_swap(psi, g[1], g[2], *(g[3:5] if len(g) > 3 else ((), None)))


def _rounded(psi, dt):
    return psi.astype(np.complex64).astype(np.complex128) if dt == "c64" else psi


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 9, 16])
def test_single_gates_match_oracle(dt, n):
    rng = np.random.default_rng(1000 + n)
    psi0 = _rounded(inputs.random_state(rng, n), dt)
    s = _state(n, dt, psi0)
    ref = psi0.copy()
    for g in inputs.random_circuit(rng, n, 40, max_ctrls=min(3, n - 2)):
        _oracle_apply(ref, g)
        if g[0] == "u":
            B.sv_apply_gate(s.h, g[1], g[2], g[3], g[4])
        elif g[0] == "x":
            B.sv_apply_gate(s.h, g[1], X, g[2], g[3])
        else:
            B.sv_apply_swap(s.h, g[1], g[2], g[3], g[4])
    out = s.get()
    assert np.abs(out - ref).max() <= TOL[dt]


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_permutations_bit_exact(dt):
    n = 14
    rng = np.random.default_rng(7)
    psi0 = _rounded(rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n), dt)
    s = _state(n, dt, psi0)
    ref = psi0.copy()
    gates = [("x", 0), ("x", 13), ("cx", 2, 9), ("x", 5, [1, 12], [1, 0]), ("swap", 0, 13), ("swap", 4, 5),
             ("swap", 3, 11, [7], [0])]
    for g in gates:
        _oracle_apply(ref, g)
        if g[0] == "swap":
            B.sv_apply_swap(s.h, *g[1:])
        elif g[0] == "cx":
            B.sv_apply_gate(s.h, g[2], X, [g[1]], [1])
        else:
            B.sv_apply_gate(s.h, g[1], X, *g[2:])
    assert np.array_equal(s.get(), ref)
    # the same permutations through the fused path
    s2 = _state(n, dt, psi0)
    B.sv_apply_circuit(s2.h, gates, 10)
    assert np.array_equal(s2.get(), ref)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,kmax", [(5, 0), (10, 8), (15, 9), (18, 12), (18, 0)])
def test_fused_circuit_matches_oracle(dt, n, kmax):
    rng = np.random.default_rng(2000 + n + kmax)
    psi0 = _rounded(inputs.random_state(rng, n), dt)
    gates = inputs.random_circuit(rng, n, 60, max_ctrls=min(3, n - 2))
    # add a few diagonal (phase) gates, which the planner fuses without locality
    for q in range(0, n, 3):
        gates.append(("u", q, np.diag([1.0, np.exp(0.37j * (q + 1))]), [(q + 1) % n], [1]))
        gates.append(("u", (q + 2) % n, np.diag([np.exp(-0.2j), np.exp(0.9j)])))
    ref = psi0.copy()
    for g in gates:
        _oracle_apply(ref, g)
    s = _state(n, dt, psi0)
    B.sv_apply_circuit(s.h, gates, kmax)
    assert np.abs(s.get() - ref).max() <= TOL[dt]
    assert B.sv_plan_passes(n, B.SV_C64 if dt == "c64" else B.SV_C128, gates, kmax) >= 1


_PERSIST_CHILD = r"""
import sys, numpy as np
from paper_2307_00391_amd import binding as B, inputs
n, kmax, dt, seed, out = int(sys.argv[1]), int(sys.argv[2]), sys.argv[3], int(sys.argv[4]), sys.argv[5]
rng = np.random.default_rng(seed)
psi0 = inputs.random_state(rng, n)
if dt == "c64":
    psi0 = psi0.astype(np.complex64).astype(np.complex128)
gates = inputs.random_circuit(rng, n, 40, max_ctrls=2)
s = B.State(n, dt)
s.set(psi0)
B.sv_apply_circuit(s.h, gates, kmax)
np.save(out, s.get())
print("child ok")
"""


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_fused_persistent_tiles_match_one_tile_per_block(dt, tmp_path):
    """A pass walks strided runs of tiles with as many workgroups as the
    device holds (here 2^20 amplitudes in 2^12 tiles of 2^8: several tiles
    per workgroup); SV_FUSED_PERSIST=0 launches one workgroup per tile.  Both
    equal the oracle, and each other bit for bit."""
    import os
    import subprocess
    import sys
    n, kmax, seed = 20, 8, 4242
    rng = np.random.default_rng(seed)
    psi0 = _rounded(inputs.random_state(rng, n), dt)
    gates = inputs.random_circuit(rng, n, 40, max_ctrls=2)
    ref = psi0.copy()
    for g in gates:
        _oracle_apply(ref, g)
    s = _state(n, dt, psi0)
    B.sv_apply_circuit(s.h, gates, kmax)
    got = s.get()
    s.close()
    assert np.abs(got - ref).max() <= TOL[dt]
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = str(tmp_path / "one_tile_per_block.npy")
    env = dict(os.environ, SV_FUSED_PERSIST="0")
    r = subprocess.run([sys.executable, "-c", _PERSIST_CHILD, str(n), str(kmax), dt, str(seed), out], cwd=root,
                       env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "child ok" in r.stdout, r.stdout + r.stderr
    assert np.array_equal(np.load(out), got)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,lo,m,kmax", [(6, 0, 6, 0), (12, 3, 7, 8), (16, 4, 10, 9), (17, 6, 11, 0),
                                         (14, 2, 12, 11)])
def test_qft_matches_oracle(dt, n, lo, m, kmax):
    rng = np.random.default_rng(3000 + n + m)
    psi0 = _rounded(inputs.random_state(rng, n), dt)
    for inverse in (False, True):
        ref = oracle.qft(psi0.copy(), lo, m, inverse)
        s = _state(n, dt, psi0)
        B.sv_qft(s.h, lo, m, inverse, True, kmax)
        assert np.abs(s.get() - ref).max() <= TOL[dt]
    # swaps = 0: cascade output is the bit-reversed DFT
    s = _state(n, dt, psi0)
    B.sv_qft(s.h, lo, m, False, False, kmax)
    ref = oracle.qft(psi0.copy(), lo, m, False)
    for a in range(m // 2):
        oracle.apply_swap(ref, lo + a, lo + m - 1 - a)
    assert np.abs(s.get() - ref).max() <= TOL[dt]


def test_qft_basis_states_closed_form():
    n, lo, m = 10, 2, 6
    M = 1 << m
    for j in (0, 1, 5, 37, 63):
        s = _state(n, "c128")
        B.sv_init_basis(s.h, (j << lo) | 0b10)
        B.sv_qft(s.h, lo, m, False, True, 0)
        out = s.get()
        k = np.arange(M)
        ref = np.zeros(1 << n, dtype=np.complex128)
        ref[(k << lo) | 0b10] = np.exp(2j * np.pi * j * k / M) / math.sqrt(M)
        assert np.abs(out - ref).max() <= 1e-13


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_uniform_ry_matches_oracle(dt):
    n, reg_lo, m, target = 12, 3, 5, 11
    rng = np.random.default_rng(44)
    psi0 = _rounded(inputs.random_state(rng, n), dt)
    y = np.arange(1 << m)
    s_ = np.where(y > 0, 1.0 / np.maximum(y, 1), 0.0)
    c_ = np.sqrt(1 - s_ ** 2)
    cs = np.stack([c_, s_], axis=1)
    ref = psi0.copy()
    for v in range(1, 1 << m):
        Ry = np.array([[c_[v], -s_[v]], [s_[v], c_[v]]])
        ctrls = [reg_lo + b for b in range(m)]
        vals = [(v >> b) & 1 for b in range(m)]
        oracle.apply_gate(ref, target, Ry, ctrls, vals)
    st = _state(n, dt, psi0)
    B.sv_apply_uniform_ry(st.h, target, reg_lo, m, cs)
    assert np.abs(st.get() - ref).max() <= TOL[dt]


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_norm_postselect_and_init(dt):
    n, n_s, c = 13, 5, 4
    rng = np.random.default_rng(5)
    b = rng.standard_normal(1 << n_s) + 1j * rng.standard_normal(1 << n_s)
    s = _state(n, dt)
    B.sv_init_b(s.h, b, n_s, c)
    out = s.get()
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[: 1 << (n_s + c)] = np.tile(b / np.linalg.norm(b), 1 << c) / math.sqrt(1 << c)
    assert np.abs(out - ref).max() <= TOL[dt]
    psi = _rounded(inputs.random_state(rng, n), dt)
    s.set(psi)
    for mask, val in ((0, 0), (1 << 12, 1 << 12), (0b1011 << 5, 0b1001 << 5)):
        p_ref = oracle.norm2(psi, mask, val)
        assert abs(B.sv_norm2(s.h, mask, val) - p_ref) <= 1e-13
        p, vec = B.sv_postselect(s.h, n, mask, val)
        p2, vref = oracle.postselect(psi, mask, val)
        assert abs(p - p2) <= 1e-13
        assert np.abs(vec - vref).max() <= (1e-13 if dt == "c128" else 1e-6)


def test_reductions_repeat_bit_for_bit():
    n = 22
    rng = np.random.default_rng(9)
    s = _state(n, "c64", inputs.random_state(rng, n))
    a = [B.sv_norm2(s.h, 1 << 21, 0) for _ in range(3)]
    assert a[0] == a[1] == a[2]
    gates = inputs.random_circuit(rng, n, 30)
    psi = s.get()
    B.sv_apply_circuit(s.h, gates)
    r1 = s.get()
    s.set(psi)
    B.sv_apply_circuit(s.h, gates)
    assert np.array_equal(r1, s.get())


def test_invalid_arguments():
    s = _state(6, "c64")
    with pytest.raises(B.SvError) as e:
        B.sv_apply_gate(s.h, 6, H)
    assert e.value.status == B.SV_EINVAL
    with pytest.raises(B.SvError):
        B.sv_apply_gate(s.h, 2, H, [2])
    with pytest.raises(B.SvError):
        B.sv_apply_swap(s.h, 1, 1)
    with pytest.raises(B.SvError):
        B.sv_qft(s.h, 3, 4)
    with pytest.raises(B.SvError) as e:
        B.sv_init_b(s.h, np.zeros(4), 2, 0)
    assert e.value.status == B.SV_EZERONORM
    with pytest.raises(B.SvError) as e:
        B.sv_postselect(s.h, 6, 0b11, 0b100)
    assert e.value.status == B.SV_EINVAL
