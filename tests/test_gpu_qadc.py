"""GPU parity of the QPP nonlinear transform (squaring by SWAP test and
amplitude estimation) against the oracle's gate-by-gate circuit: both library
modes, complex128 and complex64, the whole final state, for address registers
of 1 to 6 qubits (lane groups of 2 to 64 in the fused reflections, blocks of
up to 130 KiB of LDS); the squares, P(up = 1,
ancillas 0) and the U_avg readout against the Fejer closed form; the modes
against each other at 24 qubits; error paths.

Tolerances: every iterate of the amplitude-estimation operator is rounded in
the state's precision: each of the 2 (2^r - 1) iterates is two Householder
updates (an N-term dot and an axpy) and two SWAP-test butterflies, at most
4 (N + 4) roundings of the block's norm, so the bar is 1e-12 + 8 (2^r - 1)
(N + 4) 2^-53 for complex128 and 1e-5 + 8 (2^r - 1)(N + 4) 2^-24 for
complex64."""
import math

import numpy as np
import pytest

import oracle
from paper_2307_00391_amd import binding as B
from tests.closed_form import qadc_weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _tol(dt, n, r):
    if dt == "c128":
        return 1e-12 + 8 * ((1 << r) - 1) * ((1 << n) + 4) * 2.0 ** -53
    return 1e-5 + 8 * ((1 << r) - 1) * ((1 << n) + 4) * 2.0 ** -24


def _u(n, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(1 << n)
    u[rng.integers(1 << n)] = 0.0
    return u


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n,r", [(1, 1), (1, 4), (2, 3), (2, 5), (3, 3), (4, 3), (5, 3), (6, 2)])
def test_qadc_matches_oracle(dt, mode, n, r):
    u = _u(n, 10 * n + r)
    print(f"[qadc] {dt} mode {mode} n {n} r {r}", flush=True)
    psi_ref = oracle.qadc_square(u, r, avg=True)
    st = B.State(3 * n + r + 2, dt)
    try:
        g, res = B.sv_qadc_square(st.h, u, r, mode=mode, avg=True)
        psi = st.get()
    finally:
        st.close()
    tol = _tol(dt, n, r)
    assert np.abs(psi - psi_ref).max() <= tol
    want = qadc_weights(u, r)
    N = 1 << n
    assert np.abs(g - want).max() <= math.sqrt(N) * tol
    assert abs(res.p_sq - float(np.sum(want ** 2)) / N) <= 4 * tol
    assert abs(res.avg - float(np.sum(want)) / N) <= tol


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_qadc_basis_vector_is_exact(dt):
    """An input on a basis vector puts every eigenphase on the grid: the
    final state is sum_s |s>_add |[s = j]>_up / sqrt(N) with all ancillas 0."""
    n, r, j = 2, 4, 3
    u = np.zeros(1 << n)
    u[j] = 2.5
    st = B.State(3 * n + r + 2, dt)
    try:
        g, res = B.sv_qadc_square(st.h, u, r, mode=1, avg=False)
        psi = st.get()
    finally:
        st.close()
    want = np.zeros_like(psi)
    up = 3 * n + 1 + r
    for s in range(1 << n):
        want[(s << (2 * n)) | ((1 << up) if s == j else 0)] = 0.5
    assert np.abs(psi - want).max() <= _tol(dt, n, r)
    assert np.abs(g - np.eye(1 << n)[j]).max() <= 2 * _tol(dt, n, r)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_qadc_24_qubits_modes_agree_and_closed_form(dt):
    """A 16-point gradient (the channel's grid), r = 10 (24 qubits): the two
    modes agree on the squares and both match the closed form, which is within
    2/2^r of u_s^2."""
    y = np.arange(1, 17) / 17
    u = 1 - 2 * y                       # du/dy of the profile y (1 - y)
    n, r = 4, 10
    out = []
    for mode in (1, 0) if dt == "c128" else (1,):
        st = B.State(3 * n + r + 2, dt)
        try:
            print(f"[qadc 24q] {dt} mode {mode}", flush=True)
            out.append(B.sv_qadc_square(st.h, u, r, mode=mode, avg=True))
        finally:
            st.close()
    want = qadc_weights(u, r)
    bar = math.sqrt(16) * _tol(dt, n, r)
    for g, res in out:
        assert np.abs(g - want).max() <= bar
        assert abs(res.avg - want.sum() / 16) <= bar
    z2 = (u / np.linalg.norm(u)) ** 2
    assert np.abs(want - z2).max() <= 2.0 / (1 << r)


def test_qadc_errors():
    st = B.State(3 * 2 + 3 + 2, "c64")
    try:
        with pytest.raises(B.SvError):
            B.sv_qadc_square(st.h, np.ones(4), 4)                  # 3n + r + 2 != 11
        with pytest.raises(B.SvError):
            B.sv_qadc_square(st.h, np.zeros(4), 3)
        with pytest.raises(B.SvError):
            B.sv_qadc_square(st.h, np.array([1.0, np.nan, 0, 0]), 3)
        with pytest.raises(B.SvError):
            B.sv_qadc_square(st.h, np.ones(4), 3, mode=2)
    finally:
        st.close()
    st = B.State(3 * 7 + 1 + 2, "c64")
    try:
        with pytest.raises(B.SvError):                             # mode 1 keeps n <= 6
            B.sv_qadc_square(st.h, np.ones(128), 1, mode=1)
    finally:
        st.close()


def test_qadc_unpacked_kernels_in_a_child_process():
    """SV_QADC_PACKED=0 (read once per process): the one-column-per-wavefront
    kernels for the packed shapes n = 3 and 4, against the oracle."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = r"""
import numpy as np, oracle
from paper_2307_00391_amd import binding as B
from tests.test_gpu_qadc import _u, _tol
B.lib()
for dt in ("c128", "c64"):
    for n, r in ((3, 3), (4, 3)):
        u = _u(n, 10 * n + r)
        ref = oracle.qadc_square(u, r, avg=True)
        st = B.State(3 * n + r + 2, dt)
        B.sv_qadc_square(st.h, u, r, mode=1, avg=True)
        err = np.abs(st.get() - ref).max()
        st.close()
        assert err <= _tol(dt, n, r), (dt, n, r, err)
print("unpacked ok")
"""
    env = dict(os.environ, SV_QADC_PACKED="0")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "unpacked ok" in r.stdout, r.stdout + r.stderr
