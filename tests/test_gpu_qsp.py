"""GPU parity of QSP-1 (binary-tree state preparation) against the oracle's
gate-by-gate circuit: both library modes (the circuit pass by pass, and the
one-pass product form), complex64 to 1e-5 and complex128 to 1e-12 in
amplitude, the paper's worked example, a 22-qubit register against the
closed form b / |b|, and the error paths."""
import os

import numpy as np
import pytest

import oracle
from paper_2307_00391_amd import binding as B

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 1e-5}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _b(rng, m, kind, zeros=0.25):
    b = rng.standard_normal(1 << m)
    if kind == "complex":
        b = b + 1j * rng.standard_normal(1 << m)
    b[rng.random(1 << m) < zeros] = 0.0
    if not np.any(b):
        b[-1] = 1.0
    return b


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n,q_lo,m,kind", [(1, 0, 1, "real"), (3, 1, 2, "complex"), (6, 0, 6, "real"),
                                           (9, 2, 5, "complex"), (11, 0, 10, "complex"), (12, 3, 9, "real")])
def test_qsp_matches_oracle(dt, mode, n, q_lo, m, kind):
    rng = np.random.default_rng(100 * n + 10 * m + q_lo)
    b = _b(rng, m, kind)
    ref = oracle.qsp(n, q_lo, b)
    st = B.State(n, dt)
    B.sv_qsp_prepare(st.h, b, q_lo, mode)
    got = st.get()
    st.close()
    assert np.abs(got - ref).max() <= TOL[dt]


@pytest.mark.parametrize("mode", [0, 1])
def test_worked_example(mode):
    rows = [[float(x) for x in ln.split()] for ln in open(os.path.join(GOLDEN, "qsp1_worked_example.txt"))
            if ln.strip() and not ln.startswith("#")]
    target = np.array(rows[0])
    st = B.State(2, "c128")
    B.sv_qsp_prepare(st.h, np.sqrt(target), 0, mode)
    got = st.get()
    st.close()
    assert np.allclose(np.abs(got) ** 2, target, atol=1e-14)


@pytest.mark.parametrize("mode", [0, 1])
def test_large_register_closed_form(mode):
    n, q_lo, m = 24, 1, 22
    rng = np.random.default_rng(7)
    b = _b(rng, m, "complex", zeros=0.05)
    st = B.State(n, "c64")
    B.sv_qsp_prepare(st.h, b, q_lo, mode)
    got = st.get()
    st.close()
    ref = np.zeros(1 << n, dtype=complex)
    ref[np.arange(1 << m) << q_lo] = b / np.linalg.norm(b)
    assert np.abs(got - ref).max() <= 1e-5
    assert abs(np.linalg.norm(got) - 1.0) <= 1e-5


def test_fused_is_repeatable_and_overwrites():
    rng = np.random.default_rng(3)
    b = _b(rng, 8, "complex")
    st = B.State(10, "c64")
    st.set(np.full(1 << 10, 0.5 + 0.25j))          # stale contents must not leak
    B.sv_qsp_prepare(st.h, b, 2, 1)
    a = st.get()
    B.sv_qsp_prepare(st.h, b, 2, 1)
    assert np.array_equal(st.get(), a)
    B.sv_qsp_prepare(st.h, b, 2, 0)
    assert np.abs(st.get() - a).max() <= 1e-5
    st.close()


def test_qsp_errors():
    st = B.State(4, "c64")
    with pytest.raises(B.SvError) as e:
        B.sv_qsp_prepare(st.h, np.zeros(4), 0, 1)
    assert e.value.status == B.SV_EZERONORM
    with pytest.raises(B.SvError) as e:
        B.sv_qsp_prepare(st.h, np.ones(8), 2, 1)   # register past the top qubit
    assert e.value.status == B.SV_EINVAL
    with pytest.raises(B.SvError) as e:
        B.sv_qsp_prepare(st.h, np.ones(4), 0, 2)
    assert e.value.status == B.SV_EINVAL
    with pytest.raises(B.SvError) as e:
        B.sv_qsp_prepare(st.h, np.array([1.0, np.nan]), 0, 1)
    assert e.value.status == B.SV_EINVAL
    st.close()
