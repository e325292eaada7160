"""The allocation-free post-selection (sv_postselect_noalloc) against
sv_postselect with its vector on the device: the same kernels in the same
reduction order, so the probability and every amplitude agree bit for bit.
Two calls in a row on one device, the second on a smaller state and another
outcome, check that the shared per-device workspace carries nothing over."""
import numpy as np
import pytest

from paper_2307_00391_amd import binding as B
from paper_2307_00391_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _case(torch, n, dt, mask, value, seed):
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    st = B.State(n, dt)
    g = torch.Generator(device="cuda").manual_seed(seed)
    st.tensor.copy_(torch.randn(1 << n, dtype=tdt, device="cuda", generator=g))
    st.tensor /= torch.linalg.vector_norm(st.tensor)
    k = n - bin(mask).count("1")
    ref = torch.empty(1 << k, dtype=tdt, device="cuda")
    p_ref = B.sv_postselect_device(st.h, mask, value, ref)
    got = torch.full((1 << k,), float("nan"), dtype=tdt, device="cuda")
    prob = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    B.sv_postselect_noalloc(st.h, mask, value, prob, got)
    torch.cuda.synchronize()
    p_got = float(prob.cpu()[0])
    st.close()
    return p_ref, p_got, ref.cpu().numpy(), got.cpu().numpy()


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_noalloc_matches_postselect_twice(dt):
    torch = pytest.importorskip("torch")
    # a large state (2^27 selected amplitudes: the full 4096 reduction
    # partials) and then a small one with another mask (one partial): the
    # second call reads nothing the first left in the shared workspace
    for n, mask, value, seed in ((28, 1 << 27, 1 << 27, 1), (9, 0b100000011, 0b100000001, 2)):
        p_ref, p_got, ref, got = _case(torch, n, dt, mask, value, seed)
        assert p_got == p_ref, (n, p_got, p_ref)
        assert np.array_equal(got, ref), n
        assert 0.0 < p_got < 1.0


def test_noalloc_probability_only_and_errors():
    torch = pytest.importorskip("torch")
    st = B.State(12, "c128")
    psi = inputs.random_state(np.random.default_rng(3), 12)
    st.set(psi)
    prob = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.sv_postselect_noalloc(st.h, 0b1010, 0b1000, prob, None)
    torch.cuda.synchronize()
    idx = np.arange(1 << 12)
    want = np.sum(np.abs(psi[(idx & 0b1010) == 0b1000]) ** 2)
    assert abs(float(prob.cpu()[0]) - want) <= 1e-13
    with pytest.raises(B.SvError):
        B.sv_postselect_noalloc(st.h, 0b1010, 0b0100, prob, None)      # value outside mask
    with pytest.raises(B.SvError):
        B.sv_postselect_noalloc(st.h, 1 << 12, 0, prob, None)         # mask beyond the state
    with pytest.raises(B.SvError):
        B.sv_postselect_noalloc(st.h, 1, 0, None, None)               # no probability slot
    st.close()
