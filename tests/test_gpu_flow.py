"""Iterative backward Euler with one HHL solve per step on the GPU against
the same march driven by the FP64 oracle's gate-level HHL, and the
converged profiles against the exact steady state."""
import math

import numpy as np
import pytest

import oracle
from paper_2307_00391_amd import binding as B
from paper_2307_00391_amd import flow

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


def _oracle_march(ch, n_c, steps):
    lmax = np.linalg.eigvalsh(ch.A_be1).max()
    T0 = 2 * math.pi * (1 - 2.0 ** -n_c) / lmax
    C = 2 * math.pi / (2 ** n_c * T0)
    u = ch.u0.copy()
    out = [u]
    for _ in range(steps):
        b = u + ch.src
        _, x, p, _ = oracle.hhl(ch.A_be1, b, n_c, T0)
        u = np.linalg.norm(b) * math.sqrt(p) / C * x.real
        out.append(u)
    return np.array(out)


@pytest.mark.parametrize("kind,dt,tol", [("poiseuille", "c128", 1e-10), ("couette", "c128", 1e-10),
                                         ("poiseuille", "c64", 2e-5)])
def test_march_matches_oracle(kind, dt, tol):
    ch = flow.channel(kind, N=8, Re=10.0, dt=0.2)
    n_c = 7
    ref = _oracle_march(ch, n_c, 6)
    run = flow.iterative_be(ch, n_c, max_steps=6, tol=0.0, dtype=dt)
    assert run.u.shape == ref.shape
    assert np.abs(run.u - ref).max() <= tol * max(1.0, np.abs(ref).max())


def test_converged_profile_improves_with_clock_qubits():
    ch = flow.channel("poiseuille", N=16, Re=10.0, dt=0.5)
    steady = -0.5 * ch.Re * ch.dpdx * ch.y * (1 - ch.y)
    errs = {}
    for n_c in (6, 12):
        run = flow.iterative_be(ch, n_c, max_steps=400, tol=1e-6, dtype="c64")
        assert run.converged_at > 0
        errs[n_c] = flow.rms(run.u[-1], steady)
    assert errs[12] < errs[6] and errs[12] < 0.05, errs
