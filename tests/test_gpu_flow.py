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


@pytest.mark.parametrize("scheme", ["fe", "be"])
def test_one_shot_matches_oracle(scheme):
    ch = flow.channel("poiseuille", N=4, Re=10.0, dt=0.15)
    m, p, n_c = 5, 2, 8
    got = flow.one_shot(ch, scheme, m, p, n_c, dtype="c128")
    A_os, b_os = flow.one_shot_system(ch, scheme, m, p)
    n = A_os.shape[0]
    H = np.block([[np.zeros((n, n)), A_os], [A_os.T, np.zeros((n, n))]])
    bb = np.concatenate([b_os, np.zeros(n)])
    T0 = 2 * math.pi * 0.45 / np.linalg.norm(A_os, 2)
    _, x, pp, _ = oracle.hhl(H, bb, n_c, T0, signed_clock=True)
    C = 2 * math.pi / (2 ** n_c * T0)
    ref = (np.linalg.norm(bb) * math.sqrt(pp) / C * x.real)[n:].reshape(m + p + 1, ch.N)
    assert abs(got.p_post - pp) <= 1e-12
    assert np.abs(got.u - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


def test_one_shot_converges_to_the_classical_solution():
    ch = flow.channel("poiseuille", N=4, Re=10.0, dt=0.15)
    m, p = 11, 4
    errs = {}
    for n_c in (8, 13):
        r = flow.one_shot(ch, "be", m, p, n_c, dtype="c64")
        errs[n_c] = np.abs(r.u[-1] - r.u_classical[-1]).max()
        assert r.fidelity > 0.5
    assert errs[13] < errs[8] and errs[13] < 0.1, errs
