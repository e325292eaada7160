"""Classical parts of the iterative backward-Euler driver (no GPU): the
discrete steady states against the exact steady profiles (central
differences are exact for the Poiseuille parabola and the Couette line),
the analytical series at t = 0 against the initial conditions and at large
t against the steady profiles, and classical BE against the series."""
import numpy as np
import pytest

from paper_2307_00391_amd import flow


@pytest.mark.parametrize("kind", ["poiseuille", "couette"])
def test_classical_be_reaches_the_exact_steady_profile(kind):
    ch = flow.channel(kind, N=16, Re=10.0, dt=0.5)
    u = flow.classical_be(ch, 600)[-1]
    steady = -0.5 * ch.Re * ch.dpdx * ch.y * (1 - ch.y) if kind == "poiseuille" else ch.y
    assert np.abs(u - steady).max() <= 1e-10


@pytest.mark.parametrize("kind", ["poiseuille", "couette"])
def test_series_initial_and_final(kind):
    ch = flow.channel(kind, N=16, Re=10.0)
    u_init = flow.analytic(ch, 0.0, kmax=20001)
    assert np.abs(u_init - ch.u0).max() <= 2e-3            # slowly converging sine series
    steady = -0.5 * ch.Re * ch.dpdx * ch.y * (1 - ch.y) if kind == "poiseuille" else ch.y
    assert np.abs(flow.analytic(ch, 200.0) - steady).max() <= 1e-12


@pytest.mark.parametrize("kind", ["poiseuille", "couette"])
def test_classical_be_follows_the_series(kind):
    ch = flow.channel(kind, N=16, Re=10.0, dt=0.01)
    u = flow.classical_be(ch, 100)                          # t = 1
    err = np.abs(u[-1] - flow.analytic(ch, 1.0)).max()
    assert err <= 0.01, err                                  # O(dt + h^2)


def test_channel_matrix_is_spd_and_scaled():
    ch = flow.channel("poiseuille", N=8, Re=4.0, dt=0.2)
    ev = np.linalg.eigvalsh(ch.A_be1)
    h = 1 / 9
    assert ev.min() > 1.0 and abs(ev.max() - (1 + 0.2 / 4.0 * 4 / h ** 2 * np.sin(8 * np.pi * h / 2) ** 2)) < 1e-9
    with pytest.raises(ValueError):
        flow.channel("poiseuille", N=12)


@pytest.mark.parametrize("scheme", ["fe", "be"])
@pytest.mark.parametrize("kind", ["poiseuille", "couette"])
def test_one_shot_system_equals_marching(scheme, kind):
    ch = flow.channel(kind, N=4, Re=10.0, dt=0.15)
    m, p = 11, 4
    A, b = flow.one_shot_system(ch, scheme, m, p)
    u = np.linalg.solve(A, b).reshape(m + p + 1, 4)
    march = [ch.u0]
    I = np.eye(4)
    Adt = I - ch.A_be1
    for _ in range(m):
        prev = march[-1]
        march.append((I + Adt) @ prev + ch.src if scheme == "fe" else np.linalg.solve(ch.A_be1, prev + ch.src))
    march += [march[-1]] * p
    assert np.abs(u - np.array(march)).max() <= 1e-12
