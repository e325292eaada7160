"""Classical side of the QPP dissipation workflow: the zero-wall central
difference, the grid dissipation of the steady Poiseuille profile, and the
continuous value Re dp/dx^2 / 12 (the comparison curves of the main text's
dissipation-versus-Re figure)."""
import numpy as np
import pytest
from scipy.integrate import quad

from paper_2307_00391_amd import flow, qpp


@pytest.mark.parametrize("N", [4, 8, 32])
def test_central_difference_exact_on_quadratic(N):
    h = 1.0 / (N + 1)
    y = h * np.arange(1, N + 1)
    D = qpp.central_difference(N, h)
    np.testing.assert_allclose(D @ (y * (1 - y)), 1 - 2 * y, rtol=0, atol=1e-12)


@pytest.mark.parametrize("Re", [1.0, 10.0, 1000.0])
def test_steady_dissipation_closed_form(Re):
    """nu * int_0^1 (du/dy)^2 dy for u = Re y (1 - y) / 2 (dp/dx = -1)."""
    val, _ = quad(lambda y: (Re * (1 - 2 * y) / 2) ** 2, 0.0, 1.0)
    assert abs(qpp.dissipation_poiseuille_steady(Re) - val / Re) < 1e-12 * val


@pytest.mark.parametrize("N", [4, 8, 16, 128])
@pytest.mark.parametrize("Re", [1.0, 10.0, 1000.0])
def test_grid_dissipation_closed_form(N, Re):
    """On the exact steady profile, D u = Re (1 - 2 y_j) / 2 at the interior
    nodes y_j = j h, and (1/N) sum_j (1 - 2 j h)^2 = (N - 1) / (3 (N + 1)),
    so the grid value is the continuous one times (1 - 2h)."""
    ch = flow.channel(N=N, Re=Re)
    h = 1.0 / (N + 1)
    u = 0.5 * Re * ch.y * (1 - ch.y)
    e = qpp.dissipation_fd(u, h, 1 / Re)
    want = qpp.dissipation_poiseuille_steady(Re) * (1 - 2 * h)
    assert abs(e - want) <= 1e-12 * want


def test_classical_march_reaches_steady_quadratic():
    """Backward Euler's fixed point is the discrete steady state, which the
    finite differences make the exact quadratic."""
    ch = flow.channel(N=8, Re=10.0, dt=2.5)
    u = flow.classical_be(ch, 200)[-1]
    np.testing.assert_allclose(u, 5.0 * ch.y * (1 - ch.y), rtol=0, atol=1e-10)
