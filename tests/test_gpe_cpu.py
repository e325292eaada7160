"""The gapped-phase-estimation parameter rule against its promise, through
the pinned closed form of the flag probabilities (Fejer kernel): for
|lambda| <= eps the flag-1 probability, for |lambda| >= 2 eps the flag-0
probability, both at most delta^2; and the cut sits inside the gap."""
import math

import numpy as np
import pytest

from paper_2307_00391_amd import gpe
from tests.closed_form import gpe_weights


@pytest.mark.parametrize("eps,delta,lam_max", [(0.1, 0.3, 1.0), (0.05, 0.2, 2.0), (0.02, 0.3, 1.0), (0.25, 0.1, 1.0)])
def test_parameter_rule_keeps_the_promise(eps, delta, lam_max):
    n_c, T0, cut = gpe.parameters(eps, delta, lam_max)
    M = 1 << n_c
    lam_small = np.concatenate([np.linspace(-eps, eps, 301)])
    lam_big = np.concatenate([np.linspace(2 * eps, lam_max, 301), -np.linspace(2 * eps, lam_max, 301)])
    g_s, _ = gpe_weights(lam_small * T0 / (2 * math.pi), n_c, cut, signed=True)
    _, h_b = gpe_weights(lam_big * T0 / (2 * math.pi), n_c, cut, signed=True)
    assert g_s.max() <= delta ** 2, g_s.max()
    assert h_b.max() <= delta ** 2, h_b.max()
    y_eps = eps * T0 * M / (2 * math.pi)
    assert y_eps < cut < 2 * y_eps and cut < M // 2


def test_parameter_rule_rejects_bad_input():
    with pytest.raises(ValueError):
        gpe.parameters(0.6, 0.1, 1.0)
    with pytest.raises(ValueError):
        gpe.parameters(0.1, 1.5, 1.0)
