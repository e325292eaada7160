"""The operator identities behind the fused controlled powers of the QPP
squaring circuit, checked on the CPU against the oracle's gate-by-gate
circuit.  On one (address s, ub = t, up) column, with X, Y the a2 = 0 and
a2 = 1 planes of the (ua, a1) block (X[i][j], i = ua, j = a1):
- U_V^2 = I, so U_V S_0 U_V is the reflection I - 2 w w^T (w = U_V|0>) on
  column s of X and the identity elsewhere;
- T^2 = I and T (-S_chi) T = Z(a2) SWAP(ua, a1);
- hence Q^t = T R (Z SWAP) R ... R T (-S_chi): t reflections alternating
  between column s and row s of X, and one sign of Y after the closing T when
  t - 1 is odd.  (Q^dagger)^t moves -S_chi to the end.
The circuit below is the oracle's own, with its controlled powers replaced by
that sequence; both must give the same final state."""

import numpy as np
import pytest

import oracle


def _swap_test(X, Y):
    return (X + Y + X.T - Y.T) / 2, (X + Y - X.T + Y.T) / 2


def _powers(psi, n, r, u, inverse):
    N, B = 1 << n, 1 << (2 * n)
    z = u / np.linalg.norm(u)
    w = oracle.qadc_loader(z)[:, 0]                                  # U_V|0>
    for col in range(1 << (n + r + 1)):
        s, t = col & (N - 1), (col >> n) & ((1 << r) - 1)
        if t == 0:
            continue
        base = (s << (2 * n)) | ((col >> n) << (3 * n + 1))
        idx = base + np.arange(B)
        X = psi[idx].reshape(N, N).T.copy()
        Y = psi[idx + (1 << (3 * n))].reshape(N, N).T.copy()
        if not inverse:
            Y = -Y
        X, Y = _swap_test(X, Y)
        for k in range(t):
            if k % 2 == 0:
                X[:, s] -= 2 * w * (w @ X[:, s])
            else:
                X[s, :] -= 2 * w * (w @ X[s, :])
        X, Y = _swap_test(X, Y)
        if ((t - 1) % 2 == 1) != inverse:
            Y = -Y
        psi[idx] = X.T.ravel()
        psi[idx + (1 << (3 * n))] = Y.T.ravel()


def _circuit_with_fused_powers(u, r):
    """The oracle's circuit (same steps, same gates) with the controlled
    powers of phase estimation and of its uncompute applied as above."""
    import inspect
    src = inspect.getsource(oracle.qadc_square)
    src = src.replace("""    for k in range(r):
        for _ in range(1 << k):
            controlled_Q(ub[k], False)""", "    _powers(psi, n, r, u, False)")
    src = src.replace("""    for k in reversed(range(r)):
        for _ in range(1 << k):
            controlled_Q(ub[k], True)""", "    _powers(psi, n, r, u, True)")
    assert src.count("_powers(") == 2
    ns = dict(vars(oracle))
    ns["_powers"] = lambda psi, n, r, u, inv: _powers(psi, n, r, np.asarray(u, float), inv)
    exec(src, ns)
    return ns["qadc_square"](u, r, avg=True)


@pytest.mark.parametrize("n,r,seed", [(1, 1, 0), (1, 3, 1), (2, 2, 2), (2, 4, 3), (3, 2, 4)])
def test_fused_powers_equal_the_gate_sequence(n, r, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(1 << n)
    want = oracle.qadc_square(u, r, avg=True)
    got = _circuit_with_fused_powers(u, r)
    assert np.abs(got - want).max() < 1e-13
