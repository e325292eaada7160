"""The T0-Q_PE error diagram of the main text ("Flow simulation results":
the least error over T0 for each number of clock qubits, its power-law decay,
and where the optimal T0 sits).

The paper's sample system (8 x 8, kappa = 18.8795) is not printed; the stand-in
is the 8-point second-difference matrix shifted by sigma I so that kappa is
18.8795 exactly, with the uniform (Poiseuille) right-hand side.  Every
(T0, n_c) point is one HHL solve of the batched library path; the error is
eps_QLSA = |u_Q - u_C| = sqrt(2 - 2 F) for unit vectors (F the fidelity against
the FP64 classical solution).  T0 is reported as the factor T0 lambda_max / 2 pi.
"""
from __future__ import annotations

import math

import numpy as np

from . import binding as B
from . import inputs


def sample_system(N: int = 8, kappa: float = 18.8795):
    A = inputs.laplacian_1d(N)
    lam = np.linalg.eigvalsh(A)
    sigma = (lam.max() - kappa * lam.min()) / (kappa - 1.0)
    A = A + sigma * np.eye(N)
    return A, np.ones(N)


def diagram(n_cs=range(3, 15), factors=None, dtype: str = "c128"):
    A, b = sample_system()
    lmax = np.linalg.eigvalsh(A).max()
    if factors is None:
        factors = np.geomspace(0.25, 2.0, 256)
    t0 = np.asarray(factors) * 2 * math.pi / lmax
    res = B.sv_hhl_batch([(A, b, int(n_c), t0) for n_c in n_cs], dtype)
    F = res[:, 3].reshape(len(list(n_cs)), len(t0))
    eps = np.sqrt(np.maximum(0.0, 2.0 - 2.0 * F))
    rows = []
    for i, n_c in enumerate(n_cs):
        k = int(np.argmin(eps[i]))
        rows.append({"n_c": int(n_c), "eps_min": float(eps[i, k]), "factor_at_min": float(factors[k]),
                     "least_count": 2.0 ** -n_c})
    return rows, eps


def power_law(rows, lo: int = 5):
    """Least-squares fit of log eps_min against log n_c (n_c >= lo)."""
    x = np.array([r["n_c"] for r in rows if r["n_c"] >= lo], dtype=float)
    y = np.array([r["eps_min"] for r in rows if r["n_c"] >= lo])
    p, c = np.polyfit(np.log(x), np.log(y), 1)
    return float(p), float(math.exp(c))


def _main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="T0-Q_PE error diagram on the kappa = 18.8795 sample system")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    rows, eps = diagram()
    for r in rows:
        print(f"[tq] n_c {r['n_c']:2d}: eps_min {r['eps_min']:.3e} at T0 lambda_max / 2 pi = "
              f"{r['factor_at_min']:.4f} (least count {r['least_count']:.2e})", flush=True)
    p, c = power_law(rows)
    print(f"[tq] eps_min ~ {c:.3g} n_c^{p:.2f} (n_c >= 5)", flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"rows": rows, "power": p, "coef": c}, f, indent=1)


if __name__ == "__main__":
    _main()
