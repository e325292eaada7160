"""Pins of the QSP-1 oracle (binary-tree state preparation): the paper's
worked example (its intermediate and final states), the closed form b/|b|
for random real and complex vectors with empty subtrees, and a one-qubit
case against the textbook rotation."""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows():
    rows = []
    for line in open(os.path.join(GOLDEN, "qsp1_worked_example.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return rows


def _ket_order(sq):
    # |q1 q0> with q1 decided at the root: register value r = 2 q1 + q0
    return np.asarray(sq)


def test_worked_example_final_state():
    target, _, _ = _golden_rows()
    b = np.sqrt(target)
    psi = oracle.qsp(2, 0, b)
    assert np.allclose(np.abs(psi) ** 2, _ket_order(target), atol=1e-15)
    assert np.allclose(psi.imag, 0.0, atol=1e-15)


def test_worked_example_after_root_rotation():
    target, children, after_root = _golden_rows()
    assert np.isclose(sum(children), 1.0) and np.isclose(children[0], target[0] + target[1])
    psi = oracle.qsp(2, 0, np.sqrt(target), levels=1)
    assert np.allclose(np.abs(psi) ** 2, _ket_order(after_root), atol=1e-15)


@pytest.mark.parametrize("m,q_lo,n,kind", [(1, 0, 1, "real"), (2, 1, 4, "complex"), (5, 0, 5, "real"),
                                           (6, 2, 9, "complex"), (9, 0, 9, "complex")])
def test_closed_form(m, q_lo, n, kind):
    rng = np.random.default_rng(10 * m + q_lo)
    b = rng.standard_normal(1 << m)
    if kind == "complex":
        b = b + 1j * rng.standard_normal(1 << m)
    b[rng.random(1 << m) < 0.25] = 0.0            # empty subtrees
    if not np.any(b):
        b[0] = 1.0
    psi = oracle.qsp(n, q_lo, b)
    ref = np.zeros(1 << n, dtype=complex)
    ref[np.arange(1 << m) << q_lo] = b / np.linalg.norm(b)
    assert np.abs(psi - ref).max() <= 1e-14


def test_one_qubit_is_the_textbook_rotation():
    theta = 1.234
    b = np.array([math.cos(theta / 2), math.sin(theta / 2)])
    psi = oracle.qsp(1, 0, b)
    ry = np.array([[math.cos(theta / 2), -math.sin(theta / 2)], [math.sin(theta / 2), math.cos(theta / 2)]])
    assert np.allclose(psi, ry @ np.array([1.0, 0.0]), atol=1e-15)


def test_errors():
    with pytest.raises(oracle.OracleError):
        oracle.qsp(3, 0, np.zeros(4))
    with pytest.raises(oracle.OracleError):
        oracle.qsp(2, 1, np.ones(4))               # register past the top qubit
