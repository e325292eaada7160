"""Dense brute-force operators for small qubit counts (test helper).

Written independently of oracle.c: operators are built as Kronecker
products of per-qubit 2x2 blocks, with qubit n-1 the leftmost factor
(qubit q = bit q of the basis index).
"""
import functools

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def kron_all(blocks_msb_first):
    return functools.reduce(np.kron, blocks_msb_first, np.eye(1, dtype=np.complex128))


def gate_matrix(n, target, u, ctrls=(), cvals=None):
    """I + (prod of control projectors) (x) (u - I) on the target."""
    cvals = list(cvals) if cvals is not None else [1] * len(ctrls)
    blocks = []
    for q in reversed(range(n)):
        if q == target:
            blocks.append(np.asarray(u, dtype=np.complex128) - I2)
        elif q in ctrls:
            blocks.append(P1 if cvals[list(ctrls).index(q)] else P0)
        else:
            blocks.append(I2)
    return np.eye(1 << n, dtype=np.complex128) + kron_all(blocks)


def swap_matrix(n, q1, q2, ctrls=(), cvals=None):
    """Permutation matrix exchanging bits q1 and q2 where the controls match."""
    cvals = list(cvals) if cvals is not None else [1] * len(ctrls)
    dim = 1 << n
    M = np.zeros((dim, dim), dtype=np.complex128)
    for i in range(dim):
        ok = all(((i >> c) & 1) == v for c, v in zip(ctrls, cvals))
        j = i
        if ok and ((i >> q1) & 1) != ((i >> q2) & 1):
            j = i ^ ((1 << q1) | (1 << q2))
        M[j, i] = 1.0
    return M


def apply_on_axes(psi, n, U, qubits):
    """Apply the 2^m x 2^m matrix U to the qubits `qubits` (listed from the
    least significant register bit upward) with numpy tensordot."""
    m = len(qubits)
    t = psi.reshape((2,) * n)                   # axis a <-> qubit n-1-a
    axes = [n - 1 - q for q in reversed(qubits)]  # register MSB first
    Ut = np.asarray(U).reshape((2,) * (2 * m))
    out = np.tensordot(Ut, t, axes=(list(range(m, 2 * m)), axes))
    # tensordot puts the new register axes first; move them back
    rest = [a for a in range(n) if a not in axes]
    order = axes + rest
    inv = np.argsort(order)
    return np.transpose(out, inv).reshape(-1)
