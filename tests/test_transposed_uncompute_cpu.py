"""The identity behind k_pipe_c, checked on the CPU.

After the eigenvalue inversion the uncompute runs the QFT on the clock, the
inverse controlled powers (in the eigen frame a diagonal over the clock,
ph(y) = prod_b om_b^(y_b)) and the Hadamard layer; post-selection on clock 0
keeps z = sum_y ph(y) (F v)(y).  The pipeline kernels run the QFT as the
forward cascade F (top bit first; stage b maps the pair (a0, a1) that differs
in bit b to (a0 + a1, (a0 - a1) t_b), t_b = exp(2 pi i (y mod 2^b) / 2^(b+1))).
k_pipe_c evaluates z as sum_y v(y) K(y) with the closed form
    K(y) = prod_b (1 + (-1)^(y_b) t_b(y mod 2^b) om_b)
of the transposed cascade applied to ph, contracting lines of the top RB
clock bits from the top down and multiplying by the factors of the bits
below.  Pins:
* F is the unnormalised DFT with kernel exp(+2 pi i j k / N), output in
  bit-reversed order (numpy's inverse FFT times N), so the QFT the kernels
  transpose is the textbook one;
* the closed form K equals F^T ph built stage by stage, and the projection
  sum_y ph(y) (F v)(y) equals sum_y v(y) K(y), for every clock width the
  pipeline uses (1..16 bits, up to 10 here);
* the line contraction in the kernel's order, with the twiddles of the line
  bits split as exp(2 pi i lo / 2^(b+1)) times a 16th root of unity, gives
  the same sum;
* a planted mistake (a dropped factor, a conjugated twiddle) is caught.
"""
import numpy as np
import pytest


def cascade(v, c):
    a = np.array(v, dtype=complex)
    for b in range(c - 1, -1, -1):
        h = 1 << b
        y = np.arange(1 << c)
        lo = y[(y & h) == 0]
        t = np.exp(2j * np.pi * (lo % h) / (2 * h))
        a0, a1 = a[lo].copy(), a[lo | h].copy()
        a[lo], a[lo | h] = a0 + a1, (a0 - a1) * t
    return a


def cascade_matrix(c):
    n = 1 << c
    return np.stack([cascade(np.eye(n)[k], c) for k in range(n)], axis=1)


def bitrev(y, c):
    return int(format(y, f"0{c}b")[::-1], 2) if c else 0


def closed_form_k(om, c, conj_twiddle=False, drop=None):
    y = np.arange(1 << c)
    K = np.ones(1 << c, dtype=complex)
    for b in range(c):
        if b == drop:
            continue
        t = np.exp(2j * np.pi * (y % (1 << b)) / (2 << b))
        if conj_twiddle:
            t = np.conj(t)
        sgn = np.where((y >> b) & 1, -1.0, 1.0)
        K *= 1.0 + sgn * t * om[b]
    return K


def phase_product(om, c):
    y = np.arange(1 << c)
    ph = np.ones(1 << c, dtype=complex)
    for b in range(c):
        ph *= np.where((y >> b) & 1, om[b], 1.0)
    return ph


def line_contraction(v, om, c, rb):
    """the kernel's evaluation order: lines of the top rb bits, contracted
    from the top down, times the factors of the bits below L = c - rb"""
    L = c - rb
    z = 0.0j
    for lo in range(1 << L):
        u = np.array([v[lo + (k << L)] for k in range(1 << rb)], dtype=complex)
        for kb in range(rb - 1, -1, -1):
            b, h = L + kb, 1 << kb
            Q = om[b] * np.exp(2j * np.pi * lo / (2 << b))
            for m in range(h):
                q = Q * np.exp(2j * np.pi * m / (2 << kb))
                s, d = u[m] + u[m + h], u[m] - u[m + h]
                u[m] = s + q * d
        f = 1.0 + 0j
        for b in range(L):
            t = np.exp(2j * np.pi * (lo % (1 << b)) / (2 << b))
            f *= (1.0 - t * om[b]) if (lo >> b) & 1 else (1.0 + t * om[b])
        z += u[0] * f
    return z


@pytest.mark.parametrize("c", range(1, 9))
def test_cascade_is_the_textbook_qft_up_to_bit_order(c):
    rng = np.random.default_rng(40 + c)
    v = rng.standard_normal(1 << c) + 1j * rng.standard_normal(1 << c)
    d = np.fft.ifft(v) * (1 << c)                 # sum_k exp(+2 pi i j k / N) v_k
    br = np.array([d[bitrev(y, c)] for y in range(1 << c)])
    assert np.abs(cascade(v, c) - br).max() <= 1e-12 * (1 << c)


@pytest.mark.parametrize("c", range(1, 9))
def test_closed_form_is_the_transposed_cascade(c):
    rng = np.random.default_rng(70 + c)
    theta = rng.random()
    om = np.conj(np.exp(2j * np.pi * theta * (2.0 ** np.arange(c))))   # conjugated QPE phases
    ph = phase_product(om, c)
    K = closed_form_k(om, c)
    assert np.abs(cascade_matrix(c).T @ ph - K).max() <= 1e-11 * (1 << c)
    # and for arbitrary unit phases, not only those of one eigenvalue
    om2 = np.exp(2j * np.pi * rng.random(c))
    assert np.abs(cascade_matrix(c).T @ phase_product(om2, c) - closed_form_k(om2, c)).max() <= 1e-11 * (1 << c)


@pytest.mark.parametrize("c,rb", [(2, 1), (3, 1), (5, 2), (7, 3), (8, 4), (10, 4)])
def test_projection_three_ways(c, rb):
    rng = np.random.default_rng(100 + c)
    v = rng.standard_normal(1 << c) + 1j * rng.standard_normal(1 << c)
    om = np.exp(2j * np.pi * rng.random(c))
    z_gates = np.sum(phase_product(om, c) * cascade(v, c))
    z_closed = np.sum(v * closed_form_k(om, c))
    z_lines = line_contraction(v, om, c, rb)
    scale = np.abs(v).sum() * 2.0 ** c
    assert abs(z_gates - z_closed) <= 1e-12 * scale
    assert abs(z_gates - z_lines) <= 1e-12 * scale


@pytest.mark.parametrize("mistake", ["drop_top", "drop_bottom", "conj_twiddle"])
def test_planted_mistakes_are_caught(mistake):
    c = 6
    rng = np.random.default_rng(9)
    v = rng.standard_normal(1 << c) + 1j * rng.standard_normal(1 << c)
    om = np.exp(2j * np.pi * rng.random(c))
    z_gates = np.sum(phase_product(om, c) * cascade(v, c))
    kw = {"drop_top": {"drop": c - 1}, "drop_bottom": {"drop": 0}, "conj_twiddle": {"conj_twiddle": True}}[mistake]
    z_bad = np.sum(v * closed_form_k(om, c, **kw))
    assert abs(z_gates - z_bad) > 1e-3 * abs(z_gates)
