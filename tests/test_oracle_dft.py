"""Pins of the oracle's discrete Fourier transform (periodic setting, Sec. 2.3).

The oracle computes the DFT as separable direct sums. These tests pin it
against what the definition fixes independently: the full (non-separable)
O(V^2) triple sum written out here, single Fourier modes (exact deltas),
Hermitian symmetry of real input, Parseval's identity, the inverse, and the
library FFT (numpy.fft.fftn) as a textbook special case.
"""
import numpy as np
import pytest

import oracle as O


def brute_dft3(x):
    n3, n2, n1 = x.shape
    k3, k2, k1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    out = np.zeros(x.shape, complex)
    for m3 in range(n3):
        for m2 in range(n2):
            for m1 in range(n1):
                ph = np.exp(-2j * np.pi * (m1 * k1 / n1 + m2 * k2 / n2 + m3 * k3 / n3))
                out[m3, m2, m1] = np.sum(x * ph)
    return out


@pytest.mark.parametrize("shape", [(2, 6, 4), (6, 6, 6), (4, 3, 5), (1, 4, 6), (3, 1, 2)])
def test_dft_matches_brute_force_triple_sum(shape):
    rng = np.random.default_rng(11)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = brute_dft3(x)
    got = O.dft3(x)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)) * np.sqrt(x.size)


def test_single_mode_gives_delta():
    n3, n2, n1 = 6, 4, 8
    k3, k2, k1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    m = (3, 1, 5)  # (m1, m2, m3)
    x = np.exp(2j * np.pi * (m[0] * k1 / n1 + m[1] * k2 / n2 + m[2] * k3 / n3))
    X = O.dft3(x)
    ref = np.zeros_like(X)
    ref[m[2], m[1], m[0]] = x.size
    assert np.max(np.abs(X - ref)) <= 1e-12


def test_real_input_is_hermitian_and_parseval():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((6, 8, 4))
    X = O.dft3(x)
    n3, n2, n1 = x.shape
    for m3 in range(n3):
        for m2 in range(n2):
            for m1 in range(n1):
                a = X[m3, m2, m1]
                b = X[(-m3) % n3, (-m2) % n2, (-m1) % n1]
                assert abs(a - np.conj(b)) <= 1e-12
    assert abs(np.sum(np.abs(X) ** 2) / x.size - np.sum(x ** 2)) <= 1e-12 * np.sum(x ** 2)


def test_inverse_round_trip_and_library_fft():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((12, 16, 18)) + 1j * rng.standard_normal((12, 16, 18))
    X = O.dft3(x)
    assert np.max(np.abs(X - np.fft.fftn(x))) <= 1e-12 * np.max(np.abs(X))
    y = O.dft3(X, inverse=True)
    assert np.max(np.abs(y - x)) <= 1e-13 * np.max(np.abs(x)) * 10
