"""Pins of the oracle's central-difference gradient and Step 2 projection.

Sec. 2.3 replaces derivatives by central differences, whose symbol is
i sin(h xi)/h. Step 2 of Sec. 2.1 is the Helmholtz projection: the
displacement fluctuation u minimising |D_h u - H|^2 for H = F - Lambda/rho.
Pins:
  * the gradient of a sampled sinusoid, in closed form;
  * a manufactured displacement is recovered exactly from its gradient plus a
    discrete curl plus a constant (both orthogonal to the range of D_h);
  * the normal equations D_h^T (D_h u - H) = 0 for random H (checked with a
    stencil written here, not through the Fourier route);
  * idempotence, zero mean, null-mode (Nyquist-corner) content removed.
"""
import itertools

import numpy as np
import pytest

import oracle as O


def grid(shape):
    n3, n2, n1 = shape
    return np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")


def cdiff(f, j):
    """central difference along x_{j+1} of an array indexed (k3, k2, k1)."""
    ax = 2 - j
    return 0.5 * (np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax))


def manufactured(shape, modes, seed=0):
    """u_i = sum_m a_im sin(theta_m + phi_m) and its exact central-difference
    gradient G_ij = sum_m a_im cos(theta_m + phi_m) sin(2 pi m_j / n_j)."""
    rng = np.random.default_rng(seed)
    n3, n2, n1 = shape
    nn = (n1, n2, n3)
    k3, k2, k1 = grid(shape)
    u = np.zeros((3,) + shape)
    G = np.zeros((9,) + shape)
    for m in modes:
        th = 2 * np.pi * (m[0] * k1 / n1 + m[1] * k2 / n2 + m[2] * k3 / n3) + rng.uniform(0, 2 * np.pi)
        a = rng.standard_normal(3)
        for i in range(3):
            u[i] += a[i] * np.sin(th)
            for j in range(3):
                G[3 * i + j] += a[i] * np.cos(th) * np.sin(2 * np.pi * m[j] / nn[j])
    return u, G


def is_null(m, nn):
    return all((mj % n == 0) or (2 * (mj % n) == n) for mj, n in zip(m, nn))


SHAPE = (6, 8, 10)
MODES = [(1, 0, 0), (0, 3, 1), (2, 1, 5), (4, 2, 3), (5, 4, 1), (5, 0, 2)]  # (m1, m2, m3)


def test_gradient_of_sinusoid_closed_form():
    u, G = manufactured(SHAPE, MODES)
    Fbar = np.arange(9.0) / 10.0
    got = O.gradient(u, Fbar)
    ref = G + Fbar[:, None, None, None]
    assert np.max(np.abs(got - ref)) <= 1e-13


def test_projection_recovers_manufactured_displacement():
    n3, n2, n1 = SHAPE
    assert not any(is_null(m, (n1, n2, n3)) for m in MODES)
    u, G = manufactured(SHAPE, MODES)
    rng = np.random.default_rng(1)
    # a discrete curl: S_ij = eps_jkl d_k phi_il, annihilated by D_h^T
    phi = rng.standard_normal((3, 3) + SHAPE)
    S = np.zeros((9,) + SHAPE)
    eps = np.zeros((3, 3, 3))
    for (j, k, l), s in (((0, 1, 2), 1), ((1, 2, 0), 1), ((2, 0, 1), 1),
                         ((0, 2, 1), -1), ((2, 1, 0), -1), ((1, 0, 2), -1)):
        eps[j, k, l] = s
    for i, j, k, l in itertools.product(range(3), repeat=4):
        if eps[j, k, l]:
            S[3 * i + j] += eps[j, k, l] * cdiff(phi[i, l], k)
    H = G + S + rng.standard_normal(9)[:, None, None, None]
    got, imag = O.project(H, return_imag=True)
    assert np.max(np.abs(got - u)) <= 1e-13 * max(1.0, np.max(np.abs(u)))
    assert imag <= 1e-13


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 8, 10), (2, 6, 4), (1, 6, 8)])
def test_projection_solves_normal_equations(shape):
    rng = np.random.default_rng(7)
    H = rng.standard_normal((9,) + shape)
    u = O.project(H)
    G = np.stack([cdiff(u[i], j) for i in range(3) for j in range(3)])
    R = G - H
    # D_h^T R = -sum_j d_j R_ij must vanish
    div = np.stack([-sum(cdiff(R[3 * i + j], j) for j in range(3)) for i in range(3)])
    assert np.max(np.abs(div)) <= 1e-12 * np.max(np.abs(H))
    assert np.max(np.abs(u.mean(axis=(1, 2, 3)))) <= 1e-13


def test_projection_idempotent_and_null_modes_removed():
    rng = np.random.default_rng(9)
    shape = (8, 6, 4)
    H = rng.standard_normal((9,) + shape)
    u = O.project(H)
    G = np.stack([cdiff(u[i], j) for i in range(3) for j in range(3)])
    u2 = O.project(G)
    assert np.max(np.abs(u2 - u)) <= 1e-12 * np.max(np.abs(u))
    # a field made only of Nyquist-corner modes has zero central difference
    k3, k2, k1 = grid(shape)
    checker = (-1.0) ** k1 * (-1.0) ** (k2 + k3)
    Hn = np.stack([checker * c for c in rng.standard_normal(9)])
    assert np.max(np.abs(O.project(Hn))) <= 1e-13
