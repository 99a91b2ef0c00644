"""Pins of the oracle's local problem (Step 1 of Sec. 2.1).

Step 1 solves W_F(F) - Lambda - rho(grad u - F) = 0 at each point, i.e. F is
the minimiser of W(F) + rho/2 |F - A|^2 with A = grad u + Lambda/rho. Pins:
stationarity, local minimality against random perturbations, covariance
under rotations (prox(QA) = Q prox(A), and prox(AQ) = prox(A) Q for the
isotropic energy), the exact fixed point A = F + P(F)/rho, and the quadratic
(small-strain) limit where the prox map is a closed-form linear solve.
"""
import numpy as np
import pytest

import oracle as O
from test_oracle_material import randF, rot, unit

NH = O.material("neohooke", mu=10.0, lam=100.0)


def phi(m, rho, A, F, n):
    return O.energy(m, F, n) + 0.5 * rho * np.sum((F - A) ** 2)


@pytest.mark.parametrize("rho", [2.0, 5.0, 20.0])
@pytest.mark.parametrize("seed", range(4))
def test_neohooke_prox_stationary_and_minimal(rho, seed):
    A = randF(seed, 0.1).ravel()
    F, _, it, rc = O.prox(NH, rho, A, np.eye(3).ravel())
    assert rc == O.OK and it < 20
    g = O.stress(NH, F) + rho * (F - A)
    assert np.linalg.norm(g) <= 1e-11
    f0 = phi(NH, rho, A, F, (0, 0, 1))
    rng = np.random.default_rng(seed)
    for _ in range(20):
        d = 1e-4 * rng.standard_normal(9)
        assert phi(NH, rho, A, F + d, (0, 0, 1)) >= f0 - 1e-14


def test_neohooke_prox_covariance():
    rho = 5.0
    for s in range(4):
        A = randF(s, 0.1)
        Q, R = rot(s + 3), rot(s + 30)
        F, _, _, _ = O.prox(NH, rho, A.ravel(), np.eye(3).ravel())
        F = F.reshape(3, 3)
        FQ, _, _, _ = O.prox(NH, rho, (Q @ A).ravel(), (Q @ F).ravel() + 1e-3)
        FR, _, _, _ = O.prox(NH, rho, (A @ R).ravel(), np.eye(3).ravel())
        assert np.max(np.abs(FQ.reshape(3, 3) - Q @ F)) <= 1e-12
        assert np.max(np.abs(FR.reshape(3, 3) - F @ R)) <= 1e-12


def test_prox_fixed_point():
    # rho large against the stresses, so that the local problem is convex
    rho = 60.0
    for s in range(4):
        Fs = randF(s, 0.05).ravel()
        A = Fs + O.stress(NH, Fs) / rho
        F, _, _, rc = O.prox(NH, rho, A, np.eye(3).ravel())
        assert rc == O.OK
        assert np.max(np.abs(F - Fs)) <= 1e-12


def test_prox_quadratic_limit():
    """For tiny strains W ~ 1/2 eps:C:eps, so prox(I + dA) ~ I + (C + rho)^{-1} rho dA."""
    rho = 4.0
    C = O.tangent(NH, np.eye(3).ravel())
    rng = np.random.default_rng(0)
    dA = 1e-7 * rng.standard_normal(9)
    F, _, _, _ = O.prox(NH, rho, np.eye(3).ravel() + dA, np.eye(3).ravel())
    lin = np.linalg.solve(C + rho * np.eye(9), rho * dA)
    # the neglected terms are O(|dA|) relative; rounding of F - I is ~1e-9 relative
    assert np.max(np.abs((F - np.eye(3).ravel()) - lin)) <= 1e-6 * np.max(np.abs(lin))
