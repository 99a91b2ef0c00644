"""Pins of the oracle's constitutive functions.

Neo-Hookean W = mu/2(|F|^2 - 3) - mu ln J + lambda/2 (ln J)^2 (the compressible
energy of the benchmark workloads) and the neo-classical LCE energy of Sec. 5.1
with a volumetric penalty. Pins: finite differences of W -> P -> tangent,
major symmetry of the tangent, frame indifference and isotropy, the
small-strain limit (Lame moduli), a stress-free reference state, the
director-independence of the LCE energy at a = 1 (Sec. 5.1 notes r = 1 reduces
the entropic term to neo-Hookean), and the top-eigenvector director rule.
"""
import numpy as np
import pytest

import oracle as O


def rot(seed):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def randF(seed, amp=0.15):
    rng = np.random.default_rng(seed)
    return np.eye(3) + amp * rng.standard_normal((3, 3))


def unit(seed):
    v = np.random.default_rng(seed).standard_normal(3)
    return v / np.linalg.norm(v)


MATS = {
    "neohooke": O.material("neohooke", mu=10.0, lam=100.0),
    "lce": O.material("lce", mu=1.0, a=2.0, kappa=100.0),
}


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_stress_and_tangent_by_finite_differences(name, seed):
    m = MATS[name]
    F = randF(seed).ravel()
    n = unit(seed + 10)
    h = 1e-6
    P = O.stress(m, F, n)
    C = O.tangent(m, F, n)
    Pfd = np.array([(O.energy(m, F + h * e, n) - O.energy(m, F - h * e, n)) / (2 * h)
                    for e in np.eye(9)])
    Cfd = np.stack([(O.stress(m, F + h * e, n) - O.stress(m, F - h * e, n)) / (2 * h)
                    for e in np.eye(9)], axis=1)
    assert np.max(np.abs(P - Pfd)) <= 1e-7 * max(1.0, np.max(np.abs(P)))
    assert np.max(np.abs(C - Cfd)) <= 1e-7 * np.max(np.abs(C))
    assert np.max(np.abs(C - C.T)) <= 1e-12 * np.max(np.abs(C))


@pytest.mark.parametrize("name", list(MATS))
def test_frame_indifference(name):
    m = MATS[name]
    for s in range(4):
        F = randF(s)
        n = unit(s + 20)
        Q = rot(s + 40)
        W = O.energy(m, F.ravel(), n)
        assert abs(O.energy(m, (Q @ F).ravel(), Q @ n) - W) <= 1e-13 * max(1.0, abs(W))
        P = O.stress(m, F.ravel(), n).reshape(3, 3)
        PQ = O.stress(m, (Q @ F).ravel(), Q @ n).reshape(3, 3)
        assert np.max(np.abs(PQ - Q @ P)) <= 1e-12 * max(1.0, np.max(np.abs(P)))


def test_neohooke_isotropy_and_reference_state():
    m = MATS["neohooke"]
    for s in range(4):
        F = randF(s)
        Q = rot(s + 7)
        assert abs(O.energy(m, (F @ Q).ravel()) - O.energy(m, F.ravel())) <= 1e-12
    assert O.energy(m, np.eye(3).ravel()) == 0.0
    assert np.max(np.abs(O.stress(m, np.eye(3).ravel()))) == 0.0


def test_neohooke_small_strain_limit_is_lame():
    mu, lam = 3.0, 7.0
    m = O.material("neohooke", mu=mu, lam=lam)
    C = O.tangent(m, np.eye(3).ravel()).reshape(3, 3, 3, 3)
    d = np.eye(3)
    ref = (lam * np.einsum("ij,kl->ijkl", d, d) + mu * np.einsum("ik,jl->ijkl", d, d)
           + mu * np.einsum("il,jk->ijkl", d, d))
    assert np.max(np.abs(C - ref)) <= 1e-14


def test_lce_a1_is_director_independent_and_director_rule():
    m1 = O.material("lce", mu=2.0, a=1.0, kappa=5.0)
    F = randF(3).ravel()
    w = [O.energy(m1, F, unit(s)) for s in range(5)]
    assert np.ptp(w) <= 1e-13
    # the minimising director at fixed F is the top eigenvector of F F^T
    m = MATS["lce"]
    for s in range(5):
        F = randF(s, 0.3)
        n_prev = unit(s + 50)
        n = O.director(F.ravel(), n_prev)
        w_, V = np.linalg.eigh(F @ F.T)
        top = V[:, -1] * np.sign(V[:, -1] @ n_prev)
        assert np.max(np.abs(n - top)) <= 1e-12
        assert n @ n_prev >= 0
        e_best = O.energy(m, F.ravel(), n)
        for t in range(20):
            assert e_best <= O.energy(m, F.ravel(), unit(100 + t)) + 1e-14
    # at F = I every director is optimal: the previous one is kept
    n_prev = unit(77)
    assert np.max(np.abs(O.director(np.eye(3).ravel(), n_prev) - n_prev)) <= 1e-15
    # stretch along x2 selects e2
    F = np.diag([1.0, 1.3, 0.9]).ravel()
    assert np.max(np.abs(np.abs(O.director(F, unit(5))) - np.array([0, 1.0, 0]))) <= 1e-14
