"""Pins of the oracle's mixed boundary conditions (Sec. 2.3: some components
of <F> prescribed, the complementary components of the average stress zero;
the UNI / PE / EB protocols of Sec. 5 leave components of <F> free).

A free component of <F> is one more unknown of Step 2's minimisation; the
checks here do not use that formula:
  * a homogeneous neo-Hookean body under uniaxial stress (only <F_11>
    prescribed) ends at the homogeneous state whose lateral stretch zeroes
    the lateral stress, found here by a scalar root (brentq), with no
    fluctuation and zero average stress in every free component;
  * the two-phase laminate with <F_33> free ends at the closed-form solution
    of the two equations traction continuity and <P_33> = 0 (scipy fsolve);
  * after every iteration the multiplier's average vanishes in the free
    components (then <P> = <Lambda> = 0 there at convergence) and follows
    <Lambda> + rho (<F> - <F_{i+1}>) in the prescribed ones.
"""
import numpy as np
import pytest
from scipy.optimize import brentq, fsolve

import oracle as O
from paper_2010_06697_amd import microstructure as M


def nh_P(F, mu, lam):
    F = np.asarray(F, dtype=float).reshape(3, 3)
    Fit = np.linalg.inv(F).T
    return (mu * (F - Fit) + lam * np.log(np.linalg.det(F)) * Fit).ravel()


def test_uniaxial_stress_of_a_homogeneous_body():
    shape = (4, 6, 8)
    phase = np.zeros(shape, np.uint8)
    mu, lam, s = 3.0, 20.0, 1.1
    mats = [O.material("neohooke", mu=mu, lam=lam)]
    free = [k for k in range(9) if k != 0]
    u, F, L = O.initial_state(shape)
    p = O.params(max_iter=3000, tol_p=1e-12, tol_d=1e-12, mu_ref=mu, free=free)
    r = O.admm_run(phase, mats, np.diag([s, 1.0, 1.0]).ravel(), p, u, F, L, 10.0)
    assert r["rc"] == O.OK
    t = brentq(lambda t: nh_P(np.diag([s, t, t]), mu, lam)[4], 0.5, 1.5, xtol=1e-16)
    assert np.max(np.abs(r["Fbar"] - np.diag([s, t, t]).ravel())) <= 1e-10
    assert np.max(np.abs(u)) <= 1e-12
    Pm = O.mean_stress(phase, mats, F)
    assert np.max(np.abs(Pm[free])) <= 1e-10
    assert abs(Pm[0] - nh_P(np.diag([s, t, t]), mu, lam)[0]) <= 1e-10


def test_laminate_with_free_normal_stretch_matches_closed_form():
    case = M.laminate16_case()
    phase = case["phase"]
    (ms, ls), (mf, lf) = (10.0, 100.0), (1.0, 10.0)
    mats = [O.material("neohooke", mu=ms, lam=ls), O.material("neohooke", mu=mf, lam=lf)]
    l1 = 1.05
    u, F, L = O.initial_state(phase.shape)
    p = O.params(max_iter=5000, tol_p=1e-12, tol_d=1e-12, mu_ref=5.5, free=[8])
    r = O.admm_run(phase, mats, np.diag([l1, 1.0, 1.0]).ravel(), p, u, F, L, 5.0)
    assert r["rc"] == O.OK

    def eqs(x):
        d, f33 = x
        Ps = nh_P(np.diag([l1 + d, 1.0, f33]), ms, ls)
        Pf = nh_P(np.diag([l1 - d, 1.0, f33]), mf, lf)
        return [Ps[0] - Pf[0], 0.5 * (Ps[8] + Pf[8])]

    d, f33 = fsolve(eqs, [0.0, 1.0], xtol=1e-13)
    assert np.max(np.abs(eqs([d, f33]))) <= 1e-12
    assert abs(r["Fbar"][8] - f33) <= 1e-10
    Pm = O.mean_stress(phase, mats, F)
    Pd = 0.5 * (nh_P(np.diag([l1 + d, 1.0, f33]), ms, ls) + nh_P(np.diag([l1 - d, 1.0, f33]), mf, lf))
    assert np.max(np.abs(Pm - Pd)) <= 1e-9 * np.max(np.abs(Pd))
    assert abs(Pm[8]) <= 1e-10
    assert abs(F[0, 0, 0, 0] - (l1 + d)) <= 1e-10 and abs(F[0, 0, 0, 15] - (l1 - d)) <= 1e-10


def test_multiplier_average_in_free_and_prescribed_components():
    shape = (6, 4, 8)
    phase = M.random_two_phase(shape, 0.4, seed=5)
    mats = [O.material("neohooke", mu=10.0, lam=40.0), O.material("neohooke", mu=1.0, lam=4.0)]
    Fb = M.random_fbar(0.05, seed=2).ravel()
    free = [1, 4, 8]
    u, F, L = O.initial_state(shape)
    rho = 12.0
    p1 = O.params(max_iter=1, fixed_iters=True, mu_ref=4.0, free=free)
    for it in range(8):
        L0 = L.copy()
        r = O.admm_run(phase, mats, Fb, p1, u, F, L, rho)
        Fb_new = r["Fbar"]
        Lm = L.mean(axis=(1, 2, 3))
        assert np.max(np.abs(Lm[free])) <= 1e-12
        pres = [k for k in range(9) if k not in free]
        rhs = L0.mean(axis=(1, 2, 3)) + rho * (Fb_new - F.mean(axis=(1, 2, 3)))
        assert np.max(np.abs(Lm[pres] - rhs[pres])) <= 1e-12
        assert np.array_equal(Fb_new[pres], Fb[pres])
        Fb = Fb_new


def test_free_mask_is_validated():
    shape = (4, 4, 4)
    phase = np.zeros(shape, np.uint8)
    mats = [O.material("neohooke", mu=1.0, lam=1.0)]
    u, F, L = O.initial_state(shape)
    r = O.admm_run(phase, mats, np.eye(3).ravel(), O.params(max_iter=1, free=[9]), u, F, L, 1.0)
    assert r["rc"] == O.EINVAL
