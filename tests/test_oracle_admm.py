"""Pins of the oracle's whole ADMM iteration (Steps 1-4 of Sec. 2.1).

The converged fixed point of the iteration is the minimiser of the discrete
energy sum_x W(Fbar + D_h u(x)) (given exact local solves and the D_h^T D_h
Laplacian). What pins the oracle here, independently of its own code:
  * a homogeneous body under affine load: zero fluctuation at every
    iteration, F -> Fbar, Lambda -> P(Fbar) (Lambda converges to the stress,
    Sec. 2.1 "Connection to physics");
  * the finite-strain two-phase laminate, whose exact solution is a scalar
    root (solved here with scipy's brentq), and its small-strain limit, the
    classical closed-form laminate moduli;
  * brute-force minimisation of the discrete energy on a 4^3 grid by a dense
    Newton method written here in numpy;
  * algebraic invariants of the updates: D_h^T Lambda = 0 after every update,
    the mean of Lambda, and the weak equilibrium identity of the appendix
    D_h^T P(F_{i+1}) = -rho D_h^T (grad u_{i+1} - grad u_i);
  * independence of the converged fixed point from rho.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

import oracle as O
from paper_2010_06697_amd import microstructure as M
from test_oracle_grid import cdiff


def mats_of(defs):
    return [O.material(d["model"], mu=d["mu"], lam=d["lam"], a=d["a"], kappa=d["kappa"])
            for d in defs]


def div_h(S):
    """D_h^T of a tensor field: -sum_j d_j S_ij."""
    return np.stack([-sum(cdiff(S[3 * i + j], j) for j in range(3)) for i in range(3)])


def test_homogeneous_body_has_zero_fluctuation():
    shape = (4, 6, 8)
    phase = np.zeros(shape, np.uint8)
    mats = [O.material("neohooke", mu=3.0, lam=20.0)]
    Fbar = M.random_fbar(0.05, seed=1).ravel()
    u, F, L = O.initial_state(shape)
    p1 = O.params(max_iter=1, fixed_iters=True, mu_ref=3.0)
    rho = 8.0
    for _ in range(6):
        O.admm_run(phase, mats, Fbar, p1, u, F, L, rho)
        assert np.max(np.abs(u)) <= 1e-14
    p = O.params(max_iter=500, tol_p=1e-13, tol_d=1e-13, mu_ref=3.0)
    r = O.admm_run(phase, mats, Fbar, p, u, F, L, rho)
    assert r["rc"] == O.OK
    assert np.max(np.abs(u)) <= 1e-14
    PF = O.stress(mats[0], Fbar)
    assert np.max(np.abs(F - Fbar[:, None, None, None])) <= 1e-12
    assert np.max(np.abs(L - PF[:, None, None, None])) <= 1e-11
    Pm = O.mean_stress(phase, mats, F)
    assert np.max(np.abs(Pm - PF)) <= 1e-10 * np.max(np.abs(PF))


def laminate_exact(mu_s, lam_s, mu_f, lam_f, f33):
    """F_alpha = diag(1 +- d, 1, f33): the stiff/soft layers share P_11."""
    def P(f1, mu, lam):
        J = f1 * f33
        lj = np.log(J)
        return np.array([mu * (f1 - 1 / f1) + lam * lj / f1, lam * lj,
                         mu * (f33 - 1 / f33) + lam * lj / f33])
    d = brentq(lambda d: P(1 + d, mu_s, lam_s)[0] - P(1 - d, mu_f, lam_f)[0], -0.5, 0.5,
               xtol=1e-17, rtol=1e-15, maxiter=500)
    return d, 0.5 * (P(1 + d, mu_s, lam_s) + P(1 - d, mu_f, lam_f))


def test_laminate16_matches_exact_finite_strain_solution():
    case = M.laminate16_case()
    mats = mats_of(case["materials"])
    phase = case["phase"]
    Fbar = case["loads"][0].ravel()
    u, F, L = O.initial_state(phase.shape)
    p = O.params(max_iter=3000, tol_p=1e-12, tol_d=1e-12, mu_ref=case["mu_ref"])
    r = O.admm_run(phase, mats, Fbar, p, u, F, L, case["rho0"])
    assert r["rc"] == O.OK and r["newton_fail"] == 0
    d, Pd = laminate_exact(10.0, 100.0, 1.0, 10.0, 0.95)
    Pm = O.mean_stress(phase, mats, F)
    assert np.max(np.abs(Pm - np.diag(Pd).ravel())) <= 1e-10 * np.max(np.abs(Pd))
    assert abs(F[0, 0, 0, 0] - (1 + d)) <= 1e-10 and abs(F[0, 0, 0, 15] - (1 - d)) <= 1e-10
    # the multiplier converges to the stress (Sec. 2.1, "Connection to physics")
    Pfield = np.stack([O.stress(mats[phase[0, 0, k]], F[:, 0, 0, k]) for k in range(16)], 1)
    assert np.max(np.abs(L[:, 0, 0, :] - Pfield)) <= 1e-9


def backus(f, mu, lam, eps):
    """Closed-form effective stress of a linear-elastic laminate normal to e1."""
    f, mu, lam = map(np.asarray, (f, mu, lam))
    Mm = lam + 2 * mu
    av = lambda q: np.sum(f * q)
    s = np.zeros((3, 3))
    s[0, 0] = (eps[0, 0] + av(lam / Mm) * (eps[1, 1] + eps[2, 2])) / av(1 / Mm)
    for a in (1, 2):
        s[a, a] = (av(lam / Mm) * s[0, 0] + av(2 * lam * mu / Mm) * (eps[1, 1] + eps[2, 2])
                   + 2 * av(mu) * eps[a, a])
    s[0, 1] = s[1, 0] = 2 * eps[0, 1] / av(1 / mu)
    s[0, 2] = s[2, 0] = 2 * eps[0, 2] / av(1 / mu)
    s[1, 2] = s[2, 1] = 2 * av(mu) * eps[1, 2]
    return s


def test_laminate_small_strain_limit_matches_closed_form_moduli():
    shape = (4, 4, 8)
    phase = M.laminate(shape=shape, n_stiff=4)
    mats = [O.material("neohooke", mu=6.0, lam=15.0), O.material("neohooke", mu=1.0, lam=4.0)]
    rng = np.random.default_rng(4)
    Hh = rng.uniform(-1, 1, (3, 3))
    delta = 1e-5
    Fbar = (np.eye(3) + delta * Hh).ravel()
    u, F, L = O.initial_state(shape)
    p = O.params(max_iter=4000, tol_p=1e-14, tol_d=1e-14, mu_ref=3.5)
    r = O.admm_run(phase, mats, Fbar, p, u, F, L, 5.0)
    assert r["rc"] == O.OK
    Pm = O.mean_stress(phase, mats, F).reshape(3, 3)
    ref = backus([0.5, 0.5], [6.0, 1.0], [15.0, 4.0], 0.5 * (Hh + Hh.T))
    assert np.max(np.abs(Pm / delta - ref)) <= 1e-4 * np.max(np.abs(ref))


# ---- brute-force minimisation of the discrete energy -----------------------

def nh_stress(F, mu, lam):
    """numpy neo-Hookean P = mu (F - F^-T) + lam ln J F^-T, F: (..., 3, 3)."""
    Fit = np.linalg.inv(F).swapaxes(-1, -2)
    lj = np.log(np.linalg.det(F))[..., None, None]
    return mu[..., None, None] * (F - Fit) + lam[..., None, None] * lj * Fit


def test_admm_fixed_point_is_the_discrete_energy_minimiser():
    shape = (4, 4, 4)
    phase = M.random_two_phase(shape, 0.5, seed=3)
    mu_t = np.array([10.0, 1.0])
    lam_t = np.array([30.0, 3.0])
    mu, lam = mu_t[phase], lam_t[phase]
    Fbar = np.eye(3) + np.array([[0.02, 0.01, -0.01], [0.0, -0.03, 0.02], [0.01, 0.0, 0.01]])

    def field_F(uf):
        G = np.stack([cdiff(uf[i], j) for i in range(3) for j in range(3)])
        return np.moveaxis(G, 0, -1).reshape(shape + (3, 3)) + Fbar

    def grad_E(x):
        Fx = field_F(x.reshape((3,) + shape))
        P = nh_stress(Fx, mu, lam)
        S = np.moveaxis(P.reshape(shape + (9,)), -1, 0)
        return div_h(S).ravel()

    x = np.zeros(3 * 64)
    for _ in range(30):
        g = grad_E(x)
        if np.linalg.norm(g) < 1e-13:
            break
        h = 1e-6
        Hm = np.stack([(grad_E(x + h * e) - grad_E(x - h * e)) / (2 * h) for e in np.eye(x.size)], 1)
        x -= np.linalg.lstsq(0.5 * (Hm + Hm.T), g, rcond=1e-10)[0]
    assert np.linalg.norm(grad_E(x)) < 1e-12
    Fbf = np.moveaxis(field_F(x.reshape((3,) + shape)).reshape(shape + (9,)), -1, 0)

    mats = [O.material("neohooke", mu=10.0, lam=30.0), O.material("neohooke", mu=1.0, lam=3.0)]
    u, F, L = O.initial_state(shape)
    p = O.params(max_iter=5000, tol_p=1e-13, tol_d=1e-13, mu_ref=5.5)
    r = O.admm_run(phase, mats, Fbar.ravel(), p, u, F, L, 10.0)
    assert r["rc"] == O.OK
    assert np.max(np.abs(F - Fbf)) <= 1e-9


def test_update_invariants_and_weak_equilibrium():
    shape = (6, 4, 8)
    phase = M.random_two_phase(shape, 0.4, seed=5)
    mats = [O.material("neohooke", mu=10.0, lam=40.0), O.material("neohooke", mu=1.0, lam=4.0)]
    Fbar = M.random_fbar(0.04, seed=2).ravel()
    u, F, L = O.initial_state(shape)
    rho = 12.0
    p1 = O.params(max_iter=1, fixed_iters=True, mu_ref=4.0)
    for it in range(8):
        u0, L0 = u.copy(), L.copy()
        O.admm_run(phase, mats, Fbar, p1, u, F, L, rho)
        assert np.max(np.abs(div_h(L))) <= 1e-12 * max(1.0, np.max(np.abs(L)))
        lhs = L.mean(axis=(1, 2, 3))
        rhs = L0.mean(axis=(1, 2, 3)) + rho * (Fbar - F.mean(axis=(1, 2, 3)))
        assert np.max(np.abs(lhs - rhs)) <= 1e-12
        P = np.stack([np.stack([O.stress(mats[phase[x]], F[:, x[0], x[1], x[2]])
                                for x in np.ndindex(shape)], 1).reshape((9,) + shape)])[0]
        G1 = O.gradient(u, Fbar)
        G0 = O.gradient(u0, Fbar)
        weak = div_h(P) + rho * div_h(G1 - G0)
        assert np.max(np.abs(weak)) <= 1e-10


def test_converged_fixed_point_does_not_depend_on_rho():
    shape = (4, 4, 6)
    phase = M.random_two_phase(shape, 0.5, seed=8)
    mats = [O.material("neohooke", mu=5.0, lam=20.0), O.material("neohooke", mu=1.0, lam=4.0)]
    Fbar = M.random_fbar(0.03, seed=3).ravel()
    out = []
    for rho in (4.0, 10.0, 30.0):
        u, F, L = O.initial_state(shape)
        p = O.params(max_iter=8000, tol_p=1e-13, tol_d=1e-13, mu_ref=3.0)
        r = O.admm_run(phase, mats, Fbar, p, u, F, L, rho)
        assert r["rc"] == O.OK
        out.append(F)
    assert np.max(np.abs(out[0] - out[1])) <= 1e-10
    assert np.max(np.abs(out[0] - out[2])) <= 1e-10


def test_residual_definitions_and_adaptive_penalty():
    """Step 4: r_p = |grad u_{i+1} - F_{i+1}|, r_d = rho/mu |grad u_{i+1} - grad u_i|
    (RMS over voxels of the Frobenius norm), recomputed here from the states with
    a stencil of this file; then the adaptive rule of Sec. 2.1 applied to the
    recorded residuals must reproduce the recorded rho sequence."""
    shape = (4, 6, 8)
    phase = M.random_two_phase(shape, 0.5, seed=12)
    mats = [O.material("neohooke", mu=20.0, lam=60.0), O.material("neohooke", mu=1.0, lam=3.0)]
    Fbar = M.random_fbar(0.04, seed=6).ravel()
    u, F, L = O.initial_state(shape)
    mu_ref = 7.0
    p1 = O.params(max_iter=1, fixed_iters=True, mu_ref=mu_ref, adapt_rho=True, rho_min=1.0,
                  rho_max=50.0, kappa_rho=1.3, tau=10.0)
    branches = set()
    for it in range(24):
        if it in (0, 12):  # restart from a large and then from a small penalty
            u, F, L = O.initial_state(shape)
            rho = 40.0 if it == 0 else 1.0
        u0 = u.copy()
        r = O.admm_run(phase, mats, Fbar, p1, u, F, L, rho)
        G1 = np.stack([cdiff(u[i], j) for i in range(3) for j in range(3)]) + Fbar[:, None, None, None]
        G0 = np.stack([cdiff(u0[i], j) for i in range(3) for j in range(3)]) + Fbar[:, None, None, None]
        rp = np.sqrt(np.mean(np.sum((G1 - F) ** 2, axis=0)))
        rd = rho / mu_ref * np.sqrt(np.mean(np.sum((G1 - G0) ** 2, axis=0)))
        assert abs(r["r_p"][0] - rp) <= 1e-12 * rp and abs(r["r_d"][0] - rd) <= 1e-12 * rd
        expect = rho
        if rp / rd > 10.0:
            expect = 1.3 * rho
        elif rd / rp > 10.0:
            expect = max(rho / 1.3, 1.0)
        expect = min(expect, 50.0)
        branches.add("up" if expect > rho else ("down" if expect < rho else "keep"))
        assert abs(r["rho"] - expect) <= 1e-15 * expect
        rho = r["rho"]
    assert {"up", "down"} <= branches


def test_adaptive_penalty_recovers_from_a_poor_start():
    """Sec. 4.2: adaptive rho converges in far fewer iterations than a poor fixed rho."""
    case = M.laminate16_case()
    mats = mats_of(case["materials"])
    phase = case["phase"]
    Fbar = case["loads"][0].ravel()
    iters = {}
    for adapt in (False, True):
        u, F, L = O.initial_state(phase.shape)
        p = O.params(max_iter=3000, tol_p=1e-8, tol_d=1e-8, mu_ref=5.5, adapt_rho=adapt,
                     rho_min=1.0, rho_max=1000.0, kappa_rho=1.3, tau=10.0)
        r = O.admm_run(phase, mats, Fbar, p, u, F, L, 500.0)
        assert r["rc"] == O.OK
        iters[adapt] = r["iters"]
    assert iters[True] < 0.5 * iters[False]
