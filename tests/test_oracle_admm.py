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


def test_inexact_local_step_limits():
    """The inexact local step (Sec. 2.1, local residual held to a fraction of
    r_d): with a vanishing ratio and enough passes it reproduces the exact
    solves; with the paper's ratio 0.3 the iteration still converges to the
    same fixed point, the laminate's exact finite-strain solution."""
    case = M.laminate16_case()
    mats = mats_of(case["materials"])
    Fb = case["loads"][0].ravel()
    newton = O.newton_opts(gtol=1e-14, step_tol=1e-10)
    u0, F0, L0 = O.initial_state(case["phase"].shape)
    p = O.params(max_iter=12, fixed_iters=True, mu_ref=5.5, newton=newton)
    O.admm_run(case["phase"], mats, Fb, p, u0, F0, L0, 5.0)
    u1, F1, L1 = O.initial_state(case["phase"].shape)
    p = O.params(max_iter=12, fixed_iters=True, mu_ref=5.5, newton=newton,
                 local_ratio=1e-30, local_chunk=1, local_passes=60)
    O.admm_run(case["phase"], mats, Fb, p, u1, F1, L1, 5.0)
    assert np.max(np.abs(F1 - F0)) <= 1e-12
    assert np.max(np.abs(u1 - u0)) <= 1e-12 * max(1.0, np.max(np.abs(u0)))
    # ratio 0.3, one Newton iteration per pass: same converged state
    u2, F2, L2 = O.initial_state(case["phase"].shape)
    p = O.params(max_iter=400, tol_p=1e-10, tol_d=1e-10, mu_ref=5.5, newton=newton,
                 local_ratio=0.3, local_chunk=1, local_passes=4)
    r = O.admm_run(case["phase"], mats, Fb, p, u2, F2, L2, 5.0)
    assert r["rc"] == O.OK
    d, Pd = laminate_exact(10.0, 100.0, 1.0, 10.0, 0.95)
    P2 = O.mean_stress(case["phase"], mats, F2)
    assert np.max(np.abs(P2[[0, 4, 8]] - Pd)) <= 1e-8 * np.max(np.abs(Pd))


def test_inexact_parity_cases_are_far_from_ties():
    """The GPU parity cases of the inexact local step compare pass decisions
    (r_l <= ratio r_d, or converged count >= fraction V) taken from sums in
    different orders; on those cases the oracle's result does not move when
    the ratio moves by 1e-9 relative or the fraction by 1.5 voxels, so
    rounding of the sums (or one voxel counted differently) cannot flip a
    decision."""
    from parity_util import oracle_iterations
    from test_gpu_inexact import CASES, N_ITER, inexact_case
    for shape, loc, _ in CASES:
        phase, Fbar, mats, rho, mu_ref = inexact_case(shape, loc)
        V = phase.size
        if "local_ratio" in loc:
            moved = [dict(loc, local_ratio=loc["local_ratio"] * f) for f in (1 + 1e-9, 1 - 1e-9)]
        else:
            moved = [dict(loc, local_fraction=loc["local_fraction"] + f / V) for f in (1.5, -1.5)]
        out = [oracle_iterations(phase, mats, Fbar, N_ITER, rho, mu_ref, **kw)[1]
               for kw in [loc] + moved]
        assert np.array_equal(out[1], out[0]) and np.array_equal(out[2], out[0]), (shape, loc)


def nodal_stress(mats, phase, F, director=None):
    shape = phase.shape
    P = np.empty_like(F)
    for x in np.ndindex(shape):
        n = (0.0, 0.0, 1.0) if director is None else director[(slice(None),) + x]
        P[(slice(None),) + x] = O.stress(mats[phase[x]], F[(slice(None),) + x], n)
    return P


@pytest.mark.parametrize("lce", [False, True])
def test_truncated_local_step_satisfies_the_appendix_identity(lce):
    """One iteration whose Step 1 is cut to one Newton iteration per voxel
    (one pass; the previous r_d is taken huge so the ratio test passes at
    once). With g = W_F(F_{i+1}) - Lambda_i - rho (grad u_i - F_{i+1}) the
    local residual, Steps 2-3 give W_F(F_{i+1}) = g + Lambda_{i+1} -
    rho (grad u_{i+1} - grad u_i), so (the appendix's identity)
    D_h^T W_F(F_{i+1}) = D_h^T g - rho D_h^T (grad u_{i+1} - grad u_i), with g
    far from zero. For the LCE, W_F is the stress at the updated director."""
    shape = (6, 4, 8)
    phase = M.random_two_phase(shape, 0.4, seed=5)
    if lce:
        mats = [O.material("lce", mu=1.0, a=2.0, kappa=50.0),
                O.material("neohooke", mu=10.0, lam=40.0)]
        Fbar = np.diag([1.15, 1.15 ** -0.5, 1.15 ** -0.5]).ravel()
        rng = np.random.default_rng(9)
        d = rng.standard_normal((3,) + shape)
        d /= np.linalg.norm(d, axis=0, keepdims=True)
    else:
        mats = [O.material("neohooke", mu=10.0, lam=40.0), O.material("neohooke", mu=1.0, lam=4.0)]
        Fbar = M.random_fbar(0.08, seed=2).ravel()
        d = None
    rho = 12.0
    u, F, L = O.initial_state(shape)
    O.admm_run(phase, mats, Fbar, O.params(max_iter=2, fixed_iters=True, mu_ref=4.0),
               u, F, L, rho, director_field=d)
    u0, L0 = u.copy(), L.copy()
    p = O.params(max_iter=1, fixed_iters=True, mu_ref=4.0, local_ratio=0.3, local_chunk=1,
                 local_passes=4, local_start_iter=2, local_rd_prev=1e30)
    O.admm_run(phase, mats, Fbar, p, u, F, L, rho, director_field=d)
    P = nodal_stress(mats, phase, F, d)
    G0 = O.gradient(u0, Fbar)
    G1 = O.gradient(u, Fbar)
    g = P - L0 - rho * (G0 - F)
    assert np.max(np.abs(g)) >= 1e-4
    assert np.max(np.abs(div_h(L))) <= 1e-12 * max(1.0, np.max(np.abs(L)))
    lhs = div_h(P)
    rhs = div_h(g) - rho * div_h(G1 - G0)
    assert np.max(np.abs(lhs - rhs)) <= 1e-10 * max(1.0, np.max(np.abs(lhs)))


def test_converged_fraction_strategy_limits():
    """The converged-fraction strategy (Sec. 4: proceed once a given fraction
    of points has converged): fraction 1 with enough passes is the exact
    iteration; fraction 0.5 with two Newton iterations per pass converges to
    the laminate's exact solution."""
    case = M.laminate16_case()
    mats = mats_of(case["materials"])
    Fb = case["loads"][0].ravel()
    newton = O.newton_opts(gtol=1e-14, step_tol=1e-10)
    u0, F0, L0 = O.initial_state(case["phase"].shape)
    O.admm_run(case["phase"], mats, Fb, O.params(max_iter=12, fixed_iters=True, mu_ref=5.5,
                                                 newton=newton), u0, F0, L0, 5.0)
    u1, F1, L1 = O.initial_state(case["phase"].shape)
    p = O.params(max_iter=12, fixed_iters=True, mu_ref=5.5, newton=newton,
                 local_fraction=1.0, local_chunk=1, local_passes=60)
    O.admm_run(case["phase"], mats, Fb, p, u1, F1, L1, 5.0)
    assert np.max(np.abs(F1 - F0)) <= 1e-12
    # one pass of one iteration: far from the exact iteration
    u2, F2, L2 = O.initial_state(case["phase"].shape)
    p = O.params(max_iter=12, fixed_iters=True, mu_ref=5.5, newton=newton,
                 local_fraction=1.0, local_chunk=1, local_passes=1)
    O.admm_run(case["phase"], mats, Fb, p, u2, F2, L2, 5.0)
    assert np.max(np.abs(F2 - F0)) >= 1e-6
    u3, F3, L3 = O.initial_state(case["phase"].shape)
    p = O.params(max_iter=600, tol_p=1e-10, tol_d=1e-10, mu_ref=5.5, newton=newton,
                 local_fraction=0.5, local_chunk=2, local_passes=8)
    r = O.admm_run(case["phase"], mats, Fb, p, u3, F3, L3, 5.0)
    assert r["rc"] == O.OK
    d, Pd = laminate_exact(10.0, 100.0, 1.0, 10.0, 0.95)
    P3 = O.mean_stress(case["phase"], mats, F3)
    assert np.max(np.abs(P3[[0, 4, 8]] - Pd)) <= 1e-8 * np.max(np.abs(Pd))


def test_inexact_options_are_validated():
    shape = (4, 4, 4)
    phase = np.zeros(shape, np.uint8)
    mats = [O.material("neohooke", mu=1.0, lam=1.0)]
    for kw in (dict(local_ratio=-1.0), dict(local_fraction=1.5), dict(local_fraction=-0.1),
               dict(local_ratio=0.3, local_fraction=0.5), dict(local_ratio=0.3, local_chunk=0),
               dict(local_fraction=0.5, local_passes=0)):
        u, F, L = O.initial_state(shape)
        r = O.admm_run(phase, mats, np.eye(3).ravel(), O.params(max_iter=1, **kw), u, F, L, 1.0)
        assert r["rc"] == O.EINVAL, kw


def test_inexact_lce_reaches_the_exact_fixed_point():
    """LCE polydomain with a stiff inclusion under a stretch 1.2: the
    iteration with truncated joint (F, director) solves, r_l held to 0.3 r_d,
    converges to the state the exact iteration converges to."""
    shape = (8, 8, 8)
    g, dirs = M.voronoi_grains(n=8, n_grains=4, seed=3)
    d0 = M.director_field(g, dirs)
    phase = np.zeros(shape, np.uint8)
    z, y, x = np.indices(shape)
    phase[(x - 3.5) ** 2 + (y - 3.5) ** 2 + (z - 3.5) ** 2 <= 4.0] = 1
    mats = [O.material("lce", mu=1.0, a=2.0, kappa=50.0), O.material("neohooke", mu=10.0, lam=40.0)]
    Fbar = np.diag([1.2, 1.2 ** -0.5, 1.2 ** -0.5]).ravel()
    newton = O.newton_opts(gtol=1e-14, step_tol=1e-10)
    out = []
    for loc in ({}, dict(local_ratio=0.3, local_chunk=1, local_passes=4)):
        u, F, L = O.initial_state(shape)
        d = d0.copy()
        p = O.params(max_iter=3000, tol_p=1e-9, tol_d=1e-9, mu_ref=1.0, newton=newton,
                     adapt_rho=True, rho_min=1.0, rho_max=100.0, **loc)
        r = O.admm_run(phase, mats, Fbar, p, u, F, L, 10.0, director_field=d)
        assert r["rc"] == O.OK, loc
        out.append((F, d, O.mean_stress(phase, mats, F, director_field=d)))
    assert np.max(np.abs(out[1][0] - out[0][0])) <= 1e-7
    assert np.max(np.abs(np.einsum("i...,j...->ij...", out[1][1], out[1][1])
                         - np.einsum("i...,j...->ij...", out[0][1], out[0][1]))) <= 1e-7
    assert np.max(np.abs(out[1][2] - out[0][2])) <= 1e-8


def test_composed_parity_case_is_far_from_ties():
    """The inexact step's pass decisions in the composed GPU parity case
    (LCE full model, uniaxial stress) do not move when the ratio moves by
    1e-9 relative."""
    from parity_util import NEWTON64, omats
    from test_gpu_compose import CELLS, LOC, MATS
    (phase, d0), Fb, free = CELLS[0]
    out = []
    for f in (1.0, 1 + 1e-9, 1 - 1e-9):
        u, F, L = O.initial_state(phase.shape)
        n = d0.copy()
        op = O.params(max_iter=10, fixed_iters=True, mu_ref=1.0, dt=0.5, free=free,
                      newton=O.newton_opts(**NEWTON64), **dict(LOC, local_ratio=LOC["local_ratio"] * f))
        O.admm_run(phase, omats(MATS), Fb.ravel(), op, u, F, L, 10.0, director_field=n,
                   director0=d0)
        out.append(F)
    assert np.array_equal(out[1], out[0]) and np.array_equal(out[2], out[0])


def test_resume_is_bitwise():
    """Algorithm 1 carries (u, F, Lambda, the director, rho) from one
    iteration to the next: a run of 7 iterations continued from its output
    state for 5 more equals a run of 12 bit for bit (adaptive penalty, LCE
    director), and the ratio strategy of the inexact step continues with its
    iteration index and previous r_d."""
    shape = (8, 6, 4)
    g, dirs = M.voronoi_grains(n=8, n_grains=3, seed=5)
    phase = np.zeros(shape, np.uint8)
    phase[:, :, :3] = 1
    d0 = M.director_field(g, dirs)[:, :8, :6, :4]
    d0 = np.ascontiguousarray(d0)
    mats = [O.material("lce", mu=1.0, a=2.0, kappa=20.0), O.material("neohooke", mu=5.0, lam=20.0)]
    Fbar = np.diag([1.1, 1.1 ** -0.5, 1.1 ** -0.5]).ravel()
    newton = O.newton_opts(gtol=1e-14, step_tol=1e-10)
    for loc in ({}, dict(local_ratio=0.3, local_chunk=1, local_passes=3)):
        mk = dict(fixed_iters=True, mu_ref=1.0, newton=newton, adapt_rho=True, rho_min=1.0,
                  rho_max=100.0, **loc)
        u, F, L = O.initial_state(shape)
        d = d0.copy()
        whole = O.admm_run(phase, mats, Fbar, O.params(max_iter=12, **mk), u, F, L, 3.0,
                           director_field=d)
        u2, F2, L2 = O.initial_state(shape)
        d2 = d0.copy()
        first = O.admm_run(phase, mats, Fbar, O.params(max_iter=7, **mk), u2, F2, L2, 3.0,
                           director_field=d2)
        more = dict(mk)
        if loc:
            more.update(local_start_iter=7, local_rd_prev=first["r_d"][-1])
        second = O.admm_run(phase, mats, Fbar, O.params(max_iter=5, **more), u2, F2, L2,
                            first["rho"], director_field=d2)
        for a, b in ((u, u2), (F, F2), (L, L2), (d, d2)):
            assert np.array_equal(a, b), loc
        assert whole["rho"] == second["rho"]
        assert np.array_equal(whole["r_p"], np.concatenate([first["r_p"], second["r_p"]]))
        assert np.array_equal(whole["r_d"], np.concatenate([first["r_d"], second["r_d"]]))
