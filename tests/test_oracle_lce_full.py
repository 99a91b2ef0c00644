"""Pins of the oracle's full LCE model (Sec. 5.1): the non-ideality
W_ni = mu alpha/2 tr((I - n0 n0) F^T (n n) F), the Frank term with the
neighbours' directors lagged (the second approach of Sec. 2.1 for gradients
of internal variables), the dissipation of F and of the director, and the
orientation tensor.

With the director terms written as a quadratic form n . M(F) n, every check
here builds M in numpy from the energies as the paper states them and uses
numpy's eigensolver, not the oracle's:
  * the oracle's energy is the stated sum of terms;
  * the relaxed director minimises n . M n (brute force and eigh);
  * the relaxed stress and tangent are the central differences of
    W_iso + lambda_min(M(F)) and of that stress;
  * the converged state of a small polydomain with all terms on satisfies the
    Euler-Lagrange equations of the time-discrete energy: every director is
    the minimising eigenvector of M built from the converged neighbours, and
    D_h^T (P + nu_F/dt (F - F^n)) = 0;
  * the orientation tensor of uniform and split director fields.
"""
import numpy as np
import pytest

import oracle as O
from paper_2010_06697_amd import microstructure as M
from test_oracle_admm import div_h
from test_oracle_material import randF, unit

MU, A_, KAPPA = 1.0, 2.0, 50.0


def mat(alpha=0.0, frank=0.0, nu_F=0.0, nu_n=0.0):
    return O.material("lce", mu=MU, a=A_, kappa=KAPPA, alpha=alpha, frank=frank, nu_F=nu_F,
                      nu_n=nu_n)


def W_iso(F):
    F = F.reshape(3, 3)
    J = np.linalg.det(F)
    return 0.5 * MU * (A_ ** (1 / 3) * np.sum(F * F) - 3.0) + 0.5 * KAPPA * (J - 1.0) ** 2


def M_form(F, alpha, n0, Sc):
    F = F.reshape(3, 3)
    P0 = np.eye(3) - np.outer(n0, n0)
    return (0.5 * MU * A_ ** (1 / 3) * (1 / A_ - 1) * F @ F.T + 0.5 * MU * alpha * F @ P0 @ F.T
            + Sc.reshape(3, 3))


def W_relaxed_np(F, alpha, n0, Sc):
    return W_iso(F) + np.linalg.eigvalsh(M_form(F, alpha, n0, Sc))[0]


def cases():
    rng = np.random.default_rng(3)
    out = []
    for k in range(4):
        F = (np.diag([1.25, 0.92, 0.9]) + 0.08 * rng.standard_normal((3, 3))).ravel()
        n0 = unit(k + 30)
        S = rng.standard_normal((3, 3)) * 0.2
        out.append((F, 0.3 if k % 2 == 0 else 0.05, n0, 0.5 * (S + S.T)))
    return out


@pytest.mark.parametrize("k", range(4))
def test_energy_is_the_sum_of_the_stated_terms(k):
    F, alpha, n0, Sc = cases()[k]
    n = unit(k + 7)
    W = O.energy(mat(alpha), F, n, nref=n0, Sc=Sc)
    Fm = F.reshape(3, 3)
    ref = (W_iso(F) + 0.5 * MU * A_ ** (1 / 3) * (1 / A_ - 1) * np.sum((Fm.T @ n) ** 2)
           + 0.5 * MU * alpha * np.trace((np.eye(3) - np.outer(n0, n0)) @ Fm.T @ np.outer(n, n) @ Fm)
           + n @ Sc @ n)
    assert abs(W - ref) <= 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("k", range(4))
def test_relaxed_director_stress_and_tangent(k):
    F, alpha, n0, Sc = cases()[k]
    m = mat(alpha)
    n, P, K = O.relaxed(m, F, unit(k), nref=n0, Sc=Sc)
    Mf = M_form(F, alpha, n0, Sc)
    w, V = np.linalg.eigh(Mf)
    assert abs(abs(V[:, 0] @ n) - 1.0) <= 1e-12
    rng = np.random.default_rng(k)
    trial = rng.standard_normal((3000, 3))
    trial /= np.linalg.norm(trial, axis=1, keepdims=True)
    e0 = O.energy(m, F, n, nref=n0, Sc=Sc)
    assert min(O.energy(m, F, t, nref=n0, Sc=Sc) for t in trial) >= e0 - 1e-13
    h = 1e-6
    Pfd = np.array([(W_relaxed_np(F + h * e, alpha, n0, Sc) - W_relaxed_np(F - h * e, alpha, n0, Sc))
                    / (2 * h) for e in np.eye(9)])
    assert np.max(np.abs(P - Pfd)) <= 1e-7 * max(1.0, np.max(np.abs(P)))
    Kfd = np.stack([(O.relaxed(m, F + h * e, n, nref=n0, Sc=Sc)[1]
                     - O.relaxed(m, F - h * e, n, nref=n0, Sc=Sc)[1]) / (2 * h) for e in np.eye(9)],
                   axis=1)
    assert np.max(np.abs(K - Kfd)) <= 1e-6 * np.max(np.abs(K))
    assert np.max(np.abs(K - K.T)) <= 1e-12 * np.max(np.abs(K))


def test_ideal_terms_with_a_site_change_nothing():
    F = randF(2, 0.2).ravel()
    m = mat(0.0)
    a = O.relaxed(m, F, unit(1))
    b = O.relaxed(m, F, unit(1), nref=unit(4), Sc=np.zeros(9))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    with pytest.raises(ValueError):  # a = 1 has no director term to scale by
        O.relaxed(O.material("lce", mu=1.0, a=1.0, kappa=1.0, alpha=0.1), F, unit(1),
                  nref=unit(4))


def polydomain_case():
    g, dirs = M.voronoi_grains(n=8, n_grains=4, seed=3)
    d0 = M.director_field(g, dirs)
    shape = g.shape
    phase = np.zeros(shape, np.uint8)
    z, y, x = np.indices(shape)
    phase[(x - 3.5) ** 2 + (y - 3.5) ** 2 + (z - 3.5) ** 2 <= 4.0] = 1
    return phase, d0


def neighbour_form(d, phase, lce_phases, x):
    n3, n2, n1 = phase.shape
    k3, k2, k1 = x
    S = np.zeros((3, 3))
    for dk in ((0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)):
        y = ((k3 + dk[0]) % n3, (k2 + dk[1]) % n2, (k1 + dk[2]) % n1)
        if phase[y] in lce_phases:
            v = d[(slice(None),) + y]
            S += np.outer(v, v)
    return S


def test_converged_state_satisfies_the_time_discrete_euler_lagrange_equations():
    """Polydomain LCE (8^3, 4 grains) with a stiff inclusion, one time step
    of a stretch 1.2 with alpha, the Frank term and both dissipations on."""
    phase, d0 = polydomain_case()
    alpha, frank, nu_F, nu_n, dt = 0.1, 0.05, 0.2, 0.3, 0.5
    mats = [mat(alpha, frank, nu_F, nu_n), O.material("neohooke", mu=10.0, lam=40.0)]
    Fbar = np.diag([1.2, 1.2 ** -0.5, 1.2 ** -0.5]).ravel()
    u, F, L = O.initial_state(phase.shape)
    d = d0.copy()
    F_n, d_n = F.copy(), d.copy()
    p = O.params(max_iter=4000, tol_p=1e-11, tol_d=1e-11, mu_ref=1.0, adapt_rho=True,
                 rho_min=1.0, rho_max=100.0, dt=dt, newton=O.newton_opts(gtol=1e-14, step_tol=1e-10))
    r = O.admm_run(phase, mats, Fbar, p, u, F, L, 10.0, director_field=d, director0=d0)
    assert r["rc"] == O.OK, r["iters"]
    # equilibrium with the dissipative stress: D_h^T (P + nu_F/dt (F - F^n)) = 0
    P = np.empty_like(F)
    for x in np.ndindex(phase.shape):
        sl = (slice(None),) + x
        nref = d0[sl] if phase[x] == 0 else None
        P[sl] = O.stress(mats[phase[x]], F[sl], d[sl], nref=nref)
    Ptot = P + nu_F / dt * (F - F_n) * (phase == 0)   # the inclusion is not dissipative
    assert np.max(np.abs(div_h(Ptot))) <= 1e-8
    # every LCE director minimises n . M n, M from the converged neighbours
    worst = 0.0
    for x in np.ndindex(phase.shape):
        if phase[x] != 0:
            continue
        sl = (slice(None),) + x
        Sc = -frank * neighbour_form(d, phase, (0,), x) - 0.5 * nu_n / dt * np.outer(d_n[sl], d_n[sl])
        w, V = np.linalg.eigh(M_form(F[sl], alpha, d0[sl], Sc))
        assert w[1] - w[0] > 1e-8
        worst = max(worst, 1.0 - abs(V[:, 0] @ d[sl]))
    assert worst <= 1e-9
    # and the terms matter: without them the state differs
    u2, F2, L2 = O.initial_state(phase.shape)
    d2 = d0.copy()
    O.admm_run(phase, [mat(), mats[1]], Fbar, p, u2, F2, L2, 10.0, director_field=d2)
    assert np.max(np.abs(F2 - F)) >= 1e-3


def test_orientation_tensor():
    shape = (4, 4, 4)
    phase = np.zeros(shape, np.uint8)
    mats = [mat(), O.material("neohooke", mu=1.0, lam=1.0)]
    d = np.zeros((3,) + shape)
    n = unit(9)
    d[:] = n[:, None, None, None]
    S = O.orientation(phase, mats, d)
    assert np.max(np.abs(S - 1.5 * (np.outer(n, n) - np.eye(3) / 3))) <= 1e-14
    d[:] = 0.0
    d[0, :, :, :2] = 1.0
    d[1, :, :, 2:] = 1.0
    assert np.max(np.abs(O.orientation(phase, mats, d) - np.diag([0.25, 0.25, -0.5]))) <= 1e-15
    phase[:, :, 2:] = 1   # neo-Hookean voxels do not count
    assert np.max(np.abs(O.orientation(phase, mats, d) - np.diag([1.0, -0.5, -0.5]))) <= 1e-15
