"""Pins of the oracle's LCE local problem with the director eliminated.

The local step of Sec. 2.1 for the LCE of Sec. 5.1 minimises over F and the
unit director jointly. For a >= 1 the director part of the neo-classical
energy, mu a^(1/3)/2 (1/a - 1) |F^T n|^2, is smallest at the top eigenvector of
F F^T, so the joint minimisation is a minimisation over F of the relaxed
energy W_r(F) = min_n W(F, n). Pins, none of which uses the oracle's eigen
solver or its formula for the eigenvector sensitivity:
- the director it picks beats every other unit vector (brute force over
  random directions and a local search over angles) and agrees with numpy's
  symmetric eigensolver;
- its stress is the gradient of W_r, W_r evaluated through numpy's
  eigensolver (central differences);
- its tangent is the derivative of that stress (central differences), is
  symmetric, and lies below the fixed-director tangent by a negative
  semidefinite term of rank <= 2;
- the joint prox is stationary, beats joint perturbations of F and n, and
  equals an independent minimisation of W_r(F) + rho/2 |F - A|^2 by scipy's
  BFGS with W_r from numpy.
The oracle solves the ideal model (no site terms) in the singular basis of
A (three unknowns) and every other LCE form by Newton's method on the nine
components of F; both paths are held to the pins above, and the two paths
agree on the ideal model where a zero site sends it down the second.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
from test_oracle_material import randF, rot, unit

LCE = O.material("lce", mu=1.0, a=2.0, kappa=100.0)


def top_vec(F):
    w, V = np.linalg.eigh(F.reshape(3, 3) @ F.reshape(3, 3).T)
    return V[:, -1]


def W_relaxed_np(F):
    """min over unit n of W(F, n), the minimising n taken from numpy."""
    return O.energy(LCE, F, top_vec(F))


def F_cases():
    out = [randF(s, 0.2).ravel() for s in range(3)]
    out.append(np.diag([1.3, 1.3 ** -0.5, 1.3 ** -0.5]).ravel())
    out.append((rot(4) @ np.diag([1.1, 1.0, 0.95]) @ rot(5)).ravel())
    return out


@pytest.mark.parametrize("k", range(5))
def test_director_minimises_over_the_sphere(k):
    F = F_cases()[k]
    n, _, _ = O.relaxed(LCE, F, unit(k))
    assert abs(np.linalg.norm(n) - 1.0) <= 1e-15
    w0 = O.energy(LCE, F, n)
    rng = np.random.default_rng(k)
    trial = rng.standard_normal((2000, 3))
    trial /= np.linalg.norm(trial, axis=1, keepdims=True)
    assert min(O.energy(LCE, F, t) for t in trial) >= w0 - 1e-13

    def by_angles(x):
        t = np.array([np.sin(x[0]) * np.cos(x[1]), np.sin(x[0]) * np.sin(x[1]), np.cos(x[0])])
        return O.energy(LCE, F, t)

    best = min(minimize(by_angles, x0, method="Nelder-Mead",
                        options={"xatol": 1e-10, "fatol": 1e-15}).fun
               for x0 in rng.uniform(0, np.pi, (6, 2)))
    assert best >= w0 - 1e-12
    assert abs(abs(top_vec(F) @ n) - 1.0) <= 1e-13


@pytest.mark.parametrize("k", range(5))
def test_relaxed_stress_and_tangent_by_finite_differences(k):
    F = F_cases()[k]
    n, P, K = O.relaxed(LCE, F, unit(k))
    h = 1e-6
    Pfd = np.array([(W_relaxed_np(F + h * e) - W_relaxed_np(F - h * e)) / (2 * h)
                    for e in np.eye(9)])
    assert np.max(np.abs(P - Pfd)) <= 1e-7 * max(1.0, np.max(np.abs(P)))
    Kfd = np.stack([(O.relaxed(LCE, F + h * e, n)[1] - O.relaxed(LCE, F - h * e, n)[1]) / (2 * h)
                    for e in np.eye(9)], axis=1)
    assert np.max(np.abs(K - Kfd)) <= 1e-6 * np.max(np.abs(K))
    assert np.max(np.abs(K - K.T)) <= 1e-12 * np.max(np.abs(K))
    # softer than the fixed-director tangent, by a rank <= 2 term
    D = K - O.tangent(LCE, F, n).reshape(9, 9)
    ev = np.linalg.eigvalsh(0.5 * (D + D.T))
    assert ev.max() <= 1e-12 * np.max(np.abs(K))
    assert np.sum(np.abs(ev) > 1e-10 * np.max(np.abs(K))) <= 2


def test_relaxed_at_a1_reduces_to_fixed_director():
    m1 = O.material("lce", mu=2.0, a=1.0, kappa=5.0)
    F = randF(7, 0.2).ravel()
    n, P, K = O.relaxed(m1, F, unit(7))
    assert np.max(np.abs(K - O.tangent(m1, F, n).reshape(9, 9))) <= 1e-13 * np.max(np.abs(K))
    with pytest.raises(ValueError):
        O.relaxed(O.material("lce", mu=1.0, a=0.5, kappa=1.0), F, unit(7))


def phi_np(F, A, rho):
    return W_relaxed_np(F) + 0.5 * rho * np.sum((F - A) ** 2)


@pytest.mark.parametrize("path", ["spectral", "newton"])
@pytest.mark.parametrize("case", ["stretch", "random", "rotated"])
def test_joint_prox_is_the_minimiser(case, path):
    rho = 10.0
    if case == "stretch":
        A = np.diag([1.25, 0.9, 0.9]) + 0.02 * np.random.default_rng(1).standard_normal((3, 3))
        F0, n0 = np.eye(3).ravel(), unit(2)
    elif case == "random":
        A = randF(3, 0.15)
        F0, n0 = np.eye(3).ravel(), unit(4)
    else:
        A = rot(5) @ np.diag([1.3, 0.88, 0.88]) @ rot(6)
        F0, n0 = A.ravel() + 0.01, unit(7)
    F, n, it, rc = O.prox(LCE, rho, A.ravel(), F0, n0, **PATHS[path])
    assert rc == O.OK and it <= 25, (rc, it)
    # stationary, with the director the top eigenvector of F F^T
    g = O.stress(LCE, F, n) + rho * (F - A.ravel())
    assert np.linalg.norm(g) <= 1e-10
    assert abs(abs(top_vec(F) @ n) - 1.0) <= 1e-12
    # no joint perturbation of (F, n) does better
    f0 = O.energy(LCE, F, n) + 0.5 * rho * np.sum((F - A.ravel()) ** 2)
    rng = np.random.default_rng(11)
    for _ in range(50):
        dF = 1e-3 * rng.standard_normal(9)
        nt = n + 1e-2 * rng.standard_normal(3)
        nt /= np.linalg.norm(nt)
        assert O.energy(LCE, F + dF, nt) + 0.5 * rho * np.sum((F + dF - A.ravel()) ** 2) >= f0 - 1e-13
    # an independent minimisation of the relaxed objective lands on the same F
    res = minimize(phi_np, F, args=(A.ravel(), rho), method="BFGS",
                   options={"gtol": 1e-11, "maxiter": 500})
    assert res.fun >= f0 - 1e-13
    assert np.max(np.abs(res.x - F)) <= 1e-6


def test_joint_prox_converges_quadratically_in_the_convex_regime():
    """Well-separated top eigenvalue: a handful of Newton steps from F = I,
    where the alternation of F and director solves needs many."""
    rho = 10.0
    A = np.diag([1.2, 1.2 ** -0.5, 1.2 ** -0.5]).ravel()
    for s in range(4):
        F, n, it, rc = O.prox(LCE, rho, A, np.eye(3).ravel(), unit(s + 20))
        assert rc == O.OK and it <= 12, (s, it)
        assert abs(abs(n[0]) - 1.0) <= 1e-10


def test_joint_prox_covariance():
    rho = 10.0
    for s in range(3):
        A = randF(s, 0.15)
        n0 = unit(s + 3)
        F, n, _, rc = O.prox(LCE, rho, A.ravel(), np.eye(3).ravel(), n0)
        assert rc == O.OK
        Q = rot(s + 9)
        # the warm start rotates with the data: the problem is not convex
        # everywhere, so prox(QA) = Q prox(A) holds for the same local minimiser
        FQ, nQ, _, rcQ = O.prox(LCE, rho, (Q @ A).ravel(), Q.ravel(), Q @ n0)
        assert rcQ == O.OK
        assert np.max(np.abs(FQ.reshape(3, 3) - Q @ F.reshape(3, 3))) <= 1e-9
        # n and -n are the same state (Sec. 5.1): compare n (x) n
        assert np.max(np.abs(np.outer(nQ, nQ) - np.outer(Q @ n, Q @ n))) <= 1e-9


def hessian_np(F, A, rho, h=1e-4):
    """Central-difference Hessian of the relaxed objective with W_r from
    numpy's eigensolver (independent of the oracle's tangent)."""
    H = np.empty((9, 9))
    E = np.eye(9)
    for a in range(9):
        for b in range(a, 9):
            v = (phi_np(F + h * (E[a] + E[b]), A, rho) - phi_np(F + h * (E[a] - E[b]), A, rho)
                 - phi_np(F - h * (E[a] - E[b]), A, rho) + phi_np(F - h * (E[a] + E[b]), A, rho))
            H[a, b] = H[b, a] = v / (4 * h * h)
    return H


# Local problems where the relaxed objective is not convex at the warm start
# (prox Hessian with an eigenvalue below rho/16, often negative): the data
# near the identity (no load, the aligned state under a small stretch), the
# case where a director-rotation mode has the curvature -1/(lambda_1 -
# lambda_2) of the relaxed energy. The solve must still end at a local
# minimiser of the joint problem in (F, n).
NONCONVEX = [(1.0, 0.0, 10.0), (1.02, 0.005, 10.0), (1.001, 0.005, 10.0), (1.0, 0.005, 10.0),
             (1.02, 0.0, 30.0), (1.0, 0.003, 30.0)]


# the ideal model's two solvers: the singular-basis one (no site) and the
# nine-component Newton solve (a zero site gives the same energy)
PATHS = {"spectral": {}, "newton": {"Sc": np.zeros(9)}}


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("k", range(len(NONCONVEX)))
def test_joint_prox_is_a_local_minimiser_where_not_convex(k, path):
    s, noise, rho = NONCONVEX[k]
    rng = np.random.default_rng(100 + k)
    A = (np.diag([s, s ** -0.5, s ** -0.5]) + noise * rng.standard_normal((3, 3))).ravel()
    n0 = rng.standard_normal(3)
    n0 /= np.linalg.norm(n0)
    F0 = np.eye(3).ravel()
    F, n, it, rc = O.prox(LCE, rho, A, F0, n0, **PATHS[path])
    assert rc == O.OK and it <= 20, (rc, it)
    # jointly stationary: the fixed-director gradient vanishes at the top
    # eigenvector of F F^T (numpy's)
    g = O.stress(LCE, F, n) + rho * (F - A)
    assert np.linalg.norm(g) <= 1e-10
    assert abs(abs(top_vec(F) @ n) - 1.0) <= 1e-12
    # monotone descent from the warm start
    f0 = phi_np(F, A, rho)
    assert f0 <= phi_np(F0, A, rho) + 1e-14
    # no joint perturbation of (F, n) does better, at two scales
    phi_joint = O.energy(LCE, F, n) + 0.5 * rho * np.sum((F - A) ** 2)
    for scale in (1e-3, 3e-2):
        for _ in range(100):
            dF = scale * rng.standard_normal(9)
            nt = n + 10 * scale * rng.standard_normal(3)
            nt /= np.linalg.norm(nt)
            assert O.energy(LCE, F + dF, nt) + 0.5 * rho * np.sum((F + dF - A) ** 2) \
                >= phi_joint - 1e-13
    # second order: the relaxed objective's Hessian (finite differences of
    # the numpy-built W_r) has no negative eigenvalue beyond the difference
    # error, so the point is a local minimiser and not a saddle
    ev = np.linalg.eigvalsh(hessian_np(F, A, rho))
    assert ev[0] >= -1e-4 * rho, ev[:3]
    # BFGS on the numpy-built relaxed objective started at the result stays
    res = minimize(phi_np, F, args=(A, rho), method="BFGS", options={"gtol": 1e-11, "maxiter": 200})
    assert res.fun >= f0 - 1e-13


def test_nonconvex_cases_exercise_the_hessian_modification():
    """At least half of the cases above start where the prox Hessian of the
    relaxed objective (the oracle's tangent, checked against finite
    differences elsewhere) is not positive definite with margin rho/16, and
    at least one starts where it is indefinite."""
    low, neg = 0, 0
    for k, (s, noise, rho) in enumerate(NONCONVEX):
        rng = np.random.default_rng(100 + k)
        A = (np.diag([s, s ** -0.5, s ** -0.5]) + noise * rng.standard_normal((3, 3))).ravel()
        n0 = rng.standard_normal(3)
        n0 /= np.linalg.norm(n0)
        _, _, K = O.relaxed(LCE, np.eye(3).ravel() + 1e-9 * np.arange(9), n0)
        ev = np.linalg.eigvalsh(K + rho * np.eye(9))
        low += ev[0] < rho / 16
        neg += ev[0] < 0
    assert low >= len(NONCONVEX) // 2 and neg >= 1, (low, neg)


def test_spectral_and_newton_paths_agree():
    """The ideal model through its two solvers, from F = I and a random
    director, on data from mild to strong distortion and three penalties:
    the same F and the same director (up to sign) wherever the Newton solve
    converges, and the singular-basis solve converges everywhere in fewer
    iterations. The Newton solve stops at |g| <= gtol * scale, so on weakly
    curved problems (rho = 1) the two differ by that residual over the
    smallest curvature, hence the tolerance."""
    rng = np.random.default_rng(3)
    opts = O.newton_opts(gtol=1e-14, step_tol=1e-10)
    its_s = its_n = 0
    for k in range(90):
        amp = (0.02, 0.1, 0.3)[k % 3]
        rho = (1.0, 10.0, 30.0)[(k // 3) % 3]
        A = (np.eye(3) + rng.uniform(-amp, amp, (3, 3))).ravel()
        n0 = rng.standard_normal(3)
        n0 /= np.linalg.norm(n0)
        Fs, ns, it_s, rc_s = O.prox(LCE, rho, A, np.eye(3).ravel(), n0, opts)
        Fn, nn, it_n, rc_n = O.prox(LCE, rho, A, np.eye(3).ravel(), n0, opts, Sc=np.zeros(9))
        assert rc_s == O.OK, k
        g = O.stress(LCE, Fs, ns) + rho * (Fs - A)
        assert np.linalg.norm(g) <= 1e-10, k
        its_s += it_s
        if rc_n != O.OK:
            continue
        its_n += it_n
        assert np.max(np.abs(Fs - Fn)) <= (1e-9 if rho == 1.0 else 1e-10), k
        assert abs(abs(ns @ nn) - 1.0) <= 1e-10, k
    assert its_s < its_n


@pytest.mark.parametrize("k", range(4))
def test_spectral_prox_is_coaxial_with_the_data(k):
    """F shares A's singular vectors: F A^T and A^T F are symmetric, and the
    director is A's top left singular vector (numpy's SVD)."""
    rng = np.random.default_rng(40 + k)
    A = rot(k) @ np.diag([1.25, 1.0, 0.85]) @ rot(k + 10) + 0.05 * rng.standard_normal((3, 3))
    F, n, _, rc = O.prox(LCE, 10.0, A.ravel(), np.eye(3).ravel(), unit(k))
    assert rc == O.OK
    F = F.reshape(3, 3)
    for M in (F @ A.T, A.T @ F):
        assert np.max(np.abs(M - M.T)) <= 1e-12
    U, _, _ = np.linalg.svd(A)
    assert abs(abs(U[:, 0] @ n) - 1.0) <= 1e-12


def test_spectral_prox_at_tied_data_follows_the_previous_director():
    """A = c I: every direction is a minimiser's director; the solve keeps
    the previous one and returns the uniaxial stretch along it,
    F = f_perp I + (f_par - f_perp) n n^T with f_par > f_perp."""
    for k in range(3):
        n0 = unit(k + 30)
        F, n, _, rc = O.prox(LCE, 10.0, (1.02 * np.eye(3)).ravel(), np.eye(3).ravel(), n0)
        assert rc == O.OK
        assert np.max(np.abs(n - n0)) <= 1e-14
        F = F.reshape(3, 3)
        f_par = n0 @ F @ n0
        f_perp = (np.trace(F) - f_par) / 2
        assert f_par > f_perp + 0.05
        assert np.max(np.abs(F - (f_perp * np.eye(3) + (f_par - f_perp) * np.outer(n0, n0)))) <= 1e-13


@pytest.mark.parametrize("k", range(3))
def test_spectral_prox_with_negative_det_data(k):
    """Data A with det A < 0 (a reflection times a stretch): the signed
    singular value a3 is negative, the minimiser keeps det F > 0, is
    stationary, has no joint perturbation doing better, and agrees with the
    nine-component Newton solve; for a mild reflection of a single axis it
    stays close to A elsewhere."""
    rng = np.random.default_rng(70 + k)
    R = np.diag([1.0, 1.0, -1.0]) if k == 0 else rot(k) @ np.diag([1.0, -1.0, 1.0]) @ rot(k + 5)
    A = (R @ np.diag([1.2, 1.0, 0.3]) + 0.02 * rng.standard_normal((3, 3))).ravel()
    assert np.linalg.det(A.reshape(3, 3)) < 0
    rho = 10.0
    n0 = unit(k + 50)
    F, n, it, rc = O.prox(LCE, rho, A, np.eye(3).ravel(), n0)
    assert rc == O.OK, rc
    assert np.linalg.det(F.reshape(3, 3)) > 0
    g = O.stress(LCE, F, n) + rho * (F - A)
    assert np.linalg.norm(g) <= 1e-10
    assert abs(abs(top_vec(F) @ n) - 1.0) <= 1e-12
    phi = O.energy(LCE, F, n) + 0.5 * rho * np.sum((F - A) ** 2)
    for _ in range(100):
        dF = 1e-3 * rng.standard_normal(9)
        nt = n + 1e-2 * rng.standard_normal(3)
        nt /= np.linalg.norm(nt)
        if np.linalg.det((F + dF).reshape(3, 3)) <= 0:
            continue
        assert O.energy(LCE, F + dF, nt) + 0.5 * rho * np.sum((F + dF - A) ** 2) >= phi - 1e-13
    Fn, nn, _, rcn = O.prox(LCE, rho, A, np.eye(3).ravel(), n0, Sc=np.zeros(9))
    assert rcn == O.OK
    assert np.max(np.abs(F - Fn)) <= 1e-10
