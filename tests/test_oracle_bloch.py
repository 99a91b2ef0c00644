"""Pins of the oracle's Bloch-wave stability modulus (Sec. 2.5, Steps 1'-4'):
beta = min over unit Bloch waves p exp(i omega.x) of <D_w p, L D_w p>.

The reference is the smallest eigenvalue of the Hermitian matrix
D_w^H L D_w assembled densely in numpy on small grids (the shifted central
difference written out as a matrix, L the tangent of each voxel), which
shares nothing with the ADMM. Checked: the value on a homogeneous body (where
it is mu min |K(xi + omega)|^2 for the neo-Hookean), on a two-phase field
where it is negative (an unstable state), and on an LCE polydomain with the
director eliminated; the returned mode is a unit eigenvector; rho sigma of
Step 2' equals beta at the fixed point; a penalty below the tangent's most
negative eigenvalue is refused.
"""
import numpy as np
import pytest

import oracle as O
from paper_2010_06697_amd import microstructure as M


def dense_operator(phase, mats, F, omega, director=None):
    n3, n2, n1 = phase.shape
    V = phase.size
    nn = (n1, n2, n3)
    D = np.zeros((9 * V, 3 * V), complex)
    for x in range(V):
        k = [x % n1, (x // n1) % n2, x // (n1 * n2)]
        for j in range(3):
            kp, km = list(k), list(k)
            kp[j] = (k[j] + 1) % nn[j]
            km[j] = (k[j] - 1) % nn[j]
            xp = (kp[2] * n2 + kp[1]) * n1 + kp[0]
            xm = (km[2] * n2 + km[1]) * n1 + km[0]
            for i in range(3):
                D[(3 * i + j) * V + x, i * V + xp] += 0.5 * np.exp(1j * omega[j])
                D[(3 * i + j) * V + x, i * V + xm] -= 0.5 * np.exp(-1j * omega[j])
    L = np.zeros((9 * V, 9 * V))
    Fl = F.reshape(9, V)
    for x in range(V):
        m = mats[phase.ravel()[x]]
        if m.model == O.LCE:
            K = O.relaxed(m, Fl[:, x], director.reshape(3, V)[:, x])[2]
        else:
            K = O.tangent(m, Fl[:, x])
        idx = np.arange(9) * V + x
        L[np.ix_(idx, idx)] = K
    A = D.conj().T @ L @ D
    return 0.5 * (A + A.conj().T)


def cases():
    rng = np.random.default_rng(1)
    shape = (4, 4, 4)
    out = {}
    phase = np.zeros(shape, np.uint8)
    F = np.zeros((9,) + shape)
    F[:] = np.diag([1.1, 0.95, 1.0]).ravel()[:, None, None, None]
    out["homogeneous"] = (phase, [O.material("neohooke", mu=1.0, lam=2.0)], F, None, 5.0)
    phase = M.random_two_phase(shape, 0.5, seed=3)
    F = np.zeros((9,) + shape)
    F[[0, 4, 8]] = 1.0
    F += 0.1 * rng.standard_normal(F.shape)
    # the tangent's most negative eigenvalue here is about -18.6
    out["two_phase"] = (phase, [O.material("neohooke", mu=10.0, lam=20.0),
                                O.material("neohooke", mu=1.0, lam=2.0)], F, None, 40.0)
    g, dirs = M.voronoi_grains(n=4, n_grains=3, seed=2)
    d = M.director_field(g, dirs)
    F = np.zeros((9,) + shape)
    F[:] = np.diag([1.2, 1.2 ** -0.5, 1.2 ** -0.5]).ravel()[:, None, None, None]
    F += 0.02 * rng.standard_normal(F.shape)
    out["lce"] = (np.zeros(shape, np.uint8), [O.material("lce", mu=1.0, a=2.0, kappa=20.0)], F, d,
                  20.0)
    return out


OMEGA = np.array([2 * np.pi / 8, 2 * np.pi / 8, 0.3])


@pytest.mark.parametrize("name", ["homogeneous", "two_phase", "lce"])
def test_bloch_modulus_is_the_smallest_eigenvalue(name):
    phase, mats, F, d, rho = cases()[name]
    A = dense_operator(phase, mats, F, OMEGA, d)
    w, U = np.linalg.eigh(A)
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal((3,) + phase.shape) + 1j * rng.standard_normal((3,) + phase.shape)
    r = O.bloch(phase, mats, F, OMEGA, rho, p0, tol=1e-11, max_iter=20000, director_field=d)
    assert r["rc"] == O.OK, r
    assert abs(r["beta"] - w[0]) <= 1e-9 * max(1.0, abs(w[0]))
    assert abs(r["sigma_rho"] - r["beta"]) <= 1e-8 * max(1.0, abs(w[0]))
    p = r["p"].reshape(-1)
    assert abs(np.mean(np.abs(p) ** 2) * 3 - 1.0) <= 1e-12   # mean over voxels of |p|^2 = 1
    res = A @ p - w[0] * p
    assert np.linalg.norm(res) <= 1e-7 * np.linalg.norm(p) * max(1.0, abs(w[0]))
    if name == "two_phase":
        assert w[0] < 0.0   # an unstable state
    if name == "homogeneous":
        # plane waves: mu times the smallest shifted symbol
        n = phase.shape[0]
        xi = 2 * np.pi * np.arange(n) / n
        k2 = min(np.sin(a + OMEGA[0]) ** 2 + np.sin(b + OMEGA[1]) ** 2 + np.sin(c + OMEGA[2]) ** 2
                 for a in xi for b in xi for c in xi)
        assert abs(w[0] - 1.0 * k2) <= 1e-12


def test_bloch_penalty_must_make_the_local_problem_convex():
    phase, mats, F, d, _ = cases()["two_phase"]
    p0 = np.ones((3,) + phase.shape, complex)
    assert O.bloch(phase, mats, F, OMEGA, 10.0, p0)["rc"] == O.EDOMAIN
