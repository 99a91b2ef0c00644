"""GPU parity of the liquid-crystal-elastomer local step (neo-classical energy
of Sec. 5.1 with a volumetric penalty, director minimised per voxel) against
the CPU oracle: per-voxel local solves with directors, whole iterations on a
small periodic polydomain, and the homogenised stress in both precisions.

Directors n and -n are the same state; both sides fix the sign by
n . n_prev >= 0, so they are compared directly.
"""
import numpy as np
import pytest

import oracle as O
from paper_2010_06697_amd import admm, microstructure as M
from parity_util import NEWTON64, gpu_solver, omats, random_state, rel

pytestmark = pytest.mark.gpu

LCE = [M.lce(1.0, 2.0, 100.0)]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def polydomain(n, grains, seed):
    g, d = M.voronoi_grains(n=n, n_grains=grains, seed=seed)
    return np.zeros(g.shape, np.uint8), M.director_field(g, d)


def lce_solver(phase, n0, Fbar, precision, **kw):
    p = admm.default_params(precision, **kw)
    return admm.Solver([phase], LCE, [Fbar], p, precision=precision, directors=[n0])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("stretched", [True, False])
def test_lce_local_step_matches_oracle(precision, stretched):
    """Per-voxel local solves. With a clear stretch the top eigenvalue of
    F F^T is well separated and the F / director alternation converges on
    both sides; with a random small distortion it contracts slowly and may
    stop at its cap, the same alternation on both sides."""
    shape = (6, 8, 12)
    say("lce local", precision, "stretched" if stretched else "random")
    phase = np.zeros(shape, np.uint8)
    rng = np.random.default_rng(21)
    n0 = rng.standard_normal((3,) + shape)
    n0 /= np.linalg.norm(n0, axis=0, keepdims=True)
    u, F, L = random_state(shape, seed=22, amp_E=0.02 if stretched else 0.05, amp_L=0.3)
    if stretched:
        Fbar = np.diag([1.2, 1.2 ** -0.5, 1.2 ** -0.5])
        F = F + (Fbar - np.eye(3)).reshape(9)[:, None, None, None]
    else:
        Fbar = M.uniaxial_lce(1.03)
    rho = 10.0
    s = lce_solver(phase, n0, Fbar, precision, rho0=rho, dir_max=400)
    s.set_state(0, u=u, F=F, Lambda=L)
    st0 = s.state(0)
    s.local_step()
    out = s.state(0)
    s.close()
    G = O.gradient(st0["u"], Fbar.ravel())
    A = G + st0["Lambda"] / rho
    m = omats(LCE)[0]
    errF = errn = 0.0
    capped = 0
    for x in np.ndindex(shape):
        sl = (slice(None),) + x
        nstart = st0["director"][sl] / np.linalg.norm(st0["director"][sl])
        Fx, nx, _, rc = O.prox(m, rho, A[sl], st0["F"][sl], nstart,
                               opts=O.newton_opts(dir_max=400, **NEWTON64))
        capped += rc != O.OK
        errF = max(errF, np.max(np.abs(out["F"][sl] - Fx)))
        errn = max(errn, np.max(np.abs(out["director"][sl] - nx)))
    say("  max |dF|", errF, "max |dn|", errn, "oracle capped", capped)
    if stretched:
        assert capped == 0
    if precision == "fp64":
        assert errF <= 1e-10 and errn <= 1e-9
    else:
        assert errF <= 5e-5 and errn <= (2e-3 if stretched else 5e-2)


@pytest.mark.parametrize("stretch", [1.0, 1.2])
def test_lce_iterations_match_oracle_fp64(stretch):
    """Whole iterations on a 16^3 polydomain. At stretch 1.0 (relaxation of
    the grains' directors at zero macroscopic strain) both sides run the same
    capped alternations; at 1.2 the top eigenvalue of F F^T is well separated
    and every local problem is convex. Stretches just above 1 (about
    1.01-1.05) are left out: there the relaxed energy's curvature along the
    director-rotation mode scales like -1/(l1 - l2), the local problems have
    saddles, and which side of a saddle a voxel leaves by is decided by
    rounding."""
    phase, n0 = polydomain(16, 6, seed=7)
    Fbar = M.uniaxial_lce(stretch)
    say("lce iterations", stretch)
    n_iter, rho = 4, 10.0
    s = lce_solver(phase, n0, Fbar, "fp64", rho0=rho, mu_ref=1.0)
    rc, rp, rd, _ = s.step(n_iter)
    st = s.state(0)
    P, Lm = s.homogenized_stress(0)
    s.close()
    u, F, L = O.initial_state(phase.shape)
    n = n0.copy()
    p = O.params(max_iter=n_iter, fixed_iters=True, mu_ref=1.0, newton=O.newton_opts(**NEWTON64))
    O.admm_run(phase, omats(LCE), Fbar.ravel(), p, u, F, L, rho, director_field=n)
    Po = O.mean_stress(phase, omats(LCE), F, director_field=n)
    say("  rel u F L n P", rel(st["u"], u), rel(st["F"], F), rel(st["Lambda"], L),
        rel(st["director"], n), rel(P, Po))
    assert rc == admm.OK
    assert rel(st["u"], u) <= 1e-10 and rel(st["F"], F) <= 1e-10
    assert rel(st["Lambda"], L) <= 1e-10 and rel(st["director"], n) <= 1e-9
    assert rel(P, Po) <= 1e-10


def test_lce_fp32_homogenized_stress_within_1e5():
    phase, n0 = polydomain(16, 6, seed=7)
    Fbar = M.uniaxial_lce(1.2)
    n_iter, rho = 6, 10.0
    s = lce_solver(phase, n0, Fbar, "fp32", rho0=rho, mu_ref=1.0)
    s.step(n_iter)
    P, _ = s.homogenized_stress(0)
    s.close()
    u, F, L = O.initial_state(phase.shape)
    n = n0.copy()
    p = O.params(max_iter=n_iter, fixed_iters=True, mu_ref=1.0, newton=O.newton_opts(**NEWTON64))
    O.admm_run(phase, omats(LCE), Fbar.ravel(), p, u, F, L, rho, director_field=n)
    Po = O.mean_stress(phase, omats(LCE), F, director_field=n)
    say("lce fp32 rel P", rel(P, Po))
    assert rel(P, Po) <= 1e-5
