"""GPU parity of the inexact local step (Sec. 2.1, local residual r_l;
Sec. 4, the two strategies): Step 1 runs in passes of at most local_chunk
Newton iterations per voxel (F and, for the LCE, the director continue from
the previous pass) until r_l, the RMS over the cell of
|dW/dF + rho (F - A)| / mu_ref, is at most local_ratio times the previous
iteration's r_d (from the second iteration of a load step on), or until the
local solves have converged at local_fraction of the voxels, or local_passes
passes ran. The oracle runs the same schedule.

The pass count is decided by comparing a sum with its target; the two sides
sum in different orders (and a voxel at the edge of its Newton stopping rule
could count as converged on one side only), which could flip a decision
taken within rounding of the target: a CPU test checks that the oracle's
decisions on these cases are far from such ties. Tolerances are those of the
exact iteration (1e-10 relative in double precision).
"""
import numpy as np
import pytest

import oracle as O
from paper_2010_06697_amd import admm, microstructure as M
from parity_util import NEWTON64, gpu_solver, omats, oracle_iterations, rel

pytestmark = pytest.mark.gpu

MATS = [M.neohooke(10.0, 40.0), M.neohooke(1.0, 4.0)]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# (shape, local_* options, graph capture); inputs of inexact_case.
# tests/test_oracle_admm.py checks on the CPU that the oracle's pass decisions
# on these cases do not move when the ratio moves by 1e-9 relative or the
# fraction by 1.5 voxels.
CASES = [
    ((16, 12, 24), dict(local_ratio=0.3, local_chunk=1, local_passes=4), 1),
    ((18, 36, 48), dict(local_ratio=0.3, local_chunk=1, local_passes=4), 0),
    ((8, 6, 96), dict(local_ratio=0.1, local_chunk=2, local_passes=3), 1),
    ((32, 32, 32), dict(local_ratio=0.3, local_chunk=1, local_passes=8), 1),
    ((16, 12, 24), dict(local_fraction=0.5, local_chunk=1, local_passes=8), 1),
    ((18, 36, 48), dict(local_fraction=0.9, local_chunk=1, local_passes=8), 0),
]
N_ITER = 6
# the fraction strategy's cases need local solves that converge after
# different numbers of Newton iterations: a contrast of 100 and a larger load
MATS_FRACTION = [M.neohooke(100.0, 1000.0), M.neohooke(1.0, 4.0)]


def inexact_case(shape, loc):
    """two neo-Hookean phases, random at 40 %, a random macroscopic
    deformation of amplitude 0.08 (0.2 for the fraction strategy); rho 8,
    mu_ref 4. Returns phase, Fbar, materials, rho, mu_ref."""
    frac = "local_fraction" in loc
    return (M.random_two_phase(shape, 0.4, seed=10), M.random_fbar(0.2 if frac else 0.08, seed=11),
            MATS_FRACTION if frac else MATS, 8.0, 4.0)


@pytest.mark.parametrize("shape,loc,graph", CASES)
def test_inexact_iterations_match_oracle_fp64(shape, loc, graph):
    say("inexact iterations fp64", shape, loc, "graph" if graph else "eager")
    phase, Fbar, mats, rho, mu_ref = inexact_case(shape, loc)
    n_iter = N_ITER
    s = gpu_solver([phase], mats, [Fbar], "fp64", rho0=rho, mu_ref=mu_ref, use_graph=graph,
                   check_every=n_iter, **loc)
    rc, rp, rd, rr = s.step(n_iter)
    st = s.state(0)
    P, Lm = s.homogenized_stress(0)
    hp, hd, hr = s.history(0)
    s.close()
    u, F, L, r = oracle_iterations(phase, mats, Fbar, n_iter, rho, mu_ref, **loc)
    Po, Lo = O.mean_stress(phase, omats(mats), F, Lam=L)
    say("  rel u F L P:", rel(st["u"], u), rel(st["F"], F), rel(st["Lambda"], L), rel(P, Po))
    assert rc == admm.OK
    assert rel(st["u"], u) <= 1e-10
    assert rel(st["F"], F) <= 1e-10
    assert rel(st["Lambda"], L) <= 1e-10
    assert rel(P, Po) <= 1e-10 and rel(Lm, Lo) <= 1e-10
    assert np.allclose(hp, r["r_p"], rtol=1e-9, atol=0) and np.allclose(hd, r["r_d"], rtol=1e-9)


@pytest.mark.parametrize("k", [0, 4])
def test_inexact_differs_from_exact(k):
    """Guard that the parity cases exercise truncated solves: the fields
    after the parity cases' iterations differ from the exact iteration's by
    far more than the parity tolerance."""
    shape, loc, _ = CASES[k]
    phase, Fbar, mats, rho, mu_ref = inexact_case(shape, loc)
    out = []
    for kw in ({}, loc):
        s = gpu_solver([phase], mats, [Fbar], "fp64", rho0=rho, mu_ref=mu_ref, **kw)
        s.step(N_ITER)
        out.append(s.state(0)["F"])
        s.close()
    assert rel(out[1], out[0]) >= 1e-6


@pytest.mark.parametrize("limit", [dict(local_ratio=1e-30), dict(local_fraction=1.0)])
def test_strict_limits_reproduce_the_exact_iteration(limit):
    """A vanishing ratio, or convergence required at every voxel, with enough
    passes: the exact iteration."""
    shape = (18, 36, 48)
    phase = M.random_two_phase(shape, 0.4, seed=12)
    Fbar = M.random_fbar(0.05, seed=13)
    out = []
    for loc in ({}, dict(local_chunk=1, local_passes=60, **limit)):
        s = gpu_solver([phase], MATS, [Fbar], "fp64", rho0=8.0, mu_ref=4.0, **loc)
        s.step(5)
        out.append(s.state(0))
        s.close()
    for k in ("u", "F", "Lambda"):
        assert rel(out[1][k], out[0][k]) <= 1e-12, k


def test_inexact_lce_composite_matches_oracle_fp64():
    """Polydomain LCE with a stiff neo-Hookean inclusion under a stretch 1.2,
    every neo-Hookean solve truncated to one Newton iteration per pass (the
    ideal LCE's singular-basis solves run in full in every pass, on both
    sides)."""
    from test_gpu_lce import iteration_case
    phase, n0, Fbar, mats = iteration_case("composite")
    loc = dict(local_ratio=0.3, local_chunk=1, local_passes=4)
    rho, n_iter = 10.0, 4
    p = admm.default_params("fp64", rho0=rho, mu_ref=1.0, **loc)
    s = admm.Solver([phase], mats, [Fbar], p, precision="fp64", directors=[n0])
    rc, _, _, _ = s.step(n_iter)
    st = s.state(0)
    P, _ = s.homogenized_stress(0)
    s.close()
    u, F, L = O.initial_state(phase.shape)
    n = n0.copy()
    op = O.params(max_iter=n_iter, fixed_iters=True, mu_ref=1.0,
                  newton=O.newton_opts(**NEWTON64), **loc)
    O.admm_run(phase, omats(mats), Fbar.ravel(), op, u, F, L, rho, director_field=n)
    Po = O.mean_stress(phase, omats(mats), F, director_field=n)
    errs = {k: rel(st[k], o) for k, o in (("u", u), ("F", F), ("Lambda", L), ("director", n))}
    say("  rel", errs, "P", rel(P, Po))
    assert rc == admm.OK
    assert errs["u"] <= 1e-10 and errs["F"] <= 1e-10 and errs["Lambda"] <= 1e-10
    assert errs["director"] <= 1e-9
    assert rel(P, Po) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("strategy", [dict(local_ratio=0.3, local_chunk=1, local_passes=4),
                                      dict(local_fraction=0.5, local_chunk=1, local_passes=4)])
def test_inexact_solve_reaches_the_laminate_solution(precision, strategy):
    """With r_l held to 0.3 r_d, or half the local solves converged, the
    iteration converges to the same fixed point as the exact one, the
    laminate's closed-form finite-strain solution; in double precision the
    ratio strategy takes fewer Newton iterations in total. (In float the
    exact solves stop by their step test after about one iteration, while
    r_l cannot fall below float rounding, so near convergence the ratio
    strategy runs all its passes. The laminate's voxels of one phase all
    converge together, so the fraction strategy saves little there.)"""
    case = M.laminate16_case()
    Fb = case["loads"][0]
    d, Pd = laminate_exact()
    # the stress error of a converged state is set by the stopping tolerance
    # (the same tolerances and bounds as the exact solve's parity test)
    tol = 1e-10 if precision == "fp64" else 2e-7
    its = []
    for loc in ({}, strategy):
        s = gpu_solver([case["phase"]], case["materials"], [Fb], precision, rho0=5.0, mu_ref=5.5,
                       tol_p=tol, tol_d=tol, max_iter=600, **loc)
        rc, it, _ = s.solve()
        _, _, _, newton_its = s.info(0)
        P, _ = s.homogenized_stress(0)
        s.close()
        say(" ", precision, "inexact" if loc else "exact", "iterations", it, "newton", newton_its,
            "P diag", P.ravel()[[0, 4, 8]])
        assert rc == admm.OK
        bound = 1e-8 if precision == "fp64" else 1e-5
        assert np.max(np.abs(P.ravel()[[0, 4, 8]] - Pd)) <= bound * np.max(np.abs(Pd))
        its.append(newton_its)
    if precision == "fp64":
        assert its[1] < its[0] if "local_ratio" in strategy else its[1] <= its[0]


def laminate_exact():
    from test_oracle_admm import laminate_exact as le
    return le(10.0, 100.0, 1.0, 10.0, 0.95)
