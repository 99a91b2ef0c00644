"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Each part of the iteration is compared on the same seeded inputs, element by
element, then whole iterations, then converged solves against the closed-form
laminate. Sizes span several workgroup tiles and ragged tails (edges 6..96,
x1-rows per workgroup not dividing the row count, half-spectrum widths not
dividing the tile width).

Tolerances: double precision 1e-10 relative on u, F, Lambda and <P> (the
target of the method's FP64 form; the observed errors are ~1e-13: the GPU's
local step reaches the minimiser, the oracle's Newton stops within about
1e-12 of it); reduced precision (float fields, double reductions) 1e-5
relative on <P>.
"""
import numpy as np
import pytest

import oracle as O
from paper_2010_06697_amd import admm, microstructure as M
from parity_util import NEWTON64, gpu_solver, omats, oracle_iterations, prox_minimiser, random_state, rel

pytestmark = pytest.mark.gpu

SHAPES = [(6, 8, 12), (16, 12, 24), (18, 36, 48), (8, 6, 96), (32, 32, 32)]
MATS = [M.neohooke(10.0, 40.0), M.neohooke(1.0, 4.0)]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_projection_matches_oracle(shape, precision):
    say("projection", shape, precision)
    phase = M.random_two_phase(shape, 0.4, seed=1)
    Fbar = M.random_fbar(0.03, seed=2)
    u, F, L = random_state(shape, seed=3)
    rho = 2.5
    s = gpu_solver([phase], MATS, [Fbar], precision, rho0=rho)
    s.set_state(0, u=u, F=F, Lambda=L)
    s.project_step()
    got = s.state(0)["u_prev"]
    s.close()
    ref = O.project(F - L / rho)
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert rel(got, ref) <= tol


@pytest.mark.parametrize("shape", SHAPES[:3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_local_step_matches_oracle(shape, precision):
    say("local step", shape, precision)
    phase = M.random_two_phase(shape, 0.5, seed=4)
    Fbar = M.random_fbar(0.04, seed=5)
    u, F, L = random_state(shape, seed=6)
    rho = 12.0
    s = gpu_solver([phase], MATS, [Fbar], precision, rho0=rho)
    s.set_state(0, u=u, F=F, Lambda=L)
    st0 = s.state(0)
    s.local_step()
    got = s.state(0)["F"]
    it, status, nfail, newton_its = s.info(0)
    s.close()
    assert nfail == 0
    # oracle: per voxel, from the same (stored-precision) inputs and warm start
    G = O.gradient(st0["u"], Fbar.ravel())
    A = G + st0["Lambda"] / rho
    om = omats(MATS)
    ref = np.empty_like(got)
    n3, n2, n1 = shape
    for x in np.ndindex(shape):
        Fx, rc = prox_minimiser(om[phase[x]], rho, A[(slice(None),) + x], st0["F"][(slice(None),) + x])
        assert rc == O.OK
        ref[(slice(None),) + x] = Fx
    err = np.max(np.abs(got - ref))
    say("  max |F - F_oracle| =", err)
    assert err <= (1e-12 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_local_step_with_negative_det_data(precision):
    """Data A = grad u + Lambda/rho with det A < 0 on a third of the voxels
    (A_33 pushed below zero through Lambda): the float exact step's closed
    form (coaxial minimiser, det A > 0 only) leaves those voxels to the
    nine-component Newton of a second pass over the workgroups that have
    any; both kinds of voxel, in both precisions, match the oracle's prox
    from the same inputs and warm start (Sec. 2.1, Step 1)."""
    shape = (12, 16, 24)
    say("local step, det A < 0 on a third of the voxels", precision)
    phase = M.random_two_phase(shape, 0.5, seed=14)
    Fbar = M.random_fbar(0.04, seed=15)
    u, F, L = random_state(shape, seed=16)
    rho = 12.0
    rng = np.random.default_rng(17)
    neg = rng.random(shape) < 1.0 / 3.0
    L[8][neg] = -rho * rng.uniform(1.2, 1.6, size=int(neg.sum()))
    s = gpu_solver([phase], MATS, [Fbar], precision, rho0=rho)
    s.set_state(0, u=u, F=F, Lambda=L)
    st0 = s.state(0)
    s.local_step()
    got = s.state(0)["F"]
    it, status, nfail, newton_its = s.info(0)
    s.close()
    assert nfail == 0
    G = O.gradient(st0["u"], Fbar.ravel())
    A = G + st0["Lambda"] / rho
    detA = np.linalg.det(np.moveaxis(A.reshape((3, 3) + shape), (0, 1), (-2, -1)))
    assert (detA < 0).sum() >= neg.sum() // 2
    om = omats(MATS)
    ref = np.empty_like(got)
    for x in np.ndindex(shape):
        Fx, rc = prox_minimiser(om[phase[x]], rho, A[(slice(None),) + x], st0["F"][(slice(None),) + x])
        assert rc == O.OK
        ref[(slice(None),) + x] = Fx
    detF = np.linalg.det(np.moveaxis(got.reshape((3, 3) + shape), (0, 1), (-2, -1)))
    assert detF.min() > 0.0
    err = np.max(np.abs(got - ref))
    say("  max |F - F_oracle| =", err)
    assert err <= (1e-12 if precision == "fp64" else 1e-6)


def test_fields_written_between_calls_are_read():
    """Within a call the float form's local step reads its data as the
    previous update formed it; a call must still start from the fields the
    caller holds. Four iterations, then new u, F and Lambda written into the
    caller's buffers and three more iterations: bit for bit the result of a
    fresh context started from those fields (fixed penalty, so the contexts'
    histories do not matter)."""
    shape = (16, 12, 24)
    say("fields written between calls")
    phase = M.random_two_phase(shape, 0.5, seed=31)
    Fbar = M.random_fbar(0.04, seed=32)
    u1, F1, L1 = random_state(shape, seed=33)
    u2, F2, L2 = random_state(shape, seed=34)
    kw = dict(rho0=6.0, adapt_rho=0, mu_ref=4.0, div_growth=0.0, stall_iters=0)
    s = gpu_solver([phase], MATS, [Fbar], "fp32", **kw)
    s.set_state(0, u=u1, F=F1, Lambda=L1)
    s.step(4)
    s.set_state(0, u=u2, F=F2, Lambda=L2)
    s.step(3)
    a = s.state(0)
    s.close()
    s = gpu_solver([phase], MATS, [Fbar], "fp32", **kw)
    s.set_state(0, u=u2, F=F2, Lambda=L2)
    s.step(3)
    b = s.state(0)
    s.close()
    for k in ("u", "F", "Lambda"):
        assert np.array_equal(a[k], b[k]), k


def test_projection_after_iterations_reads_the_fields():
    """Within a call the float form's Step 2 forms its right-hand side from
    the field F - A that the local step of the iteration left; a projection
    called on its own must form it from the fields the caller holds. Four
    iterations, new u, F and Lambda written, one projection: bit for bit
    the projection of a fresh context started from those fields, and the
    oracle's projection of them."""
    shape = (16, 12, 24)
    say("projection after iterations")
    phase = M.random_two_phase(shape, 0.5, seed=35)
    Fbar = M.random_fbar(0.04, seed=36)
    u1, F1, L1 = random_state(shape, seed=37)
    u2, F2, L2 = random_state(shape, seed=38)
    kw = dict(rho0=6.0, adapt_rho=0, mu_ref=4.0, div_growth=0.0, stall_iters=0)
    s = gpu_solver([phase], MATS, [Fbar], "fp32", **kw)
    s.set_state(0, u=u1, F=F1, Lambda=L1)
    s.step(4)
    s.set_state(0, u=u2, F=F2, Lambda=L2)
    s.project_step()
    a = s.state(0)["u_prev"]  # the projection's u_{i+1}
    s.close()
    s = gpu_solver([phase], MATS, [Fbar], "fp32", **kw)
    s.set_state(0, u=u2, F=F2, Lambda=L2)
    s.project_step()
    b = s.state(0)["u_prev"]
    s.close()
    assert np.array_equal(a, b)
    assert rel(a, O.project(F2 - L2 / 6.0)) <= 2e-5


def test_cached_local_data_equals_recomputed():
    """The float form's local step reads its data as the update formed it
    while the penalty stays, and recomputes it from u and Lambda when the
    adaptive rule changes the penalty (and at every call's start). Fourteen
    iterations in one call against fourteen calls of one iteration each
    (every local step recomputing): the same penalty sequence, with changes
    during the run, and the same iterates up to float rounding (the null-mode
    removal each call repeats moves u by rounding and flips float ulps of
    the local data, which fourteen iterations carry to ~1e-8 in u); a stale
    or wrongly formed cache moves them by the size of an iteration's change."""
    shape = (16, 12, 24)
    say("cached local data vs recomputed")
    phase = M.random_two_phase(shape, 0.5, seed=41)
    Fbar = M.random_fbar(0.04, seed=42)
    u, F, L = random_state(shape, seed=43)
    kw = dict(rho0=2.0, adapt_rho=1, rho_min=0.5, rho_max=200.0, mu_ref=4.0, tau=2.0,
              div_growth=0.0, stall_iters=0)
    out = []
    for calls in ([14], [1] * 14):
        s = gpu_solver([phase], MATS, [Fbar], "fp32", **kw)
        s.set_state(0, u=u, F=F, Lambda=L)
        for n in calls:
            s.step(n)
        out.append((s.state(0), s.history(0)[2]))
        s.close()
    (a, rho_a), (b, rho_b) = out
    say("  rho sequence", rho_a)
    assert len(set(rho_a.tolist())) >= 2  # the penalty changed during the run
    assert np.array_equal(rho_a, rho_b)
    du, dF, dL = rel(a["u"], b["u"]), rel(a["F"], b["F"]), rel(a["Lambda"], b["Lambda"])
    say("  apart: u", du, "F", dF, "Lambda", dL)
    assert du <= 1e-7 and dF <= 1e-6 and dL <= 1e-5


@pytest.mark.parametrize("shape", SHAPES[:3])
def test_update_matches_definition(shape):
    say("update", shape)
    phase = M.random_two_phase(shape, 0.5, seed=7)
    Fbar = M.random_fbar(0.04, seed=8)
    u, F, L = random_state(shape, seed=9)
    rho = 7.0
    mu_ref = 3.0
    s = gpu_solver([phase], MATS, [Fbar], "fp64", rho0=rho, mu_ref=mu_ref)
    s.set_state(0, u=u, F=F, Lambda=L)
    s.project_step()
    un = s.state(0)["u_prev"]
    s.update_step()
    st = s.state(0)
    rp_h, rd_h, rho_h = s.history(0)
    s.close()
    G1 = O.gradient(un, Fbar.ravel())
    G0 = O.gradient(u, Fbar.ravel())
    Lref = L + rho * (G1 - F)
    assert rel(st["Lambda"], Lref) <= 1e-13
    assert rel(st["u"], un) == 0.0
    rp = np.sqrt(np.mean(np.sum((G1 - F) ** 2, axis=0)))
    rd = rho / mu_ref * np.sqrt(np.mean(np.sum((G1 - G0) ** 2, axis=0)))
    assert abs(rp_h[-1] - rp) <= 1e-12 * rp and abs(rd_h[-1] - rd) <= 1e-12 * rd
    assert rho_h[-1] == rho


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("n_iter", [1, 4])
def test_iterations_match_oracle_fp64(shape, n_iter):
    say("iterations fp64", shape, n_iter)
    phase = M.random_two_phase(shape, 0.4, seed=10)
    Fbar = M.random_fbar(0.04, seed=11)
    rho, mu_ref = 8.0, 4.0
    s = gpu_solver([phase], MATS, [Fbar], "fp64", rho0=rho, mu_ref=mu_ref)
    rc, rp, rd, rr = s.step(n_iter)
    st = s.state(0)
    P, Lm = s.homogenized_stress(0)
    hp, hd, hr = s.history(0)
    s.close()
    u, F, L, r = oracle_iterations(phase, MATS, Fbar, n_iter, rho, mu_ref)
    Po, Lo = O.mean_stress(phase, omats(MATS), F, Lam=L)
    say("  rel u F L P:", rel(st["u"], u), rel(st["F"], F), rel(st["Lambda"], L), rel(P, Po))
    assert rc == admm.OK
    assert rel(st["u"], u) <= 1e-10
    assert rel(st["F"], F) <= 1e-10
    assert rel(st["Lambda"], L) <= 1e-10
    assert rel(P, Po) <= 1e-10 and rel(Lm, Lo) <= 1e-10
    assert np.allclose(hp, r["r_p"], rtol=1e-9, atol=0) and np.allclose(hd, r["r_d"], rtol=1e-9)


def test_adaptive_penalty_sequence_matches_oracle():
    shape = (16, 12, 24)
    say("adaptive rho", shape)
    phase = M.random_two_phase(shape, 0.5, seed=12)
    mats = [M.neohooke(20.0, 60.0), M.neohooke(1.0, 3.0)]
    Fbar = M.random_fbar(0.04, seed=13)
    s = gpu_solver([phase], mats, [Fbar], "fp64", rho0=40.0, mu_ref=7.0, adapt_rho=1,
                   rho_min=1.0, rho_max=50.0)
    s.step(25)
    st = s.state(0)
    hp, hd, hr = s.history(0)
    s.close()
    u, F, L, r = oracle_iterations(phase, mats, Fbar, 25, 40.0, 7.0, adapt=True)
    assert np.array_equal(hr, r["rho_hist"])
    assert len(set(hr.tolist())) > 1
    assert rel(st["F"], F) <= 1e-10 and rel(st["u"], u) <= 1e-10


@pytest.mark.parametrize("shape", [(16, 12, 24), (32, 32, 32)])
def test_fp32_mode_homogenized_stress_within_1e5(shape):
    say("fp32 iterations", shape)
    phase = M.random_two_phase(shape, 0.4, seed=14)
    Fbar = M.random_fbar(0.04, seed=15)
    rho, mu_ref = 8.0, 4.0
    n_iter = 10
    s = gpu_solver([phase], MATS, [Fbar], "fp32", rho0=rho, mu_ref=mu_ref)
    s.step(n_iter)
    st = s.state(0)
    P, _ = s.homogenized_stress(0)
    s.close()
    u, F, L, r = oracle_iterations(phase, MATS, Fbar, n_iter, rho, mu_ref)
    Po = O.mean_stress(phase, omats(MATS), F)
    say("  fp32 rel u F L P:", rel(st["u"], u), rel(st["F"], F), rel(st["Lambda"], L), rel(P, Po))
    assert rel(P, Po) <= 1e-5
    assert rel(st["F"], F) <= 1e-4


def laminate_exact(mu_s, lam_s, mu_f, lam_f, f33):
    from scipy.optimize import brentq

    def P(f1, mu, lam):
        J = f1 * f33
        lj = np.log(J)
        return np.array([mu * (f1 - 1 / f1) + lam * lj / f1, lam * lj,
                         mu * (f33 - 1 / f33) + lam * lj / f33])
    d = brentq(lambda d: P(1 + d, mu_s, lam_s)[0] - P(1 - d, mu_f, lam_f)[0], -0.5, 0.5,
               xtol=1e-17, rtol=1e-15)
    return np.diag(0.5 * (P(1 + d, mu_s, lam_s) + P(1 - d, mu_f, lam_f))).ravel()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_laminate16_solve_matches_exact_solution(precision):
    say("laminate16 solve", precision)
    case = M.laminate16_case()
    # the stress error of the converged state is set by the stopping tolerance
    # (the oracle itself is 5.7e-5 off at 2e-6 and 5.6e-6 off at 2e-7)
    tol = 1e-12 if precision == "fp64" else 2e-7
    s = gpu_solver([case["phase"]], case["materials"], case["loads"], precision,
                   rho0=case["rho0"], mu_ref=case["mu_ref"], tol_p=tol, tol_d=tol,
                   max_iter=3000, check_every=50)
    rc, it, status = s.solve()
    P, L = s.homogenized_stress(0)
    s.close()
    ref = laminate_exact(10.0, 100.0, 1.0, 10.0, 0.95)
    say("  iters", it, "rel P", rel(P, ref), "rel <Lambda>", rel(L, ref))
    assert rc == admm.OK
    assert rel(P, ref) <= (1e-10 if precision == "fp64" else 1e-5)


def test_laminate16_config_matches_oracle():
    """The benchmark's 16^3 configuration as stated: rho = 5, 200 iterations or
    residual < 1e-8."""
    case = M.laminate16_case()
    say("laminate16 config")
    s = gpu_solver([case["phase"]], case["materials"], case["loads"], "fp64",
                   rho0=5.0, mu_ref=5.5, tol_p=1e-8, tol_d=1e-8, max_iter=200, check_every=10)
    rc, it, status = s.solve()
    st = s.state(0)
    P, _ = s.homogenized_stress(0)
    s.close()
    u, F, L = O.initial_state(case["phase"].shape)
    p = O.params(max_iter=200, tol_p=1e-8, tol_d=1e-8, mu_ref=5.5, newton=O.newton_opts(**NEWTON64))
    r = O.admm_run(case["phase"], omats(case["materials"]), case["loads"][0].ravel(), p, u, F, L, 5.0)
    Po = O.mean_stress(case["phase"], omats(case["materials"]), F)
    say("  gpu iters", it[0], "oracle iters", r["iters"], "rel P", rel(P, Po))
    assert it[0] == r["iters"]
    assert rel(P, Po) <= 1e-10 and rel(st["F"], F) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_cells_solved_alone(precision):
    say("batch vs single", precision)
    shapes = [(16, 16, 16), (12, 24, 48), (32, 16, 8)]
    phases = [M.random_two_phase(sh, 0.3, seed=20 + k) for k, sh in enumerate(shapes)]
    Fbars = [M.random_fbar(0.05, seed=30 + k) for k in range(3)]
    kw = dict(rho0=6.0, mu_ref=4.0, adapt_rho=1, tol_p=1e-7, tol_d=1e-7, max_iter=60,
              check_every=7)
    s = gpu_solver(phases, MATS, Fbars, precision, **kw)
    rc, it, status = s.solve()
    batch = [s.state(k) for k in range(3)]
    Pb = [s.homogenized_stress(k)[0] for k in range(3)]
    s.close()
    for k in range(3):
        s1 = gpu_solver([phases[k]], MATS, [Fbars[k]], precision, **kw)
        rc1, it1, st1 = s1.solve()
        one = s1.state(0)
        P1 = s1.homogenized_stress(0)[0]
        s1.close()
        assert it1[0] == it[k]
        for f in ("u", "F", "Lambda"):
            assert np.array_equal(one[f], batch[k][f]), (k, f)
        assert np.array_equal(P1, Pb[k])


def test_set_load_warm_start_and_load_path():
    """Two load steps through admm_set_load against the oracle's two runs."""
    shape = (12, 16, 24)
    say("load path", shape)
    phase = M.random_two_phase(shape, 0.5, seed=40)
    loads = [np.diag([1.0, 1.0, 0.98]), np.diag([1.0, 1.0, 0.96])]
    s = gpu_solver([phase], MATS, [loads[0]], "fp64", rho0=8.0, mu_ref=4.0)
    s.step(5)
    s.set_load(0, loads[1])
    s.step(5)
    st = s.state(0)
    s.close()
    u, F, L = O.initial_state(shape)
    for Fb in loads:
        p = O.params(max_iter=5, fixed_iters=True, mu_ref=4.0, newton=O.newton_opts(**NEWTON64))
        O.admm_run(phase, omats(MATS), Fb.ravel(), p, u, F, L, 8.0)
    assert rel(st["u"], u) <= 1e-10 and rel(st["F"], F) <= 1e-10 and rel(st["Lambda"], L) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_domain_error_is_reported(precision):
    """A warm start with det F <= 0 is flagged, not hidden (both the Newton
    solve and the float step's closed form check it first)."""
    shape = (8, 8, 8)
    say("domain error", shape, precision)
    phase = np.zeros(shape, np.uint8)
    s = gpu_solver([phase], [M.neohooke(1.0, 1.0)], [np.eye(3)], precision, rho0=5.0)
    F = np.zeros((9,) + shape)
    F[0] = F[4] = 1.0
    F[8] = -0.5  # det F < 0 as warm start
    s.set_state(0, F=F)
    rc = s.local_step()
    s.close()
    assert rc == admm.EDOMAIN


def test_wavy_laminate_load_path_matches_oracle():
    """The wavy-laminate compression path at reduced scale: 32^3, stiff layers
    2 voxels thick with period 8, interfaces displaced by a sinusoid of
    amplitude 0.5 along x3, mu contrast 100, lambda = 10 mu; three load steps
    Fbar = diag(1, 1, 1 - 0.005 k), each solved to 1e-8 with the adaptive
    penalty, warm-started from the previous one."""
    phase = M.wavy_laminate(n=32, period=8, stiff=2, amp=0.5)
    mats = [M.neohooke(100.0, 1000.0), M.neohooke(1.0, 10.0)]
    loads = [np.diag([1.0, 1.0, 1.0 - 0.005 * k]) for k in (1, 2, 3)]
    mu_ref = 0.25 * 100.0 + 0.75
    kw = dict(rho0=10.0, rho_min=1.0, rho_max=100.0, adapt_rho=1, mu_ref=mu_ref,
              tol_p=1e-8, tol_d=1e-8, max_iter=600, check_every=5)
    s = gpu_solver([phase], mats, [loads[0]], "fp64", **kw)
    u, F, L = O.initial_state(phase.shape)
    rho = 10.0
    for k, Fb in enumerate(loads):
        say("wavy32 load step", k)
        if k:
            s.set_load(0, Fb)
        rc, it, status = s.solve()
        P, _ = s.homogenized_stress(0)
        p = O.params(max_iter=600, tol_p=1e-8, tol_d=1e-8, mu_ref=mu_ref, adapt_rho=True,
                     rho_min=1.0, rho_max=100.0, newton=O.newton_opts(**NEWTON64))
        r = O.admm_run(phase, omats(mats), Fb.ravel(), p, u, F, L, rho)
        rho = r["rho"]
        Po = O.mean_stress(phase, omats(mats), F)
        say("  gpu iters", it[0], "oracle iters", r["iters"], "rel P", rel(P, Po))
        assert status[0] == admm.OK and r["rc"] == O.OK
        assert it[0] == r["iters"]
        assert rel(P, Po) <= 1e-9
    st = s.state(0)
    s.close()
    assert rel(st["F"], F) <= 1e-9 and rel(st["u"], u) <= 1e-9


def test_laminate16_config_matches_golden():
    """The same configuration against the oracle's stored run
    (tests/golden/oracle_laminate16.json): iteration count, the first
    residuals and <P>."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "oracle_laminate16.json")) as f:
        g = json.load(f)
    case = M.laminate16_case()
    s = gpu_solver([case["phase"]], case["materials"], case["loads"], "fp64",
                   rho0=5.0, mu_ref=5.5, tol_p=1e-8, tol_d=1e-8, max_iter=200, check_every=10)
    rc, it, status = s.solve()
    P, _ = s.homogenized_stress(0)
    hp, hd, _ = s.history(0)
    s.close()
    say("laminate16 golden: iters", it[0], g["iters"], "rel P", rel(P, g["P_mean"]))
    assert it[0] == g["iters"]
    assert rel(P, np.array(g["P_mean"])) <= 1e-10
    n = len(g["r_p"])
    assert np.allclose(hp[:n], g["r_p"], rtol=1e-9, atol=0)
    assert np.allclose(hd[:n], g["r_d"], rtol=1e-9, atol=0)
