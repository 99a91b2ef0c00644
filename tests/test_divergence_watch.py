"""admm_solve's divergence watch, replayed on recorded residual histories on
the host (admm_divergence_check runs the rule the finalize kernel runs; no
GPU needed).

Sec. 4 reports that too small a penalty diverges. On the 16^3 laminate the
oracle's history at a fixed rho = 0.1 shows what that looks like: r_p falls
to about 2e-2, jumps to about 0.3 within a few dozen iterations and stays
there (no overflow, no NaN). The growth rule catches residuals that run away
by orders of magnitude; the stagnation rule (no halving of the merit for
stall_iters iterations) catches this case.
"""
import numpy as np
import pytest

import oracle as O
from paper_2010_06697_amd import admm, microstructure as M
from parity_util import omats


def check(r_p, r_d, **kw):
    p = admm.default_params(tol_p=1e-8, tol_d=1e-8, **kw)
    return admm.admm_divergence_check(p, r_p, r_d)


def test_converging_histories_are_never_stopped():
    k = np.arange(400)
    fast = 1e-2 * 0.9 ** k
    assert check(fast, fast) == -1
    # slow but steady: halves every ~138 iterations, within the window of 500
    slow = 1e-2 * 0.995 ** k
    assert check(slow, 0.5 * slow, stall_iters=500) == -1
    # adaptive-penalty jumps of r_d by the factor kappa = 1.3 are not growth
    jumpy = slow.copy()
    jumpy[50::40] *= 1.3 ** 3
    assert check(slow, jumpy) == -1


def test_growth_rule_fires_when_the_merit_runs_away():
    k = np.arange(60)
    r = 1e-3 * 1.5 ** k
    # merit 1e5 * 1.5^k against the smallest, the first: 1.5^18 > 1e3 > 1.5^17
    assert check(r, r, stall_iters=0) == 18
    assert check(r, r, stall_iters=0, div_growth=1e6) == 35
    assert check(r, r, stall_iters=0, div_growth=0.0) == -1


def test_stagnation_rule_fires_after_the_window():
    r = np.concatenate([1e-2 * 0.5 ** np.arange(10), np.full(600, 1e-2 * 0.5 ** 9)])
    # last halving at iteration 9: stopped at 9 + window
    assert check(r, r, div_growth=0.0, stall_iters=100) == 109
    assert check(r, r, div_growth=0.0, stall_iters=500) == 509
    assert check(r, r, div_growth=0.0, stall_iters=0) == -1
    # converged before the window ends: never stopped
    conv = r.copy()
    conv[50] = 1e-9
    assert check(conv, conv, div_growth=0.0, stall_iters=100) == -1


def test_rule_matches_its_definition_on_random_histories():
    rng = np.random.default_rng(4)
    for trial in range(20):
        n = 300
        rp = 10 ** rng.uniform(-5, -1, n)
        rd = 10 ** rng.uniform(-5, -1, n)
        g, w = [0.0, 10.0, 1e3][trial % 3], [0, 7, 40][trial % 3]
        best = ref = np.inf
        ref_it, want = 0, -1
        for it in range(n):
            m = max(rp[it] / 1e-8, rd[it] / 1e-8)
            best = min(best, m)
            if m <= 0.5 * ref:
                ref, ref_it = m, it
            if (g > 0 and m > g * best) or (w > 0 and it - ref_it >= w):
                want = it
                break
        assert check(rp, rd, div_growth=g, stall_iters=w) == want, trial


def test_small_penalty_history_of_the_oracle_is_stopped():
    case = M.laminate16_case()
    u, F, L = O.initial_state(case["phase"].shape)
    p = O.params(max_iter=300, fixed_iters=True, mu_ref=5.5,
                 newton=O.newton_opts(gtol=1e-14, step_tol=1e-10))
    r = O.admm_run(case["phase"], omats(case["materials"]), case["loads"][0].ravel(), p, u, F, L,
                   0.1)
    rp, rd = r["r_p"], r["r_d"]
    assert np.all(np.isfinite(rp)) and rp.max() > 5 * rp[:20].min()
    at = check(rp, rd, div_growth=1e3, stall_iters=100)
    assert 100 <= at < 300
    # the same history with the default penalty of the laminate converges
    u, F, L = O.initial_state(case["phase"].shape)
    r5 = O.admm_run(case["phase"], omats(case["materials"]), case["loads"][0].ravel(), p, u, F, L,
                    5.0)
    assert check(r5["r_p"], r5["r_d"], div_growth=1e3, stall_iters=100) == -1
