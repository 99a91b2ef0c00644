"""GPU parity of the full LCE model of Sec. 5.1: the non-ideality with the
cross-link directors n0, the Frank term with the neighbours' directors from
the previous iteration, and the dissipation of F and of the director over a
time step dt, on the 16^3 polydomain with a stiff neo-Hookean inclusion.

Whole iterations in double precision against the oracle (1e-10 relative on
u, F, Lambda and <P>, 1e-9 on the directors, as for the ideal model), over a
load step change (the dissipation's start-of-step fields are taken again),
the orientation tensor, and <P> in float.
"""
import numpy as np
import pytest

import oracle as O
from paper_2010_06697_amd import admm, microstructure as M
from parity_util import NEWTON64, omats, rel

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


TERMS = {
    "nonideal": dict(alpha=0.1),
    "frank": dict(frank=0.05),
    "dissipative": dict(nu_F=0.2, nu_n=0.3),
    "all": dict(alpha=0.1, frank=0.05, nu_F=0.2, nu_n=0.3),
}
DT = 0.5


def case(terms):
    g, dirs = M.voronoi_grains(n=16, n_grains=6, seed=7)
    d0 = M.director_field(g, dirs)
    phase = np.zeros(g.shape, np.uint8)
    z, y, x = np.indices(phase.shape)
    phase[(x - 7.5) ** 2 + (y - 7.5) ** 2 + (z - 7.5) ** 2 <= 16.0] = 1
    mats = [M.lce(1.0, 2.0, 100.0, **terms), M.neohooke(10.0, 100.0)]
    return phase, d0, mats


def run_gpu(phase, d0, mats, loads, n_iter, precision="fp64", graph=1):
    p = admm.default_params(precision, rho0=10.0, mu_ref=1.0, dt=DT, use_graph=graph,
                            check_every=n_iter)
    s = admm.Solver([phase], mats, [loads[0]], p, precision=precision, directors=[d0],
                    directors0=[d0])
    for k, Fb in enumerate(loads):
        if k:
            s.set_load(0, Fb)
        rc, _, _, _ = s.step(n_iter)
        assert rc == admm.OK
    st = s.state(0)
    P, _ = s.homogenized_stress(0)
    S = s.orientation(0)
    s.close()
    return st, P, S


def run_oracle(phase, d0, mats, loads, n_iter):
    u, F, L = O.initial_state(phase.shape)
    n = d0.copy()
    rho = 10.0
    for Fb in loads:
        p = O.params(max_iter=n_iter, fixed_iters=True, mu_ref=1.0, dt=DT,
                     newton=O.newton_opts(**NEWTON64))
        r = O.admm_run(phase, omats(mats), np.asarray(Fb).ravel(), p, u, F, L, rho,
                       director_field=n, director0=d0)
        rho = r["rho"]
    P = O.mean_stress(phase, omats(mats), F, director_field=n, director0=d0)
    S = O.orientation(phase, omats(mats), n)
    return dict(u=u, F=F, Lambda=L, director=n), P, S


@pytest.mark.parametrize("name", list(TERMS))
def test_full_lce_iterations_match_oracle_fp64(name):
    say("full lce iterations", name)
    phase, d0, mats = case(TERMS[name])
    loads = [M.uniaxial_lce(1.2)]
    st, P, S = run_gpu(phase, d0, mats, loads, 4)
    o, Po, So = run_oracle(phase, d0, mats, loads, 4)
    errs = {k: rel(st[k], o[k]) for k in ("u", "F", "Lambda", "director")}
    say("  rel", errs, "P", rel(P, Po), "S", np.max(np.abs(S - So)))
    assert errs["u"] <= 1e-10 and errs["F"] <= 1e-10 and errs["Lambda"] <= 1e-10
    assert errs["director"] <= 1e-9
    assert rel(P, Po) <= 1e-10
    assert np.max(np.abs(S - So)) <= 1e-10


def test_full_lce_load_steps_match_oracle_fp64():
    """Two time steps: the dissipation's F^n and n^n are the fields at the
    start of each step (admm_set_load / a new oracle call)."""
    phase, d0, mats = case(TERMS["all"])
    loads = [M.uniaxial_lce(1.1), M.uniaxial_lce(1.2)]
    st, P, _ = run_gpu(phase, d0, mats, loads, 3, graph=0)
    o, Po, _ = run_oracle(phase, d0, mats, loads, 3)
    errs = {k: rel(st[k], o[k]) for k in ("u", "F", "Lambda", "director")}
    say("  rel", errs, "P", rel(P, Po))
    assert errs["u"] <= 1e-10 and errs["F"] <= 1e-10 and errs["Lambda"] <= 1e-10
    assert errs["director"] <= 1e-9
    assert rel(P, Po) <= 1e-10


def test_full_lce_terms_change_the_state():
    """Guard that the parity cases exercise the terms: the ideal model's
    state after the same iterations is far from the full model's."""
    phase, d0, mats = case(TERMS["all"])
    loads = [M.uniaxial_lce(1.2)]
    st, P, _ = run_gpu(phase, d0, mats, loads, 4)
    st0, P0, _ = run_gpu(phase, d0, [M.lce(1.0, 2.0, 100.0), mats[1]], loads, 4)
    assert rel(st["F"], st0["F"]) >= 1e-4 and rel(P, P0) >= 1e-4


def test_full_lce_fp32_homogenized_stress():
    phase, d0, mats = case(TERMS["all"])
    loads = [M.uniaxial_lce(1.2)]
    _, P, _ = run_gpu(phase, d0, mats, loads, 10, precision="fp32")
    _, Po, _ = run_oracle(phase, d0, mats, loads, 10)
    say("  fp32 rel P", rel(P, Po))
    assert rel(P, Po) <= 1e-5
