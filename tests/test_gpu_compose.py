"""The features compose: one batch with cells of different sizes that mix
the full LCE model (non-ideality, Frank, dissipation) with a stiff
inclusion, strain-controlled and mixed conditions, under the inexact local
step and captured graphs, gives every cell the same bits as a batch of that
cell alone; and one LCE cell under uniaxial stress (all components of <F>
but F_11 free) with the inexact step matches the oracle in double precision.
"""
import numpy as np
import pytest

import oracle as O
from paper_2010_06697_amd import admm, microstructure as M
from parity_util import NEWTON64, omats, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


MATS = [M.lce(1.0, 2.0, 100.0, alpha=0.1, frank=0.05, nu_F=0.2, nu_n=0.3), M.neohooke(10.0, 100.0)]
LOC = dict(local_ratio=0.3, local_chunk=1, local_passes=4)


def cell(n, seed, incl):
    g, dirs = M.voronoi_grains(n=n, n_grains=5, seed=seed)
    d0 = M.director_field(g, dirs)
    phase = np.zeros(g.shape, np.uint8)
    if incl:
        z, y, x = np.indices(phase.shape)
        c = (n - 1) / 2
        phase[(x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2 <= (n / 4) ** 2] = 1
    return phase, d0


CELLS = [(cell(16, 1, True), M.uniaxial_lce(1.15), [1, 2, 3, 4, 5, 6, 7, 8]),
         (cell(12, 2, False), M.uniaxial_lce(1.1), []),
         (cell(8, 3, True), M.uniaxial_lce(1.2), [8])]


def run(cells, precision="fp64"):
    p = admm.default_params(precision, rho0=10.0, mu_ref=1.0, dt=0.5, check_every=5, **LOC)
    s = admm.Solver([c[0][0] for c in cells], MATS, [c[1] for c in cells], p,
                    precision=precision, directors=[c[0][1] for c in cells],
                    directors0=[c[0][1] for c in cells])
    for k, c in enumerate(cells):
        if c[2]:
            s.set_free(k, c[2])
    s.step(10)
    out = [(s.state(k), s.fbar(k), s.homogenized_stress(k)[0]) for k in range(len(cells))]
    s.close()
    return out


def test_batch_of_mixed_features_equals_cells_alone():
    both = run(CELLS)
    for k, c in enumerate(CELLS):
        alone = run([c])[0]
        for f in ("u", "F", "Lambda", "director"):
            assert np.array_equal(both[k][0][f], alone[0][f]), (k, f)
        assert np.array_equal(both[k][1], alone[1]) and np.array_equal(both[k][2], alone[2])


def test_lce_uniaxial_stress_with_inexact_step_matches_oracle():
    (phase, d0), Fb, free = CELLS[0]
    g = run([CELLS[0]])[0]
    u, F, L = O.initial_state(phase.shape)
    n = d0.copy()
    op = O.params(max_iter=10, fixed_iters=True, mu_ref=1.0, dt=0.5, free=free,
                  newton=O.newton_opts(**NEWTON64), **LOC)
    r = O.admm_run(phase, omats(MATS), Fb.ravel(), op, u, F, L, 10.0, director_field=n,
                   director0=d0)
    Po = O.mean_stress(phase, omats(MATS), F, director_field=n, director0=d0)
    st, Fbar, P = g
    errs = {k: rel(st[k], o) for k, o in (("u", u), ("F", F), ("Lambda", L), ("director", n))}
    print("rel", errs, "P", rel(P, Po), "Fbar", rel(Fbar, r["Fbar"]), flush=True)
    assert errs["u"] <= 1e-10 and errs["F"] <= 1e-10 and errs["Lambda"] <= 1e-10
    assert errs["director"] <= 1e-9
    assert rel(P, Po) <= 1e-10 and rel(Fbar, r["Fbar"]) <= 1e-12
