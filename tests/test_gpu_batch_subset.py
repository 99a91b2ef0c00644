"""The 128-cell batch of the benchmark, as the benchmark runs it (float with
double reductions, rho0 = rho_min = 30, rho_max = 100, adaptive, one load step
to tol 1e-6), on a subset of four of its cells, the first of each edge length
32, 48, 64, 96: solved in one batch (one launch per pass over all four), each
cell ends exactly as when solved alone (fields, iterations, <P>, residual
history), bit for bit.
"""
import numpy as np
import pytest

from paper_2010_06697_amd import admm, microstructure as M

pytestmark = pytest.mark.gpu

RHO0, RHO_MIN, RHO_MAX = 30.0, 30.0, 100.0


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def params():
    return admm.default_params("fp32", rho0=RHO0, rho_min=RHO_MIN, rho_max=RHO_MAX, adapt_rho=1,
                               mu_ref=5.0, tol_p=1e-6, tol_d=1e-6, max_iter=2000, check_every=20)


def test_batch_subset_equals_cells_alone():
    cells = M.rve_batch(128)
    pick = []
    for n in (32, 48, 64, 96):
        pick.append(next(c for c in cells if c["n"] == n))
    mats = M.rve_batch_materials()
    say("batch subset: edges", [c["n"] for c in pick])
    b = admm.Solver([c["phase"] for c in pick], mats, [c["Fbar"] for c in pick], params(),
                    precision="fp32")
    rc, it, st = b.solve()
    batch = [(b.state(r), b.homogenized_stress(r)[0], b.history(r)) for r in range(4)]
    b.close()
    say("  batch iterations", it, "status", st)
    assert np.all(st == admm.OK)
    for r, c in enumerate(pick):
        s = admm.Solver([c["phase"]], mats, [c["Fbar"]], params(), precision="fp32")
        rc1, it1, st1 = s.solve()
        alone = (s.state(0), s.homogenized_stress(0)[0], s.history(0))
        s.close()
        assert it1[0] == it[r] and st1[0] == st[r]
        for k in ("u", "F", "Lambda"):
            assert np.array_equal(alone[0][k], batch[r][0][k]), (r, k)
        assert np.array_equal(alone[1], batch[r][1])
        assert all(np.array_equal(x, y) for x, y in zip(alone[2], batch[r][2]))
