"""The Step 2 autotuner: it must leave the method's state alone, report a
valid configuration (tile widths it was compiled for, radix sequences of
2/3/4/8 whose product is the length), and the tuned transforms must still
reproduce the oracle's iterations (the choice changes only rounding)."""
import numpy as np
import pytest
import torch

from paper_2010_06697_amd import admm, microstructure as M
from parity_util import NEWTON64, gpu_solver, oracle_iterations, rel

pytestmark = pytest.mark.gpu

MATS = [M.neohooke(10.0, 40.0), M.neohooke(1.0, 4.0)]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotune_keeps_state_and_parity(precision):
    shapes = [(24, 18, 32), (16, 48, 12)]
    phases = [M.random_two_phase(sh, 0.35, seed=80 + k) for k, sh in enumerate(shapes)]
    Fbars = [M.random_fbar(0.04, seed=90 + k) for k in range(2)]
    s = gpu_solver(phases, MATS, Fbars, precision, rho0=6.0, mu_ref=4.0)
    s.step(2)
    before = [s.state(k) for k in range(2)]
    say("autotune", precision)
    cfg = s.autotune(reps=2)
    say("  ", cfg)
    d = 16 if precision == "fp32" else 8
    assert cfg["x_points"] in (256, 512, 1024)
    widths = (d // 4, d // 2, d, 2 * d)
    assert cfg["tile_y"] in widths and cfg["tile_z"] in widths
    assert sorted(cfg["plans"]) == sorted({n for sh in shapes for n in sh})
    for n, rad in cfg["plans"].items():
        assert set(rad) <= {2, 3, 4, 8} and int(np.prod(rad)) == n
    assert cfg["ms_tuned"] > 0 and cfg["ms_tuned"] <= 1.25 * cfg["ms_default"]
    assert admm.admm_autotune(s.ctx, 0)["plans"] == cfg["plans"]
    for k in range(2):
        after = s.state(k)
        for f in ("u", "F", "Lambda"):
            assert np.array_equal(after[f], before[k][f]), (k, f)
    s.step(3)
    got = [s.state(k) for k in range(2)]
    s.close()
    for k in range(2):
        u, F, L, _ = oracle_iterations(phases[k], MATS, Fbars[k], 5, 6.0, 4.0)
        eu, eF = rel(got[k]["u"], u), rel(got[k]["F"], F)
        say("  cell", k, "rel u F", eu, eF)
        tol = 1e-10 if precision == "fp64" else 2e-5
        assert eu <= tol and eF <= tol
