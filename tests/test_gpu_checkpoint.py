"""Checkpoint and resume through admm_get_state / admm_set_state (Algorithm
1 carries the iteration state from one iteration and load step to the next):
a context restored from a checkpoint continues bit for bit as the original
(fields, penalty, residual history, Newton counters), with the autotuned
Step 2 configuration carried along, under admm_step and admm_solve, for the
neo-Hookean cells of both precisions and the full LCE model (director,
lagged directors, start-of-step copies). Mismatched blobs are refused with
nothing changed.
"""
import numpy as np
import pytest

from paper_2010_06697_amd import admm, microstructure as M

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


MATS = [M.neohooke(10.0, 40.0), M.neohooke(1.0, 4.0)]


def same(sa, sb, keys=("u", "F", "Lambda")):
    for k in keys:
        assert np.array_equal(sa[k], sb[k]), k


def neo_solver(precision, shape=(8, 12, 16), seed=1):
    phase = M.random_two_phase(shape, 0.4, seed=seed)
    p = admm.default_params(precision, rho0=8.0, mu_ref=4.0, adapt_rho=1, tol_p=1e-7,
                            tol_d=1e-7, max_iter=400)
    return admm.Solver([phase, M.random_two_phase((6, 8, 8), 0.5, seed=seed + 1)], MATS,
                       [M.random_fbar(0.03, seed=seed), M.random_fbar(0.02, seed=seed + 2)], p,
                       precision=precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_resume_step_is_bitwise(precision):
    say("checkpoint step", precision)
    a = neo_solver(precision)
    a.autotune(reps=1)
    a.step(7)
    blob = a.checkpoint()
    rc, rp, rd, rho = a.step(5)
    b = neo_solver(precision)  # fresh context: zero state, default tuning
    b.restore(blob)
    rc2, rp2, rd2, rho2 = b.step(5)
    for r in range(2):
        same(a.state(r), b.state(r))
        ha, hb = a.history(r), b.history(r)
        assert len(ha[0]) == 12 and all(np.array_equal(x, y) for x, y in zip(ha, hb))
        assert a.info(r) == b.info(r)
    assert np.array_equal(rp, rp2) and np.array_equal(rd, rd2) and np.array_equal(rho, rho2)
    assert a.autotune(reps=0)["plans"] == b.autotune(reps=0)["plans"]
    a.close()
    b.close()


def test_resume_solve_after_a_new_load_is_bitwise():
    say("checkpoint solve")
    a = neo_solver("fp64", seed=3)
    a.solve()
    a.set_load(0, M.random_fbar(0.05, seed=9))
    a.step(3)
    blob = a.checkpoint()
    rca, ita, sta = a.solve()
    b = neo_solver("fp64", seed=3)
    b.restore(blob)
    rcb, itb, stb = b.solve()
    assert rca == rcb and np.array_equal(ita, itb) and np.array_equal(sta, stb)
    for r in range(2):
        same(a.state(r), b.state(r))
        assert np.array_equal(a.homogenized_stress(r)[0], b.homogenized_stress(r)[0])
    a.close()
    b.close()


def test_resume_full_lce_model_is_bitwise():
    say("checkpoint lce")
    g, d = M.voronoi_grains(n=12, n_grains=4, seed=2)
    n0 = M.director_field(g, d)
    phase = np.zeros(g.shape, np.uint8)
    mats = [M.lce(1.0, 2.0, 50.0, alpha=0.1, frank=0.05, nu_F=0.1, nu_n=0.1)]

    def solver():
        p = admm.default_params("fp32", rho0=10.0, mu_ref=1.0, dt=0.5)
        return admm.Solver([phase], mats, [M.uniaxial_lce(1.05)], p, precision="fp32",
                           directors=[n0], directors0=[n0])

    a = solver()
    a.step(4)
    a.set_load(0, M.uniaxial_lce(1.1))
    a.step(2)
    blob = a.checkpoint()
    a.step(3)
    b = solver()
    b.restore(blob)
    b.step(3)
    same(a.state(0), b.state(0), keys=("u", "F", "Lambda", "director"))
    assert all(np.array_equal(x, y) for x, y in zip(a.history(0), b.history(0)))
    a.close()
    b.close()


def test_mismatched_blobs_are_refused():
    a = neo_solver("fp64")
    a.step(2)
    blob = a.checkpoint()
    st = a.state(0)
    other = admm.Solver([M.random_two_phase((8, 8, 8), 0.4, seed=1)], MATS, [np.eye(3)],
                        admm.default_params("fp64"), precision="fp64")
    for bad in (blob[:-8], blob + b"\0" * 8, b"X" + blob[1:]):
        with pytest.raises(admm.AdmmError) as e:
            a.restore(bad)
        assert e.value.code == admm.EINVAL
    with pytest.raises(admm.AdmmError) as e:
        other.restore(blob)
    assert e.value.code == admm.EINVAL
    f32 = neo_solver("fp32")
    with pytest.raises(admm.AdmmError) as e:
        f32.restore(blob)
    assert e.value.code == admm.EINVAL
    same(st, a.state(0))
    for s in (a, other, f32):
        s.close()
