"""The allocation-free Bloch entry point (admm_bloch_static) against the
allocating one (admm_bloch): the same kernels in the same order on the same
inputs, so the modulus, rho sigma, the iteration count and the mode agree
(to 1e-10 relative, the double-precision parity bar; in practice bit for
bit). Two calls in a row, the second on a smaller cell, so that what the
first call leaves in the fixed work array cannot leak into the second; and
a cell beyond the array's size is refused before any work.
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


MATS = [M.neohooke(10.0, 20.0), M.neohooke(1.0, 2.0)]


def field(shape, amp, seed):
    rng = np.random.default_rng(seed)
    F = np.zeros((9,) + shape)
    F[[0, 4, 8]] = 1.0
    return F + amp * rng.standard_normal(F.shape)


def start(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape)


def both(shape, amp, rho, max_iter, seed):
    phase = M.random_two_phase(shape, 0.5, seed=seed)
    F = field(shape, amp, seed + 1)
    n3, n2, n1 = shape
    omega = np.array([2 * np.pi / (2 * n1), 2 * np.pi / (2 * n2), 0.2])
    p0 = start(shape, seed + 2)
    s = admm.Solver([phase], MATS, [np.eye(3)], admm.default_params("fp64"), precision="fp64")
    s.set_state(0, F=F)
    st = s.bloch_static(0, omega, rho, p0, tol=1e-10, max_iter=max_iter)
    al = s.bloch(0, omega, rho, p0, tol=1e-10, max_iter=max_iter)
    s.close()
    return st, al


def check(st, al):
    say("  static beta", st["beta"], "alloc beta", al["beta"], "iters", st["iters"], al["iters"])
    assert st["status"] == al["status"]
    assert st["iters"] == al["iters"]
    assert abs(st["beta"] - al["beta"]) <= 1e-10 * max(1.0, abs(al["beta"]))
    assert abs(st["sigma_rho"] - al["sigma_rho"]) <= 1e-10 * max(1.0, abs(al["beta"]))
    d = np.max(np.abs(st["p"] - al["p"])) / np.max(np.abs(al["p"]))
    assert d <= 1e-10


def test_static_matches_allocating_two_calls():
    say("no-alloc bloch: 12x16x8 then 8x8x6")
    st, al = both((8, 16, 12), 0.05, 40.0, 20000, seed=11)
    assert al["status"] == admm.OK
    check(st, al)
    st, al = both((6, 8, 8), 0.1, 80.0, 20000, seed=21)
    assert al["status"] == admm.OK
    check(st, al)


def test_static_refuses_cells_beyond_the_array():
    cap = admm.admm_bloch_static_max_bytes()
    assert cap == 128 << 20
    shape = (48, 64, 64)  # 196608 voxels, about 180 MiB of work buffers
    say("no-alloc bloch: size refusal", shape)
    phase = np.zeros(shape, np.uint8)
    s = admm.Solver([phase], MATS, [np.eye(3)], admm.default_params("fp64"), precision="fp64")
    p0 = np.ones((3,) + shape, complex)
    with pytest.raises(admm.AdmmError) as e:
        s.bloch_static(0, [0.1, 0.2, 0.3], 20.0, p0)
    assert e.value.code == admm.ENOMEM
    s.close()
