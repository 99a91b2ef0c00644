"""Every Step 2 launch configuration the library can be given (admm_set_tuning)
computes the projection of Step 2: on thin cells whose one long edge is 48,
96 or 256 along x1, x2 or x3, each radix sequence of that length (every
order of every split into radix 8, 4, 2 and 3 stages, at most 8 stages),
each compiled tile width of the x2 and x3 passes (and the register-resident
width where every length along the axis is supported: 256 in double; 32, 48,
64, 96, 128 and 256 in float; refused on the others) and each x1
workgroup size
give the oracle's projection (Sec. 2.3) to 1e-12 in double and 2e-5 in
float. Invalid configurations are refused without a change; the autotuner's
persisted table (ADMM_AUTOTUNE_CACHE) is written and read back.
"""
import itertools
import os

import numpy as np
import pytest

import oracle as O
from paper_2010_06697_amd import admm, microstructure as M
from parity_util import random_state, rel

pytestmark = pytest.mark.gpu

MATS = [M.neohooke(10.0, 40.0), M.neohooke(1.0, 4.0)]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def radix_orders(n):
    """Every distinct order of every split of n = 2^a 3^b into radix-8, -4,
    at most one radix-2, and radix-3 stages (at most 8 stages)."""
    twos = threes = 0
    while n % 2 == 0:
        n //= 2
        twos += 1
    while n % 3 == 0:
        n //= 3
        threes += 1
    out = set()
    for e8 in range(twos // 3 + 1):
        for e2 in (0, 1):
            left = twos - 3 * e8 - e2
            if left < 0 or left % 2:
                continue
            r = [8] * e8 + [4] * (left // 2) + [2] * e2 + [3] * threes
            if 0 < len(r) <= 8:
                out.update(itertools.permutations(r))
    return sorted(out)


def shape_for(n, axis):
    s = [4, 4, 4]
    s[2 - axis] = n  # numpy shape (n3, n2, n1)
    return tuple(s)


def projection(s, precision, shape, ref):
    s.project_step()
    return rel(s.state(0)["u_prev"], ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [48, 96, 256])
def test_every_configuration_projects(precision, n):
    tol = 1e-12 if precision == "fp64" else 2e-5
    B = 8 if precision == "fp64" else 16  # default tile width (128 bytes of complex)
    for axis in range(3):
        shape = shape_for(n, axis)
        phase = M.random_two_phase(shape, 0.4, seed=axis)
        u, F, L = random_state(shape, seed=7 + axis)
        rho = 2.5
        ref = O.project(F - L / rho)
        p = admm.default_params(precision, rho0=rho)
        s = admm.Solver([phase], MATS, [np.eye(3)], p, precision=precision)
        s.set_state(0, u=0 * u, F=F, Lambda=L)
        worst, count = 0.0, 0
        for rad in radix_orders(n):
            s.set_tuning(B, B, 1024 if precision == "fp32" else 256, {n: list(rad)})
            worst = max(worst, projection(s, precision, shape, ref))
            count += 1
        csz = 16 if precision == "fp64" else 8
        n3, n2, _ = shape
        for ty, tz in [(B // 4, B), (B // 2, B), (2 * B, B), (B, B // 4), (B, B // 2), (B, 2 * B)]:
            if 2 * n2 * ty * csz > 65536 or 2 * n3 * tz * csz > 65536:
                with pytest.raises(admm.AdmmError):  # beyond 64 KiB of LDS: refused
                    s.set_tuning(ty, tz, 256, {})
                continue
            s.set_tuning(ty, tz, 256, {})
            worst = max(worst, projection(s, precision, shape, ref))
            count += 1
        for ty, tz, ax in [(admm.TILE_REG16, B, 1), (B, admm.TILE_REG16, 2)]:
            if axis != ax or (precision == "fp64" and n != 256):
                with pytest.raises(admm.AdmmError):  # length along the axis not supported
                    s.set_tuning(ty, tz, 256, {})
                continue
            s.set_tuning(ty, tz, 256, {})
            worst = max(worst, projection(s, precision, shape, ref))
            count += 1
        for pts in (256, 512, 1024):
            s.set_tuning(B, B, pts, {})
            worst = max(worst, projection(s, precision, shape, ref))
            count += 1
        s.close()
        say(f"  n={n} axis={axis} {precision}: {count} configurations, worst rel {worst:.2e}")
        assert worst <= tol


def test_invalid_configurations_are_refused(tmp_path):
    phase = M.random_two_phase((4, 4, 48), 0.4, seed=1)
    s = admm.Solver([phase], MATS, [np.eye(3)], admm.default_params("fp64"), precision="fp64")
    before = s.autotune(reps=0)
    for bad in [dict(tile_y=3, tile_z=8, x_points=256), dict(tile_y=8, tile_z=8, x_points=300),
                dict(tile_y=8, tile_z=8, x_points=256, plans={48: [8, 8]}),
                dict(tile_y=8, tile_z=8, x_points=256, plans={48: [8, 5]}),
                dict(tile_y=8, tile_z=8, x_points=256, plans={48: [16, 3]}),
                dict(tile_y=8, tile_z=8, x_points=256, plans={64: [8, 8]})]:
        with pytest.raises(admm.AdmmError) as e:
            s.set_tuning(**bad)
        assert e.value.code == admm.EINVAL
    assert s.autotune(reps=0) == before
    # the persisted table: written by the first tuning, applied by the second
    cache = tmp_path / "tune.txt"
    os.environ["ADMM_AUTOTUNE_CACHE"] = str(cache)
    try:
        first = s.autotune(reps=1)
        assert cache.exists() and cache.read_text().startswith("fp64|48x4x4 ")
        s.set_tuning(2, 2, 1024, {48: [3, 4, 4]})
        again = s.autotune(reps=1)
        assert again["plans"] == first["plans"] and again["tile_y"] == first["tile_y"]
        assert again["x_points"] == first["x_points"]
        assert len(cache.read_text().splitlines()) == 1
    finally:
        del os.environ["ADMM_AUTOTUNE_CACHE"]
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_register_resident_passes_on_both_column_axes(precision):
    """x2 and x3 both of length 256 at the register-resident tile width:
    both column passes (the forward and inverse x2 transforms and the x3
    transform with the Fourier-space solve) run register resident in one
    Step 2, against the oracle and against the tiled passes; x1 = 6 leaves
    partial 16-column groups (m1 = 4 columns per row)."""
    tol = 1e-12 if precision == "fp64" else 2e-5
    B = 8 if precision == "fp64" else 16
    shape = (256, 256, 6)
    phase = M.random_two_phase(shape, 0.4, seed=11)
    u, F, L = random_state(shape, seed=12)
    rho = 2.5
    ref = O.project(F - L / rho)
    p = admm.default_params(precision, rho0=rho)
    s = admm.Solver([phase], MATS, [np.eye(3)], p, precision=precision)
    s.set_state(0, u=0 * u, F=F, Lambda=L)
    s.set_tuning(admm.TILE_REG16, admm.TILE_REG16, 256, {})
    got = s.autotune(reps=0)
    assert got["tile_y"] == admm.TILE_REG16 and got["tile_z"] == admm.TILE_REG16
    err = projection(s, precision, shape, ref)
    u_reg = s.state(0)["u_prev"]
    s.set_tuning(B, B, 256, {})
    err_tiled = projection(s, precision, shape, ref)
    d = rel(u_reg, s.state(0)["u_prev"])
    s.close()
    say(f"  register-resident x2 and x3, {precision}: rel {err:.2e} (tiled {err_tiled:.2e}, apart {d:.2e})")
    assert err <= tol and err_tiled <= tol and d <= tol


def test_register_resident_passes_on_a_mixed_batch():
    """Cells of the lengths 32, 48, 64, 96, 128 and 256 along x2 and x3 in one
    float batch: both column passes at the register-resident tile width (a
    workgroup takes 256 / T columns of one cell, T threads per column; the
    launch holds cells of 12, 16 and 24 points per thread) against the oracle
    per cell and against the tiled passes; short x1 lengths leave partial
    column groups (x1 lengths 4 to 18: 3 to 10 columns per row)."""
    shapes = [(32, 96, 6), (96, 48, 4), (48, 32, 12), (64, 128, 8), (128, 64, 18), (256, 256, 4)]
    phases = [M.random_two_phase(sh, 0.4, seed=20 + k) for k, sh in enumerate(shapes)]
    rho = 2.5
    p = admm.default_params("fp32", rho0=rho)
    s = admm.Solver(phases, MATS, [np.eye(3)] * len(shapes), p, precision="fp32")
    refs = []
    for k, sh in enumerate(shapes):
        u, F, L = random_state(sh, seed=40 + k)
        refs.append(O.project(F - L / rho))
        s.set_state(k, u=0 * u, F=F, Lambda=L)
    s.set_tuning(admm.TILE_REG16, admm.TILE_REG16, 256, {})
    got = s.autotune(reps=0)
    assert got["tile_y"] == admm.TILE_REG16 and got["tile_z"] == admm.TILE_REG16
    s.project_step()
    u_reg = [s.state(k)["u_prev"] for k in range(len(shapes))]
    s.set_tuning(16, 16, 256, {})
    s.project_step()
    worst = 0.0
    for k, sh in enumerate(shapes):
        e = rel(u_reg[k], refs[k])
        d = rel(u_reg[k], s.state(k)["u_prev"])
        say(f"  {sh}: rel {e:.2e} (apart from tiled {d:.2e})")
        worst = max(worst, e, d)
    s.close()
    assert worst <= 2e-5
