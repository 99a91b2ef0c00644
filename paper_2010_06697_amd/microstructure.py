"""Seeded synthetic microstructures and load paths.

This module is geometry and bookkeeping only: phase maps, material tables,
macroscopic load paths and director fields. It holds none of the method's
arithmetic, so both the GPU path and the CPU oracle are fed from it.

The paper's own microstructures (2D circular inclusions on 1024^2-2048^2
grids, Sec. 4; LCE polydomains on 128^3, Sec. 5) come with no data; these
seeded 3D stand-ins have the shapes of the five benchmark workloads:

  laminate16      two-phase laminate, 16^3, layers normal to x1 (8 + 8)
  wavy_laminate64 64^3 laminate, stiff 4 / period 16, interfaces perturbed by a
                  0.5-voxel sinusoid of wavelength 64 along x3
  fibres256       256^3 periodic fibres along x3 (radius 8, area fraction 0.3,
                  minimum gap 2) by random sequential addition
  rve_batch       128 cells, edges in {32, 48, 64, 96}, random (overlapping)
                  spheres of radius 3-8 to a volume fraction U(0.1, 0.4)
  lce_polydomain  256^3 periodic Voronoi grains (1000 seeds) with random
                  unit directors

Arrays are (n3, n2, n1) uint8 phase maps, x1 fastest. Materials are dicts
{"model": "neohooke"|"lce", "mu", "lam", "a", "kappa"}. Macroscopic gradients
are 3x3 float64 arrays (row-major F_iJ).
"""
from __future__ import annotations

import numpy as np

SOFT_NEOHOOKE = {"model": "neohooke", "mu": 1.0, "lam": 10.0, "a": 1.0, "kappa": 0.0}


def neohooke(mu: float, lam: float) -> dict:
    return {"model": "neohooke", "mu": float(mu), "lam": float(lam), "a": 1.0, "kappa": 0.0}


def lce(mu: float, a: float, kappa: float, alpha: float = 0.0, frank: float = 0.0,
        nu_F: float = 0.0, nu_n: float = 0.0) -> dict:
    """LCE phase; alpha, frank, nu_F, nu_n: the non-ideality, Frank and
    dissipation terms of the full model (0: off)."""
    d = {"model": "lce", "mu": float(mu), "lam": 0.0, "a": float(a), "kappa": float(kappa)}
    for k, v in (("alpha", alpha), ("frank", frank), ("nu_F", nu_F), ("nu_n", nu_n)):
        if v:
            d[k] = float(v)
    return d


# ----------------------------------------------------------------------------
# laminate16: 16^3, stiff iff k1 < 8
# ----------------------------------------------------------------------------

def laminate(n: int = 16, n_stiff: int = 8, shape=None) -> np.ndarray:
    """Phase 0 (stiff) where k1 < n_stiff, phase 1 (soft) elsewhere."""
    n3, n2, n1 = shape if shape is not None else (n, n, n)
    ph = np.ones((n3, n2, n1), np.uint8)
    ph[:, :, :n_stiff] = 0
    return ph


def laminate16_case():
    return {
        "name": "laminate16",
        "phase": laminate(16, 8),
        "materials": [neohooke(10.0, 100.0), neohooke(1.0, 10.0)],
        "loads": [np.diag([1.0, 1.0, 0.95])],
        "rho0": 5.0,
        "mu_ref": 5.5,
        "max_iter": 200,
        "tol": 1e-8,
    }


# ----------------------------------------------------------------------------
# wavy_laminate64
# ----------------------------------------------------------------------------

def wavy_laminate(n: int = 64, period: int = 16, stiff: int = 4, amp: float = 0.5,
                  seed: int = 2) -> np.ndarray:
    """Stiff iff (k1 - d(k3)) mod period in [0, stiff), d = amp sin(2 pi k3/n + phi0),
    sampled at integer coordinates; phi0 ~ U[0, 2 pi) from the seed."""
    rng = np.random.default_rng(seed)
    phi0 = rng.uniform(0.0, 2.0 * np.pi)
    k3 = np.arange(n)[:, None, None]
    k1 = np.arange(n)[None, None, :]
    d = amp * np.sin(2.0 * np.pi * k3 / n + phi0)
    s = np.mod(k1 - d, period)
    stiff_mask = (s >= 0.0) & (s < stiff)
    ph = np.where(stiff_mask, 0, 1).astype(np.uint8)
    return np.ascontiguousarray(np.broadcast_to(ph, (n, n, n)))


def wavy_laminate64_case():
    return {
        "name": "wavy_laminate64",
        "phase": wavy_laminate(),
        "materials": [neohooke(100.0, 1000.0), neohooke(1.0, 10.0)],
        "loads": [np.diag([1.0, 1.0, 1.0 - 0.005 * k]) for k in range(1, 31)],
        "rho0": 10.0,
        "mu_ref": 0.25 * 100.0 + 0.75 * 1.0,
        "tol": 1e-7,
    }


# ----------------------------------------------------------------------------
# fibres256
# ----------------------------------------------------------------------------

def fibre_centres(n: int = 256, radius: float = 8.0, gap: float = 2.0,
                  fraction: float = 0.30, seed: int = 3, max_reject: int = 1_000_000):
    """Random sequential addition of periodic fibre axes (c1, c2) ~ U[0, n)^2,
    accepted when the minimum-image distance to every accepted axis is at least
    2 radius + gap; stops once the voxel-centre area fraction reaches `fraction`."""
    rng = np.random.default_rng(seed)
    centres: list[tuple[float, float]] = []
    dmin = 2.0 * radius + gap
    covered = np.zeros((n, n), bool)
    kc = np.arange(n) + 0.5
    rejects = 0
    while covered.mean() < fraction:
        c = rng.uniform(0.0, n, size=2)
        ok = True
        for (a, b) in centres:
            dx = abs(c[0] - a)
            dx = min(dx, n - dx)
            dy = abs(c[1] - b)
            dy = min(dy, n - dy)
            if dx * dx + dy * dy < dmin * dmin:
                ok = False
                break
        if not ok:
            rejects += 1
            if rejects > max_reject:
                raise RuntimeError("fibre packing jammed before the target fraction")
            continue
        centres.append((float(c[0]), float(c[1])))
        dx = np.abs(kc[None, :] - c[0])
        dx = np.minimum(dx, n - dx)
        dy = np.abs(kc[:, None] - c[1])
        dy = np.minimum(dy, n - dy)
        covered |= dx * dx + dy * dy < radius * radius
    return np.array(centres), covered


def fibres(n: int = 256, radius: float = 8.0, gap: float = 2.0, fraction: float = 0.30,
           seed: int = 3, n3: int | None = None) -> np.ndarray:
    """Fibres (phase 0) along x3 in a matrix (phase 1). The (x1, x2) section is
    n x n; the extrusion length is n3 (default n)."""
    _, covered = fibre_centres(n, radius, gap, fraction, seed)
    # covered is indexed [k2, k1]
    sec = np.where(covered, 0, 1).astype(np.uint8)
    n3 = n if n3 is None else n3
    return np.ascontiguousarray(np.broadcast_to(sec, (n3, n, n)))


def simple_shear(gamma: float) -> np.ndarray:
    F = np.eye(3)
    F[0, 1] = gamma
    return F


def fibres256_case(n: int = 256, n3: int | None = None):
    return {
        "name": "fibres256",
        "phase": fibres(n=n, n3=n3),
        "materials": [neohooke(50.0, 500.0), neohooke(1.0, 10.0)],
        "loads": [simple_shear(0.01 * k) for k in range(1, 11)],
        "rho0": 10.0,
        "rho_min": 1.0,
        "rho_max": 50.0,
        "mu_ref": 0.3 * 50.0 + 0.7 * 1.0,
        "tol_fp32": 1e-6,
        "tol_fp64": 1e-8,
    }


# ----------------------------------------------------------------------------
# rve_batch: 128 cells of uneven size with spherical inclusions
# ----------------------------------------------------------------------------

def sphere_inclusions(n: int, rng: np.random.Generator, fraction: float,
                      rmin: float = 3.0, rmax: float = 8.0) -> np.ndarray:
    """Random overlapping periodic spheres (phase 0) in a matrix (phase 1),
    added until the voxel volume fraction reaches `fraction`."""
    inc = np.zeros((n, n, n), bool)
    count = 0
    while count < fraction * inc.size:
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0.0, n, size=3)  # (x1, x2, x3)
        # voxels whose centre k + 1/2 can lie within r of c, wrapped periodically
        idx, dd = [], []
        for a in range(3):
            k = np.arange(int(np.floor(c[a] - r - 1)), int(np.ceil(c[a] + r + 1)) + 1)
            idx.append(np.mod(k, n))
            dd.append(k + 0.5 - c[a])
        dist2 = (dd[2][:, None, None] ** 2 + dd[1][None, :, None] ** 2
                 + dd[0][None, None, :] ** 2)
        block = np.ix_(idx[2], idx[1], idx[0])
        inc[block] |= dist2 < r * r
        count = int(inc.sum())
    return np.where(inc, 0, 1).astype(np.uint8)


def rve_batch(count: int = 128, sizes=(32, 48, 64, 96), seed: int = 4):
    """List of cells: dict(n, phase, fraction_target, Fbar)."""
    root = np.random.SeedSequence(seed)
    out = []
    for k, ss in enumerate(root.spawn(count)):
        rng = np.random.default_rng(ss)
        n = int(rng.choice(np.asarray(sizes)))
        frac = rng.uniform(0.1, 0.4)
        ph = sphere_inclusions(n, rng, frac)
        H = rng.uniform(-0.05, 0.05, size=(3, 3))
        out.append({"n": n, "phase": ph, "fraction_target": frac, "Fbar": np.eye(3) + H})
    return out


def rve_batch_materials():
    return [neohooke(20.0, 200.0), neohooke(1.0, 10.0)]


# ----------------------------------------------------------------------------
# lce_polydomain: periodic Voronoi grains with random directors
# ----------------------------------------------------------------------------

def voronoi_grains(n: int = 256, n_grains: int = 1000, seed: int = 5):
    """Grain index per voxel (nearest seed by minimum-image distance from the
    voxel centre) and one random unit director per grain (normalised
    N(0, I_3)). Returns (grain (n,n,n) int32, directors (n_grains, 3))."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    seeds = rng.uniform(0.0, n, size=(n_grains, 3))  # columns: x1, x2, x3
    dirs = rng.standard_normal((n_grains, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    tree = cKDTree(seeds, boxsize=float(n))
    kc = np.arange(n) + 0.5
    grain = np.empty((n, n, n), np.int32)
    x2, x1 = np.meshgrid(kc, kc, indexing="ij")
    for k3 in range(n):
        pts = np.stack([x1.ravel(), x2.ravel(), np.full(n * n, kc[k3])], axis=1)
        _, idx = tree.query(pts)
        grain[k3] = idx.reshape(n, n)
    return grain, dirs


def director_field(grain: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """(3, n3, n2, n1) float64 director field n0 from grains."""
    return np.ascontiguousarray(np.moveaxis(dirs[grain], -1, 0))


def uniaxial_lce(s: float) -> np.ndarray:
    return np.diag([s, s ** -0.5, s ** -0.5])


def lce_polydomain_case(n: int = 256, n_grains: int = 1000):
    grain, dirs = voronoi_grains(n, n_grains)
    return {
        "name": "lce_polydomain",
        "phase": np.zeros(grain.shape, np.uint8),
        "director0": director_field(grain, dirs),
        "materials": [lce(1.0, 2.0, 100.0)],
        "loads": [uniaxial_lce(1.0 + 0.01 * k) for k in range(1, 51)],
        "rho0": 10.0,
        "mu_ref": 1.0,
        "tol": 1e-6,
    }


# ----------------------------------------------------------------------------
# small random cases for parity tests
# ----------------------------------------------------------------------------

def random_two_phase(shape, fraction: float = 0.4, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.uniform(size=shape) >= fraction).astype(np.uint8)


def random_fbar(amp: float = 0.05, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.eye(3) + rng.uniform(-amp, amp, size=(3, 3))
