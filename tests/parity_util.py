"""Shared helpers of the GPU parity tests: seeded inputs and oracle runs.

Inputs come from paper_2010_06697_amd.microstructure (geometry only) and
numpy generators seeded here; expected values come only from the oracle.
"""
import numpy as np

import oracle as O
from paper_2010_06697_amd import admm


def omats(mats):
    return [O.material(m["model"], mu=m["mu"], lam=m["lam"], a=m["a"], kappa=m["kappa"],
                       **{k: m[k] for k in ("alpha", "frank", "nu_F", "nu_n") if k in m})
            for m in mats]


def random_state(shape, seed, amp_u=0.05, amp_E=0.02, amp_L=0.5):
    """A smooth-ish random state: u (3,...), F (9,...), Lambda (9,...)."""
    rng = np.random.default_rng(seed)
    n3, n2, n1 = shape
    k3, k2, k1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    u = np.zeros((3,) + shape)
    for i in range(3):
        for _ in range(4):
            m = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            u[i] += amp_u * rng.standard_normal() * np.sin(
                2 * np.pi * (m[0] * k1 / n1 + m[1] * k2 / n2 + m[2] * k3 / n3) + ph)
    F = amp_E * rng.standard_normal((9,) + shape)
    F[0] += 1.0
    F[4] += 1.0
    F[8] += 1.0
    L = amp_L * rng.standard_normal((9,) + shape)
    return u, F, L


def rel(a, b):
    d = np.max(np.abs(np.asarray(a) - np.asarray(b)))
    s = np.max(np.abs(np.asarray(b)))
    return d / s if s > 0 else d


# the local Newton stopping rule the GPU's double-precision form uses by default
NEWTON64 = dict(gtol=1e-14, step_tol=1e-10)


def prox_minimiser(mat, rho, A, Fw):
    """The oracle's local-step minimiser (Sec. 2.1, Step 1) to rounding: its
    Newton solve from the warm start Fw, continued from that point with a
    gradient test of 1e-16 (the default 1e-14 test, scaled by the moduli
    plus rho, accepts points up to about 1e-12 away along rotations, where
    the objective is only rho-stiff). Where rounding keeps the continued
    solve from meeting that test it still ends at its last accepted iterate,
    which its line search keeps no worse than its start. Returns (F, rc) with
    the status of the first solve."""
    F, _, _, rc = O.prox(mat, rho, A, Fw, opts=O.newton_opts(**NEWTON64))
    if rc != O.OK:
        return F, rc
    Fp, _, _, rc2 = O.prox(mat, rho, A, F, opts=O.newton_opts(gtol=1e-16, step_tol=1e-12))
    return (Fp if rc2 in (O.OK, O.NOT_CONVERGED) else F), rc


def oracle_iterations(phase, mats, Fbar, n_iter, rho, mu_ref, adapt=False, state=None,
                      rho_min=1.0, rho_max=50.0, **local):
    """n_iter fixed iterations of the oracle from `state` (default: the
    initial state); `local` takes the inexact local step's local_* options."""
    u, F, L = state if state is not None else O.initial_state(phase.shape)
    u, F, L = u.copy(), F.copy(), L.copy()
    p = O.params(max_iter=n_iter, fixed_iters=True, mu_ref=mu_ref, adapt_rho=adapt,
                 rho_min=rho_min, rho_max=rho_max, newton=O.newton_opts(**NEWTON64), **local)
    r = O.admm_run(phase, omats(mats), np.asarray(Fbar).ravel(), p, u, F, L, rho)
    return u, F, L, r


def gpu_solver(phases, mats, Fbars, precision="fp64", **params):
    p = admm.default_params(precision, **params)
    return admm.Solver(phases, mats, Fbars, p, precision=precision)
