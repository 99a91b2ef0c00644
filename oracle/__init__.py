"""CPU oracle for the ADMM iteration of Zhou & Bhattacharya (arXiv 2010.06697).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The product path (the
HIP library and its binding) never does, and shares no code with it.

This module is argument marshalling over the plain C library ``liboracle.so``
(``admm_oracle.c``), all in float64. Array conventions: a vector field has shape
``(3, n3, n2, n1)``, a tensor field ``(9, n3, n2, n1)`` with component
``3*i + J`` = F_iJ, the phase map ``(n3, n2, n1)`` uint8. ``F`` is the
deformation gradient itself (not F - I).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, EINVAL, EDOMAIN = 0, 1, -1, -5
NEOHOOKE, LCE = 0, 1


class Material(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("mu", ctypes.c_double),
                ("lam", ctypes.c_double), ("a", ctypes.c_double),
                ("kappa", ctypes.c_double), ("alpha", ctypes.c_double),
                ("frank", ctypes.c_double), ("nu_F", ctypes.c_double),
                ("nu_n", ctypes.c_double)]


class Site(ctypes.Structure):
    """Per-voxel data of the full LCE model: cross-link director n0 and the
    constant quadratic form Sc in the director (see admm_oracle.h)."""
    _fields_ = [("n0", ctypes.c_double * 3), ("Sc", ctypes.c_double * 9)]


class Newton(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("gtol", ctypes.c_double),
                ("step_tol", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("rho_min", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("kappa_rho", ctypes.c_double), ("tau", ctypes.c_double),
                ("adapt_rho", ctypes.c_int), ("tol_p", ctypes.c_double),
                ("tol_d", ctypes.c_double), ("mu_ref", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("fixed_iters", ctypes.c_int),
                ("newton", Newton), ("local_ratio", ctypes.c_double),
                ("local_chunk", ctypes.c_int), ("local_passes", ctypes.c_int),
                ("local_start_iter", ctypes.c_int), ("local_rd_prev", ctypes.c_double),
                ("local_fraction", ctypes.c_double), ("free_mask", ctypes.c_uint),
                ("dt", ctypes.c_double)]


_lib = None


def lib():
    """Load (building first if absent) the oracle library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        bp = ctypes.POINTER(ctypes.c_ubyte)
        mp = ctypes.POINTER(Material)
        i = ctypes.c_int
        L.or_dft3.argtypes = [i, i, i, dp, dp, dp, dp, i]
        L.or_gradient.argtypes = [i, i, i, dp, dp, dp]
        L.or_project.argtypes = [i, i, i, dp, dp, dp]
        sp = ctypes.POINTER(Site)
        L.or_energy.argtypes = [mp, dp, dp, sp]
        L.or_energy.restype = ctypes.c_double
        L.or_stress.argtypes = [mp, dp, dp, sp, dp]
        L.or_tangent.argtypes = [mp, dp, dp, sp, dp]
        L.or_director.argtypes = [dp, dp, dp]
        L.or_relaxed.argtypes = [mp, dp, sp, dp, dp, dp, dp]
        L.or_prox.argtypes = [mp, ctypes.c_double, dp, sp, ctypes.POINTER(Newton), dp, dp, ip]
        L.or_rho_update.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.POINTER(Params)]
        L.or_rho_update.restype = ctypes.c_double
        L.or_admm_run.argtypes = [i, i, i, bp, mp, i, dp, ctypes.POINTER(Params),
                                  dp, dp, dp, dp, dp, dp, dp, dp, dp, ip, ip]
        L.or_mean_stress.argtypes = [i, i, i, bp, mp, i, dp, dp, dp, dp, dp, dp]
        L.or_orientation.argtypes = [i, i, i, bp, mp, i, dp, dp]
        L.or_bloch.argtypes = [i, i, i, bp, mp, i, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                               i, dp, dp, dp, dp, ip]
        L.or_num_threads.argtypes = []
        L.or_set_num_threads.argtypes = [i]
        L.or_set_num_threads.restype = None
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))
    return a


def site(nref=None, Sc=None):
    """A Site from the cross-link director nref and the form Sc (3x3);
    None for both gives no site (the ideal model)."""
    if nref is None and Sc is None:
        return None
    s = Site()
    nv = _vec(nref if nref is not None else (0.0, 0.0, 0.0), 3)
    Sv = _vec(Sc if Sc is not None else np.zeros(9), 9)
    for k in range(3):
        s.n0[k] = nv[k]
    for k in range(9):
        s.Sc[k] = Sv[k]
    return s


def _sp(s):
    return ctypes.byref(s) if s is not None else None


def material(model="neohooke", mu=1.0, lam=0.0, a=1.0, kappa=0.0, alpha=0.0, frank=0.0,
             nu_F=0.0, nu_n=0.0):
    m = Material()
    m.model = NEOHOOKE if model == "neohooke" else LCE
    m.mu, m.lam, m.a, m.kappa = float(mu), float(lam), float(a), float(kappa)
    m.alpha, m.frank, m.nu_F, m.nu_n = float(alpha), float(frank), float(nu_F), float(nu_n)
    return m


def newton_opts(max_iter=100, gtol=1e-15, step_tol=1e-10):
    o = Newton()
    o.max_iter, o.gtol, o.step_tol = max_iter, gtol, step_tol
    return o


def params(rho_min=1.0, rho_max=50.0, kappa_rho=1.3, tau=10.0, adapt_rho=False,
           tol_p=1e-8, tol_d=1e-8, mu_ref=1.0, max_iter=200, fixed_iters=False,
           newton=None, local_ratio=0.0, local_chunk=1, local_passes=8, local_start_iter=0,
           local_rd_prev=0.0, local_fraction=0.0, free=(), dt=1.0):
    """free: indices k = 3i + j of the components of <F> left free (mixed
    boundary conditions); the others are prescribed. dt: time step of the
    load step (dissipation)."""
    p = Params()
    p.local_ratio, p.local_chunk, p.local_passes = local_ratio, local_chunk, local_passes
    p.local_start_iter, p.local_rd_prev = local_start_iter, local_rd_prev
    p.local_fraction = local_fraction
    p.free_mask = sum(1 << int(k) for k in set(free))
    p.dt = float(dt)
    p.rho_min, p.rho_max, p.kappa_rho, p.tau = rho_min, rho_max, kappa_rho, tau
    p.adapt_rho = int(bool(adapt_rho))
    p.tol_p, p.tol_d, p.mu_ref = tol_p, tol_d, mu_ref
    p.max_iter, p.fixed_iters = int(max_iter), int(bool(fixed_iters))
    p.newton = newton if newton is not None else newton_opts()
    return p


def _mats(mats):
    arr = (Material * len(mats))()
    for k, m in enumerate(mats):
        arr[k] = m
    return arr


def num_threads():
    return lib().or_num_threads()


def set_num_threads(n):
    lib().or_set_num_threads(int(n))


def dft3(x, inverse=False):
    """3D DFT of an array of shape (n3, n2, n1) (complex or real)."""
    x = np.asarray(x)
    n3, n2, n1 = x.shape
    re = np.ascontiguousarray(x.real, dtype=np.float64)
    im = np.ascontiguousarray(x.imag if np.iscomplexobj(x) else np.zeros_like(re),
                              dtype=np.float64)
    ore, oim = np.empty_like(re), np.empty_like(re)
    rc = lib().or_dft3(n1, n2, n3, _dp(re), _dp(im), _dp(ore), _dp(oim), int(inverse))
    assert rc == OK, rc
    return ore + 1j * oim


def gradient(u, Fbar):
    u = np.ascontiguousarray(u, dtype=np.float64)
    _, n3, n2, n1 = u.shape
    G = np.empty((9, n3, n2, n1))
    rc = lib().or_gradient(n1, n2, n3, _dp(u), _dp(_vec(Fbar, 9)), _dp(G))
    assert rc == OK, rc
    return G


def project(H, return_imag=False):
    H = np.ascontiguousarray(H, dtype=np.float64)
    _, n3, n2, n1 = H.shape
    u = np.empty((3, n3, n2, n1))
    mi = ctypes.c_double(0.0)
    rc = lib().or_project(n1, n2, n3, _dp(H), _dp(u), ctypes.byref(mi))
    assert rc == OK, rc
    return (u, mi.value) if return_imag else u


def energy(m, F, n=(0.0, 0.0, 1.0), nref=None, Sc=None):
    return lib().or_energy(ctypes.byref(m), _dp(_vec(F, 9)), _dp(_vec(n, 3)),
                           _sp(site(nref, Sc)))


def stress(m, F, n=(0.0, 0.0, 1.0), nref=None, Sc=None):
    P = np.empty(9)
    rc = lib().or_stress(ctypes.byref(m), _dp(_vec(F, 9)), _dp(_vec(n, 3)),
                         _sp(site(nref, Sc)), _dp(P))
    if rc != OK:
        raise FloatingPointError("det F <= 0")
    return P


def tangent(m, F, n=(0.0, 0.0, 1.0), nref=None, Sc=None):
    C = np.empty(81)
    rc = lib().or_tangent(ctypes.byref(m), _dp(_vec(F, 9)), _dp(_vec(n, 3)),
                          _sp(site(nref, Sc)), _dp(C))
    if rc != OK:
        raise FloatingPointError("det F <= 0")
    return C.reshape(9, 9)


def director(F, n_prev):
    n = np.empty(3)
    lib().or_director(_dp(_vec(F, 9)), _dp(_vec(n_prev, 3)), _dp(n))
    return n


def relaxed(m, F, n_prev, nref=None, Sc=None):
    """LCE energy with the director eliminated: returns (n, P, K) at F."""
    n = np.empty(3)
    P = np.empty(9)
    K = np.empty(81)
    rc = lib().or_relaxed(ctypes.byref(m), _dp(_vec(F, 9)), _sp(site(nref, Sc)),
                          _dp(_vec(n_prev, 3)), _dp(n), _dp(P), _dp(K))
    if rc != OK:
        raise ValueError(f"or_relaxed failed: {rc}")
    return n, P, K.reshape(9, 9)


def prox(m, rho, A, F0, n0=(0.0, 0.0, 1.0), opts=None, nref=None, Sc=None):
    """Local problem at one point from the warm start (F0, n0). Returns
    (F, n, iters, rc)."""
    F = _vec(F0, 9).copy()
    n = _vec(n0, 3).copy()
    it = ctypes.c_int(0)
    o = opts if opts is not None else newton_opts()
    rc = lib().or_prox(ctypes.byref(m), float(rho), _dp(_vec(A, 9)), _sp(site(nref, Sc)),
                       ctypes.byref(o), _dp(F), _dp(n), ctypes.byref(it))
    return F, n, it.value, rc


def rho_update(rho, r_p, r_d, p):
    return lib().or_rho_update(float(rho), float(r_p), float(r_d), ctypes.byref(p))


def admm_run(phase, mats, Fbar, p, u, F, Lam, rho, director_field=None, director0=None):
    """Runs ADMM iterations in place on (u, F, Lam[, director_field]).

    Returns a dict with rc, iters, rho, the r_p / r_d / rho histories and
    Fbar (with its free components, if any, as the iteration left them).
    """
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    n3, n2, n1 = phase.shape
    for a, c in ((u, 3), (F, 9), (Lam, 9)):
        assert a.shape == (c, n3, n2, n1) and a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    if director_field is not None:
        assert director_field.shape == (3, n3, n2, n1) and director_field.flags["C_CONTIGUOUS"]
    nh = max(int(p.max_iter), 1)
    hp, hd, hr = np.zeros(nh), np.zeros(nh), np.zeros(nh)
    r = ctypes.c_double(float(rho))
    it = ctypes.c_int(0)
    nf = ctypes.c_int(0)
    marr = _mats(mats)
    Fb = np.array(np.asarray(Fbar, dtype=np.float64).reshape(9))
    rc = lib().or_admm_run(n1, n2, n3,
                           phase.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                           marr, len(mats), _dp(Fb), ctypes.byref(p),
                           _dp(u), _dp(F), _dp(Lam), _dp(director_field), _dp(director0),
                           ctypes.byref(r), _dp(hp), _dp(hd), _dp(hr),
                           ctypes.byref(it), ctypes.byref(nf))
    k = it.value
    return {"rc": rc, "iters": k, "rho": r.value, "r_p": hp[:k].copy(),
            "r_d": hd[:k].copy(), "rho_hist": hr[:k].copy(), "newton_fail": nf.value,
            "Fbar": Fb}


def mean_stress(phase, mats, F, director_field=None, Lam=None, director0=None):
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    n3, n2, n1 = phase.shape
    P = np.empty(9)
    L = np.empty(9)
    marr = _mats(mats)
    rc = lib().or_mean_stress(n1, n2, n3,
                              phase.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                              marr, len(mats), _dp(F), _dp(director_field), _dp(director0),
                              _dp(Lam), _dp(P), _dp(L))
    if rc != OK:
        raise FloatingPointError(f"or_mean_stress rc={rc}")
    return (P, L) if Lam is not None else P


def orientation(phase, mats, director_field):
    """S = 3/2 (<n (x) n> - I/3) over the LCE voxels (3x3)."""
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    n3, n2, n1 = phase.shape
    S = np.empty(9)
    rc = lib().or_orientation(n1, n2, n3, phase.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                              _mats(mats), len(mats), _dp(director_field), _dp(S))
    assert rc == OK, rc
    return S.reshape(3, 3)


def bloch(phase, mats, F, omega, rho, p0, tol=1e-12, max_iter=5000, director_field=None):
    """Stability modulus over Bloch waves p exp(i omega.x) (omega in radians
    per voxel) of the tangent field at F. p0: complex (3, n3, n2, n1) start.
    Returns dict(rc, beta, sigma_rho, iters, p)."""
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    n3, n2, n1 = phase.shape
    pr = np.ascontiguousarray(np.real(p0), dtype=np.float64).copy()
    pi = np.ascontiguousarray(np.imag(p0), dtype=np.float64).copy()
    b, sr = ctypes.c_double(0.0), ctypes.c_double(0.0)
    it = ctypes.c_int(0)
    rc = lib().or_bloch(n1, n2, n3, phase.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                        _mats(mats), len(mats), _dp(np.ascontiguousarray(F, dtype=np.float64)),
                        _dp(director_field), _dp(_vec(omega, 3)), float(rho), float(tol),
                        int(max_iter), _dp(pr), _dp(pi), ctypes.byref(b), ctypes.byref(sr),
                        ctypes.byref(it))
    return {"rc": rc, "beta": b.value, "sigma_rho": sr.value, "iters": it.value, "p": pr + 1j * pi}


def initial_state(shape, director0=None):
    """Zero fluctuation, F = I, Lambda = 0 (the start of the first load step)."""
    n3, n2, n1 = shape
    u = np.zeros((3, n3, n2, n1))
    F = np.zeros((9, n3, n2, n1))
    F[0] = F[4] = F[8] = 1.0
    Lam = np.zeros((9, n3, n2, n1))
    return u, F, Lam
