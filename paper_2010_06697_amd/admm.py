"""ctypes binding of the C ABI in ``include/admm.h`` (``libadmm.so``).

Argument marshalling only: every step of the ADMM iteration runs in the HIP
kernels of the library. PyTorch provides device memory and the stream. The
functions ``admm_*`` mirror the C entry points one to one; ``Solver`` owns the
device buffers of a batch of cells and wraps them.

Importing this module does not load the library; the first call does, and
raises ``RuntimeError`` if ``libadmm.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadmm.so")

OK, NOT_CONVERGED = 0, 1
EINVAL, EUNSUPPORTED, EHIP, ENOMEM, EDOMAIN, EDIVERGED, ENOGPU = -1, -2, -3, -4, -5, -6, -7
FP64, FP32_FP64RED = 0, 1
TILE_REG16 = -16  # tile width of the register-resident x2 / x3 passes
NEOHOOKE, LCE = 0, 1

# entry points declared in include/admm.h, in order
ENTRY_POINTS = (
    "admm_check_grid", "admm_workspace_bytes", "admm_init", "admm_set_load", "admm_set_free",
    "admm_get_fbar", "admm_bloch", "admm_bloch_static", "admm_bloch_static_max_bytes",
    "admm_orientation", "admm_set_rho",
    "admm_step", "admm_solve", "admm_local_step", "admm_project_step", "admm_update_step",
    "admm_homogenized_stress", "admm_history", "admm_cell_info", "admm_profile_enable",
    "admm_profile_read", "admm_autotune", "admm_set_tuning", "admm_divergence_check",
    "admm_get_state",
    "admm_set_state", "admm_strerror", "admm_destroy",
)

KERNELS = ("local", "div_fwdx", "fft_y_fwd", "poisson_z", "fft_y_inv", "inv_x", "update",
           "finalize", "mean_stress")


class Tuning(ctypes.Structure):
    _fields_ = [("tile_y", ctypes.c_int32), ("tile_z", ctypes.c_int32),
                ("n_len", ctypes.c_int32), ("x_points", ctypes.c_int32),
                ("len", ctypes.c_int32 * 24), ("radix", (ctypes.c_int32 * 8) * 24),
                ("ms_default", ctypes.c_double), ("ms_tuned", ctypes.c_double)]


class Material(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("mu", ctypes.c_double), ("lam", ctypes.c_double),
                ("a", ctypes.c_double), ("kappa", ctypes.c_double),
                ("alpha", ctypes.c_double), ("frank", ctypes.c_double),
                ("nu_F", ctypes.c_double), ("nu_n", ctypes.c_double)]


class Rve(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32),
                ("phase", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("u_prev", ctypes.c_void_p), ("F", ctypes.c_void_p),
                ("Lambda", ctypes.c_void_p), ("director", ctypes.c_void_p),
                ("director0", ctypes.c_void_p), ("Fbar", ctypes.c_double * 9)]


class Params(ctypes.Structure):
    _fields_ = [("rho0", ctypes.c_double), ("rho_min", ctypes.c_double),
                ("rho_max", ctypes.c_double), ("kappa_rho", ctypes.c_double),
                ("tau", ctypes.c_double), ("tol_p", ctypes.c_double),
                ("tol_d", ctypes.c_double), ("mu_ref", ctypes.c_double),
                ("newton_gtol", ctypes.c_double), ("newton_step_tol", ctypes.c_double),
                ("adapt_rho", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("newton_max", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("local_ratio", ctypes.c_double), ("local_chunk", ctypes.c_int32),
                ("local_passes", ctypes.c_int32), ("local_fraction", ctypes.c_double),
                ("dt", ctypes.c_double), ("div_growth", ctypes.c_double),
                ("stall_iters", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded library; raises if it is not built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
        i32 = ctypes.c_int32
        L.admm_check_grid.argtypes = [i32, i32, i32]
        L.admm_workspace_bytes.argtypes = [ctypes.POINTER(Rve), i32, i32]
        L.admm_workspace_bytes.restype = ctypes.c_size_t
        L.admm_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Rve), i32,
                                ctypes.POINTER(Material), i32, ctypes.POINTER(Params), i32,
                                vp, ctypes.c_size_t, vp]
        L.admm_set_load.argtypes = [vp, i32, dp]
        L.admm_set_free.argtypes = [vp, i32, ctypes.c_uint32]
        L.admm_get_fbar.argtypes = [vp, i32, dp]
        L.admm_orientation.argtypes = [vp, i32, dp]
        L.admm_bloch.argtypes = [vp, i32, dp, ctypes.c_double, ctypes.c_double, i32, vp, dp, dp,
                                 ip, ip]
        L.admm_bloch_static.argtypes = L.admm_bloch.argtypes
        L.admm_bloch_static_max_bytes.argtypes = []
        L.admm_bloch_static_max_bytes.restype = ctypes.c_size_t
        L.admm_set_rho.argtypes = [vp, i32, ctypes.c_double]
        L.admm_step.argtypes = [vp, i32, dp, dp, dp]
        L.admm_solve.argtypes = [vp, ip, ip]
        L.admm_local_step.argtypes = [vp]
        L.admm_project_step.argtypes = [vp]
        L.admm_update_step.argtypes = [vp]
        L.admm_homogenized_stress.argtypes = [vp, i32, dp, dp]
        L.admm_history.argtypes = [vp, i32, i32, dp, dp, dp, ip]
        L.admm_cell_info.argtypes = [vp, i32, ip, ip, ip, ctypes.POINTER(ctypes.c_int64)]
        L.admm_profile_enable.argtypes = [vp, i32]
        L.admm_profile_read.argtypes = [vp, i32, dp, ip]
        L.admm_autotune.argtypes = [vp, i32, ctypes.POINTER(Tuning)]
        L.admm_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.admm_divergence_check.argtypes = [ctypes.POINTER(Params), dp, dp, i32, ip]
        L.admm_get_state.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t)]
        L.admm_set_state.argtypes = [vp, vp, ctypes.c_size_t]
        L.admm_strerror.argtypes = [ctypes.c_int]
        L.admm_strerror.restype = ctypes.c_char_p
        L.admm_destroy.argtypes = [vp]
        L.admm_destroy.restype = None
        _lib = L
    return _lib


class AdmmError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {admm_strerror(code)} ({code})")
        self.code = code


def _check(code, where, allow=(OK,)):
    if code not in allow:
        raise AdmmError(code, where)
    return code


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


# ---- one-to-one wrappers of the C entry points -----------------------------

def admm_strerror(code: int) -> str:
    return lib().admm_strerror(int(code)).decode()


def admm_check_grid(n1: int, n2: int, n3: int) -> int:
    return lib().admm_check_grid(n1, n2, n3)


def admm_workspace_bytes(rves, precision: int) -> int:
    arr = (Rve * len(rves))(*rves)
    return lib().admm_workspace_bytes(arr, len(rves), precision)


def admm_init(rves, mats, params: Params, precision: int, workspace_ptr=None,
              workspace_bytes=0, stream_ptr=None):
    ctx = ctypes.c_void_p()
    ra = (Rve * len(rves))(*rves)
    ma = (Material * len(mats))(*mats)
    rc = lib().admm_init(ctypes.byref(ctx), ra, len(rves), ma, len(mats), ctypes.byref(params),
                         precision, workspace_ptr, workspace_bytes, stream_ptr)
    _check(rc, "admm_init")
    return ctx


def admm_set_load(ctx, rve: int, Fbar) -> int:
    F = np.ascontiguousarray(np.asarray(Fbar, np.float64).reshape(9))
    return _check(lib().admm_set_load(ctx, rve, _dptr(F)), "admm_set_load")


def free_mask(free) -> int:
    """Bit mask of free components of <F> from indices k = 3i + j."""
    return sum(1 << int(k) for k in set(free))


def admm_set_free(ctx, rve: int, free) -> int:
    """free: indices k = 3i + j of the components of <F> left free."""
    return _check(lib().admm_set_free(ctx, rve, free_mask(free)), "admm_set_free")


def admm_get_fbar(ctx, rve: int) -> np.ndarray:
    F = np.zeros(9)
    _check(lib().admm_get_fbar(ctx, rve, _dptr(F)), "admm_get_fbar")
    return F


def admm_bloch(ctx, rve: int, omega, rho: float, tol: float, max_iter: int, p_ptr: int):
    """Stability modulus over Bloch waves; p_ptr: device buffer of 3V complex
    doubles (start in, mode out). Returns (beta, sigma_rho, iters, status)."""
    w = np.ascontiguousarray(np.asarray(omega, np.float64).reshape(3))
    b, s = np.zeros(1), np.zeros(1)
    it, st = np.zeros(1, np.int32), np.zeros(1, np.int32)
    _check(lib().admm_bloch(ctx, rve, _dptr(w), float(rho), float(tol), int(max_iter), p_ptr,
                            _dptr(b), _dptr(s), _iptr(it), _iptr(st)), "admm_bloch")
    return float(b[0]), float(s[0]), int(it[0]), int(st[0])


def admm_bloch_static(ctx, rve: int, omega, rho: float, tol: float, max_iter: int, p_ptr: int):
    """admm_bloch with its work buffers in the library's fixed device array
    (no device allocation). Same returns as admm_bloch."""
    w = np.ascontiguousarray(np.asarray(omega, np.float64).reshape(3))
    b, s = np.zeros(1), np.zeros(1)
    it, st = np.zeros(1, np.int32), np.zeros(1, np.int32)
    _check(lib().admm_bloch_static(ctx, rve, _dptr(w), float(rho), float(tol), int(max_iter),
                                   p_ptr, _dptr(b), _dptr(s), _iptr(it), _iptr(st)),
           "admm_bloch_static")
    return float(b[0]), float(s[0]), int(it[0]), int(st[0])


def admm_bloch_static_max_bytes() -> int:
    """Size of the fixed work array of admm_bloch_static (bytes)."""
    return int(lib().admm_bloch_static_max_bytes())


def admm_orientation(ctx, rve: int) -> np.ndarray:
    """S = 3/2 (<n (x) n> - I/3) over the LCE voxels of a cell (3x3)."""
    S = np.zeros(9)
    _check(lib().admm_orientation(ctx, rve, _dptr(S)), "admm_orientation")
    return S.reshape(3, 3)


def admm_set_rho(ctx, rve: int, rho: float) -> int:
    return _check(lib().admm_set_rho(ctx, rve, float(rho)), "admm_set_rho")


def admm_step(ctx, n_iter: int, n_rve: int):
    rp, rd, rho = np.zeros(n_rve), np.zeros(n_rve), np.zeros(n_rve)
    rc = lib().admm_step(ctx, n_iter, _dptr(rp), _dptr(rd), _dptr(rho))
    _check(rc, "admm_step", allow=(OK, EDOMAIN))
    return rc, rp, rd, rho


def admm_solve(ctx, n_rve: int):
    it = np.zeros(n_rve, np.int32)
    st = np.zeros(n_rve, np.int32)
    rc = lib().admm_solve(ctx, _iptr(it), _iptr(st))
    _check(rc, "admm_solve", allow=(OK, NOT_CONVERGED, EDOMAIN, EDIVERGED))
    return rc, it, st


def admm_local_step(ctx) -> int:
    return _check(lib().admm_local_step(ctx), "admm_local_step", allow=(OK, EDOMAIN))


def admm_project_step(ctx) -> int:
    return _check(lib().admm_project_step(ctx), "admm_project_step")


def admm_update_step(ctx) -> int:
    return _check(lib().admm_update_step(ctx), "admm_update_step", allow=(OK, EDOMAIN))


def admm_homogenized_stress(ctx, rve: int):
    P, L = np.zeros(9), np.zeros(9)
    rc = lib().admm_homogenized_stress(ctx, rve, _dptr(P), _dptr(L))
    _check(rc, "admm_homogenized_stress", allow=(OK, EDOMAIN))
    return P, L


def admm_history(ctx, rve: int, max_n: int):
    rp, rd, rho = np.zeros(max(max_n, 1)), np.zeros(max(max_n, 1)), np.zeros(max(max_n, 1))
    n = ctypes.c_int32(0)
    _check(lib().admm_history(ctx, rve, max_n, _dptr(rp), _dptr(rd), _dptr(rho),
                              ctypes.byref(n)), "admm_history")
    k = n.value
    return rp[:k], rd[:k], rho[:k]


def admm_cell_info(ctx, rve: int):
    """(iterations, status, Newton-cap hits, Newton iterations summed over voxels)"""
    it, st, nf = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    ni = ctypes.c_int64(0)
    _check(lib().admm_cell_info(ctx, rve, ctypes.byref(it), ctypes.byref(st), ctypes.byref(nf),
                                ctypes.byref(ni)), "admm_cell_info")
    return it.value, st.value, nf.value, ni.value


def admm_profile_enable(ctx, on: bool) -> int:
    return _check(lib().admm_profile_enable(ctx, int(bool(on))), "admm_profile_enable")


def admm_profile_read(ctx):
    """{kernel name: (total ms, launches)} since profiling was enabled."""
    out = {}
    for k, name in enumerate(KERNELS):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int32(0)
        _check(lib().admm_profile_read(ctx, k, ctypes.byref(ms), ctypes.byref(n)),
               "admm_profile_read")
        out[name] = (ms.value, n.value)
    return out


def admm_autotune(ctx, reps):
    """Tunes (reps > 0) or reports (reps = 0) the Step 2 launch configuration:
    {"tile_y", "tile_z", "plans": {length: [radices]}, "ms_default", "ms_tuned"}."""
    t = Tuning()
    _check(lib().admm_autotune(ctx, reps, ctypes.byref(t)), "admm_autotune")
    plans = {}
    for k in range(t.n_len):
        plans[t.len[k]] = [r for r in t.radix[k] if r]
    return {"x_points": t.x_points, "tile_y": t.tile_y, "tile_z": t.tile_z, "plans": plans,
            "ms_default": t.ms_default, "ms_tuned": t.ms_tuned}


def admm_set_tuning(ctx, tile_y: int, tile_z: int, x_points: int, plans=None) -> int:
    """Applies a Step 2 launch configuration; plans: {length: [radices]}."""
    t = Tuning()
    t.tile_y, t.tile_z, t.x_points = int(tile_y), int(tile_z), int(x_points)
    plans = plans or {}
    t.n_len = len(plans)
    for k, (n, rad) in enumerate(sorted(plans.items())):
        t.len[k] = int(n)
        for j, r in enumerate(rad):
            t.radix[k][j] = int(r)
    return _check(lib().admm_set_tuning(ctx, ctypes.byref(t)), "admm_set_tuning")


def admm_divergence_check(params: Params, r_p, r_d) -> int:
    """Index of the iteration at which admm_solve's divergence watch stops a
    cell with this residual history, or -1 (host only)."""
    rp = np.ascontiguousarray(np.asarray(r_p, np.float64))
    rd = np.ascontiguousarray(np.asarray(r_d, np.float64))
    at = np.zeros(1, np.int32)
    _check(lib().admm_divergence_check(ctypes.byref(params), _dptr(rp), _dptr(rd), len(rp),
                                       _iptr(at)), "admm_divergence_check")
    return int(at[0])


def admm_get_state(ctx) -> bytes:
    """The context's whole iteration state as a host byte string."""
    n = ctypes.c_size_t(0)
    _check(lib().admm_get_state(ctx, None, ctypes.byref(n)), "admm_get_state")
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().admm_get_state(ctx, buf, ctypes.byref(n)), "admm_get_state")
    return buf.raw


def admm_set_state(ctx, blob: bytes) -> int:
    return _check(lib().admm_set_state(ctx, blob, len(blob)), "admm_set_state")


def admm_destroy(ctx) -> None:
    lib().admm_destroy(ctx)


# ---- convenience: device buffers of a batch of cells -----------------------

def default_params(precision: str = "fp64", **kw) -> Params:
    p = Params()
    p.rho0, p.rho_min, p.rho_max, p.kappa_rho, p.tau = 10.0, 1.0, 50.0, 1.3, 10.0
    p.tol_p, p.tol_d, p.mu_ref = 1e-8, 1e-8, 1.0
    if precision == "fp64":
        p.newton_gtol, p.newton_step_tol = 1e-14, 1e-10
    else:
        p.newton_gtol, p.newton_step_tol = 1e-10, 2e-6
    p.adapt_rho, p.max_iter, p.check_every, p.newton_max = 0, 200, 10, 100
    p.use_graph = 1
    p.local_ratio, p.local_chunk, p.local_passes, p.local_fraction = 0.0, 1, 8, 0.0
    p.dt = 1.0
    p.div_growth, p.stall_iters = 1e3, 500
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def material(model="neohooke", mu=1.0, lam=0.0, a=1.0, kappa=0.0, alpha=0.0, frank=0.0,
             nu_F=0.0, nu_n=0.0) -> Material:
    m = Material()
    m.model = NEOHOOKE if model == "neohooke" else LCE
    m.mu, m.lam, m.a, m.kappa = float(mu), float(lam), float(a), float(kappa)
    m.alpha, m.frank, m.nu_F, m.nu_n = float(alpha), float(frank), float(nu_F), float(nu_n)
    return m


class Solver:
    """A batch of periodic cells on one GPU, each with its own grid, phase map
    and macroscopic gradient, sharing one material table and parameters.

    Buffers are torch tensors on ``device``: per cell ``u``/``u_prev``
    (3, n3, n2, n1, double in both precisions), ``F`` (9, n3, n2, n1) holding F - I, ``Lambda`` (9, ...),
    ``phase`` (n3, n2, n1) uint8. They start from the zero state (u = 0,
    F = I, Lambda = 0) unless overwritten with ``set_state``.
    """

    def __init__(self, phases, materials, Fbars, params: Params | None = None,
                 precision: str = "fp64", device: str = "cuda:0", stream=None,
                 directors=None, directors0=None):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.precision = FP64 if precision == "fp64" else FP32_FP64RED
        self.dtype = torch.float64 if self.precision == FP64 else torch.float32
        self.params = params if params is not None else default_params()
        mats = [m if isinstance(m, Material) else material(**m) for m in materials]
        self.cells = []
        rves = []
        any_lce = any(m.model == LCE for m in mats)
        if directors is None:
            directors = [None] * len(phases)
        if directors0 is None:
            directors0 = [None] * len(phases)
        for ph, Fb, n0, nref in zip(phases, Fbars, directors, directors0):
            ph = np.ascontiguousarray(ph, np.uint8)
            n3, n2, n1 = ph.shape
            if admm_check_grid(n1, n2, n3) != OK:
                raise AdmmError(admm_check_grid(n1, n2, n3), f"grid {ph.shape}")
            cell = {
                "shape": (n3, n2, n1),
                "phase": torch.from_numpy(ph).to(self.device),
                # the displacement fluctuation is double in both precisions
                "u": torch.zeros((3, n3, n2, n1), dtype=torch.float64, device=self.device),
                "u_prev": torch.zeros((3, n3, n2, n1), dtype=torch.float64, device=self.device),
                "F": torch.zeros((9, n3, n2, n1), dtype=self.dtype, device=self.device),
                "Lambda": torch.zeros((9, n3, n2, n1), dtype=self.dtype, device=self.device),
                "director": None,
                "director0": None,
            }
            if any_lce:
                if n0 is None:
                    raise AdmmError(EINVAL, "an LCE phase needs a director field per cell")
                n0 = np.ascontiguousarray(n0, np.float64).reshape(3, n3, n2, n1)
                cell["director"] = torch.from_numpy(n0).to(self.device, self.dtype)
            if nref is not None:
                nref = np.ascontiguousarray(nref, np.float64).reshape(3, n3, n2, n1)
                cell["director0"] = torch.from_numpy(nref).to(self.device, self.dtype)
            self.cells.append(cell)
            r = Rve()
            r.n[0], r.n[1], r.n[2] = n1, n2, n3
            r.phase = cell["phase"].data_ptr()
            r.u = cell["u"].data_ptr()
            r.u_prev = cell["u_prev"].data_ptr()
            r.F = cell["F"].data_ptr()
            r.Lambda = cell["Lambda"].data_ptr()
            r.director = cell["director"].data_ptr() if cell["director"] is not None else None
            r.director0 = cell["director0"].data_ptr() if cell["director0"] is not None else None
            for k, v in enumerate(np.asarray(Fb, np.float64).reshape(9)):
                r.Fbar[k] = v
            rves.append(r)
        self.n = len(rves)
        nbytes = admm_workspace_bytes(rves, self.precision)
        if nbytes == 0:
            raise AdmmError(EINVAL, "admm_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        torch.cuda.synchronize(self.device)
        self.ctx = admm_init(rves, mats, self.params, self.precision,
                             self.workspace.data_ptr() + off, nbytes, self.stream.cuda_stream)

    # -- iteration --
    def set_load(self, rve, Fbar):
        admm_set_load(self.ctx, rve, Fbar)

    def set_free(self, rve, free):
        admm_set_free(self.ctx, rve, free)

    def fbar(self, rve=0):
        return admm_get_fbar(self.ctx, rve)

    def orientation(self, rve=0):
        return admm_orientation(self.ctx, rve)

    def bloch(self, rve, omega, rho, p0, tol=1e-10, max_iter=5000):
        """Stability modulus over Bloch waves of the cell's current state
        (double precision). p0: complex (3, n3, n2, n1) start. Returns
        dict(beta, sigma_rho, iters, status, p)."""
        t = self.torch
        p = t.from_numpy(np.ascontiguousarray(p0, np.complex128)).to(self.device)
        self.torch.cuda.synchronize(self.device)
        b, s, it, st = admm_bloch(self.ctx, rve, omega, rho, tol, max_iter, p.data_ptr())
        return {"beta": b, "sigma_rho": s, "iters": it, "status": st, "p": p.cpu().numpy()}

    def bloch_static(self, rve, omega, rho, p0, tol=1e-10, max_iter=5000):
        """bloch() through the allocation-free entry point."""
        t = self.torch
        p = t.from_numpy(np.ascontiguousarray(p0, np.complex128)).to(self.device)
        self.torch.cuda.synchronize(self.device)
        b, s, it, st = admm_bloch_static(self.ctx, rve, omega, rho, tol, max_iter, p.data_ptr())
        return {"beta": b, "sigma_rho": s, "iters": it, "status": st, "p": p.cpu().numpy()}

    def set_rho(self, rho, rve=-1):
        admm_set_rho(self.ctx, rve, rho)

    def step(self, n_iter):
        return admm_step(self.ctx, n_iter, self.n)

    def solve(self):
        return admm_solve(self.ctx, self.n)

    def local_step(self):
        return admm_local_step(self.ctx)

    def project_step(self):
        return admm_project_step(self.ctx)

    def update_step(self):
        return admm_update_step(self.ctx)

    def homogenized_stress(self, rve=0):
        return admm_homogenized_stress(self.ctx, rve)

    def history(self, rve=0, max_n=100000):
        return admm_history(self.ctx, rve, max_n)

    def info(self, rve=0):
        return admm_cell_info(self.ctx, rve)

    def profile(self, on=True):
        admm_profile_enable(self.ctx, on)

    def profile_read(self):
        return admm_profile_read(self.ctx)

    def set_tuning(self, tile_y, tile_z, x_points, plans=None):
        admm_set_tuning(self.ctx, tile_y, tile_z, x_points, plans)

    def checkpoint(self) -> bytes:
        """admm_get_state: everything needed to resume bit for bit."""
        return admm_get_state(self.ctx)

    def restore(self, blob: bytes):
        """admm_set_state on a context built like the one checkpointed."""
        admm_set_state(self.ctx, blob)

    def autotune(self, reps=5):
        return admm_autotune(self.ctx, reps)

    # -- state as float64 numpy (F as F itself) --
    def state(self, rve=0):
        c = self.cells[rve]
        self.torch.cuda.synchronize(self.device)
        F = c["F"].double().cpu().numpy().copy()
        F[0] += 1.0
        F[4] += 1.0
        F[8] += 1.0
        out = {"u": c["u"].double().cpu().numpy(), "u_prev": c["u_prev"].double().cpu().numpy(),
               "F": F, "Lambda": c["Lambda"].double().cpu().numpy()}
        if c["director"] is not None:
            out["director"] = c["director"].double().cpu().numpy()
        return out

    def set_state(self, rve=0, u=None, F=None, Lambda=None, director=None):
        """Overwrites the fields of one cell (F given as F itself)."""
        c = self.cells[rve]
        t = self.torch
        if u is not None:
            c["u"].copy_(t.from_numpy(np.ascontiguousarray(u, np.float64)).to(self.device))
        if F is not None:
            E = np.array(F, np.float64, copy=True)
            E[0] -= 1.0
            E[4] -= 1.0
            E[8] -= 1.0
            c["F"].copy_(t.from_numpy(E).to(self.device, self.dtype))
        if Lambda is not None:
            c["Lambda"].copy_(t.from_numpy(np.ascontiguousarray(Lambda, np.float64))
                              .to(self.device, self.dtype))
        if director is not None:
            c["director"].copy_(t.from_numpy(np.ascontiguousarray(director, np.float64))
                                .to(self.device, self.dtype))
        t.cuda.synchronize(self.device)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            admm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
