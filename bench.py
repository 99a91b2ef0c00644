"""Throughput of the ADMM hot path on one MI355X.

Workload (N = 1): the 256^3 periodic fibre composite (fibres along x3, radius 8,
area fraction 0.3, gap >= 2, fibre mu=50 lambda=500, matrix mu=1 lambda=10),
first increment of the simple-shear path (Fbar = I + 0.01 e1 x e2), rho0 = 10
adapted in [1, 50], float fields with double reductions. A step is one ADMM
iteration (Steps 1-4 and the penalty rule) over the whole cell; the timed
region is `--steps` iterations plus one homogenised-stress evaluation, with
every field resident in HBM before it starts.

Also reported on the same line: the all-double form at 256^3, the 128-cell
batch (edges 32..96, one load step each to tol 1e-6) as cell solves/s, the
256^3 LCE polydomain (ideal, and with the full model's non-ideality,
Frank and dissipation terms), the 64^3 wavy laminate's 30-step compression path in
double and in float, the inexact local step against exact local solves (on
the fibre cell and the LCE polydomain), the per-kernel times from hipEvents on the library's
stream, the roofline of the dominant kernel, and the CPU oracle timed on the
host on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-ADMM-iterations/s at 256³, FP32+FP64-reduce vs FP64; RVE solves/s"
HBM_PEAK_GBS = 8000.0
# the 128-cell batch: penalty start and range
BATCH_RHO0, BATCH_RHO_MIN, BATCH_RHO_MAX = 30.0, 30.0, 100.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes_per_voxel(s, c):
    """Algorithmic HBM bytes per voxel of each kernel (every operand read or
    written once; s = scalar bytes of F, Lambda and the spectra, c =
    (n1/2+1)/n1 half-spectrum fraction, a complex half-spectrum component
    costs 2 c s per voxel). u is double in both forms; the float form solves
    Step 2 for the correction du (float), formed into u by the update. The
    float form without LCE phases (the fibre cell) also has the update store
    the next local step's data A - I (9 float) and the det F - 1 of its warm
    start (1 float), which that step reads at an unchanged penalty (every
    iteration of a call but its first) in place of u, Lambda and F; and the
    local step store F - A (9 float), from which Step 2 forms its defect in
    place of F, Lambda and u."""
    f32 = s == 4
    return {
        # float: A - I 9, det F - 1 of the warm start 1, phase in; F 9, F - A 9 out.
        # double: u 3, F 9, Lambda 9, phase in; F 9 out
        "local": 28 * s + 1 if f32 else 3 * 8 + 27 * s + 1,
        # float: F - A 9 in; double: F 9, Lambda 9 in; 3 half spectra out
        "div_fwdx": (9 * s if f32 else 18 * s) + 6 * c * s,
        "fft_y_fwd": 12 * c * s,         # 3 components in and out
        "poisson_z": 12 * c * s,
        "fft_y_inv": 12 * c * s,
        "inv_x": 6 * c * s + 3 * s if f32 else 6 * c * s + 3 * 8,  # spectra in; du or u out
        # u_i 3 (double) and du 3 in, u_{i+1} 3 out (float form) or u_{i+1}, u_i in;
        # F 9, Lambda 9 in; Lambda 9 out (float form: and A - I 9, det F - 1 1 out)
        "update": (3 * 8 + 3 * s + 3 * 8 + 10 * s if f32 else 6 * 8) + 27 * s,
        "finalize": 0.0,
        "mean_stress": 18 * s + 1,
    }


def iteration_bytes_alg(s, c, forward_components=9, u_bytes=None):
    """Minimum bytes per voxel-iteration of the method: the state once in and
    out (u_{i+1}, u_i, F, Lambda in; F, Lambda, u out: 45 scalars) plus one HBM
    round trip of the forward and of the inverse spectrum. With 9 forward
    components and u in s-byte scalars this is the plain method's count,
    s (45 + 48 c) + 1 (277.75 B in float at 256^3); this design forms the
    right-hand side of Step 2 as a divergence in real space (3 forward
    components) and keeps u in double (u_bytes = 8)."""
    ub = s if u_bytes is None else u_bytes
    return 9 * ub + 36 * s + 4 * c * (forward_components + 3) * s + 1


def run_single(case, precision, steps, warmup, profile=True):
    import torch
    from paper_2010_06697_amd import admm

    n3, n2, n1 = case["phase"].shape
    V = n1 * n2 * n3
    p = admm.default_params(precision, rho0=case["rho0"], rho_min=case["rho_min"],
                            rho_max=case["rho_max"], adapt_rho=1, mu_ref=case["mu_ref"],
                            tol_p=case["tol_fp32" if precision == "fp32" else "tol_fp64"],
                            tol_d=case["tol_fp32" if precision == "fp32" else "tol_fp64"])
    s = admm.Solver([case["phase"]], case["materials"], [case["loads"][0]], p,
                    precision=precision)
    log(f"[bench] {precision}: warmup {warmup} iterations")
    if warmup:
        s.step(warmup)
    tuning = s.autotune(reps=3)
    log(f"[bench] {precision}: autotuned Step 2 {tuning['ms_default']:.3f} -> "
        f"{tuning['ms_tuned']:.3f} ms (tiles {tuning['tile_y']}/{tuning['tile_z']})")
    # the tuner drops the captured graphs: capture them again outside the timing
    s.step(p.check_every)
    torch.cuda.synchronize()
    log(f"[bench] {precision}: timing {steps} iterations")
    t0 = time.perf_counter()
    rc, rp, rd, rho = s.step(steps)
    P, _ = s.homogenized_stress(0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel times: a further run with hipEvents around every launch
    # (kept out of the timed region above, which replays captured graphs)
    prof_steps = min(steps, 10) if profile else 0
    prof = {}
    newton_before = s.info(0)[3]
    if profile:
        s.profile(True)
        s.step(prof_steps)
        s.homogenized_stress(0)
        prof = s.profile_read()
        s.profile(False)
    it, status, nfail, newton_its = s.info(0)
    # Newton iterations per voxel over the profiled iterations, whose kernel
    # times the roofline uses
    newton_per_voxel_it = ((newton_its - newton_before) / float(V * prof_steps) if prof_steps
                           else newton_its / float(V * (warmup + p.check_every + steps)))
    s.close()
    del s
    torch.cuda.empty_cache()
    dt = t1 - t0
    out = {
        "value": V * steps / dt,
        "ms_per_step": 1e3 * dt / steps,
        "r_p": float(rp[0]), "r_d": float(rd[0]), "rho": float(rho[0]),
        "newton_fail": int(nfail),
        "newton_iters_per_voxel_iteration": newton_per_voxel_it,
        "P_mean": [float(x) for x in P],
        "kernels_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()},
        "kernels_launches": {k: v[1] for k, v in prof.items()},
        "autotune": tuning,
    }
    log(f"[bench] {precision}: {out['value']:.3e} voxel-it/s, {out['ms_per_step']:.3f} ms/it")
    return out


def run_batch(count, steps_warm=2):
    import torch
    from paper_2010_06697_amd import admm, microstructure as M

    log(f"[bench] batch: generating {count} cells")
    cells = M.rve_batch(count)
    mats = M.rve_batch_materials()
    p = admm.default_params("fp32", rho0=BATCH_RHO0, rho_min=BATCH_RHO_MIN,
                            rho_max=BATCH_RHO_MAX, adapt_rho=1, mu_ref=5.0, tol_p=1e-6,
                            tol_d=1e-6, max_iter=2000, check_every=20)
    s = admm.Solver([c["phase"] for c in cells], mats, [c["Fbar"] for c in cells], p,
                    precision="fp32")
    s.step(steps_warm)  # loads the kernels; the state is reset below
    tuning = s.autotune(reps=3)
    for k, c in enumerate(s.cells):
        for f in ("u", "u_prev", "F", "Lambda"):
            c[f].zero_()
    torch.cuda.synchronize()
    for k, c in enumerate(cells):
        s.set_load(k, c["Fbar"])
    s.set_rho(BATCH_RHO0)
    torch.cuda.synchronize()
    log("[bench] batch: timing one load step of every cell")
    t0 = time.perf_counter()
    rc, iters, status = s.solve()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.close()
    del s
    torch.cuda.empty_cache()
    vox = np.array([c["n"] ** 3 for c in cells], dtype=np.float64)
    dt = t1 - t0
    out = {
        "cells": count,
        "rve_solves_per_s": float(np.sum(status == admm.OK)) / dt,
        "seconds": dt,
        "converged": int(np.sum(status == admm.OK)),
        "voxels": int(vox.sum()),
        "iterations_mean": float(iters.mean()),
        "iterations_max": int(iters.max()),
        "voxel_iterations_per_s": float(np.sum(vox * iters)) / dt,
        "autotune": tuning,
    }
    log(f"[bench] batch: {out['rve_solves_per_s']:.2f} cell solves/s, "
        f"{out['voxel_iterations_per_s']:.3e} voxel-it/s")
    return out


# the full LCE model's terms for the lce256_full line (Sec. 5.1; Frank
# constant in units of mu x voxel^2)
LCE_FULL = dict(alpha=0.1, frank=0.05, nu_F=0.1, nu_n=0.1)


# iterations of the polydomain's relaxation at zero mean strain before the
# first load increment (untimed)
LCE_RELAX = 40


def lce_relaxed(case, mats, p, full):
    """Solver on the LCE polydomain, relaxed from F = I, n = n0 at zero mean
    strain for LCE_RELAX iterations (the polydomain preparation of Sec. 5.3;
    the grains' directors make the field heterogeneous), then loaded with the
    first increment of the uniaxial path."""
    from paper_2010_06697_amd import admm

    s = admm.Solver([case["phase"]], mats, [np.eye(3)], p, precision="fp32",
                    directors=[case["director0"]],
                    directors0=[case["director0"]] if full else None)
    s.step(LCE_RELAX)
    s.set_load(0, case["loads"][0])
    return s


def run_lce(steps, warmup, full=False):
    """The LCE polydomain at 256^3 (1000 Voronoi grains, neo-classical a = 2,
    kappa = 100), float with double reductions, rho0 = 10 adaptive in
    [1, 50]: relaxed at zero mean strain, then the first load increment of
    the uniaxial path, timed; full: with the non-ideality, Frank and
    dissipation terms of LCE_FULL (dt = 1)."""
    import torch
    from paper_2010_06697_amd import admm, microstructure as M

    log("[bench] lce: generating the 256^3 polydomain")
    case = M.lce_polydomain_case()
    V = case["phase"].size
    p = admm.default_params("fp32", rho0=case["rho0"], rho_min=1.0, rho_max=50.0, adapt_rho=1,
                            mu_ref=case["mu_ref"])
    mats = [M.lce(1.0, 2.0, 100.0, **LCE_FULL)] if full else case["materials"]
    log(f"[bench] lce: relaxing {LCE_RELAX} iterations at zero mean strain")
    s = lce_relaxed(case, mats, p, full)
    s.step(warmup)
    s.autotune(reps=3)
    torch.cuda.synchronize()
    s.profile(True)
    log(f"[bench] lce: timing {steps} iterations")
    t0 = time.perf_counter()
    rc, rp, rd, rho = s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = s.profile_read()
    it, status, nfail, newton_its = s.info(0)
    s.close()
    del s
    torch.cuda.empty_cache()
    out = {"workload": "lce256: 256^3 LCE polydomain, 1000 grains, a=2 mu=1 kappa=100, "
                       f"relaxed {LCE_RELAX} iterations at Fbar = I from F = I, n = n0, then "
                       "Fbar = diag(1.01, 1.01^-1/2, 1.01^-1/2), float with double reductions"
                       + (f", full model {LCE_FULL}" if full else ""),
           "value": V * steps / dt, "unit": "voxel-iterations/s", "ms_per_step": 1e3 * dt / steps,
           "newton_iters_per_voxel_iteration": newton_its / float(V * (warmup + steps)),
           "newton_fail": int(nfail), "r_p": float(rp[0]), "r_d": float(rd[0]),
           "kernels_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}}
    log(f"[bench] lce: {out['value']:.3e} voxel-it/s, {out['ms_per_step']:.3f} ms/it")
    return out


INEXACT = dict(local_ratio=0.3, local_chunk=1, local_passes=4)


def run_inexact(fibres, lce_steps=10, lce_warmup=3):
    """The inexact local step (r_l <= 0.3 r_d, one Newton iteration per voxel
    and pass, at most 4 passes) against exact local solves: on the 256^3
    fibre cell the time to solve the second shear increment to tol 1e-6 in
    float (after solving the first, which also captures the graphs), and on
    the 256^3 LCE polydomain (relaxed, then the first increment, as in
    run_lce) the time per iteration over fixed iterations (that cell does
    not converge within a bench-sized budget) with the residuals both
    reach."""
    import torch
    from paper_2010_06697_amd import admm, microstructure as M

    out = {"options": dict(INEXACT)}
    V = fibres["phase"].size
    res = {}
    for name, loc in (("exact", {}), ("inexact", INEXACT)):
        p = admm.default_params("fp32", rho0=fibres["rho0"], rho_min=fibres["rho_min"],
                                rho_max=fibres["rho_max"], adapt_rho=1, mu_ref=fibres["mu_ref"],
                                tol_p=fibres["tol_fp32"], tol_d=fibres["tol_fp32"], max_iter=3000,
                                **loc)
        s = admm.Solver([fibres["phase"]], fibres["materials"], [fibres["loads"][0]], p,
                        precision="fp32")
        s.solve()
        s.set_load(0, fibres["loads"][1])
        torch.cuda.synchronize()
        log(f"[bench] inexact: fibres256 fp32 {name}, second increment")
        t0 = time.perf_counter()
        rc, it, st = s.solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        P = s.homogenized_stress(0)[0]
        n_its = s.info(0)[3]
        s.close()
        del s
        torch.cuda.empty_cache()
        res[name] = {"seconds": dt, "iterations": int(it[0]), "converged": int(st[0]) == admm.OK,
                     "newton_iters_per_voxel_iteration": n_its / float(V * max(1, int(it[0]))),
                     "P": P}
    dP = float(np.abs(res["inexact"]["P"] - res["exact"]["P"]).max() /
               np.abs(res["exact"]["P"]).max())
    for r in res.values():
        r.pop("P")
    out["fibres256_fp32_increment2"] = dict(res, speedup=res["exact"]["seconds"] /
                                            res["inexact"]["seconds"], P_rel_diff=dP)
    log(f"[bench] inexact: fibres speedup {out['fibres256_fp32_increment2']['speedup']:.3f}")

    case = M.lce_polydomain_case()
    V = case["phase"].size
    res = {}
    for name, loc in (("exact", {}), ("inexact", INEXACT)):
        p = admm.default_params("fp32", rho0=case["rho0"], rho_min=1.0, rho_max=50.0, adapt_rho=1,
                                mu_ref=case["mu_ref"], **loc)
        s = lce_relaxed(case, case["materials"], p, False)
        s.step(lce_warmup)
        s.step(p.check_every)  # captures the graphs outside the timing
        torch.cuda.synchronize()
        before = s.info(0)[3]
        log(f"[bench] inexact: lce256 fp32 {name}, {lce_steps} iterations")
        t0 = time.perf_counter()
        rc, rp, rd, rho = s.step(lce_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n_its = s.info(0)[3] - before
        s.close()
        del s
        torch.cuda.empty_cache()
        res[name] = {"ms_per_step": 1e3 * dt / lce_steps, "value": V * lce_steps / dt,
                     "r_p": float(rp[0]), "r_d": float(rd[0]),
                     "newton_iters_per_voxel_iteration": n_its / float(V * lce_steps)}
    out["lce256_fp32"] = dict(res, speedup=res["exact"]["ms_per_step"] /
                              res["inexact"]["ms_per_step"])
    log(f"[bench] inexact: lce speedup {out['lce256_fp32']['speedup']:.3f}")
    return out


def run_wavy():
    """The 64^3 wavy laminate under uniaxial compression to 0.85 in 30 load
    steps, each solved to 1e-7, in double and in float with double
    reductions: time per load path and the homogenised stress of both."""
    import torch
    from paper_2010_06697_amd import admm, microstructure as M

    case = M.wavy_laminate64_case()
    out = {"workload": "wavy64: 64^3 wavy laminate (stiff 4 / period 16, mu contrast 100, "
                       "lambda = 10 mu), Fbar = diag(1, 1, s), s = 1 -> 0.85 in 30 steps, "
                       "each to tol 1e-7, rho0 = 10 adaptive in [1, 100]"}
    P = {}
    for prec in ("fp64", "fp32"):
        p = admm.default_params(prec, rho0=case["rho0"], rho_min=1.0, rho_max=100.0,
                                adapt_rho=1, mu_ref=case["mu_ref"], tol_p=case["tol"],
                                tol_d=case["tol"], max_iter=3000, check_every=10)
        s = admm.Solver([case["phase"]], case["materials"], [case["loads"][0]], p,
                        precision=prec)
        torch.cuda.synchronize()
        log(f"[bench] wavy64 {prec}: 30 load steps")
        t0 = time.perf_counter()
        iters, conv = [], 0
        for k, Fb in enumerate(case["loads"]):
            if k:
                s.set_load(0, Fb)
            rc, it, st = s.solve()
            iters.append(int(it[0]))
            conv += int(st[0] == admm.OK)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        P[prec] = s.homogenized_stress(0)[0]
        s.close()
        del s
        torch.cuda.empty_cache()
        out[prec] = {"seconds": dt, "load_steps_converged": conv,
                     "iterations_total": int(np.sum(iters)), "iterations_max": int(np.max(iters)),
                     "P33_final": float(P[prec][8])}
        log(f"[bench] wavy64 {prec}: {dt:.2f} s, {np.sum(iters)} iterations, {conv}/30 converged")
    out["P_rel_diff_fp32_vs_fp64"] = float(np.abs(P["fp32"] - P["fp64"]).max() /
                                           np.abs(P["fp64"]).max())
    return out


def run_c3(case):
    """The fibre cell's whole load path and the precision of the float form.
    (1) The 10 simple-shear increments Fbar = I + 0.01 k e1 e2, each solved
    to 1e-6 in float (warm-started, rho adaptive in [1, 50]): time, iterations
    and voxel-iterations/s of the whole path. (2) The first increment solved
    to 1e-8 in double and to 1e-7 in float: the relative difference of <P>,
    and each against the oracle's converged 256 x 256 x 2 cross-section
    (tests/golden/oracle_fibres256x2.json; the 256^3 solution does not depend
    on x3)."""
    import torch
    from paper_2010_06697_amd import admm

    V = case["phase"].size
    out = {}
    p = admm.default_params("fp32", rho0=case["rho0"], rho_min=case["rho_min"],
                            rho_max=case["rho_max"], adapt_rho=1, mu_ref=case["mu_ref"],
                            tol_p=case["tol_fp32"], tol_d=case["tol_fp32"], max_iter=3000)
    s = admm.Solver([case["phase"]], case["materials"], [case["loads"][0]], p, precision="fp32")
    s.autotune(reps=3)
    s.step(p.check_every)  # loads and captures; the state is reset below
    for f in ("u", "u_prev", "F", "Lambda"):
        s.cells[0][f].zero_()
    s.set_rho(case["rho0"])
    s.set_load(0, case["loads"][0])
    torch.cuda.synchronize()
    log("[bench] c3: 10 increments to 1e-6 in float")
    iters, conv = [], 0
    t0 = time.perf_counter()
    for k, Fb in enumerate(case["loads"]):
        if k:
            s.set_load(0, Fb)
        rc, it, st = s.solve()
        iters.append(int(it[0]))
        conv += int(st[0] == admm.OK)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.close()
    del s
    torch.cuda.empty_cache()
    out["load_path_fp32"] = {"increments": len(iters), "converged": conv,
                             "iterations": iters, "seconds": dt,
                             "voxel_iterations_per_s": V * float(np.sum(iters)) / dt,
                             "tol": case["tol_fp32"]}
    log(f"[bench] c3: {dt:.2f} s, {np.sum(iters)} iterations, {conv}/10 converged")
    P = {}
    for prec, tol in (("fp64", 1e-8), ("fp32", 1e-7)):
        p = admm.default_params(prec, rho0=case["rho0"], rho_min=case["rho_min"],
                                rho_max=case["rho_max"], adapt_rho=1, mu_ref=case["mu_ref"],
                                tol_p=tol, tol_d=tol, max_iter=2000)
        s = admm.Solver([case["phase"]], case["materials"], [case["loads"][0]], p,
                        precision=prec)
        rc, it, st = s.solve()
        P[prec] = s.homogenized_stress(0)[0]
        out[f"increment1_{prec}"] = {"tol": tol, "iterations": int(it[0]),
                                     "converged": int(st[0]) == admm.OK,
                                     "P_mean": [float(x) for x in P[prec]]}
        s.close()
        del s
        torch.cuda.empty_cache()
    scale = np.abs(P["fp64"]).max()
    out["P_rel_diff_fp32_vs_fp64"] = float(np.abs(P["fp32"] - P["fp64"]).max() / scale)
    gpath = os.path.join(ROOT, "tests", "golden", "oracle_fibres256x2.json")
    if os.path.exists(gpath):
        g = np.asarray(json.load(open(gpath))["runs"]["converged"]["P_mean"])
        out["P_rel_diff_vs_oracle"] = {k: float(np.abs(v - g).max() / np.abs(g).max())
                                       for k, v in P.items()}
    log(f"[bench] c3: <P> fp32 vs fp64 {out['P_rel_diff_fp32_vs_fp64']:.2e}")
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case):
    """The oracle (plain C, FP64, direct DFT) on the host: one ADMM iteration
    of the same 256^3 cell from the same start with all threads (the
    reported value), and, as bounded samples, two iterations of the cell's
    256 x 256 x 2 cross-section with all threads and with one thread (the
    oracle's thread scaling; its direct DFT costs less per voxel there, so
    that rate is not the 256^3 one)."""
    import oracle as O

    n3, n2, n1 = case["phase"].shape
    mats = [O.material(m["model"], mu=m["mu"], lam=m["lam"]) for m in case["materials"]]
    nthreads = O.num_threads()

    def timed(phase, iters):
        u, F, L = O.initial_state(phase.shape)
        p = O.params(max_iter=iters, fixed_iters=True, mu_ref=case["mu_ref"])
        t0 = time.perf_counter()
        O.admm_run(phase, mats, case["loads"][0].ravel(), p, u, F, L, case["rho0"])
        return time.perf_counter() - t0

    log(f"[bench] cpu baseline: oracle, 1 iteration at {n1}x{n2}x{n3}, {nthreads} threads")
    dt = timed(case["phase"], 1)
    log(f"[bench] cpu baseline: {dt:.1f} s")
    slab = np.ascontiguousarray(case["phase"][:2])
    vs = slab.size
    dt_all = timed(slab, 2)
    O.set_num_threads(1)
    try:
        dt_one = timed(slab, 2)
    finally:
        O.set_num_threads(nthreads)
    log(f"[bench] cpu baseline: cross-section {dt_all:.2f} s ({nthreads} threads), "
        f"{dt_one:.2f} s (1 thread)")
    return {"value": n1 * n2 * n3 / dt, "unit": "voxel-iterations/s", "cores": nthreads,
            "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"one ADMM iteration of the {n1}x{n2}x{n3} fibre cell from the zero "
                      f"state (FP64, direct DFT), {dt:.1f} s",
            "cross_section_256x256x2": {
                "iterations": 2,
                "threads_all": {"threads": nthreads, "seconds": dt_all,
                                "voxel_iterations_per_s": 2 * vs / dt_all},
                "threads_1": {"threads": 1, "seconds": dt_one,
                              "voxel_iterations_per_s": 2 * vs / dt_one}}}


def traffic_for(kernel, workload):
    """HBM traffic per launch from the committed rocprofv3 counter summary, or
    None when absent or when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != sources_sha():
        return None
    return rec.get("bytes_per_launch")


def sources_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2010_06697_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lce", action="store_true")
    ap.add_argument("--no-wavy", action="store_true")
    ap.add_argument("--no-inexact", action="store_true")
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB copied by a plain device copy before the timed region "
                         "(reference kernel for the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the library runs "
              "each cell on a single GPU.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_06697_amd import admm, microstructure as M

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    admm.lib()

    if args.calibrate_copy:
        nb = args.calibrate_copy << 20
        a = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    log("[bench] generating the 256^3 fibre cell")
    case = M.fibres256_case()
    n3, n2, n1 = case["phase"].shape
    V = n1 * n2 * n3
    c = (n1 // 2 + 1) / n1

    f32 = run_single(case, "fp32", args.steps, args.warmup)
    f64 = None if args.no_fp64 else run_single(case, "fp64", args.steps, args.warmup)
    batch = None if args.no_batch else run_batch(128)
    lce = None if args.no_lce else run_lce(10, 3)
    lce_full = None if args.no_lce else run_lce(10, 3, full=True)
    wavy = None if args.no_wavy else run_wavy()
    c3 = None if args.no_c3 else run_c3(case)
    inexact = None if args.no_inexact else run_inexact(case)

    # roofline of the dominant kernel (by total time in the timed region)
    kb = kernel_bytes_per_voxel(4, c)
    tot = {k: f32["kernels_ms"][k] * f32["kernels_launches"][k] for k in f32["kernels_ms"]}
    dom = max(tot, key=tot.get)
    avg_ms = f32["kernels_ms"][dom]
    bytes_launch = kb[dom] * V
    traffic = traffic_for(dom, "fibres256_fp32")
    # the dominant kernel against HBM (every kernel of the float iteration
    # moves its bytes at about a plain copy's rate)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "alg_bytes_per_launch": bytes_launch, "avg_ms": avg_ms}
    b_sv = iteration_bytes_alg(4, c, 9)
    b_it = iteration_bytes_alg(4, c, 3, u_bytes=8)
    it_roof = {"basis": "plain method: s (45 + 48 c) + 1 bytes per voxel-iteration",
               "bytes_per_voxel_iteration": b_sv,
               "achieved_GBs": b_sv * f32["value"] / 1e9,
               "frac": b_sv * f32["value"] / (HBM_PEAK_GBS * 1e9),
               "bytes_per_voxel_iteration_this_design": b_it,
               "frac_this_design": b_it * f32["value"] / (HBM_PEAK_GBS * 1e9)}
    if f64 is not None:
        b64 = iteration_bytes_alg(8, c, 9)
        it_roof["fp64_bytes_per_voxel_iteration"] = b64
        it_roof["fp64_frac"] = b64 * f64["value"] / (HBM_PEAK_GBS * 1e9)
    per_kernel = {k: {"avg_ms": f32["kernels_ms"][k],
                      "GBs": (kb[k] * V / (f32["kernels_ms"][k] * 1e-3) / 1e9
                              if f32["kernels_ms"][k] > 0 and kb[k] > 0 else None)}
                  for k in f32["kernels_ms"] if f32["kernels_launches"][k]}

    cpu = None if args.no_cpu_baseline else cpu_baseline(case)

    line = {
        "metric": METRIC,
        "value": f32["value"],
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fibres256: 256^3 periodic fibre composite (fibres along x3, "
                               "r=8, area fraction 0.3, gap>=2; fibre mu=50 lambda=500, matrix "
                               "mu=1 lambda=10), simple shear Fbar = I + 0.01 e1(x)e2, rho0=10 "
                               "adaptive in [1,50], float fields with double reductions",
                   "batch": f"128 cells, edges 32..96, spherical inclusions, one load step "
                            f"each to tol 1e-6, rho0={BATCH_RHO0:g} in [{BATCH_RHO_MIN:g}, "
                            f"{BATCH_RHO_MAX:g}]",
                   "grid": [n1, n2, n3], "voxels": V},
        "fp64": None if f64 is None else {"value": f64["value"], "ms_per_step": f64["ms_per_step"],
                                          "dtype": "f64",
                                          "kernels_ms": f64["kernels_ms"]},
        "fp32_over_fp64": None if f64 is None else f32["value"] / f64["value"],
        "autotune": f32["autotune"],
        "rve_batch": batch,
        "lce256": lce,
        "lce256_full": lce_full,
        "inexact_local_step": inexact,
        "wavy64": wavy,
        "fibres256_load_path": c3,
        "roofline": roof,
        "iteration_roofline": it_roof,
        "kernels": per_kernel,
        "residuals_after_timed_steps": {"r_p": f32["r_p"], "r_d": f32["r_d"], "rho": f32["rho"],
                                        "newton_fail": f32["newton_fail"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
