"""Benchmark: DOF-solves/s of the nested polarized-traces solver on one MI355X.

Workload (default): the n = 2047 layered medium (12 seeded layers on a linear
depth gradient, two dipping interfaces, c in [1.5, 4.5], 3-node smoothing),
48-node PML, omega for 10 points per wavelength at c_min, 32 layers x 8
cells, 64 point sources equally spaced on depth row 0.08 -- the mixed-
precision configuration and the largest one, a synthetic stand-in for the
paper's BP2004 runs (same contrast range, sampling and source geometry).

One "step" is one call of hz_solve on the whole batch of 64 right-hand sides
(RHS formation, Krylov solve of the polarized SIE with the Gauss-Seidel
sweeps, volume reconstruction; for the refinement form also the FP64 volume
residuals and corrections), inputs resident in HBM.  Forms timed on the
same sources:
  fp64_single         plain FP64, one source per solve (matrix-vector kernels)
  fp64_batched        plain FP64, the whole batch in one solve
  mixed_batched       complex64 Gauss-Seidel preconditioner inside flexible
                      FP64 GMRES; SIE matrix, volume solves in complex128
  refine_batched      the whole nested solver in complex64 (factors, local
                      solves, sweeps) inside FP64 iterative refinement on the
                      volume residual
  nested_pt_batched   nested polarized traces (inner GMRES + inner sweeps
                      instead of the inner block LU), FP64
`value` is the fastest batched form whose solutions agree with FP64 GPU
reference solves of three sources to a relative L2 error <= 1e-8 and, where
the stored oracle references exist (tests/golden), with the oracle's direct
solve on the stored rows to <= 1e-8.

Step times are taken with the solver's profiler off (plans replayed as HIP
graphs).  A separate profiled pass (HIP events on the solver's stream around
every launch, graphs bypassed) gives the per-kernel times of the roofline
records.  The CPU baseline times the oracle on the host.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-solves/sec at rel. err 1e-8: chosen form vs plain FP64, one MI355X"
PEAK = {"c128": 78.6e12, "c64": 157.3e12}          # dense FP64 / FP32 MFMA peak
HBM_PEAK = 8.0e12
ERR_BAR = 1e-8
# Krylov tolerance of every timed solve: one decade below the metric's error
# target, so that the measured errors (against FP64 reference solves at
# 1e-12 and the oracle's direct solve) meet ERR_BAR with margin.  For the
# refinement form it bounds the estimated error of the refined solution.
SOLVE_TOL = 1e-9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


_ROCTX = None


def roctx_region(on):
    """Resume / pause an external profiler started with --selected-regions
    (ROCTx profiler control), so that it records exactly one timed region."""
    global _ROCTX
    if _ROCTX is None:
        _ROCTX = ctypes.CDLL("librocprofiler-sdk-roctx.so")
    (_ROCTX.roctxProfilerResume if on else _ROCTX.roctxProfilerPause)(ctypes.c_uint64(0))


def timed_solves(solver, f, tol, steps, warmup, max_iter, prof_steps=1, region=False):
    """Warm-up, `steps` timed solves with the profiler off (graphs replayed),
    then `prof_steps` solves with the per-launch event profiler on."""
    import torch

    for _ in range(warmup):
        solver.solve(f, tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    if region:
        roctx_region(True)
    t0 = time.perf_counter()
    marks = []
    for _ in range(steps):
        u = solver.solve(f, tol=tol, max_iter=max_iter)   # returns after its own device sync
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # wall time of each timed step (no extra synchronisation: a solve ends with one)
    timed_solves.last_steps_ms = [1e3 * (b - a) for a, b in zip([t0] + marks[:-1], marks)]
    if region:
        roctx_region(False)
    stats = solver.last_stats
    prof, dt_prof = None, None
    if prof_steps > 0:
        solver.profile(True)
        t0 = time.perf_counter()
        for _ in range(prof_steps):
            solver.solve(f, tol=tol, max_iter=max_iter)
        torch.cuda.synchronize()
        dt_prof = (time.perf_counter() - t0) / prof_steps
        prof = solver.profile_read()
        solver.profile(False)
    return u, dt, prof, dt_prof, stats


KERNEL_SOURCES = {"gemm": ["k_gemm.hip", "hz_mfma.h", "hz_common.h"],
                  "cell_solve": ["k_cellsolve.hip", "hz_mfma.h", "hz_common.h"],
                  "plr": ["k_plr.hip", "hz_common.h"]}


def kernel_src_hash(family):
    """Hash of the sources of one kernel family (traffic figures recorded in
    profiles/ are used only while the kernel is unchanged)."""
    import hashlib

    group = ("plr" if family.startswith("plr") else
             "gemm" if family.startswith(("gemm", "gemv")) else "cell_solve")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[group]:
        with open(os.path.join(ROOT, "paper_1510_01831_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(family, workload, alg_bytes=None):
    """HBM bytes per launch measured with the FETCH_SIZE / WRITE_SIZE
    counters for this kernel on this workload and launch shape (a summary's
    alg_bytes, when present, must equal the record's algorithmic bytes per
    launch), from the summaries in profiles/; None when no summary covers
    the kernel as it is now."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    want = kernel_src_hash(family)
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as fh:
            for line in fh:
                if not line.startswith("traffic: "):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                if (kv.get("kernel") == family and kv.get("src") == want
                        and kv.get("workload", workload) == workload
                        and (alg_bytes is None or "alg_bytes" not in kv
                             or abs(float(kv["alg_bytes"]) - alg_bytes) <= 5e-3 * alg_bytes)):
                    return float(kv["bytes_per_launch"])
    return None


def roofline(k, B, workload):
    """Roofline record of one kernel family from the solver's event profile:
    matrix-core kernels against the dense MFMA peak of their precision,
    single-column kernels (matrix-vector products) against HBM bandwidth."""
    prec = "c64" if k["name"].endswith("_c64") else "c128"
    avg_ms = k["ms"] / k["launches"]
    rec = {"kernel": k["name"], "launches": k["launches"], "avg_launch_ms": avg_ms,
           "flops_per_launch": k["flops"] / k["launches"],
           "bytes_per_launch": k["bytes"] / k["launches"],
           "traffic": recorded_traffic(k["name"], workload, k["bytes"] / k["launches"])}
    if B > 1:
        achieved = k["flops"] / (k["ms"] * 1e-3)
        rec.update({"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[prec] / 1e12,
                    "unit": "TFLOP/s", "frac": achieved / PEAK[prec],
                    # flops counted as 8 per complex multiply-add; the matrix-core
                    # kernels use Gauss's three-product form (6 real flops each)
                    "flop_count": "8 per complex multiply-add",
                    "executed_frac": 0.75 * achieved / PEAK[prec]})
    else:
        achieved = k["bytes"] / (k["ms"] * 1e-3)
        rec.update({"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK})
    return rec


def copy_calibration(nbytes):
    """One plain device-to-device copy of nbytes (reference dispatch for the
    HBM traffic counters: FETCH_SIZE / WRITE_SIZE of a known-size copy)."""
    import torch

    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes}), flush=True)


def host_description():
    """nproc, CPU model, RAM and the BLAS thread count of this host."""
    import numpy as np  # noqa: F401  (loads the BLAS library)

    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    ram = int(line.split()[1]) * 1024
                    break
    except OSError:
        pass
    blas = None
    try:
        import threadpoolctl

        info = [x for x in threadpoolctl.threadpool_info() if x.get("user_api") == "blas"]
        blas = max(x["num_threads"] for x in info) if info else None
    except Exception:
        pass
    return {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": model, "ram_bytes": ram, "blas_threads": blas,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(w, c, gmres_iters):
    """The oracle timed on the host on a bounded sample of the workload.

    The oracle's polarized-traces solver with direct layer solves (a sparse
    LU of each layer grid; every Green's-integral application, RHS formation
    and reconstruction step is one layer solve) is timed on one interior
    layer: its factorisation (offline, x L layers) and single-RHS layer
    solves (online).  Per right-hand side the oracle's Alg. 6 performs
    2L volume layer solves (RHS formation and reconstruction), 2(L-1) layer
    applications per SIE product and 3(L-1)-2 per Gauss-Seidel
    preconditioner, with `gmres_iters` products and gmres_iters + 1
    preconditioner applications (left preconditioning), so the online time
    per RHS is that count times the measured layer-solve time."""
    import numpy as np

    from oracle.discretization import LayerGrid, Problem, partition
    from oracle.polarized import DirectLayerSolver
    from paper_1510_01831_amd import media

    host = host_description()
    prob = Problem(c, w.omega, w.n_pml)
    parts = partition(w.n, w.layers)
    li = w.layers // 2
    grid = LayerGrid(prob, parts[li][0], parts[li][1], li, w.layers)
    t0 = time.perf_counter()
    solver = DirectLayerSolver(grid)
    t_fac = time.perf_counter() - t0
    f = media.point_sources(w.n, (w.src_x[len(w.src_x) // 2],), w.src_z)[0]
    rng = np.random.default_rng(0)
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        g = np.zeros((grid.HL, prob.W), dtype=complex)
        g[grid.HL // 2] = rng.standard_normal(prob.W) * f.max()
        solver.solve(g)
    t_sol = (time.perf_counter() - t0) / reps
    K = w.layers - 1
    per_rhs = 2 * w.layers + gmres_iters * 2 * K + (gmres_iters + 1) * (3 * K - 2)
    t_online = per_rhs * t_sol
    return {
        "value": w.n * w.n / t_online,
        "unit": "DOF-solves/s",
        "cores": host["blas_threads"] or host["affinity_cpus"],
        "kind": "oracle",
        "sample": (f"oracle polarized traces with direct (SuperLU) layer solves, timed on "
                   f"layer {li} of {w.layers} ({grid.HL} x {prob.W} grid): factorisation "
                   f"{t_fac:.2f} s (offline, x{w.layers} layers = {t_fac * w.layers:.0f} s), "
                   f"single-RHS layer solve {t_sol * 1e3:.0f} ms; online per RHS = "
                   f"{per_rhs} layer solves at {gmres_iters} GMRES iterations "
                   f"= {t_online:.0f} s; value = n^2 / that time"),
        "offline_s_estimate": t_fac * w.layers,
        "online_s_per_rhs_estimate": t_online,
        "host": host,
    }


def local_refactor(solver, c, w, f_all, ref_idx, max_iter):
    """Re-factorisation after a local model update (the inversion-loop use of
    the method): velocity +2 % in a disk of radius 0.04 at the centre of the
    domain.  Times the local path against a full re-factorisation of the same
    model and compares the two solutions."""
    import numpy as np
    import torch
    n = w.n
    z, x = np.meshgrid(np.arange(1, n + 1) / (n + 1), np.arange(1, n + 1) / (n + 1), indexing="ij")
    c2 = c * (1.0 + 0.02 * (((z - 0.5) ** 2 + (x - 0.5) ** 2) <= 0.04 ** 2))
    m2 = torch.from_numpy(c2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    redone = solver.update_model_local(m2)
    torch.cuda.synchronize()
    t_loc = time.perf_counter() - t0
    ua = solver.solve(f_all, tol=1e-10, max_iter=max_iter)
    its = max(x["iters"] for x in solver.last_stats)
    t0 = time.perf_counter()
    solver.update_model(m2)
    solver.factor()
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    ub = solver.solve(f_all, tol=1e-10, max_iter=max_iter)
    diff = max(float(torch.linalg.norm(ua[k] - ub[k]) / torch.linalg.norm(ub[k])) for k in ref_idx)
    ncells = w.layers * w.cells
    log(f"[bench] local update: {redone}/{ncells} cells refactored in {t_loc:.3f} s "
        f"(full {t_full:.3f} s), rel. diff {diff:.1e}, {its} iterations")
    return {"update": "velocity +2% in a disk of radius 0.04 at the centre",
            "cells_refactored": redone, "cells": ncells, "local_refactor_s": t_loc,
            "full_refactor_s": t_full, "gmres_iters": its, "max_rel_diff_vs_full": diff}


MEDIUM = {"C1": "Gaussian bump c = 1 + 0.3 exp(-r^2/0.02)",
          "C2": "Gaussian random field c in [1.5,3] (corr. 0.05, seed 0)",
          "C3": "Gaussian random field c in [1.5,3] (corr. 0.05, seed 0)",
          "C4": "layered medium (12 seeded layers, c in [1.5,4.5], depth gradient, two dipping "
                "interfaces)",
          "C5": "lens c = 2 + 0.4 exp(-r^2/(2 0.08^2))"}

GOLDEN = {"C4": os.path.join(ROOT, "tests", "golden", "n2047_oracle_rows.npz")}


def load_golden(name):
    """Stored oracle references (the direct solve u = H^{-1} f on selected
    rows of selected sources), written by tests/golden/make_n2047_reference.py."""
    import numpy as np

    path = GOLDEN.get(name)
    if not path or not os.path.exists(path):
        return None
    z = np.load(path)
    return {"sources": [int(x) for x in z["sources"]], "rows": z["rows"], "u": z["u"]}


def golden_errors(u, golden):
    """Relative L2 error of u on the stored rows of each stored source."""
    import numpy as np

    if golden is None:
        return None
    rows = golden["rows"] - 1
    out = {}
    for i, k in enumerate(golden["sources"]):
        got = u[k][rows].cpu().numpy()
        ref = golden["u"][i]
        out[k] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return out


def run_workload(name, forms_wanted, steps, warmup, roctx_form="", want_local=False):
    """Time the forms of one workload; returns (forms, results, extras)."""
    import numpy as np
    import torch

    from paper_1510_01831_amd import hz, media

    w = media.workload(name)
    c = media.velocity(name)
    n = w.n
    B = w.n_rhs
    f_all = torch.from_numpy(media.point_sources(n, w.src_x, w.src_z)).cuda()
    max_iter = 60
    golden = load_golden(name)
    log(f"[bench] workload {w.name}: n={n} pml={w.n_pml} L={w.layers} Lc={w.cells} B={B}")
    forms, results, extras = {}, {}, {"memory": {}}

    # ---- plain FP64 (one context, used for single-RHS and batched solves)
    t0 = time.perf_counter()
    s64 = hz.Solver(torch.from_numpy(c), w.omega, w.n_pml, w.layers, w.cells,
                    precision=hz.HZ_FP64, max_batch=B)
    torch.cuda.synchronize()
    t_fac64 = time.perf_counter() - t0
    log(f"[bench] fp64 setup+factor {t_fac64:.2f} s")
    extras["memory"]["fp64_device_bytes"] = s64.info.device_bytes
    ref_idx = sorted({0, B // 2, B - 1})
    refs = {}
    for k in ref_idx:
        refs[k] = s64.solve(f_all[k:k + 1].contiguous(), tol=1e-12, max_iter=max_iter)[0]
    if "single" in forms_wanted:
        f1 = f_all[B // 2: B // 2 + 1].contiguous()
        u1, dt1, prof1, dtp1, st1 = timed_solves(s64, f1, SOLVE_TOL, steps, warmup, max_iter,
                                                 region=roctx_form == "fp64_single")
        it1 = st1[0]["iters"]
        log(f"[bench] fp64 single RHS: {dt1 * 1e3:.1f} ms/solve ({dtp1 * 1e3:.1f} profiled), "
            f"{it1} GMRES iterations")
        forms["fp64_single"] = {"dof_solves_per_s": n * n / dt1, "ms_per_solve": dt1 * 1e3,
                                "steps_ms": timed_solves.last_steps_ms,
                                "ms_per_solve_profiled": dtp1 * 1e3, "gmres_iters": it1,
                                "vol_resid": st1[0]["vol_resid"], "setup_factor_s": t_fac64,
                                "kernels": prof1,
                                "roofline": roofline(max(prof1, key=lambda k: k["ms"]), 1, name)}

    if "plr" in forms_wanted:
        # single-RHS FP64 solves whose preconditioner applies the interface
        # operators in partitioned low-rank form (eps = 1e-8, compressed in
        # hz_factor); the SIE matrix stays dense
        t0 = time.perf_counter()
        spl = hz.Solver(torch.from_numpy(c), w.omega, w.n_pml, w.layers, w.cells,
                        precision=hz.HZ_FP64, max_batch=1, plr=1, plr_eps=1e-8)
        torch.cuda.synchronize()
        t_facp = time.perf_counter() - t0
        info = spl.info
        k = B // 2
        f1 = f_all[k:k + 1].contiguous()
        up, dtp, profp, dtpp, stp = timed_solves(spl, f1, SOLVE_TOL, steps, warmup, max_iter,
                                                 region=roctx_form == "fp64_single_plr")
        errp = float(torch.linalg.norm(up[0] - refs[k]) / torch.linalg.norm(refs[k]))
        gp = None
        if golden is not None:
            gp = {}
            for i, g0 in enumerate(golden["sources"]):
                ug = spl.solve(f_all[g0:g0 + 1].contiguous(), tol=SOLVE_TOL, max_iter=max_iter)
                got = ug[0][golden["rows"] - 1].cpu().numpy()
                gp[g0] = float(np.linalg.norm(got - golden["u"][i]) / np.linalg.norm(golden["u"][i]))
                del ug
        spl.close()
        del spl, up
        torch.cuda.empty_cache()
        log(f"[bench] fp64 single RHS with PLR preconditioner: {dtp * 1e3:.1f} ms/solve "
            f"({dtpp * 1e3:.1f} profiled), {stp[0]['iters']} iterations, err vs fp64 {errp:.1e}, "
            f"stored {info.plr_bytes / max(info.plr_dense_bytes, 1):.3f} of dense")
        forms["fp64_single_plr"] = {
            "dof_solves_per_s": n * n / dtp, "ms_per_solve": dtp * 1e3,
            "ms_per_solve_profiled": dtpp * 1e3, "gmres_iters": stp[0]["iters"],
            "rel_err_vs_fp64": errp, "rel_err_vs_oracle_rows": gp, "plr_eps": 1e-8,
            "plr_bytes": info.plr_bytes, "plr_dense_bytes": info.plr_dense_bytes,
            "setup_factor_compress_s": t_facp, "kernels": profp,
            "roofline": roofline(max(profp, key=lambda k: k["ms"]), 1, name)}

    def record(key, solver, tol, dty, t_fac, region):
        u, dt, prof, dtp, st = timed_solves(solver, f_all, tol, steps, warmup, max_iter,
                                            region=roctx_form == region)
        err = max(float(torch.linalg.norm(u[k] - refs[k]) / torch.linalg.norm(refs[k]))
                  for k in ref_idx)
        gerr = golden_errors(u, golden)
        its = max(x["iters"] for x in st)
        vres = max(x["vol_resid"] for x in st)
        results[key] = dict(dt=dt, dtp=dtp, prof=prof, err=err, gerr=gerr, its=its, dty=dty,
                            t_fac=t_fac, vres=vres, refine=max(x["refine_steps"] for x in st),
                            steps_ms=timed_solves.last_steps_ms)
        g = "" if gerr is None else f", oracle rows {max(gerr.values()):.2e}"
        log(f"[bench] {key}: {dt * 1e3:.1f} ms/step ({dtp * 1e3:.1f} profiled), err vs fp64 "
            f"{err:.2e}{g}, iters {its}, max vol. resid {vres:.1e}")
        del u

    if "fp64" in forms_wanted:
        record("fp64_batched", s64, SOLVE_TOL, "c128", t_fac64, "fp64_batched")
    s64.close()
    del s64
    torch.cuda.empty_cache()
    if "mixed" in forms_wanted:
        t0 = time.perf_counter()
        smx = hz.Solver(torch.from_numpy(c), w.omega, w.n_pml, w.layers, w.cells,
                        precision=hz.HZ_MIXED, max_batch=B)
        torch.cuda.synchronize()
        t_fac = time.perf_counter() - t0
        log(f"[bench] mixed setup+factor {t_fac:.2f} s")
        record("mixed_batched", smx, SOLVE_TOL, "c64+c128", t_fac, "mixed_batched")
        if want_local:
            extras["local_refactor"] = local_refactor(smx, c, w, f_all, ref_idx, max_iter)
        smx.close()
        del smx
        torch.cuda.empty_cache()
    if "refine" in forms_wanted:
        t0 = time.perf_counter()
        srf = hz.Solver(torch.from_numpy(c), w.omega, w.n_pml, w.layers, w.cells,
                        precision=hz.HZ_MIXED_REFINE, max_batch=B)
        torch.cuda.synchronize()
        t_fac = time.perf_counter() - t0
        log(f"[bench] refine setup+factor {t_fac:.2f} s")
        # tolerance: estimated relative error of the refined volume solution
        record("refine_batched", srf, SOLVE_TOL, "c64+c128", t_fac, "refine_batched")
        srf.close()
        del srf
        torch.cuda.empty_cache()
    if "nested" in forms_wanted:
        # nested polarized traces (Sec. 4.2.1): no inner factorisation; every
        # layer application iterates the inner polarized system (inner
        # tolerance 1e-6 inside the preconditioner, flexible outer GMRES)
        t0 = time.perf_counter()
        spt = hz.Solver(torch.from_numpy(c), w.omega, w.n_pml, w.layers, w.cells,
                        precision=hz.HZ_FP64, max_batch=B, inner=hz.HZ_INNER_PT, inner_tol=1e-6)
        torch.cuda.synchronize()
        t_fac = time.perf_counter() - t0
        log(f"[bench] nested polarized traces setup+factor {t_fac:.2f} s")
        extras["memory"]["fp64_nested_pt_device_bytes"] = spt.info.device_bytes
        record("nested_pt_batched", spt, SOLVE_TOL, "c128", t_fac, "nested_pt_batched")
        spt.close()
        del spt
        torch.cuda.empty_cache()
    if "table3" in forms_wanted:
        # the iteration-count comparison of the paper (Table 3: GMRES and
        # Bi-CGstab with the Gauss-Seidel and Jacobi preconditioners, relative
        # residual 1e-7) on this workload, FP64, whole batch per solve
        table3 = {}
        for pre, pname in ((hz.HZ_PRECOND_GS, "gs"), (hz.HZ_PRECOND_JACOBI, "jacobi")):
            for kry, kname in ((hz.HZ_KRYLOV_GMRES, "gmres"), (hz.HZ_KRYLOV_BICGSTAB, "bicgstab")):
                st = hz.Solver(torch.from_numpy(c), w.omega, w.n_pml, w.layers, w.cells,
                               precision=hz.HZ_FP64, max_batch=B, precond=pre, krylov=kry)
                u, dtt, _, _, sts = timed_solves(st, f_all, 1e-7, steps, warmup, max_iter,
                                                 prof_steps=0)
                itt = max(x["iters"] for x in sts)
                errt = max(float(torch.linalg.norm(u[k] - refs[k]) / torch.linalg.norm(refs[k]))
                           for k in ref_idx)
                table3[f"{pname}_{kname}"] = {"iters": itt, "ms_per_step": dtt * 1e3,
                                              "max_rel_err_vs_fp64": errt}
                log(f"[bench] table3 {pname}/{kname}: {itt} iterations, {dtt * 1e3:.1f} ms/step, "
                    f"err {errt:.1e}")
                st.close()
                del st, u
                torch.cuda.empty_cache()
        extras["table3"] = table3
    for key, r in results.items():
        forms[key] = {"dof_solves_per_s": B * n * n / r["dt"], "ms_per_step": r["dt"] * 1e3,
                      "steps_ms": r["steps_ms"], "ms_per_step_profiled": r["dtp"] * 1e3,
                      "max_rel_err_vs_fp64": r["err"],
                      "rel_err_vs_oracle_rows": r["gerr"], "max_vol_resid": r["vres"],
                      "gmres_iters": r["its"], "refine_steps": r["refine"],
                      "dtype": r["dty"], "setup_factor_s": r["t_fac"],
                      "amortized_dof_solves_per_s": B * n * n / (r["dt"] + r["t_fac"]),
                      "kernels": r["prof"],
                      "roofline": roofline(max(r["prof"], key=lambda k: k["ms"]), B, name)}
    del f_all
    torch.cuda.empty_cache()
    return w, forms, results, extras


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C4")
    ap.add_argument("--also", default="C3",
                    help="comma list of further workloads timed in the fp64 / mixed / refine "
                         "batched forms (reported under other_workloads; '' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="single,plr,fp64,mixed,refine,nested",
                    help="comma list of single (FP64, one RHS per solve), plr (the same with the "
                         "preconditioner's operators in partitioned low-rank form), fp64, mixed, "
                         "refine, "
                         "nested (nested polarized traces: inner GMRES instead of the inner "
                         "block LU), local (re-factorisation after a local model update, on "
                         "the mixed context), table3 (Krylov x preconditioner comparison)")
    ap.add_argument("--roctx-form", default="",
                    help="mark this form's timed steps as the profiled region (fp64_single, "
                         "fp64_batched, mixed_batched, refine_batched or nested_pt_batched)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="only run one plain copy of this many bytes (counter reference)")
    args = ap.parse_args()
    if args.copy_calib:
        copy_calibration(args.copy_calib)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding the path over several GPUs is designed but not built.", file=sys.stderr)
        sys.exit(2)

    forms_wanted = set(args.forms.split(","))
    w, forms, results, extras = run_workload(args.workload, forms_wanted, args.steps,
                                             args.warmup, args.roctx_form,
                                             want_local="local" in forms_wanted)
    n, B = w.n, w.n_rhs

    def ok(r):
        if r["err"] > ERR_BAR:
            return False
        return r["gerr"] is None or max(r["gerr"].values()) <= ERR_BAR

    good = {k: v for k, v in results.items() if ok(v)}
    pool = good if good else results
    if pool:
        chosen = min(pool, key=lambda k: pool[k]["dt"])
        r = results[chosen]
        roof = roofline(max(r["prof"], key=lambda k: k["ms"]), B, w.name)
        step_dofs = B * n * n
    else:                              # only the single-RHS form was timed
        chosen = "fp64_single"
        f1 = forms["fp64_single"]
        r = dict(dt=f1["ms_per_solve"] * 1e-3, prof=f1["kernels"], err=0.0, gerr=None,
                 its=f1["gmres_iters"], dty="c128", t_fac=f1["setup_factor_s"])
        roof = f1["roofline"]
        step_dofs = n * n

    others = {}
    for name in [x for x in args.also.split(",") if x and x != args.workload]:
        wo, fo, _, _ = run_workload(name, {"fp64", "mixed", "refine", "nested"} & forms_wanted,
                                    args.steps, args.warmup)
        others[name] = {"workload": (f"{wo.name}: n={wo.n} (+{wo.n_pml} PML), {MEDIUM[wo.name]}, "
                                     f"{wo.layers} layers x {wo.cells} cells, {wo.n_rhs} sources"),
                        "forms": fo}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on the host) ...")
        from paper_1510_01831_amd import media

        cpu = cpu_baseline(w, media.velocity(w.name), results.get("fp64_batched", r)["its"])
        log(f"[bench] cpu baseline {cpu['value']:.3e} DOF-solves/s ({cpu['sample']})")

    single = forms.get("fp64_single")
    fp64b = forms.get("fp64_batched")
    line = {
        "metric": METRIC,
        "value": step_dofs / r["dt"],
        "unit": "DOF-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["dt"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": r["dty"],
        "data": "synthetic",
        "config": {"workload": (f"{w.name}: n={n} (+{w.n_pml} PML), {MEDIUM[w.name]}, "
                                f"omega={w.omega:.2f} (10 ppw at c_min), {w.layers} layers x "
                                f"{w.cells} cells, {B} point sources on depth row {w.src_z}"),
                   "form": chosen, "batch": B if pool else 1, "krylov_tol": SOLVE_TOL,
                   "max_rel_err_vs_fp64": r["err"],
                   "rel_err_vs_oracle_rows": r["gerr"], "gmres_iters": r["its"],
                   "setup_factor_s": r["t_fac"],
                   "amortized_dof_solves_per_s": step_dofs / (r["dt"] + r["t_fac"])},
        "vs_plain_fp64_single": ((step_dofs / r["dt"]) / single["dof_solves_per_s"]
                                 if single else None),
        "vs_plain_fp64_batched": ((step_dofs / r["dt"]) / fp64b["dof_solves_per_s"]
                                  if fp64b else None),
        "forms": forms,
        "kernels": r["prof"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "other_workloads": others,
        **extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
