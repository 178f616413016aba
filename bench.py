"""Benchmark: DOF-solves/s of the nested polarized-traces solver on one MI355X.

Workload (default): the n = 1023 Gaussian-random-field medium (c in
[1.5, 3.0], correlation length 0.05, seed 0), 32-node PML, omega for 10
points per wavelength at c_min, 16 layers x 4 cells, 256 point sources
equally spaced on depth row 0.1 -- a synthetic stand-in for the paper's
BP2004 runs (same contrast range, sampling and source geometry).

One "step" is one call of hz_solve on the whole batch of 256 right-hand
sides (RHS formation, GMRES on the polarized SIE with the Gauss-Seidel
sweeps, volume reconstruction), inputs resident in HBM.  Three forms are
timed: plain FP64 with one RHS, FP64 with the batch, and the mixed form
(complex64 preconditioner, complex128 SIE / volume / Krylov) with the batch.
`value` is the faster batched form whose solutions agree with the plain
FP64 solves to a relative L2 error <= 1e-8.

The dominant kernel family's roofline comes from HIP events recorded on the
solver's stream around every launch during the timed steps; the CPU baseline
is the oracle's global sparse direct solve on the same system.
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


def timed_solves(solver, f, tol, steps, warmup, max_iter, profile=False, region=False):
    import torch

    for _ in range(warmup):
        solver.solve(f, tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    if profile:
        solver.profile(True)
    if region:
        roctx_region(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        u = solver.solve(f, tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    if region:
        roctx_region(False)
    prof = solver.profile_read() if profile else None
    if profile:
        solver.profile(False)
    return u, dt, prof


KERNEL_SOURCES = {"gemm": ["k_gemm.hip", "hz_mfma.h", "hz_common.h"],
                  "cell_solve": ["k_cellsolve.hip", "hz_mfma.h", "hz_common.h"]}


def kernel_src_hash(family):
    """Hash of the sources of one kernel family (traffic figures recorded in
    profiles/ are used only while the kernel is unchanged)."""
    import hashlib

    group = "gemm" if family.startswith(("gemm", "gemv")) else "cell_solve"
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[group]:
        with open(os.path.join(ROOT, "paper_1510_01831_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(family):
    """HBM bytes per launch measured with the FETCH_SIZE / WRITE_SIZE
    counters for this kernel, from the summaries in profiles/; None when no
    summary covers the kernel as it is now."""
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
                if kv.get("kernel") == family and kv.get("src") == want:
                    return float(kv["bytes_per_launch"])
    return None


def roofline(k, B):
    """Roofline record of one kernel family from the solver's event profile:
    matrix-core kernels against the dense MFMA peak of their precision,
    single-column kernels (matrix-vector products) against HBM bandwidth."""
    prec = "c64" if k["name"].endswith("_c64") else "c128"
    avg_ms = k["ms"] / k["launches"]
    rec = {"kernel": k["name"], "launches": k["launches"], "avg_launch_ms": avg_ms,
           "flops_per_launch": k["flops"] / k["launches"],
           "bytes_per_launch": k["bytes"] / k["launches"], "traffic": recorded_traffic(k["name"])}
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


def cpu_baseline(c, omega, n_pml, src_x, src_z, nsample=8):
    """The oracle's direct solve (SuperLU via SciPy) on the same system:
    factor once, then solve a bounded sample of the batch."""
    import numpy as np
    import scipy.sparse.linalg as spla

    from oracle.discretization import Problem
    from paper_1510_01831_amd import media

    n = c.shape[0]
    t0 = time.perf_counter()
    prob = Problem(c, omega, n_pml)
    lu = spla.splu(prob.H.tocsc())
    t_fac = time.perf_counter() - t0
    idx = np.linspace(0, len(src_x) - 1, nsample).round().astype(int)
    f = media.point_sources(n, tuple(src_x[i] for i in idx), src_z)
    F = np.stack([prob.extend(x).ravel() for x in f], axis=1)
    t0 = time.perf_counter()
    lu.solve(F)
    t_sol = time.perf_counter() - t0
    return {
        "value": nsample * n * n / t_sol,
        "unit": "DOF-solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"global sparse LU of the same n={n} system (SciPy SuperLU, single "
                   f"thread): factor once ({t_fac:.1f} s, not in value), then {nsample} of "
                   f"the 256 sources solved in {t_sol:.2f} s; value = online DOF-solves/s"),
        "t_factor_s": t_fac,
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp64,mixed,local,nested",
                    help="comma list of fp64, mixed, local (re-factorisation after a local "
                         "model update, on the mixed context), nested (nested polarized "
                         "traces: inner GMRES instead of the inner block LU), table3 (Krylov "
                         "x preconditioner comparison)")
    ap.add_argument("--roctx-form", default="",
                    help="mark this form's timed steps as the profiled region "
                         "(fp64_single, fp64_batched or mixed_batched)")
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

    import numpy as np
    import torch

    from paper_1510_01831_amd import hz, media

    w = media.workload(args.workload)
    c = media.velocity(args.workload)
    n = w.n
    B = w.n_rhs
    f_all = torch.from_numpy(media.point_sources(n, w.src_x, w.src_z)).cuda()
    max_iter = 60
    log(f"[bench] workload {w.name}: n={n} pml={w.n_pml} L={w.layers} Lc={w.cells} B={B}")

    # ---- plain FP64 (one context, used for single-RHS and batched solves)
    t0 = time.perf_counter()
    s64 = hz.Solver(torch.from_numpy(c), w.omega, w.n_pml, w.layers, w.cells,
                    precision=hz.HZ_FP64, max_batch=B)
    torch.cuda.synchronize()
    t_fac64 = time.perf_counter() - t0
    log(f"[bench] fp64 setup+factor {t_fac64:.2f} s")
    f1 = f_all[B // 2: B // 2 + 1].contiguous()
    u1, dt1, prof1 = timed_solves(s64, f1, 1e-10, args.steps, args.warmup, max_iter, profile=True,
                                  region=args.roctx_form == "fp64_single")
    it1 = s64.last_stats[0]["iters"]
    log(f"[bench] fp64 single RHS: {dt1 * 1e3:.1f} ms/solve, {it1} GMRES iterations")
    forms = {"fp64_single": {"dof_solves_per_s": n * n / dt1, "ms_per_solve": dt1 * 1e3,
                             "gmres_iters": it1, "setup_factor_s": t_fac64, "kernels": prof1,
                             "roofline": roofline(max(prof1, key=lambda k: k["ms"]), 1)}}
    ref_idx = [0, B // 2, B - 1]
    refs = {}
    for k in ref_idx:
        refs[k] = s64.solve(f_all[k:k + 1].contiguous(), tol=1e-12, max_iter=max_iter)[0]
    results = {}
    local = None
    mem = {"fp64_inner_lu_device_bytes": s64.info.device_bytes}
    if "fp64" in args.forms:
        u, dt, prof = timed_solves(s64, f_all, 1e-10, args.steps, args.warmup, max_iter, True,
                                   region=args.roctx_form == "fp64_batched")
        err = max(float(torch.linalg.norm(u[k] - refs[k]) / torch.linalg.norm(refs[k]))
                  for k in ref_idx)
        its = max(x["iters"] for x in s64.last_stats)
        results["fp64_batched"] = (dt, prof, err, its, "c128", t_fac64)
        log(f"[bench] fp64 batched: {dt * 1e3:.1f} ms/step, err {err:.2e}, iters {its}")
    s64.close()
    del s64
    torch.cuda.empty_cache()
    if "mixed" in args.forms:
        t0 = time.perf_counter()
        smx = hz.Solver(torch.from_numpy(c), w.omega, w.n_pml, w.layers, w.cells,
                        precision=hz.HZ_MIXED, max_batch=B)
        torch.cuda.synchronize()
        t_facmx = time.perf_counter() - t0
        log(f"[bench] mixed setup+factor {t_facmx:.2f} s")
        u, dt, prof = timed_solves(smx, f_all, 1e-10, args.steps, args.warmup, max_iter, True,
                                   region=args.roctx_form == "mixed_batched")
        err = max(float(torch.linalg.norm(u[k] - refs[k]) / torch.linalg.norm(refs[k]))
                  for k in ref_idx)
        its = max(x["iters"] for x in smx.last_stats)
        results["mixed_batched"] = (dt, prof, err, its, "c64+c128", t_facmx)
        log(f"[bench] mixed batched: {dt * 1e3:.1f} ms/step, err {err:.2e}, iters {its}")
        if "local" in args.forms:
            local = local_refactor(smx, c, w, f_all, ref_idx, max_iter)
        smx.close()
        del smx
    if "nested" in args.forms:
        # nested polarized traces (Sec. 4.2.1): no inner factorisation; every
        # layer application iterates the inner polarized system (inner
        # tolerance 1e-6 inside the preconditioner, flexible outer GMRES)
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        spt = hz.Solver(torch.from_numpy(c), w.omega, w.n_pml, w.layers, w.cells,
                        precision=hz.HZ_FP64, max_batch=B, inner=hz.HZ_INNER_PT, inner_tol=1e-6)
        torch.cuda.synchronize()
        t_facpt = time.perf_counter() - t0
        log(f"[bench] nested polarized traces setup+factor {t_facpt:.2f} s")
        u, dt, prof = timed_solves(spt, f_all, 1e-10, args.steps, args.warmup, max_iter, True)
        err = max(float(torch.linalg.norm(u[k] - refs[k]) / torch.linalg.norm(refs[k]))
                  for k in ref_idx)
        its = max(x["iters"] for x in spt.last_stats)
        inner_its = spt.timing()["inner_iters"]
        results["nested_pt_batched"] = (dt, prof, err, its, "c128", t_facpt)
        mem["fp64_nested_pt_device_bytes"] = spt.info.device_bytes
        log(f"[bench] nested polarized traces batched: {dt * 1e3:.1f} ms/step, err {err:.2e}, "
            f"iters {its}, inner iters <= {inner_its}")
        spt.close()
        del spt
        torch.cuda.empty_cache()
    table3 = None
    if "table3" in args.forms:
        # the iteration-count comparison of the paper (Table 3: GMRES and
        # Bi-CGstab with the Gauss-Seidel and Jacobi preconditioners, relative
        # residual 1e-7) on this workload, FP64, whole batch per solve
        table3 = {}
        for pre, pname in ((hz.HZ_PRECOND_GS, "gs"), (hz.HZ_PRECOND_JACOBI, "jacobi")):
            for kry, kname in ((hz.HZ_KRYLOV_GMRES, "gmres"), (hz.HZ_KRYLOV_BICGSTAB, "bicgstab")):
                st = hz.Solver(torch.from_numpy(c), w.omega, w.n_pml, w.layers, w.cells,
                               precision=hz.HZ_FP64, max_batch=B, precond=pre, krylov=kry)
                u, dtt, _ = timed_solves(st, f_all, 1e-7, args.steps, args.warmup, max_iter)
                itt = max(x["iters"] for x in st.last_stats)
                errt = max(float(torch.linalg.norm(u[k] - refs[k]) / torch.linalg.norm(refs[k]))
                           for k in ref_idx)
                table3[f"{pname}_{kname}"] = {"iters": itt, "ms_per_step": dtt * 1e3,
                                              "max_rel_err_vs_fp64": errt}
                log(f"[bench] table3 {pname}/{kname}: {itt} iterations, {dtt * 1e3:.1f} ms/step, "
                    f"err {errt:.1e}")
                st.close()
                del st
                torch.cuda.empty_cache()
    for name, (dt, prof, err, its, dty, tf) in results.items():
        forms[name] = {"dof_solves_per_s": B * n * n / dt, "ms_per_step": dt * 1e3,
                       "max_rel_err_vs_fp64": err, "gmres_iters": its,
                       "setup_factor_s": tf,
                       "amortized_dof_solves_per_s": B * n * n / (dt + tf),
                       "kernels": prof,
                       "roofline": roofline(max(prof, key=lambda k: k["ms"]), B)}
    ok = {k: v for k, v in results.items() if v[2] <= 1e-8}
    chosen = min(ok, key=lambda k: ok[k][0]) if ok else min(results, key=lambda k: results[k][0])
    dt, prof, err, its, dty, t_fac = results[chosen]

    # ---- roofline of the dominant kernel of the chosen form (most time in
    # the timed steps; every family is one kernel, timed launch by launch
    # with HIP events on the solver's stream)
    dom = max(prof, key=lambda k: k["ms"])
    roof = roofline(dom, B)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle direct solve) ...")
        cpu = cpu_baseline(c, w.omega, w.n_pml, w.src_x, w.src_z)
        log(f"[bench] cpu baseline {cpu['value']:.3e} DOF-solves/s")

    line = {
        "metric": METRIC,
        "value": B * n * n / dt,
        "unit": "DOF-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dty,
        "data": "synthetic",
        "config": {"workload": (f"{w.name}: n={n} (+{w.n_pml} PML), {MEDIUM[w.name]}, "
                                f"omega={w.omega:.2f} (10 ppw at c_min), {w.layers} layers x "
                                f"{w.cells} cells, {B} point sources on depth row {w.src_z}"),
                   "form": chosen, "batch": B, "tol": 1e-10,
                   "max_rel_err_vs_fp64": err, "gmres_iters": its,
                   "setup_factor_s": t_fac,
                   "amortized_dof_solves_per_s": B * n * n / (dt + t_fac)},
        "vs_plain_fp64_single": (B * n * n / dt) / forms["fp64_single"]["dof_solves_per_s"],
        "forms": forms,
        "kernels": prof,
        "roofline": roof,
        "cpu_baseline": cpu,
        "table3": table3,
        "local_refactor": local,
        "memory": mem,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
