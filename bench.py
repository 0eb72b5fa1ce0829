#!/usr/bin/env python3
"""Benchmark: gated QP solves/s of the batched ADMM OCP-QP path on one MI355X.

One step = one pass of the hot path over the batch: for every instance the
FP64 block factorisation, the ADMM iterations (FP32 over the FP64 factor, or
plain FP64), the rho adaptations with their refactorisations and the FP64
stopping test, then the implicit-gradient adjoint ("+grad") of every
instance for a seeded upstream gradient.  An instance counts as solved only if its FP64-evaluated
residuals pass the stopping test at eps_abs = eps_rel = 1e-4.

Prints ONE JSON line (rank 0).  Details go to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3  # TFLOP/s, MI355X vector FP32 (published)
PEAK_FP64 = 78.6   # TFLOP/s, MI355X vector FP64 (published)
PEAK_HBM = 8000.0  # GB/s, MI355X HBM3E (published)
SCALE_P = 0.6  # exponent of the box normalisation (ocp_set_scaling_box) on the FP32 path
# PCG primal updates of the direct-vs-PCG comparison: at most 25 CG iterations
# per ADMM iteration, relative residual 1e-5 (about what FP32 iterations resolve)
PCG_ITERS, PCG_TOL = 25, 1e-5

# HBM traffic of one ADMM solve (its launches: the one-wavefront launch and,
# with the continuation on, the two-wavefront one), from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE) of `bench.py --steps 1 --warmup 0
# --cpu-sample 0 --no-fp64 --no-sub`, each scaled by the same counter's reading
# for a plain 1 GiB device copy (`bench.py --copy-calibration 1024`).  Keyed by
# (workload, precision, hash of the kernel code, comments and layout left
# out): a changed kernel reports null until it is profiled again.  Summary and commands:
# profiles/admm_solve_wave_tail_lti1024_n50.md.
TRAFFIC_BYTES = {
    # one solve = admm_solve_wave_kernel + admm_solve_tail_kernel (continuation from iteration 200):
    # FETCH_SIZE (14,708,718.4 + 699,035.4) KiB x 1.99994 + WRITE_SIZE (1,097,993.8 + 773,955.6) KiB x 1.000
    ("c2", "mixed", "439f73a5bfd54c19"): 33_470_944_306,
}


def _code_only(text: str) -> str:
    """C/C++ source without its comments, whitespace runs collapsed (string
    and character literals kept as written)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """sha256 (16 hex digits) over the code the kernels are compiled from:
    csrc/inst.hip and every header it includes, transitively (the host code
    and the SQP-only kernels do not enter it), comments and layout left out,
    so that only a change of the code itself invalidates a measurement."""
    import hashlib
    import re

    dirs = [os.path.join(ROOT, "paper_2606_24039_amd", "csrc"), os.path.join(ROOT, "include")]
    seen, todo = [], ["inst.hip"]
    while todo:
        name = todo.pop()
        if name in seen:
            continue
        path = next((os.path.join(d, name) for d in dirs if os.path.exists(os.path.join(d, name))), None)
        if path is None:
            continue  # a system header
        seen.append(name)
        with open(path, encoding="utf-8") as f:
            todo += re.findall(r'^\s*#\s*include\s+"([^"]+)"', f.read(), re.M)
    h = hashlib.sha256()
    for name in sorted(seen):
        path = next(os.path.join(d, name) for d in dirs if os.path.exists(os.path.join(d, name)))
        with open(path, encoding="utf-8") as f:
            h.update(name.encode() + b"\0" + _code_only(f.read()).encode())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# algorithmic work per unit (flops per stage per iteration / factorisation)
# ---------------------------------------------------------------------------
def lti_flops_per_stage(nx, nu, ng):
    """(FP32-path flops per stage per ADMM iteration, FP64 flops per stage per
    factorisation) for the LTI layout A^- = [A B] dense, A^+ = [-I 0], G a
    0/1 selection with ng rows."""
    n = nx + nu
    nnz = nx * n + nx + ng
    f_eta = 2 * nnz + 6 * (nx + ng + n)
    f_sub = 2 * (2 * n * n + n * (n + 1))
    f_az = 2 * nnz
    f_elem = 12 * ng + 6 * nx + 4 * n
    f_it = f_eta + f_sub + f_az + f_elem
    f_fac = 2 * nx * n * n + 2 * nx * n + n ** 3 + n ** 3 / 3 + n ** 3 / 3 + n ** 3
    return f_it, f_fac


def lti_bytes_per_stage(n, ts, blocks, k_seg=25):
    """Algorithmic bytes one ADMM iteration moves per stage, for the design
    measured here (FP32 iterations, horizons up to 55 stages): `blocks` n x n
    factor blocks stream from memory per iteration (W_t and V_t once each, the
    packed Linv_t twice: pass 1 and pass 3 read it, and an instance's blocks do
    not stay in the L2 between them); the six padded 16-entry stage vectors stay in LDS for a
    segment of `k_seg` iterations, so five of them (x, y_f, z_g, y_g, xi) move
    in and out once per segment."""
    return blocks * n * n * ts + (2 * 5 * 16 * ts) / k_seg


def seg_bytes_per_stage(n, ts):
    """The same for the segmented sweeps of the two-wavefront continuation:
    the packed Linv_t and both chain blocks are read twice per iteration (the
    particular and the true sweep of each chain), and the sweeps move 16
    padded stage vectors through global memory (eta inputs, x~, the
    exchange vector and the constraint-row state)."""
    return 6 * n * n * ts + 16 * 16 * ts


def make_workload(name):
    from workloads import random_lti

    if name == "c2":
        b = random_lti(1024, N=50, nx=12, nu=4, seed=2)
        desc = ("batched linear MPC: 1024 random LTI instances, nx=12, nu=4, N=50, "
                "A=I+0.1G (spectral radius of G 1.05), x in [-10,10], u in [-1,1]")
        return b, desc
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(batch, sample, settings_kw, grad):
    """The FP64 oracle on the host cores, one instance per task: the ADMM
    solve and (with grad) the active-set adjoint of the same instance.  Uses
    every core of the affinity mask up to 16, the CPU share of one GPU on the
    benchmark hosts."""
    import multiprocessing as mp

    global _CPU_BATCH
    _CPU_BATCH = batch
    cores = max(1, min(len(os.sched_getaffinity(0)), 16, sample))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores, initializer=_worker_init) as pool:
        res = pool.map(_oracle_one, [(i, settings_kw, grad) for i in range(sample)], chunksize=1)
    wall = time.perf_counter() - t0
    solved = sum(1 for ok, _ in res if ok)
    iters = sum(it for _, it in res)
    return {"value": solved / wall, "unit": "QP solves/s", "cores": cores, "kind": "oracle",
            "sample": (f"first {sample} of {batch.batch} instances, FP64 NumPy/SciPy oracle, eps 1e-4"
                       + (", ADMM solve + active-set adjoint (sparse LU; minimum-norm where the active rows "
                          "are dependent)" if grad else ", ADMM solve")),
            "solved": solved, "wall_s": round(wall, 3), "admm_iters_per_s": iters / wall}


def _worker_init():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    # the BLAS pools were created before the fork: cap them in each worker
    from threadpoolctl import threadpool_limits

    threadpool_limits(1)


_CPU_BATCH = None


def _oracle_one(args):
    i, kw, grad = args
    batch = _CPU_BATCH
    from oracle.admm import ADMMSettings, admm_solve
    from oracle.qp import lti_batch_qp

    qp = lti_batch_qp(batch, i)
    r = admm_solve(qp, ADMMSettings(**kw))
    if grad:
        from oracle.adjoint import active_set, adjoint_dense, qp_vjp

        S = batch.N + 1
        dl = upstream_gradient(batch)[i * S:(i + 1) * S].reshape(-1)
        lower, upper = active_set(qp, r.x, r.y_g, r.xi)
        ex, ef, eg = adjoint_dense(qp, r.x, dl, lower, upper)
        qp_vjp(qp, r.x, ex, ef, eg, lower, upper)
    return r.status == 0, r.iters


def upstream_gradient(batch, seed=11):
    """Seeded dL/dx for the "+grad" leg: one fixed cotangent per stage
    variable, standard normal (the loss itself is the caller's)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((batch.batch * (batch.N + 1), batch.nx + batch.nu))


def run_gpu(batch, precision, steps, warmup, settings_kw, grad=True, scale_p=None, tune=False, pcg=None):
    import torch

    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    hz = np.full(batch.batch, batch.N)
    s = OCPSolver(batch.nx, batch.nu, batch.ng, hz, model=A.MODEL_LTI, precision=precision)
    if scale_p is not None:
        s.set_scaling_box(scale_p)
    s.set_lti(batch.A, batch.B, batch.Qd, batch.Rd, batch.Qfd, batch.G, batch.lo, batch.hi, batch.x0)
    if pcg is not None:  # (max CG iterations, relative tolerance): PCG primal updates
        s.set_linsolve(True, max_iter=pcg[0], tol=pcg[1])
        tune = False  # no launch-shape choice for the stage-parallel PCG updates
    st = A.default_settings(**settings_kw)
    shape = s.autotune(st, reps=2) if tune else None  # launch shape picked on this batch (not timed)
    out = s.alloc_solution()
    sol = s.solution_struct(out)
    grads = s.alloc_grads()
    gstruct = s.grads_struct(grads)
    dl = torch.as_tensor(upstream_gradient(batch), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        s.solve_raw(st, None)
        A.check(s.lib.ocp_get_solution(s.h, A.C.byref(sol), A.C.c_void_p(stream.cuda_stream)), "get_solution")
        if grad:
            s.adjoint_raw(st, dl, gstruct)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    s.profile(True)
    s.profile_read()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = s.profile_read()
    s.profile(False)
    status = out["status"].cpu().numpy()
    iters = out["admm_iters"].cpu().numpy()
    nfact = out["n_factor"].cpu().numpy()
    ok = status == 0
    if grad:  # "+grad": the instance's gradient must be refined to the tolerance too
        ok &= grads["adj_status"].cpu().numpy() == 0
    solved = int(ok.sum())
    tail = shape[2] if shape else 0
    res = {"wall_s": wall, "ms_per_step": wall / steps * 1e3, "solved": solved, "batch": batch.batch,
           "iters_mean": float(iters.mean()), "iters_max": int(iters.max()), "iters_sum": int(iters.sum()),
           "iters_pct": {p: int(np.percentile(iters, p)) for p in (50, 90, 99)},
           "iters_capped": int((iters >= settings_kw.get("max_admm", 1000)).sum()),
           "nfact_sum": int(nfact.sum()),
           # instance-iterations of the one-wavefront launch and of the continuation
           "iters_split": [int(np.minimum(iters, tail).sum()) if tail else int(iters.sum()),
                           int(np.maximum(iters - tail, 0).sum()) if tail else 0],
           "status_counts": {int(k): int(v) for k, v in zip(*np.unique(status, return_counts=True))},
           "kernels": {k: {"ms_per_step": ms / steps, "launches_per_step": c / steps} for k, (ms, c) in kt.items()},
           "launch_shape": ({"segmented_from_horizon": shape[0], "segmented_from_iteration": shape[1],
                             "two_wavefront_from_iteration": shape[2]}
                            if shape else None)}
    if grad:
        ast = grads["adj_status"].cpu().numpy()
        res["adjoint"] = {"status_counts": {int(k): int(v) for k, v in zip(*np.unique(ast, return_counts=True))},
                          "ok_on_solved": int(((ast == 0) & (status == 0)).sum()),
                          "resid_max_ok": float(grads["adj_resid"].cpu().numpy()[ast == 0].max(initial=0.0))}
    s.close()
    return res


def run_bicycle(batch, precision, steps, warmup, settings_kw, grad=True, pcg=None):
    """Timed SQP solves (+ the adjoint of the last QP) of a kinematic-bicycle batch."""
    import torch

    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    s = OCPSolver(4, 2, 3, batch.horizons, model=A.MODEL_BICYCLE, precision=precision)
    if pcg is not None:
        s.set_linsolve(True, max_iter=pcg[0], tol=pcg[1])
    s.set_bicycle(batch)
    st = A.default_settings(**settings_kw)
    out = s.alloc_solution()
    grads = s.alloc_grads()
    gstruct = s.grads_struct(grads)
    dl = torch.as_tensor(np.random.default_rng(11).standard_normal((s.S, 6)), dtype=torch.float64, device="cuda")

    def step():
        s.solve(st, out=out, sync=False)
        if grad:
            s.adjoint_raw(st, dl, gstruct)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    s.profile(True)
    s.profile_read()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = s.profile_read()
    s.profile(False)
    kkt = out["sqp_kkt"].cpu().numpy()
    res = {"ms_per_step": wall / steps * 1e3,
           "kernel_ms_per_step": {k: round(ms / steps, 4) for k, (ms, c) in kt.items()},
           "sqp_kkt_max": [float(v) for v in np.nanmax(kkt, axis=0)],
           "adj_status_counts": ({int(k): int(v) for k, v in zip(*np.unique(grads["adj_status"].cpu().numpy(),
                                                                             return_counts=True))}
                                 if grad else None)}
    s.close()
    return res


def bench_bicycle(args):
    """Kinematic-bicycle workloads (implicit midpoint, 10 SQP x 50 ADMM
    iterations with fixed counts, forward + adjoint): `c3` 4096 instances of
    N = 100, `c5a` one instance of N = 8192, `c5b` 256 instances of
    N ~ U{32..2048}."""
    from workloads import bicycle_long_and_ragged

    if args.workload == "c3":
        from workloads import bicycle_batch

        batch = bicycle_batch(4096, N=100, seed=3)
        desc = "kinematic bicycle, 4096 instances N=100"
    else:
        lng, rag = bicycle_long_and_ragged(seed=5)
        batch = lng if args.workload == "c5a" else rag
        desc = ("kinematic bicycle, one instance N=8192" if args.workload == "c5a"
                else "kinematic bicycle, 256 instances N~U{32..2048}")
    kw = dict(max_sqp=10, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1)
    steps, warmup = max(1, min(args.steps, 5)), max(1, min(args.warmup, 2))
    log(f"[bench] workload: {desc}")
    pcg = (args.pcg_iters, args.pcg_tol) if args.linsolve == "pcg" else None
    mixed = run_bicycle(batch, 1, steps, warmup, kw, grad=not args.no_grad, pcg=pcg)
    out = {"metric": "SQP solves/s (10 SQP x 50 ADMM iterations, fixed counts), FP32 ADMM iterations + FP64 "
                     "factorisation" + ("" if args.no_grad else ", + adjoint of the last QP"),
           "value": round(batch.batch / (mixed["ms_per_step"] * 1e-3), 4), "unit": "SQP solves/s", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": round(mixed["ms_per_step"], 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": desc, "batch": int(batch.batch), "stages": int(np.sum(batch.horizons + 1)),
                      "nx": 4, "nu": 2, "ng": 3, "grad": not args.no_grad,
                      "parallelism": ("single GPU; one wavefront per instance" if pcg else
                                      "single GPU; one wavefront per instance, one 8-wavefront workgroup per "
                                      "instance with N >= 255"),
                      "linsolve": ({"pcg_max_iter": pcg[0], "pcg_tol": pcg[1]} if pcg else "direct")},
           "kernel_ms_per_step": mixed["kernel_ms_per_step"], "sqp_kkt_max": mixed["sqp_kkt_max"],
           "roofline": None, "cpu_baseline": None}
    if not args.no_fp64:
        fp64 = run_bicycle(batch, 0, steps, 1, kw, grad=not args.no_grad)
        out["fp64"] = {"ms_per_step": round(fp64["ms_per_step"], 3), "kernel_ms_per_step": fp64["kernel_ms_per_step"],
                       "sqp_kkt_max": fp64["sqp_kkt_max"]}
        out["speedup_vs_fp64"] = round(fp64["ms_per_step"] / mixed["ms_per_step"], 3)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c5a", "c5b"],
                    help="c2: the batched linear MPC benchmark; c3: 4096 bicycle instances, N = 100; "
                         "c5a / c5b: the long / ragged bicycle horizons")
    ap.add_argument("--cpu-sample", type=int, default=1024, help="instances timed on the oracle (0 = skip)")
    ap.add_argument("--no-sub", action="store_true", help="skip the differentiation and double-integrator sub-results")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shape (no ocp_autotune)")
    ap.add_argument("--no-scaling", action="store_true",
                    help="FP32 path without the problem rescaling (Remark 4) the headline uses")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain-FP64 comparison")
    ap.add_argument("--no-grad", action="store_true", help="forward solves only (no adjoint in the step)")
    ap.add_argument("--linsolve", default="direct", choices=["direct", "pcg"],
                    help="primal-update solver of the measured run (pcg: block-Jacobi PCG, --pcg-iters / --pcg-tol)")
    ap.add_argument("--pcg-iters", type=int, default=PCG_ITERS)
    ap.add_argument("--pcg-tol", type=float, default=PCG_TOL)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        import torch

        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "copies": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the batched solve has no "
                                   "cross-GPU exchange; run one process per GPU on disjoint instance shards"}))
        sys.exit(2)

    if args.workload in ("c3", "c5a", "c5b"):
        bench_bicycle(args)
        return
    batch, desc = make_workload(args.workload)
    settings_kw = dict(eps_abs=1e-4, eps_rel=1e-4, max_admm=1000, k_check=25, k_rho=25, eps_active=1e-4)
    scale_p = None if args.no_scaling else SCALE_P
    log(f"[bench] workload: {desc}")
    pcg = (args.pcg_iters, args.pcg_tol) if args.linsolve == "pcg" else None
    mixed = run_gpu(batch, 1, args.steps, args.warmup, settings_kw, grad=not args.no_grad, scale_p=scale_p, pcg=pcg,
                    tune=not args.no_tune)
    log(f"[bench] mixed: {json.dumps(mixed)}")
    fp64 = None
    variants = {}
    if not args.no_fp64:
        fp64 = run_gpu(batch, 0, max(3, args.steps // 4), 1, settings_kw, grad=not args.no_grad)
        log(f"[bench] fp64: {json.dumps(fp64)}")
        # the other two combinations of precision and rescaling, for context
        for name, prec, sp in (("fp32_unscaled", 1, None), ("fp64_rescaled", 0, SCALE_P)):
            if (sp is None) == (scale_p is None) and prec == 1:
                continue
            r = run_gpu(batch, prec, max(3, args.steps // 4), 1, settings_kw, grad=not args.no_grad, scale_p=sp)
            variants[name] = {"value": round(r["solved"] / (r["ms_per_step"] * 1e-3), 2),
                              "ms_per_step": round(r["ms_per_step"], 4), "solved_fraction": r["solved"] / batch.batch,
                              "iters_mean": round(r["iters_mean"], 1), "iters_capped": r["iters_capped"]}
            log(f"[bench] {name}: {json.dumps(r)}")
        if pcg is None:  # the direct-vs-PCG comparison (the PCG backend on the same FP32 rescaled path)
            r = run_gpu(batch, 1, max(3, args.steps // 4), 1, settings_kw, grad=not args.no_grad, scale_p=scale_p,
                        pcg=(args.pcg_iters, args.pcg_tol))
            variants["fp32_pcg"] = {"value": round(r["solved"] / (r["ms_per_step"] * 1e-3), 2),
                                    "ms_per_step": round(r["ms_per_step"], 4),
                                    "solved_fraction": r["solved"] / batch.batch,
                                    "iters_mean": round(r["iters_mean"], 1), "iters_capped": r["iters_capped"],
                                    "pcg": {"max_iter": args.pcg_iters, "tol": args.pcg_tol}}
            log(f"[bench] fp32_pcg: {json.dumps(r)}")

    value = mixed["solved"] / (mixed["ms_per_step"] * 1e-3)
    roof, hbm = roofline(batch, mixed, "mixed", args.workload)
    tail_it = (mixed.get("launch_shape") or {}).get("two_wavefront_from_iteration", 0)
    out = {
        "metric": "QP solves/s at 1e-4 KKT residual, FP32+grad vs plain FP64, 1 MI355X",
        "value": round(value, 2), "unit": "QP solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mixed["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": desc, "batch": batch.batch, "horizon": batch.N, "nx": batch.nx, "nu": batch.nu,
                   "ng": batch.ng, "precision": "fp32 ADMM iterations, fp64 factorisation, gate and adjoint",
                   "rescaling": (f"box normalisation, power-of-two factors, exponent {scale_p}" if scale_p is not None
                                 else "none"),
                   "eps": 1e-4, "eps_active": 1e-4, "max_admm": 1000, "grad": not args.no_grad,
                   "parallelism": ("single GPU, one instance per wavefront" +
                                   (f"; instances still running at ADMM iteration {tail_it} continue on "
                                    "two-wavefront workgroups" if tail_it else "")),
                   "linsolve": ({"pcg_max_iter": pcg[0], "pcg_tol": pcg[1]} if pcg else "direct")},
        "admm_iters_per_s": round(mixed["iters_sum"] / (mixed["ms_per_step"] * 1e-3), 1),
        "kernel_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in mixed["kernels"].items()},
        "solved_fraction": mixed["solved"] / batch.batch,
        "iters": {"mean": round(mixed["iters_mean"], 1), **{f"p{k}": v for k, v in mixed["iters_pct"].items()},
                  "max": mixed["iters_max"], "capped": mixed["iters_capped"]},
        "roofline": roof,
        "hbm_view": hbm,
        "launch_shape": mixed["launch_shape"],
    }
    if "adjoint" in mixed:
        out["adjoint_status"] = mixed["adjoint"]
    if fp64 is not None:
        out["fp64"] = {"value": round(fp64["solved"] / (fp64["ms_per_step"] * 1e-3), 2),
                       "ms_per_step": round(fp64["ms_per_step"], 4),
                       "kernel_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in fp64["kernels"].items()},
                       "solved_fraction": fp64["solved"] / batch.batch, "iters_mean": fp64["iters_mean"],
                       "iters_capped": fp64["iters_capped"]}
        out["speedup_vs_fp64"] = round(value / max(out["fp64"]["value"], 1e-9), 3)
        out["variants"] = variants
    if not args.no_sub:
        out["sub_results"] = sub_results(args)
    if args.cpu_sample > 0:
        cb_kw = dict(eps_abs=1e-4, eps_rel=1e-4, max_iter=1000, k_check=25, k_rho=25)
        out["cpu_baseline"] = cpu_baseline(batch, min(args.cpu_sample, batch.batch), cb_kw, not args.no_grad)
        log(f"[bench] cpu: {json.dumps(out['cpu_baseline'])}")
    print(json.dumps(out), flush=True)


def roofline(batch, res, prec, workload):
    """Roofline of the dominant kernel, the ADMM solve: one persistent launch
    of one wavefront per instance, followed on the same stream, when the
    two-wavefront continuation is on, by the launch that resumes the
    instances still running at its iteration (the two launches of one solve
    are timed together).  Algorithmic work of one solve: F32 =
    instance-iterations x stages x the flops of one stage-iteration, F64 =
    factorisations x stages x the flops of one stage factorisation, bytes =
    problem data in plus solution out.  Roofline time max(bytes / BW, F32 /
    peak32 + F64 / peak64); the kernels are bound by the plain vector ALUs
    (no contraction is dense enough for MFMA), so `achieved` is the
    FP32-equivalent rate against the FP32 vector peak and frac = roofline
    time / measured solve time.  The HBM view (the design's factor stream)
    is reported beside it."""
    f_it, f_fac = lti_flops_per_stage(batch.nx, batch.nu, batch.ng)
    stages = batch.N + 1
    kit = res["kernels"]["solve"]
    tail = (res.get("launch_shape") or {}).get("two_wavefront_from_iteration", 0)
    per_solve = 2 if tail else 1
    launches = max(kit["launches_per_step"] / per_solve, 1)
    t_launch = kit["ms_per_step"] * 1e-3 / launches
    F32 = res["iters_sum"] * stages * f_it / launches
    F64 = res["nfact_sum"] * stages * f_fac / launches
    n = batch.nx + batch.nu
    # FP64 problem data in (A, B, diag Q, diag R, diag Q_f, bounds, x0) and the
    # FP64 solution out (x, y_f, y_g, z_g) per instance
    b_in = 8 * (batch.nx * batch.nx + batch.nx * batch.nu + 2 * batch.nx + batch.nu + 2 * batch.ng + batch.nx)
    b_out = 8 * stages * (n + batch.nx + 2 * batch.ng)
    bytes_alg = batch.batch * (b_in + b_out)
    t_roof = max(bytes_alg / (PEAK_HBM * 1e9), F32 / (PEAK_FP32 * 1e12) + F64 / (PEAK_FP64 * 1e12))
    achieved = (F32 + F64 * PEAK_FP32 / PEAK_FP64) / t_launch / 1e12
    src = kernel_source_hash()
    traffic = TRAFFIC_BYTES.get((workload, prec, src))
    roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK_FP32, "unit": "TFLOP/s",
            "frac": round(t_roof / t_launch, 5), "traffic": traffic,
            "kernel": f"admm_solve_wave_kernel<float,{batch.nx},{batch.nu},{batch.ng},box>" + (
                f" + admm_solve_tail_kernel<float,{batch.nx},{batch.nu},{batch.ng},box> (from iteration {tail})"
                if tail else ""),
            "avg_solve_us": round(t_launch * 1e6, 2), "launches_per_step": kit["launches_per_step"],
            "launches_per_solve": per_solve,
            "flops_fp32_per_launch": F32, "flops_fp64_per_launch": F64, "bytes_per_launch": bytes_alg,
            "flops_per_stage_iteration": f_it, "flops_per_stage_factorisation": f_fac,
            "roofline_time_us": round(t_roof * 1e6, 2), "kernel_source": src}
    b_it = lti_bytes_per_stage(n, 4, 4)
    b_seg = seg_bytes_per_stage(n, 4)
    it_one, it_cont = res["iters_split"]
    design_bytes = (it_one * b_it + it_cont * b_seg) * stages / launches
    hbm = {"design_bytes_per_launch": design_bytes, "bytes_per_stage_iteration": b_it,
           "bytes_per_stage_iteration_continuation": b_seg, "instance_iterations": [it_one, it_cont],
           "achieved_GBps": round(design_bytes / t_launch / 1e9, 1), "peak_GBps": PEAK_HBM,
           "frac": round(design_bytes / t_launch / 1e9 / PEAK_HBM, 4), "measured_traffic": traffic}
    return roof, hbm


def sub_results(args):
    """The other workloads, each at a few steps: the differentiation batch
    (512 random LTI instances, N = 64, +grad, gated at 1e-4; FP32 iterations
    and plain FP64), the single double integrator (N = 20, FP64, 200
    iterations at fixed rho: per-solve latency, and 64 copies) and the
    kinematic-bicycle SQP workloads (4096 x N = 100, one N = 8192 instance,
    256 ragged horizons)."""
    from workloads import double_integrator, random_lti

    sub = {}
    b4 = random_lti(512, N=64, seed=4)
    kw = dict(eps_abs=1e-4, eps_rel=1e-4, max_admm=1000, k_check=25, k_rho=25, eps_active=1e-4)
    steps = max(3, min(args.steps, 10))
    m = run_gpu(b4, 1, steps, 2, kw, grad=True, scale_p=None if args.no_scaling else SCALE_P, tune=not args.no_tune)
    f = run_gpu(b4, 0, steps, 1, kw, grad=True)
    sub["c4_lti512_n64_grad"] = {
        "value": round(m["solved"] / (m["ms_per_step"] * 1e-3), 1), "unit": "QP solves/s (gated, +grad)",
        "ms_per_step": round(m["ms_per_step"], 4), "solved_fraction": m["solved"] / b4.batch,
        "iters_mean": round(m["iters_mean"], 1), "iters_capped": m["iters_capped"],
        "fp64_value": round(f["solved"] / (f["ms_per_step"] * 1e-3), 1), "fp64_ms_per_step": round(f["ms_per_step"], 4),
        "fp64_solved_fraction": f["solved"] / b4.batch, "steps": steps, "launch_shape": m["launch_shape"]}
    kw1 = dict(max_admm=200, k_check=0, adapt_rho=0)
    for B in (1, 64):
        b1 = double_integrator(B, N=20, seed=1)
        r = run_gpu(b1, 0, max(10, steps), 3, kw1, grad=False)
        sub[f"c1_double_integrator_b{B}"] = {
            "ms_per_step": round(r["ms_per_step"], 4), "solves_per_s": round(B / (r["ms_per_step"] * 1e-3), 1),
            "unit": "QP solves/s (200 fixed-rho FP64 iterations)", "solve_kernel_ms": round(
                r["kernels"]["solve"]["ms_per_step"], 4)}
    # the bicycle workloads (10 SQP x 50 ADMM iterations, fixed counts, FP32
    # iterations + the adjoint of the last QP), two timed steps each
    from workloads import bicycle_batch, bicycle_long_and_ragged

    lng, rag = bicycle_long_and_ragged(seed=5)
    kwb = dict(max_sqp=10, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1)
    for name, bb in (("c3_bicycle4096_n100", bicycle_batch(4096, N=100, seed=3)),
                     ("c5a_bicycle1_n8192", lng), ("c5b_bicycle256_ragged", rag)):
        r = run_bicycle(bb, 1, 2, 1, kwb, grad=True)
        sub[name] = {"value": round(bb.batch / (r["ms_per_step"] * 1e-3), 2),
                     "unit": "SQP solves/s (10 SQP x 50 ADMM iterations, + adjoint)",
                     "ms_per_step": round(r["ms_per_step"], 3), "kernel_ms_per_step": r["kernel_ms_per_step"],
                     "sqp_kkt_max": r["sqp_kkt_max"], "steps": 2}
    log(f"[bench] sub-results: {json.dumps(sub)}")
    return sub


if __name__ == "__main__":
    main()
