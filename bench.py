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

# HBM traffic of the persistent solve launch, per launch, from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE) of `bench.py --steps 1 --warmup 0
# --cpu-sample 0 --no-fp64`, each scaled by the same counter's reading for a
# plain 1 GiB device copy (`bench.py --copy-calibration 1024`: FETCH_SIZE
# reads 0.500 of the copied bytes, WRITE_SIZE 1.000).  Summary and commands:
# profiles/admm_solve_wave_lti1024_n50.md.  Keyed by (workload, precision);
# valid for the kernel as profiled -- set to None when the kernel changes.
TRAFFIC_BYTES = {("c2", "mixed"): (23642190.2 * 1.99994 + 2015575.9 * 1.0) * 1024}


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
    measured here (FP32 iterations, horizons up to 55 stages): the `blocks`
    n x n factor blocks (Linv_t, Linv_t', W_t, V_t) stream from memory once per
    iteration; the six padded 16-entry stage vectors stay in LDS for a
    segment of `k_seg` iterations, so five of them (x, y_f, z_g, y_g, xi) move
    in and out once per segment."""
    return blocks * n * n * ts + (2 * 5 * 16 * ts) / k_seg


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
    solve and (with grad) the dense-LU adjoint of the same instance."""
    import multiprocessing as mp

    global _CPU_BATCH
    _CPU_BATCH = batch
    cores = min(len(os.sched_getaffinity(0)), 16, sample)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores, initializer=_worker_init) as pool:
        res = pool.map(_oracle_one, [(i, settings_kw, grad) for i in range(sample)])
    wall = time.perf_counter() - t0
    solved = sum(1 for ok, _ in res if ok)
    iters = sum(it for _, it in res)
    return {"value": solved / wall, "unit": "QP solves/s", "cores": cores, "kind": "oracle",
            "sample": (f"first {sample} of {batch.batch} instances, FP64 NumPy/SciPy oracle, eps 1e-4"
                       + (", ADMM solve + sparse-LU adjoint" if grad else ", ADMM solve")),
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
        from oracle.adjoint import active_set, adjoint_dense, adjoint_refined, qp_vjp

        S = batch.N + 1
        dl = upstream_gradient(batch)[i * S:(i + 1) * S].reshape(-1)
        lower, upper = active_set(qp, r.x, r.y_g, r.xi)
        import warnings

        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            try:  # sparse LU of the KKT matrix (the definition)
                ex, ef, eg = adjoint_dense(qp, r.x, dl, lower, upper)
            except RuntimeError:
                ex = None
        if ex is None or not np.all(np.isfinite(ex)):
            # dependent active rows make K singular: the regularised
            # refinement (the GPU's scheme) is still defined
            ex, ef, eg = adjoint_refined(qp, r.x, dl, lower, upper, sigma_b=1e-9, rho_b=1e6, sweeps=6)
        qp_vjp(qp, r.x, ex, ef, eg, lower, upper)
    return r.status == 0, r.iters


def upstream_gradient(batch, seed=11):
    """Seeded dL/dx for the "+grad" leg: one fixed cotangent per stage
    variable, standard normal (the loss itself is the caller's)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((batch.batch * (batch.N + 1), batch.nx + batch.nu))


def run_gpu(batch, precision, steps, warmup, settings_kw, grad=True):
    import torch

    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    hz = np.full(batch.batch, batch.N)
    s = OCPSolver(batch.nx, batch.nu, batch.ng, hz, model=A.MODEL_LTI, precision=precision)
    s.set_lti(batch.A, batch.B, batch.Qd, batch.Rd, batch.Qfd, batch.G, batch.lo, batch.hi, batch.x0)
    st = A.default_settings(**settings_kw)
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
    solved = int((status == 0).sum())
    finite_grad = bool(torch.isfinite(grads["d_q"]).all().item()) if grad else None
    res = {"wall_s": wall, "ms_per_step": wall / steps * 1e3, "solved": solved, "batch": batch.batch,
           "iters_mean": float(iters.mean()), "iters_max": int(iters.max()), "iters_sum": int(iters.sum()),
           "nfact_sum": int(nfact.sum()),
           "status_counts": {int(k): int(v) for k, v in zip(*np.unique(status, return_counts=True))},
           "kernels": {k: {"ms_per_step": ms / steps, "launches_per_step": c / steps} for k, (ms, c) in kt.items()},
           "grad_finite": finite_grad}
    s.close()
    return res


def run_bicycle(batch, precision, steps, warmup, settings_kw, grad=True):
    """Timed SQP solves (+ the adjoint of the last QP) of a kinematic-bicycle batch."""
    import torch

    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    s = OCPSolver(4, 2, 3, batch.horizons, model=A.MODEL_BICYCLE, precision=precision)
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
           "grad_finite": bool(torch.isfinite(grads["eta_x"]).all().item()) if grad else None}
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
    mixed = run_bicycle(batch, 1, steps, warmup, kw, grad=not args.no_grad)
    out = {"metric": "SQP solves/s (10 SQP x 50 ADMM iterations, fixed counts), FP32 ADMM iterations + FP64 "
                     "factorisation" + ("" if args.no_grad else ", + adjoint of the last QP"),
           "value": round(batch.batch / (mixed["ms_per_step"] * 1e-3), 4), "unit": "SQP solves/s", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": round(mixed["ms_per_step"], 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": desc, "batch": int(batch.batch), "stages": int(np.sum(batch.horizons + 1)),
                      "nx": 4, "nu": 2, "ng": 3, "grad": not args.no_grad,
                      "parallelism": "single GPU, one wavefront per instance"},
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
    ap.add_argument("--cpu-sample", type=int, default=256, help="instances timed on the oracle (0 = skip)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain-FP64 comparison")
    ap.add_argument("--no-grad", action="store_true", help="forward solves only (no adjoint in the step)")
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
    settings_kw = dict(eps_abs=1e-4, eps_rel=1e-4, max_admm=1000, k_check=25, k_rho=25)
    f_it, f_fac = lti_flops_per_stage(batch.nx, batch.nu, batch.ng)
    stages = batch.N + 1

    log(f"[bench] workload: {desc}")
    mixed = run_gpu(batch, 1, args.steps, args.warmup, settings_kw, grad=not args.no_grad)
    log(f"[bench] mixed: {json.dumps(mixed)}")
    fp64 = None
    if not args.no_fp64:
        fp64 = run_gpu(batch, 0, max(3, args.steps // 4), 1, settings_kw, grad=not args.no_grad)
        log(f"[bench] fp64: {json.dumps(fp64)}")

    value = mixed["solved"] / (mixed["ms_per_step"] * 1e-3)
    # roofline of the dominant kernel (the persistent ADMM solve).  It streams
    # the factor blocks of every running instance once per iteration (the
    # stage vectors stay in LDS between boundary checks) and is bound by
    # memory traffic while the batch is full (the FP32 factor copies of 1024
    # instances, 213 MB, exceed the L2), so the bound is HBM: achieved
    # = algorithmic bytes of all its launches in a step / its GPU time in a
    # step (= average bytes per launch / average launch duration).
    kit = mixed["kernels"]["solve"]
    n = batch.nx + batch.nu
    b_it = lti_bytes_per_stage(n, 4, 4, min(k for k in (settings_kw.get("k_check", 25), settings_kw.get("k_rho", 25)) if k > 0))
    bytes_launch = mixed["iters_sum"] * stages * b_it / max(kit["launches_per_step"], 1)
    t_launch = kit["ms_per_step"] * 1e-3 / max(kit["launches_per_step"], 1)
    achieved = bytes_launch / t_launch / 1e9
    F32 = mixed["iters_sum"] * stages * f_it
    F64 = mixed["nfact_sum"] * stages * f_fac
    traffic = TRAFFIC_BYTES.get((args.workload, "mixed"))
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM, 5), "traffic": traffic,
            "kernel": f"admm_solve_wave_kernel<float,{batch.nx},{batch.nu},{batch.ng},box>",
            "avg_launch_us": round(t_launch * 1e6, 2), "launches_per_step": kit["launches_per_step"],
            "bytes_per_launch": bytes_launch, "bytes_per_stage_iteration": b_it,
            "alu_tflops": round((F32 + F64 * PEAK_FP32 / PEAK_FP64) / (t_launch * kit["launches_per_step"]) / 1e12,
                                4),
            "alu_frac_fp32_peak": round((F32 + F64 * PEAK_FP32 / PEAK_FP64) / (t_launch * kit["launches_per_step"])
                                        / 1e12 / PEAK_FP32, 6)}
    out = {
        "metric": "QP solves/s at 1e-4 KKT residual, FP32+grad vs plain FP64, 1 MI355X",
        "value": round(value, 2), "unit": "QP solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mixed["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": desc, "batch": batch.batch, "horizon": batch.N, "nx": batch.nx, "nu": batch.nu,
                   "ng": batch.ng, "precision": "fp32 ADMM iterations, fp64 factorisation, gate and adjoint",
                   "eps": 1e-4, "max_admm": 1000, "grad": not args.no_grad,
                   "parallelism": "single GPU, one instance per 16-lane row"},
        "admm_iters_per_s": round(mixed["iters_sum"] / (mixed["ms_per_step"] * 1e-3), 1),
        "kernel_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in mixed["kernels"].items()},
        "solved_fraction": mixed["solved"] / batch.batch,
        "roofline": roof,
    }
    if fp64 is not None:
        out["fp64"] = {"value": round(fp64["solved"] / (fp64["ms_per_step"] * 1e-3), 2),
                       "ms_per_step": round(fp64["ms_per_step"], 4),
                       "kernel_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in fp64["kernels"].items()},
                       "solved_fraction": fp64["solved"] / batch.batch, "iters_mean": fp64["iters_mean"]}
        out["speedup_vs_fp64"] = round(value / max(out["fp64"]["value"], 1e-9), 3)
    if args.cpu_sample > 0:
        cb_kw = dict(eps_abs=1e-4, eps_rel=1e-4, max_iter=1000, k_check=25, k_rho=25)
        out["cpu_baseline"] = cpu_baseline(batch, min(args.cpu_sample, batch.batch), cb_kw, not args.no_grad)
        log(f"[bench] cpu: {json.dumps(out['cpu_baseline'])}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
