"""Helpers shared by the GPU parity tests: run the HIP path on a workload and
split its stage-concatenated outputs per instance."""
import numpy as np


def rel(a, b):
    """Relative error of the build's convention: ||a - b||_inf / max(||b||_inf, 1)."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))) if b.size else 0.0, 1.0))


def lti_solver(batch, precision, horizons=None):
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    hz = np.full(batch.batch, batch.N) if horizons is None else np.asarray(horizons)
    s = OCPSolver(batch.nx, batch.nu, batch.ng, hz, model=A.MODEL_LTI, precision=precision)
    s.set_lti(batch.A, batch.B, batch.Qd, batch.Rd, batch.Qfd, batch.G, batch.lo, batch.hi, batch.x0)
    return s


def per_instance(solver, out, i):
    """(x [(N+1)*n], z_g, xi, y_f, y_g) of instance i as flat numpy arrays in the oracle's ordering."""
    g = lambda k: solver.split(out[k], i).detach().cpu().numpy().reshape(-1)
    return {"x": g("x"), "z_g": g("z_g"), "xi": g("xi"), "y_f": g("y_f"), "y_g": g("y_g")}


def oracle_map(fn, arglist):
    """Run an oracle function over a list of argument tuples in fresh worker
    processes (spawned: they never touch the GPU), one BLAS thread each."""
    import multiprocessing as mp
    import os

    os.environ.setdefault("OMP_NUM_THREADS", "1")
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    workers = max(1, min(16, len(os.sched_getaffinity(0)), len(arglist)))
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.starmap(fn, arglist)
