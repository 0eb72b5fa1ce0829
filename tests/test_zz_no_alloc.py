"""ocp_solve_noalloc (the entry point that allocates nothing) against the
handle path ocp_create + ocp_set_* + ocp_solve on the same data: two calls in
a row on the random LTI workload, the second with a smaller batch and shorter
horizon, then a kinematic-bicycle SQP solve; every output bit for bit (the
same kernels run on the same data, only the workspace differs).  A problem
larger than the scratch is rejected before any GPU work."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gpu_helpers import lti_solver  # noqa: E402
from workloads import bicycle_batch, random_lti  # noqa: E402

KEYS = ("x", "xi", "z_g", "y_f", "y_g", "status", "admm_iters", "sqp_iters", "n_factor", "r_prim", "r_dual", "rho",
        "sqp_kkt")


def _noalloc(solver, problem):
    """Run ocp_solve_noalloc with the dims and horizons of `solver` and return its outputs."""
    from paper_2606_24039_amd import _abi as A

    out = solver.alloc_solution()
    for v in out.values():
        v.fill_(-7)  # every output must be written by the call
    sol = solver.solution_struct(out)
    st = A.default_settings(max_admm=400, k_check=25, eps_abs=1e-4, eps_rel=1e-4, max_sqp=3)
    hz = np.ascontiguousarray(solver.horizons, dtype=np.int32)
    code = solver.lib.ocp_solve_noalloc(C.byref(solver.dims), hz.ctypes.data_as(A._ip), C.byref(problem),
                                        C.byref(st), C.byref(sol), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    A.check(code, "ocp_solve_noalloc")
    torch.cuda.current_stream().synchronize()
    return out, st


def _lti_case(B, N, precision):
    from paper_2606_24039_amd import _abi as A

    b = random_lti(B, N=N, seed=2)
    s = lti_solver(b, precision)
    keep = [torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64, device="cuda")
            for v in (b.A, b.B, b.Qd, b.Rd, b.Qfd, b.G, b.lo, b.hi, b.x0)]
    prob = A.ocp_lti(*[t.data_ptr() for t in keep])
    got, st = _noalloc(s, prob)
    ref = s.solve(st)
    return s, got, ref


def _same(got, ref, keys=KEYS):
    for k in keys:
        assert torch.equal(got[k], ref[k]), k


@pytest.mark.parametrize("precision", [1, 0], ids=["mixed", "fp64"])
def test_noalloc_matches_the_handle_path_twice_then_smaller(precision):
    s1, got1, ref1 = _lti_case(48, 50, precision)
    s2, got2, ref2 = _lti_case(16, 30, precision)  # second call: fewer instances, shorter horizon
    lti_keys = tuple(k for k in KEYS if k != "sqp_kkt")  # written for the bicycle model only
    _same(got1, ref1, lti_keys)
    _same(got2, ref2, lti_keys)
    assert int((ref1["status"] == 0).sum()) > 0
    s1.close()
    s2.close()


def test_noalloc_bicycle_sqp_matches_the_handle_path():
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    b = bicycle_batch(8, N=40, seed=3)
    s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=1)
    s.set_bicycle(b)
    keep = [torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64, device="cuda") for v in (b.ref, b.normal, b.x0)]
    prob = A.ocp_bicycle(keep[0].data_ptr(), keep[1].data_ptr(), keep[2].data_ptr(), b.dt, b.wheelbase, b.a_bound,
                         b.steer_bound, b.lat_bound, b.gamma_l1, (C.c_double * 4)(*b.Qd), (C.c_double * 2)(*b.Rd),
                         (C.c_double * 4)(*b.Qfd), int(getattr(b, "integrator", 0)))
    got, st = _noalloc(s, prob)
    ref = s.solve(st)
    _same(got, ref)
    s.close()


def test_noalloc_rejects_a_problem_larger_than_the_scratch():
    from paper_2606_24039_amd import _abi as A

    b = random_lti(1024, N=50, seed=2)
    s = lti_solver(b, 1)
    assert s.workspace_bytes() > A.NOALLOC_SCRATCH_BYTES
    hz = np.full(1024, 50, dtype=np.int32)
    prob = A.ocp_lti()
    st = A.default_settings()
    sol = A.ocp_solution()
    code = s.lib.ocp_solve_noalloc(C.byref(s.dims), hz.ctypes.data_as(A._ip), C.byref(prob), C.byref(st),
                                   C.byref(sol), None)
    assert code == A.OCP_E_SCRATCH
    s.close()
