"""Graph capture of a whole step (solve + adjoint) and its replay.

The solve is deterministic (fixed-order arithmetic, cold start), so every
replay must reproduce the eager step bit for bit; the replays are separated by
eager work on the same handle and by host synchronisations."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_helpers import lti_solver  # noqa: E402
from workloads import random_lti  # noqa: E402

MIXED, FP64 = 1, 0
KEYS = ("x", "z_g", "y_f", "y_g", "xi", "status", "admm_iters", "n_factor", "rho", "r_prim", "r_dual")
GKEYS = ("d_q", "d_Ddiag", "d_x_init", "d_lo", "d_hi", "eta_x", "active")


def _snapshot(d, keys):
    return {k: d[k].detach().cpu().numpy().copy() for k in keys}


@pytest.mark.parametrize("precision", [MIXED, FP64])
def test_captured_step_replays_match_the_eager_step(precision):
    import torch

    from paper_2606_24039_amd import default_settings

    b = random_lti(16, N=30, seed=2)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = lti_solver(b, precision)
        st = default_settings(eps_abs=1e-4, eps_rel=1e-4, max_admm=400)
        rng = np.random.default_rng(7)
        dl = torch.as_tensor(rng.standard_normal((s.S, s.n)), dtype=torch.float64, device="cuda")
        # eager reference
        ref_out = s.solve(st)
        ref_g = s.adjoint(dl, st)
        ref = _snapshot(ref_out, KEYS)
        refg = _snapshot(ref_g, GKEYS)
        # capture into buffers that stay alive for the replays
        out = s.alloc_solution()
        grads = s.alloc_grads()
        s.graph_capture(st, out, dl, grads)
        for rep in range(3):
            for v in out.values():
                v.fill_(-7)
            for v in grads.values():
                v.fill_(-7)
            s.graph_launch()
            stream.synchronize()
            got = _snapshot(out, KEYS)
            gotg = _snapshot(grads, GKEYS)
            for k in KEYS:
                assert np.array_equal(got[k], ref[k]), (rep, k)
            for k in GKEYS:
                assert np.array_equal(gotg[k], refg[k]), (rep, k)
            # eager work on the same handle between replays
            s.solve(default_settings(eps_abs=1e-3, eps_rel=1e-3, max_admm=50))
            stream.synchronize()
        s.close()


@pytest.mark.parametrize("precision", [MIXED, FP64])
def test_captured_bicycle_sqp_step(precision):
    """A kinematic-bicycle step (3 SQP iterations of linearisation, ADMM and
    line search, then the adjoint of the last QP) captured once: every replay
    equals the eager step bit for bit, and in FP64 the trajectory equals the
    oracle's SQP run (1e-8)."""
    import torch

    from oracle.admm import ADMMSettings
    from oracle.models import BicycleOCP
    from oracle.sqp import SQPSettings, sqp_solve
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd import default_settings
    from paper_2606_24039_amd.solver import OCPSolver
    from workloads import bicycle_batch

    b = bicycle_batch(6, N=40, seed=3)
    stream = torch.cuda.Stream()
    keys = ("x", "xi", "y_f", "y_g", "sqp_kkt", "sqp_iters", "status")
    gkeys = ("d_q", "d_Ddiag", "d_x_init", "eta_x", "eta_f", "active", "adj_status")
    with torch.cuda.stream(stream):
        s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=precision)
        s.set_bicycle(b)
        st = default_settings(max_sqp=3, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1)
        dl = torch.as_tensor(np.random.default_rng(5).standard_normal((s.S, 6)), dtype=torch.float64, device="cuda")
        ref = _snapshot(s.solve(st), keys)
        refg = _snapshot(s.adjoint(dl, st), gkeys)
        out = s.alloc_solution()
        grads = s.alloc_grads()
        s.graph_capture(st, out, dl, grads)
        for rep in range(3):
            for v in list(out.values()) + list(grads.values()):
                v.fill_(-7)
            s.graph_launch()
            stream.synchronize()
            got, gotg = _snapshot(out, keys), _snapshot(grads, gkeys)
            for k in keys:
                assert np.array_equal(got[k], ref[k]), (rep, k)
            for k in gkeys:
                assert np.array_equal(gotg[k], refg[k]), (rep, k)
            s.solve(default_settings(max_sqp=1, max_admm=20, k_check=0, fixed_sqp=1))  # eager work between replays
            stream.synchronize()
        if precision == FP64:
            for i in range(b.batch):
                r = sqp_solve(BicycleOCP(b, i), SQPSettings(max_sqp=3, fixed_iters=True),
                              admm=ADMMSettings(max_iter=50, k_check=0, k_rho=25))
                z = s.split(torch.as_tensor(got["x"]), i).numpy()
                assert np.max(np.abs(z - r.z)) / max(np.max(np.abs(r.z)), 1.0) < 1e-8, i
        s.close()


@pytest.mark.parametrize("precision", [MIXED, FP64])
def test_captured_bicycle_step_with_long_horizons(precision):
    """A bicycle step over horizons 1172, 244, 74 and 1042: the two long ones
    on multi-wavefront workgroups beside the one-wavefront launch (two
    streams), and the line search spread over 512-stage chunks (merit parts,
    decision, step, stopping maxima, combination).  Every replay equals the
    eager step bit for bit."""
    import torch

    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd import default_settings
    from paper_2606_24039_amd.solver import OCPSolver
    from workloads import bicycle_long_and_ragged

    _, b = bicycle_long_and_ragged(seed=13, long_N=16, ragged=4, n_lo=32, n_hi=1200)
    assert list(b.horizons) == [1172, 244, 74, 1042]
    stream = torch.cuda.Stream()
    keys = ("x", "xi", "y_f", "y_g", "sqp_kkt", "sqp_iters", "status", "rho")
    gkeys = ("d_q", "d_Ddiag", "d_x_init", "eta_x", "adj_status")
    with torch.cuda.stream(stream):
        s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=precision)
        s.set_bicycle(b)
        st = default_settings(max_sqp=2, max_admm=30, k_check=0, k_rho=25, fixed_sqp=1)
        dl = torch.as_tensor(np.random.default_rng(7).standard_normal((s.S, 6)), dtype=torch.float64, device="cuda")
        ref = _snapshot(s.solve(st), keys)
        refg = _snapshot(s.adjoint(dl, st), gkeys)
        out = s.alloc_solution()
        grads = s.alloc_grads()
        s.graph_capture(st, out, dl, grads)
        for rep in range(3):
            for v in list(out.values()) + list(grads.values()):
                v.fill_(-7)
            s.graph_launch()
            stream.synchronize()
            got, gotg = _snapshot(out, keys), _snapshot(grads, gkeys)
            for k in keys:
                assert np.array_equal(got[k], ref[k]), (rep, k)
            for k in gkeys:
                assert np.array_equal(gotg[k], refg[k]), (rep, k)
            s.solve(default_settings(max_sqp=1, max_admm=10, k_check=0, fixed_sqp=1))  # eager work between replays
            stream.synchronize()
        s.close()


def test_captured_rescaled_lti_step():
    """The same for a rescaled random-LTI step (box normalisation): the graph
    keeps the rescaled data and the unscaling of the outputs."""
    import torch

    from paper_2606_24039_amd import default_settings

    b = random_lti(16, N=30, seed=2)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = lti_solver(b, MIXED)
        s.set_scaling_box(0.6)
        s.set_lti(b.A, b.B, b.Qd, b.Rd, b.Qfd, b.G, b.lo, b.hi, b.x0)
        st = default_settings(eps_abs=1e-4, eps_rel=1e-4, max_admm=400)
        dl = torch.as_tensor(np.random.default_rng(7).standard_normal((s.S, s.n)), dtype=torch.float64, device="cuda")
        ref = _snapshot(s.solve(st), KEYS)
        refg = _snapshot(s.adjoint(dl, st), GKEYS)
        out = s.alloc_solution()
        grads = s.alloc_grads()
        s.graph_capture(st, out, dl, grads)
        for rep in range(2):
            for v in list(out.values()) + list(grads.values()):
                v.fill_(-7)
            s.graph_launch()
            stream.synchronize()
            got, gotg = _snapshot(out, KEYS), _snapshot(grads, GKEYS)
            for k in KEYS:
                assert np.array_equal(got[k], ref[k]), (rep, k)
            for k in GKEYS:
                assert np.array_equal(gotg[k], refg[k]), (rep, k)
        s.close()


@pytest.mark.parametrize("precision", [MIXED, FP64])
def test_captured_mixed_batch_with_a_workgroup_instance(precision):
    """A batch with one instance above the multi-wavefront threshold and
    short ones: the workgroup launch runs on a second stream forked from and
    joined back into the capturing stream.  Every replay equals the eager
    step bit for bit, and the eager FP64 trajectory equals the oracle's."""
    import torch

    from oracle.admm import ADMMSettings
    from oracle.models import BicycleOCP
    from oracle.sqp import SQPSettings, sqp_solve
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd import default_settings
    from paper_2606_24039_amd.solver import OCPSolver
    from workloads import bicycle_batch

    long_ = bicycle_batch(1, N=300, seed=3)
    short = bicycle_batch(3, N=30, seed=4)
    b = bicycle_batch(4, N=300, seed=3)
    b.horizons = np.array([300, 30, 30, 30])
    b.stage_off = np.concatenate([[0], np.cumsum(b.horizons + 1)]).astype(np.int64)
    b.ref = np.concatenate([long_.ref, short.ref])
    b.normal = np.concatenate([long_.normal, short.normal])
    b.x0 = np.concatenate([long_.x0, short.x0])
    stream = torch.cuda.Stream()
    keys = ("x", "xi", "y_f", "y_g", "sqp_kkt", "status")
    with torch.cuda.stream(stream):
        s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=precision)
        s.set_bicycle(b)
        st = default_settings(max_sqp=2, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1)
        ref = _snapshot(s.solve(st), keys)
        out = s.alloc_solution()
        s.graph_capture(st, out)
        for rep in range(3):
            for v in out.values():
                v.fill_(-7)
            s.graph_launch()
            stream.synchronize()
            got = _snapshot(out, keys)
            for k in keys:
                assert np.array_equal(got[k], ref[k]), (rep, k)
            s.solve(default_settings(max_sqp=1, max_admm=20, k_check=0, fixed_sqp=1))
            stream.synchronize()
    if precision == FP64:
        for i in (0, 1):
            r = sqp_solve(BicycleOCP(b, i), SQPSettings(max_sqp=2, fixed_iters=True),
                          admm=ADMMSettings(max_iter=50, k_check=0, k_rho=25))
            z = ref["x"][b.stage_off[i]:b.stage_off[i + 1]]
            assert np.max(np.abs(z - r.z)) <= 1e-8 * max(1.0, np.max(np.abs(r.z))), i
    s.close()
