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
