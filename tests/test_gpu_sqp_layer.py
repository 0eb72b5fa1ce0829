"""GPU checks of the differentiable SQP layer (paper_2606_24039_amd.diff.bicycle_mpc).

The backward restores the forward's final SQP iterate and differentiates the
KKT conditions of the OCP there with the exact Hessian of the Lagrangian
(ocp_adjoint, OCP_ADJ_SQP_EXACT).

* Parity: the parameter gradients (x0, ref, the weight diagonals) equal the
  oracle's implicit derivative of the SQP solution evaluated at the GPU's
  iterate (oracle.sqp_adjoint.sqp_param_grads, dense KKT solve), 1e-6, for
  the FP64 and the FP32-iteration solver, both integrators.  One instance
  starts off the track so that lateral rows carry nonzero L1 slack.
* Gauss-Newton mode (OCP_ADJ_SQP_GN): eta_x equals the oracle's with the
  dynamics curvature dropped.
* Central differences of tightly converged GPU SQP solves (FP64) agree with
  the layer's gradients to 1e-4.
* Checkpoint: a backward run after the handle has solved another problem
  gives bit for bit the gradients of a backward run straight after its
  forward.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from oracle.models import BicycleOCP  # noqa: E402
from oracle.sqp_adjoint import sqp_param_grads  # noqa: E402
from workloads import bicycle_batch  # noqa: E402

FP64, MIXED = 0, 1
TIGHT = dict(max_sqp=30, fixed_sqp=1, eps_abs=1e-11, eps_rel=1e-11, max_admm=40000, k_check=25, eps_active=1e-6)


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def _batch(integrator=0):
    b = bicycle_batch(3, N=12, seed=3)
    b.integrator = integrator
    o = b.stage_off[1]
    b.x0[1, :2] = b.ref[o, :2] + 2.6 * b.normal[o]
    return b


def _params(b, requires_grad=True):
    f = lambda a: torch.tensor(np.asarray(a, float), dtype=torch.float64, device="cuda",  # noqa: E731
                               requires_grad=requires_grad)
    return f(b.x0), f(b.ref), f(b.Qd), f(b.Rd), f(b.Qfd)


def _solver(b, precision):
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    return OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=precision)


def _loss_weights(S):
    return torch.as_tensor(np.random.default_rng(5).standard_normal((S, 6)), dtype=torch.float64, device="cuda")


def _forward_backward(s, b, settings, c, params=None):
    from paper_2606_24039_amd.diff import bicycle_mpc

    p = params if params is not None else _params(b)
    x, status = bicycle_mpc(s, b, *p, settings=settings)
    (c * x).sum().backward()
    return x.detach(), status, [t.grad.clone() for t in p]


@pytest.mark.parametrize("integrator", [0, 1], ids=["midpoint", "trapezoid"])
@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "fp32_iterations"])
def test_layer_gradients_match_oracle_at_the_iterate(precision, integrator):
    b = _batch(integrator)
    s = _solver(b, precision)
    tight = dict(TIGHT)
    if precision == MIXED:
        tight.update(eps_abs=1e-6, eps_rel=1e-6)
    st = _settings(**tight)
    c = _loss_weights(s.S)
    x, status, (gx0, gref, gQ, gR, gQf) = _forward_backward(s, b, st, c)
    out = s.get_solution()  # the restored checkpoint: the forward's final iterate
    assert torch.equal(out["x"], x)
    xi, yf, yg = out["xi"], out["y_f"], out["y_g"]
    want = {"Qd": np.zeros(4), "Rd": np.zeros(2), "Qfd": np.zeros(4)}
    for i in range(b.batch):
        ocp = BicycleOCP(b, i)
        z = s.split(x, i).cpu().numpy()
        r = sqp_param_grads(ocp, z, s.split(xi, i).cpu().numpy().reshape(-1),
                            s.split(yf, i).cpu().numpy().reshape(-1), s.split(yg, i).cpu().numpy().reshape(-1),
                            s.split(c, i).cpu().numpy(), exact=True, eps_active=1e-6)
        if i == 1:
            assert np.count_nonzero(s.split(xi, i).cpu().numpy()) > 0
        np.testing.assert_allclose(gx0[i].cpu().numpy(), r["x0"], rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(s.split(gref, i).cpu().numpy(), r["ref"], rtol=1e-6, atol=1e-6)
        for k in want:
            want[k] += r[k]
    np.testing.assert_allclose(gQ.cpu().numpy(), want["Qd"], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(gR.cpu().numpy(), want["Rd"], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(gQf.cpu().numpy(), want["Qfd"], rtol=1e-6, atol=1e-6)


def test_gauss_newton_mode_matches_oracle():
    from paper_2606_24039_amd import _abi as A

    b = _batch()
    s = _solver(b, FP64)
    s.set_bicycle(b)
    out = s.solve(_settings(**TIGHT))
    c = _loss_weights(s.S)
    res = {}
    for mode in (A.ADJ_SQP_GN, A.ADJ_SQP_EXACT):
        st = _settings(**TIGHT)
        st.adj_mode = mode
        res[mode] = s.adjoint(c, st)
    for i in range(b.batch):
        ocp = BicycleOCP(b, i)
        args = [s.split(out[k], i).cpu().numpy().reshape(-1) for k in ("x", "xi", "y_f", "y_g")]
        for mode, exact in ((A.ADJ_SQP_GN, False), (A.ADJ_SQP_EXACT, True)):
            r = sqp_param_grads(ocp, *args, s.split(c, i).cpu().numpy(), exact=exact, eps_active=1e-6)
            ex = s.split(res[mode]["eta_x"], i).cpu().numpy().reshape(-1)
            np.testing.assert_allclose(ex, r["eta_x"], rtol=1e-6, atol=1e-6 * max(1.0, np.abs(r["eta_x"]).max()))
    # the dynamics curvature is visible at this iterate
    assert float((res[A.ADJ_SQP_GN]["eta_x"] - res[A.ADJ_SQP_EXACT]["eta_x"]).abs().max()) > 1e-6


def test_layer_gradients_match_central_differences():
    """The loss weighs only instances whose SQP reaches stationarity 1e-9: the
    Armijo search on the L1 merit takes short steps near the solution, so
    some instances stop at 1e-8 to 1e-6, too coarse for differences at
    h = 1e-5.  (Instances with nonzero L1 slack are covered by the parity
    test above.)"""
    from paper_2606_24039_amd.diff import bicycle_mpc

    b = bicycle_batch(4, N=12, seed=4)
    s = _solver(b, FP64)
    st = _settings(**TIGHT)
    s.set_bicycle(b)
    out = s.solve(st)
    conv = (out["sqp_kkt"][:, 0] < 1e-9) & (out["status"] == 0)
    assert int(conv.sum()) >= 2, out["sqp_kkt"]
    inst = torch.repeat_interleave(torch.arange(s.B, device="cuda"),
                                   torch.as_tensor(s.horizons + 1, device="cuda", dtype=torch.long))
    c = _loss_weights(s.S) * conv[inst].to(torch.float64)[:, None]
    x, status, g = _forward_backward(s, b, st, c)
    h = 1e-5

    def loss(idx, k, delta):
        p = list(_params(b, requires_grad=False))
        p[idx] = p[idx].clone()
        p[idx].view(-1)[k] += delta
        with torch.no_grad():
            xx, _ = bicycle_mpc(s, b, *p, settings=st)
        return float((c * xx).sum())

    checks = [(0, 0), (0, 4 * 1 + 3), (1, 4 * 5 + 1), (1, 4 * (int(b.stage_off[2]) + 3) + 0), (2, 1), (2, 2),
              (3, 1), (4, 0)]
    for idx, k in checks:
        fd = (loss(idx, k, h) - loss(idx, k, -h)) / (2 * h)
        want = float(g[idx].reshape(-1)[k])
        assert abs(fd - want) <= 1e-4 * max(1.0, abs(fd)), (idx, k, fd, want)


def test_checkpoint_restore_after_handle_reuse():
    b = _batch()
    b2 = bicycle_batch(3, N=12, seed=11)
    st = _settings(**TIGHT)
    s = _solver(b, FP64)
    c = _loss_weights(s.S)
    _, _, g_direct = _forward_backward(s, b, st, c)

    from paper_2606_24039_amd.diff import bicycle_mpc

    p = _params(b)
    x, _ = bicycle_mpc(s, b, *p, settings=st)
    s.set_bicycle(b2)  # the handle solves another problem before the backward
    s.solve(st)
    (c * x).sum().backward()
    for a, want in zip(p, g_direct):
        assert torch.equal(a.grad, want)
