"""GPU parity of the implicit-differentiation adjoint (Algorithm 2) on the
differentiation workload (random LTI, nx=12, nu=4, N=64; learnable diag Q,
diag R, x0 and control bounds; loss ||u_0||^2 + ||x_N||^2).

* eta and the QP-data gradients match the oracle's dense active-set solve.
* Parameter gradients through the autograd layer match FP64 central finite
  differences of polished oracle solves (1e-3 relative) on the first 16
  instances of the differentiation batch, in FP64 and with FP32 ADMM
  iterations.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gpu_helpers import lti_solver, oracle_map, per_instance, rel  # noqa: E402
from oracle.adjoint import adjoint_dense, qp_vjp  # noqa: E402
from oracle.lti import fd_theta_grad, implicit_theta_grad, loss_and_grad_x, qp_of_theta, theta_of  # noqa: E402
from workloads import random_lti  # noqa: E402

FP64, MIXED = 0, 1


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def _loss_grad(solver, x, nx):
    """dL/dx for L = sum_b ||u_0||^2 + ||x_N||^2 on the stage-concatenated x."""
    g = torch.zeros_like(x)
    first = torch.as_tensor(solver.stage_off[:-1], device=x.device, dtype=torch.long)
    last = torch.as_tensor(solver.stage_off[1:] - 1, device=x.device, dtype=torch.long)
    g[first, nx:] = 2 * x[first, nx:]
    g[last, :nx] = 2 * x[last, :nx]
    return g


@pytest.mark.parametrize("seg", [None, 15], ids=["stagewise", "chunked"])
@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_adjoint_matches_oracle_dense_solve(precision, seg):
    """seg = 15: the solve and the adjoint factor N = 64 in chunks (segmented substitutions)."""
    b = random_lti(8, N=64, seed=4)
    s = lti_solver(b, precision)
    if seg is not None:
        s.set_segmented(seg)
    eps = 1e-9 if precision == FP64 else 1e-6
    out = s.solve(_settings(eps_abs=eps, eps_rel=eps, max_admm=5000))
    g = s.adjoint(_loss_grad(s, out["x"], b.nx), _settings(eps_active=1e-6))
    for i in range(b.batch):
        L, gtheta, sol = implicit_theta_grad(b, i)
        qp = qp_of_theta(b, i, theta_of(b, i))
        act = s.split(g["active"], i).cpu().numpy().reshape(-1)
        assert np.array_equal(act < 0, sol["lower"]) and np.array_equal(act > 0, sol["upper"])
        _, gx = loss_and_grad_x(qp, sol["x"])
        ex, ef, eg = adjoint_dense(qp, sol["x"], gx, sol["lower"], sol["upper"])
        tol = 1e-6 if precision == FP64 else 2e-3
        assert rel(s.split(g["eta_x"], i).cpu().numpy().reshape(-1), ex) < tol
        qg = qp_vjp(qp, sol["x"], ex, ef, eg, sol["lower"], sol["upper"])
        assert rel(g["d_x_init"][i].cpu().numpy(), qg["d_x_init"]) < tol
        assert rel(s.split(g["d_lo"], i).cpu().numpy(), qg["d_lo"]) < tol
        assert rel(s.split(g["d_hi"], i).cpu().numpy(), qg["d_hi"]) < tol
        assert rel(s.split(g["d_Ddiag"], i).cpu().numpy(), qg["d_Ddiag"]) < tol


_FD = {}


def _fd_reference(b):
    """FP64 central differences (h = 1e-6) of polished oracle solves, one
    instance per worker process; computed once for both precisions."""
    if "fd" not in _FD:
        _FD["fd"] = oracle_map(fd_theta_grad, [(b, i) for i in range(b.batch)])
    return _FD["fd"]


@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_parameter_gradients_match_central_fd(precision):
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.diff import lti_mpc
    from paper_2606_24039_amd.solver import OCPSolver

    b = random_lti(16, N=64, seed=4)  # the first 16 instances of the 512-instance differentiation batch
    nx, nu = b.nx, b.nu
    s = OCPSolver(nx, nu, b.ng, np.full(b.batch, b.N), model=A.MODEL_LTI, precision=precision)
    dev = dict(dtype=torch.float64, device="cuda")
    Qd = torch.tensor(b.Qd, **dev, requires_grad=True)
    Rd = torch.tensor(b.Rd, **dev, requires_grad=True)
    x0 = torch.tensor(b.x0, **dev, requires_grad=True)
    lo = torch.tensor(b.lo, **dev, requires_grad=True)
    hi = torch.tensor(b.hi, **dev, requires_grad=True)
    eps = 1e-9 if precision == FP64 else 1e-6
    st = _settings(eps_abs=eps, eps_rel=eps, max_admm=5000, eps_active=1e-6)
    x, status = lti_mpc(s, torch.tensor(b.A, **dev), torch.tensor(b.B, **dev), torch.tensor(b.G, **dev),
                        Qd, Rd, Qd, lo, hi, x0, settings=st)
    first = torch.as_tensor(s.stage_off[:-1], device="cuda", dtype=torch.long)
    last = torch.as_tensor(s.stage_off[1:] - 1, device="cuda", dtype=torch.long)
    loss = (x[first, nx:] ** 2).sum() + (x[last, :nx] ** 2).sum()
    loss.backward()
    fds = _fd_reference(b)
    for i in range(b.batch):
        fd = fds[i]
        got = np.concatenate([Qd.grad[i].cpu().numpy(), Rd.grad[i].cpu().numpy(), x0.grad[i].cpu().numpy(),
                              lo.grad[i, nx:].cpu().numpy(), hi.grad[i, nx:].cpu().numpy()])
        assert rel(got, fd) < 1e-3, (i, rel(got, fd))


def test_backward_after_the_handle_was_reused():
    """Two forwards through one solver, then both backwards: each backward
    differentiates its own forward's problem (the handle is restored and
    re-solved when another forward ran in between), matching a fresh solver
    per problem bit for bit."""
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.diff import lti_mpc
    from paper_2606_24039_amd.solver import OCPSolver

    b = random_lti(4, N=20, seed=4)
    nx = b.nx
    dev = dict(dtype=torch.float64, device="cuda")
    st = _settings(eps_abs=1e-9, eps_rel=1e-9, max_admm=5000, eps_active=1e-6)

    def run(solver, scale):
        x0 = torch.tensor(b.x0 * scale, **dev, requires_grad=True)
        x, _ = lti_mpc(solver, torch.tensor(b.A, **dev), torch.tensor(b.B, **dev), torch.tensor(b.G, **dev),
                       torch.tensor(b.Qd, **dev), torch.tensor(b.Rd, **dev), torch.tensor(b.Qfd, **dev),
                       torch.tensor(b.lo, **dev), torch.tensor(b.hi, **dev), x0, settings=st)
        return x0, x

    hz = np.full(b.batch, b.N)
    shared = OCPSolver(nx, b.nu, b.ng, hz, model=A.MODEL_LTI, precision=FP64)
    x0a, xa = run(shared, 1.0)
    x0b, xb = run(shared, 3.0)  # overwrites the handle's data and solution
    (xa ** 2).sum().backward()
    (xb ** 2).sum().backward()
    for scale, x0 in ((1.0, x0a), (3.0, x0b)):
        fresh = OCPSolver(nx, b.nu, b.ng, hz, model=A.MODEL_LTI, precision=FP64)
        x0r, xr = run(fresh, scale)
        (xr ** 2).sum().backward()
        assert torch.equal(x0.grad, x0r.grad), scale
        fresh.close()
    assert not torch.equal(x0a.grad, x0b.grad)
    shared.close()
