"""GPU parity of the multi-wavefront instances (ocp_set_multiwave): a long
horizon is solved by one workgroup of W wavefronts whose 16-lane rows each
take one chunk of the chunked factorisation and one segment of the segmented
substitutions (4 W of each), wavefront 0 keeping the schedule.  In exact
arithmetic this is the same ADMM iteration, so the FP64 iterates follow the
oracle's as closely as the one-wavefront shapes do.

* Linear MPC, stage width 16 (W = 4, 16 segments): fixed-rho FP64 iterates
  against the oracle for horizons from the smallest admissible one (63) up,
  with a short instance in the same batch on its own wavefront; rho
  adaptation with refactorisations inside the launch; FP32 iterations
  converging to the oracle's polished optimum with convergence checks.
* Kinematic bicycle, stage width 6 (W = 8, 32 segments): a fixed SQP x ADMM
  trajectory in FP64 against the oracle.
* The threshold's argument checks, and the default (horizons of 256 stages
  and more) on a batch where it applies.
* The adjoint on a workgroup (time-varying data): equal to the one-wavefront
  adjoint and to the oracle's dense KKT solve, with a slack loss.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_helpers import lti_solver, per_instance, rel  # noqa: E402
from oracle.adjoint import polish  # noqa: E402
from oracle.admm import ADMMSettings, admm_solve  # noqa: E402
from oracle.models import BicycleOCP  # noqa: E402
from oracle.qp import lti_batch_qp  # noqa: E402
from oracle.sqp import SQPSettings, sqp_solve  # noqa: E402
from workloads import bicycle_batch, random_lti  # noqa: E402

FP64, MIXED = 0, 1
# 63: the smallest multi-wavefront horizon at stage width 16 (16 segments of
# four stages); 64 .. 66: N + 1 = 1, 2, 3 mod 16; 203: uneven segments; 40:
# a short instance left on one wavefront
HORIZONS = np.array([63, 64, 65, 66, 203, 40])


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def _sub(b, i, N):
    bi = b.subset([i])
    bi.N = int(N)
    return bi


def test_multiwave_fixed_rho_iterates_fp64():
    b = random_lti(len(HORIZONS), N=int(HORIZONS.max()), seed=31)
    s = lti_solver(b, FP64, horizons=HORIZONS)
    s.set_multiwave(63)
    out = s.solve(_settings(max_admm=60, k_check=0, adapt_rho=0))
    for i, N in enumerate(HORIZONS):
        ref = admm_solve(lti_batch_qp(_sub(b, i, N), 0), ADMMSettings(max_iter=60, k_check=0, adapt_rho=False))
        got = per_instance(s, out, i)
        assert got["x"].size == (N + 1) * b.n
        for k in ("x", "z_g", "y_f", "y_g"):
            assert rel(got[k], getattr(ref, k)) < 1e-9, (int(N), k, rel(got[k], getattr(ref, k)))
    s.close()


def test_multiwave_rho_adaptation_and_refactorisation_fp64():
    hz = HORIZONS[[0, 3, 4]]
    b = random_lti(len(hz), N=int(hz.max()), seed=32)
    s = lti_solver(b, FP64, horizons=hz)
    s.set_multiwave(63)
    out = s.solve(_settings(max_admm=150, k_check=0, k_rho=25))
    for i, N in enumerate(hz):
        ref = admm_solve(lti_batch_qp(_sub(b, i, N), 0), ADMMSettings(max_iter=150, k_check=0, k_rho=25))
        got = per_instance(s, out, i)
        assert int(out["n_factor"][i]) == ref.n_factor, (int(N), int(out["n_factor"][i]), ref.n_factor)
        assert rel(got["x"], ref.x) < 1e-8, int(N)
    s.close()


def test_multiwave_mixed_precision_converges_with_checks():
    hz = HORIZONS
    b = random_lti(len(hz), N=int(hz.max()), seed=33)
    s = lti_solver(b, MIXED, horizons=hz)
    s.set_multiwave(63)
    # FP32 iterations end at the iteration cap at this tolerance (their noise
    # floor, as on one wavefront); the checks and rho changes still run
    out = s.solve(_settings(eps_abs=1e-6, eps_rel=1e-6, max_admm=6000))
    for i, N in enumerate(hz):
        qp = lti_batch_qp(_sub(b, i, N), 0)
        ref = admm_solve(qp, ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=80000))
        ok, exact = polish(qp, ref.x, ref.y_g, eps_solve=1e-8)
        assert ok
        got = per_instance(s, out, i)
        assert rel(got["x"], exact["x"]) < 1e-4, (int(N), rel(got["x"], exact["x"]))
    s.close()


def test_multiwave_bicycle_trajectory_fp64():
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    b = bicycle_batch(2, N=160, seed=3, first=40)
    s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=FP64)
    s.set_multiwave(127)
    s.set_bicycle(b)
    out = s.solve(_settings(max_sqp=6, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1))
    for i in range(b.batch):
        ref = sqp_solve(BicycleOCP(b, i), SQPSettings(max_sqp=6, fixed_iters=True),
                        admm=ADMMSettings(max_iter=50, k_check=0, k_rho=25))
        z = s.split(out["x"], i).cpu().numpy()
        assert rel(z, ref.z) < 1e-8, rel(z, ref.z)
    s.close()


def test_multiwave_threshold_checks_and_default():
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    s = OCPSolver(4, 2, 3, [300, 20], model=A.MODEL_BICYCLE, precision=MIXED)
    with pytest.raises(RuntimeError):
        s.set_multiwave(100)  # below 16 W - 1 = 127: segments of fewer than four stages
    s.set_multiwave(0)
    s.set_multiwave(127)
    s.close()
    # the default takes N >= 255: the same FP64 iterates as with it off
    b = bicycle_batch(1, N=260, seed=5)
    res = []
    for mw in (None, 0):
        s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=FP64)
        if mw is not None:
            s.set_multiwave(mw)
        s.set_bicycle(b)
        out = s.solve(_settings(max_sqp=2, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1))
        res.append(out["x"].cpu().numpy())
        s.close()
    assert rel(res[0], res[1]) < 1e-10, rel(res[0], res[1])


@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_multiwave_adjoint_matches_one_wavefront_and_oracle(precision):
    """The adjoint of a long time-varying instance on its workgroup
    (33-chunk FP64 factorisation, refinement chains on 32 segments) equals
    the one-wavefront adjoint (1e-9) and the oracle's dense KKT solve at the
    same active set (1e-6), with a loss on x and on the slacks; an instance
    starts off the track so that L1 rows carry slack."""
    from oracle.adjoint import adjoint_dense, qp_vjp
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver
    import torch

    b = bicycle_batch(2, N=300, seed=6)
    o = b.stage_off[1]
    b.x0[1, :2] = b.ref[o, :2] + 2.6 * b.normal[o]
    eps = 1e-10 if precision == FP64 else 1e-6
    st = _settings(max_sqp=1, fixed_sqp=1, eps_abs=eps, eps_rel=eps, max_admm=20000)
    res = {}
    for mw in (127, 0):
        s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=precision)
        s.set_multiwave(mw)
        s.set_bicycle(b)
        s.solve(st)
        dl = torch.as_tensor(np.random.default_rng(7).standard_normal((s.S, 6)), dtype=torch.float64, device="cuda")
        dxi = torch.as_tensor(np.random.default_rng(9).standard_normal((s.S, 3)), dtype=torch.float64, device="cuda")
        g = s.adjoint(dl, _settings(eps_active=1e-6), dL_dxi=dxi)
        out = s.get_solution()
        res[mw] = ({k: v.clone() for k, v in g.items()}, {k: v.clone() for k, v in out.items()}, s, dl, dxi)
    gm, om, sm, dl, dxi = res[127]
    g1, o1, s1, _, _ = res[0]
    assert (gm["adj_status"] == 0).all(), gm["adj_status"]
    if precision == FP64:
        assert rel(gm["eta_x"].cpu().numpy(), g1["eta_x"].cpu().numpy()) < 1e-9
        assert torch.equal(gm["active"], g1["active"])
    for i in range(b.batch):
        ocp = BicycleOCP(b, i)
        qp = ocp.convexify(ocp.initial_guess())
        act = sm.split(gm["active"], i).cpu().numpy().reshape(-1)
        r = admm_solve(qp, ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=200000))
        ok, sol = polish(qp, r.x, r.y_g, xi=r.xi, eps_solve=1e-8)
        assert ok
        dli = sm.split(dl, i).cpu().numpy().reshape(-1)
        dxii = sm.split(dxi, i).cpu().numpy().reshape(-1)
        ex, ef, eg = adjoint_dense(qp, sol["x"], dli, act < 0, act > 0, dL_dxi=dxii, xi=r.xi)
        assert rel(sm.split(gm["eta_x"], i).cpu().numpy().reshape(-1), ex) < 1e-6, i
        qg = qp_vjp(qp, sol["x"], ex, ef, eg, act < 0, act > 0, xi=r.xi, dL_dxi=dxii)
        flat = lambda a: np.asarray(a).reshape(-1)  # noqa: E731
        assert rel(flat(gm["d_x_init"][i].cpu().numpy()), flat(qg["d_x_init"])) < 1e-6, i
        for k in ("d_q", "d_lo", "d_hi", "eta_xi"):
            assert rel(flat(sm.split(gm[k], i).cpu().numpy()), flat(qg[k])) < 1e-6, (i, k)
        assert abs(float(gm["d_gamma1"][i]) - qg["d_gamma1"]) <= 1e-6 * max(1.0, abs(qg["d_gamma1"])), i
    sm.close()
    s1.close()
