"""Torch-facing wrapper of the C ABI: device memory and streams come from
PyTorch, every step of the solve runs in the HIP library."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi as A


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, dtype=torch.float64, device="cuda"):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device)


class OCPSolver:
    """A batch of optimal-control QPs / OCPs with fixed shapes and horizons."""

    def __init__(self, nx, nu, ng, horizons, model=A.MODEL_LTI, precision=A.PREC_FP64, time_invariant=False,
                 device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("OCPSolver needs a HIP device (no CPU fallback)")
        self.lib = A.lib()
        hz = np.ascontiguousarray(np.asarray(horizons, dtype=np.int32))
        self.horizons = hz
        self.B = len(hz)
        self.nx, self.nu, self.ng, self.n = nx, nu, ng, nx + nu
        self.model, self.precision = model, precision
        self.S = int(np.sum(hz + 1))
        self.stage_off = np.concatenate([[0], np.cumsum(hz + 1)]).astype(np.int64)
        self.device = device
        self.dims = A.ocp_dims(self.B, nx, nu, ng, model, precision, int(time_invariant))
        h = C.c_void_p()
        A.check(self.lib.ocp_create(C.byref(self.dims), hz.ctypes.data_as(A._ip), C.byref(h)), "ocp_create")
        self.h = h
        self._keep = []
        self.generation = 0  # bumped by every call that changes the handle's problem data or solution

    def workspace_bytes(self) -> int:
        out = C.c_size_t()
        A.check(self.lib.ocp_workspace_bytes(C.byref(self.dims), self.horizons.ctypes.data_as(A._ip), C.byref(out)),
                "ocp_workspace_bytes")
        return out.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.ocp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ setters
    def set_lti(self, A_, Bm, Qd, Rd, Qfd, G, lo, hi, x0):
        self.generation += 1
        t = [_dev(v) for v in (A_, Bm, Qd, Rd, Qfd, G, lo, hi, x0)]
        p = A.ocp_lti(*[tt.data_ptr() for tt in t])
        A.check(self.lib.ocp_set_lti(self.h, C.byref(p), _stream()), "ocp_set_lti")
        self._keep = t
        torch.cuda.current_stream().synchronize()

    def set_qp(self, D, Am, Ap, x_init, G, lo, hi, E=None, q=None, b=None, soft=None, gamma2=1.0, gamma1=1.0):
        self.generation += 1
        t = {k: (_dev(v) if v is not None else None) for k, v in dict(D=D, E=E, q=q, Am=Am, Ap=Ap, b=b, G=G, lo=lo,
                                                                         hi=hi, x_init=x_init).items()}
        st = _dev(soft, dtype=torch.uint8) if soft is not None else None
        p = A.ocp_qp(*[(t[k].data_ptr() if t[k] is not None else None) for k in
                       ("D", "E", "q", "Am", "Ap", "b", "G", "lo", "hi", "x_init")],
                     st.data_ptr() if st is not None else None, float(gamma2), float(gamma1))
        A.check(self.lib.ocp_set_qp(self.h, C.byref(p), _stream()), "ocp_set_qp")
        self._keep = list(t.values()) + [st]
        torch.cuda.current_stream().synchronize()

    def set_bicycle(self, batch, x0=None, ref=None, Qd=None, Rd=None, Qfd=None):
        """Load a workloads.BicycleBatch; x0 [B,4], ref [S,4] and the weight
        diagonals Qd [4], Rd [2], Qfd [4] override the batch's when given."""
        self.generation += 1
        t = [_dev(batch.ref if ref is None else ref), _dev(batch.normal), _dev(batch.x0 if x0 is None else x0)]
        w = lambda v, dflt: [float(e) for e in (dflt if v is None else v)]  # noqa: E731
        u_init = getattr(batch, "u_init", None)
        if u_init is not None:
            t.append(_dev(u_init))
        p = A.ocp_bicycle(t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr(), batch.dt, batch.wheelbase,
                          batch.a_bound, batch.steer_bound, batch.lat_bound, batch.gamma_l1,
                          (C.c_double * 4)(*w(Qd, batch.Qd)), (C.c_double * 2)(*w(Rd, batch.Rd)),
                          (C.c_double * 4)(*w(Qfd, batch.Qfd)), int(getattr(batch, "integrator", 0)),
                          (C.c_double * 2)(*w(None, getattr(batch, "Wd", (0.0, 0.0)))),
                          t[3].data_ptr() if u_init is not None else None)
        A.check(self.lib.ocp_set_bicycle(self.h, C.byref(p), _stream()), "ocp_set_bicycle")
        self._keep = t
        torch.cuda.current_stream().synchronize()

    # ------------------------------------------------------------------ solve
    def alloc_solution(self):
        f64 = dict(dtype=torch.float64, device=self.device)
        i32 = dict(dtype=torch.int32, device=self.device)
        S, B = self.S, self.B
        return {
            "x": torch.empty(S, self.n, **f64), "xi": torch.empty(S, self.ng, **f64),
            "z_g": torch.empty(S, self.ng, **f64), "y_f": torch.empty(S, self.nx, **f64),
            "y_g": torch.empty(S, self.ng, **f64), "status": torch.empty(B, **i32),
            "admm_iters": torch.empty(B, **i32), "sqp_iters": torch.empty(B, **i32),
            "n_factor": torch.empty(B, **i32), "r_prim": torch.empty(B, **f64), "r_dual": torch.empty(B, **f64),
            "rho": torch.empty(B, **f64), "sqp_kkt": torch.empty(B, 3, **f64),
        }

    def solve(self, settings=None, out=None, sync=True, **overrides):
        s = settings if settings is not None else A.default_settings(**overrides)
        out = out if out is not None else self.alloc_solution()
        self.generation += 1
        sol = A.ocp_solution(*[(out[k].data_ptr() if out.get(k) is not None else None) for k, _ in
                               A.ocp_solution._fields_])
        A.check(self.lib.ocp_solve(self.h, C.byref(s), C.byref(sol), _stream()), "ocp_solve")
        if sync:
            torch.cuda.current_stream().synchronize()
        return out

    def solution_struct(self, out):
        return A.ocp_solution(*[(out[k].data_ptr() if out.get(k) is not None else None) for k, _ in
                                A.ocp_solution._fields_])

    def get_solution(self, out=None, sync=True):
        out = out if out is not None else self.alloc_solution()
        sol = self.solution_struct(out)
        A.check(self.lib.ocp_get_solution(self.h, C.byref(sol), _stream()), "ocp_get_solution")
        if sync:
            torch.cuda.current_stream().synchronize()
        return out

    def solve_raw(self, settings, sol_struct):
        """Launch a solve with a prebuilt ocp_solution (no allocation, no sync)."""
        self.generation += 1
        A.check(self.lib.ocp_solve(self.h, C.byref(settings), C.byref(sol_struct) if sol_struct is not None else None,
                                   _stream()), "ocp_solve")

    def adjoint(self, dL_dx, settings=None, dL_dxi=None, **overrides):
        s = settings if settings is not None else A.default_settings(**overrides)
        g = self.alloc_grads()
        gs = self.grads_struct(g)
        dl = _dev(dL_dx)
        dxi = _dev(dL_dxi) if dL_dxi is not None else None
        A.check(self.lib.ocp_adjoint(self.h, C.byref(s), C.c_void_p(dl.data_ptr()), _ptr(dxi), C.byref(gs),
                                     _stream()), "ocp_adjoint")
        torch.cuda.current_stream().synchronize()
        return g

    def profile(self, enable=True):
        """Record HIP events around every kernel launch of later calls."""
        A.check(self.lib.ocp_profile(self.h, int(bool(enable))), "ocp_profile")

    def profile_read(self):
        """{class: (total ms, launches)} since the last read (waits for the events)."""
        t = A.ocp_kernel_times()
        A.check(self.lib.ocp_profile_read(self.h, C.byref(t)), "ocp_profile_read")
        return {name: (t.ms[k], int(t.launches[k])) for k, name in enumerate(A.K_NAMES)}

    def adjoint_raw(self, settings, dl, grads_struct, dxi=None):
        """Launch an adjoint with prebuilt arguments (no allocation, no sync)."""
        A.check(self.lib.ocp_adjoint(self.h, C.byref(settings), C.c_void_p(dl.data_ptr()), _ptr(dxi),
                                     C.byref(grads_struct), _stream()), "ocp_adjoint")

    def alloc_grads(self):
        f64 = dict(dtype=torch.float64, device=self.device)
        return {"d_q": torch.empty(self.S, self.n, **f64), "d_Ddiag": torch.empty(self.S, self.n, **f64),
                "d_x_init": torch.empty(self.B, self.nx, **f64), "d_lo": torch.empty(self.S, self.ng, **f64),
                "d_hi": torch.empty(self.S, self.ng, **f64), "eta_x": torch.empty(self.S, self.n, **f64),
                "active": torch.empty(self.S, self.ng, dtype=torch.int8, device=self.device),
                "d_gamma2": torch.empty(self.B, **f64), "eta_f": torch.empty(self.S, self.nx, **f64),
                "eta_g": torch.empty(self.S, self.ng, **f64), "adj_resid": torch.empty(self.B, **f64),
                "adj_status": torch.empty(self.B, dtype=torch.int32, device=self.device),
                "eta_xi": torch.empty(self.S, self.ng, **f64), "d_gamma1": torch.empty(self.B, **f64)}

    def grads_struct(self, g):
        return A.ocp_qp_grads(*[g[k].data_ptr() for k, _ in A.ocp_qp_grads._fields_])

    def graph_capture(self, settings, out, dl=None, grads=None, dxi=None):
        """Record one solve (and the adjoint for dl, grads) into the handle's
        HIP graph on the current stream; `out`, `dl` and `grads` must stay
        alive and in place while the graph is replayed."""
        sol = self.solution_struct(out)
        gs = self.grads_struct(grads) if grads is not None else None
        self._graph_keep = (out, dl, grads, sol, gs, dxi)
        A.check(self.lib.ocp_graph_capture(self.h, C.byref(settings), C.byref(sol),
                                           C.c_void_p(dl.data_ptr()) if dl is not None else None, _ptr(dxi),
                                           C.byref(gs) if gs is not None else None, _stream()),
                "ocp_graph_capture")

    def graph_launch(self):
        self.generation += 1
        A.check(self.lib.ocp_graph_launch(self.h, _stream()), "ocp_graph_launch")

    def set_scaling(self, d=None, e_g=None, c=None):
        """Rescale later problems by per-instance factors d [B, n], e_g [B, ng],
        c [B] (ocp_set_scaling); d = None removes the rescaling.  Load the
        problem again afterwards."""
        self.generation += 1
        if d is None:
            A.check(self.lib.ocp_set_scaling(self.h, None, None, None, _stream()), "ocp_set_scaling")
            return
        t = [_dev(d), _dev(e_g), _dev(c)]
        A.check(self.lib.ocp_set_scaling(self.h, *[C.c_void_p(v.data_ptr()) for v in t], _stream()),
                "ocp_set_scaling")

    def set_scaling_box(self, p: float = 0.6):
        """Box normalisation of later problems, derived on the device
        (ocp_set_scaling_box).  Load the problem again afterwards."""
        self.generation += 1
        A.check(self.lib.ocp_set_scaling_box(self.h, float(p)), "ocp_set_scaling_box")

    def set_iterate(self, x, xi, y_f, y_g):
        """Restore a checkpointed SQP iterate (ocp_set_iterate), in the layout
        of the solution buffers."""
        t = [_dev(v) for v in (x, xi, y_f, y_g)]
        A.check(self.lib.ocp_set_iterate(self.h, *[C.c_void_p(v.data_ptr()) for v in t], _stream()),
                "ocp_set_iterate")
        torch.cuda.current_stream().synchronize()

    def set_segmented_after(self, iteration: int):
        """Instances still running at ADMM iteration `iteration` take the
        segmented substitutions (ocp_set_segmented_after)."""
        A.check(self.lib.ocp_set_segmented_after(self.h, int(iteration)), "ocp_set_segmented_after")

    def set_tail_workgroup(self, iteration: int):
        """One-wavefront instances still running at ADMM iteration `iteration`
        continue on two-wavefront workgroups (ocp_set_tail_workgroup; 0: off)."""
        A.check(self.lib.ocp_set_tail_workgroup(self.h, int(iteration)), "ocp_set_tail_workgroup")

    def set_linsolve(self, pcg: bool, max_iter: int = 50, tol: float = 1e-6):
        """Primal updates by block-Jacobi PCG (pcg=True) or the direct
        block-tridiagonal Cholesky (ocp_set_linsolve)."""
        A.check(self.lib.ocp_set_linsolve(self.h, A.LINSOLVE_PCG if pcg else A.LINSOLVE_DIRECT, int(max_iter),
                                          float(tol)), "ocp_set_linsolve")

    def set_multiwave(self, mw_min_n: int):
        """Horizons N >= mw_min_n solve on a multi-wavefront workgroup
        (ocp_set_multiwave; 0 turns it off)."""
        A.check(self.lib.ocp_set_multiwave(self.h, int(mw_min_n)), "ocp_set_multiwave")

    def set_segmented(self, seg_min_n: int):
        """Horizons N >= seg_min_n solve with segmented substitutions (ocp_set_segmented)."""
        A.check(self.lib.ocp_set_segmented(self.h, int(seg_min_n)), "ocp_set_segmented")

    def autotune(self, settings=None, reps: int = 1, **overrides):
        """Time the launch-shape candidates on this batch and keep the fastest
        (ocp_autotune); returns (segmented-from horizon, segmented-from iteration,
        two-wavefront continuation from iteration)."""
        s = settings if settings is not None else A.default_settings(**overrides)
        n_min, after, tail = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        self.generation += 1
        A.check(self.lib.ocp_autotune(self.h, C.byref(s), int(reps), _stream(), C.byref(n_min), C.byref(after),
                                      C.byref(tail)), "ocp_autotune")
        return int(n_min.value), int(after.value), int(tail.value)

    def split(self, arr, i):
        """Rows of a stage-concatenated array that belong to instance i."""
        return arr[int(self.stage_off[i]):int(self.stage_off[i + 1])]
