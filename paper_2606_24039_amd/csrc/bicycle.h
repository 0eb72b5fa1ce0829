// Kinematic-bicycle SQP kernels (Algorithm 1): convexification of the OCP at
// the current iterate (Appendix "QP Approximation"), backtracking line search
// on the L1 merit (Appendix "Line search") and the stopping quantities of
// eq. sqp_stop.
//
// Model: state (px, py, yaw, v), control (a, delta), wheelbase Lw,
//   fc(x, u) = (v cos yaw, v sin yaw, v tan(delta) / Lw, a),
// implicit midpoint with zero-order hold on u:
//   f_t = x_t + dt fc((x_t + x_{t+1}) / 2, u_t) - x_{t+1},
//   A_t^- = [I + dt/2 Jx, dt Ju],  A_t^+ = [-I + dt/2 Jx, 0]  (at the midpoint).
// Cost 1/2 (x_t - r_t)'Q(x_t - r_t) + 1/2 u_t'R u_t (Q_f at t = N); in the
// absolute-coordinate QP q_t = grad l_t(xbar_t) - D_t xbar_t = -D_t (r_t, 0).
// Rows g_t = (a_t, delta_t, n_t'(p_t - p_ref,t)): a, delta hard, lateral L1.
#pragma once

#include "admm.h"

namespace ocpk {

__global__ void fill_i32_kernel(int32_t* p, int n, int v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

struct BikeArgs {
  const double* ref;     // [S][4]
  const double* normal;  // [S][2]
  const double* x0;      // [B][4]
  const int32_t* stage_inst;  // [S] instance of each global stage
  double dt, Lw, a_b, d_b, lat_b, gamma1;
  double Qd[4], Rd[2], Qfd[4];
  // control-rate cost 1/2 (u_t - u_{t+1})'diag(Wd)(u_t - u_{t+1}) (rate: Wd != 0)
  double Wd[2];
  int rate;
  const double* u_init;  // [B][2]: u_0 fixed (equality rows), or null
  int integ;  // 0 implicit midpoint, 1 trapezoidal rule
  // SQP state (FP64, padded [S][ROW])
  double* xbar;
  double* xibar;
  double* yfbar;
  double* ygbar;
  double* mu;       // [B] merit penalty
  double* kkt;      // [B][3]
  int32_t* done;    // [B] SQP iterations taken
  int32_t* frozen;  // [B] 1 once converged (only when not running a fixed count)
  double eps_c, armijo_eta;
  int fixed;
  // line search: chunks of LS_CHUNK stages (chunk -> instance, first stage;
  // instance -> first chunk, [B+1]); null: one chunk per instance
  const int32_t* chunk_inst;
  const int32_t* chunk_t0;
  const int32_t* chunk_off;
  double* parts;  // [chunks][LS_NF] merit parts, then (entries 0..2) the stopping maxima of the chunk;
                  // null: every horizon fits one chunk (the line-search kernel does all of it)
  double* alpha;  // [B] step length the line search took (chunked step update), with parts
};

struct BikeDeriv {
  double f[4];
  double Jx[4][4];
  double Ju[4][2];
};

__device__ __forceinline__ void bike_fc(const double* x, const double* u, double Lw, double* out) {
  out[0] = x[3] * cos(x[2]);
  out[1] = x[3] * sin(x[2]);
  out[2] = x[3] * tan(u[1]) / Lw;
  out[3] = u[0];
}

// midpoint residual f_t and its Jacobian blocks at (xt, ut, xn)
// Discrete dynamics f_t(x_t, u_t, x_{t+1}) and its Jacobians A^- (w.r.t.
// (x_t, u_t)) and A^+ (w.r.t. (x_{t+1}, u_{t+1})), zero-order hold on u:
//   integ 0, implicit midpoint: x_t + dt fc((x_t + x_{t+1})/2, u_t) - x_{t+1}
//   integ 1, trapezoidal rule (Remark A1):
//            x_t + dt/2 (fc(x_t, u_t) + fc(x_{t+1}, u_t)) - x_{t+1}
__device__ __forceinline__ void bike_fc(const double* x, const double* u, double Lw, double* fc, double (*Jx)[4],
                                        double* ju) {
  const double c = cos(x[2]), s = sin(x[2]), tn = tan(u[1]), cd = cos(u[1]);
  fc[0] = x[3] * c;
  fc[1] = x[3] * s;
  fc[2] = x[3] * tn / Lw;
  fc[3] = u[0];
  if (!Jx) return;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) Jx[r][k] = 0.0;
  Jx[0][2] = -x[3] * s;
  Jx[0][3] = c;
  Jx[1][2] = x[3] * c;
  Jx[1][3] = s;
  Jx[2][3] = tn / Lw;
  ju[0] = x[3] / (Lw * cd * cd);  // d yaw' / d delta (the only nonzero entry besides d v' / d a = 1)
}

template <int INTEG>
__device__ __forceinline__ void bike_dynamics(const double* xt, const double* ut, const double* xn, double dt,
                                              double Lw, double* f, double (*Am)[6], double (*Ap)[6]) {
  constexpr bool tr = INTEG == 1;
  double J0[4][4], J1[4][4], ju0 = 0.0, ju1 = 0.0;
  const bool jac = Am != nullptr;
  double f0[4];
  if constexpr (tr) {
    double f1[4];
    bike_fc(xt, ut, Lw, f0, jac ? J0 : nullptr, &ju0);
    bike_fc(xn, ut, Lw, f1, jac ? J1 : nullptr, &ju1);
#pragma unroll
    for (int k = 0; k < 4; ++k) f[k] = xt[k] + 0.5 * dt * (f0[k] + f1[k]) - xn[k];
  } else {
    double m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = 0.5 * (xt[k] + xn[k]);
    bike_fc(m, ut, Lw, f0, jac ? J0 : nullptr, &ju0);
#pragma unroll
    for (int k = 0; k < 4; ++k) f[k] = xt[k] + dt * f0[k] - xn[k];
  }
  if (!jac) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Am[r][k] = (r == k ? 1.0 : 0.0) + 0.5 * dt * J0[r][k];
      if constexpr (tr)
        Ap[r][k] = (r == k ? -1.0 : 0.0) + 0.5 * dt * J1[r][k];
      else
        Ap[r][k] = (r == k ? -1.0 : 0.0) + 0.5 * dt * J0[r][k];
    }
    Am[r][4] = 0.0;
    Am[r][5] = 0.0;
    Ap[r][4] = 0.0;
    Ap[r][5] = 0.0;
  }
  // control columns: d v' / d a = 1, d yaw' / d delta = ju
  Am[3][4] = dt;
  Am[2][5] = tr ? 0.5 * dt * (ju0 + ju1) : dt * ju0;
  (void)ju1;
}

// SQP initial guess: the reference with zero controls (u_0 = u_init when fixed).
__global__ void bike_init_kernel(Layout L, BikeArgs a, double rho0) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < (int64_t)L.B) {
    a.mu[s] = 0.0;
    a.done[s] = 0;
    a.frozen[s] = 0;
    L.rho[s] = rho0;
  }
  const int64_t S = L.stage_off[L.B];
  if (s >= S) return;
#pragma unroll
  for (int k = 0; k < ROW; ++k) {
    a.xbar[s * ROW + k] = (k < 4) ? a.ref[s * 4 + k] : 0.0;
    a.xibar[s * ROW + k] = 0.0;
    a.yfbar[s * ROW + k] = 0.0;
    a.ygbar[s * ROW + k] = 0.0;
  }
  if (a.u_init) {
    const int b = a.stage_inst[s];
    if (s == L.stage_off[b]) {
      a.xbar[s * ROW + 4] = a.u_init[(size_t)b * 2];
      a.xbar[s * ROW + 5] = a.u_init[(size_t)b * 2 + 1];
    }
  }
}

// Convexify at xbar and warm-start the ADMM state from the SQP iterate:
// x = xbar, y = ybar, z_g = G xbar.  One thread per global stage, blocks of
// LIN_BLOCK consecutive stages: each thread forms its stage's blocks in
// registers, and every output array (stage-major, so a block's stages are
// one contiguous range of it) is staged in LDS and written with consecutive
// lanes on consecutive elements.
// INTEG: the discretisation (0 implicit midpoint, 1 trapezoidal rule), a
// compile-time choice so that each kernel holds one rule's code.
constexpr int LIN_BLOCK = 64;
template <typename T, int INTEG>
__global__ __launch_bounds__(LIN_BLOCK) void bike_linearize_kernel(Layout L, BikeArgs a) {
  __shared__ double stg[LIN_BLOCK * 36];
  const int64_t S = L.stage_off[L.B];
  const int64_t sb = (int64_t)blockIdx.x * LIN_BLOCK;
  if (sb >= S) return;  // the whole block
  const int tid = threadIdx.x;
  const int64_t s = sb + tid;
  const int nst = (int)min<int64_t>(LIN_BLOCK, S - sb);
  const bool live = s < S;
  const int64_t sl = live ? s : S - 1;  // the idle threads read a valid stage and store nothing
  const int b = a.stage_inst[sl];
  const int64_t s0 = L.stage_off[b];
  const int t = (int)(sl - s0);
  const int N = (int)(L.stage_off[b + 1] - s0) - 1;
  const double* xb = a.xbar + sl * ROW;
  const double* Wq = (t == N) ? a.Qfd : a.Qd;
  // stage this thread's M values val(0..M-1), then store the block's range
  // of the array with consecutive lanes on consecutive elements
  auto put = [&](auto* dst, auto mc, auto&& val) {
    constexpr int M = decltype(mc)::value;
    using V = std::remove_pointer_t<decltype(dst)>;
    V* st = reinterpret_cast<V*>(stg);
    if (live) sfor<0, M>([&](auto k) { st[tid * M + decltype(k)::value] = val(decltype(k)::value); });
    __syncthreads();
    V* d = dst + sb * M;
    for (int e = tid; e < nst * M; e += LIN_BLOCK) d[e] = st[e];
    __syncthreads();
  };
  using I4 = std::integral_constant<int, 4>;
  using I3 = std::integral_constant<int, 3>;
  using I6 = std::integral_constant<int, 6>;
  using I18 = std::integral_constant<int, 18>;
  using I24 = std::integral_constant<int, 24>;
  using I36 = std::integral_constant<int, 36>;
  using IR = std::integral_constant<int, ROW>;

  // cost: D_t = diag(Q or Q_f, R) (+ the rate weights), q_t = -Q ref_t
  double dg[6], q[6];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    dg[k] = Wq[k];
    q[k] = -Wq[k] * a.ref[sl * 4 + k];
  }
  dg[4] = a.Rd[0];
  dg[5] = a.Rd[1];
  q[4] = q[5] = 0.0;
  if (a.rate) {
    // rate cost: W on the controls of the one or two differences touching
    // stage t, -W in E_t = block (t+1, t); a pure quadratic form, so q is unchanged
    const double cnt = (t < N ? 1.0 : 0.0) + (t > 0 ? 1.0 : 0.0);
    dg[4] += cnt * a.Wd[0];
    dg[5] += cnt * a.Wd[1];
    if (live && t < N) {
      double* E = const_cast<double*>(L.E) + s * 36;
#pragma unroll
      for (int k = 0; k < 36; ++k) E[k] = 0.0;
      E[4 * 6 + 4] = -a.Wd[0];
      E[5 * 6 + 5] = -a.Wd[1];
    }
  }
  // dynamics row t linearised at (xbar_t, xbar_{t+1}): A_t^- z_t + A_t^+ z_{t+1} = bd_t
  double Ml[4][6], Mr[4][6], bd[4];
  if (t < N) {
    const double* xn = xb + ROW;
    double f[4];
    bike_dynamics<INTEG>(xb, xb + 4, xn, a.dt, a.Lw, f, Ml, Mr);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double acc = -f[r];
#pragma unroll
      for (int k = 0; k < 6; ++k) acc += Ml[r][k] * xb[k] + Mr[r][k] * xn[k];
      bd[r] = acc;
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      bd[r] = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) Ml[r][k] = Mr[r][k] = 0.0;
    }
  }
  // constraint rows: a, delta and the lateral deviation n'(p - p_ref) + xi
  const double nx_ = a.normal[sl * 2], ny_ = a.normal[sl * 2 + 1];
  const double np = nx_ * a.ref[sl * 4] + ny_ * a.ref[sl * 4 + 1];
  double lo[3] = {-a.a_b, -a.d_b, -a.lat_b + np}, hi[3] = {a.a_b, a.d_b, a.lat_b + np};
  if (t == 0 && a.u_init) {  // (x_0, u_0) = (x_init, u_init): equality rows on u_0
    lo[0] = hi[0] = a.u_init[(size_t)b * 2];
    lo[1] = hi[1] = a.u_init[(size_t)b * 2 + 1];
  }
  auto Gv = [&](int k) { return k == 4 || k == 11 ? 1.0 : k == 12 ? nx_ : k == 13 ? ny_ : 0.0; };
  if (live && t == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) const_cast<double*>(L.x_init)[(size_t)b * 4 + k] = a.x0[(size_t)b * 4 + k];
  }
  put(const_cast<double*>(L.D), I36{}, [&](int k) { return (k % 7 == 0) ? dg[k / 7] : 0.0; });
  put(const_cast<double*>(L.q), I6{}, [&](int k) { return q[k]; });
  put(const_cast<double*>(L.Am), I24{}, [&](int k) { return Ml[k / 6][k % 6]; });
  put(const_cast<double*>(L.Ap), I24{}, [&](int k) { return Mr[k / 6][k % 6]; });
  put(const_cast<double*>(L.bd), I4{}, [&](int k) { return bd[k]; });
  put(const_cast<double*>(L.G), I18{}, Gv);
  put(const_cast<double*>(L.lo), I3{}, [&](int k) { return lo[k]; });
  put(const_cast<double*>(L.hi), I3{}, [&](int k) { return hi[k]; });
  // iteration-precision copies
  if constexpr (!std::is_same<T, double>::value) {
    put((T*)L.AmT, I24{}, [&](int k) { return T(Ml[k / 6][k % 6]); });
    put((T*)L.ApT, I24{}, [&](int k) { return T(Mr[k / 6][k % 6]); });
    put((T*)L.GT, I18{}, [&](int k) { return T(Gv(k)); });
    put((T*)L.qT, I6{}, [&](int k) { return T(q[k]); });
    put((T*)L.bdT, I4{}, [&](int k) { return T(bd[k]); });
    put((T*)L.loT, I3{}, [&](int k) { return T(lo[k]); });
    put((T*)L.hiT, I3{}, [&](int k) { return T(hi[k]); });
    if (live && t == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) ((T*)L.xinitT)[(size_t)b * 4 + k] = T(a.x0[(size_t)b * 4 + k]);
    }
  }
  // warm start of the ADMM state
  const double* yfb = a.yfbar + sl * ROW;
  const double* ygb = a.ygbar + sl * ROW;
  const double zg2 = nx_ * xb[0] + ny_ * xb[1];
  put((T*)L.x, IR{}, [&](int k) { return T(xb[k]); });
  put((T*)L.yf, IR{}, [&](int k) { return T(yfb[k]); });
  put((T*)L.yg, IR{}, [&](int k) { return T(ygb[k]); });
  put((T*)L.xi, IR{}, [&](int k) { return T(0); });
  put((T*)L.zg, IR{}, [&](int k) { return k == 0 ? T(xb[4]) : k == 1 ? T(xb[5]) : k == 2 ? T(zg2) : T(0); });
}

// Per-stage pieces of the merit at z = xbar + alpha (x* - xbar).
struct MeritPart {
  double cost, viol;
};

__device__ __forceinline__ void bike_point(const BikeArgs& a, const double* xb, const double* dx, double al,
                                           double* z) {
#pragma unroll
  for (int k = 0; k < 6; ++k) z[k] = xb[k] + al * dx[k];
}

// sum / max over the wavefront (every lane receives the result; fixed order)
__device__ __forceinline__ double wave_sum(double v) {
  v = row_sum(v);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  v = row_max(v);
  v = fmax(v, __shfl_xor(v, 16));
  v = fmax(v, __shfl_xor(v, 32));
  return v;
}

// Merit pieces of the stages t_begin .. t_end - 1 of instance b (lane
// stride 64): cost and constraint violation at z = xbar + alpha (x* - xbar)
// for alpha = 0, 1, 1/2, ..., 1/128 (entries 0..8), and the directional
// derivative of cost + slack penalty at xbar.
template <typename T, int INTEG>
__device__ __forceinline__ void bike_merit_stages(const Layout& L, const BikeArgs& a, int b, int64_t s0, int N,
                                                  int t_begin, int t_end, int lane, double (&cost)[9],
                                                  double (&viol)[9], double& gdir) {
  constexpr int NA = 8;
  const T* XS = (const T*)L.x;
  const T* XIS = (const T*)L.xi;
  const double* x0 = a.x0 + (size_t)b * 4;
  for (int t = t_begin + lane; t < t_end; t += 64) {
    const int64_t s = s0 + t;
    double xb[6], dx[6], xbn[6], dxn[6];
    const double xib = a.xibar[s * ROW + 2];
    const double dxi = double(XIS[s * ROW + 2]) - xib;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      xb[k] = a.xbar[s * ROW + k];
      dx[k] = double(XS[s * ROW + k]) - xb[k];
    }
    if (t < N) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        xbn[k] = a.xbar[(s + 1) * ROW + k];
        dxn[k] = double(XS[(s + 1) * ROW + k]) - xbn[k];
      }
    }
    const double* W = (t == N) ? a.Qfd : a.Qd;
    const double* r = a.ref + s * 4;
    const double nx_ = a.normal[s * 2], ny_ = a.normal[s * 2 + 1];
    const double gconst = -(nx_ * r[0] + ny_ * r[1]);
    // directional derivative of cost + slack penalty at xbar
#pragma unroll
    for (int k = 0; k < 4; ++k) gdir += W[k] * (xb[k] - r[k]) * dx[k];
    gdir += a.Rd[0] * xb[4] * dx[4] + a.Rd[1] * xb[5] * dx[5];
    gdir += a.gamma1 * ((xib != 0.0) ? (xib > 0 ? dxi : -dxi) : fabs(dxi));
    if (a.rate && t < N)
#pragma unroll
      for (int k = 0; k < 2; ++k) gdir += a.Wd[k] * (xb[4 + k] - xbn[4 + k]) * (dx[4 + k] - dxn[4 + k]);
    // bounds of the control rows (u_0 fixed when u_init is given)
    const bool fix0 = t == 0 && a.u_init;
    const double alo = fix0 ? a.u_init[(size_t)b * 2] : -a.a_b, ahi = fix0 ? alo : a.a_b;
    const double dlo = fix0 ? a.u_init[(size_t)b * 2 + 1] : -a.d_b, dhi = fix0 ? dlo : a.d_b;
#pragma unroll
    for (int j = 0; j <= NA; ++j) {
      const double al = (j == 0) ? 0.0 : ldexp(1.0, -(j - 1));
      double z[6], zn[6];
      bike_point(a, xb, dx, al, z);
      const double xi = xib + al * dxi;
      double c = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) c += 0.5 * W[k] * (z[k] - r[k]) * (z[k] - r[k]);
      c += 0.5 * (a.Rd[0] * z[4] * z[4] + a.Rd[1] * z[5] * z[5]) + a.gamma1 * fabs(xi);
      double v = 0.0;
      if (t < N) {
        bike_point(a, xbn, dxn, al, zn);
        double f[4];
        bike_dynamics<INTEG>(z, z + 4, zn, a.dt, a.Lw, f, nullptr, nullptr);
#pragma unroll
        for (int k = 0; k < 4; ++k) v += fabs(f[k]);
        if (a.rate)
#pragma unroll
          for (int k = 0; k < 2; ++k) c += 0.5 * a.Wd[k] * (z[4 + k] - zn[4 + k]) * (z[4 + k] - zn[4 + k]);
      }
      if (t == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) v += fabs(z[k] - x0[k]);
      }
      const double g0 = z[4], g1 = z[5], g2 = nx_ * z[0] + ny_ * z[1] + gconst + xi;
      v += fmax(g0 - ahi, 0.0) + fmax(alo - g0, 0.0) + fmax(g1 - dhi, 0.0) + fmax(dlo - g1, 0.0) +
           fmax(g2 - a.lat_b, 0.0) + fmax(-a.lat_b - g2, 0.0);
      cost[j] += c;
      viol[j] += v;
    }
  }
}

// SQP step with the line search's length alpha: the iterate moves towards the
// QP solution, stages t_begin .. t_end - 1 of the instance starting at stage
// s0 (lane stride 64).
template <typename T>
__device__ __forceinline__ void bike_take_step(const Layout& L, const BikeArgs& a, int64_t s0, int t_begin, int t_end,
                                               int lane, double alpha) {
  const T* XS = (const T*)L.x;
  const T* XIS = (const T*)L.xi;
  const T* YFS = (const T*)L.yf;
  const T* YGS = (const T*)L.yg;
  for (int t = t_begin + lane; t < t_end; t += 64) {
    const size_t sv = (size_t)(s0 + t) * ROW;
#pragma unroll
    for (int k = 0; k < 6; ++k) a.xbar[sv + k] += alpha * (double(XS[sv + k]) - a.xbar[sv + k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a.xibar[sv + k] += alpha * (double(XIS[sv + k]) - a.xibar[sv + k]);
      a.ygbar[sv + k] += alpha * (double(YGS[sv + k]) - a.ygbar[sv + k]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) a.yfbar[sv + k] += alpha * (double(YFS[sv + k]) - a.yfbar[sv + k]);
  }
}

// Stopping-quantity pieces (eq. sqp_stop) at the SQP iterate, stages
// t_begin .. t_end - 1 of instance b (lane stride 64): maxima of the
// stationarity residual, the equality residuals and the inequality
// violations.
template <int INTEG>
__device__ __forceinline__ void bike_stop_stages(const BikeArgs& a, int b, int64_t s0, int N, int t_begin, int t_end,
                                                 int lane, double& st, double& fe, double& gi) {
  const double* x0 = a.x0 + (size_t)b * 4;
  for (int t = t_begin + lane; t < t_end; t += 64) {
    const int64_t s = s0 + t;
    const double* xb = a.xbar + s * ROW;
    const double* W = (t == N) ? a.Qfd : a.Qd;
    const double* r = a.ref + s * 4;
    double grad[6];
#pragma unroll
    for (int k = 0; k < 4; ++k) grad[k] = W[k] * (xb[k] - r[k]);
    grad[4] = a.Rd[0] * xb[4];
    grad[5] = a.Rd[1] * xb[5];
    if (a.rate) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (t < N) grad[4 + k] += a.Wd[k] * (xb[4 + k] - xb[ROW + 4 + k]);
        if (t > 0) grad[4 + k] += a.Wd[k] * (xb[4 + k] - xb[-ROW + 4 + k]);
      }
    }
    const double* yg = a.ygbar + s * ROW;
    const double nx_ = a.normal[s * 2], ny_ = a.normal[s * 2 + 1];
    grad[4] += yg[0];
    grad[5] += yg[1];
    grad[0] += nx_ * yg[2];
    grad[1] += ny_ * yg[2];
    double f[4], Ml[4][6], Mr[4][6];
    if (t < N) {  // dynamics row t (slot t): A_t^-' y
      const double* yf = a.yfbar + s * ROW;
      bike_dynamics<INTEG>(xb, xb + 4, xb + ROW, a.dt, a.Lw, f, Ml, Mr);
#pragma unroll
      for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) grad[k] += Ml[rr][k] * yf[rr];
#pragma unroll
      for (int k = 0; k < 4; ++k) fe = fmax(fe, fabs(f[k]));
    }
    if (t > 0) {  // dynamics row t-1 (slot t-1): A_{t-1}^+' y
      const double* yf = a.yfbar + (s - 1) * ROW;
      const double* xp = xb - ROW;
      bike_dynamics<INTEG>(xp, xp + 4, xb, a.dt, a.Lw, f, Ml, Mr);
#pragma unroll
      for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) grad[k] += Mr[rr][k] * yf[rr];
    } else {  // initial-state rows (slot N)
      const double* yf = a.yfbar + (s0 + N) * ROW;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        grad[k] += yf[k];
        fe = fmax(fe, fabs(xb[k] - x0[k]));
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) st = fmax(st, fabs(grad[k]));
    const double xi = a.xibar[s * ROW + 2];
    const double g0 = xb[4], g1 = xb[5], g2 = nx_ * (xb[0] - r[0]) + ny_ * (xb[1] - r[1]) + xi;
    const bool fix0 = t == 0 && a.u_init;
    const double alo = fix0 ? a.u_init[(size_t)b * 2] : -a.a_b, ahi = fix0 ? alo : a.a_b;
    const double dlo = fix0 ? a.u_init[(size_t)b * 2 + 1] : -a.d_b, dhi = fix0 ? dlo : a.d_b;
    gi = fmax(gi, fmax(fmax(g0 - ahi, alo - g0), 0.0));
    gi = fmax(gi, fmax(fmax(g1 - dhi, dlo - g1), 0.0));
    gi = fmax(gi, fmax(fmax(g2 - a.lat_b, -a.lat_b - g2), 0.0));
  }
}

// stages per block of bike_merit_parts_kernel, and the merit parts of a block
constexpr int LS_CHUNK = 512;
constexpr int LS_NF = 19;  // cost[0..8], viol[0..8], gdir

// Merit parts of the line search, one wavefront per chunk of LS_CHUNK stages
// of an instance (a.chunk_inst / a.chunk_t0; without them one chunk per
// instance), written to a.parts[chunk][LS_NF]; bike_linesearch_kernel adds
// an instance's chunks in order.  Long horizons spread over many wavefronts.
template <typename T, int INTEG>
__global__ __launch_bounds__(64) void bike_merit_parts_kernel(Layout L, BikeArgs a, int nchunks) {
  const int c = blockIdx.x;
  if (c >= nchunks) return;
  const int b = a.chunk_inst ? a.chunk_inst[c] : c;
  if (a.frozen[b]) return;
  const int64_t s0 = L.stage_off[b];
  const int N = (int)(L.stage_off[b + 1] - s0) - 1;
  const int t0 = a.chunk_inst ? a.chunk_t0[c] : 0;
  const int t1 = a.chunk_inst ? min(t0 + LS_CHUNK, N + 1) : N + 1;
  double cost[9], viol[9], gdir = 0.0;
#pragma unroll
  for (int j = 0; j < 9; ++j) cost[j] = viol[j] = 0.0;
  bike_merit_stages<T, INTEG>(L, a, b, s0, N, t0, t1, (int)threadIdx.x, cost, viol, gdir);
  gdir = wave_sum(gdir);
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    cost[j] = wave_sum(cost[j]);
    viol[j] = wave_sum(viol[j]);
  }
  if (threadIdx.x == 0) {
    double* o = a.parts + (size_t)c * LS_NF;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      o[j] = cost[j];
      o[9 + j] = viol[j];
    }
    o[18] = gdir;
  }
}

// Line search and SQP bookkeeping, one wavefront per instance.  Lane i
// handles the stages t = i, i+64, ...; per-candidate sums are wavefront
// reductions.
template <typename T, int INTEG>
__global__ __launch_bounds__(64) void bike_linesearch_kernel(Layout L, BikeArgs a) {
  constexpr int NA = 8;  // alpha in {1, 1/2, ..., 1/128}
  const int lane = threadIdx.x;
  const int slot = blockIdx.x;
  if (slot >= L.B) return;
  const int b = L.order ? L.order[slot] : slot;
  if (a.frozen[b]) return;
  const int64_t s0 = L.stage_off[b];
  const int N = (int)(L.stage_off[b + 1] - s0) - 1;

  // merit pieces over the whole horizon: from the parts of this instance's
  // chunks (bike_merit_parts_kernel, added in chunk order: lane f sums part
  // f) when the batch has horizons longer than a chunk, else here
  double cost[NA + 1], viol[NA + 1], gdir = 0.0;
  if (a.parts) {
    const int c0 = a.chunk_off ? a.chunk_off[b] : b, c1 = a.chunk_off ? a.chunk_off[b + 1] : b + 1;
    double acc = 0.0;
    if (lane < LS_NF)
      for (int c = c0; c < c1; ++c) acc += a.parts[(size_t)c * LS_NF + lane];
#pragma unroll
    for (int j = 0; j <= NA; ++j) {
      cost[j] = __shfl(acc, j);
      viol[j] = __shfl(acc, 9 + j);
    }
    gdir = __shfl(acc, 18);
  } else {
#pragma unroll
    for (int j = 0; j <= NA; ++j) cost[j] = viol[j] = 0.0;
    bike_merit_stages<T, INTEG>(L, a, b, s0, N, 0, N + 1, lane, cost, viol, gdir);
    gdir = wave_sum(gdir);
#pragma unroll
    for (int j = 0; j <= NA; ++j) {
      cost[j] = wave_sum(cost[j]);
      viol[j] = wave_sum(viol[j]);
    }
  }
  const double mu = fmax(fmax(a.mu[b], fabs(gdir) / (0.5 * fmax(viol[0], a.eps_c))), 1.0);
  const double dmu = gdir - mu * viol[0];
  const double phi0 = cost[0] + mu * viol[0];
  double alpha = -1.0;
#pragma unroll
  for (int j = 1; j <= NA; ++j) {
    const double al = ldexp(1.0, -(j - 1));
    const double ph = cost[j] + mu * viol[j];
    if (alpha < 0.0 && isfinite(ph) && ph <= phi0 + a.armijo_eta * al * dmu) alpha = al;
  }
  if (alpha < 0.0) {  // fallback: the finite candidate with the smallest merit (ties: larger alpha)
    double best = INFINITY;
    alpha = 0.0;
#pragma unroll
    for (int j = 1; j <= NA; ++j) {
      const double ph = cost[j] + mu * viol[j];
      if (isfinite(ph) && ph < best) {
        best = ph;
        alpha = ldexp(1.0, -(j - 1));
      }
    }
  }
  if (a.parts) {  // the step and the stopping quantities follow in bike_stop_parts_kernel / bike_stop_combine_kernel
    if (lane == 0) {
      a.mu[b] = mu;
      a.alpha[b] = alpha;
    }
    return;
  }
  // take the step (lane i updates the stages t = i, i+64, ...)
  bike_take_step<T>(L, a, s0, 0, N + 1, lane, alpha);
  // the stopping quantities read the neighbouring stages other lanes wrote
  __syncthreads();
  // stopping quantities (eq. sqp_stop) at the new iterate
  double st = 0.0, fe = 0.0, gi = 0.0;
  bike_stop_stages<INTEG>(a, b, s0, N, 0, N + 1, lane, st, fe, gi);
  st = wave_max(st);
  fe = wave_max(fe);
  gi = wave_max(gi);
  if (lane == 0) {
    a.mu[b] = mu;
    a.kkt[(size_t)b * 3 + 0] = st;
    a.kkt[(size_t)b * 3 + 1] = fe;
    a.kkt[(size_t)b * 3 + 2] = gi;
    a.done[b] += 1;
    if (!a.fixed && st <= a.eps_c && fe <= a.eps_c && gi <= a.eps_c) a.frozen[b] = 1;
  }
}

// The step of a batch with horizons past one chunk, one wavefront per chunk,
// with the length bike_linesearch_kernel chose for the instance.
template <typename T>
__global__ __launch_bounds__(64) void bike_step_parts_kernel(Layout L, BikeArgs a, int nchunks) {
  const int c = blockIdx.x;
  if (c >= nchunks) return;
  const int b = a.chunk_inst ? a.chunk_inst[c] : c;
  if (a.frozen[b]) return;
  const int64_t s0 = L.stage_off[b];
  const int N = (int)(L.stage_off[b + 1] - s0) - 1;
  const int t0 = a.chunk_inst ? a.chunk_t0[c] : 0;
  const int t1 = a.chunk_inst ? min(t0 + LS_CHUNK, N + 1) : N + 1;
  bike_take_step<T>(L, a, s0, t0, t1, (int)threadIdx.x, a.alpha[b]);
}

// Stopping quantities of a batch with horizons past one chunk: their maxima
// over each chunk of LS_CHUNK stages (parts 0..2 of the chunk), after
// bike_step_parts_kernel took the step of every chunk.
template <typename T, int INTEG>
__global__ __launch_bounds__(64) void bike_stop_parts_kernel(Layout L, BikeArgs a, int nchunks) {
  const int c = blockIdx.x;
  if (c >= nchunks) return;
  const int b = a.chunk_inst ? a.chunk_inst[c] : c;
  if (a.frozen[b]) return;
  const int64_t s0 = L.stage_off[b];
  const int N = (int)(L.stage_off[b + 1] - s0) - 1;
  const int t0 = a.chunk_inst ? a.chunk_t0[c] : 0;
  const int t1 = a.chunk_inst ? min(t0 + LS_CHUNK, N + 1) : N + 1;
  double st = 0.0, fe = 0.0, gi = 0.0;
  bike_stop_stages<INTEG>(a, b, s0, N, t0, t1, (int)threadIdx.x, st, fe, gi);
  st = wave_max(st);
  fe = wave_max(fe);
  gi = wave_max(gi);
  if (threadIdx.x == 0) {
    double* o = a.parts + (size_t)c * LS_NF;
    o[0] = st, o[1] = fe, o[2] = gi;
  }
}

// The instance's stopping quantities from its chunks' maxima; the SQP
// iteration count and the convergence flag (one thread per instance).
__global__ void bike_stop_combine_kernel(Layout L, BikeArgs a) {
  const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= L.B || a.frozen[b]) return;
  const int c0 = a.chunk_off ? a.chunk_off[b] : b, c1 = a.chunk_off ? a.chunk_off[b + 1] : b + 1;
  double st = 0.0, fe = 0.0, gi = 0.0;
  for (int c = c0; c < c1; ++c) {
    const double* p = a.parts + (size_t)c * LS_NF;
    st = fmax(st, p[0]), fe = fmax(fe, p[1]), gi = fmax(gi, p[2]);
  }
  a.kkt[(size_t)b * 3 + 0] = st;
  a.kkt[(size_t)b * 3 + 1] = fe;
  a.kkt[(size_t)b * 3 + 2] = gi;
  a.done[b] += 1;
  if (!a.fixed && st <= a.eps_c && fe <= a.eps_c && gi <= a.eps_c) a.frozen[b] = 1;
}

// sum_k y_k grad^2 fc_k at (x, u) over w = (px, py, yaw, v, a, delta): the
// nonzero second derivatives of v cos(yaw), v sin(yaw), v tan(delta) / L
__device__ __forceinline__ void bike_fc_hessian(const double* x, const double* u, const double* y, double Lw,
                                                double (*A)[6]) {
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = 0; c < 6; ++c) A[r][c] = 0.0;
  const double cy = cos(x[2]), sy = sin(x[2]), v = x[3];
  const double cd = cos(u[1]), c2 = cd * cd, td = tan(u[1]);
  A[2][2] = -y[0] * v * cy - y[1] * v * sy;
  A[2][3] = A[3][2] = -y[0] * sy + y[1] * cy;
  A[3][5] = A[5][3] = y[2] / (Lw * c2);
  A[5][5] = y[2] * 2.0 * v * td / (Lw * c2);
}

// Curvature blocks of dynamics row t (multiplier y) over the stage variables
// z_t = (x_t, u_t) and x_{t+1}: left [6][6] (z_t, z_t), right [4][4]
// (x_{t+1}, x_{t+1}), cross [4][6] (x_{t+1}, z_t), all of y' grad^2 f_t.
//   midpoint:  dt M' A((x_t + x_{t+1})/2, u_t) M,  M = [[I/2, 0, I/2], [0, I, 0]]
//   trapezoid: dt/2 (A(x_t, u_t) on (x_t, u_t) + A(x_{t+1}, u_t) on (x_{t+1}, u_t))
template <int INTEG>
__device__ __forceinline__ void bike_row_hessian(const double* xt, const double* ut, const double* xn,
                                                 const double* y, double dt, double Lw, double (*left)[6],
                                                 double (*right)[4], double (*cross)[6]) {
  double A[6][6];
  if constexpr (INTEG == 0) {
    double m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = 0.5 * (xt[k] + xn[k]);
    bike_fc_hessian(m, ut, y, Lw, A);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) left[r][c] = dt * A[r][c] * (r < 4 ? 0.5 : 1.0) * (c < 4 ? 0.5 : 1.0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int c = 0; c < 4; ++c) right[r][c] = 0.25 * dt * A[r][c];
#pragma unroll
      for (int c = 0; c < 6; ++c) cross[r][c] = dt * A[r][c] * 0.5 * (c < 4 ? 0.5 : 1.0);
    }
  } else {
    double B[6][6];
    bike_fc_hessian(xt, ut, y, Lw, A);
    bike_fc_hessian(xn, ut, y, Lw, B);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) left[r][c] = 0.5 * dt * (A[r][c] + ((r >= 4 && c >= 4) ? B[r][c] : 0.0));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int c = 0; c < 4; ++c) right[r][c] = 0.5 * dt * B[r][c];
#pragma unroll
      for (int c = 0; c < 6; ++c) cross[r][c] = (c >= 4) ? 0.5 * dt * B[r][c] : 0.0;
    }
  }
}

// Exact Hessian of the Lagrangian at the SQP iterate (one thread per stage):
// D_t gains the curvature of dynamics row t (left block) and of row t-1
// (right block), E_t (block (t+1, t)) the cross block of row t.  Runs after
// bike_linearize_kernel, which leaves the cost's Hessian in D_t and, with a
// rate cost, E_t.
template <int INTEG>
__global__ void bike_hessian_kernel(Layout L, BikeArgs a) {
  const int64_t S = L.stage_off[L.B];
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const int b = a.stage_inst[s];
  const int64_t s0 = L.stage_off[b];
  const int t = (int)(s - s0);
  const int N = (int)(L.stage_off[b + 1] - s0) - 1;
  double* D = const_cast<double*>(L.D) + s * 36;
  double* E = const_cast<double*>(L.E) + s * 36;
  double left[6][6], right[4][4], cross[4][6];
  if (!a.rate)  // with a rate cost the linearisation has written E_t = -W (t < N)
#pragma unroll
    for (int k = 0; k < 36; ++k) E[k] = 0.0;
  if (t < N) {  // row t: this stage on the left
    const double* xt = a.xbar + s * ROW;
    bike_row_hessian<INTEG>(xt, xt + 4, xt + ROW, a.yfbar + s * ROW, a.dt, a.Lw, left, right, cross);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) D[r * 6 + c] += left[r][c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) E[r * 6 + c] += cross[r][c];
  }
  if (t > 0) {  // row t-1: this stage's state on the right
    const double* xp = a.xbar + (s - 1) * ROW;
    bike_row_hessian<INTEG>(xp, xp + 4, xp + ROW, a.yfbar + (s - 1) * ROW, a.dt, a.Lw, left, right, cross);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) D[r * 6 + c] += right[r][c];
  }
}

// The QP state of the adjoint set to the SQP iterate: slacks (the
// linearisation has put x and the multipliers in place)
template <typename T>
__global__ void iterate_slacks_kernel(const double* __restrict__ xibar, T* __restrict__ xi, int64_t S) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < S * ROW) xi[k] = T(xibar[k]);
}

// checkpointed iterate (output layout) -> the SQP state (padded [S][ROW]);
// y_f from the output slot convention (initial rows at the first stage,
// dynamics row t at stage t + 1) to the internal one (dynamics row t at
// stage t, initial rows at the last stage)
__global__ void load_iterate_kernel(const double* __restrict__ x, const double* __restrict__ xi,
                                    const double* __restrict__ yf, const double* __restrict__ yg,
                                    const int64_t* __restrict__ off, const int32_t* __restrict__ inst, int64_t S,
                                    int n, int nx, int ng, double* __restrict__ xbar, double* __restrict__ xibar,
                                    double* __restrict__ yfbar, double* __restrict__ ygbar) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= S * ROW) return;
  const int64_t s = k / ROW;
  const int j = (int)(k % ROW);
  xbar[k] = j < n ? x[s * n + j] : 0.0;
  xibar[k] = j < ng ? xi[s * ng + j] : 0.0;
  ygbar[k] = j < ng ? yg[s * ng + j] : 0.0;
  const int b = inst[s];
  const int64_t to = (s == off[b]) ? off[b + 1] - 1 : s - 1;
  if (j < nx) yfbar[to * ROW + j] = yf[s * nx + j];
  else yfbar[to * ROW + j] = 0.0;
}

}  // namespace ocpk
