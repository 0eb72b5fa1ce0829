// ADMM iteration of Algorithm 3 for one instance per 16-lane row, fused over
// the horizon in two sweeps:
//
//  forward  (t = 0..N):  eta_t = sigma x_t - q_t + A_t^-'(rho_f c_t - y_f,t)
//                                + A_{t-1}^+'(rho_f c_{t-1} - y_f,t-1)
//                                + [t=0] (rho_f x_init - y_init)
//                                + G_t'(rho_g z_g,t - y_g,t)
//                        v_t   = Linv_t (eta_t - M_t v_{t-1})
//  backward (t = N..0):  x~_t  = Linv_t' (v_t - M_{t+1}' x~_{t+1})
//                        then, with x~_t and x~_{t+1} in registers, the
//                        over-relaxation, projection and dual update of
//                        every constraint row that touches stage t:
//                        dynamics row t, the inequality rows of stage t and
//                        (t = 0) the initial-state rows.
//
// Residuals, the stopping test and the rho adaptation are evaluated in FP64
// from FP64 problem data every k_check / k_rho iterations (eq.
// admm:residuals, admm:termination:slack, rho:update).
#pragma once

#include "factor.h"

namespace ocpk {

template <typename T>
struct Proj {
  T z, xi;
};

// slack update for one inequality row (see oracle/admm.py `project`)
template <typename T>
__device__ __forceinline__ Proj<T> project_row(T v, T lo, T hi, int kind, T rho_g, T gamma2, T gamma1) {
  const T pv = clampv(v, lo, hi);
  Proj<T> p{pv, T(0)};
  if (kind == 1) {
    p.z = (rho_g * v + gamma2 * pv) / (gamma2 + rho_g);
    p.xi = rho_g * (pv - v) / (gamma2 + rho_g);
  } else if (kind == 2) {
    const T kap = gamma1 / rho_g;
    const T d = pv - v;
    p.xi = d - clampv(d, -kap, kap);
    p.z = pv - p.xi;
  }
  return p;
}

// Time-invariant constraint blocks held in registers for the whole solve.
template <typename T, int NX, int NU, int NG>
struct TIBlocks {
  static constexpr int n = NX + NU;
  T AmR[n], ApR[n], GR[n];  // row `lane` of A^-, A^+ (lane < NX) and G (lane < NG)
  T AmC[NX], ApC[NX];       // column `lane` of A^-, A^+ (lane < n)
  T GC[NG];                 // column `lane` of G
  __device__ void load(const Layout& L, int b, int i) {
    const T* Am = (const T*)L.AmT + (size_t)b * NX * n;
    const T* Ap = (const T*)L.ApT + (size_t)b * NX * n;
    const T* G = (const T*)L.GT + (size_t)b * NG * n;
    load_row<n>(AmR, Am + (size_t)i * n, i < NX);
    load_row<n>(ApR, Ap + (size_t)i * n, i < NX);
    load_row<n>(GR, G + (size_t)i * n, i < NG);
    load_col<NX>(AmC, Am + i, n, i < n);
    load_col<NX>(ApC, Ap + i, n, i < n);
    load_col<NG>(GC, G + i, n, i < n);
  }
};

template <typename T, int NX, int NU, int NG, bool TI>
__device__ void admm_iteration(const Layout& L, const Group& g, const TIBlocks<T, NX, NU, NG>& tb, T sigma,
                               T rho_f, T rho_g, T alpha, int kind, T gamma2, T gamma1) {
  constexpr int n = NX + NU;
  const int i = g.lane;
  const int b = g.b;
  const int N = g.N;
  const size_t nn = (size_t)n * n;
  T* __restrict__ X = (T*)L.x;
  T* __restrict__ V = (T*)L.v;
  T* __restrict__ YF = (T*)L.yf;
  T* __restrict__ ZG = (T*)L.zg;
  T* __restrict__ YG = (T*)L.yg;
  T* __restrict__ XI = (T*)L.xi;
  const T* __restrict__ qT = (const T*)L.qT;
  const T* __restrict__ bdT = (const T*)L.bdT;
  const T* __restrict__ loT = (const T*)L.loT;
  const T* __restrict__ hiT = (const T*)L.hiT;
  const T* __restrict__ LinvT = (const T*)L.LinvT;
  const T* __restrict__ MT = (const T*)L.MT;
  const T xinit = (i < NX) ? ((const T*)L.xinitT)[(size_t)b * NX + i] : T(0);

  // ---------------- forward sweep ----------------
  T vprev = T(0), wprev = T(0);
  T ApCprev[NX];
  if constexpr (TI) {
#pragma unroll
    for (int r = 0; r < NX; ++r) ApCprev[r] = tb.ApC[r];
  }
  for (int t = 0; t <= N; ++t) {
    const int64_t s = g.s0 + t;
    const size_t sv = (size_t)s * ROW + i;
    const T xv = (i < n) ? X[sv] : T(0);
    T eta = sigma * xv - ((qT && i < n) ? qT[(size_t)s * n + i] : T(0));
    T w = T(0);
    T AmC[NX];
    if constexpr (TI) {
#pragma unroll
      for (int r = 0; r < NX; ++r) AmC[r] = tb.AmC[r];
    } else {
      if (t < N) load_col<NX>(AmC, (const T*)L.AmT + (size_t)s * NX * n + i, n, i < n);
    }
    if (t < N) {
      const T bdv = (bdT && i < NX) ? bdT[ti_or_tv(TI, b, s, NX) + i] : T(0);
      w = (i < NX) ? rho_f * bdv - YF[sv + ROW] : T(0);
      eta = dotb<NX>(AmC, w, eta);
    }
    if (t > 0) eta = dotb<NX>(ApCprev, wprev, eta);
    if (t == 0 && i < NX) eta += rho_f * xinit - YF[sv];
    {
      const T u = (i < NG) ? rho_g * ZG[sv] - YG[sv] : T(0);
      T GC[NG];
      if constexpr (TI) {
#pragma unroll
        for (int r = 0; r < NG; ++r) GC[r] = tb.GC[r];
      } else {
        load_col<NG>(GC, (const T*)L.GT + (size_t)s * NG * n + i, n, i < n);
      }
      eta = dotb<NG>(GC, u, eta);
    }
    if (t > 0) {
      T Mr[n];
      load_row<n>(Mr, MT + (size_t)s * nn + (size_t)i * n, i < n);
      eta -= dotb<n>(Mr, vprev, T(0));
    }
    T Lr[n];
    load_row<n>(Lr, LinvT + (size_t)s * nn + (size_t)i * n, i < n);
    const T vv = dotb<n>(Lr, eta, T(0));
    if (i < n) V[sv] = vv;
    vprev = vv;
    wprev = w;
    if constexpr (!TI) {
      if (t < N) load_col<NX>(ApCprev, (const T*)L.ApT + (size_t)s * NX * n + i, n, i < n);
    }
  }

  // ---------------- backward sweep + constraint-row updates ----------------
  T xnext = T(0);
  const T oma = T(1) - alpha;
  for (int t = N; t >= 0; --t) {
    const int64_t s = g.s0 + t;
    const size_t sv = (size_t)s * ROW + i;
    T vv = (i < n) ? V[sv] : T(0);
    if (t < N) {
      T Mc[n];
      load_col<n>(Mc, MT + (size_t)(s + 1) * nn + i, n, i < n);
      vv -= dotb<n>(Mc, xnext, T(0));
    }
    T Lc[n];
    load_col<n>(Lc, LinvT + (size_t)s * nn + i, n, i < n);
    const T xt = dotb<n>(Lc, vv, T(0));

    if (t < N) {  // dynamics row t:  y_f += rho_f alpha (A^- x~_t + A^+ x~_{t+1} - c_t)
      T AmR[n], ApR[n];
      if constexpr (TI) {
#pragma unroll
        for (int k = 0; k < n; ++k) {
          AmR[k] = tb.AmR[k];
          ApR[k] = tb.ApR[k];
        }
      } else {
        load_row<n>(AmR, (const T*)L.AmT + (size_t)s * NX * n + (size_t)i * n, i < NX);
        load_row<n>(ApR, (const T*)L.ApT + (size_t)s * NX * n + (size_t)i * n, i < NX);
      }
      T zf = dotb<n>(AmR, xt, T(0));
      zf = dotb<n>(ApR, xnext, zf);
      if (i < NX) {
        const T bdv = bdT ? bdT[ti_or_tv(TI, b, s, NX) + i] : T(0);
        YF[sv + ROW] += rho_f * alpha * (zf - bdv);
      }
    }
    {  // inequality rows of stage t
      T GR[n];
      if constexpr (TI) {
#pragma unroll
        for (int k = 0; k < n; ++k) GR[k] = tb.GR[k];
      } else {
        load_row<n>(GR, (const T*)L.GT + (size_t)s * NG * n + (size_t)i * n, i < NG);
      }
      const T zt = dotb<n>(GR, xt, T(0));
      if (i < NG) {
        const size_t sb = ti_or_tv(TI, b, s, NG) + i;
        const T zold = ZG[sv];
        const T zh = alpha * zt + oma * zold;
        const T yold = YG[sv];
        const Proj<T> p = project_row<T>(zh + yold / rho_g, loT[sb], hiT[sb], kind, rho_g, gamma2, gamma1);
        ZG[sv] = p.z;
        XI[sv] = p.xi;
        YG[sv] = yold + rho_g * (zh - p.z);
      }
    }
    if (i < n) X[sv] = alpha * xt + oma * X[sv];
    if (t == 0 && i < NX) YF[sv] += rho_f * alpha * (xt - xinit);
    xnext = xt;
  }
}

struct Resid {
  double rp, rd, ps, ds;
  int nonfinite;
};

// FP64 residuals of eq. admm:residuals and the scales of eq.
// admm:termination:slack, evaluated from FP64 problem data.
template <typename T, int NX, int NU, int NG>
__device__ Resid residuals(const Layout& L, const Group& g, int kind, double gamma2, double gamma1) {
  constexpr int n = NX + NU;
  const int i = g.lane;
  const int b = g.b;
  const int N = g.N;
  const size_t nn = (size_t)n * n;
  const T* __restrict__ X = (const T*)L.x;
  const T* __restrict__ YF = (const T*)L.yf;
  const T* __restrict__ ZG = (const T*)L.zg;
  const T* __restrict__ YG = (const T*)L.yg;
  const T* __restrict__ XI = (const T*)L.xi;
  double m_cxc = 0, m_cx = 0, m_c = 0, m_gxz = 0, m_gx = 0, m_z = 0;
  double m_dual = 0, m_px = 0, m_aty = 0, m_q = 0, m_sres = 0, m_sscale = 0;
  int nf = 0;
  auto upd = [&](double& m, double v) {
    if (!isfinite(v)) nf = 1;
    m = fmax(m, fabs(v));
  };
  double xm = 0.0, xc = (i < n) ? double(X[(size_t)g.s0 * ROW + i]) : 0.0;
  double yfm = 0.0;  // y_f of dynamics row t-1 (lane < NX)
  double Apcm[NX], Eprev[n];
#pragma unroll
  for (int r = 0; r < NX; ++r) Apcm[r] = 0.0;
#pragma unroll
  for (int k = 0; k < n; ++k) Eprev[k] = 0.0;
  for (int t = 0; t <= N; ++t) {
    const int64_t s = g.s0 + t;
    const size_t sv = (size_t)s * ROW + i;
    const double xn = (t < N && i < n) ? double(X[sv + ROW]) : 0.0;
    // (P x)_t row i = D_t x_t + E_{t-1} x_{t-1} + E_t' x_{t+1}
    const double* Dp = L.ti ? L.D + (size_t)(2 * b + (t == N ? 1 : 0)) * nn : L.D + (size_t)s * nn;
    double Dr[n];
    load_row<n>(Dr, Dp + (size_t)i * n, i < n);
    double px = dotb<n>(Dr, xc, 0.0);
    if (t > 0) px = dotb<n>(Eprev, xm, px);
    double Ec[n];
    if (L.E && t < N) {
      const double* Ep = L.E + ti_or_tv(L.ti, b, s, nn);
      load_col<n>(Ec, Ep + i, n, i < n);
      px = dotb<n>(Ec, xn, px);
      load_row<n>(Eprev, Ep + (size_t)i * n, i < n);
    }
    // (A' y)_t row i
    const double yfc = (t < N && i < NX) ? double(YF[sv + ROW]) : 0.0;
    double aty = 0.0;
    double Amc[NX], Amr[n], Apr[n];
    if (t < N) {
      const double* Amp = L.Am + ti_or_tv(L.ti, b, s, (size_t)NX * n);
      const double* App = L.Ap + ti_or_tv(L.ti, b, s, (size_t)NX * n);
      load_col<NX>(Amc, Amp + i, n, i < n);
      load_row<n>(Amr, Amp + (size_t)i * n, i < NX);
      load_row<n>(Apr, App + (size_t)i * n, i < NX);
      aty = dotb<NX>(Amc, yfc, aty);
    }
    if (t > 0) aty = dotb<NX>(Apcm, yfm, aty);
    if (t == 0 && i < NX) aty += double(YF[sv]);
    const double* Gp = L.G + ti_or_tv(L.ti, b, s, (size_t)NG * n);
    double Gc[NG], Gr[n];
    load_col<NG>(Gc, Gp + i, n, i < n);
    load_row<n>(Gr, Gp + (size_t)i * n, i < NG);
    const double ygv = (i < NG) ? double(YG[sv]) : 0.0;
    aty = dotb<NG>(Gc, ygv, aty);
    const double qv = (L.q && i < n) ? L.q[(size_t)s * n + i] : 0.0;
    if (i < n) {
      upd(m_dual, px + qv + aty);
      upd(m_px, px);
      upd(m_aty, aty);
      upd(m_q, qv);
    }
    // equality rows touching stage t
    if (t == 0 && i < NX) {
      const double xi0 = L.x_init[(size_t)b * NX + i];
      upd(m_cxc, xc - xi0);
      upd(m_cx, xc);
      upd(m_c, xi0);
    }
    if (t < N) {
      double cx = dotb<n>(Amr, xc, 0.0);
      cx = dotb<n>(Apr, xn, cx);
      if (i < NX) {
        const double cv = L.bd ? L.bd[ti_or_tv(L.ti, b, s, NX) + i] : 0.0;
        upd(m_cxc, cx - cv);
        upd(m_cx, cx);
        upd(m_c, cv);
      }
    }
    // inequality rows of stage t
    const double gx = dotb<n>(Gr, xc, 0.0);
    if (i < NG) {
      const double zv = double(ZG[sv]);
      upd(m_gxz, gx - zv);
      upd(m_gx, gx);
      upd(m_z, zv);
      const double xiv = double(XI[sv]);
      if (kind == 1) {
        upd(m_sres, gamma2 * xiv + ygv);
        upd(m_sscale, gamma2 * xiv);
        upd(m_sscale, ygv);
      } else if (kind == 2) {
        const double r1 = (xiv != 0.0) ? fabs(ygv + gamma1 * (xiv > 0 ? 1.0 : -1.0)) : fmax(fabs(ygv) - gamma1, 0.0);
        upd(m_sres, r1);
        upd(m_sscale, xiv != 0.0 ? gamma1 : 0.0);
        upd(m_sscale, ygv);
      }
    }
    // shift the window
    if (t < N) {
      const double* App = L.Ap + ti_or_tv(L.ti, b, s, (size_t)NX * n);
      load_col<NX>(Apcm, App + i, n, i < n);
    }
    yfm = yfc;
    xm = xc;
    xc = xn;
  }
  Resid R;
  R.rp = row_max(fmax(m_cxc, m_gxz));
  R.ps = row_max(fmax(fmax(m_cx, m_gx), fmax(m_c, m_z)));
  R.rd = row_max(fmax(m_dual, m_sres));
  R.ds = row_max(fmax(fmax(m_px, m_aty), fmax(m_q, m_sscale)));
  R.nonfinite = row_max(nf);
  return R;
}

// Zero the ADMM state of one instance (cold start).
template <typename T>
__device__ void cold_start(const Layout& L, const Group& g) {
  for (int t = 0; t <= g.N; ++t) {
    const size_t sv = (size_t)(g.s0 + t) * ROW + g.lane;
    ((T*)L.x)[sv] = T(0);
    ((T*)L.yf)[sv] = T(0);
    ((T*)L.zg)[sv] = T(0);
    ((T*)L.yg)[sv] = T(0);
    ((T*)L.xi)[sv] = T(0);
  }
}

// Whole ADMM solve of one instance per 16-lane row.
template <typename T, int NX, int NU, int NG, bool TI>
__global__ __launch_bounds__(64) void admm_solve_kernel(Layout L, Settings st) {
  Group g;
  g.lane = threadIdx.x & (ROW - 1);
  const int slot = blockIdx.x * ROWS_PER_WAVE + (threadIdx.x >> 4);
  if (slot >= L.B) return;
  g.b = L.order ? L.order[slot] : slot;
  g.s0 = L.stage_off[g.b];
  g.N = (int)(L.stage_off[g.b + 1] - g.s0) - 1;
  const int i = g.lane;
  const int kind = (i < NG) ? (int)L.soft[i] : 0;

  double rho_bar = st.warm ? L.rho[g.b] : st.rho0;
  if (!(rho_bar > 0.0)) rho_bar = st.rho0;
  if (!st.warm) cold_start<T>(L, g);

  int status = 1, k = 0, nfact = 0;
  Resid R{INFINITY, INFINITY, 0, 0, 0};
  if (factor_instance<T, NX, NU, NG>(L, g, st.sigma, st.rho_f_scale * rho_bar, rho_bar, nullptr)) {
    status = 3;
  } else {
    nfact = 1;
    TIBlocks<T, NX, NU, NG> tb;
    if constexpr (TI) tb.load(L, g.b, i);
    for (k = 1; k <= st.max_iter; ++k) {
      admm_iteration<T, NX, NU, NG, TI>(L, g, tb, T(st.sigma), T(st.rho_f_scale * rho_bar), T(rho_bar),
                                        T(st.alpha), kind, T(L.gamma2), T(L.gamma1));
      const bool check = st.k_check > 0 && (k % st.k_check) == 0;
      const bool adapt = st.adapt_rho && st.k_rho > 0 && (k % st.k_rho) == 0;
      if (check || adapt || k == st.max_iter) {
        R = residuals<T, NX, NU, NG>(L, g, kind, L.gamma2, L.gamma1);
        if (R.nonfinite) {
          status = 2;
          break;
        }
        const bool conv = R.rp <= st.eps_abs + st.eps_rel * R.ps && R.rd <= st.eps_abs + st.eps_rel * R.ds;
        if ((check || (st.k_check > 0 && k == st.max_iter)) && conv) {
          status = 0;
          break;
        }
        if (adapt && !conv) {
          const double num = R.rp / fmax(R.ps, 1e-30);
          const double den = R.rd / fmax(R.ds, 1e-30);
          double cand = rho_bar * sqrt(num / fmax(den, 1e-30));
          cand = fmin(fmax(cand, st.rho_min), st.rho_max);
          if (fmax(cand / rho_bar, rho_bar / cand) > st.k_ratio) {
            rho_bar = cand;
            if (factor_instance<T, NX, NU, NG>(L, g, st.sigma, st.rho_f_scale * rho_bar, rho_bar, nullptr)) {
              status = 3;
              break;
            }
            ++nfact;
          }
        }
      }
    }
    if (k > st.max_iter) k = st.max_iter;
  }
  if (i == 0) {
    L.rho[g.b] = rho_bar;
    L.status[g.b] = status;
    L.iters[g.b] = k;
    L.nfact[g.b] = nfact;
    L.rprim[g.b] = R.rp;
    L.rdual[g.b] = R.rd;
  }
}

}  // namespace ocpk
