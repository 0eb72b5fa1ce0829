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

// Structure of the per-iteration data, fixed at compile time:
//  TI     blocks are the same at every stage (held in registers for the solve)
//  APNEG  A^+ = [-I 0] (explicit dynamics): A^+' w and A^+ x become copies
//  GSEL   every inequality row selects one variable (box bounds): G x and
//         G' u become lane gathers
template <bool TI_, bool APNEG_, bool GSEL_>
struct Structure {
  static constexpr bool TI = TI_, APNEG = APNEG_, GSEL = GSEL_;
};

// Time-invariant constraint blocks held in registers for the whole solve.
template <typename T, int NX, int NU, int NG>
struct TIBlocks {
  static constexpr int n = NX + NU;
  T AmR[n], ApR[n], GR[n];  // row `lane` of A^-, A^+ (lane < NX) and G (lane < NG)
  T AmC[NX], ApC[NX];       // column `lane` of A^-, A^+ (lane < n)
  T GC[NG];                 // column `lane` of G
  T lo, hi, bd;             // bounds of inequality row `lane`, c of dynamics row `lane`
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
    lo = (i < NG) ? ((const T*)L.loT)[(size_t)b * NG + i] : T(0);
    hi = (i < NG) ? ((const T*)L.hiT)[(size_t)b * NG + i] : T(0);
    bd = (L.bdT && i < NX) ? ((const T*)L.bdT)[(size_t)b * NX + i] : T(0);
  }
};

// Data of one stage for the forward sweep (prefetched PF stages ahead).
template <typename T, int NX, int NU, int NG, bool TI>
struct FwdStage {
  static constexpr int n = NX + NU;
  T Lr[n], Mr[n];                // row `lane` of Linv_t, M_t
  T x, yf, zg, yg, bd, q;        // state of stage t; y_f and c of dynamics row t
  T AmC[TI ? 1 : NX], ApC[TI ? 1 : NX], GC[TI ? 1 : NG];  // time-varying columns
};

template <typename T, int NX, int NU, int NG, bool TI>
__device__ __forceinline__ void load_fwd(FwdStage<T, NX, NU, NG, TI>& d, const Layout& L, const Group& g, int t) {
  constexpr int n = NX + NU;
  const size_t nn = (size_t)n * n;
  const int i = g.lane;
  const int64_t s = g.s0 + t;
  const size_t sv = (size_t)s * ROW + i;
  load_row<n>(d.Lr, (const T*)L.LinvT + (size_t)s * nn + (size_t)i * n, i < n);
  load_row<n>(d.Mr, (const T*)L.MT + (size_t)s * nn + (size_t)i * n, i < n && t > 0);
  d.x = (i < n) ? ((const T*)L.x)[sv] : T(0);
  d.yf = (i < NX && t < g.N) ? ((const T*)L.yf)[sv + ROW] : T(0);
  d.zg = (i < NG) ? ((const T*)L.zg)[sv] : T(0);
  d.yg = (i < NG) ? ((const T*)L.yg)[sv] : T(0);
  d.q = (L.qT && i < n) ? ((const T*)L.qT)[(size_t)s * n + i] : T(0);
  if constexpr (!TI) {
    d.bd = (L.bdT && i < NX && t < g.N) ? ((const T*)L.bdT)[(size_t)s * NX + i] : T(0);
    load_col<NX>(d.AmC, (const T*)L.AmT + (size_t)s * NX * n + i, n, i < n && t < g.N);
    load_col<NX>(d.ApC, (const T*)L.ApT + (size_t)s * NX * n + i, n, i < n && t < g.N);
    load_col<NG>(d.GC, (const T*)L.GT + (size_t)s * NG * n + i, n, i < n);
  }
}

// Data of one stage for the backward sweep.
template <typename T, int NX, int NU, int NG, bool TI>
struct BwdStage {
  static constexpr int n = NX + NU;
  T Lc[n], Mc[n];                // column `lane` of Linv_t and of M_{t+1}
  T v, x, zg, yg, yf;            // state of stage t; y_f of dynamics row t
  T lo, hi, bd;                  // time-varying bounds / c
  T AmR[TI ? 1 : n], ApR[TI ? 1 : n], GR[TI ? 1 : n];
};

template <typename T, int NX, int NU, int NG, bool TI>
__device__ __forceinline__ void load_bwd(BwdStage<T, NX, NU, NG, TI>& d, const Layout& L, const Group& g, int t) {
  constexpr int n = NX + NU;
  const size_t nn = (size_t)n * n;
  const int i = g.lane;
  const int64_t s = g.s0 + t;
  const size_t sv = (size_t)s * ROW + i;
  load_row<n>(d.Lc, (const T*)L.LinvTr + (size_t)s * nn + (size_t)i * n, i < n);
  load_row<n>(d.Mc, (const T*)L.MTr + (size_t)(s + 1) * nn + (size_t)i * n, i < n && t < g.N);
  d.v = (i < n) ? ((const T*)L.v)[sv] : T(0);
  d.x = (i < n) ? ((const T*)L.x)[sv] : T(0);
  d.zg = (i < NG) ? ((const T*)L.zg)[sv] : T(0);
  d.yg = (i < NG) ? ((const T*)L.yg)[sv] : T(0);
  d.yf = (i < NX && t < g.N) ? ((const T*)L.yf)[sv + ROW] : T(0);
  if constexpr (!TI) {
    d.lo = (i < NG) ? ((const T*)L.loT)[(size_t)s * NG + i] : T(0);
    d.hi = (i < NG) ? ((const T*)L.hiT)[(size_t)s * NG + i] : T(0);
    d.bd = (L.bdT && i < NX && t < g.N) ? ((const T*)L.bdT)[(size_t)s * NX + i] : T(0);
    load_row<n>(d.AmR, (const T*)L.AmT + (size_t)s * NX * n + (size_t)i * n, i < NX && t < g.N);
    load_row<n>(d.ApR, (const T*)L.ApT + (size_t)s * NX * n + (size_t)i * n, i < NX && t < g.N);
    load_row<n>(d.GR, (const T*)L.GT + (size_t)s * NG * n + (size_t)i * n, i < NG);
  }
}

// prefetch distance (stages) of both sweeps: a 4-deep register ring, halved
// for FP64 at n > 8 to stay within the register file
template <typename T, int n>
constexpr int prefetch_depth() {
  return (sizeof(T) == 8 && n > 8) ? 2 : 4;
}

template <typename T, int NX, int NU, int NG, typename ST>
__device__ void admm_iteration(const Layout& L, const Group& g, const TIBlocks<T, NX, NU, NG>& tb, T sigma,
                               T rho_f, T rho_g, T alpha, int kind, T gamma2, T gamma1) {
  constexpr int n = NX + NU;
  constexpr bool TI = ST::TI;
  constexpr int PF = prefetch_depth<T, n>();
  const int i = g.lane;
  const int b = g.b;
  const int N = g.N;
  T* __restrict__ X = (T*)L.x;
  T* __restrict__ V = (T*)L.v;
  T* __restrict__ YF = (T*)L.yf;
  T* __restrict__ ZG = (T*)L.zg;
  T* __restrict__ YG = (T*)L.yg;
  T* __restrict__ XI = (T*)L.xi;
  const T xinit = (i < NX) ? ((const T*)L.xinitT)[(size_t)b * NX + i] : T(0);
  const int gsel = L.gsel[i < NG ? i : 0];
  const int ginv = L.ginv[i];

  // ---------------- forward sweep ----------------
  {
    FwdStage<T, NX, NU, NG, TI> buf[PF];
    sfor<0, PF>([&](auto k) {
      if (decltype(k)::value <= N) load_fwd(buf[decltype(k)::value], L, g, decltype(k)::value);
    });
    T vprev = T(0), wprev = T(0);
    T ApCprev[TI ? 1 : NX];
    if constexpr (!TI) {
#pragma unroll
      for (int r = 0; r < NX; ++r) ApCprev[r] = T(0);
    }
    for (int t0 = 0; t0 <= N; t0 += PF) {
      sfor<0, PF>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const int t = t0 + k;
        if (t <= N) {
          FwdStage<T, NX, NU, NG, TI>& d = buf[k];
          const int64_t s = g.s0 + t;
          T eta = sigma * d.x - d.q;
          T w = T(0);
          if (t < N) {
            const T bdv = TI ? tb.bd : d.bd;
            w = (i < NX) ? rho_f * bdv - d.yf : T(0);
            if constexpr (TI) eta = dotb<NX>(tb.AmC, w, eta);
            else eta = dotb<NX>(d.AmC, w, eta);
          }
          if (t > 0) {
            if constexpr (ST::APNEG) {
              if (i < NX) eta -= wprev;
            } else if constexpr (TI) {
              eta = dotb<NX>(tb.ApC, wprev, eta);
            } else {
              eta = dotb<NX>(ApCprev, wprev, eta);
            }
          }
          if (t == 0 && i < NX) eta += rho_f * xinit - ((const T*)YF)[(size_t)s * ROW + i];
          const T u = (i < NG) ? rho_g * d.zg - d.yg : T(0);
          if constexpr (ST::GSEL) {
            const T gu = row_gather(u, ginv < 0 ? 0 : ginv);
            if (ginv >= 0) eta += gu;
          } else if constexpr (TI) {
            eta = dotb<NG>(tb.GC, u, eta);
          } else {
            eta = dotb<NG>(d.GC, u, eta);
          }
          if (t > 0) eta -= dotb<n>(d.Mr, vprev, T(0));
          const T vv = dotb<n>(d.Lr, eta, T(0));
          if (i < n) V[(size_t)s * ROW + i] = vv;
          vprev = vv;
          wprev = w;
          if constexpr (!TI) {
#pragma unroll
            for (int r = 0; r < NX; ++r) ApCprev[r] = d.ApC[r];
          }
          if (t + PF <= N) load_fwd(d, L, g, t + PF);
        }
      });
    }
  }

  // ---------------- backward sweep + constraint-row updates ----------------
  {
    BwdStage<T, NX, NU, NG, TI> buf[PF];
    sfor<0, PF>([&](auto k) {
      if (N - decltype(k)::value >= 0) load_bwd(buf[decltype(k)::value], L, g, N - decltype(k)::value);
    });
    T xnext = T(0);
    const T oma = T(1) - alpha;
    for (int t0 = N; t0 >= 0; t0 -= PF) {
      sfor<0, PF>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const int t = t0 - k;
        if (t >= 0) {
          BwdStage<T, NX, NU, NG, TI>& d = buf[k];
          const int64_t s = g.s0 + t;
          const size_t sv = (size_t)s * ROW + i;
          T vv = d.v;
          if (t < N) vv -= dotb<n>(d.Mc, xnext, T(0));
          const T xt = dotb<n>(d.Lc, vv, T(0));
          if (t < N) {  // dynamics row t:  y_f += rho_f alpha (A^- x~_t + A^+ x~_{t+1} - c_t)
            T zf;
            if constexpr (TI) zf = dotb<n>(tb.AmR, xt, T(0));
            else zf = dotb<n>(d.AmR, xt, T(0));
            if constexpr (ST::APNEG) {
              zf -= xnext;
            } else if constexpr (TI) {
              zf = dotb<n>(tb.ApR, xnext, zf);
            } else {
              zf = dotb<n>(d.ApR, xnext, zf);
            }
            if (i < NX) YF[sv + ROW] = d.yf + rho_f * alpha * (zf - (TI ? tb.bd : d.bd));
          }
          T zt;
          if constexpr (ST::GSEL) {
            zt = row_gather(xt, gsel);
          } else if constexpr (TI) {
            zt = dotb<n>(tb.GR, xt, T(0));
          } else {
            zt = dotb<n>(d.GR, xt, T(0));
          }
          if (i < NG) {  // inequality rows of stage t
            const T zh = alpha * zt + oma * d.zg;
            const Proj<T> p = project_row<T>(zh + d.yg / rho_g, TI ? tb.lo : d.lo, TI ? tb.hi : d.hi, kind, rho_g,
                                             gamma2, gamma1);
            ZG[sv] = p.z;
            XI[sv] = p.xi;
            YG[sv] = d.yg + rho_g * (zh - p.z);
          }
          if (i < n) X[sv] = alpha * xt + oma * d.x;
          if (t == 0 && i < NX) YF[sv] += rho_f * alpha * (xt - xinit);
          xnext = xt;
          if (t - PF >= 0) load_bwd(d, L, g, t - PF);
        }
      });
    }
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

constexpr int32_t ST_RUNNING = -1;

// Per-instance start of a solve: status, counters, rho; zero state on a cold
// start.  One thread per padded state entry (and per instance for scalars).
template <typename T>
__global__ void admm_init_kernel(Layout L, Settings st, int32_t* __restrict__ need) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < L.B) {
    L.status[k] = ST_RUNNING;
    L.iters[k] = 0;
    L.nfact[k] = 0;
    need[k] = 1;
    if (!st.warm || !(L.rho[k] > 0.0)) L.rho[k] = st.rho0;
    L.rprim[k] = INFINITY;
    L.rdual[k] = INFINITY;
  }
  if (!st.warm && k < L.stage_off[L.B] * ROW) {
    ((T*)L.x)[k] = T(0);
    ((T*)L.yf)[k] = T(0);
    ((T*)L.zg)[k] = T(0);
    ((T*)L.yg)[k] = T(0);
    ((T*)L.xi)[k] = T(0);
  }
}

__device__ __forceinline__ bool row_group(const Layout& L, Group& g) {
  g.lane = threadIdx.x & (ROW - 1);
  const int slot = blockIdx.x * ROWS_PER_WAVE + (threadIdx.x >> 4);
  if (slot >= L.B) return false;
  g.b = L.order ? L.order[slot] : slot;
  g.s0 = L.stage_off[g.b];
  g.N = (int)(L.stage_off[g.b + 1] - g.s0) - 1;
  return true;
}

// FP64 factorisation of every running instance whose rho changed.
template <typename T, int NX, int NU, int NG>
__global__ __launch_bounds__(64) void admm_factor_kernel(Layout L, Settings st, int32_t* __restrict__ need) {
  Group g;
  if (!row_group(L, g)) return;
  if (L.status[g.b] != ST_RUNNING || !need[g.b]) return;
  const double rho_bar = L.rho[g.b];
  const int bad = factor_instance<T, NX, NU, NG>(L, g, st.sigma, st.rho_f_scale * rho_bar, rho_bar, nullptr);
  if (g.lane == 0) {
    need[g.b] = 0;
    if (bad)
      L.status[g.b] = 3;
    else
      L.nfact[g.b] += 1;
  }
}

// ADMM iterations of every running instance up to iteration `kend` (the next
// stopping-test / rho-adaptation boundary or the cap).
template <typename T, int NX, int NU, int NG, typename ST>
__global__ __launch_bounds__(64) void admm_iter_kernel(Layout L, Settings st, int kend) {
  Group g;
  if (!row_group(L, g)) return;
  if (L.status[g.b] != ST_RUNNING) return;
  const int i = g.lane;
  const int kind = (i < NG) ? (int)L.soft[i] : 0;
  const double rho_bar = L.rho[g.b];
  TIBlocks<T, NX, NU, NG> tb;
  if constexpr (ST::TI) tb.load(L, g.b, i);
  int k = L.iters[g.b];
  for (; k < kend; ++k)
    admm_iteration<T, NX, NU, NG, ST>(L, g, tb, T(st.sigma), T(st.rho_f_scale * rho_bar), T(rho_bar), T(st.alpha),
                                      kind, T(L.gamma2), T(L.gamma1));
  if (i == 0) L.iters[g.b] = k;
}

// At a boundary: FP64 residuals (eq. admm:residuals), the stopping test
// (eq. admm:termination:slack) when `check`, the rho candidate (eq.
// rho:update) when `adapt` (an accepted candidate marks the instance for
// refactorisation), the iteration-cap status when `last`.
template <typename T, int NX, int NU, int NG>
__global__ __launch_bounds__(64) void admm_check_kernel(Layout L, Settings st, int32_t* __restrict__ need, int check,
                                                        int adapt, int last) {
  Group g;
  if (!row_group(L, g)) return;
  if (L.status[g.b] != ST_RUNNING) return;
  const int i = g.lane;
  const int kind = (i < NG) ? (int)L.soft[i] : 0;
  double rho_bar = L.rho[g.b];
  int status = ST_RUNNING;
  const Resid R = residuals<T, NX, NU, NG>(L, g, kind, L.gamma2, L.gamma1);
  if (R.nonfinite) {
    status = 2;
  } else {
    const bool conv = R.rp <= st.eps_abs + st.eps_rel * R.ps && R.rd <= st.eps_abs + st.eps_rel * R.ds;
    if ((check || (st.k_check > 0 && last)) && conv) {
      status = 0;
    } else if (last) {
      status = 1;
    } else if (adapt && !conv) {
      const double num = R.rp / fmax(R.ps, 1e-30);
      const double den = R.rd / fmax(R.ds, 1e-30);
      double cand = rho_bar * sqrt(num / fmax(den, 1e-30));
      cand = fmin(fmax(cand, st.rho_min), st.rho_max);
      if (fmax(cand / rho_bar, rho_bar / cand) > st.k_ratio) {
        rho_bar = cand;
        if (i == 0) need[g.b] = 1;
      }
    }
  }
  if (i == 0) {
    L.rho[g.b] = rho_bar;
    L.status[g.b] = status;
    L.rprim[g.b] = R.rp;
    L.rdual[g.b] = R.rd;
  }
}

}  // namespace ocpk
