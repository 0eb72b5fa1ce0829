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

// Constants of the slack update for one rho_g (see oracle/admm.py `project`):
// L2 rows z = c_v v + c_p Pi(v), xi = c_v (Pi(v) - v) with c_v = rho/(g2+rho),
// c_p = g2/(g2+rho); L1 rows xi = shrink(Pi(v) - v, kappa), kappa = g1/rho.
template <typename T>
struct ProjConst {
  T inv_rho, cv, cp, kap;
  __device__ ProjConst(T rho_g, T gamma2, T gamma1)
      : inv_rho(T(1) / rho_g), cv(rho_g / (gamma2 + rho_g)), cp(gamma2 / (gamma2 + rho_g)), kap(gamma1 / rho_g) {}
};

template <typename T>
__device__ __forceinline__ Proj<T> project_row(T v, T lo, T hi, int kind, const ProjConst<T>& c) {
  const T pv = clampv(v, lo, hi);
  Proj<T> p{pv, T(0)};
  if (kind == 1) {
    p.z = c.cv * v + c.cp * pv;
    p.xi = c.cv * (pv - v);
  } else if (kind == 2) {
    const T d = pv - v;
    p.xi = d - clampv(d, -c.kap, c.kap);
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

// Per-row base pointers of the per-iteration data, advanced one stage at a
// time.  Lanes past the block height read a valid row (their results are
// never broadcast or stored).
template <typename T, int NX, int NU, int NG>
struct StagePtrs {
  static constexpr int n = NX + NU;
  const T *Lr, *Mr, *Lc, *Mc;      // factor rows (Linv, M) and transposed rows
  const T *AmC, *ApC, *GC;         // column `lane` of the time-varying blocks
  const T *AmR, *ApR, *GR;         // row `lane` of the time-varying blocks
  const T *lo, *hi, *bd, *q;
  T *x, *v, *yf, *zg, *yg, *xi;    // padded state of stage t (y_f: slot of stage t)
  __device__ StagePtrs(const Layout& L, const Group& g) {
    const size_t nn = (size_t)n * n;
    const int i = g.lane;
    const int ir = i < n ? i : n - 1;
    const int ix = i < NX ? i : NX - 1;
    const int ig = i < NG ? i : NG - 1;
    const int64_t s0 = g.s0;
    Lr = (const T*)L.LinvT + (size_t)s0 * nn + (size_t)ir * n;
    Mr = (const T*)L.MT + (size_t)s0 * nn + (size_t)ir * n;
    Lc = (const T*)L.LinvTr + (size_t)s0 * nn + (size_t)ir * n;
    Mc = (const T*)L.MTr + (size_t)s0 * nn + (size_t)ir * n;
    AmC = (const T*)L.AmT + (size_t)s0 * NX * n + ir;
    ApC = (const T*)L.ApT + (size_t)s0 * NX * n + ir;
    GC = (const T*)L.GT + (size_t)s0 * NG * n + ir;
    AmR = (const T*)L.AmT + (size_t)s0 * NX * n + (size_t)ix * n;
    ApR = (const T*)L.ApT + (size_t)s0 * NX * n + (size_t)ix * n;
    GR = (const T*)L.GT + (size_t)s0 * NG * n + (size_t)ig * n;
    lo = (const T*)L.loT + (size_t)s0 * NG + ig;
    hi = (const T*)L.hiT + (size_t)s0 * NG + ig;
    bd = L.bdT ? (const T*)L.bdT + (size_t)s0 * NX + ix : nullptr;
    q = L.qT ? (const T*)L.qT + (size_t)s0 * n + ir : nullptr;
    const size_t sv = (size_t)s0 * ROW + i;
    x = (T*)L.x + sv;
    v = (T*)L.v + sv;
    yf = (T*)L.yf + sv;
    zg = (T*)L.zg + sv;
    yg = (T*)L.yg + sv;
    xi = (T*)L.xi + sv;
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
__device__ __forceinline__ void load_fwd(FwdStage<T, NX, NU, NG, TI>& d, const StagePtrs<T, NX, NU, NG>& p, int t,
                                         int N) {
  constexpr int n = NX + NU;
  const size_t nn = (size_t)n * n;
  const size_t o = (size_t)t * nn;
  load_row<n>(d.Lr, p.Lr + o, true);
  load_row<n>(d.Mr, p.Mr + o, t > 0);
  d.x = p.x[(size_t)t * ROW];
  d.yf = p.yf[(size_t)t * ROW];  // dynamics row t (slot N holds the initial-state rows)
  d.zg = p.zg[(size_t)t * ROW];
  d.yg = p.yg[(size_t)t * ROW];
  d.q = p.q ? p.q[(size_t)t * n] : T(0);
  if constexpr (!TI) {
    d.bd = p.bd ? p.bd[(size_t)t * NX] : T(0);
    load_col<NX>(d.AmC, p.AmC + (size_t)t * NX * n, n, true);
    load_col<NX>(d.ApC, p.ApC + (size_t)t * NX * n, n, true);
    load_col<NG>(d.GC, p.GC + (size_t)t * NG * n, n, true);
  }
  (void)N;
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
__device__ __forceinline__ void load_bwd(BwdStage<T, NX, NU, NG, TI>& d, const StagePtrs<T, NX, NU, NG>& p, int t,
                                         int N) {
  constexpr int n = NX + NU;
  const size_t nn = (size_t)n * n;
  load_row<n>(d.Lc, p.Lc + (size_t)t * nn, true);
  load_row<n>(d.Mc, p.Mc + (size_t)(t + 1) * nn, t < N);
  d.v = p.v[(size_t)t * ROW];
  d.x = p.x[(size_t)t * ROW];
  d.zg = p.zg[(size_t)t * ROW];
  d.yg = p.yg[(size_t)t * ROW];
  d.yf = p.yf[(size_t)t * ROW];
  if constexpr (!TI) {
    d.lo = p.lo[(size_t)t * NG];
    d.hi = p.hi[(size_t)t * NG];
    d.bd = p.bd ? p.bd[(size_t)t * NX] : T(0);
    load_row<n>(d.AmR, p.AmR + (size_t)t * NX * n, true);
    load_row<n>(d.ApR, p.ApR + (size_t)t * NX * n, true);
    load_row<n>(d.GR, p.GR + (size_t)t * NG * n, true);
  }
}

// prefetch distance (stages) of both sweeps: a 4-deep register ring, halved
// for FP64 at n > 8 to stay within the register file
template <typename T, int n>
constexpr int prefetch_depth() {
  return (sizeof(T) == 8 && n > 8) ? 2 : 4;
}

template <typename T, int NX, int NU, int NG, typename ST>
__device__ void admm_iteration(const Layout& L, const Group& g, const TIBlocks<T, NX, NU, NG>& tb,
                               const StagePtrs<T, NX, NU, NG>& P, T sigma, T rho_f, T rho_g, T alpha, int kind,
                               const ProjConst<T>& pc, T xinit, T yinit_rho) {
  constexpr int n = NX + NU;
  constexpr bool TI = ST::TI;
  constexpr int PF = prefetch_depth<T, n>();
  const int i = g.lane;
  const int N = g.N;
  const int gsel = L.gsel[i < NG ? i : 0];
  const int ginv = L.ginv[i];
  (void)yinit_rho;

  // ---------------- forward sweep ----------------
  // Branch-free stage bodies: boundary terms multiply zeros (M_0 and the
  // stage after N are zero slots; w and the A^+ term vanish at the ends).
  const T yinit = P.yf[(size_t)N * ROW];  // initial-state multipliers (slot N)
  {
    FwdStage<T, NX, NU, NG, TI> buf[PF];
    sfor<0, PF>([&](auto k) { load_fwd(buf[decltype(k)::value], P, min((int)decltype(k)::value, N), N); });
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
          T eta = sigma * d.x - d.q;
          const T w = (t < N && i < NX) ? rho_f * (TI ? tb.bd : d.bd) - d.yf : T(0);
          if constexpr (TI) eta = dotb<NX>(tb.AmC, w, eta);
          else eta = dotb<NX>(d.AmC, w, eta);
          if constexpr (ST::APNEG) {
            eta -= (i < NX) ? wprev : T(0);
          } else if constexpr (TI) {
            eta = dotb<NX>(tb.ApC, wprev, eta);
          } else {
            eta = dotb<NX>(ApCprev, wprev, eta);
          }
          eta += (t == 0 && i < NX) ? rho_f * xinit - yinit : T(0);
          const T u = (i < NG) ? rho_g * d.zg - d.yg : T(0);
          if constexpr (ST::GSEL) {
            const T gu = row_gather(u, ginv < 0 ? 0 : ginv);
            eta += (ginv >= 0) ? gu : T(0);
          } else if constexpr (TI) {
            eta = dotb<NG>(tb.GC, u, eta);
          } else {
            eta = dotb<NG>(d.GC, u, eta);
          }
          eta -= dotb<n>(d.Mr, vprev, T(0));
          const T vv = dotb<n>(d.Lr, eta, T(0));
          P.v[(size_t)t * ROW] = vv;
          vprev = vv;
          wprev = w;
          if constexpr (!TI) {
#pragma unroll
            for (int r = 0; r < NX; ++r) ApCprev[r] = d.ApC[r];
          }
          load_fwd(d, P, min(t + PF, N), N);
        }
      });
    }
  }

  // ---------------- backward sweep + constraint-row updates ----------------
  {
    BwdStage<T, NX, NU, NG, TI> buf[PF];
    sfor<0, PF>([&](auto k) { load_bwd(buf[decltype(k)::value], P, max(N - (int)decltype(k)::value, 0), N); });
    T xnext = T(0);
    const T oma = T(1) - alpha;
    const T rfa = rho_f * alpha;
    for (int t0 = N; t0 >= 0; t0 -= PF) {
      sfor<0, PF>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const int t = t0 - k;
        if (t >= 0) {
          BwdStage<T, NX, NU, NG, TI>& d = buf[k];
          const size_t o = (size_t)t * ROW;
          const T vv = d.v - dotb<n>(d.Mc, xnext, T(0));  // M_{N+1} is a zero slot
          const T xt = dotb<n>(d.Lc, vv, T(0));
          // dynamics row t:  y_f += rho_f alpha (A^- x~_t + A^+ x~_{t+1} - c_t)
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
          P.yf[o] = (t < N) ? d.yf + rfa * (zf - (TI ? tb.bd : d.bd)) : d.yf;
          // inequality rows of stage t (lanes past ng update padding)
          T zt;
          if constexpr (ST::GSEL) {
            zt = row_gather(xt, gsel);
          } else if constexpr (TI) {
            zt = dotb<n>(tb.GR, xt, T(0));
          } else {
            zt = dotb<n>(d.GR, xt, T(0));
          }
          const T zh = alpha * zt + oma * d.zg;
          const Proj<T> pr = project_row<T>(fma(d.yg, pc.inv_rho, zh), TI ? tb.lo : d.lo, TI ? tb.hi : d.hi, kind,
                                            pc);
          P.zg[o] = pr.z;
          P.xi[o] = pr.xi;
          P.yg[o] = d.yg + rho_g * (zh - pr.z);
          P.x[o] = alpha * xt + oma * d.x;
          xnext = xt;
          load_bwd(d, P, max(t - PF, 0), N);
        }
      });
    }
    // initial-state rows: y_init += rho_f alpha (x~_0 - x_init)
    if (i < NX) P.yf[(size_t)N * ROW] = yinit + rfa * (xnext - xinit);
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
    const double yfc = (t < N && i < NX) ? double(YF[sv]) : 0.0;
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
    if (t == 0 && i < NX) aty += double(YF[(size_t)(g.s0 + N) * ROW + i]);
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
  const int slot = row_slot();
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
  const int bad = L.ti ? factor_instance<T, NX, NU, NG, true>(L, g, st.sigma, st.rho_f_scale * rho_bar, rho_bar, nullptr)
                       : factor_instance<T, NX, NU, NG, false>(L, g, st.sigma, st.rho_f_scale * rho_bar, rho_bar,
                                                               nullptr);
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
  const StagePtrs<T, NX, NU, NG> P(L, g);
  const ProjConst<T> pc(T(rho_bar), T(L.gamma2), T(L.gamma1));
  const T xinit = ((const T*)L.xinitT)[(size_t)g.b * NX + (i < NX ? i : 0)];
  int k = L.iters[g.b];
  for (; k < kend; ++k)
    admm_iteration<T, NX, NU, NG, ST>(L, g, tb, P, T(st.sigma), T(st.rho_f_scale * rho_bar), T(rho_bar),
                                      T(st.alpha), kind, pc, xinit, T(0));
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
