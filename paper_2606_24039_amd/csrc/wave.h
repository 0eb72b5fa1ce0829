// ADMM iteration of Algorithm 3 with one instance per wavefront.
//
// The 64 lanes form four 16-lane rows.  Work that is independent across
// stages runs on four stages at once (stage t on row t mod 4); the two block
// substitutions of S x~ = eta are serial chains over the horizon and run on
// row 0 alone, one n-row matrix-vector product per stage, over the blocks the
// factorisation prepares (factor.h: Linv/W/V for FP32 iterations, P/K for
// FP64):
//
//   pass 1  rows   eta_t = sigma x_t - q_t + A_t^-'w_t + A_{t-1}^+'w_{t-1}
//                          + [t=0](rho_f x_init - y_init) + G_t'(rho_g z_t - y_t),
//                  w_t = rho_f c_t - y_f,t;  r_t = Linv_t eta_t (FP32) or eta_t
//   pass 2  row 0  v_t  = r_t - W_t v_{t-1}   (K_t)          (t = 0..N)
//   pass 3  rows   s_t  = Linv_t' v_t         (P_t v_t)
//   pass 4  row 0  x~_t = s_t - V_t x~_{t+1}  (Kb_t)         (t = N..0)
//   pass 5  rows   over-relaxation, projection and dual update of every
//                  constraint row of stage t from x~_t and x~_{t+1}
//
// The passes hand vectors to other lanes through the per-instance buffer v
// and are separated by workgroup barriers (the workgroup is the one
// wavefront).
#pragma once

#include "admm.h"

namespace ocpk {

struct WaveGroup {
  int lane;  // 0..15 within the row
  int row;   // 0..3
  int b;
  int64_t s0;
  int N;
};

__device__ __forceinline__ bool wave_group(const Layout& L, WaveGroup& w) {
  w.lane = threadIdx.x & (ROW - 1);
  w.row = threadIdx.x >> 4;
  const int slot = blockIdx.x;
  if (slot >= L.B) return false;
  w.b = L.order ? L.order[slot] : slot;
  w.s0 = L.stage_off[w.b];
  w.N = (int)(L.stage_off[w.b + 1] - w.s0) - 1;
  return true;
}

// pass-1 inputs of the stage on this row
template <typename T, int NX, int NU, int NG, bool TI>
struct EtaIn {
  static constexpr int n = NX + NU;
  static constexpr bool SA = sizeof(T) == 4;  // FP32 iterations multiply by Linv_t here
  T Ar[SA ? n : 1];                           // row `lane` of SubA
  T x, q, yf, yfm, zg, yg, bd, bdm;
  T AmC[TI ? 1 : NX], ApCm[TI ? 1 : NX], GC[TI ? 1 : NG];
};

// t may run up to STAGE_PAD - 1 stages past N: the padded state and factor
// buffers are read unclamped, the exactly sized problem data at min(t, N)
template <typename T, int NX, int NU, int NG, bool TI>
__device__ __forceinline__ void load_eta(EtaIn<T, NX, NU, NG, TI>& d, const StagePtrs<T, NX, NU, NG>& p, int t,
                                         int N) {
  constexpr int n = NX + NU;
  const int tc = min(t, N);
  const int tm = tc > 0 ? tc - 1 : 0;
  if constexpr (EtaIn<T, NX, NU, NG, TI>::SA) load_row<n>(d.Ar, p.SAr + (long)t * n * n, true);
  d.x = p.x[(long)t * ROW];
  d.q = p.q ? p.q[(size_t)tc * n] : T(0);
  d.yf = p.yf[(long)t * ROW];
  d.yfm = p.yf[(long)(t - 1) * ROW];
  d.zg = p.zg[(long)t * ROW];
  d.yg = p.yg[(long)t * ROW];
  if constexpr (!TI) {
    d.bd = p.bd ? p.bd[(size_t)tc * NX] : T(0);
    d.bdm = p.bd ? p.bd[(size_t)tm * NX] : T(0);
    load_col<NX>(d.AmC, p.AmC + (size_t)tc * NX * n, n, true);
    load_col<NX>(d.ApCm, p.ApC + (size_t)tm * NX * n, n, true);
    load_col<NG>(d.GC, p.GC + (size_t)tc * NG * n, n, true);
  }
}

// pass-3 inputs: row `lane` of SubB and v_t
template <typename T, int n>
struct TrIn {
  T Br[n];
  T v;
};

// pass-5 inputs of the stage on this row
template <typename T, int NX, int NU, int NG, bool TI>
struct UpdIn {
  static constexpr int n = NX + NU;
  T xt, xt1;  // x~_t, x~_{t+1}
  T x, yf, zg, yg, lo, hi, bd;
  T AmR[TI ? 1 : n], ApR[TI ? 1 : n], GR[TI ? 1 : n];
};

template <typename T, int NX, int NU, int NG, bool TI>
__device__ __forceinline__ void load_upd(UpdIn<T, NX, NU, NG, TI>& d, const StagePtrs<T, NX, NU, NG>& p,
                                         gptr<const T> R, int t, int N) {
  constexpr int n = NX + NU;
  const int tc = min(t, N);
  d.xt = R[(long)t * ROW];
  d.xt1 = (t < N) ? R[(long)(t + 1) * ROW] : T(0);
  d.x = p.x[(long)t * ROW];
  d.yf = p.yf[(long)t * ROW];
  d.zg = p.zg[(long)t * ROW];
  d.yg = p.yg[(long)t * ROW];
  if constexpr (!TI) {
    d.lo = p.lo[(size_t)tc * NG];
    d.hi = p.hi[(size_t)tc * NG];
    d.bd = p.bd ? p.bd[(size_t)tc * NX] : T(0);
    load_row<n>(d.AmR, p.AmR + (size_t)tc * NX * n, true);
    load_row<n>(d.ApR, p.ApR + (size_t)tc * NX * n, true);
    load_row<n>(d.GR, p.GR + (size_t)tc * NG * n, true);
  }
}

// the state part of the pass-5 inputs (x~ comes from elsewhere); t may lie
// up to STAGE_PAD stages outside 0..N (padded state read unclamped, problem
// data at the nearest stage)
template <typename T, int NX, int NU, int NG, bool TI>
__device__ __forceinline__ void load_upd_state(UpdIn<T, NX, NU, NG, TI>& d, const StagePtrs<T, NX, NU, NG>& p, int t,
                                               int N) {
  constexpr int n = NX + NU;
  const int tc = t < 0 ? 0 : (t > N ? N : t);
  d.x = p.x[(long)t * ROW];
  d.yf = p.yf[(long)t * ROW];
  d.zg = p.zg[(long)t * ROW];
  d.yg = p.yg[(long)t * ROW];
  if constexpr (!TI) {
    d.lo = p.lo[(size_t)tc * NG];
    d.hi = p.hi[(size_t)tc * NG];
    d.bd = p.bd ? p.bd[(size_t)tc * NX] : T(0);
    load_row<n>(d.AmR, p.AmR + (size_t)tc * NX * n, true);
    load_row<n>(d.ApR, p.ApR + (size_t)tc * NX * n, true);
    load_row<n>(d.GR, p.GR + (size_t)tc * NG * n, true);
  }
}

// chain inputs of one stage: row `lane` of a chain block and one vector entry
template <typename T, int n>
struct ChainIn {
  T A[n];
  T r;
};

template <typename T, int n>
__device__ __forceinline__ void load_chain(ChainIn<T, n>& d, gptr<const T> a, gptr<const T> r) {
#pragma unroll
  for (int k = 0; k < n; ++k) d.A[k] = a[k];
  d.r = *r;
}

__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// One substitution chain on row 0: y_t = R[t] - B_t y_prev over the stages
// in `dir` order (+1: 0..N with B = ChF; -1: N..0 with B = ChB); y_t -> R[t].
template <typename T, int n, int DIR>
__device__ __forceinline__ void chain(gptr<T> R, gptr<const T> Bm, int N) {
  constexpr int PF = chain_prefetch<T, n>();
  static_assert(PF <= STAGE_PAD, "prefetch reaches past the buffer padding");
  constexpr long dB = DIR * (long)n * n;  // block stride of one step of the sweep
  constexpr long dR = DIR * (long)ROW;
  // running pointers at the sweep's k0-th stage (t = 0 forward, t = N
  // backward); prefetches run up to PF stages past either end of the
  // instance, into the neighbouring instances or the padding
  gptr<const T> Bk = Bm + (DIR > 0 ? 0 : (long)N * n * n);
  gptr<T> Rk = R + (DIR > 0 ? 0 : (long)N * ROW);
  ChainIn<T, n> buf[PF];
  sfor<0, PF>([&](auto j) {
    constexpr int jj = decltype(j)::value;
    load_chain(buf[jj], Bk + jj * dB, Rk + jj * dR);
  });
  T yprev = T(0);
  auto body = [&](auto j) {
    constexpr int jj = decltype(j)::value;
    ChainIn<T, n>& d = buf[jj];
    const T y = d.r - dotb<n>(d.A, yprev, T(0));  // stage 0 / N chain blocks are zero slots
    Rk[jj * dR] = y;
    yprev = y;
    load_chain(d, Bk + (jj + PF) * dB, Rk + (jj + PF) * dR);
  };
  int k0 = 0;
  for (; k0 + PF - 1 <= N; k0 += PF) {
    sfor<0, PF>(body);
    Bk += PF * dB;
    Rk += PF * dR;
  }
  sfor<0, PF>([&](auto j) {
    if (k0 + decltype(j)::value <= N) body(j);
  });
}

// Scalars of one ADMM iteration of one instance (this lane's view).
template <typename T, int NX, int NU, int NG, typename ST>
struct IterCtx {
  const TIBlocks<T, NX, NU, NG>& tb;
  const StagePtrs<T, NX, NU, NG>& P;
  T sigma, rho_f, rho_g, alpha, oma, rfa;
  int kind;
  ProjConst<T> pc;
  T xinit, yinit;
  int gsel, ginv;
  int i, N;
};

// r_t of the stage on this row: eta_t, times Linv_t for FP32 iterations
template <typename T, int NX, int NU, int NG, typename ST>
__device__ __forceinline__ T stage_r(const IterCtx<T, NX, NU, NG, ST>& c, const EtaIn<T, NX, NU, NG, ST::TI>& cur,
                                     int t) {
  constexpr int n = NX + NU;
  constexpr bool TI = ST::TI;
  const int i = c.i, N = c.N;
  const auto& tb = c.tb;
  T eta = c.sigma * cur.x - cur.q;
  const T w_ = (t < N && i < NX) ? c.rho_f * (TI ? tb.bd : cur.bd) - cur.yf : T(0);
  const T wm = (t > 0 && i < NX) ? c.rho_f * (TI ? tb.bd : cur.bdm) - cur.yfm : T(0);
  if constexpr (TI)
    eta = dotb<NX>(tb.AmC, w_, eta);
  else
    eta = dotb<NX>(cur.AmC, w_, eta);
  if constexpr (ST::APNEG) {
    eta -= wm;
  } else if constexpr (TI) {
    eta = dotb<NX>(tb.ApC, wm, eta);
  } else {
    eta = dotb<NX>(cur.ApCm, wm, eta);
  }
  eta += (t == 0 && i < NX) ? c.rho_f * c.xinit - c.yinit : T(0);
  const T u = (i < NG) ? c.rho_g * cur.zg - cur.yg : T(0);
  if constexpr (ST::GSEL) {
    const T gu = row_gather(u, c.ginv < 0 ? 0 : c.ginv);
    eta += (c.ginv >= 0) ? gu : T(0);
  } else if constexpr (TI) {
    eta = dotb<NG>(tb.GC, u, eta);
  } else {
    eta = dotb<NG>(cur.GC, u, eta);
  }
  if constexpr (EtaIn<T, NX, NU, NG, TI>::SA)
    return dotb<n>(cur.Ar, eta, T(0));
  else
    return eta;
}

// over-relaxation, projection and dual update of every constraint row of
// the stage on this row, from x~_t and x~_{t+1}
template <typename T, int NX, int NU, int NG, typename ST>
__device__ __forceinline__ void stage_update(const IterCtx<T, NX, NU, NG, ST>& c,
                                             const UpdIn<T, NX, NU, NG, ST::TI>& cur, T xt, T xt1, int t) {
  constexpr int n = NX + NU;
  constexpr bool TI = ST::TI;
  const int i = c.i, N = c.N;
  const auto& tb = c.tb;
  const auto& P = c.P;
  const size_t o = (size_t)t * ROW;
  // dynamics row t: y_f += rho_f alpha (A^- x~_t + A^+ x~_{t+1} - c_t)
  T zf;
  if constexpr (TI)
    zf = dotb<n>(tb.AmR, xt, T(0));
  else
    zf = dotb<n>(cur.AmR, xt, T(0));
  if constexpr (ST::APNEG) {
    zf -= xt1;
  } else if constexpr (TI) {
    zf = dotb<n>(tb.ApR, xt1, zf);
  } else {
    zf = dotb<n>(cur.ApR, xt1, zf);
  }
  if (t < N) P.yf[o] = cur.yf + c.rfa * (zf - (TI ? tb.bd : cur.bd));
  // inequality rows of stage t (lanes past ng update padding)
  T zt;
  if constexpr (ST::GSEL)
    zt = row_gather(xt, c.gsel);
  else if constexpr (TI)
    zt = dotb<n>(tb.GR, xt, T(0));
  else
    zt = dotb<n>(cur.GR, xt, T(0));
  const T zh = c.alpha * zt + c.oma * cur.zg;
  const Proj<T> pr =
      project_row<T>(fma(cur.yg, c.pc.inv_rho, zh), TI ? tb.lo : cur.lo, TI ? tb.hi : cur.hi, c.kind, c.pc);
  P.zg[o] = pr.z;
  P.xi[o] = pr.xi;
  P.yg[o] = cur.yg + c.rho_g * (zh - pr.z);
  P.x[o] = c.alpha * xt + c.oma * cur.x;
  // initial-state rows: y_init += rho_f alpha (x~_0 - x_init)
  if (t == 0 && i < NX) P.yf[(size_t)N * ROW] = c.yinit + c.rfa * (xt - c.xinit);
}

// One iteration on one wavefront (the vectors handed between passes go
// through the instance's v buffer in global memory).
template <typename T, int NX, int NU, int NG, typename ST>
__device__ __forceinline__ void wave_iteration(const IterCtx<T, NX, NU, NG, ST>& c, int q) {
  constexpr int n = NX + NU;
  constexpr bool TI = ST::TI;
  const int N = c.N;
  const int nbl = (N + 4) / 4;  // 4-stage blocks covering 0..N
  const size_t nn = (size_t)n * n;
  const auto& P = c.P;
  const gptr<T> R = P.v;  // per-lane base of the exchange buffer

  // ---------------- pass 1: r_t on row t mod 4 ----------------
  {
    EtaIn<T, NX, NU, NG, TI> cur, nxt;
    load_eta(cur, P, q, N);  // stages past N read padding or the next instance (unused)
    for (int blk = 0; blk < nbl; ++blk) {
      const int t = 4 * blk + q;
      load_eta(nxt, P, t + 4, N);
      if (t <= N) R[(size_t)t * ROW] = stage_r(c, cur, t);
      cur = nxt;
    }
  }
  wave_sync();

  // ---------------- pass 2: forward chain (row 0) ----------------
  if (q == 0) chain<T, n, +1>(R, P.CFr, N);
  wave_sync();

  // ---------------- pass 3: s_t = SubB_t v_t on row t mod 4 ----------------
  {
    TrIn<T, n> cur, nxt;
    auto load_tr = [&](TrIn<T, n>& d, int t) {
      load_row<n>(d.Br, P.SBr + (size_t)t * nn, true);
      d.v = R[(size_t)t * ROW];
    };
    load_tr(cur, q);
    for (int blk = 0; blk < nbl; ++blk) {
      const int t = 4 * blk + q;
      load_tr(nxt, t + 4);
      if (t <= N) R[(size_t)t * ROW] = dotb<n>(cur.Br, cur.v, T(0));
      cur = nxt;
    }
  }
  wave_sync();

  // ---------------- pass 4: backward chain (row 0) ----------------
  if (q == 0) chain<T, n, -1>(R, P.CBr, N);
  wave_sync();

  // ---------------- pass 5: constraint-row updates on row t mod 4 ----------------
  {
    UpdIn<T, NX, NU, NG, TI> cur, nxt;
    load_upd(cur, P, R, q, N);
    for (int blk = 0; blk < nbl; ++blk) {
      const int t = 4 * blk + q;
      load_upd(nxt, P, R, t + 4, N);
      if (t <= N) stage_update(c, cur, cur.xt, cur.xt1, t);
      cur = nxt;
    }
  }
  wave_sync();
}

}  // namespace ocpk

namespace ocpk {

// max over the four rows (every lane receives the result)
template <typename T>
__device__ __forceinline__ T rows_max(T v) {
  v = fmax(v, (T)__shfl_xor(v, 16));
  v = fmax(v, (T)__shfl_xor(v, 32));
  return v;
}

// FP64 residuals of eq. admm:residuals and the scales of eq.
// admm:termination:slack with the stages spread over the four rows (stage t
// on row t mod 4); every row reads the neighbouring stages it needs directly.
// TI: the blocks are the same at every stage and are read once.
template <typename T, int NX, int NU, int NG, bool TI, int TAG = 0>
__device__ __noinline__ Resid residuals_wave(const Layout& L, const WaveGroup& w, int kind, double gamma2,
                                             double gamma1) {
  constexpr int n = NX + NU;
  const int i = w.lane, q = w.row, b = w.b, N = w.N;
  const int ic = i < n ? i : n - 1, ix = i < NX ? i : NX - 1, ig = i < NG ? i : NG - 1;
  const size_t nn = (size_t)n * n;
  const gptr<const T> X = as_global((const T*)L.x);
  const gptr<const T> YF = as_global((const T*)L.yf);
  const gptr<const T> ZG = as_global((const T*)L.zg);
  const gptr<const T> YG = as_global((const T*)L.yg);
  const gptr<const T> XI = as_global((const T*)L.xi);
  double m_cxc = 0, m_cx = 0, m_c = 0, m_gxz = 0, m_gx = 0, m_z = 0;
  double m_dual = 0, m_px = 0, m_aty = 0, m_q = 0, m_sres = 0, m_sscale = 0;
  int nf = 0;
  auto upd = [&](double& m, double v) {
    if (!isfinite(v)) nf = 1;
    m = fmax(m, fabs(v));
  };
  // blocks of stage t (TI: read once, the terminal D_N separately)
  double Dr[n], DrN[TI ? n : 1], Ec[n], Er[n], Amc[NX], Apc[NX], Amr[n], Apr[n], Gc[NG], Gr[n], cv = 0.0;
  auto load_blocks = [&](int t, int64_t s) {
    const double* Dp = TI ? L.D + (size_t)(2 * b) * nn : L.D + (size_t)s * nn;
    load_row<n>(Dr, Dp + (size_t)ic * n, true);
    if constexpr (TI) load_row<n>(DrN, Dp + nn + (size_t)ic * n, true);
    const size_t ob = ti_or_tv(TI, b, s, (size_t)NX * n);
    load_col<NX>(Amc, L.Am + ob + ic, n, true);
    load_row<n>(Amr, L.Am + ob + (size_t)ix * n, true);
    load_row<n>(Apr, L.Ap + ob + (size_t)ix * n, true);
    const size_t og = ti_or_tv(TI, b, s, (size_t)NG * n);
    load_col<NG>(Gc, L.G + og + ic, n, true);
    load_row<n>(Gr, L.G + og + (size_t)ig * n, true);
    if (L.E) {
      load_col<n>(Ec, L.E + ti_or_tv(TI, b, s, nn) + ic, n, true);
      load_row<n>(Er, L.E + ti_or_tv(TI, b, s, nn) + (size_t)ic * n, true);
    }
    cv = L.bd ? as_global(L.bd)[ti_or_tv(TI, b, s, NX) + ix] : 0.0;
    (void)t;
  };
  if constexpr (TI) {
    load_blocks(0, w.s0);
    load_col<NX>(Apc, L.Ap + (size_t)b * NX * n + ic, n, true);
  }
  const double yinit = double(YF[(size_t)(w.s0 + N) * ROW + i]);
  const double xi0 = as_global(L.x_init)[(size_t)b * NX + ix];
  const int nbl = (N + 4) / 4;
  for (int blk = 0; blk < nbl; ++blk) {
    const int t = 4 * blk + q;
    if (t > N) break;
    const int64_t s = w.s0 + t;
    const size_t sv = (size_t)s * ROW + i;
    const double xc = double(X[sv]);
    const double xm = (t > 0) ? double(X[sv - ROW]) : 0.0;
    const double xn = (t < N) ? double(X[sv + ROW]) : 0.0;
    const double yfc = (t < N && i < NX) ? double(YF[sv]) : 0.0;
    const double yfm = (t > 0 && i < NX) ? double(YF[sv - ROW]) : 0.0;
    if constexpr (!TI) {
      load_blocks(t, s);
      if (t > 0)
        load_col<NX>(Apc, L.Ap + (size_t)(s - 1) * NX * n + ic, n, true);
      else
#pragma unroll
        for (int r = 0; r < NX; ++r) Apc[r] = 0.0;
    }
    // (P x)_t row i = D_t x_t + E_{t-1} x_{t-1} + E_t' x_{t+1}
    double px;
    if constexpr (TI) {
      double dN[n];
#pragma unroll
      for (int k = 0; k < n; ++k) dN[k] = (t == N) ? DrN[k] : Dr[k];
      px = dotb<n>(dN, xc, 0.0);
    } else {
      px = dotb<n>(Dr, xc, 0.0);
    }
    if (L.E) {
      double Em[n];  // row i of E_{t-1}
      if constexpr (TI) {
#pragma unroll
        for (int k = 0; k < n; ++k) Em[k] = Er[k];
      } else {
        load_row<n>(Em, L.E + (size_t)(t > 0 ? s - 1 : s) * nn + (size_t)ic * n, true);
      }
      const double xm_ = (t > 0) ? xm : 0.0;
      px = dotb<n>(Em, xm_, px);
      const double xn_ = (t < N) ? xn : 0.0;
      px = dotb<n>(Ec, xn_, px);
    }
    // (A' y)_t row i
    double aty = dotb<NX>(Amc, yfc, 0.0);
    aty = dotb<NX>(Apc, yfm, aty);
    if (t == 0 && i < NX) aty += yinit;
    const double ygv = (i < NG) ? double(YG[sv]) : 0.0;
    aty = dotb<NG>(Gc, ygv, aty);
    const double qv = (L.q && i < n) ? as_global(L.q)[(size_t)s * n + i] : 0.0;
    if (i < n) {
      upd(m_dual, px + qv + aty);
      upd(m_px, px);
      upd(m_aty, aty);
      upd(m_q, qv);
    }
    // equality rows touching stage t
    if (t == 0 && i < NX) {
      upd(m_cxc, xc - xi0);
      upd(m_cx, xc);
      upd(m_c, xi0);
    }
    double cx = dotb<n>(Amr, xc, 0.0);
    cx = dotb<n>(Apr, xn, cx);
    if (t < N && i < NX) {
      upd(m_cxc, cx - cv);
      upd(m_cx, cx);
      upd(m_c, cv);
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
  }
  Resid R;
  R.rp = rows_max(row_max(fmax(m_cxc, m_gxz)));
  R.ps = rows_max(row_max(fmax(fmax(m_cx, m_gx), fmax(m_c, m_z))));
  R.rd = rows_max(row_max(fmax(m_dual, m_sres)));
  R.ds = rows_max(row_max(fmax(fmax(m_px, m_aty), fmax(m_q, m_sscale))));
  R.nonfinite = rows_max(row_max(nf));
  return R;
}

// Boundary decision of the schedule (eq. admm:termination:slack, rho:update):
// returns the new status (ST_RUNNING to continue) and may change rho_bar.
__device__ __forceinline__ int boundary_decision(const Resid& R, const Settings& st, int check, int adapt, int last,
                                                 double& rho_bar, bool& refactor) {
  refactor = false;
  if (R.nonfinite) return 2;
  const bool conv = R.rp <= st.eps_abs + st.eps_rel * R.ps && R.rd <= st.eps_abs + st.eps_rel * R.ds;
  if ((check || (st.k_check > 0 && last)) && conv) return 0;
  if (last) return 1;
  if (adapt && !conv) {
    const double num = R.rp / fmax(R.ps, 1e-30);
    const double den = R.rd / fmax(R.ds, 1e-30);
    double cand = rho_bar * sqrt(num / fmax(den, 1e-30));
    cand = fmin(fmax(cand, st.rho_min), st.rho_max);
    if (fmax(cand / rho_bar, rho_bar / cand) > st.k_ratio) {
      rho_bar = cand;
      refactor = true;
    }
  }
  return ST_RUNNING;
}

// One complete ADMM solve per wavefront (Algorithm 3 with the stopping test
// and rho adaptation): FP64 factorisation, iterations up to each boundary,
// FP64 residuals and decisions at the boundary, refactorisation after an
// accepted rho change.  Instances never wait for each other.
template <typename T, int NX, int NU, int NG, typename ST>
__global__ __launch_bounds__(64) void admm_solve_wave_kernel(Layout L, Settings st) {
  WaveGroup w;
  if (!wave_group(L, w)) return;
  if (L.status[w.b] != ST_RUNNING) return;
  const int i = w.lane;
  const Group g{w.lane, w.b, w.s0, w.N};
  const int kind = (i < NG) ? (int)L.soft[i] : 0;
  double rho_bar = L.rho[w.b];
  int nfact = L.nfact[w.b];
  int status = ST_RUNNING;
  Resid R{INFINITY, INFINITY, 0.0, 0.0, 0};

  // time-invariant blocks (ST::TI) are exactly the handles whose factor
  // products can be hoisted
  const bool adapt_on = st.adapt_rho && st.k_rho > 0;
  int k = L.iters[w.b];
  bool need = true;
  for (;;) {
    if (need) {  // the only call site of the factorisation
      constexpr int FORM = sizeof(T) == 4 ? FACTOR_WV : FACTOR_PK;
      const int bad = factor_instance<T, NX, NU, NG, ST::TI, FORM>(L, g, st.sigma, st.rho_f_scale * rho_bar,
                                                                   rho_bar, nullptr, w.row);
      wave_sync();
      if (bad) {
        status = 3;
        break;
      }
      ++nfact;
      need = false;
    }
    if (k >= st.max_iter) break;
    int nb = st.max_iter;
    if (st.k_check > 0) nb = min(nb, (k / st.k_check + 1) * st.k_check);
    if (adapt_on) nb = min(nb, (k / st.k_rho + 1) * st.k_rho);
    {
      TIBlocks<T, NX, NU, NG> tb;
      if constexpr (ST::TI) tb.load(L, w.b, i);
      const StagePtrs<T, NX, NU, NG> P(L, g);
      const ProjConst<T> pc(T(rho_bar), T(L.gamma2), T(L.gamma1));
      const T xinit = ((const T*)L.xinitT)[(size_t)w.b * NX + (i < NX ? i : 0)];
      const T rho_f = T(st.rho_f_scale * rho_bar), alpha = T(st.alpha);
      const IterCtx<T, NX, NU, NG, ST> c{tb,          P,           T(st.sigma),        rho_f, T(rho_bar), alpha,
                                         T(1) - alpha, rho_f * alpha, kind,          pc,    xinit,      T(0),
                                         L.gsel[i < NG ? i : 0],   L.ginv[i],          i,     w.N};
      for (; k < nb; ++k) {
        IterCtx<T, NX, NU, NG, ST> ck = c;
        ck.yinit = P.yf[(size_t)w.N * ROW];  // initial-state multipliers (slot N)
        wave_iteration<T, NX, NU, NG, ST>(ck, w.row);
      }
    }
    const int check = (st.k_check > 0 && nb % st.k_check == 0) ? 1 : 0;
    const int adapt = (adapt_on && nb % st.k_rho == 0 && nb < st.max_iter) ? 1 : 0;
    const int last = (nb == st.max_iter) ? 1 : 0;
    if (check || adapt || last) {
      R = residuals_wave<T, NX, NU, NG, ST::TI>(L, w, kind, L.gamma2, L.gamma1);
      status = boundary_decision(R, st, check, adapt, last, rho_bar, need);
      if (status != ST_RUNNING) break;
    }
  }
  if (threadIdx.x == 0) {
    L.iters[w.b] = k;
    L.nfact[w.b] = nfact;
    L.rho[w.b] = rho_bar;
    L.status[w.b] = status;
    L.rprim[w.b] = R.rp;
    L.rdual[w.b] = R.rd;
  }
}

}  // namespace ocpk
