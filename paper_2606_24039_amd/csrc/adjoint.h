// Implicit-differentiation adjoint (Algorithm 2; Sec. "Backward Pass";
// Appendix "Backward Pass: Sensitivities Computation"), FP64 throughout, one
// instance per wavefront in the layout of the ADMM solve (wave.h): work that
// is independent across stages runs on four stages at once (stage t on row
// t mod 4), the block substitutions are serial chains on row 0.
//
// 1. Active set (Appendix, "Active constraints identification"): the dual
//    sign decides (y < -eps_g lower, y > eps_g upper); closeness to a bound is
//    used only when |y| < eps_g.  eps_g = 10 eps_active max(1, ||y_g||_inf);
//    proximity tolerance 10 eps_active max(1, |bound|) (relative to the bound,
//    not to the multipliers).  L1-slack rows with nonzero slack keep their
//    fixed multiplier and are not active.
// 2. The KKT matrix of the active-set conditions (eq. bwd:noslack_kkt_matrix)
//      K = [[H, J'], [J, 0]],  J = [C; G_A]
//    has a zero (2,2) block and no Schur form.  Its regularisation
//      K_reg = [[H + sigma_b I, J'], [J, -rho_b^{-1} I]]
//    does: (H + sigma_b I + rho_b J'J) d_x = r_x + rho_b J' r_y,
//    d_y = rho_b (J d_x - r_y), and H + sigma_b I + rho_b J'J is block
//    tridiagonal, factored by the solve's block Cholesky (P/K form, FP64)
//    with rho_f = rho_b and per-row inequality weights rho_b [row active].
//    Iterative refinement e <- e + K_reg^{-1}(r - K e) with the residual in
//    FP64 converges to K^{-1} r (the regularisation is a perturbation of
//    size max(sigma_b, 1/rho_b)); at most refine_sweeps corrections (fewer
//    once ||r - K e||_inf / ||dL/dx||_inf is below adj_tol / 100), then the
//    final residual ||r - K e||_inf / ||dL/dx||_inf is compared with adj_tol
//    for the per-instance status.
// 3. VJP (eq. loss_gradient): dL/dq = -eta_x, dL/dx_init = eta_f(initial
//    rows), dL/dD_t[i,i] = -eta_x,t,i x_t,i, dL/dlo = eta_g on lower-active
//    rows, dL/dhi = eta_g on upper-active rows.
//
// Equality-row vectors (e_f, r_f) use the output slot convention: the
// initial-state rows at stage 0, dynamics row t at stage t + 1.
#pragma once

#include "ocp_admm.h"
#include "wave.h"

namespace ocpk {

struct AdjArgs {
  const double* dLdx;   // [S][n] (the effective right-hand side dl below when dLdxi is given)
  const double* dLdxi;  // [S][ng] loss gradient w.r.t. the slacks; may be null
  double* dl;           // [S][n] scratch: dL/dx - G_S' dL/dxi (eq. bwd:slack_reduced_system)
  double sigma_b, rho_b, eps_active;
  int sweeps;
  int chunk_min_n;  // horizons from which the factorisation runs chunked
  // scratch, FP64 padded [S][ROW] (v carries STAGE_PAD padding stages)
  double* w;    // inequality-row weights (rho_b on active rows)
  double* ex;   // eta_x
  double* ef;   // eta_f
  double* eg;   // eta_g
  double* rf;   // equality-row residual of the current sweep
  double* rg;   // inequality-row residual of the current sweep
  double* v;    // exchange buffer of the substitution passes
  int8_t* act;  // -1 lower, +1 upper, 0 inactive
  // factor of the regularised Schur matrix, FP64 P/K form (factor.h), padded
  double *P, *K, *Kb;
  // outputs (FP64, may be null)
  double *d_q, *d_Ddiag, *d_x_init, *d_lo, *d_hi, *eta_x, *d_gamma2;
  int8_t* active;
  double *eta_f, *eta_g, *adj_resid;
  int32_t* adj_status;
  double *eta_xi, *d_gamma1;
  double adj_tol;  // relative KKT residual accepted as refined
  double stop_res;  // the sweeps stop once ||r - K e||_inf <= stop_res (set per instance; 0: all sweeps)
};

// Blocks of stage t a row needs for the products with H, C and G (FP64).
template <int NX, int NU, int NG>
struct AdjBlocks {
  static constexpr int n = NX + NU;
  double Dr[n];           // row i of D_t
  double Er[n], Ec[n];    // row i of E_{t-1}, column i of E_t
  double Amc[NX], Apcm[NX];  // column i of A_t^-, of A_{t-1}^+
  double Amr[n], Apr[n];  // row i of A_t^-, A_t^+
  double Amrm[n], Aprm[n];   // row i of A_{t-1}^-, A_{t-1}^+
  double Gc[NG], Gr[n];   // column i, row i of G_t
};

template <int NX, int NU, int NG>
__device__ __forceinline__ void load_adj_blocks(AdjBlocks<NX, NU, NG>& d, const Layout& L, int b, int64_t s0,
                                                int t, int N, int i) {
  constexpr int n = NX + NU;
  const size_t nn = (size_t)n * n;
  const int ic = i < n ? i : n - 1, ix = i < NX ? i : NX - 1, ig = i < NG ? i : NG - 1;
  const int64_t s = s0 + t;
  const int64_t sm = s0 + (t > 0 ? t - 1 : 0);
  const double* Dp = L.ti ? L.D + (size_t)(2 * b + (t == N ? 1 : 0)) * nn : L.D + (size_t)s * nn;
  load_row<n>(d.Dr, Dp + (size_t)ic * n, true);
  if (L.E) {
    load_row<n>(d.Er, L.E + ti_or_tv(L.ti, b, sm, nn) + (size_t)ic * n, t > 0);
    load_col<n>(d.Ec, L.E + ti_or_tv(L.ti, b, s, nn) + ic, n, t < N);
  } else {
#pragma unroll
    for (int k = 0; k < n; ++k) d.Er[k] = d.Ec[k] = 0.0;
  }
  const size_t oa = ti_or_tv(L.ti, b, s, (size_t)NX * n), oam = ti_or_tv(L.ti, b, sm, (size_t)NX * n);
  load_col<NX>(d.Amc, L.Am + oa + ic, n, t < N);
  load_col<NX>(d.Apcm, L.Ap + oam + ic, n, t > 0);
  load_row<n>(d.Amr, L.Am + oa + (size_t)ix * n, t < N);
  load_row<n>(d.Apr, L.Ap + oa + (size_t)ix * n, t < N);
  load_row<n>(d.Amrm, L.Am + oam + (size_t)ix * n, t > 0);
  load_row<n>(d.Aprm, L.Ap + oam + (size_t)ix * n, t > 0);
  const size_t og = ti_or_tv(L.ti, b, s, (size_t)NG * n);
  load_col<NG>(d.Gc, L.G + og + ic, n, true);
  load_row<n>(d.Gr, L.G + og + (size_t)ig * n, true);
}

// pass-1 inputs of one stage of a sweep (time-invariant data)
struct AdjIn1 {
  double ec, em, en, efc, efr, wc, eg, dl;
};
// pass-5 inputs
struct AdjIn5 {
  double dx, dn, efn, rfn, wc, eg, rg, ef0, rf0, ex;
};

// Refinement sweeps for time-invariant data (the blocks of AdjTI), with the
// explicit-dynamics and selection structure of ST.  Passes as in the general
// sweep below; stage inputs are loaded two blocks ahead (stage_blocks).  The
// unpadded FP64 scratch vectors are read at stages clamped to 0..N (the
// clamped values are never used).
template <int NX, int NU, int NG, typename ST>
__device__ __forceinline__ double adjoint_sweeps_ti(const Layout& L, const AdjArgs& a, const WaveGroup& w, int bad) {
  constexpr int n = NX + NU;
  constexpr uint32_t VS = ROW * sizeof(double);
  const int i = w.lane, q = w.row, N = w.N;
  const int64_t s0 = w.s0;
  const int ic = i < n ? i : n - 1;
  const int nfull = N / 4;
  const double rb = a.rho_b;
  // rescaled QP: the loss gradient w.r.t. xh = x / d is d * dL/dx
  const double dls = L.sc ? L.sc[(size_t)w.b * 3 * ROW + i] : 1.0;
  TIBlocks64<NX, NU, NG, ST> tb;
  tb.load(L, w.b, i);
  const bool hasE = L.E != nullptr;
  const int gsel = L.gsel[i < NG ? i : 0], ginv = L.ginv[i];
  const bool gid = __ballot(i < NG && gsel != i) == 0;
  // L2-slack row (eq. bwd:slack_reduced_system): when active it sits in H as
  // gamma2 G_i'G_i (its weight in w is gamma2) instead of in J
  const bool slr = i < NG && L.soft[i] == 1;
  auto gather_t = [&](double u) { return gid ? u : row_gather(u, ginv < 0 ? 0 : ginv); };  // G' u (lane i)
  auto gather = [&](double u) { return gid ? u : row_gather(u, gsel); };                    // G u (row i)
  // instance bases (uniform) and lane offsets
  const gptr<double> ex = as_global(a.ex) + s0 * ROW, ef = as_global(a.ef) + s0 * ROW;
  const gptr<double> eg = as_global(a.eg) + s0 * ROW, rf = as_global(a.rf) + s0 * ROW;
  const gptr<double> rg = as_global(a.rg) + s0 * ROW, wv = as_global(a.w) + s0 * ROW;
  const gptr<const double> dL = as_global(a.dLdx) + s0 * n;
  const gptr<double> Rb = as_global(a.v) + (s0 - STAGE_PAD) * ROW;
  const int64_t nn = (int64_t)n * n;
  const gptr<const double> Pb = as_global((const double*)a.P) + (s0 - STAGE_PAD) * nn;
  const gptr<const double> Kb0 = as_global((const double*)a.K) + (s0 - STAGE_PAD) * nn;
  const gptr<const double> Kbb0 = as_global((const double*)a.Kb) + (s0 - STAGE_PAD) * nn;
  const uint32_t orow = (uint32_t)((STAGE_PAD * ROW + i) * (int)sizeof(double));
  const uint32_t oblk = (uint32_t)((STAGE_PAD * (int)nn + ic * n) * (int)sizeof(double));
  // offset of entry `lane` of stage t of the unpadded vectors, t clamped to 0..N
  auto ov = [&](int t) { return (uint32_t)((min(max(t, 0), N) * ROW + i) * (int)sizeof(double)); };
  // of the padded exchange buffer (no clamping needed within the padding)
  auto oR = [&](int t) { return (uint32_t)(((STAGE_PAD + t) * ROW + i) * (int)sizeof(double)); };

  // this lane's part of ||r - K e||_inf; the pass after the last sweep only
  // evaluates it
  double rres = 0.0;
  for (int sweep = 0; sweep <= a.sweeps && !bad; ++sweep) {
    rres = 0.0;
    // pass 1: residual r - K e and the Schur right-hand side
    //   rhs_t = r_x,t + rho_b (C' r_f)_t + G'(w .* r_g,t)
    {
      auto load = [&](AdjIn1& d, int blk) {
        const int t = 4 * blk + q;
        const uint32_t o = ov(t);
        d.ec = ldo(ex, o);
        d.em = ldo(ex, ov(t - 1));
        d.en = ldo(ex, ov(t + 1));
        d.efc = ldo(ef, ov(t + 1));  // dynamics row t
        d.efr = ldo(ef, o);          // dynamics row t-1, or the initial-state rows at t = 0
        d.wc = ldo(wv, o);
        d.eg = ldo(eg, o);
        d.dl = ldo(dL, (uint32_t)((min(t, N) * n + ic) * (int)sizeof(double))) * dls;
      };
      auto comp = [&](const AdjIn1& d, int blk, auto full) {
        constexpr bool FULL = decltype(full)::value;
        const int t = 4 * blk + q;
        const bool xr = i < NX, tlo = t > 0, thi = FULL || t < N;
        const double ec = (i < n) ? d.ec : 0.0;
        const double em = (tlo && i < n) ? d.em : 0.0;
        const double en = (thi && i < n) ? d.en : 0.0;
        // H e_x
        double he = dotb<n>(tb.Dr, ec, 0.0);
        if (!FULL && t == N) he = dotb<n>(tb.dDN, ec, he);
        if (hasE) {
          he = dotb<n>(tb.Er, em, he);
          he = dotb<n>(tb.Ec, en, he);
        }
        // J' e_y
        const double efc = (thi && xr) ? d.efc : 0.0;
        const double efm = (tlo && xr) ? d.efr : 0.0;
        double jte = dotb<NX>(tb.Amc, efc, 0.0);
        if constexpr (ST::APNEG)
          jte -= efm;
        else
          jte = dotb<NX>(tb.Apc, efm, jte);
        jte += (t == 0 && xr) ? d.efr : 0.0;  // initial-state rows
        const double wc = (i < NG) ? d.wc : 0.0;
        const bool slk = slr && wc != 0.0;
        double gx;
        if constexpr (ST::GSEL)
          gx = gather(ec);
        else
          gx = dotb<n>(tb.Gr, ec, 0.0);
        // J' e_y over the hard active rows, plus the active slack rows' H term G_i'(gamma2 G_i e_x)
        const double egv = (i < NG && wc != 0.0) ? (slk ? wc * gx : d.eg) : 0.0;
        if constexpr (ST::GSEL) {
          const double gt = gather_t(egv);
          jte += (ginv >= 0) ? gt : 0.0;
        } else {
          jte = dotb<NG>(tb.Gc, egv, jte);
        }
        const double rx = ((i < n) ? d.dl : 0.0) - (he + jte);
        // equality-row residuals -J e_x of the rows touching stage t
        double cx = dotb<n>(tb.Amr, ec, 0.0);
        double cxm = dotb<n>(tb.Amr, em, 0.0);
        if constexpr (ST::APNEG) {
          cx -= en;
          cxm -= ec;
        } else {
          cx = dotb<n>(tb.Apr, en, cx);
          cxm = dotb<n>(tb.Apr, ec, cxm);
        }
        const double rfc = (thi && xr) ? -cx : 0.0;   // dynamics row t
        const double rfm = (tlo && xr) ? -cxm : 0.0;  // dynamics row t-1
        const double rf0 = (t == 0 && xr) ? -ec : 0.0;  // initial-state rows
        const double rgc = (wc != 0.0 && !slk) ? -gx : 0.0;
        double tc = dotb<NX>(tb.Amc, rfc, 0.0);
        if constexpr (ST::APNEG)
          tc -= rfm;
        else
          tc = dotb<NX>(tb.Apc, rfm, tc);
        tc += rf0;
        double rhs = rx + rb * tc;
        if constexpr (ST::GSEL) {
          const double gt = gather_t(wc * rgc);
          rhs += (ginv >= 0) ? gt : 0.0;
        } else {
          rhs = dotb<NG>(tb.Gc, wc * rgc, rhs);
        }
        if (FULL || t <= N) {
          const uint32_t o = ov(t);
          if (t == 0 && xr) sto(rf, o, rf0);
          if (thi && xr) sto(rf, o + VS, rfc);
          if (i < NG) sto(rg, o, rgc);
          sto(Rb, oR(t), rhs);
          rres = fmax(rres, fmax(i < n ? fabs(rx) : 0.0, i < NG ? fabs(rgc) : 0.0));
          if (xr) rres = fmax(rres, fmax(fabs(rfc), fabs(rf0)));
        }
      };
      stage_blocks<STAGE_BLOCK_DEPTH, AdjIn1>(nfull, load, comp);
    }
    wave_sync();
    if (sweep == a.sweeps) break;
    // refined before the last sweep: this residual is the final one
    if (rows_max(row_max(rres)) <= a.stop_res) break;
    // passes 2-4: d_x = S^{-1} rhs
    if (q == 0) chain<double, n, +1>(Rb, Kb0, orow, oblk, N);
    wave_sync();
    {
      auto load = [&](TrIn<double, n>& d, int blk) {
        const int t = 4 * blk + q;
        ldo_n<n>(d.Br, Pb + (int64_t)(STAGE_PAD + t) * nn, (uint32_t)(ic * n * (int)sizeof(double)));
        d.v = ldo(Rb, oR(t));
      };
      auto comp = [&](const TrIn<double, n>& d, int blk, auto full) {
        constexpr bool FULL = decltype(full)::value;
        const int t = 4 * blk + q;
        const double r = dotb<n>(d.Br, d.v, 0.0);
        if (FULL || t <= N) sto(Rb, oR(t), r);
      };
      stage_blocks<STAGE_BLOCK_DEPTH, TrIn<double, n>>(nfull, load, comp);
    }
    wave_sync();
    if (q == 0) chain<double, n, -1>(Rb, Kbb0, orow, oblk, N);
    wave_sync();
    // pass 5: d_y = rho_b (J d_x - r_y), e += d
    {
      auto load = [&](AdjIn5& d, int blk) {
        const int t = 4 * blk + q;
        const uint32_t o = ov(t);
        d.dx = ldo(Rb, oR(t));
        d.dn = ldo(Rb, oR(t + 1));
        d.efn = ldo(ef, ov(t + 1));
        d.rfn = ldo(rf, ov(t + 1));
        d.wc = ldo(wv, o);
        d.eg = ldo(eg, o);
        d.rg = ldo(rg, o);
        d.ef0 = ldo(ef, o);
        d.rf0 = ldo(rf, o);
        d.ex = ldo(ex, o);
      };
      auto comp = [&](const AdjIn5& d, int blk, auto full) {
        constexpr bool FULL = decltype(full)::value;
        const int t = 4 * blk + q;
        const bool xr = i < NX, thi = FULL || t < N;
        const double dx = d.dx;
        const double dn = thi ? d.dn : 0.0;
        double jd = dotb<n>(tb.Amr, dx, 0.0);
        if constexpr (ST::APNEG)
          jd -= dn;
        else
          jd = dotb<n>(tb.Apr, dn, jd);
        double gd;
        if constexpr (ST::GSEL)
          gd = gather(dx);
        else
          gd = dotb<n>(tb.Gr, dx, 0.0);
        if (FULL || t <= N) {
          const uint32_t o = ov(t);
          if (thi && xr) sto(ef, o + VS, d.efn + rb * (jd - d.rfn));
          if (i < NG && d.wc != 0.0 && !slr) sto(eg, o, d.eg + rb * (gd - d.rg));
          if (t == 0 && xr) sto(ef, o, d.ef0 + rb * (dx - d.rf0));
          if (i < n) sto(ex, o, d.ex + dx);
        }
      };
      stage_blocks<STAGE_BLOCK_DEPTH, AdjIn5>(nfull, load, comp);
    }
    wave_sync();
  }
  return rres;
}

// Refinement sweeps, time-varying blocks: the same passes as the
// time-invariant form with every stage's blocks read where they are used.
// Stage-parallel passes walk 4-stage blocks with their inputs loaded ahead
// (two blocks ahead for small stages, whose block rows fit the registers;
// inputs are read at stages clamped to 0..N).
template <int n>
constexpr int ADJ_TV_DEPTH = n <= 8 ? STAGE_BLOCK_DEPTH : 1;

template <int NX, int NU, int NG>
struct AdjInTV1 {
  AdjBlocks<NX, NU, NG> B;
  double ec, em, en, efc, efm, ef0, wc, eg, dl;
};
template <int NX, int NU, int NG>
struct AdjInTV5 {
  static constexpr int n = NX + NU;
  double Amr[n], Apr[n], Gr[n];
  double dx, dn, efn, rfn, wc, eg, rg, ef0, rf0, ex;
};

// One substitution chain y_t = r_t - B_t y_prev (DIR +1: t = 0..N, B = K;
// -1: t = N..0, B = Kb; y in place of r in Rv) on R segments, segment q on
// 16-lane row q of a multi-wavefront workgroup: the particular solution of
// each segment from a zero start, the serial pass over the segment ends
// (seg_link, with the segments' transfer blocks TU), then the correction
// d_t = -B_t d_prev from the entering value added in place.
template <int n, int R, int DIR>
__device__ __forceinline__ void adj_seg_chain(gptr<double> Rv, gptr<const double> Bm, lptr<double> X,
                                              lptr<const double> TU, int N, int q, int i) {
  const SegRange sg = seg_range<R>(q, N);
  const int ir = i < n ? i : n - 1;
  const size_t nn = (size_t)n * n;
  auto stage = [&](int k) { return DIR > 0 ? sg.a + k : sg.a + sg.len - 1 - k; };
  // the next step's block row and vector entry are loaded while this one computes
  double Bn[n], rn;
  load_row<n>(Bn, Bm + (size_t)stage(0) * nn + (size_t)ir * n, sg.len > 0);
  rn = sg.len > 0 ? Rv[(size_t)stage(0) * ROW + i] : 0.0;
  double y = 0.0;
  for (int k = 0; k < sg.len; ++k) {
    const int t = stage(k);
    double Br[n];
#pragma unroll
    for (int j = 0; j < n; ++j) Br[j] = Bn[j];
    const double r = rn;
    if (k + 1 < sg.len) {
      load_row<n>(Bn, Bm + (size_t)stage(k + 1) * nn + (size_t)ir * n, true);
      rn = Rv[(size_t)stage(k + 1) * ROW + i];
    }
    y = (i < n) ? r - dotb<n>(Br, y, 0.0) : 0.0;
    Rv[(size_t)t * ROW + i] = y;
  }
  const double in = seg_link<double, n, R>(y, DIR > 0 ? 0 : 1, X, TU, q, i);
  double d = in;
  load_row<n>(Bn, Bm + (size_t)stage(0) * nn + (size_t)ir * n, sg.len > 0);
  for (int k = 0; k < sg.len; ++k) {
    const int t = stage(k);
    double Br[n];
#pragma unroll
    for (int j = 0; j < n; ++j) Br[j] = Bn[j];
    if (k + 1 < sg.len) load_row<n>(Bn, Bm + (size_t)stage(k + 1) * nn + (size_t)ir * n, true);
    d = (i < n) ? -dotb<n>(Br, d, 0.0) : 0.0;
    Rv[(size_t)t * ROW + i] += d;
  }
}

// LDS of a multi-wavefront adjoint: the chains' transfer blocks (forward,
// backward) and exchange slots, and one reduction slot per wavefront
template <int n, int R>
struct AdjMwLds {
  double tu[2 * R * n * n];
  double x[2 * R * ROW];
  double red[R / 4];
};

// cross-wavefront reductions of a multi-wavefront adjoint (R > 4): every
// lane holds its wavefront's value on entry and the workgroup's on return
template <int R, typename F>
__device__ __forceinline__ double adj_block_reduce(double v, double* red, F&& op) {
  if constexpr (R == 4) {
    return v;
  } else {
    constexpr int W = R / 4;
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int k = 1; k < W; ++k) r = op(r, red[k]);
    __syncthreads();  // the slots are reused by the next reduction
    return r;
  }
}

template <int NX, int NU, int NG, int NR = 4>
__device__ __forceinline__ double adjoint_sweeps_tv(const Layout& L, const AdjArgs& a, const WaveGroup& w, int bad,
                                                    bool slr, AdjMwLds<NX + NU, NR>* mw = nullptr) {
  constexpr int n = NX + NU;
  constexpr int D = ADJ_TV_DEPTH<n>;
  const int i = w.lane, q = w.row, N = w.N, b = w.b;
  const int64_t s0 = w.s0;
  const int ic = i < n ? i : n - 1, ix = i < NX ? i : NX - 1, ig = i < NG ? i : NG - 1;
  const int nfull = N / NR;
  const size_t nn = (size_t)n * n;
  const double rb = a.rho_b;
  const double dls = L.sc ? L.sc[(size_t)b * 3 * ROW + i] : 1.0;  // rescaled QP: d * dL/dx
  const gptr<double> ex = as_global(a.ex), ef = as_global(a.ef), eg = as_global(a.eg);
  const gptr<double> rf = as_global(a.rf), rg = as_global(a.rg), wv = as_global(a.w);
  const gptr<double> R = as_global(a.v) + (size_t)s0 * ROW + i;
  const gptr<const double> Pr = as_global((const double*)a.P) + (size_t)s0 * nn + (size_t)ic * n;
  // the chains take bases STAGE_PAD stages before stage 0 and lane offsets
  const int64_t sp = s0 - STAGE_PAD;
  const gptr<double> Rb = as_global(a.v) + sp * ROW;
  const gptr<const double> Kb0 = as_global((const double*)a.K) + sp * (int64_t)nn;
  const gptr<const double> Kbb0 = as_global((const double*)a.Kb) + sp * (int64_t)nn;
  const uint32_t orow = (uint32_t)((STAGE_PAD * ROW + i) * (int)sizeof(double));
  const uint32_t oblk = (uint32_t)((STAGE_PAD * (int)nn + ic * n) * (int)sizeof(double));
  auto tcl = [&](int blk) { return min(NR * blk + q, N); };

  double rres = 0.0;  // this lane's part of ||r - K e||_inf (the pass after the last sweep only evaluates it)
  for (int sweep = 0; sweep <= a.sweeps && !bad; ++sweep) {
    rres = 0.0;
    // pass 1: residual r - K e and the Schur right-hand side
    //   rhs_t = r_x,t + rho_b (C' r_f)_t + G_t'(w .* r_g,t)
    {
      using In = AdjInTV1<NX, NU, NG>;
      auto load = [&](In& d, int blk) {
        const int t = tcl(blk);
        const int64_t s = s0 + t;
        const size_t sv = (size_t)s * ROW + i;
        load_adj_blocks(d.B, L, b, s0, t, N, i);
        d.ec = (i < n) ? ex[sv] : 0.0;
        d.em = (t > 0 && i < n) ? ex[sv - ROW] : 0.0;
        d.en = (t < N && i < n) ? ex[sv + ROW] : 0.0;
        d.efc = (t < N && i < NX) ? ef[sv + ROW] : 0.0;  // dynamics row t
        d.efm = (t > 0 && i < NX) ? ef[sv] : 0.0;        // dynamics row t-1
        d.ef0 = (t == 0 && i < NX) ? ef[sv] : 0.0;       // initial-state rows
        d.wc = (i < NG) ? wv[sv] : 0.0;
        d.eg = (i < NG) ? eg[sv] : 0.0;
        d.dl = (i < n) ? a.dLdx[(size_t)s * n + i] * dls : 0.0;
      };
      auto comp = [&](const In& d, int blk, auto) {
        const int t = NR * blk + q;
        if (t > N) return;  // the same on all lanes of a row
        const int64_t s = s0 + t;
        const size_t sv = (size_t)s * ROW + i;
        const auto& B = d.B;
        // H e_x
        double he = dotb<n>(B.Dr, d.ec, 0.0);
        he = dotb<n>(B.Er, d.em, he);
        he = dotb<n>(B.Ec, d.en, he);
        // J' e_y
        double jte = dotb<NX>(B.Amc, d.efc, 0.0);
        jte = dotb<NX>(B.Apcm, d.efm, jte);
        jte += d.ef0;
        const double wc = d.wc;
        const bool slk = slr && wc != 0.0;
        const double gx = dotb<n>(B.Gr, d.ec, 0.0);
        // J' e_y over the hard active rows, plus the active slack rows' H term G_i'(gamma2 G_i e_x)
        const double egv = (i < NG && wc != 0.0) ? (slk ? wc * gx : d.eg) : 0.0;
        jte = dotb<NG>(B.Gc, egv, jte);
        const double rx = d.dl - (he + jte);
        // equality-row residuals -J e_x of the rows touching stage t
        double cx = dotb<n>(B.Amr, d.ec, 0.0);
        cx = dotb<n>(B.Apr, d.en, cx);
        const double rfc = (t < N && i < NX) ? -cx : 0.0;  // dynamics row t
        double cxm = dotb<n>(B.Amrm, d.em, 0.0);
        cxm = dotb<n>(B.Aprm, d.ec, cxm);
        const double rfm = (t > 0 && i < NX) ? -cxm : 0.0;  // dynamics row t-1
        const double rf0 = (t == 0 && i < NX) ? -d.ec : 0.0;  // initial-state rows
        const double rgc = (wc != 0.0 && !slk) ? -gx : 0.0;
        double tc = dotb<NX>(B.Amc, rfc, 0.0);
        tc = dotb<NX>(B.Apcm, rfm, tc);
        tc += rf0;
        double rhs = rx + rb * tc;
        rhs = dotb<NG>(B.Gc, wc * rgc, rhs);
        if (t == 0 && i < NX) rf[sv] = rf0;
        if (t < N && i < NX) rf[sv + ROW] = rfc;
        if (i < NG) rg[sv] = rgc;
        R[(size_t)t * ROW] = rhs;
        rres = fmax(rres, fmax(i < n ? fabs(rx) : 0.0, i < NG ? fabs(rgc) : 0.0));
        if (i < NX) rres = fmax(rres, fmax(fabs(rfc), fabs(rf0)));
      };
      stage_blocks<D, In>(nfull, load, comp);
    }
    wave_sync();
    if (sweep == a.sweeps) break;
    // refined before the last sweep: this residual is the final one
    const double rmax = adj_block_reduce<NR>(rows_max(row_max(rres)), mw ? mw->red : nullptr,
                                             [](double x, double y) { return fmax(x, y); });
    if (rmax <= a.stop_res) break;
    // passes 2-4: d_x = S^{-1} rhs
    if constexpr (NR == 4) {
      if (q == 0) chain<double, n, +1>(Rb, Kb0, orow, oblk, N);
    } else {
      adj_seg_chain<n, NR, +1>(as_global(a.v) + (size_t)s0 * ROW, as_global((const double*)a.K) + (size_t)s0 * nn,
                              (lptr<double>)mw->x, (lptr<const double>)mw->tu, N, q, i);
    }
    wave_sync();
    {
      auto load = [&](TrIn<double, n>& d, int blk) {
        const int t = tcl(blk);
        load_row<n>(d.Br, Pr + (size_t)t * nn, true);
        d.v = R[(size_t)t * ROW];
      };
      auto comp = [&](const TrIn<double, n>& d, int blk, auto) {
        const int t = NR * blk + q;
        if (t > N) return;
        R[(size_t)t * ROW] = dotb<n>(d.Br, d.v, 0.0);
      };
      stage_blocks<D, TrIn<double, n>>(nfull, load, comp);
    }
    wave_sync();
    if constexpr (NR == 4) {
      if (q == 0) chain<double, n, -1>(Rb, Kbb0, orow, oblk, N);
    } else {
      adj_seg_chain<n, NR, -1>(as_global(a.v) + (size_t)s0 * ROW, as_global((const double*)a.Kb) + (size_t)s0 * nn,
                              (lptr<double>)mw->x, (lptr<const double>)(mw->tu + NR * nn), N, q, i);
    }
    wave_sync();
    // pass 5: d_y = rho_b (J d_x - r_y), e += d
    {
      using In = AdjInTV5<NX, NU, NG>;
      auto load = [&](In& d, int blk) {
        const int t = tcl(blk);
        const int64_t s = s0 + t;
        const size_t sv = (size_t)s * ROW + i;
        const size_t oa = ti_or_tv(L.ti, b, s, (size_t)NX * n);
        load_row<n>(d.Amr, L.Am + oa + (size_t)ix * n, t < N);
        load_row<n>(d.Apr, L.Ap + oa + (size_t)ix * n, t < N);
        load_row<n>(d.Gr, L.G + ti_or_tv(L.ti, b, s, (size_t)NG * n) + (size_t)ig * n, true);
        d.dx = R[(size_t)t * ROW];
        d.dn = (t < N) ? R[(size_t)(t + 1) * ROW] : 0.0;
        d.efn = (t < N && i < NX) ? ef[sv + ROW] : 0.0;
        d.rfn = (t < N && i < NX) ? rf[sv + ROW] : 0.0;
        d.wc = (i < NG) ? wv[sv] : 0.0;
        d.eg = (i < NG) ? eg[sv] : 0.0;
        d.rg = (i < NG) ? rg[sv] : 0.0;
        d.ef0 = (t == 0 && i < NX) ? ef[sv] : 0.0;
        d.rf0 = (t == 0 && i < NX) ? rf[sv] : 0.0;
        d.ex = (i < n) ? ex[sv] : 0.0;
      };
      auto comp = [&](const In& d, int blk, auto) {
        const int t = NR * blk + q;
        if (t > N) return;
        const size_t sv = (size_t)(s0 + t) * ROW + i;
        double jd = dotb<n>(d.Amr, d.dx, 0.0);
        jd = dotb<n>(d.Apr, d.dn, jd);
        if (t < N && i < NX) ef[sv + ROW] = d.efn + rb * (jd - d.rfn);
        const double gd = dotb<n>(d.Gr, d.dx, 0.0);
        if (i < NG && d.wc != 0.0 && !slr) eg[sv] = d.eg + rb * (gd - d.rg);
        if (t == 0 && i < NX) ef[sv] = d.ef0 + rb * (d.dx - d.rf0);
        if (i < n) ex[sv] = d.ex + d.dx;
      };
      stage_blocks<D, In>(nfull, load, comp);
    }
    wave_sync();
  }
  return rres;
}


// The adjoint of one instance on R 16-lane rows: one wavefront (R = 4,
// time-invariant or time-varying data) or a workgroup of R / 4 wavefronts
// (time-varying data; chunked factorisation with R + 1 chunks and chains on
// R segments, FX its exchange blocks, mw its LDS).
template <typename T, int NX, int NU, int NG, typename ST, int R>
__device__ __forceinline__ void adjoint_body(const Layout& L, const AdjArgs& a, const WaveGroup& w, double* FX,
                                             AdjMwLds<NX + NU, R>* mw) {
  constexpr int n = NX + NU;
  static_assert(R == 4 || !ST::TI, "multi-wavefront adjoints take time-varying data");
  const int i = w.lane, q = w.row, b = w.b, N = w.N;
  const int64_t s0 = w.s0;
  const Group g{w.lane, w.b, w.s0, w.N};
  const int nbl = (N + R) / R;
  auto vmax = [](double x, double y) { return fmax(x, y); };
  auto vsum = [](double x, double y) { return x + y; };
  const size_t nn = (size_t)n * n;
  const gptr<const T> X = as_global((const T*)L.x);
  const gptr<const T> YG = as_global((const T*)L.yg);
  const gptr<const T> XI = as_global((const T*)L.xi);
  const gptr<double> ex = as_global(a.ex), ef = as_global(a.ef), eg = as_global(a.eg);
  const gptr<double> rf = as_global(a.rf), rg = as_global(a.rg), wv = as_global(a.w);
  const int kind = (i < NG) ? (int)L.soft[i] : 0;
  const bool slr = kind == 1;  // L2-slack row (in H when active)
  const double rb = a.rho_b;
  // rescaled QP (Remark 4): the active set is judged and the results are
  // returned in the original variables.  Lane factors: d_i (variable), e_i
  // (inequality row), c; all 1 without rescaling.
  const double* scb = L.sc ? L.sc + (size_t)b * 3 * ROW : nullptr;
  const double sd = scb ? scb[i] : 1.0, se = scb ? scb[ROW + i] : 1.0, scc = scb ? scb[2 * ROW] : 1.0;
  const double yw = se / scc;       // y_g = e yh_g / c
  const double exw = scc * sd;      // eta_x = c d etah_x
  const double efw = 1.0 / sd;      // eta_f = etah_f / d_x (lane = state component)

  // ---- 1. active set ----
  double ymax = 0.0, dlmax = 0.0;
  for (int blk = 0; blk < nbl; ++blk) {
    const int t = R * blk + q;
    if (t <= N && i < NG) ymax = fmax(ymax, fabs(double(YG[(size_t)(s0 + t) * ROW + i]) * yw));
    if (t <= N && i < n) dlmax = fmax(dlmax, fabs(a.dLdx[(size_t)(s0 + t) * n + i] * sd));
  }
  ymax = adj_block_reduce<R>(rows_max(row_max(ymax)), mw ? mw->red : nullptr, vmax);
  dlmax = adj_block_reduce<R>(rows_max(row_max(dlmax)), mw ? mw->red : nullptr, vmax);
  const double epsg = 10.0 * a.eps_active * fmax(1.0, ymax);  // dual test, relative to the multipliers
  const double epsp = 10.0 * a.eps_active;                     // proximity test, relative to the bound
  for (int blk = 0; blk < nbl; ++blk) {
    const int t = R * blk + q;
    if (t > N) break;
    const int64_t s = s0 + t;
    const size_t sv = (size_t)s * ROW + i;
    const double xc = (i < n) ? double(X[sv]) : 0.0;
    double Gr[n];
    load_row<n>(Gr, L.G + ti_or_tv(L.ti, b, s, (size_t)NG * n) + (size_t)(i < NG ? i : NG - 1) * n, true);
    const double gx = dotb<n>(Gr, xc, 0.0) / se;
    int act = 0;
    if (i < NG) {
      const size_t sb = ti_or_tv(L.ti, b, s, NG) + i;
      // original-variable row value, bounds and multiplier
      const double lo = L.lo[sb] / se, hi = L.hi[sb] / se, y = double(YG[sv]) * yw;
      const bool amb = fabs(y) < epsg;
      bool lower = (y < -epsg) || (amb && (gx - lo <= epsp * fmax(1.0, fabs(lo))));
      bool upper = (y > epsg) || (amb && (hi - gx <= epsp * fmax(1.0, fabs(hi))));
      if (lower && upper) {
        if (y > 0)
          lower = false;
        else
          upper = false;
      }
      if (kind == 2 && double(XI[sv]) != 0.0) lower = upper = false;
      act = lower ? -1 : (upper ? 1 : 0);
    }
    a.act[sv] = (int8_t)act;
    // active slack rows enter the Schur matrix with their penalty gamma2
    wv[sv] = act ? (kind == 1 ? L.gamma2 : rb) : 0.0;
    ex[sv] = 0.0;
    ef[sv] = 0.0;
    eg[sv] = 0.0;
  }
  wave_sync();
  // loss on the slacks: the rows whose slack moves with x (active L2 rows,
  // L1 rows with nonzero slack xi = bound - G x) contribute -G_i' dL/dxi_i to
  // the right-hand side of the reduced system (eq. bwd:slack_reduced_system)
  AdjArgs ar = a;
  if (a.dLdxi) {
    dlmax = 0.0;
    for (int blk = 0; blk < nbl; ++blk) {
      const int t = R * blk + q;
      if (t > N) break;
      const int64_t s = s0 + t;
      const size_t sv = (size_t)s * ROW + i;
      const bool moves = i < NG && ((kind == 1 && a.act[sv] != 0) || (kind == 2 && double(XI[sv]) != 0.0));
      const double wr = moves ? a.dLdxi[(size_t)s * NG + i] : 0.0;
      double Gc[NG];
      load_col<NG>(Gc, L.G + ti_or_tv(L.ti, b, s, (size_t)NG * n) + (i < n ? i : n - 1), n, true);
      const double e = (i < n ? a.dLdx[(size_t)s * n + i] : 0.0) - dotb<NG>(Gc, wr, 0.0);
      if (i < n) {
        a.dl[(size_t)s * n + i] = e;
        dlmax = fmax(dlmax, fabs(e * sd));
      }
    }
    dlmax = adj_block_reduce<R>(rows_max(row_max(dlmax)), mw ? mw->red : nullptr, vmax);
    wave_sync();
    ar.dLdx = a.dl;
  }

  // ---- 2. factor H + sigma_b I + rho_b (C'C + G_A'G_A) (FP64, P/K form) ----
  Layout LF = L;
  LF.SubB = a.P;
  LF.ChF = a.K;
  LF.ChB = a.Kb;
  int bad;
  if constexpr (R == 4) {
    const bool chunked = g.N >= a.chunk_min_n && g.N >= FAC_CHUNK_MIN_N;
    if (L.ti)
      bad = chunked ? factor_chunked<double, NX, NU, NG, true, FACTOR_PK>(LF, g, a.sigma_b, rb, 0.0, a.w)
                    : factor_instance<double, NX, NU, NG, true, FACTOR_PK>(LF, g, a.sigma_b, rb, 0.0, a.w, q);
    else
      bad = chunked ? factor_chunked<double, NX, NU, NG, false, FACTOR_PK>(LF, g, a.sigma_b, rb, 0.0, a.w)
                    : factor_instance<double, NX, NU, NG, false, FACTOR_PK>(LF, g, a.sigma_b, rb, 0.0, a.w, q);
    wave_sync();
  } else {
    constexpr int nn_ = n * n;
    bad = factor_chunked<double, NX, NU, NG, false, FACTOR_PK, 1, R>(LF, g, a.sigma_b, rb, 0.0, a.w, FX);
    bad = (int)adj_block_reduce<R>((double)bad, mw->red, vmax);
    // transfer blocks of the segmented chains (forward: K, backward: Kb)
    prepare_segments<double, NX, NU, NG, R>(LF, b, s0, N, (lptr<double>)mw->tu, (lptr<double>)(mw->tu + R * nn_));
    __syncthreads();
  }

  // ---- refinement sweeps, then the final FP64 residual ||r - K e||_inf ----
  // (the sweeps end early once the residual is a hundredth of the accepted one)
  ar.stop_res = 1e-2 * a.adj_tol * fmax(dlmax, 1e-300);
  double rres;
  if constexpr (ST::TI) {
    rres = adjoint_sweeps_ti<NX, NU, NG, ST>(L, ar, w, bad);
  } else {
    rres = adjoint_sweeps_tv<NX, NU, NG, R>(L, ar, w, bad, slr, mw);
  }
  rres = adj_block_reduce<R>(rows_max(row_max(rres)), mw ? mw->red : nullptr, vmax);

  // ---- 3. VJP outputs ----
  const double nanv = bad ? NAN : 0.0;
  double dgam = 0.0, dgam1 = 0.0;  // this lane's parts of dL/dgamma2, dL/dgamma1
  bool nonfin = false;
  for (int blk = 0; blk < nbl; ++blk) {
    const int t = R * blk + q;
    if (t > N) break;
    const int64_t s = s0 + t;
    const size_t sv = (size_t)s * ROW + i;
    if (i < n) {
      const double e = ex[sv] * exw + nanv;
      nonfin |= !isfinite(e);
      if (a.eta_x) a.eta_x[(size_t)s * n + i] = e;
      if (a.d_q) a.d_q[(size_t)s * n + i] = -e;
      if (a.d_Ddiag) a.d_Ddiag[(size_t)s * n + i] = -e * double(X[sv]) * sd;
    }
    // eta_y of an active slack row: gamma2 G_i eta_x (its row of the reduced system)
    double Gr[n];
    load_row<n>(Gr, L.G + ti_or_tv(L.ti, b, s, (size_t)NG * n) + (size_t)(i < NG ? i : NG - 1) * n, true);
    const double gex = dotb<n>(Gr, (i < n) ? ex[sv] : 0.0, 0.0);
    if (i < NG) {
      const int act = a.act[sv];
      const double xiv = double(XI[sv]);
      const double dxi = a.dLdxi ? a.dLdxi[(size_t)s * NG + i] : 0.0;
      const bool l2a = kind == 1 && act != 0;     // active L2-slack row
      const bool l1s = kind == 2 && xiv != 0.0;   // L1 row with nonzero slack
      // eta_y of an active L2 row: dL/dxi + gamma2 G_i eta_x (eq. bwd:slack:eta_xi_yg)
      const double e = (l2a ? L.gamma2 * gex + dxi : eg[sv]) * se + nanv;
      if (l2a) dgam += xiv * gex;
      if (l1s) dgam1 += (xiv > 0.0 ? 1.0 : -1.0) * gex;
      if (act != 0) nonfin |= !isfinite(e);
      // an L1 row with nonzero slack passes dL/dxi to its bound (xi = bound - G x)
      const double blo = (act < 0) ? e : ((l1s && xiv > 0.0) ? dxi : 0.0);
      const double bhi = (act > 0) ? e : ((l1s && xiv < 0.0) ? dxi : 0.0);
      if (a.d_lo) a.d_lo[(size_t)s * NG + i] = blo;
      if (a.d_hi) a.d_hi[(size_t)s * NG + i] = bhi;
      if (a.eta_g) a.eta_g[(size_t)s * NG + i] = (act != 0) ? e : 0.0;
      if (a.eta_xi) a.eta_xi[(size_t)s * NG + i] = (l2a || l1s) ? -gex + nanv : 0.0;
      if (a.active) a.active[(size_t)s * NG + i] = (int8_t)act;
    }
    if (i < NX) {
      // equality rows in the slot convention of y_f: the initial-state rows
      // at stage 0, dynamics row t - 1 at stage t
      const double e = ef[sv] * efw + nanv;
      nonfin |= !isfinite(e);
      if (a.eta_f) a.eta_f[(size_t)s * NX + i] = e;
      if (t == 0 && a.d_x_init) a.d_x_init[(size_t)b * NX + i] = e;
    }
  }
  dgam = row_sum(dgam);
  dgam += __shfl_xor(dgam, 16);
  dgam += __shfl_xor(dgam, 32);
  dgam1 = row_sum(dgam1);
  dgam1 += __shfl_xor(dgam1, 16);
  dgam1 += __shfl_xor(dgam1, 32);
  dgam = adj_block_reduce<R>(dgam, mw ? mw->red : nullptr, vsum);
  dgam1 = adj_block_reduce<R>(dgam1, mw ? mw->red : nullptr, vsum);
  const bool anynf = adj_block_reduce<R>(__ballot(nonfin) != 0 ? 1.0 : 0.0, mw ? mw->red : nullptr, vmax) != 0.0;
  if (threadIdx.x == 0) {
    if (a.d_gamma2) a.d_gamma2[b] = dgam + nanv;
    if (a.d_gamma1) a.d_gamma1[b] = dgam1 + nanv;
    // relative FP64 residual of the active-set KKT system after the sweeps
    const double rel = rres / fmax(dlmax, 1e-300);
    if (a.adj_resid) a.adj_resid[b] = bad ? NAN : rel;
    if (a.adj_status)
      a.adj_status[b] = bad ? OCP_ADJ_BREAKDOWN : (anynf ? OCP_ADJ_NON_FINITE : (rel <= a.adj_tol ? OCP_ADJ_OK : OCP_ADJ_RESIDUAL));
  }
}


// One instance per wavefront; with multi-wavefront instances (time-varying
// data) those are left to adjoint_mw_kernel.
template <typename T, int NX, int NU, int NG, typename ST>
__global__ __launch_bounds__(64) void adjoint_kernel(Layout L, AdjArgs a) {
  WaveGroup w;
  if (!wave_group(L, w)) return;
  if (!ST::TI && L.n_mw > 0 && w.N >= L.mw_min_n) return;
  adjoint_body<T, NX, NU, NG, ST, 4>(L, a, w, nullptr, nullptr);
}

// One instance per workgroup of mw_waves() wavefronts: L.mw_list[0 .. L.n_mw)
// (time-varying data), with the exchange blocks of the solve's workgroups.
template <typename T, int NX, int NU, int NG, typename ST>
__global__ __launch_bounds__(64 * mw_waves<NX + NU>()) void adjoint_mw_kernel(Layout L, AdjArgs a) {
  constexpr int W = mw_waves<NX + NU>(), R = 4 * W, n = NX + NU;
  __shared__ AdjMwLds<n, R> lds;
  const int slot = blockIdx.x;
  if (slot >= L.n_mw) return;
  WaveGroup w;
  w.lane = threadIdx.x & (ROW - 1);
  w.row = threadIdx.x >> 4;
  w.b = L.mw_list[slot];
  w.s0 = L.stage_off[w.b];
  w.N = (int)(L.stage_off[w.b + 1] - w.s0) - 1;
  double* FX = L.FacXmw + (size_t)slot * fx_slots(R) * n * n;
  adjoint_body<T, NX, NU, NG, ST, R>(L, a, w, FX, &lds);
}

}  // namespace ocpk
