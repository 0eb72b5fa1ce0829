// Implicit-differentiation adjoint (Algorithm 2; Sec. "Backward Pass";
// Appendix "Backward Pass: Sensitivities Computation"), one instance per
// 16-lane row, FP64 throughout.
//
// 1. Active set (Appendix, "Active constraints identification"): the dual
//    sign decides (y < -eps_g lower, y > eps_g upper); closeness to a bound is
//    used only when |y| < eps_g.  eps_g = 10 eps_active max(1, ||y_g||_inf);
//    proximity tolerance eps_g max(1, |bound|).  L1-slack rows with nonzero
//    slack keep their fixed multiplier and are not active.
// 2. The KKT matrix of the active-set conditions (eq. bwd:noslack_kkt_matrix)
//      K = [[H, J'], [J, 0]],  J = [C; G_A]
//    has a zero (2,2) block and no Schur form.  Its regularisation
//      K_reg = [[H + sigma_b I, J'], [J, -rho_b^{-1} I]]
//    does: (H + sigma_b I + rho_b J'J) e_x = r_x + rho_b J' r_y,
//    e_y = rho_b (J e_x - r_y), and H + sigma_b I + rho_b J'J is block
//    tridiagonal, factored by the forward solver's block Cholesky with
//    rho_f = rho_b and per-row inequality weights rho_b [row active].
//    Iterative refinement e <- e + K_reg^{-1}(r - K e) with the residual in
//    FP64 converges to K^{-1} r (the regularisation is a perturbation of
//    size max(sigma_b, 1/rho_b)).
// 3. VJP (eq. loss_gradient): dL/dq = -eta_x, dL/dx_init = eta_f(initial
//    rows), dL/dD_t[i,i] = -eta_x,t,i x_t,i, dL/dlo = eta_g on lower-active
//    rows, dL/dhi = eta_g on upper-active rows.
#pragma once

#include "admm.h"

namespace ocpk {

struct AdjArgs {
  const double* dLdx;  // [S][n]
  double sigma_b, rho_b, eps_active;
  int sweeps;
  // scratch, FP64 padded [S][ROW]
  double* w;    // inequality-row weights (rho_b on active rows)
  double* ex;   // eta_x
  double* ef;   // eta_f (slot convention of y_f)
  double* eg;   // eta_g
  double* rf;   // equality-row residual of the current sweep
  double* rg;   // inequality-row residual of the current sweep
  double* v;    // forward-substitution scratch
  int8_t* act;  // -1 lower, +1 upper, 0 inactive
  // outputs (FP64, may be null)
  double *d_q, *d_Ddiag, *d_x_init, *d_lo, *d_hi, *eta_x;
  int8_t* active;
};

template <typename T, int NX, int NU, int NG, bool TI>
__global__ __launch_bounds__(64) void adjoint_kernel(Layout L, AdjArgs a) {
  constexpr int n = NX + NU;
  Group g;
  g.lane = threadIdx.x & (ROW - 1);
  const int slot = row_slot();
  if (slot >= L.B) return;
  g.b = L.order ? L.order[slot] : slot;
  g.s0 = L.stage_off[g.b];
  g.N = (int)(L.stage_off[g.b + 1] - g.s0) - 1;
  const int i = g.lane, b = g.b, N = g.N;
  const size_t nn = (size_t)n * n;
  const T* X = (const T*)L.x;
  const T* YG = (const T*)L.yg;
  const T* XI = (const T*)L.xi;
  const int kind = (i < NG) ? (int)L.soft[i] : 0;

  // ---- 1. active set ----
  double ymax = 0.0;
  for (int t = 0; t <= N; ++t) {
    const size_t sv = (size_t)(g.s0 + t) * ROW + i;
    if (i < NG) ymax = fmax(ymax, fabs(double(YG[sv])));
  }
  ymax = row_max(ymax);
  const double eg = 10.0 * a.eps_active * fmax(1.0, ymax);
  for (int t = 0; t <= N; ++t) {
    const int64_t s = g.s0 + t;
    const size_t sv = (size_t)s * ROW + i;
    const double xc = (i < n) ? double(X[sv]) : 0.0;
    double Gr[n];
    load_row<n>(Gr, L.G + ti_or_tv(L.ti, b, s, (size_t)NG * n) + (size_t)i * n, i < NG);
    const double gx = dotb<n>(Gr, xc, 0.0);
    int act = 0;
    if (i < NG) {
      const size_t sb = ti_or_tv(L.ti, b, s, NG) + i;
      const double lo = L.lo[sb], hi = L.hi[sb], y = double(YG[sv]);
      const bool amb = fabs(y) < eg;
      bool lower = (y < -eg) || (amb && (gx - lo <= eg * fmax(1.0, fabs(lo))));
      bool upper = (y > eg) || (amb && (hi - gx <= eg * fmax(1.0, fabs(hi))));
      if (lower && upper) {
        if (y > 0) lower = false;
        else upper = false;
      }
      if (kind == 2 && double(XI[sv]) != 0.0) lower = upper = false;
      act = lower ? -1 : (upper ? 1 : 0);
    }
    a.act[sv] = (int8_t)act;
    a.w[sv] = act ? a.rho_b : 0.0;
    a.ex[sv] = 0.0;
    a.ef[sv] = 0.0;
    a.eg[sv] = 0.0;
  }

  // ---- 2. factor H + sigma_b I + rho_b (C'C + G_A'G_A) (FP64) ----
  const int bad = factor_instance<double, NX, NU, NG, false>(L, g, a.sigma_b, a.rho_b, 0.0, a.w);

  // ---- refinement sweeps ----
  for (int sweep = 0; sweep < a.sweeps && !bad; ++sweep) {
    // forward pass: residual r - K e and the Schur right-hand side, then
    // v_t = Linv_t (rhs_t - M_t v_{t-1})
    double em = 0.0, ec = (i < n) ? a.ex[(size_t)g.s0 * ROW + i] : 0.0;
    double efm = 0.0;  // eta_f of dynamics row t-1
    double rfm = 0.0;  // residual of dynamics row t-1
    double Apcm[NX], Eprev[n];
#pragma unroll
    for (int r = 0; r < NX; ++r) Apcm[r] = 0.0;
#pragma unroll
    for (int k = 0; k < n; ++k) Eprev[k] = 0.0;
    double vprev = 0.0;
    for (int t = 0; t <= N; ++t) {
      const int64_t s = g.s0 + t;
      const size_t sv = (size_t)s * ROW + i;
      const double en = (t < N && i < n) ? a.ex[sv + ROW] : 0.0;
      // H e_x (rows of stage t)
      const double* Dp = L.ti ? L.D + (size_t)(2 * b + (t == N ? 1 : 0)) * nn : L.D + (size_t)s * nn;
      double Dr[n];
      load_row<n>(Dr, Dp + (size_t)i * n, i < n);
      double he = dotb<n>(Dr, ec, 0.0);
      if (t > 0) he = dotb<n>(Eprev, em, he);
      if (L.E && t < N) {
        const double* Ep = L.E + ti_or_tv(L.ti, b, s, nn);
        double Ec[n];
        load_col<n>(Ec, Ep + i, n, i < n);
        he = dotb<n>(Ec, en, he);
        load_row<n>(Eprev, Ep + (size_t)i * n, i < n);
      }
      // J' e_y (rows of stage t) and J e_x (rows touching stage t)
      const double efc = (t < N && i < NX) ? a.ef[sv + ROW] : 0.0;
      double jte = 0.0;
      double Amc[NX], Amr[n], Apr[n];
      if (t < N) {
        const double* Amp = L.Am + ti_or_tv(L.ti, b, s, (size_t)NX * n);
        const double* App = L.Ap + ti_or_tv(L.ti, b, s, (size_t)NX * n);
        load_col<NX>(Amc, Amp + i, n, i < n);
        load_row<n>(Amr, Amp + (size_t)i * n, i < NX);
        load_row<n>(Apr, App + (size_t)i * n, i < NX);
        jte = dotb<NX>(Amc, efc, jte);
      }
      if (t > 0) jte = dotb<NX>(Apcm, efm, jte);
      if (t == 0 && i < NX) jte += a.ef[sv];
      const double* Gp = L.G + ti_or_tv(L.ti, b, s, (size_t)NG * n);
      double Gc[NG], Gr[n];
      load_col<NG>(Gc, Gp + i, n, i < n);
      load_row<n>(Gr, Gp + (size_t)i * n, i < NG);
      const double wv = (i < NG) ? a.w[sv] : 0.0;
      const double egv = (i < NG) ? a.eg[sv] : 0.0;
      jte = dotb<NG>(Gc, (wv != 0.0) ? egv : 0.0, jte);
      // residuals of this sweep
      const double rx = ((i < n) ? a.dLdx[(size_t)s * n + i] : 0.0) - (he + jte);
      double rf0 = 0.0;  // initial rows (t == 0)
      if (t == 0 && i < NX) rf0 = -ec;
      double rfc = 0.0;  // dynamics row t
      if (t < N) {
        double cx = dotb<n>(Amr, ec, 0.0);
        cx = dotb<n>(Apr, en, cx);
        rfc = (i < NX) ? -cx : 0.0;
      }
      const double gx = dotb<n>(Gr, ec, 0.0);
      const double rgc = (wv != 0.0) ? -gx : 0.0;
      // Schur right-hand side  r_x + rho_b C' r_f + G'(w .* r_g), w = rho_b [row active]
      double tc = 0.0;
      if (t < N) tc = dotb<NX>(Amc, rfc, tc);
      if (t > 0) tc = dotb<NX>(Apcm, rfm, tc);
      if (t == 0 && i < NX) tc += rf0;
      double rhs = rx + a.rho_b * tc;
      rhs = dotb<NG>(Gc, wv * rgc, rhs);
      if (i < NX && t == 0) a.rf[sv] = rf0;
      if (t < N && i < NX) a.rf[sv + ROW] = rfc;
      if (i < NG) a.rg[sv] = rgc;
      // forward substitution
      if (t > 0) {
        double Mr[n];
        load_row<n>(Mr, L.M64 + (size_t)s * nn + (size_t)i * n, i < n);
        rhs -= dotb<n>(Mr, vprev, 0.0);
      }
      double Lr[n];
      load_row<n>(Lr, L.Linv64 + (size_t)s * nn + (size_t)i * n, i < n);
      const double vv = dotb<n>(Lr, rhs, 0.0);
      if (i < n) a.v[sv] = vv;
      vprev = vv;
      // shift
      if (t < N) load_col<NX>(Apcm, L.Ap + ti_or_tv(L.ti, b, s, (size_t)NX * n) + i, n, i < n);
      efm = efc;
      rfm = rfc;
      em = ec;
      ec = en;
    }
    // backward pass: d_x = L^-T(...), d_y = rho_b (J d_x - r_y), e += d
    double dnext = 0.0;
    for (int t = N; t >= 0; --t) {
      const int64_t s = g.s0 + t;
      const size_t sv = (size_t)s * ROW + i;
      double vv = (i < n) ? a.v[sv] : 0.0;
      if (t < N) {
        double Mc[n];
        load_col<n>(Mc, L.M64 + (size_t)(s + 1) * nn + i, n, i < n);
        vv -= dotb<n>(Mc, dnext, 0.0);
      }
      double Lc[n];
      load_col<n>(Lc, L.Linv64 + (size_t)s * nn + i, n, i < n);
      const double dx = dotb<n>(Lc, vv, 0.0);
      if (t < N) {
        double Amr[n], Apr[n];
        load_row<n>(Amr, L.Am + ti_or_tv(L.ti, b, s, (size_t)NX * n) + (size_t)i * n, i < NX);
        load_row<n>(Apr, L.Ap + ti_or_tv(L.ti, b, s, (size_t)NX * n) + (size_t)i * n, i < NX);
        double jd = dotb<n>(Amr, dx, 0.0);
        jd = dotb<n>(Apr, dnext, jd);
        if (i < NX) a.ef[sv + ROW] += a.rho_b * (jd - a.rf[sv + ROW]);
      }
      {
        double Gr[n];
        load_row<n>(Gr, L.G + ti_or_tv(L.ti, b, s, (size_t)NG * n) + (size_t)i * n, i < NG);
        const double gd = dotb<n>(Gr, dx, 0.0);
        if (i < NG && a.w[sv] != 0.0) a.eg[sv] += a.rho_b * (gd - a.rg[sv]);
      }
      if (t == 0 && i < NX) a.ef[sv] += a.rho_b * (dx - a.rf[sv]);
      if (i < n) a.ex[sv] += dx;
      dnext = dx;
    }
  }

  // ---- 3. VJP outputs ----
  for (int t = 0; t <= N; ++t) {
    const int64_t s = g.s0 + t;
    const size_t sv = (size_t)s * ROW + i;
    const double nanv = bad ? NAN : 0.0;
    if (i < n) {
      const double e = a.ex[sv] + nanv;
      if (a.eta_x) a.eta_x[(size_t)s * n + i] = e;
      if (a.d_q) a.d_q[(size_t)s * n + i] = -e;
      if (a.d_Ddiag) a.d_Ddiag[(size_t)s * n + i] = -e * double(X[sv]);
    }
    if (i < NG) {
      const int act = a.act[sv];
      const double e = a.eg[sv] + nanv;
      if (a.d_lo) a.d_lo[(size_t)s * NG + i] = (act < 0) ? e : 0.0;
      if (a.d_hi) a.d_hi[(size_t)s * NG + i] = (act > 0) ? e : 0.0;
      if (a.active) a.active[(size_t)s * NG + i] = (int8_t)act;
    }
    if (t == 0 && i < NX && a.d_x_init) a.d_x_init[(size_t)b * NX + i] = a.ef[sv] + nanv;
  }
}

}  // namespace ocpk
