// Block-tridiagonal Cholesky of the ADMM Schur matrix (FP64).
//
//   S = P + sigma I + C' rho_f C + G' diag(rho_g) G            (Appendix "ADMM",
//       Schur complement components)
//   Theta_t = D_t + sigma I + rho_f (A_init'A_init [t=0] + A_t^-' A_t^- [t<N]
//             + A_{t-1}^+' A_{t-1}^+ [t>0]) + G_t' diag(rho_g) G_t
//   Phi_t   = E_t + rho_f A_t^+' A_t^-        (block (t+1, t))
//
// Block recurrence (textbook block Cholesky of a block-tridiagonal SPD
// matrix, S = L L' with L block lower-bidiagonal, diagonal blocks L_t and
// sub-diagonal blocks M_t):
//   L_0 L_0' = Theta_0
//   M_t      = Phi_{t-1} L_{t-1}^{-T},   L_t L_t' = Theta_t - M_t M_t'   (t >= 1)
// Stored per stage: Linv_t = L_t^{-1} (lower) and M_t, FP64 master plus an
// iteration-precision copy.  A non-positive pivot reports a factor breakdown.
#pragma once

#include "dev_common.h"

namespace ocpk {

// out[j] += scale * sum_r a[r] * (lane j's b[r]),  j < C
template <int R, int C>
__device__ __forceinline__ void cross_row(const double (&a)[R], const double (&b)[R], double (&out)[C],
                                          double scale) {
  sfor<0, C>([&](auto j) {
    constexpr int jj = decltype(j)::value;
    double acc = 0.0;
    DotC<R, double>::template f<jj>(acc, b, a);
    out[jj] = fma(scale, acc, out[jj]);
  });
}

// Per-stage FP64 inputs of the factorisation (lane i: row / column i).
template <int NX, int NU, int NG>
struct FacStage {
  static constexpr int n = NX + NU;
  double D[n], E[n];        // row i of D_t, E_t
  double Amc[NX], Apc[NX];  // column i of A_t^-, A_t^+
  double Gc[NG], w[NG];     // column i of G_t, inequality-row weights
};

template <int NX, int NU, int NG>
__device__ __forceinline__ void load_fac(FacStage<NX, NU, NG>& d, const Layout& L, const Group& g, int t, double rho_g,
                                         const double* __restrict__ rhog_rows) {
  constexpr int n = NX + NU;
  const size_t nn = (size_t)n * n;
  const int i = g.lane, b = g.b, N = g.N;
  const int ic = i < n ? i : n - 1;  // lanes past n read a valid row (results unused)
  const int64_t s = g.s0 + t;
  const double* Dp = L.ti ? L.D + (size_t)(2 * b + (t == N ? 1 : 0)) * nn : L.D + (size_t)s * nn;
  load_row<n>(d.D, Dp + (size_t)ic * n, true);
  if (L.E && t < N)
    load_row<n>(d.E, L.E + ti_or_tv(L.ti, b, s, nn) + (size_t)ic * n, true);
  else
#pragma unroll
    for (int k = 0; k < n; ++k) d.E[k] = 0.0;
  load_col<NX>(d.Amc, L.Am + ti_or_tv(L.ti, b, s, (size_t)NX * n) + ic, n, t < N);
  load_col<NX>(d.Apc, L.Ap + ti_or_tv(L.ti, b, s, (size_t)NX * n) + ic, n, t < N);
  load_col<NG>(d.Gc, L.G + ti_or_tv(L.ti, b, s, (size_t)NG * n) + ic, n, true);
#pragma unroll
  for (int r = 0; r < NG; ++r) d.w[r] = rhog_rows ? as_global(rhog_rows)[(size_t)s * ROW + r] : rho_g;
}

// a[4 q + JJ] on row q (zero past the end of a)
template <int JJ, int K, typename T>
__device__ __forceinline__ T quarter_pick(const T (&a)[K], int q) {
  T v[4];
  sfor<0, 4>([&](auto r) {
    constexpr int idx = 4 * decltype(r)::value + JJ;
    if constexpr (idx < K)
      v[decltype(r)::value] = a[idx];
    else
      v[decltype(r)::value] = T(0);
  });
  const T a0 = (q & 1) ? v[1] : v[0];
  const T a1 = (q & 1) ? v[3] : v[2];
  return (q & 2) ? a1 : a0;
}

// Factor one instance.  rhog_rows: optional per-row inequality weights
// ([S][ROW], FP64); when null every inequality row uses rho_g.
// HOIST: time-invariant blocks; the blocks are read once and the products
// A^-'A^-, A^+'A^+, A^+'A^- (and G'G under uniform weights) are formed once
// per instance, so a stage reads nothing but its row weights.
// FORM selects the outputs (all row-major, [S][n][n]):
//   FACTOR_M   (adjoint)  FP64 Linv_t and M_t.
//   FACTOR_WV  (ADMM solve, FP32 iterations) in iteration precision
//              SubA = Linv_t, SubB = Linv_t', ChF = W_t = Linv_t M_t (W_0 = 0),
//              ChB = V_t = Linv_t' M_{t+1}' (V_N = 0):
//                v_t = Linv_t eta_t - W_t v_{t-1},  x_t = Linv_t' v_t - V_t x_{t+1}.
//   FACTOR_PK  (ADMM solve, FP64 iterations) SubB = P_t = (L_t L_t')^{-1},
//              ChF = K_t = Phi_{t-1} P_{t-1} (K_0 = 0), ChB = Kb_t = K_{t+1}'
//              (Kb_N = 0):
//                v~_t = eta_t - K_t v~_{t-1},  x_t = P_t v~_t - Kb_t x_{t+1}
//              (v~_t = L_t v_t; M_{t+1}' = Linv_t Phi_t').  Three blocks per
//              stage instead of four, but P_t carries the full condition number
//              of the Schur block, so FP32 iterations keep the Linv form.
// In the two solve forms the four 16-lane rows of the wavefront each form and
// store the output columns 4 qrow .. 4 qrow + 3 (the recurrence itself runs
// on every row).  Returns 0 on success, 1 on a non-positive / non-finite pivot.
enum { FACTOR_M = 0, FACTOR_WV = 1, FACTOR_PK = 2 };

// TAG only separates the instantiations called from kernels with different
// occupancy targets (the register budget of a called function follows its
// callers).
template <typename T, int NX, int NU, int NG, bool HOIST, int FORM = FACTOR_M, int TAG = 0>
__device__ __noinline__ int factor_instance(const Layout& Lm, const Group& gm, double sigma_, double rho_f_,
                                            double rho_g_, const double* __restrict__ rhog_rows_, int qrow = 0) {
  const Layout L = uni(Lm);
  const Group g{gm.lane, uni(gm.b), uni(gm.s0), uni(gm.N)};
  const double sigma = uni(sigma_), rho_f = uni(rho_f_), rho_g = uni(rho_g_);
  const double* __restrict__ rhog_rows = uni(rhog_rows_);
  constexpr bool WV = FORM == FACTOR_WV;
  constexpr bool PK = FORM == FACTOR_PK;
  constexpr int n = NX + NU;
  const int i = g.lane;
  const bool vi = i < n;
  const int N = g.N;
  const size_t nn = (size_t)n * n;

  double Mrow[n];     // row i of M_t
  double ApcPrev[NX]; // column i of A_{t-1}^+
  double Xprev[WV ? n : 1];  // row i of Linv_{t-1}
#pragma unroll
  for (int k = 0; k < n; ++k) Mrow[k] = 0.0;
#pragma unroll
  for (int r = 0; r < NX; ++r) ApcPrev[r] = 0.0;

  // rho-independent products (row i), formed once when the blocks do not vary
  double PAm[HOIST ? n : 1], PAp[HOIST ? n : 1], PG[HOIST ? n : 1], PPhi[HOIST ? n : 1];
  double Dint[HOIST ? n : 1], Dter[HOIST ? n : 1], Erow[HOIST ? n : 1], GcH[HOIST ? NG : 1];
  FacStage<NX, NU, NG> cur, nxt;
  if constexpr (HOIST) {
    const int ic = i < n ? i : n - 1;
    const size_t b = (size_t)g.b;
    load_row<n>(Dint, L.D + (2 * b) * nn + (size_t)ic * n, true);
    load_row<n>(Dter, L.D + (2 * b + 1) * nn + (size_t)ic * n, true);
    if (L.E)
      load_row<n>(Erow, L.E + b * nn + (size_t)ic * n, true);
    else
#pragma unroll
      for (int k = 0; k < n; ++k) Erow[k] = 0.0;
    double Amc[NX], Apc[NX];
    load_col<NX>(Amc, L.Am + b * NX * n + ic, n, true);
    load_col<NX>(Apc, L.Ap + b * NX * n + ic, n, true);
    load_col<NG>(GcH, L.G + b * NG * n + ic, n, true);
#pragma unroll
    for (int k = 0; k < n; ++k) PAm[k] = PAp[k] = PG[k] = PPhi[k] = 0.0;
    cross_row<NX, n>(Amc, Amc, PAm, 1.0);
    cross_row<NX, n>(Apc, Apc, PAp, 1.0);
    cross_row<NX, n>(Apc, Amc, PPhi, 1.0);
    if (!rhog_rows) cross_row<NG, n>(GcH, GcH, PG, rho_g);
  } else {
    load_fac(cur, L, g, 0, rho_g, rhog_rows);
  }

  int bad = 0;
  for (int t = 0; t <= N; ++t) {
    const int64_t s = g.s0 + t;
    if constexpr (!HOIST) {
      if (t < N) load_fac(nxt, L, g, t + 1, rho_g, rhog_rows);  // prefetch
    }
    double S[n];
    if constexpr (HOIST) {
#pragma unroll
      for (int k = 0; k < n; ++k) S[k] = (t == N) ? Dter[k] : Dint[k];
    } else {
#pragma unroll
      for (int k = 0; k < n; ++k) S[k] = cur.D[k];
    }
    sfor<0, n>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      if (i == jj) S[jj] += sigma + ((t == 0 && jj < NX) ? rho_f : 0.0);
    });
    if constexpr (HOIST) {
      const double ca = (t < N) ? rho_f : 0.0, cp = (t > 0) ? rho_f : 0.0;
#pragma unroll
      for (int k = 0; k < n; ++k) S[k] += ca * PAm[k] + cp * PAp[k] + PG[k];
      if (rhog_rows) {  // stage weights (the same address on every lane)
        double Gw[NG];
#pragma unroll
        for (int r = 0; r < NG; ++r) Gw[r] = as_global(rhog_rows)[(size_t)s * ROW + r] * GcH[r];
        cross_row<NG, n>(Gw, GcH, S, 1.0);
      }
    } else {
      if (t < N) cross_row<NX, n>(cur.Amc, cur.Amc, S, rho_f);
      if (t > 0) cross_row<NX, n>(ApcPrev, ApcPrev, S, rho_f);
      double Gw[NG];
#pragma unroll
      for (int r = 0; r < NG; ++r) Gw[r] = cur.w[r] * cur.Gc[r];
      cross_row<NG, n>(Gw, cur.Gc, S, 1.0);
    }
    if (t > 0) cross_row<n, n>(Mrow, Mrow, S, -1.0);

    // dense Cholesky of S (lane i holds row i), L row i and 1/L_kk
    double Lr[n], invd[n];
    sfor<0, n>([&](auto k) {
      constexpr int kk = decltype(k)::value;
      double dkk = bc<kk>(S[kk]);
      if (!(dkk > 0.0) || !isfinite(dkk)) {
        bad = 1;
        dkk = 1.0;
      }
      const double dk = sqrt(dkk);
      const double id = 1.0 / dk;
      invd[kk] = id;
      const double lik = (i >= kk) ? S[kk] * id : 0.0;
      Lr[kk] = lik;
      sfor<kk + 1, n>([&](auto j) {
        constexpr int jj = decltype(j)::value;
        S[jj] = fma(-lik, bc<jj>(lik), S[jj]);
      });
    });
    // X = L^{-1}, lane i holds row i
    double X[n];
    sfor<0, n>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      X[jj] = (i == jj) ? 1.0 : 0.0;
    });
    sfor<0, n>([&](auto k) {
      constexpr int kk = decltype(k)::value;
      const double sc = (i == kk) ? invd[kk] : 1.0;
      sfor<0, kk + 1>([&](auto j) {
        constexpr int jj = decltype(j)::value;
        X[jj] *= sc;
      });
      const double lik = (i > kk) ? Lr[kk] : 0.0;
      sfor<0, kk + 1>([&](auto j) {
        constexpr int jj = decltype(j)::value;
        X[jj] = fma(-lik, bc<kk>(X[jj]), X[jj]);
      });
    });
    double Pc[PK ? 4 : 1];  // columns 4 qrow .. 4 qrow + 3 of P_t, row i
    if constexpr (WV) {
      // rows / columns 4 qrow .. 4 qrow + 3 of Linv_t, W_t and V_{t-1}
      const gptr<T> lr = as_global((T*)L.SubA + (size_t)s * nn + (size_t)i * n);
      const gptr<T> lc = as_global((T*)L.SubB + (size_t)s * nn + i);
      const gptr<T> wr = as_global((T*)L.ChF + (size_t)s * nn + (size_t)i * n);
      const gptr<T> vc = as_global((T*)L.ChB + (size_t)(t > 0 ? s - 1 : s) * nn + i);
      sfor<0, 4>([&](auto jj_) {
        constexpr int jj = decltype(jj_)::value;
        const int j = 4 * qrow + jj;
        const double xj = quarter_pick<jj>(X, qrow);
        double wij = 0.0, uji = 0.0;
        if (t > 0) {
          // W_t[i][j] = sum_k Linv_t[i][k] M_t[k][j]
          wij = dotb<n>(X, quarter_pick<jj>(Mrow, qrow), 0.0);
          // (M_t Linv_{t-1})[i][j] = sum_k M_t[i][k] Linv_{t-1}[k][j]  (= V_{t-1}[j][i])
          uji = dotb<n>(Mrow, quarter_pick<jj>(Xprev, qrow), 0.0);
        }
        if (vi && j < n) {
          lr[j] = T(xj);
          lc[(size_t)j * n] = T(xj);
          if (t > 0) {
            wr[j] = T(wij);
            vc[(size_t)j * n] = T(uji);
          }
        }
      });
#pragma unroll
      for (int k = 0; k < n; ++k) Xprev[k] = X[k];
    } else if constexpr (PK) {
      // Linv_t' through LDS: lane i receives column i of Linv_t
      __shared__ double xt_lds[16 * 17];
      if (qrow == 0 && vi) {
#pragma unroll
        for (int j = 0; j < n; ++j) xt_lds[i * 17 + j] = X[j];
      }
      __syncthreads();
      double XT[n];
      const int ic = vi ? i : n - 1;
#pragma unroll
      for (int k = 0; k < n; ++k) XT[k] = xt_lds[k * 17 + ic];
      __syncthreads();  // the buffer is rewritten at the next stage
      // P_t = Linv_t' Linv_t: P[i][j] = sum_k Linv_t[k][i] Linv_t[k][j]
      const gptr<T> pr = as_global((T*)L.SubB + (size_t)s * nn + (size_t)i * n);
      sfor<0, 4>([&](auto jj_) {
        constexpr int jj = decltype(jj_)::value;
        const int j = 4 * qrow + jj;
        Pc[jj] = dotb<n>(XT, quarter_pick<jj>(X, qrow), 0.0);
        if (vi && j < n) pr[j] = T(Pc[jj]);
      });
    } else if (vi) {
      const gptr<double> dst = as_global(L.Linv64 + (size_t)s * nn + (size_t)i * n);
#pragma unroll
      for (int j = 0; j < n; ++j) dst[j] = X[j];
    }
    if (t < N) {
      // Phi_t row i = E_t row i + rho_f sum_r A_t^+[r][i] A_t^-[r][:]
      double Phi[n];
      if constexpr (HOIST) {
#pragma unroll
        for (int k = 0; k < n; ++k) Phi[k] = Erow[k] + rho_f * PPhi[k];
      } else {
#pragma unroll
        for (int k = 0; k < n; ++k) Phi[k] = cur.E[k];
        cross_row<NX, n>(cur.Apc, cur.Amc, Phi, rho_f);
      }
      // M_{t+1} row i: M[i][j] = sum_{k<=j} Phi[i][k] Linv[j][k]
      sfor<0, n>([&](auto j) {
        constexpr int jj = decltype(j)::value;
        double acc = 0.0, xs[jj + 1], ps[jj + 1];
#pragma unroll
        for (int k = 0; k <= jj; ++k) {
          xs[k] = X[k];
          ps[k] = Phi[k];
        }
        DotC<jj + 1, double>::template f<jj>(acc, xs, ps);
        Mrow[jj] = acc;
      });
      if constexpr (PK) {
        // K_{t+1} = Phi_t P_t (columns 4 qrow .. 4 qrow + 3 of row i) and its
        // transpose Kb_t = K_{t+1}'
        const gptr<T> kr = as_global((T*)L.ChF + (size_t)(s + 1) * nn + (size_t)i * n);
        const gptr<T> kb = as_global((T*)L.ChB + (size_t)s * nn + i);
        sfor<0, 4>([&](auto jj_) {
          constexpr int jj = decltype(jj_)::value;
          const int j = 4 * qrow + jj;
          const double kij = dotb<n>(Phi, Pc[jj], 0.0);
          if (vi && j < n) {
            kr[j] = T(kij);
            kb[(size_t)j * n] = T(kij);
          }
        });
      } else if (!WV && vi) {
        const gptr<double> dst = as_global(L.M64 + (size_t)(s + 1) * nn + (size_t)i * n);
#pragma unroll
        for (int j = 0; j < n; ++j) dst[j] = Mrow[j];
      }
      if constexpr (!HOIST) {
#pragma unroll
        for (int r = 0; r < NX; ++r) ApcPrev[r] = cur.Apc[r];
        cur = nxt;
      }
    }
  }
  return bad;
}

}  // namespace ocpk
