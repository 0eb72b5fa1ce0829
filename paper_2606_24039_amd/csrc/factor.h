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

// 1/sqrt(d) for d > 0 in FP64: the hardware estimate (relative error below
// 2^-22) refined by one third-order Newton step, y <- y (1 + r/2 + 3 r^2/8)
// with r = 1 - d y^2, which leaves a relative error of a few units in the
// last place.  One transcendental and five dependent operations instead of
// a correctly rounded square root followed by a correctly rounded division.
__device__ __forceinline__ double rsqrt_pivot(double d) {
  const double y = __builtin_amdgcn_rsq(d);
  const double h = d * y;
  const double r = fma(-h, y, 1.0);
  const double c = fma(0.375, r, 0.5) * r;
  return fma(y, c, y);
}

// Cholesky S = L L' of the n x n block held by rows (lane i of the 16-lane
// row: row i of S, clobbered) and X = L^{-1} (lane i: row i).  Returns 1 on a
// non-positive or non-finite pivot (the same on every lane of the row).
template <int n>
__device__ __forceinline__ int chol_inv(double (&S)[n], double (&X)[n], int i) {
  int bad = 0;
  double Lr[n], invd[n];
  sfor<0, n>([&](auto k) {
    constexpr int kk = decltype(k)::value;
    double dkk = bc<kk>(S[kk]);
    if (!(dkk > 0.0) || !isfinite(dkk)) {
      bad = 1;
      dkk = 1.0;
    }
    const double id = rsqrt_pivot(dkk);
    invd[kk] = id;
    const double lik = (i >= kk) ? S[kk] * id : 0.0;
    Lr[kk] = lik;
    sfor<kk + 1, n>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      S[jj] = fma(-lik, bc<jj>(lik), S[jj]);
    });
  });
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
  return bad;
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
//              SubA = Linv_t packed (below), ChF = W_t = Linv_t M_t (W_0 = 0),
//              ChB = V_t = Linv_t' M_{t+1}' (V_N = 0):
//                v_t = Linv_t eta_t - W_t v_{t-1},  x_t = Linv_t' v_t - V_t x_{t+1}.
//              Packed Linv_t: row i, entry e holds Linv_t[max(i,s)][min(i,s)]
//              with s = (i - e) mod n, so one n x n block gives both
//              Linv_t eta (entries with s <= i, dotl) and Linv_t' v (s >= i,
//              dotu); SubB is not written.
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
//   FACTOR_PCG (PCG primal updates) no recursion: SubA = Theta_t^-1 (the
//              block-Jacobi preconditioner), SubB = Theta_t, ChF = Phi_t
//              (block (t+1, t) of S), ChB = Phi_t' (t < N), all in
//              iteration precision; row 0 stores them.
enum { FACTOR_M = 0, FACTOR_WV = 1, FACTOR_PK = 2, FACTOR_PCG = 3 };

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
  constexpr bool PCG = FORM == FACTOR_PCG;
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
    if (!PCG && t > 0) cross_row<n, n>(Mrow, Mrow, S, -1.0);
    double Th[PCG ? n : 1];  // row i of Theta_t (PCG: the matrix-vector products use it)
    if constexpr (PCG) {
#pragma unroll
      for (int k = 0; k < n; ++k) Th[k] = S[k];
    }

    // dense Cholesky of S and X = L^{-1} (lane i holds row i)
    double X[n];
    bad |= chol_inv<n>(S, X, i);
    if constexpr (PCG) {
      // Theta_t^-1 = X'X (row i), and Theta_t
      double XT[n], E1[n], Pi[n];
#pragma unroll
      for (int j = 0; j < n; ++j) {
        XT[j] = 0.0;
        E1[j] = (i == j) ? 1.0 : 0.0;
      }
      cross_row<n, n>(E1, X, XT, 1.0);
      sfor<0, n>([&](auto j) {
        constexpr int jj = decltype(j)::value;
        Pi[jj] = dotb<n>(XT, X[jj], 0.0);
      });
      if (qrow == 0 && vi) {
        const gptr<T> pr = as_global((T*)L.SubA + (size_t)s * nn + (size_t)i * n);
        const gptr<T> tr = as_global((T*)L.SubB + (size_t)s * nn + (size_t)i * n);
#pragma unroll
        for (int j = 0; j < n; ++j) {
          pr[j] = T(Pi[j]);
          tr[j] = T(Th[j]);
        }
      }
    }
    double Pc[PK ? 4 : 1];  // columns 4 qrow .. 4 qrow + 3 of P_t, row i
    if constexpr (WV) {
      // columns 4 qrow .. 4 qrow + 3 of Linv_t (packed), W_t and V_{t-1}
      const gptr<T> pk = as_global((T*)L.SubA + (size_t)s * nn);
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
          // Linv_t[i][j], j <= i: entry i - j of row i and entry j - i + n of row j
          if (j <= i) pk[i * n + i - j] = T(xj);
          if (j < i) pk[j * n + j - i + n] = T(xj);
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
      if constexpr (PCG) {  // Phi_t rows and, transposed, Phi_t'
        if (qrow == 0 && vi) {
          const gptr<T> fr = as_global((T*)L.ChF + (size_t)s * nn + (size_t)i * n);
          const gptr<T> fc = as_global((T*)L.ChB + (size_t)s * nn + i);
#pragma unroll
          for (int j = 0; j < n; ++j) {
            fr[j] = T(Phi[j]);
            fc[(size_t)j * n] = T(Phi[j]);
          }
        }
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
      } else if (FORM == FACTOR_M && vi) {
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

// ---------------------------------------------------------------------------
// Chunked factorisation of long horizons (same outputs as factor_instance up
// to rounding, 2 / (R + 1) of its serial depth with R 16-lane rows).
//
// The recurrence above carries one n x n state from stage to stage: what
// enters stage t is M_t (S_t = Theta_t - M_t M_t').  The horizon is cut into
// R + 1 contiguous chunks c = 0..R, chunk c covering stages a_c .. b_c (R = 4:
// the four rows of one wavefront; R = 4 W: the rows of a W-wavefront
// workgroup, all of which call this function).
//
// Phase 1, one chunk per 16-lane row: row 0 factors chunk 0 exactly and
// stores its blocks.  Row c = 1..R-1 summarises chunk c as a function of its
// entering state.  With T the block-tridiagonal matrix of the chunk's
// interior a_c .. b_c - 1 (no entering term), factored by the same recurrence
// started from M = 0 (T = L0 L0'), the entering state Z = M M' (M = M_{a_c})
// changes the interior to T - E Z E' (E: the block column of stage a_c), and
// the Woodbury identity gives the Schur complement at b_c
//   S_b = S0_b - K_ba M (I - M' K_aa M)^{-1} M' K_ba',
// where S0_b is its value for Z = 0, K_aa = E' T^{-1} E and
// K_ba = Phi_{b-1} (T^{-1})_{b-1,a}.  With U = L0^{-1} E, formed block by
// block as U_a = L0_a^{-1}, U_t = -W0_t U_{t-1} (W0_t = L0_t^{-1} M0_t), these
// are K_aa = sum_t U_t' U_t and K_ba = M0_b U_{b-1}.  I - M' K_aa M is SPD
// because T - E Z E' is (a Schur complement of the SPD Schur matrix).
// Phase 2, on every row, serially over c = 1..R-1: from M_{a_1} (row 0's
// exit) the summaries give M_{a_2} .. M_{a_R}, and L_{b_c}^{-1}, which the
// first stage of the next chunk needs for its V block.
// Phase 3, one chunk per row: rows 1..R-1 re-run chunks 1..R-1 and row 0 runs
// chunk R, each from its true entering state, storing their blocks.  Every
// row forms and stores all n columns of its outputs.
//
// Scratch: fx_slots(R) FP64 n x n exchange blocks per instance (L.FacX for
// R = 4, [B][FX_SLOTS][n][n]).
// ---------------------------------------------------------------------------
struct FacChunk {
  int a, len;  // first stage and stage count
};
template <int R = 4>
__device__ __forceinline__ FacChunk fac_chunk(int c, int N) {
  const int S = N + 1, base = S / (R + 1), rem = S % (R + 1);
  return FacChunk{c * base + min(c, rem), base + (c < rem ? 1 : 0)};
}
// shortest horizon factored in chunks by one wavefront (every chunk then
// holds at least three stages, so every summarised chunk has an interior);
// R rows need N + 1 >= 3 (R + 1)
constexpr int FAC_CHUNK_MIN_N = 15;
__host__ __device__ constexpr int fac_chunk_min_n(int R) { return 3 * (R + 1) - 1; }
// exchange slots: M_{a_1} and L_{b_0}^{-1} from row 0; per summarised chunk
// c = 1..R-1 the four blocks S0_b, K_aa, K_ba, Phi_b at FX_SUM + 4 (c - 1)
enum { FX_M1 = 0, FX_X0 = 1, FX_SUM = 2 };
__host__ __device__ constexpr int fx_slots(int R) { return FX_SUM + 4 * (R - 1); }
constexpr int FX_SLOTS = fx_slots(4);

template <typename T, int NX, int NU, int NG, bool HOIST, int FORM, int TAG = 0, int NR = 4>
__device__ __noinline__ int factor_chunked(const Layout& Lm, const Group& gm, double sigma_, double rho_f_,
                                           double rho_g_, const double* __restrict__ rhog_rows_,
                                           double* FX_ = nullptr) {
  const Layout L = uni(Lm);
  const Group g{gm.lane, uni(gm.b), uni(gm.s0), uni(gm.N)};
  const double sigma = uni(sigma_), rho_f = uni(rho_f_), rho_g = uni(rho_g_);
  const double* __restrict__ rhog_rows = uni(rhog_rows_);
  constexpr bool WV = FORM == FACTOR_WV;
  constexpr bool PK = FORM == FACTOR_PK;
  constexpr int n = NX + NU;
  const int i = g.lane;
  const int q = (int)(threadIdx.x >> 4);
  const bool vi = i < n;
  const int ic = vi ? i : n - 1;
  const int N = g.N;
  const size_t nn = (size_t)n * n;
  // exchange blocks: the caller's (multi-wavefront instances), else the instance's slots of L.FacX
  double* const FX = FX_ ? uni(FX_) : L.FacX + (size_t)g.b * FX_SLOTS * nn;

  // rho-independent products (row i), formed once when the blocks do not vary
  double PAm[HOIST ? n : 1], PAp[HOIST ? n : 1], PG[HOIST ? n : 1], PPhi[HOIST ? n : 1];
  double Dint[HOIST ? n : 1], Dter[HOIST ? n : 1], Erow[HOIST ? n : 1], GcH[HOIST ? NG : 1];
  if constexpr (HOIST) {
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
  }
  FacStage<NX, NU, NG> cur, nxt;
  double ApcPrev[NX];  // column i of A_{t-1}^+ (time-varying data)

  // row i of Theta_t (no entering term)
  auto theta = [&](int t, int64_t s, double (&S)[n]) {
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
      if (rhog_rows) {
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
  };
  // row i of Phi_t = E_t + rho_f A_t^+' A_t^-  (t < N)
  auto phi = [&](double (&Phi)[n]) {
    if constexpr (HOIST) {
#pragma unroll
      for (int k = 0; k < n; ++k) Phi[k] = Erow[k] + rho_f * PPhi[k];
    } else {
#pragma unroll
      for (int k = 0; k < n; ++k) Phi[k] = cur.E[k];
      cross_row<NX, n>(cur.Apc, cur.Amc, Phi, rho_f);
    }
  };
  auto store_row = [&](int slot, const double (&r)[n]) {
    if (vi) {
      double* dst = FX + (size_t)slot * nn + (size_t)i * n;
#pragma unroll
      for (int j = 0; j < n; ++j) dst[j] = r[j];
    }
  };

  int bad = 0;
  // One pass of the recurrence over chunk `ch` on this row.  SUM: phase 1
  // (rows 1..3 summarise; the entering state is zero).  kmax: the longest
  // chunk of the pass (rows whose chunk is shorter idle).
  double Mrow[n], Xprev[n], UT[n], Kaa[n];
  auto sweep = [&](auto sum_tag, const FacChunk ch, const bool store, const int kmax) {
    constexpr bool SUM = decltype(sum_tag)::value;
    const bool summ = SUM && q > 0;
    if constexpr (!HOIST) {
      load_fac(cur, L, g, ch.a, rho_g, rhog_rows);
      const int64_t sp = g.s0 + (ch.a > 0 ? ch.a - 1 : 0);
      load_col<NX>(ApcPrev, L.Ap + ti_or_tv(L.ti, g.b, sp, (size_t)NX * n) + ic, n, ch.a > 0);
    }
    for (int k = 0; k < kmax; ++k) {
      if (k >= ch.len) continue;  // the same on all lanes of a row
      const int t = ch.a + k;
      const int64_t s = g.s0 + t;
      if constexpr (!HOIST) {
        if (t < N) load_fac(nxt, L, g, t + 1, rho_g, rhog_rows);  // prefetch
      }
      double S[n];
      theta(t, s, S);
      if (!SUM || k > 0) cross_row<n, n>(Mrow, Mrow, S, -1.0);
      if (summ && k == ch.len - 1) {
        // exit stage b of a summarised chunk: S0_b, K_ba = M0_b U_{b-1}, Phi_b
        double Kba[n], Phi[n];
#pragma unroll
        for (int j = 0; j < n; ++j) Kba[j] = 0.0;
        cross_row<n, n>(Mrow, UT, Kba, 1.0);
        phi(Phi);
        const int base = FX_SUM + 4 * (q - 1);
        store_row(base + 0, S);
        store_row(base + 1, Kaa);
        store_row(base + 2, Kba);
        store_row(base + 3, Phi);
        continue;
      }
      double X[n];
      const int bk = chol_inv<n>(S, X, i);
      bad |= bk;
      // W_t = Linv_t M_t (row i, every column; zero where M_t = 0)
      double W[n];
      sfor<0, n>([&](auto j) {
        constexpr int jj = decltype(j)::value;
        W[jj] = dotb<n>(X, Mrow[jj], 0.0);
      });
      if (summ) {
        // U_t' rows: U_a' = Linv_a', U_t' = -U_{t-1}' W_t'; K_aa += U_t' U_t
        double Un[n];
#pragma unroll
        for (int j = 0; j < n; ++j) Un[j] = 0.0;
        if (k == 0)
          cross_row<n, n>(UT, X, Un, 1.0);
        else
          cross_row<n, n>(UT, W, Un, -1.0);
#pragma unroll
        for (int j = 0; j < n; ++j) UT[j] = Un[j];
        cross_row<n, n>(UT, UT, Kaa, 1.0);
      }
      double Phi[n];
      if (t < N) phi(Phi);
      if (store) {
        if constexpr (WV) {
          // Linv_t (packed), W_t, and V_{t-1} = (M_t Linv_{t-1})'
          double V[n];
          sfor<0, n>([&](auto j) {
            constexpr int jj = decltype(j)::value;
            V[jj] = dotb<n>(Mrow, Xprev[jj], 0.0);
          });
          if (vi) {
            // Linv_t packed: Linv_t[i][j], j <= i, to entry i - j of row i
            // and entry j - i + n of row j
            const gptr<T> pk = as_global((T*)L.SubA + (size_t)s * nn);
#pragma unroll
            for (int j = 0; j < n; ++j) {
              if (j <= i) pk[i * n + i - j] = T(X[j]);
              if (j < i) pk[j * n + j - i + n] = T(X[j]);
            }
            if (t > 0) {
              const gptr<T> wr = as_global((T*)L.ChF + (size_t)s * nn + (size_t)i * n);
              const gptr<T> vc = as_global((T*)L.ChB + (size_t)(s - 1) * nn + i);
#pragma unroll
              for (int j = 0; j < n; ++j) {
                wr[j] = T(W[j]);
                vc[(size_t)j * n] = T(V[j]);
              }
            }
          }
        } else if constexpr (PK) {
          // P_t = Linv_t' Linv_t; K_{t+1} = Phi_t P_t and Kb_t = K_{t+1}'
          double XT[n], P[n], E1[n];
#pragma unroll
          for (int j = 0; j < n; ++j) {
            XT[j] = 0.0;
            E1[j] = (i == j) ? 1.0 : 0.0;
          }
          cross_row<n, n>(E1, X, XT, 1.0);
          sfor<0, n>([&](auto j) {
            constexpr int jj = decltype(j)::value;
            P[jj] = dotb<n>(XT, X[jj], 0.0);
          });
          double K[n];
          sfor<0, n>([&](auto j) {
            constexpr int jj = decltype(j)::value;
            K[jj] = dotb<n>(Phi, P[jj], 0.0);
          });
          if (vi) {
            const gptr<T> pr = as_global((T*)L.SubB + (size_t)s * nn + (size_t)i * n);
#pragma unroll
            for (int j = 0; j < n; ++j) pr[j] = T(P[j]);
            if (t < N) {
              const gptr<T> kr = as_global((T*)L.ChF + (size_t)(s + 1) * nn + (size_t)i * n);
              const gptr<T> kb = as_global((T*)L.ChB + (size_t)s * nn + i);
#pragma unroll
              for (int j = 0; j < n; ++j) {
                kr[j] = T(K[j]);
                kb[(size_t)j * n] = T(K[j]);
              }
            }
          }
        } else if (vi) {
          const gptr<double> dst = as_global(L.Linv64 + (size_t)s * nn + (size_t)i * n);
#pragma unroll
          for (int j = 0; j < n; ++j) dst[j] = X[j];
        }
      }
      if (t < N) {
        // M_{t+1} row i: M[i][j] = sum_{k<=j} Phi[i][k] Linv[j][k]
        sfor<0, n>([&](auto j) {
          constexpr int jj = decltype(j)::value;
          double acc = 0.0, xs[jj + 1], ps[jj + 1];
#pragma unroll
          for (int kk = 0; kk <= jj; ++kk) {
            xs[kk] = X[kk];
            ps[kk] = Phi[kk];
          }
          DotC<jj + 1, double>::template f<jj>(acc, xs, ps);
          Mrow[jj] = acc;
        });
        if constexpr (FORM == FACTOR_M) {
          if (store && vi) {
            const gptr<double> dst = as_global(L.M64 + (size_t)(s + 1) * nn + (size_t)i * n);
#pragma unroll
            for (int j = 0; j < n; ++j) dst[j] = Mrow[j];
          }
        }
        if constexpr (!HOIST) {
#pragma unroll
          for (int r = 0; r < NX; ++r) ApcPrev[r] = cur.Apc[r];
          cur = nxt;
        }
      }
#pragma unroll
      for (int j = 0; j < n; ++j) Xprev[j] = X[j];
    }
  };

  // phase 1
#pragma unroll
  for (int j = 0; j < n; ++j) {
    Mrow[j] = 0.0;
    Xprev[j] = 0.0;
    UT[j] = (i == j) ? 1.0 : 0.0;
    Kaa[j] = 0.0;
  }
  sweep(std::true_type{}, fac_chunk<NR>(q, N), q == 0, fac_chunk<NR>(0, N).len);
  if (q == 0) {
    store_row(FX_M1, Mrow);
    store_row(FX_X0, Xprev);
  }
  __syncthreads();  // every wavefront of the caller's workgroup

  // phase 2: entering states of chunks 2..R (every row computes them all)
  double M[n], Xb[n];
  load_row<n>(M, FX + FX_M1 * nn + (size_t)ic * n, true);
  load_row<n>(Xb, FX + FX_X0 * nn + (size_t)ic * n, true);
#pragma unroll
  for (int j = 0; j < n; ++j) {
    Mrow[j] = M[j];
    Xprev[j] = Xb[j];
  }
  for (int c = 1; c <= NR - 1; ++c) {
    double S0[n], Ka[n], Kb[n], Ph[n];
    const size_t base = (size_t)(FX_SUM + 4 * (c - 1)) * nn + (size_t)ic * n;
    load_row<n>(S0, FX + base, true);
    load_row<n>(Ka, FX + base + nn, true);
    load_row<n>(Kb, FX + base + 2 * nn, true);
    load_row<n>(Ph, FX + base + 3 * nn, true);
    // R = I - M' K_aa M = C C'
    double MT[n], E1[n], Y[n], R[n];
#pragma unroll
    for (int j = 0; j < n; ++j) {
      MT[j] = 0.0;
      E1[j] = (i == j) ? 1.0 : 0.0;
    }
    cross_row<n, n>(E1, M, MT, 1.0);  // row i of M'
    sfor<0, n>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      Y[jj] = dotb<n>(Ka, M[jj], 0.0);  // K_aa M
    });
    sfor<0, n>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      R[jj] = E1[jj] - dotb<n>(MT, Y[jj], 0.0);
    });
    double Ci[n];
    bad |= chol_inv<n>(R, Ci, i);
    // P = K_ba M C^{-T};  S_b = S0_b - P P'
    double KM[n], P[n];
    sfor<0, n>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      KM[jj] = dotb<n>(Kb, M[jj], 0.0);
      P[jj] = 0.0;
    });
    cross_row<n, n>(KM, Ci, P, 1.0);
    cross_row<n, n>(P, P, S0, -1.0);
    bad |= chol_inv<n>(S0, Xb, i);
    // M_{a_{c+1}} = Phi_b L_b^{-T}
#pragma unroll
    for (int j = 0; j < n; ++j) M[j] = 0.0;
    cross_row<n, n>(Ph, Xb, M, 1.0);
    const bool take = (q == c + 1) || (c == NR - 1 && q == 0);
    if (take) {
#pragma unroll
      for (int j = 0; j < n; ++j) {
        Mrow[j] = M[j];
        Xprev[j] = Xb[j];
      }
    }
  }

  // phase 3
  sweep(std::false_type{}, fac_chunk<NR>(q == 0 ? NR : q, N), true, fac_chunk<NR>(1, N).len);
  return __ballot(bad != 0) != 0ull ? 1 : 0;
}

}  // namespace ocpk
