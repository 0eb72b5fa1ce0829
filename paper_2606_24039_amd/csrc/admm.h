// Building blocks of the ADMM iteration of Algorithm 3 (the iteration itself
// is in wave.h): the slack/projection update of one inequality row, the
// compile-time structure of the per-iteration data, the time-invariant blocks
// held in registers and the per-solve initialisation.
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

// Time-invariant blocks in FP64 (FP64 residuals, adjoint sweeps), read once:
// row / column `lane` of D (interior, and the terminal minus the interior),
// E (zero if absent), A^-, A^+ and G (the last two only without the
// explicit-dynamics / selection structure).
template <int NX, int NU, int NG, typename ST>
struct TIBlocks64 {
  static constexpr int n = NX + NU;
  double Dr[n], dDN[n];
  double Er[n], Ec[n];
  double Amc[NX], Amr[n];
  double Apc[ST::APNEG ? 1 : NX], Apr[ST::APNEG ? 1 : n];
  double Gc[ST::GSEL ? 1 : NG], Gr[ST::GSEL ? 1 : n];
  __device__ void load(const Layout& L, int b, int i) {
    const size_t nn = (size_t)n * n;
    const int ic = i < n ? i : n - 1, ix = i < NX ? i : NX - 1, ig = i < NG ? i : NG - 1;
    const double* D = L.D + (size_t)(2 * b) * nn;
    load_row<n>(Dr, D + (size_t)ic * n, true);
    load_row<n>(dDN, D + nn + (size_t)ic * n, true);
#pragma unroll
    for (int k = 0; k < n; ++k) dDN[k] -= Dr[k];
    if (L.E) {
      load_row<n>(Er, L.E + (size_t)b * nn + (size_t)ic * n, true);
      load_col<n>(Ec, L.E + (size_t)b * nn + ic, n, true);
    } else {
#pragma unroll
      for (int k = 0; k < n; ++k) Er[k] = Ec[k] = 0.0;
    }
    const double* Am = L.Am + (size_t)b * NX * n;
    load_col<NX>(Amc, Am + ic, n, true);
    load_row<n>(Amr, Am + (size_t)ix * n, i < NX);
    if constexpr (!ST::APNEG) {
      const double* Ap = L.Ap + (size_t)b * NX * n;
      load_col<NX>(Apc, Ap + ic, n, true);
      load_row<n>(Apr, Ap + (size_t)ix * n, i < NX);
    }
    if constexpr (!ST::GSEL) {
      const double* G = L.G + (size_t)b * NG * n;
      load_col<NG>(Gc, G + ic, n, true);
      load_row<n>(Gr, G + (size_t)ig * n, i < NG);
    }
  }
};

// prefetch distance (stages) of the substitution chains (a chain stage holds
// one n-row of a chain block plus one vector entry): eight stages, four for
// FP64 rows longer than 8 (register budget).  FP64 at n = 6 with eight:
// adjoint -6 %, plain-FP64 bicycle solve of 4096 x N = 100 -7 %.
template <typename T, int n>
constexpr int chain_prefetch() {
  return (sizeof(T) == 8 && n > 8) ? 4 : 8;
}

// residuals and scales of the QP the iterations run on (rp, rd, ps, ds: the
// step-size update), and of the original problem (the _u fields, equal without
// rescaling: the stopping test and the reported residuals)
struct Resid {
  double rp, rd, ps, ds;
  double rp_u, rd_u, ps_u, ds_u;
  int nonfinite;
};

// Per-lane weights that take a residual entry of the rescaled QP to the
// original problem: equality rows (lane = state component) d_x, inequality
// rows 1/e_g, stationarity rows (lane = variable component) 1/(c d), slack
// terms 1/c.  All 1 without rescaling.
struct ResW {
  double f, g, d, s;
  __device__ __forceinline__ void load(const Layout& L, int b, int i) {
    if (!L.sc) {
      f = g = d = s = 1.0;
      return;
    }
    const double* p = L.sc + (size_t)b * 3 * ROW;
    const double di = p[i], ei = p[ROW + i], c = p[2 * ROW + i];
    f = di;
    g = 1.0 / ei;
    d = 1.0 / (c * di);
    s = 1.0 / c;
  }
};

constexpr int32_t ST_RUNNING = -1;

// Per-instance start of a solve: status, counters, rho; zero state on a cold
// start.  One thread per padded state entry (and per instance for scalars).
template <typename T>
__global__ void admm_init_kernel(Layout L, Settings st, int32_t* __restrict__ need) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0 && L.tail_count) *L.tail_count = 0;
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

}  // namespace ocpk
