// Device-side building blocks shared by the OCP-QP kernels (gfx950 / CDNA4).
//
// Execution model: one optimal-control instance per 16-lane DPP row of a
// 64-wide wavefront.  Lane i of the row owns component i of every stage
// vector (i < n = nx + nu), row i of every dynamics block (i < nx) and row i
// of every inequality block (i < ng).  Small dense block products broadcast
// one lane's value to the whole row with DPP row_newbcast (no LDS, no
// barriers); row-wide max/sum reductions use DPP row_ror butterflies.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dpp_dot.h"

namespace ocpk {

constexpr int ROW = 16;  // lanes per instance (one DPP row)

// Padding stages on both sides of the factor-block and state buffers the
// iteration streams: prefetches run up to this many stages past either end
// of an instance without clamping (what they read there is never used).
constexpr int STAGE_PAD = 8;

// Instance slot of this 16-lane row: a workgroup of 16 * R threads holds R
// instances.  The sweeps are issue-bound per wavefront, so R = 4 (a full
// wave of instances) does four times the work per issued instruction of
// R = 1.
__device__ __forceinline__ int row_slot() { return blockIdx.x * (blockDim.x >> 4) + (threadIdx.x >> 4); }

// compile-time loop: f(std::integral_constant<int, I>) for I in [B, E)
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

// value of lane J of this 16-lane row, for every lane of the row
template <int J, typename T>
__device__ __forceinline__ T bc(T v) {
  static_assert(J >= 0 && J < ROW, "broadcast lane out of row");
  return __builtin_amdgcn_update_dpp(v, v, 0x150 + J, 0xf, 0xf, true);
}

template <int CTRL, typename T>
__device__ __forceinline__ T dpp(T v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}

// row-wide max / sum (all 16 lanes receive the result)
template <typename T>
__device__ __forceinline__ T row_max(T v) {
  v = fmax(v, dpp<0x128>(v));
  v = fmax(v, dpp<0x124>(v));
  v = fmax(v, dpp<0x122>(v));
  v = fmax(v, dpp<0x121>(v));
  return v;
}
template <typename T>
__device__ __forceinline__ T row_sum(T v) {
  v += dpp<0x128>(v);
  v += dpp<0x124>(v);
  v += dpp<0x122>(v);
  v += dpp<0x121>(v);
  return v;
}

// acc + sum_{k<K} a[k] * (value of lane k): one inline-assembly block of K
// DPP-sourced FMAs (dpp_dot.h)
template <int K, typename T>
__device__ __forceinline__ T dotb(const T (&a)[K], T v, T acc) {
  return dotb_asm<K>(a, v, acc);
}

// Products with the packed FP32 inverse factor (factor.h, FACTOR_WV): lane i
// of a row holds c[e] = Linv[max(i,s)][min(i,s)], s = (i - e) mod K, so
//   dotl: acc + sum_{j<=i} Linv[i][j] v_j       (row_shr by i - j)
//   dotu: acc + sum_{j>=i} Linv[j][i] v_j       (row_shl by j - i)
// (lanes j >= K of v must be zero in dotu)
template <int K>
__device__ __forceinline__ float dotl(const float (&c)[K], float v, float acc) {
  return dotl_asm<K>(c, v, acc);
}
template <int K>
__device__ __forceinline__ float dotu(const float (&c)[K], float v, float acc) {
  return dotu_asm<K>(c, v, acc);
}

// value of lane `src` (0..15) of this 16-lane row (ds_bpermute)
__device__ __forceinline__ float row_gather(float v, int src) {
  const int addr = ((int)(threadIdx.x & ~(ROW - 1)) + src) << 2;
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double row_gather(double v, int src) {
  const int addr = ((int)(threadIdx.x & ~(ROW - 1)) + src) << 2;
  const long long u = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(u & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(u >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Every buffer the kernels touch is device (global) memory.  Pointers that
// reach a kernel through a structure whose address escapes (passed by
// reference to a non-inlined function) lose that knowledge and would compile
// to flat accesses; the helpers below restore it.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}
template <typename T>
__device__ __forceinline__ gptr<const T> as_global(const T* p) {
  return (gptr<const T>)p;
}
template <typename T>
__device__ __forceinline__ gptr<T> as_global(gptr<T> p) {
  return p;
}
template <typename T>
__device__ __forceinline__ gptr<const T> as_global(gptr<const T> p) {
  return p;
}

template <int K, typename T, typename PT>
__device__ __forceinline__ void load_row(T (&dst)[K], PT p_, bool valid) {
  const gptr<const T> p = as_global(p_);
#pragma unroll
  for (int k = 0; k < K; ++k) dst[k] = valid ? p[k] : T(0);
}
// dst[r] = base[r * stride] for r < R
template <int R, typename T, typename PT>
__device__ __forceinline__ void load_col(T (&dst)[R], PT p_, int stride, bool valid) {
  const gptr<const T> p = as_global(p_);
#pragma unroll
  for (int r = 0; r < R; ++r) dst[r] = valid ? p[r * stride] : T(0);
}
template <int K, typename TD, typename TS>
__device__ __forceinline__ void load_row_cvt(TD (&dst)[K], const TS* __restrict__ p_, bool valid) {
  const gptr<const TS> p = as_global(p_);
#pragma unroll
  for (int k = 0; k < K; ++k) dst[k] = valid ? TD(p[k]) : TD(0);
}
template <int R, typename TD, typename TS>
__device__ __forceinline__ void load_col_cvt(TD (&dst)[R], const TS* __restrict__ p_, int stride, bool valid) {
  const gptr<const TS> p = as_global(p_);
#pragma unroll
  for (int r = 0; r < R; ++r) dst[r] = valid ? TD(p[r * stride]) : TD(0);
}

template <typename T>
__device__ __forceinline__ T clampv(T v, T lo, T hi) {
  return fmin(fmax(v, lo), hi);
}

// ---------------------------------------------------------------------------
// Problem / workspace description passed by value to every kernel.
// Stage-vector buffers use a padded stride of ROW (=16) entries per stage.
// ---------------------------------------------------------------------------
struct Layout {
  int B, nx, nu, ng, n;
  const int64_t* stage_off;  // [B+1]
  const int32_t* order;      // [B] instance processed by row g (longest horizon first)
  int ti;                    // 1: D,E,Am,Ap,bd,G,lo,hi stored once per instance

  // QP data, FP64 master copy
  const double* D;       // ti: [2B][n][n] (interior, terminal)   tv: [S][n][n]
  const double* E;       // ti: [B][n][n]  tv: [S][n][n]  (block (t+1,t)); may be null
  const double* q;       // [S][n]; may be null
  const double* Am;      // ti: [B][nx][n]  tv: [S][nx][n]
  const double* Ap;      // ti: [B][nx][n]  tv: [S][nx][n]
  const double* bd;      // ti: [B][nx]     tv: [S][nx]; may be null
  const double* G;       // ti: [B][ng][n]  tv: [S][ng][n]
  const double* lo;      // ti: [B][ng]     tv: [S][ng]
  const double* hi;
  const double* x_init;  // [B][nx]
  const uint8_t* soft;   // [ng]
  double gamma2, gamma1;
  // problem rescaling (Remark 4), [B][3][ROW]: variable factors d (x = d xh),
  // inequality-row factors e_g, and the cost factor c in every lane of the
  // third row; the data above are those of the rescaled QP.  Null: none.
  const double* sc;

  // iteration-precision copies of the data read every ADMM iteration
  const void* AmT;
  const void* ApT;
  const void* GT;
  const void* qT;
  const void* bdT;
  const void* loT;
  const void* hiT;
  const void* xinitT;

  // factor, [S][n][n] row-major.  FP64 Linv_t and M_t (adjoint); in
  // iteration precision the blocks the ADMM substitutions read (factor.h,
  // FACTOR_WV / FACTOR_PK): SubA multiplies eta_t (FP32: the packed Linv_t,
  // which also gives Linv_t' v), SubB the forward result (FP64: P_t), ChF /
  // ChB carry the forward / backward chains
  double* Linv64;
  double* M64;
  void* SubA;
  void* SubB;
  void* ChF;
  void* ChB;
  // segmented substitutions: per instance and horizon quarter q, the
  // transfer blocks of the forward / backward chain over the quarter
  // ([B][4][n][n], iteration precision) and exchange slots ([B][8][ROW])
  void* SegT;
  void* SegU;
  void* SegX;
  // chunked factorisation: per instance [FX_SLOTS][n][n] FP64 exchange blocks
  double* FacX;
  // instances solved by a multi-wavefront workgroup (horizon N >= mw_min_n):
  // their list [n_mw] and per list slot the chunked factorisation's exchange
  // blocks of the workgroup's rows
  const int32_t* mw_list;
  int n_mw, mw_min_n;
  double* FacXmw;
  // continuation of one-wavefront instances on two-wavefront workgroups
  // (Settings::tail_after): the instances handed over, their count (cleared
  // by the per-solve init), per instance the state bits of the hand-over
  // (bit 0: factorisation due, bit 1: multipliers of a check kept), and per
  // list slot the chunked factorisation's exchange blocks
  int32_t* tail_list;
  int32_t* tail_count;
  int32_t* tail_flags;
  double* FacXtail;
  // PCG primal updates (pcg != 0): at most pcg_max_it iterations to the
  // relative residual pcg_tol; vectors [S][ROW] in iteration precision,
  // padded like the state vectors (x~, r, z, p, S p)
  int pcg, pcg_max_it;
  double pcg_tol;
  void *pcg_xt, *pcg_r, *pcg_z, *pcg_p, *pcg_sp;
  // structure of time-invariant LTI data: G rows are unit selectors
  int8_t gsel[16];  // variable selected by inequality row r
  int8_t ginv[16];  // inequality row selecting variable i, or -1

  // ADMM state in iteration precision; stage vectors padded to ROW
  void* x;   // [S][ROW]
  void* v;   // [S][ROW] forward-substitution scratch
  void* yf;  // [S][ROW] slot of stage t: dynamics row t; slot of stage N: the initial-state rows
  void* zg;  // [S][ROW]
  void* yg;  // [S][ROW]
  void* xi;  // [S][ROW]
  void* ypf;  // [S][ROW] y_f and y_g at the previous convergence check (infeasibility test)
  void* ypg;

  // per instance
  double* rho;
  int32_t* status;
  int32_t* iters;
  int32_t* nfact;
  double* rprim;
  double* rdual;
  unsigned init_blocks;  // grid of the per-entry init kernels
};

struct Settings {
  double sigma, rho0, rho_f_scale, rho_min, rho_max, k_ratio, alpha, eps_abs, eps_rel;
  double eps_pinf;  // primal-infeasibility certificate tolerance (0: no test)
  int max_iter, k_rho, k_check, adapt_rho, warm;
  int seg_min_n;  // horizons N >= seg_min_n run the segmented substitutions
  int seg_after;  // from this iteration on every instance (N >= 15) runs them (the batch's tail)
  int tail_after;  // > 0: one-wavefront instances still running at this iteration continue on a
                   // two-wavefront workgroup (admm_solve_tail_kernel); 0: off
};

struct Group {
  int lane;    // 0..15
  int b;       // instance
  int64_t s0;  // first stage
  int N;       // horizon (stages 0..N)
};

// Wave-uniform copies of values that reach a non-inlined function in vector
// registers or through memory (every lane holds the same value): with them
// the callee keeps its base pointers and loop bounds in scalar registers and
// addresses memory as scalar base + vector offset.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint64_t u = (uint64_t)v;
  return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u));
}
__device__ __forceinline__ double uni(double v) { return __builtin_bit_cast(double, uni(__builtin_bit_cast(int64_t, v))); }
template <typename P>
__device__ __forceinline__ P* uni(P* p) {
  return (P*)uni((int64_t)p);
}
__device__ __forceinline__ Layout uni(const Layout& L) {
  Layout u = L;
  u.B = uni(L.B), u.nx = uni(L.nx), u.nu = uni(L.nu), u.ng = uni(L.ng), u.n = uni(L.n), u.ti = uni(L.ti);
  u.stage_off = uni(L.stage_off), u.order = uni(L.order);
  u.D = uni(L.D), u.E = uni(L.E), u.q = uni(L.q), u.Am = uni(L.Am), u.Ap = uni(L.Ap), u.bd = uni(L.bd);
  u.G = uni(L.G), u.lo = uni(L.lo), u.hi = uni(L.hi), u.x_init = uni(L.x_init), u.soft = uni(L.soft);
  u.gamma2 = uni(L.gamma2), u.gamma1 = uni(L.gamma1);
  u.AmT = uni(L.AmT), u.ApT = uni(L.ApT), u.GT = uni(L.GT), u.qT = uni(L.qT), u.bdT = uni(L.bdT);
  u.loT = uni(L.loT), u.hiT = uni(L.hiT), u.xinitT = uni(L.xinitT);
  u.Linv64 = uni(L.Linv64), u.M64 = uni(L.M64);
  u.SubA = uni(L.SubA), u.SubB = uni(L.SubB), u.ChF = uni(L.ChF), u.ChB = uni(L.ChB);
  u.SegT = uni(L.SegT), u.SegU = uni(L.SegU), u.SegX = uni(L.SegX), u.FacX = uni(L.FacX);
  u.mw_list = uni(L.mw_list), u.n_mw = uni(L.n_mw), u.mw_min_n = uni(L.mw_min_n), u.FacXmw = uni(L.FacXmw);
  u.tail_list = uni(L.tail_list), u.tail_count = uni(L.tail_count), u.tail_flags = uni(L.tail_flags);
  u.FacXtail = uni(L.FacXtail);
  u.pcg = uni(L.pcg), u.pcg_max_it = uni(L.pcg_max_it), u.pcg_tol = uni(L.pcg_tol);
  u.pcg_xt = uni(L.pcg_xt), u.pcg_r = uni(L.pcg_r), u.pcg_z = uni(L.pcg_z), u.pcg_p = uni(L.pcg_p);
  u.pcg_sp = uni(L.pcg_sp);
  u.x = uni(L.x), u.v = uni(L.v), u.yf = uni(L.yf), u.zg = uni(L.zg), u.yg = uni(L.yg), u.xi = uni(L.xi);
  u.rho = uni(L.rho), u.status = uni(L.status), u.iters = uni(L.iters), u.nfact = uni(L.nfact);
  u.rprim = uni(L.rprim), u.rdual = uni(L.rdual);
  return u;
}

__device__ __forceinline__ size_t ti_or_tv(int ti, int b, int64_t s, size_t sz) {
  return ti ? (size_t)b * sz : (size_t)s * sz;
}

}  // namespace ocpk
