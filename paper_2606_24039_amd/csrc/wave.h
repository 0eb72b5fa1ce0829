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
// wavefront).  A stage-parallel pass walks 4-stage blocks; all blocks but
// the last hold stages t < N only and run without masks.
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


// ---------------------------------------------------------------------------
// Addressing.  Every buffer the iteration streams is reached from a
// wave-uniform base pointer (scalar registers) plus a 32-bit per-lane byte
// offset, so that loads and stores take the scalar-base + vector-offset form
// and the constant stage steps fold into the instructions' immediate offsets.
// The bases of the padded buffers (factor products, stage vectors) sit
// STAGE_PAD stages before stage 0 of the instance, so the offsets of the
// accesses before stage 0 (y_f,t-1 at t = 0, the backward-chain prefetch)
// stay non-negative.
// ---------------------------------------------------------------------------
template <int IMM = 0, typename T>
__device__ __forceinline__ std::remove_const_t<T> ldo(gptr<T> base, uint32_t off) {
  return *(gptr<const T>)((gptr<const char>)base + off + IMM);
}
template <int IMM = 0, typename T>
__device__ __forceinline__ void sto(gptr<T> base, uint32_t off, T v) {
  *(gptr<T>)((gptr<char>)base + off + IMM) = v;
}
// the same for a wavefront's LDS (the per-instance exchange vector)
template <typename T>
using lptr = __attribute__((address_space(3))) T*;
template <int IMM = 0, typename T>
__device__ __forceinline__ std::remove_const_t<T> ldo(lptr<T> base, uint32_t off) {
  return *(lptr<const T>)((lptr<const char>)base + off + IMM);
}
template <int IMM = 0, typename T>
__device__ __forceinline__ void sto(lptr<T> base, uint32_t off, T v) {
  *(lptr<T>)((lptr<char>)base + off + IMM) = v;
}
// LDS stages of the exchange vector: horizons with N + 1 + 2 STAGE_PAD + 8
// stages or fewer keep it in LDS (16 KB per wavefront in FP32)
constexpr int XV_LDS_STAGES = 256;
constexpr int STATE_LDS_STAGES = 80;  // FP32: six vectors of 80 stages (30 KB), horizons up to 55
__device__ __forceinline__ bool xv_in_lds(int N) { return N + 1 + 2 * STAGE_PAD + 8 <= XV_LDS_STAGES; }
// ordering of a wavefront's own LDS writes before its later LDS reads by
// other lanes (one wavefront per workgroup: no barrier needed)
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
// K consecutive entries from base + off (16-byte aligned: whole 16-byte
// loads), or K entries STRIDE apart
template <typename T>
struct Vec16 {
  static constexpr int N = 16 / (int)sizeof(T);
  typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
};
template <int K, int STRIDE = 1, typename T>
__device__ __forceinline__ void ldo_n(T (&d)[K], gptr<const T> base, uint32_t off) {
  using V = Vec16<T>;
  if constexpr (STRIDE == 1 && K % V::N == 0) {
    const gptr<const typename V::type> p = (gptr<const typename V::type>)((gptr<const char>)base + off);
#pragma unroll
    for (int k = 0; k < K / V::N; ++k) {
      const typename V::type u = p[k];
#pragma unroll
      for (int e = 0; e < V::N; ++e) d[V::N * k + e] = u[e];
    }
  } else {
    const gptr<const T> p = (gptr<const T>)((gptr<const char>)base + off);
#pragma unroll
    for (int k = 0; k < K; ++k) d[k] = p[k * STRIDE];
  }
}

template <int K, typename T>
__device__ __forceinline__ void ldo_n(T (&d)[K], lptr<const T> base, uint32_t off) {
  const lptr<const T> p = (lptr<const T>)((lptr<const char>)base + off);
#pragma unroll
  for (int k = 0; k < K; ++k) d[k] = p[k];
}

// Uniform base pointers of one instance.
template <typename T, int NX, int NU, int NG, bool LV = false>
struct IterPtrs {
  static constexpr int n = NX + NU;
  using VP = std::conditional_t<LV, lptr<T>, gptr<T>>;
  gptr<const T> SA, SB, CF, CB;  // factor products (SubA, SubB, ChF, ChB), at stage -STAGE_PAD
  VP x, v, yf, zg, yg, xi;       // stage vectors (global, or LDS copies), at stage -STAGE_PAD
  gptr<const T> Am, Ap, G;       // TI: the instance's blocks; TV: stage 0 of the instance
  gptr<const T> lo, hi, bd;      // likewise (bd may be null)
  gptr<const T> q;               // stage 0 of the instance (may be null)
  __device__ IterPtrs(const Layout& L, int b, int64_t s0) {
    const int64_t nn = (int64_t)n * n;
    const int64_t sp = s0 - STAGE_PAD;
    const int64_t u = L.ti ? (int64_t)b : s0;  // unit of the constraint data
    SA = L.SubA ? as_global((const T*)L.SubA + sp * nn) : nullptr;
    SB = as_global((const T*)L.SubB + sp * nn);
    CF = as_global((const T*)L.ChF + sp * nn);
    CB = as_global((const T*)L.ChB + sp * nn);
    x = as_global((T*)L.x + sp * ROW);
    v = as_global((T*)L.v + sp * ROW);
    yf = as_global((T*)L.yf + sp * ROW);
    zg = as_global((T*)L.zg + sp * ROW);
    yg = as_global((T*)L.yg + sp * ROW);
    xi = as_global((T*)L.xi + sp * ROW);
    Am = as_global((const T*)L.AmT + u * NX * n);
    Ap = as_global((const T*)L.ApT + u * NX * n);
    G = as_global((const T*)L.GT + u * NG * n);
    lo = as_global((const T*)L.loT + u * NG);
    hi = as_global((const T*)L.hiT + u * NG);
    bd = L.bdT ? as_global((const T*)L.bdT + u * NX) : nullptr;
    q = L.qT ? as_global((const T*)L.qT + s0 * n) : nullptr;
  }
  // the same data with the stage vectors in LDS: vector k at base + k * stages * ROW
  template <bool LV2 = LV, typename = std::enable_if_t<LV2>>
  __device__ IterPtrs(const IterPtrs<T, NX, NU, NG, false>& g, lptr<T> base, int stages)
      : SA(g.SA), SB(g.SB), CF(g.CF), CB(g.CB), Am(g.Am), Ap(g.Ap), G(g.G), lo(g.lo), hi(g.hi), bd(g.bd), q(g.q) {
    x = base;
    v = base + stages * ROW;
    yf = base + 2 * stages * ROW;
    zg = base + 3 * stages * ROW;
    yg = base + 4 * stages * ROW;
    xi = base + 5 * stages * ROW;
  }
};

__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// chain inputs of one stage: row `lane` of a chain block and one vector entry
template <typename T, int n>
struct ChainIn {
  T A[n];
  T r;
};

// One substitution chain on row 0: y_t = R_t - B_t y_prev over the stages in
// `dir` order (+1: 0..N with B = ChF; -1: N..0 with B = ChB); y_t -> R_t.
// R, Bm: biased bases; orow / oblk: this lane's offsets at stage 0.  The
// running stage position lives in the (uniform) base pointers, the lane
// offsets stay fixed.
template <typename T, int n, int DIR, typename RP>
__device__ __forceinline__ void chain(RP R, gptr<const T> Bm, uint32_t orow, uint32_t oblk, int N) {
  constexpr int PF = chain_prefetch<T, n>();
  static_assert(PF <= STAGE_PAD, "prefetch reaches past the buffer padding");
  constexpr int VS = DIR * ROW * (int)sizeof(T);  // one step of the sweep in a vector, bytes
  constexpr long BS = DIR * (long)n * n;          // one step in the blocks, elements
  // bases at the sweep's k0-th stage (t = 0 forward, t = N backward);
  // prefetches run up to PF stages past either end of the instance, into
  // the neighbouring instances or the padding
  RP Rk = R + (DIR > 0 ? 0 : (long)N * ROW);
  gptr<const T> Bk = Bm + (DIR > 0 ? 0 : (long)N * n * n);
  ChainIn<T, n> buf[PF];
  auto load = [&](ChainIn<T, n>& d, auto j) {
    constexpr int jj = decltype(j)::value;
    ldo_n<n>(d.A, Bk + jj * BS, oblk);
    d.r = ldo<jj * VS>(Rk, orow);
  };
  sfor<0, PF>([&](auto j) { load(buf[decltype(j)::value], j); });
  T yprev = T(0);
  auto body = [&](auto j) {
    constexpr int jj = decltype(j)::value;
    ChainIn<T, n>& d = buf[jj];
    const T y = d.r - dotb<n>(d.A, yprev, T(0));  // stage 0 / N chain blocks are zero slots
    sto<jj * VS>(Rk, orow, y);
    yprev = y;
    load(d, std::integral_constant<int, jj + PF>{});
  };
  int k0 = 0;
  for (; k0 + PF - 1 <= N; k0 += PF) {
    sfor<0, PF>(body);
    Rk += PF * DIR * ROW;
    Bk += PF * BS;
  }
  sfor<0, PF>([&](auto j) {
    if (k0 + decltype(j)::value <= N) body(j);
  });
}

// The same chain on all four rows (FP32, n a multiple of 4): row q holds
// columns q n/4 .. (q+1) n/4 - 1 of the chain block's rows, multiplies them
// with the matching entries of y_prev (moved to lanes 0..n/4-1 of the row
// by a row-masked DPP shift) and the four partial sums are added across the
// rows by two permlane swaps, which leaves the same y_t on every row.  Per
// stage: three shifts, n/4 broadcast FMAs and the two swap-adds in place of
// n broadcast FMAs on one row, and one 16-byte load per lane.
template <int n, int DIR, typename RP>
__device__ __forceinline__ void chain_rows(RP R, gptr<const float> Bm, uint32_t orow, uint32_t oblk, int N) {
  static_assert(n % 4 == 0 && n <= ROW, "row-split chain needs n = 4k <= 16");
  constexpr int QS = n / 4;
  constexpr int PF = chain_prefetch<float, n>();
  static_assert(PF <= STAGE_PAD, "prefetch reaches past the buffer padding");
  constexpr int VS = DIR * ROW * (int)sizeof(float);
  constexpr long BS = DIR * (long)n * n;
  RP Rk = R + (DIR > 0 ? 0 : (long)N * ROW);
  gptr<const float> Bk = Bm + (DIR > 0 ? 0 : (long)N * n * n);
  struct In {
    float A[QS];
    float r;
  };
  In buf[PF];
  auto load = [&](In& d, auto j) {
    constexpr int jj = decltype(j)::value;
    ldo_n<QS>(d.A, Bk + jj * BS, oblk);
    d.r = ldo<jj * VS>(Rk, orow);
  };
  sfor<0, PF>([&](auto j) { load(buf[decltype(j)::value], j); });
  float y = 0.f;
  auto body = [&](auto j) {
    constexpr int jj = decltype(j)::value;
    In& d = buf[jj];
    float z = y;  // row q: y[q QS + k] at lane k
    z = __builtin_amdgcn_update_dpp(z, y, 0x100 + QS, 0x2, 0xf, false);
    z = __builtin_amdgcn_update_dpp(z, y, 0x100 + 2 * QS, 0x4, 0xf, false);
    z = __builtin_amdgcn_update_dpp(z, y, 0x100 + 3 * QS, 0x8, 0xf, false);
    const float pq = dotb<QS>(d.A, z, 0.f);
    const unsigned ub = __builtin_bit_cast(unsigned, pq);
    const auto h = __builtin_amdgcn_permlane32_swap(ub, ub, false, false);  // rows q, q^2
    const float c = __builtin_bit_cast(float, (unsigned)h[0]) + __builtin_bit_cast(float, (unsigned)h[1]);
    const unsigned uc = __builtin_bit_cast(unsigned, c);
    const auto g = __builtin_amdgcn_permlane16_swap(uc, uc, false, false);  // rows q, q^1
    const float sum = __builtin_bit_cast(float, (unsigned)g[0]) + __builtin_bit_cast(float, (unsigned)g[1]);
    y = d.r - sum;  // stage 0 / N chain blocks are zero slots
    sto<jj * VS>(Rk, orow, y);
    load(d, std::integral_constant<int, jj + PF>{});
  };
  int k0 = 0;
  for (; k0 + PF - 1 <= N; k0 += PF) {
    sfor<0, PF>(body);
    Rk += PF * DIR * ROW;
    Bk += PF * BS;
  }
  sfor<0, PF>([&](auto j) {
    if (k0 + decltype(j)::value <= N) body(j);
  });
}

// FP32 chains with n = 4k run on all four rows
template <typename T, int n>
constexpr bool ROWSPLIT_CHAIN = sizeof(T) == 4 && n % 4 == 0 && n <= ROW;

// Scalars of one ADMM iteration of one instance (this lane's view).
template <typename T, int NX, int NU, int NG, typename ST, bool LV = false>
struct IterCtx {
  const TIBlocks<T, NX, NU, NG>& tb;
  const IterPtrs<T, NX, NU, NG, LV>& P;
  T sigma, rho_f, rho_g, alpha, oma, rfa;
  int kind;
  ProjConst<T> pc;
  T xinit, yinit;
  int gsel, ginv;
  int i, q, N;
  bool gid;   // (uniform) the selection of every inequality row r < ng is variable r
  bool hard;  // (uniform) no soft inequality rows
};

// this lane's byte offsets at block 0 (stage q of row q)
template <typename T, int n>
struct LaneOff {
  static constexpr uint32_t VS = ROW * sizeof(T);          // one stage of a vector
  static constexpr uint32_t FS = (uint32_t)n * n * sizeof(T);  // one stage of a factor product
  static constexpr uint32_t VB = 4 * VS, FB = 4 * FS;      // one 4-stage block
  uint32_t v, f;  // entry `lane` of the vectors / row `lane` of the factor products
  uint32_t v0;    // entry `lane` of stage 0 (every row)
  uint32_t fq;    // stage 0, row `lane`, columns q n/4.. (row-split chains)
  __device__ LaneOff(int q, int lane) {
    const int ir = lane < n ? lane : n - 1;
    v = (uint32_t)(((STAGE_PAD + q) * ROW + lane) * (int)sizeof(T));
    f = (uint32_t)(((STAGE_PAD + q) * n * n + ir * n) * (int)sizeof(T));
    v0 = (uint32_t)((STAGE_PAD * ROW + lane) * (int)sizeof(T));
    fq = (uint32_t)((STAGE_PAD * n * n + ir * n + q * (n / 4)) * (int)sizeof(T));
  }
};

// Stage blocks of a stage-parallel pass: blocks 0..nfull-1 hold four stages
// t < N each (no masking); block nfull holds the rest (t = 4 nfull + q up to
// N, rows past N idle).  Inputs are loaded D-1 blocks ahead into D rotating
// buffers; the loop body is unrolled D times so that every buffer index is a
// compile-time constant.  Loads run at most 4 (D - 1) + 3 stages past the
// tail block's first stage (into padding or the next instance; unused).
template <int D>
constexpr int stage_blocks_reach() {
  return 4 * (D - 1) + 3;
}
template <int D, typename In, typename Load, typename Comp>
__device__ __forceinline__ void stage_blocks(int nfull, Load&& load, Comp&& comp) {
  static_assert(stage_blocks_reach<D>() - 3 <= STAGE_PAD, "stage-block prefetch reaches past the padding");
  In buf[D];
  sfor<0, D - 1>([&](auto j) { load(buf[decltype(j)::value], decltype(j)::value); });
  int blk = 0;
  for (; blk + D <= nfull; blk += D) {
    sfor<0, D>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      load(buf[(jj + D - 1) % D], blk + jj + D - 1);
      comp(buf[jj], blk + jj, std::true_type{});
    });
  }
  // fewer than D full blocks and the tail block remain
  bool done = false;
  sfor<0, D>([&](auto j) {
    constexpr int jj = decltype(j)::value;
    const int bb = blk + jj;
    if (done) return;
    if (bb + D - 1 <= nfull) load(buf[(jj + D - 1) % D], bb + D - 1);
    if (bb < nfull) {
      comp(buf[jj], bb, std::true_type{});
    } else {
      comp(buf[jj], bb, std::false_type{});
      done = true;
    }
  });
}
constexpr int STAGE_BLOCK_DEPTH = 3;

// Sequential walk over the stages of a row's quarter, k = 0..steps-1 (rows
// with shorter quarters skip their last steps inside comp); the inputs of
// step k + AHEAD are loaded while step k computes.  Loads run up to AHEAD
// steps past a quarter's end (into the neighbouring quarter or padding).
template <int AHEAD, typename In, typename Load, typename Comp>
__device__ __forceinline__ void seg_walk(int steps, Load&& load, Comp&& comp) {
  constexpr int D = AHEAD + 1;
  In buf[D];
  sfor<0, AHEAD>([&](auto j) { load(buf[decltype(j)::value], decltype(j)::value); });
  int k = 0;
  for (; k + D <= steps; k += D) {
    sfor<0, D>([&](auto j) {
      constexpr int jj = decltype(j)::value;
      load(buf[(jj + AHEAD) % D], k + jj + AHEAD);
      comp(buf[jj], k + jj);
    });
  }
  sfor<0, D>([&](auto j) {
    constexpr int jj = decltype(j)::value;
    if (k + jj < steps) {
      if (k + jj + AHEAD < steps) load(buf[(jj + AHEAD) % D], k + jj + AHEAD);
      comp(buf[jj], k + jj);
    }
  });
}

// pass-1 inputs of the stage on this row
template <typename T, int NX, int NU, int NG, bool TI>
struct EtaIn {
  static constexpr int n = NX + NU;
  static constexpr bool SA = sizeof(T) == 4;  // FP32 iterations multiply by Linv_t here
  T Ar[SA ? n : 1];                           // row `lane` of SubA (packed Linv_t)
  T x, q, yf, yfm, zg, yg, bd, bdm;
  T AmC[TI ? 1 : NX], ApCm[TI ? 1 : NX], GC[TI ? 1 : NG];
};

// pass-5 inputs of the stage on this row
template <typename T, int NX, int NU, int NG, bool TI>
struct UpdIn {
  static constexpr int n = NX + NU;
  T xt, xt1;  // x~_t, x~_{t+1} (x~_{t+1} past N is never used)
  T x, yf, zg, yg, lo, hi, bd;
  T AmR[TI ? 1 : n], ApR[TI ? 1 : n], GR[TI ? 1 : n];
};

// pass-3 inputs: row `lane` of SubB (FP32: of the packed Linv_t) and v_t
template <typename T, int n>
struct TrIn {
  T Br[n];
  T v;
};

// the block pass 3 multiplies: FP32 Linv_t' (the packed Linv_t in SubA),
// FP64 P_t (SubB)
template <typename T, typename PP>
__device__ __forceinline__ gptr<const T> sub_b_ptr(const PP& P) {
  if constexpr (sizeof(T) == 4)
    return P.SA;
  else
    return P.SB;
}
// s_t = SubB_t v_t on lane i, from row i of the block sub_b_ptr points to
// (FP32: entries past n of v are zeroed for the shifted product)
template <typename T, int n>
__device__ __forceinline__ T sub_b_mul(const T (&B)[n], T v, int i) {
  if constexpr (sizeof(T) == 4)
    return dotu<n>(B, (n < ROW && i >= n) ? 0.f : v, 0.f);
  else
    return dotb<n>(B, v, T(0));
}

// r_t of the stage on this row: eta_t, times Linv_t for FP32 iterations.
// `init` is this lane's initial-state term (rho_f x_init - y_init on lanes
// < nx), added at t = 0.
template <bool FULL, bool RAW = false, typename T, int NX, int NU, int NG, typename ST, bool LV>
__device__ __forceinline__ T stage_r(const IterCtx<T, NX, NU, NG, ST, LV>& c, const EtaIn<T, NX, NU, NG, ST::TI>& cur,
                                     int t, T init) {
  constexpr int n = NX + NU;
  constexpr bool TI = ST::TI;
  const int i = c.i;
  const auto& tb = c.tb;
  T eta = c.sigma * cur.x - cur.q;
  const T w_ = ((FULL || t < c.N) && i < NX) ? c.rho_f * (TI ? tb.bd : cur.bd) - cur.yf : T(0);
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
  eta += (t == 0) ? init : T(0);
  const T u = (i < NG) ? c.rho_g * cur.zg - cur.yg : T(0);
  if constexpr (ST::GSEL) {
    if (c.gid) {
      eta += u;
    } else {
      const T gu = row_gather(u, c.ginv < 0 ? 0 : c.ginv);
      eta += (c.ginv >= 0) ? gu : T(0);
    }
  } else if constexpr (TI) {
    eta = dotb<NG>(tb.GC, u, eta);
  } else {
    eta = dotb<NG>(cur.GC, u, eta);
  }
  if constexpr (EtaIn<T, NX, NU, NG, TI>::SA && !RAW)
    return dotl<n>(cur.Ar, eta, 0.f);
  else
    return eta;
}

// over-relaxation, projection and dual update of every constraint row of
// the stage on this row, from x~_t and x~_{t+1}; stores the new state
// (rows past N store nothing, y_f only for t < N)
template <bool FULL, typename T, int NX, int NU, int NG, typename ST, bool LV>
__device__ __forceinline__ void stage_update(const IterCtx<T, NX, NU, NG, ST, LV>& c,
                                             const UpdIn<T, NX, NU, NG, ST::TI>& cur, int t, uint32_t o) {
  constexpr int n = NX + NU;
  constexpr bool TI = ST::TI;
  const auto& tb = c.tb;
  const auto& P = c.P;
  const T xt = cur.xt, xt1 = cur.xt1;
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
  const T yfn = cur.yf + c.rfa * (zf - (TI ? tb.bd : cur.bd));
  // inequality rows of stage t (lanes past ng update padding)
  T zt;
  if constexpr (ST::GSEL)
    zt = c.gid ? xt : row_gather(xt, c.gsel);
  else if constexpr (TI)
    zt = dotb<n>(tb.GR, xt, T(0));
  else
    zt = dotb<n>(cur.GR, xt, T(0));
  const T zh = c.alpha * zt + c.oma * cur.zg;
  const T pin = fma(cur.yg, c.pc.inv_rho, zh);
  const T lo = TI ? tb.lo : cur.lo, hi = TI ? tb.hi : cur.hi;
  Proj<T> pr;
  if (c.hard)
    pr = Proj<T>{clampv(pin, lo, hi), T(0)};
  else
    pr = project_row<T>(pin, lo, hi, c.kind, c.pc);
  const T ygn = cur.yg + c.rho_g * (zh - pr.z);
  const T xn = c.alpha * xt + c.oma * cur.x;
  if (FULL || t <= c.N) {
    if (FULL || t < c.N) sto(P.yf, o, yfn);
    sto(P.zg, o, pr.z);
    sto(P.xi, o, pr.xi);
    sto(P.yg, o, ygn);
    sto(P.x, o, xn);
  }
}

// One iteration on one wavefront (the vectors handed between passes go
// through the instance's v buffer).
// XV: the exchange vector -- the instance's v buffer in global memory or an
// LDS array of XV_LDS_STAGES stages (same offsets); with LDS the passes are
// ordered by LDS waits, only the state handed to the next iteration through
// global memory needs the full wait at the end.
template <typename T, int NX, int NU, int NG, typename ST, bool LV, typename XVP>
__device__ __forceinline__ void wave_iteration(const IterCtx<T, NX, NU, NG, ST, LV>& c, const LaneOff<T, NX + NU>& lo,
                                               XVP XV) {
  constexpr bool XL = !std::is_same_v<XVP, gptr<T>>;
  auto pass_sync = [] {
    if constexpr (XL)
      lds_sync();
    else
      wave_sync();
  };
  constexpr int n = NX + NU;
  constexpr bool TI = ST::TI;
  using LO = LaneOff<T, n>;
  const int N = c.N, q = c.q, i = c.i;
  const int nfull = N / 4;  // blocks whose four stages all satisfy t < N
  const auto& P = c.P;
  const int ir = i < n ? i : n - 1, ix = i < NX ? i : NX - 1, ig = i < NG ? i : NG - 1;
  const T init = (i < NX) ? c.rho_f * c.xinit - c.yinit : T(0);

  // ---------------- pass 1: r_t on row t mod 4 ----------------
  {
    using In = EtaIn<T, NX, NU, NG, TI>;
    auto load = [&](In& d, int blk) {
      const int t = 4 * blk + q;
      const uint32_t ov = lo.v + blk * LO::VB;
      if constexpr (In::SA) ldo_n<n>(d.Ar, P.SA, lo.f + blk * LO::FB);
      d.x = ldo(P.x, ov);
      d.yf = ldo(P.yf, ov);
      d.yfm = ldo<-(int)LO::VS>(P.yf, ov);
      d.zg = ldo(P.zg, ov);
      d.yg = ldo(P.yg, ov);
      // problem data is exactly sized: read at the nearest stage
      const int tc = min(t, N);
      const int tm = tc > 0 ? tc - 1 : 0;
      d.q = P.q ? ldo(P.q, (uint32_t)((tc * n + ir) * (int)sizeof(T))) : T(0);
      if constexpr (!TI) {
        d.bd = P.bd ? ldo(P.bd, (uint32_t)((tc * NX + ix) * (int)sizeof(T))) : T(0);
        d.bdm = P.bd ? ldo(P.bd, (uint32_t)((tm * NX + ix) * (int)sizeof(T))) : T(0);
        ldo_n<NX, n>(d.AmC, P.Am, (uint32_t)((tc * NX * n + ir) * (int)sizeof(T)));
        ldo_n<NX, n>(d.ApCm, P.Ap, (uint32_t)((tm * NX * n + ir) * (int)sizeof(T)));
        ldo_n<NG, n>(d.GC, P.G, (uint32_t)((tc * NG * n + ir) * (int)sizeof(T)));
      }
    };
    auto comp = [&](const In& d, int blk, auto full) {
      constexpr bool FULL = decltype(full)::value;
      const int t = 4 * blk + q;
      const T r = stage_r<FULL>(c, d, t, init);
      if (FULL || t <= N) sto(XV, lo.v + blk * LO::VB, r);
    };
    stage_blocks<STAGE_BLOCK_DEPTH, In>(nfull, load, comp);
  }
  pass_sync();

  // ---------------- pass 2: forward chain (row 0) ----------------
  if constexpr (ROWSPLIT_CHAIN<T, n>)
    chain_rows<n, +1>(XV, P.CF, lo.v0, lo.fq, N);
  else if (q == 0)
    chain<T, n, +1>(XV, P.CF, lo.v, lo.f, N);
  pass_sync();

  // ---------------- pass 3: s_t = SubB_t v_t on row t mod 4 ----------------
  {
    using In = TrIn<T, n>;
    auto load = [&](In& d, int blk) {
      ldo_n<n>(d.Br, sub_b_ptr<T>(P), lo.f + blk * LO::FB);
      d.v = ldo(XV, lo.v + blk * LO::VB);
    };
    auto comp = [&](const In& d, int blk, auto full) {
      constexpr bool FULL = decltype(full)::value;
      const int t = 4 * blk + q;
      const T s = sub_b_mul<T, n>(d.Br, d.v, i);
      if (FULL || t <= N) sto(XV, lo.v + blk * LO::VB, s);
    };
    stage_blocks<STAGE_BLOCK_DEPTH, In>(nfull, load, comp);
  }
  pass_sync();

  // ---------------- pass 4: backward chain (row 0) ----------------
  if constexpr (ROWSPLIT_CHAIN<T, n>)
    chain_rows<n, -1>(XV, P.CB, lo.v0, lo.fq, N);
  else if (q == 0)
    chain<T, n, -1>(XV, P.CB, lo.v, lo.f, N);
  pass_sync();

  // ---------------- pass 5: constraint-row updates on row t mod 4 ----------------
  {
    using In = UpdIn<T, NX, NU, NG, TI>;
    auto load = [&](In& d, int blk) {
      const int t = 4 * blk + q;
      const uint32_t ov = lo.v + blk * LO::VB;
      d.xt = ldo(XV, ov);
      d.xt1 = ldo<(int)LO::VS>(XV, ov);
      d.x = ldo(P.x, ov);
      d.yf = ldo(P.yf, ov);
      d.zg = ldo(P.zg, ov);
      d.yg = ldo(P.yg, ov);
      if constexpr (!TI) {
        const int tc = min(t, N);
        d.lo = ldo(P.lo, (uint32_t)((tc * NG + ig) * (int)sizeof(T)));
        d.hi = ldo(P.hi, (uint32_t)((tc * NG + ig) * (int)sizeof(T)));
        d.bd = P.bd ? ldo(P.bd, (uint32_t)((tc * NX + ix) * (int)sizeof(T))) : T(0);
        ldo_n<n>(d.AmR, P.Am, (uint32_t)((tc * NX * n + ix * n) * (int)sizeof(T)));
        ldo_n<n>(d.ApR, P.Ap, (uint32_t)((tc * NX * n + ix * n) * (int)sizeof(T)));
        ldo_n<n>(d.GR, P.G, (uint32_t)((tc * NG * n + ig * n) * (int)sizeof(T)));
      }
    };
    auto comp = [&](const In& d, int blk, auto full) {
      constexpr bool FULL = decltype(full)::value;
      stage_update<FULL>(c, d, 4 * blk + q, lo.v + blk * LO::VB);
    };
    stage_blocks<STAGE_BLOCK_DEPTH, In>(nfull, load, comp);
  }
  // initial-state rows: y_init += rho_f alpha (x~_0 - x_init), slot N of y_f
  if (q == 0 && i < NX) {
    const T x0 = ldo(XV, lo.v);
    sto(P.yf, lo.v + (uint32_t)(N * LO::VS), c.yinit + c.rfa * (x0 - c.xinit));
  }
  if constexpr (LV)
    lds_sync();  // the whole state is in LDS
  else
    wave_sync();
}

// ---------------------------------------------------------------------------
// Segmented substitutions.  The horizon is cut into R contiguous segments,
// segment q on 16-lane row q (R = 4: the rows of one wavefront; R = 4 W: the
// rows of a W-wavefront workgroup).  A chain over a segment from a zero start
// gives a particular solution; the true value at the segment's end differs by
// the segment's transfer block applied to the value entering it:
//   forward   v_b = p_b + T_q v_{a-1},   T_q = (-B_b) ... (-B_a),  B = ChF
//   backward  x_a = p_a + U_q x_{b+1},   U_q = (-B_a) ... (-B_b),  B = ChB
// (segment q covers stages a..b).  One iteration: every row runs its
// segment's forward chain from zero (with the eta_t / r_t work of each stage),
// a serial pass over the R segment ends finds each segment's true entering
// value, every row re-runs its segment from that value (with the SubB_t
// product), and the same for the backward chain (with the constraint updates
// of each stage).  Serial depth per chain: two segment lengths plus up to
// R - 1 block products, in place of the whole horizon.  T_q and U_q depend
// only on the factorisation and are formed after it by pushing the identity
// through each segment's chain (prepare_segments).
// ---------------------------------------------------------------------------
constexpr int SEG_MIN_N = 128;  // default switch: shorter horizons keep the interleaved iteration
constexpr int SEG_FLOOR_N = 15;  // segments of at least four stages

struct SegRange {
  int a, len;  // first stage and stage count of this row's segment
};
template <int R = 4>
__device__ __forceinline__ SegRange seg_range(int q, int N) {
  const int S = N + 1, base = S / R, rem = S % R;
  return SegRange{q * base + min(q, rem), base + (q < rem ? 1 : 0)};
}

// T_q and U_q of every segment of one instance (all rows; row q forms its own
// segment's blocks into Tout / Uout + q n n): lane i keeps row i of the
// running product in H[0..n).
template <typename T, int NX, int NU, int NG, int R = 4, typename OP = T*>
__device__ __noinline__ void prepare_segments(const Layout& Lm, int b_, int64_t s0_, int N_, OP Tout, OP Uout) {
  constexpr int n = NX + NU;
  const Layout L = uni(Lm);
  const int N = uni(N_);
  const int64_t s0 = uni(s0_);
  const int i = threadIdx.x & (ROW - 1), q = threadIdx.x >> 4;
  const int ir = i < n ? i : n - 1;
  const SegRange sg = seg_range<R>(q, N);
  const int64_t nn = (int64_t)n * n;
  const uint32_t orow = (uint32_t)(ir * n * (int)sizeof(T));
  for (int dir = 0; dir < 2; ++dir) {
    const gptr<const T> Bm = as_global((const T*)(dir == 0 ? L.ChF : L.ChB) + s0 * nn);
    T H[n];
#pragma unroll
    for (int j = 0; j < n; ++j) H[j] = (i == j) ? T(1) : T(0);
    for (int k = 0; k < sg.len; ++k) {
      const int t = dir == 0 ? sg.a + k : sg.a + sg.len - 1 - k;
      T Br[n];
      ldo_n<n>(Br, Bm + t * nn, orow);
      T Hn[n];
#pragma unroll
      for (int j = 0; j < n; ++j) Hn[j] = -dotb<n>(Br, H[j], T(0));
#pragma unroll
      for (int j = 0; j < n; ++j) H[j] = Hn[j];
    }
    if (i < n) {
      const OP out = (dir == 0 ? Tout : Uout) + q * nn + i * n;
#pragma unroll
      for (int j = 0; j < n; ++j) out[j] = H[j];
    }
  }
  (void)b_;
}

// The serial pass over the segment ends.  Every row stores its particular
// value pe (lane i: entry i) into slot `dir * R + q`, then forms the true
// values in sweep order as far as its wavefront's rows need them and returns
// the value entering its own segment.  dir 0 (forward): v_0 = pe_0, v_k =
// pe_k + T_k v_{k-1}; row q gets v_{q-1} (zero on row 0).  dir 1 (backward):
// x_{R-1} = pe_{R-1}, x_k = pe_k + U_k x_{k+1}; row q gets x_{q+1} (zero on
// row R - 1).  X: [2 R][ROW] slots; TU: the R transfer blocks of the sweep.
template <typename T, int n, int R, typename XP, typename TP>
__device__ __forceinline__ T seg_link(T pe, int dir, XP X, TP TU, int q, int i) {
  const int ir = i < n ? i : n - 1;
  const uint32_t ol = (uint32_t)(i * (int)sizeof(T));
  sto(X + (dir * R + q) * ROW, ol, pe);
  __syncthreads();  // every row of the workgroup has stored its end value
  const uint32_t orow = (uint32_t)(ir * n * (int)sizeof(T));
  const int q_lo = (int)(threadIdx.x >> 6) * 4, q_hi = q_lo + 3;  // this wavefront's rows
  T in = T(0);
  if (dir == 0) {
    T v = ldo(X + 0 * ROW, ol);  // true end value of segment 0
    in = (q == 1) ? v : in;
    for (int k = 1; k < q_hi; ++k) {
      T Br[n];
      ldo_n<n>(Br, TU + k * n * n, orow);
      v = dotb<n>(Br, v, ldo(X + k * ROW, ol));
      in = (q == k + 1) ? v : in;
    }
  } else {
    T x = ldo(X + (2 * R - 1) * ROW, ol);  // true start value of segment R - 1
    in = (q == R - 2) ? x : in;
    for (int k = R - 2; k > q_lo; --k) {
      T Br[n];
      ldo_n<n>(Br, TU + k * n * n, orow);
      x = dotb<n>(Br, x, ldo(X + (R + k) * ROW, ol));
      in = (q == k - 1) ? x : in;
    }
  }
  return in;
}

// Prefetch distance of the segmented sweeps, in steps.  FP32 iterations of
// small stages (n <= 8) keep four steps in flight (measured: 9-11 % off the
// long and ragged bicycle solves against two); deeper buffers, or four in
// FP64, overflow the register budget into scratch memory and run slower.
// Loads reach at most SEG_AHEAD + 1 stages past either end of the horizon,
// inside the STAGE_PAD padding stages.
// Multi-wavefront workgroups (R > 4) run two wavefronts per SIMD, which
// hide part of the load latency; their register budget (256) holds two steps
// in flight (measured on one N = 8192 bicycle instance, FP32: 0.49 ms per
// ADMM iteration with two, 0.50 with one; 16 wavefronts per workgroup with
// one or none: 0.52).
#ifndef OCP_MW_AHEAD
#define OCP_MW_AHEAD 2
#endif
#ifndef OCP_SEG_AHEAD_WIDE
#define OCP_SEG_AHEAD_WIDE 2
#endif
template <typename T, int n, int R = 4>
constexpr int SEG_AHEAD = R > 4 ? OCP_MW_AHEAD : (sizeof(T) == 4 && n <= 8) ? 4 : OCP_SEG_AHEAD_WIDE;
static_assert(SEG_AHEAD<float, 6> + 1 <= STAGE_PAD, "segmented prefetch beyond the padding stages");
static_assert(SEG_AHEAD<float, 16> + 1 <= STAGE_PAD, "segmented prefetch beyond the padding stages");

// inputs of one stage of the segmented forward sweep
template <typename T, int NX, int NU, int NG, bool TI>
struct SegFwdIn {
  EtaIn<T, NX, NU, NG, TI> e;
  T Cr[NX + NU];  // row `lane` of ChF_t
};

// One ADMM iteration with segmented substitutions (see above).  X: the
// instance's exchange slots; Tq / Uq: its transfer blocks.
template <typename T, int NX, int NU, int NG, typename ST, int R, typename XP, typename TP>
__device__ __forceinline__ void wave_iteration_seg(const IterCtx<T, NX, NU, NG, ST>& c, XP X, TP Tq, TP Uq) {
  constexpr int n = NX + NU;
  constexpr bool TI = ST::TI;
  constexpr int VS = ROW * (int)sizeof(T);
  const int N = c.N, q = c.q, i = c.i;
  const auto& P = c.P;
  const int ir = i < n ? i : n - 1, ix = i < NX ? i : NX - 1, ig = i < NG ? i : NG - 1;
  const T init = (i < NX) ? c.rho_f * c.xinit - c.yinit : T(0);
  const SegRange sg = seg_range<R>(q, N);
  const int steps = (N + R) / R;  // the longest segment
  // offsets of stage t on this lane (vector entry, factor row)
  auto ov = [&](int t) { return (uint32_t)(((STAGE_PAD + t) * ROW + i) * (int)sizeof(T)); };
  auto of = [&](int t) { return (uint32_t)(((STAGE_PAD + t) * n * n + ir * n) * (int)sizeof(T)); };
  auto load_eta_t = [&](EtaIn<T, NX, NU, NG, TI>& d, int t) {
    const uint32_t o = ov(t);
    if constexpr (EtaIn<T, NX, NU, NG, TI>::SA) ldo_n<n>(d.Ar, P.SA, of(t));
    d.x = ldo(P.x, o);
    d.yf = ldo(P.yf, o);
    d.yfm = ldo<-VS>(P.yf, o);
    d.zg = ldo(P.zg, o);
    d.yg = ldo(P.yg, o);
    const int tc = min(max(t, 0), N);
    const int tm = tc > 0 ? tc - 1 : 0;
    d.q = P.q ? ldo(P.q, (uint32_t)((tc * n + ir) * (int)sizeof(T))) : T(0);
    if constexpr (!TI) {
      d.bd = P.bd ? ldo(P.bd, (uint32_t)((tc * NX + ix) * (int)sizeof(T))) : T(0);
      d.bdm = P.bd ? ldo(P.bd, (uint32_t)((tm * NX + ix) * (int)sizeof(T))) : T(0);
      ldo_n<NX, n>(d.AmC, P.Am, (uint32_t)((tc * NX * n + ir) * (int)sizeof(T)));
      ldo_n<NX, n>(d.ApCm, P.Ap, (uint32_t)((tm * NX * n + ir) * (int)sizeof(T)));
      ldo_n<NG, n>(d.GC, P.G, (uint32_t)((tc * NG * n + ir) * (int)sizeof(T)));
    }
  };

  // ---- forward, particular: r_t and p_t = r_t - ChF_t p_{t-1} from zero ----
  T pe = T(0);
  {
    using In = SegFwdIn<T, NX, NU, NG, TI>;
    auto load = [&](In& d, int k) {
      const int t = sg.a + k;
      load_eta_t(d.e, t);
      ldo_n<n>(d.Cr, P.CF, of(t));
    };
    T p = T(0);
    auto comp = [&](In& d, int k) {
      if (k >= sg.len) return;
      const int t = sg.a + k;
      const T r = stage_r<false>(c, d.e, t, init);
      sto(P.v, ov(t), r);
      p = r - dotb<n>(d.Cr, p, T(0));  // p = 0 before the quarter's first stage
    };
    seg_walk<SEG_AHEAD<T, n, R>, In>(steps, load, comp);
    pe = p;
  }
  const T vin = seg_link<T, n, R>(pe, 0, X, Tq, q, i);

  // ---- forward, true values from vin, then s_t = SubB_t v_t ----
  {
    struct In {
      T Cr[n], Br[n];
      T r;
    };
    auto load = [&](In& d, int k) {
      const int t = sg.a + k;
      ldo_n<n>(d.Cr, P.CF, of(t));
      ldo_n<n>(d.Br, sub_b_ptr<T>(P), of(t));
      d.r = ldo(P.v, ov(t));
    };
    T v = vin;
    auto comp = [&](In& d, int k) {
      if (k >= sg.len) return;
      const int t = sg.a + k;
      v = d.r - dotb<n>(d.Cr, v, T(0));
      sto(P.v, ov(t), sub_b_mul<T, n>(d.Br, v, i));
    };
    seg_walk<SEG_AHEAD<T, n, R>, In>(steps, load, comp);
  }
  wave_sync();

  // ---- backward, particular: p_t = s_t - ChB_t p_{t+1} from zero ----
  {
    struct In {
      T Cr[n];
      T s;
    };
    auto load = [&](In& d, int k) {
      const int t = sg.a + sg.len - 1 - k;
      ldo_n<n>(d.Cr, P.CB, of(t));
      d.s = ldo(P.v, ov(t));
    };
    T p = T(0);
    auto comp = [&](In& d, int k) {
      if (k >= sg.len) return;
      p = d.s - dotb<n>(d.Cr, p, T(0));  // p = 0 past the quarter's last stage
    };
    seg_walk<SEG_AHEAD<T, n, R>, In>(steps, load, comp);
    pe = p;
  }
  const T xin = seg_link<T, n, R>(pe, 1, X, Uq, q, i);

  // ---- backward, true values from xin, with the constraint-row updates ----
  {
    struct In {
      T Cr[n];
      T s;
      UpdIn<T, NX, NU, NG, TI> u;
    };
    auto load = [&](In& d, int k) {
      const int t = sg.a + sg.len - 1 - k;
      const uint32_t o = ov(t);
      ldo_n<n>(d.Cr, P.CB, of(t));
      d.s = ldo(P.v, o);
      d.u.x = ldo(P.x, o);
      d.u.yf = ldo(P.yf, o);
      d.u.zg = ldo(P.zg, o);
      d.u.yg = ldo(P.yg, o);
      if constexpr (!TI) {
        const int tc = min(max(t, 0), N);
        d.u.lo = ldo(P.lo, (uint32_t)((tc * NG + ig) * (int)sizeof(T)));
        d.u.hi = ldo(P.hi, (uint32_t)((tc * NG + ig) * (int)sizeof(T)));
        d.u.bd = P.bd ? ldo(P.bd, (uint32_t)((tc * NX + ix) * (int)sizeof(T))) : T(0);
        ldo_n<n>(d.u.AmR, P.Am, (uint32_t)((tc * NX * n + ix * n) * (int)sizeof(T)));
        ldo_n<n>(d.u.ApR, P.Ap, (uint32_t)((tc * NX * n + ix * n) * (int)sizeof(T)));
        ldo_n<n>(d.u.GR, P.G, (uint32_t)((tc * NG * n + ig * n) * (int)sizeof(T)));
      }
    };
    T xn = xin;  // x~_{t+1}
    auto comp = [&](In& d, int k) {
      if (k >= sg.len) return;
      const int t = sg.a + sg.len - 1 - k;
      const T xt = d.s - dotb<n>(d.Cr, xn, T(0));
      d.u.xt = xt;
      d.u.xt1 = xn;
      stage_update<false>(c, d.u, t, ov(t));
      // initial-state rows: y_init += rho_f alpha (x~_0 - x_init), slot N of y_f
      if (t == 0 && i < NX) sto(P.yf, ov(N), c.yinit + c.rfa * (xt - c.xinit));
      xn = xt;
    };
    seg_walk<SEG_AHEAD<T, n, R>, In>(steps, load, comp);
  }
  wave_sync();
}

// ---------------------------------------------------------------------------
// PCG primal update (the PCG backend; ocp_set_linsolve).  S x~ = eta is
// solved by block-Jacobi preconditioned conjugate gradients from the current
// primal iterate x: with Theta_t the diagonal blocks of S and Phi_t its
// block (t+1, t), (S p)_t = Theta_t p_t + Phi_{t-1} p_{t-1} + Phi_t' p_{t+1}
// and the preconditioner applies Theta_t^-1 stage by stage (blocks from
// factor_instance, FACTOR_PCG).  Every pass is stage-parallel: row q takes
// the stages t = q, q + 4, ...; the inner products are wavefront sums in
// FP64.  Stops before an iteration when ||r||_2 <= tol ||eta||_2, or after
// max_it iterations.  Then the constraint updates of every stage from x~.
// ---------------------------------------------------------------------------
template <typename T>
struct PcgPtrs {
  gptr<T> xt, r, z, p, sp;  // [stages][ROW], at stage -STAGE_PAD like the state vectors
};

template <typename T, int NX, int NU, int NG, typename ST>
__device__ __forceinline__ void wave_iteration_pcg(const IterCtx<T, NX, NU, NG, ST>& c, const PcgPtrs<T>& B, int max_it,
                                                   double tol) {
  constexpr int n = NX + NU;
  constexpr bool TI = ST::TI;
  constexpr int VS = ROW * (int)sizeof(T);
  const int N = c.N, q = c.q, i = c.i;
  const auto& P = c.P;
  const bool vi = i < n;
  const int ir = vi ? i : n - 1, ix = i < NX ? i : NX - 1, ig = i < NG ? i : NG - 1;
  const T init = (i < NX) ? c.rho_f * c.xinit - c.yinit : T(0);
  const int steps = (N + 4) / 4;
  auto ov = [&](int t) { return (uint32_t)(((STAGE_PAD + t) * ROW + i) * (int)sizeof(T)); };
  auto of = [&](int t) { return (uint32_t)(((STAGE_PAD + t) * n * n + ir * n) * (int)sizeof(T)); };
  // (S v)_t on lane i from the vector v (global, this lane's entry of stages t-1, t, t+1)
  auto smul = [&](gptr<const T> v, int t) {
    T Th[n], Fm[n], Ft[n];
    ldo_n<n>(Th, P.SB, of(t));
    T acc = dotb<n>(Th, ldo(v, ov(t)), T(0));
    if (t > 0) {
      ldo_n<n>(Fm, P.CF, of(t - 1));
      acc = dotb<n>(Fm, ldo<-VS>(v, ov(t)), acc);
    }
    if (t < N) {
      ldo_n<n>(Ft, P.CB, of(t));
      acc = dotb<n>(Ft, ldo<VS>(v, ov(t)), acc);
    }
    return acc;
  };
  auto precond = [&](T r, int t) {
    T Mi[n];
    ldo_n<n>(Mi, P.SA, of(t));
    return dotb<n>(Mi, r, T(0));
  };
  auto wsum = [](double v) {
    v = row_sum(v);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
  };

  // eta_t (raw) into r; ||eta||^2
  double bb = 0.0;
  for (int k = 0; k < steps; ++k) {
    const int t = 4 * k + q;
    if (t > N) continue;  // the same on all lanes of a row
    EtaIn<T, NX, NU, NG, TI> d;
    const uint32_t o = ov(t);
    d.x = ldo(P.x, o);
    d.yf = ldo(P.yf, o);
    d.yfm = ldo<-VS>(P.yf, o);
    d.zg = ldo(P.zg, o);
    d.yg = ldo(P.yg, o);
    const int tm = t > 0 ? t - 1 : 0;
    d.q = P.q ? ldo(P.q, (uint32_t)((t * n + ir) * (int)sizeof(T))) : T(0);
    if constexpr (!TI) {
      d.bd = P.bd ? ldo(P.bd, (uint32_t)((t * NX + ix) * (int)sizeof(T))) : T(0);
      d.bdm = P.bd ? ldo(P.bd, (uint32_t)((tm * NX + ix) * (int)sizeof(T))) : T(0);
      ldo_n<NX, n>(d.AmC, P.Am, (uint32_t)((t * NX * n + ir) * (int)sizeof(T)));
      ldo_n<NX, n>(d.ApCm, P.Ap, (uint32_t)((tm * NX * n + ir) * (int)sizeof(T)));
      ldo_n<NG, n>(d.GC, P.G, (uint32_t)((t * NG * n + ir) * (int)sizeof(T)));
    }
    const T eta = vi ? stage_r<false, true>(c, d, t, init) : T(0);
    sto(B.r, o, eta);
    bb += double(eta) * double(eta);
  }
  // r = eta - S x, z = M r, p = z from x~_0 = x
  double rz = 0.0, rr = 0.0;
  for (int k = 0; k < steps; ++k) {
    const int t = 4 * k + q;
    if (t > N) continue;
    const uint32_t o = ov(t);
    const T r = vi ? ldo(B.r, o) - smul(P.x, t) : T(0);
    const T z = vi ? precond(r, t) : T(0);
    sto(B.xt, o, vi ? ldo(P.x, o) : T(0));
    sto(B.r, o, r);
    sto(B.z, o, z);
    sto(B.p, o, z);
    rz += double(r) * double(z);
    rr += double(r) * double(r);
  }
  bb = wsum(bb);
  rz = wsum(rz);
  rr = wsum(rr);
  wave_sync();  // p of every stage stored
  const double lim = tol * tol * bb;
  for (int it = 0; it < max_it && rr > lim; ++it) {
    double pSp = 0.0;
    for (int k = 0; k < steps; ++k) {
      const int t = 4 * k + q;
      if (t > N) continue;
      const uint32_t o = ov(t);
      const T sp = vi ? smul(B.p, t) : T(0);
      sto(B.sp, o, sp);
      pSp += double(ldo(B.p, o)) * double(sp);
    }
    pSp = wsum(pSp);
    const T alpha = T(rz / pSp);
    double rz_new = 0.0;
    rr = 0.0;
    for (int k = 0; k < steps; ++k) {
      const int t = 4 * k + q;
      if (t > N) continue;
      const uint32_t o = ov(t);
      const T pv = ldo(B.p, o);
      const T x = ldo(B.xt, o) + alpha * pv;
      const T r = ldo(B.r, o) - alpha * ldo(B.sp, o);
      const T z = vi ? precond(r, t) : T(0);
      sto(B.xt, o, x);
      sto(B.r, o, r);
      sto(B.z, o, z);
      rz_new += double(r) * double(z);
      rr += double(r) * double(r);
    }
    rz_new = wsum(rz_new);
    rr = wsum(rr);
    const T beta = T(rz_new / rz);
    rz = rz_new;
    for (int k = 0; k < steps; ++k) {
      const int t = 4 * k + q;
      if (t > N) continue;
      const uint32_t o = ov(t);
      sto(B.p, o, ldo(B.z, o) + beta * ldo(B.p, o));
    }
    wave_sync();  // p of every stage stored
  }
  wave_sync();  // x~ of every stage stored
  // over-relaxation, projections and dual updates from x~
  for (int k = 0; k < steps; ++k) {
    const int t = 4 * k + q;
    if (t > N) continue;
    const uint32_t o = ov(t);
    UpdIn<T, NX, NU, NG, TI> u;
    u.x = ldo(P.x, o);
    u.yf = ldo(P.yf, o);
    u.zg = ldo(P.zg, o);
    u.yg = ldo(P.yg, o);
    if constexpr (!TI) {
      u.lo = ldo(P.lo, (uint32_t)((t * NG + ig) * (int)sizeof(T)));
      u.hi = ldo(P.hi, (uint32_t)((t * NG + ig) * (int)sizeof(T)));
      u.bd = P.bd ? ldo(P.bd, (uint32_t)((t * NX + ix) * (int)sizeof(T))) : T(0);
      ldo_n<n>(u.AmR, P.Am, (uint32_t)((t * NX * n + ix * n) * (int)sizeof(T)));
      ldo_n<n>(u.ApR, P.Ap, (uint32_t)((t * NX * n + ix * n) * (int)sizeof(T)));
      ldo_n<n>(u.GR, P.G, (uint32_t)((t * NG * n + ig * n) * (int)sizeof(T)));
    }
    u.xt = ldo(B.xt, o);
    u.xt1 = (t < N) ? ldo<VS>(B.xt, o) : T(0);
    stage_update<false>(c, u, t, o);
    // initial-state rows: y_init += rho_f alpha (x~_0 - x_init), slot N of y_f
    if (t == 0 && i < NX) sto(P.yf, ov(N), c.yinit + c.rfa * (u.xt - c.xinit));
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
// General form: the blocks of every stage are read where they are used.
template <typename T, int NX, int NU, int NG, bool TI, int RR = 4>
__device__ __forceinline__ Resid residuals_gen(const Layout& L, const WaveGroup& w, int kind, double gamma2,
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
  // the same maxima for the original problem (rescaling weights rw)
  double u_cxc = 0, u_cx = 0, u_c = 0, u_gxz = 0, u_gx = 0, u_z = 0;
  double u_dual = 0, u_px = 0, u_aty = 0, u_q = 0, u_sres = 0, u_sscale = 0;
  ResW rw;
  rw.load(L, b, i);
  int nf = 0;
  auto upd = [&](double& m, double& mu, double v, double wgt) {
    if (!isfinite(v)) nf = 1;
    m = fmax(m, fabs(v));
    mu = fmax(mu, fabs(v) * wgt);
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
  const int nbl = (N + RR) / RR;
  for (int blk = 0; blk < nbl; ++blk) {
    const int t = RR * blk + q;
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
      upd(m_dual, u_dual, px + qv + aty, rw.d);
      upd(m_px, u_px, px, rw.d);
      upd(m_aty, u_aty, aty, rw.d);
      upd(m_q, u_q, qv, rw.d);
    }
    // equality rows touching stage t
    if (t == 0 && i < NX) {
      upd(m_cxc, u_cxc, xc - xi0, rw.f);
      upd(m_cx, u_cx, xc, rw.f);
      upd(m_c, u_c, xi0, rw.f);
    }
    double cx = dotb<n>(Amr, xc, 0.0);
    cx = dotb<n>(Apr, xn, cx);
    if (t < N && i < NX) {
      upd(m_cxc, u_cxc, cx - cv, rw.f);
      upd(m_cx, u_cx, cx, rw.f);
      upd(m_c, u_c, cv, rw.f);
    }
    // inequality rows of stage t
    const double gx = dotb<n>(Gr, xc, 0.0);
    if (i < NG) {
      const double zv = double(ZG[sv]);
      upd(m_gxz, u_gxz, gx - zv, rw.g);
      upd(m_gx, u_gx, gx, rw.g);
      upd(m_z, u_z, zv, rw.g);
      const double xiv = double(XI[sv]);
      if (kind == 1) {
        upd(m_sres, u_sres, gamma2 * xiv + ygv, rw.s);
        upd(m_sscale, u_sscale, gamma2 * xiv, rw.s);
        upd(m_sscale, u_sscale, ygv, rw.s);
      } else if (kind == 2) {
        const double r1 = (xiv != 0.0) ? fabs(ygv + gamma1 * (xiv > 0 ? 1.0 : -1.0)) : fmax(fabs(ygv) - gamma1, 0.0);
        upd(m_sres, u_sres, r1, rw.s);
        upd(m_sscale, u_sscale, xiv != 0.0 ? gamma1 : 0.0, rw.s);
        upd(m_sscale, u_sscale, ygv, rw.s);
      }
    }
  }
  Resid R;
  R.rp = rows_max(row_max(fmax(m_cxc, m_gxz)));
  R.ps = rows_max(row_max(fmax(fmax(m_cx, m_gx), fmax(m_c, m_z))));
  R.rd = rows_max(row_max(fmax(m_dual, m_sres)));
  R.ds = rows_max(row_max(fmax(fmax(m_px, m_aty), fmax(m_q, m_sscale))));
  if (L.sc) {
    R.rp_u = rows_max(row_max(fmax(u_cxc, u_gxz)));
    R.ps_u = rows_max(row_max(fmax(fmax(u_cx, u_gx), fmax(u_c, u_z))));
    R.rd_u = rows_max(row_max(fmax(u_dual, u_sres)));
    R.ds_u = rows_max(row_max(fmax(fmax(u_px, u_aty), fmax(u_q, u_sscale))));
  } else {
    R.rp_u = R.rp, R.ps_u = R.ps, R.rd_u = R.rd, R.ds_u = R.ds;
  }
  R.nonfinite = rows_max(row_max(nf));
  return R;
}

// per-stage inputs of the residual evaluation (time-invariant data)
template <typename T>
struct ResIn {
  T xc, xm, xn, yfc, yfm, yg, zg, xi;
  double q;
};

// The same residuals for time-invariant data: blocks read once (FP64), the
// explicit-dynamics and selection structure of ST used, stage inputs loaded
// two blocks ahead.
template <typename T, int NX, int NU, int NG, typename ST, int RR = 4>
__device__ __forceinline__ Resid residuals_ti(const Layout& L, const WaveGroup& w, int kind, double gamma2,
                                              double gamma1) {
  constexpr int n = NX + NU;
  constexpr int VS = ROW * (int)sizeof(T);
  const int i = w.lane, q = w.row, b = w.b, N = w.N;
  const int ic = i < n ? i : n - 1, ix = i < NX ? i : NX - 1;
  const int64_t sp = w.s0 - STAGE_PAD;
  TIBlocks64<NX, NU, NG, ST> tb;
  tb.load(L, b, i);
  const bool hasE = L.E != nullptr;
  const gptr<const T> X = as_global((const T*)L.x + sp * ROW), YF = as_global((const T*)L.yf + sp * ROW);
  const gptr<const T> ZG = as_global((const T*)L.zg + sp * ROW), YG = as_global((const T*)L.yg + sp * ROW);
  const gptr<const T> XI = as_global((const T*)L.xi + sp * ROW);
  const gptr<const double> Q = L.q ? as_global(L.q + w.s0 * n) : nullptr;
  const double cv = L.bd ? L.bd[(size_t)b * NX + ix] : 0.0;
  const double xi0 = L.x_init[(size_t)b * NX + ix];
  const double yinit = double(ldo(YF, (uint32_t)(((STAGE_PAD + N) * ROW + i) * (int)sizeof(T))));
  const int gsel = L.gsel[i < NG ? i : 0], ginv = L.ginv[i];
  const bool gid = __ballot(i < NG && gsel != i) == 0;
  double m_cxc = 0, m_cx = 0, m_c = 0, m_gxz = 0, m_gx = 0, m_z = 0;
  double m_dual = 0, m_px = 0, m_aty = 0, m_q = 0, m_sres = 0, m_sscale = 0;
  // the same maxima for the original problem (rescaling weights rw)
  double u_cxc = 0, u_cx = 0, u_c = 0, u_gxz = 0, u_gx = 0, u_z = 0;
  double u_dual = 0, u_px = 0, u_aty = 0, u_q = 0, u_sres = 0, u_sscale = 0;
  ResW rw;
  rw.load(L, b, i);
  int nf = 0;
  auto upd = [&](double& m, double& mu, double v, double wgt) {
    if (!isfinite(v)) nf = 1;
    m = fmax(m, fabs(v));
    mu = fmax(mu, fabs(v) * wgt);
  };
  auto load = [&](ResIn<T>& d, int blk) {
    const int t = RR == 4 ? 4 * blk + q : min(RR * blk + q, N + 1);  // loads stay within the padding
    const uint32_t o = (uint32_t)(((STAGE_PAD + t) * ROW + i) * (int)sizeof(T));
    d.xc = ldo(X, o);
    d.xm = ldo<-VS>(X, o);
    d.xn = ldo<VS>(X, o);
    d.yfc = ldo(YF, o);
    d.yfm = ldo<-VS>(YF, o);
    d.yg = ldo(YG, o);
    d.zg = ldo(ZG, o);
    d.xi = ldo(XI, o);
    d.q = Q ? ldo(Q, (uint32_t)((min(t, N) * n + ic) * (int)sizeof(double))) : 0.0;
  };
  auto comp = [&](const ResIn<T>& d, int blk, auto full) {
    constexpr bool FULL = decltype(full)::value;
    const int t = RR * blk + q;
    if (!FULL && t > N) return;
    const bool thi = FULL || t < N, xr = i < NX;
    const double xc = double(d.xc);
    const double xm = (t > 0) ? double(d.xm) : 0.0;
    const double xn = thi ? double(d.xn) : 0.0;
    const double yfc = (thi && xr) ? double(d.yfc) : 0.0;
    const double yfm = (t > 0 && xr) ? double(d.yfm) : 0.0;
    // (P x)_t row i = D_t x_t + E_{t-1} x_{t-1} + E_t' x_{t+1}
    double px = dotb<n>(tb.Dr, xc, 0.0);
    if (!FULL && t == N) px = dotb<n>(tb.dDN, xc, px);
    if (hasE) {
      px = dotb<n>(tb.Er, xm, px);
      px = dotb<n>(tb.Ec, xn, px);
    }
    // (A' y)_t row i
    double aty = dotb<NX>(tb.Amc, yfc, 0.0);
    if constexpr (ST::APNEG)
      aty -= yfm;
    else
      aty = dotb<NX>(tb.Apc, yfm, aty);
    if (t == 0 && xr) aty += yinit;
    const double ygv = (i < NG) ? double(d.yg) : 0.0;
    if constexpr (ST::GSEL) {
      const double gt = gid ? ygv : row_gather(ygv, ginv < 0 ? 0 : ginv);
      aty += (ginv >= 0) ? gt : 0.0;
    } else {
      aty = dotb<NG>(tb.Gc, ygv, aty);
    }
    const double qv = (i < n) ? d.q : 0.0;
    if (i < n) {
      upd(m_dual, u_dual, px + qv + aty, rw.d);
      upd(m_px, u_px, px, rw.d);
      upd(m_aty, u_aty, aty, rw.d);
      upd(m_q, u_q, qv, rw.d);
    }
    // equality rows touching stage t
    if (t == 0 && xr) {
      upd(m_cxc, u_cxc, xc - xi0, rw.f);
      upd(m_cx, u_cx, xc, rw.f);
      upd(m_c, u_c, xi0, rw.f);
    }
    double cx = dotb<n>(tb.Amr, xc, 0.0);
    if constexpr (ST::APNEG)
      cx -= xn;
    else
      cx = dotb<n>(tb.Apr, xn, cx);
    if (thi && xr) {
      upd(m_cxc, u_cxc, cx - cv, rw.f);
      upd(m_cx, u_cx, cx, rw.f);
      upd(m_c, u_c, cv, rw.f);
    }
    // inequality rows of stage t
    double gx;
    if constexpr (ST::GSEL)
      gx = gid ? xc : row_gather(xc, gsel);
    else
      gx = dotb<n>(tb.Gr, xc, 0.0);
    if (i < NG) {
      const double zv = double(d.zg);
      upd(m_gxz, u_gxz, gx - zv, rw.g);
      upd(m_gx, u_gx, gx, rw.g);
      upd(m_z, u_z, zv, rw.g);
      const double xiv = double(d.xi);
      if (kind == 1) {
        upd(m_sres, u_sres, gamma2 * xiv + ygv, rw.s);
        upd(m_sscale, u_sscale, gamma2 * xiv, rw.s);
        upd(m_sscale, u_sscale, ygv, rw.s);
      } else if (kind == 2) {
        const double r1 = (xiv != 0.0) ? fabs(ygv + gamma1 * (xiv > 0 ? 1.0 : -1.0)) : fmax(fabs(ygv) - gamma1, 0.0);
        upd(m_sres, u_sres, r1, rw.s);
        upd(m_sscale, u_sscale, xiv != 0.0 ? gamma1 : 0.0, rw.s);
        upd(m_sscale, u_sscale, ygv, rw.s);
      }
    }
  };
  stage_blocks<STAGE_BLOCK_DEPTH, ResIn<T>>(N / RR, load, comp);
  Resid R;
  R.rp = rows_max(row_max(fmax(m_cxc, m_gxz)));
  R.ps = rows_max(row_max(fmax(fmax(m_cx, m_gx), fmax(m_c, m_z))));
  R.rd = rows_max(row_max(fmax(m_dual, m_sres)));
  R.ds = rows_max(row_max(fmax(fmax(m_px, m_aty), fmax(m_q, m_sscale))));
  if (L.sc) {
    R.rp_u = rows_max(row_max(fmax(u_cxc, u_gxz)));
    R.ps_u = rows_max(row_max(fmax(fmax(u_cx, u_gx), fmax(u_c, u_z))));
    R.rd_u = rows_max(row_max(fmax(u_dual, u_sres)));
    R.ds_u = rows_max(row_max(fmax(fmax(u_px, u_aty), fmax(u_q, u_sscale))));
  } else {
    R.rp_u = R.rp, R.ps_u = R.ps, R.rd_u = R.rd, R.ds_u = R.ds;
  }
  R.nonfinite = rows_max(row_max(nf));
  return R;
}

// RR: rows the stages are spread over (4: one wavefront; 4 W: the rows of a
// W-wavefront workgroup, wm.row the row in the workgroup, each wavefront's
// maxima then combined by the caller)
template <typename T, int NX, int NU, int NG, typename ST, int TAG = 0, int RR = 4>
__device__ __noinline__ Resid residuals_wave(const Layout& Lm, const WaveGroup& wm, int kind, double gamma2_,
                                             double gamma1_) {
  const Layout L = uni(Lm);
  WaveGroup w = wm;
  w.b = uni(wm.b), w.s0 = uni(wm.s0), w.N = uni(wm.N);
  const double gamma2 = uni(gamma2_), gamma1 = uni(gamma1_);
  if constexpr (ST::TI)
    return residuals_ti<T, NX, NU, NG, ST, RR>(L, w, kind, gamma2, gamma1);
  else
    return residuals_gen<T, NX, NU, NG, false, RR>(L, w, kind, gamma2, gamma1);
}

// Primal-infeasibility certificate at a convergence check (the test of
// Banjac, Goulart, Stellato and Boyd for ADMM on convex QPs, written from its
// definition): with dy the change of the multipliers since the previous
// check, the constraint set {Cx = c, lo <= Gx <= hi} is empty when
// ||A'dy||_inf <= eps ||dy||_inf and c'dy_f + hi'max(dy_g, 0) + lo'min(dy_g, 0)
// < -eps ||dy||_inf (Farkas).  Evaluated in the original variables of a
// rescaled QP; a nonzero dy on a soft row fails it.  Stages spread over the
// four rows as in the residuals; blocks read from the FP64 master data.
// parts of the test (maxima of |A'dy| and |dy|, the support value, a soft
// row with a change), reduced over the rows of one wavefront
struct PinfPart {
  double m_aty, m_dy, sup;
  int soft_bad;
};
__device__ __forceinline__ int pinf_decide(const PinfPart& p, double eps) {
  return (p.m_dy > 0.0 && !p.soft_bad && p.m_aty <= eps * p.m_dy && p.sup < -eps * p.m_dy) ? 1 : 0;
}
template <typename T, int NX, int NU, int NG, int TAG = 0, int RR = 4>
__device__ __noinline__ PinfPart pinf_parts(const Layout& Lm, const WaveGroup& wm) {
  const Layout L = uni(Lm);
  const int b = uni(wm.b), N = uni(wm.N);
  const int64_t s0 = uni(wm.s0);
  constexpr int n = NX + NU;
  const int i = wm.lane, q = wm.row;
  const int ic = i < n ? i : n - 1, ix = i < NX ? i : NX - 1, ig = i < NG ? i : NG - 1;
  const bool ti = L.ti != 0;
  const gptr<const T> YF = as_global((const T*)L.yf), YG = as_global((const T*)L.yg);
  const gptr<const T> PF = as_global((const T*)L.ypf), PG = as_global((const T*)L.ypg);
  ResW rw;
  rw.load(L, b, i);
  const int kind = (i < NG) ? (int)L.soft[i] : 0;
  const size_t vi = (size_t)(s0 + N) * ROW + i;  // initial-state slot
  const double dyinit = (i < NX) ? double(YF[vi]) - double(PF[vi]) : 0.0;
  const double xi0 = L.x_init[(size_t)b * NX + ix];
  double m_aty = 0.0, m_dy = 0.0, sup = 0.0;
  int soft_bad = 0;
  for (int t = q; t <= N; t += RR) {
    const int64_t s = s0 + t;
    const size_t sv = (size_t)s * ROW + i;
    const double dyfc = (t < N && i < NX) ? double(YF[sv]) - double(PF[sv]) : 0.0;
    const double dyfm = (t > 0 && i < NX) ? double(YF[sv - ROW]) - double(PF[sv - ROW]) : 0.0;
    const double dyg = (i < NG) ? double(YG[sv]) - double(PG[sv]) : 0.0;
    double Amc[NX], Apc[NX], Gc[NG];
    load_col<NX>(Amc, L.Am + ti_or_tv(ti, b, s, (size_t)NX * n) + ic, n, t < N);
    load_col<NX>(Apc, L.Ap + ti_or_tv(ti, b, t > 0 ? s - 1 : s, (size_t)NX * n) + ic, n, t > 0);
    load_col<NG>(Gc, L.G + ti_or_tv(ti, b, s, (size_t)NG * n) + ic, n, true);
    double aty = dotb<NX>(Amc, dyfc, 0.0);
    aty = dotb<NX>(Apc, dyfm, aty);
    if (t == 0 && i < NX) aty += dyinit;
    aty = dotb<NG>(Gc, dyg, aty);
    if (i < n) m_aty = fmax(m_aty, fabs(aty) * rw.d);
    if (i < NX) {
      m_dy = fmax(m_dy, fabs(dyfc) * rw.d);  // y_f = yh_f / (c d_x): the stationarity weight
      const double cv = (t < N && L.bd) ? L.bd[ti_or_tv(ti, b, s, NX) + ix] : 0.0;
      sup += cv * dyfc;
      if (t == 0) {
        m_dy = fmax(m_dy, fabs(dyinit) * rw.d);
        sup += xi0 * dyinit;
      }
    }
    if (i < NG) {
      m_dy = fmax(m_dy, fabs(dyg) * rw.s / rw.g);  // y_g = e yh_g / c
      const size_t sb = ti_or_tv(ti, b, s, NG) + i;
      if (dyg > 0.0) sup += L.hi[sb] * dyg;
      if (dyg < 0.0) sup += L.lo[sb] * dyg;
      if (kind != 0 && dyg != 0.0) soft_bad = 1;
    }
  }
  m_aty = rows_max(row_max(m_aty));
  m_dy = rows_max(row_max(m_dy));
  sup = row_sum(sup);
  sup += __shfl_xor(sup, 16);
  sup += __shfl_xor(sup, 32);
  sup *= rw.s;  // original variables: the support value of the rescaled QP over c
  soft_bad = rows_max(row_max(soft_bad));
  return PinfPart{m_aty, m_dy, sup, soft_bad};
}
template <typename T, int NX, int NU, int NG, int TAG = 0>
__device__ __forceinline__ int pinf_wave(const Layout& Lm, const WaveGroup& wm, double eps) {
  return pinf_decide(pinf_parts<T, NX, NU, NG, TAG>(Lm, wm), eps);
}

// y_f, y_g -> the previous-check copies (every stage of the instance)
template <typename T>
__device__ __forceinline__ void keep_multipliers(const Layout& L, const WaveGroup& w) {
  T* yf = (T*)L.yf;
  T* yg = (T*)L.yg;
  T* pf = (T*)L.ypf;
  T* pg = (T*)L.ypg;
  for (int e = threadIdx.x; e < (w.N + 1) * ROW; e += 64) {
    const size_t k = (size_t)w.s0 * ROW + e;
    pf[k] = yf[k];
    pg[k] = yg[k];
  }
}

// Boundary decision of the schedule (eq. admm:termination:slack, rho:update):
// returns the new status (ST_RUNNING to continue) and may change rho_bar.
__device__ __forceinline__ int boundary_decision(const Resid& R, const Settings& st, int check, int adapt, int last,
                                                 int infeasible, double& rho_bar, bool& refactor) {
  refactor = false;
  if (R.nonfinite) return 2;
  // stopping test on the original problem, step size from the residuals of
  // the QP the iterations run on
  const bool conv = R.rp_u <= st.eps_abs + st.eps_rel * R.ps_u && R.rd_u <= st.eps_abs + st.eps_rel * R.ds_u;
  if ((check || (st.k_check > 0 && last)) && conv) return 0;
  if (check && infeasible) return 4;  // certificate of the multiplier change (pinf_wave)
  if (adapt && !conv) {
    // also at the last boundary: the final rho_bar is the step size an SQP
    // iteration hands to its next QP (no refactorisation follows it there)
    const double num = R.rp / fmax(R.ps, 1e-30);
    const double den = R.rd / fmax(R.ds, 1e-30);
    double cand = rho_bar * sqrt(num / fmax(den, 1e-30));
    cand = fmin(fmax(cand, st.rho_min), st.rho_max);
    if (fmax(cand / rho_bar, rho_bar / cand) > st.k_ratio) {
      rho_bar = cand;
      refactor = !last;
    }
  }
  if (last) return 1;
  return ST_RUNNING;
}

// ADMM iterations k0 .. nb-1 of one instance at a fixed rho (a segment of the
// schedule between two boundaries).  Not inlined: the loop gets the register
// file to itself, the solve-level state of the caller stays out of it.
// Returns the iteration count reached.
// PCG: the PCG primal updates (its own instantiation, so that the direct
// path's register allocation does not see them).
template <typename T, int NX, int NU, int NG, typename ST, bool SEG, int R = 4, bool PCG = false>
__device__ __noinline__ int run_segment(const Layout& Lm, const Settings& st, int b_, int64_t s0_, int N_, int k0_,
                                        int nb_, double rho_bar_, lptr<T> mw_ = nullptr) {
  const Layout L = uni(Lm);
  const int b = uni(b_), N = uni(N_), nb = uni(nb_);
  const int64_t s0 = uni(s0_);
  const double rho_bar = uni(rho_bar_);
  const int i = threadIdx.x & (ROW - 1), q = threadIdx.x >> 4;
  const int kind = (i < NG) ? (int)L.soft[i] : 0;
  const bool hard = __ballot(kind != 0) == 0;
  const int gsel = L.gsel[i < NG ? i : 0], ginv = L.ginv[i];
  const bool gid = __ballot(i < NG && gsel != i) == 0;
  const IterPtrs<T, NX, NU, NG> P(L, b, s0);
  const LaneOff<T, NX + NU> lo(q, i);
  const uint32_t o_yinit = (uint32_t)(((STAGE_PAD + N) * ROW + i) * (int)sizeof(T));
  TIBlocks<T, NX, NU, NG> tb;
  if constexpr (ST::TI) tb.load(L, b, i);
  const ProjConst<T> pc(T(rho_bar), T(L.gamma2), T(L.gamma1));
  const T xinit = ((const T*)L.xinitT)[(size_t)b * NX + (i < NX ? i : 0)];
  const T rho_f = T(uni(st.rho_f_scale) * rho_bar), alpha = T(uni(st.alpha));
  const IterCtx<T, NX, NU, NG, ST> c{tb,   P,    T(uni(st.sigma)), rho_f, T(rho_bar), alpha, T(1) - alpha,
                                     rho_f * alpha, kind, pc, xinit, T(0), gsel, ginv, i, q, N, gid, hard};
  constexpr int64_t nn = (int64_t)(NX + NU) * (NX + NU);
  // exchange slots and transfer blocks: the instance's in global memory (one
  // wavefront), or the workgroup's LDS ([R][nn] T, [R][nn] U, [2R][ROW] X)
  const auto X = [&] {
    if constexpr (R == 4) return as_global((T*)L.SegX + (int64_t)b * 8 * ROW);
    else return mw_ + 2 * R * nn;
  }();
  const auto Tq = [&] {
    if constexpr (R == 4) return as_global((const T*)L.SegT + (int64_t)b * 4 * nn);
    else return (lptr<const T>)mw_;
  }();
  const auto Uq = [&] {
    if constexpr (R == 4) return as_global((const T*)L.SegU + (int64_t)b * 4 * nn);
    else return (lptr<const T>)(mw_ + R * nn);
  }();
  // LDS of the interleaved iteration: FP32 horizons up to STATE_LDS_STAGES
  // keep all six stage vectors there for the segment (copied in here and out
  // before the boundary's residuals); longer ones, and FP64, the exchange
  // vector only
  constexpr int LDS_ELEMS = sizeof(T) == 4 ? 6 * STATE_LDS_STAGES * ROW : XV_LDS_STAGES * ROW;
  __shared__ __attribute__((aligned(16))) T lds_buf[(SEG || PCG) ? 1 : LDS_ELEMS];
  const lptr<T> XVl = (lptr<T>)lds_buf;
  const bool state_lds = !SEG && sizeof(T) == 4 && N + 1 + 2 * STAGE_PAD + 8 <= STATE_LDS_STAGES;
  const bool xv_lds = !SEG && N + 1 + 2 * STAGE_PAD + 8 <= LDS_ELEMS / ROW;
  int k = uni(k0_);
  if constexpr (PCG) {
    {  // PCG primal updates (stage-parallel; no chains)
      const int64_t sp = s0 - STAGE_PAD;
      const PcgPtrs<T> B{as_global((T*)L.pcg_xt + sp * ROW), as_global((T*)L.pcg_r + sp * ROW),
                         as_global((T*)L.pcg_z + sp * ROW), as_global((T*)L.pcg_p + sp * ROW),
                         as_global((T*)L.pcg_sp + sp * ROW)};
      for (; k < nb; ++k) {
        IterCtx<T, NX, NU, NG, ST> ck = c;
        ck.yinit = ldo(P.yf, o_yinit);
        wave_iteration_pcg<T, NX, NU, NG, ST>(ck, B, L.pcg_max_it, L.pcg_tol);
      }
      return k;
    }
  }
  if constexpr (!SEG && sizeof(T) == 4) {
    if (state_lds) {
      const IterPtrs<T, NX, NU, NG, true> PL(P, XVl, STATE_LDS_STAGES);
      // stages 0..N of x, y_f (slot N: the initial-state rows), z_g, y_g, xi
      const int len = (N + 1) * ROW;
      const uint32_t o0 = (uint32_t)(STAGE_PAD * ROW * (int)sizeof(T));
      auto copy = [&](auto dst, auto src) {
        for (int e = threadIdx.x; e < len; e += 64) sto(dst, o0 + (uint32_t)(e * (int)sizeof(T)), ldo(src, o0 + (uint32_t)(e * (int)sizeof(T))));
      };
      copy(PL.x, P.x);
      copy(PL.yf, P.yf);
      copy(PL.zg, P.zg);
      copy(PL.yg, P.yg);
      copy(PL.xi, P.xi);
      lds_sync();
      const IterCtx<T, NX, NU, NG, ST, true> cl{tb, PL,   c.sigma, c.rho_f, c.rho_g, c.alpha, c.oma, c.rfa, c.kind,
                                                c.pc, c.xinit, T(0), c.gsel, c.ginv, c.i, c.q, c.N, c.gid, c.hard};
      for (; k < nb; ++k) {
        IterCtx<T, NX, NU, NG, ST, true> ck = cl;
        ck.yinit = ldo(PL.yf, o_yinit);
        wave_iteration<T, NX, NU, NG, ST>(ck, lo, PL.v);
      }
      copy(P.x, PL.x);
      copy(P.yf, PL.yf);
      copy(P.zg, PL.zg);
      copy(P.yg, PL.yg);
      copy(P.xi, PL.xi);
      wave_sync();  // the boundary's residuals read the state from global memory
      return k;
    }
  }
  for (; k < nb; ++k) {
    IterCtx<T, NX, NU, NG, ST> ck = c;
    ck.yinit = ldo(P.yf, o_yinit);  // initial-state multipliers (slot N)
    if constexpr (SEG)
      wave_iteration_seg<T, NX, NU, NG, ST, R>(ck, X, Tq, Uq);
    else if (xv_lds)
      wave_iteration<T, NX, NU, NG, ST>(ck, lo, XVl);
    else
      wave_iteration<T, NX, NU, NG, ST>(ck, lo, P.v);
  }
  return k;
}

// Multi-wavefront instances: one workgroup of W wavefronts per instance.
// Wavefront 0 runs the schedule below (stopping and rho decisions); the
// factorisation, the transfer blocks, the iterations between two boundaries
// and the boundary's FP64 evaluation are workgroup operations in which every
// 16-lane row of the W wavefronts takes one chunk / segment / set of stages
// (R = 4 W of them).  Wavefront 0 posts
// each operation in LDS and meets the others at a barrier; the others loop
// on posted operations until MW_EXIT.  Every operation ends with a barrier,
// so between operations wavefront 0 alone runs, with wavefront-local syncs.
enum { MW_EXIT = 0, MW_FACTOR = 1, MW_PREP = 2, MW_ITERS = 3, MW_CHECK = 4 };
// MW_CHECK parts (MwCmd::k): FP64 residuals, infeasibility certificate,
// keep the multipliers for the next certificate
enum { MW_CHECK_RESID = 1, MW_CHECK_PINF = 2, MW_CHECK_KEEP = 4 };
// LDS slots of the cross-wavefront reductions of MW_CHECK: per wavefront
// MW_RED_F doubles (the eight residual maxima, non-finite flag, the three
// certificate parts, its soft-row flag), then the combined values
constexpr int MW_RED_F = 16;
struct MwCmd {
  int op, k, nb;
  double rho_bar;
};
// wavefronts per workgroup: 8 for stages up to 8 wide (32 rows; two
// wavefronts per SIMD leave each 256 registers, which the segmented sweeps
// need), 4 for wider stages (the LDS transfer blocks grow as n^2)
#ifndef OCP_MW_WAVES
#define OCP_MW_WAVES 8
#endif
#ifndef OCP_MW_WAVES_WIDE
#define OCP_MW_WAVES_WIDE 4
#endif
__host__ __device__ constexpr int mw_waves_of(int n) { return n <= 8 ? OCP_MW_WAVES : OCP_MW_WAVES_WIDE; }
template <int n>
constexpr int mw_waves() { return mw_waves_of(n); }
// shortest horizon taken by a W-wavefront workgroup: four stages per segment
// (and at least three per factorisation chunk)
__host__ __device__ constexpr int mw_floor_n(int W) { return 16 * W - 1; }
static_assert(mw_floor_n(2) >= fac_chunk_min_n(8) && mw_floor_n(4) >= fac_chunk_min_n(16) &&
                  mw_floor_n(16) >= fac_chunk_min_n(64),
              "chunk floor");
// default: horizons from 256 stages take a workgroup
constexpr int MW_MIN_N = 255;

__device__ __forceinline__ void wave_local_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// One workgroup operation (all W wavefronts; ends with a barrier).  buf: the
// LDS transfer blocks and exchange slots; FX: the chunked factorisation's
// exchange blocks; bad: one flag per wavefront; red: the MW_CHECK reductions.
template <typename T, int NX, int NU, int NG, typename ST, int W>
__device__ __noinline__ void mw_op(const Layout& Lm, const Settings& st, int b_, int64_t s0_, int N_, MwCmd c,
                                   lptr<T> buf, double* FX, lptr<int> bad, lptr<double> red) {
  constexpr int R = 4 * W;
  constexpr int nn = (NX + NU) * (NX + NU);
  const int b = uni(b_), N = uni(N_), op = uni(c.op);
  const int64_t s0 = uni(s0_);
  const double rho_bar = uni(c.rho_bar);
  if (op == MW_FACTOR) {
    constexpr int FORM = sizeof(T) == 4 ? FACTOR_WV : FACTOR_PK;
    const Group g{(int)(threadIdx.x & (ROW - 1)), b, s0, N};
    const int bd = factor_chunked<T, NX, NU, NG, ST::TI, FORM, 1, R>(Lm, g, st.sigma, st.rho_f_scale * rho_bar,
                                                                      rho_bar, nullptr, FX);
    if ((threadIdx.x & 63) == 0) bad[threadIdx.x >> 6] = bd;
  } else if (op == MW_PREP) {
    prepare_segments<T, NX, NU, NG, R>(Lm, b, s0, N, buf, buf + R * nn);
  } else if (op == MW_ITERS) {
    run_segment<T, NX, NU, NG, ST, true, R>(Lm, st, b, s0, N, uni(c.k), uni(c.nb), rho_bar, buf);
  } else if (op == MW_CHECK) {
    // the boundary's FP64 work with the stages over all R rows; each
    // wavefront's maxima / sums into LDS, combined by thread 0
    const int parts = uni(c.k);
    WaveGroup wg;
    wg.lane = (int)(threadIdx.x & (ROW - 1));
    wg.row = (int)(threadIdx.x >> 4);
    wg.b = b, wg.s0 = s0, wg.N = N;
    const int i = wg.lane, wv = (int)(threadIdx.x >> 6);
    const bool lead = (threadIdx.x & 63) == 0;
    if (parts & MW_CHECK_RESID) {
      const int kind = (i < NG) ? (int)Lm.soft[i] : 0;
      const Resid P = residuals_wave<T, NX, NU, NG, ST, 1, R>(Lm, wg, kind, Lm.gamma2, Lm.gamma1);
      if (lead) {
        lptr<double> r = red + wv * MW_RED_F;
        r[0] = P.rp, r[1] = P.rd, r[2] = P.ps, r[3] = P.ds;
        r[4] = P.rp_u, r[5] = P.rd_u, r[6] = P.ps_u, r[7] = P.ds_u;
        r[8] = (double)P.nonfinite;
      }
    }
    if (parts & MW_CHECK_PINF) {
      const PinfPart P = pinf_parts<T, NX, NU, NG, 1, R>(Lm, wg);
      if (lead) {
        lptr<double> r = red + wv * MW_RED_F;
        r[9] = P.m_aty, r[10] = P.m_dy, r[11] = P.sup, r[12] = (double)P.soft_bad;
      }
    }
    if (parts & MW_CHECK_KEEP) {
      T* yf = (T*)Lm.yf;
      T* yg = (T*)Lm.yg;
      T* pf = (T*)Lm.ypf;
      T* pg = (T*)Lm.ypg;
      for (int e = (int)threadIdx.x; e < (N + 1) * ROW; e += 64 * W) {
        const size_t k = (size_t)s0 * ROW + e;
        pf[k] = yf[k];
        pg[k] = yg[k];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      lptr<double> o = red + W * MW_RED_F;
      for (int f = 0; f < MW_RED_F; ++f) {
        double v = red[f];
        for (int k = 1; k < W; ++k) v = (f == 11) ? v + red[k * MW_RED_F + f] : fmax(v, red[k * MW_RED_F + f]);
        o[f] = v;
      }
    }
  }
  __syncthreads();
}

// LDS of a multi-wavefront instance
template <typename T, int NX, int NU, int NG, int W>
struct MwShared {
  static constexpr int R = 4 * W, nn = (NX + NU) * (NX + NU);
  T buf[2 * R * nn + 2 * R * ROW];  // T blocks, U blocks, exchange slots
  MwCmd cmd;
  int bad[W];
  double red[(W + 1) * MW_RED_F];  // MW_CHECK reductions
};

// workgroup width of the continuation of a one-wavefront instance
// (Settings::tail_after)
constexpr int TAIL_W = 2;

// One complete ADMM solve of one instance (Algorithm 3 with the stopping
// test and rho adaptation): FP64 factorisation, iterations up to each
// boundary, FP64 residuals and decisions at the boundary, refactorisation
// after an accepted rho change.  W = 1: the whole solve on one wavefront;
// W > 1: wavefront 0 of a W-wavefront workgroup, the heavy parts posted as
// workgroup operations.  The iteration count, rho and the factorisation
// count start from the instance's entries; RESUME: the solve continues one
// that a one-wavefront solve handed over at st.tail_after (its factorisation
// is current unless flagged, its check multipliers kept if flagged).
template <typename T, int NX, int NU, int NG, typename ST, int W, bool RESUME = false>
__device__ __forceinline__ void admm_solve_body(const Layout& L, const Settings& st, const WaveGroup& w,
                                                MwShared<T, NX, NU, NG, W>* sh, double* FX) {
  // the non-inlined callees get copies in memory: the kernel arguments
  // themselves never have their address taken
  const Layout Lc = L;
  const Settings sc = st;
  constexpr int64_t nn = (int64_t)(NX + NU) * (NX + NU);
  constexpr int TAG = W > 1 ? 1 : 0;
  const int i = w.lane;
  const Group g{w.lane, w.b, w.s0, w.N};
  const int kind = (i < NG) ? (int)L.soft[i] : 0;
  double rho_bar = L.rho[w.b];
  int nfact = L.nfact[w.b];
  int status = ST_RUNNING;
  Resid R{INFINITY, INFINITY, 0.0, 0.0, 0};
  // post a workgroup operation and take part in it
  auto post = [&](int op, int k, int nb) {
    if constexpr (W > 1) {
      if (threadIdx.x == 0) sh->cmd = MwCmd{op, k, nb, rho_bar};
      __syncthreads();
      mw_op<T, NX, NU, NG, ST, W>(Lc, sc, w.b, w.s0, w.N, MwCmd{op, k, nb, rho_bar}, (lptr<T>)sh->buf, FX,
                                  (lptr<int>)sh->bad, (lptr<double>)sh->red);
    }
  };
  auto local_sync = [&] {
    if constexpr (W > 1)
      wave_local_sync();
    else
      wave_sync();
  };

  const bool adapt_on = st.adapt_rho && st.k_rho > 0;
  int k = L.iters[w.b];
  bool need = true;
  bool have_prev = false;  // multipliers of an earlier check are kept (ypf, ypg)
  bool seg_ready = false;  // transfer blocks of the current factorisation are formed
  if constexpr (RESUME) {
    const int f = L.tail_flags[w.b];
    need = (f & 1) != 0;
    have_prev = (f & 2) != 0;
  }
  // a one-wavefront instance hands over to a workgroup at st.tail_after
  const bool hand_over = W == 1 && st.tail_after > 0 && !L.pcg && w.N >= mw_floor_n(TAIL_W);
  // launch shape of the next iterations: long horizons always segmented; the
  // rest switch to it at iteration seg_after (few instances are left running
  // by then, and the shorter serial depth beats the extra block reads)
  auto segmented = [&](int kk) {
    if (W == 1 && L.pcg) return false;  // the PCG updates have no chains to segment
    return W > 1 || w.N >= st.seg_min_n || (kk >= st.seg_after && w.N >= SEG_FLOOR_N);
  };
  for (;;) {
    if (need) {  // the only call site of the factorisation
      int bad = 0;
      if constexpr (W > 1) {
        post(MW_FACTOR, 0, 0);
#pragma unroll
        for (int v = 0; v < W; ++v) bad |= sh->bad[v];
      } else {
        constexpr int FORM = sizeof(T) == 4 ? FACTOR_WV : FACTOR_PK;
        // long horizons: the chunked factorisation (same blocks, shorter serial depth)
        const bool chunked = !L.pcg && w.N >= st.seg_min_n && w.N >= FAC_CHUNK_MIN_N;
        if (L.pcg)  // the PCG blocks: Theta_t, Theta_t^-1, Phi_t (no recursion)
          bad = factor_instance<T, NX, NU, NG, ST::TI, FACTOR_PCG>(Lc, g, st.sigma, st.rho_f_scale * rho_bar,
                                                                   rho_bar, nullptr, w.row);
        else
          bad = chunked ? factor_chunked<T, NX, NU, NG, ST::TI, FORM>(Lc, g, st.sigma, st.rho_f_scale * rho_bar,
                                                                      rho_bar, nullptr)
                        : factor_instance<T, NX, NU, NG, ST::TI, FORM>(Lc, g, st.sigma, st.rho_f_scale * rho_bar,
                                                                       rho_bar, nullptr, w.row);
        wave_sync();
      }
      if (bad) {
        status = 3;
        break;
      }
      ++nfact;
      need = false;
      seg_ready = false;
    }
    if (k >= st.max_iter) break;
    int nb = st.max_iter;
    if (st.k_check > 0) nb = min(nb, (k / st.k_check + 1) * st.k_check);
    if (adapt_on) nb = min(nb, (k / st.k_rho + 1) * st.k_rho);
    if (st.seg_after > k && st.seg_after < nb) nb = st.seg_after;  // the shape changes at a segment start
    if (hand_over && st.tail_after > k && st.tail_after < nb) nb = st.tail_after;
    const bool seg = segmented(k);
    if (seg && !seg_ready) {
      if constexpr (W > 1) {
        post(MW_PREP, 0, 0);
      } else {
        prepare_segments<T, NX, NU, NG>(Lc, w.b, w.s0, w.N, (T*)L.SegT + (int64_t)w.b * 4 * nn,
                                        (T*)L.SegU + (int64_t)w.b * 4 * nn);
        wave_sync();
      }
      seg_ready = true;
    }
    if constexpr (W > 1) {
      post(MW_ITERS, k, nb);
      k = nb;
    } else {
      if (L.pcg)
        k = run_segment<T, NX, NU, NG, ST, false, 4, true>(Lc, sc, w.b, w.s0, w.N, k, nb, rho_bar);
      else
        k = seg ? run_segment<T, NX, NU, NG, ST, true>(Lc, sc, w.b, w.s0, w.N, k, nb, rho_bar)
                : run_segment<T, NX, NU, NG, ST, false>(Lc, sc, w.b, w.s0, w.N, k, nb, rho_bar);
    }
    const int check = (st.k_check > 0 && nb % st.k_check == 0) ? 1 : 0;
    const int adapt = (adapt_on && nb % st.k_rho == 0) ? 1 : 0;
    const int last = (nb == st.max_iter) ? 1 : 0;
    if (check || adapt || last) {
      // infeasibility test from the second check on (the first has no earlier multipliers)
      const bool want_pinf = check && have_prev && st.eps_pinf > 0.0;
      int pinf = 0;
      if constexpr (W > 1) {
        // on every row of the workgroup (MW_CHECK), the combined values in sh->red
        post(MW_CHECK, MW_CHECK_RESID | (want_pinf ? MW_CHECK_PINF : 0), 0);
        const double* o = sh->red + W * MW_RED_F;
        R = Resid{o[0], o[1], o[2], o[3], o[4], o[5], o[6], o[7], (int)o[8]};
        if (want_pinf) pinf = pinf_decide(PinfPart{o[9], o[10], o[11], (int)o[12]}, st.eps_pinf);
      } else {
        R = residuals_wave<T, NX, NU, NG, ST, TAG>(Lc, w, kind, L.gamma2, L.gamma1);
        if (want_pinf) pinf = pinf_wave<T, NX, NU, NG, TAG>(Lc, w, st.eps_pinf);
      }
      status = boundary_decision(R, st, check, adapt, last, pinf, rho_bar, need);
      if (status != ST_RUNNING) break;
      if (check && st.eps_pinf > 0.0) {
        if constexpr (W > 1) {
          post(MW_CHECK, MW_CHECK_KEEP, 0);
        } else {
          local_sync();
          keep_multipliers<T>(Lc, w);
          local_sync();
        }
        have_prev = true;
      }
    }
    if (hand_over && k >= st.tail_after) {
      // the state stays in memory; admm_solve_tail_kernel continues the solve
      if (threadIdx.x == 0) {
        L.tail_flags[w.b] = (need ? 1 : 0) | (have_prev ? 2 : 0);
        L.tail_list[atomicAdd(L.tail_count, 1)] = w.b;
      }
      break;
    }
  }
  if constexpr (W > 1) {
    if (threadIdx.x == 0) sh->cmd = MwCmd{MW_EXIT, 0, 0, 0.0};
    __syncthreads();  // releases the other wavefronts
  }
  if (threadIdx.x == 0) {
    L.iters[w.b] = k;
    L.nfact[w.b] = nfact;
    L.rho[w.b] = rho_bar;
    L.status[w.b] = status;
    L.rprim[w.b] = R.rp_u;
    L.rdual[w.b] = R.rd_u;
  }
}

// One instance per wavefront; instances with a multi-wavefront workgroup
// (horizon N >= L.mw_min_n) are left to admm_solve_mw_kernel.  Instances
// never wait for each other.
template <typename T, int NX, int NU, int NG, typename ST>
__global__ __launch_bounds__(64) void admm_solve_wave_kernel(Layout L, Settings st) {
  WaveGroup w;
  if (!wave_group(L, w)) return;
  if (L.status[w.b] != ST_RUNNING) return;
  if (L.n_mw > 0 && w.N >= L.mw_min_n) return;
  admm_solve_body<T, NX, NU, NG, ST, 1>(L, st, w, nullptr, nullptr);
}

// One instance per workgroup of W wavefronts: the instances L.mw_list[0 ..
// L.n_mw), each with its own exchange blocks for the chunked factorisation
// (L.FacXmw, fx_slots(4 W) n x n blocks per workgroup).
template <typename T, int NX, int NU, int NG, typename ST>
__global__ __launch_bounds__(64 * mw_waves<NX + NU>()) void admm_solve_mw_kernel(Layout L, Settings st) {
  constexpr int W = mw_waves<NX + NU>();
  constexpr int nn = (NX + NU) * (NX + NU);
  __shared__ MwShared<T, NX, NU, NG, W> sh;
  const int slot = blockIdx.x;
  if (slot >= L.n_mw) return;
  WaveGroup w;
  w.lane = threadIdx.x & (ROW - 1);
  w.row = (threadIdx.x >> 4) & 3;
  w.b = L.mw_list[slot];
  w.s0 = L.stage_off[w.b];
  w.N = (int)(L.stage_off[w.b + 1] - w.s0) - 1;
  if (L.status[w.b] != ST_RUNNING) return;  // the whole workgroup
  double* FX = L.FacXmw + (size_t)slot * fx_slots(4 * W) * nn;
  if (threadIdx.x < 64) {
    admm_solve_body<T, NX, NU, NG, ST, W>(L, st, w, &sh, FX);
    return;
  }
  const Layout Lc = L;
  const Settings sc = st;
  for (;;) {
    __syncthreads();  // an operation has been posted
    const MwCmd c = sh.cmd;
    if (c.op == MW_EXIT) break;
    mw_op<T, NX, NU, NG, ST, W>(Lc, sc, w.b, w.s0, w.N, c, (lptr<T>)sh.buf, FX, (lptr<int>)sh.bad,
                                (lptr<double>)sh.red);
  }
}

// The continuation: one workgroup of TAIL_W wavefronts per instance that a
// one-wavefront solve handed over (L.tail_list[0 .. *L.tail_count), list
// slot = block); launched after admm_solve_wave_kernel on the same stream
// with one block per instance of the batch, the blocks past the count exit.
template <typename T, int NX, int NU, int NG, typename ST>
__global__ __launch_bounds__(64 * TAIL_W) void admm_solve_tail_kernel(Layout L, Settings st) {
  constexpr int W = TAIL_W;
  constexpr int nn = (NX + NU) * (NX + NU);
  __shared__ MwShared<T, NX, NU, NG, W> sh;
  const int slot = blockIdx.x;
  if (slot >= *L.tail_count) return;  // the whole workgroup
  WaveGroup w;
  w.lane = threadIdx.x & (ROW - 1);
  w.row = (threadIdx.x >> 4) & 3;
  w.b = L.tail_list[slot];
  w.s0 = L.stage_off[w.b];
  w.N = (int)(L.stage_off[w.b + 1] - w.s0) - 1;
  if (L.status[w.b] != ST_RUNNING) return;
  double* FX = L.FacXtail + (size_t)slot * fx_slots(4 * W) * nn;
  if (threadIdx.x < 64) {
    admm_solve_body<T, NX, NU, NG, ST, W, true>(L, st, w, &sh, FX);
    return;
  }
  const Layout Lc = L;
  const Settings sc = st;
  for (;;) {
    __syncthreads();  // an operation has been posted
    const MwCmd c = sh.cmd;
    if (c.op == MW_EXIT) break;
    mw_op<T, NX, NU, NG, ST, W>(Lc, sc, w.b, w.s0, w.N, c, (lptr<T>)sh.buf, FX, (lptr<int>)sh.bad,
                                (lptr<double>)sh.red);
  }
}

}  // namespace ocpk
