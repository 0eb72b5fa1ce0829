// Problem setup and output kernels: expansion of a linear-quadratic OCP into
// its QP blocks (the convexification of a linear problem is exact; Appendix
// "QP Approximation"), precision conversion of the per-iteration data and the
// copy of the padded ADMM state into the caller's compact FP64 buffers.
#pragma once

#include "dev_common.h"

namespace ocpk {

// One thread per instance; n <= 16 so per-instance work is a few hundred
// stores.  Cost 1/2(x'Qx + u'Ru) for t < N, 1/2(x'Q_f x + u'Ru) at t = N;
// dynamics A x + B u - x+ = 0, i.e. A^- = [A B], A^+ = [-I 0], c = 0.
__global__ void lti_expand_kernel(int B, int nx, int nu, int ng, const double* __restrict__ A,
                                  const double* __restrict__ Bm, const double* __restrict__ Qd,
                                  const double* __restrict__ Rd, const double* __restrict__ Qfd,
                                  const double* __restrict__ Gsh, const double* __restrict__ lo,
                                  const double* __restrict__ hi, const double* __restrict__ x0, double* __restrict__ D,
                                  double* __restrict__ Am, double* __restrict__ Ap, double* __restrict__ G,
                                  double* __restrict__ lo_o, double* __restrict__ hi_o, double* __restrict__ xinit) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int n = nx + nu;
  double* D0 = D + (size_t)(2 * b) * n * n;
  double* D1 = D0 + (size_t)n * n;
  for (int k = 0; k < n * n; ++k) {
    D0[k] = 0.0;
    D1[k] = 0.0;
  }
  for (int k = 0; k < nx; ++k) {
    D0[k * n + k] = Qd[(size_t)b * nx + k];
    D1[k * n + k] = Qfd[(size_t)b * nx + k];
  }
  for (int k = 0; k < nu; ++k) {
    D0[(nx + k) * n + nx + k] = Rd[(size_t)b * nu + k];
    D1[(nx + k) * n + nx + k] = Rd[(size_t)b * nu + k];
  }
  double* am = Am + (size_t)b * nx * n;
  double* ap = Ap + (size_t)b * nx * n;
  for (int r = 0; r < nx; ++r) {
    for (int c = 0; c < nx; ++c) {
      am[r * n + c] = A[(size_t)b * nx * nx + r * nx + c];
      ap[r * n + c] = (r == c) ? -1.0 : 0.0;
    }
    for (int c = 0; c < nu; ++c) {
      am[r * n + nx + c] = Bm[(size_t)b * nx * nu + r * nu + c];
      ap[r * n + nx + c] = 0.0;
    }
    xinit[(size_t)b * nx + r] = x0[(size_t)b * nx + r];
  }
  double* gg = G + (size_t)b * ng * n;
  for (int k = 0; k < ng * n; ++k) gg[k] = Gsh[k];
  for (int r = 0; r < ng; ++r) {
    lo_o[(size_t)b * ng + r] = lo[(size_t)b * ng + r];
    hi_o[(size_t)b * ng + r] = hi[(size_t)b * ng + r];
  }
}

template <typename T>
__global__ void convert_kernel(const double* __restrict__ src, T* __restrict__ dst, size_t len) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < len) dst[k] = T(src[k]);
}

// Rescaling factors of instance b (Remark 4; Layout::sc, [B][3][ROW]).
// Factor codes: 1, d_j, 1/d_j, e_j, c, c d_j, 1/e_j, e_j / c, 1/(c d_j)
enum { SF_ONE = 0, SF_D, SF_INV_D, SF_E, SF_C, SF_CD, SF_INV_E, SF_E_OVER_C, SF_INV_CD };

__device__ __forceinline__ double scale_factor(const double* __restrict__ sc, int b, int j, int code) {
  if (code == SF_ONE || !sc) return 1.0;
  const double* p = sc + (size_t)b * 3 * ROW;
  switch (code) {
    case SF_D: return p[j];
    case SF_INV_D: return 1.0 / p[j];
    case SF_E: return p[ROW + j];
    case SF_C: return p[2 * ROW];
    case SF_CD: return p[2 * ROW] * p[j];
    case SF_INV_E: return 1.0 / p[ROW + j];
    case SF_E_OVER_C: return p[ROW + j] / p[2 * ROW];
    default: return 1.0 / (p[2 * ROW] * p[j]);
  }
}

// Entry-wise rescaling of `nblk` blocks of R x Cc entries in place: entry
// (r, j) of block k is multiplied by factor(row code, r) * factor(column code,
// j) of its instance -- k / per when the blocks are per instance (per > 0),
// stage_inst[k] when they are per stage (per = 0).
__global__ void scale_blocks_kernel(double* __restrict__ p, int64_t nblk, int R, int Cc, int per,
                                    const int32_t* __restrict__ stage_inst, const double* __restrict__ sc, int rowf,
                                    int colf) {
  const int64_t len = nblk * R * Cc;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = k / (R * Cc);
    const int r = (int)((k / Cc) % R), j = (int)(k % Cc);
    const int b = per > 0 ? (int)(blk / per) : stage_inst[blk];
    p[k] *= scale_factor(sc, b, r, rowf) * scale_factor(sc, b, j, colf);
  }
}

// padded [S][ROW] state -> compact FP64 [S][w], entry j multiplied by the
// factor `code` of the stage's instance (original variables of a rescaled QP)
template <typename T>
__global__ void unpad_kernel(const T* __restrict__ src, double* __restrict__ dst, int64_t S, int w,
                             const int32_t* __restrict__ inst, const double* __restrict__ sc, int code) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (size_t)S * w) return;
  const size_t s = k / w, j = k % w;
  const double f = sc ? scale_factor(sc, inst[s], (int)j, code) : 1.0;
  dst[k] = double(src[s * ROW + j]) * f;
}

// y_f: internal slots (dynamics row t at stage t, initial-state rows at the
// last stage of each instance) -> output order (initial rows at the first
// stage, dynamics row t at stage t+1); rescaled QPs: times 1/(c d_j)
template <typename T>
__global__ void unpad_yf_kernel(const T* __restrict__ src, double* __restrict__ dst, const int64_t* __restrict__ off,
                                const int32_t* __restrict__ inst, int64_t S, int w, const double* __restrict__ sc) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (size_t)S * w) return;
  const int64_t s = (int64_t)(k / w);
  const size_t j = k % w;
  const int b = inst[s];
  const int64_t from = (s == off[b]) ? off[b + 1] - 1 : s - 1;
  const double f = sc ? scale_factor(sc, b, (int)j, SF_INV_CD) : 1.0;
  dst[k] = double(src[(size_t)from * ROW + j]) * f;
}

// Box normalisation of instance b (one thread per instance; Remark 4), in
// powers of two so that the transform is exact: a variable j bounded by a
// hard selection row of G (read at stage 0) gets d_j = 2^rint(p log2 h_j),
// h_j the half width of its bounds, the others 1; e_g = 1/d_j on selection
// rows, 2^-rint(log2 max_j |G_rj d_j|) on the other hard rows, 1 on soft
// rows; c = 2^-rint(log2 m), m the largest diagonal entry of
// diag(d) D_t diag(d) over the instance's stages.
__global__ void box_scaling_kernel(int B, int n, int ng, int ti, const int64_t* __restrict__ off,
                                   const double* __restrict__ D, const double* __restrict__ G,
                                   const double* __restrict__ lo, const double* __restrict__ hi,
                                   const uint8_t* __restrict__ soft, double p, double* __restrict__ sc) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int64_t s0 = off[b], s1 = off[b + 1];
  const size_t g0 = ti ? (size_t)b : (size_t)s0;
  const double* Gb = G + g0 * ng * n;
  double d[ROW], e[ROW];
  int sel[ROW];
  for (int j = 0; j < ROW; ++j) d[j] = e[j] = 1.0, sel[j] = -1;
  for (int r = 0; r < ng; ++r) {
    int hit = -1, cnt = 0;
    for (int j = 0; j < n; ++j)
      if (Gb[(size_t)r * n + j] != 0.0) hit = j, ++cnt;
    if (cnt == 1 && Gb[(size_t)r * n + hit] == 1.0 && soft[r] == 0) {
      sel[r] = hit;
      const double half = 0.5 * (hi[g0 * ng + r] - lo[g0 * ng + r]);
      if (isfinite(half) && half > 0.0) d[hit] = exp2(rint(p * log2(half)));
    }
  }
  for (int r = 0; r < ng; ++r) {
    if (soft[r] != 0) continue;
    if (sel[r] >= 0) {
      e[r] = 1.0 / d[sel[r]];
    } else {
      double m = 0.0;
      for (int j = 0; j < n; ++j) m = fmax(m, fabs(Gb[(size_t)r * n + j] * d[j]));
      e[r] = m > 0.0 ? 1.0 / exp2(rint(log2(m))) : 1.0;
    }
  }
  double m = 0.0;
  const int64_t k0 = ti ? 2 * (int64_t)b : s0, k1 = ti ? 2 * (int64_t)b + 2 : s1;
  for (int64_t k = k0; k < k1; ++k)
    for (int j = 0; j < n; ++j) m = fmax(m, D[(size_t)k * n * n + (size_t)j * n + j] * d[j] * d[j]);
  const double c = m > 0.0 ? 1.0 / exp2(rint(log2(m))) : 1.0;
  double* o = sc + (size_t)b * 3 * ROW;
  for (int j = 0; j < ROW; ++j) {
    o[j] = j < n ? d[j] : 1.0;
    o[ROW + j] = j < ng ? e[j] : 1.0;
    o[2 * ROW + j] = c;
  }
}

// pack per-instance factors [B][n], [B][ng], [B] into [B][3][ROW] (padding 1)
__global__ void pack_scaling_kernel(const double* __restrict__ d, const double* __restrict__ e,
                                    const double* __restrict__ c, int B, int n, int ng, double* __restrict__ sc) {
  const int64_t len = (int64_t)B * 3 * ROW;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(k / (3 * ROW)), r = (int)((k / ROW) % 3), j = (int)(k % ROW);
    double v = 1.0;
    if (r == 0 && j < n) v = d[(size_t)b * n + j];
    if (r == 1 && j < ng) v = e[(size_t)b * ng + j];
    if (r == 2) v = c[b];
    sc[k] = v;
  }
}

// zero the unused last-stage slot of per-stage blocks (dynamics blocks of
// stage N have no row), so boundary terms in the branch-free sweeps vanish
__global__ void zero_last_stage_kernel(double* __restrict__ p, const int64_t* __restrict__ off, int B, int sz) {
  const int b = blockIdx.x;
  if (b >= B) return;
  double* q = p + (size_t)(off[b + 1] - 1) * sz;
  for (int k = threadIdx.x; k < sz; k += blockDim.x) q[k] = 0.0;
}

// clear n 64-bit words (a kernel rather than a memset node, so the clearing
// also replays correctly inside a captured graph)
__global__ void zero_u64_kernel(uint64_t* __restrict__ p, size_t n) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    p[k] = 0;
}

// Stage layout of a ragged batch on the device (one workgroup): stage
// offsets (prefix sums of N_b + 1), the longest-first processing order (a
// stable descending rank: instance b goes after every longer one and after
// the equal ones before it) and the instance of every stage.
__global__ void stage_layout_kernel(const int32_t* __restrict__ hz, int B, int64_t* __restrict__ off,
                                    int32_t* __restrict__ order, int32_t* __restrict__ stage_inst) {
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    off[0] = 0;
    for (int b = 0; b < B; ++b) off[b + 1] = (acc += hz[b] + 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    const int hb = hz[b];
    int rank = 0;
    for (int c = 0; c < B; ++c) rank += (hz[c] > hb) || (hz[c] == hb && c < b);
    order[rank] = b;
    for (int64_t k = off[b]; k < off[b + 1]; ++k) stage_inst[k] = b;
  }
}

// compact FP64 [S][w] -> padded [S][ROW] state
template <typename T>
__global__ void pad_kernel(const double* __restrict__ src, T* __restrict__ dst, int64_t S, int w) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (size_t)S * ROW) return;
  const size_t s = k / ROW, j = k % ROW;
  dst[k] = (j < (size_t)w) ? T(src[s * w + j]) : T(0);
}

}  // namespace ocpk
