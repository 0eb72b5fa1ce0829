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

// padded [S][ROW] state -> compact FP64 [S][w]
template <typename T>
__global__ void unpad_kernel(const T* __restrict__ src, double* __restrict__ dst, int64_t S, int w) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (size_t)S * w) return;
  const size_t s = k / w, j = k % w;
  dst[k] = double(src[s * ROW + j]);
}

// y_f: internal slots (dynamics row t at stage t, initial-state rows at the
// last stage of each instance) -> output order (initial rows at the first
// stage, dynamics row t at stage t+1)
template <typename T>
__global__ void unpad_yf_kernel(const T* __restrict__ src, double* __restrict__ dst, const int64_t* __restrict__ off,
                                const int32_t* __restrict__ inst, int64_t S, int w) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (size_t)S * w) return;
  const int64_t s = (int64_t)(k / w);
  const size_t j = k % w;
  const int b = inst[s];
  const int64_t from = (s == off[b]) ? off[b + 1] - 1 : s - 1;
  dst[k] = double(src[(size_t)from * ROW + j]);
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
