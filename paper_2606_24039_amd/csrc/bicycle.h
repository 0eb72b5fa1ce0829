// Kinematic-bicycle SQP kernels.
#pragma once
#include "admm.h"
namespace ocpk {
struct BikeArgs {
  int dummy;
};
__global__ void fill_i32_kernel(int32_t* p, int n, int v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}
}  // namespace ocpk
