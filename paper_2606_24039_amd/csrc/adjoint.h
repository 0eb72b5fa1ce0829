// Implicit-differentiation adjoint (filled in below the ADMM path).
#pragma once
#include "admm.h"
namespace ocpk {
struct AdjArgs {
  int dummy;
};
template <int NX, int NU, int NG, bool TI>
__global__ void adjoint_kernel(Layout L, AdjArgs a) {}
}  // namespace ocpk
