// Kernel instantiations of one compiled stage shape (OCP_NX, OCP_NU, OCP_NG)
// and one iteration precision (OCP_F32: FP32 iterations over the FP64
// factorisation, else FP64): the persistent ADMM solve and the adjoint for
// each structure variant.  The build compiles this file once per table entry
// of ocp.hip, in parallel.
#include "dispatch.h"

#ifndef OCP_NX
#define OCP_NX 4
#define OCP_NU 2
#define OCP_NG 4
#endif
#ifdef OCP_F32
using IterT = float;
#define OCP_PTAG f32
#else
using IterT = double;
#define OCP_PTAG f64
#endif

#define OCP_CAT_(a, b, c, d) ocp_entry_##a##_##b##_##c##_##d
#define OCP_CAT(a, b, c, d) OCP_CAT_(a, b, c, d)

namespace ocpk {

// host function (a namespace-scope table of host function pointers would also
// be emitted, unresolvable, for the device)
const PrecEntry* OCP_CAT(OCP_NX, OCP_NU, OCP_NG, OCP_PTAG)() {
  static const PrecEntry e = {
      {launch_solve<IterT, OCP_NX, OCP_NU, OCP_NG, StTV>, launch_solve<IterT, OCP_NX, OCP_NU, OCP_NG, StTI>,
       launch_solve<IterT, OCP_NX, OCP_NU, OCP_NG, StBox>},
      {launch_adjoint<IterT, OCP_NX, OCP_NU, OCP_NG, StTV>, launch_adjoint<IterT, OCP_NX, OCP_NU, OCP_NG, StTI>,
       launch_adjoint<IterT, OCP_NX, OCP_NU, OCP_NG, StBox>},
  };
  return &e;
}

}  // namespace ocpk
