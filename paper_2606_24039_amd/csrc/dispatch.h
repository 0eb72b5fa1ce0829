// Dispatch of the compiled stage shapes: kernel timing, the launch
// functions of the persistent solve and the adjoint, and the table entry of
// one (nx, nu, ng, iteration precision).  Each entry is instantiated in its
// own translation unit (inst.hip, compiled once per shape and precision).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "adjoint.h"
#include "ocp_admm.h"
#include "wave.h"

namespace ocpk {

// ---------------------------------------------------------------------------
// kernel timing: optional HIP-event pairs around the solver's launches, by
// kernel class (ocp_kernel_class).  Off by default; events are created on
// first use and recycled after each read.
// ---------------------------------------------------------------------------
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> ev;  // 2 per recorded launch
  std::vector<int> cls;
  size_t used = 0;
  double ms[OCP_K_COUNT] = {0};
  int64_t launches[OCP_K_COUNT] = {0};

  bool begin(int c, hipStream_t st) {
    if (!on) return false;
    if (2 * used + 2 > ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return false;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return false;
      }
      ev.push_back(a);
      ev.push_back(b);
      cls.push_back(c);
    }
    cls[used] = c;
    (void)hipEventRecord(ev[2 * used], st);
    return true;
  }
  void end(hipStream_t st) { (void)hipEventRecord(ev[2 * used++ + 1], st); }
  hipError_t collect() {
    for (size_t k = 0; k < used; ++k) {
      hipError_t e = hipEventSynchronize(ev[2 * k + 1]);
      if (e != hipSuccess) return e;
      float t = 0.f;
      e = hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]);
      if (e != hipSuccess) return e;
      ms[cls[k]] += t;
      launches[cls[k]] += 1;
    }
    used = 0;
    return hipSuccess;
  }
  void release() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
    cls.clear();
    used = 0;
  }
};

// launch `f` bracketed by a timing pair of class `c` when timing is on
template <typename F>
void timed(Prof* p, int c, hipStream_t st, F&& f) {
  const bool t = p && p->begin(c, st);
  f();
  if (t) p->end(st);
}

// ---------------------------------------------------------------------------
// dispatch table: one instantiation per compiled (nx, nu, ng)
// ---------------------------------------------------------------------------
// a second stream and two events: the multi-wavefront launch of a mixed batch
// runs beside the one-wavefront launch (fork / join on the caller's stream)
struct Fork {
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
using SolveFn = void (*)(const Layout&, const Settings&, int32_t*, hipStream_t, Prof*, const Fork*);
using AdjFn = void (*)(const Layout&, const AdjArgs&, hipStream_t, Prof*, const Fork*);

// One ADMM solve: per-solve initialisation, then one workgroup of
// mw_waves() wavefronts per long instance (N >= L.mw_min_n) and one
// wavefront per other instance run the whole of Algorithm 3 (factorisation,
// iterations, FP64 checks, rho adaptation and refactorisation) without
// waiting for other instances.
template <typename T, int NX, int NU, int NG, typename ST>
void launch_solve(const Layout& L, const Settings& s, int32_t* need, hipStream_t st, Prof* pf, const Fork* fk) {
  timed(pf, OCP_K_OTHER, st,
        [&] { hipLaunchKernelGGL((admm_init_kernel<T>), dim3(L.init_blocks), dim3(256), 0, st, L, s, need); });
  // both launches of a mixed batch side by side: the workgroup launch on the
  // second stream, forked from and joined back into the caller's stream
  const bool both = L.n_mw > 0 && L.n_mw < L.B && fk && fk->aux;
  hipStream_t mst = st;
  if (both && hipEventRecord(fk->fork, st) == hipSuccess && hipStreamWaitEvent(fk->aux, fk->fork, 0) == hipSuccess)
    mst = fk->aux;
  if (L.n_mw > 0)
    timed(pf, OCP_K_SOLVE, mst, [&] {
      hipLaunchKernelGGL((admm_solve_mw_kernel<T, NX, NU, NG, ST>), dim3(L.n_mw), dim3(64 * mw_waves<NX + NU>()), 0,
                         mst, L, s);
    });
  if (L.n_mw < L.B) {
    timed(pf, OCP_K_SOLVE, st,
          [&] { hipLaunchKernelGGL((admm_solve_wave_kernel<T, NX, NU, NG, ST>), dim3(L.B), dim3(64), 0, st, L, s); });
    // instances handed over at s.tail_after continue on two-wavefront
    // workgroups (FP32 iterations; one block per instance, the unused exit)
    if constexpr (sizeof(T) == 4) {
      if (s.tail_after > 0 && L.tail_count)
        timed(pf, OCP_K_SOLVE, st, [&] {
          hipLaunchKernelGGL((admm_solve_tail_kernel<T, NX, NU, NG, ST>), dim3(L.B), dim3(64 * TAIL_W), 0, st, L, s);
        });
    }
  }
  if (mst != st) {
    (void)hipEventRecord(fk->join, mst);
    (void)hipStreamWaitEvent(st, fk->join, 0);
  }
}

// one instance per wavefront, and (time-varying data) one workgroup per
// multi-wavefront instance, side by side as in launch_solve
template <typename T, int NX, int NU, int NG, typename ST>
void launch_adjoint(const Layout& L, const AdjArgs& a, hipStream_t st, Prof* pf, const Fork* fk) {
  const int n_mw = ST::TI ? 0 : L.n_mw;
  const bool both = n_mw > 0 && n_mw < L.B && fk && fk->aux;
  hipStream_t mst = st;
  if (both && hipEventRecord(fk->fork, st) == hipSuccess && hipStreamWaitEvent(fk->aux, fk->fork, 0) == hipSuccess)
    mst = fk->aux;
  if constexpr (!ST::TI) {
    if (n_mw > 0)
      timed(pf, OCP_K_ADJOINT, mst, [&] {
        hipLaunchKernelGGL((adjoint_mw_kernel<T, NX, NU, NG, ST>), dim3(n_mw), dim3(64 * mw_waves<NX + NU>()), 0,
                           mst, L, a);
      });
  }
  if (n_mw < L.B)
    timed(pf, OCP_K_ADJOINT, st,
          [&] { hipLaunchKernelGGL((adjoint_kernel<T, NX, NU, NG, ST>), dim3(L.B), dim3(64), 0, st, L, a); });
  if (mst != st) {
    (void)hipEventRecord(fk->join, mst);
    (void)hipStreamWaitEvent(st, fk->join, 0);
  }
}

// structure variants of the iteration kernel
enum { VAR_TV = 0, VAR_TI = 1, VAR_LTI_BOX = 2 };
using StTV = Structure<false, false, false>;
using StTI = Structure<true, false, false>;
using StBox = Structure<true, true, true>;

// launch functions of one shape and iteration precision, by structure variant
struct PrecEntry {
  SolveFn solve[3];
  AdjFn adj[3];
};

}  // namespace ocpk
