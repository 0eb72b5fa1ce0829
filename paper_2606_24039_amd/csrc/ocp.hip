// C ABI of the batched SQP-ADMM OCP-QP solver (declarations and contracts in
// include/ocp_admm.h).  Host code: workspace management, argument checks,
// kernel dispatch by compiled stage shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "bicycle.h"
#include "dispatch.h"
#include "ocp_admm.h"
#include "setup.h"

using namespace ocpk;

namespace {

struct Entry {
  int nx, nu, ng;
  const PrecEntry* (*p64)();  // FP64 iterations
  const PrecEntry* (*p32)();  // FP32 iterations over the FP64 factorisation
};

}  // namespace

// one translation unit per compiled shape and precision (inst.hip)
namespace ocpk {
const PrecEntry* ocp_entry_4_2_4_f64();  // 2-D double integrator
const PrecEntry* ocp_entry_4_2_4_f32();
const PrecEntry* ocp_entry_12_4_16_f64();  // random LTI, all variables boxed
const PrecEntry* ocp_entry_12_4_16_f32();
const PrecEntry* ocp_entry_4_2_3_f64();  // kinematic bicycle
const PrecEntry* ocp_entry_4_2_3_f32();
}  // namespace ocpk

namespace {

const Entry kTable[] = {
    {4, 2, 4, ocp_entry_4_2_4_f64, ocp_entry_4_2_4_f32},
    {12, 4, 16, ocp_entry_12_4_16_f64, ocp_entry_12_4_16_f32},
    {4, 2, 3, ocp_entry_4_2_3_f64, ocp_entry_4_2_3_f32},
};

const Entry* find_entry(int nx, int nu, int ng) {
  for (const Entry& e : kTable)
    if (e.nx == nx && e.nu == nu && e.ng == ng) return &e;
  return nullptr;
}

}  // namespace

struct ocp_handle_s {
  ocp_dims d{};
  int n = 0;
  int64_t S = 0;
  int B = 0;
  int maxN = 0;
  bool mixed = false;
  bool ti = false;
  const Entry* entry = nullptr;
  std::vector<void*> allocs;
  size_t bytes = 0;
  char* carve = nullptr;  // when set, the workspace is carved from here instead of allocated

  int64_t* stage_off = nullptr;
  int32_t* order = nullptr;
  double *D = nullptr, *E = nullptr, *q = nullptr, *Am = nullptr, *Ap = nullptr, *bd = nullptr;
  double *G = nullptr, *lo = nullptr, *hi = nullptr, *xinit = nullptr;
  uint8_t* soft = nullptr;
  void *AmT = nullptr, *ApT = nullptr, *GT = nullptr, *qT = nullptr, *bdT = nullptr;
  void *loT = nullptr, *hiT = nullptr, *xinitT = nullptr;
  double *Linv64 = nullptr, *M64 = nullptr;
  void *SubA = nullptr, *SubB = nullptr, *ChF = nullptr, *ChB = nullptr;
  void *SegT = nullptr, *SegU = nullptr, *SegX = nullptr;
  double* FacX = nullptr;
  // multi-wavefront instances: N >= mw_min_n (0: none), their device list,
  // the exchange blocks of their chunked factorisation (mw_cap slots: the
  // instances at or above the smallest admissible threshold)
  int mw_min_n = MW_MIN_N;
  int n_mw = 0, mw_cap = 0;
  bool mw_off = false;  // no multi-wavefront workgroups (workspace carved by ocp_solve_noalloc)
  int32_t* mw_list = nullptr;
  double* FacXmw = nullptr;
  // continuation of one-wavefront instances on two-wavefront workgroups from
  // ADMM iteration tail_after (0: off); buffers allocated when first enabled
  int tail_after = 0;
  int32_t *tail_list = nullptr, *tail_count = nullptr, *tail_flags = nullptr;
  double* FacXtail = nullptr;
  Fork fork;  // second stream for the workgroup launch of a mixed batch (created with the handle)
  std::vector<int32_t> horizons_host;
  // PCG primal updates (ocp_set_linsolve): mode, limits, vectors (allocated by the first switch to PCG)
  int pcg = 0, pcg_max_it = 50;
  double pcg_tol = 1e-6;
  void *pcg_xt = nullptr, *pcg_r = nullptr, *pcg_z = nullptr, *pcg_p = nullptr, *pcg_sp = nullptr;
  int variant = 0;
  int seg_min_n = SEG_MIN_N;  // launch shape: horizons from which the substitutions run segmented
  int seg_after = INT32_MAX;  // iteration from which every running instance does (the batch's tail)
  int8_t gsel[16] = {0}, ginv[16] = {0};
  void *x = nullptr, *v = nullptr, *yf = nullptr, *zg = nullptr, *yg = nullptr, *xi = nullptr;
  void *ypf = nullptr, *ypg = nullptr;  // multipliers at the previous convergence check
  double *rho = nullptr, *rprim = nullptr, *rdual = nullptr;
  int32_t *status = nullptr, *iters = nullptr, *nfact = nullptr, *need = nullptr;
  double gamma2 = 1.0, gamma1 = 1.0;
  bool has_E = false, has_q = false, has_bd = false;
  double* sc = nullptr;  // rescaling factors [B][3][ROW] (Remark 4)
  bool scaled = false;   // the loaded data are rescaled by sc
  double box_p = -1.0;   // >= 0: derive sc from each loaded problem (box normalisation, exponent box_p)
  bool data_set = false, solved = false;

  // bicycle model state
  double* bike_ref = nullptr;
  double* bike_normal = nullptr;
  double* bike_x0 = nullptr;
  double* bike_uinit = nullptr;  // [B][2] (u_0 fixed when bike.u_init is set)
  bool bike_rate = false;        // a control-rate cost: the QPs carry E_t
  ocp_bicycle bike{};
  double *xbar = nullptr, *xibar = nullptr, *yfbar = nullptr, *ygbar = nullptr, *mu = nullptr, *kkt = nullptr;
  int32_t* sqp_done = nullptr;
  int32_t* sqp_frozen = nullptr;
  int32_t* stage_inst = nullptr;
  // line-search chunks (LS_CHUNK stages; a carved workspace keeps one per instance)
  int ls_nchunks = 0;
  int32_t *ls_chunk_inst = nullptr, *ls_chunk_t0 = nullptr, *ls_chunk_off = nullptr;
  double *ls_parts = nullptr, *ls_alpha = nullptr;

  // adjoint scratch (FP64, padded [S][ROW])
  double *adj_rhog = nullptr, *adj_ex = nullptr, *adj_ey = nullptr, *adj_eg = nullptr, *adj_r = nullptr;
  double *adj_v = nullptr, *adj_rg = nullptr;
  double *adj_P = nullptr, *adj_K = nullptr, *adj_Kb = nullptr;  // adjoint factor, FP64 P/K form
  double* adj_dl = nullptr;  // [S][n] right-hand side with a loss on the slacks
  uint8_t soft_host[16] = {0};
  int8_t* adj_act = nullptr;

  Prof prof;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;

  size_t tsz() const { return mixed ? sizeof(float) : sizeof(double); }
};

namespace {

ocp_status hip_ok(hipError_t e) { return e == hipSuccess ? OCP_OK : OCP_E_HIP; }

template <typename P>
ocp_status halloc(ocp_handle h, P** p, size_t bytes, bool count_only) {
  bytes = std::max<size_t>(bytes, 8);
  bytes = (bytes + 255) & ~size_t(255);
  const size_t at = h->bytes;
  h->bytes += bytes;
  if (count_only) return OCP_OK;
  if (h->carve) {  // the caller has checked that the whole workspace fits
    *p = (P*)(h->carve + at);
    return OCP_OK;
  }
  void* ptr = nullptr;
  if (hipMalloc(&ptr, bytes) != hipSuccess) return OCP_E_NOMEM;
  h->allocs.push_back(ptr);
  *p = (P*)ptr;
  return OCP_OK;
}

void free_all(ocp_handle h) {
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
}

ocp_status check_dims(const ocp_dims* d, const int32_t* horizons) {
  if (!d || !horizons) return OCP_E_ARG;
  if (d->batch < 1 || d->nx < 1 || d->nu < 1 || d->ng < 0) return OCP_E_ARG;
  if (d->model < 0 || d->model > 2 || d->precision < 0 || d->precision > 1) return OCP_E_ARG;
  if (d->nx + d->nu > ROW || d->ng > ROW) return OCP_E_SHAPE;
  if (!find_entry(d->nx, d->nu, d->ng)) return OCP_E_SHAPE;
  if (d->model == OCP_MODEL_BICYCLE && (d->nx != 4 || d->nu != 2 || d->ng != 3)) return OCP_E_SHAPE;
  for (int b = 0; b < d->batch; ++b)
    if (horizons[b] < 1) return OCP_E_ARG;
  return OCP_OK;
}

// the list of multi-wavefront instances for the current threshold (longest
// first), host -> device
ocp_status upload_mw_list(ocp_handle h) {
  h->n_mw = 0;
  if (h->mw_off || h->mw_min_n <= 0 || h->mw_cap == 0) return OCP_OK;
  std::vector<int32_t> lst;
  for (int b = 0; b < h->B; ++b)
    if (h->horizons_host[(size_t)b] >= h->mw_min_n) lst.push_back(b);
  std::stable_sort(lst.begin(), lst.end(),
                   [&](int a, int c) { return h->horizons_host[(size_t)a] > h->horizons_host[(size_t)c]; });
  if (lst.empty()) return OCP_OK;
  if (hipMemcpy(h->mw_list, lst.data(), sizeof(int32_t) * lst.size(), hipMemcpyHostToDevice) != hipSuccess)
    return OCP_E_HIP;
  h->n_mw = (int)lst.size();
  return OCP_OK;
}

// allocate (or only count) the workspace
ocp_status build(ocp_handle h, const ocp_dims* d, const int32_t* horizons, bool count_only) {
  h->d = *d;
  h->B = d->batch;
  h->n = d->nx + d->nu;
  h->mixed = d->precision == OCP_PREC_MIXED;
  h->ti = (d->model == OCP_MODEL_LTI) || (d->model == OCP_MODEL_QP && d->time_invariant);
  h->entry = find_entry(d->nx, d->nu, d->ng);
  const int B = h->B, n = h->n, nx = d->nx, ng = d->ng;
  int64_t S = 0;
  int maxN = 0;
  for (int b = 0; b < B; ++b) {
    S += horizons[b] + 1;
    maxN = std::max(maxN, horizons[b]);
  }
  h->S = S;
  h->maxN = maxN;
  const size_t nn = (size_t)n * n;
  const size_t blkI = h->ti ? (size_t)B : (size_t)S;  // block count for per-instance/per-stage data
  const size_t ts = h->tsz();
  ocp_status st = OCP_OK;
#define A_(ptr, bytes)                                  \
  do {                                                  \
    st = halloc(h, &(ptr), (bytes), count_only);        \
    if (st != OCP_OK) return st;                        \
  } while (0)
  A_(h->stage_off, sizeof(int64_t) * (B + 1));
  A_(h->order, sizeof(int32_t) * B);
  A_(h->D, sizeof(double) * nn * (h->ti ? 2 * (size_t)B : (size_t)S));
  if (d->model != OCP_MODEL_LTI) A_(h->E, sizeof(double) * nn * blkI);  // bicycle: the Lagrangian Hessian
  if (d->model != OCP_MODEL_LTI) A_(h->bd, sizeof(double) * nx * blkI);
  if (d->model != OCP_MODEL_LTI) A_(h->q, sizeof(double) * n * (size_t)S);
  A_(h->Am, sizeof(double) * nx * n * blkI);
  A_(h->Ap, sizeof(double) * nx * n * blkI);
  A_(h->G, sizeof(double) * ng * n * blkI);
  A_(h->lo, sizeof(double) * ng * blkI);
  A_(h->hi, sizeof(double) * ng * blkI);
  A_(h->xinit, sizeof(double) * nx * B);
  A_(h->soft, 16);
  if (h->mixed) {
    A_(h->AmT, ts * nx * n * blkI);
    A_(h->ApT, ts * nx * n * blkI);
    A_(h->GT, ts * ng * n * blkI);
    A_(h->loT, ts * ng * blkI);
    A_(h->hiT, ts * ng * blkI);
    A_(h->xinitT, ts * nx * B);
    if (d->model != OCP_MODEL_LTI) {
      A_(h->qT, ts * n * (size_t)S);
      A_(h->bdT, ts * nx * blkI);
    }
  }
  // factor and state carry one zero padding stage past the last instance;
  // the buffers the iteration streams carry STAGE_PAD more stages on both
  // sides (pointers are moved past the leading ones below)
  const size_t S1 = (size_t)S + 1;
  const size_t SP = S1 + 2 * (size_t)STAGE_PAD;
  A_(h->Linv64, sizeof(double) * nn * S1);
  A_(h->M64, sizeof(double) * nn * S1);
  if (h->mixed) A_(h->SubA, ts * nn * SP);  // packed Linv_t (FP32 iterations only)
  A_(h->SubB, ts * nn * SP);
  A_(h->ChF, ts * nn * SP);
  A_(h->ChB, ts * nn * SP);
  A_(h->SegT, ts * nn * 4 * (size_t)B);
  A_(h->SegU, ts * nn * 4 * (size_t)B);
  A_(h->SegX, ts * ROW * 8 * (size_t)B);
  A_(h->FacX, sizeof(double) * nn * FX_SLOTS * (size_t)B);
  {
    const int W = mw_waves_of(n);
    h->mw_cap = 0;
    if (!h->mw_off)
      for (int b = 0; b < B; ++b) h->mw_cap += horizons[b] >= mw_floor_n(W) ? 1 : 0;
    A_(h->mw_list, sizeof(int32_t) * (size_t)B);
    if (h->mw_cap > 0) A_(h->FacXmw, sizeof(double) * nn * fx_slots(4 * W) * (size_t)h->mw_cap);
  }
  A_(h->x, ts * ROW * SP);
  A_(h->v, ts * ROW * SP);
  A_(h->yf, ts * ROW * SP);
  A_(h->zg, ts * ROW * SP);
  A_(h->yg, ts * ROW * SP);
  A_(h->xi, ts * ROW * SP);
  A_(h->ypf, ts * ROW * (size_t)S);
  A_(h->ypg, ts * ROW * (size_t)S);
  A_(h->rho, sizeof(double) * B);
  A_(h->rprim, sizeof(double) * B);
  A_(h->rdual, sizeof(double) * B);
  A_(h->status, sizeof(int32_t) * B);
  A_(h->iters, sizeof(int32_t) * B);
  A_(h->nfact, sizeof(int32_t) * B);
  A_(h->need, sizeof(int32_t) * B);
  if (d->model == OCP_MODEL_BICYCLE) {
    A_(h->bike_ref, sizeof(double) * 4 * S);
    A_(h->bike_normal, sizeof(double) * 2 * S);
    A_(h->bike_x0, sizeof(double) * 4 * B);
    A_(h->bike_uinit, sizeof(double) * 2 * B);
    A_(h->xbar, sizeof(double) * ROW * S);
    A_(h->xibar, sizeof(double) * ROW * S);
    A_(h->yfbar, sizeof(double) * ROW * S);
    A_(h->ygbar, sizeof(double) * ROW * S);
    A_(h->mu, sizeof(double) * B);
    A_(h->kkt, sizeof(double) * 3 * B);
    A_(h->sqp_done, sizeof(int32_t) * B);
    A_(h->sqp_frozen, sizeof(int32_t) * B);
    size_t nch = (size_t)B;
    if (!h->carve) {
      nch = 0;
      for (int b = 0; b < B; ++b) nch += (size_t)(horizons[b] + LS_CHUNK) / LS_CHUNK;
      A_(h->ls_chunk_inst, sizeof(int32_t) * nch);
      A_(h->ls_chunk_t0, sizeof(int32_t) * nch);
      A_(h->ls_chunk_off, sizeof(int32_t) * (B + 1));
      A_(h->ls_alpha, sizeof(double) * B);
    }
    h->ls_nchunks = (int)nch;
    A_(h->ls_parts, sizeof(double) * LS_NF * nch);
  }
  A_(h->stage_inst, sizeof(int32_t) * S);
  A_(h->sc, sizeof(double) * 3 * ROW * B);
  A_(h->adj_rhog, sizeof(double) * ROW * S);
  A_(h->adj_ex, sizeof(double) * ROW * S);
  A_(h->adj_ey, sizeof(double) * ROW * S);
  A_(h->adj_eg, sizeof(double) * ROW * S);
  A_(h->adj_r, sizeof(double) * ROW * S);
  A_(h->adj_v, sizeof(double) * ROW * SP);
  A_(h->adj_P, sizeof(double) * nn * SP);
  A_(h->adj_K, sizeof(double) * nn * SP);
  A_(h->adj_Kb, sizeof(double) * nn * SP);
  A_(h->adj_rg, sizeof(double) * ROW * S);
  A_(h->adj_act, sizeof(int8_t) * ROW * S);
  A_(h->adj_dl, sizeof(double) * n * S);
#undef A_
  if (count_only) return OCP_OK;
  if (!h->mixed) {  // iteration-precision copies alias the FP64 data
    h->AmT = h->Am;
    h->ApT = h->Ap;
    h->GT = h->G;
    h->loT = h->lo;
    h->hiT = h->hi;
    h->xinitT = h->xinit;
    h->qT = h->q;
    h->bdT = h->bd;
  }
  if (h->carve) {
    // carved workspace: the caller clears it and lays out the stages on the
    // device (no host buffers); only the padding offsets are applied here
    const size_t tsz = h->tsz();
    void** padded[] = {&h->SubA, &h->SubB, &h->ChF, &h->ChB, &h->x, &h->v, &h->yf, &h->zg, &h->yg, &h->xi,
                       (void**)&h->adj_v, (void**)&h->adj_P, (void**)&h->adj_K, (void**)&h->adj_Kb};
    const size_t stage_bytes[] = {tsz * nn,  tsz * nn,  tsz * nn,  tsz * nn,  tsz * ROW,
                                  tsz * ROW, tsz * ROW, tsz * ROW, tsz * ROW, tsz * ROW,
                                  sizeof(double) * ROW, sizeof(double) * nn, sizeof(double) * nn,
                                  sizeof(double) * nn};
    for (int k = 0; k < 14; ++k)
      if (*padded[k]) *padded[k] = (char*)*padded[k] + stage_bytes[k] * STAGE_PAD;
    return OCP_OK;
  }
  h->horizons_host.assign(horizons, horizons + B);
  {
    const ocp_status ms = upload_mw_list(h);
    if (ms != OCP_OK) return ms;
  }
  if (h->mw_cap > 0 && h->mw_cap < B) {  // a batch that may launch both solve kernels
    if (hipStreamCreateWithFlags(&h->fork.aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->fork.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->fork.join, hipEventDisableTiming) != hipSuccess)
      return OCP_E_HIP;
  }
  // line-search chunks of the bicycle model (host -> device, once)
  if (h->ls_chunk_inst) {
    std::vector<int32_t> ci, ct, co((size_t)B + 1, 0);
    for (int b = 0; b < B; ++b) {
      co[(size_t)b] = (int32_t)ci.size();
      for (int t = 0; t <= horizons[b]; t += LS_CHUNK) {
        ci.push_back(b);
        ct.push_back(t);
      }
    }
    co[(size_t)B] = (int32_t)ci.size();
    if ((int)ci.size() != h->ls_nchunks ||
        hipMemcpy(h->ls_chunk_inst, ci.data(), sizeof(int32_t) * ci.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->ls_chunk_t0, ct.data(), sizeof(int32_t) * ct.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->ls_chunk_off, co.data(), sizeof(int32_t) * co.size(), hipMemcpyHostToDevice) != hipSuccess)
      return OCP_E_HIP;
  }
  // stage offsets and longest-first processing order (host -> device, once)
  std::vector<int64_t> off(B + 1, 0);
  for (int b = 0; b < B; ++b) off[b + 1] = off[b] + horizons[b] + 1;
  std::vector<int32_t> ord(B);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return horizons[a] > horizons[c]; });
  {
    std::vector<int32_t> si((size_t)S);
    for (int b = 0; b < B; ++b)
      for (int64_t k = off[b]; k < off[b + 1]; ++k) si[(size_t)k] = b;
    if (hipMemcpy(h->stage_inst, si.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice) != hipSuccess)
      return OCP_E_HIP;
  }
  if (hipMemcpy(h->stage_off, off.data(), sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->order, ord.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(h->soft, 0, 16) != hipSuccess || hipMemset(h->rho, 0, sizeof(double) * B) != hipSuccess)
    return OCP_E_HIP;
  // M_0 and the chain blocks of stage 0 (forward) and N (backward) of every
  // instance, and all padding, stay zero for the lifetime of the handle (the
  // factorisations never write them); state starts at zero
  {
    const size_t tsz = h->tsz();
    if (hipMemset(h->M64, 0, sizeof(double) * nn * S1) != hipSuccess) return OCP_E_HIP;
    void** padded[] = {&h->SubA, &h->SubB, &h->ChF, &h->ChB, &h->x, &h->v, &h->yf, &h->zg, &h->yg, &h->xi,
                       (void**)&h->adj_v, (void**)&h->adj_P, (void**)&h->adj_K, (void**)&h->adj_Kb};
    const size_t stage_bytes[] = {tsz * nn,  tsz * nn,  tsz * nn,  tsz * nn,  tsz * ROW,
                                  tsz * ROW, tsz * ROW, tsz * ROW, tsz * ROW, tsz * ROW,
                                  sizeof(double) * ROW, sizeof(double) * nn, sizeof(double) * nn,
                                  sizeof(double) * nn};
    for (int k = 0; k < 14; ++k) {
      if (!*padded[k]) continue;
      if (hipMemset(*padded[k], 0, stage_bytes[k] * SP) != hipSuccess) return OCP_E_HIP;
      *padded[k] = (char*)*padded[k] + stage_bytes[k] * STAGE_PAD;
    }
  }
  return OCP_OK;
}

template <typename T>
void convert(const double* src, void* dst, size_t len, hipStream_t st) {
  if (!src || !dst || len == 0 || (void*)src == dst) return;
  const int threads = 256;
  const size_t blocks = (len + threads - 1) / threads;
  hipLaunchKernelGGL(convert_kernel<T>, dim3((unsigned)blocks), dim3(threads), 0, st, src, (T*)dst, len);
}

// refresh the iteration-precision copies after the FP64 data changed
void refresh_copies(ocp_handle h, hipStream_t st) {
  if (!h->mixed) return;
  const size_t blkI = h->ti ? (size_t)h->B : (size_t)h->S;
  const int n = h->n, nx = h->d.nx, ng = h->d.ng;
  convert<float>(h->Am, h->AmT, (size_t)nx * n * blkI, st);
  convert<float>(h->Ap, h->ApT, (size_t)nx * n * blkI, st);
  convert<float>(h->G, h->GT, (size_t)ng * n * blkI, st);
  convert<float>(h->lo, h->loT, (size_t)ng * blkI, st);
  convert<float>(h->hi, h->hiT, (size_t)ng * blkI, st);
  convert<float>(h->xinit, h->xinitT, (size_t)nx * h->B, st);
  if (h->q && h->has_q) convert<float>(h->q, h->qT, (size_t)n * h->S, st);
  if (h->bd && h->has_bd) convert<float>(h->bd, h->bdT, (size_t)nx * blkI, st);
}

Layout make_layout(ocp_handle h) {
  Layout L{};
  L.B = h->B;
  L.nx = h->d.nx;
  L.nu = h->d.nu;
  L.ng = h->d.ng;
  L.n = h->n;
  L.stage_off = h->stage_off;
  L.order = h->order;
  L.ti = h->ti ? 1 : 0;
  L.D = h->D;
  L.E = h->has_E ? h->E : nullptr;
  L.q = h->has_q ? h->q : nullptr;
  L.Am = h->Am;
  L.Ap = h->Ap;
  L.bd = h->has_bd ? h->bd : nullptr;
  L.G = h->G;
  L.lo = h->lo;
  L.hi = h->hi;
  L.x_init = h->xinit;
  L.soft = h->soft;
  L.gamma2 = h->gamma2;
  L.gamma1 = h->gamma1;
  L.sc = h->scaled ? h->sc : nullptr;
  L.AmT = h->AmT;
  L.ApT = h->ApT;
  L.GT = h->GT;
  L.qT = h->has_q ? h->qT : nullptr;
  L.bdT = h->has_bd ? h->bdT : nullptr;
  L.loT = h->loT;
  L.hiT = h->hiT;
  L.xinitT = h->xinitT;
  L.Linv64 = h->Linv64;
  L.M64 = h->M64;
  L.SubA = h->SubA;
  L.SubB = h->SubB;
  L.ChF = h->ChF;
  L.ChB = h->ChB;
  L.SegT = h->SegT;
  L.SegU = h->SegU;
  L.SegX = h->SegX;
  L.FacX = h->FacX;
  L.mw_list = h->mw_list;
  L.n_mw = h->pcg ? 0 : h->n_mw;  // PCG updates run one wavefront per instance
  L.pcg = h->pcg;
  L.pcg_max_it = h->pcg_max_it;
  L.pcg_tol = h->pcg_tol;
  L.pcg_xt = h->pcg_xt;
  L.pcg_r = h->pcg_r;
  L.pcg_z = h->pcg_z;
  L.pcg_p = h->pcg_p;
  L.pcg_sp = h->pcg_sp;
  L.mw_min_n = h->mw_min_n;
  L.FacXmw = h->FacXmw;
  L.tail_list = h->tail_list;
  L.tail_count = h->tail_count;
  L.tail_flags = h->tail_flags;
  L.FacXtail = h->FacXtail;
  for (int k = 0; k < 16; ++k) {
    L.gsel[k] = h->gsel[k];
    L.ginv[k] = h->ginv[k];
  }
  L.x = h->x;
  L.v = h->v;
  L.yf = h->yf;
  L.zg = h->zg;
  L.yg = h->yg;
  L.xi = h->xi;
  L.ypf = h->ypf;
  L.ypg = h->ypg;
  L.rho = h->rho;
  L.status = h->status;
  L.iters = h->iters;
  L.nfact = h->nfact;
  L.rprim = h->rprim;
  L.rdual = h->rdual;
  L.init_blocks = (unsigned)((std::max<int64_t>(h->S * ROW, h->B) + 255) / 256);
  return L;
}

Settings make_settings(const ocp_settings* s, int warm) {
  Settings o{};
  o.sigma = s->sigma;
  o.rho0 = s->rho0;
  o.rho_f_scale = s->rho_f_scale;
  o.rho_min = s->rho_min;
  o.rho_max = s->rho_max;
  o.k_ratio = s->k_ratio;
  o.alpha = s->alpha;
  o.eps_abs = s->eps_abs;
  o.eps_rel = s->eps_rel;
  o.eps_pinf = s->eps_pinf;
  o.max_iter = s->max_admm;
  o.k_rho = s->k_rho;
  o.k_check = s->k_check;
  o.adapt_rho = s->adapt_rho;
  o.warm = warm;
  return o;
}

ocp_status check_settings(const ocp_settings* s) {
  if (!s) return OCP_E_ARG;
  if (!(s->sigma > 0) || !(s->rho0 > 0) || !(s->rho_f_scale > 0) || !(s->rho_min > 0) ||
      !(s->rho_max >= s->rho_min) || !(s->alpha > 0 && s->alpha < 2) || s->max_admm < 1 || s->k_check < 0 ||
      s->k_rho < 0 || !(s->eps_abs >= 0) || !(s->eps_rel >= 0) || !(s->eps_pinf >= 0))
    return OCP_E_ARG;
  return OCP_OK;
}

// padded state -> caller's FP64 array; on a rescaled QP times the factor
// `code` that maps the entry back to the original variables
template <typename T>
void unpad(ocp_handle h, const void* src, double* dst, int w, int code, hipStream_t st) {
  if (!dst || w == 0) return;
  const size_t len = (size_t)h->S * w;
  hipLaunchKernelGGL(unpad_kernel<T>, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, (const T*)src, dst,
                     h->S, w, h->stage_inst, h->scaled ? (const double*)h->sc : nullptr, code);
}

template <typename T>
void unpad_yf(ocp_handle h, const void* src, double* dst, hipStream_t st) {
  if (!dst) return;
  const size_t len = (size_t)h->S * h->d.nx;
  hipLaunchKernelGGL(unpad_yf_kernel<T>, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, (const T*)src, dst,
                     h->stage_off, h->stage_inst, h->S, h->d.nx, h->scaled ? (const double*)h->sc : nullptr);
}

// Rescale the loaded FP64 QP data in place by the handle's factors (Remark
// 4; the transform is listed in the header at ocp_set_scaling).
void apply_scaling(ocp_handle h, hipStream_t st) {
  if (!h->scaled) return;
  const int n = h->n, nx = h->d.nx, ng = h->d.ng, B = h->B;
  const int64_t S = h->S, blkI = h->ti ? (int64_t)B : S;
  const int per = h->ti ? 1 : 0;
  if (h->box_p >= 0.0)
    hipLaunchKernelGGL(box_scaling_kernel, dim3((B + 63) / 64), dim3(64), 0, st, B, n, ng, h->ti ? 1 : 0,
                       (const int64_t*)h->stage_off, (const double*)h->D, (const double*)h->G, (const double*)h->lo,
                       (const double*)h->hi, (const uint8_t*)h->soft, h->box_p, h->sc);
  auto run = [&](double* p, int64_t nblk, int R, int Cc, int per_, int rowf, int colf) {
    const int64_t len = nblk * R * Cc;
    if (!p || len == 0) return;
    hipLaunchKernelGGL(scale_blocks_kernel, dim3((unsigned)std::min<int64_t>((len + 255) / 256, 8192)), dim3(256), 0,
                       st, p, nblk, R, Cc, per_, h->stage_inst, (const double*)h->sc, rowf, colf);
  };
  run(h->D, h->ti ? 2 * (int64_t)B : S, n, n, h->ti ? 2 : 0, SF_CD, SF_D);
  if (h->has_E) run(h->E, blkI, n, n, per, SF_CD, SF_D);
  if (h->has_q) run(h->q, S, 1, n, 0, SF_C, SF_D);
  run(h->Am, blkI, nx, n, per, SF_INV_D, SF_D);
  run(h->Ap, blkI, nx, n, per, SF_INV_D, SF_D);
  if (h->has_bd) run(h->bd, blkI, 1, nx, per, SF_ONE, SF_INV_D);
  run(h->G, blkI, ng, n, per, SF_E, SF_D);
  run(h->lo, blkI, 1, ng, per, SF_ONE, SF_E);
  run(h->hi, blkI, 1, ng, per, SF_ONE, SF_E);
  run(h->xinit, B, 1, nx, 1, SF_ONE, SF_INV_D);
}

void drop_graph(ocp_handle h) {
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->graph_exec = nullptr;
  h->graph = nullptr;
}

ocp_status copy_out(ocp_handle h, const ocp_solution* o, hipStream_t st) {
  if (!o) return OCP_OK;
  const int64_t S = h->S;
  const int B = h->B;
  if (h->mixed) {
    unpad<float>(h, h->x, o->x, h->n, SF_D, st);
    unpad<float>(h, h->xi, o->xi, h->d.ng, SF_INV_E, st);
    unpad<float>(h, h->zg, o->z_g, h->d.ng, SF_INV_E, st);
    unpad_yf<float>(h, h->yf, o->y_f, st);
    unpad<float>(h, h->yg, o->y_g, h->d.ng, SF_E_OVER_C, st);
  } else {
    unpad<double>(h, h->x, o->x, h->n, SF_D, st);
    unpad<double>(h, h->xi, o->xi, h->d.ng, SF_INV_E, st);
    unpad<double>(h, h->zg, o->z_g, h->d.ng, SF_INV_E, st);
    unpad_yf<double>(h, h->yf, o->y_f, st);
    unpad<double>(h, h->yg, o->y_g, h->d.ng, SF_E_OVER_C, st);
  }
  if (h->d.model == OCP_MODEL_BICYCLE) {  // the SQP iterate is the solution (never rescaled)
    unpad<double>(h, h->xbar, o->x, h->n, SF_ONE, st);
    unpad<double>(h, h->xibar, o->xi, h->d.ng, SF_ONE, st);
    unpad_yf<double>(h, h->yfbar, o->y_f, st);
    unpad<double>(h, h->ygbar, o->y_g, h->d.ng, SF_ONE, st);
    if (o->sqp_kkt && hipMemcpyAsync(o->sqp_kkt, h->kkt, sizeof(double) * 3 * B, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return OCP_E_HIP;
    if (o->sqp_iters &&
        hipMemcpyAsync(o->sqp_iters, h->sqp_done, sizeof(int32_t) * B, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return OCP_E_HIP;
  }
  struct {
    void* dst;
    const void* src;
    size_t sz;
  } cp[] = {{o->status, h->status, sizeof(int32_t)}, {o->admm_iters, h->iters, sizeof(int32_t)},
            {o->n_factor, h->nfact, sizeof(int32_t)}, {o->r_prim, h->rprim, sizeof(double)},
            {o->r_dual, h->rdual, sizeof(double)},    {o->rho, h->rho, sizeof(double)}};
  for (auto& c : cp)
    if (c.dst && hipMemcpyAsync(c.dst, c.src, c.sz * B, hipMemcpyDeviceToDevice, st) != hipSuccess) return OCP_E_HIP;
  if (h->d.model != OCP_MODEL_BICYCLE && o->sqp_iters) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3((B + 255) / 256), dim3(256), 0, st, o->sqp_iters, B, 1);
  }
  return hip_ok(hipGetLastError());
}

void run_admm(ocp_handle h, const Settings& s_, hipStream_t st) {
  const Layout L = make_layout(h);
  Settings s = s_;
  s.seg_min_n = h->seg_min_n;
  s.seg_after = h->seg_after;
  s.tail_after = h->tail_after;
  const int ti = h->ti ? 1 : 0;
  const int var = (h->variant == VAR_LTI_BOX) ? VAR_LTI_BOX : (ti ? VAR_TI : VAR_TV);
  if (h->mixed)
    h->entry->p32()->solve[var](L, s, h->need, st, &h->prof, &h->fork);
  else
    h->entry->p64()->solve[var](L, s, h->need, st, &h->prof, &h->fork);
}

BikeArgs make_bike(ocp_handle h, const ocp_settings* s) {
  BikeArgs a{};
  a.ref = h->bike_ref;
  a.normal = h->bike_normal;
  a.x0 = h->bike_x0;
  a.stage_inst = h->stage_inst;
  a.dt = h->bike.dt;
  a.Lw = h->bike.wheelbase;
  a.a_b = h->bike.a_bound;
  a.d_b = h->bike.steer_bound;
  a.lat_b = h->bike.lat_bound;
  a.gamma1 = h->bike.gamma1;
  a.integ = h->bike.integrator;
  for (int k = 0; k < 4; ++k) {
    a.Qd[k] = h->bike.Qd[k];
    a.Qfd[k] = h->bike.Qfd[k];
  }
  a.Rd[0] = h->bike.Rd[0];
  a.Rd[1] = h->bike.Rd[1];
  a.Wd[0] = h->bike.Wd[0];
  a.Wd[1] = h->bike.Wd[1];
  a.rate = h->bike_rate ? 1 : 0;
  a.u_init = h->bike.u_init ? h->bike_uinit : nullptr;
  a.xbar = h->xbar;
  a.xibar = h->xibar;
  a.yfbar = h->yfbar;
  a.ygbar = h->ygbar;
  a.mu = h->mu;
  a.kkt = h->kkt;
  a.done = h->sqp_done;
  a.frozen = h->sqp_frozen;
  a.eps_c = s->eps_c;
  a.armijo_eta = s->armijo_eta;
  a.fixed = s->fixed_sqp;
  a.chunk_inst = h->ls_chunk_inst;
  a.chunk_t0 = h->ls_chunk_t0;
  a.chunk_off = h->ls_chunk_off;
  a.parts = h->ls_nchunks > h->B ? h->ls_parts : nullptr;
  a.alpha = h->ls_alpha;
  return a;
}

// Algorithm 1 on every instance: linearise at the iterate, solve the QP by
// ADMM warm-started from it, take the line-search step.
ocp_status bicycle_sqp(ocp_handle h, const ocp_settings* s, hipStream_t st) {
  if (s->max_sqp < 1 || !(s->eps_c > 0) || !(s->armijo_eta > 0 && s->armijo_eta < 1)) return OCP_E_ARG;
  const BikeArgs a = make_bike(h, s);
  const Layout L = make_layout(h);
  const int64_t S = h->S;
  const unsigned gs = (unsigned)((std::max<int64_t>(S, h->B) + 255) / 256);
  const unsigned gl = (unsigned)((S + LIN_BLOCK - 1) / LIN_BLOCK);
  Prof* pf = &h->prof;
  if (!(s->warm_start && h->solved))
    timed(pf, OCP_K_OTHER, st,
          [&] { hipLaunchKernelGGL(bike_init_kernel, dim3(gs), dim3(256), 0, st, L, a, s->rho0); });
  const Settings ad = make_settings(s, 1);
  for (int k = 0; k < s->max_sqp; ++k) {
    timed(pf, OCP_K_SQP, st, [&] {
      if (h->mixed)
        hipLaunchKernelGGL((a.integ ? bike_linearize_kernel<float, 1> : bike_linearize_kernel<float, 0>), dim3(gl),
                           dim3(LIN_BLOCK), 0, st, L, a);
      else
        hipLaunchKernelGGL((a.integ ? bike_linearize_kernel<double, 1> : bike_linearize_kernel<double, 0>), dim3(gl),
                           dim3(LIN_BLOCK), 0, st, L, a);
    });
    run_admm(h, ad, st);
    timed(pf, OCP_K_SQP, st, [&] {
      const int nch = h->ls_nchunks;
      if (!a.parts) {  // every horizon within one chunk: the line-search kernel sums itself
        if (h->mixed)
          hipLaunchKernelGGL((a.integ ? bike_linesearch_kernel<float, 1> : bike_linesearch_kernel<float, 0>),
                             dim3(h->B), dim3(64), 0, st, L, a);
        else
          hipLaunchKernelGGL((a.integ ? bike_linesearch_kernel<double, 1> : bike_linesearch_kernel<double, 0>),
                             dim3(h->B), dim3(64), 0, st, L, a);
      } else {  // merit parts per chunk, the decision per instance, then the step and the stopping maxima per chunk
        if (h->mixed) {
          hipLaunchKernelGGL((a.integ ? bike_merit_parts_kernel<float, 1> : bike_merit_parts_kernel<float, 0>),
                             dim3(nch), dim3(64), 0, st, L, a, nch);
          hipLaunchKernelGGL((a.integ ? bike_linesearch_kernel<float, 1> : bike_linesearch_kernel<float, 0>),
                             dim3(h->B), dim3(64), 0, st, L, a);
          hipLaunchKernelGGL(bike_step_parts_kernel<float>, dim3(nch), dim3(64), 0, st, L, a, nch);
          hipLaunchKernelGGL((a.integ ? bike_stop_parts_kernel<float, 1> : bike_stop_parts_kernel<float, 0>),
                             dim3(nch), dim3(64), 0, st, L, a, nch);
        } else {
          hipLaunchKernelGGL((a.integ ? bike_merit_parts_kernel<double, 1> : bike_merit_parts_kernel<double, 0>),
                             dim3(nch), dim3(64), 0, st, L, a, nch);
          hipLaunchKernelGGL((a.integ ? bike_linesearch_kernel<double, 1> : bike_linesearch_kernel<double, 0>),
                             dim3(h->B), dim3(64), 0, st, L, a);
          hipLaunchKernelGGL(bike_step_parts_kernel<double>, dim3(nch), dim3(64), 0, st, L, a, nch);
          hipLaunchKernelGGL((a.integ ? bike_stop_parts_kernel<double, 1> : bike_stop_parts_kernel<double, 0>),
                             dim3(nch), dim3(64), 0, st, L, a, nch);
        }
        hipLaunchKernelGGL(bike_stop_combine_kernel, dim3((h->B + 255) / 256), dim3(256), 0, st, L, a);
      }
    });
  }
  return hip_ok(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Workspace of the no-allocation entry point: a file-scope device array, one
// copy per GPU for the life of the process.  Host code reaches it only through
// the address hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
__device__ __align__(256) unsigned char scratch[OCP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's scratch (looked up once per device)
ocp_status scratch_base(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return OCP_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OCP_E_HIP;
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return OCP_OK;
}

}  // namespace

extern "C" {

void ocp_default_settings(ocp_settings* s) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  s->sigma = 1e-6;
  s->rho0 = 0.1;
  s->rho_f_scale = 1e3;
  s->rho_min = 1e-6;
  s->rho_max = 1e6;
  s->k_ratio = 5.0;
  s->alpha = 1.6;
  s->eps_abs = 1e-4;
  s->eps_rel = 1e-4;
  s->eps_c = 1e-4;
  s->armijo_eta = 0.4;
  s->eps_active = 1e-4;
  s->adj_sigma = 1e-9;
  s->adj_rho = 1e8;
  s->adj_tol = 1e-10;
  s->eps_pinf = 1e-4;
  s->max_admm = 1000;
  s->k_rho = 25;
  s->k_check = 25;
  s->adapt_rho = 1;
  s->warm_start = 0;
  s->max_sqp = 10;
  s->fixed_sqp = 1;
  s->refine_sweeps = 8;
  s->adj_mode = OCP_ADJ_LAST_QP;
}

const char* ocp_status_string(ocp_status st) {
  switch (st) {
    case OCP_E_SCRATCH: return "problem exceeds the no-allocation scratch (OCP_NOALLOC_SCRATCH_BYTES)";
    case OCP_OK: return "ok";
    case OCP_E_ARG: return "invalid argument";
    case OCP_E_SHAPE: return "unsupported or inconsistent shape";
    case OCP_E_HIP: return "HIP runtime error";
    case OCP_E_NOMEM: return "out of device memory";
    case OCP_E_ORDER: return "call order violated";
    case OCP_E_UNSUPPORTED: return "unsupported feature";
  }
  return "unknown status";
}

int32_t ocp_supported(int32_t nx, int32_t nu, int32_t ng) { return find_entry(nx, nu, ng) ? 1 : 0; }

ocp_status ocp_workspace_bytes(const ocp_dims* d, const int32_t* horizons, size_t* bytes) {
  if (!bytes) return OCP_E_ARG;
  ocp_status st = check_dims(d, horizons);
  if (st != OCP_OK) return st;
  ocp_handle_s tmp;
  st = build(&tmp, d, horizons, true);
  *bytes = tmp.bytes;
  return st;
}

ocp_status ocp_create(const ocp_dims* d, const int32_t* horizons, ocp_handle* out) {
  if (!out) return OCP_E_ARG;
  *out = nullptr;
  ocp_status st = check_dims(d, horizons);
  if (st != OCP_OK) return st;
  ocp_handle h = new (std::nothrow) ocp_handle_s();
  if (!h) return OCP_E_NOMEM;
  st = build(h, d, horizons, false);
  if (st != OCP_OK) {
    free_all(h);
    delete h;
    return st;
  }
  *out = h;
  return OCP_OK;
}

ocp_status ocp_destroy(ocp_handle h) {
  if (!h) return OCP_OK;
  (void)hipDeviceSynchronize();
  h->prof.release();
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->fork.join) (void)hipEventDestroy(h->fork.join);
  if (h->fork.fork) (void)hipEventDestroy(h->fork.fork);
  if (h->fork.aux) (void)hipStreamDestroy(h->fork.aux);
  free_all(h);
  delete h;
  return OCP_OK;
}

ocp_status ocp_set_lti(ocp_handle h, const ocp_lti* p, void* stream) {
  if (!h || !p || !p->A || !p->Bm || !p->Qd || !p->Rd || !p->Qfd || !p->lo || !p->hi || !p->x0) return OCP_E_ARG;
  if (h->d.model != OCP_MODEL_LTI) return OCP_E_ORDER;
  if (h->d.ng > 0 && !p->G) return OCP_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int B = h->B;
  hipLaunchKernelGGL(lti_expand_kernel, dim3((B + 63) / 64), dim3(64), 0, st, B, h->d.nx, h->d.nu, h->d.ng, p->A,
                     p->Bm, p->Qd, p->Rd, p->Qfd, p->G, p->lo, p->hi, p->x0, h->D, h->Am, h->Ap, h->G, h->lo, h->hi,
                     h->xinit);
  h->has_E = h->has_q = h->has_bd = false;
  // a G whose rows each select one distinct variable takes the box-bound kernel variant
  {
    const int ng = h->d.ng, n = h->n;
    double Gh[ROW * ROW] = {0.0};  // ng, n <= ROW (checked at creation)
    if (ng > 0 && (hipMemcpyAsync(Gh, p->G, sizeof(double) * ng * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
                   hipStreamSynchronize(st) != hipSuccess))
      return OCP_E_HIP;
    bool sel = true;
    int8_t gs[16], gi[16];
    for (int k = 0; k < 16; ++k) gs[k] = 0, gi[k] = -1;
    for (int r = 0; r < ng && sel; ++r) {
      int hit = -1, cnt = 0;
      for (int c = 0; c < n; ++c) {
        if (Gh[(size_t)r * n + c] == 1.0) hit = c, ++cnt;
        else if (Gh[(size_t)r * n + c] != 0.0) cnt = 99;
      }
      if (cnt != 1 || gi[hit] != -1) sel = false;
      else gs[r] = (int8_t)hit, gi[hit] = (int8_t)r;
    }
    h->variant = sel ? VAR_LTI_BOX : VAR_TI;
    std::memcpy(h->gsel, gs, 16);
    std::memcpy(h->ginv, gi, 16);
  }
  std::memset(h->soft_host, 0, sizeof(h->soft_host));
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, (uint64_t*)h->soft, (size_t)2);
  apply_scaling(h, st);
  refresh_copies(h, st);
  h->data_set = true;
  h->solved = false;
  return hip_ok(hipGetLastError());
}

ocp_status ocp_set_qp(ocp_handle h, const ocp_qp* p, void* stream) {
  if (!h || !p || !p->D || !p->Am || !p->Ap || !p->x_init) return OCP_E_ARG;
  if (h->d.model != OCP_MODEL_QP) return OCP_E_ORDER;
  if (h->d.ng > 0 && (!p->G || !p->lo || !p->hi)) return OCP_E_ARG;
  if (!(p->gamma2 > 0) || !(p->gamma1 > 0)) return OCP_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const size_t nn = (size_t)h->n * h->n;
  const size_t blkI = h->ti ? (size_t)h->B : (size_t)h->S;
  const int nx = h->d.nx, ng = h->d.ng, n = h->n;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) == hipSuccess;
  };
  bool ok = cp(h->D, p->D, sizeof(double) * nn * (h->ti ? 2 * (size_t)h->B : (size_t)h->S)) &&
            cp(h->Am, p->Am, sizeof(double) * nx * n * blkI) && cp(h->Ap, p->Ap, sizeof(double) * nx * n * blkI) &&
            cp(h->xinit, p->x_init, sizeof(double) * nx * h->B);
  if (ng > 0)
    ok = ok && cp(h->G, p->G, sizeof(double) * ng * n * blkI) && cp(h->lo, p->lo, sizeof(double) * ng * blkI) &&
         cp(h->hi, p->hi, sizeof(double) * ng * blkI);
  h->has_E = p->E != nullptr;
  h->has_q = p->q != nullptr;
  h->has_bd = p->b != nullptr;
  if (p->E) ok = ok && cp(h->E, p->E, sizeof(double) * nn * blkI);
  if (p->q) ok = ok && cp(h->q, p->q, sizeof(double) * n * (size_t)h->S);
  if (p->b) ok = ok && cp(h->bd, p->b, sizeof(double) * nx * blkI);
  std::memset(h->soft_host, 0, sizeof(h->soft_host));
  if (p->soft) {
    ok = ok && cp(h->soft, p->soft, (size_t)ng) &&
         hipMemcpyAsync(h->soft_host, p->soft, (size_t)ng, hipMemcpyDeviceToHost, st) == hipSuccess &&
         hipStreamSynchronize(st) == hipSuccess;
    for (int r = 0; r < ng && ok; ++r)
      if (h->soft_host[r] > OCP_ROW_L1) return OCP_E_ARG;
  } else {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, (uint64_t*)h->soft, (size_t)2);
  }
  if (!ok) return OCP_E_HIP;
  if (!h->ti) {
    hipLaunchKernelGGL(zero_last_stage_kernel, dim3(h->B), dim3(64), 0, st, h->Am, h->stage_off, h->B, nx * n);
    hipLaunchKernelGGL(zero_last_stage_kernel, dim3(h->B), dim3(64), 0, st, h->Ap, h->stage_off, h->B, nx * n);
    hipLaunchKernelGGL(zero_last_stage_kernel, dim3(h->B), dim3(64), 0, st, h->bd, h->stage_off, h->B, nx);
    if (p->E) hipLaunchKernelGGL(zero_last_stage_kernel, dim3(h->B), dim3(64), 0, st, h->E, h->stage_off, h->B, n * n);
  }
  h->gamma2 = p->gamma2;
  h->gamma1 = p->gamma1;
  h->variant = h->ti ? VAR_TI : VAR_TV;
  if (h->scaled)
    for (int r = 0; r < ng; ++r)
      if (h->soft_host[r] != OCP_ROW_HARD) return OCP_E_UNSUPPORTED;  // soft rows are not rescaled
  apply_scaling(h, st);
  refresh_copies(h, st);
  h->data_set = true;
  h->solved = false;
  return hip_ok(hipGetLastError());
}

ocp_status ocp_set_bicycle(ocp_handle h, const ocp_bicycle* p, void* stream) {
  if (!h || !p || !p->ref || !p->normal || !p->x0) return OCP_E_ARG;
  if (h->d.model != OCP_MODEL_BICYCLE) return OCP_E_ORDER;
  if (!(p->dt > 0) || !(p->wheelbase > 0) || !(p->gamma1 > 0) || !(p->a_bound > 0) || !(p->steer_bound > 0) ||
      !(p->lat_bound > 0) || (p->integrator != OCP_INTEG_MIDPOINT && p->integrator != OCP_INTEG_TRAPEZOID) ||
      !(p->Wd[0] >= 0) || !(p->Wd[1] >= 0) || !std::isfinite(p->Wd[0]) || !std::isfinite(p->Wd[1]))
    return OCP_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t S = h->S;
  if (hipMemcpyAsync(h->bike_ref, p->ref, sizeof(double) * 4 * S, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h->bike_normal, p->normal, sizeof(double) * 2 * S, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h->bike_x0, p->x0, sizeof(double) * 4 * h->B, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return OCP_E_HIP;
  if (p->u_init &&
      hipMemcpyAsync(h->bike_uinit, p->u_init, sizeof(double) * 2 * h->B, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return OCP_E_HIP;
  h->bike = *p;
  h->variant = VAR_TV;
  h->gamma1 = p->gamma1;
  h->gamma2 = 1.0;
  h->bike_rate = p->Wd[0] != 0.0 || p->Wd[1] != 0.0;
  h->has_E = h->bike_rate;
  h->has_q = true;
  h->has_bd = true;
  const uint8_t kinds[16] = {OCP_ROW_HARD, OCP_ROW_HARD, OCP_ROW_L1};
  std::memcpy(h->soft_host, kinds, sizeof(kinds));
  if (hipMemcpyAsync(h->soft, kinds, 16, hipMemcpyHostToDevice, st) != hipSuccess) return OCP_E_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return OCP_E_HIP;  // `kinds` is a host stack array
  h->data_set = true;
  h->solved = false;
  return OCP_OK;
}

ocp_status ocp_solve(ocp_handle h, const ocp_settings* s, const ocp_solution* out, void* stream) {
  if (!h) return OCP_E_ARG;
  ocp_status st = check_settings(s);
  if (st != OCP_OK) return st;
  if (!h->data_set) return OCP_E_ORDER;
  hipStream_t stream_ = (hipStream_t)stream;
  if (h->d.model == OCP_MODEL_BICYCLE) {
    st = bicycle_sqp(h, s, stream_);
    if (st != OCP_OK) return st;
  } else {
    const int warm = (s->warm_start && h->solved) ? 1 : 0;
    run_admm(h, make_settings(s, warm), stream_);
    if (hipGetLastError() != hipSuccess) return OCP_E_HIP;
  }
  h->solved = true;
  return copy_out(h, out, stream_);
}

ocp_status ocp_get_solution(ocp_handle h, const ocp_solution* out, void* stream) {
  if (!h || !out) return OCP_E_ARG;
  if (!h->solved) return OCP_E_ORDER;
  return copy_out(h, out, (hipStream_t)stream);
}

ocp_status ocp_adjoint(ocp_handle h, const ocp_settings* s, const double* dL_dx, const double* dL_dxi,
                       const ocp_qp_grads* out, void* stream) {
  if (!h || !s || !dL_dx || !out) return OCP_E_ARG;
  if (!h->solved) return OCP_E_ORDER;
  if (!(s->adj_sigma > 0) || !(s->adj_rho > 0) || !(s->eps_active > 0) || !(s->adj_tol > 0) ||
      s->refine_sweeps < 1 || s->adj_mode < OCP_ADJ_LAST_QP || s->adj_mode > OCP_ADJ_SQP_EXACT)
    return OCP_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const bool at_iterate = h->d.model == OCP_MODEL_BICYCLE && s->adj_mode != OCP_ADJ_LAST_QP;
  if (at_iterate) {
    // differentiate the SQP solution: the QP convexified at the iterate, its
    // state set to the iterate, and for OCP_ADJ_SQP_EXACT the Hessian of the
    // Lagrangian in D_t, E_t
    const BikeArgs ba = make_bike(h, s);
    const Layout L0 = make_layout(h);
    const unsigned gs = (unsigned)((std::max<int64_t>(h->S, h->B) + 255) / 256);
    const unsigned gl = (unsigned)((h->S + LIN_BLOCK - 1) / LIN_BLOCK);
    const int integ = ba.integ;
    timed(&h->prof, OCP_K_SQP, st, [&] {
      if (h->mixed)
        hipLaunchKernelGGL((integ ? bike_linearize_kernel<float, 1> : bike_linearize_kernel<float, 0>), dim3(gl),
                           dim3(LIN_BLOCK), 0, st, L0, ba);
      else
        hipLaunchKernelGGL((integ ? bike_linearize_kernel<double, 1> : bike_linearize_kernel<double, 0>), dim3(gl),
                           dim3(LIN_BLOCK), 0, st, L0, ba);
      const unsigned gv = (unsigned)((h->S * ROW + 255) / 256);
      if (h->mixed)
        hipLaunchKernelGGL(iterate_slacks_kernel<float>, dim3(gv), dim3(256), 0, st, (const double*)h->xibar,
                           (float*)h->xi, h->S);
      else
        hipLaunchKernelGGL(iterate_slacks_kernel<double>, dim3(gv), dim3(256), 0, st, (const double*)h->xibar,
                           (double*)h->xi, h->S);
      if (s->adj_mode == OCP_ADJ_SQP_EXACT) {
        Layout LE = L0;
        LE.E = h->E;
        hipLaunchKernelGGL((integ ? bike_hessian_kernel<1> : bike_hessian_kernel<0>), dim3(gs), dim3(256), 0, st,
                           LE, ba);
      }
    });
    h->has_E = h->bike_rate || s->adj_mode == OCP_ADJ_SQP_EXACT;
  }
  AdjArgs a{};
  a.dLdx = dL_dx;
  a.dLdxi = dL_dxi;
  a.dl = h->adj_dl;
  a.sigma_b = s->adj_sigma;
  a.rho_b = s->adj_rho;
  a.eps_active = s->eps_active;
  a.sweeps = s->refine_sweeps;
  a.chunk_min_n = h->seg_min_n;
  a.w = h->adj_rhog;
  a.ex = h->adj_ex;
  a.ef = h->adj_ey;
  a.eg = h->adj_eg;
  a.rf = h->adj_r;
  a.rg = h->adj_rg;
  a.v = h->adj_v;
  a.act = h->adj_act;
  a.P = h->adj_P;
  a.K = h->adj_K;
  a.Kb = h->adj_Kb;
  a.d_q = out->d_q;
  a.d_Ddiag = out->d_Ddiag;
  a.d_x_init = out->d_x_init;
  a.d_gamma2 = out->d_gamma2;
  a.d_lo = out->d_lo;
  a.d_hi = out->d_hi;
  a.eta_x = out->eta_x;
  a.active = out->active;
  a.eta_f = out->eta_f;
  a.eta_g = out->eta_g;
  a.adj_resid = out->adj_resid;
  a.adj_status = out->adj_status;
  a.eta_xi = out->eta_xi;
  a.d_gamma1 = out->d_gamma1;
  a.adj_tol = s->adj_tol;
  const Layout L = make_layout(h);
  const int var = (h->variant == VAR_LTI_BOX) ? VAR_LTI_BOX : (h->ti ? VAR_TI : VAR_TV);
  if (h->mixed)
    h->entry->p32()->adj[var](L, a, st, &h->prof, &h->fork);
  else
    h->entry->p64()->adj[var](L, a, st, &h->prof, &h->fork);
  if (at_iterate) h->has_E = h->bike_rate;  // the SQP's own QPs: cross-stage blocks from a rate cost only
  return hip_ok(hipGetLastError());
}

ocp_status ocp_set_iterate(ocp_handle h, const double* x, const double* xi, const double* y_f, const double* y_g,
                           void* stream) {
  if (!h || !x || !xi || !y_f || !y_g) return OCP_E_ARG;
  if (h->d.model != OCP_MODEL_BICYCLE) return OCP_E_UNSUPPORTED;
  if (!h->data_set) return OCP_E_ORDER;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(load_iterate_kernel, dim3((unsigned)((h->S * ROW + 255) / 256)), dim3(256), 0, st, x, xi, y_f,
                     y_g, (const int64_t*)h->stage_off, (const int32_t*)h->stage_inst, h->S, h->n, h->d.nx, h->d.ng,
                     h->xbar, h->xibar, h->yfbar, h->ygbar);
  h->solved = true;  // the adjoint may differentiate at this iterate
  return hip_ok(hipGetLastError());
}

ocp_status ocp_profile(ocp_handle h, int32_t enable) {
  if (!h) return OCP_E_ARG;
  h->prof.on = enable != 0;
  return OCP_OK;
}

ocp_status ocp_profile_read(ocp_handle h, ocp_kernel_times* out) {
  if (!h || !out) return OCP_E_ARG;
  if (h->prof.collect() != hipSuccess) return OCP_E_HIP;
  for (int c = 0; c < OCP_K_COUNT; ++c) {
    out->ms[c] = h->prof.ms[c];
    out->launches[c] = h->prof.launches[c];
    h->prof.ms[c] = 0.0;
    h->prof.launches[c] = 0;
  }
  return OCP_OK;
}

ocp_status ocp_graph_capture(ocp_handle h, const ocp_settings* s, const ocp_solution* out, const double* dL_dx,
                             const double* dL_dxi, const ocp_qp_grads* grads, void* stream) {
  if (!h || !s || !stream) return OCP_E_ARG;
  if ((dL_dx == nullptr) != (grads == nullptr)) return OCP_E_ARG;
  ocp_status st = check_settings(s);
  if (st != OCP_OK) return st;
  if (!h->data_set) return OCP_E_ORDER;
  hipStream_t cs = (hipStream_t)stream;
  if (h->graph_exec) {
    (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
  }
  if (h->graph) {
    (void)hipGraphDestroy(h->graph);
    h->graph = nullptr;
  }
  const bool prof_on = h->prof.on;
  h->prof.on = false;  // no event records inside the graph
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    h->prof.on = prof_on;
    return OCP_E_HIP;
  }
  st = ocp_solve(h, s, out, stream);
  if (st == OCP_OK && dL_dx) st = ocp_adjoint(h, s, dL_dx, dL_dxi, grads, stream);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &g);
  h->prof.on = prof_on;
  if (st != OCP_OK || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return st != OCP_OK ? st : OCP_E_HIP;
  }
  if (hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    h->graph_exec = nullptr;
    return OCP_E_HIP;
  }
  h->graph = g;
  return OCP_OK;
}

ocp_status ocp_graph_launch(ocp_handle h, void* stream) {
  if (!h) return OCP_E_ARG;
  if (!h->graph_exec) return OCP_E_ORDER;
  if (hipGraphLaunch(h->graph_exec, (hipStream_t)stream) != hipSuccess) return OCP_E_HIP;
  h->solved = true;
  return OCP_OK;
}

ocp_status ocp_set_linsolve(ocp_handle h, int32_t mode, int32_t max_iter, double tol) {
  if (!h || (mode != OCP_LINSOLVE_DIRECT && mode != OCP_LINSOLVE_PCG) || max_iter < 1 || !(tol >= 0.0) ||
      !std::isfinite(tol))
    return OCP_E_ARG;
  if (h->carve) return OCP_E_UNSUPPORTED;
  drop_graph(h);  // a captured graph keeps the solver it was recorded with
  if (mode == OCP_LINSOLVE_PCG && !h->pcg_xt) {
    // five padded stage vectors and, for FP64 iterations, the preconditioner blocks
    const size_t ts = h->tsz(), nn = (size_t)h->n * h->n;
    const size_t SP = (size_t)h->S + 1 + 2 * (size_t)STAGE_PAD;
    void** vec[] = {&h->pcg_xt, &h->pcg_r, &h->pcg_z, &h->pcg_p, &h->pcg_sp};
    for (void** v : vec) {
      ocp_status st = halloc(h, v, ts * ROW * SP, false);
      if (st != OCP_OK) return st;
      if (hipMemset(*v, 0, ts * ROW * SP) != hipSuccess) return OCP_E_HIP;
      *v = (char*)*v + ts * ROW * STAGE_PAD;
    }
    if (!h->SubA) {
      ocp_status st = halloc(h, &h->SubA, ts * nn * SP, false);
      if (st != OCP_OK) return st;
      if (hipMemset(h->SubA, 0, ts * nn * SP) != hipSuccess) return OCP_E_HIP;
      h->SubA = (char*)h->SubA + ts * nn * STAGE_PAD;
    }
  }
  h->pcg = mode == OCP_LINSOLVE_PCG ? 1 : 0;
  h->pcg_max_it = max_iter;
  h->pcg_tol = tol;
  return OCP_OK;
}

ocp_status ocp_set_multiwave(ocp_handle h, int32_t mw_min_n) {
  if (!h) return OCP_E_ARG;
  const int floor_n = mw_floor_n(mw_waves_of(h->n));
  if (mw_min_n > 0 && mw_min_n < floor_n) return OCP_E_ARG;
  drop_graph(h);  // a captured graph keeps the launch shape it was recorded with
  h->mw_min_n = mw_min_n > 0 ? mw_min_n : 0;
  return upload_mw_list(h);
}

ocp_status ocp_set_tail_workgroup(ocp_handle h, int32_t iteration) {
  if (!h || iteration < 0) return OCP_E_ARG;
  if (iteration > 0 && (!h->mixed || h->carve)) return OCP_E_UNSUPPORTED;
  drop_graph(h);  // a captured graph keeps the launch shape it was recorded with
  if (iteration > 0 && !h->tail_count) {
    const size_t B = (size_t)h->B, nn = (size_t)h->n * h->n;
    ocp_status st = halloc(h, &h->tail_list, sizeof(int32_t) * B, false);
    if (st == OCP_OK) st = halloc(h, &h->tail_flags, sizeof(int32_t) * B, false);
    if (st == OCP_OK) st = halloc(h, &h->FacXtail, sizeof(double) * nn * fx_slots(4 * TAIL_W) * B, false);
    int32_t* cnt = nullptr;
    if (st == OCP_OK) st = halloc(h, &cnt, sizeof(int32_t), false);
    if (st != OCP_OK) return st;
    if (hipMemset(cnt, 0, sizeof(int32_t)) != hipSuccess) return OCP_E_HIP;
    h->tail_count = cnt;  // set last: a handle with a count has every tail buffer
  }
  h->tail_after = iteration;
  return OCP_OK;
}

ocp_status ocp_set_segmented(ocp_handle h, int32_t seg_min_n) {
  if (!h) return OCP_E_ARG;
  if (h->graph_exec) {  // a captured graph keeps the launch shape it was recorded with
    (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
  }
  if (h->graph) {
    (void)hipGraphDestroy(h->graph);
    h->graph = nullptr;
  }
  h->seg_min_n = std::max<int32_t>(seg_min_n, SEG_FLOOR_N);
  return OCP_OK;
}

ocp_status ocp_set_segmented_after(ocp_handle h, int32_t iteration) {
  if (!h || iteration < 0) return OCP_E_ARG;
  drop_graph(h);  // a captured graph keeps the launch shape it was recorded with
  h->seg_after = iteration;
  return OCP_OK;
}

ocp_status ocp_set_scaling(ocp_handle h, const double* d, const double* e_g, const double* c, void* stream) {
  if (!h) return OCP_E_ARG;
  drop_graph(h);  // a captured graph keeps the data layout it was recorded with
  h->data_set = false;
  h->solved = false;
  h->box_p = -1.0;
  if (!d) {
    h->scaled = false;
    return OCP_OK;
  }
  if ((h->d.ng > 0 && !e_g) || !c) return OCP_E_ARG;
  if (h->d.model == OCP_MODEL_BICYCLE) return OCP_E_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const int B = h->B, n = h->n, ng = h->d.ng;
  hipLaunchKernelGGL(pack_scaling_kernel, dim3((unsigned)std::min<int64_t>(((int64_t)B * 3 * ROW + 255) / 256, 4096)),
                     dim3(256), 0, st, d, ng > 0 ? e_g : d, c, B, n, ng, h->sc);
  // the factors must be positive and finite
  std::vector<double> hs((size_t)B * 3 * ROW);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(hs.data(), h->sc, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return OCP_E_HIP;
  for (double v : hs)
    if (!(v > 0.0) || !std::isfinite(v)) return OCP_E_ARG;
  h->scaled = true;
  return OCP_OK;
}

ocp_status ocp_set_scaling_box(ocp_handle h, double p) {
  if (!h || !(p >= 0.0) || !std::isfinite(p)) return OCP_E_ARG;
  if (h->d.model == OCP_MODEL_BICYCLE) return OCP_E_UNSUPPORTED;
  drop_graph(h);
  h->data_set = false;
  h->solved = false;
  h->scaled = true;
  h->box_p = p;
  return OCP_OK;
}

ocp_status ocp_autotune(ocp_handle h, const ocp_settings* s, int32_t reps, void* stream, int32_t* seg_min_n,
                        int32_t* seg_after, int32_t* tail_after) {
  if (!h || !s || reps < 1) return OCP_E_ARG;
  ocp_status st = check_settings(s);
  if (st != OCP_OK) return st;
  if (!h->data_set) return OCP_E_ORDER;
  hipStream_t stream_ = (hipStream_t)stream;
  ocp_settings cold = *s;
  cold.warm_start = 0;
  // (segmented from horizon, every running instance segmented from
  // iteration, continuation on two-wavefront workgroups from iteration);
  // the last three only with FP32 iterations
  constexpr int NC = 9;
  const int32_t cand[NC][3] = {{SEG_FLOOR_N, INT32_MAX, 0}, {SEG_MIN_N, INT32_MAX, 0}, {INT32_MAX, INT32_MAX, 0},
                               {SEG_MIN_N, 150, 0},         {SEG_MIN_N, 300, 0},       {SEG_MIN_N, 500, 0},
                               {SEG_MIN_N, INT32_MAX, 200}, {SEG_MIN_N, INT32_MAX, 300}, {SEG_MIN_N, 150, 200}};
  const int nc = h->mixed && !h->carve ? NC : 6;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return OCP_E_HIP;
  }
  const bool prof_on = h->prof.on;
  h->prof.on = false;
  float best = INFINITY;
  int32_t pick = h->seg_min_n, pick_after = h->seg_after, pick_tail = h->tail_after;
  for (int c = 0; c < nc && st == OCP_OK; ++c) {
    h->seg_min_n = cand[c][0];
    h->seg_after = cand[c][1];
    if (cand[c][2] > 0 || h->tail_after > 0) st = ocp_set_tail_workgroup(h, cand[c][2]);
    if (st != OCP_OK) break;
    st = ocp_solve(h, &cold, nullptr, stream);  // warm-up (and first touch of the transfer blocks)
    if (st != OCP_OK) break;
    if (hipEventRecord(e0, stream_) != hipSuccess) st = OCP_E_HIP;
    for (int r = 0; r < reps && st == OCP_OK; ++r) st = ocp_solve(h, &cold, nullptr, stream);
    float ms = 0.f;
    if (st == OCP_OK && (hipEventRecord(e1, stream_) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = OCP_E_HIP;
    if (st == OCP_OK && ms < best) best = ms, pick = cand[c][0], pick_after = cand[c][1], pick_tail = cand[c][2];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->prof.on = prof_on;
  if (st != OCP_OK) return st;
  ocp_status r = ocp_set_segmented(h, pick);
  if (r == OCP_OK) r = ocp_set_segmented_after(h, pick_after);
  if (r == OCP_OK) r = ocp_set_tail_workgroup(h, pick_tail);
  if (seg_min_n) *seg_min_n = h->seg_min_n;
  if (seg_after) *seg_after = h->seg_after;
  if (tail_after) *tail_after = h->tail_after;
  return r;
}

ocp_status ocp_solve_noalloc(const ocp_dims* d, const int32_t* horizons, const void* problem, const ocp_settings* s,
                             const ocp_solution* out, void* stream) {
  ocp_status st = check_dims(d, horizons);
  if (st != OCP_OK) return st;
  if (!problem) return OCP_E_ARG;
  st = check_settings(s);
  if (st != OCP_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  // host bookkeeping lives on the stack for this call (its vectors stay empty)
  ocp_handle_s h;
  h.mw_off = true;  // one wavefront per instance: no per-workgroup exchange blocks in the scratch
  st = build(&h, d, horizons, true);
  if (st != OCP_OK) return st;
  const size_t ws = h.bytes;
  const size_t hz_bytes = ((size_t)d->batch * sizeof(int32_t) + 255) & ~size_t(255);
  if (ws + hz_bytes > (size_t)OCP_NOALLOC_SCRATCH_BYTES) return OCP_E_SCRATCH;
  char* base = nullptr;
  st = scratch_base(&base);
  if (st != OCP_OK) return st;
  h = ocp_handle_s();
  h.carve = base;
  h.mw_off = true;
  st = build(&h, d, horizons, false);
  if (st != OCP_OK) return st;
  // the scratch keeps the previous call's contents: clear the workspace (the
  // zero padding stages and blocks the factorisations never write), then lay
  // out the stages from a device copy of the horizons
  int32_t* hz_dev = (int32_t*)(base + ws);
  const size_t words = ws / sizeof(uint64_t);
  hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)std::min<size_t>((words + 255) / 256, 4096)), dim3(256), 0, hs,
                     (uint64_t*)base, words);
  if (hipMemcpyAsync(hz_dev, horizons, sizeof(int32_t) * d->batch, hipMemcpyHostToDevice, hs) != hipSuccess)
    return OCP_E_HIP;
  hipLaunchKernelGGL(stage_layout_kernel, dim3(1), dim3(1024), 0, hs, hz_dev, d->batch, h.stage_off, h.order,
                     h.stage_inst);
  // the caller's horizons array may be released once this returns
  if (hipStreamSynchronize(hs) != hipSuccess || hipGetLastError() != hipSuccess) return OCP_E_HIP;
  switch (d->model) {
    case OCP_MODEL_LTI: st = ocp_set_lti(&h, (const ocp_lti*)problem, stream); break;
    case OCP_MODEL_QP: st = ocp_set_qp(&h, (const ocp_qp*)problem, stream); break;
    default: st = ocp_set_bicycle(&h, (const ocp_bicycle*)problem, stream); break;
  }
  if (st != OCP_OK) return st;
  ocp_settings cold = *s;
  cold.warm_start = 0;
  return ocp_solve(&h, &cold, out, stream);
}

}  // extern "C"
