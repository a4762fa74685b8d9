// C-ABI entry points: argument checks, device/stream plumbing, dispatch to
// the kernel launchers.
#include <string>

#include "plan.h"

using namespace mch;

// Replays the captured launch sequence of `g` when the arguments and stream
// match the captured ones; otherwise captures `issue` afresh. The legacy
// default stream cannot be captured, so calls on it (and profiled calls)
// run eagerly.
// The key holds every device pointer the captured kernels read or write,
// including those a call takes from the plan (the forward's label array).
template <typename F>
static int run_graph(mch_plan* p, mch_plan::Graph& g, const void* k0, const void* k1, const void* k2,
                     const void* k3, hipStream_t s, F issue) {
  if (!p->use_graphs || p->profiling || s == nullptr) return issue();
  if (g.exec && g.stream == s && g.key[0] == k0 && g.key[1] == k1 && g.key[2] == k2 && g.key[3] == k3)
    return hip_check(hipGraphLaunch(g.exec, s), "hipGraphLaunch");
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
  int rc = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
  if (rc) return rc;
  const int rc_issue = issue();
  hipGraph_t graph = nullptr;
  rc = hip_check(hipStreamEndCapture(s, &graph), "hipStreamEndCapture");
  if (rc_issue || rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc_issue ? rc_issue : rc;
  }
  rc = hip_check(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  if (rc) {
    (void)hipGraphDestroy(graph);
    return rc;
  }
  g.graph = graph;
  g.stream = s;
  g.key[0] = k0;
  g.key[1] = k1;
  g.key[2] = k2;
  g.key[3] = k3;
  return hip_check(hipGraphLaunch(g.exec, s), "hipGraphLaunch");
}

static int enter(mch_plan* p, void* stream, hipStream_t* s) {
  if (!p) return set_error(MCH_EINVAL, "null plan");
  int rc = hip_check(hipSetDevice(p->device), "hipSetDevice");
  if (rc) return rc;
  *s = reinterpret_cast<hipStream_t>(stream);
  return MCH_OK;
}

extern "C" int mch_solve_cells(mch_plan* p, const double* kappa, const uint8_t* label, void* stream) {
  hipStream_t s;
  int rc = enter(p, stream, &s);
  if (rc) return rc;
  if (!kappa || !label) return set_error(MCH_EINVAL, "null kappa or label");
  rc = run_graph(p, p->g_fwd, kappa, label, nullptr, nullptr, s, [&] {
    int r = launch_validate(p, kappa, label, s);
    if (r) return r;
    return p->dim == 3 ? launch_forward_3d(p, kappa, label, s) : launch_forward_2d(p, kappa, label, s);
  });
  if (rc) return rc;
  p->forward_done = 1;
  p->fwd_kappa = kappa;
  p->fwd_label = label;
  p->last_stream = s;
  return MCH_OK;
}

extern "C" int mch_effective_coeffs(mch_plan* p, const double* kappa, double* A, void* stream) {
  hipStream_t s;
  int rc = enter(p, stream, &s);
  if (rc) return rc;
  if (!kappa || !A) return set_error(MCH_EINVAL, "null kappa or A_eff");
  if (!p->forward_done) return set_error(MCH_ESTALE, "no forward solve has been issued on this plan");
  if (kappa != p->fwd_kappa)
    return set_error(MCH_EINVAL, "kappa is not the array of the most recent forward solve on this plan");
  rc = run_graph(p, p->g_eff, kappa, A, p->fwd_label, nullptr, s, [&] { return p->dim == 3 ? launch_eff_3d(p, kappa, A, s) : launch_eff_2d(p, kappa, A, s); });
  if (!rc) p->last_stream = s;
  return rc;
}

extern "C" int mch_effective_coeffs_backward(mch_plan* p, const double* kappa, const double* gA, double* glogk,
                                             void* stream) {
  hipStream_t s;
  int rc = enter(p, stream, &s);
  if (rc) return rc;
  if (!kappa || !gA || !glogk) return set_error(MCH_EINVAL, "null argument");
  if (!p->forward_done) return set_error(MCH_ESTALE, "no forward solve has been issued on this plan");
  // the adjoint reads the forward's local solutions, labels and kappa
  if (kappa != p->fwd_kappa)
    return set_error(MCH_EINVAL, "kappa is not the array of the most recent forward solve on this plan");
  rc = run_graph(p, p->g_bwd, kappa, gA, glogk, p->fwd_label, s, [&] {
    return p->dim == 3 ? launch_backward_3d(p, kappa, gA, glogk, s) : launch_backward_2d(p, kappa, gA, glogk, s);
  });
  if (!rc) p->last_stream = s;
  return rc;
}

extern "C" int mch_local_solutions(mch_plan* p, const int64_t* cells, int64_t n, double* out, void* stream) {
  hipStream_t s;
  int rc = enter(p, stream, &s);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!cells || !out))) return set_error(MCH_EINVAL, "bad cell list");
  if (!p->forward_done) return set_error(MCH_ESTALE, "no forward solve has been issued on this plan");
  for (int64_t k = 0; k < n; ++k)
    if (cells[k] < 0 || cells[k] >= p->P) return set_error(MCH_EINVAL, "macropoint index out of range");
  if (n == 0) return MCH_OK;
  return p->dim == 3 ? launch_local_solutions_3d(p, cells, n, out, s) : launch_local_solutions_2d(p, cells, n, out, s);
}

extern "C" int mch_macro_load(mch_plan* p, const double* f, double* b, void* stream) {
  hipStream_t s;
  int rc = enter(p, stream, &s);
  if (rc) return rc;
  if (!f || !b) return set_error(MCH_EINVAL, "null f or b");
  if (!p->forward_done) return set_error(MCH_ESTALE, "no forward solve has been issued on this plan");
  return launch_macro_load(p, f, b, s);
}

extern "C" int mch_macro_solve(mch_plan* p, const double* A, const double* b, double* U, double* U_block,
                               double rtol, int32_t max_iter, void* stream) {
  hipStream_t s;
  int rc = enter(p, stream, &s);
  if (rc) return rc;
  if (!A || !b || !U || !U_block) return set_error(MCH_EINVAL, "null argument");
  if (!(rtol > 0.0) || max_iter < 1) return set_error(MCH_EINVAL, "rtol must be > 0 and max_iter >= 1");
  rc = launch_macro_solve(p, A, b, U, U_block, rtol, max_iter, s);
  if (rc) return rc;
  p->macro_stream = s;
  p->macro_done = 1;
  p->macro_max_iter = max_iter;
  p->macro_rtol = rtol;
  return MCH_OK;
}

extern "C" int mch_macro_solve_noalloc(const mch_plan* p, const double* A, const double* b, double* U,
                                       double* U_block, double rtol, int32_t max_iter, int32_t* iters, double* resid,
                                       void* stream) {
  if (!p) return set_error(MCH_EINVAL, "null plan");
  int rc = hip_check(hipSetDevice(p->device), "hipSetDevice");
  if (rc) return rc;
  if (!A || !b || !U || !U_block || !iters || !resid) return set_error(MCH_EINVAL, "null argument");
  if (!(rtol > 0.0) || max_iter < 1) return set_error(MCH_EINVAL, "rtol must be > 0 and max_iter >= 1");
  return launch_macro_solve_noalloc(p, A, b, U, U_block, rtol, max_iter, iters, resid,
                                    reinterpret_cast<hipStream_t>(stream));
}
