// C-ABI entry points: argument checks, device/stream plumbing, dispatch to
// the kernel launchers.
#include <string>

#include "plan.h"

using namespace mch;

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
  rc = launch_forward_2d(p, kappa, label, s);
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
  rc = launch_eff_2d(p, kappa, A, s);
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
  rc = launch_backward_2d(p, kappa, gA, glogk, s);
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
  return launch_local_solutions_2d(p, cells, n, out, s);
}
