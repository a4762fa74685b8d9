// Input check of the forward solve: kappa must be positive and finite and
// every label below n_cont on every fine element (each element lies in some
// cell, since the cells contain their coarse blocks and those tile the grid).
//
// One pass over the global arrays, issued ahead of the cell kernels on the
// caller's stream. Every workgroup writes the smallest offending element
// index of its share, or -1, into its own slot, so nothing has to be cleared
// between calls; mch_diagnostics reads the slots.
#include <hip/hip_runtime.h>

#include "plan.h"

namespace mch {

constexpr int VALIDATE_T = 256;

__global__ __launch_bounds__(VALIDATE_T) void k_validate(const double* kappa, const uint8_t* label, long long n,
                                                          int N, long long* bad) {
  __shared__ long long wmin[VALIDATE_T / 64];
  long long first = -1;
  const long long stride = (long long)gridDim.x * VALIDATE_T;
  for (long long e = (long long)blockIdx.x * VALIDATE_T + threadIdx.x; e < n; e += stride) {
    const double k = kappa[e];
    // !(k > 0) catches NaN as well as non-positive values
    const bool ok = (k > 0.0) && (k <= 1.7976931348623157e308) && ((int)label[e] < N);
    if (!ok && first < 0) first = e;
  }
  // smallest non-negative index over the workgroup (-1 if none)
  unsigned long long u = first < 0 ? ~0ull : (unsigned long long)first;
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long v = __shfl_xor(u, off, 64);
    u = v < u ? v : u;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wmin[wave] = u == ~0ull ? -1 : (long long)u;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long r = -1;
    for (int w = 0; w < VALIDATE_T / 64; ++w)
      if (wmin[w] >= 0 && (r < 0 || wmin[w] < r)) r = wmin[w];
    bad[blockIdx.x] = r;
  }
}

int launch_validate(mch_plan* p, const double* kappa, const uint8_t* label, hipStream_t s) {
  long long n = 1;
  for (int a = 0; a < p->dim; ++a) n *= p->n;
  ProfScope ps(p, "validate", s);
  hipLaunchKernelGGL(k_validate, dim3(kValidateBlocks), dim3(VALIDATE_T), 0, s, kappa, label, n, p->cfg.n_cont,
                     p->d_bad);
  return hip_check(hipGetLastError(), "k_validate launch");
}

}  // namespace mch
