// Multilinear inheritance between levels (interp = 1).
//
// Sec. 3.3, Eq. phiXiI_all: a level-n point starts from I = sum_t c_t Phi_t
// over its neighbours t in T_(n-1) (the levels below), sum_t c_t = 1. The
// points of levels 1..L-1 have "T slots" (level-major); the fine Phi of every
// T point lives in level 1's output array, whose first rows are level 1's own
// solutions. Per level n >= 2:
//   forward:  I of each cell into its row of the level's I array (the solve,
//             effective-tensor and adjoint kernels read I from there), and for
//             n < L, Phi = I + P xi into the level's T slots;
//   backward: Ibar of each cell (Phibar - K_h P w - B_h^T mu plus the seeds the
//             cell itself received from the levels above) is passed to its
//             neighbours as c_t Ibar, gathered per neighbour in a fixed order.
// All three are streaming passes over fine-node vectors, bound by HBM. The
// interpolation and the distribution do not depend on the dimension; the
// reconstruction of Phi in 3D is in the 3D translation unit.
#include "kernels2d.h"

namespace mch {

constexpr int IT = 256;

// I[ci][al][:] = sum_k c_k Phi_T[t_k][al][:], k = 0..K-1 in order (K = 2^d
// neighbour slots, c_k = 0: unused).
template <int K>
__global__ __launch_bounds__(IT) void k_interp(int M, size_t nn, const int32_t* nbr, const double* nbw,
                                               const double* phiT, double* I) {
  const int ci = blockIdx.x / M, al = blockIdx.x % M;
  int t[K];
  double c[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    t[k] = nbr[(size_t)ci * K + k];
    c[k] = nbw[(size_t)ci * K + k];
  }
  double* dst = I + (size_t)blockIdx.x * nn;
  for (size_t nd = threadIdx.x; nd < nn; nd += IT) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (c[k] != 0.0) v += c[k] * phiT[((size_t)t[k] * M + al) * nn + nd];
    dst[nd] = v;
  }
}

// Phi = I + P xi of each cell of a level on every fine node of its cell, into
// T slot toff + ci of the store.
__global__ __launch_bounds__(IT) void k_recon2d(CellArgs a, int toff, double* phiT) {
  const int ci = blockIdx.x / a.M, al = blockIdx.x % a.M;
  const int nn1 = a.nc + 1, nn = nn1 * nn1;
  double* dst = phiT + ((size_t)(toff + ci) * a.M + al) * nn;
  for (int nd = threadIdx.x; nd < nn; nd += IT) dst[nd] = phi_at(a, ci, al, nd % nn1, nd / nn1);
}

// seedT[t] += sum over the level's cells ci inheriting from T slot t of
// c * (Ibar[ci] + own[ci]), entries in increasing ci; own (nullable) holds the
// seeds the level's cells received from the levels above.
__global__ __launch_bounds__(IT) void k_distribute(int M, size_t nn, const int32_t* dptr, const int32_t* dch,
                                                   const double* dw, const double* ibar, const double* own,
                                                   double* seedT) {
  const int t = blockIdx.x / M, al = blockIdx.x % M;
  const int e0 = dptr[t], e1 = dptr[t + 1];
  if (e0 == e1) return;
  double* dst = seedT + ((size_t)t * M + al) * nn;
  for (size_t nd = threadIdx.x; nd < nn; nd += IT) {
    double acc = 0.0;
    for (int e = e0; e < e1; ++e) {
      const size_t o = ((size_t)dch[e] * M + al) * nn + nd;
      const double v = own ? ibar[o] + own[o] : ibar[o];
      acc += dw[e] * v;
    }
    dst[nd] += acc;
  }
}

__global__ void k_zero(size_t n, double* p) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

int launch_interp(mch_plan* pl, int l, hipStream_t s) {
  const Level& lv = pl->lev[l];
  if (lv.count == 0) return MCH_OK;
  ProfScope ps(pl, "interp", s);
  const dim3 grid((unsigned)(lv.count * pl->M));
  if (pl->dim == 2)
    hipLaunchKernelGGL(k_interp<4>, grid, dim3(IT), 0, s, pl->M, (size_t)pl->nn, lv.d_nbr, lv.d_nbw, pl->lev[0].d_out,
                       lv.d_I);
  else
    hipLaunchKernelGGL(k_interp<8>, grid, dim3(IT), 0, s, pl->M, (size_t)pl->nn, lv.d_nbr, lv.d_nbw, pl->lev[0].d_out,
                       lv.d_I);
  return hip_check(hipGetLastError(), "launch k_interp");
}

int launch_recon_2d(mch_plan* pl, const CellArgs& a, int l, hipStream_t s) {
  const Level& lv = pl->lev[l];
  if (lv.count == 0) return MCH_OK;
  ProfScope ps(pl, "recon", s);
  hipLaunchKernelGGL(k_recon2d, dim3((unsigned)(lv.count * pl->M)), dim3(IT), 0, s, a, lv.toff, pl->lev[0].d_out);
  return hip_check(hipGetLastError(), "launch k_recon2d");
}

int launch_distribute(mch_plan* pl, int l, hipStream_t s) {
  const Level& lv = pl->lev[l];
  const int rows = (l + 1 < pl->L) ? lv.toff : pl->nT;
  if (lv.count == 0 || rows == 0) return MCH_OK;
  const double* own = (l + 1 < pl->L) ? pl->d_seedT + (size_t)lv.toff * pl->M * pl->nn : nullptr;
  ProfScope ps(pl, "distribute", s);
  hipLaunchKernelGGL(k_distribute, dim3((unsigned)(rows * pl->M)), dim3(IT), 0, s, pl->M, (size_t)pl->nn, lv.d_dptr,
                     lv.d_dch, lv.d_dw, pl->d_ibar, own, pl->d_seedT);
  return hip_check(hipGetLastError(), "launch k_distribute");
}

int launch_zero(double* p, size_t n, hipStream_t s) {
  if (n == 0) return MCH_OK;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, n, p);
  return hip_check(hipGetLastError(), "launch k_zero");
}

}  // namespace mch
