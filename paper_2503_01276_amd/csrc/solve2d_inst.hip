// Instances of the 2D solve kernel for one number of sub-blocks per axis,
// S = MCH_SUB; the build compiles this file once per S.
#include "solve2d_kernel.h"

#ifndef MCH_SUB
#error "compile with -DMCH_SUB=<sub-blocks per axis>"
#endif

namespace mch {

namespace {
// (cell width, node rows per thread, continua, Galerkin) shapes offered for
// every S where the sub-blocks are whole bands and m = N S^2 <= 64.
#define MCH_SHAPES(X)                                                                            \
  X(64, 4, 1, false) X(64, 4, 2, false) X(64, 4, 3, false)                                       \
  X(64, 8, 1, false) X(64, 8, 2, false) X(64, 8, 3, false)                                       \
  X(32, 4, 1, false) X(32, 4, 2, false) X(32, 4, 3, false)                                       \
  X(32, 1, 2, false) X(32, 1, 3, false) X(16, 4, 1, false) X(16, 4, 2, false) X(16, 4, 3, false) \
  X(32, 4, 1, true) X(32, 4, 2, true) X(32, 4, 3, true) X(32, 2, 2, true) X(32, 2, 3, true)      \
  X(32, 1, 2, true) X(32, 1, 3, true) X(16, 4, 1, true) X(16, 4, 2, true) X(16, 4, 3, true)      \
  X(16, 1, 2, true) X(16, 1, 3, true) X(8, 1, 1, true) X(8, 1, 2, true) X(8, 1, 3, true)

template <int NC, int RPT, int N>
constexpr bool kValid = NC % MCH_SUB == 0 && (NC / MCH_SUB) % RPT == 0 && N * MCH_SUB * MCH_SUB <= 64;
}  // namespace

template <>
const void* solve_kernel_sub<MCH_SUB>(int NC, int rpt, int N, bool gal, bool pre, int sb, int* threads) {
  // the band coarse correction needs bands of at least two node rows; two
  // sub-bands per thread exist for the 64^2 fine cells (8 rows per thread)
#define X(nc_, r_, n_, g_)                                                                           \
  if constexpr (kValid<nc_, r_, n_>) {                                                               \
    if (NC == nc_ && rpt == r_ && N == n_ && gal == g_) {                                            \
      *threads = nc_ * nc_ / r_;                                                                     \
      if constexpr (r_ >= 2) {                                                                       \
        if (pre && sb == 1) return reinterpret_cast<const void*>(k_solve2d<nc_, r_, n_, g_, MCH_SUB, true, 1>); \
      }                                                                                              \
      if constexpr (nc_ == 64 && r_ == 8 && !g_) {                                                   \
        if (pre && sb == 2) return reinterpret_cast<const void*>(k_solve2d<nc_, r_, n_, g_, MCH_SUB, true, 2>); \
      }                                                                                              \
      if (pre) return nullptr;                                                                       \
      return reinterpret_cast<const void*>(k_solve2d<nc_, r_, n_, g_, MCH_SUB, false, 1>);           \
    }                                                                                                \
  }
  MCH_SHAPES(X)
#undef X
  return nullptr;
}

}  // namespace mch
