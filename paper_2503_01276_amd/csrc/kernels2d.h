// Internal declarations shared by the 2D kernel translation units.
#pragma once

#include "device_common.h"
#include "plan.h"

namespace mch {
// Kernel arguments for the cells of level l (0-based) of a plan.
CellArgs base_args(mch_plan* pl, const double* kappa, const uint8_t* label, int l);
// The same arguments restricted to cells [start, start + count) of the level.
CellArgs chunk_args(const CellArgs& a, int start, int count);
// Launch the constrained Krylov solve of every (cell, right-hand side) of a
// (the generic kernel when a.gen_tp > 0).
int launch_solve(const CellArgs& a, int rpt, hipStream_t s);
int launch_solve_generic(const CellArgs& a, hipStream_t s);
// Workgroups of the generic solve kernel that fit on one CU at once.
int generic_blocks_per_cu(const CellArgs& a);
// The 3D generic solve (cells with a.gen_tp > 0) and its workgroups per CU.
int launch_solve3d_generic(const CellArgs& a, hipStream_t s);
int generic3_blocks_per_cu(const CellArgs& a);

// Lanes per row of the per-wave Schur solve: the largest power of two J with
// J m <= 64, so the m rows of S^-1 u fit one wave.
constexpr int schur_lanes(int m) {
  int J = 1;
  while (J * 2 * m <= 64) J *= 2;
  return J;
}

// Solve kernel for cells of S sub-blocks per axis (S = 1, 2, 4, 8; one
// translation unit each): the kernel of a (cell width, node rows per thread,
// continua, Galerkin, band coarse correction, sub-bands per thread) shape and
// its block size, or nullptr if that shape is not instantiated.
template <int S>
const void* solve_kernel_sub(int NC, int rpt, int N, bool gal, bool pre, int sb, int* threads);
template <>
const void* solve_kernel_sub<1>(int, int, int, bool, bool, int, int*);
template <>
const void* solve_kernel_sub<2>(int, int, int, bool, bool, int, int*);
template <>
const void* solve_kernel_sub<4>(int, int, int, bool, bool, int, int*);
template <>
const void* solve_kernel_sub<8>(int, int, int, bool, bool, int, int*);
// Whether a level can use the band coarse correction with sb sub-bands per
// thread's rows (kernel instantiated and its LDS within the budget).
bool prec_supported_2d(int NC, int rpt, int N, bool gal, int S, int m, int sb);
// Per-cell setup (constraint rows, right-hand sides, Galerkin data, S^-1).
int launch_setup(const CellArgs& a, hipStream_t s);
// Inherited right-hand sides of a level >= 2 (needs the level-1 solutions).
int launch_inherit(const CellArgs& a, hipStream_t s);
// Multilinear inheritance (interp = 1): I of level l's cells from the T-slot
// store (2D and 3D); Phi = I + P xi of level l into its T slots (2D); c_t Ibar
// of level l's cells into the seeds of their neighbours (2D and 3D); a fill
// with zeros.
int launch_interp(mch_plan* pl, int l, hipStream_t s);
int launch_recon_2d(mch_plan* pl, const CellArgs& a, int l, hipStream_t s);
int launch_distribute(mch_plan* pl, int l, hipStream_t s);
int launch_zero(double* p, size_t n, hipStream_t s);
}  // namespace mch
