// Internal declarations shared by the 2D kernel translation units.
#pragma once

#include "device_common.h"
#include "plan.h"

namespace mch {
// Kernel arguments for the cells of level l (0-based) of a plan.
CellArgs base_args(mch_plan* pl, const double* kappa, const uint8_t* label, int l);
// The same arguments restricted to cells [start, start + count) of the level.
CellArgs chunk_args(const CellArgs& a, int start, int count);
// Launch the constrained Krylov solve of every (cell, right-hand side) of a.
int launch_solve(const CellArgs& a, int rpt, hipStream_t s);
// Per-cell setup (constraint rows, right-hand sides, Galerkin data, S^-1).
int launch_setup(const CellArgs& a, hipStream_t s);
// Inherited right-hand sides of a level >= 2 (needs the level-1 solutions).
int launch_inherit(const CellArgs& a, hipStream_t s);
}  // namespace mch
