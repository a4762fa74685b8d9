// Host-side plan of the cell-solve library (internal header).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/mch.h"

namespace mch {

constexpr int MAX_LEVELS = 8;
// Most workgroups of the grid-wide macroscopic CG (each of its two
// partial-sum buffers holds one value per workgroup).
constexpr int kMacroGridMax = 4096;
// Workgroups of the input check (one result slot each).
constexpr int kValidateBlocks = 256;
// Fixed device buffer of the macroscopic solve without allocation (per
// device, in doubles): 16 MiB.
constexpr size_t kNoAllocScratchDoubles = (size_t)2 << 20;

// Kernel shape chosen for one level's cells.
struct KernelShape {
  int NC = 0;    // cell width in level elements
  int rpt = 0;   // node rows per thread
  int threads = 0;
  bool pre = false;  // 2D: band coarse correction in the preconditioner
  int sb = 1;        // 2D: sub-bands of the correction per thread's node rows
  int gen_tp = 0;    // 2D generic solve kernel: threads per sub-block tile (0: not used)
};

struct Level {
  int n = 0;       // 1..L
  int r = 1;       // eta^(n-1)
  int NC = 0;      // cell width in level elements
  int count = 0;   // macropoints on this level
  std::vector<int32_t> cells;   // host copy
  int32_t* d_cells = nullptr;
  int32_t* d_pslot = nullptr;   // level-1 slot of the inherited point
  double* d_out = nullptr;      // level 1: Phi [count][M][(nc+1)^d]; else xi [count][M][(NC+1)^d]
  double* d_w = nullptr;        // adjoint solution, same shape as d_out
  double* d_tabK = nullptr;     // Galerkin tables (levels >= 2)
  double* d_tabR = nullptr;
  double* d_nodeW = nullptr;    // Galerkin 9-point stencils [count][NC^d][9]
  float* d_nodeB = nullptr;     // Galerkin constraint weights [count][NC^d][4][N]
  double* d_fin = nullptr;      // inherited right-hand sides [count][M][NC^d]
  double* d_gin = nullptr;      // [count][M][m]
  // 3D cells only: fine-level windows kappa*h/12 and labels [count][NC^3],
  // 1/diag(K_n) per level node [count][NC^3], and the Krylov vectors
  // r, p, K_n p of every (cell, rhs) [count][M][(NC+1)^3] (zero boundary)
  double* d_kw = nullptr;
  uint8_t* d_labw = nullptr;
  uint16_t* d_octw = nullptr;   // 3D fine level: octant label codes per node [count][NC^3]
  double* d_dinv = nullptr;
  double* d_vr = nullptr;
  double* d_vp = nullptr;
  double* d_vap = nullptr;
  // multilinear interpolation (interp = 1). Levels >= 2: the inherited
  // fine vectors I = sum_t c_t Phi_t [count][M][nn] (d_pslot is then the
  // identity), the T slots and weights of each cell's neighbours [count][2^d]
  // (weight 0 = unused), and the CSR over the T slots of the levels below of
  // this level's cells that inherit from them (cell index and weight), for
  // passing c_t Ibar back. Levels < L: toff = first T slot of the level.
  double* d_I = nullptr;
  int32_t* d_nbr = nullptr;
  double* d_nbw = nullptr;
  int toff = 0;
  int32_t* d_dptr = nullptr;
  int32_t* d_dch = nullptr;
  double* d_dw = nullptr;
  KernelShape shape;
};

}  // namespace mch

namespace mch {
// One profiled launch: HIP events recorded on the launch's stream around it.
struct ProfRec {
  std::string name;
  hipEvent_t start = nullptr, stop = nullptr;
};
}  // namespace mch

struct mch_plan {
  mch_config cfg{};
  int dim = 2;
  int n = 0;        // fine elements per axis
  int nm = 0;       // macropoints per axis
  int H = 0;        // fine elements per coarse block
  int P = 0;        // macropoints
  int M = 0;        // right-hand sides per macropoint
  int m = 0;        // constraint rows per cell
  int L = 1;
  int nn = 0;       // fine nodes per cell, (nc+1)^d
  int device = 0;
  std::vector<int32_t> level, parent, slot;  // host, per macropoint
  // interp = 1: neighbours (point ids, -1 = unused) and weights, [P][2^d]
  std::vector<int32_t> nbr;
  std::vector<double> nbw;
  // interp = 1: the points of levels 1..L-1 (T_(L-1)) in level-major order
  // ("T slots"); level 1's output holds the fine Phi of all of them
  int nT = 0;
  double* d_seedT = nullptr;   // [nT][M][nn] seeds on the Phi of the T points
  double* d_ibar = nullptr;    // [max level count][M][nn] Ibar of one level's cells
  int32_t* d_iptr = nullptr;   // [max level count + 1] identity CSR (0, 1, 2, ...)
  mch::Level lev[mch::MAX_LEVELS];
  // per-point device scratch
  double* d_cw = nullptr;
  double* d_g = nullptr;
  double* d_sinv = nullptr;
  double* d_beta = nullptr;
  double* d_mu = nullptr;
  int32_t* d_iters = nullptr;
  double* d_resid = nullptr;
  int32_t* d_slot = nullptr;
  // input check of the last forward: per workgroup the first fine element
  // with kappa not positive and finite or a label >= n_cont, or -1
  long long* d_bad = nullptr;
  // adjoint scratch
  double* d_seed_kp = nullptr;   // [P][M][(H+1)^d]
  double* d_seed_par = nullptr;  // [n1][M][nn]
  double* d_seed_lvl[mch::MAX_LEVELS] = {};  // 2D: parent seeds of one inheriting level [n1][M][nn]
  double* d_gk = nullptr;        // [n^d] explicit part of dLoss/dkappa (K_p terms)
  double* d_gcell = nullptr;     // [P][nc^d] per-cell part of dLoss/dkappa on the cell window
  int32_t* d_iters_adj = nullptr;
  double* d_resid_adj = nullptr;
  int32_t* d_level = nullptr;    // [P]
  int32_t* d_child_ptr = nullptr;  // [n1+1] CSR of inheriting points per level-1 slot
  int32_t* d_child = nullptr;      // [P - n1] macropoint ids
  double* d_phikp = nullptr;       // 3D: Phi on the K_p nodes [P][M][(H+1)^3]
  // macroscopic system (allocated on first use): element matrices
  // [P][2^d N][2^d N], nodal stencil rows [3^d N][n] over the n = (n_macro-1)^d N
  // interior unknowns, CG vectors x, r, z, p, q [n], the inverse nodal
  // blocks [N N][n / N] and s [n] (the grid-wide CG), iterations and final
  // relative residual
  double* d_macroE = nullptr;
  double* d_macroS = nullptr;
  double* d_mvec = nullptr;        // x, r, z, p, q, the block inverses, s
  double* d_mpart = nullptr;       // 2 x kMacroGridMax partial sums (grid-wide CG)
  int32_t* d_macro_iters = nullptr;
  double* d_macro_resid = nullptr;
  hipStream_t macro_stream = nullptr;  // stream of the last macroscopic solve (may be the default stream)
  int macro_done = 0;
  int macro_max_iter = 0;
  double macro_rtol = 0.0;
  hipStream_t last_stream = nullptr;
  int forward_done = 0;
  const double* fwd_kappa = nullptr;
  const uint8_t* fwd_label = nullptr;
  std::vector<void*> allocations;
  // per-level side streams (default priority) and events for the level DAG:
  // levels >= 2 depend only on level 1, so they run as parallel branches
  hipStream_t side[mch::MAX_LEVELS] = {};
  hipEvent_t ev_fork = nullptr, ev_l1 = nullptr;
  // Level 1 runs in two chunks: cells [0, n1a) fill the GPU n times over and
  // the rest form the tail of the last round. The cells of every level >= 2
  // are ordered by the slot of their level-1 cell, so the first cntA[l] of
  // them inherit from chunk A and can run while the tail still solves.
  int n1a = 0;
  int cntA[mch::MAX_LEVELS] = {};
  hipEvent_t ev_l1a = nullptr;
  hipEvent_t ev_join[mch::MAX_LEVELS] = {};
  // Second stream per level for its cells inheriting from the level-1 tail
  // chunk: they wait for the level's setup and the end of level 1 only, not
  // for the level's first part. ev_setup marks the setup on the first stream.
  hipStream_t side2[mch::MAX_LEVELS] = {};
  hipEvent_t ev_setup[mch::MAX_LEVELS] = {};
  hipEvent_t ev_join2[mch::MAX_LEVELS] = {};
  // backward: a level's adjoint solve is done (its gradient window may still run)
  hipEvent_t ev_adj[mch::MAX_LEVELS] = {};
  // backward, 2D: the parent-seed pass of a level's cells is done
  hipEvent_t ev_ibar[mch::MAX_LEVELS] = {};
  // captured launch sequences, replayed while the arguments are unchanged
  struct Graph {
    const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
    hipStream_t stream = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
  } g_fwd, g_eff, g_bwd;
  int use_graphs = 1;
  int serial = 0;  // run every level on the caller's stream (kernel-by-kernel timing)
  int xcd_groups = 1;  // 2D solve: a cell's right-hand sides on one XCD (MCH_XCD=0: plain order)
  // profiling (off by default)
  int profiling = 0;
  std::vector<mch::ProfRec> prof;
  size_t prof_used = 0;
};

namespace mch {
// Brackets one kernel launch with events when the plan's profiling is on.
struct ProfScope {
  mch_plan* p;
  hipStream_t s;
  size_t idx;
  bool on;
  ProfScope(mch_plan* plan, const char* name, hipStream_t stream);
  ~ProfScope();
};

int set_error(int code, const std::string& msg);
// Side streams/events of the level DAG (created on first use).
int ensure_streams(mch_plan* p);
// Fork: every side stream of levels 2..L waits for the work issued so far on s.
int fork_levels(mch_plan* p, hipStream_t s);
// Join: s waits for every side stream of levels 2..L.
int join_levels(mch_plan* p, hipStream_t s);
// Record ev[l] on level l's stream (l >= 1), and make s wait for every
// level's recorded event: a partial join that leaves the rest of each level
// stream running (joined later by join_levels).
int mark_level(mch_plan* p, int l, hipEvent_t* ev);
int wait_marks(mch_plan* p, hipStream_t s, hipEvent_t* ev);
// Stream of level l (0-based) in a DAG issued on s.
inline hipStream_t level_stream(const mch_plan* p, int l, hipStream_t s) { return (l == 0 || p->serial) ? s : p->side[l]; }
inline hipStream_t level_stream2(const mch_plan* p, int l, hipStream_t s) { return (l == 0 || p->serial) ? s : p->side2[l]; }
int hip_check(hipError_t e, const char* what);

// Launchers implemented in the .hip translation units.
// Input check of kappa and labels (results read by mch_diagnostics).
int launch_validate(mch_plan* p, const double* kappa, const uint8_t* label, hipStream_t s);
int launch_forward_2d(mch_plan* p, const double* kappa, const uint8_t* label, hipStream_t s);
int launch_eff_2d(mch_plan* p, const double* kappa, double* A, hipStream_t s);
int launch_backward_2d(mch_plan* p, const double* kappa, const double* gA, double* glogk, hipStream_t s);
int launch_local_solutions_2d(mch_plan* p, const int64_t* cells, int64_t n, double* out, hipStream_t s);
// Macroscopic system: block loads from the local solutions, and the
// assembly and CG solve on the macrogrid (2D and 3D).
int launch_macro_load(mch_plan* p, const double* f, double* b, hipStream_t s);
int launch_macro_solve(mch_plan* p, const double* A, const double* b, double* U, double* Ub, double rtol,
                       int max_iter, hipStream_t s);
// Device scratch of the macroscopic solve (host-synchronous on first use).
int ensure_macro_scratch(mch_plan* p);
// The same solve on the library's fixed per-device buffer: no allocation;
// iteration count and residual into the caller's device scalars.
int launch_macro_solve_noalloc(const mch_plan* p, const double* A, const double* b, double* U, double* Ub,
                               double rtol, int max_iter, int32_t* iters, double* resid, hipStream_t s);
bool shape_supported_2d(int NC, int rpt, int N, bool galerkin, int n_sub);
// 2D generic solve kernel (any width, either boundary condition): threads per
// sub-block tile for s sub-blocks per axis (0: too many sub-blocks) and the
// kernel's LDS bytes.
int generic_tile_threads(int s);
// 3D generic solve kernel (Neumann cells): threads per sub-block tile for s
// sub-blocks per axis (0: too many).
int generic3_tile_threads(int s);
size_t generic_lds_bytes(int s, int N, int m, int threads);
int launch_forward_3d(mch_plan* p, const double* kappa, const uint8_t* label, hipStream_t s);
int launch_eff_3d(mch_plan* p, const double* kappa, double* A, hipStream_t s);
int launch_backward_3d(mch_plan* p, const double* kappa, const double* gA, double* glogk, hipStream_t s);
int launch_local_solutions_3d(mch_plan* p, const int64_t* cells, int64_t n, double* out, hipStream_t s);
bool shape_supported_3d(int NC, int s, int N);
// Workgroups of the level-1 solve kernel that fit on one CU at once.
int solve_blocks_per_cu_2d(mch_plan* p);
int solve_blocks_per_cu_3d(mch_plan* p);
}  // namespace mch
