// Device-side helpers shared by the 2D kernels (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MCH_DEV __device__ __forceinline__

namespace mch {

constexpr int WAVE = 64;
// Accelerator complex dies; a launch's workgroups are dealt to them round
// robin (workgroup b runs on die b mod kXcds), each die with its own L2.
constexpr int kXcds = 8;

// i mod n for a coordinate within one period of the grid, -n <= i < 2n (a
// cell-window coordinate: the window starts at most n/2 before the grid and
// is at most n wide): a compare and an add instead of an integer division.
MCH_DEV int wrap1(int i, int n) {
  i = i < 0 ? i + n : i;
  return i >= n ? i - n : i;
}

MCH_DEV int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Cross-lane moves of a binary64 value with DPP (VALU, no LDS round trip).
// Lanes whose source is outside the wave receive 0.
template <int CTRL>
MCH_DEV double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

MCH_DEV double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

constexpr int DPP_QUAD_XOR1 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int DPP_ROW_MIRROR = 0x140;  // lane i <- 15-i within 16
constexpr int DPP_HALF_MIRROR = 0x141; // lane i <- 7-i within 8
constexpr int DPP_WAVE_SHL1 = 0x130;   // lane i <- lane i+1
constexpr int DPP_WAVE_SHR1 = 0x138;   // lane i <- lane i-1

// Sum over aligned groups of `width` lanes (a power of two, 1..64); every lane
// of a group receives the group sum. Fixed order, so bitwise reproducible.
MCH_DEV double seg_sum(double v, int width) {
  if (width >= 2) v += dpp_f64<DPP_QUAD_XOR1>(v);
  if (width >= 4) v += dpp_f64<DPP_QUAD_XOR2>(v);
  if (width >= 8) v += dpp_f64<DPP_HALF_MIRROR>(v);
  if (width >= 16) v += dpp_f64<DPP_ROW_MIRROR>(v);
  if (width >= 32) {
    const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
    const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
    if (width == 32)
      v = ((int)(threadIdx.x & 63) < 32) ? r0 + r1 : r2 + r3;
    else
      v = (r0 + r1) + (r2 + r3);
  }
  return v;
}

// Sum over all 64 lanes; every lane gets the result.
MCH_DEV double wave_sum(double v) { return seg_sum(v, 64); }

// seg_sum of K independent values: each DPP step is issued for all K values
// before their adds, so the K dependency chains overlap instead of queueing.
// Per value the additions are those of seg_sum, in the same order.
template <int CTRL, int K>
MCH_DEV void dpp_add_n(double (&v)[K]) {
  double t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] = dpp_f64<CTRL>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += t[k];
}

template <int K>
MCH_DEV void seg_sum_n(double (&v)[K], int width) {
  if (width >= 2) dpp_add_n<DPP_QUAD_XOR1>(v);
  if (width >= 4) dpp_add_n<DPP_QUAD_XOR2>(v);
  if (width >= 8) dpp_add_n<DPP_HALF_MIRROR>(v);
  if (width >= 16) dpp_add_n<DPP_ROW_MIRROR>(v);
  if (width >= 32) {
    const bool lowhalf = (int)(threadIdx.x & 63) < 32;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double r0 = readlane_f64(v[k], 0), r1 = readlane_f64(v[k], 16);
      const double r2 = readlane_f64(v[k], 32), r3 = readlane_f64(v[k], 48);
      if (width == 32)
        v[k] = lowhalf ? r0 + r1 : r2 + r3;
      else
        v[k] = (r0 + r1) + (r2 + r3);
    }
  }
}

template <int K>
MCH_DEV void wave_sum_n(double (&v)[K]) { seg_sum_n<K>(v, 64); }

// Sum of K consecutive-stride values x[0], x[S], ..., x[(K-1)S] as a balanced
// binary tree (fixed order; depth log2 K instead of K - 1).
template <int K, int S>
MCH_DEV double tree_sum(const double* x) {
  if constexpr (K == 1) {
    return x[0];
  } else {
    constexpr int H = K / 2;
    return tree_sum<H, S>(x) + tree_sum<K - H, S>(x + H * S);
  }
}

// Relative residual sqrt(rz / rz0) of a preconditioned recurrence. NaN when
// either value is NaN, so that a solve whose recurrence turned non-finite is
// never reported as converged; 0 for a zero right-hand side (rz0 = 0).
MCH_DEV double rel_resid(double rz, double rz0) {
  if (rz != rz || rz0 != rz0) return __builtin_nan("");
  return rz0 > 0.0 ? sqrt(fmax(rz, 0.0) / rz0) : 0.0;
}

// Value held by lane+1 (0 for the last lane of a group of `width` lanes).
MCH_DEV double from_right(double v, int c, int width) {
  const double t = dpp_f64<DPP_WAVE_SHL1>(v);
  return (c == width - 1) ? 0.0 : t;
}

// Value held by lane-1 (0 for the first lane of a group).
MCH_DEV double from_left(double v, int c) {
  const double t = dpp_f64<DPP_WAVE_SHR1>(v);
  return (c == 0) ? 0.0 : t;
}

// ---- the band matrices of the preconditioner's coarse correction ----------
// The solve kernel applies T_b^-1 (tridiagonal over a band's node columns)
// by cyclic reduction, and the set-up builds the Schur matrix B G^-1 B^T with
// the same factors. Both call the functions below with contraction of
// multiply-add pairs off or made explicit, so the two compute T_b's entries
// and its factors to the last bit alike: two factorisations of a band matrix
// of condition 1e8 that differ in rounding disagree in the eighth digit, and
// a Schur matrix from one does not project the residual of the other.

// Adds one node row's K_n entries (centre, north, south, east, north-east,
// south-east) between free nodes of a band to the diagonal td and the
// super-diagonal tc of its band matrix row: the row's own entries always,
// its northern neighbour's if that row is in the band (upIn), its southern
// one's likewise (dnIn); the eastern ones only where the node to the east is
// free (frE).
MCH_DEV void band_row_add(double& td, double& tc, bool frE, bool upIn, bool dnIn, double cen, double nor,
                          double sou, double eas, double ne, double se) {
#pragma clang fp contract(off)
  td += cen + (upIn ? nor : 0.0) + (dnIn ? sou : 0.0);
  if (frE) tc += eas + (upIn ? ne : 0.0) + (dnIn ? se : 0.0);
}

// The six K_n entries of a fine-level node from the kappa / 6 of its four
// elements (south-west, south-east, north-west, north-east).
MCH_DEV void fine_stencil6(double kSW, double kSE, double kNW, double kNE, double (&k6)[6]) {
#pragma clang fp contract(off)
  const double aS = kSW + kSE, aN = kNW + kNE;
  k6[0] = 4.0 * (aS + aN);
  k6[1] = -aN;
  k6[2] = -aS;
  k6[3] = -(kSE + kNE);
  k6[4] = -2.0 * kNE;
  k6[5] = -2.0 * kSE;
}

// Offset of stride 2^k's factors in a band's block; the block holds
// pcr_offset(nc, log2 nc) values.
__host__ __device__ constexpr int pcr_offset(int nc, int k) { return 2 * (k * nc - ((1 << k) - 1)); }

// Cyclic reduction of a tridiagonal system held one row per lane in groups
// of nc lanes (a power of two, at most a wave): lane c holds its row's
// sub-diagonal a, diagonal b and super-diagonal cc. Step k (stride 2^k)
// eliminates the couplings at that stride; its factors on the rows 2^k
// below and above are stored through put(k, hasL, hasR, al, ga). Returns
// 1 / the final pivot of the lane's row.
template <typename Put>
MCH_DEV double pcr_factor(int c, int nc, int logn, double a, double b, double cc, Put&& put) {
#pragma clang fp contract(off)
#pragma unroll
  for (int k = 0; k < logn; ++k) {
    const int st = 1 << k;
    const bool hasL = c >= st, hasR = c + st < nc;
    const double aL = __shfl_up(a, st, nc), bL = __shfl_up(b, st, nc), cL = __shfl_up(cc, st, nc);
    const double aR = __shfl_down(a, st, nc), bR = __shfl_down(b, st, nc), cR = __shfl_down(cc, st, nc);
    const double al = hasL ? -a / bL : 0.0;
    const double ga = hasR ? -cc / bR : 0.0;
    put(k, hasL, hasR, al, ga);
    const double na = hasL ? al * aL : 0.0;
    const double nc2 = hasR ? ga * cR : 0.0;
    b = __builtin_fma(ga, hasR ? aR : 0.0, __builtin_fma(al, hasL ? cL : 0.0, b));
    a = na;
    cc = nc2;
  }
  return 1.0 / b;
}

// One elimination step on a right-hand side: d + al d_below + ga d_above.
MCH_DEV double pcr_rhs(double d, double al, double dL, double ga, double dR) {
  return __builtin_fma(ga, dR, __builtin_fma(al, dL, d));
}

// Arguments shared by the cell kernels. Every pointer is a device pointer;
// per-point arrays are indexed by the global macropoint index p.
struct CellArgs {
  const double* kappa;    // [n^d] fine coefficient
  const uint8_t* label;   // [n^d] continuum labels
  int n;                  // fine elements per axis (global)
  int n_macro;            // macropoints per axis
  int H;                  // fine elements per coarse block
  int nc;                 // cell width in fine elements
  int s;                  // sub-blocks per axis
  int N;                  // continua
  int M;                  // right-hand sides per macropoint
  int m;                  // constraint rows per cell (s^d * N)
  double h;
  // level being processed
  int r;                  // eta^(level-1)
  int NC;                 // nc / r
  int sbw;                // sub-block width in level elements (nc / s / r)
  const int32_t* cells;   // [count] macropoint ids of this level
  const int32_t* pslot;   // [count] level-1 slot of the inherited point (levels >= 2)
  int count;              // cells in this launch (a chunk of the level)
  int ci0;                // index within the level of the launch's first cell
  // per-point data
  double* cw;             // [P][m] 1 / (4 n_qj), 0 for inactive rows
  double* g;              // [P][M][m]
  double* sinv;           // [P][m][m]
  double* beta;           // [P][M][m] multipliers of the last solve of this point
  int32_t* iters;         // [P][M]
  double* resid;          // [P][M]
  // level-1 fine solutions [n1][M][(nc+1)^2]; this level's output [count][M][(NC+1)^2]
  const double* phi1;
  double* out;
  // Galerkin tables for this level: T[r*r][16] (R^T K_ref R), rho[r*r][4]
  const double* tabK;
  const double* tabR;
  // Galerkin level data written by the setup kernel, per cell of this level
  // (2D, every level node (X, Y) in [0, NC]^2 at Y (NC+1) + X):
  // 9-point stencil per node [count][(NC+1)^2][9] and constraint weights per
  // node, side (0: element column X-1, 1: column X), part (0: element row Y-1,
  // 1: row Y) and continuum [count][(NC+1)^2][4][N]; inherited right-hand
  // sides f [count][M][(NC+1)^2] and g' [count][M][m] from the inherit kernel.
  // (3D: the owned nodes [0, NC)^3.)
  double* nodeW;
  float* nodeB;
  double* fin;
  double* gin;
  int J;                  // lanes per Schur row in the solve kernel
  // node rows per band of the band coarse correction in the preconditioner
  // (the solve kernel's rows per thread), 0 for diagonal scaling alone
  int prec_rows;
  // adjoint mode inputs
  int adjoint;
  const double* seed_kp;  // [P][M][(H+1)^2] explicit seed on the K_p nodes
  const double* seed_par; // [n1][M][(nc+1)^2] seeds accumulated from inheriting cells (level 1)
  const int32_t* slot;    // [P] index of the point within its level
  double rtol;
  int max_iter;
  // cell boundary condition: 0 homogeneous Dirichlet (free level nodes
  // [1, NC-1]^d), 1 natural Neumann (every node [0, NC]^d free)
  int bc;
  // 2D generic solve kernel: threads per constraint sub-block (0: the
  // register-resident kernel of the level's shape)
  int gen_tp;
  // 2D register-resident solve: workgroups numbered so that a cell's
  // right-hand sides run on one XCD (1), or in plain order (0)
  int xcd_groups;
  // 3D cells (unused in 2D): windows, D^-1 and Krylov vectors of this level,
  // and Phi on the K_p nodes of every point
  double* kw;             // fine level: 3D [count][NC^3] kappa*h/12; 2D generic kernel [count][NC^2] kappa/6
  uint8_t* labw;          // fine level: [count][NC^d] labels (3D, 2D generic kernel)
  uint16_t* octw;         // fine level: [count][NC^3] labels of the 8 octant elements of each node, 2 bits each (3 = none)
  double* dinv;           // 3D: [count][NC^3]; 2D generic kernel: [count][M][(NC+1)^2]
  double* vr;             // 3D: [count][M][(NC+1)^3]; 2D generic kernel: [count][M][(NC+3)^2] (ring of zeros)
  double* vp;
  double* vap;
  double* phikp;          // [P][M][(H+1)^3]
};

// Fine local solution Phi_alpha = I + P xi of cell ci (index within its level)
// at fine node (X, Y) of the cell, X, Y in [0, nc]. For level 1, Phi is stored.
MCH_DEV double phi_at(const CellArgs& a, int ci, int alpha, int X, int Y) {
  // fine node (X, Y) of the cell, in [0, nc]
  const int nn1 = a.nc + 1;
  if (a.r == 1) return a.out[((size_t)ci * a.M + alpha) * (size_t)nn1 * nn1 + (size_t)Y * nn1 + X];
  const double* I = a.phi1 + ((size_t)a.pslot[ci] * a.M + alpha) * (size_t)nn1 * nn1;
  const double* xi = a.out + ((size_t)ci * a.M + alpha) * (size_t)(a.NC + 1) * (a.NC + 1);
  const int r = a.r, NCp = a.NC + 1;
  const int cx = X / r, cy = Y / r;
  const double tx = (X - cx * r) / (double)r, ty = (Y - cy * r) / (double)r;
  const int cx1 = cx + (tx > 0.0 ? 1 : 0), cy1 = cy + (ty > 0.0 ? 1 : 0);
  double v = (1 - tx) * (1 - ty) * xi[cy * NCp + cx] + tx * (1 - ty) * xi[cy * NCp + cx1] +
             (1 - tx) * ty * xi[cy1 * NCp + cx] + tx * ty * xi[cy1 * NCp + cx1];
  return I[(size_t)Y * nn1 + X] + v;
}


// Bilinear prolongation of a level-r vector v [(NC+1)^2] to fine node (X, Y).
MCH_DEV double prolong_at(const double* v, int r, int NC, int X, int Y) {
  if (r == 1) return v[(size_t)Y * (NC + 1) + X];
  const int NCp = NC + 1;
  const int cx = X / r, cy = Y / r;
  const double tx = (X - cx * r) / (double)r, ty = (Y - cy * r) / (double)r;
  const int cx1 = cx + (tx > 0.0 ? 1 : 0), cy1 = cy + (ty > 0.0 ? 1 : 0);
  return (1 - tx) * (1 - ty) * v[cy * NCp + cx] + tx * (1 - ty) * v[cy * NCp + cx1] +
         (1 - tx) * ty * v[cy1 * NCp + cx] + tx * ty * v[cy1 * NCp + cx1];
}

// (K_ref v)_corner * 6 for the 2D Q1 element, corners in tensor order (00,10,01,11).
MCH_DEV void kref6_apply(const double (&v)[4], double (&y)[4]) {
  y[0] = 4 * v[0] - v[1] - v[2] - 2 * v[3];
  y[1] = -v[0] + 4 * v[1] - 2 * v[2] - v[3];
  y[2] = -v[0] - 2 * v[1] + 4 * v[2] - v[3];
  y[3] = -2 * v[0] - v[1] - v[2] + 4 * v[3];
}

}  // namespace mch
