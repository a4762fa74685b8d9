// Device-side helpers shared by the 2D kernels (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MCH_DEV __device__ __forceinline__

namespace mch {

constexpr int WAVE = 64;

MCH_DEV int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Sum over all 64 lanes (butterfly; every lane gets the result).
MCH_DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Sum over aligned groups of `width` lanes (width a power of two <= 64).
MCH_DEV double seg_sum(double v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Value held by lane+1 (0 for the last lane of a group of `width` lanes).
MCH_DEV double from_right(double v, int c, int width) {
  double t = __shfl_down(v, 1, WAVE);
  return (c == width - 1) ? 0.0 : t;
}

// Value held by lane-1 (0 for the first lane of a group).
MCH_DEV double from_left(double v, int c) {
  double t = __shfl_up(v, 1, WAVE);
  return (c == 0) ? 0.0 : t;
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
  int count;
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
  // adjoint mode inputs
  int adjoint;
  const double* seed_kp;  // [P][M][(H+1)^2] explicit seed on the K_p nodes
  const double* seed_par; // [n1][M][(nc+1)^2] seeds accumulated from inheriting cells (level 1)
  const int32_t* slot;    // [P] index of the point within its level
  double rtol;
  int max_iter;
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
