// The constrained Krylov solve of the 2D cell problems for gfx950, as a
// template over the cell shape; instantiated per number of sub-blocks in
// solve2d_inst.hip.
//
// Cell problem (paper Sec. 2, Eqs. phi_avar / phi_grad; Sec. 3.3,
// Eqs. phi_avar_corrector / phi_grad_corrector): minimise the kappa-energy of
// v = I + P_n xi over the level-n Q1 space V_n of the oversampled cell,
// subject to the average constraints B_h v = g. In matrix form
//   [K_n  B_n^T][xi  ]   [ f  ]     K_n = P^T K_h P,  B_n = B_h P,
//   [B_n  0    ][beta] = [ g' ],    f = -P^T K_h I,   g' = g - B_h I.
//
// Solver: projected preconditioned CG with the constraint preconditioner
// [G B^T; B 0] (Gould, Hribar & Nocedal 2001), including their residual
// update so the residual stays orthogonal to range(B^T). The iterate starts
// feasible (x0 = G^-1 B^T S^-1 g', S = B G^-1 B^T) and every direction lies
// in null(B), so the constraints hold to rounding. The accumulated
// projections give the multipliers.
//
// G^-1 = D^-1 + sum_b Z_b T_b^-1 Z_b^T with D = diag(K_n) and, when PRE is
// set, a coarse correction per band b (the RPT node rows of one band of
// threads): Z_b has one column per node column of the band, 1 on the band's
// free nodes of that column, and T_b = Z_b^T K_n Z_b is tridiagonal (node
// columns couple only to their neighbours). In a high-contrast channel
// medium the slow modes of diagonal scaling vary slowly along the channels,
// which the band columns resolve; on the 64^2 fine cells this cuts the
// iterations about threefold. T_b^-1 is applied by parallel cyclic reduction
// across the band's lanes (one unknown per lane), with the elimination
// factors computed once per solve and kept in LDS, so the preconditioner
// needs no barrier. Without PRE, G = D. With SB = 2 the correction uses
// sub-bands of RPT / 2 node rows (two coarse unknowns per node column and
// band of threads, two tridiagonal systems per band): on the 64^2 cells of
// the three-continuum medium with inclusions this halves the iterations
// against bands of RPT rows. The factors of both then fill the LDS that the
// 64^2 iterate took, so the iterate is kept in the output array instead.
//
// Layout inside a workgroup: one (cell, right-hand side) per workgroup; lane
// c of a band row owns node column c and element column c; each band of RPT
// node rows belongs to NC consecutive threads. Node rows/columns 0..NC-1 are
// owned, row/column NC is the Dirichlet boundary and never stored. The search
// direction p lives in LDS (padded by one ring of zeros); x, r and the
// per-node operator data live in registers.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels2d.h"

namespace mch {
// Fine cells of width >= 64 keep kappa/6 and the iterate x in LDS instead of
// registers (the register file cannot hold them at 8 nodes per lane).
template <int NC, bool GAL>
constexpr bool kBig = !GAL && NC >= 64;

// One iteration of the projected PCG needs two workgroup barriers: after the
// fused reduction of (p.Ap, r.G^-1 r, r.G^-1 Ap, Ap.G^-1 Ap, B G^-1 r,
// B G^-1 Ap), and after the new search direction is written to LDS. With
// r' the projected residual, r_new = r' + alpha Ap, so both B G^-1 r_new and
// r_new.G^-1 r_new follow from those sums without another reduction. Every
// wave then solves the small Schur system S v = u on its own (same inputs,
// same order, identical results), so no wave waits on a serial section.
//
// B G^-1 r' vanishes up to rounding (the set-up's Schur matrix is formed
// with the same G^-1, the band factors included, to the last bit); it is
// folded in every ZPERIOD iterations.
constexpr int ZPERIOD = 16;

// S sub-blocks per axis, so m = N S^2 constraint rows and sub-blocks of
// NC / S level elements spanning NC / (S RPT) bands.
// Elimination factors of the cyclic reduction over NC lanes, per band: at
// stride s the factor on the value s lanes below (lanes s..NC-1) and the one
// on the value s lanes above (lanes 0..NC-1-s).
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }
template <int NC>
constexpr int pcr_per_band() { return 2 * (NC * ilog2(NC) - (NC - 1)); }
// Offset of stride 2^k's factors within a band's block (the set-up's
// pcr_offset, which takes a run-time width; this form leaves the kernel's
// LDS addressing to fold into immediate offsets).
template <int NC>
constexpr int pcr_step_offset(int k) {
  int o = 0;
  for (int q = 0; q < k; ++q) o += 2 * (NC - (1 << q));
  return o;
}
static_assert(pcr_step_offset<64>(5) == pcr_offset(64, 5) && pcr_per_band<64>() == pcr_offset(64, 6) &&
                  pcr_step_offset<16>(3) == pcr_offset(16, 3) && pcr_per_band<16>() == pcr_offset(16, 4),
              "the kernel's and the set-up's factor layouts agree");

// At least two waves per SIMD: a workgroup of fewer than eight waves would
// otherwise let the compiler spend the whole register file on one wave.
template <int NC, int RPT, int N, bool GAL, int S, bool PRE, int SB>
__global__ __launch_bounds__(NC* NC / RPT) __attribute__((amdgpu_waves_per_eu(2))) void k_solve2d(CellArgs a) {
  constexpr int NT = NC * NC / RPT;
  constexpr int NW = NT / 64;
  constexpr int NB = NC / RPT;
  constexpr int PW = NC + 2;
  constexpr bool BIG = kBig<NC, GAL>;
  constexpr int HB = RPT / SB;                 // node rows per sub-band of the correction
  constexpr bool XG = BIG && SB > 1;           // iterate in the output array, not LDS
  static_assert(SB == 1 || (PRE && RPT % SB == 0), "sub-bands need the band correction");
  constexpr int m = N * S * S, s = S, sbw = NC / S, NBS = NB / S;
  static_assert(NC % S == 0 && sbw % RPT == 0 && m <= 64, "unsupported cell shape");
  extern __shared__ double smem[];
  const int M = a.M;
  // Schur rows: lane (k, jj) = (lane / J, lane % J) takes columns jj + J t,
  // t < MS; S^-1 and u are zero-padded to MS J columns so the loop needs no
  // bounds test.
  constexpr int J = schur_lanes(m), MS = (m + J - 1) / J, UST = MS * J;
  double* pS = smem;                        // PW*PW, ring of zeros
  double* red = pS + PW * PW;               // 4*NW
  double* part = red + 4 * NW;              // [vec][iy][qx][j][band]: 2*2*s*N*NB
  double* sinvL = part + NB * 4 * s * N;    // MS*64, lane-major S^-1
  double* cwS = sinvL + MS * 64;            // m
  double* uW = cwS + m;                     // NW*UST per-wave right-hand side
  double* vW = uW + NW * UST;               // NW*m per-wave v*cw
  double* kS = vW + NW * m;                 // BIG: (NC+1)^2 kappa/6, ring of zeros at -1
  double* xS = kS + (NC + 1) * (NC + 1);    // BIG (not XG): NC*NC iterate
  double* pcr = BIG ? (XG ? xS : xS + NC * NC) : kS;  // PRE: NB SB pcr_per_band<NC>() elimination factors

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = tid % NC, band = tid / NC, y0 = band * RPT;
  // The M right-hand sides of a cell read the same kappa and label window
  // (or Galerkin stencils). Workgroups are numbered so that they land on one
  // XCD and share its L2: in a group of kXcds cells (kXcds M workgroups),
  // workgroup b takes cell b mod kXcds of the group and right-hand side
  // (b mod kXcds M) / kXcds. The cells after the last whole group (fewer
  // than kXcds) take their workgroups in plain order, so the grid is exactly
  // count M workgroups.
  int cl, alpha;
  {
    // cells in whole XCD groups (none when the numbering is off)
    const int grouped = a.xcd_groups ? (a.count / kXcds) * kXcds : 0;
    const int whole = grouped * M;
    const int b = blockIdx.x;
    if (b < whole) {
      const int grp = b / (kXcds * M), rb = b % (kXcds * M);
      cl = grp * kXcds + rb % kXcds;
      alpha = rb / kXcds;
    } else {
      cl = grouped + (b - whole) / M;
      alpha = (b - whole) % M;
    }
  }
  const int ci = a.ci0 + cl;
  const int p = a.cells[ci];
  // the iterate of node row i of the thread's column: LDS (BIG), or the
  // output array itself (XG; its row and column NC stay the zero boundary)
  double* const xg = a.out + ((size_t)ci * M + alpha) * (size_t)(NC + 1) * (NC + 1);
  auto xat = [&](int i) -> double& {
    if constexpr (XG)
      return xg[(size_t)(y0 + i) * (NC + 1) + c];
    else
      return xS[(y0 + i) * NC + c];
  };
  const int jx = p % a.n_macro, jy = p / a.n_macro;
  const int ox = a.H * jx + a.H / 2 - a.nc / 2, oy = a.H * jy + a.H / 2 - a.nc / 2;
  const bool split0 = (y0 > 0) && (y0 % sbw == 0);
  const bool anysplit = __ballot(split0) != 0;
  const int qxL = (c > 0 ? c - 1 : 0) / sbw, qxR = c / sbw;
  const int qyU = y0 / sbw, qyL = (y0 > 0 ? y0 - 1 : 0) / sbw;
  const int nn1 = a.nc + 1;

  for (int k = tid; k < PW * PW; k += NT) pS[k] = 0.0;
  for (int k = tid; k < MS * 64; k += NT) {
    const int t = k / 64, L = k % 64, row = L / J, col = L % J + J * t;
    sinvL[k] = (row < m && col < m) ? a.sinv[(size_t)p * m * m + row * m + col] : 0.0;
  }
  for (int k = tid; k < m; k += NT) cwS[k] = a.cw[(size_t)p * m + k];

  // Row c of the (sub-)band matrices T_b (PRE): diagonal Td = T[c][c],
  // Tc = T[c][c+1], one pair per sub-band.
  double Td[SB], Tc[SB];
#pragma unroll
  for (int b = 0; b < SB; ++b) Td[b] = Tc[b] = 0.0;
  // Adds node row i's K_n entries (centre, north, south, east, north-east,
  // south-east) between free nodes of its sub-band to Td and Tc.
  auto band_row = [&](int i, double cen, double nor, double sou, double eas, double ne, double se) {
    const int y = y0 + i, ib = i % HB, sb = i / HB;
    const bool fr = (c >= 1) && (y >= 1);
    const bool frE = (c + 1 <= NC - 1) && (y >= 1);
    const bool upIn = (ib + 1 < HB), dnIn = (ib >= 1) && (y - 1 >= 1);
    if (fr) band_row_add(Td[sb], Tc[sb], frE, upIn, dnIn, cen, nor, sou, eas, ne, se);
  };

  // ---- per-node operator data in registers --------------------------------
  double kq[(GAL || BIG) ? 1 : 2][(GAL || BIG) ? 1 : RPT + 1];
  double W[GAL ? RPT : 1][GAL ? 9 : 1];
  double Dinv[RPT];
  // Constraint weights (exact in binary32) per side, node row and continuum.
  // Every continuum is accumulated explicitly: deriving one from the total
  // would cancel badly, since D^-1-scaled values differ by the contrast.
  constexpr int NJ = N;
  float w[2][RPT][NJ];
  float wlo[2][NJ];     // lower quadrants of node row 0 when the band starts a sub-block row
#pragma unroll
  for (int sd = 0; sd < 2; ++sd) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) wlo[sd][j] = 0.0f;
  }
  if constexpr (!GAL) {
    int lab[2][RPT + 1];
    double kl[2][RPT + 1];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int i = 0; i <= RPT; ++i) {
        const int ex = c - 1 + sd, ey = y0 - 1 + i;
        const bool ok = ex >= 0 && ey >= 0;
        const size_t e = (size_t)wrap1(oy + ey, a.n) * a.n + wrap1(ox + ex, a.n);
        kl[sd][i] = ok ? a.kappa[e] * (1.0 / 6.0) : 0.0;
        lab[sd][i] = ok ? (int)a.label[e] : 255;
        if constexpr (!BIG) kq[sd][i] = kl[sd][i];
      }
    if constexpr (BIG) {
      for (int k = tid; k < (NC + 1) * (NC + 1); k += NT) {
        const int ex = k % (NC + 1) - 1, ey = k / (NC + 1) - 1;
        const size_t e = (size_t)wrap1(oy + ey, a.n) * a.n + wrap1(ox + ex, a.n);
        kS[k] = (ex >= 0 && ey >= 0) ? a.kappa[e] * (1.0 / 6.0) : 0.0;
      }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const bool fr = (c >= 1) && (y0 + i >= 1);
      const double ksum = kl[0][i] + kl[1][i] + kl[0][i + 1] + kl[1][i + 1];
      Dinv[i] = fr ? 1.0 / (4.0 * ksum) : 0.0;
      if constexpr (PRE) {
        double k6[6];
        fine_stencil6(kl[0][i], kl[1][i], kl[0][i + 1], kl[1][i + 1], k6);
        band_row(i, k6[0], k6[1], k6[2], k6[3], k6[4], k6[5]);
      }
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const float up = (lab[sd][i + 1] == j) ? 1.0f : 0.0f;
          const float lo = (lab[sd][i] == j) ? 1.0f : 0.0f;
          if (i == 0 && split0) {
            w[sd][i][j] = fr ? up : 0.0f;
            wlo[sd][j] = fr ? lo : 0.0f;
          } else {
            w[sd][i][j] = fr ? up + lo : 0.0f;
          }
        }
    }
  } else {
    const double* nW = a.nodeW + (size_t)ci * (NC + 1) * (NC + 1) * 9;
    const float* nB = a.nodeB + (size_t)ci * (NC + 1) * (NC + 1) * 4 * N;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int nd = (y0 + i) * (NC + 1) + c;
      const bool fr = (c >= 1) && (y0 + i >= 1);
#pragma unroll
      for (int k = 0; k < 9; ++k) W[i][k] = fr ? nW[nd * 9 + k] : 0.0;
      Dinv[i] = fr ? 1.0 / W[i][4] : 0.0;
      if constexpr (PRE) band_row(i, W[i][4], W[i][7], W[i][1], W[i][5], W[i][8], W[i][2]);
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const float lo = fr ? nB[((nd * 4) + sd * 2 + 0) * N + j] : 0.0f;
          const float up = fr ? nB[((nd * 4) + sd * 2 + 1) * N + j] : 0.0f;
          if (i == 0 && split0) {
            w[sd][i][j] = up;
            wlo[sd][j] = lo;
          } else {
            w[sd][i][j] = up + lo;
          }
        }
    }
  }

  // ---- band coarse correction: T_b and its cyclic-reduction factors ---------
  // Lane c of a band holds row c of T_b: the sum of the K_n entries between
  // the free nodes of its node column and those of columns c and c + 1 in the
  // band's rows. Column 0 is the Dirichlet boundary: an identity row.
  constexpr int LOGNC = ilog2(NC);
  double pcr_ib[SB];  // 1 / the final pivot of the lane's row, per sub-band
#pragma unroll
  for (int b = 0; b < SB; ++b) pcr_ib[b] = 0.0;
  if constexpr (PRE) {
#pragma unroll
    for (int b = 0; b < SB; ++b) {
      double td = Td[b], tc = Tc[b];
      if (c == 0) {
        td = 1.0;
        tc = 0.0;
      }
      double Ta = __shfl_up(tc, 1, NC);  // T[c][c-1] = T[c-1][c]
      if (c == 0) Ta = 0.0;
      double* blk = pcr + (size_t)(band * SB + b) * pcr_per_band<NC>();
      pcr_ib[b] = pcr_factor(c, NC, LOGNC, Ta, td, tc, [&](int k, bool hasL, bool hasR, double al, double ga) {
        double* stp = blk + pcr_step_offset<NC>(k);
        const int st = 1 << k;
        if (hasL) stp[c - st] = al;
        if (hasR) stp[(NC - st) + c] = ga;
      });
    }
  }

  // ---- building blocks -------------------------------------------------------
  // A constraint weight widened to binary64. With three continua the widened
  // copies would take 2*RPT*N double registers for the whole solve, so there
  // the binary32 value is made opaque at its point of use (the empty asm) and
  // widened there; with fewer continua the compiler's hoisting is cheaper.
  auto wide = [](float v) -> double {
    if constexpr (N >= 3) asm volatile("" : "+v"(v));
    return (double)v;
  };

  auto P_at = [&](int xx, int yy) -> double { return pS[(yy + 1) * PW + xx + 1]; };

  // out = G^-1 v on the thread's nodes: D^-1 v, plus (PRE) the band coarse
  // correction Z_b T_b^-1 Z_b^T v, whose value is one per node column: the
  // column sum of v over the band's free nodes, reduced across the band's
  // lanes by the stored elimination factors and scaled by the final pivot.
  // The same for two vectors at once: their reductions interleave, so the
  // cross-lane latency is paid once.
  auto apply_G2 = [&](const double (&v)[RPT], double (&out)[RPT], const double (&v2)[RPT], double (&out2)[RPT]) {
    if constexpr (PRE) {
      double d[SB], d2[SB];
#pragma unroll
      for (int b = 0; b < SB; ++b) d[b] = d2[b] = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        d[i / HB] += (Dinv[i] != 0.0) ? v[i] : 0.0;
        d2[i / HB] += (Dinv[i] != 0.0) ? v2[i] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < LOGNC; ++k) {
        const int st = 1 << k;
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          const double* stp = pcr + (size_t)(band * SB + b) * pcr_per_band<NC>() + pcr_step_offset<NC>(k);
          const double dL = __shfl_up(d[b], st, NC), dR = __shfl_down(d[b], st, NC);
          const double dL2 = __shfl_up(d2[b], st, NC), dR2 = __shfl_down(d2[b], st, NC);
          const double al = (c >= st) ? stp[c - st] : 0.0;
          const double ga = (c + st < NC) ? stp[(NC - st) + c] : 0.0;
          d[b] = pcr_rhs(d[b], al, dL, ga, dR);
          d2[b] = pcr_rhs(d2[b], al, dL2, ga, dR2);
        }
      }
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const double y = d[i / HB] * pcr_ib[i / HB], y2 = d2[i / HB] * pcr_ib[i / HB];
        out[i] = Dinv[i] * v[i] + ((Dinv[i] != 0.0) ? y : 0.0);
        out2[i] = Dinv[i] * v2[i] + ((Dinv[i] != 0.0) ? y2 : 0.0);
      }
    } else {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        out[i] = Dinv[i] * v[i];
        out2[i] = Dinv[i] * v2[i];
      }
    }
  };

  auto apply_G = [&](const double (&v)[RPT], double (&out)[RPT]) {
    if constexpr (PRE) {
      double d[SB];
#pragma unroll
      for (int b = 0; b < SB; ++b) d[b] = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) d[i / HB] += (Dinv[i] != 0.0) ? v[i] : 0.0;
#pragma unroll
      for (int k = 0; k < LOGNC; ++k) {
        const int st = 1 << k;
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          const double* stp = pcr + (size_t)(band * SB + b) * pcr_per_band<NC>() + pcr_step_offset<NC>(k);
          const double dL = __shfl_up(d[b], st, NC), dR = __shfl_down(d[b], st, NC);
          const double al = (c >= st) ? stp[c - st] : 0.0;
          const double ga = (c + st < NC) ? stp[(NC - st) + c] : 0.0;
          d[b] = pcr_rhs(d[b], al, dL, ga, dR);
        }
      }
#pragma unroll
      for (int i = 0; i < RPT; ++i) out[i] = Dinv[i] * v[i] + ((Dinv[i] != 0.0) ? d[i / HB] * pcr_ib[i / HB] : 0.0);
    } else {
#pragma unroll
      for (int i = 0; i < RPT; ++i) out[i] = Dinv[i] * v[i];
    }
  };

  // y = K_n v on the thread's nodes (own values in vv, neighbours from pS).
  auto apply_K = [&](const double (&vv)[RPT], double (&yv)[RPT]) {
    double Lc[RPT + 2], Rc[RPT + 2];
    const double Cb = P_at(c, y0 - 1), Ct = P_at(c, y0 + RPT);
#pragma unroll
    for (int i = 0; i < RPT + 2; ++i) {
      Lc[i] = P_at(c - 1, y0 - 1 + i);
      Rc[i] = P_at(c + 1, y0 - 1 + i);
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const double pC = vv[i];
      const double pSo = i == 0 ? Cb : vv[i - 1];
      const double pN = i == RPT - 1 ? Ct : vv[i + 1];
      if constexpr (!GAL) {
        double kSW, kSE, kNW, kNE;
        if constexpr (BIG) {
          const double* kr0 = kS + (y0 + i) * (NC + 1) + c;
          kSW = kr0[0];
          kSE = kr0[1];
          kNW = kr0[NC + 1];
          kNE = kr0[NC + 2];
        } else {
          kSW = kq[0][i];
          kSE = kq[1][i];
          kNW = kq[0][i + 1];
          kNE = kq[1][i + 1];
        }
        const double aS = kSW + kSE, aN = kNW + kNE, aW = kSW + kNW, aE = kSE + kNE;
        double t = 4.0 * (aS + aN) * pC;
        t -= aS * pSo + aN * pN + aW * Lc[i + 1] + aE * Rc[i + 1];
        t -= 2.0 * (kSW * Lc[i] + kSE * Rc[i] + kNW * Lc[i + 2] + kNE * Rc[i + 2]);
        yv[i] = t;
      } else {
        const double* Wi = W[i];
        double t = Wi[4] * pC;
        t += Wi[1] * pSo + Wi[7] * pN + Wi[3] * Lc[i + 1] + Wi[5] * Rc[i + 1];
        t += Wi[0] * Lc[i] + Wi[2] * Rc[i] + Wi[6] * Lc[i + 2] + Wi[8] * Rc[i + 2];
        yv[i] = t;
      }
    }
  };

  // Band partials of B_n tv (no row normalisation) into part[vec][..][band]. The
  // segment sums of all continua (and of the lower quadrants where a band
  // starts a sub-block row) go through the DPP steps together.
  auto accumulate_B = [&](const double (&tv)[RPT], int vec) {
    double v[2 * N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double up[2];
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) acc += wide(w[sd][i][j]) * tv[i];
        up[sd] = acc;
      }
      // element column c collects side 1 of lane c and side 0 of lane c+1
      v[j] = up[1] + from_right(up[0], c, NC);
    }
    if (anysplit) {
#pragma unroll
      for (int j = 0; j < N; ++j)
        v[N + j] = wide(wlo[1][j]) * tv[0] + from_right(wide(wlo[0][j]) * tv[0], c, NC);
      seg_sum_n<2 * N>(v, sbw);
    } else {
      double vu[N];
#pragma unroll
      for (int j = 0; j < N; ++j) vu[j] = v[j];
      seg_sum_n<N>(vu, sbw);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        v[j] = vu[j];
        v[N + j] = 0.0;
      }
    }
    if (c % sbw == 0) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        part[(((vec * 2 + 1) * s + c / sbw) * N + j) * NB + band] = v[j];
        part[(((vec * 2 + 0) * s + c / sbw) * N + j) * NB + band] = v[N + j];
      }
    }
  };

  // Row k = lane (lanes < m) of B_n applied to vector vec: the sum over the
  // NBS bands of its sub-block row (fixed order) plus the lower-quadrant part
  // of the next band, without cw. A row's band partials are contiguous.
  const int zk = lane < m ? lane : 0;
  const int zq = zk / N, zj = zk % N, zqx = zq % S, zqy = zq / S;
  const int zrow = (zqx * N + zj) * NB + zqy * NBS;
  const int zlow = zqy < S - 1 ? zrow + NBS : zrow;
  auto zsum = [&](int vec) -> double {
    const double* up = part + (vec * 2 + 1) * S * N * NB + zrow;
    double z = 0.0;
#pragma unroll
    for (int b = 0; b < NBS; ++b) z += up[b];
    const double lo = part[(vec * 2 + 0) * S * N * NB + zlow];
    return z + (zqy < S - 1 ? lo : 0.0);
  };

  // Per wave: v = S^-1 u for u in uW[wave]; vW[wave] = v*cw; returns v.u (all
  // lanes) and, for the lane holding row k (lane = k*J), v_k in *vk. v.u is
  // summed from the lanes' partial row products, alongside the row sums.
  auto wave_schur = [&](double* vk) -> double {
    __builtin_amdgcn_wave_barrier();
    const int k = lane / J, jj = lane % J;
    const double* u = uW + wave * UST;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    constexpr int MS4 = MS / 4 * 4;
#pragma unroll 4
    for (int t0 = 0; t0 < MS4; t0 += 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) a4[q] += sinvL[(t0 + q) * 64 + lane] * u[jj + J * (t0 + q)];
    }
#pragma unroll
    for (int t = MS4; t < MS; ++t) a4[t - MS4] += sinvL[t * 64 + lane] * u[jj + J * t];
    double sum = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    const double uk = u[k < m ? k : 0];
    double pu = k < m ? uk * sum : 0.0;
    sum = seg_sum(sum, J);
    *vk = 0.0;
    if (k < m && jj == 0) {
      *vk = sum;
      vW[wave * m + k] = sum * cwS[k];
    }
    pu = wave_sum(pu);
    __builtin_amdgcn_wave_barrier();
    return pu;
  };

  // tv += sign * B_n^T v for v*cw in vW[wave].
  auto scatter_B = [&](double (&tv)[RPT], double sign) {
    const double* vv = vW + wave * m;
    double vs[2][2][N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      vs[0][1][j] = vv[(qyU * s + qxL) * N + j];
      vs[1][1][j] = vv[(qyU * s + qxR) * N + j];
      vs[0][0][j] = vv[(qyL * s + qxL) * N + j];
      vs[1][0][j] = vv[(qyL * s + qxR) * N + j];
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      double t = 0.0;
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int j = 0; j < N; ++j) t += wide(w[sd][i][j]) * vs[sd][1][j];
      if (i == 0) {
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
          for (int j = 0; j < N; ++j) t += wide(wlo[sd][j]) * vs[sd][0][j];
      }
      tv[i] += sign * t;
    }
  };

  // ---- right-hand side -------------------------------------------------------
  double f[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) f[i] = 0.0;
  const int k0 = (a.nc - a.H) / 2;  // first fine node of K_p
  double* uw = uW + wave * UST;
  if (!a.adjoint) {
    if constexpr (GAL) {
      const double* fi = a.fin + ((size_t)ci * M + alpha) * (NC + 1) * (NC + 1);
#pragma unroll
      for (int i = 0; i < RPT; ++i) f[i] = fi[(y0 + i) * (NC + 1) + c];
      for (int k = lane; k < UST; k += 64) uw[k] = k < m ? a.gin[((size_t)ci * M + alpha) * m + k] : 0.0;
    } else {
      for (int k = lane; k < UST; k += 64) uw[k] = k < m ? a.g[((size_t)p * M + alpha) * m + k] : 0.0;
    }
  } else {
    // adjoint: f = P^T Phibar, g' = 0
    const double* skp = a.seed_kp + ((size_t)p * M + alpha) * (size_t)((a.H + 1) * (a.H + 1));
    const int rr = a.r;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int X = c, Y = y0 + i;
      double t = 0.0;
      if (X >= 1 && Y >= 1) {
        // the hat's support clipped to the K_p nodes (often empty)
        const int du0 = max(-(rr - 1), k0 - X * rr), du1 = min(rr - 1, k0 + a.H - X * rr);
        const int dv0 = max(-(rr - 1), k0 - Y * rr), dv1 = min(rr - 1, k0 + a.H - Y * rr);
        for (int dv = dv0; dv <= dv1; ++dv)
          for (int du = du0; du <= du1; ++du) {
            const int fx = X * rr + du - k0, fy = Y * rr + dv - k0;
            const double wgt = (1.0 - fabs((double)du) / rr) * (1.0 - fabs((double)dv) / rr);
            t += wgt * skp[fy * (a.H + 1) + fx];
          }
        if (a.seed_par != nullptr) {
          // seeds from the cells that inherit from this one, on all fine nodes
          const double* sp = a.seed_par + ((size_t)a.slot[p] * M + alpha) * (size_t)(nn1 * nn1);
          if (rr == 1) {
            t += sp[(size_t)Y * nn1 + X];
          } else {
            for (int dv = -(rr - 1); dv <= rr - 1; ++dv)
              for (int du = -(rr - 1); du <= rr - 1; ++du) {
                const double wgt = (1.0 - fabs((double)du) / rr) * (1.0 - fabs((double)dv) / rr);
                t += wgt * sp[(size_t)(Y * rr + dv) * nn1 + X * rr + du];
              }
          }
        }
      }
      f[i] = t;
    }
    for (int k = lane; k < UST; k += 64) uw[k] = 0.0;
  }
  __syncthreads();  // sinvL, cwS, kS visible
  const double zcw = lane < m ? cwS[lane] : 0.0;

  // ---- feasible start x0 = G^-1 B^T S^-1 g' ---------------------------------
  double x[RPT], r[RPT], t[RPT], pv[RPT];
  double Vacc = 0.0, vk = 0.0;
  (void)wave_schur(&vk);
#pragma unroll
  for (int i = 0; i < RPT; ++i) x[i] = 0.0;
  scatter_B(x, 1.0);
  {
    double bt[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) bt[i] = x[i];
    apply_G(bt, x);
  }
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    pS[(y0 + i + 1) * PW + c + 1] = x[i];
    if constexpr (BIG) xat(i) = x[i];
  }
  __syncthreads();
  apply_K(x, r);
  double s_rr = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) r[i] -= f[i];
  apply_G(r, t);
#pragma unroll
  for (int i = 0; i < RPT; ++i) s_rr += r[i] * t[i];
  accumulate_B(t, 0);
  s_rr = wave_sum(s_rr);
  if (lane == 0) red[wave * 4] = s_rr;
  __syncthreads();
  const double rr = tree_sum<NW, 4>(red);
  if (lane < m) uw[lane] = zcw * zsum(0);
  double vu = wave_schur(&vk);
  Vacc = vk;
  double rz = rr - vu;
  const double rz0 = rz;
  scatter_B(r, -1.0);
  apply_G(r, t);
#pragma unroll
  for (int i = 0; i < RPT; ++i) pv[i] = -t[i];
  __syncthreads();  // everyone done reading pS (x0) and part
#pragma unroll
  for (int i = 0; i < RPT; ++i) pS[(y0 + i + 1) * PW + c + 1] = pv[i];
  __syncthreads();

  const double tol2 = a.rtol * a.rtol * rz0;
  int it = 0;
  bool done = !(rz0 > 0.0);
  while (!done) {
    // t = G^-1 r' is kept from the end of the previous iteration where the
    // band correction makes G^-1 costly (its cyclic reductions outweigh the
    // registers t holds through the two barriers: level-1 solve 0.572 ->
    // 0.528 ms on the 512^2 workload, 67.4 -> 63.7 ms on the 2048^2 one);
    // with D alone it is formed again beside G^-1 Ap, which frees them
    double Ap[RPT], tA[RPT];
    apply_K(pv, Ap);
    if constexpr (PRE)
      apply_G(Ap, tA);
    else
      apply_G2(r, t, Ap, tA);
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      s4[0] += pv[i] * Ap[i];
      s4[1] += r[i] * t[i];
      s4[2] += t[i] * Ap[i];
      s4[3] += Ap[i] * tA[i];
    }
    // B G^-1 r' is folded in periodically (see ZPERIOD), which keeps the
    // constraint residual at rounding level.
    const bool withz0 = (it % ZPERIOD) == 0;
    if (withz0) accumulate_B(t, 0);
    accumulate_B(tA, 1);
    wave_sum_n<4>(s4);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) red[wave * 4 + q] = s4[q];
    }
    __syncthreads();
    // B_n G^-1 Ap and the wave partials are read together; only the final
    // combination waits for alpha. 1/rrk is formed off the critical path.
    const double z1 = zsum(1);
    const double z0 = withz0 ? zsum(0) : 0.0;
    const double pAp = tree_sum<NW, 4>(red + 0), rrk = tree_sum<NW, 4>(red + 1);
    const double rA = tree_sum<NW, 4>(red + 2), AA = tree_sum<NW, 4>(red + 3);
    const double irr = 1.0 / rrk;
    const double al = rrk / pAp;
    const double rDr = rrk + 2.0 * al * rA + al * al * AA;
    if (lane < m) uw[lane] = zcw * (z0 + al * z1);
    vu = wave_schur(&vk);
    Vacc += vk;
    const double rzn = rDr - vu;
    ++it;
    if (rzn <= tol2 || it >= a.max_iter) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if constexpr (BIG)
          xat(i) += al * pv[i];
        else
          x[i] += al * pv[i];
      }
      rz = rzn;
      break;
    }
    const double be = rzn * irr;
    rz = rzn;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      if constexpr (BIG)
        xat(i) += al * pv[i];
      else
        x[i] += al * pv[i];
      r[i] += al * Ap[i];
    }
    scatter_B(r, -1.0);
    apply_G(r, t);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      pv[i] = -t[i] + be * pv[i];
      pS[(y0 + i + 1) * PW + c + 1] = pv[i];
    }
    __syncthreads();
  }

  // ---- final projection onto B_n x = g' -------------------------------------
  // The directions keep the iterate feasible only up to the accuracy of S^-1
  // and the rounding of each projection; one correction
  // x -= D^-1 B_n^T S^-1 (B_n x - g') brings the constraint residual back to
  // rounding level (x -= G^-1 B_n^T S^-1 (B_n x - g')). Every wave leaves the loop in the same iteration, and the
  // barrier keeps the band partials until every wave has read them.
  {
    double xr[RPT], tc[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      if constexpr (BIG)
        xr[i] = xat(i);
      else
        xr[i] = x[i];
      tc[i] = 0.0;
    }
    __syncthreads();
    accumulate_B(xr, 0);
    __syncthreads();
    if (lane < m) {
      double gk = 0.0;
      if (!a.adjoint) {
        if constexpr (GAL)
          gk = a.gin[((size_t)ci * M + alpha) * m + lane];
        else
          gk = a.g[((size_t)p * M + alpha) * m + lane];
      }
      uw[lane] = zcw * zsum(0) - gk;
    }
    (void)wave_schur(&vk);
    scatter_B(tc, 1.0);
    double gc[RPT];
    apply_G(tc, gc);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      if constexpr (BIG)
        xat(i) = xr[i] - gc[i];
      else
        x[i] = xr[i] - gc[i];
    }
  }

  // ---- outputs ---------------------------------------------------------------
  const size_t vec = (size_t)(NC + 1) * (NC + 1);
  double* dst = a.out + ((size_t)ci * M + alpha) * vec;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    if constexpr (!XG) dst[(size_t)(y0 + i) * (NC + 1) + c] = BIG ? xS[(y0 + i) * NC + c] : x[i];
  }
  if (wave == 0) {
    const int k = lane / J, jj = lane % J;
    if (k < m && jj == 0) a.beta[((size_t)p * M + alpha) * m + k] = -Vacc;
  }
  if (tid == 0) {
    a.iters[(size_t)p * M + alpha] = (rz0 == rz0) ? it : -1;
    a.resid[(size_t)p * M + alpha] = rel_resid(rz, rz0);
  }
}

}  // namespace mch
