// 2D cell kernels for gfx950: constraint setup, the constrained Krylov
// solve of each cell problem, effective tensors and the adjoint.
//
// Cell problem (paper Sec. 2, Eqs. phi_avar / phi_grad; Sec. 3.3,
// Eqs. phi_avar_corrector / phi_grad_corrector): minimise the kappa-energy of
// v = I + P_n xi over the level-n Q1 space V_n of the oversampled cell,
// subject to the average constraints B_h v = g. In matrix form
//   [K_n  B_n^T][xi  ]   [ f  ]     K_n = P^T K_h P,  B_n = B_h P,
//   [B_n  0    ][beta] = [ g' ],    f = -P^T K_h I,   g' = g - B_h I.
//
// Solver: projected preconditioned CG with the constraint preconditioner
// [D B^T; B 0], D = diag(K_n) (Gould, Hribar & Nocedal 2001), including
// their residual update so the residual stays orthogonal to range(B^T).
// The iterate starts feasible (x0 = D^-1 B^T S^-1 g', S = B D^-1 B^T) and
// every direction lies in null(B), so the constraints hold to rounding.
// The accumulated projections give the multipliers.
//
// Layout inside a workgroup: one (cell, right-hand side) per workgroup; lane
// c of a band row owns node column c and element column c; each band of RPT
// node rows belongs to NC consecutive threads. Node rows/columns 0..NC-1 are
// owned, row/column NC is the Dirichlet boundary and never stored. The search
// direction p lives in LDS (padded by one ring of zeros); x, r and the
// per-node operator data live in registers.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "kernels2d.h"

namespace mch {

// Fine cells of width >= 64 keep kappa/6 and the iterate x in LDS instead of
// registers (the register file cannot hold them at 8 nodes per lane).
template <int NC, bool GAL>
constexpr bool kBig = !GAL && NC >= 64;

// One iteration of the projected PCG needs two workgroup barriers: after the
// fused reduction of (p.Ap, r.D^-1 r, r.D^-1 Ap, Ap.D^-1 Ap, B D^-1 r,
// B D^-1 Ap), and after the new search direction is written to LDS. With
// r' the projected residual, r_new = r' + alpha Ap, so both B D^-1 r_new and
// r_new.D^-1 r_new follow from those sums without another reduction. Every
// wave then solves the small Schur system S v = u on its own (same inputs,
// same order, identical results), so no wave waits on a serial section.
constexpr int ZPERIOD = 16;

template <int NC, int RPT, int N, bool GAL>
__global__ __launch_bounds__(NC* NC / RPT) void k_solve2d(CellArgs a) {
  constexpr int NT = NC * NC / RPT;
  constexpr int NW = NT / 64;
  constexpr int NB = NC / RPT;
  constexpr int PW = NC + 2;
  constexpr bool BIG = kBig<NC, GAL>;
  extern __shared__ double smem[];
  const int m = a.m, s = a.s, M = a.M, sbw = a.sbw, J = a.J;
  const int MS = (m + J - 1) / J;
  double* pS = smem;                        // PW*PW, ring of zeros
  double* red = pS + PW * PW;               // 4*NW
  double* part = red + 4 * NW;              // [band][vec][iy][qx][j]: NB*2*2*s*N
  double* sinvL = part + NB * 4 * s * N;    // MS*64, lane-major S^-1
  double* cwS = sinvL + MS * 64;            // m
  double* uW = cwS + m;                     // NW*m per-wave right-hand side
  double* vW = uW + NW * m;                 // NW*m per-wave v*cw
  double* kS = vW + NW * m;                 // BIG: (NC+1)^2 kappa/6, ring of zeros at -1
  double* xS = kS + (NC + 1) * (NC + 1);    // BIG: NC*NC iterate

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = tid % NC, band = tid / NC, y0 = band * RPT;
  const int ci = a.ci0 + blockIdx.x / M, alpha = blockIdx.x % M;
  const int p = a.cells[ci];
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
        const size_t e = (size_t)wrapi(oy + ey, a.n) * a.n + wrapi(ox + ex, a.n);
        kl[sd][i] = ok ? a.kappa[e] * (1.0 / 6.0) : 0.0;
        lab[sd][i] = ok ? (int)a.label[e] : 255;
        if constexpr (!BIG) kq[sd][i] = kl[sd][i];
      }
    if constexpr (BIG) {
      for (int k = tid; k < (NC + 1) * (NC + 1); k += NT) {
        const int ex = k % (NC + 1) - 1, ey = k / (NC + 1) - 1;
        const size_t e = (size_t)wrapi(oy + ey, a.n) * a.n + wrapi(ox + ex, a.n);
        kS[k] = (ex >= 0 && ey >= 0) ? a.kappa[e] * (1.0 / 6.0) : 0.0;
      }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const bool fr = (c >= 1) && (y0 + i >= 1);
      const double ksum = kl[0][i] + kl[1][i] + kl[0][i + 1] + kl[1][i + 1];
      Dinv[i] = fr ? 1.0 / (4.0 * ksum) : 0.0;
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
    const double* nW = a.nodeW + (size_t)ci * NC * NC * 9;
    const float* nB = a.nodeB + (size_t)ci * NC * NC * 4 * N;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int nd = (y0 + i) * NC + c;
      const bool fr = (c >= 1) && (y0 + i >= 1);
#pragma unroll
      for (int k = 0; k < 9; ++k) W[i][k] = fr ? nW[nd * 9 + k] : 0.0;
      Dinv[i] = fr ? 1.0 / W[i][4] : 0.0;
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

  // ---- building blocks -------------------------------------------------------
  auto P_at = [&](int xx, int yy) -> double { return pS[(yy + 1) * PW + xx + 1]; };

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

  // Band partials of B_n tv (no row normalisation) into part[band][vec].
  auto accumulate_B = [&](const double (&tv)[RPT], int vec) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double up[2];
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) acc += (double)w[sd][i][j] * tv[i];
        up[sd] = acc;
      }
      // element column c collects side 1 of lane c and side 0 of lane c+1
      const double v = seg_sum(up[1] + from_right(up[0], c, NC), sbw);
      if (c % sbw == 0) part[(((band * 2 + vec) * 2 + 1) * s + c / sbw) * N + j] = v;
      double vl = 0.0;
      if (anysplit) vl = seg_sum((double)wlo[1][j] * tv[0] + from_right((double)wlo[0][j] * tv[0], c, NC), sbw);
      if (c % sbw == 0) part[(((band * 2 + vec) * 2 + 0) * s + c / sbw) * N + j] = vl;
    }
  };

  // Row k of B_n (vector vec) summed over the bands (fixed order), without cw.
  auto zsum = [&](int vec, int k) -> double {
    const int q = k / N, j = k % N, qx = q % s, qy = q / s;
    const int b0 = qy * sbw / RPT, b1 = (qy + 1) * sbw / RPT;
    double z = 0.0;
#pragma unroll 4
    for (int b = b0; b < b1; ++b) z += part[(((b * 2 + vec) * 2 + 1) * s + qx) * N + j];
    if (b1 < NB) z += part[(((b1 * 2 + vec) * 2 + 0) * s + qx) * N + j];
    return z;
  };

  // Per wave: v = S^-1 u for u in uW[wave]; vW[wave] = v*cw; returns v.u (all lanes)
  // and, for the lane holding row k (lane = k*J), v_k in *vk.
  auto wave_schur = [&](double* vk) -> double {
    __builtin_amdgcn_wave_barrier();
    const int k = lane / J, jj = lane % J;
    const double* u = uW + wave * m;
    double sum = 0.0;
#pragma unroll 8
    for (int t = 0; t < MS; ++t) {
      const int j = jj + J * t;
      if (j < m) sum += sinvL[t * 64 + lane] * u[j];
    }
    sum = seg_sum(sum, J);
    double vu = 0.0;
    *vk = 0.0;
    if (k < m && jj == 0) {
      *vk = sum;
      vW[wave * m + k] = sum * cwS[k];
      vu = sum * u[k];
    }
    __builtin_amdgcn_wave_barrier();
    return wave_sum(vu);
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
        for (int j = 0; j < N; ++j) t += (double)w[sd][i][j] * vs[sd][1][j];
      if (i == 0) {
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
          for (int j = 0; j < N; ++j) t += (double)wlo[sd][j] * vs[sd][0][j];
      }
      tv[i] += sign * t;
    }
  };

  // ---- right-hand side -------------------------------------------------------
  double f[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) f[i] = 0.0;
  const int k0 = (a.nc - a.H) / 2;  // first fine node of K_p
  double* uw = uW + wave * m;
  if (!a.adjoint) {
    if constexpr (GAL) {
      const double* fi = a.fin + ((size_t)ci * M + alpha) * NC * NC;
#pragma unroll
      for (int i = 0; i < RPT; ++i) f[i] = fi[(y0 + i) * NC + c];
      for (int k = lane; k < m; k += 64) uw[k] = a.gin[((size_t)ci * M + alpha) * m + k];
    } else {
      for (int k = lane; k < m; k += 64) uw[k] = a.g[((size_t)p * M + alpha) * m + k];
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
        for (int dv = -(rr - 1); dv <= rr - 1; ++dv)
          for (int du = -(rr - 1); du <= rr - 1; ++du) {
            const int fx = X * rr + du - k0, fy = Y * rr + dv - k0;
            if (fx < 0 || fy < 0 || fx > a.H || fy > a.H) continue;
            const double wgt = (1.0 - fabs((double)du) / rr) * (1.0 - fabs((double)dv) / rr);
            t += wgt * skp[fy * (a.H + 1) + fx];
          }
        if (rr == 1 && a.seed_par != nullptr) {
          const double* sp = a.seed_par + ((size_t)a.slot[p] * M + alpha) * (size_t)(nn1 * nn1);
          t += sp[(size_t)Y * nn1 + X];
        }
      }
      f[i] = t;
    }
    for (int k = lane; k < m; k += 64) uw[k] = 0.0;
  }
  __syncthreads();  // sinvL, cwS, kS visible

  // ---- feasible start x0 = D^-1 B^T S^-1 g' ---------------------------------
  double x[RPT], r[RPT], t[RPT], pv[RPT];
  double Vacc = 0.0, vk = 0.0;
  (void)wave_schur(&vk);
#pragma unroll
  for (int i = 0; i < RPT; ++i) x[i] = 0.0;
  scatter_B(x, 1.0);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    x[i] *= Dinv[i];
    pS[(y0 + i + 1) * PW + c + 1] = x[i];
    if constexpr (BIG) xS[(y0 + i) * NC + c] = x[i];
  }
  __syncthreads();
  apply_K(x, r);
  double s_rr = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    r[i] -= f[i];
    t[i] = Dinv[i] * r[i];
    s_rr += r[i] * t[i];
  }
  accumulate_B(t, 0);
  s_rr = wave_sum(s_rr);
  if (lane == 0) red[wave * 4] = s_rr;
  __syncthreads();
  double rr = 0.0;
#pragma unroll
  for (int w2 = 0; w2 < NW; ++w2) rr += red[w2 * 4];
  for (int k = lane; k < m; k += 64) uw[k] = cwS[k] * zsum(0, k);
  double vu = wave_schur(&vk);
  Vacc = vk;
  double rz = rr - vu;
  const double rz0 = rz;
  scatter_B(r, -1.0);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    t[i] = Dinv[i] * r[i];
    pv[i] = -t[i];
  }
  __syncthreads();  // everyone done reading pS (x0) and part
#pragma unroll
  for (int i = 0; i < RPT; ++i) pS[(y0 + i + 1) * PW + c + 1] = pv[i];
  __syncthreads();

  const double tol2 = a.rtol * a.rtol * rz0;
  int it = 0;
  bool done = !(rz0 > 0.0);
  while (!done) {
    double Ap[RPT], tA[RPT];
    apply_K(pv, Ap);
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      tA[i] = Dinv[i] * Ap[i];
      s4[0] += pv[i] * Ap[i];
      s4[1] += r[i] * t[i];
      s4[2] += t[i] * Ap[i];
      s4[3] += Ap[i] * tA[i];
    }
    // B D^-1 r' vanishes up to rounding; it is folded in every ZPERIOD
    // iterations, which keeps the constraint residual at rounding level.
    const bool withz0 = (it % ZPERIOD) == 0;
    if (withz0) accumulate_B(t, 0);
    accumulate_B(tA, 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double v = wave_sum(s4[q]);
      if (lane == 0) red[wave * 4 + q] = v;
    }
    __syncthreads();
    double pAp = 0.0, rrk = 0.0, rA = 0.0, AA = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < NW; ++w2) {
      pAp += red[w2 * 4 + 0];
      rrk += red[w2 * 4 + 1];
      rA += red[w2 * 4 + 2];
      AA += red[w2 * 4 + 3];
    }
    const double al = rrk / pAp;
    const double rDr = rrk + 2.0 * al * rA + al * al * AA;
    for (int k = lane; k < m; k += 64) uw[k] = cwS[k] * ((withz0 ? zsum(0, k) : 0.0) + al * zsum(1, k));
    vu = wave_schur(&vk);
    Vacc += vk;
    const double rzn = rDr - vu;
    ++it;
    if (rzn <= tol2 || it >= a.max_iter) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if constexpr (BIG)
          xS[(y0 + i) * NC + c] += al * pv[i];
        else
          x[i] += al * pv[i];
      }
      rz = rzn;
      break;
    }
    const double be = rzn / rrk;
    rz = rzn;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      if constexpr (BIG)
        xS[(y0 + i) * NC + c] += al * pv[i];
      else
        x[i] += al * pv[i];
      r[i] += al * Ap[i];
    }
    scatter_B(r, -1.0);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      t[i] = Dinv[i] * r[i];
      pv[i] = -t[i] + be * pv[i];
      pS[(y0 + i + 1) * PW + c + 1] = pv[i];
    }
    __syncthreads();
  }

  // ---- outputs ---------------------------------------------------------------
  const size_t vec = (size_t)(NC + 1) * (NC + 1);
  double* dst = a.out + ((size_t)ci * M + alpha) * vec;
#pragma unroll
  for (int i = 0; i < RPT; ++i) dst[(size_t)(y0 + i) * (NC + 1) + c] = BIG ? xS[(y0 + i) * NC + c] : x[i];
  if (wave == 0) {
    const int k = lane / J, jj = lane % J;
    if (k < m && jj == 0) a.beta[((size_t)p * M + alpha) * m + k] = -Vacc;
  }
  if (tid == 0) {
    a.iters[(size_t)p * M + alpha] = (rz0 == rz0) ? it : -1;
    a.resid[(size_t)p * M + alpha] = (rz0 > 0.0) ? sqrt(fmax(rz, 0.0) / rz0) : 0.0;
  }
}
// ---------------------------------------------------------------------------
// Effective tensors: A[p][a][b] = sum_{e in K_p} kappa_e Phi_a|e^T K_ref Phi_b|e,
// Phi = I + P xi on the fine nodes of K_p. One workgroup per cell.
// ---------------------------------------------------------------------------
constexpr int EFF_T = 256;

template <int MM>
__global__ __launch_bounds__(EFF_T) void k_eff2d(CellArgs a, double* A) {
  extern __shared__ double sm[];
  const int H = a.H, Hp = H + 1;
  double* ph = sm;  // [MM][Hp*Hp]
  double* wr = ph + MM * Hp * Hp;  // [EFF_T/64][MM*MM]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ci = a.ci0 + blockIdx.x;
  const int p = a.cells[ci];
  const int k0 = (a.nc - H) / 2;
  for (int k = tid; k < MM * Hp * Hp; k += EFF_T) {
    const int al = k / (Hp * Hp), nd = k % (Hp * Hp);
    ph[k] = phi_at(a, ci, al, k0 + nd % Hp, k0 + nd / Hp);
  }
  __syncthreads();
  const int jx = p % a.n_macro, jy = p / a.n_macro;
  double acc[MM * (MM + 1) / 2];
#pragma unroll
  for (int k = 0; k < MM * (MM + 1) / 2; ++k) acc[k] = 0.0;
  for (int e = tid; e < H * H; e += EFF_T) {
    const int ex = e % H, ey = e / H;
    const double k6 = a.kappa[(size_t)(H * jy + ey) * a.n + (H * jx + ex)] * (1.0 / 6.0);
    double v[MM][4], y[MM][4];
#pragma unroll
    for (int al = 0; al < MM; ++al) {
#pragma unroll
      for (int d = 0; d < 4; ++d) v[al][d] = ph[al * Hp * Hp + (ey + (d >> 1)) * Hp + ex + (d & 1)];
      y[al][0] = k6 * (4 * v[al][0] - v[al][1] - v[al][2] - 2 * v[al][3]);
      y[al][1] = k6 * (-v[al][0] + 4 * v[al][1] - 2 * v[al][2] - v[al][3]);
      y[al][2] = k6 * (-v[al][0] - 2 * v[al][1] + 4 * v[al][2] - v[al][3]);
      y[al][3] = k6 * (-2 * v[al][0] - v[al][1] - v[al][2] + 4 * v[al][3]);
    }
    int k = 0;
#pragma unroll
    for (int al = 0; al < MM; ++al)
#pragma unroll
      for (int be = al; be < MM; ++be, ++k)
        acc[k] += v[al][0] * y[be][0] + v[al][1] * y[be][1] + v[al][2] * y[be][2] + v[al][3] * y[be][3];
  }
#pragma unroll
  for (int k = 0; k < MM * (MM + 1) / 2; ++k) {
    double t = wave_sum(acc[k]);
    if (lane == 0) wr[wave * MM * MM + k] = t;
  }
  __syncthreads();
  if (tid < MM * (MM + 1) / 2) {
    double t = 0.0;
    for (int w2 = 0; w2 < EFF_T / 64; ++w2) t += wr[w2 * MM * MM + tid];
    // unpack triangle index tid -> (al, be)
    int al = 0, k = tid;
    while (k >= MM - al) {
      k -= MM - al;
      ++al;
    }
    const int be = al + k;
    A[((size_t)p * MM + al) * MM + be] = t;
    A[((size_t)p * MM + be) * MM + al] = t;
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

CellArgs base_args(mch_plan* pl, const double* kappa, const uint8_t* label, int l) {
  CellArgs a{};
  const mch::Level& lv = pl->lev[l];
  a.kappa = kappa;
  a.label = label;
  a.n = pl->n;
  a.n_macro = pl->nm;
  a.H = pl->H;
  a.nc = pl->cfg.n_cell;
  a.s = pl->cfg.n_sub;
  a.N = pl->cfg.n_cont;
  a.M = pl->M;
  a.m = pl->m;
  a.h = pl->cfg.h;
  a.r = lv.r;
  a.NC = lv.NC;
  a.sbw = a.nc / a.s / lv.r;
  a.cells = lv.d_cells;
  a.pslot = lv.d_pslot;
  a.count = lv.count;
  a.cw = pl->d_cw;
  a.g = pl->d_g;
  a.sinv = pl->d_sinv;
  a.beta = pl->d_beta;
  a.iters = pl->d_iters;
  a.resid = pl->d_resid;
  a.phi1 = pl->lev[0].d_out;
  a.out = lv.d_out;
  a.tabK = lv.d_tabK;
  a.tabR = lv.d_tabR;
  a.nodeW = lv.d_nodeW;
  a.nodeB = lv.d_nodeB;
  a.fin = lv.d_fin;
  a.gin = lv.d_gin;
  a.J = 1;
  a.adjoint = 0;
  a.seed_kp = pl->d_seed_kp;
  a.seed_par = nullptr;
  a.slot = pl->d_slot;
  a.rtol = pl->cfg.rtol;
  a.max_iter = pl->cfg.max_iter;
  a.kw = lv.d_kw;
  a.labw = lv.d_labw;
  a.dinv = lv.d_dinv;
  a.vr = lv.d_vr;
  a.vp = lv.d_vp;
  a.vap = lv.d_vap;
  a.phikp = pl->d_phikp;
  return a;
}

static int schur_lanes(int m) {
  int J = 1;
  while (J * 2 * m <= 64) J *= 2;
  return J;
}

static size_t solve_lds_bytes(int NC, int rpt, int s, int N, int m, bool gal) {
  const int NT = NC * NC / rpt, NW = NT / 64, NB = NC / rpt, PW = NC + 2;
  const int J = schur_lanes(m), MS = (m + J - 1) / J;
  size_t d = (size_t)PW * PW + 4 * NW + (size_t)NB * 4 * s * N + (size_t)MS * 64 + (size_t)m + 2 * (size_t)NW * m;
  if (!gal && NC >= 64) d += (size_t)(NC + 1) * (NC + 1) + (size_t)NC * NC;
  return d * sizeof(double);
}

using SolveFn = void (*)(CellArgs);

template <int NC, int RPT, int N, bool GAL>
static int launch_solve_t(const CellArgs& a, size_t lds, hipStream_t s) {
  const int NT = NC * NC / RPT;
  auto fn = k_solve2d<NC, RPT, N, GAL>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute");
  }
  hipLaunchKernelGGL(fn, dim3(a.count * a.M), dim3(NT), lds, s, a);
  return hip_check(hipGetLastError(), "launch k_solve2d");
}

// Instantiated (cell width, node rows per thread, continua, Galerkin) shapes.
#define MCH_SHAPES(X)                                                                          \
  X(64, 4, 1, false) X(64, 4, 2, false) X(64, 4, 3, false)                                     \
  X(64, 8, 1, false) X(64, 8, 2, false) X(64, 8, 3, false)                                     \
  X(32, 4, 1, false) X(32, 4, 2, false) X(32, 4, 3, false)                                     \
  X(32, 1, 2, false) X(32, 1, 3, false) X(16, 4, 1, false) X(16, 4, 2, false) X(16, 4, 3, false) \
  X(32, 4, 1, true) X(32, 4, 2, true) X(32, 4, 3, true) X(32, 2, 2, true) X(32, 2, 3, true)    \
  X(32, 1, 2, true) X(32, 1, 3, true) X(16, 4, 1, true) X(16, 4, 2, true) X(16, 4, 3, true)    \
  X(16, 1, 2, true) X(16, 1, 3, true) X(8, 1, 1, true) X(8, 1, 2, true) X(8, 1, 3, true)

bool shape_supported_2d(int NC, int rpt, int N, bool gal) {
#define X(nc_, r_, n_, g_) \
  if (NC == nc_ && rpt == r_ && N == n_ && gal == g_) return true;
  MCH_SHAPES(X)
#undef X
  return false;
}

int launch_solve(const CellArgs& a_in, int rpt, hipStream_t s) {
  CellArgs a = a_in;
  a.J = schur_lanes(a.m);
  const bool gal = a.r > 1;
  const size_t lds = solve_lds_bytes(a.NC, rpt, a.s, a.N, a.m, gal);
  if (lds > 160 * 1024) return set_error(MCH_EINVAL, "cell solve exceeds the LDS budget");
#define X(nc_, r_, n_, g_) \
  if (a.NC == nc_ && rpt == r_ && a.N == n_ && gal == g_) return launch_solve_t<nc_, r_, n_, g_>(a, lds, s);
  MCH_SHAPES(X)
#undef X
  return set_error(MCH_ENOTIMPL, "no kernel for this cell shape");
}

int solve_blocks_per_cu_2d(mch_plan* pl) {
  CellArgs a = base_args(pl, nullptr, nullptr, 0);
  const int rpt = pl->lev[0].shape.rpt;
  const size_t lds = solve_lds_bytes(a.NC, rpt, a.s, a.N, a.m, false);
  const void* fn = nullptr;
  int threads = 0;
#define X(nc_, r_, n_, g_)                                              \
  if (!g_ && a.NC == nc_ && rpt == r_ && a.N == n_) {                   \
    fn = reinterpret_cast<const void*>(k_solve2d<nc_, r_, n_, false>); \
    threads = nc_ * nc_ / r_;                                           \
  }
  MCH_SHAPES(X)
#undef X
  if (!fn) return set_error(MCH_ENOTIMPL, "no kernel for this cell shape");
  if (lds > 64 * 1024) {
    int rc = hip_check(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                       "hipFuncSetAttribute");
    if (rc) return rc;
  }
  int nb = 0;
  int rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, lds),
                     "hipOccupancyMaxActiveBlocksPerMultiprocessor");
  return rc ? rc : nb;
}

CellArgs chunk_args(const CellArgs& a, int start, int count) {
  CellArgs c = a;
  c.ci0 = start;
  c.count = count;
  return c;
}

// Forward DAG: the setups of levels >= 2 need only kappa and labels and run
// on their side streams from the start (they fill the CUs left idle by the
// level-1 solve). Level 1 solves in two chunks; each level >= 2 inherits and
// solves the cells of chunk A once chunk A is done (alongside the tail chunk
// B of level 1), then the rest once level 1 is done.
int launch_forward_2d(mch_plan* pl, const double* kappa, const uint8_t* label, hipStream_t s) {
  char name[32];
  int rc = ensure_streams(pl);
  if (!rc) rc = fork_levels(pl, s);
  for (int l = 1; l < pl->L && !rc; ++l) {
    if (pl->lev[l].count == 0) continue;
    CellArgs a = base_args(pl, kappa, label, l);
    std::snprintf(name, sizeof(name), "setup_L%d", l + 1);
    ProfScope ps(pl, name, level_stream(pl, l, s));
    rc = launch_setup(a, level_stream(pl, l, s));
  }
  const int n1 = pl->lev[0].count, n1a = pl->n1a;
  if (!rc && n1) {
    CellArgs a = base_args(pl, kappa, label, 0);
    {
      ProfScope ps(pl, "setup_L1", s);
      rc = launch_setup(a, s);
    }
    if (!rc && n1a > 0) {
      ProfScope ps(pl, "solve_L1", s);
      rc = launch_solve(chunk_args(a, 0, n1a), pl->lev[0].shape.rpt, s);
    }
    if (!rc) rc = hip_check(hipEventRecord(pl->ev_l1a, s), "hipEventRecord");
    if (!rc && n1 > n1a) {
      ProfScope ps(pl, "solve_L1", s);
      rc = launch_solve(chunk_args(a, n1a, n1 - n1a), pl->lev[0].shape.rpt, s);
    }
  } else if (!rc) {
    rc = hip_check(hipEventRecord(pl->ev_l1a, s), "hipEventRecord");
  }
  if (!rc) rc = hip_check(hipEventRecord(pl->ev_l1, s), "hipEventRecord");
  for (int l = 1; l < pl->L && !rc; ++l) {
    const int cnt = pl->lev[l].count, ca = pl->cntA[l];
    if (cnt == 0) continue;
    hipStream_t t = level_stream(pl, l, s);
    CellArgs a = base_args(pl, kappa, label, l);
    for (int part = 0; part < 2 && !rc; ++part) {
      const int start = part ? ca : 0, num = part ? cnt - ca : ca;
      rc = hip_check(hipStreamWaitEvent(t, part ? pl->ev_l1 : pl->ev_l1a, 0), "hipStreamWaitEvent");
      if (rc || num == 0) continue;
      const CellArgs c = chunk_args(a, start, num);
      {
        std::snprintf(name, sizeof(name), "inherit_L%d", l + 1);
        ProfScope ps(pl, name, t);
        rc = launch_inherit(c, t);
      }
      if (!rc) {
        std::snprintf(name, sizeof(name), "solve_L%d", l + 1);
        ProfScope ps(pl, name, t);
        rc = launch_solve(c, pl->lev[l].shape.rpt, t);
      }
    }
  }
  if (!rc) rc = join_levels(pl, s);
  return rc;
}

int launch_eff_2d(mch_plan* pl, const double* kappa, double* A, hipStream_t s) {
  int rc = ensure_streams(pl);
  if (!rc) rc = fork_levels(pl, s);
  for (int l = 0; l < pl->L && !rc; ++l) {
    if (pl->lev[l].count == 0) continue;
    hipStream_t t = level_stream(pl, l, s);
    CellArgs a = base_args(pl, kappa, pl->fwd_label, l);
    const size_t lds = ((size_t)a.M * (a.H + 1) * (a.H + 1) + (EFF_T / 64) * (size_t)a.M * a.M) * sizeof(double);
    if (lds > 160 * 1024) return set_error(MCH_EINVAL, "effective-tensor kernel exceeds the LDS budget");
    void (*fn)(CellArgs, double*) = nullptr;
    switch (a.M) {
      case 3: fn = k_eff2d<3>; break;
      case 6: fn = k_eff2d<6>; break;
      case 9: fn = k_eff2d<9>; break;
      default: return set_error(MCH_ENOTIMPL, "M");
    }
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute");
    }
    char name[32];
    std::snprintf(name, sizeof(name), "eff_L%d", l + 1);
    {
      ProfScope ps(pl, name, t);
      hipLaunchKernelGGL(fn, dim3(a.count), dim3(EFF_T), lds, t, a, A);
    }
    rc = hip_check(hipGetLastError(), "launch k_eff2d");
  }
  if (!rc) rc = join_levels(pl, s);
  return rc;
}

// Fine local solutions of selected cells: out[k][alpha][node] over (nc+1)^2 nodes.
__global__ void k_gather_phi2d(CellArgs a, const int32_t* sel_ci, int n_sel, double* out) {
  const int k = blockIdx.y;
  if (k >= n_sel) return;
  const int ci = sel_ci[k];
  if (ci < 0) return;
  const int nn1 = a.nc + 1;
  const size_t total = (size_t)a.M * nn1 * nn1;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int al = (int)(idx / ((size_t)nn1 * nn1));
    const int nd = (int)(idx % ((size_t)nn1 * nn1));
    out[(size_t)k * total + idx] = phi_at(a, ci, al, nd % nn1, nd / nn1);
  }
}

int launch_local_solutions_2d(mch_plan* pl, const int64_t* cells, int64_t n, double* out, hipStream_t s) {
  // group requested cells by level; one launch per level with the others masked
  for (int l = 0; l < pl->L; ++l) {
    std::vector<int32_t> sel(n, -1);
    bool any = false;
    for (int64_t k = 0; k < n; ++k) {
      const int64_t q = cells[k];
      if (pl->level[q] == l + 1) {
        sel[k] = pl->slot[q];
        any = true;
      }
    }
    if (!any) continue;
    int32_t* d_sel = nullptr;
    int rc = hip_check(hipMallocAsync((void**)&d_sel, sizeof(int32_t) * n, s), "hipMallocAsync");
    if (rc) return rc;
    rc = hip_check(hipMemcpyAsync(d_sel, sel.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    if (rc) return rc;
    CellArgs a = base_args(pl, pl->fwd_kappa, pl->fwd_label, l);
    hipLaunchKernelGGL(k_gather_phi2d, dim3(64, (unsigned)n), dim3(256), 0, s, a, d_sel, (int)n, out);
    rc = hip_check(hipGetLastError(), "launch k_gather_phi2d");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    (void)hipFreeAsync(d_sel, s);
    if (rc) return rc;
  }
  return MCH_OK;
}

}  // namespace mch
