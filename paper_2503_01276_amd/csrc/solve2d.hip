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

// ---------------------------------------------------------------------------
// Setup: per cell (one workgroup of 256 threads), on the fine grid:
//   n_qj, centroid sums of R_q intersect continuum j and of K_p intersect j,
//   cw[row] = 1/(4 n_qj) (0 when empty), g[alpha][row];
// then, for the level operator, S = B_n D^-1 B_n^T and S^-1 (Cholesky).
// ---------------------------------------------------------------------------

constexpr int SETUP_T = 256;

template <int N>
struct Quad {
  // coarse element data: stiffness (4x4) and constraint weights per corner/continuum
  double K[16];
  double b[4][N];
};

// Coarse element (EX, EY) of the level-r cell: Galerkin stiffness and corner
// weights of the constraint rows (without the 1/(4 n_qj) normalisation).
template <int N>
MCH_DEV void coarse_element(const CellArgs& a, int ox, int oy, int EX, int EY, Quad<N>& q) {
#pragma unroll
  for (int k = 0; k < 16; ++k) q.K[k] = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int j = 0; j < N; ++j) q.b[c][j] = 0.0;
  const int r = a.r;
  for (int v = 0; v < r; ++v) {
    const int gy = wrapi(oy + EY * r + v, a.n);
    for (int u = 0; u < r; ++u) {
      const int gx = wrapi(ox + EX * r + u, a.n);
      const size_t e = (size_t)gy * a.n + gx;
      const double kap = a.kappa[e];
      const int lab = a.label[e];
      const int pos = u + r * v;
      const double* tk = a.tabK + pos * 16;
      const double* tr = a.tabR + pos * 4;
#pragma unroll
      for (int k = 0; k < 16; ++k) q.K[k] += kap * tk[k];
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int j = 0; j < N; ++j) q.b[c][j] += (lab == j) ? tr[c] : 0.0;
    }
  }
}

template <int N>
__global__ __launch_bounds__(SETUP_T) void k_setup2d(CellArgs a) {
  extern __shared__ double sm[];
  const int m = a.m, s = a.s, nc = a.nc;
  double* S = sm;                  // m*m
  double* X = S + m * m;           // m*m (inverse of the Cholesky factor)
  double* stat = X + m * m;        // (s*s + 1) * N * 3 : count, sum x1, sum x2
  double* wred = stat + (s * s + 1) * N * 3;  // SETUP_T/64 * N * 3
  __shared__ int singular;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ci = blockIdx.x;
  const int p = a.cells[ci];
  const int jx = p % a.n_macro, jy = p / a.n_macro;
  const int ox = a.H * jx + a.H / 2 - nc / 2, oy = a.H * jy + a.H / 2 - nc / 2;

  for (int k = tid; k < 2 * m * m; k += SETUP_T) S[k] = 0.0;
  if (tid == 0) singular = 0;

  // statistics per region: region < s*s is sub-block q, region s*s is K_p
  const int sb = nc / s;
  for (int reg = 0; reg <= s * s; ++reg) {
    int x0, y0, w;
    if (reg < s * s) {
      x0 = (reg % s) * sb;
      y0 = (reg / s) * sb;
      w = sb;
    } else {
      x0 = (nc - a.H) / 2;
      y0 = x0;
      w = a.H;
    }
    double acc[N][3];
#pragma unroll
    for (int j = 0; j < N; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.0;
    for (int k = tid; k < w * w; k += SETUP_T) {
      const int ex = x0 + k % w, ey = y0 + k / w;
      const int lab = a.label[(size_t)wrapi(oy + ey, a.n) * a.n + wrapi(ox + ex, a.n)];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if (lab == j) {
          acc[j][0] += 1.0;
          acc[j][1] += ex + 0.5;
          acc[j][2] += ey + 0.5;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        double v = wave_sum(acc[j][t]);
        if (lane == 0) wred[(wave * N + j) * 3 + t] = v;
      }
    __syncthreads();
    if (tid < N * 3) {
      double v = 0.0;
      for (int w2 = 0; w2 < SETUP_T / 64; ++w2) v += wred[w2 * N * 3 + tid];
      stat[reg * N * 3 + tid] = v;
    }
    __syncthreads();
  }

  // row weights and right-hand sides
  const int M = a.M;
  if (tid < m) {
    const int k = tid, q = k / N, j = k % N;
    const double cnt = stat[(q * N + j) * 3];
    const double cw = cnt > 0.0 ? 1.0 / (4.0 * cnt) : 0.0;
    a.cw[(size_t)p * m + k] = cw;
    const double ckp = stat[(s * s * N + j) * 3];
    for (int al = 0; al < M; ++al) {
      double v = 0.0;
      if (cnt > 0.0) {
        if (al < N) {
          v = (al == j) ? 1.0 : 0.0;
        } else {
          const int i = (al - N) / 2, mm = (al - N) % 2;
          if (i == j) {
            const double xbar = stat[(q * N + j) * 3 + 1 + mm] / cnt;
            const double cmj = ckp > 0.0 ? stat[(s * s * N + j) * 3 + 1 + mm] / ckp : nc * 0.5;
            v = (xbar - cmj) * a.h;
          }
        }
      }
      a.g[((size_t)p * M + al) * m + k] = v;
    }
  }
  __syncthreads();

  // Level data per element, and the diagonal D of K_n per level node summed
  // in the solve kernel's order (fine: ((SW+SE)+NW)+NE of kappa/6, times 4;
  // Galerkin: SW, NW, SE, NE corner entries), so S is formed with exactly the
  // preconditioner the iteration applies.
  const int NC = a.NC, sbw = a.sbw, NCp = NC + 1;
  const bool gal = a.r > 1;
  double* Dn = wred + (SETUP_T / 64) * N * 3;                  // [NCp*NCp]
  double* kdS = Dn + NCp * NCp;                                 // fine: kappa/6 [NC*NC]; Galerkin: K_E diagonal [NC*NC][4]
  float* betaS = reinterpret_cast<float*>(kdS + (gal ? NC * NC * 4 : NC * NC));  // Galerkin: [NC*NC][4][N]
  uint8_t* labS = reinterpret_cast<uint8_t*>(betaS + (gal ? NC * NC * 4 * N : 0));  // fine: [NC*NC]
  const double* cwp = a.cw + (size_t)p * m;
  for (int e = tid; e < NC * NC; e += SETUP_T) {
    const int EX = e % NC, EY = e / NC;
    if (!gal) {
      const size_t ge = (size_t)wrapi(oy + EY, a.n) * a.n + wrapi(ox + EX, a.n);
      kdS[e] = a.kappa[ge] * (1.0 / 6.0);
      labS[e] = a.label[ge];
    } else {
      Quad<N> qd;
      coarse_element<N>(a, ox, oy, EX, EY, qd);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        kdS[e * 4 + c] = qd.K[c * 4 + c];
#pragma unroll
        for (int j = 0; j < N; ++j) betaS[(e * 4 + c) * N + j] = (float)qd.b[c][j];
      }
    }
  }
  __syncthreads();
  for (int k = tid; k < NCp * NCp; k += SETUP_T) {
    const int X = k % NCp, Y = k / NCp;
    if (X < 1 || Y < 1 || X >= NC || Y >= NC) {
      Dn[k] = 1.0;
      continue;
    }
    const int eSW = (Y - 1) * NC + X - 1, eSE = eSW + 1, eNW = Y * NC + X - 1, eNE = eNW + 1;
    if (!gal) {
      const double ks = kdS[eSW] + kdS[eSE] + kdS[eNW] + kdS[eNE];
      Dn[k] = 4.0 * ks;
    } else {
      double d = 0.0;
      d += kdS[eSW * 4 + 3];
      d += kdS[eNW * 4 + 1];
      d += kdS[eSE * 4 + 2];
      d += kdS[eNE * 4 + 0];
      Dn[k] = d;
    }
  }
  __syncthreads();

  // S = B_n D^-1 B_n^T: entry (ra, rb) summed by one thread over the free
  // level nodes shared by the closures of the two sub-blocks, in a fixed order.
  for (int pr = tid; pr < m * m; pr += SETUP_T) {
    const int ra = pr / m, rb = pr % m;
    if (rb < ra) continue;
    const int qa = ra / N, ja = ra % N, qb = rb / N, jb = rb % N;
    const int qax = qa % s, qay = qa / s, qbx = qb % s, qby = qb / s;
    const double cwa = cwp[ra], cwb = cwp[rb];
    double acc = 0.0;
    if (abs(qax - qbx) <= 1 && abs(qay - qby) <= 1 && cwa != 0.0 && cwb != 0.0) {
      const int X0 = max(max(qax, qbx) * sbw, 1), X1 = min((min(qax, qbx) + 1) * sbw, NC - 1);
      const int Y0 = max(max(qay, qby) * sbw, 1), Y1 = min((min(qay, qby) + 1) * sbw, NC - 1);
      for (int Y = Y0; Y <= Y1; ++Y)
        for (int X = X0; X <= X1; ++X) {
          double ba = 0.0, bb = 0.0;
#pragma unroll
          for (int Qd = 0; Qd < 4; ++Qd) {
            const int EX = X - 1 + (Qd & 1), EY = Y - 1 + (Qd >> 1);
            const int corner = 3 - Qd;
            const int e = EY * NC + EX;
            const int qE = (EY / sbw) * s + EX / sbw;
            double wa, wb;
            if (!gal) {
              const int lab = labS[e];
              wa = (lab == ja) ? 1.0 : 0.0;
              wb = (lab == jb) ? 1.0 : 0.0;
            } else {
              wa = (double)betaS[(e * 4 + corner) * N + ja];
              wb = (double)betaS[(e * 4 + corner) * N + jb];
            }
            if (qE == qa) ba += wa;
            if (qE == qb) bb += wb;
          }
          acc += (cwa * ba) * (cwb * bb) * (1.0 / Dn[Y * NCp + X]);
        }
    }
    S[ra * m + rb] = acc;
    S[rb * m + ra] = acc;
  }
  __syncthreads();

  // Cholesky S = L L^T in place (lower triangle), one wave; inactive rows get 1.
  if (wave == 0) {
    for (int k = lane; k < m; k += 64)
      if (cwp[k] == 0.0) S[k * m + k] = 1.0;
    __builtin_amdgcn_wave_barrier();
    for (int k = 0; k < m; ++k) {
      const double piv = S[k * m + k];
      if (!(piv > 0.0)) {
        if (lane == 0) singular = 1;
      }
      const double lkk = sqrt(piv > 0.0 ? piv : 1.0);
      __builtin_amdgcn_wave_barrier();
      for (int i = k + 1 + lane; i < m; i += 64) S[i * m + k] /= lkk;
      if (lane == 0) S[k * m + k] = lkk;
      __builtin_amdgcn_wave_barrier();
      for (int i = k + 1 + lane; i < m; i += 64) {
        const double lik = S[i * m + k];
        for (int jj = k + 1; jj <= i; ++jj) S[i * m + jj] -= lik * S[jj * m + k];
      }
      __builtin_amdgcn_wave_barrier();
    }
    // X = L^-1 (lower triangular), lane = column
    for (int col = lane; col < m; col += 64) {
      for (int i = 0; i < m; ++i) {
        double v = (i == col) ? 1.0 : 0.0;
        for (int jj = col; jj < i; ++jj) v -= S[i * m + jj] * X[jj * m + col];
        X[i * m + col] = (i >= col) ? v / S[i * m + i] : 0.0;
      }
    }
  }
  __syncthreads();
  // S^-1 = X^T X
  const bool bad = singular != 0;
  for (int k = tid; k < m * m; k += SETUP_T) {
    const int i = k / m, j = k % m;
    double v = 0.0;
    for (int t = (i > j ? i : j); t < m; ++t) v += X[t * m + i] * X[t * m + j];
    a.sinv[(size_t)p * m * m + k] = bad ? __builtin_nan("") : v;
  }
}

// ---------------------------------------------------------------------------
// The cell solve.
// ---------------------------------------------------------------------------

// Fine cells of width >= 64 keep kappa/6 and the iterate x in LDS instead of
// registers (the register file cannot hold them at 4-8 nodes per lane).
template <int NC, bool GAL>
constexpr bool kBig = !GAL && NC >= 64;

template <int NC, int RPT, int N, bool GAL>
struct NodeData {
  // fine level: kappa/6 of the quadrant elements (columns c-1, c; rows y0-1..y0+RPT-1)
  double kq[(GAL || kBig<NC, GAL>) ? 1 : 2][(GAL || kBig<NC, GAL>) ? 1 : RPT + 1];
  // Galerkin level: 9-point stencil per node, index (dy+1)*3 + dx+1
  double W[GAL ? RPT : 1][GAL ? 9 : 1];
  double Dinv[RPT];
  // constraint weights without row normalisation: side (0: element column
  // c-1, 1: column c), node row, continuum; lower quadrants of node row 0 on
  // their own when the band starts a new sub-block row. The weights are sums
  // of multiples of 1/r^2 below 2^24/r^2, hence exact in binary32.
  float w[2][RPT][N];
  float wlo[2][N];
};

template <int NC, int RPT, int N, bool GAL>
__global__ __launch_bounds__(NC* NC / RPT) void k_solve2d(CellArgs a) {
  constexpr int NT = NC * NC / RPT;
  constexpr int NW = NT / 64;
  constexpr int NB = NC / RPT;
  constexpr int PW = NC + 2;
  extern __shared__ double smem[];
  const int m = a.m, s = a.s, M = a.M, sbw = a.sbw;
  double* pS = smem;                       // PW*PW (ring of zeros)
  double* red = pS + PW * PW;              // 2*NW
  double* part = red + 2 * NW;             // NB*2*s*N
  double* sinvS = part + NB * 2 * s * N;   // m*m
  double* uS = sinvS + m * m;              // m
  double* vS = uS + m;                     // m  (v * cw)
  double* cwS = vS + m;                    // m
  double* scal = cwS + m;                  // 8
  double* feS = scal + 8;                  // GAL: NC*NC*4 coarse-element load vectors
  constexpr bool BIG = kBig<NC, GAL>;
  double* kS = scal + 8;                   // BIG: (NC+1)^2 kappa/6, ring of zeros at -1
  double* xS = kS + (NC + 1) * (NC + 1);   // BIG: NC*NC iterate

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = tid % NC, band = tid / NC, y0 = band * RPT;
  const int ci = blockIdx.x / M, alpha = blockIdx.x % M;
  const int p = a.cells[ci];
  const int jx = p % a.n_macro, jy = p / a.n_macro;
  const int ox = a.H * jx + a.H / 2 - a.nc / 2, oy = a.H * jy + a.H / 2 - a.nc / 2;
  const bool split0 = (y0 > 0) && (y0 % sbw == 0);
  const int qxL = (c > 0 ? c - 1 : 0) / sbw, qxR = c / sbw;
  const int qyU = y0 / sbw, qyL = (y0 > 0 ? y0 - 1 : 0) / sbw;

  for (int k = tid; k < PW * PW; k += NT) pS[k] = 0.0;
  for (int k = tid; k < m * m; k += NT) sinvS[k] = a.sinv[(size_t)p * m * m + k];
  for (int k = tid; k < m; k += NT) cwS[k] = a.cw[(size_t)p * m + k];

  NodeData<NC, RPT, N, GAL> nd;
  double x[RPT], r[RPT], pv[RPT];
  double f[RPT];

  // ---- operator data --------------------------------------------------------
#pragma unroll
  for (int sd = 0; sd < 2; ++sd) {
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) nd.w[sd][i][j] = 0.0f;
#pragma unroll
    for (int j = 0; j < N; ++j) nd.wlo[sd][j] = 0.0f;
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
        if constexpr (!BIG) nd.kq[sd][i] = kl[sd][i];
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
      nd.Dinv[i] = fr ? 1.0 / (4.0 * ksum) : 0.0;
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const float up = (lab[sd][i + 1] == j) ? 1.0f : 0.0f;
          const float lo = (lab[sd][i] == j) ? 1.0f : 0.0f;
          if (i == 0 && split0) {
            nd.w[sd][i][j] = fr ? up : 0.0f;
            nd.wlo[sd][j] = fr ? lo : 0.0f;
          } else {
            nd.w[sd][i][j] = fr ? up + lo : 0.0f;
          }
        }
    }
  } else {
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
      for (int k = 0; k < 9; ++k) nd.W[i][k] = 0.0;
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
#pragma unroll
      for (int ip = 0; ip <= RPT; ++ip) {
        const int EX = c - 1 + sd, EY = y0 - 1 + ip;
        if (EX < 0 || EY < 0) continue;
        Quad<N> qd;
        coarse_element<N>(a, ox, oy, EX, EY, qd);
        // lower quadrant of node row ip (SW for sd=0, SE for sd=1)
        if (ip < RPT) {
          const int cn = sd == 0 ? 3 : 2;
          const int ax = cn & 1, ay = cn >> 1;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int dx = (b & 1) - ax, dy = (b >> 1) - ay;
            nd.W[ip][(dy + 1) * 3 + dx + 1] += qd.K[cn * 4 + b];
          }
#pragma unroll
          for (int j = 0; j < N; ++j) {
            if (ip == 0 && split0)
              nd.wlo[sd][j] += (float)qd.b[cn][j];
            else
              nd.w[sd][ip][j] += (float)qd.b[cn][j];
          }
        }
        // upper quadrant of node row ip-1 (NW for sd=0, NE for sd=1)
        if (ip >= 1) {
          const int cn = sd == 0 ? 1 : 0;
          const int ax = cn & 1, ay = cn >> 1;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int dx = (b & 1) - ax, dy = (b >> 1) - ay;
            nd.W[ip - 1][(dy + 1) * 3 + dx + 1] += qd.K[cn * 4 + b];
          }
#pragma unroll
          for (int j = 0; j < N; ++j) nd.w[sd][ip - 1][j] += (float)qd.b[cn][j];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const bool fr = (c >= 1) && (y0 + i >= 1);
      nd.Dinv[i] = fr ? 1.0 / nd.W[i][4] : 0.0;
      if (!fr) {
#pragma unroll
        for (int k = 0; k < 9; ++k) nd.W[i][k] = 0.0;
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
          for (int j = 0; j < N; ++j) nd.w[sd][i][j] = 0.0f;
        if (i == 0) {
#pragma unroll
          for (int sd = 0; sd < 2; ++sd)
#pragma unroll
            for (int j = 0; j < N; ++j) nd.wlo[sd][j] = 0.0f;
        }
      }
    }
  }

  // ---- helpers over the band ------------------------------------------------
  auto P_at = [&](int xx, int yy) -> double { return pS[(yy + 1) * PW + xx + 1]; };

  // y = K_n v for the thread's nodes; v own values in `vv`, neighbours from pS.
  auto apply_K = [&](const double (&vv)[RPT], double (&yv)[RPT]) {
    double Lc[RPT + 2], Rc[RPT + 2];
    double Cb = P_at(c, y0 - 1), Ct = P_at(c, y0 + RPT);
#pragma unroll
    for (int i = 0; i < RPT + 2; ++i) {
      Lc[i] = P_at(c - 1, y0 - 1 + i);
      Rc[i] = P_at(c + 1, y0 - 1 + i);
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const double pC = vv[i];
      const double pS_ = i == 0 ? Cb : vv[i - 1];
      const double pN = i == RPT - 1 ? Ct : vv[i + 1];
      if constexpr (!GAL) {
        double kSW, kSE, kNW, kNE;
        if constexpr (BIG) {
          const double* kr0 = kS + (y0 + i) * (NC + 1) + c;  // element row y0-1+i, column c-1
          kSW = kr0[0];
          kSE = kr0[1];
          kNW = kr0[NC + 1];
          kNE = kr0[NC + 2];
        } else {
          kSW = nd.kq[0][i];
          kSE = nd.kq[1][i];
          kNW = nd.kq[0][i + 1];
          kNE = nd.kq[1][i + 1];
        }
        const double aS = kSW + kSE, aN = kNW + kNE, aW = kSW + kNW, aE = kSE + kNE;
        double t = 4.0 * (aS + aN) * pC;
        t -= aS * pS_ + aN * pN + aW * Lc[i + 1] + aE * Rc[i + 1];
        t -= 2.0 * (kSW * Lc[i] + kSE * Rc[i] + kNW * Lc[i + 2] + kNE * Rc[i + 2]);
        yv[i] = t;
      } else {
        const double* W = nd.W[i];
        double t = W[4] * pC;
        t += W[1] * pS_ + W[7] * pN + W[3] * Lc[i + 1] + W[5] * Rc[i + 1];
        t += W[0] * Lc[i] + W[2] * Rc[i] + W[6] * Lc[i + 2] + W[8] * Rc[i + 2];
        yv[i] = t;
      }
    }
  };

  // Block sum of one value per thread into red[slot]; returns the total.
  auto block_sum = [&](double v, int slot) -> double {
    v = wave_sum(v);
    if (lane == 0) red[slot * NW + wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < NW; ++w2) t += red[slot * NW + w2];
    return t;
  };

  // Partial sums of B_n t (without the row normalisation) into `part`.
  auto accumulate_B = [&](const double (&tv)[RPT]) {
    double acc[2][2][N];  // side, iy (0: below the band's sub-block row), j
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        double up = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) up += (double)nd.w[sd][i][j] * tv[i];
        acc[sd][1][j] = up;
        acc[sd][0][j] = (double)nd.wlo[sd][j] * tv[0];
      }
    // element column c collects side 1 of lane c and side 0 of lane c+1
#pragma unroll
    for (int iy = 0; iy < 2; ++iy)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        double v = acc[1][iy][j] + from_right(acc[0][iy][j], c, NC);
        v = seg_sum(v, sbw);
        if (c % sbw == 0) part[((band * 2 + iy) * s + c / sbw) * N + j] = v;
      }
  };

  // Row k of B_n t from the band partials (called by threads k < m).
  auto finalize_u = [&](int k) -> double {
    const int q = k / N, j = k % N, qx = q % s, qy = q / s;
    double u = 0.0;
    for (int b = 0; b < NB; ++b) {
      const int yb = b * RPT;
      if (yb / sbw == qy) u += part[((b * 2 + 1) * s + qx) * N + j];
      if (yb > 0 && yb % sbw == 0 && (yb - 1) / sbw == qy) u += part[((b * 2 + 0) * s + qx) * N + j];
    }
    return u * cwS[k];
  };

  // Wave 0: v = S^-1 u (u in uS), vS = v*cw, returns v.u in lane 0 (all lanes).
  auto schur_solve = [&](double* Vacc) -> double {
    int J = 1;
    while (J * 2 * m <= 64) J *= 2;
    const int k = lane / J, jj = lane % J;
    double sum = 0.0;
    if (k < m)
      for (int j = jj; j < m; j += J) sum += sinvS[k * m + j] * uS[j];
    sum = seg_sum(sum, J);
    double vu = 0.0;
    if (k < m && jj == 0) {
      vS[k] = sum * cwS[k];
      *Vacc += sum;
      vu = sum * uS[k];
    }
    return wave_sum(vu);
  };

  // r -= B_n^T v (or x += D^-1 B_n^T v with sign), node-local with vS.
  auto scatter_B = [&](double (&tv)[RPT], double sign) {
    double vs[2][2][N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      vs[0][1][j] = vS[(qyU * s + qxL) * N + j];
      vs[1][1][j] = vS[(qyU * s + qxR) * N + j];
      vs[0][0][j] = vS[(qyL * s + qxL) * N + j];
      vs[1][0][j] = vS[(qyL * s + qxR) * N + j];
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      double t = 0.0;
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int j = 0; j < N; ++j) t += nd.w[sd][i][j] * vs[sd][1][j];
      if (i == 0) {
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
          for (int j = 0; j < N; ++j) t += nd.wlo[sd][j] * vs[sd][0][j];
      }
      tv[i] += sign * t;
    }
  };

  // ---- right-hand side ------------------------------------------------------
  double Vacc = 0.0;  // wave 0, lanes holding a row: accumulated projections
#pragma unroll
  for (int i = 0; i < RPT; ++i) f[i] = 0.0;
  const size_t NNl = (size_t)(NC + 1) * (NC + 1);
  const int nn1 = (a.nc + 1);
  const int k0 = (a.nc - a.H) / 2;  // first fine node index of K_p
  __syncthreads();
  if (!a.adjoint) {
    if constexpr (GAL) {
      // inherited solution I = Phi of the level-1 point (same local coordinates)
      const double* I = a.phi1 + ((size_t)a.pslot[ci] * M + alpha) * (size_t)(nn1 * nn1);
      const int rr = a.r;
      double accI[N];
#pragma unroll
      for (int j = 0; j < N; ++j) accI[j] = 0.0;
      for (int i = 0; i < RPT; ++i) {
        const int EX = c, EY = y0 + i;
        double FE[4] = {0.0, 0.0, 0.0, 0.0};
        for (int v = 0; v < rr; ++v)
          for (int u = 0; u < rr; ++u) {
            const int fx = EX * rr + u, fy = EY * rr + v;
            const size_t e = (size_t)wrapi(oy + fy, a.n) * a.n + wrapi(ox + fx, a.n);
            const double k6 = a.kappa[e] * (1.0 / 6.0);
            const int lab = a.label[e];
            double Iv[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) Iv[d] = I[(size_t)(fy + (d >> 1)) * nn1 + fx + (d & 1)];
            const double y00 = k6 * (4 * Iv[0] - Iv[1] - Iv[2] - 2 * Iv[3]);
            const double y10 = k6 * (-Iv[0] + 4 * Iv[1] - 2 * Iv[2] - Iv[3]);
            const double y01 = k6 * (-Iv[0] - 2 * Iv[1] + 4 * Iv[2] - Iv[3]);
            const double y11 = k6 * (-2 * Iv[0] - Iv[1] - Iv[2] + 4 * Iv[3]);
            const double yv[4] = {y00, y10, y01, y11};
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              const double xi = (u + (d & 1)) / (double)rr, ze = (v + (d >> 1)) / (double)rr;
              FE[0] += (1.0 - xi) * (1.0 - ze) * yv[d];
              FE[1] += xi * (1.0 - ze) * yv[d];
              FE[2] += (1.0 - xi) * ze * yv[d];
              FE[3] += xi * ze * yv[d];
            }
            const double es = Iv[0] + Iv[1] + Iv[2] + Iv[3];
#pragma unroll
            for (int j = 0; j < N; ++j) accI[j] += (lab == j) ? es : 0.0;
          }
#pragma unroll
        for (int d = 0; d < 4; ++d) feS[(EY * NC + EX) * 4 + d] = FE[d];
      }
      // B_h I partials: all own elements lie in sub-block (c/sbw, y0/sbw)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        double v = seg_sum(accI[j], sbw);
        if (c % sbw == 0) {
          part[((band * 2 + 1) * s + c / sbw) * N + j] = v;
          part[((band * 2 + 0) * s + c / sbw) * N + j] = 0.0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int X = c, Y = y0 + i;
        const bool fr = X >= 1 && Y >= 1;
        double t = feS[(Y * NC + X) * 4 + 0];
        if (X >= 1) t += feS[(Y * NC + X - 1) * 4 + 1];
        if (Y >= 1) t += feS[((Y - 1) * NC + X) * 4 + 2];
        if (X >= 1 && Y >= 1) t += feS[((Y - 1) * NC + X - 1) * 4 + 3];
        f[i] = fr ? -t : 0.0;
      }
      if (wave == 0) {
        for (int k = lane; k < m; k += 64)
          uS[k] = a.g[((size_t)p * M + alpha) * m + k] - finalize_u(k);
      }
    } else {
      if (wave == 0)
        for (int k = lane; k < m; k += 64) uS[k] = a.g[((size_t)p * M + alpha) * m + k];
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
    if (wave == 0)
      for (int k = lane; k < m; k += 64) uS[k] = 0.0;
  }
  __syncthreads();

  // ---- feasible start: x0 = D^-1 B^T S^-1 g' --------------------------------
  if (wave == 0) (void)schur_solve(&Vacc);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RPT; ++i) x[i] = 0.0;
  scatter_B(x, 1.0);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    x[i] *= nd.Dinv[i];
    pS[(y0 + i + 1) * PW + c + 1] = x[i];
    if constexpr (BIG) xS[(y0 + i) * NC + c] = x[i];
  }
  if (wave == 0 && lane < 64) Vacc = 0.0;  // x0's multiplier part is not a projection of r
  __syncthreads();
  apply_K(x, r);
#pragma unroll
  for (int i = 0; i < RPT; ++i) r[i] -= f[i];
  __syncthreads();

  // ---- project the initial residual -----------------------------------------
  double t[RPT];
  double rDr = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    t[i] = nd.Dinv[i] * r[i];
    rDr += r[i] * t[i];
  }
  accumulate_B(t);
  rDr = block_sum(rDr, 0);  // includes __syncthreads (part visible)
  if (wave == 0) {
    for (int k = lane; k < m; k += 64) uS[k] = finalize_u(k);
    __builtin_amdgcn_wave_barrier();
    const double vu = schur_solve(&Vacc);
    if (lane == 0) scal[0] = rDr - vu;
  }
  __syncthreads();
  double rz = scal[0];
  const double rz0 = rz;
  scatter_B(r, -1.0);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    pv[i] = -nd.Dinv[i] * r[i];
    pS[(y0 + i + 1) * PW + c + 1] = pv[i];
  }
  __syncthreads();

  const double tol2 = a.rtol * a.rtol * rz0;
  int it = 0;
  bool done = !(rz0 > 0.0) || rz0 <= 0.0;
  while (!done) {
    // Ap and p.Ap
    double Ap[RPT];
    apply_K(pv, Ap);
    double pAp = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) pAp += pv[i] * Ap[i];
    pAp = block_sum(pAp, 0);
    const double al = rz / pAp;
    rDr = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      if constexpr (BIG)
        xS[(y0 + i) * NC + c] += al * pv[i];
      else
        x[i] += al * pv[i];
      r[i] += al * Ap[i];
      t[i] = nd.Dinv[i] * r[i];
      rDr += r[i] * t[i];
    }
    accumulate_B(t);
    rDr = block_sum(rDr, 1);
    if (wave == 0) {
      for (int k = lane; k < m; k += 64) uS[k] = finalize_u(k);
      __builtin_amdgcn_wave_barrier();
      const double vu = schur_solve(&Vacc);
      if (lane == 0) scal[1] = rDr - vu;
    }
    __syncthreads();
    const double rzn = scal[1];
    ++it;
    if (rzn <= tol2 || it >= a.max_iter) {
      rz = rzn;
      break;
    }
    scatter_B(r, -1.0);
    const double be = rzn / rz;
    rz = rzn;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      pv[i] = -nd.Dinv[i] * r[i] + be * pv[i];
      pS[(y0 + i + 1) * PW + c + 1] = pv[i];
    }
    __syncthreads();
  }

  // ---- outputs ---------------------------------------------------------------
  double* dst;
  size_t vec;
  if (a.r == 1) {
    vec = (size_t)nn1 * nn1;
  } else {
    vec = NNl;
  }
  dst = a.out + ((size_t)ci * M + alpha) * vec;
#pragma unroll
  for (int i = 0; i < RPT; ++i) dst[(size_t)(y0 + i) * (NC + 1) + c] = BIG ? xS[(y0 + i) * NC + c] : x[i];
  if (wave == 0) {
    int J = 1;
    while (J * 2 * m <= 64) J *= 2;
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
  const int ci = blockIdx.x;
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
  a.adjoint = 0;
  a.seed_kp = pl->d_seed_kp;
  a.seed_par = nullptr;
  a.slot = pl->d_slot;
  a.rtol = pl->cfg.rtol;
  a.max_iter = pl->cfg.max_iter;
  return a;
}

static size_t solve_lds_bytes(int NC, int rpt, int s, int N, int m, bool gal) {
  const int NT = NC * NC / rpt, NW = NT / 64, NB = NC / rpt, PW = NC + 2;
  size_t d = (size_t)PW * PW + 2 * NW + (size_t)NB * 2 * s * N + (size_t)m * m + 3 * (size_t)m + 8;
  if (gal) d += (size_t)NC * NC * 4;
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
  X(32, 1, 2, false) X(32, 1, 3, false) X(16, 4, 2, false) X(16, 4, 3, false)                 \
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

int launch_solve(const CellArgs& a, int rpt, hipStream_t s) {
  const bool gal = a.r > 1;
  const size_t lds = solve_lds_bytes(a.NC, rpt, a.s, a.N, a.m, gal);
  if (lds > 160 * 1024) return set_error(MCH_EINVAL, "cell solve exceeds the LDS budget");
#define X(nc_, r_, n_, g_) \
  if (a.NC == nc_ && rpt == r_ && a.N == n_ && gal == g_) return launch_solve_t<nc_, r_, n_, g_>(a, lds, s);
  MCH_SHAPES(X)
#undef X
  return set_error(MCH_ENOTIMPL, "no kernel for this cell shape");
}

static size_t setup_lds_bytes(const CellArgs& a) {
  const size_t NC = a.NC, NCp = NC + 1;
  size_t d = (size_t)2 * a.m * a.m + (size_t)(a.s * a.s + 1) * a.N * 3 + (SETUP_T / 64) * a.N * 3 + NCp * NCp;
  size_t bytes;
  if (a.r > 1)
    bytes = (d + NC * NC * 4) * sizeof(double) + NC * NC * 4 * a.N * sizeof(float);
  else
    bytes = (d + NC * NC) * sizeof(double) + NC * NC;
  return bytes;
}

static int launch_setup(const CellArgs& a, hipStream_t s) {
  const size_t lds = setup_lds_bytes(a);
  if (lds > 160 * 1024) return set_error(MCH_EINVAL, "setup exceeds the LDS budget");
  void (*fn)(CellArgs) = nullptr;
  if (a.N == 1) fn = k_setup2d<1>;
  if (a.N == 2) fn = k_setup2d<2>;
  if (a.N == 3) fn = k_setup2d<3>;
  if (!fn) return set_error(MCH_ENOTIMPL, "n_cont");
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute");
  }
  hipLaunchKernelGGL(fn, dim3(a.count), dim3(SETUP_T), lds, s, a);
  return hip_check(hipGetLastError(), "launch k_setup2d");
}

int launch_forward_2d(mch_plan* pl, const double* kappa, const uint8_t* label, hipStream_t s) {
  char name[32];
  for (int l = 0; l < pl->L; ++l) {
    if (pl->lev[l].count == 0) continue;
    CellArgs a = base_args(pl, kappa, label, l);
    int rc;
    {
      std::snprintf(name, sizeof(name), "setup_L%d", l + 1);
      ProfScope ps(pl, name, s);
      rc = launch_setup(a, s);
    }
    if (rc) return rc;
    {
      std::snprintf(name, sizeof(name), "solve_L%d", l + 1);
      ProfScope ps(pl, name, s);
      rc = launch_solve(a, pl->lev[l].shape.rpt, s);
    }
    if (rc) return rc;
  }
  return MCH_OK;
}

int launch_eff_2d(mch_plan* pl, const double* kappa, double* A, hipStream_t s) {
  for (int l = 0; l < pl->L; ++l) {
    if (pl->lev[l].count == 0) continue;
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
      ProfScope ps(pl, name, s);
      hipLaunchKernelGGL(fn, dim3(a.count), dim3(EFF_T), lds, s, a, A);
    }
    int rc = hip_check(hipGetLastError(), "launch k_eff2d");
    if (rc) return rc;
  }
  return MCH_OK;
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
