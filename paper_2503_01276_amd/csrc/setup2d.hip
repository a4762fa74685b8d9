// 2D per-cell preparation kernels for gfx950.
//
// k_setup2d (one workgroup per cell of a level):
//   * constraint statistics on the fine grid: for every sub-block R_q and
//     continuum j the element count n_qj and centroid, and the continuum
//     centroids c_mj in K_p; row weights cw = 1/(4 n_qj) (0: inactive row) and
//     right-hand sides g (paper Eqs. phi_avar and phi_grad, constraints
//     normalised to averages);
//   * for Galerkin levels (r = eta^(n-1) > 1, Sec. 3.2 with V_n a subspace of
//     V_h): the coarse element matrices sum_s kappa_s R^T K_ref R assembled into
//     a 9-point stencil per level node, and the constraint weights of B_n = B_h P
//     per node, side and part (written to global memory for the solve kernel);
//   * S = B_n D^-1 B_n^T with D = diag(K_n), and S^-1 by Gauss-Jordan
//     elimination (S is symmetric positive definite: no pivoting).
// k_inherit2d (levels >= 2, one workgroup per cell): the inherited
//   right-hand sides f = -P^T K_h I and g' = g - B_h I of Eqs.
//   phi_avar_corrector / phi_grad_corrector, I = Phi of the inherited level-1 cell.
//
// Every reduction runs in a fixed order (no floating-point atomics), so the
// results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#include "kernels2d.h"

namespace mch {

constexpr int SETUP_T = 256;
// Bands whose Schur corrections the setup forms at once (one group of at
// most 64 lanes each).
constexpr int PREC_GROUP = 4;
static_assert(PREC_GROUP * 64 <= SETUP_T, "a set-up workgroup reduces PREC_GROUP band matrices at once");

// Most constraint rows a band of prec_rows node rows can meet (the rows of
// every sub-block row whose nodes reach into the band) and the bands formed
// at once, for the setup's LDS.
__host__ __device__ inline void prec_group_sizes(const CellArgs& a, int* NA, int* G) {
  const int R = a.prec_rows, nbands = a.NC / R;
  const int rows_of_blocks = R / a.sbw + 2;
  *NA = rows_of_blocks * a.s * a.N < a.m ? rows_of_blocks * a.s * a.N : a.m;
  *G = nbands < PREC_GROUP ? nbands : PREC_GROUP;
}

// Coarse element data, flat so that one DPP pass sums it over lanes: the
// element stiffness [16] (corners in tensor order), then the constraint
// weights per corner and continuum [4][N] (no 1/(4 n_qj)).
template <int N>
constexpr int quad_len() { return 16 + 4 * N; }

// The part of coarse element (EX, EY) of the level-r cell from its fine
// elements first, first + stride, ... (of the r^2, x fastest).
template <int N>
MCH_DEV void coarse_element_part(const CellArgs& a, int ox, int oy, int EX, int EY, int first, int stride,
                                 double (&q)[quad_len<N>()]) {
#pragma unroll
  for (int k = 0; k < quad_len<N>(); ++k) q[k] = 0.0;
  const int r = a.r;
  for (int pos = first; pos < r * r; pos += stride) {
    const int u = pos % r, v = pos / r;
    const size_t e = (size_t)wrap1(oy + EY * r + v, a.n) * a.n + wrap1(ox + EX * r + u, a.n);
    const double kap = a.kappa[e];
    const int lab = a.label[e];
    const double* tk = a.tabK + pos * 16;
    const double* tr = a.tabR + pos * 4;
#pragma unroll
    for (int k = 0; k < 16; ++k) q[k] += kap * tk[k];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < N; ++j) q[16 + c * N + j] += (lab == j) ? tr[c] : 0.0;
  }
}

template <int N, int T>
__global__ __launch_bounds__(T) void k_setup2d(CellArgs a) {
  extern __shared__ double sm[];
  const int m = a.m, s = a.s, nc = a.nc, NC = a.NC, NCp = NC + 1, sbw = a.sbw;
  const bool gal = a.r > 1;
  double* S = sm;                        // m*m
  double* X = S + m * m;                 // 2*m: pivot row and column
  double* stat = X + 2 * m;              // (s*s+1)*N*3
  double* wred = stat + (s * s + 1) * N * 3;  // 4*N*3
  // band coarse correction (prec_rows > 0), for a group of G bands: the
  // band-summed weights of the constraint rows active in each [G][NA][NC],
  // T_b^-1 applied to them [G][NA][NC], the cyclic-reduction factors of each
  // T_b [G][pcr_offset(NC, log2 NC)] and 1 / its final pivots [G][NC]
  const bool prec = a.prec_rows > 0;
  const int nbands = prec ? NC / a.prec_rows : 0;
  int pNA = 0, pG = 0;
  if (prec) prec_group_sizes(a, &pNA, &pG);
  const int logNC = 31 - __builtin_clz(NC), pcb = pcr_offset(NC, logNC);
  double* BZ = wred + (T / 64) * N * 3;
  double* Ys = BZ + pG * pNA * NC;
  double* Fs = Ys + pG * pNA * NC;
  double* IBs = Fs + pG * pcb;
  uint8_t* labS = reinterpret_cast<uint8_t*>(IBs + pG * NC);  // fine: NC*NC labels
  uint8_t* regS = labS + NC * NC;        // NC*NC sub-block of each element
  __shared__ int singular;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ci = a.ci0 + blockIdx.x;
  const int p = a.cells[ci];
  const int jx = p % a.n_macro, jy = p / a.n_macro;
  const int ox = a.H * jx + a.H / 2 - nc / 2, oy = a.H * jy + a.H / 2 - nc / 2;
  if (tid == 0) singular = 0;

  // ---- constraint statistics per region (sub-blocks, then K_p) -------------
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
    for (int k = tid; k < w * w; k += T) {
      const int ex = x0 + k % w, ey = y0 + k / w;
      const int lab = a.label[(size_t)wrap1(oy + ey, a.n) * a.n + wrap1(ox + ex, a.n)];
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
      for (int w2 = 0; w2 < T / 64; ++w2) v += wred[w2 * N * 3 + tid];
      stat[reg * N * 3 + tid] = v;
    }
    __syncthreads();
  }
  const int M = a.M;
  double* cwp = a.cw + (size_t)p * m;
  if (tid < m) {
    const int k = tid, q = k / N, j = k % N;
    const double cnt = stat[(q * N + j) * 3];
    cwp[k] = cnt > 0.0 ? 1.0 / (4.0 * cnt) : 0.0;
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

  // ---- level operator data ------------------------------------------------
  // Free level nodes: [lo, hi]^2 (Dirichlet: the interior; Neumann: all).
  const int lo = a.bc ? 0 : 1, hi = a.bc ? NC : NC - 1;
  double* nW = gal ? a.nodeW + (size_t)ci * NCp * NCp * 9 : nullptr;
  float* nB = gal ? a.nodeB + (size_t)ci * NCp * NCp * 4 * N : nullptr;
  if (gal) {
    for (int k = tid; k < NCp * NCp * 9; k += T) nW[k] = 0.0;
    for (int k = tid; k < NCp * NCp * 4 * N; k += T) nB[k] = 0.0f;
    __syncthreads();
    // four colour passes: elements of one colour share no node. When a pass
    // has fewer elements than lanes, a group of tpe lanes (a power of two)
    // shares an element's fine elements and sums its data with DPP; every
    // lane of a group runs the same trips.
    for (int color = 0; color < 4; ++color) {
      const int cx = color & 1, cy = color >> 1;
      const int hx = (NC - cx + 1) / 2, hy = (NC - cy + 1) / 2, ne = hx * hy;
      int tpe = 1;
      while (tpe * 2 * ne <= T && tpe < 64) tpe *= 2;
      const int g0 = tid / tpe, groups = T / tpe;
      for (int k = g0; k - g0 < ne; k += groups) {
        const bool live = k < ne;
        const int EX = live ? cx + 2 * (k % hx) : 0, EY = live ? cy + 2 * (k / hx) : 0;
        constexpr int QL = quad_len<N>();
        double qv[QL];
        coarse_element_part<N>(a, ox, oy, EX, EY, live ? tid % tpe : a.r * a.r, tpe, qv);
        if (tpe > 1) {
#pragma unroll
          for (int c0 = 0; c0 < QL; c0 += 4) {
            double v4[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) v4[t] = c0 + t < QL ? qv[c0 + t] : 0.0;
            seg_sum_n<4>(v4, tpe);
#pragma unroll
            for (int t = 0; t < 4; ++t)
              if (c0 + t < QL) qv[c0 + t] = v4[t];
          }
        }
        if (!live || tid % tpe != 0) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int Xn = EX + (c & 1), Yn = EY + (c >> 1);
          const int nd = Yn * NCp + Xn;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int dx = (b & 1) - (c & 1), dy = (b >> 1) - (c >> 1);
            nW[nd * 9 + (dy + 1) * 3 + dx + 1] += qv[c * 4 + b];
          }
          const int side = (c & 1) ? 0 : 1;   // element left of the node -> side 0
          const int part = (c >> 1) ? 0 : 1;  // element below the node -> part 0
#pragma unroll
          for (int j = 0; j < N; ++j) nB[((nd * 4) + side * 2 + part) * N + j] += (float)qv[16 + c * N + j];
        }
      }
      __syncthreads();
    }
  } else {
    // fine level on the generic solve kernel: the cell's kappa/6 and label
    // windows for it (a.kw, a.labw; null otherwise)
    double* kwc = a.kw ? a.kw + (size_t)ci * NC * NC : nullptr;
    uint8_t* lwc = a.labw ? a.labw + (size_t)ci * NC * NC : nullptr;
    for (int e = tid; e < NC * NC; e += T) {
      const int EX = e % NC, EY = e / NC;
      const size_t ge = (size_t)wrap1(oy + EY, a.n) * a.n + wrap1(ox + EX, a.n);
      labS[e] = a.label[ge];
      if (kwc) {
        kwc[e] = a.kappa[ge] * (1.0 / 6.0);
        lwc[e] = a.label[ge];
      }
    }
  }
  // 1/D at free level node (Xn, Yn): the Galerkin diagonal, or on the fine
  // level D = 4*(((SW + SE) + NW) + NE) of kappa/6 (the solve kernels' order;
  // elements outside the cell count 0)
  auto inv_d = [&](int Xn, int Yn) -> double {
    if (gal) return 1.0 / nW[(Yn * NCp + Xn) * 9 + 4];
    auto kq = [&](int ex, int ey) {
      if (ex < 0 || ey < 0 || ex >= NC || ey >= NC) return 0.0;
      return a.kappa[(size_t)wrap1(oy + ey, a.n) * a.n + wrap1(ox + ex, a.n)] * (1.0 / 6.0);
    };
    const double ks = kq(Xn - 1, Yn - 1) + kq(Xn, Yn - 1) + kq(Xn - 1, Yn) + kq(Xn, Yn);
    return 1.0 / (4.0 * ks);
  };
  // sub-block of every level element
  for (int e = tid; e < NC * NC; e += T) regS[e] = (uint8_t)(((e / NC) / sbw) * s + (e % NC) / sbw);
  __syncthreads();

  // ---- S = B_n D^-1 B_n^T --------------------------------------------------
  // One wave per pair of adjacent sub-blocks qa <= qb (blocks of sub-blocks
  // further apart are zero): its lanes visit the level nodes the two share
  // (the whole sub-block when qa = qb), take per continuum the weight of the
  // node's elements in qa and in qb (element counts, or the Galerkin weights),
  // and accumulate all N x N products times 1/D; a wave sum in fixed order
  // gives the block, scaled by the row weights.
  for (int k = tid; k < m * m; k += T) S[k] = 0.0;
  __syncthreads();
  for (int t = wave; t < s * s * 9; t += T / 64) {
    const int qa = t / 9, d9 = t % 9;
    const int qax = qa % s, qay = qa / s;
    const int qbx = qax + d9 % 3 - 1, qby = qay + d9 / 3 - 1;
    if (qbx < 0 || qby < 0 || qbx >= s || qby >= s) continue;  // uniform across the wave
    const int qb = qby * s + qbx;
    if (qb < qa) continue;
    const int X0 = max(max(qax, qbx) * sbw, lo), X1 = min((min(qax, qbx) + 1) * sbw, hi);
    const int Y0 = max(max(qay, qby) * sbw, lo), Y1 = min((min(qay, qby) + 1) * sbw, hi);
    const int wX = X1 - X0 + 1, wY = Y1 - Y0 + 1;
    double acc[N * N];
#pragma unroll
    for (int k = 0; k < N * N; ++k) acc[k] = 0.0;
    const int nodes = (wX > 0 && wY > 0) ? wX * wY : 0;
    for (int k = lane; k < nodes; k += 64) {
      const int Xn = X0 + k % wX, Yn = Y0 + k / wX;
      double ba[N], bb[N];
#pragma unroll
      for (int j = 0; j < N; ++j) ba[j] = bb[j] = 0.0;
#pragma unroll
      for (int Qd = 0; Qd < 4; ++Qd) {
        const int EX = Xn - 1 + (Qd & 1), EY = Yn - 1 + (Qd >> 1);
        if (EX < 0 || EY < 0 || EX >= NC || EY >= NC) continue;  // outside the cell (Neumann boundary)
        const int qE = regS[EY * NC + EX];
        if (!gal) {
          const int lab = labS[EY * NC + EX];
#pragma unroll
          for (int j = 0; j < N; ++j) {
            if (qE == qa && lab == j) ba[j] += 1.0;
            if (qE == qb && lab == j) bb[j] += 1.0;
          }
        } else {
          const int side = Qd & 1, part = Qd >> 1;
          const float* w4 = nB + ((Yn * NCp + Xn) * 4 + side * 2 + part) * N;
#pragma unroll
          for (int j = 0; j < N; ++j) {
            const double wj = (double)w4[j];
            if (qE == qa) ba[j] += wj;
            if (qE == qb) bb[j] += wj;
          }
        }
      }
      const double id = inv_d(Xn, Yn);
#pragma unroll
      for (int j = 0; j < N; ++j)
#pragma unroll
        for (int j2 = 0; j2 < N; ++j2) acc[j * N + j2] += ba[j] * bb[j2] * id;
    }
    wave_sum_n<N * N>(acc);
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < N; ++j)
#pragma unroll
        for (int j2 = 0; j2 < N; ++j2) {
          const int ra = qa * N + j, rb = qb * N + j2;
          const double v = cwp[ra] * cwp[rb] * acc[j * N + j2];
          S[ra * m + rb] = v;
          S[rb * m + ra] = v;
        }
    }
  }
  __syncthreads();

  // ---- band coarse correction of the preconditioner -----------------------
  // The solve kernel preconditions with G^-1 = D^-1 + sum_b Z_b T_b^-1 Z_b^T
  // (bands of prec_rows node rows, one coarse unknown per node column of a
  // band; see the kernel), so its Schur matrix is B G^-1 B^T: add
  // (B Z_b) T_b^-1 (B Z_b)^T per band. T_b (tridiagonal over the node
  // columns; column 0 is the Dirichlet boundary, an identity row) is reduced
  // as in the kernel, one row per lane in groups of NC lanes, with the same
  // factors to the last bit, and its inverse applied to each active
  // constraint row's band sums (B Z_b)^T.
  if (prec) {
    const int R = a.prec_rows;
    // K_n entries of level node (X, Y): centre, north, south, east,
    // north-east, south-east
    auto stencil_at = [&](int X, int Y, double (&k6)[6]) {
      if (gal) {
        const double* w9 = nW + (size_t)(Y * NCp + X) * 9;
        k6[0] = w9[4];
        k6[1] = w9[7];
        k6[2] = w9[1];
        k6[3] = w9[5];
        k6[4] = w9[8];
        k6[5] = w9[2];
      } else {
        auto kq = [&](int ex, int ey) {
          return a.kappa[(size_t)wrap1(oy + ey, a.n) * a.n + wrap1(ox + ex, a.n)] * (1.0 / 6.0);
        };
        fine_stencil6(kq(X - 1, Y - 1), kq(X, Y - 1), kq(X - 1, Y), kq(X, Y), k6);
      }
    };
    // constraint weight of level node (X, Y) for sub-block q and continuum j
    // (no row factor), as in S above
    auto node_weight = [&](int X, int Y, int q, int j) -> double {
      double w = 0.0;
      for (int Qd = 0; Qd < 4; ++Qd) {
        const int EX = X - 1 + (Qd & 1), EY = Y - 1 + (Qd >> 1);
        if (regS[EY * NC + EX] != q) continue;
        if (!gal) {
          w += (labS[EY * NC + EX] == j) ? 1.0 : 0.0;
        } else {
          const int side = Qd & 1, part = Qd >> 1;
          w += (double)nB[((Y * NCp + X) * 4 + side * 2 + part) * N + j];
        }
      }
      return w;
    };
    // Per band only the rows of sub-blocks whose node rows meet the band's
    // carry weight there (act[], at most NA of them, inv[] the inverse map);
    // PREC_GROUP bands at a time, each with its own slices of BZ, Ys, Fs, IBs
    // and the NC lanes tid / NC == g.
    int NA, G;
    prec_group_sizes(a, &NA, &G);
    __shared__ int act[PREC_GROUP][64];
    __shared__ int inv[PREC_GROUP][64];
    __shared__ int n_act[PREC_GROUP];
    for (int b0 = 0; b0 < nbands; b0 += G) {
      const int gb = min(G, nbands - b0);
      if (tid < gb) {
        const int yb0 = (b0 + tid) * R;
        int na = 0;
        for (int k = 0; k < m; ++k) {
          const int qy = (k / N) / s;
          inv[tid][k] = -1;
          if (cwp[k] != 0.0 && qy * sbw <= yb0 + R - 1 && (qy + 1) * sbw >= yb0) {
            inv[tid][k] = na;
            act[tid][na++] = k;
          }
        }
        // the bound NA holds by construction; if it did not, the cell would
        // be reported singular rather than solved with a truncated correction
        if (na > NA) singular = 1;
        n_act[tid] = na < NA ? na : NA;
      }
      // row X of T_b, then its cyclic reduction (the lanes of a group are
      // consecutive threads of one wave, NC <= 64)
      if (tid < gb * NC) {
        const int g = tid / NC, X = tid % NC, yb0 = (b0 + g) * R;
        double td = 0.0, tc = 0.0;
        for (int i = 0; i < R; ++i) {
          const int Y = yb0 + i;
          const bool fr = X >= 1 && Y >= 1, frE = X + 1 <= NC - 1 && Y >= 1;
          const bool upIn = i + 1 < R, dnIn = i >= 1 && Y - 1 >= 1;
          if (!fr) continue;
          double k6[6];
          stencil_at(X, Y, k6);
          band_row_add(td, tc, frE, upIn, dnIn, k6[0], k6[1], k6[2], k6[3], k6[4], k6[5]);
        }
        if (X == 0) {
          td = 1.0;
          tc = 0.0;
        }
        double ta = __shfl_up(tc, 1, NC);  // T[X][X-1] = T[X-1][X]
        if (X == 0) ta = 0.0;
        double* blk = Fs + g * pcb;
        IBs[g * NC + X] = pcr_factor(X, NC, logNC, ta, td, tc, [&](int k, bool hasL, bool hasR, double al, double ga) {
          double* stp = blk + pcr_offset(NC, k);
          const int st = 1 << k;
          if (hasL) stp[X - st] = al;
          if (hasR) stp[(NC - st) + X] = ga;
        });
      }
      __syncthreads();
      for (int e = tid; e < gb * NA * NC; e += T) {
        const int g = e / (NA * NC), ia = (e / NC) % NA, X = e % NC;
        if (ia >= n_act[g]) continue;
        const int k = act[g][ia], q = k / N, j = k % N, qx = q % s, yb0 = (b0 + g) * R;
        double acc = 0.0;
        if (X >= 1 && X >= qx * sbw && X <= (qx + 1) * sbw) {
          for (int i = 0; i < R; ++i) {
            const int Y = yb0 + i;
            if (Y >= 1) acc += node_weight(X, Y, q, j);
          }
        }
        BZ[e] = cwp[k] * acc;
      }
      __syncthreads();
      // Ys = T_b^-1 BZ, one active row at a time per group of lanes
      if (tid < gb * NC) {
        const int g = tid / NC, X = tid % NC;
        const double* blk = Fs + g * pcb;
        const double ib = IBs[g * NC + X];
        for (int ia = 0; ia < n_act[g]; ++ia) {
          double d = BZ[(g * NA + ia) * NC + X];
          for (int k = 0; k < logNC; ++k) {
            const int st = 1 << k;
            const double* stp = blk + pcr_offset(NC, k);
            const double dL = __shfl_up(d, st, NC), dR = __shfl_down(d, st, NC);
            const double al = (X >= st) ? stp[X - st] : 0.0;
            const double ga = (X + st < NC) ? stp[(NC - st) + X] : 0.0;
            d = pcr_rhs(d, al, dL, ga, dR);
          }
          Ys[(g * NA + ia) * NC + X] = d * ib;
        }
      }
      __syncthreads();
      for (int e = tid; e < m * m; e += T) {
        const int k = e / m, k2 = e % m;
        double acc = 0.0;
        for (int g = 0; g < gb; ++g) {
          const int ia = inv[g][k], ib = inv[g][k2];
          if (ia < 0 || ib < 0) continue;
          const double* bz = BZ + (size_t)(g * NA + ia) * NC;
          const double* ys = Ys + (size_t)(g * NA + ib) * NC;
          for (int X = 0; X < NC; ++X) acc += bz[X] * ys[X];
        }
        S[e] += acc;
      }
      __syncthreads();
    }
  }

  // ---- S^-1 in place by Gauss-Jordan elimination; inactive rows get 1 -----
  // Pivot k: p = S_kk; row k becomes S_kj / p, column k becomes -S_ik / p,
  // the pivot 1 / p, and S_ij -= S_ik S_kj / p elsewhere. S is symmetric
  // positive definite, so every pivot is positive without row exchanges.
  for (int k = tid; k < m; k += T)
    if (cwp[k] == 0.0) S[k * m + k] = 1.0;
  double* rowk = X;       // S_kj / p
  double* colk = X + m;   // S_ik
  for (int k = 0; k < m; ++k) {
    __syncthreads();
    const double piv = S[k * m + k];
    if (!(piv > 0.0) && tid == 0) singular = 1;
    const double ip = piv > 0.0 ? 1.0 / piv : 1.0;
    for (int j = tid; j < m; j += T) {
      rowk[j] = S[k * m + j] * ip;
      colk[j] = S[j * m + k];
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += T) {
      const int i = e / m, j = e % m;
      double v;
      if (i == k)
        v = (j == k) ? ip : rowk[j];
      else if (j == k)
        v = -colk[i] * ip;
      else
        v = S[e] - colk[i] * rowk[j];
      S[e] = v;
    }
  }
  __syncthreads();
  const bool bad = singular != 0;
  for (int k = tid; k < m * m; k += T) a.sinv[(size_t)p * m * m + k] = bad ? __builtin_nan("") : S[k];
}

// Whether the inherit kernel sums B_h I in its element pass: its per-element
// sums (NC^2 N values) and the corner sums of f (4 NC^2) fit the LDS.
__host__ __device__ inline bool inherit_fused(int NC, int N) {
  return (size_t)NC * NC * (4 + N) * sizeof(double) <= 160 * 1024;
}

// Inherited right-hand sides of a level >= 2 cell, one workgroup per
// (cell, alpha): f = -P^T K_h I on the level nodes and g' = g - B_h I, with I
// the inherited level-1 solution. f is formed element by element: a fine
// element's K_e I_e (its four corner values) goes to the four corners of the
// level element containing it with the bilinear weights of its corners, so
// each fine element is visited once (kappa and I straight from global
// memory). The level elements are split over groups of lanes, whose partial
// corner sums are reduced with DPP into LDS; a level node then adds the
// corners of its (up to four) level elements in a fixed order. The same pass
// sums I over each fine element per continuum (B_h I): a level element lies
// in one sub-block, so its per-continuum sums go to LDS too and each
// constraint row adds those of its sub-block's level elements in order.
template <int N>
__global__ __launch_bounds__(SETUP_T) void k_inherit2d(CellArgs a) {
  extern __shared__ double Fc[];  // [NC^2][4] corner sums of f, then (fused) [NC^2][N] element sums of I
                                  // per continuum, or [s*s][NW][N] wave partials of B_h I
  constexpr int NW = SETUP_T / 64;
  const int nc = a.nc, nn1 = nc + 1, NC = a.NC, r = a.r, m = a.m, s = a.s, M = a.M;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // B_h I in the element pass unless the per-element sums would not fit the
  // LDS (level cells of 64^2 elements); then in a pass of its own
  const bool fused = inherit_fused(NC, N);
  const int ci = a.ci0 + blockIdx.x / M, al = blockIdx.x % M;
  const int p = a.cells[ci];
  const int jx = p % a.n_macro, jy = p / a.n_macro;
  const int ox = a.H * jx + a.H / 2 - nc / 2, oy = a.H * jy + a.H / 2 - nc / 2;
  const double* I = a.phi1 + ((size_t)a.pslot[ci] * M + al) * (size_t)nn1 * nn1;
  const double inv_r = 1.0 / r;
  const int NCp = NC + 1, L2e = NC * NC;
  double* fo = a.fin + ((size_t)ci * M + al) * NCp * NCp;
  double* Eb = Fc + (size_t)L2e * 4;
  double* wred = Eb;
  // free level nodes [lo, hi]^2
  const int lo = a.bc ? 0 : 1, hi = a.bc ? NC : NC - 1;
  // lanes per level element: the largest power of two with L2e groups fitting
  // the workgroup (1 when there are more level elements than lanes)
  int tpe = 1;
  while (tpe * 2 * L2e <= SETUP_T && tpe < 64) tpe *= 2;
  const int groups = SETUP_T / tpe;
  for (int E0 = tid / tpe; E0 - tid / tpe < L2e; E0 += groups) {
    // every lane of a group runs the same trip; groups past the last level
    // element contribute nothing
    const bool live = E0 < L2e;
    const int EX = live ? E0 % NC : 0, EY = live ? E0 / NC : 0;
    // corner sums of f (4), then element sums of I per continuum (N)
    double fc[4 + N];
#pragma unroll
    for (int t = 0; t < 4 + N; ++t) fc[t] = 0.0;
    for (int k = tid % tpe; live && k < r * r; k += tpe) {
      const int u = k % r, v = k / r;
      const int ex = EX * r + u, ey = EY * r + v;
      const size_t ge = (size_t)wrap1(oy + ey, a.n) * a.n + wrap1(ox + ex, a.n);
      const double k6 = a.kappa[ge] * (1.0 / 6.0);
      const int lab = a.label[ge];
      double Iv[4], y[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) Iv[d] = I[(size_t)(ey + (d >> 1)) * nn1 + ex + (d & 1)];
      const double es = (Iv[0] + Iv[1]) + (Iv[2] + Iv[3]);
#pragma unroll
      for (int j = 0; j < N; ++j) fc[4 + j] += (lab == j) ? es : 0.0;
      kref6_apply(Iv, y);
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const double tx = (u + (d & 1)) * inv_r, ty = (v + (d >> 1)) * inv_r;
        const double yd = k6 * y[d];
        fc[0] += (1.0 - tx) * (1.0 - ty) * yd;
        fc[1] += tx * (1.0 - ty) * yd;
        fc[2] += (1.0 - tx) * ty * yd;
        fc[3] += tx * ty * yd;
      }
    }
    if (tpe > 1) seg_sum_n<4 + N>(fc, tpe);
    if (live && tid % tpe == 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) Fc[(size_t)E0 * 4 + c] = fc[c];
      if (fused) {
#pragma unroll
        for (int j = 0; j < N; ++j) Eb[(size_t)E0 * N + j] = fc[4 + j];
      }
    }
  }
  __syncthreads();
  for (int nd = tid; nd < NCp * NCp; nd += SETUP_T) {
    const int Xn = nd % NCp, Yn = nd / NCp;
    double acc = 0.0;
    if (Xn >= lo && Yn >= lo && Xn <= hi && Yn <= hi) {
      // node (Xn, Yn) is corner c of level element (Xn - cx, Yn - cy)
#pragma unroll
      for (int c = 3; c >= 0; --c) {
        const int EX = Xn - (c & 1), EY = Yn - (c >> 1);
        if (EX < 0 || EY < 0 || EX >= NC || EY >= NC) continue;
        acc += Fc[((size_t)EY * NC + EX) * 4 + c];
      }
    }
    fo[nd] = -acc;
  }
  if (!fused) {
    // B_h I: element sums of I per sub-block and continuum, wave partials
    const int sb = nc / s;
    for (int reg = 0; reg < s * s; ++reg) {
      const int x0 = (reg % s) * sb, y0 = (reg / s) * sb;
      double acc[N];
#pragma unroll
      for (int j = 0; j < N; ++j) acc[j] = 0.0;
      for (int k = tid; k < sb * sb; k += SETUP_T) {
        const int ex = x0 + k % sb, ey = y0 + k / sb;
        const int lab = a.label[(size_t)wrap1(oy + ey, a.n) * a.n + wrap1(ox + ex, a.n)];
        const double es = (I[(size_t)ey * nn1 + ex] + I[(size_t)ey * nn1 + ex + 1]) +
                          (I[(size_t)(ey + 1) * nn1 + ex] + I[(size_t)(ey + 1) * nn1 + ex + 1]);
#pragma unroll
        for (int j = 0; j < N; ++j) acc[j] += (lab == j) ? es : 0.0;
      }
      wave_sum_n<N>(acc);
      if (lane == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) wred[(reg * NW + wave) * N + j] = acc[j];
      }
    }
    __syncthreads();
  }
  // B_h I per constraint row: (fused) the sums of the sub-block's level
  // elements, one wave per row with a fixed-order wave sum, or the waves'
  // partials in order
  const int sbw = a.sbw;
  if (fused) {
    for (int k = wave; k < m; k += NW) {
      const int q = k / N, j = k % N, qx = q % s, qy = q / s;
      double bI = 0.0;
      for (int e = lane; e < sbw * sbw; e += 64)
        bI += Eb[((size_t)(qy * sbw + e / sbw) * NC + qx * sbw + e % sbw) * N + j];
      bI = wave_sum(bI);
      if (lane == 0)
        a.gin[((size_t)ci * M + al) * m + k] = a.g[((size_t)p * M + al) * m + k] - a.cw[(size_t)p * m + k] * bI;
    }
  } else {
    for (int k = tid; k < m; k += SETUP_T) {
      const int q = k / N, j = k % N;
      double bI = 0.0;
      for (int w2 = 0; w2 < NW; ++w2) bI += wred[(q * NW + w2) * N + j];
      a.gin[((size_t)ci * M + al) * m + k] = a.g[((size_t)p * M + al) * m + k] - a.cw[(size_t)p * m + k] * bI;
    }
  }
}

static size_t setup_lds_bytes(const CellArgs& a, int threads) {
  size_t d = (size_t)a.m * a.m + 2 * (size_t)a.m + (size_t)(a.s * a.s + 1) * a.N * 3 + (threads / 64) * a.N * 3;
  if (a.prec_rows > 0) {
    int NA, G;
    prec_group_sizes(a, &NA, &G);
    int lg = 0;
    while ((1 << (lg + 1)) <= a.NC) ++lg;
    d += 2 * (size_t)G * NA * a.NC + (size_t)G * (pcr_offset(a.NC, lg) + a.NC);
  }
  // labels and sub-block per element (bytes)
  return d * sizeof(double) + 2 * (size_t)a.NC * a.NC;
}

template <typename F>
static int lds_attr(F fn, size_t lds) {
  if (lds > 160 * 1024) return set_error(MCH_EINVAL, "kernel exceeds the LDS budget");
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute");
  }
  return MCH_OK;
}

// Threads of the set-up workgroup: a level of few cells (the fine level of a
// small macrogrid, whose set-up precedes its solve on the critical path) gets
// 1024 so that the workgroups still fill much of the GPU.
static int setup_threads(const CellArgs& a) {
  static const int wide = [] {
    const char* v = std::getenv("MCH_SETUP_WIDE");
    return v ? std::atoi(v) : 1;
  }();
  return (wide && a.count <= 128) ? 1024 : SETUP_T;
}

int launch_setup(const CellArgs& a, hipStream_t s) {
  const int threads = setup_threads(a);
  const size_t lds = setup_lds_bytes(a, threads);
  void (*fn)(CellArgs) = nullptr;
#define MCH_SETUP(n_)                                              \
  if (a.N == n_) fn = threads == 1024 ? k_setup2d<n_, 1024> : k_setup2d<n_, SETUP_T>;
  MCH_SETUP(1) MCH_SETUP(2) MCH_SETUP(3)
#undef MCH_SETUP
  if (!fn) return set_error(MCH_ENOTIMPL, "n_cont");
  int rc = lds_attr(fn, lds);
  if (rc) return rc;
  hipLaunchKernelGGL(fn, dim3(a.count), dim3(threads), lds, s, a);
  return hip_check(hipGetLastError(), "launch k_setup2d");
}

int launch_inherit(const CellArgs& a, hipStream_t s) {
  if (a.m > 64) return set_error(MCH_ENOTIMPL, "more than 64 constraint rows");
  void (*fn)(CellArgs) = nullptr;
  if (a.N == 1) fn = k_inherit2d<1>;
  if (a.N == 2) fn = k_inherit2d<2>;
  if (a.N == 3) fn = k_inherit2d<3>;
  if (!fn) return set_error(MCH_ENOTIMPL, "n_cont");
  const size_t L2e = (size_t)a.NC * a.NC;
  const size_t lds = (L2e * 4 + (inherit_fused(a.NC, a.N) ? L2e * a.N : (size_t)a.s * a.s * (SETUP_T / 64) * a.N)) *
                     sizeof(double);
  int rc = lds_attr(fn, lds);
  if (rc) return rc;
  hipLaunchKernelGGL(fn, dim3(a.count * a.M), dim3(SETUP_T), lds, s, a);
  return hip_check(hipGetLastError(), "launch k_inherit2d");
}

}  // namespace mch
