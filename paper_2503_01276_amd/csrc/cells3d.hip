// 3D cell kernels for gfx950: per-cell setup, inherited right-hand sides,
// the constrained Krylov solve of every (cell, right-hand side), Phi on K_p,
// effective tensors, the adjoint gradient and the local-solution test hook.
//
// Same method as the 2D kernels (paper Sec. 2, Eqs. phi_avar / phi_grad;
// Sec. 3.3, Eqs. phi_avar_corrector / phi_grad_corrector; Eq. Bs_defi) on Q1
// hexahedra. The trilinear element matrix of the Laplacian couples a corner
// with itself (4h/12), with its three face-diagonal corners and with its
// body-diagonal corner (-h/12 each); edge-adjacent corners do not couple, so
// a fine node has a 21-point stencil. Corners are in tensor order
// c = cx + 2 cy + 4 cz; the face diagonals of c are c^3, c^5, c^6 and its body
// diagonal is c^7.
//
// A fine 3D cell (32^3 elements, 29,791 unknowns per right-hand side) does
// not fit in the LDS and registers of one CU, so the Krylov vectors of each
// (cell, rhs) live in global memory and the workgroup streams them twice per
// iteration (L2 / MALL / HBM). Reductions, the per-wave Schur solve and the
// constraint bookkeeping follow the 2D kernel; every reduction runs in a fixed
// order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <type_traits>
#include <vector>

#include "kernels2d.h"

namespace mch {

constexpr int T3 = 256;   // threads of the set-up and auxiliary kernels
constexpr int S3D = 2;    // constraint sub-blocks per axis handled by the 3D solve

MCH_DEV size_t nidx3(int X, int Y, int Z, int NP) {
  return (size_t)X + (size_t)NP * ((size_t)Y + (size_t)NP * (size_t)Z);
}

MCH_DEV void cell_origin3(const CellArgs& a, int p, int& ox, int& oy, int& oz) {
  const int nm = a.n_macro;
  const int jx = p % nm, jy = (p / nm) % nm, jz = p / (nm * nm);
  ox = a.H * jx + a.H / 2 - a.nc / 2;
  oy = a.H * jy + a.H / 2 - a.nc / 2;
  oz = a.H * jz + a.H / 2 - a.nc / 2;
}

// Global element index of cell-local element (ex, ey, ez), periodic wrap.
MCH_DEV size_t gel3(const CellArgs& a, int ox, int oy, int oz, int ex, int ey, int ez) {
  const int n = a.n;
  return ((size_t)wrap1(oz + ez, n) * n + (size_t)wrap1(oy + ey, n)) * n + (size_t)wrap1(ox + ex, n);
}

// y = (12/h) K_ref v for one hexahedron.
MCH_DEV void kref12_apply(const double (&v)[8], double (&y)[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c) y[c] = 4.0 * v[c] - v[c ^ 3] - v[c ^ 5] - v[c ^ 6] - v[c ^ 7];
}

// Trilinear weight of coarse corner `a` at the point (tx, ty, tz) of a coarse element.
MCH_DEV double tri_w(int a, double tx, double ty, double tz) {
  return ((a & 1) ? tx : 1.0 - tx) * (((a >> 1) & 1) ? ty : 1.0 - ty) * ((a >> 2) ? tz : 1.0 - tz);
}

// Trilinear prolongation of a level-r vector v [(NC+1)^3] to fine node (X, Y, Z).
MCH_DEV double prolong3(const double* v, int r, int NC, int X, int Y, int Z) {
  const int NP = NC + 1;
  if (r == 1) return v[nidx3(X, Y, Z, NP)];
  const int cx = X / r, cy = Y / r, cz = Z / r;
  const double tx = (X - cx * r) / (double)r, ty = (Y - cy * r) / (double)r, tz = (Z - cz * r) / (double)r;
  const int cx1 = cx + (tx > 0.0 ? 1 : 0), cy1 = cy + (ty > 0.0 ? 1 : 0), cz1 = cz + (tz > 0.0 ? 1 : 0);
  const double v000 = v[nidx3(cx, cy, cz, NP)], v100 = v[nidx3(cx1, cy, cz, NP)];
  const double v010 = v[nidx3(cx, cy1, cz, NP)], v110 = v[nidx3(cx1, cy1, cz, NP)];
  const double v001 = v[nidx3(cx, cy, cz1, NP)], v101 = v[nidx3(cx1, cy, cz1, NP)];
  const double v011 = v[nidx3(cx, cy1, cz1, NP)], v111 = v[nidx3(cx1, cy1, cz1, NP)];
  const double a0 = (1 - tx) * v000 + tx * v100, a1 = (1 - tx) * v010 + tx * v110;
  const double a2 = (1 - tx) * v001 + tx * v101, a3 = (1 - tx) * v011 + tx * v111;
  const double b0 = (1 - ty) * a0 + ty * a1, b1 = (1 - ty) * a2 + ty * a3;
  return (1 - tz) * b0 + tz * b1;
}

// Fine local solution Phi_alpha = I + P xi of cell ci of this level at fine
// node (X, Y, Z) in [0, nc]^3. Level 1 stores Phi itself.
MCH_DEV double phi_at3(const CellArgs& a, int ci, int alpha, int X, int Y, int Z) {
  const int nn1 = a.nc + 1;
  const size_t nn = (size_t)nn1 * nn1 * nn1;
  if (a.r == 1) return a.out[((size_t)ci * a.M + alpha) * nn + nidx3(X, Y, Z, nn1)];
  const double* I = a.phi1 + ((size_t)a.pslot[ci] * a.M + alpha) * nn;
  const size_t NN = (size_t)(a.NC + 1) * (a.NC + 1) * (a.NC + 1);
  const double* xi = a.out + ((size_t)ci * a.M + alpha) * NN;
  return I[nidx3(X, Y, Z, nn1)] + prolong3(xi, a.r, a.NC, X, Y, Z);
}

// ---------------------------------------------------------------------------
// Set-up (one workgroup per cell of a level): constraint statistics, cw and g;
// fine level: kappa*h/12 and label windows; Galerkin level: 27-point stencil
// and per-octant constraint weights of every level node; D^-1;
// S = B_n D^-1 B_n^T and S^-1 by Cholesky.
// ---------------------------------------------------------------------------
template <int N, int TB>
__global__ __launch_bounds__(TB) void k_setup3d(CellArgs a) {
  extern __shared__ double sm[];
  const int m = a.m, s = a.s, nc = a.nc, NC = a.NC, sbw = a.sbw, r = a.r, H = a.H;
  const bool gal = r > 1;
  const int s3 = s * s * s;
  const int npairs = m * (m + 1) / 2;
  double* S = sm;                            // m*m
  double* Xm = S + m * m;                    // m*m
  double* stat = Xm + m * m;                 // (s3+1)*N*4
  double* wred = stat + (s3 + 1) * N * 4;    // (TB/64)*N*4
  double* partS = wred + (TB / 64) * N * 4;  // npairs * node planes
  __shared__ int singular;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ci = a.ci0 + blockIdx.x;
  const int p = a.cells[ci];
  int ox, oy, oz;
  cell_origin3(a, p, ox, oy, oz);
  if (tid == 0) singular = 0;

  // ---- constraint statistics per region (sub-blocks, then K_p) -------------
  const int sb = nc / s;
  for (int reg = 0; reg <= s3; ++reg) {
    int x0, y0, z0, w;
    if (reg < s3) {
      x0 = (reg % s) * sb;
      y0 = ((reg / s) % s) * sb;
      z0 = (reg / (s * s)) * sb;
      w = sb;
    } else {
      x0 = y0 = z0 = (nc - H) / 2;
      w = H;
    }
    double acc[N][4];
#pragma unroll
    for (int j = 0; j < N; ++j) acc[j][0] = acc[j][1] = acc[j][2] = acc[j][3] = 0.0;
    for (int k = tid; k < w * w * w; k += TB) {
      const int ex = x0 + k % w, ey = y0 + (k / w) % w, ez = z0 + k / (w * w);
      const int lab = a.label[gel3(a, ox, oy, oz, ex, ey, ez)];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if (lab == j) {
          acc[j][0] += 1.0;
          acc[j][1] += ex + 0.5;
          acc[j][2] += ey + 0.5;
          acc[j][3] += ez + 0.5;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double v = wave_sum(acc[j][t]);
        if (lane == 0) wred[(wave * N + j) * 4 + t] = v;
      }
    __syncthreads();
    if (tid < N * 4) {
      double v = 0.0;
      for (int w2 = 0; w2 < TB / 64; ++w2) v += wred[w2 * N * 4 + tid];
      stat[reg * N * 4 + tid] = v;
    }
    __syncthreads();
  }
  const int M = a.M;
  double* cwp = a.cw + (size_t)p * m;
  if (tid < m) {
    const int k = tid, q = k / N, j = k % N;
    const double cnt = stat[(q * N + j) * 4];
    cwp[k] = cnt > 0.0 ? 1.0 / (8.0 * cnt) : 0.0;
    const double ckp = stat[(s3 * N + j) * 4];
    for (int al = 0; al < M; ++al) {
      double v = 0.0;
      if (cnt > 0.0) {
        if (al < N) {
          v = (al == j) ? 1.0 : 0.0;
        } else {
          const int i = (al - N) / 3, mm = (al - N) % 3;
          if (i == j) {
            const double xbar = stat[(q * N + j) * 4 + 1 + mm] / cnt;
            const double cmj = ckp > 0.0 ? stat[(s3 * N + j) * 4 + 1 + mm] / ckp : nc * 0.5;
            v = (xbar - cmj) * a.h;
          }
        }
      }
      a.g[((size_t)p * M + al) * m + k] = v;
    }
  }

  // ---- level operator data ------------------------------------------------
  // Level nodes stored per axis: NC (the owned [0, NC), node NC a zero
  // boundary) for the column-marching solve, NC + 1 (every node) for the
  // generic one. Free nodes [lo, hi]^3: the interior (Dirichlet) or all
  // (Neumann); octant elements outside the cell weigh nothing.
  const bool gen = a.gen_tp > 0;
  const int NPn = gen ? NC + 1 : NC;
  const int lo = a.bc ? 0 : 1, hi = a.bc ? NC : NC - 1;
  auto is_free = [&](int X, int Y, int Z) {
    return X >= lo && Y >= lo && Z >= lo && X <= hi && Y <= hi && Z <= hi;
  };
  auto el_in = [&](int EX, int EY, int EZ) {
    return EX >= 0 && EY >= 0 && EZ >= 0 && EX < NC && EY < NC && EZ < NC;
  };
  const size_t nodes = (size_t)NPn * NPn * NPn;
  const size_t elems = (size_t)NC * NC * NC;
  double* dinv = a.dinv + (size_t)ci * nodes;
  const double hk = a.h / 12.0;
  if (!gal) {
    double* kwc = a.kw + (size_t)ci * elems;
    uint8_t* lbc = a.labw + (size_t)ci * elems;
    for (int e = tid; e < (int)elems; e += TB) {
      const size_t ge = gel3(a, ox, oy, oz, e % NC, (e / NC) % NC, e / (NC * NC));
      kwc[e] = a.kappa[ge] * hk;
      lbc[e] = a.label[ge];
    }
    __syncthreads();
    // labels of every node's eight octant elements, 2 bits each (3 = none),
    // for the column-marching solve
    uint16_t* octc = gen ? nullptr : a.octw + (size_t)ci * nodes;
    for (int nd = tid; nd < (gen ? 0 : (int)nodes); nd += TB) {
      const int X = nd % NC, Y = (nd / NC) % NC, Z = nd / (NC * NC);
      unsigned code = 0;
      if (X >= 1 && Y >= 1 && Z >= 1) {
        for (int o = 0; o < 8; ++o) {
          const int lab = lbc[(X - 1 + (o & 1)) + NC * ((Y - 1 + ((o >> 1) & 1)) + NC * (Z - 1 + (o >> 2)))];
          code |= (unsigned)(lab < 3 ? lab : 3) << (2 * o);
        }
      }
      octc[nd] = (uint16_t)code;
    }
    for (int nd = tid; nd < (int)nodes; nd += TB) {
      const int X = nd % NPn, Y = (nd / NPn) % NPn, Z = nd / (NPn * NPn);
      if (is_free(X, Y, Z)) {
        double k8[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) {
          const int EX = X - 1 + (o & 1), EY = Y - 1 + ((o >> 1) & 1), EZ = Z - 1 + (o >> 2);
          k8[o] = el_in(EX, EY, EZ) ? kwc[EX + NC * (EY + NC * EZ)] : 0.0;
        }
        // same order as the diagonal of the solve kernel's operator
        dinv[nd] = 1.0 / (4.0 * (((k8[0] + k8[1]) + (k8[2] + k8[3])) + ((k8[4] + k8[5]) + (k8[6] + k8[7]))));
      } else {
        dinv[nd] = 0.0;
      }
    }
  } else {
    double* nW = a.nodeW + (size_t)ci * nodes * 27;
    float* nB = a.nodeB + (size_t)ci * nodes * 8 * N;
    for (int nd = tid; nd < (int)nodes; nd += TB) {
      const int X = nd % NPn, Y = (nd / NPn) % NPn, Z = nd / (NPn * NPn);
      const bool fr = is_free(X, Y, Z);
      double W[27];
      float B8[8][N];
#pragma unroll
      for (int k = 0; k < 27; ++k) W[k] = 0.0;
#pragma unroll
      for (int o = 0; o < 8; ++o)
#pragma unroll
        for (int j = 0; j < N; ++j) B8[o][j] = 0.0f;
      if (fr) {
#pragma unroll
        for (int o = 0; o < 8; ++o) {
          const int ex_ = o & 1, ey_ = (o >> 1) & 1, ez_ = o >> 2;
          const int EX = X - 1 + ex_, EY = Y - 1 + ey_, EZ = Z - 1 + ez_;
          if (!el_in(EX, EY, EZ)) continue;
          const int ac = (1 - ex_) + 2 * (1 - ey_) + 4 * (1 - ez_);  // corner of the node in element o
          for (int wz = 0; wz < r; ++wz)
            for (int wy = 0; wy < r; ++wy)
              for (int wx = 0; wx < r; ++wx) {
                const size_t ge = gel3(a, ox, oy, oz, EX * r + wx, EY * r + wy, EZ * r + wz);
                const double kap = a.kappa[ge];
                const int lab = a.label[ge];
                const int pos = wx + r * (wy + r * wz);
                const double* tk = a.tabK + pos * 64 + ac * 8;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                  const int dx = (b & 1) - (ac & 1), dy = ((b >> 1) & 1) - ((ac >> 1) & 1), dz = (b >> 2) - (ac >> 2);
                  W[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] += kap * tk[b];
                }
                const float rho = (float)a.tabR[pos * 8 + ac];
#pragma unroll
                for (int j = 0; j < N; ++j)
                  if (lab == j) B8[o][j] += rho;
              }
        }
      }
#pragma unroll
      for (int k = 0; k < 27; ++k) nW[(size_t)nd * 27 + k] = W[k];
#pragma unroll
      for (int o = 0; o < 8; ++o)
#pragma unroll
        for (int j = 0; j < N; ++j) nB[((size_t)nd * 8 + o) * N + j] = B8[o][j];
      dinv[nd] = fr ? 1.0 / W[13] : 0.0;
    }
  }
  __syncthreads();

  // ---- S = B_n D^-1 B_n^T: (pair, node plane) partials, fixed-order sums --
  const uint8_t* lbc = gal ? nullptr : a.labw + (size_t)ci * elems;
  const float* nB = gal ? a.nodeB + (size_t)ci * nodes * 8 * N : nullptr;
  for (int item = tid; item < npairs * NPn; item += TB) {
    int pr = item / NPn;
    const int Z = item % NPn;
    int ra = 0;
    while (pr >= m - ra) {
      pr -= m - ra;
      ++ra;
    }
    const int rb = ra + pr;
    const int qa = ra / N, ja = ra % N, qb = rb / N, jb = rb % N;
    const int qax = qa % s, qay = (qa / s) % s, qaz = qa / (s * s);
    const int qbx = qb % s, qby = (qb / s) % s, qbz = qb / (s * s);
    const double cwa = cwp[ra], cwb = cwp[rb];
    double acc = 0.0;
    if (abs(qax - qbx) <= 1 && abs(qay - qby) <= 1 && abs(qaz - qbz) <= 1 && cwa != 0.0 && cwb != 0.0) {
      const int Z0 = max(max(qaz, qbz) * sbw, lo), Z1 = min((min(qaz, qbz) + 1) * sbw, hi);
      if (Z >= Z0 && Z <= Z1) {
        const int X0 = max(max(qax, qbx) * sbw, lo), X1 = min((min(qax, qbx) + 1) * sbw, hi);
        const int Y0 = max(max(qay, qby) * sbw, lo), Y1 = min((min(qay, qby) + 1) * sbw, hi);
        for (int Y = Y0; Y <= Y1; ++Y)
          for (int X = X0; X <= X1; ++X) {
            const size_t nd = (size_t)X + NPn * ((size_t)Y + NPn * (size_t)Z);
            double ba = 0.0, bb = 0.0;
#pragma unroll
            for (int o = 0; o < 8; ++o) {
              const int EX = X - 1 + (o & 1), EY = Y - 1 + ((o >> 1) & 1), EZ = Z - 1 + (o >> 2);
              if (!el_in(EX, EY, EZ)) continue;
              const int qE = EX / sbw + s * (EY / sbw + s * (EZ / sbw));
              double wa, wb;
              if (gal) {
                wa = (double)nB[(nd * 8 + o) * N + ja];
                wb = (double)nB[(nd * 8 + o) * N + jb];
              } else {
                const int lab = lbc[EX + NC * (EY + NC * EZ)];
                wa = (lab == ja) ? 1.0 : 0.0;
                wb = (lab == jb) ? 1.0 : 0.0;
              }
              if (qE == qa) ba += wa;
              if (qE == qb) bb += wb;
            }
            acc += (cwa * ba) * (cwb * bb) * dinv[nd];
          }
      }
    }
    partS[item] = acc;
  }
  __syncthreads();
  for (int pr0 = tid; pr0 < npairs; pr0 += TB) {
    int pr = pr0, ra = 0;
    while (pr >= m - ra) {
      pr -= m - ra;
      ++ra;
    }
    const int rb = ra + pr;
    double acc = 0.0;
    for (int zz = 0; zz < NPn; ++zz) acc += partS[pr0 * NPn + zz];
    S[ra * m + rb] = acc;
    S[rb * m + ra] = acc;
  }
  __syncthreads();

  // ---- Cholesky S = L L^T in place, one wave; inactive rows get 1 ---------
  if (wave == 0) {
    for (int k = lane; k < m; k += 64)
      if (cwp[k] == 0.0) S[k * m + k] = 1.0;
    __builtin_amdgcn_wave_barrier();
    for (int k = 0; k < m; ++k) {
      const double piv = S[k * m + k];
      if (!(piv > 0.0) && lane == 0) singular = 1;
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
    for (int col = lane; col < m; col += 64) {
      for (int i = 0; i < m; ++i) {
        double v = (i == col) ? 1.0 : 0.0;
        for (int jj = col; jj < i; ++jj) v -= S[i * m + jj] * Xm[jj * m + col];
        Xm[i * m + col] = (i >= col) ? v / S[i * m + i] : 0.0;
      }
    }
  }
  __syncthreads();
  const bool bad = singular != 0;
  for (int k = tid; k < m * m; k += TB) {
    const int i = k / m, j = k % m;
    double v = 0.0;
    for (int t = (i > j ? i : j); t < m; ++t) v += Xm[t * m + i] * Xm[t * m + j];
    a.sinv[(size_t)p * m * m + k] = bad ? __builtin_nan("") : v;
  }
}

// ---------------------------------------------------------------------------
// Inherited right-hand sides of a level >= 2 cell (one workgroup per
// (cell, alpha)): f = -P^T K_h I on the level nodes, g' = g - B_h I, with I
// the inherited level-1 solution. Coarse-element load vectors are built one
// element layer at a time in a two-layer LDS ring; a thread owns one coarse
// element column (NC^2 <= T3).
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(T3) void k_inherit3d(CellArgs a) {
  extern __shared__ double sm[];
  const int nc = a.nc, nn1 = nc + 1, NC = a.NC, r = a.r, m = a.m, s = a.s, sbw = a.sbw, M = a.M;
  const int L2 = NC * NC;
  double* F = sm;                 // [2][L2][8]
  double* accR = F + 2 * L2 * 8;  // [T3][2][N]
  const int tid = threadIdx.x;
  const int ci = a.ci0 + blockIdx.x / M, al = blockIdx.x % M;
  const int p = a.cells[ci];
  int ox, oy, oz;
  cell_origin3(a, p, ox, oy, oz);
  const double* I = a.phi1 + ((size_t)a.pslot[ci] * M + al) * (size_t)nn1 * nn1 * nn1;
  // level nodes stored per axis (see the setup) and the free ones
  const int NPn = a.gen_tp > 0 ? NC + 1 : NC;
  const int lo = a.bc ? 0 : 1, hi = a.bc ? NC : NC - 1;
  const size_t nodes = (size_t)NPn * NPn * NPn;
  double* fo = a.fin + ((size_t)ci * M + al) * nodes;
  const double hk = a.h / 12.0, inv_r = 1.0 / r;
  const bool own = tid < L2;
  const int EX = tid % NC, EY = tid / NC;
  double acc[2][N];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < N; ++j) acc[t][j] = 0.0;
  // element layer EZ, then node plane Z = EZ from layers EZ - 1 and EZ
  for (int EZ = 0; EZ <= NC; ++EZ) {
    if (own && EZ < NC) {
      double Fe[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) Fe[c] = 0.0;
      const int qz = EZ / sbw;
      for (int wz = 0; wz < r; ++wz)
        for (int wy = 0; wy < r; ++wy)
          for (int wx = 0; wx < r; ++wx) {
            const int fx = EX * r + wx, fy = EY * r + wy, fz = EZ * r + wz;
            double Iv[8], y[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) Iv[c] = I[nidx3(fx + (c & 1), fy + ((c >> 1) & 1), fz + (c >> 2), nn1)];
            kref12_apply(Iv, y);
            const size_t ge = gel3(a, ox, oy, oz, fx, fy, fz);
            const double kap = a.kappa[ge] * hk;
            const int lab = a.label[ge];
#pragma unroll
            for (int dl = 0; dl < 8; ++dl) {
              const double yd = kap * y[dl];
              const double tx = (wx + (dl & 1)) * inv_r, ty = (wy + ((dl >> 1) & 1)) * inv_r,
                           tz = (wz + (dl >> 2)) * inv_r;
#pragma unroll
              for (int c = 0; c < 8; ++c) Fe[c] += tri_w(c, tx, ty, tz) * yd;
            }
            const double es = ((Iv[0] + Iv[1]) + (Iv[2] + Iv[3])) + ((Iv[4] + Iv[5]) + (Iv[6] + Iv[7]));
#pragma unroll
            for (int j = 0; j < N; ++j) {
              if (lab == j) {
                if (qz == 0)
                  acc[0][j] += es;
                else
                  acc[1][j] += es;
              }
            }
          }
      double* Fl = F + ((size_t)(EZ & 1) * L2 + tid) * 8;
#pragma unroll
      for (int c = 0; c < 8; ++c) Fl[c] = Fe[c];
    }
    __syncthreads();
    const int Z = EZ;
    for (int col = tid; Z < NPn && col < NPn * NPn; col += T3) {
      const int X = col % NPn, Y = col / NPn;
      double t = 0.0;
      if (X >= lo && Y >= lo && Z >= lo && X <= hi && Y <= hi && Z <= hi) {
#pragma unroll
        for (int o = 0; o < 8; ++o) {
          const int ex_ = o & 1, ey_ = (o >> 1) & 1, ez_ = o >> 2;
          const int EXo = X - 1 + ex_, EYo = Y - 1 + ey_, EZo = Z - 1 + ez_;
          if (EXo < 0 || EYo < 0 || EZo < 0 || EXo >= NC || EYo >= NC || EZo >= NC) continue;
          const int layer = EZo & 1;
          const int c = (1 - ex_) + 2 * (1 - ey_) + 4 * (1 - ez_);
          t += F[((size_t)layer * L2 + EYo * NC + EXo) * 8 + c];
        }
      }
      fo[(size_t)X + NPn * ((size_t)Y + NPn * (size_t)Z)] = -t;
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < N; ++j) accR[((size_t)tid * 2 + t) * N + j] = acc[t][j];
  __syncthreads();
  for (int k = tid; k < m; k += T3) {
    const int q = k / N, j = k % N, qx = q % s, qy = (q / s) % s, qz = q / (s * s);
    double bI = 0.0;
    for (int t2 = 0; t2 < L2; ++t2) {
      if ((t2 % NC) / sbw == qx && (t2 / NC) / sbw == qy) bI += accR[((size_t)t2 * 2 + qz) * N + j];
    }
    a.gin[((size_t)ci * M + al) * m + k] = a.g[((size_t)p * M + al) * m + k] - a.cw[(size_t)p * m + k] * bI;
  }
}

// ---------------------------------------------------------------------------
// Constrained solve of one (cell, rhs) per workgroup: projected PCG with the
// constraint preconditioner [D B^T; B 0] and the Gould-Hribar-Nocedal
// residual update, feasible start x0 = D^-1 B^T S^-1 g', two barriers per
// iteration, B D^-1 r' re-projected every ZPERIOD3 iterations.
//
// Thread t owns node column (X, Y) = (t mod NC, (t / NC) mod NC) and the node
// planes Z = g + G i (g = t / NC^2, G = NT / NC^2), so Z is uniform across a
// wave and the constraint regions of a wave's nodes differ only in x and y.
// Vectors x (the output), r, p and K_n p are padded (NC+1)^3 arrays with a
// zero boundary.
// ---------------------------------------------------------------------------
constexpr int ZPERIOD3 = 16;

// At most 512 threads: the sweep bodies need about 250 VGPRs, which a
// 1024-thread workgroup cannot give (it would spill inside the loop). At most
// NC^2 threads, so every thread walks whole node columns plane by plane (one
// plane group), which the z-march below needs.
template <int NC, bool GAL>
constexpr int nt3() {
  return NC * NC >= 512 ? 512 : NC * NC;
}

template <int V>
using IC = std::integral_constant<int, V>;

// At least two waves per SIMD (a smaller workgroup would otherwise let the
// compiler spend the whole register file on one wave).
template <int NC, int N, bool GAL>
__global__ __launch_bounds__((nt3<NC, GAL>())) __attribute__((amdgpu_waves_per_eu(2))) void k_solve3d(CellArgs a) {
  constexpr int NT = nt3<NC, GAL>();
  constexpr int NW = NT / 64;
  constexpr int NP = NC + 1;
  constexpr int NODES = NC * NC * NC;
  constexpr int CPT = NC * NC > NT ? NC * NC / NT : 1;  // node columns per thread
  constexpr int G = NT > NC * NC ? NT / (NC * NC) : 1;  // plane groups
  constexpr int SPT = NC / G;                           // planes per thread
  constexpr int YS = NC / CPT;                          // row stride between a thread's columns
  constexpr int S = S3D;
  constexpr int PARTV = G * NC * 2 * S * S * N;
  constexpr long SY = NP, SZ = (long)NP * NP;
  extern __shared__ double smem[];
  const int m = a.m, M = a.M, sbw = a.sbw, J = a.J;
  const int MS = (m + J - 1) / J;
  double* red = smem;               // 4*NW
  double* part = red + 4 * NW;      // 2*PARTV
  double* sinvL = part + 2 * PARTV; // MS*64 lane-major S^-1
  double* cwS = sinvL + MS * 64;    // m
  double* uW = cwS + m;             // NW*m
  double* vW = uW + NW * m;         // NW*m

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // columns (X, Y0 + c YS), c < CPT; planes Z = g + G i (g uniform across a wave)
  const int X = tid % NC, Y0 = (tid / NC) % YS;
  const int g = __builtin_amdgcn_readfirstlane(tid / (NC * YS));
  // Workgroups are dealt to the XCDs round robin (block b runs on XCD b % 8),
  // and the M right-hand sides of a cell share its operator data (D^-1 and
  // kappa/labels, or the Galerkin weights), which every iteration re-reads.
  // Blocks are therefore numbered so that all right-hand sides of a cell land
  // on one XCD and share its L2: in a group of 8 cells (8 M blocks), block b
  // takes cell b % 8 of the group and right-hand side (b mod 8 M) / 8. The
  // grid is padded to whole groups; padding blocks leave at once.
  const int grp = blockIdx.x / (kXcds * M), rb = blockIdx.x % (kXcds * M);
  const int cl = grp * kXcds + rb % kXcds, alpha = rb / kXcds;
  if (cl >= a.count) return;
  const int ci = a.ci0 + cl;
  const int p = a.cells[ci];
  const size_t vbase = ((size_t)ci * M + alpha) * (size_t)NP * NP * NP;
  double* __restrict__ xv = a.out + vbase;
  double* __restrict__ rv = a.vr + vbase;
  double* __restrict__ pv = a.vp + vbase;
  double* __restrict__ av = a.vap + vbase;
  const double* __restrict__ dinv = a.dinv + (size_t)ci * NODES;
  const double* __restrict__ kwc = GAL ? nullptr : a.kw + (size_t)ci * NODES;
  const uint16_t* __restrict__ octc = GAL ? nullptr : a.octw + (size_t)ci * NODES;
  const double* __restrict__ nW = GAL ? a.nodeW + (size_t)ci * NODES * 27 : nullptr;
  const float* __restrict__ nB = GAL ? a.nodeB + (size_t)ci * NODES * 8 * N : nullptr;
  const int qx0 = (X >= 1 ? X - 1 : 0) / sbw, qx1 = X / sbw;
  auto Yc = [&](int c) { return Y0 + c * YS; };
  auto colfree = [&](int c) { return X >= 1 && Yc(c) >= 1; };

  // Planes of this thread: Z = g + G i (plane 0 is the Dirichlet boundary).
  // The lower octants (elements of layer Z-1) of plane Z lie in constraint
  // region m0 = (Z-1)/sbw and the upper ones in m1 = Z/sbw. A sweep visits the
  // thread's columns one after another and each column's planes in order;
  // consecutive planes with the same (m0, m1) form a segment (at most three).
  // Per-octant sums are kept by octant (oz) and mapped to regions only when a
  // segment ends, so the loop body carries no region logic. Taking the
  // columns one at a time keeps one column's sums and windows in registers
  // rather than all of the thread's.
  const int iFirst = (g == 0) ? 1 : 0;
  auto sweep = [&](auto&& seg_begin, auto&& body, auto&& seg_end) {
#pragma unroll 1
    for (int c = 0; c < CPT; ++c) {
#pragma unroll 1
      for (int i = iFirst; i < SPT; ++i) {
        const int Z = g + G * i;
        const int m0 = (Z - 1) / sbw, m1 = Z / sbw;
        const int Zp = Z - G, Zn = Z + G;
        if (i == iFirst || (Zp - 1) / sbw != m0 || Zp / sbw != m1) seg_begin(c, m0, m1);
        if (colfree(c)) body(c, Z);
        if (i + 1 == SPT || (Zn - 1) / sbw != m0 || Zn / sbw != m1) seg_end(c, m0, m1);
      }
    }
  };
  auto nop3 = [](int, int, int) {};

  for (int k = tid; k < MS * 64; k += NT) {
    const int t = k / 64, L = k % 64, row = L / J, col = L % J + J * t;
    sinvL[k] = (row < m && col < m) ? a.sinv[(size_t)p * m * m + row * m + col] : 0.0;
  }
  for (int k = tid; k < m; k += NT) cwS[k] = a.cw[(size_t)p * m + k];

  // ---- building blocks -------------------------------------------------------
  auto node_of = [&](int Y, int Z) -> size_t { return (size_t)X + NC * ((size_t)Y + NC * (size_t)Z); };

  // (K_n v) at node (X, Y, Z) from the padded global vector v.
  auto applyK = [&](const double* __restrict__ v, int Y, int Z) -> double {
    const long c = (long)nidx3(X, Y, Z, NP);
    if constexpr (!GAL) {
      double k8[8];
#pragma unroll
      for (int o = 0; o < 8; ++o)
        k8[o] = kwc[(X - 1 + (o & 1)) + NC * ((Y - 1 + ((o >> 1) & 1)) + NC * (Z - 1 + (o >> 2)))];
      // plane Z: the four (x, y) diagonals couple through both element layers
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long sx = 2 * (q & 1) - 1, sy = (2 * (q >> 1) - 1) * SY;
        t += (k8[q] + k8[q + 4]) * v[c + sx + sy];
      }
      // planes Z -+ 1: edge-adjacent in-plane offsets and the corners
#pragma unroll
      for (int oz = 0; oz < 2; ++oz) {
        const long sz = (2 * oz - 1) * SZ;
        const double* k4 = k8 + 4 * oz;
        t += (k4[0] + k4[2]) * v[c - 1 + sz] + (k4[1] + k4[3]) * v[c + 1 + sz];
        t += (k4[0] + k4[1]) * v[c - SY + sz] + (k4[2] + k4[3]) * v[c + SY + sz];
        t += k4[0] * v[c - 1 - SY + sz] + k4[1] * v[c + 1 - SY + sz] + k4[2] * v[c - 1 + SY + sz] +
             k4[3] * v[c + 1 + SY + sz];
      }
      const double D = 4.0 * (((k8[0] + k8[1]) + (k8[2] + k8[3])) + ((k8[4] + k8[5]) + (k8[6] + k8[7])));
      return D * v[c] - t;
    } else {
      const double* w = nW + node_of(Y, Z) * 27;
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < 27; ++k) {
        const long o = (long)(k % 3 - 1) + (long)((k / 3) % 3 - 1) * SY + (long)(k / 9 - 1) * SZ;
        t += w[k] * v[c + o];
      }
      return t;
    }
  };

  // Constraint weights of node (X, Y, Z) per octant element and continuum.
  auto node_weights = [&](int Y, int Z, float (&w)[8][N]) {
    if constexpr (!GAL) {
      // one 16-bit load: the labels of the eight octant elements
      const unsigned code = octc[node_of(Y, Z)];
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const unsigned lab = (code >> (2 * o)) & 3u;
#pragma unroll
        for (int j = 0; j < N; ++j) w[o][j] = (lab == (unsigned)j) ? 1.0f : 0.0f;
      }
    } else {
      const float* b = nB + node_of(Y, Z) * 8 * N;
#pragma unroll
      for (int o = 0; o < 8; ++o)
#pragma unroll
        for (int j = 0; j < N; ++j) w[o][j] = b[o * N + j];
    }
  };

  // per column: [ox][oy][oz][continuum]
  using Acc = double[2][2][2][N];

  // acc[ox][oy][oz][j] += w * tv over the node's octants.
  auto accB = [&](Acc& acc, const float (&w)[8][N], double tv) {
#pragma unroll
    for (int o = 0; o < 8; ++o)
#pragma unroll
      for (int j = 0; j < N; ++j) acc[o & 1][(o >> 1) & 1][o >> 2][j] += (double)w[o][j] * tv;
  };

  // Element-column combination and segment sums over each region's columns of
  // the octant sums; the leader lane of every region adds them to the per-(g, Y)
  // partials of B_n tv (without cw) in part[vec], regions m0 (oz = 0) and m1.
  auto flushB = [&](Acc& acc, int c, int vec, int m0, int m1) {
#pragma unroll
    for (int ey_ = 0; ey_ < 2; ++ey_)
#pragma unroll
      for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int j = 0; j < N; ++j) {
          double v = acc[1][ey_][oz][j] + from_right(acc[0][ey_][oz][j], X, NC);
          v = seg_sum(v, sbw);
          const int qz = oz ? m1 : m0;
          if (X % sbw == 0)
            part[vec * PARTV + ((((g * NC + Yc(c)) * 2 + ey_) * S + X / sbw) * S + qz) * N + j] += v;
        }
  };

  // Clear the partials owned by this lane (region leaders) before a sweep.
  auto clear_part = [&](int vec) {
    if (X % sbw == 0) {
      for (int c = 0; c < CPT; ++c)
        for (int ey_ = 0; ey_ < 2; ++ey_)
          for (int qz = 0; qz < S; ++qz)
            for (int j = 0; j < N; ++j)
              part[vec * PARTV + ((((g * NC + Yc(c)) * 2 + ey_) * S + X / sbw) * S + qz) * N + j] = 0.0;
    }
  };

  auto zero_acc = [&](Acc& acc) {
#pragma unroll
    for (int ex_ = 0; ex_ < 2; ++ex_)
#pragma unroll
      for (int ey_ = 0; ey_ < 2; ++ey_)
#pragma unroll
        for (int oz = 0; oz < 2; ++oz)
#pragma unroll
          for (int j = 0; j < N; ++j) acc[ex_][ey_][oz][j] = 0.0;
  };

  // Row k of B_n (vector vec) summed over planes and node rows in fixed order.
  auto zsum = [&](int vec, int k) -> double {
    const int q = k / N, j = k % N, qx = q % S, qy = (q / S) % S, qz = q / (S * S);
    double z = 0.0;
    for (int gg = 0; gg < G; ++gg)
      for (int EY = qy * sbw; EY < (qy + 1) * sbw; ++EY) {
        if (EY + 1 <= NC - 1) z += part[vec * PARTV + ((((gg * NC + EY + 1) * 2 + 0) * S + qx) * S + qz) * N + j];
        z += part[vec * PARTV + ((((gg * NC + EY) * 2 + 1) * S + qx) * S + qz) * N + j];
      }
    return z;
  };

  // Per wave: v = S^-1 u for u in uW[wave]; vW[wave] = v*cw; returns v.u and
  // v_k in *vk for the lane holding row k.
  auto wave_schur = [&](double* vk) -> double {
    __builtin_amdgcn_wave_barrier();
    const int k = lane / J, jj = lane % J;
    const double* u = uW + wave * m;
    double sum = 0.0;
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

  // cw*v of the octant regions of column c for a segment.
  auto load_vs = [&](Acc& vs, int c, int m0, int m1) {
    const double* vv = vW + wave * m;
    const int Y = Yc(c);
    const int qy0 = (Y >= 1 ? Y - 1 : 0) / sbw, qy1 = Y / sbw;
#pragma unroll
    for (int ex_ = 0; ex_ < 2; ++ex_)
#pragma unroll
      for (int ey_ = 0; ey_ < 2; ++ey_)
#pragma unroll
        for (int oz = 0; oz < 2; ++oz)
#pragma unroll
          for (int j = 0; j < N; ++j) {
            const int qx = ex_ ? qx1 : qx0, qy = ey_ ? qy1 : qy0, qz = oz ? m1 : m0;
            vs[ex_][ey_][oz][j] = vv[((qz * S + qy) * S + qx) * N + j];
          }
  };

  // (B_n^T cw v) at a node.
  auto scatB = [&](const Acc& vs, const float (&w)[8][N]) -> double {
    double t = 0.0;
#pragma unroll
    for (int o = 0; o < 8; ++o)
#pragma unroll
      for (int j = 0; j < N; ++j) t += (double)w[o][j] * vs[o & 1][(o >> 1) & 1][o >> 2][j];
    return t;
  };

  // Right-hand side f at node (X, Y, Z).
  const int nn1 = a.nc + 1;
  auto rhs = [&](int Y, int Z) -> double {
    if (!a.adjoint) {
      if constexpr (GAL) return a.fin[((size_t)ci * M + alpha) * NODES + node_of(Y, Z)];
      return 0.0;
    }
    const int r = a.r, H = a.H, Hp = H + 1, k0 = (a.nc - H) / 2;
    const double* skp = a.seed_kp + ((size_t)p * M + alpha) * (size_t)Hp * Hp * Hp;
    double t = 0.0;
    // the hat's support clipped to the K_p nodes (often empty)
    const int du0 = max(-(r - 1), k0 - X * r), du1 = min(r - 1, k0 + H - X * r);
    const int dv0 = max(-(r - 1), k0 - Y * r), dv1 = min(r - 1, k0 + H - Y * r);
    const int dw0 = max(-(r - 1), k0 - Z * r), dw1 = min(r - 1, k0 + H - Z * r);
    for (int dw = dw0; dw <= dw1; ++dw)
      for (int dv = dv0; dv <= dv1; ++dv)
        for (int du = du0; du <= du1; ++du) {
          const int fx = X * r + du - k0, fy = Y * r + dv - k0, fz = Z * r + dw - k0;
          const double wgt = (1.0 - fabs((double)du) / r) * (1.0 - fabs((double)dv) / r) * (1.0 - fabs((double)dw) / r);
          t += wgt * skp[nidx3(fx, fy, fz, Hp)];
        }
    if (a.seed_par != nullptr) {
      // seeds from the cells that inherit from this one, on all fine nodes
      const double* sp = a.seed_par + ((size_t)a.slot[p] * M + alpha) * (size_t)nn1 * nn1 * nn1;
      if (r == 1) {
        t += sp[nidx3(X, Y, Z, nn1)];
      } else {
        for (int dw = -(r - 1); dw <= r - 1; ++dw)
          for (int dv = -(r - 1); dv <= r - 1; ++dv)
            for (int du = -(r - 1); du <= r - 1; ++du) {
              const double wgt =
                  (1.0 - fabs((double)du) / r) * (1.0 - fabs((double)dv) / r) * (1.0 - fabs((double)dw) / r);
              t += wgt * sp[nidx3(X * r + du, Y * r + dv, Z * r + dw, nn1)];
            }
      }
    }
    return t;
  };

  // Phase A as a z-march: every thread walks its columns plane by plane with
  // a register window of p (planes Z-1, Z, Z+1 x rows Y-1, Y, Y+1 at its own
  // x) and of the element coefficients of its x column; x-1 / x+1 values come
  // from the neighbouring lanes by DPP (lanes of a row hold consecutive x).
  // The loads run one plane ahead: step Z issues plane Z+2 of p, element
  // layer Z+1 and the node data (r, D^-1) of plane Z+1, and computes plane Z
  // from what the previous step loaded, so a step's arithmetic overlaps the
  // next step's loads (on the 128^3 workload: Galerkin level 62.7 -> 58.6 ms,
  // fine level 72.2 -> 68.2 ms once phase B no longer held the registers).
  // Every lane runs the march (DPP needs them all); nodes off the free set
  // contribute nothing.
  constexpr bool ZM = G == 1;
  auto phaseA_zmarch = [&](double (&s4)[4]) {
    if constexpr (ZM) {
      clear_part(1);
      auto ld_p = [&](int Yr, int Z) -> double {
        return (Yr >= 0 && Yr <= NC && Z <= NC - 1) ? pv[nidx3(X, Yr, Z, NP)] : 0.0;
      };
      auto ld_k = [&](int Ye, int layer) -> double {
        return (Ye >= 0 && Ye <= NC - 1 && layer <= NC - 1) ? kwc[X + NC * (Ye + NC * layer)] : 0.0;
      };
      constexpr int KW = GAL ? 1 : 2;  // element windows only on the fine level
#pragma unroll 1
      for (int c = 0; c < CPT; ++c) {
        const int Y = Yc(c);
        const bool fr = colfree(c);
        // node data of plane Z of this column (zero off the free set)
        auto ld_r = [&](int Z) -> double { return (fr && Z <= NC - 1) ? rv[nidx3(X, Y, Z, NP)] : 0.0; };
        auto ld_d = [&](int Z) -> double { return (fr && Z <= NC - 1) ? dinv[node_of(Y, Z)] : 0.0; };
        Acc accA;
        zero_acc(accA);
        double wp[3][3];    // [plane Z-1, Z, Z+1][row Y-1, Y, Y+1]
        double kr[KW][KW];  // [layer Z-1, Z][oy]: elements (X, Y-1+oy); (X-1, .) by DPP
#pragma unroll
        for (int row = 0; row < 3; ++row) {
          wp[0][row] = 0.0;
          wp[1][row] = ld_p(Y - 1 + row, 1);
          wp[2][row] = ld_p(Y - 1 + row, 2);
        }
        if constexpr (!GAL) {
#pragma unroll
          for (int oy = 0; oy < 2; ++oy) {
            kr[0][oy] = ld_k(Y - 1 + oy, 0);
            kr[1][oy] = ld_k(Y - 1 + oy, 1);
          }
        }
        double rn = ld_r(1), di = ld_d(1);
#pragma unroll 1
        for (int Z = 1; Z <= NC - 1; ++Z) {
          const int m0 = (Z - 1) / sbw, m1 = Z / sbw;
          // loads of the next step
          double wpn[3];
          double krn[KW] = {};
#pragma unroll
          for (int row = 0; row < 3; ++row) wpn[row] = ld_p(Y - 1 + row, Z + 2);
          if constexpr (!GAL) {
#pragma unroll
            for (int oy = 0; oy < 2; ++oy) krn[oy] = ld_k(Y - 1 + oy, Z + 1);
          }
          const double rnn = ld_r(Z + 1), dnn = ld_d(Z + 1);
          // neighbour (dx, dy, dz) of the node from the window
          auto nb = [&](int dx, int dy, int dz) -> double {
            const double v = wp[dz + 1][dy + 1];
            return dx == 0 ? v : (dx < 0 ? from_left(v, X) : from_right(v, X, NC));
          };
          double Ap;
          if constexpr (!GAL) {
            double k8[8];
#pragma unroll
            for (int oz = 0; oz < 2; ++oz)
#pragma unroll
              for (int oy = 0; oy < 2; ++oy) {
                k8[2 * oy + 4 * oz] = from_left(kr[oz][oy], X);
                k8[1 + 2 * oy + 4 * oz] = kr[oz][oy];
              }
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) t += (k8[q] + k8[q + 4]) * nb(2 * (q & 1) - 1, 2 * (q >> 1) - 1, 0);
#pragma unroll
            for (int oz = 0; oz < 2; ++oz) {
              const int sz = 2 * oz - 1;
              const double* k4 = k8 + 4 * oz;
              t += (k4[0] + k4[2]) * nb(-1, 0, sz) + (k4[1] + k4[3]) * nb(1, 0, sz);
              t += (k4[0] + k4[1]) * nb(0, -1, sz) + (k4[2] + k4[3]) * nb(0, 1, sz);
              t += k4[0] * nb(-1, -1, sz) + k4[1] * nb(1, -1, sz) + k4[2] * nb(-1, 1, sz) + k4[3] * nb(1, 1, sz);
            }
            const double D = 4.0 * (((k8[0] + k8[1]) + (k8[2] + k8[3])) + ((k8[4] + k8[5]) + (k8[6] + k8[7])));
            Ap = D * wp[1][1] - t;
          } else {
            // Galerkin level: the node's 27 stored weights (row of K_n)
            const double* w = nW + node_of(Y, Z) * 27;
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < 27; ++k) t += w[k] * nb(k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1);
            Ap = t;
          }
          if (fr) {
            av[nidx3(X, Y, Z, NP)] = Ap;
            const double pn = wp[1][1];
            const double tr = di * rn, tA = di * Ap;
            s4[0] += pn * Ap;
            s4[1] += rn * tr;
            s4[2] += tr * Ap;
            s4[3] += Ap * tA;
            float w[8][N];
            node_weights(Y, Z, w);
            accB(accA, w, tA);
          }
#pragma unroll
          for (int row = 0; row < 3; ++row) {
            wp[0][row] = wp[1][row];
            wp[1][row] = wp[2][row];
            wp[2][row] = wpn[row];
          }
          if constexpr (!GAL) {
#pragma unroll
            for (int oy = 0; oy < 2; ++oy) {
              kr[0][oy] = kr[1][oy];
              kr[1][oy] = krn[oy];
            }
          }
          rn = rnn;
          di = dnn;
          const int Zn = Z + 1;
          if (Z == NC - 1 || (Zn - 1) / sbw != m0 || Zn / sbw != m1) {
            flushB(accA, c, 1, m0, m1);
            zero_acc(accA);
          }
        }
      }
    }
  };

  // Phase B (x, the projected residual and the new direction) as a z-march
  // with the loads two planes ahead: step Z issues the node data of plane
  // Z+2 (p, x, r, K p, D^-1) and updates plane Z from what earlier steps
  // loaded, so a step's stores and arithmetic overlap the loads of the next
  // two (fine-level solve of the 128^3 workload: 80.1 ms with the plain
  // sweep, 72.4 ms one plane ahead, 62.9 ms two planes ahead with phase A's
  // loads ahead too: 4.1 TB/s of algorithmic traffic).
  auto phaseB_zmarch = [&](double al, double be) {
#pragma unroll 1
    for (int c = 0; c < CPT; ++c) {
      if (!colfree(c)) continue;
      const int Y = Yc(c);
      auto q_of = [&](int Z) -> size_t { return nidx3(X, Y, Z, NP); };
      // node data of planes Z (0) and Z+1 (1)
      double pn[2], xn[2], rn[2], an[2], di[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int Zk = (1 + k <= NC - 1) ? 1 + k : 1;
        pn[k] = pv[q_of(Zk)];
        xn[k] = xv[q_of(Zk)];
        rn[k] = rv[q_of(Zk)];
        an[k] = av[q_of(Zk)];
        di[k] = dinv[node_of(Y, Zk)];
      }
      Acc vs;
#pragma unroll 1
      for (int Z = 1; Z <= NC - 1; ++Z) {
        const int m0 = (Z - 1) / sbw, m1 = Z / sbw;
        if (Z == 1 || (Z - 2) / sbw != m0 || (Z - 1) / sbw != m1) load_vs(vs, c, m0, m1);
        // plane Z+2 (the last steps reload plane Z; those values go unused)
        const int Zn = (Z + 2 <= NC - 1) ? Z + 2 : Z;
        const size_t qn = q_of(Zn);
        const double pn2 = pv[qn], xn2 = xv[qn], rn2 = rv[qn], an2 = av[qn];
        const double di2 = dinv[node_of(Y, Zn)];
        float w[8][N];
        node_weights(Y, Z, w);
        const size_t q = q_of(Z);
        xv[q] = xn[0] + al * pn[0];
        const double r2 = rn[0] + al * an[0] - scatB(vs, w);
        rv[q] = r2;
        pv[q] = -di[0] * r2 + be * pn[0];
        pn[0] = pn[1];
        xn[0] = xn[1];
        rn[0] = rn[1];
        an[0] = an[1];
        di[0] = di[1];
        pn[1] = pn2;
        xn[1] = xn2;
        rn[1] = rn2;
        an[1] = an2;
        di[1] = di2;
      }
    }
  };

  // ---- right-hand side of the constraints -------------------------------------
  double* uw = uW + wave * m;
  if (!a.adjoint) {
    const double* src = GAL ? a.gin + ((size_t)ci * M + alpha) * m : a.g + ((size_t)p * M + alpha) * m;
    for (int k = lane; k < m; k += 64) uw[k] = src[k];
  } else {
    for (int k = lane; k < m; k += 64) uw[k] = 0.0;
  }
  __syncthreads();  // sinvL, cwS visible

  // ---- feasible start x0 = D^-1 B^T S^-1 g' -----------------------------------
  double Vacc = 0.0, vk = 0.0;
  (void)wave_schur(&vk);
  {
    Acc vs;
    sweep([&](int c, int m0, int m1) { load_vs(vs, c, m0, m1); },
          [&](int c, int Z) {
            const int Y = Yc(c);
            float w[8][N];
            node_weights(Y, Z, w);
            const double x0 = dinv[node_of(Y, Z)] * scatB(vs, w);
            const size_t q = nidx3(X, Y, Z, NP);
            pv[q] = x0;
            xv[q] = x0;
          },
          nop3);
  }
  __syncthreads();
  // r0 = K x0 - f, t0 = D^-1 r0, r0.t0 and B t0
  {
    Acc acc;
    zero_acc(acc);
    clear_part(0);
    double s_rr = 0.0;
    sweep(nop3,
          [&](int c, int Z) {
            const int Y = Yc(c);
            float w[8][N];
            node_weights(Y, Z, w);
            const size_t q = nidx3(X, Y, Z, NP);
            const double rr0 = applyK(pv, Y, Z) - rhs(Y, Z);
            const double t = dinv[node_of(Y, Z)] * rr0;
            s_rr += rr0 * t;
            accB(acc, w, t);
            rv[q] = rr0;
          },
          [&](int c, int m0, int m1) {
            flushB(acc, c, 0, m0, m1);
            zero_acc(acc);
          });
    s_rr = wave_sum(s_rr);
    if (lane == 0) red[wave * 4] = s_rr;
  }
  __syncthreads();
  const double rr = wave_sum(lane < NW ? red[lane * 4] : 0.0);
  for (int k = lane; k < m; k += 64) uw[k] = cwS[k] * zsum(0, k);
  double vu = wave_schur(&vk);
  Vacc = vk;
  double rz = rr - vu;
  const double rz0 = rz;
  {
    Acc vs;
    sweep([&](int c, int m0, int m1) { load_vs(vs, c, m0, m1); },
          [&](int c, int Z) {
            const int Y = Yc(c);
            float w[8][N];
            node_weights(Y, Z, w);
            const size_t q = nidx3(X, Y, Z, NP);
            const double rp = rv[q] - scatB(vs, w);
            rv[q] = rp;
            pv[q] = -dinv[node_of(Y, Z)] * rp;
          },
          nop3);
  }
  __syncthreads();

  const double tol2 = a.rtol * a.rtol * rz0;
  int it = 0;
  bool done = !(rz0 > 0.0);
  while (!done) {
    const bool withz0 = (it % ZPERIOD3) == 0;
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    // phase A: K p, the dot products and the constraint partials B D^-1 Ap
    if constexpr (ZM) {
      phaseA_zmarch(s4);
    } else {
      Acc accA;
      zero_acc(accA);
      clear_part(1);
      sweep(nop3,
            [&](int c, int Z) {
              const int Y = Yc(c);
              const size_t q = nidx3(X, Y, Z, NP);
              const double Ap = applyK(pv, Y, Z);
              av[q] = Ap;
              const double rn = rv[q], pn = pv[q];
              const double di = dinv[node_of(Y, Z)];
              const double t = di * rn, tA = di * Ap;
              s4[0] += pn * Ap;
              s4[1] += rn * t;
              s4[2] += t * Ap;
              s4[3] += Ap * tA;
              float w[8][N];
              node_weights(Y, Z, w);
              accB(accA, w, tA);
            },
            [&](int c, int m0, int m1) {
              flushB(accA, c, 1, m0, m1);
              zero_acc(accA);
            });
    }
    // every ZPERIOD3 iterations: B D^-1 r' from scratch (a separate sweep)
    if (withz0) {
      Acc accT;
      zero_acc(accT);
      clear_part(0);
      sweep(nop3,
            [&](int c, int Z) {
              const int Y = Yc(c);
              float w[8][N];
              node_weights(Y, Z, w);
              accB(accT, w, dinv[node_of(Y, Z)] * rv[nidx3(X, Y, Z, NP)]);
            },
            [&](int c, int m0, int m1) {
              flushB(accT, c, 0, m0, m1);
              zero_acc(accT);
            });
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double v = wave_sum(s4[q]);
      if (lane == 0) red[wave * 4 + q] = v;
    }
    __syncthreads();
    // cross-wave sums: lane w2 < NW holds wave w2's partials (fixed DPP order)
    const double pAp = wave_sum(lane < NW ? red[lane * 4 + 0] : 0.0);
    const double rrk = wave_sum(lane < NW ? red[lane * 4 + 1] : 0.0);
    const double rA = wave_sum(lane < NW ? red[lane * 4 + 2] : 0.0);
    const double AA = wave_sum(lane < NW ? red[lane * 4 + 3] : 0.0);
    const double al = rrk / pAp;
    const double rDr = rrk + 2.0 * al * rA + al * al * AA;
    for (int k = lane; k < m; k += 64) uw[k] = cwS[k] * ((withz0 ? zsum(0, k) : 0.0) + al * zsum(1, k));
    vu = wave_schur(&vk);
    Vacc += vk;
    const double rzn = rDr - vu;
    ++it;
    if (rzn <= tol2 || it >= a.max_iter) {
      sweep(nop3,
            [&](int c, int Z) {
              const size_t q = nidx3(X, Yc(c), Z, NP);
              xv[q] += al * pv[q];
            },
            nop3);
      rz = rzn;
      break;
    }
    const double be = rzn / rrk;
    rz = rzn;
    // phase B: x, projected residual and the new direction
    if constexpr (ZM) {
      phaseB_zmarch(al, be);
    } else {
      Acc vs;
      sweep([&](int c, int m0, int m1) { load_vs(vs, c, m0, m1); },
            [&](int c, int Z) {
              const int Y = Yc(c);
              float w[8][N];
              node_weights(Y, Z, w);
              const size_t q = nidx3(X, Y, Z, NP);
              const double pn = pv[q];
              xv[q] += al * pn;
              const double rn = rv[q] + al * av[q] - scatB(vs, w);
              rv[q] = rn;
              pv[q] = -dinv[node_of(Y, Z)] * rn + be * pn;
            },
            nop3);
    }
    __syncthreads();
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

// ---------------------------------------------------------------------------
// Phi on the K_p nodes of every cell of a level: phikp[p][alpha][(H+1)^3].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(T3) void k_phikp3d(CellArgs a) {
  const int ci = a.ci0 + blockIdx.x / a.M, al = blockIdx.x % a.M;
  const int p = a.cells[ci];
  const int H = a.H, Hp = H + 1, k0 = (a.nc - H) / 2;
  const int tot = Hp * Hp * Hp;
  double* dst = a.phikp + ((size_t)p * a.M + al) * tot;
  for (int nd = threadIdx.x; nd < tot; nd += T3)
    dst[nd] = phi_at3(a, ci, al, k0 + nd % Hp, k0 + (nd / Hp) % Hp, k0 + nd / (Hp * Hp));
}

// Corner node offsets of K_p element (ex, ey, ez) in the (H+1)^3 node array.
MCH_DEV void kp_corners(int ex, int ey, int ez, int Hp, size_t (&nd)[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c) nd[c] = nidx3(ex + (c & 1), ey + ((c >> 1) & 1), ez + (c >> 2), Hp);
}

// ---------------------------------------------------------------------------
// Effective tensors A[p][a][b] = sum_{e in K_p} kappa_e Phi_a|e^T K_ref Phi_b|e
// (one workgroup per cell; Phi from phikp).
// ---------------------------------------------------------------------------
template <int MM>
__global__ __launch_bounds__(T3) void k_eff3d(CellArgs a, double* A) {
  __shared__ double wr[T3 / 64][MM * MM];
  const int H = a.H, Hp = H + 1, n = a.n, nm = a.n_macro;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = a.cells[a.ci0 + blockIdx.x];
  const int jx = p % nm, jy = (p / nm) % nm, jz = p / (nm * nm);
  const size_t tot = (size_t)Hp * Hp * Hp;
  const double* ph = a.phikp + (size_t)p * MM * tot;
  const double hk = a.h / 12.0;
  for (int al = 0; al < MM; ++al) {
    double acc[MM];
#pragma unroll
    for (int b = 0; b < MM; ++b) acc[b] = 0.0;
    for (int e = tid; e < H * H * H; e += T3) {
      const int ex = e % H, ey = (e / H) % H, ez = e / (H * H);
      const double kw = a.kappa[((size_t)(H * jz + ez) * n + (H * jy + ey)) * n + (H * jx + ex)] * hk;
      size_t nd[8];
      kp_corners(ex, ey, ez, Hp, nd);
      double v[8], y[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) v[c] = ph[al * tot + nd[c]];
      kref12_apply(v, y);
#pragma unroll
      for (int b = 0; b < MM; ++b) {
        if (b < al) continue;
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) t += ph[b * tot + nd[c]] * y[c];
        acc[b] += kw * t;
      }
    }
#pragma unroll
    for (int b = 0; b < MM; ++b) {
      const double t = wave_sum(acc[b]);
      if (lane == 0) wr[wave][al * MM + b] = t;
    }
  }
  __syncthreads();
  if (tid < MM * MM) {
    const int i = tid / MM, j = tid % MM;
    if (i <= j) {
      double t = 0.0;
      for (int w2 = 0; w2 < T3 / 64; ++w2) t += wr[w2][i * MM + j];
      A[((size_t)p * MM + i) * MM + j] = t;
      A[((size_t)p * MM + j) * MM + i] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint (see backward2d.hip for the derivation): explicit seeds on the K_p
// nodes and the explicit K_p gradient term.
// ---------------------------------------------------------------------------
template <int MM>
__global__ __launch_bounds__(T3) void k_seed3d(CellArgs a, const double* gA, double* seed_kp, double* gk) {
  __shared__ double G[MM * MM];
  const int H = a.H, Hp = H + 1, n = a.n, nm = a.n_macro;
  const int tid = threadIdx.x;
  const int p = a.cells[a.ci0 + blockIdx.x];
  const int jx = p % nm, jy = (p / nm) % nm, jz = p / (nm * nm);
  const size_t tot = (size_t)Hp * Hp * Hp;
  const double* ph = a.phikp + (size_t)p * MM * tot;
  const double hk = a.h / 12.0;
  for (int k = tid; k < MM * MM; k += T3) G[k] = gA[(size_t)p * MM * MM + k];
  __syncthreads();
  auto kap = [&](int ex, int ey, int ez) -> double {
    return a.kappa[((size_t)(H * jz + ez) * n + (H * jy + ey)) * n + (H * jx + ex)] * hk;
  };
  for (int nd0 = tid; nd0 < (int)tot; nd0 += T3) {
    const int X = nd0 % Hp, Y = (nd0 / Hp) % Hp, Z = nd0 / (Hp * Hp);
    double kphi[MM];
#pragma unroll
    for (int b = 0; b < MM; ++b) kphi[b] = 0.0;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int ex = X - 1 + (o & 1), ey = Y - 1 + ((o >> 1) & 1), ez = Z - 1 + (o >> 2);
      if (ex < 0 || ey < 0 || ez < 0 || ex >= H || ey >= H || ez >= H) continue;
      const double kw = kap(ex, ey, ez);
      const int c = (X - ex) + 2 * (Y - ey) + 4 * (Z - ez);
      size_t nd[8];
      kp_corners(ex, ey, ez, Hp, nd);
#pragma unroll
      for (int b = 0; b < MM; ++b) {
        const double* v = ph + b * tot;
        kphi[b] += kw * (4.0 * v[nd[c]] - v[nd[c ^ 3]] - v[nd[c ^ 5]] - v[nd[c ^ 6]] - v[nd[c ^ 7]]);
      }
    }
#pragma unroll
    for (int al = 0; al < MM; ++al) {
      double sacc = 0.0;
#pragma unroll
      for (int b = 0; b < MM; ++b) sacc += (G[al * MM + b] + G[b * MM + al]) * kphi[b];
      seed_kp[((size_t)p * MM + al) * tot + nd0] = sacc;
    }
  }
  for (int e = tid; e < H * H * H; e += T3) {
    const int ex = e % H, ey = (e / H) % H, ez = e / (H * H);
    size_t nd[8];
    kp_corners(ex, ey, ez, Hp, nd);
    double t = 0.0;
    for (int al = 0; al < MM; ++al) {
      double v[8], y[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) v[c] = ph[al * tot + nd[c]];
      kref12_apply(v, y);
#pragma unroll
      for (int b = 0; b < MM; ++b) {
        double d = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) d += ph[b * tot + nd[c]] * y[c];
        t += G[b * MM + al] * d;
      }
    }
    gk[((size_t)(H * jz + ez) * n + (H * jy + ey)) * n + (H * jx + ex)] = t * hk;
  }
}

// Per-cell gradient window gcell[p][e] = -sum_a (P w_a)|_e^T K_ref Phi_a|_e over
// the nc^3 fine elements of the cell (one workgroup per cell).
__global__ __launch_bounds__(T3) void k_grad3d(CellArgs a, const double* w, double* gcell) {
  const int nc = a.nc, nn1 = nc + 1, r = a.r, NC = a.NC, NP = NC + 1, M = a.M;
  const int ci = a.ci0 + blockIdx.x;
  const int p = a.cells[ci];
  const size_t NN = (size_t)NP * NP * NP, nn = (size_t)nn1 * nn1 * nn1;
  const double hk = a.h / 12.0, inv_r = 1.0 / r;
  const int ncube = nc * nc * nc;
  for (int e = threadIdx.x; e < ncube; e += T3) {
    const int fx = e % nc, fy = (e / nc) % nc, fz = e / (nc * nc);
    const int EX = fx / r, EY = fy / r, EZ = fz / r;
    const int ux = fx - EX * r, uy = fy - EY * r, uz = fz - EZ * r;
    double acc = 0.0;
    for (int al = 0; al < M; ++al) {
      const double* wv = w + ((size_t)ci * M + al) * NN;
      double phi[8], pw[8], y[8];
      if (r == 1) {
        const double* xv = a.out + ((size_t)ci * M + al) * nn;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const size_t q = nidx3(fx + (c & 1), fy + ((c >> 1) & 1), fz + (c >> 2), nn1);
          phi[c] = xv[q];
          pw[c] = wv[q];
        }
      } else {
        const double* I = a.phi1 + ((size_t)a.pslot[ci] * M + al) * nn;
        const double* xi = a.out + ((size_t)ci * M + al) * NN;
        double xe[8], we[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const size_t q = nidx3(EX + (c & 1), EY + ((c >> 1) & 1), EZ + (c >> 2), NP);
          xe[c] = xi[q];
          we[c] = wv[q];
        }
#pragma unroll
        for (int dl = 0; dl < 8; ++dl) {
          const double tx = (ux + (dl & 1)) * inv_r, ty = (uy + ((dl >> 1) & 1)) * inv_r, tz = (uz + (dl >> 2)) * inv_r;
          double sx = 0.0, sw = 0.0;
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const double t = tri_w(c, tx, ty, tz);
            sx += t * xe[c];
            sw += t * we[c];
          }
          phi[dl] = I[nidx3(fx + (dl & 1), fy + ((dl >> 1) & 1), fz + (dl >> 2), nn1)] + sx;
          pw[dl] = sw;
        }
      }
      kref12_apply(phi, y);
      double t = 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c) t += pw[c] * y[c];
      acc -= t;
    }
    gcell[(size_t)p * ncube + e] = acc * hk;
  }
}

struct LevelTab3 {
  int r[MAX_LEVELS];
  int NC[MAX_LEVELS];
  const double* w[MAX_LEVELS];
};

// Seeds of level-1 cell t for right-hand side alpha (one workgroup per
// (t, alpha)): the sum over its inheriting cells c, in a fixed order, of
// Ibar_c = Phibar_c - K_h(c) P w_c - B_h(c)^T mu_c on the free fine nodes.
// K_h P w and B^T mu are scattered element by element in 8 colour passes
// (elements of one colour share no node), so every node's sum has a fixed order.
__global__ __launch_bounds__(T3) void k_ibar3d(CellArgs a, LevelTab3 lt, const int32_t* level, const int32_t* child_ptr,
                                               const int32_t* child, const double* mu, double* seed_par) {
  const int nc = a.nc, nn1 = nc + 1, H = a.H, Hp = H + 1, m = a.m, N = a.N, s = a.s, M = a.M;
  const int tid = threadIdx.x;
  const int t = a.ci0 + blockIdx.x / M, al = blockIdx.x % M;
  const int k0 = (nc - H) / 2, sb = nc / s;
  const int flo = a.bc ? 0 : 1, fhi = a.bc ? nc : nc - 1;  // free fine nodes
  const size_t nn = (size_t)nn1 * nn1 * nn1;
  double* acc = seed_par + ((size_t)t * M + al) * nn;
  const double hk = a.h / 12.0;
  for (size_t nd = tid; nd < nn; nd += T3) acc[nd] = 0.0;
  const int half = nc / 2;
  for (int ch = child_ptr[t]; ch < child_ptr[t + 1]; ++ch) {
    const int p = child[ch];
    const int l = level[p] - 1;
    const int ci = a.slot[p];
    const int r = lt.r[l], NC = lt.NC[l], NP = NC + 1;
    const double inv_r = 1.0 / r;
    int ox, oy, oz;
    cell_origin3(a, p, ox, oy, oz);
    const double* wv = lt.w[l] + ((size_t)ci * M + al) * (size_t)NP * NP * NP;
    const double* cwp = a.cw + (size_t)p * m;
    const double* mup = mu + ((size_t)p * M + al) * m;
    for (int colour = 0; colour < 8; ++colour) {
      __syncthreads();
      const int cx = colour & 1, cy = (colour >> 1) & 1, cz = colour >> 2;
      for (int k = tid; k < half * half * half; k += T3) {
        const int fx = 2 * (k % half) + cx, fy = 2 * ((k / half) % half) + cy, fz = 2 * (k / (half * half)) + cz;
        const size_t ge = gel3(a, ox, oy, oz, fx, fy, fz);
        const double kw = a.kappa[ge] * hk;
        const int lab = a.label[ge];
        const int EX = fx / r, EY = fy / r, EZ = fz / r;
        const int ux = fx - EX * r, uy = fy - EY * r, uz = fz - EZ * r;
        double we[8], pw[8], y[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) we[c] = wv[nidx3(EX + (c & 1), EY + ((c >> 1) & 1), EZ + (c >> 2), NP)];
#pragma unroll
        for (int dl = 0; dl < 8; ++dl) {
          const double tx = (ux + (dl & 1)) * inv_r, ty = (uy + ((dl >> 1) & 1)) * inv_r, tz = (uz + (dl >> 2)) * inv_r;
          double sw = 0.0;
#pragma unroll
          for (int c = 0; c < 8; ++c) sw += tri_w(c, tx, ty, tz) * we[c];
          pw[dl] = sw;
        }
        kref12_apply(pw, y);
        double cm = 0.0;
        if (lab < N) {
          const int q = fx / sb + s * (fy / sb + s * (fz / sb));
          cm = cwp[q * N + lab] * mup[q * N + lab];
        }
#pragma unroll
        for (int dl = 0; dl < 8; ++dl) {
          const int X = fx + (dl & 1), Y = fy + ((dl >> 1) & 1), Z = fz + (dl >> 2);
          if (X < flo || Y < flo || Z < flo || X > fhi || Y > fhi || Z > fhi) continue;
          acc[nidx3(X, Y, Z, nn1)] -= kw * y[dl] + cm;
        }
      }
    }
    __syncthreads();
    const double* skp = a.seed_kp + ((size_t)p * M + al) * (size_t)Hp * Hp * Hp;
    for (int nd = tid; nd < Hp * Hp * Hp; nd += T3) {
      const int X = k0 + nd % Hp, Y = k0 + (nd / Hp) % Hp, Z = k0 + nd / (Hp * Hp);
      if (X < flo || Y < flo || Z < flo || X > fhi || Y > fhi || Z > fhi) continue;
      acc[nidx3(X, Y, Z, nn1)] += skp[nd];
    }
  }
}

// Multilinear mode (interp = 1): Phi = I + P xi of each cell of a level on
// every fine node of its cell, into T slot toff + ci of the store.
__global__ __launch_bounds__(T3) void k_recon3d(CellArgs a, int toff, double* phiT) {
  const int ci = blockIdx.x / a.M, al = blockIdx.x % a.M;
  const int nn1 = a.nc + 1;
  const size_t nn = (size_t)nn1 * nn1 * nn1;
  double* dst = phiT + ((size_t)(toff + ci) * a.M + al) * nn;
  for (size_t nd = threadIdx.x; nd < nn; nd += T3)
    dst[nd] = phi_at3(a, ci, al, (int)(nd % nn1), (int)((nd / nn1) % nn1), (int)(nd / ((size_t)nn1 * nn1)));
}

MCH_DEV int floordiv3(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// glogk[e] = kappa_e * (explicit K_p term + sum of the cell windows covering e).
__global__ void k_gather_grad3d(CellArgs a, const double* gk, const double* gcell, double* glogk) {
  const int n = a.n, H = a.H, nc = a.nc, nm = a.n_macro;
  const size_t total = (size_t)n * n * n, cube = (size_t)nc * nc * nc;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i1 = (int)(e % n), i2 = (int)((e / n) % n), i3 = (int)(e / ((size_t)n * n));
    const int t1 = i1 + nc / 2 - H / 2, t2 = i2 + nc / 2 - H / 2, t3 = i3 + nc / 2 - H / 2;
    double acc = gk[e];
    for (int j3 = floordiv3(t3 - nc, H) + 1; j3 <= floordiv3(t3, H); ++j3) {
      const int a3 = t3 - H * j3, jj3 = wrapi(j3, nm);
      for (int j2 = floordiv3(t2 - nc, H) + 1; j2 <= floordiv3(t2, H); ++j2) {
        const int a2 = t2 - H * j2, jj2 = wrapi(j2, nm);
        for (int j1 = floordiv3(t1 - nc, H) + 1; j1 <= floordiv3(t1, H); ++j1) {
          const int a1 = t1 - H * j1;
          const int q = wrapi(j1, nm) + nm * (jj2 + nm * jj3);
          acc += gcell[(size_t)q * cube + (size_t)a1 + nc * ((size_t)a2 + nc * (size_t)a3)];
        }
      }
    }
    glogk[e] = a.kappa[e] * acc;
  }
}

// Fine local solutions of selected cells: out[k][alpha][node] over (nc+1)^3 nodes.
__global__ void k_gather_phi3d(CellArgs a, const int32_t* sel_ci, int n_sel, double* out) {
  const int k = blockIdx.y;
  if (k >= n_sel) return;
  const int ci = sel_ci[k];
  if (ci < 0) return;
  const int nn1 = a.nc + 1;
  const size_t per = (size_t)nn1 * nn1 * nn1;
  const size_t total = (size_t)a.M * per;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const int al = (int)(idx / per);
    const int nd = (int)(idx % per);
    out[(size_t)k * total + idx] = phi_at3(a, ci, al, nd % nn1, (nd / nn1) % nn1, nd / (nn1 * nn1));
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

template <typename F>
static int lds_attr3(F fn, size_t lds) {
  if (lds > 160 * 1024) return set_error(MCH_EINVAL, "kernel exceeds the LDS budget");
  if (lds > 64 * 1024) {
    hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute");
  }
  return MCH_OK;
}

static int schur_lanes3(int m) {
  int J = 1;
  while (J * 2 * m <= 64) J *= 2;
  return J;
}

#define MCH_SHAPES3(X) \
  X(32, 1, false) X(32, 2, false) X(32, 3, false) X(16, 1, false) X(16, 2, false) X(16, 3, false) \
  X(16, 1, true) X(16, 2, true) X(16, 3, true) X(8, 1, true) X(8, 2, true) X(8, 3, true)

bool shape_supported_3d(int NC, int s, int N) {
  if (s != S3D) return false;
  bool any = false;
#define X(nc_, n_, g_) \
  if (NC == nc_ && N == n_) any = true;
  MCH_SHAPES3(X)
#undef X
  return any;
}

template <int NC, int N, bool GAL>
static int launch_solve3_t(const CellArgs& a, hipStream_t s) {
  constexpr int NT = nt3<NC, GAL>();
  constexpr int NW = NT / 64, G = NT > NC * NC ? NT / (NC * NC) : 1;
  const int MS = (a.m + a.J - 1) / a.J;
  const size_t lds =
      ((size_t)4 * NW + 2 * (size_t)G * NC * 2 * S3D * S3D * N + (size_t)MS * 64 + a.m + 2 * (size_t)NW * a.m) *
      sizeof(double);
  auto fn = k_solve3d<NC, N, GAL>;
  int rc = lds_attr3(fn, lds);
  if (rc) return rc;
  const int groups = (a.count + kXcds - 1) / kXcds;
  hipLaunchKernelGGL(fn, dim3(groups * kXcds * a.M), dim3(NT), lds, s, a);
  return hip_check(hipGetLastError(), "launch k_solve3d");
}

int solve_blocks_per_cu_3d(mch_plan* pl) {
  CellArgs a = base_args(pl, nullptr, nullptr, 0);
  if (a.gen_tp > 0) return generic3_blocks_per_cu(a);
  a.J = schur_lanes3(a.m);
  const void* fn = nullptr;
  int threads = 0;
  size_t lds = 0;
#define X(nc_, n_, g_)                                                                                  \
  if constexpr (!g_) {                                                                                  \
    if (a.NC == nc_ && a.N == n_) {                                                                     \
      constexpr int NT = nt3<nc_, false>(), NW = NT / 64, G = NT > nc_ * nc_ ? NT / (nc_ * nc_) : 1;    \
      const int MS = (a.m + a.J - 1) / a.J;                                                             \
      lds = ((size_t)4 * NW + 2 * (size_t)G * nc_ * 2 * S3D * S3D * n_ + (size_t)MS * 64 + a.m +        \
             2 * (size_t)NW * a.m) * sizeof(double);                                                    \
      fn = reinterpret_cast<const void*>(k_solve3d<nc_, n_, false>);                                    \
      threads = NT;                                                                                     \
    }                                                                                                   \
  }
  MCH_SHAPES3(X)
#undef X
  if (!fn) return set_error(MCH_ENOTIMPL, "no 3D solve kernel for this cell shape");
  int nb = 0;
  int rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, lds),
                     "hipOccupancyMaxActiveBlocksPerMultiprocessor");
  return rc ? rc : nb;
}

static int launch_solve3(const CellArgs& a_in, hipStream_t s) {
  if (a_in.gen_tp > 0) return launch_solve3d_generic(a_in, s);
  if (a_in.bc != 0) return set_error(MCH_EINVAL, "the column-marching 3D solve takes Dirichlet cells only");
  CellArgs a = a_in;
  a.J = schur_lanes3(a.m);
  const bool gal = a.r > 1;
#define X(nc_, n_, g_) \
  if (a.NC == nc_ && a.N == n_ && gal == g_) return launch_solve3_t<nc_, n_, g_>(a, s);
  MCH_SHAPES3(X)
#undef X
  return set_error(MCH_ENOTIMPL, "no 3D solve kernel for this cell shape");
}

static int launch_setup3(const CellArgs& a, hipStream_t s) {
  // a level of few cells (the fine level of a small macrogrid, which heads
  // the critical path) gets 1024 threads per cell so that its workgroups
  // still use much of the GPU
  const int tb = a.count <= 128 ? 1024 : T3;
  const size_t npairs = (size_t)a.m * (a.m + 1) / 2;
  const size_t s3 = (size_t)a.s * a.s * a.s;
  const size_t planes = a.gen_tp > 0 ? a.NC + 1 : a.NC;  // node planes of the S partials
  const size_t lds = ((size_t)2 * a.m * a.m + (s3 + 1) * a.N * 4 + (size_t)(tb / 64) * a.N * 4 + npairs * planes) *
                     sizeof(double);
  void (*fn)(CellArgs) = nullptr;
#define MCH_SETUP3(n_) \
  if (a.N == n_) fn = tb == 1024 ? k_setup3d<n_, 1024> : k_setup3d<n_, T3>;
  MCH_SETUP3(1) MCH_SETUP3(2) MCH_SETUP3(3)
#undef MCH_SETUP3
  if (!fn) return set_error(MCH_ENOTIMPL, "n_cont");
  int rc = lds_attr3(fn, lds);
  if (rc) return rc;
  hipLaunchKernelGGL(fn, dim3(a.count), dim3(tb), lds, s, a);
  return hip_check(hipGetLastError(), "launch k_setup3d");
}

static int launch_inherit3(const CellArgs& a, hipStream_t s) {
  if (a.NC * a.NC > T3) return set_error(MCH_ENOTIMPL, "3D inherited right-hand sides need NC^2 <= 256");
  const size_t lds = ((size_t)2 * a.NC * a.NC * 8 + (size_t)T3 * 2 * a.N) * sizeof(double);
  void (*fn)(CellArgs) = nullptr;
  if (a.N == 1) fn = k_inherit3d<1>;
  if (a.N == 2) fn = k_inherit3d<2>;
  if (a.N == 3) fn = k_inherit3d<3>;
  if (!fn) return set_error(MCH_ENOTIMPL, "n_cont");
  int rc = lds_attr3(fn, lds);
  if (rc) return rc;
  hipLaunchKernelGGL(fn, dim3(a.count * a.M), dim3(T3), lds, s, a);
  return hip_check(hipGetLastError(), "launch k_inherit3d");
}

static int launch_phikp3(const CellArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_phikp3d, dim3(a.count * a.M), dim3(T3), 0, s, a);
  return hip_check(hipGetLastError(), "launch k_phikp3d");
}

// Forward DAG, as in 2D: setups of levels >= 2 on their side streams from the
// start; level 1 set-up and solve on s in two chunks; every level >= 2
// inherits, solves and writes Phi on K_p for the cells of chunk A once chunk
// A is done, the rest once level 1 is done; Phi on K_p of level 1 on s.
// interp = 1: the levels run as a chain on s (level n reads the fine Phi of
// every level below it), as in 2D: the setups of levels >= 2 on their level
// streams from the start; then per level the interpolation of I, the
// inherited right-hand sides, the solve, Phi on K_p and, below L, the fine
// Phi into the level's T slots.
static int launch_forward_3d_chain(mch_plan* pl, const double* kappa, const uint8_t* label, hipStream_t s) {
  char name[32];
  int rc = ensure_streams(pl);
  if (!rc) rc = fork_levels(pl, s);
  for (int l = 1; l < pl->L && !rc; ++l) {
    if (pl->lev[l].count == 0) continue;
    hipStream_t t = level_stream(pl, l, s);
    std::snprintf(name, sizeof(name), "setup_L%d", l + 1);
    {
      ProfScope ps(pl, name, t);
      rc = launch_setup3(base_args(pl, kappa, label, l), t);
    }
    if (!rc && !pl->serial) rc = hip_check(hipEventRecord(pl->ev_setup[l], t), "hipEventRecord");
  }
  for (int l = 0; l < pl->L && !rc; ++l) {
    const Level& lv = pl->lev[l];
    if (lv.count == 0) continue;
    CellArgs a = base_args(pl, kappa, label, l);
    if (l == 0) {
      ProfScope ps(pl, "setup_L1", s);
      rc = launch_setup3(a, s);
    } else {
      rc = launch_interp(pl, l, s);
      if (!rc && !pl->serial) rc = hip_check(hipStreamWaitEvent(s, pl->ev_setup[l], 0), "hipStreamWaitEvent");
      if (!rc) {
        std::snprintf(name, sizeof(name), "inherit_L%d", l + 1);
        ProfScope ps(pl, name, s);
        rc = launch_inherit3(a, s);
      }
    }
    if (!rc) {
      std::snprintf(name, sizeof(name), "solve_L%d", l + 1);
      ProfScope ps(pl, name, s);
      rc = launch_solve3(a, s);
    }
    if (!rc) {
      std::snprintf(name, sizeof(name), "phikp_L%d", l + 1);
      ProfScope ps(pl, name, s);
      rc = launch_phikp3(a, s);
    }
    if (!rc && l > 0 && l + 1 < pl->L) {
      ProfScope ps(pl, "recon", s);
      hipLaunchKernelGGL(k_recon3d, dim3((unsigned)(lv.count * pl->M)), dim3(T3), 0, s, a, lv.toff, pl->lev[0].d_out);
      rc = hip_check(hipGetLastError(), "launch k_recon3d");
    }
  }
  if (!rc) rc = join_levels(pl, s);
  return rc;
}

int launch_forward_3d(mch_plan* pl, const double* kappa, const uint8_t* label, hipStream_t s) {
  if (pl->nT > 0) return launch_forward_3d_chain(pl, kappa, label, s);
  char name[32];
  int rc = ensure_streams(pl);
  if (!rc) rc = fork_levels(pl, s);
  // the level-1 set-up first: it heads the critical path
  const int n1 = pl->lev[0].count, n1a = pl->n1a;
  const CellArgs a1 = base_args(pl, kappa, label, 0);
  if (!rc && n1) {
    ProfScope ps(pl, "setup_L1", s);
    rc = launch_setup3(a1, s);
  }
  for (int l = 1; l < pl->L && !rc; ++l) {
    if (pl->lev[l].count == 0) continue;
    CellArgs a = base_args(pl, kappa, label, l);
    std::snprintf(name, sizeof(name), "setup_L%d", l + 1);
    ProfScope ps(pl, name, level_stream(pl, l, s));
    rc = launch_setup3(a, level_stream(pl, l, s));
  }
  if (!rc && n1) {
    const CellArgs& a = a1;
    if (!rc && n1a > 0) {
      ProfScope ps(pl, "solve_L1", s);
      rc = launch_solve3(chunk_args(a, 0, n1a), s);
    }
    if (!rc) rc = hip_check(hipEventRecord(pl->ev_l1a, s), "hipEventRecord");
    if (!rc && n1 > n1a) {
      ProfScope ps(pl, "solve_L1", s);
      rc = launch_solve3(chunk_args(a, n1a, n1 - n1a), s);
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
        rc = launch_inherit3(c, t);
      }
      if (!rc) {
        std::snprintf(name, sizeof(name), "solve_L%d", l + 1);
        ProfScope ps(pl, name, t);
        rc = launch_solve3(c, t);
      }
      if (!rc) {
        std::snprintf(name, sizeof(name), "phikp_L%d", l + 1);
        ProfScope ps(pl, name, t);
        rc = launch_phikp3(c, t);
      }
    }
  }
  if (!rc && n1) {
    CellArgs a = base_args(pl, kappa, label, 0);
    ProfScope ps(pl, "phikp_L1", s);
    rc = launch_phikp3(a, s);
  }
  if (!rc) rc = join_levels(pl, s);
  return rc;
}

int launch_eff_3d(mch_plan* pl, const double* kappa, double* A, hipStream_t s) {
  int rc = ensure_streams(pl);
  if (!rc) rc = fork_levels(pl, s);
  for (int l = 0; l < pl->L && !rc; ++l) {
    if (pl->lev[l].count == 0) continue;
    hipStream_t t = level_stream(pl, l, s);
    CellArgs a = base_args(pl, kappa, pl->fwd_label, l);
    void (*fn)(CellArgs, double*) = nullptr;
    switch (a.M) {
      case 4: fn = k_eff3d<4>; break;
      case 8: fn = k_eff3d<8>; break;
      case 12: fn = k_eff3d<12>; break;
      default: return set_error(MCH_ENOTIMPL, "M");
    }
    char name[32];
    std::snprintf(name, sizeof(name), "eff_L%d", l + 1);
    {
      ProfScope ps(pl, name, t);
      hipLaunchKernelGGL(fn, dim3(a.count), dim3(T3), 0, t, a, A);
    }
    rc = hip_check(hipGetLastError(), "launch k_eff3d");
  }
  if (!rc) rc = join_levels(pl, s);
  return rc;
}

// interp = 1, as in 2D: from level L down on s, each level's adjoint solve
// (with the seeds its cells received from the levels above), then Ibar per
// cell (the parent-seed kernel over an identity map) and c_t Ibar into the
// neighbours' seeds; explicit seeds up front and the gradient windows on the
// level streams.
static int launch_backward_3d_chain(mch_plan* pl, const double* kappa, const double* gA, double* glogk,
                                    hipStream_t s) {
  const int M = pl->M;
  char name[32];
  void (*seed)(CellArgs, const double*, double*, double*) = nullptr;
  switch (M) {
    case 4: seed = k_seed3d<4>; break;
    case 8: seed = k_seed3d<8>; break;
    case 12: seed = k_seed3d<12>; break;
    default: return set_error(MCH_ENOTIMPL, "M");
  }
  int rc = ensure_streams(pl);
  if (!rc) rc = launch_zero(pl->d_seedT, (size_t)pl->nT * M * pl->nn, s);
  if (!rc) rc = fork_levels(pl, s);
  const CellArgs a1 = base_args(pl, kappa, pl->fwd_label, 0);
  LevelTab3 lt{};
  for (int l = 0; l < pl->L; ++l) {
    lt.r[l] = pl->lev[l].r;
    lt.NC[l] = pl->lev[l].NC;
    lt.w[l] = pl->lev[l].d_w;
  }
  for (int l = 0; l < pl->L && !rc; ++l) {
    if (pl->lev[l].count == 0) continue;
    hipStream_t t = level_stream(pl, l, s);
    CellArgs a = base_args(pl, kappa, pl->fwd_label, l);
    std::snprintf(name, sizeof(name), "seed_L%d", l + 1);
    {
      ProfScope ps(pl, name, t);
      hipLaunchKernelGGL(seed, dim3(a.count), dim3(T3), 0, t, a, gA, pl->d_seed_kp, pl->d_gk);
    }
    rc = hip_check(hipGetLastError(), "launch k_seed3d");
    if (!rc && l > 0 && !pl->serial) rc = hip_check(hipEventRecord(pl->ev_setup[l], t), "hipEventRecord");
  }
  for (int l = pl->L - 1; l >= 0 && !rc; --l) {
    const Level& lv = pl->lev[l];
    if (lv.count == 0) continue;
    CellArgs a = base_args(pl, kappa, pl->fwd_label, l);
    if (l > 0 && !pl->serial && (rc = hip_check(hipStreamWaitEvent(s, pl->ev_setup[l], 0), "hipStreamWaitEvent")))
      break;
    CellArgs b = a;
    b.adjoint = 1;
    b.out = lv.d_w;
    b.beta = pl->d_mu;
    b.iters = pl->d_iters_adj;
    b.resid = pl->d_resid_adj;
    b.seed_par = (l + 1 < pl->L) ? pl->d_seedT + (size_t)lv.toff * M * pl->nn : nullptr;
    std::snprintf(name, sizeof(name), "adjsolve_L%d", l + 1);
    {
      ProfScope ps(pl, name, s);
      rc = launch_solve3(b, s);
    }
    if (!rc && l > 0) {
      {
        ProfScope ps(pl, "ibar", s);
        hipLaunchKernelGGL(k_ibar3d, dim3(lv.count * M), dim3(T3), 0, s, a1, lt, pl->d_level, pl->d_iptr, lv.d_cells,
                           pl->d_mu, pl->d_ibar);
        rc = hip_check(hipGetLastError(), "launch k_ibar3d");
      }
      if (!rc) rc = launch_distribute(pl, l, s);
    }
    hipStream_t t = level_stream(pl, l, s);
    if (!rc && t != s) {
      rc = hip_check(hipEventRecord(pl->ev_adj[l], s), "hipEventRecord");
      if (!rc) rc = hip_check(hipStreamWaitEvent(t, pl->ev_adj[l], 0), "hipStreamWaitEvent");
    }
    if (!rc) {
      std::snprintf(name, sizeof(name), "grad_L%d", l + 1);
      ProfScope ps(pl, name, t);
      hipLaunchKernelGGL(k_grad3d, dim3(a.count), dim3(T3), 0, t, a, lv.d_w, pl->d_gcell);
      rc = hip_check(hipGetLastError(), "launch k_grad3d");
    }
  }
  if (!rc) rc = join_levels(pl, s);
  if (rc) return rc;
  const size_t total = (size_t)pl->n * pl->n * pl->n;
  const unsigned blocks = (unsigned)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
  {
    ProfScope ps(pl, "gather", s);
    hipLaunchKernelGGL(k_gather_grad3d, dim3(blocks), dim3(256), 0, s, a1, pl->d_gk, pl->d_gcell, glogk);
  }
  return hip_check(hipGetLastError(), "launch k_gather_grad3d");
}

// Backward DAG, as in 2D.
int launch_backward_3d(mch_plan* pl, const double* kappa, const double* gA, double* glogk, hipStream_t s) {
  if (pl->nT > 0) return launch_backward_3d_chain(pl, kappa, gA, glogk, s);
  const int M = pl->M;
  char name[32];
  int rc = ensure_streams(pl);
  if (!rc) rc = fork_levels(pl, s);
  if (rc) return rc;
  void (*seed)(CellArgs, const double*, double*, double*) = nullptr;
  switch (M) {
    case 4: seed = k_seed3d<4>; break;
    case 8: seed = k_seed3d<8>; break;
    case 12: seed = k_seed3d<12>; break;
    default: return set_error(MCH_ENOTIMPL, "M");
  }
  auto launch_grad = [&](const CellArgs& g, hipStream_t t, int l) -> int {
    if (g.count == 0) return MCH_OK;
    std::snprintf(name, sizeof(name), "grad_L%d", l + 1);
    ProfScope ps(pl, name, t);
    hipLaunchKernelGGL(k_grad3d, dim3(g.count), dim3(T3), 0, t, g, pl->lev[l].d_w, pl->d_gcell);
    return hip_check(hipGetLastError(), "launch k_grad3d");
  };
  auto adjoint_args = [&](int l) {
    CellArgs a = base_args(pl, kappa, pl->fwd_label, l);
    a.adjoint = 1;
    a.out = pl->lev[l].d_w;
    a.beta = pl->d_mu;
    a.iters = pl->d_iters_adj;
    a.resid = pl->d_resid_adj;
    return a;
  };
  for (int l = pl->L - 1; l >= 0; --l) {
    if (pl->lev[l].count == 0) continue;
    hipStream_t t = level_stream(pl, l, s);
    CellArgs a = base_args(pl, kappa, pl->fwd_label, l);
    std::snprintf(name, sizeof(name), "seed_L%d", l + 1);
    {
      ProfScope ps(pl, name, t);
      hipLaunchKernelGGL(seed, dim3(a.count), dim3(T3), 0, t, a, gA, pl->d_seed_kp, pl->d_gk);
    }
    if ((rc = hip_check(hipGetLastError(), "launch k_seed3d"))) return rc;
    if (l == 0) continue;
    std::snprintf(name, sizeof(name), "adjsolve_L%d", l + 1);
    {
      ProfScope ps(pl, name, t);
      rc = launch_solve3(adjoint_args(l), t);
    }
    if (!rc) rc = launch_grad(base_args(pl, kappa, pl->fwd_label, l), t, l);
    if (rc) return rc;
  }
  const int n1 = pl->lev[0].count;
  const bool inherit = pl->L > 1 && n1 > 0 && n1 < pl->P;
  CellArgs a1 = base_args(pl, kappa, pl->fwd_label, 0);
  LevelTab3 lt{};
  for (int l = 0; l < pl->L; ++l) {
    lt.r[l] = pl->lev[l].r;
    lt.NC[l] = pl->lev[l].NC;
    lt.w[l] = pl->lev[l].d_w;
  }
  rc = join_levels(pl, s);
  if (!rc && n1 > 0) {
    if (inherit) {
      ProfScope ps(pl, "ibar", s);
      hipLaunchKernelGGL(k_ibar3d, dim3(n1 * M), dim3(T3), 0, s, a1, lt, pl->d_level, pl->d_child_ptr, pl->d_child,
                         pl->d_mu, pl->d_seed_par);
      rc = hip_check(hipGetLastError(), "launch k_ibar3d");
    }
    if (!rc) {
      CellArgs a = adjoint_args(0);
      a.seed_par = inherit ? pl->d_seed_par : nullptr;
      ProfScope ps(pl, "adjsolve_L1", s);
      rc = launch_solve3(a, s);
    }
    if (!rc) rc = launch_grad(a1, s, 0);
  }
  if (rc) return rc;
  const size_t total = (size_t)pl->n * pl->n * pl->n;
  const unsigned blocks = (unsigned)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
  {
    ProfScope ps(pl, "gather", s);
    hipLaunchKernelGGL(k_gather_grad3d, dim3(blocks), dim3(256), 0, s, a1, pl->d_gk, pl->d_gcell, glogk);
  }
  return hip_check(hipGetLastError(), "launch k_gather_grad3d");
}

int launch_local_solutions_3d(mch_plan* pl, const int64_t* cells, int64_t n, double* out, hipStream_t s) {
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
    hipLaunchKernelGGL(k_gather_phi3d, dim3(64, (unsigned)n), dim3(256), 0, s, a, d_sel, (int)n, out);
    rc = hip_check(hipGetLastError(), "launch k_gather_phi3d");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    (void)hipFreeAsync(d_sel, s);
    if (rc) return rc;
  }
  return MCH_OK;
}

}  // namespace mch
