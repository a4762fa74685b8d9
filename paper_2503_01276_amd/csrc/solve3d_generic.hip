// The 3D constrained cell solve for either cell boundary condition, with the
// Krylov vectors in global memory: the 2D generic kernel's design
// (solve2d_generic.hip) on Q1 hexahedra.
//
// Same problem and method as the column-marching kernel k_solve3d (paper
// Sec. 2, Eqs. phi_avar / phi_grad; Sec. 3.3, Eqs. phi_avar_corrector /
// phi_grad_corrector): projected PCG with the constraint preconditioner
// [D B^T; B 0], the Gould-Hribar-Nocedal residual update, a feasible start,
// fused reductions, a per-wave Schur solve with the setup's S^-1 and a final
// projection. It serves natural Neumann cells, whose (NC+1)^3 free nodes do
// not fit the column-marching kernel's owned planes [0, NC) with a zero
// boundary plane at NC.
//
// The trilinear element matrix (times 12/h) couples a corner with itself (4),
// its three face-diagonal corners and its body-diagonal corner (-1 each); the
// setup stores kappa h / 12 per element, so a node's row is a 27-point
// stencil (21 nonzero on the fine level).
//
// Layout: one workgroup per (cell, right-hand side), at most 512 threads,
// one tile of TP lanes per constraint sub-block; a tile owns the nodes whose
// lower-left-front element lies in its sub-block (plus the last node plane of
// each axis in the last tiles). A node's eight octant elements fall in the
// tile's own sub-block or in one of its seven lower neighbours, so a thread's
// share of B_n v is eight partial sums per continuum; they are summed over
// segments of min(TP, 64) lanes with DPP and across segments and tiles in a
// fixed order. p, r and K_n p are ring-padded (NC+3)^3 arrays in global
// memory; D^-1 per level node comes from the setup; x is kept in the output.
#include <hip/hip_runtime.h>

#include "kernels2d.h"

namespace mch {

constexpr int GEN3_T = 512;

template <int N>
constexpr int gen3_nv() { return 4 + 16 * N; }
template <int N>
constexpr int bslot3(int b, int sl, int j) { return 4 + (b * 8 + sl) * N + j; }

template <int N, bool GAL, int SEG>
__global__ __launch_bounds__(GEN3_T) __attribute__((amdgpu_waves_per_eu(2))) void k_solve3d_g(CellArgs a) {
  extern __shared__ double smem[];
  constexpr int NV = gen3_nv<N>();
  const int NC = a.NC, NP = NC + 1, PW = NC + 3, s = a.s, sbw = a.sbw, m = a.m, M = a.M;
  const int NT = blockDim.x, NW = NT / 64, ntile = s * s * s, TP = a.gen_tp;
  const int SPT = TP / SEG, nseg = ntile * SPT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tile = tid / TP, tl = tid % TP, seg = tid / SEG;
  const bool in_tile = tile < ntile;
  const int qx = in_tile ? tile % s : 0, qy = in_tile ? (tile / s) % s : 0, qz = in_tile ? tile / (s * s) : 0;
  const int X0 = qx * sbw, Y0 = qy * sbw, Z0 = qz * sbw;
  const int wX = in_tile ? (qx == s - 1 ? sbw + 1 : sbw) : 0;
  const int wY = in_tile ? (qy == s - 1 ? sbw + 1 : sbw) : 0;
  const int wZ = in_tile ? (qz == s - 1 ? sbw + 1 : sbw) : 0;
  const int tnodes = wX * wY * wZ;
  const int lo = a.bc ? 0 : 1, hi = a.bc ? NC : NC - 1;

  double* sinvS = smem;            // m*m
  double* cwS = sinvS + m * m;     // m
  double* uW = cwS + m;            // NW*64
  double* vW = uW + NW * 64;       // NW*64
  double* red = vW + NW * 64;      // nseg*4
  double* part = red + nseg * 4;   // [vec 2][segment][slot 8][N]

  const int cl = blockIdx.x / M, alpha = blockIdx.x % M;
  const int ci = a.ci0 + cl;
  const int p = a.cells[ci];
  const size_t vbase = (size_t)ci * M + alpha;
  const size_t nodes = (size_t)NP * NP * NP, padded = (size_t)PW * PW * PW;
  double* vr = a.vr + vbase * padded;
  double* vp = a.vp + vbase * padded;
  double* vap = a.vap + vbase * padded;
  const double* dinv = a.dinv + (size_t)ci * nodes;
  double* xo = a.out + vbase * nodes;
  const double* kwc = GAL ? nullptr : a.kw + (size_t)ci * NC * NC * NC;
  const uint8_t* lwc = GAL ? nullptr : a.labw + (size_t)ci * NC * NC * NC;
  const double* nW = GAL ? a.nodeW + (size_t)ci * nodes * 27 : nullptr;
  const float* nB = GAL ? a.nodeB + (size_t)ci * nodes * 8 * N : nullptr;

  for (int k = tid; k < m * m; k += NT) sinvS[k] = a.sinv[(size_t)p * m * m + k];
  for (int k = tid; k < m; k += NT) cwS[k] = a.cw[(size_t)p * m + k];

  auto pidx = [&](int X, int Y, int Z) { return ((size_t)(Z + 1) * PW + (Y + 1)) * PW + (X + 1); };
  auto nidx = [&](int X, int Y, int Z) { return ((size_t)Z * NP + Y) * NP + X; };
  auto is_free = [&](int X, int Y, int Z) {
    return X >= lo && Y >= lo && Z >= lo && X <= hi && Y <= hi && Z <= hi;
  };
  auto node_of = [&](int k, int& X, int& Y, int& Z) {
    X = X0 + k % wX;
    Y = Y0 + (k / wX) % wY;
    Z = Z0 + k / (wX * wY);
  };
  auto el_in = [&](int ex, int ey, int ez) { return ex >= 0 && ey >= 0 && ez >= 0 && ex < NC && ey < NC && ez < NC; };
  // constraint weights of node (X, Y, Z) per octant o (element
  // (X - 1 + o&1, Y - 1 + (o>>1)&1, Z - 1 + o>>2)) and continuum
  auto weights = [&](int X, int Y, int Z, float (&w)[8][N]) {
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int ex = X - 1 + (o & 1), ey = Y - 1 + ((o >> 1) & 1), ez = Z - 1 + (o >> 2);
      const bool inside = el_in(ex, ey, ez);
      if constexpr (GAL) {
        const float* b = nB + (nidx(X, Y, Z) * 8 + o) * N;
#pragma unroll
        for (int j = 0; j < N; ++j) w[o][j] = inside ? b[j] : 0.0f;
      } else {
        const int lab = inside ? (int)lwc[ex + NC * (ey + NC * ez)] : 255;
#pragma unroll
        for (int j = 0; j < N; ++j) w[o][j] = (lab == j) ? 1.0f : 0.0f;
      }
    }
  };
  // (K_n v)(X, Y, Z) from the ring-padded vector v
  auto stencil = [&](const double* v, int X, int Y, int Z) -> double {
    const double* c = v + pidx(X, Y, Z);
    auto at = [&](int dx, int dy, int dz) { return c[((ptrdiff_t)dz * PW + dy) * PW + dx]; };
    if constexpr (GAL) {
      const double* W = nW + nidx(X, Y, Z) * 27;
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < 27; ++k) t += W[k] * at(k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1);
      return t;
    } else {
      // element o on side (2 bit - 1) of each axis; the node is its corner
      // opposite to o: self 4, face diagonals and body diagonal -1
      const double c0 = at(0, 0, 0);
      double t = 0.0;
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const int sx = 2 * (o & 1) - 1, sy = 2 * ((o >> 1) & 1) - 1, sz = 2 * (o >> 2) - 1;
        const int ex = X - 1 + (o & 1), ey = Y - 1 + ((o >> 1) & 1), ez = Z - 1 + (o >> 2);
        const double kap = el_in(ex, ey, ez) ? kwc[ex + NC * (ey + NC * ez)] : 0.0;
        t += kap * (4.0 * c0 - at(sx, sy, 0) - at(sx, 0, sz) - at(0, sy, sz) - at(sx, sy, sz));
      }
      return t;
    }
  };
  // acc's B partials of vector b += w * v at (X, Y, Z): octant o falls in the
  // sub-block shifted down along each axis where the node is on the tile's
  // first plane and o lies below it
  auto add_B = [&](double (&acc)[NV], int b, const float (&w)[8][N], int X, int Y, int Z, double v) {
    const bool eL = X == X0, eB = Y == Y0, eD = Z == Z0;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int zmask = ((o & 1) ? 0 : 1) | (((o >> 1) & 1) ? 0 : 2) | ((o >> 2) ? 0 : 4);
      const int so = ((eL && !(o & 1)) ? 1 : 0) | ((eB && !((o >> 1) & 1)) ? 2 : 0) | ((eD && !(o >> 2)) ? 4 : 0);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const double val = (double)w[o][j] * v;
#pragma unroll
        for (int sl = 0; sl < 8; ++sl)
          if ((sl & ~zmask) == 0) acc[bslot3<N>(b, sl, j)] += (so == sl) ? val : 0.0;
      }
    }
  };
  auto zero_acc = [&](double (&acc)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  };
  // (B_n^T vcw)(X, Y, Z) from the wave's v*cw
  auto scatter = [&](const float (&w)[8][N], int X, int Y, int Z) -> double {
    const double* vv = vW + wave * 64;
    const bool eL = X == X0, eB = Y == Y0, eD = Z == Z0;
    double t = 0.0;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int bx = qx - ((eL && !(o & 1)) ? 1 : 0), by = qy - ((eB && !((o >> 1) & 1)) ? 1 : 0),
                bz = qz - ((eD && !(o >> 2)) ? 1 : 0);
      if (bx < 0 || by < 0 || bz < 0) continue;  // only octants outside the cell (weight 0)
      const int row = ((bz * s + by) * s + bx) * N;
#pragma unroll
      for (int j = 0; j < N; ++j) t += (double)w[o][j] * vv[row + j];
    }
    return t;
  };
  auto reduce = [&](double (&acc)[NV], int K, int nvec, int vec0) {
#pragma unroll
    for (int c0 = 0; c0 < NV; c0 += 4) {
      double v4[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v4[k] = c0 + k < NV ? acc[c0 + k] : 0.0;
      seg_sum_n<4>(v4, SEG);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (c0 + k < NV) acc[c0 + k] = v4[k];
    }
    if (seg < nseg && tid % SEG == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < K) red[seg * 4 + k] = acc[k];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (b >= nvec) continue;
#pragma unroll
        for (int sl = 0; sl < 8; ++sl)
#pragma unroll
          for (int j = 0; j < N; ++j) part[(((vec0 + b) * nseg + seg) * 8 + sl) * N + j] = acc[bslot3<N>(b, sl, j)];
      }
    }
  };
  // row k = (q, j) of B_n v (no cw): the shares of tile q (slot 0) and of its
  // upper neighbours (the slot of the shift), in a fixed order
  auto zrow = [&](int vec, int k) -> double {
    const int q = k / N, j = k % N, bx = q % s, by = (q / s) % s, bz = q / (s * s);
    const double* pv = part + (size_t)vec * nseg * 8 * N;
    double z = 0.0;
    for (int sl = 0; sl < 8; ++sl) {
      const int tx = bx + (sl & 1), ty = by + ((sl >> 1) & 1), tz = bz + (sl >> 2);
      if (tx >= s || ty >= s || tz >= s) continue;
      const int t = (tz * s + ty) * s + tx;
      for (int g = 0; g < SPT; ++g) z += pv[((t * SPT + g) * 8 + sl) * N + j];
    }
    return z;
  };
  auto seg_total = [&](int k) -> double {
    double t = 0.0;
    for (int g = 0; g < nseg; ++g) t += red[g * 4 + k];
    return t;
  };
  auto wave_schur = [&](double* vk) -> double {
    __builtin_amdgcn_wave_barrier();
    const double* u = uW + wave * 64;
    double v = 0.0;
    if (lane < m) {
      const double* row = sinvS + lane * m;
      for (int j = 0; j < m; ++j) v += row[j] * u[j];
    }
    const double uk = lane < m ? u[lane] : 0.0;
    *vk = lane < m ? v : 0.0;
    if (lane < m) vW[wave * 64 + lane] = v * cwS[lane];
    const double pu = wave_sum(lane < m ? v * uk : 0.0);
    __builtin_amdgcn_wave_barrier();
    return pu;
  };

  // ---- right-hand side f (parked in K_n p's slot until r is formed) ----------------
  const int nn1 = a.nc + 1;
  for (int k = tl; k < tnodes; k += TP) {
    int X, Y, Z;
    node_of(k, X, Y, Z);
    double f = 0.0;
    if (is_free(X, Y, Z)) {
      if (!a.adjoint) {
        if constexpr (GAL) f = a.fin[vbase * nodes + nidx(X, Y, Z)];
      } else {
        // adjoint: f = P^T Phibar, the explicit seed on the K_p nodes and the
        // seeds from the cells that inherit from this one (all fine nodes)
        const int r = a.r, H = a.H, Hp = H + 1, k0 = (a.nc - H) / 2;
        const double* skp = a.seed_kp + ((size_t)p * M + alpha) * (size_t)Hp * Hp * Hp;
        // the hat's support clipped to the K_p nodes (often empty)
        const int du0 = max(-(r - 1), k0 - X * r), du1 = min(r - 1, k0 + H - X * r);
        const int dv0 = max(-(r - 1), k0 - Y * r), dv1 = min(r - 1, k0 + H - Y * r);
        const int dw0 = max(-(r - 1), k0 - Z * r), dw1 = min(r - 1, k0 + H - Z * r);
        for (int dw = dw0; dw <= dw1; ++dw)
          for (int dv = dv0; dv <= dv1; ++dv)
            for (int du = du0; du <= du1; ++du) {
              const int fx = X * r + du - k0, fy = Y * r + dv - k0, fz = Z * r + dw - k0;
              const double wgt =
                  (1.0 - fabs((double)du) / r) * (1.0 - fabs((double)dv) / r) * (1.0 - fabs((double)dw) / r);
              f += wgt * skp[((size_t)fz * Hp + fy) * Hp + fx];
            }
        if (a.seed_par != nullptr) {
          const double* sp = a.seed_par + ((size_t)a.slot[p] * M + alpha) * (size_t)nn1 * nn1 * nn1;
          for (int dw = -(r - 1); dw <= r - 1; ++dw)
            for (int dv = -(r - 1); dv <= r - 1; ++dv)
              for (int du = -(r - 1); du <= r - 1; ++du) {
                const int fx = X * r + du, fy = Y * r + dv, fz = Z * r + dw;
                if (fx < 0 || fy < 0 || fz < 0 || fx > a.nc || fy > a.nc || fz > a.nc) continue;
                const double wgt =
                    (1.0 - fabs((double)du) / r) * (1.0 - fabs((double)dv) / r) * (1.0 - fabs((double)dw) / r);
                f += wgt * sp[((size_t)fz * nn1 + fy) * nn1 + fx];
              }
        }
      }
    }
    vap[pidx(X, Y, Z)] = f;
  }
  double* uw = uW + wave * 64;
  if (lane < m) {
    double gk = 0.0;
    if (!a.adjoint) gk = GAL ? a.gin[vbase * m + lane] : a.g[((size_t)p * M + alpha) * m + lane];
    uw[lane] = gk;
  }
  __syncthreads();  // sinvS, cwS

  // ---- feasible start x0 = D^-1 B^T S^-1 g' -----------------------------------------
  double vk = 0.0, Vacc = 0.0;
  (void)wave_schur(&vk);
  for (int k = tl; k < tnodes; k += TP) {
    int X, Y, Z;
    node_of(k, X, Y, Z);
    double x = 0.0;
    if (is_free(X, Y, Z)) {
      float w[8][N];
      weights(X, Y, Z, w);
      x = dinv[nidx(X, Y, Z)] * scatter(w, X, Y, Z);
    }
    xo[nidx(X, Y, Z)] = x;
    vp[pidx(X, Y, Z)] = x;
  }
  __syncthreads();
  double acc[NV];
  zero_acc(acc);
  for (int k = tl; k < tnodes; k += TP) {
    int X, Y, Z;
    node_of(k, X, Y, Z);
    double r = 0.0;
    if (is_free(X, Y, Z)) {
      r = stencil(vp, X, Y, Z) - vap[pidx(X, Y, Z)];
      const double t = dinv[nidx(X, Y, Z)] * r;
      acc[0] += r * t;
      float w[8][N];
      weights(X, Y, Z, w);
      add_B(acc, 0, w, X, Y, Z, t);
    }
    vr[pidx(X, Y, Z)] = r;
  }
  reduce(acc, 1, 1, 0);
  __syncthreads();
  const double rr0 = seg_total(0);
  if (lane < m) uw[lane] = cwS[lane] * zrow(0, lane);
  double vu = wave_schur(&vk);
  Vacc = vk;
  double rz = rr0 - vu;
  const double rz0 = rz;
  for (int k = tl; k < tnodes; k += TP) {
    int X, Y, Z;
    node_of(k, X, Y, Z);
    double r = 0.0, pv = 0.0;
    if (is_free(X, Y, Z)) {
      float w[8][N];
      weights(X, Y, Z, w);
      r = vr[pidx(X, Y, Z)] - scatter(w, X, Y, Z);
      pv = -dinv[nidx(X, Y, Z)] * r;
    }
    vr[pidx(X, Y, Z)] = r;
    vp[pidx(X, Y, Z)] = pv;
  }
  __syncthreads();

  const double tol2 = a.rtol * a.rtol * rz0;
  int it = 0;
  bool done = !(rz0 > 0.0);
  while (!done) {
    const bool withz0 = (it % 16) == 0;
    zero_acc(acc);
    for (int k = tl; k < tnodes; k += TP) {
      int X, Y, Z;
      node_of(k, X, Y, Z);
      if (!is_free(X, Y, Z)) continue;
      const size_t id = pidx(X, Y, Z);
      const double Ap = stencil(vp, X, Y, Z);
      const double di = dinv[nidx(X, Y, Z)];
      const double r = vr[id], pv = vp[id];
      const double t = di * r, tA = di * Ap;
      acc[0] += pv * Ap;
      acc[1] += r * t;
      acc[2] += t * Ap;
      acc[3] += Ap * tA;
      float w[8][N];
      weights(X, Y, Z, w);
      add_B(acc, 1, w, X, Y, Z, tA);
      if (withz0) add_B(acc, 0, w, X, Y, Z, t);
      vap[id] = Ap;
    }
    if (withz0) {
      reduce(acc, 4, 2, 0);
    } else {
#pragma unroll
      for (int k = 0; k < 8 * N; ++k) acc[bslot3<N>(0, 0, 0) + k] = acc[bslot3<N>(1, 0, 0) + k];
      reduce(acc, 4, 1, 1);
    }
    __syncthreads();
    const double pAp = seg_total(0), rrk = seg_total(1), rA = seg_total(2), AA = seg_total(3);
    const double irr = 1.0 / rrk;
    const double al = rrk / pAp;
    const double rDr = rrk + 2.0 * al * rA + al * al * AA;
    if (lane < m) uw[lane] = cwS[lane] * ((withz0 ? zrow(0, lane) : 0.0) + al * zrow(1, lane));
    vu = wave_schur(&vk);
    Vacc += vk;
    const double rzn = rDr - vu;
    ++it;
    const bool last = rzn <= tol2 || it >= a.max_iter;
    const double be = rzn * irr;
    rz = rzn;
    for (int k = tl; k < tnodes; k += TP) {
      int X, Y, Z;
      node_of(k, X, Y, Z);
      if (!is_free(X, Y, Z)) continue;
      const size_t id = pidx(X, Y, Z);
      const double pv = vp[id];
      xo[nidx(X, Y, Z)] += al * pv;
      if (last) continue;
      float w[8][N];
      weights(X, Y, Z, w);
      const double r = vr[id] + al * vap[id] - scatter(w, X, Y, Z);
      vr[id] = r;
      vp[id] = -dinv[nidx(X, Y, Z)] * r + be * pv;
    }
    __syncthreads();
    if (last) break;
  }

  // ---- final projection onto B_n x = g' --------------------------------------------
  {
    zero_acc(acc);
    for (int k = tl; k < tnodes; k += TP) {
      int X, Y, Z;
      node_of(k, X, Y, Z);
      if (!is_free(X, Y, Z)) continue;
      float w[8][N];
      weights(X, Y, Z, w);
      add_B(acc, 0, w, X, Y, Z, xo[nidx(X, Y, Z)]);
    }
    reduce(acc, 0, 1, 0);
    __syncthreads();
    if (lane < m) {
      double gk = 0.0;
      if (!a.adjoint) gk = GAL ? a.gin[vbase * m + lane] : a.g[((size_t)p * M + alpha) * m + lane];
      uw[lane] = cwS[lane] * zrow(0, lane) - gk;
    }
    (void)wave_schur(&vk);
    for (int k = tl; k < tnodes; k += TP) {
      int X, Y, Z;
      node_of(k, X, Y, Z);
      if (!is_free(X, Y, Z)) continue;
      float w[8][N];
      weights(X, Y, Z, w);
      xo[nidx(X, Y, Z)] -= dinv[nidx(X, Y, Z)] * scatter(w, X, Y, Z);
    }
  }

  if (wave == 0 && lane < m) a.beta[((size_t)p * M + alpha) * m + lane] = -Vacc;
  if (tid == 0) {
    a.iters[(size_t)p * M + alpha] = (rz0 == rz0) ? it : -1;
    a.resid[(size_t)p * M + alpha] = rel_resid(rz, rz0);
  }
}

// Threads per sub-block tile: the largest power of two TP with TP s^3 <= 512
// (at least 8), 0 if s^3 > 64.
int generic3_tile_threads(int s) {
  const int t = s * s * s;
  if (t > 64) return 0;
  int tp = GEN3_T;
  while (tp * t > GEN3_T) tp /= 2;
  return tp;
}

static size_t generic3_lds_bytes(int s, int N, int m, int threads, int tp) {
  const int NW = threads / 64, seg = tp < 64 ? tp : 64, nseg = s * s * s * (tp / seg);
  return ((size_t)m * m + m + 2 * (size_t)NW * 64 + (size_t)nseg * 4 + 2 * (size_t)nseg * 8 * N) * sizeof(double);
}

static const void* generic3_fn(int N, int TP, bool gal) {
  const int seg = TP < 64 ? TP : 64;
#define MCH_GEN3(n_, seg_)                                                                    \
  if (N == n_ && seg == seg_)                                                                 \
    return gal ? reinterpret_cast<const void*>(k_solve3d_g<n_, true, seg_>)                  \
               : reinterpret_cast<const void*>(k_solve3d_g<n_, false, seg_>);
  MCH_GEN3(1, 64) MCH_GEN3(2, 64) MCH_GEN3(3, 64) MCH_GEN3(1, 16) MCH_GEN3(2, 16) MCH_GEN3(1, 8)
#undef MCH_GEN3
  return nullptr;
}

int generic3_blocks_per_cu(const CellArgs& a) {
  const int threads = (a.gen_tp * a.s * a.s * a.s + 63) / 64 * 64;
  const void* fn = generic3_fn(a.N, a.gen_tp, false);
  if (!fn) return set_error(MCH_ENOTIMPL, "generic 3D solve: no kernel for this shape");
  int nb = 0;
  int rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                         &nb, fn, threads, generic3_lds_bytes(a.s, a.N, a.m, threads, a.gen_tp)),
                     "hipOccupancyMaxActiveBlocksPerMultiprocessor");
  return rc ? rc : nb;
}

int launch_solve3d_generic(const CellArgs& a, hipStream_t st) {
  const int TP = a.gen_tp;
  if (TP != generic3_tile_threads(a.s)) return set_error(MCH_EINVAL, "generic 3D solve: tile threads differ from the plan's");
  const int threads = (TP * a.s * a.s * a.s + 63) / 64 * 64;
  const void* fn = generic3_fn(a.N, TP, a.r > 1);
  if (!fn) return set_error(MCH_ENOTIMPL, "generic 3D solve: no kernel for this shape");
  const size_t lds = generic3_lds_bytes(a.s, a.N, a.m, threads, TP);
  if (lds > 64 * 1024) return set_error(MCH_EINVAL, "generic 3D solve exceeds its LDS budget");
  if (a.count == 0) return MCH_OK;
  CellArgs b = a;
  void* args[] = {&b};
  return hip_check(hipLaunchKernel(fn, dim3(a.count * a.M), dim3(threads), args, lds, st), "launch k_solve3d_g");
}

}  // namespace mch
