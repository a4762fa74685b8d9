// The 2D constrained cell solve for any level width and either cell
// boundary condition, with the Krylov vectors in global memory.
//
// The same problem and the same method as the register-resident kernel
// (solve2d_kernel.h): projected preconditioned CG with the constraint
// preconditioner [D B^T; B 0] (D = diag(K_n)) on
//   [K_n  B_n^T][xi  ]   [ f  ]
//   [B_n  0    ][beta] = [ g' ]
// (paper Sec. 2, Eqs. phi_avar / phi_grad; Sec. 3.3, Eqs.
// phi_avar_corrector / phi_grad_corrector), with the Gould-Hribar-Nocedal
// residual update, a feasible start x0 = D^-1 B^T S^-1 g', the fused
// reductions of one iteration and a per-wave Schur solve with the S^-1 of the
// setup kernel. It serves the shapes the register-resident kernel does not
// hold: cells wider than 64 level elements (the paper's larger oversampled
// cells), widths that are not powers of two (cells of an odd number of coarse
// blocks), and natural Neumann conditions on the cell boundary, where every
// node of [0, NC]^2 is free (the extra node row and column do not fit the
// other kernel's one-lane-per-column layout).
//
// Layout: one workgroup per (cell, right-hand side), at most 512 threads.
// The threads form one tile of TP lanes per constraint sub-block R_q (TP a
// power of two); a tile owns the level nodes whose lower-left element lies in
// R_q (plus node row/column NC in the last tiles) and loops over them. A
// node's quadrant elements belong to R_q or to its left, lower or lower-left
// neighbour, so a thread's share of B_n v is four partial sums per continuum.
// Partials are summed over segments of SEG = min(TP, 64) lanes with DPP and
// combined across segments and tiles in a fixed order: every result is
// bitwise reproducible. The search direction p lives in global memory with a ring of
// zeros ((NC+3)^2 per vector), so the 9-point stencil needs no bounds tests;
// r, K_n p and D^-1 likewise; x is kept in the output array. Two workgroup
// barriers per iteration: after the fused reduction and after p is written.
#include <hip/hip_runtime.h>

#include "kernels2d.h"

namespace mch {

constexpr int GEN_T = 512;  // most threads of a generic-solve workgroup
constexpr int UN = 2;       // nodes per thread whose loads an iteration sweep issues together

// A thread's partial sums, flat so that one DPP pass reduces them all: four
// dot products, then B_n partials [vector 2][slot: own, left, lower,
// lower-left][continuum].
template <int N>
constexpr int gen_nv() { return 4 + 8 * N; }
template <int N>
constexpr int bslot(int b, int sl, int j) { return 4 + (b * 4 + sl) * N + j; }

template <int N, bool GAL, int SEG>
__global__ __launch_bounds__(GEN_T) __attribute__((amdgpu_waves_per_eu(2))) void k_solve2d_g(CellArgs a) {
  extern __shared__ double smem[];
  constexpr int NV = gen_nv<N>();
  const int NC = a.NC, NP = NC + 1, PW = NC + 3, s = a.s, sbw = a.sbw, m = a.m, M = a.M;
  const int NT = blockDim.x, NW = NT / 64, ntile = s * s, TP = a.gen_tp;
  const int SPT = TP / SEG, nseg = ntile * SPT;  // segments per tile, in tiles
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tile = tid / TP, tl = tid % TP, seg = tid / SEG;
  const bool in_tile = tile < ntile;
  const int qx = in_tile ? tile % s : 0, qy = in_tile ? tile / s : 0;
  // tile's nodes: [X0, X0 + wX) x [Y0, Y0 + wY)
  const int X0 = qx * sbw, Y0 = qy * sbw;
  const int wX = in_tile ? (qx == s - 1 ? sbw + 1 : sbw) : 0;
  const int wY = in_tile ? (qy == s - 1 ? sbw + 1 : sbw) : 0;
  const int tnodes = wX * wY;
  const int lo = a.bc ? 0 : 1, hi = a.bc ? NC : NC - 1;

  double* sinvS = smem;                 // m*m, S^-1 row-major
  double* cwS = sinvS + m * m;          // m
  double* uW = cwS + m;                 // NW*64 per-wave right-hand side of the Schur solve
  double* vW = uW + NW * 64;            // NW*64 per-wave v*cw
  double* red = vW + NW * 64;           // nseg*4 dot-product partials
  double* part = red + nseg * 4;        // [vec 2][segment][slot 4][N]

  const int cl = blockIdx.x / M, alpha = blockIdx.x % M;
  const int ci = a.ci0 + cl;
  const int p = a.cells[ci];
  const size_t vbase = ((size_t)ci * M + alpha);
  double* vr = a.vr + vbase * PW * PW;
  double* vp = a.vp + vbase * PW * PW;
  double* vap = a.vap + vbase * PW * PW;
  double* dinv = a.dinv + vbase * NP * NP;
  double* xo = a.out + vbase * NP * NP;  // the iterate (level-1: Phi; else xi)
  const double* nW = GAL ? a.nodeW + (size_t)ci * NP * NP * 9 : nullptr;
  const float* nB = GAL ? a.nodeB + (size_t)ci * NP * NP * 4 * N : nullptr;

  for (int k = tid; k < m * m; k += NT) sinvS[k] = a.sinv[(size_t)p * m * m + k];
  for (int k = tid; k < m; k += NT) cwS[k] = a.cw[(size_t)p * m + k];

  auto pidx = [&](int X, int Y) { return (size_t)(Y + 1) * PW + (X + 1); };
  auto is_free = [&](int X, int Y) { return X >= lo && Y >= lo && X <= hi && Y <= hi; };
  // fine level: the cell's kappa/6 and label windows (written by the setup
  // kernel); kappa/6 of element (ex, ey), 0 outside the cell
  const double* kwc = GAL ? nullptr : a.kw + (size_t)ci * NC * NC;
  const uint8_t* lwc = GAL ? nullptr : a.labw + (size_t)ci * NC * NC;
  auto kq = [&](int ex, int ey) -> double {
    const bool in = ex >= 0 && ey >= 0 && ex < NC && ey < NC;
    const double v = kwc[(in ? ey : 0) * NC + (in ? ex : 0)];
    return in ? v : 0.0;
  };
  // constraint weights of node (X, Y) per quadrant (side + 2 part) and
  // continuum; quadrants outside the cell weigh 0. The quadrant's sub-block
  // is the tile's own, or its left (side 0 on the tile's first node column),
  // lower (part 0 on its first node row) or lower-left neighbour.
  auto weights = [&](int X, int Y, float (&w)[4][N]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int sd = q & 1, pt = q >> 1;
      const int ex = X - 1 + sd, ey = Y - 1 + pt;
      const bool inside = ex >= 0 && ey >= 0 && ex < NC && ey < NC;
      if constexpr (GAL) {
        const float* b = nB + ((size_t)(Y * NP + X) * 4 + sd * 2 + pt) * N;
#pragma unroll
        for (int j = 0; j < N; ++j) w[q][j] = inside ? b[j] : 0.0f;
      } else {
        const int l0 = lwc[(inside ? ey : 0) * NC + (inside ? ex : 0)];
        const int lab = inside ? l0 : 255;
#pragma unroll
        for (int j = 0; j < N; ++j) w[q][j] = (lab == j) ? 1.0f : 0.0f;
      }
    }
  };
  // (K_n v)(X, Y) from the ring-padded vector v
  auto stencil = [&](const double* v, int X, int Y) -> double {
    const double* c = v + pidx(X, Y);
    if constexpr (GAL) {
      const double* W = nW + (size_t)(Y * NP + X) * 9;
      double t = W[4] * c[0];
      t += W[1] * c[-PW] + W[7] * c[PW] + W[3] * c[-1] + W[5] * c[1];
      t += W[0] * c[-PW - 1] + W[2] * c[-PW + 1] + W[6] * c[PW - 1] + W[8] * c[PW + 1];
      return t;
    } else {
      const double kSW = kq(X - 1, Y - 1), kSE = kq(X, Y - 1), kNW = kq(X - 1, Y), kNE = kq(X, Y);
      const double aS = kSW + kSE, aN = kNW + kNE, aW = kSW + kNW, aE = kSE + kNE;
      double t = 4.0 * (aS + aN) * c[0];
      t -= aS * c[-PW] + aN * c[PW] + aW * c[-1] + aE * c[1];
      t -= 2.0 * (kSW * c[-PW - 1] + kSE * c[-PW + 1] + kNW * c[PW - 1] + kNE * c[PW + 1]);
      return t;
    }
  };
  // acc's B partials of vector b += w * v at node (X, Y): quadrant 3 always
  // falls in the tile's own sub-block, quadrant 1 (part 0) in the lower one
  // on the first node row, quadrant 2 (side 0) in the left one on the first
  // node column, quadrant 0 in either or the lower-left one
  auto add_B = [&](double (&acc)[NV], int b, const float (&w)[4][N], int X, int Y, double v) {
    const bool eL = X == X0, eB = Y == Y0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const double w0 = (double)w[0][j] * v, w1 = (double)w[1][j] * v;
      const double w2 = (double)w[2][j] * v, w3 = (double)w[3][j] * v;
      acc[bslot<N>(b, 0, j)] += ((w3 + (eB ? 0.0 : w1)) + (eL ? 0.0 : w2)) + ((eL || eB) ? 0.0 : w0);
      acc[bslot<N>(b, 1, j)] += (eL ? w2 : 0.0) + ((eL && !eB) ? w0 : 0.0);
      acc[bslot<N>(b, 2, j)] += (eB ? w1 : 0.0) + ((eB && !eL) ? w0 : 0.0);
      acc[bslot<N>(b, 3, j)] += (eL && eB) ? w0 : 0.0;
    }
  };
  auto zero_acc = [&](double (&acc)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  };
  // (B_n^T vcw)(X, Y) from the wave's v*cw
  auto scatter = [&](const float (&w)[4][N], int X, int Y) -> double {
    const double* vv = vW + wave * 64;
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int bx = qx - ((X == X0 && (q & 1) == 0) ? 1 : 0), by = qy - ((Y == Y0 && (q >> 1) == 0) ? 1 : 0);
      if (bx < 0 || by < 0) continue;  // only quadrants outside the cell (weight 0)
      const int row = (by * s + bx) * N;
#pragma unroll
      for (int j = 0; j < N; ++j) t += (double)w[q][j] * vv[row + j];
    }
    return t;
  };
  // segment sums of acc: the first K dot products into red, nvec (1 or 2)
  // B partial sets into part vectors vec0.. (lane 0 of each segment)
  auto reduce = [&](double (&acc)[NV], int K, int nvec, int vec0) {
    // four values per DPP pass: fewer registers held in flight
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
        for (int sl = 0; sl < 4; ++sl)
#pragma unroll
          for (int j = 0; j < N; ++j) part[(((vec0 + b) * nseg + seg) * 4 + sl) * N + j] = acc[bslot<N>(b, sl, j)];
      }
    }
  };
  // row k = (q, j) of B_n v (no cw) from the segment partials of vector vec,
  // in a fixed order: tile q's own share, then the right, upper and
  // upper-right tiles' shares
  auto zrow = [&](int vec, int k) -> double {
    const int q = k / N, j = k % N, bx = q % s, by = q / s;
    const double* pv = part + (size_t)vec * nseg * 4 * N;
    auto share = [&](int tx, int ty, int sl) {
      double z = 0.0;
      for (int g = 0; g < SPT; ++g) z += pv[(((ty * s + tx) * SPT + g) * 4 + sl) * N + j];
      return z;
    };
    double z = share(bx, by, 0);
    if (bx + 1 < s) z += share(bx + 1, by, 1);
    if (by + 1 < s) z += share(bx, by + 1, 2);
    if (bx + 1 < s && by + 1 < s) z += share(bx + 1, by + 1, 3);
    return z;
  };
  auto seg_total = [&](int k) -> double {
    double t = 0.0;
    for (int g = 0; g < nseg; ++g) t += red[g * 4 + k];
    return t;
  };
  // Per wave: v = S^-1 u for u in uW[wave] (lanes < m); vW[wave] = v*cw;
  // returns v.u on every lane and v_k on lane k
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

  // ---- D^-1 and the right-hand side f ------------------------------------------
  const int k0 = (a.nc - a.H) / 2;  // first fine node of K_p
  const int nn1 = a.nc + 1;
  for (int k = tl; k < tnodes; k += TP) {
    const int X = X0 + k % wX, Y = Y0 + k / wX;
    double di = 0.0;
    if (is_free(X, Y)) {
      if constexpr (GAL) {
        di = 1.0 / nW[(size_t)(Y * NP + X) * 9 + 4];
      } else {
        const double ks = kq(X - 1, Y - 1) + kq(X, Y - 1) + kq(X - 1, Y) + kq(X, Y);
        di = 1.0 / (4.0 * ks);
      }
    }
    dinv[Y * NP + X] = di;
    double f = 0.0;
    if (is_free(X, Y)) {
      if (!a.adjoint) {
        if constexpr (GAL) f = a.fin[vbase * NP * NP + Y * NP + X];
      } else {
        // adjoint: f = P^T Phibar, the explicit seed on the K_p nodes and the
        // seeds from the cells that inherit from this one (all fine nodes)
        const double* skp = a.seed_kp + ((size_t)p * M + alpha) * (size_t)((a.H + 1) * (a.H + 1));
        const int rr = a.r;
        // the hat's support clipped to the K_p nodes (often empty)
        const int du0 = max(-(rr - 1), k0 - X * rr), du1 = min(rr - 1, k0 + a.H - X * rr);
        const int dv0 = max(-(rr - 1), k0 - Y * rr), dv1 = min(rr - 1, k0 + a.H - Y * rr);
        for (int dv = dv0; dv <= dv1; ++dv)
          for (int du = du0; du <= du1; ++du) {
            const int fx = X * rr + du - k0, fy = Y * rr + dv - k0;
            const double wgt = (1.0 - fabs((double)du) / rr) * (1.0 - fabs((double)dv) / rr);
            f += wgt * skp[fy * (a.H + 1) + fx];
          }
        if (a.seed_par != nullptr) {
          const double* sp = a.seed_par + ((size_t)a.slot[p] * M + alpha) * (size_t)(nn1 * nn1);
          for (int dv = -(rr - 1); dv <= rr - 1; ++dv)
            for (int du = -(rr - 1); du <= rr - 1; ++du) {
              const int fx = X * rr + du, fy = Y * rr + dv;
              if (fx < 0 || fy < 0 || fx > a.nc || fy > a.nc) continue;
              const double wgt = (1.0 - fabs((double)du) / rr) * (1.0 - fabs((double)dv) / rr);
              f += wgt * sp[(size_t)fy * nn1 + fx];
            }
        }
      }
    }
    vap[pidx(X, Y)] = f;  // f parked in K_n p's slot until r is formed
  }
  double* uw = uW + wave * 64;
  if (lane < m) {
    double gk = 0.0;
    if (!a.adjoint) gk = GAL ? a.gin[vbase * m + lane] : a.g[((size_t)p * M + alpha) * m + lane];
    uw[lane] = gk;
  }
  __syncthreads();  // sinvS, cwS

  // ---- feasible start x0 = D^-1 B^T S^-1 g' -------------------------------------
  double vk = 0.0, Vacc = 0.0;
  (void)wave_schur(&vk);
  for (int k = tl; k < tnodes; k += TP) {
    const int X = X0 + k % wX, Y = Y0 + k / wX;
    double x = 0.0;
    if (is_free(X, Y)) {
      float w[4][N];
      weights(X, Y, w);
      x = dinv[Y * NP + X] * scatter(w, X, Y);
    }
    xo[Y * NP + X] = x;
    vp[pidx(X, Y)] = x;
  }
  __syncthreads();
  // r = K x0 - f, t = D^-1 r; r.t and B t
  double acc[NV];
  zero_acc(acc);
  for (int k = tl; k < tnodes; k += TP) {
    const int X = X0 + k % wX, Y = Y0 + k / wX;
    double r = 0.0;
    if (is_free(X, Y)) {
      r = stencil(vp, X, Y) - vap[pidx(X, Y)];
      const double t = dinv[Y * NP + X] * r;
      acc[0] += r * t;
      float w[4][N];
      weights(X, Y, w);
      add_B(acc, 0, w, X, Y, t);
    }
    vr[pidx(X, Y)] = r;
  }
  reduce(acc, 1, 1, 0);
  __syncthreads();
  const double rr0 = seg_total(0);
  if (lane < m) uw[lane] = cwS[lane] * zrow(0, lane);
  double vu = wave_schur(&vk);
  Vacc = vk;
  double rz = rr0 - vu;
  const double rz0 = rz;
  // projected residual and p = -D^-1 r
  for (int k = tl; k < tnodes; k += TP) {
    const int X = X0 + k % wX, Y = Y0 + k / wX;
    double r = 0.0, pv = 0.0;
    if (is_free(X, Y)) {
      float w[4][N];
      weights(X, Y, w);
      r = vr[pidx(X, Y)] - scatter(w, X, Y);
      pv = -dinv[Y * NP + X] * r;
    }
    vr[pidx(X, Y)] = r;
    vp[pidx(X, Y)] = pv;
  }
  __syncthreads();

  const double tol2 = a.rtol * a.rtol * rz0;
  int it = 0;
  bool done = !(rz0 > 0.0);
  while (!done) {
    // K p, p.Kp, r.D^-1 r, r.D^-1 Kp, Kp.D^-1 Kp, B D^-1 r (every
    // ZPERIOD iterations; it vanishes up to rounding) and B D^-1 Kp
    const bool withz0 = (it % 16) == 0;
    zero_acc(acc);
    // UN nodes per pass: their loads are issued together (node indices past
    // the tile's last are clamped to its first node and their results dropped)
    for (int kb = tl; kb < tnodes; kb += UN * TP) {
      int Xs[UN], Ys[UN];
      bool use[UN];
      double Ap[UN], r[UN], pv[UN], di[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int k = kb + u * TP;
        const int kk = k < tnodes ? k : kb;
        Xs[u] = X0 + kk % wX;
        Ys[u] = Y0 + kk / wX;
        use[u] = k < tnodes && is_free(Xs[u], Ys[u]);
        const size_t id = pidx(Xs[u], Ys[u]);
        Ap[u] = stencil(vp, Xs[u], Ys[u]);
        r[u] = vr[id];
        pv[u] = vp[id];
        di[u] = dinv[Ys[u] * NP + Xs[u]];
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        if (!use[u]) continue;
        const double t = di[u] * r[u], tA = di[u] * Ap[u];
        acc[0] += pv[u] * Ap[u];
        acc[1] += r[u] * t;
        acc[2] += t * Ap[u];
        acc[3] += Ap[u] * tA;
        float w[4][N];
        weights(Xs[u], Ys[u], w);
        add_B(acc, 1, w, Xs[u], Ys[u], tA);
        if (withz0) add_B(acc, 0, w, Xs[u], Ys[u], t);
        vap[pidx(Xs[u], Ys[u])] = Ap[u];
      }
    }
    // vec 0 of part holds B D^-1 r, vec 1 B D^-1 Kp (the partials of vector
    // 1 are moved to set 0 when set 0 is not formed, so one set is reduced)
    if (withz0) {
      reduce(acc, 4, 2, 0);
    } else {
#pragma unroll
      for (int k = 0; k < 4 * N; ++k) acc[bslot<N>(0, 0, 0) + k] = acc[bslot<N>(1, 0, 0) + k];
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
    for (int kb = tl; kb < tnodes; kb += UN * TP) {
      int Xs[UN], Ys[UN];
      bool use[UN];
      double xv[UN], pv[UN], r[UN], Ap[UN], di[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int k = kb + u * TP;
        const int kk = k < tnodes ? k : kb;
        Xs[u] = X0 + kk % wX;
        Ys[u] = Y0 + kk / wX;
        use[u] = k < tnodes && is_free(Xs[u], Ys[u]);
        const size_t id = pidx(Xs[u], Ys[u]);
        xv[u] = xo[Ys[u] * NP + Xs[u]];
        pv[u] = vp[id];
        r[u] = vr[id];
        Ap[u] = vap[id];
        di[u] = dinv[Ys[u] * NP + Xs[u]];
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        if (!use[u]) continue;
        const size_t id = pidx(Xs[u], Ys[u]);
        xo[Ys[u] * NP + Xs[u]] = xv[u] + al * pv[u];
        if (last) continue;
        float w[4][N];
        weights(Xs[u], Ys[u], w);
        const double rn = r[u] + al * Ap[u] - scatter(w, Xs[u], Ys[u]);
        vr[id] = rn;
        vp[id] = -di[u] * rn + be * pv[u];
      }
    }
    __syncthreads();
    if (last) break;
  }

  // ---- final projection onto B_n x = g' -------------------------------------------
  // x -= D^-1 B_n^T S^-1 (B_n x - g'): one correction brings the constraint
  // residual back to rounding level
  {
    zero_acc(acc);
    for (int k = tl; k < tnodes; k += TP) {
      const int X = X0 + k % wX, Y = Y0 + k / wX;
      if (!is_free(X, Y)) continue;
      float w[4][N];
      weights(X, Y, w);
      add_B(acc, 0, w, X, Y, xo[Y * NP + X]);
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
      const int X = X0 + k % wX, Y = Y0 + k / wX;
      if (!is_free(X, Y)) continue;
      float w[4][N];
      weights(X, Y, w);
      xo[Y * NP + X] -= dinv[Y * NP + X] * scatter(w, X, Y);
    }
  }

  // ---- outputs ----------------------------------------------------------------------
  if (wave == 0 && lane < m) a.beta[((size_t)p * M + alpha) * m + lane] = -Vacc;
  if (tid == 0) {
    a.iters[(size_t)p * M + alpha] = (rz0 == rz0) ? it : -1;
    a.resid[(size_t)p * M + alpha] = rel_resid(rz, rz0);
  }
}

// Threads per sub-block tile for s sub-blocks per axis: the largest power of
// two TP with TP s^2 <= 512 (at least 8), 0 if s^2 > 64.
int generic_tile_threads(int s) {
  const int t = s * s;
  if (t > 64) return 0;
  int tp = GEN_T;
  while (tp * t > GEN_T) tp /= 2;
  return tp;
}

size_t generic_lds_bytes(int s, int N, int m, int threads) {
  const int NW = threads / 64, tp = generic_tile_threads(s), seg = tp < 64 ? tp : 64;
  const int nseg = s * s * (tp / seg);
  return ((size_t)m * m + m + 2 * (size_t)NW * 64 + (size_t)nseg * 4 + 2 * (size_t)nseg * 4 * N) * sizeof(double);
}

static const void* generic_fn(int N, int TP, bool gal) {
  const int seg = TP < 64 ? TP : 64;
#define MCH_GEN(n_, seg_)                                                                     \
  if (N == n_ && seg == seg_)                                                                 \
    return gal ? reinterpret_cast<const void*>(k_solve2d_g<n_, true, seg_>)                  \
               : reinterpret_cast<const void*>(k_solve2d_g<n_, false, seg_>);
  MCH_GEN(1, 64) MCH_GEN(1, 32) MCH_GEN(1, 16) MCH_GEN(1, 8) MCH_GEN(1, 4)
  MCH_GEN(2, 64) MCH_GEN(2, 32) MCH_GEN(2, 16) MCH_GEN(2, 8)
  MCH_GEN(3, 64) MCH_GEN(3, 32) MCH_GEN(3, 16)
#undef MCH_GEN
  return nullptr;
}

int generic_blocks_per_cu(const CellArgs& a) {
  const int threads = (a.gen_tp * a.s * a.s + 63) / 64 * 64;
  const void* fn = generic_fn(a.N, a.gen_tp, false);
  if (!fn) return set_error(MCH_ENOTIMPL, "generic solve: no kernel for this number of continua");
  int nb = 0;
  int rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, generic_lds_bytes(a.s, a.N, a.m, threads)),
                     "hipOccupancyMaxActiveBlocksPerMultiprocessor");
  return rc ? rc : nb;
}

int launch_solve_generic(const CellArgs& a, hipStream_t st) {
  const int TP = a.gen_tp;
  if (TP != generic_tile_threads(a.s)) return set_error(MCH_EINVAL, "generic solve: tile threads differ from the plan's");
  const int threads = (TP * a.s * a.s + 63) / 64 * 64;
  const void* fn = generic_fn(a.N, TP, a.r > 1);
  if (!fn) return set_error(MCH_ENOTIMPL, "generic solve: no kernel for this number of continua");
  const size_t lds = generic_lds_bytes(a.s, a.N, a.m, threads);
  if (lds > 64 * 1024) return set_error(MCH_EINVAL, "generic solve exceeds its LDS budget");
  if (a.count == 0) return MCH_OK;
  CellArgs b = a;
  void* args[] = {&b};
  return hip_check(hipLaunchKernel(fn, dim3(a.count * a.M), dim3(threads), args, lds, st), "launch k_solve2d_g");
}

}  // namespace mch
