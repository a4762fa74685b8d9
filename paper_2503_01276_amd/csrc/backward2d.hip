// 2D adjoint of the effective tensors with respect to log kappa.
//
// The paper gives no adjoint; it follows from the cell equations
// (Eqs. phi_avar_corrector / phi_grad_corrector with I = 0 on level 1) and
// Eq. Bs_defi. For a loss with G_p = dLoss/dA_eff(p), per cell
//   Phibar_a = sum_b (G_ab + G_ba) K^{K_p} Phi_b  (+ seeds from inheriting cells),
//   [K_n B_n^T; B_n 0][w_a; mu_a] = [P^T Phibar_a; 0],
//   dLoss/dkappa_e += -(P w_a)|_e^T K_ref Phi_a|_e           (every element of the cell)
//                   + sum_ab G_ab Phi_a|_e^T K_ref Phi_b|_e   (elements of K_p),
//   Ibar_a = Phibar_a - K_h P w_a - B_h^T mu_a                (seed of the inherited cell),
// processed from the last level down to level 1, then dLoss/dlog kappa = kappa dLoss/dkappa.
//
// Determinism: no floating-point atomics. Each cell writes its gradient
// window to its own buffer, the seeds of a level-1 cell are summed over its
// inheriting cells in a fixed order, and a gather kernel adds the windows
// covering each fine element in a fixed order.
#include <cstdio>

#include "kernels2d.h"

namespace mch {

constexpr int BT = 256;

// Explicit seeds on the K_p nodes and the explicit K_p gradient term.
template <int MM>
__global__ __launch_bounds__(BT) void k_seed2d(CellArgs a, const double* gA, double* seed_kp, double* gk) {
  extern __shared__ double sm[];
  const int H = a.H, Hp = H + 1;
  double* ph = sm;                // [MM][Hp*Hp]
  double* G = ph + MM * Hp * Hp;  // [MM*MM]
  const int tid = threadIdx.x;
  const int ci = a.ci0 + blockIdx.x;
  const int p = a.cells[ci];
  const int k0 = (a.nc - H) / 2;
  for (int k = tid; k < MM * Hp * Hp; k += BT) {
    const int al = k / (Hp * Hp), nd = k % (Hp * Hp);
    ph[k] = phi_at(a, ci, al, k0 + nd % Hp, k0 + nd / Hp);
  }
  for (int k = tid; k < MM * MM; k += BT) G[k] = gA[(size_t)p * MM * MM + k];
  __syncthreads();
  const int jx = p % a.n_macro, jy = p / a.n_macro;
  for (int nd = tid; nd < Hp * Hp; nd += BT) {
    const int X = nd % Hp, Y = nd / Hp;
    double kphi[MM];
#pragma unroll
    for (int b = 0; b < MM; ++b) kphi[b] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ex = X - 1 + (q & 1), ey = Y - 1 + (q >> 1);
      if (ex < 0 || ey < 0 || ex >= H || ey >= H) continue;
      const double k6 = a.kappa[(size_t)(H * jy + ey) * a.n + (H * jx + ex)] * (1.0 / 6.0);
      // node (X, Y) is corner c of the element; only row c of 6 K_ref is
      // needed: 4 v_c - 2 v_(c^3) - v_(c^1) - v_(c^2)
      const int c = (X - ex) + 2 * (Y - ey);
      const int o0 = (ey + (c >> 1)) * Hp + ex + (c & 1);
      const int o3 = (ey + ((c ^ 3) >> 1)) * Hp + ex + ((c ^ 3) & 1);
      const int o1 = (ey + ((c ^ 1) >> 1)) * Hp + ex + ((c ^ 1) & 1);
      const int o2 = (ey + ((c ^ 2) >> 1)) * Hp + ex + ((c ^ 2) & 1);
#pragma unroll
      for (int b = 0; b < MM; ++b) {
        const double* pb = ph + b * Hp * Hp;
        kphi[b] += k6 * (4.0 * pb[o0] - 2.0 * pb[o3] - pb[o1] - pb[o2]);
      }
    }
#pragma unroll
    for (int al = 0; al < MM; ++al) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < MM; ++b) s += (G[al * MM + b] + G[b * MM + al]) * kphi[b];
      seed_kp[((size_t)p * MM + al) * Hp * Hp + nd] = s;
    }
  }
  // explicit kappa term per element: sum_ab G_ab Phi_a^T K_ref Phi_b
  // = sum_a Phi_a^T K_ref w_a with w_a = sum_b G_ab Phi_b (element corners)
  for (int e = tid; e < H * H; e += BT) {
    const int ex = e % H, ey = e / H;
    double v[MM][4];
#pragma unroll
    for (int al = 0; al < MM; ++al) {
#pragma unroll
      for (int d = 0; d < 4; ++d) v[al][d] = ph[al * Hp * Hp + (ey + (d >> 1)) * Hp + ex + (d & 1)];
    }
    double t = 0.0;
#pragma unroll 1
    for (int al = 0; al < MM; ++al) {
      double w[4] = {0.0, 0.0, 0.0, 0.0}, y[4], va[4];
#pragma unroll
      for (int b = 0; b < MM; ++b) {
        const double g = G[al * MM + b];
#pragma unroll
        for (int d = 0; d < 4; ++d) w[d] += g * v[b][d];
      }
      kref6_apply(w, y);
      // Phi_a at the corners again from LDS (a runtime index into v would
      // put the array in scratch memory)
#pragma unroll
      for (int d = 0; d < 4; ++d) va[d] = ph[al * Hp * Hp + (ey + (d >> 1)) * Hp + ex + (d & 1)];
      t += va[0] * y[0] + va[1] * y[1] + va[2] * y[2] + va[3] * y[3];
    }
    gk[(size_t)(H * jy + ey) * a.n + (H * jx + ex)] = t * (1.0 / 6.0);
  }
}

// Per-cell gradient window: gcell[p][e] = -sum_a (P w_a)|_e^T K_ref Phi_a|_e.
// A thread owns fine elements and loops over the right-hand sides; Phi and
// P w at the element's corners come from the coarse element's corner values
// (no LDS, so many workgroups share a CU).
__global__ __launch_bounds__(BT) void k_grad2d(CellArgs a, const double* w, double* gcell) {
  const int nc = a.nc, nn1 = nc + 1, r = a.r, NC = a.NC, NP = NC + 1, M = a.M;
  const int ci = a.ci0 + blockIdx.x;
  const int p = a.cells[ci];
  const size_t NN = (size_t)NP * NP, nn = (size_t)nn1 * nn1;
  const double inv_r = 1.0 / r;
  for (int e = threadIdx.x; e < nc * nc; e += BT) {
    const int fx = e % nc, fy = e / nc;
    const int EX = fx / r, EY = fy / r, ux = fx - EX * r, uy = fy - EY * r;
    double acc = 0.0;
    for (int al = 0; al < M; ++al) {
      const double* wv = w + ((size_t)ci * M + al) * NN;
      double phi[4], pw[4], y[4];
      if (r == 1) {
        const double* xv = a.out + ((size_t)ci * M + al) * nn;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const size_t q = (size_t)(fy + (d >> 1)) * nn1 + fx + (d & 1);
          phi[d] = xv[q];
          pw[d] = wv[q];
        }
      } else {
        const double* I = a.phi1 + ((size_t)a.pslot[ci] * M + al) * nn;
        const double* xi = a.out + ((size_t)ci * M + al) * NN;
        double xe[4], we[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const size_t q = (size_t)(EY + (c >> 1)) * NP + EX + (c & 1);
          xe[c] = xi[q];
          we[c] = wv[q];
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const double tx = (ux + (d & 1)) * inv_r, ty = (uy + (d >> 1)) * inv_r;
          const double w00 = (1.0 - tx) * (1.0 - ty), w10 = tx * (1.0 - ty), w01 = (1.0 - tx) * ty, w11 = tx * ty;
          phi[d] = I[(size_t)(fy + (d >> 1)) * nn1 + fx + (d & 1)] +
                   ((w00 * xe[0] + w10 * xe[1]) + (w01 * xe[2] + w11 * xe[3]));
          pw[d] = (w00 * we[0] + w10 * we[1]) + (w01 * we[2] + w11 * we[3]);
        }
      }
      kref6_apply(phi, y);
      acc -= (pw[0] * y[0] + pw[1] * y[1]) + (pw[2] * y[2] + pw[3] * y[3]);
    }
    gcell[(size_t)p * nc * nc + e] = acc * (1.0 / 6.0);
  }
}

struct LevelTab {
  int r[MAX_LEVELS];
  int NC[MAX_LEVELS];
  const double* w[MAX_LEVELS];
};

// Seeds of level-1 cell t for right-hand side alpha: sum over its inheriting
// cells c of Ibar_c = Phibar_c - K_h(c) P w_c - B_h(c)^T mu_c on the free fine
// nodes. 1024 threads; a thread owns up to NODES fine nodes and keeps their
// sums in registers; per child the LDS holds P w, labels, cw*mu and (KLDS)
// kappa/6: about 70 KB for 64^2 cells. 128^2 cells read kappa from global
// memory instead (P w alone is 133 KB there) and add each child's term to
// the output in place (the same thread's nodes in every pass, so no race;
// 17 sums per thread would not fit the registers of 1024 threads).
constexpr int IBT = 1024;
constexpr int IB_NODES = 5;       // ceil(65^2 / 1024): cells up to 64 elements wide
constexpr int IB_NODES_BIG = 17;  // ceil(129^2 / 1024): cells up to 128 elements wide

// prolong_at for a power-of-two ratio r = 2^sh (inv = 1 / r): shifts and
// masks instead of integer division, the same interpolation formula.
MCH_DEV double prolong_p2(const double* v, int sh, double inv, int NC, int X, int Y) {
  const int NCp = NC + 1, msk = (1 << sh) - 1;
  const int cx = X >> sh, cy = Y >> sh, fx = X & msk, fy = Y & msk;
  const double tx = fx * inv, ty = fy * inv;
  const int cx1 = cx + (fx > 0 ? 1 : 0), cy1 = cy + (fy > 0 ? 1 : 0);
  return (1 - tx) * (1 - ty) * v[cy * NCp + cx] + tx * (1 - ty) * v[cy * NCp + cx1] +
         (1 - tx) * ty * v[cy1 * NCp + cx] + tx * ty * v[cy1 * NCp + cx1];
}

template <int NODES, bool KLDS>
__global__ __launch_bounds__(IBT) void k_ibar2d(CellArgs a, LevelTab lt, const int32_t* level, const int32_t* child_ptr,
                                                const int32_t* child, const double* mu, double* seed_par,
                                                int only_level, int accumulate) {
  extern __shared__ double sm[];
  const int nc = a.nc, nn1 = nc + 1, H = a.H, Hp = H + 1, m = a.m, N = a.N, s = a.s;
  const int nn = nn1 * nn1;
  const int flo = a.bc ? 0 : 1, fhi = a.bc ? nc : nc - 1;  // free fine nodes
  double* pwS = sm;                       // [nn1^2]
  double* kS = pwS + nn;                  // KLDS: [nc^2] kappa/6
  double* cmS = KLDS ? kS + nc * nc : kS; // [m] cw * mu
  uint8_t* labS = reinterpret_cast<uint8_t*>(cmS + m);  // [nc^2]
  const int tid = threadIdx.x;
  const int t = a.ci0 + blockIdx.x / a.M, al = blockIdx.x % a.M;
  const int k0 = (nc - H) / 2, sb = nc / s;
  double acc[KLDS ? NODES : 1];
#pragma unroll
  for (int i = 0; i < (KLDS ? NODES : 1); ++i) acc[i] = 0.0;
  double* dst = seed_par + ((size_t)t * a.M + al) * nn;
  if constexpr (!KLDS) {
    if (!accumulate)
      for (int nd = tid; nd < nn; nd += IBT) dst[nd] = 0.0;
  }
  for (int ch = child_ptr[t]; ch < child_ptr[t + 1]; ++ch) {
    const int p = child[ch];
    const int l = level[p] - 1;
    if (only_level >= 0 && l != only_level) continue;  // uniform across the block
    const int ci = a.slot[p];
    const int jx = p % a.n_macro, jy = p / a.n_macro;
    const int ox = H * jx + H / 2 - nc / 2, oy = H * jy + H / 2 - nc / 2;
    __syncthreads();  // previous child's data fully consumed
    for (int e = tid; e < nc * nc; e += IBT) {
      const int ex = e % nc, ey = e / nc;
      const size_t ge = (size_t)wrap1(oy + ey, a.n) * a.n + wrap1(ox + ex, a.n);
      if constexpr (KLDS) kS[e] = a.kappa[ge] * (1.0 / 6.0);
      labS[e] = a.label[ge];
    }
    for (int k = tid; k < m; k += IBT) cmS[k] = a.cw[(size_t)p * m + k] * mu[((size_t)p * a.M + al) * m + k];
    const double* wv = lt.w[l] + ((size_t)ci * a.M + al) * (size_t)(lt.NC[l] + 1) * (lt.NC[l] + 1);
    const int rl = lt.r[l];
    if ((rl & (rl - 1)) == 0) {
      const int sh = __builtin_ctz(rl);
      const double inv = 1.0 / rl;
      for (int nd = tid; nd < nn; nd += IBT) pwS[nd] = prolong_p2(wv, sh, inv, lt.NC[l], nd % nn1, nd / nn1);
    } else {
      for (int nd = tid; nd < nn; nd += IBT) pwS[nd] = prolong_at(wv, rl, lt.NC[l], nd % nn1, nd / nn1);
    }
    __syncthreads();
    const double* skp = a.seed_kp + ((size_t)p * a.M + al) * Hp * Hp;
    // (unrolled when the sums stay in registers; a runtime loop otherwise,
    // which keeps the per-node temporaries of one node live at a time)
#pragma unroll(KLDS ? NODES : 1)
    for (int i = 0; i < NODES; ++i) {
      const int nd = tid + i * IBT;
      if (nd >= nn) break;
      const int X = nd % nn1, Y = nd / nn1;
      if (X < flo || Y < flo || X > fhi || Y > fhi) continue;
      double v[3][3];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) v[dy][dx] = pwS[(Y - 1 + dy) * nn1 + X - 1 + dx];
      double kpw = 0.0, btmu = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int qx = q & 1, qy = q >> 1;
        const int ex = X - 1 + qx, ey = Y - 1 + qy;
        if (ex < 0 || ey < 0 || ex >= nc || ey >= nc) continue;  // outside the cell (Neumann boundary)
        const int e = ey * nc + ex;
        const double c[4] = {v[qy][qx], v[qy][qx + 1], v[qy + 1][qx], v[qy + 1][qx + 1]};
        // the node is corner cn of the element: row cn of 6 K_ref only
        const int cn = (1 - qx) + 2 * (1 - qy);
        double ke;
        if constexpr (KLDS)
          ke = kS[e];
        else
          ke = a.kappa[(size_t)wrap1(oy + ey, a.n) * a.n + wrap1(ox + ex, a.n)] * (1.0 / 6.0);
        kpw += ke * (4.0 * c[cn] - 2.0 * c[cn ^ 3] - c[cn ^ 1] - c[cn ^ 2]);
        const int lab = labS[e];
        if (lab < N) btmu += cmS[((ey / sb) * s + ex / sb) * N + lab];
      }
      double pb = 0.0;
      if (X >= k0 && Y >= k0 && X <= k0 + H && Y <= k0 + H) pb = skp[(Y - k0) * Hp + (X - k0)];
      if constexpr (KLDS)
        acc[i] += pb - kpw - btmu;
      else
        dst[nd] += pb - kpw - btmu;
    }
  }
  if constexpr (KLDS) {
#pragma unroll
    for (int i = 0; i < NODES; ++i) {
      const int nd = tid + i * IBT;
      if (nd < nn) dst[nd] = accumulate ? dst[nd] + acc[i] : acc[i];
    }
  }
}

using IbarFn = void (*)(CellArgs, LevelTab, const int32_t*, const int32_t*, const int32_t*, const double*, double*,
                       int, int);
// The parent-seed kernel for cells nc elements wide and its LDS bytes (nullptr
// beyond 128 elements).
static IbarFn ibar_kernel(int nc, int m, size_t* lds) {
  const size_t nn = (size_t)(nc + 1) * (nc + 1), e = (size_t)nc * nc;
  if (nc <= 64) {
    *lds = (nn + e + m) * sizeof(double) + e;
    return k_ibar2d<IB_NODES, true>;
  }
  if (nc <= 128) {
    *lds = (nn + m) * sizeof(double) + e;
    return k_ibar2d<IB_NODES_BIG, false>;
  }
  return nullptr;
}

// dst[i] += b_1[i] + ... in the order given (the per-level parent seeds)
struct SeedBufs {
  const double* b[MAX_LEVELS];
  int n;
};
__global__ void k_sum_seeds(size_t count, double* dst, SeedBufs sb) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
    double v = dst[i];
    for (int k = 0; k < sb.n; ++k) v += sb.b[k][i];
    dst[i] = v;
  }
}

MCH_DEV int floordiv(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// glogk[e] = kappa_e * (explicit K_p term + sum of the cell windows covering e).
__global__ void k_gather_grad2d(CellArgs a, const double* gk, const double* gcell, double* glogk) {
  const int n = a.n, H = a.H, nc = a.nc, nm = a.n_macro;
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i1 = (int)(e % n), i2 = (int)(e / n);
    const int t1 = i1 + nc / 2 - H / 2, t2 = i2 + nc / 2 - H / 2;
    double acc = gk[e];
    for (int j2 = floordiv(t2 - nc, H) + 1; j2 <= floordiv(t2, H); ++j2) {
      const int a2 = t2 - H * j2;
      const int jj2 = wrapi(j2, nm);
      for (int j1 = floordiv(t1 - nc, H) + 1; j1 <= floordiv(t1, H); ++j1) {
        const int a1 = t1 - H * j1;
        const int q = wrapi(j1, nm) + nm * jj2;
        acc += gcell[(size_t)q * nc * nc + (size_t)a2 * nc + a1];
      }
    }
    glogk[e] = a.kappa[e] * acc;
  }
}

template <typename F>
static int set_lds(F fn, size_t lds) {
  if (lds > 160 * 1024) return set_error(MCH_EINVAL, "kernel exceeds the LDS budget");
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute");
  }
  return MCH_OK;
}

// Backward DAG: seeds of every level in parallel; each inheriting level's
// adjoint solve, its pass of the level-1 parent seeds and its gradient window
// on its side stream (the passes chained deepest level first); on s, after
// the last pass, the level-1 adjoint and gradient, then the gather after the
// full join. (A parent-seed pass is latency-bound per workgroup, so it is not
// split into chunks of level-1 cells.)
// interp = 1: levels from L down to 1 as a chain on s. Per level the
// adjoint solve (its right-hand side includes the seeds the level's cells
// received from the levels above, for n < L), then for n >= 2 Ibar of each
// cell and c_t Ibar into its neighbours' seeds. The explicit seeds of levels
// >= 2 run on their level streams from the start, and each level's gradient
// window there once its adjoint solve is done; the gather after the join.
static int launch_backward_2d_chain(mch_plan* pl, const double* kappa, const double* gA, double* glogk,
                                    hipStream_t s) {
  const int M = pl->M, nc = pl->cfg.n_cell, nn1 = nc + 1;
  char name[32];
  void (*seed)(CellArgs, const double*, double*, double*) = nullptr;
  switch (M) {
    case 3: seed = k_seed2d<3>; break;
    case 6: seed = k_seed2d<6>; break;
    case 9: seed = k_seed2d<9>; break;
    default: return set_error(MCH_ENOTIMPL, "M");
  }
  size_t lds_ibar = 0;
  const IbarFn ibar = ibar_kernel(nc, pl->m, &lds_ibar);
  if (!ibar) return set_error(MCH_ENOTIMPL, "2D cells wider than 128 elements");
  int rc = set_lds(ibar, lds_ibar);
  if (!rc) rc = ensure_streams(pl);
  if (!rc) rc = launch_zero(pl->d_seedT, (size_t)pl->nT * M * pl->nn, s);
  if (!rc) rc = fork_levels(pl, s);
  const CellArgs a1 = base_args(pl, kappa, pl->fwd_label, 0);
  LevelTab lt{};
  for (int l = 0; l < pl->L; ++l) {
    lt.r[l] = pl->lev[l].r;
    lt.NC[l] = pl->lev[l].NC;
    lt.w[l] = pl->lev[l].d_w;
  }
  for (int l = 0; l < pl->L && !rc; ++l) {
    if (pl->lev[l].count == 0) continue;
    hipStream_t t = level_stream(pl, l, s);
    CellArgs a = base_args(pl, kappa, pl->fwd_label, l);
    const size_t lds = ((size_t)M * (a.H + 1) * (a.H + 1) + (size_t)M * M) * sizeof(double);
    if ((rc = set_lds(seed, lds))) break;
    std::snprintf(name, sizeof(name), "seed_L%d", l + 1);
    {
      ProfScope ps(pl, name, t);
      hipLaunchKernelGGL(seed, dim3(a.count), dim3(BT), lds, t, a, gA, pl->d_seed_kp, pl->d_gk);
    }
    if ((rc = hip_check(hipGetLastError(), "launch k_seed2d"))) break;
    if (l > 0 && !pl->serial) rc = hip_check(hipEventRecord(pl->ev_setup[l], t), "hipEventRecord");
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
      rc = launch_solve(b, lv.shape.rpt, s);
    }
    if (!rc && l > 0) {
      // Ibar per cell: the parent-seed kernel over the identity map (each
      // cell its own single "child") into d_ibar, row = cell index
      {
        ProfScope ps(pl, "ibar", s);
        hipLaunchKernelGGL(ibar, dim3(lv.count * M), dim3(IBT), lds_ibar, s, a1, lt, pl->d_level, pl->d_iptr,
                           lv.d_cells, pl->d_mu, pl->d_ibar, l, 0);
        rc = hip_check(hipGetLastError(), "launch k_ibar2d");
      }
      if (!rc) rc = launch_distribute(pl, l, s);
    }
    // the gradient window needs only this level's adjoint solution
    hipStream_t t = level_stream(pl, l, s);
    if (!rc && t != s) {
      rc = hip_check(hipEventRecord(pl->ev_adj[l], s), "hipEventRecord");
      if (!rc) rc = hip_check(hipStreamWaitEvent(t, pl->ev_adj[l], 0), "hipStreamWaitEvent");
    }
    if (!rc) {
      std::snprintf(name, sizeof(name), "grad_L%d", l + 1);
      ProfScope ps(pl, name, t);
      hipLaunchKernelGGL(k_grad2d, dim3(a.count), dim3(BT), 0, t, a, lv.d_w, pl->d_gcell);
      rc = hip_check(hipGetLastError(), "launch k_grad2d");
    }
  }
  if (!rc) rc = join_levels(pl, s);
  if (rc) return rc;
  const size_t total = (size_t)pl->n * pl->n;
  const unsigned blocks = (unsigned)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
  {
    ProfScope ps(pl, "gather", s);
    hipLaunchKernelGGL(k_gather_grad2d, dim3(blocks), dim3(256), 0, s, a1, pl->d_gk, pl->d_gcell, glogk);
  }
  return hip_check(hipGetLastError(), "launch k_gather_grad2d");
}

int launch_backward_2d(mch_plan* pl, const double* kappa, const double* gA, double* glogk, hipStream_t s) {
  if (pl->nT > 0) return launch_backward_2d_chain(pl, kappa, gA, glogk, s);
  const int M = pl->M, nc = pl->cfg.n_cell, nn1 = nc + 1;
  char name[32];
  int rc = ensure_streams(pl);
  if (!rc) rc = fork_levels(pl, s);
  if (rc) return rc;
  void (*seed)(CellArgs, const double*, double*, double*) = nullptr;
  switch (M) {
    case 3: seed = k_seed2d<3>; break;
    case 6: seed = k_seed2d<6>; break;
    case 9: seed = k_seed2d<9>; break;
    default: return set_error(MCH_ENOTIMPL, "M");
  }
  auto launch_grad = [&](const CellArgs& g, hipStream_t t, int l) -> int {
    if (g.count == 0) return MCH_OK;
    std::snprintf(name, sizeof(name), "grad_L%d", l + 1);
    ProfScope ps(pl, name, t);
    hipLaunchKernelGGL(k_grad2d, dim3(g.count), dim3(BT), 0, t, g, pl->lev[l].d_w, pl->d_gcell);
    return hip_check(hipGetLastError(), "launch k_grad2d");
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
  const int n1 = pl->lev[0].count;
  const bool inherit = pl->L > 1 && n1 > 0 && n1 < pl->P;
  CellArgs a1 = base_args(pl, kappa, pl->fwd_label, 0);
  LevelTab lt{};
  for (int l = 0; l < pl->L; ++l) {
    lt.r[l] = pl->lev[l].r;
    lt.NC[l] = pl->lev[l].NC;
    lt.w[l] = pl->lev[l].d_w;
  }
  size_t lds_ibar = 0;
  const IbarFn ibar = ibar_kernel(nc, pl->m, &lds_ibar);
  if (!ibar) return set_error(MCH_ENOTIMPL, "2D cells wider than 128 elements");
  if (inherit && (rc = set_lds(ibar, lds_ibar))) return rc;
  // Parent seeds from the cells of one inheriting level, on that level's
  // stream once its adjoint solve is done, into a buffer of its own (the
  // deepest level's straight into d_seed_par), so the passes run in parallel;
  // the others are then added deepest level first, a fixed order.
  int deepest = -1;
  SeedBufs extra{};
  auto ibar_pass = [&](int l, hipStream_t t) -> int {
    if (deepest < 0) deepest = l;
    double* dst = (l == deepest) ? pl->d_seed_par : pl->d_seed_lvl[l];
    if (l != deepest) extra.b[extra.n++] = dst;
    int r = MCH_OK;
    {
      ProfScope ps(pl, "ibar", t);
      hipLaunchKernelGGL(ibar, dim3(n1 * M), dim3(IBT), lds_ibar, t, a1, lt, pl->d_level, pl->d_child_ptr,
                         pl->d_child, pl->d_mu, dst, l, 0);
      r = hip_check(hipGetLastError(), "launch k_ibar2d");
    }
    if (!r) r = mark_level(pl, l, pl->ev_ibar);
    return r;
  };
  for (int l = pl->L - 1; l >= 0; --l) {
    if (pl->lev[l].count == 0) continue;
    hipStream_t t = level_stream(pl, l, s);
    CellArgs a = base_args(pl, kappa, pl->fwd_label, l);
    const size_t lds = ((size_t)M * (a.H + 1) * (a.H + 1) + (size_t)M * M) * sizeof(double);
    rc = set_lds(seed, lds);
    if (rc) return rc;
    std::snprintf(name, sizeof(name), "seed_L%d", l + 1);
    {
      ProfScope ps(pl, name, t);
      hipLaunchKernelGGL(seed, dim3(a.count), dim3(BT), lds, t, a, gA, pl->d_seed_kp, pl->d_gk);
    }
    if ((rc = hip_check(hipGetLastError(), "launch k_seed2d"))) return rc;
    if (l == 0) continue;
    std::snprintf(name, sizeof(name), "adjsolve_L%d", l + 1);
    {
      ProfScope ps(pl, name, t);
      rc = launch_solve(adjoint_args(l), pl->lev[l].shape.rpt, t);
    }
    // the parent seeds and the level-1 adjoint need this level's adjoint
    // solution, not its gradient window, which runs on alongside them
    if (!rc && inherit) rc = ibar_pass(l, t);
    if (!rc) rc = launch_grad(base_args(pl, kappa, pl->fwd_label, l), t, l);
    if (rc) return rc;
  }
  // the level-1 adjoint waits for every level's parent-seed pass (each after
  // its level's adjoint solve), then the passes' sum
  if (inherit && deepest >= 0) {
    if (!pl->serial) rc = wait_marks(pl, s, pl->ev_ibar);
    if (!rc && extra.n > 0) {
      const size_t count = (size_t)n1 * M * nn1 * nn1;
      ProfScope ps(pl, "ibar_sum", s);
      hipLaunchKernelGGL(k_sum_seeds, dim3((unsigned)std::min<size_t>((count + 255) / 256, 4096)), dim3(256), 0, s,
                         count, pl->d_seed_par, extra);
      rc = hip_check(hipGetLastError(), "launch k_sum_seeds");
    }
  }
  if (!rc && n1 > 0) {
    CellArgs a = adjoint_args(0);
    a.seed_par = inherit ? pl->d_seed_par : nullptr;
    ProfScope ps(pl, "adjsolve_L1", s);
    rc = launch_solve(a, pl->lev[0].shape.rpt, s);
  }
  if (!rc && n1 > 0) rc = launch_grad(a1, s, 0);
  if (!rc) rc = join_levels(pl, s);  // the gradient windows of levels >= 2
  if (rc) return rc;
  const size_t total = (size_t)pl->n * pl->n;
  const unsigned blocks = (unsigned)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
  {
    ProfScope ps(pl, "gather", s);
    hipLaunchKernelGGL(k_gather_grad2d, dim3(blocks), dim3(256), 0, s, a1, pl->d_gk, pl->d_gcell, glogk);
  }
  return hip_check(hipGetLastError(), "launch k_gather_grad2d");
}

}  // namespace mch
