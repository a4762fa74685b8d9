// The upscaled multicontinuum system on the macrogrid, 2D (Sec. 2, Eq.
// macro_eq with the coefficients of Eq. Bs_defi; the last step of Algorithm 1).
//
// Weak form over the coarse blocks K_p: sum_p int_{K_p} w_V^T (A_eff(p)/|K_p|)
// w_U = sum_p int_{K_p} (b(p)/|K_p|) . V, with w = (U_0 .. U_{N-1},
// d_1 U_0, d_2 U_0, d_1 U_1, ...) in the right-hand-side order of the cell
// problems, so the blocks of A_eff are B_ji, B^m_ji, Bbar^n_ji and B^mn_ji.
// U is continuous and bilinear on the blocks with nodes at the block corners
// of [0, 1]^2 and U = 0 on its boundary; the block densities are integrated
// exactly against the Q1 functions; b_j(p) = int_{K_p} f phi_j. The operator
// is symmetric positive semi-definite (a sum of Gram forms) and is solved by
// Jacobi-preconditioned CG.
//
// Unknowns: interior node (k1, k2), 1 <= k <= n_macro - 1, continuum j at
// ((k2 - 1)(n_macro - 1) + k1 - 1) N + j. Element matrices E_p[(a, j), (b, i)]
// (index a N + j, corners a in tensor order) are formed once per solve; the
// CG applies the operator by gathering, per node, the rows of its four blocks.
// The CG runs in one workgroup: the macro systems of the workloads here have
// a few thousand unknowns, and one workgroup needs no device-wide
// synchronisation (at 2048^2 it is bound by one CU's bandwidth).
#include "kernels2d.h"

namespace mch {

constexpr int MT = 256;    // load and element kernels
constexpr int CGT = 1024;  // the CG workgroup
constexpr int CGW = CGT / 64;

// b[p][j] = int_{K_p} f phi_j, j < N: per fine element of K_p, |e| f_e times
// the mean of phi_j at its four corners (exact for bilinear phi_j).
__global__ __launch_bounds__(MT) void k_macro_load2d(CellArgs a, const double* f, double* b) {
  __shared__ double red[3][MT / 64];
  const int ci = a.ci0 + blockIdx.x;
  const int p = a.cells[ci];
  const int H = a.H, N = a.N, k0 = (a.nc - H) / 2;
  const int jx = p % a.n_macro, jy = p / a.n_macro;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int e = tid; e < H * H; e += MT) {
    const int ex = e % H, ey = e / H;
    const double fe = f[(size_t)(H * jy + ey) * a.n + (H * jx + ex)] * a.h * a.h;
    for (int j = 0; j < N; ++j) {
      const double m = 0.25 * ((phi_at(a, ci, j, k0 + ex, k0 + ey) + phi_at(a, ci, j, k0 + ex + 1, k0 + ey)) +
                               (phi_at(a, ci, j, k0 + ex, k0 + ey + 1) + phi_at(a, ci, j, k0 + ex + 1, k0 + ey + 1)));
      acc[j] += fe * m;
    }
  }
  for (int j = 0; j < N; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) red[j][wave] = v;
  }
  __syncthreads();
  if (tid < N) b[(size_t)p * N + tid] = tree_sum<MT / 64, 1>(red[tid]);
}

// One-dimensional Q1 integrals on [0, Hc]: value or derivative of the test
// function (corner x) against value or derivative of the trial function
// (corner y).
MCH_DEV double q1_1d(bool dtest, bool dtrial, int x, int y, double Hc) {
  if (!dtest && !dtrial) return Hc * (x == y ? 1.0 / 3.0 : 1.0 / 6.0);
  if (!dtest && dtrial) return y == 1 ? 0.5 : -0.5;
  if (dtest && !dtrial) return x == 1 ? 0.5 : -0.5;
  return (x == y ? 1.0 : -1.0) / Hc;
}

// E_p[(a, j), (b, i)] = (1/|K|) sum over the value / derivative components
// (s of the test, t of the trial) of A_p[alpha(j, s)][alpha(i, t)] times the
// Q1 integral of the two components; alpha(j, 0) = j, alpha(j, 1 + m) = N + 2 j + m.
__global__ __launch_bounds__(MT) void k_macro_elem2d(const double* A, int N, double Hc, double* E) {
  const int p = blockIdx.x, M = 3 * N, K4 = 4 * N;
  const double* Ap = A + (size_t)p * M * M;
  double* Ep = E + (size_t)p * K4 * K4;
  for (int k = threadIdx.x; k < K4 * K4; k += MT) {
    const int row = k / K4, col = k % K4;
    const int a = row / N, j = row % N, b = col / N, i = col % N;
    double s = 0.0;
    for (int sa = 0; sa < 3; ++sa) {
      const int al = sa == 0 ? j : N + 2 * j + sa - 1;
      for (int tb = 0; tb < 3; ++tb) {
        const int be = tb == 0 ? i : N + 2 * i + tb - 1;
        const double t = q1_1d(sa == 1, tb == 1, a & 1, b & 1, Hc) * q1_1d(sa == 2, tb == 2, a >> 1, b >> 1, Hc);
        s += Ap[(size_t)al * M + be] * t;
      }
    }
    Ep[k] = s / (Hc * Hc);
  }
}

// Sum over the workgroup in a fixed order; every thread gets the result.
MCH_DEV double cg_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  const double t = tree_sum<CGW, 1>(red);
  __syncthreads();  // red is reused by the next sum
  return t;
}

struct MacroArgs {
  int nm, N;
  const double* E;  // [P][4N][4N]
  const double* b;  // [P][N]
  double *x, *r, *z, *p, *q, *dinv;
  double rtol;
  int max_iter;
  double* U;   // [(nm+1)^2][N]
  double* Ub;  // [P][N]
  int32_t* iters;
  double* resid;
};

// Diagonal entry of unknown (interior node k1, k2; continuum j).
MCH_DEV double macro_diag(const MacroArgs& m, int k1, int k2, int j) {
  const int nm = m.nm, N = m.N, K4 = 4 * N;
  double d = 0.0;
  for (int a = 0; a < 4; ++a) {
    const int B1 = k1 - (a & 1), B2 = k2 - (a >> 1);  // the block whose corner a this node is
    d += m.E[((size_t)(B2 * nm + B1) * K4 + a * N + j) * K4 + a * N + j];
  }
  return d;
}

// The row of that unknown applied to v.
MCH_DEV double macro_row(const MacroArgs& m, int k1, int k2, int j, const double* v) {
  const int nm = m.nm, N = m.N, K4 = 4 * N, ni = nm - 1;
  double y = 0.0;
  for (int a = 0; a < 4; ++a) {
    const int B1 = k1 - (a & 1), B2 = k2 - (a >> 1);  // the block whose corner a this node is
    const double* Er = m.E + ((size_t)(B2 * nm + B1) * K4 + a * N + j) * K4;
    for (int bb = 0; bb < 4; ++bb) {
      const int n1 = B1 + (bb & 1), n2 = B2 + (bb >> 1);
      if (n1 < 1 || n2 < 1 || n1 > ni || n2 > ni) continue;  // boundary node: U = 0
      const double* vv = v + ((size_t)(n2 - 1) * ni + (n1 - 1)) * N;
      for (int i = 0; i < N; ++i) y += Er[bb * N + i] * vv[i];
    }
  }
  return y;
}

// Jacobi-preconditioned CG in one workgroup; every thread reads the same
// reduced scalars, so all leave the loop in the same iteration.
__global__ __launch_bounds__(CGT) void k_macro_cg2d(MacroArgs m) {
  __shared__ double red[CGW];
  const int nm = m.nm, N = m.N, ni = nm - 1, n = ni * ni * N;
  const int tid = threadIdx.x;
  auto node = [&](int u, int& k1, int& k2, int& j) {
    j = u % N;
    const int nd = u / N;
    k1 = 1 + nd % ni;
    k2 = 1 + nd / ni;
  };
  // x = 0, r = F, z = D^-1 r, p = z
  double rz = 0.0;
  for (int u = tid; u < n; u += CGT) {
    int k1, k2, j;
    node(u, k1, k2, j);
    double F = 0.0;
    for (int a = 0; a < 4; ++a) F += 0.25 * m.b[(size_t)((k2 - (a >> 1)) * nm + (k1 - (a & 1))) * N + j];
    const double di = 1.0 / macro_diag(m, k1, k2, j);
    m.dinv[u] = di;
    m.x[u] = 0.0;
    m.r[u] = F;
    const double zu = F * di;
    m.z[u] = zu;
    m.p[u] = zu;
    rz += F * zu;
  }
  rz = cg_sum(rz, red);  // the barrier also publishes p
  const double rz0 = rz;
  int it = 0;
  bool done = !(rz0 > 0.0);
  while (!done) {
    double pq = 0.0;
    for (int u = tid; u < n; u += CGT) {
      int k1, k2, j;
      node(u, k1, k2, j);
      const double qu = macro_row(m, k1, k2, j, m.p);
      m.q[u] = qu;
      pq += m.p[u] * qu;
    }
    pq = cg_sum(pq, red);
    const double al = rz / pq;
    double rzn = 0.0;
    for (int u = tid; u < n; u += CGT) {
      m.x[u] += al * m.p[u];
      const double ru = m.r[u] - al * m.q[u];
      m.r[u] = ru;
      const double zu = ru * m.dinv[u];
      m.z[u] = zu;
      rzn += ru * zu;
    }
    rzn = cg_sum(rzn, red);
    ++it;
    if (rzn <= m.rtol * m.rtol * rz0 || it >= m.max_iter) {
      rz = rzn;
      break;
    }
    const double be = rzn / rz;
    rz = rzn;
    for (int u = tid; u < n; u += CGT) m.p[u] = m.z[u] + be * m.p[u];
    __syncthreads();  // p complete before the next product
  }
  // nodal values (zero on the boundary) and block averages
  const int nn = nm + 1;
  for (int u = tid; u < nn * nn * N; u += CGT) {
    const int j = u % N, nd = u / N, k1 = nd % nn, k2 = nd / nn;
    const bool in = k1 >= 1 && k2 >= 1 && k1 <= ni && k2 <= ni;
    m.U[u] = in ? m.x[((size_t)(k2 - 1) * ni + (k1 - 1)) * N + j] : 0.0;
  }
  __syncthreads();
  for (int u = tid; u < nm * nm * N; u += CGT) {
    const int j = u % N, pb = u / N, B1 = pb % nm, B2 = pb / nm;
    const double s = (m.U[((size_t)B2 * nn + B1) * N + j] + m.U[((size_t)B2 * nn + B1 + 1) * N + j]) +
                     (m.U[((size_t)(B2 + 1) * nn + B1) * N + j] + m.U[((size_t)(B2 + 1) * nn + B1 + 1) * N + j]);
    m.Ub[u] = 0.25 * s;
  }
  if (tid == 0) {
    *m.iters = it;
    *m.resid = rz0 > 0.0 ? sqrt(fmax(rz, 0.0) / rz0) : 0.0;
  }
}

int launch_macro_load_2d(mch_plan* pl, const double* f, double* b, hipStream_t s) {
  for (int l = 0; l < pl->L; ++l) {
    if (pl->lev[l].count == 0) continue;
    CellArgs a = base_args(pl, pl->fwd_kappa, pl->fwd_label, l);
    ProfScope ps(pl, "macro_load", s);
    hipLaunchKernelGGL(k_macro_load2d, dim3(a.count), dim3(MT), 0, s, a, f, b);
    int rc = hip_check(hipGetLastError(), "launch k_macro_load2d");
    if (rc) return rc;
  }
  return MCH_OK;
}

int launch_macro_solve_2d(mch_plan* pl, const double* A, const double* b, double* U, double* Ub, double rtol,
                          int max_iter, hipStream_t s) {
  const int N = pl->cfg.n_cont, nm = pl->nm;
  if (nm < 2) return set_error(MCH_EINVAL, "the macroscopic system needs at least 2 blocks per axis");
  int rc = ensure_macro_scratch(pl);
  if (rc) return rc;
  {
    ProfScope ps(pl, "macro_elem", s);
    hipLaunchKernelGGL(k_macro_elem2d, dim3(pl->P), dim3(MT), 0, s, A, N, 1.0 / nm, pl->d_macroE);
    rc = hip_check(hipGetLastError(), "launch k_macro_elem2d");
  }
  if (rc) return rc;
  const size_t nint = (size_t)(nm - 1) * (nm - 1) * N;
  MacroArgs m{};
  m.nm = nm;
  m.N = N;
  m.E = pl->d_macroE;
  m.b = b;
  m.x = pl->d_mvec;
  m.r = m.x + nint;
  m.z = m.r + nint;
  m.p = m.z + nint;
  m.q = m.p + nint;
  m.dinv = m.q + nint;
  m.rtol = rtol;
  m.max_iter = max_iter;
  m.U = U;
  m.Ub = Ub;
  m.iters = pl->d_macro_iters;
  m.resid = pl->d_macro_resid;
  ProfScope ps(pl, "macro_cg", s);
  hipLaunchKernelGGL(k_macro_cg2d, dim3(1), dim3(CGT), 0, s, m);
  return hip_check(hipGetLastError(), "launch k_macro_cg2d");
}

}  // namespace mch
