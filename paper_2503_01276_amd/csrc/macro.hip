// The upscaled multicontinuum system on the macrogrid (Sec. 2, Eq. macro_eq
// with the coefficients of Eq. Bs_defi; the last step of Algorithm 1), 2D and 3D.
//
// Weak form over the coarse blocks K_p: sum_p int_{K_p} w_V^T (A_eff(p)/|K_p|)
// w_U = sum_p int_{K_p} (b(p)/|K_p|) . V, with w = (U_0 .. U_{N-1},
// d_1 U_0 .. d_d U_0, d_1 U_1, ...) in the right-hand-side order of the cell
// problems, so the blocks of A_eff are B_ji, B^m_ji, Bbar^n_ji and B^mn_ji.
// U is continuous and multilinear on the blocks with nodes at the block
// corners of [0, 1]^d and U = 0 on its boundary; the block densities are
// integrated exactly against the Q1 functions; b_j(p) = int_{K_p} f phi_j.
// The operator is symmetric positive semi-definite (a sum of Gram forms) and
// is solved by CG preconditioned with the inverses of the nodal N x N blocks
// (the continua at one node are strongly coupled through the exchange terms
// B_ji; point Jacobi ignores that coupling and needs over ten times the
// iterations on hierarchical tensors).
//
// Unknowns: interior node k (1 <= k_a <= n_macro - 1 per axis, axis 1
// fastest), continuum j at (node index) N + j. Element matrices
// E_p[(a, j), (b, i)] (index a N + j, corners a in tensor order) are formed
// once per solve and summed into nodal block rows over the 3^d neighbours of
// each node, which the CG applies. Systems whose vectors fit in LDS (a few
// thousand unknowns, as on the 512^2 and 128^3 grids) are solved by one
// workgroup, which needs no device-wide synchronisation; larger ones by one
// cooperative launch over the device with grid barriers.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <string>

#include "kernels2d.h"

namespace mch {

constexpr int MT = 256;    // load and element kernels
constexpr int CGT = 1024;  // the CG workgroup
constexpr int CGW = CGT / 64;
// LDS for the vectors of the LDS-resident CG (152 KiB of the workgroup's
// 160 KiB; the reduction buffers take 256 bytes).
constexpr size_t kMacroLdsDoubles = 19 * 1024;
// The grid-wide CG: threads per workgroup, and its default number of
// workgroups (its grid barriers cost in proportion to the workgroups, its
// stencil stream wants many threads in flight; measured best near 64 x 1024).
constexpr int GGT = 1024;
constexpr int GGW = GGT / 64;
constexpr int kMacroGridDefault = 64;

// 2D: b[p][j] = int_{K_p} f phi_j, j < N: per fine element of K_p, |e| f_e
// times the mean of phi_j at its four corners (exact for bilinear phi_j).
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

// 3D: the same from Phi on the K_p nodes, phikp [P][M][(H+1)^3] (X fastest),
// which the 3D forward stores for every point.
__global__ __launch_bounds__(MT) void k_macro_load3d(const double* phikp, const double* f, int n, int nm, int H,
                                                     int M, int N, double h, double* b) {
  __shared__ double red[3][MT / 64];
  const int p = blockIdx.x;
  const int jx = p % nm, jy = (p / nm) % nm, jz = p / (nm * nm), Hp = H + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int e = tid; e < H * H * H; e += MT) {
    const int ex = e % H, ey = (e / H) % H, ez = e / (H * H);
    const double fe = f[((size_t)(H * jz + ez) * n + (H * jy + ey)) * n + (H * jx + ex)] * h * h * h;
    for (int j = 0; j < N; ++j) {
      const double* ph = phikp + ((size_t)p * M + j) * (size_t)Hp * Hp * Hp;
      double s = 0.0;
      for (int c = 0; c < 8; ++c)
        s += ph[(ex + (c & 1)) + Hp * ((ey + ((c >> 1) & 1)) + Hp * (ez + (c >> 2)))];
      acc[j] += fe * (0.125 * s);
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
// Q1 integral of the two components, a product over the axes;
// alpha(j, 0) = j, alpha(j, 1 + m) = N + D j + m.
template <int D>
__global__ __launch_bounds__(MT) void k_macro_elem(const double* A, int N, double Hc, double* E) {
  constexpr int K = 1 << D;
  const int p = blockIdx.x, M = (1 + D) * N, KN = K * N;
  const double* Ap = A + (size_t)p * M * M;
  double* Ep = E + (size_t)p * KN * KN;
  double vol = 1.0;
  for (int ax = 0; ax < D; ++ax) vol *= Hc;
  for (int k = threadIdx.x; k < KN * KN; k += MT) {
    const int row = k / KN, col = k % KN;
    const int a = row / N, j = row % N, bc = col / N, i = col % N;
    double s = 0.0;
    for (int sa = 0; sa <= D; ++sa) {
      const int al = sa == 0 ? j : N + D * j + sa - 1;
      for (int tb = 0; tb <= D; ++tb) {
        const int be = tb == 0 ? i : N + D * i + tb - 1;
        double t = 1.0;
        for (int ax = 0; ax < D; ++ax)
          t *= q1_1d(sa == 1 + ax, tb == 1 + ax, (a >> ax) & 1, (bc >> ax) & 1, Hc);
        s += Ap[(size_t)al * M + be] * t;
      }
    }
    Ep[k] = s / vol;
  }
}

// Sum over the workgroup in a fixed order; every thread gets the result. The
// buffer may be written again only after a later barrier (the CG alternates
// two buffers, and each sum is followed by at least one other barrier before
// its buffer comes round again).
MCH_DEV double cg_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return tree_sum<CGW, 1>(red);
}

struct MacroArgs {
  int nm;
  const double* S;     // nodal stencil rows [3^D N][n]
  const double* Dinv;  // inverse diagonal blocks [N N][n / N]
  const double* b;     // [P][N]
  double *x, *r, *z, *p, *q;
  double* sv;  // s = A p of the grid-wide CG
  double rtol;
  int max_iter;
  double* U;   // [(nm+1)^D][N]
  double* Ub;  // [P][N]
  int32_t* iters;
  double* resid;
};

// Interior node index of multi-index k (1-based per axis), -1 on the boundary.
template <int D>
MCH_DEV int interior_index(const int (&k)[3], int ni) {
  int idx = 0, str = 1;
  for (int ax = 0; ax < D; ++ax) {
    if (k[ax] < 1 || k[ax] > ni) return -1;
    idx += (k[ax] - 1) * str;
    str *= ni;
  }
  return idx;
}

// Multi-index of interior node nd.
template <int D>
MCH_DEV void node_index(int nd, int ni, int (&k)[3]) {
  k[2] = 1;
  for (int ax = 0; ax < D; ++ax) {
    k[ax] = 1 + nd % ni;
    nd /= ni;
  }
}

// Neighbour s of node k, 0 <= s < 3^D: offset (s mod 3) - 1 on axis 1, and so
// on, axis 1 fastest; s = (3^D - 1) / 2 is the node itself.
template <int D>
MCH_DEV void neighbour(const int (&k)[3], int s, int (&nb)[3]) {
  nb[2] = 1;
  for (int ax = 0; ax < D; ++ax) {
    nb[ax] = k[ax] + s % 3 - 1;
    s /= 3;
  }
}

// Block index of the block whose corner a node k is, and the block's corner
// multi-index.
template <int D>
MCH_DEV int block_of(const int (&k)[3], int a, int nm, int (&B)[3]) {
  int idx = 0, str = 1;
  for (int ax = 0; ax < D; ++ax) {
    B[ax] = k[ax] - ((a >> ax) & 1);
    idx += B[ax] * str;
    str *= nm;
  }
  return idx;
}

// Assembled operator as nodal block rows: S[(s N + i) n + u] couples row
// u = (node, j) to unknown (neighbour s of the node, i); it is the sum, over
// the blocks that hold both nodes, of their element entries, and zero where
// the neighbour lies on the boundary (U = 0 there). One thread per row;
// consecutive rows are consecutive addresses for every (s, i).
template <int D>
__global__ __launch_bounds__(MT) void k_macro_stencil(const double* E, int nm, int N, int n, double* S) {
  constexpr int K = 1 << D, NS = D == 2 ? 9 : 27;
  const int u = blockIdx.x * MT + threadIdx.x;
  if (u >= n) return;
  const int KN = K * N, ni = nm - 1, j = u % N;
  int k[3];
  node_index<D>(u / N, ni, k);
  for (int s = 0; s < NS; ++s) {
    int nb[3];
    neighbour<D>(k, s, nb);
    const bool inside = interior_index<D>(nb, ni) >= 0;
    for (int i = 0; i < N; ++i) {
      double v = 0.0;
      for (int a = 0; inside && a < K; ++a) {
        int B[3];
        const int pb = block_of<D>(k, a, nm, B);
        int c = 0;
        bool shared = true;
        for (int ax = 0; ax < D; ++ax) {
          const int o = nb[ax] - B[ax];
          shared = shared && (o == 0 || o == 1);
          c |= (o & 1) << ax;
        }
        if (shared) v += E[((size_t)pb * KN + a * N + j) * KN + c * N + i];
      }
      S[(size_t)(s * N + i) * n + u] = v;
    }
  }
}

// Inverse of every node's N x N diagonal block (the continua at one node),
// Dinv[(j N + i) nn + nd]. The block is symmetric positive definite, so
// Gauss-Jordan elimination without pivoting is stable.
template <int NB>
__global__ __launch_bounds__(MT) void k_macro_blockinv(const double* S, int n, int centre, double* Dinv) {
  const int nn = n / NB, nd = blockIdx.x * MT + threadIdx.x;
  if (nd >= nn) return;
  double a[NB][NB], x[NB][NB];
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      a[j][i] = S[(size_t)(centre * NB + i) * n + nd * NB + j];
      x[j][i] = i == j ? 1.0 : 0.0;
    }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const double piv = 1.0 / a[c][c];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      a[c][i] *= piv;
      x[c][i] *= piv;
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      if (r == c) continue;
      const double f = a[r][c];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        a[r][i] -= f * a[c][i];
        x[r][i] -= f * x[c][i];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int i = 0; i < NB; ++i) Dinv[(size_t)(j * NB + i) * nn + nd] = x[j][i];
}

// z = Dinv r on node nd (r given for its NB rows); returns r . z there.
template <int NB>
MCH_DEV double node_precond(const double* Dinv, int nn, int nd, const double (&r)[NB], double* z) {
  double rz = 0.0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double zj = 0.0;
#pragma unroll
    for (int i = 0; i < NB; ++i) zj += Dinv[(size_t)(j * NB + i) * nn + nd] * r[i];
    z[(size_t)nd * NB + j] = zj;
    rz += r[j] * zj;
  }
  return rz;
}

// CG preconditioned by the nodal block inverses, in one workgroup; every
// thread reads the same reduced scalars, so all leave the loop in the same
// iteration. The product runs one thread per row, the updates and the
// preconditioner one thread per node. The vectors x, r, z, p, q and the block
// inverses live in LDS (systems of up to kMacroLdsDoubles / (5 + N)
// unknowns), so that only the stencil rows stream from the caches.
template <int D, int NB>
__global__ __launch_bounds__(CGT) void k_macro_cg(MacroArgs m) {
  constexpr int K = 1 << D, NS = D == 2 ? 9 : 27;
  __shared__ double red[2][CGW];  // alternating reduction buffers
  extern __shared__ double lds_vec[];
  const int nm = m.nm, ni = nm - 1;
  int nn = 1;
  for (int ax = 0; ax < D; ++ax) nn *= ni;
  const int n = nn * NB;
  const int tid = threadIdx.x;
  double* vx = lds_vec;
  double* vr = vx + n;
  double* vz = vr + n;
  double* vp = vz + n;
  double* vq = vp + n;
  double* dinv = vq + n;
  for (int k = tid; k < NB * n; k += CGT) dinv[k] = m.Dinv[k];
  __syncthreads();
  // x = 0, r = F, z = M^-1 r, p = z
  double rz = 0.0;
  for (int nd = tid; nd < nn; nd += CGT) {
    int k[3];
    node_index<D>(nd, ni, k);
    double F[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      F[j] = 0.0;
      for (int a = 0; a < K; ++a) {
        int B[3];
        F[j] += m.b[(size_t)block_of<D>(k, a, nm, B) * NB + j] / K;
      }
      vx[(size_t)nd * NB + j] = 0.0;
      vr[(size_t)nd * NB + j] = F[j];
    }
    rz += node_precond<NB>(dinv, nn, nd, F, vz);
#pragma unroll
    for (int j = 0; j < NB; ++j) vp[(size_t)nd * NB + j] = vz[(size_t)nd * NB + j];
  }
  rz = cg_sum(rz, red[0]);  // the barrier also publishes p
  const double rz0 = rz;
  int it = 0;
  bool done = !(rz0 > 0.0);
  while (!done) {
    double pq = 0.0;
    for (int u = tid; u < n; u += CGT) {
      int k[3];
      node_index<D>(u / NB, ni, k);
      double qu = 0.0;
      for (int s = 0; s < NS; ++s) {
        int nb[3];
        neighbour<D>(k, s, nb);
        const int vi = interior_index<D>(nb, ni);
        if (vi < 0) continue;  // boundary node: U = 0
#pragma unroll
        for (int i = 0; i < NB; ++i) qu += m.S[(size_t)(s * NB + i) * n + u] * vp[(size_t)vi * NB + i];
      }
      vq[u] = qu;
      pq += vp[u] * qu;
    }
    pq = cg_sum(pq, red[1]);
    const double al = rz / pq;
    double rzn = 0.0;
    for (int nd = tid; nd < nn; nd += CGT) {
      double rr[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const size_t u = (size_t)nd * NB + j;
        vx[u] += al * vp[u];
        rr[j] = vr[u] - al * vq[u];
        vr[u] = rr[j];
      }
      rzn += node_precond<NB>(dinv, nn, nd, rr, vz);
    }
    rzn = cg_sum(rzn, red[0]);
    ++it;
    if (rzn <= m.rtol * m.rtol * rz0 || it >= m.max_iter) {
      rz = rzn;
      break;
    }
    const double be = rzn / rz;
    rz = rzn;
    for (int u = tid; u < n; u += CGT) vp[u] = vz[u] + be * vp[u];
    __syncthreads();  // p complete before the next product
  }
  // nodal values (zero on the boundary) and block averages
  const int nnp = nm + 1;
  int nnodes = 1, nblocks = 1;
  for (int ax = 0; ax < D; ++ax) {
    nnodes *= nnp;
    nblocks *= nm;
  }
  for (int u = tid; u < nnodes * NB; u += CGT) {
    const int j = u % NB;
    int nd = u / NB, k[3] = {0, 0, 1};
    for (int ax = 0; ax < D; ++ax) {
      k[ax] = nd % nnp;
      nd /= nnp;
    }
    const int vi = interior_index<D>(k, ni);
    m.U[u] = vi >= 0 ? vx[(size_t)vi * NB + j] : 0.0;
  }
  __syncthreads();
  for (int u = tid; u < nblocks * NB; u += CGT) {
    const int j = u % NB;
    int pb = u / NB, B[3] = {0, 0, 0};
    for (int ax = 0; ax < D; ++ax) {
      B[ax] = pb % nm;
      pb /= nm;
    }
    double s = 0.0;
    for (int c = 0; c < K; ++c) {
      size_t idx = 0, str = 1;
      for (int ax = 0; ax < D; ++ax) {
        idx += (size_t)(B[ax] + ((c >> ax) & 1)) * str;
        str *= nnp;
      }
      s += m.U[idx * NB + j];
    }
    m.Ub[u] = s / K;
  }
  if (tid == 0) {
    *m.iters = it;
    *m.resid = rel_resid(rz, rz0);
  }
}

// The CG over the whole grid for systems that do not fit in LDS: one
// cooperative launch, vectors in global memory, rows and nodes strided over
// all threads. A grid barrier costs in proportion to the number of
// workgroups, so the loop is the single-reduction form of preconditioned CG
// of Chronopoulos and Gear (1989), which carries s = A p alongside p and
// reduces r.z and (A z).z together: two grid barriers per iteration (z
// published for the product, the fused sum) against four. In exact
// arithmetic its iterates are those of the loop above. The fused sum stores
// each workgroup's two sums in part[2 block + {0, 1}]; after the barrier every
// wave adds part[] lane-strided and across its lanes in a fixed order, so all
// waves of all workgroups hold bitwise the same scalars and leave the loop in
// the same iteration, after the same number of barriers.
MCH_DEV void grid_sum2(double& a, double& b, double* part, double (*red)[GGW], cooperative_groups::grid_group& grid) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = tree_sum<GGW, 1>(red[0]);
    part[2 * blockIdx.x + 1] = tree_sum<GGW, 1>(red[1]);
  }
  grid.sync();
  double sa = 0.0, sb = 0.0;
  for (int k = lane; k < (int)gridDim.x; k += 64) {
    sa += part[2 * k];
    sb += part[2 * k + 1];
  }
  a = wave_sum(sa);
  b = wave_sum(sb);
}

template <int D, int NB>
__global__ __launch_bounds__(GGT) void k_macro_cg_grid(MacroArgs m, double* part) {
  constexpr int K = 1 << D, NS = D == 2 ? 9 : 27;
  __shared__ double red[2][GGW];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int nm = m.nm, ni = nm - 1;
  int nn = 1;
  for (int ax = 0; ax < D; ++ax) nn *= ni;
  const int n = nn * NB;
  const int g0 = blockIdx.x * GGT + threadIdx.x, gs = gridDim.x * GGT;
  // w = A z on this thread's rows; returns its share of w.z
  auto product = [&]() -> double {
    double wz = 0.0;
    for (int u = g0; u < n; u += gs) {
      int k[3];
      node_index<D>(u / NB, ni, k);
      double wu = 0.0;
      for (int s = 0; s < NS; ++s) {
        int nb[3];
        neighbour<D>(k, s, nb);
        const int vi = interior_index<D>(nb, ni);
        if (vi < 0) continue;  // boundary node: U = 0
#pragma unroll
        for (int i = 0; i < NB; ++i) wu += m.S[(size_t)(s * NB + i) * n + u] * m.z[(size_t)vi * NB + i];
      }
      m.q[u] = wu;
      wz += wu * m.z[u];
    }
    return wz;
  };
  // x = 0, r = F, z = M^-1 r
  double g = 0.0;
  for (int nd = g0; nd < nn; nd += gs) {
    int k[3];
    node_index<D>(nd, ni, k);
    double F[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      F[j] = 0.0;
      for (int a = 0; a < K; ++a) {
        int B[3];
        F[j] += m.b[(size_t)block_of<D>(k, a, nm, B) * NB + j] / K;
      }
      m.x[(size_t)nd * NB + j] = 0.0;
      m.r[(size_t)nd * NB + j] = F[j];
    }
    g += node_precond<NB>(m.Dinv, nn, nd, F, m.z);
  }
  grid.sync();  // z complete before the product
  double dl = product();
  grid_sum2(g, dl, part, red, grid);
  const double g0r = g;
  double gam = g, al = dl != 0.0 ? g / dl : 0.0, be = 0.0;
  int it = 0;
  bool done = !(g0r > 0.0);
  while (!done) {
    // p = z + be p, s = w + be s (w in q), x += al p, r -= al s, z = M^-1 r
    double gn = 0.0;
    for (int nd = g0; nd < nn; nd += gs) {
      double rr[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const size_t u = (size_t)nd * NB + j;
        const double pu = it == 0 ? m.z[u] : m.z[u] + be * m.p[u];
        const double su = it == 0 ? m.q[u] : m.q[u] + be * m.sv[u];
        m.p[u] = pu;
        m.sv[u] = su;
        m.x[u] += al * pu;
        rr[j] = m.r[u] - al * su;
        m.r[u] = rr[j];
      }
      gn += node_precond<NB>(m.Dinv, nn, nd, rr, m.z);
    }
    grid.sync();  // z complete before the product
    double dn = product();
    grid_sum2(gn, dn, part, red, grid);
    ++it;
    if (gn <= m.rtol * m.rtol * g0r || it >= m.max_iter) {
      gam = gn;
      break;
    }
    be = gn / gam;
    al = gn / (dn - be * gn / al);
    gam = gn;
  }
  const int nnp = nm + 1;
  int nnodes = 1, nblocks = 1;
  for (int ax = 0; ax < D; ++ax) {
    nnodes *= nnp;
    nblocks *= nm;
  }
  for (int u = g0; u < nnodes * NB; u += gs) {
    const int j = u % NB;
    int nd = u / NB, k[3] = {0, 0, 1};
    for (int ax = 0; ax < D; ++ax) {
      k[ax] = nd % nnp;
      nd /= nnp;
    }
    const int vi = interior_index<D>(k, ni);
    m.U[u] = vi >= 0 ? m.x[(size_t)vi * NB + j] : 0.0;
  }
  grid.sync();
  for (int u = g0; u < nblocks * NB; u += gs) {
    const int j = u % NB;
    int pb = u / NB, B[3] = {0, 0, 0};
    for (int ax = 0; ax < D; ++ax) {
      B[ax] = pb % nm;
      pb /= nm;
    }
    double sum = 0.0;
    for (int c = 0; c < K; ++c) {
      size_t idx = 0, str = 1;
      for (int ax = 0; ax < D; ++ax) {
        idx += (size_t)(B[ax] + ((c >> ax) & 1)) * str;
        str *= nnp;
      }
      sum += m.U[idx * NB + j];
    }
    m.Ub[u] = sum / K;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *m.iters = it;
    *m.resid = rel_resid(gam, g0r);
  }
}

int launch_macro_load(mch_plan* pl, const double* f, double* b, hipStream_t s) {
  const int N = pl->cfg.n_cont;
  if (pl->dim == 3) {
    ProfScope ps(pl, "macro_load", s);
    hipLaunchKernelGGL(k_macro_load3d, dim3(pl->P), dim3(MT), 0, s, pl->d_phikp, f, pl->n, pl->nm, pl->H, pl->M, N,
                       pl->cfg.h, b);
    return hip_check(hipGetLastError(), "launch k_macro_load3d");
  }
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

// Device arrays of one macroscopic solve: element matrices [P][KN][KN],
// nodal stencil rows [3^D N][n], vectors x, r, z, p, q [n], block inverses
// [N N][n / N], s [n], the grid-wide partial sums [2 kMacroGridMax], and the
// iteration count and final residual.
struct MacroScratch {
  double* E;
  double* S;
  double* vec;
  double* part;
  int32_t* iters;
  double* resid;
};

// Doubles of the arrays above for a plan (the two counts are not included).
static size_t macro_scratch_doubles(const mch_plan* pl) {
  const int N = pl->cfg.n_cont, D = pl->dim, nm = pl->nm;
  size_t nn = 1;
  for (int ax = 0; ax < D; ++ax) nn *= (size_t)(nm - 1);
  const size_t n = nn * N, KN = (size_t)(1 << D) * N, NS = D == 2 ? 9 : 27;
  return (size_t)pl->P * KN * KN + NS * N * n + (6 + (size_t)N) * n + 2 * (size_t)kMacroGridMax;
}

// The launch sequence of a macroscopic solve on the given scratch. prof is
// the plan whose profiling brackets the launches, or nullptr (no events).
static int macro_solve_on(const mch_plan* pl, mch_plan* prof, const MacroScratch& sc, const double* A,
                          const double* b, double* U, double* Ub, double rtol, int max_iter, hipStream_t s) {
  const int N = pl->cfg.n_cont, nm = pl->nm, D = pl->dim;
  int rc = MCH_OK;
  {
    ProfScope ps(prof, "macro_elem", s);
    if (D == 2)
      hipLaunchKernelGGL(k_macro_elem<2>, dim3(pl->P), dim3(MT), 0, s, A, N, 1.0 / nm, sc.E);
    else
      hipLaunchKernelGGL(k_macro_elem<3>, dim3(pl->P), dim3(MT), 0, s, A, N, 1.0 / nm, sc.E);
    rc = hip_check(hipGetLastError(), "launch k_macro_elem");
  }
  if (rc) return rc;
  size_t nn = 1;
  for (int ax = 0; ax < D; ++ax) nn *= (size_t)(nm - 1);
  const size_t n = nn * N;
  const int NS = D == 2 ? 9 : 27, grid = (int)((n + MT - 1) / MT);
  {
    ProfScope ps(prof, "macro_stencil", s);
    if (D == 2)
      hipLaunchKernelGGL(k_macro_stencil<2>, dim3(grid), dim3(MT), 0, s, sc.E, nm, N, (int)n, sc.S);
    else
      hipLaunchKernelGGL(k_macro_stencil<3>, dim3(grid), dim3(MT), 0, s, sc.E, nm, N, (int)n, sc.S);
    rc = hip_check(hipGetLastError(), "launch k_macro_stencil");
  }
  if (rc) return rc;
  MacroArgs m{};
  m.nm = nm;
  m.S = sc.S;
  m.b = b;
  m.x = sc.vec;
  m.r = m.x + n;
  m.z = m.r + n;
  m.p = m.z + n;
  m.q = m.p + n;
  double* dinv = m.q + n;  // [N N][nn]
  m.sv = dinv + (size_t)N * n;
  m.Dinv = dinv;
  m.rtol = rtol;
  m.max_iter = max_iter;
  m.U = U;
  m.Ub = Ub;
  m.iters = sc.iters;
  m.resid = sc.resid;
  const int ngrid = (int)((nn + MT - 1) / MT), centre = (NS - 1) / 2;
  {
    ProfScope ps(prof, "macro_blockinv", s);
    if (N == 1)
      hipLaunchKernelGGL(k_macro_blockinv<1>, dim3(ngrid), dim3(MT), 0, s, sc.S, (int)n, centre, dinv);
    else if (N == 2)
      hipLaunchKernelGGL(k_macro_blockinv<2>, dim3(ngrid), dim3(MT), 0, s, sc.S, (int)n, centre, dinv);
    else
      hipLaunchKernelGGL(k_macro_blockinv<3>, dim3(ngrid), dim3(MT), 0, s, sc.S, (int)n, centre, dinv);
    rc = hip_check(hipGetLastError(), "launch k_macro_blockinv");
  }
  if (rc) return rc;
  const size_t lds_doubles = (5 + (size_t)N) * n;
  if (lds_doubles <= kMacroLdsDoubles) {
    const size_t lds = lds_doubles * sizeof(double);
    auto go = [&](auto kernel) -> int {
      int e = hip_check(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                        "hipFuncSetAttribute");
      if (e) return e;
      ProfScope ps(prof, "macro_cg", s);
      hipLaunchKernelGGL(kernel, dim3(1), dim3(CGT), lds, s, m);
      return hip_check(hipGetLastError(), "launch k_macro_cg");
    };
    if (D == 2) {
      if (N == 1) return go(k_macro_cg<2, 1>);
      if (N == 2) return go(k_macro_cg<2, 2>);
      return go(k_macro_cg<2, 3>);
    }
    if (N == 1) return go(k_macro_cg<3, 1>);
    if (N == 2) return go(k_macro_cg<3, 2>);
    return go(k_macro_cg<3, 3>);
  }
  // grid-wide: kMacroGridDefault workgroups of GGT threads (fewer if the rows
  // need fewer), all co-resident
  int cus = 0;
  rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device), "hipDeviceGetAttribute");
  if (rc) return rc;
  auto go_grid = [&](auto kernel) -> int {
    const void* fn = reinterpret_cast<const void*>(kernel);
    int per_cu = 0;
    int e = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, GGT, 0), "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (e) return e;
    if (per_cu < 1) return set_error(MCH_EINVAL, "the grid-wide macroscopic CG cannot be resident");
    size_t want = (n + GGT - 1) / GGT;
    if (const char* v = std::getenv("MCH_MACRO_GRID")) want = std::max(1, std::atoi(v));  // tuning override
    else want = std::min<size_t>(want, kMacroGridDefault);
    const int grid = (int)std::min<size_t>(want, (size_t)cus * per_cu);
    if (grid > kMacroGridMax) return set_error(MCH_EINVAL, "grid-wide macroscopic CG: too many workgroups");
    double* part = sc.part;
    void* args[] = {&m, &part};
    ProfScope ps(prof, "macro_cg", s);
    return hip_check(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(GGT), args, 0, s), "hipLaunchCooperativeKernel");
  };
  if (D == 2) {
    if (N == 1) return go_grid(k_macro_cg_grid<2, 1>);
    if (N == 2) return go_grid(k_macro_cg_grid<2, 2>);
    return go_grid(k_macro_cg_grid<2, 3>);
  }
  if (N == 1) return go_grid(k_macro_cg_grid<3, 1>);
  if (N == 2) return go_grid(k_macro_cg_grid<3, 2>);
  return go_grid(k_macro_cg_grid<3, 3>);
}

int launch_macro_solve(mch_plan* pl, const double* A, const double* b, double* U, double* Ub, double rtol,
                       int max_iter, hipStream_t s) {
  if (pl->nm < 2) return set_error(MCH_EINVAL, "the macroscopic system needs at least 2 blocks per axis");
  int rc = ensure_macro_scratch(pl);
  if (rc) return rc;
  const MacroScratch sc{pl->d_macroE, pl->d_macroS, pl->d_mvec, pl->d_mpart, pl->d_macro_iters, pl->d_macro_resid};
  return macro_solve_on(pl, pl, sc, A, b, U, Ub, rtol, max_iter, s);
}

// ---- the solve without allocation ------------------------------------------
// One fixed buffer per device for the arrays of macro_solve_on, for callers
// that cannot allocate. In host code `scratch` names a host-side stand-in, not
// device memory: its device address comes from hipGetSymbolAddress, once per
// device with that device current, and only that address is handed to
// kernels. Every call on a device shares the buffer and leaves its contents
// behind; the kernels write every array before they read it, so nothing needs
// clearing. Calls that overlap on one device race on it.
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

static int noalloc_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return set_error(MCH_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    int rc = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    if (rc) return rc;
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return MCH_OK;
}

int launch_macro_solve_noalloc(const mch_plan* pl, const double* A, const double* b, double* U, double* Ub,
                               double rtol, int max_iter, int32_t* iters, double* resid, hipStream_t s) {
  if (pl->nm < 2) return set_error(MCH_EINVAL, "the macroscopic system needs at least 2 blocks per axis");
  const size_t need = macro_scratch_doubles(pl);
  if (need > kNoAllocScratchDoubles)
    return set_error(MCH_EINVAL, "macroscopic system too large for the fixed scratch buffer: needs " +
                                     std::to_string(need * sizeof(double)) + " bytes, the buffer holds " +
                                     std::to_string(kNoAllocScratchDoubles * sizeof(double)));
  double* base = nullptr;
  int rc = noalloc_scratch(pl->device, &base);
  if (rc) return rc;
  const int N = pl->cfg.n_cont, D = pl->dim;
  size_t nn = 1;
  for (int ax = 0; ax < D; ++ax) nn *= (size_t)(pl->nm - 1);
  const size_t n = nn * N, KN = (size_t)(1 << D) * N, NS = D == 2 ? 9 : 27;
  MacroScratch sc{};
  sc.E = base;
  sc.S = sc.E + (size_t)pl->P * KN * KN;
  sc.vec = sc.S + NS * N * n;
  sc.part = sc.vec + (6 + (size_t)N) * n;
  sc.iters = iters;
  sc.resid = resid;
  return macro_solve_on(pl, nullptr, sc, A, b, U, Ub, rtol, max_iter, s);
}

}  // namespace mch
