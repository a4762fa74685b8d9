// 2D cell kernels for gfx950: effective tensors and the host side of the
// constrained cell solves (launch configuration, the level DAG). The solve
// kernel itself is in solve2d_kernel.h.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "kernels2d.h"

namespace mch {
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
  // inherited fine vectors: level 1's solutions (interp = 0, indexed by the
  // level-1 slot) or the level's own interpolated I (interp = 1, identity slot)
  a.phi1 = (pl->nT > 0 && l > 0) ? lv.d_I : pl->lev[0].d_out;
  a.out = lv.d_out;
  a.tabK = lv.d_tabK;
  a.tabR = lv.d_tabR;
  a.nodeW = lv.d_nodeW;
  a.nodeB = lv.d_nodeB;
  a.fin = lv.d_fin;
  a.gin = lv.d_gin;
  a.J = 1;
  a.prec_rows = lv.shape.pre ? lv.shape.rpt / lv.shape.sb : 0;
  a.bc = pl->cfg.bc;
  a.gen_tp = lv.shape.gen_tp;
  a.xcd_groups = pl->xcd_groups;
  a.adjoint = 0;
  a.seed_kp = pl->d_seed_kp;
  a.seed_par = nullptr;
  a.slot = pl->d_slot;
  a.rtol = pl->cfg.rtol;
  a.max_iter = pl->cfg.max_iter;
  a.kw = lv.d_kw;
  a.labw = lv.d_labw;
  a.octw = lv.d_octw;
  a.dinv = lv.d_dinv;
  a.vr = lv.d_vr;
  a.vp = lv.d_vp;
  a.vap = lv.d_vap;
  a.phikp = pl->d_phikp;
  return a;
}

static int ilog2i(int v) {
  int k = 0;
  while ((1 << (k + 1)) <= v) ++k;
  return k;
}

static size_t solve_lds_bytes(int NC, int rpt, int s, int N, int m, bool gal, bool pre, int sb) {
  const int NT = NC * NC / rpt, NW = NT / 64, NB = NC / rpt, PW = NC + 2;
  const int J = schur_lanes(m), MS = (m + J - 1) / J, UST = MS * J;
  size_t d = (size_t)PW * PW + 4 * NW + (size_t)NB * 4 * s * N + (size_t)MS * 64 + (size_t)m + (size_t)NW * UST +
             (size_t)NW * m;
  // 64^2 fine cells: kappa/6 and (one band per thread) the iterate
  if (!gal && NC >= 64) d += (size_t)(NC + 1) * (NC + 1) + (sb > 1 ? 0 : (size_t)NC * NC);
  // elimination factors of the band coarse correction (see the kernel)
  if (pre) d += (size_t)NB * sb * 2 * ((size_t)NC * ilog2i(NC) - (NC - 1));
  return d * sizeof(double);
}

// Solve kernel of a shape (nullptr if not instantiated) and its block size.
static const void* solve_kernel(int NC, int rpt, int N, bool gal, bool pre, int sb, int S, int* threads) {
  switch (S) {
    case 1: return solve_kernel_sub<1>(NC, rpt, N, gal, pre, sb, threads);
    case 2: return solve_kernel_sub<2>(NC, rpt, N, gal, pre, sb, threads);
    case 4: return solve_kernel_sub<4>(NC, rpt, N, gal, pre, sb, threads);
    case 8: return solve_kernel_sub<8>(NC, rpt, N, gal, pre, sb, threads);
    default: return nullptr;
  }
}

bool shape_supported_2d(int NC, int rpt, int N, bool gal, int S) {
  int threads = 0;
  return solve_kernel(NC, rpt, N, gal, false, 1, S, &threads) != nullptr;
}

bool prec_supported_2d(int NC, int rpt, int N, bool gal, int S, int m, int sb) {
  int threads = 0;
  return solve_kernel(NC, rpt, N, gal, true, sb, S, &threads) != nullptr &&
         solve_lds_bytes(NC, rpt, S, N, m, gal, true, sb) <= 160 * 1024;
}

int launch_solve(const CellArgs& a_in, int rpt, hipStream_t s) {
  if (a_in.gen_tp > 0) return launch_solve_generic(a_in, s);
  if (a_in.bc != 0) return set_error(MCH_EINVAL, "the register-resident solve kernel takes Dirichlet cells only");
  CellArgs a = a_in;
  a.J = schur_lanes(a.m);
  const bool gal = a.r > 1;
  const bool pre = a.prec_rows > 0;
  // sub-bands per thread's rows: the correction's band height divides them
  const int sb = pre ? rpt / a.prec_rows : 1;
  if (pre && a.prec_rows * sb != rpt) return set_error(MCH_EINVAL, "band coarse correction rows do not divide the kernel's");
  const size_t lds = solve_lds_bytes(a.NC, rpt, a.s, a.N, a.m, gal, pre, sb);
  if (lds > 160 * 1024) return set_error(MCH_EINVAL, "cell solve exceeds the LDS budget");
  int threads = 0;
  const void* fn = solve_kernel(a.NC, rpt, a.N, gal, pre, sb, a.s, &threads);
  if (!fn) return set_error(MCH_ENOTIMPL, "no kernel for this cell shape");
  if (lds > 64 * 1024) {
    int rc = hip_check(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                       "hipFuncSetAttribute");
    if (rc) return rc;
  }
  void* args[] = {&a};
  int rc = hip_check(hipLaunchKernel(fn, dim3(a.count * a.M), dim3(threads), args, lds, s), "launch k_solve2d");
  return rc;
}

int solve_blocks_per_cu_2d(mch_plan* pl) {
  CellArgs a = base_args(pl, nullptr, nullptr, 0);
  if (a.gen_tp > 0) return generic_blocks_per_cu(a);
  const int rpt = pl->lev[0].shape.rpt;
  const bool pre = a.prec_rows > 0;
  const int sb = pre ? rpt / a.prec_rows : 1;
  const size_t lds = solve_lds_bytes(a.NC, rpt, a.s, a.N, a.m, false, pre, sb);
  int threads = 0;
  const void* fn = solve_kernel(a.NC, rpt, a.N, false, pre, sb, a.s, &threads);
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

// interp = 1: level n inherits from every level below it, so the levels run
// as a chain on s: level 1, then per level n >= 2 the interpolation of I, the
// inherited right-hand sides and the solve, and for n < L the fine
// Phi = I + P xi into the level's T slots. The setups need only kappa and
// labels; they run on the level streams from the start, beside level 1.
static int launch_forward_2d_chain(mch_plan* pl, const double* kappa, const uint8_t* label, hipStream_t s) {
  char name[32];
  int rc = ensure_streams(pl);
  if (!rc) rc = fork_levels(pl, s);
  for (int l = 1; l < pl->L && !rc; ++l) {
    if (pl->lev[l].count == 0) continue;
    hipStream_t t = level_stream(pl, l, s);
    std::snprintf(name, sizeof(name), "setup_L%d", l + 1);
    {
      ProfScope ps(pl, name, t);
      rc = launch_setup(base_args(pl, kappa, label, l), t);
    }
    if (!rc && !pl->serial) rc = hip_check(hipEventRecord(pl->ev_setup[l], t), "hipEventRecord");
  }
  for (int l = 0; l < pl->L && !rc; ++l) {
    if (pl->lev[l].count == 0) continue;
    CellArgs a = base_args(pl, kappa, label, l);
    if (l == 0) {
      ProfScope ps(pl, "setup_L1", s);
      rc = launch_setup(a, s);
    } else {
      rc = launch_interp(pl, l, s);
      if (!rc && !pl->serial) rc = hip_check(hipStreamWaitEvent(s, pl->ev_setup[l], 0), "hipStreamWaitEvent");
      if (!rc) {
        std::snprintf(name, sizeof(name), "inherit_L%d", l + 1);
        ProfScope ps(pl, name, s);
        rc = launch_inherit(a, s);
      }
    }
    if (!rc) {
      std::snprintf(name, sizeof(name), "solve_L%d", l + 1);
      ProfScope ps(pl, name, s);
      rc = launch_solve(a, pl->lev[l].shape.rpt, s);
    }
    if (!rc && l > 0 && l + 1 < pl->L) rc = launch_recon_2d(pl, a, l, s);
  }
  if (!rc) rc = join_levels(pl, s);
  return rc;
}

// Forward DAG: the setups of levels >= 2 need only kappa and labels and run
// on their side streams from the start (they fill the CUs left idle by the
// level-1 solve). Level 1 solves in two chunks; each level >= 2 inherits and
// solves the cells of chunk A once chunk A is done (alongside the tail chunk
// B of level 1), and the rest, on a second stream of the level, as soon as
// level 1 is done.
int launch_forward_2d(mch_plan* pl, const double* kappa, const uint8_t* label, hipStream_t s) {
  if (pl->nT > 0) return launch_forward_2d_chain(pl, kappa, label, s);
  char name[32];
  int rc = ensure_streams(pl);
  if (!rc) rc = fork_levels(pl, s);
  // The level-1 set-up is issued first: it heads the critical path, and
  // issued after the other levels' set-ups its workgroups (1024 threads on
  // the small fine levels) waited for CUs those had taken.
  const int n1 = pl->lev[0].count, n1a = pl->n1a;
  const CellArgs a1 = base_args(pl, kappa, label, 0);
  if (!rc && n1) {
    ProfScope ps(pl, "setup_L1", s);
    rc = launch_setup(a1, s);
  }
  for (int l = 1; l < pl->L && !rc; ++l) {
    if (pl->lev[l].count == 0) continue;
    CellArgs a = base_args(pl, kappa, label, l);
    std::snprintf(name, sizeof(name), "setup_L%d", l + 1);
    {
      ProfScope ps(pl, name, level_stream(pl, l, s));
      rc = launch_setup(a, level_stream(pl, l, s));
    }
    if (!rc && !pl->serial) rc = hip_check(hipEventRecord(pl->ev_setup[l], pl->side[l]), "hipEventRecord");
  }
  if (!rc && n1) {
    const CellArgs& a = a1;
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
    CellArgs a = base_args(pl, kappa, label, l);
    for (int part = 0; part < 2 && !rc; ++part) {
      const int start = part ? ca : 0, num = part ? cnt - ca : ca;
      // the second part has a stream of its own: it waits for the level's
      // setup and the end of level 1, not for the first part's solve
      hipStream_t t = part ? level_stream2(pl, l, s) : level_stream(pl, l, s);
      if (part && !pl->serial) rc = hip_check(hipStreamWaitEvent(t, pl->ev_setup[l], 0), "hipStreamWaitEvent");
      if (!rc) rc = hip_check(hipStreamWaitEvent(t, part ? pl->ev_l1 : pl->ev_l1a, 0), "hipStreamWaitEvent");
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
