// Plan construction: configuration checks, the macrogrid hierarchy
// (Sec. 3.1, Eq. defi_Sn), per-level kernel shapes, Galerkin tables for the
// nested spaces V_n (Sec. 3.2) and device scratch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "kernels2d.h"
#include "plan.h"

namespace mch {

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return MCH_OK;
  return set_error(MCH_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

static int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Node rows per thread for a level's cell width. A shape is valid when the
// band height divides the sub-block width (bands never straddle constraint
// regions) and the block holds whole waves of at most 1024 threads. An
// environment override MCH_RPT_<NC> lets the tuner sweep the choice.
static bool rpt_ok(int NC, int sbw, int rpt) {
  int t = NC * NC / rpt;
  return rpt >= 1 && NC % rpt == 0 && sbw % rpt == 0 && t <= 1024 && t >= 64 && t % 64 == 0;
}

static int default_rpt(int NC, int sbw) {
  int want = NC >= 64 ? 8 : 4;
  char name[32];
  std::snprintf(name, sizeof(name), "MCH_RPT_%d", NC);
  if (const char* v = std::getenv(name)) want = std::atoi(v);
  if (rpt_ok(NC, sbw, want)) return want;
  for (int rpt : {4, 8, 2, 1, 16})
    if (rpt_ok(NC, sbw, rpt)) return rpt;
  return 0;
}

// 2D level of width NCl: 0 for the register-resident solve kernel, else the
// generic kernel's threads per sub-block tile (Neumann cells, widths without
// an instantiated shape, or MCH_GENERIC=1); -1 if neither kernel takes it.
static int generic_choice_2d(const mch_config& c, int NCl, int r) {
  const int sbw = c.n_cell / c.n_sub / r;
  bool gen = c.bc != 0;
  if (const char* v = std::getenv("MCH_GENERIC")) gen = gen || std::atoi(v) != 0;
  if (!gen) {
    const int rpt = default_rpt(NCl, sbw);
    if (rpt != 0 && shape_supported_2d(NCl, rpt, c.n_cont, r > 1, c.n_sub)) return 0;
  }
  // the per-cell kernels around the solve hold a fine cell's nodes in LDS
  if (c.n_cell > 128) return -1;
  const int tp = generic_tile_threads(c.n_sub);
  return tp > 0 ? tp : -1;
}

// 3D level of width NCl: 0 for the column-marching solve kernel, else the
// generic 3D kernel's threads per sub-block tile (Neumann cells, or
// MCH_GENERIC=1); -1 if neither kernel takes it. Both need 2 sub-blocks per
// axis (the inherited right-hand sides assume it).
static int generic_choice_3d(const mch_config& c, int NCl) {
  bool gen = c.bc != 0;
  if (const char* v = std::getenv("MCH_GENERIC")) gen = gen || std::atoi(v) != 0;
  if (!gen) return shape_supported_3d(NCl, c.n_sub, c.n_cont) ? 0 : -1;
  if (c.n_sub != 2 || NCl > 32) return -1;
  const int tp = generic3_tile_threads(c.n_sub);
  return tp > 0 ? tp : -1;
}

template <typename T>
static int dev_alloc(mch_plan* p, T** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) count = 1;
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, count * sizeof(T));
  if (e != hipSuccess) return hip_check(e, "hipMalloc");
  e = hipMemset(v, 0, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipFree(v);
    return hip_check(e, "hipMemset");
  }
  p->allocations.push_back(v);
  *ptr = static_cast<T*>(v);
  return MCH_OK;
}

template <typename T>
static int upload(mch_plan* p, T** ptr, const std::vector<T>& host) {
  int rc = dev_alloc(p, ptr, host.size());
  if (rc) return rc;
  if (host.empty()) return MCH_OK;
  return hip_check(hipMemcpy(*ptr, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
}

// Level of every macropoint: T_n keeps indices = o (mod eta^(L-n)) per axis,
// o = floor(eta^(L-1)/2); the level is the smallest n with the point in T_n.
static void build_hierarchy(mch_plan* p) {
  const int d = p->dim, nm = p->nm, L = p->L, eta = p->cfg.eta;
  const int g = ipow(eta, L - 1), o = g / 2;
  p->level.assign(p->P, 0);
  p->parent.assign(p->P, -1);
  p->slot.assign(p->P, 0);
  for (int q = 0; q < p->P; ++q) {
    int j[3] = {q % nm, (q / nm) % nm, (q / (nm * nm)) % nm};
    int lvl = L;
    for (int n = 1; n <= L; ++n) {
      int step = ipow(eta, L - n);
      bool in = true;
      for (int a = 0; a < d; ++a) in = in && (((j[a] - o) % step + step) % step == 0);
      if (in) {
        lvl = n;
        break;
      }
    }
    p->level[q] = lvl;
    if (lvl > 1) {
      int par = 0, stride = 1;
      for (int a = 0; a < d; ++a) {
        par += ((j[a] / g) * g + o) * stride;
        stride *= nm;
      }
      p->parent[q] = par;
    }
  }
  for (int n = 0; n < L; ++n) p->lev[n].cells.clear();
  for (int q = 0; q < p->P; ++q) {
    mch::Level& lv = p->lev[p->level[q] - 1];
    p->slot[q] = (int32_t)lv.cells.size();
    lv.cells.push_back(q);
  }
  // levels >= 2: order by the slot of the inherited level-1 cell (stable)
  for (int n = 1; n < L; ++n) {
    std::vector<int32_t>& c = p->lev[n].cells;
    std::stable_sort(c.begin(), c.end(),
                     [&](int32_t a, int32_t b) { return p->slot[p->parent[a]] < p->slot[p->parent[b]]; });
    for (size_t k = 0; k < c.size(); ++k) p->slot[c[k]] = (int32_t)k;
  }
}

// Multilinear neighbours (interp = 1, Sec. 3.3, Eq. phiXiI_all): a level-n
// point takes the T_(n-1) lattice indices (step eta^(L-n+1), phase o) that
// bracket its index per axis, periodic in the macropoint index, with the 1D
// linear weights (1 - f, f); the neighbours are the tensor products, axis 1
// fastest, weight = product of the 1D weights, zero weights left out.
static int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

static void build_interp(mch_plan* p) {
  const int d = p->dim, nm = p->nm, L = p->L, eta = p->cfg.eta, K = 1 << d;
  const int o = ipow(eta, L - 1) / 2;
  p->nbr.assign((size_t)p->P * K, -1);
  p->nbw.assign((size_t)p->P * K, 0.0);
  for (int q = 0; q < p->P; ++q) {
    const int n = p->level[q];
    if (n == 1) continue;
    const int step = ipow(eta, L - n + 1);
    const int j[3] = {q % nm, (q / nm) % nm, (q / (nm * nm)) % nm};
    int cnt = 1, ids[8] = {0}, str = 1;
    double ws[8] = {1.0};
    for (int a = 0; a < d; ++a) {
      const int lo = o + floor_div(j[a] - o, step) * step;
      const double f = (double)(j[a] - lo) / (double)step;
      const int lw = ((lo % nm) + nm) % nm, hi = (lo + step) % nm;
      if (f == 0.0) {
        for (int k = 0; k < cnt; ++k) ids[k] += lw * str;
      } else {
        // the new axis is the outer loop: entries [0, cnt) take lo, [cnt, 2 cnt) take hi
        for (int k = 0; k < cnt; ++k) {
          ids[cnt + k] = ids[k] + hi * str;
          ws[cnt + k] = ws[k] * f;
          ids[k] += lw * str;
          ws[k] = ws[k] * (1.0 - f);
        }
        cnt *= 2;
      }
      str *= nm;
    }
    for (int k = 0; k < cnt; ++k) {
      p->nbr[(size_t)q * K + k] = ids[k];
      p->nbw[(size_t)q * K + k] = ws[k];
    }
  }
}

// Coarse-element tables of the Galerkin operator for a level with ratio r:
// fine element at position (u, v) inside a coarse element contributes
// kappa_s * R^T K_ref R to the coarse element matrix, and rho[a] = sum of
// R[delta][a] over its corners to the coarse constraint weights.
static void galerkin_tables(int r, std::vector<double>& tk, std::vector<double>& tr) {
  static const double kref[4][4] = {{4, -1, -1, -2}, {-1, 4, -2, -1}, {-1, -2, 4, -1}, {-2, -1, -1, 4}};
  tk.assign((size_t)r * r * 16, 0.0);
  tr.assign((size_t)r * r * 4, 0.0);
  for (int v = 0; v < r; ++v)
    for (int u = 0; u < r; ++u) {
      double R[4][4];
      for (int dlt = 0; dlt < 4; ++dlt) {
        double xi = (u + (dlt & 1)) / (double)r, ze = (v + (dlt >> 1)) / (double)r;
        for (int a = 0; a < 4; ++a) R[dlt][a] = ((a & 1) ? xi : 1.0 - xi) * ((a >> 1) ? ze : 1.0 - ze);
      }
      const int pos = u + r * v;
      for (int a = 0; a < 4; ++a) {
        double s = 0;
        for (int dlt = 0; dlt < 4; ++dlt) s += R[dlt][a];
        tr[pos * 4 + a] = s;
        for (int b = 0; b < 4; ++b) {
          double t = 0;
          for (int x = 0; x < 4; ++x)
            for (int y = 0; y < 4; ++y) t += R[x][a] * (kref[x][y] / 6.0) * R[y][b];
          tk[pos * 16 + a * 4 + b] = t;
        }
      }
    }
}

// 3D version: trilinear R, the Q1 hexahedron element matrix h*(4, 0, -1, -1)/12
// (diagonal, edge, face-diagonal, body-diagonal corner pairs); corners in
// tensor order a = ax + 2 ay + 4 az. Tables T[r^3][64] and rho[r^3][8].
static void galerkin_tables_3d(int r, double h, std::vector<double>& tk, std::vector<double>& tr) {
  double kref[8][8];
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) {
      const int dif = __builtin_popcount(a ^ b);
      kref[a][b] = h * (dif == 0 ? 4.0 : dif == 1 ? 0.0 : -1.0) / 12.0;
    }
  const size_t r3 = (size_t)r * r * r;
  tk.assign(r3 * 64, 0.0);
  tr.assign(r3 * 8, 0.0);
  for (int w = 0; w < r; ++w)
    for (int v = 0; v < r; ++v)
      for (int u = 0; u < r; ++u) {
        double R[8][8];
        for (int dl = 0; dl < 8; ++dl) {
          const double xi = (u + (dl & 1)) / (double)r, et = (v + ((dl >> 1) & 1)) / (double)r,
                       ze = (w + (dl >> 2)) / (double)r;
          for (int a = 0; a < 8; ++a)
            R[dl][a] = ((a & 1) ? xi : 1.0 - xi) * (((a >> 1) & 1) ? et : 1.0 - et) * ((a >> 2) ? ze : 1.0 - ze);
        }
        const int pos = u + r * (v + r * w);
        for (int a = 0; a < 8; ++a) {
          double sr = 0;
          for (int dl = 0; dl < 8; ++dl) sr += R[dl][a];
          tr[pos * 8 + a] = sr;
          for (int b = 0; b < 8; ++b) {
            double t = 0;
            for (int x = 0; x < 8; ++x)
              for (int y = 0; y < 8; ++y) t += R[x][a] * kref[x][y] * R[y][b];
            tk[pos * 64 + a * 8 + b] = t;
          }
        }
      }
}

ProfScope::ProfScope(mch_plan* plan, const char* name, hipStream_t stream) : p(plan), s(stream), idx(0), on(false) {
  if (!p || !p->profiling) return;
  if (p->prof_used == p->prof.size()) {
    ProfRec r;
    if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) return;
    p->prof.push_back(r);
  }
  idx = p->prof_used++;
  p->prof[idx].name = name;
  on = hipEventRecord(p->prof[idx].start, s) == hipSuccess;
}

ProfScope::~ProfScope() {
  if (on) (void)hipEventRecord(p->prof[idx].stop, s);
}

int ensure_streams(mch_plan* p) {
  if (p->ev_fork) return MCH_OK;
  int rc = hip_check(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming), "hipEventCreate");
  if (!rc) rc = hip_check(hipEventCreateWithFlags(&p->ev_l1, hipEventDisableTiming), "hipEventCreate");
  if (!rc) rc = hip_check(hipEventCreateWithFlags(&p->ev_l1a, hipEventDisableTiming), "hipEventCreate");
  for (int l = 1; l < p->L && !rc; ++l) {
    rc = hip_check(hipStreamCreateWithFlags(&p->side[l], hipStreamNonBlocking), "hipStreamCreate");
    if (!rc) rc = hip_check(hipStreamCreateWithFlags(&p->side2[l], hipStreamNonBlocking), "hipStreamCreate");
    if (!rc) rc = hip_check(hipEventCreateWithFlags(&p->ev_join[l], hipEventDisableTiming), "hipEventCreate");
    if (!rc) rc = hip_check(hipEventCreateWithFlags(&p->ev_join2[l], hipEventDisableTiming), "hipEventCreate");
    if (!rc) rc = hip_check(hipEventCreateWithFlags(&p->ev_setup[l], hipEventDisableTiming), "hipEventCreate");
    if (!rc) rc = hip_check(hipEventCreateWithFlags(&p->ev_adj[l], hipEventDisableTiming), "hipEventCreate");
    if (!rc) rc = hip_check(hipEventCreateWithFlags(&p->ev_ibar[l], hipEventDisableTiming), "hipEventCreate");
  }
  return rc;
}

int fork_levels(mch_plan* p, hipStream_t s) {
  if (p->serial) return MCH_OK;
  int rc = hip_check(hipEventRecord(p->ev_fork, s), "hipEventRecord");
  for (int l = 1; l < p->L && !rc; ++l)
    if (p->lev[l].count) {
      rc = hip_check(hipStreamWaitEvent(p->side[l], p->ev_fork, 0), "hipStreamWaitEvent");
      if (!rc) rc = hip_check(hipStreamWaitEvent(p->side2[l], p->ev_fork, 0), "hipStreamWaitEvent");
    }
  return rc;
}

int mark_level(mch_plan* p, int l, hipEvent_t* ev) {
  if (p->serial || l < 1) return MCH_OK;
  return hip_check(hipEventRecord(ev[l], p->side[l]), "hipEventRecord");
}

int wait_marks(mch_plan* p, hipStream_t s, hipEvent_t* ev) {
  if (p->serial) return MCH_OK;
  int rc = MCH_OK;
  for (int l = 1; l < p->L && !rc; ++l)
    if (p->lev[l].count) rc = hip_check(hipStreamWaitEvent(s, ev[l], 0), "hipStreamWaitEvent");
  return rc;
}

int join_levels(mch_plan* p, hipStream_t s) {
  if (p->serial) return MCH_OK;
  int rc = MCH_OK;
  for (int l = 1; l < p->L && !rc; ++l) {
    if (!p->lev[l].count) continue;
    rc = hip_check(hipEventRecord(p->ev_join[l], p->side[l]), "hipEventRecord");
    if (!rc) rc = hip_check(hipStreamWaitEvent(s, p->ev_join[l], 0), "hipStreamWaitEvent");
    if (!rc) rc = hip_check(hipEventRecord(p->ev_join2[l], p->side2[l]), "hipEventRecord");
    if (!rc) rc = hip_check(hipStreamWaitEvent(s, p->ev_join2[l], 0), "hipStreamWaitEvent");
  }
  return rc;
}

}  // namespace mch

using namespace mch;

extern "C" const char* mch_last_error(void) { return g_last_error.c_str(); }

extern "C" void mch_destroy(mch_plan* plan) {
  if (!plan) return;
  // the plan's streams, graphs and memory belong to its device
  (void)hipSetDevice(plan->device);
  (void)hipDeviceSynchronize();
  for (auto* g : {&plan->g_fwd, &plan->g_eff, &plan->g_bwd}) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
  }
  for (int l = 0; l < MAX_LEVELS; ++l) {
    if (plan->side[l]) (void)hipStreamDestroy(plan->side[l]);
    if (plan->side2[l]) (void)hipStreamDestroy(plan->side2[l]);
    if (plan->ev_join[l]) (void)hipEventDestroy(plan->ev_join[l]);
    if (plan->ev_join2[l]) (void)hipEventDestroy(plan->ev_join2[l]);
    if (plan->ev_setup[l]) (void)hipEventDestroy(plan->ev_setup[l]);
    if (plan->ev_adj[l]) (void)hipEventDestroy(plan->ev_adj[l]);
    if (plan->ev_ibar[l]) (void)hipEventDestroy(plan->ev_ibar[l]);
  }
  if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
  if (plan->ev_l1) (void)hipEventDestroy(plan->ev_l1);
  if (plan->ev_l1a) (void)hipEventDestroy(plan->ev_l1a);
  for (auto& r : plan->prof) {
    if (r.start) (void)hipEventDestroy(r.start);
    if (r.stop) (void)hipEventDestroy(r.stop);
  }
  for (void* v : plan->allocations) (void)hipFree(v);
  delete plan;
}

extern "C" int mch_build_levels(const mch_config* cfg, mch_plan** out) {
  g_last_error.clear();
  if (!cfg || !out) return set_error(MCH_EINVAL, "null argument");
  *out = nullptr;
  const mch_config& c = *cfg;
  if (c.dim != 2 && c.dim != 3) return set_error(MCH_EINVAL, "dim must be 2 or 3");
  const int d = c.dim, n = c.n_fine[0], nm = c.n_macro[0];
  for (int a = 0; a < d; ++a) {
    if (c.n_fine[a] != n || c.n_macro[a] != nm) return set_error(MCH_EINVAL, "grid must be cubic (equal sizes per axis)");
  }
  if (n < 2 || nm < 1 || n % nm != 0) return set_error(MCH_EINVAL, "n_fine must be a positive multiple of n_macro");
  if (!(std::fabs(c.h * n - 1.0) < 1e-12)) return set_error(MCH_EINVAL, "h must equal 1/n_fine");
  const int H = n / nm;
  if (H % 2 != 0) return set_error(MCH_EINVAL, "coarse block size H = n_fine/n_macro must be even");
  if (c.levels < 1 || c.levels > MAX_LEVELS) return set_error(MCH_EINVAL, "levels out of range");
  if (c.eta < 1) return set_error(MCH_EINVAL, "eta must be >= 1");
  if (c.n_cont < 1 || c.n_cont > 3) return set_error(MCH_EINVAL, "n_cont must be 1..3");
  if (c.n_sub < 1) return set_error(MCH_EINVAL, "n_sub must be >= 1");
  if (c.interp != 0 && c.interp != 1) return set_error(MCH_EINVAL, "interp must be 0 or 1");
  if (c.bc != 0 && c.bc != 1) return set_error(MCH_EINVAL, "bc must be 0 (Dirichlet) or 1 (Neumann)");
  if (c.bc == 1 && c.interp == 1) return set_error(MCH_ENOTIMPL, "Neumann cells with multilinear inheritance");
  if (!(c.rtol > 0.0) || c.max_iter < 1) return set_error(MCH_EINVAL, "rtol must be > 0 and max_iter >= 1");
  const int nc = c.n_cell;
  const int gL = ipow(c.eta, c.levels - 1);
  if (nc < 2 || nc % 2 != 0 || nc > n) return set_error(MCH_EINVAL, "n_cell must be even and at most n_fine");
  if (nc < H) return set_error(MCH_EINVAL, "n_cell must be at least H (the cell contains K_p)");
  if (nc % c.n_sub != 0 || (nc / c.n_sub) % gL != 0)
    return set_error(MCH_EINVAL, "n_cell must be divisible by n_sub * eta^(L-1)");
  if (nm % gL != 0) return set_error(MCH_EINVAL, "n_macro must be divisible by eta^(L-1)");

  mch_plan* p = new mch_plan();
  p->cfg = c;
  p->dim = d;
  p->n = n;
  p->nm = nm;
  p->H = H;
  p->L = c.levels;
  p->P = ipow(nm, d);
  p->M = c.n_cont * (1 + d);
  p->m = c.n_cont * ipow(c.n_sub, d);
  p->nn = ipow(nc + 1, d);
  const int coarsest = nc / gL;
  const int free_coarsest = ipow(c.bc ? coarsest + 1 : coarsest - 1, d);
  if (p->m > 64) {
    delete p;
    return set_error(MCH_ENOTIMPL, "more than 64 constraint rows per cell");
  }
  if (p->m > free_coarsest) {
    delete p;
    return set_error(MCH_ESINGULAR, "over-constrained: " + std::to_string(c.n_cont * ipow(c.n_sub, d)) +
                                        " constraint rows but " + std::to_string(free_coarsest) +
                                        " free unknowns at the coarsest level");
  }
  // kernel shapes per level, checked before any device work so that a
  // configuration without a kernel fails the same way with or without a GPU
  for (int l = 0; l < p->L; ++l) {
    const int r = ipow(c.eta, l), NCl = nc / r, sbw = nc / c.n_sub / r;
    if (d == 3) {
      if (generic_choice_3d(c, NCl) < 0) {
        delete p;
        return set_error(MCH_ENOTIMPL, "no 3D kernel instantiated for level cell width " + std::to_string(NCl) +
                                           " n_sub=" + std::to_string(c.n_sub) + " N=" + std::to_string(c.n_cont));
      }
      continue;
    }
    (void)sbw;
    if (generic_choice_2d(c, NCl, r) < 0) {
      delete p;
      return set_error(MCH_ENOTIMPL, "no 2D solve kernel for level cell width " + std::to_string(NCl) + " n_sub=" +
                                         std::to_string(c.n_sub) + " n_cell=" + std::to_string(nc) +
                                         " (the generic kernel takes n_cell <= 128 and n_sub <= 8)");
    }
  }
  if (const char* v = std::getenv("MCH_GRAPHS")) p->use_graphs = std::atoi(v) != 0;
  if (const char* v = std::getenv("MCH_SERIAL")) p->serial = std::atoi(v) != 0;
  if (const char* v = std::getenv("MCH_XCD")) p->xcd_groups = std::atoi(v) != 0;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return set_error(MCH_EHIP, "no HIP device");
  }
  build_hierarchy(p);
  // interp = 1 with more than one level: multilinear neighbours, T slots
  const bool ml = c.interp == 1 && p->L > 1;
  if (ml) {
    build_interp(p);
    int off = 0;
    for (int l = 0; l + 1 < p->L; ++l) {
      p->lev[l].toff = off;
      off += (int)p->lev[l].cells.size();
    }
    p->nT = off;
  }
  int rc = MCH_OK;
  size_t max_count = 0;
  for (int l = 0; l < p->L && rc == MCH_OK; ++l) {
    Level& lv = p->lev[l];
    lv.n = l + 1;
    lv.r = ipow(c.eta, l);
    lv.NC = nc / lv.r;
    lv.count = (int)lv.cells.size();
    const int sbw = nc / c.n_sub / lv.r;
    lv.shape.NC = lv.NC;
    if (d == 3) {
      lv.shape.rpt = 0;
      lv.shape.threads = ipow(lv.NC, 3) >= 1024 ? 1024 : ipow(lv.NC, 3);
      lv.shape.gen_tp = generic_choice_3d(c, lv.NC);
      if (lv.shape.gen_tp < 0) {
        rc = set_error(MCH_ENOTIMPL, "no 3D kernel instantiated for level cell width " + std::to_string(lv.NC) +
                                         " n_sub=" + std::to_string(c.n_sub) + " N=" + std::to_string(c.n_cont));
        break;
      }
    } else if ((lv.shape.gen_tp = generic_choice_2d(c, lv.NC, lv.r)) > 0) {
      lv.shape.rpt = 0;
      lv.shape.threads = (lv.shape.gen_tp * c.n_sub * c.n_sub + 63) / 64 * 64;
      lv.shape.pre = false;
    } else {
      lv.shape.rpt = default_rpt(lv.NC, sbw);
      lv.shape.threads = lv.NC * lv.NC / lv.shape.rpt;
      // band coarse correction where its kernel exists and fits, by default
      // on cells of 64 level elements per side (measured: it pays there on
      // the channel media; on 32^2 and 16^2 cells the fewer iterations do
      // not make up for the costlier iterations and setup); MCH_PREC=0 turns
      // it off, 1 keeps the default, 2 uses it on every level that has the
      // kernel (comparisons)
      int mode = 1;
      if (const char* v = std::getenv("MCH_PREC")) mode = std::atoi(v);
      bool want = mode == 2 || (mode == 1 && lv.NC >= 64);
      // per cell width (the size-class tuner's knob): MCH_PREC_<NC> = 0 (off),
      // 1 (bands of a thread's node rows) or 2 (two sub-bands per thread's
      // rows, where that kernel exists and fits)
      int sb = 1;
      char pname[32];
      std::snprintf(pname, sizeof(pname), "MCH_PREC_%d", lv.NC);
      if (const char* v = std::getenv(pname)) {
        const int k = std::atoi(v);
        want = k != 0;
        sb = k >= 2 ? 2 : 1;
      }
      lv.shape.pre = want && prec_supported_2d(lv.NC, lv.shape.rpt, c.n_cont, lv.r > 1, c.n_sub, p->m, sb);
      lv.shape.sb = lv.shape.pre ? sb : 1;
    }
    if (d == 2 && lv.shape.gen_tp == 0 && !shape_supported_2d(lv.NC, lv.shape.rpt, c.n_cont, lv.r > 1, c.n_sub)) {
      rc = set_error(MCH_ENOTIMPL, "no kernel instantiated for level cell width " + std::to_string(lv.NC) +
                                       " rows/thread " + std::to_string(lv.shape.rpt) + " N=" +
                                       std::to_string(c.n_cont));
      break;
    }
    if (lv.count == 0) continue;
    if (l > 0) max_count = std::max(max_count, (size_t)lv.count);
    std::vector<int32_t> ps(lv.count, -1);
    for (int k = 0; k < lv.count; ++k) {
      int q = lv.cells[k];
      // interp = 1: I of a level >= 2 cell is its own row of d_I
      ps[k] = ml ? k : (p->parent[q] >= 0) ? p->slot[p->parent[q]] : -1;
    }
    if ((rc = upload(p, &lv.d_cells, lv.cells))) break;
    if ((rc = upload(p, &lv.d_pslot, ps))) break;
    size_t vec = (l == 0) ? (size_t)p->nn : (size_t)ipow(lv.NC + 1, d);
    // interp = 1: level 1's output holds the fine Phi of every T point
    const size_t rows = (l == 0 && ml) ? (size_t)p->nT : (size_t)lv.count;
    if ((rc = dev_alloc(p, &lv.d_out, rows * p->M * vec))) break;
    if ((rc = dev_alloc(p, &lv.d_w, (size_t)lv.count * p->M * vec))) break;
    // 2D level data (and 3D on the generic kernel) cover every level node
    // [0, NC]^d; the column-marching 3D kernel's the owned [0, NC)^3
    const size_t nodes = (size_t)ipow((d == 2 || lv.shape.gen_tp > 0) ? lv.NC + 1 : lv.NC, d);
    if (d == 2 && lv.shape.gen_tp > 0) {
      // generic solve: D^-1 and the ring-padded r, p and K_n p per (cell, rhs)
      const size_t cm = (size_t)lv.count * p->M, padded = cm * ipow(lv.NC + 3, 2);
      if ((rc = dev_alloc(p, &lv.d_dinv, cm * ipow(lv.NC + 1, 2)))) break;
      if ((rc = dev_alloc(p, &lv.d_vr, padded))) break;
      if ((rc = dev_alloc(p, &lv.d_vp, padded))) break;
      if ((rc = dev_alloc(p, &lv.d_vap, padded))) break;
      if (lv.r == 1) {
        // the fine cell's kappa/6 and label windows, written by the setup
        if ((rc = dev_alloc(p, &lv.d_kw, (size_t)lv.count * lv.NC * lv.NC))) break;
        if ((rc = dev_alloc(p, &lv.d_labw, (size_t)lv.count * lv.NC * lv.NC))) break;
      }
    }
    if (lv.r > 1) {
      std::vector<double> tk, tr;
      if (d == 3)
        galerkin_tables_3d(lv.r, c.h, tk, tr);
      else
        galerkin_tables(lv.r, tk, tr);
      if ((rc = upload(p, &lv.d_tabK, tk))) break;
      if ((rc = upload(p, &lv.d_tabR, tr))) break;
      if ((rc = dev_alloc(p, &lv.d_nodeW, (size_t)lv.count * nodes * ipow(3, d)))) break;
      if ((rc = dev_alloc(p, &lv.d_nodeB, (size_t)lv.count * nodes * ipow(2, d) * c.n_cont))) break;
      if ((rc = dev_alloc(p, &lv.d_fin, (size_t)lv.count * p->M * nodes))) break;
      if ((rc = dev_alloc(p, &lv.d_gin, (size_t)lv.count * p->M * p->m))) break;
    }
    if (ml && l > 0) {
      const int K = 1 << d;
      std::vector<int32_t> nb((size_t)lv.count * K, 0);
      std::vector<double> nw((size_t)lv.count * K, 0.0);
      // CSR over the T slots of the levels below: this level's cells that
      // inherit from each, in increasing cell order
      const int rows_below = (l + 1 < p->L) ? lv.toff : p->nT;  // T slots of levels < l
      std::vector<int32_t> ptr((size_t)rows_below + 1, 0), ch;
      std::vector<double> cw;
      for (int k = 0; k < lv.count; ++k) {
        const int q = lv.cells[k];
        for (int e = 0; e < K; ++e) {
          const int t = p->nbr[(size_t)q * K + e];
          if (t < 0) continue;
          const int ts = p->lev[p->level[t] - 1].toff + p->slot[t];
          nb[(size_t)k * K + e] = ts;
          nw[(size_t)k * K + e] = p->nbw[(size_t)q * K + e];
          ptr[ts + 1]++;
        }
      }
      for (size_t t = 0; t + 1 < ptr.size(); ++t) ptr[t + 1] += ptr[t];
      ch.assign(ptr.back(), 0);
      cw.assign(ptr.back(), 0.0);
      std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
      for (int k = 0; k < lv.count; ++k)
        for (int e = 0; e < K; ++e)
          if (nw[(size_t)k * K + e] != 0.0) {
            const int ts = nb[(size_t)k * K + e];
            ch[fill[ts]] = k;
            cw[fill[ts]++] = nw[(size_t)k * K + e];
          }
      if ((rc = upload(p, &lv.d_nbr, nb))) break;
      if ((rc = upload(p, &lv.d_nbw, nw))) break;
      if ((rc = upload(p, &lv.d_dptr, ptr))) break;
      if ((rc = upload(p, &lv.d_dch, ch))) break;
      if ((rc = upload(p, &lv.d_dw, cw))) break;
      if ((rc = dev_alloc(p, &lv.d_I, (size_t)lv.count * p->M * p->nn))) break;
    }
    if (d == 3) {
      const size_t elems = (size_t)ipow(lv.NC, 3);
      if (lv.r == 1) {
        if ((rc = dev_alloc(p, &lv.d_kw, (size_t)lv.count * elems))) break;
        if ((rc = dev_alloc(p, &lv.d_labw, (size_t)lv.count * elems))) break;
        if (lv.shape.gen_tp == 0 && (rc = dev_alloc(p, &lv.d_octw, (size_t)lv.count * nodes))) break;
      }
      // Krylov vectors: a zero boundary plane at NC (column-marching kernel)
      // or a ring of zeros around [0, NC]^3 (generic kernel)
      const size_t padded = (size_t)lv.count * p->M * ipow(lv.NC + (lv.shape.gen_tp > 0 ? 3 : 1), 3);
      if ((rc = dev_alloc(p, &lv.d_dinv, (size_t)lv.count * nodes))) break;
      if ((rc = dev_alloc(p, &lv.d_vr, padded))) break;
      if ((rc = dev_alloc(p, &lv.d_vp, padded))) break;
      if ((rc = dev_alloc(p, &lv.d_vap, padded))) break;
    }
  }
  const size_t P = p->P, M = p->M, m = p->m;
  const size_t n1 = p->lev[0].count;
  if (!rc) rc = dev_alloc(p, &p->d_cw, P * m);
  if (!rc) rc = dev_alloc(p, &p->d_g, P * M * m);
  if (!rc) rc = dev_alloc(p, &p->d_sinv, P * m * m);
  if (!rc) rc = dev_alloc(p, &p->d_beta, P * M * m);
  if (!rc) rc = dev_alloc(p, &p->d_mu, P * M * m);
  if (!rc) rc = dev_alloc(p, &p->d_iters, P * M);
  if (!rc) rc = dev_alloc(p, &p->d_resid, P * M);
  if (!rc) rc = dev_alloc(p, &p->d_bad, (size_t)kValidateBlocks);
  if (!rc) rc = upload(p, &p->d_slot, p->slot);
  if (!rc) rc = dev_alloc(p, &p->d_seed_kp, P * M * (size_t)ipow(H + 1, d));
  if (!rc) rc = dev_alloc(p, &p->d_seed_par, n1 * M * (size_t)p->nn);
  // 2D: each inheriting level but the deepest keeps its parent seeds apart
  // (the deepest writes d_seed_par), so the per-level passes run in parallel
  for (int l = 1; l + 1 < p->L && !rc && d == 2 && n1 < (size_t)p->P; ++l)
    rc = dev_alloc(p, &p->d_seed_lvl[l], n1 * M * (size_t)p->nn);
  if (!rc && ml) {
    rc = dev_alloc(p, &p->d_seedT, (size_t)p->nT * M * p->nn);
    if (!rc) rc = dev_alloc(p, &p->d_ibar, max_count * M * p->nn);
    std::vector<int32_t> id(max_count + 1);
    for (size_t k = 0; k <= max_count; ++k) id[k] = (int32_t)k;
    if (!rc) rc = upload(p, &p->d_iptr, id);
  }
  if (!rc) rc = dev_alloc(p, &p->d_gk, (size_t)ipow(n, d));
  if (!rc) rc = dev_alloc(p, &p->d_gcell, P * (size_t)ipow(nc, d));
  if (!rc) rc = dev_alloc(p, &p->d_iters_adj, P * M);
  if (!rc) rc = dev_alloc(p, &p->d_resid_adj, P * M);
  if (!rc) rc = upload(p, &p->d_level, p->level);
  if (!rc && d == 3) rc = dev_alloc(p, &p->d_phikp, P * M * (size_t)ipow(H + 1, 3));
  if (!rc) {
    std::vector<int32_t> ptr(n1 + 1, 0), child;
    for (int q = 0; q < p->P; ++q)
      if (p->parent[q] >= 0) ptr[p->slot[p->parent[q]] + 1]++;
    for (size_t t = 0; t < n1; ++t) ptr[t + 1] += ptr[t];
    child.assign(ptr[n1], 0);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int q = 0; q < p->P; ++q)
      if (p->parent[q] >= 0) child[fill[p->slot[p->parent[q]]]++] = q;
    rc = upload(p, &p->d_child_ptr, ptr);
    if (!rc) rc = upload(p, &p->d_child, child);
  }
  // level-1 chunks (see plan.h): the tail is the last partial round of
  // workgroups; with no partial round, or a single level, there is one chunk
  if (!rc) {
    const size_t n1c = p->lev[0].count;
    p->n1a = (int)n1c;
    int cus = 0;
    rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device),
                   "hipDeviceGetAttribute");
    int bpc = 0;
    if (!rc && p->L > 1 && n1c > 0) {
      bpc = d == 3 ? solve_blocks_per_cu_3d(p) : solve_blocks_per_cu_2d(p);
      if (bpc < 0) rc = bpc;
    }
    // MCH_SPLIT=0 runs level 1 as one launch (a scheduling knob of the tuner)
    bool split = true;
    if (const char* v = std::getenv("MCH_SPLIT")) split = std::atoi(v) != 0;
    if (!rc && bpc > 0 && !ml && split) {  // interp = 1 runs the levels as a chain: one chunk
      const size_t slots = (size_t)cus * bpc, W = n1c * p->M, T = W % slots;
      if (W > slots && T != 0) p->n1a = (int)(n1c - (T + p->M - 1) / p->M);
    }
    for (int l = 1; l < p->L && !rc; ++l) {
      int c = 0;
      for (int32_t q : p->lev[l].cells)
        if (p->slot[p->parent[q]] < p->n1a) ++c;
      p->cntA[l] = c;
    }
  }
  if (rc) {
    mch_destroy(p);
    return rc;
  }
  *out = p;
  return MCH_OK;
}

extern "C" int mch_build_hierarchy(const mch_config* cfg, int32_t* level, int32_t* parent) {
  g_last_error.clear();
  if (!cfg || !level || !parent) return set_error(MCH_EINVAL, "null argument");
  const mch_config& c = *cfg;
  if (c.dim != 2 && c.dim != 3) return set_error(MCH_EINVAL, "dim must be 2 or 3");
  const int nm = c.n_macro[0];
  for (int a = 0; a < c.dim; ++a)
    if (c.n_macro[a] != nm) return set_error(MCH_EINVAL, "n_macro must be equal on every axis");
  if (nm < 1 || c.levels < 1 || c.levels > MAX_LEVELS || c.eta < 1)
    return set_error(MCH_EINVAL, "bad n_macro, levels or eta");
  if (nm % ipow(c.eta, c.levels - 1) != 0) return set_error(MCH_EINVAL, "n_macro must be divisible by eta^(L-1)");
  mch_plan tmp;
  tmp.cfg = c;
  tmp.dim = c.dim;
  tmp.nm = nm;
  tmp.L = c.levels;
  tmp.P = ipow(nm, c.dim);
  build_hierarchy(&tmp);
  std::memcpy(level, tmp.level.data(), sizeof(int32_t) * tmp.P);
  std::memcpy(parent, tmp.parent.data(), sizeof(int32_t) * tmp.P);
  return MCH_OK;
}

int mch::ensure_macro_scratch(mch_plan* p) {
  if (p->d_macroE) return MCH_OK;
  const size_t KN = (size_t)ipow(2, p->dim) * p->cfg.n_cont;
  const size_t nint = (size_t)ipow(p->nm - 1, p->dim) * p->cfg.n_cont;
  int rc = dev_alloc(p, &p->d_macroE, (size_t)p->P * KN * KN);
  if (!rc) rc = dev_alloc(p, &p->d_macroS, (size_t)ipow(3, p->dim) * p->cfg.n_cont * nint);
  if (!rc) rc = dev_alloc(p, &p->d_mvec, (6 + (size_t)p->cfg.n_cont) * nint);
  if (!rc) rc = dev_alloc(p, &p->d_mpart, 2 * (size_t)kMacroGridMax);
  if (!rc) rc = dev_alloc(p, &p->d_macro_iters, 1);
  if (!rc) rc = dev_alloc(p, &p->d_macro_resid, 1);
  return rc;
}

extern "C" int mch_macro_diagnostics(const mch_plan* p, int32_t* iters, double* resid) {
  if (!p || !iters || !resid) return set_error(MCH_EINVAL, "null argument");
  if (!p->macro_done) return set_error(MCH_ESTALE, "no macroscopic solve has been issued");
  int rc = hip_check(hipSetDevice(p->device), "hipSetDevice");
  if (!rc) rc = hip_check(hipStreamSynchronize(p->macro_stream), "hipStreamSynchronize");
  if (!rc) rc = hip_check(hipMemcpy(iters, p->d_macro_iters, sizeof(int32_t), hipMemcpyDeviceToHost), "hipMemcpy");
  if (!rc) rc = hip_check(hipMemcpy(resid, p->d_macro_resid, sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
  if (rc) return rc;
  if (!std::isfinite(*resid) || (*iters >= p->macro_max_iter && !(*resid <= p->macro_rtol)))
    return set_error(MCH_ENOCONV, "the macroscopic solve reached max_iter before rtol");
  return MCH_OK;
}

extern "C" int mch_build_interp(const mch_config* cfg, int32_t* nbr, double* weight) {
  g_last_error.clear();
  if (!cfg || !nbr || !weight) return set_error(MCH_EINVAL, "null argument");
  const mch_config& c = *cfg;
  if (c.dim != 2 && c.dim != 3) return set_error(MCH_EINVAL, "dim must be 2 or 3");
  const int nm = c.n_macro[0];
  for (int a = 0; a < c.dim; ++a)
    if (c.n_macro[a] != nm) return set_error(MCH_EINVAL, "n_macro must be equal on every axis");
  if (nm < 1 || c.levels < 1 || c.levels > MAX_LEVELS || c.eta < 1)
    return set_error(MCH_EINVAL, "bad n_macro, levels or eta");
  if (nm % ipow(c.eta, c.levels - 1) != 0) return set_error(MCH_EINVAL, "n_macro must be divisible by eta^(L-1)");
  mch_plan tmp;
  tmp.cfg = c;
  tmp.dim = c.dim;
  tmp.nm = nm;
  tmp.L = c.levels;
  tmp.P = ipow(nm, c.dim);
  build_hierarchy(&tmp);
  build_interp(&tmp);
  std::memcpy(nbr, tmp.nbr.data(), sizeof(int32_t) * tmp.nbr.size());
  std::memcpy(weight, tmp.nbw.data(), sizeof(double) * tmp.nbw.size());
  return MCH_OK;
}

extern "C" int mch_plan_info(const mch_plan* p, int64_t* info) {
  if (!p || !info) return set_error(MCH_EINVAL, "null argument");
  for (int k = 0; k < 4 + 3 * MAX_LEVELS; ++k) info[k] = 0;
  info[0] = p->P;
  info[1] = p->M;
  info[2] = p->m;
  info[3] = p->L;
  for (int l = 0; l < p->L; ++l) {
    info[4 + l] = p->lev[l].count;
    info[4 + p->L + l] = p->lev[l].shape.rpt;
    info[4 + 2 * p->L + l] = p->lev[l].shape.pre ? p->lev[l].shape.sb : 0;
  }
  return MCH_OK;
}

extern "C" int mch_hierarchy(const mch_plan* p, int32_t* level, int32_t* parent) {
  if (!p || !level || !parent) return set_error(MCH_EINVAL, "null argument");
  std::memcpy(level, p->level.data(), sizeof(int32_t) * p->P);
  std::memcpy(parent, p->parent.data(), sizeof(int32_t) * p->P);
  return MCH_OK;
}

static int diagnostics_impl(const mch_plan* p, int32_t* iters, double* resid, bool adjoint) {
  if (!p || !iters || !resid) return set_error(MCH_EINVAL, "null argument");
  if (!p->forward_done) return set_error(MCH_ESTALE, "no forward solve has been issued on this plan");
  int rc = hip_check(hipSetDevice(p->device), "hipSetDevice");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(p->last_stream), "hipStreamSynchronize");
  if (rc) return rc;
  long long bad[kValidateBlocks];
  rc = hip_check(hipMemcpy(bad, p->d_bad, sizeof(bad), hipMemcpyDeviceToHost), "hipMemcpy");
  if (rc) return rc;
  long long first = -1;
  for (long long b : bad)
    if (b >= 0 && (first < 0 || b < first)) first = b;
  if (first >= 0)
    return set_error(MCH_EINVAL, "kappa must be positive and finite and labels below n_cont; first offending "
                                 "fine element " + std::to_string(first));
  size_t cnt = (size_t)p->P * p->M;
  rc = hip_check(hipMemcpy(iters, adjoint ? p->d_iters_adj : p->d_iters, cnt * sizeof(int32_t), hipMemcpyDeviceToHost),
                 "hipMemcpy");
  if (rc) return rc;
  rc = hip_check(hipMemcpy(resid, adjoint ? p->d_resid_adj : p->d_resid, cnt * sizeof(double), hipMemcpyDeviceToHost),
                 "hipMemcpy");
  if (rc) return rc;
  return mch_classify_solves(iters, resid, (int64_t)cnt, p->cfg.max_iter, p->cfg.rtol);
}

extern "C" int mch_classify_solves(const int32_t* iters, const double* resid, int64_t n, int32_t max_iter,
                                   double rtol) {
  if (n < 0 || (n > 0 && (!iters || !resid))) return set_error(MCH_EINVAL, "bad solve record arrays");
  for (int64_t k = 0; k < n; ++k) {
    if (iters[k] < 0)
      return set_error(MCH_ESINGULAR, "singular constraint Schur matrix in a cell (solve " + std::to_string(k) + ")");
  }
  for (int64_t k = 0; k < n; ++k) {
    // a solve whose recurrence turned non-finite reports resid NaN
    if (!std::isfinite(resid[k]) || (iters[k] >= max_iter && !(resid[k] <= rtol)))
      return set_error(MCH_ENOCONV, "a cell solve reached max_iter before rtol or its residual is not finite "
                                    "(solve " + std::to_string(k) + ")");
  }
  return MCH_OK;
}

extern "C" int mch_diagnostics(const mch_plan* p, int32_t* iters, double* resid) {
  return diagnostics_impl(p, iters, resid, false);
}

extern "C" int mch_adjoint_diagnostics(const mch_plan* p, int32_t* iters, double* resid) {
  return diagnostics_impl(p, iters, resid, true);
}

extern "C" int mch_profile(mch_plan* p, int32_t mode) {
  if (!p) return set_error(MCH_EINVAL, "null plan");
  if (mode == 0 || mode == 1) p->profiling = mode;
  p->prof_used = 0;
  return MCH_OK;
}

extern "C" int mch_profile_read(mch_plan* p, int32_t idx, char* name, int32_t cap, double* ms) {
  if (!p) return set_error(MCH_EINVAL, "null plan");
  const int count = (int)p->prof_used;
  if (idx < 0) return count;
  if (idx >= count || !name || cap < 1 || !ms) return set_error(MCH_EINVAL, "bad profile record request");
  ProfRec& r = p->prof[idx];
  int rc = hip_check(hipEventSynchronize(r.stop), "hipEventSynchronize");
  if (rc) return rc;
  float t = 0.0f;
  rc = hip_check(hipEventElapsedTime(&t, r.start, r.stop), "hipEventElapsedTime");
  if (rc) return rc;
  *ms = t;
  std::snprintf(name, (size_t)cap, "%s", r.name.c_str());
  return count;
}
