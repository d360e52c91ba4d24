// Host side of the DP-SE library: parameter derivation and validation,
// plan tables and workspace, and the stage sequence of one solve
// (Sec. 5.2.2 steps 1-7 of the paper plus the near field of Sec. 4.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <utility>
#include <vector>

#include "dpse_internal.h"

using dpse::Geom;

namespace {

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Owner records of the workspaces: for every workspace base (a plan's own
// workspace or an arena shared by several plans), the plan and full solve
// whose far field (far4, the gauge constant, the wall partials) it holds.
// dpse_solve_near reuses that far field only if the record names the
// calling plan's own last full solve.
std::atomic<uint64_t> g_next_uid{1};
std::mutex g_owner_mu;
std::unordered_map<const void*, std::pair<uint64_t, uint64_t>> g_owner;

void note_full_solve(dpse_plan* p, int64_t n) {
  p->far_n = n;
  ++p->full_solves;
  std::lock_guard<std::mutex> lk(g_owner_mu);
  g_owner[(const void*)p->w.status] = {p->uid, p->full_solves};
}

// Static device scratch of dpse_solve_static: the workspace of callers that
// cannot allocate. Each device holds its own copy of the array from the
// first load of the library's code on it until the process ends; host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in), only the device address looked up once per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::unordered_map<int, void*> g_scratch;

// Looks up this device's address of the scratch array (the device must be
// current); once per device.
hipError_t scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch.count(device)) return hipSuccess;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (ptr == nullptr) return hipErrorInvalidSymbol;
  g_scratch[device] = ptr;
  return hipSuccess;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(device);
  return it == g_scratch.end() ? nullptr : it->second;
}

bool owns_far_field(const dpse_plan* p) {
  std::lock_guard<std::mutex> lk(g_owner_mu);
  auto it = g_owner.find((const void*)p->w.status);
  return it != g_owner.end() && it->second.first == p->uid && it->second.second == p->full_solves;
}

// d/dr of [erf(r/a) - erf(r/b)]/r with a = sqrt2 g_w (a = 0: the term is 1/r)
// and b = sqrt(2 g_w^2 + xi^-2) (b absent when xi = 0): eq. Gnear without the
// 1/(4 pi eps) factor.
double dgnear(double r, double g_w, double xi) {
  auto term = [](double rr, double s) {
    if (s == 0.0) return -1.0 / (rr * rr);
    double u = rr / s;
    return 2.0 / std::sqrt(dpse::kPi) * std::exp(-u * u) / (s * rr) - std::erf(u) / (rr * rr);
  };
  double t1 = term(r, std::sqrt(2.0) * g_w);
  if (xi == 0.0) return t1;
  return t1 - term(r, std::sqrt(2.0 * g_w * g_w + 1.0 / (xi * xi)));
}

// Smallest r with |dG(r; g_w, xi) / dG(r; g_w, 0)| < delta (eq. rnf).
double derive_rnf(double g_w, double xi, double delta) {
  auto ratio = [&](double r) { return std::fabs(dgnear(r, g_w, xi) / dgnear(r, g_w, 0.0)); };
  double step = 0.01 / xi, r = 1e-6 / xi;
  while (ratio(r) >= delta) {
    r += step;
    if (r > 100.0 / xi) return -1.0;
  }
  double lo = r - step, hi = r;
  for (int it = 0; it < 100; ++it) {
    double mid = 0.5 * (lo + hi);
    if (ratio(mid) < delta) hi = mid; else lo = mid;
  }
  return hi;
}

int derive_all(const dpse_params* p, dpse_info* info, Geom* g) {
  if (!p || !info) return DPSE_EINVAL;
  auto pos_finite = [](double v) { return std::isfinite(v) && v > 0.0; };
  if (!pos_finite(p->Lx) || !pos_finite(p->Ly) || !pos_finite(p->H) || !pos_finite(p->eps) ||
      !pos_finite(p->eps_bottom) || !pos_finite(p->eps_top) || !pos_finite(p->xi))
    return DPSE_EINVAL;
  if (!std::isfinite(p->g_w) || p->g_w < 0.0) return DPSE_EINVAL;
  if (!is_pow2(p->Nx) || !is_pow2(p->Ny) || p->Nx < 32 || p->Ny < 32 || p->Nx > 1024 || p->Ny > 1024)
    return DPSE_EINVAL;
  if (p->flags & ~(DPSE_GAUGE_NONE | DPSE_KMAX_GT | DPSE_UNIFORM_FAST | DPSE_ONE_JUMP | DPSE_TRIPLY |
                   DPSE_DETERMINISTIC))
    return DPSE_EINVAL;
  const bool tp = (p->flags & DPSE_TRIPLY) != 0;
  if (tp ? (p->Nz < 32 || !is_pow2(p->Nz) || p->Nz > 1024) : (p->Nz < 33 || !is_pow2(p->Nz - 1) || p->Nz - 1 > 1024))
    return DPSE_EINVAL;
  if (p->precision != DPSE_FP64 && p->precision != DPSE_MIXED) return DPSE_EINVAL;
  const bool uniform = (p->flags & DPSE_UNIFORM_FAST) != 0;
  const bool one = (p->flags & DPSE_ONE_JUMP) != 0;
  if (uniform && one) return DPSE_EINVAL;
  if (tp && (uniform || one || p->eps_bottom != p->eps || p->eps_top != p->eps)) return DPSE_EINVAL;
  if (uniform && !(p->eps_bottom == p->eps && p->eps_top == p->eps)) return DPSE_EINVAL;
  const bool jump_b = p->eps_bottom != p->eps, jump_t = p->eps_top != p->eps;
  if (one && jump_b == jump_t) return DPSE_EINVAL;
  // the free-space solve (no wall group, no correction) serves both
  const bool fast = uniform || one;
  double h = p->Lx / p->Nx, hy = p->Ly / p->Ny;
  if (std::fabs(h - hy) > 1e-12 * h) return DPSE_EINVAL;
  double g_t = std::sqrt(1.0 / (4.0 * p->xi * p->xi) + p->g_w * p->g_w);
  if (!std::isfinite(g_t) || !(g_t > 0.0)) return DPSE_EINVAL;
  int ng = p->support;
  if (ng == 0) {
    const double half = std::ceil(4.3 * g_t / h);  // compared before it becomes an int
    if (!(half <= 0.5 * dpse::kMaxSupport)) return DPSE_EINVAL;
    ng = 2 * (int)half;
  }
  if (ng < 2 || (ng & 1) || ng > dpse::kMaxSupport) return DPSE_EINVAL;
  double H_E = ng * h / 2.0;
  double rc = p->r_cut;
  if (rc == 0.0) {
    double delta = p->delta > 0.0 ? p->delta : 1e-4;
    rc = derive_rnf(p->g_w, p->xi, delta);
    if (rc <= 0.0) return DPSE_EINVAL;
    rc += 4.0 * p->g_w;  // r_cut = r_nf + n_sigma g_w (Sec. 5.1)
  }
  if (!(rc > 0.0) || rc >= 0.5 * std::fmin(p->Lx, p->Ly)) return DPSE_EINVAL;
  if (tp && (rc >= 0.5 * p->H || p->H < 4.0 * H_E)) return DPSE_EINVAL;
  // position-independent necessary conditions of Sec. 4.2 / 5.3 (h_min <= H/2);
  // they concern the images, which the uniform-permittivity solver has none of
  if (!fast && !tp && (rc >= 1.5 * p->H || 2.0 * H_E >= 1.5 * p->H)) return DPSE_EINVAL;
  // Chebyshev domain: [-3 H_E, H + 3 H_E] with two jumps (Sec. 5.2.2); the
  // free-space solve (Sec. 3.1.1) needs only the span of the sources, and
  // with one jump of its images too
  double za = -3.0 * H_E, zb = p->H + 3.0 * H_E;
  if (uniform) {
    za = -H_E;
    zb = p->H + H_E;
  } else if (one) {
    za = jump_b ? -p->H - H_E : -H_E;
    zb = jump_b ? p->H + H_E : 2.0 * p->H + H_E;
  } else if (tp) {  // the uniform periodic nodes, z_c = (Nz - 1 - c) H / Nz
    za = 0.0;
    zb = p->H - p->H / p->Nz;
  }

  // z buckets of the spreading bins (width H_E / 2 over the span of the
  // charges and images): bounded so that the bin arrays stay small
  const double nzb_d = std::ceil((tp ? p->H + 2.0 * H_E : zb - za - 2.0 * H_E) / (0.5 * H_E)) + 1.0;
  if (!(nzb_d <= 16384.0)) return DPSE_EINVAL;

  std::memset(info, 0, sizeof(*info));
  info->h = h;
  info->g_t = g_t;
  info->H_E = H_E;
  info->n_sigma = H_E / g_t;
  info->z_lo = za;
  info->z_hi = zb;
  info->r_cut = rc;
  info->xi_e = 1.0 / std::sqrt(4.0 * p->g_w * p->g_w + 1.0 / (p->xi * p->xi));
  info->support = ng;
  info->n_modes = p->Ny * (p->Nx / 2 + 1);

  if (g) {
    std::memset(g, 0, sizeof(*g));
    g->Lx = p->Lx; g->Ly = p->Ly; g->H = p->H;
    g->eps = p->eps; g->eps_b = p->eps_bottom; g->eps_t = p->eps_top;
    g->xi = p->xi; g->g_w = p->g_w;
    g->h = h; g->inv_h = 1.0 / h; g->g_t = g_t; g->H_E = H_E;
    g->za = za; g->zb = zb;
    g->zc = 0.5 * (g->za + g->zb); g->zR = 0.5 * (g->zb - g->za);
    g->gamma_b = (p->eps - p->eps_bottom) / (p->eps + p->eps_bottom);
    g->gamma_t = (p->eps - p->eps_top) / (p->eps + p->eps_top);
    g->tau_b = 2.0 * p->eps / (p->eps_bottom + p->eps);
    g->tau_t = 2.0 * p->eps / (p->eps_top + p->eps);
    g->xi_e = info->xi_e;
    g->r_cut = rc;
    g->sbar_norm = std::pow(2.0 * dpse::kPi * g_t * g_t, -1.5);
    g->inv2g2 = 1.0 / (2.0 * g_t * g_t);
    g->zmin_ok = 4.0 * p->g_w;
    g->zmax_ok = p->H - 4.0 * p->g_w;
    g->Nx = p->Nx; g->Ny = p->Ny; g->Nz = p->Nz; g->nkx = p->Nx / 2 + 1;
    // the one-jump solver runs the free-space path of the uniform solver; the
    // triply periodic one has no groups, images, correction or gauge either
    g->ng = ng;
    g->flags = p->flags | (one ? DPSE_UNIFORM_FAST : 0) | (tp ? (DPSE_UNIFORM_FAST | DPSE_GAUGE_NONE) : 0);
    if (tp) {  // any height, wrapped into [0, H)
      g->zmin_ok = -HUGE_VAL;
      g->zmax_ok = HUGE_VAL;
    }
    g->B = std::min(dpse::kBin, std::min(p->Nx, p->Ny));
    g->nbx = p->Nx / g->B; g->nby = p->Ny / g->B;
    // z buckets of the particles (charges and images: centres within H_E of
    // the domain's interior)
    g->zb_lo = tp ? -H_E : za + H_E;  // periodic copies reach H_E beyond either end
    g->zb_w = 0.5 * H_E;
    g->nzb = (int)nzb_d;
    // cells per direction, clamped to [1, 1024] before the conversion to int
    auto cells = [](double len, double c) { return (int)std::fmax(1.0, std::fmin(1024.0, std::floor(len / c))); };
    g->ncx = cells(p->Lx, rc);
    g->ncy = cells(p->Ly, rc);
    g->ncz = cells(p->H, rc);
    g->cwx = p->Lx / g->ncx; g->cwy = p->Ly / g->ncy; g->cwz = p->H / g->ncz;
    // wall bands of psi_o*: the wall group's charges lie in 0 < z < 2 H_E or
    // H - 2 H_E < z < H and reach the nodes within H_E of them, so their
    // spread is non-zero only at H - 3 H_E < z_j < H + H_E (top) and
    // -H_E < z_j < 3 H_E (bottom); the bounds H + H_E and -H_E are kept
    // inclusive. Nodes descend with the index j.
    int N = p->Nz;
    int top_lo = N, top_end = 0, bot_begin = N, bot_end = 0;
    for (int j = 0; j < N; ++j) {
      double z = g->zc + g->zR * std::cos(dpse::kPi * j / (N - 1));
      if (z > p->H - 3.0 * H_E && z <= p->H + H_E) {
        top_lo = std::min(top_lo, j);
        top_end = j + 1;
      }
      if (z < 3.0 * H_E && z >= -H_E) {
        bot_begin = std::min(bot_begin, j);
        bot_end = j + 1;
      }
    }
    if (fast || tp || top_end == 0 || bot_end == 0) {  // one group: no wall band
      top_lo = top_end = 0;
      bot_begin = bot_end = N;
    }
    g->top_lo = top_lo;
    g->top_end = top_end;
    g->bot_begin = bot_begin;
    g->bot_end = bot_end;
  }
  return DPSE_OK;
}

// Carves 256-byte aligned sub-buffers out of one allocation: with base ==
// nullptr it only accumulates the size.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  void take(T** ptr, size_t count) {
    off = (off + 255) & ~size_t(255);
    if (base) *ptr = reinterpret_cast<T*>(base + off);
    off += std::max<size_t>(count, 1) * sizeof(T);
  }
};

void plan_sizes(dpse_plan* p) {
  const Geom& g = p->g;
  p->nkeys = g.nbx * g.nby * g.nzb;
  p->ncells = g.ncx * g.ncy * g.ncz;
  p->npartials = 1024;
}

// Workspace of one solve (all per-solve device buffers), for max_n charges.
size_t carve_workspace(dpse_plan* p, char* base) {
  const Geom& g = p->g;
  const size_t rs = p->prm.precision == DPSE_MIXED ? 4 : 8;
  const size_t G = (size_t)g.Nz * g.Ny * g.Nx;
  const size_t C = (size_t)g.Nz * g.Ny * g.nkx;
  const size_t max_n = (size_t)p->max_n;
  Carver c{base};
  dpse::Workspace& w = p->w;
  // the status word first: at the same place for every plan bound to an
  // arena, whatever its sizes, so that plans sharing the arena share it
  c.take(&w.status, 4);
  size_t next = 3 * max_n;
  c.take(&w.ext, next); c.take(&w.ext_meta, next); c.take(&w.srt, next); c.take(&w.srt_meta, next);
  c.take(&w.bin_cnt, p->nkeys + 1); c.take(&w.bin_off, p->nkeys + 1); c.take(&w.bin_cur, p->nkeys + 1);
  c.take(&w.n_img, 4);
  c.take(&w.nsrt, max_n); c.take(&w.nsrt_idx, max_n);
  c.take(&w.cell_cnt, p->ncells + 1); c.take(&w.cell_off, p->ncells + 1); c.take(&w.cell_cur, p->ncells + 1);
  c.take((char**)&w.f_i, G * rs);
  c.take((char**)&w.f_o, G * rs);
  char** cgrids[] = {(char**)&w.fx_i, (char**)&w.fx_o, (char**)&w.psi, (char**)&w.psiz,
                     (char**)&w.p0, (char**)&w.py, (char**)&w.pz};
  for (char** gp : cgrids) c.take(gp, C * 2 * rs);
  c.take((char**)&w.u4, 4 * G * rs);
  c.take(&w.far4, max_n); c.take(&w.near4, max_n);
  // partials: near part at the origin, finalize, far part at the origin per
  // node (two blocks of npartials: Nz <= 2 npartials), wall energy
  c.take(&w.scal, 16); c.take(&w.partials, 5 * (size_t)p->npartials);
  c.take(&w.qpart, 2 * ((max_n + 255) / 256));
  c.take(&w.scan_bin, 3 * (size_t)(dpse::scan_blocks(p->nkeys) + 1));
  c.take(&w.scan_cell, 3 * (size_t)(dpse::scan_blocks(p->ncells) + 1));
  return (c.off + 255) & ~size_t(255);
}

size_t carve_tables(dpse_plan* p, char* base) {
  const Geom& g = p->g;
  Carver c{base};
  dpse::Tables& t = p->t;
  c.take(&t.z, g.Nz); c.take(&t.wq, g.Nz); c.take(&t.T0, g.Nz); c.take(&t.TH, g.Nz);
  c.take(&t.dT0, g.Nz); c.take(&t.dTH, g.Nz);
  c.take(&t.twx, g.Nx / 2); c.take(&t.twy, g.Ny / 2); c.take(&t.twz, g.Nz - 1);
  c.take(&t.twx_f, g.Nx / 2); c.take(&t.twy_f, g.Ny / 2);
  c.take(&t.ctab, dpse::kCtabRows * g.Nz + dpse::kNumFun * (g.Nz + 2));
  c.take(&t.cpiv, (size_t)g.Nz * g.Ny * g.nkx);
  c.take(&t.hfun, 16 * (size_t)g.Ny * g.nkx);
  return c.off;
}

void free_all(dpse_plan* p) {
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  p->graph_exec = nullptr;
  if (p->side) (void)hipStreamSynchronize(p->side);
  if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
  if (p->join_ev) (void)hipEventDestroy(p->join_ev);
  if (p->side) (void)hipStreamDestroy(p->side);
  p->side = nullptr;
  p->fork_ev = p->join_ev = nullptr;
  for (void* a : p->allocs) (void)hipFree(a);
  p->allocs.clear();
}

// Chebyshev T_n(s) and T_n'(s) for n < N by the three-term recurrences.
void cheb_table(int N, long double s, std::vector<double>& T, std::vector<double>& dT) {
  T.assign(N, 0.0);
  dT.assign(N, 0.0);
  long double t0 = 1.0L, t1 = s, u0 = 1.0L, u1 = 2.0L * s;  // U_{n-1} for T_n' = n U_{n-1}
  for (int n = 0; n < N; ++n) {
    long double tn = (n == 0) ? 1.0L : (n == 1 ? s : 0.0L);
    if (n >= 2) {
      tn = 2.0L * s * t1 - t0;
      t0 = t1;
      t1 = tn;
    }
    T[n] = (double)((n == 0) ? 1.0L : (n == 1 ? s : tn));
    long double un1;  // U_{n-1}
    if (n == 0) un1 = 0.0L;
    else if (n == 1) un1 = 1.0L;
    else if (n == 2) un1 = u1;
    else {
      long double un = 2.0L * s * u1 - u0;
      u0 = u1;
      u1 = un;
      un1 = un;
    }
    dT[n] = (double)(n * un1);
  }
}

}  // namespace

extern "C" {

const char* dpse_status_string(int s) {
  switch (s) {
    case DPSE_OK: return "ok";
    case DPSE_EINVAL: return "invalid argument or parameters";
    case DPSE_ENOMEM: return "device allocation failed";
    case DPSE_EHIP: return "HIP runtime error";
    case DPSE_ENONNEUTRAL: return "charges are not neutral";
    case DPSE_EOUTSIDE: return "charge outside the slab or non-finite coordinate";
    case DPSE_ECONSTRAINT: return "near-field or far-field image constraint violated (Sec. 5.3)";
    case DPSE_ETOOMANY: return "more charges than the plan's max_n";
    case DPSE_ESCRATCH: return "the plan's workspace is larger than the static scratch buffer (64 MiB)";
    default: return "unknown status";
  }
}

int dpse_derive(const dpse_params* params, dpse_info* info) {
  dpse_info tmp;
  int s = derive_all(params, &tmp, nullptr);
  if (s == DPSE_OK) *info = tmp;
  return s;
}

static int plan_create(const dpse_params* params, int64_t max_n, void* stream, dpse_plan** out,
                       bool unbound) {
  if (!out || max_n <= 0 || max_n > (int64_t(1) << 28)) return DPSE_EINVAL;
  dpse_plan* p = new (std::nothrow) dpse_plan();
  if (!p) return DPSE_ENOMEM;
  int s = derive_all(params, &p->info, &p->g);
  if (s != DPSE_OK) {
    delete p;
    return s;
  }
  p->prm = *params;
  p->stream = (hipStream_t)stream;
  p->max_n = max_n;
  p->uid = g_next_uid.fetch_add(1);
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return DPSE_EHIP;
  }
  const Geom& g = p->g;
  plan_sizes(p);
  hipError_t e = hipSuccess;
  void* tbl = nullptr;
  size_t tbytes = carve_tables(p, nullptr);
  e = hipMalloc(&tbl, tbytes);
  if (e != hipSuccess) {
    delete p;
    return DPSE_ENOMEM;
  }
  p->allocs.push_back(tbl);
  carve_tables(p, (char*)tbl);
  dpse::Workspace& w = p->w;
  dpse::Tables& t = p->t;
  size_t wbytes = carve_workspace(p, nullptr);
  if (!unbound) {
    void* ws = nullptr;
    e = hipMalloc(&ws, wbytes);
    if (e != hipSuccess) {
      free_all(p);
      delete p;
      return DPSE_ENOMEM;
    }
    p->allocs.push_back(ws);
    carve_workspace(p, (char*)ws);
    p->bound = true;
    p->owns_workspace = true;
  }
  p->info.workspace_bytes = (int64_t)wbytes;
  p->info.table_bytes = (int64_t)tbytes;
  p->info.max_n = max_n;

  // plan tables
  const int N = g.Nz;
  std::vector<double> z(N), wq(N);
  const int nint = N - 1;
  for (int j = 0; j < N; ++j) {
    long double th = (long double)dpse::kPi * j / nint;
    z[j] = (double)(g.zc + g.zR * std::cos(th));
    // Clenshaw-Curtis weight on [-1,1] (cosine-series form), scaled by R and h^2
    long double acc = 1.0L;
    for (int k = 1; k <= nint / 2; ++k) {
      long double b = (2 * k == nint) ? 1.0L : 2.0L;
      acc -= b / (4.0L * k * k - 1.0L) * std::cos(2.0L * (long double)dpse::kPi * j * k / nint);
    }
    long double c = (j == 0 || j == nint) ? 1.0L : 2.0L;
    wq[j] = (double)(c / nint * acc * g.zR * g.h * g.h);
  }
  const bool tp = (g.flags & DPSE_TRIPLY) != 0;
  if (tp) {  // uniform periodic nodes, descending like the Chebyshev ones; weight h^2 h_z
    const double hz = g.H / N;
    for (int j = 0; j < N; ++j) {
      z[j] = (N - 1 - j) * hz;
      wq[j] = g.h * g.h * hz;
    }
  }
  std::vector<double> T0, dT0, TH, dTH;
  cheb_table(N, ((long double)0.0 - g.zc) / g.zR, T0, dT0);
  cheb_table(N, ((long double)g.H - g.zc) / g.zR, TH, dTH);
  for (int n = 0; n < N; ++n) {
    dT0[n] /= g.zR;
    dTH[n] /= g.zR;
  }
  // Per-mode solver tables. With u = (y''_0..y''_{N-1}, y_0, y'_0), the
  // integral relations of App. A give y'_n = P[n] . u (eq. ds) and
  // y_n = Y[n] . u (eq. cs), with y''_n = 0 for n > N-1 and y'_N = 0.
  const int NU = N + 2;
  std::vector<long double> Pm((size_t)N * NU, 0.0L), Ym((size_t)N * NU, 0.0L);
  auto Pr = [&](int n) { return &Pm[(size_t)n * NU]; };
  auto Yr = [&](int n) { return &Ym[(size_t)n * NU]; };
  Pr(0)[N + 1] = 1.0L;
  Pr(1)[0] = 1.0L;
  Pr(1)[2] = -0.5L;
  for (int n = 2; n < N; ++n) {
    Pr(n)[n - 1] = 1.0L / (2.0L * n);
    if (n + 1 < N) Pr(n)[n + 1] = -1.0L / (2.0L * n);
  }
  Yr(0)[N] = 1.0L;
  for (int j = 0; j < NU; ++j) Yr(1)[j] = Pr(0)[j] - 0.5L * Pr(2)[j];
  for (int n = 2; n < N; ++n)
    for (int j = 0; j < NU; ++j)
      Yr(n)[j] = (Pr(n - 1)[j] - (n + 1 < N ? Pr(n + 1)[j] : 0.0L)) / (2.0L * n);
  std::vector<double> ctab((size_t)dpse::kCtabRows * N + (size_t)dpse::kNumFun * NU, 0.0);
  for (int n = 0; n < N; ++n) {
    // mode equation n: y''_n - kappa^2 y_n = g_n, y_n = a y''_{n-2} - b y''_n + c y''_{n+2} (+ free constants)
    ctab[n] = n >= 2 ? (double)Yr(n)[n - 2] : 0.0;
    ctab[N + n] = n >= 1 ? (double)(-Yr(n)[n]) : 0.0;
    ctab[2 * N + n] = (n >= 1 && n + 2 < N) ? (double)Yr(n)[n + 2] : 0.0;
    // g_n = -R^2/eps * fhat_n, fhat_n = DCT-I_n / ((N-1) cbar_n), cbar = 2 at both ends
    ctab[3 * N + n] = -(g.zR * g.zR) / (g.eps * (N - 1)) * ((n == 0 || n == N - 1) ? 0.5 : 1.0);
  }
  {
    double* W = ctab.data() + (size_t)dpse::kCtabRows * N;
    for (int n = 0; n < N; ++n) {
      long double sg = (n & 1) ? -1.0L : 1.0L;
      long double n2 = (long double)n * n / g.zR;
      const long double fy[dpse::kNumFun] = {0.0L, 1.0L, 0.0L, sg, T0[n], TH[n], dT0[n], dTH[n], -sg * n2, n2};
      const long double fp[dpse::kNumFun] = {1.0L, 0.0L, sg, 0.0L, 0, 0, 0, 0, 0, 0};
      for (int f = 0; f < dpse::kNumFun; ++f)
        for (int j = 0; j < NU; ++j)
          W[(size_t)f * NU + j] += (double)(fy[f] * Yr(n)[j] + fp[f] * Pr(n)[j]);
    }
  }
  auto twid = [](int L) {
    std::vector<double2> tw(std::max(L / 2, 1));
    for (int k = 0; k < L / 2; ++k) {
      long double a = -2.0L * (long double)dpse::kPi * k / L;
      tw[k] = make_double2((double)std::cos(a), (double)std::sin(a));
    }
    return tw;
  };
  // z twiddles: the DCT's even extension (length 2(Nz - 1)), or the periodic z transform (length Nz)
  auto tox = twid(g.Nx), toy = twid(g.Ny), toz = twid(tp ? N : 2 * (N - 1));
  std::vector<float2> txf(tox.size()), tyf(toy.size());
  for (size_t i = 0; i < tox.size(); ++i) txf[i] = make_float2((float)tox[i].x, (float)tox[i].y);
  for (size_t i = 0; i < toy.size(); ++i) tyf[i] = make_float2((float)toy[i].x, (float)toy[i].y);
  auto H2D = [&](void* dst, const void* src, size_t b) {
    if (e == hipSuccess) e = hipMemcpy(dst, src, b, hipMemcpyHostToDevice);
  };
  H2D(t.z, z.data(), N * 8); H2D(t.wq, wq.data(), N * 8);
  H2D(t.T0, T0.data(), N * 8); H2D(t.TH, TH.data(), N * 8);
  H2D(t.dT0, dT0.data(), N * 8); H2D(t.dTH, dTH.data(), N * 8);
  H2D(t.twx, tox.data(), tox.size() * sizeof(double2));
  H2D(t.twy, toy.data(), toy.size() * sizeof(double2));
  H2D(t.twz, toz.data(), toz.size() * sizeof(double2));
  H2D(t.ctab, ctab.data(), ctab.size() * sizeof(double));
  H2D(t.twx_f, txf.data(), txf.size() * sizeof(float2));
  H2D(t.twy_f, tyf.data(), tyf.size() * sizeof(float2));
  int zero4[4] = {0, 0, 0, 0};
  if (p->bound) H2D(w.status, zero4, sizeof(zero4));
  if (e == hipSuccess) e = dpse::prepare_kernels();
  if (e == hipSuccess) e = scratch_init(p->device);  // set-up of dpse_solve_static on this device
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming);
  // factorise the per-mode chains once (they depend on the plan only), on a
  // private stream so that work already queued on other streams is not waited for
  if (e == hipSuccess) {
    hipStream_t ps = nullptr;
    e = hipStreamCreateWithFlags(&ps, hipStreamNonBlocking);
    if (e == hipSuccess) e = dpse::launch_pivots(p, ps);
    if (e == hipSuccess) e = hipStreamSynchronize(ps);
    if (ps) (void)hipStreamDestroy(ps);
  }
  if (e != hipSuccess) {
    free_all(p);
    delete p;
    return DPSE_EHIP;
  }
  *out = p;
  return DPSE_OK;
}

int dpse_plan_create(const dpse_params* params, int64_t max_n, void* stream, dpse_plan** out) {
  return plan_create(params, max_n, stream, out, false);
}

int dpse_plan_create_unbound(const dpse_params* params, int64_t max_n, dpse_plan** out) {
  return plan_create(params, max_n, nullptr, out, true);
}

int dpse_workspace_size(const dpse_params* params, int64_t max_n, int64_t* bytes) {
  if (!params || !bytes || max_n <= 0 || max_n > (int64_t(1) << 28)) return DPSE_EINVAL;
  dpse_plan tmp;
  int s = derive_all(params, &tmp.info, &tmp.g);
  if (s != DPSE_OK) return s;
  tmp.prm = *params;
  tmp.max_n = max_n;
  plan_sizes(&tmp);
  *bytes = (int64_t)carve_workspace(&tmp, nullptr);
  return DPSE_OK;
}

int dpse_plan_bind(dpse_plan* p, void* workspace, int64_t bytes, void* stream) {
  if (!p || !workspace || bytes < p->info.workspace_bytes) return DPSE_EINVAL;
  if (((uintptr_t)workspace & 255) != 0) return DPSE_EINVAL;
  if (p->owns_workspace) return DPSE_EINVAL;  // created by dpse_plan_create
  if (hipSetDevice(p->device) != hipSuccess) return DPSE_EHIP;
  carve_workspace(p, (char*)workspace);
  p->stream = (hipStream_t)stream;
  p->bound = true;
  p->far_n = 0;
  if (p->graph_exec) {
    (void)hipGraphExecDestroy(p->graph_exec);
    p->graph_exec = nullptr;
  }
  hipError_t e = dpse::fill_int(p->w.status, 0, 4, p->stream);
  return e == hipSuccess ? DPSE_OK : DPSE_EHIP;
}

int dpse_plan_info(const dpse_plan* plan, dpse_info* info) {
  if (!plan || !info) return DPSE_EINVAL;
  *info = plan->info;
  return DPSE_OK;
}

static const char* kStageNames[DPSE_NUM_STAGES] = {
    "prep", "bin", "spread", "fft_forward", "column", "fft_inverse", "interp", "near", "gauge", "finalize"};

}  // extern "C"

// One solve: validation and images, the grid bins, spreading and forward
// transforms, then the cell list and the near field on the plan's side stream
// while the column solve and the remaining far-field stages run on the plan's
// stream, joined before the gauge constant and the outputs.
template <typename R>
static hipError_t solve_stages(dpse_plan* p, int64_t n, const double* pos, const double* q, double* energy,
                               double* phi, double* force, hipEvent_t* ev) {
  hipError_t e = hipSuccess;
  hipStream_t main = p->stream;
  auto start = [&](int st, hipStream_t s) {
    if (ev && e == hipSuccess) e = hipEventRecord(ev[2 * st], s);
  };
  auto end = [&](int st, hipStream_t s) {
    if (ev && e == hipSuccess) e = hipEventRecord(ev[2 * st + 1], s);
  };
  auto run = [&](hipError_t (*f)(dpse_plan*)) {
    if (e == hipSuccess) e = f(p);
  };
  p->wall_part = nullptr;  // set by whichever kernel forms the wall term
  p->wall_nparts = 0;
  start(0, main); if (e == hipSuccess) e = dpse::launch_prep(p, n, pos, q); end(0, main);
  // The near field (stage 7) and its part of the gauge go to the side stream.
  // In the FP32 path of the slab they are forked right after validation and
  // share the CUs with the grid binning, spreading and forward transforms;
  // in the FP64 path (whose near field is several times longer) and in the
  // triply periodic variant (whose column solve is short and near field
  // long) once the forward transforms are queued, beside the column solve.
  // Measured: large slab 14.2-14.5 -> 14.0 ms mixed with the early fork,
  // 24.0 -> 24.4 ms in FP64; triply periodic workload 0.42 -> 0.49 ms mixed.
  // Inside a graph capture they stay on the capturing stream (see
  // dpse_solve_graph).
  const bool fork = !p->capturing;
  hipStream_t ns = fork ? p->side : main;
  auto near_field = [&]() {
    if (fork && e == hipSuccess) e = hipEventRecord(p->fork_ev, main);
    if (fork && e == hipSuccess) e = hipStreamWaitEvent(p->side, p->fork_ev, 0);
    p->stream = ns;
    start(7, ns);
    if (e == hipSuccess) e = dpse::launch_bin_cells(p, n);  // only the near field needs the cell list
    if (e == hipSuccess) e = dpse::launch_near<R>(p, n);
    if (e == hipSuccess) e = dpse::launch_near_origin(p, n);
    end(7, ns);
    if (fork && e == hipSuccess) e = hipEventRecord(p->join_ev, p->side);
    p->stream = main;
  };
  const bool early_near = sizeof(R) == 4 && !(p->g.flags & DPSE_TRIPLY);
  if (early_near) near_field();
  start(1, main); if (e == hipSuccess) e = dpse::launch_bin_grid(p, n); end(1, main);
  start(2, main); run(dpse::launch_spread<R>); end(2, main);
  start(3, main); run(dpse::launch_fft_forward<R>); end(3, main);
  if (!early_near) near_field();
  start(4, main); run(dpse::launch_column<R>); end(4, main);
  start(5, main); run(dpse::launch_fft_inverse<R>); end(5, main);
  start(6, main); if (e == hipSuccess) e = dpse::launch_interp<R>(p, n); end(6, main);
  start(8, main);
  run(dpse::launch_gauge_far<R>);
  if (fork && e == hipSuccess) e = hipStreamWaitEvent(main, p->join_ev, 0);
  end(8, main);
  start(9, main);
  if (p->walls_on && energy && !p->wall_part && e == hipSuccess) e = dpse::launch_wall_energy<R>(p, n);
  if (e == hipSuccess) e = dpse::launch_finalize(p, n, q, energy, phi, force, true);  // forms the gauge constant first
  end(9, main);
  return e;
}

// Near-field-only solve: the far-field averages (far4), the gauge constant
// (scal[2]) and the wall-term partials of the last full solve stay as they are.
template <typename R>
static hipError_t solve_near_stages(dpse_plan* p, int64_t n, const double* pos, const double* q, double* energy,
                                    double* phi, double* force) {
  hipError_t e = dpse::launch_prep(p, n, pos, q);
  if (e == hipSuccess) e = dpse::launch_bin(p, n);
  if (e == hipSuccess) e = dpse::launch_near<R>(p, n);
  if (e == hipSuccess) e = dpse::launch_finalize(p, n, q, energy, phi, force, false);
  return e;
}

extern "C" {

static int solve_impl(dpse_plan* p, int64_t n, const double* pos, const double* q,
                      double* energy, double* phi, double* force, bool allow_timing = true) {
  if (!p || !pos || !q || n <= 0 || !p->bound) return DPSE_EINVAL;
  if (n > p->max_n) return DPSE_ETOOMANY;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
    if (hipSetDevice(p->device) != hipSuccess) return DPSE_EHIP;
  }
  p->last_n = n;
  hipEvent_t* ev = nullptr;
  if (p->timing && allow_timing) {
    size_t need = (size_t)(p->timed_solves + 1) * (2 * DPSE_NUM_STAGES);
    while (p->events.size() < need) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return DPSE_EHIP;
      p->events.push_back(e);
    }
    ev = p->events.data() + (size_t)p->timed_solves * (2 * DPSE_NUM_STAGES);
    p->timed_solves++;
  }
  hipError_t e = p->prm.precision == DPSE_MIXED ? solve_stages<float>(p, n, pos, q, energy, phi, force, ev)
                                                : solve_stages<double>(p, n, pos, q, energy, phi, force, ev);
  if (e == hipSuccess) note_full_solve(p, n);
  else p->far_n = 0;
  return e == hipSuccess ? DPSE_OK : DPSE_EHIP;
}

int dpse_solve_near(dpse_plan* p, int64_t n, const double* pos, const double* q, double* energy, double* phi,
                    double* force) {
  if (!p || !pos || !q || n <= 0 || !p->bound) return DPSE_EINVAL;
  if (n > p->max_n) return DPSE_ETOOMANY;
  // a full solve of these charges whose far field the workspace still holds
  // (no other plan has solved in a shared arena since)
  if (p->far_n != n || !owns_far_field(p)) return DPSE_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
    if (hipSetDevice(p->device) != hipSuccess) return DPSE_EHIP;
  }
  p->last_n = n;
  hipError_t e = p->prm.precision == DPSE_MIXED ? solve_near_stages<float>(p, n, pos, q, energy, phi, force)
                                                : solve_near_stages<double>(p, n, pos, q, energy, phi, force);
  return e == hipSuccess ? DPSE_OK : DPSE_EHIP;
}

int dpse_bd_step(dpse_plan* p, int64_t n, const double* pos, const double* force, const double* w_prev,
                 const double* w_next, double mu_dt, double noise, double* pos_out, int32_t* escaped) {
  if (!p || n <= 0 || !pos || !force || !w_prev || !w_next || !pos_out || !escaped || pos_out == pos)
    return DPSE_EINVAL;
  if (!std::isfinite(mu_dt) || !std::isfinite(noise) || mu_dt < 0.0 || noise < 0.0) return DPSE_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return DPSE_EHIP;
  return dpse::launch_bd_step(p, n, pos, force, w_prev, w_next, mu_dt, noise, pos_out, escaped) == hipSuccess
             ? DPSE_OK
             : DPSE_EHIP;
}

int dpse_solve(dpse_plan* plan, int64_t n, const double* pos, const double* q, double* energy,
               double* phi, double* force) {
  return solve_impl(plan, n, pos, q, energy, phi, force);
}

int dpse_solve_static(dpse_plan* p, void* stream, int64_t n, const double* pos, const double* q,
                      double* energy, double* phi, double* force) {
  if (!p || !pos || !q || n <= 0) return DPSE_EINVAL;
  if (p->owns_workspace) return DPSE_EINVAL;  // created by dpse_plan_create
  if (n > p->max_n) return DPSE_ETOOMANY;
  if (p->info.workspace_bytes > (int64_t)kScratchBytes) return DPSE_ESCRATCH;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
    if (hipSetDevice(p->device) != hipSuccess) return DPSE_EHIP;
  }
  void* base = scratch_ptr(p->device);  // looked up when the plan was created
  if (base == nullptr) return DPSE_EHIP;
  carve_workspace(p, (char*)base);
  p->stream = (hipStream_t)stream;
  p->bound = true;
  // the array keeps the last call's contents: the status word starts at zero
  // (a fill kernel, no memset node under capture); every other buffer a
  // solve reads is cleared or written by its own kernels first
  if (dpse::fill_int(p->w.status, 0, 4, p->stream) != hipSuccess) {
    p->far_n = 0;
    return DPSE_EHIP;
  }
  return solve_impl(p, n, pos, q, energy, phi, force, false);
}

int dpse_solve_graph(dpse_plan* p, int64_t n, const double* pos, const double* q, double* energy,
                     double* phi, double* force) {
  if (!p || !pos || !q || n <= 0 || !p->bound) return DPSE_EINVAL;
  if (n > p->max_n) return DPSE_ETOOMANY;
  const void* sig[8] = {(const void*)(intptr_t)n, pos, q, energy, phi, force, (const void*)p->w.ext,
                        (const void*)(intptr_t)(p->walls_on ? p->walls_version : -1)};
  bool same = p->graph_exec != nullptr && p->graph_stream == p->stream;
  for (int i = 0; i < 8 && same; ++i) same = p->graph_sig[i] == sig[i];
  if (!same) {
    if (p->graph_exec) {
      (void)hipGraphExecDestroy(p->graph_exec);
      p->graph_exec = nullptr;
    }
    hipStream_t cs = p->stream;
    bool own_stream = false;
    if (cs == nullptr) {  // the null stream cannot be captured: capture on a private stream
      if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return DPSE_EHIP;
      own_stream = true;
    }
    hipStream_t keep = p->stream;
    bool timing = p->timing;
    p->stream = cs;
    p->timing = false;
    p->capturing = true;
    hipGraph_t graph = nullptr;
    int st = DPSE_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = DPSE_EHIP;
    if (st == DPSE_OK) st = solve_impl(p, n, pos, q, energy, phi, force);
    hipError_t ec = hipStreamEndCapture(cs, &graph);
    p->stream = keep;
    p->timing = timing;
    p->capturing = false;
    if (own_stream) (void)hipStreamDestroy(cs);
    if (st != DPSE_OK || ec != hipSuccess || graph == nullptr) {
      if (graph) (void)hipGraphDestroy(graph);
      return st != DPSE_OK ? st : DPSE_EHIP;
    }
    hipError_t ei = hipGraphInstantiate(&p->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      p->graph_exec = nullptr;
      return DPSE_EHIP;
    }
    for (int i = 0; i < 8; ++i) p->graph_sig[i] = sig[i];
    p->graph_stream = p->stream;
  }
  p->last_n = n;
  if (hipGraphLaunch(p->graph_exec, p->stream) != hipSuccess) {
    p->far_n = 0;
    return DPSE_EHIP;
  }
  note_full_solve(p, n);
  return DPSE_OK;
}

struct dpse_graph {
  hipGraphExec_t exec = nullptr;
  int device = 0;
  // the systems in capture order: a launch makes each plan the owner of its
  // workspace's far field again (the last system of a shared arena wins)
  std::vector<std::pair<dpse_plan*, int64_t>> systems;
};

int dpse_batch_graph_create(int n_sys, dpse_plan* const* plans, const int64_t* n,
                            const double* const* pos, const double* const* q,
                            double* const* energy, double* const* phi, double* const* force,
                            const int32_t* branch, int n_branches, dpse_graph** out) {
  if (!out || n_sys <= 0 || !plans || !n || !pos || !q || n_branches <= 0 || n_branches > 64)
    return DPSE_EINVAL;
  for (int i = 0; i < n_sys; ++i) {
    if (!plans[i] || !plans[i]->bound || n[i] <= 0 || !pos[i] || !q[i]) return DPSE_EINVAL;
    if (n[i] > plans[i]->max_n) return DPSE_ETOOMANY;
    if (branch && (branch[i] < 0 || branch[i] >= n_branches)) return DPSE_EINVAL;
  }
  std::vector<hipStream_t> st(n_branches + 1, nullptr);
  std::vector<hipEvent_t> ev(n_branches + 1, nullptr);
  int status = DPSE_OK;
  for (int b = 0; b <= n_branches && status == DPSE_OK; ++b) {
    if (hipStreamCreateWithFlags(&st[b], hipStreamNonBlocking) != hipSuccess) status = DPSE_EHIP;
    else if (hipEventCreateWithFlags(&ev[b], hipEventDisableTiming) != hipSuccess) status = DPSE_EHIP;
  }
  hipGraph_t graph = nullptr;
  hipStream_t root = st[n_branches];
  bool capturing = false;
  if (status == DPSE_OK) {
    if (hipStreamBeginCapture(root, hipStreamCaptureModeThreadLocal) != hipSuccess) status = DPSE_EHIP;
    else capturing = true;
  }
  // fork: every branch stream joins the capture through an event of the root
  if (status == DPSE_OK && hipEventRecord(ev[n_branches], root) != hipSuccess) status = DPSE_EHIP;
  for (int b = 0; b < n_branches && status == DPSE_OK; ++b)
    if (hipStreamWaitEvent(st[b], ev[n_branches], 0) != hipSuccess) status = DPSE_EHIP;
  for (int i = 0; i < n_sys && status == DPSE_OK; ++i) {
    dpse_plan* p = plans[i];
    const int b = branch ? branch[i] : i % n_branches;
    hipStream_t keep = p->stream;
    bool timing = p->timing;
    p->stream = st[b];
    p->timing = false;
    p->capturing = true;
    status = solve_impl(p, n[i], pos[i], q[i], energy ? energy[i] : nullptr, phi ? phi[i] : nullptr,
                        force ? force[i] : nullptr);
    p->stream = keep;
    p->timing = timing;
    p->capturing = false;
  }
  // join
  for (int b = 0; b < n_branches && status == DPSE_OK; ++b) {
    if (hipEventRecord(ev[b], st[b]) != hipSuccess || hipStreamWaitEvent(root, ev[b], 0) != hipSuccess)
      status = DPSE_EHIP;
  }
  if (capturing) {
    hipError_t ec = hipStreamEndCapture(root, &graph);
    if (status == DPSE_OK && ec != hipSuccess) status = DPSE_EHIP;
  }
  dpse_graph* gr = nullptr;
  if (status == DPSE_OK && graph) {
    gr = new (std::nothrow) dpse_graph();
    if (!gr) status = DPSE_ENOMEM;
    else if (hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0) != hipSuccess) status = DPSE_EHIP;
    if (gr) {
      gr->device = plans[0]->device;
      for (int i = 0; i < n_sys; ++i) gr->systems.emplace_back(plans[i], n[i]);
    }
  }
  if (graph) (void)hipGraphDestroy(graph);
  for (int b = 0; b <= n_branches; ++b) {
    if (ev[b]) (void)hipEventDestroy(ev[b]);
    if (st[b]) (void)hipStreamDestroy(st[b]);
  }
  if (status != DPSE_OK) {
    if (gr && gr->exec) (void)hipGraphExecDestroy(gr->exec);
    delete gr;
    return status;
  }
  *out = gr;
  return DPSE_OK;
}

int dpse_graph_launch(dpse_graph* g, void* stream) {
  if (!g || !g->exec) return DPSE_EINVAL;
  if (hipGraphLaunch(g->exec, (hipStream_t)stream) != hipSuccess) return DPSE_EHIP;
  for (auto& s : g->systems) note_full_solve(s.first, s.second);
  return DPSE_OK;
}

int dpse_graph_destroy(dpse_graph* g) {
  if (!g) return DPSE_EINVAL;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  delete g;
  return DPSE_OK;
}

int dpse_solve_batch(int n_sys, dpse_plan* const* plans, const int64_t* n,
                     const double* const* pos, const double* const* q, double* const* energy,
                     double* const* phi, double* const* force) {
  if (n_sys <= 0 || !plans || !n || !pos || !q) return DPSE_EINVAL;
  for (int i = 0; i < n_sys; ++i) {
    if (!plans[i]) return DPSE_EINVAL;
    if (n[i] <= 0) return DPSE_EINVAL;
    if (n[i] > plans[i]->max_n) return DPSE_ETOOMANY;
  }
  // Each solve is independent. Solves of plans on stream 0 (the first plan's)
  // run in order on it; the others run on their own streams, and stream 0
  // waits for each of them through an event, so that the whole batch is done
  // when stream 0's work is. The events are released on every return.
  hipStream_t s0 = plans[0]->stream;
  std::vector<hipEvent_t> done;
  int status = DPSE_OK;
  for (int i = 0; i < n_sys && status == DPSE_OK; ++i) {
    status = solve_impl(plans[i], n[i], pos[i], q[i], energy ? energy[i] : nullptr,
                        phi ? phi[i] : nullptr, force ? force[i] : nullptr);
    if (status != DPSE_OK || plans[i]->stream == s0) continue;
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      status = DPSE_EHIP;
      break;
    }
    done.push_back(ev);
    if (hipEventRecord(ev, plans[i]->stream) != hipSuccess || hipStreamWaitEvent(s0, ev, 0) != hipSuccess)
      status = DPSE_EHIP;
  }
  for (hipEvent_t d : done) (void)hipEventDestroy(d);
  return status;
}

// Tuned launch shapes: stage 0 spreading tiles, 1 interpolation tiles, 2
// column-kernel blocks.
static int tuned_count(int s) { return s < 2 ? dpse::tile_candidates(s) : dpse::column_candidates(); }

static bool tuned_valid(const dpse_plan* p, int s, int i) {
  const bool fp64 = p->prm.precision != DPSE_MIXED;
  return s < 2 ? dpse::tile_valid(p->g, s, i, fp64) : dpse::column_valid(p->g, i);
}

static int& tuned_cfg(dpse_plan* p, int s) {
  return s == 0 ? p->spread_cfg : (s == 1 ? p->interp_cfg : p->column_cfg);
}

static hipError_t launch_tuned(dpse_plan* p, int s, int64_t n) {
  const bool fp64 = p->prm.precision != DPSE_MIXED;
  if (s == 0) return fp64 ? dpse::launch_spread<double>(p) : dpse::launch_spread<float>(p);
  if (s == 1) return fp64 ? dpse::launch_interp<double>(p, n) : dpse::launch_interp<float>(p, n);
  return fp64 ? dpse::launch_column<double>(p) : dpse::launch_column<float>(p);
}

static void drop_graph(dpse_plan* p) {
  if (p->graph_exec) {  // the captured kernels no longer match
    (void)hipGraphExecDestroy(p->graph_exec);
    p->graph_exec = nullptr;
  }
}

int dpse_plan_set_walls(dpse_plan* p, const double* sigma_b, const double* sigma_t) {
  if (!p) return DPSE_EINVAL;
  p->far_n = 0;  // the workspace's far field belongs to the old walls
  if (!sigma_b && !sigma_t) {
    p->walls_on = false;
    p->walls_version++;
    drop_graph(p);
    return DPSE_OK;
  }
  if (!p->bound || (p->g.flags & DPSE_UNIFORM_FAST)) return DPSE_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return DPSE_EHIP;
  const Geom& g = p->g;
  const bool mixed = p->prm.precision == DPSE_MIXED;
  const size_t rs = mixed ? 4 : 8;
  const size_t plane = (size_t)g.Ny * g.Nx, G = (size_t)g.Nz * plane, nm = (size_t)g.Ny * g.nkx;
  dpse::Walls& wl = p->walls;
  if (!wl.stage) {  // first use: one allocation kept with the plan
    auto carve = [&](char* base) {
      Carver c{base};
      c.take(&wl.stage, 2 * plane);
      c.take(&wl.hat, 2 * nm);
      c.take((char**)&wl.phis, G * rs);
      c.take(&wl.scal, 8);
      // one partial per block of the gather interpolation (x,y tiles of 16,
      // at least 4 nodes per block, split over more blocks below 512 of them)
      const size_t nbl = (size_t)(g.Nx / 16) * (g.Ny / 16) * ((g.Nz + 3) / 4);
      c.take(&wl.part, std::max<size_t>(nbl, 2048));
      return c.off;
    };
    const size_t bytes = carve(nullptr);
    void* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) {
      (void)hipGetLastError();
      wl = dpse::Walls{};
      return DPSE_ENOMEM;
    }
    p->allocs.push_back(mem);
    carve((char*)mem);
  }
  hipStream_t s = p->stream;
  hipError_t e = sigma_b ? hipMemcpyAsync(wl.stage, sigma_b, plane * sizeof(double), hipMemcpyDeviceToDevice, s)
                         : dpse::fill_double(wl.stage, 0.0, (int64_t)plane, s);
  if (e == hipSuccess)
    e = sigma_t ? hipMemcpyAsync(wl.stage + plane, sigma_t, plane * sizeof(double), hipMemcpyDeviceToDevice, s)
                : dpse::fill_double(wl.stage + plane, 0.0, (int64_t)plane, s);
  // transforms, the wall potential per mode (through the workspace's psi,
  // psiz and the inverse transforms) and its grid, the wall scalars
  if (e == hipSuccess) e = dpse::launch_wall_transforms(p);
  if (e == hipSuccess) e = mixed ? dpse::launch_wall_modes<float>(p) : dpse::launch_wall_modes<double>(p);
  if (e == hipSuccess) e = mixed ? dpse::launch_fft_inverse<float>(p) : dpse::launch_fft_inverse<double>(p);
  if (e == hipSuccess) e = mixed ? dpse::launch_wall_keep_phi<float>(p) : dpse::launch_wall_keep_phi<double>(p);
  if (e != hipSuccess) return DPSE_EHIP;
  p->walls_on = true;
  p->walls_version++;
  drop_graph(p);
  return DPSE_OK;
}

int dpse_plan_set_tiles(dpse_plan* p, const int32_t* choice) {
  if (!p || !choice) return DPSE_EINVAL;
  for (int s = 0; s < DPSE_NUM_TUNED; ++s)
    if (choice[s] != -1 && !tuned_valid(p, s, choice[s])) return DPSE_EINVAL;
  for (int s = 0; s < DPSE_NUM_TUNED; ++s) tuned_cfg(p, s) = choice[s];
  drop_graph(p);
  return DPSE_OK;
}

int dpse_plan_autotune(dpse_plan* p, int64_t n, const double* pos, const double* q, int reps,
                       int32_t* choice, double* ms) {
  if (!p || !pos || !q || n <= 0 || !p->bound || reps <= 0) return DPSE_EINVAL;
  if (n > p->max_n) return DPSE_ETOOMANY;
  const bool timing = p->timing;
  p->timing = false;
  int st = solve_impl(p, n, pos, q, nullptr, nullptr, nullptr);  // bins and grids for the stage runs
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (st == DPSE_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = DPSE_EHIP;
  if (ms)
    for (int i = 0; i < DPSE_MAX_CANDIDATES * DPSE_NUM_TUNED; ++i) ms[i] = -1.0;
  for (int s = 0; s < DPSE_NUM_TUNED && st == DPSE_OK; ++s) {
    // the deterministic mode fixes the spreading and interpolation kernels
    if (s < 2 && (p->g.flags & DPSE_DETERMINISTIC)) continue;
    int best = -1;
    double tbest = 0.0;
    for (int i = 0; i < tuned_count(s) && st == DPSE_OK; ++i) {
      if (!tuned_valid(p, s, i)) continue;
      tuned_cfg(p, s) = i;
      hipError_t e = hipSuccess;
      for (int r = -1; r < reps && e == hipSuccess; ++r) {  // one untimed run first
        if (r == 0) e = hipEventRecord(e0, p->stream);
        if (e == hipSuccess) e = launch_tuned(p, s, n);
      }
      float t = 0.0f;
      if (e == hipSuccess) e = hipEventRecord(e1, p->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      if (e != hipSuccess) {
        st = DPSE_EHIP;
        break;
      }
      const double tm = (double)t / reps;
      if (ms) ms[s * DPSE_MAX_CANDIDATES + i] = tm;
      if (best < 0 || tm < tbest) {
        best = i;
        tbest = tm;
      }
    }
    tuned_cfg(p, s) = best;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  p->timing = timing;
  drop_graph(p);
  if (choice)
    for (int s = 0; s < DPSE_NUM_TUNED; ++s) choice[s] = tuned_cfg(p, s);
  if (st != DPSE_OK) return st;
  return dpse_sync(p);
}

int dpse_sync(dpse_plan* p) {
  if (!p || !p->bound) return DPSE_EINVAL;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return DPSE_EHIP;
  int st[4] = {0, 0, 0, 0};
  if (hipMemcpy(st, p->w.status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return DPSE_EHIP;
  int zero4[4] = {0, 0, 0, 0};
  if (hipMemcpy(p->w.status, zero4, sizeof(zero4), hipMemcpyHostToDevice) != hipSuccess)
    return DPSE_EHIP;
  // priority: outside > constraint > non-neutral
  if (st[0] & 1) return DPSE_EOUTSIDE;
  if (st[0] & 2) return DPSE_ECONSTRAINT;
  if (st[0] & 4) return DPSE_ENONNEUTRAL;
  return DPSE_OK;
}

int dpse_set_timing(dpse_plan* p, int enable) {
  if (!p) return DPSE_EINVAL;
  p->timing = enable != 0;
  return DPSE_OK;
}

int dpse_stage_times(dpse_plan* p, double* ms, int max_stages, int* n_solves) {
  if (!p || (!ms && max_stages > 0)) return DPSE_EINVAL;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return DPSE_EHIP;
  const int ns = DPSE_NUM_STAGES;
  std::vector<double> acc(ns, 0.0);
  for (int s = 0; s < p->timed_solves; ++s) {
    hipEvent_t* ev = p->events.data() + (size_t)s * (2 * ns);
    for (int k = 0; k < ns; ++k) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]) != hipSuccess) return DPSE_EHIP;
      acc[k] += t;
    }
  }
  int m = max_stages < ns ? max_stages : ns;
  for (int k = 0; k < m; ++k) ms[k] = p->timed_solves ? acc[k] / p->timed_solves : 0.0;
  if (n_solves) *n_solves = p->timed_solves;
  p->timed_solves = 0;
  return DPSE_OK;
}

const char* dpse_stage_name(int stage) {
  return (stage >= 0 && stage < DPSE_NUM_STAGES) ? kStageNames[stage] : "unknown";
}

int dpse_plan_destroy(dpse_plan* p) {
  if (!p) return DPSE_EINVAL;
  (void)hipStreamSynchronize(p->stream);
  if (p->owns_workspace) {  // its workspace is freed below: forget its owner record
    std::lock_guard<std::mutex> lk(g_owner_mu);
    g_owner.erase((const void*)p->w.status);
  }
  for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
  p->events.clear();
  free_all(p);
  delete p;
  return DPSE_OK;
}

int dpse_debug_copy(dpse_plan* p, int which, void* dst, int64_t bytes, int32_t* elem_bytes,
                    int64_t* count) {
  if (!p || !dst || bytes < 0 || !p->bound) return DPSE_EINVAL;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return DPSE_EHIP;
  const dpse::Geom& g = p->g;
  const bool mixed = p->prm.precision == DPSE_MIXED;
  const int rs = mixed ? 4 : 8;
  const int64_t G = (int64_t)g.Nz * g.Ny * g.Nx;
  const int64_t C = (int64_t)g.Nz * g.Ny * g.nkx * 2;
  const void* src = nullptr;
  int64_t cnt = 0;
  int eb = rs;
  switch (which) {
    case DPSE_STAGE_F_I: src = p->w.f_i; cnt = G; break;
    case DPSE_STAGE_F_O: src = p->w.f_o; cnt = G; break;
    case DPSE_STAGE_FH_I: src = p->w.fx_i; cnt = C; break;
    case DPSE_STAGE_FH_O: src = p->w.fx_o; cnt = C; break;
    case DPSE_STAGE_PSI: src = p->w.psi; cnt = C; break;
    case DPSE_STAGE_PSIZ: src = p->w.psiz; cnt = C; break;
    case DPSE_STAGE_GRIDS: src = p->w.u4; cnt = 4 * G; break;
    case DPSE_STAGE_FAR: src = p->w.far4; cnt = 4 * p->last_n; eb = 8; break;
    case DPSE_STAGE_NEAR: src = p->w.near4; cnt = 4 * p->last_n; eb = 8; break;
    case DPSE_STAGE_SCALARS: src = p->w.scal; cnt = 8; eb = 8; break;
    case DPSE_STAGE_WALL_HAT: src = p->walls.hat; cnt = 4 * (int64_t)g.Ny * g.nkx; eb = 8; break;
    case DPSE_STAGE_WALL_PHI: src = p->walls.phis; cnt = G; break;
    case DPSE_STAGE_WALL_SCALARS: src = p->walls.scal; cnt = 4; eb = 8; break;
    default: return DPSE_EINVAL;
  }
  if (!src) return DPSE_EINVAL;  // wall data before dpse_plan_set_walls
  if (cnt * eb > bytes) return DPSE_EINVAL;
  if (hipMemcpy(dst, src, cnt * eb, hipMemcpyDeviceToHost) != hipSuccess) return DPSE_EHIP;
  if (which == DPSE_STAGE_F_O || which == DPSE_STAGE_FH_O) {
    // only the wall-band planes are computed; report zeros elsewhere
    int64_t plane = (which == DPSE_STAGE_F_O ? (int64_t)g.Ny * g.Nx : (int64_t)g.Ny * g.nkx * 2) * eb;
    for (int j = 0; j < g.Nz; ++j)
      if (!dpse::in_band(g, j)) std::memset((char*)dst + j * plane, 0, plane);
  }
  if (elem_bytes) *elem_bytes = eb;
  if (count) *count = cnt;
  return DPSE_OK;
}

}  // extern "C"
