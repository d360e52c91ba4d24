// Particle-side kernels: validation and charge groups with their images
// (Sec. 5.2.2 step 1, eq. ims), counting sorts into spreading bins and the
// near-field cell list, the near-field pair sums (Sec. 3.2 eqs. GnearK,
// EnearK; Sec. 4.2), the gauge constant (Sec. 5.2.2, last paragraph) and the
// combination of far and near parts into potentials, forces and energy
// (eqs. Ufinal, fqE, self term of Sec. 6.3).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dpse_internal.h"

namespace dpse {

namespace {

constexpr int kThreads = 256;

__global__ void k_fill_int(int* p, int v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_double(double* p, double v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__device__ inline double block_sum(double v, double* sh) {
  // wavefront reduction, then across the block's waves
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  }
  __syncthreads();
  return t;  // valid in thread 0
}

__device__ inline int spread_key(const Geom& g, double x, double y, double z) {
  int ix = (int)floor(x / g.h);
  int iy = (int)floor(y / g.h);
  ix %= g.Nx; if (ix < 0) ix += g.Nx;
  iy %= g.Ny; if (iy < 0) iy += g.Ny;
  int bx = ix / g.B, by = iy / g.B;
  int zb = (int)floor((z - g.zb_lo) / g.zb_w);
  zb = zb < 0 ? 0 : (zb >= g.nzb ? g.nzb - 1 : zb);
  return (by * g.nbx + bx) * g.nzb + zb;
}

__device__ inline int cell_of(const Geom& g, double x, double y, double z) {
  int cx = (int)floor(x / g.cwx), cy = (int)floor(y / g.cwy), cz = (int)floor(z / g.cwz);
  cx = cx < 0 ? 0 : (cx >= g.ncx ? g.ncx - 1 : cx);
  cy = cy < 0 ? 0 : (cy >= g.ncy ? g.ncy - 1 : cy);
  cz = cz < 0 ? 0 : (cz >= g.ncz ? g.ncz - 1 : cz);
  return (cz * g.ncy + cy) * g.ncx + cx;
}

// Validation, periodic wrap, groups C_o / C_>, images of C_o charges.
__global__ void __launch_bounds__(kThreads) k_prep(Geom g, int64_t n, const double* __restrict__ pos,
                                                   const double* __restrict__ q, Part* ext, int* meta,
                                                   int* n_img, double* qpart, int* status, int* bin_cnt,
                                                   int* cell_cnt) {
  __shared__ double sh[kThreads / 64];
  int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  const int lane = threadIdx.x & 63;
  double qq = 0.0, x = 0.0, y = 0.0, z = 0.0;
  // images and periodic copies this charge makes
  bool img_b = false, img_t = false, cp_lo = false, cp_hi = false;
  const bool tp = (g.flags & DPSE_TRIPLY) != 0;  // z periodic with period H
  if (i < n) {
    x = pos[3 * i]; y = pos[3 * i + 1]; z = pos[3 * i + 2];
    qq = q[i];
    int st = 0;
    bool fin = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(qq);
    if (!fin || !(z > g.zmin_ok && z < g.zmax_ok)) st |= 1;
    if (!fin) {
      x = 0.0; y = 0.0; z = 0.5 * g.H; qq = 0.0;
    }
    if (tp) {
      z -= g.H * floor(z / g.H);
      if (!(z < g.H)) z = 0.0;
    } else {
      z = fmin(fmax(z, 0.0), g.H);
    }
    x -= g.Lx * floor(x / g.Lx);
    if (!(x < g.Lx)) x = 0.0;
    y -= g.Ly * floor(y / g.Ly);
    if (!(y < g.Ly)) y = 0.0;
    const bool fast = (g.flags & DPSE_UNIFORM_FAST) != 0;  // no walls: one group, no images
    double hmin = fmin(z, g.H - z);
    if (!fast && (g.r_cut >= g.H + hmin || 2.0 * g.H_E >= g.H + hmin)) st |= 2;
    bool low = !fast && z < 2.0 * g.H_E, high = !fast && z > g.H - 2.0 * g.H_E;
    ext[i] = Part{x, y, z, qq};
    meta[i] = ((low || high) ? GRP_WALL : GRP_INNER) | (int)(i << 2);
    // counts of the two counting sorts (spreading bins, near-field cells)
    atomicAdd(&bin_cnt[spread_key(g, x, y, z)], 1);
    atomicAdd(&cell_cnt[cell_of(g, x, y, z)], 1);
    if (g.flags & DPSE_ONE_JUMP) {  // one jump: every charge imaged across that wall
      low = true;
      high = true;  // the wall without a jump has gamma = 0: no image
    }
    img_b = low && g.gamma_b != 0.0;
    img_t = high && g.gamma_t != 0.0;
    // periodic z windows: a copy of a charge within H_E of an end of the
    // period, shifted by one period, spreads to the nodes across that end and
    // gathers its field for the same output index (group of a charge)
    cp_lo = tp && z < g.H_E;
    cp_hi = tp && z >= g.H - g.H_E;
    if (st) atomicOr(status, st);
  }
  // slots of the extra entries: one atomic per block and kind on the shared
  // counter (the waves in order after it, the lanes in order in their wave)
  __shared__ int wcnt[4][kThreads / 64];
  __shared__ int bbase[4];
  const int wv = threadIdx.x >> 6;
  const bool want[4] = {img_b, img_t, cp_lo, cp_hi};
  unsigned long long msk[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    msk[k] = __ballot(want[k]);
    if (lane == 0) wcnt[k][wv] = __popcll(msk[k]);
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    int tot = 0;
    for (int w = 0; w < kThreads / 64; ++w) tot += wcnt[threadIdx.x][w];
    bbase[threadIdx.x] = tot ? atomicAdd(n_img, tot) : 0;
  }
  __syncthreads();
  auto claim = [&](int k) -> int {
    int base = bbase[k];
    for (int w = 0; w < wv; ++w) base += wcnt[k][w];
    return base + __popcll(msk[k] & ((1ull << lane) - 1));
  };
  const int sb = claim(0), stt = claim(1), sl = claim(2), sh_ = claim(3);
  if (img_b) {
    ext[n + sb] = Part{x, y, -z, g.gamma_b * qq};
    meta[n + sb] = GRP_IMAGE | (int)(i << 2);
    atomicAdd(&bin_cnt[spread_key(g, x, y, -z)], 1);
  }
  if (img_t) {
    ext[n + stt] = Part{x, y, 2.0 * g.H - z, g.gamma_t * qq};
    meta[n + stt] = GRP_IMAGE | (int)(i << 2);
    atomicAdd(&bin_cnt[spread_key(g, x, y, 2.0 * g.H - z)], 1);
  }
  if (cp_lo) {
    ext[n + sl] = Part{x, y, z + g.H, qq};
    meta[n + sl] = GRP_INNER | (int)(i << 2);
    atomicAdd(&bin_cnt[spread_key(g, x, y, z + g.H)], 1);
  }
  if (cp_hi) {
    ext[n + sh_] = Part{x, y, z - g.H, qq};
    meta[n + sh_] = GRP_INNER | (int)(i << 2);
    atomicAdd(&bin_cnt[spread_key(g, x, y, z - g.H)], 1);
  }
  // the block's sums of q and |q| (summed over the blocks in a fixed order by k_scatter_ext)
  double s1 = block_sum(qq, sh);
  double s2 = block_sum(fabs(qq), sh);
  if (threadIdx.x == 0) {
    qpart[2 * blockIdx.x] = s1;
    qpart[2 * blockIdx.x + 1] = s2;
  }
}

// What a solve accumulates into, cleared in one launch before the prep
// kernel: the image counter and the bin counters of the grid stages and of
// the near-field cell list (the gauge constant scal[2] of the last full
// solve stays, for dpse_solve_near).
__global__ void __launch_bounds__(kThreads) k_reset(int* n_img, int* bin_cnt, int nbin, int* cell_cnt, int ncell) {
  const int t = blockIdx.x * kThreads + threadIdx.x, stride = gridDim.x * kThreads;
  if (t == 0) *n_img = 0;
  for (int i = t; i < nbin; i += stride) bin_cnt[i] = 0;
  for (int i = t; i < ncell; i += stride) cell_cnt[i] = 0;
}

// Scatter of charges and images into the spreading bins (counted by the prep
// kernel). The first block also sums the prep kernel's nqb block sums of q
// and |q| in a fixed order (strided per thread, then a fixed tree), stores
// them in scal[0], scal[1] and checks the neutrality of the charges and the
// wall charges together (eq. elecneu; ws = the wall scalars (int sigma,
// int |sigma|), or null without walls).
__global__ void __launch_bounds__(kThreads) k_scatter_ext(Geom g, int64_t n, const Part* __restrict__ ext,
                                                          const int* __restrict__ meta,
                                                          const int* __restrict__ n_img, int* cur,
                                                          Part* srt, int* srt_meta, const double* qpart, int nqb,
                                                          double* scal, const double* ws, int* status) {
  __shared__ double sh[kThreads / 64];
  int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (blockIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nqb; k += kThreads) {
      a += qpart[2 * k];
      b += qpart[2 * k + 1];
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
      scal[0] = a;
      scal[1] = b;
      const double net = a + (ws ? ws[0] : 0.0), tot = b + (ws ? ws[1] : 0.0);
      if (!(fabs(net) <= 1e-12 * tot)) atomicOr(status, 4);
    }
  }
  if (i >= n + *n_img) return;
  Part p = ext[i];
  int s = atomicAdd(&cur[spread_key(g, p.x, p.y, p.z)], 1);
  srt[s] = p;
  srt_meta[s] = meta[i];
}

__global__ void __launch_bounds__(kThreads) k_scatter_cells(Geom g, int64_t n, const Part* __restrict__ ext,
                                                            int* cur, Part* srt, int* idx) {
  int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= n) return;
  Part p = ext[i];
  int s = atomicAdd(&cur[cell_of(g, p.x, p.y, p.z)], 1);
  srt[s] = p;
  idx[s] = (int)i;
}

// Deterministic order inside the segments of a counting sort (the scatters
// claim slots with atomics, so the order within a segment follows the
// scheduling): one thread per segment [off[b], off[b+1]) puts its entries in
// increasing key order by insertion (segments hold a few entries at the
// densities of the workloads; the cost grows with the square of a segment's
// length). The keys are unique: spreading bins sort by (meta, z) (a charge,
// each of its images and each periodic copy differ in group or height),
// cells by the charge index.
__global__ void __launch_bounds__(kThreads) k_sort_bins(int nseg, const int* __restrict__ off, Part* srt,
                                                        int* key) {
  const int b = blockIdx.x * kThreads + threadIdx.x;
  if (b >= nseg) return;
  const int a = off[b], e = off[b + 1];
  for (int i = a + 1; i < e; ++i) {
    const Part p = srt[i];
    const int m = key[i];
    int j = i - 1;
    while (j >= a && (key[j] > m || (key[j] == m && srt[j].z > p.z))) {
      srt[j + 1] = srt[j];
      key[j + 1] = key[j];
      --j;
    }
    srt[j + 1] = p;
    key[j + 1] = m;
  }
}

// Exclusive scan of cnt[0..m) into off[0..m] and cur[0..m) by one block:
// per-thread runs, a shuffle scan inside each wave, one barrier for the wave
// totals.
__global__ void __launch_bounds__(1024) k_scan(const int* __restrict__ cnt, int* off, int* cur, int m) {
  __shared__ int wsum[1024 / 64];
  const int T = 1024, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int per = (m + T - 1) / T;
  const int b = threadIdx.x * per, e = min(m, b + per);
  int s = 0;
  for (int i = b; i < e; ++i) s += cnt[i];
  int incl = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int wofs = 0;
  for (int i = 0; i < w; ++i) wofs += wsum[i];
  int run = wofs + incl - s;
  for (int i = b; i < e; ++i) {
    off[i] = run;
    cur[i] = run;
    run += cnt[i];
  }
  if (threadIdx.x == T - 1) off[m] = wofs + incl;
}

// Multi-block form of the same scan for long counter arrays: block sums of
// chunks of kScanChunk counters, one-block scan of the sums, then every chunk
// scanned again with its offset (each thread a run of 8 consecutive counters).
constexpr int kScanChunk = 8192;

__global__ void __launch_bounds__(1024) k_scan_sums(const int* __restrict__ cnt, int m, int* __restrict__ part) {
  __shared__ int ws[1024 / 64];
  const int base = blockIdx.x * kScanChunk, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int s = 0;
  for (int i = threadIdx.x; i < kScanChunk; i += 1024)
    if (base + i < m) s += cnt[base + i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) ws[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < 1024 / 64; ++i) t += ws[i];
    part[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(1024) k_scan_apply(const int* __restrict__ cnt, int m, const int* __restrict__ pofs,
                                                     int nb, int* off, int* cur) {
  __shared__ int wsum[1024 / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.x * kScanChunk + threadIdx.x * 8;
  int v[8], s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[k] = b + k < m ? cnt[b + k] : 0;
    s += v[k];
  }
  int incl = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(incl, o, 64);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int run = pofs[blockIdx.x] + incl - s;
  for (int i = 0; i < w; ++i) run += wsum[i];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (b + k < m) {
      off[b + k] = run;
      cur[b + k] = run;
    }
    run += v[k];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) off[m] = pofs[nb];
}

// Exclusive scan of cnt[0..m) into off[0..m] and cur[0..m); scratch holds
// 3 (scan_blocks(m) + 1) ints.
void launch_scan(const int* cnt, int* off, int* cur, int m, int* scratch, hipStream_t s) {
  const int nb = scan_blocks(m);
  if (nb == 0) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, cnt, off, cur, m);
    return;
  }
  int* part = scratch;
  int* pofs = scratch + (nb + 1);
  int* pcur = scratch + 2 * (nb + 1);
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(1024), 0, s, cnt, m, part);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, (const int*)part, pofs, pcur, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(1024), 0, s, cnt, m, (const int*)pofs, nb, off, cur);
}

}  // namespace

int scan_blocks(int64_t m) { return m <= 4 * kScanChunk ? 0 : (int)((m + kScanChunk - 1) / kScanChunk); }

namespace {

// --- near field -------------------------------------------------------------

template <typename R>
__device__ inline void near_pair(const Geom& g, double dx, double dy, double dz, double qs,
                                 R& ph, R& ex, R& ey, R& ez) {
  double r2 = dx * dx + dy * dy + dz * dz;
  if (!(r2 < g.r_cut * g.r_cut)) return;
  R r;
  if constexpr (sizeof(R) == 4) r = sqrtf((float)r2);  // the FP32 path takes no FP64 square root
  else r = sqrt(r2);
  R G, e;
  if (g.g_w > 0.0) {
    R a1 = (R)(1.0 / (2.0 * g.g_w)), b1 = (R)g.xi_e;
    if (r < (R)(1e-3 * g.g_w)) {
      const R c = (R)(2.0 / sqrt(kPi));
      R c0 = c * (a1 - b1);
      R c2 = -c * (a1 * a1 * a1 - b1 * b1 * b1) / (R)3;
      R c4 = c * (a1 * a1 * a1 * a1 * a1 - b1 * b1 * b1 * b1 * b1) / (R)10;
      G = c0 + c2 * r * r + c4 * r * r * r * r;
      e = -(2 * c2 + 4 * c4 * r * r);
    } else {
      G = (erf(a1 * r) - erf(b1 * r)) / r;
      R dG = (R)(2.0 / sqrt(kPi)) * (a1 * exp(-(a1 * r) * (a1 * r)) - b1 * exp(-(b1 * r) * (b1 * r))) / r - G / r;
      e = -dG / r;
    }
  } else {
    R xr = (R)g.xi_e * r;
    G = erfc(xr) / r;
    e = (G + (R)(2.0 / sqrt(kPi)) * (R)g.xi_e * exp(-xr * xr)) / (r * r);
  }
  R qr = (R)qs;
  ph += qr * G;
  ex += qr * e * (R)dx;
  ey += qr * e * (R)dy;
  ez += qr * e * (R)dz;
}

// L lanes per target charge (cell-sorted order); the lanes' sums are combined
// by a butterfly inside the lane group. With BY_CELL each lane takes every
// L-th of the neighbouring cells (few candidates per cell); otherwise every
// lane visits every cell and takes every L-th charge in it (many candidates:
// short serial chains per lane and many waves in flight). Sources: other
// charges in the 27 neighbouring cells (minimal image), and the bottom/top
// images of all charges, found through the mirror points (x, y, -z) and
// (x, y, 2H - z).
template <typename R, int L, bool BY_CELL>
__global__ void __launch_bounds__(kThreads) k_near(Geom g, int64_t n, const Part* __restrict__ srt,
                                                   const int* __restrict__ idx, const int* __restrict__ off,
                                                   double4* near4) {
  static_assert(kThreads % L == 0 && L <= 64, "lane groups inside a wave");
  const int64_t gt = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  const int64_t t = gt / L;
  const int sub = (int)(gt % L);
  const bool active = t < n;  // lane groups never straddle the end (kThreads is a multiple of L)
  R ph = 0, ex = 0, ey = 0, ez = 0;
  if (active) {
    const Part me = srt[t];
    int cx = (int)floor(me.x / g.cwx), cy = (int)floor(me.y / g.cwy);
    cx = min(max(cx, 0), g.ncx - 1);
    cy = min(max(cy, 0), g.ncy - 1);
    int xlo = -1, xhi = 1, ylo = -1, yhi = 1;
    const bool xall = g.ncx < 3, yall = g.ncy < 3;
    if (xall) { xlo = 0; xhi = g.ncx - 1; }
    if (yall) { ylo = 0; yhi = g.ncy - 1; }
    const bool tp = (g.flags & DPSE_TRIPLY) != 0;  // z periodic: wrapped cells, minimal image in z
    const int nxc = xhi - xlo + 1, nyc = yhi - ylo + 1;
    // three source families: direct (mirror sign +1), bottom images, top images
    for (int fam = 0; fam < 3; ++fam) {
      double zt, qf;  // z of the point whose neighbours are searched; strength factor
      if (fam == 0) { zt = me.z; qf = 1.0; }
      else if (fam == 1) { if (g.gamma_b == 0.0 || me.z >= g.r_cut) continue; zt = -me.z; qf = g.gamma_b; }
      else { if (g.gamma_t == 0.0 || g.H - me.z >= g.r_cut) continue; zt = 2.0 * g.H - me.z; qf = g.gamma_t; }
      int zlo = (int)floor((zt - g.r_cut) / g.cwz), zhi = (int)floor((zt + g.r_cut) / g.cwz);
      int cz0 = 0;
      if (tp) {
        cz0 = min(max((int)floor(zt / g.cwz), 0), g.ncz - 1);
        zlo = g.ncz < 3 ? 0 : -1;
        zhi = g.ncz < 3 ? g.ncz - 1 : 1;
      } else {
        zlo = max(zlo, 0);
        zhi = min(zhi, g.ncz - 1);
      }
      // the family's cells, x fastest; with BY_CELL lane sub takes cells
      // sub, sub + L, ... (all lanes of a group busy at once)
      const int ncell = (zhi - zlo + 1) * nyc * nxc;
      for (int v = BY_CELL ? sub : 0; v < ncell; v += BY_CELL ? L : 1) {
        const int vyz = v / nxc, ox = xlo + (v - vyz * nxc);
        const int oz = zlo + vyz / nyc, oy = ylo + (vyz - (vyz / nyc) * nyc);
        const int cz = !tp ? oz : (g.ncz < 3 ? oz : (cz0 + oz + g.ncz) % g.ncz);
        const int yy = yall ? oy : (cy + oy + g.ncy) % g.ncy;
        const int xx = xall ? ox : (cx + ox + g.ncx) % g.ncx;
        const int c = (cz * g.ncy + yy) * g.ncx + xx;
        for (int s = off[c] + (BY_CELL ? 0 : sub); s < off[c + 1]; s += (BY_CELL ? 1 : L)) {
          if (fam == 0 && s == t) continue;
          const Part o = srt[s];
          // minimal image: the coordinates were wrapped into [0, L), so
          // |dx| < L and one shift at most (no division)
          double dx = me.x - o.x, dy = me.y - o.y;
          if (dx > 0.5 * g.Lx) dx -= g.Lx;
          else if (dx < -0.5 * g.Lx) dx += g.Lx;
          if (dy > 0.5 * g.Ly) dy -= g.Ly;
          else if (dy < -0.5 * g.Ly) dy += g.Ly;
          const double zs = fam == 0 ? o.z : (fam == 1 ? -o.z : 2.0 * g.H - o.z);
          double dz = me.z - zs;
          if (tp) {
            if (dz > 0.5 * g.H) dz -= g.H;
            else if (dz < -0.5 * g.H) dz += g.H;
          }
          near_pair<R>(g, dx, dy, dz, qf * o.q, ph, ex, ey, ez);
        }
      }
    }
  }
#pragma unroll
  for (int o = 1; o < L; o <<= 1) {
    ph += __shfl_xor(ph, o, 64);
    ex += __shfl_xor(ex, o, 64);
    ey += __shfl_xor(ey, o, 64);
    ez += __shfl_xor(ez, o, 64);
  }
  if (active && sub == 0) {
    const double c = 1.0 / (4.0 * kPi * g.eps);
    near4[idx[t]] = make_double4(c * (double)ph, c * (double)ex, c * (double)ey, c * (double)ez);
  }
}

// Pointwise near-field potential at the origin (gauge of Sec. 5.2.2): kernel
// G^(n)(r; g_w, xi) of eq. Gnear over the charges and their first images.
__global__ void __launch_bounds__(kThreads) k_near_origin(Geom g, int64_t n, const Part* __restrict__ ext,
                                                          double* partials) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  const double xp = 1.0 / sqrt(2.0 * g.g_w * g.g_w + 1.0 / (g.xi * g.xi));
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    Part p = ext[i];
    double dx = -p.x - g.Lx * rint(-p.x / g.Lx);
    double dy = -p.y - g.Ly * rint(-p.y / g.Ly);
    double zs[3] = {p.z, -p.z, 2.0 * g.H - p.z};
    double qs[3] = {p.q, g.gamma_b * p.q, g.gamma_t * p.q};
    for (int f = 0; f < 3; ++f) {
      if (qs[f] == 0.0) continue;
      double r = sqrt(dx * dx + dy * dy + zs[f] * zs[f]);
      if (!(r < g.r_cut)) continue;
      double G = g.g_w > 0.0 ? (erf(r / (sqrt(2.0) * g.g_w)) - erf(xp * r)) / r : erfc(xp * r) / r;
      acc += qs[f] * G;
    }
  }
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// phibar = far + near + B_i - q * 2 xi_e / (4 pi eps sqrt(pi)); F = q (E_far + E_near).
// With gnear non-null the gauge constant B_i is formed here first: the first
// wave of every block sums the near part at the origin from gnb block
// partials and the far part from the per-node partials gfar[0 .. Nz), in a
// fixed order (every block gets the same bits), and block 0 stores it with
// its parts in scal[2], scal[4], scal[5]; otherwise B_i is scal[2] as it
// stands (the near-field-only solve keeps that of the last full solve).
__global__ void __launch_bounds__(kThreads) k_finalize(Geom g, int64_t n, const double* __restrict__ q,
                                                       const double4* __restrict__ far4,
                                                       const double4* __restrict__ near4, double* scal,
                                                       double* phi, double* force, double* partials,
                                                       const double* gnear, int gnb, const double* gfar) {
  __shared__ double sh[kThreads / 64];
  __shared__ double bsh;
  const double selfc = 2.0 * g.xi_e / (4.0 * kPi * g.eps * sqrt(kPi));
  if (gnear) {
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      double sn = 0.0, sf = 0.0;
      for (int i = lane; i < gnb; i += 64) sn += gnear[i];
      for (int i = lane; i < g.Nz; i += 64) sf += gfar[i];
      for (int o = 32; o > 0; o >>= 1) {
        sn += __shfl_down(sn, o, 64);
        sf += __shfl_down(sf, o, 64);
      }
      if (lane == 0) {
        const double near0 = sn / (4.0 * kPi * g.eps);
        const double b = (g.flags & DPSE_GAUGE_NONE) ? 0.0 : -(sf + near0);
        bsh = b;
        if (blockIdx.x == 0) {
          scal[4] = sf;
          scal[5] = near0;
          scal[2] = b;
        }
      }
    }
    __syncthreads();
  }
  const double Bi = gnear ? bsh : scal[2];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    double qi = q[i];
    double4 f = far4[i], r = near4[i];
    double ph = f.x + r.x + Bi - qi * selfc;
    if (phi) phi[i] = ph;
    if (force) {
      force[3 * i] = qi * (f.y + r.y);
      force[3 * i + 1] = qi * (f.z + r.z);
      force[3 * i + 2] = qi * (f.w + r.w);
    }
    acc += qi * ph;
  }
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// U = 1/2 sum q phibar (eq. Ufinal), plus with wall charges half their
// integral by reciprocity: sum q phi_s(z_k) (nbw partials in wpart), int sigma
// phi_s (ws[2]) and B_i int sigma (scal[2] ws[0]).
// One wave: lane-strided sums of the partials, then a fixed shuffle tree (the
// order does not depend on timing).
__global__ void k_energy_final(int nb, const double* partials, double* energy, double* scal, int nbw,
                               const double* wpart, const double* ws) {
  const int lane = threadIdx.x;
  double s = 0.0, sw = 0.0;
  for (int i = lane; i < nb; i += 64) s += partials[i];
  if (wpart)
    for (int i = lane; i < nbw; i += 64) sw += wpart[i];
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_down(s, o, 64);
    sw += __shfl_down(sw, o, 64);
  }
  if (lane == 0) {
    if (wpart) s += sw + ws[2] + scal[2] * ws[0];
    scal[6] = 0.5 * s;
    if (energy) *energy = 0.5 * s;
  }
}

// Brownian-dynamics step (eq. leimkuhler); counts charges leaving the
// admissible heights.
__global__ void __launch_bounds__(kThreads) k_bd_step(Geom g, int64_t n, const double* __restrict__ pos,
                                                      const double* __restrict__ F,
                                                      const double* __restrict__ wp,
                                                      const double* __restrict__ wn, double mu_dt, double noise,
                                                      double* __restrict__ out, int* escaped) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i >= n) return;
  double v[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t k = 3 * i + c;
    v[c] = pos[k] + mu_dt * F[k] + noise * (wp[k] + wn[k]);
    out[k] = v[c];
  }
  if (!(v[2] > g.zmin_ok && v[2] < g.zmax_ok)) atomicAdd(escaped, 1);
}

inline int blocks_for(int64_t n, int cap) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  return (int)(b < cap ? b : cap);
}

}  // namespace

hipError_t fill_int(int* ptr, int value, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(count, 4096)), dim3(kThreads), 0, s, ptr, value, count);
  return hipGetLastError();
}

hipError_t fill_double(double* ptr, double value, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_double, dim3(blocks_for(count, 4096)), dim3(kThreads), 0, s, ptr, value, count);
  return hipGetLastError();
}

hipError_t launch_prep(dpse_plan* p, int64_t n, const double* pos, const double* q) {
  hipStream_t s = p->stream;
  Workspace& w = p->w;
  const int nbin = (int)p->nkeys + 1, ncell = (int)p->ncells + 1;
  hipLaunchKernelGGL(k_reset, dim3(blocks_for(std::max(nbin, ncell), 64)), dim3(kThreads), 0, s, w.n_img,
                     w.bin_cnt, nbin, w.cell_cnt, ncell);
  int nb = (int)((n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_prep, dim3(nb), dim3(kThreads), 0, s, p->g, n, pos, q, w.ext, w.ext_meta,
                     w.n_img, w.qpart, w.status, w.bin_cnt, w.cell_cnt);
  return hipGetLastError();
}

// Bins of the grid stages: counting sort of charges and images by (x,y tile
// bin, z bucket); launch_prep cleared and filled the counts.
hipError_t launch_bin_grid(dpse_plan* p, int64_t n) {
  hipStream_t s = p->stream;
  Workspace& w = p->w;
  int nb3 = (int)((3 * n + kThreads - 1) / kThreads);
  launch_scan((const int*)w.bin_cnt, w.bin_off, w.bin_cur, p->nkeys, w.scan_bin, s);
  const int nqb = (int)((n + kThreads - 1) / kThreads);  // blocks of the prep kernel
  hipLaunchKernelGGL(k_scatter_ext, dim3(nb3), dim3(kThreads), 0, s, p->g, n, (const Part*)w.ext,
                     (const int*)w.ext_meta, (const int*)w.n_img, w.bin_cur, w.srt, w.srt_meta,
                     (const double*)w.qpart, nqb, w.scal, p->walls_on ? (const double*)p->walls.scal : nullptr,
                     w.status);
  if (p->g.flags & DPSE_DETERMINISTIC)
    hipLaunchKernelGGL(k_sort_bins, dim3((p->nkeys + kThreads - 1) / kThreads), dim3(kThreads), 0, s, p->nkeys,
                       (const int*)w.bin_off, w.srt, w.srt_meta);
  return hipGetLastError();
}

// Cell list of the near field: counting sort of the charges by cell;
// launch_prep cleared and filled the counts.
hipError_t launch_bin_cells(dpse_plan* p, int64_t n) {
  hipStream_t s = p->stream;
  Workspace& w = p->w;
  int nb = (int)((n + kThreads - 1) / kThreads);
  launch_scan((const int*)w.cell_cnt, w.cell_off, w.cell_cur, p->ncells, w.scan_cell, s);
  hipLaunchKernelGGL(k_scatter_cells, dim3(nb), dim3(kThreads), 0, s, p->g, n, (const Part*)w.ext,
                     w.cell_cur, w.nsrt, w.nsrt_idx);
  if (p->g.flags & DPSE_DETERMINISTIC)
    hipLaunchKernelGGL(k_sort_bins, dim3((p->ncells + kThreads - 1) / kThreads), dim3(kThreads), 0, s, p->ncells,
                       (const int*)w.cell_off, w.nsrt, w.nsrt_idx);
  return hipGetLastError();
}

hipError_t launch_bin(dpse_plan* p, int64_t n) {
  hipError_t e = launch_bin_grid(p, n);
  return e == hipSuccess ? launch_bin_cells(p, n) : e;
}

template <typename R, int L, bool BY_CELL>
void near_as(dpse_plan* p, int64_t n) {
  int nb = (int)((n * L + kThreads - 1) / kThreads);
  hipLaunchKernelGGL((k_near<R, L, BY_CELL>), dim3(nb), dim3(kThreads), 0, p->stream, p->g, n,
                     (const Part*)p->w.nsrt, (const int*)p->w.nsrt_idx, (const int*)p->w.cell_off, p->w.near4);
}

// Lanes per target from the expected candidates per target (charges in the
// neighbouring cells at uniform density): 8 lanes over cells below 256
// candidates (the slab workloads: 25-100), 32 or 64 lanes over the charges
// of every cell beyond (the triply periodic workload: ~2100).
template <typename R>
hipError_t launch_near(dpse_plan* p, int64_t n) {
  const Geom& g = p->g;
  const double cells = (double)std::min(g.ncx, 3) * std::min(g.ncy, 3) * std::min(g.ncz, 3);
  const double cand = (double)n * cells / ((double)g.ncx * g.ncy * g.ncz);
  if (cand < 256.0) near_as<R, 8, true>(p, n);
  else if (cand < 1024.0) near_as<R, 32, false>(p, n);
  else near_as<R, 64, false>(p, n);
  return hipGetLastError();
}

// Near part of the gauge: per-block partials at the origin (independent of
// the far field, so it can run beside it).
hipError_t launch_near_origin(dpse_plan* p, int64_t n) {
  int nb = blocks_for(n, p->npartials);
  hipLaunchKernelGGL(k_near_origin, dim3(nb), dim3(kThreads), 0, p->stream, p->g, n, (const Part*)p->w.ext,
                     p->w.partials);
  return hipGetLastError();
}

// Gauge constant from the near partials and the far per-node partials.
hipError_t launch_finalize(dpse_plan* p, int64_t n, const double* q, double* energy, double* phi,
                           double* force, bool gauge) {
  int nb = blocks_for(n, p->npartials);
  // the near-origin partials (nb of them, partials[0 ..)) and the far per-node
  // partials (partials[2 npartials ..)) of the gauge constant
  hipLaunchKernelGGL(k_finalize, dim3(nb), dim3(kThreads), 0, p->stream, p->g, n, q,
                     (const double4*)p->w.far4, (const double4*)p->w.near4, p->w.scal, phi, force,
                     p->w.partials + p->npartials, gauge ? (const double*)p->w.partials : nullptr, nb,
                     (const double*)(p->w.partials + 2 * p->npartials));
  // the partials of the wall term, from the interpolation or the per-charge kernel
  const bool wall = p->walls_on && energy && p->wall_part;
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64), 0, p->stream, nb,
                     (const double*)(p->w.partials + p->npartials), energy, p->w.scal,
                     wall ? p->wall_nparts : 0, wall ? (const double*)p->wall_part : nullptr,
                     wall ? (const double*)p->walls.scal : nullptr);
  return hipGetLastError();
}

hipError_t launch_bd_step(dpse_plan* p, int64_t n, const double* pos, const double* force, const double* w_prev,
                          const double* w_next, double mu_dt, double noise, double* pos_out, int* escaped) {
  hipError_t e = fill_int(escaped, 0, 1, p->stream);
  if (e != hipSuccess) return e;
  const int nb = (int)((n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_bd_step, dim3(nb), dim3(kThreads), 0, p->stream, p->g, n, pos, force, w_prev, w_next, mu_dt,
                     noise, pos_out, escaped);
  return hipGetLastError();
}

template hipError_t launch_near<double>(dpse_plan*, int64_t);
template hipError_t launch_near<float>(dpse_plan*, int64_t);

}  // namespace dpse
