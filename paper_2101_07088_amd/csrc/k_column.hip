// Per-mode work of the far field (Sec. 5.2.2 steps 2-6, App. A), one
// workgroup per block of transverse modes, all in FP64 whatever the storage
// precision of the grids:
//  1. Chebyshev coefficients of F_o and F_i in z: DCT-I of the Nz node values
//     through a complex FFT of the even extension (length 2(Nz-1)) in LDS.
//  2. The integral-formulation BVP of App. A for psi_o* and psi_i*: in the
//     unknowns y''_n the mode equations y''_n - kappa^2 y_n = g_n split into an
//     even and an odd tridiagonal chain; the free constants y_0 and y'_0 enter
//     only the first row of each chain. Each chain is solved once for the
//     right-hand sides and once for the unit free constant, and the two
//     boundary conditions (Robin for k != 0, homogeneous Dirichlet for k = 0)
//     fix y_0 and y'_0 through a 2x2 Schur complement (eq. blocksys).
//  3. Values and z-derivatives at z = 0 and z = H, the mismatches of eqs.
//     mm1-mm4 with psi_b* = tau_b psi_o*, psi_t* = tau_t psi_o*, and the
//     harmonic correction: with E = e^{-kH}, the jump conditions reduce to a
//     2x2 system whose solution gives psi_c(z) = alpha e^{k(z-H)} + beta e^{-kz}
//     inside the slab (evaluated at nodes with -H_E <= z <= H + H_E, for
//     |k| <= k_max only, Sec. 5.2.2 step 4).
//  4. k = 0: A_b, A_t from the end slopes of psi_o* (eq. CE) and the mean of
//     the two expressions for A_i (eqs. ai1, ai2), added as A_i z.
//  5. Psi and Psi_z at the nodes: inverse DCT of the series and of its exact
//     derivative (coefficient recurrence), plus the analytic correction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "dpse_internal.h"
#include "fft_lds.h"

namespace dpse {

namespace {

constexpr int kThreads = 256;
// KE (a template parameter) = complex elements per LDS buffer = modes per
// block x 2(Nz-1); one of kColumnKE, chosen per grid by the autotuner.
// Candidates 0-4: k_column (Nz > 257); candidate 5: k_column_scan (Nz <= 257).
constexpr int kColumnKE[] = {2048, 1024, 4096, 2048, 4096, 2048};
constexpr int kColumnNT[] = {256, 256, 256, 512, 512, 256};  // threads per workgroup
constexpr int kNumColumn = 6;
constexpr int kScanCand = 5;
constexpr int kMaxMB = 32;    // modes per block (16 MB chain threads <= the block's threads)
// dynamic LDS per block: 160 KB per workgroup less a margin for the static
// arrays of the kernel (under 3 KB)
constexpr size_t kMaxLds = 156 * 1024;

template <typename R>
struct CT;
template <>
struct CT<double> { using T = double2; };
template <>
struct CT<float> { using T = float2; };

__device__ inline int ilog2d(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Reciprocal of a double: hardware estimate refined by two Newton steps
// (relative error at the level of the last bit; the solve needs no correctly
// rounded division).
__device__ inline double rcp_refined(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// |k|, kappa = |k| R and whether the harmonic correction applies, of mode mi
// (mode index ky * (Nx/2+1) + kx of the half spectrum).
__device__ inline void mode_wave(const Geom& g, int mi, double& kk, int& keep) {
  const int kyi = mi / g.nkx, kxi = mi % g.nkx;
  const int nx = kxi == g.Nx / 2 ? -(g.Nx / 2) : kxi;
  const int ny = kyi < g.Ny / 2 ? kyi : kyi - g.Ny;
  const double kx = 2.0 * kPi * nx / g.Lx, ky = 2.0 * kPi * ny / g.Ly;
  kk = sqrt(kx * kx + ky * ky);
  const long long lhs = 4LL * ((long long)nx * nx * g.Ny * g.Ny + (long long)ny * ny * g.Nx * g.Nx);
  const long long rhs = (long long)g.Nx * g.Ny * (long long)g.Nx * g.Ny;
  keep = (lhs <= rhs) ? 1 : 0;
  if ((g.flags & DPSE_KMAX_GT) && !(kk <= 4.2 / g.g_t)) keep = 0;
  if (g.flags & DPSE_UNIFORM_FAST) keep = 0;  // nothing to correct without jumps
}

// Plan-time factorisation of the per-mode chains (they depend on kappa only)
// for the twisted elimination of the column kernel: for the even (rows n =
// 2r) and odd (n = 2r+1) chain of L rows, the downward multipliers cp_r above
// the middle row t = L/2, the upward ones cq_r below it and the inverse of the
// middle row's pivot at t; chain-major, cpiv[(par * ceil(N/2) + r) * nmodes + mode].
__global__ void __launch_bounds__(kThreads) k_pivots(Geom g, const double* __restrict__ ctab,
                                                     double* __restrict__ cpiv) {
  const int nmodes = g.Ny * g.nkx, N = g.Nz;
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= 2 * nmodes) return;
  const int mi = t % nmodes, par = t / nmodes;
  double kk;
  int keep;
  mode_wave(g, mi, kk, keep);
  const double kap = kk * g.zR, kap2 = kap * kap;
  const double* ca = ctab;
  const double* cb = ctab + N;
  const double* cc = ctab + 2 * N;
  const int half0 = (N + 1) / 2;
  const int L = par == 0 ? (N + 1) / 2 : N / 2, mt = L / 2;
  double* out = cpiv + (size_t)par * half0 * nmodes + mi;
  // downwards to the middle row: cp_r = sup_r / (dia_r - sub_r cp_{r-1})
  double cp = 0.0;
  for (int r = 0; r < mt; ++r) {
    const int n = par + 2 * r;
    const double sub = -kap2 * ca[n], dia = fma(kap2, cb[n], 1.0), sup = -kap2 * cc[n];
    cp = sup * rcp_refined(fma(-sub, cp, dia));
    out[(size_t)r * nmodes] = cp;
  }
  // upwards to the middle row: cq_r = sub_r / (dia_r - sup_r cq_{r+1})
  double cq = 0.0;
  for (int r = L - 1; r > mt; --r) {
    const int n = par + 2 * r;
    const double sub = -kap2 * ca[n], dia = fma(kap2, cb[n], 1.0), sup = -kap2 * cc[n];
    cq = sub * rcp_refined(fma(-sup, cq, dia));
    out[(size_t)r * nmodes] = cq;
  }
  // the middle row's pivot, inverted
  const int n = par + 2 * mt;
  const double sub = -kap2 * ca[n], dia = fma(kap2, cb[n], 1.0), sup = -kap2 * cc[n];
  out[(size_t)mt * nmodes] = rcp_refined(dia - sub * cp - sup * cq);
}

// The two FFTs of a column workgroup: in lockstep where each thread holds at
// most two radix-4 butterflies per buffer (one barrier per pass for both),
// one after the other where the pair's registers would spill.
template <int KE, int NT>
__device__ __forceinline__ void fft2(double2* A, double2* B, int logM, int logMB, const double2* tw, int tid) {
  constexpr int kBpt4 = KE / 4 / NT;  // KE == M * MB elements per buffer
  if constexpr (kBpt4 <= 2) {
    fft_lds_r22_pair<double2, true, kBpt4, NT>(A, B, logM, logMB, 1, 1 << logMB, tw, false, tid);
  } else {
    fft_lds_r22<double2, true, kBpt4, NT>(A, logM, logMB, 1, 1 << logMB, tw, false, tid);
    fft_lds_r22<double2, true, kBpt4, NT>(B, logM, logMB, 1, 1 << logMB, tw, false, tid);
  }
}

template <typename R, int KE, int NT>
__global__ void __launch_bounds__(NT) k_column(Geom g, const typename CT<R>::T* __restrict__ fx_i,
                                                     const typename CT<R>::T* __restrict__ fx_o,
                                                     typename CT<R>::T* __restrict__ psi,
                                                     typename CT<R>::T* __restrict__ psiz,
                                                     const double* __restrict__ zn,
                                                     const double* __restrict__ ctab,
                                                     const double2* __restrict__ twz,
                                                     const double* __restrict__ cpiv, double* scal,
                                                     const double2* __restrict__ wall_hat) {
  using C = typename CT<R>::T;
  extern __shared__ double2 smem2[];
  constexpr int kElems = KE;
  double2* A = smem2;               // psi_o* work, later the final series of psi_i*
  double2* B = smem2 + kElems;      // psi_i* work, later its derivative series
  double2* tw = smem2 + 2 * kElems; // twiddles exp(-2 pi i k / M), k < M/2
  // chain coefficients a_n, b_n, c_n and rhs scales (4 Nz doubles), then the
  // functionals of phase 3 (MB x 44 doubles)
  double* lco = reinterpret_cast<double*>(tw + (g.Nz - 1));
  __shared__ double s_k[kMaxMB], s_kap[kMaxMB];
  __shared__ int s_keep[kMaxMB];
  __shared__ double2 s_c[kMaxMB][2];      // free constants (y_0, y'_0) of psi_i*
  __shared__ double2 s_ab[kMaxMB][2];     // correction alpha, beta
  __shared__ double s_Ai[kMaxMB];

  const int N = g.Nz, M = 2 * (N - 1), logM = ilog2d(M);
  const int MB = kElems / M;
  const int logMB = ilog2d(KE) - logM;
  const int NU = N + 2;
  const int nmodes = g.Ny * g.nkx;
  const int m0 = xcd_block(blockIdx.x, gridDim.x) * MB;
  const int tid = threadIdx.x;
  const double Rz = g.zR;
  for (int i = tid; i < kCtabRows * N; i += NT) lco[i] = ctab[i];
  const double* ca = lco;
  const double* cb = lco + N;
  const double* cc = lco + 2 * N;
  const double* gsc = lco + 3 * N;
  const double* W = ctab + kCtabRows * N;

  if (tid < MB) {
    int mi = m0 + tid;
    double kk = 0.0;
    int keep = 0;
    if (mi < nmodes) mode_wave(g, mi, kk, keep);
    s_k[tid] = kk;
    s_kap[tid] = kk * Rz;
    s_keep[tid] = keep;
  }

  // the plan-time chain multipliers of the block's modes (N MB values), and
  // the functional weights W when they fit the spare storage, are fetched
  // into registers now and put in LDS once the buffers they share are free
  constexpr int kCp = KE / (2 * NT) + 1;  // >= N MB / NT
  constexpr int kWr = 3072 / NT;                // W staged when 10 (N+2) <= 3072
  double cpr[kCp], wr[kWr];
#pragma unroll
  for (int q = 0; q < kCp; ++q) {
    const int t = tid + q * NT, row = t >> logMB, m = t & (MB - 1);
    cpr[q] = (row < N && m0 + m < nmodes) ? cpiv[(size_t)row * nmodes + m0 + m] : 0.0;
  }
  const bool w_lds = kNumFun * NU <= kWr * NT && kNumFun * NU <= 2 * (N - 2) * MB;
  if (w_lds) {
#pragma unroll
    for (int q = 0; q < kWr; ++q) {
      const int t = tid + q * NT;
      wr[q] = t < kNumFun * NU ? W[t] : 0.0;
    }
  }

  for (int i = tid; i < M / 2; i += NT) tw[i] = twz[i];
  // 1. even extension of the node values in bit-reversed order, then FFT;
  //    slot p takes node j = bitrev(p) (each z row is a separate contiguous
  //    piece of MB modes in global memory, so the reversal costs the loads
  //    nothing, and the LDS stores run in order); all global loads of the
  //    thread are issued before the stores
  {
    constexpr int kPer = KE / NT;  // M * MB == KE
    C va[kPer], vb[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = tid + q * NT;
      const int j = bitrev(t >> logMB, logM), m = t & (MB - 1), mi = m0 + m;
      const int c = j < N ? j : M - j;
      va[q].x = 0; va[q].y = 0; vb[q].x = 0; vb[q].y = 0;
      if (mi < nmodes) {
        const size_t o = (size_t)c * nmodes + mi;
        va[q] = fx_i[o];
        if (in_band(g, c)) vb[q] = fx_o[o];
      }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = tid + q * NT;
      A[t] = make_double2((double)vb[q].x, (double)vb[q].y);
      B[t] = make_double2((double)va[q].x, (double)va[q].y);
    }
  }
  __syncthreads();
  fft2<KE, NT>(A, B, logM, logMB, tw, tid);

  // spare storage beyond index N of each buffer (N-2 complex = 2N-4 doubles per mode)
  double* spA = reinterpret_cast<double*>(A + N * MB);  // chain pivots
  double* spB = reinterpret_cast<double*>(B + N * MB);  // homogeneous solutions
  // per mode, a row of cst doubles: index par * ceil(N/2) + r for row r of
  // the parity-par chain (fits: MB (N + 8) <= 2 (N - 2) MB for N >= 12)
  const int cst = N + 8;
  auto spare = [&](double* base, int m, int idx) -> double& { return base[m * cst + idx]; };
  const int half0 = (N + 1) / 2;  // rows of the even chain
  double* s_fun = lco + kCtabRows * N;  // [MB][10][6]
#pragma unroll
  for (int q = 0; q < kCp; ++q) {
    const int t = tid + q * NT, row = t >> logMB, m = t & (MB - 1);
    if (row < N) spare(spA, m, row) = cpr[q];
  }
  __syncthreads();
  // homogeneous y'' of chain parity n&1 at index n
  auto hval = [&](int m, int n) -> double { return spare(spB, m, (n & 1) * half0 + (n >> 1)); };

  // 2. tridiagonal chains: for each mode and parity, the mode equations in the
  //    unknowns y''_n of that parity, with right-hand sides Re/Im g of psi_i*,
  //    psi_o*, and the unit free constant (kappa^2 on the chain's first row).
  //    Twisted (two-ended) elimination: for every chain and right-hand side
  //    one thread eliminates downwards from the first row to the middle row
  //    t = L/2 and another upwards from the last row, with the plan's
  //    multipliers of each direction; both then form the middle unknown and
  //    substitute back outwards, so the serial recurrences are half as long.
  //    Four right-hand sides per chain (the first thread of each side also
  //    carries the free constant, whose right-hand side vanishes below row 0).
  constexpr int kSweep = 8;
  if (tid < 16 * MB) {
    const int side = tid >> (logMB + 3);         // 0: rows 0 .. t-1, 1: rows L-1 .. t+1
    const int u = tid & (8 * MB - 1);
    const int k = u >> (logMB + 1);              // right-hand side: 0 Re i, 1 Im i, 2 Re o, 3 Im o
    const int cm = u & (2 * MB - 1);
    const int m = cm & (MB - 1), par = cm >> logMB;
    // row r of the chain: X at Xp[r * s4], coefficients at ap[2 r] etc., multiplier at crow[r]
    double* Xp = reinterpret_cast<double*>(k < 2 ? B : A) + 2 * m + (k & 1) + par * 2 * MB;
    const int s4 = 4 * MB;
    const double* ap = ca + par;
    const double* bp = cb + par;
    const double* cp = cc + par;
    const double* gp = gsc + par;
    const double* crow = spA + m * cst + par * half0;
    double* hrow = spB + m * cst + par * half0;
    const double kap2 = s_kap[m] * s_kap[m];
    const int L = par == 0 ? (N + 1) / 2 : N / 2, mt = L / 2;
    // rows go in groups of kSweep: the LDS operands of a group are loaded
    // together and its results stored together, so the serial recurrence
    // runs on registers and the LDS latency is paid once per group
    if (side == 0) {
      // d_r = (g_r x_r - sub_r d_{r-1}) / (dia_r - sub_r cp_{r-1})
      double d = 0.0, dh = 0.0;
      auto row = [&](int r, double av, double bv, double gv, double xv, double pv, double& dv, double& hv) {
        const double inv = rcp_refined(fma(kap2 * av, pv, fma(kap2, bv, 1.0)));
        const double sub = -kap2 * av;
        d = (gv * xv - sub * d) * inv;
        dh = ((r == 0 ? kap2 : 0.0) - sub * dh) * inv;
        dv = d;
        hv = dh;
      };
      int r0 = 0;
      for (; r0 + kSweep <= mt; r0 += kSweep) {
        double av[kSweep], bv[kSweep], gv[kSweep], xv[kSweep], pv[kSweep], dv[kSweep], hv[kSweep];
#pragma unroll
        for (int q = 0; q < kSweep; ++q) {
          const int r = r0 + q;
          av[q] = ap[2 * r];
          bv[q] = bp[2 * r];
          gv[q] = gp[2 * r];
          xv[q] = Xp[r * s4];
          pv[q] = r > 0 ? crow[r - 1] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kSweep; ++q) row(r0 + q, av[q], bv[q], gv[q], xv[q], pv[q], dv[q], hv[q]);
#pragma unroll
        for (int q = 0; q < kSweep; ++q) Xp[(r0 + q) * s4] = dv[q];
        if (k == 0) {
#pragma unroll
          for (int q = 0; q < kSweep; ++q) hrow[r0 + q] = hv[q];
        }
      }
      for (int r = r0; r < mt; ++r) {
        double dv, hv;
        row(r, ap[2 * r], bp[2 * r], gp[2 * r], Xp[r * s4], r > 0 ? crow[r - 1] : 0.0, dv, hv);
        Xp[r * s4] = dv;
        if (k == 0) hrow[r] = hv;
      }
    } else {
      // e_r = (g_r x_r - sup_r e_{r+1}) / (dia_r - sup_r cq_{r+1}); the free
      // constant's right-hand side is zero here
      double e = 0.0;
      auto row = [&](double cv, double bv, double gv, double xv, double qv) {
        const double inv = rcp_refined(fma(kap2 * cv, qv, fma(kap2, bv, 1.0)));
        const double sup = -kap2 * cv;
        e = (gv * xv - sup * e) * inv;
        return e;
      };
      int r0 = L - 1;  // rows r0, r0 - 1, ..., r0 - kSweep + 1 > mt
      for (; r0 - kSweep >= mt; r0 -= kSweep) {
        double cv[kSweep], bv[kSweep], gv[kSweep], xv[kSweep], qv[kSweep], ev[kSweep];
#pragma unroll
        for (int q = 0; q < kSweep; ++q) {
          const int r = r0 - q;
          cv[q] = cp[2 * r];
          bv[q] = bp[2 * r];
          gv[q] = gp[2 * r];
          xv[q] = Xp[r * s4];
          qv[q] = r < L - 1 ? crow[r + 1] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kSweep; ++q) ev[q] = row(cv[q], bv[q], gv[q], xv[q], qv[q]);
#pragma unroll
        for (int q = 0; q < kSweep; ++q) Xp[(r0 - q) * s4] = ev[q];
        if (k == 0) {
#pragma unroll
          for (int q = 0; q < kSweep; ++q) hrow[r0 - q] = 0.0;
        }
      }
      for (int r = r0; r > mt; --r) {
        Xp[r * s4] = row(cp[2 * r], bp[2 * r], gp[2 * r], Xp[r * s4], r < L - 1 ? crow[r + 1] : 0.0);
        if (k == 0) hrow[r] = 0.0;
      }
    }
  }
  __syncthreads();
  {
    // the middle row from both sides' eliminations, then back substitution:
    // x_r = d_r - cp_r x_{r+1} above it, x_r = e_r - cq_r x_{r-1} below it
    double xm = 0.0, xhm = 0.0;
    int side = 0, k = 0, mt = 0, L = 0, s4 = 4 * MB;
    double* Xp = nullptr;
    double* hrow = nullptr;
    const double* crow = nullptr;
    if (tid < 16 * MB) {
      side = tid >> (logMB + 3);
      const int u = tid & (8 * MB - 1);
      k = u >> (logMB + 1);
      const int cm = u & (2 * MB - 1);
      const int m = cm & (MB - 1), par = cm >> logMB;
      Xp = reinterpret_cast<double*>(k < 2 ? B : A) + 2 * m + (k & 1) + par * 2 * MB;
      crow = spA + m * cst + par * half0;
      hrow = spB + m * cst + par * half0;
      const double kap2 = s_kap[m] * s_kap[m];
      L = par == 0 ? (N + 1) / 2 : N / 2;
      mt = L / 2;
      const double sub = -kap2 * ca[par + 2 * mt], sup = -kap2 * cc[par + 2 * mt];
      const double itw = crow[mt];  // 1 / (dia_t - sub_t cp_{t-1} - sup_t cq_{t+1})
      xm = (gsc[par + 2 * mt] * Xp[mt * s4] - sub * Xp[(mt - 1) * s4] - sup * Xp[(mt + 1) * s4]) * itw;
      xhm = (-sub * hrow[mt - 1] - sup * hrow[mt + 1]) * itw;
    }
    __syncthreads();  // every read of the middle row precedes its overwrite
    if (tid < 16 * MB) {
      double x = xm, xh = xhm;
      // rows r = a + dir q in groups of kSweep, with the same loads-first layout
      const int dir = side == 0 ? -1 : 1;
      int a = side == 0 ? mt - 1 : mt + 1;
      const int cnt = side == 0 ? mt : L - 1 - mt;
      if (side == 0) {
        Xp[mt * s4] = xm;
        if (k == 0) hrow[mt] = xhm;
      }
      int done = 0;
      for (; done + kSweep <= cnt; done += kSweep, a += dir * kSweep) {
        double cv[kSweep], xv[kSweep], hv[kSweep];
#pragma unroll
        for (int q = 0; q < kSweep; ++q) {
          const int r = a + dir * q;
          cv[q] = crow[r];
          xv[q] = Xp[r * s4];
          hv[q] = hrow[r];
        }
#pragma unroll
        for (int q = 0; q < kSweep; ++q) {
          x = fma(-cv[q], x, xv[q]);
          xh = fma(-cv[q], xh, hv[q]);
          xv[q] = x;
          hv[q] = xh;
        }
#pragma unroll
        for (int q = 0; q < kSweep; ++q) Xp[(a + dir * q) * s4] = xv[q];
        if (k == 0) {
#pragma unroll
          for (int q = 0; q < kSweep; ++q) hrow[a + dir * q] = hv[q];
        }
      }
      for (; done < cnt; ++done, a += dir) {
        const double c = crow[a];
        x = fma(-c, x, Xp[a * s4]);
        xh = fma(-c, xh, hrow[a]);
        Xp[a * s4] = x;
        if (k == 0) hrow[a] = xh;
      }
    }
  }
  __syncthreads();

  // 3. linear functionals of each solution vector: dot products of y'' (and
  //    the free constants) with the plan's weight vectors S1..S4 (boundary
  //    rows), V0, VH, D0, DH (values and z-derivatives at z = 0, H), Ea, Eb
  //    (slopes at the domain ends). One thread per (mode, weight vector) sums
  //    over all indices for six vectors: psi_i* re/im, psi_o* re/im, h1, h2.
  //    s_fun[(m * 10 + f) * 6 + v].
  //    Two lanes (adjacent, same wave) share a dot product: each sums half
  //    of the indices and a lane exchange adds the halves.
  //    The weights come from LDS (the multipliers' storage, free after the
  //    back substitution) when they fit there, else from global memory.
  if (w_lds) {
#pragma unroll
    for (int q = 0; q < kWr; ++q) {
      const int t = tid + q * NT;
      if (t < kNumFun * NU) spA[t] = wr[q];
    }
  }
  __syncthreads();
  auto functionals = [&](const double* Wsrc) {
    for (int t = tid; t < MB * 20; t += NT) {
      const int pr = t >> 1, part = t & 1;
      const int m = pr / 10, f = pr - 10 * m;
      const double* Wf = Wsrc + f * NU;
      const int jh = (N + 1) / 2, ja = part ? jh : 0, jb = part ? N : jh;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = part ? 0.0 : Wf[N], a5 = part ? 0.0 : Wf[N + 1];
#pragma unroll 4
      for (int j = ja; j < jb; ++j) {
        const double w = Wf[j];
        const double2 xi = B[j * MB + m], xo = A[j * MB + m];
        const double hv = hval(m, j);
        a0 = fma(w, xi.x, a0);
        a1 = fma(w, xi.y, a1);
        a2 = fma(w, xo.x, a2);
        a3 = fma(w, xo.y, a3);
        if (j & 1) a5 = fma(w, hv, a5); else a4 = fma(w, hv, a4);
      }
      a0 += __shfl_xor(a0, 1, 64);
      a1 += __shfl_xor(a1, 1, 64);
      a2 += __shfl_xor(a2, 1, 64);
      a3 += __shfl_xor(a3, 1, 64);
      a4 += __shfl_xor(a4, 1, 64);
      a5 += __shfl_xor(a5, 1, 64);
      if (part == 0) {
        double* o = s_fun + (m * 10 + f) * 6;
        o[0] = a0; o[1] = a1; o[2] = a2; o[3] = a3; o[4] = a4; o[5] = a5;
      }
    }
  };
  if (w_lds) functionals(spA);
  else functionals(W);
  __syncthreads();

  // 4. per mode: free constants, wall values, mismatches, harmonic correction, k = 0
  if (tid < MB) {
    const int m = tid;
    const double* F = s_fun + m * 60;  // F[f * 6 + v]
    const double kap = s_kap[m];
    const bool dir = !(s_k[m] > 0.0);
    // boundary rows: Robin top S1 + kap S2, bottom S3 - kap S4; Dirichlet S2, S4
    auto top = [&](int v) { return dir ? F[FUN_S2 * 6 + v] : fma(kap, F[FUN_S2 * 6 + v], F[FUN_S1 * 6 + v]); };
    auto bot = [&](int v) { return dir ? F[FUN_S4 * 6 + v] : fma(-kap, F[FUN_S4 * 6 + v], F[FUN_S3 * 6 + v]); };
    const double t1 = top(4), t2 = top(5), b1 = bot(4), b2 = bot(5);
    const double det = t1 * b2 - t2 * b1;
    auto solve2 = [&](double tP, double bP, double& c0, double& c1) {
      c0 = -(tP * b2 - t2 * bP) / det;
      c1 = -(t1 * bP - tP * b1) / det;
    };
    double ci0r, ci1r, ci0i, ci1i, co0r, co1r, co0i, co1i;
    solve2(top(0), bot(0), ci0r, ci1r);
    solve2(top(1), bot(1), ci0i, ci1i);
    solve2(top(2), bot(2), co0r, co1r);
    solve2(top(3), bot(3), co0i, co1i);
    s_c[m][0] = make_double2(ci0r, ci0i);
    s_c[m][1] = make_double2(ci1r, ci1i);
    // functional f of the final solutions: particular + y_0 h1 + y'_0 h2
    auto fin_i = [&](int f) {
      return make_double2(F[f * 6 + 0] + ci0r * F[f * 6 + 4] + ci1r * F[f * 6 + 5],
                          F[f * 6 + 1] + ci0i * F[f * 6 + 4] + ci1i * F[f * 6 + 5]);
    };
    auto fin_o = [&](int f) {
      return make_double2(F[f * 6 + 2] + co0r * F[f * 6 + 4] + co1r * F[f * 6 + 5],
                          F[f * 6 + 3] + co0i * F[f * 6 + 4] + co1i * F[f * 6 + 5]);
    };
    const double2 vi0 = fin_i(FUN_V0), viH = fin_i(FUN_VH), di0 = fin_i(FUN_D0), diH = fin_i(FUN_DH);
    const double2 vo0 = fin_o(FUN_V0), voH = fin_o(FUN_VH), do0 = fin_o(FUN_D0), doH = fin_o(FUN_DH);
    const double k = s_k[m];
    double2 al = make_double2(0, 0), be = make_double2(0, 0);
    double Ai = 0.0;
    if (k > 0.0 && s_keep[m]) {
      const double e = g.eps, eb = g.eps_b, et = g.eps_t, tb = g.tau_b, tt = g.tau_t;
      // mismatches (eqs. mm1-mm4, no wall charges)
      double2 mpb = make_double2(vi0.x - tb * vo0.x, vi0.y - tb * vo0.y);
      double2 meb = make_double2(e * di0.x - eb * tb * do0.x, e * di0.y - eb * tb * do0.y);
      double2 mpt = make_double2(viH.x - tt * voH.x, viH.y - tt * voH.y);
      double2 met = make_double2(e * diH.x - et * tt * doH.x, e * diH.y - et * tt * doH.y);
      if (wall_hat) {  // wall charges: + sigma_b in mm2, - sigma_t in mm4
        const double2 sb = wall_hat[m0 + m], st = wall_hat[nmodes + m0 + m];
        meb.x += sb.x;
        meb.y += sb.y;
        met.x -= st.x;
        met.y -= st.y;
      }
      double2 Rb = make_double2((eb * k * mpb.x - meb.x) / k, (eb * k * mpb.y - meb.y) / k);
      double2 Rt = make_double2(-(met.x + et * k * mpt.x) / k, -(met.y + et * k * mpt.y) / k);
      double E = exp(-k * g.H);
      double D = (e + eb) * (e + et) - (eb - e) * (et - e) * E * E;
      al = make_double2((Rb.x * (et - e) * E + (e + eb) * Rt.x) / D, (Rb.y * (et - e) * E + (e + eb) * Rt.y) / D);
      be = make_double2(((e - eb) * E * Rt.x - (e + et) * Rb.x) / D, ((e - eb) * E * Rt.y - (e + et) * Rb.y) / D);
    }
    if (m0 + m == 0) {
      if (g.flags & DPSE_UNIFORM_FAST) {
        // free space (Sec. 3.1.1): the field of the neutral set vanishes
        // outside the sources, so A_i cancels psi_i*' at both domain ends
        Ai = -0.5 * (fin_i(FUN_EA).x + fin_i(FUN_EB).x);
      } else {
        const double e = g.eps, tb = g.tau_b, tt = g.tau_t;
        const double2 ea = fin_o(FUN_EA), ebd = fin_o(FUN_EB);
        double Ab = -tb * ea.x, At = -tt * ebd.x;
        double A1 = (g.eps_b * (tb * do0.x + Ab) - e * di0.x) / e;
        double A2 = (g.eps_t * (tt * doH.x + At) - e * diH.x) / e;
        if (wall_hat) {  // wall charges in eqs. ai1, ai2
          A1 -= wall_hat[0].x / e;
          A2 += wall_hat[nmodes].x / e;
        }
        Ai = 0.5 * (A1 + A2);
      }
      scal[3] = Ai;
    }
    s_ab[m][0] = al;
    s_ab[m][1] = be;
    s_Ai[m] = Ai;
  }
  __syncthreads();

  // 5. final series of psi_i* into A: y_n = Y[n].(P) + y_0 Y[n].(h1) + y'_0 Y[n].(h2)
  for (int t = tid; t < N * MB; t += NT) {
    const int n = t >> logMB, m = t & (MB - 1);
    double2 yP = make_double2(0.0, 0.0);
    double yh = 0.0;
    if (n >= 1) {
      const double a = ca[n], b = cb[n], c = cc[n];
      double2 x0 = B[n * MB + m];
      double h0 = hval(m, n);
      yP.x = -b * x0.x;
      yP.y = -b * x0.y;
      yh = -b * h0;
      if (n >= 2) {
        double2 xm = B[(n - 2) * MB + m];
        yP.x = fma(a, xm.x, yP.x);
        yP.y = fma(a, xm.y, yP.y);
        yh = fma(a, hval(m, n - 2), yh);
      }
      if (n + 2 < N) {
        double2 xp = B[(n + 2) * MB + m];
        yP.x = fma(c, xp.x, yP.x);
        yP.y = fma(c, xp.y, yP.y);
        yh = fma(c, hval(m, n + 2), yh);
      }
    }
    if (n <= 1) yh += 1.0;  // y_0 = 1 in h1; y_1 = y'_0 + ... with y'_0 = 1 in h2
    const double2 cf = s_c[m][n & 1];
    A[n * MB + m] = make_double2(fma(cf.x, yh, yP.x), fma(cf.y, yh, yP.y));
  }
  __syncthreads();

  // 6. derivative series into B: d_j = (2/R) sum_{m > j, m = j+1 mod 2} m y_m
  //    (d_{N-1} = 0, d_0 halved), a suffix sum per mode and parity: all
  //    2 MB chains at once, G lanes per chain (the chains of a wave side by
  //    side), lanes own consecutive entries, scanned from the top.
  {
    constexpr int kW = NT / 64;                 // waves
    const int cpw = (2 * MB + kW - 1) / kW;     // chains per wave (a power of two)
    const int G = 64 / cpw;                     // lanes per chain
    const int ch = tid / G, gl = tid & (G - 1);
    const double ir = 1.0 / Rz;
    if (ch < 2 * MB) {  // whole lane groups
      const int m = ch & (MB - 1), q = ch >> logMB;  // q: parity of the output index j
      // outputs j = q, q+2, ... <= N-1; entry t (from the top) is j = jt - 2t
      const int jt = (N - 1) - (((N - 1) - q) & 1);
      const int Lc = jt / 2 + 1;
      const int E = (Lc + G - 1) / G;
      const int t0 = gl * E, t1 = min(Lc, t0 + E);
      double sx = 0.0, sy = 0.0;
      for (int t = t0; t < t1; ++t) {
        const int j = jt - 2 * t;
        if (j + 1 < N) {
          const double2 y = A[(j + 1) * MB + m];
          const double f = 2.0 * (j + 1);
          sx = fma(f, y.x, sx);
          sy = fma(f, y.y, sy);
        }
      }
      for (int o = 1; o < G; o <<= 1) {
        const double cx = __shfl_up(sx, o, G), cy = __shfl_up(sy, o, G);
        if (gl >= o) { sx += cx; sy += cy; }
      }
      double ax = __shfl_up(sx, 1, G), ay = __shfl_up(sy, 1, G);
      if (gl == 0) { ax = 0.0; ay = 0.0; }
      for (int t = t0; t < t1; ++t) {
        const int j = jt - 2 * t;
        if (j + 1 < N) {
          const double2 y = A[(j + 1) * MB + m];
          const double f = 2.0 * (j + 1);
          ax = fma(f, y.x, ax);
          ay = fma(f, y.y, ay);
        }
        const double sc = (j == 0) ? 0.5 * ir : ir;
        B[j * MB + m] = make_double2(sc * ax, sc * ay);
      }
    }
  }
  __syncthreads();

  // 7. inverse DCT-I of A (series) and B (derivative series): v_j = 1/2 FFT(e)[j]
  //    with e the even extension of (2 c_0, c_1, ..., c_{N-2}, 2 c_{N-1})
  {
    constexpr int kPer = kElems / NT;  // M * MB == kElems
    double2 ra[kPer], rb[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      int t = tid + q * NT;
      int j = t >> logMB, m = t & (MB - 1);
      int n = j < N ? j : M - j;
      double f = (n == 0 || n == N - 1) ? 2.0 : 1.0;
      double2 a = A[n * MB + m], b = B[n * MB + m];
      ra[q] = make_double2(f * a.x, f * a.y);
      rb[q] = make_double2(f * b.x, f * b.y);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      int t = tid + q * NT;
      int j = t >> logMB, m = t & (MB - 1);
      int pos = bitrev(j, logM) * MB + m;
      A[pos] = ra[q];
      B[pos] = rb[q];
    }
    __syncthreads();
  }
  fft2<KE, NT>(A, B, logM, logMB, tw, tid);

  // 8. add the correction at the window nodes and the k = 0 linear mode; write out
  for (int t = tid; t < N * MB; t += NT) {
    int j = t >> logMB, m = t & (MB - 1), mi = m0 + m;
    if (mi >= nmodes) continue;
    double2 v = A[j * MB + m], d = B[j * MB + m];
    double ps_x = 0.5 * v.x, ps_y = 0.5 * v.y, pz_x = 0.5 * d.x, pz_y = 0.5 * d.y;
    double z = zn[j];
    double k = s_k[m];
    if (k > 0.0 && s_keep[m] && z >= -g.H_E && z <= g.H + g.H_E) {
      // the exponentials in the storage precision of Psi (FP32 in the mixed
      // path: no overflow, |k z| <= pi n_g / 2 + k H), the sums in FP64
      double e1, e2;
      if (sizeof(R) == 8) {
        e1 = exp(k * (z - g.H));
        e2 = exp(-k * z);
      } else {
        e1 = (double)expf((float)(k * (z - g.H)));
        e2 = (double)expf((float)(-k * z));
      }
      double2 al = s_ab[m][0], be = s_ab[m][1];
      ps_x += al.x * e1 + be.x * e2;
      ps_y += al.y * e1 + be.y * e2;
      pz_x += k * (al.x * e1 - be.x * e2);
      pz_y += k * (al.y * e1 - be.y * e2);
    }
    if (mi == 0) {
      ps_x += s_Ai[m] * z;
      pz_x += s_Ai[m];
    }
    size_t o = (size_t)j * nmodes + mi;
    C a, b;
    a.x = (R)ps_x; a.y = (R)ps_y;
    b.x = (R)pz_x; b.y = (R)pz_y;
    psi[o] = a;
    psiz[o] = b;
  }
}

// ---------------------------------------------------------------------------
// Column solve for Nz <= 257 with every phase spread over all lanes. Same
// mathematics as k_column (Sec. 5.2.2 steps 2-6, App. A); what differs is the
// work split:
//  * the z transforms run in the storage precision (FP32 in the mixed path,
//    where the Chebyshev transform is one of the FFTs; FP64 otherwise);
//  * the chains are solved with the plan's LU factors (inverse pivots per
//    mode, mode-major) by a segmented scan: lane (mode, parity, segment)
//    owns about four consecutive rows of one chain for all five right-hand
//    sides (Re/Im of psi_i*, Re/Im of psi_o*, the unit free constant), sweeps
//    them with carry 0 while forming the product of the multipliers, and the
//    carries of the segments come from an inclusive scan of those affine maps
//    over the lanes of the chain; back substitution likewise, from the top;
//  * the linear functionals are partial dot products over each lane's rows,
//    summed over the segments by a reduce-scatter (each lane ends with a few
//    of the sums, which it stores);
//  * the final series, its exact derivative (a segmented suffix sum) and the
//    even extension for the inverse transform are formed in the same lanes
//    and written straight to LDS.
// Cross-lane steps use DPP row and wave moves (VALU) where the partner lies
// in the same row of 16 lanes or one lane away, LDS permutes otherwise.
// KE = 2048 complex elements per transform buffer, 256 threads: for S = 2^LOGS
// segments per chain, M = 2(Nz - 1) = 16 S, MB = KE / M = 128 / S modes per
// block, 2 S MB = 256 lanes; LOGS = 2..5 for Nz = 33..257. LDS rows j of a
// buffer are padded by one element every 2^(LOGS - 2) rows (element (j, m) at
// j MB + m + (j >> (LOGS - 2))), which keeps the chain lanes' row reads and
// the bit-reversed stores of the inverse transform off shared banks.
constexpr int kScanKE = 2048;
constexpr int kScanNT = 256;
constexpr int kScanRows = 5;   // rows per lane: ceil(L / S) <= ceil(4 (Nz + 1) / (Nz - 1)) = 5
constexpr int kNumFunBC = 8;   // S1..S4, V0, VH, D0, DH (Ea, Eb only for k = 0)

// Plan-time LU factorisation of the chains of k_column_scan: for each mode
// and parity, the inverse pivots 1 / (dia_r - sub_r c_{r-1}) with c_r = sup_r
// times the inverse pivot, at cinv[mode * Nz + parity * ceil(Nz/2) + r].
// The same pass forms the functionals S1..DH of the chain's homogeneous
// solution (right-hand side kappa^2 in row 0): with the forward sweep
// d_r = al_r d_{r-1} + inv_r rhs_r and the back substitution x_r = d_r +
// gam_r x_{r+1} (U x = d), a functional w.x equals y.d with U^T y = w, i.e.
// y_r = w_r + gam_{r-1} y_{r-1}: both recurrences run forward, so one sweep
// gives all eight (plus the free constant's weight), stored at
// hfun[mode * 16 + parity * 8 + f].
__global__ void __launch_bounds__(kThreads) k_pivots_scan(Geom g, const double* __restrict__ ctab,
                                                          double* __restrict__ cinv, double* __restrict__ hfun) {
  const int nmodes = g.Ny * g.nkx, N = g.Nz;
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= 2 * nmodes) return;
  const int mi = t >> 1, par = t & 1;
  double kk;
  int keep;
  mode_wave(g, mi, kk, keep);
  const double kap = kk * g.zR, kap2 = kap * kap;
  const int half0 = (N + 1) / 2, L = par == 0 ? half0 : N / 2;
  const int NU = N + 2;
  const double* W = ctab + kCtabRows * N;
  double* out = cinv + (size_t)mi * N + par * half0;
  double cp = 0.0, d = 0.0, gprev = 0.0;
  double y[kNumFunBC], F[kNumFunBC];
#pragma unroll
  for (int f = 0; f < kNumFunBC; ++f) { y[f] = 0.0; F[f] = 0.0; }
  for (int r = 0; r < L; ++r) {
    const int n = par + 2 * r;
    const double sub = -kap2 * ctab[n], dia = fma(kap2, ctab[N + n], 1.0), sup = -kap2 * ctab[2 * N + n];
    const double inv = rcp_refined(fma(-sub, cp, dia));
    out[r] = inv;
    cp = sup * inv;
    // the column kernel's multipliers: al_r = kappa^2 a_n inv_r, gam_r = kappa^2 c_n inv_r
    const double al = kap2 * ctab[n] * inv, gam = kap2 * ctab[2 * N + n] * inv;
    d = fma(al, d, inv * (r == 0 ? kap2 : 0.0));
#pragma unroll
    for (int f = 0; f < kNumFunBC; ++f) {
      y[f] = fma(gprev, y[f], W[f * NU + n]);
      F[f] = fma(y[f], d, F[f]);
    }
    gprev = gam;
  }
  double* h = hfun + (size_t)mi * 16 + par * 8;
#pragma unroll
  for (int f = 0; f < kNumFunBC; ++f) h[f] = F[f] + W[f * NU + N + par];
}

// DPP controls (GFX9 encoding).
constexpr int kDppQuadXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppRowShl = 0x100;       // + n: lane i takes lane i + n of its row of 16
constexpr int kDppRowShr = 0x110;       // + n: lane i takes lane i - n of its row of 16
constexpr int kDppWaveShl1 = 0x130;     // lane i takes lane i + 1 of the wave
constexpr int kDppWaveShr1 = 0x138;     // lane i takes lane i - 1 of the wave
constexpr int kDppRowMirror = 0x140;    // lane i takes lane 15 - i of its row
constexpr int kDppRowHalfMirror = 0x141;  // lane i takes lane 7 - i of its half row
constexpr int kDppRowBcast15 = 0x142;   // rows 1, 3 take lane 15 of the row below

// A DPP move of a double (both halves); lanes without a source read 0.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The same move with 1.0 where there is no source lane (or the row is masked
// off): the identity of a product, so that a scan step needs no branch.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_one(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0x3FF00000, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Decimation-in-time FFTs of the MB sequences of both buffers in lockstep
// (input in bit-reversed order, output natural), with the padded row layout,
// in passes of three radix-2 stages (two where the stage count requires);
// forward twiddles tw[k] = exp(-2 pi i k / M).
template <typename C, int LOGS>
__device__ __forceinline__ void fft_scan_pair(C* A, C* B, const C* tw, int tid) {
  constexpr int LOGM = LOGS + 4, M = 1 << LOGM, LOGMB = 7 - LOGS, MB = 1 << LOGMB, PS = LOGS - 2;
  constexpr int NT = kScanNT;
  auto ix = [](int k, int s) { return k * MB + s + (k >> PS); };
  using Rr = decltype(C{}.x);
  // radix-2^3 pass fusing the stages lh, lh + 1, lh + 2 on eight elements
  // k0 + e half (one group per thread and buffer); the twiddles of the two
  // later stages are those of the first kind times -i and powers of
  // exp(-i pi / 4). The first pass maps consecutive threads to consecutive
  // groups of one sequence where that keeps its LDS accesses off shared banks.
  // Element addresses: ix(k0 + e half, s) = base + e stride when the padding
  // term (k >> PS) is linear in e, i.e. for half >= 2^PS (every pass after the
  // first, half >= 8 >= 2^PS) and, in the first pass (half = 1, k0 a multiple
  // of 8), for PS = 0 or PS >= 3.
  auto pass8 = [&](auto first_tag, int lh, bool gfast) {
    constexpr bool FIRST = decltype(first_tag)::value;
    constexpr int LG = LOGM - 3;  // groups per sequence: M / 8
    if constexpr (FIRST) lh = 0;
    const int half = 1 << lh, ts1 = (M >> 1) >> lh, ts2 = ts1 >> 1, ts3 = ts1 >> 2;
    int s, b;
    if (gfast) {
      b = tid & ((1 << LG) - 1);
      s = tid >> LG;
    } else {
      s = tid & (MB - 1);
      b = tid >> LOGMB;
    }
    const int grp = b >> lh, pos = b & (half - 1);
    const int k0 = (grp << (lh + 3)) + pos;
    constexpr bool kLin = !FIRST || PS == 0 || PS >= 3;
    const int base = ix(k0, s), stride = half * MB + (half >> PS);
    auto at = [&](int e) { return kLin ? base + e * stride : ix(k0 + e * half, s); };
    const C w1 = tw[pos << __builtin_ctz(ts1)], w2 = tw[pos << __builtin_ctz(ts2)], w3 = tw[pos << __builtin_ctz(ts3)];
    C a[2][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[0][e] = A[at(e)];
      a[1][e] = B[at(e)];
    }
    const Rr r2 = (Rr)0.70710678118654752440;
    C w2m, w3e[4];  // w2 times -i; w3 times exp(-i pi e / 4)
    w2m.x = w2.y;
    w2m.y = -w2.x;
    w3e[0] = w3;
    w3e[1].x = r2 * (w3.x + w3.y);
    w3e[1].y = r2 * (w3.y - w3.x);
    w3e[2].x = w3.y;
    w3e[2].y = -w3.x;
    w3e[3].x = r2 * (w3.y - w3.x);
    w3e[3].y = -r2 * (w3.x + w3.y);
    if (sizeof(Rr) == 4 && FIRST) {
      // first pass: every twiddle is 1, -i or exp(-i pi e / 4) (no products
      // with table values; FP32 only, where the registers allow the second
      // code path)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        C* v = a[bi];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          const C t = v[e + 1];
          v[e + 1] = csub(v[e], t);
          v[e] = cadd(v[e], t);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if (e & 2) continue;
          C t = v[e + 2];
          if (e & 1) {  // times -i
            const Rr re = t.x;
            t.x = t.y;
            t.y = -re;
          }
          v[e + 2] = csub(v[e], t);
          v[e] = cadd(v[e], t);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          C t = v[e + 4];
          const Rr x = t.x, y = t.y;
          if (e == 1) { t.x = r2 * (x + y); t.y = r2 * (y - x); }
          if (e == 2) { t.x = y; t.y = -x; }
          if (e == 3) { t.x = r2 * (y - x); t.y = -r2 * (x + y); }
          v[e + 4] = csub(v[e], t);
          v[e] = cadd(v[e], t);
        }
      }
    } else {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        C* v = a[bi];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          const C t = cmul(v[e + 1], w1);
          v[e + 1] = csub(v[e], t);
          v[e] = cadd(v[e], t);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if (e & 2) continue;
          const C t = cmul(v[e + 2], (e & 1) ? w2m : w2);
          v[e + 2] = csub(v[e], t);
          v[e] = cadd(v[e], t);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const C t = cmul(v[e + 4], w3e[e]);
          v[e + 4] = csub(v[e], t);
          v[e] = cadd(v[e], t);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      A[at(e)] = a[0][e];
      B[at(e)] = a[1][e];
    }
    __syncthreads();
  };
  // radix-2^2 pass (stages lh, lh + 1), two groups per thread and buffer
  auto pass4 = [&](int lh) {
    constexpr int BPT4 = M * MB / 4 / NT;
    const int half = 1 << lh, ts1 = (M >> 1) >> lh, ts2 = ts1 >> 1, st4 = half * MB + (half >> PS);
    C a[2][BPT4][4], w1[BPT4], w2[BPT4];
    int k0[BPT4];
#pragma unroll
    for (int q = 0; q < BPT4; ++q) {
      const int t = tid + q * NT, s = t & (MB - 1), b = t >> LOGMB;
      const int grp = b >> lh, pos = b & (half - 1);
      k0[q] = ix((grp << (lh + 2)) + pos, s);  // half >= 8 >= 2^PS: base + e stride
      w1[q] = tw[pos << __builtin_ctz(ts1)];
      w2[q] = tw[pos << __builtin_ctz(ts2)];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a[0][q][e] = A[k0[q] + e * st4];
        a[1][q][e] = B[k0[q] + e * st4];
      }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      C* buf = bi == 0 ? A : B;
#pragma unroll
      for (int q = 0; q < BPT4; ++q) {
        const C t1 = cmul(a[bi][q][1], w1[q]), t3 = cmul(a[bi][q][3], w1[q]);
        const C b0 = cadd(a[bi][q][0], t1), b1 = csub(a[bi][q][0], t1);
        const C b2 = cadd(a[bi][q][2], t3), b3 = csub(a[bi][q][2], t3);
        const C u2 = cmul(b2, w2[q]);
        C u3 = cmul(b3, w2[q]);  // times -i
        {
          const auto re = u3.x;
          u3.x = u3.y;
          u3.y = -re;
        }
        buf[k0[q]] = cadd(b0, u2);
        buf[k0[q] + 2 * st4] = csub(b0, u2);
        buf[k0[q] + st4] = cadd(b1, u3);
        buf[k0[q] + 3 * st4] = csub(b1, u3);
      }
    }
    __syncthreads();
  };
  // stage plans: 2^9 = 8 8 8, 2^8 = 8 8 4, 2^7 = 8 4 4, 2^6 = 8 8 (passes
  // in loops that are not unrolled: unrolled, their hoisted addresses cost
  // ~40 VGPRs)
  constexpr int n8 = LOGM == 7 ? 1 : LOGM / 3, n4 = (LOGM - 3 * n8) / 2;
  pass8(std::true_type{}, 0, LOGS >= 4);
#pragma nounroll
  for (int p = 1; p < n8; ++p) pass8(std::false_type{}, 3 * p, false);
#pragma nounroll
  for (int p = 0; p < n4; ++p) pass4(3 * n8 + 2 * p);
}

template <typename R, int LOGS>
__global__ void __launch_bounds__(kScanNT) k_column_scan(Geom g, const typename CT<R>::T* __restrict__ fx_i,
                                                         const typename CT<R>::T* __restrict__ fx_o,
                                                         typename CT<R>::T* __restrict__ psi,
                                                         typename CT<R>::T* __restrict__ psiz,
                                                         const double* __restrict__ zn,
                                                         const double* __restrict__ ctab,
                                                         const double2* __restrict__ twz,
                                                         const double* __restrict__ cinv,
                                                         const double* __restrict__ hfun, double* scal,
                                                         const double2* __restrict__ wall_hat) {
  using C = typename CT<R>::T;
  constexpr int KE = kScanKE, NT = kScanNT, RW = kScanRows;
  constexpr int S = 1 << LOGS, LOGM = LOGS + 4, M = 1 << LOGM, N = M / 2 + 1;
  constexpr int LOGMB = 7 - LOGS, MB = 1 << LOGMB, PS = LOGS - 2;
  constexpr int KEP = KE + (M >> PS);    // padded buffer length
  auto ix = [](int j, int m) { return j * MB + m + (j >> PS); };
  extern __shared__ double2 smem2[];
  C* A = reinterpret_cast<C*>(smem2);  // F_o, later the series of psi_i*
  C* B = A + KEP;                      // F_i, later the derivative series
  C* tw = B + KEP;                     // twiddles exp(-2 pi i k / M), k < M/2
  // reduced functionals [mode][parity][f][rhs] after the tables above
  double* sfun = reinterpret_cast<double*>(tw + M / 2);
  __shared__ double s_k[MB], s_kap[MB];
  __shared__ int s_keep[MB];
  __shared__ double2 s_c[MB][2];   // free constants (y_0, y'_0) of psi_i*
  __shared__ double2 s_ab[MB][2];  // correction alpha, beta
  __shared__ double s_Ai[MB];
  __shared__ double s_e[2][2][5];  // Ea, Eb of the k = 0 mode per parity and right-hand side

  constexpr int NU = N + 2;
  const int nmodes = g.Ny * g.nkx;
  const int m0 = xcd_block(blockIdx.x, gridDim.x) * MB;
  const int tid = threadIdx.x, lane = tid & 63;
  const double* W = ctab + kCtabRows * N;
  if (tid < MB) {
    const int mi = m0 + tid;
    double kk = 0.0;
    int keep = 0;
    if (mi < nmodes) mode_wave(g, mi, kk, keep);
    s_k[tid] = kk;
    s_kap[tid] = kk * g.zR;
    s_keep[tid] = keep;
  }
  for (int i = tid; i < M / 2; i += NT) {
    const double2 w = twz[i];
    C c;
    c.x = (R)w.x;
    c.y = (R)w.y;
    tw[i] = c;
  }

  // 1. even extension of the node values in bit-reversed order (slot p takes
  //    node bitrev(p)), all global loads first, then the forward transforms
  //    Thread tid takes slot rows (tid >> LOGMB) + q NT / MB, q < 8, so its
  //    nodes are bitrev(tid >> LOGMB) * 8 + bitrev3(q); byte offsets fit 32
  //    bits (N_z <= 257 nodes of at most 2^20 modes of 16 bytes). A mode
  //    beyond the last (the last block's tail) loads the last mode's values:
  //    its chains have no multipliers (zero solution) and it is never stored.
  {
    constexpr int kPer = KE / NT;
    static_assert(kPer == 8 && (NT >> LOGMB) * kPer == M, "eight slot rows per thread");
    const int mi_ld = min(m0 + (tid & (MB - 1)), nmodes - 1);
    const int jb = bitrev(tid >> LOGMB, LOGM - 3) << 3;
    const char* pi = reinterpret_cast<const char*>(fx_i);
    const char* po = reinterpret_cast<const char*>(fx_o);
    C va[kPer], vb[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int j = jb | (((q & 1) << 2) | (q & 2) | (q >> 2));
      const int c = j < N ? j : M - j;
      const unsigned off = (__umul24((unsigned)c, (unsigned)nmodes) + (unsigned)mi_ld) * (unsigned)sizeof(C);
      va[q] = *reinterpret_cast<const C*>(pi + off);
      vb[q].x = 0;
      vb[q].y = 0;
      if (in_band(g, c)) vb[q] = *reinterpret_cast<const C*>(po + off);
    }
    const int p0 = ix(tid >> LOGMB, tid & (MB - 1));
    constexpr int kRowStep = (NT >> LOGMB) * MB + ((NT >> LOGMB) >> PS);  // ix of NT / MB rows further
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      A[p0 + q * kRowStep] = vb[q];
      B[p0 + q * kRowStep] = va[q];
    }
  }
  // 2. the chains. Lane (m, par, seg): rows r0 .. r0 + cnt - 1 of chain par
  //    (unknowns y''_n, n = par + 2r) of mode m; a chain's S lanes are
  //    consecutive lanes of one wave. The lane's elimination multipliers are
  //    loaded before the forward transforms, which then cover their latency.
  const int seg = tid & (S - 1), par = (tid >> LOGS) & 1, m = tid >> (LOGS + 1);
  constexpr int half0 = (N + 1) / 2;
  // a chain has 4 S or 4 S + 1 rows: lane seg takes rows 4 seg .. 4 seg + 3,
  // and the last segment of the even chain one more (the partition
  // [seg L / S, (seg + 1) L / S) written out), so every lane has at least
  // RW - 1 rows; with FP32 transforms the
  // rows below RW - 1 are taken without a test, which lets their table loads
  // issue together (large slab column 4.43 -> 4.16 ms); the FP64 kernel
  // measured slower that way (6.7 -> 6.9 ms) and keeps the test
  static_assert((N / 2) == (RW - 1) * S && half0 == (RW - 1) * S + 1, "rows per lane");
  const int r0 = (RW - 1) * seg, cnt = RW - 1 + (par == 0 && seg == S - 1 ? 1 : 0);
  auto rows_all = [&](int q) { return (sizeof(R) == 4 && q < RW - 1) || q < cnt; };
  const int mi = m0 + m;
  const bool live = mi < nmodes;
  double invp[RW];
#pragma unroll
  for (int q = 0; q < RW; ++q) invp[q] = live && rows_all(q) ? cinv[(size_t)mi * N + par * half0 + r0 + q] : 0.0;
  __syncthreads();
  fft_scan_pair<C, LOGS>(A, B, tw, tid);
  const double kap2 = s_kap[m] * s_kap[m];
  // the plan's functionals of the homogeneous solutions that this lane stores
  // in phase 3 (loaded now, used after the chains)
  constexpr int NH = (kNumFunBC + S - 1) / S;
  double hpre[NH];
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    const int f = seg + j * S;
    hpre[j] = live && f < kNumFunBC ? hfun[(size_t)mi * 16 + par * 8 + f] : 0.0;
  }
  double X[RW][5];   // per row: Re psi_i*, Im psi_i*, Re psi_o*, Im psi_o*, homogeneous
  double gam[RW], PP[RW];
  {
    // forward elimination with carry 0: d_r = inv_r rhs_r + al_r d_{r-1},
    // al_r = kappa^2 a_n inv_r; PP holds the running product of the al
    double d[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, P = 1.0;
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      gam[q] = 0.0;
      if (rows_all(q)) {
        const int r = r0 + q, n = par + 2 * r;
        const double inv = invp[q];
        const double al = kap2 * ctab[n] * inv;
        gam[q] = kap2 * ctab[2 * N + n] * inv;  // back substitution: x_r = d_r + gam_r x_{r+1}
        const double gs = ctab[3 * N + n];
        const C fo = A[ix(n, m)], fi = B[ix(n, m)];
        const double rhs[5] = {gs * (double)fi.x, gs * (double)fi.y, gs * (double)fo.x, gs * (double)fo.y,
                               r == 0 ? kap2 : 0.0};
#pragma unroll
        for (int k = 0; k < 5; ++k) d[k] = fma(al, d[k], inv * rhs[k]);
        P *= al;
      }
#pragma unroll
      for (int k = 0; k < 5; ++k) X[q][k] = d[k];
      PP[q] = P;
    }
    // inclusive scan of the segment maps d_end = P d_in + d over the chain:
    // within rows of 16 lanes by DPP row shifts, then across the two rows
    double Ps = P, Ds[5] = {d[0], d[1], d[2], d[3], d[4]};
    // With 16 or 32 segments a lane takes a step exactly when the DPP move has
    // a source lane for it (the rows of 16 lanes are chains or halves of
    // one): lanes without one receive the identity map (P = 1, d = 0) and
    // the step needs no branch.
    auto fstep = [&](auto ctrl_tag, int o, bool take, auto rows_tag) {
      constexpr int CT_ = decltype(ctrl_tag)::value, RM = decltype(rows_tag)::value;
      double dp[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) dp[k] = dpp_d<CT_, RM>(Ds[k]);
      if constexpr (S >= 16) {
        const double pp = dpp_one<CT_, RM>(Ps);
#pragma unroll
        for (int k = 0; k < 5; ++k) Ds[k] = fma(Ps, dp[k], Ds[k]);
        Ps *= pp;
      } else {
        const double pp = dpp_d<CT_, RM>(Ps);
        if (take) {
#pragma unroll
          for (int k = 0; k < 5; ++k) Ds[k] = fma(Ps, dp[k], Ds[k]);
          Ps *= pp;
        }
      }
      (void)o;
      (void)take;
    };
    using I1 = std::integral_constant<int, kDppRowShr + 1>;
    using I2 = std::integral_constant<int, kDppRowShr + 2>;
    using I4 = std::integral_constant<int, kDppRowShr + 4>;
    using I8 = std::integral_constant<int, kDppRowShr + 8>;
    using IB = std::integral_constant<int, kDppRowBcast15>;
    using RA = std::integral_constant<int, 0xF>;
    using RB = std::integral_constant<int, 0xA>;
    fstep(I1{}, 1, seg >= 1 && (lane & 15) >= 1, RA{});
    fstep(I2{}, 2, seg >= 2 && (lane & 15) >= 2, RA{});
    if constexpr (S > 4) fstep(I4{}, 4, seg >= 4 && (lane & 15) >= 4, RA{});
    if constexpr (S > 8) fstep(I8{}, 8, seg >= 8 && (lane & 15) >= 8, RA{});
    if constexpr (S > 16) fstep(IB{}, 16, seg >= 16, RB{});
    double din[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      din[k] = dpp_d<kDppWaveShr1>(Ds[k]);
      if (seg == 0) din[k] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < RW; ++q)
      if (rows_all(q)) {
#pragma unroll
        for (int k = 0; k < 5; ++k) X[q][k] = fma(PP[q], din[k], X[q][k]);
      }
  }
  {
    // back substitution with carry 0 from the top of the segment, then the
    // carries x_in (the first unknown of the segment above) by a reverse scan
    double x[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, Q = 1.0;
#pragma unroll
    for (int q = RW - 1; q >= 0; --q) {
      if (rows_all(q)) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          x[k] = fma(gam[q], x[k], X[q][k]);
          X[q][k] = x[k];
        }
        Q *= gam[q];
        PP[q] = Q;
      }
    }
    double Qs = Q, Xs[5] = {x[0], x[1], x[2], x[3], x[4]};
    auto bstep = [&](auto ctrl_tag, bool take) {
      constexpr int CT_ = decltype(ctrl_tag)::value;
      double xn[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) xn[k] = dpp_d<CT_>(Xs[k]);
      if constexpr (S >= 16) {  // as in the forward scan: no branch
        const double qn = dpp_one<CT_>(Qs);
#pragma unroll
        for (int k = 0; k < 5; ++k) Xs[k] = fma(Qs, xn[k], Xs[k]);
        Qs *= qn;
      } else {
        const double qn = dpp_d<CT_>(Qs);
        if (take) {
#pragma unroll
          for (int k = 0; k < 5; ++k) Xs[k] = fma(Qs, xn[k], Xs[k]);
          Qs *= qn;
        }
      }
      (void)take;
    };
    using J1 = std::integral_constant<int, kDppRowShl + 1>;
    using J2 = std::integral_constant<int, kDppRowShl + 2>;
    using J4 = std::integral_constant<int, kDppRowShl + 4>;
    using J8 = std::integral_constant<int, kDppRowShl + 8>;
    bstep(J1{}, seg + 1 < S && (lane & 15) + 1 < 16);
    bstep(J2{}, seg + 2 < S && (lane & 15) + 2 < 16);
    if constexpr (S > 4) bstep(J4{}, seg + 4 < S && (lane & 15) + 4 < 16);
    if constexpr (S > 8) bstep(J8{}, seg + 8 < S && (lane & 15) + 8 < 16);
    if constexpr (S > 16) {
      // the lower row of the chain takes the upper row's composition (lane 16 of the chain)
      const int src = (lane & ~31) | 16;
      const double qn = __shfl(Qs, src, 64);
      double xn[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) xn[k] = __shfl(Xs[k], src, 64);
      if (seg < 16) {
#pragma unroll
        for (int k = 0; k < 5; ++k) Xs[k] = fma(Qs, xn[k], Xs[k]);
        Qs *= qn;
      }
    }
    double xin[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      xin[k] = dpp_d<kDppWaveShl1>(Xs[k]);
      if (seg == S - 1) xin[k] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < RW; ++q)
      if (rows_all(q)) {
#pragma unroll
        for (int k = 0; k < 5; ++k) X[q][k] = fma(PP[q], xin[k], X[q][k]);
      }
  }

  // 3. linear functionals (dot products of y'' with the plan's weight
  //    vectors) of the four particular solutions, summed over the lane's rows,
  //    then over the chain's segments by a reduce-scatter: in passes of NF
  //    functionals (all eight at once for 32 segments, two passes of four
  //    otherwise, which keeps the registers at three waves per SIMD), the V =
  //    4 NF partials are halved at each step (partners at distance S/2, ...,
  //    1 within the chain); a lane ends with entries [seg K, seg K + K), K =
  //    V / S, or, with fewer values than segments, the groups of S / V lanes
  //    add their one entry (all-reduce steps) and its first lane keeps it.
  //    Those of the homogeneous solutions (the even chain with y_0 = 1, the
  //    odd one with y'_0 = 1) depend on the mode only and come from the plan
  //    (hfun). The weight rows are staged in LDS first, over the transform
  //    buffers (free until the final series), with a row's entry n at
  //    n + n / 8 (the lanes of a chain, eight entries apart, then meet
  //    distinct banks): their loads issue together instead of one round trip
  //    to the cache per few rows.
  constexpr int NUP = N + (N >> 3) + 1;
  static_assert(kNumFunBC * NUP * sizeof(double) <= 2 * KEP * sizeof(C), "weight rows fit the buffers");
  const double* sW = reinterpret_cast<const double*>(A);
  {
    __syncthreads();  // every lane has read its transform values
    // thread n copies entry n of every row (one address, constant row offsets)
    double* dW = reinterpret_cast<double*>(A);
    for (int n = tid; n < N; n += NT) {
      double wv[kNumFunBC];
#pragma unroll
      for (int f = 0; f < kNumFunBC; ++f) wv[f] = W[f * NU + n];
#pragma unroll
      for (int f = 0; f < kNumFunBC; ++f) dW[f * NUP + n + (n >> 3)] = wv[f];
    }
    __syncthreads();
  }
  {
    constexpr int NF = S == 32 ? kNumFunBC : kNumFunBC / 2;
    constexpr int FB = NF == 8 ? 3 : 2;  // bits of a functional's index within a pass
    constexpr int V = 4 * NF;
    double* my_fun = sfun + (m * 2 + par) * kNumFunBC * 5;
    // The partner moves of the chain's lanes, partner distance S/2 first:
    // xor 16 (an LDS swizzle), then the DPP row mirror (i <-> 15 - i), half
    // mirror (i <-> 7 - i), quad xor 2 and xor 1. The first FB of them halve
    // the functionals held (a lane keeps NF/2, then NF/4, ...), the rest add
    // the four entries left over the remaining lanes. A lane stores its
    // partial of functional f at slot f ^ fl, with fl made of the lane-bit
    // functions g = b4, b3, b3^b2, b2^b1, b2^b0 (b = bits of seg) of those
    // FB halving moves: each halving move flips its own g between partners
    // and leaves the later ones unchanged, so both partners keep their first
    // half of slots and send the second, and no select is needed; the lane
    // then holds functional fl, summed over the chain.
    auto bit = [&](int b) { return (seg >> b) & 1; };
    auto gfun = [&](int kind) {
      return kind == 16 ? bit(4) : kind == 8 ? bit(3) : kind == 4 ? (bit(3) ^ bit(2))
                                                      : kind == 2 ? (bit(2) ^ bit(1)) : (bit(2) ^ bit(0));
    };
    int fl = 0;
#pragma unroll
    for (int j = 0; j < FB; ++j) fl = (fl << 1) | gfun(S >> (j + 1));
    auto mv = [&](auto kind_tag, double x) {
      constexpr int KD = decltype(kind_tag)::value;
      if constexpr (KD == 16) return __shfl_xor(x, 16, 64);
      else if constexpr (KD == 8) return dpp_d<kDppRowMirror>(x);
      else if constexpr (KD == 4) return dpp_d<kDppRowHalfMirror>(x);
      else if constexpr (KD == 2) return dpp_d<kDppQuadXor2>(x);
      else return dpp_d<kDppQuadXor1>(x);
    };
#pragma unroll
    for (int f0 = 0; f0 < kNumFunBC; f0 += NF) {
      double v[V];
#pragma unroll
      for (int i = 0; i < V; ++i) v[i] = 0.0;
#pragma unroll
      for (int q = 0; q < RW; ++q)
        if (rows_all(q)) {
          const int n = par + 2 * (r0 + q);
#pragma unroll
          for (int fp = 0; fp < NF; ++fp) {
            const double w = sW[(f0 + (fp ^ fl)) * NUP + n + (n >> 3)];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[fp * 4 + k] = fma(w, X[q][k], v[fp * 4 + k]);
          }
          // one row's weights in flight at a time (registers)
          __builtin_amdgcn_sched_barrier(0);
        }
      // move J has partner distance S >> (J + 1)
      auto move = [&](auto j_tag) {
        constexpr int J = decltype(j_tag)::value;
        using KT = std::integral_constant<int, (S >> (J + 1))>;
        if constexpr (J < FB) {
          constexpr int hh = V >> (J + 1);
#pragma unroll
          for (int i = 0; i < hh; ++i) v[i] += mv(KT{}, v[hh + i]);
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] += mv(KT{}, v[k]);
        }
      };
      move(std::integral_constant<int, 0>{});
      move(std::integral_constant<int, 1>{});
      if constexpr (LOGS > 2) move(std::integral_constant<int, 2>{});
      if constexpr (LOGS > 3) move(std::integral_constant<int, 3>{});
      if constexpr (LOGS > 4) move(std::integral_constant<int, 4>{});
      if ((seg & ((S >> FB) - 1)) == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) my_fun[(f0 + fl) * 5 + k] = v[k];
      }
    }
#pragma unroll
    for (int j = 0; j < NH; ++j)
      if (seg + j * S < kNumFunBC) my_fun[(seg + j * S) * 5 + 4] = hpre[j];
  }
  if (mi == 0) {
    // Ea, Eb of the k = 0 mode (FUN_EA, FUN_EB follow DH): a plain reduction
    double ea[5] = {0, 0, 0, 0, 0}, eb[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < RW; ++q)
      if (rows_all(q)) {
        const int n = par + 2 * (r0 + q);
        const double wa = W[FUN_EA * NU + n], wb = W[FUN_EB * NU + n];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          ea[k] = fma(wa, X[q][k], ea[k]);
          eb[k] = fma(wb, X[q][k], eb[k]);
        }
      }
    if (seg == 0) {
      ea[4] += W[FUN_EA * NU + N + par];
      eb[4] += W[FUN_EB * NU + N + par];
    }
    for (int o = S >> 1; o > 0; o >>= 1) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        ea[k] += __shfl_xor(ea[k], o, S);
        eb[k] += __shfl_xor(eb[k], o, S);
      }
    }
    if (seg == 0) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        s_e[par][0][k] = ea[k];
        s_e[par][1][k] = eb[k];
      }
    }
  }
  __syncthreads();

  // 4. per mode: free constants, wall values, mismatches, harmonic correction, k = 0
  if (tid < MB) {
    const int mm = tid;
    const double* fe = sfun + (mm * 2 + 0) * kNumFunBC * 5;
    const double* fo_ = sfun + (mm * 2 + 1) * kNumFunBC * 5;
    // functional f of vector v: 0..3 the particular solutions (Re/Im psi_i*,
    // Re/Im psi_o*), 4 the homogeneous solution of y_0 (even chain), 5 of y'_0 (odd)
    auto F = [&](int f, int v) -> double {
      if (f >= kNumFunBC) {
        const double* e0 = &s_e[0][f - kNumFunBC][0];
        const double* e1 = &s_e[1][f - kNumFunBC][0];
        return v < 4 ? e0[v] + e1[v] : (v == 4 ? e0[4] : e1[4]);
      }
      return v < 4 ? fe[f * 5 + v] + fo_[f * 5 + v] : (v == 4 ? fe[f * 5 + 4] : fo_[f * 5 + 4]);
    };
    const double kap = s_kap[mm];
    const bool dir = !(s_k[mm] > 0.0);
    // boundary rows: Robin top S1 + kap S2, bottom S3 - kap S4; Dirichlet S2, S4
    auto top = [&](int v) { return dir ? F(FUN_S2, v) : fma(kap, F(FUN_S2, v), F(FUN_S1, v)); };
    auto bot = [&](int v) { return dir ? F(FUN_S4, v) : fma(-kap, F(FUN_S4, v), F(FUN_S3, v)); };
    const double t1 = top(4), t2 = top(5), b1 = bot(4), b2 = bot(5);
    const double idet = 1.0 / (t1 * b2 - t2 * b1);
    auto solve2 = [&](double tP, double bP, double& c0, double& c1) {
      c0 = -(tP * b2 - t2 * bP) * idet;
      c1 = -(t1 * bP - tP * b1) * idet;
    };
    double ci0r, ci1r, ci0i, ci1i, co0r, co1r, co0i, co1i;
    solve2(top(0), bot(0), ci0r, ci1r);
    solve2(top(1), bot(1), ci0i, ci1i);
    solve2(top(2), bot(2), co0r, co1r);
    solve2(top(3), bot(3), co0i, co1i);
    s_c[mm][0] = make_double2(ci0r, ci0i);
    s_c[mm][1] = make_double2(ci1r, ci1i);
    auto fin_i = [&](int f) {
      return make_double2(F(f, 0) + ci0r * F(f, 4) + ci1r * F(f, 5), F(f, 1) + ci0i * F(f, 4) + ci1i * F(f, 5));
    };
    auto fin_o = [&](int f) {
      return make_double2(F(f, 2) + co0r * F(f, 4) + co1r * F(f, 5), F(f, 3) + co0i * F(f, 4) + co1i * F(f, 5));
    };
    const double2 vi0 = fin_i(FUN_V0), viH = fin_i(FUN_VH), di0 = fin_i(FUN_D0), diH = fin_i(FUN_DH);
    const double2 vo0 = fin_o(FUN_V0), voH = fin_o(FUN_VH), do0 = fin_o(FUN_D0), doH = fin_o(FUN_DH);
    const double k = s_k[mm];
    double2 al = make_double2(0, 0), be = make_double2(0, 0);
    double Ai = 0.0;
    if (k > 0.0 && s_keep[mm]) {
      const double e = g.eps, eb = g.eps_b, et = g.eps_t, tb = g.tau_b, tt = g.tau_t;
      // mismatches (eqs. mm1-mm4)
      double2 mpb = make_double2(vi0.x - tb * vo0.x, vi0.y - tb * vo0.y);
      double2 meb = make_double2(e * di0.x - eb * tb * do0.x, e * di0.y - eb * tb * do0.y);
      double2 mpt = make_double2(viH.x - tt * voH.x, viH.y - tt * voH.y);
      double2 met = make_double2(e * diH.x - et * tt * doH.x, e * diH.y - et * tt * doH.y);
      if (wall_hat) {  // wall charges: + sigma_b in mm2, - sigma_t in mm4
        const double2 sb = wall_hat[m0 + mm], st = wall_hat[nmodes + m0 + mm];
        meb.x += sb.x;
        meb.y += sb.y;
        met.x -= st.x;
        met.y -= st.y;
      }
      const double ik = 1.0 / k;
      const double2 Rb = make_double2((eb * k * mpb.x - meb.x) * ik, (eb * k * mpb.y - meb.y) * ik);
      const double2 Rt = make_double2(-(met.x + et * k * mpt.x) * ik, -(met.y + et * k * mpt.y) * ik);
      const double E = exp(-k * g.H);
      const double iD = 1.0 / ((e + eb) * (e + et) - (eb - e) * (et - e) * E * E);
      al = make_double2((Rb.x * (et - e) * E + (e + eb) * Rt.x) * iD, (Rb.y * (et - e) * E + (e + eb) * Rt.y) * iD);
      be = make_double2(((e - eb) * E * Rt.x - (e + et) * Rb.x) * iD, ((e - eb) * E * Rt.y - (e + et) * Rb.y) * iD);
    }
    if (m0 + mm == 0) {
      if (g.flags & DPSE_UNIFORM_FAST) {
        // free space (Sec. 3.1.1): A_i cancels psi_i*' at both domain ends
        Ai = -0.5 * (fin_i(FUN_EA).x + fin_i(FUN_EB).x);
      } else {
        const double e = g.eps, tb = g.tau_b, tt = g.tau_t;
        const double2 ea = fin_o(FUN_EA), ebd = fin_o(FUN_EB);
        const double Ab = -tb * ea.x, At = -tt * ebd.x;
        double A1 = (g.eps_b * (tb * do0.x + Ab) - e * di0.x) / e;
        double A2 = (g.eps_t * (tt * doH.x + At) - e * diH.x) / e;
        if (wall_hat) {  // wall charges in eqs. ai1, ai2
          A1 -= wall_hat[0].x / e;
          A2 += wall_hat[nmodes].x / e;
        }
        Ai = 0.5 * (A1 + A2);
      }
      scal[3] = Ai;
    }
    s_ab[mm][0] = al;
    s_ab[mm][1] = be;
    s_Ai[mm] = Ai;
  }
  __syncthreads();

  // 5. final series of psi_i* (y = particular + y_0 h, y'_0 h by chain
  //    parity): y_n = a_n x_{n-2} - b_n x_n + c_n x_{n+2}, plus the free
  //    constant itself at n = 0, 1; its exact derivative d_j = sum over m > j,
  //    m = j + 1 mod 2, of 2 m y_m (scaled by 1/R, d_0 halved) is a suffix sum
  //    over this lane's chain, which gives d_{n-1} at each of the lane's rows;
  //    both go to the transform buffers as even extensions (factor 2 at the
  //    ends), in bit-reversed slots
  {
    const double2 cf = s_c[m][par];
    double xr[RW], xi[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      xr[q] = fma(cf.x, X[q][4], X[q][0]);
      xi[q] = fma(cf.y, X[q][4], X[q][1]);
    }
    double lr = xr[0], li = xi[0];
#pragma unroll
    for (int q = 1; q < RW; ++q)
      if (q == cnt - 1) {
        lr = xr[q];
        li = xi[q];
      }
    double pr = dpp_d<kDppWaveShr1>(lr), pi = dpp_d<kDppWaveShr1>(li);
    double nr = dpp_d<kDppWaveShl1>(xr[0]), ni = dpp_d<kDppWaveShl1>(xi[0]);
    if (seg == 0) pr = pi = 0.0;
    if (seg == S - 1) nr = ni = 0.0;
    double yr[RW], yi[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      yr[q] = 0.0;
      yi[q] = 0.0;
      if (rows_all(q)) {
        const int n = par + 2 * (r0 + q);
        const double xmr = q == 0 ? pr : xr[q > 0 ? q - 1 : 0], xmi = q == 0 ? pi : xi[q > 0 ? q - 1 : 0];
        const double xpr = q + 1 < cnt ? xr[q + 1 < RW ? q + 1 : RW - 1] : nr;
        const double xpi = q + 1 < cnt ? xi[q + 1 < RW ? q + 1 : RW - 1] : ni;
        const double a = ctab[n], b = ctab[N + n], c = ctab[2 * N + n];
        yr[q] = fma(a, xmr, fma(-b, xr[q], c * xpr));
        yi[q] = fma(a, xmi, fma(-b, xi[q], c * xpi));
        if (n <= 1) {
          yr[q] += cf.x;
          yi[q] += cf.y;
        }
      }
    }
    // suffix sums of 2 n y_n inside the segment, then over the segments above
    double sr = 0.0, si = 0.0, sufr[RW], sufi[RW];
#pragma unroll
    for (int q = RW - 1; q >= 0; --q) {
      sufr[q] = 0.0;
      sufi[q] = 0.0;
      if (rows_all(q)) {
        const double f = 2.0 * (par + 2 * (r0 + q));
        sr = fma(f, yr[q], sr);
        si = fma(f, yi[q], si);
        sufr[q] = sr;
        sufi[q] = si;
      }
    }
    double ar = sr, ai = si;
    auto sstep = [&](auto ctrl_tag, bool take) {
      constexpr int CT_ = decltype(ctrl_tag)::value;
      const double ur = dpp_d<CT_>(ar), ui = dpp_d<CT_>(ai);
      if (S >= 16 || take) {  // 16 or 32 segments: lanes without a source add 0
        ar += ur;
        ai += ui;
      }
    };
    using K1 = std::integral_constant<int, kDppRowShl + 1>;
    using K2 = std::integral_constant<int, kDppRowShl + 2>;
    using K4 = std::integral_constant<int, kDppRowShl + 4>;
    using K8 = std::integral_constant<int, kDppRowShl + 8>;
    sstep(K1{}, seg + 1 < S && (lane & 15) + 1 < 16);
    sstep(K2{}, seg + 2 < S && (lane & 15) + 2 < 16);
    if constexpr (S > 4) sstep(K4{}, seg + 4 < S && (lane & 15) + 4 < 16);
    if constexpr (S > 8) sstep(K8{}, seg + 8 < S && (lane & 15) + 8 < 16);
    if constexpr (S > 16) {
      const int src = (lane & ~31) | 16;
      const double ur = __shfl(ar, src, 64), ui = __shfl(ai, src, 64);
      if (seg < 16) {
        ar += ur;
        ai += ui;
      }
    }
    double abr = dpp_d<kDppWaveShl1>(ar), abi = dpp_d<kDppWaveShl1>(ai);
    if (seg == S - 1) abr = abi = 0.0;
    const double ir = 1.0 / g.zR;
    auto put = [&](C* buf, int j, double vr, double vi) {
      const double f = (j == 0 || j == N - 1) ? 2.0 : 1.0;
      C c;
      c.x = (R)(f * vr);
      c.y = (R)(f * vi);
      buf[ix(bitrev(j, LOGM), m)] = c;
      if (j > 0 && j < N - 1) buf[ix(bitrev(M - j, LOGM), m)] = c;
    };
#pragma unroll
    for (int q = 0; q < RW; ++q)
      if (rows_all(q)) {
        const int n = par + 2 * (r0 + q);
        put(A, n, yr[q], yi[q]);
        if (n >= 1) {
          const double sc = n == 1 ? 0.5 * ir : ir;
          put(B, n - 1, sc * (sufr[q] + abr), sc * (sufi[q] + abi));
        }
        if (n == N - 1) put(B, N - 1, 0.0, 0.0);
      }
  }
  __syncthreads();
  fft_scan_pair<C, LOGS>(A, B, tw, tid);

  // 6. add the correction at the window nodes and the k = 0 linear mode; write out
  for (int t = tid; t < N * MB; t += NT) {
    const int j = t >> LOGMB, mm = t & (MB - 1), mo = m0 + mm;
    if (mo >= nmodes) continue;
    const C v = A[ix(j, mm)], d = B[ix(j, mm)];
    double ps_x = 0.5 * (double)v.x, ps_y = 0.5 * (double)v.y, pz_x = 0.5 * (double)d.x, pz_y = 0.5 * (double)d.y;
    const double z = zn[j];
    const double k = s_k[mm];
    if (k > 0.0 && s_keep[mm] && z >= -g.H_E && z <= g.H + g.H_E) {
      // the exponentials in the storage precision of Psi, the sums in FP64
      double e1, e2;
      if (sizeof(R) == 8) {
        e1 = exp(k * (z - g.H));
        e2 = exp(-k * z);
      } else {
        e1 = (double)expf((float)(k * (z - g.H)));
        e2 = (double)expf((float)(-k * z));
      }
      const double2 al = s_ab[mm][0], be = s_ab[mm][1];
      ps_x += al.x * e1 + be.x * e2;
      ps_y += al.y * e1 + be.y * e2;
      pz_x += k * (al.x * e1 - be.x * e2);
      pz_y += k * (al.y * e1 - be.y * e2);
    }
    if (mo == 0) {
      ps_x += s_Ai[mm] * z;
      pz_x += s_Ai[mm];
    }
    const unsigned off = (__umul24((unsigned)j, (unsigned)nmodes) + (unsigned)mo) * (unsigned)sizeof(C);  // as the loads
    C a, b;
    a.x = (R)ps_x; a.y = (R)ps_y;
    b.x = (R)pz_x; b.y = (R)pz_y;
    *reinterpret_cast<C*>(reinterpret_cast<char*>(psi) + off) = a;
    *reinterpret_cast<C*>(reinterpret_cast<char*>(psiz) + off) = b;
  }
}

}  // namespace

namespace {
size_t column_lds(const Geom& g, int KE) {
  const int M = 2 * (g.Nz - 1);
  const int MB = KE / M;
  return (size_t)(2 * KE + M / 2) * sizeof(double2) + (size_t)(kCtabRows * g.Nz + MB * 60) * sizeof(double);
}

// Whether a plan's chains use k_column_scan (and its factor table layout).
bool scan_applies(const Geom& g) { return !(g.flags & DPSE_TRIPLY) && g.Nz >= 33 && g.Nz <= 257; }

// Dynamic LDS of k_column_scan: two padded transform buffers, the twiddles
// and the reduced functionals.
size_t column_scan_lds(const Geom& g, size_t creal) {
  const int M = 2 * (g.Nz - 1), MB = kScanKE / M;
  int logS = -4;
  while ((1 << (logS + 4)) < M) ++logS;
  const size_t kep = (size_t)kScanKE + (M >> (logS - 2));
  return (2 * kep + M / 2) * 2 * creal + (size_t)MB * 2 * kNumFunBC * 5 * sizeof(double);
}

template <typename R, int LOGS>
void column_scan_as(dpse_plan* p) {
  using C = typename CT<R>::T;
  const Geom& g = p->g;
  constexpr int MB = 128 >> LOGS;
  const int nmodes = g.Ny * g.nkx;
  const int nb = (nmodes + MB - 1) / MB;
  hipLaunchKernelGGL((k_column_scan<R, LOGS>), dim3(nb), dim3(kScanNT), column_scan_lds(g, sizeof(R)), p->stream,
                     g, (const C*)p->w.fx_i, (const C*)p->w.fx_o, (C*)p->w.psi, (C*)p->w.psiz, (const double*)p->t.z,
                     (const double*)p->t.ctab, (const double2*)p->t.twz, (const double*)p->t.cpiv,
                     (const double*)p->t.hfun, p->w.scal, p->walls_on ? (const double2*)p->walls.hat : nullptr);
}

template <typename R>
void column_scan_dispatch(dpse_plan* p) {
  switch (p->g.Nz) {
    case 33: column_scan_as<R, 2>(p); break;
    case 65: column_scan_as<R, 3>(p); break;
    case 129: column_scan_as<R, 4>(p); break;
    default: column_scan_as<R, 5>(p); break;
  }
}

template <typename R, int KE, int NT>
void column_as(dpse_plan* p) {
  using C = typename CT<R>::T;
  const Geom& g = p->g;
  const int M = 2 * (g.Nz - 1);
  const int MB = KE / M;
  const int nmodes = g.Ny * g.nkx;
  const int nb = (nmodes + MB - 1) / MB;
  hipLaunchKernelGGL((k_column<R, KE, NT>), dim3(nb), dim3(NT), column_lds(g, KE), p->stream, g,
                     (const C*)p->w.fx_i, (const C*)p->w.fx_o, (C*)p->w.psi, (C*)p->w.psiz, (const double*)p->t.z,
                     (const double*)p->t.ctab, (const double2*)p->t.twz, (const double*)p->t.cpiv, p->w.scal,
                     p->walls_on ? (const double2*)p->walls.hat : nullptr);
}

// Triply periodic variant: per block of MB = KE / Nz modes (k_x, k_y), the
// periodic z transform of each column, psi^ = F^ / (eps |k|^2) (0 at k = 0),
// psi_z^ = -i k_z psi^ (0 at the Nyquist k_z), and the inverse transforms, in
// FP64 in both precisions. The nodes descend, z_c = (Nz - 1 - c) h_z, so in
// node-index space the z derivative multiplies index frequency m by -i k_z,
// k_z = 2 pi m / H (m signed); the 1/Nz of the z transform is folded in here.
constexpr int kTpKE = 1024;  // complex LDS elements per buffer (two buffers: 32 KB)

template <typename R>
__global__ void __launch_bounds__(kThreads) k_tp_column(Geom g, const typename CT<R>::T* __restrict__ fx,
                                                        typename CT<R>::T* __restrict__ psi,
                                                        typename CT<R>::T* __restrict__ psiz,
                                                        const double2* __restrict__ twz) {
  using C = typename CT<R>::T;
  extern __shared__ double2 smem2[];
  double2* A = smem2;
  double2* B = smem2 + kTpKE;
  double2* tw = smem2 + 2 * kTpKE;
  const int N = g.Nz, logN = ilog2d(N), MB = kTpKE / N, logMB = ilog2d(kTpKE) - logN;
  const int nmodes = g.Ny * g.nkx;
  const int m0 = xcd_block(blockIdx.x, gridDim.x) * MB;
  const int tid = threadIdx.x;
  constexpr int kPer = kTpKE / kThreads;
  for (int i = tid; i < N / 2; i += kThreads) tw[i] = twz[i];
  {
    C v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = tid + q * kThreads, j = t >> logMB, m = t & (MB - 1), mi = m0 + m;
      v[q].x = 0;
      v[q].y = 0;
      if (mi < nmodes) v[q] = fx[(size_t)j * nmodes + mi];
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = tid + q * kThreads, j = t >> logMB, m = t & (MB - 1);
      A[bitrev(j, logN) * MB + m] = make_double2((double)v[q].x, (double)v[q].y);
    }
  }
  __syncthreads();
  fft_lds_r22<double2, true, kTpKE / 4 / kThreads, kThreads>(A, logN, logMB, 1, MB, tw, false, tid);
  {
    double2 a[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) a[q] = A[tid + q * kThreads];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = tid + q * kThreads, f = t >> logMB, m = t & (MB - 1), mi = m0 + m;
      const int kyi = mi / g.nkx, kxi = mi - kyi * g.nkx;
      const int nx = kxi == g.Nx / 2 ? -(g.Nx / 2) : kxi;
      const int ny = kyi < g.Ny / 2 ? kyi : kyi - g.Ny;
      const int mz = f < N / 2 ? f : f - N;
      const double kx = 2.0 * kPi * nx / g.Lx, ky = 2.0 * kPi * ny / g.Ly, kz = 2.0 * kPi * mz / g.H;
      const double k2 = kx * kx + ky * ky + kz * kz;
      const double G = (k2 > 0.0 && mi < nmodes) ? 1.0 / (g.eps * k2 * N) : 0.0;
      const double2 ps = make_double2(a[q].x * G, a[q].y * G);
      const double d = f == N / 2 ? 0.0 : -kz;  // psi_z^ = i d psi^
      const int pos = bitrev(f, logN) * MB + m;
      A[pos] = ps;
      B[pos] = make_double2(-d * ps.y, d * ps.x);
    }
  }
  __syncthreads();
  fft_lds_r22<double2, true, kTpKE / 4 / kThreads, kThreads>(A, logN, logMB, 1, MB, tw, true, tid);
  fft_lds_r22<double2, true, kTpKE / 4 / kThreads, kThreads>(B, logN, logMB, 1, MB, tw, true, tid);
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int t = tid + q * kThreads, j = t >> logMB, m = t & (MB - 1), mi = m0 + m;
    if (mi >= nmodes) continue;
    const double2 a = A[j * MB + m], b = B[j * MB + m];
    C u, w;
    u.x = (R)a.x;
    u.y = (R)a.y;
    w.x = (R)b.x;
    w.y = (R)b.y;
    psi[(size_t)j * nmodes + mi] = u;
    psiz[(size_t)j * nmodes + mi] = w;
  }
}

// Harmonic correction of the walls alone for a mode with k > 0: the closed
// form of the column kernel with m_phi = 0, m_E^b = sigma_b, m_E^t = -sigma_t,
// so R_b = -sigma_b / k and R_t = sigma_t / k.
__device__ inline void wall_coeffs(const Geom& g, double k, double2 sb, double2 st, double2& al, double2& be) {
  const double e = g.eps, eb = g.eps_b, et = g.eps_t;
  const double E = exp(-k * g.H);
  const double D = (e + eb) * (e + et) - (eb - e) * (et - e) * E * E;
  const double2 Rb = make_double2(-sb.x / k, -sb.y / k), Rt = make_double2(st.x / k, st.y / k);
  al = make_double2((Rb.x * (et - e) * E + (e + eb) * Rt.x) / D, (Rb.y * (et - e) * E + (e + eb) * Rt.y) / D);
  be = make_double2(((e - eb) * E * Rt.x - (e + et) * Rb.x) / D, ((e - eb) * E * Rt.y - (e + et) * Rb.y) / D);
}

// k = 0 slope of the walls alone: the mean of eqs. ai1 and ai2 without charges.
__device__ inline double wall_slope(const Geom& g, const double2* hat, int nmodes) {
  return 0.5 * (hat[nmodes].x - hat[0].x) / g.eps;
}

// Potential of the walls alone per mode at every node into psi (the correction
// at the window nodes -H_E <= z <= H + H_E of corrected modes, A_s z at
// k = 0, zero elsewhere); psiz is cleared.
template <typename R>
__global__ void __launch_bounds__(kThreads) k_wall_modes(Geom g, const double2* __restrict__ hat,
                                                         const double* __restrict__ zn,
                                                         typename CT<R>::T* __restrict__ psi,
                                                         typename CT<R>::T* __restrict__ psiz) {
  using C = typename CT<R>::T;
  const int nmodes = g.Ny * g.nkx;
  const int64_t total = (int64_t)g.Nz * nmodes;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < total; i += (int64_t)gridDim.x * kThreads) {
    const int c = (int)(i / nmodes), mi = (int)(i - (int64_t)c * nmodes);
    const double z = zn[c];
    double kk;
    int keep;
    mode_wave(g, mi, kk, keep);
    double2 v = make_double2(0.0, 0.0);
    if (mi == 0) {
      v.x = wall_slope(g, hat, nmodes) * z;
    } else if (kk > 0.0 && keep && z >= -g.H_E && z <= g.H + g.H_E) {
      double2 al, be;
      wall_coeffs(g, kk, hat[mi], hat[nmodes + mi], al, be);
      const double e1 = exp(kk * (z - g.H)), e2 = exp(-kk * z);
      v = make_double2(al.x * e1 + be.x * e2, al.y * e1 + be.y * e2);
    }
    C a, zero;
    a.x = (R)v.x;
    a.y = (R)v.y;
    zero.x = (R)0;
    zero.y = (R)0;
    psi[i] = a;
    psiz[i] = zero;
  }
}

// Wall scalars, one block: ws[0] = int sigma = Lx Ly (sigma_b^(0) + sigma_t^(0)),
// ws[1] = int |sigma| (trapezoid sum of the staged densities), ws[2] =
// int (sigma_b phi_s(.,0) + sigma_t phi_s(.,H)) = Lx Ly sum_k Re(conj(sigma^) phi_s^)
// over the full spectrum (the half spectrum with columns 0 < kx < Nx/2 twice),
// ws[3] = the k = 0 slope A_s. Fixed summation order.
__global__ void __launch_bounds__(kThreads) k_wall_scalars(Geom g, const double2* __restrict__ hat,
                                                           const double* __restrict__ stage, double* ws) {
  __shared__ double sa[kThreads], sb_[kThreads];
  const int nmodes = g.Ny * g.nkx;
  const double As = wall_slope(g, hat, nmodes);
  double acc = 0.0, aab = 0.0;
  for (int mi = threadIdx.x; mi < nmodes; mi += kThreads) {
    double kk;
    int keep;
    mode_wave(g, mi, kk, keep);
    const int kxi = mi % g.nkx;
    const double cw = (kxi == 0 || kxi == g.Nx / 2) ? 1.0 : 2.0;
    const double2 sb = hat[mi], st = hat[nmodes + mi];
    double2 p0 = make_double2(0.0, 0.0), pH = make_double2(0.0, 0.0);
    if (mi == 0) {
      pH.x = As * g.H;
    } else if (kk > 0.0 && keep) {
      double2 al, be;
      wall_coeffs(g, kk, sb, st, al, be);
      const double E = exp(-kk * g.H);
      p0 = make_double2(al.x * E + be.x, al.y * E + be.y);
      pH = make_double2(al.x + be.x * E, al.y + be.y * E);
    }
    acc += cw * (sb.x * p0.x + sb.y * p0.y + st.x * pH.x + st.y * pH.y);
  }
  const int64_t ns = 2LL * g.Ny * g.Nx;
  for (int64_t i = threadIdx.x; i < ns; i += kThreads) aab += fabs(stage[i]);
  sa[threadIdx.x] = acc;
  sb_[threadIdx.x] = aab;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sa[threadIdx.x] += sa[threadIdx.x + s];
      sb_[threadIdx.x] += sb_[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double area = g.Lx * g.Ly;
    ws[0] = area * (hat[0].x + hat[nmodes].x);
    ws[1] = g.h * g.h * sb_[0];
    ws[2] = area * sa[0];
    ws[3] = As;
  }
}
}  // namespace

bool g_column_ok[kNumColumn] = {};  // set by prepare_kernels

int column_candidates() { return kNumColumn; }

hipError_t launch_pivots(dpse_plan* p, hipStream_t s) {
  const Geom& g = p->g;
  const int nt = 2 * g.Ny * g.nkx;
  if (scan_applies(g))
    hipLaunchKernelGGL(k_pivots_scan, dim3((nt + kThreads - 1) / kThreads), dim3(kThreads), 0, s, g,
                       (const double*)p->t.ctab, p->t.cpiv, p->t.hfun);
  else
    hipLaunchKernelGGL(k_pivots, dim3((nt + kThreads - 1) / kThreads), dim3(kThreads), 0, s, g,
                       (const double*)p->t.ctab, p->t.cpiv);
  return hipGetLastError();
}

int column_block(int i) { return kColumnKE[i]; }
int column_threads(int i) { return kColumnNT[i]; }

// A block of KE / M modes needs M <= KE, at most kMaxMB modes and its LDS.
bool column_valid(const Geom& g, int i) {
  if (i < 0 || i >= kNumColumn) return false;
  // the plan's factor table has the layout of one kernel family
  if (i == kScanCand) return g_column_ok[i] && scan_applies(g);
  if (scan_applies(g)) return false;
  const int KE = kColumnKE[i], M = 2 * (g.Nz - 1);
  return g_column_ok[i] && M <= KE && KE / M <= kMaxMB && 16 * (KE / M) <= kColumnNT[i] &&
         column_lds(g, KE) <= kMaxLds;
}

template <typename R>
hipError_t launch_column(dpse_plan* p) {
  if (p->g.flags & DPSE_TRIPLY) {
    using C = typename CT<R>::T;
    const Geom& g = p->g;
    const int MB = kTpKE / g.Nz;
    const int nb = (g.Ny * g.nkx + MB - 1) / MB;
    const size_t lds = (size_t)(2 * kTpKE + g.Nz / 2) * sizeof(double2);
    hipLaunchKernelGGL(k_tp_column<R>, dim3(nb), dim3(kThreads), lds, p->stream, g, (const C*)p->w.fx_i,
                       (C*)p->w.psi, (C*)p->w.psiz, (const double2*)p->t.twz);
    return hipGetLastError();
  }
  int c = p->column_cfg;
  if (!column_valid(p->g, c)) {
    const int order[] = {kScanCand, 0, 1, 2, 3, 4};
    c = 2;
    for (int i : order)
      if (column_valid(p->g, i)) {
        c = i;
        break;
      }
  }
  switch (c) {
    case kScanCand: column_scan_dispatch<R>(p); break;
    case 0: column_as<R, 2048, 256>(p); break;
    case 1: column_as<R, 1024, 256>(p); break;
    case 2: column_as<R, 4096, 256>(p); break;
    case 3: column_as<R, 2048, 512>(p); break;
    default: column_as<R, 4096, 512>(p); break;
  }
  return hipGetLastError();
}

// Raises the dynamic LDS limit of the column kernels on the current device;
// called at plan creation so that no attribute call happens inside a solve
// (which may be captured into a graph).
// A candidate whose limit cannot be raised is left out of column_valid().
hipError_t prepare_kernels() {
  const void* fns[kNumColumn][8] = {
      {(const void*)k_column<double, 2048, 256>, (const void*)k_column<float, 2048, 256>},
      {(const void*)k_column<double, 1024, 256>, (const void*)k_column<float, 1024, 256>},
      {(const void*)k_column<double, 4096, 256>, (const void*)k_column<float, 4096, 256>},
      {(const void*)k_column<double, 2048, 512>, (const void*)k_column<float, 2048, 512>},
      {(const void*)k_column<double, 4096, 512>, (const void*)k_column<float, 4096, 512>},
      {(const void*)k_column_scan<double, 2>, (const void*)k_column_scan<float, 2>,
       (const void*)k_column_scan<double, 3>, (const void*)k_column_scan<float, 3>,
       (const void*)k_column_scan<double, 4>, (const void*)k_column_scan<float, 4>,
       (const void*)k_column_scan<double, 5>, (const void*)k_column_scan<float, 5>}};
  bool any = false;
  for (int i = 0; i < kNumColumn; ++i) {
    bool ok = true;
    for (const void* f : fns[i])
      if (f) ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds) == hipSuccess;
    g_column_ok[i] = ok;
    any = any || ok;
  }
  (void)hipGetLastError();  // clear a failed attribute call
  return any ? hipSuccess : hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_wall_modes(dpse_plan* p) {
  using C = typename CT<R>::T;
  const Geom& g = p->g;
  const int64_t total = (int64_t)g.Nz * g.Ny * g.nkx;
  const int nb = (int)std::min<int64_t>((total + kThreads - 1) / kThreads, 8192);
  hipLaunchKernelGGL(k_wall_modes<R>, dim3(nb), dim3(kThreads), 0, p->stream, g, (const double2*)p->walls.hat,
                     (const double*)p->t.z, (C*)p->w.psi, (C*)p->w.psiz);
  hipLaunchKernelGGL(k_wall_scalars, dim3(1), dim3(kThreads), 0, p->stream, g, (const double2*)p->walls.hat,
                     (const double*)p->walls.stage, p->walls.scal);
  return hipGetLastError();
}

template hipError_t launch_column<double>(dpse_plan*);
template hipError_t launch_column<float>(dpse_plan*);
template hipError_t launch_wall_modes<double>(dpse_plan*);
template hipError_t launch_wall_modes<float>(dpse_plan*);

}  // namespace dpse
