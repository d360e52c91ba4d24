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

#include "dpse_internal.h"
#include "fft_lds.h"

namespace dpse {

namespace {

constexpr int kThreads = 256;
constexpr int kElems = 2048;  // complex elements per buffer (modes x 2(Nz-1))
constexpr int kMaxMB = 32;    // modes per block for the smallest Nz

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

// Coefficients of y_n = a_n y''_{n-2} - b_n y''_n + c_n y''_{n+2} (n >= 2) and
// y_1 = y'_0 - b_1 y''_1 + c_1 y''_3, from eqs. ds and cs with y''_n = 0 for
// n > N-1 and y'_N = 0.
__device__ inline void chain_coeffs(int n, int N, double& a, double& b, double& c) {
  double dn = (double)n;
  if (n == 0) { a = 0.0; b = 0.0; c = 0.0; return; }
  if (n == 1) { a = 0.0; b = 0.125; c = 0.125; return; }
  if (n == 2) { a = 0.25; b = 1.0 / 6.0; c = 1.0 / 24.0; }
  else {
    a = 1.0 / (4.0 * dn * (dn - 1.0));
    b = 1.0 / (2.0 * (dn * dn - 1.0));
    c = 1.0 / (4.0 * dn * (dn + 1.0));
  }
  if (n >= N - 2) c = 0.0;
  if (n == N - 1) b = 1.0 / (4.0 * dn * (dn - 1.0));
}

template <typename R>
__global__ void __launch_bounds__(kThreads) k_column(Geom g, const typename CT<R>::T* __restrict__ fx_i,
                                                     const typename CT<R>::T* __restrict__ fx_o,
                                                     typename CT<R>::T* __restrict__ psi,
                                                     typename CT<R>::T* __restrict__ psiz,
                                                     const double* __restrict__ zn, const double* __restrict__ T0,
                                                     const double* __restrict__ TH, const double* __restrict__ dT0,
                                                     const double* __restrict__ dTH,
                                                     const double2* __restrict__ twz, double* scal) {
  using C = typename CT<R>::T;
  __shared__ double2 A[kElems];  // psi_o* work, later derivative coefficients
  __shared__ double2 B[kElems];  // psi_i* work
  __shared__ double s_k[kMaxMB], s_kap[kMaxMB];
  __shared__ int s_keep[kMaxMB];
  __shared__ double2 s_val[2][kMaxMB][4];  // [i/o][mode][v0, vH, d0, dH]
  __shared__ double s_end[kMaxMB][2];      // d psi_o*/dz at z = a, b (k = 0)
  __shared__ double2 s_ab[kMaxMB][2];      // alpha, beta
  __shared__ double s_Ai[kMaxMB];

  const int N = g.Nz, M = 2 * (N - 1), logM = ilog2d(M);
  const int MB = kElems / M;
  const int nmodes = g.Ny * g.nkx;
  const int m0 = blockIdx.x * MB;
  const int tid = threadIdx.x;
  const double Rz = g.zR;

  if (tid < MB) {
    int mi = m0 + tid;
    double kk = 0.0;
    int keep = 0;
    if (mi < nmodes) {
      int kyi = mi / g.nkx, kxi = mi % g.nkx;
      int nx = kxi == g.Nx / 2 ? -(g.Nx / 2) : kxi;
      int ny = kyi < g.Ny / 2 ? kyi : kyi - g.Ny;
      double kx = 2.0 * kPi * nx / g.Lx, ky = 2.0 * kPi * ny / g.Ly;
      kk = sqrt(kx * kx + ky * ky);
      long long lhs = 4LL * ((long long)nx * nx * g.Ny * g.Ny + (long long)ny * ny * g.Nx * g.Nx);
      long long rhs = (long long)g.Nx * g.Ny * (long long)g.Nx * g.Ny;
      keep = (lhs <= rhs) ? 1 : 0;
      if ((g.flags & DPSE_KMAX_GT) && !(kk <= 4.2 / g.g_t)) keep = 0;
    }
    s_k[tid] = kk;
    s_kap[tid] = kk * Rz;
    s_keep[tid] = keep;
  }

  // 1. even extension of the node values in bit-reversed order, then FFT
  for (int t = tid; t < M * MB; t += kThreads) {
    int j = t / MB, m = t % MB, mi = m0 + m;
    int c = j < N ? j : M - j;
    double2 vo = make_double2(0.0, 0.0), vi = make_double2(0.0, 0.0);
    if (mi < nmodes) {
      size_t o = (size_t)c * nmodes + mi;
      C a = fx_i[o];
      vi = make_double2((double)a.x, (double)a.y);
      if (c < g.top_end || c >= g.bot_begin) {
        C b = fx_o[o];
        vo = make_double2((double)b.x, (double)b.y);
      }
    }
    int pos = bitrev(j, logM) * MB + m;
    A[pos] = vo;
    B[pos] = vi;
  }
  __syncthreads();
  fft_lds<double2, true>(A, logM, MB, 1, MB, twz, false, tid, kThreads);
  fft_lds<double2, true>(B, logM, MB, 1, MB, twz, false, tid, kThreads);

  // 2. tridiagonal chains; thread = (mode, parity)
  double* spA = reinterpret_cast<double*>(A + N * MB);  // spare: chain pivots cp
  double* spB = reinterpret_cast<double*>(B + N * MB);  // spare: homogeneous solutions
  // spare slot of (mode m, index idx): idx-th double after position N of mode m
  auto spare = [&](double* base, int m, int idx) -> double& {
    return base[(idx >> 1) * 2 * MB + 2 * m + (idx & 1)];
  };
  const int half0 = (N + 1) / 2;  // rows of the even chain
  if (tid < 2 * MB) {
    const int m = tid % MB, par = tid / MB;
    const double kap2 = s_kap[m] * s_kap[m];
    const double gs = -Rz * Rz / (g.eps * (double)(N - 1));
    double cp = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0, dh = 0.0;
    int r = 0;
    for (int n = par; n < N; n += 2, ++r) {
      double a, b, c;
      chain_coeffs(n, N, a, b, c);
      double sub = -kap2 * a, dia = 1.0 + kap2 * b, sup = -kap2 * c;
      double den = r == 0 ? dia : dia - sub * cp;
      double inv = 1.0 / den;
      double scale = gs * ((n == 0 || n == N - 1) ? 0.5 : 1.0);
      double2 gi = B[n * MB + m], go = A[n * MB + m];
      double rh0 = scale * gi.x, rh1 = scale * gi.y, rh2 = scale * go.x, rh3 = scale * go.y;
      double rhh = r == 0 ? kap2 : 0.0;
      if (r == 0) {
        d0 = rh0 * inv; d1 = rh1 * inv; d2 = rh2 * inv; d3 = rh3 * inv; dh = rhh * inv;
      } else {
        d0 = (rh0 - sub * d0) * inv; d1 = (rh1 - sub * d1) * inv;
        d2 = (rh2 - sub * d2) * inv; d3 = (rh3 - sub * d3) * inv;
        dh = (rhh - sub * dh) * inv;
      }
      cp = sup * inv;
      spare(spA, m, par * half0 + r) = cp;
      B[n * MB + m] = make_double2(d0, d1);
      A[n * MB + m] = make_double2(d2, d3);
      spare(spB, m, par * half0 + r) = dh;
    }
    // back substitution
    int rl = r - 1;
    int nl = par + 2 * rl;
    double2 xi = B[nl * MB + m], xo = A[nl * MB + m];
    double xh = spare(spB, m, par * half0 + rl);
    for (int rr = rl - 1; rr >= 0; --rr) {
      int n = par + 2 * rr;
      double c = spare(spA, m, par * half0 + rr);
      double2 di = B[n * MB + m], dd = A[n * MB + m];
      double dhh = spare(spB, m, par * half0 + rr);
      xi = make_double2(di.x - c * xi.x, di.y - c * xi.y);
      xo = make_double2(dd.x - c * xo.x, dd.y - c * xo.y);
      xh = dhh - c * xh;
      B[n * MB + m] = xi;
      A[n * MB + m] = xo;
      spare(spB, m, par * half0 + rr) = xh;
    }
  }
  __syncthreads();

  // 3. boundary conditions, 2x2 Schur step, final coefficients; thread = (mode, i/o)
  if (tid < 2 * MB) {
    const int m = tid % MB, which = tid / MB;  // 0: psi_i* in B, 1: psi_o* in A
    double2* X = which == 0 ? B : A;
    const double kap = s_kap[m];
    const bool dir = !(s_k[m] > 0.0);
    auto ypp = [&](int n) -> double2 { return n < N ? X[n * MB + m] : make_double2(0.0, 0.0); };
    auto hpp = [&](int n) -> double {  // homogeneous y'' (h1 on even n, h2 on odd n)
      return n < N ? spare(spB, m, (n & 1) * half0 + (n >> 1)) : 0.0;
    };
    // derivative coefficient y'_n of the particular solution and of h1, h2
    auto yp = [&](int n, double2& P, double& h1, double& h2) {
      if (n == 0) { P = make_double2(0.0, 0.0); h1 = 0.0; h2 = 1.0; return; }
      if (n >= N) { P = make_double2(0.0, 0.0); h1 = 0.0; h2 = 0.0; return; }
      double2 lo = ypp(n - 1), hi = ypp(n + 1);
      double hl = hpp(n - 1), hh = hpp(n + 1);
      if (n == 1) {
        P = make_double2(lo.x - 0.5 * hi.x, lo.y - 0.5 * hi.y);
        double v = hl - 0.5 * hh;
        h1 = (n - 1) % 2 == 0 ? v : 0.0;  // y''_0, y''_2 belong to the even chain (h1)
        h2 = (n - 1) % 2 == 0 ? 0.0 : v;
        return;
      }
      double f = 1.0 / (2.0 * n);
      P = make_double2(f * (lo.x - hi.x), f * (lo.y - hi.y));
      double v = f * (hl - hh);
      // y''_{n-1}, y''_{n+1} have the parity of n-1
      h1 = ((n - 1) & 1) == 0 ? v : 0.0;
      h2 = ((n - 1) & 1) == 0 ? 0.0 : v;
    };
    // pass 1: boundary functionals
    double2 tP = make_double2(0.0, 0.0), bP = make_double2(0.0, 0.0);
    double t1 = 0.0, t2 = 0.0, b1 = 0.0, b2 = 0.0;
    double2 pm, pc, pp;
    double hm1, hm2, hc1, hc2, hp1, hp2;
    // sliding window: pm = y'_{n-1}, pc = y'_n, pp = y'_{n+1}
    pm = make_double2(0.0, 0.0); hm1 = 0.0; hm2 = 0.0;
    yp(0, pc, hc1, hc2);
    for (int n = 0; n < N; ++n) {
      yp(n + 1, pp, hp1, hp2);
      double2 Py;
      double y1, y2;
      if (n == 0) { Py = make_double2(0.0, 0.0); y1 = 1.0; y2 = 0.0; }
      else if (n == 1) {  // y_1 = y'_0 - y'_2 / 2
        Py = make_double2(pm.x - 0.5 * pp.x, pm.y - 0.5 * pp.y);
        y1 = hm1 - 0.5 * hp1; y2 = hm2 - 0.5 * hp2;
      } else {
        double f = 1.0 / (2.0 * n);
        double2 q = n + 1 < N ? pp : make_double2(0.0, 0.0);
        double q1 = n + 1 < N ? hp1 : 0.0, q2 = n + 1 < N ? hp2 : 0.0;
        Py = make_double2(f * (pm.x - q.x), f * (pm.y - q.y));
        y1 = f * (hm1 - q1); y2 = f * (hm2 - q2);
      }
      double sg = (n & 1) ? -1.0 : 1.0;
      if (dir) {
        tP.x += Py.x; tP.y += Py.y; t1 += y1; t2 += y2;
        bP.x += sg * Py.x; bP.y += sg * Py.y; b1 += sg * y1; b2 += sg * y2;
      } else {
        tP.x += pc.x + kap * Py.x; tP.y += pc.y + kap * Py.y;
        t1 += hc1 + kap * y1; t2 += hc2 + kap * y2;
        bP.x += sg * (pc.x - kap * Py.x); bP.y += sg * (pc.y - kap * Py.y);
        b1 += sg * (hc1 - kap * y1); b2 += sg * (hc2 - kap * y2);
      }
      pm = pc; hm1 = hc1; hm2 = hc2;
      pc = pp; hc1 = hp1; hc2 = hp2;
    }
    // [t1 t2; b1 b2] [y0; y0'] = -[tP; bP]
    double det = t1 * b2 - t2 * b1;
    double2 c0 = make_double2(-(tP.x * b2 - t2 * bP.x) / det, -(tP.y * b2 - t2 * bP.y) / det);
    double2 c1 = make_double2(-(t1 * bP.x - tP.x * b1) / det, -(t1 * bP.y - tP.y * b1) / det);
    // pass 2: final coefficients y_n = P_n + c0 h1_n + c1 h2_n, written in place
    pm = make_double2(0.0, 0.0); hm1 = 0.0; hm2 = 0.0;
    yp(0, pc, hc1, hc2);
    for (int n = 0; n < N; ++n) {
      yp(n + 1, pp, hp1, hp2);
      double2 Py;
      double y1, y2;
      if (n == 0) { Py = make_double2(0.0, 0.0); y1 = 1.0; y2 = 0.0; }
      else if (n == 1) {
        Py = make_double2(pm.x - 0.5 * pp.x, pm.y - 0.5 * pp.y);
        y1 = hm1 - 0.5 * hp1; y2 = hm2 - 0.5 * hp2;
      } else {
        double f = 1.0 / (2.0 * n);
        double2 q = n + 1 < N ? pp : make_double2(0.0, 0.0);
        double q1 = n + 1 < N ? hp1 : 0.0, q2 = n + 1 < N ? hp2 : 0.0;
        Py = make_double2(f * (pm.x - q.x), f * (pm.y - q.y));
        y1 = f * (hm1 - q1); y2 = f * (hm2 - q2);
      }
      pm = pc; hm1 = hc1; hm2 = hc2;
      pc = pp; hc1 = hp1; hc2 = hp2;
      // position n is no longer read: y''_n was consumed by y'_{n-1} and y'_{n+1}
      X[n * MB + m] = make_double2(Py.x + c0.x * y1 + c1.x * y2, Py.y + c0.y * y1 + c1.y * y2);
    }
  }
  __syncthreads();

  // 4. values and derivatives at the walls (and slopes at the domain ends)
  if (tid < 2 * MB) {
    const int m = tid % MB, which = tid / MB;
    const double2* X = which == 0 ? B : A;
    double2 v0 = make_double2(0, 0), vH = v0, d0 = v0, dH = v0;
    double ea = 0.0, eb = 0.0;
    for (int n = 0; n < N; ++n) {
      double2 y = X[n * MB + m];
      double t0 = T0[n], tH = TH[n], e0 = dT0[n], eH = dTH[n];
      v0.x += y.x * t0; v0.y += y.y * t0;
      vH.x += y.x * tH; vH.y += y.y * tH;
      d0.x += y.x * e0; d0.y += y.y * e0;
      dH.x += y.x * eH; dH.y += y.y * eH;
      double n2 = (double)n * n;
      eb += y.x * n2;
      ea += ((n & 1) ? 1.0 : -1.0) * y.x * n2;  // T_n'(-1) = (-1)^(n+1) n^2
    }
    s_val[which][m][0] = v0;
    s_val[which][m][1] = vH;
    s_val[which][m][2] = d0;
    s_val[which][m][3] = dH;
    if (which == 1) {
      s_end[m][0] = ea / Rz;
      s_end[m][1] = eb / Rz;
    }
  }
  __syncthreads();

  // 5. mismatches, harmonic correction, k = 0 linear mode; derivative coefficients
  if (tid < MB) {
    const int m = tid;
    const double k = s_k[m];
    double2 al = make_double2(0, 0), be = make_double2(0, 0);
    double Ai = 0.0;
    const double2* vi = s_val[0][m];
    const double2* vo = s_val[1][m];
    if (k > 0.0 && s_keep[m]) {
      const double e = g.eps, eb = g.eps_b, et = g.eps_t, tb = g.tau_b, tt = g.tau_t;
      double2 mpb = make_double2(vi[0].x - tb * vo[0].x, vi[0].y - tb * vo[0].y);
      double2 meb = make_double2(e * vi[2].x - eb * tb * vo[2].x, e * vi[2].y - eb * tb * vo[2].y);
      double2 mpt = make_double2(vi[1].x - tt * vo[1].x, vi[1].y - tt * vo[1].y);
      double2 met = make_double2(e * vi[3].x - et * tt * vo[3].x, e * vi[3].y - et * tt * vo[3].y);
      double2 Rb = make_double2((eb * k * mpb.x - meb.x) / k, (eb * k * mpb.y - meb.y) / k);
      double2 Rt = make_double2(-(met.x + et * k * mpt.x) / k, -(met.y + et * k * mpt.y) / k);
      double E = exp(-k * g.H);
      double D = (e + eb) * (e + et) - (eb - e) * (et - e) * E * E;
      al = make_double2((Rb.x * (et - e) * E + (e + eb) * Rt.x) / D, (Rb.y * (et - e) * E + (e + eb) * Rt.y) / D);
      be = make_double2(((e - eb) * E * Rt.x - (e + et) * Rb.x) / D, ((e - eb) * E * Rt.y - (e + et) * Rb.y) / D);
    }
    if (m0 + m == 0) {
      const double e = g.eps, tb = g.tau_b, tt = g.tau_t;
      double Ab = -tb * s_end[m][0], At = -tt * s_end[m][1];
      double A1 = (g.eps_b * (tb * vo[2].x + Ab) - e * vi[2].x) / e;
      double A2 = (g.eps_t * (tt * vo[3].x + At) - e * vi[3].x) / e;
      Ai = 0.5 * (A1 + A2);
      scal[3] = Ai;
    }
    s_ab[m][0] = al;
    s_ab[m][1] = be;
    s_Ai[m] = Ai;
    // derivative series of psi_i*: d_{n-1} = d_{n+1} + 2 n y_n, d_0 halved, times 1/R
    double2 dn1 = make_double2(0, 0), dn2 = make_double2(0, 0);  // d_{n}, d_{n+1}
    A[(N - 1) * MB + m] = make_double2(0.0, 0.0);
    for (int n = N - 1; n >= 1; --n) {
      double2 y = B[n * MB + m];
      double2 d = make_double2(dn2.x + 2.0 * n * y.x, dn2.y + 2.0 * n * y.y);  // d_{n-1}
      dn2 = dn1;
      dn1 = d;
      double f = (n - 1 == 0) ? 0.5 / Rz : 1.0 / Rz;
      A[(n - 1) * MB + m] = make_double2(f * d.x, f * d.y);
    }
  }
  __syncthreads();

  // 6. inverse DCT-I of B (series) and A (derivative series): v_j = 1/2 FFT(e)[j]
  //    with e the even extension of (2 c_0, c_1, ..., c_{N-2}, 2 c_{N-1})
  {
    constexpr int kPer = kElems / kThreads;  // M * MB == kElems
    double2 ra[kPer], rb[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      int t = tid + q * kThreads;
      int j = t / MB, m = t % MB;
      int n = j < N ? j : M - j;
      double f = (n == 0 || n == N - 1) ? 2.0 : 1.0;
      double2 a = A[n * MB + m], b = B[n * MB + m];
      ra[q] = make_double2(f * a.x, f * a.y);
      rb[q] = make_double2(f * b.x, f * b.y);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      int t = tid + q * kThreads;
      int j = t / MB, m = t % MB;
      int pos = bitrev(j, logM) * MB + m;
      A[pos] = ra[q];
      B[pos] = rb[q];
    }
    __syncthreads();
  }
  fft_lds<double2, true>(A, logM, MB, 1, MB, twz, false, tid, kThreads);
  fft_lds<double2, true>(B, logM, MB, 1, MB, twz, false, tid, kThreads);

  // 7. add the correction at the window nodes and the k = 0 linear mode; write out
  for (int t = tid; t < N * MB; t += kThreads) {
    int j = t / MB, m = t % MB, mi = m0 + m;
    if (mi >= nmodes) continue;
    double2 v = B[j * MB + m], d = A[j * MB + m];
    double ps_x = 0.5 * v.x, ps_y = 0.5 * v.y, pz_x = 0.5 * d.x, pz_y = 0.5 * d.y;
    double z = zn[j];
    double k = s_k[m];
    if (k > 0.0 && s_keep[m] && z >= -g.H_E && z <= g.H + g.H_E) {
      double e1 = exp(k * (z - g.H)), e2 = exp(-k * z);
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

}  // namespace

template <typename R>
hipError_t launch_column(dpse_plan* p) {
  using C = typename CT<R>::T;
  const Geom& g = p->g;
  const int M = 2 * (g.Nz - 1);
  const int MB = kElems / M;
  const int nmodes = g.Ny * g.nkx;
  const int nb = (nmodes + MB - 1) / MB;
  hipLaunchKernelGGL(k_column<R>, dim3(nb), dim3(kThreads), 0, p->stream, g, (const C*)p->w.fx_i,
                     (const C*)p->w.fx_o, (C*)p->w.psi, (C*)p->w.psiz, (const double*)p->t.z,
                     (const double*)p->t.T0, (const double*)p->t.TH, (const double*)p->t.dT0,
                     (const double*)p->t.dTH, (const double2*)p->t.twz, p->w.scal);
  return hipGetLastError();
}

template hipError_t launch_column<double>(dpse_plan*);
template hipError_t launch_column<float>(dpse_plan*);

}  // namespace dpse
