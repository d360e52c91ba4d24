// x,y Fourier transforms of the grids (Sec. 5.2.1 steps 2 and 5).
// Forward: F(k, z_c) = (1/(Nx Ny)) sum_ij f e^{-i(kx x_i + ky y_j)} as an R2C
// pass along x (two real rows packed in one complex FFT) and a C2C pass along
// y. Inverse: from Psi and Psi_z per mode, the y pass forms Psi, -i k_y Psi
// and Psi_z; the x pass forms -i k_x Psi and returns phi, Ex, Ey, Ez = -Psi_z
// on the grid (E = -grad psi, Sec. 5.2.1 step 4), interleaved per point.
// Derivative multipliers vanish on Nyquist indices; the imaginary parts of the
// x-DC and x-Nyquist bins are dropped by the C2R pass.
#include <hip/hip_runtime.h>

#include "dpse_internal.h"
#include "fft_lds.h"

namespace dpse {

namespace {

constexpr int kThreads = 256;
constexpr int kElems = 2048;  // complex elements per LDS FFT buffer (x passes)
// y passes: kYElems complex elements per LDS buffer in blocks of kYThreads, a
// block spanning KB = kYElems / Ny consecutive kx columns (row pieces of KB
// values, 64 B; the XCD-aware block order keeps the neighbours that share
// their lines in one L2)
template <typename R>
constexpr int kYElems = sizeof(R) == 4 ? 8192 : 4096;
constexpr int kYThreads = 512;

template <typename R>
struct CT;
template <>
struct CT<double> { using T = double2; };
template <>
struct CT<float> { using T = float2; };

__host__ __device__ inline int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Up to three ranges of one forward pass in one launch (the grid of the
// inner charges and the one or two z bands of the outer grid): range s takes
// rows (x pass) or planes (y pass) [lo[s], lo[s] + cnt[s]) of in[s] (x pass)
// into out[s], with the blocks [first[s], first[s + 1]).
template <typename R>
struct FftJobs {
  const R* in[3];
  typename CT<R>::T* out[3];
  int lo[3], cnt[3];
  int first[4];
  int n;
};

// the range of block b (uniform; kernel-argument arrays read at constant indices)
template <typename R>
__device__ inline int job_of(const FftJobs<R>& J, int b) {
  return (J.n > 1 && b >= J.first[1]) + (J.n > 2 && b >= J.first[2]);
}
template <typename T, int K>
__device__ inline T pick3(const T (&a)[K], int s) {
  return s == 0 ? a[0] : (s == 1 ? a[1] : a[2]);
}

// Element at a 32-bit unsigned byte offset from a block-uniform base (the
// offsets within a plane or a block's rows stay below 2^32 bytes): the load
// or store then adds the offset to the scalar base, with no 64-bit address
// arithmetic per lane.
template <typename T>
__device__ __forceinline__ T& at_b(T* base, unsigned byte_off) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ const T& at_b(const T* base, unsigned byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

// R2C along x of the row ranges of J (rows of length Nx).
template <typename R>
__global__ void __launch_bounds__(kThreads) k_fft_x_r2c(Geom g, const FftJobs<R> J,
                                                        const typename CT<R>::T* __restrict__ twg) {
  using C = typename CT<R>::T;
  __shared__ C buf[kElems + kElems / 8];
  __shared__ C tw[512];
  const int Nx = g.Nx, logN = ilog2(Nx), nkx = g.nkx;
  const int nseq = kElems / Nx;              // row pairs per block
  const int js = job_of(J, blockIdx.x);
  const R* __restrict__ in = pick3(J.in, js);
  C* __restrict__ out = pick3(J.out, js);
  const int64_t row0 = pick3(J.lo, js), nrows = pick3(J.cnt, js);
  const int64_t r_base = row0 + (int64_t)(blockIdx.x - pick3(J.first, js)) * 2 * nseq;
  const int nr = (int)min((int64_t)2 * nseq, row0 + nrows - r_base);
  for (int i = threadIdx.x; i < Nx / 2; i += kThreads) tw[i] = twg[i];
  if constexpr (sizeof(R) == 4) {
    // slot p of sequence s (nseq * Nx == kElems) takes x = bitrev(p) of rows
    // 2s and 2s + 1. Each thread loads 4 consecutive x of both rows (16-byte
    // loads, consecutive across the lanes) and stores them to the slots
    // bitrev(x + j) = bitrev(x) + bitrev(j) Nx / 4, which the row padding
    // keeps off shared banks
    constexpr int kQ = kElems / 4 / kThreads;
    const int nq = Nx >> 2;
    const R* inb = in + r_base * Nx;  // the block's rows: 32-bit offsets from here
    float4 v0[kQ], v1[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int gq = threadIdx.x + q * kThreads, s = gq >> (logN - 2), u = gq & (nq - 1);
      const int o = ((2 * s) << logN) + 4 * u;
      v0[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      v1[q] = v0[q];
      if (2 * s < nr) v0[q] = at_b(reinterpret_cast<const float4*>(inb), (unsigned)o * 4u);
      if (2 * s + 1 < nr) v1[q] = at_b(reinterpret_cast<const float4*>(inb), (unsigned)(o + Nx) * 4u);
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int gq = threadIdx.x + q * kThreads, s = gq >> (logN - 2), u = gq & (nq - 1);
      const int p = bitrev(4 * u, logN), qn = Nx >> 2;
      C d;
      d.x = v0[q].x; d.y = v1[q].x;
      buf[rowpad_ix(s, p, Nx)] = d;
      d.x = v0[q].y; d.y = v1[q].y;
      buf[rowpad_ix(s, p + 2 * qn, Nx)] = d;
      d.x = v0[q].z; d.y = v1[q].z;
      buf[rowpad_ix(s, p + qn, Nx)] = d;
      d.x = v0[q].w; d.y = v1[q].w;
      buf[rowpad_ix(s, p + 3 * qn, Nx)] = d;
    }
  } else {
    // slot p of sequence s (nseq * Nx == kElems) takes x = bitrev(p) of rows
    // 2s and 2s + 1: the bit reversal is a gather within the row's 128-byte
    // lines and the LDS stores run in order (no bank conflicts); all global
    // loads of the thread are issued before the LDS stores
    constexpr int kPer = kElems / kThreads;
    R v0[kPer], v1[kPer];
    const R* inb = in + r_base * Nx;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = threadIdx.x + q * kThreads, s = i >> logN, x = bitrev(i & (Nx - 1), logN);
      const int o = ((2 * s) << logN) + x;
      v0[q] = 2 * s < nr ? at_b(inb, (unsigned)o * (unsigned)sizeof(R)) : (R)0;
      v1[q] = 2 * s + 1 < nr ? at_b(inb, (unsigned)(o + Nx) * (unsigned)sizeof(R)) : (R)0;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = threadIdx.x + q * kThreads;
      C d;
      d.x = v0[q];
      d.y = v1[q];
      buf[rowpad_ix(i >> logN, i & (Nx - 1), Nx)] = d;
    }
  }
  __syncthreads();
  fft_rows_r8<C, kThreads>(buf, logN, tw, false, threadIdx.x);
  const R scale = (R)(1.0 / ((double)g.Nx * (double)g.Ny));
  for (int s = 0; s < nseq; ++s)
  for (int k = threadIdx.x; k < nkx; k += kThreads) {
    C z = buf[rowpad_ix(s, k, Nx)], zc = buf[rowpad_ix(s, (Nx - k) & (Nx - 1), Nx)];
    zc.y = -zc.y;
    C a, b;
    a.x = (R)0.5 * (z.x + zc.x) * scale;
    a.y = (R)0.5 * (z.y + zc.y) * scale;
    b.x = (R)0.5 * (z.y - zc.y) * scale;
    b.y = (R)-0.5 * (z.x - zc.x) * scale;
    const int rl = 2 * s;
    C* outb = out + r_base * nkx;
    if (rl < nr) at_b(outb, __umul24((unsigned)rl, (unsigned)nkx * (unsigned)sizeof(C)) + (unsigned)k * (unsigned)sizeof(C)) = a;
    if (rl + 1 < nr) at_b(outb, __umul24((unsigned)(rl + 1), (unsigned)nkx * (unsigned)sizeof(C)) + (unsigned)k * (unsigned)sizeof(C)) = b;
  }
}

// Where thread t's values of a y-pass block go. Value q (of kPer) belongs to
// column kl = t mod KB and LDS slot p = t / KB + q step (step = kYThreads / KB
// = Ny / kPer rows), which holds row bitrev(p) = rev_t + bitrev(q) on input
// (the top bits of p are q's) and row p on output. The LDS index is
// lds0 + q lds_step: step is a multiple of the padding period wherever
// there is padding.
template <typename C, int kPer>
struct YMap {
  int kl, row_in, row_out, step, lds0, lds_step;
  __device__ YMap(int t, int logN, int logKB, int ps) {
    constexpr int logQ = kPer == 16 ? 4 : (kPer == 8 ? 3 : 2);
    static_assert((1 << logQ) == kPer, "kPer a power of two");
    const int a = t >> logKB;
    kl = t & ((1 << logKB) - 1);
    step = kYThreads >> logKB;
    row_out = a;
    row_in = bitrev(a, logN);
    lds0 = colpad_ix(a, kl, logKB, ps);
    lds_step = kYThreads + (step >> ps);
  }
  static __device__ constexpr int rev(int q) {
    constexpr int logQ = kPer == 16 ? 4 : (kPer == 8 ? 3 : 2);
    int r = 0;
    for (int b = 0; b < logQ; ++b) r |= ((q >> b) & 1) << (logQ - 1 - b);
    return r;
  }
};

// Forward C2C along y, in place, for the plane ranges of J.
template <typename R>
__global__ void __launch_bounds__(kYThreads) k_fft_y(Geom g, const FftJobs<R> J,
                                                    const typename CT<R>::T* __restrict__ twg) {
  using C = typename CT<R>::T;
  constexpr int KE = kYElems<R>;
  constexpr int kPer = KE / kYThreads;
  __shared__ C buf[colpad_elems<C>(KE)];
  __shared__ C tw[512];
  const int Ny = g.Ny, logN = ilog2(Ny), nkx = g.nkx;
  const int KB = KE / Ny, logKB = ilog2(KB), ps = colpad_shift<C>(logKB);
  const int nblk = (nkx + KB - 1) / KB;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int js = job_of(J, blk);
  typename CT<R>::T* data = pick3(J.out, js);
  const int lb = blk - pick3(J.first, js);
  const int plane = pick3(J.lo, js) + lb / nblk;
  const int kb = (lb % nblk) * KB;
  for (int i = threadIdx.x; i < Ny / 2; i += kYThreads) tw[i] = twg[i];
  // rows in bit-reversed order into the LDS slots (every row piece is read
  // on its own, so the reversal costs the loads nothing)
  const YMap<C, kPer> m(threadIdx.x, logN, logKB, ps);
  const bool valid = kb + m.kl < nkx;
  // the plane's base (uniform), then 32-bit offsets within the plane
  C* base = data + (size_t)plane * Ny * nkx;
  const int col = kb + m.kl;
  // byte offsets: row stride rs, the thread's first input and output rows
  const unsigned rs = (unsigned)nkx * (unsigned)sizeof(C), rstep = (unsigned)m.step * rs;
  const unsigned b_in = (unsigned)col * (unsigned)sizeof(C) + __umul24((unsigned)m.row_in, rs);
  const unsigned b_out = (unsigned)col * (unsigned)sizeof(C) + __umul24((unsigned)m.row_out, rs);
  C v[kPer];
  if (valid) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) v[q] = at_b(base, b_in + (unsigned)YMap<C, kPer>::rev(q) * rs);
  } else {
#pragma unroll
    for (int q = 0; q < kPer; ++q) { v[q].x = 0; v[q].y = 0; }
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) buf[m.lds0 + q * m.lds_step] = v[q];
  __syncthreads();
  fft_cols_r8<C, KE, kYThreads, false>(buf, nullptr, logN, logKB, tw, false, threadIdx.x);
  if (valid) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) at_b(base, b_out + (unsigned)q * rstep) = buf[m.lds0 + q * m.lds_step];
  }
}

// Inverse C2C along y: (Psi, Psi_z) -> (P0 = Psi, PY = -i ky Psi, PZ = Psi_z),
// y-transformed. The three transforms take turns in one LDS buffer (two
// buffers, with Psi's and -i ky Psi's transforms in lockstep, would leave room
// for one block per CU); Psi stays in registers for -i ky Psi, and Psi_z's
// loads are issued when Psi's registers are free, ahead of the second transform.
template <typename R>
__global__ void __launch_bounds__(kYThreads) k_ifft_y(Geom g, const typename CT<R>::T* __restrict__ psi,
                                                      const typename CT<R>::T* __restrict__ psiz,
                                                      typename CT<R>::T* p0, typename CT<R>::T* py,
                                                      typename CT<R>::T* pz,
                                                      const typename CT<R>::T* __restrict__ twg) {
  using C = typename CT<R>::T;
  constexpr int KE = kYElems<R>;
  constexpr int kPer = KE / kYThreads;
  __shared__ C buf[colpad_elems<C>(KE)];
  __shared__ C tw[512];
  const int Ny = g.Ny, logN = ilog2(Ny), nkx = g.nkx;
  const int KB = KE / Ny, logKB = ilog2(KB), ps = colpad_shift<C>(logKB);
  const int nblk = (nkx + KB - 1) / KB;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int plane = blk / nblk;
  const int kb = (blk % nblk) * KB;
  for (int i = threadIdx.x; i < Ny / 2; i += kYThreads) tw[i] = twg[i];
  // rows in bit-reversed order into the LDS slots (separate row pieces: the
  // reversal costs the loads nothing)
  const YMap<C, kPer> m(threadIdx.x, logN, logKB, ps);
  const bool valid = kb + m.kl < nkx;
  // the plane's offset (uniform), then 32-bit offsets within the plane
  const size_t poff = (size_t)plane * Ny * nkx;
  const int col = kb + m.kl;
  const unsigned rs = (unsigned)nkx * (unsigned)sizeof(C), rstep = (unsigned)m.step * rs;
  const unsigned b_in = (unsigned)col * (unsigned)sizeof(C) + __umul24((unsigned)m.row_in, rs);
  const unsigned b_out = (unsigned)col * (unsigned)sizeof(C) + __umul24((unsigned)m.row_out, rs);
  auto load = [&](C (&v)[kPer], const C* __restrict__ src) {
    const C* sp = src + poff;
    if (valid) {
#pragma unroll
      for (int q = 0; q < kPer; ++q) v[q] = at_b(sp, b_in + (unsigned)YMap<C, kPer>::rev(q) * rs);
    } else {
#pragma unroll
      for (int q = 0; q < kPer; ++q) { v[q].x = 0; v[q].y = 0; }
    }
  };
  const double kyf = 2.0 * kPi / g.Ly;
  auto put = [&](const C (&v)[kPer], bool deriv) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      C d = v[q];
      if (deriv) {  // -i ky Psi
        const int ky = m.row_in + YMap<C, kPer>::rev(q);
        const int ny = ky < Ny / 2 ? ky : ky - Ny;
        const R kyv = (ky == Ny / 2) ? (R)0 : (R)(kyf * ny);
        d.x = kyv * v[q].y;
        d.y = -kyv * v[q].x;
      }
      buf[m.lds0 + q * m.lds_step] = d;
    }
  };
  auto store = [&](C* dst) {
    C* dp = dst + poff;
    if (valid) {
#pragma unroll
      for (int q = 0; q < kPer; ++q) at_b(dp, b_out + (unsigned)q * rstep) = buf[m.lds0 + q * m.lds_step];
    }
  };
  C v[kPer];
  load(v, psi);
  put(v, false);
  __syncthreads();
  fft_cols_r8<C, KE, kYThreads, false>(buf, nullptr, logN, logKB, tw, true, threadIdx.x);
  store(p0);
  __syncthreads();
  put(v, true);
  load(v, psiz);
  __syncthreads();
  fft_cols_r8<C, KE, kYThreads, false>(buf, nullptr, logN, logKB, tw, true, threadIdx.x);
  store(py);
  __syncthreads();
  put(v, false);
  __syncthreads();
  fft_cols_r8<C, KE, kYThreads, false>(buf, nullptr, logN, logKB, tw, true, threadIdx.x);
  store(pz);
}

// Inverse C2R along x: rows of (P0, PY, PZ) -> u4[row][x] = (phi, Ex, Ey, Ez).
template <typename R>
__global__ void __launch_bounds__(kThreads) k_ifft_x_c2r(Geom g, const typename CT<R>::T* __restrict__ p0,
                                                         const typename CT<R>::T* __restrict__ py,
                                                         const typename CT<R>::T* __restrict__ pz, R* __restrict__ u4,
                                                         int64_t nrows, const typename CT<R>::T* __restrict__ twg) {
  using C = typename CT<R>::T;
  __shared__ C buf[kElems + kElems / 8];
  __shared__ C tw[512];
  const int Nx = g.Nx, logN = ilog2(Nx), nkx = g.nkx;
  const int nrow_blk = kElems / (2 * Nx);  // rows per block (2 sequences per row)
  const int64_t r_base = (int64_t)xcd_block(blockIdx.x, gridDim.x) * nrow_blk;
  const int nr = (int)min((int64_t)nrow_blk, nrows - r_base);
  for (int i = threadIdx.x; i < Nx / 2; i += kThreads) tw[i] = twg[i];
  const double kxf = 2.0 * kPi / g.Lx;
  // the block's rows (uniform bases), then 32-bit offsets
  const C* p0b = p0 + r_base * nkx;
  const C* pyb = py + r_base * nkx;
  const C* pzb = pz + r_base * nkx;
  // the two sequences of row rl at wavenumber k (slot bitrev(k)), formed from
  // the stored half spectrum at kk = min(k, Nx - k) (conjugated for k > Nx/2):
  // z1 = phi_hat + i Ex_hat, z2 = Ey_hat + i Ez_hat, Ex_hat = -i kx phi_hat,
  // Ez_hat = -Psi_z_hat
  auto seqs = [&](C a, C b, C c, int kk, bool cj, C& z1, C& z2) {
    if (kk == 0 || kk == Nx / 2) { a.y = 0; b.y = 0; c.y = 0; }
    const R kxv = (kk == Nx / 2) ? (R)0 : (R)(kxf * kk);
    C ex;
    ex.x = kxv * a.y;
    ex.y = -kxv * a.x;
    C ez;
    ez.x = -c.x;
    ez.y = -c.y;
    if (cj) { a.y = -a.y; ex.y = -ex.y; b.y = -b.y; ez.y = -ez.y; }
    z1.x = a.x - ex.y; z1.y = a.y + ex.x;
    z2.x = b.x - ez.y; z2.y = b.y + ez.x;
  };
  if constexpr (sizeof(R) == 4) {
    // each stored coefficient kk < Nx/2 is loaded once (consecutive across
    // the lanes) and fills the slots of k = kk and k = Nx - kk; the Nyquist
    // coefficients by one thread per row
    constexpr int kQ = kElems / 4 / kThreads;
    const int hx = Nx >> 1;
    C la[kQ], lb[kQ], lc[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int gq = threadIdx.x + q * kThreads, rl = gq >> (logN - 1), kk = gq & (hx - 1);
      la[q].x = 0; la[q].y = 0; lb[q] = la[q]; lc[q] = la[q];
      if (rl < nr) {
        const unsigned o = __umul24((unsigned)rl, (unsigned)nkx * (unsigned)sizeof(C)) + (unsigned)kk * (unsigned)sizeof(C);
        la[q] = at_b(p0b, o);
        lb[q] = at_b(pyb, o);
        lc[q] = at_b(pzb, o);
      }
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int gq = threadIdx.x + q * kThreads, rl = gq >> (logN - 1), kk = gq & (hx - 1);
      C z1, z2;
      seqs(la[q], lb[q], lc[q], kk, false, z1, z2);
      const int p = bitrev(kk, logN);
      buf[rowpad_ix(2 * rl, p, Nx)] = z1;
      buf[rowpad_ix(2 * rl + 1, p, Nx)] = z2;
      if (kk > 0) {
        seqs(la[q], lb[q], lc[q], kk, true, z1, z2);
        const int pm = bitrev(Nx - kk, logN);
        buf[rowpad_ix(2 * rl, pm, Nx)] = z1;
        buf[rowpad_ix(2 * rl + 1, pm, Nx)] = z2;
      }
    }
    if (threadIdx.x < nrow_blk) {
      const int rl = threadIdx.x;
      C a, b, c;
      a.x = 0; a.y = 0; b = a; c = a;
      if (rl < nr) {
        const unsigned o = __umul24((unsigned)rl, (unsigned)nkx * (unsigned)sizeof(C)) + (unsigned)hx * (unsigned)sizeof(C);
        a = at_b(p0b, o);
        b = at_b(pyb, o);
        c = at_b(pzb, o);
      }
      C z1, z2;
      seqs(a, b, c, hx, false, z1, z2);
      buf[rowpad_ix(2 * rl, 1, Nx)] = z1;  // bitrev(Nx / 2) = 1
      buf[rowpad_ix(2 * rl + 1, 1, Nx)] = z2;
    }
  } else {
    // nrow_blk * Nx == kElems / 2 slots; slot p of row rl takes k = bitrev(p)
    // (a gather within the row's lines; LDS stores in order); all global loads
    // of the thread are issued before the LDS stores
    constexpr int kPer = kElems / 2 / kThreads;
    C la[kPer], lb[kPer], lc[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = threadIdx.x + q * kThreads, rl = i >> logN, k = bitrev(i & (Nx - 1), logN);
      la[q].x = 0; la[q].y = 0; lb[q] = la[q]; lc[q] = la[q];
      if (rl < nr) {
        const int kk = k <= Nx / 2 ? k : Nx - k;
        const unsigned o = __umul24((unsigned)rl, (unsigned)nkx * (unsigned)sizeof(C)) + (unsigned)kk * (unsigned)sizeof(C);
        la[q] = at_b(p0b, o);
        lb[q] = at_b(pyb, o);
        lc[q] = at_b(pzb, o);
      }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = threadIdx.x + q * kThreads, rl = i >> logN, pos = i & (Nx - 1), k = bitrev(pos, logN);
      C z1, z2;
      z1.x = 0; z1.y = 0; z2.x = 0; z2.y = 0;
      if (rl < nr) seqs(la[q], lb[q], lc[q], k <= Nx / 2 ? k : Nx - k, k > Nx / 2, z1, z2);
      buf[rowpad_ix(2 * rl, pos, Nx)] = z1;
      buf[rowpad_ix(2 * rl + 1, pos, Nx)] = z2;
    }
  }
  __syncthreads();
  fft_rows_r8<C, kThreads>(buf, logN, tw, true, threadIdx.x);
  using V = typename std::conditional<sizeof(R) == 8, double4, float4>::type;
  V* out = reinterpret_cast<V*>(u4) + r_base * Nx;  // the block's rows: 32-bit offsets from here
  for (int i = threadIdx.x; i < nr * Nx; i += kThreads) {
    const int rl = i >> logN, x = i & (Nx - 1);
    C z1 = buf[rowpad_ix(2 * rl, x, Nx)], z2 = buf[rowpad_ix(2 * rl + 1, x, Nx)];
    V v;
    v.x = z1.x; v.y = z1.y; v.z = z2.x; v.w = z2.y;
    at_b(out, (unsigned)i * (unsigned)sizeof(V)) = v;
  }
}

template <typename R>
const typename CT<R>::T* twx(dpse_plan* p);
template <>
const double2* twx<double>(dpse_plan* p) { return p->t.twx; }
template <>
const float2* twx<float>(dpse_plan* p) { return p->t.twx_f; }
template <typename R>
const typename CT<R>::T* twy(dpse_plan* p);
template <>
const double2* twy<double>(dpse_plan* p) { return p->t.twy; }
template <>
const float2* twy<float>(dpse_plan* p) { return p->t.twy_f; }

template <typename R>
void add_x_rows(const Geom& g, FftJobs<R>& J, const R* in, typename CT<R>::T* out, int plane_a, int plane_b) {
  if (plane_b <= plane_a) return;
  const int rows = (plane_b - plane_a) * g.Ny, rows_per = 2 * (kElems / g.Nx);
  J.in[J.n] = in;
  J.out[J.n] = out;
  J.lo[J.n] = plane_a * g.Ny;
  J.cnt[J.n] = rows;
  J.first[J.n + 1] = J.first[J.n] + (rows + rows_per - 1) / rows_per;
  ++J.n;
}

template <typename R>
void add_y_planes(const Geom& g, FftJobs<R>& J, typename CT<R>::T* data, int plane_a, int plane_b) {
  if (plane_b <= plane_a) return;
  const int KB = kYElems<R> / g.Ny, nblk = (g.nkx + KB - 1) / KB;
  J.in[J.n] = nullptr;
  J.out[J.n] = data;
  J.lo[J.n] = plane_a;
  J.cnt[J.n] = plane_b - plane_a;
  J.first[J.n + 1] = J.first[J.n] + nblk * (plane_b - plane_a);
  ++J.n;
}

template <typename R>
FftJobs<R> no_jobs() {
  FftJobs<R> J{};
  J.first[0] = 0;
  J.n = 0;
  return J;
}

template <typename R>
void launch_x(dpse_plan* p, const FftJobs<R>& J) {
  if (J.n > 0)
    hipLaunchKernelGGL(k_fft_x_r2c<R>, dim3(J.first[J.n]), dim3(kThreads), 0, p->stream, p->g, J, twx<R>(p));
}

template <typename R>
void launch_y(dpse_plan* p, const FftJobs<R>& J) {
  if (J.n > 0)
    hipLaunchKernelGGL(k_fft_y<R>, dim3(J.first[J.n]), dim3(kYThreads), 0, p->stream, p->g, J, twy<R>(p));
}

}  // namespace

template <typename R>
hipError_t launch_fft_forward(dpse_plan* p) {
  using C = typename CT<R>::T;
  const Geom& g = p->g;
  FftJobs<R> X = no_jobs<R>(), Y = no_jobs<R>();
  add_x_rows<R>(g, X, (const R*)p->w.f_i, (C*)p->w.fx_i, 0, g.Nz);
  add_y_planes<R>(g, Y, (C*)p->w.fx_i, 0, g.Nz);
  // the wall-group grid only on its bands (one range where they meet)
  if (g.top_end >= g.bot_begin) {
    const int a = std::min(g.top_lo, g.bot_begin), b = std::max(g.top_end, g.bot_end);
    add_x_rows<R>(g, X, (const R*)p->w.f_o, (C*)p->w.fx_o, a, b);
    add_y_planes<R>(g, Y, (C*)p->w.fx_o, a, b);
  } else {
    add_x_rows<R>(g, X, (const R*)p->w.f_o, (C*)p->w.fx_o, g.top_lo, g.top_end);
    add_x_rows<R>(g, X, (const R*)p->w.f_o, (C*)p->w.fx_o, g.bot_begin, g.bot_end);
    add_y_planes<R>(g, Y, (C*)p->w.fx_o, g.top_lo, g.top_end);
    add_y_planes<R>(g, Y, (C*)p->w.fx_o, g.bot_begin, g.bot_end);
  }
  launch_x<R>(p, X);
  launch_y<R>(p, Y);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fft_inverse(dpse_plan* p) {
  using C = typename CT<R>::T;
  const Geom& g = p->g;
  int KB = kYElems<R> / g.Ny;
  int nblk = (g.nkx + KB - 1) / KB;
  hipLaunchKernelGGL(k_ifft_y<R>, dim3(nblk * g.Nz), dim3(kYThreads), 0, p->stream, g, (const C*)p->w.psi,
                     (const C*)p->w.psiz, (C*)p->w.p0, (C*)p->w.py, (C*)p->w.pz, twy<R>(p));
  int64_t nrows = (int64_t)g.Nz * g.Ny;
  int rows_per = kElems / (2 * g.Nx);
  int nb = (int)((nrows + rows_per - 1) / rows_per);
  hipLaunchKernelGGL(k_ifft_x_c2r<R>, dim3(nb), dim3(kThreads), 0, p->stream, g, (const C*)p->w.p0,
                     (const C*)p->w.py, (const C*)p->w.pz, (R*)p->w.u4, nrows, twx<R>(p));
  return hipGetLastError();
}

// x,y transforms (FP64, the normalisation of the forward transform) of the
// two staged wall densities, planes 0 (bottom) and 1 (top).
hipError_t launch_wall_transforms(dpse_plan* p) {
  FftJobs<double> X = no_jobs<double>(), Y = no_jobs<double>();
  add_x_rows<double>(p->g, X, (const double*)p->walls.stage, (double2*)p->walls.hat, 0, 2);
  add_y_planes<double>(p->g, Y, (double2*)p->walls.hat, 0, 2);
  launch_x<double>(p, X);
  launch_y<double>(p, Y);
  return hipGetLastError();
}

namespace {
// The potential channel of the interleaved field grid [G][4] into out [G].
template <typename R>
__global__ void __launch_bounds__(kThreads) k_keep_phi(int64_t G, const R* __restrict__ u4, R* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < G; i += (int64_t)gridDim.x * kThreads)
    out[i] = u4[4 * i];
}
}  // namespace

template <typename R>
hipError_t launch_wall_keep_phi(dpse_plan* p) {
  const Geom& g = p->g;
  const int64_t G = (int64_t)g.Nz * g.Ny * g.Nx;
  const int nb = (int)((G + kThreads - 1) / kThreads < 8192 ? (G + kThreads - 1) / kThreads : 8192);
  hipLaunchKernelGGL(k_keep_phi<R>, dim3(nb), dim3(kThreads), 0, p->stream, G, (const R*)p->w.u4,
                     (R*)p->walls.phis);
  return hipGetLastError();
}

template hipError_t launch_wall_keep_phi<double>(dpse_plan*);
template hipError_t launch_wall_keep_phi<float>(dpse_plan*);
template hipError_t launch_fft_forward<double>(dpse_plan*);
template hipError_t launch_fft_forward<float>(dpse_plan*);
template hipError_t launch_fft_inverse<double>(dpse_plan*);
template hipError_t launch_fft_inverse<float>(dpse_plan*);

}  // namespace dpse
