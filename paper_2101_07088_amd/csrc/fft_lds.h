// Batched complex FFTs on data held in LDS (in-place radix-2, decimation in
// time, input in bit-reversed order), shared by the x,y transforms and the
// Chebyshev (DCT-I) transforms of the column kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace dpse {

template <typename C>
__device__ inline C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C>
__device__ inline C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C>
__device__ inline C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

__device__ inline int bitrev(int k, int logL) { return (int)(__brev((unsigned)k) >> (32 - logL)); }

// Twiddle strides ts of the passes below are powers of two (L / (2 half) and
// its halves), so pos * ts is taken as pos << ctz(ts): a shift by a uniform
// amount instead of a per-lane 32-bit multiply.

// nseq sequences of length L = 2^logL; element k of sequence s lives at
// buf[s * ss + k * es]; input in bit-reversed order, output natural order.
// tw[k] = exp(-2 pi i k / L) for k < L/2 (conjugated when inverse).
// SEQ_FAST maps consecutive threads to consecutive sequences (use when es == 1
// is false and ss == 1), otherwise to consecutive butterflies.
template <typename C, bool SEQ_FAST>
__device__ void fft_lds(C* buf, int logL, int nseq, int ss, int es, const C* tw, bool inverse,
                        int tid, int nthr) {
  const int L = 1 << logL;
  const int nb = L >> 1;
  for (int lh = 0; lh < logL; ++lh) {
    const int half = 1 << lh;
    const int tstride = nb >> lh;
    for (int t = tid; t < nseq * nb; t += nthr) {
      int s, b;
      if (SEQ_FAST) { s = t % nseq; b = t / nseq; }
      else { b = t % nb; s = t / nb; }
      int grp = b >> lh, pos = b & (half - 1);
      int i0 = (grp << (lh + 1)) + pos, i1 = i0 + half;
      C w = tw[pos * tstride];
      if (inverse) w.y = -w.y;
      C* p0 = buf + s * ss + i0 * es;
      C* p1 = buf + s * ss + i1 * es;
      C u = *p0, v = cmul(*p1, w);
      *p0 = cadd(u, v);
      *p1 = csub(u, v);
    }
    __syncthreads();
  }
}

// Same transform with a compile-time count of butterflies per thread and
// stage (nseq * L/2 == BPT * nthr): the loads of all BPT butterflies are
// issued before any arithmetic, so their latencies overlap.
template <typename C, bool SEQ_FAST, int BPT, int NTHR>
__device__ void fft_lds_u(C* buf, int logL, int nseq, int ss, int es, const C* tw, bool inverse, int tid) {
  const int nb = (1 << logL) >> 1;
  for (int lh = 0; lh < logL; ++lh) {
    const int half = 1 << lh;
    const int tstride = nb >> lh;
    C u[BPT], v[BPT], w[BPT];
    int p0[BPT], p1[BPT];
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int t = tid + q * NTHR;
      int s, b;
      if (SEQ_FAST) { s = t % nseq; b = t / nseq; }
      else { b = t % nb; s = t / nb; }
      const int grp = b >> lh, pos = b & (half - 1);
      const int i0 = (grp << (lh + 1)) + pos;
      p0[q] = s * ss + i0 * es;
      p1[q] = p0[q] + half * es;
      w[q] = tw[pos * tstride];
      u[q] = buf[p0[q]];
      v[q] = buf[p1[q]];
    }
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      C ww = w[q];
      if (inverse) ww.y = -ww.y;
      const C vw = cmul(v[q], ww);
      buf[p0[q]] = cadd(u[q], vw);
      buf[p1[q]] = csub(u[q], vw);
    }
    __syncthreads();
  }
}

// Radix-2^2 version: one pass fuses the radix-2 stages lh and lh+1 on four
// elements (i, i+h, i+2h, i+3h), halving LDS traffic and barriers; an odd
// log-length starts with one radix-2 stage. BPT4 = nseq * L/4 / NTHR.
template <typename C, bool SEQ_FAST, int BPT4, int NTHR>
__device__ void fft_lds_r22(C* buf, int logL, int lognseq, int ss, int es, const C* tw, bool inverse, int tid) {
  const int nseq = 1 << lognseq;
  const int L = 1 << logL;
  const int nb4 = L >> 2;
  const int lognb4 = logL - 2;
  int lh = 0;
  if (logL & 1) {
    // first radix-2 stage (half = 1, twiddle 1): pairs (2b, 2b+1)
#pragma unroll
    for (int q = 0; q < 2 * BPT4; ++q) {
      const int t = tid + q * NTHR;
      int s, b;
      if (SEQ_FAST) { s = t & (nseq - 1); b = t >> lognseq; }
      else { b = t & ((L >> 1) - 1); s = t >> (logL - 1); }
      C* p0 = buf + s * ss + (2 * b) * es;
      C* p1 = p0 + es;
      const C u = *p0, v = *p1;
      *p0 = cadd(u, v);
      *p1 = csub(u, v);
    }
    __syncthreads();
    lh = 1;
  }
  for (; lh < logL; lh += 2) {
    const int half = 1 << lh;
    const int ts1 = (L >> 1) >> lh;   // twiddle stride of stage lh: L / (2 half)
    const int ts2 = ts1 >> 1;         // of stage lh + 1: L / (4 half)
    C a[BPT4][4], w1[BPT4], w2[BPT4];
    int base[BPT4];
#pragma unroll
    for (int q = 0; q < BPT4; ++q) {
      const int t = tid + q * NTHR;
      int s, b;
      if (SEQ_FAST) { s = t & (nseq - 1); b = t >> lognseq; }
      else { b = t & (nb4 - 1); s = t >> lognb4; }
      const int grp = b >> lh, pos = b & (half - 1);
      base[q] = s * ss + ((grp << (lh + 2)) + pos) * es;
      w1[q] = tw[pos << __builtin_ctz(ts1)];
      w2[q] = tw[pos << __builtin_ctz(ts2)];
#pragma unroll
      for (int e = 0; e < 4; ++e) a[q][e] = buf[base[q] + e * half * es];
    }
#pragma unroll
    for (int q = 0; q < BPT4; ++q) {
      C x1 = w1[q], x2 = w2[q];
      if (inverse) { x1.y = -x1.y; x2.y = -x2.y; }
      const C t1 = cmul(a[q][1], x1), t3 = cmul(a[q][3], x1);
      const C b0 = cadd(a[q][0], t1), b1 = csub(a[q][0], t1);
      const C b2 = cadd(a[q][2], t3), b3 = csub(a[q][2], t3);
      const C u2 = cmul(b2, x2);
      C u3 = cmul(b3, x2);  // times -i (forward) or +i (inverse)
      {
        const auto re = u3.x;
        if (inverse) { u3.x = -u3.y; u3.y = re; }
        else { u3.x = u3.y; u3.y = -re; }
      }
      buf[base[q]] = cadd(b0, u2);
      buf[base[q] + 2 * half * es] = csub(b0, u2);
      buf[base[q] + half * es] = cadd(b1, u3);
      buf[base[q] + 3 * half * es] = csub(b1, u3);
    }
    __syncthreads();
  }
}

// Two transforms of the same shape (two buffers, same twiddles) in lockstep:
// every pass does the butterflies of both buffers, so the pair costs the
// barriers of one transform and each thread has twice the independent work
// between them.
template <typename C, bool SEQ_FAST, int BPT4, int NTHR>
__device__ void fft_lds_r22_pair(C* buf0, C* buf1, int logL, int lognseq, int ss, int es, const C* tw, bool inverse,
                                 int tid) {
  const int nseq = 1 << lognseq;
  const int L = 1 << logL;
  const int nb4 = L >> 2;
  const int lognb4 = logL - 2;
  int lh = 0;
  if (logL & 1) {
#pragma unroll
    for (int q = 0; q < 2 * BPT4; ++q) {
      const int t = tid + q * NTHR;
      int s, b;
      if (SEQ_FAST) { s = t & (nseq - 1); b = t >> lognseq; }
      else { b = t & ((L >> 1) - 1); s = t >> (logL - 1); }
      const int o = s * ss + (2 * b) * es;
      const C u0 = buf0[o], v0 = buf0[o + es], u1 = buf1[o], v1 = buf1[o + es];
      buf0[o] = cadd(u0, v0);
      buf0[o + es] = csub(u0, v0);
      buf1[o] = cadd(u1, v1);
      buf1[o + es] = csub(u1, v1);
    }
    __syncthreads();
    lh = 1;
  }
  for (; lh < logL; lh += 2) {
    const int half = 1 << lh;
    const int ts1 = (L >> 1) >> lh;
    const int ts2 = ts1 >> 1;
    C a[2][BPT4][4], w1[BPT4], w2[BPT4];
    int base[BPT4];
#pragma unroll
    for (int q = 0; q < BPT4; ++q) {
      const int t = tid + q * NTHR;
      int s, b;
      if (SEQ_FAST) { s = t & (nseq - 1); b = t >> lognseq; }
      else { b = t & (nb4 - 1); s = t >> lognb4; }
      const int grp = b >> lh, pos = b & (half - 1);
      base[q] = s * ss + ((grp << (lh + 2)) + pos) * es;
      w1[q] = tw[pos << __builtin_ctz(ts1)];
      w2[q] = tw[pos << __builtin_ctz(ts2)];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a[0][q][e] = buf0[base[q] + e * half * es];
        a[1][q][e] = buf1[base[q] + e * half * es];
      }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      C* buf = bi == 0 ? buf0 : buf1;
#pragma unroll
      for (int q = 0; q < BPT4; ++q) {
        C x1 = w1[q], x2 = w2[q];
        if (inverse) { x1.y = -x1.y; x2.y = -x2.y; }
        const C t1 = cmul(a[bi][q][1], x1), t3 = cmul(a[bi][q][3], x1);
        const C b0 = cadd(a[bi][q][0], t1), b1 = csub(a[bi][q][0], t1);
        const C b2 = cadd(a[bi][q][2], t3), b3 = csub(a[bi][q][2], t3);
        const C u2 = cmul(b2, x2);
        C u3 = cmul(b3, x2);  // times -i (forward) or +i (inverse)
        {
          const auto re = u3.x;
          if (inverse) { u3.x = -u3.y; u3.y = re; }
          else { u3.x = u3.y; u3.y = -re; }
        }
        buf[base[q]] = cadd(b0, u2);
        buf[base[q] + 2 * half * es] = csub(b0, u2);
        buf[base[q] + half * es] = cadd(b1, u3);
        buf[base[q] + 3 * half * es] = csub(b1, u3);
      }
    }
    __syncthreads();
  }
}

}  // namespace dpse

namespace dpse {

// Row-major batches of nseq sequences of length N = 2^logN in LDS, element k of
// sequence s at rowpad_ix(s, k, N) (one padding element after every 8, which
// keeps the radix-2^3 passes below off shared banks). Input in bit-reversed
// order, output natural; tw[k] = exp(-2 pi i k / N) for k < N/2 (conjugated
// when inverse). Passes of three radix-2 stages (k0 + e half, e < 8), two where
// the stage count requires: 2^10 = 8 8 4 4, 2^9 = 8 8 8, 2^8 = 8 8 4, 2^7 =
// 8 4 4, 2^6 = 8 8, 2^5 = 8 4. nseq N == NTHR 8. Threads take consecutive
// groups of one sequence.
__device__ __forceinline__ int rowpad_ix(int s, int k, int N) { return s * (N + (N >> 3)) + k + (k >> 3); }

template <typename C, int NTHR>
__device__ void fft_rows_r8(C* buf, int logN, const C* tw, bool inverse, int tid) {
  using Rr = decltype(C{}.x);
  const int N = 1 << logN;
  const Rr r2 = (Rr)0.70710678118654752440;
  const Rr sg = inverse ? (Rr)-1 : (Rr)1;  // forward: times -i and exp(-i pi/4); inverse: the conjugates
  // a pass's elements k0 + e half sit at base + e stride: for rows of 32 and
  // more, half is 1 (k0 a multiple of 8) or a multiple of 8, so the padding
  // adds e (half / 8)
  auto pass8 = [&](int lh) {
    const int half = 1 << lh, ts1 = (N >> 1) >> lh, ts2 = ts1 >> 1, ts3 = ts1 >> 2;
    const int lg = logN - 3, b = tid & ((1 << lg) - 1), s = tid >> lg;
    const int grp = b >> lh, pos = b & (half - 1), k0 = (grp << (lh + 3)) + pos;
    const int base = rowpad_ix(s, k0, N), stride = half + (half >> 3);
    C v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = buf[base + e * stride];
    if (lh == 0) {
      // first pass: the twiddles are 1, -i and exp(-i pi e / 4) (conjugated
      // when inverse), no table products
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
        if (e & 1) {
          const Rr x = t.x;
          t.x = sg * t.y;
          t.y = -sg * x;
        }
        v[e + 2] = csub(v[e], t);
        v[e] = cadd(v[e], t);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        C t = v[e + 4];
        const Rr x = t.x, y = t.y;
        if (e == 1) { t.x = r2 * (x + sg * y); t.y = r2 * (y - sg * x); }
        if (e == 2) { t.x = sg * y; t.y = -sg * x; }
        if (e == 3) { t.x = r2 * (sg * y - x); t.y = -r2 * (y + sg * x); }
        v[e + 4] = csub(v[e], t);
        v[e] = cadd(v[e], t);
      }
    } else {
      C w1 = tw[pos << __builtin_ctz(ts1)], w2 = tw[pos << __builtin_ctz(ts2)], w3 = tw[pos << __builtin_ctz(ts3)];
      if (inverse) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
      C w2m, w3e[4];
      w2m.x = sg * w2.y;
      w2m.y = -sg * w2.x;
      w3e[0] = w3;
      w3e[1].x = r2 * (w3.x + sg * w3.y);
      w3e[1].y = r2 * (w3.y - sg * w3.x);
      w3e[2].x = sg * w3.y;
      w3e[2].y = -sg * w3.x;
      w3e[3].x = r2 * (sg * w3.y - w3.x);
      w3e[3].y = -r2 * (sg * w3.x + w3.y);
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
#pragma unroll
    for (int e = 0; e < 8; ++e) buf[base + e * stride] = v[e];
    __syncthreads();
  };
  auto pass4 = [&](int lh) {
    const int half = 1 << lh, ts1 = (N >> 1) >> lh, ts2 = ts1 >> 1;
    const int lg = logN - 2, stride = half + (half >> 3);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int t = tid + q * NTHR, b = t & ((1 << lg) - 1), s = t >> lg;
      const int grp = b >> lh, pos = b & (half - 1), k0 = (grp << (lh + 2)) + pos;
      const int base = rowpad_ix(s, k0, N);
      C x1 = tw[pos << __builtin_ctz(ts1)], x2 = tw[pos << __builtin_ctz(ts2)];
      if (inverse) { x1.y = -x1.y; x2.y = -x2.y; }
      C a[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = buf[base + e * stride];
      const C t1 = cmul(a[1], x1), t3 = cmul(a[3], x1);
      const C b0 = cadd(a[0], t1), b1 = csub(a[0], t1);
      const C b2 = cadd(a[2], t3), b3 = csub(a[2], t3);
      const C u2 = cmul(b2, x2);
      C u3 = cmul(b3, x2);  // times -i (forward) or +i (inverse)
      {
        const auto re = u3.x;
        if (inverse) { u3.x = -u3.y; u3.y = re; }
        else { u3.x = u3.y; u3.y = -re; }
      }
      buf[base] = cadd(b0, u2);
      buf[base + 2 * stride] = csub(b0, u2);
      buf[base + stride] = cadd(b1, u3);
      buf[base + 3 * stride] = csub(b1, u3);
    }
    __syncthreads();
  };
  const int n8 = logN % 3 == 0 ? logN / 3 : (logN % 3 == 1 ? (logN - 4) / 3 : (logN - 2) / 3);
  const int n4 = (logN - 3 * n8) / 2;
#pragma nounroll
  for (int p = 0; p < n8; ++p) pass8(3 * p);
#pragma nounroll
  for (int p = 0; p < n4; ++p) pass4(3 * n8 + 2 * p);
}

}  // namespace dpse

namespace dpse {

// Column-interleaved batches: 2^logS sequences (columns) of length M = 2^logM
// stored row by row, element k of sequence s at colpad_ix(k, s) (with fewer
// than 32 columns, one padding element every 2^ps rows, ps = colpad_shift: the
// passes below then stay off shared banks). Input in bit-reversed order, output
// natural; tw[k] = exp(-2 pi i k / M), k < M/2 (conjugated when inverse).
// Radix-2^3 passes (two stages where the count requires, as fft_rows_r8), on
// one buffer or on two in lockstep (PAIR); with fewer than 32 columns the first
// pass gives a wave consecutive groups of one column. M 2^logS == KE.
template <typename C>
__device__ __forceinline__ int colpad_shift(int logS) {
  return logS >= 5 ? 30 : (sizeof(C) == 8 ? 3 : 4);
}
__device__ __forceinline__ int colpad_ix(int k, int s, int logS, int ps) { return (k << logS) + s + (k >> ps); }
// LDS elements a column-interleaved buffer of KE elements takes with padding
template <typename C>
constexpr int colpad_elems(int KE) { return KE + 1024 / (sizeof(C) == 8 ? 8 : 16); }

template <typename C, int KE, int NTHR, bool PAIR>
__device__ void fft_cols_r8(C* A, C* B, int logM, int logS, const C* tw, bool inverse, int tid) {
  using Rr = decltype(C{}.x);
  static_assert(KE % (8 * NTHR) == 0, "whole radix-8 groups per thread");
  const int M = 1 << logM, S = 1 << logS, ps = colpad_shift<C>(logS);
  const bool gfirst = logS < 5;
  auto pass8 = [&](int lh, bool gfast) {
    const int half = 1 << lh, ts1 = (M >> 1) >> lh, ts2 = ts1 >> 1, ts3 = ts1 >> 2;
    const int logG = logM - 3;
#pragma nounroll
    for (int q = 0; q < KE / (8 * NTHR); ++q) {
    const int t = tid + q * NTHR;
    int s, b;
    if (gfast) {
      b = t & ((1 << logG) - 1);
      s = t >> logG;
    } else {
      s = t & (S - 1);
      b = t >> logS;
    }
    const int grp = b >> lh, pos = b & (half - 1), k0 = (grp << (lh + 3)) + pos;
    C w1 = tw[pos << __builtin_ctz(ts1)], w2 = tw[pos << __builtin_ctz(ts2)], w3 = tw[pos << __builtin_ctz(ts3)];
    if (inverse) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
    const Rr r2 = (Rr)0.70710678118654752440;
    const Rr sg = inverse ? (Rr)-1 : (Rr)1;
    C w2m, w3e[4];
    w2m.x = sg * w2.y;
    w2m.y = -sg * w2.x;
    w3e[0] = w3;
    w3e[1].x = r2 * (w3.x + sg * w3.y);
    w3e[1].y = r2 * (w3.y - sg * w3.x);
    w3e[2].x = sg * w3.y;
    w3e[2].y = -sg * w3.x;
    w3e[3].x = r2 * (sg * w3.y - w3.x);
    w3e[3].y = -r2 * (sg * w3.x + w3.y);
    constexpr int NB = PAIR ? 2 : 1;
    C v[NB][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int ix = colpad_ix(k0 + e * half, s, logS, ps);
      v[0][e] = A[ix];
      if (PAIR) v[NB - 1][e] = B[ix];
    }
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
      C* u = v[bi];
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        const C t = cmul(u[e + 1], w1);
        u[e + 1] = csub(u[e], t);
        u[e] = cadd(u[e], t);
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (e & 2) continue;
        const C t = cmul(u[e + 2], (e & 1) ? w2m : w2);
        u[e + 2] = csub(u[e], t);
        u[e] = cadd(u[e], t);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const C t = cmul(u[e + 4], w3e[e]);
        u[e + 4] = csub(u[e], t);
        u[e] = cadd(u[e], t);
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int ix = colpad_ix(k0 + e * half, s, logS, ps);
      A[ix] = v[0][e];
      if (PAIR) B[ix] = v[NB - 1][e];
    }
    }
    __syncthreads();
  };
  auto pass4 = [&](int lh) {
    const int half = 1 << lh, ts1 = (M >> 1) >> lh, ts2 = ts1 >> 1;
#pragma nounroll
    for (int q = 0; q < KE / (4 * NTHR); ++q) {
      const int t = tid + q * NTHR, s = t & (S - 1), b = t >> logS;
      const int grp = b >> lh, pos = b & (half - 1), k0 = (grp << (lh + 2)) + pos;
      C x1 = tw[pos << __builtin_ctz(ts1)], x2 = tw[pos << __builtin_ctz(ts2)];
      if (inverse) { x1.y = -x1.y; x2.y = -x2.y; }
      constexpr int NB = PAIR ? 2 : 1;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi) {
        C* buf = bi == 0 ? A : B;
        C a[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = buf[colpad_ix(k0 + e * half, s, logS, ps)];
        const C t1 = cmul(a[1], x1), t3 = cmul(a[3], x1);
        const C b0 = cadd(a[0], t1), b1 = csub(a[0], t1);
        const C b2 = cadd(a[2], t3), b3 = csub(a[2], t3);
        const C u2 = cmul(b2, x2);
        C u3 = cmul(b3, x2);  // times -i (forward) or +i (inverse)
        {
          const auto re = u3.x;
          if (inverse) { u3.x = -u3.y; u3.y = re; }
          else { u3.x = u3.y; u3.y = -re; }
        }
        buf[colpad_ix(k0, s, logS, ps)] = cadd(b0, u2);
        buf[colpad_ix(k0 + 2 * half, s, logS, ps)] = csub(b0, u2);
        buf[colpad_ix(k0 + half, s, logS, ps)] = cadd(b1, u3);
        buf[colpad_ix(k0 + 3 * half, s, logS, ps)] = csub(b1, u3);
      }
    }
    __syncthreads();
  };
  const int n8 = logM % 3 == 0 ? logM / 3 : (logM % 3 == 1 ? (logM - 4) / 3 : (logM - 2) / 3);
  const int n4 = (logM - 3 * n8) / 2;
#pragma nounroll
  for (int p = 0; p < n8; ++p) pass8(3 * p, p == 0 && gfirst);
#pragma nounroll
  for (int p = 0; p < n4; ++p) pass4(3 * n8 + 2 * p);
}

}  // namespace dpse
