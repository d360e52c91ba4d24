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

}  // namespace dpse
