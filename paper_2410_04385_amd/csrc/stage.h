// Index helpers shared by the staging loops of several kernels.
#pragma once
#include "common.h"

namespace hatt {

// Three-digit counter (i0 fastest, radices n0, n1) stepped by a fixed stride
// with carries instead of a division per element.
struct Rad3 {
  int i0, i1, i2, n0, n1, s0, s1, s2;
  __device__ Rad3(int start, int stride, int n0_, int n1_) : n0(n0_), n1(n1_) {
    i0 = start % n0;
    i1 = (start / n0) % n1;
    i2 = start / (n0 * n1);
    s0 = stride % n0;
    s1 = (stride / n0) % n1;
    s2 = stride / (n0 * n1);
  }
  __device__ __forceinline__ void next() {
    i0 += s0;
    i1 += s1;
    i2 += s2;
    if (i0 >= n0) { i0 -= n0; ++i1; }
    if (i1 >= n1) { i1 -= n1; ++i2; }
  }
};

// Global -> LDS staging with U loads in flight per thread: element e of the
// block (digits in d, advanced by the block stride) is read by src(d) and
// stored at dst[idx(d)].
template <int U, typename Src, typename Idx>
__device__ __forceinline__ void stage_lds(int total, Rad3 d, double *dst, Src src, Idx idx) {
  for (int e0 = threadIdx.x; e0 < total; e0 += 256 * U) {
    double v[U];
    int di[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (e0 + 256 * u < total) {
        v[u] = src(d);
        di[u] = idx(d);
      }
      d.next();
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + 256 * u < total) dst[di[u]] = v[u];
  }
}


__device__ __forceinline__ int fdiv(int x, FastDiv f) { return f.m ? (int)__umulhi((unsigned)x, f.m) : x; }

}  // namespace hatt
