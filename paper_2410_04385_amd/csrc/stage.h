// Index helpers shared by the staging loops of several kernels.
#pragma once
#include "common.h"

#include <type_traits>

namespace hatt {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// One 16 x 16 x 4 MFMA step in the compute type.  Operand layouts are the
// same for both (lane l holds A(l%16, l/16) and B(l/16, l%16)); the result
// rows held by lane l differ: l/16 + 4v for FP64, 4 (l/16) + v for FP32
// (both checked on gfx950 with one-wave probes).
__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma16(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// The four-block FP64 4 x 4 x 4 MFMA reads the same operand registers as the
// 16 x 16 x 4 one (lane 16k + 4b + i holds A(4b + i, k), lane 16k + 4b + j
// holds B(k, 4b + j)) and forms only the four diagonal 4 x 4 blocks of that
// product: lane 16i + 4b + j receives C(4b + i, 4b + j) (probed on gfx950).
// It issues a quarter of the work in a quarter of the time, but a dependent
// chain of them waits about 52 cycles per step, so chains are interleaved
// with 16 x 16 x 4 MFMAs.
__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}
template <typename CT>
__device__ __forceinline__ int mfma_row(int rq, int v) {
  return std::is_same<CT, double>::value ? rq + 4 * v : 4 * rq + v;
}

// BF16 operands (BF16 range finding): kept as __bf16 in LDS, accumulated in
// FP32.  The 16 x 16 x 16 BF16 MFMA takes four K values per lane; lane l,
// element e is given the operand that the 16 x 16 x 4 layout puts at K step
// 4 e + l / 16.  The instruction sums over all (l / 16, e), and A and B use
// the same assignment, so the product is that of the four K steps (a
// permutation of K).  The result rows held by lane l are the FP32 ones,
// 4 (l / 16) + v.  K must be padded with zeros to a multiple of 16.
typedef short s4_t __attribute__((ext_vector_type(4)));
template <typename CT>
struct is_bf16 : std::is_same<CT, __bf16> {};
template <typename CT>
__device__ __forceinline__ CT to_ct(double x) {
  return (CT)x;
}
template <>
__device__ __forceinline__ __bf16 to_ct<__bf16>(double x) {
  return (__bf16)(float)x;  // round to nearest even (through FP32)
}
__device__ __forceinline__ short bf16_bits(__bf16 x) { return __builtin_bit_cast(short, x); }
// One K-16 step: a[e] = A(l % 16, step 4 e + l / 16), b[e] likewise for B.
__device__ __forceinline__ f4_t mfma16_bf16(const __bf16 (&a)[4], const __bf16 (&b)[4], f4_t c) {
  const s4_t av = {bf16_bits(a[0]), bf16_bits(a[1]), bf16_bits(a[2]), bf16_bits(a[3])};
  const s4_t bv = {bf16_bits(b[0]), bf16_bits(b[1]), bf16_bits(b[2]), bf16_bits(b[3])};
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c, 0, 0, 0);
}


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
template <int U, typename T, typename Src, typename Idx>
__device__ __forceinline__ void stage_lds(int total, Rad3 d, T *dst, Src src, Idx idx) {
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
      if (e0 + 256 * u < total) dst[di[u]] = to_ct<T>(v[u]);
  }
}


__device__ __forceinline__ int fdiv(int x, FastDiv f) { return f.m ? (int)__umulhi((unsigned)x, f.m) : x; }

}  // namespace hatt
