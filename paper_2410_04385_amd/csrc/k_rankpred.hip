// Per-bond width predictor: cheap statistics of the two input cores, and a
// 21-128-128-2 tanh MLP in FP32 (inference, gradient of the mean squared
// error, Adam).  The network is tiny (19586 parameters), so every kernel
// keeps what it reuses in LDS and is launch/latency bound; the statistics
// read each core once, coalesced.
//
// Layouts:
//   theta  W1[128][21] b1[128] W2[128][128] b2[128] W3[2][128] b3[2]
//   stats  mu_x[21] sd_x[21] mu_y[2] sd_y[2]
//   a feature row of bond k (1-based) of a pair of order d:
//     ln r_k(x), ln r_k(y), ln n_k, k/d, ln d,
//     8 quantiles (q = j/7, linear between order statistics) of
//     ln max(c_a, 1e-300), c_a the squared norm of column a of V(x_k),
//     the same 8 for y.
#include <mutex>
#include "common.h"

namespace hatt {

namespace {
constexpr int kIn = kRpIn, kH = kRpH, kOut = kRpOut;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kOut * kH;
static_assert(oB3 + kOut == kRpTheta, "parameter layout");
constexpr int sMx = 0, sSx = kIn, sMy = 2 * kIn, sSy = 2 * kIn + kOut;
constexpr int kRows = kRpRowsPerBlock;  // rows of a gradient block
}  // namespace

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void rp_features_kernel(RpFeatArgs a) {
  __shared__ double vals[kRpMaxRank];
  __shared__ double srt[kRpMaxRank];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int k = a.k0 + b;
  float *row = a.out + (int64_t)b * kIn;
  if (tid == 0) {
    row[0] = (float)log((double)a.rxn[b]);
    row[1] = (float)log((double)a.ryn[b]);
    row[2] = (float)log((double)a.n[b]);
    row[3] = (float)((double)k / (double)a.d);
    row[4] = (float)log((double)a.d);
  }
  for (int side = 0; side < 2; ++side) {
    const double *core = side ? a.cy[b] : a.cx[b];
    const int r = side ? a.ryn[b] : a.rxn[b];
    const int64_t rows = (int64_t)(side ? a.ryp[b] : a.rxp[b]) * a.n[b];
    // squared column norms of V(core): consecutive threads take consecutive columns
    for (int c = tid; c < r; c += 256) {
      double s = 0.0;
      for (int64_t t = 0; t < rows; ++t) {
        const double v = core[t * r + c];
        s += v * v;
      }
      vals[c] = log(fmax(s, 1e-300));
    }
    __syncthreads();
    for (int c = tid; c < r; c += 256) {  // rank sort (ties by index)
      const double v = vals[c];
      int rk = 0;
      for (int j = 0; j < r; ++j) {
        const double u = vals[j];
        rk += (u < v) || (u == v && j < c);
      }
      srt[rk] = v;
    }
    __syncthreads();
    if (tid < 8) {
      const double h = (double)(r - 1) * ((double)tid / 7.0);
      const int lo = (int)floor(h);
      const int hi = min(lo + 1, r - 1);
      row[5 + 8 * side + tid] = (float)(srt[lo] + (h - (double)lo) * (srt[hi] - srt[lo]));
    }
    __syncthreads();
  }
}

hipError_t launch_rp_features(const RpFeatArgs &a, int bonds, hipStream_t s) {
  if (bonds < 1 || bonds > kRpMaxBonds) return hipErrorInvalidValue;
  rp_features_kernel<<<bonds, 256, 0, s>>>(a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inference: one thread per row, the parameters staged in LDS (every lane of
// a wave reads the same weight: a broadcast).
__global__ __launch_bounds__(256) void rp_forward_kernel(const float *theta, const float *stats, const float *feat,
                                                         int64_t rows, float *pred) {
  extern __shared__ float W[];
  for (int e = threadIdx.x; e < kRpTheta; e += 256) W[e] = theta[e];
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= rows) return;
  float xh[kIn];
#pragma unroll
  for (int f = 0; f < kIn; ++f) xh[f] = (feat[row * kIn + f] - stats[sMx + f]) / stats[sSx + f];
  float h1[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    float acc = W[oB1 + j];
#pragma unroll
    for (int f = 0; f < kIn; ++f) acc += W[oW1 + j * kIn + f] * xh[f];
    h1[j] = tanhf(acc);
  }
  float o0 = W[oB3], o1 = W[oB3 + 1];
  for (int j = 0; j < kH; ++j) {
    float acc = W[oB2 + j];
#pragma unroll
    for (int i = 0; i < kH; ++i) acc += W[oW2 + j * kH + i] * h1[i];
    const float h2 = tanhf(acc);
    o0 += W[oW3 + j] * h2;
    o1 += W[oW3 + kH + j] * h2;
  }
  pred[row * 2] = o0 * stats[sSy] + stats[sMy];
  pred[row * 2 + 1] = o1 * stats[sSy + 1] + stats[sMy + 1];
}

hipError_t launch_rp_forward(const float *theta, const float *stats, const float *feat, int64_t rows, float *pred,
                             hipStream_t s) {
  static std::once_flag attr;
  const size_t lds = (size_t)kRpTheta * sizeof(float);
  std::call_once(attr, [&] {
    hipFuncSetAttribute((const void *)rp_forward_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  });
  if (rows < 1) return hipSuccess;
  const int64_t grid = (rows + 255) / 256;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  rp_forward_kernel<<<(unsigned)grid, 256, lds, s>>>(theta, stats, feat, rows, pred);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gradient of L = 1/(2B) sum_b sum_o (o_bo - t_bo)^2 (t: standardised
// targets) over the rows idx[0..B).  Block g takes rows idx[64 g ..) and
// writes the sum of its rows' contributions (already divided by B) to
// part[g][.] in theta's layout and its share of L to loss_part[g].  Rows past
// B enter as zeros with zero error, so they add nothing.
__global__ __launch_bounds__(256) void rp_grad_kernel(const float *theta, const float *stats, const float *feat,
                                                      const float *label, const int32_t *idx, int64_t batch,
                                                      float inv_b, float *part, float *loss_part) {
  extern __shared__ float sm[];
  float *xh = sm;                 // [64][21]
  float *tg = xh + kRows * kIn;   // [64][2]
  float *h1 = tg + kRows * kOut;  // [64][128]
  float *h2 = h1 + kRows * kH;    // [64][128]; later d1
  float *d2 = h2 + kRows * kH;    // [64][128]
  float *d3 = d2 + kRows * kH;    // [64][2]
  __shared__ float red[256];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  const int nv = (int)min<int64_t>(kRows, batch - r0);
  for (int e = tid; e < kRows * kIn; e += 256) {
    const int b = e / kIn, f = e - b * kIn;
    float v = 0.f;
    if (b < nv) {
      const int64_t rr = idx[r0 + b];
      v = (feat[rr * kIn + f] - stats[sMx + f]) / stats[sSx + f];
    }
    xh[e] = v;
  }
  if (tid < kRows * kOut) {
    const int b = tid >> 1, c = tid & 1;
    float v = 0.f;
    if (b < nv) {
      const int64_t rr = idx[r0 + b];
      v = (label[rr * kOut + c] - stats[sMy + c]) / stats[sSy + c];
    }
    tg[tid] = v;
  }
  __syncthreads();
  const int j = tid & (kH - 1), half = tid >> 7;  // unit j, rows 32 half .. 32 half + 31
  {
    float w[kIn];
#pragma unroll
    for (int f = 0; f < kIn; ++f) w[f] = theta[oW1 + j * kIn + f];
    const float bj = theta[oB1 + j];
    for (int bb = 0; bb < kRows / 2; ++bb) {
      const int b = half * (kRows / 2) + bb;
      float acc = bj;
#pragma unroll
      for (int f = 0; f < kIn; ++f) acc += w[f] * xh[b * kIn + f];
      h1[b * kH + j] = tanhf(acc);
    }
  }
  __syncthreads();
  {
    float w[kH];
#pragma unroll
    for (int i = 0; i < kH; ++i) w[i] = theta[oW2 + j * kH + i];
    const float bj = theta[oB2 + j];
    for (int bb = 0; bb < kRows / 2; ++bb) {
      const int b = half * (kRows / 2) + bb;
      float acc = bj;
#pragma unroll
      for (int i = 0; i < kH; ++i) acc += w[i] * h1[b * kH + i];
      h2[b * kH + j] = tanhf(acc);
    }
  }
  __syncthreads();
  float lsum = 0.f;
  if (tid < kRows * kOut) {
    const int b = tid >> 1, c = tid & 1;
    float o = theta[oB3 + c];
    for (int jj = 0; jj < kH; ++jj) o += theta[oW3 + c * kH + jj] * h2[b * kH + jj];
    const float df = (b < nv) ? (o - tg[tid]) : 0.f;
    d3[tid] = df * inv_b;
    lsum = 0.5f * df * df;
  }
  red[tid] = lsum;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) loss_part[blockIdx.x] = red[0] * inv_b;
  for (int e = tid; e < kRows * kH; e += 256) {
    const int b = e >> 7, jj = e & (kH - 1);
    const float g = d3[b * 2] * theta[oW3 + jj] + d3[b * 2 + 1] * theta[oW3 + kH + jj];
    const float hv = h2[e];
    d2[e] = g * (1.f - hv * hv);
  }
  __syncthreads();
  float *pb = part + (int64_t)blockIdx.x * kRpTheta;
  {
    const int c = tid >> 7, jj = tid & (kH - 1);
    float s = 0.f;
    for (int b = 0; b < kRows; ++b) s += d3[b * 2 + c] * h2[b * kH + jj];
    pb[oW3 + c * kH + jj] = s;
  }
  if (tid < kOut) {
    float s = 0.f;
    for (int b = 0; b < kRows; ++b) s += d3[b * 2 + tid];
    pb[oB3 + tid] = s;
  }
  {
    // dW2[j][i] = sum_b d2[b][j] h1[b][i], an 8 x 8 block per thread
    const int jb = (tid >> 4) * 8, ib = (tid & 15) * 8;
    float acc[8][8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int t = 0; t < 8; ++t) acc[q][t] = 0.f;
    for (int b = 0; b < kRows; ++b) {
      float dv[8], hv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        dv[q] = d2[b * kH + jb + q];
        hv[q] = h1[b * kH + ib + q];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[q][t] += dv[q] * hv[t];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int t = 0; t < 8; ++t) pb[oW2 + (jb + q) * kH + ib + t] = acc[q][t];
  }
  if (tid < kH) {
    float s = 0.f;
    for (int b = 0; b < kRows; ++b) s += d2[b * kH + tid];
    pb[oB2 + tid] = s;
  }
  __syncthreads();  // h2 is overwritten by d1 below
  {
    // d1[b][i] = (sum_j W2[j][i] d2[b][j]) (1 - h1[b][i]^2), thread i = j
    float w[kH];
#pragma unroll
    for (int jj = 0; jj < kH; ++jj) w[jj] = theta[oW2 + jj * kH + j];
    for (int bb = 0; bb < kRows / 2; ++bb) {
      const int b = half * (kRows / 2) + bb;
      float g = 0.f;
#pragma unroll
      for (int jj = 0; jj < kH; ++jj) g += w[jj] * d2[b * kH + jj];
      const float hv = h1[b * kH + j];
      h2[b * kH + j] = g * (1.f - hv * hv);
    }
  }
  __syncthreads();
  for (int e = tid; e < kH * kIn; e += 256) {
    const int jj = e / kIn, f = e - jj * kIn;
    float s = 0.f;
    for (int b = 0; b < kRows; ++b) s += h2[b * kH + jj] * xh[b * kIn + f];
    pb[oW1 + e] = s;
  }
  if (tid < kH) {
    float s = 0.f;
    for (int b = 0; b < kRows; ++b) s += h2[b * kH + tid];
    pb[oB1 + tid] = s;
  }
}

size_t rp_grad_lds_bytes() { return (size_t)(kRows * kIn + 2 * kRows * kOut + 3 * kRows * kH) * sizeof(float); }

// Sum of the blocks' partial gradients in block order (deterministic), then
// optionally one Adam step on theta (c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)).
__global__ __launch_bounds__(256) void rp_reduce_kernel(const float *part, int nblk, const float *loss_part,
                                                        float *grad, float *loss, RpAdam ad) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < kRpTheta) {
    float g = 0.f;
    for (int w = 0; w < nblk; ++w) g += part[(int64_t)w * kRpTheta + p];
    if (grad != nullptr) grad[p] = g;
    if (ad.theta != nullptr) {
      const float mm = ad.b1 * ad.m[p] + (1.f - ad.b1) * g;
      const float vv = ad.b2 * ad.v[p] + (1.f - ad.b2) * g * g;
      ad.m[p] = mm;
      ad.v[p] = vv;
      ad.theta[p] -= ad.lr * (mm * ad.c1) / (sqrtf(vv * ad.c2) + ad.eps);
    }
  }
  if (p == 0 && loss != nullptr) {
    float s = 0.f;
    for (int w = 0; w < nblk; ++w) s += loss_part[w];
    *loss = s;
  }
}

hipError_t launch_rp_grad(const float *theta, const float *stats, const float *feat, const float *label,
                          const int32_t *idx, int64_t batch, float *part, float *loss_part, float *grad,
                          float *loss, const RpAdam &ad, hipStream_t s) {
  static std::once_flag attr;
  const size_t lds = rp_grad_lds_bytes();
  std::call_once(attr, [&] {
    hipFuncSetAttribute((const void *)rp_grad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  });
  const int64_t nblk = (batch + kRows - 1) / kRows;
  if (batch < 1 || nblk > 0x7fffffff) return hipErrorInvalidValue;
  rp_grad_kernel<<<(unsigned)nblk, 256, lds, s>>>(theta, stats, feat, label, idx, batch, 1.0f / (float)batch, part,
                                                  loss_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  rp_reduce_kernel<<<(kRpTheta + 255) / 256, 256, 0, s>>>(part, (int)nblk, loss_part, grad, loss, ad);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Means and population standard deviations of the 21 feature and 2 target
// columns (FP64 sums; a deviation below 1e-8 becomes 1).
__global__ __launch_bounds__(256) void rp_stats_kernel(const float *feat, const float *label, int64_t rows,
                                                       float *stats) {
  __shared__ double red[256];
  const int col = blockIdx.x, tid = threadIdx.x;
  const float *src = (col < kIn) ? feat : label;
  const int ld = (col < kIn) ? kIn : kOut, c = (col < kIn) ? col : col - kIn;
  double s = 0.0;
  for (int64_t r = tid; r < rows; r += 256) s += (double)src[r * ld + c];
  red[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  const double mean = red[0] / (double)rows;
  __syncthreads();
  double s2 = 0.0;
  for (int64_t r = tid; r < rows; r += 256) {
    const double dv = (double)src[r * ld + c] - mean;
    s2 += dv * dv;
  }
  red[tid] = s2;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    double sd = sqrt(red[0] / (double)rows);
    if (sd < 1e-8) sd = 1.0;
    if (col < kIn) {
      stats[sMx + c] = (float)mean;
      stats[sSx + c] = (float)sd;
    } else {
      stats[sMy + c] = (float)mean;
      stats[sSy + c] = (float)sd;
    }
  }
}

hipError_t launch_rp_stats(const float *feat, const float *label, int64_t rows, float *stats, hipStream_t s) {
  if (rows < 1) return hipErrorInvalidValue;
  rp_stats_kernel<<<kIn + kOut, 256, 0, s>>>(feat, label, rows, stats);
  return hipGetLastError();
}

}  // namespace hatt
