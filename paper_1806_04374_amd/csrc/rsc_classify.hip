// Texture classifier of Sec. III-B ("Classifier"): patch labels from per-class coding
// errors, per-image label frequencies and the chi^2 nearest neighbour.
//
// The per-class pursuits are the library's encoder, one launch per class dictionary;
// this file holds what follows them:
//   * classify_min_kernel: after class c's pursuit, a patch keeps the smaller of its
//     running error and class c's (strictly smaller replaces, so ties stay with the
//     smaller class index);
//   * label_hist_kernel: one block per group of consecutive patches (an image's
//     windows) counts its labels in LDS with integer atomics (exact, order-free) and
//     writes count / n, rounded once from FP64;
//   * chi2_nearest_kernel: one block per test histogram; each thread takes training
//     histograms in turn, d = sum_i (a_i - b_i)^2 / (a_i + b_i) over the bins with
//     a_i + b_i > 0 in FP64, and the block keeps the smallest (ties: smaller index).
#include <hip/hip_runtime.h>

#include <cfloat>

#include "rsc_internal.h"

namespace rsc {
namespace {

__global__ __launch_bounds__(256) void classify_min_kernel(const float* __restrict__ resid2, int64_t P, int c,
                                                           int32_t* __restrict__ label, float* __restrict__ sse) {
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= P) return;
  const float r = resid2[p];
  if (c == 0 || r < sse[p]) {
    sse[p] = r;
    label[p] = c;
  }
}

__global__ __launch_bounds__(256) void label_hist_kernel(const int32_t* __restrict__ label, int64_t P,
                                                         const int64_t* __restrict__ offset, int C,
                                                         float* __restrict__ hist) {
  extern __shared__ int cnt[];   // [C]
  const int g = blockIdx.x, t = threadIdx.x;
  for (int i = t; i < C; i += 256) cnt[i] = 0;
  __syncthreads();
  // the group's range, clamped into [0, P]
  int64_t a = offset[g], b = offset[g + 1];
  a = a < 0 ? 0 : a > P ? P : a;
  b = b < a ? a : b > P ? P : b;
  for (int64_t p = a + t; p < b; p += 256) {
    const int l = label[p];
    if (l >= 0 && l < C) atomicAdd(&cnt[l], 1);
  }
  __syncthreads();
  const double n = double(b - a);
  for (int i = t; i < C; i += 256) hist[size_t(g) * C + i] = n > 0 ? float(double(cnt[i]) / n) : 0.f;
}

__global__ __launch_bounds__(256) void chi2_nearest_kernel(const float* __restrict__ train, int n_train,
                                                           const float* __restrict__ test, int C,
                                                           int32_t* __restrict__ nearest, float* __restrict__ dist) {
  __shared__ double bd[256];
  __shared__ int bj[256];
  const int q = blockIdx.x, t = threadIdx.x;
  const float* a = test + size_t(q) * C;
  double best = DBL_MAX;
  int bestj = -1;
  for (int j = t; j < n_train; j += 256) {
    const float* b = train + size_t(j) * C;
    double d = 0.0;
    for (int i = 0; i < C; ++i) {
      const double x = a[i], y = b[i], s = x + y;
      if (s > 0.0) {
        const double df = x - y;
        d += df * df / s;
      }
    }
    if (d < best) {   // j increases per thread: strict < keeps the smaller index
      best = d;
      bestj = j;
    }
  }
  bd[t] = best;
  bj[t] = bestj;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      const double d2 = bd[t + s];
      const int j2 = bj[t + s];
      if (j2 >= 0 && (bj[t] < 0 || d2 < bd[t] || (d2 == bd[t] && j2 < bj[t]))) {
        bd[t] = d2;
        bj[t] = j2;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    nearest[q] = bj[0];
    if (dist) dist[q] = float(bd[0]);
  }
}

}  // namespace

int launch_classify_min(const float* resid2, int64_t P, int c, int32_t* label, float* sse, void* stream) {
  hipLaunchKernelGGL(classify_min_kernel, dim3(unsigned((P + 255) / 256)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), resid2, P, c, label, sse);
  return int(hipGetLastError());
}

int launch_label_hist(const int32_t* label, int64_t P, const int64_t* offset, int n_groups, int C, float* hist,
                      void* stream) {
  hipLaunchKernelGGL(label_hist_kernel, dim3(unsigned(n_groups)), dim3(256), sizeof(int) * size_t(C),
                     reinterpret_cast<hipStream_t>(stream), label, P, offset, C, hist);
  return int(hipGetLastError());
}

int launch_chi2_nearest(const float* train, int n_train, const float* test, int n_test, int C, int32_t* nearest,
                        float* dist, void* stream) {
  hipLaunchKernelGGL(chi2_nearest_kernel, dim3(unsigned(n_test)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), train, n_train, test, C, nearest, dist);
  return int(hipGetLastError());
}

}  // namespace rsc
