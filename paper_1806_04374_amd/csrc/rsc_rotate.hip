// Patch rotation (Sec. IV, rotation speed): by interpolation, and by steering.
//
// Interpolation: a plan holds the rotation as a table of taps, the rows of the paper's
// N^2 x N^2 matrix R_nearest or R_bicubic (at most 1 or 16 nonzeros per output pixel),
// built once on the host in FP64; rotate_taps_kernel applies it to a batch of patches.
//   Output pixel (x, y) (x = col - c, y = c - row, c = (N-1)/2) reads the input at
//   R_{-theta}(x, y): nearest-neighbour (coordinates rounded half up) or bicubic (Keys'
//   cubic convolution, a = -1/2, over the 4 x 4 neighbours); input pixels outside the
//   patch count as 0.
// Steering: steer_kernel multiplies harmonic k of hat coordinates by exp(-i k theta)
// (the diagonal S of eq. (8), at any angle); synth_hat_kernel maps hat coordinates back
// to pixels, Phi x_hat (zero off the disk).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "rsc_internal.h"

namespace rsc {
namespace {

constexpr int kRotPatches = 16;   // patches per block pass in rotate_taps_kernel

// Each block stages kRotPatches patches in LDS (coalesced), applies the taps (in LDS),
// and writes the rotated patches (coalesced).
template <int NTAP>
__global__ __launch_bounds__(256) void rotate_taps_kernel(const float* __restrict__ in, int64_t P, int NN,
                                                         const int32_t* __restrict__ src,
                                                         const float* __restrict__ wgt, float* __restrict__ out) {
  extern __shared__ float lds[];
  float* xs = lds;                                            // [kRotPatches][NN]
  float* ws = xs + kRotPatches * NN;                          // [NN][NTAP]
  int* ss = reinterpret_cast<int*>(ws + NN * NTAP);           // [NN][NTAP]
  const int t = threadIdx.x;
  for (int i = t; i < NN * NTAP; i += 256) {
    ws[i] = wgt[i];
    ss[i] = src[i];
  }
  for (int64_t p0 = int64_t(blockIdx.x) * kRotPatches; p0 < P; p0 += int64_t(gridDim.x) * kRotPatches) {
    const int np = P - p0 < kRotPatches ? int(P - p0) : kRotPatches;
    __syncthreads();
    for (int i = t; i < np * NN; i += 256) xs[i] = in[p0 * NN + i];
    __syncthreads();
    for (int i = t; i < np * NN; i += 256) {
      const int p = i / NN, q = i - p * NN;
      const float* x = xs + p * NN;
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < NTAP; ++k) acc += ws[q * NTAP + k] * x[ss[q * NTAP + k]];
      out[p0 * NN + i] = acc;
    }
  }
}

struct SteerParams {
  const float* xhat;
  float* out;
  int64_t P;
  int B, S;
  const float* theta;   // per patch, or null
  float cs[16], sn[16]; // cos, sin of k theta0 for k = 0..T (T <= 15), when theta is null
};

// One thread per coordinate: harmonic k of the packed pair (a, b) -> (a cos + b sin,
// b cos - a sin) with angle k theta (harmonic 0 unchanged).
__global__ __launch_bounds__(256) void steer_kernel(SteerParams prm) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= prm.P * prm.B) return;
  const int64_t p = i / prm.B;
  const int b = int(i - p * prm.B), S = prm.S;
  const float own = prm.xhat[i];
  if (b < S) {
    prm.out[i] = own;
    return;
  }
  const int q = b - S, k = 1 + q / (2 * S), rem = q - (k - 1) * 2 * S;
  const bool re = rem < S;
  const float other = prm.xhat[i + (re ? S : -S)];
  float c, s;
  if (prm.theta) {
    sincosf(float(k) * prm.theta[p], &s, &c);
  } else {
    c = prm.cs[k];
    s = prm.sn[k];
  }
  prm.out[i] = re ? own * c + other * s : own * c - other * s;
}

// Phi x_hat on the N x N grid: a block stages 8 patches' hat rows in LDS, the synthesis
// matrix [N*N][B] is read through the caches; one thread per output pixel.
__global__ __launch_bounds__(256) void synth_hat_kernel(const float* __restrict__ xhat, int64_t P, int B, int NN,
                                                       const float* __restrict__ phi, float* __restrict__ out) {
  __shared__ float xs[8 * 128];
  const int t = threadIdx.x;
  for (int64_t p0 = int64_t(blockIdx.x) * 8; p0 < P; p0 += int64_t(gridDim.x) * 8) {
    const int np = P - p0 < 8 ? int(P - p0) : 8;
    __syncthreads();
    for (int i = t; i < np * B; i += 256) xs[i] = xhat[p0 * B + i];
    __syncthreads();
    for (int i = t; i < np * NN; i += 256) {
      const int p = i / NN, q = i - p * NN;
      const float* ph = phi + size_t(q) * B;
      const float* x = xs + p * B;
      float acc = 0.f;
      for (int b = 0; b < B; ++b) acc += ph[b] * x[b];
      out[p0 * NN + i] = acc;
    }
  }
}

double keys(double t) {
  const double a = -0.5;
  t = std::fabs(t);
  if (t <= 1.0) return (a + 2.0) * t * t * t - (a + 3.0) * t * t + 1.0;
  if (t < 2.0) return a * t * t * t - 5.0 * a * t * t + 8.0 * a * t - 4.0 * a;
  return 0.0;
}

}  // namespace

int rotation_taps(int N, double theta, int mode, std::vector<int32_t>& src, std::vector<float>& w) {
  const int NN = N * N, ntap = mode == 0 ? 1 : 16;
  src.assign(size_t(NN) * ntap, 0);
  w.assign(size_t(NN) * ntap, 0.f);
  const double c = (N - 1) / 2.0, cs = std::cos(theta), sn = std::sin(theta);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const double x = j - c, y = c - i;
      const double xs = cs * x + sn * y, ys = -sn * x + cs * y;   // R_{-theta} (x, y)
      const double col = c + xs, row = c - ys;
      const int q = i * N + j;
      if (mode == 0) {
        const int r0 = int(std::floor(row + 0.5)), c0 = int(std::floor(col + 0.5));
        if (r0 >= 0 && r0 < N && c0 >= 0 && c0 < N) {
          src[q] = r0 * N + c0;
          w[q] = 1.f;
        }
      } else {
        const int r0 = int(std::floor(row)), c0 = int(std::floor(col));
        int k = 0;
        for (int di = -1; di <= 2; ++di)
          for (int dj = -1; dj <= 2; ++dj, ++k) {
            const int rr = r0 + di, cc = c0 + dj;
            if (rr < 0 || rr >= N || cc < 0 || cc >= N) continue;
            src[size_t(q) * 16 + k] = rr * N + cc;
            w[size_t(q) * 16 + k] = float(keys(row - rr) * keys(col - cc));
          }
      }
    }
  return ntap;
}

size_t rotate_lds_bytes(int N, int ntap) {
  return sizeof(float) * size_t(kRotPatches) * N * N + (sizeof(float) + sizeof(int32_t)) * size_t(N) * N * ntap;
}

int launch_rotate_taps(int N, int ntap, const float* in, int64_t P, const int32_t* src, const float* w, float* out,
                       void* stream) {
  const int NN = N * N;
  const size_t lds = rotate_lds_bytes(N, ntap);
  const int64_t want = (P + kRotPatches - 1) / kRotPatches;
  const unsigned grid = unsigned(want < 4096 ? want : 4096);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (ntap == 1) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(rotate_taps_kernel<1>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return int(e);
    hipLaunchKernelGGL(rotate_taps_kernel<1>, dim3(grid), dim3(256), lds, st, in, P, NN, src, w, out);
  } else {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(rotate_taps_kernel<16>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return int(e);
    hipLaunchKernelGGL(rotate_taps_kernel<16>, dim3(grid), dim3(256), lds, st, in, P, NN, src, w, out);
  }
  return int(hipGetLastError());
}

int launch_steer(const DeviceTables& t, const float* xhat, int64_t P, const float* theta, double theta0, float* out,
                 void* stream) {
  SteerParams prm{};
  prm.xhat = xhat;
  prm.out = out;
  prm.P = P;
  prm.B = t.B;
  prm.S = t.S;
  prm.theta = theta;
  for (int k = 0; k <= t.T && k < 16; ++k) {
    prm.cs[k] = float(std::cos(k * theta0));
    prm.sn[k] = float(std::sin(k * theta0));
  }
  hipLaunchKernelGGL(steer_kernel, dim3(unsigned((P * t.B + 255) / 256)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), prm);
  return int(hipGetLastError());
}

int launch_synth_hat(const DeviceTables& t, const float* xhat, int64_t P, float* out, void* stream) {
  const int64_t want = (P + 7) / 8;
  const unsigned grid = unsigned(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(synth_hat_kernel, dim3(grid), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), xhat, P,
                     t.B, t.N * t.N, t.phiPad, out);
  return int(hipGetLastError());
}

}  // namespace rsc
