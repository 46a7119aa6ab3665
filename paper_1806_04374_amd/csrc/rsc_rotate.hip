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
#include "rsc_launch.h"

namespace rsc {
namespace {

constexpr int kRotPatches = 32;   // patches per block pass in rotate_taps_kernel

// Thread t owns output pixels t, t + 256, ... (QPT of them) and keeps their taps in
// registers for every patch; each block stages kRotPatches patches in LDS (coalesced),
// applies the taps to them, and writes the rotated patches (coalesced).
template <int NTAP, int QPT>
__global__ __launch_bounds__(256) void rotate_taps_kernel(const float* __restrict__ in, int64_t P, int NN,
                                                         const int32_t* __restrict__ src,
                                                         const float* __restrict__ wgt, float* __restrict__ out) {
  extern __shared__ float xs[];   // [kRotPatches][NN]
  const int t = threadIdx.x;
  float w[QPT][NTAP];
  int sidx[QPT][NTAP];
#pragma unroll
  for (int j = 0; j < QPT; ++j) {
    const int q = t + 256 * j < NN ? t + 256 * j : 0;
#pragma unroll
    for (int k = 0; k < NTAP; ++k) {
      w[j][k] = wgt[q * NTAP + k];
      sidx[j][k] = src[q * NTAP + k];
    }
  }
  for (int64_t p0 = int64_t(blockIdx.x) * kRotPatches; p0 < P; p0 += int64_t(gridDim.x) * kRotPatches) {
    const int np = P - p0 < kRotPatches ? int(P - p0) : kRotPatches;
    __syncthreads();
    for (int i = t; i < np * NN; i += 256) xs[i] = in[p0 * NN + i];
    __syncthreads();
    for (int p = 0; p < np; ++p) {
      const float* x = xs + p * NN;
#pragma unroll
      for (int j = 0; j < QPT; ++j) {
        const int q = t + 256 * j;
        if (q >= NN) continue;
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < NTAP; ++k) acc += w[j][k] * x[sidx[j][k]];
        out[(p0 + p) * NN + q] = acc;
      }
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

// One thread per (patch, profile s, harmonic k >= 1) pair, or per harmonic-0
// coordinate: (a, b) -> (a cos + b sin, b cos - a sin) with angle k theta.  The geometry
// is a template parameter, so the index arithmetic is by constants.
template <int S, int T>
__global__ __launch_bounds__(256) void steer_kernel(SteerParams prm) {
  constexpr int B = S * (2 * T + 1), W = S * (T + 1);   // work items per patch
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= prm.P * W) return;
  const int64_t p = i / W;
  const int w = int(i - p * W);
  const float* x = prm.xhat + p * B;
  float* o = prm.out + p * B;
  if (w < S) {
    o[w] = x[w];
    return;
  }
  const int k = 1 + (w - S) / S, sp = (w - S) - (k - 1) * S;
  const int ire = S + 2 * S * (k - 1) + sp, iim = ire + S;
  const float a = x[ire], bb = x[iim];
  float c, sn;
  if (prm.theta) {
    sincosf(float(k) * prm.theta[p], &sn, &c);
  } else {
    c = prm.cs[k];
    sn = prm.sn[k];
  }
  o[ire] = a * c + bb * sn;
  o[iim] = bb * c - a * sn;
}

// Phi x_hat on the N x N grid: the synthesis matrix [N*N][B] sits in LDS for the
// block's lifetime; a block stages 8 patches' hat rows, one thread per output pixel.
__global__ __launch_bounds__(256) void synth_hat_kernel(const float* __restrict__ xhat, int64_t P, int B, int NN,
                                                       const float* __restrict__ phi, float* __restrict__ out) {
  extern __shared__ float lds[];
  float* ph = lds;              // [NN][B]
  float* xs = ph + NN * B;      // [8][B]
  const int t = threadIdx.x;
  for (int i = t; i < NN * B; i += 256) ph[i] = phi[i];
  for (int64_t p0 = int64_t(blockIdx.x) * 8; p0 < P; p0 += int64_t(gridDim.x) * 8) {
    const int np = P - p0 < 8 ? int(P - p0) : 8;
    __syncthreads();
    for (int i = t; i < np * B; i += 256) xs[i] = xhat[p0 * B + i];
    __syncthreads();
    for (int i = t; i < np * NN; i += 256) {
      const int p = i / NN, q = i - p * NN;
      const float* a = ph + q * B;
      const float* x = xs + p * B;
      float acc0 = 0.f, acc1 = 0.f;
      int b = 0;
      for (; b + 1 < B; b += 2) {
        acc0 += a[b] * x[b];
        acc1 += a[b + 1] * x[b + 1];
      }
      if (b < B) acc0 += a[b] * x[b];
      out[p0 * NN + i] = acc0 + acc1;
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
  (void)ntap;
  return sizeof(float) * size_t(kRotPatches) * N * N;
}

int launch_rotate_taps(int N, int ntap, const float* in, int64_t P, const int32_t* src, const float* w, float* out,
                       void* stream) {
  const int NN = N * N;
  const int64_t want = (P + kRotPatches - 1) / kRotPatches;
  const int64_t cap = int64_t(num_cus()) * 8;
  const unsigned grid = unsigned(want < cap ? want : cap);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int qpt = (NN + 255) / 256;
  const size_t lds = rotate_lds_bytes(N, ntap);
  auto go = [&](auto kern) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(lds));
    if (e != hipSuccess) return int(e);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, st, in, P, NN, src, w, out);
    return int(hipGetLastError());
  };
  if (ntap == 1) return qpt == 1 ? go(rotate_taps_kernel<1, 1>) : qpt == 2 ? go(rotate_taps_kernel<1, 2>)
                                                                          : go(rotate_taps_kernel<1, 3>);
  return qpt == 1 ? go(rotate_taps_kernel<16, 1>) : qpt == 2 ? go(rotate_taps_kernel<16, 2>)
                                                             : go(rotate_taps_kernel<16, 3>);
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
  const int64_t items = P * int64_t(t.S) * (t.T + 1);
  const dim3 grid(unsigned((items + 255) / 256));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (t.S == 5 && t.T == 5) hipLaunchKernelGGL((steer_kernel<5, 5>), grid, dim3(256), 0, st, prm);
  else if (t.S == 7 && t.T == 7) hipLaunchKernelGGL((steer_kernel<7, 7>), grid, dim3(256), 0, st, prm);
  else return int(hipErrorInvalidValue);
  return int(hipGetLastError());
}

int launch_synth_hat(const DeviceTables& t, const float* xhat, int64_t P, float* out, void* stream) {
  const int NN = t.N * t.N;
  const size_t lds = sizeof(float) * (size_t(NN) * t.B + 8 * size_t(t.B));
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(synth_hat_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return int(e);
  const int64_t want = (P + 7) / 8;
  const int64_t cap = int64_t(num_cus()) * 2;
  const unsigned grid = unsigned(want < cap ? want : cap);
  hipLaunchKernelGGL(synth_hat_kernel, dim3(grid), dim3(256), lds, reinterpret_cast<hipStream_t>(stream), xhat, P,
                     t.B, NN, t.phiPad, out);
  return int(hipGetLastError());
}

}  // namespace rsc
