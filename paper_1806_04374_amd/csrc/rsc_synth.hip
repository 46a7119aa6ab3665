// Pixels of coded or synthetic patches: x_p = Phi sum_j w_j S(theta_j) d_{m_j} (+ noise),
// the map back to pixels of Sec. II-E step 4 with the steering of eq. (6)/(8).
// Not on the timed path: one block per 8 patches builds the hat vectors in LDS,
// then every pixel is a dot product with a row of Phi.
#include <hip/hip_runtime.h>

#include "rsc_internal.h"

namespace rsc {
namespace {

struct SynthParams {
  const int32_t* atom;
  const int32_t* angle_idx;   // grid angles (reconstruction), or null
  const float* theta;         // continuous angles (synthesis), or null
  const float* weight;
  const float* noise;
  float* out;
  int64_t P;
  int J, M, R, S, T, B, NN;
  const float* dictHat;       // [.][B]
  const float* cs;            // [2][T+1][R]
  const float* phiPad;        // [NN][B]
  const int* steerTab;        // annular basis: (k << 16) | (partner offset + 32768) per
                              // coordinate; null for the (S, T) grid
};

constexpr int kSynthPB = 8;

__global__ __launch_bounds__(128) void synth_kernel(SynthParams p) {
  extern __shared__ float hat[];  // [kSynthPB][B]
  const int B = p.B, S = p.S;
  const int64_t p0 = int64_t(blockIdx.x) * kSynthPB;
  for (int e = threadIdx.x; e < kSynthPB * B; e += blockDim.x) {
    const int pl = e / B, c = e % B;
    const int64_t pp = p0 + pl;
    float acc = 0.f;
    if (pp < p.P) {
      for (int j = 0; j < p.J; ++j) {
        const int m = p.atom[pp * p.J + j];
        if (m < 0 || m >= p.M) continue;
        int r = 0;
        if (p.angle_idx) {
          r = p.angle_idx[pp * p.J + j];
          if (r < 0 || r >= p.R) continue;
        }
        const float w = p.weight[pp * p.J + j];
        const float* d = p.dictHat + int64_t(m) * B;
        float v;
        if (p.steerTab) {
          // ragged layout: harmonic k and the offset of the Re/Im partner from the table
          const int e2 = p.steerTab[c], k = e2 >> 16, off = (e2 & 0xffff) - 32768;
          if (k == 0) {
            v = d[c];
          } else {
            float co, sn;
            if (p.angle_idx) {
              co = p.cs[k * p.R + r];
              sn = p.cs[(p.T + 1 + k) * p.R + r];
            } else {
              sincosf(float(k) * p.theta[pp * p.J + j], &sn, &co);
            }
            const float own = d[c], partner = d[c + off];
            v = off > 0 ? (own * co + partner * sn) : (own * co - partner * sn);
          }
        } else if (c < S) {
          v = d[c];
        } else {
          const int q = c - S, k = 1 + q / (2 * S), rem = q % (2 * S), s = rem % S;
          const bool im_part = rem >= S;
          const int base = S + 2 * S * (k - 1);
          float co, sn;
          if (p.angle_idx) {
            co = p.cs[k * p.R + r];
            sn = p.cs[(p.T + 1 + k) * p.R + r];
          } else {
            sincosf(float(k) * p.theta[pp * p.J + j], &sn, &co);
          }
          const float re = d[base + s], im = d[base + S + s];
          v = im_part ? (im * co - re * sn) : (re * co + im * sn);
        }
        acc += w * v;
      }
    }
    hat[pl * B + c] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kSynthPB * p.NN; e += blockDim.x) {
    const int pl = e / p.NN, q = e % p.NN;
    const int64_t pp = p0 + pl;
    if (pp >= p.P) continue;
    float acc = 0.f;
    const float* ph = p.phiPad + int64_t(q) * B;
    for (int b = 0; b < B; ++b) acc += ph[b] * hat[pl * B + b];
    if (p.noise) acc += p.noise[pp * p.NN + q];
    p.out[pp * p.NN + q] = acc;
  }
}

}  // namespace

int launch_synthesize(const DeviceTables& t, const int32_t* atom, const int32_t* angle_idx,
                      const float* theta, const float* weight, int64_t P, int J, const float* noise,
                      float* out, void* stream) {
  if (P <= 0) return 0;
  SynthParams p{atom, angle_idx, theta, weight, noise, out, P, J, t.M, t.R, t.S, t.T, t.B,
                t.N * t.N, t.dictHat, t.cs, t.phiPad, t.geo == kGeoGrid ? nullptr : t.steerTab};
  const int64_t blocks = (P + kSynthPB - 1) / kSynthPB;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(synth_kernel, dim3(unsigned(blocks)), dim3(128), sizeof(float) * kSynthPB * t.B,
                     st, p);
  return int(hipGetLastError());
}

}  // namespace rsc
