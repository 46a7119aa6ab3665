// gfx950 kernels of the rotational sparse coding path.
//
//  * project_kernel   -- hat coordinates x_hat = (Phi^T Phi)^{-1} Phi^T x (Sec. II-E
//                        step 2) as an FP32 MFMA GEMM, patches staged through LDS.
//  * encode_kernel    -- rotational OMP (Fig. 2 with R_r -> S_r, Sec. II-C/II-E) for
//                        32 patches per wave, all K steps in one launch:
//      (b) correlation with every rotation of every atom.  Steering is diagonal per
//          harmonic (eq. (8)), so <S_r d_m, x> = C_0 + sum_k Re(exp(i k 2 pi r/R) C_k)
//          with C_k = sum_s conj(d_{m,s,k}) x_{s,k}.  Stage 1 forms the C_k on MFMA
//          (rows = 16 atoms x {Re, Im}, columns = 32 patches), a half-wave swap turns
//          its output into the operand of stage 2, which evaluates the R-point angle
//          DFT on MFMA (rows = 32 angles), and the |score| argmax runs on the
//          accumulators in registers.
//      (c) incremental Cholesky least squares on the selected columns and the residual
//          update, per patch, in registers (both half-waves of a patch hold the same
//          small factor; each holds half of the residual).
//  * synth_kernel     -- Phi sum_j w_j S(theta_j) d_{m_j} (+ noise): reconstruction
//                        of codes (Sec. II-E step 4) and synthetic inputs.
//
// MFMA v_mfma_f32_32x32x2f32 operand layout (one block): lane l supplies
// A[l % 32][l / 32] and B[l / 32][l % 32]; accumulator register v of lane l holds
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
#include <hip/hip_runtime.h>

#include "rsc_internal.h"

namespace rsc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr float kTau2 = 1e-10f;  // early stop when ||r||^2 <= kTau2 ||x||^2

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.f;
  return z;
}

// Exchange lanes 32..63 of x with lanes 0..31 of y:
// afterwards x = [x_lo | y_lo] and y = [x_hi | y_hi].
__device__ __forceinline__ void swap_halves(float& x, float& y) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}

// Sum of a value over the two half-waves holding one patch (identical in both).
__device__ __forceinline__ float pair_sum(float x) { return x + __shfl_xor(x, 32); }

// ------------------------------------------------------------------ projection
// One block = 2 waves = 64 patches.  Rows of the MFMA are hat coordinates (RTB tiles
// of 32), columns are patches, the contraction runs over the N*N grid pixels (pinv
// has zero columns outside the disk).
template <int RTB>
__global__ __launch_bounds__(128) void project_kernel(const float* __restrict__ patches, int64_t P,
                                                      int NN, int B,
                                                      const float* __restrict__ pinvA,
                                                      float* __restrict__ xhat) {
  extern __shared__ float tile[];  // [64][NN] patches, reused as [64][B] output
  constexpr int PT = 64;
  const int KP = (NN + 1) / 2;
  const int64_t p0 = int64_t(blockIdx.x) * PT;
  const int np = int(P - p0 < PT ? P - p0 : PT);
  const float* src = patches + p0 * NN;
  const int total = np * NN;
  for (int i = threadIdx.x; i < PT * NN; i += blockDim.x) tile[i] = i < total ? src[i] : 0.f;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, hh = lane >> 5;
  const float* mine = tile + (wave * 32 + col) * NN;
  f32x16 acc[RTB];
#pragma unroll
  for (int t = 0; t < RTB; ++t) acc[t] = zero16();
  const float* A = pinvA + lane;
#pragma unroll 4
  for (int j = 0; j < KP; ++j) {
    const int px = 2 * j + hh;
    const float b = px < NN ? mine[px] : 0.f;
#pragma unroll
    for (int t = 0; t < RTB; ++t) acc[t] = mfma32(A[(t * KP + j) * 64], b, acc[t]);
  }
  __syncthreads();
  float* out = tile;
#pragma unroll
  for (int t = 0; t < RTB; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int c = 32 * t + 8 * (v / 4) + 4 * hh + (v % 4);
      if (c < B) out[(wave * 32 + col) * B + c] = acc[t][v];
    }
  __syncthreads();
  float* dst = xhat + p0 * B;
  for (int i = threadIdx.x; i < np * B; i += blockDim.x) dst[i] = out[i];
}

// ------------------------------------------------------------------ encoder
struct EncodeParams {
  const float* xhat;
  int64_t P;
  int K, M, R, NG;
  const float* dictA;
  const float* dictHat;
  const float* dftA;
  const float* cs;
  int32_t* atom;
  int32_t* angle;
  float* coef;
  float* resid2;
};

template <int S, int T>
struct Geo {
  static constexpr int B = S * (2 * T + 1);
  static constexpr int K0 = k0_steps(S);
  static constexpr int NKS = stage1_steps(S, T);
  static constexpr int NQ = T + 1;
  // Packed hat index held by half-wave hh at stage-1 step ks (-1: padding).
  __device__ static constexpr int coord(int ks, int hh) {
    if (ks < K0) return (2 * ks + hh < S) ? 2 * ks + hh : -1;
    const int q = ks - K0, k = 1 + q / S, s = q % S;
    return S + 2 * S * (k - 1) + hh * S + s;
  }
};

// Steered atom S_r d_m restricted to the coordinates this half-wave holds.
template <int S, int T>
__device__ __forceinline__ void steer_atom(const float* __restrict__ hat, const float* __restrict__ cs,
                                           int R, int m, int r, int hh,
                                           float (&out)[Geo<S, T>::NKS]) {
  using G = Geo<S, T>;
  const float* d = hat + m * G::B;
#pragma unroll
  for (int ks = 0; ks < G::K0; ++ks) {
    const int s = 2 * ks + hh;
    const float v = d[s < S ? s : 0];
    out[ks] = s < S ? v : 0.f;
  }
#pragma unroll
  for (int k = 1; k <= T; ++k) {
    const float c = cs[k * R + r];
    const float sn = cs[(G::NQ + k) * R + r];
    // Re part: re c + im sn ; Im part: im c - re sn  (multiplication by exp(-i k theta))
    const float ca = hh ? -sn : c;
    const float cb = hh ? c : sn;
    const int base = S + 2 * S * (k - 1);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float re = d[base + s], im = d[base + S + s];
      out[G::K0 + (k - 1) * S + s] = re * ca + im * cb;
    }
  }
}

template <int S, int T, int RT, int KMAX>
__global__ __launch_bounds__(256, 2) void encode_kernel(EncodeParams prm) {
  using G = Geo<S, T>;
  constexpr int B = G::B, K0 = G::K0, NKS = G::NKS, NQ = G::NQ;
  extern __shared__ float lds[];
  const int NG = prm.NG, R = prm.R, M = prm.M, K = prm.K;
  float* sA = lds;                       // [NG][NKS][64]
  float* sHat = sA + NG * NKS * 64;      // [NG*16][B]
  float* sCs = sHat + NG * 16 * B;       // [2][NQ][R]
  {
    const int nA = NG * NKS * 64, nH = NG * 16 * B, nC = 2 * NQ * R;
    for (int i = threadIdx.x; i < nA; i += blockDim.x) sA[i] = prm.dictA[i];
    for (int i = threadIdx.x; i < nH; i += blockDim.x) sHat[i] = prm.dictHat[i];
    for (int i = threadIdx.x; i < nC; i += blockDim.x) sCs[i] = prm.cs[i];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, hh = lane >> 5;
  float F[RT][NQ];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int q = 0; q < NQ; ++q) F[t][q] = prm.dftA[(t * NQ + q) * 64 + lane];

  const int64_t nwt = (prm.P + 31) / 32;
  for (int64_t wt = int64_t(blockIdx.x) * 4 + wave; wt < nwt; wt += int64_t(gridDim.x) * 4) {
    const int64_t p = wt * 32 + col;
    const bool valid = p < prm.P;
    float xh[NKS], res[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int c = G::coord(ks, hh);
      xh[ks] = (valid && c >= 0) ? prm.xhat[p * B + c] : 0.f;
      res[ks] = xh[ks];
    }
    float nx2 = 0.f;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) nx2 += xh[ks] * xh[ks];
    nx2 = pair_sum(nx2);

    int selm[KMAX], selr[KMAX];
    float L[KMAX][KMAX], bv[KMAX], cf[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      selm[i] = -1;
      selr[i] = -1;
      bv[i] = 0.f;
      cf[i] = 0.f;
#pragma unroll
      for (int j = 0; j < KMAX; ++j) L[i][j] = 0.f;
    }
    bool active = valid;
    int nsel = 0;

#pragma unroll
    for (int it = 0; it < KMAX; ++it) {
      if (it >= K) break;
      {
        float rn2 = 0.f;
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) rn2 += res[ks] * res[ks];
        rn2 = pair_sum(rn2);
        active = active && (rn2 > kTau2 * nx2);
      }
      if (!__any(active)) break;

      // ---------------- (b) correlation with all (atom, angle) and argmax
      float best = -1.f;
      int bcode = 0;
      for (int g = 0; g < NG; ++g) {
        const float* Ag = sA + g * NKS * 64 + lane;
        f32x16 acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = zero16();
#pragma unroll
        for (int j = 0; j < K0; ++j) acc[0] = mfma32(Ag[j * 64], res[j], acc[0]);
#pragma unroll
        for (int k = 1; k <= T; ++k)
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const int j = K0 + (k - 1) * S + s;
            acc[k] = mfma32(Ag[j * 64], res[j], acc[k]);
          }
        // rows 0..15 hold Re C (atoms 0..15), rows 16..31 Im C; after the swap register
        // v (< 8) holds [Re | Im] of atom 8(v/4)+v%4 and register v+8 of that atom + 4.
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            float x = acc[q][v], y = acc[q][v + 8];
            swap_halves(x, y);
            acc[q][v] = x;
            acc[q][v + 8] = y;
          }
#pragma unroll
        for (int a = 0; a < 16; ++a) {
          const int m = g * 16 + a;
          if (m >= M) break;
          const int v = 4 * (a / 8) + (a % 4) + 8 * ((a / 4) % 2);
          const int mcode = m << 7;
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            f32x16 o = zero16();
#pragma unroll
            for (int q = 0; q < NQ; ++q) o = mfma32(F[t][q], acc[q][v], o);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              const float val = fabsf(o[i]);
              const int rc = 32 * t + 8 * (i / 4) + (i % 4);
              const bool gt = val > best;
              best = gt ? val : best;
              bcode = gt ? (mcode | rc) : bcode;
            }
          }
        }
      }
      bcode += 4 * hh;
      {
        const float ob = __shfl_xor(best, 32);
        const int oc = __shfl_xor(bcode, 32);
        const bool take = (ob > best) || (ob == best && oc < bcode);
        best = take ? ob : best;
        bcode = take ? oc : bcode;
      }
      int ms = bcode >> 7, rs = bcode & 127;
      ms = ms < M ? ms : M - 1;
      rs = rs < R ? rs : R - 1;
      bool dup = false;
#pragma unroll
      for (int i = 0; i < it; ++i) dup = dup || (selm[i] == ms && selr[i] == rs);
      bool upd = active && !dup;

      // ---------------- (c) Cholesky update, least squares, residual
      float dn[NKS];
      steer_atom<S, T>(sHat, sCs, R, ms, rs, hh, dn);
      float gcol[KMAX];
#pragma unroll
      for (int i = 0; i < it; ++i) {
        float di[NKS];
        steer_atom<S, T>(sHat, sCs, R, selm[i] < 0 ? 0 : selm[i], selr[i] < 0 ? 0 : selr[i], hh, di);
        float acc = 0.f;
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) acc += di[ks] * dn[ks];
        gcol[i] = pair_sum(acc);
      }
      float dd = 0.f, bx = 0.f;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        dd += dn[ks] * dn[ks];
        bx += dn[ks] * xh[ks];
      }
      dd = pair_sum(dd);
      bx = pair_sum(bx);
      float w[KMAX];
      float l2 = dd;
#pragma unroll
      for (int i = 0; i < it; ++i) {
        float s = gcol[i];
#pragma unroll
        for (int j = 0; j < i; ++j) s -= L[i][j] * w[j];
        w[i] = s / L[i][i];
        l2 -= w[i] * w[i];
      }
      upd = upd && (l2 > 1e-6f * dd);
#pragma unroll
      for (int i = 0; i < it; ++i) L[it][i] = upd ? w[i] : L[it][i];
      L[it][it] = upd ? sqrtf(l2) : L[it][it];
      bv[it] = upd ? bx : bv[it];
      selm[it] = upd ? ms : selm[it];
      selr[it] = upd ? rs : selr[it];
      float y[KMAX], an[KMAX];
#pragma unroll
      for (int i = 0; i <= it; ++i) {
        float s = bv[i];
#pragma unroll
        for (int j = 0; j < i; ++j) s -= L[i][j] * y[j];
        y[i] = s / L[i][i];
      }
#pragma unroll
      for (int i = it; i >= 0; --i) {
        float s = y[i];
#pragma unroll
        for (int j = i + 1; j <= it; ++j) s -= L[j][i] * an[j];
        an[i] = s / L[i][i];
      }
#pragma unroll
      for (int i = 0; i <= it; ++i) cf[i] = upd ? an[i] : cf[i];
      nsel = upd ? it + 1 : nsel;
      active = upd;
      if (__any(upd)) {
        float nr[NKS];
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) nr[ks] = xh[ks] - cf[it] * dn[ks];
#pragma unroll
        for (int i = 0; i < it; ++i) {
          float di[NKS];
          steer_atom<S, T>(sHat, sCs, R, selm[i] < 0 ? 0 : selm[i], selr[i] < 0 ? 0 : selr[i], hh, di);
#pragma unroll
          for (int ks = 0; ks < NKS; ++ks) nr[ks] -= cf[i] * di[ks];
        }
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) res[ks] = upd ? nr[ks] : res[ks];
      }
    }

    float rn2 = 0.f;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) rn2 += res[ks] * res[ks];
    rn2 = pair_sum(rn2);
    if (valid && hh == 0) {
#pragma unroll
      for (int i = 0; i < KMAX; ++i) {
        if (i < K) {
          const bool s = i < nsel;
          prm.atom[p * K + i] = s ? selm[i] : -1;
          prm.angle[p * K + i] = s ? selr[i] : -1;
          prm.coef[p * K + i] = s ? cf[i] : 0.f;
        }
      }
      if (prm.resid2) prm.resid2[p] = rn2;
    }
  }
}

// ------------------------------------------------------------------ synthesis
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
        if (c < S) {
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

int num_cus() {
  static int cached = -1;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (cached < 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cached = n;
  }
  return cached;
}

template <int S, int T, int RT, int KMAX>
int launch_encode_t(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  const size_t lds = encode_lds_bytes(t);
  auto kern = encode_kernel<S, T, RT, KMAX>;
  static bool attr_set = false;
  if (!attr_set && lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return int(e);
    attr_set = true;
  }
  const int64_t nwt = (prm.P + 31) / 32;
  int64_t blocks = (nwt + 3) / 4;
  const int64_t cap = int64_t(num_cus()) * 2;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(256), lds, st, prm);
  return int(hipGetLastError());
}

template <int S, int T, int RT>
int dispatch_k(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  if (prm.K <= 2) return launch_encode_t<S, T, RT, 2>(t, prm, st);
  if (prm.K <= 4) return launch_encode_t<S, T, RT, 4>(t, prm, st);
  return launch_encode_t<S, T, RT, 8>(t, prm, st);
}

template <int S, int T>
int dispatch_rt(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  if (t.RT == 1) return dispatch_k<S, T, 1>(t, prm, st);
  if (t.RT == 2) return dispatch_k<S, T, 2>(t, prm, st);
  return dispatch_k<S, T, 4>(t, prm, st);
}

}  // namespace

bool encode_supported(int S, int T) { return (S == 5 && T == 5) || (S == 7 && T == 7); }

size_t encode_lds_bytes(const DeviceTables& t) {
  const int nks = stage1_steps(t.S, t.T);
  return sizeof(float) * (size_t(t.NG) * nks * 64 + size_t(t.NG) * 16 * t.B + 2 * size_t(t.T + 1) * t.R);
}

int launch_project(const DeviceTables& t, const float* patches, int64_t P, float* xhat, void* stream) {
  if (P <= 0) return 0;
  const int NN = t.N * t.N;
  const int64_t blocks = (P + 63) / 64;
  size_t lds = sizeof(float) * 64 * size_t(NN > t.B ? NN : t.B);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int rtb = (t.B + 31) / 32;
  if (rtb <= 2)
    hipLaunchKernelGGL(project_kernel<2>, dim3(unsigned(blocks)), dim3(128), lds, st, patches, P, NN,
                       t.B, t.pinvA, xhat);
  else if (rtb <= 4)
    hipLaunchKernelGGL(project_kernel<4>, dim3(unsigned(blocks)), dim3(128), lds, st, patches, P, NN,
                       t.B, t.pinvA, xhat);
  else
    return int(hipErrorInvalidValue);
  return int(hipGetLastError());
}

int launch_encode(const DeviceTables& t, const float* xhat, int64_t P, int K, int32_t* atom,
                  int32_t* angle, float* coef, float* resid2, void* stream) {
  if (P <= 0) return 0;
  EncodeParams prm{xhat, P, K, t.M, t.R, t.NG, t.dictA, t.dictHat, t.dftA, t.cs, atom, angle, coef, resid2};
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (t.S == 5 && t.T == 5) return dispatch_rt<5, 5>(t, prm, st);
  if (t.S == 7 && t.T == 7) return dispatch_rt<7, 7>(t, prm, st);
  return int(hipErrorInvalidValue);
}

int launch_synthesize(const DeviceTables& t, const int32_t* atom, const int32_t* angle_idx,
                      const float* theta, const float* weight, int64_t P, int J, const float* noise,
                      float* out, void* stream) {
  if (P <= 0) return 0;
  SynthParams p{atom, angle_idx, theta, weight, noise, out, P, J, t.M, t.R, t.S, t.T, t.B,
                t.N * t.N, t.dictHat, t.cs, t.phiPad};
  const int64_t blocks = (P + kSynthPB - 1) / kSynthPB;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(synth_kernel, dim3(unsigned(blocks)), dim3(128), sizeof(float) * kSynthPB * t.B,
                     st, p);
  return int(hipGetLastError());
}

}  // namespace rsc
