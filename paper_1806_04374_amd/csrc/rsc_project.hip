// Projection onto the steerable basis (Sec. II-E step 2):
//   xhat_p = (Phi^T Phi)^{-1} Phi^T x_p,
// an FP32 MFMA GEMM with rows = hat coordinates, columns = patches and the
// contraction over disk pixels.
//
//  * project_reg_kernel (11x11 with B <= 96, 15x15 with B in 97..160; 16-byte aligned
//    patches): the operand in registers, one 32-row tile per wave, 32-patch chunks staged
//    in LDS with the next one prefetched into registers, the partial last chunk in the
//    same launch.
//  * project_tiled_kernel (11x11 patches that are not 16-byte aligned): one block of 8
//    waves per CU loops over
//    tiles of 8 x 32 patches.  Each wave copies its 32 contiguous patches to its
//    own LDS tile with 16-byte loads, the (Phi^T Phi)^{-1} Phi^T operand stays in
//    LDS for the whole launch, and the results leave through the same tile as
//    contiguous 16-byte stores; the waves need no block-wide barrier.
//  * project_reg_lp_kernel / project_tiled_lp_kernel (aligned / unaligned 11x11 input of
//    16-bit handles): the layouts above (6 waves per block for the tiled one) with 16-bit MFMA
//    operands (v_mfma_f32_32x32x16_{bf16,f16}, contraction over 16 disk pixels per
//    step) in compensated form: the patch values and the operand are split into
//    16-bit parts and the products down to FP32 order are accumulated in FP32 --
//    FP16: x = hi + lo, hi*hi + hi*lo + lo*hi; BF16: x = hi + mid + lo,
//    hi*hi + hi*mid + mid*hi + hi*lo + lo*hi + mid*mid.  This keeps the coordinates
//    at FP32 accuracy; a single 16-bit product would be amplified by the basis'
//    conditioning.  FP16 has a narrow exponent range, so each patch is first scaled
//    by a power of two that puts its largest value in [2^10, 2^11) (the operand is
//    pre-scaled the same way on the host), keeping the remainders normal; the
//    scales are exact and removed per column after the accumulation.
//  * project_kernel (any size): blocks of 64 patches, operand read from global.
#include <hip/hip_runtime.h>

#include "rsc_device.h"
#include "rsc_internal.h"
#include "rsc_launch.h"
#include "rsc_lp.h"

namespace rsc {
namespace {

constexpr int kProjWaves = 8;

// Orders a wave's LDS accesses to its own tile (waits for its LDS operations; no
// block-wide barrier, so the waves of a block run their load / compute / store
// phases independently).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// pinvD: [2][KPD][64] operand over disk pixels (contraction index 2j + u is disk
// pixel 2j+u in row-major order); pix: [2*KPD] grid index of each disk pixel or -1.
template <int NN, int KPD>
__global__ __launch_bounds__(512) void project_tiled_kernel(const float* __restrict__ patches, int64_t P,
                                                            int B, const float* __restrict__ pinvD,
                                                            const int* __restrict__ pix, bool vec_in,
                                                            bool vec_out, float* __restrict__ xhat) {
  extern __shared__ float lds[];
  float* sA = lds;                                    // [2][KPD][64]
  constexpr int kPixPad = (2 * KPD + 3) & ~3;        // keeps the tiles 16-byte aligned
  int* sPix = reinterpret_cast<int*>(sA + 2 * KPD * 64);  // [2*KPD]
  float* tiles = sA + 2 * KPD * 64 + kPixPad;         // [waves][32*NN]
  for (int i = threadIdx.x; i < 2 * KPD * 64; i += blockDim.x) sA[i] = pinvD[i];
  for (int i = threadIdx.x; i < 2 * KPD; i += blockDim.x) sPix[i] = pix[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, u = lane >> 5;
  float* tile = tiles + wave * 32 * NN;
  const int64_t ntile = (P + 31) / 32;
  for (int64_t bt = blockIdx.x; bt * kProjWaves < ntile; bt += gridDim.x) {
    asm volatile("" ::: "memory");   // keep the LDS operand reads inside the loop
    const int64_t wt = bt * kProjWaves + wave;
    const int64_t p0 = wt * 32;
    const int np = wt < ntile ? int(P - p0 < 32 ? P - p0 : 32) : 0;
    const float* src = patches + p0 * NN;
    if (np == 32 && vec_in) {
      const float4* s4 = reinterpret_cast<const float4*>(src);
      float4* d4 = reinterpret_cast<float4*>(tile);
#pragma unroll 4
      for (int i = lane; i < 8 * NN; i += 64) d4[i] = s4[i];
    } else {
      for (int i = lane; i < 32 * NN; i += 64) tile[i] = i < np * NN ? src[i] : 0.f;
    }
    wave_lds_fence();
    f32x16 acc0, acc1;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc0[i] = acc1[i] = 0.f;
    const float* mine = tile + col * NN;
#pragma unroll 7
    for (int j = 0; j < KPD; ++j) {
      const int q = sPix[2 * j + u];
      const float b = q >= 0 ? mine[q] : 0.f;
      acc0 = mfma32(sA[j * 64 + lane], b, acc0);
      acc1 = mfma32(sA[(KPD + j) * 64 + lane], b, acc1);
    }
    wave_lds_fence();
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int c0 = 8 * (v / 4) + 4 * u + (v % 4);
      tile[col * B + c0] = acc0[v];
      if (32 + c0 < B) tile[col * B + 32 + c0] = acc1[v];
    }
    wave_lds_fence();
    float* dst = xhat + p0 * B;
    if (np == 32 && vec_out) {
      const float4* s4 = reinterpret_cast<const float4*>(tile);
      float4* d4 = reinterpret_cast<float4*>(dst);
      for (int i = lane; i < 8 * B; i += 64) d4[i] = s4[i];
    } else {
      for (int i = lane; i < np * B; i += 64) dst[i] = tile[i];
    }
    wave_lds_fence();
  }
}

constexpr int kProjWavesLp = 6;

// pinvP: NP parts of the operand, each [2][KS][64] x 8 16-bit (NP = 3 for BF16: hi,
// mid, lo; NP = 2 for FP16: hi, lo); lane l gives row 32t + l%32 and disk pixels
// 16j + 8(l/32) + i.  pix16: [16 KS] grid index of disk pixel i, -1 past n_pix.
template <int NN, int KS, int PREC>
__global__ __launch_bounds__(64 * kProjWavesLp) void project_tiled_lp_kernel(
    const float* __restrict__ patches, int64_t P, int B, const uint4* __restrict__ pinvP,
    const int* __restrict__ pix16, float a_unscale, bool vec_in, bool vec_out, float* __restrict__ xhat) {
  using Pr = Lp<PREC>;
  using V8 = typename Pr::V8;
  constexpr int NP = PREC == RSC_BF16 ? 3 : 2;
  extern __shared__ uint4 lds4[];
  uint4* sA = lds4;                                         // [NP][2][KS][64]
  int* sPix = reinterpret_cast<int*>(sA + NP * 2 * KS * 64);  // [16 KS]
  float* tiles = reinterpret_cast<float*>(sPix + 16 * KS);    // [waves][32*NN]
  for (int i = threadIdx.x; i < NP * 2 * KS * 64; i += blockDim.x) sA[i] = pinvP[i];
  for (int i = threadIdx.x; i < 16 * KS; i += blockDim.x) sPix[i] = pix16[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, u = lane >> 5;
  float* tile = tiles + wave * 32 * NN;
  const int64_t ntile = (P + 31) / 32;
  auto A = [&](int part, int t, int j) { return __builtin_bit_cast(V8, sA[((part * 2 + t) * KS + j) * 64 + lane]); };
  for (int64_t bt = blockIdx.x; bt * kProjWavesLp < ntile; bt += gridDim.x) {
    asm volatile("" ::: "memory");
    const int64_t wt = bt * kProjWavesLp + wave;
    const int64_t p0 = wt * 32;
    const int np = wt < ntile ? int(P - p0 < 32 ? P - p0 : 32) : 0;
    const float* src = patches + p0 * NN;
    if (np == 32 && vec_in) {
      const float4* s4 = reinterpret_cast<const float4*>(src);
      float4* d4 = reinterpret_cast<float4*>(tile);
#pragma unroll 4
      for (int i = lane; i < 8 * NN; i += 64) d4[i] = s4[i];
    } else {
      for (int i = lane; i < 32 * NN; i += 64) tile[i] = i < np * NN ? src[i] : 0.f;
    }
    wave_lds_fence();
    f32x16 acc[2];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[0][i] = acc[1][i] = 0.f;
    const float* mine = tile + col * NN;
    float xs[KS][8];
#pragma unroll
    for (int j = 0; j < KS; ++j)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int q = sPix[16 * j + 8 * u + i];
        xs[j][i] = q >= 0 ? mine[q >= 0 ? q : 0] : 0.f;
      }
    float unscale = a_unscale;
    if (NP == 2) {
      // power-of-two scale of this patch (both half-waves of the column agree)
      float m = 0.f;
#pragma unroll
      for (int j = 0; j < KS; ++j)
#pragma unroll
        for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(xs[j][i]));
      m = max_halves(m);
      int ex = 0;
      (void)frexpf(m, &ex);                 // m in [2^(ex-1), 2^ex)
      const int e = m > 0.f ? 11 - ex : 0;  // largest value in [2^10, 2^11)
      const float sc = ldexpf(1.f, e);
      unscale = ldexpf(a_unscale, -e);
#pragma unroll
      for (int j = 0; j < KS; ++j)
#pragma unroll
        for (int i = 0; i < 8; ++i) xs[j][i] *= sc;
    }
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      if (NP == 3) {
        V8 xh, xm, xl;
        split8x3<Pr>(xs[j], xh, xm, xl);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          acc[t] = Pr::mfma(A(0, t, j), xh, acc[t]);
          acc[t] = Pr::mfma(A(0, t, j), xm, acc[t]);
          acc[t] = Pr::mfma(A(1, t, j), xh, acc[t]);
          acc[t] = Pr::mfma(A(0, t, j), xl, acc[t]);
          acc[t] = Pr::mfma(A(2, t, j), xh, acc[t]);
          acc[t] = Pr::mfma(A(1, t, j), xm, acc[t]);
        }
      } else {
        V8 xh, xl;
        split8<Pr>(xs[j], xh, xl);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          acc[t] = Pr::mfma(A(0, t, j), xh, acc[t]);
          acc[t] = Pr::mfma(A(0, t, j), xl, acc[t]);
          acc[t] = Pr::mfma(A(1, t, j), xh, acc[t]);
        }
      }
    }
    if (unscale != 1.f) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc[0][v] *= unscale;
        acc[1][v] *= unscale;
      }
    }
    wave_lds_fence();
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int c0 = 8 * (v / 4) + 4 * u + (v % 4);
      tile[col * B + c0] = acc[0][v];
      if (32 + c0 < B) tile[col * B + 32 + c0] = acc[1][v];
    }
    wave_lds_fence();
    float* dst = xhat + p0 * B;
    if (np == 32 && vec_out) {
      const float4* s4 = reinterpret_cast<const float4*>(tile);
      float4* d4 = reinterpret_cast<float4*>(dst);
      for (int i = lane; i < 8 * B; i += 64) d4[i] = s4[i];
    } else {
      for (int i = lane; i < np * B; i += 64) dst[i] = tile[i];
    }
    wave_lds_fence();
  }
}

// Patch arrays (N*N = NNC, B <= 32 NT): block of NT waves, wave w computes hat
// coordinates 32w..32w+31 and keeps its operand rows (KPD contraction steps over disk
// pixels) in registers.  The block takes 32 patches at a time: the chunk is staged in LDS,
// the next one is loaded into registers while the current one is contracted, and the
// results leave through an LDS staging tile with coalesced 16-byte stores.
constexpr int kProjRegPatches = 32;

template <int NNC, int KPD, int NT>
__global__ __launch_bounds__(64 * NT) void project_reg_kernel(const float* __restrict__ patches, int64_t nfull,
                                                             int tail, int B, const float* __restrict__ pinvI,
                                                             const int* __restrict__ pix, bool vec_out,
                                                             float* __restrict__ xhat) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  constexpr int NTH = 64 * NT, NV = kProjRegPatches * NNC / 4, VPT = (NV + NTH - 1) / NTH;
  __shared__ v4f tile4[VPT * NTH];               // [32][NNC] used; the rest takes clamped copies
  __shared__ int sPix[2 * KPD];
  __shared__ float stage[kProjRegPatches * 32 * NT];   // [32 patches][B] used
  const float* tile = reinterpret_cast<const float*>(tile4);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, col = lane & 31, u = lane >> 5;
  float a[KPD];
#pragma unroll
  for (int j = 0; j < KPD; ++j) a[j] = pinvI[(w * KPD + j) * 64 + lane];
  // contraction slots past the disk have zero operand rows: point them at disk pixel 0
  // (any finite pixel gives the same sum), so the gathers need no condition
  for (int i = t; i < 2 * KPD; i += NTH) sPix[i] = pix[i] >= 0 ? pix[i] : pix[0];
  int vi[VPT];
#pragma unroll
  for (int v = 0; v < VPT; ++v) vi[v] = t + NTH * v < NV ? t + NTH * v : NV - 1;
  // chunks 0..nfull-1 hold 32 patches, chunk nfull (if tail > 0) the last tail patches; the
  // launch has at most nfull + (tail > 0) blocks, so every block starts on a chunk.  Whole
  // chunks go through the 16-byte register prefetch, the partial one is staged directly.
  const int64_t nchunk = nfull + (tail > 0 ? 1 : 0);
  v4f nxt[VPT];
  int64_t c = blockIdx.x;
  if (nfull > 0) {
    const int64_t c0 = c < nfull ? c : nfull - 1;
    const v4f* s4 = reinterpret_cast<const v4f*>(patches + c0 * kProjRegPatches * NNC);
#pragma unroll
    for (int v = 0; v < VPT; ++v) nxt[v] = s4[vi[v]];
  }
  const float* mine = tile + col * NNC;
  for (; c < nchunk; c += gridDim.x) {
    __syncthreads();   // the previous chunk's reads of the tile and the staging tile are done
    if (c < nfull) {
#pragma unroll
      for (int v = 0; v < VPT; ++v) tile4[t + NTH * v] = nxt[v];
    } else {
      const float* src = patches + c * kProjRegPatches * NNC;
      float* tw = reinterpret_cast<float*>(tile4);
      for (int i = t; i < kProjRegPatches * NNC; i += NTH) tw[i] = i < tail * NNC ? src[i] : 0.f;
    }
    __syncthreads();
    if (nfull > 0) {
      // the next whole chunk (otherwise the block's last whole one again, unused)
      const int64_t nx = c + gridDim.x, cn = nx < nfull ? nx : (c < nfull ? c : nfull - 1);
      const v4f* s4 = reinterpret_cast<const v4f*>(patches + cn * kProjRegPatches * NNC);
#pragma unroll
      for (int v = 0; v < VPT; ++v) nxt[v] = s4[vi[v]];
    }
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll
    for (int j = 0; j < KPD; ++j) {
      acc = mfma32(a[j], mine[sPix[2 * j + u]], acc);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 32 * w + 8 * (v / 4) + 4 * u + (v % 4);
      if (r < B) stage[col * B + r] = acc[v];
    }
    __syncthreads();
    const int nout = (c < nfull ? kProjRegPatches : tail) * B;
    float* dst = xhat + c * kProjRegPatches * B;
    if (vec_out && c < nfull) {
      const v4f* s4 = reinterpret_cast<const v4f*>(stage);
      for (int i = t; i < nout / 4; i += NTH) reinterpret_cast<v4f*>(dst)[i] = s4[i];
    } else {
      for (int i = t; i < nout; i += NTH) dst[i] = stage[i];
    }
  }
}

// The compensated 16-bit projection (as project_tiled_lp_kernel) with the structure of
// project_reg_kernel: a block of two waves (one 32-row operand tile each, its NP 16-bit
// parts in registers) takes 32 patches at a time from LDS, the next chunk is prefetched
// into registers, the partial last chunk is staged element-wise, and the results leave
// through an LDS staging tile.  Both waves gather and split the same patch values.
template <int NNC, int KS, int PREC>
__global__ __launch_bounds__(128) void project_reg_lp_kernel(const float* __restrict__ patches, int64_t nfull,
                                                            int tail, int B, const uint4* __restrict__ pinvP,
                                                            const int* __restrict__ pix16, float a_unscale,
                                                            bool vec_out, float* __restrict__ xhat) {
  using Pr = Lp<PREC>;
  using V8 = typename Pr::V8;
  typedef float v4f __attribute__((ext_vector_type(4)));
  constexpr int NP = PREC == RSC_BF16 ? 3 : 2;
  constexpr int NTH = 128, NV = kProjRegPatches * NNC / 4, VPT = (NV + NTH - 1) / NTH;
  __shared__ v4f tile4[VPT * NTH];                   // [32][NNC] used; the rest takes clamped copies
  __shared__ int sPix[16 * KS];
  __shared__ float stage[kProjRegPatches * 64];      // [32 patches][B], B <= 64
  const float* tile = reinterpret_cast<const float*>(tile4);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, col = lane & 31, u = lane >> 5;
  uint4 a[NP][KS];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int j = 0; j < KS; ++j) a[p][j] = pinvP[((p * 2 + w) * KS + j) * 64 + lane];
  // slots past the disk have zero operand parts: point them at disk pixel 0, a pixel the
  // patch's scale already covers, so the gathers need no condition
  for (int i = t; i < 16 * KS; i += NTH) sPix[i] = pix16[i] >= 0 ? pix16[i] : pix16[0];
  int vi[VPT];
#pragma unroll
  for (int v = 0; v < VPT; ++v) vi[v] = t + NTH * v < NV ? t + NTH * v : NV - 1;
  const int64_t nchunk = nfull + (tail > 0 ? 1 : 0);
  v4f nxt[VPT];
  int64_t c = blockIdx.x;
  if (nfull > 0) {
    const int64_t c0 = c < nfull ? c : nfull - 1;
    const v4f* s4 = reinterpret_cast<const v4f*>(patches + c0 * kProjRegPatches * NNC);
#pragma unroll
    for (int v = 0; v < VPT; ++v) nxt[v] = s4[vi[v]];
  }
  const float* mine = tile + col * NNC;
  for (; c < nchunk; c += gridDim.x) {
    __syncthreads();   // the previous chunk's reads of the tile and the staging tile are done
    if (c < nfull) {
#pragma unroll
      for (int v = 0; v < VPT; ++v) tile4[t + NTH * v] = nxt[v];
    } else {
      const float* src = patches + c * kProjRegPatches * NNC;
      float* tw = reinterpret_cast<float*>(tile4);
      for (int i = t; i < kProjRegPatches * NNC; i += NTH) tw[i] = i < tail * NNC ? src[i] : 0.f;
    }
    __syncthreads();
    if (nfull > 0) {
      const int64_t nx = c + gridDim.x, cn = nx < nfull ? nx : (c < nfull ? c : nfull - 1);
      const v4f* s4 = reinterpret_cast<const v4f*>(patches + cn * kProjRegPatches * NNC);
#pragma unroll
      for (int v = 0; v < VPT; ++v) nxt[v] = s4[vi[v]];
    }
    float xs[KS][8];
#pragma unroll
    for (int j = 0; j < KS; ++j)
#pragma unroll
      for (int i = 0; i < 8; ++i) xs[j][i] = mine[sPix[16 * j + 8 * u + i]];
    float unscale = a_unscale;
    if (NP == 2) {
      // power-of-two scale of this patch (both half-waves of the column agree)
      float m = 0.f;
#pragma unroll
      for (int j = 0; j < KS; ++j)
#pragma unroll
        for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(xs[j][i]));
      m = max_halves(m);
      int ex = 0;
      (void)frexpf(m, &ex);                 // m in [2^(ex-1), 2^ex)
      const int e = m > 0.f ? 11 - ex : 0;  // largest value in [2^10, 2^11)
      const float sc = ldexpf(1.f, e);
      unscale = ldexpf(a_unscale, -e);
#pragma unroll
      for (int j = 0; j < KS; ++j)
#pragma unroll
        for (int i = 0; i < 8; ++i) xs[j][i] *= sc;
    }
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      if (NP == 3) {
        V8 xh, xm, xl;
        split8x3<Pr>(xs[j], xh, xm, xl);
        const V8 a0 = __builtin_bit_cast(V8, a[0][j]), a1 = __builtin_bit_cast(V8, a[1][j]),
                 a2 = __builtin_bit_cast(V8, a[NP - 1][j]);
        acc = Pr::mfma(a0, xh, acc);
        acc = Pr::mfma(a0, xm, acc);
        acc = Pr::mfma(a1, xh, acc);
        acc = Pr::mfma(a0, xl, acc);
        acc = Pr::mfma(a2, xh, acc);
        acc = Pr::mfma(a1, xm, acc);
      } else {
        V8 xh, xl;
        split8<Pr>(xs[j], xh, xl);
        const V8 a0 = __builtin_bit_cast(V8, a[0][j]), a1 = __builtin_bit_cast(V8, a[1][j]);
        acc = Pr::mfma(a0, xh, acc);
        acc = Pr::mfma(a0, xl, acc);
        acc = Pr::mfma(a1, xh, acc);
      }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 32 * w + 8 * (v / 4) + 4 * u + (v % 4);
      if (r < B) stage[col * B + r] = acc[v] * unscale;
    }
    __syncthreads();
    const int nout = (c < nfull ? kProjRegPatches : tail) * B;
    float* dst = xhat + c * kProjRegPatches * B;
    if (vec_out && c < nfull) {
      const v4f* s4 = reinterpret_cast<const v4f*>(stage);
      for (int i = t; i < nout / 4; i += NTH) reinterpret_cast<v4f*>(dst)[i] = s4[i];
    } else {
      for (int i = t; i < nout; i += NTH) dst[i] = stage[i];
    }
  }
}

// Generic fallback: one block = 2 waves = 64 patches, operand from global memory.
template <int RTB>
__global__ __launch_bounds__(128) void project_kernel(const float* __restrict__ patches, int64_t P, int NN,
                                                      int B, const float* __restrict__ pinvA,
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
  const int col = lane & 31, u = lane >> 5;
  const float* mine = tile + (wave * 32 + col) * NN;
  f32x16 acc[RTB];
#pragma unroll
  for (int t = 0; t < RTB; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;
  const float* A = pinvA + lane;
  for (int j = 0; j < KP; ++j) {
    const int px = 2 * j + u;
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
      const int c = 32 * t + 8 * (v / 4) + 4 * u + (v % 4);
      if (c < B) out[(wave * 32 + col) * B + c] = acc[t][v];
    }
  __syncthreads();
  float* dst = xhat + p0 * B;
  for (int i = threadIdx.x; i < np * B; i += blockDim.x) dst[i] = out[i];
}

int cus() { return num_cus(); }

}  // namespace

size_t project_tiled_lds_bytes(int N, int n_pix) {
  const int kpd = (n_pix + 1) / 2;
  return sizeof(float) * (2 * size_t(kpd) * 64 + size_t((2 * kpd + 3) & ~3) + size_t(kProjWaves) * 32 * N * N);
}

size_t project_lp_lds_bytes(int N, int n_pix, int prec) {
  const int ks = (n_pix + 15) / 16, np = prec == RSC_BF16 ? 3 : 2;
  return size_t(np) * 2 * ks * 64 * 16 + sizeof(int) * 16 * size_t(ks) +
         sizeof(float) * size_t(kProjWavesLp) * 32 * N * N;
}

int launch_project(const DeviceTables& t, const float* patches, int64_t P, float* xhat, void* stream) {
  if (P <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int NN = t.N * t.N;
  if (t.prec != RSC_FP32 && t.N == 11 && t.S == 5 && t.T == 5 && t.lpPinv &&
      (reinterpret_cast<uintptr_t>(patches) & 15) == 0) {
    // 16-byte aligned patches: the register-operand form, whole chunks and the partial last one
    constexpr int kNN = 121, kKS = 7;
    if ((t.n_pix + 15) / 16 != kKS) return int(hipErrorInvalidValue);
    auto kern = t.prec == RSC_BF16 ? project_reg_lp_kernel<kNN, kKS, RSC_BF16>
                                   : project_reg_lp_kernel<kNN, kKS, RSC_FP16>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 128, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    const int64_t nfull = P / kProjRegPatches, tail = P - nfull * kProjRegPatches;
    const int64_t work = nfull + (tail > 0), cap = int64_t(cus()) * per_cu;
    const bool vout = (reinterpret_cast<uintptr_t>(xhat) & 15) == 0 && (kProjRegPatches * t.B) % 4 == 0;
    hipLaunchKernelGGL(kern, dim3(unsigned(work < cap ? work : cap)), dim3(128), 0, st, patches, nfull, int(tail),
                       t.B, reinterpret_cast<const uint4*>(t.lpPinv), t.lpPix16, t.lpPinvUnscale, vout, xhat);
    return int(hipGetLastError());
  }
  if (t.prec != RSC_FP32 && t.N == 11 && t.S == 5 && t.T == 5 && t.lpPinv) {
    constexpr int kNN = 121, kKS = 7;
    if ((t.n_pix + 15) / 16 != kKS) return int(hipErrorInvalidValue);
    const size_t lds = project_lp_lds_bytes(t.N, t.n_pix, t.prec);
    auto kern = t.prec == RSC_BF16 ? project_tiled_lp_kernel<kNN, kKS, RSC_BF16>
                                   : project_tiled_lp_kernel<kNN, kKS, RSC_FP16>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return int(e);
    const int64_t ntile = (P + 31) / 32;
    int64_t blocks = (ntile + kProjWavesLp - 1) / kProjWavesLp;
    if (blocks > cus()) blocks = cus();
    const bool vin = (reinterpret_cast<uintptr_t>(patches) & 15) == 0;
    const bool vout = (reinterpret_cast<uintptr_t>(xhat) & 15) == 0 && (t.B * 32) % 4 == 0;
    hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(64 * kProjWavesLp), lds, st, patches, P, t.B,
                       reinterpret_cast<const uint4*>(t.lpPinv), t.lpPix16, t.lpPinvUnscale, vin, vout, xhat);
    return int(hipGetLastError());
  }
  // register-operand kernel (16-byte aligned patches): 11x11 with B <= 64 or 96 (2 or 3 row
  // tiles) and 15x15 with B in 97..128 or 129..160 (4 or 5 row tiles); whole 32-patch chunks
  // and the partial last one
  const bool aligned = (reinterpret_cast<uintptr_t>(patches) & 15) == 0;
  const bool vout = (reinterpret_cast<uintptr_t>(xhat) & 15) == 0 && (kProjRegPatches * t.B) % 4 == 0;
  auto go_reg = [&](auto kern, int nt) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * nt, 0) != hipSuccess || per_cu < 1)
      per_cu = 1;
    const int64_t nfull = P / kProjRegPatches, tail = P - nfull * kProjRegPatches;
    const int64_t work = nfull + (tail > 0), cap = int64_t(cus()) * per_cu;
    hipLaunchKernelGGL(kern, dim3(unsigned(work < cap ? work : cap)), dim3(64 * nt), 0, st, patches, nfull,
                       int(tail), t.B, t.pinvI, t.pixD, vout, xhat);
    return int(hipGetLastError());
  };
  if (aligned && t.N == 11 && t.n_pix == 97 && t.B <= 64 && t.pinvI && t.pixD)
    return go_reg(project_reg_kernel<121, 49, 2>, 2);
  if (aligned && t.N == 11 && t.n_pix == 97 && t.B > 64 && t.B <= 96 && t.pinvI && t.pixD)   // annular, B = 81
    return go_reg(project_reg_kernel<121, 49, 3>, 3);
  if (aligned && t.N == 15 && t.n_pix == 177 && t.B > 96 && t.B <= 128 && t.pinvI && t.pixD)
    return go_reg(project_reg_kernel<225, 89, 4>, 4);
  if (aligned && t.N == 15 && t.n_pix == 177 && t.B > 128 && t.B <= 160 && t.pinvI && t.pixD)  // annular, B = 153
    return go_reg(project_reg_kernel<225, 89, 5>, 5);
  // unaligned 11x11 input (S = T = 5): the LDS-operand tiled kernel
  if (t.N == 11 && t.S == 5 && t.T == 5 && t.pinvD) {
    constexpr int kNN = 121, kKPD = 49;
    if ((t.n_pix + 1) / 2 != kKPD) return int(hipErrorInvalidValue);
    const size_t lds = project_tiled_lds_bytes(t.N, t.n_pix);
    auto kern = project_tiled_kernel<kNN, kKPD>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return int(e);
    const int64_t ntile = (P + 31) / 32;
    int64_t blocks = (ntile + kProjWaves - 1) / kProjWaves;
    if (blocks > cus()) blocks = cus();
    hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(64 * kProjWaves), lds, st, patches, P, t.B,
                       t.pinvD, t.pixD, aligned, vout, xhat);
    return int(hipGetLastError());
  }
  const int64_t blocks = (P + 63) / 64;
  const size_t lds = sizeof(float) * 64 * size_t(NN > t.B ? NN : t.B);
  const int rtb = (t.B + 31) / 32;
  if (rtb <= 2)
    hipLaunchKernelGGL(project_kernel<2>, dim3(unsigned(blocks)), dim3(128), lds, st, patches, P, NN, t.B,
                       t.pinvA, xhat);
  else if (rtb <= 4)
    hipLaunchKernelGGL(project_kernel<4>, dim3(unsigned(blocks)), dim3(128), lds, st, patches, P, NN, t.B,
                       t.pinvA, xhat);
  else if (rtb <= 6)
    hipLaunchKernelGGL(project_kernel<6>, dim3(unsigned(blocks)), dim3(128), lds, st, patches, P, NN, t.B,
                       t.pinvA, xhat);
  else
    return int(hipErrorInvalidValue);
  return int(hipGetLastError());
}


// Rotation of 11x11 patches by a fixed operator from the 97 disk pixels to the 121 grid
// pixels (Phi S_theta Phi^+, built by the plan): the register-operand projection kernel
// with 121 output rows in four 32-row tiles.  16-byte aligned patches only.
int launch_rotate_operator(const float* op, const int* pix, const float* patches, int64_t P, float* out,
                           void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((reinterpret_cast<uintptr_t>(patches) & 15) != 0) return int(hipErrorInvalidValue);
  auto kern = project_reg_kernel<121, 49, 4>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t nfull = P / kProjRegPatches, tail = P - nfull * kProjRegPatches;
  const int64_t work = nfull + (tail > 0), cap = int64_t(cus()) * per_cu;
  const bool vout = (reinterpret_cast<uintptr_t>(out) & 15) == 0;   // 32 x 121 floats per chunk: whole float4s
  hipLaunchKernelGGL(kern, dim3(unsigned(work < cap ? work : cap)), dim3(256), 0, st, patches, nfull, int(tail), 121,
                     op, pix, vout, out);
  return int(hipGetLastError());
}

}  // namespace rsc
