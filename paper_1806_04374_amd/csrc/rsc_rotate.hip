// Patch rotation (Sec. III-C, rotation speed): by interpolation, and by steering.
//
// Interpolation: a plan holds the rotation as a table of taps, the rows of the paper's
// N^2 x N^2 matrix R_nearest or R_bicubic (at most 1 or 16 nonzeros per output pixel),
// built once on the host in FP64; rotate_taps_kernel / rotate_taps_fixed_kernel (11x11,
// 15x15) apply it to a batch of patches.
//   Output pixel (x, y) (x = col - c, y = c - row, c = (N-1)/2) reads the input at
//   R_{-theta}(x, y): nearest-neighbour (coordinates rounded half up) or bicubic (Keys'
//   cubic convolution, a = -1/2, over the 4 x 4 neighbours); input pixels outside the
//   patch count as 0.
// Steering multiplies harmonic k of hat coordinates by exp(-i k theta) (the diagonal S of
// eq. (8), at any angle): steer_stream_kernel (compiled geometries, one angle),
// steer_kernel / steer_any_kernel (per-patch angles, other geometries), and the
// table-driven steer_table_*_kernel for the annular basis' ragged layout.  Synthesis maps
// hat coordinates back to pixels, Phi x_hat (zero off the disk): synth_mfma_kernel
// (compiled geometries), synth_reg_kernel (N*N <= 256), synth_hat_kernel (larger).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "rsc_device.h"
#include "rsc_internal.h"
#include "rsc_launch.h"

namespace rsc {
namespace {

constexpr int kRotPatches = 32;   // patches per block pass in rotate_taps_kernel

// The block's threads form 256 / G groups of G lanes; lane g of a group owns the output
// pixels pix[g], pix[g + G], ... (QPT of them; pix is the plan's lane order) and keeps
// their taps in registers.  Each block stages kRotPatches patches in LDS (coalesced,
// 16-byte loads where aligned), group h applies the taps to patches h, h + 256 / G, ...,
// and writes them (a wave's stores stay within one patch).  G is the smallest of 64, 128,
// 256 that covers N*N (256 for N*N > 256), so few lanes idle.
template <int NTAP, int QPT, int G>
__global__ __launch_bounds__(256) void rotate_taps_kernel(const float* __restrict__ in, int64_t P, int NN,
                                                         const int32_t* __restrict__ src,
                                                         const float* __restrict__ wgt,
                                                         const int32_t* __restrict__ pix, bool vec,
                                                         float* __restrict__ out) {
  constexpr int NSUB = 256 / G;
  extern __shared__ float xs[];   // [kRotPatches][NN]
  const int t = threadIdx.x, g = t % G, sub = t / G;
  float w[QPT][NTAP];
  int sidx[QPT][NTAP], qo[QPT];
#pragma unroll
  for (int j = 0; j < QPT; ++j) {
    const int q = g + G * j < NN ? g + G * j : 0;
    qo[j] = pix[q];
#pragma unroll
    for (int k = 0; k < NTAP; ++k) {
      w[j][k] = wgt[q * NTAP + k];
      sidx[j][k] = src[q * NTAP + k];
    }
  }
  for (int64_t p0 = int64_t(blockIdx.x) * kRotPatches; p0 < P; p0 += int64_t(gridDim.x) * kRotPatches) {
    const int np = P - p0 < kRotPatches ? int(P - p0) : kRotPatches;
    __syncthreads();
    if (vec && np == kRotPatches) {
      const float4* s4 = reinterpret_cast<const float4*>(in + p0 * NN);
      for (int i = t; i < kRotPatches * NN / 4; i += 256) reinterpret_cast<float4*>(xs)[i] = s4[i];
    } else {
      for (int i = t; i < np * NN; i += 256) xs[i] = in[p0 * NN + i];
    }
    __syncthreads();
    for (int p = sub; p < np; p += NSUB) {
      const float* x = xs + p * NN;
#pragma unroll
      for (int j = 0; j < QPT; ++j) {
        const int q = g + G * j;
        if (q >= NN) continue;
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < NTAP; ++k) acc += w[j][k] * x[sidx[j][k]];
        out[(p0 + p) * NN + qo[j]] = acc;
      }
    }
  }
}

// The same for N*N = NNC known at compile time (NNC <= 256, one output pixel per lane,
// G = 128 or 256), whole chunks only, 16-byte aligned input: the next chunk is loaded into
// registers while the current one is computed, and every LDS gather uses the lane's tap
// offset plus an immediate patch offset (no address arithmetic per tap).
typedef float v4f __attribute__((ext_vector_type(4)));

template <int NTAP, int NNC, int G>
__global__ __launch_bounds__(256, 4) void rotate_taps_fixed_kernel(const float* __restrict__ in, int64_t nchunk,
                                                               const int32_t* __restrict__ src,
                                                               const float* __restrict__ wgt,
                                                               const int32_t* __restrict__ pix,
                                                               float* __restrict__ out) {
  constexpr int NSUB = 256 / G, PPG = kRotPatches / NSUB;   // patches per lane group and chunk
  constexpr int NV = kRotPatches * NNC / 4, VPT = (NV + 255) / 256;
  static_assert(NNC <= G && kRotPatches % NSUB == 0, "one output pixel per lane");
  __shared__ v4f xs4[VPT * 256];   // NV used; the rest takes the clamped loads' copies
  const float* xs = reinterpret_cast<const float*>(xs4);
  const int t = threadIdx.x, g = t % G, sub = t / G;
  const bool own = g < NNC;
  const int q = own ? g : 0, qo = pix[q];
  float w[NTAP];
  const float* base[NTAP];
#pragma unroll
  for (int k = 0; k < NTAP; ++k) {
    w[k] = wgt[q * NTAP + k];
    base[k] = xs + sub * NNC + src[q * NTAP + k];
  }
  // loads clamped to the chunk's last float4 (unconditional, so nothing waits on them early)
  int vi[VPT];
#pragma unroll
  for (int v = 0; v < VPT; ++v) vi[v] = t + 256 * v < NV ? t + 256 * v : NV - 1;
  // the launch has at most nchunk blocks, so every block starts on a chunk
  v4f nxt[VPT];
  int64_t c = blockIdx.x;
  {
    const v4f* s4 = reinterpret_cast<const v4f*>(in + c * kRotPatches * NNC);
#pragma unroll
    for (int v = 0; v < VPT; ++v) nxt[v] = s4[vi[v]];
  }
  for (; c < nchunk; c += gridDim.x) {
    __syncthreads();   // the previous chunk's gathers are done
#pragma unroll
    for (int v = 0; v < VPT; ++v) xs4[t + 256 * v] = nxt[v];
    __syncthreads();
    {
      // the next chunk (the last one re-reads its own, unused)
      const int64_t cn = c + gridDim.x < nchunk ? c + gridDim.x : c;
      const v4f* s4 = reinterpret_cast<const v4f*>(in + cn * kRotPatches * NNC);
#pragma unroll
      for (int v = 0; v < VPT; ++v) nxt[v] = s4[vi[v]];
    }
    if (own) {
      float* o = out + c * kRotPatches * NNC + sub * NNC + qo;
#pragma unroll
      for (int i = 0; i < PPG; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < NTAP; ++k) acc += w[k] * base[k][i * NSUB * NNC];
        o[i * NSUB * NNC] = acc;
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
  float cs[32], sn[32]; // cos, sin of k theta0 for k = 0..T (T <= 31), when theta is null
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

// One angle for all patches, compiled geometry: the array is streamed in chunks of
// kSteerChunk whole patches (kSteerChunk * B floats, a multiple of 4) with 16-byte loads
// and stores.  A chunk is staged in LDS, where each output element finds its partner
// (Re <-> Im, S apart).  Since a chunk holds whole patches, the coordinate of each of a
// thread's elements is the same in every chunk, so its coefficients are set up once:
//   out[c] = alpha_c x[c] + beta_c x[c + delta_c],
// alpha = 1, beta = 0 on harmonic 0; alpha = cos k theta, beta = +sin k theta, delta = +S
// on Re; alpha = cos k theta, beta = -sin k theta, delta = -S on Im.
constexpr int kSteerChunk = 64;

template <int S, int T>
__global__ __launch_bounds__(256) void steer_stream_kernel(SteerParams prm, int64_t nchunk, int tail) {
  constexpr int B = S * (2 * T + 1), CF = kSteerChunk * B, NV = CF / 4, VPT = (NV + 255) / 256;
  static_assert(CF % 4 == 0, "a chunk must be whole float4s");
  __shared__ float buf[CF];
  const int t = threadIdx.x;
  float alpha[VPT][4], beta[VPT][4];
  int partner[VPT][4];
#pragma unroll
  for (int v = 0; v < VPT; ++v)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = 4 * (t + 256 * v) + j;   // element of the chunk
      const int c = e % B;                   // its coordinate in the patch
      float a = 1.f, b = 0.f;
      int d = 0;
      if (c >= S && e < CF) {
        const int cc = c - S, k = 1 + cc / (2 * S), im = (cc % (2 * S)) >= S;
        a = prm.cs[k];
        b = im ? -prm.sn[k] : prm.sn[k];
        d = im ? -S : S;
      }
      alpha[v][j] = a;
      beta[v][j] = b;
      partner[v][j] = e < CF ? e + d : 0;
    }
  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const float4* src = reinterpret_cast<const float4*>(prm.xhat + ch * CF);
    float4 x[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v)
      if (t + 256 * v < NV) x[v] = src[t + 256 * v];
    __syncthreads();   // the previous chunk's partner reads are done
#pragma unroll
    for (int v = 0; v < VPT; ++v)
      if (t + 256 * v < NV) reinterpret_cast<float4*>(buf)[t + 256 * v] = x[v];
    __syncthreads();
    float4* dst = reinterpret_cast<float4*>(prm.out + ch * CF);
#pragma unroll
    for (int v = 0; v < VPT; ++v)
      if (t + 256 * v < NV) {
        float4 o;
        o.x = alpha[v][0] * x[v].x + beta[v][0] * buf[partner[v][0]];
        o.y = alpha[v][1] * x[v].y + beta[v][1] * buf[partner[v][1]];
        o.z = alpha[v][2] * x[v].z + beta[v][2] * buf[partner[v][2]];
        o.w = alpha[v][3] * x[v].w + beta[v][3] * buf[partner[v][3]];
        dst[t + 256 * v] = o;
      }
  }
  // the last tail (< kSteerChunk) patches, element by element
  if (tail > 0 && blockIdx.x == nchunk % gridDim.x) {
    const int nel = tail * B;
    const float* src = prm.xhat + nchunk * CF;
    __syncthreads();   // the block's last chunk's partner reads are done
    for (int e = t; e < nel; e += 256) buf[e] = src[e];
    __syncthreads();
    float* dst = prm.out + nchunk * CF;
    for (int e = t; e < nel; e += 256) {   // coefficients recomputed: the arrays above are dead here
      const int c = e % B;
      float o = buf[e];
      if (c >= S) {
        const int cc = c - S, k = 1 + cc / (2 * S);
        const bool im = (cc % (2 * S)) >= S;
        o = prm.cs[k] * o + (im ? -prm.sn[k] * buf[e - S] : prm.sn[k] * buf[e + S]);
      }
      dst[e] = o;
    }
  }
}

// Steering in a layout given by a table (the annular basis): tab[c] = (k << 16) | (off +
// 32768) for coordinate c of harmonic k whose Re/Im partner sits off floats away (off > 0
// for a Re coordinate, < 0 for an Im one, 0 on harmonic 0).  One angle for all patches:
// the chunk pipeline of steer_stream_kernel with B at run time (chunk = 64 patches in
// dynamic LDS, NT threads with VPT >= 16 B / NT float4 each; larger B takes larger blocks
// rather than more registers per thread) and coefficients from the table.
__device__ __forceinline__ void steer_coef(const SteerParams& prm, int code, float& a, float& b, int& off) {
  const int k = code >> 16;
  off = (code & 0xffff) - 32768;
  a = prm.cs[k];
  b = off > 0 ? prm.sn[k] : off < 0 ? -prm.sn[k] : 0.f;
}

template <int VPT, int NT>
__global__ __launch_bounds__(NT) void steer_table_stream_kernel(SteerParams prm, const int* __restrict__ tab,
                                                                int64_t nchunk, int tail) {
  extern __shared__ float buf[];   // [kSteerChunk * B]
  const int B = prm.B, CF = kSteerChunk * B, NV = CF / 4;
  const int t = threadIdx.x;
  float alpha[VPT][4], beta[VPT][4];
  int partner[VPT][4];
#pragma unroll
  for (int v = 0; v < VPT; ++v)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = 4 * (t + NT * v) + j;
      float a = 0.f, b = 0.f;
      int off = 0;
      if (e < CF) steer_coef(prm, tab[e % B], a, b, off);
      alpha[v][j] = a;
      beta[v][j] = b;
      partner[v][j] = e < CF ? e + off : 0;
    }
  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const float4* src = reinterpret_cast<const float4*>(prm.xhat + ch * CF);
    float4 x[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v)
      if (t + NT * v < NV) x[v] = src[t + NT * v];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < VPT; ++v)
      if (t + NT * v < NV) reinterpret_cast<float4*>(buf)[t + NT * v] = x[v];
    __syncthreads();
    float4* dst = reinterpret_cast<float4*>(prm.out + ch * CF);
#pragma unroll
    for (int v = 0; v < VPT; ++v)
      if (t + NT * v < NV) {
        float4 o;
        o.x = alpha[v][0] * x[v].x + beta[v][0] * buf[partner[v][0]];
        o.y = alpha[v][1] * x[v].y + beta[v][1] * buf[partner[v][1]];
        o.z = alpha[v][2] * x[v].z + beta[v][2] * buf[partner[v][2]];
        o.w = alpha[v][3] * x[v].w + beta[v][3] * buf[partner[v][3]];
        dst[t + NT * v] = o;
      }
  }
  if (tail > 0 && blockIdx.x == nchunk % gridDim.x) {
    const int nel = tail * B;
    const float* src = prm.xhat + nchunk * CF;
    __syncthreads();
    for (int e = t; e < nel; e += NT) buf[e] = src[e];
    __syncthreads();
    float* dst = prm.out + nchunk * CF;
    for (int e = t; e < nel; e += NT) {
      float a, b;
      int off;
      steer_coef(prm, tab[e % B], a, b, off);
      dst[e] = a * buf[e] + b * buf[e + off];
    }
  }
}

// Table layout, any buffers, per-patch angles or one angle: one thread per coordinate.
__global__ __launch_bounds__(256) void steer_table_kernel(SteerParams prm, const int* __restrict__ tab) {
  const int B = prm.B;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= prm.P * B) return;
  const int64_t p = i / B;
  const int c = int(i - p * B);
  const int code = tab[c];
  const int k = code >> 16, off = (code & 0xffff) - 32768;
  float a, b;
  if (prm.theta) {
    float sn;
    sincosf(float(k) * prm.theta[p], &sn, &a);
    b = off > 0 ? sn : off < 0 ? -sn : 0.f;
  } else {
    int o2;
    steer_coef(prm, code, a, b, o2);
  }
  prm.out[i] = a * prm.xhat[i] + b * prm.xhat[i + off];
}

// The same for any geometry (index arithmetic at run time).
__global__ __launch_bounds__(256) void steer_any_kernel(SteerParams prm, int T) {
  const int S = prm.S, B = prm.B, W = S * (T + 1);
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

// Phi x_hat for N*N <= 256, B <= 192: lane g of a G-lane group owns output pixel g and
// keeps row g of Phi in registers (BV float4, zero past B); a block stages kSynP patches'
// hat rows in LDS at a padded stride of 4 BV floats (the pads stay zero), and group h
// forms patches h, h + 256 / G, ... with one broadcast 16-byte LDS read per 4 FMAs.
constexpr int kSynP = 32;

template <int BV, int G>
__global__ __launch_bounds__(256) void synth_reg_kernel(const float* __restrict__ xhat, int64_t P, int B, int NN,
                                                       const float* __restrict__ phi, float* __restrict__ out) {
  constexpr int NSUB = 256 / G, BP = 4 * BV;
  __shared__ float4 xs4[kSynP * BV];
  float* xs = reinterpret_cast<float*>(xs4);
  const int t = threadIdx.x, g = t % G, sub = t / G, lane = t & 63, wave = t >> 6;
  const bool own = g < NN;
  float4 ph[BV];
#pragma unroll
  for (int v = 0; v < BV; ++v) {
    float e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = (own && 4 * v + i < B) ? phi[g * B + 4 * v + i] : 0.f;
    ph[v] = make_float4(e[0], e[1], e[2], e[3]);
  }
  for (int i = t; i < kSynP * BP; i += 256) xs[i] = 0.f;
  for (int64_t p0 = int64_t(blockIdx.x) * kSynP; p0 < P; p0 += int64_t(gridDim.x) * kSynP) {
    const int np = P - p0 < kSynP ? int(P - p0) : kSynP;
    __syncthreads();   // also orders the zero fill before the first staging
    for (int pp = wave; pp < np; pp += 4)
      for (int c = lane; c < B; c += 64) xs[pp * BP + c] = xhat[(p0 + pp) * B + c];
    __syncthreads();
    if (own) {
      for (int p = sub; p < np; p += NSUB) {
        const float4* x = xs4 + p * BV;
        float a0 = 0.f, a1 = 0.f;
#pragma unroll
        for (int v = 0; v < BV; ++v) {
          const float4 xv = x[v];
          a0 += ph[v].x * xv.x;
          a1 += ph[v].y * xv.y;
          a0 += ph[v].z * xv.z;
          a1 += ph[v].w * xv.w;
        }
        out[(p0 + p) * NN + g] = a0 + a1;
      }
    }
  }
}

// Blocks of 256 threads (no dynamic LDS) that fit on the whole chip at once: a grid of
// this size runs in one round, each block looping over its share of chunks.
// Cached per kernel (the query is host work on every launch otherwise).
template <class Kern>
int64_t resident_blocks(Kern kern) {
  static std::mutex mu;
  static std::unordered_map<const void*, int64_t> cache;
  const void* key = reinterpret_cast<const void*>(kern);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess || per_cu < 1) per_cu = 4;
  return cache[key] = int64_t(num_cus()) * per_cu;
}

// Phi x_hat on FP32 MFMA for the compiled geometries (N*N = NNC, B = BB): rows = output
// pixels (tiles of 32; wave w owns tiles w*TPW .. w*TPW+TPW-1 with its rows of Phi in
// registers), columns = 32 patches, contraction over hat coordinates in steps of 2.  The
// block takes 32 patches at a time: their hat rows are staged in LDS (the next chunk's
// loaded into registers meanwhile) and the pixels leave through an LDS staging tile with
// coalesced 16-byte stores.  synA: [NTT][KB][64], lane l of step j in tile tt holds
// Phi[32 tt + l % 32][2 j + l / 32] (zero past N*N or B).
constexpr int kSynMP = 32;

template <int NNC, int BB, int TPW>
__global__ __launch_bounds__(256) void synth_mfma_kernel(const float* __restrict__ xhat, int64_t nchunk,
                                                        const float* __restrict__ synA, bool vec_out,
                                                        float* __restrict__ out) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  constexpr int KB = (BB + 1) / 2, NV = kSynMP * BB / 4, VPT = (NV + 255) / 256;
  static_assert((kSynMP * BB) % 4 == 0 && (kSynMP * NNC) % 4 == 0, "chunks of whole float4s");
  static_assert(4 * TPW * 32 >= NNC, "row tiles must cover the pixels");
  __shared__ v4f xs4[VPT * 256];                 // [32][BB] used; the rest takes clamped copies
  __shared__ v4f st4[kSynMP * NNC / 4];          // [32 patches][NNC]
  const float* xs = reinterpret_cast<const float*>(xs4);
  float* st = reinterpret_cast<float*>(st4);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, col = lane & 31, u = lane >> 5;
  float a[TPW][KB];
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int j = 0; j < KB; ++j) a[i][j] = synA[((w * TPW + i) * KB + j) * 64 + lane];
  int vi[VPT];
#pragma unroll
  for (int v = 0; v < VPT; ++v) vi[v] = t + 256 * v < NV ? t + 256 * v : NV - 1;
  // the launch has at most nchunk blocks, so every block starts on a chunk
  v4f nxt[VPT];
  int64_t c = blockIdx.x;
  {
    const v4f* s4 = reinterpret_cast<const v4f*>(xhat + c * kSynMP * BB);
#pragma unroll
    for (int v = 0; v < VPT; ++v) nxt[v] = s4[vi[v]];
  }
  const float* mine = xs + col * BB + u;
  for (; c < nchunk; c += gridDim.x) {
    __syncthreads();   // the previous chunk's hat and staging reads are done
#pragma unroll
    for (int v = 0; v < VPT; ++v) xs4[t + 256 * v] = nxt[v];
    __syncthreads();
    {
      const int64_t cn = c + gridDim.x < nchunk ? c + gridDim.x : c;   // the last re-reads its own
      const v4f* s4 = reinterpret_cast<const v4f*>(xhat + cn * kSynMP * BB);
#pragma unroll
      for (int v = 0; v < VPT; ++v) nxt[v] = s4[vi[v]];
    }
    f32x16 acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const float b = 2 * j + u < BB ? mine[2 * j] : 0.f;   // odd B: the last slot is padding
#pragma unroll
      for (int i = 0; i < TPW; ++i) acc[i] = mfma32(a[i][j], b, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int q = 32 * (w * TPW + i) + 8 * (r / 4) + 4 * u + (r % 4);
        if (q < NNC) st[col * NNC + q] = acc[i][r];
      }
    __syncthreads();
    float* dst = out + c * kSynMP * NNC;
    if (vec_out) {
      for (int i = t; i < kSynMP * NNC / 4; i += 256) reinterpret_cast<v4f*>(dst)[i] = st4[i];
    } else {
      for (int i = t; i < kSynMP * NNC; i += 256) dst[i] = st[i];
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

int rotation_taps(int N, double theta, int mode, std::vector<int32_t>& src, std::vector<float>& w,
                  std::vector<int32_t>& pix) {
  const int NN = N * N, ntap = mode == 0 ? 1 : 16;
  src.assign(size_t(NN) * ntap, 0);
  w.assign(size_t(NN) * ntap, 0.f);
  std::vector<int64_t> key(NN);
  const double c = (N - 1) / 2.0, cs = std::cos(theta), sn = std::sin(theta);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const double x = j - c, y = c - i;
      const double xs = cs * x + sn * y, ys = -sn * x + cs * y;   // R_{-theta} (x, y)
      const double col = c + xs, row = c - ys;
      const int q = i * N + j;
      key[q] = int64_t(std::floor(row)) * N + int64_t(std::floor(col));
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
  // Lane order.  Bicubic with N*N <= 128 (lane groups of 64 or 128): output pixels sorted
  // by the input position they read (row-major), so that neighbouring lanes gather from
  // neighbouring LDS words and a wave's 16 gathers per pixel spread over the banks instead
  // of striding across the patch (at 11x11 this takes the kernel from bank-conflict bound
  // to about 0.6 of its time).  Elsewhere the natural order, which measured faster: with one
  // tap there are few gathers to spread, and with 256-lane groups (15x15) the sorted order
  // was slower even with its stores staged through LDS.
  // pix[g] is the output pixel of lane g; the tap rows are stored in lane order.
  pix.resize(NN);
  for (int q = 0; q < NN; ++q) pix[q] = q;
  if (mode == 1 && NN <= 128)
    std::stable_sort(pix.begin(), pix.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  std::vector<int32_t> src2(src.size());
  std::vector<float> w2(w.size());
  for (int g = 0; g < NN; ++g)
    for (int k = 0; k < ntap; ++k) {
      src2[size_t(g) * ntap + k] = src[size_t(pix[g]) * ntap + k];
      w2[size_t(g) * ntap + k] = w[size_t(pix[g]) * ntap + k];
    }
  src.swap(src2);
  w.swap(w2);
  return ntap;
}

size_t rotate_lds_bytes(int N, int ntap) {
  (void)ntap;
  return sizeof(float) * size_t(kRotPatches) * N * N;
}

int launch_rotate_taps(int N, int ntap, const float* in, int64_t P, const int32_t* src, const float* w,
                       const int32_t* pix, float* out, void* stream) {
  const int NN = N * N;
  const int64_t cap = int64_t(num_cus()) * 8;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int qpt = (NN + 255) / 256;
  const size_t lds = rotate_lds_bytes(N, ntap);
  const bool vec = (reinterpret_cast<uintptr_t>(in) & 15) == 0;   // kRotPatches * NN is a multiple of 4
  // 11x11 and 15x15: whole chunks by the pipelined kernel, the rest by the general one
  const int64_t nfull = vec && (NN == 121 || NN == 225) ? P / kRotPatches : 0;
  if (nfull > 0) {
    // one resident round of blocks (as many as fit on every CU at once), each looping
    // over chunks, so no CU idles on a partial second round
    auto fixed = [&](auto kern) {
      const int64_t blocks = resident_blocks(kern);
      hipLaunchKernelGGL(kern, dim3(unsigned(nfull < blocks ? nfull : blocks)), dim3(256), 0, st, in, nfull, src,
                         w, pix, out);
      return hipGetLastError();
    };
    hipError_t e;
    if (NN == 121) e = ntap == 1 ? fixed(rotate_taps_fixed_kernel<1, 121, 128>) : fixed(rotate_taps_fixed_kernel<16, 121, 128>);
    else e = ntap == 1 ? fixed(rotate_taps_fixed_kernel<1, 225, 256>) : fixed(rotate_taps_fixed_kernel<16, 225, 256>);
    if (e != hipSuccess) return int(e);
    const int64_t done = nfull * kRotPatches;
    if (done == P) return 0;
    in += done * NN;
    out += done * NN;
    P -= done;
  }
  const int64_t want = (P + kRotPatches - 1) / kRotPatches;
  const unsigned grid = unsigned(want < cap ? want : cap);
  auto go = [&](auto kern) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(lds));
    if (e != hipSuccess) return int(e);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, st, in, P, NN, src, w, pix, vec, out);
    return int(hipGetLastError());
  };
  if (ntap == 1) {
    if (NN <= 64) return go(rotate_taps_kernel<1, 1, 64>);
    if (NN <= 128) return go(rotate_taps_kernel<1, 1, 128>);
    return qpt == 1 ? go(rotate_taps_kernel<1, 1, 256>) : qpt == 2 ? go(rotate_taps_kernel<1, 2, 256>)
                                                                : go(rotate_taps_kernel<1, 3, 256>);
  }
  if (NN <= 64) return go(rotate_taps_kernel<16, 1, 64>);
  if (NN <= 128) return go(rotate_taps_kernel<16, 1, 128>);
  return qpt == 1 ? go(rotate_taps_kernel<16, 1, 256>) : qpt == 2 ? go(rotate_taps_kernel<16, 2, 256>)
                                                               : go(rotate_taps_kernel<16, 3, 256>);
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
  for (int k = 0; k <= t.T && k < 32; ++k) {
    prm.cs[k] = float(std::cos(k * theta0));
    prm.sn[k] = float(std::sin(k * theta0));
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (t.steerTab) {
    // table layout: chunks streamed for one angle and 16-byte aligned buffers, else one
    // thread per coordinate
    const bool al = ((reinterpret_cast<uintptr_t>(xhat) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    if (!theta && al && t.B <= 192) {
      const int64_t nchunk = P / kSteerChunk;
      const int tail = int(P - nchunk * kSteerChunk);
      const int64_t work = nchunk + (tail > 0);
      const size_t lds = sizeof(float) * kSteerChunk * size_t(t.B);
      auto go = [&](auto kern, int nt) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, lds) != hipSuccess || per_cu < 1)
          per_cu = 1;
        const int64_t blocks = int64_t(num_cus()) * per_cu;
        hipLaunchKernelGGL(kern, dim3(unsigned(work < blocks ? work : blocks)), dim3(nt), lds, st, prm,
                           static_cast<const int*>(t.steerTab), nchunk, tail);
        return hipGetLastError();
      };
      // NV = 16 B float4 per chunk: B <= 64 -> 4 x 256, <= 96 -> 3 x 512, <= 128 -> 4 x 512, else 3 x 1024
      return int(t.B <= 64   ? go(steer_table_stream_kernel<4, 256>, 256)
                 : t.B <= 96 ? go(steer_table_stream_kernel<3, 512>, 512)
                 : t.B <= 128 ? go(steer_table_stream_kernel<4, 512>, 512)
                              : go(steer_table_stream_kernel<3, 1024>, 1024));
    }
    const int64_t items = P * int64_t(t.B);
    hipLaunchKernelGGL(steer_table_kernel, dim3(unsigned((items + 255) / 256)), dim3(256), 0, st, prm,
                       static_cast<const int*>(t.steerTab));
    return int(hipGetLastError());
  }
  // one angle, compiled geometry, 16-byte aligned buffers: the streaming kernel; otherwise
  // the per-coordinate kernels below
  const bool aligned = ((reinterpret_cast<uintptr_t>(xhat) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  const int geo = t.S == 5 && t.T == 5 ? 0 : t.S == 7 && t.T == 7 ? 1 : t.S == 5 && t.T == 2 ? 2
                : t.S == 7 && t.T == 3 ? 3 : -1;
  if (!theta && aligned && geo >= 0) {
    // whole chunks streamed, the last partial chunk by one block of the same launch
    const int64_t nchunk = P / kSteerChunk;
    const int tail = int(P - nchunk * kSteerChunk);
    const int64_t work = nchunk + (tail > 0);
    auto go = [&](auto kern) {
      const int64_t blocks = resident_blocks(kern);
      hipLaunchKernelGGL(kern, dim3(unsigned(work < blocks ? work : blocks)), dim3(256), 0, st, prm, nchunk, tail);
      return hipGetLastError();
    };
    hipError_t e = geo == 0 ? go(steer_stream_kernel<5, 5>) : geo == 1 ? go(steer_stream_kernel<7, 7>)
                 : geo == 2 ? go(steer_stream_kernel<5, 2>) : go(steer_stream_kernel<7, 3>);
    return int(e);
  }
  const int64_t items = P * int64_t(t.S) * (t.T + 1);
  const dim3 grid(unsigned((items + 255) / 256));
  if (t.S == 5 && t.T == 5) hipLaunchKernelGGL((steer_kernel<5, 5>), grid, dim3(256), 0, st, prm);
  else if (t.S == 7 && t.T == 7) hipLaunchKernelGGL((steer_kernel<7, 7>), grid, dim3(256), 0, st, prm);
  else if (t.S == 5 && t.T == 2) hipLaunchKernelGGL((steer_kernel<5, 2>), grid, dim3(256), 0, st, prm);
  else if (t.S == 7 && t.T == 3) hipLaunchKernelGGL((steer_kernel<7, 3>), grid, dim3(256), 0, st, prm);
  else hipLaunchKernelGGL(steer_any_kernel, grid, dim3(256), 0, st, prm, t.T);
  return int(hipGetLastError());
}

int launch_synth_hat(const DeviceTables& t, const float* xhat, int64_t P, float* out, void* stream) {
  const int NN = t.N * t.N;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // compiled geometries, 16-byte aligned hat rows: whole 32-patch chunks on MFMA, the rest below
  const int geo = NN == 121 && t.B == 55 ? 0 : NN == 225 && t.B == 105 ? 1 : -1;
  const int64_t nm = (geo >= 0 && t.synA && (reinterpret_cast<uintptr_t>(xhat) & 15) == 0) ? P / kSynMP : 0;
  if (nm > 0) {
    const bool vout = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
    auto go = [&](auto kern) {
      const int64_t blocks = resident_blocks(kern);
      hipLaunchKernelGGL(kern, dim3(unsigned(nm < blocks ? nm : blocks)), dim3(256), 0, st, xhat, nm, t.synA, vout,
                         out);
      return hipGetLastError();
    };
    hipError_t e = geo == 0 ? go(synth_mfma_kernel<121, 55, 1>) : go(synth_mfma_kernel<225, 105, 2>);
    if (e != hipSuccess) return int(e);
    const int64_t done = nm * kSynMP;
    if (done == P) return 0;
    xhat += done * t.B;
    out += done * NN;
    P -= done;
  }
  if (NN <= 256 && t.B <= 192) {
    const int bv = (t.B + 3) / 4;
    const int64_t want = (P + kSynP - 1) / kSynP;
    const int64_t cap = int64_t(num_cus()) * 8;
    const dim3 grid(unsigned(want < cap ? want : cap));
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, xhat, P, t.B, NN, t.phiPad, out);
      return int(hipGetLastError());
    };
    // exact row lengths of the compiled geometries, else rounded up (zero pads)
    auto pick = [&](auto g_tag) -> int {
      constexpr int G = decltype(g_tag)::value;
      switch (bv) {
        case 7: return go(synth_reg_kernel<7, G>);
        case 13: return go(synth_reg_kernel<13, G>);
        case 14: return go(synth_reg_kernel<14, G>);
        case 27: return go(synth_reg_kernel<27, G>);
        default: return bv <= 16 ? go(synth_reg_kernel<16, G>) : bv <= 32 ? go(synth_reg_kernel<32, G>)
                                                                         : go(synth_reg_kernel<48, G>);
      }
    };
    if (NN <= 64) return pick(std::integral_constant<int, 64>{});
    if (NN <= 128) return pick(std::integral_constant<int, 128>{});
    return pick(std::integral_constant<int, 256>{});
  }
  const size_t lds = sizeof(float) * (size_t(NN) * t.B + 8 * size_t(t.B));
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(synth_hat_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return int(e);
  const int64_t want = (P + 7) / 8;
  const int64_t cap = int64_t(num_cus()) * 2;
  const unsigned grid = unsigned(want < cap ? want : cap);
  hipLaunchKernelGGL(synth_hat_kernel, dim3(grid), dim3(256), lds, st, xhat, P, t.B, NN, t.phiPad, out);
  return int(hipGetLastError());
}

}  // namespace rsc
