// Dictionary update of rotational K-SVD (Fig. 2, the loop over atoms; Sec. II-C), in
// hat coordinates (Sec. II-E).
//
// The augmented dictionary is built once per outer iteration, so every atom is
// updated from the same codes and the same old dictionary, all atoms at once:
//   1. a counting sort of the (patch, slot) pairs by atom, keeping for each patch
//      only the first slot that holds a given atom: per-block counts
//      (rk_count_kernel), one scan (rk_plan_kernel: bucket offsets per block and
//      atom, and fixed-size chunks of each bucket), and an in-order scatter
//      (rk_scatter_kernel), so every bucket lists its patches in increasing order;
//   2. rk_resid_kernel: every patch's residual r = x - D b over its whole code, in
//      FP64; then, by the identity x - sum_{j != i0} c_j S_{r_j} d_{m_j} = r + c_{i0} S_{r0} d_m,
//      the vector of a pair (patch, its first slot i0 holding atom m, angle r0) is
//        y = S_{-r0} r + c_{i0} d_m;
//   2'. rk_accum_kernel, one block per chunk of a bucket: y of each pair is formed in
//      FP64 and sum y y^T is taken on the FP64 matrix cores; each chunk writes its
//      partial sum, and rk_reduce_kernel adds each atom's partials in chunk order;
//   3. rk_eig_kernel, one block per atom: C_m = Y_m Y_m^T goes to LDS; its top eigenvector, the first left
//      singular vector of Y_m, comes from a Householder tridiagonalisation in place,
//      a multisection on Sturm counts for the largest eigenvalue, inverse iteration
//      on the tridiagonal matrix and the back-transformation through the stored
//      reflectors.  Its sign makes it agree with the old atom;
//   4. rk_reset_kernel: atoms that no patch uses take, in index order, the
//      directions of the patches with the largest coding error (positive ones only;
//      ties to the smaller patch index).
// Every sum is taken in a fixed order, so the update is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "rsc_internal.h"
#include "rsc_launch.h"

namespace rsc {
namespace {

constexpr int kSortBlocks = 1024;
constexpr size_t kResidLdsPaired = 96 * 1024;   // above this the residual kernel keeps single values
constexpr int kChunkTarget = 4096;
constexpr int kChunkMin = 256;

// Workspace layout of the update (offsets in bytes, 256-byte aligned).
struct RkWs {
  size_t cnt, off, tot, bucket, chunk, scal, lp, lr, lc, resid, partial, total;
};

// Row stride of the residuals: one, two or three whole waves per patch, so that a wave's
// patch index is uniform (its code entries come through scalar loads).
__host__ __device__ inline int resid_stride(int B) { return B <= 64 ? 64 : B <= 128 ? 128 : 192; }

__host__ __device__ inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Upper bound on the chunks of a plan: each bucket of n pairs makes ceil(n / CH)
// chunks with CH >= max(kChunkMin, total / kChunkTarget), so there are at most
// min(kChunkTarget, P K / kChunkMin) + M.
__host__ __device__ inline int64_t max_chunks(int M, int64_t P, int K) {
  const int64_t a = (P * K + kChunkMin - 1) / kChunkMin;
  return (a < kChunkTarget ? a : kChunkTarget) + M;
}

__host__ __device__ inline RkWs rk_ws(int M, int B, int64_t P, int K) {
  RkWs w;
  w.cnt = 0;
  w.off = w.cnt + al256(sizeof(int64_t) * size_t(kSortBlocks) * M);
  w.tot = w.off + al256(sizeof(int64_t) * size_t(kSortBlocks) * M);
  w.bucket = w.tot + al256(sizeof(int64_t) * (size_t(M) + 1));
  w.chunk = w.bucket + al256(sizeof(int64_t) * (size_t(M) + 1));
  w.scal = w.chunk + al256(sizeof(int32_t) * (size_t(M) + 1));
  w.lp = w.scal + al256(sizeof(int64_t) * 8);
  w.lr = w.lp + al256(sizeof(int32_t) * size_t(P) * K);
  w.lc = w.lr + al256(sizeof(int32_t) * size_t(P) * K);
  w.resid = w.lc + al256(sizeof(float) * size_t(P) * K);
  w.partial = w.resid + al256(sizeof(double) * size_t(P) * resid_stride(B));
  w.total = w.partial + al256(sizeof(double) * size_t(max_chunks(M, P, K)) * B * B);
  return w;
}

struct SortParams {
  const int32_t* atom;
  const int32_t* angle;
  const float* coef;
  int64_t P;
  int K, M;
  int64_t* cnt;       // [kSortBlocks][M]
  int64_t* off;       // [kSortBlocks][M] offset of each block's pairs within the atom's bucket
  int64_t* tot;       // [M] pairs per atom
  int64_t* bucket;    // [M + 1] start of each atom's bucket in list
  int32_t* chunk;     // [M + 1] first chunk of each atom
  int64_t* scal;      // [0] pairs per chunk, [1] chunks
  // the pairs by atom, patches increasing: patch, angle r0 and coefficient of the slot
  int32_t* lp;        // [P K]
  int32_t* lr;        // [P K]
  float* lc;          // [P K]
};

__device__ __forceinline__ bool first_use(const int32_t* a, int i) {
  for (int j = 0; j < i; ++j)
    if (a[j] == a[i]) return false;
  return a[i] >= 0;
}

__global__ __launch_bounds__(256) void rk_count_kernel(SortParams prm) {
  extern __shared__ int cnt_s[];   // [M]
  for (int i = threadIdx.x; i < prm.M; i += 256) cnt_s[i] = 0;
  __syncthreads();
  const int64_t per = (prm.P + kSortBlocks - 1) / kSortBlocks;
  const int64_t p0 = int64_t(blockIdx.x) * per, p1 = p0 + per < prm.P ? p0 + per : prm.P;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
    const int32_t* a = prm.atom + p * prm.K;
    for (int i = 0; i < prm.K; ++i)
      if (first_use(a, i) && a[i] < prm.M) atomicAdd(&cnt_s[a[i]], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < prm.M; i += 256) prm.cnt[size_t(blockIdx.x) * prm.M + i] = cnt_s[i];
}

// One block per atom: exclusive scan of its per-block counts in block order, and the
// atom's total.
__global__ __launch_bounds__(256) void rk_scan_kernel(SortParams prm) {
  constexpr int G = kSortBlocks / 256;   // blocks per thread
  static_assert(kSortBlocks % 256 == 0, "whole blocks per thread");
  __shared__ int64_t sh[2][256];
  const int m = blockIdx.x, t = threadIdx.x, M = prm.M;
  int64_t c[G], mine = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    c[g] = prm.cnt[size_t(t * G + g) * M + m];
    mine += c[g];
  }
  // inclusive scan of the 256 thread sums (Hillis-Steele, double-buffered)
  int cur = 0;
  sh[0][t] = mine;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    const int64_t v = sh[cur][t] + (t >= d ? sh[cur][t - d] : 0);
    sh[cur ^ 1][t] = v;
    cur ^= 1;
    __syncthreads();
  }
  int64_t run = sh[cur][t] - mine;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    prm.off[size_t(t * G + g) * M + m] = run;
    run += c[g];
  }
  if (t == 255) prm.tot[m] = sh[cur][255];
}

// One block: bucket starts and the chunking of each bucket into pieces of CH pairs
// (CH chosen so that about kChunkTarget chunks exist).
__global__ __launch_bounds__(256) void rk_plan_kernel(SortParams prm) {
  __shared__ int64_t start[257];
  __shared__ int32_t nch[257];
  const int M = prm.M, t = threadIdx.x;
  if (t == 0) {
    int64_t run = 0;
    for (int m = 0; m < M; ++m) {
      start[m] = run;
      run += prm.tot[m];
    }
    start[M] = run;
    int64_t ch = (run + kChunkTarget - 1) / kChunkTarget;
    ch = ch < kChunkMin ? kChunkMin : ch;
    int32_t c = 0;
    for (int m = 0; m < M; ++m) {
      nch[m] = c;
      c += int32_t((start[m + 1] - start[m] + ch - 1) / ch);
    }
    nch[M] = c;
    prm.scal[0] = ch;
    prm.scal[1] = c;
  }
  __syncthreads();
  for (int m = t; m <= M; m += 256) {
    prm.bucket[m] = start[m];
    prm.chunk[m] = nch[m];
  }
}

// In-order scatter, one wave per block over its patches 64 at a time: a lane's rank
// within an atom's bucket is the number of lower lanes whose patch uses that atom,
// read from a per-atom lane mask, so each bucket lists patches in increasing order.
__global__ __launch_bounds__(64) void rk_scatter_kernel(SortParams prm) {
  extern __shared__ int64_t off_s[];   // [M] next free position, then [M] lane masks
  unsigned long long* mask = reinterpret_cast<unsigned long long*>(off_s + prm.M);
  const int M = prm.M, K = prm.K, l = threadIdx.x;
  for (int i = l; i < M; i += 64) {
    off_s[i] = prm.bucket[i] + prm.off[size_t(blockIdx.x) * M + i];
    mask[i] = 0ull;
  }
  __syncthreads();
  const unsigned long long below = (1ull << l) - 1ull;
  const int64_t per = (prm.P + kSortBlocks - 1) / kSortBlocks;
  const int64_t p0 = int64_t(blockIdx.x) * per, p1 = p0 + per < prm.P ? p0 + per : prm.P;
  for (int64_t pb = p0; pb < p1; pb += 64) {
    const int64_t p = pb + l;
    int a[8];
    unsigned use = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      a[i] = -1;
      if (i < K && p < p1) a[i] = prm.atom[p * K + i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      bool first = a[i] >= 0 && a[i] < M;
#pragma unroll
      for (int j = 0; j < i; ++j) first = first && a[j] != a[i];
      if (first) {
        use |= 1u << i;
        atomicOr(&mask[a[i]], 1ull << l);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (use & (1u << i)) {
        const int64_t pos = off_s[a[i]] + __popcll(mask[a[i]] & below);
        prm.lp[pos] = int32_t(p);
        prm.lr[pos] = prm.angle[p * K + i];
        prm.lc[pos] = prm.coef[p * K + i];
      }
    __syncthreads();
    for (int i = l; i < M; i += 64) {
      off_s[i] += __popcll(mask[i]);
      mask[i] = 0ull;
    }
    __syncthreads();
  }
}

// Harmonic blocks of the packed coordinates: harmonic 0 on [kb[0], kb[1]), harmonic k >= 1
// on [kb[k], kb[k+1]) as [Re][Im] halves.  The (S, T) grid has kb[k] = S + 2 S (k - 1); the
// annular basis has as many profiles per harmonic as annuli carry it.
struct HarmBlocks {
  int T;
  int kb[33];
};

struct AccParams {
  const double* __restrict__ resid;   // [P][BP] residuals
  int BP, M, R, B, T;
  HarmBlocks hb;
  const float* __restrict__ dict;     // [16 NG][B] old dictionary
  const double* __restrict__ cs64;    // [2][T+1][R]
  const int64_t* __restrict__ bucket; // [M + 1]
  const int32_t* __restrict__ chunk;  // [M + 1]
  const int64_t* __restrict__ scal;   // pairs per chunk, chunks
  const int32_t* __restrict__ lp;
  const int32_t* __restrict__ lr;
  const float* __restrict__ lc;
  double* __restrict__ partial;       // [chunks][B][B]
};

// Coordinate b of S_theta v, with theta = sgn * 2 pi r / R, for a packed vector v in
// memory (harmonic k multiplied by exp(-i k theta)).
struct Coord {
  int k, part, partner;  // harmonic, 0 = Re / 1 = Im, index of the other part (b for k = 0)
};

__device__ __forceinline__ Coord coord_of(int b, const HarmBlocks& hb) {
  if (b < hb.kb[1]) return {0, 0, b};
  int k = 1;
  while (k < hb.T && b >= hb.kb[k + 1]) ++k;
  const int nk = (hb.kb[k + 1] - hb.kb[k]) / 2, rem = b - hb.kb[k];
  return rem < nk ? Coord{k, 0, b + nk} : Coord{k, 1, b - nk};
}

// Coordinate of S_theta v, theta = sgn 2 pi r / R, from the coordinate's own value, its
// partner's and (cos, sin) of k theta for its harmonic k: harmonic k is multiplied by
// exp(-i k theta), so Re' = a cos + b sin and Im' = b cos - a sin, i.e. sigma = +sgn for a
// real part and -sgn for an imaginary part.  For harmonic 0 the table holds
// (cos, sin) = (1, 0), which returns own exactly.
__device__ __forceinline__ double rot(double own, double other, double cs, double sn, double sigma) {
  return fma(own, cs, other * (sigma * sn));
}

// Upper-triangle tiles of a symmetric matrix of NR x NR 16 x 16 tiles, row by row:
// tile u is (r, s) with r <= s.
__host__ __device__ constexpr int tile_r(int u, int NR) {
  int r = 0;
  while (u >= NR - r) {
    u -= NR - r;
    ++r;
  }
  return r;
}
__host__ __device__ constexpr int tile_s(int u, int NR) {
  int r = 0;
  while (u >= NR - r) {
    u -= NR - r;
    ++r;
  }
  return r + u;
}

struct ResidParams {
  const float* __restrict__ xhat;
  const int32_t* __restrict__ atom;
  const int32_t* __restrict__ angle;
  const float* __restrict__ coef;
  const float* __restrict__ dict;     // [16 NG][B]
  const double* __restrict__ cs64;    // [2][T+1][R]
  int64_t P;
  int K, M, R, B, BP, T;
  HarmBlocks hb;
  double* __restrict__ resid;         // [P][BP]
};

// Residual of every patch over its whole code, r = x - sum_j c_j S_{r_j} d_{m_j} (slots in
// order; an absent entry adds 0 d_0), in FP64; coordinates B..BP-1 are zero.  The
// dictionary and the rotation table sit in LDS; a block of G BP threads strides over
// the patches G at a time, thread (g, b) owning coordinate b of one patch.
// PAIRED: the dictionary in LDS as (own, partner) pairs, one read per atom and
// coordinate; otherwise as single values (half the LDS, for large M B), two reads.
template <int KMAX, bool PAIRED>
__global__ __launch_bounds__(256) void rk_resid_kernel(ResidParams prm) {
  extern __shared__ double ldsd[];
  const int B = prm.B, BP = prm.BP, R = prm.R, M = prm.M, K = prm.K, NQ = prm.T + 1;
  double2* sc = reinterpret_cast<double2*>(ldsd);            // [R][NQ] (cos, sin)
  float2* sd = reinterpret_cast<float2*>(sc + R * NQ);        // [M][B] (d_b, d_partner(b)) if PAIRED
  float* sd1 = reinterpret_cast<float*>(sc + R * NQ);         // [M][B] otherwise
  const int t = threadIdx.x, nt = blockDim.x, G = nt / BP;
  __shared__ int spart[kRkMaxB];   // partner of each coordinate, found once per block
  for (int i = t; i < B; i += nt) spart[i] = coord_of(i, prm.hb).partner;
  for (int i = t; i < R * NQ; i += nt) {
    const int r = i / NQ, k = i - r * NQ;
    sc[i] = double2{prm.cs64[k * R + r], prm.cs64[(NQ + k) * R + r]};
  }
  if constexpr (PAIRED) __syncthreads();   // spart
  for (int i = t; i < M * B; i += nt) {
    if constexpr (PAIRED) {
      const int a = i / B, bb = i - a * B;
      sd[i] = float2{prm.dict[i], prm.dict[a * B + spart[bb]]};
    } else {
      sd1[i] = prm.dict[i];
    }
  }
  __syncthreads();
  const int g = __builtin_amdgcn_readfirstlane(t / BP), b = t - g * BP, bc = b < B ? b : 0;
  const Coord cd = coord_of(bc, prm.hb);
  const double sig = cd.part == 0 ? 1.0 : -1.0;
  // Two patches per wave and pass.  Lane j of the wave loads code entry j of each (a
  // vector load, so no wait on the shared LDS/scalar counter), and the entries are
  // broadcast with readlane; every load is issued before any value is used.
  constexpr int U = 2;
  const int64_t stride = int64_t(gridDim.x) * G;
  const int lane = t % 64, jl = lane < K ? lane : 0;
  // the next pass's codes and coordinates are loaded while this pass is computed (indices
  // clamped to the last patch, so the loads need no branch)
  int an[U], rn[U];
  float cn[U], xn[U];
  auto fetch = [&](int64_t q0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t p = q0 + u * stride < prm.P ? q0 + u * stride : prm.P - 1;
      an[u] = prm.atom[p * K + jl];
      rn[u] = prm.angle[p * K + jl];
      cn[u] = prm.coef[p * K + jl];
      xn[u] = prm.xhat[p * B + bc];
    }
  };
  int64_t p0 = int64_t(blockIdx.x) * G + g;
  if (p0 < prm.P) fetch(p0);
  for (; p0 < prm.P; p0 += U * stride) {
    int av[U], rv[U];
    float cv[U];
    double r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      av[u] = an[u];
      rv[u] = rn[u];
      cv[u] = cn[u];
      r[u] = xn[u];
    }
    fetch(p0 + U * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int j = 0; j < KMAX; ++j) {
        const int aj = __builtin_amdgcn_readlane(av[u], j), rj = __builtin_amdgcn_readlane(rv[u], j);
        const float cj = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, cv[u]), j));
        // an angle outside 0..R-1 (not produced by the pursuit) reads angle 0, in bounds
        const bool use = j < K && aj >= 0 && aj < M;
        float2 dd;
        if constexpr (PAIRED) {
          dd = sd[(use ? aj : 0) * B + bc];
        } else {
          const float* d = sd1 + (use ? aj : 0) * B;
          dd = float2{d[bc], d[cd.partner]};
        }
        const double2 cs = sc[(use && unsigned(rj) < unsigned(R) ? rj : 0) * NQ + cd.k];
        r[u] = fma(-double(use ? cj : 0.f), rot(dd.x, dd.y, cs.x, cs.y, sig), r[u]);
      }
      const int64_t p = p0 + u * stride;
      if (p < prm.P) prm.resid[p * BP + b] = b < B ? r[u] : 0.0;
    }
  }
}

// BT (64, 128 or 192) covers B; W waves per block, NH = 64 W / BT groups of BT threads,
// group h forming pairs h KP .. h KP + KP - 1 of each batch of KQ.  Thread (row, h)
// forms coordinate row of y = S_{-r0} r + c d_m for its pairs into Y (LDS, [KQ][BT]);
// sum y y^T is the symmetric product Y^T Y, taken on the FP64 matrix cores in 16 x 16
// tiles of the upper triangle of the ceil(B/16) row blocks that B needs (at most NRMAX),
// four pairs per product, tiles shared out among the waves.  Software pipeline: the pair
// records (patch, r0, c) of batch b + 2 and the residual rows of batch b + 1 are loaded
// while batch b is formed and multiplied.  FULL: B needs all NRMAX row blocks and every
// wave has the same number of tiles, so the tile loop needs no test.
template <int BT, int W, int KQ, int NRMAX, bool FULL>
__global__ __launch_bounds__(64 * W) void rk_accum_kernel(AccParams prm) {
  constexpr int NT = 64 * W, NH = NT / BT, KP = KQ / NH;
  constexpr int TW = (NRMAX * (NRMAX + 1) / 2 + W - 1) / W;
  static_assert(NT % BT == 0 && KQ % NH == 0 && KQ % 4 == 0 && BT % 64 == 0 && 16 * NRMAX <= BT, "block shape");
  static_assert(!FULL || (NRMAX * (NRMAX + 1) / 2) % W == 0, "FULL needs whole tile rounds");
  typedef double d4 __attribute__((ext_vector_type(4)));
  extern __shared__ double ldsd[];
  const int B = prm.B, BP = prm.BP, R = prm.R, M = prm.M, NQ = prm.T + 1;
  // NR <= NRMAX (checked by the host); NR == NRMAX when FULL
  const int NR = FULL ? NRMAX : (B + 15) / 16, NTILE = NR * (NR + 1) / 2;
  double* yb = ldsd;                                         // [KQ][BT]
  double2* sc = reinterpret_cast<double2*>(yb + KQ * BT);    // [R][NQ] (cos, sin) of k 2 pi r / R
  const int t = threadIdx.x, row = t % BT, lane = t % 64;
  const int h = __builtin_amdgcn_readfirstlane(t / BT);      // BT is a multiple of 64: one h per wave
  const int wv = __builtin_amdgcn_readfirstlane(t / 64);
  const int64_t nchunks = prm.scal[1], ch = prm.scal[0];
  const int c = blockIdx.x;
  if (c >= nchunks) return;
  // atom of this chunk: last m with chunk[m] <= c
  int lo = 0, hi = M - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prm.chunk[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  const int m = lo;
  const int64_t q0 = prm.bucket[m] + int64_t(c - prm.chunk[m]) * ch;
  const int64_t q1 = q0 + ch < prm.bucket[m + 1] ? q0 + ch : prm.bucket[m + 1];
  for (int i = t; i < R * NQ; i += NT) {
    const int r = i / NQ, k = i - r * NQ;
    sc[i] = double2{prm.cs64[k * R + r], prm.cs64[(NQ + k) * R + r]};
  }
  const Coord cd = coord_of(row < B ? row : 0, prm.hb);
  const int rowc = row < B ? row : 0;
  const double dm = row < B ? double(prm.dict[size_t(m) * B + row]) : 0.0;
  const double sig = cd.part == 0 ? -1.0 : 1.0;   // turning back by -r0

  // Loads from indices clamped into the chunk: issued without a branch, masked where
  // consumed (k < nq).
  auto clampq = [&](int64_t i) { return i < q1 ? i : q1 - 1; };
  // Pair records (patch, r0, c) of a batch: lane kk of each wave loads pair h KP + kk (a
  // vector load: scalar loads would share the LDS wait counter and be waited for at
  // the first LDS access), and readlane broadcasts them.
  const int lk = lane % KP;
  int32_t pN, rN, pF, rF;   // records of the next batch and of the one after
  float cN, cF;
  auto fetch_rec = [&](int64_t qb, int32_t& pp, int32_t& rr, float& cc) {
    const int64_t i = clampq(qb + h * KP + lk);
    pp = prm.lp[i];
    rr = prm.lr[i];
    cc = prm.lc[i];
  };
  double rv[KP], rp[KP];    // residual coordinates row and partner of this batch's pairs
  auto fetch_res = [&](int32_t pp, double* a, double* b) {
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
      const double* rr = prm.resid + int64_t(__builtin_amdgcn_readlane(pp, kk)) * BP;
      a[kk] = rr[rowc];
      b[kk] = rr[cd.partner];
    }
  };

  d4 acc[TW];
  int ta[TW], tb[TW];   // LDS offsets of this wave's tiles' row and column blocks (-1: no tile)
#pragma unroll
  for (int i = 0; i < TW; ++i) {
    acc[i] = d4{0.0, 0.0, 0.0, 0.0};
    const int u = wv + W * i;
    ta[i] = u < NTILE ? 16 * tile_r(u, NR) : -1;
    tb[i] = u < NTILE ? 16 * tile_s(u, NR) : -1;
  }
  int32_t rC;
  float cC;
  {
    int32_t pC;
    fetch_rec(q0, pC, rC, cC);
    fetch_rec(q0 + KQ, pN, rN, cN);
    fetch_res(pC, rv, rp);
  }
  __syncthreads();   // sc
  for (int64_t q = q0; q < q1; q += KQ) {
    const int nq = q1 - q < KQ ? int(q1 - q) : KQ;
    // y of this batch
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
      const int k = h * KP + kk;
      double y = 0.0;
      if (k < nq && row < B) {
        const int r0 = __builtin_amdgcn_readlane(rC, kk);
        const float c0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, cC), kk));
        const double2 cs = sc[(unsigned(r0) < unsigned(R) ? r0 : 0) * NQ + cd.k];
        y = fma(double(c0), dm, rot(rv[kk], rp[kk], cs.x, cs.y, sig));
      }
      yb[k * BT + row] = y;
    }
    // residual rows of the next batch, records of the one after
    fetch_res(pN, rv, rp);
    fetch_rec(q + 2 * KQ, pF, rF, cF);
    __syncthreads();
    // C += Y^T Y on the upper-triangle tiles: lane l supplies Y[4g + l / 16][16 r + l % 16]
    // as the A operand of tile row r and as the B operand of tile column r
    for (int g = 0; g < (nq + 3) / 4; ++g) {
      const double* yg = yb + (4 * g + lane / 16) * BT + lane % 16;
#pragma unroll
      for (int i = 0; i < TW; ++i)
        if (FULL || ta[i] >= 0) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(yg[ta[i]], yg[tb[i]], acc[i], 0, 0, 0);
    }
    __syncthreads();
    rC = rN;
    cC = cN;
    pN = pF;
    rN = rF;
    cN = cF;
  }
  // tile (r, s), lane l, register i holds C[16 r + l / 16 + 4 i][16 s + l % 16] (the FP64
  // 16 x 16 product's layout); the lower triangle is its mirror image
  double* out = prm.partial + size_t(c) * B * B;
#pragma unroll
  for (int i = 0; i < TW; ++i) {
    const int u = wv + W * i;
    if (u >= NTILE) continue;
    const int r = tile_r(u, NR), s2 = tile_s(u, NR);
    const int col = 16 * s2 + lane % 16;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int rr = 16 * r + lane / 16 + 4 * e;
      if (rr < B && col < B) {
        out[size_t(rr) * B + col] = acc[i][e];
        if (r != s2) out[size_t(col) * B + rr] = acc[i][e];
      }
    }
  }
}

// Sums each atom's chunk partials, in chunk order, into its first chunk's slot
// (thread per element: every element is read and written by one thread only).
__global__ __launch_bounds__(256) void rk_reduce_kernel(double* partial, const int32_t* chunk, int BB) {
  const int m = blockIdx.y;
  const int c0 = chunk[m], c1 = chunk[m + 1];
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c1 - c0 < 2 || i >= BB) return;
  double s = partial[size_t(c0) * BB + i];
#pragma unroll 8
  for (int c = c0 + 1; c < c1; ++c) s += partial[size_t(c) * BB + i];
  partial[size_t(c0) * BB + i] = s;
}

struct EigParams {
  const double* partial;  // [chunks][B][B]
  const int64_t* bucket;  // [M + 1]
  const int32_t* chunk;   // [M + 1]
  int M, B;
  const float* dict_old;  // [M][B] (rows of the old dictionary)
  float* d_new;           // [M][B]
  int32_t* usage;         // [M]
};

constexpr int kMaxSquarings = 40;

// Symmetric NP x NP matrices in LDS as their upper-triangle 16 x 16 tiles: tile (r, s),
// r <= s, is number r NR - r (r - 1) / 2 + (s - r) (the order of tile_r / tile_s), stored
// row-major with a row stride of kEigTS doubles (17: a tile's columns, read transposed for
// the lower triangle, then fall in distinct banks).  The diagonal tiles hold both halves.
constexpr int kEigTS = 17;
__device__ __forceinline__ int tile_index(int r, int s, int NR) { return r * NR - r * (r - 1) / 2 + (s - r); }
__device__ __forceinline__ double sym_at(const double* A, int i, int j, int NR) {
  const int bi = i >> 4, bj = j >> 4;
  return bi <= bj ? A[(tile_index(bi, bj, NR) * 16 + (i & 15)) * kEigTS + (j & 15)]
                  : A[(tile_index(bj, bi, NR) * 16 + (j & 15)) * kEigTS + (i & 15)];
}

__host__ __device__ inline size_t eig_lds_bytes(int B, int W) {
  const int NR = (B + 15) / 16;
  return sizeof(double) * (size_t(NR) * (NR + 1) / 2 * 16 * kEigTS + W + 16 * size_t(NR));
}

// Top eigenvector of one atom's C_m = Y_m Y_m^T (symmetric positive semidefinite), one
// block per atom, W waves.  C is scaled to unit trace and squared repeatedly,
// C <- C^2 / trace(C^2), on the FP64 matrix cores (16 x 16 tiles of the upper triangle of
// the zero-padded NP x NP matrix, NP = 16 ceil(B / 16) <= 16 NRMAX, kept in LDS as those
// tiles only; as C is symmetric, lane l's A operand of tile row r is
// C[4g + l/16][16r + l%16], the same pattern as its B operand).  With the eigenvalues of
// the scaled C written mu_i (sum 1), trace(C^2) = sum mu_i^2; it reaches 1 - 2 eps when the
// second share is eps, so the loop stops once 1 - trace(C^2) < 1e-14 (every other direction
// then carries a weight below 1e-14), or after kMaxSquarings.  The result is C d_old
// (or, if d_old has no component in that eigenspace, the column of largest diagonal),
// normalised and signed to agree with d_old.  A repeated top eigenvalue gives the
// projection of d_old onto its eigenspace.
template <int W, int NRMAX>
__global__ __launch_bounds__(64 * W) void rk_eig_kernel(EigParams prm) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int NT = 64 * W, TW = (NRMAX * (NRMAX + 1) / 2 + W - 1) / W;
  extern __shared__ double ldsd[];
  const int n = prm.B, m = blockIdx.x, t = threadIdx.x, lane = t % 64;
  const int wv = __builtin_amdgcn_readfirstlane(t / 64);
  const int NR = (n + 15) / 16, NP = 16 * NR, NTILE = NR * (NR + 1) / 2;   // NR <= NRMAX (host)
  double* A = ldsd;                          // [NTILE][16][kEigTS]
  double* red = A + NTILE * 16 * kEigTS;     // [W] reduction slots, then [NP] vector
  double* vec = red + W;
  const int used = int(prm.bucket[m + 1] - prm.bucket[m]);
  if (t == 0) prm.usage[m] = used;
  if (used == 0) {
    for (int i = t; i < n; i += NT) prm.d_new[size_t(m) * n + i] = prm.dict_old[size_t(m) * n + i];
    return;
  }
  // load C_m (the sum of its chunk partials sits in its first chunk's slot), zero padding
  const double* Cm = prm.partial + size_t(prm.chunk[m]) * n * n;
  for (int i = t; i < NTILE * 256; i += NT) {
    const int u = i >> 8, ii = (i >> 4) & 15, jj = i & 15;
    const int row = 16 * tile_r(u, NR) + ii, col = 16 * tile_s(u, NR) + jj;
    A[(u * 16 + ii) * kEigTS + jj] = row < n && col < n ? Cm[size_t(row) * n + col] : 0.0;
  }
  __syncthreads();   // the trace below reads diagonal entries other threads wrote
  // block sum in a fixed order: per wave a butterfly (identical bits in every lane),
  // then the W wave sums in wave order
  auto block_sum = [&](double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < W; ++i) s += red[i];
    return s;
  };
  double tr = 0.0;
  {
    double p = 0.0;
    for (int i = t; i < n; i += NT) p += sym_at(A, i, i, NR);
    tr = block_sum(p);
  }
  if (!(tr > 0.0)) {   // C_m = 0: nothing to fit
    for (int i = t; i < n; i += NT) prm.d_new[size_t(m) * n + i] = prm.dict_old[size_t(m) * n + i];
    return;
  }
  {
    const double sc = 1.0 / tr;
    for (int i = t; i < NTILE * 256; i += NT) A[(i >> 4) * kEigTS + (i & 15)] *= sc;
  }
  __syncthreads();
  int ta[TW], tb[TW];   // block row and column of this wave's tiles (-1: no tile)
#pragma unroll
  for (int i = 0; i < TW; ++i) {
    const int u = wv + W * i;
    ta[i] = u < NTILE ? tile_r(u, NR) : -1;
    tb[i] = u < NTILE ? tile_s(u, NR) : -1;
  }
  const int l16 = lane / 16, lc = lane % 16;
  for (int it = 0; it < kMaxSquarings; ++it) {
    d4 acc[TW];
#pragma unroll
    for (int i = 0; i < TW; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
    for (int g = 0; g < NP / 4; ++g) {
      // rows 4g .. 4g + 3 of C lie in row block kb (the same for the whole wave)
      const int kb = g >> 2, i0 = 4 * (g & 3) + l16;
      auto opnd = [&](int rb) {
        return kb <= rb ? A[(tile_index(kb, rb, NR) * 16 + i0) * kEigTS + lc]
                        : A[(tile_index(rb, kb, NR) * 16 + lc) * kEigTS + i0];
      };
#pragma unroll
      for (int i = 0; i < TW; ++i)
        if (ta[i] >= 0) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(opnd(ta[i]), opnd(tb[i]), acc[i], 0, 0, 0);
    }
    // trace of the square from the diagonal tiles: lane l register e holds row
    // 16r + l/16 + 4e, column 16r + l%16
    double p = 0.0;
#pragma unroll
    for (int i = 0; i < TW; ++i)
      if (ta[i] >= 0 && ta[i] == tb[i])
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (l16 + 4 * e == lc) p += acc[i][e];
    const double tr2 = block_sum(p);   // its barriers also end every read of A
    const double sc = 1.0 / tr2;
#pragma unroll
    for (int i = 0; i < TW; ++i) {
      if (ta[i] < 0) continue;
      double* tile = A + tile_index(ta[i], tb[i], NR) * 16 * kEigTS;
#pragma unroll
      for (int e = 0; e < 4; ++e) tile[(l16 + 4 * e) * kEigTS + lc] = acc[i][e] * sc;
    }
    __syncthreads();
    if (1.0 - tr2 < 1e-14) break;
  }
  // z = C d_old, or the column of largest diagonal when d_old misses the eigenspace
  for (int i = t; i < n; i += NT) vec[i] = double(prm.dict_old[size_t(m) * n + i]);
  __syncthreads();
  double zt = 0.0;
  if (t < n)
    for (int j = 0; j < n; ++j) zt += sym_at(A, t, j, NR) * vec[j];
  double nz = block_sum(t < n ? zt * zt : 0.0);
  if (!(nz > 1e-20)) {
    int jm = 0;
    for (int j = 1; j < n; ++j)
      if (sym_at(A, j, j, NR) > sym_at(A, jm, jm, NR)) jm = j;
    zt = t < n ? sym_at(A, t, jm, NR) : 0.0;
    nz = block_sum(t < n ? zt * zt : 0.0);
  }
  const double dot = block_sum(t < n ? zt * vec[t] : 0.0);
  double sgn = dot < 0.0 ? -1.0 : 1.0;
  if (dot == 0.0) {   // the largest-magnitude coordinate (the first on ties) is made positive
    __syncthreads();
    if (t < n) vec[t] = zt;
    __syncthreads();
    int im = 0;
    for (int i = 1; i < n; ++i)
      if (fabs(vec[i]) > fabs(vec[im])) im = i;
    sgn = vec[im] < 0.0 ? -1.0 : 1.0;
  }
  if (t < n) prm.d_new[size_t(m) * n + t] = float(sgn * zt / sqrt(nz));
}

struct ResetParams {
  const float* xhat;
  const float* resid2;
  int64_t P;
  int M, B;
  const int32_t* usage;
  float* d_new;
  int32_t* reset;   // [M] patch an unused atom was reset to, -1 otherwise
};

__global__ __launch_bounds__(256) void rk_reset_kernel(ResetParams prm) {
  __shared__ float bv[256];
  __shared__ long long bi[256];
  __shared__ long long chosen[256];
  __shared__ double nrm[256];
  const int t = threadIdx.x;
  int nchosen = 0;
  for (int m = t; m < prm.M; m += 256) prm.reset[m] = -1;
  __syncthreads();
  for (int m = 0; m < prm.M; ++m) {
    if (prm.usage[m] > 0) continue;
    // largest coding error among the patches not chosen yet (ties: smaller index)
    float best = 0.f;
    long long bp = -1;
    for (int64_t p = t; p < prm.P; p += 256) {
      const float r = prm.resid2[p];
      if (!(r > best)) continue;
      bool taken = false;
      for (int i = 0; i < nchosen; ++i) taken = taken || chosen[i] == p;
      if (!taken) {
        best = r;
        bp = p;
      }
    }
    bv[t] = best;
    bi[t] = bp;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) {
        const bool take = bv[t + s] > bv[t] || (bv[t + s] == bv[t] && bi[t + s] >= 0 &&
                                                (bi[t] < 0 || bi[t + s] < bi[t]));
        if (take) {
          bv[t] = bv[t + s];
          bi[t] = bi[t + s];
        }
      }
      __syncthreads();
    }
    const long long p = bi[0];
    __syncthreads();
    if (p < 0) break;                 // no patch with a positive error is left
    const float x = t < prm.B ? prm.xhat[p * prm.B + t] : 0.f;
    nrm[t] = double(x) * x;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) nrm[t] += nrm[t + s];
      __syncthreads();
    }
    const double n2 = nrm[0];
    if (t < prm.B) prm.d_new[size_t(m) * prm.B + t] = float(double(x) / sqrt(n2));
    if (t == 0) prm.reset[m] = int32_t(p);
    if (t == 0) chosen[nchosen] = p;
    ++nchosen;
    __syncthreads();
    if (nchosen == 256) break;
  }
}

// Sum of a float array in FP64 for the coding-error history, in two fixed-order
// stages: kSumBlocks block sums of contiguous ranges into out[1..], then their sum
// into out[0].
__device__ __forceinline__ double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  return red[0];
}

__global__ __launch_bounds__(256) void rk_sum_part_kernel(const float* x, int64_t n, double* out) {
  __shared__ double red[256];
  const int64_t per = (n + kSumBlocks - 1) / kSumBlocks;
  const int64_t i0 = int64_t(blockIdx.x) * per, i1 = i0 + per < n ? i0 + per : n;
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) s += x[i];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) out[1 + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void rk_sum_final_kernel(double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < kSumBlocks; i += 256) s += out[1 + i];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

}  // namespace

bool rksvd_fits(const DeviceTables& t) {
  if (t.B < 1 || t.B > kRkMaxB) return false;
  const size_t lim = 160 * 1024;
  const size_t table = sizeof(double) * 2 * size_t(t.R) * (t.T + 1);
  // the single-value form, plus the partner table in static LDS
  const size_t resid = table + sizeof(float) * size_t(t.M) * t.B + sizeof(int) * kRkMaxB;
  const int bt = t.B <= 64 ? 64 : t.B <= 128 ? 128 : 192;
  const size_t acc = sizeof(double) * (16 * size_t(bt) + 2 * size_t(t.T + 1) * t.R);
  return resid <= lim && acc <= lim && eig_lds_bytes(t.B, 8) <= lim;
}

size_t rksvd_workspace_bytes(const DeviceTables& t, int64_t P, int K) {
  return rk_ws(t.M, t.B, P, K).total + al256(sizeof(double) * kSumSlots);
}

int launch_rksvd_update(const DeviceTables& t, const float* xhat, int64_t P, int K, const int32_t* atom,
                        const int32_t* angle, const float* coef, const float* resid2, void* ws,
                        float* d_new, int32_t* usage, int32_t* reset, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const RkWs L = rk_ws(t.M, t.B, P, K);
  char* w = reinterpret_cast<char*>(ws);
  SortParams sp{atom, angle, coef, P, K, t.M, reinterpret_cast<int64_t*>(w + L.cnt),
                reinterpret_cast<int64_t*>(w + L.off), reinterpret_cast<int64_t*>(w + L.tot),
                reinterpret_cast<int64_t*>(w + L.bucket), reinterpret_cast<int32_t*>(w + L.chunk),
                reinterpret_cast<int64_t*>(w + L.scal), reinterpret_cast<int32_t*>(w + L.lp),
                reinterpret_cast<int32_t*>(w + L.lr), reinterpret_cast<float*>(w + L.lc)};
  hipLaunchKernelGGL(rk_count_kernel, dim3(kSortBlocks), dim3(256), sizeof(int) * t.M, st, sp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return int(e);
  hipLaunchKernelGGL(rk_scan_kernel, dim3(unsigned(t.M)), dim3(256), 0, st, sp);
  e = hipGetLastError();
  if (e != hipSuccess) return int(e);
  hipLaunchKernelGGL(rk_plan_kernel, dim3(1), dim3(256), 0, st, sp);
  e = hipGetLastError();
  if (e != hipSuccess) return int(e);
  hipLaunchKernelGGL(rk_scatter_kernel, dim3(kSortBlocks), dim3(64), 2 * sizeof(int64_t) * t.M, st, sp);
  e = hipGetLastError();
  if (e != hipSuccess) return int(e);
  double* partial = reinterpret_cast<double*>(w + L.partial);
  double* resid = reinterpret_cast<double*>(w + L.resid);
  const int BP = resid_stride(t.B);
  HarmBlocks hb{};
  hb.T = t.T;
  hb.kb[0] = 0;
  hb.kb[1] = t.sk[0];
  for (int k = 1; k <= t.T; ++k) hb.kb[k + 1] = hb.kb[k] + 2 * t.sk[k];
  ResidParams qp{xhat, atom, angle, coef, t.dictHat, t.cs64, P, K, t.M, t.R, t.B, BP, t.T, hb, resid};
  {
    const int G = 256 / BP, nt = G * BP;
    const size_t table = sizeof(double) * 2 * size_t(t.R) * (t.T + 1);
    const bool paired = table + sizeof(float) * 2 * size_t(t.M) * t.B <= kResidLdsPaired;
    const size_t lds = table + sizeof(float) * (paired ? 2 : 1) * size_t(t.M) * t.B;
    auto kern = paired ? (K <= 4 ? rk_resid_kernel<4, true> : rk_resid_kernel<8, true>)
                       : (K <= 4 ? rk_resid_kernel<4, false> : rk_resid_kernel<8, false>);
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return int(e);
    // one resident round of blocks: every block fills its LDS with the dictionary once, so
    // more blocks than fit at a time would only repeat that fill
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    const int64_t want = (P + G - 1) / G, cap = int64_t(num_cus()) * per_cu;
    const unsigned grid = unsigned(want < cap ? want : cap);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(nt), lds, st, qp);
    e = hipGetLastError();
    if (e != hipSuccess) return int(e);
  }
  AccParams ap{resid,     BP,       t.M,     t.R,   t.B,   t.T,  hb,   t.dictHat, t.cs64,
               sp.bucket, sp.chunk, sp.scal, sp.lp, sp.lr, sp.lc, partial};
  EigParams ep{partial, sp.bucket, sp.chunk, t.M, t.B, t.dictHat, d_new, usage};
  const int NQ = t.T + 1;
  const int64_t nblk = max_chunks(t.M, P, K);
  auto run = [&](auto acc_kern, auto eig_kern, int bt, int nt, int kq, int eig_threads) -> int {
    const size_t lds1 = sizeof(double) * (size_t(kq) * bt + 2 * size_t(NQ) * t.R);
    const size_t lds2 = eig_lds_bytes(t.B, 8);
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(acc_kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, int(lds1));
    if (err == hipSuccess)
      err = hipFuncSetAttribute(reinterpret_cast<const void*>(eig_kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                int(lds2));
    if (err != hipSuccess) return int(err);
    // one block per chunk; blocks past the plan's count return at once
    hipLaunchKernelGGL(acc_kern, dim3(unsigned(nblk)), dim3(nt), lds1, st, ap);
    err = hipGetLastError();
    if (err != hipSuccess) return int(err);
    const int BB = t.B * t.B;
    hipLaunchKernelGGL(rk_reduce_kernel, dim3(unsigned((BB + 255) / 256), unsigned(t.M)), dim3(256), 0, st, partial,
                       sp.chunk, BB);
    err = hipGetLastError();
    if (err != hipSuccess) return int(err);
    hipLaunchKernelGGL(eig_kern, dim3(unsigned(t.M)), dim3(eig_threads), lds2, st, ep);
    return int(hipGetLastError());
  };
  if (t.B > kRkMaxB) return int(hipErrorInvalidValue);
  // 49..64 (the 11x11 grid, B = 55) fills the fourth row block: the tile loop needs no test;
  // any other B up to 128 (the 15x15 grid, the annular basis at N = 11) takes the general
  // 128-row form, B up to 160 (the annular basis at N = 15) the 192-row one
  const int r = t.B > 48 && t.B <= 64
                    ? run(rk_accum_kernel<64, 2, 16, 4, true>, rk_eig_kernel<4, 4>, 64, 128, 16, 256)
                : t.B <= 128 ? (t.B <= 64 ? run(rk_accum_kernel<128, 4, 16, 8, false>, rk_eig_kernel<4, 4>, 128, 256, 16, 256)
                                          : run(rk_accum_kernel<128, 4, 16, 8, false>, rk_eig_kernel<8, 8>, 128, 256, 16, 512))
                             : run(rk_accum_kernel<192, 6, 16, 10, false>, rk_eig_kernel<8, 10>, 192, 384, 16, 512);
  if (r) return r;
  ResetParams rp{xhat, resid2, P, t.M, t.B, usage, d_new, reset};
  hipLaunchKernelGGL(rk_reset_kernel, dim3(1), dim3(256), 0, st, rp);
  return int(hipGetLastError());
}

int launch_sum(const float* x, int64_t n, double* out, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(rk_sum_part_kernel, dim3(kSumBlocks), dim3(256), 0, st, x, n, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return int(e);
  hipLaunchKernelGGL(rk_sum_final_kernel, dim3(1), dim3(256), 0, st, out);
  return int(hipGetLastError());
}

}  // namespace rsc
