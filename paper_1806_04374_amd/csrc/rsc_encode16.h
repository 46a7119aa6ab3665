// Shared by the encoder translation units: the launch parameters, the code output and
// the 16x16-tile encoder (encode16_kernel), templated on the per-harmonic profile counts
// of the coordinate layout (LayoutBase), so that the (S, T) grid of Gaussian profiles
// and the paper's annular basis are instantiated in separate files.
#pragma once

#include <hip/hip_runtime.h>

#include "rsc_device.h"
#include "rsc_internal.h"

namespace rsc {
namespace enc {

struct EncodeParams {
  const float* xhat;
  int64_t P;
  int K, M, R;
  const float* dictA;     // encode32 stage-1 operand [NG][NKS][64]
  const float* dictHat;   // [NG8*8 or NG*16][B]
  const float* dftA;      // stage-2 operand (layout per tile shape)
  const float* cs;        // [2][T+1][R]
  const float* gramH;     // [M][M][2T+1] per-pair harmonic inner products
  const double* gramH64;  // the same in FP64 (FP64 re-solve)
  const double* cs64;     // [2][T+1][R] in FP64
  int32_t* atom;
  int32_t* angle;
  float* coef;
  float* resid2;
  unsigned long long* stats;   // [4]: [3] counts pursuit steps solved in FP64
  const float* dictHatI;       // i * dictionary rows, as dictHat (16x16 tile with IROWS; else unused)
};

// Adds this wave's count of FP64 least-squares steps to stats[3] (one atomic per wave).
__device__ __forceinline__ void count_fp64(unsigned long long* stats, unsigned n, int lane) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) n += __shfl_xor(n, off);
  if (lane == 0 && stats && n) atomicAdd(stats + 3, (unsigned long long)n);
}

template <class L, int KMAX>
__device__ __forceinline__ void write_codes(const EncodeParams& prm, int64_t p, const PursuitState<KMAX>& st,
                                            float rn2) {
  const int K = prm.K;
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    if (i < K) {
      const bool s = i < st.nsel;
      prm.atom[p * K + i] = s ? st.selm[i] : -1;
      prm.angle[p * K + i] = s ? st.selr[i] : -1;
      prm.coef[p * K + i] = s ? st.cf[i] : 0.f;
    }
  }
  if (prm.resid2) prm.resid2[p] = rn2;
}

// Complex harmonic products C_k = sum_s conj(d_{m,s,k}) x_{s,k} of atom m for this lane's
// patch in the quarter-wave layout (W = 4), complete in all four lanes of the patch:
// cre[k], cim[k].  Lane u holds profiles 4j + u of harmonic 0 and, for k >= 1, profile
// 2jj + (u >> 1) of part u & 1 (0: Re, 1: Im); each lane multiplies its coordinates with the
// matching parts of the atom and two exchanges complete the sums.  Padding coordinates of
// the residual are 0, so what the atom row holds there does not matter.
template <class L>
__device__ __forceinline__ void atom_products4(const float* __restrict__ hat, int m, int u,
                                               const float (&res)[L::NKS], float (&cre)[L::NQ],
                                               float (&cim)[L::NQ]) {
  static_assert(L::W == 4, "four quarter-waves per patch");
  const float* d = hat + m * L::B;
  float p0 = 0.f;
#pragma unroll
  for (int j = 0; j < L::J0; ++j) {
    const int s = 4 * j + u;
    p0 = fmaf(d[s < L::S ? s : 0], res[j], p0);
  }
  cre[0] = p0;
  cim[0] = 0.f;
  const int part = u & 1, so = u >> 1;
  static_for<L::T>([&](auto K1) {
    constexpr int k = decltype(K1)::value + 1;
    constexpr int bk = L::base(k), nk = L::Sk(k), j0 = L::joff(k), nj = L::J1k(k);
    // part 0 (x = Re): Re += dRe x, Im -= dIm x; part 1 (x = Im): Re += dIm x, Im += dRe x
    const float* dA = d + bk + (part ? nk : 0);
    const float* dB = d + bk + (part ? 0 : nk);
    const float sb = part ? 1.f : -1.f;
    float pr = 0.f, pi = 0.f;
#pragma unroll
    for (int jj = 0; jj < nj; ++jj) {
      const int s = 2 * jj + so;
      const int o = s < nk ? s : 0;
      pr = fmaf(dA[o], res[j0 + jj], pr);
      pi = fmaf(dB[o], res[j0 + jj], pi);
    }
    cre[k] = pr;
    cim[k] = sb * pi;
  });
#pragma unroll
  for (int k = 0; k < L::NQ; ++k) {
    cre[k] = cre[k] + __shfl_xor(cre[k], 16);
    cre[k] = cre[k] + __shfl_xor(cre[k], 32);
    cim[k] = cim[k] + __shfl_xor(cim[k], 16);
    cim[k] = cim[k] + __shfl_xor(cim[k], 32);
  }
}

// ============================================================== 16x16 tiles
// SPLIT (even R): each stage-2 step contracts a pair of harmonics of one parity,
// (4j, 4j+2) for E and (4j+1, 4j+3) for O; HT tiles of 16 angle rows cover r < R/2.
// dftA: [HT][SE + SO][64] (E steps first).
// Direct (odd R): steps contract harmonic pairs (2q, 2q+1); HT tiles cover r < R.
// dftA: [HT][NP][64].
// C: the profile counts per harmonic (LayoutBase): the (S, T) grid or the annular basis.
// IROWS: the stage-1 Im rows read i * d (dictHatI, a second LDS table) at the offsets where
// the Re rows read d, so no lane applies a sign; without it (dictionaries too large for two
// tables) the Im rows negate what they read.  Blocks of 4 or 8 waves (256 or 512 threads;
// with 8, one block per CU shares the tables).
template <class C, int HT, int KMAX, bool SPLIT, bool IROWS>
__global__ __launch_bounds__(IROWS ? 512 : 256, 2) void encode16_kernel(EncodeParams prm) {
  using L = LayoutBase<C, 4>;
  const int NW = int(blockDim.x) >> 6;                       // waves per block (4 or 8)
  constexpr int NKS = L::NKS, NQ = L::NQ, B = L::B, T = L::T;
  constexpr int NE = T / 2 + 1, NO = (T + 1) / 2;           // even / odd harmonics
  constexpr int SE = SPLIT ? (NE + 1) / 2 : (NQ + 1) / 2;   // steps feeding the E (or only) chain
  constexpr int SO = SPLIT ? (NO + 1) / 2 : 0;              // steps feeding the O chain
  constexpr int NS = SE + SO;
  extern __shared__ float lds[];
  const int R = prm.R, M = prm.M, K = prm.K, HALF = SPLIT ? prm.R / 2 : prm.R;
  const int NG = (M + 7) / 8;
  float* sHat = lds;                              // [NG*8][B]
  float* sHatI = sHat + (IROWS ? NG * 8 * B : 0);  // [NG*8][B] with IROWS
  float* sCs = sHatI + NG * 8 * B;                // [2][NQ][R]
  {
    const int nH = NG * 8 * B, nC = 2 * NQ * R;
    for (int i = threadIdx.x; i < nH; i += blockDim.x) sHat[i] = prm.dictHat[i];
    if (IROWS)
      for (int i = threadIdx.x; i < nH; i += blockDim.x) sHatI[i] = prm.dictHatI[i];
    for (int i = threadIdx.x; i < nC; i += blockDim.x) sCs[i] = prm.cs[i];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, u = lane >> 4;
  const LsTables tb{prm.gramH, prm.gramH64, prm.cs64, prm.xhat, M, R, kCondMaxFp32};
  unsigned n64 = 0;
  // stage-1 operand row of this lane: rows 0-3 Re of atoms 0-3, 4-7 Im of atoms 0-3,
  // 8-11 Re of atoms 4-7, 12-15 Im of atoms 4-7; contraction index 4j+u
  const int arow = lane & 15;
  const int a_of_row = (arow & 3) + 4 * (arow >> 3);
  const bool is_im = (arow >> 2) & 1;
  const int part = u & 1;
  // without IROWS: the Im rows read the partner part of d (Re <-> Im), negated for x's Re part
  const bool other = IROWS ? bool(part) : bool(part ^ int(is_im));
  const float sgn = (!IROWS && is_im && part == 0) ? -1.f : 1.f;
  const float* arow_hat = (IROWS && is_im ? sHatI : sHat) + a_of_row * B;

  float F[HT][NS];
#pragma unroll
  for (int t = 0; t < HT; ++t)
#pragma unroll
    for (int q = 0; q < NS; ++q) F[t][q] = prm.dftA[(t * NS + q) * 64 + lane];

  // harmonics contracted by step q: (k1, k2)
  auto k1_of = [](int q) { return SPLIT ? (q < SE ? 4 * q : 4 * (q - SE) + 1) : 2 * q; };
  auto k2_of = [](int q) { return SPLIT ? (q < SE ? 4 * q + 2 : 4 * (q - SE) + 3) : 2 * q + 1; };

  const int64_t nwt = (prm.P + 15) / 16;
  for (int64_t wt = int64_t(blockIdx.x) * NW + wave; wt < nwt; wt += int64_t(gridDim.x) * NW) {
    const int64_t p = wt * 16 + col;
    const bool valid = p < prm.P;
    float res[NKS];
    static_for<NKS>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const int c = L::template coord_u<j>(u);
      res[j] = (valid && c >= 0) ? prm.xhat[p * B + c] : 0.f;
    });
    const float nx2 = norm2<L>(res);
    PursuitState<KMAX> st;
    init_state(st, valid);
    LsState<KMAX> ls;
    init_ls(ls);

    for (int it = 0; it < K; ++it) {
      st.active = st.active && (norm2<L>(res) > kTau2 * nx2);
      if (!__any(st.active)) break;

      // pass 1: every atom's maximum over its angles.  Four atoms at a time are reduced over
      // the quarter-waves with two exchanges per pair, leaving one atom per quarter; each
      // quarter keeps its own best atom (first on equal maxima, atoms in increasing order),
      // and the quarters are compared once per step.
      float bq = -1.f;
      int aq = 0;
      const int qperm = ((u & 1) << 1) | (u >> 1);   // atom of this quarter within a batch of 4
      for (int g = 0; g < NG; ++g) {
        const float* hg = arow_hat + g * 8 * B;
        f32x4 acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
        static_for<NKS>([&](auto J) {
          constexpr int j = decltype(J)::value;
          constexpr int k = L::harm(j);
          // A lane past its harmonic's count (a padding coordinate, at most three past
          // harmonic 0's and one past any other's) reads the next values of the row, or of
          // the next row (after the last row of a table comes the other table or the angle
          // table): finite values that meet a residual coordinate held at exactly 0.
          float av;
          if constexpr (k == 0) {
            if constexpr (IROWS) {
              av = hg[4 * j + u];                             // i * d is 0 at harmonic 0
            } else {
              const float h = hg[4 * j + u];
              av = is_im ? 0.f : h;                           // the Im rows of harmonic 0 are 0
            }
          } else {
            constexpr int jj = L::pair(j), bk = L::base(k), sk = L::Sk(k);
            const int off = bk + 2 * jj + (u >> 1) + (other ? sk : 0);
            if constexpr (IROWS) {
              av = hg[off];
            } else {
              av = sgn * hg[off];
            }
          }
          acc[k] = mfma16(av, res[j], acc[k]);
        });
        // quarters 0,1 hold (Re, Im) of atom v, quarters 2,3 of atom v+4.  Swapping
        // harmonics (k1, k2) of a step gives the operand [Re_k1 Im_k1 Re_k2 Im_k2]
        // of atoms v and v+4, kept in place: atom a < 4 in acc[k1][a], atom a >= 4 in
        // acc[k2][a-4] (or pad[q][a-4] when k2 > T).
        float pad[NS][4];
#pragma unroll
        for (int q = 0; q < NS; ++q)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int k1 = k1_of(q), k2 = k2_of(q);
            float x = acc[k1][v];
            float y = k2 <= T ? acc[k2][v] : 0.f;
            swap32(x, y);
            acc[k1][v] = x;
            if (k2 <= T) acc[k2][v] = y;
            pad[q][v] = y;
          }
        auto opnd = [&](int q, int a) -> float {
          const int k1 = k1_of(q), k2 = k2_of(q);
          return a < 4 ? acc[k1][a] : (k2 <= T ? acc[k2][a - 4] : pad[q][a - 4]);
        };
        // per atom: HT tiles x (E, O) chains; the chains of the next atom are issued
        // before the reduction of the current one.  Atoms past M have all-zero operands:
        // their maxima are exactly 0 and lose every tie to a smaller atom.
        f32x4 ob[2][2][HT];
        auto chains = [&](int a, f32x4 (&o)[2][HT]) {
#pragma unroll
          for (int t = 0; t < HT; ++t) o[0][t] = o[1][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < NS; ++q)
#pragma unroll
            for (int t = 0; t < HT; ++t) {
              const int c = q < SE ? 0 : 1;
              o[c][t] = mfma16(F[t][q], opnd(q, a), o[c][t]);
            }
        };
        float amq[8];   // this lane's part of each atom's maximum (its four angle rows per tile)
        chains(0, ob[0]);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          if (a + 1 < 8) chains(a + 1, ob[(a + 1) & 1]);
          const f32x4 (&o)[2][HT] = ob[a & 1];
          float am = 0.f;
#pragma unroll
          for (int t = 0; t < HT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i)
              am = fmaxf(am, SPLIT ? fabsf(o[0][t][i]) + fabsf(o[1][t][i]) : fabsf(o[0][t][i]));
          amq[a] = am;
        }
        // atoms (4b, 4b+1) and (4b+2, 4b+3): one exchange of the half-waves per pair, then
        // one of the odd and even rows, leaves atom 4b + qperm's maximum in quarter u
        // (non-negative floats compared as integers)
        auto umax = [](float x, float y) { return __uint_as_float(max(__float_as_uint(x), __float_as_uint(y))); };
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          float x0 = amq[4 * b], y0 = amq[4 * b + 1], x1 = amq[4 * b + 2], y1 = amq[4 * b + 3];
          swap32(x0, y0);
          swap32(x1, y1);
          float v = umax(x0, y0), w = umax(x1, y1);
          swap16(v, w);
          const float mx = umax(v, w);
          const bool gt = mx > bq;
          bq = gt ? mx : bq;
          aq = gt ? g * 8 + 4 * b + qperm : aq;
        }
      }
      // the best atom over the quarters: the larger maximum, the smaller atom on equal ones
      int bm;
#pragma unroll
      for (int sh = 16; sh <= 32; sh *= 2) {
        const float ob2 = __shfl_xor(bq, sh);
        const int oa = __shfl_xor(aq, sh);
        const bool take = (ob2 > bq) || (ob2 == bq && oa < aq);
        bq = take ? ob2 : bq;
        aq = take ? oa : aq;
      }
      bm = aq;
      // pass 2: the winner's stage-2 operand formed again from its dictionary row, then its
      // angles
      int rs;
      float cval;
      {
        float cre[NQ], cim[NQ];
        atom_products4<L>(sHat, bm, u, res, cre, cim);
        float bop[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const int k1 = k1_of(q), k2 = k2_of(q);
          const float re2 = k2 <= T ? cre[k2 <= T ? k2 : 0] : 0.f, im2 = k2 <= T ? cim[k2 <= T ? k2 : 0] : 0.f;
          bop[q] = u == 0 ? cre[k1] : u == 1 ? cim[k1] : u == 2 ? re2 : im2;
        }
        f32x4 o[2][HT];
#pragma unroll
        for (int t = 0; t < HT; ++t) o[0][t] = o[1][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < NS; ++q)
#pragma unroll
          for (int t = 0; t < HT; ++t) {
            const int c = q < SE ? 0 : 1;
            o[c][t] = mfma16(F[t][q], bop[q], o[c][t]);
          }
        // Rows past HALF have all-zero operand rows, so their scores are exactly 0.  A lane
        // reaches them after its valid rows (its rows ascend), and a 0 never beats an earlier
        // value under the strict '>'; a quarter with no valid row ends with 0 at an index of
        // at least HALF, which loses the cross-quarter tie to a valid row (row 0 always is).
        // So no row mask is needed.
        float rb = -1.f, rv = 0.f;
        int rc = 0;
#pragma unroll
        for (int h = 0; h < (SPLIT ? 2 : 1); ++h)   // angles r < R/2 first, then r + R/2
#pragma unroll
          for (int t = 0; t < HT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int row = 16 * t + 4 * u + i;
              const float sc = SPLIT ? (h == 0 ? o[0][t][i] + o[1][t][i] : o[0][t][i] - o[1][t][i]) : o[0][t][i];
              const float val = fabsf(sc);
              const bool gt = val > rb;
              rb = gt ? val : rb;
              rv = gt ? sc : rv;
              rc = gt ? row + h * HALF : rc;
            }
#pragma unroll
        for (int sh = 16; sh <= 32; sh *= 2) {
          const float ob2 = __shfl_xor(rb, sh), ov = __shfl_xor(rv, sh);
          const int oc = __shfl_xor(rc, sh);
          const bool take = (ob2 > rb) || (ob2 == rb && oc < rc);
          rb = take ? ob2 : rb;
          rv = take ? ov : rv;
          rc = take ? oc : rc;
        }
        rs = rc < R ? rc : R - 1;
        cval = rv;
      }
      n64 += (ls_update<L, KMAX>(st, ls, it, bm, rs, cval, sHat, sCs, tb, p, u, res) && u == 0) ? 1u : 0u;
    }
    const float rn2 = norm2<L>(res);
    if (valid && u == 0) write_codes<L, KMAX>(prm, p, st, rn2);
  }
  count_fp64(prm.stats, n64, lane);
}

}  // namespace enc
}  // namespace rsc
