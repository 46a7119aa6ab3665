// Rotational OMP with 16-bit correlation (BF16 or FP16 operands, FP32 accumulation)
// and an FP32 re-score of the candidates: the precision form of the pursuit of
// Fig. 2 with rotations replaced by steering (Sec. II-C, eq. (8); Sec. II-E step 3).
//
// Each wave owns 32 patches (MFMA columns).  Per pursuit step:
//   stage 1, v_mfma_f32_32x32x16_{bf16,f16}: C_k = sum_s conj(d_{m,s,k}) x_{s,k} for 16
//     atoms at once, one instruction per harmonic k.  Rows are (atom, Re/Im); the
//     contraction runs over the residual's harmonic-k block, whose Re parts sit in
//     the low half-wave and Im parts in the high half-wave (Layout<S, T, 2>).
//     Accumulator register a then holds Re C_k of atom a in the low half-wave and
//     Im C_k in the high half-wave.
//   stage 2, same instruction: per atom and per 32 angles, rows = angles, the
//     contraction slots 0..T of the low half-wave take (cos k theta_r, Re C_k) and
//     those of the high half-wave (-sin k theta_r, Im C_k).  Only the largest
//     |score| of each atom over its angles is kept.
//   candidates: atoms whose 16-bit maximum lies within 4u ||r|| of the largest one
//     (u: unit roundoff of the 16-bit format).  The 16-bit scores stay well inside
//     +-u ||r|| of the exact ones on the workloads here, so the atom with the exact
//     maximum is among them; each half-wave keeps a bit mask of its atoms and its
//     own running maximum, and a new maximum more than the window above the old one
//     clears the mask.
//   FP32 re-score: per candidate, C_k in FP32 from the packed dictionary (each lane
//     its half of the coordinates, a half-wave swap completes the sums) and the
//     angle DFT on v_mfma_f32_32x32x2f32; the best candidate by exact maximum, then
//     its angles again with the same instructions for the argmax.  Candidates are
//     visited in increasing atom order, so ties go to the smallest atom, then angle.
//   least squares: the Cholesky-based update of the FP32 encoders.  It also tracks
//     k ||L^{-1}||_F^2, an upper bound on cond_2 of the Gram matrix of the k
//     selected unit columns; once that bound exceeds 1e6 (or the new pivot is tiny)
//     the patch's least squares are re-solved from scratch in FP64 for this and every
//     later step: FP64 Gram from an FP64 pair table, FP64 Cholesky, <column, x_hat>
//     from the input coordinates, residual x_hat - sum a_i column_i.
#include <hip/hip_runtime.h>

#include "rsc_device.h"
#include "rsc_internal.h"
#include "rsc_launch.h"
#include "rsc_lp.h"

namespace rsc {
namespace {

struct LpParams {
  const float* xhat;
  int64_t P;
  int K, M, R;
  const uint4* dictA;      // stage-1 operand [NG][T+1][64] x 8 16-bit values
  const float* dictHat;    // [16 NG][B]
  const uint4* dft16;      // stage-2 operand [RT][64] x 8 16-bit values
  const float* dft32;      // FP32 re-score operand [RT][T+1][64]
  const float* cs;         // [2][T+1][R]
  const float* gramH;      // [M][M][2T+1]
  const double* gramH64;   // [M][M][2T+1]
  const double* cs64;      // [2][T+1][R]
  int32_t* atom;
  int32_t* angle;
  float* coef;
  float* resid2;
  unsigned long long* stats;   // [4], see rsc_precision_stats
};

// <S_{ra} d_a, S_{rb} d_b> in FP64 (same table layout as pair_gram).
template <int T>
__device__ __forceinline__ double pair_gram64(const double* __restrict__ H, const double* __restrict__ cs,
                                              int M, int R, int a, int ra, int b, int rb) {
  const double* h = H + (size_t(a) * M + b) * (2 * T + 1);
  int dr = ra - rb;
  dr += dr < 0 ? R : 0;
  double g = h[0];
#pragma unroll
  for (int k = 1; k <= T; ++k) g += cs[k * R + dr] * h[2 * k - 1] - cs[(T + 1 + k) * R + dr] * h[2 * k];
  return g;
}

// Coordinate j (of sub-lane u) of S_r d_m in FP64; 0 for padding.
template <class L>
__device__ __forceinline__ double steer64(const float* __restrict__ hat, const double* __restrict__ cs, int R,
                                          int m, int r, int j, int u) {
  const float* d = hat + m * L::B;
  const int k = L::harm(j), pr = L::prof(j, u);
  if (pr >= L::S) return 0.0;
  if (k == 0) return double(d[pr]);
  const double c = cs[k * R + r], s = cs[(L::NQ + k) * R + r];
  const double ca = L::part(u) ? -s : c, cb = L::part(u) ? c : s;
  return double(d[L::base(k) + pr]) * ca + double(d[L::base(k) + L::S + pr]) * cb;
}

// FP64 least squares over the it selected columns plus (ms, rs), for the lanes with
// go set.  Returns whether the new column was accepted (its FP64 pivot is not
// negligible); then the coefficients, the selection and the residual are replaced.
template <class L, int KMAX>
__device__ __forceinline__ bool lp_solve64(PursuitState<KMAX>& st, int it, int ms, int rs, bool go, const float* hat,
                           const LpParams& prm, int64_t p, int u, float (&res)[L::NKS]) {
  const int M = prm.M, R = prm.R;
  int cm[KMAX], cr[KMAX];
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    cm[i] = i < it ? (st.selm[i] < 0 ? 0 : st.selm[i]) : ms;
    cr[i] = i < it ? (st.selr[i] < 0 ? 0 : st.selr[i]) : rs;
  }
  double Lc[KMAX][KMAX];
  bool good = go;
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      if (i <= it) {
        const double g0 = pair_gram64<L::T>(prm.gramH64, prm.cs64, M, R, cm[i], cr[i], cm[j], cr[j]);
        double g = g0;
#pragma unroll
        for (int l = 0; l < j; ++l) g -= Lc[i][l] * Lc[j][l];
        if (j < i) {
          Lc[i][j] = g / Lc[j][j];
        } else {
          if (i == it) good = good && g > 1e-14 * g0;
          Lc[i][i] = sqrt(g > 1e-300 ? g : 1e-300);
        }
      } else {
        Lc[i][j] = j == i ? 1.0 : 0.0;
      }
    }
  }
  // b_i = <column_i, x_hat> over this lane's coordinates, completed across the half-waves
  const int64_t pp = good ? p : 0;
  double y[KMAX];
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    double b = 0.0;
    if (i <= it) {
#pragma unroll 1
      for (int j = 0; j < L::NKS; ++j) {
        const int c = L::coord(j, u);
        const double x = (good && c >= 0) ? double(prm.xhat[pp * L::B + c]) : 0.0;
        b += steer64<L>(hat, prm.cs64, R, cm[i], cr[i], j, u) * x;
      }
    }
    b += __shfl_xor(b, 32);
#pragma unroll
    for (int l = 0; l < i; ++l) b -= Lc[i][l] * y[l];
    y[i] = i <= it ? b / Lc[i][i] : 0.0;
  }
  double a[KMAX];
#pragma unroll
  for (int i = KMAX - 1; i >= 0; --i) {
    double s = y[i];
#pragma unroll
    for (int l = i + 1; l < KMAX; ++l) s -= Lc[l][i] * a[l];
    a[i] = i <= it ? s / Lc[i][i] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < L::NKS; ++j) {
    asm volatile("" ::: "memory");
    const int c = L::coord(j, u);
    double r = (good && c >= 0) ? double(prm.xhat[pp * L::B + c]) : 0.0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
      if (i <= it) r -= a[i] * steer64<L>(hat, prm.cs64, R, cm[i], cr[i], j, u);
    res[j] = good ? float(r) : res[j];
  }
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    st.cf[i] = (good && i <= it) ? float(a[i]) : st.cf[i];
    st.selm[i] = (good && i == it) ? ms : st.selm[i];
    st.selr[i] = (good && i == it) ? rs : st.selr[i];
  }
  return good;
}

// Least-squares step after the it-th selection (ms, rs) with signed correlation cval.
// FP32 Cholesky extension as in pursuit_update, plus the cond(Gram) bound; FP64
// re-solve where the bound is exceeded or the patch is already in FP64.  Returns
// whether this lane went through the FP64 solve.
template <class L, int KMAX>
__device__ __forceinline__ bool lp_update(PursuitState<KMAX>& st, float (&Ld)[KMAX], float& condF, bool& fp64,
                                          int it, int ms, int rs, float cval, const float* hat, const float* cs,
                                          const LpParams& prm, int64_t p, int u, float (&res)[L::NKS]) {
  const int M = prm.M, R = prm.R;
  bool dup = false;
#pragma unroll
  for (int i = 0; i < KMAX; ++i) dup = dup || (i < it && st.selm[i] == ms && st.selr[i] == rs);
  const bool upd = st.active && !dup;

  const float dd = pair_gram<L::T>(prm.gramH, cs, M, R, ms, rs, ms, rs);
  float gcol[KMAX];
  float bx = cval;
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    gcol[i] = 0.f;
    if (i < it) {
      const int mi = st.selm[i] < 0 ? 0 : st.selm[i], ri = st.selr[i] < 0 ? 0 : st.selr[i];
      gcol[i] = pair_gram<L::T>(prm.gramH, cs, M, R, mi, ri, ms, rs);
      bx += gcol[i] * st.cf[i];
    }
  }
  float w[KMAX];
  float l2 = dd;
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    float s = gcol[i];
#pragma unroll
    for (int j = 0; j < i; ++j) s -= st.L[i][j] * w[j];
    w[i] = i < it ? s * Ld[i] : 0.f;
    l2 -= w[i] * w[i];
  }
  // new row of L^{-1}: [-(L^{-T} w)^T, 1] / l, so ||L^{-1}||_F^2 grows by (|L^{-T} w|^2 + 1) / l^2
  float z[KMAX];
  float zz = 0.f;
#pragma unroll
  for (int i = KMAX - 1; i >= 0; --i) {
    float s = w[i];
#pragma unroll
    for (int j = i + 1; j < KMAX; ++j) s -= (j < it ? st.L[j][i] : 0.f) * z[j];
    z[i] = i < it ? s * Ld[i] : 0.f;
    zz += z[i] * z[i];
  }
  const float Fn = condF + (zz + 1.f) / fmaxf(l2, 1e-30f);
  const bool ok32 = !fp64 && l2 > 1e-6f * dd && float(it + 1) * Fn <= 1e6f;
  const bool up32 = upd && ok32;
  const bool go64 = upd && !ok32;
#pragma unroll
  for (int r = 0; r < KMAX; ++r) {
    const bool row = up32 && r == it;
#pragma unroll
    for (int i = 0; i < r; ++i) st.L[r][i] = row ? w[i] : st.L[r][i];
    Ld[r] = row ? rsqrtf(l2) : Ld[r];
    st.bv[r] = row ? bx : st.bv[r];
    st.selm[r] = row ? ms : st.selm[r];
    st.selr[r] = row ? rs : st.selr[r];
  }
  float y[KMAX], an[KMAX];
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    float s = st.bv[i];
#pragma unroll
    for (int j = 0; j < i; ++j) s -= st.L[i][j] * y[j];
    y[i] = i <= it ? s * Ld[i] : 0.f;
  }
#pragma unroll
  for (int i = KMAX - 1; i >= 0; --i) {
    float s = y[i];
#pragma unroll
    for (int j = i + 1; j < KMAX; ++j) s -= st.L[j][i] * an[j];
    an[i] = i <= it ? s * Ld[i] : 0.f;
  }
  if (__any(up32)) {
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      if (i <= it) {
        const float delta = up32 ? an[i] - st.cf[i] : 0.f;
        const int mi = st.selm[i] < 0 ? 0 : st.selm[i], ri = st.selr[i] < 0 ? 0 : st.selr[i];
        steer_axpy<L>(res, -delta, hat, cs, R, mi, ri, u);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < KMAX; ++i) st.cf[i] = (up32 && i <= it) ? an[i] : st.cf[i];
  condF = up32 ? Fn : condF;
  bool ok64 = false;
  if (__any(go64)) ok64 = lp_solve64<L, KMAX>(st, it, ms, rs, go64, hat, prm, p, u, res);
  fp64 = fp64 || ok64;
  st.nsel = (up32 || ok64) ? it + 1 : st.nsel;
  st.active = up32 || ok64;
  return go64;
}

// RT: 32-angle tiles of the 16-bit stage 2 (ceil(R/32)).  SPLIT: the FP32 re-score
// uses the radix-2 angle split (even R, R/2 <= 32 rows: E from even harmonics, O
// from odd ones, score(r) = E + O and score(r + R/2) = E - O); otherwise RT tiles
// of the direct angle DFT.
template <int S, int T, int KMAX, int PREC, int RT, bool SPLIT>
__global__ __launch_bounds__(256, (S <= 5 && KMAX <= 4) ? 2 : 1) void encode_lp_kernel(LpParams prm) {
  using L = Layout<S, T, 2>;
  using P = Lp<PREC>;
  using V8 = typename P::V8;
  constexpr int NKS = L::NKS, NQ = L::NQ, B = L::B, J0 = L::J0;
  static_assert(NQ <= 8 && S <= 8 && J0 <= 8, "a harmonic block must fit one half-wave's 8 slots");
  extern __shared__ uint4 lds4[];
  const int R = prm.R, M = prm.M, K = prm.K, NG = (M + 15) / 16;
  const V8* sA = reinterpret_cast<const V8*>(lds4);           // [NG][NQ][64]
  float* sHat = reinterpret_cast<float*>(lds4 + NG * NQ * 64);  // [16 NG][B]
  float* sCs = sHat + NG * 16 * B;                              // [2][NQ][R]
  float* sF = sCs + 2 * NQ * R;                                 // [SPLIT ? 1 : RT][NQ][64]
  constexpr int FT = SPLIT ? 1 : RT;
  {
    const int nA = NG * NQ * 64, nH = NG * 16 * B, nC = 2 * NQ * R, nF = FT * NQ * 64;
    for (int i = threadIdx.x; i < nA; i += blockDim.x) lds4[i] = prm.dictA[i];
    for (int i = threadIdx.x; i < nH; i += blockDim.x) sHat[i] = prm.dictHat[i];
    for (int i = threadIdx.x; i < nC; i += blockDim.x) sCs[i] = prm.cs[i];
    for (int i = threadIdx.x; i < nF; i += blockDim.x) sF[i] = prm.dft32[i];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, u = lane >> 5;
  V8 F16[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const uint4 w = prm.dft16[t * 64 + lane];
    __builtin_memcpy(&F16[t], &w, sizeof(w));
  }
  const float wfac = 4.f * P::unit;
  unsigned long long n_sel = 0, n_cand = 0, n_fp64 = 0, max_cand = 0;

  const int64_t nwt = (prm.P + 31) / 32;
  for (int64_t wt = int64_t(blockIdx.x) * 4 + wave; wt < nwt; wt += int64_t(gridDim.x) * 4) {
    const int64_t p = wt * 32 + col;
    const bool valid = p < prm.P;
    float res[NKS];
#pragma unroll
    for (int j = 0; j < NKS; ++j) {
      const int c = L::coord(j, u);
      res[j] = (valid && c >= 0) ? prm.xhat[p * B + c] : 0.f;
    }
    const float nx2 = norm2<L>(res);
    PursuitState<KMAX> st;
    init_state(st, valid);
    float Ld[KMAX];          // 1 / L[i][i]
    zero(Ld);
    float condF = 0.f;
    bool fp64 = false;

    for (int it = 0; it < K; ++it) {
      const float n2 = norm2<L>(res);
      st.active = st.active && (n2 > kTau2 * nx2);
      if (!__any(st.active)) break;

      // ---------------- 16-bit residual operand, one per harmonic
      V8 r16[NQ];
#pragma unroll
      for (int k = 0; k < NQ; ++k) {
        const int j0 = k == 0 ? 0 : J0 + (k - 1) * S, cnt = k == 0 ? J0 : S;
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = i < cnt ? res[i < cnt ? j0 + i : 0] : 0.f;
        r16[k] = pack8<P>(v);
      }
      const float wnd = wfac * sqrtf(n2);

      // ---------------- 16-bit scores: per-atom maxima and the candidate mask
      float vh = -1.f;          // running maximum over this half-wave's atoms
      uint64_t mask = 0;        // bit i: atom 2i + u is a candidate
      for (int g = 0; g < NG; ++g) {
        asm volatile("" ::: "memory");
        const V8* Ag = sA + g * NQ * 64 + lane;
        // stage 1 by pairs of harmonics; each pair is rounded at once into one 32-bit
        // register (two 16-bit slots) of every atom's stage-2 operand
        u32x4 opk[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k0 = 2 * j, k1 = 2 * j + 1;
          if (k0 >= NQ) {
#pragma unroll
            for (int a = 0; a < 16; ++a) opk[a][j] = 0u;
            continue;
          }
          f32x16 z, a0, a1;
#pragma unroll
          for (int i = 0; i < 16; ++i) z[i] = 0.f;
          a0 = P::mfma(Ag[k0 * 64], r16[k0], z);
          a1 = k1 < NQ ? P::mfma(Ag[(k1 < NQ ? k1 : k0) * 64], r16[k1 < NQ ? k1 : k0], z) : z;
#pragma unroll
          for (int a = 0; a < 16; ++a) opk[a][j] = pack2<P>(a0[a], a1[a]);
        }
        const int ab = 16 * g;
        // stage 2 by (atom, angle tile) units, one unit in flight: the next unit's
        // MFMA is issued before the current one's reduction
        auto issue = [&](int q) {
          f32x16 z;
#pragma unroll
          for (int i = 0; i < 16; ++i) z[i] = 0.f;
          return P::mfma(F16[q % RT], __builtin_bit_cast(V8, opk[q / RT]), z);
        };
        float vs[8];          // slot i: maximum of atom ab + 2i + u over its angles
        f32x16 cur = issue(0);
        float part = 0.f, mprev = 0.f;
#pragma unroll
        for (int q = 0; q < 16 * RT; ++q) {
          const int a = q / RT, t = q % RT;
          f32x16 nxt;
          if (q + 1 < 16 * RT) nxt = issue(q + 1);
          float m = fabsf(cur[0]);
#pragma unroll
          for (int i = 1; i < 16; ++i) m = fmaxf(m, fabsf(cur[i]));
          part = t == 0 ? m : fmaxf(part, m);
          if (t == RT - 1) {
            if (a % 2 == 0) {
              mprev = part;
            } else {
              // atoms a-1 and a completed across the half-waves: atom ab + a - 1 in
              // the low half-wave, ab + a in the high one
              float m0 = mprev, m1 = part;
              swap32(m0, m1);
              vs[a / 2] = fmaxf(m0, m1);
            }
          }
          if (q + 1 < 16 * RT) cur = nxt;
        }
        if (ab + 16 > M) {
#pragma unroll
          for (int i = 0; i < 8; ++i) vs[i] = ab + 2 * i + u < M ? vs[i] : -1.f;
        }
        // candidates of this group against the running maximum; a rise of the maximum
        // by more than the window drops every earlier candidate
        float gm = vs[0];
#pragma unroll
        for (int i = 1; i < 8; ++i) gm = fmaxf(gm, vs[i]);
        const float nvh = fmaxf(vh, gm), thr = nvh - wnd;
        mask = vh < thr ? uint64_t(0) : mask;
        unsigned gb = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) gb |= (vs[i] >= thr && vs[i] >= 0.f) ? (1u << i) : 0u;
        mask |= uint64_t(gb) << (8 * g);
        vh = nvh;
      }
      const float vmax = fmaxf(vh, __shfl_xor(vh, 32));
      if (!(vh >= vmax - wnd) || !st.active) mask = 0;

      // ---------------- FP32 re-score of the candidates, in increasing atom order
      float best = -1.f;
      int bm = 0, nc = 0;
      float bop[NQ];
      zero(bop);
      while (true) {
        const int mine = mask ? 2 * int(__builtin_ctzll(mask)) + u : 0x7fffffff;
        const int m = min(mine, __shfl_xor(mine, 32));
        const bool has = m != 0x7fffffff;
        if (!__any(has)) break;
        if (has && mine == m) mask &= mask - 1;
        nc += has ? 1 : 0;
        const int mc = has ? m : 0;
        const float* d = sHat + mc * B;
        float op32[NQ];
        {
          float p0 = 0.f;
#pragma unroll
          for (int i = 0; i < J0; ++i) {
            const int s = 2 * i + u;
            p0 = fmaf(s < S ? d[s < S ? s : 0] : 0.f, res[i], p0);
          }
          float zz = 0.f;
          swap32(p0, zz);
          op32[0] = p0 + zz;
        }
        // harmonic k >= 1: the low half-wave holds Re x, the high half-wave Im x;
        // partial sums (Re C, Im C) from this lane's coordinates, completed by the swap.
        // The dictionary values of harmonic k + 1 are loaded before harmonic k's FMAs.
        float c1[S], c2[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          c1[s] = d[L::base(1) + u * S + s];
          c2[s] = d[L::base(1) + (1 - u) * S + s];
        }
#pragma unroll
        for (int k = 1; k < NQ; ++k) {
          float n1[S], n2[S];
          if (k + 1 < NQ) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
              n1[s] = d[L::base(k + 1 < NQ ? k + 1 : k) + u * S + s];
              n2[s] = d[L::base(k + 1 < NQ ? k + 1 : k) + (1 - u) * S + s];
            }
          }
          asm volatile("" ::: "memory");
          const int j0 = J0 + (k - 1) * S;
          float pr = 0.f, pi = 0.f;
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const float xv = res[j0 + s];
            pr = fmaf(c1[s], xv, pr);
            pi = fmaf(c2[s], xv, pi);
          }
          pi = u ? pi : -pi;
          swap32(pr, pi);
          op32[k] = pr + pi;
          if (k + 1 < NQ) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
              c1[s] = n1[s];
              c2[s] = n2[s];
            }
          }
        }
        float cm = 0.f;
        if (SPLIT) {
          f32x16 e, o;
#pragma unroll
          for (int i = 0; i < 16; ++i) e[i] = o[i] = 0.f;
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            if (q % 2 == 0) e = mfma32(sF[q * 64 + lane], op32[q], e);
            else o = mfma32(sF[q * 64 + lane], op32[q], o);
          }
#pragma unroll
          for (int i = 0; i < 16; ++i) cm = fmaxf(cm, fabsf(e[i]) + fabsf(o[i]));
        } else {
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            f32x16 sc;
#pragma unroll
            for (int i = 0; i < 16; ++i) sc[i] = 0.f;
#pragma unroll
            for (int q = 0; q < NQ; ++q) sc = mfma32(sF[(t * NQ + q) * 64 + lane], op32[q], sc);
#pragma unroll
            for (int i = 0; i < 16; ++i) cm = fmaxf(cm, fabsf(sc[i]));
          }
        }
        cm = max_halves(cm);
        const bool gt = has && cm > best;
        best = gt ? cm : best;
        bm = gt ? mc : bm;
#pragma unroll
        for (int q = 0; q < NQ; ++q) bop[q] = gt ? op32[q] : bop[q];
      }
      // ---------------- angles of the best atom (same instructions as its maximum)
      int rs;
      float cval;
      {
        float rb = -1.f, rv = 0.f;
        int rc = 0;
        if (SPLIT) {
          const int HALF = R / 2;
          f32x16 e, o;
#pragma unroll
          for (int i = 0; i < 16; ++i) e[i] = o[i] = 0.f;
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            if (q % 2 == 0) e = mfma32(sF[q * 64 + lane], bop[q], e);
            else o = mfma32(sF[q * 64 + lane], bop[q], o);
          }
#pragma unroll
          for (int h = 0; h < 2; ++h)          // angles r < R/2 first, then r + R/2
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              const int row = 8 * (i / 4) + 4 * u + (i % 4);
              const float sc = h == 0 ? e[i] + o[i] : e[i] - o[i];
              const float val = row < HALF ? fabsf(sc) : -1.f;
              const bool gt = val > rb;
              rb = gt ? val : rb;
              rv = gt ? sc : rv;
              rc = gt ? row + h * HALF : rc;
            }
        } else {
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            f32x16 sc;
#pragma unroll
            for (int i = 0; i < 16; ++i) sc[i] = 0.f;
#pragma unroll
            for (int q = 0; q < NQ; ++q) sc = mfma32(sF[(t * NQ + q) * 64 + lane], bop[q], sc);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              const int r = 32 * t + 8 * (i / 4) + 4 * u + (i % 4);
              const float val = r < R ? fabsf(sc[i]) : -1.f;
              const bool gt = val > rb;
              rb = gt ? val : rb;
              rv = gt ? sc[i] : rv;
              rc = gt ? r : rc;
            }
          }
        }
        const float ob = __shfl_xor(rb, 32), ov = __shfl_xor(rv, 32);
        const int oc = __shfl_xor(rc, 32);
        const bool take = (ob > rb) || (ob == rb && oc < rc);
        rs = take ? oc : rc;
        cval = take ? ov : rv;
        rs = rs < R ? rs : R - 1;
      }
      // ---------------- (c)
      const bool counted = u == 0 && nc > 0;
      n_sel += counted ? 1 : 0;
      n_cand += u == 0 ? nc : 0;
      max_cand = (u == 0 && unsigned(nc) > max_cand) ? unsigned(nc) : max_cand;
      const bool went64 = lp_update<L, KMAX>(st, Ld, condF, fp64, it, bm, rs, cval, sHat, sCs, prm, p, u, res);
      n_fp64 += (u == 0 && went64) ? 1 : 0;
    }
    const float rn2 = norm2<L>(res);
    if (valid && u == 0) {
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
  }
  // per-wave totals of the counters, one atomic update per wave
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    n_sel += __shfl_xor(n_sel, off);
    n_cand += __shfl_xor(n_cand, off);
    n_fp64 += __shfl_xor(n_fp64, off);
    const unsigned long long o = __shfl_xor(max_cand, off);
    max_cand = o > max_cand ? o : max_cand;
  }
  if (lane == 0 && prm.stats) {
    atomicAdd(prm.stats + 0, n_sel);
    atomicAdd(prm.stats + 1, n_cand);
    atomicMax(prm.stats + 2, max_cand);
    atomicAdd(prm.stats + 3, n_fp64);
  }
}

template <int S, int T, int KMAX, int PREC, int RT, bool SPLIT>
int launch_lp(const DeviceTables& t, const LpParams& prm, hipStream_t st) {
  return launch_persistent(encode_lp_kernel<S, T, KMAX, PREC, RT, SPLIT>, encode_lp_lds_bytes(t),
                           (prm.P + 31) / 32, t.enc_bpc, st, prm);
}

template <int S, int T, int KMAX, int PREC>
int angles_lp(const DeviceTables& t, const LpParams& prm, hipStream_t st) {
  if (t.R <= 32) return launch_lp<S, T, KMAX, PREC, 1, false>(t, prm, st);
  if (t.lpSplit) return launch_lp<S, T, KMAX, PREC, 2, true>(t, prm, st);
  return launch_lp<S, T, KMAX, PREC, 2, false>(t, prm, st);
}

template <int PREC>
int dispatch_lp(const DeviceTables& t, const LpParams& prm, hipStream_t st) {
  if (t.S == 5 && t.T == 5) {
    if (prm.K <= 4) return angles_lp<5, 5, 4, PREC>(t, prm, st);
    return angles_lp<5, 5, 8, PREC>(t, prm, st);
  }
  if (t.S == 7 && t.T == 7) return angles_lp<7, 7, 8, PREC>(t, prm, st);
  return int(hipErrorInvalidValue);
}

}  // namespace

bool encode_lp_supported(int S, int T, int M, int R) {
  return ((S == 5 && T == 5) || (S == 7 && T == 7)) && M >= 1 && M <= 128 && R >= 1 && R <= 64;
}

size_t encode_lp_lds_bytes(const DeviceTables& t) {
  const int NG = (t.M + 15) / 16, NQ = t.T + 1, FT = (t.R <= 32 || t.lpSplit) ? 1 : 2;
  return size_t(NG) * NQ * 64 * 16 + sizeof(float) * (size_t(NG) * 16 * t.B + 2 * size_t(NQ) * t.R +
                                                       size_t(FT) * NQ * 64);
}

double encode_lp_mfma_flops_per_patch(const DeviceTables& t, int K) {
  // per step and 32 patches: NG (T+1) stage-1 and 16 NG RT stage-2 32x32x16 instructions
  const int NG = (t.M + 15) / 16, RT = (t.R + 31) / 32 <= 1 ? 1 : 2;
  const double per_instr = 2.0 * 32 * 32 * 16;
  return double(K) * (double(NG) * (t.T + 1) + 16.0 * NG * RT) * per_instr / 32.0;
}

int launch_encode_lp(const DeviceTables& t, int prec, const float* xhat, int64_t P, int K, int32_t* atom,
                     int32_t* angle, float* coef, float* resid2, void* stream) {
  if (P <= 0) return 0;
  LpParams prm{xhat, P, K, t.M, t.R,
               reinterpret_cast<const uint4*>(t.lpA), t.dictHat, reinterpret_cast<const uint4*>(t.lpF16),
               t.lpF32, t.cs, t.gramH, t.gramH64, t.cs64, atom, angle, coef, resid2, t.lpStats};
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == RSC_BF16) return dispatch_lp<RSC_BF16>(t, prm, st);
  if (prec == RSC_FP16) return dispatch_lp<RSC_FP16>(t, prm, st);
  return int(hipErrorInvalidValue);
}

}  // namespace rsc
