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
//   candidates: atoms whose 16-bit maximum lies within 8.5u ||r|| of the largest one
//     (u: unit roundoff of the 16-bit format).  Per harmonic k, rounding the atom and
//     the residual moves C_k by at most (2u + u^2) sum_s |d_{k,s}| |x_{k,s}| (complex
//     magnitudes), and rounding the stage-2 operand C_k and (cos, -sin) moves the term
//     cos Re C_k - sin Im C_k by at most (2u + u^2) |C_k| (Cauchy-Schwarz on the
//     2-vectors).  Summed over k with unit-norm atoms (Cauchy-Schwarz again), a 16-bit
//     score is within (2u + u^2)(1 + (1 + u)^2) ||r|| = 4.02u ||r|| (BF16; less for FP16)
//     of the exact one; FP32 accumulation adds below 1e-3 of that.  An atom's 16-bit
//     maximum over the angles is then within that of its exact maximum, so the atom
//     with the exact maximum lies within twice that (8.05u ||r||) of the largest 16-bit
//     maximum: the window keeps it.  FP16
//     residuals are scaled by a power of two to a norm in [0.5, 1) first, so that no
//     coordinate that matters falls into the subnormal range, where the rounding is
//     absolute.  Each half-wave keeps a bit mask of its atoms and its own running
//     maximum, and a new maximum more than the window above the old one clears the
//     mask (an atom it drops lies below the final maximum minus the window).
//   FP32 re-score: per candidate, C_k in FP32 from the packed dictionary (each lane
//     its half of the coordinates, a half-wave swap completes the sums) and the
//     angle DFT on v_mfma_f32_32x32x2f32; the best candidate by exact maximum, then
//     its angles again with the same instructions for the argmax.  Candidates are
//     visited in increasing atom order; equal maxima go to the smaller atom, then angle.
//   BF16 candidate filter: the window holds several atoms per step (and a wave loops
//     over its patches' largest candidate count), so the atom with the largest 16-bit
//     maximum is re-scored first, and of the others only those whose 16-bit maximum
//     reaches its FP32 maximum minus the error bound (4.02u ||r||, taken as 4.25u) are
//     kept: the atom with the largest FP32 maximum E has a 16-bit maximum of at least
//     E - 4.02u ||r||, and E is at least the first one's.  The 16-bit maxima are kept for
//     this in LDS as FP16 fractions of ||r|| (each lane its own), read with a margin
//     of 2^-10 for their rounding.
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

// Offset, in 16-byte units from the start of the kernel's LDS, of the per-wave copies of
// the atoms' 16-bit maxima: after the stage-1 operand (NG NQ 64 x 16 B) and the FP32
// tables (dictionary, cos/sin, re-score operand), rounded up to 16 bytes.
__host__ __device__ constexpr size_t lp_vmax_offset16(int NG, int NQ, int B, int R, int FT) {
  return size_t(NG) * NQ * 64 + (sizeof(float) * (size_t(NG) * 16 * B + 2 * size_t(NQ) * R +
                                                  size_t(FT) * NQ * 64) + 15) / 16;
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
  // [4 waves][NG][64 lanes] x 8 FP16: each lane's 16-bit atom maxima of the current step,
  // divided by ||r|| (read back by the same lane only)
  uint4* sV = lds4 + lp_vmax_offset16(NG, NQ, B, R, FT);
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
  const LsTables tb{prm.gramH, prm.gramH64, prm.cs64, prm.xhat, prm.M, prm.R, kCondMax16};
  const float wfac = 8.5f * P::unit;
  // a candidate is re-scored only if its 16-bit maximum reaches the best FP32 maximum found
  // so far minus the bound on a 16-bit score's error (4.02u ||r||, taken as 4.25u), less the
  // error of its FP16 copy (below 2^-10 in units of ||r||)
  const float efac = 4.25f * P::unit + 0x1p-10f;
  // BF16 only: its window holds several candidates per step; FP16's holds about one, and
  // the bookkeeping would cost more than it saves
  constexpr bool kFilter = PREC == RSC_BF16;
  unsigned long long n_sel = 0, n_cand = 0, n_fp64 = 0, max_cand = 0;

  const int64_t nwt = (prm.P + 31) / 32;
  for (int64_t wt = int64_t(blockIdx.x) * 4 + wave; wt < nwt; wt += int64_t(gridDim.x) * 4) {
    const int64_t p = wt * 32 + col;
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
      const float n2 = norm2<L>(res);
      st.active = st.active && (n2 > kTau2 * nx2);
      if (!__any(st.active)) break;

      // ---------------- 16-bit residual operand, one per harmonic (FP16: the residual
      // scaled by 2^-e, ||r|| = f 2^e with f in [0.5, 1); the scores and the window are
      // compared in the scaled units)
      const float rn = sqrtf(n2);
      int ex = 0;
      if (PREC == RSC_FP16) (void)frexpf(rn, &ex);
      const float sc = PREC == RSC_FP16 ? ldexpf(1.f, -ex) : 1.f;
      V8 r16[NQ];
#pragma unroll
      for (int k = 0; k < NQ; ++k) {
        const int j0 = k == 0 ? 0 : J0 + (k - 1) * S, cnt = k == 0 ? J0 : S;
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = i < cnt ? sc * res[i < cnt ? j0 + i : 0] : 0.f;
        r16[k] = pack8<P>(v);
      }
      const float wnd = wfac * rn * sc;
      const float invn = rn > 0.f ? 1.f / (rn * sc) : 0.f;

      // ---------------- 16-bit scores: per-atom maxima and the candidate mask
      float vh = -1.f;          // running maximum over this half-wave's atoms
      int va = 0;               // its atom (the first one on equal maxima)
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
        if constexpr (kFilter) {
          int gi = 7;
#pragma unroll
          for (int i = 7; i >= 0; --i) gi = vs[i] == gm ? i : gi;
          va = gm > vh ? ab + 2 * gi + u : va;
        }
        vh = nvh;
        if constexpr (kFilter) {
          _Float16 hv[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) hv[i] = _Float16(vs[i] * invn);
          uint4 w;
          __builtin_memcpy(&w, hv, sizeof(w));
          sV[(wave * NG + g) * 64 + lane] = w;
        }
      }
      const float vo = __shfl_xor(vh, 32);
      const int vao = __shfl_xor(va, 32);
      const float vmax = fmaxf(vh, vo);
      if (!(vh >= vmax - wnd) || !st.active) mask = 0;
      // the patch's atom with the largest 16-bit maximum (the low half-wave's on equal maxima)
      // is re-scored first; its FP32 maximum then bounds which other candidates can win
      const int m1 = (u == 0 ? vh >= vo : vo < vh) ? va : vao;
      const bool has1 = st.active && vmax >= 0.f;
      if (kFilter && has1 && (m1 & 1) == u) mask &= ~(uint64_t(1) << (m1 >> 1));

      // ---------------- FP32 re-score of the candidates, in increasing atom order
      float best = -1.f;
      int bm = 0, nc = 0;
      float bop[NQ];
      zero(bop);
      for (int pass = 0;; ++pass) {
        int m;
        bool has;
        if (kFilter && pass == 0) {
          has = has1;
          m = m1;
        } else {
          const int mine = mask ? 2 * int(__builtin_ctzll(mask)) + u : 0x7fffffff;
          m = min(mine, __shfl_xor(mine, 32));
          has = m != 0x7fffffff;
          if (has && mine == m) mask &= mask - 1;
        }
        if (!__any(has)) break;
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
        // candidates after the first come in increasing atom order: equal maxima go to the
        // smaller atom
        const bool gt = has && (cm > best || (cm == best && mc < bm));
        best = gt ? cm : best;
        bm = gt ? mc : bm;
#pragma unroll
        for (int q = 0; q < NQ; ++q) bop[q] = gt ? op32[q] : bop[q];
        if (kFilter && pass == 0) {
          // keep the candidates whose 16-bit maximum reaches best - the error bound: the atom
          // with the largest FP32 maximum E has a 16-bit maximum of at least E - 4.02u ||r||,
          // and E >= best
          const float thrn = has ? best / rn - efac : -2.f;
          uint64_t mm = mask, keep = 0;
          const uint4* vrow = sV + wave * NG * 64 + lane;
          while (mm) {
            const int i = int(__builtin_ctzll(mm));
            mm &= mm - 1;
            const uint4 w = vrow[(i >> 3) * 64];
            _Float16 hv[8];
            __builtin_memcpy(hv, &w, sizeof(w));
            if (float(hv[i & 7]) >= thrn) keep |= uint64_t(1) << i;
          }
          mask = keep;
        }
      }
      // ---------------- angles of the best atom (same instructions as its maximum)
      int rs;
      float cval;
      {
        // Rows past the valid angles have all-zero operand rows, so their scores are exactly
        // 0.  A lane reaches them after its valid rows (its rows ascend), and a 0 never beats
        // an earlier value under the strict '>'; a lane with no valid row ends with 0 at an
        // index past the valid ones, which loses the cross-lane tie to the other lane (row 0
        // is always valid).  So no row mask is needed.
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
              const float val = fabsf(sc);
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
              const float val = fabsf(sc[i]);
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
      const bool went64 = ls_update<L, KMAX>(st, ls, it, bm, rs, cval, sHat, sCs, tb, p, u, res);
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
  if (t.S == 7 && t.T == 7) {
    if (prm.K <= 6) return angles_lp<7, 7, 6, PREC>(t, prm, st);   // the six-slot state: fewer registers
    return angles_lp<7, 7, 8, PREC>(t, prm, st);
  }
  return int(hipErrorInvalidValue);
}

}  // namespace

bool encode_lp_supported(int S, int T, int M, int R) {
  return ((S == 5 && T == 5) || (S == 7 && T == 7)) && M >= 1 && M <= 128 && R >= 1 && R <= 64;
}

size_t encode_lp_lds_bytes(const DeviceTables& t) {
  const int NG = (t.M + 15) / 16, NQ = t.T + 1, FT = (t.R <= 32 || t.lpSplit) ? 1 : 2;
  // tables, then (BF16) 4 waves x NG x 64 lanes x 16 B of FP16 atom maxima
  return 16 * (lp_vmax_offset16(NG, NQ, t.B, t.R, FT) + (t.prec == RSC_BF16 ? size_t(4) * NG * 64 : 0));
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
