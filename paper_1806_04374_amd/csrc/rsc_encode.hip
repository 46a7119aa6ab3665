// Rotational OMP encoders (Fig. 2 with R_r -> S_r; Sec. II-C, II-E step 3).
//
// One launch runs all K pursuit steps for every patch.  Each wave owns a tile of
// patches (the MFMA columns) and, per step:
//   (b) correlates the residual with every rotation of every atom.  Steering is
//       diagonal per harmonic (eq. (8)), so
//         <S_r d_m, x> = C_0 + sum_{k>=1} [cos(2 pi k r/R) Re C_k - sin(2 pi k r/R) Im C_k],
//         C_k = sum_s conj(d_{m,s,k}) x_{s,k}.
//       Stage 1 forms Re C_k and Im C_k on MFMA (rows: atoms x {Re, Im}); its
//       accumulators are the operand of stage 2 (as they stand with the 32x32 tiles'
//       row order, after a cross-lane swap with the 16x16 tiles), the angle DFT on MFMA
//       (rows: angles).  For even R the DFT is split by harmonic
//       parity (one radix-2 step): with E(r) the sum over even k and O(r) over odd k,
//       score(r) = E(r) + O(r) and score(r + R/2) = E(r) - O(r), so only R/2 angle
//       rows are computed, and the largest |score| of an atom over all R angles is
//       max_r (|E(r)| + |O(r)|), bit-identical to the maximum of the rounded scores.
//       The argmax runs in two passes: per atom only that maximum is compared; the
//       winning atom's angles are then recomputed and searched from its stage-2 operand
//       formed again from its dictionary row (one product per coordinate per step instead
//       of a register copy per atom).  Exact ties go to the smallest atom, then the
//       smallest angle.
//   (c) extends the Cholesky factor of the selected columns, solves the least
//       squares and updates the residual, all in registers; a patch whose Gram matrix
//       grows ill-conditioned (bound k ||L^{-1}||_F^2 above 1e3) or whose new pivot is
//       negligible has its least squares re-solved in FP64 from then on (ls_update).
//
// Two tile shapes:
//   encode32: v_mfma_f32_32x32x2f32, 32 patches per wave, 16 atoms per stage-1
//             tile; dictionary operand pre-arranged in LDS.  (S, T) = (5, 5), K <= 4,
//             even R <= 64.
//   encode16: v_mfma_f32_16x16x4f32, 16 patches per wave, 8 atoms per stage-1
//             tile; dictionary operand read from the packed dictionary in LDS (the Im
//             rows from a second table holding i * d where both fit).
//             Any compiled (S, T), K <= 8, any R (odd R without the split).
#include <hip/hip_runtime.h>

#include "rsc_device.h"
#include "rsc_encode16.h"
#include "rsc_internal.h"
#include "rsc_launch.h"

namespace rsc {
namespace {

using enc::EncodeParams;
using enc::count_fp64;
using enc::encode16_kernel;
using enc::write_codes;

// ============================================================== 32x32 tiles
// F[q]: stage-2 operand of harmonic q for angle rows r < R/2 (rows past R/2 zero).
template <int S, int T, int KMAX>
__global__ __launch_bounds__(256, 2) void encode32_kernel(EncodeParams prm, int NG) {
  using L = Layout<S, T, 2>;
  constexpr int NKS = L::NKS, NQ = L::NQ, B = L::B;
  extern __shared__ float lds[];
  const int R = prm.R, M = prm.M, K = prm.K, HALF = prm.R / 2;
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
  const int col = lane & 31, u = lane >> 5;
  const LsTables tb{prm.gramH, prm.gramH64, prm.cs64, prm.xhat, M, R, kCondMaxFp32};
  unsigned n64 = 0;
  float F[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) F[q] = prm.dftA[q * 64 + lane];

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
      st.active = st.active && (norm2<L>(res) > kTau2 * nx2);
      if (!__any(st.active)) break;

      // ---------------- (b) pass 1: best atom by its maximum over all angles
      float best = -1.f;
      int bm = 0;
      for (int g = 0; g < NG; ++g) {
        const float* Ag = sA + g * NKS * 64 + lane;
        f32x16 acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[q][i] = 0.f;
#pragma unroll
        for (int j = 0; j < NKS; ++j) {
          const int k = L::harm(j);
          acc[k] = mfma32(Ag[j * 64], res[j], acc[k]);
        }
        // Operand rows 8i..8i+3 give Re C of atoms 4i..4i+3 and rows 8i+4..8i+7 their Im C.
        // In the accumulator layout register a of the low half-wave then holds Re C of atom
        // a and register a of the high half-wave its Im C: acc[q][a] is the stage-2 operand
        // [Re | Im] of atom a as it stands, with no data movement.
        // Per atom: E (even harmonics) and O (odd harmonics) chains; the E chain of
        // the next atom is issued before the reduction of the current one.  Atoms
        // past M have all-zero operands: their scores are exactly 0 and never beat
        // the first atom under the strict '>'.
        auto vreg = [](int a) { return a; };
        auto chain = [&](int a, int parity) {
          f32x16 o;
#pragma unroll
          for (int i = 0; i < 16; ++i) o[i] = 0.f;
#pragma unroll
          for (int q = parity; q < NQ; q += 2) o = mfma32(F[q], acc[q][vreg(a)], o);
          return o;
        };
        // each half-wave's maximum of every atom first (16 angle rows per lane)
        float amh[16];
        f32x16 e_cur = chain(0, 0), o_cur = chain(0, 1);
#pragma unroll
        for (int a = 0; a < 16; ++a) {
          f32x16 e_next;
          if (a + 1 < 16) e_next = chain(a + 1, 0);
          float am = fabsf(e_cur[0]) + fabsf(o_cur[0]);
#pragma unroll
          for (int i = 1; i < 16; ++i) am = fmaxf(am, fabsf(e_cur[i]) + fabsf(o_cur[i]));
          amh[a] = am;
          if (a + 1 < 16) {
            o_cur = chain(a + 1, 1);
            e_cur = e_next;
          }
        }
        // then the maximum over both half-waves, two atoms per swap: [a_lo | a_hi] and
        // [b_lo | b_hi] give [A | B] (A, B the atoms' maxima), and one more swap of [A | B]
        // with itself broadcasts [A | A] and [B | B] (non-negative floats compared as integers)
        float amx[16];
#pragma unroll
        for (int a = 0; a < 16; a += 2) {
          float x = amh[a], y = amh[a + 1];
          swap32(x, y);
          float m1 = __uint_as_float(max(__float_as_uint(x), __float_as_uint(y))), m2 = m1;
          swap32(m1, m2);
          amx[a] = m1;
          amx[a + 1] = m2;
        }
        // the winner inside the group is kept as a constant (ba) and a lane mask (upd), and
        // turned into the atom index once per group
        int ba = 0;
        bool upd = false;
#pragma unroll
        for (int a = 0; a < 16; ++a) {
          const bool gt = amx[a] > best;
          best = gt ? amx[a] : best;
          ba = gt ? a : ba;
          upd = upd || gt;
        }
        bm = upd ? g * 16 + ba : bm;
      }
      // ---------------- (b) pass 2: angles of the best atom, its stage-2 operand formed
      // again from its dictionary row (no per-atom copy is kept in pass 1)
      int rs;
      float cval;
      {
        float op[NQ];
        atom_operand<L>(sHat, bm, u, res, op);
        f32x16 e, o;
#pragma unroll
        for (int i = 0; i < 16; ++i) e[i] = o[i] = 0.f;
#pragma unroll
        for (int q = 0; q < NQ; q += 2) e = mfma32(F[q], op[q], e);
#pragma unroll
        for (int q = 1; q < NQ; q += 2) o = mfma32(F[q], op[q], o);
        // Rows past R/2 have all-zero operand rows, so their scores are exactly 0.  A lane
        // reaches them after its valid rows (its rows ascend), and a 0 never beats an earlier
        // value under the strict '>'; a lane with no valid row ends with 0 at an index of at
        // least R/2, which loses the cross-lane tie to the other lane (row 0 is always valid).
        // So no row mask is needed.
        float rb = -1.f, rv = 0.f;
        int rc = 0;
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
        const float ob = __shfl_xor(rb, 32), ov = __shfl_xor(rv, 32);
        const int oc = __shfl_xor(rc, 32);
        const bool take = (ob > rb) || (ob == rb && oc < rc);
        rs = take ? oc : rc;
        cval = take ? ov : rv;
        rs = rs < R ? rs : R - 1;
      }
      // ---------------- (c)
      n64 += (ls_update<L, KMAX>(st, ls, it, bm, rs, cval, sHat, sCs, tb, p, u, res) && u == 0) ? 1u : 0u;
    }
    const float rn2 = norm2<L>(res);
    if (valid && u == 0) write_codes<L, KMAX>(prm, p, st, rn2);
  }
  count_fp64(prm.stats, n64, lane);
}

// ============================================================== launchers
template <int S, int T, int KMAX>
int launch32(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  return launch_persistent(encode32_kernel<S, T, KMAX>, encode_lds_bytes(t, RSC_TILE_32), (prm.P + 31) / 32,
                           t.enc_bpc, st, prm, t.NG);
}

template <class C, int HT, int KMAX, bool SPLIT>
int launch16(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  const int64_t tiles = (prm.P + 15) / 16;
  if (encode16_irows(t))
    return launch_persistent_n(encode16_kernel<C, HT, KMAX, SPLIT, true>, encode16_threads(tiles),
                               encode16_lds_bytes(t, true), tiles, t.enc_bpc, st, prm);
  return launch_persistent(encode16_kernel<C, HT, KMAX, SPLIT, false>, encode16_lds_bytes(t, false), tiles,
                           t.enc_bpc, st, prm);
}

template <class C, int HT, bool SPLIT>
int k16(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  if (prm.K <= 2) return launch16<C, HT, 2, SPLIT>(t, prm, st);
  if (prm.K <= 4) return launch16<C, HT, 4, SPLIT>(t, prm, st);
  if (prm.K <= 6) return launch16<C, HT, 6, SPLIT>(t, prm, st);   // fewer registers than 8 slots
  return launch16<C, HT, 8, SPLIT>(t, prm, st);
}

// angle tiles of 16 rows: R/2 rows with the split (even R), R rows without
template <class C>
int r16(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  if (t.R % 2 == 0) {
    const int ht = (t.R / 2 + 15) / 16;
    if (ht <= 1) return k16<C, 1, true>(t, prm, st);
    if (ht <= 2) return k16<C, 2, true>(t, prm, st);
    return k16<C, 4, true>(t, prm, st);
  }
  const int ht = (t.R + 15) / 16;
  if (ht <= 1) return k16<C, 1, false>(t, prm, st);
  if (ht <= 2) return k16<C, 2, false>(t, prm, st);
  if (ht <= 4) return k16<C, 4, false>(t, prm, st);
  return k16<C, 8, false>(t, prm, st);
}

int r32(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  if (prm.K <= 2) return launch32<5, 5, 2>(t, prm, st);
  return launch32<5, 5, 4>(t, prm, st);
}

}  // namespace

bool encode_supported(int S, int T) { return (S == 5 && T == 5) || (S == 7 && T == 7); }

bool encode_supported_geo(const DeviceTables& t) {
  if (t.geo == kGeoAnnular11) return t.T == AnnularCounts11::T && t.B == LayoutBase<AnnularCounts11, 4>::B;
  if (t.geo == kGeoAnnular15) return t.T == AnnularCounts15::T && t.B == LayoutBase<AnnularCounts15, 4>::B;
  return t.geo == kGeoGrid && encode_supported(t.S, t.T);
}

size_t encode16_lds_bytes(const DeviceTables& t, bool irows) {
  const size_t cs = 2 * size_t(t.T + 1) * t.R;
  const int ng = (t.M + 7) / 8;
  return sizeof(float) * (size_t(ng) * 8 * t.B * (irows ? 2 : 1) + cs);
}

bool encode16_irows(const DeviceTables& t) {
  return t.dictHatI != nullptr && encode16_lds_bytes(t, true) <= 160 * 1024;
}

int encode16_threads(int64_t wave_tiles) { return wave_tiles >= 8 * int64_t(num_cus()) ? 512 : 256; }

size_t encode_lds_bytes(const DeviceTables& t, int tile) {
  if (tile == RSC_TILE_32) {
    const size_t cs = 2 * size_t(t.T + 1) * t.R;
    const int ng = (t.M + 15) / 16;
    return sizeof(float) * (size_t(ng) * stage1_steps(t.S, t.T) * 64 + size_t(ng) * 16 * t.B + cs);
  }
  return encode16_lds_bytes(t, false);   // the smaller form, used when the copy does not fit
}

bool tile32_usable(const DeviceTables& t, int K) {
  return t.S == 5 && t.T == 5 && K <= 4 && t.R <= 64 && t.R % 2 == 0 && t.dictA &&
         encode_lds_bytes(t, RSC_TILE_32) <= 80 * 1024;
}

double encode_mfma_flops_per_patch(const DeviceTables& t, int tile, int K) {
  const int S = t.S, T = t.T, NQ = T + 1;
  if (tile == RSC_TILE_32) {
    // per wave of 32 patches and step: NG stage-1 tiles of stage1_steps MFMAs, 16 atoms x
    // (T+1) stage-2 MFMAs per group, plus the winner's recompute; 2*32*32*2 flops each
    const double per_step = double(t.NG) * (stage1_steps(S, T) + 16.0 * NQ) + NQ;
    return K * per_step * 4096.0 / 32.0;
  }
  const int W = 4;
  int NKS = (t.sk[0] + W - 1) / W;
  for (int k = 1; k <= T; ++k) NKS += (2 * t.sk[k] + W - 1) / W;
  int ht, ns;
  if (t.R % 2 == 0) {
    const int NE = T / 2 + 1, NO = (T + 1) / 2;
    ht = (t.R / 2 + 15) / 16;
    ht = ht <= 1 ? 1 : (ht <= 2 ? 2 : 4);
    ns = (NE + 1) / 2 + (NO + 1) / 2;
  } else {
    ht = (t.R + 15) / 16;
    ht = ht <= 1 ? 1 : (ht <= 2 ? 2 : (ht <= 4 ? 4 : 8));
    ns = (NQ + 1) / 2;
  }
  const int ng8 = (t.M + 7) / 8;
  const double per_step = double(ng8) * (NKS + 8.0 * ht * ns) + ht * ns;
  return K * per_step * 2048.0 / 16.0;
}

int launch_encode(const DeviceTables& t, int tile, const float* xhat, int64_t P, int K, int32_t* atom,
                  int32_t* angle, float* coef, float* resid2, void* stream) {
  if (P <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (tile == RSC_TILE_32) {
    if (!tile32_usable(t, K)) return int(hipErrorInvalidValue);
    EncodeParams prm{xhat, P, K, t.M, t.R, t.dictA, t.dictHat, t.dftA32, t.cs, t.gramH, t.gramH64, t.cs64,
                     atom, angle, coef, resid2, t.lpStats, nullptr};
    return r32(t, prm, st);
  }
  EncodeParams prm{xhat, P, K, t.M, t.R, nullptr, t.dictHat, t.R % 2 == 0 ? t.dftA16s : t.dftA16, t.cs, t.gramH,
                   t.gramH64, t.cs64, atom, angle, coef, resid2, t.lpStats, t.dictHatI};
  if (t.geo == kGeoAnnular11 || t.geo == kGeoAnnular15)
    return launch_encode_annular(t, xhat, P, K, atom, angle, coef, resid2, stream);
  if (t.geo != kGeoGrid) return int(hipErrorInvalidValue);
  if (t.S == 5 && t.T == 5) return r16<UniformCounts<5, 5>>(t, prm, st);
  if (t.S == 7 && t.T == 7) return r16<UniformCounts<7, 7>>(t, prm, st);
  return int(hipErrorInvalidValue);
}

}  // namespace rsc
