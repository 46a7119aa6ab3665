// Rotational OMP encoders (Fig. 2 with R_r -> S_r; Sec. II-C, II-E step 3).
//
// One launch runs all K pursuit steps for every patch.  Each wave owns a tile of
// patches (the MFMA columns) and, per step:
//   (b) correlates the residual with every rotation of every atom.  Steering is
//       diagonal per harmonic (eq. (8)), so
//         <S_r d_m, x> = C_0 + sum_{k>=1} [cos(2 pi k r/R) Re C_k - sin(2 pi k r/R) Im C_k],
//         C_k = sum_s conj(d_{m,s,k}) x_{s,k}.
//       Stage 1 forms Re C_k and Im C_k on MFMA (rows: atoms x {Re, Im}), a
//       cross-lane swap turns its accumulators into the operand of stage 2, the
//       R-point angle DFT on MFMA (rows: angles).  The argmax of |score| runs in
//       two passes: per atom only the maximum over angles is compared (max3
//       reductions), and the winning atom's stage-2 operand is kept; its angles are
//       then recomputed with the same instructions (bit-identical scores) and
//       searched for the argmax.  Exact ties go to the smallest atom, then the
//       smallest angle.
//   (c) extends the Cholesky factor of the selected columns, solves the least
//       squares and recomputes the residual, all in registers.
//
// Two tile shapes:
//   encode32: v_mfma_f32_32x32x2f32, 32 patches per wave, 16 atoms per stage-1
//             tile; dictionary operand pre-arranged in LDS.  (S, T) = (5, 5), K <= 4,
//             R <= 64.
//   encode16: v_mfma_f32_16x16x4f32, 16 patches per wave, 8 atoms per stage-1
//             tile; dictionary operand read from the packed dictionary in LDS.
//             Any compiled (S, T), K <= 8.
#include <hip/hip_runtime.h>

#include "rsc_device.h"
#include "rsc_internal.h"

namespace rsc {
namespace {

struct EncodeParams {
  const float* xhat;
  int64_t P;
  int K, M, R;
  const float* dictA;     // encode32 stage-1 operand [NG][NKS][64]
  const float* dictHat;   // [NG8*8 or NG*16][B]
  const float* dftA;      // stage-2 operand (layout per tile shape)
  const float* cs;        // [2][T+1][R]
  const float* gramH;     // [M][M][2T+1] per-pair harmonic inner products
  int32_t* atom;
  int32_t* angle;
  float* coef;
  float* resid2;
};

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

// ============================================================== 32x32 tiles
template <int S, int T, int RT, int KMAX>
__global__ __launch_bounds__(256, 2) void encode32_kernel(EncodeParams prm, int NG) {
  using L = Layout<S, T, 2>;
  constexpr int NKS = L::NKS, NQ = L::NQ, B = L::B, J0 = L::J0;
  extern __shared__ float lds[];
  const int R = prm.R, M = prm.M, K = prm.K;
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
  float F[RT][NQ];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int q = 0; q < NQ; ++q) F[t][q] = prm.dftA[(t * NQ + q) * 64 + lane];

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

    for (int it = 0; it < K; ++it) {
      st.active = st.active && (norm2<L>(res) > kTau2 * nx2);
      if (!__any(st.active)) break;

      // ---------------- (b) pass 1: best atom by its maximum over all angles
      float best = -1.f;
      int bm = 0;
      float bop[NQ];
      zero(bop);
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
        // rows 0..15: Re C of atoms 0..15, rows 16..31: Im C.  After the swap,
        // register v < 8 is the stage-2 operand [Re | Im] of atom 8(v/4)+v%4 and
        // register v+8 that of atom 8(v/4)+v%4+4.
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            float x = acc[q][v], y = acc[q][v + 8];
            swap32(x, y);
            acc[q][v] = x;
            acc[q][v + 8] = y;
          }
        // Pass 1 over the 16 atoms x RT angle tiles of the group, software-pipelined:
        // the MFMA chain of the next (atom, tile) unit is issued before the |.| max
        // reduction of the current one.  Atoms past M have all-zero operands, so their
        // scores are exactly 0 and never beat the first atom under the strict '>'.
        constexpr int NU = 16 * RT;
        f32x16 ob[2];
        auto chain = [&](int a, int t) {
          const int v = 4 * (a / 8) + (a % 4) + 8 * ((a / 4) % 2);
          f32x16 o;
#pragma unroll
          for (int i = 0; i < 16; ++i) o[i] = 0.f;
#pragma unroll
          for (int q = 0; q < NQ; ++q) o = mfma32(F[t][q], acc[q][v], o);
          return o;
        };
        ob[0] = chain(0, 0);
        float amax = 0.f;
#pragma unroll
        for (int un = 0; un < NU; ++un) {
          const int a = un / RT, t = un % RT;
          if (un + 1 < NU) ob[(un + 1) & 1] = chain((un + 1) / RT, (un + 1) % RT);
          const f32x16& o = ob[un & 1];
          float tm = fabsf(o[0]);
#pragma unroll
          for (int i = 1; i < 16; ++i) tm = fmaxf(tm, fabsf(o[i]));
          amax = t == 0 ? tm : fmaxf(amax, tm);
          if (t == RT - 1) {
            const int v = 4 * (a / 8) + (a % 4) + 8 * ((a / 4) % 2);
            const float am = max_halves(amax);
            const bool gt = am > best;
            best = gt ? am : best;
            bm = gt ? g * 16 + a : bm;
#pragma unroll
            for (int q = 0; q < NQ; ++q) bop[q] = gt ? acc[q][v] : bop[q];
          }
        }
      }
      // ---------------- (b) pass 2: angles of the best atom, same arithmetic
      int rs;
      float cval;
      {
        f32x16 o[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int i = 0; i < 16; ++i) o[t][i] = 0.f;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int t = 0; t < RT; ++t) o[t] = mfma32(F[t][q], bop[q], o[t]);
        float rb = -1.f, rv = 0.f;
        int rc = 0;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const float val = fabsf(o[t][i]);
            const bool gt = val > rb;
            rb = gt ? val : rb;
            rv = gt ? o[t][i] : rv;
            rc = gt ? 32 * t + 8 * (i / 4) + (i % 4) : rc;
          }
        rc += 4 * u;
        const float ob = __shfl_xor(rb, 32), ov = __shfl_xor(rv, 32);
        const int oc = __shfl_xor(rc, 32);
        const bool take = (ob > rb) || (ob == rb && oc < rc);
        rs = take ? oc : rc;
        cval = take ? ov : rv;
        rs = rs < R ? rs : R - 1;
      }
      // ---------------- (c)
      pursuit_update<L, KMAX>(st, it, bm, rs, cval, sHat, sCs, prm.gramH, M, R, u, res);
    }
    const float rn2 = norm2<L>(res);
    if (valid && u == 0) write_codes<L, KMAX>(prm, p, st, rn2);
  }
}

// ============================================================== 16x16 tiles
template <int S, int T, int RT, int KMAX>
__global__ __launch_bounds__(256, 2) void encode16_kernel(EncodeParams prm) {
  using L = Layout<S, T, 4>;
  constexpr int NKS = L::NKS, NQ = L::NQ, B = L::B, J0 = L::J0, J1 = L::J1;
  constexpr int NP = (NQ + 1) / 2;       // harmonic pairs per stage-2 step
  extern __shared__ float lds[];
  const int R = prm.R, M = prm.M, K = prm.K;
  const int NG = (M + 7) / 8;
  float* sHat = lds;                     // [NG*8][B]
  float* sCs = sHat + NG * 8 * B;        // [2][NQ][R]
  {
    const int nH = NG * 8 * B, nC = 2 * NQ * R;
    for (int i = threadIdx.x; i < nH; i += blockDim.x) sHat[i] = prm.dictHat[i];
    for (int i = threadIdx.x; i < nC; i += blockDim.x) sCs[i] = prm.cs[i];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, u = lane >> 4;
  // stage-1 operand row of this lane: rows 0-3 Re of atoms 0-3, 4-7 Im of atoms 0-3,
  // 8-11 Re of atoms 4-7, 12-15 Im of atoms 4-7; contraction index 4j+u
  const int arow = lane & 15;
  const int a_of_row = (arow & 3) + 4 * (arow >> 3);
  const bool is_im = (arow >> 2) & 1;
  const int part = u & 1;
  const int sel_off = ((part ^ int(is_im)) ? S : 0) + (u >> 1);   // Re/Im column + profile offset
  const float sgn = (is_im && part == 0) ? -1.f : 1.f;
  const float* arow_hat = sHat + a_of_row * B;

  float F[RT][NP];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int q = 0; q < NP; ++q) F[t][q] = prm.dftA[(t * NP + q) * 64 + lane];

  const int64_t nwt = (prm.P + 15) / 16;
  for (int64_t wt = int64_t(blockIdx.x) * 4 + wave; wt < nwt; wt += int64_t(gridDim.x) * 4) {
    const int64_t p = wt * 16 + col;
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

    for (int it = 0; it < K; ++it) {
      st.active = st.active && (norm2<L>(res) > kTau2 * nx2);
      if (!__any(st.active)) break;

      float best = -1.f;
      int bm = 0;
      float bop[NP];
      zero(bop);
      for (int g = 0; g < NG; ++g) {
        const float* hg = arow_hat + g * 8 * B;
        f32x4 acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < NKS; ++j) {
          const int k = L::harm(j);
          float av;
          if (k == 0) {
            const int s = 4 * j + u;
            const float h = hg[s < S ? s : 0];
            av = (!is_im && s < S) ? h : 0.f;
          } else {
            const int jj = L::pair(j);
            const int s = 2 * jj + (u >> 1);
            const int off = L::base(k) + 2 * jj + sel_off;
            const float h = hg[s < S ? off : 0];
            av = s < S ? sgn * h : 0.f;
          }
          acc[k] = mfma16(av, res[j], acc[k]);
        }
        // quarters 0,1 hold (Re, Im) of atom v, quarters 2,3 of atom v+4; the swap of
        // harmonics (2q, 2q+1) gives the operand [Re_k Im_k Re_k' Im_k'] of atoms v, v+4
        // (in place: operand of atom a < 4 is acc[2q][a], of atom a >= 4 acc[2q+1][a-4])
        f32x4 acc_pad = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < NP; ++q)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float x = acc[2 * q][v];
            float y = (2 * q + 1 < NQ) ? acc[2 * q + 1][v] : 0.f;
            swap32(x, y);
            acc[2 * q][v] = x;
            if (2 * q + 1 < NQ) acc[2 * q + 1][v] = y;
            else acc_pad[v] = y;
          }
        // pass 1 over the 8 atoms, software-pipelined by atom: the RT independent
        // MFMA chains of the next atom are issued before the |.| max of the current one
        auto opnd = [&](int q, int a) -> float {
          return a < 4 ? acc[2 * q][a] : (2 * q + 1 < NQ ? acc[2 * q + 1][a - 4] : acc_pad[a - 4]);
        };
        f32x4 ob[2][RT];
        auto chains = [&](int a, f32x4 (&o)[RT]) {
#pragma unroll
          for (int t = 0; t < RT; ++t) o[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < NP; ++q)
#pragma unroll
            for (int t = 0; t < RT; ++t) o[t] = mfma16(F[t][q], opnd(q, a), o[t]);
        };
        chains(0, ob[0]);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          if (a + 1 < 8) chains(a + 1, ob[(a + 1) & 1]);
          float amax = fabsf(ob[a & 1][0][0]);
#pragma unroll
          for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) amax = fmaxf(amax, fabsf(ob[a & 1][t][i]));
          const float am = max_quarters(amax);
          const bool gt = am > best;
          best = gt ? am : best;
          bm = gt ? g * 8 + a : bm;
#pragma unroll
          for (int q = 0; q < NP; ++q) bop[q] = gt ? opnd(q, a) : bop[q];
        }
      }
      int rs;
      float cval;
      {
        f32x4 o[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) o[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < NP; ++q)
#pragma unroll
          for (int t = 0; t < RT; ++t) o[t] = mfma16(F[t][q], bop[q], o[t]);
        float rb = -1.f, rv = 0.f;
        int rc = 0;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float val = fabsf(o[t][i]);
            const bool gt = val > rb;
            rb = gt ? val : rb;
            rv = gt ? o[t][i] : rv;
            rc = gt ? 16 * t + i : rc;
          }
        rc += 4 * u;
#pragma unroll
        for (int sh = 16; sh <= 32; sh *= 2) {
          const float ob = __shfl_xor(rb, sh), ov = __shfl_xor(rv, sh);
          const int oc = __shfl_xor(rc, sh);
          const bool take = (ob > rb) || (ob == rb && oc < rc);
          rb = take ? ob : rb;
          rv = take ? ov : rv;
          rc = take ? oc : rc;
        }
        rs = rc < R ? rc : R - 1;
        cval = rv;
      }
      pursuit_update<L, KMAX>(st, it, bm, rs, cval, sHat, sCs, prm.gramH, M, R, u, res);
    }
    const float rn2 = norm2<L>(res);
    if (valid && u == 0) write_codes<L, KMAX>(prm, p, st, rn2);
  }
}

// ============================================================== launchers
int num_cus() {
  static int cached = -1;
  if (cached < 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cached = n;
  }
  return cached;
}

// Persistent grid: at most as many blocks as fit on the device at once; each wave
// then walks the patch tiles with a stride of the whole grid.
template <class Kern, class... Args>
int launch_persistent(Kern kern, size_t lds, int64_t wave_tiles, int bpc, hipStream_t st, Args... args) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return int(e);
  }
  int64_t blocks = (wave_tiles + 3) / 4;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (bpc > 0 && bpc < per_cu) per_cu = bpc;
  const int64_t cap = int64_t(num_cus()) * per_cu;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(256), lds, st, args...);
  return int(hipGetLastError());
}

template <int S, int T, int RT, int KMAX>
int launch32(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  return launch_persistent(encode32_kernel<S, T, RT, KMAX>, encode_lds_bytes(t, RSC_TILE_32),
                           (prm.P + 31) / 32, t.enc_bpc, st, prm, t.NG);
}

template <int S, int T, int RT, int KMAX>
int launch16(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  return launch_persistent(encode16_kernel<S, T, RT, KMAX>, encode_lds_bytes(t, RSC_TILE_16),
                           (prm.P + 15) / 16, t.enc_bpc, st, prm);
}

template <int S, int T, int RT>
int k16(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  if (prm.K <= 2) return launch16<S, T, RT, 2>(t, prm, st);
  if (prm.K <= 4) return launch16<S, T, RT, 4>(t, prm, st);
  return launch16<S, T, RT, 8>(t, prm, st);
}

template <int S, int T>
int r16(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  const int rt = (t.R + 15) / 16;
  if (rt <= 1) return k16<S, T, 1>(t, prm, st);
  if (rt <= 2) return k16<S, T, 2>(t, prm, st);
  if (rt <= 4) return k16<S, T, 4>(t, prm, st);
  return k16<S, T, 8>(t, prm, st);
}

int r32(const DeviceTables& t, const EncodeParams& prm, hipStream_t st) {
  const int rt = (t.R + 31) / 32;
  if (prm.K <= 2) return rt <= 1 ? launch32<5, 5, 1, 2>(t, prm, st) : launch32<5, 5, 2, 2>(t, prm, st);
  return rt <= 1 ? launch32<5, 5, 1, 4>(t, prm, st) : launch32<5, 5, 2, 4>(t, prm, st);
}

}  // namespace

bool encode_supported(int S, int T) { return (S == 5 && T == 5) || (S == 7 && T == 7); }

size_t encode_lds_bytes(const DeviceTables& t, int tile) {
  const size_t cs = 2 * size_t(t.T + 1) * t.R;
  if (tile == RSC_TILE_32) {
    const int ng = (t.M + 15) / 16;
    return sizeof(float) * (size_t(ng) * stage1_steps(t.S, t.T) * 64 + size_t(ng) * 16 * t.B + cs);
  }
  const int ng = (t.M + 7) / 8;
  return sizeof(float) * (size_t(ng) * 8 * t.B + cs);
}

bool tile32_usable(const DeviceTables& t, int K) {
  return t.S == 5 && t.T == 5 && K <= 4 && t.R <= 64 && t.dictA &&
         encode_lds_bytes(t, RSC_TILE_32) <= 80 * 1024;
}

int launch_encode(const DeviceTables& t, int tile, const float* xhat, int64_t P, int K, int32_t* atom,
                  int32_t* angle, float* coef, float* resid2, void* stream) {
  if (P <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (tile == RSC_TILE_32) {
    if (!tile32_usable(t, K)) return int(hipErrorInvalidValue);
    EncodeParams prm{xhat, P, K, t.M, t.R, t.dictA, t.dictHat, t.dftA32, t.cs, t.gramH, atom, angle, coef, resid2};
    return r32(t, prm, st);
  }
  EncodeParams prm{xhat, P, K, t.M, t.R, nullptr, t.dictHat, t.dftA16, t.cs, t.gramH, atom, angle, coef, resid2};
  if (t.S == 5 && t.T == 5) return r16<5, 5>(t, prm, st);
  if (t.S == 7 && t.T == 7) return r16<7, 7>(t, prm, st);
  return int(hipErrorInvalidValue);
}

}  // namespace rsc
