// Device helpers shared by the gfx950 kernels: MFMA wrappers, cross-lane swaps,
// the distribution of one patch's packed hat coordinates over the lanes that hold
// it, and the per-patch least-squares update of orthogonal matching pursuit.
//
// MFMA operand layouts used here (single block):
//   v_mfma_f32_32x32x2f32: lane l supplies A[l%32][l/32] and B[l/32][l%32];
//     accumulator register v of lane l holds D[8(v/4) + 4(l/32) + v%4][l%32].
//   v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l/16] and B[l/16][l%16];
//     accumulator register v of lane l holds D[4(l/16) + v][l%16].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

namespace rsc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Early stop of the pursuit when ||r||^2 <= kTau2 ||x||^2 (tau = 1e-5).
constexpr float kTau2 = 1e-10f;

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int N>
__device__ __forceinline__ void zero(float (&x)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = 0.f;
}

// Exchange lanes 32..63 of x with lanes 0..31 of y: afterwards x = [x_lo | y_lo],
// y = [x_hi | y_hi].
__device__ __forceinline__ void swap32(float& x, float& y) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}

// Exchange the odd 16-lane rows of x with the even rows of y: afterwards
// x = [x0 y0 x2 y2], y = [x1 y1 x3 y3] (rows of 16 lanes).
__device__ __forceinline__ void swap16(float& x, float& y) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}

// Maximum of x over the two half-waves (the result is the same in every lane pair).
__device__ __forceinline__ float max_halves(float x) {
  float a = x, b = x;
  swap32(a, b);
  return fmaxf(a, b);
}

// The same for x >= 0 (a maximum of absolute values): non-negative floats order like their
// bit patterns, so an integer maximum needs none of the NaN quieting a float maximum of
// cross-lane values costs (a NaN, if any, wins instead of being dropped).
__device__ __forceinline__ float max_halves_nonneg(float x) {
  float a = x, b = x;
  swap32(a, b);
  return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}

__device__ __forceinline__ float max_quarters_nonneg(float x) {
  float a = x, b = x;
  swap16(a, b);
  return max_halves_nonneg(__uint_as_float(max(__float_as_uint(a), __float_as_uint(b))));
}

// Maximum of x over the four quarter-waves.
__device__ __forceinline__ float max_quarters(float x) {
  float a = x, b = x;
  swap16(a, b);
  return max_halves(fmaxf(a, b));
}

// Calls f(std::integral_constant<int, i>{}) for i = 0 .. N-1, so that the body can evaluate
// layout lookups of index i as constant expressions.  The ragged layout's lookups loop over
// harmonics; called from an unrolled loop, the optimiser does not always fold them, and an
// accumulator array indexed by an unfolded value is demoted to private memory.
template <class F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// ----------------------------------------------------------------------------
// Coordinate layouts.  A patch's B packed hat coordinates are harmonic-major with Sk(k)
// radial profiles (or annuli) in harmonic k: [k=0: Sk(0)], then for each k >= 1
// [Re: Sk(k)][Im: Sk(k)].  They are spread over W lanes (W = 2: the two half-waves of a
// 32x32 tile; W = 4: the four quarter-waves of a 16x16 tile).  Register j of sub-lane u
// holds one coordinate:
//   harmonic 0 block (j < J0): profile s = W j + u;
//   harmonic k >= 1 block (joff(k) <= j < joff(k+1)): the pair index jj = j - joff(k)
//     selects profile s = SW jj + soff(u) and part(u) (0 = Re, 1 = Im).
// These are also the contraction orders of the stage-1 MFMAs.  The profile counts come
// from C (C::T and C::sk(k)): the same S for every harmonic in the (S, T) grid of Gaussian
// profiles, ragged for the paper's annular basis, whose harmonic k lives on the annuli
// whose cut-off reaches k.
template <class C, int W_>
struct LayoutBase {
  static constexpr int W = W_, T = C::T, NQ = T + 1;
  static constexpr int SW = W / 2;                       // profiles advanced per k>=1 step
  __host__ __device__ static constexpr int Sk(int k) { return C::sk(k); }
  static constexpr int S = C::sk(0);                     // profiles of harmonic 0 (the most)
  static constexpr int J0 = (S + W - 1) / W;
  __host__ __device__ static constexpr int J1k(int k) { return (2 * Sk(k) + W - 1) / W; }
  __host__ __device__ static constexpr int joff(int k) {
    int j = J0;
    for (int q = 1; q < k; ++q) j += J1k(q);
    return k == 0 ? 0 : j;
  }
  static constexpr int NKS = joff(T + 1);
  __host__ __device__ static constexpr int base(int k) {
    int b = Sk(0);
    for (int q = 1; q < k; ++q) b += 2 * Sk(q);
    return k == 0 ? 0 : b;
  }
  static constexpr int B = base(T + 1);
  __host__ __device__ static constexpr int harm(int j) {
    int k = 0;
    while (k < T && j >= joff(k + 1)) ++k;
    return k;
  }
  __host__ __device__ static constexpr int pair(int j) { return j < J0 ? j : j - joff(harm(j)); }
  __host__ __device__ static constexpr int soff(int u) { return W == 2 ? 0 : (u >> 1); }
  __host__ __device__ static constexpr int part(int u) { return W == 2 ? u : (u & 1); }
  // profile index of register j in sub-lane u
  __host__ __device__ static constexpr int prof(int j, int u) {
    return harm(j) == 0 ? W * j + u : SW * pair(j) + soff(u);
  }
  // packed coordinate of register j in sub-lane u, or -1 for padding
  __host__ __device__ static constexpr int coord(int j, int u) {
    return prof(j, u) >= Sk(harm(j)) ? -1
           : (harm(j) == 0 ? prof(j, u) : base(harm(j)) + part(u) * Sk(harm(j)) + prof(j, u));
  }
  // coord(J, u) for a run-time sub-lane u: the W candidates are constants, so the harmonic
  // search inside coord never runs on the device (left to the optimiser it can stay a
  // run-time loop nest for layouts with many harmonics)
  template <int J>
  __device__ static int coord_u(int u) {
    constexpr int c0 = coord(J, 0), c1 = coord(J, 1);
    constexpr int c2 = W == 4 ? coord(J, 2) : -1, c3 = W == 4 ? coord(J, 3) : -1;
    return u == 0 ? c0 : u == 1 ? c1 : u == 2 ? c2 : c3;
  }
};

// The (S, T) grid: every harmonic 0..T on all S profiles.
template <int S_, int T_>
struct UniformCounts {
  static constexpr int T = T_;
  __host__ __device__ static constexpr int sk(int) { return S_; }
};

template <int S, int T, int W>
using Layout = LayoutBase<UniformCounts<S, T>, W>;

// The paper's annular basis (eq. (5)-(7)) at N = 11 and N = 15: per-annulus cut-offs
// T_s = (1, 3, 8, 11, 15) and (1, 3, 8, 11, 13, 18, 19) (half the circumference, lowered
// where the annulus' pixels cannot carry that many harmonics); harmonic k lives on the
// annuli with T_s >= k.
struct AnnularCounts11 {
  static constexpr int T = 15;
  __host__ __device__ static constexpr int sk(int k) {
    return k <= 1 ? 5 : k <= 3 ? 4 : k <= 8 ? 3 : k <= 11 ? 2 : 1;
  }
};
struct AnnularCounts15 {
  static constexpr int T = 19;
  __host__ __device__ static constexpr int sk(int k) {
    return k <= 1 ? 7 : k <= 3 ? 6 : k <= 8 ? 5 : k <= 11 ? 4 : k <= 13 ? 3 : k <= 18 ? 2 : 1;
  }
};

// Stage-2 operand of atom m for this lane's patch in the two-half-wave layout (W = 2):
// op[k] = Re C_k in the low half-wave and Im C_k in the high one, C_k = sum_s conj(d_{m,s,k})
// x_{s,k}, from the atom's row of the packed dictionary.  Each half-wave multiplies its
// residual coordinates (Re parts in the low half, Im parts in the high one; profiles 2j + u
// of harmonic 0) with the matching parts of the atom, and one swap per harmonic adds the
// two halves' partial sums into the operand layout.  Padding coordinates of the residual
// are 0, so what the atom row holds there does not matter.
template <class L>
__device__ __forceinline__ void atom_operand(const float* __restrict__ hat, int m, int u,
                                             const float (&res)[L::NKS], float (&op)[L::NQ]) {
  static_assert(L::W == 2, "two half-waves per patch");
  const float* d = hat + m * L::B;
  float p0 = 0.f;
#pragma unroll
  for (int j = 0; j < L::J0; ++j) {
    const int s = 2 * j + u;
    p0 = fmaf(d[s < L::S ? s : 0], res[j], p0);
  }
  {
    float x = p0, y = 0.f;
    swap32(x, y);
    op[0] = x + y;
  }
  // low half-wave (Re parts): Re += dRe r, Im -= dIm r; high half-wave (Im parts):
  // Re += dIm r, Im += dRe r
  const float sg = u ? 1.f : -1.f;
#pragma unroll
  for (int k = 1; k <= L::T; ++k) {
    const float* dA = d + L::base(k) + (u ? L::Sk(k) : 0);
    const float* dB = d + L::base(k) + (u ? 0 : L::Sk(k));
    float pr = 0.f, pi = 0.f;
#pragma unroll
    for (int jj = 0; jj < L::J1k(k); ++jj) {
      const int j = L::joff(k) + jj;
      if (jj < L::Sk(k)) {
        pr = fmaf(dA[jj], res[j], pr);
        pi = fmaf(dB[jj], res[j], pi);
      }
    }
    float x = pr, y = sg * pi;
    swap32(x, y);
    op[k] = x + y;
  }
}

// Sum over the W lanes of a patch; bit-identical in all of them.
template <int W>
__device__ __forceinline__ float patch_sum(float x) {
  if (W == 4) x = x + __shfl_xor(x, 16);
  return x + __shfl_xor(x, 32);
}

// acc += alpha * S_r d_m on the coordinates sub-lane u holds (steering computed on
// the fly, nothing else kept in registers).  Steering multiplies harmonic k by
// e^{-i k theta}: Re' = c Re + s Im, Im' = c Im - s Re.  A lane reads its own part of the
// atom's pair (pA: Re on Re lanes, Im on Im lanes) and the other part (pB), with alpha
// folded into the harmonic's two factors, so a coordinate costs two fused multiply-adds.
template <class L>
__device__ __forceinline__ void steer_axpy(float (&acc)[L::NKS], float alpha, const float* __restrict__ hat,
                                           const float* __restrict__ cs, int R, int m, int r, int u) {
  const float* d = hat + m * L::B;
  // harmonic 0: profile W j + u
#pragma unroll
  for (int j = 0; j < L::J0; ++j) {
    const int s = L::W * j + u;
    const bool valid = s < L::Sk(0);
    acc[j] = fmaf(valid ? alpha : 0.f, d[valid ? s : 0], acc[j]);
  }
  const int pt = L::part(u), so = L::soff(u);
  const float as = pt ? -alpha : alpha;
  // harmonics as compile-time indices: the register of each coordinate is a constant
  static_for<L::T>([&](auto K1) {
    constexpr int k = decltype(K1)::value + 1;
    constexpr int bk = L::base(k), nk = L::Sk(k), j0 = L::joff(k), nj = L::J1k(k);
    const float* pA = d + bk + (pt ? nk : 0) + so;
    const float* pB = d + bk + (pt ? 0 : nk) + so;
    const float ck = alpha * cs[k * R + r];
    const float sk = as * cs[(L::NQ + k) * R + r];
#pragma unroll
    for (int jj = 0; jj < nj; ++jj) {
      if (L::SW * jj >= nk) continue;                   // padding in every lane
      float a = ck, b = sk;
      int off = L::SW * jj;
      if (L::SW * jj + L::SW - 1 >= nk) {               // padding in some lanes
        const bool valid = L::SW * jj + so < nk;
        a = valid ? a : 0.f;
        b = valid ? b : 0.f;
        off = valid ? off : -so;
      }
      acc[j0 + jj] = fmaf(pA[off], a, fmaf(pB[off], b, acc[j0 + jj]));
    }
  });
}

// <S_{ra} d_a, S_{rb} d_b> from the per-pair harmonic table
//   H[(a M + b)(2T+1) + 0]    = sum_s d_{a,s,0} d_{b,s,0}
//   H[(a M + b)(2T+1) + 2k-1] = Re sum_s conj(w_{a,s,k}) w_{b,s,k}
//   H[(a M + b)(2T+1) + 2k]   = Im sum_s conj(w_{a,s,k}) w_{b,s,k}
// as H_0 + sum_k [cos(k phi) Re H_k - sin(k phi) Im H_k], phi = 2 pi (ra - rb) / R.
template <int T>
__device__ __forceinline__ float pair_gram(const float* __restrict__ H, const float* __restrict__ cs, int M,
                                           int R, int a, int ra, int b, int rb) {
  const float* h = H + (size_t(a) * M + b) * (2 * T + 1);
  int dr = ra - rb;
  dr += dr < 0 ? R : 0;
  float g = h[0];
#pragma unroll
  for (int k = 1; k <= T; ++k) g += cs[k * R + dr] * h[2 * k - 1] - cs[(T + 1 + k) * R + dr] * h[2 * k];
  return g;
}

// Per-patch state of the pursuit (identical in the W lanes of a patch).
template <int KMAX>
struct PursuitState {
  int selm[KMAX], selr[KMAX];
  float L[KMAX][KMAX];   // Cholesky factor of the Gram matrix of the selected columns
  float bv[KMAX];        // <selected column i, x>
  float cf[KMAX];        // current least-squares coefficients
  int nsel;
  bool active;
};

template <int KMAX>
__device__ __forceinline__ void init_state(PursuitState<KMAX>& st, bool valid) {
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    st.selm[i] = -1;
    st.selr[i] = -1;
    st.bv[i] = 0.f;
    st.cf[i] = 0.f;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) st.L[i][j] = 0.f;
  }
  st.nsel = 0;
  st.active = valid;
}

// FP64 re-solve thresholds on k ||L^{-1}||_F^2, an upper bound on cond_2 of the Gram matrix
// of the selected columns.  FP32 handles: FP32 rounding of the Gram entries (a few u) is
// amplified by up to the bound in the coefficients, so 1e3 keeps them within about 1e-4 of
// exact.  16-bit handles: the FP64 trigger of their precision form, cond > 1e6.
constexpr float kCondMaxFp32 = 1e3f;
constexpr float kCondMax16 = 1e6f;

// Tables of the least-squares step: the FP32 pair table of the Cholesky update and the
// FP64 pair and cos/sin tables plus the input coordinates of the FP64 re-solve.
struct LsTables {
  const float* gramH;      // [M][M][2T+1] (pair_gram)
  const double* gramH64;   // the same in FP64
  const double* cs64;      // [2][T+1][R] cos, sin in FP64
  const float* xhat;       // [P][B] input coordinates
  int M, R;
  float cond_max;          // FP64 re-solve once k ||L^{-1}||_F^2 exceeds this
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
  if (pr >= L::Sk(k)) return 0.0;
  if (k == 0) return double(d[pr]);
  const double c = cs[k * R + r], s = cs[(L::NQ + k) * R + r];
  const double ca = L::part(u) ? -s : c, cb = L::part(u) ? c : s;
  return double(d[L::base(k) + pr]) * ca + double(d[L::base(k) + L::Sk(k) + pr]) * cb;
}

// Sum of a double over the W lanes of a patch.
template <int W>
__device__ __forceinline__ double patch_sum64(double x) {
  if (W == 4) x = x + __shfl_xor(x, 16);
  return x + __shfl_xor(x, 32);
}

// FP64 least squares over the it selected columns plus (ms, rs), for the lanes with
// go set.  Returns whether the new column was accepted (its FP64 pivot is more than
// 1e-14 of its squared norm: a column numerically inside the span of the selected ones
// ends the pursuit); then the coefficients, the selection and the residual
// x_hat - sum_i a_i column_i are replaced.  The factor and the solution live in
// dynamically indexed local arrays (private memory): the path is rare, and its loops
// indexed at run time keep the factor out of the registers of the pursuit's main path.
template <class L, int KMAX>
__device__ __forceinline__ bool ls_solve64(PursuitState<KMAX>& st, int it, int ms, int rs, bool go,
                                                     const float* hat, const LsTables& tb, int64_t p, int u,
                                                     float (&res)[L::NKS]) {
  const int M = tb.M, R = tb.R;
  int cm[KMAX], cr[KMAX];
  double Lc[KMAX][KMAX], y[KMAX], a[KMAX];
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    cm[i] = i < it ? (st.selm[i] < 0 ? 0 : st.selm[i]) : ms;
    cr[i] = i < it ? (st.selr[i] < 0 ? 0 : st.selr[i]) : rs;
  }
  bool good = go;
#pragma unroll 1
  for (int i = 0; i <= it; ++i) {
#pragma unroll 1
    for (int j = 0; j <= i; ++j) {
      const double g0 = pair_gram64<L::T>(tb.gramH64, tb.cs64, M, R, cm[i], cr[i], cm[j], cr[j]);
      double g = g0;
#pragma unroll 1
      for (int l = 0; l < j; ++l) g -= Lc[i][l] * Lc[j][l];
      if (j < i) {
        Lc[i][j] = g / Lc[j][j];
      } else {
        if (i == it) good = good && g > 1e-14 * g0;
        Lc[i][i] = sqrt(g > 1e-300 ? g : 1e-300);
      }
    }
  }
  // b_i = <column_i, x_hat> over this lane's coordinates, completed across the patch's lanes
  const int64_t pp = good ? p : 0;
#pragma unroll 1
  for (int i = 0; i <= it; ++i) {
    double b = 0.0;
#pragma unroll 1
    for (int j = 0; j < L::NKS; ++j) {
      const int c = L::coord(j, u);
      const double x = (good && c >= 0) ? double(tb.xhat[pp * L::B + c]) : 0.0;
      b += steer64<L>(hat, tb.cs64, R, cm[i], cr[i], j, u) * x;
    }
    b = patch_sum64<L::W>(b);
#pragma unroll 1
    for (int l = 0; l < i; ++l) b -= Lc[i][l] * y[l];
    y[i] = b / Lc[i][i];
  }
#pragma unroll 1
  for (int i = it; i >= 0; --i) {
    double s = y[i];
#pragma unroll 1
    for (int l = i + 1; l <= it; ++l) s -= Lc[l][i] * a[l];
    a[i] = s / Lc[i][i];
  }
  // the new residual goes through a local array first: the loop over its coordinates runs
  // at run time, and only the copy into res (indexed at compile time) touches the registers
  float rn[L::NKS];
#pragma unroll 1
  for (int j = 0; j < L::NKS; ++j) {
    const int c = L::coord(j, u);
    double r = (good && c >= 0) ? double(tb.xhat[pp * L::B + c]) : 0.0;
#pragma unroll 1
    for (int i = 0; i <= it; ++i) r -= a[i] * steer64<L>(hat, tb.cs64, R, cm[i], cr[i], j, u);
    rn[j] = float(r);
  }
#pragma unroll
  for (int j = 0; j < L::NKS; ++j) res[j] = good ? rn[j] : res[j];
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    st.cf[i] = (good && i <= it) ? float(a[i]) : st.cf[i];
    st.selm[i] = (good && i == it) ? ms : st.selm[i];
    st.selr[i] = (good && i == it) ? rs : st.selr[i];
  }
  return good;
}

// Extra per-patch state of the least-squares step.
template <int KMAX>
struct LsState {
  float Ld[KMAX];     // 1 / L[i][i]
  float condF;        // ||L^{-1}||_F^2
  bool fp64;          // the patch's least squares run in FP64 from now on
};

template <int KMAX>
__device__ __forceinline__ void init_ls(LsState<KMAX>& ls) {
#pragma unroll
  for (int i = 0; i < KMAX; ++i) ls.Ld[i] = 0.f;
  ls.condF = 0.f;
  ls.fp64 = false;
}

// Least-squares step after the it-th selection (ms, rs) whose signed correlation with the
// current residual is cval (Cholesky-based OMP):
//   g_i = <column i, new column> (pair table), <new, x> = cval + sum_i g_i a_i,
//   L is extended by w = L^{-1} g and sqrt(<new,new> - |w|^2),
//   the coefficients solve L L^T a = [<column i, x>]_i,
//   the residual moves by -sum_i (a_i - a_i^old) column_i.
// It also tracks k ||L^{-1}||_F^2, an upper bound on cond_2 of the Gram matrix of the k
// selected unit columns (||G||_2 <= k, ||G^{-1}||_2 <= ||L^{-1}||_F^2).  Once the bound
// exceeds tb.cond_max, or the new FP32 pivot is below 1e-6 of the column's squared norm,
// the patch's least squares are re-solved from scratch in FP64 for this and every later
// step (ls_solve64).  it is a run-time value (the same in the whole wave); all state arrays
// are indexed statically with predicates so that they stay in registers.  Returns whether
// this lane went through the FP64 solve.
template <class L, int KMAX>
__device__ __forceinline__ bool ls_update(PursuitState<KMAX>& st, LsState<KMAX>& ls, int it, int ms, int rs,
                                          float cval, const float* hat, const float* cs, const LsTables& tb,
                                          int64_t p, int u, float (&res)[L::NKS]) {
  const int M = tb.M, R = tb.R;
  bool dup = false;
#pragma unroll
  for (int i = 0; i < KMAX; ++i) dup = dup || (i < it && st.selm[i] == ms && st.selr[i] == rs);
  const bool upd = st.active && !dup;

  const float dd = pair_gram<L::T>(tb.gramH, cs, M, R, ms, rs, ms, rs);
  float gcol[KMAX];
  float bx = cval;
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    gcol[i] = 0.f;
    if (i < it) {
      const int mi = st.selm[i] < 0 ? 0 : st.selm[i], ri = st.selr[i] < 0 ? 0 : st.selr[i];
      gcol[i] = pair_gram<L::T>(tb.gramH, cs, M, R, mi, ri, ms, rs);
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
    w[i] = i < it ? s * ls.Ld[i] : 0.f;
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
    z[i] = i < it ? s * ls.Ld[i] : 0.f;
    zz += z[i] * z[i];
  }
  const float Fn = ls.condF + (zz + 1.f) / fmaxf(l2, 1e-30f);
  const bool ok32 = !ls.fp64 && l2 > 1e-6f * dd && float(it + 1) * Fn <= tb.cond_max;
  const bool up32 = upd && ok32;
  const bool go64 = upd && !ok32;
#pragma unroll
  for (int r = 0; r < KMAX; ++r) {
    const bool row = up32 && r == it;
#pragma unroll
    for (int i = 0; i < r; ++i) st.L[r][i] = row ? w[i] : st.L[r][i];
    ls.Ld[r] = row ? rsqrtf(l2) : ls.Ld[r];
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
    y[i] = i <= it ? s * ls.Ld[i] : 0.f;
  }
#pragma unroll
  for (int i = KMAX - 1; i >= 0; --i) {
    float s = y[i];
#pragma unroll
    for (int j = i + 1; j < KMAX; ++j) s -= st.L[j][i] * an[j];
    an[i] = i <= it ? s * ls.Ld[i] : 0.f;
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
  ls.condF = up32 ? Fn : ls.condF;
  bool ok64 = false;
  if (__any(go64)) ok64 = ls_solve64<L, KMAX>(st, it, ms, rs, go64, hat, tb, p, u, res);
  ls.fp64 = ls.fp64 || ok64;
  st.nsel = (up32 || ok64) ? it + 1 : st.nsel;
  st.active = up32 || ok64;
  return go64;
}

template <class L>
__device__ __forceinline__ float norm2(const float (&v)[L::NKS]) {
  float a = 0.f;
#pragma unroll
  for (int j = 0; j < L::NKS; ++j) a += v[j] * v[j];
  return patch_sum<L::W>(a);
}

}  // namespace rsc
