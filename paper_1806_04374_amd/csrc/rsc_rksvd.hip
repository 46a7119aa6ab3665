// Dictionary update of rotational K-SVD (Fig. 2, the loop over atoms; Sec. II-C), in
// hat coordinates (Sec. II-E).
//
// The augmented dictionary is built once per outer iteration, so every atom is
// updated from the same codes and the same old dictionary, all atoms at once:
//   1. rk_partial_kernel, grid (patch chunk, atom): the patches of the chunk whose
//      code uses atom m are compacted in patch order; for each, with r0 the angle of
//      the first slot holding m and b the code without that entry,
//        y = S_{-r0} (x - sum_{j != i0} c_j S_{r_j} d_{m_j})
//      is formed in FP64 (thread b owns coordinate b) and y y^T is accumulated in
//      FP64 registers (thread b owns row b).  Each block writes its partial sum.
//   2. rk_eig_kernel, one block per atom: the partials are added in chunk order
//      (deterministic) into C_m = Y_m Y_m^T in LDS; its top eigenvector, the first
//      left singular vector of Y_m, comes from a Householder tridiagonalisation in
//      place, a multisection on Sturm counts for the largest eigenvalue, inverse
//      iteration on the tridiagonal matrix and the back-transformation through the
//      stored reflectors.  Its sign makes it agree with the old atom.
//   3. rk_reset_kernel: atoms that no patch uses take, in index order, the
//      directions of the patches with the largest coding error (positive ones only;
//      ties to the smaller patch index).
#include <hip/hip_runtime.h>

#include <cfloat>

#include "rsc_internal.h"

namespace rsc {
namespace {

constexpr int kQ = 16;  // pairs per batch in rk_partial_kernel

struct RkParams {
  const float* xhat;
  int64_t P;
  int K, M, R, B, S, T;
  const int32_t* atom;
  const int32_t* angle;
  const float* coef;
  const float* dict;     // [16 NG][B] old dictionary
  const double* cs64;    // [2][T+1][R]
  int NC;                // patch chunks
  int64_t chunk;         // patches per chunk
  double* partial;       // [M][NC][B][B]
  int32_t* counts;       // [M][NC]
};

// Coordinate b of S_theta v, with theta = sgn * 2 pi r / R, for a packed vector v in
// memory (harmonic k multiplied by exp(-i k theta)).
struct Coord {
  int k, part, partner;  // harmonic, 0 = Re / 1 = Im, index of the other part (b for k = 0)
};

__device__ __forceinline__ Coord coord_of(int b, int S) {
  if (b < S) return {0, 0, b};
  const int q = b - S, k = 1 + q / (2 * S), rem = q % (2 * S);
  return rem < S ? Coord{k, 0, b + S} : Coord{k, 1, b - S};
}

__device__ __forceinline__ double steered(double own, double other, const Coord& c, double cs, double sn, int sgn) {
  if (c.k == 0) return own;
  const double s = sgn * sn;
  // (a + i b) exp(-i k theta): Re' = a cos + b sin, Im' = b cos - a sin
  return c.part == 0 ? own * cs + other * s : own * cs - other * s;
}

template <int BT>
__global__ __launch_bounds__(BT) void rk_partial_kernel(RkParams prm) {
  extern __shared__ double ldsd[];
  const int B = prm.B, R = prm.R, K = prm.K, NQ = prm.T + 1;
  double* zb = ldsd;                                   // [kQ][BT]
  double* yb = zb + kQ * BT;                           // [kQ][BT]
  double* sc = yb + kQ * BT;                           // [2][NQ][R]
  int* queue = reinterpret_cast<int*>(sc + 2 * NQ * R);        // [BT] pair = p_local * 8 + i0
  int* wcount = queue + BT;                                      // [BT / 64 + 1]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = blockIdx.y, c = blockIdx.x;
  for (int i = t; i < 2 * NQ * R; i += BT) sc[i] = prm.cs64[i];
  const Coord cd = coord_of(t < B ? t : 0, prm.S);
  double acc[BT];
#pragma unroll
  for (int j = 0; j < BT; ++j) acc[j] = 0.0;
  int n = 0;
  const int64_t p0 = int64_t(c) * prm.chunk;
  const int64_t p1 = p0 + prm.chunk < prm.P ? p0 + prm.chunk : prm.P;
  __syncthreads();
  for (int64_t base = p0; base < p1; base += BT) {
    // compaction of the patches of this window that use atom m, in patch order
    const int64_t p = base + t;
    int i0 = -1;
    if (p < p1)
      for (int i = K - 1; i >= 0; --i)
        if (prm.atom[p * K + i] == m) i0 = i;
    const unsigned long long bal = __ballot(i0 >= 0);
    if (lane == 0) wcount[wave] = __popcll(bal);
    __syncthreads();
    int off = 0, total = 0;
    for (int w = 0; w < BT / 64; ++w) {
      off += w < wave ? wcount[w] : 0;
      total += wcount[w];
    }
    if (i0 >= 0) queue[off + __popcll(bal & ((1ull << lane) - 1))] = t * 8 + i0;
    __syncthreads();
    n += total;
    for (int q0 = 0; q0 < total; q0 += kQ) {
      const int nq = total - q0 < kQ ? total - q0 : kQ;
      // z = x - sum_{j != i0} c_j S_{r_j} d_{m_j}, coordinate t of each pair
      for (int q = 0; q < nq; ++q) {
        const int e = queue[q0 + q];
        const int64_t pp = base + (e >> 3);
        const int ii = e & 7;
        double z = 0.0;
        if (t < B) {
          z = prm.xhat[pp * B + t];
          for (int j = 0; j < K; ++j) {
            const int mj = prm.atom[pp * K + j];
            if (j == ii || mj < 0) continue;
            const int rj = prm.angle[pp * K + j];
            const float* d = prm.dict + size_t(mj) * B;
            const double v = steered(d[t], d[cd.partner], cd, sc[cd.k * R + rj], sc[(NQ + cd.k) * R + rj], 1);
            z -= double(prm.coef[pp * K + j]) * v;
          }
        }
        zb[q * BT + t] = z;
      }
      __syncthreads();
      // y = S_{-r0} z
      for (int q = 0; q < nq; ++q) {
        const int e = queue[q0 + q];
        const int64_t pp = base + (e >> 3);
        const int r0 = prm.angle[pp * K + (e & 7)];
        double y = 0.0;
        if (t < B)
          y = steered(zb[q * BT + t], zb[q * BT + cd.partner], cd, sc[cd.k * R + r0], sc[(NQ + cd.k) * R + r0], -1);
        yb[q * BT + t] = y;
      }
      __syncthreads();
      for (int q = 0; q < nq; ++q) {
        const double yt = yb[q * BT + t];
#pragma unroll
        for (int j = 0; j < BT; ++j) acc[j] = fma(yt, yb[q * BT + j], acc[j]);
      }
      __syncthreads();
    }
  }
  double* out = prm.partial + (size_t(m) * prm.NC + c) * size_t(B) * B;
  if (t < B) {
#pragma unroll
    for (int j = 0; j < BT; ++j)
      if (j < B) out[size_t(t) * B + j] = acc[j];
  }
  if (t == 0) prm.counts[m * prm.NC + c] = n;
}

// Block-wide sum of one double per thread (BT threads, scratch of BT doubles).
template <int BT>
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = BT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x (Sturm count).
__device__ int sturm_below(const double* d, const double* e, int n, double x, double tiny) {
  int cnt = 0;
  double q = d[0] - x;
  if (q == 0.0) q = -tiny;
  cnt += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (q == 0.0) q = -tiny;
    cnt += q < 0.0;
  }
  return cnt;
}

struct EigParams {
  const double* partial;  // [M][NC][B][B]
  const int32_t* counts;  // [M][NC]
  int M, NC, B;
  const float* dict_old;  // [M][B] (rows of the old dictionary)
  float* d_new;           // [M][B]
  int32_t* usage;         // [M]
};

template <int BT>
__global__ __launch_bounds__(BT) void rk_eig_kernel(EigParams prm) {
  extern __shared__ double ldsd[];
  const int n = prm.B, t = threadIdx.x, m = blockIdx.x;
  double* A = ldsd;                 // [n][n]
  double* v = A + n * n;            // [BT]
  double* pw = v + BT;              // [BT]
  double* red = pw + BT;            // [BT]
  double* d = red + BT;             // [BT]
  double* e = d + BT;               // [BT]
  double* beta = e + BT;            // [BT]
  double* z = beta + BT;            // [BT]
  int* cnt = reinterpret_cast<int*>(z + BT);  // [BT]
  // C_m = sum of the chunk partials, in chunk order
  int used = 0;
  for (int c = 0; c < prm.NC; ++c) used += prm.counts[m * prm.NC + c];
  if (t < n) {
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int c = 0; c < prm.NC; ++c) s += prm.partial[((size_t(m) * prm.NC + c) * n + t) * n + j];
      A[t * n + j] = s;
    }
  }
  if (t == 0) prm.usage[m] = used;
  if (used == 0) {
    if (t < n) prm.d_new[size_t(m) * n + t] = prm.dict_old[size_t(m) * n + t];
    return;
  }
  __syncthreads();
  // Householder tridiagonalisation: A = Q T Q^T, reflector k stored in A[k+1.., k]
  for (int k = 0; k + 2 < n; ++k) {
    const double xv = t > k && t < n ? A[t * n + k] : 0.0;
    const double xx = block_sum<BT>(xv * xv, red);
    const double x0 = A[(k + 1) * n + k];
    const double alpha = x0 >= 0.0 ? -sqrt(xx) : sqrt(xx);
    const double vv = xx - x0 * x0 + (x0 - alpha) * (x0 - alpha);
    if (vv <= 0.0) {                // the column is already reduced
      if (t == 0) {
        e[k] = x0;
        beta[k] = 0.0;
      }
      __syncthreads();
      continue;
    }
    const double bt = 2.0 / vv;
    if (t < n) v[t] = t > k + 1 ? A[t * n + k] : (t == k + 1 ? x0 - alpha : 0.0);
    __syncthreads();
    double pt = 0.0;
    if (t > k && t < n) {
      for (int j = k + 1; j < n; ++j) pt += A[t * n + j] * v[j];
      pt *= bt;
    }
    const double kk = 0.5 * bt * block_sum<BT>(pt * (t < n ? v[t] : 0.0), red);
    if (t < n) pw[t] = t > k ? pt - kk * v[t] : 0.0;
    __syncthreads();
    if (t > k && t < n)
      for (int j = k + 1; j < n; ++j) A[t * n + j] -= v[t] * pw[j] + pw[t] * v[j];
    __syncthreads();
    if (t > k && t < n) A[t * n + k] = v[t];
    if (t == 0) {
      e[k] = alpha;
      beta[k] = bt;
    }
    __syncthreads();
  }
  if (t < n) d[t] = A[t * n + t];
  if (t == 0) {
    if (n >= 2) e[n - 2] = A[(n - 1) * n + (n - 2)];
    if (n >= 2) beta[n - 2] = 0.0;
  }
  __syncthreads();
  // largest eigenvalue: multisection on Sturm counts inside the Gershgorin interval
  double lo = 0.0, hi = 0.0, scale = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    lo = i == 0 ? d[i] - r : fmin(lo, d[i] - r);
    hi = i == 0 ? d[i] + r : fmax(hi, d[i] + r);
    scale = fmax(scale, fabs(d[i]) + r);
  }
  const double tiny = DBL_MIN * fmax(scale, 1.0);
  for (int iter = 0; iter < 64 && hi - lo > 4.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)); ++iter) {
    const double x = lo + (hi - lo) * double(t + 1) / double(BT + 1);
    cnt[t] = sturm_below(d, e, n, x, tiny);
    __syncthreads();
    // the largest eigenvalue lies above the last point with fewer than n eigenvalues below
    int first = BT;
    for (int i = 0; i < BT; ++i)
      if (cnt[i] >= n) {
        first = i;
        break;
      }
    const double nlo = first == 0 ? lo : lo + (hi - lo) * double(first) / double(BT + 1);
    const double nhi = first == BT ? hi : lo + (hi - lo) * double(first + 1) / double(BT + 1);
    lo = nlo;
    hi = nhi;
    __syncthreads();
  }
  const double lam = 0.5 * (lo + hi);
  // eigenvector of the tridiagonal matrix: inverse iteration (Gaussian elimination with
  // partial pivoting of T - lam I), three sweeps from a constant start, one thread
  if (t == 0) {
    double* u1 = pw;   // super-diagonal after elimination
    double* u2 = v;    // second super-diagonal (fill-in from pivoting)
    double* dd = red;  // pivots
    int* piv = cnt;
    const double eps = DBL_EPSILON * fmax(scale, DBL_MIN);
    // factor once
    double a = d[0] - lam, b = n > 1 ? e[0] : 0.0;
    for (int i = 0; i + 1 < n; ++i) {
      const double cl = e[i], dn = d[i + 1] - lam, up = i + 2 < n ? e[i + 1] : 0.0;
      if (fabs(a) >= fabs(cl)) {       // no swap
        piv[i] = 0;
        const double mlt = a != 0.0 ? cl / a : 0.0;
        dd[i] = a != 0.0 ? a : eps;
        u1[i] = b;
        u2[i] = 0.0;
        z[i] = mlt;                     // multiplier
        a = dn - mlt * b;
        b = up;
      } else {                          // swap rows i and i+1
        piv[i] = 1;
        const double mlt = a / cl;
        dd[i] = cl;
        u1[i] = dn;
        u2[i] = up;
        z[i] = mlt;
        a = b - mlt * dn;
        b = -mlt * up;
      }
    }
    dd[n - 1] = a != 0.0 ? a : eps;
    double* y = A;                      // row 0 of A holds no reflector: free now
    for (int i = 0; i < n; ++i) y[i] = 1.0;
    for (int sweep = 0; sweep < 3; ++sweep) {
      // forward elimination on the right-hand side
      for (int i = 0; i + 1 < n; ++i) {
        if (piv[i]) {
          const double tmp = y[i];
          y[i] = y[i + 1];
          y[i + 1] = tmp - z[i] * y[i + 1];
        } else {
          y[i + 1] -= z[i] * y[i];
        }
      }
      // back substitution with the upper factor (diagonal dd, u1, u2)
      for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        if (i + 1 < n) s -= u1[i] * y[i + 1];
        if (i + 2 < n) s -= u2[i] * y[i + 2];
        y[i] = s / dd[i];
      }
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += y[i] * y[i];
      nrm = sqrt(nrm);
      for (int i = 0; i < n; ++i) y[i] /= nrm;
    }
  }
  __syncthreads();
  // the eigenvector of T is in A[0][0..n-1]; back-transform through the reflectors.
  // Row 0 of A is not part of any stored reflector (those live below the diagonal).
  double zt = t < n ? A[t] : 0.0;
  __syncthreads();
  if (t < n) z[t] = zt;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    if (beta[k] == 0.0) continue;
    const double vt = t > k && t < n ? A[t * n + k] : 0.0;
    const double s = beta[k] * block_sum<BT>(vt * (t < n ? z[t] : 0.0), red);
    if (t > k && t < n) z[t] -= s * vt;
    __syncthreads();
  }
  // unit norm, sign of the old atom (largest-magnitude coordinate positive on a tie at 0)
  const double zz = t < n ? z[t] : 0.0;
  const double nrm = sqrt(block_sum<BT>(zz * zz, red));
  const double dot = block_sum<BT>(t < n ? zz * double(prm.dict_old[size_t(m) * n + t]) : 0.0, red);
  double sgn = dot < 0.0 ? -1.0 : 1.0;
  if (dot == 0.0) {
    if (t == 0) {
      int im = 0;
      for (int i = 1; i < n; ++i)
        if (fabs(z[i]) > fabs(z[im])) im = i;
      red[0] = z[im] < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();
    sgn = red[0];
  }
  if (t < n) prm.d_new[size_t(m) * n + t] = float(sgn * zz / nrm);
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

// Sum of a float array in FP64 (single block; for the coding-error history).
__global__ __launch_bounds__(256) void rk_sum_kernel(const float* x, int64_t n, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

int rksvd_chunks(int M, int64_t P) {
  int nc = (2048 + M - 1) / M;
  const int64_t cap = (P + 1023) / 1024;
  if (nc > cap) nc = int(cap);
  return nc < 1 ? 1 : (nc > 64 ? 64 : nc);
}

size_t rksvd_workspace_bytes(const DeviceTables& t, int64_t P) {
  const int NC = rksvd_chunks(t.M, P);
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return al(sizeof(double) * size_t(t.M) * NC * t.B * t.B) + al(sizeof(int32_t) * size_t(t.M) * NC) +
         al(sizeof(double) * 8);
}

int launch_rksvd_update(const DeviceTables& t, const float* xhat, int64_t P, int K, const int32_t* atom,
                        const int32_t* angle, const float* coef, const float* resid2, void* ws,
                        float* d_new, int32_t* usage, int32_t* reset, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int NC = rksvd_chunks(t.M, P);
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  char* w = reinterpret_cast<char*>(ws);
  double* partial = reinterpret_cast<double*>(w);
  int32_t* counts = reinterpret_cast<int32_t*>(w + al(sizeof(double) * size_t(t.M) * NC * t.B * t.B));
  RkParams prm{xhat, P, K, t.M, t.R, t.B, t.S, t.T, atom, angle, coef, t.dictHat, t.cs64, NC,
               (P + NC - 1) / NC, partial, counts};
  const int NQ = t.T + 1;
  EigParams ep{partial, counts, t.M, NC, t.B, t.dictHat, d_new, usage};
  auto run = [&](auto partial_kern, auto eig_kern, int bt) -> int {
    const size_t lds1 = sizeof(double) * (2 * kQ * size_t(bt) + 2 * size_t(NQ) * t.R) + sizeof(int) * (bt + bt / 64 + 1);
    const size_t lds2 = sizeof(double) * (size_t(t.B) * t.B + 7 * size_t(bt)) + sizeof(int) * bt;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(partial_kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds1));
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(eig_kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(lds2));
    if (e != hipSuccess) return int(e);
    hipLaunchKernelGGL(partial_kern, dim3(unsigned(NC), unsigned(t.M)), dim3(bt), lds1, st, prm);
    e = hipGetLastError();
    if (e != hipSuccess) return int(e);
    hipLaunchKernelGGL(eig_kern, dim3(unsigned(t.M)), dim3(bt), lds2, st, ep);
    return int(hipGetLastError());
  };
  int e = t.B <= 64 ? run(rk_partial_kernel<64>, rk_eig_kernel<64>, 64)
                    : run(rk_partial_kernel<128>, rk_eig_kernel<128>, 128);
  if (e) return e;
  ResetParams rp{xhat, resid2, P, t.M, t.B, usage, d_new, reset};
  hipLaunchKernelGGL(rk_reset_kernel, dim3(1), dim3(256), 0, st, rp);
  return int(hipGetLastError());
}

int launch_sum(const float* x, int64_t n, double* out, void* stream) {
  hipLaunchKernelGGL(rk_sum_kernel, dim3(1), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), x, n, out);
  return int(hipGetLastError());
}

}  // namespace rsc
