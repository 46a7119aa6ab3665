// Host-side FP64 construction of the discrete steerable basis (Sec. II-D,
// eq. (5)-(7)) and its biorthogonal partner (Phi^T Phi)^{-1} Phi^T.
//
// Plain C++ with no device code; the GPU kernels only ever see FP32 copies.
#include "rsc_internal.h"

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

namespace rsc {

namespace {

// Cyclic Jacobi eigen-decomposition of a real symmetric n x n matrix A (row-major).
// On return w holds the eigenvalues and V (row-major) the eigenvectors as columns.
void jacobi_eig(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& V) {
  V.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[size_t(p) * n + q] * A[size_t(p) * n + q];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[size_t(p) * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = A[size_t(p) * n + p], aqq = A[size_t(q) * n + q];
        double tau = (aqq - app) / (2.0 * apq);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
          double akp = A[size_t(k) * n + p], akq = A[size_t(k) * n + q];
          A[size_t(k) * n + p] = c * akp - s * akq;
          A[size_t(k) * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
          double apk = A[size_t(p) * n + k], aqk = A[size_t(q) * n + k];
          A[size_t(p) * n + k] = c * apk - s * aqk;
          A[size_t(q) * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[size_t(k) * n + p], vkq = V[size_t(k) * n + q];
          V[size_t(k) * n + p] = c * vkp - s * vkq;
          V[size_t(k) * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[size_t(i) * n + i];
}

// In-place Cholesky A = L L^T of an n x n SPD matrix (row-major, lower part used).
bool cholesky(int n, std::vector<double>& A) {
  for (int j = 0; j < n; ++j) {
    double d = A[size_t(j) * n + j];
    for (int k = 0; k < j; ++k) d -= A[size_t(j) * n + k] * A[size_t(j) * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    A[size_t(j) * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[size_t(i) * n + j];
      for (int k = 0; k < j; ++k) v -= A[size_t(i) * n + k] * A[size_t(j) * n + k];
      A[size_t(i) * n + j] = v / d;
    }
    for (int k = j + 1; k < n; ++k) A[size_t(j) * n + k] = 0.0;
  }
  return true;
}

// Gram matrix, condition number and biorthogonal partner of a packed real synthesis
// matrix phid [n][B] over the disk pixels pix; fills out (except S and T).
bool finish_basis(int N, const std::vector<int>& pix, const std::vector<double>& phid, int B, HostBasis& out,
                  std::string& err) {
  const int n = int(pix.size());
  // Gram, its Cholesky factor, eigenvalues for the condition number
  std::vector<double> G(size_t(B) * B, 0.0);
  for (int a = 0; a < B; ++a)
    for (int b = 0; b <= a; ++b) {
      double v = 0.0;
      for (int p = 0; p < n; ++p) v += phid[size_t(p) * B + a] * phid[size_t(p) * B + b];
      G[size_t(a) * B + b] = G[size_t(b) * B + a] = v;
    }
  std::vector<double> w, V;
  jacobi_eig(B, G, w, V);
  double wmin = w[0], wmax = w[0];
  for (double x : w) {
    wmin = std::min(wmin, x);
    wmax = std::max(wmax, x);
  }
  std::vector<double> L = G;
  if (!(wmin > 0.0) || !cholesky(B, L)) {
    err = "basis Gram matrix is not positive definite";
    return false;
  }
  // pinv_d = G^{-1} Phi_d^T : solve L L^T X = Phi_d^T column by column (pixel by pixel)
  std::vector<double> pinvd(size_t(B) * n);
  std::vector<double> y(B);
  for (int p = 0; p < n; ++p) {
    for (int i = 0; i < B; ++i) {
      double v = phid[size_t(p) * B + i];
      for (int k = 0; k < i; ++k) v -= L[size_t(i) * B + k] * y[k];
      y[i] = v / L[size_t(i) * B + i];
    }
    for (int i = B - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < B; ++k) v -= L[size_t(k) * B + i] * y[k];
      y[i] = v / L[size_t(i) * B + i];
    }
    for (int i = 0; i < B; ++i) pinvd[size_t(i) * n + p] = y[i];
  }
  out.N = N;
  out.B = B;
  out.n_pix = n;
  out.cond = wmax / wmin;
  out.pix = pix;
  out.phi.assign(size_t(N) * N * B, 0.0);
  out.pinv.assign(size_t(B) * N * N, 0.0);
  for (int p = 0; p < n; ++p)
    for (int b = 0; b < B; ++b) {
      out.phi[size_t(pix[p]) * B + b] = phid[size_t(p) * B + b];
      out.pinv[size_t(b) * N * N + pix[p]] = pinvd[size_t(b) * n + p];
    }
  return true;
}

}  // namespace

bool build_basis(int N, int S, int T, const double* centres_in, double sigma_in, HostBasis& out,
                 std::string& err) {
  const double half = 0.5 * N;
  std::vector<double> centres(S);
  double sigma = sigma_in;
  if (centres_in) {
    for (int s = 0; s < S; ++s) centres[s] = centres_in[s];
    if (!(sigma > 0.0)) sigma = half / S;
  } else {
    sigma = half / S;
    for (int s = 0; s < S; ++s) centres[s] = (s + 1) * sigma;
  }
  const int B = S * (2 * T + 1);
  const double c0 = 0.5 * (N - 1);
  // disk pixels in row-major order
  std::vector<int> pix;
  std::vector<double> rho, th;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double x = j - c0, y = c0 - i;
      double r = std::sqrt(x * x + y * y);
      if (r < half) {
        pix.push_back(i * N + j);
        rho.push_back(r);
        th.push_back(std::atan2(y, x));
      }
    }
  const int n = int(pix.size());
  if (B > n) {
    err = "basis has more columns than disk pixels";
    return false;
  }
  // complex columns per harmonic: re/im [T+1][S][n]
  std::vector<double> cre(size_t(T + 1) * S * n), cim(size_t(T + 1) * S * n);
  auto at = [&](int k, int s, int p) { return (size_t(k) * S + s) * n + p; };
  for (int k = 0; k <= T; ++k) {
    for (int s = 0; s < S; ++s) {
      double nrm = 0.0;
      for (int p = 0; p < n; ++p) {
        double g = std::exp(-(rho[p] - centres[s]) * (rho[p] - centres[s]) / (2.0 * sigma * sigma));
        double re = g * std::cos(k * th[p]), im = g * std::sin(k * th[p]);
        if (k != 0 && rho[p] == 0.0) re = im = 0.0;
        cre[at(k, s, p)] = re;
        cim[at(k, s, p)] = im;
        nrm += re * re + im * im;
      }
      nrm = std::sqrt(nrm);
      if (!(nrm > 0.0)) {
        err = "empty radial profile";
        return false;
      }
      for (int p = 0; p < n; ++p) {
        cre[at(k, s, p)] /= nrm;
        cim[at(k, s, p)] /= nrm;
      }
    }
    // Loewdin: columns of one harmonic share the angular factor, so their Gram is
    // the real symmetric matrix G[s][t] = sum_p conj(phi_s) phi_t (imaginary part
    // cancels); replace the columns by Phi_k G^{-1/2}.
    std::vector<double> G(size_t(S) * S, 0.0);
    for (int s = 0; s < S; ++s)
      for (int t = 0; t < S; ++t) {
        double v = 0.0;
        for (int p = 0; p < n; ++p)
          v += cre[at(k, s, p)] * cre[at(k, t, p)] + cim[at(k, s, p)] * cim[at(k, t, p)];
        G[size_t(s) * S + t] = v;
      }
    std::vector<double> w, V;
    jacobi_eig(S, G, w, V);
    for (int s = 0; s < S; ++s)
      if (!(w[s] > 1e-14)) {
        err = "radial profiles are linearly dependent";
        return false;
      }
    std::vector<double> Gis(size_t(S) * S, 0.0);  // G^{-1/2} = V diag(w^-1/2) V^T
    for (int a = 0; a < S; ++a)
      for (int b = 0; b < S; ++b) {
        double v = 0.0;
        for (int e = 0; e < S; ++e) v += V[size_t(a) * S + e] * V[size_t(b) * S + e] / std::sqrt(w[e]);
        Gis[size_t(a) * S + b] = v;
      }
    std::vector<double> nre(size_t(S) * n), nim(size_t(S) * n);
    for (int t = 0; t < S; ++t)
      for (int p = 0; p < n; ++p) {
        double vr = 0.0, vi = 0.0;
        for (int s = 0; s < S; ++s) {
          vr += cre[at(k, s, p)] * Gis[size_t(s) * S + t];
          vi += cim[at(k, s, p)] * Gis[size_t(s) * S + t];
        }
        nre[size_t(t) * n + p] = vr;
        nim[size_t(t) * n + p] = vi;
      }
    for (int s = 0; s < S; ++s)
      for (int p = 0; p < n; ++p) {
        cre[at(k, s, p)] = nre[size_t(s) * n + p];
        cim[at(k, s, p)] = nim[size_t(s) * n + p];
      }
  }
  // packed real synthesis matrix on the disk: phi_d [n][B]
  std::vector<double> phid(size_t(n) * B);
  const double r2 = std::sqrt(2.0);
  for (int p = 0; p < n; ++p) {
    for (int s = 0; s < S; ++s) phid[size_t(p) * B + s] = cre[at(0, s, p)];
    for (int k = 1; k <= T; ++k) {
      int base = S + 2 * S * (k - 1);
      for (int s = 0; s < S; ++s) {
        phid[size_t(p) * B + base + s] = r2 * cre[at(k, s, p)];
        phid[size_t(p) * B + base + S + s] = -r2 * cim[at(k, s, p)];
      }
    }
  }
  if (!finish_basis(N, pix, phid, B, out, err)) return false;
  out.S = S;
  out.T = T;
  return true;
}

// The paper's annular basis (eq. (5)-(7)): annulus s = 1..S (S = floor(N/2)) is
// N(s-1)/(2S) <= r < N s/(2S); its cut-off is half its circumference, floor(pi r_mid),
// lowered to the largest T for which its 2T + 1 real harmonic columns (the indicator,
// cos k theta and sin k theta for k = 1..T, which span the same space as the complex
// exp(i t theta), |t| <= T) are linearly independent on the annulus' pixels: the smallest
// eigenvalue of their Gram matrix (columns normalised) above 1e-12 of the largest.  The
// low-pass basis halves the cut-offs.  Columns are normalised on the disk; the centre
// pixel is 0 for k != 0.  Packed layout: harmonic-major, the annuli with T_s >= k in
// block k ([Re][Im] for k >= 1, sqrt 2 Re and -sqrt 2 Im of the normalised complex column).
bool build_annular_basis(int N, bool lowpass, HostBasis& out, std::vector<int>& Ts, std::string& err) {
  const int S = N / 2;
  const double half = 0.5 * N, c0 = 0.5 * (N - 1);
  const double pi = 3.14159265358979323846;
  if (S < 1) {
    err = "N must be at least 3";
    return false;
  }
  std::vector<int> pix, ring;
  std::vector<double> rho, th;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const double x = j - c0, y = c0 - i, r = std::sqrt(x * x + y * y);
      if (r < half) {
        pix.push_back(i * N + j);
        rho.push_back(r);
        th.push_back(std::atan2(y, x));
        int s = int(std::floor(r * 2.0 * S / N)) + 1;   // N(s-1)/(2S) <= r < N s/(2S)
        if (s > S) s = S;
        if (s > 1 && r < N * (s - 1) / (2.0 * S)) --s;  // guard the boundary against rounding
        if (s < S && r >= N * s / (2.0 * S)) ++s;
        ring.push_back(s);
      }
    }
  const int n = int(pix.size());
  // real harmonic value of column (k, part) at pixel p: part 0 cos, part 1 sin
  auto val = [&](int k, int part, int p) -> double {
    if (k == 0) return part == 0 ? 1.0 : 0.0;
    if (rho[p] == 0.0) return 0.0;
    return part == 0 ? std::cos(k * th[p]) : std::sin(k * th[p]);
  };
  Ts.assign(S, 0);
  for (int s = 1; s <= S; ++s) {
    std::vector<int> ps;
    for (int p = 0; p < n; ++p)
      if (ring[p] == s) ps.push_back(p);
    const int cap = int(std::floor(pi * (N * (s - 0.5) / (2.0 * S))));
    int T = -1;
    for (int t = 0; t <= cap; ++t) {
      const int m = 2 * t + 1;
      if (m > int(ps.size())) break;
      // columns: (0, cos), then (k, cos), (k, sin) for k = 1..t, each normalised
      std::vector<std::pair<int, int>> cols{{0, 0}};
      for (int k = 1; k <= t; ++k) {
        cols.push_back({k, 0});
        cols.push_back({k, 1});
      }
      std::vector<double> nrm(m, 0.0);
      for (int a = 0; a < m; ++a)
        for (int p : ps) nrm[a] += val(cols[a].first, cols[a].second, p) * val(cols[a].first, cols[a].second, p);
      bool zero = false;
      for (int a = 0; a < m; ++a) zero = zero || !(nrm[a] > 0.0);
      if (zero) break;
      std::vector<double> G(size_t(m) * m);
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
          double v = 0.0;
          for (int p : ps) v += val(cols[a].first, cols[a].second, p) * val(cols[b].first, cols[b].second, p);
          G[size_t(a) * m + b] = v / std::sqrt(nrm[a] * nrm[b]);
        }
      std::vector<double> w, V;
      jacobi_eig(m, G, w, V);
      double wmin = w[0], wmax = w[0];
      for (double x : w) {
        wmin = std::min(wmin, x);
        wmax = std::max(wmax, x);
      }
      if (!(wmin > 1e-12 * wmax)) break;
      T = t;
    }
    if (T < 0) {
      err = "an annulus holds no pixel";
      return false;
    }
    Ts[s - 1] = lowpass ? T / 2 : T;
  }
  int Tmax = 0, B = 0;
  for (int t : Ts) {
    Tmax = std::max(Tmax, t);
    B += 2 * t + 1;
  }
  // packed real synthesis matrix on the disk
  std::vector<double> phid(size_t(n) * B, 0.0);
  const double r2 = std::sqrt(2.0);
  int col = 0;
  for (int k = 0; k <= Tmax; ++k) {
    std::vector<int> rs;
    for (int s = 1; s <= S; ++s)
      if (Ts[s - 1] >= k) rs.push_back(s);
    const int nk = int(rs.size());
    for (int i = 0; i < nk; ++i) {
      double nrm = 0.0;   // |exp(i k theta)| = 1 on the annulus, 0 at the centre for k != 0
      for (int p = 0; p < n; ++p)
        if (ring[p] == rs[i] && (k == 0 || rho[p] != 0.0)) nrm += 1.0;
      nrm = std::sqrt(nrm);
      for (int p = 0; p < n; ++p) {
        if (ring[p] != rs[i]) continue;
        if (k == 0) {
          phid[size_t(p) * B + col + i] = 1.0 / nrm;
        } else {
          phid[size_t(p) * B + col + i] = r2 * val(k, 0, p) / nrm;
          phid[size_t(p) * B + col + nk + i] = -r2 * val(k, 1, p) / nrm;
        }
      }
    }
    col += k == 0 ? nk : 2 * nk;
  }
  if (!finish_basis(N, pix, phid, B, out, err)) return false;
  out.S = S;
  out.T = Tmax;
  return true;
}

}  // namespace rsc
