// C ABI of librsc: handles, argument validation, host-side table arrangement and
// device uploads.  All compute is enqueued through the launchers of rsc_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rsc.h"
#include "rsc_internal.h"

// One of the two device arenas that hold a handle's dictionary tables.  Uploads go to the
// arena that is not bound, so tables that launches in flight still read are never
// overwritten; before an arena is refilled, the upload stream waits for every launch that
// read it (an event per stream, recorded after each launch).
struct DictSlot {
  void* arena = nullptr;
  size_t bytes = 0;
  void* pinned = nullptr;            // page-locked host staging of the upload
  size_t pinned_bytes = 0;
  hipEvent_t copied = nullptr;       // recorded after the upload's copy
  std::vector<std::pair<hipStream_t, hipEvent_t>> users;   // launches that read this arena
};

struct rsc_handle {
  rsc::HostBasis basis;
  rsc::DeviceTables dev;
  rsc_precision prec = RSC_FP32;
  rsc_tile tile = RSC_TILE_AUTO;
  bool has_dict = false;
  bool annular = false;      // the paper's annular basis (projection, steering, synthesis only)
  std::vector<int> Ts;       // its per-annulus cut-offs
  // Sticky device fault: a failed launch, copy or synchronisation on this handle makes
  // every later call on it return RSC_E_DEVICE with this message.
  mutable rsc_status fault = RSC_OK;
  mutable std::string fault_msg;
  mutable DictSlot slot[2];
  int cur = -1;                          // slot whose tables are bound (-1: none)
  hipStream_t dict_stream = nullptr;     // stream of the last upload
};

namespace {

thread_local std::string g_err;

rsc_status fail(rsc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

rsc_status ok() {
  g_err.clear();
  return RSC_OK;
}

rsc_status device_fail(int e, const char* what) {
  return fail(RSC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(hipError_t(e)));
}

// A device failure on a handle: reported now and on every later call (sticky).
rsc_status handle_fail(const rsc_handle* h, int e, const char* what) {
  const std::string msg = std::string(what) + ": " + hipGetErrorString(hipError_t(e));
  if (h && h->fault == RSC_OK) {
    h->fault = RSC_E_DEVICE;
    h->fault_msg = msg;
  }
  return fail(RSC_E_DEVICE, msg);
}

// RSC_E_DEVICE if the handle carries a sticky fault.
rsc_status check_fault(const rsc_handle* h) {
  if (h && h->fault != RSC_OK) return fail(h->fault, "earlier device fault on this handle: " + h->fault_msg);
  return RSC_OK;
}

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Before a launch that reads the dictionary tables: order it after the upload when the
// upload ran on another stream and may still be in flight.
rsc_status dict_before(const rsc_handle* h, void* stream) {
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const DictSlot& s = h->slot[h->cur];
  if (st != h->dict_stream && s.copied && !capturing(st) && hipEventQuery(s.copied) == hipErrorNotReady) {
    const hipError_t e = hipStreamWaitEvent(st, s.copied, 0);
    if (e != hipSuccess) return handle_fail(h, int(e), "stream wait on the dictionary upload");
  }
  return RSC_OK;
}

// After a launch that reads the dictionary tables: mark the stream as a reader of the bound
// arena (not under graph capture: a captured graph reads the tables bound at capture time).
rsc_status dict_after(const rsc_handle* h, void* stream) {
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (capturing(st)) return RSC_OK;
  DictSlot& s = h->slot[h->cur];
  hipEvent_t ev = nullptr;
  for (auto& u : s.users)
    if (u.first == st) ev = u.second;
  if (!ev) {
    const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return handle_fail(h, int(e), "event creation");
    s.users.emplace_back(st, ev);
  }
  const hipError_t e = hipEventRecord(ev, st);
  return e == hipSuccess ? RSC_OK : handle_fail(h, int(e), "event record after a launch");
}

// A launch that reads the dictionary: fault check, ordering, launch, reader mark.
template <class F>
rsc_status dict_launch(const rsc_handle* h, void* stream, const char* what, F launch) {
  rsc_status s = dict_before(h, stream);
  if (s != RSC_OK) return s;
  const int e = launch();
  if (e) return handle_fail(h, e, what);
  s = dict_after(h, stream);
  return s != RSC_OK ? s : ok();
}

// Wait for every launch recorded against the slot and for its upload, then release it.
void release_slot(DictSlot& s) {
  for (auto& u : s.users) {
    (void)hipEventSynchronize(u.second);
    (void)hipEventDestroy(u.second);
  }
  s.users.clear();
  if (s.copied) {
    (void)hipEventSynchronize(s.copied);
    (void)hipEventDestroy(s.copied);
    s.copied = nullptr;
  }
  if (s.arena) (void)hipFree(s.arena);
  if (s.pinned) (void)hipHostFree(s.pinned);
  s = DictSlot();
}

template <class X>
void free_dev(X*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

template <class X>
rsc_status upload(X*& dst, const std::vector<X>& src, const char* what) {
  free_dev(dst);
  if (src.empty()) return RSC_OK;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&dst), src.size() * sizeof(X));
  if (e != hipSuccess) {
    dst = nullptr;
    return fail(RSC_E_NOMEM, std::string("hipMalloc for ") + what + " failed");
  }
  e = hipMemcpy(dst, src.data(), src.size() * sizeof(X), hipMemcpyHostToDevice);
  if (e != hipSuccess) return device_fail(int(e), what);
  return RSC_OK;
}

// Packs host tables into one staging buffer at 256-byte aligned offsets; bind() then points
// each registered device pointer into the arena (nullptr for an empty table).
struct Arena {
  std::vector<char> staging;
  std::vector<std::pair<void**, size_t>> slots;  // (pointer to set, offset), offset ~0 for empty
  template <class X>
  void add(X*& dst, const std::vector<X>& src) {
    if (src.empty()) {
      slots.emplace_back(reinterpret_cast<void**>(&dst), ~size_t(0));
      return;
    }
    const size_t off = (staging.size() + 255) & ~size_t(255);
    staging.resize(off + src.size() * sizeof(X));
    std::memcpy(staging.data() + off, src.data(), src.size() * sizeof(X));
    slots.emplace_back(reinterpret_cast<void**>(&dst), off);
  }
  void bind(char* base) {
    for (auto& sl : slots) *sl.first = (base && sl.second != ~size_t(0)) ? base + sl.second : nullptr;
  }
};

// Round to the nearest BF16 / FP16 value (ties to even); returns the bit pattern.
uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, sizeof(u));
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

uint16_t to_f16(float f) {
  const _Float16 h = static_cast<_Float16>(f);
  uint16_t r;
  std::memcpy(&r, &h, sizeof(r));
  return r;
}

float from_bf16(uint16_t b) {
  const uint32_t u = uint32_t(b) << 16;
  float f;
  std::memcpy(&f, &u, sizeof(f));
  return f;
}

float from_f16(uint16_t b) {
  _Float16 h;
  std::memcpy(&h, &b, sizeof(h));
  return float(h);
}

// Device tables of a handle whose host basis is built (shared by every kind of handle).
// On failure the handle is destroyed.
rsc_status init_tables(rsc_handle* h, int N, int S, int T, rsc_precision prec) {
  const rsc::HostBasis& b = h->basis;
  h->prec = prec;
  rsc::DeviceTables& d = h->dev;
  d.N = N;
  d.S = S;
  d.T = T;
  d.B = b.B;
  d.geo = rsc::kGeoGrid;
  for (int k = 0; k <= T && k < 64; ++k) d.sk[k] = S;
  const int NN = N * N, KP = (NN + 1) / 2;
  const int RTB = (b.B + 31) / 32 <= 2 ? 2 : (b.B + 31) / 32 <= 4 ? 4 : 6;  // row tiles of the projection kernels
  // projection A operand: row = hat coordinate, contraction = grid pixel
  std::vector<float> pinvA(size_t(RTB) * KP * 64, 0.f);
  for (int t = 0; t < RTB; ++t)
    for (int j = 0; j < KP; ++j)
      for (int l = 0; l < 64; ++l) {
        const int row = 32 * t + (l % 32), px = 2 * j + l / 32;
        if (row < b.B && px < NN) pinvA[(size_t(t) * KP + j) * 64 + l] = float(b.pinv[size_t(row) * NN + px]);
      }
  // projection operand over disk pixels only (contraction index 2j + u = disk pixel)
  d.n_pix = b.n_pix;
  const int KPD = (b.n_pix + 1) / 2;
  std::vector<float> pinvD;
  std::vector<int> pixD;
  pixD.assign(size_t(2) * KPD, -1);
  for (int i = 0; i < b.n_pix; ++i) pixD[i] = b.pix[i];
  if (b.B <= 64) {
    pinvD.assign(size_t(2) * KPD * 64, 0.f);
    for (int t = 0; t < 2; ++t)
      for (int j = 0; j < KPD; ++j)
        for (int l = 0; l < 64; ++l) {
          const int row = 32 * t + (l % 32), i = 2 * j + l / 32;
          if (row < b.B && i < b.n_pix)
            pinvD[(size_t(t) * KPD + j) * 64 + l] = float(b.pinv[size_t(row) * NN + b.pix[i]]);
        }
  }
  // image projection operand (row tiles of 32 hat coordinates, disk-pixel contraction)
  const int RTBI = b.B <= 64 ? 2 : b.B <= 128 ? 4 : (b.B + 31) / 32;
  std::vector<float> pinvI(size_t(RTBI) * KPD * 64, 0.f);
  std::vector<int> dpixI(size_t(2) * KPD, -1);
  for (int i = 0; i < b.n_pix; ++i) dpixI[i] = ((b.pix[i] / N) << 8) | (b.pix[i] % N);
  for (int t = 0; t < RTBI; ++t)
    for (int j = 0; j < KPD; ++j)
      for (int l = 0; l < 64; ++l) {
        const int row = 32 * t + (l % 32), i = 2 * j + l / 32;
        if (row < b.B && i < b.n_pix)
          pinvI[(size_t(t) * KPD + j) * 64 + l] = float(b.pinv[size_t(row) * NN + b.pix[i]]);
      }
  std::vector<float> phiPad(size_t(NN) * b.B);
  for (size_t i = 0; i < phiPad.size(); ++i) phiPad[i] = float(b.phi[i]);
  // synthesis MFMA operand: row = output pixel, contraction = hat coordinate
  std::vector<float> synA;
  if (NN <= 256) {
    const int NTT = (NN + 31) / 32, KB = (b.B + 1) / 2;
    synA.assign(size_t(NTT) * KB * 64, 0.f);
    for (int tt = 0; tt < NTT; ++tt)
      for (int j = 0; j < KB; ++j)
        for (int l = 0; l < 64; ++l) {
          const int q = 32 * tt + l % 32, c = 2 * j + l / 32;
          if (q < NN && c < b.B) synA[(size_t(tt) * KB + j) * 64 + l] = phiPad[size_t(q) * b.B + c];
        }
  }
  rsc_status s = upload(d.pinvA, pinvA, "projection table");
  if (s == RSC_OK) s = upload(d.pinvD, pinvD, "projection table");
  if (s == RSC_OK) s = upload(d.pixD, pixD, "pixel table");
  if (s == RSC_OK) s = upload(d.phiPad, phiPad, "synthesis table");
  if (s == RSC_OK) s = upload(d.synA, synA, "synthesis operand");
  if (s == RSC_OK) s = upload(d.pinvI, pinvI, "image projection table");
  if (s == RSC_OK) s = upload(d.dpixI, dpixI, "image pixel table");
  d.prec = prec;
  if (s == RSC_OK) s = upload(d.lpStats, std::vector<unsigned long long>(4, 0ull), "counters");
  if (s == RSC_OK && prec != RSC_FP32 && b.B <= 64) {
    // compensated 16-bit projection operand: pinv split into 16-bit parts, each the
    // rounding of what the previous parts leave (3 parts for BF16, 2 for FP16)
    const int KS = (b.n_pix + 15) / 16, NP = prec == RSC_BF16 ? 3 : 2;
    const size_t part = size_t(2) * KS * 64 * 8;
    // FP16: operand scaled by 2^sh so that its largest entry lies in [2^10, 2^11)
    double amax = 0.0;
    for (double v : b.pinv) amax = std::max(amax, std::fabs(v));
    int ex = 0;
    (void)std::frexp(amax, &ex);
    const int sh = (prec == RSC_FP16 && amax > 0.0) ? 11 - ex : 0;
    d.lpPinvUnscale = float(std::ldexp(1.0, -sh));
    std::vector<uint16_t> pp(NP * part, 0);
    std::vector<int> pix16(size_t(16) * KS, -1);
    for (int i = 0; i < b.n_pix; ++i) pix16[i] = b.pix[i];
    for (int t = 0; t < 2; ++t)
      for (int j = 0; j < KS; ++j)
        for (int l = 0; l < 64; ++l)
          for (int i = 0; i < 8; ++i) {
            const int row = 32 * t + l % 32, px = 16 * j + 8 * (l / 32) + i;
            if (row >= b.B || px >= b.n_pix) continue;
            double rem = std::ldexp(b.pinv[size_t(row) * NN + b.pix[px]], sh);
            for (int q = 0; q < NP; ++q) {
              const uint16_t hb = prec == RSC_BF16 ? to_bf16(float(rem)) : to_f16(float(rem));
              pp[q * part + ((size_t(t) * KS + j) * 64 + l) * 8 + i] = hb;
              rem -= prec == RSC_BF16 ? double(from_bf16(hb)) : double(from_f16(hb));
            }
          }
    s = upload(d.lpPinv, pp, "16-bit projection table");
    if (s == RSC_OK) s = upload(d.lpPix16, pix16, "pixel table");
  }
  if (s != RSC_OK) {
    rsc_destroy(h);
    return s;
  }
  return RSC_OK;
}


}  // namespace

namespace {

// Workspace of the dictionary update: partial covariances, per-chunk counts, the FP64
// sum slot, then (for training) the new dictionary, usage and reset arrays.
struct RkLayout {
  size_t update = 0, dnew = 0, usage = 0, reset = 0, total = 0;
};

RkLayout rk_layout(const rsc::DeviceTables& d, int64_t P, int K) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  RkLayout L;
  L.update = al(rsc::rksvd_workspace_bytes(d, P, K));
  L.dnew = L.update;
  L.usage = L.dnew + al(sizeof(float) * size_t(d.M) * d.B);
  L.reset = L.usage + al(sizeof(int32_t) * size_t(d.M));
  L.total = L.reset + al(sizeof(int32_t) * size_t(d.M));
  return L;
}

double* rk_sum_slot(const rsc::DeviceTables& d, int64_t P, int K, void* ws) {
  // the last kSumSlots doubles of the update area
  return reinterpret_cast<double*>(reinterpret_cast<char*>(ws) + rsc::rksvd_workspace_bytes(d, P, K) -
                                   rsc::kSumSlots * sizeof(double));
}

}  // namespace

namespace {
struct ClsLayout {
  size_t atom, angle, coef, resid, total;
};
ClsLayout cls_layout(int64_t P, int K) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  ClsLayout L;
  L.atom = 0;
  L.angle = L.atom + al(sizeof(int32_t) * size_t(P) * K);
  L.coef = L.angle + al(sizeof(int32_t) * size_t(P) * K);
  L.resid = L.coef + al(sizeof(float) * size_t(P) * K);
  L.total = L.resid + al(sizeof(float) * size_t(P));
  return L;
}
}  // namespace

extern "C" {

const char* rsc_last_error(const rsc_handle* h) {
  if (g_err.empty() && h && h->fault != RSC_OK) return h->fault_msg.c_str();
  return g_err.c_str();
}

rsc_status rsc_create(int N, int S, int T, const double* centres, double sigma, rsc_precision prec,
                      rsc_handle** out) {
  if (!out) return fail(RSC_E_INVALID, "out is NULL");
  *out = nullptr;
  if (N < 3 || N > 31 || N % 2 == 0) return fail(RSC_E_INVALID, "N must be odd, 3..31");
  if (S < 1 || T < 0) return fail(RSC_E_INVALID, "S must be >= 1 and T >= 0");
  if (S * (2 * T + 1) > 128) return fail(RSC_E_UNSUPPORTED, "B = S(2T+1) must be <= 128");
  if (T > 15) return fail(RSC_E_UNSUPPORTED, "T must be <= 15");
  if (prec != RSC_FP32 && prec != RSC_BF16 && prec != RSC_FP16) return fail(RSC_E_INVALID, "unknown precision");
  if (!rsc::encode_supported(S, T) && prec != RSC_FP32)
    return fail(RSC_E_UNSUPPORTED, "16-bit handles need (S, T) = (5, 5) or (7, 7)");
  if (centres) {
    for (int s = 0; s < S; ++s)
      if (!std::isfinite(centres[s])) return fail(RSC_E_INVALID, "non-finite profile centre");
  }
  rsc_handle* h = new (std::nothrow) rsc_handle();
  if (!h) return fail(RSC_E_NOMEM, "handle allocation failed");
  std::string err;
  if (!rsc::build_basis(N, S, T, centres, sigma, h->basis, err)) {
    delete h;
    return fail(RSC_E_INVALID, "basis construction failed: " + err);
  }
  rsc_status st = init_tables(h, N, S, T, prec);
  if (st != RSC_OK) return st;
  *out = h;
  return ok();
}

rsc_status rsc_create_annular(int N, int lowpass, rsc_handle** out) {
  if (!out) return fail(RSC_E_INVALID, "out is NULL");
  *out = nullptr;
  if (N < 3 || N > 31 || N % 2 == 0) return fail(RSC_E_INVALID, "N must be odd, 3..31");
  rsc_handle* h = new (std::nothrow) rsc_handle();
  if (!h) return fail(RSC_E_NOMEM, "handle allocation failed");
  std::string err;
  if (!rsc::build_annular_basis(N, lowpass != 0, h->basis, h->Ts, err)) {
    delete h;
    return fail(RSC_E_INVALID, "basis construction failed: " + err);
  }
  const rsc::HostBasis& b = h->basis;
  if (b.B > 192 || b.T > 31) {
    delete h;
    return fail(RSC_E_UNSUPPORTED, "annular basis with B = " + std::to_string(b.B) + ", T = " +
                                       std::to_string(b.T) + ": the library handles B <= 192 and T <= 31");
  }
  h->annular = true;
  rsc_status st = init_tables(h, N, b.S, b.T, RSC_FP32);
  if (st != RSC_OK) return st;
  // per-harmonic annulus counts, and the layouts the pursuit is compiled for
  for (int k = 0; k <= b.T; ++k) {
    int nk = 0;
    for (int t : h->Ts) nk += t >= k ? 1 : 0;
    h->dev.sk[k] = nk;
  }
  const std::vector<int> ts11 = {1, 3, 8, 11, 15}, ts15 = {1, 3, 8, 11, 13, 18, 19};
  h->dev.geo = (N == 11 && !lowpass && h->Ts == ts11)   ? rsc::kGeoAnnular11
               : (N == 15 && !lowpass && h->Ts == ts15) ? rsc::kGeoAnnular15
                                                        : rsc::kGeoAnnularOther;
  // steering table: coordinate -> (harmonic k, offset of its Re/Im partner)
  std::vector<int> tab(b.B);
  int col = 0;
  for (int k = 0; k <= b.T; ++k) {
    int nk = 0;
    for (int t : h->Ts) nk += t >= k ? 1 : 0;
    for (int i = 0; i < nk; ++i) {
      if (k == 0) {
        tab[col + i] = 32768;
      } else {
        tab[col + i] = (k << 16) | (nk + 32768);
        tab[col + nk + i] = (k << 16) | (-nk + 32768);
      }
    }
    col += k == 0 ? nk : 2 * nk;
  }
  st = upload(h->dev.steerTab, tab, "steering table");
  if (st != RSC_OK) {
    rsc_destroy(h);
    return st;
  }
  *out = h;
  return ok();
}

rsc_status rsc_annular_basis_host(int N, int lowpass, double* phi, double* pinv, int* Ts, int* B, double* cond_gram) {
  if (N < 3 || N > 63 || N % 2 == 0) return fail(RSC_E_INVALID, "N must be odd, 3..63");
  rsc::HostBasis b;
  std::vector<int> ts;
  std::string err;
  if (!rsc::build_annular_basis(N, lowpass != 0, b, ts, err))
    return fail(RSC_E_INVALID, "basis construction failed: " + err);
  if (phi) std::memcpy(phi, b.phi.data(), b.phi.size() * sizeof(double));
  if (pinv) std::memcpy(pinv, b.pinv.data(), b.pinv.size() * sizeof(double));
  if (Ts) std::memcpy(Ts, ts.data(), ts.size() * sizeof(int));
  if (B) *B = b.B;
  if (cond_gram) *cond_gram = b.cond;
  return ok();
}

rsc_status rsc_basis_host(int N, int S, int T, const double* centres, double sigma, double* phi,
                          double* pinv, int* n_pix, int* B, double* cond_gram) {
  if (N < 1 || N > 63 || N % 2 == 0) return fail(RSC_E_INVALID, "N must be odd, 1..63");
  if (S < 1 || T < 0 || S > 64 || T > 64) return fail(RSC_E_INVALID, "S must be 1..64 and T 0..64");
  rsc::HostBasis b;
  std::string err;
  if (!rsc::build_basis(N, S, T, centres, sigma, b, err))
    return fail(RSC_E_INVALID, "basis construction failed: " + err);
  if (phi) std::memcpy(phi, b.phi.data(), b.phi.size() * sizeof(double));
  if (pinv) std::memcpy(pinv, b.pinv.data(), b.pinv.size() * sizeof(double));
  if (n_pix) *n_pix = b.n_pix;
  if (B) *B = b.B;
  if (cond_gram) *cond_gram = b.cond;
  return ok();
}

rsc_status rsc_destroy(rsc_handle* h) {
  if (!h) return ok();
  rsc::DeviceTables& d = h->dev;
  free_dev(d.pinvA);
  free_dev(d.pinvD);
  free_dev(d.pixD);
  free_dev(d.pinvI);
  free_dev(d.dpixI);
  free_dev(d.phiPad);
  free_dev(d.synA);
  free_dev(d.steerTab);
  release_slot(h->slot[0]);
  release_slot(h->slot[1]);
  d.dictArena = nullptr;
  free_dev(d.lpStats);
  free_dev(d.lpPinv);
  free_dev(d.lpPix16);
  delete h;
  return ok();
}

rsc_status rsc_basis_info(const rsc_handle* h, int* n_pix, int* B, double* cond_gram) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (n_pix) *n_pix = h->basis.n_pix;
  if (B) *B = h->basis.B;
  if (cond_gram) *cond_gram = h->basis.cond;
  return ok();
}

rsc_status rsc_get_basis(const rsc_handle* h, double* phi, double* pinv) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (phi) std::memcpy(phi, h->basis.phi.data(), h->basis.phi.size() * sizeof(double));
  if (pinv) std::memcpy(pinv, h->basis.pinv.data(), h->basis.pinv.size() * sizeof(double));
  return ok();
}

rsc_status rsc_set_dictionary(rsc_handle* h, const float* d_hat, int M, int R, void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (rsc_status f = check_fault(h)) return f;
  if (!d_hat) return fail(RSC_E_INVALID, "d_hat is NULL");
  if (M < 1 || M > 256) return fail(RSC_E_INVALID, "M must be in 1..256");
  if (R < 1 || R > 128) return fail(RSC_E_INVALID, "R must be in 1..128");
  rsc::DeviceTables& d = h->dev;
  const int S = d.S, T = d.T, B = d.B;
  if (!rsc::encode_supported_geo(d))
    return fail(RSC_E_UNSUPPORTED,
                h->annular ? "the pursuit on the annular basis is compiled for its full form at N = 11 and N = 15; "
                             "this handle supports projection, steering and synthesis only"
                           : "the encoders are compiled for (S, T) = (5, 5) and (7, 7); this geometry supports "
                             "projection, steering and synthesis only");
  if ((d.geo == rsc::kGeoAnnular11 || d.geo == rsc::kGeoAnnular15) && (R % 2 != 0 || R > rsc::kAnnularMaxR))
    return fail(RSC_E_UNSUPPORTED, "the pursuit on the annular basis is compiled for even R <= 64");
  for (int m = 0; m < M; ++m) {
    double n2 = 0.0;
    for (int b = 0; b < B; ++b) {
      const double v = d_hat[size_t(m) * B + b];
      if (!std::isfinite(v)) return fail(RSC_E_INVALID, "non-finite dictionary entry");
      n2 += v * v;
    }
    if (std::fabs(1.0 - std::sqrt(n2)) > 1e-5)
      return fail(RSC_E_INVALID, "dictionary row " + std::to_string(m) + " is not unit norm");
  }
  const int NG = (M + 15) / 16;
  const int K0 = rsc::k0_steps(S), NKS = rsc::stage1_steps(S, T), NQ = T + 1;
  auto D = [&](int m, int c) -> float { return m < M ? d_hat[size_t(m) * B + c] : 0.f; };
  // 32x32 tiles, stage-1 operand: row 8i + j (j < 4) gives Re C_k of atom 16g + 4i + j and
  // row 8i + 4 + j its Im C_k, so that the accumulator register of an atom holds its Re C_k
  // in the low half-wave and its Im C_k in the high one; the two contraction lanes of a
  // step are (Re, Im) of one profile (k >= 1) or two consecutive profiles (k = 0, where
  // the Im rows are zero).
  std::vector<float> dictA;
  if (S == 5 && T == 5) {
    dictA.assign(size_t(NG) * NKS * 64, 0.f);
    for (int g = 0; g < NG; ++g)
      for (int ks = 0; ks < NKS; ++ks)
        for (int l = 0; l < 64; ++l) {
          const int row = l % 32, hh = l / 32, a = 4 * (row / 8) + row % 4, m = 16 * g + a;
          const bool im_row = (row / 4) % 2 == 1;
          float v = 0.f;
          if (ks < K0) {
            const int s = 2 * ks + hh;
            if (!im_row && s < S) v = D(m, s);
          } else {
            const int q = ks - K0, k = 1 + q / S, s = q % S, base = S + 2 * S * (k - 1);
            const float re = D(m, base + s), im = D(m, base + S + s);
            if (!im_row) v = hh == 0 ? re : im;
            else v = hh == 0 ? -im : re;
          }
          dictA[(size_t(g) * NKS + ks) * 64 + l] = v;
        }
  }
  std::vector<float> hat(size_t(NG) * 16 * B, 0.f);
  for (int m = 0; m < M; ++m)
    for (int b = 0; b < B; ++b) hat[size_t(m) * B + b] = d_hat[size_t(m) * B + b];
  const double two_pi = 6.283185307179586476925286766559;
  auto cosk = [&](int k, int r) { return float(std::cos(two_pi * double(k) * double(r) / double(R))); };
  auto sink = [&](int k, int r) { return float(std::sin(two_pi * double(k) * double(r) / double(R))); };
  // 32x32 tiles, stage-2 operand (even R <= 64): row = angle r < R/2, contraction
  // lanes (cos, -sin) of one harmonic, (1, 0) for k = 0
  std::vector<float> dftA32;
  if (R % 2 == 0 && R <= 64) {
    dftA32.assign(size_t(NQ) * 64, 0.f);
    for (int q = 0; q < NQ; ++q)
      for (int l = 0; l < 64; ++l) {
        const int r = l % 32, hh = l / 32;
        if (r >= R / 2) continue;
        dftA32[size_t(q) * 64 + l] = q == 0 ? (hh == 0 ? 1.f : 0.f) : (hh == 0 ? cosk(q, r) : -sink(q, r));
      }
  }
  // 16x16 tiles: four contraction lanes (cos k1, -sin k1, cos k2, -sin k2) per step.
  auto lane16 = [&](int k1, int k2, int r, int kk) -> float {
    const int k = kk < 2 ? k1 : k2;
    if (k > T) return 0.f;
    if (kk % 2 == 0) return k == 0 ? 1.f : cosk(k, r);
    return k == 0 ? 0.f : -sink(k, r);
  };
  // direct (odd R): steps (2q, 2q+1), tiles of 16 angles covering r < R
  const int RT16 = R <= 16 ? 1 : (R <= 32 ? 2 : (R <= 64 ? 4 : 8));
  const int NP = (NQ + 1) / 2;
  std::vector<float> dftA16(size_t(RT16) * NP * 64, 0.f);
  for (int t = 0; t < RT16; ++t)
    for (int q = 0; q < NP; ++q)
      for (int l = 0; l < 64; ++l) {
        const int r = 16 * t + (l % 16);
        if (r < R) dftA16[(size_t(t) * NP + q) * 64 + l] = lane16(2 * q, 2 * q + 1, r, l / 16);
      }
  // split (even R): E steps (4j, 4j+2) then O steps (4j+1, 4j+3), tiles covering r < R/2
  std::vector<float> dftA16s;
  if (R % 2 == 0) {
    const int NE = T / 2 + 1, NO = (T + 1) / 2, SE = (NE + 1) / 2, SO = (NO + 1) / 2, NS = SE + SO;
    const int half = R / 2, HT = half <= 16 ? 1 : (half <= 32 ? 2 : 4);
    dftA16s.assign(size_t(HT) * NS * 64, 0.f);
    for (int t = 0; t < HT; ++t)
      for (int q = 0; q < NS; ++q)
        for (int l = 0; l < 64; ++l) {
          const int r = 16 * t + (l % 16);
          const int k1 = q < SE ? 4 * q : 4 * (q - SE) + 1;
          if (r < half) dftA16s[(size_t(t) * NS + q) * 64 + l] = lane16(k1, k1 + 2, r, l / 16);
        }
  }
  std::vector<float> cs(size_t(2) * NQ * R);
  for (int k = 0; k < NQ; ++k)
    for (int r = 0; r < R; ++r) {
      cs[size_t(k) * R + r] = cosk(k, r);
      cs[size_t(NQ + k) * R + r] = sink(k, r);
    }
  // per-pair harmonic inner products in FP64: H_0 = sum_s a_s b_s (k = 0 block),
  // H_k = sum_s conj(a_k,s) b_k,s as (Re, Im) for k >= 1, over the sk[k] profiles (or
  // annuli) of harmonic k, whose [Re][Im] block starts at kbase[k]
  const int HQ = 2 * T + 1;
  std::vector<int> kbase(T + 1, 0);
  for (int k = 1; k <= T; ++k) kbase[k] = k == 1 ? d.sk[0] : kbase[k - 1] + 2 * d.sk[k - 1];
  const bool lp = h->prec != RSC_FP32;
  // i * d in the row layout of hat (FP32 16x16 tile): the stage-1 Im rows read it at the
  // offsets the Re rows read d, so neither needs a sign; zero at harmonic 0, whose Im row is 0
  std::vector<float> hatI;
  if (!lp) {
    hatI.assign(hat.size(), 0.f);
    for (int m = 0; m < M; ++m)
      for (int k = 1; k <= T; ++k) {
        const int base = kbase[k], nk = d.sk[k];
        for (int s = 0; s < nk; ++s) {
          hatI[size_t(m) * B + base + s] = -D(m, base + nk + s);
          hatI[size_t(m) * B + base + nk + s] = D(m, base + s);
        }
      }
  }
  std::vector<float> gramH(size_t(M) * M * HQ);
  std::vector<double> gramH64(gramH.size());
  for (int a = 0; a < M; ++a)
    for (int bb = 0; bb < M; ++bb) {
      float* hh = &gramH[(size_t(a) * M + bb) * HQ];
      double h0 = 0.0;
      for (int s = 0; s < d.sk[0]; ++s) h0 += double(D(a, s)) * double(D(bb, s));
      hh[0] = float(h0);
      gramH64[(size_t(a) * M + bb) * HQ] = h0;
      for (int k = 1; k <= T; ++k) {
        const int base = kbase[k], nk = d.sk[k];
        double re = 0.0, im = 0.0;
        for (int s = 0; s < nk; ++s) {
          const double ar = D(a, base + s), ai = D(a, base + nk + s);
          const double br = D(bb, base + s), bi = D(bb, base + nk + s);
          re += ar * br + ai * bi;
          im += ar * bi - ai * br;
        }
        hh[2 * k - 1] = float(re);
        hh[2 * k] = float(im);
        gramH64[(size_t(a) * M + bb) * HQ + 2 * k - 1] = re;
        gramH64[(size_t(a) * M + bb) * HQ + 2 * k] = im;
      }
    }
  // 16-bit encoder tables
  std::vector<uint16_t> lpA, lpF16;
  std::vector<float> lpF32;
  std::vector<double> cs64;
  bool split = false;
  if (lp) {
    if (!rsc::encode_lp_supported(S, T, M, R))
      return fail(RSC_E_UNSUPPORTED, "16-bit encoder: needs M <= 128 and R <= 64");
    auto cvt = [&](float v) { return h->prec == RSC_BF16 ? to_bf16(v) : to_f16(v); };
    // stage 1: lane l gives row l % 32 = (atom 4(row/8) + row%4, Re/Im = (row/4)%2) and
    // contraction slots 8(l/32)..+7: the residual's harmonic-k block, Re parts (k = 0:
    // even profiles) in the low half-wave, Im parts (k = 0: odd profiles) in the high
    lpA.assign(size_t(NG) * NQ * 64 * 8, 0);
    for (int g = 0; g < NG; ++g)
      for (int k = 0; k < NQ; ++k)
        for (int l = 0; l < 64; ++l) {
          const int row = l % 32, hh = l / 32, a = 4 * (row / 8) + row % 4, part = (row / 4) % 2;
          const int m = 16 * g + a;
          for (int i = 0; i < 8; ++i) {
            float v = 0.f;
            if (k == 0) {
              const int s = 2 * i + hh;
              if (part == 0 && s < S) v = D(m, s);
            } else if (i < S) {
              const int base = S + 2 * S * (k - 1);
              const float re = D(m, base + i), im = D(m, base + S + i);
              v = part == 0 ? (hh == 0 ? re : im) : (hh == 0 ? -im : re);
            }
            lpA[((size_t(g) * NQ + k) * 64 + l) * 8 + i] = cvt(v);
          }
        }
    const int RT = (R + 31) / 32;
    // stage 2: row = angle 32t + l%32, slots k of the low half-wave cos(k theta),
    // of the high half-wave -sin(k theta)
    lpF16.assign(size_t(RT) * 64 * 8, 0);
    for (int t = 0; t < RT; ++t)
      for (int l = 0; l < 64; ++l) {
        const int r = 32 * t + l % 32, hh = l / 32;
        if (r >= R) continue;
        for (int k = 0; k < NQ; ++k) {
          const float v = hh == 0 ? (k == 0 ? 1.f : cosk(k, r)) : (k == 0 ? 0.f : -sink(k, r));
          lpF16[(size_t(t) * 64 + l) * 8 + k] = cvt(v);
        }
      }
    // FP32 re-score operand: radix-2 split (rows r < R/2) for even R in 33..64, else
    // RT tiles of the direct DFT; contraction lanes (cos, -sin), (1, 0) for k = 0
    split = R % 2 == 0 && R > 32;
    const int FT = split ? 1 : RT, rows = split ? R / 2 : R;
    lpF32.assign(size_t(FT) * NQ * 64, 0.f);
    for (int t = 0; t < FT; ++t)
      for (int l = 0; l < 64; ++l) {
        const int r = 32 * t + l % 32, hh = l / 32;
        if (r >= rows) continue;
        for (int k = 0; k < NQ; ++k)
          lpF32[(size_t(t) * NQ + k) * 64 + l] = hh == 0 ? (k == 0 ? 1.f : cosk(k, r)) : (k == 0 ? 0.f : -sink(k, r));
      }
  }
  cs64.resize(cs.size());
  for (int k = 0; k < NQ; ++k)
    for (int r = 0; r < R; ++r) {
      cs64[size_t(k) * R + r] = std::cos(two_pi * double(k) * double(r) / double(R));
      cs64[size_t(NQ + k) * R + r] = std::sin(two_pi * double(k) * double(r) / double(R));
    }
  // the new tables must fit a CU's LDS; checked before the handle changes, so a refused
  // upload leaves the current dictionary in place
  rsc::DeviceTables nd = d;
  nd.M = M;
  nd.R = R;
  nd.NG = NG;
  nd.lpSplit = split;
  if (lp && rsc::encode_lp_lds_bytes(nd) > 160 * 1024)
    return fail(RSC_E_UNSUPPORTED, "dictionary tables exceed the 160 KiB LDS of a CU");
  if (!lp && rsc::encode_lds_bytes(nd, RSC_TILE_16) > 160 * 1024)
    return fail(RSC_E_UNSUPPORTED, "dictionary tables exceed the 160 KiB LDS of a CU");
  // one host staging buffer, one copy into the arena that is not bound
  Arena arena;
  arena.add(d.dictA, dictA);
  arena.add(d.dictHat, hat);
  arena.add(d.dictHatI, hatI);
  arena.add(d.dftA32, dftA32);
  arena.add(d.dftA16, dftA16);
  arena.add(d.dftA16s, dftA16s);
  arena.add(d.cs, cs);
  arena.add(d.gramH, gramH);
  arena.add(d.lpA, lpA);
  arena.add(d.lpF16, lpF16);
  arena.add(d.lpF32, lpF32);
  arena.add(d.gramH64, gramH64);
  arena.add(d.cs64, cs64);
  const size_t need = arena.staging.size();
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  DictSlot& sl = h->slot[h->cur < 0 ? 0 : 1 - h->cur];
  hipError_t e = hipSuccess;
  if (sl.copied && (e = hipEventSynchronize(sl.copied)) != hipSuccess)   // staging of its last upload
    return handle_fail(h, int(e), "wait for an earlier dictionary upload");
  if (sl.pinned_bytes < need) {
    if (sl.pinned) (void)hipHostFree(sl.pinned);
    sl.pinned = nullptr;
    sl.pinned_bytes = 0;
    if (hipHostMalloc(&sl.pinned, need, hipHostMallocDefault) != hipSuccess) {
      sl.pinned = nullptr;
      return fail(RSC_E_NOMEM, "hipHostMalloc for the dictionary staging failed");
    }
    sl.pinned_bytes = need;
  }
  if (sl.bytes < need) {
    // launches in flight may still read the arena: wait for them before it is freed
    for (auto& u : sl.users)
      if ((e = hipEventSynchronize(u.second)) != hipSuccess) return handle_fail(h, int(e), "wait for readers");
    if (sl.arena) (void)hipFree(sl.arena);
    sl.arena = nullptr;
    sl.bytes = 0;
    if (hipMalloc(&sl.arena, need) != hipSuccess) {
      sl.arena = nullptr;
      return fail(RSC_E_NOMEM, "hipMalloc for the dictionary tables failed");
    }
    sl.bytes = need;
  }
  if (!sl.copied && (e = hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming)) != hipSuccess)
    return handle_fail(h, int(e), "event creation");
  std::memcpy(sl.pinned, arena.staging.data(), need);
  // the copy waits for every launch that read this arena (events recorded after them)
  for (auto& u : sl.users)
    if ((e = hipStreamWaitEvent(st, u.second, 0)) != hipSuccess)
      return handle_fail(h, int(e), "stream wait before the dictionary upload");
  if ((e = hipMemcpyAsync(sl.arena, sl.pinned, need, hipMemcpyHostToDevice, st)) != hipSuccess)
    return handle_fail(h, int(e), "dictionary upload");
  if ((e = hipEventRecord(sl.copied, st)) != hipSuccess) return handle_fail(h, int(e), "event record");
  // later launches read the new arena
  arena.bind(static_cast<char*>(sl.arena));
  d.M = M;
  d.R = R;
  d.NG = NG;
  d.lpSplit = split;
  d.dictArena = sl.arena;
  d.dictArenaBytes = need;
  h->cur = int(&sl - h->slot);
  h->dict_stream = st;
  h->has_dict = true;
  return ok();
}

rsc_status rsc_set_tile(rsc_handle* h, rsc_tile tile) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (tile != RSC_TILE_AUTO && tile != RSC_TILE_16 && tile != RSC_TILE_32)
    return fail(RSC_E_INVALID, "unknown tile shape");
  h->tile = tile;
  return ok();
}

rsc_status rsc_set_launch(rsc_handle* h, rsc_tile tile, int blocks_per_cu) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (tile != RSC_TILE_AUTO && tile != RSC_TILE_16 && tile != RSC_TILE_32)
    return fail(RSC_E_INVALID, "unknown tile shape");
  if (blocks_per_cu < 0 || blocks_per_cu > 16) return fail(RSC_E_INVALID, "blocks_per_cu must be in 0..16");
  h->tile = tile;
  h->dev.enc_bpc = blocks_per_cu;
  return ok();
}

rsc_status rsc_autotune_encode(rsc_handle* h, const float* xhat, int64_t P, int K, int32_t* atom,
                               int32_t* angle, float* coef, int reps, double* report, int* n_report,
                               void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (!h->has_dict) return fail(RSC_E_NOT_READY, "no dictionary loaded");
  if (K < 1 || K > 8 || K > h->dev.B) return fail(RSC_E_INVALID, "K must be in 1..min(8, B)");
  if (P < 1 || !xhat || !atom || !angle || !coef) return fail(RSC_E_INVALID, "need a non-empty sample");
  if (reps < 1 || reps > 100) return fail(RSC_E_INVALID, "reps must be in 1..100");
  if (rsc_status f = check_fault(h)) return f;
  if (rsc_status f = dict_before(h, stream)) return f;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bool lp = h->prec != RSC_FP32;
  int tiles[2] = {lp ? RSC_TILE_32 : RSC_TILE_16, RSC_TILE_32};
  const int ntiles = (!lp && rsc::tile32_usable(h->dev, K)) ? 2 : 1;
  auto run = [&](int tile) {
    return lp ? rsc::launch_encode_lp(h->dev, h->prec, xhat, P, K, atom, angle, coef, nullptr, stream)
              : rsc::launch_encode(h->dev, tile, xhat, P, K, atom, angle, coef, nullptr, stream);
  };
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(RSC_E_DEVICE, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(RSC_E_DEVICE, "hipEventCreate failed");
  }
  const int saved_bpc = h->dev.enc_bpc;
  double best_ms = 1e300;
  int best_tile = RSC_TILE_16, best_bpc = 0, nrep = 0;
  rsc_status status = RSC_OK;
  for (int ti = 0; ti < ntiles && status == RSC_OK; ++ti) {
    for (int bpc = 1; bpc <= 4 && status == RSC_OK; ++bpc) {
      h->dev.enc_bpc = bpc;
      int e = run(tiles[ti]);
      if (e) { status = handle_fail(h, e, "autotune launch"); break; }
      std::vector<float> ms(reps);
      for (int r = 0; r < reps && status == RSC_OK; ++r) {
        if (hipEventRecord(e0, st) != hipSuccess) { status = fail(RSC_E_DEVICE, "event record"); break; }
        e = run(tiles[ti]);
        if (e) { status = handle_fail(h, e, "autotune launch"); break; }
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms[r], e0, e1) != hipSuccess) {
          status = fail(RSC_E_DEVICE, "event timing");
          break;
        }
      }
      if (status != RSC_OK) break;
      std::sort(ms.begin(), ms.end());
      const double med = ms[reps / 2];
      if (report && nrep < 8) {
        report[3 * nrep] = tiles[ti];
        report[3 * nrep + 1] = bpc;
        report[3 * nrep + 2] = med;
      }
      ++nrep;
      if (med < best_ms) {
        best_ms = med;
        best_tile = tiles[ti];
        best_bpc = bpc;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status == RSC_OK) status = dict_after(h, stream);
  if (status != RSC_OK) {
    h->dev.enc_bpc = saved_bpc;
    return status;
  }
  h->tile = rsc_tile(best_tile);
  h->dev.enc_bpc = best_bpc;
  if (n_report) *n_report = nrep < 8 ? nrep : 8;
  return ok();
}

// Tile shape of the FP32 encoder: RSC_TILE_32 when asked for (or, under RSC_TILE_AUTO, when
// R > 32) and compiled for the geometry and K; else RSC_TILE_16.  With R <= 32 the 32x32
// tile's 32 angle rows are half empty (R/2 <= 16 rows after the parity split), and the 16x16
// tile does less work per patch and runs twice as many waves.
int encoder_tile(const rsc_handle* h, int K) {
  const bool want32 = h->tile == RSC_TILE_32 || (h->tile == RSC_TILE_AUTO && h->dev.R > 32);
  return want32 && rsc::tile32_usable(h->dev, K) ? RSC_TILE_32 : RSC_TILE_16;
}

rsc_status rsc_encode_info(const rsc_handle* h, int K, int* tile, double* mfma_flops_per_patch) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (!h->has_dict) return fail(RSC_E_NOT_READY, "no dictionary loaded");
  if (K < 1 || K > 8 || K > h->dev.B) return fail(RSC_E_INVALID, "K must be in 1..min(8, B)");
  if (h->prec != RSC_FP32) {
    if (tile) *tile = RSC_TILE_32;
    if (mfma_flops_per_patch) *mfma_flops_per_patch = rsc::encode_lp_mfma_flops_per_patch(h->dev, K);
    return ok();
  }
  const int t = encoder_tile(h, K);
  if (tile) *tile = t;
  if (mfma_flops_per_patch) *mfma_flops_per_patch = rsc::encode_mfma_flops_per_patch(h->dev, t, K);
  return ok();
}

rsc_status rsc_get_launch(const rsc_handle* h, int* tile, int* blocks_per_cu) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (tile) *tile = h->tile;
  if (blocks_per_cu) *blocks_per_cu = h->dev.enc_bpc;
  return ok();
}

rsc_status rsc_project(const rsc_handle* h, const float* patches, int64_t P, float* xhat, void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (P < 0) return fail(RSC_E_INVALID, "P must be >= 0");
  if (P == 0) return ok();
  if (!patches || !xhat) return fail(RSC_E_INVALID, "null device pointer");
  if (P > (int64_t(1) << 31) * 64) return fail(RSC_E_INVALID, "P too large");
  if (rsc_status f = check_fault(h)) return f;
  int e = rsc::launch_project(h->dev, patches, P, xhat, stream);
  return e ? handle_fail(h, e, "projection launch") : ok();
}

rsc_status rsc_omp_encode(const rsc_handle* h, const float* xhat, int64_t P, int K, void* workspace,
                          size_t ws_bytes, int32_t* atom, int32_t* angle, float* coef, float* resid2,
                          void* stream) {
  (void)workspace;   // the pursuit keeps every per-patch value in registers: no workspace is read
  (void)ws_bytes;    // (rsc_encode_workspace_size is 0, so every ws_bytes is enough)
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (!h->has_dict) return fail(RSC_E_NOT_READY, "no dictionary loaded");
  if (K < 1 || K > 8 || K > h->dev.B) return fail(RSC_E_INVALID, "K must be in 1..min(8, B)");
  if (h->annular && K > rsc::kAnnularMaxK)
    return fail(RSC_E_UNSUPPORTED, "the pursuit on the annular basis is compiled for K <= 4");
  if (P < 0) return fail(RSC_E_INVALID, "P must be >= 0");
  if (P == 0) return ok();
  if (!xhat || !atom || !angle || !coef) return fail(RSC_E_INVALID, "null device pointer");
  if (rsc_status f = check_fault(h)) return f;
  if (h->prec != RSC_FP32)
    return dict_launch(h, stream, "encode launch", [&] {
      return rsc::launch_encode_lp(h->dev, h->prec, xhat, P, K, atom, angle, coef, resid2, stream);
    });
  const int tile = encoder_tile(h, K);
  return dict_launch(h, stream, "encode launch", [&] {
    return rsc::launch_encode(h->dev, tile, xhat, P, K, atom, angle, coef, resid2, stream);
  });
}

rsc_status rsc_reconstruct(const rsc_handle* h, const int32_t* atom, const int32_t* angle,
                           const float* coef, int64_t P, int K, float* out, void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (!h->has_dict) return fail(RSC_E_NOT_READY, "no dictionary loaded");
  if (K < 1 || K > 16) return fail(RSC_E_INVALID, "K must be in 1..16");
  if (P < 0) return fail(RSC_E_INVALID, "P must be >= 0");
  if (P == 0) return ok();
  if (!atom || !angle || !coef || !out) return fail(RSC_E_INVALID, "null device pointer");
  if (P > (int64_t(1) << 31) * 8) return fail(RSC_E_INVALID, "P too large");
  if (rsc_status f = check_fault(h)) return f;
  return dict_launch(h, stream, "reconstruct launch", [&] {
    return rsc::launch_synthesize(h->dev, atom, angle, nullptr, coef, P, K, nullptr, out, stream);
  });
}

rsc_status rsc_synthesize(const rsc_handle* h, const int32_t* atom, const float* theta,
                          const float* weight, int64_t P, int J, const float* noise, float* out,
                          void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (!h->has_dict) return fail(RSC_E_NOT_READY, "no dictionary loaded");
  if (J < 1 || J > 16) return fail(RSC_E_INVALID, "J must be in 1..16");
  if (P < 0) return fail(RSC_E_INVALID, "P must be >= 0");
  if (P == 0) return ok();
  if (!atom || !theta || !weight || !out) return fail(RSC_E_INVALID, "null device pointer");
  if (P > (int64_t(1) << 31) * 8) return fail(RSC_E_INVALID, "P too large");
  if (rsc_status f = check_fault(h)) return f;
  return dict_launch(h, stream, "synthesize launch", [&] {
    return rsc::launch_synthesize(h->dev, atom, nullptr, theta, weight, P, J, noise, out, stream);
  });
}

// Image projection instances: 11x11 windows (97 disk pixels) with B <= 96 (the 11x11 grid
// of profiles and the annular basis) and 15x15 windows (177 disk pixels) with 64 < B <= 160
// (the 15x15 grid and the annular basis).
static bool images_supported(const rsc_handle* h) {
  const auto& d = h->dev;
  return (d.N == 11 && d.n_pix == 97 && d.B <= 96) || (d.N == 15 && d.n_pix == 177 && d.B > 64 && d.B <= 160);
}

rsc_status rsc_images_workspace_size(int n_images, size_t* bytes) {
  if (!bytes) return fail(RSC_E_INVALID, "bytes is NULL");
  if (n_images < 0) return fail(RSC_E_INVALID, "n_images must be >= 0");
  *bytes = rsc::images_workspace_bytes(n_images);
  return ok();
}

rsc_status rsc_project_images(const rsc_handle* h, const float* pixels, const int64_t* img_offset,
                              const int32_t* H, const int32_t* W, int n_images, int64_t P_total,
                              void* workspace, size_t ws_bytes, float* xhat, void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (n_images < 0 || n_images > (1 << 20)) return fail(RSC_E_INVALID, "n_images must be in 0..2^20");
  if (P_total < 0) return fail(RSC_E_INVALID, "P_total must be >= 0");
  if (n_images == 0 || P_total == 0) return ok();
  if (!pixels || !img_offset || !H || !W || !workspace || !xhat)
    return fail(RSC_E_INVALID, "null device pointer");
  if (ws_bytes < rsc::images_workspace_bytes(n_images)) return fail(RSC_E_INVALID, "workspace too small");
  if ((reinterpret_cast<uintptr_t>(workspace) & 7) != 0) return fail(RSC_E_INVALID, "workspace not 8-byte aligned");
  if (!images_supported(h))
    return fail(RSC_E_UNSUPPORTED, "image projection is compiled for 11x11 windows with B <= 96 and 15x15 "
                                   "windows with 64 < B <= 160");
  if (rsc_status f = check_fault(h)) return f;
  int e = rsc::launch_project_images(h->dev, pixels, img_offset, H, W, n_images, P_total, workspace, xhat,
                                     stream);
  return e ? handle_fail(h, e, "image projection launch") : ok();
}

rsc_status rsc_project_images_noalloc(const rsc_handle* h, const float* pixels, const int64_t* img_offset,
                                      const int32_t* H, const int32_t* W, int n_images, int64_t P_total,
                                      float* xhat, void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (n_images < 0 || n_images > rsc::kNoAllocMaxImages)
    return fail(RSC_E_INVALID, "n_images must be in 0.." + std::to_string(rsc::kNoAllocMaxImages) +
                                   " (the size of the library's static plan buffer)");
  if (P_total < 0) return fail(RSC_E_INVALID, "P_total must be >= 0");
  if (n_images == 0 || P_total == 0) return ok();
  if (!pixels || !img_offset || !H || !W || !xhat) return fail(RSC_E_INVALID, "null device pointer");
  if (!images_supported(h))
    return fail(RSC_E_UNSUPPORTED, "image projection is compiled for 11x11 windows with B <= 96 and 15x15 "
                                   "windows with 64 < B <= 160");
  if (rsc_status f = check_fault(h)) return f;
  int e = rsc::launch_project_images_noalloc(h->dev, pixels, img_offset, H, W, n_images, P_total, xhat, stream);
  return e ? handle_fail(h, e, "image projection launch") : ok();
}

rsc_status rsc_synthesize_images(const rsc_handle* h, const int32_t* atom, const float* theta,
                                 const float* amplitude, const int32_t* centre, const int32_t* image,
                                 int64_t n_stamps, const int64_t* img_offset, const int32_t* H,
                                 const int32_t* W, int n_images, float* pixels, void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (!h->has_dict) return fail(RSC_E_NOT_READY, "no dictionary loaded");
  if (n_stamps < 0 || n_stamps > (int64_t(1) << 31) - 1) return fail(RSC_E_INVALID, "n_stamps out of range");
  if (h->annular) return fail(RSC_E_UNSUPPORTED, "image stamping is compiled for the (S, T) grid of profiles");
  if (n_stamps == 0) return ok();
  if (!atom || !theta || !amplitude || !centre || !image || !img_offset || !H || !W || !pixels)
    return fail(RSC_E_INVALID, "null device pointer");
  if (rsc_status f = check_fault(h)) return f;
  return dict_launch(h, stream, "stamp launch", [&] {
    return rsc::launch_stamps(h->dev, atom, theta, amplitude, centre, image, n_stamps, img_offset, H, W,
                              n_images, pixels, stream);
  });
}


rsc_status rsc_rksvd_workspace_size(const rsc_handle* h, int64_t P, int K, size_t* bytes) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (!bytes) return fail(RSC_E_INVALID, "bytes is NULL");
  if (!h->has_dict) return fail(RSC_E_NOT_READY, "no dictionary loaded");
  if (P < 1 || P > INT32_MAX) return fail(RSC_E_INVALID, "P must be in 1..2^31-1");
  if (K < 1 || K > 8) return fail(RSC_E_INVALID, "K must be in 1..8");
  *bytes = rk_layout(h->dev, P, K).total;
  return ok();
}

rsc_status rsc_rksvd_update(const rsc_handle* h, const float* xhat, int64_t P, int K, const int32_t* atom,
                            const int32_t* angle, const float* coef, const float* resid2, void* workspace,
                            size_t ws_bytes, float* d_new, int32_t* usage, int32_t* reset, void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (!h->has_dict) return fail(RSC_E_NOT_READY, "no dictionary loaded");
  if (K < 1 || K > 8) return fail(RSC_E_INVALID, "K must be in 1..8");
  if (P < 1 || P > INT32_MAX) return fail(RSC_E_INVALID, "P must be in 1..2^31-1");
  if (!xhat || !atom || !angle || !coef || !resid2 || !workspace || !d_new || !usage)
    return fail(RSC_E_INVALID, "null device pointer");
  if (!rsc::rksvd_fits(h->dev))
    return fail(RSC_E_UNSUPPORTED, "the dictionary update is compiled for B <= 160 with its tables within the "
                                   "160 KiB LDS of a CU");
  const RkLayout L = rk_layout(h->dev, P, K);
  if (ws_bytes < L.total) return fail(RSC_E_INVALID, "workspace too small");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(RSC_E_INVALID, "workspace not 256-byte aligned");
  int32_t* rs = reset ? reset : reinterpret_cast<int32_t*>(reinterpret_cast<char*>(workspace) + L.reset);
  if (rsc_status f = check_fault(h)) return f;
  return dict_launch(h, stream, "dictionary update launch", [&] {
    return rsc::launch_rksvd_update(h->dev, xhat, P, K, atom, angle, coef, resid2, workspace, d_new, usage, rs,
                                    stream);
  });
}

rsc_status rsc_rksvd_train(rsc_handle* h, const float* xhat, int64_t P, int K, int n_iter, const float* d_init,
                           int M, int R, void* workspace, size_t ws_bytes, int32_t* atom, int32_t* angle,
                           float* coef, float* resid2, float* d_out, double* history, void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (n_iter < 0 || n_iter > 10000) return fail(RSC_E_INVALID, "n_iter must be in 0..10000");
  if (!d_init || !d_out) return fail(RSC_E_INVALID, "null host pointer");
  if (K < 1 || K > 8) return fail(RSC_E_INVALID, "K must be in 1..8");
  if (P > INT32_MAX) return fail(RSC_E_INVALID, "P must be in 1..2^31-1");
  if (P < 1 || !xhat || !atom || !angle || !coef || !resid2 || !workspace)
    return fail(RSC_E_INVALID, "null device pointer or empty input");
  {
    rsc::DeviceTables want = h->dev;   // the update's sizes with the new dictionary (a shallow copy)
    want.M = M;
    want.R = R;
    if (!rsc::rksvd_fits(want))
      return fail(RSC_E_UNSUPPORTED, "the dictionary update is compiled for B <= 160 with its tables within the "
                                     "160 KiB LDS of a CU");
  }
  rsc_status s = rsc_set_dictionary(h, d_init, M, R, stream);
  if (s != RSC_OK) return s;
  const RkLayout L = rk_layout(h->dev, P, K);
  if (ws_bytes < L.total) return fail(RSC_E_INVALID, "workspace too small");
  char* w = reinterpret_cast<char*>(workspace);
  float* dn = reinterpret_cast<float*>(w + L.dnew);
  int32_t* us = reinterpret_cast<int32_t*>(w + L.usage);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<float> host(size_t(M) * h->dev.B);
  std::memcpy(host.data(), d_init, host.size() * sizeof(float));
  auto coding_error = [&](int at) -> rsc_status {
    if (!history) return RSC_OK;
    double* slot = rk_sum_slot(h->dev, P, K, workspace);
    int e = rsc::launch_sum(resid2, P, slot, stream);
    if (e) return handle_fail(h, e, "sum launch");
    hipError_t he = hipMemcpyAsync(&history[at], slot, sizeof(double), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    return he == hipSuccess ? RSC_OK : handle_fail(h, int(he), "history copy");
  };
  for (int it = 0; it <= n_iter; ++it) {
    s = rsc_omp_encode(h, xhat, P, K, nullptr, 0, atom, angle, coef, resid2, stream);
    if (s == RSC_OK) s = coding_error(it);
    if (s != RSC_OK || it == n_iter) break;
    s = rsc_rksvd_update(h, xhat, P, K, atom, angle, coef, resid2, workspace, ws_bytes, dn, us, nullptr, stream);
    if (s != RSC_OK) break;
    hipError_t he = hipMemcpyAsync(host.data(), dn, host.size() * sizeof(float), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return handle_fail(h, int(he), "dictionary copy");
    // rows leave the device at unit norm up to FP32 rounding; renormalise in FP64
    for (int m = 0; m < M; ++m) {
      double n2 = 0.0;
      for (int b = 0; b < h->dev.B; ++b) n2 += double(host[size_t(m) * h->dev.B + b]) * host[size_t(m) * h->dev.B + b];
      const double inv = n2 > 0.0 ? 1.0 / std::sqrt(n2) : 0.0;
      for (int b = 0; b < h->dev.B; ++b)
        host[size_t(m) * h->dev.B + b] = float(host[size_t(m) * h->dev.B + b] * inv);
    }
    s = rsc_set_dictionary(h, host.data(), M, R, stream);
    if (s != RSC_OK) break;
  }
  if (s != RSC_OK) return s;
  std::memcpy(d_out, host.data(), host.size() * sizeof(float));
  return ok();
}


rsc_status rsc_classify_workspace_size(int64_t P, int K, size_t* bytes) {
  if (!bytes) return fail(RSC_E_INVALID, "bytes is NULL");
  if (P < 0) return fail(RSC_E_INVALID, "P must be >= 0");
  if (K < 1 || K > 8) return fail(RSC_E_INVALID, "K must be in 1..8");
  *bytes = cls_layout(P, K).total;
  return ok();
}

rsc_status rsc_classify(const rsc_handle* const* classes, int C, const float* xhat, int64_t P, int K,
                        void* workspace, size_t ws_bytes, int32_t* label, float* sse, void* stream) {
  if (!classes) return fail(RSC_E_INVALID, "classes is NULL");
  if (C < 1 || C > 1024) return fail(RSC_E_INVALID, "C must be in 1..1024");
  for (int c = 0; c < C; ++c) {
    if (!classes[c]) return fail(RSC_E_INVALID, "a class handle is NULL");
    if (!classes[c]->has_dict) return fail(RSC_E_NOT_READY, "a class handle has no dictionary");
    const rsc::HostBasis& b0 = classes[0]->basis;
    const rsc::HostBasis& bc = classes[c]->basis;
    if (bc.N != b0.N || bc.S != b0.S || bc.T != b0.T || classes[c]->annular != classes[0]->annular ||
        classes[c]->dev.B != classes[0]->dev.B)
      return fail(RSC_E_INVALID, "class handles must share the geometry: the same (N, S, T) grid or the same "
                                 "annular basis");
  }
  if (K < 1 || K > 8 || K > classes[0]->dev.B) return fail(RSC_E_INVALID, "K must be in 1..min(8, B)");
  if (P < 0) return fail(RSC_E_INVALID, "P must be >= 0");
  if (P == 0) return ok();
  if (!xhat || !workspace || !label || !sse) return fail(RSC_E_INVALID, "null device pointer");
  const ClsLayout L = cls_layout(P, K);
  if (ws_bytes < L.total) return fail(RSC_E_INVALID, "workspace too small");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(RSC_E_INVALID, "workspace not 256-byte aligned");
  char* w = static_cast<char*>(workspace);
  int32_t* atom = reinterpret_cast<int32_t*>(w + L.atom);
  int32_t* angle = reinterpret_cast<int32_t*>(w + L.angle);
  float* coef = reinterpret_cast<float*>(w + L.coef);
  float* r2 = reinterpret_cast<float*>(w + L.resid);
  for (int c = 0; c < C; ++c) {
    rsc_status s = rsc_omp_encode(classes[c], xhat, P, K, nullptr, 0, atom, angle, coef, r2, stream);
    if (s != RSC_OK) return s;
    int e = rsc::launch_classify_min(r2, P, c, label, sse, stream);
    if (e) return handle_fail(classes[c], e, "classify launch");
  }
  return ok();
}

rsc_status rsc_label_histogram(const int32_t* label, int64_t P, const int64_t* offset, int n_groups, int C,
                               float* hist, void* stream) {
  if (n_groups < 0) return fail(RSC_E_INVALID, "n_groups must be >= 0");
  if (C < 1 || C > 4096) return fail(RSC_E_INVALID, "C must be in 1..4096");
  if (P < 0) return fail(RSC_E_INVALID, "P must be >= 0");
  if (n_groups == 0) return ok();
  if (n_groups > (1 << 30)) return fail(RSC_E_INVALID, "too many groups");
  if (!offset || !hist || (P > 0 && !label)) return fail(RSC_E_INVALID, "null device pointer");
  int e = rsc::launch_label_hist(label, P, offset, n_groups, C, hist, stream);
  return e ? device_fail(e, "histogram launch") : ok();
}

rsc_status rsc_chi2_nearest(const float* train, int n_train, const float* test, int n_test, int C,
                            int32_t* nearest, float* dist, void* stream) {
  if (n_train < 1) return fail(RSC_E_INVALID, "n_train must be >= 1");
  if (n_test < 0) return fail(RSC_E_INVALID, "n_test must be >= 0");
  if (C < 1 || C > 4096) return fail(RSC_E_INVALID, "C must be in 1..4096");
  if (n_test == 0) return ok();
  if (n_test > (1 << 30)) return fail(RSC_E_INVALID, "too many test histograms");
  if (!train || !test || !nearest) return fail(RSC_E_INVALID, "null device pointer");
  int e = rsc::launch_chi2_nearest(train, n_train, test, n_test, C, nearest, dist, stream);
  return e ? device_fail(e, "nearest-neighbour launch") : ok();
}

struct rsc_rotation_plan {
  int N = 0, ntap = 0;
  int32_t* src = nullptr;   // [N*N][ntap] in lane order
  float* w = nullptr;
  int32_t* pix = nullptr;   // output pixel of each lane
  float* op = nullptr;      // steering plans: Phi S_theta Phi^+ as 4 row tiles x 49 x 64 operands
  int* opPix = nullptr;     // its contraction order (disk pixels, -1 past the disk)
};

rsc_status rsc_rotation_plan_create(int N, double theta, int mode, rsc_rotation_plan** plan) {
  if (!plan) return fail(RSC_E_INVALID, "plan is NULL");
  *plan = nullptr;
  if (N < 3 || N > 25 || N % 2 == 0) return fail(RSC_E_INVALID, "N must be odd, 3..25");
  if (mode != 0 && mode != 1) return fail(RSC_E_INVALID, "mode must be 0 (nearest) or 1 (bicubic)");
  if (!std::isfinite(theta)) return fail(RSC_E_INVALID, "theta must be finite");
  std::vector<int32_t> src, pix;
  std::vector<float> w;
  const int ntap = rsc::rotation_taps(N, theta, mode, src, w, pix);
  auto* p = new (std::nothrow) rsc_rotation_plan;
  if (!p) return fail(RSC_E_NOMEM, "plan allocation failed");
  p->N = N;
  p->ntap = ntap;
  rsc_status s = upload(p->src, src, "rotation taps");
  if (s == RSC_OK) s = upload(p->w, w, "rotation weights");
  if (s == RSC_OK) s = upload(p->pix, pix, "rotation lane order");
  if (s != RSC_OK) {
    free_dev(p->src);
    free_dev(p->w);
    free_dev(p->pix);
    delete p;
    return s;
  }
  *plan = p;
  return ok();
}

rsc_status rsc_rotation_plan_create_steer(const rsc_handle* h, double theta, rsc_rotation_plan** plan) {
  if (!plan) return fail(RSC_E_INVALID, "plan is NULL");
  *plan = nullptr;
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (!std::isfinite(theta)) return fail(RSC_E_INVALID, "theta must be finite");
  const rsc::HostBasis& b = h->basis;
  if (h->annular || b.N != 11 || b.n_pix != 97)
    return fail(RSC_E_UNSUPPORTED, "steering plans are compiled for 11x11 handles of rsc_create");
  const int NN = b.N * b.N, S = b.S, T = b.T, B = b.B, KPD = 49;
  // column i of the operator: Phi (S_theta (column pix[i] of Phi^+)); harmonic k >= 1 of the
  // packed coordinates (Re block, then Im block, S profiles each) turns by k theta
  std::vector<double> M(size_t(NN) * b.n_pix, 0.0), v(B), sv(B);
  for (int i = 0; i < b.n_pix; ++i) {
    for (int c = 0; c < B; ++c) v[c] = b.pinv[size_t(c) * NN + b.pix[i]];
    for (int c = 0; c < S; ++c) sv[c] = v[c];
    for (int k = 1; k <= T; ++k) {
      const double ck = std::cos(k * theta), sk = std::sin(k * theta);
      for (int s = 0; s < S; ++s) {
        const int re = S + 2 * S * (k - 1) + s, im = re + S;
        sv[re] = v[re] * ck + v[im] * sk;
        sv[im] = v[im] * ck - v[re] * sk;
      }
    }
    for (int q = 0; q < NN; ++q) {
      double acc = 0.0;
      for (int c = 0; c < B; ++c) acc += b.phi[size_t(q) * B + c] * sv[c];
      M[size_t(q) * b.n_pix + i] = acc;
    }
  }
  std::vector<float> op(size_t(4) * KPD * 64, 0.f);
  for (int t = 0; t < 4; ++t)
    for (int j = 0; j < KPD; ++j)
      for (int l = 0; l < 64; ++l) {
        const int row = 32 * t + (l % 32), i = 2 * j + l / 32;
        if (row < NN && i < b.n_pix) op[(size_t(t) * KPD + j) * 64 + l] = float(M[size_t(row) * b.n_pix + i]);
      }
  std::vector<int> opPix(size_t(2) * KPD, -1);
  for (int i = 0; i < b.n_pix; ++i) opPix[i] = b.pix[i];
  auto* p = new (std::nothrow) rsc_rotation_plan;
  if (!p) return fail(RSC_E_NOMEM, "plan allocation failed");
  p->N = b.N;
  p->ntap = 0;
  rsc_status st = upload(p->op, op, "steering operator");
  if (st == RSC_OK) st = upload(p->opPix, opPix, "steering operator pixels");
  if (st != RSC_OK) {
    free_dev(p->op);
    free_dev(p->opPix);
    delete p;
    return st;
  }
  *plan = p;
  return ok();
}

rsc_status rsc_rotation_plan_destroy(rsc_rotation_plan* plan) {
  if (!plan) return ok();
  free_dev(plan->src);
  free_dev(plan->w);
  free_dev(plan->pix);
  free_dev(plan->op);
  free_dev(plan->opPix);
  delete plan;
  return ok();
}

rsc_status rsc_rotate_interp(const rsc_rotation_plan* plan, const float* patches, int64_t P, float* out,
                             void* stream) {
  if (!plan) return fail(RSC_E_INVALID, "plan is NULL");
  if (P < 0) return fail(RSC_E_INVALID, "P must be >= 0");
  if (P == 0) return ok();
  if (!patches || !out) return fail(RSC_E_INVALID, "null device pointer");
  if (patches == out) return fail(RSC_E_INVALID, "patches and out must be distinct");
  if (plan->op) {
    if ((reinterpret_cast<uintptr_t>(patches) & 15) != 0)
      return fail(RSC_E_INVALID, "steering plans need 16-byte aligned patches");
    const int e = rsc::launch_rotate_operator(plan->op, plan->opPix, patches, P, out, stream);
    return e ? device_fail(e, "rotation launch") : ok();
  }
  int e = rsc::launch_rotate_taps(plan->N, plan->ntap, patches, P, plan->src, plan->w, plan->pix, out, stream);
  return e ? device_fail(e, "rotation launch") : ok();
}

rsc_status rsc_steer(const rsc_handle* h, const float* xhat, int64_t P, const float* theta, double theta0,
                     float* out, void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (P < 0) return fail(RSC_E_INVALID, "P must be >= 0");
  if (h->dev.T > 31) return fail(RSC_E_UNSUPPORTED, "steering is compiled for T <= 31");
  if (!theta && !std::isfinite(theta0)) return fail(RSC_E_INVALID, "theta0 must be finite");
  if (P == 0) return ok();
  if (!xhat || !out) return fail(RSC_E_INVALID, "null device pointer");
  if (xhat == out) return fail(RSC_E_INVALID, "xhat and out must be distinct");
  if (rsc_status f = check_fault(h)) return f;
  int e = rsc::launch_steer(h->dev, xhat, P, theta, theta0, out, stream);
  return e ? handle_fail(h, e, "steering launch") : ok();
}

rsc_status rsc_synthesize_hat(const rsc_handle* h, const float* xhat, int64_t P, float* pixels, void* stream) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (P < 0) return fail(RSC_E_INVALID, "P must be >= 0");
  if (h->dev.B > 192) return fail(RSC_E_UNSUPPORTED, "synthesis is compiled for B <= 192");
  if (P == 0) return ok();
  if (!xhat || !pixels) return fail(RSC_E_INVALID, "null device pointer");
  if (rsc_status f = check_fault(h)) return f;
  int e = rsc::launch_synth_hat(h->dev, xhat, P, pixels, stream);
  return e ? handle_fail(h, e, "synthesis launch") : ok();
}

rsc_status rsc_precision_stats(rsc_handle* h, int64_t* out, int reset) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (!h->dev.lpStats) return fail(RSC_E_UNSUPPORTED, "this handle keeps no counters");
  if (rsc_status f = check_fault(h)) return f;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return handle_fail(h, int(e), "device synchronize");
  unsigned long long v[4];
  e = hipMemcpy(v, h->dev.lpStats, sizeof(v), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return handle_fail(h, int(e), "counter read");
  if (out)
    for (int i = 0; i < 4; ++i) out[i] = int64_t(v[i]);
  if (reset) {
    e = hipMemset(h->dev.lpStats, 0, sizeof(v));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return handle_fail(h, int(e), "counter reset");
  }
  return ok();
}

rsc_status rsc_sync(rsc_handle* h, void* stream) {
  hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return handle_fail(h, int(e), "stream synchronize");
  if (rsc_status f = check_fault(h)) return f;
  return ok();
}

rsc_status rsc_encode_workspace_size(const rsc_handle* h, int64_t P, int K, size_t* bytes) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (!bytes) return fail(RSC_E_INVALID, "bytes is NULL");
  if (P < 0) return fail(RSC_E_INVALID, "P must be >= 0");
  if (K < 1 || K > 8 || K > h->dev.B) return fail(RSC_E_INVALID, "K must be in 1..min(8, B)");
  *bytes = 0;   // every per-patch value of the pursuit stays in registers
  return ok();
}

rsc_status rsc_set_fault(rsc_handle* h, const char* msg) {
  if (!h) return fail(RSC_E_INVALID, "handle is NULL");
  if (h->fault == RSC_OK) {
    h->fault = RSC_E_DEVICE;
    h->fault_msg = msg ? msg : "fault set by the caller";
  }
  return ok();
}

}  // extern "C"
