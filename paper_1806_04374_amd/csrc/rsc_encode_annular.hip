// Rotational OMP on the paper's own discrete steerable basis (eq. (5)-(7): annuli with
// harmonics up to half their circumference; steering eq. (8)), Fig. 2 with R_r -> S_r.
//
// The coordinates are ragged: harmonic k lives on the Sk(k) annuli whose cut-off reaches
// it (5, 5, 4, 4, 3 x5, 2 x3, 1 x4 at N = 11, B = 81; up to harmonic 19 at N = 15,
// B = 153).  The 16x16-tile encoder of rsc_encode16.h handles that layout as it handles
// the (S, T) grid: stage 1 contracts each harmonic over its own annuli (ceil(Sk/2) steps
// of 4 lanes, (Re, Im) of two annuli each), stage 2 is the angle DFT over the T + 1
// harmonics, split once by parity for even R; the least squares and the residual update
// steer each harmonic block by its own count.  Compiled for even R <= 64 and K <= 4.
#include <hip/hip_runtime.h>

#include "rsc_device.h"
#include "rsc_encode16.h"
#include "rsc_internal.h"
#include "rsc_launch.h"

namespace rsc {
namespace {

template <class C, int HT, int KMAX>
int launchA(const DeviceTables& t, const enc::EncodeParams& prm, hipStream_t st) {
  const int64_t tiles = (prm.P + 15) / 16;
  if (encode16_irows(t))
    return launch_persistent_n(enc::encode16_kernel<C, HT, KMAX, true, true>, encode16_threads(tiles),
                               encode16_lds_bytes(t, true), tiles, t.enc_bpc, st, prm);
  return launch_persistent(enc::encode16_kernel<C, HT, KMAX, true, false>, encode16_lds_bytes(t, false), tiles,
                           t.enc_bpc, st, prm);
}

template <class C>
int dispatchA(const DeviceTables& t, const enc::EncodeParams& prm, hipStream_t st) {
  const bool two_tiles = t.R / 2 > 16;           // 16-row angle tiles covering r < R/2
  if (prm.K <= 2) return two_tiles ? launchA<C, 2, 2>(t, prm, st) : launchA<C, 1, 2>(t, prm, st);
  return two_tiles ? launchA<C, 2, 4>(t, prm, st) : launchA<C, 1, 4>(t, prm, st);
}

}  // namespace

int launch_encode_annular(const DeviceTables& t, const float* xhat, int64_t P, int K, int32_t* atom,
                          int32_t* angle, float* coef, float* resid2, void* stream) {
  if (P <= 0) return 0;
  if (K < 1 || K > kAnnularMaxK || t.R % 2 != 0 || t.R > kAnnularMaxR) return int(hipErrorInvalidValue);
  const enc::EncodeParams prm{xhat, P, K, t.M, t.R, nullptr, t.dictHat, t.dftA16s, t.cs, t.gramH, t.gramH64,
                              t.cs64, atom, angle, coef, resid2, t.lpStats, t.dictHatI};
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (t.geo == kGeoAnnular11) return dispatchA<AnnularCounts11>(t, prm, st);
  if (t.geo == kGeoAnnular15) return dispatchA<AnnularCounts15>(t, prm, st);
  return int(hipErrorInvalidValue);
}

}  // namespace rsc
