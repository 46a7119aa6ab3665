// Internal interfaces of librsc (not part of the C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "rsc.h"

namespace rsc {

// FP64 steerable basis on the host.  phi is [N*N][B] and pinv is [B][N*N] with
// zero rows / columns for pixels outside the disk.
struct HostBasis {
  int N = 0, S = 0, T = 0, B = 0, n_pix = 0;
  double cond = 0.0;
  std::vector<int> pix;        // disk pixels, row-major grid index
  std::vector<double> phi;     // [N*N][B]
  std::vector<double> pinv;    // [B][N*N]
};

bool build_basis(int N, int S, int T, const double* centres, double sigma, HostBasis& out,
                 std::string& err);
// The paper's annular basis; Ts receives the cut-off of each annulus.
bool build_annular_basis(int N, bool lowpass, HostBasis& out, std::vector<int>& Ts, std::string& err);

// Geometry-dependent constants of the encoder.  Stage-1 contraction steps: the
// k = 0 block pairs profiles (s, s+1) per step, every k >= 1 block uses one step
// per profile with (Re, Im) as the two contraction lanes.
constexpr int k0_steps(int S) { return (S + 1) / 2; }
constexpr int stage1_steps(int S, int T) { return k0_steps(S) + T * S; }

// Coordinate layouts the encoders are compiled for: the (S, T) grid of Gaussian profiles,
// and the paper's annular basis at N = 11 and N = 15 (ragged counts per harmonic).
constexpr int kGeoGrid = 0, kGeoAnnular11 = 11, kGeoAnnular15 = 15, kGeoAnnularOther = -1;

// Device tables owned by a handle (FP32 operand arrangements built on the host).
struct DeviceTables {
  int N = 0, S = 0, T = 0, B = 0, n_pix = 0;
  int geo = kGeoGrid;        // coordinate layout (kGeo*)
  int sk[64] = {};           // profiles (annuli) carrying harmonic k, k = 0..T
  int prec = RSC_FP32;       // rsc_precision of the handle
  int M = 0, R = 0, NG = 0;
  int enc_bpc = 0;           // encoder blocks per CU (0: as many as fit)
  float* pinvA = nullptr;    // projection operand over the grid [RTB][ceil(N*N/2)][64]
  float* pinvD = nullptr;    // projection operand over disk pixels [2][ceil(n_pix/2)][64] (B <= 64)
  int* pixD = nullptr;       // grid index of disk pixel i, -1 past n_pix [2*ceil(n_pix/2)] (every B)
  float* pinvI = nullptr;    // projection operand over disk pixels [tiles][ceil(n_pix/2)][64], tiles = 2 (B <= 64), 4 (B <= 128) or ceil(B/32)
  int* dpixI = nullptr;      // (dy << 8 | dx) of disk pixel i, -1 past n_pix [2*ceil(n_pix/2)]
  int* steerTab = nullptr;   // annular basis: per coordinate, harmonic k and partner offset
                             // ((k << 16) | (offset + 32768)); null for the full (S, T) grid
  float* phiPad = nullptr;   // synthesis matrix [N*N][B]
  float* synA = nullptr;     // synthesis MFMA operand [ceil(N*N/32)][ceil(B/2)][64] (N*N <= 256)
  // Dictionary tables (dictA .. cs64 below) point into the bound one of the handle's two
  // device copies (dictArena, dictArenaBytes); each upload fills the other copy.
  void* dictArena = nullptr;
  size_t dictArenaBytes = 0;
  float* dictA = nullptr;    // 32x32-tile stage-1 operand [NG][stage1_steps][64] (S = T = 5 only)
  float* dictHat = nullptr;  // dictionary rows [16*ceil(M/16)][B] (zero rows past M)
  float* dictHatI = nullptr; // i times the dictionary rows, same shape: per harmonic k >= 1 the
                             // (Re, Im) slots hold (-Im d, Re d); zero at k = 0 (16x16 FP32 tile)
  float* dftA32 = nullptr;   // 32x32-tile stage-2 operand, angles r < R/2 [T+1][64] (even R <= 64)
  float* dftA16 = nullptr;   // 16x16-tile stage-2 operand, all angles [ceil(R/16)->1,2,4,8][(T+2)/2][64]
  float* dftA16s = nullptr;  // 16x16-tile stage-2 operand, parity split [ceil(R/32)->1,2,4][E+O steps][64]
  float* cs = nullptr;       // [2][T+1][R]: cos, then sin, of 2 pi k r / R
  float* gramH = nullptr;    // [M][M][2T+1]: per-atom-pair harmonic inner products (see pair_gram)
  // 16-bit encoder (BF16 / FP16 handles)
  uint16_t* lpA = nullptr;   // stage-1 operand [NG][T+1][64][8]
  uint16_t* lpF16 = nullptr; // stage-2 operand [ceil(R/32)][64][8]
  float* lpF32 = nullptr;    // FP32 re-score angle DFT operand: [T+1][64] rows r < R/2 when
                             // lpSplit, else [ceil(R/32)][T+1][64]
  bool lpSplit = false;      // even R in 33..64: radix-2 split in the FP32 re-score
  double* gramH64 = nullptr; // FP64 pair table [M][M][2T+1]
  double* cs64 = nullptr;    // FP64 [2][T+1][R] cos, sin (every handle)
  unsigned long long* lpStats = nullptr;  // [4] counters (rsc_precision_stats)
  // compensated 16-bit projection (N = 11): 3 (BF16) or 2 (FP16) 16-bit parts of the
  // operand over disk pixels [parts][2][ceil(n_pix/16)][64][8], and the grid index of
  // disk pixel i [16 ceil(n_pix/16)]
  uint16_t* lpPinv = nullptr;
  int* lpPix16 = nullptr;
  float lpPinvUnscale = 1.f;  // 2^-s where the operand parts hold 2^s (Phi^T Phi)^{-1} Phi^T
};

// Kernel launchers.  Return a hipError_t as int.
int launch_project(const DeviceTables& t, const float* patches, int64_t P, float* xhat, void* stream);
int launch_encode(const DeviceTables& t, int tile, const float* xhat, int64_t P, int K, int32_t* atom,
                  int32_t* angle, float* coef, float* resid2, void* stream);
int launch_synthesize(const DeviceTables& t, const int32_t* atom, const int32_t* angle_idx,
                      const float* theta, const float* weight, int64_t P, int J,
                      const float* noise, float* out, void* stream);
bool encode_supported(int S, int T);
bool encode_supported_geo(const DeviceTables& t);   // the encoder is compiled for t's layout
// The pursuit on the paper's annular basis (rsc_encode_annular.hip): 16x16 tiles, even
// R <= 64, K <= 4.
constexpr int kAnnularMaxK = 4, kAnnularMaxR = 64;
int launch_encode_annular(const DeviceTables& t, const float* xhat, int64_t P, int K, int32_t* atom,
                          int32_t* angle, float* coef, float* resid2, void* stream);
size_t encode_lds_bytes(const DeviceTables& t, int tile);
// 16x16 FP32 tile: LDS of one block with (irows) or without the i * dictionary copy, whether
// the copy is used (both tables fit a CU), and the block size of a launch over wave_tiles
// tiles of 16 patches with the copy: 512 threads (one block per CU, 8 waves) once the tiles
// fill every CU with 8 waves, else 256 (fewer tiles run faster one wave per SIMD).
size_t encode16_lds_bytes(const DeviceTables& t, bool irows);
bool encode16_irows(const DeviceTables& t);
int encode16_threads(int64_t wave_tiles);
bool tile32_usable(const DeviceTables& t, int K);
double encode_mfma_flops_per_patch(const DeviceTables& t, int tile, int K);
size_t project_tiled_lds_bytes(int N, int n_pix);
// Largest B the dictionary update is compiled for (its covariance tiles: 10 x 10 of 16).
constexpr int kRkMaxB = 160;
// Whether the dictionary update's kernels fit this handle (B <= kRkMaxB and each kernel's
// tables within the 160 KiB LDS of a CU).
bool rksvd_fits(const DeviceTables& t);
size_t rksvd_workspace_bytes(const DeviceTables& t, int64_t P, int K);
int launch_rksvd_update(const DeviceTables& t, const float* xhat, int64_t P, int K, const int32_t* atom,
                        const int32_t* angle, const float* coef, const float* resid2, void* ws,
                        float* d_new, int32_t* usage, int32_t* reset, void* stream);
// Patch rotation (rsc_rotate.hip).
int rotation_taps(int N, double theta, int mode, std::vector<int32_t>& src, std::vector<float>& w,
                  std::vector<int32_t>& pix);
size_t rotate_lds_bytes(int N, int ntap);
int launch_rotate_taps(int N, int ntap, const float* in, int64_t P, const int32_t* src, const float* w,
                       const int32_t* pix, float* out, void* stream);
int launch_rotate_operator(const float* op, const int* pix, const float* patches, int64_t P, float* out,
                           void* stream);
int launch_steer(const DeviceTables& t, const float* xhat, int64_t P, const float* theta, double theta0, float* out,
                 void* stream);
int launch_synth_hat(const DeviceTables& t, const float* xhat, int64_t P, float* out, void* stream);

// Texture classifier (rsc_classify.hip).
int launch_classify_min(const float* resid2, int64_t P, int c, int32_t* label, float* sse, void* stream);
int launch_label_hist(const int32_t* label, int64_t P, const int64_t* offset, int n_groups, int C, float* hist,
                      void* stream);
int launch_chi2_nearest(const float* train, int n_train, const float* test, int n_test, int C, int32_t* nearest,
                        float* dist, void* stream);

// Sum of n floats in FP64 into out[0]; out holds kSumSlots doubles (the rest is scratch).
constexpr int kSumBlocks = 256;
constexpr int kSumSlots = kSumBlocks + 1;
int launch_sum(const float* x, int64_t n, double* out, void* stream);
bool encode_lp_supported(int S, int T, int M, int R);
size_t encode_lp_lds_bytes(const DeviceTables& t);
double encode_lp_mfma_flops_per_patch(const DeviceTables& t, int K);
int launch_encode_lp(const DeviceTables& t, int prec, const float* xhat, int64_t P, int K, int32_t* atom,
                     int32_t* angle, float* coef, float* resid2, void* stream);
size_t images_workspace_bytes(int n_images);
// rsc_project_images_noalloc: the plan in a static device array of this many images.
constexpr int kNoAllocMaxImages = 65535;
int launch_project_images_noalloc(const DeviceTables& t, const float* pixels, const int64_t* img_offset,
                                  const int32_t* H, const int32_t* W, int n, int64_t P_total, float* xhat,
                                  void* stream);
int launch_project_images(const DeviceTables& t, const float* pixels, const int64_t* img_offset,
                          const int32_t* H, const int32_t* W, int n, int64_t P_total, void* ws, float* xhat,
                          void* stream);
int launch_stamps(const DeviceTables& t, const int32_t* atom, const float* theta, const float* amplitude,
                  const int32_t* centre, const int32_t* image, int64_t n_stamps, const int64_t* img_offset,
                  const int32_t* H, const int32_t* W, int n_images, float* pixels, void* stream);

}  // namespace rsc
