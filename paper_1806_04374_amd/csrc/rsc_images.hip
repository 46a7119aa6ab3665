// Ragged image batches: every stride-1 N x N window of every image is a patch.
//
//  * images_plan_kernel: per-image patch and wave-tile prefix sums, computed on the
//    device from device arrays of image sizes, so a batch needs no host round trip
//    and can be captured in a HIP graph.
//  * project_images_reg_kernel: persistent im2col projection (Sec. II-E step 2).  A
//    block takes tiles of 32 consecutive window origins of one image row; the tile's
//    pixel region is staged in LDS, each wave keeps one 32-row tile of the
//    (Phi^T Phi)^{-1} Phi^T operand in registers, and the results leave as contiguous
//    runs of x_hat rows.
//  * stamp_kernel: adds amplitude * Phi S_theta d_m stamps into images (synthetic
//    inputs), one block per stamp.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rsc_device.h"
#include "rsc_internal.h"
#include "rsc_launch.h"

namespace rsc {
namespace {

constexpr int kPlanThreads = 1024;

// ws: int64 patch_start[n+1], tile_start[n+1] (exclusive prefix sums).
__global__ __launch_bounds__(kPlanThreads) void images_plan_kernel(const int32_t* __restrict__ H,
                                                                  const int32_t* __restrict__ W, int n,
                                                                  int N, int64_t* __restrict__ ws) {
  __shared__ int64_t sp[kPlanThreads], st[kPlanThreads];
  int64_t* patch_start = ws;
  int64_t* tile_start = ws + n + 1;
  int64_t run_p = 0, run_t = 0;
  for (int base = 0; base < n; base += kPlanThreads) {
    const int i = base + threadIdx.x;
    int64_t cp = 0, ct = 0;
    if (i < n) {
      const int64_t hp = H[i] - N + 1, wp = W[i] - N + 1;
      if (hp > 0 && wp > 0) {
        cp = hp * wp;
        ct = hp * ((wp + 31) / 32);
      }
    }
    sp[threadIdx.x] = cp;
    st[threadIdx.x] = ct;
    __syncthreads();
    for (int off = 1; off < kPlanThreads; off *= 2) {  // inclusive Hillis-Steele scan
      const int64_t ap = threadIdx.x >= off ? sp[threadIdx.x - off] : 0;
      const int64_t at = threadIdx.x >= off ? st[threadIdx.x - off] : 0;
      __syncthreads();
      sp[threadIdx.x] += ap;
      st[threadIdx.x] += at;
      __syncthreads();
    }
    if (i < n) {
      patch_start[i] = run_p + sp[threadIdx.x] - cp;
      tile_start[i] = run_t + st[threadIdx.x] - ct;
    }
    run_p += sp[kPlanThreads - 1];
    run_t += st[kPlanThreads - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    patch_start[n] = run_p;
    tile_start[n] = run_t;
  }
}

// Wave tile wt -> (image, window row y, first window column x0) through the plan.
struct ImgTile {
  int img, w, wp, y, x0;
};

// from: an image index whose tile_start <= wt (the previous tile's), or -1 for a binary
// search; tiles only move forward, so the walk from the previous image is usually short.
template <int N>
__device__ __forceinline__ ImgTile img_tile(const int64_t* __restrict__ tile_start, const int32_t* __restrict__ W,
                                            int n, int64_t wt, int from) {
  int lo = 0;                              // last image with tile_start <= wt
  if (from < 0) {
    int hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tile_start[mid] <= wt) lo = mid;
      else hi = mid - 1;
    }
  } else {
    lo = from;
    while (lo + 1 < n && tile_start[lo + 1] <= wt) ++lo;
  }
  ImgTile r;
  r.img = lo;
  r.w = W[lo];
  r.wp = r.w - N + 1;
  const int tpr = (r.wp + 31) >> 5;
  const int local = int(wt - tile_start[lo]);   // < H * tpr, fits in 32 bits
  r.y = local / tpr;
  r.x0 = (local - r.y * tpr) * 32;
  return r;
}

// The same projection with the operand in registers: a block of NT waves takes TPB tiles of
// 32 windows at a time (wave w computes hat coordinates 32w..32w+31 from its KPD operand
// steps in registers, one accumulator per tile, so the tiles' MFMA chains interleave).  Each
// tile's pixels, an N x (32 + N - 1) region of one image (zero past its right edge), are
// staged in LDS, the next tiles' regions are loaded into registers while the current ones
// are contracted, and the 32 x B results of a tile leave through an LDS staging tile as one
// contiguous run of x_hat rows (consecutive windows are consecutive rows).
template <int N, int KPD, int NT, int TPB>
__global__ __launch_bounds__(64 * NT) void project_images_reg_kernel(
    const float* __restrict__ pixels, const int64_t* __restrict__ img_offset, const int32_t* __restrict__ H,
    const int32_t* __restrict__ W, int n, const int64_t* __restrict__ ws, int64_t P_total, int B,
    const float* __restrict__ pinvI, const int* __restrict__ dpix, float* __restrict__ xhat) {
  constexpr int NTH = 64 * NT, RW = 32 + N - 1, RSZ = N * RW, RPT = (RSZ + NTH - 1) / NTH;
  __shared__ float region[TPB][RSZ];
  __shared__ int sPix[2 * KPD];
  __shared__ float stage[TPB][32 * 32 * NT];     // [32 windows][B] per tile, B <= 32 NT
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, col = lane & 31, u = lane >> 5;
  float a[KPD];
#pragma unroll
  for (int j = 0; j < KPD; ++j) a[j] = pinvI[(w * KPD + j) * 64 + lane];
  // slots past the disk have zero operand rows: point them at disk pixel 0
  for (int i = t; i < 2 * KPD; i += NTH) sPix[i] = dpix[i] >= 0 ? dpix[i] : dpix[0];
  const int64_t* patch_start = ws;
  const int64_t* tile_start = ws + n + 1;
  const int64_t ntiles = tile_start[n];
  // region element e of a tile: row e / RW, column e % RW (fixed per thread)
  int er[RPT], ec[RPT];
#pragma unroll
  for (int v = 0; v < RPT; ++v) {
    const int e = t + NTH * v;
    er[v] = e < RSZ ? e / RW : 0;
    ec[v] = e < RSZ ? e - (e / RW) * RW : 0;
  }
  float nxt[TPB][RPT];
  ImgTile cur[TPB];
  bool has[TPB];
  // Blocks go to the XCDs round-robin (block b to XCD b % 8), each XCD with its own L2.  The
  // tiles are cut into one contiguous range per such group of blocks, which its blocks stride
  // over, so the window rows that share 14 of their 15 pixel rows are taken on one XCD in
  // consecutive rounds and their pixels come from its L2.  (Only where the tiles run; every
  // tile is taken once whatever the placement.)
  constexpr int kXcd = 8;
  const int grp = int(blockIdx.x) % kXcd, slot = int(blockIdx.x) / kXcd;
  const int ngrp = gridDim.x < kXcd ? int(gridDim.x) : kXcd;
  const int nblk = (int(gridDim.x) - grp + kXcd - 1) / kXcd;   // blocks in this group
  const int64_t hi = ntiles * (grp + 1) / ngrp;
  const int64_t stride = int64_t(nblk) * TPB;
  // decode tiles wt0 .. wt0 + TPB - 1 (those below hi) and load their regions
  auto fetch = [&](int64_t wt0, bool first) {
#pragma unroll
    for (int k = 0; k < TPB; ++k) {
      has[k] = wt0 + k < hi;
      if (has[k]) {
        cur[k] = img_tile<N>(tile_start, W, n, wt0 + k, first ? -1 : cur[k].img);
        const float* img = pixels + img_offset[cur[k].img] + int64_t(cur[k].y) * cur[k].w + cur[k].x0;
#pragma unroll
        for (int v = 0; v < RPT; ++v)
          nxt[k][v] = (t + NTH * v < RSZ && cur[k].x0 + ec[v] < cur[k].w) ? img[er[v] * cur[k].w + ec[v]] : 0.f;
      }
    }
  };
  int64_t wt0 = ntiles * grp / ngrp + int64_t(slot) * TPB;
  if (wt0 < hi) fetch(wt0, true);
  for (; wt0 < hi; wt0 += stride) {
    __syncthreads();   // the previous tiles' region and staging reads are done
#pragma unroll
    for (int k = 0; k < TPB; ++k)
#pragma unroll
      for (int v = 0; v < RPT; ++v)
        if (t + NTH * v < RSZ) region[k][t + NTH * v] = has[k] ? nxt[k][v] : 0.f;
    __syncthreads();
    ImgTile now[TPB];
    bool nhas[TPB];
#pragma unroll
    for (int k = 0; k < TPB; ++k) {
      now[k] = cur[k];
      nhas[k] = has[k];
    }
    if (wt0 + stride < hi) fetch(wt0 + stride, false);
    f32x16 acc[TPB];
#pragma unroll
    for (int k = 0; k < TPB; ++k)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[k][i] = 0.f;
#pragma unroll
    for (int j = 0; j < KPD; ++j) {
      const int q = sPix[2 * j + u];
      const int off = (q >> 8) * RW + (q & 255) + col;
#pragma unroll
      for (int k = 0; k < TPB; ++k) acc[k] = mfma32(a[j], region[k][off], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < TPB; ++k)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = 32 * w + 8 * (v / 4) + 4 * u + (v % 4);
        if (r < B) stage[k][col * B + r] = acc[k][v];
      }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TPB; ++k) {
      if (!nhas[k]) continue;
      const int nv = now[k].wp - now[k].x0 < 32 ? now[k].wp - now[k].x0 : 32;   // valid windows
      const int64_t p0 = patch_start[now[k].img] + int64_t(now[k].y) * now[k].wp + now[k].x0;
      const int64_t np = p0 + nv <= P_total ? nv : (P_total > p0 ? P_total - p0 : 0);
      float* dst = xhat + p0 * B;
      for (int i = t; i < int(np) * B; i += NTH) dst[i] = stage[k][i];
    }
  }
}

struct StampParams {
  const int32_t* atom;
  const float* theta;
  const float* amplitude;
  const int32_t* centre;   // [n][2] (row, col)
  const int32_t* image;
  const int64_t* img_offset;
  const int32_t* H;
  const int32_t* W;
  int n_images;
  int64_t n_stamps;
  int M, S, T, B, N;
  const float* dictHat;
  const float* phiPad;
  float* pixels;
};

__global__ __launch_bounds__(256) void stamp_kernel(StampParams p) {
  extern __shared__ float hat[];  // [B]
  const int64_t s = blockIdx.x;
  const int m = p.atom[s];
  const int im = p.image[s];
  if (m < 0 || m >= p.M || im < 0 || im >= p.n_images) return;
  const float amp = p.amplitude[s], th = p.theta[s];
  const float* d = p.dictHat + int64_t(m) * p.B;
  const int S = p.S;
  for (int c = threadIdx.x; c < p.B; c += blockDim.x) {
    float v;
    if (c < S) {
      v = d[c];
    } else {
      const int q = c - S, k = 1 + q / (2 * S), rem = q % (2 * S), sp = rem % S;
      const int base = S + 2 * S * (k - 1);
      float sn, co;
      sincosf(float(k) * th, &sn, &co);
      const float re = d[base + sp], im_ = d[base + S + sp];
      v = rem >= S ? (im_ * co - re * sn) : (re * co + im_ * sn);
    }
    hat[c] = amp * v;
  }
  __syncthreads();
  const int N = p.N, c0 = (N - 1) / 2;
  const int h = p.H[im], w = p.W[im];
  const int r0 = p.centre[2 * s] - c0, q0 = p.centre[2 * s + 1] - c0;
  for (int q = threadIdx.x; q < N * N; q += blockDim.x) {
    const int row = r0 + q / N, col = q0 + q % N;
    if (row < 0 || row >= h || col < 0 || col >= w) continue;
    const float* ph = p.phiPad + int64_t(q) * p.B;
    float acc = 0.f;
    for (int b = 0; b < p.B; ++b) acc += ph[b] * hat[b];
    if (acc != 0.f) atomicAdd(p.pixels + p.img_offset[im] + int64_t(row) * w + col, acc);
  }
}

}  // namespace

size_t images_workspace_bytes(int n_images) { return sizeof(int64_t) * 2 * (size_t(n_images) + 1); }

int launch_project_images(const DeviceTables& t, const float* pixels, const int64_t* img_offset,
                          const int32_t* H, const int32_t* W, int n, int64_t P_total, void* ws, float* xhat,
                          void* stream) {
  if (n <= 0 || P_total <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(images_plan_kernel, dim3(1), dim3(kPlanThreads), 0, st, H, W, n, t.N,
                     reinterpret_cast<int64_t*>(ws));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return int(e);
  const int cus = num_cus();
  // two 32-window tiles per block step, grid of one resident round
  auto go_reg = [&](auto kern, int nt) -> int {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * nt, 0) != hipSuccess || per_cu < 1)
      per_cu = 1;
    const int64_t max_tiles = (P_total + 31) / 32 + int64_t(n);   // upper bound on tiles
    int64_t blocks = (max_tiles + 1) / 2;                          // two tiles per block step
    if (blocks > int64_t(cus) * per_cu) blocks = int64_t(cus) * per_cu;
    hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(64 * nt), 0, st, pixels, img_offset, H, W, n,
                       reinterpret_cast<const int64_t*>(ws), P_total, t.B, t.pinvI, t.dpixI, xhat);
    return int(hipGetLastError());
  };
  // one wave per 32 coordinates: the 11x11 grid (B = 55) and annular (B = 81) bases, the
  // 15x15 grid (B = 105) and annular (B = 153) bases
  if (t.N == 11 && t.n_pix == 97 && t.B <= 64) return go_reg(project_images_reg_kernel<11, 49, 2, 2>, 2);
  if (t.N == 11 && t.n_pix == 97 && t.B <= 96) return go_reg(project_images_reg_kernel<11, 49, 3, 2>, 3);
  if (t.N == 15 && t.n_pix == 177 && t.B > 64 && t.B <= 128)
    return go_reg(project_images_reg_kernel<15, 89, 4, 2>, 4);
  if (t.N == 15 && t.n_pix == 177 && t.B > 128 && t.B <= 160)
    return go_reg(project_images_reg_kernel<15, 89, 5, 2>, 5);
  return int(hipErrorInvalidValue);
}

// Plan of rsc_project_images_noalloc: the two prefix-sum arrays of images_plan_kernel for
// up to kNoAllocMaxImages images (1 MiB), held by every device the library runs on until
// the process ends.  Every call on a device shares its copy: the plan kernel writes every
// entry the projection reads, so nothing needs clearing, and calls that overlap on one
// device race.  In host code `scratch` is only a stand-in for the symbol: its device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) int64_t scratch[2 * (kNoAllocMaxImages + 1)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int64_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (looked up on the first call per device).
int scratch_address(int64_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return int(e);
  if (dev < 0 || dev >= kMaxDevices) return int(hipErrorInvalidDevice);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return int(e);
    if (!p) return int(hipErrorInvalidSymbol);
    g_scratch_ptr[dev] = static_cast<int64_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return 0;
}
}  // namespace

int launch_project_images_noalloc(const DeviceTables& t, const float* pixels, const int64_t* img_offset,
                                  const int32_t* H, const int32_t* W, int n, int64_t P_total, float* xhat,
                                  void* stream) {
  if (n > kNoAllocMaxImages) return int(hipErrorInvalidValue);
  if (n <= 0 || P_total <= 0) return 0;
  int64_t* ws = nullptr;
  const int e = scratch_address(&ws);
  if (e) return e;
  return launch_project_images(t, pixels, img_offset, H, W, n, P_total, ws, xhat, stream);
}

int launch_stamps(const DeviceTables& t, const int32_t* atom, const float* theta, const float* amplitude,
                  const int32_t* centre, const int32_t* image, int64_t n_stamps, const int64_t* img_offset,
                  const int32_t* H, const int32_t* W, int n_images, float* pixels, void* stream) {
  if (n_stamps <= 0) return 0;
  StampParams p{atom, theta, amplitude, centre, image, img_offset, H, W, n_images, n_stamps,
                t.M, t.S, t.T, t.B, t.N, t.dictHat, t.phiPad, pixels};
  hipLaunchKernelGGL(stamp_kernel, dim3(unsigned(n_stamps)), dim3(256), sizeof(float) * t.B,
                     reinterpret_cast<hipStream_t>(stream), p);
  return int(hipGetLastError());
}

}  // namespace rsc
