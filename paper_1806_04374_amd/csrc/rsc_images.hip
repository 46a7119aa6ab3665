// Ragged image batches: every stride-1 N x N window of every image is a patch.
//
//  * images_plan_kernel: per-image patch and wave-tile prefix sums, computed on the
//    device from device arrays of image sizes, so a batch needs no host round trip
//    and can be captured in a HIP graph.
//  * project_images_kernel: persistent im2col projection (Sec. II-E step 2).  A wave
//    owns 32 consecutive window origins of one image row; lanes read the disk pixels
//    of their windows straight from the image (consecutive lanes = consecutive
//    columns), the (Phi^T Phi)^{-1} Phi^T operand stays in LDS for the whole launch.
//  * stamp_kernel: adds amplitude * Phi S_theta d_m stamps into images (synthetic
//    inputs), one block per stamp.
#include <hip/hip_runtime.h>

#include "rsc_device.h"
#include "rsc_internal.h"

namespace rsc {
namespace {

constexpr int kPlanThreads = 1024;
constexpr int kImgWaves = 8;

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

// pinvD: [RTB][KPD][64] operand over disk pixels; dpix: [2*KPD] (dy << 8 | dx) or -1.
template <int N, int KPD, int RTB>
__global__ __launch_bounds__(64 * kImgWaves) void project_images_kernel(
    const float* __restrict__ pixels, const int64_t* __restrict__ img_offset, const int32_t* __restrict__ H,
    const int32_t* __restrict__ W, int n, const int64_t* __restrict__ ws, int64_t P_total, int B,
    const float* __restrict__ pinvD, const int* __restrict__ dpix, float* __restrict__ xhat) {
  extern __shared__ float lds[];
  float* sA = lds;                                            // [RTB][KPD][64]
  int* sPix = reinterpret_cast<int*>(sA + RTB * KPD * 64);    // [2*KPD]
  for (int i = threadIdx.x; i < RTB * KPD * 64; i += blockDim.x) sA[i] = pinvD[i];
  for (int i = threadIdx.x; i < 2 * KPD; i += blockDim.x) sPix[i] = dpix[i];
  __syncthreads();
  const int64_t* patch_start = ws;
  const int64_t* tile_start = ws + n + 1;
  const int64_t ntiles = tile_start[n];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, u = lane >> 5;
  for (int64_t wt = int64_t(blockIdx.x) * kImgWaves + wave; wt < ntiles; wt += int64_t(gridDim.x) * kImgWaves) {
    // keeps the operand reads from LDS inside the loop (hoisting them all out of it
    // would need hundreds of registers)
    asm volatile("" ::: "memory");
    int lo = 0, hi = n - 1;                  // last image with tile_start <= wt
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tile_start[mid] <= wt) lo = mid;
      else hi = mid - 1;
    }
    const int img = lo;
    const int w = W[img];
    const int wp = w - N + 1;
    const int tpr = (wp + 31) >> 5;
    const int local = int(wt - tile_start[img]);      // < H * tpr, fits in 32 bits
    const int y = local / tpr;
    const int x = (local - y * tpr) * 32 + col;
    const bool valid = x < wp;
    const float* base = pixels + img_offset[img] + int64_t(y) * w + (valid ? x : 0);
    f32x16 acc[RTB];
#pragma unroll
    for (int t = 0; t < RTB; ++t)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;
#pragma unroll 8
    for (int j = 0; j < KPD; ++j) {
      const int q = sPix[2 * j + u];
      const float b = (valid && q >= 0) ? base[(q >> 8) * w + (q & 255)] : 0.f;
#pragma unroll
      for (int t = 0; t < RTB; ++t) acc[t] = mfma32(sA[(t * KPD + j) * 64 + lane], b, acc[t]);
    }
    const int64_t pidx = patch_start[img] + int64_t(y) * wp + x;
    if (valid && pidx < P_total) {
      float* dst = xhat + pidx * B;
#pragma unroll
      for (int t = 0; t < RTB; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int c = 32 * t + 8 * (v / 4) + 4 * u + (v % 4);
          if (c < B) dst[c] = acc[t][v];
        }
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

size_t project_images_lds_bytes(const DeviceTables& t) {
  const int kpd = (t.n_pix + 1) / 2;
  const int rtb = (t.B + 31) / 32 <= 2 ? 2 : 4;
  return sizeof(float) * (size_t(rtb) * kpd * 64 + 2 * size_t(kpd));
}

int launch_project_images(const DeviceTables& t, const float* pixels, const int64_t* img_offset,
                          const int32_t* H, const int32_t* W, int n, int64_t P_total, void* ws, float* xhat,
                          void* stream) {
  if (n <= 0 || P_total <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(images_plan_kernel, dim3(1), dim3(kPlanThreads), 0, st, H, W, n, t.N,
                     reinterpret_cast<int64_t*>(ws));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return int(e);
  const size_t lds = project_images_lds_bytes(t);
  static int cus = -1;
  if (cus < 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  auto go = [&](auto kern) -> int {
    static bool attr = false;
    if (!attr) {
      hipError_t e2 = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      if (e2 != hipSuccess) return int(e2);
      attr = true;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * kImgWaves, lds) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    const int64_t max_tiles = (P_total + 31) / 32 + int64_t(n);   // upper bound on wave tiles
    int64_t blocks = (max_tiles + kImgWaves - 1) / kImgWaves;
    if (blocks > int64_t(cus) * per_cu) blocks = int64_t(cus) * per_cu;
    hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(64 * kImgWaves), lds, st, pixels, img_offset, H, W,
                       n, reinterpret_cast<const int64_t*>(ws), P_total, t.B, t.pinvI, t.dpixI, xhat);
    return int(hipGetLastError());
  };
  if (t.N == 11 && t.n_pix == 97) return go(project_images_kernel<11, 49, 2>);
  if (t.N == 15 && t.n_pix == 177) return go(project_images_kernel<15, 89, 4>);
  return int(hipErrorInvalidValue);
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
