// Launch helpers shared by the persistent encoders.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

namespace rsc {

// Compute units of the current device, queried once per device (atomic slots, so threads
// that race for the first query store the same value).
inline int num_cus() {
  static std::atomic<int> cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int n = cached[dev].load(std::memory_order_relaxed);
  if (n <= 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev].store(n, std::memory_order_relaxed);
  }
  return n;
}

// Persistent grid of blocks of `threads` threads (256 or 512: 4 or 8 waves): at most as
// many blocks as fit on the device at once (bpc > 0 caps the blocks per CU, counted in
// units of 4 waves); each wave then walks the patch tiles with a stride of the whole grid.
template <class Kern, class... Args>
int launch_persistent_n(Kern kern, int threads, size_t lds, int64_t wave_tiles, int bpc, hipStream_t st,
                        Args... args) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return int(e);
  }
  const int waves = threads / 64;
  int64_t blocks = (wave_tiles + waves - 1) / waves;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (bpc > 0) {
    int cap_cu = bpc * 4 / waves;
    if (cap_cu < 1) cap_cu = 1;
    if (cap_cu < per_cu) per_cu = cap_cu;
  }
  const int64_t cap = int64_t(num_cus()) * per_cu;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(unsigned(threads)), lds, st, args...);
  return int(hipGetLastError());
}

template <class Kern, class... Args>
int launch_persistent(Kern kern, size_t lds, int64_t wave_tiles, int bpc, hipStream_t st, Args... args) {
  return launch_persistent_n(kern, 256, lds, wave_tiles, bpc, st, args...);
}

}  // namespace rsc
