// Launch helpers shared by the persistent encoders.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rsc {

inline int num_cus() {
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

// Persistent grid of 256-thread blocks (4 waves): at most as many blocks as fit on
// the device at once (bpc > 0 caps the blocks per CU); each wave then walks the
// patch tiles with a stride of the whole grid.
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

}  // namespace rsc
