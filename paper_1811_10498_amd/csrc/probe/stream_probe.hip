// Bandwidth reference kernels for the roofline of the scan (measurement
// only; not part of the matching library).  They move exactly the scan's
// algorithmic traffic in the scan's access shape, with nothing else:
// persistent 1024-thread workgroups, one wave per tile, tiles handed out
// grid-stride; per tile a wave reads `tile` text bytes with 16-byte
// non-temporal loads and writes 4*`tile` bytes of int32 output with 16-byte
// non-temporal stores (mode 0), only reads (mode 1) or only writes (mode 2).
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// flags: bit 0 = plain (write-back) stores instead of non-temporal ones,
// bit 1 = plain loads instead of non-temporal ones.
template <uint32_t TILE>
__global__ __launch_bounds__(1024) void stream_probe_kernel(const uint8_t* src, int32_t* dst,
                                                            uint64_t tiles, uint32_t mode,
                                                            uint32_t flags, uint32_t* sink) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = (uint64_t)blockIdx.x * 16 + (threadIdx.x >> 6);
  const uint64_t nwaves = (uint64_t)gridDim.x * 16;
  uint32_t acc = 0;
  for (uint64_t t = wave; t < tiles; t += nwaves) {
    if (mode != 2) {
      #pragma unroll
      for (uint32_t k = 0; k < TILE / 1024; ++k) {
        const u32x4* a = reinterpret_cast<const u32x4*>(src + t * TILE + k * 1024) + lane;
        const u32x4 v = (flags & 2u) ? *a : __builtin_nontemporal_load(a);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
      }
    }
    if (mode != 1) {
      const i32x4 z = {(int32_t)(acc & 1u), 0, 0, 0};
      #pragma unroll
      for (uint32_t k = 0; k < TILE / 256; ++k) {
        i32x4* d = reinterpret_cast<i32x4*>(dst + t * TILE + k * 256) + lane;
        if (flags & 1u) *d = z; else __builtin_nontemporal_store(z, d);
      }
    }
  }
  if (acc == 0x9E3779B1u) sink[0] = acc;   // keeps the loads; practically never taken
}

// Mode 0 with the next tile's loads issued before this tile's stores: the
// wait for those loads then leaves the stores in flight (vmcnt(8)) instead
// of draining them (the vector-memory counter of gfx950 retires loads and
// stores in issue order).  Tiles are handed out as in the scan: wave w of
// workgroup b starts at tile w*G + b (G workgroups), so neighbouring tiles
// belong to neighbouring workgroups.
__global__ __launch_bounds__(1024) void stream_probe_pipelined(const uint8_t* src, int32_t* dst,
                                                               uint64_t tiles, uint32_t* sink) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = (uint64_t)(threadIdx.x >> 6) * gridDim.x + blockIdx.x;
  const uint64_t nwaves = (uint64_t)gridDim.x * 16;
  if (wave >= tiles) return;
  uint32_t acc = 0;
  u32x4 a0 = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src + wave * 2048) + lane);
  u32x4 a1 =
      __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src + wave * 2048 + 1024) + lane);
  for (uint64_t t = wave; t < tiles; t += nwaves) {
    acc ^= a0.x ^ a0.y ^ a0.z ^ a0.w ^ a1.x ^ a1.y ^ a1.z ^ a1.w;
    // the next tile (the last one again at the end: always issued, so every
    // path has the same two loads before the eight stores)
    const uint64_t tn = t + nwaves < tiles ? t + nwaves : t;
    a0 = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src + tn * 2048) + lane);
    a1 = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src + tn * 2048 + 1024) + lane);
    const i32x4 z = {(int32_t)(acc & 1u), 0, 0, 0};
    #pragma unroll
    for (uint32_t k = 0; k < 8; ++k)
      __builtin_nontemporal_store(z, reinterpret_cast<i32x4*>(dst + t * 2048 + k * 256) + lane);
  }
  acc ^= a0.x ^ a1.x;
  if (acc == 0x9E3779B1u) sink[0] = acc;
}

extern "C" {

// Run the probe over `tiles` tiles of 2048 positions on `stream`: src holds
// tiles*2048 bytes, dst tiles*2048 int32.  grid = 0: one workgroup per CU.
// flags as the kernel's; mode 3 = mode 0 pipelined (stream_probe_pipelined).
int pfac_probe_stream(const void* src, int32_t* dst, uint64_t tiles, uint32_t mode,
                      uint32_t flags, uint32_t grid, uint32_t* sink, void* stream) {
  if (mode > 3 || (mode != 2 && !src) || (mode != 1 && !dst) || !sink) return -1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -5;
  const uint32_t g = grid ? grid : (uint32_t)cus;
  if (mode == 3)
    hipLaunchKernelGGL(stream_probe_pipelined, dim3(g), dim3(1024), 0,
                       static_cast<hipStream_t>(stream), static_cast<const uint8_t*>(src), dst,
                       tiles, sink);
  else
    hipLaunchKernelGGL(stream_probe_kernel<2048>, dim3(g), dim3(1024), 0,
                       static_cast<hipStream_t>(stream), static_cast<const uint8_t*>(src), dst,
                       tiles, mode, flags, sink);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"
