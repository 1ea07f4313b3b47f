// Instantiations of the scan kernel for one workgroup size (PFAC_BLOCK) and
// one launch kind (PFAC_SINGLE: 1 = one text, 0 = batch).  The build
// compiles this file once per combination, in parallel.
#include "scan_device.h"

#if !defined(PFAC_BLOCK) || !defined(PFAC_SINGLE)
#error "compile with -DPFAC_BLOCK=<256|512|768|1024> -DPFAC_SINGLE=<0|1>"
#endif

#define PFAC_CAT2(a, b) a##b
#define PFAC_CAT(a, b) PFAC_CAT2(a, b)
#if PFAC_SINGLE
#define PFAC_PICK PFAC_CAT(pick_scan_single_, PFAC_BLOCK)
#else
#define PFAC_PICK PFAC_CAT(pick_scan_batch_, PFAC_BLOCK)
#endif

namespace pfac {

template <bool DEFER, uint32_t TILE, bool PZ = false>
static ScanFn by_depth(uint32_t D) {
  constexpr bool S = PFAC_SINGLE != 0;
  switch (D) {
    case 6: return pfac_scan_kernel<PFAC_BLOCK, false, 6, S, DEFER, TILE, PZ>;
    case 7: return pfac_scan_kernel<PFAC_BLOCK, false, 7, S, DEFER, TILE, PZ>;
    case 8: return pfac_scan_kernel<PFAC_BLOCK, false, 8, S, DEFER, TILE, PZ>;
    case 9: return pfac_scan_kernel<PFAC_BLOCK, false, 9, S, DEFER, TILE, PZ>;
    case 10: return pfac_scan_kernel<PFAC_BLOCK, false, 10, S, DEFER, TILE, PZ>;
    default: return nullptr;
  }
}

template <uint32_t TILE>
static ScanFn by_walks(uint32_t D, bool defer) {
  return defer ? by_depth<true, TILE>(D) : by_depth<false, TILE>(D);
}

ScanFn PFAC_PICK(bool global, uint32_t D, bool defer, uint32_t tile, bool pz) {
#if PFAC_SINGLE
  // pre-zeroing variants: deferred walks, 2048-position tiles
  if (pz) return (!global && defer && tile == 2048) ? by_depth<true, 2048, true>(D) : nullptr;
  // global-memory variants: D names the transition table layout
  if (global) {
    if (tile != kTileSingle) return nullptr;
    switch (D) {
      case 0: return pfac_scan_kernel<PFAC_BLOCK, true, 0, true, false, kTileSingle, false>;
      case 1: return pfac_scan_kernel<PFAC_BLOCK, true, 1, true, false, kTileSingle, false>;
      case 2: return pfac_scan_kernel<PFAC_BLOCK, true, 2, true, false, kTileSingle, false>;
      default: return nullptr;
    }
  }
  switch (tile) {
    case 2048: return by_walks<2048>(D, defer);
    case 1024: return by_walks<1024>(D, defer);
    default: return nullptr;
  }
#else
  // pre-zeroing variants: deferred walks, 2048-position tiles
  if (pz) return (!global && defer && tile == 2048) ? by_depth<true, 2048, true>(D) : nullptr;
  if (global) return (tile == kTileBatch && D == 0)
                        ? pfac_scan_kernel<PFAC_BLOCK, true, 0, false, false, kTileBatch, false>
                        : nullptr;
  switch (tile) {
    case 2048: return by_walks<2048>(D, defer);
    case 1024: return by_walks<1024>(D, defer);
    case 256: return by_walks<256>(D, defer);
    default: return nullptr;
  }
#endif
}

}  // namespace pfac
