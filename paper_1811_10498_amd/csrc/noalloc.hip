// pfac_match on a scratch area of fixed size that the library never
// allocates: a file-scope device array, one copy per GPU, whose device
// address is looked up once per device.  Same kernels, same outputs as
// pfac_match; for callers that cannot allocate device memory.
#include <map>
#include <mutex>

#include "pfac_host.h"

namespace pfac {

constexpr uint64_t kNoallocScratchBytes = 64ull << 20;

// Host code must not pass `scratch` itself to a kernel (its host-side name is
// not a device address): it uses the address from hipGetSymbolAddress.
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

static std::mutex g_noalloc_mu;
static std::map<int, uint8_t*> g_noalloc_ptr;

// Device address of this device's copy of `scratch` (dev is current).
static int noalloc_scratch_ptr(int dev, uint8_t** out) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc_ptr.find(dev);
  if (it != g_noalloc_ptr.end()) {
    *out = it->second;
    return PFAC_OK;
  }
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
    return PFAC_E_HIP;
  g_noalloc_ptr[dev] = static_cast<uint8_t*>(p);
  *out = static_cast<uint8_t*>(p);
  return PFAC_OK;
}

}  // namespace pfac

using namespace pfac;

extern "C" {

uint64_t pfac_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

int pfac_match_noalloc(const pfac_table* t, const void* d_text, uint64_t n, int enc,
                     int32_t* d_match, pfac_hit* d_hits, uint64_t hit_cap,
                     uint64_t* d_counters, const pfac_plan* plan, void* stream_) {
  if (!t || !d_counters || (n && !d_text) || n >= (1ull << 32)) return PFAC_E_ARG;
  if (enc != PFAC_TEXT_ASCII && enc != PFAC_TEXT_2BIT) return PFAC_E_ARG;
  if (t->alphabet != 4) return PFAC_E_ARG;    // byte tables: pfac_match only
  // the paper's two-array and merged layouts are built on first use
  // (an allocation): only once pfac_match has built them
  if (plan && (plan->variant == PFAC_VARIANT_GLOBAL_TWO_ARRAYS ||
               plan->variant == PFAC_VARIANT_GLOBAL_MERGED) && !t->cells_mem)
    return PFAC_E_ARG;
  if (d_hits == nullptr) hit_cap = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFAC_E_NODEV;
  if (dev != t->device) return PFAC_E_ARG;
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  unsigned long long* counters = reinterpret_cast<unsigned long long*>(d_counters);
  SinglePrep P;
  int rc = prepare_single(t, n, enc, plan, dev, &P);
  if (rc) return rc;
  if (P.tiles == 0) return launch_zero(counters, 2u, stream);
  const ScratchLayout L = scratch_layout(P.tiles, false, P.walks);
  if (L.bytes > kNoallocScratchBytes) return PFAC_E_SCRATCH;
  uint8_t* base = nullptr;
  rc = noalloc_scratch_ptr(dev, &base);
  if (rc) return rc;
  // the look-back words and counters must start at zero; the array keeps
  // whatever the last call left, so clear them (a fill kernel, no memset)
  rc = launch_zero(reinterpret_cast<unsigned long long*>(base + L.o_st),
                   (uint32_t)(L.zero_bytes / 8), stream);
  if (rc) return rc;
  const Scratch sc = carve(base, L, P.tiles, P.walks);
  return enqueue_single(t, P, sc, d_text, d_match, d_hits, hit_cap, counters, dev, stream);
}

}  // extern "C"
