// PFAC over the byte alphabet: every byte value is a symbol, patterns are
// any non-empty byte strings -- the general-purpose setting of the original
// PFAC library (paper Sec. I, II), whose large alphabet makes a dense
// transition table wasteful; the table is hash-compressed instead (the hash
// method of that library's follow-up, Sec. II): the root's 256 edges stay a
// dense row (held in LDS), every other edge lives in one open-addressing
// hash table keyed by (state, byte).  The walk is PFAC's (Sec. IV): from
// every start position, one edge per byte, stop at the first missing edge
// or the text end, report the longest pattern passed.  Outputs as
// pfac_match: the dense int32 array, the position-ordered hit list (through
// the same per-tile counts, slots and finish kernel) and the totals.
#include <string.h>

#include <algorithm>

#include "pfac_host.h"

namespace pfac {

constexpr uint32_t kBytesTile = 2048;     // positions per wave tile: 32 per lane

struct BytesParams {
  const uint8_t* text;
  uint64_t n;
  uint64_t tiles;
  const uint32_t* root;       // [256]
  const uint32_t* slots;      // [2 << bits]: key, value
  uint32_t bits;
  const OutEntry* out;
  int32_t* match;
  uint32_t* tile_hits;
  unsigned long long* tile_occ;
  Slot* hslots;
};

// The edge of (s, b) in the hash table: the child with its final bit, 0 if
// none.
__device__ __forceinline__ uint32_t bytes_edge(const BytesParams& p, uint32_t s, uint32_t b) {
  const uint32_t key = (s << 8) | b;
  const uint32_t mask = (1u << p.bits) - 1u;
  uint32_t h = (uint32_t)(key * 0x9E3779B1u) >> (32 - p.bits);
  for (;;) {
    const u32x2 e = *reinterpret_cast<const u32x2*>(p.slots + 2ull * h);
    if (e.x == key) return e.y;
    if (e.x == kBytesEmptyKey) return 0u;
    h = (h + 1) & mask;
  }
}

// One wave per tile of 2048 positions, lanes on consecutive positions
// (position t0 + 64k + lane at step k: coalesced text reads and output
// writes); hits counted per tile and the first 32 parked in position order.
__global__ __launch_bounds__(1024) void pfac_bytes_kernel(BytesParams p) {
  __shared__ uint32_t root[256];
  for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) root[i] = p.root[i];
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / 64);
  for (uint64_t t = (uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); t < p.tiles;
       t += nwaves) {
    const uint64_t t0 = t * kBytesTile;
    uint32_t hits = 0;
    unsigned long long occ = 0;
    for (uint32_t k = 0; k < kBytesTile / 64; ++k) {
      const uint64_t q0 = t0 + 64ull * k + lane;
      int32_t best = 0;
      if (q0 < p.n) {
        uint32_t e = root[p.text[q0]];
        uint64_t q = q0 + 1;
        while (e) {
          const uint32_t s = e & kStateMask;
          if (e & kFinalBit) {
            const OutEntry o = p.out[s];
            best = o.pid;
            occ += o.mult;
          }
          if (q >= p.n) break;
          e = bytes_edge(p, s, p.text[q]);
          ++q;
        }
        if (p.match) p.match[q0] = best;
      }
      const uint64_t m = __ballot(best != 0);
      if (m) {
        const uint32_t before = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        const uint32_t slot = hits + before;
        if (best && p.hslots && slot < kSlot)
          p.hslots[t * kSlot + slot] = Slot{(uint32_t)q0, best};
        hits += (uint32_t)__popcll(m);
      }
    }
    occ = wave_sum(occ);
    if (lane == 0) {
      p.tile_hits[t] = hits;
      p.tile_occ[t] = occ;
    }
  }
}

// Scan + finish of a one-text call on a byte table.  The finish kernel
// takes the hits of tiles with more than their slots from the dense output,
// so a dense array is always written (the caller's, or `dense_scratch`).
static int enqueue_bytes(const pfac_table* t, const uint8_t* text, uint64_t n, int32_t* d_match,
                         int32_t* dense_scratch, pfac_hit* d_hits, uint64_t hit_cap,
                         unsigned long long* counters, const Scratch& sc, uint64_t tiles,
                         uint32_t grid, hipStream_t stream) {
  BytesParams bp;
  memset(&bp, 0, sizeof(bp));
  bp.text = text;
  bp.n = n;
  bp.tiles = tiles;
  bp.root = t->bdev.root;
  bp.slots = t->bdev.slots;
  bp.bits = t->bdev.hash_bits;
  bp.out = t->bdev.out;
  bp.match = d_match ? d_match : dense_scratch;
  bp.tile_hits = sc.tile_hits;
  bp.tile_occ = sc.tile_occ;
  bp.hslots = d_hits ? sc.slots : nullptr;
  hipLaunchKernelGGL(pfac_bytes_kernel, dim3(grid), dim3(1024), 0, stream, bp);
  if (hipGetLastError() != hipSuccess) return PFAC_E_HIP;
  return launch_finish_single(sc, tiles, kBytesTile, n, counters, d_hits, hit_cap, bp.match,
                              stream);
}

}  // namespace pfac

using namespace pfac;

extern "C" {

int pfac_build_table_bytes(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                           pfac_table** out, int64_t* bad_index) {
  if (!out) return PFAC_E_ARG;
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFAC_E_NODEV;
  if (!device_ok(dev)) return PFAC_E_NODEV;
  pfac_table* t = new (std::nothrow) pfac_table();
  if (!t) return PFAC_E_NOMEM;
  int rc = build_host_bytes(patterns, lengths, num, &t->bytes, bad_index);
  if (rc != PFAC_OK) {
    delete t;
    return rc;
  }
  t->device = dev;
  t->alphabet = 256;
  const HostBytes& h = t->bytes;
  // the shared info fields
  t->host.num_states = h.num_states;
  t->host.num_patterns = h.num_patterns;
  t->host.max_len = h.max_len;
  t->host.min_len = h.min_len;
  t->host.depth_start = h.depth_start;
  const uint64_t o_root = 0, o_slots = al256(256 * 4);
  const uint64_t o_out = o_slots + al256(h.slots.size() * 4);
  const uint64_t bytes = o_out + al256(h.out.size() * sizeof(OutEntry));
  if (hipMalloc(&t->dmem, bytes) != hipSuccess) {
    delete t;
    return PFAC_E_NOMEM;
  }
  t->dbytes = bytes;
  uint8_t* b = static_cast<uint8_t*>(t->dmem);
  if (hipMemcpy(b + o_root, h.root, 256 * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b + o_slots, h.slots.data(), h.slots.size() * 4, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(b + o_out, h.out.data(), h.out.size() * sizeof(OutEntry),
                hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(t->dmem);
    delete t;
    return PFAC_E_HIP;
  }
  t->bdev.root = reinterpret_cast<const uint32_t*>(b + o_root);
  t->bdev.slots = reinterpret_cast<const uint32_t*>(b + o_slots);
  t->bdev.out = reinterpret_cast<const OutEntry*>(b + o_out);
  t->bdev.hash_bits = h.hash_bits;
  *out = t;
  return PFAC_OK;
}

}  // extern "C"

namespace pfac {

int match_bytes(const pfac_table* t, const void* d_text, uint64_t n, int32_t* d_match,
                pfac_hit* d_hits, uint64_t hit_cap, unsigned long long* counters,
                const pfac_plan* plan, int dev, hipStream_t stream) {
  if (plan && (plan->variant || plan->depth || plan->levels || plan->hash_bits || plan->walks ||
               plan->tile || plan->prefix || (plan->block && plan->block != 1024)))
    return PFAC_E_ARG;     // byte tables have one kernel; only the grid is a choice
  const uint64_t tiles = (n + kBytesTile - 1) / kBytesTile;
  if (tiles == 0) return launch_zero(counters, 2u, stream);
  const bool need_dense = d_match == nullptr && d_hits != nullptr && hit_cap > 0;
  int rc = PFAC_OK;
  Workspace* ws = workspace_for(dev, stream, tiles, 0, need_dense ? n * 4 : 0, &rc);
  if (!ws) return rc;
  const uint32_t cus = device_cus(dev);
  uint64_t grid = plan && plan->grid ? plan->grid : (uint64_t)cus * 2;
  grid = std::min<uint64_t>(std::max<uint64_t>(1, std::min<uint64_t>(grid, (tiles + 15) / 16)),
                            2048);
  return enqueue_bytes(t, static_cast<const uint8_t*>(d_text), n, d_match,
                       need_dense ? reinterpret_cast<int32_t*>(workspace_extra(ws)) : nullptr,
                       d_hits, hit_cap, counters, workspace_scratch(ws), tiles, (uint32_t)grid,
                       stream);
}

}  // namespace pfac
