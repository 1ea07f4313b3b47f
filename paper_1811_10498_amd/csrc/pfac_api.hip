
// Host side of libpfac.so: the finish kernels, plans, scratch, batch layout
// and the C entry points of include/pfac.h.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "pfac_host.h"

namespace pfac {

// Parameters of the finish kernel.
struct FinishParams {
  const uint32_t* tile_hits;
  const unsigned long long* tile_occ;
  Slot* slots;
  uint64_t tiles;
  uint32_t tile;                  // one text: start positions per tile
  void* hits;                     // pfac_hit* (single) or pfac_batch_hit* (batch); null: none
  uint64_t hit_cap;
  uint32_t single;
  // per workgroup: look-back word and occurrence sum; two counters (work
  // ticket, finished look-backs), zero between launches
  unsigned long long* status;
  unsigned long long* block_occ;
  uint32_t* sync;
  unsigned long long* counters;   // [0] hits, [1] occurrences
  // tile -> text (batch), and what an overflowing tile needs to redo its hits
  uint32_t nsegs;
  const DevSeg* segs;
  const uint64_t* tile_prefix;
  DevSeg seg0;
  const uint8_t* text;
  const int32_t* match;           // dense output if it was written, else nullptr
  const DevTable* tables;         // batch: device array indexed by DevSeg::table
  DevTable tab0;
};

__device__ __forceinline__ void put_hit(const FinishParams& p, uint64_t o, uint32_t text,
                                        uint32_t pos, int32_t pid) {
  if (o >= p.hit_cap) return;
  if (p.single) {
    reinterpret_cast<pfac_hit*>(p.hits)[o] = pfac_hit{pos, pid};
  } else {
    reinterpret_cast<pfac_batch_hit*>(p.hits)[o] = pfac_batch_hit{text, pos, pid};
  }
}

__device__ __forceinline__ uint32_t text_of_tile(const FinishParams& p, uint64_t t) {
  uint32_t lo = 0, hi = p.nsegs;   // tile_prefix[lo] <= t < tile_prefix[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (p.tile_prefix[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// Look-back word of a workgroup: bits 62..63 what it holds (0 nothing yet,
// 1 the workgroup's own hit count, 2 the count of it and every workgroup
// before it), bits 0..61 the count.
constexpr unsigned long long kLbAgg = 1ull << 62;
constexpr unsigned long long kLbIncl = 2ull << 62;
constexpr unsigned long long kLbMask = (1ull << 62) - 1;
constexpr uint32_t kLbSpinLimit = 1u << 22;

// Hit list and totals after the scan, one launch.  Workgroups take tickets in
// the order they start and handle kRedTiles tiles in ticket order: the hit
// and occurrence sums of their tiles, then the hits before them by looking
// back over the words of the workgroups with earlier tickets (one lane per
// workgroup, 64 at a time; a workgroup with a ticket has started, so every
// wait ends), then every tile's hits at their position-ordered offsets.  The
// last workgroup to finish its look-back writes the totals and clears the
// words and counters for the next launch.  Tiles with more hits than their
// slots hold take them from the dense output when it was written, otherwise
// walk their positions again from the root.
__global__ __launch_bounds__(1024) void pfac_finish_kernel(FinishParams p) {
  __shared__ uint32_t wsum[16];
  __shared__ unsigned long long wocc[16];
  __shared__ uint32_t ovf_tile[kRedTiles];
  __shared__ unsigned long long ovf_off[kRedTiles];
  __shared__ uint32_t novf, s_vb, s_last;
  __shared__ unsigned long long s_excl;
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) {
    novf = 0;
    s_vb = __hip_atomic_fetch_add(&p.sync[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // workgroups almost always start in index order: load the tiles of this
  // index while the ticket is taken, again if the ticket differs
  uint32_t h[4];
  unsigned long long oc;
  auto load = [&](uint64_t tt) {
    oc = 0;
    if (tt + 4 <= p.tiles) {
      const u32x4 hv = *reinterpret_cast<const u32x4*>(p.tile_hits + tt);
      h[0] = hv.x; h[1] = hv.y; h[2] = hv.z; h[3] = hv.w;
      oc = p.tile_occ[tt] + p.tile_occ[tt + 1] + p.tile_occ[tt + 2] + p.tile_occ[tt + 3];
    } else {
      #pragma unroll
      for (int k = 0; k < 4; ++k) {
        h[k] = tt + k < p.tiles ? p.tile_hits[tt + k] : 0u;
        oc += tt + k < p.tiles ? p.tile_occ[tt + k] : 0ull;
      }
    }
  };
  load((uint64_t)blockIdx.x * kRedTiles + 4 * threadIdx.x);
  __syncthreads();
  const uint32_t vb = s_vb;
  const uint64_t base = (uint64_t)vb * kRedTiles;
  const uint64_t tt = base + 4 * threadIdx.x;   // 4 consecutive tiles per thread
  if (vb != blockIdx.x) load(tt);
  // order each tile's slots by position (hits found by deferred walks were
  // appended after the scan's, in no particular order); needs no offset, so
  // waves 1.. do it while wave 0 looks back, and wave 0 after that (the
  // first slot of each tile is then read ahead of the offsets)
  Slot first[4];
  auto sort_slots = [&]() {
    if (!p.hits || !p.hit_cap) return;
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (h[k] == 0 || h[k] > kSlot) continue;
      Slot* sl = p.slots + (tt + k) * kSlot;
      for (uint32_t i = 1; i < h[k]; ++i) {
        const Slot key = sl[i];
        uint32_t m = i;
        while (m > 0 && sl[m - 1].pos > key.pos) {
          sl[m] = sl[m - 1];
          --m;
        }
        sl[m] = key;
      }
      first[k] = sl[0];
    }
  };
  const uint32_t sum = h[0] + h[1] + h[2] + h[3];
  const uint32_t inc = wave_incl_dpp(sum);
  oc = wave_sum(oc);
  if (lane == 63) wsum[w] = inc;
  if (lane == 0) wocc[w] = oc;
  __syncthreads();
  if (w == 0) {
    unsigned long long agg = lane < 16 ? wsum[lane] : 0u;
    unsigned long long occ = lane < 16 ? wocc[lane] : 0ull;
    agg = wave_sum(agg);
    occ = wave_sum(occ);
    // a look-back word carries its own data: relaxed atomics suffice
    if (lane == 0) {
      __hip_atomic_store(&p.block_occ[vb], occ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&p.status[vb], (vb == 0 ? kLbIncl : kLbAgg) | agg, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    // look back: lane l reads the word of workgroup j - l
    unsigned long long excl = 0;
    int64_t j = (int64_t)vb - 1;
    uint32_t spins = 0;
    while (j >= 0) {
      const int64_t jj = j - (int64_t)lane;
      const unsigned long long v =
          jj >= 0 ? __hip_atomic_load(&p.status[jj], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                  : kLbIncl;
      const uint64_t stop = __ballot((v & ~kLbMask) == kLbIncl);
      const uint32_t first = stop ? (uint32_t)__builtin_ctzll(stop) : 64u;
      const uint64_t upto = first >= 63 ? ~0ull : ((2ull << first) - 1ull);
      if (__ballot((v & ~kLbMask) == 0) & upto) {
        if (++spins >= kLbSpinLimit) {
          // never expected (every awaited workgroup is running): give up
          // rather than hang; this workgroup writes no hits and the hit
          // total reads as all ones
          excl = ~0ull;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        continue;
      }
      excl += wave_sum(lane <= first ? (v & kLbMask) : 0ull);
      if (first < 64) break;
      j -= 64;
    }
    if (lane == 0) {
      if (vb != 0)
        __hip_atomic_store(&p.status[vb], kLbIncl | ((excl + agg) & kLbMask), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      s_excl = excl;
      // release: this workgroup's words before the count of finished
      // look-backs; acquire: the last one then sees every workgroup's words
      const uint32_t prev = __hip_atomic_fetch_add(&p.sync[1], 1u, __ATOMIC_ACQ_REL,
                                                   __HIP_MEMORY_SCOPE_AGENT);
      s_last = prev == gridDim.x - 1;
    }
  }
  sort_slots();
  __syncthreads();
  if (p.hits && p.hit_cap && s_excl != ~0ull) {
    uint64_t off = s_excl;
    for (uint32_t k = 0; k < w; ++k) off += wsum[k];
    off += inc - sum;
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t t = tt + k;
      if (h[k] && off < p.hit_cap) {
        if (h[k] <= kSlot) {
          const uint32_t text = p.single ? 0u : text_of_tile(p, t);
          const Slot* sl = p.slots + t * kSlot;
          put_hit(p, off, text, first[k].pos, first[k].pid);
          for (uint32_t i = 1; i < h[k]; ++i) {
            const Slot s = sl[i];
            put_hit(p, off + i, text, s.pos, s.pid);
          }
        } else {
          const uint32_t i = atomicAdd(&novf, 1u);
          ovf_tile[i] = 4 * threadIdx.x + k;
          ovf_off[i] = off;
        }
      }
      off += h[k];
    }
    __syncthreads();
    // tiles whose hits did not fit their slots: one wave each
    for (uint32_t i = w; i < novf; i += 16) {
      const uint64_t t = base + ovf_tile[i];
      uint64_t o = ovf_off[i];
      uint32_t text = 0;
      DevSeg seg = p.seg0;
      uint64_t ts = t;
      DevTable tab = p.tab0;
      uint32_t tile = p.tile;
      if (!p.single) {
        text = text_of_tile(p, t);
        seg = p.segs[text];
        ts = t - seg.first_tile;
        tab = p.tables[seg.table];
        tile = 1u << seg.tile_shift;
      }
      const uint64_t t0 = ts * tile;
      const uint8_t* tx = p.text + seg.text_off;
      for (uint32_t k = 0; k < tile / 256; ++k) {   // 64 lanes x 4 positions per step
        const uint64_t pos0 = t0 + k * 256 + 4 * lane;
        int32_t v[4] = {0, 0, 0, 0};
        #pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
          if (pos0 + r >= seg.n) continue;
          if (p.match) {
            v[r] = p.match[seg.match_off + pos0 + r];
          } else {
            unsigned long long unused = 0;
            walk<true>(0u, pos0 + r, nullptr, nullptr, tab.next, tab.out, tx, seg.n, seg.enc,
                       v[r], unused);
          }
        }
        const uint32_t c = (v[0] != 0) + (v[1] != 0) + (v[2] != 0) + (v[3] != 0);
        uint32_t tot;
        uint64_t oo = o + wave_excl(c, &tot);
        #pragma unroll
        for (uint32_t r = 0; r < 4; ++r)
          if (v[r]) put_hit(p, oo++, text, (uint32_t)(pos0 + r), v[r]);
        o += tot;
      }
    }
  }
  if (s_last) {
    // every workgroup has published its counts and finished its look-back:
    // totals, then clear the words and counters for the next launch
    __shared__ unsigned long long tot_occ[16];
    const uint32_t nb = gridDim.x;
    unsigned long long o = 0;
    for (uint32_t b = threadIdx.x; b < nb; b += 1024)
      o += __hip_atomic_load(&p.block_occ[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    o = wave_sum(o);
    if (lane == 0) tot_occ[w] = o;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long to = 0;
      for (int k = 0; k < 16; ++k) to += tot_occ[k];
      const unsigned long long last =
          __hip_atomic_load(&p.status[nb - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      p.counters[0] = (s_excl == ~0ull) ? ~0ull : (last & kLbMask);
      p.counters[1] = to;
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += 1024)
      __hip_atomic_store(&p.status[b], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) {
      __hip_atomic_store(&p.sync[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&p.sync[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Batch: per-text hit and occurrence totals, one wave per text.
__global__ __launch_bounds__(256) void pfac_text_totals_kernel(
    const uint32_t* tile_hits, const unsigned long long* tile_occ, const uint64_t* tile_prefix,
    uint32_t nsegs, unsigned long long* seg_counters) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t s = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= nsegs) return;
  unsigned long long h = 0, o = 0;
  for (uint64_t t = tile_prefix[s] + lane; t < tile_prefix[s + 1]; t += 64) {
    h += tile_hits[t];
    o += tile_occ[t];
  }
  h = wave_sum(h);
  o = wave_sum(o);
  if (lane == 0) {
    seg_counters[2 * s] = h;
    seg_counters[2 * s + 1] = o;
  }
}

// Zero the counters of a call that has no tiles at all.
__global__ void pfac_zero_kernel(unsigned long long* c, uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0;
}

// The paper's layouts of the transition table from the edge words: per
// cell the child state and the smallest ID of the patterns ending at it.
__global__ __launch_bounds__(256) void pfac_cells_kernel(const uint32_t* next, const OutEntry* out,
                                                         uint64_t cells, uint32_t* next2,
                                                         int32_t* cell_pid, u32x2* merged) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < cells;
       i += (uint64_t)gridDim.x * 256) {
    const uint32_t e = next[i];
    const uint32_t child = e & kStateMask;
    const int32_t id = (e & kFinalBit) ? out[child].pid : 0;
    next2[i] = child;
    cell_pid[i] = id;
    merged[i] = u32x2{child, (uint32_t)id};
  }
}

// Pair table of depth D from the depth-D filter bitmap: four strings m per
// thread (one 32-bit word of the table).
__global__ __launch_bounds__(256) void pfac_pair_kernel(const uint32_t* bitmap, uint32_t D,
                                                        uint32_t* pair) {
  const uint32_t nm = 1u << (2 * (D - 1));
  const uint32_t hi = 2 * (D - 1);
  auto bit = [&](uint32_t x) { return (bitmap[x >> 5] >> (x & 31u)) & 1u; };
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nm / 4; i += gridDim.x * 256) {
    uint32_t word = 0;
    for (uint32_t k = 0; k < 4; ++k) {
      const uint32_t m = 4 * i + k;
      uint32_t e = 0;
      for (uint32_t a = 0; a < 4; ++a) e |= bit((a << hi) | m) << a;
      for (uint32_t b = 0; b < 4; ++b) e |= bit((m << 2) | b) << (4 + b);
      word |= e << (8 * k);
    }
    pair[i] = word;
  }
}

// Node records of the deferred walks: per state its four edge words, its run
// record and its output, 32 bytes, so that a walk step reads one record
// (one cache line) instead of an edge word, a run record and an output in
// three arrays.
__global__ __launch_bounds__(256) void pfac_node_kernel(const uint32_t* next, const uint32_t* chain,
                                                        const OutEntry* out, uint64_t S,
                                                        uint32_t* node) {
  for (uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x; s < S;
       s += (uint64_t)gridDim.x * 256) {
    const u32x4 a = reinterpret_cast<const u32x4*>(next)[s];
    const OutEntry o = out[s];
    const u32x4 b = {chain[2 * s], chain[2 * s + 1], (uint32_t)o.pid, o.mult};
    reinterpret_cast<u32x4*>(node)[2 * s] = a;
    reinterpret_cast<u32x4*>(node)[2 * s + 1] = b;
  }
}

// Batch work items: one wave per text writes the items of its tiles (text
// offsets, length and encoding, tile index in the call and in the text, text
// index) from item_start[text] on.
__global__ __launch_bounds__(256) void pfac_items_kernel(const DevSeg* segs,
                                                         const uint64_t* item_start,
                                                         uint32_t ntexts, TileItem* items) {
  const uint64_t t = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= ntexts) return;
  const DevSeg s = segs[t];
  const uint64_t tiles = ((uint64_t)s.n + (1u << s.tile_shift) - 1) >> s.tile_shift;
  TileItem* dst = items + item_start[t];
  for (uint64_t j = threadIdx.x & 63; j < tiles; j += 64)
    dst[j] = TileItem{s.text_off, s.match_off, s.n, s.first_tile + (uint32_t)j, (uint32_t)j,
                      (uint32_t)t | ((uint32_t)s.enc << 31)};
}

// ---------------------------------------------------------------- host side

static std::mutex g_mu;
std::mutex& host_mutex() { return g_mu; }

// The variants that walk every position from the root in global memory.
static bool global_variant(uint32_t v) {
  return v == PFAC_VARIANT_GLOBAL || v == PFAC_VARIANT_GLOBAL_TWO_ARRAYS ||
         v == PFAC_VARIANT_GLOBAL_MERGED;
}


struct DeviceInfo {
  int cus = 0;
  int lds_per_block = 0;
  bool ok = false;
};

static DeviceInfo device_info(int dev) {
  static std::map<int, DeviceInfo> cache;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  DeviceInfo d;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    d.cus = prop.multiProcessorCount;
    d.lds_per_block = (int)prop.sharedMemPerBlock;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > d.lds_per_block)
      d.lds_per_block = v;
    d.ok = strstr(prop.gcnArchName, "gfx950") != nullptr;
  }
  cache[dev] = d;
  return d;
}

uint64_t al256(uint64_t x) { return (x + 255) / 256 * 256; }

ScratchLayout scratch_layout(uint64_t tiles, bool items, uint64_t walks) {
  ScratchLayout L;
  const uint64_t blocks = (tiles + kRedTiles - 1) / kRedTiles;
  L.o_hits = 0;
  L.o_occ = al256(L.o_hits + tiles * 4);
  L.o_slots = al256(L.o_occ + tiles * 8);
  L.o_st = al256(L.o_slots + tiles * kSlot * sizeof(Slot));
  L.o_bo = al256(L.o_st + blocks * 8);
  L.o_sync = al256(L.o_bo + blocks * 8);
  L.zero_bytes = al256(L.o_sync + 256) - L.o_st;   // look-back words .. counters
  L.o_items = al256(L.o_sync + 256);
  L.o_walk = al256(L.o_items + (items ? tiles * sizeof(TileItem) : 0));
  L.o_dummy = al256(L.o_walk + walks * sizeof(WalkEntry));
  L.bytes = al256(L.o_dummy + (uint64_t)kPzSlots * kTileSingle * 4);
  return L;
}

Scratch carve(uint8_t* mem, const ScratchLayout& L, uint64_t tiles, uint64_t walks) {
  Scratch s;
  s.tile_hits = reinterpret_cast<uint32_t*>(mem + L.o_hits);
  s.tile_occ = reinterpret_cast<unsigned long long*>(mem + L.o_occ);
  s.slots = reinterpret_cast<Slot*>(mem + L.o_slots);
  s.status = reinterpret_cast<unsigned long long*>(mem + L.o_st);
  s.block_occ = reinterpret_cast<unsigned long long*>(mem + L.o_bo);
  s.sync = reinterpret_cast<uint32_t*>(mem + L.o_sync);
  s.items = reinterpret_cast<TileItem*>(mem + L.o_items);
  s.walk = reinterpret_cast<WalkEntry*>(mem + L.o_walk);
  s.dummy = reinterpret_cast<int32_t*>(mem + L.o_dummy);
  s.tiles = tiles;
  s.walk_cap = walks;
  return s;
}

// Library-owned scratch of one (device, stream), grown on demand, plus the
// device copy of a batch layout and its pinned staging buffer.  Calls on one
// stream use it in stream order.
struct Workspace {
  uint8_t* mem = nullptr;
  uint64_t bytes = 0;
  Scratch sc;
  void* batch = nullptr;           // descriptors, prefixes, item starts, table views
  uint64_t batch_cap = 0;
  uint8_t* stage = nullptr;        // pinned host copy of `batch` being uploaded
  hipEvent_t staged = nullptr;     // recorded after the upload that read `stage`
  bool staged_pending = false;
  uint8_t* extra = nullptr;        // scratch of passes after the scan (all occurrences)
  uint64_t extra_cap = 0;
};

static std::map<std::pair<int, void*>, Workspace*> g_ws;

// Room for `tiles` tiles (with batch items when `items`) and `walks`
// deferred walks.  The look-back words and counters start at zero and the
// finish kernel leaves them so; a grown block is cleared once.
static int ensure_scratch(Workspace* ws, uint64_t tiles, bool items, uint64_t walks,
                          hipStream_t stream) {
  const uint64_t need_t = std::max<uint64_t>(tiles, 1);
  if (ws->mem && need_t <= ws->sc.tiles && walks <= ws->sc.walk_cap &&
      (!items || ws->sc.items != nullptr))
    return PFAC_OK;
  const uint64_t cap_t = std::max<uint64_t>(std::max(need_t + need_t / 4, ws->sc.tiles), 4096);
  const uint64_t cap_w = std::max(walks + walks / 4, ws->sc.walk_cap);
  const ScratchLayout L = scratch_layout(cap_t, true, cap_w);
  if (ws->mem) {
    if (hipStreamSynchronize(stream) != hipSuccess) return PFAC_E_HIP;
    (void)hipFree(ws->mem);
    ws->mem = nullptr;
    ws->sc = Scratch();
  }
  void* m = nullptr;
  if (hipMalloc(&m, L.bytes) != hipSuccess) return PFAC_E_NOMEM;
  ws->mem = static_cast<uint8_t*>(m);
  ws->bytes = L.bytes;
  if (hipMemset(ws->mem + L.o_st, 0, L.zero_bytes) != hipSuccess) return PFAC_E_HIP;
  ws->sc = carve(ws->mem, L, cap_t, cap_w);
  return PFAC_OK;
}

static int ensure_batch(Workspace* ws, uint64_t bytes, hipStream_t stream) {
  if (!ws->staged && hipEventCreateWithFlags(&ws->staged, hipEventDisableTiming) != hipSuccess)
    return PFAC_E_HIP;
  // the previous upload must have finished reading the pinned stage
  if (ws->staged_pending) {
    if (hipEventSynchronize(ws->staged) != hipSuccess) return PFAC_E_HIP;
    ws->staged_pending = false;
  }
  if (bytes <= ws->batch_cap && ws->batch) return PFAC_OK;
  const uint64_t cap = std::max<uint64_t>(bytes + bytes / 2, 1 << 16);
  if (ws->batch) {
    if (hipStreamSynchronize(stream) != hipSuccess) return PFAC_E_HIP;
    (void)hipFree(ws->batch);
    (void)hipHostFree(ws->stage);
    ws->batch = nullptr;
    ws->stage = nullptr;
    ws->batch_cap = 0;
  }
  if (hipMalloc(&ws->batch, cap) != hipSuccess) {
    ws->batch = nullptr;
    return PFAC_E_NOMEM;
  }
  void* st = nullptr;
  if (hipHostMalloc(&st, cap, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(ws->batch);
    ws->batch = nullptr;
    return PFAC_E_NOMEM;
  }
  ws->stage = static_cast<uint8_t*>(st);
  ws->batch_cap = cap;
  return PFAC_OK;
}

static Workspace* get_workspace(int dev, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace*& ws = g_ws[{dev, (void*)stream}];
  if (!ws) ws = new (std::nothrow) Workspace();
  return ws;
}

static int ensure_extra(Workspace* ws, uint64_t bytes, hipStream_t stream) {
  if (bytes <= ws->extra_cap && (ws->extra || bytes == 0)) return PFAC_OK;
  const uint64_t cap = std::max<uint64_t>(bytes + bytes / 4, 1 << 16);
  if (ws->extra) {
    if (hipStreamSynchronize(stream) != hipSuccess) return PFAC_E_HIP;
    (void)hipFree(ws->extra);
    ws->extra = nullptr;
    ws->extra_cap = 0;
  }
  void* m = nullptr;
  if (hipMalloc(&m, cap) != hipSuccess) return PFAC_E_NOMEM;
  ws->extra = static_cast<uint8_t*>(m);
  ws->extra_cap = cap;
  return PFAC_OK;
}

Workspace* workspace_for(int dev, hipStream_t stream, uint64_t tiles, uint64_t walks,
                         uint64_t extra, int* rc) {
  Workspace* ws = get_workspace(dev, stream);
  if (!ws) {
    *rc = PFAC_E_NOMEM;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  *rc = ensure_scratch(ws, tiles, false, walks, stream);
  if (!*rc) *rc = ensure_extra(ws, extra, stream);
  return *rc ? nullptr : ws;
}

const Scratch& workspace_scratch(const Workspace* ws) { return ws->sc; }
uint8_t* workspace_extra(const Workspace* ws) { return ws->extra; }

static void free_workspace(Workspace* ws) {
  if (ws->extra) (void)hipFree(ws->extra);
  if (ws->mem) (void)hipFree(ws->mem);
  if (ws->batch) (void)hipFree(ws->batch);
  if (ws->stage) (void)hipHostFree(ws->stage);
  if (ws->staged) (void)hipEventDestroy(ws->staged);
  *ws = Workspace();
}

static uint32_t halo_for(uint32_t max_len) {
  uint32_t h = max_len > 1 ? max_len - 1 : 0;
  if (h < 16) h = 16;   // room for the filter window of the last positions
  return (h + 63) / 64 * 64;
}

// Image words the scan kernel copies for depth D with `levels` trie levels
// (lds_trie) or the bare filter bitmap (otherwise).
static uint32_t image_words(const HostTable& h, uint32_t D, bool lds_trie, uint32_t levels) {
  const uint32_t bits = (1u << (2 * D)) / 32;
  if (!lds_trie) return bits;
  if (levels == 0) return bits + bits / 4;
  return h.image[D].upto[levels - 1];
}

// LDS of a scan launch with `tile`-position tiles.
static uint32_t scan_lds_bytes(uint32_t block, uint32_t img_words, uint32_t halo, uint32_t tile) {
  return 4u * (img_words + kLvlWords + (block / 64) * wave_words(tile, halo) + kCtlWords);
}

static ScanFn pick_scan(uint32_t block, bool global, uint32_t D, bool single, bool defer,
                        uint32_t tile, bool pz = false) {
  switch (block) {
    case 256: return single ? pick_scan_single_256(global, D, defer, tile, pz)
                            : pick_scan_batch_256(global, D, defer, tile, pz);
    case 512: return single ? pick_scan_single_512(global, D, defer, tile, pz)
                            : pick_scan_batch_512(global, D, defer, tile, pz);
    case 768: return single ? pick_scan_single_768(global, D, defer, tile, pz)
                            : pick_scan_batch_768(global, D, defer, tile, pz);
    case 1024: return single ? pick_scan_single_1024(global, D, defer, tile, pz)
                             : pick_scan_batch_1024(global, D, defer, tile, pz);
    default: return nullptr;
  }
}

// Filter depth the library picks: deepen while at least 5 % of the windows
// of the next level are trie prefixes, up to 10 (a 128 KB bitmap, which only
// fits beside the text of 512-thread or smaller workgroups).
static uint32_t auto_depth(const HostTable& h) {
  uint32_t D = kMinJump;
  for (uint32_t d = kMinJump; d <= kMaxJump; ++d) {
    const uint64_t at_d = (d + 1 < h.depth_start.size())
                              ? h.depth_start[d + 1] - h.depth_start[d] : 0;
    D = d;
    if ((double)at_d < 0.05 * (double)(1ull << (2 * d))) break;
  }
  return D;
}

// Second-filter size the library picks: 2^18 bits while the patterns number
// at most 26,000 (two bits each leave under 0.5 % of random windows
// passing; smaller bitmaps were measured no faster on 1,000 to 10,000
// patterns), 2^19 up to 210,000 patterns, none beyond.
static uint32_t auto_hash_bits(const HostTable& h) {
  if (h.num_patterns <= 26000) return 18;
  if ((double)h.num_patterns <= 0.4 * (double)(1u << 19)) return 19;
  return PFAC_HASH_NONE;
}

// The prefix filter pays when the hashed bitmap is weak or absent.
static bool auto_prefix(const HostTable& h, uint32_t D, uint32_t hb) {
  if (h.pfx_k <= D) return false;
  return hb == PFAC_HASH_NONE || h.num_patterns > 26000;
}

constexpr int kNoFit = 1;

// Place the depth-D image in LDS next to `hw` words of second filter: with
// every pattern longer than D, rank words and as many trie levels as asked
// for (levels 0 = as many as fit); otherwise, or with PFAC_LEVELS_NONE, the
// bare filter bitmap.  Sets p->levels on success; kNoFit when it does not fit.
static int place_image(const HostTable& h, uint32_t D, uint32_t hw, uint32_t halo,
                       uint32_t budget, uint32_t tile, pfac_plan* p) {
  if (h.min_len > D && p->levels != PFAC_LEVELS_NONE && p->pair != 1) {
    const uint32_t have = h.image[D].levels;
    const uint32_t want = p->levels == 0 ? have : std::min(p->levels, have);
    for (int32_t L = (int32_t)want; L >= 0; --L) {
      if (scan_lds_bytes(p->block, image_words(h, D, true, (uint32_t)L) + hw, halo, tile) <=
          budget) {
        if (p->levels != 0 && (uint32_t)L < want) return kNoFit;   // explicit, too big
        p->levels = (uint32_t)L;
        p->pair = PFAC_PAIR_NONE;
        return PFAC_OK;
      }
    }
    if (p->levels != 0) return kNoFit;
  }
  if (p->levels != PFAC_LEVELS_NONE && p->levels != 0) return kNoFit;   // levels asked for
  // filter bitmap only (or its pair table); survivors read the global
  // depth-D jump table
  const uint32_t bits = image_words(h, D, false, 0);
  if (p->pair != PFAC_PAIR_NONE && D <= kPairMaxDepth) {
    if (scan_lds_bytes(p->block, 2 * bits + hw, halo, tile) <= budget) {
      p->levels = PFAC_LEVELS_NONE;
      p->pair = 1;
      return PFAC_OK;
    }
    if (p->pair == 1) return kNoFit;             // explicit, does not fit
  }
  if (p->pair == 1) return kNoFit;               // no pair table at this depth
  if (scan_lds_bytes(p->block, bits + hw, halo, tile) <= budget) {
    p->levels = PFAC_LEVELS_NONE;
    p->pair = PFAC_PAIR_NONE;
    return PFAC_OK;
  }
  return kNoFit;
}

// The plan of a call.  `single`: a one-text call (tile 256 is for batches);
// the LDS is sized for the largest tile the plan may run with (2048 when the
// tile is left to the library in a batch: texts get 256 or 1024).
static int resolve_plan(const pfac_plan* in, const HostTable& h, int dev, bool single,
                        pfac_plan* out) {
  const DeviceInfo di = device_info(dev);
  if (!di.ok) return PFAC_E_NODEV;
  pfac_plan p = in ? *in : pfac_plan{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (p.pair != 0 && p.pair != 1 && p.pair != PFAC_PAIR_NONE) return PFAC_E_ARG;
  if (p.variant != PFAC_VARIANT_TILED && !global_variant(p.variant)) return PFAC_E_ARG;
  if (!single && p.variant != PFAC_VARIANT_TILED && p.variant != PFAC_VARIANT_GLOBAL)
    return PFAC_E_ARG;
  if (p.tile != 0 && p.tile != 1024 && p.tile != 2048 && !(p.tile == 256 && !single))
    return PFAC_E_ARG;
  if (p.prefix != 0 && p.prefix != 1 && p.prefix != PFAC_PREFIX_NONE) return PFAC_E_ARG;
  const uint32_t halo = halo_for(h.max_len);
  if (p.variant == PFAC_VARIANT_TILED && halo > kMaxHalo) {
    if (in && in->depth) return PFAC_E_ARG;
    p.variant = PFAC_VARIANT_GLOBAL;  // patterns too long to stage a halo in LDS
  }
  // Library choice when every pattern is longer than the filter depth and
  // the second filter is worth keeping: bitmap + second filter only (the few
  // windows that pass both are walked from the global jump table), depth 9
  // when the patterns' first K bases go past it, in 1024-thread workgroups --
  // measured faster than keeping trie levels in LDS, whose walks the second
  // filter has already cut down, and than shallower bitmaps or 512-thread
  // workgroups.  Otherwise 1024-thread workgroups and as many LDS trie
  // levels as fit.
  const bool auto_b = p.block == 0;
  const bool auto_d = p.depth == 0;
  if (p.variant == PFAC_VARIANT_TILED && p.levels == 0 && p.hash_bits == 0) {
    uint32_t D = p.depth ? p.depth : std::min<uint32_t>(auto_depth(h), 9u);
    if (!p.depth && h.hash_k > 9) D = 9;
    const uint32_t hb = auto_hash_bits(h);
    if (h.hash_k > D && hb != PFAC_HASH_NONE) {
      p.levels = PFAC_LEVELS_NONE;
      p.depth = D;
    }
  }
  if (p.block == 0) p.block = 1024;
  if (p.block != 256 && p.block != 512 && p.block != 768 && p.block != 1024) return PFAC_E_ARG;
  if (p.walks != 0 && p.walks != PFAC_WALKS_INLINE && p.walks != PFAC_WALKS_DEFERRED)
    return PFAC_E_ARG;
  if (global_variant(p.variant)) {
    if (p.tile != 0 && p.tile != (single ? kTileSingle : kTileBatch)) return PFAC_E_ARG;
    p.depth = 0;
    p.levels = PFAC_LEVELS_NONE;
    p.hash_bits = PFAC_HASH_NONE;
    p.walks = PFAC_WALKS_INLINE;
    p.prefix = PFAC_PREFIX_NONE;
    p.pair = PFAC_PAIR_NONE;
    p.tile = single ? kTileSingle : kTileBatch;
    *out = p;
    return PFAC_OK;
  }
  const uint32_t tile_lds = p.tile ? p.tile : kTileSingle;
  const uint32_t budget = (uint32_t)di.lds_per_block;
  const bool auto_h = p.hash_bits == 0;
  if (!auto_h && p.hash_bits != PFAC_HASH_NONE &&
      (p.hash_bits < kHashMinBits || p.hash_bits > kHashMaxBits))
    return PFAC_E_ARG;
  if (p.depth == 0) p.depth = auto_depth(h);
  for (;;) {
    if (p.depth < kMinJump || p.depth > kMaxJump) return PFAC_E_ARG;
    const uint32_t D = p.depth;
    // the second filter only helps when every pattern is longer than D;
    // when the image does not fit beside it, the library's choice tries a
    // smaller bitmap, then drops it, before it drops trie levels or depth
    uint32_t hb = PFAC_HASH_NONE;
    if (h.hash_k > D && p.hash_bits != PFAC_HASH_NONE)
      hb = auto_h ? auto_hash_bits(h) : p.hash_bits;
    const uint32_t block0 = p.block;
    for (;;) {
      const uint32_t hw = hb == PFAC_HASH_NONE ? 0u : (1u << hb) / 32;
      const int rc = place_image(h, D, hw, halo, budget, tile_lds, &p);
      if (rc == PFAC_OK) {
        p.hash_bits = hb;
        if (p.prefix == 1 && h.pfx_k <= D) return PFAC_E_ARG;
        if (p.prefix == 0) p.prefix = auto_prefix(h, D, hb) ? 1u : PFAC_PREFIX_NONE;
        if (h.pfx_k <= D) p.prefix = PFAC_PREFIX_NONE;
        // walks that survive the filters are few: keep them for the end of
        // the wave so the streaming scan never waits on their table reads --
        // when the 64 bases copied with each cover every pattern (past them a
        // deferred walk reads the text one base at a time)
        if (p.walks == 0)
          p.walks = ((hb != PFAC_HASH_NONE || p.prefix == 1) && h.max_len <= kWindow)
                        ? PFAC_WALKS_DEFERRED : PFAC_WALKS_INLINE;
        if (p.tile == 0 && single) p.tile = kTileSingle;
        *out = p;
        return PFAC_OK;
      }
      if (rc != kNoFit) return rc;
      if (auto_b && p.block > 256) {
        p.block = p.block > 512 ? 512 : 256;
        continue;
      }
      if (hb == PFAC_HASH_NONE || !auto_h) break;
      hb = hb > 18 ? hb - 1 : PFAC_HASH_NONE;
      p.block = block0;
    }
    p.block = block0;
    if (!auto_d || D == kMinJump) return PFAC_E_ARG;
    --p.depth;
  }
}

// Resident workgroups per CU for (kernel, block, LDS bytes), cached: the
// occupancy query and the LDS attribute are set once per combination.
static int blocks_per_cu(ScanFn fn, uint32_t block, uint32_t lds) {
  static std::map<std::tuple<void*, uint32_t, uint32_t>, int> cache;
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(reinterpret_cast<void*>(fn), block, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  // raise the kernel's dynamic-LDS limit to the largest any plan may ask for,
  // so that a smaller request later never lowers it below a cached one
  if (lds > 48 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)std::max<uint32_t>(lds, kImageMaxBytes));
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn),
                                                   (int)block, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  cache[key] = per_cu;
  return per_cu;
}

static uint64_t grid_for(ScanFn fn, const pfac_plan& plan, uint32_t lds, int dev,
                         uint64_t tiles) {
  const int per_cu = blocks_per_cu(fn, plan.block, lds);
  uint64_t g = plan.grid ? plan.grid : (uint64_t)per_cu * (uint64_t)device_info(dev).cus;
  if (g > 2048) g = 2048;
  const uint64_t waves = plan.block / 64;
  const uint64_t need = (tiles + waves - 1) / waves;
  if (g > need) g = need;
  return g ? g : 1;
}

// Kernel, dynamic LDS and grid of a scan launch of `tile`-position tiles.
static int scan_shape(const ScanParams& sp, const pfac_plan& plan, bool single, uint32_t tile,
                      int dev, ScanFn* fn, uint32_t* lds, uint64_t* grid) {
  const bool global = global_variant(plan.variant);
  *fn = pick_scan(plan.block, global, sp.D, single, sp.defer != 0, tile);
  if (!*fn) return PFAC_E_ARG;
  *lds = global ? 4u * ((plan.block / 64) * kGlobalWaveWords + kCtlWords)
                : scan_lds_bytes(plan.block, sp.image_words + (sp.hash_on ? sp.hash_words : 0u),
                                 sp.halo, tile);
  *grid = grid_for(*fn, plan, *lds, dev, sp.local_tiles);
  return PFAC_OK;
}

static int launch_scan(const ScanParams& sp, const pfac_plan& plan, bool single, uint32_t tile,
                       int dev, hipStream_t stream) {
  if (sp.local_tiles == 0) return PFAC_OK;
  ScanFn fn;
  uint32_t lds;
  uint64_t grid;
  const int rc = scan_shape(sp, plan, single, tile, dev, &fn, &lds, &grid);
  if (rc) return rc;
  if (sp.defer && grid * (plan.block / 64) > sp.wq_waves) return PFAC_E_ARG;
  // deferred-walk scans with a dense output (16-byte aligned for one text;
  // a batch checks each text's): the pre-zeroing kernel, when it has the same
  // occupancy (hence grid)
  if (sp.defer && sp.match && sp.pz_dummy && !global_variant(plan.variant) &&
      (!single || (reinterpret_cast<uintptr_t>(sp.match) & 15) == 0)) {
    const ScanFn pz = pick_scan(plan.block, false, sp.D, single, true, tile, true);
    if (pz && blocks_per_cu(pz, plan.block, lds) == blocks_per_cu(fn, plan.block, lds)) fn = pz;
  }
  hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(plan.block), lds, stream, sp);
  return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
}

static int launch_tail(const Scratch& sc, uint64_t tiles, unsigned long long* counters,
                       FinishParams* fp, bool want_hits, hipStream_t stream) {
  const uint32_t blocks = (uint32_t)((tiles + kRedTiles - 1) / kRedTiles);
  fp->tile_hits = sc.tile_hits;
  fp->tile_occ = sc.tile_occ;
  fp->slots = sc.slots;
  fp->tiles = tiles;
  fp->status = sc.status;
  fp->block_occ = sc.block_occ;
  fp->sync = sc.sync;
  fp->counters = counters;
  if (!want_hits) {
    fp->hits = nullptr;
    fp->hit_cap = 0;
  }
  hipLaunchKernelGGL(pfac_finish_kernel, dim3(blocks), dim3(1024), 0, stream, *fp);
  return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
}

// The two-array and merged-cell tables of `t`, built once (synchronously).
static int ensure_cells(const pfac_table* t) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (t->cells_mem) return PFAC_OK;
  const uint64_t cells = t->host.num_states * 4;
  const uint64_t o_cp = al256(cells * 4), o_m = o_cp + al256(cells * 4);
  void* m = nullptr;
  if (hipMalloc(&m, o_m + cells * 8) != hipSuccess) return PFAC_E_NOMEM;
  uint8_t* b = static_cast<uint8_t*>(m);
  const uint64_t grid = std::min<uint64_t>((cells + 255) / 256, 65536);
  hipLaunchKernelGGL(pfac_cells_kernel, dim3((uint32_t)grid), dim3(256), 0, nullptr, t->dev.next,
                     t->dev.out, cells, reinterpret_cast<uint32_t*>(b),
                     reinterpret_cast<int32_t*>(b + o_cp), reinterpret_cast<u32x2*>(b + o_m));
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(m);
    return PFAC_E_HIP;
  }
  t->next2 = reinterpret_cast<const uint32_t*>(b);
  t->cell_pid = reinterpret_cast<const int32_t*>(b + o_cp);
  t->cells = b + o_m;
  t->cells_mem = m;
  return PFAC_OK;
}

// The second filter takes its one-hash form (and is tested while
// classifying) when most windows pass the depth-D bitmap (large pattern
// sets) and the K-base key fits in 24 bits.
static bool hash_one(const HostTable& h, uint32_t D) {
  if (h.hash_k == 0 || h.hash_k > kHash1MaxK || D < kMinJump || D > kMaxJump) return false;
  return (double)h.bitmap_set[D] / (double)(1ull << (2 * D)) > 0.3;
}

static void fill_table(ScanParams& sp, const pfac_table* t, const pfac_plan& pl) {
  sp.next = t->dev.next;
  sp.out = t->dev.out;
  sp.chain = t->dev.chain;
  sp.node = reinterpret_cast<const u32x4*>(t->dev.node);
  if (pl.variant == PFAC_VARIANT_GLOBAL_TWO_ARRAYS || pl.variant == PFAC_VARIANT_GLOBAL_MERGED) {
    // the kernel's depth parameter names the layout for global variants
    sp.D = pl.variant == PFAC_VARIANT_GLOBAL_TWO_ARRAYS ? 1u : 2u;
    sp.next2 = t->next2;
    sp.cell_pid = t->cell_pid;
    sp.cells = static_cast<const u32x2*>(t->cells);
  }
  if (pl.variant == PFAC_VARIANT_TILED) {
    const HostTable& h = t->host;
    const uint32_t D = pl.depth;
    sp.D = D;
    sp.jump = t->dev.jump[D];
    sp.jres = t->dev.jres[D];
    sp.image = t->dev.image[D];
    sp.longer = h.min_len > D ? 1u : 0u;
    sp.lds_trie = (h.min_len > D && pl.levels != PFAC_LEVELS_NONE) ? 1u : 0u;
    sp.levels = sp.lds_trie ? pl.levels : 0u;
    sp.image_words = image_words(h, D, sp.lds_trie, sp.levels);
    if (pl.pair == 1 && !sp.lds_trie) {
      sp.pair = 1;
      sp.image = reinterpret_cast<const uint32_t*>(t->dev.pair[D]);
      sp.image_words = 2 * image_words(h, D, false, 0);
    }
    sp.lvl = reinterpret_cast<const u32x4*>(t->dev.levels[D]);
    if (pl.hash_bits != PFAC_HASH_NONE) {
      const uint32_t b = pl.hash_bits, K = h.hash_k;
      sp.hash_on = 1;
      sp.hash = t->dev.hash[b];
      sp.hash_words = (1u << b) / 32;
      sp.hash_shift = 32 - b;
      sp.hash_kmask = K >= 16 ? 0xFFFFFFFFu : ~((1u << (32 - 2 * K)) - 1u);
      sp.hash_imask = (1u << K) - 1u;
      // when most windows pass the depth-D bitmap (large pattern sets), every
      // window of a tile takes the second filter while it is classified
      // instead of through the queue (its K bases then fit the 16 bases a
      // group of four positions holds)
      if (hash_one(h, D) && t->dev.hash1[b]) {
        sp.hash_cls = 1;
        sp.hash = t->dev.hash1[b];
        sp.hash_kshift = 32 - 2 * K;
      }
    }
    if (pl.prefix == 1 && h.pfx_k > D) {
      sp.pfx_on = 1;
      sp.pfx = t->dev.pfx;
      sp.pfx_shift = 32 - 2 * h.pfx_k;
      sp.pfx_imask = (1u << h.pfx_k) - 1u;
    }
  }
}

// Deferred walks a tile keeps room for: about twice the walks the filters
// let through on random text, at least 4, at most 32.  With the exact prefix
// filter that is the fraction of K2-base windows that start a pattern;
// otherwise the windows passing the depth-D bitmap, times the square of the
// hashed bitmap's fill (its false positives; the true matches are few).
static uint32_t defer_per_tile(const HostTable& h, const pfac_plan& pl, uint32_t tile) {
  double pass;
  if (pl.prefix == 1 && h.pfx_k > pl.depth) {
    pass = (double)h.pfx_set / (double)(1ull << (2 * h.pfx_k));
  } else {
    pass = (double)h.bitmap_set[pl.depth] / (double)(1ull << (2 * pl.depth));
    if (pl.hash_bits != PFAC_HASH_NONE && hash_one(h, pl.depth)) {
      pass *= (double)h.hash1_set[pl.hash_bits] / (double)(1ull << pl.hash_bits);
    } else if (pl.hash_bits != PFAC_HASH_NONE) {
      const double f = (double)h.hash_set[pl.hash_bits] / (double)(1ull << pl.hash_bits);
      pass *= f * f;
    }
  }
  const double per = std::ceil(2.0 * pass * tile) + 4.0;
  return (uint32_t)std::min(32.0, std::max(4.0, per));
}

// Byte offsets of every array of a table in its one device allocation:
// next | out | chain | per depth: jump, jres, image, level descriptors |
// second-filter bitmaps | prefix bitmap | duplicate IDs.  Computed from the
// table's metadata (state count, depth starts, image layouts, filter K's),
// so a table built on the host and one built on the device share it.
void table_layout(const HostTable& h, uint64_t ndups, TableLayout* L) {
  const uint64_t S = h.num_states;
  uint64_t off = 0;
  L->o_next = off; off = al256(off + S * 16);
  L->o_out = off; off = al256(off + S * sizeof(OutEntry));
  L->o_chain = off; off = al256(off + S * 8);
  L->o_node = off; off = al256(off + S * 32);
  for (uint32_t D = kMinJump; D <= kMaxJump; ++D) {
    const uint64_t E = 1ull << (2 * D);
    const HostTable::Image& im = h.image[D];
    L->image_words[D] = im.levels ? im.upto[im.levels - 1] : (uint32_t)(E / 32 + E / 128);
    L->o_jump[D] = off; off = al256(off + E * 4);
    L->o_jres[D] = off; off = al256(off + E * sizeof(OutEntry));
    L->o_im[D] = off; off = al256(off + (uint64_t)L->image_words[D] * 4);
    L->lvdesc[D].assign(4 * kImageLevels, 0);
    for (uint32_t k = 0; k < kImageLevels; ++k) {
      if (k < im.levels) {
        L->lvdesc[D][4 * k] = im.byte_off[k];
        L->lvdesc[D][4 * k + 1] = im.pre_off[k];
      }
      if (D + k < h.depth_start.size()) L->lvdesc[D][4 * k + 2] = (uint32_t)h.depth_start[D + k];
    }
    L->o_lv[D] = off; off = al256(off + L->lvdesc[D].size() * 4);
    if (D <= kPairMaxDepth) {
      L->o_pair[D] = off;
      off = al256(off + (E >> 2));
    }
  }
  for (uint32_t b = kHashMinBits; b <= kHashMaxBits; ++b) {
    L->hash_words[b] = h.hash_k ? (1u << b) / 32 : 0;
    L->o_hash[b] = off; off = al256(off + (uint64_t)L->hash_words[b] * 4);
  }
  for (uint32_t b = kHashMinBits; b <= kHashMaxBits; ++b) {
    L->hash1_words[b] = (h.hash_k && h.hash_k <= kHash1MaxK) ? (1u << b) / 32 : 0;
    L->o_hash1[b] = off; off = al256(off + (uint64_t)L->hash1_words[b] * 4);
  }
  L->pfx_words = h.pfx_k ? (1ull << (2 * h.pfx_k)) / 32 : 0;
  L->o_pfx = off; off = al256(off + L->pfx_words * 4);
  L->ndups = ndups;
  L->o_dups = off; off = al256(off + ndups * 4);
  L->o_dupi = off; off = al256(off + ndups * 4);
  L->bytes = off;
}

// Allocate (zeroed) and point t->dev at the arrays of t's layout; uploads
// the level descriptors.
int alloc_table(pfac_table* t, uint64_t ndups) {
  TableLayout& L = t->layout;
  table_layout(t->host, ndups, &L);
  if (hipMalloc(&t->dmem, L.bytes) != hipSuccess) {
    t->dmem = nullptr;
    return PFAC_E_NOMEM;
  }
  t->dbytes = L.bytes;
  char* base = static_cast<char*>(t->dmem);
  if (hipMemset(base, 0, L.bytes) != hipSuccess) return PFAC_E_HIP;
  DevTable& v = t->dev;
  memset(&v, 0, sizeof(v));
  v.next = reinterpret_cast<const uint32_t*>(base + L.o_next);
  v.out = reinterpret_cast<const OutEntry*>(base + L.o_out);
  v.chain = reinterpret_cast<const uint32_t*>(base + L.o_chain);
  v.node = reinterpret_cast<const uint32_t*>(base + L.o_node);
  v.pfx = L.pfx_words ? reinterpret_cast<const uint32_t*>(base + L.o_pfx) : nullptr;
  v.dup_state = reinterpret_cast<const uint32_t*>(base + L.o_dups);
  v.dup_id = reinterpret_cast<const int32_t*>(base + L.o_dupi);
  v.num_dups = (uint32_t)ndups;
  v.num_states = (uint32_t)t->host.num_states;
  v.max_len = t->host.max_len;
  for (uint32_t D = kMinJump; D <= kMaxJump; ++D) {
    v.levels[D] = reinterpret_cast<const uint32_t*>(base + L.o_lv[D]);
    v.jump[D] = reinterpret_cast<const uint32_t*>(base + L.o_jump[D]);
    v.jres[D] = reinterpret_cast<const OutEntry*>(base + L.o_jres[D]);
    v.image[D] = reinterpret_cast<const uint32_t*>(base + L.o_im[D]);
    v.pair[D] = D <= kPairMaxDepth ? reinterpret_cast<const uint8_t*>(base + L.o_pair[D])
                                   : nullptr;
    if (hipMemcpy(base + L.o_lv[D], L.lvdesc[D].data(), L.lvdesc[D].size() * 4,
                  hipMemcpyHostToDevice) != hipSuccess)
      return PFAC_E_HIP;
  }
  for (uint32_t b = kHashMinBits; b <= kHashMaxBits; ++b) {
    v.hash[b] = reinterpret_cast<const uint32_t*>(base + L.o_hash[b]);
    v.hash1[b] = L.hash1_words[b] ? reinterpret_cast<const uint32_t*>(base + L.o_hash1[b])
                                  : nullptr;
  }
  return PFAC_OK;
}

// Copy a host-built table's arrays into its device allocation.
int upload_host_table(pfac_table* t) {
  const HostTable& h = t->host;
  const TableLayout& L = t->layout;
  char* base = static_cast<char*>(t->dmem);
  auto put = [&](uint64_t o, const void* src, size_t bytes) {
    return bytes == 0 || hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  bool ok = put(L.o_next, h.next.data(), h.next.size() * 4) &&
            put(L.o_out, h.out.data(), h.out.size() * sizeof(OutEntry)) &&
            put(L.o_chain, h.chain.data(), h.chain.size() * 4) &&
            put(L.o_pfx, h.pfx.data(), h.pfx.size() * 4) &&
            put(L.o_dups, h.dup_state.data(), h.dup_state.size() * 4) &&
            put(L.o_dupi, h.dup_id.data(), h.dup_id.size() * 4);
  for (uint32_t D = kMinJump; D <= kMaxJump; ++D)
    ok = ok && put(L.o_jump[D], h.jump[D].data(), h.jump[D].size() * 4) &&
         put(L.o_jres[D], h.jres[D].data(), h.jres[D].size() * sizeof(OutEntry)) &&
         put(L.o_im[D], h.image[D].words.data(), h.image[D].words.size() * 4);
  for (uint32_t b = kHashMinBits; b <= kHashMaxBits; ++b)
    ok = ok && put(L.o_hash[b], h.hash[b].data(), h.hash[b].size() * 4) &&
         put(L.o_hash1[b], h.hash1[b].data(), h.hash1[b].size() * 4);
  return ok ? PFAC_OK : PFAC_E_HIP;
}

// The arrays derived from others in a table's device allocation (either
// build): the node records and the pair tables; synchronous.
int build_derived(pfac_table* t) {
  const uint64_t S = t->host.num_states;
  if (S) {
    const uint64_t blocks = std::min<uint64_t>((S + 255) / 256, 65535);
    hipLaunchKernelGGL(pfac_node_kernel, dim3((uint32_t)blocks), dim3(256), 0, nullptr,
                       t->dev.next, t->dev.chain, t->dev.out, S,
                       const_cast<uint32_t*>(t->dev.node));
    if (hipGetLastError() != hipSuccess) return PFAC_E_HIP;
  }
  for (uint32_t D = kMinJump; D <= kPairMaxDepth; ++D) {
    const uint32_t words = (1u << (2 * (D - 1))) / 4;
    hipLaunchKernelGGL(pfac_pair_kernel, dim3((words + 255) / 256), dim3(256), 0, nullptr,
                       t->dev.image[D], D, const_cast<uint32_t*>(
                           reinterpret_cast<const uint32_t*>(t->dev.pair[D])));
    if (hipGetLastError() != hipSuccess) return PFAC_E_HIP;
  }
  return hipDeviceSynchronize() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
}

// Keep the pattern set (bytes and IDs) with the table, for updates.
int remember_patterns(pfac_table* t, const char* const* patterns, const uint32_t* lengths,
                      uint32_t num, const int32_t* ids) {
  try {
    t->pats.resize(num);
    t->ids.resize(num);
    for (uint32_t k = 0; k < num; ++k) {
      t->pats[k].assign(patterns[k], lengths[k]);
      t->ids[k] = ids ? ids[k] : (int32_t)(k + 1);
    }
  } catch (const std::bad_alloc&) {
    return PFAC_E_NOMEM;
  }
  return PFAC_OK;
}

}  // namespace pfac

using namespace pfac;

extern "C" {

int pfac_table_blob(const pfac_table* t, void* host, uint64_t cap, uint64_t* bytes) {
  if (!t || !bytes) return PFAC_E_ARG;
  *bytes = t->dbytes;
  if (host && cap >= t->dbytes) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (hipSetDevice(t->device) != hipSuccess) return PFAC_E_HIP;
    const hipError_t e = hipMemcpy(host, t->dmem, t->dbytes, hipMemcpyDeviceToHost);
    (void)hipSetDevice(cur);
    if (e != hipSuccess) return PFAC_E_HIP;
  }
  return PFAC_OK;
}

const char* pfac_strerror(int s) {
  switch (s) {
    case PFAC_OK: return "ok";
    case PFAC_E_ARG: return "invalid argument";
    case PFAC_E_PATTERN: return "empty pattern or pattern byte outside A,C,G,T";
    case PFAC_E_TOO_LARGE: return "trie needs 2^31 or more states";
    case PFAC_E_NOMEM: return "out of memory";
    case PFAC_E_HIP: return "HIP runtime error";
    case PFAC_E_NODEV: return "no gfx950 device";
    case PFAC_E_SCRATCH:
      return "input needs more scratch than the allocation-free entry point's fixed array";
    default: return "unknown status";
  }
}

const char* pfac_version(void) { return "pfac-mi355x 0.3 (gfx950)"; }

int pfac_build_table(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                     pfac_table** out, int64_t* bad_index) {
  if (!out) return PFAC_E_ARG;
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFAC_E_NODEV;
  if (!device_info(dev).ok) return PFAC_E_NODEV;
  pfac_table* t = new (std::nothrow) pfac_table();
  if (!t) return PFAC_E_NOMEM;
  int rc = build_host_table(patterns, lengths, num, &t->host, bad_index);
  if (rc != PFAC_OK) {
    delete t;
    return rc;
  }
  t->device = dev;
  rc = remember_patterns(t, patterns, lengths, num, nullptr);
  if (!rc) rc = alloc_table(t, t->host.dup_state.size());
  if (!rc) rc = upload_host_table(t);
  if (!rc) rc = build_derived(t);
  if (rc) {
    if (t->dmem) (void)hipFree(t->dmem);
    delete t;
    return rc;
  }
  *out = t;
  return PFAC_OK;
}

int pfac_table_info(const pfac_table* t, pfac_table_stats* o) {
  if (!t || !o) return PFAC_E_ARG;
  memset(o, 0, sizeof(*o));
  o->num_states = t->host.num_states;
  o->num_patterns = t->host.num_patterns;
  o->max_len = t->host.max_len;
  o->min_len = t->host.min_len;
  o->max_depth_full = t->host.max_depth_full;
  o->device_bytes = t->dbytes;
  const auto& ds = t->host.depth_start;
  for (uint32_t d = 0; d <= 8; ++d)
    o->states_to_depth[d] = (d + 1 < ds.size()) ? ds[d + 1] : t->host.num_states;
  o->prefix_k = t->host.pfx_k;
  o->prefix_keys = t->host.pfx_set;
  return PFAC_OK;
}

void pfac_free_table(pfac_table* t) {
  if (!t) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(t->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(t->dmem);
  if (t->cells_mem) (void)hipFree(t->cells_mem);
  (void)hipSetDevice(cur);
  delete t;
}

int pfac_default_plan(const pfac_table* t, uint64_t n, int enc, pfac_plan* out) {
  (void)n;
  if (!t || !out || (enc != PFAC_TEXT_ASCII && enc != PFAC_TEXT_2BIT)) return PFAC_E_ARG;
  if (t->alphabet != 4) {
    // byte tables have one kernel: 1024-thread workgroups, the grid by size
    *out = pfac_plan{1024, 0, 0, PFAC_VARIANT_GLOBAL, PFAC_LEVELS_NONE, PFAC_HASH_NONE,
                     PFAC_WALKS_INLINE, 2048, PFAC_PREFIX_NONE, PFAC_PAIR_NONE};
    return enc == PFAC_TEXT_ASCII ? PFAC_OK : PFAC_E_ARG;
  }
  return resolve_plan(nullptr, t->host, t->device, true, out);
}

}  // extern "C"

namespace pfac {

int prepare_single(const pfac_table* t, uint64_t n, int enc, const pfac_plan* plan,
                          int dev, SinglePrep* P) {
  if (t->alphabet != 4) return PFAC_E_ARG;      // byte tables: pfac_match only
  int rc = resolve_plan(plan, t->host, dev, true, &P->pl);
  if (rc) return rc;
  const pfac_plan& pl = P->pl;
  if (pl.variant == PFAC_VARIANT_GLOBAL_TWO_ARRAYS || pl.variant == PFAC_VARIANT_GLOBAL_MERGED) {
    rc = ensure_cells(t);
    if (rc) return rc;
  }
  const uint32_t tile = pl.tile;
  P->tiles = (n + tile - 1) / tile;
  P->walks = 0;
  ScanParams& sp = P->sp;
  memset(&sp, 0, sizeof(sp));
  fill_table(sp, t, pl);
  sp.halo = pl.variant == PFAC_VARIANT_TILED ? halo_for(t->host.max_len) : 0;
  sp.seg0 = DevSeg{0, 0, (uint32_t)n, 0, 0, (uint16_t)enc, (uint16_t)__builtin_ctz(tile)};
  sp.local_tiles = P->tiles;
  if (pl.variant == PFAC_VARIANT_TILED && pl.walks == PFAC_WALKS_DEFERRED && P->tiles) {
    // every scan wave gets room for a number of walks per tile it will scan
    // (about twice what the filters let through on random-like text; walks
    // beyond it run at once) and walks them after its last tile (the kernel,
    // hence its grid, depends on `defer`: set it first)
    sp.defer = 1;
    ScanFn fn;
    uint32_t lds;
    uint64_t grid;
    rc = scan_shape(sp, pl, true, tile, dev, &fn, &lds, &grid);
    if (rc) return rc;
    const uint64_t nwaves = grid * (pl.block / 64);
    const uint64_t per = std::max<uint64_t>(
        (uint64_t)defer_per_tile(t->host, pl, tile) * ((P->tiles + nwaves - 1) / nwaves), 64);
    sp.wq_cap = (uint32_t)per;
    sp.wq_waves = nwaves;
    P->walks = per * nwaves;
  }
  return PFAC_OK;
}

int enqueue_single(const pfac_table* t, SinglePrep& P, const Scratch& sc, const void* d_text,
                          int32_t* d_match, pfac_hit* d_hits, uint64_t hit_cap,
                          unsigned long long* counters, int dev, hipStream_t stream,
                          bool keep_slots) {
  ScanParams& sp = P.sp;
  sp.text = static_cast<const uint8_t*>(d_text);
  sp.match = d_match;
  sp.tile_hits = sc.tile_hits;
  sp.tile_occ = sc.tile_occ;
  sp.slots = (d_hits || keep_slots) ? sc.slots : nullptr;
  sp.wq = sc.walk;
  sp.pz_dummy = sc.dummy;
  int rc = launch_scan(sp, P.pl, true, P.pl.tile, dev, stream);
  if (rc) return rc;
  FinishParams fp;
  memset(&fp, 0, sizeof(fp));
  fp.hits = d_hits;
  fp.hit_cap = hit_cap;
  fp.single = 1;
  fp.tile = P.pl.tile;
  fp.seg0 = sp.seg0;
  fp.text = sp.text;
  fp.match = d_match;
  fp.tab0 = t->dev;
  return launch_tail(sc, P.tiles, counters, &fp, d_hits != nullptr && hit_cap > 0, stream);
}

int launch_finish_single(const Scratch& sc, uint64_t tiles, uint32_t tile, uint64_t n,
                         unsigned long long* counters, pfac_hit* d_hits, uint64_t hit_cap,
                         const int32_t* match, hipStream_t stream) {
  FinishParams fp;
  memset(&fp, 0, sizeof(fp));
  fp.hits = d_hits;
  fp.hit_cap = hit_cap;
  fp.single = 1;
  fp.tile = tile;
  fp.seg0 = DevSeg{0, 0, (uint32_t)n, 0, 0, 0, (uint16_t)__builtin_ctz(tile)};
  fp.match = match;
  return launch_tail(sc, tiles, counters, &fp, d_hits != nullptr && hit_cap > 0, stream);
}

bool device_ok(int dev) { return device_info(dev).ok; }
uint32_t device_cus(int dev) { return (uint32_t)device_info(dev).cus; }

int launch_zero(unsigned long long* p, uint32_t n, hipStream_t stream) {
  hipLaunchKernelGGL(pfac_zero_kernel, dim3(1), dim3(1024), 0, stream, p, n);
  return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
}

}  // namespace pfac

extern "C" {

int pfac_match(const pfac_table* t, const void* d_text, uint64_t n, int enc, int32_t* d_match,
               pfac_hit* d_hits, uint64_t hit_cap, uint64_t* d_counters, const pfac_plan* plan,
               void* stream_) {
  if (!t || !d_counters || (n && !d_text) || n >= (1ull << 32)) return PFAC_E_ARG;
  if (enc != PFAC_TEXT_ASCII && enc != PFAC_TEXT_2BIT) return PFAC_E_ARG;
  if (d_hits == nullptr) hit_cap = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFAC_E_NODEV;
  if (dev != t->device) return PFAC_E_ARG;
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  unsigned long long* counters = reinterpret_cast<unsigned long long*>(d_counters);
  if (t->alphabet != 4) {
    if (enc != PFAC_TEXT_ASCII) return PFAC_E_ARG;      // texts of a byte table are bytes
    return match_bytes(t, d_text, n, d_match, d_hits, hit_cap, counters, plan, dev, stream);
  }
  SinglePrep P;
  int rc = prepare_single(t, n, enc, plan, dev, &P);
  if (rc) return rc;
  if (P.tiles == 0) {
    hipLaunchKernelGGL(pfac_zero_kernel, dim3(1), dim3(64), 0, stream, counters, 2u);
    return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
  }
  Workspace* ws = get_workspace(dev, stream);
  if (!ws) return PFAC_E_NOMEM;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    rc = ensure_scratch(ws, P.tiles, false, P.walks, stream);
  }
  if (rc) return rc;
  return enqueue_single(t, P, ws->sc, d_text, d_match, d_hits, hit_cap, counters, dev, stream);
}

}  // extern "C"


namespace pfac {

// Host-side layout of a batch: per-table plans; per text its tile size
// (from the plan, or by length: 256 up to kShortText bases, else 1024), its
// first tile among the tiles of the call (text order) and the first of its
// work items; launch groups of (table, tile size), each a contiguous run of
// work items; and the byte layout of the device copy (descriptors | tile
// prefix | item starts | table views).
constexpr uint64_t kShortText = 512;

struct LaunchGroup {
  uint32_t table;
  uint32_t tile;
  uint64_t first_item, items;
  uint64_t walks;        // deferred-walk entries it needs (0: walks inline)
  uint32_t wq_cap;
  uint64_t wq_waves;
};

struct BatchLayout {
  std::vector<const pfac_table*> tables;
  std::vector<pfac_plan> plans;
  std::vector<DevSeg> segs;
  std::vector<uint64_t> tile_prefix;
  std::vector<uint64_t> item_start;
  std::vector<LaunchGroup> groups;
  uint64_t o_segs = 0, o_tp = 0, o_is = 0, o_tab = 0, bytes = 0, tiles = 0, walks = 0;
  uint32_t num_texts = 0;
  uint64_t text_extent = 0;      // bytes of d_text_base the texts reach
  uint64_t match_extent = 0;     // int32 elements of d_match_base they reach
};

static uint32_t text_tile(const pfac_plan& pl, uint64_t n, bool fold_short) {
  if (global_variant(pl.variant)) return kTileBatch;
  if (pl.tile) return pl.tile;
  // short texts: 256-position tiles (a 150-base read fills 59 % of one);
  // longer ones 2048 like a one-text call, the fixed cost of a tile spread
  // over more positions (a text wastes half a tile at its end on average).
  // A few short texts among long ones of the same table go with the long
  // ones: their own launch (about 15 us) costs more than a few thousand
  // mostly empty 2048-position tiles
  return (n <= kShortText && !fold_short) ? kTileShort : kTileSingle;
}

// Short texts of a table are folded into its long texts' tiles when they
// would need fewer 256-position tiles than this.
constexpr uint64_t kFoldShort = 4096;

static int layout_batch(const pfac_table* const* tables, uint32_t num_tables,
                        const pfac_text_desc* descs, uint32_t num_texts, const pfac_plan* plan,
                        int dev, BatchLayout* L) {
  if (!tables || num_tables == 0 || (num_texts && !descs) || num_texts >= (1u << 31))
    return PFAC_E_ARG;
  for (uint32_t i = 0; i < num_tables; ++i)
    if (!tables[i] || tables[i]->device != dev || tables[i]->alphabet != 4) return PFAC_E_ARG;
  for (uint32_t s = 0; s < num_texts; ++s) {
    const pfac_text_desc& d = descs[s];
    if (d.n >= (1ull << 32) || d.table >= num_tables ||
        (d.enc != PFAC_TEXT_ASCII && d.enc != PFAC_TEXT_2BIT))
      return PFAC_E_ARG;
  }
  L->tables.assign(tables, tables + num_tables);
  L->plans.resize(num_tables);
  for (uint32_t i = 0; i < num_tables; ++i) {
    const int rc = resolve_plan(plan, tables[i]->host, dev, false, &L->plans[i]);
    if (rc) return rc;
  }
  // per table: short and long texts, for folding a few short ones in
  std::vector<uint64_t> nshort(num_tables, 0), nlong(num_tables, 0);
  for (uint32_t s = 0; s < num_texts; ++s) {
    if (descs[s].n == 0) continue;
    if (descs[s].n <= kShortText) ++nshort[descs[s].table];
    else ++nlong[descs[s].table];
  }
  L->num_texts = num_texts;
  L->segs.resize(num_texts);
  L->tile_prefix.assign(num_texts + 1, 0);
  L->text_extent = 0;
  L->match_extent = 0;
  for (uint32_t s = 0; s < num_texts; ++s) {
    const pfac_text_desc& d = descs[s];
    const uint32_t tile = text_tile(L->plans[d.table], d.n,
                                    nlong[d.table] > 0 && nshort[d.table] < kFoldShort);
    const uint64_t nt = (d.n + tile - 1) / tile;
    L->tile_prefix[s + 1] = L->tile_prefix[s] + nt;
    if (L->tile_prefix[s + 1] >= (1ull << 32)) return PFAC_E_ARG;
    L->segs[s] = DevSeg{d.text_offset, d.match_offset, (uint32_t)d.n,
                        (uint32_t)L->tile_prefix[s], d.table, (uint16_t)d.enc,
                        (uint16_t)__builtin_ctz(tile)};
    if (d.n) {
      const uint64_t bytes = d.enc == PFAC_TEXT_ASCII ? d.n : (d.n + 3) / 4;
      L->text_extent = std::max(L->text_extent, d.text_offset + bytes);
      L->match_extent = std::max(L->match_extent, d.match_offset + d.n);
    }
  }
  L->tiles = L->tile_prefix[num_texts];
  // launch groups: per table, per tile size, texts in text order
  L->item_start.assign(num_texts, 0);
  L->groups.clear();
  uint64_t item = 0;
  static const uint32_t kTiles[3] = {kTileShort, kTileBatch, kTileSingle};
  for (uint32_t g = 0; g < num_tables; ++g) {
    for (uint32_t tile : kTiles) {
      LaunchGroup G{g, tile, item, 0, 0, 0, 0};
      for (uint32_t s = 0; s < num_texts; ++s) {
        if (descs[s].table != g || descs[s].n == 0 || (1u << L->segs[s].tile_shift) != tile)
          continue;
        L->item_start[s] = item;
        const uint64_t nt = L->tile_prefix[s + 1] - L->tile_prefix[s];
        item += nt;
        G.items += nt;
      }
      if (G.items) L->groups.push_back(G);
    }
  }
  uint64_t off = 0;
  L->o_segs = off; off = al256(off + num_texts * sizeof(DevSeg));
  L->o_tp = off; off = al256(off + (num_texts + 1) * 8);
  L->o_is = off; off = al256(off + num_texts * 8);
  L->o_tab = off; off = al256(off + num_tables * sizeof(DevTable));
  L->bytes = off;
  // deferred walks: the room of the largest group (groups run one after
  // another on the stream and share it)
  L->walks = 0;
  for (LaunchGroup& G : L->groups) {
    const pfac_plan& pl = L->plans[G.table];
    if (pl.variant != PFAC_VARIANT_TILED || pl.walks != PFAC_WALKS_DEFERRED) continue;
    ScanParams sp;
    memset(&sp, 0, sizeof(sp));
    fill_table(sp, L->tables[G.table], pl);
    sp.halo = halo_for(L->tables[G.table]->host.max_len);
    sp.local_tiles = G.items;
    sp.defer = 1;
    ScanFn fn;
    uint32_t lds;
    uint64_t grid;
    const int rc = scan_shape(sp, pl, false, G.tile, dev, &fn, &lds, &grid);
    if (rc) return rc;
    const uint64_t nwaves = grid * (pl.block / 64);
    const uint64_t per = std::max<uint64_t>(
        (uint64_t)defer_per_tile(L->tables[G.table]->host, pl, G.tile) *
            ((G.items + nwaves - 1) / nwaves), 64);
    G.wq_cap = (uint32_t)per;
    G.wq_waves = nwaves;
    G.walks = per * nwaves;
    L->walks = std::max(L->walks, G.walks);
  }
  return PFAC_OK;
}

static void fill_batch(const BatchLayout& L, uint8_t* host) {
  memset(host, 0, L.bytes);
  if (L.num_texts) {
    memcpy(host + L.o_segs, L.segs.data(), L.num_texts * sizeof(DevSeg));
    memcpy(host + L.o_is, L.item_start.data(), L.num_texts * 8);
  }
  memcpy(host + L.o_tp, L.tile_prefix.data(), L.tile_prefix.size() * 8);
  for (size_t i = 0; i < L.tables.size(); ++i)
    memcpy(host + L.o_tab + i * sizeof(DevTable), &L.tables[i]->dev, sizeof(DevTable));
}

// The work items of every launch group, from the device copy of the layout.
static int enqueue_items(const BatchLayout& L, const Scratch& sc, const uint8_t* db,
                         hipStream_t stream) {
  if (L.num_texts == 0 || L.tiles == 0) return PFAC_OK;
  hipLaunchKernelGGL(pfac_items_kernel, dim3((L.num_texts + 3) / 4), dim3(256), 0, stream,
                     reinterpret_cast<const DevSeg*>(db + L.o_segs),
                     reinterpret_cast<const uint64_t*>(db + L.o_is), L.num_texts, sc.items);
  return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
}

// Enqueue the kernels of a batch whose layout and work items are on the
// device: one scan launch per group, then the finish and per-text totals.
// Kernel launches only (no allocation, copy or memset).
static int enqueue_batch(const BatchLayout& L, const Scratch& sc, const uint8_t* db,
                         const void* d_text_base, int32_t* d_match_base,
                         pfac_batch_hit* d_hits, uint64_t hit_cap, unsigned long long* counters,
                         int dev, hipStream_t stream) {
  if (L.tiles == 0) {
    hipLaunchKernelGGL(pfac_zero_kernel, dim3(1), dim3(256), 0, stream, counters,
                       2u + 2u * L.num_texts);
    return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
  }
  for (const LaunchGroup& G : L.groups) {
    ScanParams sp;
    memset(&sp, 0, sizeof(sp));
    fill_table(sp, L.tables[G.table], L.plans[G.table]);
    sp.halo = L.plans[G.table].variant == PFAC_VARIANT_TILED
                  ? halo_for(L.tables[G.table]->host.max_len) : 0;
    sp.segs = reinterpret_cast<const DevSeg*>(db + L.o_segs);
    sp.items = sc.items + G.first_item;
    sp.local_tiles = G.items;
    sp.text = static_cast<const uint8_t*>(d_text_base);
    sp.match = d_match_base;
    sp.tile_hits = sc.tile_hits;
    sp.tile_occ = sc.tile_occ;
    sp.slots = d_hits ? sc.slots : nullptr;
    if (G.walks) {
      sp.defer = 1;
      sp.wq = sc.walk;
      sp.wq_cap = G.wq_cap;
      sp.wq_waves = G.wq_waves;
    }
    sp.pz_dummy = sc.dummy;
    const int rc = launch_scan(sp, L.plans[G.table], false, G.tile, dev, stream);
    if (rc) return rc;
  }
  FinishParams fp;
  memset(&fp, 0, sizeof(fp));
  fp.hits = d_hits;
  fp.hit_cap = hit_cap;
  fp.single = 0;
  fp.nsegs = L.num_texts;
  fp.segs = reinterpret_cast<const DevSeg*>(db + L.o_segs);
  fp.tile_prefix = reinterpret_cast<const uint64_t*>(db + L.o_tp);
  fp.text = static_cast<const uint8_t*>(d_text_base);
  fp.match = d_match_base;
  fp.tables = reinterpret_cast<const DevTable*>(db + L.o_tab);
  const int rc = launch_tail(sc, L.tiles, counters, &fp, d_hits != nullptr && hit_cap > 0,
                             stream);
  if (rc) return rc;
  hipLaunchKernelGGL(pfac_text_totals_kernel, dim3((L.num_texts + 3) / 4), dim3(256), 0, stream,
                     sc.tile_hits, sc.tile_occ, fp.tile_prefix, L.num_texts, counters + 2);
  return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
}

static bool text_base_ok(const BatchLayout& L, const void* d_text_base) {
  return d_text_base != nullptr || L.text_extent == 0;
}

}  // namespace pfac

struct pfac_batch {
  int device = 0;
  pfac::BatchLayout layout;
  pfac::Workspace ws;      // owned scratch and device copy of the layout
};

extern "C" {

int pfac_match_batch(const pfac_table* const* tables, uint32_t num_tables,
                     const pfac_text_desc* descs, uint32_t num_texts, const void* d_text_base,
                     int32_t* d_match_base, pfac_batch_hit* d_hits, uint64_t hit_cap,
                     uint64_t* d_counters, const pfac_plan* plan, void* stream_) {
  if (!d_counters) return PFAC_E_ARG;
  if (d_hits == nullptr) hit_cap = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFAC_E_NODEV;
  BatchLayout L;
  int rc = layout_batch(tables, num_tables, descs, num_texts, plan, dev, &L);
  if (rc) return rc;
  if (!text_base_ok(L, d_text_base)) return PFAC_E_ARG;
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  unsigned long long* counters = reinterpret_cast<unsigned long long*>(d_counters);
  if (L.tiles == 0) return enqueue_batch(L, Scratch(), nullptr, d_text_base, d_match_base, d_hits,
                                         hit_cap, counters, dev, stream);
  Workspace* ws = get_workspace(dev, stream);
  if (!ws) return PFAC_E_NOMEM;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    rc = ensure_scratch(ws, L.tiles, true, L.walks, stream);
    if (!rc) rc = ensure_batch(ws, L.bytes, stream);
  }
  if (rc) return rc;
  fill_batch(L, ws->stage);
  if (hipMemcpyAsync(ws->batch, ws->stage, L.bytes, hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      hipEventRecord(ws->staged, stream) != hipSuccess)
    return PFAC_E_HIP;
  ws->staged_pending = true;
  const uint8_t* db = static_cast<const uint8_t*>(ws->batch);
  rc = enqueue_items(L, ws->sc, db, stream);
  if (rc) return rc;
  return enqueue_batch(L, ws->sc, db, d_text_base, d_match_base, d_hits, hit_cap, counters, dev,
                       stream);
}

int pfac_batch_create(const pfac_table* const* tables, uint32_t num_tables,
                      const pfac_text_desc* descs, uint32_t num_texts, const pfac_plan* plan,
                      pfac_batch** out) {
  if (!out) return PFAC_E_ARG;
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFAC_E_NODEV;
  pfac_batch* b = new (std::nothrow) pfac_batch();
  if (!b) return PFAC_E_NOMEM;
  b->device = dev;
  int rc = layout_batch(tables, num_tables, descs, num_texts, plan, dev, &b->layout);
  if (!rc && b->layout.tiles) {
    rc = ensure_scratch(&b->ws, b->layout.tiles, true, b->layout.walks, nullptr);
    if (!rc) rc = ensure_batch(&b->ws, b->layout.bytes, nullptr);
    if (!rc) {
      fill_batch(b->layout, b->ws.stage);
      if (hipMemcpy(b->ws.batch, b->ws.stage, b->layout.bytes, hipMemcpyHostToDevice) !=
          hipSuccess)
        rc = PFAC_E_HIP;
    }
    if (!rc) rc = enqueue_items(b->layout, b->ws.sc, static_cast<const uint8_t*>(b->ws.batch),
                                nullptr);
    if (!rc && hipStreamSynchronize(nullptr) != hipSuccess) rc = PFAC_E_HIP;
  }
  if (rc) {
    free_workspace(&b->ws);
    delete b;
    return rc;
  }
  *out = b;
  return PFAC_OK;
}

int pfac_batch_launch(pfac_batch* b, const void* d_text_base, int32_t* d_match_base,
                      pfac_batch_hit* d_hits, uint64_t hit_cap, uint64_t* d_counters,
                      void* stream) {
  if (!b || !d_counters) return PFAC_E_ARG;
  if (d_hits == nullptr) hit_cap = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFAC_E_NODEV;
  if (dev != b->device || !text_base_ok(b->layout, d_text_base)) return PFAC_E_ARG;
  return enqueue_batch(b->layout, b->ws.sc, static_cast<const uint8_t*>(b->ws.batch), d_text_base,
                       d_match_base, d_hits, hit_cap,
                       reinterpret_cast<unsigned long long*>(d_counters), dev,
                       static_cast<hipStream_t>(stream));
}

int pfac_batch_info(const pfac_batch* b, uint64_t* text_extent, uint64_t* match_extent,
                    uint64_t* tiles) {
  if (!b) return PFAC_E_ARG;
  if (text_extent) *text_extent = b->layout.text_extent;
  if (match_extent) *match_extent = b->layout.match_extent;
  if (tiles) *tiles = b->layout.tiles;
  return PFAC_OK;
}

void pfac_batch_free(pfac_batch* b) {
  if (!b) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  free_workspace(&b->ws);
  (void)hipSetDevice(cur);
  delete b;
}

}  // extern "C"
