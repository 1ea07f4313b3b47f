// PFAC matching kernels for gfx950 and the C ABI around them.
//
// Semantics (paper Sec. IV): every start position of the text walks the
// failure-less goto trie from the root, one base per step, stops at the
// first missing transition, and reports the last (= longest) pattern it
// passed.  The paper launches one thread per character with the text staged
// in shared memory and the table read through the texture cache (Sec. V.B,
// V.C, Sec. VII).  The gfx950 design keeps the walk and reorganises the
// memory side:
//   * text: 16-byte coalesced loads of a tile plus a halo of max_len-1
//     bases, converted once to 2 bits per base (plus an "invalid" bit) in LDS;
//   * table: the first K levels of every walk are one LDS lookup of a root
//     jump table indexed by the K-base window (K = 4..7); deeper levels read
//     the breadth-first numbered next-state table, optionally with its
//     hot prefix staged in LDS, the rest served by L2 / Infinity Cache;
//   * outputs: dense int32 per position with 16-byte non-temporal stores,
//     and a position-ordered hit list built with a block scan plus a
//     decoupled look-back across tiles (tiles are taken from an atomic
//     ticket, so every tile's predecessors are already running);
//   * the launch is persistent: workgroups loop over tiles (and over the
//     texts of a batch) until the ticket passes the last tile.
#include <hip/hip_runtime.h>
#include <string.h>

#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "pfac_internal.h"

namespace pfac {

constexpr uint32_t kPPT = 16;               // start positions per thread per tile
constexpr uint32_t kGroups = kPPT / 4;      // groups of 4 consecutive positions
constexpr uint32_t kMaxHaloLds = 4096;      // longest halo staged in LDS (bases)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

struct DevSeg {
  uint64_t text_off;
  uint64_t n;
  uint64_t match_off;
  uint32_t table;
  uint32_t enc;
};
static_assert(sizeof(DevSeg) == sizeof(pfac_text_desc), "descriptor layout");

// Look-back status word: [63:42] launch epoch, [41:40] flag, [39:0] value.
constexpr uint32_t kEpochBits = 22;
constexpr uint64_t kValMask = (1ull << 40) - 1;
constexpr unsigned long long kFlagAgg = 1ull << 40;
constexpr unsigned long long kFlagIncl = 2ull << 40;

struct KParams {
  const DevTable* tables;         // device array, indexed by DevSeg::table (batch)
  const DevSeg* segs;             // device array (batch)
  const uint64_t* tile_prefix;    // device [nsegs+1] first tile of each text (batch)
  uint32_t nsegs;
  uint32_t single;                // 1: one text, described by seg0/tab0
  uint64_t total_tiles;
  const uint8_t* text;
  int32_t* match;
  void* hits;
  uint64_t hit_cap;
  unsigned long long* counters;   // [2]
  unsigned long long* seg_counters;  // [2*nsegs] (batch) or nullptr
  uint32_t* ticket;
  unsigned long long* status;
  uint32_t epoch;
  uint32_t K;
  uint32_t hot;
  uint32_t halo;                  // staged halo, multiple of 64 bases
  DevSeg seg0;
  DevTable tab0;
};

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ int ascii_code(uint32_t b) {
  return b == 'A' ? 0 : b == 'C' ? 1 : b == 'G' ? 2 : b == 'T' ? 3 : -1;
}

// Four ASCII bytes -> four 2-bit codes (low byte first, 8 bits) and a 4-bit
// "not a base" mask.  code = ((b >> 1) ^ (b >> 2)) & 3 maps A,C,G,T to
// 0,1,2,3; a byte is a base iff re-encoding its code gives the byte back.
__device__ __forceinline__ void ascii4(uint32_t x, uint32_t& code8, uint32_t& inv4) {
  const uint32_t cb = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
  const uint32_t expect = __builtin_amdgcn_perm(0u, 0x54474341u, cb);  // bytes 'A','C','G','T'
  const uint32_t t = x ^ expect;
  const uint32_t nz = (((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t) & 0x80808080u;
  inv4 = ((nz >> 7) * 0x01020408u) >> 24;
  code8 = (cb * 0x01041040u) >> 24;
}

template <int BLOCK>
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long* red) {
  #pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  unsigned long long s = 0;
  #pragma unroll
  for (int i = 0; i < BLOCK / 64; ++i) s += red[i];
  return s;
}

// Exclusive block scan of a small per-thread count; *total gets the sum.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = v;
  #pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  __syncthreads();
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
  #pragma unroll
  for (int i = 0; i < BLOCK / 64; ++i) {
    const uint32_t s = wsum[i];
    before += (i < w) ? s : 0u;
    all += s;
  }
  *total = all;
  return before + inc - v;
}

// Decoupled look-back (run by all 64 lanes of one wave): publishes this
// tile's aggregate, sums predecessors back to the nearest inclusive prefix,
// publishes the inclusive prefix and returns the exclusive one.
__device__ uint64_t lookback(unsigned long long* status, uint64_t tile, uint64_t agg,
                             uint32_t epoch) {
  const int lane = threadIdx.x & 63;
  const unsigned long long tag = (unsigned long long)epoch << 42;
  if (tile == 0) {
    if (lane == 0)
      __hip_atomic_store(&status[0], tag | kFlagIncl | (agg & kValMask), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane == 0)
    __hip_atomic_store(&status[tile], tag | kFlagAgg | (agg & kValMask), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  uint64_t prefix = 0;
  int64_t base = (int64_t)tile - 1;
  for (;;) {
    const int64_t idx = base - lane;
    unsigned long long v = 0;
    uint32_t flag = 2;
    if (idx >= 0) {
      v = __hip_atomic_load(&status[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      flag = ((uint32_t)(v >> 42) == epoch) ? (uint32_t)((v >> 40) & 3) : 0u;
    }
    const uint64_t incl = __ballot(flag == 2);
    const uint64_t notready = __ballot(flag == 0);
    const int first = incl ? __builtin_ctzll(incl) : 64;
    const uint64_t upto = (first >= 63) ? ~0ull : ((2ull << first) - 1);
    if (notready & upto) {
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    unsigned long long val = (lane <= first) ? (v & kValMask) : 0ull;
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) val += __shfl_xor(val, o, 64);
    prefix += val;
    if (first < 64) break;
    base -= 64;
  }
  if (lane == 0)
    __hip_atomic_store(&status[tile], tag | kFlagIncl | ((prefix + agg) & kValMask),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return prefix;
}

// One base of the text for the global-memory variant (out of range = invalid).
__device__ __forceinline__ int global_base(const uint8_t* t, uint64_t n, uint32_t enc,
                                           uint64_t q) {
  if (q >= n) return -1;
  if (enc == PFAC_TEXT_ASCII) return ascii_code(t[q]);
  return (t[q >> 2] >> (2 * (q & 3))) & 3;
}

// Continue one walk from state s at text index q (tile-local for LDS text).
// s == 0 means "at the root": the root row is row 0 and no edge points back
// to it, so the loop needs no special case.
template <bool GLOBAL>
__device__ __forceinline__ void walk(uint32_t s, uint32_t q, const uint32_t* __restrict__ pk,
                                     const uint32_t* __restrict__ iv,
                                     const uint32_t* __restrict__ hot_l, uint32_t hot,
                                     const DevTable& tab, const uint8_t* gtext, uint64_t gn,
                                     uint32_t genc, uint64_t gq0, int32_t& best,
                                     unsigned long long& occ) {
  for (;;) {
    uint32_t c;
    if (GLOBAL) {
      const int b = global_base(gtext, gn, genc, gq0 + q);
      if (b < 0) break;
      c = (uint32_t)b;
    } else {
      if ((iv[q >> 5] >> (q & 31)) & 1u) break;
      c = (pk[q >> 4] >> (2 * (q & 15))) & 3u;
    }
    const uint32_t e = (s < hot) ? hot_l[s * 4 + c] : tab.next[(uint64_t)s * 4 + c];
    if (e == 0) break;
    s = e & kStateMask;
    if (e & kFinalBit) {
      const OutEntry o = tab.out[s];
      best = o.pid;
      occ += o.mult;
    }
    ++q;
  }
}

// Stage the text of [t0, t0+span) of one text into LDS as 2-bit codes (16
// per word) plus an invalid bit per base (32 per word).  Bases past the end
// of the text are invalid.
template <int BLOCK>
__device__ __forceinline__ void stage_text(const uint8_t* __restrict__ t, uint64_t n, uint32_t enc,
                                           uint64_t t0, uint32_t span, uint32_t* pk,
                                           uint32_t* iv) {
  const uint32_t nwords = span / 16;
  uint16_t* iv16 = reinterpret_cast<uint16_t*>(iv);
  if (enc == PFAC_TEXT_ASCII) {
    const bool aligned = ((reinterpret_cast<uintptr_t>(t) & 15) == 0);
    for (uint32_t c = threadIdx.x; c < nwords; c += BLOCK) {
      const uint64_t g = t0 + 16ull * c;
      uint32_t w[4];
      if (aligned && g + 16 <= n) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(t + g));
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
      } else {
        #pragma unroll
        for (int k = 0; k < 4; ++k) {
          uint32_t x = 0;
          #pragma unroll
          for (int b = 0; b < 4; ++b) {
            const uint64_t q = g + 4 * k + b;
            x |= (uint32_t)(q < n ? t[q] : 0u) << (8 * b);
          }
          w[k] = x;
        }
      }
      uint32_t packed = 0, inv = 0;
      #pragma unroll
      for (int k = 0; k < 4; ++k) {
        uint32_t c8, i4;
        ascii4(w[k], c8, i4);
        packed |= c8 << (8 * k);
        inv |= i4 << (4 * k);
      }
      pk[c] = packed;
      iv16[c] = (uint16_t)inv;
    }
  } else {
    const uint8_t* tb = t;  // byte k holds bases 4k..4k+3
    const bool aligned = ((reinterpret_cast<uintptr_t>(tb) & 15) == 0);
    const uint32_t nchunks = span / 64;   // 16 bytes = 64 bases
    for (uint32_t c = threadIdx.x; c < nchunks; c += BLOCK) {
      const uint64_t g = t0 + 64ull * c;
      uint32_t w[4];
      uint32_t inv[4] = {0, 0, 0, 0};
      if (aligned && g + 64 <= n) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(tb + g / 4));
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
      } else {
        #pragma unroll
        for (int k = 0; k < 4; ++k) {
          uint32_t x = 0, m = 0;
          for (int b = 0; b < 16; ++b) {
            const uint64_t q = g + 16 * k + b;
            if (q < n) x |= (uint32_t)((tb[q >> 2] >> (2 * (q & 3))) & 3u) << (2 * b);
            else m |= 1u << b;
          }
          w[k] = x;
          inv[k] = m;
        }
      }
      #pragma unroll
      for (int k = 0; k < 4; ++k) {
        pk[4 * c + k] = w[k];
        iv16[4 * c + k] = (uint16_t)inv[k];
      }
    }
  }
  // sentinel words after the staged span: no bases, all invalid
  if (threadIdx.x < 2) {
    pk[nwords + threadIdx.x] = 0;
    iv[span / 32 + threadIdx.x] = 0xFFFFFFFFu;
  }
}

template <int BLOCK, bool GLOBAL>
__global__ __launch_bounds__(BLOCK) void pfac_kernel(KParams p) {
  extern __shared__ uint32_t lds[];
  constexpr uint32_t TILE = BLOCK * kPPT;
  __shared__ uint32_t s_tile_lo, s_seg;
  __shared__ unsigned long long s_red[BLOCK / 64];
  __shared__ uint32_t s_wsum[BLOCK / 64];
  __shared__ unsigned long long s_prefix;

  const uint32_t K = GLOBAL ? 0u : p.K;
  const uint32_t hot = GLOBAL ? 0u : p.hot;
  const uint32_t jsize = K ? (1u << (2 * K)) : 0u;
  const uint32_t span = TILE + p.halo;
  uint32_t* jump_l = lds;
  uint32_t* hot_l = lds + jsize;
  uint32_t* pk = hot_l + 4 * hot;
  uint32_t* iv = pk + span / 16 + 2;

  uint32_t loaded_table = 0xFFFFFFFFu;
  unsigned long long occ_acc = 0, hits_acc = 0;  // single-text totals of this workgroup

  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t tk = atomicAdd(p.ticket, 1u);
      s_tile_lo = tk;
      uint32_t sg = 0;
      if (!p.single && tk < p.total_tiles) {
        // last text whose first tile is <= tk (texts with no tiles are skipped)
        uint32_t lo = 0, hi = p.nsegs;   // invariant: prefix[lo] <= tk < prefix[hi]
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (p.tile_prefix[mid] <= tk) lo = mid; else hi = mid;
        }
        sg = lo;
      }
      s_seg = sg;
    }
    __syncthreads();
    const uint64_t tile = s_tile_lo;
    if (tile >= p.total_tiles) break;
    const uint32_t segi = s_seg;
    const DevSeg seg = p.single ? p.seg0 : p.segs[segi];
    const uint64_t ts = p.single ? tile : tile - p.tile_prefix[segi];
    const DevTable tab = p.single ? p.tab0 : p.tables[seg.table];
    const uint64_t t0 = ts * TILE;
    const uint64_t n = seg.n;
    const uint8_t* text = p.text + seg.text_off;

    if (!GLOBAL) {
      if (seg.table != loaded_table) {
        // root jump table and hot rows of this trie into LDS
        const uint4* js = reinterpret_cast<const uint4*>(tab.jump);
        uint4* jd = reinterpret_cast<uint4*>(jump_l);
        for (uint32_t i = threadIdx.x; i < jsize / 4; i += BLOCK) jd[i] = js[i];
        const uint32_t hrows = min(hot, tab.num_states);
        for (uint32_t i = threadIdx.x; i < 4 * hot; i += BLOCK)
          hot_l[i] = (i < 4 * hrows) ? tab.next[i] : 0u;
        loaded_table = seg.table;
      }
      stage_text<BLOCK>(text, n, seg.enc, t0, span, pk, iv);
      __syncthreads();
    }

    // ---- walks: first K levels from the jump table, then the deep loop
    int32_t best[kPPT];
    uint32_t st[kPPT];
    uint32_t pend = 0, slow = 0;
    unsigned long long occ = 0;
    const uint32_t kmask = (1u << K) - 1u;
    const uint32_t xmask = (1u << (2 * K)) - 1u;
    #pragma unroll
    for (uint32_t g = 0; g < kGroups; ++g) {
      const uint32_t q0 = g * 4 * BLOCK + 4 * threadIdx.x;
      uint64_t win = 0, ivw = 0;
      if (!GLOBAL && K) {
        win = ((uint64_t)pk[(q0 >> 4) + 1] << 32 | pk[q0 >> 4]) >> (2 * (q0 & 15));
        ivw = ((uint64_t)iv[(q0 >> 5) + 1] << 32 | iv[q0 >> 5]) >> (q0 & 31);
      }
      #pragma unroll
      for (uint32_t r = 0; r < 4; ++r) {
        const uint32_t i = g * 4 + r;
        best[i] = 0;
        st[i] = 0;
        if (!GLOBAL && K && ((uint32_t)(ivw >> r) & kmask) == 0) {
          const uint32_t x = (uint32_t)(win >> (2 * r)) & xmask;
          const uint32_t e = jump_l[x];
          st[i] = e & kStateMask;
          if (e & kFinalBit) {
            const OutEntry o = tab.jres[x];
            best[i] = o.pid;
            occ += o.mult;
          }
          if (st[i]) pend |= 1u << i;
        } else {
          pend |= 1u << i;
          slow |= 1u << i;
        }
      }
    }
    #pragma unroll
    for (uint32_t i = 0; i < kPPT; ++i) {
      if ((pend >> i) & 1u) {
        const uint32_t q = (i / 4) * 4 * BLOCK + 4 * threadIdx.x + (i % 4) +
                           (((slow >> i) & 1u) ? 0u : K);
        walk<GLOBAL>(st[i], q, pk, iv, hot_l, hot, tab, text, n, seg.enc, t0, best[i], occ);
      }
    }

    // ---- dense output: 16-byte non-temporal stores of 4 consecutive positions
    uint32_t hc[kGroups];
    uint32_t th_hits = 0;
    int32_t* mrow = p.match ? p.match + seg.match_off : nullptr;
    const bool maligned = mrow && ((reinterpret_cast<uintptr_t>(mrow) & 15) == 0);
    #pragma unroll
    for (uint32_t g = 0; g < kGroups; ++g) {
      const uint64_t pos = t0 + g * 4 * BLOCK + 4 * threadIdx.x;
      hc[g] = (best[4 * g] != 0) + (best[4 * g + 1] != 0) + (best[4 * g + 2] != 0) +
              (best[4 * g + 3] != 0);
      th_hits += hc[g];
      if (mrow) {
        if (maligned && pos + 4 <= n) {
          const i32x4 v = {best[4 * g], best[4 * g + 1], best[4 * g + 2], best[4 * g + 3]};
          __builtin_nontemporal_store(v, reinterpret_cast<i32x4*>(mrow + pos));
        } else {
          #pragma unroll
          for (uint32_t r = 0; r < 4; ++r)
            if (pos + r < n) mrow[pos + r] = best[4 * g + r];
        }
      }
    }

    // ---- tile totals, ordered hit list
    const unsigned long long tile_hits = block_sum_u64<BLOCK>(th_hits, s_red);
    if (p.single) {
      hits_acc += tile_hits;
      occ_acc += occ;
    } else {
      const unsigned long long tile_occ = block_sum_u64<BLOCK>(occ, s_red);
      if (threadIdx.x == 0) {
        if (tile_hits) {
          atomicAdd(&p.counters[0], tile_hits);
          atomicAdd(&p.seg_counters[2 * segi], tile_hits);
        }
        if (tile_occ) {
          atomicAdd(&p.counters[1], tile_occ);
          atomicAdd(&p.seg_counters[2 * segi + 1], tile_occ);
        }
      }
    }
    if (p.hits) {
      if (threadIdx.x < 64) {
        const uint64_t pre = lookback(p.status, tile, tile_hits, p.epoch);
        if (threadIdx.x == 0) s_prefix = pre;
      }
      __syncthreads();
      if (tile_hits) {
        uint64_t off = s_prefix;
        #pragma unroll
        for (uint32_t g = 0; g < kGroups; ++g) {
          uint32_t tot;
          const uint32_t ex = block_excl_scan<BLOCK>(hc[g], s_wsum, &tot);
          uint64_t o = off + ex;
          #pragma unroll
          for (uint32_t r = 0; r < 4; ++r) {
            const int32_t b = best[4 * g + r];
            if (b) {
              if (o < p.hit_cap) {
                const uint32_t pos = (uint32_t)(t0 + g * 4 * BLOCK + 4 * threadIdx.x + r);
                if (p.single) {
                  pfac_hit h; h.pos = pos; h.pid = b;
                  reinterpret_cast<pfac_hit*>(p.hits)[o] = h;
                } else {
                  pfac_batch_hit h; h.text = segi; h.pos = pos; h.pid = b;
                  reinterpret_cast<pfac_batch_hit*>(p.hits)[o] = h;
                }
              }
              ++o;
            }
          }
          off += tot;
        }
      }
    }
  }

  if (p.single) {
    // hits_acc is already a workgroup total (same value in every thread)
    const unsigned long long o = block_sum_u64<BLOCK>(occ_acc, s_red);
    if (threadIdx.x == 0) {
      if (hits_acc) atomicAdd(&p.counters[0], hits_acc);
      if (o) atomicAdd(&p.counters[1], o);
    }
  }
}

// Zero the counters and the ticket; for a batch also compute the first
// tile of every text (one workgroup).
__global__ __launch_bounds__(1024) void pfac_prep_kernel(const DevSeg* segs, uint32_t nsegs,
                                                         uint32_t tile, uint64_t* tile_prefix,
                                                         unsigned long long* counters,
                                                         unsigned long long* seg_counters,
                                                         uint32_t* ticket) {
  __shared__ uint64_t wsum[16];
  __shared__ uint64_t carry;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) {
    counters[0] = 0;
    counters[1] = 0;
    *ticket = 0;
    carry = 0;
  }
  if (seg_counters)
    for (uint32_t i = threadIdx.x; i < 2 * nsegs; i += 1024) seg_counters[i] = 0;
  if (!tile_prefix) return;
  __syncthreads();
  for (uint32_t b = 0; b < nsegs; b += 1024) {
    const uint32_t i = b + threadIdx.x;
    const uint64_t v = (i < nsegs) ? (segs[i].n + tile - 1) / tile : 0;
    uint64_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint64_t before = carry;
    for (int k = 0; k < w; ++k) before += wsum[k];
    if (i < nsegs) tile_prefix[i] = before + inc - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = before + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) tile_prefix[nsegs] = carry;
}

// ---------------------------------------------------------------- host side

static std::mutex g_mu;

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

// Scratch of one (device, stream): ticket, look-back status words, and the
// batch descriptor copies.
struct Workspace {
  uint32_t* ticket = nullptr;
  unsigned long long* status = nullptr;
  uint64_t status_cap = 0;
  uint64_t* tile_prefix = nullptr;
  DevSeg* segs = nullptr;
  uint64_t segs_cap = 0;
  DevTable* tabs = nullptr;
  uint64_t tabs_cap = 0;
  uint32_t epoch = 0;
};

static std::map<std::pair<int, void*>, Workspace*> g_ws;

static int grow(void** ptr, uint64_t* cap, uint64_t need, size_t elem, hipStream_t stream,
                bool zero) {
  if (*cap >= need && *ptr) return PFAC_OK;
  uint64_t nc = need < 1024 ? 1024 : need + need / 2;
  if (*ptr) {
    if (hipStreamSynchronize(stream) != hipSuccess) return PFAC_E_HIP;
    (void)hipFree(*ptr);
    *ptr = nullptr;
    *cap = 0;
  }
  if (hipMalloc(ptr, nc * elem) != hipSuccess) {
    *ptr = nullptr;
    return PFAC_E_NOMEM;
  }
  if (zero && hipMemset(*ptr, 0, nc * elem) != hipSuccess) return PFAC_E_HIP;
  *cap = nc;
  return PFAC_OK;
}

static int get_workspace(int dev, hipStream_t stream, uint64_t tiles, uint64_t nsegs,
                         uint64_t ntabs, Workspace** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace*& ws = g_ws[{dev, (void*)stream}];
  if (!ws) {
    ws = new (std::nothrow) Workspace();
    if (!ws) return PFAC_E_NOMEM;
    if (hipMalloc(&ws->ticket, 256) != hipSuccess) return PFAC_E_NOMEM;
  }
  const uint64_t old_cap = ws->status_cap;
  int rc = grow(reinterpret_cast<void**>(&ws->status), &ws->status_cap, tiles,
                sizeof(unsigned long long), stream, true);
  if (rc) return rc;
  if (ws->status_cap != old_cap) ws->epoch = 0;   // fresh zeroed status words
  if (nsegs) {
    uint64_t cap_prefix = ws->segs_cap;
    rc = grow(reinterpret_cast<void**>(&ws->segs), &ws->segs_cap, nsegs, sizeof(DevSeg), stream,
              false);
    if (rc) return rc;
    if (ws->segs_cap != cap_prefix || !ws->tile_prefix) {
      if (ws->tile_prefix) (void)hipFree(ws->tile_prefix);
      ws->tile_prefix = nullptr;
      if (hipMalloc(&ws->tile_prefix, (ws->segs_cap + 1) * sizeof(uint64_t)) != hipSuccess)
        return PFAC_E_NOMEM;
    }
  }
  if (ntabs) {
    rc = grow(reinterpret_cast<void**>(&ws->tabs), &ws->tabs_cap, ntabs, sizeof(DevTable), stream,
              false);
    if (rc) return rc;
  }
  // launch epochs tag the status words, so they never need clearing; when
  // the tag would wrap, clear them once
  ws->epoch += 1;
  if (ws->epoch >= (1u << kEpochBits)) {
    if (hipMemsetAsync(ws->status, 0, ws->status_cap * sizeof(unsigned long long), stream) !=
        hipSuccess)
      return PFAC_E_HIP;
    ws->epoch = 1;
  }
  *out = ws;
  return PFAC_OK;
}

static uint32_t lds_bytes(uint32_t block, uint32_t K, uint32_t hot, uint32_t halo) {
  const uint32_t span = block * kPPT + halo;
  const uint32_t words = (K ? (1u << (2 * K)) : 0u) + 4 * hot + (span / 16 + 2) + (span / 32 + 2);
  return 4 * words;
}

static uint32_t halo_for(uint32_t max_len) {
  uint32_t h = max_len > 1 ? max_len - 1 : 0;
  if (h < 16) h = 16;   // room for the root jump window of the last positions
  return (h + 63) / 64 * 64;
}

using KernelFn = void (*)(KParams);

static KernelFn pick_kernel(uint32_t block, bool global) {
  switch (block) {
    case 256: return global ? pfac_kernel<256, true> : pfac_kernel<256, false>;
    case 512: return global ? pfac_kernel<512, true> : pfac_kernel<512, false>;
    case 1024: return global ? pfac_kernel<1024, true> : pfac_kernel<1024, false>;
    default: return nullptr;
  }
}

// Fill unset plan fields; reject plans that cannot run.
static int resolve_plan(const pfac_plan* in, uint32_t max_len, uint64_t num_states, int dev,
                        pfac_plan* out) {
  const DeviceInfo di = device_info(dev);
  if (!di.ok) return PFAC_E_NODEV;
  pfac_plan p = in ? *in : pfac_plan{0, 0, 0, 0, 0};
  if (p.variant != PFAC_VARIANT_TILED && p.variant != PFAC_VARIANT_GLOBAL) return PFAC_E_ARG;
  const uint32_t halo = halo_for(max_len);
  if (p.variant == PFAC_VARIANT_TILED && halo > kMaxHaloLds) {
    if (in && in->variant == PFAC_VARIANT_TILED && in->block) return PFAC_E_ARG;
    p.variant = PFAC_VARIANT_GLOBAL;  // patterns too long to stage a halo in LDS
  }
  if (p.block == 0) p.block = 512;
  if (p.block != 256 && p.block != 512 && p.block != 1024) return PFAC_E_ARG;
  if (p.variant == PFAC_VARIANT_GLOBAL) {
    p.jump_depth = PFAC_JUMP_OFF;
    p.hot_states = PFAC_HOT_NONE;
  } else {
    const uint32_t budget = (uint32_t)di.lds_per_block;
    if (p.jump_depth == 0)
      p.jump_depth = lds_bytes(p.block, 7, 0, halo) <= budget ? 7u : 6u;
    if (p.jump_depth != PFAC_JUMP_OFF && (p.jump_depth < kMinJump || p.jump_depth > kMaxJump))
      return PFAC_E_ARG;
    const uint32_t K = p.jump_depth == PFAC_JUMP_OFF ? 0 : p.jump_depth;
    if (p.hot_states == 0) {
      // stage the whole table when it fits in what the jump table leaves
      const uint32_t base = lds_bytes(p.block, K, 0, halo);
      const uint64_t want = num_states;
      const uint64_t room = budget > base ? (budget - base) / 16 : 0;
      p.hot_states = (want <= room && want * 16 <= 48 * 1024) ? (uint32_t)want : PFAC_HOT_NONE;
    }
    const uint32_t hot = p.hot_states == PFAC_HOT_NONE ? 0 : p.hot_states;
    if (lds_bytes(p.block, K, hot, halo) > (uint32_t)di.lds_per_block) return PFAC_E_ARG;
  }
  *out = p;
  return PFAC_OK;
}

static int launch(const KParams& kp_in, const pfac_plan& plan, uint32_t halo, int dev,
                  hipStream_t stream, const DevSeg* d_segs, uint32_t nsegs, uint64_t* d_prefix,
                  unsigned long long* d_seg_counters) {
  KParams kp = kp_in;
  const bool global = plan.variant == PFAC_VARIANT_GLOBAL;
  kp.K = (global || plan.jump_depth == PFAC_JUMP_OFF) ? 0 : plan.jump_depth;
  kp.hot = (global || plan.hot_states == PFAC_HOT_NONE) ? 0 : plan.hot_states;
  kp.halo = global ? 0 : halo;
  const uint32_t lds = global ? 0 : lds_bytes(plan.block, kp.K, kp.hot, halo);
  KernelFn fn = pick_kernel(plan.block, global);
  if (!fn) return PFAC_E_ARG;
  hipLaunchKernelGGL(pfac_prep_kernel, dim3(1), dim3(1024), 0, stream, d_segs, nsegs,
                     plan.block * kPPT, d_prefix, kp.counters, d_seg_counters, kp.ticket);
  if (hipGetLastError() != hipSuccess) return PFAC_E_HIP;
  if (kp.total_tiles == 0) return PFAC_OK;
  uint64_t grid = plan.grid;
  if (grid == 0) {
    if (lds > 48 * 1024)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn),
                                                     (int)plan.block, lds) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    grid = (uint64_t)per_cu * (uint64_t)device_info(dev).cus;
  } else if (lds > 48 * 1024) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  if (grid > kp.total_tiles) grid = kp.total_tiles;
  hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(plan.block), lds, stream, kp);
  if (hipGetLastError() != hipSuccess) return PFAC_E_HIP;
  return PFAC_OK;
}

}  // namespace pfac

using namespace pfac;

extern "C" {

const char* pfac_strerror(int s) {
  switch (s) {
    case PFAC_OK: return "ok";
    case PFAC_E_ARG: return "invalid argument";
    case PFAC_E_PATTERN: return "empty pattern or pattern byte outside A,C,G,T";
    case PFAC_E_TOO_LARGE: return "trie needs 2^31 or more states";
    case PFAC_E_NOMEM: return "out of memory";
    case PFAC_E_HIP: return "HIP runtime error";
    case PFAC_E_NODEV: return "no gfx950 device";
    default: return "unknown status";
  }
}

const char* pfac_version(void) { return "pfac-mi355x 0.1 (gfx950)"; }

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
  const HostTable& h = t->host;
  // one device allocation: next | out | jump[K] | jres[K] | views
  auto align = [](uint64_t x) { return (x + 255) / 256 * 256; };
  uint64_t off = 0;
  const uint64_t o_next = off; off = align(off + h.next.size() * 4);
  const uint64_t o_out = off; off = align(off + h.out.size() * sizeof(OutEntry));
  uint64_t o_jump[kMaxJump + 1] = {}, o_jres[kMaxJump + 1] = {};
  for (uint32_t K = kMinJump; K <= kMaxJump; ++K) {
    o_jump[K] = off; off = align(off + h.jump[K].size() * 4);
    o_jres[K] = off; off = align(off + h.jres[K].size() * sizeof(OutEntry));
  }
  const uint64_t o_views = off; off = align(off + (kMaxJump + 1) * sizeof(DevTable));
  if (hipMalloc(&t->dmem, off) != hipSuccess) {
    delete t;
    return PFAC_E_NOMEM;
  }
  t->dbytes = off;
  char* base = static_cast<char*>(t->dmem);
  t->d_next = reinterpret_cast<uint32_t*>(base + o_next);
  t->d_out = reinterpret_cast<OutEntry*>(base + o_out);
  bool ok = hipMemcpy(t->d_next, h.next.data(), h.next.size() * 4, hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemcpy(t->d_out, h.out.data(), h.out.size() * sizeof(OutEntry),
                      hipMemcpyHostToDevice) == hipSuccess;
  DevTable views[kMaxJump + 1];
  for (uint32_t K = 0; K <= kMaxJump; ++K) {
    views[K] = DevTable{t->d_next, t->d_out, nullptr, nullptr, (uint32_t)h.num_states, h.max_len};
    if (K >= kMinJump) {
      t->d_jump[K] = reinterpret_cast<uint32_t*>(base + o_jump[K]);
      t->d_jres[K] = reinterpret_cast<OutEntry*>(base + o_jres[K]);
      ok = ok && hipMemcpy(t->d_jump[K], h.jump[K].data(), h.jump[K].size() * 4,
                           hipMemcpyHostToDevice) == hipSuccess;
      ok = ok && hipMemcpy(t->d_jres[K], h.jres[K].data(), h.jres[K].size() * sizeof(OutEntry),
                           hipMemcpyHostToDevice) == hipSuccess;
      views[K].jump = t->d_jump[K];
      views[K].jres = t->d_jres[K];
    }
  }
  t->d_views = reinterpret_cast<DevTable*>(base + o_views);
  ok = ok && hipMemcpy(t->d_views, views, sizeof(views), hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    (void)hipFree(t->dmem);
    delete t;
    return PFAC_E_HIP;
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
  return PFAC_OK;
}

void pfac_free_table(pfac_table* t) {
  if (!t) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(t->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(t->dmem);
  (void)hipSetDevice(cur);
  delete t;
}

int pfac_default_plan(const pfac_table* t, uint64_t n, int enc, pfac_plan* out) {
  (void)n;
  if (!t || !out || (enc != PFAC_TEXT_ASCII && enc != PFAC_TEXT_2BIT)) return PFAC_E_ARG;
  return resolve_plan(nullptr, t->host.max_len, t->host.num_states, t->device, out);
}

static DevTable view_of(const pfac_table* t, uint32_t K) {
  const HostTable& h = t->host;
  DevTable v{t->d_next, t->d_out, nullptr, nullptr, (uint32_t)h.num_states, h.max_len};
  if (K >= kMinJump && K <= kMaxJump) {
    v.jump = t->d_jump[K];
    v.jres = t->d_jres[K];
  }
  return v;
}

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
  pfac_plan pl;
  int rc = resolve_plan(plan, t->host.max_len, t->host.num_states, dev, &pl);
  if (rc) return rc;
  const uint64_t tile = (uint64_t)pl.block * kPPT;
  const uint64_t tiles = (n + tile - 1) / tile;
  Workspace* ws = nullptr;
  rc = get_workspace(dev, stream, tiles ? tiles : 1, 0, 0, &ws);
  if (rc) return rc;
  KParams kp;
  memset(&kp, 0, sizeof(kp));
  kp.single = 1;
  kp.nsegs = 1;
  kp.total_tiles = tiles;
  kp.text = static_cast<const uint8_t*>(d_text);
  kp.match = d_match;
  kp.hits = d_hits;
  kp.hit_cap = hit_cap;
  kp.counters = reinterpret_cast<unsigned long long*>(d_counters);
  kp.ticket = ws->ticket;
  kp.status = ws->status;
  kp.epoch = ws->epoch;
  kp.seg0 = DevSeg{0, n, 0, 0, (uint32_t)enc};
  const uint32_t K = (pl.variant == PFAC_VARIANT_GLOBAL || pl.jump_depth == PFAC_JUMP_OFF)
                         ? 0 : pl.jump_depth;
  kp.tab0 = view_of(t, K);
  return launch(kp, pl, halo_for(t->host.max_len), dev, stream, nullptr, 0, nullptr, nullptr);
}

int pfac_match_batch(const pfac_table* const* tables, uint32_t num_tables,
                     const pfac_text_desc* descs, uint32_t num_texts, const void* d_text_base,
                     int32_t* d_match_base, pfac_batch_hit* d_hits, uint64_t hit_cap,
                     uint64_t* d_counters, const pfac_plan* plan, void* stream_) {
  if (!tables || num_tables == 0 || !d_counters || (num_texts && !descs)) return PFAC_E_ARG;
  if (d_hits == nullptr) hit_cap = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFAC_E_NODEV;
  uint32_t max_len = 0;
  uint64_t max_states = 0;
  for (uint32_t i = 0; i < num_tables; ++i) {
    if (!tables[i] || tables[i]->device != dev) return PFAC_E_ARG;
    max_len = std::max(max_len, tables[i]->host.max_len);
    max_states = std::max<uint64_t>(max_states, tables[i]->host.num_states);
  }
  for (uint32_t s = 0; s < num_texts; ++s) {
    const pfac_text_desc& d = descs[s];
    if (d.n >= (1ull << 32) || d.table >= num_tables ||
        (d.enc != PFAC_TEXT_ASCII && d.enc != PFAC_TEXT_2BIT) || (d.n && !d_text_base))
      return PFAC_E_ARG;
  }
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  pfac_plan pl;
  int rc = resolve_plan(plan, max_len, max_states, dev, &pl);
  if (rc) return rc;
  // hot rows only when every table fits
  if (pl.hot_states != PFAC_HOT_NONE && pl.hot_states > 0) {
    for (uint32_t i = 0; i < num_tables; ++i)
      if (tables[i]->host.num_states > pl.hot_states) pl.hot_states = PFAC_HOT_NONE;
  }
  const uint64_t tile = (uint64_t)pl.block * kPPT;
  uint64_t tiles = 0;
  for (uint32_t s = 0; s < num_texts; ++s) tiles += (descs[s].n + tile - 1) / tile;
  Workspace* ws = nullptr;
  rc = get_workspace(dev, stream, tiles ? tiles : 1, num_texts ? num_texts : 1, num_tables, &ws);
  if (rc) return rc;
  const uint32_t K = (pl.variant == PFAC_VARIANT_GLOBAL || pl.jump_depth == PFAC_JUMP_OFF)
                         ? 0 : pl.jump_depth;
  std::vector<DevTable> views(num_tables);
  for (uint32_t i = 0; i < num_tables; ++i) views[i] = view_of(tables[i], K);
  if (num_texts &&
      hipMemcpyAsync(ws->segs, descs, num_texts * sizeof(DevSeg), hipMemcpyHostToDevice, stream) !=
          hipSuccess)
    return PFAC_E_HIP;
  if (hipMemcpyAsync(ws->tabs, views.data(), num_tables * sizeof(DevTable), hipMemcpyHostToDevice,
                     stream) != hipSuccess)
    return PFAC_E_HIP;
  KParams kp;
  memset(&kp, 0, sizeof(kp));
  kp.single = 0;
  kp.tables = ws->tabs;
  kp.segs = ws->segs;
  kp.tile_prefix = ws->tile_prefix;
  kp.nsegs = num_texts;
  kp.total_tiles = tiles;
  kp.text = static_cast<const uint8_t*>(d_text_base);
  kp.match = d_match_base;
  kp.hits = d_hits;
  kp.hit_cap = hit_cap;
  kp.counters = reinterpret_cast<unsigned long long*>(d_counters);
  kp.seg_counters = reinterpret_cast<unsigned long long*>(d_counters) + 2;
  kp.ticket = ws->ticket;
  kp.status = ws->status;
  kp.epoch = ws->epoch;
  return launch(kp, pl, halo_for(max_len), dev, stream, ws->segs, num_texts, ws->tile_prefix,
                kp.seg_counters);
}

}  // extern "C"
