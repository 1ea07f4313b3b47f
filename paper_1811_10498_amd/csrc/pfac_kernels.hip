// PFAC matching kernels for gfx950 and the C ABI around them.
//
// Semantics (paper Sec. IV): every start position of the text walks the
// failure-less goto trie from the root, one base per step, stops at the
// first missing transition, and reports the last (= longest) pattern it
// passed.  The paper launches one thread per character, stages the text in
// shared memory and reads the table through the texture cache (Sec. V.B,
// V.C, VII).  The gfx950 design keeps the walk and reorganises the memory
// side around one observation: in a random-like text almost every walk ends
// within the first log4(#patterns) levels, where the trie is dense.
//   * Filter: the first D steps of every walk (D = 6..10) depend only on the
//     D-base window at the position.  A bitmap of 4^D bits in LDS says which
//     windows lead anywhere (continue past depth D, or pass a final state);
//     every other position reports nothing after one LDS lookup.
//   * Second filter: survivors whose first K bases have a cleared bit in a
//     two-hash LDS bitmap of the patterns' first K bases stop there too.
//   * Deep walks: the surviving positions of a wave are compacted into an
//     LDS queue and walked by all 64 lanes together (or, when they are rare,
//     after the wave's last tile): one global read of the depth-D jump
//     table, then the breadth-first numbered next-state table (L2 /
//     Infinity Cache resident), runs of single-child states in one step.
//   * Text: each wave stages its tile (2048 positions, 1024 in a batch) plus a halo of
//     max_len-1 bases with 16-byte loads, as 2-bit codes plus an "invalid"
//     bit per base (bytes other than A,C,G,T, and everything past the end).
//   * Outputs: the dense int32 array leaves with 16-byte non-temporal
//     stores; hits are counted per tile and parked in a fixed-size slot per
//     tile; one finish kernel (decoupled look-back over its workgroups)
//     places them in position order.  No scan workgroup waits for another.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <mutex>
#include <utility>
#include <vector>

#include "pfac_internal.h"

namespace pfac {

// Start positions per wave tile: one text per launch takes 2048 (the fixed
// cost of a tile -- staging, locating, one round of deep walks -- spread over
// more positions); a batch takes 1024 (short texts waste less of a tile).
constexpr uint32_t kTileSingle = 2048;
constexpr uint32_t kTileBatch = 1024;
constexpr uint32_t kQueue = 256;       // deep-walk queue entries per wave
constexpr uint32_t kSlot = 32;         // hits parked per tile
constexpr uint32_t kMaxHalo = 4096;    // longest halo staged in LDS (bases)
constexpr uint32_t kRedTiles = 4096;   // tiles per reduce/scatter workgroup

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

struct DevSeg {
  uint64_t text_off;
  uint64_t n;
  uint64_t match_off;
  uint32_t table;
  uint32_t enc;
};
static_assert(sizeof(DevSeg) == sizeof(pfac_text_desc), "descriptor layout");

struct Slot {
  uint32_t pos;
  int32_t pid;
};

// A walk deferred to the end of the wave that found it: its start position
// and a copy of the next kWindow bases (2-bit codes, 16 per word, first base
// in the top bits of codes[0]; invalid bits, base k in bit k of inv).
constexpr uint32_t kWindow = 64;
struct WalkEntry {
  uint32_t pos;
  uint32_t slow;       // 1: a non-base within the first D bases (walk from the root)
  uint32_t codes[4];
  uint32_t inv[2];
};
static_assert(sizeof(WalkEntry) == 32, "walk entry layout");

// Parameters of the scan kernel (one table per launch).
struct ScanParams {
  const uint32_t* next;
  const OutEntry* out;
  const uint32_t* chain;          // runs of single-child steps (TILED)
  const uint32_t* jump;           // depth-D jump table (TILED)
  const OutEntry* jres;
  const uint32_t* image;          // LDS image of depth D (TILED): filter bitmap, its
                                  // rank words, node bytes of the levels below
  uint32_t image_words;           // image words copied into LDS
  uint32_t levels;                // trie levels held in LDS (D .. D+levels-1)
  uint32_t longer;                // 1: every pattern is longer than D bases
  uint32_t lds_trie;              // 1: no pattern is D bases or shorter, so a set
                                  // filter bit is a depth-D node found by rank
  const u32x4* lvl;                  // per LDS level: image word offset of its node
                                     // bytes, of its rank words, its first state
  uint32_t D;
  const uint32_t* hash;           // second-filter bitmap (hash_on)
  uint32_t hash_on;               // 1: queued windows pass the second filter first
  uint32_t hash_words;            // its words, copied into LDS after the image
  uint32_t hash_shift;            // 32 - bits
  uint32_t hash_kmask;            // key bits of the K-base window (top 2K bits)
  uint32_t hash_imask;            // invalid bits of the K-base window ((1 << K) - 1)
  uint32_t halo;                  // staged bases past the tile, multiple of 64
  uint32_t single;                // 1: one text (seg0), tiles 0..local_tiles-1
  uint32_t ngroup;                // batch: texts handled by this launch
  DevSeg seg0;
  const DevSeg* segs;             // batch: all texts
  const uint32_t* group_segs;     // batch: text index of each text of this launch
  const uint64_t* group_prefix;   // batch: [ngroup+1] first local tile of each
  const uint64_t* tile_prefix;    // batch: [nsegs+1] first global tile of each text
  uint64_t local_tiles;
  const uint8_t* text;
  int32_t* match;
  uint32_t* tile_hits;            // [tiles]
  unsigned long long* tile_occ;   // [tiles]
  Slot* slots;                    // [tiles * kSlot] or nullptr
  // deferred walks (one-text launches): every wave owns wq_cap entries of wq
  // (wave w from w*wq_cap) and walks them after its last tile
  uint32_t defer;
  uint32_t wq_cap;
  WalkEntry* wq;
  uint64_t wq_waves;              // waves wq has room for
};

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ int ascii_code(uint32_t b) {
  return b == 'A' ? 0 : b == 'C' ? 1 : b == 'G' ? 2 : b == 'T' ? 3 : -1;
}

// (x << s) | y as one VALU instruction.  Written as an instruction so that
// the compiler cannot merge a chain of such steps on bit-disjoint operands
// into a quarter-rate 32-bit multiply.
template <int S>
__device__ __forceinline__ uint32_t shl_or(uint32_t x, uint32_t y) {
  uint32_t r;
  asm("v_lshl_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "i"(S), "v"(y));
  return r;
}

// Four ASCII bytes -> four 2-bit codes (first byte in the top two bits of
// the 8-bit result) and a 4-bit "not a base" mask (first byte in bit 0).
// code = ((b >> 1) ^ (b >> 2)) & 3 maps A,C,G,T to 0,1,2,3; a byte is a base
// iff re-encoding its code gives the byte back.
__device__ __forceinline__ void ascii4(uint32_t x, uint32_t& code8, uint32_t& inv4) {
  const uint32_t cb = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
  const uint32_t expect = __builtin_amdgcn_perm(0u, 0x54474341u, cb);  // 'A','C','G','T'
  const uint32_t t = x ^ expect;
  const uint32_t nz = (((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t) & 0x80808080u;
  inv4 = ((nz >> 7) * 0x01020408u) >> 24;
  const uint32_t t1 = shl_or<10>(cb, cb);   // as in ascii_chunk
  code8 = shl_or<20>(t1, t1) >> 24;
}

// The 32-bit LDS word at byte address a.  The kernels declare no static LDS,
// so the dynamic area (the filter bitmap first) starts at LDS address 0 and a
// bitmap word is read at its byte offset with no base added.
typedef const uint32_t __attribute__((address_space(3))) lds_u32;
__device__ __forceinline__ uint32_t lds_word(uint32_t a) {
  return *reinterpret_cast<lds_u32*>(static_cast<uintptr_t>(a));
}

// The lane index as a value the compiler must take anew where it is asked
// for: conditions on it inside the tile loop are then recomputed (one
// compare) instead of hoisted out as 64-bit masks that do not fit in the
// scalar registers and go to spill slots.
__device__ __forceinline__ uint32_t fresh_lane() {
  uint32_t l = threadIdx.x & 63;
  asm volatile("" : "+v"(l));
  return l;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  #pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Exclusive prefix over the 64 lanes; *total receives the wave sum.
__device__ __forceinline__ uint32_t wave_excl(uint32_t v, uint32_t* total) {
  const int lane = threadIdx.x & 63;
  uint32_t inc = v;
  #pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  *total = __shfl(inc, 63, 64);
  return inc - v;
}

// Inclusive prefix sum over the 64 lanes with DPP lane moves (no LDS): lane
// shifts of 1, 2, 4 and 8 within each row of 16 lanes, then the running total
// of lane 15 carried into rows 1 and 3 and that of lane 31 into rows 2 and 3.
// Every lane of the wave must be active.
__device__ __forceinline__ uint32_t wave_incl_dpp(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}

// Exclusive prefix over the 64 lanes; *total receives the wave sum (uniform).
__device__ __forceinline__ uint32_t wave_excl_dpp(uint32_t v, uint32_t* total) {
  const uint32_t inc = wave_incl_dpp(v);
  *total = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
  return inc - v;
}

// One base of a text in global memory (out of range = invalid).
__device__ __forceinline__ int global_base(const uint8_t* t, uint64_t n, uint32_t enc,
                                           uint64_t q) {
  if (q >= n) return -1;
  if (enc == PFAC_TEXT_ASCII) return ascii_code(t[q]);
  return (t[q >> 2] >> (2 * (q & 3))) & 3;
}

// Continue a walk from state s.  LDS text: q is a tile-local index into the
// staged codes; global text: q is the text index.  s == 0 is the root: the
// root row is row 0 and no edge leads back to it.
template <bool GLOBAL>
__device__ __forceinline__ void walk(uint32_t s, uint64_t q, const uint32_t* __restrict__ pk,
                                     const uint32_t* __restrict__ iv,
                                     const uint32_t* __restrict__ next,
                                     const OutEntry* __restrict__ out, const uint8_t* gtext,
                                     uint64_t gn, uint32_t genc, int32_t& best,
                                     unsigned long long& occ) {
  for (;;) {
    uint32_t c;
    if (GLOBAL) {
      const int b = global_base(gtext, gn, genc, q);
      if (b < 0) break;
      c = (uint32_t)b;
    } else {
      const uint32_t qq = (uint32_t)q;
      if ((iv[qq >> 5] >> (qq & 31)) & 1u) break;
      c = (pk[qq >> 4] >> (30 - 2 * (qq & 15))) & 3u;
    }
    const uint32_t e = next[(uint64_t)s * 4 + c];
    if (e == 0) break;
    s = e & kStateMask;
    if (e & kFinalBit) {
      const OutEntry o = out[s];
      best = o.pid;
      occ += o.mult;
    }
    ++q;
  }
}

// The walk over LDS text with path compression: at a state with a run of
// single-child steps (chain record, see the table layout) the next bases are
// compared with the whole run at once -- all of them match and the walk jumps
// to the end of the run, or the walk ends inside it, where no pattern ends.
// The run record and the ordinary edge for the next base are loaded together,
// so a step costs one round trip either way.
__device__ __forceinline__ void walk_lds(uint32_t s, uint32_t q, const uint32_t* __restrict__ pk,
                                         const uint32_t* __restrict__ iv,
                                         const uint32_t* __restrict__ next,
                                         const OutEntry* __restrict__ out,
                                         const uint32_t* __restrict__ chain, int32_t& best,
                                         unsigned long long& occ) {
  for (;;) {
    // validity bits and codes of the 16 bases from q (first base on top)
    const uint32_t ivw = __builtin_amdgcn_alignbit(iv[(q >> 5) + 1], iv[q >> 5], q & 31u);
    const uint32_t win =
        (uint32_t)(((((uint64_t)pk[q >> 4] << 32) | pk[(q >> 4) + 1]) << (2 * (q & 15u))) >> 32);
    const u32x2 ch = *reinterpret_cast<const u32x2*>(chain + 2ull * s);
    const uint32_t e = next[(uint64_t)s * 4 + (win >> 30)];
    const uint32_t len = ch.x & 15u;
    if (len >= 2) {
      if ((ivw & ((1u << len) - 1u)) | ((win ^ ch.x) & (0xFFFFFFFFu << (32 - 2 * len)))) break;
      s = ch.y & kStateMask;
      q += len;
      if (ch.y & kFinalBit) {
        const OutEntry o = out[s];
        best = o.pid;
        occ += o.mult;
      }
      continue;
    }
    if ((ivw & 1u) || e == 0) break;
    s = e & kStateMask;
    if (e & kFinalBit) {
      const OutEntry o = out[s];
      best = o.pid;
      occ += o.mult;
    }
    ++q;
  }
}

// Set bits among the first t (0..15) node bytes of a 16-node group (child
// bits only, the low nibble of each byte).
__device__ __forceinline__ uint32_t children_before(const u32x4& g, uint32_t t) {
  const uint32_t m = 0x0F0F0F0Fu;
  const uint32_t wi = t >> 2;
  const uint32_t part = (1u << (8 * (t & 3))) - 1u;   // bytes before t in its word
  uint32_t c = 0;
  c += __builtin_popcount(g.x & m & (wi > 0 ? ~0u : part));
  c += __builtin_popcount(g.y & m & (wi > 1 ? ~0u : wi == 1 ? part : 0u));
  c += __builtin_popcount(g.z & m & (wi > 2 ? ~0u : wi == 2 ? part : 0u));
  c += __builtin_popcount(g.w & m & (wi == 3 ? part : 0u));
  return c;
}

// One queued walk of the tiled kernel.  Entry e: tile index of the start
// position in bits 0..14, bit 15 set when the position's D-base window holds
// a non-base (then the walk starts at the root).  Otherwise the first D
// bases are the key x of the window:
//   * lds_trie: x names a depth-D node; its index within the level is the
//     rank of x among the set filter bits.  The walk goes on through the
//     trie levels held in LDS (a child's index = child bits of the level's
//     earlier nodes + the node's own lower child bits), then hands over to
//     the global next-state table at the last LDS level;
//   * otherwise the global depth-D jump table gives the state reached and
//     the finals passed within the first D bases.
// Every route ends in the same global-table loop.
__device__ __forceinline__ int32_t deep_walk(uint32_t e, uint32_t D, uint32_t lds_trie,
                                             uint32_t levels, const uint32_t* lds,
                                             const uint32_t* bmpre, const u32x4* lvl,
                                             const uint32_t* __restrict__ pk,
                                             const uint32_t* __restrict__ iv,
                                             const uint32_t* __restrict__ next,
                                             const OutEntry* __restrict__ out,
                                             const uint32_t* __restrict__ jump,
                                             const OutEntry* __restrict__ jres,
                                             const uint32_t* __restrict__ chain,
                                             unsigned long long& occ) {
  const uint32_t qt = e & 0x7FFFu;
  int32_t best = 0;
  uint32_t s = 0, q = qt;
  if (!(e & 0x8000u)) {
    const uint32_t x = (uint32_t)((((uint64_t)pk[qt >> 4] << 32) | pk[(qt >> 4) + 1])
                                  << (2 * (qt & 15)) >> (64 - 2 * D));
    q = qt + D;
    if (lds_trie) {
      const u32x4 bg = *reinterpret_cast<const u32x4*>(lds + ((x >> 7) << 2));
      const uint32_t wi = (x >> 5) & 3u, part = (1u << (x & 31u)) - 1u;
      uint32_t j = bmpre[x >> 7];
      j += __builtin_popcount(bg.x & (wi > 0 ? ~0u : part));
      j += __builtin_popcount(bg.y & (wi > 1 ? ~0u : wi == 1 ? part : 0u));
      j += __builtin_popcount(bg.z & (wi > 2 ? ~0u : wi == 2 ? part : 0u));
      j += __builtin_popcount(bg.w & (wi == 3 ? part : 0u));
      // all active lanes move down one level per step: the level is uniform
      u32x4 L = lvl[0];
      if (levels) {
        for (uint32_t k = 0;;) {
          const u32x4 g = *reinterpret_cast<const u32x4*>(lds + L.x + ((j >> 4) << 2));
          const uint32_t pre = lds[L.y + (j >> 4)];
          const uint32_t t = j & 15u;
          const uint32_t word = t < 4 ? g.x : t < 8 ? g.y : t < 12 ? g.z : g.w;
          const uint32_t b = (word >> (8 * (t & 3))) & 0xFFu;
          if (b & 0x10u) {
            const OutEntry o = out[L.z + j];
            best = o.pid;
            occ += o.mult;
          }
          if ((iv[q >> 5] >> (q & 31)) & 1u) return best;
          const uint32_t c = (pk[q >> 4] >> (30 - 2 * (q & 15))) & 3u;
          if (!((b >> c) & 1u)) return best;
          if (++k == levels) break;                 // hand over below this node
          j = pre + children_before(g, t) + __builtin_popcount(b & ((1u << c) - 1u));
          ++q;
          L = lvl[__builtin_amdgcn_readfirstlane(k)];
        }
      }
      s = L.z + j;
    } else {
      const uint32_t jj = jump[x];
      if (jj & kFinalBit) {
        const OutEntry o = jres[x];
        best = o.pid;
        occ += o.mult;
      }
      s = jj & kStateMask;
      if (!s) return best;
    }
  }
  walk_lds(s, q, pk, iv, next, out, chain, best, occ);
  return best;
}

// Second filter for one queued entry (see deep_walk for the entry format):
// true when the walk must go on -- both hashes of its first K bases have
// their bits set (or it is an entry that walks from the root).  Every pattern
// has at least K bases, so a window with a non-base among its first K bases,
// or whose first K bases are no pattern's first K bases (a cleared bit),
// reports nothing.
__device__ __forceinline__ bool hash_pass(uint32_t e, const uint32_t* __restrict__ pk,
                                          const uint32_t* __restrict__ iv,
                                          const uint32_t* __restrict__ hl, uint32_t kmask,
                                          uint32_t imask, uint32_t shift) {
  if (e & 0x8000u) return true;
  const uint32_t qt = e & 0x7FFFu;
  // a non-base among the first K bases: every pattern has at least K bases,
  // so none starts here
  if (__builtin_amdgcn_alignbit(iv[(qt >> 5) + 1], iv[qt >> 5], qt & 31u) & imask) return false;
  const uint32_t wi = qt >> 4;
  const uint32_t key =
      (uint32_t)(((((uint64_t)pk[wi] << 32) | pk[wi + 1]) << (2 * (qt & 15u))) >> 32) & kmask;
  const uint32_t h = (key * kHashMul) >> shift;
  const uint32_t h2 = (key * kHashMul2) >> shift;
  return (hl[h >> 5] >> (h & 31u)) & (hl[h2 >> 5] >> (h2 & 31u)) & 1u;
}

// Text of one wave tile: bases [t0, t0+span) of one text, span = TILE + halo.
// Staged into the wave's LDS area as 2-bit codes, 16 per word with the first
// base in the top bits (a window of bases then reads as a key with its first
// base most significant), and an invalid bit per base, 32 per word with the
// first base in bit 0.  Bases past the end of the text are invalid; two
// sentinel words follow the span.  Staging is split in two: fetch() issues
// the 16-byte loads of the lane's chunks into registers (for the next tile,
// while the current one is processed) and commit() converts them into LDS.
struct TextRef {
  const uint8_t* t;
  uint64_t n;
  uint64_t t0;
  uint32_t enc;
};

struct Prefetch {
  u32x4 a, b;          // ASCII: the lane's 16-byte chunk of the tile (a);
                       // 2-bit: chunks lane and lane+64 (a, b)
  uint32_t h;          // ASCII: the lane's 4-byte piece of the halo
  uint32_t fast;       // bit 0: a loaded, bit 1: b loaded, bit 2: h loaded
};

template <uint32_t TILE>
__device__ __forceinline__ Prefetch fetch(const TextRef& r, uint32_t halo) {
  const uint32_t lane = fresh_lane();
  const uintptr_t addr = reinterpret_cast<uintptr_t>(r.t);
  Prefetch f;
  f.fast = 0;
  f.a = u32x4{0, 0, 0, 0};
  f.b = u32x4{0, 0, 0, 0};
  f.h = 0;
  if (r.enc == PFAC_TEXT_ASCII) {
    const uint64_t ga = r.t0 + 16ull * lane;
    if ((addr & 15) == 0 && ga + 16 <= r.n) {
      f.a = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(r.t + ga));
      f.fast |= 1u;
    }
    if (TILE == 2048) {
      const uint64_t gb = ga + 1024;
      if ((addr & 15) == 0 && gb + 16 <= r.n) {
        f.b = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(r.t + gb));
        f.fast |= 2u;
      }
    }
    const uint64_t gh = r.t0 + TILE + 4ull * lane;
    if ((addr & 3) == 0 && lane < halo / 4 && gh + 4 <= r.n) {
      f.h = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(r.t + gh));
      f.fast |= 4u;
    }
  } else {
    const uint32_t nch = (TILE + halo) / 64;   // 64 bases per 16-byte chunk
    const bool al = (addr & 15) == 0;
    const uint64_t ga = r.t0 + 64ull * lane;
    if (al && lane < nch && ga + 64 <= r.n) {
      f.a = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(r.t + ga / 4));
      f.fast |= 1u;
    }
    const uint64_t gb = ga + 64ull * 64;
    if (al && lane + 64 < nch && gb + 64 <= r.n) {
      f.b = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(r.t + gb / 4));
      f.fast |= 2u;
    }
  }
  return f;
}

// One 16-byte ASCII chunk -> 16 codes (big-endian word) and 16 invalid bits.
__device__ __forceinline__ void ascii_chunk(const u32x4& v, uint32_t& packed, uint32_t& inv) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  uint32_t cb[4], t[4];
  #pragma unroll
  for (int k = 0; k < 4; ++k) {
    cb[k] = ((w[k] >> 1) ^ (w[k] >> 2)) & 0x03030303u;
    t[k] = w[k] ^ __builtin_amdgcn_perm(0u, 0x54474341u, cb[k]);   // 0 where a base
  }
  // code byte of word k (first base in the top bits) in bits 24..31 of
  // top[k]: cb | cb << 10 | cb << 20 | cb << 30, no two terms overlap there
  uint32_t top[4];
  #pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t t1 = shl_or<10>(cb[k], cb[k]);
    top[k] = shl_or<20>(t1, t1);
  }
  packed = __builtin_amdgcn_perm(top[0], top[1], 0x07030C0Cu) |
           __builtin_amdgcn_perm(top[2], top[3], 0x0C0C0703u);
  inv = 0;
  if ((t[0] | t[1] | t[2] | t[3]) != 0) {
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t nz = (((t[k] & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t[k]) & 0x80808080u;
      inv |= (((nz >> 7) * 0x01020408u) >> 24) << (4 * k);
    }
  }
}

// ASCII bytes [g, g+16) of the text (misaligned or crossing its end: byte
// loads, 0 past the end, which reads as a non-base).
__device__ __forceinline__ u32x4 gather16(const TextRef& r, uint64_t g) {
  uint32_t w[4];
  #pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t y = 0;
    #pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint64_t q = g + 4 * k + b;
      y |= (uint32_t)(q < r.n ? r.t[q] : 0u) << (8 * b);
    }
    w[k] = y;
  }
  return u32x4{w[0], w[1], w[2], w[3]};
}

__device__ __forceinline__ uint32_t gather4(const TextRef& r, uint64_t g) {
  uint32_t y = 0;
  #pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint64_t q = g + b;
    y |= (uint32_t)(q < r.n ? r.t[q] : 0u) << (8 * b);
  }
  return y;
}

// 2-bit chunk c (64 bases) -> four code words and 64 invalid bits.
__device__ __forceinline__ void commit_2bit_chunk(const TextRef& r, uint32_t c, bool loaded,
                                                  const u32x4& v, uint32_t* pk, uint32_t* iv) {
  uint16_t* iv16 = reinterpret_cast<uint16_t*>(iv);
  uint32_t w[4] = {v.x, v.y, v.z, v.w};
  uint32_t inv[4] = {0, 0, 0, 0};
  if (!loaded) {
    const uint64_t g = r.t0 + 64ull * c;
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t y = 0, m = 0;
      for (int b = 0; b < 16; ++b) {
        const uint64_t q = g + 16 * k + b;
        if (q < r.n) y |= (uint32_t)((r.t[q >> 2] >> (2 * (q & 3))) & 3u) << (2 * b);
        else m |= 1u << b;
      }
      w[k] = y;
      inv[k] = m;
    }
  }
  #pragma unroll
  for (int k = 0; k < 4; ++k) {
    // base b sits in bits 2b..2b+1: reverse the order of the 2-bit fields
    const uint32_t rv = __builtin_bitreverse32(w[k]);
    pk[4 * c + k] = ((rv >> 1) & 0x55555555u) | ((rv & 0x55555555u) << 1);
    iv16[4 * c + k] = (uint16_t)inv[k];
  }
}

// Convert the prefetched text of a tile into the wave's LDS area.  ASCII:
// every lane converts its 16-byte chunk of the tile; the halo is converted
// in 4-byte pieces, one per lane (one byte of codes and four invalid bits
// each; two neighbouring lanes join their invalid bits into one byte).
template <uint32_t TILE>
__device__ __forceinline__ void commit(const TextRef& r, uint32_t halo, const Prefetch& f,
                                       uint32_t* pk, uint32_t* iv) {
  const uint32_t lane = fresh_lane();
  const uint32_t span = TILE + halo;
  if (r.enc == PFAC_TEXT_ASCII) {
    uint32_t packed, inv;
    ascii_chunk((f.fast & 1u) ? f.a : gather16(r, r.t0 + 16ull * lane), packed, inv);
    pk[lane] = packed;
    reinterpret_cast<uint16_t*>(iv)[lane] = (uint16_t)inv;
    if (TILE == 2048) {
      ascii_chunk((f.fast & 2u) ? f.b : gather16(r, r.t0 + 1024 + 16ull * lane), packed, inv);
      pk[64 + lane] = packed;
      reinterpret_cast<uint16_t*>(iv)[64 + lane] = (uint16_t)inv;
    }
    uint8_t* pk8 = reinterpret_cast<uint8_t*>(pk);
    uint8_t* iv8 = reinterpret_cast<uint8_t*>(iv);
    const uint32_t npieces = halo / 4;
    for (uint32_t p0 = 0; p0 < npieces; p0 += 64) {
      const uint32_t pc = p0 + lane;
      const uint32_t v = (p0 == 0 && (f.fast & 4u)) ? f.h : gather4(r, r.t0 + TILE + 4ull * pc);
      uint32_t code8, inv4;
      ascii4(v, code8, inv4);
      // invalid bits of lane ^ 1 (quad permutation 1,0,3,2)
      const uint32_t other = (uint32_t)__builtin_amdgcn_mov_dpp((int)inv4, 0xB1, 0xF, 0xF, false);
      if (pc < npieces) {
        // bases TILE+4pc .. +3: byte 3 - (pc & 3) of code word TILE/16 + pc/4
        pk8[4 * (TILE / 16 + (pc >> 2)) + 3 - (pc & 3)] = (uint8_t)code8;
        if (!(pc & 1u)) iv8[(TILE + 4 * pc) / 8] = (uint8_t)(inv4 | (other << 4));
      }
    }
  } else {
    const uint32_t nch = span / 64;
    if (lane < nch) commit_2bit_chunk(r, lane, f.fast & 1u, f.a, pk, iv);
    if (lane + 64 < nch) commit_2bit_chunk(r, lane + 64, f.fast & 2u, f.b, pk, iv);
  }
  if (lane < 2) {
    pk[span / 16 + lane] = 0;
    iv[span / 32 + lane] = 0xFFFFFFFFu;
  }
}

// LDS of one wave, in 32-bit words, each part a multiple of 4 words so the
// 16-byte LDS accesses stay aligned: text codes (+2 sentinel words), invalid
// bits (+2), deep-walk results, deep-walk queue and the list of queue entries
// that pass the second filter (16-bit entries).
__host__ __device__ constexpr uint32_t round4(uint32_t x) { return (x + 3) & ~3u; }
__host__ __device__ constexpr uint32_t pk_words(uint32_t tile, uint32_t halo) {
  return round4((tile + halo) / 16 + 2);
}
__host__ __device__ constexpr uint32_t iv_words(uint32_t tile, uint32_t halo) {
  return round4((tile + halo) / 32 + 2);
}
// LDS of one wave of the global-memory variant: results and queue.
constexpr uint32_t kGlobalWaveWords = kQueue + kQueue / 2;
// Trie-level descriptors copied into LDS after the image and the second filter.
constexpr uint32_t kLvlWords = 4 * kImageLevels;
// After the waves' areas: the workgroup's tile counter (padded to 16 bytes).
constexpr uint32_t kCtlWords = 4;
__host__ __device__ constexpr uint32_t wave_words(uint32_t tile, uint32_t halo) {
  return pk_words(tile, halo) + iv_words(tile, halo) + kQueue + kQueue / 2 + kQueue / 2;
}

// A tile's text and place.  One-text launches read their one segment (text
// and output at offset 0) from the parameters instead, and ts = gtile there.
struct TileLoc {
  DevSeg seg;       // batch only
  uint64_t ts;      // tile index within its text
  uint64_t gtile;   // tile index in the call
};

template <bool SINGLE>
__device__ __forceinline__ TileLoc locate(const ScanParams& p, uint64_t lt) {
  TileLoc L;
  if (SINGLE) {
    L.ts = lt;
    L.gtile = lt;
  } else {
    uint32_t lo = 0, hi = p.ngroup;   // prefix[lo] <= lt < prefix[hi]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (p.group_prefix[mid] <= lt) lo = mid; else hi = mid;
    }
    const uint32_t si = p.group_segs[lo];
    L.seg = p.segs[si];
    L.ts = lt - p.group_prefix[lo];
    L.gtile = p.tile_prefix[si] + L.ts;
  }
  return L;
}

// Per-tile counts of a scan.  Atomic stores: deferred walks of the same
// launch add to them with atomics.
__device__ __forceinline__ void put_counts(const ScanParams& p, uint64_t tile, uint32_t hits,
                                           unsigned long long occ) {
  __hip_atomic_store(&p.tile_hits[tile], hits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p.tile_occ[tile], occ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One deferred walk (one-text launches): the depth-D jump entry of the
// window, then the walk with path compression over the 64 bases copied with
// the entry, continued on the text in global memory past them.  A pattern
// found is written to the dense output and appended to its tile's hit slots
// (the finish kernel orders each tile's slots by position).
template <uint32_t D>
__device__ __forceinline__ void deferred_walk(const ScanParams& p, const WalkEntry& we) {
  const u32x4 a = reinterpret_cast<const u32x4*>(&we)[0];
  const u32x4 b = reinterpret_cast<const u32x4*>(&we)[1];
  const uint32_t pos = a.x;
  const uint32_t c0 = a.z, c1 = a.w, c2 = b.x, c3 = b.y;
  const uint64_t ivall = ((uint64_t)b.w << 32) | b.z;
  const uint64_t n = p.seg0.n;
  const uint32_t enc = p.seg0.enc;
  int32_t best = 0;
  unsigned long long occ = 0;
  uint32_t s = 0, q = 0;
  bool live = true;
  if (!a.y) {
    const uint32_t x = c0 >> (32 - 2 * D);
    const uint32_t jj = p.jump[x];
    if (jj & kFinalBit) {
      const OutEntry o = p.jres[x];
      best = o.pid;
      occ += o.mult;
    }
    s = jj & kStateMask;
    q = D;
    live = s != 0;
  }
  while (live) {
    if (q >= kWindow) {
      // past the copied bases: go on reading the text itself
      walk<true>(s, (uint64_t)pos + q, nullptr, nullptr, p.next, p.out, p.text, n, enc, best,
                 occ);
      break;
    }
    const uint32_t wk = q >> 4, sh = 2 * (q & 15u);
    const uint32_t hi = wk == 0 ? c0 : wk == 1 ? c1 : wk == 2 ? c2 : c3;
    const uint32_t lo = wk == 0 ? c1 : wk == 1 ? c2 : wk == 2 ? c3 : 0u;
    const uint32_t win = (uint32_t)(((((uint64_t)hi << 32) | lo) << sh) >> 32);
    const uint32_t ivw = (uint32_t)(ivall >> q);
    const u32x2 ch = *reinterpret_cast<const u32x2*>(p.chain + 2ull * s);
    const uint32_t e = p.next[(uint64_t)s * 4 + (win >> 30)];
    const uint32_t len = ch.x & 15u;
    if (len >= 2) {
      if (q + len > kWindow) {
        // the run reaches past the copied bases
        walk<true>(s, (uint64_t)pos + q, nullptr, nullptr, p.next, p.out, p.text, n, enc, best,
                   occ);
        break;
      }
      if ((ivw & ((1u << len) - 1u)) | ((win ^ ch.x) & (0xFFFFFFFFu << (32 - 2 * len)))) break;
      s = ch.y & kStateMask;
      q += len;
      if (ch.y & kFinalBit) {
        const OutEntry o = p.out[s];
        best = o.pid;
        occ += o.mult;
      }
      continue;
    }
    if ((ivw & 1u) || e == 0) break;
    s = e & kStateMask;
    if (e & kFinalBit) {
      const OutEntry o = p.out[s];
      best = o.pid;
      occ += o.mult;
    }
    ++q;
  }
  const uint64_t gt = pos / kTileSingle;
  if (best) {
    if (p.match) p.match[pos] = best;
    const uint32_t slot = atomicAdd(&p.tile_hits[gt], 1u);
    if (p.slots && slot < kSlot) p.slots[gt * kSlot + slot] = Slot{pos, best};
  }
  if (occ) atomicAdd(&p.tile_occ[gt], occ);
}

// Zero dense output of a whole tile of nt positions (mt 16-byte aligned or
// not), the lane's NG groups of four.
template <uint32_t NG>
__device__ __forceinline__ void zero_tile(int32_t* mt, uint32_t nt, bool aligned) {
  const uint32_t lane = threadIdx.x & 63;
  const i32x4 z = {0, 0, 0, 0};
  if (aligned && nt == NG * 256) {
    #pragma unroll
    for (uint32_t g = 0; g < NG; ++g)
      __builtin_nontemporal_store(z, reinterpret_cast<i32x4*>(mt + g * 256) + lane);
    return;
  }
  #pragma unroll 1
  for (uint32_t g = 0; g < NG; ++g) {
    const uint32_t q0 = g * 256 + 4 * lane;
    if (aligned && q0 + 4 <= nt) {
      __builtin_nontemporal_store(z, reinterpret_cast<i32x4*>(mt + q0));
    } else {
      if (q0 < nt) mt[q0] = 0;
      if (q0 + 1 < nt) mt[q0 + 1] = 0;
      if (q0 + 2 < nt) mt[q0 + 2] = 0;
      if (q0 + 3 < nt) mt[q0 + 3] = 0;
    }
  }
}

// Main scan.  Each wave takes whole tiles of TILE positions (grid-stride).  A
// lane owns 4*NG positions of a tile, NG = TILE/256 groups of four
// consecutive ones: q = g*256 + 4*lane + r.  Positions whose walk goes on past the filter are
// queued and walked by all lanes together; their results come back through
// a result slot per queue entry.
template <int BLOCK, bool GLOBAL, int DT, bool SINGLE, bool DEFER>
__global__ __launch_bounds__(BLOCK) void pfac_scan_kernel(ScanParams p) {
  extern __shared__ uint32_t lds[];
  // the wave index is uniform across the wave: keep it (and every tile
  // index and text offset derived from it) in scalar registers
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr uint32_t D = GLOBAL ? 0u : (uint32_t)DT;   // filter depth (compile time)
  constexpr uint32_t TILE = SINGLE ? kTileSingle : kTileBatch;
  constexpr uint32_t NG = TILE / 256;                   // groups of 4 positions per lane
  const uint32_t img_words = GLOBAL ? 0u : p.image_words;
  uint32_t* bm = lds;                             // image: filter bitmap first
  const uint32_t* bmpre = lds + (GLOBAL ? 0u : (1u << (2 * D)) / 32);
  // all LDS is dynamic (no static arrays), so its base is the constant 0
  const bool hashed = !GLOBAL && p.hash_on;
  const uint32_t* hl = lds + img_words;           // second-filter bitmap
  uint32_t* pk = nullptr;
  uint32_t* iv = nullptr;
  int32_t* res;
  uint16_t* queue;
  uint16_t* queue2 = nullptr;
  // tiles are handed out to the workgroup's waves one at a time from a
  // counter in LDS: waves that the CU issues more often take more tiles, and
  // all end within about one tile of each other
  uint32_t* ctl;
  if (GLOBAL) {
    res = reinterpret_cast<int32_t*>(lds + wave * kGlobalWaveWords);
    queue = reinterpret_cast<uint16_t*>(res + kQueue);
    ctl = lds + (BLOCK / 64) * kGlobalWaveWords;
  } else {
    ctl = lds + img_words + (hashed ? p.hash_words : 0u) + kLvlWords +
          (BLOCK / 64) * wave_words(TILE, p.halo);
    pk = lds + img_words + (hashed ? p.hash_words : 0u) + kLvlWords +
         wave * wave_words(TILE, p.halo);
    iv = pk + pk_words(TILE, p.halo);
    res = reinterpret_cast<int32_t*>(iv + iv_words(TILE, p.halo));
    queue = reinterpret_cast<uint16_t*>(res + kQueue);
    queue2 = queue + kQueue;
  }

  if (!GLOBAL) {
    const u32x4* src = reinterpret_cast<const u32x4*>(p.image);
    u32x4* dst = reinterpret_cast<u32x4*>(bm);
    for (uint32_t i = threadIdx.x; i < img_words / 4; i += BLOCK) dst[i] = src[i];
    if (hashed) {
      const u32x4* hs = reinterpret_cast<const u32x4*>(p.hash);
      u32x4* hd = reinterpret_cast<u32x4*>(bm + img_words);
      for (uint32_t i = threadIdx.x; i < p.hash_words / 4; i += BLOCK) hd[i] = hs[i];
    }
    if (p.lds_trie && threadIdx.x < kLvlWords / 4)
      reinterpret_cast<u32x4*>(bm + img_words + (hashed ? p.hash_words : 0u))[threadIdx.x] =
          p.lvl[threadIdx.x];
  }
  if (threadIdx.x == 0) ctl[0] = BLOCK / 64;   // wave w starts with local tile w
  __syncthreads();
  const u32x4* lvl = reinterpret_cast<const u32x4*>(lds + img_words +
                                                    (hashed ? p.hash_words : 0u));

  const uint32_t dmask = (1u << D) - 1u;
  const uint32_t gmask = (1u << (D + 3)) - 1u;   // bases of the 4 windows of a group
  // byte selector of the 4 bases the lane's group starts at within a pair of
  // code words {first, second}: bytes 7-k .. 4-k of the pair, k = lane & 3
  const uint32_t k8 = lane & 3u;
  const uint32_t bsel = ((7u - k8) << 24) | ((6u - k8) << 16) | ((5u - k8) << 8) | (4u - k8);
  const uint32_t sh4 = 4u * (lane & 7u);          // its bit in the invalid-bit word
  const uint64_t nwaves = (uint64_t)gridDim.x * (BLOCK / 64);
  const uint32_t gwave = blockIdx.x * (BLOCK / 64) + wave;
  uint64_t lt = gwave;
  uint32_t wq_n = 0;                                // deferred walks of this wave
  WalkEntry* wq = DEFER ? p.wq + (uint64_t)gwave * p.wq_cap : nullptr;
  if (lt >= p.local_tiles) return;
  TileLoc cur = locate<SINGLE>(p, lt);
  Prefetch pf{};
  // the all-zero dense output and the counters of the previous tile, written
  // after the next tile's text is in LDS: the wait for that text (the
  // vector-memory counter also counts stores, completing in issue order) then
  // does not wait for stores issued just before it
  int32_t* zmt = nullptr;
  uint32_t znt = 0;
  bool zal = false;
  bool cpend = false;
  uint64_t ctile = 0;
  uint32_t chits = 0;
  unsigned long long cocc = 0;
  // the segment of a tile: one-text launches have text and output at offset 0
  auto seg_n = [&](const TileLoc& L) -> uint64_t { return SINGLE ? p.seg0.n : L.seg.n; };
  auto seg_enc = [&](const TileLoc& L) -> uint32_t { return SINGLE ? p.seg0.enc : L.seg.enc; };
  auto seg_text = [&](const TileLoc& L) -> const uint8_t* {
    return SINGLE ? p.text : p.text + L.seg.text_off;
  };
  auto seg_match = [&](const TileLoc& L) -> int32_t* {
    return SINGLE ? p.match : p.match + L.seg.match_off;
  };
  if (!GLOBAL)
    pf = fetch<TILE>(TextRef{seg_text(cur), seg_n(cur), cur.ts * TILE, seg_enc(cur)}, p.halo);

  for (;;) {
    const uint64_t t0 = cur.ts * TILE;
    const uint64_t n = seg_n(cur);
    const uint32_t nt = (uint32_t)((n - t0) < TILE ? (n - t0) : TILE);  // positions in text
    const bool full = nt == TILE;
    const uint8_t* text = seg_text(cur);
    const uint32_t enc = seg_enc(cur);
    const uint64_t gtile = cur.gtile;
    int32_t* mt = p.match ? seg_match(cur) + t0 : nullptr;
    const bool maligned = mt && ((reinterpret_cast<uintptr_t>(mt) & 15) == 0);

    if (!GLOBAL) {
      commit<TILE>(TextRef{text, n, t0, enc}, p.halo, pf, pk, iv);
      wave_sync();
    }
    // next tile: take it, locate it and start loading its text now.  Local
    // tile i of workgroup b is b*W + i%W + (i/W)*nwaves (W waves per
    // workgroup), increasing in i: the first one past the end ends the wave
    const uint32_t li = __builtin_amdgcn_readfirstlane(lane == 0 ? atomicAdd(ctl, 1u) : 0u);
    const uint64_t lt_next = (uint64_t)blockIdx.x * (BLOCK / 64) + li % (BLOCK / 64) +
                             (uint64_t)(li / (BLOCK / 64)) * nwaves;
    const bool more = lt_next < p.local_tiles;
    TileLoc nxt = cur;
    if (more) {
      nxt = locate<SINGLE>(p, lt_next);
      if (!GLOBAL)
        pf = fetch<TILE>(TextRef{seg_text(nxt), seg_n(nxt), nxt.ts * TILE, seg_enc(nxt)},
                         p.halo);
    }
    if (DEFER && zmt) {
      zero_tile<NG>(zmt, znt, zal);
      zmt = nullptr;
    }
    if (cpend) {
      if (lane == 0) put_counts(p, ctile, chits, cocc);
      cpend = false;
    }

    // ---- classify the lane's 4*NG positions: bit 4g+r of want / slow
    uint32_t want = 0, slow = 0;
    #pragma unroll
    for (uint32_t g = 0; g < NG; ++g) {
      const uint32_t q0 = g * 256 + 4 * lane;
      const uint32_t vmask =
          full ? 0xFu : (q0 >= nt ? 0u : (nt - q0 >= 4 ? 0xFu : (1u << (nt - q0)) - 1u));
      uint32_t m4 = 0, s4 = 0;
      if (GLOBAL) {
        m4 = s4 = vmask;
      } else {
        const uint32_t wi = q0 >> 4, ii = q0 >> 5;
        // 16 bases from q0, first base in the top bits
        const uint32_t w = __builtin_amdgcn_perm(pk[wi], pk[wi + 1], bsel);
        const uint32_t inv = __builtin_amdgcn_alignbit(iv[ii + 1], iv[ii], sh4);
        // window key x_r = bits [o_r, o_r+2D) of w, o_r = 32-2r-2D: its
        // bitmap word is bits [o_r+5, o_r+2D) (read at byte offset 4x that)
        // and its bit within the word bits [o_r, o_r+5) (a bit-field offset
        // uses the low 5 bits of its operand).  All four reads are issued
        // before the first is used.
        uint32_t word[4];
        #pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
          const uint32_t o = 32 - 2 * r - 2 * D;
          word[r] = lds_word((w >> (o + 3)) & (((1u << (2 * D - 5)) - 1u) << 2));
        }
        #pragma unroll
        for (uint32_t r = 0; r < 4; ++r)
          m4 |= __builtin_amdgcn_ubfe(word[r], w >> (32 - 2 * r - 2 * D), 1u) << r;
        if (inv & gmask) {
          // a window holds a non-base (or runs past the text): such
          // positions walk from the root -- or, when every pattern is longer
          // than D, report nothing (no pattern fits before the non-base)
          #pragma unroll
          for (uint32_t r = 0; r < 4; ++r)
            if ((inv >> r) & dmask) s4 |= 1u << r;
          if (p.longer) {
            m4 &= ~s4;
            s4 = 0;
          } else {
            m4 |= s4;
          }
        }
        m4 &= vmask;
        s4 &= vmask;
      }
      want |= m4 << (4 * g);
      slow |= s4 << (4 * g);
    }

    // ---- queue the surviving positions (lane order, then position order):
    //      one pass over the whole tile when the queue holds it, else one
    //      pass per group of positions
    unsigned long long occ = 0;
    uint32_t tile_hits = 0;
    uint32_t total;
    const uint32_t base = wave_excl_dpp(__builtin_popcount(want), &total);
    const uint32_t passes = total <= kQueue ? 1u : NG;
    for (uint32_t pass = 0; pass < passes; ++pass) {
      const uint32_t sel = passes == 1 ? (0xFFFFFFFFu >> (32 - 4 * NG)) : (0xFu << (4 * pass));
      const uint32_t wsel = want & sel;
      uint32_t pbase = base, ptotal = total;
      if (passes != 1) pbase = wave_excl_dpp(__builtin_popcount(wsel), &ptotal);
      {
        uint32_t m = wsel, k = pbase;
        while (m) {
          const uint32_t bit = __builtin_ctz(m);
          m &= m - 1u;
          const uint32_t q = (bit >> 2) * 256 + 4 * lane + (bit & 3);
          queue[k++] = (uint16_t)(q | (((slow >> bit) & 1u) << 15));
        }
      }
      wave_sync();
      // ---- second filter: queue entries that must walk on, listed in queue2
      uint32_t nwalk = ptotal;
      if (hashed) {
        nwalk = 0;
        #pragma unroll 1
        for (uint32_t i0 = 0; i0 < ptotal; i0 += 64) {
          const uint32_t i = i0 + lane;
          bool go = false;
          if (i < ptotal) {
            res[i] = 0;
            go = hash_pass(queue[i], pk, iv, hl, p.hash_kmask, p.hash_imask, p.hash_shift);
          }
          const uint64_t m = __ballot(go);
          if (go)
            queue2[nwalk + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
                (uint16_t)i;
          nwalk += (uint32_t)__popcll(m);
        }
        wave_sync();
      }
      // ---- launches with deferred walks keep them for the end of the
      //      wave: each lane copies an entry into the wave's own part of the
      //      buffer; the entries that do not fit there are walked here
      uint32_t ndef = 0;
      if (DEFER && nwalk > 0) {
        const uint32_t wbase = wq_n;
        ndef = min(nwalk, p.wq_cap - wq_n);
        wq_n += ndef;
        #pragma unroll 1
        for (uint32_t j = lane; j < ndef; j += 64) {
          const uint32_t i = hashed ? (uint32_t)queue2[j] : j;
          const uint32_t e = queue[i];
          const uint32_t qt = e & 0x7FFFu;
          const uint32_t wi = qt >> 4, sh = 2 * (qt & 15u);
          const uint32_t ii = qt >> 5, s5 = qt & 31u;
          u32x4 c;
          c.x = (uint32_t)(((((uint64_t)pk[wi] << 32) | pk[wi + 1]) << sh) >> 32);
          c.y = (uint32_t)(((((uint64_t)pk[wi + 1] << 32) | pk[wi + 2]) << sh) >> 32);
          c.z = (uint32_t)(((((uint64_t)pk[wi + 2] << 32) | pk[wi + 3]) << sh) >> 32);
          c.w = (uint32_t)(((((uint64_t)pk[wi + 3] << 32) | pk[wi + 4]) << sh) >> 32);
          const uint32_t inv0 = __builtin_amdgcn_alignbit(iv[ii + 1], iv[ii], s5);
          const uint32_t inv1 = __builtin_amdgcn_alignbit(iv[ii + 2], iv[ii + 1], s5);
          // entry = {pos, slow, codes[0..1]}, {codes[2..3], inv[0..1]}
          u32x4* dst = reinterpret_cast<u32x4*>(wq + wbase + j);
          dst[0] = u32x4{(uint32_t)(t0 + qt), (e >> 15) & 1u, c.x, c.y};
          dst[1] = u32x4{c.z, c.w, inv0, inv1};
          res[i] = 0;       // the deferred walk writes its result
        }
      }
      // ---- walk them with all lanes
      uint32_t nz = 0;
      #pragma unroll 1
      for (uint32_t j = ndef + lane; j < nwalk; j += 64) {
        const uint32_t i = hashed ? (uint32_t)queue2[j] : j;
        const uint32_t e = queue[i];
        const uint32_t qt = e & 0x7FFFu;                 // index within the tile
        int32_t best = 0;
        if (GLOBAL) {
          walk<true>(0u, t0 + qt, nullptr, nullptr, p.next, p.out, text, n, enc, best, occ);
        } else {
          best = deep_walk(e, D, p.lds_trie, p.levels, lds, bmpre, lvl, pk, iv, p.next, p.out,
                           p.jump, p.jres, p.chain, occ);
        }
        res[i] = best;
        nz |= (uint32_t)best;
      }
      // almost every pass ends with no walk reporting a pattern: then the
      // dense output of its positions is all zero and it has no hits
      const bool any = __ballot(nz != 0) != 0;
      wave_sync();
      // ---- the groups of this pass: pick up results, dense output, hits
      #pragma unroll 1
      for (uint32_t g = 0; g < NG; ++g) {
        if (!((sel >> (4 * g)) & 1u)) continue;
        const uint32_t q0 = g * 256 + 4 * lane;
        if (!any) {
          if (DEFER && mt && passes == 1) {
            // the whole tile is zero: written with the next tile
            zmt = mt;
            znt = nt;
            zal = maligned;
            break;
          }
          if (mt) {
            const i32x4 z = {0, 0, 0, 0};
            if (maligned && q0 + 4 <= nt) {
              __builtin_nontemporal_store(z, reinterpret_cast<i32x4*>(mt + q0));
            } else {
              if (q0 < nt) mt[q0] = 0;
              if (q0 + 1 < nt) mt[q0 + 1] = 0;
              if (q0 + 2 < nt) mt[q0 + 2] = 0;
              if (q0 + 3 < nt) mt[q0 + 3] = 0;
            }
          }
          continue;
        }
        int32_t vv[4];
        #pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
          const uint32_t bit = 4 * g + r;
          vv[r] = ((wsel >> bit) & 1u) ? res[pbase + __builtin_popcount(wsel & ((1u << bit) - 1u))]
                                       : 0;
        }
        const i32x4 v = {vv[0], vv[1], vv[2], vv[3]};
        if (mt) {
          if (maligned && q0 + 4 <= nt) {
            __builtin_nontemporal_store(v, reinterpret_cast<i32x4*>(mt + q0));
          } else {
            if (q0 < nt) mt[q0] = v.x;
            if (q0 + 1 < nt) mt[q0 + 1] = v.y;
            if (q0 + 2 < nt) mt[q0 + 2] = v.z;
            if (q0 + 3 < nt) mt[q0 + 3] = v.w;
          }
        }
        const bool any = (vv[0] | vv[1] | vv[2] | vv[3]) != 0;
        if (__ballot(any)) {
          const uint32_t c = (vv[0] != 0) + (vv[1] != 0) + (vv[2] != 0) + (vv[3] != 0);
          uint32_t tot;
          uint32_t o = tile_hits + wave_excl_dpp(c, &tot);
          if (p.slots) {
            Slot* sl = p.slots + gtile * kSlot;
            #pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {
              if (vv[r]) {
                if (o < kSlot) sl[o] = Slot{(uint32_t)(t0 + q0 + r), vv[r]};
                ++o;
              }
            }
          }
          tile_hits += tot;
        }
      }
      wave_sync();
    }
    cocc = __ballot(occ != 0) ? wave_sum(occ) : 0ull;
    chits = tile_hits;
    ctile = gtile;
    cpend = true;
    if (!more) break;
    lt = lt_next;
    cur = nxt;
  }
  if (DEFER && zmt) zero_tile<NG>(zmt, znt, zal);
  if (lane == 0) put_counts(p, ctile, chits, cocc);
  if constexpr (DEFER) {
    if (wq_n) {
      // the deferred walks of this wave's tiles, one per lane: their results
      // go over the zeros and counts stored above, so those stores complete
      // first
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      #pragma unroll 1
      for (uint32_t j = lane; j < wq_n; j += 64) deferred_walk<D>(p, wq[j]);
    }
  }
}

// Parameters of the finish kernel.
struct FinishParams {
  const uint32_t* tile_hits;
  const unsigned long long* tile_occ;
  Slot* slots;
  uint64_t tiles;
  uint32_t tile;                  // start positions per tile
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
      if (!p.single) {
        text = text_of_tile(p, t);
        seg = p.segs[text];
        ts = t - p.tile_prefix[text];
        tab = p.tables[seg.table];
      }
      const uint64_t t0 = ts * p.tile;
      const uint8_t* tx = p.text + seg.text_off;
      for (uint32_t k = 0; k < p.tile / 256; ++k) {   // 64 lanes x 4 positions per step
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

// Library-owned scratch of one (device, stream): per-tile counts and hit
// slots, block sums, the reduce ticket, and batch descriptor copies.  Calls
// on one stream use it in stream order.
struct Workspace {
  uint8_t* mem = nullptr;
  uint64_t cap_tiles = 0;
  uint32_t* tile_hits = nullptr;
  unsigned long long* tile_occ = nullptr;
  Slot* slots = nullptr;
  unsigned long long* status = nullptr;     // finish kernel: look-back word per workgroup
  unsigned long long* block_occ = nullptr;
  uint32_t* sync = nullptr;                 // finish kernel: ticket, finished look-backs
  void* batch = nullptr;           // descriptors, prefixes, group lists, table views
  uint64_t batch_cap = 0;
  uint8_t* stage = nullptr;        // pinned host copy of `batch` being uploaded
  hipEvent_t staged = nullptr;     // recorded after the upload that read `stage`
  bool staged_pending = false;
  WalkEntry* walk = nullptr;       // deferred walks of one-text calls
  uint64_t walk_cap = 0;           // entries
};

static std::map<std::pair<int, void*>, Workspace*> g_ws;

static int ensure_tiles(Workspace* ws, uint64_t tiles, hipStream_t stream) {
  if (tiles <= ws->cap_tiles && ws->mem) return PFAC_OK;
  const uint64_t cap = std::max<uint64_t>(tiles + tiles / 4, 4096);
  const uint64_t blocks = (cap + kRedTiles - 1) / kRedTiles;
  auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
  const uint64_t o_hits = 0;
  const uint64_t o_occ = al(o_hits + cap * 4);
  const uint64_t o_slots = al(o_occ + cap * 8);
  const uint64_t o_st = al(o_slots + cap * kSlot * sizeof(Slot));
  const uint64_t o_bo = al(o_st + blocks * 8);
  const uint64_t o_sync = al(o_bo + blocks * 8);
  const uint64_t total = al(o_sync + 256);
  if (ws->mem) {
    if (hipStreamSynchronize(stream) != hipSuccess) return PFAC_E_HIP;
    (void)hipFree(ws->mem);
    ws->mem = nullptr;
    ws->cap_tiles = 0;
  }
  void* m = nullptr;
  if (hipMalloc(&m, total) != hipSuccess) return PFAC_E_NOMEM;
  ws->mem = static_cast<uint8_t*>(m);
  // look-back words and counters start at zero; the finish kernel leaves them so
  if (hipMemset(ws->mem + o_st, 0, total - o_st) != hipSuccess) return PFAC_E_HIP;
  ws->cap_tiles = cap;
  ws->tile_hits = reinterpret_cast<uint32_t*>(ws->mem + o_hits);
  ws->tile_occ = reinterpret_cast<unsigned long long*>(ws->mem + o_occ);
  ws->slots = reinterpret_cast<Slot*>(ws->mem + o_slots);
  ws->status = reinterpret_cast<unsigned long long*>(ws->mem + o_st);
  ws->block_occ = reinterpret_cast<unsigned long long*>(ws->mem + o_bo);
  ws->sync = reinterpret_cast<uint32_t*>(ws->mem + o_sync);
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

// Room for `cap` deferred walks (grown, never shrunk).
static int ensure_walk(Workspace* ws, uint64_t cap, hipStream_t stream) {
  if (cap <= ws->walk_cap && ws->walk) return PFAC_OK;
  if (ws->walk) {
    if (hipStreamSynchronize(stream) != hipSuccess) return PFAC_E_HIP;
    (void)hipFree(ws->walk);
    ws->walk = nullptr;
    ws->walk_cap = 0;
  }
  void* m = nullptr;
  if (hipMalloc(&m, cap * sizeof(WalkEntry)) != hipSuccess) return PFAC_E_NOMEM;
  ws->walk = static_cast<WalkEntry*>(m);
  ws->walk_cap = cap;
  return PFAC_OK;
}

static Workspace* get_workspace(int dev, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace*& ws = g_ws[{dev, (void*)stream}];
  if (!ws) ws = new (std::nothrow) Workspace();
  return ws;
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

// LDS of a scan launch.  The planner sizes for the larger (one-text) tile, so
// a plan fits both kinds of launch.
static uint32_t scan_lds_bytes(uint32_t block, uint32_t img_words, uint32_t halo,
                               uint32_t tile = kTileSingle) {
  return 4u * (img_words + kLvlWords + (block / 64) * wave_words(tile, halo) + kCtlWords);
}

using ScanFn = void (*)(ScanParams);

template <int BLOCK, bool SINGLE, bool DEFER>
static ScanFn pick_depth(uint32_t D) {
  switch (D) {
    case 6: return pfac_scan_kernel<BLOCK, false, 6, SINGLE, DEFER>;
    case 7: return pfac_scan_kernel<BLOCK, false, 7, SINGLE, DEFER>;
    case 8: return pfac_scan_kernel<BLOCK, false, 8, SINGLE, DEFER>;
    case 9: return pfac_scan_kernel<BLOCK, false, 9, SINGLE, DEFER>;
    case 10: return pfac_scan_kernel<BLOCK, false, 10, SINGLE, DEFER>;
    default: return nullptr;
  }
}

// One instantiation per (workgroup size, filter depth, one text or a batch,
// walks at once or deferred): the depth fixes every window shift at compile
// time, a one-text launch carries none of the batch bookkeeping, and only
// launches with deferred walks (few survivors per tile) carry their hand-off
// and the deferred zero stores.
template <int BLOCK>
static ScanFn pick_block(bool global, uint32_t D, bool single, bool defer) {
  if (global)
    return single ? pfac_scan_kernel<BLOCK, true, 0, true, false>
                  : pfac_scan_kernel<BLOCK, true, 0, false, false>;
  if (!single) return pick_depth<BLOCK, false, false>(D);
  return defer ? pick_depth<BLOCK, true, true>(D) : pick_depth<BLOCK, true, false>(D);
}

static ScanFn pick_scan(uint32_t block, bool global, uint32_t D, bool single, bool defer) {
  switch (block) {
    case 256: return pick_block<256>(global, D, single, defer);
    case 512: return pick_block<512>(global, D, single, defer);
    case 768: return pick_block<768>(global, D, single, defer);
    case 1024: return pick_block<1024>(global, D, single, defer);
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

// Second-filter size the library picks: the largest bitmap (fewest windows
// let through; its LDS fits beside a depth-9 bitmap and 1024 threads' text)
// while the patterns number at most 40 % of its bits (beyond that it passes
// too much to pay for its lookups).  Smaller bitmaps were measured no faster
// on 1,000 to 10,000 patterns.
static uint32_t auto_hash_bits(const HostTable& h) {
  if ((double)h.num_patterns <= 0.4 * (double)(1u << kHashMaxBits)) return kHashMaxBits;
  return PFAC_HASH_NONE;
}

constexpr int kNoFit = 1;

// Place the depth-D image in LDS next to `hw` words of second filter: with
// every pattern longer than D, rank words and as many trie levels as asked
// for (levels 0 = as many as fit); otherwise, or with PFAC_LEVELS_NONE, the
// bare filter bitmap.  Sets p->levels on success; kNoFit when it does not fit.
static int place_image(const HostTable& h, uint32_t D, uint32_t hw, uint32_t halo,
                       uint32_t budget, pfac_plan* p) {
  if (h.min_len > D && p->levels != PFAC_LEVELS_NONE) {
    const uint32_t have = h.image[D].levels;
    const uint32_t want = p->levels == 0 ? have : std::min(p->levels, have);
    for (int32_t L = (int32_t)want; L >= 0; --L) {
      if (scan_lds_bytes(p->block, image_words(h, D, true, (uint32_t)L) + hw, halo) <= budget) {
        if (p->levels != 0 && (uint32_t)L < want) return kNoFit;   // explicit, too big
        p->levels = (uint32_t)L;
        return PFAC_OK;
      }
    }
    if (p->levels != 0) return kNoFit;
  }
  // filter bitmap only; survivors read the global depth-D jump table
  if (scan_lds_bytes(p->block, image_words(h, D, false, 0) + hw, halo) <= budget) {
    p->levels = PFAC_LEVELS_NONE;
    return PFAC_OK;
  }
  return kNoFit;
}

static int resolve_plan(const pfac_plan* in, const HostTable& h, int dev, pfac_plan* out) {
  const DeviceInfo di = device_info(dev);
  if (!di.ok) return PFAC_E_NODEV;
  pfac_plan p = in ? *in : pfac_plan{0, 0, 0, 0, 0, 0, 0};
  if (p.variant != PFAC_VARIANT_TILED && p.variant != PFAC_VARIANT_GLOBAL) return PFAC_E_ARG;
  const uint32_t halo = halo_for(h.max_len);
  if (p.variant == PFAC_VARIANT_TILED && halo > kMaxHalo) {
    if (in && in->depth) return PFAC_E_ARG;
    p.variant = PFAC_VARIANT_GLOBAL;  // patterns too long to stage a halo in LDS
  }
  // Library choice when every pattern is longer than the filter depth and
  // the second filter is worth keeping: bitmap + second filter only (the few
  // windows that pass both are walked from the global jump table), depth 9
  // when the patterns' first K bases go past it (a 32 KB bitmap next to the
  // filter), in 1024-thread workgroups -- measured faster than keeping trie
  // levels in LDS, whose walks the second filter has already cut down, and
  // than shallower bitmaps or 512-thread workgroups.  Otherwise 1024-thread
  // workgroups and as many LDS trie levels as fit.
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
  // with the workgroup size left to the library, a depth whose image does
  // not fit beside 1024 threads' text tries 512, then 256, before a
  // shallower depth
  if (p.block == 0) p.block = 1024;
  if (p.block != 256 && p.block != 512 && p.block != 768 && p.block != 1024) return PFAC_E_ARG;
  if (p.walks != 0 && p.walks != PFAC_WALKS_INLINE && p.walks != PFAC_WALKS_DEFERRED)
    return PFAC_E_ARG;
  if (p.variant == PFAC_VARIANT_GLOBAL) {
    p.depth = 0;
    p.levels = PFAC_LEVELS_NONE;
    p.hash_bits = PFAC_HASH_NONE;
    p.walks = PFAC_WALKS_INLINE;
    *out = p;
    return PFAC_OK;
  }
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
    // when the image does not fit beside it, the library's choice drops it
    // before it drops trie levels or depth
    uint32_t hb = PFAC_HASH_NONE;
    if (h.hash_k > D && p.hash_bits != PFAC_HASH_NONE)
      hb = auto_h ? auto_hash_bits(h) : p.hash_bits;
    const uint32_t block0 = p.block;
    for (;;) {
      const uint32_t hw = hb == PFAC_HASH_NONE ? 0u : (1u << hb) / 32;
      const int rc = place_image(h, D, hw, halo, budget, &p);
      if (rc == PFAC_OK) {
        p.hash_bits = hb;
        // walks that survive the second filter are few: keep them for the end
        // of the wave so the streaming scan never waits on their table reads
        // -- when the 64 bases copied with each cover every pattern (past
        // them a deferred walk reads the text one base at a time)
        if (p.walks == 0)
          p.walks = (hb != PFAC_HASH_NONE && h.max_len <= kWindow) ? PFAC_WALKS_DEFERRED
                                                                    : PFAC_WALKS_INLINE;
        *out = p;
        return PFAC_OK;
      }
      if (rc != kNoFit) return rc;
      if (auto_b && p.block > 256) {
        p.block = p.block > 512 ? 512 : 256;
        continue;
      }
      if (hb == PFAC_HASH_NONE || !auto_h) break;
      hb = PFAC_HASH_NONE;
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
  const uint64_t waves = plan.block / 64;
  const uint64_t need = (tiles + waves - 1) / waves;
  if (g > need) g = need;
  return g ? g : 1;
}

// Kernel, dynamic LDS and grid of a scan launch.
static int scan_shape(const ScanParams& sp, const pfac_plan& plan, int dev, ScanFn* fn,
                      uint32_t* lds, uint64_t* grid) {
  const bool global = plan.variant == PFAC_VARIANT_GLOBAL;
  *fn = pick_scan(plan.block, global, sp.D, sp.single != 0, sp.defer != 0);
  if (!*fn) return PFAC_E_ARG;
  *lds = global ? 4u * ((plan.block / 64) * kGlobalWaveWords + kCtlWords)
                : scan_lds_bytes(plan.block, sp.image_words + (sp.hash_on ? sp.hash_words : 0u),
                                 sp.halo, sp.single ? kTileSingle : kTileBatch);
  *grid = grid_for(*fn, plan, *lds, dev, sp.local_tiles);
  return PFAC_OK;
}

static int launch_scan(const ScanParams& sp, const pfac_plan& plan, int dev, hipStream_t stream) {
  if (sp.local_tiles == 0) return PFAC_OK;
  ScanFn fn;
  uint32_t lds;
  uint64_t grid;
  const int rc = scan_shape(sp, plan, dev, &fn, &lds, &grid);
  if (rc) return rc;
  if (sp.defer && grid * (plan.block / 64) > sp.wq_waves) return PFAC_E_ARG;
  hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(plan.block), lds, stream, sp);
  return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
}

static int launch_tail(Workspace* ws, uint64_t tiles, unsigned long long* counters,
                       FinishParams* sc, bool want_hits, hipStream_t stream) {
  const uint32_t blocks = (uint32_t)((tiles + kRedTiles - 1) / kRedTiles);
  sc->tile_hits = ws->tile_hits;
  sc->tile_occ = ws->tile_occ;
  sc->slots = ws->slots;
  sc->tiles = tiles;
  sc->status = ws->status;
  sc->block_occ = ws->block_occ;
  sc->sync = ws->sync;
  sc->counters = counters;
  if (!want_hits) {
    sc->hits = nullptr;
    sc->hit_cap = 0;
  }
  hipLaunchKernelGGL(pfac_finish_kernel, dim3(blocks), dim3(1024), 0, stream, *sc);
  return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
}

static void fill_table(ScanParams& sp, const pfac_table* t, const pfac_plan& pl) {
  sp.next = t->dev.next;
  sp.out = t->dev.out;
  sp.chain = t->dev.chain;
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
    sp.lvl = reinterpret_cast<const u32x4*>(t->dev.levels[D]);
    if (pl.hash_bits != PFAC_HASH_NONE) {
      const uint32_t b = pl.hash_bits, K = h.hash_k;
      sp.hash_on = 1;
      sp.hash = t->dev.hash[b];
      sp.hash_words = (1u << b) / 32;
      sp.hash_shift = 32 - b;
      sp.hash_kmask = K >= 16 ? 0xFFFFFFFFu : ~((1u << (32 - 2 * K)) - 1u);
      sp.hash_imask = (1u << K) - 1u;
    }
  }
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

const char* pfac_version(void) { return "pfac-mi355x 0.2 (gfx950)"; }

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
  // one device allocation: next | out | per depth: jump, jres, bitmap
  auto align = [](uint64_t x) { return (x + 255) / 256 * 256; };
  uint64_t off = 0;
  const uint64_t o_next = off; off = align(off + h.next.size() * 4);
  const uint64_t o_out = off; off = align(off + h.out.size() * sizeof(OutEntry));
  const uint64_t o_chain = off; off = align(off + h.chain.size() * 4);
  uint64_t o_jump[kMaxJump + 1] = {}, o_jres[kMaxJump + 1] = {}, o_im[kMaxJump + 1] = {};
  uint64_t o_lv[kMaxJump + 1] = {};
  std::vector<uint32_t> lvdesc[kMaxJump + 1];
  for (uint32_t D = kMinJump; D <= kMaxJump; ++D) {
    o_jump[D] = off; off = align(off + h.jump[D].size() * 4);
    o_jres[D] = off; off = align(off + h.jres[D].size() * sizeof(OutEntry));
    o_im[D] = off; off = align(off + h.image[D].words.size() * 4);
    lvdesc[D].assign(4 * kImageLevels, 0);
    for (uint32_t k = 0; k < kImageLevels; ++k) {
      if (k < h.image[D].levels) {
        lvdesc[D][4 * k] = h.image[D].byte_off[k];
        lvdesc[D][4 * k + 1] = h.image[D].pre_off[k];
      }
      if (D + k < h.depth_start.size()) lvdesc[D][4 * k + 2] = (uint32_t)h.depth_start[D + k];
    }
    o_lv[D] = off; off = align(off + lvdesc[D].size() * 4);
  }
  uint64_t o_hash[kHashMaxBits + 1] = {};
  for (uint32_t b = kHashMinBits; b <= kHashMaxBits; ++b) {
    o_hash[b] = off; off = align(off + h.hash[b].size() * 4);
  }
  if (hipMalloc(&t->dmem, off) != hipSuccess) {
    delete t;
    return PFAC_E_NOMEM;
  }
  t->dbytes = off;
  char* base = static_cast<char*>(t->dmem);
  auto put = [&](uint64_t o, const void* src, size_t bytes) {
    return hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  bool ok = put(o_next, h.next.data(), h.next.size() * 4) &&
            put(o_out, h.out.data(), h.out.size() * sizeof(OutEntry)) &&
            put(o_chain, h.chain.data(), h.chain.size() * 4);
  DevTable& v = t->dev;
  memset(&v, 0, sizeof(v));
  v.next = reinterpret_cast<const uint32_t*>(base + o_next);
  v.out = reinterpret_cast<const OutEntry*>(base + o_out);
  v.chain = reinterpret_cast<const uint32_t*>(base + o_chain);
  v.num_states = (uint32_t)h.num_states;
  v.max_len = h.max_len;
  for (uint32_t D = kMinJump; D <= kMaxJump; ++D) {
    ok = ok && put(o_jump[D], h.jump[D].data(), h.jump[D].size() * 4) &&
         put(o_jres[D], h.jres[D].data(), h.jres[D].size() * sizeof(OutEntry)) &&
         put(o_im[D], h.image[D].words.data(), h.image[D].words.size() * 4) &&
         put(o_lv[D], lvdesc[D].data(), lvdesc[D].size() * 4);
    v.levels[D] = reinterpret_cast<const uint32_t*>(base + o_lv[D]);
    v.jump[D] = reinterpret_cast<const uint32_t*>(base + o_jump[D]);
    v.jres[D] = reinterpret_cast<const OutEntry*>(base + o_jres[D]);
    v.image[D] = reinterpret_cast<const uint32_t*>(base + o_im[D]);
  }
  for (uint32_t b = kHashMinBits; b <= kHashMaxBits; ++b) {
    if (!h.hash[b].empty()) ok = ok && put(o_hash[b], h.hash[b].data(), h.hash[b].size() * 4);
    v.hash[b] = reinterpret_cast<const uint32_t*>(base + o_hash[b]);
  }
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
  return resolve_plan(nullptr, t->host, t->device, out);
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
  int rc = resolve_plan(plan, t->host, dev, &pl);
  if (rc) return rc;
  unsigned long long* counters = reinterpret_cast<unsigned long long*>(d_counters);
  const uint64_t tiles = (n + kTileSingle - 1) / kTileSingle;
  if (tiles == 0) {
    hipLaunchKernelGGL(pfac_zero_kernel, dim3(1), dim3(64), 0, stream, counters, 2u);
    return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
  }
  Workspace* ws = get_workspace(dev, stream);
  if (!ws) return PFAC_E_NOMEM;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    rc = ensure_tiles(ws, tiles, stream);
  }
  if (rc) return rc;
  ScanParams sp;
  memset(&sp, 0, sizeof(sp));
  fill_table(sp, t, pl);
  sp.halo = pl.variant == PFAC_VARIANT_TILED ? halo_for(t->host.max_len) : 0;
  sp.single = 1;
  sp.seg0 = DevSeg{0, n, 0, 0, (uint32_t)enc};
  sp.local_tiles = tiles;
  sp.text = static_cast<const uint8_t*>(d_text);
  sp.match = d_match;
  sp.tile_hits = ws->tile_hits;
  sp.tile_occ = ws->tile_occ;
  sp.slots = d_hits ? ws->slots : nullptr;
  const bool defer = pl.variant == PFAC_VARIANT_TILED && pl.walks == PFAC_WALKS_DEFERRED;
  if (defer) {
    // every scan wave gets room for 4 walks per tile it will scan (about
    // four times what the second filter lets through on random-like text;
    // walks beyond it run at once) and walks them after its last tile
    // (the kernel, hence its grid, depends on `defer`: set it first)
    sp.defer = 1;
    ScanFn fn;
    uint32_t lds;
    uint64_t grid;
    rc = scan_shape(sp, pl, dev, &fn, &lds, &grid);
    if (rc) return rc;
    const uint64_t nwaves = grid * (pl.block / 64);
    const uint64_t per = std::max<uint64_t>(4 * ((tiles + nwaves - 1) / nwaves), 64);
    {
      std::lock_guard<std::mutex> lk(g_mu);
      rc = ensure_walk(ws, per * nwaves, stream);
    }
    if (rc) return rc;
    sp.wq = ws->walk;
    sp.wq_cap = (uint32_t)per;
    sp.wq_waves = nwaves;
  }
  rc = launch_scan(sp, pl, dev, stream);
  if (rc) return rc;
  FinishParams sc;
  memset(&sc, 0, sizeof(sc));
  sc.hits = d_hits;
  sc.hit_cap = hit_cap;
  sc.single = 1;
  sc.tile = kTileSingle;
  sc.seg0 = sp.seg0;
  sc.text = sp.text;
  sc.match = d_match;
  sc.tab0 = t->dev;
  return launch_tail(ws, tiles, counters, &sc, d_hits != nullptr && hit_cap > 0, stream);
}

}  // extern "C"

namespace pfac {

// Host-side layout of a batch: per-table plans, global tile numbering in
// text order, per table its texts and their local tile prefixes, and the
// byte layout of the device copy (descriptors | tile prefix | per table: text
// list, local prefix | table views).
struct BatchLayout {
  std::vector<const pfac_table*> tables;
  std::vector<pfac_plan> plans;
  std::vector<DevSeg> segs;
  std::vector<uint64_t> tile_prefix;
  std::vector<std::vector<uint32_t>> groups;
  std::vector<std::vector<uint64_t>> local_prefix;
  std::vector<uint64_t> o_gs, o_gp;
  uint64_t o_segs = 0, o_tp = 0, o_tab = 0, bytes = 0, tiles = 0;
  uint32_t num_texts = 0;
};

static uint64_t al256(uint64_t x) { return (x + 255) / 256 * 256; }

static int layout_batch(const pfac_table* const* tables, uint32_t num_tables,
                        const pfac_text_desc* descs, uint32_t num_texts, const pfac_plan* plan,
                        int dev, BatchLayout* L) {
  if (!tables || num_tables == 0 || (num_texts && !descs)) return PFAC_E_ARG;
  for (uint32_t i = 0; i < num_tables; ++i)
    if (!tables[i] || tables[i]->device != dev) return PFAC_E_ARG;
  for (uint32_t s = 0; s < num_texts; ++s) {
    const pfac_text_desc& d = descs[s];
    if (d.n >= (1ull << 32) || d.table >= num_tables ||
        (d.enc != PFAC_TEXT_ASCII && d.enc != PFAC_TEXT_2BIT))
      return PFAC_E_ARG;
  }
  L->tables.assign(tables, tables + num_tables);
  L->plans.resize(num_tables);
  for (uint32_t i = 0; i < num_tables; ++i) {
    const int rc = resolve_plan(plan, tables[i]->host, dev, &L->plans[i]);
    if (rc) return rc;
  }
  L->num_texts = num_texts;
  L->segs.resize(num_texts);
  if (num_texts) memcpy(L->segs.data(), descs, num_texts * sizeof(DevSeg));
  L->tile_prefix.assign(num_texts + 1, 0);
  for (uint32_t s = 0; s < num_texts; ++s)
    L->tile_prefix[s + 1] = L->tile_prefix[s] + (descs[s].n + kTileBatch - 1) / kTileBatch;
  L->tiles = L->tile_prefix[num_texts];
  L->groups.assign(num_tables, {});
  for (uint32_t s = 0; s < num_texts; ++s)
    if (descs[s].n) L->groups[descs[s].table].push_back(s);
  L->local_prefix.assign(num_tables, {});
  L->o_gs.assign(num_tables, 0);
  L->o_gp.assign(num_tables, 0);
  uint64_t off = 0;
  L->o_segs = off; off = al256(off + num_texts * sizeof(DevSeg));
  L->o_tp = off; off = al256(off + (num_texts + 1) * 8);
  for (uint32_t g = 0; g < num_tables; ++g) {
    std::vector<uint64_t>& lp = L->local_prefix[g];
    lp.assign(L->groups[g].size() + 1, 0);
    for (size_t i = 0; i < L->groups[g].size(); ++i)
      lp[i + 1] = lp[i] + (descs[L->groups[g][i]].n + kTileBatch - 1) / kTileBatch;
    L->o_gs[g] = off; off = al256(off + L->groups[g].size() * 4);
    L->o_gp[g] = off; off = al256(off + lp.size() * 8);
  }
  L->o_tab = off; off = al256(off + num_tables * sizeof(DevTable));
  L->bytes = off;
  return PFAC_OK;
}

static void fill_batch(const BatchLayout& L, uint8_t* host) {
  memset(host, 0, L.bytes);
  if (L.num_texts) memcpy(host + L.o_segs, L.segs.data(), L.num_texts * sizeof(DevSeg));
  memcpy(host + L.o_tp, L.tile_prefix.data(), L.tile_prefix.size() * 8);
  for (size_t g = 0; g < L.tables.size(); ++g) {
    if (!L.groups[g].empty())
      memcpy(host + L.o_gs[g], L.groups[g].data(), L.groups[g].size() * 4);
    memcpy(host + L.o_gp[g], L.local_prefix[g].data(), L.local_prefix[g].size() * 8);
  }
  for (size_t i = 0; i < L.tables.size(); ++i)
    memcpy(host + L.o_tab + i * sizeof(DevTable), &L.tables[i]->dev, sizeof(DevTable));
}

// Enqueue the kernels of a batch whose layout is already on the device at
// db: one scan launch per table, then reduce, scatter and per-text totals.
// Kernel launches only (no allocation, copy or memset).
static int enqueue_batch(const BatchLayout& L, const Workspace* ws, const uint8_t* db,
                         const void* d_text_base, int32_t* d_match_base,
                         pfac_batch_hit* d_hits, uint64_t hit_cap, unsigned long long* counters,
                         int dev, hipStream_t stream) {
  if (L.tiles == 0) {
    hipLaunchKernelGGL(pfac_zero_kernel, dim3(1), dim3(256), 0, stream, counters,
                       2u + 2u * L.num_texts);
    return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
  }
  for (size_t g = 0; g < L.tables.size(); ++g) {
    const uint64_t gt = L.local_prefix[g].back();
    if (gt == 0) continue;
    ScanParams sp;
    memset(&sp, 0, sizeof(sp));
    fill_table(sp, L.tables[g], L.plans[g]);
    sp.halo = L.plans[g].variant == PFAC_VARIANT_TILED ? halo_for(L.tables[g]->host.max_len) : 0;
    sp.single = 0;
    sp.ngroup = (uint32_t)L.groups[g].size();
    sp.segs = reinterpret_cast<const DevSeg*>(db + L.o_segs);
    sp.group_segs = reinterpret_cast<const uint32_t*>(db + L.o_gs[g]);
    sp.group_prefix = reinterpret_cast<const uint64_t*>(db + L.o_gp[g]);
    sp.tile_prefix = reinterpret_cast<const uint64_t*>(db + L.o_tp);
    sp.local_tiles = gt;
    sp.text = static_cast<const uint8_t*>(d_text_base);
    sp.match = d_match_base;
    sp.tile_hits = ws->tile_hits;
    sp.tile_occ = ws->tile_occ;
    sp.slots = d_hits ? ws->slots : nullptr;
    const int rc = launch_scan(sp, L.plans[g], dev, stream);
    if (rc) return rc;
  }
  FinishParams sc;
  memset(&sc, 0, sizeof(sc));
  sc.hits = d_hits;
  sc.hit_cap = hit_cap;
  sc.single = 0;
  sc.tile = kTileBatch;
  sc.nsegs = L.num_texts;
  sc.segs = reinterpret_cast<const DevSeg*>(db + L.o_segs);
  sc.tile_prefix = reinterpret_cast<const uint64_t*>(db + L.o_tp);
  sc.text = static_cast<const uint8_t*>(d_text_base);
  sc.match = d_match_base;
  sc.tables = reinterpret_cast<const DevTable*>(db + L.o_tab);
  const int rc = launch_tail(const_cast<Workspace*>(ws), L.tiles, counters, &sc,
                             d_hits != nullptr && hit_cap > 0, stream);
  if (rc) return rc;
  hipLaunchKernelGGL(pfac_text_totals_kernel, dim3((L.num_texts + 3) / 4), dim3(256), 0, stream,
                     ws->tile_hits, ws->tile_occ, sc.tile_prefix, L.num_texts, counters + 2);
  return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
}

static bool text_base_ok(const BatchLayout& L, const void* d_text_base) {
  if (d_text_base) return true;
  for (const DevSeg& d : L.segs)
    if (d.n) return false;
  return true;
}

static void free_workspace(Workspace* ws) {
  if (ws->mem) (void)hipFree(ws->mem);
  if (ws->batch) (void)hipFree(ws->batch);
  if (ws->stage) (void)hipHostFree(ws->stage);
  if (ws->staged) (void)hipEventDestroy(ws->staged);
  if (ws->walk) (void)hipFree(ws->walk);
  *ws = Workspace();
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
  if (L.tiles == 0) return enqueue_batch(L, nullptr, nullptr, d_text_base, d_match_base, d_hits,
                                         hit_cap, counters, dev, stream);
  Workspace* ws = get_workspace(dev, stream);
  if (!ws) return PFAC_E_NOMEM;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    rc = ensure_tiles(ws, L.tiles, stream);
    if (!rc) rc = ensure_batch(ws, L.bytes, stream);
  }
  if (rc) return rc;
  fill_batch(L, ws->stage);
  if (hipMemcpyAsync(ws->batch, ws->stage, L.bytes, hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      hipEventRecord(ws->staged, stream) != hipSuccess)
    return PFAC_E_HIP;
  ws->staged_pending = true;
  return enqueue_batch(L, ws, static_cast<const uint8_t*>(ws->batch), d_text_base, d_match_base,
                       d_hits, hit_cap, counters, dev, stream);
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
    rc = ensure_tiles(&b->ws, b->layout.tiles, nullptr);
    if (!rc) rc = ensure_batch(&b->ws, b->layout.bytes, nullptr);
    if (!rc) {
      fill_batch(b->layout, b->ws.stage);
      if (hipMemcpy(b->ws.batch, b->ws.stage, b->layout.bytes, hipMemcpyHostToDevice) !=
          hipSuccess)
        rc = PFAC_E_HIP;
    }
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
  return enqueue_batch(b->layout, &b->ws, static_cast<const uint8_t*>(b->ws.batch), d_text_base,
                       d_match_base, d_hits, hit_cap,
                       reinterpret_cast<unsigned long long*>(d_counters), dev,
                       static_cast<hipStream_t>(stream));
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
