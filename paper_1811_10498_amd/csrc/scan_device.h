// Device code of the PFAC scan: helpers, text staging, walks and the scan
// kernel template.  Included by the instantiation units (one per workgroup
// size and launch kind, compiled in parallel) and by the host API unit.
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
//   * Prefix filter (large pattern sets, where a hashed bitmap fills up): an
//     exact bitmap of every pattern's first K2 bases (4^K2 bits, at most
//     2 MB, read from L2) tested by the survivors of the LDS filter.
//   * Deep walks: the surviving positions of a wave are compacted into an
//     LDS queue and walked by all 64 lanes together (or, when they are rare,
//     after the wave's last tile): one global read of the depth-D jump
//     table, then the breadth-first numbered next-state table (L2 /
//     Infinity Cache resident), runs of single-child states in one step.
//   * Text: each wave stages its tile (256, 1024 or 2048 positions) plus a
//     halo of max_len-1 bases with 16-byte loads, as 2-bit codes plus an
//     "invalid" bit per base (bytes other than A,C,G,T, and everything past
//     the end).
//   * Outputs: the dense int32 array leaves with 16-byte non-temporal
//     stores; hits are counted per tile and parked in a fixed-size slot per
//     tile; one finish kernel (decoupled look-back over its workgroups)
//     places them in position order.  No scan workgroup waits for another.
#pragma once

#include <hip/hip_runtime.h>

#include "pfac_internal.h"

namespace pfac {

// Start positions per wave tile (a template parameter of the scan): 2048 by
// default (the fixed cost of a tile -- staging, locating, one round of deep
// walks -- spread over more positions), 256 for the short texts of a batch
// (a 150-base read then leaves less of its tile empty), 1024 on request and
// for the global-memory variants of a batch.
constexpr uint32_t kTileSingle = 2048;
constexpr uint32_t kTileBatch = 1024;
constexpr uint32_t kTileShort = 256;
// Scratch areas of pre-zeroing scans: one per workgroup slot (workgroup
// index mod kPzSlots), kTileSingle int32 each.
constexpr uint32_t kPzSlots = 256;
constexpr uint32_t kQueue = 256;       // deep-walk queue entries per wave
constexpr uint32_t kSlot = 32;         // hits parked per tile
constexpr uint32_t kMaxHalo = 4096;    // longest halo staged in LDS (bases)
constexpr uint32_t kRedTiles = 4096;   // tiles per finish workgroup

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// A text of a launch, as the device sees it: where its bases and its dense
// output start, its length, the index of its first tile among the tiles of
// the call (counts and hit slots), its table, its encoding and the log2 of
// the positions per tile the layout gave it.
struct DevSeg {
  uint64_t text_off;
  uint64_t match_off;
  uint32_t n;
  uint32_t first_tile;
  uint32_t table;
  uint16_t enc;
  uint16_t tile_shift;
};
static_assert(sizeof(DevSeg) == 32, "descriptor layout");

// One work item of a batched launch: everything a wave needs to start its
// tile (the text's offsets, length and encoding, the tile's index within the
// text and within the call, the text's index), so that locating the next
// tile is one 32-byte load instead of an item load and a dependent
// descriptor load.
struct TileItem {
  uint64_t text_off;
  uint64_t match_off;
  uint32_t n;
  uint32_t gtile;       // tile index in the call
  uint32_t ts;          // tile index within the text
  uint32_t si_enc;      // text index in bits 0..30, encoding in bit 31
};
static_assert(sizeof(TileItem) == 32, "work item layout");

struct Slot {
  uint32_t pos;
  int32_t pid;
};

// A walk deferred to the end of the wave that found it: its start position
// within its text, bit 0 of `slow` set when its window held a non-base
// within the first D bases (then it walks from the root) and bits 1..31 the
// text's index (batched launches), and a copy of the next kWindow bases
// (2-bit codes, 16 per word, first base in the top bits of codes[0];
// invalid bits, base k in bit k of inv).
constexpr uint32_t kWindow = 64;
struct WalkEntry {
  uint32_t pos;
  uint32_t slow;
  uint32_t codes[4];
  uint32_t inv[2];
};
static_assert(sizeof(WalkEntry) == 32, "walk entry layout");

// Parameters of the scan kernel (one table per launch).
struct ScanParams {
  const uint32_t* next;
  const OutEntry* out;
  const uint32_t* chain;          // runs of single-child steps (TILED)
  const u32x4* node;              // per state {next[4]}, {run record, output} (TILED)
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
  uint32_t pair;                  // 1: the LDS image is the depth-D pair table
  uint32_t hash_cls;              // 1 (K <= 12 only): the second filter is the one-hash
                                  // form (`hash` its bitmap), and tiles with only
                                  // A/C/G/T staged test it on every window while
                                  // classifying (large pattern sets, whose depth-D
                                  // bitmap lets most windows through)
  uint32_t hash_kshift;           // hash_cls: 32 - 2K (the key's shift to the right)
  // the paper's layouts of the transition table (global-memory variants):
  // next state and matched pattern ID per cell as two arrays, or merged
  const uint32_t* next2;          // [S*4] child state, 0 = none
  const int32_t* cell_pid;        // [S*4] ID of the pattern ending at the child, 0 = none
  const u32x2* cells;             // [S*4] {child state, pattern ID}
  const uint32_t* pfx;            // prefix filter: 4^K2-bit bitmap in global memory
  uint32_t pfx_on;
  uint32_t pfx_shift;             // 32 - 2*K2 (the K2-base key is the top 2*K2 bits)
  uint32_t pfx_imask;             // (1 << K2) - 1
  uint32_t halo;                  // staged bases past the tile, multiple of 64
  DevSeg seg0;                    // one-text launches: the text (offsets 0)
  const DevSeg* segs;             // batch: all texts of the call
  const TileItem* items;          // batch: the work items of this launch
  uint64_t local_tiles;           // tiles (one text) or work items (batch) of the launch
  const uint8_t* text;
  int32_t* match;
  uint32_t* tile_hits;            // [tiles of the call]
  unsigned long long* tile_occ;   // [tiles of the call]
  Slot* slots;                    // [tiles * kSlot] or nullptr
  // deferred walks: every wave owns wq_cap entries of wq (wave w from
  // w*wq_cap) and walks them after its last tile
  uint32_t defer;
  uint32_t wq_cap;
  WalkEntry* wq;
  uint64_t wq_waves;              // waves wq has room for
  int32_t* pz_dummy;              // pre-zeroing kernels: kPzSlots areas of kTileSingle
                                  // int32, written in place of a tile that is not full
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

// The walk from the root over the text in global memory with the paper's
// transition table layouts (Sec. V.B, VII): LAYOUT 1 reads the next state and
// the matched pattern ID of a cell from two arrays, LAYOUT 2 from one array
// of merged cells; a cell with an ID also reads the state's occurrence count.
template <int LAYOUT>
__device__ __forceinline__ void walk_cells(uint64_t q, const ScanParams& p, const uint8_t* gtext,
                                           uint64_t gn, uint32_t genc, int32_t& best,
                                           unsigned long long& occ) {
  uint32_t s = 0;
  for (;;) {
    const int b = global_base(gtext, gn, genc, q);
    if (b < 0) break;
    const uint64_t cell = (uint64_t)s * 4 + (uint32_t)b;
    uint32_t nx;
    int32_t id;
    if (LAYOUT == 1) {
      nx = p.next2[cell];
      id = p.cell_pid[cell];
    } else {
      const u32x2 c = p.cells[cell];
      nx = c.x;
      id = (int32_t)c.y;
    }
    if (nx == 0) break;
    s = nx;
    if (id) {
      best = id;
      occ += p.out[s].mult;
    }
    ++q;
  }
}

// The walk over LDS text with path compression: at a state with a run of
// single-child steps (chain record, see the table layout) the next bases are
// compared with the whole run at once -- all of them match and the walk jumps
// to the end of the run, or the walk ends inside it, where no pattern ends.
// A step reads the state's node record: the edge word of the next base and
// the run record with the state's output, from one cache line, so a step
// costs one round trip either way.  `fin`: s is final and its output is
// still to be counted (it comes with s's record).
__device__ __forceinline__ void walk_lds(uint32_t s, uint32_t q, const uint32_t* __restrict__ pk,
                                         const uint32_t* __restrict__ iv,
                                         const u32x4* __restrict__ node, bool fin,
                                         int32_t& best, unsigned long long& occ) {
  for (;;) {
    // validity bits and codes of the 16 bases from q (first base on top)
    const uint32_t ivw = __builtin_amdgcn_alignbit(iv[(q >> 5) + 1], iv[q >> 5], q & 31u);
    const uint32_t win =
        (uint32_t)(((((uint64_t)pk[q >> 4] << 32) | pk[(q >> 4) + 1]) << (2 * (q & 15u))) >> 32);
    const u32x4 nb = node[2ull * s + 1];
    const uint32_t e = reinterpret_cast<const uint32_t*>(node)[8ull * s + (win >> 30)];
    if (fin) {
      best = (int32_t)nb.z;
      occ += nb.w;
    }
    const uint32_t len = nb.x & 15u;
    if (len >= 2) {
      if ((ivw & ((1u << len) - 1u)) | ((win ^ nb.x) & (0xFFFFFFFFu << (32 - 2 * len)))) break;
      s = nb.y & kStateMask;
      fin = (nb.y & kFinalBit) != 0;
      q += len;
      continue;
    }
    if ((ivw & 1u) || e == 0) break;
    s = e & kStateMask;
    fin = (e & kFinalBit) != 0;
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
                                             const u32x4* __restrict__ node,
                                             const OutEntry* __restrict__ out,
                                             const uint32_t* __restrict__ jump,
                                             const OutEntry* __restrict__ jres,
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
      // the state after D steps; the finals passed on the way (the jump
      // entry's output: the longest ID and every occurrence) are counted here
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
  walk_lds(s, q, pk, iv, node, false, best, occ);
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
                                          uint32_t imask, uint32_t shift, bool one,
                                          uint32_t kshift) {
  if (e & 0x8000u) return true;
  const uint32_t qt = e & 0x7FFFu;
  // a non-base among the first K bases: every pattern has at least K bases,
  // so none starts here
  if (__builtin_amdgcn_alignbit(iv[(qt >> 5) + 1], iv[qt >> 5], qt & 31u) & imask) return false;
  const uint32_t wi = qt >> 4;
  const uint32_t key =
      (uint32_t)(((((uint64_t)pk[wi] << 32) | pk[wi + 1]) << (2 * (qt & 15u))) >> 32) & kmask;
  if (one) {
    // the one-hash form: the key right-aligned (at most 24 bits), one 24-bit multiply
    const uint32_t h = (((key >> kshift) & 0xFFFFFFu) * kHash1Mul) >> shift;
    return (hl[h >> 5] >> (h & 31u)) & 1u;
  }
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
    if ((TILE >= 1024 || lane < TILE / 16) && (addr & 15) == 0 && ga + 16 <= r.n) {
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
__device__ __forceinline__ uint32_t commit_2bit_chunk(const TextRef& r, uint32_t c, bool loaded,
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
  return inv[0] | inv[1] | inv[2] | inv[3];
}

// Convert the prefetched text of a tile into the wave's LDS area.  ASCII:
// every lane converts its 16-byte chunk of the tile; the halo is converted
// in 4-byte pieces, one per lane (one byte of codes and four invalid bits
// each; two neighbouring lanes join their invalid bits into one byte).
template <uint32_t TILE>
__device__ __forceinline__ bool commit(const TextRef& r, uint32_t halo, const Prefetch& f,
                                       uint32_t* pk, uint32_t* iv) {
  const uint32_t lane = fresh_lane();
  const uint32_t span = TILE + halo;
  uint32_t any_inv = 0;     // invalid bits this lane staged
  if (r.enc == PFAC_TEXT_ASCII) {
    uint32_t packed, inv;
    if (TILE >= 1024 || lane < TILE / 16) {
      ascii_chunk((f.fast & 1u) ? f.a : gather16(r, r.t0 + 16ull * lane), packed, inv);
      pk[lane] = packed;
      reinterpret_cast<uint16_t*>(iv)[lane] = (uint16_t)inv;
      any_inv |= inv;
    }
    if (TILE == 2048) {
      ascii_chunk((f.fast & 2u) ? f.b : gather16(r, r.t0 + 1024 + 16ull * lane), packed, inv);
      pk[64 + lane] = packed;
      reinterpret_cast<uint16_t*>(iv)[64 + lane] = (uint16_t)inv;
      any_inv |= inv;
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
        any_inv |= inv4;
      }
    }
  } else {
    const uint32_t nch = span / 64;
    if (lane < nch) any_inv |= commit_2bit_chunk(r, lane, f.fast & 1u, f.a, pk, iv);
    if (lane + 64 < nch) any_inv |= commit_2bit_chunk(r, lane + 64, f.fast & 2u, f.b, pk, iv);
  }
  if (lane < 2) {
    pk[span / 16 + lane] = 0;
    iv[span / 32 + lane] = 0xFFFFFFFFu;
  }
  return any_inv != 0;
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
// and output at offset 0) from the parameters instead, and the tile index
// within the call is the tile index within the text there.
struct TileLoc {
  DevSeg seg;       // batch only
  uint32_t si;      // batch: index of the text in the call
  uint64_t ts;      // tile index within its text
  uint64_t gtile;   // tile index in the call
};

template <bool SINGLE>
__device__ __forceinline__ TileLoc locate(const ScanParams& p, uint64_t lt) {
  TileLoc L;
  if (SINGLE) {
    L.si = 0;
    L.ts = lt;
    L.gtile = lt;
  } else {
    const TileItem it = p.items[lt];
    L.si = it.si_enc & 0x7FFFFFFFu;
    L.seg = DevSeg{it.text_off, it.match_off, it.n, 0u, 0u, (uint16_t)(it.si_enc >> 31), 0};
    L.ts = it.ts;
    L.gtile = it.gtile;
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

// The deferred walks of a wave, four per lane at a time: the depth-D jump
// entry of each window, then the walk with path compression over the 64
// bases copied with the entry (continued on the text in global memory past
// them).  Each step reads the state's 32-byte node record (edge words, run
// record, output: one cache line).  The four walks of a lane issue their
// table reads together, so each step waits for one round trip instead of
// four.  A pattern found is written
// to the dense output and appended to its tile's hit slots (the finish
// kernel orders each tile's slots by position).
template <uint32_t D, bool SINGLE, uint32_t TILE>
__device__ __forceinline__ void deferred_walks(const ScanParams& p, const WalkEntry* wq,
                                               uint32_t count) {
  constexpr int M = 4;
  const uint32_t lane = threadIdx.x & 63;
  #pragma unroll 1
  for (uint32_t j0 = 0; j0 < count; j0 += 64 * M) {
    uint32_t pos[M], c[M][4], ivlo[M], ivhi[M], s[M], q[M], si[M];
    int32_t best[M];
    unsigned long long occ[M];
    bool live[M], valid[M], slow[M];
    uint32_t jj[M];
    #pragma unroll
    for (int m = 0; m < M; ++m) {
      const uint32_t j = j0 + 64 * m + lane;
      valid[m] = j < count;
      best[m] = 0;
      occ[m] = 0;
      s[m] = 0;
      q[m] = 0;
      jj[m] = 0;
      if (valid[m]) {
        const u32x4 a = reinterpret_cast<const u32x4*>(wq + j)[0];
        const u32x4 b = reinterpret_cast<const u32x4*>(wq + j)[1];
        pos[m] = a.x;
        slow[m] = (a.y & 1u) != 0;
        si[m] = a.y >> 1;
        c[m][0] = a.z; c[m][1] = a.w; c[m][2] = b.x; c[m][3] = b.y;
        ivlo[m] = b.z;
        ivhi[m] = b.w;
      } else {
        pos[m] = 0; slow[m] = true; si[m] = 0;
        c[m][0] = c[m][1] = c[m][2] = c[m][3] = 0;
        ivlo[m] = ivhi[m] = 0;
      }
    }
    // the jump entries of the windows (walks from the root start at state 0):
    // the finals passed within the first D bases come with the entry's
    // output; every later state's output is read from its node record with
    // its next step
    bool fin[M];
    #pragma unroll
    for (int m = 0; m < M; ++m)
      if (valid[m] && !slow[m]) jj[m] = p.jump[c[m][0] >> (32 - 2 * D)];
    #pragma unroll
    for (int m = 0; m < M; ++m) {
      live[m] = valid[m];
      fin[m] = false;
      if (valid[m] && !slow[m]) {
        if (jj[m] & kFinalBit) {
          const OutEntry o = p.jres[c[m][0] >> (32 - 2 * D)];
          best[m] = o.pid;
          occ[m] += o.mult;
        }
        s[m] = jj[m] & kStateMask;
        q[m] = D;
        live[m] = s[m] != 0;
      }
    }
    for (;;) {
      bool any = false;
      u32x4 nb[M];
      uint32_t win[M], e[M];
      #pragma unroll
      for (int m = 0; m < M; ++m) {
        nb[m] = u32x4{0u, 0u, 0u, 0u};
        e[m] = 0;
        win[m] = 0;
        if (live[m] && q[m] < kWindow) {
          const uint32_t wk = q[m] >> 4, sh = 2 * (q[m] & 15u);
          const uint32_t hi = wk == 0 ? c[m][0] : wk == 1 ? c[m][1] : wk == 2 ? c[m][2] : c[m][3];
          const uint32_t lo = wk == 0 ? c[m][1] : wk == 1 ? c[m][2] : wk == 2 ? c[m][3] : 0u;
          win[m] = (uint32_t)(((((uint64_t)hi << 32) | lo) << sh) >> 32);
          // the state's node record: the edge word of the next base, the run
          // record and the output (one cache line)
          e[m] = reinterpret_cast<const uint32_t*>(p.node)[8ull * s[m] + (win[m] >> 30)];
          nb[m] = p.node[2ull * s[m] + 1];
        }
      }
      #pragma unroll
      for (int m = 0; m < M; ++m) {
        if (!live[m]) continue;
        bool global = q[m] >= kWindow;
        if (!global && fin[m]) {
          best[m] = (int32_t)nb[m].z;
          occ[m] += nb[m].w;
          fin[m] = false;
        }
        const uint32_t len = nb[m].x & 15u;
        if (!global && len >= 2 && q[m] + len > kWindow) global = true;
        if (global) {
          // past the copied bases: go on reading the text itself
          if (fin[m]) {
            const OutEntry o = p.out[s[m]];
            best[m] = o.pid;
            occ[m] += o.mult;
            fin[m] = false;
          }
          const uint8_t* text;
          uint64_t n;
          uint32_t enc;
          if (SINGLE) {
            text = p.text; n = p.seg0.n; enc = p.seg0.enc;
          } else {
            const DevSeg sg = p.segs[si[m]];
            text = p.text + sg.text_off; n = sg.n; enc = sg.enc;
          }
          walk<true>(s[m], (uint64_t)pos[m] + q[m], nullptr, nullptr, p.next, p.out, text, n, enc,
                     best[m], occ[m]);
          live[m] = false;
          continue;
        }
        const uint64_t ivall = ((uint64_t)ivhi[m] << 32) | ivlo[m];
        const uint32_t ivw = (uint32_t)(ivall >> q[m]);
        if (len >= 2) {
          if ((ivw & ((1u << len) - 1u)) | ((win[m] ^ nb[m].x) & (0xFFFFFFFFu << (32 - 2 * len)))) {
            live[m] = false;
            continue;
          }
          s[m] = nb[m].y & kStateMask;
          fin[m] = (nb[m].y & kFinalBit) != 0;
          q[m] += len;
        } else {
          if ((ivw & 1u) || e[m] == 0) {
            live[m] = false;
            continue;
          }
          s[m] = e[m] & kStateMask;
          fin[m] = (e[m] & kFinalBit) != 0;
          ++q[m];
        }
        any = true;
      }
      if (!any) break;
    }
    // results: dense output, hit slot, tile counts
    #pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!valid[m] || (!best[m] && !occ[m])) continue;
      int32_t* match;
      uint64_t gt;
      if (SINGLE) {
        match = p.match;
        gt = pos[m] / TILE;
      } else {
        const DevSeg sg = p.segs[si[m]];
        match = p.match ? p.match + sg.match_off : nullptr;
        gt = (uint64_t)sg.first_tile + pos[m] / TILE;
      }
      if (best[m]) {
        if (match) match[pos[m]] = best[m];
        const uint32_t slot = atomicAdd(&p.tile_hits[gt], 1u);
        if (p.slots && slot < kSlot) p.slots[gt * kSlot + slot] = Slot{pos[m], best[m]};
      }
      if (occ[m]) atomicAdd(&p.tile_occ[gt], occ[m]);
    }
  }
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

// Prefix filter for one queued entry (every pattern has at least K2 > D
// bases, so no entry walks from the root): false when a non-base lies
// among its first K2 bases; otherwise *word receives the index of the
// bitmap word of its K2-base key and *bit the bit within it.
__device__ __forceinline__ bool pfx_locate(uint32_t e, const uint32_t* __restrict__ pk,
                                           const uint32_t* __restrict__ iv, uint32_t shift,
                                           uint32_t imask, uint32_t* word, uint32_t* bit) {
  const uint32_t qt = e & 0x7FFFu;
  if (__builtin_amdgcn_alignbit(iv[(qt >> 5) + 1], iv[qt >> 5], qt & 31u) & imask) return false;
  const uint32_t wi = qt >> 4;
  const uint32_t key =
      (uint32_t)(((((uint64_t)pk[wi] << 32) | pk[wi + 1]) << (2 * (qt & 15u))) >> 32) >> shift;
  *word = key >> 5;
  *bit = key & 31u;
  return true;
}

// Main scan.  GLOBAL: the paper's kernel, every position walks from the root
// with text and table in global memory, DT = the table layout (0 edge words
// with a final bit, 1 two arrays, 2 merged cells); otherwise DT = the filter
// depth D.  Each wave takes whole tiles of TILE positions.  A lane owns
// 4*NG positions of a tile, NG = TILE/256 groups of four consecutive ones:
// q = g*256 + 4*lane + r.  Positions whose walk goes on past the filters are
// queued and walked by all lanes together (or kept for the end of the wave);
// their results come back through a result slot per queue entry.
// A uniform pointer copied into vector registers.  The scan keeps its
// per-tile state in scalar registers; the table pointers the rare paths use
// (walks, filters, hit slots) would otherwise hold scalar registers across
// the tile loop and push that state out into spill lanes.
template <typename T>
__device__ __forceinline__ T* in_vgpr(T* ptr) {
  const uint64_t x = reinterpret_cast<uint64_t>(ptr);
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  asm volatile("v_mov_b32 %0, %1" : "=v"(lo) : "s"(lo));
  asm volatile("v_mov_b32 %0, %1" : "=v"(hi) : "s"(hi));
  // rebuilt as a global-memory pointer: accesses through it stay global
  // (not flat) instructions, whose waits count vector memory only
  typedef __attribute__((address_space(1))) T GT;
  GT* g = reinterpret_cast<GT*>(((uint64_t)hi << 32) | lo);
  return (T*)g;
}

template <int BLOCK, bool GLOBAL, int DT, bool SINGLE, bool DEFER, uint32_t TILE, bool PZ>
__global__ __launch_bounds__(BLOCK) void pfac_scan_kernel(ScanParams p0) {
  static_assert(!PZ || (DEFER && !GLOBAL), "pre-zeroing: deferred-walk scans");
  ScanParams p = p0;
  p.next = in_vgpr(p0.next);
  p.out = in_vgpr(p0.out);
  p.chain = in_vgpr(p0.chain);
  if (SINGLE) p.node = in_vgpr(p0.node);   // (batch kernels: no vector registers to spare)
  p.jump = in_vgpr(p0.jump);
  p.jres = in_vgpr(p0.jres);
  p.pfx = in_vgpr(p0.pfx);
  p.slots = in_vgpr(p0.slots);
  p.tile_hits = in_vgpr(p0.tile_hits);
  p.tile_occ = in_vgpr(p0.tile_occ);
  p.wq = in_vgpr(p0.wq);
  if (GLOBAL) {
    p.next2 = in_vgpr(p0.next2);
    p.cell_pid = in_vgpr(p0.cell_pid);
    p.cells = in_vgpr(p0.cells);
  }
  extern __shared__ uint32_t lds[];
  // the wave index is uniform across the wave: keep it (and every tile
  // index and text offset derived from it) in scalar registers
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr uint32_t D = GLOBAL ? 0u : (uint32_t)DT;   // filter depth (compile time)
  constexpr uint32_t NG = TILE / 256;                   // groups of 4 positions per lane
  static_assert(TILE == 256 || TILE == 1024 || TILE == 2048, "tile size");
  const uint32_t img_words = GLOBAL ? 0u : p.image_words;
  uint32_t* bm = lds;                             // image: filter bitmap first
  const uint32_t* bmpre = lds + (GLOBAL ? 0u : (1u << (2 * D)) / 32);
  // all LDS is dynamic (no static arrays), so its base is the constant 0
  const bool hashed = !GLOBAL && p.hash_on;
  const bool pairm = !GLOBAL && p.pair;           // the image is the pair table
  const bool pfxon = !GLOBAL && p.pfx_on;
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
  // windows with a non-base among their first D bases: they walk from the
  // root (keep_slow all ones) or, when every pattern is longer than D,
  // report nothing (keep_slow 0)
  const uint32_t keep_slow = (GLOBAL || p.longer) ? 0u : 0xFu;
  const uint32_t gmask = (1u << (D + 3)) - 1u;   // bases of the 4 windows of a group
  // byte selector of the 4 bases the lane's group starts at within a pair of
  // code words {first, second}: bytes 7-k .. 4-k of the pair, k = lane & 3
  const uint32_t k8 = lane & 3u;
  const uint32_t bsel = ((7u - k8) << 24) | ((6u - k8) << 16) | ((5u - k8) << 8) | (4u - k8);
  const uint32_t sh4 = 4u * (lane & 7u);          // its bit in the invalid-bit word
  const uint64_t nwaves = (uint64_t)gridDim.x * (BLOCK / 64);
  const uint32_t gwave = blockIdx.x * (BLOCK / 64) + wave;
  uint64_t lt = (uint64_t)wave * gridDim.x + blockIdx.x;
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
  // pre-zeroing (deferred-walk scans with a dense output): a tile's output
  // is zeroed right after its text loads are issued, and its few non-zero
  // positions are written over it later (by the lanes that wrote the zeros,
  // or after the wave's fence).  The eight stores sit in the same block as
  // the loads, so they follow them on every path to the wait for the text,
  // and that wait leaves them in flight (measured on the scan's traffic
  // shape: 0.266 -> 0.239 ms).  Issued at the end of the iteration instead
  // they measured slower (0.311 against 0.294 ms on the large-text scan).  A
  // tile that is not full, or whose output is not 16-byte aligned, writes
  // them to the workgroup's scratch area instead (kTileSingle int32 per
  // workgroup slot) and is written at its end as without pre-zeroing.
  int32_t* const pz_own =
      PZ ? p.pz_dummy + (uint64_t)(blockIdx.x & (kPzSlots - 1)) * kTileSingle : nullptr;
  auto prezero = [&](const TileLoc& L) {
    const uint64_t s0 = L.ts * TILE;
    int32_t* const mb = SINGLE ? p.match : p.match + L.seg.match_off;
    const bool ok = s0 + TILE <= seg_n(L) &&
                    (SINGLE || (reinterpret_cast<uintptr_t>(mb) & 15) == 0);
    int32_t* zt = ok ? mb + s0 : pz_own;
    const i32x4 z = {0, 0, 0, 0};
    #pragma unroll
    for (uint32_t g = 0; g < NG; ++g)
      __builtin_nontemporal_store(z, reinterpret_cast<i32x4*>(zt + g * 256) + lane);
  };
  if (!GLOBAL) {
    pf = fetch<TILE>(TextRef{seg_text(cur), seg_n(cur), cur.ts * TILE, seg_enc(cur)}, p.halo);
    if constexpr (PZ) prezero(cur);
  }

  for (;;) {
    const uint64_t t0 = cur.ts * TILE;
    const uint64_t n = seg_n(cur);
    const uint32_t nt = (uint32_t)((n - t0) < TILE ? (n - t0) : TILE);  // positions in text
    const bool full = nt == TILE;
    const uint8_t* text = seg_text(cur);
    const uint32_t enc = seg_enc(cur);
    const uint64_t gtile = cur.gtile;
    const uint32_t si = cur.si;
    int32_t* mt = p.match ? seg_match(cur) + t0 : nullptr;
    const bool maligned = mt && ((reinterpret_cast<uintptr_t>(mt) & 15) == 0);

    bool dirty = true;   // this lane staged a non-base (or a base past the text)
    if (!GLOBAL) {
      dirty = commit<TILE>(TextRef{text, n, t0, enc}, p.halo, pf, pk, iv);
      wave_sync();
    }
    // next tile: take it, locate it and start loading its text now.  Local
    // tile i of workgroup b (of G) is (i%W)*G + b + (i/W)*nwaves (W waves
    // per workgroup): neighbouring tiles go to neighbouring workgroups, which
    // the dispatcher places on different XCDs (measured 0.8 % faster on the
    // large-text scan than W consecutive tiles per workgroup); increasing in
    // i, so the first one past the end ends the wave
    const uint32_t li = __builtin_amdgcn_readfirstlane(lane == 0 ? atomicAdd(ctl, 1u) : 0u);
    const uint64_t lt_next = (uint64_t)(li % (BLOCK / 64)) * gridDim.x + blockIdx.x +
                             (uint64_t)(li / (BLOCK / 64)) * nwaves;
    const bool more = lt_next < p.local_tiles;
    TileLoc nxt = cur;
    if (more) {
      nxt = locate<SINGLE>(p, lt_next);
      if (!GLOBAL) {
        pf = fetch<TILE>(TextRef{seg_text(nxt), seg_n(nxt), nxt.ts * TILE, seg_enc(nxt)},
                         p.halo);
        if constexpr (PZ) prezero(nxt);
      }
    }
    if (!PZ && DEFER && zmt) {
      zero_tile<NG>(zmt, znt, zal);
      zmt = nullptr;
    }
    if (cpend) {
      if (lane == 0) put_counts(p, ctile, chits, cocc);
      cpend = false;
    }

    // ---- classify the lane's 4*NG positions: bit 4g+r of want / slow.
    //      A full tile whose staged bases are all A/C/G/T (the common case)
    //      takes the short path: one bitmap bit per window, nothing else.
    uint32_t want = 0, slow = 0;
    // bit-field offset of window r's bit within its bitmap word, and the word
    // address: window key x_r = bits [o_r, o_r+2D) of w, o_r = 32-2r-2D; the
    // word is bits [o_r+5, o_r+2D) (read at byte offset 4x that), the bit
    // bits [o_r, o_r+5) (a bit-field offset uses the low 5 bits of its
    // operand).  All four reads of a group are issued before the first is used.
    constexpr uint32_t DL = GLOBAL ? kMinJump : D;      // (unused by the global variants)
    // pair table: byte m = the filter bits of the windows a.m (bits 0..3, by
    // the base a before m) and m.b (bits 4..7, by the base b after m).  The
    // windows at r = 0, 1 share m = bases 1..D-1 of w, those at r = 2, 3
    // m = bases 3..D+1 (base k of w is bits [30-2k, 32-2k)).
    auto pair4 = [&](uint32_t w) -> uint32_t {
      constexpr uint32_t M = (1u << (2 * (DL - 1))) - 1u;
      const uint8_t* pt = reinterpret_cast<const uint8_t*>(lds);
      const uint32_t e0 = pt[(w >> (32 - 2 * DL)) & M];
      const uint32_t e1 = pt[(w >> (28 - 2 * DL)) & M];
      const uint32_t r0 = __builtin_amdgcn_ubfe(e0, w >> 30, 1u);
      const uint32_t r1 = __builtin_amdgcn_ubfe(e0, 4u + ((w >> (30 - 2 * DL)) & 3u), 1u);
      const uint32_t r2 = __builtin_amdgcn_ubfe(e1, (w >> 26) & 3u, 1u);
      const uint32_t r3 = __builtin_amdgcn_ubfe(e1, 4u + ((w >> (26 - 2 * DL)) & 3u), 1u);
      return r0 | (r1 << 1) | (r2 << 2) | (r3 << 3);
    };
    auto lookup4 = [&](uint32_t w) -> uint32_t {
      uint32_t word[4];
      #pragma unroll
      for (uint32_t r = 0; r < 4; ++r) {
        const uint32_t o = 32 - 2 * r - 2 * DL;
        word[r] = lds_word((w >> (o + 3)) & (((1u << (2 * DL - 5)) - 1u) << 2));
      }
      uint32_t m4 = 0;
      #pragma unroll
      for (uint32_t r = 0; r < 4; ++r)
        m4 |= __builtin_amdgcn_ubfe(word[r], w >> (32 - 2 * r - 2 * DL), 1u) << r;
      return m4;
    };
    const bool clean =
        !GLOBAL && __builtin_amdgcn_readfirstlane((uint32_t)(__ballot(dirty) != 0)) == 0;
    // windows of a clean tile of a large pattern set have passed the second
    // filter here already
    const bool hash_cls = clean && hashed && p.hash_cls;
    const bool hash_q = hashed && !hash_cls;     // queue entries still to test
    if (clean) {
      // every group's 16 bases (from q0, first base in the top bits) first,
      // then the bitmap words of two groups at a time
      uint32_t wv[NG];
      #pragma unroll
      for (uint32_t g = 0; g < NG; ++g) {
        const uint32_t wi = (g * 256 + 4 * lane) >> 4;
        wv[g] = __builtin_amdgcn_perm(pk[wi], pk[wi + 1], bsel);
      }
      constexpr uint32_t GS = NG >= 2 ? 2u : 1u;   // groups per batch of reads
      if (pairm) {
        #pragma unroll
        for (uint32_t g = 0; g < NG; ++g) want |= pair4(wv[g]) << (4 * g);
      } else {
      #pragma unroll
      for (uint32_t g = 0; g < NG; g += GS) {
        uint32_t word[4 * GS];
        #pragma unroll
        for (uint32_t k = 0; k < 4 * GS; ++k) {
          const uint32_t o = 32 - 2 * (k & 3) - 2 * DL;
          word[k] = lds_word((wv[g + (k >> 2)] >> (o + 3)) & (((1u << (2 * DL - 5)) - 1u) << 2));
        }
        #pragma unroll
        for (uint32_t k = 0; k < 4 * GS; ++k)
          want |= __builtin_amdgcn_ubfe(word[k], wv[g + (k >> 2)] >> (32 - 2 * (k & 3) - 2 * DL),
                                        1u) << (4 * g + k);
      }
      }
      if (hash_cls) {
        // the one-hash second filter on every window: its K <= 12 bases from
        // position r of the group are bits [32-2K-2r, 32-2r) of the group's
        // 16 bases, right-aligned into at most 24 bits for one 24-bit multiply
        uint32_t hbits = 0;
        const uint32_t kw = 32u - p.hash_kshift;             // 2K
        #pragma unroll
        for (uint32_t g = 0; g < NG; ++g) {
          uint32_t hw[4];
          uint32_t hh[4];
          #pragma unroll
          for (uint32_t r = 0; r < 4; ++r) {
            const uint32_t key =
                __builtin_amdgcn_ubfe(wv[g], p.hash_kshift - 2 * r, kw) & 0xFFFFFFu;
            hh[r] = (key * kHash1Mul) >> p.hash_shift;
            hw[r] = hl[hh[r] >> 5];
          }
          #pragma unroll
          for (uint32_t r = 0; r < 4; ++r)
            hbits |= ((hw[r] >> (hh[r] & 31u)) & 1u) << (4 * g + r);
        }
        want &= hbits;
      }
    } else {
      // positions of the lane inside the text: all of them in a full tile
      uint32_t valid = 0xFFFFFFFFu >> (32 - 4 * NG);
      if (!full) {
        valid = 0;
        #pragma unroll
        for (uint32_t g = 0; g < NG; ++g) {
          const int32_t left = (int32_t)nt - (int32_t)(g * 256 + 4 * lane);
          valid |= ((1u << (uint32_t)min(max(left, 0), 4)) - 1u) << (4 * g);
        }
      }
      #pragma unroll
      for (uint32_t g = 0; g < NG; ++g) {
        const uint32_t q0 = g * 256 + 4 * lane;
        uint32_t m4 = 0xFu, s4 = 0xFu;
        if (!GLOBAL) {
          const uint32_t wi = q0 >> 4, ii = q0 >> 5;
          const uint32_t w = __builtin_amdgcn_perm(pk[wi], pk[wi + 1], bsel);
          const uint32_t inv = __builtin_amdgcn_alignbit(iv[ii + 1], iv[ii], sh4);
          m4 = pairm ? pair4(w) : lookup4(w);
          s4 = 0;
          if (inv & gmask) {
            // a window holds a non-base (or runs past the text): such
            // positions walk from the root -- or, when every pattern is
            // longer than D, report nothing (no pattern fits before the
            // non-base): keep_slow is 0 then, else all ones
            #pragma unroll
            for (uint32_t r = 0; r < 4; ++r)
              if ((inv >> r) & dmask) s4 |= 1u << r;
            m4 = (m4 & ~s4) | (s4 & keep_slow);
            s4 &= keep_slow;
          }
        }
        want |= m4 << (4 * g);
        slow |= s4 << (4 * g);
      }
      want &= valid;
      slow &= valid;
    }

    // ---- queue the surviving positions (lane order, then position order):
    //      one pass over the whole tile when the queue holds it, else one
    //      pass per group of positions
    unsigned long long occ = 0;
    uint32_t tile_hits = 0;
    uint32_t total;
    const uint32_t base = wave_excl_dpp(__builtin_popcount(want), &total);
    // passes over the tile: one when the queue holds every survivor, else
    // one per half of the groups when each half fits, else one per group
    uint32_t passes = 1, gpp = NG;               // groups per pass
    if (total > kQueue) {
      passes = NG;
      gpp = 1;
      if (NG >= 2) {
        const uint32_t lo = __builtin_popcount(want & ((1u << (2 * NG)) - 1u));
        const uint32_t both = wave_sum(lo | ((__builtin_popcount(want) - lo) << 16));
        if ((both & 0xFFFFu) <= kQueue && (both >> 16) <= kQueue) {
          passes = 2;
          gpp = NG / 2;
        }
      }
    }
    for (uint32_t pass = 0; pass < passes; ++pass) {
      const uint32_t sel = passes == 1 ? (0xFFFFFFFFu >> (32 - 4 * NG))
                                       : ((0xFFFFFFFFu >> (32 - 4 * gpp)) << (4 * gpp * pass));
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
      // ---- second filter (LDS) and prefix filter (global): queue entries
      //      that must walk on, listed in queue2.  Up to four entries per
      //      lane at once, so their prefix-bitmap reads are in flight together
      uint32_t nwalk = ptotal;
      if (hash_q || pfxon) {
        // second filter (LDS): one queue entry per lane at a time; the
        // entries that pass are listed in queue2
        uint32_t nh = ptotal;
        if (hash_q) {
          nh = 0;
          #pragma unroll 1
          for (uint32_t i0 = 0; i0 < ptotal; i0 += 64) {
            const uint32_t i = i0 + lane;
            bool go = false;
            if (i < ptotal) {
              res[i] = 0;
              go = hash_pass(queue[i], pk, iv, hl, p.hash_kmask, p.hash_imask, p.hash_shift,
                             p.hash_cls != 0, p.hash_kshift);
            }
            const uint64_t m = __ballot(go);
            if (go)
              queue2[nh + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
                  (uint16_t)i;
            nh += (uint32_t)__popcll(m);
          }
          wave_sync();
        }
        nwalk = nh;
        if (pfxon) {
          // prefix filter (global): the candidates (queue2, or every queue
          // entry without a second filter) read their prefix bit, up to four
          // per lane in flight; those whose bit is set are listed in queue2
          // again, in place (an iteration reads its entries before it writes
          // the list, which never runs ahead of the reads)
          nwalk = 0;
          #pragma unroll 1
          for (uint32_t i0 = 0; i0 < nh; i0 += 256) {
            bool go[4];
            uint32_t idx[4], pw[4], pb[4];
            #pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {
              const uint32_t j = i0 + 64 * r + lane;
              go[r] = false;
              idx[r] = j;
              pw[r] = 0;
              pb[r] = 0;
              if (j < nh) {
                if (hash_q) {
                  idx[r] = queue2[j];
                } else {
                  res[j] = 0;
                }
                uint32_t wd, bt;
                go[r] = pfx_locate(queue[idx[r]], pk, iv, p.pfx_shift, p.pfx_imask, &wd, &bt);
                if (go[r]) {
                  pw[r] = p.pfx[wd];
                  pb[r] = bt;
                }
              }
            }
            #pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {
              const bool g2 = go[r] && ((pw[r] >> pb[r]) & 1u);
              const uint64_t m = __ballot(g2);
              if (g2)
                queue2[nwalk + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
                    (uint16_t)idx[r];
              nwalk += (uint32_t)__popcll(m);
            }
          }
          wave_sync();
        }
      }
      const bool listed = hash_q || pfxon;
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
          const uint32_t i = listed ? (uint32_t)queue2[j] : j;
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
          // entry = {pos, slow | text << 1, codes[0..1]}, {codes[2..3], inv[0..1]}
          u32x4* dst = reinterpret_cast<u32x4*>(wq + wbase + j);
          dst[0] = u32x4{(uint32_t)(t0 + qt), ((e >> 15) & 1u) | (si << 1), c.x, c.y};
          dst[1] = u32x4{c.z, c.w, inv0, inv1};
          res[i] = 0;       // the deferred walk writes its result
        }
      }
      // ---- walk them with all lanes
      uint32_t nz = 0;
      #pragma unroll 1
      for (uint32_t j = ndef + lane; j < nwalk; j += 64) {
        const uint32_t i = listed ? (uint32_t)queue2[j] : j;
        const uint32_t e = queue[i];
        const uint32_t qt = e & 0x7FFFu;                 // index within the tile
        int32_t best = 0;
        if (GLOBAL) {
          // the global-memory variants: DT names the table layout
          if (DT == 1 || DT == 2)
            walk_cells<DT>(t0 + qt, p, text, n, enc, best, occ);
          else
            walk<true>(0u, t0 + qt, nullptr, nullptr, p.next, p.out, text, n, enc, best, occ);
        } else {
          best = deep_walk(e, D, p.lds_trie, p.levels, lds, bmpre, lvl, pk, iv, p.node, p.out,
                           p.jump, p.jres, occ);
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
          if (PZ && full && maligned) break;   // zeroed when its text was fetched
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
      deferred_walks<D, SINGLE, TILE>(p, wq, wq_n);
    }
  }
}

}  // namespace pfac

// Kernel selection, one function per instantiation unit (workgroup size x
// launch kind): the scan kernel for a variant, filter depth, walk placement,
// tile size and pre-zeroing, or nullptr when that combination is not built.
namespace pfac {
using ScanFn = void (*)(ScanParams);
#define PFAC_DECLARE_PICK(B)                                                          \
  ScanFn pick_scan_single_##B(bool global, uint32_t D, bool defer, uint32_t tile, bool pz); \
  ScanFn pick_scan_batch_##B(bool global, uint32_t D, bool defer, uint32_t tile, bool pz);
PFAC_DECLARE_PICK(256)
PFAC_DECLARE_PICK(512)
PFAC_DECLARE_PICK(768)
PFAC_DECLARE_PICK(1024)
#undef PFAC_DECLARE_PICK
}  // namespace pfac
