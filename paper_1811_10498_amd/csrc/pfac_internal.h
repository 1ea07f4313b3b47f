// Internal declarations shared by the host trie builder and the HIP kernels.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "pfac.h"

namespace pfac {

// Root jump tables (and their LDS filter bitmaps) exist for these depths.
constexpr uint32_t kMinJump = 6;
constexpr uint32_t kMaxJump = 10;
constexpr uint32_t kImageLevels = 8;      // trie levels an LDS image may hold
constexpr uint32_t kImageMaxBytes = 160 * 1024;
// Pair tables (filter depths kMinJump..kPairMaxDepth): one byte per
// (D-1)-base string m; bits 0..3: the window a.m passes the depth-D filter
// (a = the base before m), bits 4..7: the window m.b passes (b = the base
// after m).  Two neighbouring positions share m, so one byte read tests both.
constexpr uint32_t kPairMaxDepth = 9;

// Second filter: the first K = min(shortest pattern, kHashK) bases of a
// window, left-aligned in 32 bits (first base most significant), hashed
// multiplicatively to `bits` bits (kHashMinBits..kHashMaxBits) with two
// multipliers; a window passes when both of its bits are set (a Bloom filter
// with two hash functions).
constexpr uint32_t kHashK = 16;
constexpr uint32_t kHashMinBits = 12;
constexpr uint32_t kHashMaxBits = 20;
constexpr uint32_t kHashMul = 0x9E3779B1u;
constexpr uint32_t kHashMul2 = 0x85EBCA77u;

// One-hash form of the second filter, for K <= 12: the K-base key
// right-aligned in 2K bits (at most 24) times a 24-bit multiplier, whose
// product's low 32 bits the GPU forms in one full-rate 24-bit multiply; its
// top `bits` bits are the window's one bit.  Used for pattern sets that most
// windows pass at depth D, where the exact prefix filter follows it and the
// second hash would only halve the few prefix-bitmap reads.  (0xC6A4A7 maps
// every 24-bit key range evenly: each 2^19-bit slot gets 30..33 keys.)
constexpr uint32_t kHash1Mul = 0xC6A4A7u;
constexpr uint32_t kHash1MaxK = 12;

// Prefix filter: an exact bitmap of the first K2 = min(shortest pattern,
// kPfxMaxK) bases of every pattern (4^K2 bits, 2 MB at K2 = 12), kept in
// global memory (L2-resident) for pattern sets too large for the hashed one.
constexpr uint32_t kPfxMinK = 7;
constexpr uint32_t kPfxMaxK = 12;

// Longest run of single-child trie steps a walk takes at once.
constexpr uint32_t kChainMax = 14;

// Edge word of the next-state table: child state in bits 0..30 (0 = no edge,
// the root is never a child), bit 31 set when the child is a final state.
constexpr uint32_t kFinalBit = 0x80000000u;
constexpr uint32_t kStateMask = 0x7FFFFFFFu;

// Per final state: smallest pattern ID ending there and how many pattern
// IDs end there.
struct OutEntry {
  int32_t pid;
  uint32_t mult;
};

// Window keys put the first base in the most significant bits, so keys of
// one trie level sort exactly like the breadth-first numbering of that level.
// Root jump entry for a D-base window x:
// bits 0..30 = state reached after all D bases (0 if the walk stopped
// earlier), bit 31 = at least one final state was passed within the D
// steps; then jres[x] holds {longest such pattern ID, occurrences}.
// The filter bitmap has bit x set iff jump[x] != 0, i.e. iff a walk from a
// position whose next D bases are x either continues past depth D or has
// passed a final state; every other such walk reports nothing.
struct HostTable {
  uint64_t num_states = 0;
  uint32_t num_patterns = 0;
  uint32_t max_len = 0;
  uint32_t min_len = 0;
  uint32_t max_depth_full = 0;
  std::vector<uint32_t> next;             // [S*4], columns A,C,G,T
  std::vector<OutEntry> out;              // [S]
  std::vector<uint64_t> depth_start;      // first BFS index of each depth, plus S at the end
  std::vector<uint32_t> jump[kMaxJump + 1];
  std::vector<OutEntry> jres[kMaxJump + 1];
  std::vector<uint32_t> bitmap[kMaxJump + 1];   // 4^D bits
  std::vector<uint8_t> node;              // [S]: bits 0..3 child exists (A,C,G,T), bit 4 final
  // Path compression of the walk: chain[2s] = the bases of the run of
  // single-child steps below s (first base in the top bits, up to kChainMax
  // of them) with the run length in bits 0..3, chain[2s+1] = the state the run
  // ends at, bit 31 set when it is final.  Every state strictly inside the
  // run has exactly one child and is not final, so a walk either matches the
  // whole run or ends inside it with nothing to report.  Length < 2: no run.
  std::vector<uint32_t> chain;            // [2S]
  // LDS image per filter depth D: what the scan kernel copies into LDS.
  //   words [0, 4^D/32)           filter bitmap
  //   then 4^D/128 words          set bits before each 128-bit group (rank)
  //   then for d = D .. D+levels-1: node bytes of level d (padded to 16 nodes),
  //        then one word per 16 nodes: child bits of the level before the group
  struct Image {
    std::vector<uint32_t> words;
    uint32_t levels = 0;                  // trie levels stored (D .. D+levels-1)
    uint32_t byte_off[kImageLevels];      // word offset of level D+k's node bytes
    uint32_t pre_off[kImageLevels];       // word offset of its rank words
    uint32_t upto[kImageLevels];          // image words needed to hold levels D..D+k
  };
  Image image[kMaxJump + 1];
  uint32_t hash_k = 0;                      // K of the second filter
  std::vector<uint32_t> hash[kHashMaxBits + 1];   // 2^bits-bit bitmaps
  uint32_t hash_set[kHashMaxBits + 1] = {};       // set bits of each
  std::vector<uint32_t> hash1[kHashMaxBits + 1];  // one-hash bitmaps (hash_k <= 12)
  uint32_t hash1_set[kHashMaxBits + 1] = {};
  uint32_t pfx_k = 0;                       // K2 of the prefix filter (0 = none)
  std::vector<uint32_t> pfx;                // 4^K2-bit bitmap
  uint64_t pfx_set = 0;                     // distinct K2-base pattern prefixes
  uint64_t bitmap_set[kMaxJump + 1] = {};   // set bits of each depth-D filter bitmap
  // every pattern ID of a final state but its smallest (the output entry
  // holds that one), as (state, id) pairs sorted by state, then id
  std::vector<uint32_t> dup_state;
  std::vector<int32_t> dup_id;
};

// Host build: validate, insert in input order, renumber breadth-first, pack.
int build_host_table(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                     HostTable* out, int64_t* bad_index);

// Byte-alphabet trie (every byte value a symbol): states renumbered
// breadth-first, the edges of every state but the root in one open-addressing
// hash table keyed by (state, byte), the root's 256 edges in a dense row.
// Edge value: child in bits 0..30, bit 31 set when the child is final.
constexpr uint32_t kBytesMaxStates = (1u << 24) - 1;
constexpr uint32_t kBytesEmptyKey = 0xFFFFFFFFu;
struct HostBytes {
  uint64_t num_states = 0;
  uint32_t num_patterns = 0, max_len = 0, min_len = 0;
  uint32_t root[256] = {};
  uint32_t hash_bits = 0;
  std::vector<uint32_t> slots;             // [2 << hash_bits]: key (state << 8 | byte), value
  std::vector<OutEntry> out;               // [S]
  std::vector<uint64_t> depth_start;
  uint64_t edges = 0;
};
int build_host_bytes(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                     HostBytes* out, int64_t* bad_index);

// Slot of (state, byte) in the byte trie's hash table: Fibonacci hashing of
// the key, linear probing.
inline uint32_t bytes_hash(uint32_t key, uint32_t bits) {
  return (uint32_t)(key * 0x9E3779B1u) >> (32 - bits);
}

// Device arrays of one table.
struct DevTable {
  const uint32_t* next;
  const OutEntry* out;
  const uint32_t* jump[kMaxJump + 1];
  const OutEntry* jres[kMaxJump + 1];
  const uint32_t* image[kMaxJump + 1];   // LDS image words (HostTable::Image)
  const uint8_t* pair[kMaxJump + 1];     // pair tables (D <= kPairMaxDepth)
  const uint32_t* levels[kMaxJump + 1];  // per image level: {byte_off, pre_off, first state, 0}
  const uint32_t* hash[kHashMaxBits + 1]; // second-filter bitmaps
  const uint32_t* hash1[kHashMaxBits + 1]; // one-hash second-filter bitmaps (or null)
  const uint32_t* chain;                  // [2S] runs of single-child steps
  const uint32_t* node;                   // [8S] per state: next[4], chain[2], out (pid, mult)
  const uint32_t* pfx;                    // prefix-filter bitmap (or null)
  const uint32_t* dup_state;              // further IDs of final states (HostTable)
  const int32_t* dup_id;
  uint32_t num_dups;
  uint32_t num_states;
  uint32_t max_len;
};

// Offsets of a table's arrays in its one device allocation (table_layout).
struct TableLayout {
  uint64_t o_next = 0, o_out = 0, o_chain = 0, o_node = 0;
  uint64_t o_jump[kMaxJump + 1] = {}, o_jres[kMaxJump + 1] = {}, o_im[kMaxJump + 1] = {};
  uint64_t o_lv[kMaxJump + 1] = {};
  uint64_t o_pair[kMaxJump + 1] = {};
  uint32_t image_words[kMaxJump + 1] = {};
  std::vector<uint32_t> lvdesc[kMaxJump + 1];
  uint64_t o_hash[kHashMaxBits + 1] = {};
  uint32_t hash_words[kHashMaxBits + 1] = {};
  uint64_t o_hash1[kHashMaxBits + 1] = {};
  uint32_t hash1_words[kHashMaxBits + 1] = {};
  uint64_t o_pfx = 0, pfx_words = 0;
  uint64_t o_dups = 0, o_dupi = 0, ndups = 0;
  uint64_t bytes = 0;
};

}  // namespace pfac

struct pfac_table {
  int device = 0;
  uint32_t alphabet = 4;            // 4: DNA table; 256: byte table (`bytes`, `bdev`)
  pfac::HostTable host;             // kept for info queries
  pfac::HostBytes bytes;
  struct {
    const uint32_t* root;           // [256]
    const uint32_t* slots;          // [2 << hash_bits]
    const pfac::OutEntry* out;      // [S]
    uint32_t hash_bits;
  } bdev{};
  void* dmem = nullptr;             // one device allocation for every array
  uint64_t dbytes = 0;
  pfac::DevTable dev{};             // device pointers into dmem
  pfac::TableLayout layout;
  std::vector<std::string> pats;    // the pattern set and its IDs (updates start from it)
  std::vector<int32_t> ids;
  // the paper's two-array and merged-cell layouts, built on first use
  mutable void* cells_mem = nullptr;
  mutable const uint32_t* next2 = nullptr;
  mutable const int32_t* cell_pid = nullptr;
  mutable const void* cells = nullptr;
};
