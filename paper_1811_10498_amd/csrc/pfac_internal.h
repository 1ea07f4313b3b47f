// Internal declarations shared by the host trie builder and the HIP kernels.
#pragma once

#include <stdint.h>

#include <vector>

#include "pfac.h"

namespace pfac {

// Root jump tables (and their LDS filter bitmaps) exist for these depths.
constexpr uint32_t kMinJump = 6;
constexpr uint32_t kMaxJump = 10;

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

// Root jump entry for a D-base window x (first base in the low bits):
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
};

// Host build: validate, insert in input order, renumber breadth-first, pack.
int build_host_table(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                     HostTable* out, int64_t* bad_index);

// Device arrays of one table.
struct DevTable {
  const uint32_t* next;
  const OutEntry* out;
  const uint32_t* jump[kMaxJump + 1];
  const OutEntry* jres[kMaxJump + 1];
  const uint32_t* bitmap[kMaxJump + 1];
  uint32_t num_states;
  uint32_t max_len;
};

}  // namespace pfac

struct pfac_table {
  int device = 0;
  pfac::HostTable host;             // kept for info queries
  void* dmem = nullptr;             // one device allocation for every array
  uint64_t dbytes = 0;
  pfac::DevTable dev{};             // device pointers into dmem
};
