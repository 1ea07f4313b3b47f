// Host-side pieces of libpfac.so shared between its translation units: the
// scratch layout of a one-text call and the two halves of pfac_match
// (prepare: plan, parameters and scratch size; enqueue: the kernels).
#pragma once

#include <mutex>

#include "scan_device.h"

namespace pfac {

std::mutex& host_mutex();

uint64_t al256(uint64_t x);

// Scratch of the scan and finish kernels, carved out of one device block:
// per-tile hit counts, occurrence counts and hit slots; the finish kernel's
// look-back word and occurrence sum per workgroup and its two counters
// (zero between launches); batch work items; deferred walks; the area a
// pre-zeroing scan writes in place of a tile that is not full.
struct Scratch {
  uint32_t* tile_hits = nullptr;
  unsigned long long* tile_occ = nullptr;
  Slot* slots = nullptr;
  unsigned long long* status = nullptr;
  unsigned long long* block_occ = nullptr;
  uint32_t* sync = nullptr;
  TileItem* items = nullptr;
  WalkEntry* walk = nullptr;
  int32_t* dummy = nullptr;
  uint64_t tiles = 0, walk_cap = 0;
};

// Byte offsets of the parts of a scratch block for `tiles` tiles (and as
// many batch work items when `items`) and `walks` deferred walks; bytes =
// the total, [o_st, o_st + zero_bytes) = the part that must start at zero.
struct ScratchLayout {
  uint64_t o_hits, o_occ, o_slots, o_st, o_bo, o_sync, o_items, o_walk, o_dummy, bytes,
      zero_bytes;
};
ScratchLayout scratch_layout(uint64_t tiles, bool items, uint64_t walks);
Scratch carve(uint8_t* mem, const ScratchLayout& L, uint64_t tiles, uint64_t walks);

// Everything of a one-text call that does not depend on the buffers: the
// plan, the scan parameters (without buffers), the tiles and the
// deferred-walk entries the launch needs.
struct SinglePrep {
  pfac_plan pl;
  ScanParams sp;
  uint64_t tiles;
  uint64_t walks;
};

int prepare_single(const pfac_table* t, uint64_t n, int enc, const pfac_plan* plan, int dev,
                   SinglePrep* P);

// Enqueue a prepared one-text call on the scratch `sc` (kernel launches
// only).  `keep_slots`: the scan parks each tile's hits in its slots even
// when no hit list is asked for (the all-occurrence pass reads them).
int enqueue_single(const pfac_table* t, SinglePrep& P, const Scratch& sc, const void* d_text,
                   int32_t* d_match, pfac_hit* d_hits, uint64_t hit_cap,
                   unsigned long long* counters, int dev, hipStream_t stream,
                   bool keep_slots = false);

// Workspace of (device, stream) holding scratch for `tiles` tiles and
// `walks` deferred walks, plus `extra` bytes after it; nullptr on failure
// (*rc says why).
struct Workspace;
Workspace* workspace_for(int dev, hipStream_t stream, uint64_t tiles, uint64_t walks,
                         uint64_t extra, int* rc);
const Scratch& workspace_scratch(const Workspace* ws);
uint8_t* workspace_extra(const Workspace* ws);

// Zero n 64-bit words at p with a fill kernel on `stream`.
int launch_zero(unsigned long long* p, uint32_t n, hipStream_t stream);

// The finish kernel of a one-text call of `tiles` tiles of `tile` positions
// over a text of n positions whose dense output `match` was written (tiles
// with more hits than slots take them from it).
int launch_finish_single(const Scratch& sc, uint64_t tiles, uint32_t tile, uint64_t n,
                         unsigned long long* counters, pfac_hit* d_hits, uint64_t hit_cap,
                         const int32_t* match, hipStream_t stream);

// A gfx950 device, and its compute units.
bool device_ok(int dev);
uint32_t device_cus(int dev);

// Device memory of a table: layout from its metadata, zeroed allocation,
// pointers; the host-built arrays uploaded; the pattern set kept.
void table_layout(const HostTable& h, uint64_t ndups, TableLayout* L);
int alloc_table(pfac_table* t, uint64_t ndups);
int upload_host_table(pfac_table* t);
int build_derived(pfac_table* t);      // node records, pair tables
int remember_patterns(pfac_table* t, const char* const* patterns, const uint32_t* lengths,
                      uint32_t num, const int32_t* ids);

// pfac_match on a byte-alphabet table (bytes.hip).
int match_bytes(const pfac_table* t, const void* d_text, uint64_t n, int32_t* d_match,
                pfac_hit* d_hits, uint64_t hit_cap, unsigned long long* counters,
                const pfac_plan* plan, int dev, hipStream_t stream);

}  // namespace pfac
