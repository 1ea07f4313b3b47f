// Every occurrence: the list of all (start position, pattern ID) pairs of a
// text, the sub-patterns PFAC itself does not report included (the paper
// names that limitation, Sec. IV).  Three steps after the ordinary scan:
//   count  -- the scan already sums the occurrences of every tile (each walk
//             adds the number of IDs of every final state it passes);
//   scan   -- exclusive prefix of those counts over the tiles;
//   write  -- one wave per tile walks again from the root, at the tile's
//             matching positions only (the hit slots the scan parked, or
//             every position of a tile with more hits than slots), and
//             writes each final state's IDs at the tile's offset plus the
//             position's own prefix.
// Order of the list: ascending position, then ascending pattern length (the
// order a walk passes its final states), then ascending ID among equal
// patterns.
#include <string.h>

#include <algorithm>

#include "pfac_host.h"

namespace pfac {

constexpr uint32_t kOccBlock = 1024;
constexpr uint32_t kOccPerBlock = 4 * kOccBlock;   // tiles per workgroup of the scan steps

// Sum of the occurrence counts of 4096 tiles per workgroup.
__global__ __launch_bounds__(kOccBlock) void occ_block_sum_kernel(
    const unsigned long long* tile_occ, uint64_t tiles, unsigned long long* block_sum) {
  __shared__ unsigned long long ws[kOccBlock / 64];
  const uint64_t t0 = (uint64_t)blockIdx.x * kOccPerBlock + 4 * threadIdx.x;
  unsigned long long v = 0;
  for (uint32_t k = 0; k < 4; ++k)
    if (t0 + k < tiles) v += tile_occ[t0 + k];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (uint32_t w = 0; w < kOccBlock / 64; ++w) s += ws[w];
    block_sum[blockIdx.x] = s;
  }
}

// Exclusive prefix (in place) of nb block sums, one workgroup: each thread
// takes a contiguous run, the runs' totals are scanned across the threads.
__global__ __launch_bounds__(kOccBlock) void occ_block_scan_kernel(unsigned long long* v,
                                                                   uint32_t nb) {
  __shared__ unsigned long long part[kOccBlock];
  const uint32_t per = (nb + kOccBlock - 1) / kOccBlock;
  const uint32_t lo = threadIdx.x * per, hi = min(nb, lo + per);
  unsigned long long s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += v[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (uint32_t i = 0; i < kOccBlock; ++i) {
      const unsigned long long x = part[i];
      part[i] = run;
      run += x;
    }
  }
  __syncthreads();
  unsigned long long run = part[threadIdx.x];
  for (uint32_t i = lo; i < hi; ++i) {
    const unsigned long long x = v[i];
    v[i] = run;
    run += x;
  }
}

// Exclusive prefix of the tiles' counts: within the workgroup's 4096 tiles,
// plus the prefix of the workgroups before.
__global__ __launch_bounds__(kOccBlock) void occ_tile_offset_kernel(
    const unsigned long long* tile_occ, uint64_t tiles, const unsigned long long* block_off,
    unsigned long long* tile_off) {
  __shared__ unsigned long long ws[kOccBlock / 64];
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t t0 = (uint64_t)blockIdx.x * kOccPerBlock + 4 * threadIdx.x;
  unsigned long long c[4], sum = 0;
  for (uint32_t k = 0; k < 4; ++k) {
    c[k] = t0 + k < tiles ? tile_occ[t0 + k] : 0ull;
    sum += c[k];
  }
  // inclusive prefix of `sum` over the wave
  unsigned long long inc = sum;
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  unsigned long long before = block_off[blockIdx.x];
  for (uint32_t k = 0; k < w; ++k) before += ws[k];
  unsigned long long off = before + inc - sum;
  for (uint32_t k = 0; k < 4; ++k) {
    if (t0 + k < tiles) tile_off[t0 + k] = off;
    off += c[k];
  }
}

struct OccParams {
  const uint8_t* text;
  uint64_t n;
  uint32_t enc;
  uint32_t tile;
  uint64_t tiles;
  DevTable tab;
  const uint32_t* tile_hits;
  const Slot* slots;
  const unsigned long long* tile_off;
  pfac_hit* occ;
  uint64_t cap;
};

// The walk from the root at `pos` on the text in global memory.  Returns
// the number of pattern IDs of the final states it passes; with `emit`,
// writes them from list index `o` on (the first `cap` of the list only).
__device__ uint32_t occ_walk(const OccParams& p, uint64_t pos, bool emit, uint64_t o) {
  uint32_t s = 0, cnt = 0;
  for (uint64_t q = pos;; ++q) {
    const int b = global_base(p.text, p.n, p.enc, q);
    if (b < 0) break;
    const uint32_t e = p.tab.next[(uint64_t)s * 4 + (uint32_t)b];
    if (e == 0) break;
    s = e & kStateMask;
    if (!(e & kFinalBit)) continue;
    const OutEntry oe = p.tab.out[s];
    if (emit) {
      if (o < p.cap) p.occ[o] = pfac_hit{(uint32_t)pos, oe.pid};
      ++o;
      if (oe.mult > 1) {
        // the further IDs of this state: sorted by (state, id)
        uint32_t lo = 0, hi = p.tab.num_dups;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (p.tab.dup_state[mid] < s) lo = mid + 1; else hi = mid;
        }
        for (uint32_t k = 0; k + 1 < oe.mult; ++k, ++o)
          if (o < p.cap) p.occ[o] = pfac_hit{(uint32_t)pos, p.tab.dup_id[lo + k]};
      }
    }
    cnt += oe.mult;
  }
  return cnt;
}

// One wave per tile (grid-stride): the tile's matching positions in
// position order, each one's count, the wave's prefix, then the writes.
__global__ __launch_bounds__(256) void occ_write_kernel(OccParams p) {
  __shared__ uint32_t sorted[4][kSlot];
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t nwaves = (uint64_t)gridDim.x * 4;
  for (uint64_t t = (uint64_t)blockIdx.x * 4 + w; t < p.tiles; t += nwaves) {
    const uint32_t h = p.tile_hits[t];
    if (h == 0) continue;
    unsigned long long base = p.tile_off[t];
    const uint64_t t0 = t * p.tile;
    if (h <= kSlot) {
      // the parked hits, ordered by position (ranks: positions are distinct)
      const Slot* sl = p.slots + t * kSlot;
      if (lane < h) {
        const uint32_t mine = sl[lane].pos;
        uint32_t rank = 0;
        for (uint32_t j = 0; j < h; ++j) rank += sl[j].pos < mine;
        sorted[w][rank] = mine;
      }
      wave_sync();
      const uint32_t pos = lane < h ? sorted[w][lane] : 0u;
      const uint32_t cnt = lane < h ? occ_walk(p, pos, false, 0) : 0u;
      uint32_t tot;
      const uint32_t ex = wave_excl(cnt, &tot);
      if (lane < h && cnt) occ_walk(p, pos, true, base + ex);
      wave_sync();
    } else {
      // more hits than slots: every position of the tile
      for (uint32_t k0 = 0; k0 < p.tile; k0 += 64) {
        const uint64_t pos = t0 + k0 + lane;
        const uint32_t cnt = pos < p.n ? occ_walk(p, pos, false, 0) : 0u;
        uint32_t tot;
        const uint32_t ex = wave_excl(cnt, &tot);
        if (cnt) occ_walk(p, pos, true, base + ex);
        base += tot;
      }
    }
  }
}

}  // namespace pfac

using namespace pfac;

extern "C" {

int pfac_match_all(const pfac_table* t, const void* d_text, uint64_t n, int enc,
                   pfac_hit* d_occ, uint64_t occ_cap, uint64_t* d_counters,
                   const pfac_plan* plan, void* stream_) {
  if (!t || !d_counters || (n && !d_text) || n >= (1ull << 32)) return PFAC_E_ARG;
  if (enc != PFAC_TEXT_ASCII && enc != PFAC_TEXT_2BIT) return PFAC_E_ARG;
  if (!d_occ) occ_cap = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFAC_E_NODEV;
  if (dev != t->device) return PFAC_E_ARG;
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  SinglePrep P;
  int rc = prepare_single(t, n, enc, plan, dev, &P);
  if (rc) return rc;
  unsigned long long* counters = reinterpret_cast<unsigned long long*>(d_counters);
  if (P.tiles == 0) return launch_zero(counters, 2u, stream);
  const uint64_t nb = (P.tiles + kOccPerBlock - 1) / kOccPerBlock;
  const uint64_t extra = al256(nb * 8) + al256(P.tiles * 8);
  Workspace* ws = workspace_for(dev, stream, P.tiles, P.walks, extra, &rc);
  if (!ws) return rc;
  const Scratch& sc = workspace_scratch(ws);
  // count: the scan (per-tile occurrence counts, hit slots kept) and the
  // finish kernel (totals; no hit list)
  rc = enqueue_single(t, P, sc, d_text, nullptr, nullptr, 0, counters, dev, stream, true);
  if (rc) return rc;
  if (occ_cap == 0) return PFAC_OK;
  // scan
  unsigned long long* block = reinterpret_cast<unsigned long long*>(workspace_extra(ws));
  unsigned long long* tile_off =
      reinterpret_cast<unsigned long long*>(workspace_extra(ws) + al256(nb * 8));
  hipLaunchKernelGGL(occ_block_sum_kernel, dim3((uint32_t)nb), dim3(kOccBlock), 0, stream,
                     sc.tile_occ, P.tiles, block);
  hipLaunchKernelGGL(occ_block_scan_kernel, dim3(1), dim3(kOccBlock), 0, stream, block,
                     (uint32_t)nb);
  hipLaunchKernelGGL(occ_tile_offset_kernel, dim3((uint32_t)nb), dim3(kOccBlock), 0, stream,
                     sc.tile_occ, P.tiles, block, tile_off);
  // write
  OccParams op;
  memset(&op, 0, sizeof(op));
  op.text = static_cast<const uint8_t*>(d_text);
  op.n = n;
  op.enc = (uint32_t)enc;
  op.tile = P.pl.tile;
  op.tiles = P.tiles;
  op.tab = t->dev;
  op.tile_hits = sc.tile_hits;
  op.slots = sc.slots;
  op.tile_off = tile_off;
  op.occ = d_occ;
  op.cap = occ_cap;
  const uint64_t grid = std::min<uint64_t>((P.tiles + 3) / 4, 4096);
  hipLaunchKernelGGL(occ_write_kernel, dim3((uint32_t)grid), dim3(256), 0, stream, op);
  return hipGetLastError() == hipSuccess ? PFAC_OK : PFAC_E_HIP;
}

}  // extern "C"
