// Building the table on the device, and updating a table (patterns added,
// patterns removed) by building the new one there.
//
// The table is the one pfac_build_table makes on the host (insertion order
// of Sec. V.A, then breadth-first numbering with children in A,C,G,T order),
// reached without inserting patterns one at a time: with the patterns sorted
// as base strings (a prefix before its extensions), the states of depth d are
// exactly the distinct d-base prefixes of the patterns at least d long, and
// breadth-first order within a level is their sorted order.  A pattern whose
// longest common prefix with the pattern before it is l creates the states
// of depths l+1 .. its length; per depth, an inclusive scan of "creates a
// state at this depth" over the sorted patterns numbers them.  Every other
// array (edges, outputs, runs of single-child states, jump tables, LDS
// images, filter bitmaps, duplicate IDs) follows from the states with one
// thread per state, key or pattern.  The arrays equal the host build's byte
// for byte (a GPU test compares them).  Patterns of at most 64 bases.
#include <string.h>

#include <algorithm>
#include <vector>

#include <rocprim/rocprim.hpp>

#include "pfac_host.h"

namespace pfac {

constexpr uint32_t kDbMaxLen = 64;        // bases a pattern may have (two 64-bit key words)
constexpr uint32_t kDbBlock = 256;

static uint32_t db_grid(uint64_t n) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + kDbBlock - 1) / kDbBlock, 65535));
}

#define DB_FOR(i, n) \
  for (uint64_t i = (uint64_t)blockIdx.x * kDbBlock + threadIdx.x; i < (n); \
       i += (uint64_t)gridDim.x * kDbBlock)

// Base k of a packed pattern: first base in the top two bits of w0.
__device__ __forceinline__ uint32_t db_base(uint64_t w0, uint64_t w1, uint32_t k) {
  return k < 32 ? (uint32_t)(w0 >> (62 - 2 * k)) & 3u : (uint32_t)(w1 >> (62 - 2 * (k - 32))) & 3u;
}

__global__ void db_iota(uint32_t* v, uint64_t n) {
  DB_FOR(i, n) v[i] = (uint32_t)i;
}

template <typename T>
__global__ void db_gather(const T* src, const uint32_t* perm, T* dst, uint64_t n) {
  DB_FOR(i, n) dst[i] = src[perm[i]];
}

// Longest common prefix of sorted pattern i with pattern i-1 (0 for the first).
__global__ void db_lcp(const uint64_t* w0, const uint64_t* w1, const uint32_t* len, uint64_t n,
                       uint32_t* lcp) {
  DB_FOR(i, n) {
    uint32_t c = 0;
    if (i > 0) {
      const uint64_t a = w0[i] ^ w0[i - 1];
      if (a) {
        c = (uint32_t)__builtin_clzll(a) / 2;
      } else {
        const uint64_t b = w1[i] ^ w1[i - 1];
        c = b ? 32 + (uint32_t)__builtin_clzll(b) / 2 : 64;
      }
      c = min(c, min(len[i], len[i - 1]));
    }
    lcp[i] = c;
  }
}

__global__ void db_flags(const uint32_t* lcp, const uint32_t* len, uint64_t n, uint32_t d,
                         uint32_t* flag) {
  DB_FOR(i, n) flag[i] = (lcp[i] < d && d <= len[i]) ? 1u : 0u;
}

// ds[d] = first state of depth d (ds[1] = 1).  Pattern i's state at depth d.
__global__ void db_states(const uint32_t* cnt, const uint32_t* len, uint64_t n, uint32_t d,
                          const uint64_t* ds, uint32_t* st) {
  DB_FOR(i, n) if (d <= len[i]) st[i * kDbMaxLen + d - 1] = (uint32_t)(ds[d] + cnt[i] - 1);
}

__global__ void db_level_end(const uint32_t* cnt, uint64_t n, uint32_t d, uint64_t* ds) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ds[d + 1] = ds[d] + cnt[n - 1];
}

// Final states: smallest ID and count of IDs per state (pid starts at INT_MAX).
__global__ void db_finals(const uint32_t* st, const uint32_t* len, const int32_t* id, uint64_t n,
                          OutEntry* out, uint8_t* fin) {
  DB_FOR(i, n) {
    const uint32_t s = st[i * kDbMaxLen + len[i] - 1];
    atomicMin(&out[s].pid, id[i]);
    atomicAdd(&out[s].mult, 1u);
    fin[s] = 1;
  }
}

__global__ void db_out_init(OutEntry* out, uint64_t S) {
  DB_FOR(s, S) out[s] = OutEntry{0x7FFFFFFF, 0u};
}

__global__ void db_out_fix(OutEntry* out, uint64_t S) {
  DB_FOR(s, S) if (out[s].mult == 0) out[s].pid = 0;
}

// Edges created by pattern i: depths lcp .. len-1 (shallower ones belong to
// the patterns before it; a repeated edge would be written with the same word).
__global__ void db_edges(const uint32_t* st, const uint32_t* len, const uint32_t* lcp,
                         const uint64_t* w0, const uint64_t* w1, const uint8_t* fin, uint64_t n,
                         uint32_t* next) {
  DB_FOR(i, n) {
    for (uint32_t d = lcp[i]; d < len[i]; ++d) {
      const uint32_t parent = d ? st[i * kDbMaxLen + d - 1] : 0u;
      const uint32_t child = st[i * kDbMaxLen + d];
      const uint32_t c = db_base(w0[i], w1[i], d);
      next[(uint64_t)parent * 4 + c] = child | (fin[child] ? kFinalBit : 0u);
    }
  }
}

// Node byte of every state: child bits A,C,G,T and the final bit.
__global__ void db_nodes(const uint32_t* next, const OutEntry* out, uint64_t S, uint8_t* node) {
  DB_FOR(s, S) {
    uint8_t v = out[s].pid ? 0x10 : 0;
    for (int a = 0; a < 4; ++a)
      if (next[s * 4 + a]) v |= (uint8_t)(1u << a);
    node[s] = v;
  }
}

// Runs of single-child steps below every state (the host build's rule).
__global__ void db_chains(const uint32_t* next, const uint8_t* node, uint64_t S, uint32_t* chain) {
  DB_FOR(i, S) {
    uint32_t len = 0, codes = 0;
    uint64_t cur = i;
    bool fin = false;
    while (len < kChainMax) {
      const uint32_t kids = node[cur] & 0x0Fu;
      if (__builtin_popcount(kids) != 1) break;
      const uint32_t a = (uint32_t)__builtin_ctz(kids);
      const uint32_t e = next[cur * 4 + a];
      codes |= a << (30 - 2 * len);
      ++len;
      cur = e & kStateMask;
      fin = (e & kFinalBit) != 0;
      if (fin) break;
    }
    if (len >= 2) {
      chain[2 * i] = codes | len;
      chain[2 * i + 1] = (uint32_t)cur | (fin ? kFinalBit : 0u);
    }
  }
}

// Jump table of depth D: the first D steps of the walk for every D-base key.
__global__ void db_jump(const uint32_t* next, const OutEntry* out, uint32_t D, uint32_t* jump,
                        OutEntry* jres) {
  DB_FOR(x, 1ull << (2 * D)) {
    uint32_t s = 0, cnt = 0;
    int32_t best = 0;
    bool whole = true;
    for (uint32_t k = 0; k < D; ++k) {
      const uint32_t c = (uint32_t)(x >> (2 * (D - 1 - k))) & 3u;
      const uint32_t e = next[(uint64_t)s * 4 + c];
      if (!e) {
        whole = false;
        break;
      }
      s = e & kStateMask;
      if (e & kFinalBit) {
        best = out[s].pid;
        cnt += out[s].mult;
      }
    }
    if (whole) {
      jump[x] = s | (cnt ? kFinalBit : 0u);
      jres[x] = OutEntry{best, cnt};
    } else {
      jump[x] = cnt ? kFinalBit : 0u;
      jres[x] = cnt ? OutEntry{best, cnt} : OutEntry{0, 0u};
    }
  }
}

// Filter bitmap words (bit x: jump[x] != 0) and their set bits.
__global__ void db_bitmap(const uint32_t* jump, uint64_t words, uint32_t* bm,
                          unsigned long long* set) {
  DB_FOR(w, words) {
    uint32_t v = 0;
    for (uint32_t b = 0; b < 32; ++b)
      if (jump[w * 32 + b]) v |= 1u << b;
    bm[w] = v;
    if (v) atomicAdd(set, (unsigned long long)__builtin_popcount(v));
  }
}

// Exclusive prefix over `n` counts, one workgroup (each thread a run):
// out[i] = sum of cnt[j], j < i.  cnt(i) is given as a functor.
template <typename F>
__device__ void db_block_scan(F cnt, uint64_t n, uint32_t* out) {
  __shared__ uint32_t part[1024];
  const uint64_t per = (n + blockDim.x - 1) / blockDim.x;
  const uint64_t lo = threadIdx.x * per, hi = min(n, lo + per);
  uint32_t s = 0;
  for (uint64_t i = lo; i < hi; ++i) s += cnt(i);
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (uint32_t i = 0; i < blockDim.x; ++i) {
      const uint32_t x = part[i];
      part[i] = run;
      run += x;
    }
  }
  __syncthreads();
  uint32_t run = part[threadIdx.x];
  for (uint64_t i = lo; i < hi; ++i) {
    const uint32_t x = cnt(i);
    out[i] = run;
    run += x;
  }
}

// Rank words of an image: set bits before each 128-bit group of the bitmap.
__global__ __launch_bounds__(1024) void db_rank(const uint32_t* bm, uint64_t groups,
                                                uint32_t* out) {
  db_block_scan([&](uint64_t g) {
    return (uint32_t)(__builtin_popcount(bm[4 * g]) + __builtin_popcount(bm[4 * g + 1]) +
                      __builtin_popcount(bm[4 * g + 2]) + __builtin_popcount(bm[4 * g + 3]));
  }, groups, out);
}

// Node bytes of one trie level (4 per word, first node in the low byte,
// padded to 16 nodes with zero bytes).
__global__ void db_level_bytes(const uint8_t* node, uint64_t first, uint64_t count,
                               uint64_t words, uint32_t* out) {
  DB_FOR(w, words) {
    uint32_t v = 0;
    for (uint32_t k = 0; k < 4; ++k)
      if (4 * w + k < count) v |= (uint32_t)node[first + 4 * w + k] << (8 * k);
    out[w] = v;
  }
}

// Rank words of a level: child bits of the level before each 16-node group.
__global__ __launch_bounds__(1024) void db_level_rank(const uint32_t* bytes, uint64_t groups,
                                                      uint32_t* out) {
  db_block_scan([&](uint64_t g) {
    uint32_t c = 0;
    for (int w = 0; w < 4; ++w) c += __builtin_popcount(bytes[4 * g + w] & 0x0F0F0F0Fu);
    return c;
  }, groups, out);
}

// Second filter at its largest size (two hashes of the first K bases of
// every pattern; the one-hash form too when `hash1` is set) and the prefix
// filter (the first K2 bases, exactly).
__global__ void db_filters(const uint64_t* w0, uint64_t n, uint32_t K, uint32_t* hash,
                           uint32_t* hash1, uint32_t K2, uint32_t* pfx) {
  DB_FOR(i, n) {
    const uint32_t top = (uint32_t)(w0[i] >> 32);     // first 16 bases, first on top
    const uint32_t key = K >= 16 ? top : top & ~((1u << (32 - 2 * K)) - 1u);
    const uint32_t h = (key * kHashMul) >> (32 - kHashMaxBits);
    const uint32_t h2 = (key * kHashMul2) >> (32 - kHashMaxBits);
    atomicOr(&hash[h >> 5], 1u << (h & 31));
    atomicOr(&hash[h2 >> 5], 1u << (h2 & 31));
    if (hash1) {
      const uint32_t x = (key >> (32 - 2 * K)) * kHash1Mul >> (32 - kHashMaxBits);
      atomicOr(&hash1[x >> 5], 1u << (x & 31));
    }
    if (K2) {
      const uint32_t x = (uint32_t)(w0[i] >> (64 - 2 * K2));
      atomicOr(&pfx[x >> 5], 1u << (x & 31));
    }
  }
}

// A smaller second-filter bitmap: the OR-fold of the largest.
__global__ void db_fold(const uint32_t* big, uint32_t fold, uint64_t words, uint32_t* out) {
  DB_FOR(w, words) {
    uint32_t v = 0;
    for (uint32_t b = 0; b < 32; ++b) {
      const uint64_t g = w * 32 + b;                  // target bit
      const uint64_t lo = g << fold, hi = (g + 1) << fold;
      bool any = false;
      for (uint64_t h = lo; h < hi && !any; h += 32) {
        const uint32_t word = big[h >> 5];
        const uint32_t span = (uint32_t)min<uint64_t>(32, hi - h);
        const uint32_t sh = (uint32_t)(h & 31);
        const uint32_t m = span == 32 ? 0xFFFFFFFFu : ((1u << span) - 1u) << sh;
        any = (word & m) != 0;
      }
      if (any) v |= 1u << b;
    }
    out[w] = v;
  }
}

__global__ void db_popcount(const uint32_t* v, uint64_t words, unsigned long long* set) {
  DB_FOR(w, words) if (v[w]) atomicAdd(set, (unsigned long long)__builtin_popcount(v[w]));
}

// Duplicates: a sorted pattern equal to the one before it (same string) is a
// further ID of its end state: key (state << 32 | id).
__global__ void db_dup_keys(const uint32_t* st, const uint32_t* len, const uint32_t* lcp,
                            const int32_t* id, uint64_t n, uint32_t* flag,
                            unsigned long long* key) {
  DB_FOR(i, n) {
    const bool dup = i > 0 && lcp[i] == len[i] && len[i - 1] == len[i];
    flag[i] = dup ? 1u : 0u;
    key[i] = ((unsigned long long)st[i * kDbMaxLen + len[i] - 1] << 32) | (uint32_t)id[i];
  }
}

__global__ void db_dup_compact(const uint32_t* flag, const uint32_t* pos,
                               const unsigned long long* key, uint64_t n,
                               unsigned long long* out) {
  DB_FOR(i, n) if (flag[i]) out[pos[i] - 1] = key[i];
}

__global__ void db_dup_split(const unsigned long long* key, uint64_t n, uint32_t* st,
                             int32_t* id) {
  DB_FOR(i, n) {
    st[i] = (uint32_t)(key[i] >> 32);
    id[i] = (int32_t)(uint32_t)key[i];
  }
}

// Device scratch of one build, freed at the end.
struct DbScratch {
  std::vector<void*> blocks;
  template <typename T>
  T* get(uint64_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<uint64_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
    blocks.push_back(p);
    return static_cast<T*>(p);
  }
  ~DbScratch() {
    for (void* p : blocks) (void)hipFree(p);
  }
};

#define DB_CHECK(x)                    \
  do {                                 \
    if (!(x)) return PFAC_E_NOMEM;     \
  } while (0)
#define DB_HIP(x)                                      \
  do {                                                 \
    if ((x) != hipSuccess) return PFAC_E_HIP;          \
  } while (0)
#define DB_LAUNCH() DB_HIP(hipGetLastError())

template <typename K, typename V>
static int db_sort_pairs(DbScratch& sc, const K* kin, K* kout, const V* vin, V* vout, uint64_t n,
                         uint32_t bits) {
  size_t bytes = 0;
  DB_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, (size_t)n, 0, bits));
  void* tmp = sc.get<uint8_t>(bytes);
  DB_CHECK(tmp);
  DB_HIP(rocprim::radix_sort_pairs(tmp, bytes, kin, kout, vin, vout, (size_t)n, 0, bits));
  return PFAC_OK;
}

static int db_scan(DbScratch& sc, const uint32_t* in, uint32_t* out, uint64_t n) {
  size_t bytes = 0;
  DB_HIP(rocprim::inclusive_scan(nullptr, bytes, in, out, (size_t)n, rocprim::plus<uint32_t>()));
  void* tmp = sc.get<uint8_t>(bytes);
  DB_CHECK(tmp);
  DB_HIP(rocprim::inclusive_scan(tmp, bytes, in, out, (size_t)n, rocprim::plus<uint32_t>()));
  return PFAC_OK;
}

// The device build.  Patterns validated (non-empty, A/C/G/T, at most 64
// bases) and packed on the host; ids[k] = ID of pattern k.
static int device_build(pfac_table* t, const char* const* patterns, const uint32_t* lengths,
                        const int32_t* ids, uint32_t num) {
  const uint64_t n = num;
  std::vector<uint64_t> hw0(n, 0), hw1(n, 0);
  std::vector<uint32_t> hlen(n);
  uint32_t maxl = 0, minl = UINT32_MAX;
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t L = lengths[i];
    for (uint32_t k = 0; k < L; ++k) {
      const uint8_t b = (uint8_t)patterns[i][k];
      const uint64_t c = b == 'A' ? 0 : b == 'C' ? 1 : b == 'G' ? 2 : 3;
      if (k < 32) hw0[i] |= c << (62 - 2 * k);
      else hw1[i] |= c << (62 - 2 * (k - 32));
    }
    hlen[i] = L;
    maxl = std::max(maxl, L);
    minl = std::min(minl, L);
  }
  DbScratch sc;
  uint64_t* w0 = sc.get<uint64_t>(n);
  uint64_t* w1 = sc.get<uint64_t>(n);
  uint64_t* tw = sc.get<uint64_t>(n);
  uint32_t* len = sc.get<uint32_t>(n);
  uint32_t* tl = sc.get<uint32_t>(n);
  int32_t* id = sc.get<int32_t>(n);
  int32_t* tid = sc.get<int32_t>(n);
  uint32_t* perm = sc.get<uint32_t>(n);
  uint32_t* perm2 = sc.get<uint32_t>(n);
  DB_CHECK(w0 && w1 && tw && len && tl && id && tid && perm && perm2);
  DB_HIP(hipMemcpy(tw, hw0.data(), n * 8, hipMemcpyHostToDevice));
  DB_HIP(hipMemcpy(w1, hw1.data(), n * 8, hipMemcpyHostToDevice));
  DB_HIP(hipMemcpy(tl, hlen.data(), n * 4, hipMemcpyHostToDevice));
  DB_HIP(hipMemcpy(tid, ids, n * 4, hipMemcpyHostToDevice));
  // 1. sort: least significant key first (ID, length, bases 32..63, bases
  //    0..31), each pass stable, carrying the permutation
  hipLaunchKernelGGL(db_iota, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, perm, n);
  DB_LAUNCH();
  {
    uint32_t* ukey = reinterpret_cast<uint32_t*>(len);   // scratch keys
    hipLaunchKernelGGL(db_gather<int32_t>, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, tid,
                       perm, reinterpret_cast<int32_t*>(ukey), n);
    DB_LAUNCH();
    uint32_t* sorted_keys = reinterpret_cast<uint32_t*>(id);
    int rc = db_sort_pairs<uint32_t, uint32_t>(sc, ukey, sorted_keys, perm, perm2, n, 32);
    if (rc) return rc;
    hipLaunchKernelGGL(db_gather<uint32_t>, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, tl,
                       perm2, ukey, n);
    DB_LAUNCH();
    rc = db_sort_pairs<uint32_t, uint32_t>(sc, ukey, sorted_keys, perm2, perm, n, 7);
    if (rc) return rc;
    hipLaunchKernelGGL(db_gather<uint64_t>, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, w1,
                       perm, w0, n);
    DB_LAUNCH();
    uint64_t* k64 = sc.get<uint64_t>(n);
    DB_CHECK(k64);
    rc = db_sort_pairs<uint64_t, uint32_t>(sc, w0, k64, perm, perm2, n, 64);
    if (rc) return rc;
    hipLaunchKernelGGL(db_gather<uint64_t>, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, tw,
                       perm2, w0, n);
    DB_LAUNCH();
    rc = db_sort_pairs<uint64_t, uint32_t>(sc, w0, k64, perm2, perm, n, 64);
    if (rc) return rc;
  }
  // sorted arrays
  uint64_t* w1s = sc.get<uint64_t>(n);
  DB_CHECK(w1s);
  hipLaunchKernelGGL(db_gather<uint64_t>, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, tw, perm,
                     w0, n);
  hipLaunchKernelGGL(db_gather<uint64_t>, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, w1, perm,
                     w1s, n);
  hipLaunchKernelGGL(db_gather<uint32_t>, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, tl, perm,
                     len, n);
  hipLaunchKernelGGL(db_gather<int32_t>, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, tid, perm,
                     id, n);
  DB_LAUNCH();
  // 2. states: per depth, the patterns that create one, numbered by a scan
  uint32_t* lcp = sc.get<uint32_t>(n);
  uint32_t* flag = sc.get<uint32_t>(n);
  uint32_t* cnt = sc.get<uint32_t>(n);
  uint32_t* st = sc.get<uint32_t>(n * kDbMaxLen);
  uint64_t* ds = sc.get<uint64_t>(kDbMaxLen + 2);
  DB_CHECK(lcp && flag && cnt && st && ds);
  hipLaunchKernelGGL(db_lcp, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, w0, w1s, len, n, lcp);
  DB_LAUNCH();
  const uint64_t one = 1;
  DB_HIP(hipMemcpy(ds + 1, &one, 8, hipMemcpyHostToDevice));
  for (uint32_t d = 1; d <= maxl; ++d) {
    hipLaunchKernelGGL(db_flags, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, lcp, len, n, d,
                       flag);
    DB_LAUNCH();
    int rc = db_scan(sc, flag, cnt, n);
    if (rc) return rc;
    hipLaunchKernelGGL(db_states, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, cnt, len, n, d, ds,
                       st);
    hipLaunchKernelGGL(db_level_end, dim3(1), dim3(64), 0, nullptr, cnt, n, d, ds);
    DB_LAUNCH();
  }
  std::vector<uint64_t> hds(maxl + 2, 0);
  DB_HIP(hipMemcpy(hds.data() + 1, ds + 1, (maxl + 1) * 8, hipMemcpyDeviceToHost));
  const uint64_t S = hds[maxl + 1];
  if (S >= kStateMask) return PFAC_E_TOO_LARGE;
  // 3. metadata the planner needs (what the host build would have)
  HostTable& h = t->host;
  h.num_states = S;
  h.num_patterns = num;
  h.max_len = maxl;
  h.min_len = minl;
  h.depth_start.assign(1, 0);
  for (uint32_t d = 1; d <= maxl; ++d) h.depth_start.push_back(hds[d]);
  h.depth_start.push_back(S);
  uint32_t full = 0;
  for (uint32_t d = 1; d + 1 < h.depth_start.size(); ++d) {
    const uint64_t c = h.depth_start[d + 1] - h.depth_start[d];
    if (d < 32 && c == (1ull << (2 * d))) full = d; else break;
  }
  h.max_depth_full = full;
  for (uint32_t D = kMinJump; D <= kMaxJump; ++D) {
    HostTable::Image& im = h.image[D];
    const uint64_t E = 1ull << (2 * D);
    uint64_t words = E / 32 + E / 128;
    im.levels = 0;
    for (uint32_t k = 0; k < kImageLevels; ++k) {
      const uint32_t d = D + k;
      if (d + 1 >= h.depth_start.size()) break;
      const uint64_t count = h.depth_start[d + 1] - h.depth_start[d];
      const uint64_t groups = (count + 15) / 16;
      const uint64_t need = words + groups * 4 + ((groups + 3) & ~3ull);
      if (need * 4 > kImageMaxBytes) break;
      im.byte_off[k] = (uint32_t)words;
      words += groups * 4;
      im.pre_off[k] = (uint32_t)words;
      words += groups;
      words = (words + 3) & ~3ull;
      im.upto[k] = (uint32_t)words;
      im.levels = k + 1;
    }
  }
  h.hash_k = std::min(minl, kHashK);
  h.pfx_k = minl >= kPfxMinK ? std::min(minl, kPfxMaxK) : 0;
  // duplicates (needed for the layout): equal strings are adjacent
  unsigned long long* dkey = sc.get<unsigned long long>(n);
  unsigned long long* dsorted = sc.get<unsigned long long>(n);
  uint32_t* dpos = sc.get<uint32_t>(n);
  DB_CHECK(dkey && dsorted && dpos);
  hipLaunchKernelGGL(db_dup_keys, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, st, len, lcp, id, n,
                     flag, dkey);
  DB_LAUNCH();
  int rc = db_scan(sc, flag, dpos, n);
  if (rc) return rc;
  uint32_t ndup = 0;
  DB_HIP(hipMemcpy(&ndup, dpos + n - 1, 4, hipMemcpyDeviceToHost));
  // 4. the table's memory, then every array
  rc = alloc_table(t, ndup);
  if (rc) return rc;
  const TableLayout& L = t->layout;
  uint8_t* base = static_cast<uint8_t*>(t->dmem);
  uint32_t* next = reinterpret_cast<uint32_t*>(base + L.o_next);
  OutEntry* out = reinterpret_cast<OutEntry*>(base + L.o_out);
  uint32_t* chain = reinterpret_cast<uint32_t*>(base + L.o_chain);
  uint8_t* fin = sc.get<uint8_t>(S);
  uint8_t* node = sc.get<uint8_t>(S);
  unsigned long long* sets = sc.get<unsigned long long>(48);
  DB_CHECK(fin && node && sets);
  DB_HIP(hipMemset(fin, 0, S));
  DB_HIP(hipMemset(sets, 0, 48 * 8));
  hipLaunchKernelGGL(db_out_init, dim3(db_grid(S)), dim3(kDbBlock), 0, nullptr, out, S);
  hipLaunchKernelGGL(db_finals, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, st, len, id, n, out,
                     fin);
  hipLaunchKernelGGL(db_out_fix, dim3(db_grid(S)), dim3(kDbBlock), 0, nullptr, out, S);
  hipLaunchKernelGGL(db_edges, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, st, len, lcp, w0, w1s,
                     fin, n, next);
  hipLaunchKernelGGL(db_nodes, dim3(db_grid(S)), dim3(kDbBlock), 0, nullptr, next, out, S, node);
  hipLaunchKernelGGL(db_chains, dim3(db_grid(S)), dim3(kDbBlock), 0, nullptr, next, node, S, chain);
  DB_LAUNCH();
  for (uint32_t D = kMinJump; D <= kMaxJump; ++D) {
    const uint64_t E = 1ull << (2 * D);
    uint32_t* jump = reinterpret_cast<uint32_t*>(base + L.o_jump[D]);
    OutEntry* jres = reinterpret_cast<OutEntry*>(base + L.o_jres[D]);
    uint32_t* im = reinterpret_cast<uint32_t*>(base + L.o_im[D]);
    hipLaunchKernelGGL(db_jump, dim3(db_grid(E)), dim3(kDbBlock), 0, nullptr, next, out, D, jump,
                       jres);
    hipLaunchKernelGGL(db_bitmap, dim3(db_grid(E / 32)), dim3(kDbBlock), 0, nullptr, jump, E / 32,
                       im, sets + D);
    hipLaunchKernelGGL(db_rank, dim3(1), dim3(1024), 0, nullptr, im, E / 128, im + E / 32);
    DB_LAUNCH();
    const HostTable::Image& hi = h.image[D];
    for (uint32_t k = 0; k < hi.levels; ++k) {
      const uint32_t d = D + k;
      const uint64_t first = h.depth_start[d], count = h.depth_start[d + 1] - first;
      const uint64_t groups = (count + 15) / 16;
      hipLaunchKernelGGL(db_level_bytes, dim3(db_grid(groups * 4)), dim3(kDbBlock), 0, nullptr,
                         node, first, count, groups * 4, im + hi.byte_off[k]);
      hipLaunchKernelGGL(db_level_rank, dim3(1), dim3(1024), 0, nullptr, im + hi.byte_off[k],
                         groups, im + hi.pre_off[k]);
      DB_LAUNCH();
    }
  }
  uint32_t* big = reinterpret_cast<uint32_t*>(base + L.o_hash[kHashMaxBits]);
  uint32_t* big1 = L.hash1_words[kHashMaxBits]
                       ? reinterpret_cast<uint32_t*>(base + L.o_hash1[kHashMaxBits]) : nullptr;
  uint32_t* pfx = reinterpret_cast<uint32_t*>(base + L.o_pfx);
  hipLaunchKernelGGL(db_filters, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, w0, n, h.hash_k, big,
                     big1, h.pfx_k, pfx);
  DB_LAUNCH();
  for (uint32_t b = kHashMinBits; b <= kHashMaxBits; ++b) {
    uint32_t* hb = reinterpret_cast<uint32_t*>(base + L.o_hash[b]);
    if (b < kHashMaxBits)
      hipLaunchKernelGGL(db_fold, dim3(db_grid(L.hash_words[b])), dim3(kDbBlock), 0, nullptr, big,
                         kHashMaxBits - b, (uint64_t)L.hash_words[b], hb);
    hipLaunchKernelGGL(db_popcount, dim3(db_grid(L.hash_words[b])), dim3(kDbBlock), 0, nullptr, hb,
                       (uint64_t)L.hash_words[b], sets + 11 + (b - kHashMinBits));
    DB_LAUNCH();
    if (big1) {
      uint32_t* h1 = reinterpret_cast<uint32_t*>(base + L.o_hash1[b]);
      if (b < kHashMaxBits)
        hipLaunchKernelGGL(db_fold, dim3(db_grid(L.hash1_words[b])), dim3(kDbBlock), 0, nullptr,
                           big1, kHashMaxBits - b, (uint64_t)L.hash1_words[b], h1);
      hipLaunchKernelGGL(db_popcount, dim3(db_grid(L.hash1_words[b])), dim3(kDbBlock), 0, nullptr,
                         h1, (uint64_t)L.hash1_words[b], sets + 31 + (b - kHashMinBits));
      DB_LAUNCH();
    }
  }
  if (L.pfx_words) {
    hipLaunchKernelGGL(db_popcount, dim3(db_grid(L.pfx_words)), dim3(kDbBlock), 0, nullptr, pfx,
                       L.pfx_words, sets + 30);
    DB_LAUNCH();
  }
  if (ndup) {
    unsigned long long* comp = sc.get<unsigned long long>(ndup);
    DB_CHECK(comp);
    hipLaunchKernelGGL(db_dup_compact, dim3(db_grid(n)), dim3(kDbBlock), 0, nullptr, flag, dpos,
                       dkey, n, comp);
    DB_LAUNCH();
    size_t bytes = 0;
    DB_HIP(rocprim::radix_sort_keys(nullptr, bytes, comp, dsorted, (size_t)ndup));
    void* tmp = sc.get<uint8_t>(bytes);
    DB_CHECK(tmp);
    DB_HIP(rocprim::radix_sort_keys(tmp, bytes, comp, dsorted, (size_t)ndup));
    hipLaunchKernelGGL(db_dup_split, dim3(db_grid(ndup)), dim3(kDbBlock), 0, nullptr, dsorted,
                       (uint64_t)ndup, reinterpret_cast<uint32_t*>(base + L.o_dups),
                       reinterpret_cast<int32_t*>(base + L.o_dupi));
    DB_LAUNCH();
  }
  unsigned long long hs[48];
  DB_HIP(hipMemcpy(hs, sets, sizeof(hs), hipMemcpyDeviceToHost));   // waits for every kernel
  for (uint32_t D = kMinJump; D <= kMaxJump; ++D) h.bitmap_set[D] = hs[D];
  for (uint32_t b = kHashMinBits; b <= kHashMaxBits; ++b) {
    h.hash_set[b] = (uint32_t)hs[11 + (b - kHashMinBits)];
    h.hash1_set[b] = big1 ? (uint32_t)hs[31 + (b - kHashMinBits)] : 0u;
  }
  h.pfx_set = L.pfx_words ? hs[30] : 0;
  return build_derived(t);
}

// Check, then build on the device; pattern k gets ID ids[k].
static int build_on_device(const char* const* patterns, const uint32_t* lengths,
                           const int32_t* ids, uint32_t num, pfac_table** out,
                           int64_t* bad_index) {
  if (bad_index) *bad_index = -1;
  if (!out || !patterns || !lengths || num == 0 || !ids) return PFAC_E_ARG;
  *out = nullptr;
  for (uint32_t k = 0; k < num; ++k) {
    bool ok = lengths[k] > 0 && lengths[k] <= kDbMaxLen && patterns[k] != nullptr && ids[k] > 0;
    for (uint32_t i = 0; ok && i < lengths[k]; ++i) {
      const uint8_t b = (uint8_t)patterns[k][i];
      ok = b == 'A' || b == 'C' || b == 'G' || b == 'T';
    }
    if (!ok) {
      if (bad_index) *bad_index = k;
      return lengths[k] > kDbMaxLen || ids[k] <= 0 ? PFAC_E_ARG : PFAC_E_PATTERN;
    }
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PFAC_E_NODEV;
  if (!device_ok(dev)) return PFAC_E_NODEV;
  pfac_table* t = new (std::nothrow) pfac_table();
  if (!t) return PFAC_E_NOMEM;
  t->device = dev;
  int rc = remember_patterns(t, patterns, lengths, num, ids);
  if (!rc) rc = device_build(t, patterns, lengths, ids, num);
  if (rc) {
    if (t->dmem) (void)hipFree(t->dmem);
    delete t;
    return rc;
  }
  *out = t;
  return PFAC_OK;
}

}  // namespace pfac

using namespace pfac;

extern "C" {

int pfac_build_table_device(const char* const* patterns, const uint32_t* lengths,
                            const int32_t* ids, uint32_t num, pfac_table** out,
                            int64_t* bad_index) {
  if (ids) return build_on_device(patterns, lengths, ids, num, out, bad_index);
  std::vector<int32_t> seq(num);
  for (uint32_t k = 0; k < num; ++k) seq[k] = (int32_t)(k + 1);
  return build_on_device(patterns, lengths, seq.data(), num, out, bad_index);
}

int pfac_table_update(const pfac_table* base, const char* const* add, const uint32_t* add_lens,
                      uint32_t num_add, const int32_t* remove_ids, uint32_t num_remove,
                      pfac_table** out, int32_t* first_new_id) {
  if (!base || !out || (num_add && (!add || !add_lens)) || (num_remove && !remove_ids) ||
      base->alphabet != 4)
    return PFAC_E_ARG;
  *out = nullptr;
  try {
    std::vector<int32_t> gone(remove_ids, remove_ids + num_remove);
    std::sort(gone.begin(), gone.end());
    int32_t next_id = 0;
    for (int32_t v : base->ids) next_id = std::max(next_id, v);
    ++next_id;
    std::vector<const char*> p;
    std::vector<uint32_t> l;
    std::vector<int32_t> ids;
    for (size_t k = 0; k < base->pats.size(); ++k) {
      if (std::binary_search(gone.begin(), gone.end(), base->ids[k])) continue;
      p.push_back(base->pats[k].data());
      l.push_back((uint32_t)base->pats[k].size());
      ids.push_back(base->ids[k]);
    }
    if (first_new_id) *first_new_id = next_id;
    for (uint32_t k = 0; k < num_add; ++k) {
      p.push_back(add[k]);
      l.push_back(add_lens[k]);
      ids.push_back(next_id + (int32_t)k);
    }
    if (p.empty()) return PFAC_E_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PFAC_E_NODEV;
    if (dev != base->device) return PFAC_E_ARG;
    int64_t bad = -1;
    return build_on_device(p.data(), l.data(), ids.data(), (uint32_t)p.size(), out, &bad);
  } catch (const std::bad_alloc&) {
    return PFAC_E_NOMEM;
  }
}

}  // extern "C"
