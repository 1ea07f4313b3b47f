// Host-side construction of the failure-less goto trie.
//
// Paper Sec. V.A: the table has one row per state and four columns (one
// per base); patterns are inserted one at a time, each new character that
// has no transition yet creating a new state; Sec. V.B: the host builds the
// table and copies it to the device.  Differences from the paper's table:
//   * a pattern's last character also allocates a fresh state (the printed
//     sample table reuses the number it gives the last cell, which makes two
//     prefixes share a row);
//   * states are renumbered breadth-first after insertion (the state order
//     Nishimura et al. use for cache locality, Sec. II), so the shallow states
//     that every walk visits form a contiguous prefix that fits in LDS;
//   * the matched-pattern ID moves out of the cell into a per-state output
//     entry; the cell keeps one bit saying the child is final.
#include <string.h>

#include <algorithm>
#include <array>
#include <new>
#include <utility>

#include "pfac_internal.h"

namespace pfac {

static inline int base_code(uint8_t b) {
  switch (b) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
  }
}

int build_host_table(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                     HostTable* out, int64_t* bad_index) {
  if (bad_index) *bad_index = -1;
  if (!patterns || !lengths || num == 0 || !out) return PFAC_E_ARG;
  for (uint32_t k = 0; k < num; ++k) {
    bool ok = lengths[k] > 0 && patterns[k] != nullptr;
    for (uint32_t t = 0; ok && t < lengths[k]; ++t)
      ok = base_code((uint8_t)patterns[k][t]) >= 0;
    if (!ok) {
      if (bad_index) *bad_index = k;
      return PFAC_E_PATTERN;
    }
  }
  try {
    // 1. insertion-order trie
    std::vector<std::array<uint32_t, 4>> kids(1, {0, 0, 0, 0});
    std::vector<int32_t> fin_pid(1, 0);
    std::vector<uint32_t> fin_mult(1, 0);
    std::vector<std::pair<uint32_t, int32_t>> dups;   // (insertion-order state, id)
    uint32_t maxl = 0, minl = UINT32_MAX;
    for (uint32_t k = 0; k < num; ++k) {
      uint32_t s = 0;
      for (uint32_t t = 0; t < lengths[k]; ++t) {
        int a = base_code((uint8_t)patterns[k][t]);
        if (kids[s][a] == 0) {
          if (kids.size() >= (size_t)kStateMask) return PFAC_E_TOO_LARGE;
          kids[s][a] = (uint32_t)kids.size();
          kids.push_back({0, 0, 0, 0});
          fin_pid.push_back(0);
          fin_mult.push_back(0);
        }
        s = kids[s][a];
      }
      if (fin_pid[s] == 0) fin_pid[s] = (int32_t)(k + 1);   // smallest ID wins
      else dups.emplace_back(s, (int32_t)(k + 1));          // a further ID of the same string
      fin_mult[s] += 1;
      maxl = std::max(maxl, lengths[k]);
      minl = std::min(minl, lengths[k]);
    }
    const uint64_t S = kids.size();
    // 2. breadth-first renumbering (children visited in A,C,G,T order)
    std::vector<uint32_t> order;  // order[new] = old
    order.reserve(S);
    std::vector<uint32_t> newid(S, 0);
    std::vector<uint64_t> depth_start;
    order.push_back(0);
    depth_start.push_back(0);
    size_t level_begin = 0;
    while (level_begin < order.size()) {
      size_t level_end = order.size();
      for (size_t i = level_begin; i < level_end; ++i) {
        for (int a = 0; a < 4; ++a) {
          uint32_t c = kids[order[i]][a];
          if (c) order.push_back(c);
        }
      }
      if (order.size() > level_end) depth_start.push_back(level_end);
      level_begin = level_end;
    }
    depth_start.push_back(S);
    for (uint64_t i = 0; i < S; ++i) newid[order[i]] = (uint32_t)i;
    // 3. packed tables
    out->next.assign(S * 4, 0);
    out->out.assign(S, OutEntry{0, 0});
    for (uint64_t i = 0; i < S; ++i) {
      uint32_t o = order[i];
      for (int a = 0; a < 4; ++a) {
        uint32_t c = kids[o][a];
        if (c) out->next[i * 4 + a] = newid[c] | (fin_pid[c] ? kFinalBit : 0u);
      }
      out->out[i] = OutEntry{fin_pid[o], fin_mult[o]};
    }
    for (auto& d : dups) d.first = newid[d.first];
    std::sort(dups.begin(), dups.end());
    out->dup_state.resize(dups.size());
    out->dup_id.resize(dups.size());
    for (size_t i = 0; i < dups.size(); ++i) {
      out->dup_state[i] = dups[i].first;
      out->dup_id[i] = dups[i].second;
    }
    out->num_states = S;
    out->num_patterns = num;
    out->max_len = maxl;
    out->min_len = minl;
    out->depth_start = depth_start;
    // deepest fully populated level
    uint32_t full = 0;
    for (uint32_t d = 1; d + 1 < depth_start.size(); ++d) {
      uint64_t cnt = depth_start[d + 1] - depth_start[d];
      if (d < 32 && cnt == (1ull << (2 * d))) full = d; else break;
    }
    out->max_depth_full = full;
    // 4. node bytes: child mask and final flag of every state
    out->node.assign(S, 0);
    for (uint64_t i = 0; i < S; ++i) {
      uint8_t v = out->out[i].pid ? 0x10 : 0;
      for (int a = 0; a < 4; ++a)
        if (out->next[i * 4 + a]) v |= (uint8_t)(1u << a);
      out->node[i] = v;
    }
    // 4b. runs of single-child steps below every state (path compression)
    out->chain.assign(2 * S, 0);
    for (uint64_t i = 0; i < S; ++i) {
      uint32_t len = 0, codes = 0;
      uint64_t cur = i;
      bool fin = false;
      while (len < kChainMax) {
        const uint8_t nb = out->node[cur];
        const uint32_t kids_mask = nb & 0x0Fu;
        if (__builtin_popcount(kids_mask) != 1) break;      // not a single child
        const uint32_t a = (uint32_t)__builtin_ctz(kids_mask);
        const uint32_t e = out->next[cur * 4 + a];
        codes |= a << (30 - 2 * len);
        ++len;
        cur = e & kStateMask;
        fin = (e & kFinalBit) != 0;
        if (fin) break;                                      // a pattern ends here
      }
      if (len >= 2) {
        out->chain[2 * i] = codes | len;
        out->chain[2 * i + 1] = (uint32_t)cur | (fin ? kFinalBit : 0u);
      }
    }
    // 5. root jump tables of depth D: the result of the first D steps of the
    //    walk for every D-base window (first base most significant), filled by
    //    a depth-first pass over the trie; windows that leave the trie early
    //    form one contiguous key range each
    for (uint32_t D = kMinJump; D <= kMaxJump; ++D) {
      const uint64_t E = 1ull << (2 * D);
      out->jump[D].assign(E, 0);
      out->jres[D].assign(E, OutEntry{0, 0});
      out->bitmap[D].assign(E / 32, 0);
      struct Frame { uint32_t s; uint32_t d; uint64_t key; int32_t best; uint32_t cnt; };
      std::vector<Frame> stack;
      stack.push_back(Frame{0, 0, 0, 0, 0});
      while (!stack.empty()) {
        const Frame f = stack.back();
        stack.pop_back();
        if (f.d == D) {
          out->jump[D][f.key] = f.s | (f.cnt ? kFinalBit : 0u);
          out->jres[D][f.key] = OutEntry{f.best, f.cnt};
          continue;
        }
        for (uint32_t a = 0; a < 4; ++a) {
          const uint32_t e = out->next[(uint64_t)f.s * 4 + a];
          const uint64_t key = (f.key << 2) | a;
          if (e == 0) {
            // the walk stops after d bases: every window with this d+1 base
            // prefix gets the finals passed so far (nothing if none)
            if (f.cnt) {
              const uint64_t span = 1ull << (2 * (D - f.d - 1));
              for (uint64_t x = key * span; x < (key + 1) * span; ++x) {
                out->jump[D][x] = kFinalBit;
                out->jres[D][x] = OutEntry{f.best, f.cnt};
              }
            }
            continue;
          }
          const uint32_t c = e & kStateMask;
          Frame g{c, f.d + 1, key, f.best, f.cnt};
          if (e & kFinalBit) {
            g.best = out->out[c].pid;
            g.cnt += out->out[c].mult;
          }
          stack.push_back(g);
        }
      }
      for (uint64_t x = 0; x < E; ++x)
        if (out->jump[D][x]) out->bitmap[D][x >> 5] |= 1u << (x & 31);
      for (uint32_t w : out->bitmap[D]) out->bitmap_set[D] += (uint32_t)__builtin_popcount(w);
      // LDS image: bitmap, its rank words, then node bytes and rank words of
      // levels D, D+1, ... while the image stays within kImageMaxBytes
      HostTable::Image& im = out->image[D];
      im.words = out->bitmap[D];
      uint32_t run = 0;
      for (uint64_t g = 0; g < E / 128; ++g) {
        im.words.push_back(run);
        for (int k = 0; k < 4; ++k) run += (uint32_t)__builtin_popcount(out->bitmap[D][4 * g + k]);
      }
      im.levels = 0;
      for (uint32_t k = 0; k < kImageLevels; ++k) {
        const uint32_t d = D + k;
        if (d + 1 >= depth_start.size()) break;
        const uint64_t first = depth_start[d], count = depth_start[d + 1] - depth_start[d];
        const uint64_t groups = (count + 15) / 16;
        const uint64_t need = im.words.size() + groups * 4 + ((groups + 3) & ~3ull);
        if (need * 4 > kImageMaxBytes) break;
        im.byte_off[k] = (uint32_t)im.words.size();
        std::vector<uint32_t> bytes(groups * 4, 0);
        for (uint64_t i = 0; i < count; ++i)
          bytes[i >> 2] |= (uint32_t)out->node[first + i] << (8 * (i & 3));
        im.words.insert(im.words.end(), bytes.begin(), bytes.end());
        im.pre_off[k] = (uint32_t)im.words.size();
        uint32_t c = 0;
        for (uint64_t g = 0; g < groups; ++g) {
          im.words.push_back(c);
          for (int w = 0; w < 4; ++w) c += (uint32_t)__builtin_popcount(bytes[4 * g + w] & 0x0F0F0F0Fu);
        }
        while (im.words.size() & 3) im.words.push_back(0);
        im.upto[k] = (uint32_t)im.words.size();
        im.levels = k + 1;
      }
    }
    // 6. second filter: two hashes of the first K bases of every pattern,
    //    one bitmap per size; a smaller one is the OR of adjacent bits of the
    //    largest (a hash of `bits` bits is the top bits of its product)
    out->hash_k = num ? std::min(minl, kHashK) : 0;
    if (out->hash_k) {
      std::vector<uint32_t>& big = out->hash[kHashMaxBits];
      big.assign((1u << kHashMaxBits) / 32, 0);
      const uint32_t K = out->hash_k;
      for (uint32_t i = 0; i < num; ++i) {
        uint32_t key = 0;
        for (uint32_t k = 0; k < K; ++k)
          key |= (uint32_t)base_code((uint8_t)patterns[i][k]) << (30 - 2 * k);
        const uint32_t h = (key * kHashMul) >> (32 - kHashMaxBits);
        const uint32_t h2 = (key * kHashMul2) >> (32 - kHashMaxBits);
        big[h >> 5] |= 1u << (h & 31);
        big[h2 >> 5] |= 1u << (h2 & 31);
      }
      for (uint32_t b = kHashMinBits; b < kHashMaxBits; ++b) {
        std::vector<uint32_t>& v = out->hash[b];
        v.assign((1u << b) / 32, 0);
        const uint32_t fold = kHashMaxBits - b;
        for (uint32_t h = 0; h < (1u << kHashMaxBits); ++h)
          if ((big[h >> 5] >> (h & 31)) & 1u) {
            const uint32_t g = h >> fold;
            v[g >> 5] |= 1u << (g & 31);
          }
      }
      for (uint32_t b = kHashMinBits; b <= kHashMaxBits; ++b)
        for (uint32_t w : out->hash[b]) out->hash_set[b] += (uint32_t)__builtin_popcount(w);
    }
    //    the one-hash form (K <= 12), folded the same way
    if (out->hash_k && out->hash_k <= kHash1MaxK) {
      const uint32_t K = out->hash_k;
      std::vector<uint32_t>& big = out->hash1[kHashMaxBits];
      big.assign((1u << kHashMaxBits) / 32, 0);
      for (uint32_t i = 0; i < num; ++i) {
        uint32_t key = 0;
        for (uint32_t k = 0; k < K; ++k)
          key = (key << 2) | (uint32_t)base_code((uint8_t)patterns[i][k]);
        const uint32_t h = (key * kHash1Mul) >> (32 - kHashMaxBits);
        big[h >> 5] |= 1u << (h & 31);
      }
      for (uint32_t b = kHashMinBits; b < kHashMaxBits; ++b) {
        std::vector<uint32_t>& v = out->hash1[b];
        v.assign((1u << b) / 32, 0);
        const uint32_t fold = kHashMaxBits - b;
        for (uint32_t h = 0; h < (1u << kHashMaxBits); ++h)
          if ((big[h >> 5] >> (h & 31)) & 1u) {
            const uint32_t g = h >> fold;
            v[g >> 5] |= 1u << (g & 31);
          }
      }
      for (uint32_t b = kHashMinBits; b <= kHashMaxBits; ++b)
        for (uint32_t w : out->hash1[b]) out->hash1_set[b] += (uint32_t)__builtin_popcount(w);
    }
    // 7. prefix filter: the first K2 bases of every pattern, exactly, one bit
    //    per K2-base key (first base most significant)
    out->pfx_k = (num && minl >= kPfxMinK) ? std::min(minl, kPfxMaxK) : 0;
    if (out->pfx_k) {
      const uint32_t K2 = out->pfx_k;
      out->pfx.assign((size_t)1 << (2 * K2 - 5), 0);
      for (uint32_t i = 0; i < num; ++i) {
        uint32_t key = 0;
        for (uint32_t k = 0; k < K2; ++k)
          key = (key << 2) | (uint32_t)base_code((uint8_t)patterns[i][k]);
        out->pfx[key >> 5] |= 1u << (key & 31);
      }
      for (uint32_t w : out->pfx) out->pfx_set += (uint32_t)__builtin_popcount(w);
    }
  } catch (const std::bad_alloc&) {
    return PFAC_E_NOMEM;
  }
  return PFAC_OK;
}

int build_host_bytes(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                     HostBytes* out, int64_t* bad_index) {
  if (bad_index) *bad_index = -1;
  if (!patterns || !lengths || num == 0 || !out) return PFAC_E_ARG;
  for (uint32_t k = 0; k < num; ++k) {
    if (lengths[k] == 0 || patterns[k] == nullptr) {
      if (bad_index) *bad_index = k;
      return PFAC_E_PATTERN;
    }
  }
  try {
    // 1. insertion-order trie, one new state per new byte (children kept as
    //    sorted (byte, child) lists)
    std::vector<std::vector<std::pair<uint8_t, uint32_t>>> kids(1);
    std::vector<int32_t> fin_pid(1, 0);
    std::vector<uint32_t> fin_mult(1, 0);
    uint32_t maxl = 0, minl = UINT32_MAX;
    for (uint32_t k = 0; k < num; ++k) {
      uint32_t s = 0;
      for (uint32_t t = 0; t < lengths[k]; ++t) {
        const uint8_t a = (uint8_t)patterns[k][t];
        auto& v = kids[s];
        auto it = std::lower_bound(v.begin(), v.end(), std::make_pair(a, 0u),
                                   [](const std::pair<uint8_t, uint32_t>& x,
                                      const std::pair<uint8_t, uint32_t>& y) {
                                     return x.first < y.first;
                                   });
        if (it == v.end() || it->first != a) {
          if (kids.size() >= kBytesMaxStates) return PFAC_E_TOO_LARGE;
          const uint32_t c = (uint32_t)kids.size();
          it = kids[s].insert(it, std::make_pair(a, c));
          kids.emplace_back();
          fin_pid.push_back(0);
          fin_mult.push_back(0);
          s = c;
        } else {
          s = it->second;
        }
      }
      if (fin_pid[s] == 0) fin_pid[s] = (int32_t)(k + 1);   // smallest ID wins
      fin_mult[s] += 1;
      maxl = std::max(maxl, lengths[k]);
      minl = std::min(minl, lengths[k]);
    }
    const uint64_t S = kids.size();
    // 2. breadth-first renumbering (children in byte order)
    std::vector<uint32_t> order;
    order.reserve(S);
    std::vector<uint32_t> newid(S, 0);
    std::vector<uint64_t> depth_start;
    order.push_back(0);
    depth_start.push_back(0);
    size_t level_begin = 0;
    while (level_begin < order.size()) {
      const size_t level_end = order.size();
      for (size_t i = level_begin; i < level_end; ++i)
        for (const auto& e : kids[order[i]]) order.push_back(e.second);
      if (order.size() > level_end) depth_start.push_back(level_end);
      level_begin = level_end;
    }
    depth_start.push_back(S);
    for (uint64_t i = 0; i < S; ++i) newid[order[i]] = (uint32_t)i;
    // 3. outputs, root row, hash table of the other edges (load <= 1/2)
    out->out.assign(S, OutEntry{0, 0});
    uint64_t edges = 0;
    for (uint64_t i = 0; i < S; ++i) {
      out->out[i] = OutEntry{fin_pid[order[i]], fin_mult[order[i]]};
      edges += kids[order[i]].size();
    }
    memset(out->root, 0, sizeof(out->root));
    for (const auto& e : kids[0])
      out->root[e.first] = newid[e.second] | (fin_pid[e.second] ? kFinalBit : 0u);
    const uint64_t inner = edges - kids[0].size();
    uint32_t bits = 8;
    while ((1ull << bits) < 2 * inner) ++bits;
    out->hash_bits = bits;
    out->slots.assign(2ull << bits, kBytesEmptyKey);
    for (uint64_t i = 1; i < S; ++i) {
      for (const auto& e : kids[order[i]]) {
        const uint32_t key = ((uint32_t)i << 8) | e.first;
        uint32_t h = bytes_hash(key, bits);
        while (out->slots[2 * h] != kBytesEmptyKey) h = (h + 1) & ((1u << bits) - 1);
        out->slots[2 * h] = key;
        out->slots[2 * h + 1] = newid[e.second] | (fin_pid[e.second] ? kFinalBit : 0u);
      }
    }
    out->num_states = S;
    out->num_patterns = num;
    out->max_len = maxl;
    out->min_len = minl;
    out->depth_start = depth_start;
    out->edges = edges;
  } catch (const std::bad_alloc&) {
    return PFAC_E_NOMEM;
  }
  return PFAC_OK;
}

}  // namespace pfac

extern "C" int pfac_build_host(const char* const* patterns, const uint32_t* lengths, uint32_t num,
                               uint32_t* next, int32_t* pid, uint32_t* mult, uint64_t cap,
                               uint32_t depth, uint32_t* jump, int32_t* jump_pid,
                               uint32_t* jump_cnt, uint64_t* num_states, int64_t* bad_index) {
  using namespace pfac;
  if (!num_states) return PFAC_E_ARG;
  if (jump && (depth < kMinJump || depth > kMaxJump)) return PFAC_E_ARG;
  HostTable h;
  int rc = build_host_table(patterns, lengths, num, &h, bad_index);
  if (rc != PFAC_OK) return rc;
  *num_states = h.num_states;
  if (h.num_states <= cap) {
    if (next) memcpy(next, h.next.data(), h.next.size() * sizeof(uint32_t));
    for (uint64_t s = 0; s < h.num_states; ++s) {
      if (pid) pid[s] = h.out[s].pid;
      if (mult) mult[s] = h.out[s].mult;
    }
  }
  if (jump) {
    const uint64_t E = 1ull << (2 * depth);
    memcpy(jump, h.jump[depth].data(), E * sizeof(uint32_t));
    for (uint64_t x = 0; x < E; ++x) {
      if (jump_pid) jump_pid[x] = h.jres[depth][x].pid;
      if (jump_cnt) jump_cnt[x] = h.jres[depth][x].mult;
    }
  }
  return PFAC_OK;
}

extern "C" int pfac_build_host_image(const char* const* patterns, const uint32_t* lengths,
                                     uint32_t num, uint32_t depth, uint32_t* words, uint64_t cap,
                                     uint32_t* meta, uint64_t* num_words, int64_t* bad_index) {
  using namespace pfac;
  if (!num_words || depth < kMinJump || depth > kMaxJump) return PFAC_E_ARG;
  HostTable h;
  int rc = build_host_table(patterns, lengths, num, &h, bad_index);
  if (rc != PFAC_OK) return rc;
  const HostTable::Image& im = h.image[depth];
  *num_words = im.words.size();
  if (im.words.size() <= cap) {
    if (words) memcpy(words, im.words.data(), im.words.size() * sizeof(uint32_t));
    if (meta) {
      meta[0] = im.levels;
      for (uint32_t k = 0; k < kImageLevels; ++k) {
        meta[1 + 3 * k] = k < im.levels ? im.byte_off[k] : 0;
        meta[2 + 3 * k] = k < im.levels ? im.pre_off[k] : 0;
        meta[3 + 3 * k] = k < im.levels ? im.upto[k] : 0;
      }
    }
  }
  return PFAC_OK;
}

extern "C" int pfac_build_host_hash(const char* const* patterns, const uint32_t* lengths,
                                    uint32_t num, uint32_t bits, uint32_t* words, uint32_t* k,
                                    int64_t* bad_index) {
  using namespace pfac;
  if (bits < kHashMinBits || bits > kHashMaxBits) return PFAC_E_ARG;
  HostTable h;
  int rc = build_host_table(patterns, lengths, num, &h, bad_index);
  if (rc != PFAC_OK) return rc;
  if (k) *k = h.hash_k;
  if (words) {
    if (h.hash_k) memcpy(words, h.hash[bits].data(), h.hash[bits].size() * sizeof(uint32_t));
    else memset(words, 0, ((size_t)1 << bits) / 8);
  }
  return PFAC_OK;
}

extern "C" int pfac_build_host_hash1(const char* const* patterns, const uint32_t* lengths,
                                     uint32_t num, uint32_t bits, uint32_t* words, uint32_t* k,
                                     int64_t* bad_index) {
  using namespace pfac;
  if (bits < kHashMinBits || bits > kHashMaxBits) return PFAC_E_ARG;
  HostTable h;
  int rc = build_host_table(patterns, lengths, num, &h, bad_index);
  if (rc != PFAC_OK) return rc;
  if (k) *k = h.hash_k;
  if (words) {
    if (!h.hash1[bits].empty())
      memcpy(words, h.hash1[bits].data(), h.hash1[bits].size() * sizeof(uint32_t));
    else
      memset(words, 0, ((size_t)1 << bits) / 8);
  }
  return h.hash_k && h.hash_k <= kHash1MaxK ? PFAC_OK : PFAC_E_ARG;
}

extern "C" int pfac_build_host_chain(const char* const* patterns, const uint32_t* lengths,
                                     uint32_t num, uint32_t* chain, uint64_t cap,
                                     uint64_t* num_states, int64_t* bad_index) {
  using namespace pfac;
  if (!num_states) return PFAC_E_ARG;
  HostTable h;
  int rc = build_host_table(patterns, lengths, num, &h, bad_index);
  if (rc != PFAC_OK) return rc;
  *num_states = h.num_states;
  if (chain && h.num_states <= cap)
    memcpy(chain, h.chain.data(), h.chain.size() * sizeof(uint32_t));
  return PFAC_OK;
}

extern "C" int pfac_build_host_prefix(const char* const* patterns, const uint32_t* lengths,
                                      uint32_t num, uint32_t* words, uint64_t cap_words,
                                      uint32_t* k, uint64_t* num_keys, int64_t* bad_index) {
  using namespace pfac;
  HostTable h;
  int rc = build_host_table(patterns, lengths, num, &h, bad_index);
  if (rc != PFAC_OK) return rc;
  if (k) *k = h.pfx_k;
  if (num_keys) *num_keys = h.pfx_set;
  if (words && h.pfx.size() <= cap_words)
    memcpy(words, h.pfx.data(), h.pfx.size() * sizeof(uint32_t));
  return PFAC_OK;
}
