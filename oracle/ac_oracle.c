/*
 * Correctness oracle for PFAC DNA matching -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this code.  The GPU library never links, calls or
 * includes it, and this file includes nothing from the GPU library.
 *
 * What it computes (the plain definition the PFAC walk reaches exactly):
 *   For a text T[0..n) and patterns p_1..p_P over {A,C,G,T} (IDs 1..P in
 *   input order, as the rows of the sample transition table in Sec. V.A,
 *   Table I, are numbered),
 *     match[i] = ID of the LONGEST pattern p_k with T[i..i+|p_k|) == p_k,
 *                the smallest such ID when several equal patterns tie,
 *                0 when no pattern starts at i.  PFAC reports only the
 *                longest pattern per start position (Sec. IV), at the
 *                position its thread starts from (Sec. IV, Fig. 3).
 *     total    = number of pairs (k, i) with T[i..i+|p_k|) == p_k, every
 *                pattern ID counted (duplicates included).
 *   Only the four upper-case bytes A, C, G and T are bases (the table has
 *   four columns, Sec. V.A); any other text byte has no transition.
 *   The same definitions over the byte alphabet (every byte value a symbol,
 *   patterns any non-empty byte strings) are computed by the *_bytes entry
 *   points: the general-purpose setting of the original PFAC library.
 *   Optionally also
 *     count[i] = number of pattern IDs k with T[i..i+|p_k|) == p_k, and
 *     the list of every such pair (i, k) -- the sub-patterns too, which PFAC
 *     itself does not report (Sec. IV names that limitation).
 *
 * How it computes it: the classic sequential Aho-Corasick machine the paper
 * summarises in Sec. III -- goto function built by inserting the keywords
 * one at a time (Sec. III, Fig. 1; Sec. V.A), failure function over all
 * goto states in breadth-first order (Sec. III, Fig. 2), output function,
 * then one left-to-right pass over the text following failure links on a
 * missing goto (Sec. III).  Each reported occurrence ending at j with
 * length l is converted to its start j-l+1 and folded into match[] with the
 * longest-wins / smaller-ID-on-tie rule.  A dictionary (output) link per
 * state -- the nearest state on the failure chain with a non-empty output
 * -- enumerates every keyword ending at j.
 *
 * Nothing here is blocked, fused or reordered for speed.  The
 * multi-threaded entry point only splits start positions into contiguous
 * chunks, runs the same scan on each chunk (extended by the longest
 * pattern length minus one so every occurrence starting in the chunk is
 * seen), and keeps occurrences whose start lies inside the chunk; the
 * result is identical to the single-threaded scan.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ORACLE_MUTANT (tests only): plants one plausible mistake so the pin tests
 * can show they catch it.  1: no dictionary links; 2: ties go to the larger
 * ID; 3: start position off by one; 4: non-bases read as 'A'; 5: shortest
 * pattern wins; 6: failure links never followed. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

#define OR_OK 0
#define OR_E_ARG -1
#define OR_E_PATTERN -2
#define OR_E_NOMEM -4

/* symbol index of a byte: A=0 C=1 G=2 T=3, -1 for every other byte */
static int sym(uint8_t b) {
  switch (b) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
  }
}

/* symbol of a pattern byte under alphabet A: DNA codes, or the byte itself */
static int pat_sym(int A, uint8_t b) { return A == 4 ? sym(b) : (int)b; }

static int text_sym(int A, uint8_t b) {
  if (A != 4) return (int)b;
#if ORACLE_MUTANT == 4
  return sym(b) < 0 ? 0 : sym(b);
#else
  return sym(b);
#endif
}

typedef struct {
  int A;               /* alphabet size: 4 (DNA: A,C,G,T) or 256 (every byte a symbol) */
  int64_t nstates;     /* states allocated so far, root = 0 */
  int64_t cap;
  int64_t *go;         /* go[A*s + a]: goto(s, a), -1 = fail */
  int64_t *fail;       /* failure function */
  int64_t *dict;       /* nearest failure-chain state with output, -1 = none */
  int64_t *out_head;   /* first keyword index (0-based) ending at s, -1 = none */
  int64_t *out_next;   /* per keyword: next keyword ending at the same state */
  uint32_t *kw_len;    /* per keyword: its length */
  uint32_t nkw;
  uint32_t max_len;
} machine;

static void machine_free(machine *m) {
  free(m->go); free(m->fail); free(m->dict); free(m->out_head);
  free(m->out_next); free(m->kw_len);
  memset(m, 0, sizeof(*m));
}

static int new_state(machine *m) {
  if (m->nstates == m->cap) {
    int64_t nc = m->cap ? 2 * m->cap : 64;
    int64_t *g = (int64_t *)realloc(m->go, (size_t)nc * m->A * sizeof(int64_t));
    if (!g) return OR_E_NOMEM;
    m->go = g;
    int64_t *h = (int64_t *)realloc(m->out_head, (size_t)nc * sizeof(int64_t));
    if (!h) return OR_E_NOMEM;
    m->out_head = h;
    m->cap = nc;
  }
  int64_t s = m->nstates++;
  for (int a = 0; a < m->A; ++a) m->go[(int64_t)m->A * s + a] = -1;
  m->out_head[s] = -1;
  return OR_OK;
}

/* Goto function and output function: insert each keyword in input order;
 * a new state is created for every character that has no transition yet
 * (Sec. III, Fig. 1 numbering; Sec. V.A insertion). */
static int build_goto(machine *m, int A, const char *const *pats, const uint32_t *lens,
                      uint32_t num, int64_t *bad_index) {
  memset(m, 0, sizeof(*m));
  m->A = A;
  m->nkw = num;
  m->out_next = (int64_t *)malloc((size_t)(num ? num : 1) * sizeof(int64_t));
  m->kw_len = (uint32_t *)malloc((size_t)(num ? num : 1) * sizeof(uint32_t));
  if (!m->out_next || !m->kw_len) return OR_E_NOMEM;
  if (new_state(m) != OR_OK) return OR_E_NOMEM;
  for (uint32_t k = 0; k < num; ++k) {
    if (lens[k] == 0) { if (bad_index) *bad_index = k; return OR_E_PATTERN; }
    for (uint32_t t = 0; t < lens[k]; ++t)
      if (pat_sym(A, (uint8_t)pats[k][t]) < 0) { if (bad_index) *bad_index = k; return OR_E_PATTERN; }
  }
  for (uint32_t k = 0; k < num; ++k) {
    int64_t s = 0;
    for (uint32_t t = 0; t < lens[k]; ++t) {
      int a = pat_sym(A, (uint8_t)pats[k][t]);
      if (m->go[(int64_t)A * s + a] < 0) {
        if (new_state(m) != OR_OK) return OR_E_NOMEM;
        m->go[(int64_t)A * s + a] = m->nstates - 1;
      }
      s = m->go[(int64_t)A * s + a];
    }
    /* append keyword k to output(s), keeping keyword order */
    m->kw_len[k] = lens[k];
    m->out_next[k] = -1;
    if (m->out_head[s] < 0) {
      m->out_head[s] = k;
    } else {
      int64_t q = m->out_head[s];
      while (m->out_next[q] >= 0) q = m->out_next[q];
      m->out_next[q] = k;
    }
    if (lens[k] > m->max_len) m->max_len = lens[k];
  }
  return OR_OK;
}

/* Failure function in breadth-first order (Sec. III, Fig. 2), plus the
 * dictionary link used to enumerate every output on the failure chain. */
static int build_failure(machine *m) {
  int64_t S = m->nstates;
  m->fail = (int64_t *)malloc((size_t)S * sizeof(int64_t));
  m->dict = (int64_t *)malloc((size_t)S * sizeof(int64_t));
  int64_t *queue = (int64_t *)malloc((size_t)S * sizeof(int64_t));
  if (!m->fail || !m->dict || !queue) { free(queue); return OR_E_NOMEM; }
  int64_t head = 0, tail = 0;
  m->fail[0] = 0;
  m->dict[0] = -1;
  const int64_t A = m->A;
  for (int a = 0; a < A; ++a) {
    int64_t u = m->go[a];
    if (u >= 0) { m->fail[u] = 0; m->dict[u] = -1; queue[tail++] = u; }
  }
  while (head < tail) {
    int64_t r = queue[head++];
    for (int a = 0; a < A; ++a) {
      int64_t u = m->go[A * r + a];
      if (u < 0) continue;
      queue[tail++] = u;
      /* f(u): longest proper suffix of u's string that is a trie state */
      int64_t v = m->fail[r];
      while (v != 0 && m->go[A * v + a] < 0) v = m->fail[v];
      int64_t w = m->go[A * v + a];
      m->fail[u] = (w >= 0 && w != u) ? w : 0;
      int64_t f = m->fail[u];
      m->dict[u] = (m->out_head[f] >= 0) ? f : m->dict[f];
    }
  }
  free(queue);
  return OR_OK;
}

/* Where the occurrences of one scan go: the longest-wins match array
 * (PFAC's report, Sec. IV), the total, and optionally the number of
 * occurrences per start position and the list of every occurrence. */
typedef struct {
  int32_t *match;
  uint32_t *bestlen;
  uint64_t total;
  uint32_t *count;     /* NULL or [n]: occurrences starting at each position */
  uint32_t *occ_pos;   /* NULL or [cap]: start of each occurrence, in scan order */
  int32_t *occ_id;     /* NULL or [cap]: its pattern ID */
  uint64_t cap, nocc;  /* room in occ_pos/occ_id; occurrences seen (may exceed cap) */
} sink;

/* Record keyword k of length l ending at text index j. */
static void record(sink *o, uint64_t lo, uint64_t hi, uint64_t j, uint32_t k, uint32_t l) {
#if ORACLE_MUTANT == 3
  uint64_t s = j - l + (l > j ? 1 : 0);
#else
  uint64_t s = j + 1 - l;
#endif
  if (s < lo || s >= hi) return;
  o->total += 1;
  int32_t id = (int32_t)k + 1;
  if (o->count) o->count[s] += 1;
  if (o->occ_pos) {
    if (o->nocc < o->cap) {
      o->occ_pos[o->nocc] = (uint32_t)s;
      o->occ_id[o->nocc] = id;
    }
    o->nocc += 1;
  }
  int32_t *match = o->match;
  uint32_t *bestlen = o->bestlen;
#if ORACLE_MUTANT == 2
  if (l > bestlen[s] || (l == bestlen[s] && id > match[s])) {
#elif ORACLE_MUTANT == 5
  if (bestlen[s] == 0 || l < bestlen[s]) {
#else
  if (l > bestlen[s] || (l == bestlen[s] && id < match[s])) {
#endif
    bestlen[s] = l;
    match[s] = id;
  }
}

/* One left-to-right pass (Sec. III) over text[lo .. min(n, hi+max_len-1)),
 * starting from the root at lo, keeping occurrences that start in [lo, hi). */
static void scan_range(const machine *m, const uint8_t *text, uint64_t n,
                       uint64_t lo, uint64_t hi, sink *o) {
  uint64_t end = hi + (m->max_len ? m->max_len - 1 : 0);
  if (end > n) end = n;
  int64_t s = 0;
  const int64_t A = m->A;
  for (uint64_t j = lo; j < end; ++j) {
    int a = text_sym(m->A, text[j]);
    if (a < 0) { s = 0; continue; }          /* no transition: restart at the root */
#if ORACLE_MUTANT == 6
    if (s != 0 && m->go[A * s + a] < 0) s = 0;
#else
    while (s != 0 && m->go[A * s + a] < 0) s = m->fail[s];
#endif
    int64_t nx = m->go[A * s + a];
    s = nx >= 0 ? nx : 0;
    int64_t t = (m->out_head[s] >= 0) ? s : m->dict[s];
    while (t >= 0) {
      for (int64_t k = m->out_head[t]; k >= 0; k = m->out_next[k])
        record(o, lo, hi, j, (uint32_t)k, m->kw_len[k]);
#if ORACLE_MUTANT == 1
      t = -1;
#else
      t = m->dict[t];
#endif
    }
  }
}

static int build_machine(machine *m, int A, const char *const *pats, const uint32_t *lens,
                         uint32_t num, int64_t *bad_index) {
  int rc = build_goto(m, A, pats, lens, num, bad_index);
  if (rc == OR_OK) rc = build_failure(m);
  if (rc != OR_OK) machine_free(m);
  return rc;
}

/* Single-threaded oracle scan. match has n entries. */
int oracle_scan(const char *const *pats, const uint32_t *lens, uint32_t num,
                const uint8_t *text, uint64_t n, int32_t *match, uint64_t *total,
                int64_t *bad_index) {
  if ((num && (!pats || !lens)) || (n && (!text || !match)) || !total) return OR_E_ARG;
  machine m;
  int rc = build_machine(&m, 4, pats, lens, num, bad_index);
  if (rc != OR_OK) return rc;
  uint32_t *bestlen = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
  if (!bestlen) { machine_free(&m); return OR_E_NOMEM; }
  memset(match, 0, n * sizeof(int32_t));
  sink o = {match, bestlen, 0, NULL, NULL, NULL, 0, 0};
  scan_range(&m, text, n, 0, n, &o);
  *total = o.total;
  free(bestlen);
  machine_free(&m);
  return OR_OK;
}

/* Every occurrence, one scan (single thread): match[] and *total as in
 * oracle_scan; count[i] (optional, n entries) = occurrences starting at i;
 * occ_pos/occ_id (optional, cap entries) = start and pattern ID of every
 * occurrence in the order the scan reports them (by end position, then
 * along the dictionary links); *num_occ = the number of occurrences, which
 * may exceed cap (only the first cap are written). */
static int occurrences_alpha(int A, const char *const *pats, const uint32_t *lens, uint32_t num,
                             const uint8_t *text, uint64_t n, int32_t *match, uint32_t *count,
                             uint32_t *occ_pos, int32_t *occ_id, uint64_t cap,
                             uint64_t *num_occ, uint64_t *total, int64_t *bad_index) {
  if ((num && (!pats || !lens)) || (n && (!text || !match)) || !total || !num_occ ||
      (cap && (!occ_pos || !occ_id)))
    return OR_E_ARG;
  machine m;
  int rc = build_machine(&m, A, pats, lens, num, bad_index);
  if (rc != OR_OK) return rc;
  uint32_t *bestlen = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
  if (!bestlen) { machine_free(&m); return OR_E_NOMEM; }
  memset(match, 0, n * sizeof(int32_t));
  if (count) memset(count, 0, n * sizeof(uint32_t));
  uint32_t dummy_pos = 0;
  int32_t dummy_id = 0;
  sink o = {match, bestlen, 0, count, cap ? occ_pos : &dummy_pos, cap ? occ_id : &dummy_id,
            cap, 0};
  scan_range(&m, text, n, 0, n, &o);
  *total = o.total;
  *num_occ = o.nocc;
  free(bestlen);
  machine_free(&m);
  return OR_OK;
}

int oracle_occurrences(const char *const *pats, const uint32_t *lens, uint32_t num,
                       const uint8_t *text, uint64_t n, int32_t *match, uint32_t *count,
                       uint32_t *occ_pos, int32_t *occ_id, uint64_t cap, uint64_t *num_occ,
                       uint64_t *total, int64_t *bad_index) {
  return occurrences_alpha(4, pats, lens, num, text, n, match, count, occ_pos, occ_id, cap,
                           num_occ, total, bad_index);
}

/* The same over the byte alphabet: every byte value (0..255) is a symbol,
 * patterns are any non-empty byte strings, no text byte stops a scan. */
int oracle_occurrences_bytes(const char *const *pats, const uint32_t *lens, uint32_t num,
                             const uint8_t *text, uint64_t n, int32_t *match, uint32_t *count,
                             uint32_t *occ_pos, int32_t *occ_id, uint64_t cap,
                             uint64_t *num_occ, uint64_t *total, int64_t *bad_index) {
  return occurrences_alpha(256, pats, lens, num, text, n, match, count, occ_pos, occ_id, cap,
                           num_occ, total, bad_index);
}

typedef struct {
  const machine *m;
  const uint8_t *text;
  uint64_t n, lo, hi;
  sink o;
} chunk_job;

static void *chunk_main(void *arg) {
  chunk_job *jb = (chunk_job *)arg;
  scan_range(jb->m, jb->text, jb->n, jb->lo, jb->hi, &jb->o);
  return NULL;
}

/* Multi-threaded oracle scan: contiguous chunks of start positions, one
 * thread each.  Identical result to oracle_scan; count (optional, n
 * entries) receives the occurrences starting at each position. */
static int scan_mt_alpha(int A, const char *const *pats, const uint32_t *lens, uint32_t num,
                         const uint8_t *text, uint64_t n, int32_t *match, uint64_t *total,
                         int64_t *bad_index, int nthreads, uint32_t *count) {
  if ((num && (!pats || !lens)) || (n && (!text || !match)) || !total || nthreads < 1)
    return OR_E_ARG;
  machine m;
  int rc = build_machine(&m, A, pats, lens, num, bad_index);
  if (rc != OR_OK) return rc;
  uint32_t *bestlen = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
  chunk_job *jobs = (chunk_job *)calloc((size_t)nthreads, sizeof(chunk_job));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!bestlen || !jobs || !th) {
    free(bestlen); free(jobs); free(th); machine_free(&m); return OR_E_NOMEM;
  }
  memset(match, 0, n * sizeof(int32_t));
  if (count) memset(count, 0, n * sizeof(uint32_t));
  uint64_t per = (n + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
  for (int t = 0; t < nthreads; ++t) {
    uint64_t lo = per * (uint64_t)t, hi = lo + per;
    if (lo > n) lo = n;
    if (hi > n) hi = n;
    jobs[t] = (chunk_job){&m, text, n, lo, hi, {match, bestlen, 0, count, NULL, NULL, 0, 0}};
    pthread_create(&th[t], NULL, chunk_main, &jobs[t]);
  }
  *total = 0;
  for (int t = 0; t < nthreads; ++t) {
    pthread_join(th[t], NULL);
    *total += jobs[t].o.total;
  }
  free(bestlen); free(jobs); free(th);
  machine_free(&m);
  return OR_OK;
}

int oracle_scan_mt(const char *const *pats, const uint32_t *lens, uint32_t num,
                   const uint8_t *text, uint64_t n, int32_t *match, uint64_t *total,
                   int64_t *bad_index, int nthreads, uint32_t *count) {
  return scan_mt_alpha(4, pats, lens, num, text, n, match, total, bad_index, nthreads, count);
}

/* The chunked scan over the byte alphabet (see oracle_occurrences_bytes). */
int oracle_scan_bytes_mt(const char *const *pats, const uint32_t *lens, uint32_t num,
                         const uint8_t *text, uint64_t n, int32_t *match, uint64_t *total,
                         int64_t *bad_index, int nthreads, uint32_t *count) {
  return scan_mt_alpha(256, pats, lens, num, text, n, match, total, bad_index, nthreads, count);
}

/* Expose the insertion-order goto function, before any renumbering, so
 * tests can compare it with the state numbering of Sec. III, Fig. 1 and the
 * edges of Sec. V.A, Table I.  go_out gets 4*cap entries (A,C,G,T order,
 * -1 = fail), final_out gets cap entries (smallest keyword ID ending at the
 * state, 0 = none).  Returns the state count, or a negative error. */
int64_t oracle_goto(const char *const *pats, const uint32_t *lens, uint32_t num,
                    int64_t *go_out, int32_t *final_out, int64_t cap) {
  machine m;
  int64_t bad = -1;
  int rc = build_goto(&m, 4, pats, lens, num, &bad);
  if (rc != OR_OK) { machine_free(&m); return rc; }
  int64_t S = m.nstates;
  if (S <= cap) {
    memcpy(go_out, m.go, (size_t)S * 4 * sizeof(int64_t));
    for (int64_t s = 0; s < S; ++s)
      final_out[s] = m.out_head[s] >= 0 ? (int32_t)m.out_head[s] + 1 : 0;
  }
  machine_free(&m);
  return S;
}
