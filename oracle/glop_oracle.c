/*
 * CPU ORACLE for exact multi-pattern matching -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header, table or helper with the GPU
 * matcher; it is the plain definition of the result written out.
 *
 * What is computed (the result the failureless-trie walk of Section 5 reaches):
 * every start offset of the text begins an independent walk that follows the
 * text while it spells a pattern prefix, so pattern j occurs at offset i exactly
 * when the |p_j| bytes of the text starting at i equal p_j.  The paper reports
 * the number of suspicious events and where they are in the log (Section 1), so
 * the output is
 *
 *   M = { (i, j) : 0 <= i, i + |p_j| <= N, T[i .. i+|p_j|) == p_j }
 *
 * listed by ascending offset i, then ascending pattern index j, plus
 * C[j] = #{ i : (i, j) in M }.  Overlapping occurrences all count (a match
 * lets the walk run on into the following bytes, Section 5) and so does every
 * pattern ending at the same start; duplicate patterns each report their own
 * index.  Nothing spans two calls: the text is one independent string.
 *
 * Three loops give the same M:
 *   plain     -- for each i, for each j ascending: memcmp.
 *   bucketed  -- for each i, only the j whose first byte equals T[i], in
 *                ascending j (a pattern with another first byte cannot match).
 *   bucketed by two bytes -- for each i, the j of length 1 (a side list) and
 *                the j of length >= 2 whose first two bytes equal T[i], T[i+1]
 *                (when i + 1 < N), the two ascending lists merged into one
 *                ascending j; a pattern with other first two bytes cannot
 *                match, and at the last offset only a 1-byte pattern fits.
 * Work is split over threads by contiguous ranges of i; each range's pairs are
 * produced in order and the ranges are concatenated in order, so the output is
 * identical for any thread count.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    const uint8_t *text;
    uint64_t n_text;
    const uint8_t *pat_bytes;   /* all patterns back to back */
    const uint64_t *pat_off;    /* start of pattern j inside pat_bytes */
    const uint32_t *pat_len;    /* |p_j| >= 1 */
    uint32_t n_pat;
    const uint32_t *bucket_ids; /* pattern ids grouped by first byte, ascending */
    const uint64_t *bucket_at;  /* 257 entries: bucket b is bucket_ids[at[b] .. at[b+1]) */
    /* two-byte buckets: patterns of length >= 2 grouped by key p[0] * 256 + p[1],
       ascending in each bucket (65537 entries in pair_at); patterns of length 1
       in short_ids, ascending */
    const uint32_t *pair_ids;
    const uint64_t *pair_at;
    const uint32_t *short_ids;
    uint32_t n_short;
    int bucketed; /* 0 plain, 1 first byte, 2 first two bytes */
} problem_t;

typedef struct {
    const problem_t *pb;
    uint64_t lo, hi;      /* start offsets handled: [lo, hi) */
    uint64_t found;       /* pairs found in [lo, hi) */
    uint64_t *counts;     /* per-pattern counts of this range (n_pat entries) */
    /* fill pass */
    uint64_t out_base, cap;
    uint64_t *out_off;
    uint32_t *out_id;
} range_t;

static inline int occurs_at(const problem_t *pb, uint64_t i, uint32_t j) {
    uint64_t len = pb->pat_len[j];
    if (len > pb->n_text - i) return 0; /* the pattern must fit: i + |p_j| <= N */
    return memcmp(pb->text + i, pb->pat_bytes + pb->pat_off[j], (size_t)len) == 0;
}

static inline void record(range_t *r, uint64_t i, uint32_t j) {
    if (r->counts) r->counts[j] += 1;
    if (r->out_off) {
        uint64_t k = r->out_base + r->found;
        if (k < r->cap) {
            r->out_off[k] = i;
            r->out_id[k] = j;
        }
    }
    r->found += 1;
}

/* Two-byte buckets at offset i: the side list of 1-byte patterns and the
   bucket of T[i], T[i+1] (none at the last offset), merged in ascending j. */
static void scan_pairs_at(range_t *r, uint64_t i) {
    const problem_t *pb = r->pb;
    uint64_t a = 0, a_end = pb->n_short, b = 0, b_end = 0;
    if (i + 1 < pb->n_text) {
        uint32_t key = (uint32_t)pb->text[i] * 256u + pb->text[i + 1];
        b = pb->pair_at[key];
        b_end = pb->pair_at[key + 1];
    }
    while (a < a_end || b < b_end) {
        uint32_t j;
        if (b == b_end || (a < a_end && pb->short_ids[a] < pb->pair_ids[b]))
            j = pb->short_ids[a++];
        else
            j = pb->pair_ids[b++];
        if (occurs_at(pb, i, j)) record(r, i, j);
    }
}

static void *scan_range(void *arg) {
    range_t *r = (range_t *)arg;
    const problem_t *pb = r->pb;
    r->found = 0;
    for (uint64_t i = r->lo; i < r->hi; i++) {
        if (pb->bucketed == 2) {
            scan_pairs_at(r, i);
        } else if (pb->bucketed) {
            uint8_t first = pb->text[i];
            for (uint64_t k = pb->bucket_at[first]; k < pb->bucket_at[first + 1]; k++) {
                uint32_t j = pb->bucket_ids[k];
                if (occurs_at(pb, i, j)) record(r, i, j);
            }
        } else {
            for (uint32_t j = 0; j < pb->n_pat; j++)
                if (occurs_at(pb, i, j)) record(r, i, j);
        }
    }
    return NULL;
}

static void run_ranges(range_t *rs, int threads) {
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    for (int t = 1; t < threads; t++) pthread_create(&tid[t], NULL, scan_range, &rs[t]);
    scan_range(&rs[0]);
    for (int t = 1; t < threads; t++) pthread_join(tid[t], NULL);
    free(tid);
}

/*
 * Match n_pat patterns against text[0 .. n_text).
 *   bucketed:       0 plain, 1 first-byte buckets, 2 two-byte buckets (same M).
 *   out_off/out_id: room for `cap` pairs (may be NULL with cap 0); the first
 *                   min(cap, |M|) pairs of M in order are written.
 *   counts:         n_pat entries, overwritten with C (may be NULL).
 * Returns |M|, or UINT64_MAX on invalid input (an empty pattern, or a NULL
 * pointer that is needed).
 */
uint64_t oracle_match(const uint8_t *text, uint64_t n_text, const uint8_t *pat_bytes,
                      const uint64_t *pat_off, const uint32_t *pat_len, uint32_t n_pat,
                      int bucketed, int threads, uint64_t cap, uint64_t *out_off, uint32_t *out_id,
                      uint64_t *counts) {
    if ((n_text > 0 && !text) || (n_pat > 0 && (!pat_bytes || !pat_off || !pat_len)) ||
        (cap > 0 && (!out_off || !out_id)))
        return UINT64_MAX;
    for (uint32_t j = 0; j < n_pat; j++)
        if (pat_len[j] == 0) return UINT64_MAX;
    if (counts) memset(counts, 0, sizeof(uint64_t) * n_pat);
    if (n_text == 0 || n_pat == 0) return 0;
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > n_text) threads = (int)n_text;

    problem_t pb = {text, n_text, pat_bytes, pat_off, pat_len, n_pat, NULL, NULL, NULL, NULL, NULL, 0, bucketed};
    uint32_t *bucket_ids = NULL, *pair_ids = NULL, *short_ids = NULL;
    uint64_t *bucket_at = NULL, *pair_at = NULL;
    if (bucketed == 2) {
        /* counting sort by key: ids stay ascending within each bucket */
        pair_ids = (uint32_t *)malloc(sizeof(uint32_t) * n_pat);
        short_ids = (uint32_t *)malloc(sizeof(uint32_t) * n_pat);
        pair_at = (uint64_t *)calloc(65537, sizeof(uint64_t));
        uint32_t n_short = 0;
        for (uint32_t j = 0; j < n_pat; j++) {
            const uint8_t *p = pat_bytes + pat_off[j];
            if (pat_len[j] == 1)
                short_ids[n_short++] = j;
            else
                pair_at[(uint32_t)p[0] * 256u + p[1] + 1] += 1;
        }
        for (uint32_t k = 0; k < 65536; k++) pair_at[k + 1] += pair_at[k];
        uint64_t *fill = (uint64_t *)malloc(sizeof(uint64_t) * 65536);
        memcpy(fill, pair_at, sizeof(uint64_t) * 65536);
        for (uint32_t j = 0; j < n_pat; j++) {
            const uint8_t *p = pat_bytes + pat_off[j];
            if (pat_len[j] >= 2) pair_ids[fill[(uint32_t)p[0] * 256u + p[1]]++] = j;
        }
        free(fill);
        pb.pair_ids = pair_ids;
        pb.pair_at = pair_at;
        pb.short_ids = short_ids;
        pb.n_short = n_short;
    } else if (bucketed) {
        bucket_ids = (uint32_t *)malloc(sizeof(uint32_t) * n_pat);
        bucket_at = (uint64_t *)calloc(257, sizeof(uint64_t));
        for (uint32_t j = 0; j < n_pat; j++) bucket_at[pat_bytes[pat_off[j]] + 1] += 1;
        for (int b = 0; b < 256; b++) bucket_at[b + 1] += bucket_at[b];
        uint64_t fill[256];
        memcpy(fill, bucket_at, sizeof(fill));
        for (uint32_t j = 0; j < n_pat; j++) bucket_ids[fill[pat_bytes[pat_off[j]]]++] = j;
        pb.bucket_ids = bucket_ids;
        pb.bucket_at = bucket_at;
    }

    range_t *rs = (range_t *)calloc((size_t)threads, sizeof(range_t));
    uint64_t *range_counts = counts ? (uint64_t *)calloc((size_t)threads * n_pat, sizeof(uint64_t)) : NULL;
    for (int t = 0; t < threads; t++) {
        rs[t].pb = &pb;
        rs[t].lo = n_text * (uint64_t)t / (uint64_t)threads;
        rs[t].hi = n_text * (uint64_t)(t + 1) / (uint64_t)threads;
        rs[t].counts = range_counts ? range_counts + (size_t)t * n_pat : NULL;
    }
    /* Pass 1: how many pairs each range holds (and the counts). */
    run_ranges(rs, threads);
    uint64_t total = 0;
    for (int t = 0; t < threads; t++) {
        rs[t].out_base = total;
        total += rs[t].found;
    }
    if (counts)
        for (int t = 0; t < threads; t++)
            for (uint32_t j = 0; j < n_pat; j++) counts[j] += range_counts[(size_t)t * n_pat + j];
    /* Pass 2: write the pairs, each range at its place in the order. */
    if (cap > 0) {
        for (int t = 0; t < threads; t++) {
            rs[t].counts = NULL;
            rs[t].cap = cap;
            rs[t].out_off = out_off;
            rs[t].out_id = out_id;
        }
        run_ranges(rs, threads);
    }
    free(range_counts);
    free(rs);
    free(bucket_ids);
    free(bucket_at);
    free(pair_ids);
    free(pair_at);
    free(short_ids);
    return total;
}
