/*
 * Seeded synthetic inputs for the log matcher: raw pseudo-random streams and
 * the fill of synthetic log text.  Nothing in this file knows about patterns,
 * tries or matching; it only produces bytes.  Both the CPU oracle's tests and
 * the GPU path's tests/bench draw their inputs from here.
 *
 * Generator: MT19937-64 (Matsumoto & Nishimura, "Mersenne Twister: a
 * 623-dimensionally equidistributed uniform pseudo-random number generator",
 * ACM TOMACS 1998; 64-bit variant by Nishimura 2000), the generator family the
 * paper uses for its synthetic logs (Section 6).  Each (seed, stream, block)
 * triple selects an independent MT state whose seed is derived with SplitMix64
 * (Steele, Lea & Flood, OOPSLA 2014), so text blocks can be filled by any
 * number of threads with identical output.
 *
 * Uniform integers in [lo, hi] use the top 32 bits of a draw scaled by the
 * range (multiply-shift); the bias is below range / 2^32.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MT_NN 312
#define MT_MM 156
#define MT_UPPER 0xFFFFFFFF80000000ULL
#define MT_LOWER 0x000000007FFFFFFFULL

typedef struct {
    uint64_t mt[MT_NN];
    int idx;
} mt64_t;

static void mt64_seed(mt64_t *s, uint64_t seed) {
    s->mt[0] = seed;
    for (int i = 1; i < MT_NN; i++)
        s->mt[i] = 6364136223846793005ULL * (s->mt[i - 1] ^ (s->mt[i - 1] >> 62)) + (uint64_t)i;
    s->idx = MT_NN;
}

static void mt64_twist(mt64_t *s) {
    const uint64_t matrix_a = 0xB5026F5AA96619E9ULL;
    for (int i = 0; i < MT_NN; i++) {
        uint64_t y = (s->mt[i] & MT_UPPER) | (s->mt[(i + 1) % MT_NN] & MT_LOWER);
        uint64_t v = s->mt[(i + MT_MM) % MT_NN] ^ (y >> 1);
        if (y & 1ULL) v ^= matrix_a;
        s->mt[i] = v;
    }
    s->idx = 0;
}

static inline uint64_t mt64_next(mt64_t *s) {
    if (s->idx >= MT_NN) mt64_twist(s);
    uint64_t x = s->mt[s->idx++];
    x ^= (x >> 29) & 0x5555555555555555ULL;
    x ^= (x << 17) & 0x71D67FFFEDA60000ULL;
    x ^= (x << 37) & 0xFFF7EEE000000000ULL;
    x ^= (x >> 43);
    return x;
}

static inline uint64_t splitmix64_next(uint64_t *state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Seed of the MT state for (seed, stream, block). */
uint64_t synth_substream_seed(uint64_t seed, uint64_t stream, uint64_t block) {
    uint64_t st = seed;
    uint64_t a = splitmix64_next(&st);
    st = a ^ stream;
    uint64_t b = splitmix64_next(&st);
    st = b ^ block;
    return splitmix64_next(&st);
}

/* Raw MT19937-64 output of an explicitly seeded state (used to pin the
 * implementation against the published reference values). */
void synth_mt64_raw(uint64_t mt_seed, uint64_t count, uint64_t *out) {
    mt64_t s;
    mt64_seed(&s, mt_seed);
    for (uint64_t i = 0; i < count; i++) out[i] = mt64_next(&s);
}

/* The first `count` raw outputs of substream (seed, stream, block 0). */
void synth_stream(uint64_t seed, uint64_t stream, uint64_t count, uint64_t *out) {
    synth_mt64_raw(synth_substream_seed(seed, stream, 0), count, out);
}

/* Text shape: lines of content length U{line_min..line_max} followed by '\n';
 * content is words of U{word_min..word_max} bytes drawn from
 * U{byte_lo..byte_hi}, separated by single spaces (0x20).  A word that would
 * run past the end of its line is cut there. */
typedef struct {
    uint32_t line_min, line_max;
    uint32_t word_min, word_max;
    uint32_t byte_lo, byte_hi;
    uint64_t block_bytes; /* independent substream per block; lines restart at each block */
} synth_text_cfg;

typedef struct {
    mt64_t g;
    uint64_t pending;
    int have;
} draw32_t;

static inline uint32_t draw_u32(draw32_t *d) {
    if (d->have) {
        d->have = 0;
        return (uint32_t)d->pending;
    }
    uint64_t x = mt64_next(&d->g);
    d->pending = x;
    d->have = 1;
    return (uint32_t)(x >> 32);
}

static inline uint32_t draw_range(draw32_t *d, uint32_t lo, uint32_t hi) {
    uint64_t span = (uint64_t)hi - lo + 1;
    return lo + (uint32_t)(((uint64_t)draw_u32(d) * span) >> 32);
}

static void fill_block(uint64_t seed, uint64_t stream, uint64_t block, uint8_t *out, uint64_t n,
                       const synth_text_cfg *c) {
    draw32_t d;
    mt64_seed(&d.g, synth_substream_seed(seed, stream, block));
    d.have = 0;
    uint64_t pos = 0;
    while (pos < n) {
        uint64_t line = draw_range(&d, c->line_min, c->line_max);
        if (pos + line + 1 > n) line = n - pos - 1; /* last line of the block ends exactly at n */
        uint64_t end = pos + line;
        while (pos < end) {
            uint64_t w = draw_range(&d, c->word_min, c->word_max);
            if (w > end - pos) w = end - pos;
            for (uint64_t k = 0; k < w; k++) out[pos++] = (uint8_t)draw_range(&d, c->byte_lo, c->byte_hi);
            if (pos < end) out[pos++] = 0x20;
        }
        out[pos++] = 0x0A;
    }
}

typedef struct {
    uint64_t seed, stream;
    uint8_t *out;
    uint64_t n;
    const synth_text_cfg *cfg;
    uint64_t first_block, end_block;
} text_job_t;

static void *text_worker(void *arg) {
    text_job_t *j = (text_job_t *)arg;
    uint64_t bs = j->cfg->block_bytes;
    for (uint64_t b = j->first_block; b < j->end_block; b++) {
        uint64_t lo = b * bs;
        uint64_t hi = lo + bs < j->n ? lo + bs : j->n;
        fill_block(j->seed, j->stream, b, j->out + lo, hi - lo, j->cfg);
    }
    return NULL;
}

/* Fill out[0..n) with synthetic log text.  Output is independent of `threads`.
 * Returns 0, or -1 on invalid configuration. */
int synth_text(uint64_t seed, uint64_t stream, uint8_t *out, uint64_t n, const synth_text_cfg *cfg,
               int threads) {
    if (!cfg || cfg->block_bytes == 0 || cfg->line_min > cfg->line_max || cfg->word_min == 0 ||
        cfg->word_min > cfg->word_max || cfg->byte_lo > cfg->byte_hi || cfg->byte_hi > 255)
        return -1;
    if (n == 0) return 0;
    uint64_t nblocks = (n + cfg->block_bytes - 1) / cfg->block_bytes;
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > nblocks) threads = (int)nblocks;
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    text_job_t *jobs = (text_job_t *)calloc((size_t)threads, sizeof(text_job_t));
    if (!tid || !jobs) {
        free(tid);
        free(jobs);
        return -1;
    }
    for (int t = 0; t < threads; t++) {
        jobs[t].seed = seed;
        jobs[t].stream = stream;
        jobs[t].out = out;
        jobs[t].n = n;
        jobs[t].cfg = cfg;
        jobs[t].first_block = nblocks * (uint64_t)t / (uint64_t)threads;
        jobs[t].end_block = nblocks * (uint64_t)(t + 1) / (uint64_t)threads;
    }
    for (int t = 1; t < threads; t++) pthread_create(&tid[t], NULL, text_worker, &jobs[t]);
    text_worker(&jobs[0]);
    for (int t = 1; t < threads; t++) pthread_join(tid[t], NULL);
    free(tid);
    free(jobs);
    return 0;
}
