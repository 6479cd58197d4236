// Device-side layout of a compiled dictionary, shared by the host compiler
// (which writes it) and the kernels (which read it).
//
// Transition table (Section 6 keeps the state-transition table as an int array
// indexed by character code; here the 256 byte values are first folded into
// classes so a row holds only the bytes some pattern uses):
//   delta[s * num_classes + cls[b]] = next state | GLOP_TERM_BIT if the next
//   state ends at least one pattern, or 0 when the trie has no edge (the walk
//   ends: Section 5 drops the failure transitions).  The root is state 0 and is
//   never a target, so 0 is free to mean "no edge".  Class 0 collects the bytes
//   no pattern contains; its column is all zeros.
// States are numbered breadth-first, so the rows of the short prefixes that
// almost every walk touches are packed together at the front of the table.
//
// Output lists: term[s] = (first, count) into outids for a terminal state s;
// outids[first .. first+count) are the ids of every pattern that ends on the
// path root..s (s itself and its terminal ancestors), ascending.  A walk keeps
// only the deepest terminal it passed and emits that one list, which is already
// in id order.
//
// Filter: a blocked Bloom filter of 2^bitmap_log2 bits, read as 32-bit
// words.  For every pattern p and every t in [0, stride), the q bytes
// p[t .. t+q) (little-endian in a 32-bit word, zero above q bytes) hash to
// h = glop_qgram_hash(g); the top (bitmap_log2 - 5) bits of h pick a word and
// the next 5 bits a bit b1 in it; with two probe bits, a second bit
// b2 = b1 ^ (16 | next 4 bits) (always different from b1) is set in the same
// word.  A text position whose word lacks any of its bits cannot be where any
// pattern's t-th q-gram sits.
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define GLOP_HD __host__ __device__ __forceinline__
#else
#define GLOP_HD inline
#endif

#define GLOP_TERM_BIT 0x80000000u
#define GLOP_STATE_MASK 0x7FFFFFFFu

// Multiplicative (Fibonacci) hashing, Knuth TAOCP vol. 3, 6.4: the top bits
// of g * floor(2^32 / phi) spread consecutive and structured keys well.
GLOP_HD uint32_t glop_qgram_hash(uint32_t g) { return g * 0x9E3779B1u; }

// Right shift that leaves the word index of h (bitmap_log2 in 12..28).
GLOP_HD uint32_t glop_word_shift(uint32_t bitmap_log2) { return 37u - bitmap_log2; }

// Word index and the probe-bit mask of h (probe_bits 1 or 2).
GLOP_HD uint32_t glop_bloom_word(uint32_t h, uint32_t wsh) { return h >> wsh; }
GLOP_HD uint32_t glop_bloom_bit1(uint32_t h, uint32_t wsh) { return (h >> (wsh - 5u)) & 31u; }
GLOP_HD uint32_t glop_bloom_bit2(uint32_t h, uint32_t wsh) {
    return glop_bloom_bit1(h, wsh) ^ (16u | ((h >> (wsh - 9u)) & 15u));
}

struct GlopDevDict {
    const uint32_t *delta;   // num_states * num_classes
    const uint32_t *term;    // 2 * num_states: (first, count) per state
    const uint32_t *outids;  // output lists
    const uint32_t *bitmap;  // 2^bitmap_log2 bits
    const uint8_t *cls;      // 256 byte classes
    uint32_t num_classes;
    uint32_t num_states;
    uint32_t num_patterns;
    uint32_t min_len, max_len;
    uint32_t qgram, qmask, stride, bitmap_log2, probe_bits;
    int32_t filter;  // GLOP_FILTER_NONE or GLOP_FILTER_QGRAM
};
