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
// Hybrid layout (GLOP_LAYOUT_HYBRID): only the rows of states below n_dense
// (those of depth <= 2, a prefix of the breadth-first numbering) are dense.
// Breadth-first numbering gives the children of a state consecutive ids in
// class order, so a deeper state s is described by one 64-bit node,
// nodes[s - n_dense]:
//   bits 0..31  first child's id (children: first .. first + count - 1)
//   bits 32..39 number of children
//   bits 40..47 the class of the edge to the only child (count == 1)
//   bit  48     the only child is terminal (count == 1)
// and, for every state c >= n_dense, in_edge[c - n_dense] = the class of the
// edge into c | (c is terminal) << 8, which a state with several children
// scans.  Every child of a state at or past n_dense is itself past n_dense.
#define GLOP_NODE_COUNT_SHIFT 32u
#define GLOP_NODE_CLASS_SHIFT 40u
#define GLOP_NODE_TERM_SHIFT 48u
//
// Filter: a Bloom filter of 2^bitmap_log2 bits.  For every pattern p and
// every t in [0, stride), the q bytes p[t .. t+q) (little-endian in a 32-bit
// word g, zero above q bytes) set bit glop_slot1(g) and, with two probe bits,
// also bit glop_slot2(g).  A text position whose q-gram misses any of its bits
// cannot be where any pattern's t-th q-gram sits.
//
// Second filter (stride 1, when the first filter probes one bit or a blocked
// pair, both from glop_hash1): the same keys in a Bloom filter of
// 2^GLOP_FILTER2_LOG2 bits, five bits per key from glop_hash2, an independent
// hash: the top bits of h = glop_hash2(g), of k = glop_f2_mix(h), of h + k,
// h + 2k and h + 3k (double hashing).  It is checked only for the
// offsets the first filter lets through, before they are walked: at stride 1
// most walks start at the first filter's false positives, and the walks, not
// the probes, are most of the time.  (On 20,000 4-byte prefixes in log text,
// one bit per key passed 0.099 % of all offsets, three bits 0.044 %; 0.026 %
// start a pattern's first four bytes.  With 15,699 keys, five bits leave the
// filter 45 % full and pass about 1.9 % of the keys not in it, against 2.75 %
// with three bits; six, the best for this size, would pass 1.8 %.)
#define GLOP_FILTER2_LOG2 17u
//
// Prefix table: when every pattern (as the trie holds it) is at least D bytes
// long, D = 8 if it can be and 4 otherwise (none below 4), an exact hash table
// maps each distinct D-byte pattern prefix (little-endian 64-bit key, zero
// above D bytes) to the delta entry of the depth-D state it reaches (state |
// GLOP_TERM_BIT if it ends a pattern).  No pattern ends above depth D, so a
// walk may begin with one lookup there instead of D dependent table steps, and
// a start whose first D bytes begin no pattern ends at that lookup; when the
// trie is cut at depth D (pt_leaf) the lookup is the whole walk.  The scan
// kernel uses the table when it fits in LDS.  The table has 2^pt_lg slots of
// four words (key low, key high, entry, 0) with entry 0 marking an empty slot;
// a key's home slot is glop_pt_slot(key), a key whose home is taken sits in
// the next free slot (linear probing), and no key sits more than pt_probes
// slots past its home.
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

// Two hashes of a q-gram, each a 24x24-bit multiply-add (one full-rate
// v_mad_u32_u24 on CDNA): the product mixes the low three bytes upwards and the
// added key brings the fourth byte into the top bits that pick the slot.  The
// second hash first rotates the key by one byte.  Slots are the top
// bitmap_log2 bits.  The multipliers are 24-bit truncations of well-mixed odd
// constants: the golden ratio times 2^24 (0x9E3779) and MurmurHash3's 32-bit
// finaliser multipliers 0x85EBCA6B and 0xC2B2AE35.
GLOP_HD uint32_t glop_hash1(uint32_t g) { return (g & 0xFFFFFFu) * 0x9E3779u + g; }
GLOP_HD uint32_t glop_hash2(uint32_t g) {
    const uint32_t r = (g >> 8) | (g << 24);
    return (r & 0xFFFFFFu) * 0x85EBCAu + r;
}
GLOP_HD uint32_t glop_slot1(uint32_t g, uint32_t bitmap_log2) { return glop_hash1(g) >> (32u - bitmap_log2); }
GLOP_HD uint32_t glop_slot2(uint32_t g, uint32_t bitmap_log2) { return glop_hash2(g) >> (32u - bitmap_log2); }
// The second filter's second hash: one more 24x24-bit multiply-add, of h's
// upper 24 bits, so its top bits depend on the bits below the first slot too.
GLOP_HD uint32_t glop_f2_mix(uint32_t h) { return ((h >> 8) & 0xFFFFFFu) * 0xC2B2AEu + h; }

// Blocked variant (probe_bits 3): both bits of a q-gram lie in one 32-bit word,
// so a probe is one hash and one LDS read.  The word comes from the top
// bitmap_log2 - 5 bits of glop_hash1 (which mixes every byte of the key); the
// two bit positions are the low five bits of the key's first and second bytes
// (0 for the second when q = 1).  A shift takes its amount modulo 32, so the
// kernels test those bits by shifting the word by the key itself and by the
// key one byte on, with no instruction to extract the positions.  (On 15,699
// 4-byte keys in log text this passes 0.667 % of offsets against 0.681 % for
// positions taken from hash bits 8..17.)
GLOP_HD uint32_t glop_block_word(uint32_t h, uint32_t bitmap_log2) { return h >> (37u - bitmap_log2); }
GLOP_HD uint32_t glop_block_bits(uint32_t g) { return (1u << (g & 31u)) | (1u << ((g >> 8) & 31u)); }

// Paired variant (probe_bits 4; stride 1, 4-byte q-grams, a 2^19-bit filter):
// 16-bit blocks, the block of key g chosen by a 16-bit hash of its two
// halves (bits 1..15 of glop_hash16(g) are the block index, so the block's
// byte address in LDS is glop_hash16(g) & 0xFFFE), its two bits by the low
// four bits of the key's first and second bytes.  Everything about a probe
// then fits in 16 bits, so the kernel probes two offsets u and u + 2 with
// one instruction per step on packed 16-bit halves: the keys at u and u + 2
// overlap by two bytes, so the halves their hashes need are exactly the
// 32-bit words at u and u + 2 of the text.  (On 15,699 4-byte keys in log
// text this filter passes 1.0 % of offsets, against 0.667 % for 32-bit
// blocks; its scan issues 13 % fewer vector instructions per tile than the
// blocked one on the large workload but measured 3 % slower, so it is an
// option the autotuner tries, not the default.)
#define GLOP_HASH16_A 0xC2B3u
#define GLOP_HASH16_B 0xAE35u
GLOP_HD uint32_t glop_hash16(uint32_t g) {
    return ((g & 0xFFFFu) * GLOP_HASH16_A + (g >> 16) * GLOP_HASH16_B) & 0xFFFFu;
}
GLOP_HD uint32_t glop_pair_bits(uint32_t g) { return (1u << (g & 15u)) | (1u << ((g >> 8) & 15u)); }

// Home slot of a prefix-table key: the high word folded into the low one,
// then Knuth's multiplicative hash (the golden ratio times 2^32), top pt_lg
// bits.
GLOP_HD uint32_t glop_pt_slot(uint32_t lo, uint32_t hi, uint32_t pt_lg) {
    return ((lo ^ (hi * 0x85EBCA6Bu)) * 0x9E3779B1u) >> (32u - pt_lg);
}

// One step of the walk below the dense rows (hybrid layout): the next state
// with GLOP_TERM_BIT, or 0 when state s has no edge of class k.
GLOP_HD uint32_t glop_node_step(const uint64_t *nodes, const uint16_t *in_edge, uint32_t n_dense, uint32_t s,
                                uint32_t k) {
    const uint64_t node = nodes[s - n_dense];
    const uint32_t first = (uint32_t)node, count = (uint32_t)(node >> GLOP_NODE_COUNT_SHIFT) & 0xFFu;
    if (count == 1u) {
        if (((uint32_t)(node >> GLOP_NODE_CLASS_SHIFT) & 0xFFu) != k) return 0u;
        return first | ((uint32_t)(node >> GLOP_NODE_TERM_SHIFT) & 1u) * GLOP_TERM_BIT;
    }
    for (uint32_t j = 0; j < count; ++j) {
        const uint32_t e = in_edge[first + j - n_dense];
        if ((e & 0xFFu) == k) return (first + j) | ((e >> 8) & 1u) * GLOP_TERM_BIT;
    }
    return 0u;
}

struct GlopDevDict {
    const uint32_t *delta;   // n_dense * num_classes (every row with the dense layout)
    const uint32_t *term;    // 2 * num_states: (first, count) per state
    const uint32_t *outids;  // output lists
    const uint32_t *bitmap;  // 2^bitmap_log2 bits
    const uint8_t *cls;      // 256 byte classes
    uint32_t num_classes;
    uint32_t num_states;
    uint32_t num_patterns;
    uint32_t min_len, max_len;
    uint32_t qgram, qmask, stride, bitmap_log2, probe_bits, tile_kib;
    int32_t filter;  // GLOP_FILTER_NONE or GLOP_FILTER_QGRAM
    // Truncated trie with verification: a terminal's listed pattern j is a
    // match only if bytes [verify_from, len_j) of the text also equal it.
    uint32_t verify_from;      // 0 = every listed pattern matches (no verify stage)
    const uint8_t *pat_bytes;  // all patterns back to back
    const uint64_t *pat_off;   // first byte of pattern j in pat_bytes
    const uint32_t *pat_len;   // length of pattern j
    const uint32_t *bitmap2;   // second filter, 2^GLOP_FILTER2_LOG2 bits (null: none)
    // Prefix table (null when some pattern is shorter than 4 bytes).
    const uint32_t *pt;        // 2^pt_lg slots of (key low, key high, entry, 0)
    uint32_t pt_lg, pt_probes;
    uint32_t pt_depth;         // D: 4 or 8
    uint32_t pt_leaf;          // 1 if the trie ends at depth D (the lookup is the walk)
    // Transition table layout (see above): states below n_dense have dense
    // rows; with the hybrid layout the others have nodes.
    uint32_t n_dense;
    const uint64_t *nodes;     // null with the dense layout
    const uint16_t *in_edge;
    uint32_t table_lds;        // 1: the scan kernel stages the dense rows in LDS
};
