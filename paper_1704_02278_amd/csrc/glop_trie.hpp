// Host-side compiler of the failureless trie and its device tables.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "glop.h"

namespace glop {

// Text per CU up to which the stride-1 blocked filter runs 4 KiB tiles by
// default: five 8 KiB tiles per wave slot (16 per CU).  Below it the halved
// tile gives short texts twice the waves (a 1 MiB text 0.0206 -> 0.0174 ms,
// 128 MiB 0.0842 -> 0.0821 ms); above it the longer tile keeps each lane's
// loads in flight (256 MiB: 0.1259 vs 0.1314 ms, 4 GiB: 1.40 vs 1.63 ms).
constexpr uint64_t kShortTextPerCu = 640ull << 10;
// The same for a batch's byte bound, lower: a batch pays an item end per work
// item, so halved tiles only pay on small ones (batches of 2-4 texts, 7 MB:
// 3-5 % faster; 108 MB: 2 % slower).
constexpr uint64_t kShortBatchPerCu = 64ull << 10;

struct Compiled {
    uint32_t num_patterns = 0;
    uint32_t min_len = 0, max_len = 0;
    uint32_t num_classes = 1;
    uint8_t cls[256] = {};
    uint32_t num_states = 1;
    std::vector<uint32_t> delta;   // num_states * num_classes
    std::vector<uint32_t> term;    // 2 * num_states
    std::vector<uint32_t> outids;  // output lists
    int32_t filter = GLOP_FILTER_NONE;
    uint32_t qgram = 0, qmask = 0, stride = 1, bitmap_log2 = 12, probe_bits = 1, tile_kib = 8;
    // Automatic tile for short texts (0 = none): calls over at most
    // kShortTextPerCu bytes of text per CU run tile_kib_short KiB tiles.
    uint32_t tile_kib_short = 0;
    bool tile_auto = true;  // tile_kib was not given
    uint64_t filter_keys = 0;
    std::vector<uint32_t> bitmap;  // 2^bitmap_log2 bits
    std::vector<uint32_t> bitmap2; // second filter, 2^GLOP_FILTER2_LOG2 bits, or empty
    // Truncated trie (prefix_len > 0): the trie holds each pattern's first
    // prefix_len bytes; unless `candidates`, the rest is verified per match.
    uint32_t prefix_len = 0, candidates = 0;
    std::vector<uint8_t> pat_bytes;   // verification copy of the patterns, back to back
    std::vector<uint64_t> pat_off;
    std::vector<uint32_t> pat_len;
    // Exact table of the D-byte prefixes (empty when some pattern is shorter
    // than 4 bytes; layout in glop_layout.hpp).
    std::vector<uint32_t> pt;  // 2^pt_lg slots of 4 words
    uint32_t pt_lg = 0, pt_probes = 0, pt_keys = 0, pt_depth = 0, pt_leaf = 0;
    // Device layout of the transition table (glop_layout.hpp).  `delta` above
    // always holds every row (the host walk and the prefix table use it); the
    // device gets rows [0, n_dense) and, with the hybrid layout, one node per
    // state from n_dense on and the edge byte of each of those states.
    uint32_t layout = GLOP_LAYOUT_DENSE;
    uint32_t placement = GLOP_PLACE_AUTO;  // as requested; resolved at upload
    uint32_t n_dense = 1;
    std::vector<uint64_t> nodes;    // hybrid: num_states - n_dense
    std::vector<uint16_t> in_edge;  // hybrid: num_states - n_dense
    bool verifies() const { return prefix_len && !candidates; }
    // KiB per tile for one call over len bytes of text on num_cus CUs.
    uint32_t call_tile_kib(uint64_t len, int num_cus) const {
        const uint64_t cus = num_cus > 0 ? (uint64_t)num_cus : 1;
        return tile_kib_short && len <= kShortTextPerCu * cus ? tile_kib_short : tile_kib;
    }
    // KiB per tile for a batch of at most max_total_bytes: a given tile_kib,
    // else 4 KiB for a short batch (kShortBatchPerCu) where the filter has
    // 4 KiB kernels and 8 KiB for a long one (4 KiB tiles halve the text of
    // each work item, and every item end stops its workgroup's stream: 16 %
    // slower on 7.7 GiB).
    uint32_t batch_tile_kib(uint64_t max_total_bytes, int num_cus) const {
        if (!tile_auto) return tile_kib;
        const uint64_t cus = num_cus > 0 ? (uint64_t)num_cus : 1;
        const bool has4 = tile_kib == 4 || tile_kib_short == 4;
        return has4 && max_total_bytes <= kShortBatchPerCu * cus ? 4u : 8u;
    }
    // The next state (with GLOP_TERM_BIT) or 0, read from the device layout.
    uint32_t step(uint32_t s, uint32_t k) const;
    uint64_t device_table_bytes() const {
        return (uint64_t)n_dense * num_classes * 4 + nodes.size() * 8 + in_edge.size() * 2;
    }
};

// Returns GLOP_OK or an error code with `err` set.
int compile(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n,
            const glop_build_opts *opts, Compiled &out, std::string &err);

// The filter stage of compile() alone: from c.min_len and the options, set
// c's filter fields (filter, qgram, qmask, stride, bitmap_log2, probe_bits,
// tile_kib, filter_keys, bitmap).  The trie fields of c are left as they are.
int build_filter(const uint8_t *const *patterns, uint32_t n, const glop_build_opts &o, Compiled &c,
                 std::string &err);

// CPU failureless-trie walk over a compiled dictionary (timing baseline).
int cpu_walk(const Compiled &c, const uint8_t *text, uint64_t len, glop_match_t *out,
             uint64_t max_matches, uint64_t *counts, uint64_t *total, int threads);

}  // namespace glop
