// Host-side compiler of the failureless trie (Section 4's first phase, with the
// failure transitions of Section 5 removed) and the CPU walk over it.
#include "glop_trie.hpp"

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <thread>

#include "glop_layout.hpp"

namespace glop {

namespace {

constexpr uint64_t kMaxTableBytes = 16ull << 30;  // dense table ceiling (host rows)
constexpr uint64_t kAutoHybridBytes = 32ull << 20; // automatic layout: hybrid above this dense size
constexpr uint32_t kDenseDepth = 2;                // hybrid: dense rows for depth <= 2
constexpr uint32_t kNone = 0xFFFFFFFFu;

uint32_t ceil_log2(uint64_t v) {
    uint32_t k = 0;
    while ((1ull << k) < v) ++k;
    return k;
}

// The exact table of the patterns' D-byte prefixes (layout in
// glop_layout.hpp), from the finished transition table: every path of D edges
// from the root spells one prefix.  Byte classes are one per pattern byte, so
// a class path names its bytes.
void build_prefix_table(Compiled &c, uint32_t D) {
    const uint32_t C = c.num_classes;
    uint8_t byte_of[256] = {};
    for (int b = 0; b < 256; ++b)
        if (c.cls[b]) byte_of[c.cls[b]] = (uint8_t)b;
    struct Node {
        uint32_t state, depth;
        uint64_t key;
    };
    std::vector<Node> todo{{0u, 0u, 0ull}};
    std::vector<std::pair<uint64_t, uint32_t>> keys;  // (key, entry)
    while (!todo.empty()) {
        const Node f = todo.back();
        todo.pop_back();
        for (uint32_t k = 1; k < C; ++k) {
            const uint32_t e = c.delta[(uint64_t)f.state * C + k];
            if (!e) continue;
            const uint64_t key = f.key | ((uint64_t)byte_of[k] << (8 * f.depth));
            if (f.depth + 1 == D)
                keys.emplace_back(key, e);
            else
                todo.push_back({e & GLOP_STATE_MASK, f.depth + 1, key});
        }
    }
    const uint32_t lg = std::max<uint32_t>(6, ceil_log2(2ull * keys.size()));  // at most half full
    const uint32_t mask = (1u << lg) - 1u;
    c.pt.assign(4ull << lg, 0u);
    uint32_t far = 0;
    for (const auto &kv : keys) {
        const uint32_t lo = (uint32_t)kv.first, hi = (uint32_t)(kv.first >> 32);
        const uint32_t home = glop_pt_slot(lo, hi, lg);
        uint32_t d = 0;
        while (c.pt[4 * ((home + d) & mask) + 2] != 0) ++d;
        uint32_t *slot = &c.pt[4 * ((home + d) & mask)];
        slot[0] = lo;
        slot[1] = hi;
        slot[2] = kv.second;
        far = std::max(far, d);
    }
    c.pt_lg = lg;
    c.pt_probes = far;
    c.pt_keys = (uint32_t)keys.size();
    c.pt_depth = D;
    // Cut at depth D: no state below it, so the lookup ends every walk.
    c.pt_leaf = c.prefix_len == D ? 1u : 0u;
}

uint32_t load_qgram(const uint8_t *p, uint32_t q) {
    uint32_t g = 0;
    for (uint32_t k = 0; k < q; ++k) g |= (uint32_t)p[k] << (8 * k);
    return g;
}

// Automatic truncation: 8 bytes when some pattern is longer (so truncation
// shortens walks) and at most 16 patterns share one 8-byte prefix (so each
// candidate verifies a short list); 0 (whole patterns) otherwise.  Lengths
// are checked by the caller; invalid input just yields 0 here.
uint32_t auto_prefix_len(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n) {
    constexpr uint32_t kLen = 8, kMaxShare = 16;
    uint32_t longest = 0;
    for (uint32_t j = 0; j < n; ++j) {
        if (!patterns[j] || lengths[j] == 0 || lengths[j] > GLOP_MAX_PATTERN_LEN) return 0;
        longest = std::max(longest, lengths[j]);
    }
    if (longest <= kLen) return 0;
    std::vector<std::string> heads(n);
    for (uint32_t j = 0; j < n; ++j)
        heads[j].assign(reinterpret_cast<const char *>(patterns[j]), std::min(kLen, lengths[j]));
    std::sort(heads.begin(), heads.end());
    uint32_t run = 1;
    for (uint32_t j = 1; j < n; ++j) {
        run = heads[j] == heads[j - 1] ? run + 1 : 1;
        if (run > kMaxShare) return 0;
    }
    return kLen;
}

// Hybrid layout (glop_layout.hpp): dense rows for the states of depth <=
// kDenseDepth, a node per deeper state.  Breadth-first numbering makes those
// states a prefix of the ids and every state's children consecutive.
int build_hybrid(Compiled &c, std::string &err) {
    const uint64_t S = c.num_states;
    const uint32_t C = c.num_classes;
    std::vector<uint8_t> depth(S, 0);
    uint64_t n_dense = S;
    for (uint64_t s = 0; s < S; ++s) {
        if (depth[s] > kDenseDepth && n_dense == S) n_dense = s;
        for (uint32_t k = 1; k < C; ++k) {
            const uint32_t e = c.delta[s * C + k];
            if (e) depth[e & GLOP_STATE_MASK] = (uint8_t)std::min<uint32_t>(depth[s] + 1u, 255u);
        }
    }
    c.n_dense = (uint32_t)n_dense;
    c.nodes.assign(S - n_dense, 0ull);
    c.in_edge.assign(S - n_dense, 0u);
    for (uint64_t s = 0; s < S; ++s) {
        uint32_t first = 0, count = 0, k1 = 0, e1 = 0;
        for (uint32_t k = 1; k < C; ++k) {
            const uint32_t e = c.delta[s * C + k];
            if (!e) continue;
            const uint32_t ch = e & GLOP_STATE_MASK;
            if (count == 0) {
                first = ch;
                k1 = k;
                e1 = e;
            } else if (ch != first + count) {
                err = "internal: children are not numbered consecutively";
                return GLOP_EINTERNAL;
            }
            ++count;
            if (ch >= n_dense) c.in_edge[ch - n_dense] = (uint16_t)(k | ((e & GLOP_TERM_BIT) ? 0x100u : 0u));
            else if (s >= n_dense) {
                err = "internal: a dense state below a node";
                return GLOP_EINTERNAL;
            }
        }
        if (s < n_dense) continue;
        uint64_t node = (uint64_t)first | ((uint64_t)count << GLOP_NODE_COUNT_SHIFT);
        if (count == 1)
            node |= ((uint64_t)k1 << GLOP_NODE_CLASS_SHIFT) |
                    ((uint64_t)((e1 & GLOP_TERM_BIT) ? 1u : 0u) << GLOP_NODE_TERM_SHIFT);
        c.nodes[s - n_dense] = node;
    }
    return GLOP_OK;
}

}  // namespace

uint32_t Compiled::step(uint32_t s, uint32_t k) const {
    if (s < n_dense) return delta[(uint64_t)s * num_classes + k];
    return glop_node_step(nodes.data(), in_edge.data(), n_dense, s, k);
}

// Filter stage: q-gram bitmap parameters and keys (Sections 2 and 5 filter
// candidates by a short prefix before the full comparison).  Reads
// c.min_len; sets the filter fields of c.  Patterns are not validated here.
int build_filter(const uint8_t *const *patterns, uint32_t n, const glop_build_opts &o, Compiled &c,
                 std::string &err) {
    if (o.filter != GLOP_FILTER_AUTO && o.filter != GLOP_FILTER_NONE && o.filter != GLOP_FILTER_QGRAM) {
        err = "filter must be GLOP_FILTER_AUTO, GLOP_FILTER_NONE or GLOP_FILTER_QGRAM";
        return GLOP_EINVAL;
    }
    try {
        int32_t filter = o.filter == GLOP_FILTER_AUTO ? (n ? GLOP_FILTER_QGRAM : GLOP_FILTER_NONE) : o.filter;
        if (n == 0) filter = GLOP_FILTER_NONE;
        c.filter = filter;
        if (filter == GLOP_FILTER_QGRAM) {
            uint32_t q = o.qgram ? o.qgram : std::min<uint32_t>(4, c.min_len);
            if (q < 1 || q > 4 || q > c.min_len) {
                err = "qgram must be 1..4 and at most the shortest pattern length";
                return GLOP_EINVAL;
            }
            uint32_t stride = o.stride ? o.stride : (c.min_len >= q + 3 ? 4u : 1u);
            if (stride != 1 && stride != 4) {
                err = "stride must be 1 or 4";
                return GLOP_EINVAL;
            }
            if (stride == 4 && c.min_len < q + 3) {
                err = "stride 4 needs every pattern to be at least qgram + 3 bytes";
                return GLOP_EINVAL;
            }
            std::vector<uint32_t> keys;
            keys.reserve((size_t)n * stride);
            for (uint32_t j = 0; j < n; ++j)
                for (uint32_t t = 0; t < stride; ++t) keys.push_back(load_qgram(patterns[j] + t, q));
            std::sort(keys.begin(), keys.end());
            keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
            uint32_t lg = o.bitmap_log2;
            if (lg == 0) lg = std::min<uint32_t>(19, std::max<uint32_t>(12, ceil_log2(keys.size()) + 8));
            if (lg < 12 || lg > 19) {
                err = "bitmap_log2 must be 12..19";
                return GLOP_EINVAL;
            }
            // Automatic probe: at stride 1 every offset is probed and the LDS
            // reads dominate, so one read per probe (blocked, 3) wins despite
            // its higher false-positive rate; at stride 4 walks dominate and
            // two independent bits (2) win.
            // The paired 16-bit-block probe (4) is an option only: it issues
            // 13 % fewer vector instructions per tile on the large workload
            // but ran 3 % slower there (its shorter dependency chains leave
            // the LDS latency exposed; the blocked probe's work hides it).
            uint32_t k = o.probe_bits ? o.probe_bits : (stride == 1 ? 3u : 2u);
            if (k < 1 || k > 4) {
                err = "probe_bits must be 1, 2, 3 or 4";
                return GLOP_EINVAL;
            }
            if (k == 4 && (stride != 1 || q != 4)) {
                err = "probe_bits 4 needs stride 1 and 4-byte q-grams";
                return GLOP_EINVAL;
            }
            if (k == 4) {
                if (o.bitmap_log2 && o.bitmap_log2 != 19) {
                    err = "probe_bits 4 needs bitmap_log2 19";
                    return GLOP_EINVAL;
                }
                lg = 19;
            }
            c.qgram = q;
            c.qmask = q == 4 ? 0xFFFFFFFFu : ((1u << (8 * q)) - 1u);
            c.stride = stride;
            c.bitmap_log2 = lg;
            c.probe_bits = k;
            c.filter_keys = keys.size();
            c.bitmap.assign((1u << lg) / 32, 0);
            for (uint32_t g : keys) {
                if (k == 4) {
                    const uint32_t b = glop_hash16(g) >> 1;  // 16-bit block
                    c.bitmap[b >> 1] |= glop_pair_bits(g) << (16u * (b & 1u));
                    continue;
                }
                if (k == 3) {
                    const uint32_t h = glop_hash1(g);
                    c.bitmap[glop_block_word(h, lg)] |= glop_block_bits(g);
                    continue;
                }
                const uint32_t s1 = glop_slot1(g, lg);
                c.bitmap[s1 >> 5] |= 1u << (s1 & 31);
                if (k == 2) {
                    const uint32_t s2 = glop_slot2(g, lg);
                    c.bitmap[s2 >> 5] |= 1u << (s2 & 31);
                }
            }
            // Second filter: stride 1 with a first filter that does not use
            // glop_hash2 (layout in glop_layout.hpp).
            c.bitmap2.clear();
            if (stride == 1 && k != 2) {
                c.bitmap2.assign((1u << GLOP_FILTER2_LOG2) / 32, 0u);
                for (uint32_t g : keys) {
                    const uint32_t h = glop_hash2(g), k = glop_f2_mix(h);
                    for (uint32_t x : {h, k, h + k, h + 2u * k, h + 3u * k}) {
                        const uint32_t s2 = x >> (32u - GLOP_FILTER2_LOG2);
                        c.bitmap2[s2 >> 5] |= 1u << (s2 & 31);
                    }
                }
            }
        } else {
            if (o.stride > 1 || o.qgram || o.bitmap_log2 || o.probe_bits) {
                err = "stride/qgram/bitmap/probe options need the q-gram filter";
                return GLOP_EINVAL;
            }
            c.qgram = 0;
            c.qmask = 0;
            c.stride = 1;
            c.bitmap_log2 = 12;
            c.bitmap.assign((1u << 12) / 32, 0);
            c.bitmap2.clear();
        }
        // Automatic: 4 KiB tiles for stride 4 with two hash bits (the filter
        // of dictionaries whose patterns are all 7 bytes or longer), where a
        // single text ran 1-6 % faster with them at every length; with the
        // stride-1 blocked filter, 4 KiB for short texts (kShortTextPerCu) and
        // 8 KiB above; 8 KiB otherwise.  (Batches: Compiled::batch_tile_kib.)
        const bool q4 = c.filter == GLOP_FILTER_QGRAM && c.qgram == 4;
        const bool small_tiles = q4 && c.stride == 4 && c.probe_bits == 2;
        const bool short_tiles = q4 && c.stride == 1 && c.probe_bits == 3;
        c.tile_kib = o.tile_kib ? o.tile_kib : (small_tiles ? 4u : 8u);
        c.tile_kib_short = !o.tile_kib && short_tiles ? 4u : 0u;
        c.tile_auto = o.tile_kib == 0;
        if (c.tile_kib != 8 && c.tile_kib != 4) {
            err = "tile_kib must be 0 (automatic), 4 or 8";
            return GLOP_EINVAL;
        }
        // 4 KiB tiles exist for the two default filters only.
        if (c.tile_kib == 4 &&
            !(c.filter == GLOP_FILTER_QGRAM && c.qgram == 4 &&
              ((c.stride == 4 && c.probe_bits == 2) || (c.stride == 1 && c.probe_bits == 3)))) {
            err = "tile_kib 4 needs 4-byte q-grams with stride 4 and probe_bits 2, or stride 1 and probe_bits 3";
            return GLOP_EINVAL;
        }
    } catch (const std::bad_alloc &) {
        err = "host allocation failed while building the filter";
        return GLOP_ENOMEM;
    }
    return GLOP_OK;
}

int compile(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n,
            const glop_build_opts *opts, Compiled &c, std::string &err) {
    glop_build_opts o{};
    if (opts) o = *opts;
    if (n > GLOP_MAX_PATTERNS) {
        err = "too many patterns";
        return GLOP_EINVAL;
    }
    if (n > 0 && (!patterns || !lengths)) {
        err = "NULL pattern or length array";
        return GLOP_EINVAL;
    }
    if (o.layout > GLOP_LAYOUT_HYBRID || o.placement > GLOP_PLACE_LDS) {
        err = "layout must be GLOP_LAYOUT_AUTO, _DENSE or _HYBRID and placement GLOP_PLACE_AUTO, _GLOBAL or _LDS";
        return GLOP_EINVAL;
    }
    if ((o.prefix_len > 255 && o.prefix_len != GLOP_PREFIX_FULL) ||
        (o.candidates && (o.prefix_len == 0 || o.prefix_len == GLOP_PREFIX_FULL))) {
        err = "prefix_len must be 0, 1..255 or GLOP_PREFIX_FULL, and candidates needs an explicit prefix_len";
        return GLOP_EINVAL;
    }
    c = Compiled{};
    c.num_patterns = n;
    c.prefix_len = o.prefix_len == GLOP_PREFIX_FULL ? 0u : o.prefix_len;
    if (o.prefix_len == 0 && n > 0 && patterns && lengths) c.prefix_len = auto_prefix_len(patterns, lengths, n);
    c.candidates = o.candidates ? 1u : 0u;
    c.min_len = n ? 0xFFFFFFFFu : 0;
    bool used[256] = {};
    // Bytes of pattern j the trie holds (all of it, or its first prefix_len).
    auto trie_len = [&](uint32_t j) { return c.prefix_len ? std::min(c.prefix_len, lengths[j]) : lengths[j]; };
    for (uint32_t j = 0; j < n; ++j) {
        if (lengths[j] == 0) {
            err = "pattern " + std::to_string(j) + " is empty";
            return GLOP_EINVAL;
        }
        if (lengths[j] > GLOP_MAX_PATTERN_LEN) {
            err = "pattern " + std::to_string(j) + " is longer than GLOP_MAX_PATTERN_LEN";
            return GLOP_ETOOLONG;
        }
        if (!patterns[j]) {
            err = "pattern " + std::to_string(j) + " is NULL";
            return GLOP_EINVAL;
        }
        // min_len bounds where a trie match can start (the filter and the
        // valid starts use it); max_len is the longest full pattern (the
        // overlap a split text needs, and how far verification reads).
        c.min_len = std::min(c.min_len, trie_len(j));
        c.max_len = std::max(c.max_len, lengths[j]);
        for (uint32_t k = 0; k < trie_len(j); ++k) used[patterns[j][k]] = true;
    }
    if (o.filter != GLOP_FILTER_AUTO && o.filter != GLOP_FILTER_NONE && o.filter != GLOP_FILTER_QGRAM) {
        err = "unknown filter option";
        return GLOP_EINVAL;
    }

    // Byte classes: class 0 = no pattern uses the byte; the rest in byte order.
    uint32_t C = 1;
    for (int b = 0; b < 256; ++b)
        if (used[b]) c.cls[b] = (uint8_t)C++;
    c.num_classes = C;

    try {
        // Insert every pattern (goto edges only), first-come state numbering.
        std::vector<uint32_t> rows(C, 0);
        std::vector<uint32_t> end_state(n);
        uint64_t S = 1;
        for (uint32_t j = 0; j < n; ++j) {
            uint64_t s = 0;
            for (uint32_t k = 0; k < trie_len(j); ++k) {
                uint64_t idx = s * C + c.cls[patterns[j][k]];
                uint32_t nx = rows[idx];
                if (nx == 0) {
                    if ((S + 1) * C * 4 > kMaxTableBytes || S + 1 > GLOP_STATE_MASK) {
                        err = "dictionary too large for the dense transition table";
                        return GLOP_ENOMEM;
                    }
                    nx = (uint32_t)S++;
                    rows.resize(S * C, 0);
                    rows[idx] = nx;
                }
                s = nx;
            }
            end_state[j] = (uint32_t)s;
        }
        c.num_states = (uint32_t)S;

        // Pattern ids ending at each (old) state, ascending: counting sort.
        std::vector<uint32_t> ids_at(S + 1, 0), ids(n);
        for (uint32_t j = 0; j < n; ++j) ids_at[end_state[j] + 1]++;
        for (uint64_t s = 0; s < S; ++s) ids_at[s + 1] += ids_at[s];
        {
            std::vector<uint32_t> fill(ids_at.begin(), ids_at.end() - 1);
            for (uint32_t j = 0; j < n; ++j) ids[fill[end_state[j]]++] = j;
        }
        auto is_term_old = [&](uint32_t s) { return ids_at[s + 1] > ids_at[s]; };

        // Breadth-first renumbering (children visited in class order).
        std::vector<uint32_t> order;
        order.reserve(S);
        std::vector<uint32_t> new_id(S, kNone);
        order.push_back(0);
        new_id[0] = 0;
        for (size_t q = 0; q < order.size(); ++q) {
            uint32_t s = order[q];
            for (uint32_t k = 1; k < C; ++k) {
                uint32_t ch = rows[(uint64_t)s * C + k];
                if (ch) {
                    new_id[ch] = (uint32_t)order.size();
                    order.push_back(ch);
                }
            }
        }

        c.delta.assign(S * C, 0);
        c.term.assign(2 * S, 0);
        std::vector<uint32_t> anc(S, kNone);  // nearest terminal strict ancestor (new ids)
        std::vector<uint32_t> merged;
        for (uint64_t ns = 0; ns < S; ++ns) {
            uint32_t old = order[ns];
            bool term = is_term_old(old);
            if (term) {
                // Output list = the nearest terminal ancestor's list merged with
                // the ids ending here; both are ascending.
                merged.clear();
                const uint32_t *own = ids.data() + ids_at[old];
                size_t own_n = ids_at[old + 1] - ids_at[old];
                if (anc[ns] != kNone) {
                    size_t a_first = c.term[2 * anc[ns]], a_n = c.term[2 * anc[ns] + 1];
                    merged.resize(a_n + own_n);
                    std::merge(c.outids.begin() + a_first, c.outids.begin() + a_first + a_n, own, own + own_n,
                               merged.begin());
                } else {
                    merged.assign(own, own + own_n);
                }
                if (c.outids.size() + merged.size() > 0xFFFFFFFFull) {
                    err = "output lists too large";
                    return GLOP_ENOMEM;
                }
                c.term[2 * ns] = (uint32_t)c.outids.size();
                c.term[2 * ns + 1] = (uint32_t)merged.size();
                c.outids.insert(c.outids.end(), merged.begin(), merged.end());
            }
            for (uint32_t k = 1; k < C; ++k) {
                uint32_t ch = rows[(uint64_t)old * C + k];
                if (!ch) continue;
                uint32_t nch = new_id[ch];
                c.delta[ns * C + k] = nch | (is_term_old(ch) ? GLOP_TERM_BIT : 0u);
                anc[nch] = term ? (uint32_t)ns : anc[ns];
            }
        }

        if (c.verifies()) {
            // Each pattern starts 8-byte aligned (the GPU verify stage compares
            // words); the zero padding is never compared.
            c.pat_off.resize(n);
            c.pat_len.resize(n);
            uint64_t total = 0;
            for (uint32_t j = 0; j < n; ++j) {
                c.pat_off[j] = total;
                c.pat_len[j] = lengths[j];
                total += (lengths[j] + 7u) & ~7u;
            }
            c.pat_bytes.assign(total, 0);
            for (uint32_t j = 0; j < n; ++j) std::memcpy(c.pat_bytes.data() + c.pat_off[j], patterns[j], lengths[j]);
        }

        if (c.min_len >= 4) build_prefix_table(c, c.min_len >= 8 ? 8u : 4u);
        int rc = build_filter(patterns, n, o, c, err);
        if (rc != GLOP_OK) return rc;

        // Device layout of the table.
        c.layout = o.layout ? o.layout : (S * C * 4 > kAutoHybridBytes ? GLOP_LAYOUT_HYBRID : GLOP_LAYOUT_DENSE);
        c.placement = o.placement;
        c.n_dense = (uint32_t)S;
        if (c.layout == GLOP_LAYOUT_HYBRID && (rc = build_hybrid(c, err)) != GLOP_OK) return rc;
    } catch (const std::bad_alloc &) {
        err = "host allocation failed while compiling the dictionary";
        return GLOP_ENOMEM;
    }
    return GLOP_OK;
}

namespace {

struct Found {
    uint64_t offset;
    uint32_t state;
};

// Walk from every start in [lo, hi); record (start, deepest terminal).  A
// hybrid table is walked in its device form (dense rows, then nodes).
void walk_range(const Compiled &c, const uint8_t *text, uint64_t len, uint64_t lo, uint64_t hi,
                std::vector<Found> &found) {
    const uint32_t C = c.num_classes;
    if (c.layout == GLOP_LAYOUT_HYBRID) {
        for (uint64_t i = lo; i < hi; ++i) {
            uint32_t s = 0, last = 0;
            for (uint64_t p = i; p < len; ++p) {
                const uint32_t e = c.step(s, c.cls[text[p]]);
                if (e == 0) break;
                s = e & GLOP_STATE_MASK;
                if (e & GLOP_TERM_BIT) last = s;
            }
            if (last) found.push_back({i, last});
        }
        return;
    }
    for (uint64_t i = lo; i < hi; ++i) {
        uint32_t s = 0, last = 0;
        for (uint64_t p = i; p < len; ++p) {
            uint32_t e = c.delta[(uint64_t)s * C + c.cls[text[p]]];
            if (e == 0) break;
            s = e & GLOP_STATE_MASK;
            if (e & GLOP_TERM_BIT) last = s;
        }
        if (last) found.push_back({i, last});
    }
}

}  // namespace

int cpu_walk(const Compiled &c, const uint8_t *text, uint64_t len, glop_match_t *out,
             uint64_t max_matches, uint64_t *counts, uint64_t *total, int threads) {
    if ((len > 0 && !text) || (max_matches > 0 && !out) || (c.num_patterns > 0 && !counts))
        return GLOP_EINVAL;
    if (counts) std::memset(counts, 0, sizeof(uint64_t) * c.num_patterns);
    uint64_t emitted = 0;
    if (c.num_patterns > 0 && len > 0) {
        if (threads < 1) threads = 1;
        if ((uint64_t)threads > len) threads = (int)len;
        std::vector<std::vector<Found>> parts(threads);
        try {
            std::vector<std::thread> pool;
            for (int t = 1; t < threads; ++t)
                pool.emplace_back(walk_range, std::cref(c), text, len, len * t / threads, len * (t + 1) / threads,
                                  std::ref(parts[t]));
            walk_range(c, text, len, 0, len / threads, parts[0]);
            for (auto &th : pool) th.join();
        } catch (const std::exception &) {
            return GLOP_ENOMEM;
        }
        for (const auto &part : parts)
            for (const Found &f : part) {
                uint32_t first = c.term[2 * f.state], cnt = c.term[2 * f.state + 1];
                for (uint32_t k = 0; k < cnt; ++k) {
                    uint32_t id = c.outids[first + k];
                    if (c.verifies() && c.pat_len[id] > c.prefix_len) {
                        const uint32_t L = c.pat_len[id], P = c.prefix_len;
                        if (f.offset + L > len ||
                            std::memcmp(text + f.offset + P, c.pat_bytes.data() + c.pat_off[id] + P, L - P) != 0)
                            continue;
                    }
                    counts[id] += 1;
                    if (emitted < max_matches) out[emitted] = glop_match_t{f.offset, id, 0};
                    ++emitted;
                }
            }
    }
    if (total) *total = emitted;
    return GLOP_OK;
}

}  // namespace glop
