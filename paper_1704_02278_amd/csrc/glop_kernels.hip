// Matching kernels for gfx950 (CDNA4, wave64).
//
// Every byte offset of the text starts a walk of the failureless trie
// (Section 5).  The work is split in two kernels:
//
// scan  -- streams the text once from HBM.  Each wave owns 8 KiB tiles; a lane
//          holds 16 consecutive bytes per 1 KiB round (one coalesced 16-byte
//          load).  With the q-gram filter, the lane first probes an LDS Bloom
//          filter that summarises the trie's first q levels: an offset whose
//          q-gram misses the filter cannot start any pattern and needs no walk.
//          At stride 4 only aligned 4-byte words are probed; a word that hits
//          stands for the four offsets whose patterns must contain it.  This is
//          the prefix-filter stage of Sections 2 and 5, made exact because
//          every surviving offset is then walked through the full trie.
//          Survivors are appended in order to a per-wave LDS ring and walked
//          64 at a time, one per lane, so walks run with full waves instead of
//          the few divergent lanes Section 5 describes.  A tile's next loads
//          are issued as soon as its filter bits are known, before its walks.  A walk reads bytes
//          past its tile as needed (the overlap of at least the longest
//          pattern minus one byte that Section 4 requires between chunks).
//          Each tile's matched starts (offset, deepest terminal state) are
//          staged in workspace; the tile's record count is written out.
// emit  -- turns the per-tile record counts into output positions (sum over
//          earlier workgroups, then a block scan over the tiles) and writes the
//          (offset, id) records in order, plus the per-pattern counts.  A tile
//          with more matched starts than the staging slots is rescanned here
//          and written directly.
//
// No workgroup ever waits for another, so the kernels are safe to run beside
// any other work on the device.
#include <hip/hip_runtime.h>

#include "glop_kernels.hpp"

namespace glop {

namespace {

constexpr int kWave = 64;
constexpr int kWaves = 16;                        // waves per workgroup
constexpr int kBlock = kWave * kWaves;            // 1024 threads
constexpr int kRoundBytes = kWave * 16;           // 1 KiB: 16 bytes per lane
constexpr int kRounds = 8;                        // rounds per tile
constexpr int kTileBytes = kRoundBytes * kRounds; // 8 KiB per wave tile
constexpr uint32_t kStageCap = 16;                // staged matched starts per tile
// Per-wave LDS rings (u16 entries).  Stride 1 queues offsets: at most 63 left
// over plus 1024 from one round.  Stride 4 queues hit words: at most 15 left
// over plus 256 from one round plus the word after the tile.
constexpr uint32_t kRing1 = 2048;
constexpr uint32_t kRing4 = 512;
// Stride 4 defers the walks of a workgroup's interior tiles: hit words go to a
// workgroup-wide LDS list (entry = tile index in the range << 14 | word
// position 0..8192) and are walked after the whole range has streamed by.
constexpr uint32_t kHitCap = 8192;
// Tiles per workgroup at most (per-tile result counters live in LDS).
constexpr uint32_t kMaxTilesPerWg = 512;

template <int STRIDE>
constexpr uint32_t ring_cap() { return STRIDE == 4 ? kRing4 : kRing1; }

// Dynamic LDS: bitmap | byte classes | per-wave rings | hit list (stride 4) |
// per-tile matched-start counts | per-tile record counts.
template <int STRIDE>
struct LdsLayout {
    uint32_t bm_bytes;
    __host__ __device__ constexpr uint32_t cls_off() const { return bm_bytes; }
    __host__ __device__ constexpr uint32_t ring_off() const { return bm_bytes + 256; }
    __host__ __device__ constexpr uint32_t hits_off() const { return ring_off() + kWaves * ring_cap<STRIDE>() * 2; }
    __host__ __device__ constexpr uint32_t nm_off() const { return hits_off() + (STRIDE == 4 ? kHitCap * 4 : 0); }
    __host__ __device__ constexpr uint32_t rec_off() const { return nm_off() + kMaxTilesPerWg * 4; }
    __host__ __device__ constexpr uint32_t bytes() const { return rec_off() + kMaxTilesPerWg * 8; }
};

struct ScanParams {
    GlopDevDict d;
    const uint8_t *text;   // caller's text
    const uint8_t *abase;  // text rounded down to 16 bytes; coordinates x are relative to it
    uint64_t len;
    uint64_t head;         // text - abase (0..15)
    uint64_t span_end;     // head + len
    uint64_t valid_end;    // x < valid_end (and x >= head) can start a pattern
    uint64_t ntiles;
    uint64_t tiles_per_wg;
    uint64_t int_begin, int_end;  // tiles in [int_begin, int_end) lie inside the text with their extra word
    uint32_t bm_bytes;     // bitmap bytes staged in LDS (0 without filter)
    uint64_t *tile_rec;    // records per tile
    uint32_t *tile_nm;     // matched starts per tile
    uint64_t *staging;     // kStageCap per tile: (offset in tile << 32) | state
    uint64_t *wgsum;       // records per scan workgroup
    uint64_t *counts;      // per-pattern counts (zeroed by the scan kernel)
};

struct EmitParams {
    glop_match_t *out;
    uint64_t max_matches;
    uint64_t *total;
};

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Exclusive scan over the wave; `total` = sum.
__device__ __forceinline__ uint32_t wave_excl_scan_u32(uint32_t v, uint32_t &total) {
    const uint32_t lane = lane_id();
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t y = __shfl_up(incl, o);
        if (lane >= (uint32_t)o) incl += y;
    }
    total = __shfl(incl, kWave - 1);
    return incl - v;
}

// Exclusive prefix over the wave of small counts c < 2^BITS, and the total.
template <int BITS>
__device__ __forceinline__ uint32_t wave_prefix_small(uint32_t c, uint32_t &total) {
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint64_t bal = __ballot((c >> b) & 1u);
        pre += (uint32_t)__popcll(bal & lanemask_lt()) << b;
        tot += (uint32_t)__popcll(bal) << b;
    }
    total = tot;
    return pre;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 16 text bytes at aligned coordinate x; bytes outside the text read as 0.
__device__ __forceinline__ uint4 load16(const ScanParams &P, uint64_t x) {
    if (x >= P.head && x + 16 <= P.span_end) return *reinterpret_cast<const uint4 *>(P.abase + x);
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint64_t y = x + k;
        const uint32_t b = (y >= P.head && y < P.span_end) ? (uint32_t)P.abase[y] : 0u;
        const uint32_t sh = 8 * (k & 3);
        if (k < 4) w0 |= b << sh;
        else if (k < 8) w1 |= b << sh;
        else if (k < 12) w2 |= b << sh;
        else w3 |= b << sh;
    }
    return make_uint4(w0, w1, w2, w3);
}

// 4 text bytes at aligned coordinate x (multiple of 4); outside reads as 0.
__device__ __forceinline__ uint32_t load4(const ScanParams &P, uint64_t x) {
    if (x >= P.head && x + 4 <= P.span_end) return *reinterpret_cast<const uint32_t *>(P.abase + x);
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t y = x + k;
        w |= ((y >= P.head && y < P.span_end) ? (uint32_t)P.abase[y] : 0u) << (8 * k);
    }
    return w;
}

// Bloom probe: 1 if every probe bit of q-gram g is set.
template <int K, bool Q4>
__device__ __forceinline__ uint32_t probe(const uint32_t *bm, uint32_t g, uint32_t qmask, uint32_t sh) {
    if (!Q4) g &= qmask;
    const uint32_t s1 = glop_hash1(g) >> sh;
    uint32_t hit = bm[s1 >> 5] >> (s1 & 31);
    if (K == 2) {
        const uint32_t s2 = glop_hash2(g) >> sh;
        hit &= bm[s2 >> 5] >> (s2 & 31);
    }
    return hit & 1u;
}

// Offsets x .. x+15 that may start a pattern: head <= x+u < valid_end.
__device__ __forceinline__ uint32_t valid_mask16(const ScanParams &P, uint64_t x) {
    int64_t lo = (int64_t)P.head - (int64_t)x;
    int64_t hi = (int64_t)P.valid_end - (int64_t)x;
    lo = lo < 0 ? 0 : (lo > 16 ? 16 : lo);
    hi = hi < 0 ? 0 : (hi > 16 ? 16 : hi);
    if (hi <= lo) return 0u;
    return ((1u << hi) - 1u) & ~((1u << lo) - 1u);
}

// Every offset of tile t can start a pattern (no masking needed).
__device__ __forceinline__ bool tile_fully_valid(const ScanParams &P, uint64_t t) {
    const uint64_t x0 = t * (uint64_t)kTileBytes;
    return x0 >= P.head && x0 + kTileBytes <= P.valid_end;
}

// The failureless walk from text offset i (Section 5): follow goto edges while
// they exist; return the deepest terminal state passed (0 = none).  Text bytes
// come 8 at a time from aligned loads.
__device__ __forceinline__ uint32_t walk(const ScanParams &P, const uint8_t *cls, uint64_t i) {
    const uint32_t C = P.d.num_classes;
    const uint32_t *delta = P.d.delta;
    uint32_t s = 0, last = 0;
    uint64_t x = i + P.head;  // coordinate of the current byte
    uint64_t win = 0;
    uint32_t have = 0;
    while (x < P.span_end) {
        if (have == 0) {
            const uint64_t xa = x & ~7ull;
            if (xa >= P.head && xa + 8 <= P.span_end) {
                win = *reinterpret_cast<const uint64_t *>(P.abase + xa);
            } else {
                win = 0;
                for (int k = 0; k < 8; ++k) {
                    const uint64_t y = xa + k;
                    if (y >= P.head && y < P.span_end) win |= (uint64_t)P.abase[y] << (8 * k);
                }
            }
            win >>= 8 * (x - xa);
            have = 8 - (uint32_t)(x - xa);
        }
        const uint32_t c = cls[win & 0xFFu];
        win >>= 8;
        --have;
        const uint32_t e = delta[(uint64_t)s * C + c];
        if (e == 0) break;
        s = e & GLOP_STATE_MASK;
        if (e & GLOP_TERM_BIT) last = s;
        ++x;
    }
    return last;
}

// Sink of the scan kernel: stage matched starts of the tile, count records;
// the tile's totals go to the workgroup's LDS counters.
struct StageSink {
    uint32_t *nm_l;    // per-tile matched starts (LDS), indexed by t - tb
    uint64_t *rec_l;   // per-tile records (LDS)
    uint64_t tb;
    uint32_t nm = 0;   // matched starts so far (wave-uniform)
    uint64_t rec = 0;  // records so far (wave-uniform)

    __device__ __forceinline__ StageSink(uint32_t *nm_, uint64_t *rec_, uint64_t tb_)
        : nm_l(nm_), rec_l(rec_), tb(tb_) {}

    __device__ __forceinline__ void batch(const ScanParams &P, uint64_t t, uint64_t /*x0*/, uint32_t off,
                                          uint32_t last) {
        const bool m = last != 0;
        const uint64_t bal = __ballot(m);
        if (bal == 0) return;
        const uint32_t pos = nm + (uint32_t)__popcll(bal & lanemask_lt());
        if (m && pos < kStageCap) P.staging[t * kStageCap + pos] = ((uint64_t)off << 32) | last;
        nm += (uint32_t)__popcll(bal);
        rec += wave_sum_u32(m ? P.d.term[2 * last + 1] : 0u);
    }
    __device__ __forceinline__ void finish(const ScanParams &, uint64_t t) {
        if (lane_id() == 0) {
            nm_l[t - tb] = nm;
            rec_l[t - tb] = rec;
        }
    }
};

// Sink of the emit kernel's rescan: write the records directly, in order.
struct DirectSink {
    const EmitParams *E;
    uint64_t base;        // output position of the tile's first record
    uint64_t cursor = 0;  // records written so far in the tile

    __device__ __forceinline__ void batch(const ScanParams &P, uint64_t /*t*/, uint64_t x0, uint32_t off,
                                          uint32_t last) {
        const bool m = last != 0;
        if (__ballot(m) == 0) return;
        const uint32_t first = m ? P.d.term[2 * last] : 0u;
        const uint32_t cnt = m ? P.d.term[2 * last + 1] : 0u;
        uint32_t tot;
        const uint32_t excl = wave_excl_scan_u32(cnt, tot);
        if (m) {
            const uint64_t i = x0 + off - P.head;
            for (uint32_t k = 0; k < cnt; ++k) {
                const uint32_t id = P.d.outids[first + k];
                const uint64_t pos = base + cursor + excl + k;
                if (pos < E->max_matches) E->out[pos] = glop_match_t{i, id, 0u};
                atomicAdd(reinterpret_cast<unsigned long long *>(P.counts + id), 1ull);
            }
        }
        cursor += tot;
    }
    __device__ __forceinline__ void finish(const ScanParams &, uint64_t) {}
};

// A wave's tile in registers: 16 bytes per lane per round, plus the first
// word after the tile (for the probes of the tile's last offsets).
struct TileRegs {
    uint4 v[kRounds];
    uint32_t extra;
};

// Any tile: every byte checked against the text bounds.
template <bool FILTER>
__device__ __forceinline__ void load_tile(const ScanParams &P, uint64_t t, TileRegs &r) {
    const uint64_t x0 = t * (uint64_t)kTileBytes;
#pragma unroll
    for (int k = 0; k < kRounds; ++k) r.v[k] = load16(P, x0 + (uint64_t)k * kRoundBytes + lane_id() * 16u);
    r.extra = FILTER ? load4(P, x0 + kTileBytes) : 0u;
}

// Interior tile (int_begin <= t < int_end): plain coalesced 16-byte loads.
template <bool FILTER>
__device__ __forceinline__ void load_tile_interior(const ScanParams &P, uint64_t t, TileRegs &r) {
    const uint8_t *p = P.abase + t * (uint64_t)kTileBytes + lane_id() * 16u;
#pragma unroll
    for (int k = 0; k < kRounds; ++k) r.v[k] = *reinterpret_cast<const uint4 *>(p + k * kRoundBytes);
    r.extra = FILTER ? *reinterpret_cast<const uint32_t *>(P.abase + (t + 1) * (uint64_t)kTileBytes) : 0u;
}

// ---- stride 4: one probe per aligned word ---------------------------------
//
// Offset x needs the word at roundup4(x) to hit (every pattern is at least
// q + 3 bytes, so that word lies inside any occurrence starting at x, at
// pattern position t = roundup4(x) - x in 0..3).  Bit 4k+w of the lane's
// result is the word at x0 + k*1024 + lane*16 + 4w; `extra` is the word after
// the tile (it serves the tile's last three offsets).
template <int K, bool Q4>
__device__ __forceinline__ void tile_hits4(const ScanParams &P, const TileRegs &r, const uint32_t *bm,
                                           uint32_t &pbits, uint32_t &extra_bit) {
    const uint32_t qmask = P.d.qmask, sh = 32u - P.d.bitmap_log2;
    uint32_t b = 0;
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
        b |= probe<K, Q4>(bm, r.v[k].x, qmask, sh) << (4 * k);
        b |= probe<K, Q4>(bm, r.v[k].y, qmask, sh) << (4 * k + 1);
        b |= probe<K, Q4>(bm, r.v[k].z, qmask, sh) << (4 * k + 2);
        b |= probe<K, Q4>(bm, r.v[k].w, qmask, sh) << (4 * k + 3);
        // Finish each round's probes in place (see tile_masks1).
        __asm__ volatile("" : "+v"(b));
        __builtin_amdgcn_sched_barrier(0);
    }
    pbits = b;
    extra_bit = probe<K, Q4>(bm, r.extra, qmask, sh);
}

// Walk the four offsets of each queued hit word: lanes 4h..4h+3 take hit h's
// offsets p-3, p-2, p-1, p, so a batch of 16 hits is in offset order.
template <class Sink>
__device__ __forceinline__ void walk_hit_batch(const ScanParams &P, uint64_t t, const uint8_t *cls,
                                               const uint16_t *queue, uint32_t qhead, uint32_t n, Sink &sink) {
    const uint32_t lane = lane_id();
    const uint64_t x0 = t * (uint64_t)kTileBytes;
    const uint32_t h = lane >> 2;
    bool act = h < n;
    const int32_t p = act ? (int32_t)queue[(qhead + h) & (kRing4 - 1)] : 0;
    const int32_t off = p - 3 + (int32_t)(lane & 3);
    const uint64_t x = x0 + (int64_t)off;
    act = act && off >= 0 && off < kTileBytes && x >= P.head && x < P.valid_end;
    const uint32_t last = act ? walk(P, cls, x - P.head) : 0u;
    sink.batch(P, t, x0, act ? (uint32_t)off : 0u, last);
}

template <class Sink>
__device__ __forceinline__ void walk_hits4(const ScanParams &P, uint64_t t, uint32_t pbits, uint32_t extra_bit,
                                           const uint8_t *cls, uint16_t *queue, Sink &sink) {
    const uint32_t lane = lane_id();
    if (__ballot(pbits != 0) != 0 || extra_bit) {
        uint32_t qhead = 0, qtail = 0;  // wave-uniform ring indices
#pragma unroll
        for (int k = 0; k < kRounds; ++k) {
            uint32_t bits = (pbits >> (4 * k)) & 0xFu;
            if (__ballot(bits != 0) == 0) continue;
            uint32_t tot;
            uint32_t pos = qtail + wave_prefix_small<3>((uint32_t)__popc(bits), tot);
            const uint32_t base = (uint32_t)k * kRoundBytes + lane * 16u;
            while (bits) {
                const uint32_t w = (uint32_t)__builtin_ctz(bits);
                bits &= bits - 1u;
                queue[(pos++) & (kRing4 - 1)] = (uint16_t)(base + 4u * w);
            }
            qtail += tot;
            wave_lds_sync();
            for (; qtail - qhead >= 16u; qhead += 16u) walk_hit_batch(P, t, cls, queue, qhead, 16u, sink);
        }
        if (extra_bit) {
            if (lane == 0) queue[qtail & (kRing4 - 1)] = (uint16_t)kTileBytes;
            qtail += 1;
            wave_lds_sync();
        }
        for (; qtail != qhead;) {
            const uint32_t n = min(16u, qtail - qhead);
            walk_hit_batch(P, t, cls, queue, qhead, n, sink);
            qhead += n;
        }
    }
    sink.finish(P, t);
    __builtin_amdgcn_wave_barrier();
}

// ---- stride 1: one probe per offset (or none: walk every offset) ----------
//
// Bit u of round k's 16-bit mask (word k/2, half k%2) marks offset
// x0 + k*1024 + lane*16 + u as not ruled out.
template <bool FILTER, int K, bool Q4>
__device__ __forceinline__ void tile_masks1(const ScanParams &P, uint64_t t, const TileRegs &r,
                                            const uint32_t *bm, uint32_t (&m)[kRounds / 2]) {
    const uint32_t lane = lane_id();
    const uint64_t x0 = t * (uint64_t)kTileBytes;
    const uint32_t qmask = P.d.qmask, sh = 32u - P.d.bitmap_log2;
    const bool full = tile_fully_valid(P, t);
#pragma unroll
    for (int k = 0; k < kRounds / 2; ++k) m[k] = 0;
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
        uint32_t mask = 0xFFFFu;
        if (FILTER) {
            // Bytes 16..19 of the lane are the next lane's first word; for the
            // last lane, the next round's lane 0 (read wave-wide, before any
            // divergence) or the word after the tile.
            const uint32_t next0 =
                (k + 1 < kRounds) ? __builtin_amdgcn_readfirstlane(r.v[(k + 1) % kRounds].x) : r.extra;
            uint32_t nx = __shfl_down(r.v[k].x, 1);
            if (lane == kWave - 1) nx = next0;
            const uint32_t w[5] = {r.v[k].x, r.v[k].y, r.v[k].z, r.v[k].w, nx};
            mask = 0;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const uint32_t g = (u & 3) ? __builtin_amdgcn_alignbyte(w[(u >> 2) + 1], w[u >> 2], u & 3)
                                           : w[u >> 2];
                mask |= probe<K, Q4>(bm, g, qmask, sh) << u;
                if ((u & 3) == 3) {
                    // Finish these probes here; left alone, the compiler
                    // defers the bit tests and spills every hash and word.
                    __asm__ volatile("" : "+v"(mask));
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        if (!full) mask &= valid_mask16(P, x0 + (uint64_t)k * kRoundBytes + lane * 16u);
        m[k / 2] |= mask << (16 * (k % 2));
        // Keep rounds apart: interleaving all probes of the tile costs more
        // registers than the wave has.
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <class Sink>
__device__ __forceinline__ void walk_offsets1(const ScanParams &P, uint64_t t, const uint32_t (&m)[kRounds / 2],
                                              const uint8_t *cls, uint16_t *queue, Sink &sink) {
    const uint32_t lane = lane_id();
    const uint64_t x0 = t * (uint64_t)kTileBytes;
    uint32_t qhead = 0, qtail = 0;  // wave-uniform ring indices
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
        uint32_t mask = (m[k / 2] >> (16 * (k % 2))) & 0xFFFFu;
        if (__ballot(mask != 0) == 0) continue;
        uint32_t tot;
        uint32_t pos = qtail + wave_prefix_small<5>((uint32_t)__popc(mask), tot);
        const uint32_t base = (uint32_t)k * kRoundBytes + lane * 16u;
        while (mask) {
            const uint32_t u = (uint32_t)__builtin_ctz(mask);
            mask &= mask - 1u;
            queue[(pos++) & (kRing1 - 1)] = (uint16_t)(base + u);
        }
        qtail += tot;
        wave_lds_sync();
        for (; qtail - qhead >= (uint32_t)kWave; qhead += kWave) {
            const uint32_t off = queue[(qhead + lane) & (kRing1 - 1)];
            const uint32_t last = walk(P, cls, x0 + off - P.head);
            sink.batch(P, t, x0, off, last);
        }
    }
    if (qtail != qhead) {
        const uint32_t n = qtail - qhead;
        const bool act = lane < n;
        const uint32_t off = act ? queue[(qhead + lane) & (kRing1 - 1)] : 0u;
        const uint32_t last = act ? walk(P, cls, x0 + off - P.head) : 0u;
        sink.batch(P, t, x0, off, last);
    }
    sink.finish(P, t);
    __builtin_amdgcn_wave_barrier();
}

// Filter then walk one tile already in registers (no prefetch).
template <int STRIDE, bool FILTER, int K, bool Q4, class Sink>
__device__ __forceinline__ void scan_loaded_tile(const ScanParams &P, uint64_t t, const TileRegs &r,
                                                 const uint32_t *bm, const uint8_t *cls, uint16_t *queue,
                                                 Sink &sink) {
    if constexpr (STRIDE == 4) {
        uint32_t pbits, xb;
        tile_hits4<K, Q4>(P, r, bm, pbits, xb);
        walk_hits4(P, t, pbits, xb, cls, queue, sink);
    } else {
        uint32_t m[kRounds / 2];
        tile_masks1<FILTER, K, Q4>(P, t, r, bm, m);
        walk_offsets1(P, t, m, cls, queue, sink);
    }
}

// Copy the bitmap and byte classes into LDS.
template <bool FILTER>
__device__ __forceinline__ void stage_tables(const ScanParams &P, uint32_t *bm, uint8_t *cls) {
    if (FILTER) {
        const uint4 *src = reinterpret_cast<const uint4 *>(P.d.bitmap);
        uint4 *dst = reinterpret_cast<uint4 *>(bm);
        for (uint32_t k = threadIdx.x; k < P.bm_bytes / 16; k += kBlock) dst[k] = src[k];
    }
    if (threadIdx.x < 64)
        reinterpret_cast<uint32_t *>(cls)[threadIdx.x] = reinterpret_cast<const uint32_t *>(P.d.cls)[threadIdx.x];
}

// Record tile t's hit words in the workgroup list; false if the list is full
// (then the tile must be walked right away).
__device__ __forceinline__ bool list_hits(uint64_t t_rel, uint32_t pbits, uint32_t extra_bit, uint32_t *hits,
                                          uint32_t *hl_count, uint32_t *hl_limit) {
    const uint32_t lane = lane_id();
    uint32_t tot;
    const uint32_t pre = wave_prefix_small<6>((uint32_t)__popc(pbits), tot);
    const uint32_t n = tot + extra_bit;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(hl_count, n);
    base = __builtin_amdgcn_readfirstlane(base);
    if (base + n > kHitCap) {
        if (lane == 0) atomicMin(hl_limit, base);
        return false;
    }
    const uint32_t tag = (uint32_t)t_rel << 14;
    uint32_t pos = base + pre, b = pbits;
    while (b) {
        const uint32_t i = (uint32_t)__builtin_ctz(b);
        b &= b - 1u;
        hits[pos++] = tag | ((i >> 2) * kRoundBytes + lane * 16u + 4u * (i & 3u));
    }
    if (extra_bit && lane == 0) hits[base + tot] = tag | (uint32_t)kTileBytes;
    return true;
}

template <int STRIDE, bool FILTER, int K, bool Q4>
__global__ __launch_bounds__(kBlock) void glop_scan_kernel(ScanParams P) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t hl_count, hl_limit;
    __shared__ uint64_t wsum[kWaves];
    constexpr bool kDefer = STRIDE == 4;
    const LdsLayout<STRIDE> L{P.bm_bytes};
    uint32_t *bm = reinterpret_cast<uint32_t *>(lds);
    uint8_t *cls = lds + L.cls_off();
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    uint16_t *queue = reinterpret_cast<uint16_t *>(lds + L.ring_off()) + wave * ring_cap<STRIDE>();
    uint32_t *hits = reinterpret_cast<uint32_t *>(lds + L.hits_off());
    uint32_t *nm_l = reinterpret_cast<uint32_t *>(lds + L.nm_off());
    uint64_t *rec_l = reinterpret_cast<uint64_t *>(lds + L.rec_off());

    // Counts are accumulated by the emit kernel, which runs after this one.
    for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < P.d.num_patterns;
         k += (uint64_t)gridDim.x * kBlock)
        P.counts[k] = 0;
    stage_tables<FILTER>(P, bm, cls);
    for (uint32_t k = threadIdx.x; k < kMaxTilesPerWg; k += kBlock) {
        nm_l[k] = 0;
        rec_l[k] = 0;
    }
    if (threadIdx.x == 0) {
        hl_count = 0;
        hl_limit = kHitCap;
    }
    __syncthreads();

    const uint64_t tb = (uint64_t)blockIdx.x * P.tiles_per_wg;
    const uint64_t te = min(P.ntiles, tb + P.tiles_per_wg);
    // Interior tiles, pipelined: once a tile's filter bits are known its bytes
    // are dead, so the next tile's loads go out before anything else.
    const uint64_t ib = max(tb, P.int_begin), ie = min(te, P.int_end);
    TileRegs r;
    uint64_t t = ib + wave;
    if (t < ie) load_tile_interior<FILTER>(P, t, r);
    for (; t < ie; t += kWaves) {
        if constexpr (STRIDE == 4) {
            uint32_t pbits, xb;
            tile_hits4<K, Q4>(P, r, bm, pbits, xb);
            if (t + kWaves < ie) load_tile_interior<FILTER>(P, t + kWaves, r);
            if (__ballot(pbits != 0) == 0 && !xb) continue;  // no candidate: counters stay 0
            if (list_hits(t - tb, pbits, xb, hits, &hl_count, &hl_limit)) continue;
            StageSink sink(nm_l, rec_l, tb);
            walk_hits4(P, t, pbits, xb, cls, queue, sink);
        } else {
            uint32_t m[kRounds / 2];
            tile_masks1<FILTER, K, Q4>(P, t, r, bm, m);
            if (t + kWaves < ie) load_tile_interior<FILTER>(P, t + kWaves, r);
            StageSink sink(nm_l, rec_l, tb);
            walk_offsets1(P, t, m, cls, queue, sink);
        }
    }
    // Edge tiles (the first and last of the text): bounds-checked loads.
    for (uint64_t e = tb + wave; e < te; e += kWaves) {
        if (e >= ib && e < ie) continue;
        load_tile<FILTER>(P, e, r);
        StageSink sink(nm_l, rec_l, tb);
        scan_loaded_tile<STRIDE, FILTER, K, Q4>(P, e, r, bm, cls, queue, sink);
    }

    if (kDefer) {
        // Deferred walks: all waves take 16 listed hit words at a time, four
        // offsets each.  Matched starts claim staging slots with LDS atomics,
        // so a tile's slots are in no particular order (the emit kernel sorts
        // them).
        __syncthreads();
        const uint32_t nlist = min(hl_count, hl_limit);
        for (uint32_t b0 = wave * 16u; b0 < nlist; b0 += kWaves * 16u) {
            const uint32_t idx = b0 + (lane >> 2);
            bool act = idx < nlist;
            const uint32_t ent = act ? hits[idx] : 0u;
            const uint32_t t_rel = ent >> 14;
            const int32_t off = (int32_t)(ent & 0x3FFFu) - 3 + (int32_t)(lane & 3);
            const uint64_t tt = tb + t_rel;
            const uint64_t x = tt * (uint64_t)kTileBytes + (int64_t)off;
            act = act && off >= 0 && off < kTileBytes && x >= P.head && x < P.valid_end;
            const uint32_t last = act ? walk(P, cls, x - P.head) : 0u;
            if (last) {
                const uint32_t slot = atomicAdd(&nm_l[t_rel], 1u);
                if (slot < kStageCap) P.staging[tt * kStageCap + slot] = ((uint64_t)off << 32) | last;
                atomicAdd(reinterpret_cast<unsigned long long *>(&rec_l[t_rel]),
                          (unsigned long long)P.d.term[2 * last + 1]);
            }
        }
    }
    __syncthreads();
    // The range's tile results, coalesced, and the workgroup total.
    uint64_t part = 0;
    for (uint64_t k = tb + threadIdx.x; k < te; k += kBlock) {
        const uint64_t rc = rec_l[k - tb];
        P.tile_rec[k] = rc;
        P.tile_nm[k] = nm_l[k - tb];
        part += rc;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) wsum[wave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int w = 0; w < kWaves; ++w) s += wsum[w];
        P.wgsum[blockIdx.x] = s;
    }
}

// Exclusive scan over the block (1024 threads); `total` = block sum.
__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t v, uint64_t *sh, uint64_t &total) {
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    uint64_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint64_t y = __shfl_up(incl, o);
        if (lane >= (uint32_t)o) incl += y;
    }
    if (lane == kWave - 1) sh[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const uint64_t w = lane < kWaves ? sh[lane] : 0ull;
        uint64_t wi = w;
#pragma unroll
        for (int o = 1; o < kWaves; o <<= 1) {
            uint64_t y = __shfl_up(wi, o);
            if (lane >= (uint32_t)o) wi += y;
        }
        if (lane < kWaves) sh[lane] = wi - w;
        if (lane == kWaves - 1) sh[kWaves] = wi;
    }
    __syncthreads();
    const uint64_t excl = sh[wave] + incl - v;
    total = sh[kWaves];
    __syncthreads();
    return excl;
}

template <int STRIDE, bool FILTER, int K, bool Q4>
__global__ __launch_bounds__(kBlock) void glop_emit_kernel(ScanParams P, EmitParams E) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint64_t scan_sh[kWaves + 1];
    __shared__ uint64_t red[kWaves];
    __shared__ uint32_t n_over, any_over;
    __shared__ uint64_t over_tile[kBlock];
    __shared__ uint64_t over_base[kBlock];
    const LdsLayout<STRIDE> L{P.bm_bytes};
    uint32_t *bm = reinterpret_cast<uint32_t *>(lds);
    uint8_t *cls = lds + L.cls_off();
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    uint16_t *queue = reinterpret_cast<uint16_t *>(lds + L.ring_off()) + wave * ring_cap<STRIDE>();

    const uint64_t tb = (uint64_t)blockIdx.x * P.tiles_per_wg;
    const uint64_t te = min(P.ntiles, tb + P.tiles_per_wg);

    // Records of all earlier workgroups, and whether any tile here overflowed.
    uint64_t part = 0;
    for (uint32_t g = threadIdx.x; g < blockIdx.x; g += kBlock) part += P.wgsum[g];
    uint32_t over = 0;
    for (uint64_t t = tb + threadIdx.x; t < te; t += kBlock) over |= P.tile_nm[t] > kStageCap;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (threadIdx.x == 0) any_over = 0;
    __syncthreads();
    if (lane == 0) red[wave] = part;
    if (over) atomicOr(&any_over, 1u);
    __syncthreads();
    uint64_t base = 0;
    for (int w = 0; w < kWaves; ++w) base += red[w];
    if (any_over) {
        stage_tables<FILTER>(P, bm, cls);
        __syncthreads();
    }

    for (uint64_t c0 = tb; c0 < te; c0 += kBlock) {
        const uint64_t t = c0 + threadIdx.x;
        const bool in = t < te;
        const uint64_t rec = in ? P.tile_rec[t] : 0ull;
        uint64_t chunk_total;
        const uint64_t tile_base = base + block_excl_scan_u64(rec, scan_sh, chunk_total);
        if (threadIdx.x == 0) n_over = 0;
        __syncthreads();
        if (rec > 0) {
            const uint32_t nm = P.tile_nm[t];
            if (nm <= kStageCap) {
                // Staged starts, in ascending offset (slots may be unordered;
                // offsets are distinct, so the smallest entry above the last
                // one written is the next).
                uint64_t pos = tile_base;
                uint64_t prev = 0;
                for (uint32_t e = 0; e < nm; ++e) {
                    uint64_t ent = ~0ull;
                    for (uint32_t j = 0; j < nm; ++j) {
                        const uint64_t c = P.staging[t * kStageCap + j];
                        if ((e == 0 || c > prev) && c < ent) ent = c;
                    }
                    prev = ent;
                    const uint32_t st = (uint32_t)ent;
                    const uint64_t i = t * (uint64_t)kTileBytes + (ent >> 32) - P.head;
                    const uint32_t first = P.d.term[2 * st], cnt = P.d.term[2 * st + 1];
                    for (uint32_t k = 0; k < cnt; ++k, ++pos) {
                        const uint32_t id = P.d.outids[first + k];
                        if (pos < E.max_matches) E.out[pos] = glop_match_t{i, id, 0u};
                        atomicAdd(reinterpret_cast<unsigned long long *>(P.counts + id), 1ull);
                    }
                }
            } else {
                const uint32_t slot = atomicAdd(&n_over, 1u);
                over_tile[slot] = t;
                over_base[slot] = tile_base;
            }
        }
        __syncthreads();
        for (uint32_t o = wave; o < n_over; o += kWaves) {
            const uint64_t ot = over_tile[o];
            TileRegs r;
            load_tile<FILTER>(P, ot, r);
            DirectSink sink{&E, over_base[o]};
            scan_loaded_tile<STRIDE, FILTER, K, Q4>(P, ot, r, bm, cls, queue, sink);
        }
        __syncthreads();
        base += chunk_total;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0 && E.total) *E.total = base;
}

__global__ void glop_zero_kernel(uint64_t *counts, uint32_t n, uint64_t *total) {
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) counts[k] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && total) *total = 0;
}

struct Geometry {
    uint64_t ntiles, tiles_per_wg;
    uint32_t grid;
    uint64_t off_rec, off_nm, off_stage, off_wgsum, bytes;
};

constexpr uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

Geometry geometry(uint64_t len, int num_cus) {
    Geometry g{};
    // Tiles cover the text plus up to 15 leading bytes of alignment.
    g.ntiles = (len + 15 + kTileBytes - 1) / kTileBytes;
    const uint64_t wgs = (uint64_t)(num_cus > 0 ? num_cus : 1);
    g.tiles_per_wg = g.ntiles ? (g.ntiles + wgs - 1) / wgs : 1;
    if (g.tiles_per_wg > kMaxTilesPerWg) g.tiles_per_wg = kMaxTilesPerWg;
    g.grid = (uint32_t)(g.ntiles ? (g.ntiles + g.tiles_per_wg - 1) / g.tiles_per_wg : 0);
    g.off_rec = 0;
    g.off_nm = align256(g.off_rec + g.ntiles * 8);
    g.off_stage = align256(g.off_nm + g.ntiles * 4);
    g.off_wgsum = align256(g.off_stage + g.ntiles * kStageCap * 8);
    g.bytes = align256(g.off_wgsum + (uint64_t)g.grid * 8);
    if (g.bytes == 0) g.bytes = 256;
    return g;
}

template <int STRIDE>
constexpr size_t dyn_lds(uint32_t bm_bytes) {
    return LdsLayout<STRIDE>{bm_bytes}.bytes();
}

template <int STRIDE, bool FILTER, int K, bool Q4>
hipError_t launch_pair(const ScanParams &P, const EmitParams &E, uint32_t grid, hipStream_t stream,
                       const glop_events_t *ev) {
    const size_t lds = dyn_lds<STRIDE>(P.bm_bytes);
    if (ev && ev->scan_begin) {
        hipError_t e = hipEventRecord((hipEvent_t)ev->scan_begin, stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((glop_scan_kernel<STRIDE, FILTER, K, Q4>), dim3(grid), dim3(kBlock), lds, stream, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev && ev->scan_end) {
        e = hipEventRecord((hipEvent_t)ev->scan_end, stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((glop_emit_kernel<STRIDE, FILTER, K, Q4>), dim3(grid), dim3(kBlock), lds, stream, P, E);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev && ev->emit_end) e = hipEventRecord((hipEvent_t)ev->emit_end, stream);
    return e;
}

template <int STRIDE, bool FILTER, int K, bool Q4>
hipError_t set_lds_limit() {
    const int bytes = (int)dyn_lds<STRIDE>((1u << 19) / 8);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&glop_scan_kernel<STRIDE, FILTER, K, Q4>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&glop_emit_kernel<STRIDE, FILTER, K, Q4>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int STRIDE, int K, bool Q4>
hipError_t launch_filtered(const ScanParams &P, const EmitParams &E, uint32_t grid, hipStream_t s,
                           const glop_events_t *ev) {
    return launch_pair<STRIDE, true, K, Q4>(P, E, grid, s, ev);
}

}  // namespace

uint64_t workspace_bytes(uint64_t len, int num_cus) { return geometry(len, num_cus).bytes; }

hipError_t prepare_kernels() {
    hipError_t e = set_lds_limit<1, false, 1, false>();
    if (e == hipSuccess) e = set_lds_limit<1, true, 1, false>();
    if (e == hipSuccess) e = set_lds_limit<1, true, 1, true>();
    if (e == hipSuccess) e = set_lds_limit<1, true, 2, false>();
    if (e == hipSuccess) e = set_lds_limit<1, true, 2, true>();
    if (e == hipSuccess) e = set_lds_limit<4, true, 1, false>();
    if (e == hipSuccess) e = set_lds_limit<4, true, 1, true>();
    if (e == hipSuccess) e = set_lds_limit<4, true, 2, false>();
    if (e == hipSuccess) e = set_lds_limit<4, true, 2, true>();
    return e;
}

hipError_t launch_match(const MatchLaunch &a, hipStream_t stream) {
    const GlopDevDict &d = a.d;
    const bool trivial = d.num_patterns == 0 || a.len < d.min_len;
    if (trivial) {
        if (a.events && a.events->scan_begin) (void)hipEventRecord((hipEvent_t)a.events->scan_begin, stream);
        const uint32_t n = d.num_patterns;
        const uint32_t blocks = n ? (n + 255) / 256 : 1;
        hipLaunchKernelGGL(glop_zero_kernel, dim3(blocks > 1024 ? 1024 : blocks), dim3(256), 0, stream,
                           a.counts, n, a.total);
        hipError_t e = hipGetLastError();
        if (a.events && a.events->scan_end) (void)hipEventRecord((hipEvent_t)a.events->scan_end, stream);
        if (a.events && a.events->emit_end) (void)hipEventRecord((hipEvent_t)a.events->emit_end, stream);
        return e;
    }
    const Geometry g = geometry(a.len, a.num_cus);
    ScanParams P{};
    P.d = d;
    P.text = a.text;
    P.head = reinterpret_cast<uintptr_t>(a.text) & 15u;
    P.abase = a.text - P.head;
    P.len = a.len;
    P.span_end = P.head + a.len;
    P.valid_end = P.head + a.len - d.min_len + 1;
    P.ntiles = g.ntiles;
    P.tiles_per_wg = g.tiles_per_wg;
    P.int_begin = P.head ? 1 : 0;
    P.int_end = P.span_end >= 4 ? (P.span_end - 4) / kTileBytes : 0;
    P.bm_bytes = d.filter == GLOP_FILTER_QGRAM ? (1u << d.bitmap_log2) / 8 : 0u;
    uint8_t *ws = static_cast<uint8_t *>(a.workspace);
    P.tile_rec = reinterpret_cast<uint64_t *>(ws + g.off_rec);
    P.tile_nm = reinterpret_cast<uint32_t *>(ws + g.off_nm);
    P.staging = reinterpret_cast<uint64_t *>(ws + g.off_stage);
    P.wgsum = reinterpret_cast<uint64_t *>(ws + g.off_wgsum);
    P.counts = a.counts;
    EmitParams E{a.out, a.max_matches, a.total};
    const ScanParams &Pc = P;
    if (d.filter != GLOP_FILTER_QGRAM) return launch_pair<1, false, 1, false>(Pc, E, g.grid, stream, a.events);
    const bool q4 = d.qgram == 4;
    const bool k2 = d.probe_bits == 2;
    if (d.stride == 4) {
        if (k2) return q4 ? launch_filtered<4, 2, true>(Pc, E, g.grid, stream, a.events)
                          : launch_filtered<4, 2, false>(Pc, E, g.grid, stream, a.events);
        return q4 ? launch_filtered<4, 1, true>(Pc, E, g.grid, stream, a.events)
                  : launch_filtered<4, 1, false>(Pc, E, g.grid, stream, a.events);
    }
    if (k2) return q4 ? launch_filtered<1, 2, true>(Pc, E, g.grid, stream, a.events)
                      : launch_filtered<1, 2, false>(Pc, E, g.grid, stream, a.events);
    return q4 ? launch_filtered<1, 1, true>(Pc, E, g.grid, stream, a.events)
              : launch_filtered<1, 1, false>(Pc, E, g.grid, stream, a.events);
}

}  // namespace glop
