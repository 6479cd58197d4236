/*
 * glop.h -- exact multi-pattern matching of a pattern dictionary against log
 * text on one MI355X (gfx950), after the failureless-trie method of
 * "GLoP: Enabling Massively Parallel Incident Response Through GPU Log
 * Processing" (arXiv 1704.02278).
 *
 * The problem (Section 1): rules (byte patterns) and logs (text) go in; out
 * come the number of suspicious events and their locations.  The method
 * (Sections 4-5) first builds a state machine from the patterns -- here a
 * failureless trie, i.e. goto edges only -- and then starts one walk of that
 * trie at every byte offset of the text; a walk follows the text while it
 * spells a pattern prefix and ends at the first byte with no edge.  Every
 * overlapping occurrence is therefore found:
 *
 *   M = { (i, j) : i + |p_j| <= len and text[i .. i+|p_j|) == p_j }
 *
 * reported as glop_match_t records sorted by ascending offset, then ascending
 * pattern id, plus per-pattern counts C[j] = #{ i : (i, j) in M }.
 *
 * Conventions for every call below:
 *   - integers are fixed width; text and patterns are raw bytes (any of the
 *     256 values, no terminator, case-sensitive);
 *   - pattern id j is the index of the pattern in the array given to the
 *     build call; identical patterns are accepted and each reports its own id;
 *   - "device pointer" means memory on the GPU the handle was built on (for
 *     example the data pointer of a torch CUDA tensor); "host pointer" means
 *     ordinary process memory;
 *   - calls returning int return GLOP_OK (0) or a negative glop error code;
 *     calls returning a handle return NULL on error; in both cases
 *     glop_last_error() / glop_last_error_message() describe the failure
 *     (per calling thread).
 */
#ifndef GLOP_H
#define GLOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define GLOP_OK 0
#define GLOP_EINVAL (-1)   /* invalid argument (NULL pointer, empty pattern, bad option, small workspace) */
#define GLOP_ENOMEM (-2)   /* host or device allocation failed, or the dictionary is too large */
#define GLOP_EHIP (-3)     /* a HIP runtime call failed (message names it) */
#define GLOP_ETOOLONG (-4) /* a pattern is longer than GLOP_MAX_PATTERN_LEN, or a text too long for glop_match_static */
#define GLOP_ENODEV (-5)   /* no usable GPU, or the handle has no device copy */
#define GLOP_EINTERNAL (-6) /* an internal consistency check failed */

#define GLOP_MAX_PATTERN_LEN 65535u
#define GLOP_MAX_PATTERNS (1u << 24)

/* One reported occurrence: 16 bytes, naturally aligned. */
typedef struct {
    uint64_t offset;     /* byte offset of the occurrence in the text of the call */
    uint32_t pattern_id; /* index of the pattern in the build call's array */
    uint32_t reserved;   /* always written as 0 */
} glop_match_t;

/* A compiled dictionary (the trie and its lookup tables); immutable once built. */
typedef struct glop_dict *glop_handle_t;

/*
 * Build options (glop_build_ex).  Zero-initialise and set what you need; every
 * setting except `candidates` changes only how the work is done, never the
 * result.
 *
 *   filter      GLOP_FILTER_AUTO (0) = automatic (the q-gram filter whenever the
 *                    dictionary is not empty);
 *               GLOP_FILTER_NONE  = walk the trie from every offset, exactly as
 *                    the one-walk-per-byte scheme of Section 5 does;
 *               GLOP_FILTER_QGRAM = two stages: a bitmap summary of the
 *                    patterns' leading q-byte strings rules out most offsets,
 *                    and the trie walk runs from every offset not ruled out
 *                    (the prefix filter + verify split of Sections 2 and 5,
 *                    with the verify stage on the GPU and exact).
 *   stride      0 = automatic; 1 = one filter probe per offset; 4 = one probe
 *               per aligned 4-byte word (needs every pattern to be at least
 *               qgram + 3 bytes long).
 *   qgram       0 = automatic (min(4, shortest pattern)); else 1..4 and at most
 *               the shortest pattern length.
 *   bitmap_log2 0 = automatic; else 12..19 (filter bitmap of 2^bitmap_log2 bits,
 *               resident in LDS).
 *   probe_bits  0 = automatic (3 at stride 1, where every offset is probed
 *               and the probes' LDS reads dominate; 2 at stride 4, where the
 *               walks of false positives do);
 *               1 or 2 bits per q-gram at independent positions (a Bloom
 *               filter with one or two hash functions); 3 = two bits within
 *               one 32-bit word chosen by one hash (a blocked Bloom filter:
 *               one lookup per probe); 4 = two bits within one 16-bit block
 *               (stride 1, 4-byte q-grams, bitmap_log2 19 only), which lets
 *               the kernel probe two offsets per instruction on packed
 *               16-bit halves.
 *   tile_kib    0 = automatic, 8 or 4: KiB of text one wavefront streams
 *               per tile in glop_match / glop_match_ws, 16 bytes per lane
 *               per round (8 rounds: 128 bytes per lane per tile; 4 rounds:
 *               64).  4 exists for 4-byte q-grams with stride 4 and
 *               probe_bits 2 or stride 1 and probe_bits 3 (the automatic
 *               filters); GLOP_EINVAL otherwise.  Automatic: 4 for stride 4
 *               with probe_bits 2; for stride 1 with probe_bits 3, 4 per call
 *               on texts of at most 640 KiB per CU (160 MiB on 256 CUs) and
 *               8 above; else 8.  glop_get_info reports the long-text tile.
 *               The workspace holds per-tile results, so
 *               glop_workspace_bytes (of the same length) grows with
 *               smaller tiles.  glop_match_host runs every piece with the
 *               tile of its longest piece.
 *               Batches (glop_match_batch) take the given tile_kib; when
 *               automatic, 4 for a max_total_bytes of at most 64 KiB per CU
 *               where the filter has 4 KiB kernels, else 8 (as does
 *               glop_batch_workspace_bytes of the same max_total_bytes).
 *   prefix_len  GLOP_PREFIX_FULL = the trie holds the whole patterns;
 *               1..255 = the trie holds each pattern's first prefix_len bytes
 *               only (the library of Sections 2 and 5 truncates patterns to 8
 *               characters), and a verify stage on the GPU compares the rest
 *               of every candidate against its full pattern, so the result is
 *               still exact; 0 = automatic: 8 when some pattern is longer than
 *               8 bytes and no more than 16 patterns share one 8-byte prefix
 *               (the verify stage then replaces most of each long walk's
 *               dependent trie steps with a few word compares), else whole.
 *   candidates  with prefix_len: 1 = report the unverified candidates instead,
 *               i.e. every (offset, id) whose first min(prefix_len, length)
 *               bytes match (the truncated matching of Sections 2 and 5, which
 *               can report false positives).  This changes the result.
 *   layout      how the transition table is stored on the device (Section 5
 *               ties the table's footprint to the cache hit rate; Section 8
 *               names a smaller footprint for larger state machines):
 *               GLOP_LAYOUT_DENSE = one row of num_classes next states per
 *                    state (one lookup per step);
 *               GLOP_LAYOUT_HYBRID = dense rows for the states of depth <= 2
 *                    (where walks branch), and below them one 8-byte node per
 *                    state naming its children, which breadth-first numbering
 *                    keeps contiguous (a state with one child, the common case
 *                    deep in a trie, is one lookup; with more, one more read of
 *                    the children's edge bytes): a few MB where the dense table
 *                    needs a hundred;
 *               GLOP_LAYOUT_AUTO (0) = hybrid when the dense table would exceed
 *                    32 MiB, else dense.
 *   placement   where the walks read the dense rows from:
 *               GLOP_PLACE_GLOBAL = device memory (through L2 / MALL);
 *               GLOP_PLACE_LDS = a copy staged in each workgroup's LDS (the
 *                    role Section 6 gives texture memory); GLOP_EINVAL at build
 *                    if it does not fit beside the scan kernel's other tables;
 *               GLOP_PLACE_AUTO (0) = LDS when the dense rows take at most
 *                    32 KiB and fit, else global.
 */
#define GLOP_PREFIX_FULL 0xFFFFFFFFu
#define GLOP_FILTER_AUTO 0
#define GLOP_FILTER_NONE 1
#define GLOP_FILTER_QGRAM 2
#define GLOP_LAYOUT_AUTO 0
#define GLOP_LAYOUT_DENSE 1
#define GLOP_LAYOUT_HYBRID 2
#define GLOP_PLACE_AUTO 0
#define GLOP_PLACE_GLOBAL 1
#define GLOP_PLACE_LDS 2
typedef struct {
    int32_t filter;
    uint32_t stride;
    uint32_t qgram;
    uint32_t bitmap_log2;
    uint32_t probe_bits;
    uint32_t tile_kib;
    uint32_t prefix_len;
    uint32_t candidates;
    uint32_t layout;
    uint32_t placement;
} glop_build_opts;

/*
 * Build a dictionary from n patterns (Section 4: the first phase builds the
 * state machine from the patterns; Section 5: the failure transitions are
 * dropped, leaving a trie of goto edges).
 *
 *   patterns  host array of n host pointers; pattern j is
 *             patterns[j][0 .. lengths[j]).  May be NULL when n == 0.
 *   lengths   host array of n lengths, each 1..GLOP_MAX_PATTERN_LEN.
 *   n         0..GLOP_MAX_PATTERNS; n == 0 is a valid empty dictionary.
 *
 * The patterns are copied; the caller may free its arrays on return.  The
 * compiled tables are uploaded to the current HIP device, to which the handle
 * is bound.  Errors: GLOP_EINVAL (NULL array, zero length), GLOP_ETOOLONG,
 * GLOP_ENOMEM, GLOP_EHIP / GLOP_ENODEV (upload failed or no GPU).
 */
glop_handle_t glop_build(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n);

/* As glop_build, with options (opts may be NULL = all automatic). */
glop_handle_t glop_build_ex(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n,
                            const glop_build_opts *opts);

/*
 * Host-only compile: the same trie and tables as glop_build_ex, without any
 * device upload (usable on machines with no GPU).  Such a handle serves the
 * introspection calls and glop_cpu_walk; glop_match on it fails with
 * GLOP_ENODEV.
 */
glop_handle_t glop_compile(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n,
                           const glop_build_opts *opts);

/* Release a handle and its device tables.  No match using it may still be in
 * flight on any stream.  NULL is ignored. */
void glop_free(glop_handle_t h);

/*
 * Match the dictionary against one text on the GPU (Section 5: one trie walk
 * per byte offset; a mismatch ends the walk, a match carries it on into the
 * following bytes).  Asynchronous on `stream`.
 *
 *   h            handle from glop_build / glop_build_ex, bound to the current device.
 *   d_text       device pointer to len bytes (any alignment); may be NULL iff len == 0.
 *   len          text length in bytes (0 allowed).
 *   d_out        device array of max_matches records; receives the first
 *                min(max_matches, |M|) records of M in (offset, id) order.
 *                May be NULL iff max_matches == 0.
 *   max_matches  capacity of d_out in records.  Truncation is not an error:
 *                the counts are always complete, and the caller detects it
 *                after the stream completes as sum(counts) > max_matches.
 *   d_counts     device array of n uint64 counts, overwritten with C.  May be
 *                NULL iff n == 0.
 *   stream       a hipStream_t (NULL = the default stream).
 *
 * Device scratch is taken from the stream-ordered allocator of `stream` and
 * released on it.  Returns once the work is enqueued.  The caller keeps every
 * buffer alive until the stream has completed it.  Concurrent calls on one
 * handle from different streams are safe (the handle is read-only).
 * Errors: GLOP_EINVAL, GLOP_ENODEV (host-only handle or another device is
 * current), GLOP_ENOMEM, GLOP_EHIP.
 */
int glop_match(glop_handle_t h, const uint8_t *d_text, uint64_t len, glop_match_t *d_out,
               uint64_t max_matches, uint64_t *d_counts, void *stream);

/*
 * Match a text held in host memory (any pageable buffer).  The text is
 * streamed to the device in pieces of chunk_bytes start offsets, each piece
 * carrying the next max_len - 1 bytes as well (Section 4: consecutive chunks
 * overlap by the longest pattern minus one, so no occurrence is cut).  Two
 * pinned staging buffers and two device buffers form a pipeline: host
 * threads copy piece k+1 into pinned memory and a copy stream moves it to the
 * device while piece k is matched on `stream` (Section 6: streams overlap the
 * next batch's transfer with the kernel).  Every piece adds its records to
 * one output in order and its counts to one set of counts, so the result is
 * exactly glop_match's on the whole text.  A text already in pinned host
 * memory (hipHostMalloc, or a pinned torch tensor) is uploaded from where it
 * is, without the staging copy.
 *
 *   h_text, len   host text (not modified; read during the call only).
 *   d_out, max_matches, d_counts   as for glop_match.
 *   d_total       device uint64_t for the record total, or NULL.
 *   chunk_bytes   start offsets per piece; 0 = 64 MiB; at least 4096.
 *   stream        hipStream_t or NULL; the call returns after the result is
 *                 complete on the device (it synchronizes the stream).
 * Errors: GLOP_EINVAL, GLOP_ENODEV, GLOP_ENOMEM, GLOP_EHIP.
 */
int glop_match_host(glop_handle_t h, const uint8_t *h_text, uint64_t len, glop_match_t *d_out,
                    uint64_t max_matches, uint64_t *d_counts, uint64_t *d_total, uint64_t chunk_bytes,
                    void *stream);

/* Bytes of device workspace glop_match_ws needs for a text of len bytes. */
uint64_t glop_workspace_bytes(glop_handle_t h, uint64_t len);

/*
 * Optional timing hooks for benchmarks: non-NULL members are hipEvent_t
 * handles that glop_match_ws records on the stream around its kernels.
 */
typedef struct {
    void *scan_begin; /* before the scan kernel (the text-streaming kernel) */
    void *scan_end;   /* after the scan kernel, before the emit kernel */
    void *emit_end;   /* after the emit kernel */
} glop_events_t;

/*
 * glop_match with caller-provided device workspace and an optional total.
 *
 *   d_total      pointer to one uint64 receiving |M| (may be NULL): device
 *                memory, or pinned host memory (hipHostMalloc), which the
 *                emit kernel then writes directly, visible to the host once
 *                the stream has completed the call.
 *   d_workspace  device pointer, 256-byte aligned, at least
 *                glop_workspace_bytes(h, len) bytes; owned by the caller, who
 *                must not use it for anything else until the stream has
 *                completed the call.  Two calls in flight at once need two
 *                workspaces.
 *   events       optional timing hooks (NULL = none).
 * Allocates nothing.  Other arguments and errors as glop_match; a workspace
 * that is NULL, misaligned or too small gives GLOP_EINVAL.
 */
int glop_match_ws(glop_handle_t h, const uint8_t *d_text, uint64_t len, glop_match_t *d_out,
                  uint64_t max_matches, uint64_t *d_counts, uint64_t *d_total, void *d_workspace,
                  uint64_t workspace_bytes, void *stream, const glop_events_t *events);

/*
 * For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, hosts that forbid allocation): glop_match_ws
 * with the library's own workspace, a static device array of 32 MiB that each
 * device holds from the library's first use on it until the process ends.
 * Allocates nothing.
 *
 *   d_total      as in glop_match_ws (may be NULL).
 *   other arguments as glop_match.
 *
 * Every call on one device shares that device's array: calls that overlap on
 * one device (two streams, or two host threads) race and give wrong results.
 * Serialise them, or use glop_match_ws with a workspace per stream.  The
 * kernels write every workspace word they later read, so nothing needs
 * clearing between calls.  A text whose workspace would exceed the array
 * (longer than glop_static_max_len(h) bytes: about 0.9 GiB with 4 KiB tiles,
 * 1.8 GiB with 8 KiB tiles, on 256 CUs) gives
 * GLOP_ETOOLONG before anything is enqueued.  Other errors as glop_match_ws.
 */
int glop_match_static(glop_handle_t h, const uint8_t *d_text, uint64_t len, glop_match_t *d_out,
                      uint64_t max_matches, uint64_t *d_counts, uint64_t *d_total, void *stream);

/* Longest text glop_match_static accepts for this handle's device (0 for NULL). */
uint64_t glop_static_max_len(glop_handle_t h);

/*
 * Batches: many independent texts ("chunks", e.g. log files of uneven size)
 * matched in one enqueue.  Each chunk is its own text: offsets are relative to
 * its first byte and no occurrence spans two chunks.  Per chunk the result is
 * exactly what glop_match returns for that chunk alone.
 */
typedef struct {
    const uint8_t *text; /* device pointer to the chunk (any alignment; NULL iff len == 0) */
    uint64_t len;        /* chunk length in bytes */
} glop_chunk_t;          /* 16 bytes */

typedef struct {
    uint64_t offset;     /* byte offset within the chunk */
    uint32_t pattern_id; /* index of the pattern in the build call's array */
    uint32_t chunk;      /* index of the chunk in the chunk table */
} glop_batch_match_t;    /* 16 bytes, same layout as glop_match_t */

/* Device workspace glop_match_batch needs for up to nchunks chunks of at most
 * max_total_bytes bytes in total. */
uint64_t glop_batch_workspace_bytes(glop_handle_t h, uint32_t nchunks, uint64_t max_total_bytes);

/*
 * Match every chunk of a batch in one persistent scan launch that takes work
 * items (runs of tiles, any mix of chunks) from a device work
 * queue, then one ordered emit launch.  Everything is enqueued on `stream`
 * and reads its inputs from device memory only, so a captured hipGraph can be
 * replayed after the chunk table (and the chunks) change, as long as nchunks
 * and max_total_bytes still hold.
 *
 *   d_chunks         device array of nchunks glop_chunk_t.
 *   nchunks          1..2^31.
 *   max_total_bytes  upper bound on the sum of the chunks' lengths (sizes the
 *                    workspace).  If the chunks exceed it the call does no
 *                    matching and writes *d_total = UINT64_MAX.
 *   d_out            device array of max_matches records: the batch's
 *                    occurrences in chunk order, then (offset, id) order; the
 *                    first max_matches are written.
 *   d_chunk_first    device array of nchunks: index in that order of chunk
 *                    c's first occurrence (where it would be if max_matches
 *                    were unlimited).
 *   d_chunk_count    device array of nchunks: occurrences in chunk c.
 *   d_counts         device array of n: per-pattern counts over the batch
 *                    (NULL iff n == 0).
 *   d_total          device pointer to the batch's occurrence count (required).
 *   d_workspace      256-byte aligned, >= glop_batch_workspace_bytes(...).
 * Allocates nothing.  Errors: as glop_match_ws.
 */
int glop_match_batch(glop_handle_t h, const glop_chunk_t *d_chunks, uint32_t nchunks, uint64_t max_total_bytes,
                     glop_batch_match_t *d_out, uint64_t max_matches, uint64_t *d_chunk_first,
                     uint64_t *d_chunk_count, uint64_t *d_counts, uint64_t *d_total, void *d_workspace,
                     uint64_t workspace_bytes, void *stream);

/*
 * glop_match_batch with a fixed output slice per chunk, so that what one chunk
 * receives does not depend on the other chunks of the batch (a server batches
 * independent requests, each with its own output capacity).
 *
 *   d_slice_first    device array of nchunks: index in d_out of chunk c's
 *                    first record.
 *   d_slice_cap      device array of nchunks: records chunk c may receive.
 *                    Chunk c's first min(d_chunk_count[c], d_slice_cap[c])
 *                    occurrences, in (offset, id) order, are written to
 *                    d_out[d_slice_first[c] ...]; nothing is written past the
 *                    slice, nor at an index >= max_matches.  Slices should not
 *                    overlap (overlapping slices receive both chunks' records
 *                    in no defined order).
 *   d_chunk_first    as in glop_match_batch: where chunk c's first occurrence
 *                    would be in the batch's concatenated order (the number
 *                    of occurrences in chunks before c), not its slice.
 * Other arguments, the per-pattern counts (always complete) and errors as
 * glop_match_batch; NULL slice arrays give GLOP_EINVAL.  Allocates nothing.
 */
int glop_match_batch_sliced(glop_handle_t h, const glop_chunk_t *d_chunks, uint32_t nchunks,
                            uint64_t max_total_bytes, glop_batch_match_t *d_out, uint64_t max_matches,
                            const uint64_t *d_slice_first, const uint64_t *d_slice_cap, uint64_t *d_chunk_first,
                            uint64_t *d_chunk_count, uint64_t *d_counts, uint64_t *d_total, void *d_workspace,
                            uint64_t workspace_bytes, void *stream);

/*
 * The failureless-trie walk on the host CPU over the same compiled trie (the
 * CPU side of the comparison in Section 7).  A timing baseline and a
 * check of the trie compiler; glop_match never calls it.
 *
 *   text         host pointer to len bytes.
 *   out          host array of max_matches records (NULL iff max_matches == 0).
 *   counts       host array of n counts (NULL iff n == 0), overwritten.
 *   total        receives |M| (may be NULL).
 *   threads      worker threads (<= 0 means 1); the result does not depend on it.
 * Errors: GLOP_EINVAL, GLOP_ENOMEM.
 */
int glop_cpu_walk(glop_handle_t h, const uint8_t *text, uint64_t len, glop_match_t *out,
                  uint64_t max_matches, uint64_t *counts, uint64_t *total, int threads);

/* Introspection of a compiled dictionary. */
typedef struct {
    uint32_t num_patterns;
    uint32_t min_len, max_len;
    uint32_t num_classes;    /* byte classes incl. class 0 ("no pattern uses this byte") */
    uint64_t num_states;     /* trie states incl. the root */
    uint64_t table_bytes;    /* transition table size on the device (dense rows, plus
                                the nodes and edge bytes of the hybrid layout) */
    uint64_t outlist_ids;    /* total entries of the per-state output lists */
    int32_t filter;          /* GLOP_FILTER_NONE or GLOP_FILTER_QGRAM as chosen */
    uint32_t stride, qgram, bitmap_log2, probe_bits, tile_kib;
    uint64_t filter_keys;    /* distinct q-grams set in the bitmap */
    uint32_t prefix_len;     /* 0, or the trie's truncation length */
    uint32_t candidates;     /* 1 if unverified prefix candidates are reported */
    uint64_t device_bytes;   /* device memory held by the handle */
    int32_t device;          /* HIP device id, or -1 for a host-only handle */
    uint32_t prefix_keys;    /* distinct prefix_depth-byte pattern prefixes in the prefix
                                table (0: no table, some pattern is shorter than 4 bytes) */
    uint32_t prefix_slots;   /* slots of the prefix table (a power of two, or 0) */
    uint32_t prefix_depth;   /* 8 if every pattern is at least 8 bytes, else 4 (or 0) */
    uint32_t filter2_log2;   /* bits (log2) of the second filter checked before
                                stride-1 walks (five bits per key), or 0 when
                                there is none */
    uint32_t layout;         /* GLOP_LAYOUT_DENSE or GLOP_LAYOUT_HYBRID as chosen */
    uint32_t placement;      /* GLOP_PLACE_GLOBAL or GLOP_PLACE_LDS as chosen
                                (GLOP_PLACE_GLOBAL for a host-only handle) */
    uint64_t dense_states;   /* states stored as dense rows (all of them when dense) */
} glop_info_t;
int glop_get_info(glop_handle_t h, glop_info_t *out);

/* Number of patterns and the longest pattern length of a dictionary (0 for a
 * null handle).  The longest length minus one is the overlap that a caller
 * splitting one text into independent pieces must give each piece (Section 4:
 * consecutive chunks share that many bytes so that no occurrence is cut). */
uint32_t glop_num_patterns(glop_handle_t h);
uint32_t glop_max_len(glop_handle_t h);

/* ---- Served matching: resident dictionaries, continuous batching ---------------
 *
 * A server holds several dictionaries resident on one device and matches
 * requests (device-resident texts, each tagged with one dictionary) as they
 * arrive.  A scheduler thread forms batches continuously: whenever one of its
 * stream slots is free it takes the dictionary whose oldest waiting request
 * arrived first and packs that dictionary's waiting requests, oldest first,
 * into one glop_match_batch launch (a lone request takes the single-text
 * kernels), up to max_batch_requests requests and max_batch_bytes bytes, and
 * as far as the HBM budget allows.  Requests that
 * arrive while batches run join the next launch.  The scheduler polls its
 * in-flight launches without sleeping (and for 2 ms after its last progress),
 * and glop_server_poll spins for up to 2 ms before it sleeps: a small
 * request's GPU time is about 20 us, far less than a thread's wake-up, so a
 * busy server keeps one host core busy.  The paper streams batches
 * of logs through the device so transfers overlap matching (Section 6) and
 * names real-time operation as future work (Section 8); this is that
 * operation for many concurrent streams.
 *
 * HBM budget: a request holds its payload bytes (if count_payload), its
 * output capacity (16 bytes per record, max(64, len / 256) records) and its
 * share of the batch workspace from admission until it is released.  A
 * request that does not fit waits; one that could never fit fails at submit.
 *
 * Plain mode (mode = GLOP_SERVE_PLAIN) is the baseline: no batching, every
 * request is one glop_match_ws call, in arrival order, on one stream.
 *
 * Results: a completion names the request, its record count and a device
 * pointer to its records (offsets relative to its own text, ascending, then
 * pattern ids ascending, as glop_match).  Records beyond the request's output
 * capacity are not written (truncated = 1; the count stays exact).  They stay
 * valid until glop_server_release(request id).  Results do not depend on
 * which requests share a batch.
 *
 * Threads: submit, poll and release may be called from any threads.  The
 * texts must stay valid and unchanged until the request completes.  Handles
 * added to a server must outlive it.
 */
#define GLOP_SERVE_BATCHED 0
#define GLOP_SERVE_PLAIN 1

typedef struct glop_server *glop_server_t;

typedef struct {
    int32_t mode;                /* GLOP_SERVE_BATCHED or GLOP_SERVE_PLAIN */
    uint32_t max_inflight;       /* batches in flight at once (stream slots); 0 = 8 */
    uint32_t max_batch_requests; /* 0 = 4096 */
    uint64_t max_batch_bytes;    /* 0 = 1 GiB */
    uint64_t hbm_budget_bytes;   /* 0 = 4 GiB */
    uint32_t count_payload;      /* 1: payload bytes count against the budget */
    uint32_t reserved;
} glop_server_opts;

typedef struct {
    uint64_t request_id;
    uint64_t tag;                  /* the caller's tag from submit */
    uint32_t dict;                 /* dictionary index */
    uint32_t truncated;            /* 1 if records were cut at the output capacity */
    uint64_t matches;              /* number of (offset, id) records of the request */
    uint64_t records;              /* records written at d_records (matches unless truncated) */
    const glop_match_t *d_records; /* device records of the request */
    int64_t arrival_ns;            /* arrival time given at submit (steady clock) */
    int64_t launch_ns;             /* when its batch was launched */
    int64_t done_ns;               /* when the scheduler saw its batch finish */
    uint32_t batch_requests;       /* requests in its batch */
    uint32_t reserved;
} glop_completion_t;

/* Create a server on the current device (opts may be NULL = defaults).
 * NULL on error (glop_last_error: GLOP_EINVAL for a bad mode, GLOP_EHIP,
 * GLOP_ENOMEM). */
glop_server_t glop_server_create(const glop_server_opts *opts);

/* Make dictionary h resident as index *dict (0, 1, ... in call order). */
int glop_server_add_dict(glop_server_t s, glop_handle_t h, uint32_t *dict);

/* Enqueue a request; arrival_ns is its arrival time on the steady clock
 * (glop_now_ns), or a negative value for "now".  *request_id receives its id.
 * Errors: GLOP_EINVAL (bad dictionary, NULL text with len > 0, a request
 * larger than the whole budget or than max_batch_bytes). */
int glop_server_submit(glop_server_t s, uint32_t dict, const uint8_t *d_text, uint64_t len, uint64_t tag,
                       int64_t arrival_ns, uint64_t *request_id);

/* Take up to max completions, waiting up to wait_us microseconds for the
 * first one; *n receives how many were written. */
int glop_server_poll(glop_server_t s, glop_completion_t *out, uint32_t max, uint32_t wait_us, uint32_t *n);

/* Release a completed request's records and HBM budget. */
int glop_server_release(glop_server_t s, uint64_t request_id);

/* Stop accepting releases, finish all submitted work, stop the scheduler and
 * free everything.  Records of completed requests, released or not, are
 * invalid once this is called. */
void glop_server_destroy(glop_server_t s);

/* Steady-clock time in nanoseconds (the clock of arrival_ns). */
int64_t glop_now_ns(void);

/* Open-loop trace replay (measurement): submit request k at t0 + at_ns[k]
 * from a submitter thread (t0 = the call's start), poll completions, record
 * each request's latency from its scheduled arrival to the moment its result
 * was visible on the host, and release it.  If copy_out is non-NULL, each
 * request's records are first copied (device to device) to
 * copy_out + copy_base[k] (records), at most copy_cap[k] of them.
 *   dicts, texts, lens, at_ns: n requests (at_ns ascending).
 *   latency_ns, matches, truncated: n outputs; batch_requests: n outputs or
 *   NULL (requests in the batch that served each one).
 *   *wall_ns: first scheduled arrival to last completion seen.
 */
int glop_server_run_trace(glop_server_t s, uint32_t n, const uint32_t *dicts, const uint8_t *const *texts,
                          const uint64_t *lens, const int64_t *at_ns, glop_match_t *copy_out,
                          const uint64_t *copy_base, const uint64_t *copy_cap, int64_t *latency_ns,
                          uint64_t *matches, uint32_t *truncated, uint32_t *batch_requests, int64_t *wall_ns);

/* ---- Autotuning ---------------------------------------------------------------
 *
 * glop_autotune: choose build options for a dictionary by timing them on a
 * device sample of representative text.  The filter of Sections 2 and 5
 * (prefilter, then full comparison) has free parameters the paper fixes for
 * its own hardware; here they are measured.  Starting from the automatic
 * options, the engine (whole patterns or 8-byte prefixes) and then one
 * parameter at a time is varied (filter on or off, q-gram length, stride,
 * probe bits, bitmap size, tile size) and a change is kept when it is at
 * least 3 % faster (median of 11 timed calls after 2 warm-up calls, and
 * after 50 ms of settling calls before the first candidate).  The
 * sample should be as large as the texts to be matched: per-call costs that do not scale
 * with the text (table staging, the end of each work item) weigh more on a
 * small one.  Every option set is exact, so all of them must report the same
 * number of matches on the sample; a difference fails the call.  The trie is
 * built and uploaded once; candidates differ only in their filter tables.
 *
 * Results are cached per device architecture and compute-unit count,
 * dictionary statistics (pattern count, shortest and longest length, trie
 * states rounded up to a power of two) and sample size (rounded up to a power
 * of two): in memory for the process, and in the text file named by the
 * environment variable GLOP_TUNE_CACHE if it is set (read once, appended).
 *
 *   patterns, lengths, n   as for glop_build.
 *   d_sample, sample_len   device text to time on (any alignment); at least
 *                          1 byte.  64 MiB or more gives stable timings.
 *   stream                 hipStream_t or NULL; the call synchronizes it.
 *   out                    receives the chosen options (pass out->opts to
 *                          glop_build_ex), their time and that of the
 *                          automatic options on the sample.
 * Errors: GLOP_EINVAL, GLOP_ETOOLONG, GLOP_ENOMEM, GLOP_EHIP, GLOP_ENODEV,
 *         GLOP_EINTERNAL (two option sets gave different match counts).
 */
typedef struct {
    glop_build_opts opts; /* chosen options, all explicit but tile_kib: 0 (automatic,
                             chosen per text length) where the automatic tile won */
    float ms;             /* median time of one match of the sample with them */
    float auto_ms;        /* the same with the automatic options */
    uint32_t evaluated;   /* option sets timed (0 when taken from the cache) */
    uint32_t from_cache;  /* 1 if the result came from the cache */
} glop_tune_result_t;

int glop_autotune(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n, const uint8_t *d_sample,
                  uint64_t sample_len, void *stream, glop_tune_result_t *out);

/* ---- Measurement helper -----------------------------------------------------
 *
 * glop_stream_read: read the first floor(len / 16) * 16 bytes at d_data once,
 * with the scan kernel's load shape at 8 KiB tiles (the same split into
 * per-workgroup items of 8 KiB tiles, 16-byte coalesced non-temporal loads per lane, one tile of
 * loads in flight ahead of use) and nothing else, and fold
 * them into the device uint64_t at d_sink (its value afterwards depends on
 * every byte read and is otherwise unspecified).  Its rate is
 * the practical ceiling for a pure HBM read stream on this device, against
 * which the matcher's rate is reported (Eq. 1 counts text bytes per second).
 *   d_data  device pointer, 16-byte aligned; not modified.
 *   d_sink  device pointer to one uint64_t.
 *   stream  hipStream_t or NULL (the null stream); the call is asynchronous.
 * Errors: GLOP_EINVAL (null or misaligned pointer with len >= 16),
 *         GLOP_EHIP (launch failure).
 */
int glop_stream_read(const uint8_t *d_data, uint64_t len, uint64_t *d_sink, void *stream);

int glop_last_error(void);
const char *glop_last_error_message(void);
const char *glop_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* GLOP_H */
