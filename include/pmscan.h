/*
 * pmscan.h -- C ABI of libpmscan.so, the MI355X (gfx950) k-mismatch
 * character-class DNA scan of arXiv 1611.06115 ("Fast low-level pattern
 * matching algorithm").
 *
 * The problem (paper Sect. 1.1): a text t over {A,C,G,T} and a pattern p whose
 * positions are IUPAC character classes; report every window i whose number
 * of positions j with t[i+j] outside p[j] is at most k (eq. (4), Sect. 2.4),
 * with that number.  Positions are 0-based here (the paper's location i is
 * position i-1).
 *
 * Conventions shared by every entry point:
 *  - Every function returns pm_status (PM_OK = 0) or a size; no exception or
 *    abort crosses the ABI.  pm_last_error_detail() describes the last failure
 *    of the calling thread.
 *  - "_dev" pointers are device (HBM) pointers owned by the caller (for
 *    example PyTorch tensors); the library allocates no device memory in the
 *    scan entry points and keeps no pointer after a call returns.  Host
 *    pointers are read during the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  GPU
 *    work is enqueued asynchronously on it; device-side results are valid
 *    once the stream has been synchronised.
 *  - Conditions detectable on the host (bad pattern symbol, m = 0, k too
 *    large, buffers too small, null pointers) are reported synchronously.
 *    Conditions found on the device are reported through device words the
 *    caller reads after synchronising: the index of the first bad text
 *    symbol, and hit totals that may exceed the output capacity.
 */
#ifndef PMSCAN_H
#define PMSCAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pm_status;
#define PM_OK 0
#define PM_ERR_ARG (-1)         /* invalid argument (null pointer, m = 0, k > 65535, ...) */
#define PM_ERR_SYMBOL (-2)      /* pattern symbol outside Table 2 / malformed class        */
#define PM_ERR_HIP (-3)         /* a HIP runtime call failed                                */
#define PM_ERR_WORKSPACE (-4)   /* workspace or output buffer smaller than required         */
#define PM_ERR_UNSUPPORTED (-5) /* valid request the library does not support              */
#define PM_ERR_BUSY (-6)        /* serving engine: no free slot or memory for the query     */
#define PM_ERR_NOT_FOUND (-7)   /* serving engine: unknown query id                          */

/* Human-readable name of a status code (static storage). */
const char* pm_status_string(pm_status s);
/* Detail of the last failure on the calling thread (thread-local storage). */
const char* pm_last_error_detail(void);
/* Library version string. */
const char* pm_version(void);

/* ------------------------------------------------------------------------ *
 * Text encoding -- Sect. 2.1, Table 1: A,C,G,T -> 00,01,10,11.
 *
 * Device layout ("planar 2-bit"): the text is cut into blocks of 32 bases;
 * block b is two 32-bit words, word 2b holding the high code bit of bases
 * 32b..32b+31 (bit i <-> base 32b+i) and word 2b+1 the low code bit.  That
 * is 8 bytes per 32 bases; a tail of zero blocks pads the buffer so that the
 * kernels may read whole 16-byte groups past the last base.
 * ------------------------------------------------------------------------ */

/* Bytes of the encoded text buffer for n bases (including the padding). */
uint64_t pm_text_bytes(uint64_t n);

/* Encode n ASCII bases (A, C, G, T in either case) from ascii_dev into
 * text_dev (pm_text_bytes(n) bytes).  bad_index_dev (one uint64 on the device)
 * receives the smallest index of a byte that is not a base, or UINT64_MAX if
 * there is none; bases at bad positions are encoded as A.  Text positions past
 * n are encoded as zero blocks.  Asynchronous on `stream`. */
pm_status pm_encode_text(const uint8_t* ascii_dev, uint64_t n, void* text_dev,
                         uint64_t* bad_index_dev, void* stream);

/* ------------------------------------------------------------------------ *
 * Pattern encoding -- Sect. 2.2, Table 2 (4-bit IUPAC class codes 0..15)
 * and Sect. 2.3, Table 3 (the 64-entry pair dictionary).
 * ------------------------------------------------------------------------ */

/* Parse a pattern of IUPAC letters (ACGTMRWSYKVHDBN, either case), '-'
 * (missing symbol, code 15, matches no base) and bracketed classes such as
 * "[CGT]" (canonicalised to their IUPAC code).  Writes min(m, cap) codes to
 * `codes` (host) and the pattern length to *m_out.  PM_ERR_SYMBOL on an
 * unknown symbol, an empty "[]", '-' inside brackets or an unclosed bracket. */
pm_status pm_encode_pattern(const char* pattern, uint64_t len, uint8_t* codes, uint64_t cap,
                            uint32_t* m_out);

/* Fill table[64] (host) with the pair dictionary L of Table 3, index
 * (p << 2) | t, value 0 for a match and 1 for a mismatch.  The values are
 * derived from prime coding: base t gets prime q_t of (2, 3, 5, 7), class p
 * the product of its members' primes (1 for '-'), and L = [q_t does not
 * divide that product]. */
pm_status pm_pair_table(uint8_t table[64]);

/* Bytes of the device pattern image for a pattern of length m. */
uint64_t pm_pattern_bytes(uint32_t m);

/* Build the device pattern image on the host (image_host, `bytes` >=
 * pm_pattern_bytes(m)); the caller copies it to device memory and passes it
 * to pm_scan.  Layout: for each 32-position chunk c, four uint32 words, word
 * 4c+t having bit j set iff text code t mismatches pattern position 32c+j
 * (the Table 3 value of that pair); bits past m are 0. */
pm_status pm_pattern_image(const uint8_t* codes, uint32_t m, void* image_host, uint64_t bytes);

/* ------------------------------------------------------------------------ *
 * Scan -- eq. (4) with the early stop of Sect. 2.4 and the text tiling of
 * Sect. 2.6, for one pattern.
 * ------------------------------------------------------------------------ */

/* Workspace bytes pm_scan needs for a text of n bases (any m). */
uint64_t pm_scan_workspace_bytes(uint64_t n);

/* Scan windows [win_begin, win_end) (clipped to [0, n-m+1)) of the encoded
 * text (n bases) against the pattern (host `codes`, m of them, and its device
 * image from pm_pattern_image) with at most k mismatches (k <= 65535).
 * Writes the hits in ascending position order: the first `capacity` of them
 * to pos_dev (int64) and cnt_dev (uint16, the exact mismatch count, <= k);
 * *n_hits_dev (device uint64) receives the total number of hits, which may
 * exceed capacity (then the call can be repeated with a larger buffer).
 * ws_dev: device workspace of at least pm_scan_workspace_bytes(n) bytes; it
 * needs no initialisation, holds nothing between calls, and must not be used
 * by two calls that can run at the same time.  m > n gives 0 hits.
 * Asynchronous on `stream`.  The filter plan of a pattern of 4096 positions
 * or more is kept for the calling thread (up to 16 plans, each with a copy of
 * its codes, used again only for the same k and identical codes). */
pm_status pm_scan(const void* text_dev, uint64_t n, const uint8_t* codes, uint32_t m,
                  uint32_t k, const void* image_dev, uint64_t win_begin, uint64_t win_end,
                  int64_t* pos_dev, uint16_t* cnt_dev, uint64_t capacity, uint64_t* n_hits_dev,
                  void* ws_dev, uint64_t ws_bytes, void* stream);

/* pm_scan without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid allocation.  Same arguments and results as pm_scan
 * minus ws_dev/ws_bytes.  Its scratch (per-tile hit counts, staged hits) is
 * a static 32 MiB device array of the library, one per GPU it runs on, held
 * until the process ends; the call allocates no device memory (its first
 * call on a device looks up that device's copy of the array).  The window
 * range [win_begin, win_end) (after clipping to [0, n-m+1)) may span at most
 * pm_scan_noalloc_max_windows() windows, else PM_ERR_WORKSPACE (scan a longer
 * text in several ranges).  The scratch needs no initialisation and keeps the
 * last call's contents; every call on one GPU shares it, so calls that can
 * overlap on the same GPU (other streams, other host threads) race and must
 * be serialised by the caller. */
uint64_t pm_scan_noalloc_max_windows(void);
pm_status pm_scan_noalloc(const void* text_dev, uint64_t n, const uint8_t* codes, uint32_t m,
                          uint32_t k, const void* image_dev, uint64_t win_begin, uint64_t win_end,
                          int64_t* pos_dev, uint16_t* cnt_dev, uint64_t capacity,
                          uint64_t* n_hits_dev, void* stream);

/* ------------------------------------------------------------------------ *
 * FASTA input -- the paper scans a chromosome read from a FASTA file
 * (Sect. 3); its text alphabet is Table 1's four bases.  Reading of a real
 * assembly: records are separate texts; lower-case (soft-masked) letters are
 * the same bases; any other sequence letter (N or another IUPAC code, '-',
 * '*') is an unknown base, for which eq. (4) has no pair value, so a window
 * covering one has no count and is never reported; a window never spans two
 * records.  Positions are offsets in the concatenation of the records'
 * letters (headers, line breaks and blanks removed).
 * ------------------------------------------------------------------------ */

typedef struct pm_fasta pm_fasta;

/* Parse FASTA text (host memory, `len` bytes): '>' header lines (the name is
 * the text up to the first blank), sequence lines, ';' comment lines, any
 * line breaks.  *out receives a handle owning the parsed data (free it with
 * pm_fasta_free).  PM_ERR_SYMBOL for a byte that is not a sequence letter, a
 * sequence before the first header, or no header at all. */
pm_status pm_fasta_parse(const char* data, uint64_t len, pm_fasta** out);
void pm_fasta_free(pm_fasta* f);

/* Bases of all records, concatenated, and their ASCII letters (host memory
 * owned by the handle; A, C, G, T upper case, unknown bases written as 'A'):
 * the caller copies them to the device and encodes them with
 * pm_encode_text. */
uint64_t pm_fasta_length(const pm_fasta* f);
const uint8_t* pm_fasta_bases(const pm_fasta* f);

/* Records: name (owned by the handle), offset and length in the bases. */
uint32_t pm_fasta_record_count(const pm_fasta* f);
pm_status pm_fasta_record(const pm_fasta* f, uint32_t i, const char** name, uint64_t* offset,
                          uint64_t* length);

/* Maximal runs of unknown bases (offset and length), ascending. */
uint64_t pm_fasta_unknown_run_count(const pm_fasta* f);
pm_status pm_fasta_unknown_run(const pm_fasta* f, uint64_t i, uint64_t* start, uint64_t* length);

/* The window ranges [begin[r], end[r]) of a pattern of length m that lie in
 * one record and cover no unknown base, ascending and disjoint: *count gets
 * their number; the first `cap` are written to begin/end (host). */
pm_status pm_fasta_window_ranges(const pm_fasta* f, uint32_t m, uint64_t* begin, uint64_t* end,
                                 uint64_t cap, uint64_t* count);

/* pm_scan over those window ranges of the encoded concatenation (text_dev,
 * pm_fasta_length(f) bases): the hits of every range, in ascending position
 * order, the first `capacity` to pos_dev/cnt_dev; *n_hits (host) receives the
 * total.  ws_dev: at least pm_scan_fasta_workspace_bytes(f) bytes, 256-byte
 * aligned.  Returns when the scan is complete (it waits on `stream` after
 * each range to place the next one's hits). */
uint64_t pm_scan_fasta_workspace_bytes(const pm_fasta* f);
pm_status pm_scan_fasta(const pm_fasta* f, const void* text_dev, const uint8_t* codes, uint32_t m,
                        uint32_t k, const void* image_dev, int64_t* pos_dev, uint16_t* cnt_dev,
                        uint64_t capacity, uint64_t* n_hits, void* ws_dev, uint64_t ws_bytes,
                        void* stream);

/* Scan of a text kept in host memory (Sect. 2.6's split into pieces with an
 * m-1 overlap).  ascii_host: n bases of A/C/G/T (either case) in host
 * memory; allocated with hipHostMalloc (pinned) the copies run at the full
 * speed of the link, pageable memory works more slowly.  The windows are cut
 * into chunks of chunk_bases windows; each chunk's bases (with the m-1 that
 * follow) are copied into one of two device buffers on copy_stream while the
 * previous chunk is encoded and scanned on `stream`.  Results equal pm_scan
 * over the whole text: ascending text positions and exact counts, the first
 * `capacity` hits in pos_dev / cnt_dev, *n_hits_dev = the total.  ws_dev:
 * 256-byte aligned, at least pm_scan_host_workspace_bytes(chunk_bases, m)
 * bytes (0 for an invalid chunk_bases or m).  chunk_bases: 1..2^48, else
 * PM_ERR_ARG.  A byte other than A/C/G/T gives PM_ERR_SYMBOL (the detail
 * names its index); with m > n there are no windows and the text is not
 * read.  Returns when the scan is complete (it waits for both streams); the
 * host text must stay valid until then. */
uint64_t pm_scan_host_workspace_bytes(uint64_t chunk_bases, uint32_t m);
pm_status pm_scan_host(const uint8_t* ascii_host, uint64_t n, const uint8_t* codes, uint32_t m,
                       uint32_t k, const void* image_dev, uint64_t chunk_bases, int64_t* pos_dev,
                       uint16_t* cnt_dev, uint64_t capacity, uint64_t* n_hits_dev, void* ws_dev,
                       uint64_t ws_bytes, void* stream, void* copy_stream);

/* Mismatch counts of every window by the Linhart-Shamir route of Sect. 1.3
 * (eqs. 1-3): the correlation of the CRT-coded pattern with the text, carried
 * as its residues modulo four primes above m (the full value outgrows 64
 * bits, Sect. 1.3.5) and computed with number-theoretic transforms over text
 * blocks that overlap by m-1.  A second exact route beside pm_scan: it gives
 * every window's count whatever k, at a cost that does not depend on k.
 * text_dev: the encoded text (16-byte aligned), n bases of any length the
 * encoding holds (block offsets and window indexes are 64-bit; tested past
 * 2^32 windows); codes: m Table 2 codes (host; m in 1..2^22, larger is
 * PM_ERR_UNSUPPORTED).  counts_dev receives
 * counts_dev[i] = number of mismatches of window i, for i in [0, n-m+1)
 * (nothing when m > n).  ws_dev: 256-byte aligned, at least
 * pm_crt_counts_workspace_bytes(n, m) bytes (0 for an invalid m).  Returns
 * once the pattern has been staged (one small synchronous copy); the rest
 * runs asynchronously on `stream`. */
uint64_t pm_crt_counts_workspace_bytes(uint64_t n, uint32_t m);
pm_status pm_crt_counts(const void* text_dev, uint64_t n, const uint8_t* codes, uint32_t m,
                        uint32_t* counts_dev, void* ws_dev, uint64_t ws_bytes, void* stream);

/* Measurement hook: the next pm_scan or pm_scan_batch call made by this
 * thread records ev_begin on its stream right before its main kernel launch
 * (the count kernel; the batched kernels) and ev_end right after it, so that
 * a caller can time that kernel alone with hipEventElapsedTime.  Events are
 * hipEvent_t passed as void*, created by the caller; both or neither. */
pm_status pm_time_next_scan(void* ev_begin, void* ev_end);

/* Expected number of hits of a pattern in a text of n i.i.d. uniform bases:
 * (n-m+1) times the Poisson-binomial probability that at most k of the
 * pattern's positions mismatch (per-position mismatch probability = number
 * of bases outside the class / 4).  For sizing output buffers. */
pm_status pm_expected_hits(const uint8_t* codes, uint32_t m, uint32_t k, uint64_t n, double* out);

/* ------------------------------------------------------------------------ *
 * Batched scan -- many patterns, each with its own k, in one persistent
 * launch over one encoded text (the scan of each pattern is the one above).
 * ------------------------------------------------------------------------ */

typedef struct {
    uint32_t group_size;  /* patterns sharing each text tile (1..16); 0 = 8          */
    uint32_t sub_ranges;  /* text sub-ranges per pattern group (1..4096); 0 = auto:  */
                          /* about 32768 work items per call                          */
    uint32_t lane_words;  /* 32-window words per lane: 4 or 6; 0 = auto: 6 for calls */
                          /* of 2 to 16 patterns, 4 otherwise (other values: 4)      */
    uint32_t reserved;
} pm_batch_config;

/* Workspace bytes pm_scan_batch needs (depends on the patterns' lengths and
 * output capacities and on cfg, which may be NULL for the defaults); 0 when
 * the capacities sum to more than 2^44 hits. */
uint64_t pm_scan_batch_workspace_bytes(uint64_t n, uint32_t count, const uint32_t* m,
                                       const uint64_t* capacity, const pm_batch_config* cfg);

/* Scan windows [win_begin, win_end) of the encoded text for `count` patterns.
 * Host inputs: codes (all patterns' Table 2 codes, concatenated), m[count],
 * k[count] (each <= 65535), out_off[count] and capacity[count] (summing to
 * at most 2^44, else PM_ERR_ARG): pattern p's
 * hits go to pos_dev/cnt_dev[out_off[p] .. out_off[p]+capacity[p]), in
 * ascending position order, with exact counts.  Device outputs per pattern:
 * n_hits_dev[p] = its total number of hits; status_dev[p] = 0 when its list
 * is complete, 1 when it is not (more than capacity[p] hits, or more than its
 * share of staging in one text sub-range): such a pattern must be scanned
 * again (e.g. with pm_scan and an exact buffer).  ws_dev: at least
 * pm_scan_batch_workspace_bytes(...) bytes, no initialisation needed, used by
 * one call at a time.  One host-to-device copy of the batch description is
 * enqueued on `stream` (the host buffer is released before the call returns),
 * then the kernels. */
pm_status pm_scan_batch(const void* text_dev, uint64_t n, uint32_t count, const uint8_t* codes,
                        const uint32_t* m, const uint32_t* k, const uint64_t* out_off,
                        const uint64_t* capacity, uint64_t win_begin, uint64_t win_end,
                        int64_t* pos_dev, uint16_t* cnt_dev, uint64_t* n_hits_dev,
                        uint32_t* status_dev, void* ws_dev, uint64_t ws_bytes,
                        const pm_batch_config* cfg, void* stream);

/* ------------------------------------------------------------------------ *
 * Query server -- a text resident in HBM, pattern queries arriving at any
 * time, scanned together (continuous batching).  Each query's result is the
 * pm_scan result of (text, pattern, k) over all windows, bit for bit.
 *
 * An engine thread owned by the server admits queries in arrival order while
 * a slot (config.max_active) and arena memory (hit segments sized from
 * pm_expected_hits, the pattern image, its share of the batch workspace)
 * are free.  It scans the text in `chunks` revolving window ranges: one chunk
 * step is one pm_scan_batch launch over chunk c for every admitted query, so
 * a query submitted while others are on the GPU joins them at the next step.
 * After it has been through every chunk, its per-chunk hits are joined in
 * chunk order (ascending positions) inside the arena and it is complete.  A
 * chunk whose hits overflow the query's segment is re-scanned with pm_scan
 * into an exact segment.  Queries wait (they are not refused) while memory
 * is short; a query that could never fit the arena fails with
 * PM_ERR_WORKSPACE.
 * ------------------------------------------------------------------------ */

typedef struct pm_server pm_server;

typedef struct {
    uint32_t chunks;          /* window ranges per revolution of the text; 0 = 1      */
    uint32_t max_active;      /* queries scanned together (slots); 0 = 1024           */
    uint64_t workspace_bytes; /* arena bytes kept for the batch workspace; 0 = 1/4   */
    pm_batch_config batch;    /* shape of the batched launches; zeros = defaults.     */
                              /* sub_ranges 0: admission sizes the workspace for 64   */
                              /* per group, each step takes up to the automatic count */
                              /* for its queries as far as the workspace allows       */
} pm_server_config;

#define PM_QUERY_WAITING 0    /* submitted, not admitted yet           */
#define PM_QUERY_ACTIVE 1     /* admitted, being scanned               */
#define PM_QUERY_DONE 2       /* result ready in the arena             */
#define PM_QUERY_FAILED 3     /* see pm_query_info.error               */

typedef struct {
    int32_t state;            /* PM_QUERY_*                                              */
    int32_t error;            /* pm_status of a failed query                             */
    uint64_t n_hits;          /* DONE: number of hits                                    */
    const int64_t* pos_dev;   /* DONE: n_hits positions, ascending (NULL if none); arena */
    const uint16_t* cnt_dev;  /* DONE: their mismatch counts; both valid until release   */
    uint64_t arrival_ns;      /* pm_server_now_ns clock                                  */
    uint64_t admit_ns;
    uint64_t complete_ns;
    uint32_t first_chunk;     /* chunk of its first step                                 */
    uint32_t reruns;          /* chunks re-scanned after an overflow                     */
} pm_query_info;

typedef struct {
    uint64_t steps;           /* chunk steps launched                                    */
    uint64_t submitted, admitted, completed, failed;
    uint64_t reruns;
    uint64_t comparisons;     /* sum over completed queries of (n - m + 1) * m           */
    uint32_t active, waiting; /* now: admitted and not complete; not admitted yet      */
    uint32_t peak_active;     /* most queries in one chunk step (at most max_active)     */
    uint32_t chunks;
    uint64_t hit_slots;       /* hit slots (10 bytes each) in the arena                  */
    uint64_t hit_slots_used, hit_slots_peak;
    uint64_t workspace_bytes;
} pm_server_stats;

/* Monotonic clock of the server, in nanoseconds. */
uint64_t pm_server_now_ns(void);

/* Create a server over the encoded text (text_dev, n bases; it must stay
 * valid and unchanged until pm_server_destroy).  arena_dev/arena_bytes:
 * caller-owned device memory, 256-byte aligned, used for every buffer of the
 * server (at least pm_server_min_arena_bytes).  `stream`: the stream of the
 * chunk steps (a second stream is created for the joins and re-scans; both
 * are at the default priority).  cfg may be NULL. */
uint64_t pm_server_min_arena_bytes(uint64_t n, const pm_server_config* cfg);
pm_status pm_server_create(const void* text_dev, uint64_t n, void* arena_dev, uint64_t arena_bytes,
                           const pm_server_config* cfg, void* stream, pm_server** out);

/* Submit a query: Table 2 codes (host, copied), length m >= 1, k <= 65535.
 * arrival_ns: the time the query arrived on pm_server_now_ns's clock (0 =
 * now); latency is complete_ns - arrival_ns.  Thread-safe. */
pm_status pm_server_submit(pm_server* srv, const uint8_t* codes, uint32_t m, uint32_t k, uint64_t arrival_ns,
                           uint64_t* id_out);

/* State of a query (PM_ERR_NOT_FOUND for an unknown or released id). */
pm_status pm_server_poll(pm_server* srv, uint64_t id, pm_query_info* info);

/* Wait until the query is DONE or FAILED (PM_ERR_BUSY after timeout_ms;
 * timeout_ms < 0 waits without limit). */
pm_status pm_server_wait(pm_server* srv, uint64_t id, int64_t timeout_ms, pm_query_info* info);

/* Hand a DONE or FAILED query's memory back to the server; its pointers are
 * invalid afterwards (the caller must have finished reading them, e.g. by
 * synchronising the stream of its copy).  PM_ERR_BUSY if not finished. */
pm_status pm_server_release(pm_server* srv, uint64_t id);

/* Wait until every submitted query is DONE or FAILED (PM_ERR_BUSY after
 * timeout_ms). */
pm_status pm_server_drain(pm_server* srv, int64_t timeout_ms);

pm_status pm_server_stats_get(pm_server* srv, pm_server_stats* out);

/* Detail of the error that stopped the engine ("" if none). */
const char* pm_server_error_detail(pm_server* srv);

/* Stop the engine: GPU work in flight finishes, queries not DONE become
 * FAILED (PM_ERR_BUSY), and the server is freed (the arena stays the
 * caller's). */
pm_status pm_server_destroy(pm_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* PMSCAN_H */
