/*
 * aceapex.h -- C ABI of the MI355X (gfx950) decoder for absolute-offset LZ77
 * streams (ACEAPEX, arXiv 2606.04268).
 *
 * What is decoded.  Every back-reference of the stream names an absolute
 * byte position of the decoded output rather than a backward distance
 * (Sec. 3.1), so a copy only needs its source bytes to be final.  The output
 * is cut into self-contained blocks of 2^block_log2 bytes (Sec. 3.1).  Each
 * block stores the four streams of Sec. 3.2 -- raw literals lit[], match
 * lengths len[], absolute sources off[], and the command sequence cmd[]
 * (literal-run lengths, one before each match plus a trailing run) -- plus
 * lvl[], the dependency level of every match (Sec. 7.1: 0 when every source
 * byte is a literal, else 1 + the highest level among the matches that wrote
 * its source bytes), and a chunk index that lets a block be split into
 * independently parsed pieces of 2^chunk_log2 sequences.
 *
 * How it is decoded on the GPU.  Literal runs are scattered to their output
 * positions in parallel, then the matches execute level by level: all level-k
 * copies are mutually independent, and level k only reads bytes written by
 * literals or by levels < k (Sec. 7.1, the wavefront schedule of Sec. 7.1 and
 * Sec. 7.4).  The decoder trusts lvl[] for ordering; a stream whose levels
 * violate the definition decodes to unspecified bytes (never out of bounds).
 *
 * Stream layout (all integers little-endian):
 *   header, 64 bytes:
 *      0 char[4] "ACX1"        4 u16 version (1)      6 u16 flags
 *      8 u8 block_log2          9 u8 min_match        10 u8 chunk_log2   11 u8 0
 *     12 u32 max_depth (0 = unlimited)                 16 u64 decoded_bytes
 *     24 u64 comp_bytes (whole stream)                 32 u32 n_blocks
 *     36 u32 max_level         40 u32 n_seq (matches) 44 u32 n_deep (level >= 1)
 *     48 u32 n_chunks          52 u32 0               56 u64 content hash (XXH3-64, 0 = absent)
 *   block table at 64: (n_blocks + 1) x {u64 offset, u32 seq_base, u32 chunk_base};
 *     entry n_blocks is {comp_bytes, n_seq, n_chunks}; offsets are 16-aligned
 *   level table: (max_level + 1) x u32, the number of matches at each level,
 *     zero-padded to a multiple of 16 bytes; the first block starts right after it
 *   block payload: {u32 n_seq, n_lit, n_chunks, max_level, cmd_bytes,
 *     len_bytes, lvl_bytes, 0}, then n_chunks x {u32 cmd_off, len_off,
 *     lvl_off, lit_off, dst_off, 0, 0, 0}, then off[n_seq] (u32), cmd[]
 *     (n_seq + 1 LEB128 runs), len[] (n_seq LEB128 values of length -
 *     min_match), lvl[] (n_seq LEB128), lit[n_lit]; every section zero-padded
 *     to a multiple of 16 bytes.  Every LEB128 value is at most 4 bytes long.
 *   flags: bit0 flattened within blocks (Sec. 3.3), bit1 flattened along
 *     literal-rooted chains only, bit2 depth-limited (Sec. 7.4), bit3 levels
 *     present.  Without bit3 the stream holds the four streams of Sec. 3.2
 *     only: max_level and n_deep are 0, there is no level table (the first
 *     block follows the block table) and every block's lvl[] is empty; the
 *     decoder then derives the levels on the device (aceapex_decode_derive).
 *
 * Conventions.  All pointers named d_* are device pointers on the current HIP
 * device; h_* are host pointers.  The caller owns every buffer.  Calls that
 * take a hip_stream (a hipStream_t, NULL = the null stream) enqueue work and
 * return at once; problems the host can see are returned synchronously,
 * problems found on the device are written to *d_status (0 = success) and
 * are readable after the stream has been synchronised.  When the status is
 * nonzero the output bytes are unspecified, but no write ever leaves
 * [d_out, d_out + decoded_bytes) and no read leaves the compressed buffer or
 * the output.  The library allocates no device memory on these paths.
 *
 * GPU limits of this version: decoded_bytes and comp_bytes below 2^32,
 * 3 <= block_log2 <= 20, chunk_log2 <= 10, min_match >= 1, n_chunks <= 2^24.
 */
#ifndef ACEAPEX_H
#define ACEAPEX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ACEAPEX_OK 0
#define ACEAPEX_E_INVAL -1       /* null pointer, misaligned buffer, bad argument          */
#define ACEAPEX_E_FORMAT -2      /* bad magic / version / flags, inconsistent header       */
#define ACEAPEX_E_CORRUPT -3     /* inconsistency found while parsing (device status)      */
#define ACEAPEX_E_CAPACITY -4    /* out_capacity < decoded_bytes                           */
#define ACEAPEX_E_WORKSPACE -5   /* workspace missing or too small                         */
#define ACEAPEX_E_UNSUPPORTED -6 /* outside the GPU limits listed above                    */
#define ACEAPEX_E_TIMEOUT -7     /* reserved for a device-side wait that hits a spin limit; */
                                 /* no kernel of this version waits on another, so no call  */
                                 /* returns it                                              */
#define ACEAPEX_E_HIP -8         /* HIP runtime error, see aceapex_last_hip_error()        */
#define ACEAPEX_E_NOMEM -9       /* host allocation failed (encoder)                       */

/* Header fields, filled on the host by aceapex_probe from a host copy of the
 * first 64 bytes of the stream. */
typedef struct {
    uint64_t decoded_bytes; /* N: bytes the stream decodes to                       */
    uint64_t comp_bytes;    /* size of the whole compressed stream                  */
    uint32_t n_blocks;      /* ceil(N / 2^block_log2)                               */
    uint32_t block_log2;
    uint32_t min_match;
    uint32_t chunk_log2;
    uint32_t max_depth;     /* encoder depth limit, 0 = unlimited (Sec. 7.4)        */
    uint32_t max_level;     /* highest match level; levels run 0..max_level         */
    uint32_t flags;
    uint32_t n_seq;         /* matches in the stream                                */
    uint32_t n_deep;        /* matches with level >= 1                              */
    uint32_t n_chunks;      /* chunk-index entries over all blocks                  */
    uint64_t content_hash;  /* XXH3-64 of the decoded bytes, 0 if absent            */
} aceapex_info;

/* One compressed stream resident on the device. */
typedef struct {
    const void *d_comp;         /* device, caller-owned, comp_bytes long, 16-byte aligned    */
    aceapex_info info;          /* from aceapex_probe on the same bytes                      */
    const uint32_t *h_levels;   /* host copy of the level table (max_level + 1 counts, from  */
                                /* aceapex_level_table), or NULL.  With it the wavefront is  */
                                /* launched level by level at the size each level needs;     */
                                /* without it every level gets a full-size launch.  Read     */
                                /* during the decode call only.                              */
} aceapex_stream;

/* Per-stream descriptor of the batched call. */
typedef struct {
    aceapex_stream s;
    void *d_out;            /* device, caller-owned, >= out_capacity bytes, 16-byte aligned */
    uint64_t out_capacity;
    int32_t *d_status;      /* device int32 written by the decoder (0 = ok); may be NULL   */
} aceapex_desc;

/* Parse and check the 64-byte header.  Blocks carry no context of their own
 * (Sec. 3.1: any block decodes once the bytes its absolute sources name
 * exist), so the header alone fixes the decode's shape: decoded size, block
 * count and size, and the deepest dependency level (Sec. 7.1) that sets the
 * number of wavefronts.  h_len must be >= 64.  Pure host code.  Returns
 * ACEAPEX_OK, ACEAPEX_E_INVAL (null pointer or h_len < 64) or
 * ACEAPEX_E_FORMAT (bad magic or version, unknown flags, or fields that
 * contradict each other). */
int aceapex_probe(const void *h_stream_prefix, size_t h_len, aceapex_info *info);

/* Copy the stream's level table (the number of matches at each dependency
 * level 0..max_level, Sec. 7.1) from a host copy of the stream prefix of at
 * least 64 + 16 * (n_blocks + 1) + 4 * (max_level + 1) bytes into counts[0, n),
 * n >= max_level + 1.  Pure host code.  Returns ACEAPEX_OK, ACEAPEX_E_INVAL
 * (null pointer, prefix or n too short) or ACEAPEX_E_FORMAT (bad header, or
 * counts that do not add up to n_seq). */
int aceapex_level_table(const void *h_stream_prefix, size_t h_len, uint32_t *counts, uint32_t n);

/* Device workspace, in bytes, that aceapex_decode_many needs for these n
 * descriptors (n = 1 for aceapex_decode): per chunk a 64-byte descriptor of
 * its slices of the Sec. 3.2 streams, per level of Sec. 7.1 three slot
 * counters (n = 1: the fill counter on a 128-byte line of its own), and 12
 * bytes per match for the level-grouped match records
 * (n = 1 and at most 64 levels: also 4 bytes per (level, chunk) for the
 * ordered record slots described at aceapex_decode); for a stream without
 * levels, the workspace of aceapex_decode_derive; with
 * ACEAPEX_VALIDATE_LEVELS set, a stream with levels needs the larger of its
 * own and the derive workspace.  Pure host code; returns 0 when a
 * descriptor's info is inconsistent. */
size_t aceapex_workspace_bytes(const aceapex_desc *h_descs, uint32_t n);

/* Decode one stream into d_out (Sec. 3.2, Sec. 7.1).  d_workspace must hold
 * aceapex_workspace_bytes() for this stream, 256-byte aligned; its contents
 * on entry do not matter.  d_status may be NULL (the status is then kept in
 * the workspace).  Asynchronous on hip_stream.  A host level table
 * (stream->h_levels) whose counts do not add up to n_seq is refused with
 * ACEAPEX_E_FORMAT; one that differs from the stream's own level table makes
 * the device status ACEAPEX_E_CORRUPT.
 *
 * The level launches trust the stored levels for their order.  With the
 * environment variable ACEAPEX_VALIDATE_LEVELS set (to anything but "" or
 * "0", read at each call), this call first checks them on the device: every
 * match's level must exceed the level of each match that writes one of its
 * source bytes (Sec. 7.1); a stream that breaks this gets ACEAPEX_E_CORRUPT.
 * The check costs a derive-mode parse and one pass over the matches, and the
 * larger workspace stated above.  aceapex_decode_many, plans and
 * aceapex_decode_noalloc do not check.
 *
 * Record order.  For a stream of at most 64 levels and at least 4M matches
 * (2^22), each chunk's matches per level are counted and scanned before the
 * parse, so that every level's match records lie in output order, which
 * the level launches copy faster; other streams reserve their records'
 * slots with atomics, in the order the chunks finish.  The environment
 * variable ACEAPEX_ORDERED_SLOTS overrides the size rule for streams of at
 * most 64 levels: "0" never, any other non-empty value always (read at each
 * call of aceapex_decode and aceapex_decode_noalloc, and when a plan is
 * made).  The decoded bytes and the status do not depend on it. */
int aceapex_decode(const aceapex_stream *stream, void *d_out, uint64_t out_capacity,
                   void *d_workspace, size_t ws_bytes, int32_t *d_status, void *hip_stream);

/* Decode one stream, deriving every match's level on the device instead of
 * reading lvl[] (Sec. 7.1: a match's level is 0 when every source byte is a
 * literal, else 1 + the highest level among the matches that wrote its source
 * bytes; the paper computes them on the CPU, Sec. 4.4).  aceapex_decode takes
 * this path for a stream without levels (flag bit3 clear); this call takes it
 * for any stream, ignoring lvl[] and the level table.  The matches run level
 * by level as their levels are found: at level k each waiting match resumes a
 * scan of the writers of its source bytes, parks on the first writer that has
 * not run, or runs when every writer has.  d_levels, when not NULL, receives
 * each match's level in stream order (n_seq u32, 4-byte aligned).  The
 * workspace must hold aceapex_workspace_bytes_derive(&stream->info) bytes,
 * 256-byte aligned.  The number of levels is found on the device: the call
 * reads a queue length back from the device every few levels (synchronising
 * hip_stream) and returns once the last level is enqueued.  Errors as
 * aceapex_decode; a stream whose sources admit no order fails with
 * ACEAPEX_E_CORRUPT in *d_status. */
int aceapex_decode_derive(const aceapex_stream *stream, void *d_out, uint64_t out_capacity, void *d_workspace,
                          size_t ws_bytes, uint32_t *d_levels, int32_t *d_status, void *hip_stream);

/* Workspace of aceapex_decode_derive for a stream with this header (0 when
 * the header is inconsistent).  Pure host code. */
size_t aceapex_workspace_bytes_derive(const aceapex_info *info);

/* Decode n independent streams (Sec. 7.5: blocks and streams are independent)
 * as one batch on hip_stream.  h_descs is a host array; the workspace must
 * hold aceapex_workspace_bytes(h_descs, n).  When every descriptor carries
 * h_levels, the streams run as one launch sequence (one setup, one parse over
 * all their chunks, one launch per level over all their matches); a batch of
 * more than 2048 streams, or whose match, chunk or block counts would
 * overflow the 32-bit indexes of one sequence, runs as several consecutive
 * sequences.  Without the tables the streams are decoded one after the other.
 * Returns the first synchronous error; per-stream device errors go to each
 * d_status.  Streams without stored levels (flags bit 3 clear) are decoded
 * after the others, one by one, with their levels derived on the device as
 * in aceapex_decode_derive; their derivation reads counters back, so a call
 * that holds such a stream returns only once it is decoded.  Host level
 * tables are checked as in aceapex_decode: a table
 * whose counts do not add up to n_seq is refused (ACEAPEX_E_FORMAT), one that
 * differs from the stream's own table fails that stream (ACEAPEX_E_CORRUPT). */
int aceapex_decode_many(const aceapex_desc *h_descs, uint32_t n, void *d_workspace,
                        size_t ws_bytes, void *hip_stream);

/* Decode one stream exactly as aceapex_decode does, with no workspace
 * argument and no allocation of any kind: for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The workspace is a library-static device array of
 * ACEAPEX_NOALLOC_WORKSPACE_MAX bytes that every device the library runs on
 * holds until the process ends; a stream whose aceapex_workspace_bytes
 * exceeds it is refused with ACEAPEX_E_WORKSPACE before anything is
 * enqueued.  The array belongs to the device that is current at the call,
 * which must be the device of hip_stream.  Every call on one device shares
 * that device's array and overwrites what the previous call left there, so
 * calls that overlap on one device (other streams, other host threads) race:
 * the caller must order them.  d_status may be NULL (the status then stays in
 * the array, unreadable).  Asynchronous on hip_stream; returns the synchronous
 * errors of aceapex_decode. */
#define ACEAPEX_NOALLOC_WORKSPACE_MAX ((size_t)64 << 20)
int aceapex_decode_noalloc(const aceapex_stream *stream, void *d_out, uint64_t out_capacity, int32_t *d_status,
                           void *hip_stream);

/* Decode one stream on the host CPU into h_out, for requests a GPU launch
 * serves slower: small streams, and very deep ones whose wavefront pays one
 * level boundary per level (Sec. 7.2 finds such a stream slower on the GPU;
 * Sec. 8.2 suggests choosing the device per input).  Blocks are decoded in
 * parallel by `threads` host threads (0 = all), each block's sequences in
 * order (Sec. 3.2), a copy from an earlier block waiting until that block has
 * published its source bytes (Sec. 3.1: blocks carry no context, sources are
 * absolute).  h_stream is the whole stream (len = comp_bytes); h_out holds at
 * least decoded_bytes.  Synchronous; the lvl[] section and the level table
 * are not used.  Returns ACEAPEX_OK, ACEAPEX_E_INVAL, ACEAPEX_E_FORMAT,
 * ACEAPEX_E_CAPACITY, ACEAPEX_E_UNSUPPORTED, ACEAPEX_E_NOMEM or
 * ACEAPEX_E_CORRUPT (h_out then holds unspecified bytes; no write leaves
 * [h_out, h_out + decoded_bytes)). */
int aceapex_decode_host(const void *h_stream, size_t len, void *h_out, uint64_t out_capacity, uint32_t threads);

/* Static English text for an error code (ACEAPEX_E_* above; "unknown error"
 * for any other value).  Pure host code. */
const char *aceapex_strerror(int code);

/* The last hipError_t seen by a call that returned ACEAPEX_E_HIP (0 if none). */
int aceapex_last_hip_error(void);

/* ------------------------------------------------------------ measurement */

/* Kernel timing, for benchmarks.  aceapex_timing(1) clears the record and
 * makes every following decode on the calling host thread bracket each of
 * its kernels with HIP events on the decode's stream; aceapex_timing(0)
 * stops recording.  Groups: 0 setup (block and chunk-index checks, level
 * offsets), 1 parse (LEB128 decode, literal scatter, match records by
 * level), 2 levels (the match wavefront).  The set of kernels a decode
 * launches is an implementation detail and may change between versions. */
int aceapex_timing(int enable);

/* Wait for the last recorded event, then write, for groups 0..n-1, the summed
 * duration in milliseconds (ms[i]) and the number of recorded decodes that
 * launched the group (count[i]); clears the record.  Returns ACEAPEX_OK,
 * ACEAPEX_E_INVAL or ACEAPEX_E_HIP. */
int aceapex_timing_read(float *ms, uint32_t *count, uint32_t n);

/* ---------------------------------------------------- plans (batched mode) */

/* A plan lays a batch out once and launches it many times (Sec. 7.5: the
 * streams of a batch are independent).  aceapex_plan_create checks the
 * descriptors as aceapex_decode_many does -- every descriptor must carry
 * h_levels -- and writes the batch's host-side tables into the workspace
 * (synchronously, on hip_stream); the level counts are copied, so h_levels
 * need not outlive the call.  A launch then only enqueues kernels: no
 * host-to-device copy, no allocation and no memset, so aceapex_plan_launch
 * may be captured into the caller's HIP graph, and aceapex_plan_launch_graph
 * captures the sequence once into a graph of its own and replays it.
 *
 * Ownership: the plan is host memory of the library until
 * aceapex_plan_destroy.  The compressed inputs, outputs, status words and
 * the workspace stay the caller's; they must stay allocated, and the
 * workspace untouched by anything else, while the plan lives.  Launches of
 * one plan must not overlap (they share the workspace), and run on the
 * device that was current at creation.  Each launch decodes every stream
 * again and rewrites each status word. */
typedef struct aceapex_plan aceapex_plan;

/* Schedule of the level phase (Sec. 7.1 wavefront).  Any values in range give
 * the same bytes; they only change the speed. */
typedef struct {
    uint32_t level_wg_max;   /* workgroups of one level launch, at most (1..65535; default 512)     */
    uint32_t tail_level_max; /* the deepest levels, while each holds at most this many matches, run  */
                             /* together in one workgroup (default 2048; 0 = one launch per level)   */
    uint32_t long_copy;      /* matches longer than this are copied by a whole wave (16..2^21; 128)  */
    uint32_t xcd_parts;      /* contiguous parts of a level's matches, one per XCD (1..8; default 8) */
} aceapex_tuning;

/* The default schedule (the one aceapex_decode and aceapex_decode_many use). */
void aceapex_tuning_defaults(aceapex_tuning *t);

/* Create a plan for h_descs[0, n) with workspace d_workspace (at least
 * aceapex_workspace_bytes(h_descs, n), 256-byte aligned).  tuning may be NULL
 * (defaults).  Returns ACEAPEX_OK, ACEAPEX_E_INVAL (null plan, a descriptor
 * without h_levels, a tuning value out of range), the argument errors of
 * aceapex_decode_many, ACEAPEX_E_NOMEM or ACEAPEX_E_HIP. */
int aceapex_plan_create(const aceapex_desc *h_descs, uint32_t n, void *d_workspace, size_t ws_bytes,
                        const aceapex_tuning *tuning, void *hip_stream, aceapex_plan **plan);

/* Enqueue one decode of every stream of the plan on hip_stream (kernel
 * launches only).  Returns ACEAPEX_OK, ACEAPEX_E_INVAL or ACEAPEX_E_HIP. */
int aceapex_plan_launch(aceapex_plan *plan, void *hip_stream);

/* As aceapex_plan_launch, through a HIP graph captured (on a private stream
 * of default priority) at the first call after creation or a tuning change. */
int aceapex_plan_launch_graph(aceapex_plan *plan, void *hip_stream);

/* Replace / read the plan's schedule (a change drops the captured graph). */
int aceapex_plan_set_tuning(aceapex_plan *plan, const aceapex_tuning *tuning);
int aceapex_plan_get_tuning(const aceapex_plan *plan, aceapex_tuning *tuning);

/* Autotune the schedule on this plan's own streams: coordinate descent over
 * level_wg_max, tail_level_max, long_copy and xcd_parts, each candidate timed
 * with HIP events over reps launches after one warm-up; a candidate is kept
 * when it is at least 1% faster.  The plan keeps the winner, also written to
 * *best when best is not NULL.  Synchronous; runs about 16 * (reps + 1)
 * decodes of the batch, each leaving the outputs decoded. */
int aceapex_plan_tune(aceapex_plan *plan, void *hip_stream, uint32_t reps, aceapex_tuning *best);

/* Free the plan (NULL is ignored).  Call it once no launch is in flight. */
void aceapex_plan_destroy(aceapex_plan *plan);

/* ------------------------------------------------------------ verification */

/* Compare two device buffers of n bytes on the GPU (the decode must give back
 * its input byte for byte, Sec. 4.3): d_result[0] receives the number of
 * differing bytes and d_result[1] the index of the first one (n when none).
 * d_result is a device pointer to two u64, 8-byte aligned, written by the
 * call's own kernels (no memset).  Asynchronous on hip_stream; read d_result
 * after synchronizing.  Returns ACEAPEX_OK, ACEAPEX_E_INVAL (null pointers,
 * misaligned result) or ACEAPEX_E_HIP. */
int aceapex_compare(const void *d_a, const void *d_b, uint64_t n, uint64_t *d_result, void *hip_stream);

/* ---------------------------------------------- entropy stage (literals) */

/* tANS-coded byte buffers, the entropy stage the paper names for its streams
 * and leaves to future work (Sec. 4.4, Sec. 8).  A container ("ACT1") holds
 * the normalized counts of its bytes (summing to 2^table_log) and `lanes`
 * independent lanes: byte i belongs to lane i mod lanes, so one GPU thread
 * decodes one lane and a wave writes 64 consecutive bytes per step.  Layout:
 *   0 "ACT1", 4 u32 n, 8 u32 table_log (8..12), 12 u32 lanes,
 *   16 u64 container bytes, 24 u32 bitstream bytes, 28 u32 0,
 *   32 u16 counts[256], 544 lanes x {u32 end bit, u32 initial state},
 *   then the lanes' bits (LSB-first, each lane from the previous one's end
 *   bit) and 8 zero bytes.
 * Coding: the i-th table entry in symbol order sits at position (i * step)
 * mod 2^R, step = 2^R/2 + 2^R/8 + 3; each symbol's positions, in increasing
 * order, carry state values c_s .. 2 c_s - 1; a decoder in state x reads
 * position x - 2^R, outputs its symbol and moves to (y << nb) + the next nb
 * bits, nb = R - floor(log2 y), reading its lane from the end. */
typedef struct {
    uint64_t n;               /* decoded bytes                        */
    uint64_t container_bytes;
    uint32_t table_log;
    uint32_t lanes;
    uint32_t bitstream_bytes;
} aceapex_tans_info;

/* Parse and check a container's header and counts from a host copy of its
 * first 544 bytes.  Pure host code.  Returns ACEAPEX_OK, ACEAPEX_E_INVAL or
 * ACEAPEX_E_FORMAT. */
int aceapex_tans_probe(const void *h_prefix, size_t h_len, aceapex_tans_info *info);

/* Device workspace of aceapex_tans_decode (the decode table). */
size_t aceapex_tans_workspace_bytes(const aceapex_tans_info *info);

/* Decode a device-resident container (d_in, 8-byte aligned, container_bytes
 * long) into d_out (n bytes).  The workspace (aceapex_tans_workspace_bytes,
 * 256-byte aligned) holds the decode table, built on the device from the
 * counts.  *d_status (required) becomes 0, or ACEAPEX_E_CORRUPT when a lane's
 * bits or states are inconsistent; no write leaves [d_out, d_out + n) and no
 * read leaves the container.  Asynchronous on hip_stream. */
int aceapex_tans_decode(const void *d_in, const aceapex_tans_info *info, void *d_out, uint64_t out_capacity,
                        void *d_workspace, size_t ws_bytes, int32_t *d_status, void *hip_stream);

/* Encode h_in[0, n) (host) into a container with 2^table_log table entries
 * and `lanes` lanes; *h_out receives a malloc'd buffer (release with
 * aceapex_free) and the container length is returned, or a negative
 * ACEAPEX_E_* code.  Pure host code (threads over lanes). */
int64_t aceapex_tans_encode(const void *h_in, uint64_t n, uint32_t table_log, uint32_t lanes, void **h_out);

/* ------------------------------------------------------------ host encoder */

/* Encoder parameters.  The parse is greedy over hash chains of 4-byte
 * hashes; its back-references are absolute output positions (Sec. 3.1). */
typedef struct {
    uint32_t block_log2;  /* self-contained blocks of 2^block_log2 bytes (paper: 1 MB = 20)      */
    uint32_t min_match;   /* shortest match, >= 4                                                 */
    uint32_t flatten;     /* Sec. 3.3 chain flattening: 0 off; 1 trace every match byte back      */
                          /* through earlier copies of its block to a literal or to the first     */
                          /* position outside the block; 2 only along chains that end at a        */
                          /* literal of the block                                                 */
    uint32_t max_depth;   /* Sec. 7.4 depth limit D: every match level <= D - 1; 0 = unlimited   */
    uint32_t chain_depth; /* hash-chain candidates examined per position (32)                     */
    uint32_t hash_bits;   /* log2 of the hash table (22)                                          */
    uint32_t tiebreak;    /* among candidates of equal length: 0 lowest level, 1 most recent      */
    uint32_t chunk_log2;  /* sequences per chunk-index entry (10)                                 */
    uint32_t threads;     /* host threads, 0 = all                                                */
    uint32_t verbose;     /* nonzero: the in-order pass reports its progress on stderr every 64  */
                          /* blocks                                                               */
    uint32_t levels;      /* 1: store lvl[] and the level table (1); 0: the four streams of       */
                          /* Sec. 3.2 only, levels derived by the decoder                          */
} aceapex_enc_opts;

/* Fill *o with the defaults above.  Pure host code. */
void aceapex_enc_defaults(aceapex_enc_opts *o);

/* Encode h_in[0, n) (host memory) into a stream in the layout above, with
 * content hash 0.  On success *h_stream points to a malloc'd buffer owned by
 * the caller (release with aceapex_free) and the stream length is returned;
 * on failure a negative ACEAPEX_E_* code is returned and *h_stream is NULL.
 * Pure host code; n must be below 2^32. */
int64_t aceapex_encode(const void *h_in, uint64_t n, const aceapex_enc_opts *opts, void **h_stream);

/* Release a buffer returned by aceapex_encode. */
void aceapex_free(void *h_stream);

#ifdef __cplusplus
}
#endif

#endif /* ACEAPEX_H */
