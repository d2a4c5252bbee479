// MI355X (gfx950) decoder for absolute-offset LZ77 streams (ACEAPEX,
// arXiv 2606.04268) behind the C ABI of include/aceapex.h.
//
// One stream or a batch of independent streams (Sec. 7.5) is decoded by a
// short sequence of launches on the caller's stream, with no host round trip:
//
//   k_map     (batches) global block and chunk indices -> stream
//   k_setup   one workgroup per block checks the block table, block header and
//             chunk index and writes a 64-byte descriptor per chunk (absolute
//             slices of cmd/len/lvl/lit/off and the output span).  The first
//             workgroups also clear each stream's status and level cursors;
//             for a single stream, workgroup 0 turns the stream's level table
//             (matches per level) into the record slots of every level.
//   k_parse   one workgroup per chunk, four sequences per thread.  The chunk's
//             literal bytes are first copied into LDS by direct global-to-LDS
//             loads.  When every cmd/len/lvl value of the chunk is one byte
//             long (the slice length equals the value count) each thread reads
//             its four values with a single 4-byte load per stream; otherwise
//             three waves decode the LEB128 slices into LDS.  A workgroup scan
//             turns run and match lengths into output and literal offsets.
//             The literal runs are placed, as whole aligned words, in an LDS
//             image of the chunk's output span, which is written with aligned
//             16-byte stores (Sec. 3.2); every match becomes a 12-byte record
//             (dst, src, len | stream << 21) in the slots of its level (on
//             deep streams grouped by level in LDS first).
//   k_count, k_otiles, k_oapply  (large single streams of at most 64 levels,
//             before k_parse) count each chunk's matches per level and scan
//             the counts, so that k_parse places every level's records in
//             output order instead of taking their slots with atomics.
//   k_seal    (batches) record slots a corrupt stream left unfilled get length 0.
//   k_level   one launch per level k (Sec. 7.1): the copies of level k read
//             only bytes written by literals or by lower levels and are
//             independent of each other, so every thread runs one record per
//             round (two on levels larger than the launch).  Launch
//             boundaries order the levels.
//   k_tail    the deep levels that hold few matches run in a single workgroup,
//             level after level, separated by workgroup barriers: one CU, so
//             no cache maintenance between levels.
//
// k_parse, k_level and k_tail are compiled for one stream, whose output, size
// and status are kernel arguments, and for batches, where each chunk and
// record names its stream (k_parse also in three LDS shapes by the deepest
// level, and once more for ordered slots).  A plan (aceapex_plan_*) lays a batch out
// once and replays the same launches, optionally as a captured HIP graph.
//
// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// their index; k_level hands each XCD one contiguous range of a level's
// records so that neighbouring work shares an L2.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "aceapex.h"
#include "internal.h"

using aceapex_impl::has_table;
using aceapex_impl::info_consistent;
using aceapex_impl::prefix_bytes;

namespace {

constexpr int NT = 256;                     // threads per workgroup
constexpr int NT_TAIL = 512;                // threads of the tail workgroup
constexpr uint32_t TAIL_RANGES = 8192;      // tail levels whose slot ranges k_tail keeps in LDS
constexpr uint32_t K_LOG2_MAX = 10;         // sequences per chunk, at most
constexpr uint32_t K_MAX = 1u << K_LOG2_MAX;
constexpr uint32_t PER = K_MAX / NT;        // sequences per thread in k_parse
constexpr uint32_t HDR = 64, BLKHDR = 32, CHUNK_ENT = 32;
constexpr uint32_t BLOCK_LOG2_MAX = 20;
constexpr uint32_t LEN_BITS = 21;           // a match length needs 21 bits (blocks of at most 2^20 bytes)
constexpr uint32_t LEN_MASK = (1u << LEN_BITS) - 1;
constexpr uint32_t JOBS_MAX = 1u << (32 - LEN_BITS);  // streams per launch sequence
constexpr uint32_t ROUND_LEVEL = 2;         // records per thread per round of k_level on levels beyond one per thread
constexpr uint32_t ROUND_TAIL = 4;          // records per thread per round of k_tail
// Default schedule (each value can be changed per plan, see aceapex_tuning):
constexpr uint32_t LONG_COPY = 128;         // matches longer than this are copied by a whole wave
constexpr uint32_t LEVEL_WG_MAX = 512;      // workgroups of one level launch, at most
constexpr uint32_t TAIL_LEVEL_MAX = 2048;   // levels with at most this many matches may join the tail
constexpr uint32_t XCD_PARTS = 8;           // contiguous parts of a level's records, one per XCD
constexpr uint32_t TILE_BYTES = 16384;      // output span of a chunk assembled in LDS by k_parse
constexpr uint64_t CHUNKS_MAX = 1ull << 24;  // chunks of one launch sequence (the k_parse grid), at most
constexpr uint32_t COOP_RUNS = 8;          // k_parse: longer literal runs of a wave slot placed by the whole wave
constexpr uint32_t LEVEL_WG1 = 64;          // k_level with one record per thread: workgroup size (one wave)

typedef uint16_t u16u __attribute__((aligned(1)));
typedef uint32_t u32u __attribute__((aligned(1)));
typedef uint64_t u64u __attribute__((aligned(1)));
struct __attribute__((aligned(1))) u128u { uint32_t a, b, c, d; };

struct ChunkDesc {
    uint32_t out_base, out_len;   // output span of the chunk, relative to its stream's output
    uint32_t cmd_at, cmd_n;       // byte slices inside the compressed stream
    uint32_t len_at, len_n;
    uint32_t lvl_at, lvl_n;
    uint32_t lit_at, lit_n;
    uint32_t off_at;              // first off[] entry of the chunk
    uint32_t nseq_last;           // sequences in the chunk | (1 << 31) if it holds the trailing run
    uint32_t seq0;                // index of the chunk's first match in its stream
    uint32_t pad[3];
};
static_assert(sizeof(ChunkDesc) == 64, "descriptor layout");

// One stream as the kernels see it.
struct Job {
    const uint8_t *comp;
    uint8_t *out;
    int32_t *status;
    ChunkDesc *chunks;   // [n_chunks]
    uint8_t *blk_ok;     // [n_blocks] 1 when the block passed the checks of k_setup
    uint32_t n, comp_bytes;
    uint32_t n_blocks, block_log2, min_match, chunk_log2;
    uint32_t max_level, n_chunks, n_seq;
    uint32_t c0, b0;     // first global chunk and block of the stream in its batch
    uint32_t lv0;        // first entry of the stream in the per-(stream, level) arrays
    uint32_t table;      // 1: the stream stores lvl[] and a level table; 0: the four streams of Sec. 3.2 only
    uint32_t derive;     // 1: levels derived on the device (records in stream order, single stream only)
    uint32_t validate;   // 1: the stored levels are being checked (derive pass), or were (decode keeps the verdict)
};

// A decode: one stream (jobs == nullptr) or a batch of streams.
struct Batch {
    Job one;                    // the stream of a single-stream decode
    const Job *jobs;            // device table of a batched decode, or nullptr
    uint32_t *blk_job;          // [n_blocks] global block -> stream (batched)
    uint32_t *chunk_job;        // [n_chunks] global chunk -> stream (batched)
    const ChunkDesc *chunks_all;  // batched: every stream's chunk descriptors, by global chunk
    uint32_t *rec_lo, *rec_hi;  // per (stream, level): record slots [rec_lo, rec_hi)
    uint32_t *cursor;           // per (stream, level): next free slot
    const uint32_t *level_lo;   // [max_level + 2] slots of each level over the batch (batched)
    uint32_t *recs;             // 3 u32 per match: dst, src, len | stream << LEN_BITS
    uint32_t n_jobs, n_blocks, n_chunks, max_level;  // totals over the batch, highest level
    uint32_t n_seq;             // matches over the batch
    uint32_t long_copy;         // matches longer than this are copied by a whole wave
    uint32_t xcd_parts;         // k_level: contiguous parts of a level's records (1..8)
    uint32_t has_sig;           // single stream: the host scheduled the levels from a table
    uint64_t level_sig;         //   whose signature (level_signature) is this
    // ordered record slots (single stream, at most ORD_LEVELS levels): per
    // (level, chunk) the count of its matches, then its first slot
    uint32_t ordered;
    uint32_t *ocnt;             // [levels * n_chunks], level-major
    uint32_t *otile;            // [tiles] sums of OTILE elements of ocnt, then their offsets
    // levels derived on the device (single stream): per match, in stream order
    uint32_t *dlevel;           // level once run, NONE before
    uint32_t *dhead, *dnext;    // matches parked on a match (linked list through dnext)
    uint32_t *dcur, *dmax;      // where the scan of its source resumes, 1 + highest level seen
    uint32_t *dq[2];            // matches to scan at the next level (two, by level parity)
    uint32_t *dready;           // matches found ready at this level
    uint32_t *dpage;            // per 2^PAGE_LOG2 output bytes: first match whose dst is at or past it
    uint32_t *dcnt;             // counters (DC_*)
};

// The arguments of a level launch: what k_level reads of a Batch, under the
// same member names, so that its launch carries a small kernel-argument
// block (a launch per level; measured faster than passing the whole Batch).
struct LevelArgs {
    struct {
        uint8_t *out;
        int32_t *status;
        uint32_t n, max_level;
    } one;                      // the stream of a single-stream decode
    const Job *jobs;            // batched: the stream table, or nullptr
    uint32_t *recs;
    const uint32_t *rec_lo, *rec_hi, *cursor, *level_lo;
    uint32_t n_jobs, long_copy, xcd_parts;
};

constexpr uint32_t NONE = 0xffffffffu;
constexpr uint32_t PAGE_LOG2 = 5;  // derive: output bytes per page-index entry, log2
constexpr uint32_t NO_SLOT = 0xffffffffu;  // k_parse: a level whose slots ran out
constexpr uint32_t CUR_STRIDE = 32;  // single stream: words per level cursor (one 128-byte line each)
constexpr uint32_t ORD_LEVELS = 64;          // single streams with at most this many levels get ordered slots
constexpr uint64_t ORD_MIN_SEQ = 1ull << 22;  // ... and at least this many matches (unless asked for)
constexpr uint32_t OTILE = 4096;             // elements of ocnt per tile of its scan

// counters of the derive path
constexpr uint32_t DC_Q = 0;      // [2] matches queued to scan, by level parity
constexpr uint32_t DC_READY = 2;  // [2] matches ready, by level parity
constexpr uint32_t DC_DONE = 4;   // matches run
constexpr uint32_t DC_LEVELS = 5; // levels run (highest level + 1)
constexpr uint32_t DC_N = 8;
constexpr uint32_t NO_RANGE = 0xffffffffu;  // k_level: read the level's slot range on the device

// Signature of a level table: the sum over levels k of a 64-bit mix of
// (k, count_k) (the SplitMix64 finalizer).  The single-stream decode sizes its
// level launches from the caller's host copy of the table and the device
// builds the record slots from the stream's own table; k_setup compares the
// two signatures so that a stale host table fails the decode instead of
// skipping a level.
__host__ __device__ __forceinline__ uint64_t level_mix(uint32_t k, uint32_t c)
{
    uint64_t z = (((uint64_t)k << 32) | c) + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ const Job &job_of(const Batch &B, uint32_t s) { return B.jobs ? B.jobs[s] : B.one; }

__device__ __forceinline__ uint32_t ld32(const uint8_t *p) { return *(const u32u *)p; }
__device__ __forceinline__ uint64_t ld64(const uint8_t *p) { return *(const u64u *)p; }
__device__ __forceinline__ uint64_t pad16(uint64_t v) { return (v + 15) & ~(uint64_t)15; }

__device__ __forceinline__ void fail(const Job &j, int code) { atomicCAS(j.status, 0, code); }

// Copy n bytes between non-overlapping ranges with unaligned 16/8/4/2/1-byte
// accesses; every access touches exactly the bytes of the copy.
__device__ __forceinline__ void copy_bytes(uint8_t *d, const uint8_t *s, uint32_t n)
{
    while (n >= 16) {
        u128u v = *(const u128u *)s;
        *(u128u *)d = v;
        d += 16; s += 16; n -= 16;
    }
    if (n & 8) { u64u v = *(const u64u *)s; *(u64u *)d = v; d += 8; s += 8; }
    if (n & 4) { u32u v = *(const u32u *)s; *(u32u *)d = v; d += 4; s += 4; }
    if (n & 2) { u16u v = *(const u16u *)s; *(u16u *)d = v; d += 2; s += 2; }
    if (n & 1) *d = *s;
}

// Store the first n (1..16) bytes of lo:hi at d with at most two unaligned
// stores that touch exactly those bytes: a head and a tail of the same width
// that overlap when n is not a power of two (both carry the bytes' own
// values), so that every length from 4 to 16 costs one or two requests.
__device__ __forceinline__ void store_upto16(uint8_t *d, uint64_t lo, uint64_t hi, uint32_t n)
{
    if (n >= 8) {
        if (n == 16) {
            u128u v;
            v.a = (uint32_t)lo; v.b = (uint32_t)(lo >> 32); v.c = (uint32_t)hi; v.d = (uint32_t)(hi >> 32);
            *(u128u *)d = v;
            return;
        }
        const uint32_t k = 8 * (n - 8);  // bits of lo:hi below the tail
        const uint64_t tail = k ? (lo >> k) | (hi << (64 - k)) : lo;
        *(u64u *)d = lo;
        *(u64u *)(d + n - 8) = tail;
    } else if (n >= 4) {
        *(u32u *)d = (uint32_t)lo;
        *(u32u *)(d + n - 4) = (uint32_t)(lo >> (8 * (n - 4)));
    } else if (n >= 2) {
        *(u16u *)d = (uint16_t)lo;
        *(u16u *)(d + n - 2) = (uint16_t)(lo >> (8 * (n - 2)));
    } else {
        *d = (uint8_t)lo;
    }
}

// Whole-wave copy of one long range: lane i moves the 16-byte pieces i, i+64, ...
__device__ __forceinline__ void wave_copy(uint8_t *d, const uint8_t *s, uint32_t n)
{
    const uint32_t lane = threadIdx.x & 63;
    for (uint32_t o = lane * 16; o < n; o += 64 * 16) copy_bytes(d + o, s + o, min(16u, n - o));
}

// Run up to R match records held by this thread, each into its own
// stream's output ob[u] of on[u] bytes.  Matches of at most 16 bytes take one
// 16-byte load of their source (when 16 bytes are there to read: bytes past
// the match are read and discarded) and exact stores; all loads of the round
// are issued before the stores.  Matches up to long_copy bytes are copied by
// their own lane; longer ones are then copied by the whole wave, one at a time.
// run_loads issues the source loads (and rejects records that do not fit);
// run_stores does the rest, so that other loads may be issued in between.
template <uint32_t R>
__device__ __forceinline__ void run_loads(const uint32_t *on, int32_t *const *sp, uint8_t *const *ob,
                                          const uint32_t *dst, const uint32_t *src, uint32_t *len,
                                          uint64_t *lo, uint64_t *hi)
{
#pragma unroll
    for (uint32_t u = 0; u < R; u++) {
        if (len[u] && ((uint64_t)dst[u] + len[u] > on[u] || (uint64_t)src[u] + len[u] > dst[u])) {
            atomicCAS(sp[u], 0, ACEAPEX_E_CORRUPT);
            len[u] = 0;
        }
        const bool small = len[u] && len[u] <= 16 && (uint64_t)src[u] + 16 <= on[u];
        lo[u] = 0; hi[u] = 0;
        if (small) {
            const u128u v = *(const u128u *)(ob[u] + src[u]);
            lo[u] = ((uint64_t)v.b << 32) | v.a;
            hi[u] = ((uint64_t)v.d << 32) | v.c;
        }
    }
}

template <uint32_t R>
__device__ __forceinline__ void run_stores(uint8_t *const *ob, const uint32_t *on, const uint32_t *dst,
                                           const uint32_t *src, const uint32_t *len, const uint64_t *lo,
                                           const uint64_t *hi, uint32_t long_copy)
{
#pragma unroll
    for (uint32_t u = 0; u < R; u++) {
        if (!len[u]) continue;
        if (len[u] <= 16 && (uint64_t)src[u] + 16 <= on[u]) {
            store_upto16(ob[u] + dst[u], lo[u], hi[u], len[u]);
        } else if (len[u] <= long_copy) {
            copy_bytes(ob[u] + dst[u], ob[u] + src[u], len[u]);
        }
    }
#pragma unroll
    for (uint32_t u = 0; u < R; u++) {
        uint64_t m = __ballot(len[u] > long_copy);
        while (m) {
            const int lane = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const uint32_t d0 = __shfl(dst[u], lane, 64), s0 = __shfl(src[u], lane, 64);
            const uint32_t n0 = __shfl(len[u], lane, 64);
            uint8_t *o = (uint8_t *)__shfl((unsigned long long)(uintptr_t)ob[u], lane, 64);
            wave_copy(o + d0, o + s0, n0);
        }
    }
}

template <uint32_t R>
__device__ __forceinline__ void run_records(uint8_t *const *ob, const uint32_t *on, int32_t *const *sp,
                                            const uint32_t *dst, const uint32_t *src, uint32_t *len,
                                            uint32_t long_copy)
{
    uint64_t lo[R], hi[R];
    run_loads<R>(on, sp, ob, dst, src, len, lo, hi);
    run_stores<R>(ob, on, dst, src, len, lo, hi, long_copy);
}

// Slots [lo, hi) of level k: in a single-stream decode the filled part of the
// level; in a batch the level's slots over all streams (unfilled slots are
// rejected record by record).
template <class A>
__device__ __forceinline__ void level_range(const A &B, uint32_t k, uint32_t &lo, uint32_t &hi)
{
    if (B.jobs) {
        lo = B.level_lo[k];
        hi = B.level_lo[k + 1];
    } else {
        lo = B.rec_lo[k];
        hi = min(B.cursor[(size_t)k * CUR_STRIDE], B.rec_hi[k]);
    }
}

// Raw words of the records r0 + u*stride (u < R), without waiting
// between them; a slot at or past r_end gets lj = 0 (no match).
template <uint32_t R, class A>
__device__ __forceinline__ void fetch_records(const A &B, uint32_t r0, uint32_t stride, uint32_t r_end,
                                              uint32_t *dst, uint32_t *src, uint32_t *lj)
{
#pragma unroll
    for (uint32_t u = 0; u < R; u++) {
        const uint32_t i = r0 + u * stride;
        const bool ok = i < r_end;
        const uint32_t *r = B.recs + 3ull * (ok ? i : r0);
        dst[u] = r[0];
        src[u] = r[1];
        lj[u] = ok ? r[2] : 0u;
    }
}

// The stream of each fetched record: its output, size and status.  In a
// batch every slot of a level was filled in this decode or given length 0 by
// k_seal, so the stream index carried by the record is all that is needed.
template <bool BATCH, uint32_t R, class A>
__device__ __forceinline__ void resolve_records(const A &B, const uint32_t *lj, uint8_t **ob, uint32_t *on,
                                                int32_t **sp, uint32_t *len)
{
#pragma unroll
    for (uint32_t u = 0; u < R; u++) {
        len[u] = lj[u] & LEN_MASK;
        if (!BATCH) {
            ob[u] = B.one.out;
            on[u] = B.one.n;
            sp[u] = B.one.status;
        } else {
            const uint32_t s = lj[u] >> LEN_BITS;
            ob[u] = nullptr;
            on[u] = 0;
            sp[u] = nullptr;
            if (len[u] && s < B.n_jobs) {
                const Job &j = B.jobs[s];
                ob[u] = j.out;
                on[u] = j.n;
                sp[u] = j.status;
            }
            if (!ob[u]) len[u] = 0;
        }
    }
}

// Fetch and resolve R records (see fetch_records, resolve_records).
template <bool BATCH, uint32_t R, class A>
__device__ __forceinline__ void load_records(const A &B, uint32_t r0, uint32_t stride,
                                             uint32_t r_end, uint8_t **ob, uint32_t *on, int32_t **sp,
                                             uint32_t *dst, uint32_t *src, uint32_t *len)
{
    uint32_t lj[R];
    fetch_records<R>(B, r0, stride, r_end, dst, src, lj);
    resolve_records<BATCH, R>(B, lj, ob, on, sp, len);
}

// ------------------------------------------------------------------- scans

// DPP moves of one 64-bit value (two 32-bit halves); lanes the control word
// leaves without a source, or disables by row_mask, read 0.
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ uint64_t dpp64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROW_MASK, 0xf, BOUND_ZERO);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROW_MASK, 0xf, BOUND_ZERO);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive scan over the 64 lanes of a wave with DPP moves only (no LDS):
// row_shr 1, 2, 4, 8 scan each row of 16 lanes, then row_bcast 15 and 31 add
// the totals of the rows below.
__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t x)
{
    x += dpp64<0x111, 0xf, true>(x);  // row_shr:1
    x += dpp64<0x112, 0xf, true>(x);  // row_shr:2
    x += dpp64<0x114, 0xf, true>(x);  // row_shr:4
    x += dpp64<0x118, 0xf, true>(x);  // row_shr:8
    x += dpp64<0x142, 0xa, false>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp64<0x143, 0xc, false>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

// exclusive scan of one u64 per thread over the workgroup; tmp holds NT/64 u64
__device__ uint64_t wg_excl_scan64(uint64_t v, uint64_t *tmp, uint64_t &total)
{
    const int wid = threadIdx.x >> 6;
    uint64_t x = wave_incl_scan64(v);
    if ((threadIdx.x & 63) == 63) tmp[wid] = x;
    __syncthreads();
    uint64_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) {
        uint64_t t = tmp[w];
        before += (w < wid) ? t : 0;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return before + x - v;
}

// DPP control word of a whole-wave shift by one lane: lane i reads lane i-1,
// and lane 0 keeps the old value.
constexpr int DPP_WAVE_SHR1 = 0x138;

// One wave decodes exactly cnt LEB128 values (at most 4 bytes each) from the
// global bytes p[0, nb) into vals[0, cnt); p[0, avail) may be read.  Lane i
// holds bytes 4i..4i+3 of each 256-byte window, all loaded before any is
// decoded.  A value ends at a byte below 0x80.  Values ending in lanes below
// are counted with one ballot per byte position (no cross-lane scan), and
// each value is assembled without branches from the 8 bytes made of the
// lane's dword and its left neighbour's (one DPP move): it starts after the
// last end byte among the three bytes before its own end byte.  Returns true
// (uniformly) iff the slice holds exactly cnt well-formed values.
__device__ __forceinline__ bool wave_varints(const uint8_t *p, uint32_t nb, uint32_t avail, uint32_t cnt,
                                             uint32_t *vals)
{
    constexpr uint32_t WINDOWS = (4 * (K_MAX + 1) + 255) / 256;  // the longest slice a chunk may hold
    constexpr uint32_t WPRE = 8;  // windows loaded up front; later ones (slices over 2 KiB) when decoded
    const uint32_t lane = threadIdx.x & 63;
    auto load = [&](uint32_t i) {
        const uint32_t o = 256 * i + 4 * lane;
        uint32_t x = 0x80808080u;  // bytes past the slice: continuation, never a value end
        if (o < nb) {
            if (o + 4 <= avail) {
                x = ld32(p + o);
            } else {  // the last bytes of the stream
                x = 0;
                for (uint32_t k = 0; k < 4; k++)
                    if (o + k < avail) x |= (uint32_t)p[o + k] << (8 * k);
            }
            if (o + 4 > nb) {
                const uint32_t keep = (1u << (8 * (nb - o))) - 1;
                x = (x & keep) | (0x80808080u & ~keep);
            }
        }
        return x;
    };
    uint32_t v[WPRE];
#pragma unroll
    for (uint32_t i = 0; i < WPRE; i++) v[i] = load(i);
    uint32_t prev_last = 0;  // dword left of the window; zero bytes end any value before the slice
    uint32_t base = 0;
    bool ok = nb <= 256 * WINDOWS;
    const uint32_t last = nb - 1;  // the slice's last byte must end a value
#pragma unroll
    for (uint32_t i = 0; i < WINDOWS; i++) {
        if (256 * i >= nb) break;  // (uniform) past the slice
        const uint32_t x = i < WPRE ? v[i] : load(i);
        const uint32_t o = 256 * i + 4 * lane;
        const uint32_t pv = (uint32_t)__builtin_amdgcn_update_dpp((int)prev_last, (int)x, DPP_WAVE_SHR1, 0xf, 0xf, false);
        const uint32_t term = ~x & 0x80808080u;
        uint32_t idx = base, tot = 0;
#pragma unroll
        for (uint32_t k = 0; k < 4; k++) {
            const uint64_t m = __ballot(term & (0x80u << (8 * k)));
            idx += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            tot += (uint32_t)__popcll(m);
        }
        if (o <= last && last < o + 4 && ((x >> (8 * (last - o) + 7)) & 1)) ok = false;
#pragma unroll
        for (uint32_t k = 0; k < 4; k++) {
            // bytes k+1 .. k+4 of the window pv:x; the top one (byte k of x) ends the value
            const uint32_t y4 = k == 3 ? x : __builtin_amdgcn_alignbyte(x, pv, k + 1);
            const uint32_t ends = ~y4 & 0x00808080u;  // end bytes among the three before it
            const uint32_t y = y4 >> (32 - __clz(ends));  // the value's bytes, first one lowest
            const uint32_t val = (y & 0x7fu) | ((y >> 1) & 0x3f80u) | ((y >> 2) & 0x1fc000u) | ((y >> 3) & 0xfe00000u);
            if (term & (0x80u << (8 * k))) {
                if (ends == 0 && ((pv >> (8 * k + 7)) & 1)) ok = false;  // a fifth byte
                if (idx < cnt) vals[idx] = val;
                idx++;
            }
        }
        base += tot;
        prev_last = __builtin_amdgcn_readlane(x, 63);
    }
    ok = ok && base == cnt;
    return __ballot(!ok) == 0;
}

// Descriptor checks that keep every access of the chunk inside the stream
// and the output, whatever the workspace held before.
__device__ __forceinline__ bool desc_in_bounds(const Job &j, const ChunkDesc &d, uint32_t K)
{
    const uint32_t ns = d.nseq_last & 0x7fffffffu;
    return ns <= K && (uint64_t)d.out_base + d.out_len <= j.n &&
           (uint64_t)d.cmd_at + d.cmd_n <= j.comp_bytes && d.cmd_n <= 4 * (ns + 1) &&
           (uint64_t)d.len_at + d.len_n <= j.comp_bytes && d.len_n <= 4 * ns &&
           (uint64_t)d.lvl_at + d.lvl_n <= j.comp_bytes && d.lvl_n <= 4 * ns &&
           (uint64_t)d.lit_at + d.lit_n <= j.comp_bytes && (uint64_t)d.off_at + 4ull * ns <= j.comp_bytes;
}

// The 4 bytes of a one-byte-per-value slice that belong to values [e, e+4),
// zero past the slice's count.
__device__ __forceinline__ uint32_t bytes4(const uint8_t *p, uint32_t e, uint32_t cnt)
{
    if (e + 4 <= cnt) return ld32(p + e);
    uint32_t v = 0;
    for (uint32_t k = 0; k < 4; k++)
        if (e + k < cnt) v |= (uint32_t)p[e + k] << (8 * k);
    return v;
}

// --------------------------------------------------------------- k_map

// Batches: global block / chunk index -> stream.
__global__ void __launch_bounds__(NT) k_map(Batch B)
{
    const Job &j = B.jobs[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < j.n_blocks; i += NT) B.blk_job[j.b0 + i] = blockIdx.x;
    for (uint32_t i = threadIdx.x; i < j.n_chunks; i += NT) B.chunk_job[j.c0 + i] = blockIdx.x;
}

// --------------------------------------------------------------- k_setup

__global__ void __launch_bounds__(NT) k_setup(Batch B)
{
    __shared__ uint32_t ok_blk;
    __shared__ uint64_t tmp[NT / 64];
    const uint32_t t = threadIdx.x;

    if (!B.jobs && blockIdx.x == 0 && B.one.derive) {
        // single stream without levels: the counters of the level derivation
        if (t < DC_N) B.dcnt[t] = 0;
        if (t == 0) *B.one.status = 0;
    }
    if (!B.jobs && blockIdx.x == 0 && !B.one.derive) {
        // single stream: its level table -> record slots of every level
        const Job &j = B.one;
        const uint64_t lvl_tab = HDR + 16ull * (j.n_blocks + 1);
        uint64_t carry = 0, sig = 0;
        for (uint32_t s = 0; s <= j.max_level; s += NT) {
            const uint32_t i = s + t;
            const uint32_t c = i <= j.max_level ? ld32(j.comp + lvl_tab + 4ull * i) : 0;
            uint64_t tot, mixed;
            const uint64_t ex = wg_excl_scan64(c, tmp, tot);
            (void)wg_excl_scan64(i <= j.max_level ? level_mix(i, c) : 0, tmp, mixed);
            if (i <= j.max_level) {
                const uint32_t lo = (uint32_t)min(carry + ex, (uint64_t)j.n_seq);
                const uint32_t hi = (uint32_t)min(carry + ex + c, (uint64_t)j.n_seq);
                B.rec_lo[i] = lo;
                B.cursor[(size_t)i * CUR_STRIDE] = B.ordered ? hi : lo;  // ordered slots are placed, not appended
                B.rec_hi[i] = hi;
            }
            carry += tot;
            sig += mixed;
        }
        // every match counted exactly once, and the levels the host scheduled are these
        if (t == 0) {
            const int32_t before = j.validate ? *j.status : 0;  // the verdict of the level check, if one ran
            *j.status = (carry != j.n_seq || (B.has_sig && sig != B.level_sig)) ? ACEAPEX_E_CORRUPT : before;
        }
    }
    if (B.jobs && blockIdx.x < B.n_jobs) {
        // batch: this stream's level cursors (slots were laid out on the host
        // from its host level table, which must equal the stream's own), then
        // its status
        const Job &j = B.jobs[blockIdx.x];
        const uint64_t lvl_tab = HDR + 16ull * (j.n_blocks + 1);
        if (t == 0) ok_blk = 1;
        __syncthreads();
        for (uint32_t i = t; i <= j.max_level; i += NT) {
            const uint32_t lo = B.rec_lo[j.lv0 + i];
            B.cursor[j.lv0 + i] = lo;
            if (ld32(j.comp + lvl_tab + 4ull * i) != B.rec_hi[j.lv0 + i] - lo) ok_blk = 0;
        }
        __syncthreads();
        if (t == 0) *j.status = ok_blk ? 0 : ACEAPEX_E_CORRUPT;
        __syncthreads();
    }

    for (uint32_t gb = blockIdx.x; gb < B.n_blocks; gb += gridDim.x) {
        const Job &j = job_of(B, B.jobs ? B.blk_job[gb] : 0u);
        const uint32_t b = gb - j.b0;
        const uint64_t Bsz = (uint64_t)1 << j.block_log2;
        const uint32_t K = 1u << j.chunk_log2;
        const uint64_t prefix = HDR + 16ull * (j.n_blocks + 1) + (j.table ? pad16(4ull * (j.max_level + 1)) : 0);
        const uint8_t *tb = j.comp + HDR + 16ull * b;
        const uint64_t o0 = ld64(tb), o1 = ld64(tb + 16);
        const uint32_t sb0 = ld32(tb + 8), cb0 = ld32(tb + 12), sb1 = ld32(tb + 24), cb1 = ld32(tb + 28);
        bool ok = (o0 & 15) == 0 && o0 >= prefix && o1 >= o0 + BLKHDR && o1 <= j.comp_bytes &&
                  cb1 >= cb0 && cb1 <= j.n_chunks && sb1 >= sb0 && sb1 <= j.n_seq;
        if (b == 0) ok = ok && cb0 == 0 && sb0 == 0 && o0 == prefix;
        if (b + 1 == j.n_blocks) ok = ok && o1 == j.comp_bytes && cb1 == j.n_chunks && sb1 == j.n_seq;
        uint32_t ns = 0, nl = 0, nc = 0, cmdb = 0, lenb = 0, lvlb = 0;
        uint64_t off_at = 0, cmd_at = 0, len_at = 0, lvl_at = 0, lit_at = 0;
        if (ok) {
            const uint8_t *bh = j.comp + o0;
            ns = ld32(bh); nl = ld32(bh + 4); nc = ld32(bh + 8);
            const uint32_t bmax = ld32(bh + 12);
            cmdb = ld32(bh + 16); lenb = ld32(bh + 20); lvlb = ld32(bh + 24);
            const uint32_t want_nc = ns ? (uint32_t)((ns + (uint64_t)K - 1) / K) : 1u;
            ok = nc == cb1 - cb0 && ns == sb1 - sb0 && nc == want_nc && bmax <= j.max_level;
            off_at = o0 + BLKHDR + (uint64_t)CHUNK_ENT * nc;
            cmd_at = off_at + pad16(4ull * ns);
            len_at = cmd_at + pad16(cmdb);
            lvl_at = len_at + pad16(lenb);
            lit_at = lvl_at + pad16(lvlb);
            ok = ok && lit_at + pad16(nl) == o1;
        }
        if (t == 0) ok_blk = ok;
        __syncthreads();
        const bool blk_good = ok_blk;
        __syncthreads();
        if (!blk_good) {
            if (t == 0) j.blk_ok[b] = 0;
            continue;
        }
        const uint32_t blen = (uint32_t)min(Bsz, (uint64_t)j.n - b * Bsz);
        bool all = true;
        for (uint32_t c = t; c < nc; c += NT) {
            const uint8_t *e = j.comp + o0 + BLKHDR + (uint64_t)CHUNK_ENT * c;
            const uint32_t c0 = ld32(e), l0 = ld32(e + 4), v0 = ld32(e + 8), q0 = ld32(e + 12), d0 = ld32(e + 16);
            uint32_t c1 = cmdb, l1 = lenb, v1 = lvlb, q1 = nl, d1 = blen;
            if (c + 1 < nc) { c1 = ld32(e + 32); l1 = ld32(e + 36); v1 = ld32(e + 40); q1 = ld32(e + 44); d1 = ld32(e + 48); }
            const uint32_t n_in = ns ? min(K, ns - c * K) : 0;
            const bool last = c + 1 == nc;
            const bool cok = c0 <= c1 && c1 <= cmdb && l0 <= l1 && l1 <= lenb && v0 <= v1 && v1 <= lvlb &&
                             q0 <= q1 && q1 <= nl && d0 <= d1 && d1 <= blen &&
                             c1 - c0 <= 4 * (n_in + 1) && l1 - l0 <= 4 * n_in && v1 - v0 <= 4 * n_in;
            ChunkDesc cd;
            cd.out_base = (uint32_t)(b * Bsz) + d0;
            cd.out_len = d1 - d0;
            cd.cmd_at = (uint32_t)cmd_at + c0; cd.cmd_n = c1 - c0;
            cd.len_at = (uint32_t)len_at + l0; cd.len_n = l1 - l0;
            cd.lvl_at = (uint32_t)lvl_at + v0; cd.lvl_n = v1 - v0;
            cd.lit_at = (uint32_t)lit_at + q0; cd.lit_n = q1 - q0;
            cd.off_at = (uint32_t)(off_at + 4ull * c * K);
            cd.nseq_last = n_in | (last ? 0x80000000u : 0u);
            cd.seq0 = sb0 + c * K;
            cd.pad[0] = cd.pad[1] = cd.pad[2] = 0;
            if (!cok) {  // a descriptor that k_parse rejects
                cd.out_len = 0xffffffffu;
                all = false;
            }
            j.chunks[cb0 + c] = cd;
        }
        if (t == 0) ok_blk = 1;
        __syncthreads();
        if (!all) ok_blk = 0;
        __syncthreads();
        if (t == 0) j.blk_ok[b] = (uint8_t)ok_blk;
        __syncthreads();
    }
}

// --------------------------------------------------------------- k_parse

// Set the bits of the 16-byte tile segments that tile bytes [a, a + n)
// (n > 0) touch.
__device__ __forceinline__ void mark_segments(uint32_t *seg, uint32_t a, uint32_t n)
{
    const uint32_t s0 = a >> 4, s1 = (a + n - 1) >> 4;
    for (uint32_t w = s0 >> 5; w <= (s1 >> 5); w++) {
        const uint32_t lo = max(s0, w << 5) & 31, hi = min(s1, (w << 5) + 31) & 31;
        const uint32_t upto = hi == 31 ? 0xffffffffu : ((2u << hi) - 1);
        atomicOr(&seg[w], upto & ~((1u << lo) - 1));
    }
}

// k_parse comes in three LDS shapes, picked by the deepest level of the
// launch: LH levels are ranked in LDS (deeper ones take one global atomic per
// match), and up to STAGE bytes of a chunk's literals are staged in LDS.  Each
// shape keeps six workgroups per CU.
template <uint32_t LH, uint32_t STAGE>
struct ParseLds {
    union {
        struct {
            uint32_t run[K_MAX + 1];   // LEB128 path: literal runs
            uint32_t mlen[K_MAX];      // LEB128 path: match lengths - min_match
            uint32_t lvl[K_MAX];       // LEB128 path: match levels
        } v;
        uint8_t tile[TILE_BYTES];      // after the scan: the chunk's output span, literals in place
    } u;
    uint32_t stage[STAGE / 4 + 8];  // the chunk's literal bytes from a 16-byte boundary (+ read slack)
    uint32_t seg[TILE_BYTES / 512];  // tile 16-byte segments that hold literal bytes, one bit each
    uint32_t lcount[LH];         // matches of the chunk per level (levels < LH)
    uint32_t lbase[LH];          // record slot reserved for them
    uint64_t tmp[NT / 64];
    uint32_t bad;
} __attribute__((aligned(16)));

// ORD: a single stream with ordered slots (its chunks' first slots per level
// were counted and scanned before the parse).
template <bool BATCH, uint32_t LH, uint32_t STAGE, bool ORD>
__global__ void __launch_bounds__(NT, BATCH ? 5 : 6) k_parse(Batch B)
{
    __shared__ ParseLds<LH, STAGE> L;
    const uint32_t t = threadIdx.x, wave = t >> 6;
    // Chunks in dispatch order: workgroups finish roughly in that order, so
    // each level's records are appended roughly in output order (exactly so
    // with ordered slots) and every contiguous part of a level that k_level
    // gives one XCD covers one stretch of the output.
    const uint32_t g = blockIdx.x;  // global chunk
    const uint32_t sj = BATCH ? B.chunk_job[g] : 0u;     // its stream
    // batched: the descriptor is read by its global index, beside the stream
    // lookup rather than after it (one dependent load less per workgroup)
    ChunkDesc d;
    if constexpr (BATCH) d = B.chunks_all[g];
    const Job &j = BATCH ? B.jobs[sj] : B.one;
    const uint32_t c = g - j.c0;
    const uint32_t K = 1u << j.chunk_log2;
    const uint32_t nl = min(j.max_level + 1, LH);

    if (c == 0) {  // any block of the stream that failed its checks fails the stream
        bool bad = false;
        for (uint32_t b = t; b < j.n_blocks; b += NT) bad |= j.blk_ok[b] == 0;
        if (bad) fail(j, ACEAPEX_E_CORRUPT);
    }
    if (t == 0) L.bad = 0;
    for (uint32_t i = t; i < nl; i += NT) L.lcount[i] = 0;
    if (t < TILE_BYTES / 512) L.seg[t] = 0;
    __syncthreads();
    if (c >= j.n_chunks) return;
    if constexpr (!BATCH) d = j.chunks[c];
    const uint32_t blk = d.out_base >> j.block_log2;
    if (!desc_in_bounds(j, d, K) || blk >= j.n_blocks) {
        if (t == 0) fail(j, ACEAPEX_E_CORRUPT);
        return;
    }
    const uint32_t ns = d.nseq_last & 0x7fffffffu;
    const uint32_t ncmd = ns + (d.nseq_last >> 31);
    const bool one_byte = d.cmd_n == ncmd && d.len_n == ns && d.lvl_n == (j.table ? ns : 0u);
    const uint32_t e0 = t * PER;

    // Literal placement.  When the chunk's output span fits the LDS tile, the
    // runs are placed in the tile and the span is written with aligned
    // 16-byte stores (its match bytes are written later by the level
    // launches; in chunks dense in literals, segments of match bytes only
    // are not written at all).  With matches of at least 3 bytes between runs, no 4-byte
    // word of the output holds literal bytes of two runs, so a run is placed
    // as the whole aligned words that cover it; their other bytes lie in the
    // neighbouring matches.  The chunk's literal bytes, from the 16-byte
    // boundary at or below lit_at - 4, are first copied into LDS by direct
    // global-to-LDS loads issued here and awaited before the scan.
    const uint32_t base16 = d.out_base & ~15u;
    const uint32_t span_end = d.out_base + d.out_len;
    const bool tiled = span_end - base16 <= TILE_BYTES;
    const bool words = tiled && j.min_match >= 3;
    const uint64_t la = ((uint64_t)d.lit_at - 4) & ~(uint64_t)15;
    const uint64_t lend = ((uint64_t)d.lit_at + d.lit_n + 15) & ~(uint64_t)15;
    const bool staged = STAGE && words && d.lit_at >= 4 && lend - la <= STAGE && lend <= j.comp_bytes;
    if (staged) {
        const uint32_t nblk = (uint32_t)((lend - la) >> 4);
        for (uint32_t b0 = 64 * wave; b0 < nblk; b0 += NT) {  // b0: the wave's first 16-byte block
            if (b0 + (t & 63) < nblk)
                __builtin_amdgcn_global_load_lds(j.comp + la + 16ull * (b0 + (t & 63)),
                                                 (__attribute__((address_space(3))) void *)((uint8_t *)L.stage + 16 * b0),
                                                 16, 0, 0);
        }
    }
    // a full chunk (NT * PER sequences) that also holds its block's trailing
    // run: that run is the command past every thread's range.  Every thread
    // reads it (it ends the chunk's span and its literals); the last thread
    // adds it to the scan, and the workgroup copies it after the other runs.
    const bool tail_cmd = ncmd > NT * PER;

    // this thread's sequences e0 .. e0+3: run, match length and level
    uint32_t r[PER], m[PER], l[PER];
    uint32_t rt = 0;  // the trailing run when tail_cmd (uniform)
    bool bad = false;
    if (one_byte) {
        const uint32_t cw = bytes4(j.comp + d.cmd_at, e0, ncmd);
        const uint32_t lw = bytes4(j.comp + d.len_at, e0, ns);
        const uint32_t vw = j.table ? bytes4(j.comp + d.lvl_at, e0, ns) : 0u;
        if ((cw | lw | vw) & 0x80808080u) bad = true;  // a continuation byte where every value is one byte
        if (tail_cmd) {
            rt = j.comp[d.cmd_at + NT * PER];
            if (rt & 0x80u) bad = true;
        }
#pragma unroll
        for (uint32_t u = 0; u < PER; u++) {
            r[u] = (cw >> (8 * u)) & 0xff;
            m[u] = e0 + u < ns ? ((lw >> (8 * u)) & 0xff) + j.min_match : 0;
            l[u] = (vw >> (8 * u)) & 0xff;
        }
    } else {
        bool ok = true;
        const uint32_t wv = __builtin_amdgcn_readfirstlane(wave);
        if (wv < (j.table ? 3u : 2u)) {  // waves 0, 1, 2: the cmd, len and lvl slices
            const uint32_t at = wv == 0 ? d.cmd_at : wv == 1 ? d.len_at : d.lvl_at;
            const uint32_t nb = wv == 0 ? d.cmd_n : wv == 1 ? d.len_n : d.lvl_n;
            uint32_t *vals = wv == 0 ? L.u.v.run : wv == 1 ? L.u.v.mlen : L.u.v.lvl;
            ok = wave_varints(j.comp + at, nb, j.comp_bytes - at, wv == 0 ? ncmd : ns, vals);
        }
        if (!ok && (t & 63) == 0) L.bad = 1;
        __syncthreads();
        if (L.bad) {
            if (t == 0) fail(j, ACEAPEX_E_CORRUPT);
            if (staged) __builtin_amdgcn_s_waitcnt(0);  // no direct-to-LDS load left in flight at exit
            return;
        }
#pragma unroll
        for (uint32_t u = 0; u < PER; u++) {
            const uint32_t e = e0 + u;
            r[u] = e < ncmd ? L.u.v.run[e] : 0;
            m[u] = e < ns ? L.u.v.mlen[e] + j.min_match : 0;
            l[u] = e < ns && j.table ? L.u.v.lvl[e] : 0;
        }
        if (tail_cmd) rt = L.u.v.run[NT * PER];
    }

    // output and literal offsets: workgroup scan over (run + match, run)
    uint64_t acc = 0;
#pragma unroll
    for (uint32_t u = 0; u < PER; u++) {
        if (r[u] > d.out_len || m[u] > d.out_len || (e0 + u < ns && l[u] > j.max_level)) bad = true;
        acc += ((uint64_t)(r[u] + m[u]) << 32) | r[u];
    }
    rt = __builtin_amdgcn_readfirstlane(rt);
    if (rt > d.out_len) bad = true;
    if (t == NT - 1) acc += ((uint64_t)rt << 32) | rt;
    if (staged) __builtin_amdgcn_s_waitcnt(0);  // this thread's staging loads; the scan's barrier publishes them
    uint64_t tot;
    const uint64_t ex = wg_excl_scan64(bad ? 0 : acc, L.tmp, tot);
    if (bad) L.bad = 1;
    __syncthreads();
    if (L.bad || (uint32_t)(tot >> 32) != d.out_len || (uint32_t)tot != d.lit_n) {
        if (t == 0) fail(j, ACEAPEX_E_CORRUPT);
        return;
    }

    // the match sources, needed only by the records: loaded here, so that
    // they are not held through the varint decode and arrive while the
    // literals are placed
    uint32_t src[PER];
    {
        const u128u o4 = e0 + PER <= ns ? *(const u128u *)(j.comp + d.off_at + 4 * e0) : u128u{0, 0, 0, 0};
        src[0] = o4.a; src[1] = o4.b; src[2] = o4.c; src[3] = o4.d;
        if (e0 + PER > ns)
            for (uint32_t u = 0; u < PER; u++) src[u] = e0 + u < ns ? ld32(j.comp + d.off_at + 4 * (e0 + u)) : 0;
    }

    uint32_t pos = d.out_base + (uint32_t)(ex >> 32), lq = (uint32_t)ex;
    uint32_t dst[PER], rank[PER];
    uint32_t cw[PER], ce[PER], cq[PER];  // staged runs: tile words [cw, ce) still to place, staged byte of cw
#pragma unroll
    for (uint32_t u = 0; u < PER; u++) {
        cw[u] = ce[u] = cq[u] = 0;
        if (r[u] && tiled) mark_segments(L.seg, pos - base16, r[u]);
        if (r[u] && staged) {
            const uint32_t a0 = pos - base16;
            cw[u] = a0 & ~3u;
            ce[u] = (a0 + r[u] + 3) & ~3u;
            cq[u] = (uint32_t)((uint64_t)d.lit_at + lq - (a0 - cw[u]) - la);
        } else if (r[u] && words) {
            const uint32_t a0 = pos - base16, w0 = a0 & ~3u, w1 = (a0 + r[u] + 3) & ~3u;
            const uint64_t s0 = (uint64_t)d.lit_at + lq - (a0 - w0);  // stream byte that lands on tile byte w0
            for (uint32_t o = w0; o < w1; o += 16) {
                const uint64_t sa = s0 + (o - w0);
                u128u v;
                if (sa + 16 <= j.comp_bytes) {
                    v = *(const u128u *)(j.comp + sa);
                } else {
                    uint32_t x[4] = {0, 0, 0, 0};
                    for (uint32_t k = 0; k < 16 && sa + k < j.comp_bytes; k++) x[k >> 2] |= (uint32_t)j.comp[sa + k] << (8 * (k & 3));
                    v = u128u{x[0], x[1], x[2], x[3]};
                }
                uint32_t *tw = (uint32_t *)(L.u.tile + o);
                const uint32_t nw = min(4u, (w1 - o) >> 2);
                tw[0] = v.a;
                if (nw > 1) tw[1] = v.b;
                if (nw > 2) tw[2] = v.c;
                if (nw > 3) tw[3] = v.d;
            }
        } else if (r[u]) {
            const uint8_t *ls = j.comp + d.lit_at + lq;
            if (!tiled) {
                copy_bytes(j.out + pos, ls, r[u]);
            } else {
                uint8_t *td = L.u.tile + (pos - base16);
                for (uint32_t o = 0; o < r[u]; o += 16) {
                    const uint32_t n = min(16u, r[u] - o);
                    if ((uint64_t)(d.lit_at + lq + o) + 16 <= j.comp_bytes) {
                        const u128u v = *(const u128u *)(ls + o);
                        store_upto16(td + o, ((uint64_t)v.b << 32) | v.a, ((uint64_t)v.d << 32) | v.c, n);
                    } else {
                        for (uint32_t k = 0; k < n; k++) td[o + k] = ls[o + k];
                    }
                }
            }
        }
        pos += r[u];
        lq += r[u];
        dst[u] = pos;
        pos += m[u];
    }
    if (staged) {
        // The staged runs.  Each lane places the first four words of each of
        // its runs.  The words past those of the longer runs are then placed
        // per run slot u: when only a few lanes have a longer run in slot u,
        // the whole wave places those runs one at a time, a word per lane, so
        // that a long run costs one step instead of holding its lane for many;
        // otherwise every lane places the rest of its own run, four words per
        // pass.
        uint32_t sw[PER][5];  // every run's first staged words, read at once
#pragma unroll
        for (uint32_t u = 0; u < PER; u++)
#pragma unroll
            for (uint32_t k = 0; k < 5; k++) sw[u][k] = L.stage[(cq[u] >> 2) + k];
#pragma unroll
        for (uint32_t u = 0; u < PER; u++) {
            const uint32_t w = cw[u], e = ce[u], sh = cq[u] & 3;
            uint32_t *tw = (uint32_t *)(L.u.tile + w);
            if (w < e) tw[0] = __builtin_amdgcn_alignbyte(sw[u][1], sw[u][0], sh);
            if (w + 4 < e) tw[1] = __builtin_amdgcn_alignbyte(sw[u][2], sw[u][1], sh);
            if (w + 8 < e) tw[2] = __builtin_amdgcn_alignbyte(sw[u][3], sw[u][2], sh);
            if (w + 12 < e) tw[3] = __builtin_amdgcn_alignbyte(sw[u][4], sw[u][3], sh);
        }
        const uint32_t lane = t & 63;
#pragma unroll
        for (uint32_t u = 0; u < PER; u++) {
            uint64_t m = __ballot(cw[u] + 16 < ce[u]);
            if (__popcll(m) <= COOP_RUNS) {
                for (; m; m &= m - 1) {
                    const uint32_t src_lane = (uint32_t)__builtin_ctzll(m);
                    const uint32_t w = __builtin_amdgcn_readlane(cw[u], src_lane) + 16;
                    const uint32_t e = __builtin_amdgcn_readlane(ce[u], src_lane);
                    const uint32_t q = __builtin_amdgcn_readlane(cq[u], src_lane) + 16;
                    for (uint32_t o = 4 * lane; w + o < e; o += 256) {
                        const uint32_t qq = q + o;
                        *(uint32_t *)(L.u.tile + w + o) =
                            __builtin_amdgcn_alignbyte(L.stage[(qq >> 2) + 1], L.stage[qq >> 2], qq & 3);
                    }
                }
            } else {
                const uint32_t e = ce[u];
                for (uint32_t w = cw[u] + 16, q = cq[u] + 16;; w += 16, q += 16) {
                    const bool act = w < e;
                    if (__ballot(act) == 0) break;
                    if (act) {
                        const uint32_t qi = q >> 2, sh = q & 3;
                        const uint32_t s0 = L.stage[qi], s1 = L.stage[qi + 1], s2 = L.stage[qi + 2],
                                       s3 = L.stage[qi + 3], s4 = L.stage[qi + 4];
                        uint32_t *tw = (uint32_t *)(L.u.tile + w);
                        tw[0] = __builtin_amdgcn_alignbyte(s1, s0, sh);
                        if (w + 4 < e) tw[1] = __builtin_amdgcn_alignbyte(s2, s1, sh);
                        if (w + 8 < e) tw[2] = __builtin_amdgcn_alignbyte(s3, s2, sh);
                        if (w + 12 < e) tw[3] = __builtin_amdgcn_alignbyte(s4, s3, sh);
                    }
                }
            }
        }
    }
    if (rt) {  // the trailing run of a full chunk, copied by the whole workgroup
        const uint32_t at = d.out_base + d.out_len - rt;
        if (tiled && t == 0) mark_segments(L.seg, at - base16, rt);
        const uint8_t *ls = j.comp + d.lit_at + (d.lit_n - rt);
        for (uint32_t o = 16 * t; o < rt; o += 16 * NT) {
            const uint32_t n = min(16u, rt - o);
            if (!tiled) {
                copy_bytes(j.out + at + o, ls + o, n);
            } else if ((uint64_t)d.lit_at + (d.lit_n - rt) + o + 16 <= j.comp_bytes) {
                const u128u x = *(const u128u *)(ls + o);
                store_upto16(L.u.tile + (at - base16) + o, ((uint64_t)x.b << 32) | x.a, ((uint64_t)x.d << 32) | x.c, n);
            } else {
                for (uint32_t k = 0; k < n; k++) L.u.tile[at - base16 + o + k] = ls[o + k];
            }
        }
    }
    if (tiled) {
        __syncthreads();
        const uint32_t nseg = (span_end - base16 + 15) / 16;
        // Segments of match bytes only are skipped in chunks of at least a
        // quarter literals.  In chunks of sparse literals writing the whole
        // span measured faster on deep streams (the span's stores space out
        // the workgroups' level atomics) and no slower elsewhere.
        const bool sparse_skip = 4ull * d.lit_n >= d.out_len;
        for (uint32_t i = t; i < nseg; i += NT) {
            if (sparse_skip && !((L.seg[i >> 5] >> (i & 31)) & 1u)) continue;  // match bytes only
            const uint32_t a = base16 + 16 * i;
            const uint8_t *tsrc = L.u.tile + 16 * i;
            if (a >= d.out_base && a + 16 <= span_end) {
                *(uint4 *)(j.out + a) = *(const uint4 *)tsrc;
            } else {
                for (uint32_t k = 0; k < 16; k++)
                    if (a + k >= d.out_base && a + k < span_end) j.out[a + k] = tsrc[k];
            }
        }
    }

    if (!BATCH && j.derive) {
        // levels derived on the device: every match -> its record in stream
        // order, with the state of its derivation: not run, nothing parked
        // on it, its source to scan
        for (uint32_t u = 0; u < PER; u++) {
            if (e0 + u >= ns) continue;
            const uint32_t i = d.seq0 + e0 + u;
            if ((uint64_t)src[u] + m[u] > dst[u] || i >= j.n_seq) {
                bad = true;
                continue;
            }
            uint32_t *rr = B.recs + 3ull * i;
            rr[0] = dst[u]; rr[1] = src[u]; rr[2] = m[u];
            B.dlevel[i] = j.validate ? l[u] : NONE;  // the stored level, when it is being checked
            B.dhead[i] = NONE;
            B.dcur[i] = src[u];
            B.dmax[i] = 0;
        }
        if (bad) fail(j, ACEAPEX_E_CORRUPT);
        return;
    }

    // every match -> record in the slots of its level
    const uint32_t tag = sj << LEN_BITS;
#pragma unroll
    for (uint32_t u = 0; u < PER; u++) {
        rank[u] = 0xffffffffu;
        if (e0 + u >= ns) continue;
        if ((uint64_t)src[u] + m[u] > dst[u]) {  // a source must end before its destination
            bad = true;
            continue;
        }
        if (l[u] < LH) {
            rank[u] = atomicAdd(&L.lcount[l[u]], 1u);
        } else {
            const uint32_t e = j.lv0 + l[u];
            const uint32_t slot = atomicAdd(&B.cursor[BATCH ? e : (size_t)e * CUR_STRIDE], 1u);
            if (slot < B.rec_hi[e]) {
                uint32_t *rr = B.recs + 3ull * slot;
                rr[0] = dst[u]; rr[1] = src[u]; rr[2] = m[u] | tag;
            } else {
                bad = true;
            }
        }
    }
    __syncthreads();
    if constexpr (LH >= 1024) {
        // Deep streams, whose chunks spread their matches over tens of
        // levels: the records go out grouped by level.  Each is first put in
        // LDS (the tile, free by now) at its level's first position among the
        // chunk's records plus its rank, then the workgroup writes them in
        // that order, so that neighbouring lanes write neighbouring slots of
        // one level; written straight from each match, a store instruction
        // would touch as many separate regions as it has levels.  (On streams
        // of few levels per chunk the extra barriers cost more than this
        // saves.)  Thread t scans the counts of levels t*NI .. t*NI+NI-1;
        // each level's first position then replaces its count in lcount.
        constexpr uint32_t NI = (LH + NT - 1) / NT;
        static_assert(TILE_BYTES >= 16 * K_MAX, "a chunk's records fit the tile");
        uint4 *const grp = (uint4 *)L.u.tile;
        uint32_t grouped;  // the chunk's matches of levels below LH
        {
            uint32_t cnt[NI], own = 0;
#pragma unroll
            for (uint32_t k = 0; k < NI; k++) {
                cnt[k] = t * NI + k < nl ? L.lcount[t * NI + k] : 0u;
                own += cnt[k];
            }
            uint64_t tot;
            uint32_t at = (uint32_t)wg_excl_scan64(own, L.tmp, tot);  // its barriers end every read of lcount above
            grouped = (uint32_t)tot;
#pragma unroll
            for (uint32_t k = 0; k < NI; k++) {
                if (t * NI + k < nl) L.lcount[t * NI + k] = at;
                at += cnt[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t u = 0; u < PER; u++)
            if (rank[u] != 0xffffffffu) grp[L.lcount[l[u]] + rank[u]] = make_uint4(dst[u], src[u], m[u] | tag, l[u]);
        // the first slot of each level present in the chunk: with ordered slots
        // the chunk's own (counted and scanned before the parse, so that a
        // level's records follow the chunks' order), else one global atomic per
        // level, all issued before any returns.  A level whose slots would leave
        // its range (more matches than the level table announced) gets no
        // records.  A level's count is the distance to the next level's first
        // position.
        {
            uint32_t got[NI], cap[NI], cnt[NI];
#pragma unroll
            for (uint32_t k = 0; k < NI; k++) {
                const uint32_t i = t + k * NT;
                cnt[k] = i < nl ? (i + 1 < nl ? L.lcount[i + 1] : grouped) - L.lcount[i] : 0u;
                if (ORD)
                    got[k] = cnt[k] ? B.ocnt[(size_t)i * j.n_chunks + c] : 0u;
                else
                    got[k] = cnt[k] ? atomicAdd(&B.cursor[BATCH ? j.lv0 + i : (size_t)i * CUR_STRIDE], cnt[k]) : 0u;
                cap[k] = cnt[k] ? B.rec_hi[j.lv0 + i] : 0u;
            }
#pragma unroll
            for (uint32_t k = 0; k < NI; k++) {
                const uint32_t i = t + k * NT;
                // an appended base never lies below the level's first slot; a
                // placed one is checked against it too
                const bool above = !ORD || got[k] >= B.rec_lo[j.lv0 + i];
                if (cnt[k]) L.lbase[i] = above && got[k] <= cap[k] && cnt[k] <= cap[k] - got[k] ? got[k] : NO_SLOT;
            }
        }
        __syncthreads();
        for (uint32_t q = t; q < grouped; q += NT) {
            const uint4 v = grp[q];
            const uint32_t lb = L.lbase[v.w];
            if (lb == NO_SLOT) {
                bad = true;
                continue;
            }
            uint32_t *rr = B.recs + 3ull * (lb + (q - L.lcount[v.w]));
            rr[0] = v.x; rr[1] = v.y; rr[2] = v.z;
        }
    } else {
        // the first slot of each level present in the chunk: with ordered slots
        // the chunk's own (counted and scanned before the parse, so that a
        // level's records follow the chunks' order), else one global atomic per
        // level, all issued before any returns.  A level whose slots would leave
        // its range (more matches than the level table announced) gets no
        // records.
        {
            constexpr uint32_t NI = (LH + NT - 1) / NT;
            uint32_t got[NI], cap[NI];
#pragma unroll
            for (uint32_t k = 0; k < NI; k++) {
                const uint32_t i = t + k * NT;
                const uint32_t cn = i < nl ? L.lcount[i] : 0u;
                if (ORD)
                    got[k] = cn ? B.ocnt[(size_t)i * j.n_chunks + c] : 0u;
                else
                    got[k] = cn ? atomicAdd(&B.cursor[BATCH ? j.lv0 + i : (size_t)i * CUR_STRIDE], cn) : 0u;
                cap[k] = cn ? B.rec_hi[j.lv0 + i] : 0u;
            }
#pragma unroll
            for (uint32_t k = 0; k < NI; k++) {
                const uint32_t i = t + k * NT;
                // an appended base never lies below the level's first slot; a
                // placed one is checked against it too
                const bool above = !ORD || got[k] >= B.rec_lo[j.lv0 + i];
                if (i < nl && L.lcount[i])
                    L.lbase[i] = above && got[k] <= cap[k] && L.lcount[i] <= cap[k] - got[k] ? got[k] : NO_SLOT;
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t u = 0; u < PER; u++) {
            if (rank[u] == 0xffffffffu) continue;
            const uint32_t lb = L.lbase[l[u]];
            const uint32_t slot = lb + rank[u];
            if (lb == NO_SLOT) {
                bad = true;
                continue;
            }
            uint32_t *rr = B.recs + 3ull * slot;
            rr[0] = dst[u]; rr[1] = src[u]; rr[2] = m[u] | tag;
        }
    }
    if (bad) fail(j, ACEAPEX_E_CORRUPT);
}

// The k_parse shape for a launch whose deepest level is max_level.
template <bool BATCH>
void launch_parse(const Batch &B, uint32_t grid, hipStream_t st)
{
    static_assert(ORD_LEVELS <= 256, "ordered slots use the shallow parse shape");
    if (!BATCH && B.ordered)
        hipLaunchKernelGGL((k_parse<false, 256, 7680, true>), dim3(grid), dim3(NT), 0, st, B);
    else if (B.max_level < 256)
        hipLaunchKernelGGL((k_parse<BATCH, 256, 7680, false>), dim3(grid), dim3(NT), 0, st, B);
    else if (B.max_level < 1024)
        hipLaunchKernelGGL((k_parse<BATCH, 1024, 1536, false>), dim3(grid), dim3(NT), 0, st, B);
    else
        hipLaunchKernelGGL((k_parse<BATCH, 4096, 0, false>), dim3(grid), dim3(NT), 0, st, B);
}

// ---------------------------------------------------- ordered record slots

// A single stream with few levels gets its record slots in chunk order: each
// chunk's matches of a level go to the slots after those of the chunks
// before it, so that a level's records follow the output, as its copies'
// destinations do (the level launches then write nearby lines together).
// k_count counts each chunk's matches per level, k_otiles and k_oapply turn
// the level-major counts into first slots (an exclusive scan whose running
// total passes through each level's first slot; each k_oapply workgroup sums
// the tile totals before its own), and k_parse reads its chunk's first slots
// instead of taking them with atomics.

// One wave per CPW chunks: each chunk's matches per level into
// ocnt[level * C + chunk].  A malformed level section counts nothing (k_parse
// fails the stream).  Lanes count into HCOPIES histograms by lane (rows padded
// to a bank offset), so that a run of equal levels among a wave's values does
// not serialise on one LDS address.  The loads of both chunks (descriptors,
// then their one-byte level words) are issued before the first count: the
// kernel is bound by the latency of those two dependent loads.
constexpr uint32_t HCOPIES = 4;
constexpr uint32_t CPW = 2;
__global__ void __launch_bounds__(NT) k_count(Batch B)
{
    __shared__ uint32_t vals[NT / 64][K_MAX];
    __shared__ uint32_t hist[NT / 64][HCOPIES][ORD_LEVELS + 1];
    static_assert(ORD_LEVELS <= 64, "one lane per level");
    constexpr uint32_t ROUNDS = K_MAX / (4 * 64);
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const Job &j = B.one;
    const uint32_t C = j.n_chunks, nl = j.max_level + 1, K = 1u << j.chunk_log2;
    // the same on every lane of the wave: made scalar, so that descriptors
    // are read by scalar loads into scalar registers
    const uint32_t c0 = __builtin_amdgcn_readfirstlane((blockIdx.x * (NT / 64) + wave) * CPW);
    if (c0 >= C) return;  // no workgroup barrier below: each wave works alone
    uint32_t *const h = &hist[wave][0][0];
    uint32_t *const mine = h + (lane % HCOPIES) * (ORD_LEVELS + 1);
    ChunkDesc d[CPW];
    uint32_t ns[CPW], kind[CPW], w4[CPW][ROUNDS];  // kind: 0 nothing to count, 1 one byte per level, 2 LEB128
#pragma unroll
    for (uint32_t k = 0; k < CPW; k++) {
        kind[k] = 0;
        ns[k] = 0;
        if (c0 + k < C) {
            d[k] = j.chunks[c0 + k];
            ns[k] = d[k].nseq_last & 0x7fffffffu;
            if (desc_in_bounds(j, d[k], K) && (d[k].out_base >> j.block_log2) < j.n_blocks)
                kind[k] = d[k].lvl_n == ns[k] ? 1u : 2u;
        }
    }
#pragma unroll
    for (uint32_t k = 0; k < CPW; k++)
#pragma unroll
        for (uint32_t r = 0; r < ROUNDS; r++) {
            const uint32_t e = 4 * lane + 4 * 64 * r;
            w4[k][r] = kind[k] == 1 && e < ns[k] ? bytes4(j.comp + d[k].lvl_at, e, ns[k]) : 0u;
        }
    static_assert(CPW == 2, "the counting loop picks chunk k's values by selects");
#pragma unroll 1
    for (uint32_t k = 0; k < CPW; k++) {  // not unrolled: one copy of the counting code
        const uint32_t c = c0 + k;
        if (c >= C) break;
        const uint32_t kk = k ? kind[1] : kind[0], n = k ? ns[1] : ns[0];
        for (uint32_t i = lane; i < HCOPIES * (ORD_LEVELS + 1); i += 64) h[i] = 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the wave's LDS accesses stay in program order
        if (kk == 1) {
#pragma unroll
            for (uint32_t r = 0; r < ROUNDS; r++) {
                const uint32_t e = 4 * lane + 4 * 64 * r;
                const uint32_t wr = k ? w4[1][r] : w4[0][r];
#pragma unroll
                for (uint32_t b = 0; b < 4; b++) {
                    const uint32_t v = (wr >> (8 * b)) & 0xffu;
                    if (e + b < n && v < nl) atomicAdd(&mine[v], 1u);
                }
            }
        } else if (kk == 2) {
            const uint32_t at = k ? d[1].lvl_at : d[0].lvl_at, nb = k ? d[1].lvl_n : d[0].lvl_n;
            if (wave_varints(j.comp + at, nb, j.comp_bytes - at, n, vals[wave])) {
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                for (uint32_t e = lane; e < n; e += 64) {
                    const uint32_t v = vals[wave][e];
                    if (v < nl) atomicAdd(&mine[v], 1u);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (lane < nl) {
            uint32_t cnt = 0;
#pragma unroll
            for (uint32_t q = 0; q < HCOPIES; q++) cnt += h[q * (ORD_LEVELS + 1) + lane];
            B.ocnt[(size_t)lane * C + c] = cnt;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// The sum of each OTILE elements of ocnt.
__global__ void __launch_bounds__(NT) k_otiles(Batch B)
{
    __shared__ uint64_t tmp[NT / 64];
    const uint64_t E = (uint64_t)(B.one.max_level + 1) * B.one.n_chunks, t0 = (uint64_t)blockIdx.x * OTILE;
    const uint64_t t1 = min(E, t0 + OTILE);
    uint64_t sum = 0, tot;
    for (uint64_t i = t0 + threadIdx.x; i < t1; i += NT) sum += B.ocnt[i];
    (void)wg_excl_scan64(sum, tmp, tot);
    if (threadIdx.x == 0) B.otile[blockIdx.x] = (uint32_t)tot;
}

// Each count becomes its first slot.  The element of each level's first
// chunk must land on the level's first slot and the last one must end at
// the last slot, else the stream's chunks and its level table disagree and
// the decode fails.
__global__ void __launch_bounds__(NT) k_oapply(Batch B)
{
    __shared__ uint64_t tmp[NT / 64];
    const uint32_t C = B.one.n_chunks, nl = B.one.max_level + 1;
    const uint64_t E = (uint64_t)nl * C, t0 = (uint64_t)blockIdx.x * OTILE;
    const uint64_t t1 = min(E, t0 + OTILE);
    uint64_t before = 0, carry;  // the tiles before this one, summed by the workgroup
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += NT) before += B.otile[i];
    (void)wg_excl_scan64(before, tmp, carry);
    for (uint64_t s0 = t0; s0 < t1; s0 += NT) {
        const uint64_t i = s0 + threadIdx.x;
        const uint64_t v = i < t1 ? B.ocnt[i] : 0;
        uint64_t tot;
        const uint64_t ex = wg_excl_scan64(v, tmp, tot);
        if (i < t1) {
            const uint64_t at = carry + ex;
            B.ocnt[i] = (uint32_t)at;
            if (i % C == 0 && at != B.rec_lo[i / C]) fail(B.one, ACEAPEX_E_CORRUPT);
            if (i == E - 1 && at + v != B.rec_hi[nl - 1]) fail(B.one, ACEAPEX_E_CORRUPT);
        }
        carry += tot;
    }
}

// --------------------------------------------------------------- k_seal

// Batches: after the parse, every record slot of a stream that the parse did
// not fill in this decode (possible only for a corrupt stream) gets length 0,
// so that the level launches may run every slot of a level without checking
// which decode wrote it.  One workgroup per stream.
__global__ void __launch_bounds__(NT) k_seal(Batch B)
{
    const Job &j = B.jobs[blockIdx.x];
    for (uint32_t i = 0; i <= j.max_level; i++) {
        const uint32_t e = j.lv0 + i;
        const uint32_t hi = B.rec_hi[e], filled = min(max(B.cursor[e], B.rec_lo[e]), hi);
        if (filled == hi) continue;
        for (uint32_t r = filled + threadIdx.x; r < hi; r += NT) B.recs[3ull * r + 2] = 0;
        if (threadIdx.x == 0) fail(j, ACEAPEX_E_CORRUPT);
    }
}

// --------------------------------------------------------------- k_level

// One level: each thread takes R records per round (R = 1 while the level
// fits the launch at one record per thread, in workgroups of one wave, so
// that a mid-size level is spread over every CU it can use; R = 2, in
// workgroups of NT threads, for larger levels).
// The level's slots are split into one contiguous part per XCD; the
// workgroups of an XCD sweep its part together, tile after tile, so that the
// destinations and sources they touch at one time share its L2.  Workgroup i
// works on part i % P, which keeps each part on one XCD.
//
// The slots [lo, hi) come from the host's level table as kernel arguments,
// so that no dependent load stands before the first record fetch (lo =
// NO_RANGE: read them from the workspace).  In a batch every slot was filled
// or sealed by k_seal.  A single stream has no seal pass: workgroup 0 of its
// first level launch (check != 0) compares every level's fill cursor with
// the level's end and fails the decode when a slot was left unfilled, which
// only a corrupt stream can do; such a slot's stale record is still bounds-
// checked like any other.  With ordered slots the cursors start at the
// levels' ends; k_oapply has checked that the chunks' counts tile every
// level's range, and a chunk whose parse leaves its slots unfilled fails
// the decode itself.
template <bool BATCH, uint32_t R>
__global__ void __launch_bounds__(NT) k_level(LevelArgs B, uint32_t k, uint32_t lo, uint32_t hi, uint32_t check)
{
    uint32_t R0 = lo, R1 = hi;
    if (lo == NO_RANGE) level_range(B, k, R0, R1);
    if (!BATCH && check && blockIdx.x == 0) {
        for (uint32_t i = threadIdx.x; i <= B.one.max_level; i += blockDim.x)
            if (B.cursor[(size_t)i * CUR_STRIDE] != B.rec_hi[i]) atomicCAS(B.one.status, 0, ACEAPEX_E_CORRUPT);
    }
    const uint32_t G = gridDim.x, P = G < B.xcd_parts ? G : B.xcd_parts;
    const uint32_t x = blockIdx.x % P, w = blockIdx.x / P, W = (G - x + P - 1) / P;
    const uint64_t S = R1 > R0 ? R1 - R0 : 0;
    const uint32_t p0 = R0 + (uint32_t)(S * x / P), p1 = R0 + (uint32_t)(S * (x + 1) / P);
    const uint32_t BS = blockDim.x;
    for (uint32_t r0 = p0 + w * (BS * R) + threadIdx.x;; r0 += W * (BS * R)) {
        if (__ballot(r0 < p1) == 0) break;
        uint8_t *ob[R];
        int32_t *sp[R];
        uint32_t on[R], dst[R], src[R], len[R];
        load_records<BATCH, R>(B, min(r0, p1 - 1), BS, r0 < p1 ? p1 : 0, ob, on, sp, dst, src, len);
        run_records<R>(ob, on, sp, dst, src, len, B.long_copy);
    }
}

// The tail of deep levels [k0, max_level] in one workgroup of NT_TAIL
// threads.  The slot ranges of the first TAIL_RANGES tail levels are read into
// LDS once, so that each level's first round of records is fetched at the
// start of the level before it, with no dependent load in front; after each
// barrier only the source reads remain.
template <bool BATCH>
__global__ void __launch_bounds__(NT_TAIL) k_tail(Batch B, uint32_t k0)
{
    __shared__ uint32_t rlo[TAIL_RANGES], rhi[TAIL_RANGES];
    const uint32_t nt = B.max_level + 1 - k0;  // tail levels
    for (uint32_t i = threadIdx.x; i < min(nt, TAIL_RANGES); i += NT_TAIL) level_range(B, k0 + i, rlo[i], rhi[i]);
    __syncthreads();
    auto range = [&](uint32_t k, uint32_t &lo, uint32_t &hi) {
        if (k - k0 < TAIL_RANGES) {
            lo = rlo[k - k0];
            hi = rhi[k - k0];
        } else {
            level_range(B, k, lo, hi);
        }
    };
    uint32_t nd[ROUND_TAIL], nsr[ROUND_TAIL], nlj[ROUND_TAIL];
    uint32_t lo, hi;
    range(k0, lo, hi);
    fetch_records<ROUND_TAIL>(B, hi ? min(lo + threadIdx.x, hi - 1) : 0, NT_TAIL, lo + threadIdx.x < hi ? hi : 0, nd, nsr, nlj);
    for (uint32_t k = k0; k <= B.max_level; k++) {
        const uint32_t lo_k = lo, hi_k = hi;
        uint32_t dst[ROUND_TAIL], src[ROUND_TAIL], lj[ROUND_TAIL];
#pragma unroll
        for (uint32_t u = 0; u < ROUND_TAIL; u++) { dst[u] = nd[u]; src[u] = nsr[u]; lj[u] = nlj[u]; }
        if (k < B.max_level) {
            range(k + 1, lo, hi);
            fetch_records<ROUND_TAIL>(B, hi ? min(lo + threadIdx.x, hi - 1) : 0, NT_TAIL, lo + threadIdx.x < hi ? hi : 0, nd,
                          nsr, nlj);
        }
        uint8_t *ob[ROUND_TAIL];
        int32_t *sp[ROUND_TAIL];
        uint32_t on[ROUND_TAIL], len[ROUND_TAIL];
        resolve_records<BATCH, ROUND_TAIL>(B, lj, ob, on, sp, len);
        run_records<ROUND_TAIL>(ob, on, sp, dst, src, len, B.long_copy);
        for (uint32_t r = lo_k + ROUND_TAIL * NT_TAIL + threadIdx.x;; r += ROUND_TAIL * NT_TAIL) {
            if (__ballot(r < hi_k) == 0) break;
            load_records<BATCH, ROUND_TAIL>(B, min(r, hi_k - 1), NT_TAIL, r < hi_k ? hi_k : 0, ob, on, sp, dst, src, len);
            run_records<ROUND_TAIL>(ob, on, sp, dst, src, len, B.long_copy);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- level derivation

// A stream without stored levels (the four streams of Sec. 3.2) is decoded
// by deriving each match's level on the device while running the wavefront
// (Sec. 7.1: a match's level is 0 when every source byte is a literal, else
// 1 + the highest level among the matches that wrote its source bytes).
// The parse leaves the matches in stream order, that is by destination.  At
// level k, every queued match scans its source range writer by writer from
// where its scan stopped: a literal run is skipped, a match that has run
// adds its level, and the first match that has not run yet stops the scan --
// the scanning match parks on that writer's list.  A match whose scan reaches
// the end of its source is ready: every writer of its source has run, at
// level k - 1 at the latest, and the writer that woke it at level k - 1, so
// its level is k.  The ready matches then run (their copies read only bytes
// final before level k) and wake the matches parked on them into the queue
// of level k + 1.  Each match parks at most once per writer, so the work is
// the matches plus the writer edges, at two launches per level; once the
// queue is small a single workgroup runs the remaining levels with workgroup
// barriers and stops by itself when the queue is empty.

// A load that reads the value in L2, past this CU's L1: for words that other
// waves change with atomics while a kernel runs.
__device__ __forceinline__ uint32_t load_l2(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The match that writes output byte b (of N), or NONE when a literal does;
// run_end gets the end of the run of bytes that writer (or literal run)
// covers.  B.dpage[b >> PAGE_LOG2] is the first match whose destination is
// at or past the start of b's page; a page of 32 bytes holds a few matches,
// so the walk from there is short.
__device__ __forceinline__ uint32_t writer_of(const Batch &B, uint32_t b, uint32_t M, uint32_t N, uint32_t &run_end)
{
    uint32_t c = B.dpage[b >> PAGE_LOG2];
    while (c < M && B.recs[3ull * c] <= b) c++;  // c: the first match whose destination is past b
    if (c > 0) {
        const uint32_t *r = B.recs + 3ull * (c - 1);
        if ((uint64_t)b < (uint64_t)r[0] + r[2]) {
            run_end = r[0] + r[2];
            return c - 1;
        }
    }
    run_end = c < M ? B.recs[3ull * c] : N;
    return NONE;
}

// Resume the scan of match m's source; true when every writer has run.
__device__ __forceinline__ bool derive_scan(const Batch &B, uint32_t m, uint32_t M, uint32_t N)
{
    const uint32_t *r = B.recs + 3ull * m;
    const uint32_t end = r[1] + r[2];
    uint32_t b = B.dcur[m], mx = B.dmax[m];
    while (b < end) {
        uint32_t run_end;
        const uint32_t w = writer_of(B, b, M, N, run_end);
        if (w != NONE) {
            const uint32_t lv = B.dlevel[w];
            if (lv == NONE) {  // not run yet: park on it
                B.dcur[m] = b;
                B.dmax[m] = mx;
                B.dnext[m] = atomicExch(&B.dhead[w], m);
                return false;
            }
            mx = max(mx, lv + 1);
        }
        b = min(end, max(run_end, b + 1));
    }
    return true;
}

// Append the lanes' items (flag set) to list[*count...] with one atomic per wave.
__device__ __forceinline__ void wave_append(uint32_t *list, uint32_t *count, bool flag, uint32_t item)
{
    const uint64_t mask = __ballot(flag);
    if (!mask) return;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t leader = (uint32_t)__builtin_ctzll(mask);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(mask));
    base = __shfl(base, (int)leader, 64);
    if (flag) list[base + __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u))] = item;
}

// Run the ready match m (NONE for an idle lane) at level k: its copy, its
// level, and the matches parked on it into the queue of level k + 1.  Every
// lane of the wave calls it.
__device__ __forceinline__ void derive_run(const Batch &B, uint32_t m, uint32_t k)
{
    uint8_t *ob[1] = {B.one.out};
    uint32_t on[1] = {B.one.n};
    int32_t *sp[1] = {B.one.status};
    uint32_t dst[1] = {0}, src[1] = {0}, len[1] = {0};
    if (m != NONE) {
        const uint32_t *r = B.recs + 3ull * m;
        dst[0] = r[0];
        src[0] = r[1];
        len[0] = r[2];
    }
    run_records<1>(ob, on, sp, dst, src, len, B.long_copy);
    uint32_t n_wake = 0;
    if (m != NONE) {
        B.dlevel[m] = k;
        for (uint32_t x = load_l2(&B.dhead[m]); x != NONE && n_wake <= B.n_seq; x = B.dnext[x]) n_wake++;
    }
    // the wave's wake-ups: one atomic, then each lane writes its list
    const uint64_t incl = wave_incl_scan64(n_wake);
    const uint64_t total = (uint64_t)__shfl((unsigned long long)incl, 63, 64);
    uint32_t base = 0;
    if ((threadIdx.x & 63) == 63 && total) base = atomicAdd(&B.dcnt[DC_Q + ((k + 1) & 1)], (uint32_t)total);
    base = __shfl(base, 63, 64) + (uint32_t)(incl - n_wake);
    uint32_t *q = B.dq[(k + 1) & 1];
    if (m != NONE) {
        uint32_t i = 0;
        for (uint32_t x = load_l2(&B.dhead[m]); x != NONE && i < n_wake; x = B.dnext[x], i++) q[base + i] = x;
    }
    const uint64_t ran = __ballot(m != NONE);
    if ((threadIdx.x & 63) == 0 && ran) atomicAdd(&B.dcnt[DC_DONE], (uint32_t)__popcll(ran));
}

// Per page of the output (2^PAGE_LOG2 bytes): the first match whose
// destination is at or past the page's start.
__global__ void __launch_bounds__(NT) k_pages(Batch B)
{
    if (*B.one.status) return;
    const uint32_t M = B.n_seq, np = (B.one.n >> PAGE_LOG2) + 1;
    for (uint32_t r = blockIdx.x * NT + threadIdx.x; r <= M; r += gridDim.x * NT) {
        const uint32_t lo = r == 0 ? 0u : (B.recs[3ull * (r - 1)] >> PAGE_LOG2) + 1;
        const uint32_t hi = r == M ? np - 1 : B.recs[3ull * r] >> PAGE_LOG2;
        for (uint32_t pg = lo; pg <= hi && pg < np; pg++) B.dpage[pg] = r;
    }
}

// Level k, scan: every queued match (at level 0, every match) resumes its scan.
__global__ void __launch_bounds__(NT) k_derive_scan(Batch B, uint32_t k)
{
    if (*B.one.status) return;
    const uint32_t M = B.n_seq, N = B.one.n;
    const uint32_t cnt = k == 0 ? M : B.dcnt[DC_Q + (k & 1)];
    if (blockIdx.x == 0 && threadIdx.x == 0) B.dcnt[DC_Q + ((k + 1) & 1)] = 0;
    const uint32_t *q = B.dq[k & 1];
    for (uint32_t i0 = blockIdx.x * NT;; i0 += gridDim.x * NT) {
        const uint32_t i = i0 + threadIdx.x;
        if (__ballot(i < cnt) == 0) break;
        const uint32_t m = i < cnt ? (k == 0 ? i : q[i]) : NONE;
        const bool ready = m < M && derive_scan(B, m, M, N);
        wave_append(B.dready, &B.dcnt[DC_READY + (k & 1)], ready, m);
    }
}

// Level k, run: every ready match runs and wakes the matches parked on it.
__global__ void __launch_bounds__(NT) k_derive_run(Batch B, uint32_t k)
{
    if (*B.one.status) return;
    const uint32_t cnt = B.dcnt[DC_READY + (k & 1)];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        B.dcnt[DC_READY + ((k + 1) & 1)] = 0;
        if (cnt) atomicMax(&B.dcnt[DC_LEVELS], k + 1);
    }
    for (uint32_t i0 = blockIdx.x * NT;; i0 += gridDim.x * NT) {
        const uint32_t i = i0 + threadIdx.x;
        if (__ballot(i < cnt) == 0) break;
        derive_run(B, i < cnt ? B.dready[i] : NONE, k);
    }
}

// The remaining levels from k0 in one workgroup, until the queue is empty.
__global__ void __launch_bounds__(NT_TAIL) k_derive_tail(Batch B, uint32_t k0)
{
    if (*B.one.status) return;
    const uint32_t M = B.n_seq, N = B.one.n;
    for (uint32_t k = k0; k < k0 + M + 1; k++) {
        const uint32_t cnt = load_l2(&B.dcnt[DC_Q + (k & 1)]);
        __syncthreads();
        if (cnt == 0) break;
        if (threadIdx.x == 0) {
            B.dcnt[DC_Q + ((k + 1) & 1)] = 0;
            B.dcnt[DC_READY + (k & 1)] = 0;
        }
        __syncthreads();
        const uint32_t *q = B.dq[k & 1];
        for (uint32_t i0 = 0;; i0 += NT_TAIL) {
            const uint32_t i = i0 + threadIdx.x;
            if (__ballot(i < cnt) == 0) break;
            const uint32_t m = i < cnt ? q[i] : NONE;
            const bool ready = m < M && derive_scan(B, m, M, N);
            wave_append(B.dready, &B.dcnt[DC_READY + (k & 1)], ready, m);
        }
        __syncthreads();
        const uint32_t nr = load_l2(&B.dcnt[DC_READY + (k & 1)]);
        if (threadIdx.x == 0 && nr) atomicMax(&B.dcnt[DC_LEVELS], k + 1);
        for (uint32_t i0 = 0;; i0 += NT_TAIL) {
            const uint32_t i = i0 + threadIdx.x;
            if (__ballot(i < nr) == 0) break;
            derive_run(B, i < nr ? B.dready[i] : NONE, k);
        }
        __syncthreads();
    }
}

// Every match must have run (a stream whose sources form no valid order fails).
// Check of stored levels (Sec. 7.1), on the records in stream order with
// their stored levels (a derive-mode parse with validate set): every writer
// of a match's source bytes must have a lower level than the match, or the
// level launches would run the match before its source is final.  A stream
// that breaks this fails the decode; literal bytes have no writer.
__global__ void __launch_bounds__(NT) k_validate(Batch B)
{
    const uint32_t M = B.n_seq, N = B.one.n;
    if (*B.one.status) return;  // already failed (corrupt sections): the records may be incomplete
    for (uint32_t m = blockIdx.x * NT + threadIdx.x; m < M; m += gridDim.x * NT) {
        const uint32_t *r = B.recs + 3ull * m;
        const uint32_t dst = r[0], src = r[1], len = r[2], lv = B.dlevel[m];
        if ((uint64_t)src + len > dst || (uint64_t)dst + len > N) continue;  // rejected by the parse
        for (uint32_t b = src; b < src + len;) {
            uint32_t run_end;
            const uint32_t w = writer_of(B, b, M, N, run_end);
            if (w != NONE && B.dlevel[w] >= lv) {
                fail(B.one, ACEAPEX_E_CORRUPT);
                break;
            }
            b = min(src + len, max(run_end, b + 1));
        }
    }
}

__global__ void k_derive_final(Batch B)
{
    if (threadIdx.x == 0 && *B.one.status == 0 && B.dcnt[DC_DONE] != B.n_seq) fail(B.one, ACEAPEX_E_CORRUPT);
}

// ----------------------------------------------------------------- host side

thread_local int g_last_hip = 0;

// Kernel timing for measurement (off by default): while enabled, every kernel
// group of a decode is bracketed by two HIP events on the decode's stream.
enum Phase { PH_SETUP, PH_PARSE, PH_LEVELS, PH_COUNT };

struct Timing {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<std::pair<int, size_t>> marks;  // (phase, index of its start event)
};
thread_local Timing g_timing;

hipEvent_t timing_event()
{
    Timing &t = g_timing;
    if (t.used == t.pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        t.pool.push_back(e);
    }
    return t.pool[t.used++];
}

struct PhaseScope {
    int ph;
    hipStream_t st;
    size_t i0 = 0;
    bool on;
    PhaseScope(int p, hipStream_t s, bool timed = true) : ph(p), st(s), on(g_timing.on && timed)
    {
        if (!on) return;
        i0 = g_timing.used;
        hipEvent_t e = timing_event();
        if (!e) { on = false; return; }
        (void)hipEventRecord(e, st);
    }
    ~PhaseScope()
    {
        if (!on) return;
        hipEvent_t e = timing_event();
        if (!e) return;
        (void)hipEventRecord(e, st);
        g_timing.marks.push_back({ph, i0});
    }
};

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
inline uint32_t rd32h(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
inline uint64_t rd64h(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }

int gpu_supported(const aceapex_info &in)
{
    if (in.decoded_bytes >= (1ull << 32) || in.comp_bytes >= (1ull << 32)) return ACEAPEX_E_UNSUPPORTED;
    if (in.block_log2 > BLOCK_LOG2_MAX || in.chunk_log2 > K_LOG2_MAX) return ACEAPEX_E_UNSUPPORTED;
    if ((uint64_t)in.n_seq * 3 >= (1ull << 32)) return ACEAPEX_E_UNSUPPORTED;
    if (in.n_chunks > CHUNKS_MAX) return ACEAPEX_E_UNSUPPORTED;
    return ACEAPEX_OK;
}

int hip_fail(hipError_t e)
{
    g_last_hip = (int)e;
    return ACEAPEX_E_HIP;
}

// The schedule of the level phase (aceapex_tuning).
struct Tune {
    uint32_t level_wg_max = LEVEL_WG_MAX, tail_level_max = TAIL_LEVEL_MAX;
    uint32_t long_copy = LONG_COPY, xcd_parts = XCD_PARTS;
};

bool tune_valid(const Tune &t)
{
    return t.level_wg_max >= 1 && t.level_wg_max <= 65535 && t.long_copy >= 16 && t.long_copy <= (1u << 21) &&
           t.xcd_parts >= 1 && t.xcd_parts <= 8;
}

uint32_t level_wgs(uint64_t records, uint32_t per_thread, const Tune &tn)
{
    const uint64_t per_wg = (uint64_t)NT * per_thread;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(tn.level_wg_max, (records + per_wg - 1) / per_wg));
}

template <bool BATCH>
void launch_level(const Batch &B, uint32_t k, uint64_t cnt, uint32_t lo, uint32_t hi, uint32_t check, const Tune &tn,
                  hipStream_t st)
{
    LevelArgs a;
    a.one.out = B.one.out;
    a.one.status = B.one.status;
    a.one.n = B.one.n;
    a.one.max_level = B.one.max_level;
    a.jobs = B.jobs;
    a.recs = B.recs;
    a.rec_lo = B.rec_lo;
    a.rec_hi = B.rec_hi;
    a.cursor = B.cursor;
    a.level_lo = B.level_lo;
    a.n_jobs = B.n_jobs;
    a.long_copy = B.long_copy;
    a.xcd_parts = B.xcd_parts;
    if (cnt <= (uint64_t)tn.level_wg_max * NT)  // one record per thread, in workgroups of one wave
        hipLaunchKernelGGL((k_level<BATCH, 1>), dim3((uint32_t)std::max<uint64_t>(1, (cnt + LEVEL_WG1 - 1) / LEVEL_WG1)),
                           dim3(LEVEL_WG1), 0, st, a, k, lo, hi, check);
    else
        hipLaunchKernelGGL((k_level<BATCH, ROUND_LEVEL>), dim3(level_wgs(cnt, ROUND_LEVEL, tn)), dim3(NT), 0, st, a, k,
                           lo, hi, check);
}

// Level launches: one per level with records, sized to its count, and the
// deep levels that hold few matches together in the tail workgroup.  counts
// is null when the host does not know them (full-size launch per level, slot
// ranges read on the device); otherwise level k's slots are [sum of counts
// below k, that sum + counts[k]), the layout k_setup (single stream) and the
// batch layout build.
template <typename C>
void launch_levels(const Batch &B, const C *counts, uint64_t n_seq, const Tune &tn, hipStream_t st, bool timed)
{
    PhaseScope ps(PH_LEVELS, st, timed);
    uint32_t tail = B.max_level + 1;
    if (counts) {
        while (tail > 1 && counts[tail - 1] <= tn.tail_level_max) tail--;
        if (B.max_level + 1 - tail < 2) tail = B.max_level + 1;
    }
    uint64_t at = 0;
    uint32_t check = 1;
    for (uint32_t k = 0; k < tail; k++) {
        const uint64_t cnt = counts ? counts[k] : n_seq;
        const uint32_t lo = counts ? (uint32_t)at : NO_RANGE, hi = counts ? (uint32_t)(at + cnt) : 0;
        at += counts ? cnt : 0;
        if (counts && !cnt) continue;
        if (B.jobs)
            launch_level<true>(B, k, cnt, lo, hi, 0, tn, st);
        else
            launch_level<false>(B, k, cnt, lo, hi, counts ? check : 0, tn, st);
        check = 0;
    }
    if (tail <= B.max_level) {
        if (B.jobs)
            hipLaunchKernelGGL(k_tail<true>, dim3(1), dim3(NT_TAIL), 0, st, B, tail);
        else
            hipLaunchKernelGGL(k_tail<false>, dim3(1), dim3(NT_TAIL), 0, st, B, tail);
    }
}

// ---- one stream

struct WsLayout {
    size_t status, chunks, blk_ok, rec_lo, rec_hi, cursor, recs, ocnt, otile, total;
};

// Ordered record slots apply to streams with stored levels and at most
// ORD_LEVELS of them, whose workspace always holds the counts.  They are
// used for such streams of at least ORD_MIN_SEQ matches: on smaller ones the
// four extra launches cost more than the order saves (the 4 MiB Markov
// text, 0.68M matches: 0.114 -> 0.131 ms).  ACEAPEX_ORDERED_SLOTS, read at
// each call, overrides that: "0" never, anything else non-empty always.
bool ordered_eligible(const aceapex_info &in)
{
    return has_table(in) && in.max_level + 1u <= ORD_LEVELS && in.n_chunks > 0 && in.n_seq > 0;
}

bool ordered_slots(const aceapex_info &in)
{
    if (!ordered_eligible(in)) return false;
    const char *v = getenv("ACEAPEX_ORDERED_SLOTS");
    if (v && v[0]) return strcmp(v, "0") != 0;
    return in.n_seq >= ORD_MIN_SEQ;
}

uint64_t ord_tiles(const aceapex_info &in)
{
    return ((uint64_t)(in.max_level + 1) * in.n_chunks + OTILE - 1) / OTILE;
}

WsLayout ws_single(const aceapex_info &in)
{
    WsLayout w;
    size_t o = 0;
    const size_t nl = (size_t)in.max_level + 1;
    w.status = o; o += 256;
    w.chunks = o; o = align256(o + sizeof(ChunkDesc) * (size_t)in.n_chunks);
    w.blk_ok = o; o = align256(o + (size_t)in.n_blocks);
    w.rec_lo = o; o = align256(o + 4 * nl);
    w.rec_hi = o; o = align256(o + 4 * nl);
    w.cursor = o; o = align256(o + 4 * CUR_STRIDE * nl);
    w.recs = o; o = align256(o + 12ull * (size_t)in.n_seq);
    const bool ord = ordered_eligible(in);
    w.ocnt = o; o = align256(o + (ord ? 4 * nl * (size_t)in.n_chunks : 0));
    w.otile = o; o = align256(o + (ord ? 4 * (size_t)ord_tiles(in) : 0));
    w.total = o;
    return w;
}

Job make_job(const aceapex_stream &s, void *d_out, int32_t *status, ChunkDesc *chunks, uint8_t *blk_ok,
             uint32_t c0, uint32_t b0, uint32_t lv0)
{
    const aceapex_info &in = s.info;
    Job j;
    j.comp = (const uint8_t *)s.d_comp;
    j.out = (uint8_t *)d_out;
    j.status = status;
    j.chunks = chunks;
    j.blk_ok = blk_ok;
    j.n = (uint32_t)in.decoded_bytes;
    j.comp_bytes = (uint32_t)in.comp_bytes;
    j.n_blocks = in.n_blocks;
    j.block_log2 = in.block_log2;
    j.min_match = in.min_match;
    j.chunk_log2 = in.chunk_log2;
    j.max_level = in.max_level;
    j.n_chunks = in.n_chunks;
    j.n_seq = in.n_seq;
    j.c0 = c0;
    j.b0 = b0;
    j.lv0 = lv0;
    j.table = has_table(in) ? 1u : 0u;
    j.derive = 0;
    return j;
}

// One launch sequence: one stream (single, kernel arguments name it) or a
// batch (each chunk and record names its stream), with the level counts the
// host schedule needs.
struct Group {
    Batch B;
    std::vector<uint64_t> tot;  // matches per level, or empty when unknown (one launch per level)
    uint64_t n_blocks = 0, n_chunks = 0, n_seq = 0;
    uint32_t n = 0;
    bool single = false;
};

// The kernel arguments of a single-stream decode (no host allocation).
void single_batch(const aceapex_stream &s, void *d_out, uint8_t *ws, int32_t *d_status, Batch &B)
{
    const aceapex_info &in = s.info;
    const WsLayout w = ws_single(in);
    memset(&B, 0, sizeof B);
    B.one = make_job(s, d_out, d_status ? d_status : (int32_t *)(ws + w.status), (ChunkDesc *)(ws + w.chunks),
                     ws + w.blk_ok, 0, 0, 0);
    B.rec_lo = (uint32_t *)(ws + w.rec_lo);
    B.rec_hi = (uint32_t *)(ws + w.rec_hi);
    B.cursor = (uint32_t *)(ws + w.cursor);
    B.recs = (uint32_t *)(ws + w.recs);
    B.ordered = ordered_slots(in) ? 1u : 0u;
    B.ocnt = (uint32_t *)(ws + w.ocnt);
    B.otile = (uint32_t *)(ws + w.otile);
    B.n_jobs = 1;
    B.n_blocks = in.n_blocks;
    B.n_chunks = in.n_chunks;
    B.max_level = in.max_level;
    B.n_seq = in.n_seq;
    if (s.h_levels) {
        B.has_sig = 1;
        for (uint32_t k = 0; k <= in.max_level; k++) B.level_sig += level_mix(k, s.h_levels[k]);
    }
}

void build_single(const aceapex_stream &s, void *d_out, uint8_t *ws, int32_t *d_status, Group &g)
{
    const aceapex_info &in = s.info;
    single_batch(s, d_out, ws, d_status, g.B);
    g.tot.clear();
    if (s.h_levels) g.tot.assign(s.h_levels, s.h_levels + in.max_level + 1);
    g.n_blocks = in.n_blocks;
    g.n_chunks = in.n_chunks;
    g.n_seq = in.n_seq;
    g.n = 1;
    g.single = true;
}

// ---- one stream, levels derived on the device

constexpr uint32_t DERIVE_TAIL = 4096;  // queued matches at or below which one workgroup runs the rest
constexpr uint32_t DERIVE_WG_MAX = 2048;  // workgroups of a derive launch, at most

struct WsDerive {
    size_t status, cnt, chunks, blk_ok, recs, level, head, next, cur, max, q0, q1, ready, page, total;
};

WsDerive ws_derive(const aceapex_info &in)
{
    WsDerive w;
    size_t o = 0;
    const size_t m4 = 4 * (size_t)in.n_seq;
    w.status = o; o += 256;
    w.cnt = o; o += 256;
    w.chunks = o; o = align256(o + sizeof(ChunkDesc) * (size_t)in.n_chunks);
    w.blk_ok = o; o = align256(o + (size_t)in.n_blocks);
    w.recs = o; o = align256(o + 3 * m4);
    w.level = o; o = align256(o + m4);
    w.head = o; o = align256(o + m4);
    w.next = o; o = align256(o + m4);
    w.cur = o; o = align256(o + m4);
    w.max = o; o = align256(o + m4);
    w.q0 = o; o = align256(o + m4);
    w.q1 = o; o = align256(o + m4);
    w.ready = o; o = align256(o + m4);
    w.page = o; o = align256(o + 4 * ((size_t)(in.decoded_bytes >> PAGE_LOG2) + 1));
    w.total = o;
    return w;
}

// ACEAPEX_VALIDATE_LEVELS set to anything but "" or "0": aceapex_decode
// checks a stream's stored levels before it trusts them.
bool validate_levels()
{
    const char *v = getenv("ACEAPEX_VALIDATE_LEVELS");
    return v && v[0] && strcmp(v, "0") != 0;
}

// The workspace of the stream's own decode: stored levels (and their check,
// when asked for) or derived ones.
size_t ws_one(const aceapex_info &in)
{
    if (!has_table(in)) return ws_derive(in).total;
    return validate_levels() ? std::max(ws_single(in).total, ws_derive(in).total) : ws_single(in).total;
}

// Decode one stream deriving its levels on the device (see the level
// derivation kernels); d_levels, when not null, receives each match's level
// in stream order.  The host reads the queue length back every few levels
// (the number of levels is found on the device), so this call returns once
// the last level has been enqueued.
// The kernel arguments of a derive-mode decode (records in stream order).
void derive_batch(const aceapex_stream &s, void *d_out, uint8_t *ws, int32_t *d_status, uint32_t *d_levels,
                  Batch &B)
{
    const aceapex_info &in = s.info;
    const WsDerive w = ws_derive(in);
    memset(&B, 0, sizeof B);
    B.one = make_job(s, d_out, d_status ? d_status : (int32_t *)(ws + w.status), (ChunkDesc *)(ws + w.chunks),
                     ws + w.blk_ok, 0, 0, 0);
    B.one.derive = 1;
    B.recs = (uint32_t *)(ws + w.recs);
    B.dlevel = d_levels ? d_levels : (uint32_t *)(ws + w.level);
    B.dhead = (uint32_t *)(ws + w.head);
    B.dnext = (uint32_t *)(ws + w.next);
    B.dcur = (uint32_t *)(ws + w.cur);
    B.dmax = (uint32_t *)(ws + w.max);
    B.dq[0] = (uint32_t *)(ws + w.q0);
    B.dq[1] = (uint32_t *)(ws + w.q1);
    B.dready = (uint32_t *)(ws + w.ready);
    B.dpage = (uint32_t *)(ws + w.page);
    B.dcnt = (uint32_t *)(ws + w.cnt);
    B.n_jobs = 1;
    B.n_blocks = in.n_blocks;
    B.n_chunks = in.n_chunks;
    B.max_level = 0;  // the parse ranks no levels
    B.n_seq = in.n_seq;
    B.long_copy = LONG_COPY;
    B.xcd_parts = XCD_PARTS;
}

// Setup, derive-mode parse (literals placed, records in stream order) and
// the page index.
void enqueue_derive_parse(const Batch &B, hipStream_t st)
{
    {
        PhaseScope ps(PH_SETUP, st);
        hipLaunchKernelGGL(k_setup, dim3(std::max<uint32_t>(1, std::min<uint32_t>(B.n_blocks, 65535))), dim3(NT), 0,
                           st, B);
    }
    if (B.n_blocks) {
        PhaseScope ps(PH_PARSE, st);
        launch_parse<false>(B, B.n_chunks, st);
        if (B.n_seq)
            hipLaunchKernelGGL(k_pages, dim3(std::min<uint32_t>(DERIVE_WG_MAX, B.n_seq / NT + 1)), dim3(NT), 0, st, B);
    }
}

int launch_derive(const aceapex_stream &s, void *d_out, uint8_t *ws, int32_t *d_status, uint32_t *d_levels,
                  hipStream_t st)
{
    Batch B;
    derive_batch(s, d_out, ws, d_status, d_levels, B);
    const uint32_t M = B.n_seq;
    enqueue_derive_parse(B, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
    if (!M) return ACEAPEX_OK;
    PhaseScope ps(PH_LEVELS, st);
    const uint32_t G = std::max<uint32_t>(1, std::min<uint32_t>(DERIVE_WG_MAX, (M + NT - 1) / NT));
    for (uint32_t k = 0; k <= M;) {
        hipLaunchKernelGGL(k_derive_scan, dim3(G), dim3(NT), 0, st, B, k);
        hipLaunchKernelGGL(k_derive_run, dim3(G), dim3(NT), 0, st, B, k);
        k++;
        if (k <= 2 || k % 4 == 0) {  // the queue of level k
            uint32_t q = 0;
            if ((e = hipMemcpyAsync(&q, B.dcnt + DC_Q + (k & 1), 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
                (e = hipStreamSynchronize(st)) != hipSuccess)
                return hip_fail(e);
            if (!q) break;
            if (q <= DERIVE_TAIL) {
                hipLaunchKernelGGL(k_derive_tail, dim3(1), dim3(NT_TAIL), 0, st, B, k);
                break;
            }
        }
    }
    hipLaunchKernelGGL(k_derive_final, dim3(1), dim3(64), 0, st, B);
    e = hipGetLastError();
    return e == hipSuccess ? ACEAPEX_OK : hip_fail(e);
}

// The check of a stream's stored levels that ACEAPEX_VALIDATE_LEVELS asks
// for: a derive-mode parse that keeps the stored levels, the page index,
// then k_validate.  It leaves its verdict in the status word, which the
// decode that follows keeps.
int launch_validate(const aceapex_stream &s, void *d_out, uint8_t *ws, int32_t *d_status, hipStream_t st)
{
    Batch B;
    derive_batch(s, d_out, ws, d_status, nullptr, B);
    B.one.validate = 1;
    enqueue_derive_parse(B, st);
    if (B.n_seq) {
        PhaseScope ps(PH_PARSE, st);
        hipLaunchKernelGGL(k_validate, dim3(std::min<uint32_t>(DERIVE_WG_MAX, B.n_seq / NT + 1)), dim3(NT), 0, st, B);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ACEAPEX_OK : hip_fail(e);
}

// ---- a batch of streams (all with host level tables), at most JOBS_MAX

struct BatchLayout {
    size_t jobs, rec_lo, rec_hi, level_lo, staged;  // staged = bytes copied from the host
    size_t cursor, blk_job, chunk_job, chunks, blk_ok, status, recs, total;
    uint64_t n_lv, n_blocks, n_chunks, n_seq;
    uint32_t max_level;
};

BatchLayout ws_batch(const aceapex_desc *d, uint32_t n)
{
    BatchLayout w;
    w.n_lv = w.n_blocks = w.n_chunks = w.n_seq = 0;
    w.max_level = 0;
    for (uint32_t i = 0; i < n; i++) {
        const aceapex_info &in = d[i].s.info;
        w.n_lv += (uint64_t)in.max_level + 1;
        w.n_blocks += in.n_blocks;
        w.n_chunks += in.n_chunks;
        w.n_seq += in.n_seq;
        w.max_level = std::max(w.max_level, in.max_level);
    }
    size_t o = 0;
    w.jobs = o; o = align256(o + sizeof(Job) * (size_t)n);
    w.rec_lo = o; o = align256(o + 4 * w.n_lv);
    w.rec_hi = o; o = align256(o + 4 * w.n_lv);
    w.level_lo = o; o = align256(o + 4 * ((size_t)w.max_level + 2));
    w.staged = o;
    w.cursor = o; o = align256(o + 4 * w.n_lv);
    w.blk_job = o; o = align256(o + 4 * w.n_blocks);
    w.chunk_job = o; o = align256(o + 4 * w.n_chunks);
    w.chunks = o; o = align256(o + sizeof(ChunkDesc) * w.n_chunks);
    w.blk_ok = o; o = align256(o + w.n_blocks);
    w.status = o; o = align256(o + 4 * (size_t)n);
    w.recs = o; o = align256(o + 12 * w.n_seq);
    w.total = o;
    return w;
}

// Pinned host buffers that carry the per-batch tables to the device; a
// buffer is reused only after the copy that last read it has run.
struct Staging {
    void *p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};
thread_local Staging g_stage[4];
thread_local unsigned g_stage_next = 0;

int stage_buffer(size_t bytes, Staging *&out)
{
    Staging &s = g_stage[g_stage_next++ % 4];
    hipError_t e;
    if (s.pending && (e = hipEventSynchronize(s.ev)) != hipSuccess) return hip_fail(e);
    s.pending = false;
    if (!s.ev && (e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming)) != hipSuccess) return hip_fail(e);
    if (s.cap < bytes) {
        if (s.p) (void)hipHostFree(s.p);
        s.p = nullptr;
        s.cap = 0;
        if ((e = hipHostMalloc(&s.p, bytes, hipHostMallocDefault)) != hipSuccess) return hip_fail(e);
        s.cap = bytes;
    }
    out = &s;
    return ACEAPEX_OK;
}

// One launch sequence of a batch: the kernel arguments and the level counts
// the host schedule needs.

// Lay out the group d[0, n) in the workspace ws: the host tables (stream
// table, per-(stream, level) slot ranges, per-level slot offsets) are written
// to h, which holds ws_batch(d, n).staged bytes and must then be copied to
// the start of ws; g receives the kernel arguments.
void build_group(const aceapex_desc *d, uint32_t n, uint8_t *ws, uint8_t *h, Group &g)
{
    const BatchLayout w = ws_batch(d, n);
    Job *hj = (Job *)(h + w.jobs);
    uint32_t *lo = (uint32_t *)(h + w.rec_lo), *hi = (uint32_t *)(h + w.rec_hi), *llo = (uint32_t *)(h + w.level_lo);
    // per level: matches over the batch; then each stream's slots inside its level
    g.tot.assign((size_t)w.max_level + 1, 0);
    for (uint32_t i = 0; i < n; i++)
        for (uint32_t k = 0; k <= d[i].s.info.max_level; k++) g.tot[k] += d[i].s.h_levels[k];
    std::vector<uint64_t> at((size_t)w.max_level + 1, 0);
    uint64_t acc = 0;
    for (uint32_t k = 0; k <= w.max_level; k++) {
        llo[k] = (uint32_t)acc;
        at[k] = acc;
        acc += g.tot[k];
    }
    llo[w.max_level + 1] = (uint32_t)acc;
    uint64_t c0 = 0, b0 = 0, lv0 = 0;
    for (uint32_t i = 0; i < n; i++) {
        const aceapex_info &in = d[i].s.info;
        int32_t *status = d[i].d_status ? d[i].d_status : (int32_t *)(ws + w.status) + i;
        hj[i] = make_job(d[i].s, d[i].d_out, status, (ChunkDesc *)(ws + w.chunks) + c0, ws + w.blk_ok + b0,
                         (uint32_t)c0, (uint32_t)b0, (uint32_t)lv0);
        for (uint32_t k = 0; k <= in.max_level; k++) {
            lo[lv0 + k] = (uint32_t)at[k];
            at[k] += d[i].s.h_levels[k];
            hi[lv0 + k] = (uint32_t)at[k];
        }
        c0 += in.n_chunks;
        b0 += in.n_blocks;
        lv0 += (uint64_t)in.max_level + 1;
    }
    Batch &B = g.B;
    memset(&B, 0, sizeof B);
    B.jobs = (const Job *)(ws + w.jobs);
    B.blk_job = (uint32_t *)(ws + w.blk_job);
    B.chunk_job = (uint32_t *)(ws + w.chunk_job);
    B.chunks_all = (const ChunkDesc *)(ws + w.chunks);
    B.rec_lo = (uint32_t *)(ws + w.rec_lo);
    B.rec_hi = (uint32_t *)(ws + w.rec_hi);
    B.cursor = (uint32_t *)(ws + w.cursor);
    B.level_lo = (const uint32_t *)(ws + w.level_lo);
    B.recs = (uint32_t *)(ws + w.recs);
    B.n_jobs = n;
    B.n_blocks = (uint32_t)w.n_blocks;
    B.n_chunks = (uint32_t)w.n_chunks;
    B.max_level = w.max_level;
    B.n_seq = (uint32_t)w.n_seq;
    g.n_blocks = w.n_blocks;
    g.n_chunks = w.n_chunks;
    g.n_seq = w.n_seq;
    g.n = n;
}

// The kernels of a single-stream decode; counts (matches per level) may be
// null.
template <typename C>
void enqueue_single(Batch B, const C *counts, const Tune &tn, hipStream_t st, bool timed)
{
    B.long_copy = tn.long_copy;
    B.xcd_parts = tn.xcd_parts;
    {
        PhaseScope ps(PH_SETUP, st, timed);
        hipLaunchKernelGGL(k_setup, dim3(std::max<uint32_t>(1, std::min<uint32_t>(B.n_blocks, 65535))), dim3(NT), 0,
                           st, B);
    }
    if (B.n_blocks) {
        {
            PhaseScope ps(PH_PARSE, st, timed);
            if (B.ordered) {  // the chunks' first slots per level, before the parse
                const uint32_t tiles = (uint32_t)(((uint64_t)(B.max_level + 1) * B.n_chunks + OTILE - 1) / OTILE);
                const uint32_t per_wg = NT / 64 * CPW;  // chunks per k_count workgroup
                hipLaunchKernelGGL(k_count, dim3((B.n_chunks + per_wg - 1) / per_wg), dim3(NT), 0, st, B);
                hipLaunchKernelGGL(k_otiles, dim3(tiles), dim3(NT), 0, st, B);
                hipLaunchKernelGGL(k_oapply, dim3(tiles), dim3(NT), 0, st, B);
            }
            launch_parse<false>(B, B.n_chunks, st);
        }
        if (B.n_seq) launch_levels(B, counts, B.n_seq, tn, st, timed);
    }
}

// The kernels of one group (nothing else: no copy, no allocation, no
// memset), so that the sequence can be captured into a graph.
void enqueue_group(const Group &g, const Tune &tn, hipStream_t st, bool timed)
{
    const uint64_t *counts = g.tot.empty() ? nullptr : g.tot.data();
    if (g.single) {
        enqueue_single(g.B, counts, tn, st, timed);
        return;
    }
    Batch B = g.B;
    B.long_copy = tn.long_copy;
    B.xcd_parts = tn.xcd_parts;
    {
        PhaseScope ps(PH_SETUP, st, timed);
        hipLaunchKernelGGL(k_map, dim3(g.n), dim3(NT), 0, st, B);
        const uint64_t gs = std::max<uint64_t>(std::max<uint64_t>(1, g.n), std::min<uint64_t>(g.n_blocks, 65535));
        hipLaunchKernelGGL(k_setup, dim3((uint32_t)gs), dim3(NT), 0, st, B);
    }
    if (g.n_chunks) {
        PhaseScope ps(PH_PARSE, st, timed);
        launch_parse<true>(B, (uint32_t)g.n_chunks, st);
    }
    if (g.n_seq) {
        {
            PhaseScope ps(PH_PARSE, st, timed);
            hipLaunchKernelGGL(k_seal, dim3(g.n), dim3(NT), 0, st, B);
        }
        launch_levels(B, counts, g.n_seq, tn, st, timed);
    }
}

int launch_single(const aceapex_stream &s, void *d_out, uint8_t *ws, int32_t *d_status, hipStream_t st,
                  bool keep_verdict = false)
{
    Group g;
    build_single(s, d_out, ws, d_status, g);
    g.B.one.validate = keep_verdict ? 1u : 0u;
    enqueue_group(g, Tune(), st, true);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
    return ACEAPEX_OK;
}

int launch_batch(const aceapex_desc *d, uint32_t n, uint8_t *ws, hipStream_t st)
{
    const BatchLayout w = ws_batch(d, n);
    Staging *sb = nullptr;
    int rc = stage_buffer(w.staged, sb);
    if (rc) return rc;
    Group g;
    build_group(d, n, ws, (uint8_t *)sb->p, g);
    hipError_t e = hipMemcpyAsync(ws, sb->p, w.staged, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e);
    if ((e = hipEventRecord(sb->ev, st)) != hipSuccess) return hip_fail(e);
    sb->pending = true;
    enqueue_group(g, Tune(), st, true);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
    return ACEAPEX_OK;
}

int check_stream_args(const aceapex_stream *s, const void *d_out, uint64_t cap)
{
    if (!s || !s->d_comp) return ACEAPEX_E_INVAL;
    if (((uintptr_t)s->d_comp & 15) || ((uintptr_t)d_out & 15)) return ACEAPEX_E_INVAL;
    if (!info_consistent(s->info)) return ACEAPEX_E_FORMAT;
    int rc = gpu_supported(s->info);
    if (rc) return rc;
    if (s->info.decoded_bytes && !d_out) return ACEAPEX_E_INVAL;
    if (cap < s->info.decoded_bytes) return ACEAPEX_E_CAPACITY;
    if (s->h_levels) {  // a host level table must count every match once (its slots are laid out from it)
        uint64_t sum = 0;
        for (uint32_t k = 0; k <= s->info.max_level; k++) sum += s->h_levels[k];
        if (sum != s->info.n_seq) return ACEAPEX_E_FORMAT;
    }
    return ACEAPEX_OK;
}

// Streams d[0, m) that one launch sequence takes, m >= 1: at most JOBS_MAX
// streams, and batch-wide record, chunk, block and level counts that keep
// every 32-bit index of the batch layout (and the k_parse grid) in range.
uint32_t group_size(const aceapex_desc *d, uint32_t n)
{
    uint64_t seq = 0, chunks = 0, blocks = 0, levels = 0;
    uint32_t m = 0;
    while (m < n && m < JOBS_MAX) {
        const aceapex_info &in = d[m].s.info;
        seq += in.n_seq;
        chunks += in.n_chunks;
        blocks += in.n_blocks;
        levels += (uint64_t)in.max_level + 1;
        if (m && (seq * 3 >= (1ull << 32) || chunks > CHUNKS_MAX || blocks >= (1ull << 31) || levels >= (1ull << 31)))
            break;
        m++;
    }
    return m;
}

// Workspace of decode_many: the batched layout per group of streams, or one
// single-stream layout per stream, whichever is larger.
size_t many_bytes(const aceapex_desc *d, uint32_t n)
{
    size_t batched = 0, single = 0;
    for (uint32_t i = 0, m; i < n; i += m) {
        m = group_size(d + i, n - i);
        batched += ws_batch(d + i, m).total;
    }
    for (uint32_t i = 0; i < n; i++) single += ws_one(d[i].s.info);
    return std::max(batched, single);
}

// A batch laid out once in its workspace; launches only enqueue kernels.
struct PlanImpl {
    std::vector<Group> groups;
    Tune tune;
    hipStream_t cap = nullptr;       // private stream the graph is captured on
    hipGraphExec_t exec = nullptr;   // captured launch sequence, made on first use
    int device = 0;
};

void plan_drop_graph(PlanImpl *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    p->exec = nullptr;
}

Tune tune_from(const aceapex_tuning &t)
{
    Tune tn;
    tn.level_wg_max = t.level_wg_max;
    tn.tail_level_max = t.tail_level_max;
    tn.long_copy = t.long_copy;
    tn.xcd_parts = t.xcd_parts;
    return tn;
}

void tune_to(const Tune &tn, aceapex_tuning *t)
{
    t->level_wg_max = tn.level_wg_max;
    t->tail_level_max = tn.tail_level_max;
    t->long_copy = tn.long_copy;
    t->xcd_parts = tn.xcd_parts;
}

int enqueue_plan(const PlanImpl *p, const Tune &tn, hipStream_t st, bool timed)
{
    for (const Group &g : p->groups) enqueue_group(g, tn, st, timed);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ACEAPEX_OK : hip_fail(e);
}

}  // namespace

void aceapex_impl::set_last_hip_error(int e) { g_last_hip = e; }

// Workspace of aceapex_decode_noalloc: one library-static device array that
// every device the library runs on holds until the process ends.  In host
// code the symbol is only a stand-in; the array is reached through the
// address hipGetSymbolAddress returns on each device (scratch_on_device).
static constexpr size_t SCRATCH_BYTES = ACEAPEX_NOALLOC_WORKSPACE_MAX;
static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_at[SCRATCH_DEVICES];  // device address of scratch, per device, once known

// The address of the scratch array on the current device, looked up once per
// device (with that device current) and kept.
int scratch_on_device(uint8_t **at)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= SCRATCH_DEVICES) return ACEAPEX_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_at[dev]) {
        void *p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return hip_fail(e);
        if (!p) return ACEAPEX_E_HIP;
        g_scratch_at[dev] = (uint8_t *)p;
    }
    *at = g_scratch_at[dev];
    return ACEAPEX_OK;
}

}  // namespace

extern "C" {

int aceapex_level_table(const void *h_stream_prefix, size_t h_len, uint32_t *counts, uint32_t n)
{
    aceapex_info in;
    int rc = aceapex_probe(h_stream_prefix, h_len, &in);
    if (rc) return rc;
    if (!has_table(in)) return ACEAPEX_E_FORMAT;  // the four streams of Sec. 3.2 carry no level table
    const uint64_t at = HDR + 16ull * (in.n_blocks + 1ull), cnt = (uint64_t)in.max_level + 1;
    if (!counts || n < cnt || h_len < at + 4 * cnt) return ACEAPEX_E_INVAL;
    uint64_t sum = 0;
    for (uint64_t i = 0; i < cnt; i++) {
        counts[i] = rd32h((const uint8_t *)h_stream_prefix + at + 4 * i);
        sum += counts[i];
    }
    return sum == in.n_seq ? ACEAPEX_OK : ACEAPEX_E_FORMAT;
}

size_t aceapex_workspace_bytes(const aceapex_desc *h_descs, uint32_t n)
{
    if (!h_descs) return 0;
    for (uint32_t i = 0; i < n; i++)
        if (!info_consistent(h_descs[i].s.info)) return 0;
    return many_bytes(h_descs, n);
}

int aceapex_decode(const aceapex_stream *stream, void *d_out, uint64_t out_capacity, void *d_workspace,
                   size_t ws_bytes, int32_t *d_status, void *hip_stream)
{
    int rc = check_stream_args(stream, d_out, out_capacity);
    if (rc) return rc;
    const size_t need = ws_one(stream->info);
    if (!d_workspace || ((uintptr_t)d_workspace & 255) || ws_bytes < need) return ACEAPEX_E_WORKSPACE;
    if (!has_table(stream->info))  // no stored levels: derived on the device
        return launch_derive(*stream, d_out, (uint8_t *)d_workspace, d_status, nullptr, (hipStream_t)hip_stream);
    const bool check = validate_levels();
    if (check && (rc = launch_validate(*stream, d_out, (uint8_t *)d_workspace, d_status, (hipStream_t)hip_stream)))
        return rc;
    return launch_single(*stream, d_out, (uint8_t *)d_workspace, d_status, (hipStream_t)hip_stream, check);
}

int aceapex_decode_derive(const aceapex_stream *stream, void *d_out, uint64_t out_capacity, void *d_workspace,
                          size_t ws_bytes, uint32_t *d_levels, int32_t *d_status, void *hip_stream)
{
    int rc = check_stream_args(stream, d_out, out_capacity);
    if (rc) return rc;
    if (((uintptr_t)d_levels & 3)) return ACEAPEX_E_INVAL;
    const size_t need = ws_derive(stream->info).total;
    if (!d_workspace || ((uintptr_t)d_workspace & 255) || ws_bytes < need) return ACEAPEX_E_WORKSPACE;
    return launch_derive(*stream, d_out, (uint8_t *)d_workspace, d_status, d_levels, (hipStream_t)hip_stream);
}

size_t aceapex_workspace_bytes_derive(const aceapex_info *info)
{
    if (!info || !info_consistent(*info)) return 0;
    return ws_derive(*info).total;
}

int aceapex_decode_noalloc(const aceapex_stream *stream, void *d_out, uint64_t out_capacity, int32_t *d_status,
                           void *hip_stream)
{
    int rc = check_stream_args(stream, d_out, out_capacity);
    if (rc) return rc;
    if (!has_table(stream->info)) return ACEAPEX_E_UNSUPPORTED;  // derived levels need host read-backs
    if (ws_single(stream->info).total > SCRATCH_BYTES) return ACEAPEX_E_WORKSPACE;
    uint8_t *ws = nullptr;
    if ((rc = scratch_on_device(&ws))) return rc;
    Batch B;
    single_batch(*stream, d_out, ws, d_status, B);
    // the same kernels as aceapex_decode, untimed (timing would create events)
    enqueue_single(B, stream->h_levels, Tune(), (hipStream_t)hip_stream, false);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ACEAPEX_OK : hip_fail(e);
}

int aceapex_decode_many(const aceapex_desc *h_descs, uint32_t n, void *d_workspace, size_t ws_bytes,
                        void *hip_stream)
{
    if (!h_descs && n) return ACEAPEX_E_INVAL;
    bool tables = true;
    uint32_t n_free = 0;  // streams without stored levels
    for (uint32_t i = 0; i < n; i++) {
        int rc = check_stream_args(&h_descs[i].s, h_descs[i].d_out, h_descs[i].out_capacity);
        if (rc) return rc;
        if (!has_table(h_descs[i].s.info)) {
            n_free++;
            continue;
        }
        tables = tables && h_descs[i].s.h_levels;
    }
    if (n && (!d_workspace || ((uintptr_t)d_workspace & 255) || ws_bytes < many_bytes(h_descs, n)))
        return ACEAPEX_E_WORKSPACE;
    hipStream_t st = (hipStream_t)hip_stream;
    // the streams with stored levels (all of them, when none lacks levels)
    std::vector<aceapex_desc> kept;
    const aceapex_desc *d = h_descs;
    uint32_t m_levels = n;
    if (n_free) {
        try {
            for (uint32_t i = 0; i < n; i++)
                if (has_table(h_descs[i].s.info)) kept.push_back(h_descs[i]);
        } catch (const std::bad_alloc &) {
            return ACEAPEX_E_NOMEM;
        }
        d = kept.data();
        m_levels = (uint32_t)kept.size();
    }
    uint8_t *ws = (uint8_t *)d_workspace;
    if (!tables) {  // without the host level tables: one stream after the other
        for (uint32_t i = 0; i < m_levels; i++) {
            int rc = launch_single(d[i].s, d[i].d_out, ws, d[i].d_status, st);
            if (rc) return rc;
            ws += ws_single(d[i].s.info).total;
        }
    } else {
        for (uint32_t i = 0, m; i < m_levels; i += m) {
            m = group_size(d + i, m_levels - i);
            int rc = launch_batch(d + i, m, ws, st);
            if (rc) return rc;
            ws += ws_batch(d + i, m).total;
        }
    }
    // then the streams without levels, one after the other from the start of
    // the workspace (the launches above come first on the stream): their
    // derivation reads counters back, so the call returns once they are done
    for (uint32_t i = 0; i < n && n_free; i++) {
        if (has_table(h_descs[i].s.info)) continue;
        int rc = launch_derive(h_descs[i].s, h_descs[i].d_out, (uint8_t *)d_workspace, h_descs[i].d_status, nullptr, st);
        if (rc) return rc;
    }
    return ACEAPEX_OK;
}

const char *aceapex_strerror(int code)
{
    switch (code) {
    case ACEAPEX_OK: return "ok";
    case ACEAPEX_E_INVAL: return "invalid argument";
    case ACEAPEX_E_FORMAT: return "not a valid stream header";
    case ACEAPEX_E_CORRUPT: return "corrupt stream";
    case ACEAPEX_E_CAPACITY: return "output buffer too small";
    case ACEAPEX_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case ACEAPEX_E_UNSUPPORTED: return "stream outside the limits of this decoder";
    case ACEAPEX_E_TIMEOUT: return "device wait timed out";
    case ACEAPEX_E_HIP: return "HIP runtime error";
    case ACEAPEX_E_NOMEM: return "host allocation failed";
    default: return "unknown error";
    }
}

int aceapex_last_hip_error(void) { return g_last_hip; }

void aceapex_tuning_defaults(aceapex_tuning *t)
{
    if (t) tune_to(Tune(), t);
}

int aceapex_plan_create(const aceapex_desc *h_descs, uint32_t n, void *d_workspace, size_t ws_bytes,
                        const aceapex_tuning *tuning, void *hip_stream, aceapex_plan **plan)
{
    if (!plan || (!h_descs && n)) return ACEAPEX_E_INVAL;
    *plan = nullptr;
    for (uint32_t i = 0; i < n; i++) {
        int rc = check_stream_args(&h_descs[i].s, h_descs[i].d_out, h_descs[i].out_capacity);
        if (rc) return rc;
        if (!has_table(h_descs[i].s.info)) return ACEAPEX_E_UNSUPPORTED;
        if (!h_descs[i].s.h_levels) return ACEAPEX_E_INVAL;
    }
    if (n && (!d_workspace || ((uintptr_t)d_workspace & 255) || ws_bytes < many_bytes(h_descs, n)))
        return ACEAPEX_E_WORKSPACE;
    Tune tn;
    if (tuning) {
        tn = tune_from(*tuning);
        if (!tune_valid(tn)) return ACEAPEX_E_INVAL;
    }
    PlanImpl *p = new (std::nothrow) PlanImpl;
    if (!p) return ACEAPEX_E_NOMEM;
    p->tune = tn;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e);
    }
    hipStream_t st = (hipStream_t)hip_stream;
    uint8_t *ws = (uint8_t *)d_workspace;
    if (n == 1) {  // one stream: the single-stream kernels, nothing staged
        Group g;
        build_single(h_descs[0].s, h_descs[0].d_out, ws, h_descs[0].d_status, g);
        p->groups.push_back(std::move(g));
        *plan = (aceapex_plan *)p;
        return ACEAPEX_OK;
    }
    std::vector<uint8_t> h;
    for (uint32_t i = 0, m; i < n; i += m) {
        m = group_size(h_descs + i, n - i);
        const BatchLayout w = ws_batch(h_descs + i, m);
        h.assign(w.staged, 0);
        Group g;
        build_group(h_descs + i, m, ws, h.data(), g);
        if ((e = hipMemcpyAsync(ws, h.data(), w.staged, hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess) {
            delete p;
            return hip_fail(e);
        }
        p->groups.push_back(std::move(g));
        ws += w.total;
    }
    *plan = (aceapex_plan *)p;
    return ACEAPEX_OK;
}

int aceapex_plan_launch(aceapex_plan *plan, void *hip_stream)
{
    PlanImpl *p = (PlanImpl *)plan;
    if (!p) return ACEAPEX_E_INVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return hip_fail(e);
    return enqueue_plan(p, p->tune, st, cs == hipStreamCaptureStatusNone);
}

int aceapex_plan_launch_graph(aceapex_plan *plan, void *hip_stream)
{
    PlanImpl *p = (PlanImpl *)plan;
    if (!p) return ACEAPEX_E_INVAL;
    hipError_t e;
    if (!p->exec) {
        if (!p->cap && (e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e);
        if ((e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) return hip_fail(e);
        for (const Group &g : p->groups) enqueue_group(g, p->tune, p->cap, false);
        hipGraph_t graph = nullptr;
        const hipError_t le = hipGetLastError();
        e = hipStreamEndCapture(p->cap, &graph);
        if (le != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(le != hipSuccess ? le : e);
        }
        e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            p->exec = nullptr;
            return hip_fail(e);
        }
    }
    if ((e = hipGraphLaunch(p->exec, (hipStream_t)hip_stream)) != hipSuccess) return hip_fail(e);
    return ACEAPEX_OK;
}

int aceapex_plan_set_tuning(aceapex_plan *plan, const aceapex_tuning *tuning)
{
    PlanImpl *p = (PlanImpl *)plan;
    if (!p || !tuning) return ACEAPEX_E_INVAL;
    const Tune tn = tune_from(*tuning);
    if (!tune_valid(tn)) return ACEAPEX_E_INVAL;
    p->tune = tn;
    plan_drop_graph(p);
    return ACEAPEX_OK;
}

int aceapex_plan_get_tuning(const aceapex_plan *plan, aceapex_tuning *tuning)
{
    const PlanImpl *p = (const PlanImpl *)plan;
    if (!p || !tuning) return ACEAPEX_E_INVAL;
    tune_to(p->tune, tuning);
    return ACEAPEX_OK;
}

int aceapex_plan_tune(aceapex_plan *plan, void *hip_stream, uint32_t reps, aceapex_tuning *best)
{
    PlanImpl *p = (PlanImpl *)plan;
    if (!p) return ACEAPEX_E_INVAL;
    reps = std::max<uint32_t>(1, reps);
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e);
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e);
    }
    // time of one launch of the plan under tn: one warm-up, then the mean of reps
    auto timed_run = [&](const Tune &tn, float &ms) -> int {
        int rc = enqueue_plan(p, tn, st, false);
        if (rc) return rc;
        if ((e = hipEventRecord(e0, st)) != hipSuccess) return hip_fail(e);
        for (uint32_t r = 0; r < reps; r++)
            if ((rc = enqueue_plan(p, tn, st, false))) return rc;
        if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
            return hip_fail(e);
        ms /= (float)reps;
        return ACEAPEX_OK;
    };
    // coordinate descent over the knobs, one at a time, from the current schedule
    static const uint32_t wg[] = {512, 1024, 2048, 4096, 8192};
    static const uint32_t tail[] = {0, 1024, 2048, 8192, 32768};
    static const uint32_t longc[] = {32, 64, 128, 512};
    static const uint32_t parts[] = {1, 2, 4, 8};
    Tune cur = p->tune;
    float best_ms = 0.f;
    int rc = timed_run(cur, best_ms);
    auto sweep = [&](uint32_t Tune::*knob, const uint32_t *vals, size_t nv) {
        for (size_t i = 0; i < nv && !rc; i++) {
            if (cur.*knob == vals[i]) continue;
            Tune t = cur;
            t.*knob = vals[i];
            float ms = 0.f;
            rc = timed_run(t, ms);
            if (!rc && ms < 0.99f * best_ms) {  // keep a change only when it is clearly faster
                best_ms = ms;
                cur = t;
            }
        }
    };
    sweep(&Tune::level_wg_max, wg, sizeof wg / sizeof wg[0]);
    sweep(&Tune::tail_level_max, tail, sizeof tail / sizeof tail[0]);
    sweep(&Tune::long_copy, longc, sizeof longc / sizeof longc[0]);
    sweep(&Tune::xcd_parts, parts, sizeof parts / sizeof parts[0]);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    p->tune = cur;
    plan_drop_graph(p);
    if (best) tune_to(cur, best);
    return ACEAPEX_OK;
}

void aceapex_plan_destroy(aceapex_plan *plan)
{
    PlanImpl *p = (PlanImpl *)plan;
    if (!p) return;
    plan_drop_graph(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    delete p;
}

int aceapex_timing(int enable)
{
    Timing &t = g_timing;
    t.on = enable != 0;
    t.used = 0;
    t.marks.clear();
    return ACEAPEX_OK;
}

int aceapex_timing_read(float *ms, uint32_t *count, uint32_t n)
{
    if (!ms || !count) return ACEAPEX_E_INVAL;
    Timing &t = g_timing;
    for (uint32_t i = 0; i < n; i++) { ms[i] = 0.f; count[i] = 0; }
    if (t.used) {
        hipError_t e = hipEventSynchronize(t.pool[t.used - 1]);
        if (e != hipSuccess) return hip_fail(e);
    }
    for (const auto &m : t.marks) {
        float v = 0.f;
        hipError_t e = hipEventElapsedTime(&v, t.pool[m.second], t.pool[m.second + 1]);
        if (e != hipSuccess) return hip_fail(e);
        if ((uint32_t)m.first < n) { ms[m.first] += v; count[m.first]++; }
    }
    t.used = 0;
    t.marks.clear();
    return ACEAPEX_OK;
}

}  // extern "C"
