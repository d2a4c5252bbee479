// MI355X (gfx950) decoder for absolute-offset LZ77 streams (ACEAPEX,
// arXiv 2606.04268) behind the C ABI of include/aceapex.h.
//
// Pipeline for one stream (all on one HIP stream, no host round trip):
//   k_init     clear level counters, status and the chunk descriptors
//   k_setup    one workgroup per block: check the block table, block header
//              and chunk index, and write a 48-byte descriptor per chunk
//              (absolute slices of cmd/len/lvl/lit/off and the output span)
//   k_phase1   one workgroup per chunk: LEB128-decode cmd/len/lvl from LDS,
//              prefix-scan run and match lengths into output and literal
//              offsets, scatter the literal runs (Sec. 3.2) and count the
//              matches of every level >= 1
//   k_lscan    prefix over the level histogram -> bucket bases
//   k_phase2   one workgroup per chunk: parse again, run every level-0 match
//              at once (its source bytes are literals, already final), and
//              append each deeper match to the bucket of its level
//   k_level    for k = 1..max_level: run the bucket of level k.  Level k reads
//              only bytes written by literals or by levels < k (Sec. 7.1), so
//              the copies of one level are independent of each other.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "aceapex.h"

namespace {

constexpr int NT = 256;                     // threads per workgroup
constexpr uint32_t K_LOG2_MAX = 10;         // sequences per chunk, at most
constexpr uint32_t K_MAX = 1u << K_LOG2_MAX;
constexpr uint32_t STAGE = 4 * (K_MAX + 1) + 12;  // one LEB128 slice, 4 bytes per value at most
constexpr uint32_t STAGE_PAD = (STAGE + 15) & ~15u;
constexpr uint32_t LVL_LDS = 1024;          // levels counted in LDS; deeper ones use global atomics
constexpr uint32_t SKIP = 0xffffffffu;      // descriptor of a chunk that must not be executed
constexpr uint32_t HDR = 64, BLKHDR = 32, CHUNK_ENT = 32;
constexpr uint32_t BLOCK_LOG2_MAX = 20;
constexpr int LEVEL_GRID = 1024;            // workgroups of a per-level launch

typedef uint16_t u16u __attribute__((aligned(1)));
typedef uint32_t u32u __attribute__((aligned(1)));
typedef uint64_t u64u __attribute__((aligned(1)));
struct __attribute__((aligned(1))) u128u { uint32_t a, b, c, d; };

struct ChunkDesc {
    uint32_t out_base, out_len;   // absolute output span of the chunk
    uint32_t cmd_at, cmd_n;       // byte slices inside the compressed stream
    uint32_t len_at, len_n;
    uint32_t lvl_at, lvl_n;
    uint32_t lit_at, lit_n;
    uint32_t off_at;              // first off[] entry of the chunk
    uint32_t nseq_last;           // sequences in the chunk | (1 << 31) if it holds the trailing run
};
static_assert(sizeof(ChunkDesc) == 48, "descriptor layout");

struct Job {
    const uint8_t *comp;
    uint8_t *out;
    uint32_t n, comp_bytes;
    uint32_t n_blocks, block_log2, min_match, chunk_log2;
    uint32_t max_level, n_chunks, n_seq, n_deep;
    ChunkDesc *chunks;   // [n_chunks]
    uint32_t *hist;      // [max_level + 1] deep matches per level
    uint32_t *base;      // [max_level + 2] bucket starts
    uint32_t *cursor;    // [max_level + 1] next free slot per bucket
    uint32_t *recs;      // [3 * n_deep] (dst, src, len) of every deep match
    int32_t *status;
};

__device__ __forceinline__ uint32_t ld32(const uint8_t *p) { return *(const u32u *)p; }
__device__ __forceinline__ uint64_t ld64(const uint8_t *p) { return *(const u64u *)p; }
__device__ __forceinline__ uint64_t pad16(uint64_t v) { return (v + 15) & ~(uint64_t)15; }

__device__ __forceinline__ void fail(const Job &j, int code)
{
    atomicCAS(j.status, 0, code);
}

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

// ------------------------------------------------------------ workgroup scans

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
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

// ------------------------------------------------------------------ LDS state

struct Lds {
    union {
        uint8_t stage[3][STAGE_PAD];   // raw cmd/len/lvl slices
        uint64_t scan[K_MAX + 1];      // per run: (output offset << 32) | literal offset
    } u;
    uint32_t run[K_MAX + 1];
    uint32_t mlen[K_MAX];
    uint32_t lvl[K_MAX];
    uint16_t rank[K_MAX];
    uint32_t hist[LVL_LDS];
    uint32_t hbase[LVL_LDS];
    uint64_t tmp[NT / 64];
    ChunkDesc d;
    uint32_t bad;
};

// Decode exactly cnt LEB128 values from b[0, nb) into vals; false (uniform
// over the workgroup) if the slice does not hold exactly cnt well-formed values.
__device__ bool wg_varints(Lds &L, const uint8_t *b, uint32_t nb, uint32_t cnt, uint32_t *vals)
{
    const uint32_t t = threadIdx.x;
    const uint32_t seg = (nb + NT - 1) / NT;
    const uint32_t s0 = min(nb, t * seg), s1 = min(nb, s0 + seg);
    uint32_t c = 0;
    for (uint32_t i = s0; i < s1; i++) c += b[i] < 0x80;
    uint64_t tot;
    uint32_t idx = (uint32_t)wg_excl_scan64(c, L.tmp, tot);
    if (tot != cnt || (nb && b[nb - 1] >= 0x80)) return false;
    bool ok = true;
    for (uint32_t i = s0; i < s1; i++) {
        if (b[i] >= 0x80) continue;
        uint32_t k = i, ncont = 0;
        while (k > 0 && b[k - 1] >= 0x80 && ncont < 4) { k--; ncont++; }
        if (ncont > 3) { ok = false; break; }
        uint32_t v = 0;
        for (uint32_t q = 0; q <= ncont; q++) v |= (uint32_t)(b[k + q] & 0x7f) << (7 * q);
        vals[idx++] = v;
    }
    if (!ok) L.bad = 1;
    __syncthreads();
    return L.bad == 0;
}

// stage one slice of the compressed stream into LDS (exact bytes, no over-read)
__device__ __forceinline__ void stage_slice(uint8_t *dst, const uint8_t *src, uint32_t n)
{
    for (uint32_t i = threadIdx.x * 4; i < n; i += NT * 4) {
        if (i + 4 <= n) {
            *(uint32_t *)(dst + i) = ld32(src + i);
        } else {
            for (uint32_t k = i; k < n; k++) dst[k] = src[k];
        }
    }
}

// Load and parse the chunk g into LDS.  Returns the number of cmd values
// (> 0) or 0 when the chunk is skipped or corrupt (uniform).
__device__ uint32_t parse_chunk(const Job &j, uint32_t g, Lds &L, bool want_lvl)
{
    const uint32_t t = threadIdx.x;
    if (t < 12) ((uint32_t *)&L.d)[t] = ((const uint32_t *)(j.chunks + g))[t];
    if (t == 0) L.bad = 0;
    __syncthreads();
    const ChunkDesc d = L.d;
    if (d.nseq_last == SKIP) return 0;
    const uint32_t ns = d.nseq_last & 0x7fffffffu;
    const uint32_t ncmd = ns + (d.nseq_last >> 31);
    stage_slice(L.u.stage[0], j.comp + d.cmd_at, d.cmd_n);
    stage_slice(L.u.stage[1], j.comp + d.len_at, d.len_n);
    if (want_lvl) stage_slice(L.u.stage[2], j.comp + d.lvl_at, d.lvl_n);
    __syncthreads();
    bool ok = wg_varints(L, L.u.stage[0], d.cmd_n, ncmd, L.run);
    ok = ok && wg_varints(L, L.u.stage[1], d.len_n, ns, L.mlen);
    if (want_lvl) ok = ok && wg_varints(L, L.u.stage[2], d.lvl_n, ns, L.lvl);
    if (!ok) {
        if (t == 0) fail(j, ACEAPEX_E_CORRUPT);
        return 0;
    }
    __syncthreads();  // the stage area is reused for the scan below
    // per run: output bytes it spans together with its match, and literal bytes
    const uint32_t per = (ncmd + NT - 1) / NT;
    const uint32_t e0 = min(ncmd, t * per), e1 = min(ncmd, e0 + per);
    uint64_t acc = 0;
    bool bad = false;
    for (uint32_t e = e0; e < e1; e++) {
        uint32_t r = L.run[e];
        uint32_t m = 0;
        if (e < ns) {
            m = L.mlen[e] + j.min_match;
            L.mlen[e] = m;
            if (m > d.out_len || (want_lvl && L.lvl[e] > j.max_level)) bad = true;
        }
        if (r > d.out_len) bad = true;
        acc += ((uint64_t)(r + m) << 32) | r;
    }
    uint64_t tot;
    uint64_t ex = wg_excl_scan64(bad ? 0 : acc, L.tmp, tot);
    for (uint32_t e = e0; e < e1; e++) {
        L.u.scan[e] = ex;
        uint32_t r = L.run[e];
        uint32_t m = e < ns ? L.mlen[e] : 0;
        ex += ((uint64_t)(r + m) << 32) | r;
    }
    if (bad) L.bad = 1;
    __syncthreads();
    if (L.bad || (uint32_t)(tot >> 32) != d.out_len || (uint32_t)tot != d.lit_n) {
        if (t == 0) fail(j, ACEAPEX_E_CORRUPT);
        return 0;
    }
    return ncmd;
}

// --------------------------------------------------------------------- kernels

__global__ void k_init(Job j)
{
    const uint32_t gid = blockIdx.x * NT + threadIdx.x, gsz = gridDim.x * NT;
    if (gid == 0) *j.status = 0;
    for (uint32_t i = gid; i <= j.max_level; i += gsz) {
        j.hist[i] = 0;
        j.cursor[i] = 0;
    }
    for (uint32_t i = gid; i < j.n_chunks; i += gsz) j.chunks[i].nseq_last = SKIP;
}

__global__ void __launch_bounds__(NT) k_setup(Job j)
{
    __shared__ uint32_t ok_blk;
    const uint64_t B = (uint64_t)1 << j.block_log2;
    const uint32_t K = 1u << j.chunk_log2;
    const uint64_t tbl_end = HDR + 16ull * (j.n_blocks + 1);
    for (uint32_t b = blockIdx.x; b < j.n_blocks; b += gridDim.x) {
        const uint8_t *tb = j.comp + HDR + 16ull * b;
        const uint64_t o0 = ld64(tb), o1 = ld64(tb + 16);
        const uint32_t sb0 = ld32(tb + 8), cb0 = ld32(tb + 12), sb1 = ld32(tb + 24), cb1 = ld32(tb + 28);
        bool ok = (o0 & 15) == 0 && o0 >= tbl_end && o1 >= o0 + BLKHDR && o1 <= j.comp_bytes &&
                  cb1 >= cb0 && cb1 <= j.n_chunks && sb1 >= sb0 && sb1 <= j.n_seq;
        if (b == 0) ok = ok && cb0 == 0 && sb0 == 0;
        if (b + 1 == j.n_blocks) ok = ok && o1 == j.comp_bytes && cb1 == j.n_chunks && sb1 == j.n_seq;
        uint32_t ns = 0, nl = 0, nc = 0, cmdb = 0, lenb = 0, lvlb = 0;
        uint64_t off_at = 0, cmd_at = 0, len_at = 0, lvl_at = 0, lit_at = 0;
        if (ok) {
            const uint8_t *bh = j.comp + o0;
            ns = ld32(bh); nl = ld32(bh + 4); nc = ld32(bh + 8);
            uint32_t bmax = ld32(bh + 12);
            cmdb = ld32(bh + 16); lenb = ld32(bh + 20); lvlb = ld32(bh + 24);
            uint32_t want_nc = ns ? (uint32_t)((ns + (uint64_t)K - 1) / K) : 1u;
            ok = nc == cb1 - cb0 && ns == sb1 - sb0 && nc == want_nc && bmax <= j.max_level;
            off_at = o0 + BLKHDR + (uint64_t)CHUNK_ENT * nc;
            cmd_at = off_at + pad16(4ull * ns);
            len_at = cmd_at + pad16(cmdb);
            lvl_at = len_at + pad16(lenb);
            lit_at = lvl_at + pad16(lvlb);
            ok = ok && lit_at + pad16(nl) == o1;
        }
        if (threadIdx.x == 0) ok_blk = ok;
        __syncthreads();
        if (!ok_blk) {
            if (threadIdx.x == 0) fail(j, ACEAPEX_E_CORRUPT);
            __syncthreads();
            continue;
        }
        const uint32_t blen = (uint32_t)min(B, (uint64_t)j.n - b * B);
        for (uint32_t c = threadIdx.x; c < nc; c += NT) {
            const uint8_t *e = j.comp + o0 + BLKHDR + (uint64_t)CHUNK_ENT * c;
            uint32_t c0 = ld32(e), l0 = ld32(e + 4), v0 = ld32(e + 8), q0 = ld32(e + 12), d0 = ld32(e + 16);
            uint32_t c1 = cmdb, l1 = lenb, v1 = lvlb, q1 = nl, d1 = blen;
            if (c + 1 < nc) { c1 = ld32(e + 32); l1 = ld32(e + 36); v1 = ld32(e + 40); q1 = ld32(e + 44); d1 = ld32(e + 48); }
            const uint32_t n_in = ns ? min(K, ns - c * K) : 0;
            const bool last = c + 1 == nc;
            bool cok = c0 <= c1 && c1 <= cmdb && l0 <= l1 && l1 <= lenb && v0 <= v1 && v1 <= lvlb &&
                       q0 <= q1 && q1 <= nl && d0 <= d1 && d1 <= blen &&
                       c1 - c0 <= 4 * (n_in + 1) && l1 - l0 <= 4 * n_in && v1 - v0 <= 4 * n_in;
            if (!cok) {
                fail(j, ACEAPEX_E_CORRUPT);
                continue;
            }
            ChunkDesc cd;
            cd.out_base = (uint32_t)(b * B) + d0;
            cd.out_len = d1 - d0;
            cd.cmd_at = (uint32_t)cmd_at + c0; cd.cmd_n = c1 - c0;
            cd.len_at = (uint32_t)len_at + l0; cd.len_n = l1 - l0;
            cd.lvl_at = (uint32_t)lvl_at + v0; cd.lvl_n = v1 - v0;
            cd.lit_at = (uint32_t)lit_at + q0; cd.lit_n = q1 - q0;
            cd.off_at = (uint32_t)(off_at + 4ull * c * K);
            cd.nseq_last = n_in | (last ? 0x80000000u : 0u);
            j.chunks[cb0 + c] = cd;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(NT) k_phase1(Job j)
{
    __shared__ Lds L;
    const uint32_t t = threadIdx.x;
    const uint32_t nh = min(j.max_level + 1, LVL_LDS);
    for (uint32_t i = t; i < nh; i += NT) L.hist[i] = 0;
    const uint32_t ncmd = parse_chunk(j, blockIdx.x, L, true);
    if (!ncmd) return;
    const ChunkDesc &d = L.d;
    const uint32_t ns = d.nseq_last & 0x7fffffffu;
    for (uint32_t e = t; e < ncmd; e += NT) {
        const uint32_t r = L.run[e];
        if (r) {
            const uint64_t sc = L.u.scan[e];
            copy_bytes(j.out + d.out_base + (uint32_t)(sc >> 32), j.comp + d.lit_at + (uint32_t)sc, r);
        }
    }
    for (uint32_t e = t; e < ns; e += NT) {
        const uint32_t l = L.lvl[e];
        if (l == 0) continue;
        if (l < LVL_LDS) atomicAdd(&L.hist[l], 1u);
        else atomicAdd(&j.hist[l], 1u);
    }
    __syncthreads();
    for (uint32_t i = t; i < nh; i += NT)
        if (L.hist[i]) atomicAdd(&j.hist[i], L.hist[i]);
}

__global__ void __launch_bounds__(NT) k_lscan(Job j)
{
    __shared__ uint64_t tmp[NT / 64];
    uint64_t carry = 0;
    for (uint32_t s = 0; s <= j.max_level; s += NT) {
        const uint32_t i = s + threadIdx.x;
        const uint32_t h = (i <= j.max_level && i > 0) ? j.hist[i] : 0;
        uint64_t tot;
        const uint64_t ex = wg_excl_scan64(h, tmp, tot);
        if (i <= j.max_level) {
            const uint64_t b = carry + ex;
            j.base[i] = (uint32_t)min(b, (uint64_t)j.n_deep);
            j.cursor[i] = (uint32_t)min(b, (uint64_t)j.n_deep);
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        j.base[j.max_level + 1] = (uint32_t)min(carry, (uint64_t)j.n_deep);
        if (carry != j.n_deep) fail(j, ACEAPEX_E_CORRUPT);
    }
}

__global__ void __launch_bounds__(NT) k_phase2(Job j)
{
    __shared__ Lds L;
    const uint32_t t = threadIdx.x;
    const uint32_t nh = min(j.max_level + 1, LVL_LDS);
    for (uint32_t i = t; i < nh; i += NT) L.hist[i] = 0;
    const uint32_t ncmd = parse_chunk(j, blockIdx.x, L, true);
    if (!ncmd) return;
    const ChunkDesc &d = L.d;
    const uint32_t ns = d.nseq_last & 0x7fffffffu;
    bool bad = false;
    for (uint32_t e = t; e < ns; e += NT) {
        const uint32_t dst = d.out_base + (uint32_t)(L.u.scan[e] >> 32) + L.run[e];
        const uint32_t src = ld32(j.comp + d.off_at + 4 * e);
        const uint32_t m = L.mlen[e];
        const uint32_t l = L.lvl[e];
        if ((uint64_t)src + m > dst) {  // a source must end before its destination
            bad = true;
            L.lvl[e] = SKIP;
            continue;
        }
        if (l == 0) {
            copy_bytes(j.out + dst, j.out + src, m);
        } else if (l < LVL_LDS) {
            L.rank[e] = (uint16_t)atomicAdd(&L.hist[l], 1u);
        }
    }
    if (bad) fail(j, ACEAPEX_E_CORRUPT);
    __syncthreads();
    for (uint32_t i = t; i < nh; i += NT)
        if (L.hist[i]) L.hbase[i] = atomicAdd(&j.cursor[i], L.hist[i]);
    __syncthreads();
    for (uint32_t e = t; e < ns; e += NT) {
        const uint32_t l = L.lvl[e];
        if (l == 0 || l == SKIP) continue;
        const uint32_t slot = l < LVL_LDS ? L.hbase[l] + L.rank[e] : atomicAdd(&j.cursor[l], 1u);
        if (slot >= j.base[l + 1]) {  // more deep matches than the histogram announced
            fail(j, ACEAPEX_E_CORRUPT);
            continue;
        }
        const uint32_t dst = d.out_base + (uint32_t)(L.u.scan[e] >> 32) + L.run[e];
        uint32_t *r = j.recs + 3ull * slot;
        r[0] = dst;
        r[1] = ld32(j.comp + d.off_at + 4 * e);
        r[2] = L.mlen[e];
    }
}

__global__ void __launch_bounds__(NT) k_level(Job j, uint32_t k)
{
    const uint32_t b0 = j.base[k];
    const uint32_t b1 = min(j.cursor[k], j.base[k + 1]);
    for (uint32_t i = b0 + blockIdx.x * NT + threadIdx.x; i < b1; i += gridDim.x * NT) {
        const uint32_t *r = j.recs + 3ull * i;
        const uint32_t dst = r[0], src = r[1], m = r[2];
        if ((uint64_t)dst + m > j.n || (uint64_t)src + m > dst) {
            fail(j, ACEAPEX_E_CORRUPT);
            continue;
        }
        copy_bytes(j.out + dst, j.out + src, m);
    }
}

// ----------------------------------------------------------------- host side

thread_local int g_last_hip = 0;

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct WsLayout {
    size_t status, chunks, hist, base, cursor, recs, total;
};

WsLayout ws_layout(const aceapex_info &in)
{
    WsLayout w;
    size_t o = 0;
    w.status = o; o += 256;
    w.chunks = o; o = align256(o + sizeof(ChunkDesc) * (size_t)in.n_chunks);
    w.hist = o; o = align256(o + 4ull * ((size_t)in.max_level + 1));
    w.base = o; o = align256(o + 4ull * ((size_t)in.max_level + 2));
    w.cursor = o; o = align256(o + 4ull * ((size_t)in.max_level + 1));
    w.recs = o; o = align256(o + 12ull * (size_t)in.n_deep);
    w.total = o;
    return w;
}

inline uint16_t rd16h(const uint8_t *p) { uint16_t v; memcpy(&v, p, 2); return v; }
inline uint32_t rd32h(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
inline uint64_t rd64h(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }

bool info_consistent(const aceapex_info &in)
{
    if (in.block_log2 < 3 || in.block_log2 > 30 || in.min_match < 1 || in.chunk_log2 > 20) return false;
    const uint64_t B = 1ull << in.block_log2;
    if ((in.decoded_bytes + B - 1) / B != in.n_blocks) return false;
    if (in.comp_bytes < HDR + 16ull * (in.n_blocks + 1ull)) return false;
    if (in.n_deep > in.n_seq) return false;
    if (in.n_blocks == 0 && (in.n_seq || in.n_chunks)) return false;
    if (in.n_blocks && in.n_chunks < in.n_blocks) return false;
    return true;
}

int gpu_supported(const aceapex_info &in)
{
    if (in.decoded_bytes >= (1ull << 32) || in.comp_bytes >= (1ull << 32)) return ACEAPEX_E_UNSUPPORTED;
    if (in.block_log2 > BLOCK_LOG2_MAX || in.chunk_log2 > K_LOG2_MAX) return ACEAPEX_E_UNSUPPORTED;
    if (in.max_level >= (1u << 28)) return ACEAPEX_E_UNSUPPORTED;
    return ACEAPEX_OK;
}

int hip_fail(hipError_t e)
{
    g_last_hip = (int)e;
    return ACEAPEX_E_HIP;
}

int launch_one(const aceapex_stream &s, void *d_out, uint64_t cap, uint8_t *ws, int32_t *d_status,
               hipStream_t st)
{
    const aceapex_info &in = s.info;
    const WsLayout w = ws_layout(in);
    Job j;
    j.comp = (const uint8_t *)s.d_comp;
    j.out = (uint8_t *)d_out;
    j.n = (uint32_t)in.decoded_bytes;
    j.comp_bytes = (uint32_t)in.comp_bytes;
    j.n_blocks = in.n_blocks;
    j.block_log2 = in.block_log2;
    j.min_match = in.min_match;
    j.chunk_log2 = in.chunk_log2;
    j.max_level = in.max_level;
    j.n_chunks = in.n_chunks;
    j.n_seq = in.n_seq;
    j.n_deep = in.n_deep;
    j.chunks = (ChunkDesc *)(ws + w.chunks);
    j.hist = (uint32_t *)(ws + w.hist);
    j.base = (uint32_t *)(ws + w.base);
    j.cursor = (uint32_t *)(ws + w.cursor);
    j.recs = (uint32_t *)(ws + w.recs);
    j.status = d_status ? d_status : (int32_t *)(ws + w.status);
    (void)cap;
    const uint32_t init_grid = (uint32_t)std::min<uint64_t>(1024, (std::max<uint64_t>(in.n_chunks, in.max_level + 1ull) + NT - 1) / NT + 1);
    hipLaunchKernelGGL(k_init, dim3(init_grid), dim3(NT), 0, st, j);
    if (in.n_blocks) {
        hipLaunchKernelGGL(k_setup, dim3(std::min<uint32_t>(in.n_blocks, 65535)), dim3(NT), 0, st, j);
        hipLaunchKernelGGL(k_phase1, dim3(in.n_chunks), dim3(NT), 0, st, j);
        hipLaunchKernelGGL(k_lscan, dim3(1), dim3(NT), 0, st, j);
        hipLaunchKernelGGL(k_phase2, dim3(in.n_chunks), dim3(NT), 0, st, j);
        for (uint32_t k = 1; k <= in.max_level; k++)
            hipLaunchKernelGGL(k_level, dim3(LEVEL_GRID), dim3(NT), 0, st, j, k);
    }
    hipError_t e = hipGetLastError();
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
    return ACEAPEX_OK;
}

}  // namespace

extern "C" {

int aceapex_probe(const void *h_stream_prefix, size_t h_len, aceapex_info *info)
{
    if (!h_stream_prefix || !info || h_len < HDR) return ACEAPEX_E_INVAL;
    const uint8_t *h = (const uint8_t *)h_stream_prefix;
    if (memcmp(h, "ACX1", 4) != 0 || rd16h(h + 4) != 1) return ACEAPEX_E_FORMAT;
    aceapex_info in;
    in.flags = rd16h(h + 6);
    in.block_log2 = h[8];
    in.min_match = h[9];
    in.chunk_log2 = h[10];
    in.max_depth = rd32h(h + 12);
    in.decoded_bytes = rd64h(h + 16);
    in.comp_bytes = rd64h(h + 24);
    in.n_blocks = rd32h(h + 32);
    in.max_level = rd32h(h + 36);
    in.n_seq = rd32h(h + 40);
    in.n_deep = rd32h(h + 44);
    in.n_chunks = rd32h(h + 48);
    in.content_hash = rd64h(h + 56);
    if ((in.flags & ~0xFu) || !(in.flags & 8u) || h[11] != 0 || rd32h(h + 52) != 0) return ACEAPEX_E_FORMAT;
    if (!info_consistent(in)) return ACEAPEX_E_FORMAT;
    *info = in;
    return ACEAPEX_OK;
}

size_t aceapex_workspace_bytes(const aceapex_desc *h_descs, uint32_t n)
{
    if (!h_descs) return 0;
    size_t tot = 0;
    for (uint32_t i = 0; i < n; i++) {
        if (!info_consistent(h_descs[i].s.info)) return 0;
        tot += ws_layout(h_descs[i].s.info).total;
    }
    return tot;
}

int aceapex_decode(const aceapex_stream *stream, void *d_out, uint64_t out_capacity, void *d_workspace,
                   size_t ws_bytes, int32_t *d_status, void *hip_stream)
{
    int rc = check_stream_args(stream, d_out, out_capacity);
    if (rc) return rc;
    const size_t need = ws_layout(stream->info).total;
    if (!d_workspace || ((uintptr_t)d_workspace & 255) || ws_bytes < need) return ACEAPEX_E_WORKSPACE;
    return launch_one(*stream, d_out, out_capacity, (uint8_t *)d_workspace, d_status, (hipStream_t)hip_stream);
}

int aceapex_decode_many(const aceapex_desc *h_descs, uint32_t n, void *d_workspace, size_t ws_bytes,
                        void *hip_stream)
{
    if (!h_descs && n) return ACEAPEX_E_INVAL;
    size_t need = 0;
    for (uint32_t i = 0; i < n; i++) {
        int rc = check_stream_args(&h_descs[i].s, h_descs[i].d_out, h_descs[i].out_capacity);
        if (rc) return rc;
        need += ws_layout(h_descs[i].s.info).total;
    }
    if (n && (!d_workspace || ((uintptr_t)d_workspace & 255) || ws_bytes < need)) return ACEAPEX_E_WORKSPACE;
    size_t off = 0;
    for (uint32_t i = 0; i < n; i++) {
        int rc = launch_one(h_descs[i].s, h_descs[i].d_out, h_descs[i].out_capacity,
                            (uint8_t *)d_workspace + off, h_descs[i].d_status, (hipStream_t)hip_stream);
        if (rc) return rc;
        off += ws_layout(h_descs[i].s.info).total;
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
    default: return "unknown error";
    }
}

int aceapex_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
