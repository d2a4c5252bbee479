// Host (CPU) decoder for absolute-offset LZ77 streams (ACEAPEX, arXiv
// 2606.04268), for the requests a GPU launch serves slower: small streams,
// whose decode is shorter than a launch sequence, and very deep ones, whose
// wavefront pays one level boundary per level (Sec. 7.2 finds such a stream
// slower on the GPU than on the CPU; Sec. 8.2 suggests choosing the device
// per input).
//
// Method (Sec. 3.1, last paragraph): blocks are self-contained in their
// sequence tables and every source is an absolute output position, so any
// block can be decoded by any thread once the bytes its sources name exist.
// Threads take blocks in increasing order from a shared counter and run each
// block's sequences in order (Sec. 3.2: a literal run, then a copy from the
// absolute source).  Each block publishes how many of its bytes are final
// with a release store; a copy whose source ends in an earlier block that is
// still being decoded waits, with acquire loads, until that block has
// published past the source's end.  A thread only waits on blocks taken
// before its own, which are held by running threads, so every wait ends;
// a thread that finds its block corrupt raises a shared abort flag that ends
// every wait.
//
// Every field is checked before use: no read leaves the stream and no write
// leaves [out, out + decoded_bytes).
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "aceapex.h"
#include "internal.h"

namespace {

constexpr uint32_t HDR = 64, BLKHDR = 32, CHUNK_ENT = 32;

inline uint32_t rd32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
inline uint64_t rd64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }
inline uint64_t pad16(uint64_t v) { return (v + 15) & ~(uint64_t)15; }

// LEB128 of at most 4 bytes from p[0, end); 0 on a malformed value.
inline uint32_t leb(const uint8_t *&p, const uint8_t *end, uint32_t &v)
{
    uint32_t x = 0;
    for (uint32_t i = 0; i < 4 && p < end; i++) {
        const uint8_t c = *p++;
        x |= (uint32_t)(c & 0x7f) << (7 * i);
        if (!(c & 0x80)) {
            v = x;
            return 1;
        }
    }
    return 0;
}

struct alignas(64) Progress {  // one cache line per block, so that blocks do not share a line
    std::atomic<uint64_t> v{0};
};

struct Shared {
    const uint8_t *s;
    uint64_t len;
    uint8_t *out;
    aceapex_info in;
    uint64_t first_block;                    // byte offset of block 0's payload
    std::unique_ptr<Progress[]> done;        // per block: bytes final from its start
    std::atomic<uint64_t> next{0};
    std::atomic<int> abort{0};
};

// Wait until every byte of [a, b) is final; false when the decode aborts.
bool wait_final(Shared &S, uint64_t a, uint64_t b, uint64_t own_block)
{
    const uint64_t B = 1ull << S.in.block_log2;
    const uint64_t last = (b - 1) >> S.in.block_log2;
    for (uint64_t blk = a >> S.in.block_log2; blk <= last && blk < own_block; blk++) {
        const uint64_t need = std::min(b, (blk + 1) * B) - blk * B;
        while (S.done[blk].v.load(std::memory_order_acquire) < need) {
            if (S.abort.load(std::memory_order_relaxed)) return false;
            std::this_thread::yield();
        }
    }
    return true;
}

// Decode block b; false when it is corrupt.
bool decode_block(Shared &S, uint64_t b)
{
    const aceapex_info &in = S.in;
    const uint64_t B = 1ull << in.block_log2;
    const uint64_t base = b * B, blen = std::min(B, in.decoded_bytes - base);
    const uint8_t *tb = S.s + HDR + 16 * b;
    const uint64_t o0 = rd64(tb), o1 = rd64(tb + 16);
    if ((o0 & 15) || o0 < S.first_block || o1 < o0 + BLKHDR || o1 > S.len) return false;
    const uint8_t *bh = S.s + o0;
    const uint32_t ns = rd32(bh), nl = rd32(bh + 4), nc = rd32(bh + 8);
    const uint32_t cmdb = rd32(bh + 16), lenb = rd32(bh + 20), lvlb = rd32(bh + 24);
    const uint64_t off_at = o0 + BLKHDR + (uint64_t)CHUNK_ENT * nc;
    const uint64_t cmd_at = off_at + pad16(4ull * ns);
    const uint64_t len_at = cmd_at + pad16(cmdb);
    const uint64_t lvl_at = len_at + pad16(lenb);
    const uint64_t lit_at = lvl_at + pad16(lvlb);
    if (lit_at + pad16(nl) != o1 || nc == 0) return false;
    const uint8_t *offs = S.s + off_at;
    const uint8_t *cp = S.s + cmd_at, *ce = cp + cmdb;
    const uint8_t *lp = S.s + len_at, *le = lp + lenb;
    const uint8_t *lit = S.s + lit_at, *lit_end = lit + nl;
    uint8_t *out = S.out;
    std::atomic<uint64_t> &done = S.done[b].v;
    uint64_t p = base;
    const uint64_t end = base + blen;
    constexpr uint32_t AHEAD = 16;  // matches whose source is prefetched ahead of its copy
    for (uint32_t i = 0; i < std::min(ns, AHEAD); i++) {
        const uint64_t src = rd32(offs + 4ull * i);
        if (src < in.decoded_bytes) __builtin_prefetch(out + src);
    }
    for (uint32_t i = 0; i <= ns; i++) {
        uint32_t r;
        if (!leb(cp, ce, r) || r > end - p || r > (uint64_t)(lit_end - lit)) return false;
        if (r <= 16 && p + 16 <= end && lit + 16 <= S.s + S.len) {
            memcpy(out + p, lit, 16);  // bytes past the run are rewritten by what follows in the block
        } else {
            memcpy(out + p, lit, r);
        }
        lit += r;
        p += r;
        if (i == ns) break;
        if (i + AHEAD < ns) {
            const uint64_t ahead = rd32(offs + 4ull * (i + AHEAD));
            if (ahead < in.decoded_bytes) __builtin_prefetch(out + ahead);
        }
        uint32_t m;
        if (!leb(lp, le, m)) return false;
        const uint64_t ml = (uint64_t)m + in.min_match;
        const uint64_t src = rd32(offs + 4ull * i);
        if (ml > end - p || src + ml > p) return false;  // inside the block, source strictly before
        if (ml <= 16 && src + 16 <= p && p + 16 <= end) {
            // one 16-byte copy: its source bytes are all final (before p), and
            // its bytes past the match are rewritten by what follows in the block
            if (src < base && !wait_final(S, src, std::min(src + 16, base), b)) return false;
            memcpy(out + p, out + src, 16);
        } else {
            if (src < base && !wait_final(S, src, std::min(src + ml, base), b)) return false;
            memcpy(out + p, out + src, ml);
        }
        p += ml;
        done.store(p - base, std::memory_order_release);
    }
    if (p != end || lit != lit_end || cp != ce || lp != le) return false;
    done.store(blen, std::memory_order_release);
    return true;
}

void worker(Shared &S)
{
    for (;;) {
        const uint64_t b = S.next.fetch_add(1);
        if (b >= S.in.n_blocks || S.abort.load(std::memory_order_relaxed)) return;
        if (!decode_block(S, b)) {
            S.abort.store(1);
            return;
        }
    }
}

}  // namespace

extern "C" int aceapex_decode_host(const void *h_stream, size_t len, void *h_out, uint64_t out_capacity,
                                   uint32_t threads)
{
    if (!h_stream || len < HDR) return ACEAPEX_E_INVAL;
    Shared S;
    int rc = aceapex_probe(h_stream, len, &S.in);
    if (rc) return rc;
    const aceapex_info &in = S.in;
    if (in.comp_bytes != len) return ACEAPEX_E_FORMAT;
    if (out_capacity < in.decoded_bytes) return ACEAPEX_E_CAPACITY;
    if (in.decoded_bytes && !h_out) return ACEAPEX_E_INVAL;
    if (in.decoded_bytes >= (1ull << 32) || in.block_log2 > 30) return ACEAPEX_E_UNSUPPORTED;
    S.s = (const uint8_t *)h_stream;
    S.len = len;
    S.out = (uint8_t *)h_out;
    S.first_block = aceapex_impl::prefix_bytes(in);  // header, block table, level table if any
    if (S.first_block > len) return ACEAPEX_E_FORMAT;
    if (in.n_blocks == 0) return ACEAPEX_OK;
    if (rd64(S.s + HDR) != S.first_block || rd64(S.s + HDR + 16ull * in.n_blocks) != len) return ACEAPEX_E_CORRUPT;
    try {
        S.done.reset(new Progress[in.n_blocks]);
    } catch (const std::bad_alloc &) {
        return ACEAPEX_E_NOMEM;
    }
    unsigned t = threads ? threads : std::max(1u, std::thread::hardware_concurrency());
    t = (unsigned)std::min<uint64_t>(t, in.n_blocks);
    std::vector<std::thread> pool;
    try {
        for (unsigned i = 1; i < t; i++) pool.emplace_back(worker, std::ref(S));
    } catch (...) {
        S.abort.store(1);
        for (auto &th : pool) th.join();
        return ACEAPEX_E_NOMEM;
    }
    worker(S);
    for (auto &th : pool) th.join();
    return S.abort.load() ? ACEAPEX_E_CORRUPT : ACEAPEX_OK;
}
