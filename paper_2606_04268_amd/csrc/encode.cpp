// Host-side encoder for absolute-offset LZ77 streams (ACEAPEX, arXiv
// 2606.04268): the producer of the streams the GPU decoder consumes.
//
// Method (Sec. 3): a greedy hash-chain parse whose back-references are
// absolute output positions (Sec. 3.1), cut into self-contained blocks
// (Sec. 3.1); optional within-block chain flattening (Sec. 3.3); optional
// depth limit (Sec. 7.4); every match carries its dependency level (Sec. 7.1).
//
// Structure, chosen for a many-core host:
//   1. chain links: because every position is entered into the hash chains
//      in increasing order, the candidates examined at position p are
//      exactly p's predecessors with the same 4-byte hash, most recent
//      first; those links are computed once, independently of the parse.
//   2. without a depth limit the greedy parse (which positions start a match
//      and how long it is) does not depend on levels, so blocks are parsed in
//      parallel; each match keeps every candidate that reaches its length.
//   3. one pass over the blocks in order then picks, among the tied
//      candidates, the lowest resulting level (most recent on equal level),
//      applies flattening and fixes every level, since a block's levels
//      depend on the final levels of all earlier blocks.
//   4. blocks are serialized in parallel and concatenated.
// With a depth limit (Sec. 7.4) a candidate's usable length is cut where its
// source reaches a byte of level > max_depth - 2, which depends on levels.
// Where the level-independent parse picks a match whose level stays within
// the limit, none of its tied candidates is cut, so the limited greedy parse
// makes the same choice; the in-order pass therefore follows the parallel
// parse and walks the hash chain with cut lengths itself only where the
// chosen match would be too deep, and at the positions after it until the
// two parses meet again (a position the parallel parse decided at: a match
// start or a literal).
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <vector>

#include "aceapex.h"

namespace {

constexpr uint32_t NIL = 0xffffffffu;

struct Piece {
    uint32_t dst, src, len;
    int32_t lvl;
};

struct Found {               // one match of the level-independent parse
    uint32_t dst, len;
    uint32_t tie0, nties;    // tied candidates in BlockParse::ties
    uint32_t alt0, nalts;    // with a depth limit: the longest candidates in BlockParse::alts
};

struct Alt {                 // a candidate source and its match length
    uint32_t src, len;
};

constexpr uint32_t ALTS = 8;  // candidates kept per match for the depth-limited pass

struct BlockParse {
    std::vector<Found> found;
    std::vector<uint32_t> ties;
    std::vector<Alt> alts;
    std::vector<Piece> pieces;   // final matches of the block
    std::vector<uint8_t> bytes;  // serialized payload
    std::vector<uint32_t> per_level;  // matches of the block at each level
    uint32_t max_level = 0, n_deep = 0;
};

class Encoder {
public:
    Encoder(const uint8_t *x, uint64_t n, const aceapex_enc_opts &o) : x_(x), n_(n), o_(o)
    {
        B_ = 1ull << o.block_log2;
        nb_ = (n + B_ - 1) / B_;
    }

    int64_t run(uint8_t **out);

private:
    const uint8_t *x_;
    uint64_t n_, B_, nb_;
    aceapex_enc_opts o_;
    std::vector<uint32_t> link_;   // previous position with the same 4-byte hash
    std::vector<int32_t> wlev_;    // final level of the writer of each byte, -1 literal
    std::vector<BlockParse> blk_;

    uint32_t hash_at(uint64_t q) const
    {
        uint32_t v;
        memcpy(&v, x_ + q, 4);
        return (v * 2654435761u) >> (32 - o_.hash_bits);
    }

    void build_links();
    void parse_free(uint64_t b);          // level-independent parse: every candidate of the longest length
    void resolve_limited(uint64_t b);     // depth limit, needs final levels of earlier bytes
    void resolve(uint64_t b);
    void flatten(uint64_t b);
    void relevel(uint64_t b);
    void serialize(uint64_t b);

    int32_t level_over(uint64_t s, uint64_t l) const
    {
        int32_t hi = -1;
        const int32_t *w = wlev_.data() + s;
        for (uint64_t k = 0; k < l; k++) hi = std::max(hi, w[k]);
        return hi + 1;
    }

    uint64_t common_prefix(uint64_t s, uint64_t p, uint64_t cap) const
    {
        uint64_t l = 0;
        while (l + 8 <= cap) {
            uint64_t a, b;
            memcpy(&a, x_ + s + l, 8);
            memcpy(&b, x_ + p + l, 8);
            if (a != b) return l + (uint64_t)(__builtin_ctzll(a ^ b) >> 3);
            l += 8;
        }
        while (l < cap && x_[s + l] == x_[p + l]) l++;
        return l;
    }
};

void Encoder::build_links()
{
    link_.assign(n_ ? n_ : 1, NIL);
    if (n_ < 4) return;
    std::vector<uint32_t> head(1u << o_.hash_bits, NIL);
    for (uint64_t q = 0; q + 4 <= n_; q++) {
        uint32_t h = hash_at(q);
        link_[q] = head[h];
        head[h] = (uint32_t)q;
    }
}

void Encoder::parse_free(uint64_t b)
{
    BlockParse &bp = blk_[b];
    const uint64_t bs = b * B_, be = std::min(n_, bs + B_);
    const uint64_t m0 = o_.min_match;
    const bool keep_alts = o_.max_depth != 0;
    Alt cand[64];
    uint64_t p = bs;
    while (p < be) {
        uint64_t best = 0;
        uint32_t t0 = (uint32_t)bp.ties.size(), nt = 0, nc = 0;
        if (p + m0 <= be && p + 4 <= n_) {
            uint32_t s = link_[p];
            for (uint32_t step = 0; s != NIL && step < o_.chain_depth; step++, s = link_[s]) {
                uint64_t cap = std::min(be - p, p - s);
                if (cap < m0 || (!keep_alts && cap < best)) continue;
                uint64_t l = common_prefix(s, p, cap);
                if (l < m0) continue;
                if (keep_alts && nc < 64) cand[nc++] = {s, (uint32_t)l};
                if (l < best) continue;
                if (l > best) {
                    best = l;
                    bp.ties.resize(t0);
                    nt = 0;
                }
                bp.ties.push_back(s);
                nt++;
            }
        }
        if (best >= m0) {
            uint32_t a0 = (uint32_t)bp.alts.size(), na = 0;
            if (keep_alts) {  // the ALTS longest candidates, most recent first among equal lengths
                std::stable_sort(cand, cand + nc, [](const Alt &a, const Alt &b) { return a.len > b.len; });
                na = std::min<uint32_t>(nc, ALTS);
                bp.alts.insert(bp.alts.end(), cand, cand + na);
            }
            bp.found.push_back({(uint32_t)p, (uint32_t)best, t0, nt, a0, na});
            p += best;
        } else {
            bp.ties.resize(t0);
            p++;
        }
    }
}

// The depth-limited parse of block b (Sec. 7.4: every match level at most
// max_depth - 1), from the level-independent one.  A match of that parse
// whose level stays within the limit is kept whole (its least deep tied
// candidate, as without the limit).  A deeper one is re-cut over its own
// span [p, p + len): at each position q of the span, the kept candidates
// shifted by q - p are still copies of the bytes at q; each is cut where its
// source reaches a byte of level > max_depth - 2, the longest cut piece (the
// least deep among equal lengths, the most recent among equal levels) of at
// least min_match bytes is taken, else q becomes a literal.  The pieces end
// inside the span, so the pass meets the level-independent parse again at
// p + len.
void Encoder::resolve_limited(uint64_t b)
{
    BlockParse &bp = blk_[b];
    const uint64_t bs = b * B_, be = std::min(n_, bs + B_);
    const uint64_t m0 = o_.min_match;
    const int32_t top = (int32_t)o_.max_depth - 1, lim = top - 1;
    bp.pieces.clear();
    bp.pieces.reserve(bp.found.size());
    uint64_t cur = bs;
    for (const Found &f : bp.found) {
        for (uint64_t q = cur; q < f.dst; q++) wlev_[q] = -1;
        uint32_t src = bp.ties[f.tie0];
        int32_t lv = level_over(src, f.len);
        if (o_.tiebreak == 0) {
            for (uint32_t k = 1; k < f.nties && lv > 0; k++) {
                const uint32_t s2 = bp.ties[f.tie0 + k];
                const int32_t l2 = level_over(s2, f.len);
                if (l2 < lv) { lv = l2; src = s2; }
            }
        }
        const uint64_t end = (uint64_t)f.dst + f.len;
        if (lv <= top) {
            bp.pieces.push_back({f.dst, src, f.len, lv});
            std::fill(wlev_.begin() + f.dst, wlev_.begin() + end, lv);
            cur = end;
            continue;
        }
        const Alt *alt = bp.alts.data() + f.alt0;
        for (uint64_t q = f.dst; q < end;) {
            const uint64_t d = q - f.dst;
            uint64_t best = 0, best_src = 0;
            int32_t best_lvl = 0;
            for (uint32_t k = 0; k < f.nalts; k++) {
                if (alt[k].len < d + m0 || alt[k].len - d < best) continue;
                const uint64_t s = alt[k].src + d, room = alt[k].len - d;
                const int32_t *w = wlev_.data() + s;
                uint64_t l = 0;
                while (l < room && w[l] <= lim) l++;
                if (l < m0 || l < best) continue;
                const int32_t lv2 = level_over(s, l);
                if (l > best || (o_.tiebreak == 0 && lv2 < best_lvl)) {
                    best = l;
                    best_src = s;
                    best_lvl = lv2;
                }
            }
            if (best >= m0) {
                bp.pieces.push_back({(uint32_t)q, (uint32_t)best_src, (uint32_t)best, best_lvl});
                std::fill(wlev_.begin() + q, wlev_.begin() + q + best, best_lvl);
                q += best;
            } else {
                wlev_[q] = -1;
                q++;
            }
        }
        cur = end;
    }
    for (uint64_t q = cur; q < be; q++) wlev_[q] = -1;
    std::vector<Found>().swap(bp.found);
    std::vector<uint32_t>().swap(bp.ties);
    std::vector<Alt>().swap(bp.alts);
}

void Encoder::resolve(uint64_t b)
{
    BlockParse &bp = blk_[b];
    const uint64_t bs = b * B_, be = std::min(n_, bs + B_);
    bp.pieces.clear();
    bp.pieces.reserve(bp.found.size());
    uint64_t cur = bs;
    for (const Found &f : bp.found) {
        for (uint64_t q = cur; q < f.dst; q++) wlev_[q] = -1;
        uint32_t src = bp.ties[f.tie0];
        int32_t lv;
        if (o_.tiebreak == 0) {
            lv = level_over(src, f.len);
            for (uint32_t k = 1; k < f.nties && lv > 0; k++) {
                uint32_t s = bp.ties[f.tie0 + k];
                int32_t l2 = level_over(s, f.len);
                if (l2 < lv) { lv = l2; src = s; }
            }
        } else {
            lv = level_over(src, f.len);
        }
        bp.pieces.push_back({f.dst, src, f.len, lv});
        std::fill(wlev_.begin() + f.dst, wlev_.begin() + f.dst + f.len, lv);
        cur = (uint64_t)f.dst + f.len;
    }
    for (uint64_t q = cur; q < be; q++) wlev_[q] = -1;
    std::vector<Found>().swap(bp.found);
    std::vector<uint32_t>().swap(bp.ties);
}

// Sec. 3.3: trace every match byte back through earlier copies of the same
// block; the trace ends at a literal of the block or at the first position
// outside it (mode 1).  In mode 2 a byte is only re-pointed when its trace
// ends at a literal of the block.  Matches are re-cut where the traced
// sources stop being consecutive; cuts shorter than min_match become literals.
void Encoder::flatten(uint64_t b)
{
    BlockParse &bp = blk_[b];
    const uint64_t bs = b * B_, be = std::min(n_, bs + B_);
    const uint64_t len = be - bs;
    std::vector<uint32_t> root(len);
    std::vector<uint8_t> at_literal(len);
    size_t i = 0;
    for (uint64_t q = bs; q < be;) {
        if (i < bp.pieces.size() && bp.pieces[i].dst == q) {
            const Piece &m = bp.pieces[i++];
            for (uint32_t k = 0; k < m.len; k++) {
                const uint64_t y = (uint64_t)m.src + k, r = q + k - bs;
                if (y >= bs && (o_.flatten == 1 || at_literal[y - bs])) {
                    root[r] = root[y - bs];
                    at_literal[r] = at_literal[y - bs];
                } else {
                    root[r] = (uint32_t)y;
                    at_literal[r] = 0;
                }
            }
            q += m.len;
        } else {
            root[q - bs] = (uint32_t)q;
            at_literal[q - bs] = 1;
            q++;
        }
    }
    std::vector<Piece> cut;
    cut.reserve(bp.pieces.size());
    for (const Piece &m : bp.pieces) {
        uint64_t a = m.dst;
        const uint64_t end = (uint64_t)m.dst + m.len;
        while (a < end) {
            uint64_t e = a + 1;
            while (e < end && root[e - bs] == root[e - 1 - bs] + 1) e++;
            if (e - a >= o_.min_match) cut.push_back({(uint32_t)a, root[a - bs], (uint32_t)(e - a), 0});
            a = e;
        }
    }
    bp.pieces.swap(cut);
}

void Encoder::relevel(uint64_t b)
{
    BlockParse &bp = blk_[b];
    const uint64_t bs = b * B_, be = std::min(n_, bs + B_);
    uint64_t cur = bs;
    for (Piece &m : bp.pieces) {
        for (uint64_t q = cur; q < m.dst; q++) wlev_[q] = -1;
        m.lvl = level_over(m.src, m.len);
        std::fill(wlev_.begin() + m.dst, wlev_.begin() + m.dst + m.len, m.lvl);
        cur = (uint64_t)m.dst + m.len;
    }
    for (uint64_t q = cur; q < be; q++) wlev_[q] = -1;
}

inline void put_leb(std::vector<uint8_t> &v, uint32_t x)
{
    do {
        uint8_t c = x & 0x7f;
        x >>= 7;
        v.push_back(c | (x ? 0x80 : 0));
    } while (x);
}

inline void put_u32(std::vector<uint8_t> &v, uint32_t x)
{
    uint8_t t[4];
    memcpy(t, &x, 4);
    v.insert(v.end(), t, t + 4);
}

inline void pad_to16(std::vector<uint8_t> &v) { v.resize((v.size() + 15) & ~(size_t)15, 0); }

void Encoder::serialize(uint64_t b)
{
    BlockParse &bp = blk_[b];
    const uint64_t bs = b * B_, be = std::min(n_, bs + B_);
    const uint32_t K = 1u << o_.chunk_log2;
    const size_t ns = bp.pieces.size();
    const size_t nch = ns ? (ns + K - 1) / K : 1;
    std::vector<uint8_t> cmd, len, lvl, lit, off;
    std::vector<uint32_t> idx(nch * 8, 0);
    cmd.reserve(ns + 1); len.reserve(ns); lvl.reserve(ns); off.reserve(4 * ns);
    uint64_t q = bs;
    for (size_t i = 0; i <= ns; i++) {
        const uint64_t stop = i < ns ? bp.pieces[i].dst : be;
        if (i < ns && i % K == 0) {
            uint32_t *c = &idx[(i / K) * 8];
            c[0] = (uint32_t)cmd.size(); c[1] = (uint32_t)len.size(); c[2] = (uint32_t)lvl.size();
            c[3] = (uint32_t)lit.size(); c[4] = (uint32_t)(q - bs);
        }
        put_leb(cmd, (uint32_t)(stop - q));
        lit.insert(lit.end(), x_ + q, x_ + stop);
        q = stop;
        if (i < ns) {
            const Piece &m = bp.pieces[i];
            put_leb(len, m.len - o_.min_match);
            put_u32(off, m.src);
            if (o_.levels) {
                put_leb(lvl, (uint32_t)m.lvl);
                bp.max_level = std::max(bp.max_level, (uint32_t)m.lvl);
                bp.n_deep += m.lvl > 0;
                if ((size_t)m.lvl >= bp.per_level.size()) bp.per_level.resize((size_t)m.lvl + 1, 0);
                bp.per_level[m.lvl]++;
            }
            q += m.len;
        }
    }
    std::vector<uint8_t> &o = bp.bytes;
    o.clear();
    const uint32_t hdr[8] = {(uint32_t)ns, (uint32_t)lit.size(), (uint32_t)nch, bp.max_level,
                             (uint32_t)cmd.size(), (uint32_t)len.size(), (uint32_t)lvl.size(), 0};
    o.insert(o.end(), (const uint8_t *)hdr, (const uint8_t *)hdr + 32);
    o.insert(o.end(), (const uint8_t *)idx.data(), (const uint8_t *)idx.data() + 4 * idx.size());
    for (std::vector<uint8_t> *s : {&off, &cmd, &len, &lvl, &lit}) {
        o.insert(o.end(), s->begin(), s->end());
        pad_to16(o);
    }
    std::vector<Piece>().swap(bp.pieces);
}

template <class F>
void parallel_for(uint64_t count, unsigned threads, F &&f)
{
    std::atomic<uint64_t> next{0};
    auto work = [&]() {
        for (uint64_t i; (i = next.fetch_add(1)) < count;) f(i);
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < threads; t++) pool.emplace_back(work);
    work();
    for (auto &th : pool) th.join();
}

int64_t Encoder::run(uint8_t **result)
{
    unsigned threads = o_.threads ? o_.threads : std::max(1u, std::thread::hardware_concurrency());
    threads = (unsigned)std::min<uint64_t>(threads, std::max<uint64_t>(nb_, 1));
    blk_.resize(nb_);
    wlev_.assign(n_ ? n_ : 1, -1);
    build_links();
    {
        // parallel parse; one resolver consumes the blocks in order as they finish
        std::vector<uint8_t> done(nb_, 0);
        std::mutex mu;
        std::condition_variable cv;
        std::thread resolver([&]() {
            for (uint64_t b = 0; b < nb_; b++) {
                {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait(lk, [&] { return done[b] != 0; });
                }
                if (o_.max_depth)
                    resolve_limited(b);
                else
                    resolve(b);
                if (o_.flatten) { flatten(b); relevel(b); }
                if (o_.verbose && (b + 1) % 64 == 0)
                    fprintf(stderr, "aceapex_encode: %llu of %llu blocks resolved\n", (unsigned long long)(b + 1),
                            (unsigned long long)nb_);
            }
        });
        parallel_for(nb_, threads, [&](uint64_t b) {
            parse_free(b);
            {
                std::lock_guard<std::mutex> lk(mu);
                done[b] = 1;
            }
            cv.notify_all();
        });
        resolver.join();
    }
    std::vector<uint32_t>().swap(link_);
    std::vector<int32_t>().swap(wlev_);
    parallel_for(nb_, threads, [&](uint64_t b) { serialize(b); });

    uint32_t max_level = 0, n_seq = 0, n_deep = 0, n_chunks = 0;
    for (uint64_t b = 0; b < nb_; b++) max_level = std::max(max_level, blk_[b].max_level);
    // level table: matches per level over the whole stream, after the block table
    std::vector<uint32_t> levels((size_t)max_level + 1, 0);
    for (uint64_t b = 0; b < nb_; b++)
        for (size_t l = 0; l < blk_[b].per_level.size(); l++) levels[l] += blk_[b].per_level[l];
    const uint64_t level_at = 64 + 16 * (nb_ + 1);
    // without levels (the four streams of Sec. 3.2 only) there is no level table
    const uint64_t table = level_at + (o_.levels ? ((4 * levels.size() + 15) & ~(size_t)15) : 0);
    uint64_t total = table;
    std::vector<uint64_t> at(nb_ + 1);
    std::vector<uint32_t> seq_base(nb_ + 1), chunk_base(nb_ + 1);
    for (uint64_t b = 0; b < nb_; b++) {
        const BlockParse &bp = blk_[b];
        at[b] = total;
        seq_base[b] = n_seq;
        chunk_base[b] = n_chunks;
        uint32_t hdr[8];
        memcpy(hdr, bp.bytes.data(), 32);
        n_seq += hdr[0];
        n_chunks += hdr[2];
        n_deep += bp.n_deep;
        total += bp.bytes.size();
    }
    at[nb_] = total;
    seq_base[nb_] = n_seq;
    chunk_base[nb_] = n_chunks;
    uint8_t *out = (uint8_t *)calloc(total, 1);
    if (!out) return ACEAPEX_E_NOMEM;
    if (o_.levels) memcpy(out + level_at, levels.data(), 4 * levels.size());
    uint8_t h[64] = {0};
    memcpy(h, "ACX1", 4);
    const uint16_t version = 1;
    uint16_t flags = o_.levels ? 8 : 0;
    if (o_.flatten == 1) flags |= 1;
    if (o_.flatten == 2) flags |= 2;
    if (o_.max_depth) flags |= 4;
    memcpy(h + 4, &version, 2);
    memcpy(h + 6, &flags, 2);
    h[8] = (uint8_t)o_.block_log2;
    h[9] = (uint8_t)o_.min_match;
    h[10] = (uint8_t)o_.chunk_log2;
    memcpy(h + 12, &o_.max_depth, 4);
    memcpy(h + 16, &n_, 8);
    memcpy(h + 24, &total, 8);
    const uint32_t nb32 = (uint32_t)nb_;
    memcpy(h + 32, &nb32, 4);
    memcpy(h + 36, &max_level, 4);
    memcpy(h + 40, &n_seq, 4);
    memcpy(h + 44, &n_deep, 4);
    memcpy(h + 48, &n_chunks, 4);
    memcpy(out, h, 64);
    for (uint64_t b = 0; b <= nb_; b++) {
        uint8_t *t = out + 64 + 16 * b;
        memcpy(t, &at[b], 8);
        memcpy(t + 8, &seq_base[b], 4);
        memcpy(t + 12, &chunk_base[b], 4);
    }
    parallel_for(nb_, threads, [&](uint64_t b) {
        memcpy(out + at[b], blk_[b].bytes.data(), blk_[b].bytes.size());
        std::vector<uint8_t>().swap(blk_[b].bytes);
    });
    *result = out;
    return (int64_t)total;
}

bool opts_valid(const aceapex_enc_opts *o)
{
    return o && o->block_log2 >= 3 && o->block_log2 <= 30 && o->min_match >= 4 && o->min_match <= 255 &&
           o->flatten <= 2 && o->chain_depth >= 1 && o->hash_bits >= 8 && o->hash_bits <= 28 &&
           o->tiebreak <= 1 && o->chunk_log2 <= 20 && o->levels <= 1;
}

}  // namespace

extern "C" {

void aceapex_enc_defaults(aceapex_enc_opts *o)
{
    if (!o) return;
    o->block_log2 = 20;
    o->min_match = 4;
    o->flatten = 0;
    o->max_depth = 0;
    o->chain_depth = 32;
    o->hash_bits = 22;
    o->tiebreak = 0;
    o->chunk_log2 = 10;
    o->threads = 0;
    o->verbose = 0;
    o->levels = 1;
}

int64_t aceapex_encode(const void *h_in, uint64_t n, const aceapex_enc_opts *opts, void **h_stream)
{
    if (!h_stream) return ACEAPEX_E_INVAL;
    *h_stream = NULL;
    if (!opts_valid(opts) || (n && !h_in)) return ACEAPEX_E_INVAL;
    if (n >= (1ull << 32)) return ACEAPEX_E_UNSUPPORTED;
    try {
        Encoder e((const uint8_t *)h_in, n, *opts);
        return e.run((uint8_t **)h_stream);
    } catch (const std::bad_alloc &) {
        return ACEAPEX_E_NOMEM;
    }
}

void aceapex_free(void *h_stream) { free(h_stream); }

}  // extern "C"
