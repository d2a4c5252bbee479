/*
 * ORACLE -- test infrastructure only.
 *
 * A plain CPU implementation of the absolute-offset LZ77 codec that the GPU
 * decoder must agree with, written from the paper (ACEAPEX, arXiv 2606.04268):
 *
 *   - encoder: greedy hash-chain parse whose back-references are absolute
 *     positions in the decoded output (Sec. 3.1), cut into self-contained
 *     blocks (Sec. 3.1), optional within-block chain flattening (Sec. 3.3),
 *     optional depth limit (Sec. 7.4), per-match dependency levels (Sec. 7.1),
 *     serialized as the per-block streams lit/len/off/cmd (Sec. 3.2) plus a
 *     level stream and a chunk index;
 *   - decode_seq: the sequential reference decoder (Sec. 3.2: walk cmd[] in
 *     order) -- its output is the definition of the decoded result;
 *   - decode_mt: block-parallel CPU decoder with per-block progress counters
 *     (Sec. 3.1, last paragraph);
 *   - check: an independent recomputation of every level from a per-byte
 *     writer map plus the stream invariants.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file.  It shares no code with the GPU decoder.
 *
 * Readings of the paper taken where it is silent (byte layout, tie-breaks,
 * overlap, how far flattening traces, depth-limit off-by-one) are listed in
 * the project design notes; the stream layout is described at the top of the
 * serializer below.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <stdatomic.h>

#define ORC_OK 0
#define ORC_E_INVAL -1
#define ORC_E_FORMAT -2
#define ORC_E_CORRUPT -3
#define ORC_E_CAPACITY -4
#define ORC_E_NOMEM -9

#define FLAG_FLATTEN 1u
#define FLAG_FLATTEN_LITONLY 2u
#define FLAG_DEPTH_LIMITED 4u
#define FLAG_LEVELS 8u

#define HDR_BYTES 64u
#define BLK_HDR_BYTES 32u
#define CHUNK_BYTES 32u
#define MAX_VARINT 4u              /* every varint value is < 2^28 */
#define VARINT_LIMIT (1u << 28)

typedef struct {
    int32_t block_log2;  /* block = 2^block_log2 decoded bytes (paper: 1 MB) */
    int32_t min_match;   /* shortest match, >= 4 */
    int32_t flatten;     /* 0 none, 1 trace roots within the block, 2 literal-rooted chains only */
    int32_t max_depth;   /* 0 = unlimited, else every match level <= max_depth-1 */
    int32_t chain_depth; /* hash-chain candidates examined per position */
    int32_t hash_bits;   /* log2 of the hash head table */
    int32_t tiebreak;    /* 0: equal length -> lowest level, 1: most recent */
    int32_t chunk_log2;  /* sequences per chunk-index entry */
    int32_t levels;      /* 1: write lvl[] and the level table; 0: the four streams of Sec. 3.2 only */
} orc_opts;

typedef struct {
    uint64_t n_seq, n_lit_bytes, match_bytes, n_deep;
    uint64_t level_sum;
    uint32_t max_level;
    uint32_t n_blocks;
    uint64_t inblock_nonliteral_src_bytes; /* source bytes inside the match's own block not written by a literal */
    uint64_t level_mismatch;               /* matches whose stored level differs from the recomputed one */
    uint64_t depth_violations;             /* matches with level > max_depth-1 when depth-limited */
} orc_report;

typedef struct { uint32_t dst, src, len, lvl; } orc_token;

void orc_free(void *p) { free(p); }

/* ------------------------------------------------------------ byte helpers */

static inline uint32_t rd32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static inline uint64_t rd64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }
static inline uint16_t rd16(const uint8_t *p) { uint16_t v; memcpy(&v, p, 2); return v; }
static inline void wr32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static inline void wr64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static inline void wr16(uint8_t *p, uint16_t v) { memcpy(p, &v, 2); }
static inline uint64_t pad16(uint64_t v) { return (v + 15) & ~(uint64_t)15; }

typedef struct { uint8_t *p; uint64_t len, cap; int oom; } buf_t;

static void buf_reserve(buf_t *b, uint64_t extra)
{
    if (b->oom || b->len + extra <= b->cap) return;
    uint64_t nc = b->cap ? b->cap : 4096;
    while (nc < b->len + extra) nc *= 2;
    uint8_t *np = realloc(b->p, nc);
    if (!np) { b->oom = 1; return; }
    b->p = np;
    b->cap = nc;
}

static void buf_put(buf_t *b, const void *src, uint64_t n)
{
    if (n == 0) return; /* src may be NULL for an empty section */
    buf_reserve(b, n);
    if (b->oom) return;
    memcpy(b->p + b->len, src, n);
    b->len += n;
}

static void buf_zero(buf_t *b, uint64_t n)
{
    if (n == 0) return;
    buf_reserve(b, n);
    if (b->oom) return;
    memset(b->p + b->len, 0, n);
    b->len += n;
}

static void buf_varint(buf_t *b, uint32_t v)
{
    uint8_t t[5];
    unsigned k = 0;
    do { uint8_t c = v & 0x7f; v >>= 7; t[k++] = c | (v ? 0x80 : 0); } while (v);
    buf_put(b, t, k);
}

/* LEB128 read of at most MAX_VARINT bytes; returns bytes used or 0 on error */
static unsigned get_varint(const uint8_t *p, uint64_t avail, uint32_t *out)
{
    uint32_t v = 0;
    for (unsigned i = 0; i < MAX_VARINT && i < avail; i++) {
        v |= (uint32_t)(p[i] & 0x7f) << (7 * i);
        if (!(p[i] & 0x80)) { *out = v; return i + 1; }
    }
    return 0;
}

/* ----------------------------------------------------------------- encoder */

typedef struct { uint32_t dst, src, len; int32_t lvl; } match_t;

typedef struct { match_t *m; uint64_t n, cap; } mvec_t;

static int mvec_push(mvec_t *v, match_t x)
{
    if (v->n == v->cap) {
        uint64_t nc = v->cap ? v->cap * 2 : 1024;
        match_t *nm = realloc(v->m, nc * sizeof(match_t));
        if (!nm) return -1;
        v->m = nm;
        v->cap = nc;
    }
    v->m[v->n++] = x;
    return 0;
}

#define NONE UINT32_MAX

typedef struct {
    const uint8_t *x;
    uint64_t n;
    orc_opts o;
    uint32_t *head, *prev;
    int32_t *lvb; /* level of the token that wrote each byte; -1 for a literal byte */
} enc_t;

/* Knuth multiplicative hash of the 4 bytes at q */
static inline uint32_t hash4(const enc_t *e, uint64_t q)
{
    return (uint32_t)(rd32(e->x + q) * 2654435761u) >> (32 - e->o.hash_bits);
}

static inline void insert_pos(enc_t *e, uint64_t q)
{
    if (q + 4 > e->n) return;
    uint32_t h = hash4(e, q);
    e->prev[q] = e->head[h];
    e->head[h] = (uint32_t)q;
}

/* 1 + the highest writer level over [s, s+l); 0 when every source byte is a literal (Sec. 7.1) */
static int32_t level_of(const enc_t *e, uint64_t s, uint64_t l)
{
    int32_t mx = -1;
    for (uint64_t j = 0; j < l; j++) if (e->lvb[s + j] > mx) mx = e->lvb[s + j];
    return mx + 1;
}

/* greedy parse of one block; matches appended to out in increasing dst */
static int parse_block(enc_t *e, uint64_t bs, uint64_t be, mvec_t *out)
{
    const uint8_t *x = e->x;
    const uint64_t m0 = (uint64_t)e->o.min_match;
    uint64_t p = bs;
    while (p < be) {
        uint64_t best_len = 0, best_src = 0;
        int32_t best_lvl = 0;
        if (p + m0 <= be && p + 4 <= e->n) {
            uint32_t cand = e->head[hash4(e, p)];
            for (int steps = 0; cand != NONE && steps < e->o.chain_depth; steps++) {
                uint64_t s = cand;
                uint64_t cap = be - p;
                if (p - s < cap) cap = p - s; /* no overlap: s + l <= p */
                uint64_t l = 0;
                while (l < cap && x[s + l] == x[p + l]) l++;
                if (e->o.max_depth > 0) {
                    uint64_t ok = 0;
                    while (ok < l && e->lvb[s + ok] <= e->o.max_depth - 2) ok++;
                    l = ok;
                }
                if (l >= m0) {
                    int32_t lv = level_of(e, s, l);
                    int better = l > best_len ||
                                 (l == best_len && e->o.tiebreak == 0 && lv < best_lvl);
                    if (better) { best_len = l; best_src = s; best_lvl = lv; }
                }
                cand = e->prev[s];
            }
        }
        if (best_len >= m0) {
            match_t m = {(uint32_t)p, (uint32_t)best_src, (uint32_t)best_len, best_lvl};
            if (mvec_push(out, m)) return -1;
            for (uint64_t j = 0; j < best_len; j++) { e->lvb[p + j] = best_lvl; insert_pos(e, p + j); }
            p += best_len;
        } else {
            e->lvb[p] = -1;
            insert_pos(e, p);
            p++;
        }
    }
    return 0;
}

/*
 * Within-block chain flattening (Sec. 3.3).  root[x] follows the copy chain
 * from x while it stays inside the block: a literal is its own root; a match
 * byte whose source y lies in the block takes root[y]; a source outside the
 * block ends the trace at y (mode 1).  In mode 2 only chains that end at a
 * literal inside the block are followed; any other byte keeps its source y.
 * Each match is re-emitted as maximal pieces whose roots are consecutive;
 * pieces shorter than min_match become literal bytes.
 */
static int flatten_block(enc_t *e, uint64_t bs, uint64_t be, mvec_t *ms, int mode)
{
    uint64_t bl = be - bs;
    uint32_t *root = malloc(bl * sizeof(uint32_t));
    uint8_t *litroot = malloc(bl);
    mvec_t out = {0};
    if (!root || !litroot) { free(root); free(litroot); return -1; }
    uint64_t mi = 0;
    for (uint64_t x = bs; x < be;) {
        if (mi < ms->n && ms->m[mi].dst == x) {
            const match_t *m = &ms->m[mi];
            for (uint64_t k = 0; k < m->len; k++) {
                uint64_t xx = x + k, y = m->src + k;
                if (y >= bs && (mode == 1 || litroot[y - bs])) {
                    root[xx - bs] = root[y - bs];
                    litroot[xx - bs] = litroot[y - bs];
                } else {
                    root[xx - bs] = (uint32_t)y;
                    litroot[xx - bs] = 0;
                }
            }
            x += m->len;
            mi++;
        } else {
            root[x - bs] = (uint32_t)x;
            litroot[x - bs] = 1;
            x++;
        }
    }
    const uint64_t m0 = (uint64_t)e->o.min_match;
    for (uint64_t i = 0; i < ms->n; i++) {
        const match_t *m = &ms->m[i];
        uint64_t a = m->dst, end = (uint64_t)m->dst + m->len;
        while (a < end) {
            uint64_t b = a + 1;
            while (b < end && root[b - bs] == root[b - 1 - bs] + 1) b++;
            if (b - a >= m0) {
                match_t piece = {(uint32_t)a, root[a - bs], (uint32_t)(b - a), 0};
                if (mvec_push(&out, piece)) { free(root); free(litroot); free(out.m); return -1; }
            }
            a = b;
        }
    }
    free(root);
    free(litroot);
    free(ms->m);
    *ms = out;
    return 0;
}

/* set final per-byte writer levels of the block and each match's level */
static void relevel_block(enc_t *e, uint64_t bs, uint64_t be, mvec_t *ms)
{
    uint64_t mi = 0;
    for (uint64_t x = bs; x < be;) {
        if (mi < ms->n && ms->m[mi].dst == x) {
            match_t *m = &ms->m[mi];
            m->lvl = level_of(e, m->src, m->len);
            for (uint64_t k = 0; k < m->len; k++) e->lvb[x + k] = m->lvl;
            x += m->len;
            mi++;
        } else {
            e->lvb[x] = -1;
            x++;
        }
    }
}

/*
 * Stream layout (all integers little-endian):
 *   header (64 B): "ACX1", u16 version=1, u16 flags, u8 block_log2,
 *     u8 min_match, u8 chunk_log2, u8 0, u32 max_depth, u64 decoded_bytes,
 *     u64 comp_bytes, u32 n_blocks, u32 max_level, u32 n_seq, u32 n_deep,
 *     u32 n_chunks, u32 0, u64 content_hash (0 = absent)
 *   block table: (n_blocks+1) x {u64 offset, u32 seq_base, u32 chunk_base};
 *     the last entry is {comp_bytes, n_seq, n_chunks}
 *   level table: (max_level+1) x u32, the number of matches at each level,
 *     zero-padded to a multiple of 16 bytes; the first block follows it
 *   per block, at its 16-aligned offset:
 *     header (32 B): u32 n_seq, n_lit, n_chunks, max_level, cmd_bytes,
 *       len_bytes, lvl_bytes, 0
 *     chunk index: n_chunks x 32 B {u32 cmd_off, len_off, lvl_off, lit_off,
 *       dst_off, 0, 0, 0}; chunk c starts at sequence c*2^chunk_log2
 *     off[n_seq] u32 absolute sources | cmd[] LEB128 literal runs (n_seq+1)
 *     | len[] LEB128 (length - min_match) | lvl[] LEB128 levels | lit[n_lit]
 *     every section padded with zeros to a multiple of 16 bytes
 *   without levels (levels = 0: the four streams of Sec. 3.2 only) the level
 *   flag is clear, the header's max_level and n_deep are 0, there is no level
 *   table and every block's lvl[] is empty; a decoder then computes each
 *   match's level from the definition of Sec. 7.1 as it goes
 */
typedef struct {
    buf_t s;          /* block payloads, offsets relative to the first block */
    uint32_t max_level, n_seq, n_deep, n_chunks;
    uint32_t *hist;   /* matches per level */
    uint64_t hist_cap;
    int oom;
} writer_t;

static void count_level(writer_t *w, uint32_t lv)
{
    if (lv >= w->hist_cap) {
        uint64_t nc = w->hist_cap ? w->hist_cap : 64;
        while (nc <= lv) nc *= 2;
        uint32_t *nh = realloc(w->hist, nc * sizeof(uint32_t));
        if (!nh) { w->oom = 1; return; }
        memset(nh + w->hist_cap, 0, (nc - w->hist_cap) * sizeof(uint32_t));
        w->hist = nh;
        w->hist_cap = nc;
    }
    w->hist[lv]++;
}

static int write_block(writer_t *w, const enc_t *e, uint64_t bs, uint64_t be, const mvec_t *ms,
                       uint64_t *tbl_seq_base, uint64_t *tbl_chunk_base)
{
    const uint32_t K = 1u << e->o.chunk_log2;
    const uint32_t m0 = (uint32_t)e->o.min_match;
    uint64_t nseq = ms->n;
    uint64_t nchunks = nseq ? (nseq + K - 1) / K : 1;
    buf_t cmd = {0}, len = {0}, lvl = {0}, lit = {0}, off = {0};
    uint32_t *chunk = calloc(nchunks * 8, sizeof(uint32_t));
    if (!chunk) return -1;
    uint32_t blk_max = 0;
    uint64_t x = bs;
    for (uint64_t i = 0; i <= nseq; i++) {
        uint64_t stop = i < nseq ? ms->m[i].dst : be;
        if (i % K == 0 && i < nseq) {
            uint32_t *c = chunk + (i / K) * 8;
            c[0] = (uint32_t)cmd.len; c[1] = (uint32_t)len.len; c[2] = (uint32_t)lvl.len;
            c[3] = (uint32_t)lit.len; c[4] = (uint32_t)(x - bs);
        }
        buf_varint(&cmd, (uint32_t)(stop - x));
        buf_put(&lit, e->x + x, stop - x);
        x = stop;
        if (i < nseq) {
            const match_t *m = &ms->m[i];
            buf_varint(&len, m->len - m0);
            buf_put(&off, &m->src, 4);
            if (e->o.levels) {
                buf_varint(&lvl, (uint32_t)m->lvl);
                if ((uint32_t)m->lvl > blk_max) blk_max = (uint32_t)m->lvl;
                if ((uint32_t)m->lvl > w->max_level) w->max_level = (uint32_t)m->lvl;
                if (m->lvl > 0) w->n_deep++;
                count_level(w, (uint32_t)m->lvl);
            }
            x += m->len;
        }
    }
    uint8_t hdr[BLK_HDR_BYTES] = {0};
    wr32(hdr + 0, (uint32_t)nseq);
    wr32(hdr + 4, (uint32_t)lit.len);
    wr32(hdr + 8, (uint32_t)nchunks);
    wr32(hdr + 12, blk_max);
    wr32(hdr + 16, (uint32_t)cmd.len);
    wr32(hdr + 20, (uint32_t)len.len);
    wr32(hdr + 24, (uint32_t)lvl.len);
    *tbl_seq_base = w->n_seq;
    *tbl_chunk_base = w->n_chunks;
    buf_put(&w->s, hdr, sizeof hdr);
    buf_put(&w->s, chunk, nchunks * CHUNK_BYTES);
    buf_t *secs[5] = {&off, &cmd, &len, &lvl, &lit};
    for (int k = 0; k < 5; k++) {
        buf_put(&w->s, secs[k]->p, secs[k]->len);
        buf_zero(&w->s, pad16(secs[k]->len) - secs[k]->len);
    }
    int oom = cmd.oom | len.oom | lvl.oom | lit.oom | off.oom | w->s.oom | w->oom;
    free(cmd.p); free(len.p); free(lvl.p); free(lit.p); free(off.p); free(chunk);
    w->n_seq += (uint32_t)nseq;
    w->n_chunks += (uint32_t)nchunks;
    return oom ? -1 : 0;
}

static int opts_ok(const orc_opts *o)
{
    return o->block_log2 >= 3 && o->block_log2 <= 30 && o->min_match >= 4 && o->min_match <= 255 &&
           o->flatten >= 0 && o->flatten <= 2 && o->max_depth >= 0 && o->chain_depth >= 1 &&
           o->hash_bits >= 8 && o->hash_bits <= 28 && (o->tiebreak == 0 || o->tiebreak == 1) &&
           o->chunk_log2 >= 0 && o->chunk_log2 <= 20 && (o->levels == 0 || o->levels == 1);
}

/* encode x[0..n) into a newly allocated stream; returns its length or < 0 */
int64_t orc_encode(const uint8_t *x, uint64_t n, const orc_opts *o, uint8_t **out)
{
    *out = NULL;
    if (!o || !opts_ok(o) || (n && !x)) return ORC_E_INVAL;
    if (n >= ((uint64_t)1 << 32)) return ORC_E_INVAL;
    enc_t e = {x, n, *o, NULL, NULL, NULL};
    e.head = malloc(((size_t)1 << o->hash_bits) * sizeof(uint32_t));
    e.prev = malloc((n ? n : 1) * sizeof(uint32_t));
    e.lvb = malloc((n ? n : 1) * sizeof(int32_t));
    const uint64_t B = (uint64_t)1 << o->block_log2;
    const uint64_t nb = (n + B - 1) / B;
    uint64_t *tbl = calloc((nb + 1) * 3, sizeof(uint64_t));
    writer_t w;
    memset(&w, 0, sizeof w);
    uint8_t *final = NULL;
    uint64_t total = 0;
    int rc = ORC_OK;
    if (!e.head || !e.prev || !e.lvb || !tbl) { rc = ORC_E_NOMEM; goto done; }
    memset(e.head, 0xff, ((size_t)1 << o->hash_bits) * sizeof(uint32_t));

    for (uint64_t b = 0; b < nb; b++) {
        uint64_t bs = b * B, be = bs + B < n ? bs + B : n;
        mvec_t ms = {0};
        if (parse_block(&e, bs, be, &ms)) { free(ms.m); rc = ORC_E_NOMEM; goto done; }
        if (o->flatten && flatten_block(&e, bs, be, &ms, o->flatten)) { free(ms.m); rc = ORC_E_NOMEM; goto done; }
        relevel_block(&e, bs, be, &ms);
        tbl[b * 3 + 0] = w.s.len;
        if (write_block(&w, &e, bs, be, &ms, &tbl[b * 3 + 1], &tbl[b * 3 + 2])) {
            free(ms.m); rc = ORC_E_NOMEM; goto done;
        }
        free(ms.m);
    }
    if (w.s.oom || w.oom) { rc = ORC_E_NOMEM; goto done; }
    const uint64_t hist_n = o->levels ? (uint64_t)w.max_level + 1 : 0; /* no level table without levels */
    const uint64_t prefix = HDR_BYTES + (nb + 1) * 16 + pad16(4 * hist_n);
    total = prefix + w.s.len;
    final = calloc(total, 1);
    if (!final) { rc = ORC_E_NOMEM; goto done; }
    if (w.s.len) memcpy(final + prefix, w.s.p, w.s.len);
    for (uint64_t l = 0; l < hist_n; l++)
        wr32(final + HDR_BYTES + (nb + 1) * 16 + 4 * l, l < w.hist_cap ? w.hist[l] : 0);
    for (uint64_t b = 0; b < nb; b++) tbl[b * 3 + 0] += prefix;
    tbl[nb * 3 + 0] = total;
    tbl[nb * 3 + 1] = w.n_seq;
    tbl[nb * 3 + 2] = w.n_chunks;
    uint8_t *h = final;
    memcpy(h, "ACX1", 4);
    wr16(h + 4, 1);
    uint16_t flags = o->levels ? FLAG_LEVELS : 0;
    if (o->flatten == 1) flags |= FLAG_FLATTEN;
    if (o->flatten == 2) flags |= FLAG_FLATTEN_LITONLY;
    if (o->max_depth > 0) flags |= FLAG_DEPTH_LIMITED;
    wr16(h + 6, flags);
    h[8] = (uint8_t)o->block_log2;
    h[9] = (uint8_t)o->min_match;
    h[10] = (uint8_t)o->chunk_log2;
    wr32(h + 12, (uint32_t)o->max_depth);
    wr64(h + 16, n);
    wr64(h + 24, total);
    wr32(h + 32, (uint32_t)nb);
    wr32(h + 36, w.max_level);
    wr32(h + 40, w.n_seq);
    wr32(h + 44, w.n_deep);
    wr32(h + 48, w.n_chunks);
    for (uint64_t b = 0; b <= nb; b++) {
        uint8_t *t = h + HDR_BYTES + b * 16;
        wr64(t, tbl[b * 3 + 0]);
        wr32(t + 8, (uint32_t)tbl[b * 3 + 1]);
        wr32(t + 12, (uint32_t)tbl[b * 3 + 2]);
    }
done:
    free(e.head); free(e.prev); free(e.lvb); free(tbl); free(w.s.p); free(w.hist);
    if (rc != ORC_OK) { free(final); return rc; }
    *out = final;
    return (int64_t)total;
}

/* ------------------------------------------------------------ stream reader */

typedef struct {
    uint16_t flags;
    uint32_t block_log2, min_match, chunk_log2, max_depth;
    uint64_t n, comp;
    uint32_t n_blocks, max_level, n_seq, n_deep, n_chunks;
} shdr_t;

typedef struct {
    const uint8_t *base; /* block start */
    uint32_t n_seq, n_lit, n_chunks, max_level, cmd_bytes, len_bytes, lvl_bytes;
    const uint8_t *chunks, *off, *cmd, *len, *lvl, *lit;
    uint64_t out_start, out_end;
} sblk_t;

/* header + block table + level table (present only with levels) */
static uint64_t prefix_bytes(const shdr_t *h)
{
    const uint64_t table = (h->flags & FLAG_LEVELS) ? pad16(4 * ((uint64_t)h->max_level + 1)) : 0;
    return HDR_BYTES + ((uint64_t)h->n_blocks + 1) * 16 + table;
}

static int read_header(const uint8_t *s, uint64_t slen, shdr_t *h)
{
    if (slen < HDR_BYTES || memcmp(s, "ACX1", 4) != 0 || rd16(s + 4) != 1) return ORC_E_FORMAT;
    h->flags = rd16(s + 6);
    h->block_log2 = s[8];
    h->min_match = s[9];
    h->chunk_log2 = s[10];
    h->max_depth = rd32(s + 12);
    h->n = rd64(s + 16);
    h->comp = rd64(s + 24);
    h->n_blocks = rd32(s + 32);
    h->max_level = rd32(s + 36);
    h->n_seq = rd32(s + 40);
    h->n_deep = rd32(s + 44);
    h->n_chunks = rd32(s + 48);
    if ((h->flags & ~0xFu) || h->block_log2 < 3 || h->block_log2 > 30 ||
        h->min_match < 1 || h->chunk_log2 > 20 || s[11] != 0 || h->n >= ((uint64_t)1 << 32))
        return ORC_E_FORMAT;
    /* without levels (the four streams of Sec. 3.2) the level fields are unused and zero */
    if (!(h->flags & FLAG_LEVELS) && (h->max_level || h->n_deep)) return ORC_E_FORMAT;
    uint64_t B = (uint64_t)1 << h->block_log2;
    if ((h->n + B - 1) / B != h->n_blocks) return ORC_E_FORMAT;
    if (h->comp != slen) return ORC_E_FORMAT;
    if (h->max_level >= VARINT_LIMIT) return ORC_E_FORMAT;
    if (prefix_bytes(h) > slen) return ORC_E_FORMAT;
    return ORC_OK;
}

static int read_block(const uint8_t *s, const shdr_t *h, uint32_t b, sblk_t *k)
{
    const uint8_t *t = s + HDR_BYTES + (uint64_t)b * 16;
    uint64_t o0 = rd64(t), o1 = rd64(t + 16);
    if ((o0 & 15) || o1 < o0 || o1 > h->comp || o0 < prefix_bytes(h))
        return ORC_E_FORMAT;
    if (o1 - o0 < BLK_HDR_BYTES) return ORC_E_CORRUPT;
    const uint8_t *p = s + o0;
    k->base = p;
    k->n_seq = rd32(p);
    k->n_lit = rd32(p + 4);
    k->n_chunks = rd32(p + 8);
    k->max_level = rd32(p + 12);
    k->cmd_bytes = rd32(p + 16);
    k->len_bytes = rd32(p + 20);
    k->lvl_bytes = rd32(p + 24);
    uint64_t K = (uint64_t)1 << h->chunk_log2;
    uint64_t want_chunks = k->n_seq ? (k->n_seq + K - 1) / K : 1;
    if (k->n_chunks != want_chunks) return ORC_E_CORRUPT;
    if (rd32(t + 8) + (uint64_t)k->n_seq != rd32(t + 24) || rd32(t + 12) + (uint64_t)k->n_chunks != rd32(t + 28))
        return ORC_E_CORRUPT;
    uint64_t q = BLK_HDR_BYTES + (uint64_t)k->n_chunks * CHUNK_BYTES;
    k->chunks = p + BLK_HDR_BYTES;
    k->off = p + q; q += pad16((uint64_t)k->n_seq * 4);
    k->cmd = p + q; q += pad16(k->cmd_bytes);
    k->len = p + q; q += pad16(k->len_bytes);
    k->lvl = p + q; q += pad16(k->lvl_bytes);
    k->lit = p + q; q += pad16(k->n_lit);
    if (q != o1 - o0) return ORC_E_CORRUPT;
    if (!(h->flags & FLAG_LEVELS) && (k->lvl_bytes || k->max_level)) return ORC_E_CORRUPT;
    uint64_t B = (uint64_t)1 << h->block_log2;
    k->out_start = (uint64_t)b * B;
    k->out_end = k->out_start + B < h->n ? k->out_start + B : h->n;
    return ORC_OK;
}

static int check_table(const uint8_t *s, const shdr_t *h)
{
    const uint8_t *last = s + HDR_BYTES + (uint64_t)h->n_blocks * 16;
    if (rd64(last) != h->comp || rd32(last + 8) != h->n_seq || rd32(last + 12) != h->n_chunks) return ORC_E_FORMAT;
    if (h->n_blocks == 0 && (h->n_seq || h->n_chunks || h->comp != prefix_bytes(h))) return ORC_E_FORMAT;
    if (h->n_blocks && rd64(s + HDR_BYTES) != prefix_bytes(h)) return ORC_E_FORMAT;
    if (h->n_blocks && rd32(s + HDR_BYTES + 8) != 0) return ORC_E_FORMAT;
    if (h->n_blocks && rd32(s + HDR_BYTES + 12) != 0) return ORC_E_FORMAT;
    return ORC_OK;
}

/*
 * Walk one block's cmd[] in order (Sec. 3.2): literal run, then match, with
 * every check a decoder needs before writing.  writer_lvl, when given, gets
 * the level of the token writing each byte (-1 for literals).  tok, when
 * given, receives every match.
 */
typedef struct {
    uint8_t *out;
    int32_t *writer_lvl;
    orc_token *tok;
    uint64_t tok_cap, tok_n;
    uint32_t max_level;
    uint64_t n_deep;
    uint64_t *level_count; /* [max_level + 1] matches seen per level, may be NULL */
    /* for the multi-threaded decoder */
    _Atomic uint64_t *progress;
    uint64_t B;
    uint32_t n_blocks;
    int (*wait)(void *ctx, uint64_t s, uint64_t e);
    void *wait_ctx;
} exec_t;

static int run_block(const shdr_t *h, const sblk_t *k, exec_t *x, uint32_t b)
{
    const uint64_t K = (uint64_t)1 << h->chunk_log2;
    uint64_t ci = 0, li = 0, vi = 0, q = 0, p = k->out_start;
    for (uint64_t i = 0; i <= k->n_seq; i++) {
        if (i % K == 0 && (i < k->n_seq || k->n_seq == 0)) {
            const uint8_t *c = k->chunks + (i / K) * CHUNK_BYTES;
            if (rd32(c) != ci || rd32(c + 4) != li || rd32(c + 8) != vi || rd32(c + 12) != q ||
                rd32(c + 16) != p - k->out_start || rd32(c + 20) || rd32(c + 24) || rd32(c + 28))
                return ORC_E_CORRUPT;
        }
        uint32_t r;
        unsigned u = get_varint(k->cmd + ci, k->cmd_bytes - ci, &r);
        if (!u) return ORC_E_CORRUPT;
        ci += u;
        if (r > k->n_lit - q || r > k->out_end - p) return ORC_E_CORRUPT;
        memcpy(x->out + p, k->lit + q, r);
        if (x->writer_lvl) for (uint32_t j = 0; j < r; j++) x->writer_lvl[p + j] = -1;
        p += r;
        q += r;
        if (x->progress) atomic_store_explicit(&x->progress[b], p - k->out_start, memory_order_release);
        if (i == k->n_seq) break;
        uint32_t lm, lv = 0;
        u = get_varint(k->len + li, k->len_bytes - li, &lm);
        if (!u) return ORC_E_CORRUPT;
        li += u;
        const int levels = (h->flags & FLAG_LEVELS) != 0;
        if (levels) {
            u = get_varint(k->lvl + vi, k->lvl_bytes - vi, &lv);
            if (!u) return ORC_E_CORRUPT;
            vi += u;
        }
        uint64_t m = (uint64_t)lm + h->min_match;
        uint64_t s = rd32(k->off + i * 4);
        if (m > k->out_end - p) return ORC_E_CORRUPT;
        if (s + m > p) return ORC_E_CORRUPT; /* source must lie entirely before the destination */
        if (levels && (lv > h->max_level || lv > k->max_level)) return ORC_E_CORRUPT;
        /* the source bytes, and their writer levels, are read only once final */
        if (x->wait && x->wait(x->wait_ctx, s, s + m)) return ORC_E_CORRUPT;
        if (!levels) {
            /* no stored level: the definition of Sec. 7.1 from the writers of the source bytes */
            int32_t mx = -1;
            for (uint64_t j = 0; j < m; j++) if (x->writer_lvl[s + j] > mx) mx = x->writer_lvl[s + j];
            lv = (uint32_t)(mx + 1);
        }
        memcpy(x->out + p, x->out + s, m); /* s + m <= p: the ranges never overlap */
        if (x->writer_lvl) for (uint64_t j = 0; j < m; j++) x->writer_lvl[p + j] = (int32_t)lv;
        if (x->tok) {
            if (x->tok_n < x->tok_cap) {
                orc_token t = {(uint32_t)p, (uint32_t)s, (uint32_t)m, lv};
                x->tok[x->tok_n] = t;
            }
            x->tok_n++;
        }
        if (lv > x->max_level) x->max_level = lv;
        if (lv > 0) x->n_deep++;
        if (x->level_count && levels) x->level_count[lv]++;
        p += m;
        if (x->progress) atomic_store_explicit(&x->progress[b], p - k->out_start, memory_order_release);
    }
    if (p != k->out_end || q != k->n_lit || ci != k->cmd_bytes || li != k->len_bytes || vi != k->lvl_bytes)
        return ORC_E_CORRUPT;
    return ORC_OK;
}

static int decode_all(const uint8_t *s, uint64_t slen, exec_t *x, uint64_t cap, uint64_t *n_out)
{
    shdr_t h;
    int rc = read_header(s, slen, &h);
    if (rc) return rc;
    if ((rc = check_table(s, &h))) return rc;
    if (n_out) *n_out = h.n;
    if (cap < h.n) return ORC_E_CAPACITY;
    uint64_t seqs = 0;
    const int levels = (h.flags & FLAG_LEVELS) != 0;
    int32_t *own_wl = NULL; /* without levels, the writer-level map computes them */
    if (!levels && !x->writer_lvl) {
        own_wl = malloc((h.n ? h.n : 1) * sizeof(int32_t));
        if (!own_wl) return ORC_E_NOMEM;
        x->writer_lvl = own_wl;
    }
    uint64_t *cnt = calloc((uint64_t)h.max_level + 1, sizeof(uint64_t));
    if (!cnt) { free(own_wl); return ORC_E_NOMEM; }
    x->level_count = cnt;
    for (uint32_t b = 0; b < h.n_blocks && !rc; b++) {
        sblk_t k;
        if ((rc = read_block(s, &h, b, &k))) break;
        if ((rc = run_block(&h, &k, x, b))) break;
        seqs += k.n_seq;
    }
    x->level_count = NULL;
    if (own_wl) {
        free(own_wl);
        x->writer_lvl = NULL;
    }
    if (!rc && seqs != h.n_seq) rc = ORC_E_CORRUPT;
    if (!rc && levels && (x->n_deep != h.n_deep || x->max_level != h.max_level)) rc = ORC_E_CORRUPT;
    /* the level table must count exactly the matches of every level */
    const uint8_t *lt = s + HDR_BYTES + ((uint64_t)h.n_blocks + 1) * 16;
    for (uint64_t l = 0; levels && !rc && l <= h.max_level; l++)
        if (rd32(lt + 4 * l) != cnt[l]) rc = ORC_E_CORRUPT;
    for (uint64_t q = 4 * ((uint64_t)h.max_level + 1); levels && !rc && q < pad16(4 * ((uint64_t)h.max_level + 1)); q++)
        if (lt[q]) rc = ORC_E_CORRUPT;
    free(cnt);
    return rc;
}

/* sequential decode; the output is the definition of the decoded result */
int orc_decode(const uint8_t *s, uint64_t slen, uint8_t *out, uint64_t cap, uint64_t *n_out)
{
    if (!s) return ORC_E_INVAL;
    exec_t x;
    memset(&x, 0, sizeof x);
    x.out = out;
    return decode_all(s, slen, &x, cap, n_out);
}

/* every match (dst, src, len, level) in stream order; returns the count or < 0 */
int64_t orc_tokens(const uint8_t *s, uint64_t slen, orc_token *tok, uint64_t cap)
{
    shdr_t h;
    int rc = read_header(s, slen, &h);
    if (rc) return rc;
    uint8_t *out = malloc(h.n ? h.n : 1);
    if (!out) return ORC_E_NOMEM;
    exec_t x;
    memset(&x, 0, sizeof x);
    x.out = out;
    x.tok = tok;
    x.tok_cap = cap;
    rc = decode_all(s, slen, &x, h.n, NULL);
    free(out);
    return rc ? rc : (int64_t)x.tok_n;
}

/* -------------------------------------------------- block-parallel decoder */

typedef struct {
    const uint8_t *s;
    shdr_t h;
    uint8_t *out;
    int32_t *writer_lvl; /* without stored levels: the writer level of every byte */
    _Atomic uint64_t *progress;
    _Atomic int failed;
    int nthreads;
} mt_t;

typedef struct { mt_t *m; int tid; int rc; } mt_arg_t;

/* wait until every byte of [s, e) is final in the blocks that hold it */
static int mt_wait(void *ctx, uint64_t s, uint64_t e)
{
    mt_t *m = ctx;
    const uint64_t B = (uint64_t)1 << m->h.block_log2;
    for (uint64_t b = s / B; b * B < e; b++) {
        uint64_t need = (e < (b + 1) * B ? e : (b + 1) * B) - b * B;
        while (atomic_load_explicit(&m->progress[b], memory_order_acquire) < need)
            if (atomic_load_explicit(&m->failed, memory_order_relaxed)) return -1;
    }
    return 0;
}

static void *mt_worker(void *arg)
{
    mt_arg_t *a = arg;
    mt_t *m = a->m;
    exec_t x;
    memset(&x, 0, sizeof x);
    x.out = m->out;
    x.writer_lvl = m->writer_lvl;
    x.progress = m->progress;
    x.wait = mt_wait;
    x.wait_ctx = m;
    for (uint32_t b = (uint32_t)a->tid; b < m->h.n_blocks; b += (uint32_t)m->nthreads) {
        sblk_t k;
        int rc = read_block(m->s, &m->h, b, &k);
        if (!rc) rc = run_block(&m->h, &k, &x, b);
        if (rc) {
            a->rc = rc;
            atomic_store(&m->failed, 1);
            return NULL;
        }
    }
    return NULL;
}

/*
 * Block-parallel decode (Sec. 3.1): thread t owns blocks t, t+T, ...; each
 * block publishes how many of its bytes are final; a match whose source lies
 * in earlier blocks waits on those counters.  Blocks only wait on earlier
 * blocks, so the lowest unfinished block always progresses.
 */
int orc_decode_mt(const uint8_t *s, uint64_t slen, uint8_t *out, uint64_t cap, int nthreads)
{
    if (!s || nthreads < 1) return ORC_E_INVAL;
    mt_t m;
    memset(&m, 0, sizeof m);
    int rc = read_header(s, slen, &m.h);
    if (rc) return rc;
    if ((rc = check_table(s, &m.h))) return rc;
    if (cap < m.h.n) return ORC_E_CAPACITY;
    m.s = s;
    m.out = out;
    m.nthreads = nthreads;
    m.progress = calloc(m.h.n_blocks ? m.h.n_blocks : 1, sizeof(uint64_t));
    if (!(m.h.flags & FLAG_LEVELS)) m.writer_lvl = malloc((m.h.n ? m.h.n : 1) * sizeof(int32_t));
    pthread_t *th = malloc(sizeof(pthread_t) * (size_t)nthreads);
    mt_arg_t *args = calloc((size_t)nthreads, sizeof(mt_arg_t));
    if (!m.progress || !th || !args || (!(m.h.flags & FLAG_LEVELS) && !m.writer_lvl)) {
        free(m.progress); free(m.writer_lvl); free(th); free(args);
        return ORC_E_NOMEM;
    }
    int started = 0;
    for (int t = 0; t < nthreads; t++) {
        args[t].m = &m;
        args[t].tid = t;
        if (pthread_create(&th[t], NULL, mt_worker, &args[t])) { atomic_store(&m.failed, 1); break; }
        started++;
    }
    for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
    rc = started == nthreads ? ORC_OK : ORC_E_NOMEM;
    for (int t = 0; t < nthreads; t++) if (args[t].rc && rc == ORC_OK) rc = args[t].rc;
    free(m.progress); free(m.writer_lvl); free(th); free(args);
    return rc;
}

/* ------------------------------------------------------------------ checker */

/*
 * Independent check of a stream against the bytes it should decode to:
 * decodes it sequentially while recording the level of the token writing
 * every byte, then recomputes each match's level from the definition in
 * Sec. 7.1 (0 when every source byte is a literal, else 1 + the highest level
 * among the writers of its source bytes), and counts source bytes inside the
 * match's own block that were not written by a literal (zero after
 * within-block flattening, Sec. 3.3).
 */
int orc_check(const uint8_t *x, uint64_t n, const uint8_t *s, uint64_t slen, orc_report *rep)
{
    memset(rep, 0, sizeof *rep);
    shdr_t h;
    int rc = read_header(s, slen, &h);
    if (rc) return rc;
    if (h.n != n) return ORC_E_CORRUPT;
    uint8_t *out = malloc(n ? n : 1);
    int32_t *wl = malloc((n ? n : 1) * sizeof(int32_t));
    orc_token *tok = malloc(((uint64_t)h.n_seq + 1) * sizeof(orc_token));
    if (!out || !wl || !tok) { free(out); free(wl); free(tok); return ORC_E_NOMEM; }
    exec_t e;
    memset(&e, 0, sizeof e);
    e.out = out;
    e.writer_lvl = wl;
    e.tok = tok;
    e.tok_cap = (uint64_t)h.n_seq + 1;
    rc = decode_all(s, slen, &e, n, NULL);
    if (!rc && n && memcmp(out, x, n) != 0) rc = ORC_E_CORRUPT;
    if (!rc) {
        const uint64_t B = (uint64_t)1 << h.block_log2;
        rep->n_blocks = h.n_blocks;
        rep->n_seq = e.tok_n;
        for (uint64_t i = 0; i < e.tok_n; i++) {
            const orc_token *t = &tok[i];
            int32_t mx = -1;
            uint64_t bs = (t->dst / B) * B;
            for (uint64_t j = 0; j < t->len; j++) {
                uint64_t y = (uint64_t)t->src + j;
                if (wl[y] > mx) mx = wl[y];
                if (y >= bs && wl[y] != -1) rep->inblock_nonliteral_src_bytes++;
            }
            uint32_t want = (uint32_t)(mx + 1);
            if (t->lvl != want) rep->level_mismatch++;
            if (h.max_depth && t->lvl > h.max_depth - 1) rep->depth_violations++;
            if (t->lvl > rep->max_level) rep->max_level = t->lvl;
            if (t->lvl > 0) rep->n_deep++;
            rep->level_sum += t->lvl;
            rep->match_bytes += t->len;
        }
        rep->n_lit_bytes = n - rep->match_bytes;
        if ((h.flags & FLAG_LEVELS) && rep->n_deep != h.n_deep) rc = ORC_E_CORRUPT;
    }
    free(out); free(wl); free(tok);
    return rc;
}
