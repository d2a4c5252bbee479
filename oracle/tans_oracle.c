/*
 * ORACLE -- test infrastructure only.
 *
 * Table-based asymmetric numeral systems (tANS) for the literal stream, the
 * entropy stage the paper leaves to future work for its four streams
 * (Sec. 4.4, Sec. 8: FSE-coded lit/len/off/cmd).  Written plainly from the
 * definition of tANS (Duda, "Asymmetric numeral systems", 2013/2014) with the
 * choices below; the GPU decoder is written separately from the same
 * definition and shares no code with this file.
 *
 * Definition used here:
 *   - alphabet: bytes; table size L = 2^R (R = table_log);
 *   - normalized counts c_s > 0 for every symbol present, summing to L:
 *     c_s = floor(h_s * L / n), raised to 1 for a present symbol, then the
 *     sum corrected one unit at a time on the symbol with the largest count
 *     (lowest byte value among equal counts);
 *   - spread: with cum_s = sum of c_t over t < s, the i-th entry in symbol
 *     order (i = cum_s + j for the j-th entry of symbol s) goes to table
 *     position (i * step) mod L, step = L/2 + L/8 + 3 (odd, so every
 *     position is used once);
 *   - the positions holding symbol s, in increasing order, are given the
 *     state values y = c_s, c_s + 1, ..., 2 c_s - 1 (so that a larger y
 *     leads to a larger next state, which keeps the coder close to the
 *     entropy);
 *   - decoding state x in [L, 2L): position p = x - L holds (s, y); output s;
 *     nb = R - floor(log2 y); the next state is (y << nb) + the next nb bits;
 *   - encoding state x in [L, 2L): to put symbol s, emit the nb low bits of x
 *     where nb makes y = x >> nb fall in [c_s, 2 c_s), then x = L + the
 *     position given state value y;
 *   - symbols are split over `lanes` independent coders: symbol i belongs to
 *     lane i mod lanes; each lane encodes its symbols last to first from
 *     state L, so that its decoder meets them first to last; a lane's bits
 *     are written LSB-first in the order emitted and read back from its end.
 *
 * Container ("ACT1"), little-endian:
 *   0 char[4] "ACT1"   4 u32 n (symbols)   8 u32 table_log   12 u32 lanes
 *   16 u64 total bytes  24 u32 bitstream bytes  28 u32 0
 *   32: u16 counts[256]
 *   544: lanes x {u32 end bit of the lane's bits, u32 final encoder state}
 *   then the lanes' bits, lane after lane, each starting at the previous
 *   lane's end bit, plus 8 zero bytes of slack.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TANS_OK 0
#define TANS_E_INVAL -1
#define TANS_E_FORMAT -2
#define TANS_E_CORRUPT -3
#define TANS_E_CAPACITY -4
#define TANS_E_NOMEM -9

#define TANS_HDR 32u
#define TANS_COUNTS 512u

static uint32_t rd32t(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t rd64t(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }
static uint16_t rd16t(const uint8_t *p) { uint16_t v; memcpy(&v, p, 2); return v; }
static void wr32t(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static void wr64t(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static void wr16t(uint8_t *p, uint16_t v) { memcpy(p, &v, 2); }

static uint32_t floor_log2(uint32_t v)
{
    uint32_t r = 0;
    while (v >>= 1) r++;
    return r;
}

/* normalized counts of x[0, n) for a table of 2^R entries (see the definition) */
int orc_tans_counts(const uint8_t *x, uint64_t n, uint32_t R, uint16_t *c)
{
    if (R < 8 || R > 15) return TANS_E_INVAL;
    const uint32_t L = 1u << R;
    uint64_t h[256] = {0};
    for (uint64_t i = 0; i < n; i++) h[x[i]]++;
    int64_t sum = 0;
    for (int s = 0; s < 256; s++) {
        uint64_t v = n ? (h[s] * L) / n : 0;
        if (h[s] && v == 0) v = 1;
        c[s] = (uint16_t)v;
        sum += (int64_t)v;
    }
    if (n == 0) {
        memset(c, 0, 256 * sizeof(uint16_t));
        return TANS_OK;
    }
    while (sum != (int64_t)L) {
        int big = 0;
        for (int s = 1; s < 256; s++)
            if (c[s] > c[big]) big = s;
        if (sum < (int64_t)L) {
            c[big]++;
            sum++;
        } else {
            /* take from the largest count that can spare a unit */
            int t = -1;
            for (int s = 0; s < 256; s++)
                if (c[s] > 1 && (t < 0 || c[s] > c[t])) t = s;
            if (t < 0) return TANS_E_INVAL; /* more distinct symbols than table entries */
            c[t]--;
            sum--;
        }
    }
    return TANS_OK;
}

/* The spread (see the definition): sym[p] for every table position p, and
   pos_of[cum_s + y - c_s] = the position given state value y of symbol s. */
static void spread(const uint32_t *c, const uint32_t *cum, uint32_t R, uint16_t *sym, uint32_t *pos_of)
{
    const uint32_t L = 1u << R, step = (L >> 1) + (L >> 3) + 3;
    for (uint32_t s = 0; s < 256; s++)
        for (uint32_t j = 0; j < c[s]; j++) sym[((uint64_t)(cum[s] + j) * step) & (L - 1)] = (uint16_t)s;
    uint32_t next[256];
    for (uint32_t s = 0; s < 256; s++) next[s] = cum[s];
    for (uint32_t p = 0; p < L; p++) pos_of[next[sym[p]]++] = p;
}

typedef struct { uint8_t *p; uint64_t bits, cap; } bitw_t;

static int put_bits(bitw_t *w, uint32_t v, uint32_t nb)
{
    for (uint32_t i = 0; i < nb; i++) {
        uint64_t byte = w->bits >> 3;
        if (byte >= w->cap) {
            uint64_t nc = w->cap ? w->cap * 2 : 4096;
            uint8_t *np = realloc(w->p, nc);
            if (!np) return -1;
            memset(np + w->cap, 0, nc - w->cap);
            w->p = np;
            w->cap = nc;
        }
        if ((v >> i) & 1u) w->p[byte] |= (uint8_t)(1u << (w->bits & 7));
        w->bits++;
    }
    return 0;
}

/* encode x[0, n) into a newly allocated container; returns its length or < 0 */
int64_t orc_tans_encode(const uint8_t *x, uint64_t n, uint32_t R, uint32_t lanes, uint8_t **out)
{
    *out = NULL;
    if ((n && !x) || R < 8 || R > 15 || lanes == 0 || lanes > (1u << 20) || n >= (1ull << 32)) return TANS_E_INVAL;
    const uint32_t L = 1u << R;
    uint16_t c[256];
    int rc = orc_tans_counts(x, n, R, c);
    if (rc) return rc;
    uint32_t cum[257], cc[256];
    cum[0] = 0;
    for (int s = 0; s < 256; s++) {
        cc[s] = c[s];
        cum[s + 1] = cum[s] + c[s];
    }
    /* the encoding table: the position given each state value of each symbol */
    uint16_t *sym = malloc(sizeof(uint16_t) * L);
    uint32_t *pos_of = malloc(sizeof(uint32_t) * L);
    if (!sym || !pos_of) { free(sym); free(pos_of); return TANS_E_NOMEM; }
    if (n) spread(cc, cum, R, sym, pos_of);
    bitw_t w = {0};
    uint32_t *lane_end = malloc(sizeof(uint32_t) * lanes), *lane_state = malloc(sizeof(uint32_t) * lanes);
    uint32_t *chunk_v = NULL, *chunk_n = NULL;
    uint64_t per = (n + lanes - 1) / lanes + 1;
    chunk_v = malloc(sizeof(uint32_t) * per);
    chunk_n = malloc(sizeof(uint32_t) * per);
    if (!lane_end || !lane_state || !chunk_v || !chunk_n) { rc = TANS_E_NOMEM; goto fail; }
    for (uint32_t l = 0; l < lanes; l++) {
        /* symbols l, l + lanes, ... encoded last to first; their bits are
           written in the order the decoder reads them backwards */
        uint64_t cnt = n > l ? (n - l + lanes - 1) / lanes : 0;
        uint32_t st = L;
        for (uint64_t j = cnt; j-- > 0;) {
            const uint32_t s = x[l + j * lanes];
            uint32_t nb = 0;
            while ((st >> nb) >= 2u * c[s]) nb++;
            chunk_v[j] = st & ((1u << nb) - 1);
            chunk_n[j] = nb;
            const uint32_t y = st >> nb; /* in [c_s, 2 c_s) */
            st = L + pos_of[cum[s] + y - c[s]];
        }
        /* the decoder reads from the lane's end backwards: the chunk of the
           first symbol must be last */
        for (uint64_t j = cnt; j-- > 0;)
            if (put_bits(&w, chunk_v[j], chunk_n[j])) { rc = TANS_E_NOMEM; goto fail; }
        if (w.bits >= (1ull << 32)) { rc = TANS_E_INVAL; goto fail; }
        lane_end[l] = (uint32_t)w.bits;
        lane_state[l] = st;
    }
    {
        const uint64_t bs_bytes = (w.bits + 7) / 8;
        const uint64_t total = TANS_HDR + TANS_COUNTS + 8ull * lanes + bs_bytes + 8;
        uint8_t *o = calloc(total, 1);
        if (!o) { rc = TANS_E_NOMEM; goto fail; }
        memcpy(o, "ACT1", 4);
        wr32t(o + 4, (uint32_t)n);
        wr32t(o + 8, R);
        wr32t(o + 12, lanes);
        wr64t(o + 16, total);
        wr32t(o + 24, (uint32_t)bs_bytes);
        for (int s = 0; s < 256; s++) wr16t(o + TANS_HDR + 2 * s, c[s]);
        for (uint32_t l = 0; l < lanes; l++) {
            wr32t(o + TANS_HDR + TANS_COUNTS + 8ull * l, lane_end[l]);
            wr32t(o + TANS_HDR + TANS_COUNTS + 8ull * l + 4, lane_state[l]);
        }
        if (bs_bytes) memcpy(o + TANS_HDR + TANS_COUNTS + 8ull * lanes, w.p, bs_bytes);
        free(w.p); free(lane_end); free(lane_state); free(chunk_v); free(chunk_n); free(sym); free(pos_of);
        *out = o;
        return (int64_t)total;
    }
fail:
    free(w.p); free(lane_end); free(lane_state); free(chunk_v); free(chunk_n); free(sym); free(pos_of);
    return rc;
}

/* read nb bits ending at bit position `end` (exclusive), LSB-first order */
static uint32_t get_bits(const uint8_t *p, uint64_t start, uint32_t nb)
{
    uint32_t v = 0;
    for (uint32_t i = 0; i < nb; i++) {
        const uint64_t b = start + i;
        v |= (uint32_t)((p[b >> 3] >> (b & 7)) & 1u) << i;
    }
    return v;
}

/* decode a container into out[0, cap); the number of symbols goes to *n_out */
int orc_tans_decode(const uint8_t *in, uint64_t len, uint8_t *out, uint64_t cap, uint64_t *n_out)
{
    if (!in || len < TANS_HDR + TANS_COUNTS || memcmp(in, "ACT1", 4) != 0) return TANS_E_FORMAT;
    const uint32_t n = rd32t(in + 4), R = rd32t(in + 8), lanes = rd32t(in + 12);
    const uint64_t total = rd64t(in + 16);
    const uint32_t bs_bytes = rd32t(in + 24);
    if (R < 8 || R > 15 || lanes == 0 || total != len || rd32t(in + 28) != 0) return TANS_E_FORMAT;
    if ((uint64_t)TANS_HDR + TANS_COUNTS + 8ull * lanes + bs_bytes + 8 != len) return TANS_E_FORMAT;
    if (n_out) *n_out = n;
    if (cap < n) return TANS_E_CAPACITY;
    const uint32_t L = 1u << R;
    uint32_t c[256], cum[257];
    cum[0] = 0;
    for (int s = 0; s < 256; s++) {
        c[s] = rd16t(in + TANS_HDR + 2 * s);
        cum[s + 1] = cum[s] + c[s];
    }
    if (n && cum[256] != L) return TANS_E_CORRUPT;
    /* the decoding table: for each position, its symbol and state value */
    uint16_t *sym = malloc(sizeof(uint16_t) * L);
    uint32_t *pos_of = malloc(sizeof(uint32_t) * L), *yv = malloc(sizeof(uint32_t) * L);
    if (!sym || !pos_of || !yv) { free(sym); free(pos_of); free(yv); return TANS_E_NOMEM; }
    if (n) {
        spread(c, cum, R, sym, pos_of);
        for (uint32_t s = 0; s < 256; s++)
            for (uint32_t j = 0; j < c[s]; j++) yv[pos_of[cum[s] + j]] = c[s] + j;
    }
    const uint8_t *lt = in + TANS_HDR + TANS_COUNTS;
    const uint8_t *bits = lt + 8ull * lanes;
    int rc = TANS_OK;
    uint64_t prev_end = 0;
    for (uint32_t l = 0; l < lanes && !rc; l++) {
        const uint64_t end = rd32t(lt + 8ull * l);
        uint32_t st = rd32t(lt + 8ull * l + 4);
        if (end < prev_end || end > 8ull * bs_bytes || st < L || st >= 2 * L) { rc = TANS_E_CORRUPT; break; }
        uint64_t pos = end;
        const uint64_t cnt = n > l ? ((uint64_t)n - l + lanes - 1) / lanes : 0;
        for (uint64_t j = 0; j < cnt; j++) {
            const uint32_t p = st - L;
            const uint32_t s = sym[p];
            out[l + j * lanes] = (uint8_t)s;
            const uint32_t y = yv[p];
            const uint32_t nb = R - floor_log2(y);
            if (pos < prev_end + nb) { rc = TANS_E_CORRUPT; break; }
            pos -= nb;
            st = (y << nb) + get_bits(bits, pos, nb);
            if (st < L || st >= 2 * L) { rc = TANS_E_CORRUPT; break; }
        }
        /* every bit of the lane read, and the encoder's start state reached */
        if (!rc && (pos != prev_end || st != L)) rc = TANS_E_CORRUPT;
        prev_end = end;
    }
    free(sym);
    free(pos_of);
    free(yv);
    return rc;
}
