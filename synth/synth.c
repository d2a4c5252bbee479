/*
 * Seeded synthetic inputs for the absolute-offset LZ77 decoder.
 *
 * This module produces raw bytes only.  It holds none of the codec's
 * arithmetic (no match finding, no offsets, no levels): both the oracle and
 * the GPU path consume what it writes.  The paper measures on enwik9, FASTQ
 * NA12878, silesia and nci (Sec. 4.2); those corpora are not available, so
 * these generators stand in for them with the same kind of structure:
 *
 *   markov  - order-2 Markov text over 64 printable symbols plus an overlay of
 *             copies of earlier substrings (text-like, moderate repetition)
 *   fastq   - FASTQ-like records: header, 150 bp read over ACGT with 1% N,
 *             '+', 150 Phred+33 qualities from a clipped normal; 10% of the
 *             reads are near-duplicates of an earlier read
 *   wiki    - wiki-markup-like text: Zipf(1.1) words from a seeded 50k-word
 *             vocabulary, sentences, XML-style tags, repeated template lines
 *   random  - uniform bytes plus a copy overlay
 *
 * Randomness: xoshiro256** (Blackman and Vigna, 2018) seeded through
 * SplitMix64 (Steele, Lea and Flood, 2014), both from their published
 * definitions.  Every draw is an integer or a double built from the top 53
 * bits, so the output is bit-identical on every platform.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64_next(uint64_t *x)
{
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t synth_splitmix64(uint64_t x) { return splitmix64_next(&x); }

static void rng_seed(rng_t *r, uint64_t seed)
{
    uint64_t x = seed;
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64_next(&x);
}

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t *r)
{
    uint64_t *s = r->s;
    uint64_t result = rotl64(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

/* uniform integer in [0, n), n > 0, by rejection of the biased tail */
static uint64_t rng_below(rng_t *r, uint64_t n)
{
    uint64_t lim = UINT64_MAX - (UINT64_MAX % n);
    uint64_t v;
    do { v = rng_next(r); } while (v >= lim);
    return v % n;
}

/* uniform integer in [a, b] */
static uint64_t rng_range(rng_t *r, uint64_t a, uint64_t b) { return a + rng_below(r, b - a + 1); }

/* uniform double in [0, 1) */
static double rng_unit(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* standard normal, Box-Muller (cosine branch only) */
static double rng_normal(rng_t *r)
{
    double u1 = 1.0 - rng_unit(r); /* (0, 1] */
    double u2 = rng_unit(r);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* ---------------------------------------------------------------- overlay */

typedef struct { uint64_t d, l; } span_t;

static int span_cmp(const void *a, const void *b)
{
    const span_t *x = a, *y = b;
    return (x->d > y->d) - (x->d < y->d);
}

/*
 * Overwrite about frac*n bytes with copies of earlier substrings: pick
 * non-intersecting destinations d ~ U[64, n-64] with lengths l ~ U[4, 64]
 * until their total reaches frac*n, then, in increasing d, copy
 * x[s, s+l) -> x[d, d+l) from s ~ U[0, d-l] of the current buffer.
 */
static int overlay(uint8_t *x, uint64_t n, double frac, rng_t *r)
{
    if (n < 256 || frac <= 0.0) return 0;
    uint8_t *taken = calloc(n, 1);
    uint64_t cap = 1024, cnt = 0, total = 0;
    span_t *sp = malloc(cap * sizeof(span_t));
    if (!taken || !sp) { free(taken); free(sp); return -1; }
    double target = frac * (double)n;
    uint64_t attempts = 0, max_attempts = 64 * n + 1024;
    while ((double)total < target && attempts++ < max_attempts) {
        uint64_t d = rng_range(r, 64, n - 64);
        uint64_t l = rng_range(r, 4, 64);
        int clash = 0;
        for (uint64_t k = 0; k < l; k++) if (taken[d + k]) { clash = 1; break; }
        if (clash) continue;
        memset(taken + d, 1, l);
        if (cnt == cap) {
            cap *= 2;
            span_t *ns = realloc(sp, cap * sizeof(span_t));
            if (!ns) { free(taken); free(sp); return -1; }
            sp = ns;
        }
        sp[cnt].d = d; sp[cnt].l = l; cnt++;
        total += l;
    }
    qsort(sp, cnt, sizeof(span_t), span_cmp);
    for (uint64_t i = 0; i < cnt; i++) {
        uint64_t s = rng_range(r, 0, sp[i].d - sp[i].l);
        memmove(x + sp[i].d, x + s, sp[i].l);
    }
    free(taken);
    free(sp);
    return 0;
}

/* ----------------------------------------------------------------- markov */

static const char ALPHA64[65] =
    "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ0123456789 .";

int synth_markov(uint8_t *out, uint64_t n, uint64_t seed, double copy_frac)
{
    rng_t r;
    rng_seed(&r, seed);
    double *cdf = malloc(sizeof(double) * 4096 * 64);
    if (!cdf) return -1;
    for (int c = 0; c < 4096; c++) {
        double *w = cdf + (size_t)c * 64, sum = 0.0;
        for (int j = 0; j < 64; j++) {
            double u = rng_unit(&r);
            double u2 = u * u, u4 = u2 * u2;
            w[j] = u4 * u4;
            sum += w[j];
        }
        double acc = 0.0;
        for (int j = 0; j < 64; j++) { acc += w[j] / sum; w[j] = acc; }
        w[63] = 2.0; /* every draw in [0,1) lands somewhere */
    }
    unsigned a = 0, b = 0;
    for (uint64_t i = 0; i < n; i++) {
        unsigned sym;
        if (i < 2) {
            sym = (unsigned)rng_below(&r, 64);
        } else {
            const double *w = cdf + (size_t)(a * 64 + b) * 64;
            double u = rng_unit(&r);
            unsigned lo = 0, hi = 63;
            while (lo < hi) { unsigned mid = (lo + hi) / 2; if (w[mid] > u) hi = mid; else lo = mid + 1; }
            sym = lo;
        }
        out[i] = (uint8_t)ALPHA64[sym];
        a = b; b = sym;
    }
    free(cdf);
    return overlay(out, n, copy_frac, &r);
}

/* ------------------------------------------------------------------ fastq */

static uint64_t put_u64(uint8_t *p, uint64_t v)
{
    char tmp[24];
    int k = 0;
    do { tmp[k++] = (char)('0' + v % 10); v /= 10; } while (v);
    for (int i = 0; i < k; i++) p[i] = (uint8_t)tmp[k - 1 - i];
    return (uint64_t)k;
}

int synth_fastq(uint8_t *out, uint64_t n, uint64_t seed)
{
    static const char ACGT[4] = {'A', 'C', 'G', 'T'};
    rng_t r;
    rng_seed(&r, seed);
    uint8_t *buf = malloc(n + 1024);
    uint64_t rcap = 1024, nreads = 0;
    uint64_t *read_at = malloc(rcap * sizeof(uint64_t));
    if (!buf || !read_at) { free(buf); free(read_at); return -1; }
    uint64_t p = 0;
    for (uint64_t i = 1; p < n; i++) {
        buf[p++] = '@';
        buf[p++] = 'R';
        p += put_u64(buf + p, i);
        buf[p++] = ':';
        p += put_u64(buf + p, rng_range(&r, 1, 8));
        buf[p++] = ':';
        p += put_u64(buf + p, rng_range(&r, 1101, 2228));
        buf[p++] = '\n';
        uint8_t *rd = buf + p;
        if (i > 1 && rng_unit(&r) < 0.10) {
            uint64_t j = rng_range(&r, 1, i - 1);
            memcpy(rd, buf + read_at[j - 1], 150);
            unsigned k = (unsigned)rng_range(&r, 1, 3), pos[3];
            for (unsigned t = 0; t < k; t++) {
                unsigned q, dup;
                do {
                    q = (unsigned)rng_below(&r, 150);
                    dup = 0;
                    for (unsigned u = 0; u < t; u++) dup |= (pos[u] == q);
                } while (dup);
                pos[t] = q;
                int cur = -1;
                for (int c = 0; c < 4; c++) if (rd[q] == (uint8_t)ACGT[c]) cur = c;
                if (cur < 0) {
                    rd[q] = (uint8_t)ACGT[rng_below(&r, 4)];
                } else {
                    unsigned v = (unsigned)rng_below(&r, 3);
                    rd[q] = (uint8_t)ACGT[v >= (unsigned)cur ? v + 1 : v];
                }
            }
        } else {
            for (int t = 0; t < 150; t++)
                rd[t] = rng_unit(&r) < 0.01 ? 'N' : (uint8_t)ACGT[rng_below(&r, 4)];
        }
        if (nreads == rcap) {
            rcap *= 2;
            uint64_t *nr = realloc(read_at, rcap * sizeof(uint64_t));
            if (!nr) { free(buf); free(read_at); return -1; }
            read_at = nr;
        }
        read_at[nreads++] = p;
        p += 150;
        buf[p++] = '\n';
        buf[p++] = '+';
        buf[p++] = '\n';
        for (int t = 0; t < 150; t++) {
            double q = nearbyint(36.0 + 4.0 * rng_normal(&r));
            if (q < 2.0) q = 2.0;
            if (q > 41.0) q = 41.0;
            buf[p++] = (uint8_t)(33 + (int)q);
        }
        buf[p++] = '\n';
    }
    memcpy(out, buf, n);
    free(buf);
    free(read_at);
    return 0;
}

/* ------------------------------------------------------------------- wiki */

#define WIKI_VOCAB 50000

static uint64_t fnv1a(const uint8_t *s, unsigned len)
{
    uint64_t h = 1469598103934665603ULL;
    for (unsigned i = 0; i < len; i++) { h ^= s[i]; h *= 1099511628211ULL; }
    return h;
}

typedef struct { uint8_t *dst; uint64_t p, n; } sink_t;

static void sink_put(sink_t *k, const void *src, uint64_t len)
{
    const uint8_t *s = src;
    for (uint64_t i = 0; i < len && k->p < k->n; i++) k->dst[k->p++] = s[i];
}

int synth_wiki(uint8_t *out, uint64_t n, uint64_t seed)
{
    /* word-length weights for lengths 2..12 */
    static const unsigned LW[11] = {6, 10, 12, 12, 11, 10, 9, 8, 7, 6, 5};
    static const char *SKEL[8][2] = {
        {"{{", "}}"}, {"[[", "]]"}, {"* ", ""}, {"== ", " =="},
        {"| ", " |"}, {"<ref>", "</ref>"}, {"'''", "'''"}, {"# ", ":"},
    };
    static const char SEP[8] = {'|', ':', ' ', ' ', '|', ' ', ' ', ','};
    rng_t r;
    rng_seed(&r, seed);
    unsigned lw_tot = 0;
    for (int i = 0; i < 11; i++) lw_tot += LW[i];

    uint8_t *words = malloc((size_t)WIKI_VOCAB * 12);
    uint8_t *wlen = malloc(WIKI_VOCAB);
    const uint32_t HT = 1u << 17;
    int32_t *ht = malloc(sizeof(int32_t) * HT);
    double *zcdf = malloc(sizeof(double) * WIKI_VOCAB);
    if (!words || !wlen || !ht || !zcdf) { free(words); free(wlen); free(ht); free(zcdf); return -1; }
    for (uint32_t i = 0; i < HT; i++) ht[i] = -1;
    for (int w = 0; w < WIKI_VOCAB;) {
        unsigned pick = (unsigned)rng_below(&r, lw_tot), len = 2;
        for (int i = 0; i < 11; i++) { if (pick < LW[i]) { len = 2 + i; break; } pick -= LW[i]; }
        uint8_t *cw = words + (size_t)w * 12;
        for (unsigned t = 0; t < len; t++) cw[t] = (uint8_t)('a' + rng_below(&r, 26));
        uint32_t h = (uint32_t)(fnv1a(cw, len) & (HT - 1));
        int dup = 0;
        while (ht[h] >= 0) {
            int o = ht[h];
            if (wlen[o] == len && memcmp(words + (size_t)o * 12, cw, len) == 0) { dup = 1; break; }
            h = (h + 1) & (HT - 1);
        }
        if (dup) continue;
        ht[h] = w;
        wlen[w] = (uint8_t)len;
        w++;
    }
    double acc = 0.0;
    for (int i = 0; i < WIKI_VOCAB; i++) { acc += pow((double)(i + 1), -1.1); zcdf[i] = acc; }
    for (int i = 0; i < WIKI_VOCAB; i++) zcdf[i] /= acc;
    zcdf[WIKI_VOCAB - 1] = 2.0;

    int tags[8];
    for (int t = 0; t < 8; t++) tags[t] = (int)rng_below(&r, WIKI_VOCAB);

    /* 16 template lines, fixed once per corpus */
    uint8_t tmpl[16][128];
    unsigned tlen[16];
    for (int t = 0; t < 16; t++) {
        int sk = (int)rng_below(&r, 8);
        unsigned nw = (unsigned)rng_range(&r, 2, 6), p = 0;
        const char *o = SKEL[sk][0], *c = SKEL[sk][1];
        memcpy(tmpl[t] + p, o, strlen(o)); p += (unsigned)strlen(o);
        for (unsigned k = 0; k < nw; k++) {
            if (k) tmpl[t][p++] = (uint8_t)SEP[sk];
            int w = (int)rng_below(&r, WIKI_VOCAB);
            memcpy(tmpl[t] + p, words + (size_t)w * 12, wlen[w]); p += wlen[w];
        }
        memcpy(tmpl[t] + p, c, strlen(c)); p += (unsigned)strlen(c);
        tlen[t] = p;
    }

    sink_t k = {out, 0, n};
    uint64_t since_tag = 0, gap = rng_range(&r, 300, 500);
    int open_tag = -1;
    while (k.p < n) {
        unsigned nw = (unsigned)rng_range(&r, 5, 30);
        uint64_t start = k.p;
        for (unsigned i = 0; i < nw; i++) {
            double u = rng_unit(&r);
            unsigned lo = 0, hi = WIKI_VOCAB - 1;
            while (lo < hi) { unsigned mid = (lo + hi) / 2; if (zcdf[mid] > u) hi = mid; else lo = mid + 1; }
            const uint8_t *w = words + (size_t)lo * 12;
            if (i) sink_put(&k, " ", 1);
            if (i == 0) {
                uint8_t cap = (uint8_t)(w[0] - 'a' + 'A');
                sink_put(&k, &cap, 1);
                sink_put(&k, w + 1, wlen[lo] - 1);
            } else {
                sink_put(&k, w, wlen[lo]);
            }
        }
        sink_put(&k, ". ", 2);
        since_tag += k.p - start;
        if (since_tag >= gap) {
            if (open_tag < 0) {
                open_tag = tags[rng_below(&r, 8)];
                sink_put(&k, "\n<", 2);
                sink_put(&k, words + (size_t)open_tag * 12, wlen[open_tag]);
                sink_put(&k, ">", 1);
            } else {
                sink_put(&k, "</", 2);
                sink_put(&k, words + (size_t)open_tag * 12, wlen[open_tag]);
                sink_put(&k, ">\n", 2);
                open_tag = -1;
            }
            since_tag = 0;
            gap = rng_range(&r, 300, 500);
        }
        if (rng_unit(&r) < 0.05) {
            int t = (int)rng_below(&r, 16);
            sink_put(&k, "\n", 1);
            sink_put(&k, tmpl[t], tlen[t]);
            sink_put(&k, "\n", 1);
        }
    }
    free(words); free(wlen); free(ht); free(zcdf);
    return 0;
}

/* ----------------------------------------------------------------- random */

int synth_random(uint8_t *out, uint64_t n, uint64_t seed, double copy_frac)
{
    rng_t r;
    rng_seed(&r, seed);
    uint64_t i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t v = rng_next(&r);
        memcpy(out + i, &v, 8);
    }
    if (i < n) {
        uint64_t v = rng_next(&r);
        memcpy(out + i, &v, n - i);
    }
    return overlay(out, n, copy_frac, &r);
}

/* --------------------------------------------------------- plain draws */

/* n doubles uniform in [0,1) from the generator seeded with `seed` */
void synth_uniform(double *out, uint64_t n, uint64_t seed)
{
    rng_t r;
    rng_seed(&r, seed);
    for (uint64_t i = 0; i < n; i++) out[i] = rng_unit(&r);
}

/* n raw 64-bit outputs of xoshiro256** from the state s[0..3] as given */
void synth_raw_state(uint64_t *out, uint64_t n, const uint64_t *state)
{
    rng_t r;
    for (int i = 0; i < 4; i++) r.s[i] = state[i];
    for (uint64_t i = 0; i < n; i++) out[i] = rng_next(&r);
}

/* n raw 64-bit outputs of xoshiro256** seeded with `seed` */
void synth_raw(uint64_t *out, uint64_t n, uint64_t seed)
{
    rng_t r;
    rng_seed(&r, seed);
    for (uint64_t i = 0; i < n; i++) out[i] = rng_next(&r);
}
