/*
 * Sanitizer driver for the oracle (test infrastructure only): built by
 * tests/test_sanitizers.py with gcc under AddressSanitizer + UBSan and, for the
 * threaded block decoder, ThreadSanitizer.  For each input file it encodes
 * under several option sets, decodes sequentially and block-parallel with
 * 1, 3 and 8 threads, recomputes every level, then decodes damaged copies of
 * each stream (single-byte flips), and round-trips the tANS coder and damaged
 * containers of it.  Any mismatch exits non-zero; any memory error, data race
 * or undefined behaviour aborts through the sanitizer.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t block_log2, min_match, flatten, max_depth, chain_depth, hash_bits, tiebreak, chunk_log2, levels;
} orc_opts;
typedef struct {
    uint64_t n_seq, n_lit_bytes, match_bytes, n_deep, level_sum;
    uint32_t max_level, n_blocks;
    uint64_t inblock_nonliteral_src_bytes, level_mismatch, depth_violations;
} orc_report;

int64_t orc_encode(const uint8_t *x, uint64_t n, const orc_opts *o, uint8_t **out);
int orc_decode(const uint8_t *s, uint64_t slen, uint8_t *out, uint64_t cap, uint64_t *n_out);
int orc_decode_mt(const uint8_t *s, uint64_t slen, uint8_t *out, uint64_t cap, int nthreads);
int orc_check(const uint8_t *x, uint64_t n, const uint8_t *s, uint64_t slen, orc_report *rep);
int64_t orc_tans_encode(const uint8_t *x, uint64_t n, uint32_t R, uint32_t lanes, uint8_t **out);
int orc_tans_decode(const uint8_t *in, uint64_t len, uint8_t *out, uint64_t cap, uint64_t *n_out);
void orc_free(void *p);

static uint64_t rng = 0x243F6A8885A308D3ull;
static uint64_t next(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
}

#define FAIL(...) do { fprintf(stderr, __VA_ARGS__); fputc('\n', stderr); exit(1); } while (0)

static void lz(const uint8_t *x, uint64_t n, orc_opts o, int flips, int mt)
{
    uint8_t *s = NULL;
    int64_t sl = orc_encode(x, n, &o, &s);
    if (sl < 0) FAIL("encode rc %lld", (long long)sl);
    uint8_t *y = malloc(n ? n : 1);
    uint64_t got = 0;
    if (orc_decode(s, (uint64_t)sl, y, n, &got) || got != n || memcmp(x, y, n)) FAIL("sequential decode differs");
    if (mt) {
        for (int t = 1; t <= 8; t += t == 1 ? 2 : 5) {
            memset(y, 0, n);
            if (orc_decode_mt(s, (uint64_t)sl, y, n, t) || memcmp(x, y, n)) FAIL("decode_mt(%d) differs", t);
        }
    }
    orc_report r;
    if (orc_check(x, n, s, (uint64_t)sl, &r) || r.level_mismatch || r.depth_violations) FAIL("check failed");
    uint8_t *d = malloc((size_t)sl);
    for (int k = 0; k < flips; k++) {
        memcpy(d, s, (size_t)sl);
        d[next() % (uint64_t)sl] ^= (uint8_t)(1u << (next() % 8));
        (void)orc_decode(d, (uint64_t)sl, y, n, &got);
        if (mt && k % 4 == 0) (void)orc_decode_mt(d, (uint64_t)sl, y, n, 4);
    }
    free(d);
    free(y);
    orc_free(s);
}

static void tans(const uint8_t *x, uint64_t n, uint32_t R, uint32_t lanes, int flips)
{
    uint8_t *c = NULL;
    int64_t cl = orc_tans_encode(x, n, R, lanes, &c);
    if (cl < 0) FAIL("tans encode rc %lld", (long long)cl);
    uint8_t *y = malloc(n ? n : 1);
    uint64_t got = 0;
    if (orc_tans_decode(c, (uint64_t)cl, y, n, &got) || got != n || memcmp(x, y, n)) FAIL("tans decode differs");
    uint8_t *d = malloc((size_t)cl);
    for (int k = 0; k < flips; k++) {
        memcpy(d, c, (size_t)cl);
        d[next() % (uint64_t)cl] ^= (uint8_t)(1u << (next() % 8));
        (void)orc_tans_decode(d, (uint64_t)cl, y, n, &got);
    }
    free(d);
    free(y);
    orc_free(c);
}

int main(int argc, char **argv)
{
    const int mt_only = argc > 1 && !strcmp(argv[1], "--mt-only");
    for (int a = 1 + mt_only; a < argc; a++) {
        FILE *f = fopen(argv[a], "rb");
        if (!f) FAIL("cannot open %s", argv[a]);
        fseek(f, 0, SEEK_END);
        const long n = ftell(f);
        fseek(f, 0, SEEK_SET);
        uint8_t *x = malloc(n ? (size_t)n : 1);
        if (fread(x, 1, (size_t)n, f) != (size_t)n) FAIL("short read");
        fclose(f);
        const orc_opts base = {16, 4, 0, 0, 32, 16, 0, 10, 1};
        orc_opts o[5] = {base, base, base, base, base};
        o[1].flatten = 1;
        o[2].max_depth = 4;
        o[3].levels = 0, o[3].block_log2 = 12;
        o[4].block_log2 = 9, o[4].chunk_log2 = 2, o[4].flatten = 2;
        for (int k = 0; k < 5; k++) lz(x, (uint64_t)n, o[k], mt_only ? 8 : 64, 1);
        if (!mt_only) {
            const uint32_t lanes[3] = {1, 5, 32};
            for (int k = 0; k < 3; k++) tans(x, (uint64_t)n, k == 1 ? 9 : 11, lanes[k], 32);
        }
        printf("ok %s %ld\n", argv[a], n);
        free(x);
    }
    return 0;
}
