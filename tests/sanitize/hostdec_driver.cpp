// Sanitizer driver for the library's host decoder (aceapex_decode_host):
// built by tests/test_sanitizers.py with g++ from the library's host-only
// sources under AddressSanitizer + UBSan and under ThreadSanitizer.  Arguments
// come in pairs, a stream file and the bytes it must decode to.  Each stream
// is decoded with 1, 2 and 8 threads into an output of exactly the decoded
// size, then damaged copies (single-byte flips) are decoded with 1 and 4
// threads: they may decode or be rejected, but any read or write outside the
// buffers, data race or undefined behaviour aborts through the sanitizer.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "aceapex.h"

static std::vector<uint8_t> slurp(const char *path)
{
    std::vector<uint8_t> v;
    FILE *f = fopen(path, "rb");
    if (!f) return v;
    fseek(f, 0, SEEK_END);
    v.resize((size_t)ftell(f));
    fseek(f, 0, SEEK_SET);
    if (fread(v.data(), 1, v.size(), f) != v.size()) v.clear();
    fclose(f);
    return v;
}

int main(int argc, char **argv)
{
    uint64_t r = 0x9E3779B97F4A7C15ull;
    auto next = [&r]() {
        r ^= r << 13;
        r ^= r >> 7;
        r ^= r << 17;
        return r;
    };
    const int flips = argc > 1 && !strcmp(argv[1], "--few") ? 16 : 96;
    for (int a = 1 + (flips == 16); a + 1 < argc; a += 2) {
        const std::vector<uint8_t> s = slurp(argv[a]), want = slurp(argv[a + 1]);
        if (s.empty()) {
            fprintf(stderr, "cannot read %s\n", argv[a]);
            return 1;
        }
        std::vector<uint8_t> out(want.size());
        for (uint32_t t : {1u, 2u, 8u}) {
            std::fill(out.begin(), out.end(), 0);
            const int rc = aceapex_decode_host(s.data(), s.size(), out.data(), out.size(), t);
            if (rc != ACEAPEX_OK || out != want) {
                fprintf(stderr, "%s: threads %u rc %d, output %s\n", argv[a], t, rc, out == want ? "equal" : "differs");
                return 1;
            }
        }
        std::vector<uint8_t> d(s.size());
        int rejected = 0;
        for (int k = 0; k < flips; k++) {
            d = s;
            d[next() % d.size()] ^= (uint8_t)(1u << (next() % 8));
            // an output of exactly the stated size: a corrupt header that
            // claims more is rejected by the capacity check, never written past
            std::vector<uint8_t> o(want.size());
            rejected += aceapex_decode_host(d.data(), d.size(), o.data(), o.size(), k % 2 ? 4 : 1) != ACEAPEX_OK;
        }
        printf("ok %s %zu bytes, %d of %d damaged copies rejected\n", argv[a], want.size(), rejected, flips);
    }
    return 0;
}
