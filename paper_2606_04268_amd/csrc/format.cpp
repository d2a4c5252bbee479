// Stream header parsing (host only): the 64-byte header of the absolute-offset
// LZ77 stream (ACEAPEX, arXiv 2606.04268, Sec. 3.1-3.2 for the block layout,
// Sec. 7.1 for the optional level table) and the consistency rules every
// decoder applies before it trusts the header's sizes.  Shared by the GPU
// decoder, the host decoder and the planners; no HIP here, so the host
// decoder builds and runs without a GPU toolchain.
#include <stdint.h>
#include <string.h>

#include "aceapex.h"
#include "internal.h"

namespace {

constexpr uint64_t HDR = 64;

inline uint16_t rd16(const uint8_t *p) { uint16_t v; memcpy(&v, p, 2); return v; }
inline uint32_t rd32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
inline uint64_t rd64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }

}  // namespace

namespace aceapex_impl {

bool has_table(const aceapex_info &in) { return (in.flags & 8u) != 0; }

uint64_t prefix_bytes(const aceapex_info &in)
{
    const uint64_t table = has_table(in) ? ((4ull * (in.max_level + 1ull) + 15) & ~15ull) : 0;
    return HDR + 16ull * (in.n_blocks + 1ull) + table;
}

bool info_consistent(const aceapex_info &in)
{
    if (in.block_log2 < 3 || in.block_log2 > 30 || in.min_match < 1 || in.chunk_log2 > 20) return false;
    const uint64_t B = 1ull << in.block_log2;
    if ((in.decoded_bytes + B - 1) / B != in.n_blocks) return false;
    if (in.max_level >= (1u << 28) || in.comp_bytes < prefix_bytes(in)) return false;
    if (in.n_deep > in.n_seq) return false;
    if (!has_table(in) && (in.max_level || in.n_deep)) return false;  // level fields unused without levels
    if (in.n_blocks == 0 && (in.n_seq || in.n_chunks)) return false;
    if (in.n_blocks && in.n_chunks < in.n_blocks) return false;
    return true;
}

}  // namespace aceapex_impl

extern "C" int aceapex_probe(const void *h_stream_prefix, size_t h_len, aceapex_info *info)
{
    if (!h_stream_prefix || !info || h_len < HDR) return ACEAPEX_E_INVAL;
    const uint8_t *h = (const uint8_t *)h_stream_prefix;
    if (memcmp(h, "ACX1", 4) != 0 || rd16(h + 4) != 1) return ACEAPEX_E_FORMAT;
    aceapex_info in;
    in.flags = rd16(h + 6);
    in.block_log2 = h[8];
    in.min_match = h[9];
    in.chunk_log2 = h[10];
    in.max_depth = rd32(h + 12);
    in.decoded_bytes = rd64(h + 16);
    in.comp_bytes = rd64(h + 24);
    in.n_blocks = rd32(h + 32);
    in.max_level = rd32(h + 36);
    in.n_seq = rd32(h + 40);
    in.n_deep = rd32(h + 44);
    in.n_chunks = rd32(h + 48);
    in.content_hash = rd64(h + 56);
    if ((in.flags & ~0xFu) || h[11] != 0 || rd32(h + 52) != 0) return ACEAPEX_E_FORMAT;
    if (!aceapex_impl::info_consistent(in)) return ACEAPEX_E_FORMAT;
    *info = in;
    return ACEAPEX_OK;
}
