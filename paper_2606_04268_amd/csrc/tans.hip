// Entropy stage for the literal stream on MI355X (gfx950): table-based
// asymmetric numeral systems (tANS), the coding the paper names for its four
// streams and leaves to future work (Sec. 4.4, Sec. 8).  A container holds the
// normalized counts of its bytes and many independent lanes: symbol i belongs
// to lane i mod lanes, and each lane is coded on its own, so that one GPU
// thread decodes one lane and the 64 lanes of a wave write 64 consecutive
// output bytes per step.
//
// Container ("ACT1", little-endian):
//   0 char[4] "ACT1"   4 u32 n (symbols)   8 u32 table_log R   12 u32 lanes
//   16 u64 total bytes  24 u32 bitstream bytes  28 u32 0
//   32: u16 counts[256], summing to L = 2^R
//   544: lanes x {u32 end bit of the lane's bits, u32 initial decoder state}
//   then the lanes' bits (LSB-first, lane after lane, each from the previous
//   lane's end bit) and 8 zero bytes of slack.
//
// Coding (tANS): the i-th table entry in symbol order (cumulative counts)
// goes to position (i * step) mod L, step = L/2 + L/8 + 3; the positions of
// symbol s, in increasing order, carry the state values y = c_s .. 2 c_s - 1.
// A decoder in state x in [L, 2L) reads position x - L: its symbol is the
// output, and the next state is (y << nb) + the next nb bits of the lane, nb =
// R - floor(log2 y), reading the lane's bits from its end towards its start.
// The encoder (host, below) runs each lane's symbols last to first from state
// L, emitting for symbol s the nb low bits of x that bring x >> nb into
// [c_s, 2 c_s) and moving to L + the position of state value x >> nb.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <thread>
#include <vector>

#include "aceapex.h"
#include "internal.h"

namespace {

constexpr uint32_t TH = 32, TC = 512;     // header and counts bytes
constexpr uint32_t R_MIN = 8, R_MAX = 12;  // table sizes 256 .. 4096 entries
constexpr int NTT = 256;                   // threads of the lane decoder
constexpr int NTB = 256;                   // threads per workgroup of the table build (one per symbol and entry)


__host__ __device__ inline uint32_t rd32(const uint8_t *p)
{
    uint32_t v;
    memcpy(&v, p, 4);
    return v;
}
inline uint64_t rd64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }

struct TansArgs {
    const uint8_t *in;      // container
    uint8_t *out;
    uint32_t *table;        // L decode entries: symbol | nb << 8 | (y << nb) << 13
    int32_t *status;
    uint32_t n, R, lanes, bs_bytes;
};

// sum_{i<n} floor((a*i + b) / m) for m >= 1 and a, b >= 0, by the Euclidean
// reduction of floor sums (O(log m) steps).  In 32 bits: for tables of at
// most 2^12 entries every term here stays below 2^26.
__device__ __forceinline__ uint32_t floor_sum(uint32_t n, uint32_t m, uint32_t a, uint32_t b)
{
    uint32_t ans = 0;
    for (;;) {
        if (a >= m) {
            ans += (n - 1) * n / 2 * (a / m);
            a %= m;
        }
        if (b >= m) {
            ans += n * (b / m);
            b %= m;
        }
        const uint32_t y = a * n + b;
        if (y < m) return ans;
        n = y / m;
        b = y % m;
        const uint32_t t = m;
        m = a;
        a = t;
    }
}

// The decode table from the counts, one thread per table entry in L / 256
// workgroups that each scan the counts.  Each table entry i in symbol order
// finds its symbol s
// by binary search and its position p = (i * step) mod L.  Its state value
// is c_s plus the number of s's entries whose positions lie below p; entry j
// of s sits at (j * step) mod L, and [x mod L < p] = 1 + floor(x / L) -
// floor((x + L - p) / L), so that number is c_s plus a difference of two
// floor sums over s's range of entries, with no pass over the table.
__global__ void __launch_bounds__(NTB) k_tans_table(TansArgs A)
{
    __shared__ uint32_t cum[257];
    const uint32_t t = threadIdx.x, L = 1u << A.R, step = (L >> 1) + (L >> 3) + 3;
    cum[t + 1] = A.in[TH + 2 * t] | ((uint32_t)A.in[TH + 2 * t + 1] << 8);
    if (t == 0) cum[0] = 0;
    __syncthreads();
    for (uint32_t d = 1; d < 256; d <<= 1) {  // inclusive scan of cum[1..256]
        const uint32_t v = t >= d ? cum[t + 1 - d] : 0;
        __syncthreads();
        cum[t + 1] += v;
        __syncthreads();
    }
    if (blockIdx.x == 0 && t == 0)
        *A.status = (A.n && cum[256] != L) ? ACEAPEX_E_CORRUPT : 0;  // the decode's status starts here
    if (cum[256] != L) return;
    {
        const uint32_t i = blockIdx.x * NTB + t;  // < L: the grid is L / NTB workgroups
        uint32_t lo = 0, hi = 255;  // the symbol whose cumulative range holds i
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (cum[mid] <= i) lo = mid; else hi = mid - 1;
        }
        const uint32_t c0 = cum[lo], c = cum[lo + 1] - c0, p = (uint32_t)(((uint64_t)i * step) & (L - 1));
        const uint32_t x0 = step * c0;
        const uint32_t below = c + floor_sum(c, L, step, x0) - floor_sum(c, L, step, x0 + L - p);
        const uint32_t y = c + below;
        const uint32_t nb = A.R - (31 - __clz(y));
        A.table[p] = lo | (nb << 8) | ((y << nb) << 13);
    }
}

// The 32 bits at bit offset b (a multiple of 32) of the lane bits; zero
// before the start.
__device__ __forceinline__ uint64_t bits32(const uint8_t *bits, int64_t b)
{
    return b < 0 ? 0 : (uint64_t)*(const uint32_t *)(bits + (b >> 3));
}

// One thread per lane: the table in LDS, the lane's bits read backwards
// through a 64-bit window held in registers.  The window covers bits
// [wpos, wpos + 64) with wpos a multiple of 32 and at least 32 bits of it
// below the read position, so every read of at most R <= 12 bits comes from
// the window; a read that leaves fewer than 32 bits below the position slides
// the window down by one aligned 32-bit word.  Reads past the end of the
// last lane fall in the container's 8 bytes of slack.
__global__ void __launch_bounds__(NTT) k_tans(TansArgs A)
{
    __shared__ uint32_t T[1u << R_MAX];
    const uint32_t L = 1u << A.R;
    for (uint32_t i = threadIdx.x; i < L; i += NTT) T[i] = A.table[i];
    __syncthreads();
    if (*A.status) return;
    const uint32_t lane = blockIdx.x * NTT + threadIdx.x;
    if (lane >= A.lanes) return;
    const uint8_t *lt = A.in + TH + TC;
    const uint8_t *bits = lt + 8ull * A.lanes;
    const uint64_t start = lane ? rd32(lt + 8ull * (lane - 1)) : 0, end = rd32(lt + 8ull * lane);
    uint32_t st = rd32(lt + 8ull * lane + 4);
    if (end < start || end > 8ull * A.bs_bytes || st < L || st >= 2 * L) {
        atomicCAS(A.status, 0, ACEAPEX_E_CORRUPT);
        return;
    }
    const uint32_t cnt = A.n > lane ? (A.n - lane + A.lanes - 1) / A.lanes : 0;
    int64_t pos = (int64_t)end;
    int64_t wpos = ((pos >> 5) << 5) - 32;
    uint64_t win = bits32(bits, wpos) | (bits32(bits, wpos + 32) << 32);
    uint8_t *o = A.out + lane;
    bool bad = false;
    for (uint32_t j = 0; j < cnt; j++) {
        const uint32_t e = T[st - L];
        o[(uint64_t)j * A.lanes] = (uint8_t)e;
        const uint32_t nb = (e >> 8) & 31;
        if (pos - (int64_t)start < (int64_t)nb) {
            bad = true;
            break;
        }
        pos -= nb;
        st = (e >> 13) + ((uint32_t)(win >> (uint32_t)(pos - wpos)) & ((1u << nb) - 1));
        if (pos - wpos < 32) {
            wpos -= 32;
            win = (win << 32) | bits32(bits, wpos);
        }
    }
    if (bad || pos != (int64_t)start || st != L) atomicCAS(A.status, 0, ACEAPEX_E_CORRUPT);
}

}  // namespace

extern "C" {

int aceapex_tans_probe(const void *h_prefix, size_t h_len, aceapex_tans_info *info)
{
    if (!h_prefix || !info || h_len < TH + TC) return ACEAPEX_E_INVAL;
    const uint8_t *h = (const uint8_t *)h_prefix;
    if (memcmp(h, "ACT1", 4) != 0 || rd32(h + 28) != 0) return ACEAPEX_E_FORMAT;
    aceapex_tans_info in;
    in.n = rd32(h + 4);
    in.table_log = rd32(h + 8);
    in.lanes = rd32(h + 12);
    in.container_bytes = rd64(h + 16);
    in.bitstream_bytes = rd32(h + 24);
    if (in.table_log < R_MIN || in.table_log > R_MAX || in.lanes == 0) return ACEAPEX_E_FORMAT;
    if ((uint64_t)TH + TC + 8ull * in.lanes + in.bitstream_bytes + 8 != in.container_bytes) return ACEAPEX_E_FORMAT;
    uint32_t sum = 0;
    for (uint32_t s = 0; s < 256; s++) sum += h[TH + 2 * s] | ((uint32_t)h[TH + 2 * s + 1] << 8);
    if (in.n && sum != (1u << in.table_log)) return ACEAPEX_E_FORMAT;
    *info = in;
    return ACEAPEX_OK;
}

size_t aceapex_tans_workspace_bytes(const aceapex_tans_info *info)
{
    if (!info || info->table_log > R_MAX) return 0;
    return 256 + 4ull * (1u << info->table_log);
}

int aceapex_tans_decode(const void *d_in, const aceapex_tans_info *info, void *d_out, uint64_t out_capacity,
                        void *d_workspace, size_t ws_bytes, int32_t *d_status, void *hip_stream)
{
    if (!d_in || !info || (info->n && !d_out) || !d_status) return ACEAPEX_E_INVAL;
    if (info->table_log < R_MIN || info->table_log > R_MAX || info->lanes == 0 ||
        info->container_bytes != (uint64_t)TH + TC + 8ull * info->lanes + info->bitstream_bytes + 8)
        return ACEAPEX_E_FORMAT;
    if (out_capacity < info->n) return ACEAPEX_E_CAPACITY;
    if (!d_workspace || ((uintptr_t)d_workspace & 255) || ws_bytes < aceapex_tans_workspace_bytes(info))
        return ACEAPEX_E_WORKSPACE;
    hipStream_t st = (hipStream_t)hip_stream;
    TansArgs A;
    A.in = (const uint8_t *)d_in;
    A.out = (uint8_t *)d_out;
    A.table = (uint32_t *)((uint8_t *)d_workspace + 256);
    A.status = d_status;
    A.n = (uint32_t)info->n;
    A.R = info->table_log;
    A.lanes = info->lanes;
    A.bs_bytes = info->bitstream_bytes;
    hipLaunchKernelGGL(k_tans_table, dim3((1u << info->table_log) / NTB), dim3(NTB), 0, st, A);
    hipLaunchKernelGGL(k_tans, dim3((info->lanes + NTT - 1) / NTT), dim3(NTT), 0, st, A);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        aceapex_impl::set_last_hip_error((int)e);
        return ACEAPEX_E_HIP;
    }
    return ACEAPEX_OK;
}

// Host encoder of the same container.  The normalized counts follow the
// definition in the header; lanes are coded in parallel into their own bit
// buffers, then packed one after the other.
int64_t aceapex_tans_encode(const void *h_in, uint64_t n, uint32_t table_log, uint32_t lanes, void **h_out)
{
    if (!h_out) return ACEAPEX_E_INVAL;
    *h_out = nullptr;
    if ((n && !h_in) || table_log < R_MIN || table_log > R_MAX || lanes == 0 || lanes > (1u << 24) ||
        n >= (1ull << 32))
        return ACEAPEX_E_INVAL;
    const uint8_t *x = (const uint8_t *)h_in;
    const uint32_t R = table_log, L = 1u << R, step = (L >> 1) + (L >> 3) + 3;
    try {
        // counts: floor(h_s * L / n), at least 1 for a present symbol, then
        // one unit at a time on the largest (lowest byte among equals)
        uint64_t h[256] = {0};
        for (uint64_t i = 0; i < n; i++) h[x[i]]++;
        uint32_t c[256];
        int64_t sum = 0;
        for (int s = 0; s < 256; s++) {
            uint64_t v = n ? h[s] * L / n : 0;
            if (h[s] && !v) v = 1;
            c[s] = (uint32_t)v;
            sum += v;
        }
        while (n && sum != (int64_t)L) {
            if (sum < (int64_t)L) {
                int big = (int)(std::max_element(c, c + 256) - c);
                c[big]++;
                sum++;
            } else {
                int t = -1;
                for (int s = 0; s < 256; s++)
                    if (c[s] > 1 && (t < 0 || c[s] > c[t])) t = s;
                if (t < 0) return ACEAPEX_E_INVAL;
                c[t]--;
                sum--;
            }
        }
        // where each state value of each symbol sits: the spread, then the
        // positions of each symbol in increasing order
        std::vector<uint32_t> cum(257, 0), at(n ? L : 1);
        for (int s = 0; s < 256; s++) cum[s + 1] = cum[s] + c[s];
        if (n) {
            std::vector<uint8_t> sym(L);
            for (uint32_t s = 0; s < 256; s++)
                for (uint32_t j = 0; j < c[s]; j++) sym[(uint32_t)(((uint64_t)(cum[s] + j) * step) & (L - 1))] = (uint8_t)s;
            std::vector<uint32_t> next(cum.begin(), cum.end() - 1);
            for (uint32_t p = 0; p < L; p++) at[next[sym[p]]++] = p;
        }
        // each lane: symbols last to first, chunks kept, then written so that
        // the first symbol's chunk ends the lane
        std::vector<std::vector<uint64_t>> lane_words(lanes);
        std::vector<uint64_t> lane_bits(lanes, 0);
        std::vector<uint32_t> lane_state(lanes, L);
        auto code_lane = [&](uint32_t l) {
            const uint64_t cnt = n > l ? (n - l + lanes - 1) / lanes : 0;
            std::vector<uint32_t> cv(cnt), cb(cnt);
            uint32_t xs = L;
            for (uint64_t j = cnt; j-- > 0;) {
                const uint32_t s = x[l + j * lanes];
                uint32_t nb = 0;
                while ((xs >> nb) >= 2 * c[s]) nb++;
                cv[j] = xs & ((1u << nb) - 1);
                cb[j] = nb;
                xs = L + at[cum[s] + (xs >> nb) - c[s]];
            }
            std::vector<uint64_t> &wv = lane_words[l];
            uint64_t bits = 0;
            for (uint64_t j = cnt; j-- > 0;) {
                if ((bits >> 6) + 1 >= wv.size()) wv.resize((bits >> 6) + 2, 0);
                wv[bits >> 6] |= (uint64_t)cv[j] << (bits & 63);
                if ((bits & 63) + cb[j] > 64) wv[(bits >> 6) + 1] |= (uint64_t)cv[j] >> (64 - (bits & 63));
                bits += cb[j];
            }
            lane_bits[l] = bits;
            lane_state[l] = xs;
        };
        const unsigned nt = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 32));
        std::vector<std::thread> pool;
        for (unsigned t = 0; t < nt; t++)
            pool.emplace_back([&, t]() {
                for (uint32_t l = t; l < lanes; l += nt) code_lane(l);
            });
        for (auto &th : pool) th.join();
        uint64_t total_bits = 0;
        for (uint32_t l = 0; l < lanes; l++) total_bits += lane_bits[l];
        if (total_bits >= (1ull << 32)) return ACEAPEX_E_INVAL;
        const uint64_t bs = (total_bits + 7) / 8;
        const uint64_t total = TH + TC + 8ull * lanes + bs + 8;
        uint8_t *o = (uint8_t *)calloc(total + 8, 1);  // + 8: whole-word writes past the end
        if (!o) return ACEAPEX_E_NOMEM;
        memcpy(o, "ACT1", 4);
        const uint32_t n32 = (uint32_t)n, bs32 = (uint32_t)bs;
        memcpy(o + 4, &n32, 4);
        memcpy(o + 8, &R, 4);
        memcpy(o + 12, &lanes, 4);
        memcpy(o + 16, &total, 8);
        memcpy(o + 24, &bs32, 4);
        for (int s = 0; s < 256; s++) {
            const uint16_t v = (uint16_t)c[s];
            memcpy(o + TH + 2 * s, &v, 2);
        }
        uint8_t *bits = o + TH + TC + 8ull * lanes;
        uint64_t at_bit = 0;
        for (uint32_t l = 0; l < lanes; l++) {
            const std::vector<uint64_t> &wv = lane_words[l];
            for (uint64_t b = 0; b < lane_bits[l]; b += 64) {
                const uint32_t k = (uint32_t)std::min<uint64_t>(64, lane_bits[l] - b);
                uint64_t v = wv[b >> 6];
                if (k < 64) v &= (1ull << k) - 1;
                // OR v into the bit string at at_bit + b (little-endian bytes)
                const uint64_t p = at_bit + b;
                uint64_t lo, hi;
                memcpy(&lo, bits + (p >> 3), 8);
                lo |= v << (p & 7);
                memcpy(bits + (p >> 3), &lo, 8);
                if ((p & 7) && (v >> (64 - (p & 7)))) {
                    memcpy(&hi, bits + (p >> 3) + 8, 8);
                    hi |= v >> (64 - (p & 7));
                    memcpy(bits + (p >> 3) + 8, &hi, 8);
                }
            }
            at_bit += lane_bits[l];
            const uint32_t e32 = (uint32_t)at_bit;
            memcpy(o + TH + TC + 8ull * l, &e32, 4);
            memcpy(o + TH + TC + 8ull * l + 4, &lane_state[l], 4);
        }
        *h_out = o;
        return (int64_t)total;
    } catch (const std::bad_alloc &) {
        return ACEAPEX_E_NOMEM;
    }
}

}  // extern "C"
