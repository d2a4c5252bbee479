// Verification of a decode (ACEAPEX, arXiv 2606.04268: every decode must
// reproduce its input exactly, Sec. 4.3): a full byte compare of two device
// buffers on the GPU, giving the number of differing bytes and the index of
// the first one.  Off the decode's latency path; the host hash of the
// output is the second check.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aceapex.h"
#include "internal.h"

namespace {

constexpr int NTC = 256;          // threads per workgroup
constexpr uint32_t CMP_WGS = 2048;  // workgroups of the grid-stride compare

// result[0] = 0 mismatches, result[1] = n (no first mismatch yet).
__global__ void k_cmp_init(unsigned long long *result, uint64_t n)
{
    result[0] = 0;
    result[1] = n;
}

// Differing bytes between two 16-byte words.
__device__ __forceinline__ uint32_t diff16(const uint4 &x, const uint4 &y, uint32_t &first)
{
    uint32_t cnt = 0;
    first = 16;
    const uint32_t xa[4] = {x.x, x.y, x.z, x.w}, ya[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
    for (int k = 3; k >= 0; k--) {
        const uint32_t d = xa[k] ^ ya[k];
        // a byte differs when any of its bits does
        const uint32_t m = ((d & 0x7f7f7f7fu) + 0x7f7f7f7fu) | d;
        const uint32_t bytes = m & 0x80808080u;
        cnt += __popc(bytes);
        if (bytes) first = 4 * k + (__ffs(bytes) - 1) / 8;
    }
    return cnt;
}

// Grid-stride over the 16-byte words both buffers share in alignment; the
// bytes before the first aligned word and after the last are compared one
// by one.  One atomic add and one atomic min per wave that saw a mismatch.
__global__ void __launch_bounds__(NTC) k_cmp(const uint8_t *a, const uint8_t *b, uint64_t n, uint64_t head,
                                              uint64_t words, unsigned long long *result)
{
    uint64_t cnt = 0, first = n;
    const uint64_t stride = (uint64_t)gridDim.x * NTC;
    const uint64_t t0 = (uint64_t)blockIdx.x * NTC + threadIdx.x;
    for (uint64_t i = t0; i < head; i += stride)
        if (a[i] != b[i]) {
            cnt++;
            first = first < i ? first : i;
        }
    const uint4 *wa = (const uint4 *)(a + head), *wb = (const uint4 *)(b + head);
    for (uint64_t w = t0; w < words; w += stride) {
        uint32_t f;
        const uint32_t c = diff16(wa[w], wb[w], f);
        if (c) {
            cnt += c;
            const uint64_t at = head + 16 * w + f;
            first = first < at ? first : at;
        }
    }
    for (uint64_t i = head + 16 * words + t0; i < n; i += stride)
        if (a[i] != b[i]) {
            cnt++;
            first = first < i ? first : i;
        }
    // wave reduction, then one atomic pair per wave that found anything
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o, 64);
        const uint64_t f2 = __shfl_xor(first, o, 64);
        first = first < f2 ? first : f2;
    }
    if ((threadIdx.x & 63) == 0 && cnt) {
        atomicAdd(&result[0], (unsigned long long)cnt);
        atomicMin(&result[1], (unsigned long long)first);
    }
}

}  // namespace

extern "C" int aceapex_compare(const void *d_a, const void *d_b, uint64_t n, uint64_t *d_result, void *hip_stream)
{
    if (!d_result || (n && (!d_a || !d_b)) || ((uintptr_t)d_result & 7)) return ACEAPEX_E_INVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    const uintptr_t pa = (uintptr_t)d_a, pb = (uintptr_t)d_b;
    // 16-byte words only where both buffers are 16-byte aligned at the same offset
    uint64_t head = n, words = 0;
    if ((pa & 15) == (pb & 15)) {
        head = (16 - (pa & 15)) & 15;
        if (head > n) head = n;
        words = (n - head) / 16;
    }
    unsigned long long *r = (unsigned long long *)d_result;
    hipLaunchKernelGGL(k_cmp_init, dim3(1), dim3(1), 0, st, r, n);
    const uint64_t need = (words + (n - 16 * words) + NTC - 1) / NTC;
    const uint32_t wgs = (uint32_t)(need < CMP_WGS ? (need ? need : 1) : CMP_WGS);
    hipLaunchKernelGGL(k_cmp, dim3(wgs), dim3(NTC), 0, st, (const uint8_t *)d_a, (const uint8_t *)d_b, n, head,
                       words, r);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        aceapex_impl::set_last_hip_error((int)e);
        return ACEAPEX_E_HIP;
    }
    return ACEAPEX_OK;
}
