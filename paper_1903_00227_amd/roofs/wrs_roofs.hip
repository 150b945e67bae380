// wrs_roofs.hip -- two ceiling kernels the benchmark measures the sampler
// against (not part of the sampling library; built into libwrs_roofs.so).
//
//   wrs_roof_gather: for s in [0, k), the bucket r of the alias query of draw s
//     (Philox-4x32-10 under key `seed`, counter (s lo, s hi, 0, 0), r = the high
//     64 bits of (x1 2^32 + x0) * n), one 8-byte load of buf[r], and a
//     coalesced 4-byte store of its two halves XORed: the sampler's memory
//     traffic without the coin and the select.
//   wrs_roof_philox: the same Philox blocks with no memory access; each block
//     XOR-reduces its draws' four output words and stores one word.
// Both use the sampler's launch shape (256 threads, `unroll` draws per thread).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
    // Philox-4x32-10 (Salmon et al., SC'11): the published round multipliers
    // and key increments
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

constexpr int TPB = 256;
constexpr int UMAX = 8;

__global__ __launch_bounds__(TPB) void k_roof_gather(const uint64_t* __restrict__ buf, uint64_t n, uint64_t seed,
                                                     int64_t k, int unroll, uint32_t* __restrict__ out) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int64_t s0 = (int64_t)blockIdx.x * TPB * unroll + threadIdx.x;
    uint32_t r[UMAX];
#pragma unroll
    for (int e = 0; e < UMAX; ++e) {
        if (e < unroll) {
            const uint64_t c = (uint64_t)(s0 + (int64_t)e * TPB);
            const uint4 x = philox(make_uint4((uint32_t)c, (uint32_t)(c >> 32), 0u, 0u), k0, k1);
            const uint64_t lo = ((uint64_t)x.x * n) >> 32;
            const uint64_t hi = (uint64_t)x.y * n + lo;
            r[e] = (uint32_t)(hi >> 32);
        }
    }
    uint64_t v[UMAX];
#pragma unroll
    for (int e = 0; e < UMAX; ++e) {
        const int64_t s = s0 + (int64_t)e * TPB;
        if (e < unroll) v[e] = (s < k) ? buf[r[e]] : 0ull;
    }
#pragma unroll
    for (int e = 0; e < UMAX; ++e) {
        const int64_t s = s0 + (int64_t)e * TPB;
        if (e < unroll && s < k) out[s] = (uint32_t)v[e] ^ (uint32_t)(v[e] >> 32);
    }
}

__global__ __launch_bounds__(TPB) void k_roof_philox(uint64_t seed, int64_t k, int unroll, uint32_t* __restrict__ out) {
    __shared__ uint32_t red[TPB / 64];
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int64_t s0 = (int64_t)blockIdx.x * TPB * unroll + threadIdx.x;
    uint32_t acc = 0;
    for (int e = 0; e < unroll; ++e) {
        const int64_t s = s0 + (int64_t)e * TPB;
        if (s < k) {
            const uint4 x = philox(make_uint4((uint32_t)s, (uint32_t)((uint64_t)s >> 32), 0u, 0u), k0, k1);
            acc ^= x.x ^ x.y ^ x.z ^ x.w;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = red[0] ^ red[1] ^ red[2] ^ red[3];
}

}  // namespace

extern "C" int64_t wrs_roof_blocks(int64_t k, int unroll) { return (k + (int64_t)TPB * unroll - 1) / ((int64_t)TPB * unroll); }

// buf: n 8-byte words (device); out: k uint32 (device).  0 or a hipError_t.
extern "C" int wrs_roof_gather(const uint64_t* buf, int64_t n, uint64_t seed, int64_t k, int unroll, uint32_t* out,
                               void* stream) {
    if (!buf || !out || n < 1 || n > 2147483647LL || k < 1 || unroll < 1 || unroll > UMAX) return -1;
    hipLaunchKernelGGL(k_roof_gather, dim3((unsigned)wrs_roof_blocks(k, unroll)), dim3(TPB), 0, (hipStream_t)stream,
                       buf, (uint64_t)n, seed, k, unroll, out);
    return (int)hipGetLastError();
}

// out: wrs_roof_blocks(k, unroll) uint32 (device).  0 or a hipError_t.
extern "C" int wrs_roof_philox(uint64_t seed, int64_t k, int unroll, uint32_t* out, void* stream) {
    if (!out || k < 1 || unroll < 1 || unroll > UMAX) return -1;
    hipLaunchKernelGGL(k_roof_philox, dim3((unsigned)wrs_roof_blocks(k, unroll)), dim3(TPB), 0, (hipStream_t)stream,
                       seed, k, unroll, out);
    return (int)hipGetLastError();
}
