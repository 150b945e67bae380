// wrs_device.h -- device helpers shared by the HIP kernels.
#pragma once
#include "wrs_internal.h"

namespace wrs {

// ---------------------------------------------------------------------------
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies with the published multipliers, the key bumped by the published
// Weyl increments between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit product each (a single v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// ---------------------------------------------------------------------------
// Exact grid arithmetic.  A weight w is represented by q = w / 2^G rounded to an
// integer (exact when w's last mantissa bit weighs at least 2^G).
// ---------------------------------------------------------------------------
__device__ __forceinline__ u128 quantize(float w, int G) {
    const uint32_t bits = __float_as_uint(w);
    const uint32_t e = bits >> 23;              // w >= 0: no sign bit
    uint32_t m = bits & 0x7FFFFFu;
    if (e) m |= 0x800000u;
    const int s = (int)(e ? e : 1u) - 150 - G;  // w = m * 2^(s + G)
    if (s > 103) return ~(u128)0;               // far above any weight <= W: saturate
    if (s >= 0) return (u128)m << s;
    if (s <= -32) return 0;
    const int sh = -s;
    const uint32_t r = m >> sh;
    const uint32_t rem = m & ((1u << sh) - 1u);
    const uint32_t half = 1u << (sh - 1);
    return (u128)(r + ((rem > half) || (rem == half && (r & 1u))));
}

// n * quantize(w, G), exactly: (n m) 2^s with one 32x32 product when the
// weight lies on the grid (s >= 0), else n times the rounded q.
__device__ __forceinline__ u128 nscaled(float w, int G, uint32_t n) {
    const uint32_t bits = __float_as_uint(w);
    const uint32_t e = bits >> 23;
    uint32_t m = bits & 0x7FFFFFu;
    if (e) m |= 0x800000u;
    const int s = (int)(e ? e : 1u) - 150 - G;
    if (s > 72) return ~(u128)0;  // only for weights far above W (never for valid input)
    if (s >= 0) return (u128)((uint64_t)m * n) << s;
    return (u128)((uint64_t)quantize(w, G) * n);
}

__device__ __forceinline__ double u128_to_double(u128 v) {
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    return (double)hi * 18446744073709551616.0 + (double)lo;
}

__device__ __forceinline__ u128 shfl_up_u128(u128 v, int d) {
    const uint64_t lo = __shfl_up((unsigned long long)(uint64_t)v, d, 64);
    const uint64_t hi = __shfl_up((unsigned long long)(uint64_t)(v >> 64), d, 64);
    return ((u128)hi << 64) | lo;
}

__device__ __forceinline__ u128 shfl_u128(u128 v, int src) {
    const uint64_t lo = __shfl((unsigned long long)(uint64_t)v, src, 64);
    const uint64_t hi = __shfl((unsigned long long)(uint64_t)(v >> 64), src, 64);
    return ((u128)hi << 64) | lo;
}

// ---------------------------------------------------------------------------
// Double-double helpers (TwoSum accumulation), used for the total weight only.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dd_acc(double& hi, double& lo, double x) {
    const double s = hi + x;
    const double bp = s - hi;
    const double err = (hi - (s - bp)) + (x - bp);
    hi = s;
    lo += err;
}

__device__ __forceinline__ void dd_add(double& ah, double& al, double bh, double bl) {
    const double s = ah + bh;
    const double bp = s - ah;
    double e = (ah - (s - bp)) + (bh - bp);
    e += al + bl;
    const double r = s + e;
    al = e - (r - s);
    ah = r;
}

// ---------------------------------------------------------------------------
// Block-wide (TPB = 256 threads, 4 waves of 64) exclusive scans.
// ---------------------------------------------------------------------------
struct ScanTmp {
    u128 a[TPB / 64];
    u128 b[TPB / 64];
    uint32_t c[TPB / 64];
};

// Exclusive scan of (cnt, a, b) over the block; returns prefixes and totals.
__device__ __forceinline__ void block_scan3(uint32_t cnt, u128 a, u128 b, uint32_t& cnt_ex, u128& a_ex,
                                            u128& b_ex, uint32_t& cnt_tot, u128& a_tot, u128& b_tot,
                                            ScanTmp& tmp) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    uint32_t ci = cnt;
    u128 ai = a, bi = b;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t cu = __shfl_up(ci, d, 64);
        const u128 au = shfl_up_u128(ai, d);
        const u128 bu = shfl_up_u128(bi, d);
        if (lane >= d) {
            ci += cu;
            ai += au;
            bi += bu;
        }
    }
    if (lane == 63) {
        tmp.c[wv] = ci;
        tmp.a[wv] = ai;
        tmp.b[wv] = bi;
    }
    __syncthreads();
    uint32_t cp = 0;
    u128 ap = 0, bp = 0;
    for (int k = 0; k < wv; ++k) {
        cp += tmp.c[k];
        ap += tmp.a[k];
        bp += tmp.b[k];
    }
    cnt_tot = 0;
    a_tot = 0;
    b_tot = 0;
    for (int k = 0; k < TPB / 64; ++k) {
        cnt_tot += tmp.c[k];
        a_tot += tmp.a[k];
        b_tot += tmp.b[k];
    }
    cnt_ex = cp + ci - cnt;
    a_ex = ap + ai - a;
    b_ex = bp + bi - b;
    __syncthreads();
}

// Locate the job and the block index within the job for the current block.
__device__ __forceinline__ const JobDesc& job_of_block(const JobTable& jt, int64_t& lb, int* s_job) {
    if (jt.jobs == nullptr) {
        lb = blockIdx.x;
        return jt.one;
    }
    const int64_t* off = jt.off + (int64_t)jt.phase * (jt.njobs + 1);
    const int64_t b = blockIdx.x;
    if (threadIdx.x == 0) {
        int lo = 0, hi = jt.njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= b) lo = mid; else hi = mid - 1;
        }
        *s_job = lo;
    }
    __syncthreads();
    const int j = *s_job;
    lb = b - off[j];
    return jt.jobs[j];
}

}  // namespace wrs
