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

// A weight with its sign bit cleared: -0 (which the domain check accepts, as
// -0 >= 0) becomes +0, the only form the bit-pattern arithmetic below expects.
__device__ __forceinline__ float canonical_weight(float w) { return __uint_as_float(__float_as_uint(w) & 0x7FFFFFFFu); }

// Exponent of w on the grid: w = m 2^s (s < 0: below the grid).
__device__ __forceinline__ int grid_shift(float w, int G) {
    const uint32_t e = __float_as_uint(w) >> 23;
    return (int)max(e, 1u) - 150 - G;
}

// quantize() for a weight on the grid (0 <= s <= 103), without branches:
// m 2^s with m < 2^24 is two 64-bit shifts.
__device__ __forceinline__ u128 quantize_on_grid(float w, int G) {
    const uint32_t bits = __float_as_uint(w);
    const uint32_t e = bits >> 23;
    const uint64_t m = (bits & 0x7FFFFFu) | (e ? 0x800000u : 0u);
    const int s = min((int)max(e, 1u) - 150 - G, 103);
    const uint64_t t = m << (s & 63);          // low word (s < 64) or high word (s >= 64)
    const uint64_t c = m >> ((64 - s) & 63);  // bits carried into the high word, s in [1, 63]
    const uint64_t lo = s < 64 ? t : 0ull;
    const uint64_t hi = s < 64 ? (s == 0 ? 0ull : c) : t;
    return ((u128)hi << 64) | lo;
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
// Wave-wide (64 lanes) inclusive prefix sums in registers: DPP row shifts by
// 1, 2, 4, 8 inside each row of 16 lanes, then the row broadcasts of lanes 15
// and 31 carry the row totals forward.  A lane whose source lies outside its
// row, or whose row is masked off, adds 0.
// ---------------------------------------------------------------------------
// (BC: a row shift's source outside the row reads 0 by bound control, with no
// identity in the destination first.)
template <int CTRL, int ROW_MASK, bool BC = false>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v, uint32_t identity = 0) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, ROW_MASK, 0xf, BC);
}
template <int CTRL, int ROW_MASK, bool BC = false>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    const uint32_t lo = dpp_u32<CTRL, ROW_MASK, BC>((uint32_t)v);
    const uint32_t hi = dpp_u32<CTRL, ROW_MASK, BC>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
constexpr int DPP_ROW_SHR = 0x110, DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += dpp_u32<DPP_ROW_SHR + 1, 0xf>(x);
    x += dpp_u32<DPP_ROW_SHR + 2, 0xf>(x);
    x += dpp_u32<DPP_ROW_SHR + 4, 0xf>(x);
    x += dpp_u32<DPP_ROW_SHR + 8, 0xf>(x);
    x += dpp_u32<DPP_ROW_BCAST15, 0xa>(x);
    x += dpp_u32<DPP_ROW_BCAST31, 0xc>(x);
    return x;
}

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x) {
    x += dpp_u64<DPP_ROW_SHR + 1, 0xf, true>(x);
    x += dpp_u64<DPP_ROW_SHR + 2, 0xf, true>(x);
    x += dpp_u64<DPP_ROW_SHR + 4, 0xf, true>(x);
    x += dpp_u64<DPP_ROW_SHR + 8, 0xf, true>(x);
    x += dpp_u64<DPP_ROW_BCAST15, 0xa>(x);
    x += dpp_u64<DPP_ROW_BCAST31, 0xc>(x);
    return x;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ u128 dpp_u128(u128 v) {
    const uint64_t lo = dpp_u64<CTRL, ROW_MASK>((uint64_t)v);
    const uint64_t hi = dpp_u64<CTRL, ROW_MASK>((uint64_t)(v >> 64));
    return ((u128)hi << 64) | lo;
}

__device__ __forceinline__ u128 wave_incl_scan(u128 x) {
    x += dpp_u128<DPP_ROW_SHR + 1, 0xf>(x);
    x += dpp_u128<DPP_ROW_SHR + 2, 0xf>(x);
    x += dpp_u128<DPP_ROW_SHR + 4, 0xf>(x);
    x += dpp_u128<DPP_ROW_SHR + 8, 0xf>(x);
    x += dpp_u128<DPP_ROW_BCAST15, 0xa>(x);
    x += dpp_u128<DPP_ROW_BCAST31, 0xc>(x);
    return x;
}

// Running minimum over lanes 0..lane (signed).
__device__ __forceinline__ int32_t wave_incl_min(int32_t x) {
    constexpr uint32_t I = 0x7fffffffu;
    x = min(x, (int32_t)dpp_u32<DPP_ROW_SHR + 1, 0xf>((uint32_t)x, I));
    x = min(x, (int32_t)dpp_u32<DPP_ROW_SHR + 2, 0xf>((uint32_t)x, I));
    x = min(x, (int32_t)dpp_u32<DPP_ROW_SHR + 4, 0xf>((uint32_t)x, I));
    x = min(x, (int32_t)dpp_u32<DPP_ROW_SHR + 8, 0xf>((uint32_t)x, I));
    x = min(x, (int32_t)dpp_u32<DPP_ROW_BCAST15, 0xa>((uint32_t)x, I));
    x = min(x, (int32_t)dpp_u32<DPP_ROW_BCAST31, 0xc>((uint32_t)x, I));
    return x;
}

// Value of lane 63 (the wave total after an inclusive scan), to every lane.
__device__ __forceinline__ uint32_t lane63(uint32_t v) { return __builtin_amdgcn_readlane(v, 63); }
__device__ __forceinline__ uint64_t lane63(uint64_t v) {
    return ((uint64_t)lane63((uint32_t)(v >> 32)) << 32) | lane63((uint32_t)v);
}
__device__ __forceinline__ u128 lane63(u128 v) {
    return ((u128)lane63((uint64_t)(v >> 64)) << 64) | lane63((uint64_t)v);
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

// Global-memory view of a pointer.  Pointers read from a job descriptor are
// generic to the compiler, and generic (flat) accesses count against the LDS
// wait counter too, so every LDS wait after one would also wait for it; the
// hot kernels access device memory through this view instead.
#define WRS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ WRS_GLOBAL T* glb(T* p) {
    return (WRS_GLOBAL T*)p;
}
// Plain clang vectors: HIP's float4 / uint2 classes cannot be read or written
// through an address-space-qualified pointer.
typedef float vfloat4 __attribute__((ext_vector_type(4)));
typedef uint32_t vuint2 __attribute__((ext_vector_type(2)));
typedef uint32_t vuint4 __attribute__((ext_vector_type(4)));

// Values that every lane holds alike, moved to scalar registers.  The job
// descriptor and the build scalars are read once per block this way; left in
// vector registers they are reloaded per lane inside loops, and each reload's
// wait also waits for every load in flight (the tile prefetches included).
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int32_t uni(int32_t v) { return (int32_t)uni((uint32_t)v); }
__device__ __forceinline__ uint64_t uni(uint64_t v) {
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
__device__ __forceinline__ int64_t uni(int64_t v) { return (int64_t)uni((uint64_t)v); }
__device__ __forceinline__ double uni(double v) {
    return __longlong_as_double((long long)uni((uint64_t)__double_as_longlong(v)));
}
__device__ __forceinline__ u128 uni(u128 v) { return ((u128)uni((uint64_t)(v >> 64)) << 64) | uni((uint64_t)v); }
template <class T>
__device__ __forceinline__ T* uni(T* p) {
    return (T*)uni((uint64_t)(uintptr_t)p);
}

// Every field is copied: a field added to JobDesc or BuildScalars must be
// added here too (the size checks catch a forgotten one).
static_assert(sizeof(JobDesc) == 256, "job_uniform copies every JobDesc field");
static_assert(sizeof(BuildScalars) == 128, "scalars_uniform copies every BuildScalars field");

__device__ __forceinline__ JobDesc job_uniform(const JobDesc& J) {
    JobDesc u;
    u.w = uni(J.w);
    u.table = uni(J.table);
    u.out = uni(J.out);
    u.n = uni(J.n);
    u.k = uni(J.k);
    u.seed = uni(J.seed);
    u.first_counter = uni(J.first_counter);
    u.stream_id = uni(J.stream_id);
    u.ntiles = uni(J.ntiles);
    u.nred = uni(J.nred);
    u.nseg = uni(J.nseg);
    u.sc = uni(J.sc);
    u.red = uni(J.red);
    u.redinfo = uni(J.redinfo);
    u.NL = uni(J.NL);
    u.DP = uni(J.DP);
    u.EP = uni(J.EP);
    u.DP64 = uni(J.DP64);
    u.EP64 = uni(J.EP64);
    u.FH = uni(J.FH);
    u.WP = uni(J.WP);
    u.PO = uni(J.PO);
    u.pstart = uni(J.pstart);
    u.npack = uni(J.npack);
    u.psteps = uni(J.psteps);
    u.sunroll = uni(J.sunroll);
    u.sNL = uni(J.sNL);
    u.sDP = uni(J.sDP);
    u.sEP = uni(J.sEP);
    u.sFH = uni(J.sFH);
    u.lidx = uni(J.lidx);
    u.lres = uni(J.lres);
    u.lresf = uni(J.lresf);
    u.PI = uni(J.PI);
    u.nmul = uni(J.nmul);
    u.pad = 0;
    return u;
}

__device__ __forceinline__ BuildScalars scalars_uniform(const BuildScalars* p) {
    BuildScalars u;
    u.status = uni(p->status);
    u.G = uni(p->G);
    u.pad[0] = u.pad[1] = 0;
    u.Q = uni(p->Q);
    u.W_hi = uni(p->W_hi);
    u.W_lo = uni(p->W_lo);
    u.Qd = uni(p->Qd);
    u.rQ = uni(p->rQ);
    u.nscale = uni(p->nscale);
    u.Qn = uni(p->Qn);
    u.npos = uni(p->npos);
    u.kshift = uni(p->kshift);
    u.wthr = uni(p->wthr);
    u.tscale = uni(p->tscale);
    u.Qk = uni(p->Qk);
    u.nleft = uni(p->nleft);
    return u;
}

// Workgroups are dispatched to the 8 XCDs round robin (block b to XCD b mod 8),
// each XCD with its own L2.  This bijection gives each XCD a contiguous run of
// block indices, in dispatch order, so neighbouring work shares an L2.
__device__ __forceinline__ int64_t xcd_contiguous_block() {
    const int64_t b = blockIdx.x, g = gridDim.x;
    const int64_t q = g >> 3, r = g & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// Locate the job and the block index within the job for block b of the grid.
__device__ __forceinline__ const JobDesc& job_of_block(const JobTable& jt, int64_t& lb, int* s_job,
                                                       int64_t b = blockIdx.x) {
    if (jt.jobs == nullptr) {
        lb = b;
        return jt.one;
    }
    const int64_t* off = jt.off + (int64_t)jt.phase * (jt.njobs + 1);
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

// ---------------------------------------------------------------------------
// Merge helpers of the table construction (tile merge and greedy blocks).
// ---------------------------------------------------------------------------
static constexpr int32_t FH_NONE = 0x7fffffff;

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// n q(w) / 2^kshift rounded to nearest (ties up): the item's size in key
// units.  On the grid (s >= 0) n q = (n m) 2^s exactly; below it q is rounded
// first.  The result is below 2^62 for every weight <= W.
__device__ __forceinline__ uint64_t size_keyunits_any(float w, const BuildScalars& sc, uint32_t n);

// size_keyunits for every lane of a wave: the common case (a zero weight, or
// a weight on the grid whose size needs a right shift of 1 to 63 bits: every
// weight within a factor of about 2^17 above and 2^40 below the mean) in a
// few instructions; a wave with any other lane takes the general function.
__device__ __forceinline__ uint64_t size_keyunits(float w, const BuildScalars& sc, uint32_t n) {
    const uint32_t bits = __float_as_uint(w);
    const uint32_t e = bits >> 23;
    const uint32_t m = (bits & 0x7FFFFFu) | 0x800000u;
    const int r = sc.kshift - ((int)e - 150 - sc.G);  // right shift of n m (e >= 1)
    const bool zero = bits == 0u;
    const bool common = zero || (e != 0u && r >= 1 && r <= 63);
    if (__builtin_expect(__ballot(!common) == 0, 1)) {
        const uint64_t x = (uint64_t)m * n;
        const uint64_t z = (x + (1ull << ((r - 1) & 63))) >> (r & 63);
        return zero ? 0ull : z;
    }
    return size_keyunits_any(w, sc, n);
}

__device__ __forceinline__ uint64_t size_keyunits_any(float w, const BuildScalars& sc, uint32_t n) {
    const uint32_t bits = __float_as_uint(w);
    const uint32_t e = bits >> 23;
    const uint32_t m = (bits & 0x7FFFFFu) | (e ? 0x800000u : 0u);
    const int s = (int)max(e, 1u) - 150 - sc.G;
    uint64_t x = (uint64_t)m * n;  // < 2^55
    int r = sc.kshift - s;         // right shift
    if (s < 0) {
        x = (uint64_t)quantize(w, sc.G) * n;
        r = sc.kshift;
    }
    const uint64_t down = (x + (1ull << ((r - 1) & 63))) >> (r & 63);  // r in [1, 63]: no overflow
    const uint64_t up = x << (r <= 0 ? min(-r, 63) : 0);
    return r <= 0 ? up : (r >= 64 ? 0ull : down);
}

// First position p in [from, to) with !(key[p] < v) (keys non-decreasing): a
// 64-ary search by one wave, two rounds for a tile.
template <bool LE>
__device__ __forceinline__ int wave_search(const uint64_t* key, int from, int to, uint64_t v) {
    const int lane = threadIdx.x & 63;
    int lo = from, hi = to;  // answer in [lo, hi]
    while (lo < hi) {
        const int step = (hi - lo + 63) >> 6;
        const int p = lo + lane * step;
        const bool pr = (p < hi) && (LE ? (key[p] <= v) : (key[p] < v));
        const uint64_t mask = __ballot(pr);
        const int K = __popcll(mask);
        if (K == 0) {
            hi = lo;
        } else {
            const int pk1 = lo + (K - 1) * step;
            const int nhi = min(hi, pk1 + step);
            lo = pk1 + 1;
            hi = nhi;
        }
    }
    return lo;
}

__device__ __forceinline__ void store_entry(wrs_entry* table, int64_t item, float t, int32_t alias) {
    vuint2 v;
    v.x = __float_as_uint(t);
    v.y = (uint32_t)alias;
    *(WRS_GLOBAL vuint2*)(table + item) = v;
}

// A light's bucket keeps t = n w / W; lscale = n 2^-G / Q.
__device__ __forceinline__ float light_t(float w, double lscale) { return (float)((double)w * lscale); }

// A heavy's bucket keeps t = 1 + (E - D) / W, from a key difference.
__device__ __forceinline__ float heavy_t(uint64_t E, uint64_t D, double tscale) {
    const float t = (float)fma((double)(int64_t)(E - D), tscale, 1.0);
    return fminf(fmaxf(t, 0.0f), 1.0f);
}

// ---------------------------------------------------------------------------
// Exponential clocks (Section 2.3): the variate -ln(u) of item i, u from the
// Philox counter (i, stream id, 1).  Shared by sampling without replacement
// and the weighted permutation, so both order items by the same keys.
// ---------------------------------------------------------------------------
// -ln(u) for u = (x0 + 1) 2^-32, accurate near u = 1 through log1p.
__device__ __forceinline__ double neg_log_u(uint32_t x0) {
    if (x0 >= 0x7FFFFFFFu) {  // u >= 1/2
        const double d = (double)(0xFFFFFFFFu - x0) * (1.0 / 4294967296.0);  // 1 - u, exact
        return -log1p(-d);
    }
    return -log(((double)x0 + 1.0) * (1.0 / 4294967296.0));
}

}  // namespace wrs
