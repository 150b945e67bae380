// wrs_os.hip -- output-sensitive sampling with replacement (Section 5).
//
// A sample of k draws is returned as the s distinct items drawn and their
// multiplicities; expected work O(s + log n) (Section 5).
//
// Structure (built once, resident like an alias table):
//   - items with w > 0 in groups of weights within a factor of two: the group
//     of w is its binary exponent e, w = M 2^(e-23) with integer M in
//     [2^23, 2^24); groups heaviest first, items of a group by index.  The
//     order comes from stable radix passes over the key (127 - e) << 24 | M
//     (zero weights get key 511 << 24 and sort last): one 8-bit digit, or two
//     when a key reaches bit 32;
//   - exact prefix sums P of M over that order (u64), from which every node
//     mass inside a group, and each weight M, is a difference;
//   - the divide-and-conquer (DC) tree over the groups: heap-indexed FP64
//     masses, a leaf = the group's exact total scaled by 2^(e-23), an inner
//     node = left + right.  A node over [lo, hi) splits at floor((lo + hi)/2).
// Query: a breadth-first descent, one launch per tree level.  A node asked for
// m draws passes Binomial(m, left mass / node mass) of them to its left child
// (top-tree nodes always; group nodes when m >= 2), a group node asked for one
// draw takes it from the group's bucket table by rejection (buckets of
// capacity 2^(e+1) = 2^24 units of 2^(e-23), one item each), and a one-item
// node emits (item, m).  Every frontier node covers positive items disjoint
// from the others' and holds at least one draw, so a frontier and the output
// never exceed min(k, n).
//
// Random bits: Philox-4x32-10 keyed by the seed, one counter block per attempt
// at a node: (heap index low word, high word, tag, attempt) with tag = the
// group's position (group trees) or 0xFFFFFFFF (top tree).  Binomial variates:
// inversion (Kachitvichyanukul & Schmeiser, CACM 1988) below mean 10, else
// transformed rejection with squeeze (Hoermann, J. Statist. Comput. Simul.
// 1993).  Their logarithm, square root and log-factorial are series and
// Newton iterations in IEEE basic operations, compiled without contraction,
// so the variates do not depend on a math library.
#include <math.h>

#include "wrs_device.h"

#pragma clang fp contract(off)

namespace wrs {

constexpr uint32_t OS_TOP = 0xFFFFFFFFu;
constexpr int OS_MAX_GROUPS = 277;  // binary exponents -149..127 of positive floats
constexpr int OS_KEY_ZERO = 511;    // sort key of a zero weight (after every group)
constexpr int OS_HEAP = 2048;       // top-tree heap indices (< 2^(ceil(log2 277) + 1))
constexpr int OS_LEVELS = 42;       // >= depth of the top tree (9) + a group tree (31) + 1
constexpr int OS_TPB = 256;
constexpr int OS_SCAN_IPT = 16;
constexpr int OS_SCAN_TILE = OS_TPB * OS_SCAN_IPT;
// Attempts of one rejection loop before it reports an error (each attempt is
// accepted with probability above 1/2, so the bound only guards termination).
constexpr uint32_t OS_ATTEMPTS = 1u << 16;

struct OsHeader {
    int32_t status;
    int32_t u;   // nonempty groups
    int64_t n;
    int64_t np;  // positive items
    int32_t wide;  // some sort key needs a second digit: a zero weight, or e < -128
    int32_t pad[57];
};
static_assert(sizeof(OsHeader) == 256, "header is one 256-byte line");

struct OsGroup {
    int64_t start, count;
    int32_t e;
    int32_t pad;
};

struct OsLayout {
    OsHeader* hdr;
    OsGroup* groups;
    double* V;    // top-tree masses by heap index
    uint32_t* A;  // item at each position
    uint64_t* P;  // P[j] = M[0] + ... + M[j-1], j <= n, M[j] = the integer weight at position j
};

static inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct OsOffsets {
    size_t groups, V, A, P, total;
};

static OsOffsets os_offsets(int64_t n) {
    OsOffsets o;
    size_t p = sizeof(OsHeader);
    o.groups = p; p = a256(p + sizeof(OsGroup) * OS_MAX_GROUPS);
    o.V = p;      p = a256(p + sizeof(double) * OS_HEAP);
    o.A = p;      p = a256(p + sizeof(uint32_t) * n);
    o.P = p;      p = a256(p + sizeof(uint64_t) * (n + 1));
    o.total = p;
    return o;
}

size_t os_bytes(int64_t n) { return os_offsets(n).total; }

static OsLayout os_layout(const void* os, int64_t n) {
    const OsOffsets o = os_offsets(n);
    char* b = (char*)os;
    OsLayout L;
    L.hdr = (OsHeader*)b;
    L.groups = (OsGroup*)(b + o.groups);
    L.V = (double*)(b + o.V);
    L.A = (uint32_t*)(b + o.A);
    L.P = (uint64_t*)(b + o.P);
    return L;
}

// Build workspace: the radix buffers, then the block sums of the prefix sums.
static size_t os_bsum_offset(int64_t n) { return a256(perm_ws_bytes(n)); }
static size_t os_build_ws_bytes(int64_t n) {
    return os_bsum_offset(n) + a256(sizeof(uint64_t) * (cdiv(n, OS_SCAN_TILE) + 1));
}

// Sample workspace: status, level counters, output count, two frontiers.
struct OsNode {
    uint64_t h;
    uint32_t lo, hi, m, tag;
};
static_assert(sizeof(OsNode) == 24, "frontier node");

struct OsSampleHdr {
    int32_t status;
    int32_t pad0;
    uint64_t nres;
    uint32_t cnt[64];  // nodes of each level
    int32_t pad[60];
};
static_assert(sizeof(OsSampleHdr) == 512, "sample header");

static int64_t os_cap(int64_t n, int64_t k) { return std::max<int64_t>(1, std::min(n, k)); }

static size_t os_sample_ws_bytes(int64_t n, int64_t k) {
    return sizeof(OsSampleHdr) + 2 * a256(sizeof(OsNode) * os_cap(n, k));
}

size_t os_ws_bytes(int64_t n, int64_t k) { return std::max(os_build_ws_bytes(n), os_sample_ws_bytes(n, k)); }

// ---------------------------------------------------------------------------
// Elementary functions and binomial variates from IEEE basic operations.
// ---------------------------------------------------------------------------
__device__ double os_u53(uint32_t lo, uint32_t hi) {
    return (double)((((uint64_t)hi << 32) | lo) >> 11) * 0x1p-53;
}

__device__ double os_dbl(uint64_t x) { return (double)(uint32_t)(x >> 32) * 4294967296.0 + (double)(uint32_t)x; }

// ln x = E ln 2 + 2 atanh(s), s = (f - 1)/(f + 1), f in [sqrt(1/2), sqrt(2)):
// 2 s (1 + z/3 + ... + z^13/27), z = s^2, in Horner form.
__device__ double os_log(double x) {
    if (x == 0.0) return -INFINITY;
    int E = 0;
    double f = frexp(x, &E);
    if (f < 0.7071067811865476) {
        f = f * 2.0;
        E = E - 1;
    }
    const double s = (f - 1.0) / (f + 1.0);
    const double z = s * s;
    double t = 1.0 / 27.0;
    for (int j = 12; j >= 0; --j) t = t * z + 1.0 / (double)(2 * j + 1);
    return (double)E * 0.6931471805599453 + (2.0 * s) * t;
}

// sqrt x, x > 0: eight Newton steps from 2^floor(E/2).
__device__ double os_sqrt(double x) {
    int E = 0;
    (void)frexp(x, &E);
    const int e2 = (E - (E & 1)) / 2;
    double y = ldexp(1.0, e2);
    for (int i = 0; i < 8; ++i) y = 0.5 * (y + x / y);
    return y;
}

// ln(j!): summed logarithms below 10, else Stirling's series with three terms.
__device__ double os_lfact(double j) {
    if (j < 10.0) {
        double r = 0.0;
        for (int i = 2; i <= (int)j; ++i) r += os_log((double)i);
        return r;
    }
    const double x = j + 1.0;
    const double x2 = x * x;
    const double tail = (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0) / x2) / x2) / x;
    return (j + 0.5) * os_log(x) - x + 0.9189385332046728 + tail;
}

__device__ uint4 os_block(uint64_t seed, uint64_t heap, uint32_t tag, uint32_t attempt) {
    return philox4x32_10(make_uint4((uint32_t)heap, (uint32_t)(heap >> 32), tag, attempt), (uint32_t)seed,
                         (uint32_t)(seed >> 32));
}

__device__ int64_t os_binv(int64_t m, double p, uint64_t seed, uint64_t heap, uint32_t tag, bool& fail) {
    const double q = 1.0 - p;
    const double s = p / q;
    const double a = (double)(m + 1) * s;
    double r0 = 1.0, b = q;
    for (int64_t e = m; e > 0;) {
        if (e & 1) r0 = r0 * b;
        e >>= 1;
        if (e) b = b * b;
    }
    for (uint32_t t = 0; t < OS_ATTEMPTS; ++t) {
        const uint4 x = os_block(seed, heap, tag, t);
        double u = os_u53(x.x, x.y);
        double r = r0;
        int64_t j = 0;
        for (;;) {
            if (u < r) return j;
            u = u - r;
            if (j >= m || j >= 110) break;
            j = j + 1;
            r = r * (a / (double)j - s);
        }
    }
    fail = true;
    return 0;
}

__device__ int64_t os_btrs(int64_t m, double p, uint64_t seed, uint64_t heap, uint32_t tag, bool& fail) {
    const double q = 1.0 - p;
    const double mp = (double)m * p;
    const double spq = os_sqrt(mp * q);
    const double b = 1.15 + 2.53 * spq;
    const double a = -0.0873 + 0.0248 * b + 0.01 * p;
    const double c = mp + 0.5;
    const double vr = 0.92 - 4.2 / b;
    const double alpha = (2.83 + 5.1 / b) * spq;
    const double lpq = os_log(p / q);
    const double mode = floor((double)(m + 1) * p);
    const double h = os_lfact(mode) + os_lfact((double)m - mode);
    for (uint32_t t = 0; t < OS_ATTEMPTS; ++t) {
        const uint4 x = os_block(seed, heap, tag, t);
        const double u = os_u53(x.x, x.y) - 0.5;
        double v = os_u53(x.z, x.w);
        const double us = 0.5 - fabs(u);
        const double kd = floor((2.0 * a / us + b) * u + c);
        if (!(kd >= 0.0 && kd <= (double)m)) continue;
        if (us >= 0.07 && v <= vr) return (int64_t)kd;
        v = v * alpha / (a / (us * us) + b);
        const double bound = h - os_lfact(kd) - os_lfact((double)m - kd) + (kd - mode) * lpq;
        if (os_log(v) <= bound) return (int64_t)kd;
    }
    fail = true;
    return 0;
}

__device__ int64_t os_binomial(int64_t m, double rho, uint64_t seed, uint64_t heap, uint32_t tag, bool& fail) {
    if (m == 0 || rho <= 0.0) return 0;
    if (rho >= 1.0) return m;
    const bool flip = rho > 0.5;
    const double p = flip ? 1.0 - rho : rho;
    const int64_t k = ((double)m * p < 10.0) ? os_binv(m, p, seed, heap, tag, fail)
                                             : os_btrs(m, p, seed, heap, tag, fail);
    return flip ? m - k : k;
}

// ---------------------------------------------------------------------------
// Build.
// ---------------------------------------------------------------------------
__global__ void k_os_init(OsHeader* hdr, int64_t n) {
    if (threadIdx.x == 0) {
        hdr->status = WRS_OK;
        hdr->u = 0;
        hdr->n = n;
        hdr->np = 0;
        hdr->wide = 0;
    }
}

// Sort key (127 - e) << 24 | M of each item, value = the item; domain check;
// one flag per wave if a key has bit 32 set (the sort then needs two digits).
__global__ __launch_bounds__(OS_TPB) void k_os_keys(const float* __restrict__ w, int64_t n, uint64_t* keys,
                                                     uint32_t* vals, OsHeader* hdr) {
    const int64_t i = (int64_t)blockIdx.x * OS_TPB + threadIdx.x;
    if (i >= n) return;
    const float x = w[i];
    const uint32_t bits = __float_as_uint(x);
    const bool bad = !(x >= 0.0f) || isinf(x);
    if (bad) hdr->status = WRS_EDOMAIN;
    uint64_t key = (uint64_t)OS_KEY_ZERO << 24;
    if (!bad && x > 0.0f) {
        const uint32_t E = (bits >> 23) & 0xFFu, F = bits & 0x7FFFFFu;
        int32_t e;
        uint32_t M;
        if (E > 0) {
            e = (int32_t)E - 127;
            M = F | 0x800000u;
        } else {
            const int bl = 32 - __clz((int)F);  // bit length of the subnormal's significand
            e = bl - 150;
            M = F << (24 - bl);
        }
        key = ((uint64_t)(127 - e) << 24) | M;
    }
    keys[i] = key;
    vals[i] = (uint32_t)i;
    const uint64_t wide = __ballot((key >> 32) != 0);
    if (wide && (threadIdx.x & 63) == __ffsll((unsigned long long)wide) - 1) atomicOr(&hdr->wide, 1);
}

__device__ uint64_t os_block_sum(uint64_t v, uint64_t* s_w) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) s_w[wv] = v;
    __syncthreads();
    uint64_t t = 0;
    for (int k = 0; k < OS_TPB / 64; ++k) t += s_w[k];
    return t;
}

// Sum of M over each tile of OS_SCAN_TILE sorted positions.
__global__ __launch_bounds__(OS_TPB) void k_os_bsum(const uint64_t* __restrict__ keys, int64_t n, uint64_t* bsum) {
    __shared__ uint64_t s_w[OS_TPB / 64];
    const int64_t base = (int64_t)blockIdx.x * OS_SCAN_TILE;
    uint64_t v = 0;
    for (int e = 0; e < OS_SCAN_IPT; ++e) {
        const int64_t j = base + (int64_t)e * OS_TPB + threadIdx.x;
        if (j < n) v += keys[j] & 0xFFFFFFu;
    }
    const uint64_t t = os_block_sum(v, s_w);
    if (threadIdx.x == 0) bsum[blockIdx.x] = t;
}

// Exclusive prefix of the nb tile sums in place; bsum[nb] = the total.
__global__ __launch_bounds__(1024) void k_os_bscan(uint64_t* bsum, int64_t nb) {
    __shared__ uint64_t s[1024];
    const int64_t per = cdiv(nb, (int64_t)1024);
    const int64_t b0 = (int64_t)threadIdx.x * per;
    const int64_t b1 = min(nb, b0 + per);
    uint64_t sum = 0;
    for (int64_t b = b0; b < b1; ++b) sum += bsum[b];
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // Hillis-Steele inclusive scan
        const uint64_t add = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    uint64_t run = s[threadIdx.x] - sum;
    for (int64_t b = b0; b < b1; ++b) {
        const uint64_t x = bsum[b];
        bsum[b] = run;
        run += x;
    }
    if (threadIdx.x == 1023) bsum[nb] = s[1023];
}

// Positions of each tile: A and the exclusive prefix P.
__global__ __launch_bounds__(OS_TPB) void k_os_apply(const uint64_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals, int64_t n,
                                                      const uint64_t* __restrict__ bsum, OsLayout L, int64_t nb) {
    __shared__ uint32_t s_m[OS_SCAN_TILE];
    __shared__ uint64_t s_p[OS_SCAN_TILE];
    __shared__ uint64_t s_t[OS_TPB];
    const int64_t base = (int64_t)blockIdx.x * OS_SCAN_TILE;
    for (int e = 0; e < OS_SCAN_IPT; ++e) {  // coalesced: A and the staged weights
        const int r = e * OS_TPB + (int)threadIdx.x;
        const int64_t j = base + r;
        uint32_t m = 0;
        if (j < n) {
            m = (uint32_t)(keys[j] & 0xFFFFFFu);
            L.A[j] = vals[j];
        }
        s_m[r] = m;
    }
    __syncthreads();
    // each thread: OS_SCAN_IPT consecutive positions
    const int r0 = (int)threadIdx.x * OS_SCAN_IPT;
    uint64_t sum = 0;
    for (int e = 0; e < OS_SCAN_IPT; ++e) sum += s_m[r0 + e];
    s_t[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < OS_TPB; o <<= 1) {
        const uint64_t add = threadIdx.x >= (unsigned)o ? s_t[threadIdx.x - o] : 0;
        __syncthreads();
        s_t[threadIdx.x] += add;
        __syncthreads();
    }
    uint64_t run = bsum[blockIdx.x] + s_t[threadIdx.x] - sum;
    for (int e = 0; e < OS_SCAN_IPT; ++e) {
        s_p[r0 + e] = run;
        run += s_m[r0 + e];
    }
    __syncthreads();
    for (int e = 0; e < OS_SCAN_IPT; ++e) {
        const int r = e * OS_TPB + (int)threadIdx.x;
        const int64_t j = base + r;
        if (j < n) L.P[j] = s_p[r];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) L.P[n] = bsum[nb];
}

__device__ int64_t os_lower_bound(const uint64_t* keys, int64_t n, uint64_t d) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if ((keys[mid] >> 24) < d) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Group table and the top tree's masses (one block).
__global__ __launch_bounds__(512) void k_os_groups(const uint64_t* __restrict__ keys, int64_t n, OsLayout L) {
    __shared__ int64_t s_start[OS_MAX_GROUPS + 1];
    __shared__ int32_t s_lo[OS_HEAP], s_hi[OS_HEAP];
    for (int d = threadIdx.x; d <= OS_MAX_GROUPS; d += 512) s_start[d] = os_lower_bound(keys, n, (uint64_t)d);
    for (int h = threadIdx.x; h < OS_HEAP; h += 512) s_lo[h] = s_hi[h] = -1;
    __syncthreads();
    if (threadIdx.x != 0) return;
    OsHeader* H = L.hdr;
    int32_t u = 0;
    for (int d = 0; d < OS_MAX_GROUPS; ++d) {
        const int64_t c = s_start[d + 1] - s_start[d];
        if (c > 0) {
            OsGroup g;
            g.start = s_start[d];
            g.count = c;
            g.e = 127 - d;
            g.pad = 0;
            L.groups[u++] = g;
        }
    }
    H->u = u;
    H->np = s_start[OS_MAX_GROUPS];
    if (H->status != WRS_OK) return;
    if (u == 0) {
        H->status = WRS_EDOMAIN;  // no positive weight
        return;
    }
    // heap ranges top-down, masses bottom-up (children have larger indices)
    s_lo[1] = 0;
    s_hi[1] = u;
    int hmax = 1;
    for (int h = 1; h < OS_HEAP / 2; ++h) {
        if (s_lo[h] < 0 || s_hi[h] - s_lo[h] < 2) continue;
        const int mid = (s_lo[h] + s_hi[h]) / 2;
        s_lo[2 * h] = s_lo[h];
        s_hi[2 * h] = mid;
        s_lo[2 * h + 1] = mid;
        s_hi[2 * h + 1] = s_hi[h];
        hmax = 2 * h + 1;
    }
    for (int h = hmax; h >= 1; --h) {
        if (s_lo[h] < 0) continue;
        if (s_hi[h] - s_lo[h] == 1) {
            const OsGroup g = L.groups[s_lo[h]];
            L.V[h] = ldexp(os_dbl(L.P[g.start + g.count] - L.P[g.start]), g.e - 23);
        } else {
            L.V[h] = L.V[2 * h] + L.V[2 * h + 1];
        }
    }
}

int launch_os_build(const float* d_w, int64_t n, void* d_os, void* d_ws, hipStream_t st) {
    const OsLayout L = os_layout(d_os, n);
    uint64_t* k0;
    uint32_t* v0;
    radix_inputs(d_ws, n, &k0, &v0);
    uint64_t* bsum = (uint64_t*)((char*)d_ws + os_bsum_offset(n));
    const int64_t nb = cdiv(n, OS_SCAN_TILE);
    hipLaunchKernelGGL(k_os_init, dim3(1), dim3(64), 0, st, L.hdr, n);
    hipLaunchKernelGGL(k_os_keys, dim3((unsigned)cdiv(n, OS_TPB)), dim3(OS_TPB), 0, st, d_w, n, k0, v0, L.hdr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    const uint64_t* K;
    const uint32_t* V;
    // One 8-bit digit (bits 24..31) orders the keys unless some key reaches
    // bit 32; the flag is read on the host to skip the second pass.
    int32_t wide = 1;
    e = hipMemcpyAsync(&wide, &L.hdr->wide, sizeof wide, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return (int)e;
    const int rc = launch_radix(d_ws, n, 24, wide ? 2 : 1, st, &K, &V);
    if (rc) return rc;
    hipLaunchKernelGGL(k_os_bsum, dim3((unsigned)nb), dim3(OS_TPB), 0, st, K, n, bsum);
    hipLaunchKernelGGL(k_os_bscan, dim3(1), dim3(1024), 0, st, bsum, nb);
    hipLaunchKernelGGL(k_os_apply, dim3((unsigned)nb), dim3(OS_TPB), 0, st, K, V, n, (const uint64_t*)bsum, L, nb);
    hipLaunchKernelGGL(k_os_groups, dim3(1), dim3(512), 0, st, K, n, L);
    e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

// ---------------------------------------------------------------------------
// Query.
// ---------------------------------------------------------------------------
struct OsQuery {
    OsSampleHdr* sh;
    OsNode* front[2];
    int32_t* items;
    int32_t* counts;
    int64_t cap;
    uint64_t seed;
};

// Reads only the header and the group table (fixed offsets), so a structure
// built for another n is refused before any n-dependent array is touched.
__global__ void k_os_qinit(OsLayout L, OsQuery Q, int64_t n, int64_t k) {
    const int t = threadIdx.x;  // 64 threads
    Q.sh->cnt[t] = 0;
    if (t != 0) return;
    Q.sh->nres = 0;
    const int32_t st = (L.hdr->n != n) ? WRS_EINVAL : L.hdr->status;
    Q.sh->status = st;
    if (st != WRS_OK || k == 0) return;
    OsNode r;
    r.h = 1;
    r.m = (uint32_t)k;
    if (L.hdr->u == 1) {
        r.tag = 0;
        r.lo = 0;
        r.hi = (uint32_t)L.groups[0].count;
    } else {
        r.tag = OS_TOP;
        r.lo = 0;
        r.hi = (uint32_t)L.hdr->u;
    }
    Q.front[0][0] = r;
    Q.sh->cnt[0] = 1;
}

// One node of a level: what it emits or pushes.
struct OsStep {
    bool emit;
    uint32_t item, m;  // emitted pair
    int npush;         // children pushed: a (if m > 0), then b (if m > 0)
    OsNode a, b;
};

__device__ OsStep os_step(const OsLayout& L, const OsQuery& Q, OsNode nd) {
    OsStep r;
    r.emit = false;
    r.npush = 0;
    if (nd.tag == OS_TOP && nd.hi - nd.lo == 1) {  // a top leaf: its group's root
        const uint32_t g = nd.lo;
        nd.tag = g;
        nd.lo = 0;
        nd.hi = (uint32_t)L.groups[g].count;
        nd.h = 1;
    }
    const uint32_t mid = nd.lo + (nd.hi - nd.lo) / 2;
    double rho;
    if (nd.tag != OS_TOP) {
        const OsGroup G = L.groups[nd.tag];
        if (nd.hi - nd.lo == 1) {
            r.emit = true;
            r.item = L.A[G.start + nd.lo];
            r.m = nd.m;
            return r;
        }
        if (nd.m == 1) {  // bucket table with rejection
            for (uint32_t t = 0; t < OS_ATTEMPTS; ++t) {
                const uint4 x = os_block(Q.seed, nd.h, nd.tag, t);
                const uint64_t u = ((uint64_t)x.y << 32) | x.x;
                const int64_t j = (int64_t)nd.lo + (int64_t)__umul64hi(u, (uint64_t)(nd.hi - nd.lo));
                if ((x.z >> 8) < L.P[G.start + j + 1] - L.P[G.start + j]) {
                    r.emit = true;
                    r.item = L.A[G.start + j];
                    r.m = 1;
                    return r;
                }
            }
            Q.sh->status = WRS_EDEVICE;
            return r;
        }
        const uint64_t l = L.P[G.start + mid] - L.P[G.start + nd.lo];
        const uint64_t t = L.P[G.start + nd.hi] - L.P[G.start + nd.lo];
        rho = os_dbl(l) / os_dbl(t);
    } else {
        rho = L.V[2 * nd.h] / L.V[nd.h];
    }
    bool fail = false;
    const int64_t ml = os_binomial((int64_t)nd.m, rho, Q.seed, nd.h, nd.tag, fail);
    if (fail) Q.sh->status = WRS_EDEVICE;
    r.a = nd;
    r.b = nd;
    r.a.h = 2 * nd.h;
    r.a.hi = mid;
    r.a.m = (uint32_t)ml;
    r.b.h = 2 * nd.h + 1;
    r.b.lo = mid;
    r.b.m = nd.m - (uint32_t)ml;
    if (r.a.m == 0) {
        r.a = r.b;
        r.npush = 1;
    } else {
        r.npush = r.b.m > 0 ? 2 : 1;
    }
    return r;
}

// Blocks of OS_LVL_TPB threads take that many consecutive nodes of a level per
// round; a round reserves the block's outputs and children with one atomic
// each (wave counts by ballot, wave offsets in LDS), so the level's counters
// see one atomic per OS_LVL_TPB nodes and a block's children stay together.
constexpr int OS_LVL_TPB = 512;
constexpr int OS_LVL_WAVES = OS_LVL_TPB / 64;

__global__ __launch_bounds__(OS_LVL_TPB) void k_os_level(OsLayout L, OsQuery Q, int level) {
    __shared__ uint32_t s_e[OS_LVL_WAVES], s_c[OS_LVL_WAVES];
    __shared__ unsigned long long s_ebase;
    __shared__ uint32_t s_cbase;
    const uint32_t nin = Q.sh->cnt[level];
    const OsNode* in = Q.front[level & 1];
    OsNode* out = Q.front[(level + 1) & 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t stride = gridDim.x * OS_LVL_TPB;
    for (uint32_t base = blockIdx.x * OS_LVL_TPB; base < nin; base += stride) {
        const uint32_t i = base + threadIdx.x;
        OsStep r;
        r.emit = false;
        r.npush = 0;
        if (i < nin) r = os_step(L, Q, in[i]);
        const uint64_t em = __ballot(r.emit);
        const uint64_t m1 = __ballot(r.npush >= 1), m2 = __ballot(r.npush == 2);
        if (lane == 0) {
            s_e[wv] = (uint32_t)__popcll(em);
            s_c[wv] = (uint32_t)(__popcll(m1) + __popcll(m2));
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t te = 0, tc = 0;
            for (int w = 0; w < OS_LVL_WAVES; ++w) {  // exclusive wave offsets
                const uint32_t e = s_e[w], c = s_c[w];
                s_e[w] = te;
                s_c[w] = tc;
                te += e;
                tc += c;
            }
            s_ebase = te ? atomicAdd((unsigned long long*)&Q.sh->nres, (unsigned long long)te) : 0ull;
            s_cbase = tc ? atomicAdd(&Q.sh->cnt[level + 1], tc) : 0u;
        }
        __syncthreads();
        if (r.emit) {
            const uint64_t pos = s_ebase + s_e[wv] + lanes_below(em);
            if (pos < (uint64_t)Q.cap) {
                Q.items[pos] = (int32_t)r.item;
                Q.counts[pos] = (int32_t)r.m;
            } else {
                Q.sh->status = WRS_EDEVICE;  // cannot happen: outputs are distinct positive items
            }
        }
        if (r.npush) {
            const uint64_t pos = (uint64_t)s_cbase + s_c[wv] + lanes_below(m1) + lanes_below(m2);
            if (pos + (uint64_t)r.npush <= (uint64_t)Q.cap) {
                out[pos] = r.a;
                if (r.npush == 2) out[pos + 1] = r.b;
            } else {
                Q.sh->status = WRS_EDEVICE;  // cannot happen: frontier nodes are disjoint
            }
        }
        __syncthreads();  // the offsets are rewritten next round
    }
}

__global__ void k_os_qend(OsQuery Q, int64_t* d_s) {
    if (Q.sh->cnt[OS_LEVELS] != 0) Q.sh->status = WRS_EDEVICE;  // deeper than any tree: cannot happen
    *d_s = (Q.sh->status == WRS_OK) ? (int64_t)Q.sh->nres : 0;
}

int launch_os_sample(const void* d_os, int64_t n, int64_t k, uint64_t seed, int32_t* d_items, int32_t* d_counts,
                     int64_t* d_s, void* d_ws, hipStream_t st) {
    const OsLayout L = os_layout(d_os, n);
    OsQuery Q;
    Q.sh = (OsSampleHdr*)d_ws;
    Q.cap = os_cap(n, k);
    const size_t fb = a256(sizeof(OsNode) * Q.cap);
    Q.front[0] = (OsNode*)((char*)d_ws + sizeof(OsSampleHdr));
    Q.front[1] = (OsNode*)((char*)d_ws + sizeof(OsSampleHdr) + fb);
    Q.items = d_items;
    Q.counts = d_counts;
    Q.seed = seed;
    hipLaunchKernelGGL(k_os_qinit, dim3(1), dim3(64), 0, st, L, Q, n, k);
    const unsigned grid = (unsigned)std::min<int64_t>(cdiv(Q.cap, OS_LVL_TPB), 4096);
    for (int level = 0; level < OS_LEVELS; ++level)
        hipLaunchKernelGGL(k_os_level, dim3(grid), dim3(OS_LVL_TPB), 0, st, L, Q, level);
    hipLaunchKernelGGL(k_os_qend, dim3(1), dim3(1), 0, st, Q, d_s);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

}  // namespace wrs
