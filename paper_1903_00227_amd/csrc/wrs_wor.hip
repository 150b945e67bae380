// wrs_wor.hip -- sampling without replacement by exponential clocks (Section 2.3).
//
// key_i = -ln(u_i) / w_i with u_i = (x_j + 1) 2^-32 from word j = i mod 4 of
// the Philox block with counter (floor(i / 4), stream_id, 1); the k smallest
// keys (ties: smaller index) are the sample.
// Keys are generated once, in one pass over the weights:
//   k_wor_tau     threshold tau with E[#{key <= tau}] ~ 1.02 k + 4 sqrt(k) + 64,
//                 from a strided subsample of the weights (Newton on the
//                 expected count sum_i 1 - exp(-w_i tau), which is concave)
//   k_wor_filter  one Philox block per four items; since -ln(u) >= 1 - u, an item with
//                 1 - u > tau w cannot have key <= tau and skips the logarithm;
//                 survivors are staged in LDS, get the exact FP64 key together
//                 (one per lane, no divergence) and are appended if <= tau.
//                 A second, predicated pass with tau = +inf runs only if fewer
//                 than k candidates were found.  Blocks reserve output slots
//                 from 64 counters (block b uses counter b mod 64), each owning
//                 its own region of the candidate arrays, so that no address
//                 takes more than a few hundred atomics; k_wor_shards turns
//                 the 64 counts into a prefix table, and later kernels address
//                 candidate c through it.
//   k_wor_hist / k_wor_find / k_wor_radix   select of the k-th smallest key over the
//                 candidates, by levels of 16384 bins until at most 8192
//                 candidates share the target bin: two levels of linear bins on
//                 the key (enough when the candidates are the threshold pass's),
//                 then radix levels on the key's FP64 bit pattern, 14 bits at a
//                 time from the top (a non-negative double's bit pattern orders
//                 like its value), which resolve any spread of keys, such as
//                 the fallback pass's, unless more than 8192 keys are equal
//                 (the radix levels run in one workgroup, k_wor_radix)
//   k_wor_gather / k_wor_final  sort that bin in LDS, take the exact k-th (key, idx)
//   k_wor_mark    set one bit per selected item in an n-bit map
//   k_wor_popc / k_wor_popscan / k_wor_compact   emit the set bits in index order
#include <math.h>

#include "wrs_device.h"

namespace wrs {

constexpr int WOR_TPB = 256;
constexpr int WOR_IPT = 8;                       // items per thread in the filter
constexpr int WOR_NB = 16384;                    // bins per select level
constexpr int WOR_NLIN = 2;                      // linear select levels
constexpr int WOR_NLEV = WOR_NLIN + 5;           // then radix levels: bit shifts 50, 36, 22, 8, 0
constexpr int WOR_SMALL = 8192;                  // final in-LDS sort capacity
constexpr int WOR_TAU_M = 4096;                  // subsample size for tau
constexpr int WOR_WPB = WOR_TPB * 16;            // bitmap words per compaction block
constexpr int WOR_CAND_TPB = 256;
constexpr int WOR_SHARDS = 64;                   // candidate counters / regions
constexpr int WOR_SHARD_STRIDE = 32;             // u64 words between counters (256 B)

struct WorScalars {
    int32_t status;          // first word of the workspace, as for the build
    uint32_t bad;
    uint32_t count;          // candidates of the tau pass
    uint32_t count2;         // candidates of the fallback pass
    double tau;
    double kkey;
    double level_lo[WOR_NLEV];
    double level_scale[WOR_NLEV];
    unsigned long long maxkey_bits;
    uint32_t prefix[2][WOR_SHARDS + 1];  // per pass: candidates in the shards before s
    int64_t k;
    int64_t rank;            // remaining 1-based rank inside the current bin
    int32_t level_bin[WOR_NLEV];
    uint64_t radix_prefix;   // radix levels: the chosen digits so far (bits above the level's shift)
    int32_t nlev;            // levels used; set when resolved
    int32_t resolved;
    uint32_t small_count;
    int32_t kidx;
    uint32_t total_bits;
};

struct WorLayout {
    size_t sc, shard, hist, small_key, small_idx, cand_key, cand_idx, bitmap, blk, total;
};

static inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// Candidate slots per shard: every item of the shard's blocks.
static inline int64_t wor_shard_cap(int64_t n) {
    const int64_t fblocks = cdiv(n, (int64_t)WOR_TPB * WOR_IPT);
    return cdiv(fblocks, (int64_t)WOR_SHARDS) * (WOR_TPB * WOR_IPT);
}

static WorLayout wor_layout(int64_t n) {
    WorLayout L;
    size_t o = 0;
    const int64_t nwords = cdiv(n, 32);
    const int64_t nblk = cdiv(nwords, WOR_WPB);
    L.sc = o;        o = a256(o + sizeof(WorScalars));
    // per pass and shard: a counter and a max-key word, WOR_SHARD_STRIDE apart
    L.shard = o;     o = a256(o + sizeof(unsigned long long) * 2 * 2 * WOR_SHARDS * WOR_SHARD_STRIDE);
    L.hist = o;      o = a256(o + sizeof(uint32_t) * WOR_NB * WOR_NLEV);
    L.small_key = o; o = a256(o + sizeof(double) * WOR_SMALL);
    L.small_idx = o; o = a256(o + sizeof(int32_t) * WOR_SMALL);
    const int64_t cap = WOR_SHARDS * wor_shard_cap(n);
    L.cand_key = o;  o = a256(o + sizeof(double) * cap);
    L.cand_idx = o;  o = a256(o + sizeof(int32_t) * cap);
    L.bitmap = o;    o = a256(o + sizeof(uint32_t) * nwords);
    L.blk = o;       o = a256(o + sizeof(uint32_t) * (nblk + 1));
    L.total = o;
    return L;
}

size_t wor_ws_bytes(int64_t n, int64_t) { return wor_layout(n).total; }
int wor_status_offset() { return (int)offsetof(WorScalars, status); }

struct WorArgs {
    const float* w;
    int64_t n;
    int64_t k;
    uint64_t seed;
    uint32_t sid;
    int32_t* out;
    WorScalars* S;
    uint32_t* hist;
    double* skey;
    int32_t* sidx;
    double* ckey;
    int32_t* cidx;
    uint32_t* bitmap;
    uint32_t* blk;
    int64_t nwords;
    unsigned long long* shard;  // [pass][counter | max key][shard * WOR_SHARD_STRIDE]
    int64_t scap;               // candidate slots per shard
};

__device__ __forceinline__ unsigned long long* shard_word(const WorArgs& A, int pass, int what, int s) {
    return A.shard + ((size_t)((pass - 1) * 2 + what) * WOR_SHARDS + s) * WOR_SHARD_STRIDE;
}

// The Philox block of items 4g .. 4g+3: item 4g + j takes word j.
__device__ __forceinline__ uint4 wor_block(const WorArgs& A, int64_t g) {
    return philox4x32_10(make_uint4((uint32_t)g, (uint32_t)((uint64_t)g >> 32), A.sid, 1u), (uint32_t)A.seed,
                         (uint32_t)(A.seed >> 32));
}


// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_wor_tau(WorArgs A) {
    __shared__ double red[32];
    WorScalars* S = A.S;
    // reset state (the whole select pipeline starts from here)
    for (int i = threadIdx.x; i < WOR_NB * WOR_NLEV; i += blockDim.x) A.hist[i] = 0;
    for (int i = threadIdx.x; i < 2 * 2 * WOR_SHARDS; i += blockDim.x) A.shard[(size_t)i * WOR_SHARD_STRIDE] = 0;
    if (threadIdx.x == 0) {
        S->status = WRS_OK;
        S->bad = 0;
        S->count = 0;
        S->count2 = 0;
        S->maxkey_bits = 0;
        S->k = A.k;
        S->rank = A.k;
        S->resolved = 0;
        S->nlev = 0;
        S->small_count = 0;
        S->total_bits = 0;
        S->kkey = 0.0;
        S->kidx = -1;
    }
    const int64_t n = A.n;
    const int m = (int)min((int64_t)WOR_TAU_M, n);
    const double stride = (double)n / (double)m;
    const double kt = (double)A.k * 1.02 + 4.0 * sqrt((double)A.k) + 64.0;
    const double scale = (double)n / (double)m;
    // local weights
    double wl[WOR_TAU_M / 1024];
    double wsum = 0.0;
    for (int e = 0; e < WOR_TAU_M / 1024; ++e) {
        const int s = threadIdx.x + e * 1024;
        double v = 0.0;
        if (s < m) {
            const int64_t i = min((int64_t)((double)s * stride), n - 1);
            const float f = A.w[i];
            v = (f > 0.0f && !isinf(f)) ? (double)f : 0.0;
        }
        wl[e] = v;
        wsum += v;
    }
    auto block_sum = [&](double x) -> double {
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        const int wv = threadIdx.x >> 6;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[wv] = x;
        __syncthreads();
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
        return t;
    };
    const double W = block_sum(wsum) * scale;
    double tau;
    if (!(W > 0.0) || kt >= 0.5 * (double)n) {
        tau = INFINITY;
    } else {
        tau = kt / W;  // F(tau) <= kt; Newton from below on a concave F
        for (int it = 0; it < 40; ++it) {
            double f = 0.0, fp = 0.0;
            for (int e = 0; e < WOR_TAU_M / 1024; ++e) {
                const double v = wl[e];
                const double ex = exp(-v * tau);
                f += -expm1(-v * tau);
                fp += v * ex;
            }
            const double F = block_sum(f) * scale;
            const double Fp = block_sum(fp) * scale;
            if (!(Fp > 0.0)) { tau = INFINITY; break; }
            const double step = (kt - F) / Fp;
            tau += step;
            if (fabs(kt - F) < 0.25 || step <= tau * 1e-12) break;
        }
        if (!(tau < INFINITY)) tau = INFINITY;
    }
    if (threadIdx.x == 0) S->tau = tau;
}

// ---------------------------------------------------------------------------
// Candidates are staged in LDS per block (at most WOR_TPB * WOR_IPT of them)
// and reserved in the output with one atomic per block.
__global__ __launch_bounds__(WOR_TPB) void k_wor_filter(WorArgs A, int pass) {
    // Each wave stages, in its own region, the items that pass the prefilter:
    // (index, x0 << 32 | weight bits); then, compacted in place, its
    // candidates (index, key).
    constexpr int WREG = 64 * WOR_IPT;  // staging entries per wave
    __shared__ uint64_t s_key[WOR_TPB * WOR_IPT];
    __shared__ int32_t s_idx[WOR_TPB * WOR_IPT];
    __shared__ double s_max[WOR_TPB / 64];
    __shared__ uint32_t s_bad[WOR_TPB / 64];
    __shared__ uint32_t s_wc[WOR_TPB / 64];
    __shared__ uint32_t s_base;
    WorScalars* S = A.S;
    if (pass == 2) {
        if (S->status != WRS_OK || (int64_t)S->count >= A.k) return;
    }
    const double tau = (pass == 2) ? (double)INFINITY : S->tau;
    const int shard = (int)(blockIdx.x % WOR_SHARDS);
    const int64_t n = A.n;
    if (pass == 1) {  // clear this block's share of the bitmap
        const int64_t per = cdiv(A.nwords, (int64_t)gridDim.x);
        const int64_t w0 = (int64_t)blockIdx.x * per;
        const int64_t w1 = min(A.nwords, w0 + per);
        for (int64_t i = w0 + threadIdx.x; i < w1; i += WOR_TPB) A.bitmap[i] = 0u;
    }
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int wbase = wv * WREG;
    uint32_t bad = 0;
    const int64_t base = (int64_t)blockIdx.x * (WOR_TPB * WOR_IPT);
    // Phase 1, per item: domain check, Philox, and the prefilter 1 - u <= tau w
    // (a key -ln(u) / w <= tau implies it since -ln(u) >= 1 - u).  Survivors are
    // staged; the logarithm waits for phase 2, where every lane has one.  A
    // thread takes four consecutive items at a time, the four words of one
    // Philox block.
    const bool vec = (((uintptr_t)A.w) & 15) == 0;
    uint32_t nst = 0;  // staged by this wave (the same in all its lanes)
    for (int e = 0; e < WOR_IPT / 4; ++e) {
        const int64_t i0 = base + 4 * ((int64_t)e * WOR_TPB + threadIdx.x);
        float v4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (vec && i0 + 3 < n) {
            const vfloat4 x = *(const WRS_GLOBAL vfloat4*)(glb(A.w) + i0);
            v4[0] = x.x; v4[1] = x.y; v4[2] = x.z; v4[3] = x.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (i0 + j < n) v4[j] = glb(A.w)[i0 + j];
        }
        const uint4 xb = wor_block(A, i0 >> 2);
        const uint32_t xw[4] = {xb.x, xb.y, xb.z, xb.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = i0 + j;
            const float v = v4[j];
            bool pre = false;
            if (i < n) {
                bad |= (uint32_t)(!(v >= 0.0f) || isinf(v));
                if (v > 0.0f && !isinf(v)) {
                    const double omu = (double)(0xFFFFFFFFu - xw[j]) * (1.0 / 4294967296.0);  // 1 - u
                    pre = omu <= tau * (double)v * (1.0 + 1e-12);
                }
            }
            const unsigned long long mask = __ballot(pre);
            if (pre) {
                const uint32_t p = wbase + nst + __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                s_key[p] = ((uint64_t)xw[j] << 32) | __float_as_uint(v);
                s_idx[p] = (int32_t)i;
            }
            nst += (uint32_t)__popcll(mask);
        }
    }
    // Phase 2 (per wave): keys of the staged items, 64 at a time, and an
    // ordered compaction of the candidates (key <= tau) in place.  A lane's
    // output slot is at or below its input slot, and the wave's LDS accesses
    // run in program order, so no entry is overwritten before it is read.
    double kmax = 0.0;
    uint32_t nc = 0;  // this wave's candidates
    for (uint32_t r0 = 0; r0 < nst; r0 += 64) {
        const uint32_t c = r0 + lane;
        bool cand = false;
        double key = 0.0;
        int32_t idx = 0;
        if (c < nst) {
            const uint64_t st = s_key[wbase + c];
            idx = s_idx[wbase + c];
            const float v = __uint_as_float((uint32_t)st);
            key = neg_log_u((uint32_t)(st >> 32)) / (double)v;
            cand = key <= tau;
        }
        const unsigned long long mask = __ballot(cand);
        if (cand) {
            const uint32_t p = wbase + nc + __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            s_key[p] = (uint64_t)__double_as_longlong(key);
            s_idx[p] = idx;
            kmax = fmax(kmax, key);
        }
        nc += (uint32_t)__popcll(mask);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        kmax = fmax(kmax, __shfl_xor(kmax, off, 64));
        bad |= __shfl_xor(bad, off, 64);
    }
    if (lane == 0) {
        s_max[wv] = kmax;
        s_bad[wv] = bad;
        s_wc[wv] = nc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int k = 0; k < WOR_TPB / 64; ++k) {
            kmax = fmax(kmax, s_max[k]);
            bad |= s_bad[k];
            tot += s_wc[k];
        }
        s_base = tot ? (uint32_t)atomicAdd(shard_word(A, pass, 0, shard), (unsigned long long)tot) : 0u;
        if (kmax > 0.0) atomicMax(shard_word(A, pass, 1, shard), (unsigned long long)__double_as_longlong(kmax));
        if (pass == 1 && bad) atomicOr(&S->bad, 1u);
    }
    __syncthreads();
    // this block's slots: shard region + reserved offset + earlier waves
    int64_t b0 = (int64_t)shard * A.scap + s_base;
    for (int k = 0; k < wv; ++k) b0 += s_wc[k];
    for (uint32_t c = lane; c < nc; c += 64) {
        const int64_t p = b0 + c;  // < (shard + 1) * scap: the shard's blocks hold at most scap items
        A.ckey[p] = __longlong_as_double((long long)s_key[wbase + c]);
        A.cidx[p] = s_idx[wbase + c];
    }
}

// After a filter pass: candidates per shard -> prefix table, total, max key.
__global__ __launch_bounds__(WOR_SHARDS) void k_wor_shards(WorArgs A, int pass) {
    WorScalars* S = A.S;
    if (pass == 2 && (S->status != WRS_OK || (int64_t)S->count >= A.k)) return;
    const int s = threadIdx.x;  // one wave, one lane per shard
    const uint32_t c = (uint32_t)*shard_word(A, pass, 0, s);
    const unsigned long long m = *shard_word(A, pass, 1, s);
    const uint32_t incl = wave_incl_scan(c);
    S->prefix[pass - 1][s] = incl - c;
    unsigned long long mx = m;
    for (int off = 32; off >= 1; off >>= 1) mx = max(mx, (unsigned long long)__shfl_xor(mx, off, 64));
    if (s == WOR_SHARDS - 1) {
        S->prefix[pass - 1][WOR_SHARDS] = incl;
        if (pass == 1) S->count = incl; else S->count2 = incl;
        S->maxkey_bits = max(S->maxkey_bits, mx);  // non-negative doubles order as their bits
    }
}

// Number of candidates of the pass that holds the answer.
__device__ __forceinline__ uint32_t wor_ncand(const WorScalars* S) {
    return ((int64_t)S->count >= S->k) ? S->count : S->count2;
}

// Candidate c (0 <= c < wor_ncand) of the pass in use lives in shard s, the
// largest with P[s] <= c, at slot s * scap + c - P[s].  P is the pass's prefix
// table, copied to LDS by every block (all threads, then a barrier).
__device__ __forceinline__ void load_cand_map(const WorScalars* S, uint32_t* P) {
    const int pass = ((int64_t)S->count >= S->k) ? 0 : 1;
    for (int i = threadIdx.x; i <= WOR_SHARDS; i += blockDim.x) P[i] = S->prefix[pass][i];
    __syncthreads();
}

__device__ __forceinline__ int64_t cand_slot(const uint32_t* P, int64_t scap, uint32_t c) {
    int lo = 0, hi = WOR_SHARDS - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P[mid] <= c) lo = mid; else hi = mid - 1;
    }
    return (int64_t)lo * scap + (c - P[lo]);
}

__device__ __forceinline__ int wor_bin(double key, double lo, double scale) {
    const double b = floor((key - lo) * scale);
    return (int)fmin(fmax(b, 0.0), (double)(WOR_NB - 1));
}

// Radix level l >= WOR_NLIN: the 14-bit digit of the key's bit pattern at this
// shift (the last level takes the 8 lowest bits).
__device__ __forceinline__ int wor_shift(int l) { return max(0, 50 - 14 * (l - WOR_NLIN)); }
__device__ __forceinline__ int wor_digit(double key, int l) {
    const uint64_t bits = (uint64_t)__double_as_longlong(key);
    return (int)(l == WOR_NLEV - 1 ? (bits & 0xFFu) : ((bits >> wor_shift(l)) & (uint64_t)(WOR_NB - 1)));
}

// Bin of a key at level l (linear, or radix).
__device__ __forceinline__ int wor_level_bin(const WorScalars* S, double key, int l) {
    return l < WOR_NLIN ? wor_bin(key, S->level_lo[l], S->level_scale[l]) : wor_digit(key, l);
}

// Does candidate key fall into the chosen bins of levels [0, upto)?
__device__ __forceinline__ bool wor_in_set(const WorScalars* S, double key, int upto) {
    for (int l = 0; l < min(upto, WOR_NLIN); ++l)
        if (wor_bin(key, S->level_lo[l], S->level_scale[l]) != S->level_bin[l]) return false;
    if (upto > WOR_NLIN) {
        // radix levels [WOR_NLIN, upto): the bits above the last chosen level's shift
        const uint64_t bits = (uint64_t)__double_as_longlong(key);
        const int sh = wor_shift(upto - 1);
        if ((bits >> sh) != S->radix_prefix) return false;
    }
    return true;
}

__global__ __launch_bounds__(WOR_CAND_TPB) void k_wor_hist(WorArgs A, int level) {
    __shared__ uint32_t h[WOR_NB];
    __shared__ uint32_t P[WOR_SHARDS + 1];
    WorScalars* S = A.S;
    if (S->status != WRS_OK || S->resolved || S->bad) return;
    const uint32_t nc = wor_ncand(S);
    if ((int64_t)nc < A.k) return;
    load_cand_map(S, P);
    double lo, scale;
    if (level == 0) {
        const double mx = __longlong_as_double((long long)S->maxkey_bits);
        lo = 0.0;
        scale = (mx > 0.0) ? (double)WOR_NB / (mx * (1.0 + 1e-9)) : 1.0;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            S->level_lo[0] = lo;
            S->level_scale[0] = scale;
        }
    } else if (level < WOR_NLIN) {
        lo = S->level_lo[level];
        scale = S->level_scale[level];
    } else {
        lo = 0.0;
        scale = 1.0;
    }
    for (int i = threadIdx.x; i < WOR_NB; i += WOR_CAND_TPB) h[i] = 0;
    __syncthreads();
    for (int64_t c = (int64_t)blockIdx.x * WOR_CAND_TPB + threadIdx.x; c < nc; c += (int64_t)gridDim.x * WOR_CAND_TPB) {
        const double key = A.ckey[cand_slot(P, A.scap, (uint32_t)c)];
        if (level == 0 || wor_in_set(S, key, level))
            atomicAdd(&h[level < WOR_NLIN ? wor_bin(key, lo, scale) : wor_digit(key, level)], 1u);
    }
    __syncthreads();
    uint32_t* g = A.hist + (size_t)level * WOR_NB;
    for (int i = threadIdx.x; i < WOR_NB; i += WOR_CAND_TPB)
        if (h[i]) atomicAdd(&g[i], h[i]);
}

// Pick the bin of this level that holds the rank-th key, from the level's
// histogram g (1024 threads): update the rank, the chosen bins, and whether
// the select is resolved.  Runs the domain checks first.
__device__ void wor_pick(const WorArgs& A, int level, const uint32_t* g, uint32_t* wsum) {
    WorScalars* S = A.S;
    if (threadIdx.x == 0) {
        // domain checks once every candidate pass is complete
        if (S->status == WRS_OK && S->bad) S->status = WRS_EDOMAIN;
        if (S->status == WRS_OK && (int64_t)wor_ncand(S) < A.k) S->status = WRS_EDOMAIN;
    }
    __syncthreads();
    if (S->status != WRS_OK || S->resolved) return;
    constexpr int PER = WOR_NB / 1024;  // consecutive bins per thread
    const int t = threadIdx.x;
    uint32_t local = 0;
    for (int e = 0; e < PER; ++e) local += g[t * PER + e];
    // block scan of the per-thread counts: wave scans, then the wave totals
    const uint32_t winc = wave_incl_scan(local);
    if ((t & 63) == 63) wsum[t >> 6] = winc;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < (t >> 6); ++w) before += wsum[w];
    const int64_t excl = (int64_t)before + winc - local, incl = excl + local;
    // the one thread whose bins hold the rank-th key (the last thread if the
    // counts fall short, which the checks above rule out)
    const int64_t rank = S->rank;
    if ((excl < rank && rank <= incl) || (t == 1023 && rank > incl)) {
        int64_t cum = excl;
        int b = t * PER;
        while (b < (t + 1) * PER - 1 && cum + g[b] < rank) cum += g[b++];
        const uint32_t cnt = g[b];
        S->rank = rank - cum;
        S->level_bin[level] = b;
        if (level >= WOR_NLIN)  // the digits chosen so far: the bits above this level's shift
            S->radix_prefix = level == WOR_NLIN       ? (uint64_t)b
                              : level == WOR_NLEV - 1 ? (S->radix_prefix << 8) | (uint64_t)b
                                                      : (S->radix_prefix << 14) | (uint64_t)b;
        if (cnt <= (uint32_t)WOR_SMALL) {
            S->resolved = 1;
            S->nlev = level + 1;
            S->small_count = 0;
        } else if (level + 1 < WOR_NLIN) {
            const double lo = S->level_lo[level], sc = S->level_scale[level];
            S->level_lo[level + 1] = lo + (double)b / sc;
            S->level_scale[level + 1] = sc * (double)WOR_NB;
        } else if (level + 1 < WOR_NLEV) {
            // the next level refines the chosen bin (radix levels keep radix_prefix)
        } else {
            S->status = WRS_EDEVICE;  // more than WOR_SMALL keys equal at the boundary
        }
    }
}

__global__ __launch_bounds__(1024) void k_wor_find(WorArgs A, int level) {
    __shared__ uint32_t wsum[1024 / 64];
    wor_pick(A, level, A.hist + (size_t)level * WOR_NB, wsum);
}

// The radix levels, all in one workgroup: each level counts the candidates
// still in the set into an LDS histogram and picks its bin.  They are needed
// only when the linear levels leave more than WOR_SMALL candidates in the
// target bin (the fallback pass's candidate set, or keys piled into a tiny
// range); otherwise the kernel finds the select resolved and exits, one
// launch in place of a histogram and a pick per radix level.
__global__ __launch_bounds__(1024) void k_wor_radix(WorArgs A) {
    __shared__ uint32_t h[WOR_NB];
    __shared__ uint32_t P[WOR_SHARDS + 1];
    __shared__ uint32_t wsum[1024 / 64];
    WorScalars* S = A.S;
    for (int level = WOR_NLIN; level < WOR_NLEV; ++level) {
        const uint32_t nc = wor_ncand(S);
        const bool active = S->status == WRS_OK && !S->resolved && !S->bad && (int64_t)nc >= A.k;
        if (active) {
            load_cand_map(S, P);
            for (int i = threadIdx.x; i < WOR_NB; i += 1024) h[i] = 0;
            __syncthreads();
            for (int64_t c = threadIdx.x; c < nc; c += 1024) {
                const double key = A.ckey[cand_slot(P, A.scap, (uint32_t)c)];
                if (wor_in_set(S, key, level)) atomicAdd(&h[wor_digit(key, level)], 1u);
            }
            __syncthreads();
        }
        wor_pick(A, level, h, wsum);  // runs the domain checks even when inactive
        __syncthreads();
        if (!active) return;
    }
}

__global__ __launch_bounds__(WOR_CAND_TPB) void k_wor_gather(WorArgs A) {
    __shared__ uint32_t P[WOR_SHARDS + 1];
    WorScalars* S = A.S;
    if (S->status != WRS_OK || !S->resolved) return;
    const uint32_t nc = wor_ncand(S);
    const int nlev = S->nlev;
    load_cand_map(S, P);
    const int lane = threadIdx.x & 63;
    // every lane of the block runs the same number of iterations (the ballot needs the whole wave)
    const int64_t stride = (int64_t)gridDim.x * WOR_CAND_TPB;
    for (int64_t c0 = (int64_t)blockIdx.x * WOR_CAND_TPB; c0 < nc; c0 += stride) {
        const int64_t c = c0 + threadIdx.x;
        bool in = false;
        double key = 0.0;
        int64_t q = 0;
        if (c < nc) {
            q = cand_slot(P, A.scap, (uint32_t)c);
            key = A.ckey[q];
            in = wor_in_set(S, key, nlev);
        }
        // one atomic per wave
        const unsigned long long mask = __ballot(in);
        if (mask) {
            const int leader = __ffsll((long long)mask) - 1;
            uint32_t b = 0;
            if (lane == leader) b = atomicAdd(&S->small_count, (uint32_t)__popcll(mask));
            b = __shfl(b, leader, 64);
            if (in) {
                const uint32_t p = b + __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                if (p < (uint32_t)WOR_SMALL) {
                    A.skey[p] = key;
                    A.sidx[p] = A.cidx[q];
                }
            }
        }
    }
}

// Bitonic sort of the bin in LDS by (key, idx); the rank-th element is the
// last one selected.
__global__ __launch_bounds__(1024) void k_wor_final(WorArgs A) {
    __shared__ double sk[WOR_SMALL];
    __shared__ int32_t si[WOR_SMALL];
    WorScalars* S = A.S;
    if (S->status != WRS_OK || !S->resolved) return;
    const int m = (int)min(S->small_count, (uint32_t)WOR_SMALL);
    int P = 1;
    while (P < m) P <<= 1;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        if (i < m) {
            sk[i] = A.skey[i];
            si[i] = A.sidx[i];
        } else {
            sk[i] = INFINITY;
            si[i] = 0x7fffffff;
        }
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const bool gt = sk[i] > sk[j] || (sk[i] == sk[j] && si[i] > si[j]);
                    if (gt == up) {
                        const double tk = sk[i];
                        sk[i] = sk[j];
                        sk[j] = tk;
                        const int32_t ti = si[i];
                        si[i] = si[j];
                        si[j] = ti;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        const int64_t r = S->rank;  // 1-based
        if (r < 1 || r > m) {
            S->status = WRS_EDEVICE;
        } else {
            S->kkey = sk[r - 1];
            S->kidx = si[r - 1];
        }
    }
}

__global__ __launch_bounds__(WOR_CAND_TPB) void k_wor_mark(WorArgs A) {
    __shared__ uint32_t P[WOR_SHARDS + 1];
    WorScalars* S = A.S;
    if (S->status != WRS_OK) return;
    const uint32_t nc = wor_ncand(S);
    const double kk = S->kkey;
    const int32_t ki = S->kidx;
    load_cand_map(S, P);
    for (int64_t c = (int64_t)blockIdx.x * WOR_CAND_TPB + threadIdx.x; c < nc; c += (int64_t)gridDim.x * WOR_CAND_TPB) {
        const int64_t q = cand_slot(P, A.scap, (uint32_t)c);
        const double key = A.ckey[q];
        const int32_t idx = A.cidx[q];
        if (key < kk || (key == kk && idx <= ki)) atomicOr(&A.bitmap[idx >> 5], 1u << (idx & 31));
    }
}

__global__ __launch_bounds__(WOR_TPB) void k_wor_popc(WorArgs A) {
    __shared__ uint32_t s[WOR_TPB / 64];
    if (A.S->status != WRS_OK) return;
    const int64_t w0 = (int64_t)blockIdx.x * WOR_WPB;
    uint32_t c = 0;
    for (int e = 0; e < WOR_WPB / WOR_TPB; ++e) {
        const int64_t i = w0 + (int64_t)e * WOR_TPB + threadIdx.x;
        if (i < A.nwords) c += __popc(A.bitmap[i]);
    }
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) A.blk[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(1024) void k_wor_popscan(WorArgs A, int nblk) {
    __shared__ uint32_t s[1024];
    WorScalars* S = A.S;
    if (S->status != WRS_OK) return;
    // exclusive scan of nblk block totals, sequential per thread chunk
    const int per = (nblk + 1023) / 1024;
    uint32_t loc = 0;
    for (int e = 0; e < per; ++e) {
        const int i = threadIdx.x * per + e;
        if (i < nblk) loc += A.blk[i];
    }
    s[threadIdx.x] = loc;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = (threadIdx.x >= (unsigned)d) ? s[threadIdx.x - d] : 0u;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = s[threadIdx.x] - loc;
    for (int e = 0; e < per; ++e) {
        const int i = threadIdx.x * per + e;
        if (i < nblk) {
            const uint32_t v = A.blk[i];
            A.blk[i] = run;
            run += v;
        }
    }
    if (threadIdx.x == 1023) {
        S->total_bits = s[1023];
        if ((int64_t)s[1023] != A.k) S->status = WRS_EDEVICE;
    }
}

__global__ __launch_bounds__(WOR_TPB) void k_wor_compact(WorArgs A) {
    __shared__ uint32_t s[WOR_TPB / 64];
    if (A.S->status != WRS_OK) return;
    constexpr int PER = WOR_WPB / WOR_TPB;  // consecutive words per thread
    const int64_t w0 = (int64_t)blockIdx.x * WOR_WPB + (int64_t)threadIdx.x * PER;
    uint32_t words[PER];
    uint32_t c = 0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int64_t i = w0 + e;
        words[e] = (i < A.nwords) ? A.bitmap[i] : 0u;
        c += __popc(words[e]);
    }
    // block exclusive scan of c
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t incl = c;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) s[wv] = incl;
    __syncthreads();
    uint32_t pre = 0;
    for (int k = 0; k < wv; ++k) pre += s[k];
    uint32_t p = A.blk[blockIdx.x] + pre + incl - c;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        uint32_t wd = words[e];
        while (wd) {
            const int b = __ffs(wd) - 1;
            wd &= wd - 1;
            A.out[p++] = (int32_t)((w0 + e) * 32 + b);
        }
    }
}

int launch_wor(const float* w, int64_t n, int64_t k, uint64_t seed, uint32_t sid, int32_t* out, void* ws,
               hipStream_t st) {
    const WorLayout L = wor_layout(n);
    char* b = (char*)ws;
    WorArgs A;
    A.w = w;
    A.n = n;
    A.k = k;
    A.seed = seed;
    A.sid = sid;
    A.out = out;
    A.S = (WorScalars*)(b + L.sc);
    A.hist = (uint32_t*)(b + L.hist);
    A.skey = (double*)(b + L.small_key);
    A.sidx = (int32_t*)(b + L.small_idx);
    A.ckey = (double*)(b + L.cand_key);
    A.cidx = (int32_t*)(b + L.cand_idx);
    A.bitmap = (uint32_t*)(b + L.bitmap);
    A.blk = (uint32_t*)(b + L.blk);
    A.nwords = cdiv(n, 32);
    A.shard = (unsigned long long*)(b + L.shard);
    A.scap = wor_shard_cap(n);
    const int64_t fblocks = cdiv(n, (int64_t)WOR_TPB * WOR_IPT);
    const int nblk = (int)cdiv(A.nwords, WOR_WPB);
    // candidate kernels: enough blocks to fill the chip, few enough for cheap atomics
    const int cblocks = 512;
    hipLaunchKernelGGL(k_wor_tau, dim3(1), dim3(1024), 0, st, A);
    hipLaunchKernelGGL(k_wor_filter, dim3((unsigned)fblocks), dim3(WOR_TPB), 0, st, A, 1);
    hipLaunchKernelGGL(k_wor_shards, dim3(1), dim3(WOR_SHARDS), 0, st, A, 1);
    hipLaunchKernelGGL(k_wor_filter, dim3((unsigned)fblocks), dim3(WOR_TPB), 0, st, A, 2);
    hipLaunchKernelGGL(k_wor_shards, dim3(1), dim3(WOR_SHARDS), 0, st, A, 2);
    for (int l = 0; l < WOR_NLIN; ++l) {
        hipLaunchKernelGGL(k_wor_hist, dim3(cblocks), dim3(WOR_CAND_TPB), 0, st, A, l);
        hipLaunchKernelGGL(k_wor_find, dim3(1), dim3(1024), 0, st, A, l);
    }
    hipLaunchKernelGGL(k_wor_radix, dim3(1), dim3(1024), 0, st, A);
    hipLaunchKernelGGL(k_wor_gather, dim3(cblocks), dim3(WOR_CAND_TPB), 0, st, A);
    hipLaunchKernelGGL(k_wor_final, dim3(1), dim3(1024), 0, st, A);
    hipLaunchKernelGGL(k_wor_mark, dim3(cblocks), dim3(WOR_CAND_TPB), 0, st, A);
    hipLaunchKernelGGL(k_wor_popc, dim3(nblk), dim3(WOR_TPB), 0, st, A);
    hipLaunchKernelGGL(k_wor_popscan, dim3(1), dim3(1024), 0, st, A, nblk);
    hipLaunchKernelGGL(k_wor_compact, dim3(nblk), dim3(WOR_TPB), 0, st, A);
    return hipGetLastError() == hipSuccess ? WRS_OK : WRS_EDEVICE;
}

}  // namespace wrs
