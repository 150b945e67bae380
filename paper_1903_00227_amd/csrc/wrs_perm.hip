// wrs_perm.hip -- weighted random permutation (problem WRP, Sections 1 and 7).
//
// WRP permutes the items by the process of sampling without replacement run
// to k = n.  With the exponential clocks of Section 2.3 that is the order of
// the keys -ln(u_i)/w_i (ties by index), and Section 7 reduces it to sorting
// random keys; its bucketing makes buckets of constant expected occupancy for
// any weights.  Here the keys are the WOR keys in FP64 (the same Philox
// counters, the same -ln u), so the permutation's first k items are the WOR
// sample of size k.  The sort is a stable LSD radix sort over the top 40 bits
// of the keys' bit patterns (non-negative doubles order like their bits): the
// top bits of a double are a piecewise-linear log2 of it, the same kind of
// scale as the paper's logarithmic bucket map, so runs of equal top bits hold
// a constant expected number of items.  Starting from index order, the stable
// passes leave each run in index order; a last pass orders the runs of two or
// more items by their full keys.
//
// Per pass (digit = 8 bits): an upsweep counts each block's digits, a flat
// exclusive scan over the digit-major counts gives every (digit, block) its
// output offset, and a downsweep ranks the block's items stably (ballots over
// the digit bits inside each wave, wave and block prefixes in LDS), reorders
// them in LDS by digit and writes each digit's run contiguously.
#include "wrs_device.h"

namespace wrs {

constexpr int RS_TPB = 512;              // threads per radix block
constexpr int RS_IPT = 8;                // items per thread
constexpr int RS_TILE = RS_TPB * RS_IPT; // 4096 items per block
constexpr int RS_WAVES = RS_TPB / 64;
constexpr int RS_WITEMS = RS_IPT * 64;   // consecutive items of one wave
constexpr int RS_PASSES = 5;             // digits at bits 24..63
constexpr int RS_LOW = 24;               // bits below the sorted digits
constexpr int CH = 64;                   // radix blocks per chunk of the count scan

struct PermScalars {
    int32_t status;
    int32_t pad[63];
};

struct PermLayout {
    PermScalars* sc;
    uint64_t* kA;
    uint64_t* kB;
    uint32_t* vA;
    uint32_t* vB;
    uint32_t* cnt;   // [NB * 256] block-major digit counts: cnt[b * 256 + d]
    uint32_t* off;   // [NB * 256] output offset of block b's items of digit d
    uint32_t* part;  // [NC * 256] chunk column sums, then their column prefixes
    uint32_t* tot;   // [256] items of each digit
};

static inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct PermOffsets {
    size_t kA, kB, vA, vB, cnt, off, part, tot, total;
};

static PermOffsets perm_offsets(int64_t n) {
    const int64_t NB = cdiv(n, RS_TILE);
    const int64_t L = 256 * NB;
    PermOffsets o;
    size_t p = a256(sizeof(PermScalars));
    o.kA = p;   p = a256(p + sizeof(uint64_t) * n);
    o.kB = p;   p = a256(p + sizeof(uint64_t) * n);
    o.vA = p;   p = a256(p + sizeof(uint32_t) * n);
    o.vB = p;   p = a256(p + sizeof(uint32_t) * n);
    o.cnt = p;  p = a256(p + sizeof(uint32_t) * L);
    o.off = p;  p = a256(p + sizeof(uint32_t) * L);
    o.part = p; p = a256(p + sizeof(uint32_t) * 256 * cdiv(NB, CH));
    o.tot = p;  p = a256(p + sizeof(uint32_t) * 256);
    o.total = p;
    return o;
}

size_t perm_ws_bytes(int64_t n) { return perm_offsets(n).total; }

static PermLayout perm_layout(void* ws, int64_t n) {
    const PermOffsets o = perm_offsets(n);
    char* b = (char*)ws;
    PermLayout P;
    P.sc = (PermScalars*)b;
    P.kA = (uint64_t*)(b + o.kA);
    P.kB = (uint64_t*)(b + o.kB);
    P.vA = (uint32_t*)(b + o.vA);
    P.vB = (uint32_t*)(b + o.vB);
    P.cnt = (uint32_t*)(b + o.cnt);
    P.off = (uint32_t*)(b + o.off);
    P.part = (uint32_t*)(b + o.part);
    P.tot = (uint32_t*)(b + o.tot);
    return P;
}

__global__ void k_perm_init(PermScalars* sc) {
    if (threadIdx.x == 0) sc->status = WRS_OK;
}

// Key of every item: bits of -ln(u_i)/w_i (+inf for a zero weight), value i.
// A thread takes four consecutive items, the four words of one Philox block
// (item 4g + j takes word j of block g).
constexpr int PK_TPB = 256;
__global__ __launch_bounds__(PK_TPB) void k_perm_keys(const float* w, int64_t n, uint64_t seed, uint32_t sid,
                                                      uint64_t* keys, uint32_t* vals, PermScalars* sc) {
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * PK_TPB + threadIdx.x;
    const int64_t i0 = 4 * g;
    if (i0 < n) {
        float raw[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if ((((uintptr_t)w) & 15) == 0 && i0 + 3 < n) {
            const vfloat4 x = *(const WRS_GLOBAL vfloat4*)(glb(w) + i0);
            raw[0] = x.x; raw[1] = x.y; raw[2] = x.z; raw[3] = x.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (i0 + j < n) raw[j] = glb(w)[i0 + j];
        }
        const uint4 x = philox4x32_10(make_uint4((uint32_t)g, (uint32_t)((uint64_t)g >> 32), sid, 1u),
                                      (uint32_t)seed, (uint32_t)(seed >> 32));
        const uint32_t xw[4] = {x.x, x.y, x.z, x.w};
        bool bad = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i0 + j < n) {
                bad |= !(raw[j] >= 0.0f) || isinf(raw[j]);  // on the weight as given (-0 passes)
                const float v = canonical_weight(raw[j]);
                const double key = (v > 0.0f) ? neg_log_u(xw[j]) / (double)v : INFINITY;
                glb(keys)[i0 + j] = (uint64_t)__double_as_longlong(key);
                glb(vals)[i0 + j] = (uint32_t)(i0 + j);
            }
        }
        if (bad) s_bad = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_bad) atomicExch(&sc->status, (int32_t)WRS_EDOMAIN);
}

// Lanes of the wave whose valid item has digit dg (ballots over its 8 bits).
__device__ __forceinline__ uint64_t digit_peers(uint32_t dg, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const uint64_t bb = __ballot((dg >> bit) & 1u);
        peers &= ((dg >> bit) & 1u) ? bb : ~bb;
    }
    return peers;
}

// Digit counts of each block of RS_TILE items, block-major: cnt[b * 256 + d].
// 256 threads with 16 loads each keep more bytes in flight per CU than the
// downsweep's shape; a wave adds one count per distinct digit and round.
constexpr int UP_TPB = 256, UP_IPT = RS_TILE / UP_TPB;

__global__ __launch_bounds__(UP_TPB) void k_rs_up(const uint64_t* keys, int64_t n, int sh, uint32_t* cnt,
                                                  int64_t NB) {
    __shared__ uint32_t s_h[256];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    s_h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const int c = (int)min((int64_t)RS_TILE, n - base);
    uint64_t key[UP_IPT];
#pragma unroll
    for (int r = 0; r < UP_IPT; ++r) {
        const int p = wv * (UP_IPT * 64) + r * 64 + lane;
        key[r] = (p < c) ? glb(keys)[base + p] : 0ull;
    }
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < UP_IPT; ++r) {
        const int p = wv * (UP_IPT * 64) + r * 64 + lane;
        const bool valid = p < c;
        const uint32_t dg = (uint32_t)(key[r] >> sh) & 255u;
        const uint64_t peers = digit_peers(dg, valid);
        if (valid && (peers & lt) == 0) atomicAdd(&s_h[dg], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    glb(cnt)[(int64_t)blockIdx.x * 256 + tid] = s_h[tid];
}

// Output offsets off[b][d] = (items of digits below d) + (items of digit d in
// blocks before b), from the block-major counts: column sums over chunks of
// CH blocks (coalesced over d), one block per digit scans its column over the
// chunks, then each chunk adds the digit starts and its running sums.
__global__ __launch_bounds__(256) void k_col_part(const uint32_t* cnt, int64_t NB, uint32_t* part) {
    const int d = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * CH;
    uint32_t s = 0;
    for (int64_t b = b0; b < min(b0 + CH, NB); ++b) s += glb(cnt)[b * 256 + d];
    glb(part)[(int64_t)blockIdx.x * 256 + d] = s;
}

__global__ __launch_bounds__(256) void k_col_scan(uint32_t* part, int64_t NC, uint32_t* tot) {
    __shared__ uint32_t s_w[4], s_carry;
    const int d = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < NC; c0 += 256) {
        const int64_t c = c0 + tid;
        const uint32_t v = (c < NC) ? glb(part)[c * 256 + d] : 0u;
        const uint32_t inc = wave_incl_scan(v);
        if (lane == 63) s_w[wv] = inc;
        __syncthreads();
        uint32_t ex = s_carry + inc - v, t = 0;
        for (int q = 0; q < 4; ++q) {
            if (q < wv) ex += s_w[q];
            t += s_w[q];
        }
        if (c < NC) glb(part)[c * 256 + d] = ex;
        __syncthreads();
        if (tid == 0) s_carry += t;
        __syncthreads();
    }
    if (tid == 0) glb(tot)[d] = s_carry;
}

__global__ __launch_bounds__(256) void k_col_apply(const uint32_t* cnt, const uint32_t* part, const uint32_t* tot,
                                                   int64_t NB, uint32_t* off) {
    __shared__ uint32_t s_w[4];
    const int d = threadIdx.x, lane = d & 63, wv = d >> 6;
    const uint32_t t = glb(tot)[d];
    const uint32_t inc = wave_incl_scan(t);
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint32_t start = inc - t;
    for (int q = 0; q < wv; ++q) start += s_w[q];
    const int64_t b0 = (int64_t)blockIdx.x * CH;
    uint32_t run = start + glb(part)[(int64_t)blockIdx.x * 256 + d];
    for (int64_t b = b0; b < min(b0 + CH, NB); ++b) {
        glb(off)[b * 256 + d] = run;
        run += glb(cnt)[b * 256 + d];
    }
}

// One stable pass on the digit at bit sh.
__global__ __launch_bounds__(RS_TPB) void k_rs_down(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                                                    uint32_t* vout, const uint32_t* off, int64_t n, int sh,
                                                    int64_t NB) {
    __shared__ uint32_t s_wc[RS_WAVES][256];  // per-wave digit counts, then each wave's start
    __shared__ uint32_t s_dstart[256];        // block-local start of each digit
    __shared__ uint32_t s_goff[256];          // global start of this block's items of each digit
    __shared__ uint32_t s_tmp[RS_WAVES];
    __shared__ uint64_t s_key[RS_TILE];
    __shared__ uint32_t s_val[RS_TILE];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t b = blockIdx.x, base = b * RS_TILE;
    const int c = (int)min((int64_t)RS_TILE, n - base);
    for (int q = tid; q < RS_WAVES * 256; q += RS_TPB) (&s_wc[0][0])[q] = 0;
    if (tid < 256) s_goff[tid] = glb(off)[b * 256 + tid];
    __syncthreads();
    uint64_t key[RS_IPT];
    uint32_t val[RS_IPT], rk[RS_IPT];
    const uint64_t lt = (1ull << lane) - 1ull;
    // rank inside the wave: the wave's items in order, 64 per round
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const int p = wv * RS_WITEMS + r * 64 + lane;
        const bool valid = p < c;
        key[r] = valid ? glb(kin)[base + p] : ~0ull;
        val[r] = valid ? glb(vin)[base + p] : 0u;
    }
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const int p = wv * RS_WITEMS + r * 64 + lane;
        const bool valid = p < c;
        const uint32_t dg = (uint32_t)(key[r] >> sh) & 255u;
        const uint64_t peers = digit_peers(dg, valid);
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        // every peer reads the count before its lowest lane writes the new
        // one (one wave: its LDS accesses run in program order)
        const uint32_t before = valid ? s_wc[wv][dg] : 0u;
        rk[r] = before + below;
        if (valid && below == 0) s_wc[wv][dg] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // digit starts in the block, and each wave's start inside its digit
    // (threads 0..255 own one digit each; every thread reaches each barrier)
    uint32_t cw[RS_WAVES], tot = 0;
    if (tid < 256) {
#pragma unroll
        for (int q = 0; q < RS_WAVES; ++q) {
            cw[q] = s_wc[q][tid];
            tot += cw[q];
        }
    }
    const uint32_t inc = wave_incl_scan(tot);
    if (lane == 63) s_tmp[wv] = inc;
    __syncthreads();
    if (tid < 256) {
        uint32_t ex = inc - tot;
        for (int q = 0; q < wv; ++q) ex += s_tmp[q];
        s_dstart[tid] = ex;
#pragma unroll
        for (int q = 0; q < RS_WAVES; ++q) {  // column tid: read above by this thread only
            s_wc[q][tid] = ex;
            ex += cw[q];
        }
    }
    __syncthreads();
    // the block's items in digit order, stable
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const int p = wv * RS_WITEMS + r * 64 + lane;
        if (p < c) {
            const uint32_t dg = (uint32_t)(key[r] >> sh) & 255u;
            const uint32_t lp = s_wc[wv][dg] + rk[r];
            s_key[lp] = key[r];
            s_val[lp] = val[r];
        }
    }
    __syncthreads();
    // each digit's run to its global place (consecutive threads, consecutive slots)
    for (int q = tid; q < c; q += RS_TPB) {
        const uint64_t k = s_key[q];
        const uint32_t dg = (uint32_t)(k >> sh) & 255u;
        const int64_t g = (int64_t)s_goff[dg] + (q - (int32_t)s_dstart[dg]);
        glb(kout)[g] = k;
        glb(vout)[g] = s_val[q];
    }
}

// Runs of two or more items with equal sorted bits, ordered by the full key
// and then the index (a run is in index order after the stable passes; runs
// hold a constant expected number of items).  A run of +inf keys (zero
// weights) is already in index order.  The sorted keys are only read here, so
// every thread finds the same runs; the thread of a run's first item copies
// the run's keys to the same positions of the idle key buffer and sorts them
// there together with the run's indices (runs are disjoint).
constexpr int FIX_IPT = 8;  // items per thread of the fix-up (enough loads in flight per wave)

__device__ void sort_run(const WRS_GLOBAL uint64_t* K, WRS_GLOBAL uint64_t* S, WRS_GLOBAL uint32_t* V, int64_t i,
                         int64_t n) {
    const uint64_t top = K[i] >> RS_LOW;
    int64_t e = i + 2;
    while (e < n && (K[e] >> RS_LOW) == top) ++e;
    for (int64_t a = i; a < e; ++a) S[a] = K[a];
    for (int64_t a = i + 1; a < e; ++a) {  // insertion sort by (key, index)
        const uint64_t ka = S[a];
        const uint32_t va = V[a];
        int64_t j = a - 1;
        while (j >= i && (S[j] > ka || (S[j] == ka && V[j] > va))) {
            S[j + 1] = S[j];
            V[j + 1] = V[j];
            --j;
        }
        S[j + 1] = ka;
        V[j + 1] = va;
    }
}

__global__ __launch_bounds__(256) void k_rs_fix(const uint64_t* keys, uint64_t* scratch, uint32_t* vals,
                                                int64_t n) {
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * FIX_IPT;
    if (i0 >= n) return;
    const WRS_GLOBAL uint64_t* K = glb(keys);
    uint64_t k[FIX_IPT + 2];  // items i0 - 1 .. i0 + FIX_IPT
    if (i0 + FIX_IPT <= n) {  // whole run of items: four 16-byte loads (i0 is a multiple of 8)
#pragma unroll
        for (int q = 0; q < FIX_IPT / 2; ++q) {
            const vuint4 x = *(const WRS_GLOBAL vuint4*)(K + i0 + 2 * q);
            k[1 + 2 * q] = ((uint64_t)x.y << 32) | x.x;
            k[2 + 2 * q] = ((uint64_t)x.w << 32) | x.z;
        }
    } else {
#pragma unroll
        for (int e = 1; e <= FIX_IPT; ++e) k[e] = (i0 - 1 + e < n) ? K[i0 - 1 + e] : ~0ull;
    }
    k[0] = (i0 > 0) ? K[i0 - 1] : ~0ull;
    k[FIX_IPT + 1] = (i0 + FIX_IPT < n) ? K[i0 + FIX_IPT] : ~0ull;
#pragma unroll
    for (int e = 1; e <= FIX_IPT; ++e) {
        const int64_t i = i0 - 1 + e;
        if (i >= n) break;
        const uint64_t top = k[e] >> RS_LOW;
        if ((k[e] >> 52) >= 0x7FFull) continue;  // +inf (or NaN on rejected input): nothing to order
        if (i > 0 && (k[e - 1] >> RS_LOW) == top) continue;
        if (i + 1 >= n || (k[e + 1] >> RS_LOW) != top) continue;
        if (e + 1 <= FIX_IPT && (i + 2 >= n || (k[e + 2] >> RS_LOW) != top)) {
            // a run of two (the common case), in registers: its indices are in
            // index order, so they swap only when the keys are out of order
            if (k[e] > k[e + 1]) {
                WRS_GLOBAL uint32_t* V = glb(vals);
                const uint32_t a = V[i], b = V[i + 1];
                V[i] = b;
                V[i + 1] = a;
            }
            continue;
        }
        sort_run(K, glb(scratch), glb(vals), i, n);
    }
}

int launch_perm(const float* d_w, int64_t n, uint64_t seed, uint32_t sid, int32_t* d_out, void* ws,
                hipStream_t st) {
    const PermLayout P = perm_layout(ws, n);
    const int64_t NB = cdiv(n, RS_TILE);
    const int64_t NC = cdiv(NB, CH);
#define WRS_CHECK()                                      \
    do {                                                 \
        hipError_t e_ = hipGetLastError();               \
        if (e_ != hipSuccess) return (int)e_;            \
    } while (0)
    hipLaunchKernelGGL(k_perm_init, dim3(1), dim3(64), 0, st, P.sc);
    WRS_CHECK();
    hipLaunchKernelGGL(k_perm_keys, dim3((unsigned)cdiv(n, 4 * PK_TPB)), dim3(PK_TPB), 0, st, d_w, n, seed, sid, P.kA, P.vA,
                       P.sc);
    WRS_CHECK();
    uint64_t* kin = P.kA;
    uint32_t* vin = P.vA;
    for (int pass = 0; pass < RS_PASSES; ++pass) {
        const int sh = RS_LOW + 8 * pass;
        const bool last = pass == RS_PASSES - 1;
        uint64_t* kout = (kin == P.kA) ? P.kB : P.kA;
        uint32_t* vout = last ? (uint32_t*)d_out : ((vin == P.vA) ? P.vB : P.vA);
        hipLaunchKernelGGL(k_rs_up, dim3((unsigned)NB), dim3(UP_TPB), 0, st, (const uint64_t*)kin, n, sh, P.cnt, NB);
        WRS_CHECK();
        hipLaunchKernelGGL(k_col_part, dim3((unsigned)NC), dim3(256), 0, st, (const uint32_t*)P.cnt, NB, P.part);
        WRS_CHECK();
        hipLaunchKernelGGL(k_col_scan, dim3(256), dim3(256), 0, st, P.part, NC, P.tot);
        WRS_CHECK();
        hipLaunchKernelGGL(k_col_apply, dim3((unsigned)NC), dim3(256), 0, st, (const uint32_t*)P.cnt,
                           (const uint32_t*)P.part, (const uint32_t*)P.tot, NB, P.off);
        WRS_CHECK();
        hipLaunchKernelGGL(k_rs_down, dim3((unsigned)NB), dim3(RS_TPB), 0, st, (const uint64_t*)kin,
                           (const uint32_t*)vin, kout, vout, (const uint32_t*)P.off, n, sh, NB);
        WRS_CHECK();
        kin = kout;
        vin = vout;
    }
    uint64_t* idle = (kin == P.kA) ? P.kB : P.kA;
    hipLaunchKernelGGL(k_rs_fix, dim3((unsigned)cdiv(n, 256 * FIX_IPT)), dim3(256), 0, st, (const uint64_t*)kin, idle,
                       (uint32_t*)d_out, n);
    WRS_CHECK();
#undef WRS_CHECK
    return 0;
}

void radix_inputs(void* ws, int64_t n, uint64_t** keys, uint32_t** vals) {
    const PermLayout P = perm_layout(ws, n);
    *keys = P.kA;
    *vals = P.vA;
}

int launch_radix(void* ws, int64_t n, int first_shift, int passes, hipStream_t st, const uint64_t** keys,
                 const uint32_t** vals) {
    const PermLayout P = perm_layout(ws, n);
    const int64_t NB = cdiv(n, RS_TILE);
    const int64_t NC = cdiv(NB, CH);
    uint64_t* kin = P.kA;
    uint32_t* vin = P.vA;
    for (int pass = 0; pass < passes; ++pass) {
        const int sh = first_shift + 8 * pass;
        uint64_t* kout = (kin == P.kA) ? P.kB : P.kA;
        uint32_t* vout = (vin == P.vA) ? P.vB : P.vA;
        hipLaunchKernelGGL(k_rs_up, dim3((unsigned)NB), dim3(UP_TPB), 0, st, (const uint64_t*)kin, n, sh, P.cnt, NB);
        hipLaunchKernelGGL(k_col_part, dim3((unsigned)NC), dim3(256), 0, st, (const uint32_t*)P.cnt, NB, P.part);
        hipLaunchKernelGGL(k_col_scan, dim3(256), dim3(256), 0, st, P.part, NC, P.tot);
        hipLaunchKernelGGL(k_col_apply, dim3((unsigned)NC), dim3(256), 0, st, (const uint32_t*)P.cnt,
                           (const uint32_t*)P.part, (const uint32_t*)P.tot, NB, P.off);
        hipLaunchKernelGGL(k_rs_down, dim3((unsigned)NB), dim3(RS_TPB), 0, st, (const uint64_t*)kin,
                           (const uint32_t*)vin, kout, vout, (const uint32_t*)P.off, n, sh, NB);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return (int)e;
        kin = kout;
        vin = vout;
    }
    *keys = kin;
    *vals = vin;
    return 0;
}

}  // namespace wrs
