// wrs_build.hip -- alias-table construction and sampling kernels for gfx950.
//
// Construction follows the sweeping algorithm of Section 4.1 (Algorithm 2),
// split into independent pieces as in Section 4.2 (Algorithm 3) with the
// block-wise prefix sums of Section 4.2.2.  Everything is n-scaled: item i has
// size n*w_i and every bucket holds W.  The sweep is a stable merge of the
// light items, keyed by the deficit of the lights before them, with the heavy
// items, keyed by their own cumulative excess (a heavy goes first on ties):
//   D(i) = sum over the first i lights of (W - n w),  A_i = D(i-1),
//   E(j) = sum over the first j heavies of (n w - W), B_j = E(j).
// Light i keeps t = n w_i / W and takes the next heavy not yet emitted as its
// alias; heavy j keeps t = 1 + (E(j) - D(I)) / W where I lights precede it and
// takes the next heavy as its alias.  The paper's split() finds such merge
// states by binary search over prefix sums; here the prefix sums are exact
// integers on the grid 2^G (see quantize), so every block decides every
// comparison identically and the merge can be cut anywhere.
//
// Phases (one launch each, all jobs of a batch share every launch):
//   k_reduce    W as a double-double, weight domain check
//   k_finalize  grid exponent G and integer capacity Q = round(W / 2^G)
//   k_tileagg   per tile of 1024 items: #lights, light deficit, heavy excess,
//               and the tile rewritten lights first, then heavies
//   k_scan_*    exclusive prefix over tiles (segmented)
//   k_split     start event of every pack block (merge path over tile prefixes)
//   k_pack      merge, cut at tile events, each block handling 4..32 events
//   k_sample    alias queries
// A job with one reduction block (n <= 65536) finalizes inside k_reduce, and a
// job with one scan segment (n <= 2^21) finishes the scan and the split inside
// k_scan_seg; such jobs add no block to the launches they skip.
#include <float.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "wrs_device.h"

namespace wrs {


// ---------------------------------------------------------------------------
// Workspace layout of one table.
// ---------------------------------------------------------------------------
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BuildLayout {
    size_t sc, red, redinfo, NL, DP, EP, DP64, EP64, FH, WP, PO, pstart, sNL, sDP, sEP, sFH, total;
};

static int64_t pack_blocks(int64_t C, int32_t psteps) { return cdiv(2 * C, psteps); }

static BuildLayout layout_for(int64_t n) {
    const int64_t C = cdiv(n, TILE);
    const int64_t R = cdiv(n, RED_CHUNK);
    const int64_t S = cdiv(C, SCAN_SEG);
    BuildLayout L;
    size_t o = 0;
    L.sc = o;      o = align256(o + sizeof(BuildScalars));
    L.red = o;     o = align256(o + sizeof(double2) * R);
    L.redinfo = o; o = align256(o + sizeof(uint32_t) * 2 * R);
    L.NL = o;      o = align256(o + sizeof(uint32_t) * (C + 1));
    L.DP = o;      o = align256(o + sizeof(u128) * (C + 1));
    L.EP = o;      o = align256(o + sizeof(u128) * (C + 1));
    L.DP64 = o;    o = align256(o + sizeof(uint64_t) * (C + 1));
    L.EP64 = o;    o = align256(o + sizeof(uint64_t) * (C + 1));
    L.FH = o;      o = align256(o + sizeof(int32_t) * (C + 1));
    L.WP = o;      o = align256(o + sizeof(float) * C * TILE);
    L.PO = o;      o = align256(o + sizeof(uint16_t) * C * TILE);
    L.pstart = o;  o = align256(o + sizeof(int32_t) * pack_blocks(C, PACK_STEPS_MIN));
    L.sNL = o;     o = align256(o + sizeof(uint32_t) * (S + 1));
    L.sDP = o;     o = align256(o + sizeof(u128) * (S + 1));
    L.sEP = o;     o = align256(o + sizeof(u128) * (S + 1));
    L.sFH = o;     o = align256(o + sizeof(int32_t) * (S + 1));
    L.total = o;
    return L;
}

size_t build_ws_bytes(int64_t n) { return layout_for(n).total; }

void build_ws_layout(JobDesc& J, void* ws, int64_t n, int32_t psteps) {
    const BuildLayout L = layout_for(n);
    char* b = (char*)ws;
    J.n = n;
    J.ntiles = (int32_t)cdiv(n, TILE);
    J.nred = (int32_t)cdiv(n, RED_CHUNK);
    J.nseg = (int32_t)cdiv(J.ntiles, SCAN_SEG);
    J.sc = (BuildScalars*)(b + L.sc);
    J.red = (double2*)(b + L.red);
    J.redinfo = (uint32_t*)(b + L.redinfo);
    J.NL = (uint32_t*)(b + L.NL);
    J.DP = (u128*)(b + L.DP);
    J.EP = (u128*)(b + L.EP);
    J.DP64 = (uint64_t*)(b + L.DP64);
    J.EP64 = (uint64_t*)(b + L.EP64);
    J.FH = (int32_t*)(b + L.FH);
    J.WP = (float*)(b + L.WP);
    J.PO = (uint16_t*)(b + L.PO);
    J.pstart = (int32_t*)(b + L.pstart);
    J.psteps = psteps > 0 ? psteps : pack_steps_for(n);
    J.npack = (int32_t)pack_blocks(J.ntiles, J.psteps);
    J.sNL = (uint32_t*)(b + L.sNL);
    J.sDP = (u128*)(b + L.sDP);
    J.sEP = (u128*)(b + L.sEP);
    J.sFH = (int32_t*)(b + L.sFH);
    J.lidx = nullptr;
    J.lres = nullptr;
    J.lresf = nullptr;
    J.PI = nullptr;
    J.nmul = (uint32_t)n;
}

void build_list_layout(JobDesc& J, int64_t m) {
    J.n = m;
    J.ntiles = (int32_t)cdiv(m, TILE);
    J.nred = 0;
    J.nseg = (int32_t)cdiv(J.ntiles, SCAN_SEG);
    J.psteps = pack_steps_for(m);
    J.npack = (int32_t)pack_blocks(J.ntiles, J.psteps);
}

// PSA+ workspace: the build workspace of n items, then the greedy arrays.
struct PlusOffsets {
    size_t cnt, goff, part, res, sidx, sw, lidx, lw, PI, total;
};

static PlusOffsets plus_offsets(int64_t n) {
    const int64_t G = cdiv(n, GTILE);
    const int64_t C = cdiv(n, TILE);
    PlusOffsets P;
    size_t o = layout_for(n).total;
    P.cnt = o;  o = align256(o + sizeof(uint32_t) * G);
    P.goff = o; o = align256(o + sizeof(uint32_t) * G);
    P.part = o; o = align256(o + sizeof(uint32_t) * cdiv(G, 512));
    P.res = o;  o = align256(o + sizeof(u128) * G);
    P.sidx = o; o = align256(o + sizeof(uint32_t) * G * GTILE);
    P.sw = o;   o = align256(o + sizeof(float) * G * GTILE);
    P.lidx = o; o = align256(o + sizeof(uint32_t) * C * TILE);
    P.lw = o;   o = align256(o + sizeof(float) * C * TILE);
    P.PI = o;   o = align256(o + sizeof(uint32_t) * C * TILE);
    P.total = o;
    return P;
}

size_t plus_ws_bytes(int64_t n) { return plus_offsets(n).total; }

// 2-level workspace: the main job's scalars and reduction partials (the head of
// its build layout), the top job's build workspace, then the meta-item lists.
struct TwoOffsets {
    size_t top, lidx, lw, lres, lresf, PI, total;
};

static TwoOffsets two_offsets(int64_t n) {
    const int64_t G = cdiv(n, GTILE);
    const int64_t Ct = cdiv(G, TILE);
    TwoOffsets o;
    size_t p = align256(layout_for(n).NL);
    o.top = p;  p = align256(p + layout_for(G).total);
    o.lidx = p; p = align256(p + sizeof(uint32_t) * Ct * TILE);
    o.lw = p;   p = align256(p + sizeof(float) * Ct * TILE);
    o.lres = p; p = align256(p + sizeof(u128) * G);
    o.lresf = p; p = align256(p + sizeof(double) * G);
    o.PI = p;   p = align256(p + sizeof(uint32_t) * Ct * TILE);
    o.total = p;
    return o;
}

size_t twolevel_ws_bytes(int64_t n) { return two_offsets(n).total; }

void twolevel_layout(void* ws, int64_t n, JobDesc& J, JobDesc& top, TwoLayout& T) {
    const TwoOffsets o = two_offsets(n);
    const int64_t G = cdiv(n, GTILE);
    char* b = (char*)ws;
    build_ws_layout(J, ws, n);  // only sc, red and redinfo are used (the head)
    build_ws_layout(top, b + o.top, G);
    T.lidx = (uint32_t*)(b + o.lidx);
    T.lw = (float*)(b + o.lw);
    T.lres = (u128*)(b + o.lres);
    T.lresf = (double*)(b + o.lresf);
    T.PI = (uint32_t*)(b + o.PI);
    top.w = T.lw;
    top.lidx = T.lidx;
    top.lres = T.lres;
    top.lresf = T.lresf;
    top.PI = T.PI;
    top.nmul = (uint32_t)G;
    build_list_layout(top, G);
}

PlusLayout plus_layout(void* ws, int64_t n) {
    const PlusOffsets o = plus_offsets(n);
    char* b = (char*)ws;
    PlusLayout P;
    P.cnt = (uint32_t*)(b + o.cnt);
    P.goff = (uint32_t*)(b + o.goff);
    P.part = (uint32_t*)(b + o.part);
    P.res = (u128*)(b + o.res);
    P.sidx = (uint32_t*)(b + o.sidx);
    P.sw = (float*)(b + o.sw);
    P.lidx = (uint32_t*)(b + o.lidx);
    P.lw = (float*)(b + o.lw);
    P.PI = (uint32_t*)(b + o.PI);
    return P;
}

// ---------------------------------------------------------------------------
// a1: total weight (double-double) and domain check, RED_CHUNK items per block.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void red_item(float v, double& hi, double& lo, uint32_t& bad, uint32_t& pos) {
    bad |= (uint32_t)(!(v >= 0.0f) || isinf(v));
    pos += (uint32_t)(v > 0.0f);
    dd_acc(hi, lo, (double)v);
}

__device__ __forceinline__ void block_reduce_dd(double& hi, double& lo, uint32_t& bad, uint32_t& pos,
                                                double* s_hi, double* s_lo, uint32_t* s_bad, uint32_t* s_pos) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double oh = __shfl_xor(hi, off, 64);
        const double ol = __shfl_xor(lo, off, 64);
        bad |= __shfl_xor(bad, off, 64);
        pos += __shfl_xor(pos, off, 64);
        dd_add(hi, lo, oh, ol);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_hi[wv] = hi;
        s_lo[wv] = lo;
        s_bad[wv] = bad;
        s_pos[wv] = pos;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        hi = s_hi[0];
        lo = s_lo[0];
        bad = s_bad[0];
        pos = s_pos[0];
        for (int k = 1; k < TPB / 64; ++k) {
            dd_add(hi, lo, s_hi[k], s_lo[k]);
            bad |= s_bad[k];
            pos += s_pos[k];
        }
    }
}

__device__ void finalize_scalars(const JobDesc& J, double hi, double lo, uint32_t bad, uint32_t pos);

// The block bodies of the construction's phases take (job, block of the
// job, LDS): the phase kernels run one body per block, and the fused kernel
// for small batched tables runs every phase's bodies in one workgroup.
struct RedShared {
    double hi[TPB / 64], lo[TPB / 64];
    uint32_t bad[TPB / 64], pos[TPB / 64];
};

__device__ __forceinline__ void reduce_block(const JobDesc& J, int64_t lb, RedShared& sh) {
    const int64_t base = lb * RED_CHUNK;
    const int64_t end = min(base + (int64_t)RED_CHUNK, J.n);
    const WRS_GLOBAL float* w = glb(J.w);
    double hi = 0.0, lo = 0.0;
    uint32_t bad = 0, pos = 0;
    if ((((uintptr_t)(w + base)) & 15) == 0) {
        const int64_t nv = (end - base) >> 2;
        const WRS_GLOBAL vfloat4* w4 = (const WRS_GLOBAL vfloat4*)(w + base);
        for (int64_t g = threadIdx.x; g < nv; g += TPB) {
            const vfloat4 v = w4[g];
            red_item(v.x, hi, lo, bad, pos);
            red_item(v.y, hi, lo, bad, pos);
            red_item(v.z, hi, lo, bad, pos);
            red_item(v.w, hi, lo, bad, pos);
        }
        for (int64_t i = base + 4 * nv + threadIdx.x; i < end; i += TPB) red_item(w[i], hi, lo, bad, pos);
    } else {
        for (int64_t i = base + threadIdx.x; i < end; i += TPB) red_item(w[i], hi, lo, bad, pos);
    }
    block_reduce_dd(hi, lo, bad, pos, sh.hi, sh.lo, sh.bad, sh.pos);
    if (threadIdx.x == 0) {
        J.red[lb] = make_double2(hi, lo);
        J.redinfo[2 * lb] = bad;
        J.redinfo[2 * lb + 1] = pos;
        // a single block holds the whole total: finalize here (k_finalize gets
        // no block for this job; the scalars are the same bits either way)
        if (J.nred == 1) finalize_scalars(J, hi, lo, bad, pos);
    }
}

__global__ __launch_bounds__(TPB) void k_reduce(JobTable jt) {
    __shared__ int s_job;
    __shared__ RedShared sh;
    int64_t lb;
    const JobDesc J = job_uniform(job_of_block(jt, lb, &s_job));
    reduce_block(J, lb, sh);
}

__device__ __forceinline__ u128 u128_from_integral_double(double d) {
    const uint64_t bits = (uint64_t)__double_as_longlong(d);
    const int e = (int)((bits >> 52) & 0x7FF) - 1075;
    const uint64_t m = (bits & ((1ull << 52) - 1)) | (1ull << 52);
    return e >= 0 ? ((u128)m << e) : (u128)(m >> (-e));
}

// a1 (second half): combine partials in a fixed order, derive the grid.
// Grid exponent G, integer capacity Q and the derived scalars, from the total
// weight hi + lo (double-double) and the domain flags; one thread.
// The scalars that depend on the item count n, given the grid exponent G and
// the capacity Q (status OK).
__device__ void derive_scalars(BuildScalars& S, int64_t n) {
    const int G = S.G;
    const u128 Q = S.Q;
    S.Qd = u128_to_double(Q);
    S.rQ = 1.0 / S.Qd;
    S.nscale = ldexp((double)n, -G);
    // floor(Q / n) without 128-bit division: estimate, then correct (the
    // estimate is off by at most one or two; the loops are bounded anyway).
    // A job over few meta-items on the items' grid can have Q / n >= 2^64:
    // its items are markers with exact sizes, so Qn (the FP32 light test) is
    // unused there and saturates.
    uint64_t qn = ~0ull;
    if ((uint64_t)(Q >> 64) < (uint64_t)n) {
        qn = (uint64_t)fmin(S.Qd / (double)n, 18446744073709549568.0);  // largest double below 2^64
        const i128 rem = (i128)Q - (i128)n * (i128)qn;
        qn = (uint64_t)((i128)qn + rem / (i128)n);
        for (int it = 0; it < 4 && (u128)n * (u128)(qn + 1) <= Q; ++it) ++qn;
        for (int it = 0; it < 4 && (u128)n * (u128)qn > Q; ++it) --qn;
    }
    S.Qn = qn;
    // merge keys: prefix sums (at most n Q) shifted right to fit 62 bits
    const uint64_t qh = (uint64_t)(Q >> 64), ql = (uint64_t)Q;
    const int qbits = qh ? 128 - __clzll((long long)qh) : 64 - __clzll((long long)ql);
    const int nbits = 64 - __clzll((long long)n);
    const int sh = max(0, qbits + nbits - 62);
    S.kshift = sh;
    S.tscale = ldexp(1.0, sh) * S.rQ;
    S.Qk = (uint64_t)((Q + (sh > 0 ? ((u128)1 << (sh - 1)) : (u128)0)) >> sh);
    // quantize is monotone in w and FP32 bit patterns of w >= 0 are ordered
    // like the values: find the smallest pattern with q > Qn.
    uint32_t lo = 0, hi = 0x7F800000u;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (quantize(__uint_as_float(mid), G) > (u128)qn) hi = mid; else lo = mid + 1;
    }
    S.wthr = lo;
}

__device__ void finalize_scalars(const JobDesc& J, double hi, double lo, uint32_t bad, uint32_t pos) {
    BuildScalars S;
    S.status = WRS_OK;
    S.npos = pos;
    const double s = hi + lo;
    lo = lo - (s - hi);
    hi = s;
    S.W_hi = hi;
    S.W_lo = lo;
    S.G = 0;
    S.Q = 0;
    S.Qd = 0;
    S.rQ = 0;
    S.nscale = 0;
    S.Qn = 0;
    S.kshift = 0;
    S.wthr = 0;
    S.tscale = 0;
    S.Qk = 0;
    S.nleft = 0;
    if (bad || !(hi > 0.0)) {
        S.status = WRS_EDOMAIN;
    } else {
        const int64_t n = J.n;
        int e;
        frexp(hi, &e);                               // hi in [2^(e-1), 2^e)
        const int lgn = 63 - __clzll((long long)n);  // floor(log2 n)
        const int G = (e - 1) - lgn - 62;            // W / 2^G in [2^(lgn+62), 2^(lgn+63))
        const double Qh = ldexp(hi, -G);             // integral (>= 2^62 with 53 bits)
        const double Ql = rint(ldexp(lo, -G));
        u128 Q = u128_from_integral_double(Qh);
        Q = (u128)((i128)Q + (i128)(int64_t)Ql);
        S.G = G;
        S.Q = Q;
        derive_scalars(S, n);
    }
    *J.sc = S;
}

// Scalars of a job over m <= n meta-items on the grid of a finished job over
// the n items (same G and Q, so its sizes are exact in the same integers).
__global__ void k_finalize_on_grid(JobDesc top, const BuildScalars* base) {
    if (threadIdx.x != 0) return;
    BuildScalars S = *base;
    S.nleft = 0;
    if (S.status == WRS_OK) derive_scalars(S, top.n);
    *top.sc = S;
}

hipError_t launch_finalize_on_grid(const JobDesc& top, const BuildScalars* base, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize_on_grid, dim3(1), dim3(64), 0, st, top, base);
    return hipGetLastError();
}

__global__ __launch_bounds__(TPB) void k_finalize(JobTable jt) {
    __shared__ int s_job;
    __shared__ double s_hi[TPB / 64], s_lo[TPB / 64];
    __shared__ uint32_t s_bad[TPB / 64], s_pos[TPB / 64];
    int64_t lb;
    const JobDesc J = job_uniform(job_of_block(jt, lb, &s_job));
    double hi = 0.0, lo = 0.0;
    uint32_t bad = 0, pos = 0;
    for (int r = threadIdx.x; r < J.nred; r += TPB) {
        const double2 p = J.red[r];
        dd_add(hi, lo, p.x, p.y);
        bad |= J.redinfo[2 * r];
        pos += J.redinfo[2 * r + 1];
    }
    block_reduce_dd(hi, lo, bad, pos, s_hi, s_lo, s_bad, s_pos);
    if (threadIdx.x == 0) finalize_scalars(J, hi, lo, bad, pos);
}

// ---------------------------------------------------------------------------
// a2: per-tile aggregates.  Item i is light iff n q_i <= Q, i.e. q_i <= Qn.
// ---------------------------------------------------------------------------
// One wave per tile: each lane reads 4 float4 (lane-interleaved, 1 KiB per
// instruction across the wave), so the aggregates need no block
// synchronisation.  The wave also writes the tile in partitioned order (its
// lights, then its heavies, each in index order) with every item's offset, so
// that the merge stages one side of a tile without classifying it again.
constexpr int AGG_VEC = TILE / 256;  // float4 loads per lane


// List mode (LIST = true, the splitting stage of the greedy construction):
// the items are a list of original items in index order; a residual marker
// stands for the exact n-scaled size lres[slot] (light iff it is at most Q),
// FH holds original indices, and the partitioned copy carries original
// indices (PI) instead of tile offsets.
template <bool LIST>
struct TileaggShared {
    float w[TILES_PER_AGG_BLOCK][TILE];
    uint32_t o[TILES_PER_AGG_BLOCK][LIST ? TILE : TILE / 2];  // u16 offsets, or u32 indices
};

template <bool LIST>
__device__ __forceinline__ void tileagg_block(const JobDesc& J, int64_t lb, TileaggShared<LIST>& sh) {
    const BuildScalars* sc = J.sc;
    if (sc->status != WRS_OK) return;  // the same for the whole block
    const int wv = threadIdx.x >> 6;
    const int64_t c = lb * TILES_PER_AGG_BLOCK + wv;
    const bool active = c < J.ntiles;  // the same for the whole wave
    const int lane = threadIdx.x & 63;
    const int G = uni(sc->G);
    const uint32_t wthr = uni(sc->wthr);
    const u128 Q = uni(sc->Q);
    const int64_t n = J.n;
    const uint32_t nmul = J.nmul;
    const int64_t base = c * TILE;
    uint16_t* s_o16 = (uint16_t*)&sh.o[wv][0];
    if (active) {
        const int cnt = (int)min((int64_t)TILE, n - base);
        const WRS_GLOBAL float* w = glb(J.w) + base;
        const bool vec = (cnt == TILE) && ((((uintptr_t)w) & 15) == 0);
        float v[4 * AGG_VEC];
        uint32_t oid[LIST ? 4 * AGG_VEC : 1];
        if (vec) {  // all loads in flight together
            vfloat4 x[AGG_VEC];
#pragma unroll
            for (int r = 0; r < AGG_VEC; ++r) x[r] = *(const WRS_GLOBAL vfloat4*)(w + r * 256 + lane * 4);
            if constexpr (LIST) {
                vuint4 y[AGG_VEC];
#pragma unroll
                for (int r = 0; r < AGG_VEC; ++r) y[r] = *(const WRS_GLOBAL vuint4*)(glb(J.lidx) + base + r * 256 + lane * 4);
#pragma unroll
                for (int r = 0; r < AGG_VEC; ++r) {
                    oid[4 * r] = y[r].x; oid[4 * r + 1] = y[r].y; oid[4 * r + 2] = y[r].z; oid[4 * r + 3] = y[r].w;
                }
            }
#pragma unroll
            for (int r = 0; r < AGG_VEC; ++r) {
                v[4 * r] = x[r].x; v[4 * r + 1] = x[r].y; v[4 * r + 2] = x[r].z; v[4 * r + 3] = x[r].w;
            }
        } else {
#pragma unroll
            for (int r = 0; r < AGG_VEC; ++r) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int i = r * 256 + lane * 4 + e;
                    v[4 * r + e] = (i < cnt) ? w[i] : 0.0f;
                    if constexpr (LIST) oid[4 * r + e] = (i < cnt) ? glb(J.lidx)[base + i] : 0u;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4 * AGG_VEC; ++k) v[k] = canonical_weight(v[k]);
        // List mode: residual markers (rare) carry exact sizes; their q is 0
        // in the sums below and their sizes are added separately.
        uint32_t lmask = 0;  // LIST: bit k = item k is light
        u128 mres_l = 0, mres_h = 0;
        if constexpr (LIST) {
            bool anym = false;
#pragma unroll
            for (int k = 0; k < 4 * AGG_VEC; ++k) anym |= is_residual_marker(__float_as_uint(v[k]));
#pragma unroll
            for (int k = 0; k < 4 * AGG_VEC; ++k) {
                const int i = (k >> 2) * 256 + lane * 4 + (k & 3);
                lmask |= (uint32_t)((i < cnt) && (__float_as_uint(v[k]) < wthr)) << k;
            }
            if (__ballot(anym) != 0) {
                for (int k = 0; k < 4 * AGG_VEC; ++k) {
                    const uint32_t bits = __float_as_uint(v[k]);
                    if (is_residual_marker(bits)) {
                        const u128 m = glb(J.lres)[residual_slot(bits)];
                        const bool light = m <= Q;
                        lmask |= (uint32_t)light << k;
                        if (light) mres_l += m; else mres_h += m;
                    }
                }
                mres_l = lane63(wave_incl_scan(mres_l));
                mres_h = lane63(wave_incl_scan(mres_h));
            }
        }
        // light flags, as one ballot per (load, element)
        // (items past the tile's end hold 0, which adds nothing)
        auto is_light = [&](int r, int e) -> bool {
            if constexpr (LIST) return (lmask >> (4 * r + e)) & 1u;
            return (r * 256 + lane * 4 + e < cnt) && (__float_as_uint(v[4 * r + e]) < wthr);
        };
        // the weight whose q enters the sums (a marker's size is added apart)
        auto qw = [&](int k) -> float {
            if constexpr (LIST) return is_residual_marker(__float_as_uint(v[k])) ? 0.0f : v[k];
            return v[k];
        };
        uint32_t nl = 0;
        u128 sq = 0, sql = 0;
        int fh = FH_NONE;
        // Narrow lanes: when every nonzero weight of a lane lies on the grid,
        // within 2^36 of the lane's smallest one, each of its 16 q values is
        // below 2^60 at the scale of that smallest one, so the lane's two sums
        // are exact in one 64-bit word each and are scaled up once.
        bool narrow = false;
        if constexpr (!LIST) {
            int slo = 0x7FFFFFFF, shi = -1;
#pragma unroll
            for (int k = 0; k < 4 * AGG_VEC; ++k) {
                const uint32_t bits = __float_as_uint(v[k]);
                const int sk = grid_shift(v[k], G);
                slo = bits != 0u ? min(slo, sk) : slo;
                shi = bits != 0u ? max(shi, sk) : shi;
            }
            const bool ok = shi < 0 ? slo == 0x7FFFFFFF : (slo >= 0 && shi - slo <= 36);
            narrow = __ballot(!ok) == 0;
            if (narrow) {
                const int s0 = shi < 0 ? 0 : slo;  // a lane of zeros sums to 0 at any scale
                uint64_t a = 0, al = 0;
#pragma unroll
                for (int r = 0; r < AGG_VEC; ++r) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const uint32_t bits = __float_as_uint(v[4 * r + e]);
                        const uint32_t ex = bits >> 23;
                        const uint64_t m = (bits & 0x7FFFFFu) | (ex ? 0x800000u : 0u);
                        const uint64_t x = m << ((grid_shift(v[4 * r + e], G) - s0) & 63);
                        a += x;
                        al += is_light(r, e) ? x : 0ull;
                    }
                }
                sq = (u128)a << s0;
                sql = (u128)al << s0;
            }
        }
        if (!narrow) {
            int smin = 0;
            // (a zero weight, and a marker's 0, is 0 on the branch-free path too)
#pragma unroll
            for (int k = 0; k < 4 * AGG_VEC; ++k) smin = min(smin, qw(k) != 0.0f ? grid_shift(qw(k), G) : 0);
            if (__ballot(smin < 0) == 0) {
                // every weight of the tile lies on the grid
#pragma unroll
                for (int r = 0; r < AGG_VEC; ++r) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const bool light = is_light(r, e);
                        const u128 q = quantize_on_grid(qw(4 * r + e), G);
                        sq += q;
                        sql += light ? q : (u128)0;
                    }
                }
            } else {
                for (int k = 0; k < 4 * AGG_VEC; ++k) {
                    const bool light = is_light(k >> 2, k & 3);
                    const u128 q = quantize(qw(k), G);
                    sq += q;
                    sql += light ? q : (u128)0;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < AGG_VEC; ++r) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = r * 256 + lane * 4 + e;
                const bool light = is_light(r, e);
                nl += (uint32_t)__popcll(__ballot(light));
                fh = (i < cnt && !light) ? min(fh, (int)(base + i)) : fh;
            }
        }
        // partitioned order: lights before item i, then the heavies after all lights
        uint32_t lbefore = 0;  // lights in earlier loads
#pragma unroll
        for (int r = 0; r < AGG_VEC; ++r) {
            uint64_t lm[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) lm[e] = __ballot(is_light(r, e));
            uint32_t lr = lbefore + lanes_below(lm[0]) + lanes_below(lm[1]) + lanes_below(lm[2]) + lanes_below(lm[3]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = r * 256 + lane * 4 + e;
                const bool light = (lm[e] >> lane) & 1ull;
                const int p = light ? (int)lr : (int)(nl + (uint32_t)i - lr);
                if (i < cnt) {
                    sh.w[wv][p] = v[4 * r + e];
                    if constexpr (LIST) sh.o[wv][p] = oid[4 * r + e]; else s_o16[p] = (uint16_t)i;
                }
                lr += light;
            }
            lbefore += (uint32_t)(__popcll(lm[0]) + __popcll(lm[1]) + __popcll(lm[2]) + __popcll(lm[3]));
        }
        fh = (int)lane63((uint32_t)wave_incl_min(fh));
        sql = lane63(wave_incl_scan(sql));
        const u128 sqh = lane63(wave_incl_scan(sq)) - sql;
        if (lane == 0) {
            const uint32_t nh = (uint32_t)cnt - nl;
            glb(J.NL)[c] = nl;
            glb(J.DP)[c] = (u128)nl * Q - (u128)nmul * sql - mres_l;
            glb(J.EP)[c] = (u128)nmul * sqh + mres_h - (u128)nh * Q;
            if constexpr (LIST) fh = (fh == FH_NONE) ? FH_NONE : (int)glb(J.lidx)[fh];
            glb(J.FH)[c] = fh;
        }
    }
    __syncthreads();
    if (active) {
        // whole tile (the arrays are padded to whole tiles); entries past the
        // tile's item count are never read
        WRS_GLOBAL float* wp = glb(J.WP) + base;
#pragma unroll
        for (int r = 0; r < AGG_VEC; ++r) {
            const int i0 = r * 256 + lane * 4;
            vfloat4 x;
            x.x = sh.w[wv][i0]; x.y = sh.w[wv][i0 + 1]; x.z = sh.w[wv][i0 + 2]; x.w = sh.w[wv][i0 + 3];
            *(WRS_GLOBAL vfloat4*)(wp + i0) = x;
            if constexpr (LIST) {
                vuint4 o;
                o.x = sh.o[wv][i0]; o.y = sh.o[wv][i0 + 1]; o.z = sh.o[wv][i0 + 2]; o.w = sh.o[wv][i0 + 3];
                *(WRS_GLOBAL vuint4*)(glb(J.PI) + base + i0) = o;
            } else {
                vuint2 o;
                o.x = (uint32_t)s_o16[i0] | ((uint32_t)s_o16[i0 + 1] << 16);
                o.y = (uint32_t)s_o16[i0 + 2] | ((uint32_t)s_o16[i0 + 3] << 16);
                *(WRS_GLOBAL vuint2*)(glb(J.PO) + base + i0) = o;
            }
        }
    }
}

template <bool LIST>
__global__ __launch_bounds__(TPB) void k_tileagg(JobTable jt) {
    __shared__ int s_job;
    __shared__ TileaggShared<LIST> sh;
    int64_t lb;
    const JobDesc J = job_uniform(job_of_block(jt, lb, &s_job));
    tileagg_block<LIST>(J, lb, sh);
}

// ---------------------------------------------------------------------------
// a3: exclusive prefix over tiles (NL, DP, EP) and "first heavy at or after"
// (FH), in segments of SCAN_SEG tiles, then over segments, then fixed up.
// ---------------------------------------------------------------------------
constexpr int SEG_PER_THREAD = SCAN_SEG / TPB;

__device__ __forceinline__ int block_suffix_min_excl(int v, int* s_w) {
    // minimum of v over threads with a larger index
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_down(incl, d, 64);
        if (lane + d < 64) incl = min(incl, o);
    }
    if (lane == 0) s_w[wv] = incl;
    __syncthreads();
    int later = FH_NONE;
    for (int k = wv + 1; k < TPB / 64; ++k) later = min(later, s_w[k]);
    const int nxt = __shfl_down(incl, 1, 64);
    const int excl_in_wave = (lane == 63) ? FH_NONE : nxt;
    __syncthreads();
    return min(excl_in_wave, later);
}

// Light events before pack block b's first event (the paper's split(), on
// tile prefixes): the largest x with x == 0, or light event x before heavy
// event s0 - x + 1, where s0 = b * psteps.  Needs DP64 and EP64.
__device__ __forceinline__ int32_t pack_start(const JobDesc& J, int64_t b) {
    const int64_t C = J.ntiles;
    const int64_t s0 = b * J.psteps;
    const WRS_GLOBAL uint64_t* DP = glb(J.DP64);
    const WRS_GLOBAL uint64_t* EP = glb(J.EP64);
    int64_t lo = max((int64_t)0, s0 - C), hi = min(s0, C);
    while (lo < hi) {
        const int64_t x = (lo + hi + 1) >> 1;
        const int64_t y1 = s0 - x + 1;
        const bool ok = (y1 > C) || (x < C && DP[x] < EP[y1]);
        if (ok) lo = x; else hi = x - 1;
    }
    return (int32_t)lo;
}

struct ScanSegShared {
    ScanTmp tmp;
    int w[TPB / 64];
};

__device__ __forceinline__ void scan_seg_block(const JobDesc& J, int64_t lb, ScanSegShared& sh) {
    if (J.sc->status != WRS_OK) return;
    const int64_t C = J.ntiles;
    const int64_t t0 = lb * SCAN_SEG + (int64_t)threadIdx.x * SEG_PER_THREAD;
    uint32_t nl[SEG_PER_THREAD];
    u128 dp[SEG_PER_THREAD], ep[SEG_PER_THREAD];
    int fh[SEG_PER_THREAD];
    uint32_t snl = 0;
    u128 sdp = 0, sep = 0;
    int fmin = FH_NONE;
#pragma unroll
    for (int e = 0; e < SEG_PER_THREAD; ++e) {
        const int64_t c = t0 + e;
        if (c < C) {
            nl[e] = J.NL[c];
            dp[e] = J.DP[c];
            ep[e] = J.EP[c];
            fh[e] = J.FH[c];
        } else {
            nl[e] = 0;
            dp[e] = 0;
            ep[e] = 0;
            fh[e] = FH_NONE;
        }
        snl += nl[e];
        sdp += dp[e];
        sep += ep[e];
        fmin = min(fmin, fh[e]);
    }
    uint32_t nl_ex, nl_tot;
    u128 dp_ex, ep_ex, dp_tot, ep_tot;
    block_scan3(snl, sdp, sep, nl_ex, dp_ex, ep_ex, nl_tot, dp_tot, ep_tot, sh.tmp);
    const int later = block_suffix_min_excl(fmin, sh.w);
    int suf = later;
#pragma unroll
    for (int e = SEG_PER_THREAD - 1; e >= 0; --e) {
        suf = min(suf, fh[e]);
        fh[e] = suf;
    }
    // The only segment: its prefixes are final, so this block also writes the
    // 64-bit keys and the totals (k_scan_top and k_scan_fix get no blocks).
    const bool single = J.nseg == 1;
    const int ks = uni(J.sc->kshift);
#pragma unroll
    for (int e = 0; e < SEG_PER_THREAD; ++e) {
        const int64_t c = t0 + e;
        if (c < C) {
            J.NL[c] = nl_ex;
            J.DP[c] = dp_ex;
            J.EP[c] = ep_ex;
            J.FH[c] = fh[e];
            if (single) {
                J.DP64[c] = (uint64_t)(dp_ex >> ks);
                J.EP64[c] = (uint64_t)(ep_ex >> ks);
            }
        }
        nl_ex += nl[e];
        dp_ex += dp[e];
        ep_ex += ep[e];
    }
    if (threadIdx.x == 0) {
        J.sNL[lb] = nl_tot;
        J.sDP[lb] = dp_tot;
        J.sEP[lb] = ep_tot;
        J.sFH[lb] = min(fmin, later);  // thread 0 holds the first tiles: the segment minimum
    }
    if (single) {
        if (threadIdx.x == 0) {
            J.NL[C] = nl_tot;
            J.DP[C] = dp_tot;
            J.EP[C] = ep_tot;
            J.DP64[C] = (uint64_t)(dp_tot >> ks);
            J.EP64[C] = (uint64_t)(ep_tot >> ks);
            J.FH[C] = FH_NONE;
        }
        // every key is written (and visible to the block): the pack starts too
        __syncthreads();
        for (int64_t b = threadIdx.x; b < J.npack; b += TPB) glb(J.pstart)[b] = pack_start(J, b);
    }
}

__global__ __launch_bounds__(TPB) void k_scan_seg(JobTable jt) {
    __shared__ int s_job;
    __shared__ ScanSegShared sh;
    int64_t lb;
    const JobDesc J = job_uniform(job_of_block(jt, lb, &s_job));
    scan_seg_block(J, lb, sh);
}

__global__ __launch_bounds__(TPB) void k_scan_top(JobTable jt) {
    __shared__ int s_job;
    __shared__ ScanTmp tmp;
    __shared__ int s_w[TPB / 64];
    int64_t lb;
    const JobDesc J = job_uniform(job_of_block(jt, lb, &s_job));
    if (J.sc->status != WRS_OK) return;
    const int S = J.nseg;
    const int per = (S + TPB - 1) / TPB;   // segments per thread (<= 4 for n < 2^31)
    const int s0 = threadIdx.x * per;
    uint32_t snl = 0;
    u128 sdp = 0, sep = 0;
    int fmin = FH_NONE;
    for (int e = 0; e < per; ++e) {
        const int s = s0 + e;
        if (s < S) {
            snl += J.sNL[s];
            sdp += J.sDP[s];
            sep += J.sEP[s];
            fmin = min(fmin, J.sFH[s]);
        }
    }
    uint32_t nl_ex, nl_tot;
    u128 dp_ex, ep_ex, dp_tot, ep_tot;
    block_scan3(snl, sdp, sep, nl_ex, dp_ex, ep_ex, nl_tot, dp_tot, ep_tot, tmp);
    const int later = block_suffix_min_excl(fmin, s_w);
    // suffix minimum, inclusive, over this thread's segments
    int fsuf[4];
    int suf = later;
    for (int e = per - 1; e >= 0; --e) {
        const int s = s0 + e;
        if (s < S) suf = min(suf, J.sFH[s]);
        if (e < 4) fsuf[e] = suf;
    }
    __syncthreads();
    for (int e = 0; e < per; ++e) {
        const int s = s0 + e;
        if (s < S) {
            const uint32_t a = J.sNL[s];
            const u128 b = J.sDP[s], c = J.sEP[s];
            J.sNL[s] = nl_ex;
            J.sDP[s] = dp_ex;
            J.sEP[s] = ep_ex;
            J.sFH[s] = fsuf[e];
            nl_ex += a;
            dp_ex += b;
            ep_ex += c;
        }
    }
    if (threadIdx.x == 0) {
        const int64_t C = J.ntiles;
        const int ks = uni(J.sc->kshift);
        J.NL[C] = nl_tot;
        J.DP[C] = dp_tot;
        J.EP[C] = ep_tot;
        J.DP64[C] = (uint64_t)(dp_tot >> ks);
        J.EP64[C] = (uint64_t)(ep_tot >> ks);
        J.FH[C] = FH_NONE;
        J.sFH[S] = FH_NONE;
    }
}

__global__ __launch_bounds__(TPB) void k_scan_fix(JobTable jt) {
    __shared__ int s_job;
    int64_t lb;
    const JobDesc J = job_uniform(job_of_block(jt, lb, &s_job));
    if (J.sc->status != WRS_OK) return;
    const int64_t C = J.ntiles;
    const uint32_t pnl = J.sNL[lb];
    const u128 pdp = J.sDP[lb], pep = J.sEP[lb];
    const int nxt = J.sFH[lb + 1];
    const int ks = uni(J.sc->kshift);
    for (int e = 0; e < SEG_PER_THREAD; ++e) {
        const int64_t c = lb * SCAN_SEG + (int64_t)e * TPB + threadIdx.x;
        if (c < C) {
            J.NL[c] += pnl;
            const u128 dp = J.DP[c] + pdp;
            const u128 ep = J.EP[c] + pep;
            J.DP[c] = dp;
            J.EP[c] = ep;
            J.DP64[c] = (uint64_t)(dp >> ks);
            J.EP64[c] = (uint64_t)(ep >> ks);
            const int f = J.FH[c];
            J.FH[c] = (f != FH_NONE) ? f : nxt;
        }
    }
}

// ---------------------------------------------------------------------------
// a4 + a5: split and pack.
//
// Tile events: light event x (x = 1..C) is the merge state just before the
// first light of tile x (key DP[x]; the last one, x = C, comes after every
// heavy); heavy event y (y = 1..C) is the state just after the last heavy of
// tile y-1 (key EP[y]).  Heavy event y precedes light event x iff
// EP[y] <= DP[x].  The 2C events in merge order cut the sweep into cells; in
// each cell the lights come from one tile and the heavies from one tile.
// Pack block b handles events [16 b, 16 b + 16).  k_split finds where each
// block starts (the paper's split(), on tile granularity); the block refines
// the exact state inside its first two tiles and merges cell by cell.
//
// Merge keys are 64-bit: the exact tile prefix shifted right by kshift (key
// unit 2^kshift / Q bucket, about 2 n 2^-62: 2^-33 at n = 2^28) plus, inside a
// tile, the item sizes rounded to that unit.  Every key is a deterministic
// function of the input and the keys of a tile are non-decreasing, so every
// block makes the same decisions and the cuts agree.  Inside a tile the
// rounding can move a key by at most half a unit per item before it; the merge
// then differs from the exact sweep only where a light's and a heavy's sums are
// that close, and a heavy's t by at most that much.  On small inputs the item
// sizes are exact multiples of the unit and the table equals the sweep's.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void k_split(JobTable jt) {
    __shared__ int s_job;
    int64_t lb;
    const JobDesc J = job_uniform(job_of_block(jt, lb, &s_job));
    if (J.sc->status != WRS_OK) return;
    const int64_t b = lb * TPB + threadIdx.x;
    if (b >= J.npack) return;
    glb(J.pstart)[b] = pack_start(J, b);
}

// Number of entries of key[0, len) that are <= v (LE) or < v (!LE), for
// ascending keys: a bisection whose trip count depends on len only (block-
// uniform), with every probe inside [0, len).
template <bool LE>
__device__ __forceinline__ int count_below(const uint64_t* key, int len, uint64_t v) {
    int base = 0;  // the count lies in [base, base + n]
    int n = len;
    while (n > 1) {
        const int half = n >> 1;
        const uint64_t k = key[base + half - 1];
        base += (LE ? k <= v : k < v) ? half : 0;
        n -= half;
    }
    if (len > 0) {
        const uint64_t k = key[base];
        base += (LE ? k <= v : k < v) ? 1 : 0;
    }
    return base;
}

// The two sides of the merge staged in LDS: the lights of tile x with the
// deficit sum before each as key, and the heavies of tile y with the excess
// sum through each.  Both come in index order from the partitioned copy of
// the tile that k_tileagg wrote.  An item is named by its offset inside the
// tile, or in list mode by its original index.
template <bool LIST> struct ItemId { typedef uint16_t type; };
template <> struct ItemId<true> { typedef uint32_t type; };

template <bool LIST>
struct LightSlot {
    uint64_t key[TILE];
    float t[TILE];        // a light's bucket keeps n w / W (at most 1)
    typename ItemId<LIST>::type id[TILE];
};

template <bool LIST>
struct HeavySlot {
    uint64_t key[TILE];
    typename ItemId<LIST>::type id[TILE];
};

template <bool LIST>
struct PackShared {
    LightSlot<LIST> A;
    HeavySlot<LIST> B;
    uint64_t tmp[TPB / 64];
    uint64_t dp[PACK_STEPS_MAX + 2];   // DP64[x0 + i]
    uint64_t ep[PACK_STEPS_MAX + 2];   // EP64[y0 + i]
    int32_t fh[PACK_STEPS_MAX + 2];    // FH[y0 + i]
    uint32_t nlx[PACK_STEPS_MAX + 2];  // NL[x0 + i]
    uint32_t nly[PACK_STEPS_MAX + 2];  // NL[y0 + i]
    int s_job;
};

// One side of a tile, loaded ahead of its fill: thread t holds the side's
// items [t k, t k + k), k = ceil(count / TPB).
struct SideFetch {
    float v[IPT];
    uint32_t o[IPT];
    uint64_t base;  // DP64[c] for the lights, EP64[c] for the heavies
    int cnt;        // items on this side
};

// side items [first, first + cnt) of the partitioned tile c.  Every lane
// loads each of the block-uniform k slots (a slot past cnt re-reads item
// cnt - 1), so the loads write their registers unmasked and nothing waits for
// them before the side is staged.
template <bool LIST>
__device__ __forceinline__ void fetch_side(const JobDesc& J, int64_t c, int first, int cnt, bool light,
                                           SideFetch& f) {
    f.cnt = cnt;
    f.base = 0;  // set from the window when the side is staged
    if (cnt == 0) return;
    const int k = uni((cnt + TPB - 1) / TPB);  // block-uniform: slots past it are skipped, not masked
    const int j0 = (int)threadIdx.x * k;
    const WRS_GLOBAL float* wp = glb(J.WP) + c * TILE + first;
    const WRS_GLOBAL uint16_t* po = glb(J.PO) + c * TILE + first;
    const WRS_GLOBAL uint32_t* pi = glb(J.PI) + c * TILE + first;
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        if (e < k) {
            const int j = min(j0 + e, cnt - 1);
            f.v[e] = wp[j];
            if constexpr (LIST) f.o[e] = pi[j]; else f.o[e] = po[j];
        }
    }
}


// Stage one side of a tile: keys are the tile's exact prefix plus the rounded
// sizes of the side's items before (lights) or through (heavies) each item.
// A light's t is computed here too.  List mode: a residual marker's size is
// its exact n-scaled size from lres, rounded to key units; a light marker's
// threshold comes from lresf where that array holds its size.
template <bool LIGHT, bool LIST, class Id>
__device__ __forceinline__ void fill_side(uint64_t* key, float* tl, Id* id, const SideFetch& f,
                                          const BuildScalars& sc, uint32_t n, double lscale,
                                          const u128* lres, const double* lresf, uint64_t* tmp) {
    const int k = uni((f.cnt + TPB - 1) / TPB);  // block-uniform: slots past it are skipped, not masked
    const int j0 = (int)threadIdx.x * k;
    const uint64_t Qk = sc.Qk;
    uint64_t inc[IPT];
    float tv[LIGHT ? IPT : 1];
    uint64_t sum = 0;
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        inc[e] = 0;
        if (e >= k) continue;
        if constexpr (!LIST) {
            // every lane computes the slot (a slot past the side holds a copy
            // of its last item) and a slot past the side adds 0
            const uint64_t z = size_keyunits(f.v[e], sc, n);
            if constexpr (LIGHT) tv[e] = fminf(light_t(f.v[e], lscale), 1.0f);
            const uint64_t d = LIGHT ? Qk - z : z - Qk;
            inc[e] = (j0 + e < f.cnt) ? d : 0ull;
            sum += inc[e];
        } else if (j0 + e < f.cnt) {
            uint64_t z;
            float t = 0.0f;
            if (is_residual_marker(__float_as_uint(f.v[e]))) {
                const uint32_t slot = residual_slot(__float_as_uint(f.v[e]));
                const u128 m = glb(lres)[slot];
                const int ks = sc.kshift;
                z = (uint64_t)(ks > 0 ? (m + ((u128)1 << (ks - 1))) >> ks : m);
                if (LIGHT) {
                    const double fs = lresf != nullptr ? glb(lresf)[slot] : -1.0;
                    t = (float)((fs >= 0.0 ? fs : u128_to_double(m)) * sc.rQ);
                }
            } else {
                z = size_keyunits(f.v[e], sc, n);
                if (LIGHT) t = light_t(f.v[e], lscale);
            }
            if constexpr (LIGHT) tv[e] = fminf(t, 1.0f);
            inc[e] = LIGHT ? Qk - z : z - Qk;
            sum += inc[e];
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t incl = wave_incl_scan(sum);
    if (lane == 63) tmp[wv] = incl;
    __syncthreads();  // also: every thread is done with the slot's previous contents
    uint64_t acc = f.base + incl - sum;
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w)
        if (w < wv) acc += tmp[w];
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        if (e < k) {
            // j < k TPB <= TILE: a slot past the side writes an entry that no
            // search or output reads
            const int j = j0 + e;
            if (LIST && j >= f.cnt) continue;
            if constexpr (LIGHT) {
                key[j] = acc;
                tl[j] = tv[e];
                acc += inc[e];
            } else {
                acc += inc[e];
                key[j] = acc;
            }
            id[j] = (Id)f.o[e];
        }
    }
    __syncthreads();
}





template <bool LIST>
__device__ __forceinline__ void pack_block(const JobDesc& J, int64_t lb, PackShared<LIST>& sh) {
    if (J.sc->status != WRS_OK) return;
    const BuildScalars sc = scalars_uniform(J.sc);
    const uint32_t n32 = J.nmul;
    const double lscale = sc.nscale * sc.rQ;
    const u128* lres = J.lres;
    const double* lresf = J.lresf;
    const int64_t C = J.ntiles;
    const int psteps = J.psteps;  // PACK_STEPS_MIN..PACK_STEPS_MAX
    const int64_t s0 = lb * psteps;
    const int64_t s1 = min(s0 + (int64_t)psteps, 2 * C);
    const int64_t x0 = glb(J.pstart)[lb];
    const int64_t y0 = s0 - x0;
    for (int i = threadIdx.x; i < psteps + 2; i += TPB) {
        const int64_t xi = x0 + i, yi = y0 + i;
        sh.dp[i] = (xi <= C) ? glb(J.DP64)[xi] : ~0ull;
        sh.ep[i] = (yi <= C) ? glb(J.EP64)[yi] : ~0ull;
        sh.fh[i] = (yi <= C) ? glb(J.FH)[yi] : FH_NONE;
        sh.nlx[i] = glb(J.NL)[min(xi, C)];
        sh.nly[i] = glb(J.NL)[min(yi, C)];
    }
    __syncthreads();
    // lights / heavies of tile c, from the window
    auto tile_cnt = [&](int64_t c) -> int { return (int)min((int64_t)TILE, J.n - c * TILE); };
    auto lights_of = [&](int64_t c) -> int {
        return c < C ? (int)(sh.nlx[c - x0 + 1] - sh.nlx[c - x0]) : 0;
    };
    auto heavies_of = [&](int64_t c) -> int {
        return c < C ? tile_cnt(c) - (int)(sh.nly[c - y0 + 1] - sh.nly[c - y0]) : 0;
    };
    SideFetch fa, fb;
    {
        const int la = lights_of(x0);
        fetch_side<LIST>(J, x0, 0, la, true, fa);
        const int hb = heavies_of(y0);
        fetch_side<LIST>(J, y0, y0 < C ? tile_cnt(y0) - hb : 0, hb, false, fb);
    }
    fa.base = sh.dp[0];
    fb.base = sh.ep[0];
    fill_side<true, LIST>(sh.A.key, sh.A.t, sh.A.id, fa, sc, n32, lscale, lres, lresf, sh.tmp);
    fill_side<false, LIST>(sh.B.key, (float*)nullptr, sh.B.id, fb, sc, n32, lscale, lres, lresf, sh.tmp);
    int nlx = fa.cnt, nhy = fb.cnt;
    int64_t x = x0, y = y0;
    // DPkey(x) < v, with DPkey(C) = +infinity
    auto dpkey_lt = [&](int64_t xx, uint64_t v) -> bool { return xx < C && sh.dp[xx - x0] < v; };
    int pl = 0, ph = 0;
    if (s0 > 0) {
        const bool last_light = x >= 1 && (y == 0 || !dpkey_lt(x, sh.ep[0]));  // EP[y] <= DPkey(x)
        if (last_light) {
            ph = (x < C) ? wave_search<true>(sh.B.key, 0, nhy, sh.dp[0]) : 0;
        } else {
            pl = wave_search<false>(sh.A.key, 0, nlx, sh.ep[0]);
        }
    }
    const double tscale = sc.tscale;
    const LightSlot<LIST>& A = sh.A;
    const HeavySlot<LIST>& B = sh.B;
    // original item of a staged entry: tile base + offset, or the list's index
    auto item = [&](int64_t tbase, uint32_t id) -> int64_t { return LIST ? (int64_t)id : tbase + id; };
    // A table index is a tile's base plus an offset that k_tileagg wrote for
    // an item of that tile, so it lies in [0, n) whatever the weights held
    // when each kernel read them.  The guard turns a violation into
    // WRS_EDEVICE instead of a stray write.  (List mode writes the original
    // indices of a list that the host's earlier stage built.)
    // (Selects, not a branch: a violation is recorded and the write goes to
    // entry n - 1 of a table whose build then fails.)
    bool bad = false;
    auto put = [&](int64_t own, float t, int32_t al) {
        if constexpr (!LIST) {
            const bool out = (uint64_t)own >= (uint64_t)J.n;
            bad |= out;
            own = out ? J.n - 1 : own;
        }
        store_entry(J.table, own, t, al);
    };
    for (int64_t s = s0; s < s1; ++s) {
        const int xi = (int)(x - x0), yi = (int)(y - y0);
        const bool has_h = y + 1 <= C;
        const bool has_l = x + 1 <= C;
        const uint64_t EPn = sh.ep[yi + 1];
        const bool heavy_ev = has_h && (!has_l || !dpkey_lt(x + 1, EPn));
        // the tile side this event opens: fetched now, staged after the merge
        const bool need = s + 1 < s1;
        SideFetch fn;
        if (need) {
            const int64_t cn = heavy_ev ? y + 1 : x + 1;
            const int hc = heavies_of(y + 1);
            const int cntn = heavy_ev ? hc : lights_of(x + 1);
            const int firstn = (heavy_ev && y + 1 < C) ? tile_cnt(y + 1) - hc : 0;
            fetch_side<LIST>(J, cn, firstn, cntn, !heavy_ev, fn);
        }
        const int64_t abase = x * TILE, bbase = y * TILE;
        int nlc, nhc;
        if (heavy_ev) {
            nhc = nhy - ph;
            nlc = wave_search<false>(A.key, pl, nlx, EPn) - pl;
        } else {
            nlc = nlx - pl;
            nhc = (y < C) ? wave_search<true>(B.key, ph, nhy, sh.dp[xi + 1]) - ph : 0;
        }
        const int32_t nextH = has_h ? sh.fh[yi + 1] : FH_NONE;
        const uint64_t Dend = (x < C) ? sh.dp[xi + 1] : sh.dp[xi];
        const int m = nlc + nhc;
        if (nhc == 0 && nlc > 0) {
            // lights only: all take the same alias; lanes take consecutive lights
            const bool hv = ph < nhy;
            const int32_t al = hv ? (int32_t)item(bbase, B.id[ph]) : nextH;
            for (int d = threadIdx.x; d < nlc; d += TPB) {
                const int lp = pl + d;
                const int64_t own = item(abase, A.id[lp]);
                const float t = A.t[lp];
                const int32_t a2 = (!hv && al == FH_NONE) ? (int32_t)own : al;
                put(own, t, a2);
            }
        } else if (nlc == 0 && nhc > 0) {
            // heavies only: each keeps 1 + (E - D) with the same next light
            const uint64_t Dn = (pl < nlx) ? A.key[pl] : Dend;
            for (int d = threadIdx.x; d < nhc; d += TPB) {
                const int hp = ph + d;
                const float t = heavy_t(B.key[hp], Dn, tscale);
                const int64_t own = item(bbase, B.id[hp]);
                const int32_t al = (hp + 1 < nhy) ? (int32_t)item(bbase, B.id[hp + 1])
                                                  : (nextH != FH_NONE ? nextH : (int32_t)own);
                put(own, t, al);
            }
        } else if (m > 0) {
            // Both kinds: every output takes its rank in the other side of the
            // cell.  A light comes after the cell's heavies whose key is at
            // most its own (ties put the heavy first), so it aliases the
            // heavy at that rank; a heavy comes after the cell's lights whose
            // key is below its own, so the next light is the one at that rank
            // (Dend past the tile's last light).  Lanes take consecutive
            // lights, then consecutive heavies.
            const int nlc_u = uni(nlc), nhc_u = uni(nhc);
            for (int d = threadIdx.x; d < m; d += TPB) {
                if (d < nlc_u) {
                    const int lp = pl + d;
                    const int r = count_below<true>(B.key + ph, nhc_u, A.key[lp]);
                    const int q = ph + r;
                    const int64_t own = item(abase, A.id[lp]);
                    const int32_t al = (q < nhy) ? (int32_t)item(bbase, B.id[min(q, TILE - 1)])
                                                 : (nextH != FH_NONE ? nextH : (int32_t)own);
                    put(own, A.t[lp], al);
                } else {
                    const int hp = ph + (d - nlc_u);
                    const uint64_t E = B.key[hp];
                    const int r = count_below<false>(A.key + pl, nlc_u, E);
                    const uint64_t Dn = (pl + r < nlx) ? A.key[min(pl + r, TILE - 1)] : Dend;
                    const int64_t own = item(bbase, B.id[hp]);
                    const int32_t al = (hp + 1 < nhy) ? (int32_t)item(bbase, B.id[min(hp + 1, TILE - 1)])
                                                      : (nextH != FH_NONE ? nextH : (int32_t)own);
                    put(own, heavy_t(E, Dn, tscale), al);
                }
            }
        }
        pl += nlc;
        ph += nhc;
        if (heavy_ev) {
            ++y;
            ph = 0;
            if (need) {
                fn.base = sh.ep[y - y0];
                fill_side<false, LIST>(sh.B.key, (float*)nullptr, sh.B.id, fn, sc, n32, lscale, lres, lresf, sh.tmp);
                nhy = fn.cnt;
            }
        } else {
            ++x;
            pl = 0;
            if (need) {
                fn.base = sh.dp[x - x0];
                fill_side<true, LIST>(sh.A.key, sh.A.t, sh.A.id, fn, sc, n32, lscale, lres, lresf, sh.tmp);
                nlx = fn.cnt;
            }
        }
    }
    if (!LIST && __ballot(bad) != 0 && (threadIdx.x & 63) == 0) glb(J.sc)->status = WRS_EDEVICE;
}

template <bool LIST>
__global__ __launch_bounds__(TPB) void k_pack(JobTable jt) {
    __shared__ PackShared<LIST> sh;
    int64_t lb;
    const JobDesc J = job_uniform(job_of_block(jt, lb, &sh.s_job, xcd_contiguous_block()));
    pack_block<LIST>(J, lb, sh);
}

// ---------------------------------------------------------------------------
// a6: alias queries (Section 2.2 query; select without a branch as in Section 10).
// ---------------------------------------------------------------------------
// Bucket r in [0, n) and coin u in [0, 1) of the draw with counter c: one
// Philox block; r = floor((x1 2^32 + x0) n / 2^64) for n < 2^31, u from 24 bits.
__device__ __forceinline__ void draw_of(uint64_t c, uint32_t sid, uint32_t k0, uint32_t k1, uint64_t n, uint32_t& r,
                                        float& u) {
    const uint4 x = philox4x32_10(make_uint4((uint32_t)c, (uint32_t)(c >> 32), sid, 0u), k0, k1);
    const uint64_t lo = ((uint64_t)x.x * n) >> 32;
    const uint64_t hi = (uint64_t)x.y * n + lo;
    r = (uint32_t)(hi >> 32);
    u = (float)(x.z >> 8) * (1.0f / 16777216.0f);
}

__global__ __launch_bounds__(SAMPLE_TPB) void k_sample(JobTable jt) {
    __shared__ int s_job;
    int64_t lb;
    // XCD-contiguous block order: a job's blocks share one or two L2s, so a
    // small table stays in the L2 of the XCDs that sample it
    const JobDesc J = job_uniform(job_of_block(jt, lb, &s_job, xcd_contiguous_block()));
    if (J.sc != nullptr && J.sc->status != WRS_OK) return;
    const int64_t k = J.k;
    const uint64_t n = (uint64_t)J.n;
    const uint32_t k0 = (uint32_t)J.seed, k1 = (uint32_t)(J.seed >> 32);
    const WRS_GLOBAL uint64_t* table = (const WRS_GLOBAL uint64_t*)glb(J.table);
    const int U = J.sunroll;  // 1..SAMPLE_UNROLL_MAX draws per thread
    const int64_t s0 = lb * (int64_t)(SAMPLE_TPB * U) + threadIdx.x;
    uint32_t r[SAMPLE_UNROLL_MAX];
    float u[SAMPLE_UNROLL_MAX];
#pragma unroll
    for (int e = 0; e < SAMPLE_UNROLL_MAX; ++e) {
        if (e < U) {
            const int64_t s = s0 + (int64_t)e * SAMPLE_TPB;
            draw_of(J.first_counter + (uint64_t)s, J.stream_id, k0, k1, n, r[e], u[e]);
        }
    }
    uint64_t ent[SAMPLE_UNROLL_MAX];
#pragma unroll
    for (int e = 0; e < SAMPLE_UNROLL_MAX; ++e) {
        if (e < U) {
            const int64_t s = s0 + (int64_t)e * SAMPLE_TPB;
            ent[e] = (s < k) ? table[r[e]] : 0ull;  // cached: small tables stay in L2 / MALL
        }
    }
#pragma unroll
    for (int e = 0; e < SAMPLE_UNROLL_MAX; ++e) {
        const int64_t s = s0 + (int64_t)e * SAMPLE_TPB;
        if (e < U && s < k) {
            const float t = __uint_as_float((uint32_t)ent[e]);
            const int32_t a = (int32_t)(uint32_t)(ent[e] >> 32);
            glb(J.out)[s] = (u[e] < t) ? (int32_t)r[e] : a;
        }
    }
}

// ---------------------------------------------------------------------------
// Small batched tables (n <= FUSE_MAX): one persistent launch in which a
// workgroup takes a job at a time through every phase above (the same block
// bodies, one after another, with a barrier between phases), then copies the
// finished table into LDS and draws the job's samples from there.  A job's
// table and draws are the ones its single calls give, bit for bit: each phase
// computes the same values whichever workgroup runs its blocks, and draw s is
// a function of its counter alone.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void k_fused_small(JobTable jt, const int32_t* small, int32_t nsmall) {
    __shared__ union FusedShared {
        RedShared r;
        TileaggShared<false> t;
        ScanSegShared s;
        PackShared<false> p;
    } u;
    __shared__ uint64_t s_tab[FUSE_MAX];
    for (int32_t q = (int32_t)blockIdx.x; q < nsmall; q += (int32_t)gridDim.x) {
        const JobDesc J = job_uniform(jt.jobs[glb(small)[q]]);
        // one block of each phase whose job size allows one (n <= FUSE_MAX:
        // one reduction block, one scan segment), every block of the others
        reduce_block(J, 0, u.r);
        __syncthreads();
        for (int64_t lb = 0; lb < cdiv(J.ntiles, TILES_PER_AGG_BLOCK); ++lb) {
            tileagg_block<false>(J, lb, u.t);
            __syncthreads();
        }
        scan_seg_block(J, 0, u.s);
        __syncthreads();
        for (int64_t lb = 0; lb < J.npack; ++lb) {
            pack_block<false>(J, lb, u.p);
            __syncthreads();
        }
        const bool ok = uni((uint32_t)glb(J.sc)->status) == (uint32_t)WRS_OK;
        if (ok && J.k > 0) {
            const WRS_GLOBAL uint64_t* table = (const WRS_GLOBAL uint64_t*)glb(J.table);
            for (int64_t i = threadIdx.x; i < J.n; i += TPB) s_tab[i] = table[i];
            __syncthreads();
            const uint32_t k0 = (uint32_t)J.seed, k1 = (uint32_t)(J.seed >> 32);
            for (int64_t s = threadIdx.x; s < J.k; s += TPB) {
                uint32_t r;
                float uu;
                draw_of(J.first_counter + (uint64_t)s, J.stream_id, k0, k1, (uint64_t)J.n, r, uu);
                const uint64_t ent = s_tab[r];
                const float t = __uint_as_float((uint32_t)ent);
                const int32_t a = (int32_t)(uint32_t)(ent >> 32);
                glb(J.out)[s] = (uu < t) ? (int32_t)r : a;
            }
        }
        __syncthreads();  // before the next job reuses the LDS
    }
}

hipError_t launch_fused_small(const JobTable& jt, const int32_t* d_small, int32_t nsmall, hipStream_t st) {
    if (nsmall <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fused_small, dim3((unsigned)min(nsmall, FUSE_BLOCKS)), dim3(TPB), 0, st, jt, d_small, nsmall);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
void set_sample_job(JobDesc& J, int64_t k, int32_t sunroll) {
    J.k = k;
    J.sunroll = sunroll > 0 ? sunroll : sample_unroll_for(k);
}

int64_t sample_blocks(const JobDesc& J) {
    return J.k > 0 ? cdiv(J.k, (int64_t)SAMPLE_TPB * J.sunroll) : 0;
}

void phase_blocks(const JobDesc& J, int64_t b[PH_COUNT]) {
    b[PH_RED] = J.nred;
    b[PH_FIN] = J.nred > 1 ? 1 : 0;  // one reduction block finalizes in place
    b[PH_TILE] = cdiv(J.ntiles, TILES_PER_AGG_BLOCK);
    b[PH_SEG] = J.nseg;
    // one segment: k_scan_seg finishes the scan itself
    b[PH_TOP] = J.nseg > 1 ? 1 : 0;
    b[PH_FIX] = J.nseg > 1 ? J.nseg : 0;
    b[PH_SPLIT] = J.nseg > 1 ? cdiv(J.npack, TPB) : 0;
    b[PH_PACK] = J.npack;
    b[PH_SAMPLE] = sample_blocks(J);
}

hipError_t launch_build(const JobTable& jt0, const int64_t* blocks, hipStream_t st, bool list) {
    JobTable jt = jt0;
#define WRS_LAUNCH(kern, ph)                                                       \
    do {                                                                           \
        if (blocks[ph] > 0) {                                                      \
            jt.phase = ph;                                                         \
            hipLaunchKernelGGL(kern, dim3((unsigned)blocks[ph]), dim3(TPB), 0, st, jt); \
            hipError_t e_ = hipGetLastError();                                     \
            if (e_ != hipSuccess) return e_;                                       \
        }                                                                          \
    } while (0)
    WRS_LAUNCH(k_reduce, PH_RED);
    WRS_LAUNCH(k_finalize, PH_FIN);
    if (list) WRS_LAUNCH(k_tileagg<true>, PH_TILE); else WRS_LAUNCH(k_tileagg<false>, PH_TILE);
    WRS_LAUNCH(k_scan_seg, PH_SEG);
    WRS_LAUNCH(k_scan_top, PH_TOP);
    WRS_LAUNCH(k_scan_fix, PH_FIX);
    WRS_LAUNCH(k_split, PH_SPLIT);
    if (list) WRS_LAUNCH(k_pack<true>, PH_PACK); else WRS_LAUNCH(k_pack<false>, PH_PACK);
#undef WRS_LAUNCH
    return hipSuccess;
}

// Status word of every job of a job table, gathered into d_dst[0..njobs).
__global__ __launch_bounds__(TPB) void k_collect_status(JobTable jt, int32_t* d_dst) {
    for (int j = (int)(blockIdx.x * TPB + threadIdx.x); j < jt.njobs; j += (int)(gridDim.x * TPB))
        d_dst[j] = jt.jobs[j].sc->status;
}

hipError_t launch_collect_status(const JobTable& jt, int32_t* d_dst, hipStream_t st) {
    if (jt.njobs < 1) return hipSuccess;
    hipLaunchKernelGGL(k_collect_status, dim3((unsigned)cdiv(jt.njobs, TPB)), dim3(TPB), 0, st, jt, d_dst);
    return hipGetLastError();
}

hipError_t launch_sample(const JobTable& jt0, int64_t blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    JobTable jt = jt0;
    jt.phase = PH_SAMPLE;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)blocks), dim3(SAMPLE_TPB), 0, st, jt);
    return hipGetLastError();
}

}  // namespace wrs
