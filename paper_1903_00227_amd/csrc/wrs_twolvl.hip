// wrs_twolvl.hip -- 2-level alias tables (Section 4.4, replicated top level).
//
// The items are cut into blocks of GTILE consecutive items; block b is a
// meta-item of weight W_b.  Every block gets its own alias table over its m
// items, built by one workgroup as the complete sweep of Section 4.1 with the
// block as the instance (bucket capacity W_b / m): in n-scaled grid integers,
// item j of the block has size m q_j and the bucket holds S_b = sum of the
// block's q (exact, u128).  Keys are 64-bit key units of that block's own
// scale, as in the tile merge.  The tables are stored in place with global
// item indices.  The meta-items then go through the splitting construction in
// list mode, each as a residual marker carrying its exact G-scaled size G S_b
// (G = number of blocks), which gives the top-level table over the blocks.
// The top job keeps the items' grid (exponent and capacity Q), with only the
// count-dependent scalars derived for G items, so those sizes are exact.
// A block far lighter than the total (its sum below 2^40 units of that grid)
// builds its own table on a finer grid of its own, set by its largest weight,
// and gives the top level its size as a double for the meta-item's light
// threshold: on the items' grid its sum would keep too few bits for a
// relative error below 1e-6 (and be 0 for a block below the grid).
// A query draws a block from the top table, then an item from the block's
// table: the second level's table holds global indices, and the top table is
// G entries (a few MB at most, resident in L2).
#include "wrs_device.h"

namespace wrs {

struct TwoShared {
    uint64_t key[GTILE];  // lights' keys at [0, nL), heavies' at [nL, nL + nH)
    float t[GTILE];       // a light's t
    uint16_t off[GTILE];  // offset in the block of each entry
    uint64_t d64[2][GTPB / 64];
    uint32_t d32[GTPB / 64];
    u128 d128[GTPB / 64];
    int32_t emx[GTPB / 64];
};

__device__ __forceinline__ int bitlen_u128(u128 v) {
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    return hi ? 128 - __clzll((long long)hi) : (lo ? 64 - __clzll((long long)lo) : 0);
}

__global__ __launch_bounds__(GTPB) void k_twolvl(JobDesc J, TwoLayout T) {
    __shared__ TwoShared sh;
    if (J.sc->status != WRS_OK) return;  // the same for every block
    const BuildScalars sc = scalars_uniform(J.sc);
    const int64_t n = J.n;
    const uint32_t g = blockIdx.x;
    const uint32_t nblocks = gridDim.x;
    const int64_t base = (int64_t)g * GTILE;
    const int m = (int)min((int64_t)GTILE, n - base);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int i0 = tid * GIPT;
    const WRS_GLOBAL float* w = glb(J.w) + base;
    float v[GIPT];
    if (m == GTILE && (((uintptr_t)w) & 15) == 0) {
        const vfloat4 a = *(const WRS_GLOBAL vfloat4*)(w + i0);
        const vfloat4 b = *(const WRS_GLOBAL vfloat4*)(w + i0 + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < GIPT; ++k) v[k] = (i0 + k < m) ? w[i0 + k] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < GIPT; ++k) v[k] = canonical_weight(v[k]);
    const int G = sc.G;
    // the block's exact sum S_b (every thread gets it)
    u128 s = 0;
#pragma unroll
    for (int k = 0; k < GIPT; ++k) s += quantize(v[k], G);  // items past the end hold 0
    const u128 ws = wave_incl_scan(s);
    if (lane == 63) sh.d128[wv] = ws;
    __syncthreads();
    u128 S = 0;
#pragma unroll
    for (int q = 0; q < GTPB / 64; ++q) S += sh.d128[q];
    const u128 Sg = S;  // on the items' grid: the meta-item's size
    // The grid of the block's own table: the items' grid, or for a block whose
    // sum is below 2^40 units of it, the grid Gq = e - 226 set by the largest
    // weight's biased exponent e, which puts every size below 2^100 and m S
    // below 2^122 (a weight more than 2^76 below the largest is rounded on it).
    int Gq = G;
    if ((uint64_t)(Sg >> 64) == 0 && (uint64_t)Sg < (1ull << 40)) {  // the same for the whole block
        int e = 0;
#pragma unroll
        for (int k = 0; k < GIPT; ++k) e = max(e, (int)(__float_as_uint(v[k]) >> 23));
        const int we = -wave_incl_min(-e);  // lane 63: the wave's largest
        if (lane == 63) sh.emx[wv] = we;
        __syncthreads();  // also: every thread has read d128 above
        int emax = 0;
#pragma unroll
        for (int q = 0; q < GTPB / 64; ++q) emax = max(emax, sh.emx[q]);
        const int Gb = max(emax, 1) - 226;
        if (Gb < G) {
            Gq = Gb;
            u128 s2 = 0;
#pragma unroll
            for (int k = 0; k < GIPT; ++k) s2 += quantize(v[k], Gb);
            const u128 ws2 = wave_incl_scan(s2);
            if (lane == 63) sh.d128[wv] = ws2;
            __syncthreads();
            S = 0;
#pragma unroll
            for (int q = 0; q < GTPB / 64; ++q) S += sh.d128[q];
        }
    }
    if (tid == 0) {  // the meta-item: a marker with its exact G-scaled size
        glb(T.lidx)[g] = g;
        glb(T.lw)[g] = __uint_as_float(residual_marker(g));
        glb(T.lres)[g] = (u128)nblocks * Sg;
        glb(T.lresf)[g] = Gq < G ? (double)nblocks * ldexp(u128_to_double(S), Gq - G) : -1.0;
    }
    if (S == 0) {  // a block of weight 0: every bucket keeps its item (never drawn)
#pragma unroll
        for (int k = 0; k < GIPT; ++k)
            if (i0 + k < m) store_entry(J.table, base + i0 + k, 1.0f, (int32_t)(base + i0 + k));
        return;  // the same for the whole block
    }
    // the block's own scale: sizes m q, bucket S, keys >> ks below 2^62
    const u128 mS = (u128)(uint32_t)m * S;
    const int ks = max(0, bitlen_u128(mS) - 62);
    const u128 half = ks > 0 ? ((u128)1 << (ks - 1)) : (u128)0;
    const uint64_t Qk = (uint64_t)((S + half) >> ks);
    const double Sd = u128_to_double(S);
    const double tscale = ldexp(1.0, ks) / Sd;
    const double lscale = ldexp((double)m, -Gq) / Sd;
    uint32_t lbits = 0, hbits = 0;
    uint64_t z[GIPT];
    uint64_t sD = 0, sE = 0;
    uint32_t cL = 0, cH = 0;
#pragma unroll
    for (int k = 0; k < GIPT; ++k) {
        const bool valid = i0 + k < m;
        const u128 mq = (u128)(uint32_t)m * quantize(v[k], Gq);
        const bool light = valid && mq <= S;
        const bool heavy = valid && !light;
        z[k] = (uint64_t)((mq + half) >> ks);
        lbits |= (uint32_t)light << k;
        hbits |= (uint32_t)heavy << k;
        sD += light ? Qk - z[k] : 0ull;  // a light's size is at most the bucket, also in key units
        sE += heavy ? z[k] - Qk : 0ull;
        cL += light;
        cH += heavy;
    }
    const uint32_t pc = cL | (cH << 16);
    const uint64_t iD = wave_incl_scan(sD), iE = wave_incl_scan(sE);
    const uint32_t iC = wave_incl_scan(pc);
    __syncthreads();  // d128 read by every thread above
    if (lane == 63) {
        sh.d64[0][wv] = iD;
        sh.d64[1][wv] = iE;
        sh.d32[wv] = iC;
    }
    __syncthreads();
    uint64_t pD = 0, pE = 0, Dt = 0;
    uint32_t pC = 0, tC = 0;
#pragma unroll
    for (int q = 0; q < GTPB / 64; ++q) {
        const uint64_t a = sh.d64[0][q], b = sh.d64[1][q];
        const uint32_t c = sh.d32[q];
        if (q < wv) {
            pD += a;
            pE += b;
            pC += c;
        }
        Dt += a;
        tC += c;
    }
    const int nL = (int)(tC & 0xFFFFu), nH = (int)(tC >> 16);
    {
        const uint32_t exC = pC + iC - pc;
        uint64_t D = pD + iD - sD, E = pE + iE - sE;
        int rl = (int)(exC & 0xFFFFu), rh = (int)(exC >> 16);
#pragma unroll
        for (int k = 0; k < GIPT; ++k) {
            if ((lbits >> k) & 1u) {
                sh.key[rl] = D;
                sh.t[rl] = fminf(light_t(v[k], lscale), 1.0f);
                sh.off[rl] = (uint16_t)(i0 + k);
                D += Qk - z[k];
                ++rl;
            } else if ((hbits >> k) & 1u) {
                E += z[k] - Qk;
                sh.key[nL + rh] = E;
                sh.off[nL + rh] = (uint16_t)(i0 + k);
                ++rh;
            }
        }
    }
    __syncthreads();
    // the whole sweep of the block: merge path over every light and heavy.
    // A light takes the next heavy not yet packed, a heavy the heavy after it;
    // with none left (the end of the sweep) the bucket aliases its own item.
    const uint64_t* A = sh.key;
    const uint64_t* B = sh.key + nL;
    const int d0 = (int)(((int64_t)m * tid) / GTPB);
    const int d1 = (int)(((int64_t)m * (tid + 1)) / GTPB);
    if (d1 > d0) {
        int jlo = max(0, d0 - nL), jhi = min(d0, nH);
        while (jlo < jhi) {
            const int mid = (jlo + jhi + 1) >> 1;
            const bool ok = (d0 - mid >= nL) || (B[mid - 1] <= A[d0 - mid]);
            if (ok) jlo = mid; else jhi = mid - 1;
        }
        int j = jlo, i = d0 - jlo;
        uint64_t kb = (j < nH) ? B[j] : ~0ull;
        uint64_t ka = (i < nL) ? A[i] : Dt;
        for (int d = d0; d < d1; ++d) {
            const bool take_h = (j < nH) && (i >= nL || kb <= ka);
            // take_h: j < nH; else i < nL (d < m), so both reads stay inside the block
            const int own = take_h ? sh.off[nL + j] : sh.off[min(i, GTILE - 1)];
            const int q = j + (take_h ? 1 : 0);
            const int32_t al = (int32_t)(base + ((q < nH) ? sh.off[nL + q] : own));
            const float t = take_h ? heavy_t(kb, ka, tscale) : sh.t[min(i, GTILE - 1)];
            store_entry(J.table, base + own, t, al);
            if (take_h) {
                ++j;
                kb = (j < nH) ? B[j] : ~0ull;
            } else {
                ++i;
                ka = (i < nL) ? A[i] : Dt;
            }
        }
    }
}

// Two-step query: the top table picks the block, the block's table the item.
constexpr int S2_IPT = 4;

__global__ __launch_bounds__(SAMPLE_TPB) void k_sample2(const wrs_entry* top, const wrs_entry* table, int64_t n,
                                                        uint64_t seed, uint32_t sid, uint64_t first, int64_t k,
                                                        int32_t* out) {
    const uint64_t G = (uint64_t)cdiv(n, GTILE);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int64_t s0 = (int64_t)xcd_contiguous_block() * (SAMPLE_TPB * S2_IPT) + threadIdx.x;
    const WRS_GLOBAL uint64_t* Tt = (const WRS_GLOBAL uint64_t*)glb(top);
    const WRS_GLOBAL uint64_t* Tb = (const WRS_GLOBAL uint64_t*)glb(table);
    uint32_t gsel[S2_IPT];
#pragma unroll
    for (int e = 0; e < S2_IPT; ++e) {
        const int64_t s = s0 + (int64_t)e * SAMPLE_TPB;
        gsel[e] = 0;
        if (s < k) {
            const uint64_t c = first + (uint64_t)s;
            const uint4 x = philox4x32_10(make_uint4((uint32_t)c, (uint32_t)(c >> 32), sid, 0u), k0, k1);
            const uint64_t lo = ((uint64_t)x.x * G) >> 32;
            const uint32_t r = (uint32_t)(((uint64_t)x.y * G + lo) >> 32);
            const float u = (float)(x.z >> 8) * (1.0f / 16777216.0f);
            const uint64_t ent = Tt[r];
            gsel[e] = (u < __uint_as_float((uint32_t)ent)) ? r : (uint32_t)(ent >> 32);
        }
    }
#pragma unroll
    for (int e = 0; e < S2_IPT; ++e) {
        const int64_t s = s0 + (int64_t)e * SAMPLE_TPB;
        if (s < k) {
            const uint64_t c = first + (uint64_t)s;
            const uint4 y = philox4x32_10(make_uint4((uint32_t)c, (uint32_t)(c >> 32), sid, 2u), k0, k1);
            const int64_t b0 = (int64_t)gsel[e] * GTILE;
            const uint64_t m = (uint64_t)min((int64_t)GTILE, n - b0);
            const uint64_t lo = ((uint64_t)y.x * m) >> 32;
            const uint32_t r = (uint32_t)(((uint64_t)y.y * m + lo) >> 32);
            const float u = (float)(y.z >> 8) * (1.0f / 16777216.0f);
            const uint64_t ent = Tb[b0 + r];
            glb(out)[s] = (u < __uint_as_float((uint32_t)ent)) ? (int32_t)(b0 + r) : (int32_t)(uint32_t)(ent >> 32);
        }
    }
}

hipError_t launch_twolvl(const JobDesc& J, const TwoLayout& T, hipStream_t st) {
    const int64_t nb = cdiv(J.n, GTILE);
    hipLaunchKernelGGL(k_twolvl, dim3((unsigned)nb), dim3(GTPB), 0, st, J, T);
    return hipGetLastError();
}

hipError_t launch_sample2(const wrs_entry* top, const wrs_entry* table, int64_t n, uint64_t seed, uint32_t sid,
                          uint64_t first, int64_t k, int32_t* out, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    const int64_t blocks = cdiv(k, (int64_t)SAMPLE_TPB * S2_IPT);
    hipLaunchKernelGGL(k_sample2, dim3((unsigned)blocks), dim3(SAMPLE_TPB), 0, st, top, table, n, seed, sid, first,
                       k, out);
    return hipGetLastError();
}

}  // namespace wrs
