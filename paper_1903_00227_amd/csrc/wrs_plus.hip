// wrs_plus.hip -- greedy blocks before the splitting construction (PSA+).
//
// Section 4.2.1: before splitting, consecutive ranges of items are assigned
// greedily.  Here a block of GTILE items is one workgroup.  It runs the sweep
// of Section 4.1 on its own items, as the same merge the tile kernels use
// (lights keyed by the deficit before them, heavies by the excess through
// them, a heavy first on ties), and stops where the sequential sweep would
// need a light or a next heavy that the block does not have:
//   - out of lights (excess Et > deficit Dt): every light and the heavies
//     with excess sum at most Dt are packed.  The first heavy past Dt is left
//     with the part of its size not yet placed (still above a bucket), and
//     the heavies after it are left untouched.
//   - out of heavies (Et <= Dt): the lights whose deficit before them is below
//     Et, and every heavy but the last, are packed.  The last heavy is left
//     with what remains of it (at most a bucket, so it continues as a light),
//     and the later lights are left untouched.
//   - a block without lights or without heavies packs nothing.
// Packed buckets are final and written to the table at once.  The items left
// are written to the block's staging area in index order: a residual item as
// a marker naming its block, whose exact n-scaled size n S - F Q (S the sum of
// q over every item of the block not left untouched, F the buckets packed) is
// stored beside it.  A prefix over the blocks' counts and a compaction then
// give the list that the splitting construction processes in list mode.
//
// Keys are 64-bit key units as in k_pack (sizes rounded to 2^kshift of the
// exact n-scaled grid), so the packed buckets follow the exact sweep except
// where a light's and a heavy's sums lie within that rounding; the residual
// sizes themselves are exact.
#include "wrs_device.h"

namespace wrs {

struct GreedyShared {
    uint64_t key[GTILE];  // lights' keys at [0, nL), heavies' at [nL, nL + nH)
    float t[GTILE];       // a light's t
    uint16_t off[GTILE];  // offset in the block of each entry
    uint64_t d64[2][GTPB / 64];
    uint32_t d32[2][GTPB / 64];
    u128 d128[GTPB / 64];
};

__global__ __launch_bounds__(GTPB) void k_greedy(JobDesc J, PlusLayout P) {
    __shared__ GreedyShared sh;
    if (J.sc->status != WRS_OK) return;  // the same for every block
    const BuildScalars sc = scalars_uniform(J.sc);
    const int64_t n = J.n;
    const uint32_t n32 = J.nmul;
    const uint32_t g = blockIdx.x;
    const int64_t base = (int64_t)g * GTILE;
    const int cnt = (int)min((int64_t)GTILE, n - base);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int i0 = tid * GIPT;  // this thread's items, in index order
    const WRS_GLOBAL float* w = glb(J.w) + base;
    float v[GIPT];
    if (cnt == GTILE && (((uintptr_t)w) & 15) == 0) {
        const vfloat4 a = *(const WRS_GLOBAL vfloat4*)(w + i0);
        const vfloat4 b = *(const WRS_GLOBAL vfloat4*)(w + i0 + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < GIPT; ++k) v[k] = (i0 + k < cnt) ? w[i0 + k] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < GIPT; ++k) v[k] = canonical_weight(v[k]);
    // classify; sizes in key units; per-thread sums
    const uint32_t wthr = sc.wthr;
    const uint64_t Qk = sc.Qk;
    uint32_t lbits = 0, hbits = 0;
    uint64_t z[GIPT];
    uint64_t sD = 0, sE = 0;
    uint32_t cL = 0, cH = 0;
#pragma unroll
    for (int k = 0; k < GIPT; ++k) {
        const bool valid = i0 + k < cnt;
        const bool light = valid && __float_as_uint(v[k]) < wthr;
        const bool heavy = valid && !light;
        z[k] = size_keyunits(v[k], sc, n32);
        lbits |= (uint32_t)light << k;
        hbits |= (uint32_t)heavy << k;
        sD += light ? Qk - z[k] : 0ull;
        sE += heavy ? z[k] - Qk : 0ull;
        cL += light;
        cH += heavy;
    }
    // block-wide exclusive prefixes: deficit, excess, light and heavy ranks
    const uint32_t pc = cL | (cH << 16);  // at most GTILE each: no carry
    const uint64_t iD = wave_incl_scan(sD), iE = wave_incl_scan(sE);
    const uint32_t iC = wave_incl_scan(pc);
    if (lane == 63) {
        sh.d64[0][wv] = iD;
        sh.d64[1][wv] = iE;
        sh.d32[0][wv] = iC;
    }
    __syncthreads();
    uint64_t pD = 0, pE = 0, Dt = 0, Et = 0;
    uint32_t pC = 0, tC = 0;
#pragma unroll
    for (int q = 0; q < GTPB / 64; ++q) {
        const uint64_t a = sh.d64[0][q], b = sh.d64[1][q];
        const uint32_t c = sh.d32[0][q];
        if (q < wv) {
            pD += a;
            pE += b;
            pC += c;
        }
        Dt += a;
        Et += b;
        tC += c;
    }
    const int nL = (int)(tC & 0xFFFFu), nH = (int)(tC >> 16);
    const uint32_t exC = pC + iC - pc;
    const int rl0 = (int)(exC & 0xFFFFu), rh0 = (int)(exC >> 16);
    {
        uint64_t D = pD + iD - sD, E = pE + iE - sE;
        int rl = rl0, rh = rh0;
        const double lscale = sc.nscale * sc.rQ;
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
    // where the sweep stops (every wave computes the same values)
    const uint64_t* A = sh.key;
    const uint64_t* B = sh.key + nL;
    int nLf = 0, nHf = 0;      // lights / heavies packed (the first ones of each kind)
    int ul_from = 0, uh_from = 0;  // lights / heavies of rank >= these are left untouched
    int rho = -1;              // heavy rank of the residual item, if any
    if (nH > 0 && nL > 0) {
        if (Et > Dt) {
            const int js = wave_search<true>(B, 0, nH, Dt);  // heavies with excess sum <= Dt
            nLf = nL;
            nHf = js;
            rho = js;
            ul_from = nL;
            uh_from = js + 1;
        } else {
            const int is = wave_search<false>(A, 0, nL, Et);  // lights with deficit before them < Et
            nLf = is;
            nHf = nH - 1;
            rho = nH - 1;
            ul_from = is;
            uh_from = nH;
        }
    }
    // packed buckets: merge path over (lights [0, nLf), heavies [0, nHf))
    const int m = nLf + nHf;
    if (m > 0) {
        const int d0 = (int)(((int64_t)m * tid) / GTPB);
        const int d1 = (int)(((int64_t)m * (tid + 1)) / GTPB);
        if (d1 > d0) {
            int jlo = max(0, d0 - nLf), jhi = min(d0, nHf);
            while (jlo < jhi) {
                const int mid = (jlo + jhi + 1) >> 1;
                const bool ok = (d0 - mid >= nLf) || (B[mid - 1] <= A[d0 - mid]);
                if (ok) jlo = mid; else jhi = mid - 1;
            }
            int j = jlo, i = d0 - jlo;
            // keys at the cursors (the next heavy to pack, the deficit before
            // the next light, Dt past the last light), and the key after each
            // cursor read ahead, so no step waits for an LDS read
            uint64_t kb = (j < nHf) ? B[j] : ~0ull;
            uint64_t ka = (i < nL) ? A[i] : Dt;
            uint64_t nb = (j + 1 < nHf) ? B[j + 1] : ~0ull;
            uint64_t na = (i + 1 < nL) ? A[i + 1] : Dt;
            const double tscale = sc.tscale;
            for (int d = d0; d < d1; ++d) {
                const bool take_h = (j < nHf) && (i >= nLf || kb <= ka);
                // j <= nHf <= nH - 1 and i <= nL, so every read below is inside the block
                const int own = take_h ? sh.off[nL + j] : sh.off[min(i, GTILE - 1)];
                const int q = j + (take_h ? 1 : 0);  // a packed bucket's alias: the next heavy
                const int32_t al = (int32_t)(base + sh.off[nL + q]);
                const float t = take_h ? heavy_t(kb, ka, tscale) : sh.t[min(i, GTILE - 1)];
                store_entry(J.table, base + own, t, al);
                if (take_h) {
                    ++j;
                    kb = nb;
                    nb = (j + 1 < nHf) ? B[j + 1] : ~0ull;
                } else {
                    ++i;
                    ka = na;
                    na = (i + 1 < nL) ? A[i + 1] : Dt;
                }
            }
        }
    }
    // items left, in index order; exact sum of q over the items not untouched
    uint32_t lflag = 0, rflag = 0;
    u128 S = 0;
    {
        int rl = rl0, rh = rh0;
        const int G = sc.G;
#pragma unroll
        for (int k = 0; k < GIPT; ++k) {
            bool untouched = false, res = false;
            if ((lbits >> k) & 1u) {
                untouched = rl >= ul_from;
                ++rl;
            } else if ((hbits >> k) & 1u) {
                untouched = rh >= uh_from;
                res = rh == rho;
                ++rh;
            }
            lflag |= (uint32_t)(untouched || res) << k;
            rflag |= (uint32_t)res << k;
            if (i0 + k < cnt && !untouched) S += quantize(v[k], G);
        }
    }
    const uint32_t nlt = (uint32_t)__popc(lflag);
    const uint32_t iLt = wave_incl_scan(nlt);
    const u128 iS = wave_incl_scan(S);
    if (lane == 63) {
        sh.d32[1][wv] = iLt;
        sh.d128[wv] = iS;
    }
    __syncthreads();
    uint32_t pL = 0, tL = 0;
    u128 tS = 0;
#pragma unroll
    for (int q = 0; q < GTPB / 64; ++q) {
        const uint32_t c = sh.d32[1][q];
        if (q < wv) pL += c;
        tL += c;
        tS += sh.d128[q];
    }
    {
        uint32_t pos = pL + iLt - nlt;
        WRS_GLOBAL uint32_t* si = glb(P.sidx) + base;
        WRS_GLOBAL float* sw = glb(P.sw) + base;
#pragma unroll
        for (int k = 0; k < GIPT; ++k) {
            if ((lflag >> k) & 1u) {
                si[pos] = (uint32_t)(base + i0 + k);
                sw[pos] = ((rflag >> k) & 1u) ? __uint_as_float(residual_marker(g)) : v[k];
                ++pos;
            }
        }
    }
    if (tid == 0) {
        const uint32_t F = (uint32_t)cnt - tL;  // buckets packed here
        glb(P.cnt)[g] = tL;
        glb(P.res)[g] = (u128)n32 * tS - (u128)F * sc.Q;
    }
}

// Exclusive prefix of the blocks' left counts, in two launches over parts of
// LPART consecutive greedy blocks: part sums, then each part's prefix (from
// the part sums before it) and its blocks' offsets; the total into nleft.
constexpr int LPART = 512;  // greedy blocks per part (2 per thread)
constexpr int LPART_TPB = 256;

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t* s_w) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint32_t tot = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) tot += s_w[q];
    __syncthreads();
    return tot;
}

__global__ __launch_bounds__(LPART_TPB) void k_left_part(const BuildScalars* scp, const uint32_t* cnt,
                                                          uint32_t* part, int64_t G) {
    __shared__ uint32_t s_w[LPART_TPB / 64];
    if (scp->status != WRS_OK) return;
    const int64_t b0 = (int64_t)blockIdx.x * LPART;
    uint32_t v = 0;
    for (int64_t b = b0 + threadIdx.x; b < min(b0 + LPART, G); b += LPART_TPB) v += glb(cnt)[b];
    const uint32_t tot = block_sum_u32(v, s_w);
    if (threadIdx.x == 0) glb(part)[blockIdx.x] = tot;
}

__global__ __launch_bounds__(LPART_TPB) void k_left_offsets(BuildScalars* scp, const uint32_t* cnt,
                                                             const uint32_t* part, uint32_t* goff, int64_t G) {
    __shared__ uint32_t s_w[LPART_TPB / 64];
    if (scp->status != WRS_OK) {  // the greedy blocks did not run
        if (blockIdx.x == 0 && threadIdx.x == 0) scp->nleft = 0;
        return;
    }
    const int64_t P = gridDim.x;
    // this part's offset: the part sums before it
    uint32_t v = 0;
    for (int64_t p = threadIdx.x; p < blockIdx.x; p += LPART_TPB) v += glb(part)[p];
    const uint32_t before = block_sum_u32(v, s_w);
    // scan of this part's counts, two consecutive blocks per thread
    const int64_t b0 = (int64_t)blockIdx.x * LPART + 2 * threadIdx.x;
    const uint32_t c0 = (b0 < G) ? glb(cnt)[b0] : 0u, c1 = (b0 + 1 < G) ? glb(cnt)[b0 + 1] : 0u;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(c0 + c1);
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint32_t ex = before + inc - (c0 + c1), tot = before;
    for (int q = 0; q < LPART_TPB / 64; ++q) {
        if (q < wv) ex += s_w[q];
        tot += s_w[q];
    }
    if (b0 < G) glb(goff)[b0] = ex;
    if (b0 + 1 < G) glb(goff)[b0 + 1] = ex + c0;
    if (blockIdx.x == P - 1 && threadIdx.x == 0) scp->nleft = (int64_t)tot;
}

// Each block's left items to their place in the list.
__global__ __launch_bounds__(GTPB) void k_left_compact(const BuildScalars* scp, PlusLayout P) {
    if (scp->status != WRS_OK) return;
    const int64_t g = blockIdx.x;
    const uint32_t c = glb(P.cnt)[g], o = glb(P.goff)[g];
    const WRS_GLOBAL uint32_t* si = glb(P.sidx) + g * GTILE;
    const WRS_GLOBAL float* sw = glb(P.sw) + g * GTILE;
    for (uint32_t k = threadIdx.x; k < c; k += GTPB) {
        glb(P.lidx)[o + k] = si[k];
        glb(P.lw)[o + k] = sw[k];
    }
}

hipError_t launch_greedy(const JobDesc& J, const PlusLayout& P, hipStream_t st) {
    const int64_t G = cdiv(J.n, GTILE);
    hipLaunchKernelGGL(k_greedy, dim3((unsigned)G), dim3(GTPB), 0, st, J, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t parts = cdiv(G, LPART);
    hipLaunchKernelGGL(k_left_part, dim3((unsigned)parts), dim3(LPART_TPB), 0, st, (const BuildScalars*)J.sc,
                       (const uint32_t*)P.cnt, P.part, G);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_left_offsets, dim3((unsigned)parts), dim3(LPART_TPB), 0, st, J.sc, (const uint32_t*)P.cnt,
                       (const uint32_t*)P.part, P.goff, G);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_left_compact, dim3((unsigned)G), dim3(GTPB), 0, st, (const BuildScalars*)J.sc, P);
    return hipGetLastError();
}

}  // namespace wrs
