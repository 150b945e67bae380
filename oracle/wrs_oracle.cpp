/*
 * wrs_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU reference for the weighted-random-sampling hot
 * path of Huebschle-Schneider & Sanders, "Parallel Weighted Random Sampling"
 * (arXiv 1903.00227).  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * helper with the HIP library; neither side includes or links the other.
 *
 * What it computes (each function below cites the passage it follows):
 *   orc_philox4x32_10   Philox-4x32-10 counter RNG from its published definition
 *                       (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 *                       as easy as 1, 2, 3", SC'11).  The paper itself draws from
 *                       Mersenne Twisters (Section 10), so the bit stream is
 *                       "parity unpinned" by the paper; the tests pin it against
 *                       PyTorch's independent Philox engine instead.
 *   orc_total_weight    W = sum of all weights (Section 1 / Section 2.2), exact.
 *   orc_vose_build      Vose's construction, Algorithm 1 (Section 2.2), in FP64.
 *   orc_sweep_build     the sweeping construction, Algorithm 2 (Section 4.1), in
 *                       exact arithmetic.  The parallel splitting algorithm of
 *                       Section 4.2 (Algorithm 3) produces exactly this table.
 *   orc_psaplus_build   greedy assignment inside blocks, then the sweep over the
 *                       items left (Section 4.2.1, PSA+), in exact arithmetic.
 *   orc_twolevel_*      2-level alias table (Section 4.4, replicated top level):
 *                       block tables by the sweep, a top table over the block
 *                       sums, and its two-step query.
 *   orc_alias_sample*   alias queries (Section 2.2, last paragraph; branchless
 *                       select of Section 10), one Philox call per draw.
 *   orc_reconstruct     per-item mass implied by a table (alias-table definition,
 *                       Section 2.2) compared against n*w_i/W.
 *   orc_wor_keys,       exponential clocks (Section 2.3): key_i = -ln(u_i)/w_i,
 *   orc_sample_wor      the k smallest keys form the sample without replacement
 *                       (problem WRS-N of Section 1).
 *   orc_permutation     problem WRP (Sections 1 and 7): all items in key order.
 *   orc_os_*            output-sensitive sampling with replacement (Section 5),
 *                       in wrs_oracle_os.cpp.
 *
 * Readings where the paper leaves details open are listed in the project's
 * design notes; the ones that affect results are repeated at the functions.
 *
 * Conventions: items are 0-based; tables are (float t, int32 alias) pairs where
 * t is the fraction of the bucket kept by the bucket's own item.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_EDOMAIN -2
#define ORC_ENOMEM -3

/* ------------------------------------------------------------------------- */
/* Philox-4x32-10 (SC'11).  One round maps (x0,x1,x2,x3) with key (k0,k1) to  */
/* (hi(M1*x2)^x1^k0, lo(M1*x2), hi(M0*x0)^x3^k1, lo(M0*x0)); the key is bumped */
/* by the Weyl constants between rounds.                                      */
/* ------------------------------------------------------------------------- */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

extern "C" void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_at(uint64_t seed, uint64_t c01, uint32_t c2, uint32_t c3, uint32_t out[4]) {
    uint32_t ctr[4] = {(uint32_t)c01, (uint32_t)(c01 >> 32), c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------- */
/* Exact non-negative fixed-point numbers: value = sum_k d[k] 2^(32k) 2^-160.  */
/* Every finite FP32 value (smallest subnormal 2^-149) and every product of one */
/* with an integer below 2^31, and every sum of 2^31 such products, is exact.   */
/* ------------------------------------------------------------------------- */
#define XL 12          /* limbs of 32 bits: 384 bits, 160 of them fractional */
#define XFRAC 160
typedef struct { uint32_t d[XL]; } xnum;

static void x_zero(xnum* a) { memset(a, 0, sizeof(*a)); }

static int x_is_zero(const xnum* a) {
    for (int k = 0; k < XL; ++k) if (a->d[k]) return 0;
    return 1;
}

static int x_cmp(const xnum* a, const xnum* b) {
    for (int k = XL - 1; k >= 0; --k) {
        if (a->d[k] != b->d[k]) return a->d[k] < b->d[k] ? -1 : 1;
    }
    return 0;
}

/* a += b */
static void x_add(xnum* a, const xnum* b) {
    uint64_t carry = 0;
    for (int k = 0; k < XL; ++k) {
        uint64_t s = (uint64_t)a->d[k] + b->d[k] + carry;
        a->d[k] = (uint32_t)s;
        carry = s >> 32;
    }
    if (carry) abort(); /* out of range: cannot happen for FP32 inputs, n < 2^31 */
}

/* a -= b, requires a >= b */
static void x_sub(xnum* a, const xnum* b) {
    int64_t borrow = 0;
    for (int k = 0; k < XL; ++k) {
        int64_t s = (int64_t)a->d[k] - (int64_t)b->d[k] - borrow;
        borrow = s < 0;
        a->d[k] = (uint32_t)(s + (borrow ? ((int64_t)1 << 32) : 0));
    }
    if (borrow) abort();
}

/* exact value mult * w for a finite w >= 0 and mult < 2^31 */
static void x_from_float_times(xnum* a, float w, uint32_t mult) {
    x_zero(a);
    uint32_t bits;
    memcpy(&bits, &w, 4);
    uint32_t e = (bits >> 23) & 0xFFu;
    uint32_t m = bits & 0x7FFFFFu;
    if (e != 0) m |= 0x800000u;
    if (m == 0 || mult == 0) return;
    /* w = m * 2^(max(e,1) - 150); in units of 2^-160 that is m << (max(e,1) + 10) */
    int p = (int)(e == 0 ? 1 : e) + 10;
    unsigned __int128 v = (unsigned __int128)((uint64_t)m * mult) << (p % 32);
    int k = p / 32;
    while (v != 0) {
        if (k >= XL) abort();
        a->d[k] = (uint32_t)v;
        v >>= 32;
        ++k;
    }
}

static void x_add_float_times(xnum* a, float w, uint32_t mult) {
    xnum t;
    x_from_float_times(&t, w, mult);
    x_add(a, &t);
}

/* Wide scratch numbers for division: value = sum d[k] 2^(32k) (plain integer). */
#define WL 26
typedef struct { uint32_t d[WL]; } wnum;

static int w_bitlen(const wnum* a) {
    for (int k = WL - 1; k >= 0; --k)
        if (a->d[k]) { int b = 32; while (!((a->d[k] >> (b - 1)) & 1u)) --b; return 32 * k + b; }
    return 0;
}
static int w_cmp(const wnum* a, const wnum* b) {
    for (int k = WL - 1; k >= 0; --k)
        if (a->d[k] != b->d[k]) return a->d[k] < b->d[k] ? -1 : 1;
    return 0;
}
static void w_sub(wnum* a, const wnum* b) {
    int64_t borrow = 0;
    for (int k = 0; k < WL; ++k) {
        int64_t s = (int64_t)a->d[k] - (int64_t)b->d[k] - borrow;
        borrow = s < 0;
        a->d[k] = (uint32_t)(s + (borrow ? ((int64_t)1 << 32) : 0));
    }
    if (borrow) abort();
}
static void w_shl(wnum* r, const wnum* a, int s) { /* r = a << s, s >= 0 */
    wnum t;
    memset(&t, 0, sizeof t);
    int q = s / 32, b = s % 32;
    for (int k = WL - 1; k >= 0; --k) {
        int src = k - q;
        if (src < 0) continue;
        uint64_t v = (uint64_t)a->d[src] << b;
        if (src >= 1 && b) v |= (uint64_t)a->d[src - 1] >> (32 - b);
        t.d[k] = (uint32_t)v;
    }
    /* the caller guarantees no bits are shifted out */
    *r = t;
}
static void w_from_x(wnum* r, const xnum* a) {
    memset(r, 0, sizeof *r);
    for (int k = 0; k < XL; ++k) r->d[k] = a->d[k];
}

/* Correctly rounded (to nearest, ties to even) FP32 value of num/den, den > 0. */
static float x_ratio_to_f32(const xnum* num, const xnum* den) {
    if (x_is_zero(num)) return 0.0f;
    wnum A, B;
    w_from_x(&A, num);
    w_from_x(&B, den);
    int k = w_bitlen(&A) - w_bitlen(&B); /* num/den lies in (2^(k-1), 2^(k+1)) */
    if (k > 130) return INFINITY;
    if (k < -152) return 0.0f;            /* below half the smallest subnormal */
    int s = 26 - k;                        /* q = floor(num 2^s / den) in (2^25, 2^27) */
    if (s >= 0) w_shl(&A, &A, s); else w_shl(&B, &B, -s);
    uint64_t q = 0;
    for (int bit = 27; bit >= 0; --bit) {
        wnum Bs;
        w_shl(&Bs, &B, bit);
        if (w_cmp(&A, &Bs) >= 0) { w_sub(&A, &Bs); q |= (uint64_t)1 << bit; }
    }
    int sticky = 0;
    for (int i = 0; i < WL; ++i) if (A.d[i]) { sticky = 1; break; }
    /* value = (q + rem) * 2^-s, bit i of q weighs 2^(i-s) */
    int nb = 64 - __builtin_clzll(q);
    int d = nb - 24;
    if (s - 149 > d) d = s - 149;          /* subnormal: keep bits of weight >= 2^-149 */
    uint64_t mant, rbits = 0, half = 0;
    if (d <= 0) { mant = q << (-d); }
    else if (d >= 64) { mant = 0; sticky = sticky || q != 0; }
    else { mant = q >> d; rbits = q & (((uint64_t)1 << d) - 1); half = (uint64_t)1 << (d - 1); }
    if (d > 0 && d < 64) {
        if (rbits > half || (rbits == half && (sticky || (mant & 1)))) ++mant;
    }
    return (float)ldexp((double)mant, d - s);
}

/* Round-to-nearest double value of an xnum, and the rounded remainder. */
static double x_to_double(const xnum* a) {
    double v = 0.0;
    /* exact summation from the top: at most 384 bits, so accumulate the top
       limbs exactly into an integer window, then round once */
    wnum A;
    w_from_x(&A, a);
    int bl = w_bitlen(&A);
    if (bl == 0) return 0.0;
    int drop = bl - 53;
    if (drop <= 0) {
        for (int k = XL - 1; k >= 0; --k) v = v * 4294967296.0 + a->d[k];
        return ldexp(v, -XFRAC);
    }
    /* mantissa = top 53 bits, round half even on the remainder */
    uint64_t mant = 0;
    for (int b = bl - 1; b >= drop; --b) mant = (mant << 1) | ((A.d[b / 32] >> (b % 32)) & 1u);
    int rb = (A.d[(drop - 1) / 32] >> ((drop - 1) % 32)) & 1u;
    int sticky = 0;
    for (int b = drop - 2; b >= 0 && !sticky; --b) sticky = (A.d[b / 32] >> (b % 32)) & 1u;
    if (rb && (sticky || (mant & 1))) ++mant;
    return ldexp((double)mant, drop - XFRAC);
}

/* exact value of a double that is a multiple of 2^-160 and below 2^224 */
static void x_from_double(xnum* a, double v) {
    x_zero(a);
    if (v == 0.0) return;
    int e;
    double f = frexp(v, &e);                      /* v = f 2^e, f in [0.5,1) */
    uint64_t m = (uint64_t)ldexp(f, 53);          /* v = m 2^(e-53) */
    int p = e - 53 + XFRAC;
    if (p < 0) { if (m & ((((uint64_t)1) << (-p)) - 1)) abort(); m >>= -p; p = 0; }
    unsigned __int128 t = (unsigned __int128)m << (p % 32);
    int k = p / 32;
    while (t) { if (k >= XL) abort(); a->d[k] = (uint32_t)t; t >>= 32; ++k; }
}

static int valid_weights(const float* w, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        float v = w[i];
        if (!(v >= 0.0f) || std::isinf(v)) return 0; /* NaN, negative or infinite */
    }
    return 1;
}

/* W = sum of all weights, exactly (Section 1 defines W).  Returned as the
   round-to-nearest double hi and the round-to-nearest double of W - hi. */
static void exact_sum(const float* w, int64_t n, xnum* W) {
    x_zero(W);
    for (int64_t i = 0; i < n; ++i) x_add_float_times(W, w[i], 1u);
}

extern "C" int orc_total_weight(const float* w, int64_t n, double* hi, double* lo) {
    if (!w || n < 1 || n > 2147483647LL || !hi || !lo) return ORC_EINVAL;
    if (!valid_weights(w, n)) return ORC_EDOMAIN;
    xnum W;
    exact_sum(w, n, &W);
    double h = x_to_double(&W);
    xnum H;
    x_from_double(&H, h);
    double l;
    if (x_cmp(&W, &H) >= 0) { xnum r = W; x_sub(&r, &H); l = x_to_double(&r); }
    else { xnum r = H; x_sub(&r, &W); l = -x_to_double(&r); }
    *hi = h;
    *lo = l;
    return x_is_zero(&W) ? ORC_EDOMAIN : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1 (Section 2.2): Vose's construction in FP64.                    */
/* Stacks are filled in ascending index order and popped last-in-first-out;  */
/* the bucket update is (b[j].w + b[i].w) - W/n as printed.  Buckets left with */
/* the dummy alias keep their own item (alias := self); t = b.w n / W rounded  */
/* to FP32 and clamped to [0,1].  W is the exactly rounded FP64 total.         */
/* ------------------------------------------------------------------------- */
extern "C" int orc_vose_build(const float* w, int64_t n, float* t, int32_t* alias) {
    if (!w || !t || !alias || n < 1 || n > 2147483647LL) return ORC_EINVAL;
    if (!valid_weights(w, n)) return ORC_EDOMAIN;
    double hi, lo;
    int rc = orc_total_weight(w, n, &hi, &lo);
    if (rc) return rc;
    const double cap = hi / (double)n;
    std::vector<double> bw((size_t)n);
    std::vector<int64_t> ba((size_t)n, -1);
    std::vector<int64_t> heavy, light;
    for (int64_t i = 0; i < n; ++i) {
        bw[i] = (double)w[i];
        if (bw[i] > cap) heavy.push_back(i); else light.push_back(i);
    }
    while (!heavy.empty()) {
        int64_t j = heavy.back();
        heavy.pop_back();
        while (bw[j] > cap && !light.empty()) {
            int64_t i = light.back();
            light.pop_back();
            ba[i] = j;
            bw[j] = (bw[j] + bw[i]) - cap;
        }
        light.push_back(j);
    }
    for (int64_t r = 0; r < n; ++r) {
        double f = bw[r] / cap;
        if (ba[r] < 0) { ba[r] = r; }
        float tf = (float)f;
        if (tf > 1.0f) tf = 1.0f;
        if (tf < 0.0f) tf = 0.0f;
        t[r] = tf;
        alias[r] = (int32_t)ba[r];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 2 (Section 4.1): the sweeping construction, in exact arithmetic. */
/* Everything is kept n-scaled: item i has size n*w_i, every bucket holds W.  */
/* i walks the light items (n*w_i <= W), j the heavy ones, r is the part of    */
/* heavy j not yet placed.  While r > W, light bucket i is filled from j;      */
/* otherwise heavy bucket j keeps r and takes the next heavy as its alias.     */
/* Readings: with no heavy item every bucket keeps its item; the last heavy and */
/* any light bucket left when the heavies are used up take alias := self.      */
/* t is the exact ratio rounded once to FP32 (to nearest, ties to even).       */
/* ------------------------------------------------------------------------- */
extern "C" int orc_sweep_build(const float* w, int64_t n, float* t, int32_t* alias) {
    if (!w || !t || !alias || n < 1 || n > 2147483647LL) return ORC_EINVAL;
    if (!valid_weights(w, n)) return ORC_EDOMAIN;
    xnum W;
    exact_sum(w, n, &W);
    if (x_is_zero(&W)) return ORC_EDOMAIN;
    const uint32_t nn = (uint32_t)n;
    std::vector<unsigned char> is_light((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        xnum s;
        x_from_float_times(&s, w[i], nn);
        is_light[i] = x_cmp(&s, &W) <= 0;
    }
    auto next_light = [&](int64_t from) { while (from < n && !is_light[from]) ++from; return from; };
    auto next_heavy = [&](int64_t from) { while (from < n && is_light[from]) ++from; return from; };
    int64_t i = next_light(0);
    int64_t j = next_heavy(0);
    xnum r;
    if (j < n) x_from_float_times(&r, w[j], nn);
    while (j < n) {
        if (x_cmp(&r, &W) > 0) {            /* pack light bucket i from heavy j */
            if (i >= n) return ORC_EDOMAIN;  /* impossible in exact arithmetic */
            xnum s;
            x_from_float_times(&s, w[i], nn);
            t[i] = x_ratio_to_f32(&s, &W);
            alias[i] = (int32_t)j;
            x_add(&r, &s);
            x_sub(&r, &W);
            i = next_light(i + 1);
        } else {                              /* pack heavy bucket j */
            t[j] = x_ratio_to_f32(&r, &W);
            int64_t jn = next_heavy(j + 1);
            alias[j] = (int32_t)(jn < n ? jn : j);
            if (jn < n) {
                x_add_float_times(&r, w[jn], nn);
                x_sub(&r, &W);
            }
            j = jn;
        }
    }
    while (i < n) {                           /* heavies used up: keep own item */
        xnum s;
        x_from_float_times(&s, w[i], nn);
        float tf = x_ratio_to_f32(&s, &W);
        t[i] = tf > 1.0f ? 1.0f : tf;
        alias[i] = (int32_t)i;
        i = next_light(i + 1);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Section 4.2.1: greedy assignment by blocks, then the splitting algorithm  */
/* on what is left (PSA+).  Items are cut into consecutive blocks of `block` */
/* items.  Inside each block the sweep of Algorithm 2 runs on the block's own */
/* lights and heavies and stops as soon as it needs a light or a next heavy   */
/* that the block does not have.  Everything it packed is final.  The items   */
/* not packed go on, in index order, to a second sweep over all blocks'        */
/* leftovers; the parallel splitting algorithm (Algorithm 3) computes exactly */
/* that sweep, since it only skips the finished items.                        */
/* Reading: the heavy the block stopped at enters the second sweep with the   */
/* part of its size not yet placed (its bucket is not filled yet), as a heavy */
/* if that part exceeds W and as a light otherwise; the untouched items keep  */
/* their sizes.  The second sweep uses the readings of orc_sweep_build.       */
/* ------------------------------------------------------------------------- */
static void sweep_list(const std::vector<int64_t>& idx, const std::vector<xnum>& size, const xnum* W,
                       float* t, int32_t* alias) {
    const size_t m = idx.size();
    std::vector<unsigned char> is_light(m);
    for (size_t k = 0; k < m; ++k) is_light[k] = x_cmp(&size[k], W) <= 0;
    auto next_light = [&](size_t from) { while (from < m && !is_light[from]) ++from; return from; };
    auto next_heavy = [&](size_t from) { while (from < m && is_light[from]) ++from; return from; };
    size_t i = next_light(0), j = next_heavy(0);
    xnum r;
    if (j < m) r = size[j];
    while (j < m) {
        if (x_cmp(&r, W) > 0) {
            if (i >= m) abort();  /* the leftovers fill whole buckets: cannot happen */
            t[idx[i]] = x_ratio_to_f32(&size[i], W);
            alias[idx[i]] = (int32_t)idx[j];
            x_add(&r, &size[i]);
            x_sub(&r, W);
            i = next_light(i + 1);
        } else {
            t[idx[j]] = x_ratio_to_f32(&r, W);
            const size_t jn = next_heavy(j + 1);
            alias[idx[j]] = (int32_t)idx[jn < m ? jn : j];
            if (jn < m) {
                x_add(&r, &size[jn]);
                x_sub(&r, W);
            }
            j = jn;
        }
    }
    while (i < m) {
        float tf = x_ratio_to_f32(&size[i], W);
        t[idx[i]] = tf > 1.0f ? 1.0f : tf;
        alias[idx[i]] = (int32_t)idx[i];
        i = next_light(i + 1);
    }
}

extern "C" int orc_psaplus_build(const float* w, int64_t n, int64_t block, float* t, int32_t* alias) {
    if (!w || !t || !alias || n < 1 || n > 2147483647LL || block < 1) return ORC_EINVAL;
    if (!valid_weights(w, n)) return ORC_EDOMAIN;
    xnum W;
    exact_sum(w, n, &W);
    if (x_is_zero(&W)) return ORC_EDOMAIN;
    const uint32_t nn = (uint32_t)n;
    std::vector<int64_t> left_idx;
    std::vector<xnum> left_size;
    for (int64_t b0 = 0; b0 < n; b0 += block) {
        const int64_t b1 = std::min(n, b0 + block);
        std::vector<xnum> s((size_t)(b1 - b0));
        std::vector<unsigned char> light((size_t)(b1 - b0));
        for (int64_t i = b0; i < b1; ++i) {
            x_from_float_times(&s[i - b0], w[i], nn);
            light[i - b0] = x_cmp(&s[i - b0], &W) <= 0;
        }
        auto next_light = [&](int64_t from) { while (from < b1 && !light[from - b0]) ++from; return from; };
        auto next_heavy = [&](int64_t from) { while (from < b1 && light[from - b0]) ++from; return from; };
        std::vector<std::pair<int64_t, xnum>> left;
        int64_t i = next_light(b0), j = next_heavy(b0);
        if (j >= b1) {                    /* no heavy in the block: every light is left */
            for (; i < b1; i = next_light(i + 1)) left.push_back({i, s[i - b0]});
        } else {
            xnum r = s[j - b0];
            while (true) {
                if (x_cmp(&r, &W) > 0) {
                    if (i >= b1) {        /* out of lights: j (part placed) and later heavies are left */
                        left.push_back({j, r});
                        for (int64_t h = next_heavy(j + 1); h < b1; h = next_heavy(h + 1)) left.push_back({h, s[h - b0]});
                        break;
                    }
                    t[i] = x_ratio_to_f32(&s[i - b0], &W);
                    alias[i] = (int32_t)j;
                    x_add(&r, &s[i - b0]);
                    x_sub(&r, &W);
                    i = next_light(i + 1);
                } else {
                    const int64_t jn = next_heavy(j + 1);
                    if (jn >= b1) {       /* out of heavies: j (rest below W) and later lights are left */
                        left.push_back({j, r});
                        for (; i < b1; i = next_light(i + 1)) left.push_back({i, s[i - b0]});
                        break;
                    }
                    t[j] = x_ratio_to_f32(&r, &W);
                    alias[j] = (int32_t)jn;
                    x_add(&r, &s[jn - b0]);
                    x_sub(&r, &W);
                    j = jn;
                }
            }
        }
        std::sort(left.begin(), left.end(),
                  [](const std::pair<int64_t, xnum>& a, const std::pair<int64_t, xnum>& b) { return a.first < b.first; });
        for (auto& e : left) {
            left_idx.push_back(e.first);
            left_size.push_back(e.second);
        }
    }
    sweep_list(left_idx, left_size, &W, t, alias);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Section 4.4 (replicated top level): a 2-level alias table.  The items are  */
/* cut into consecutive blocks of `block` items; block b is a meta-item of    */
/* weight W_b (the sum of its weights).  Each block gets its own alias table  */
/* over its items (the sweep of Algorithm 2 with the block as the instance),  */
/* stored in place in t/alias with global item indices; the top-level table   */
/* over the meta-items is the sweep over the W_b, in exact arithmetic.        */
/* Reading: a block of total weight 0 keeps (t = 1, alias = self) in every    */
/* bucket; its meta-item has weight 0 and is never drawn.                     */
/* ------------------------------------------------------------------------- */
extern "C" int orc_twolevel_build(const float* w, int64_t n, int64_t block, float* t_top, int32_t* a_top,
                                  float* t, int32_t* alias) {
    if (!w || !t || !alias || !t_top || !a_top || n < 1 || n > 2147483647LL || block < 1) return ORC_EINVAL;
    if (!valid_weights(w, n)) return ORC_EDOMAIN;
    xnum W;
    exact_sum(w, n, &W);
    if (x_is_zero(&W)) return ORC_EDOMAIN;
    const int64_t G = (n + block - 1) / block;
    std::vector<int64_t> meta_idx((size_t)G);
    std::vector<xnum> meta_size((size_t)G);
    for (int64_t b = 0; b < G; ++b) {
        const int64_t b0 = b * block, b1 = std::min(n, b0 + block);
        xnum Wb;
        x_zero(&Wb);
        for (int64_t i = b0; i < b1; ++i) x_add_float_times(&Wb, w[i], 1u);
        if (x_is_zero(&Wb)) {
            for (int64_t i = b0; i < b1; ++i) { t[i] = 1.0f; alias[i] = (int32_t)i; }
        } else {
            int rc = orc_sweep_build(w + b0, b1 - b0, t + b0, alias + b0);
            if (rc) return rc;
            for (int64_t i = b0; i < b1; ++i) alias[i] += (int32_t)b0;
        }
        /* the meta-item's G-scaled size G * W_b, against the bucket W */
        meta_idx[b] = b;
        x_zero(&meta_size[b]);
        for (int64_t i = b0; i < b1; ++i) x_add_float_times(&meta_size[b], w[i], (uint32_t)G);
    }
    sweep_list(meta_idx, meta_size, &W, t_top, a_top);
    return ORC_OK;
}

/* Draws from a 2-level table: a top-level alias query picks the block g
   (Philox block (s lo, s hi, stream_id, 0), the mapping of orc_alias_sample
   over the G meta buckets), then an alias query inside block g picks the item
   (Philox block (s lo, s hi, stream_id, 2), the same mapping over the block's
   m items; its table entries hold global indices).  s = first_counter + j. */
static inline int32_t twolevel_query(const float* t_top, const int32_t* a_top, const float* t,
                                     const int32_t* alias, int64_t n, int64_t block, uint64_t seed,
                                     uint32_t stream_id, uint64_t s) {
    const int64_t G = (n + block - 1) / block;
    uint32_t x[4];
    philox_at(seed, s, stream_id, 0u, x);
    uint64_t hi64 = ((uint64_t)x[1] << 32) | x[0];
    int64_t r = (int64_t)(((unsigned __int128)hi64 * (uint64_t)G) >> 64);
    float u = (float)(x[2] >> 8) * (1.0f / 16777216.0f);
    const int64_t g = (u < t_top[r]) ? r : a_top[r];
    const int64_t b0 = g * block, m = std::min(n, b0 + block) - b0;
    philox_at(seed, s, stream_id, 2u, x);
    hi64 = ((uint64_t)x[1] << 32) | x[0];
    r = (int64_t)(((unsigned __int128)hi64 * (uint64_t)m) >> 64);
    u = (float)(x[2] >> 8) * (1.0f / 16777216.0f);
    return (u < t[b0 + r]) ? (int32_t)(b0 + r) : alias[b0 + r];
}

extern "C" int orc_twolevel_sample(const float* t_top, const int32_t* a_top, const float* t, const int32_t* alias,
                                   int64_t n, int64_t block, uint64_t seed, uint32_t stream_id,
                                   uint64_t first_counter, int64_t k, int32_t* out) {
    if (!t_top || !a_top || !t || !alias || n < 1 || block < 1 || k < 0 || (k > 0 && !out)) return ORC_EINVAL;
    for (int64_t j = 0; j < k; ++j)
        out[j] = twolevel_query(t_top, a_top, t, alias, n, block, seed, stream_id, first_counter + (uint64_t)j);
    return ORC_OK;
}

extern "C" int orc_twolevel_sample_at(const float* t_top, const int32_t* a_top, const float* t,
                                      const int32_t* alias, int64_t n, int64_t block, uint64_t seed,
                                      uint32_t stream_id, const uint64_t* counters, int64_t m, int32_t* out) {
    if (!t_top || !a_top || !t || !alias || !counters || n < 1 || block < 1 || m < 0 || (m > 0 && !out))
        return ORC_EINVAL;
    for (int64_t j = 0; j < m; ++j)
        out[j] = twolevel_query(t_top, a_top, t, alias, n, block, seed, stream_id, counters[j]);
    return ORC_OK;
}

/* Number of items the greedy blocks of orc_psaplus_build leave to the second
   sweep (a diagnostic of the same construction). */
extern "C" int64_t orc_psaplus_leftovers(const float* w, int64_t n, int64_t block) {
    if (!w || n < 1 || n > 2147483647LL || block < 1) return ORC_EINVAL;
    if (!valid_weights(w, n)) return ORC_EDOMAIN;
    xnum W;
    exact_sum(w, n, &W);
    if (x_is_zero(&W)) return ORC_EDOMAIN;
    const uint32_t nn = (uint32_t)n;
    int64_t total = 0;
    for (int64_t b0 = 0; b0 < n; b0 += block) {
        const int64_t b1 = std::min(n, b0 + block);
        std::vector<xnum> L, H;
        for (int64_t i = b0; i < b1; ++i) {
            xnum s;
            x_from_float_times(&s, w[i], nn);
            if (x_cmp(&s, &W) <= 0) L.push_back(s); else H.push_back(s);
        }
        if (H.empty() || L.empty()) { total += (int64_t)(L.size() + H.size()); continue; }
        size_t i = 0, j = 0;
        xnum r = H[0];
        while (true) {
            if (x_cmp(&r, &W) > 0) {
                if (i >= L.size()) { total += (int64_t)(H.size() - j); break; }
                x_add(&r, &L[i]);
                x_sub(&r, &W);
                ++i;
            } else {
                if (j + 1 >= H.size()) { total += 1 + (int64_t)(L.size() - i); break; }
                ++j;
                x_add(&r, &H[j]);
                x_sub(&r, &W);
            }
        }
    }
    return total;
}

/* Light buckets one by one (Section 2.2: a light item keeps its whole weight in
   its own bucket, so t_i = n w_i / W): for each requested index, whether the
   item is light (n w_i <= W) and the correctly rounded t_i. */
extern "C" int orc_light_t_at(const float* w, int64_t n, const int64_t* idx, int64_t m, float* t_out,
                              int32_t* is_light) {
    if (!w || !idx || !t_out || !is_light || n < 1 || n > 2147483647LL || m < 0) return ORC_EINVAL;
    if (!valid_weights(w, n)) return ORC_EDOMAIN;
    xnum W;
    exact_sum(w, n, &W);
    if (x_is_zero(&W)) return ORC_EDOMAIN;
    for (int64_t s = 0; s < m; ++s) {
        if (idx[s] < 0 || idx[s] >= n) return ORC_EINVAL;
        xnum v;
        x_from_float_times(&v, w[idx[s]], (uint32_t)n);
        is_light[s] = x_cmp(&v, &W) <= 0;
        t_out[s] = x_ratio_to_f32(&v, &W);
    }
    return ORC_OK;
}

/* Correctly rounded FP32 of a/b for exact non-negative FP32-derived values:
   exposed for the tests of the rounding helper. a = wa*ma, b = wb*mb. */
extern "C" float orc_ratio_f32(float wa, uint32_t ma, float wb, uint32_t mb) {
    xnum a, b;
    x_from_float_times(&a, wa, ma);
    x_from_float_times(&b, wb, mb);
    return x_ratio_to_f32(&a, &b);
}

/* ------------------------------------------------------------------------- */
/* Alias query (Section 2.2, last paragraph): pick a bucket r uniformly, toss */
/* a coin that shows heads with probability t_r, return r on heads and the     */
/* alias a_r otherwise; Section 10 selects between the two without a branch.  */
/* Bits: Philox key = seed, counter = (c lo, c hi, stream id, 0) with          */
/* c = first_counter + draw index; r = floor((x1 2^32 + x0) n / 2^64);         */
/* u = (x2 >> 8) 2^-24; heads iff u < t_r.                                     */
/* ------------------------------------------------------------------------- */
static inline int32_t alias_query(const float* t, const int32_t* a, int64_t n, uint64_t seed,
                                  uint32_t sid, uint64_t c) {
    uint32_t x[4];
    philox_at(seed, c, sid, 0u, x);
    uint64_t X = ((uint64_t)x[1] << 32) | x[0];
    int64_t r = (int64_t)(((unsigned __int128)X * (uint64_t)n) >> 64);
    float u = (float)(x[2] >> 8) * (1.0f / 16777216.0f);
    int32_t pick[2] = {(int32_t)r, a[r]};
    return pick[!(u < t[r])];
}

extern "C" int orc_alias_sample(const float* t, const int32_t* a, int64_t n, uint64_t seed,
                                uint32_t stream_id, uint64_t first_counter, int64_t k, int32_t* out) {
    if (!t || !a || n < 1 || n > 2147483647LL || k < 0 || (k > 0 && !out)) return ORC_EINVAL;
    for (int64_t s = 0; s < k; ++s) out[s] = alias_query(t, a, n, seed, stream_id, first_counter + (uint64_t)s);
    return ORC_OK;
}

extern "C" int orc_alias_sample_at(const float* t, const int32_t* a, int64_t n, uint64_t seed,
                                   uint32_t stream_id, const uint64_t* counters, int64_t m, int32_t* out) {
    if (!t || !a || n < 1 || n > 2147483647LL || m < 0 || (m > 0 && (!out || !counters))) return ORC_EINVAL;
    for (int64_t s = 0; s < m; ++s) out[s] = alias_query(t, a, n, seed, stream_id, counters[s]);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Reconstruction (alias-table definition, Section 2.2): bucket r gives t_r of */
/* a bucket to item r and 1 - t_r to a_r; item i's total, in buckets, must be  */
/* n w_i / W.  Masses are accumulated as unevaluated double pairs (TwoSum).    */
/* Returns ORC_EDOMAIN if an entry is malformed (t outside [0,1] or NaN, alias */
/* out of range).  rel_err[i] = |mass_i - n w_i/W| / (n w_i/W) for w_i > 0,    */
/* and mass_i itself for w_i = 0.                                               */
/* ------------------------------------------------------------------------- */
static inline void two_sum_acc(double* hi, double* lo, double x) {
    double s = *hi + x;
    double bp = s - *hi;
    double err = (*hi - (s - bp)) + (x - bp);
    *hi = s;
    *lo += err;
}

extern "C" int orc_reconstruct(const float* w, const float* t, const int32_t* a, int64_t n,
                               double* mass, double* rel_err) {
    if (!w || !t || !a || !mass || !rel_err || n < 1 || n > 2147483647LL) return ORC_EINVAL;
    double Whi, Wlo;
    int rc = orc_total_weight(w, n, &Whi, &Wlo);
    if (rc) return rc;
    std::vector<double> mlo((size_t)n, 0.0);
    for (int64_t i = 0; i < n; ++i) mass[i] = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        float tr = t[r];
        if (!(tr >= 0.0f && tr <= 1.0f)) return ORC_EDOMAIN;
        if (a[r] < 0 || (int64_t)a[r] >= n) return ORC_EDOMAIN;
        two_sum_acc(&mass[r], &mlo[r], (double)tr);
        /* 1 - t_r as an exact pair */
        double one_minus_hi = 1.0 - (double)tr;
        double one_minus_lo = (1.0 - one_minus_hi) - (double)tr;
        two_sum_acc(&mass[a[r]], &mlo[a[r]], one_minus_hi);
        two_sum_acc(&mass[a[r]], &mlo[a[r]], one_minus_lo);
    }
    const double W = Whi + Wlo;
    for (int64_t i = 0; i < n; ++i) {
        double m = mass[i] + mlo[i];
        mass[i] = m;
        if (w[i] > 0.0f) {
            double expect = ((double)n * (double)w[i]) / W;
            rel_err[i] = fabs(m - expect) / expect;
        } else {
            rel_err[i] = m;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Exponential clocks (Section 2.3): key_i = -ln(u_i) / w_i with u_i uniform  */
/* in (0,1]; the k smallest keys are a weighted sample without replacement.   */
/* Bits: one Philox block serves four consecutive items: key = seed, counter  */
/* = (g lo, g hi, stream id, 1) for g = floor(i / 4), and u_i = (x_j + 1) 2^-32 */
/* with j = i mod 4.  Zero weights get key +inf.  Ties in the key are broken   */
/* by the smaller item index.  FP64 throughout.                                 */
static double wor_uniform(uint64_t seed, uint32_t stream_id, int64_t i) {
    uint32_t x[4];
    philox_at(seed, (uint64_t)i >> 2, stream_id, 1u, x);
    return ((double)x[i & 3] + 1.0) * (1.0 / 4294967296.0);
}

/* ------------------------------------------------------------------------- */
extern "C" int orc_wor_keys(const float* w, int64_t n, uint64_t seed, uint32_t stream_id, double* keys) {
    if (!w || !keys || n < 1 || n > 2147483647LL) return ORC_EINVAL;
    if (!valid_weights(w, n)) return ORC_EDOMAIN;
    for (int64_t i = 0; i < n; ++i) {
        double e = -log(wor_uniform(seed, stream_id, i));
        keys[i] = w[i] > 0.0f ? e / (double)w[i] : INFINITY;
    }
    return ORC_OK;
}

/* Problem WRP (Section 1; Section 7): permute the items by the process of
   WRS-N run to k = n.  By the exponential clocks of Section 2.3 that is the
   order of the keys -ln(u_i)/w_i (the same keys as orc_wor_keys), ascending,
   ties broken by the smaller index.  Reading: an item of weight 0 has key +inf,
   so the zero-weight items follow every positive one, in index order. */
extern "C" int orc_permutation(const float* w, int64_t n, uint64_t seed, uint32_t stream_id, int32_t* out) {
    if (!w || !out || n < 1 || n > 2147483647LL) return ORC_EINVAL;
    std::vector<double> keys((size_t)n);
    int rc = orc_wor_keys(w, n, seed, stream_id, keys.data());
    if (rc) return rc;
    std::vector<int32_t> idx((size_t)n);
    for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)i;
    std::sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
        return keys[a] < keys[b] || (keys[a] == keys[b] && a < b);
    });
    memcpy(out, idx.data(), sizeof(int32_t) * (size_t)n);
    return ORC_OK;
}

/* The keys of orc_wor_keys at the requested items only (the GPU tests check
   sampled items at sizes where all n keys would not fit); the whole weight
   array is validated as orc_wor_keys validates it. */
extern "C" int orc_wor_keys_at(const float* w, int64_t n, uint64_t seed, uint32_t stream_id,
                               const int64_t* idx, int64_t m, double* keys) {
    if (!w || !keys || !idx || n < 1 || n > 2147483647LL || m < 0) return ORC_EINVAL;
    if (!valid_weights(w, n)) return ORC_EDOMAIN;
    for (int64_t s = 0; s < m; ++s) {
        int64_t i = idx[s];
        if (i < 0 || i >= n) return ORC_EINVAL;
        keys[s] = w[i] > 0.0f ? -log(wor_uniform(seed, stream_id, i)) / (double)w[i] : INFINITY;
    }
    return ORC_OK;
}

struct KeyIdx { double key; int32_t idx; };

extern "C" int orc_sample_wor(const float* w, int64_t n, int64_t k, uint64_t seed, uint32_t stream_id,
                              int32_t* out, double* kth_key) {
    if (!w || n < 1 || n > 2147483647LL || k < 0 || (k > 0 && !out)) return ORC_EINVAL;
    if (!valid_weights(w, n)) return ORC_EDOMAIN;
    int64_t positive = 0;
    for (int64_t i = 0; i < n; ++i) positive += w[i] > 0.0f;
    if (k > positive) return ORC_EDOMAIN;
    if (k == 0) { if (kth_key) *kth_key = 0.0; return ORC_OK; }
    std::vector<double> keys((size_t)n);
    orc_wor_keys(w, n, seed, stream_id, keys.data());
    std::vector<KeyIdx> v((size_t)n);
    for (int64_t i = 0; i < n; ++i) v[i] = KeyIdx{keys[i], (int32_t)i};
    auto less = [](const KeyIdx& a, const KeyIdx& b) {
        return a.key < b.key || (a.key == b.key && a.idx < b.idx);
    };
    std::nth_element(v.begin(), v.begin() + (k - 1), v.end(), less);
    if (kth_key) *kth_key = v[k - 1].key;
    std::vector<int32_t> sel((size_t)k);
    for (int64_t s = 0; s < k; ++s) sel[s] = v[s].idx;
    std::sort(sel.begin(), sel.end());
    memcpy(out, sel.data(), sizeof(int32_t) * (size_t)k);
    return ORC_OK;
}
