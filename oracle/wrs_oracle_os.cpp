/*
 * wrs_oracle_os.cpp -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain sequential reference for output-sensitive sampling with replacement
 * (Section 5 of Huebschle-Schneider & Sanders, "Parallel Weighted Random
 * Sampling"): the sample of k draws is returned as the distinct items drawn
 * with their multiplicities, with expected work O(s + log n) for s distinct
 * items (Theorem on output-sensitive sampling, Section 5).  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load this code; it shares
 * nothing with the HIP library.
 *
 * Structure (Section 5):
 *   - items with w > 0 are put into groups of weights within a factor of two;
 *     the group of w is its binary exponent e = floor(log2 w), and
 *     w = M 2^(e-23) with an integer M in [2^23, 2^24);
 *   - groups are ordered by e, heaviest first; items of a group by index;
 *   - a divide-and-conquer (DC) tree over the groups, and one over each group's
 *     items; a node covering [lo, hi) splits at mid = floor((lo + hi) / 2);
 *   - a node asked for m >= 2 draws (or any top-tree node) passes
 *     Binomial(m, L / (L + R)) of them to its left child (Section 2.4 and
 *     Section 5), a group node asked for exactly one draw takes it from the
 *     group's bucket table by rejection (buckets of capacity 2^(e+1), one item
 *     each), and a one-item node emits (item, m).
 * Node masses: inside a group, exact integer sums of M; over groups, FP64 sums
 * of the exact group totals scaled by 2^(e-23), added in tree order.
 *
 * Random bits: Philox-4x32-10 keyed by the seed, one counter block per attempt
 * at a node: (heap index of the node, low and high word; tag; attempt), tag =
 * the group's position for group-tree nodes and 0xFFFFFFFF for the top tree.
 *
 * Binomial variates (the paper leaves the generator open): inversion (BINV,
 * Kachitvichyanukul & Schmeiser, "Binomial random variate generation", CACM
 * 1988) when the mean is below 10, else transformed rejection with squeeze
 * (BTRS, Hoermann, "The generation of binomial random variates", J. Statist.
 * Comput. Simul. 1993).  Their logarithm, square root and log-factorial are
 * written out below from series and Newton's method with IEEE basic operations
 * only (no libm), so that any implementation following the same definitions
 * draws the same variates bit for bit.  Build without floating-point
 * contraction.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_EDOMAIN -2

extern "C" void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

namespace {

const uint32_t TOP_TAG = 0xFFFFFFFFu;

void block_at(uint64_t seed, uint64_t heap, uint32_t tag, uint32_t attempt, uint32_t x[4]) {
    const uint32_t ctr[4] = {(uint32_t)heap, (uint32_t)(heap >> 32), tag, attempt};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, x);
}

// Uniform in [0, 1) from 53 bits of two words.
double u53(uint32_t lo, uint32_t hi) { return (double)((((uint64_t)hi << 32) | lo) >> 11) * 0x1p-53; }

// A 64-bit integer as the nearest double (one rounding).
double dbl(uint64_t x) { return (double)(uint32_t)(x >> 32) * 4294967296.0 + (double)(uint32_t)x; }

}  // namespace

/* ------------------------------------------------------------------------- */
/* Elementary functions from IEEE basic operations.                           */
/* ------------------------------------------------------------------------- */

// ln x: x = f 2^E with f in [sqrt(1/2), sqrt(2)), ln f = 2 atanh(s) with
// s = (f - 1)/(f + 1) summed as 2 s (1 + z/3 + z^2/5 + ... + z^13/27), z = s^2.
extern "C" double orc_os_log(double x) {
    if (x == 0.0) return -INFINITY;
    int E = 0;
    double f = std::frexp(x, &E);
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

// sqrt x (x > 0): eight Newton steps y <- (y + x/y)/2 from 2^floor(E/2).
extern "C" double orc_os_sqrt(double x) {
    int E = 0;
    (void)std::frexp(x, &E);
    const int e2 = (E - (E & 1)) / 2;
    double y = std::ldexp(1.0, e2);
    for (int i = 0; i < 8; ++i) y = 0.5 * (y + x / y);
    return y;
}

// ln(j!) for an integer-valued j >= 0: a sum of logarithms below 10, else
// Stirling's series ln j! = (j + 1/2) ln(j + 1) - (j + 1) + ln(2 pi)/2
// + 1/(12 x) - 1/(360 x^3) + 1/(1260 x^5), x = j + 1.
extern "C" double orc_os_lfact(double j) {
    if (j < 10.0) {
        double r = 0.0;
        for (int i = 2; i <= (int)j; ++i) r += orc_os_log((double)i);
        return r;
    }
    const double x = j + 1.0;
    const double x2 = x * x;
    const double tail = (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0) / x2) / x2) / x;
    return (j + 0.5) * orc_os_log(x) - x + 0.9189385332046728 + tail;
}

/* ------------------------------------------------------------------------- */
/* Binomial(m, rho) with the counter blocks of node (heap, tag).              */
/* ------------------------------------------------------------------------- */
static int64_t binv(int64_t m, double p, uint64_t seed, uint64_t heap, uint32_t tag) {
    const double q = 1.0 - p;
    const double s = p / q;
    const double a = (double)(m + 1) * s;
    double r0 = 1.0, b = q;  // q^m by binary powering
    for (int64_t e = m; e > 0;) {
        if (e & 1) r0 = r0 * b;
        e >>= 1;
        if (e) b = b * b;
    }
    for (uint32_t t = 0;; ++t) {
        uint32_t x[4];
        block_at(seed, heap, tag, t, x);
        double u = u53(x[0], x[1]);
        double r = r0;
        int64_t j = 0;
        for (;;) {
            if (u < r) return j;
            u = u - r;
            if (j >= m || j >= 110) break;  // a new attempt
            j = j + 1;
            r = r * (a / (double)j - s);
        }
    }
}

static int64_t btrs(int64_t m, double p, uint64_t seed, uint64_t heap, uint32_t tag) {
    const double q = 1.0 - p;
    const double mp = (double)m * p;
    const double spq = orc_os_sqrt(mp * q);
    const double b = 1.15 + 2.53 * spq;
    const double a = -0.0873 + 0.0248 * b + 0.01 * p;
    const double c = mp + 0.5;
    const double vr = 0.92 - 4.2 / b;
    const double alpha = (2.83 + 5.1 / b) * spq;
    const double lpq = orc_os_log(p / q);
    const double mode = std::floor((double)(m + 1) * p);
    const double h = orc_os_lfact(mode) + orc_os_lfact((double)m - mode);
    for (uint32_t t = 0;; ++t) {
        uint32_t x[4];
        block_at(seed, heap, tag, t, x);
        const double u = u53(x[0], x[1]) - 0.5;
        double v = u53(x[2], x[3]);
        const double us = 0.5 - std::fabs(u);
        const double kd = std::floor((2.0 * a / us + b) * u + c);
        if (!(kd >= 0.0 && kd <= (double)m)) continue;
        if (us >= 0.07 && v <= vr) return (int64_t)kd;
        v = v * alpha / (a / (us * us) + b);
        const double bound = h - orc_os_lfact(kd) - orc_os_lfact((double)m - kd) + (kd - mode) * lpq;
        if (orc_os_log(v) <= bound) return (int64_t)kd;
    }
}

static int64_t binomial(int64_t m, double rho, uint64_t seed, uint64_t heap, uint32_t tag) {
    if (m == 0 || rho <= 0.0) return 0;
    if (rho >= 1.0) return m;
    const bool flip = rho > 0.5;
    const double p = flip ? 1.0 - rho : rho;
    const int64_t k = ((double)m * p < 10.0) ? binv(m, p, seed, heap, tag) : btrs(m, p, seed, heap, tag);
    return flip ? m - k : k;
}

extern "C" int orc_os_binomial(int64_t m, double rho, uint64_t seed, uint64_t heap, uint32_t tag, int64_t* out) {
    if (m < 0 || !(rho >= 0.0 && rho <= 1.0) || !out) return ORC_EINVAL;
    *out = binomial(m, rho, seed, heap, tag);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* The structure of Section 5.                                                */
/* ------------------------------------------------------------------------- */
namespace {

struct OsGroup {
    int32_t e;          // binary exponent of the group's weights
    int64_t start, count;
};

struct Os {
    std::vector<int32_t> A;    // item of each position (groups heaviest first)
    std::vector<uint32_t> M;   // integer weight of each position (w = M 2^(e-23))
    std::vector<uint64_t> P;   // P[j] = M[0] + ... + M[j-1]
    std::vector<OsGroup> G;
    std::vector<double> V;     // top-tree node masses by heap index
};

// w = M 2^(e-23), M in [2^23, 2^24), for a positive finite float.
void split_float(float w, int32_t* e, uint32_t* M) {
    uint32_t bits;
    std::memcpy(&bits, &w, 4);
    const uint32_t E = (bits >> 23) & 0xFFu, F = bits & 0x7FFFFFu;
    if (E > 0) {
        *e = (int32_t)E - 127;
        *M = F | 0x800000u;
    } else {
        int bl = 0;
        while ((F >> bl) != 0) ++bl;  // bit length of the subnormal's significand
        *e = bl - 150;
        *M = F << (24 - bl);
    }
}

double top_mass(Os& S, int64_t lo, int64_t hi, uint64_t h) {
    double v;
    if (hi - lo == 1) {
        const OsGroup& g = S.G[lo];
        v = std::ldexp(dbl(S.P[g.start + g.count] - S.P[g.start]), g.e - 23);
    } else {
        const int64_t mid = (lo + hi) / 2;
        const double l = top_mass(S, lo, mid, 2 * h);
        const double r = top_mass(S, mid, hi, 2 * h + 1);
        v = l + r;
    }
    if (S.V.size() <= h) S.V.resize(2 * h + 2, 0.0);
    S.V[h] = v;
    return v;
}

int os_build(const float* w, int64_t n, Os& S) {
    struct It { int32_t e; int32_t i; uint32_t M; };
    std::vector<It> items;
    for (int64_t i = 0; i < n; ++i) {
        const float x = w[i];
        if (!(x >= 0.0f) || std::isinf(x)) return ORC_EDOMAIN;
        if (x == 0.0f) continue;
        It t;
        t.i = (int32_t)i;
        split_float(x, &t.e, &t.M);
        items.push_back(t);
    }
    if (items.empty()) return ORC_EDOMAIN;
    std::stable_sort(items.begin(), items.end(), [](const It& a, const It& b) { return a.e > b.e; });
    const int64_t np = (int64_t)items.size();
    S.A.resize(np);
    S.M.resize(np);
    S.P.assign(np + 1, 0);
    for (int64_t j = 0; j < np; ++j) {
        S.A[j] = items[j].i;
        S.M[j] = items[j].M;
        S.P[j + 1] = S.P[j] + items[j].M;
        if (j == 0 || items[j].e != items[j - 1].e) S.G.push_back(OsGroup{items[j].e, j, 0});
        S.G.back().count++;
    }
    top_mass(S, 0, (int64_t)S.G.size(), 1);
    return ORC_OK;
}

struct Emit { int32_t item; int64_t count; };

// A group-tree node: positions [lo, hi) of group g, asked for m >= 1 draws.
void visit_group(const Os& S, int64_t g, int64_t lo, int64_t hi, uint64_t h, int64_t m, uint64_t seed,
                 std::vector<Emit>& out) {
    const OsGroup& G = S.G[g];
    if (hi - lo == 1) {
        out.push_back(Emit{S.A[G.start + lo], m});
        return;
    }
    if (m == 1) {
        // bucket table with rejection: a uniform bucket, then a uniform point
        // of its capacity 2^(e+1) = 2^24 units of 2^(e-23)
        for (uint32_t t = 0;; ++t) {
            uint32_t x[4];
            block_at(seed, h, (uint32_t)g, t, x);
            const uint64_t r = ((uint64_t)x[1] << 32) | x[0];
            const int64_t j = lo + (int64_t)(((unsigned __int128)r * (uint64_t)(hi - lo)) >> 64);
            const uint32_t Y = x[2] >> 8;
            if (Y < S.M[G.start + j]) {
                out.push_back(Emit{S.A[G.start + j], 1});
                return;
            }
        }
    }
    const int64_t mid = (lo + hi) / 2;
    const uint64_t L = S.P[G.start + mid] - S.P[G.start + lo];
    const uint64_t T = S.P[G.start + hi] - S.P[G.start + lo];
    const int64_t ml = binomial(m, dbl(L) / dbl(T), seed, h, (uint32_t)g);
    if (ml > 0) visit_group(S, g, lo, mid, 2 * h, ml, seed, out);
    if (m - ml > 0) visit_group(S, g, mid, hi, 2 * h + 1, m - ml, seed, out);
}

// A top-tree node: groups [lo, hi), asked for m >= 1 draws.
void visit_top(const Os& S, int64_t lo, int64_t hi, uint64_t h, int64_t m, uint64_t seed, std::vector<Emit>& out) {
    if (hi - lo == 1) {
        visit_group(S, lo, 0, S.G[lo].count, 1, m, seed, out);
        return;
    }
    const int64_t mid = (lo + hi) / 2;
    const int64_t ml = binomial(m, S.V[2 * h] / S.V[h], seed, h, TOP_TAG);
    if (ml > 0) visit_top(S, lo, mid, 2 * h, ml, seed, out);
    if (m - ml > 0) visit_top(S, mid, hi, 2 * h + 1, m - ml, seed, out);
}

}  // namespace

// Groups of the structure: for each group (heaviest first) its exponent, first
// position and size; order[j] = the item at position j.  *u = group count,
// *np = positive items.  Arrays sized n (order) and 300 (groups).
extern "C" int orc_os_groups(const float* w, int64_t n, int32_t* order, int32_t* gexp, int64_t* gstart,
                             int64_t* gcount, int64_t* u, int64_t* np) {
    if (!w || n < 1 || n > 2147483647LL || !order || !gexp || !gstart || !gcount || !u || !np) return ORC_EINVAL;
    Os S;
    const int rc = os_build(w, n, S);
    if (rc) return rc;
    for (size_t j = 0; j < S.A.size(); ++j) order[j] = S.A[j];
    for (size_t g = 0; g < S.G.size(); ++g) {
        gexp[g] = S.G[g].e;
        gstart[g] = S.G[g].start;
        gcount[g] = S.G[g].count;
    }
    *u = (int64_t)S.G.size();
    *np = (int64_t)S.A.size();
    return ORC_OK;
}

// k draws with replacement, output-sensitively: s distinct items, sorted by
// item, with their multiplicities (items[0..s), counts[0..s), s <= min(k, n)).
extern "C" int orc_os_sample(const float* w, int64_t n, int64_t k, uint64_t seed, int32_t* items, int64_t* counts,
                             int64_t* s) {
    if (!w || n < 1 || n > 2147483647LL || k < 0 || k > 2147483647LL || !s || (k > 0 && (!items || !counts)))
        return ORC_EINVAL;
    Os S;
    const int rc = os_build(w, n, S);
    if (rc) return rc;
    std::vector<Emit> out;
    if (k > 0) visit_top(S, 0, (int64_t)S.G.size(), 1, k, seed, out);
    std::sort(out.begin(), out.end(), [](const Emit& a, const Emit& b) { return a.item < b.item; });
    for (size_t j = 0; j < out.size(); ++j) {
        items[j] = out[j].item;
        counts[j] = out[j].count;
    }
    *s = (int64_t)out.size();
    return ORC_OK;
}
